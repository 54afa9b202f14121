// Batched cases (continuous batching): n_slots independent cases packed into
// one set of arrays.  Slot s owns particles [off_s, off_s + n_s) and cell keys
// [cbase_s, cbase_s + ncell_s] (the last one for its particles outside its
// grid), so one radix sort, one set of cell ranges, one interaction launch
// and one update serve every case with its own constants, dt and t, and
// every slot keeps its particle range through every sort.
#include "sph_dev.h"
#include "sph_kernels.h"
#include "sph_pair.h"
#include "sph_slots.h"

namespace sph {

__global__ void k_batch_cell_keys(const SlotEntry* __restrict__ tab, int ns, int64_t n,
                                  const double* __restrict__ pos, const uint8_t* __restrict__ type,
                                  uint32_t* __restrict__ key, SlotAccum* __restrict__ acc,
                                  uint32_t* __restrict__ disp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)ns * kAccCopies) acc[i] = SlotAccum{0u, 0u, 0u, 0u, 0ull, 0ull};
  if (i < (int64_t)ns * kDispSlots) disp[i] = 0u;  // nothing moved since this binning
  if (i >= n) return;
  const int s = find_slot(tab, ns, i);
  key[i] = tab[s].cbase + cell_key_local(tab[s].kp, pos, type, n, i);
}

__global__ void k_batch_reorder(const SlotEntry* __restrict__ tab, int ns, int64_t n,
                                const uint32_t* __restrict__ perm, const uint32_t* __restrict__ key,
                                sph_state in, sph_state out, sph_state cin, sph_state cout,
                                int carry, float4* __restrict__ pr, float4* __restrict__ vp,
                                uint32_t* __restrict__ err, uint32_t* __restrict__ slot_err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = find_slot(tab, ns, i);
  if (reorder_one(tab[s].kp, n, i, perm[i], key[i] - tab[s].cbase, in, out, cin, cout, carry, pr,
                  vp)) {
    set_error(err, SPH_ERR_EXCLUDED);
    set_error(&slot_err[s], SPH_ERR_EXCLUDED);
  }
}

// As the single-case view refresh, per slot: the view of the current state
// relative to each particle's cell from the last binning; a particle now
// outside its slot's grid is excluded and its view entry can meet no target
// (NaN offsets) and is no target (zero density).  Like a binning, it starts
// the per-slot accumulators of the next interaction pass from zero.
__global__ void k_batch_refresh_view(const SlotEntry* __restrict__ tab, int ns, int64_t n,
                                     const uint32_t* __restrict__ key, sph_state s,
                                     float4* __restrict__ pr, float4* __restrict__ vp,
                                     uint32_t* __restrict__ err, uint32_t* __restrict__ slot_err,
                                     SlotAccum* __restrict__ acc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)ns * kAccCopies) acc[i] = SlotAccum{0u, 0u, 0u, 0u, 0ull, 0ull};
  if (i >= n) return;
  const uint8_t t = s.type[i];
  if (t & SPH_EXCLUDED) return;  // its entry was written by the binning
  const int sl = find_slot(tab, ns, i);
  const KParams& kp = tab[sl].kp;
  if (cell_key_local(kp, s.pos, s.type, n, i) == kp.ncell_total) {
    s.type[i] = t | SPH_EXCLUDED;
    set_error(err, SPH_ERR_EXCLUDED);
    set_error(&slot_err[sl], SPH_ERR_EXCLUDED);
    const float nan = __builtin_nanf("");
    pr[i] = make_float4(0.f, nan, nan, 0.f);
    vp[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  const double x[3] = {s.pos[i], s.pos[n + i], s.pos[2 * n + i]};
  const float v[3] = {s.vel[i], s.vel[n + i], s.vel[2 * n + i]};
  write_view(kp, i, x, v, s.rho[i], t, key[i] - tab[sl].cbase, pr, vp);
}

// One slot's targets among the wave's lanes (`mine`), with that slot's
// constants: each lane walks its own cells (gather_walk) and writes its
// target; returns the lane's contributions to the slot's sums.  The slot's
// error words get SPH_ERR_MARGIN (STALE: cells reused after particles moved
// half a cell or more) from lane `leader`.  LPT > 1: LPT adjacent lanes
// share target a, each walking every LPT-th stencil row (lane `sub`); every
// lane of the wave takes part (the lanes' sums are combined by shuffles),
// and lane sub = 0 writes the target.
template <int R, bool STALE, bool GEN, bool PER, int LPT = 1>
__device__ __forceinline__ void batch_slot_pass(
    const SlotEntry* __restrict__ tab, int rs, int leader, bool mine, int64_t n, int64_t a,
    const float4* __restrict__ pr, const float4* __restrict__ vp, const uint32_t* __restrict__ key,
    const uint32_t* __restrict__ cstart, float* __restrict__ ace, float* __restrict__ arho,
    float* __restrict__ visc, uint32_t* __restrict__ nbr, const uint32_t* __restrict__ disp,
    uint32_t* __restrict__ err, uint32_t* __restrict__ slot_err, float& fmag, float& vmx,
    uint32_t& cnt, uint32_t& cntw, uint32_t& nfl, int sub = 0) {
  const KParams kp = tab[rs].kp;
  const uint32_t cbase = tab[rs].cbase;
  float cull2 = kp.support2_f * 1.0002f;
  if (STALE) {
    const float delta = read_displacement(disp + (size_t)rs * kDispSlots);
    const float rc = __builtin_amdgcn_sqrtf(kp.support2_f) * 1.0001f + delta;
    cull2 = rc * rc;
    if (!(2.f * delta < kp.cs_f) && (threadIdx.x & 63) == leader) {
      set_error(err, SPH_ERR_MARGIN);
      set_error(&slot_err[rs], SPH_ERR_MARGIN);
    }
  }
  if (LPT == 1 && !mine) return;
  PairAcc acc{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0u};
  TargetData T{false, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, false, 0.f};
  uint32_t c64 = 0;
  bool active = false;
  if (mine) {
    const uint32_t lk = key[a] - cbase;
    // a particle the view refresh excluded keeps its cell but has density 0
    const float4 pa = pr[a];
    active = lk < kp.ncell_total && (!STALE || pa.w != 0.f);
    if (active) {
      const float4 va = vp[a];
      T.fluid = pa.w > 0.f;
      T.rho = fabsf(pa.w);
      T.irho = __builtin_amdgcn_rcpf(T.rho);
      T.ik = kp.kvc_f * T.irho;
      T.p = va.w;
      T.vx = va.x;
      T.vy = va.y;
      T.vz = va.z;
      const int cx = (int)(lk % (uint32_t)kp.ncx);
      const uint32_t rest = lk / (uint32_t)kp.ncx;
      const int cy = (int)(rest % (uint32_t)kp.ncy);
      const int cz = (int)(rest / (uint32_t)kp.ncy);
      gather_walk<3, R, false, false, GEN, PER, LPT>(kp, cbase, n, a, pa, T, cx, cy, cz, pr,
                                                     vp, cstart, nullptr, acc, c64, cull2, sub);
    }
  }
  if (LPT > 1) combine_lanes<LPT>(acc, c64);  // every lane: its target's sums
  if (!mine || sub != 0) return;
  if (active) {
    if (T.fluid) acc.cnt -= 1u;  // the self pair: counted, added nothing
    write_target<3>(kp, n, a, T, acc, acc.cnt, ace, arho, visc, nbr, fmag, vmx, nfl);
    cnt = acc.cnt;
    cntw = T.fluid ? 0u : acc.cnt;
  } else {
    write_zero<3>(n, a, ace, arho, visc, nbr);
  }
}

// The interaction over all slots in one launch: one lane per target, with
// the constants of the target's slot.  ALIGNED: every slot's particle range
// is a whole number of wavefronts (sph_batch_describe's flag), so each wave
// lies in one slot and makes one pass; otherwise the lanes of a wave are
// processed slot by slot (almost always one slot), keeping the constants
// uniform, which costs registers.  Per-slot maxima and pair counts are
// combined with order-independent atomics (max of non-negative float bits,
// integer adds).  STALE: the cells of the last binning are reused for a
// refreshed view (the search reaches R, one cell beyond the cells' own
// stencil, and culls with the support widened by the slot's recorded
// displacement).  GEN: some slot takes a formulation option (cubic spline
// kernel, laminar viscosity, Fourtakas DDT); every slot then runs the
// general pair terms with its own options, whose default-formulation
// arithmetic is that of the default kernel, operation for operation.  PER:
// some slot has periodic components; each slot's walk then takes the
// nearest image along its own (kp.periodic), and a slot without any walks as
// in the plain kernel.
template <int R, bool STALE, bool ALIGNED, bool GEN, bool PER>
__global__ __launch_bounds__(kBlock) void k_batch_interact(
    const SlotEntry* __restrict__ tab, int ns, int64_t n, int64_t lanes,
    const float4* __restrict__ pr, const float4* __restrict__ vp, const uint32_t* __restrict__ key,
    const uint32_t* __restrict__ cstart, float* __restrict__ ace, float* __restrict__ arho,
    float* __restrict__ visc, uint32_t* __restrict__ nbr, SlotAccum* __restrict__ sacc,
    const uint32_t* __restrict__ disp, uint32_t* __restrict__ err,
    uint32_t* __restrict__ slot_err) {
  const int lane = threadIdx.x & 63;
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  // ALIGNED: thread = interaction lane (each slot's lanes are a whole number
  // of wavefronts, with the slot's own lane count per target); otherwise
  // thread = target particle
  const int64_t t = (int64_t)lb * kBlock + threadIdx.x;
  const int64_t lim = ALIGNED ? lanes : n;
  int sa = t < lim ? (ALIGNED ? find_slot_lane(tab, ns, t) : find_slot(tab, ns, t)) : -1;
  int64_t a = t;
  float fmag = 0.f, vmx = 0.f;
  uint32_t cnt = 0, cntw = 0, nfl = 0;
  if (ALIGNED) {
    // one slot (and lane count) for the whole wave, or a wave wholly past
    // the lanes (rs = -1)
    const int rs = __builtin_amdgcn_readfirstlane(sa);
    if (rs >= 0) {
      const int lpt = __builtin_amdgcn_readfirstlane(tab[rs].lpt);
      const int64_t u = t - tab[rs].loff;
      if (lpt == kMaxLanes) {
        a = tab[rs].off + u / kMaxLanes;
        batch_slot_pass<R, STALE, GEN, PER, kMaxLanes>(tab, rs, 0, t < lanes, n, a, pr, vp, key,
                                                  cstart, ace, arho, visc, nbr, disp, err,
                                                  slot_err, fmag, vmx, cnt, cntw, nfl,
                                                  (int)(u % kMaxLanes));
      } else {
        a = tab[rs].off + u;
        batch_slot_pass<R, STALE, GEN, PER>(tab, rs, 0, t < lanes, n, a, pr, vp, key, cstart, ace,
                                       arho, visc, nbr, disp, err, slot_err, fmag, vmx, cnt,
                                       cntw, nfl);
      }
    }
  } else {
    bool todo = a < n;
    while (__ballot(todo) != 0ull) {
      const int leader = (int)__builtin_ctzll(__ballot(todo));
      const int rs = __builtin_amdgcn_readlane(sa, leader);
      const bool mine = todo && sa == rs;
      batch_slot_pass<R, STALE, GEN, PER>(tab, rs, leader, mine, n, a, pr, vp, key, cstart, ace,
                                     arho, visc, nbr, disp, err, slot_err, fmag, vmx, cnt, cntw,
                                     nfl);
      todo = todo && !mine;
    }
  }
  // per-slot combination into copy lb % kAccCopies of the slot's sums: the
  // block's waves combined in LDS when the block lies in one slot (one set
  // of atomics per block), else one set per wave and slot
  const int2 bs = block_slots<ALIGNED>(tab, ns, lim, (int64_t)lb * kBlock);
  if (bs.x >= 0 && bs.x == bs.y) {
    __shared__ float sf[kBlock / 64], sv[kBlock / 64];
    __shared__ uint32_t sc[kBlock / 64], sw[kBlock / 64], sk[kBlock / 64];
    const float f = wave_max(fmag), v = wave_max(vmx);
    const uint32_t c = wave_sum(cnt), w = wave_sum(cntw), k = wave_sum(nfl);
    const int wave = threadIdx.x >> 6;
    if (lane == 0) {
      sf[wave] = f;
      sv[wave] = v;
      sc[wave] = c;
      sw[wave] = w;
      sk[wave] = k;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float bf = 0.f, bv = 0.f;
      unsigned long long bc = 0, bw = 0;
      uint32_t bk = 0;
      for (int q = 0; q < kBlock / 64; ++q) {
        bf = fmaxf(bf, sf[q]);
        bv = fmaxf(bv, sv[q]);
        bc += sc[q];
        bw += sw[q];
        bk += sk[q];
      }
      SlotAccum* A = &sacc[(size_t)bs.x * kAccCopies + lb % kAccCopies];
      atomicMax(&A->fmax_bits, __float_as_uint(bf));
      atomicMax(&A->vmax_bits, __float_as_uint(bv));
      atomicAdd(&A->nfluid, bk);
      atomicAdd(&A->count, bc);
      atomicAdd(&A->count_wall, bw);
    }
    return;
  }
  bool pend = t < lim;
  while (__ballot(pend) != 0ull) {
    const int leader = (int)__builtin_ctzll(__ballot(pend));
    const int rs = __builtin_amdgcn_readlane(sa, leader);
    const bool mine = pend && sa == rs;
    float f = mine ? fmag : 0.f, v = mine ? vmx : 0.f;
    uint32_t c = mine ? cnt : 0u, w = mine ? cntw : 0u, k = mine ? nfl : 0u;
    f = wave_max(f);
    v = wave_max(v);
    c = wave_sum(c);
    w = wave_sum(w);
    k = wave_sum(k);
    if (lane == leader) {
      SlotAccum* A = &sacc[(size_t)rs * kAccCopies + lb % kAccCopies];
      atomicMax(&A->fmax_bits, __float_as_uint(f));
      atomicMax(&A->vmax_bits, __float_as_uint(v));
      atomicAdd(&A->nfluid, k);
      atomicAdd(&A->count, (unsigned long long)c);
      atomicAdd(&A->count_wall, (unsigned long long)w);
    }
    pend = pend && !mine;
  }
}

// Eq. 35 per slot: one wavefront per slot (block s), lane q reading the
// slot's accumulator copy q; maxima and integer sums, so the result does not
// depend on the order of the copies.
__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, off, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), off, 64);
    v += ((unsigned long long)hi << 32) | lo;
  }
  return v;
}

__global__ __launch_bounds__(64) void k_batch_reduce_dt(
    const SlotEntry* __restrict__ tab, const SlotAccum* __restrict__ sacc,
    double* __restrict__ dt, uint64_t* __restrict__ inter, uint32_t* __restrict__ err,
    uint32_t* __restrict__ slot_err) {
  static_assert(kAccCopies == 64, "one lane per accumulator copy");
  const int s = blockIdx.x;
  const SlotAccum B = sacc[(size_t)s * kAccCopies + threadIdx.x];
  const uint32_t fb = wave_max_u32(B.fmax_bits), vb = wave_max_u32(B.vmax_bits);
  const uint32_t nfl = wave_sum(B.nfluid);
  const unsigned long long cnt = wave_sum_u64(B.count), cntw = wave_sum_u64(B.count_wall);
  if (threadIdx.x != 0) return;
  const KParams& kp = tab[s].kp;
  const double f = (double)__uint_as_float(fb);
  const double v = (double)__uint_as_float(vb);
  double d = INFINITY;
  if (nfl > 0) {
    const double dtf = f > 0.0 ? sqrt(kp.h / f) : INFINITY;
    const double dtcv = kp.h / (kp.c0 + v);
    d = kp.cfl * (dtf < dtcv ? dtf : dtcv);
  }
  dt[s] = d;
  if (!(d >= kp.dt_floor) || !isfinite(d)) {
    set_error(err, SPH_ERR_DT_FLOOR);
    set_error(&slot_err[s], SPH_ERR_DT_FLOOR);
  }
  if (inter) {
    inter[2 * s] += (uint64_t)cnt;
    inter[2 * s + 1] += (uint64_t)cntw;
  }
}

// The imposed wall motion of an update phase per slot (Eq. 37).  PHASE 1
// also advances the slot's time by dt: the corrector that follows reads only
// the motion written here.
template <int PHASE>
__global__ void k_batch_motion(const SlotEntry* __restrict__ tab, int ns,
                               const double* __restrict__ dt, double* __restrict__ t,
                               SlotMotion* __restrict__ mot) {
  for (int s = threadIdx.x; s < ns; s += blockDim.x) {
    const KParams& kp = tab[s].kp;
    const double d = dt[s], t0 = t[s];
    const double t1 = PHASE == 0 ? t0 + 0.5 * d : t0 + d;
    mot[s] = SlotMotion{d, motion_disp(kp, t1) - motion_disp(kp, t0), motion_vel(kp, t1), 0.0};
    if (PHASE == 1) t[s] = t1;
  }
}

// Raises slot sl's displacement record to cover the distance sqrt(d2) (as
// record_displacement, per slot): each wave makes one atomic per slot among
// its lanes, into that slot's word of the wave's index modulo kDispSlots.
// Every lane of the wave calls this; lanes without a particle pass sl = -1.
__device__ inline void record_displacement_slots(double d2, int sl, uint32_t* __restrict__ disp) {
  const float r = __fsqrt_rn(__double2float_ru(d2));
  const uint32_t b = __float_as_uint(r) + (r > 0.f ? 1u : 0u);
  const int lane = threadIdx.x & 63;
  const uint32_t w = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % kDispSlots;
  bool pend = sl >= 0;
  while (__ballot(pend) != 0ull) {
    const int leader = (int)__builtin_ctzll(__ballot(pend));
    const int rs = __builtin_amdgcn_readlane(sl, leader);
    const bool mine = pend && sl == rs;
    const uint32_t m = wave_max_u32(mine ? b : 0u);
    if (lane == leader && m) atomicMax(&disp[(size_t)rs * kDispSlots + w], m);
    pend = pend && !mine;
  }
}

template <int PHASE>
__global__ __launch_bounds__(kBlock) void k_batch_symplectic(
    const SlotEntry* __restrict__ tab, int ns, int64_t n, const SlotMotion* __restrict__ mot,
    sph_state saved, sph_state s, const float* __restrict__ ace, const float* __restrict__ arho,
    uint32_t* __restrict__ err, uint32_t* __restrict__ slot_err, uint32_t* __restrict__ disp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int sl = i < n ? find_slot(tab, ns, i) : -1;
  double disp2 = 0.0;
  if (i < n) {
    const SlotMotion M = mot[sl];
    if (symplectic_one<PHASE>(tab[sl].kp, n, i, M.dt, M.dmove, M.vmove, saved, s, ace, arho,
                              disp2)) {
      set_error(err, SPH_ERR_NONFINITE);
      set_error(&slot_err[sl], SPH_ERR_NONFINITE);
    }
  }
  // the predictor's moves since the binning, for an interaction reusing its
  // cells: one atomic per block when the block lies in one slot
  if (PHASE == 0) {
    const int2 bs = block_slots(tab, ns, n, (int64_t)blockIdx.x * kBlock);
    if (bs.x >= 0 && bs.x == bs.y)
      record_displacement(disp2, disp + (size_t)bs.x * kDispSlots);
    else
      record_displacement_slots(disp2, sl, disp);
  }
}

__global__ void k_batch_clear_errors(int ns, uint32_t* __restrict__ err,
                                     uint32_t* __restrict__ slot_err) {
  if (threadIdx.x == 0) *err = 0u;
  for (int s = threadIdx.x; s < ns; s += blockDim.x) slot_err[s] = 0u;
}

// ------------------------------------------------------------------ host --
static unsigned grid_for(int64_t n) {
  const int64_t g = (n + kBlock - 1) / kBlock;
  return (unsigned)(g > 0 ? g : 1);
}

hipError_t launch_batch_bin_cells(const BatchDesc& B, const sph_state& in, sph_state& out,
                                  const sph_state* cin, sph_state* cout, uint32_t* key,
                                  uint32_t* perm, uint32_t* cell_start, void* ws, hipStream_t st) {
  const int64_t n = B.n_total;
  const BatchWsLayout W = batch_ws_layout(B.n_slots, n);
  const SlotEntry* tab = (const SlotEntry*)B.table;
  SlotAccum* sacc = ws_ptr<SlotAccum>(ws, W.accum);
  const int64_t nd = (int64_t)B.n_slots * (kDispSlots > kAccCopies ? kDispSlots : kAccCopies);
  const int64_t nk = n > nd ? n : nd;
  hipLaunchKernelGGL(k_batch_cell_keys, dim3(grid_for(nk)), dim3(kBlock), 0, st, tab, B.n_slots,
                     n, in.pos, in.type, ws_ptr<uint32_t>(ws, W.base.keyA), sacc,
                     ws_ptr<uint32_t>(ws, W.disp));
  const uint32_t last_key = (uint32_t)(B.key_cells - 1);
  if (n > 0) {
    const hipError_t e = radix_sort(n, last_key, key, perm, ws, st);
    if (e != hipSuccess) return e;
  }
  launch_cell_start(key, n, last_key + 1, cell_start, st);
  if (n > 0) {
    sph_state ci{}, co{};
    const int carry = (cin && cout) ? 1 : 0;
    if (carry) {
      ci = *cin;
      co = *cout;
    }
    hipLaunchKernelGGL(k_batch_reorder, dim3(grid_for(n)), dim3(kBlock), 0, st, tab, B.n_slots, n,
                       perm, key, in, out, ci, co, carry, ws_ptr<float4>(ws, W.base.view_pr),
                       ws_ptr<float4>(ws, W.base.view_vp), ws_ptr<uint32_t>(ws, W.base.err),
                       ws_ptr<uint32_t>(ws, W.slot_err));
  }
  return hipGetLastError();
}

hipError_t launch_batch_interact(const BatchDesc& B, const uint32_t* key,
                                 const uint32_t* cell_start, float* ace, float* arho, float* visc,
                                 uint32_t* nbr, bool reuse, void* ws, hipStream_t st) {
  const int64_t n = B.n_total;
  const BatchWsLayout W = batch_ws_layout(B.n_slots, n);
  const SlotEntry* tab = (const SlotEntry*)B.table;
  const bool aligned = (B.flags & SPH_BATCH_WAVE_ALIGNED) != 0;
  const bool general = (B.flags & SPH_BATCH_GENERAL) != 0;
  const bool per = (B.flags & SPH_BATCH_PERIODIC) != 0;
  // aligned batches: one thread per interaction lane
  const int64_t lanes = aligned ? (int64_t)B.lanes : n;
  const unsigned grid = grid_for(lanes);
#define SPH_BATCH_LAUNCH_GP(RR, STALE, AL, G, PE)                                              \
  hipLaunchKernelGGL((k_batch_interact<RR, STALE, AL, G, PE>), dim3(grid), dim3(kBlock), 0, st,  \
                     tab,                                                                       \
                     B.n_slots, n, lanes, ws_ptr<float4>(ws, W.base.view_pr),                   \
                     ws_ptr<float4>(ws, W.base.view_vp), key, cell_start, ace, arho, visc, nbr, \
                     ws_ptr<SlotAccum>(ws, W.accum), ws_ptr<uint32_t>(ws, W.disp),              \
                     ws_ptr<uint32_t>(ws, W.base.err), ws_ptr<uint32_t>(ws, W.slot_err))
#define SPH_BATCH_LAUNCH_G(RR, STALE, AL, G)        \
  do {                                              \
    if (per)                                        \
      SPH_BATCH_LAUNCH_GP(RR, STALE, AL, G, true);  \
    else                                            \
      SPH_BATCH_LAUNCH_GP(RR, STALE, AL, G, false); \
  } while (0)
#define SPH_BATCH_LAUNCH(RR, STALE, AL)      \
  do {                                       \
    if (general)                             \
      SPH_BATCH_LAUNCH_G(RR, STALE, AL, true); \
    else                                     \
      SPH_BATCH_LAUNCH_G(RR, STALE, AL, false); \
  } while (0)
#define SPH_BATCH_LAUNCH_R(RR, STALE)         \
  do {                                        \
    if (aligned)                              \
      SPH_BATCH_LAUNCH(RR, STALE, true);      \
    else                                      \
      SPH_BATCH_LAUNCH(RR, STALE, false);     \
  } while (0)
  // reused cells: the search reaches one cell further than the cells' stencil
  const int reach = B.cell_div + (reuse ? 1 : 0);
  if (reach == 1) {
    SPH_BATCH_LAUNCH_R(1, false);
  } else if (reach == 2 && !reuse) {
    SPH_BATCH_LAUNCH_R(2, false);
  } else if (reach == 2) {
    SPH_BATCH_LAUNCH_R(2, true);
  } else {
    SPH_BATCH_LAUNCH_R(3, true);
  }
#undef SPH_BATCH_LAUNCH_R
#undef SPH_BATCH_LAUNCH
#undef SPH_BATCH_LAUNCH_G
#undef SPH_BATCH_LAUNCH_GP
  return hipGetLastError();
}

hipError_t launch_batch_refresh_view(const BatchDesc& B, const sph_state& s, const uint32_t* key,
                                     void* ws, hipStream_t st) {
  const int64_t n = B.n_total;
  const BatchWsLayout W = batch_ws_layout(B.n_slots, n);
  const int64_t na = (int64_t)B.n_slots * kAccCopies;
  const int64_t nk = n > na ? n : na;
  hipLaunchKernelGGL(k_batch_refresh_view, dim3(grid_for(nk)), dim3(kBlock), 0, st,
                     (const SlotEntry*)B.table, B.n_slots, n, key, s,
                     ws_ptr<float4>(ws, W.base.view_pr), ws_ptr<float4>(ws, W.base.view_vp),
                     ws_ptr<uint32_t>(ws, W.base.err), ws_ptr<uint32_t>(ws, W.slot_err),
                     ws_ptr<SlotAccum>(ws, W.accum));
  return hipGetLastError();
}

hipError_t launch_batch_reduce_dt(const BatchDesc& B, double* dt, uint64_t* interactions, void* ws,
                                  hipStream_t st) {
  const BatchWsLayout W = batch_ws_layout(B.n_slots, B.n_total);
  hipLaunchKernelGGL(k_batch_reduce_dt, dim3(B.n_slots), dim3(64), 0, st,
                     (const SlotEntry*)B.table, ws_ptr<SlotAccum>(ws, W.accum), dt, interactions,
                     ws_ptr<uint32_t>(ws, W.base.err), ws_ptr<uint32_t>(ws, W.slot_err));
  return hipGetLastError();
}

hipError_t launch_batch_symplectic(const BatchDesc& B, int phase, const double* dt, double* t,
                                   sph_state& saved, sph_state& s, const float* ace,
                                   const float* arho, void* ws, hipStream_t st) {
  const int64_t n = B.n_total;
  const BatchWsLayout W = batch_ws_layout(B.n_slots, n);
  const SlotEntry* tab = (const SlotEntry*)B.table;
  SlotMotion* mot = ws_ptr<SlotMotion>(ws, W.motion);
  uint32_t* err = ws_ptr<uint32_t>(ws, W.base.err);
  uint32_t* serr = ws_ptr<uint32_t>(ws, W.slot_err);
  if (phase == 0) {
    hipLaunchKernelGGL(k_batch_motion<0>, dim3(1), dim3(kBlock), 0, st, tab, B.n_slots, dt, t, mot);
    if (n > 0)
      hipLaunchKernelGGL(k_batch_symplectic<0>, dim3(grid_for(n)), dim3(kBlock), 0, st, tab,
                         B.n_slots, n, mot, saved, s, ace, arho, err, serr,
                         ws_ptr<uint32_t>(ws, W.disp));
  } else {
    hipLaunchKernelGGL(k_batch_motion<1>, dim3(1), dim3(kBlock), 0, st, tab, B.n_slots, dt, t, mot);
    if (n > 0)
      hipLaunchKernelGGL(k_batch_symplectic<1>, dim3(grid_for(n)), dim3(kBlock), 0, st, tab,
                         B.n_slots, n, mot, saved, s, ace, arho, err, serr,
                         ws_ptr<uint32_t>(ws, W.disp));
  }
  return hipGetLastError();
}

hipError_t launch_batch_clear_errors(const BatchDesc& B, void* ws, hipStream_t st) {
  const BatchWsLayout W = batch_ws_layout(B.n_slots, B.n_total);
  hipLaunchKernelGGL(k_batch_clear_errors, dim3(1), dim3(kBlock), 0, st, B.n_slots,
                     ws_ptr<uint32_t>(ws, W.base.err), ws_ptr<uint32_t>(ws, W.slot_err));
  return hipGetLastError();
}

}  // namespace sph
