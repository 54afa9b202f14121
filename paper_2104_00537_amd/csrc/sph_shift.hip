// Particle shifting (Section 2.8 of the DualSPHysics v5.0 paper: Eq. 40-41
// with the concentration and its gradient of Eq. 53) on gfx950.
//
// Two gathers over the interaction view of the state n+1/2: the
// concentration C of every particle, then, for fluid particles, its
// gradient and the shift, added to the corrected FP64 positions.  One lane
// per particle in sorted order, blocks placed per XCD as in the
// interaction; sums per lane, no atomics.
#include "sph_kernels.h"
#include "sph_slots.h"

namespace sph {

// Visits every candidate b within 2h of a target (view position pa, key
// cell (cx, cy, cz), cell keys offset by cbase): the rows of the neighbour
// cells, each cut to the key cells the support sphere reaches, as in the
// interaction's walk (periodic components wrapped the same way when PER), in
// groups of 4 candidates.  Calls f(j, dx, dy, dz, r2, pb) with
// r_ab = (dx, dy, dz) and |r_ab|^2 < 4h^2.
template <int DIM, int R, bool PER, typename F>
__device__ inline void visit_neighbours(const KParams& kp, uint32_t cbase, const float4& pa,
                                        int cx, int cy, int cz, const float4* __restrict__ pr,
                                        const uint32_t* __restrict__ cstart, float cull2,
                                        F&& f) {
  const float cs = kp.cs_f;
  const uint32_t xa = __float_as_uint(pa.x);
  const int fcells = kFrameCells << kp.lg_xsub;
  const float fx =
      (float)(int32_t)(xa - ((uint32_t)(cx % fcells) << (29 - kp.lg_xsub))) * kp.unit_x_f;
  const int reach = R * kp.x_sub;
  const bool perx = PER && (kp.periodic & 1);
  const bool pery = PER && (kp.periodic & 2);
  const bool perz = PER && DIM == 3 && (kp.periodic & 4);
  const int xlo = cx - reach < 0 && !perx ? 0 : cx - reach;
  const int xhi = cx + reach >= kp.ncx && !perx ? kp.ncx - 1 : cx + reach;
  const int zlo = DIM == 3 ? -R : 0, zhi = DIM == 3 ? R : 0;
  for (int dz = zlo; dz <= zhi; ++dz) {
    int z = cz + dz;
    if (z < 0 || z >= kp.ncz) {
      if (!perz) continue;
      z += z < 0 ? kp.ncz : -kp.ncz;
    }
    const float ez0 = (float)dz * cs - pa.z;
    const float ez = dz > 0 ? ez0 : (dz < 0 ? -(ez0 + cs) : 0.f);
    for (int dy = -R; dy <= R; ++dy) {
      int y = cy + dy;
      if (y < 0 || y >= kp.ncy) {
        if (!pery) continue;
        y += y < 0 ? kp.ncy : -kp.ncy;
      }
      const float ey0 = (float)dy * cs - pa.y;
      const float ey = dy > 0 ? ey0 : (dy < 0 ? -(ey0 + cs) : 0.f);
      const float w2 = cull2 - ey * ey - ez * ez;
      if (!(w2 > 0.f)) continue;
      const float w = __builtin_amdgcn_sqrtf(w2);
      int x0 = cx + (int)floorf((fx - w) * kp.inv_csx_f);
      int x1 = cx + (int)floorf((fx + w) * kp.inv_csx_f);
      x0 = x0 < xlo ? xlo : x0;
      x1 = x1 > xhi ? xhi : x1;
      const uint32_t row =
          cbase + (uint32_t)kp.ncx * ((uint32_t)y + (uint32_t)kp.ncy * (uint32_t)z);
      const float ys = pa.y - (float)dy * cs, zs = pa.z - (float)dz * cs;
      // candidates 4 at a time, all loads in flight (the view is padded by
      // kViewPad entries, so a group may read past the last particle;
      // those candidates are masked)
      auto range = [&](int c0, int c1, uint32_t xv) {
        const uint32_t j1 = cstart[row + c1 + 1];
        for (uint32_t j = cstart[row + c0]; j < j1; j += 4) {
          float4 pb[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) pb[u] = pr[j + u];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float dx = (float)(int32_t)(xv - __float_as_uint(pb[u].x)) * kp.unit_x_f;
            const float ddy = ys - pb[u].y;
            const float ddz = DIM == 3 ? zs - pb[u].z : 0.f;
            // explicit fma chains: a zero component (2-D cases, and 2-D
            // slots of a batch in the packed (x, 0, z) layout) adds exactly
            // nothing, so both layouts round alike
            const float r2 = fmaf(ddz, ddz, fmaf(ddy, ddy, dx * dx));
            if (j + u < j1 && r2 < kp.support2_f) f(j + u, dx, ddy, ddz, r2, pb[u]);
          }
        }
      };
      if (perx) {
        if (x0 < 0) {
          range(kp.ncx + x0, kp.ncx - 1, xa + kp.lu);
          x0 = 0;
        }
        if (x1 >= kp.ncx) {
          range(0, x1 - kp.ncx, xa - kp.lu);
          x1 = kp.ncx - 1;
        }
      }
      range(x0, x1, xa);
    }
  }
}

// W(r) of the case's kernel: Wendland C2 (Eq. 11) alpha_D (1 - q/2)^4 (2q + 1)
// or cubic spline (Eq. 10).
__device__ inline float kernel_w_f(const KParams& kp, float r2) {
  const float q = __builtin_amdgcn_sqrtf(r2) * kp.inv_h_f;
  if (kp.kernel == 0) {
    const float w = fmaf(-0.5f, q, 1.f), ww = w * w;
    return kp.w_alpha_f * ww * ww * fmaf(2.f, q, 1.f);
  }
  if (q <= 1.f) return kp.w_alpha_f * fmaf(q * q, fmaf(0.75f, q, -1.5f), 1.f);
  const float u = 2.f - q;
  return kp.w_alpha_f * 0.25f * u * u * u;
}

// F_ab with grad_a W_ab = F_ab r_ab (as in the interaction's pair terms).
__device__ inline float kernel_f_f(const KParams& kp, float kfab, float r2) {
  const float s = __builtin_amdgcn_sqrtf(r2);
  if (kp.kernel == 0) {
    const float w = fmaf(s, kp.mhalf_inv_h_f, 1.f);
    return kfab * w * w * w;
  }
  const float q = s * kp.inv_h_f, u = 2.f - q;
  return kfab * (q <= 1.f ? fmaf(2.25f, q, -3.f) : -0.75f * u * u * __builtin_amdgcn_rcpf(q));
}

__device__ inline void target_cell(const KParams& kp, uint32_t k, int& cx, int& cy, int& cz) {
  cx = (int)(k % (uint32_t)kp.ncx);
  const uint32_t rest = k / (uint32_t)kp.ncx;
  cy = (int)(rest % (uint32_t)kp.ncy);
  cz = (int)(rest / (uint32_t)kp.ncy);
}

// C_a = sum_b V_b W_ab (Eq. 53), every non-excluded particle, a included.
// The culling radius squared of a walk: the support (with a margin above the
// FP32 error of the offsets) when the cells are those of the view's own
// binning; widened by the largest recorded displacement when they are reused
// (R above the cells' stencil), with SPH_ERR_MARGIN past half a cell, or
// when particles moved since the binning but the cells' own reach is used.
template <int R>
__device__ inline float shift_cull2(const KParams& kp, const uint32_t* __restrict__ disp,
                                    uint32_t* __restrict__ err) {
  if (R <= kp.cell_div) {
    // the cells' own reach after particles moved since the binning: pairs
    // may be missed
    if (blockIdx.x == 0 && threadIdx.x == 0 && read_displacement(disp) > 0.f)
      set_error(err, SPH_ERR_MARGIN);
    return kp.support2_f * 1.0002f;
  }
  const float delta = read_displacement(disp);
  const float rc = __builtin_amdgcn_sqrtf(kp.support2_f) * 1.0001f + delta;
  if (!(2.f * delta < kp.cs_f) && blockIdx.x == 0 && threadIdx.x == 0)
    set_error(err, SPH_ERR_MARGIN);
  return rc * rc;
}

// C_a of one non-excluded target (local key lk, cell keys offset by cbase).
template <int DIM, int R, bool PER>
__device__ inline float conc_one(const KParams& kp, uint32_t cbase, uint32_t lk, const float4& pa,
                                 const float4* __restrict__ pr,
                                 const uint32_t* __restrict__ cstart, float cull2) {
  const float mf = (float)kp.mass_f, mw = (float)kp.mass_b;
  int cx, cy, cz;
  target_cell(kp, lk, cx, cy, cz);
  float c = 0.f;
  visit_neighbours<DIM, R, PER>(kp, cbase, pa, cx, cy, cz, pr, cstart, cull2,
                                [&](uint32_t, float, float, float, float r2, const float4& pb) {
                                  const float vb = (pb.w > 0.f ? mf : mw) *
                                                   __builtin_amdgcn_rcpf(fabsf(pb.w));
                                  c = fmaf(vb, kernel_w_f(kp, r2), c);
                                });
  return c;
}

// grad C_a = sum_b V_b (C_b - C_a) F_ab r_ab and dr_a = -A_s h |v_a| dt grad C_a
// (Eq. 40-41, 53) for one fluid target i, with the tangential projection
// below the surface threshold (Eq. 54, a_n = 0); dr_a is added to the
// positions (and written to `shift` when given).
template <int DIM, int R, bool PER>
__device__ inline void shift_one(const KParams& kp, uint32_t cbase, uint32_t lk, int64_t n,
                                 int64_t i, const float4* __restrict__ pr,
                                 const float4* __restrict__ vp,
                                 const uint32_t* __restrict__ cstart,
                                 const float* __restrict__ conc, double dt, float cull2,
                                 double* __restrict__ pos, float* __restrict__ shift) {
  const float mf = (float)kp.mass_f, mw = (float)kp.mass_b, kfab = (float)kp.kfab;
  const float4 pa = pr[i], va = vp[i];
  const float ca = conc[i];
  int cx, cy, cz;
  target_cell(kp, lk, cx, cy, cz);
  float g0 = 0.f, g1 = 0.f, g2 = 0.f;
  visit_neighbours<DIM, R, PER>(
      kp, cbase, pa, cx, cy, cz, pr, cstart, cull2,
      [&](uint32_t j, float dx, float dy, float dz, float r2, const float4& pb) {
        const float vb = (pb.w > 0.f ? mf : mw) * __builtin_amdgcn_rcpf(fabsf(pb.w));
        const float w = vb * (conc[j] - ca) * kernel_f_f(kp, kfab, r2);
        g0 = fmaf(w, dx, g0);
        g1 = fmaf(w, dy, g1);
        g2 = fmaf(w, dz, g2);
      });
  // sums over components as explicit fma chains (see visit_neighbours)
  const float speed =
      __builtin_amdgcn_sqrtf(fmaf(va.z, va.z, fmaf(va.y, va.y, va.x * va.x)));
  const float ds = kp.shift_k_f * speed * (float)dt;
  float d[3] = {-ds * g0, -ds * g1, DIM == 3 ? -ds * g2 : 0.f};
  if (kp.shift_fs_f > 0.f && ca < kp.shift_fs_f) {
    const float gg = fmaf(g2, g2, fmaf(g1, g1, g0 * g0));
    if (gg > 0.f) {
      const float k = fmaf(d[2], g2, fmaf(d[1], g1, d[0] * g0)) / gg;
      d[0] = fmaf(-k, g0, d[0]);
      d[1] = fmaf(-k, g1, d[1]);
      d[2] = fmaf(-k, g2, d[2]);
    }
  }
  for (int c = 0; c < DIM; ++c) {
    pos[c * n + i] += (double)d[c];
    if (shift) shift[c * n + i] = d[c];
  }
}

template <int DIM, int R, bool PER>
__global__ __launch_bounds__(kBlock) void k_shift_conc(KParams kp, int64_t n,
                                                       const float4* __restrict__ pr,
                                                       const uint32_t* __restrict__ key,
                                                       const uint32_t* __restrict__ cstart,
                                                       const uint8_t* __restrict__ type,
                                                       float* __restrict__ conc,
                                                       const uint32_t* __restrict__ disp,
                                                       uint32_t* __restrict__ err) {
  const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const float cull2 = shift_cull2<R>(kp, disp, err);
  if (i >= n) return;
  conc[i] = is_excluded(type[i])
                ? 0.f
                : conc_one<DIM, R, PER>(kp, 0u, key[i], pr[i], pr, cstart, cull2);
}

template <int DIM, int R, bool PER>
__global__ __launch_bounds__(kBlock) void k_shift_apply(
    KParams kp, int64_t n, const float4* __restrict__ pr, const float4* __restrict__ vp,
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ cstart,
    const uint8_t* __restrict__ type, const float* __restrict__ conc,
    const double* __restrict__ dtp, double* __restrict__ pos, float* __restrict__ shift,
    const uint32_t* __restrict__ disp, uint32_t* __restrict__ err) {
  const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const float cull2 = shift_cull2<R>(kp, disp, err);
  if (i >= n) return;
  const uint8_t t = type[i];
  if (!is_fluid(t) || is_excluded(t)) {
    if (shift)
      for (int d = 0; d < DIM; ++d) shift[d * n + i] = 0.f;
    return;
  }
  shift_one<DIM, R, PER>(kp, 0u, key[i], n, i, pr, vp, cstart, conc, *dtp, cull2, pos, shift);
}

// ------------------------------------------------------------- batches --
// Shifting over the slots of a batch (packed 3-component arrays, cell keys
// offset per slot): each slot with its own constants, dt and displacement
// record; slots whose A_s is zero are left as they are (C = 0, no shift).
// The lanes of a wave are taken slot by slot (one pass when the wave lies in
// one slot), so every pass has its slot's constants uniform.

// The culling radius squared of a slot's walk, as shift_cull2 with the
// slot's own displacement record and error word (reported by lane `leader`).
template <int R>
__device__ inline float batch_shift_cull2(const KParams& kp, const uint32_t* __restrict__ disp,
                                          uint32_t* __restrict__ err,
                                          uint32_t* __restrict__ slot_err, int leader) {
  const float delta = read_displacement(disp);
  if (R <= kp.cell_div) {
    // the cells' own reach after particles moved since the binning
    if (delta > 0.f && (threadIdx.x & 63) == leader) {
      set_error(err, SPH_ERR_MARGIN);
      set_error(slot_err, SPH_ERR_MARGIN);
    }
    return kp.support2_f * 1.0002f;
  }
  const float rc = __builtin_amdgcn_sqrtf(kp.support2_f) * 1.0001f + delta;
  if (!(2.f * delta < kp.cs_f) && (threadIdx.x & 63) == leader) {
    set_error(err, SPH_ERR_MARGIN);
    set_error(slot_err, SPH_ERR_MARGIN);
  }
  return rc * rc;
}

template <int R, bool APPLY, bool PER>
__global__ __launch_bounds__(kBlock) void k_batch_shift(
    const SlotEntry* __restrict__ tab, int ns, int64_t n, const float4* __restrict__ pr,
    const float4* __restrict__ vp, const uint32_t* __restrict__ key,
    const uint32_t* __restrict__ cstart, const uint8_t* __restrict__ type,
    float* __restrict__ conc, const double* __restrict__ dt, double* __restrict__ pos,
    float* __restrict__ shift, const uint32_t* __restrict__ disp, uint32_t* __restrict__ err,
    uint32_t* __restrict__ slot_err) {
  const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const int sa = i < n ? find_slot(tab, ns, i) : -1;
  bool todo = i < n;
  while (__ballot(todo) != 0ull) {
    const int leader = (int)__builtin_ctzll(__ballot(todo));
    const int rs = __builtin_amdgcn_readlane(sa, leader);
    const bool mine = todo && sa == rs;
    todo = todo && !mine;
    const KParams& kp = tab[rs].kp;
    if (!(kp.shift_k_f > 0.f)) {  // no shifting in this slot
      if (mine && !APPLY) conc[i] = 0.f;
      if (mine && APPLY && shift)
        for (int d = 0; d < 3; ++d) shift[d * n + i] = 0.f;
      continue;
    }
    const uint32_t cbase = tab[rs].cbase;
    const float cull2 =
        batch_shift_cull2<R>(kp, disp + (size_t)rs * kDispSlots, err, &slot_err[rs], leader);
    if (!mine) continue;
    const uint8_t t = type[i];
    if (!APPLY) {
      conc[i] = is_excluded(t)
                    ? 0.f
                    : conc_one<3, R, PER>(kp, cbase, key[i] - cbase, pr[i], pr, cstart, cull2);
    } else if (!is_fluid(t) || is_excluded(t)) {
      if (shift)
        for (int d = 0; d < 3; ++d) shift[d * n + i] = 0.f;
    } else {
      shift_one<3, R, PER>(kp, cbase, key[i] - cbase, n, i, pr, vp, cstart, conc, dt[rs], cull2,
                           pos, shift);
    }
  }
}

hipError_t launch_shifting(const KParams& kp, int64_t n, const sph_state& s, const uint32_t* key,
                           const uint32_t* cell_start, const double* dt, float* conc,
                           float* shift, bool reuse, void* ws, hipStream_t st) {
  const WsLayout L = ws_layout(n);
  const float4* pr = ws_ptr<float4>(ws, L.view_pr);
  const float4* vp = ws_ptr<float4>(ws, L.view_vp);
  float* c = conc ? conc : ws_ptr<float>(ws, L.keyA);
  const uint32_t* disp = ws_ptr<uint32_t>(ws, L.disp);
  uint32_t* err = ws_ptr<uint32_t>(ws, L.err);
  const unsigned grid = (unsigned)L.nblk_interact;
  const bool per = kp.periodic != 0;
  // reused cells: one more cell of reach, cut widened by the displacement
  const int reach = kp.cell_div + (reuse ? 1 : 0);
#define SPH_SHIFT(D, RR, PE)                                                                  \
  do {                                                                                        \
    hipLaunchKernelGGL((k_shift_conc<D, RR, PE>), dim3(grid), dim3(kBlock), 0, st, kp, n, pr, \
                       key, cell_start, s.type, c, disp, err);                                \
    hipLaunchKernelGGL((k_shift_apply<D, RR, PE>), dim3(grid), dim3(kBlock), 0, st, kp, n,    \
                       pr, vp, key, cell_start, s.type, c, dt, s.pos, shift, disp, err);      \
  } while (0)
#define SPH_SHIFT_P(D, RR) \
  if (per) SPH_SHIFT(D, RR, true); else SPH_SHIFT(D, RR, false)
#define SPH_SHIFT_R(D)                      \
  if (reach == 1) SPH_SHIFT_P(D, 1);        \
  else if (reach == 2) SPH_SHIFT_P(D, 2);   \
  else SPH_SHIFT_P(D, 3)
  if (kp.dim == 2) {
    SPH_SHIFT_R(2);
  } else {
    SPH_SHIFT_R(3);
  }
#undef SPH_SHIFT_R
#undef SPH_SHIFT_P
#undef SPH_SHIFT
  return hipGetLastError();
}

hipError_t launch_batch_shifting(const BatchDesc& B, const sph_state& s, const uint32_t* key,
                                 const uint32_t* cell_start, const double* dt, float* conc,
                                 float* shift, bool reuse, void* ws, hipStream_t st) {
  const int64_t n = B.n_total;
  const BatchWsLayout W = batch_ws_layout(B.n_slots, n);
  const SlotEntry* tab = (const SlotEntry*)B.table;
  const float4* pr = ws_ptr<float4>(ws, W.base.view_pr);
  const float4* vp = ws_ptr<float4>(ws, W.base.view_vp);
  float* c = conc ? conc : ws_ptr<float>(ws, W.base.keyA);
  const uint32_t* disp = ws_ptr<uint32_t>(ws, W.disp);
  uint32_t* err = ws_ptr<uint32_t>(ws, W.base.err);
  uint32_t* serr = ws_ptr<uint32_t>(ws, W.slot_err);
  const int64_t g = (n + kBlock - 1) / kBlock;
  const unsigned grid = (unsigned)(g > 0 ? g : 1);
  // reused cells: one more cell of reach, cut widened by each slot's record
  const int reach = B.cell_div + (reuse ? 1 : 0);
  const bool per = (B.flags & SPH_BATCH_PERIODIC) != 0;
#define SPH_BSHIFT_P(RR, PE)                                                                    \
  do {                                                                                          \
    hipLaunchKernelGGL((k_batch_shift<RR, false, PE>), dim3(grid), dim3(kBlock), 0, st, tab,    \
                       B.n_slots, n, pr, vp, key, cell_start, s.type, c, dt, s.pos, shift, disp, \
                       err, serr);                                                              \
    hipLaunchKernelGGL((k_batch_shift<RR, true, PE>), dim3(grid), dim3(kBlock), 0, st, tab,     \
                       B.n_slots, n, pr, vp, key, cell_start, s.type, c, dt, s.pos, shift, disp, \
                       err, serr);                                                              \
  } while (0)
#define SPH_BSHIFT(RR)             \
  do {                             \
    if (per)                       \
      SPH_BSHIFT_P(RR, true);      \
    else                           \
      SPH_BSHIFT_P(RR, false);     \
  } while (0)
  if (reach == 1) {
    SPH_BSHIFT(1);
  } else if (reach == 2) {
    SPH_BSHIFT(2);
  } else {
    SPH_BSHIFT(3);
  }
#undef SPH_BSHIFT
#undef SPH_BSHIFT_P
  return hipGetLastError();
}

}  // namespace sph
