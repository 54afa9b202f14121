// Particle interaction (Section 2.3 of the DualSPHysics v5.0 paper): the
// continuity and momentum sums over neighbours within 2h, on gfx950.
//
// One lane per target particle in sorted order walks the rows of its
// neighbour cells (gather_walk).  Blocks cover consecutive targets and are
// dealt to the XCDs in chunks of 16 consecutive blocks (xcd_block): the blocks
// of a chunk share neighbour views through their XCD's L2, and every XCD gets
// chunks from every part of the domain, which balances the work across the
// XCDs.  Sums are gathered per target (no atomics): results are
// deterministic.
#include <type_traits>

#include "sph_kernels.h"
#include "sph_dev.h"
#include "sph_pair.h"

namespace sph {

// ------------------------------------------------- interaction: gather --
// The target's own terms from its view entry (sorted slot i).
template <bool GEN>
__device__ __forceinline__ void target_data(const KParams& kp, int64_t i,
                                            const float4* __restrict__ pr,
                                            const float4* __restrict__ vp,
                                            const uint8_t* __restrict__ type, TargetData& T) {
  const float4 pa = pr[i], va = vp[i];
  T.fluid = pa.w > 0.f;
  T.rho = fabsf(pa.w);
  T.irho = __builtin_amdgcn_rcpf(T.rho);
  T.ik = kp.kvc_f * T.irho;
  T.p = va.w;
  T.vx = va.x;
  T.vy = va.y;
  T.vz = va.z;
  T.flt = GEN && kp.floating && is_floating(type[i]);
}

// Cell coordinates (in key cells) of key k.
__device__ __forceinline__ void key_cell(const KParams& kp, uint32_t k, int& cx, int& cy,
                                         int& cz) {
  cx = (int)(k % (uint32_t)kp.ncx);
  const uint32_t rest = k / (uint32_t)kp.ncx;
  cy = (int)(rest % (uint32_t)kp.ncy);
  cz = (int)(rest / (uint32_t)kp.ncy);
}

// LPT lanes per target particle (sorted order); LPT = 1 is the production
// kernel of large cases, LPT = 4 deals each target's rows to four lanes for
// cases too small to fill the GPU.
template <int DIM, int R, bool DIAG, bool EQM, bool GEN, bool PER, int LPT>
__global__ __launch_bounds__(kBlock) void k_interact_gather(
    KParams kp, int64_t n, const float4* __restrict__ pr, const float4* __restrict__ vp,
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ cstart,
    const uint8_t* __restrict__ type, const double* __restrict__ pos64, float* __restrict__ ace,
    float* __restrict__ arho, float* __restrict__ visc, uint32_t* __restrict__ nbr,
    BlockRed* __restrict__ red, WsHeader* __restrict__ hdr, const uint32_t* __restrict__ disp) {
  static_assert(LPT == 1 || LPT == 2 || LPT == 4, "lanes per target: 1, 2 or 4");
  const int64_t t = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const int64_t i = t / LPT;
  const int sub = (int)(t % LPT);
  float fmag = 0.f, vmax_out = 0.f;
  uint32_t cnt_out = 0, cnt_wall = 0, nfl = 0;
  // cells reused after a view refresh (R above the cells' own stencil): cull
  // with the support widened by the largest displacement since the binning
  float cull2 = kp.support2_f * 1.0002f;
  if (R > kp.cell_div) {
    const float delta = read_displacement(disp);
    const float rc = __builtin_amdgcn_sqrtf(kp.support2_f) * 1.0001f + delta;
    cull2 = rc * rc;
    if (!(2.f * delta < kp.cs_f) && blockIdx.x == 0 && threadIdx.x == 0)
      set_error(&hdr->err, SPH_ERR_MARGIN);
  } else if (blockIdx.x == 0 && threadIdx.x == 0 && read_displacement(disp) > 0.f) {
    // particles moved since the binning (a predictor ran) but the walk keeps
    // the cells' own reach: pairs may be missed
    set_error(&hdr->err, SPH_ERR_MARGIN);
  }
  if constexpr (LPT == 1) {
    if (i < n) {
      PairAcc acc{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0u};
      TargetData T{false, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, false, 0.f};
      uint32_t c64 = 0;
      // with modified DBC the wall densities come from Eq. 38 (sph_mdbc): wall
      // targets take no sums
      if (!is_excluded(type[i]) && (kp.boundary == 0 || is_fluid(type[i]))) {
        const float4 pa = pr[i], va = vp[i];
        T.fluid = pa.w > 0.f;
        T.rho = fabsf(pa.w);
        T.irho = __builtin_amdgcn_rcpf(T.rho);
        T.ik = kp.kvc_f * T.irho;
        T.p = va.w;
        T.vx = va.x;
        T.vy = va.y;
        T.vz = va.z;
        T.flt = GEN && kp.floating && is_floating(type[i]);
        const uint32_t k = key[i];
        const int cx = (int)(k % (uint32_t)kp.ncx);
        const uint32_t rest = k / (uint32_t)kp.ncx;
        const int cy = (int)(rest % (uint32_t)kp.ncy);
        const int cz = (int)(rest / (uint32_t)kp.ncy);
        gather_walk<DIM, R, DIAG, EQM, GEN, PER>(kp, 0u, n, i, pa, T, cx, cy, cz, pr, vp, cstart,
                                                pos64, acc, c64, cull2);
        if (T.fluid) acc.cnt -= 1u;  // the self pair: counted, added nothing
        const uint32_t c = DIAG ? c64 : acc.cnt;
        write_target<DIM>(kp, n, i, T, acc, c, ace, arho, visc, nbr, fmag, vmax_out, nfl);
        cnt_out = acc.cnt;
        cnt_wall = T.fluid ? 0u : acc.cnt;
      } else {
        write_zero<DIM>(n, i, ace, arho, visc, nbr);
      }
    }
  } else {
    PairAcc acc{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0u};
    TargetData T{false, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, false, 0.f};
    uint32_t c64 = 0;
    const bool active =
        i < n && !is_excluded(type[i]) && (kp.boundary == 0 || is_fluid(type[i]));
    if (active) {
      target_data<GEN>(kp, i, pr, vp, type, T);
      int cx, cy, cz;
      key_cell(kp, key[i], cx, cy, cz);
      gather_walk<DIM, R, DIAG, EQM, GEN, PER, LPT>(kp, 0u, n, i, pr[i], T, cx, cy, cz, pr, vp,
                                                    cstart, pos64, acc, c64, cull2, sub);
    }
    combine_lanes<LPT>(acc, c64);  // every lane: the sums of its target's lanes
    if (i < n && sub == 0) {
      if (active) {
        if (T.fluid) acc.cnt -= 1u;  // the self pair: counted, added nothing
        const uint32_t c = DIAG ? c64 : acc.cnt;
        write_target<DIM>(kp, n, i, T, acc, c, ace, arho, visc, nbr, fmag, vmax_out, nfl);
        cnt_out = acc.cnt;
        cnt_wall = T.fluid ? 0u : acc.cnt;
      } else {
        write_zero<DIM>(n, i, ace, arho, visc, nbr);
      }
    }
  }
  write_block_red<kBlock / 64>(fmag, vmax_out, cnt_out, cnt_wall, nfl, red, hdr);
}

// ---------------------------------------------- precision-study arms --
// Two reference forms of the interaction for the precision study of
// Section 5.1 (not the production path): with T = double every pair is
// evaluated in FP64 from the FP64 positions, with the pressure recomputed in
// FP64 from the density (Eq. 28); with T = float the distances come from
// positions rounded to FP32 as absolute coordinates (the scheme the
// cell-relative offsets replace) and the rest is FP32.  Velocities and
// densities are the stored FP32 values in both.  Every candidate of the
// (2R+1)^d neighbour cells is tested against (2h)^2 and the pair terms of
// Eq. 11, 15, 17-18, 21-22 and 36 are applied as written, with plain division
// and square root.
template <typename T>
struct ArmAcc {
  T ax, ay, az, cont, diff, vmax;
  uint32_t cnt;
};

// F64S (with T = double): the all-FP64 arm, whose velocities and densities
// come from the state's FP64 copies (vel64, rho64) and whose rates are
// written as FP64 arrays; otherwise ace and arho are FP32 arrays.
template <int DIM, int R, typename T, bool F64S>
__global__ __launch_bounds__(kBlock) void k_interact_arm(
    KParams kp, int64_t n, const float4* __restrict__ pr, const float4* __restrict__ vp,
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ cstart,
    const uint8_t* __restrict__ type, const double* __restrict__ pos64,
    const double* __restrict__ vel64, const double* __restrict__ rho64, void* __restrict__ ace_out,
    void* __restrict__ arho_out, float* __restrict__ visc, uint32_t* __restrict__ nbr,
    BlockRed* __restrict__ red, WsHeader* __restrict__ hdr) {
  static_assert(!F64S || sizeof(T) == 8, "the all-FP64 arm evaluates pairs in FP64");
  using Out = typename std::conditional<F64S, double, float>::type;
  Out* ace = static_cast<Out*>(ace_out);
  Out* arho = static_cast<Out*>(arho_out);
  const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  float fmag = 0.f, vmax_out = 0.f;
  uint32_t cnt_out = 0, cnt_wall = 0, nfl = 0;
  if (i < n) {
    if (!is_excluded(type[i]) && (kp.boundary == 0 || is_fluid(type[i]))) {
      const float4 pa = pr[i], va = vp[i];
      const bool fa = pa.w > 0.f;
      const T rho_a = F64S ? (T)rho64[i] : (T)fabsf(pa.w);
      const T p_a = sizeof(T) == 8 ? (T)(kp.b_tait * tait_ratio(kp, (double)rho_a)) : (T)va.w;
      T v_a[3] = {(T)va.x, (T)va.y, (T)va.z};
      if (F64S)
        for (int d = 0; d < DIM; ++d) v_a[d] = (T)vel64[d * n + i];
      T x_a[3] = {0, 0, 0};
      for (int d = 0; d < DIM; ++d) x_a[d] = (T)pos64[d * n + i];
      const T h = (T)kp.h, support2 = (T)kp.support2, kfab = (T)kp.kfab;
      ArmAcc<T> acc{0, 0, 0, 0, 0, 0, 0u};
      const uint32_t k = key[i];
      const int cx = (int)(k % (uint32_t)kp.ncx);
      const uint32_t rest = k / (uint32_t)kp.ncx;
      const int cy = (int)(rest % (uint32_t)kp.ncy);
      const int cz = (int)(rest / (uint32_t)kp.ncy);
      const int reach = R * kp.x_sub;  // key cells along x
      const int x0 = cx - reach < 0 ? 0 : cx - reach;
      const int x1 = cx + reach >= kp.ncx ? kp.ncx - 1 : cx + reach;
      const int zlo = DIM == 3 ? -R : 0, zhi = DIM == 3 ? R : 0;
      for (int dz = zlo; dz <= zhi; ++dz) {
        const int z = cz + dz;
        if (z < 0 || z >= kp.ncz) continue;
        for (int dy = -R; dy <= R; ++dy) {
          const int y = cy + dy;
          if (y < 0 || y >= kp.ncy) continue;
          const uint32_t row = (uint32_t)kp.ncx * ((uint32_t)y + (uint32_t)kp.ncy * (uint32_t)z);
          const uint32_t j1 = cstart[row + x1 + 1];
          for (uint32_t j = cstart[row + x0]; j < j1; ++j) {
            if ((int64_t)j == i) continue;
            const float4 pb = pr[j];
            const bool fb = pb.w > 0.f;
            if (!fa && !fb) continue;  // Eq. 36: walls see fluid neighbours only
            T r[3] = {0, 0, 0};
            T r2 = 0;
            for (int d = 0; d < DIM; ++d) {
              r[d] = x_a[d] - (T)pos64[d * n + j];
              r2 += r[d] * r[d];
            }
            if (!(r2 < support2)) continue;
            const float4 vb = vp[j];
            const T rho_b = F64S ? (T)rho64[j] : (T)fabsf(pb.w);
            const T p_b = sizeof(T) == 8 ? (T)(kp.b_tait * tait_ratio(kp, (double)rho_b)) : (T)vb.w;
            T v_b[3] = {(T)vb.x, (T)vb.y, (T)vb.z};
            if (F64S)
              for (int d = 0; d < DIM; ++d) v_b[d] = (T)vel64[d * n + j];
            const T m_b = (T)(fb ? kp.mass_f : kp.mass_b);
            const T q = sqrt(r2) / h;
            const T w = (T)1 - q / (T)2;
            const T fab = kfab * w * w * w;  // grad_a W_ab = fab r_ab
            T vr = 0;
            for (int d = 0; d < DIM; ++d) vr += (v_a[d] - v_b[d]) * r[d];
            const T vol_b = m_b / rho_b;
            acc.cont += vol_b * fab * vr;
            acc.cnt += 1u;
            if (fa) {
              const T mu = h * vr / (r2 + (T)kp.eta2);
              const T pi = vr < 0 ? -(T)kp.alpha_c0 * mu / ((rho_a + rho_b) / (T)2) : (T)0;
              const T coef = m_b * ((p_a + p_b) / (rho_a * rho_b) + pi) * fab;
              acc.ax -= coef * r[0];
              acc.ay -= coef * r[1];
              if (DIM == 3) acc.az -= coef * r[2];
              acc.vmax = fmax(acc.vmax, fabs(mu));
              if (fb) acc.diff += (rho_b - rho_a) * fabs(fab) * vol_b;
            }
          }
        }
      }
      T ax = 0, ay = 0, az = 0;
      T ar = rho_a * acc.cont;
      if (fa) {
        ax = acc.ax + (T)kp.gx;
        ay = acc.ay + (T)kp.gy;
        az = DIM == 3 ? acc.az + (T)kp.gz : (T)0;
        ar += (T)kp.ddt_coef * acc.diff;
        fmag = (float)sqrt(ax * ax + ay * ay + az * az);
        vmax_out = (float)acc.vmax;
        nfl = 1;
      }
      ace[i] = (Out)ax;
      ace[n + i] = (Out)ay;
      if (DIM == 3) ace[2 * n + i] = (Out)az;
      arho[i] = (Out)ar;
      if (visc) visc[i] = (float)acc.vmax;
      if (nbr) nbr[i] = acc.cnt;
      cnt_out = acc.cnt;
      cnt_wall = fa ? 0u : acc.cnt;
    } else {
      ace[i] = 0;
      ace[n + i] = 0;
      if (DIM == 3) ace[2 * n + i] = 0;
      arho[i] = 0;
      if (visc) visc[i] = 0.f;
      if (nbr) nbr[i] = 0u;
    }
  }
  write_block_red<kBlock / 64>(fmag, vmax_out, cnt_out, cnt_wall, nfl, red, hdr);
}

hipError_t launch_interact(const KParams& kp, int64_t n, const sph_state& s, const uint32_t* key,
                           const uint32_t* cell_start, float* ace, float* arho, float* visc,
                           uint32_t* nbr, uint32_t flags, void* ws, hipStream_t st) {
  const WsLayout L = ws_layout(n);
  const InteractScratch w{ws_ptr<float4>(ws, L.view_pr), ws_ptr<float4>(ws, L.view_vp),
                          ws_ptr<BlockRed>(ws, L.red), ws_ptr<WsHeader>(ws, L.err),
                          ws_ptr<uint32_t>(ws, L.disp)};
  return launch_interact_on(kp, n, s, key, cell_start, ace, arho, visc, nbr, flags, w, st);
}

hipError_t launch_interact_on(const KParams& kp, int64_t n, const sph_state& s,
                              const uint32_t* key, const uint32_t* cell_start, float* ace,
                              float* arho, float* visc, uint32_t* nbr, uint32_t flags,
                              const InteractScratch& w, hipStream_t st) {
  const float4* pr = w.pr;
  const float4* vp = w.vp;
  BlockRed* red = w.red;
  WsHeader* hdr = w.hdr;
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock > 0 ? (n + kBlock - 1) / kBlock : 1);
  const uint32_t arm = flags & ~(uint32_t)SPH_INTERACT_ONE_LANE;  // the arms take one lane
  if (arm == SPH_INTERACT_F64 || arm == SPH_INTERACT_ABS_F32 || arm == SPH_INTERACT_F64_STATE) {
    const bool f64 = arm == SPH_INTERACT_F64;
    const bool f64s = arm == SPH_INTERACT_F64_STATE;
#define SPH_ARM(D, RR, T, FS)                                                                 \
  hipLaunchKernelGGL((k_interact_arm<D, RR, T, FS>), dim3(grid), dim3(kBlock), 0, st, kp, n,   \
                     pr, vp, key, cell_start, s.type, s.pos, s.vel64, s.rho64, (void*)ace,     \
                     (void*)arho, visc, nbr, red, hdr)
#define SPH_ARM_T(D, RR)                                                 \
  if (f64s) SPH_ARM(D, RR, double, true);                                \
  else if (f64) SPH_ARM(D, RR, double, false);                           \
  else SPH_ARM(D, RR, float, false)
    if (kp.dim == 2) {
      if (kp.cell_div == 1) SPH_ARM_T(2, 1); else SPH_ARM_T(2, 2);
    } else {
      if (kp.cell_div == 1) SPH_ARM_T(3, 1); else SPH_ARM_T(3, 2);
    }
#undef SPH_ARM_T
#undef SPH_ARM
    return hipGetLastError();
  }
  const bool diag = (flags & SPH_DIAG_COUNT_F64) != 0;
  // reused cells: one more cell of reach (the kernels read the displacement)
  const int reach = kp.cell_div + ((flags & SPH_INTERACT_REUSE_CELLS) ? 1 : 0);
  const bool eqm = kp.mass_f == kp.mass_b;
  const bool gen = kp.kernel != 0 || kp.viscosity != 0 || kp.ddt == 2 || kp.floating != 0;
  const bool per = kp.periodic != 0;  // periodic cases run the general kernel with PER
  // small cases of the default formulation: four lanes per target
  const bool lanes4 = !gen && !per && !(flags & SPH_INTERACT_ONE_LANE) && n <= kLanesMaxN;
  const unsigned grid4 = (unsigned)((n * kMaxLanes + kBlock - 1) / kBlock);
#define SPH_LAUNCH(D, RR, G, PP, GG, PE, LP)                                                 \
  hipLaunchKernelGGL((k_interact_gather<D, RR, G, PP, GG, PE, LP>),                          \
                     dim3(LP == 1 ? grid : (grid4 > 0 ? grid4 : 1)), dim3(kBlock), 0, st, kp, n, \
                     pr, vp, key, cell_start, s.type, s.pos, ace, arho, visc, nbr, red, hdr,   \
                     w.disp)
#define SPH_LAUNCH_G(D, RR, G, PP)                                       \
  if (per) SPH_LAUNCH(D, RR, G, PP, true, true, 1);                      \
  else if (gen) SPH_LAUNCH(D, RR, G, PP, true, false, 1);                \
  else if (lanes4) SPH_LAUNCH(D, RR, G, PP, false, false, kMaxLanes);    \
  else SPH_LAUNCH(D, RR, G, PP, false, false, 1)
#define SPH_LAUNCH_P(D, RR, G) \
  if (eqm) SPH_LAUNCH_G(D, RR, G, true); else SPH_LAUNCH_G(D, RR, G, false)
#define SPH_LAUNCH_R(D, RR) \
  if (diag) SPH_LAUNCH_P(D, RR, true); else SPH_LAUNCH_P(D, RR, false)
  if (kp.dim == 2) {
    if (reach == 1) { SPH_LAUNCH_R(2, 1); }
    else if (reach == 2) { SPH_LAUNCH_R(2, 2); }
    else { SPH_LAUNCH_R(2, 3); }
  } else {
    if (reach == 1) { SPH_LAUNCH_R(3, 1); }
    else if (reach == 2) { SPH_LAUNCH_R(3, 2); }
    else { SPH_LAUNCH_R(3, 3); }
  }
#undef SPH_LAUNCH_R
#undef SPH_LAUNCH_G
#undef SPH_LAUNCH_P
#undef SPH_LAUNCH
  return hipGetLastError();
}

}  // namespace sph
