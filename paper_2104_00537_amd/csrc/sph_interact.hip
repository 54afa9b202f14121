// Particle interaction (Section 2.3 of the DualSPHysics v5.0 paper): the
// continuity and momentum sums over neighbours within 2h, on gfx950.
//
// One lane per target particle in sorted order walks the rows of its
// neighbour cells (gather_walk).  Consecutive blocks cover consecutive targets
// and are placed so that each XCD runs one contiguous share of them: the
// neighbour views a block reads were then mostly brought into that XCD's L2
// by its predecessors.  Sums are gathered per target (no atomics): results are
// deterministic.
#include "sph_kernels.h"
#include "sph_pair.h"

namespace sph {

// ------------------------------------------------- interaction: gather --
// One lane per target particle (sorted order): the production kernel.
template <int DIM, int R, bool DIAG, bool EQM>
__global__ __launch_bounds__(kBlock) void k_interact_gather(
    KParams kp, int64_t n, const float4* __restrict__ pr, const float4* __restrict__ vp,
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ cstart,
    const uint8_t* __restrict__ type, const double* __restrict__ pos64, float* __restrict__ ace,
    float* __restrict__ arho, float* __restrict__ visc, uint32_t* __restrict__ nbr,
    BlockRed* __restrict__ red, WsHeader* __restrict__ hdr) {
  const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  float fmag = 0.f, vmax_out = 0.f;
  uint32_t cnt_out = 0, cnt_wall = 0, nfl = 0;
  if (i < n) {
    PairAcc acc{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0u};
    TargetData T{false, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    uint32_t c64 = 0;
    if (!is_excluded(type[i])) {
      const float4 pa = pr[i], va = vp[i];
      T.fluid = pa.w > 0.f;
      T.rho = fabsf(pa.w);
      T.irho = __builtin_amdgcn_rcpf(T.rho);
      T.p = va.w;
      T.vx = va.x;
      T.vy = va.y;
      T.vz = va.z;
      const uint32_t k = key[i];
      const int cx = (int)(k % (uint32_t)kp.ncx);
      const uint32_t rest = k / (uint32_t)kp.ncx;
      const int cy = (int)(rest % (uint32_t)kp.ncy);
      const int cz = (int)(rest / (uint32_t)kp.ncy);
      gather_walk<DIM, R, DIAG, EQM>(kp, 0u, n, i, pa, T, cx, cy, cz, pr, vp, cstart, pos64, acc, c64);
      const uint32_t c = DIAG ? c64 : acc.cnt;
      write_target<DIM>(kp, n, i, T, acc, c, ace, arho, visc, nbr, fmag, vmax_out, nfl);
      cnt_out = acc.cnt;
      cnt_wall = T.fluid ? 0u : acc.cnt;
    } else {
      write_zero<DIM>(n, i, ace, arho, visc, nbr);
    }
  }
  write_block_red<kBlock / 64>(fmag, vmax_out, cnt_out, cnt_wall, nfl, red, hdr);
}

hipError_t launch_interact(const KParams& kp, int64_t n, const sph_state& s, const uint32_t* key,
                           const uint32_t* cell_start, float* ace, float* arho, float* visc,
                           uint32_t* nbr, uint32_t flags, void* ws, hipStream_t st) {
  const WsLayout L = ws_layout(n);
  const float4* pr = ws_ptr<float4>(ws, L.view_pr);
  const float4* vp = ws_ptr<float4>(ws, L.view_vp);
  BlockRed* red = ws_ptr<BlockRed>(ws, L.red);
  WsHeader* hdr = ws_ptr<WsHeader>(ws, L.err);
  const unsigned grid = (unsigned)L.nblk_interact;
  const bool diag = (flags & SPH_DIAG_COUNT_F64) != 0;
  const bool eqm = kp.mass_f == kp.mass_b;
#define SPH_LAUNCH(D, RR, G, PP)                                                               \
  hipLaunchKernelGGL((k_interact_gather<D, RR, G, PP>), dim3(grid), dim3(kBlock), 0, st, kp, n, \
                     pr, vp, key, cell_start, s.type, s.pos, ace, arho, visc, nbr, red, hdr)
#define SPH_LAUNCH_P(D, RR, G) \
  if (eqm) SPH_LAUNCH(D, RR, G, true); else SPH_LAUNCH(D, RR, G, false)
  if (kp.dim == 2) {
    if (kp.cell_div == 1) {
      if (diag) SPH_LAUNCH_P(2, 1, true); else SPH_LAUNCH_P(2, 1, false);
    } else {
      if (diag) SPH_LAUNCH_P(2, 2, true); else SPH_LAUNCH_P(2, 2, false);
    }
  } else {
    if (kp.cell_div == 1) {
      if (diag) SPH_LAUNCH_P(3, 1, true); else SPH_LAUNCH_P(3, 1, false);
    } else {
      if (diag) SPH_LAUNCH_P(3, 2, true); else SPH_LAUNCH_P(3, 2, false);
    }
  }
#undef SPH_LAUNCH_P
#undef SPH_LAUNCH
  return hipGetLastError();
}

}  // namespace sph
