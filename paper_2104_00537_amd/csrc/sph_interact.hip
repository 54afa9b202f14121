// Particle interaction (Section 2.3 of the DualSPHysics v5.0 paper): the
// continuity and momentum sums over neighbours within 2h, on gfx950.
#include "sph_kernels.h"

namespace sph {

// ------------------------------------------------- block partial results --
__device__ inline void write_block_red(float fmag, float vmax, uint32_t cnt, uint32_t cntw,
                                       uint32_t nfl, BlockRed* red) {
  __shared__ float sf[kBlock / 64], sv[kBlock / 64];
  __shared__ uint32_t sc[kBlock / 64], sw[kBlock / 64], sn[kBlock / 64];
  fmag = wave_max(fmag);
  vmax = wave_max(vmax);
  cnt = wave_sum(cnt);
  cntw = wave_sum(cntw);
  nfl = wave_sum(nfl);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { sf[wave] = fmag; sv[wave] = vmax; sc[wave] = cnt; sw[wave] = cntw; sn[wave] = nfl; }
  __syncthreads();
  if (threadIdx.x == 0) {
    BlockRed b{0.f, 0.f, 0u, 0u, 0u, 0u};
    for (int w = 0; w < kBlock / 64; ++w) {
      b.fmax = fmaxf(b.fmax, sf[w]);
      b.vmax = fmaxf(b.vmax, sv[w]);
      b.count += sc[w];
      b.count_wall += sw[w];
      b.nfluid += sn[w];
    }
    red[blockIdx.x] = b;
  }
}

// ------------------------------------------------- interaction, version 1 --
// One lane per target particle (sorted order).  The lane walks the (2R+1)^d
// cells around its own cell (R = cell_div), reads each candidate's view from
// global memory, and accumulates in registers; sums are gathered per target,
// so results are deterministic.
template <int DIM, int R>
__global__ __launch_bounds__(kBlock) void k_interact_gather(
    KParams kp, int64_t n, const float4* __restrict__ pr, const float4* __restrict__ vp,
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ cstart,
    const uint8_t* __restrict__ type, const double* __restrict__ pos64, float* __restrict__ ace,
    float* __restrict__ arho, float* __restrict__ visc, uint32_t* __restrict__ nbr,
    uint32_t flags, BlockRed* __restrict__ red) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float fmag = 0.f, vmax_out = 0.f;
  uint32_t cnt_out = 0, cnt_wall = 0, nfl = 0;
  if (i < n) {
    float acc[3] = {0.f, 0.f, 0.f};
    float cont = 0.f, diff = 0.f, vmax = 0.f, rhoa = 0.f;
    uint32_t c32 = 0, c64 = 0;
    bool fa = false;
    const bool active = !is_excluded(type[i]);
    if (active) {
      const float4 pa = pr[i], va = vp[i];
      fa = pa.w > 0.f;
      rhoa = fabsf(pa.w);
      const float Pa = va.w;
      const uint32_t k = key[i];
      const int cx = (int)(k % (uint32_t)kp.ncx);
      const uint32_t rest = k / (uint32_t)kp.ncx;
      const int cy = (int)(rest % (uint32_t)kp.ncy);
      const int cz = (int)(rest / (uint32_t)kp.ncy);
      const bool diag = (flags & SPH_DIAG_COUNT_F64) != 0;
      double pa64[3] = {0.0, 0.0, 0.0};
      if (diag)
        for (int d = 0; d < DIM; ++d) pa64[d] = pos64[d * n + i];
      const int zlo = DIM == 3 ? -R : 0, zhi = DIM == 3 ? R : 0;
      for (int dz = zlo; dz <= zhi; ++dz) {
        const int z = cz + dz;
        if (z < 0 || z >= kp.ncz) continue;
        for (int dy = -R; dy <= R; ++dy) {
          const int y = cy + dy;
          if (y < 0 || y >= kp.ncy) continue;
          const int x0 = cx - R < 0 ? 0 : cx - R;
          const int x1 = cx + R >= kp.ncx ? kp.ncx - 1 : cx + R;
          const uint32_t row = (uint32_t)kp.ncx * ((uint32_t)y + (uint32_t)kp.ncy * (uint32_t)z);
          const float sy = (float)dy * kp.cs_f, sz = (float)dz * kp.cs_f;
          for (int x = x0; x <= x1; ++x) {
            const uint32_t j0 = cstart[row + x], j1 = cstart[row + x + 1];
            const float sx = (float)(x - cx) * kp.cs_f;
            for (uint32_t j = j0; j < j1; ++j) {
              if ((int64_t)j == i) continue;
              const float4 pb = pr[j];
              const bool fb = pb.w > 0.f;
              if (!fa && !fb) continue;  // Eq. 36: walls see fluid only
              const float dx = pa.x - (pb.x + sx);
              const float dy_ = pa.y - (pb.y + sy);
              const float dz_ = DIM == 3 ? pa.z - (pb.z + sz) : 0.f;
              const float r2 = dx * dx + dy_ * dy_ + dz_ * dz_;
              if (diag) {
                double r2d = 0.0;
                for (int d = 0; d < DIM; ++d) {
                  const double e = __dsub_rn(pa64[d], pos64[d * n + j]);
                  r2d = __dadd_rn(r2d, __dmul_rn(e, e));
                }
                c64 += (r2d < kp.support2) ? 1u : 0u;
              }
              if (!(r2 < kp.support2_f)) continue;
              const float4 vb = vp[j];
              const float rhob = fabsf(pb.w);
              const float vr = (va.x - vb.x) * dx + (va.y - vb.y) * dy_ +
                               (DIM == 3 ? (va.z - vb.z) * dz_ : 0.f);
              const float q = sqrtf(r2) * kp.inv_h_f;
              const float w = 1.f - 0.5f * q;
              const float fab = kp.kfab_f * w * w * w;  // grad_a W_ab = fab r_ab
              const float mb = fb ? kp.mass_f_f : kp.mass_b_f;
              const float volb = mb / rhob;
              cont += volb * fab * vr;
              ++c32;
              if (fa) {
                const float pterm = (Pa + vb.w) / (rhoa * rhob);
                const float mu = kp.h_f * vr / (r2 + kp.eta2_f);
                const float pi = vr < 0.f ? -kp.visc_coef_f * mu / (0.5f * (rhoa + rhob)) : 0.f;
                const float coef = mb * (pterm + pi) * fab;
                acc[0] -= coef * dx;
                acc[1] -= coef * dy_;
                if (DIM == 3) acc[2] -= coef * dz_;
                vmax = fmaxf(vmax, fabsf(mu));
                if (fb) diff += (rhob - rhoa) * (-fab) * volb;
              }
            }
          }
        }
      }
    }
    float ar = rhoa * cont;
    if (active && fa) {
      acc[0] += kp.gx_f;
      acc[1] += kp.gy_f;
      if (DIM == 3) acc[2] += kp.gz_f;
      ar += kp.ddt_coef_f * diff;
      fmag = sqrtf(acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2]);
      vmax_out = vmax;
      nfl = 1;
    } else {
      acc[0] = acc[1] = acc[2] = 0.f;
    }
    for (int d = 0; d < DIM; ++d) ace[d * n + i] = acc[d];
    arho[i] = ar;
    if (visc) visc[i] = vmax;
    if (nbr) nbr[i] = (flags & SPH_DIAG_COUNT_F64) ? c64 : c32;
    cnt_out = c32;
    cnt_wall = (active && !fa) ? c32 : 0u;
  }
  write_block_red(fmag, vmax_out, cnt_out, cnt_wall, nfl, red);
}

hipError_t launch_interact(const KParams& kp, int64_t n, const sph_state& s, const uint32_t* key,
                           const uint32_t* cell_start, float* ace, float* arho, float* visc,
                           uint32_t* nbr, uint32_t flags, void* ws, hipStream_t st) {
  const WsLayout L = ws_layout(n);
  const float4* pr = ws_ptr<float4>(ws, L.view_pr);
  const float4* vp = ws_ptr<float4>(ws, L.view_vp);
  BlockRed* red = ws_ptr<BlockRed>(ws, L.red);
  const unsigned grid = (unsigned)L.nblk_interact;
#define SPH_LAUNCH(D, RR)                                                                      \
  hipLaunchKernelGGL((k_interact_gather<D, RR>), dim3(grid), dim3(kBlock), 0, st, kp, n, pr, vp, \
                     key, cell_start, s.type, s.pos, ace, arho, visc, nbr, flags, red)
  if (kp.dim == 2) {
    if (kp.cell_div == 1) SPH_LAUNCH(2, 1); else SPH_LAUNCH(2, 2);
  } else {
    if (kp.cell_div == 1) SPH_LAUNCH(3, 1); else SPH_LAUNCH(3, 2);
  }
#undef SPH_LAUNCH
  return hipGetLastError();
}

}  // namespace sph
