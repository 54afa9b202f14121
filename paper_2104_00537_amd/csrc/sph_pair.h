// Device code shared by the single-case and the batched interaction kernels:
// the pair terms of the WCSPH interaction and the per-lane neighbour walk
// (Section 2.3 of the DualSPHysics v5.0 paper).
#pragma once

#include "sph_internal.h"

namespace sph {

struct PairAcc {
  float ax, ay, az;  // sum of -m_b [(P_a+P_b)/(rho_a rho_b) + Pi_ab] F_ab r_ab
  float cont;        // sum of (m_b/rho_b) F_ab v_ab.r_ab
  float diff;        // sum over fluid b of (rho_b - rho_a)|F_ab| m_b/rho_b
  float vmax;        // max of |h v_ab.r_ab/(r^2+eta^2)|
  uint32_t cnt;      // pairs evaluated
};

struct TargetData {
  bool fluid;
  float rho, irho, p;
  float vx, vy, vz;
};

// The pair terms of Eq. 11 (gradient), 15, 17-18, 21-22 and 36 for one pair
// (a, b) with r_ab = (dx, dy, dz), |r_ab|^2 = r2 < 4h^2.  pb.w is +rho_b for a
// fluid particle and -rho_b for a wall; vb.w is P_b.  The caller has already
// dropped wall-wall pairs (Eq. 36 sums over fluid neighbours only).
template <int DIM>
__device__ __forceinline__ void pair_terms(const KParams& kp, const TargetData& a, float dx,
                                           float dy, float dz, float r2, const float4& pb,
                                           const float4& vb, PairAcc& acc) {
  const bool fb = pb.w > 0.f;
  const float rhob = fabsf(pb.w);
  const float vr = (a.vx - vb.x) * dx + (a.vy - vb.y) * dy + (DIM == 3 ? (a.vz - vb.z) * dz : 0.f);
  const float q = __builtin_amdgcn_sqrtf(r2) * kp.inv_h_f;
  const float w = 1.f - 0.5f * q;
  const float fab = kp.kfab_f * w * w * w;  // grad_a W_ab = fab r_ab, fab <= 0
  const float irhob = __builtin_amdgcn_rcpf(rhob);
  const float mb = fb ? kp.mass_f_f : kp.mass_b_f;
  const float fv = fab * (mb * irhob);
  acc.cont += fv * vr;
  acc.cnt += 1u;
  if (a.fluid) {
    const float pterm = (a.p + vb.w) * (a.irho * irhob);
    const float mu = kp.h_f * vr * __builtin_amdgcn_rcpf(r2 + kp.eta2_f);
    // Pi_ab = -alpha c0 mu / ((rho_a + rho_b)/2) for approaching pairs (Eq. 21)
    const float pi =
        vr < 0.f ? -2.f * kp.visc_coef_f * mu * __builtin_amdgcn_rcpf(a.rho + rhob) : 0.f;
    const float coef = mb * (pterm + pi) * fab;
    acc.ax -= coef * dx;
    acc.ay -= coef * dy;
    if (DIM == 3) acc.az -= coef * dz;
    acc.vmax = fmaxf(acc.vmax, fabsf(mu));
    if (fb) acc.diff -= (rhob - a.rho) * fv;
  }
}

// ------------------------------------------------- block partial results --
template <int WAVES>
__device__ inline void write_block_red(float fmag, float vmax, uint32_t cnt, uint32_t cntw,
                                       uint32_t nfl, BlockRed* red, WsHeader* hdr) {
  __shared__ float sf[WAVES], sv[WAVES];
  __shared__ uint32_t sc[WAVES], sw[WAVES], sn[WAVES];
  fmag = wave_max(fmag);
  vmax = wave_max(vmax);
  cnt = wave_sum(cnt);
  cntw = wave_sum(cntw);
  nfl = wave_sum(nfl);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sf[wave] = fmag;
    sv[wave] = vmax;
    sc[wave] = cnt;
    sw[wave] = cntw;
    sn[wave] = nfl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    BlockRed b{0.f, 0.f, 0u, 0u, 0u, 0u};
    for (int w = 0; w < WAVES; ++w) {
      b.fmax = fmaxf(b.fmax, sf[w]);
      b.vmax = fmaxf(b.vmax, sv[w]);
      b.count += sc[w];
      b.count_wall += sw[w];
      b.nfluid += sn[w];
    }
    red[blockIdx.x] = b;
    if (blockIdx.x == 0) hdr->nred = gridDim.x;
  }
}

// Per-target outputs: dv/dt (with gravity) for fluid targets, drho/dt, visc
// and the pair count; returns |dv/dt|, visc and the fluid flag for the block
// partial results.
template <int DIM>
__device__ __forceinline__ void write_target(const KParams& kp, int64_t n, int64_t a,
                                             const TargetData& t, const PairAcc& acc,
                                             uint32_t count_out, float* ace, float* arho,
                                             float* visc, uint32_t* nbr, float& fmag,
                                             float& vmax_out, uint32_t& nfl) {
  float ax = 0.f, ay = 0.f, az = 0.f;
  float ar = t.rho * acc.cont;
  if (t.fluid) {
    ax = acc.ax + kp.gx_f;
    ay = acc.ay + kp.gy_f;
    az = DIM == 3 ? acc.az + kp.gz_f : 0.f;
    ar += kp.ddt_coef_f * acc.diff;
    fmag = sqrtf(ax * ax + ay * ay + az * az);
    vmax_out = acc.vmax;
    nfl = 1;
  }
  ace[a] = ax;
  ace[n + a] = ay;
  if (DIM == 3) ace[2 * n + a] = az;
  arho[a] = ar;
  if (visc) visc[a] = acc.vmax;
  if (nbr) nbr[a] = count_out;
}

template <int DIM>
__device__ __forceinline__ void write_zero(int64_t n, int64_t a, float* ace, float* arho,
                                           float* visc, uint32_t* nbr) {
  ace[a] = 0.f;
  ace[n + a] = 0.f;
  if (DIM == 3) ace[2 * n + a] = 0.f;
  arho[a] = 0.f;
  if (visc) visc[a] = 0.f;
  if (nbr) nbr[a] = 0u;
}

// ---------------------------------------------------------- gather walk --
// The candidate walk of one target lane over the (2R+1)^(d-1) rows of its
// neighbour cells (cell indices offset by cbase).  The 2R+1 cells of a row
// are consecutive in the sorted order, so each row is one candidate range.
// Candidates are read in groups of 4 with all loads in flight together (the
// views are padded, so a group may run past the range), tested, then the
// velocities of the group's neighbours are loaded together and their pair
// terms accumulated.  Along x the view holds the offset from the start of the
// particle's block of kFrameCells cells; the difference of two such offsets
// is off by a whole block length when the pair straddles a block edge, which
// the rounding to the nearest block multiple removes exactly (|x_ab| is below
// (R+1) cells, under half a block).  Along y and z the offsets are
// cell-relative and the row's cell shift is applied by the target.  DIAG also
// counts neighbours with an FP64 test on the FP64 positions (c64).  Wall
// targets ignore wall candidates (Eq. 36); the target itself is skipped.
template <int DIM, int R, bool DIAG>
__device__ __forceinline__ void gather_walk(const KParams& kp, uint32_t cbase, int64_t n,
                                            int64_t i, const float4& pa, const TargetData& T,
                                            int cx, int cy, int cz,
                                            const float4* __restrict__ pr,
                                            const float4* __restrict__ vp,
                                            const uint32_t* __restrict__ cstart,
                                            const double* __restrict__ pos64, PairAcc& acc,
                                            uint32_t& c64) {
  static_assert(2 * (R + 1) < kFrameCells, "frame block must exceed twice the stencil reach");
  double pa64[3] = {0.0, 0.0, 0.0};
  if (DIAG)
    for (int d = 0; d < DIM; ++d) pa64[d] = pos64[d * n + i];
  const float thr_any = kp.support2_f;
  const float thr_fluid = T.fluid ? kp.support2_f : -1.f;
  const int x0 = cx - R < 0 ? 0 : cx - R;
  const int x1 = cx + R >= kp.ncx ? kp.ncx - 1 : cx + R;
  const int zlo = DIM == 3 ? -R : 0, zhi = DIM == 3 ? R : 0;
  for (int dz = zlo; dz <= zhi; ++dz) {
    const int z = cz + dz;
    if (z < 0 || z >= kp.ncz) continue;
    for (int dy = -R; dy <= R; ++dy) {
      const int y = cy + dy;
      if (y < 0 || y >= kp.ncy) continue;
      const uint32_t row =
          cbase + (uint32_t)kp.ncx * ((uint32_t)y + (uint32_t)kp.ncy * (uint32_t)z);
      const uint32_t j0 = cstart[row + x0], j1 = cstart[row + x1 + 1];
      const float ys = pa.y - (float)dy * kp.cs_f, zs = pa.z - (float)dz * kp.cs_f;
      for (uint32_t j = j0; j < j1; j += 4) {
        float4 pb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pb[u] = pr[j + u];
        bool hit[4];
        float dxs[4], dys[4], dzs[4], r2s[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t jj = j + u;
          const float ex = pa.x - pb[u].x;
          dxs[u] = fmaf(-kp.frame_f, rintf(ex * kp.inv_frame_f), ex);
          dys[u] = ys - pb[u].y;
          dzs[u] = DIM == 3 ? zs - pb[u].z : 0.f;
          r2s[u] = dxs[u] * dxs[u] + dys[u] * dys[u] + dzs[u] * dzs[u];
          const float thr = __float_as_int(pb[u].w) > 0 ? thr_any : thr_fluid;
          hit[u] = jj < j1 && (int64_t)jj != i && r2s[u] < thr;
          if (DIAG && jj < j1 && (int64_t)jj != i && (T.fluid || pb[u].w > 0.f)) {
            double r2d = 0.0;
            for (int d = 0; d < DIM; ++d) {
              const double e = __dsub_rn(pa64[d], pos64[d * n + jj]);
              r2d = __dadd_rn(r2d, __dmul_rn(e, e));
            }
            c64 += (r2d < kp.support2) ? 1u : 0u;
          }
        }
        float4 vb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (hit[u]) vb[u] = vp[j + u];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (hit[u]) pair_terms<DIM>(kp, T, dxs[u], dys[u], dzs[u], r2s[u], pb[u], vb[u], acc);
      }
    }
  }
}

}  // namespace sph
