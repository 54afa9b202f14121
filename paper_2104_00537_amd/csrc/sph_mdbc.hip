// Modified dynamic boundary condition (Section 2.6.2 of the DualSPHysics
// v5.0 paper, Eq. 38-39): wall densities and velocities from ghost nodes.
//
// One lane per wall particle (sorted order).  Its ghost node G = r_B +
// normal_B is binned like a particle and placed in the view's frame
// (fixed-point x, cell-relative y and z); the rows of G's neighbour cells are
// walked as in the interaction (one range per row, cut to the support sphere
// of G).  Distances, kernel weights and volumes are FP32 as in the
// interaction; the moment sums and the solve are FP64.  The (d+1) x (d+1) corrected system is
// solved by Gaussian elimination with partial pivoting in registers.  Only
// wall entries of the state density and of the interaction view are written;
// the fluid entries that the walk reads are never changed, and the sign of a
// wall's view density (the only thing read of a wall candidate) stays
// negative.
#include "sph_dev.h"
#include "sph_kernels.h"

namespace sph {

// Kernel value and gradient factor (grad W = F r) in FP32: Wendland C2
// (Eq. 11), W = alpha_D (1 - q/2)^4 (2q + 1), F = kfab (1 - q/2)^3, or cubic
// spline (Eq. 10), with alpha_D and kfab of the case.  The weights enter the
// corrected system both as W and as F; exactness for linear fields holds for
// any weights, so their FP32 rounding only perturbs the result at ~1e-7.
__device__ inline void kernel_wf32(const KParams& kp, float r, float& w, float& f) {
  const float q = r * kp.inv_h_f;
  if (kp.kernel == 0) {
    const float u = 1.f - 0.5f * q;
    const float u3 = u * u * u;
    w = kp.w_alpha_f * u3 * u * (2.f * q + 1.f);
    f = kp.f_coef_f * u3;
  } else if (q <= 1.f) {
    w = kp.w_alpha_f * (1.f - 1.5f * q * q + 0.75f * q * q * q);
    f = kp.f_coef_f * (-3.f + 2.25f * q);
  } else {
    const float u = 2.f - q;
    w = kp.w_alpha_f * 0.25f * u * u * u;
    f = -0.75f * kp.f_coef_f * u * u / q;
  }
}

// Solves the M x M system A x = b in place (x returned in b) by Gaussian
// elimination with partial pivoting; the row exchanges are compare-and-swap
// steps with fixed indices, so the arrays stay in registers.  Returns the
// determinant (0 if a pivot vanished).
template <int M>
__device__ inline double solve_small(double (&A)[M][M], double (&b)[M]) {
  double det = 1.0;
#pragma unroll
  for (int c = 0; c < M; ++c) {
#pragma unroll
    for (int r = c + 1; r < M; ++r) {
      if (fabs(A[r][c]) > fabs(A[c][c])) {
#pragma unroll
        for (int k = 0; k < M; ++k) {
          const double t = A[c][k];
          A[c][k] = A[r][k];
          A[r][k] = t;
        }
        const double t = b[c];
        b[c] = b[r];
        b[r] = t;
        det = -det;
      }
    }
    if (A[c][c] == 0.0) return 0.0;
    det *= A[c][c];
    const double inv = 1.0 / A[c][c];
#pragma unroll
    for (int r = c + 1; r < M; ++r) {
      const double f = A[r][c] * inv;
#pragma unroll
      for (int k = c; k < M; ++k) A[r][k] -= f * A[c][k];
      b[r] -= f * b[c];
    }
  }
#pragma unroll
  for (int c = M - 1; c >= 0; --c) {
    double s = b[c];
#pragma unroll
    for (int k = c + 1; k < M; ++k) s -= A[c][k] * b[k];
    b[c] = s / A[c][c];
  }
  return det;
}

template <int DIM, int R>
__global__ __launch_bounds__(kBlock) void k_mdbc(KParams kp, int64_t n, sph_state s,
                                                 const uint32_t* __restrict__ cstart,
                                                 float4* __restrict__ pr,
                                                 float4* __restrict__ vp) {
  constexpr int M = DIM + 1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint8_t t = s.type[i];
  if (is_excluded(t) || is_fluid(t)) return;
  double g[3] = {0.0, 0.0, 0.0}, rb[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    rb[d] = s.pos[d * n + i];
    g[d] = rb[d] + (double)s.normal[d * n + i];
  }
  // key cell of the ghost node; a ghost node outside the grid has no fluid
  // around it (the wall is treated as dry)
  const double org[3] = {kp.ox, kp.oy, kp.oz};
  const int nc[3] = {kp.ncx, kp.ncy, kp.ncz};
  int c[3] = {0, 0, 0};
  bool inside = true;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double f = floor((g[d] - org[d]) * (d == 0 ? kp.inv_csx : kp.inv_cs));
    inside = inside && f >= 0.0 && f < (double)nc[d];
    c[d] = inside ? (int)f : 0;
  }
  // sums of the corrected system: sw = sum V w, swr = sum V w r,
  // sfr = sum V F r, sfrr = sum V F r r^T (symmetric, upper part), b0 =
  // sum m w, bf = sum m F r; and the Shepard velocity sum
  double sw = 0.0, swr[3] = {0.0, 0.0, 0.0}, sfr[3] = {0.0, 0.0, 0.0};
  double sfrr[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double b0 = 0.0, bf[3] = {0.0, 0.0, 0.0}, sv[3] = {0.0, 0.0, 0.0};
  // the ghost node in the view's frame: fixed-point x (as the reorder writes
  // it), y and z relative to the ghost's cell
  const double fr = (g[0] - kp.ox) * kp.inv_frame;
  const uint32_t xg = (uint32_t)(uint64_t)((fr - floor(fr)) * 4294967296.0);
  const float yg = DIM >= 2 ? (float)(g[1] - (kp.oy + (double)c[1] * kp.cs)) : 0.f;
  const float zg = DIM == 3 ? (float)(g[2] - (kp.oz + (double)c[2] * kp.cs)) : 0.f;
  const int fcells = kFrameCells << kp.lg_xsub;
  const float fx =
      (float)(int32_t)(xg - ((uint32_t)(c[0] % fcells) << (29 - kp.lg_xsub))) * kp.unit_x_f;
  const float cs = kp.cs_f;
  // rows cut with the support enlarged by 2e-4 (far above the FP32 error)
  const float pre2 = kp.support2_f * 1.0002f;
  const float mf_f = (float)kp.mass_f;
  const int reach = R * kp.x_sub;
  const int xlo = c[0] - reach < 0 ? 0 : c[0] - reach;
  const int xhi = c[0] + reach >= kp.ncx ? kp.ncx - 1 : c[0] + reach;
  const int zlo = DIM == 3 ? -R : 0, zhi = DIM == 3 ? R : 0;
  for (int dz = zlo; dz <= (inside ? zhi : zlo - 1); ++dz) {
    const int z = c[2] + dz;
    if (z < 0 || z >= kp.ncz) continue;
    const float ez0 = (float)dz * cs - zg;
    const float ez = DIM == 3 ? (dz > 0 ? ez0 : (dz < 0 ? -(ez0 + cs) : 0.f)) : 0.f;
    for (int dy = -R; dy <= R; ++dy) {
      const int y = c[1] + dy;
      if (y < 0 || y >= kp.ncy) continue;
      const float ey0 = (float)dy * cs - yg;
      const float ey = dy > 0 ? ey0 : (dy < 0 ? -(ey0 + cs) : 0.f);
      const float w2 = pre2 - ey * ey - ez * ez;
      if (!(w2 > 0.f)) continue;
      const float wx = sqrtf(w2);
      int x0 = c[0] + (int)floorf((fx - wx) * kp.inv_csx_f);
      int x1 = c[0] + (int)floorf((fx + wx) * kp.inv_csx_f);
      x0 = x0 < xlo ? xlo : x0;
      x1 = x1 > xhi ? xhi : x1;
      const uint32_t row = (uint32_t)kp.ncx * ((uint32_t)y + (uint32_t)kp.ncy * (uint32_t)z);
      const uint32_t j1 = cstart[row + x1 + 1];
      const float ys = yg - (float)dy * cs, zs = zg - (float)dz * cs;
      for (uint32_t j = cstart[row + x0]; j < j1; ++j) {
        const float4 pb = pr[j];
        if (!(pb.w > 0.f)) continue;  // fluid particles only
        // r = r_b - r_G from the view's offsets (FP32)
        const float rx = (float)(int32_t)(__float_as_uint(pb.x) - xg) * kp.unit_x_f;
        const float ry = pb.y - ys, rz = DIM == 3 ? pb.z - zs : 0.f;
        const float r2 = rx * rx + ry * ry + rz * rz;
        if (!(r2 < kp.support2_f)) continue;
        float w, f;
        kernel_wf32(kp, sqrtf(r2), w, f);
        const float vbf = mf_f / pb.w;
        const double vw = (double)(vbf * w), vf = (double)(vbf * f);
        const double mw = (double)(mf_f * w), mf = (double)(mf_f * f);
        const double r[3] = {(double)rx, (double)ry, (double)rz};
        sw += vw;
        b0 += mw;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
          swr[a] += vw * r[a];
          sfr[a] += vf * r[a];
          bf[a] += mf * r[a];
        }
        sfrr[0] += vf * r[0] * r[0];
        sfrr[1] += vf * r[0] * r[1];
        sfrr[3] += vf * r[1] * r[1];
        if (DIM == 3) {
          sfrr[2] += vf * r[0] * r[2];
          sfrr[4] += vf * r[1] * r[2];
          sfrr[5] += vf * r[2] * r[2];
        }
        const float4 v = vp[j];
        sv[0] += vw * (double)v.x;
        sv[1] += vw * (double)v.y;
        if (DIM == 3) sv[2] += vw * (double)v.z;
      }
    }
  }
  double rho_b = kp.rho0;
  double vout[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int d = 0; d < DIM; ++d) vout[d] = (double)s.vel[d * n + i];
  if (sw > 0.0) {
    double A[M][M], x[M];
    A[0][0] = sw;
    x[0] = b0;
    const int sym[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      A[0][1 + a] = swr[a];
      A[1 + a][0] = sfr[a];
      x[1 + a] = bf[a];
#pragma unroll
      for (int k = 0; k < DIM; ++k) A[1 + a][1 + k] = sfrr[sym[a][k]];
    }
    const double det = solve_small<M>(A, x);
    if (fabs(det) >= 1e-3) {
      rho_b = x[0];
#pragma unroll
      for (int d = 0; d < DIM; ++d) rho_b += (rb[d] - g[d]) * x[1 + d];
    } else {
      rho_b = b0 / sw;
    }
#pragma unroll
    for (int d = 0; d < DIM; ++d) vout[d] = 2.0 * vout[d] - sv[d] / sw;
  }
  const float rf = (float)rho_b;
  s.rho[i] = rf;
  pr[i].w = -rf;
  const double pw = tait_ratio(kp, (double)rf);
  vp[i] = make_float4((float)vout[0], (float)vout[1], DIM == 3 ? (float)vout[2] : 0.f,
                      (float)(kp.b_tait * pw));
}

hipError_t launch_mdbc(const KParams& kp, int64_t n, const sph_state& s, const uint32_t* key,
                       const uint32_t* cell_start, void* ws, hipStream_t st) {
  (void)key;
  const WsLayout L = ws_layout(n);
  float4* pr = ws_ptr<float4>(ws, L.view_pr);
  float4* vp = ws_ptr<float4>(ws, L.view_vp);
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
#define SPH_MDBC(D, RR) \
  hipLaunchKernelGGL((k_mdbc<D, RR>), dim3(grid), dim3(kBlock), 0, st, kp, n, s, cell_start, pr, vp)
  if (kp.dim == 2) {
    if (kp.cell_div == 1) SPH_MDBC(2, 1); else SPH_MDBC(2, 2);
  } else {
    if (kp.cell_div == 1) SPH_MDBC(3, 1); else SPH_MDBC(3, 2);
  }
#undef SPH_MDBC
  return hipGetLastError();
}

}  // namespace sph
