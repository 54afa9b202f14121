// Modified dynamic boundary condition (Section 2.6.2 of the DualSPHysics
// v5.0 paper, Eq. 38-39): wall densities and velocities from ghost nodes.
//
// A first kernel lists the wall particles; then one lane per listed wall.  Its ghost node G = r_B +
// normal_B is binned like a particle; the rows of G's neighbour cells are
// walked as in the interaction (one range per row, cut to the support sphere
// of G), candidates are screened in FP32 on the view's offsets with a margin,
// and the pairs that pass are tested and summed in FP64 on the FP64
// positions.  The (d+1) x (d+1) corrected system is
// solved by Gaussian elimination with partial pivoting in registers.  Only
// wall entries of the state density and of the interaction view are written;
// the fluid entries that the walk reads are never changed, and the sign of a
// wall's view density (the only thing read of a wall candidate) stays
// negative.
#include "sph_dev.h"
#include "sph_kernels.h"

namespace sph {

// Kernel value and gradient factor (grad W = F r) in FP64: Wendland C2
// (Eq. 11), W = alpha_D (1 - q/2)^4 (2q + 1), F = kfab (1 - q/2)^3, or cubic
// spline (Eq. 10), with alpha_D and kfab of the case.
__device__ inline void kernel_wf64(const KParams& kp, double r, double& w, double& f) {
  const double q = r * kp.inv_h;
  if (kp.kernel == 0) {
    const double u = 1.0 - 0.5 * q;
    const double u3 = u * u * u;
    w = kp.w_alpha * u3 * u * (2.0 * q + 1.0);
    f = kp.f_coef * u3;
  } else if (q <= 1.0) {
    w = kp.w_alpha * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
    f = kp.f_coef * (-3.0 + 2.25 * q);
  } else {
    const double u = 2.0 - q;
    w = kp.w_alpha * 0.25 * u * u * u;
    f = -0.75 * kp.f_coef * u * u / q;
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

__global__ void k_zero_wall_count(WsHeader* __restrict__ hdr) {
  if (threadIdx.x == 0) hdr->nwall = 0u;
}

// The wall particles (not excluded) of the sorted state, appended to a work
// list in any order (one atomic per wave); each wall's result depends only on
// its own inputs, so the order does not matter.
__global__ __launch_bounds__(kBlock) void k_wall_list(int64_t n, const uint8_t* __restrict__ type,
                                                      uint32_t* __restrict__ list,
                                                      WsHeader* __restrict__ hdr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool wall = i < n && !is_excluded(type[i]) && !is_fluid(type[i]);
  const uint64_t mask = __ballot(wall);
  if (mask == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int leader = (int)__builtin_ctzll(mask);
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(&hdr->nwall, (uint32_t)__popcll(mask));
  base = __shfl(base, leader, 64);
  if (wall) {
    const uint64_t below = lane == 0 ? 0ull : (mask & (~0ull >> (64 - lane)));
    list[base + (uint32_t)__popcll(below)] = (uint32_t)i;
  }
}

template <int DIM, int R>
__global__ __launch_bounds__(kBlock) void k_mdbc(KParams kp, int64_t n, sph_state s,
                                                 const uint32_t* __restrict__ cstart,
                                                 float4* __restrict__ pr,
                                                 float4* __restrict__ vp,
                                                 const uint32_t* __restrict__ list,
                                                 const WsHeader* __restrict__ hdr) {
  constexpr int M = DIM + 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)hdr->nwall) return;
  const int64_t i = list[t];
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
  // FP32 pre-test with a margin far above its rounding; the FP64 test on the
  // FP64 positions decides
  const float pre2 = kp.support2_f * 1.0002f;
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
      // groups of 4 candidates: their views are loaded together (padded), the
      // screened ones then load their FP64 positions and velocities together
      for (uint32_t j = cstart[row + x0]; j < j1; j += 4) {
        const float4* q = pr + j;
        float4 pb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pb[u] = q[u];
        bool hit[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float ex = (float)(int32_t)(xg - __float_as_uint(pb[u].x)) * kp.unit_x_f;
          const float ey1 = ys - pb[u].y, ez1 = DIM == 3 ? zs - pb[u].z : 0.f;
          hit[u] = j + u < j1 && pb[u].w > 0.f && ex * ex + ey1 * ey1 + ez1 * ez1 < pre2;
        }
        double pbx[4][3];
        float4 vb4[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (hit[u]) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) pbx[u][d] = s.pos[d * n + j + u];
            vb4[u] = vp[j + u];
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (!hit[u]) continue;
          double r[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
#pragma unroll
          for (int d = 0; d < DIM; ++d) {
            r[d] = pbx[u][d] - g[d];
            r2 += r[d] * r[d];
          }
          if (!(r2 < kp.support2)) continue;
          double w, f;
          kernel_wf64(kp, sqrt(r2), w, f);
          const double mb = kp.mass_f;
          const double vb = mb / (double)pb[u].w;
          const double vw = vb * w, vf = vb * f;
          sw += vw;
          b0 += mb * w;
#pragma unroll
          for (int a = 0; a < DIM; ++a) {
            swr[a] += vw * r[a];
            sfr[a] += vf * r[a];
            bf[a] += mb * f * r[a];
          }
          sfrr[0] += vf * r[0] * r[0];
          sfrr[1] += vf * r[0] * r[1];
          sfrr[3] += vf * r[1] * r[1];
          if (DIM == 3) {
            sfrr[2] += vf * r[0] * r[2];
            sfrr[4] += vf * r[1] * r[2];
            sfrr[5] += vf * r[2] * r[2];
          }
          sv[0] += vw * (double)vb4[u].x;
          sv[1] += vw * (double)vb4[u].y;
          if (DIM == 3) sv[2] += vw * (double)vb4[u].z;
        }
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
  WsHeader* hdr = ws_ptr<WsHeader>(ws, L.err);
  // the work list lives in the sort's key buffer, free once the cells are
  // binned (sph_bin_cells must not run between this and the next launch)
  uint32_t* list = ws_ptr<uint32_t>(ws, L.keyA);
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_zero_wall_count, dim3(1), dim3(64), 0, st, hdr);
  hipLaunchKernelGGL(k_wall_list, dim3(grid), dim3(kBlock), 0, st, n, s.type, list, hdr);
#define SPH_MDBC(D, RR)                                                                    \
  hipLaunchKernelGGL((k_mdbc<D, RR>), dim3(grid), dim3(kBlock), 0, st, kp, n, s, cell_start, \
                     pr, vp, list, hdr)
  if (kp.dim == 2) {
    if (kp.cell_div == 1) SPH_MDBC(2, 1); else SPH_MDBC(2, 2);
  } else {
    if (kp.cell_div == 1) SPH_MDBC(3, 1); else SPH_MDBC(3, 2);
  }
#undef SPH_MDBC
  return hipGetLastError();
}

}  // namespace sph
