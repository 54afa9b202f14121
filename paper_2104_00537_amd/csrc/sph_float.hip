// Rigid floating bodies (Section 3.2, Eq. 47-50 of the DualSPHysics v5.0
// paper) on gfx950: per-body force, torque and inertia from the
// interaction's per-particle accelerations, the symplectic update of each
// body (Section 2.5.2 applied to its centre and orientation), and the rigid
// motion of its particles.
//
// A body's particles are found through an id map: body b owns the dense
// slots [base_b, base_b + count_b) (bodies laid out in table order) and
// particle id id_first_b + k sits in slot base_b + k.  One pass over the
// sorted state writes each floating particle's sorted index into its slot;
// the reductions and the motion then walk the slots of each body in id
// order, so sums are taken in a fixed order whatever the particle order.
// A slot is trusted only if the particle it names carries the slot's id and
// is a live floating particle (stale entries from earlier calls never pass).
#include "sph_kernels.h"

namespace sph {

// Motion of one body for the particle pass, in the workspace (kFloatMotion
// doubles): rotation matrix, centre before (state n) and after, velocity and
// angular velocity after the phase.
struct BodyMotion {
  double q[9];
  double from[3], to[3];
  double vel[3], omega[3];
  double pad[3];
};
static_assert(sizeof(BodyMotion) == kFloatMotion * sizeof(double), "motion record size");

// First dense slot of body b (sum of the counts before it).
__device__ inline int64_t body_base(const sph_body* __restrict__ bodies, int b) {
  int64_t base = 0;
  for (int k = 0; k < b; ++k) base += bodies[k].count;
  return base;
}

// -------------------------------------------------------------- id map --
__global__ __launch_bounds__(kBlock) void k_float_map(int64_t n, const uint8_t* __restrict__ type,
                                                      const uint32_t* __restrict__ id,
                                                      const sph_body* __restrict__ bodies, int nb,
                                                      uint32_t* __restrict__ map,
                                                      uint32_t* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint8_t t = type[i];
  if (!is_floating(t) || is_excluded(t)) return;
  const int64_t pid = (int64_t)id[i];
  int64_t base = 0;
  for (int b = 0; b < nb; ++b) {
    const int64_t f = bodies[b].id_first, c = bodies[b].count;
    if (pid >= f && pid < f + c) {
      const int64_t slot = base + (pid - f);
      if (slot < n)
        map[slot] = (uint32_t)i;
      else
        set_error(err, SPH_ERR_FLOATING);
      return;
    }
    base += c;
  }
  set_error(err, SPH_ERR_FLOATING);  // a floating particle of no body
}

// The sorted index of slot k of a body, or -1 if the slot names no live
// floating particle with the slot's id.
__device__ inline int64_t slot_particle(int64_t n, const uint32_t* __restrict__ map,
                                        const uint8_t* __restrict__ type,
                                        const uint32_t* __restrict__ id, int64_t slot,
                                        int64_t want_id) {
  if (slot >= n) return -1;
  const uint32_t i = map[slot];
  if ((int64_t)i >= n) return -1;
  const uint8_t t = type[i];
  if (!is_floating(t) || is_excluded(t) || (int64_t)id[i] != want_id) return -1;
  return (int64_t)i;
}

__device__ inline double wave_sum_f64(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ------------------------------------------------------- body reduction --
// Block (part, body): the slots part*kBlock + tid + j*kFloatParts*kBlock of
// the body.  Partial sums (FP64): sum a (dim), sum r' x a (3 or 1), the
// unweighted inertia sum(|r'|^2 1 - r' r'^T) (6 unique entries xx yy zz xy
// xz yz, or |r'|^2 in 2-D) and the particle count; r' = r - R0 (current).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_float_reduce(
    int64_t n, const sph_body* __restrict__ bodies, const uint32_t* __restrict__ map,
    const uint8_t* __restrict__ type, const uint32_t* __restrict__ id,
    const double* __restrict__ pos, const float* __restrict__ ace, double* __restrict__ part) {
  const int b = blockIdx.y, p = blockIdx.x;
  const int64_t base = body_base(bodies, b);
  const int64_t first = bodies[b].id_first, count = bodies[b].count;
  double c[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < DIM; ++d) c[d] = bodies[b].center[d];
  double s[kFloatSums];
#pragma unroll
  for (int j = 0; j < kFloatSums; ++j) s[j] = 0.0;
  for (int64_t k = (int64_t)p * kBlock + threadIdx.x; k < count;
       k += (int64_t)kFloatParts * kBlock) {
    const int64_t i = slot_particle(n, map, type, id, base + k, first + k);
    if (i < 0) continue;
    double r[3] = {0.0, 0.0, 0.0}, a[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < DIM; ++d) {
      r[d] = pos[d * n + i] - c[d];
      a[d] = (double)ace[d * n + i];
      s[d] += a[d];
    }
    if (DIM == 2) {
      s[3] += r[0] * a[1] - r[1] * a[0];
      s[6] += r[0] * r[0] + r[1] * r[1];
    } else {
      s[3] += r[1] * a[2] - r[2] * a[1];
      s[4] += r[2] * a[0] - r[0] * a[2];
      s[5] += r[0] * a[1] - r[1] * a[0];
      const double xx = r[0] * r[0], yy = r[1] * r[1], zz = r[2] * r[2];
      s[6] += yy + zz;
      s[7] += xx + zz;
      s[8] += xx + yy;
      s[9] -= r[0] * r[1];
      s[10] -= r[0] * r[2];
      s[11] -= r[1] * r[2];
    }
    s[12] += 1.0;
  }
  __shared__ double sh[kBlock / 64][kFloatSums];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kFloatSums; ++j) {
    const double v = wave_sum_f64(s[j]);
    if (lane == 0) sh[wave][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < kFloatSums) {
    double v = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) v += sh[w][threadIdx.x];
    part[((int64_t)b * kFloatParts + p) * kFloatSums + threadIdx.x] = v;
  }
}

// Rotation matrix of the rotation vector th (right-handed about th, by the
// angle |th|): Q = 1 + (sin f / f) K + ((1 - cos f) / f^2) K^2 with K the
// cross-product matrix of th and f = |th|; the last factor is evaluated as
// 2 sin^2(f/2) / f^2 (no cancellation), and for tiny f both factors by the
// first two terms of their series.  2-D: the plane rotation by th[0].
template <int DIM>
__device__ inline void rotation_matrix(const double* th, double* q) {
  if (DIM == 2) {
    const double cs = cos(th[0]), sn = sin(th[0]);
    q[0] = cs; q[1] = -sn; q[2] = 0.0;
    q[3] = sn; q[4] = cs;  q[5] = 0.0;
    q[6] = 0.0; q[7] = 0.0; q[8] = 1.0;
    return;
  }
  const double f2 = th[0] * th[0] + th[1] * th[1] + th[2] * th[2];
  const double f = sqrt(f2);
  double a, b;
  if (f < 1e-4) {
    a = 1.0 - f2 / 6.0;
    b = 0.5 - f2 / 24.0;
  } else {
    a = sin(f) / f;
    const double hs = sin(0.5 * f) / f;
    b = 2.0 * hs * hs;
  }
  const double K[9] = {0.0, -th[2], th[1], th[2], 0.0, -th[0], -th[1], th[0], 0.0};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double k2 = 0.0;
      for (int m = 0; m < 3; ++m) k2 += K[r * 3 + m] * K[m * 3 + c];
      q[r * 3 + c] = (r == c ? 1.0 : 0.0) + a * K[r * 3 + c] + b * k2;
    }
}

// ------------------------------------------------------- body update --
// One thread per body: totals of the partial sums (fixed order), Eq. 48-49,
// the phase's update of the body state and the motion record.
template <int DIM, int PHASE>
__global__ void k_float_finish(KParams kp, const double* __restrict__ dtp,
                               sph_body* __restrict__ bodies, int nb,
                               const double* __restrict__ part, BodyMotion* __restrict__ motion,
                               uint32_t* __restrict__ err) {
  const int b = threadIdx.x;
  if (b >= nb) return;
  double s[kFloatSums];
  for (int j = 0; j < kFloatSums; ++j) s[j] = 0.0;
  for (int p = 0; p < kFloatParts; ++p)
    for (int j = 0; j < kFloatSums; ++j) s[j] += part[((int64_t)b * kFloatParts + p) * kFloatSums + j];
  sph_body& B = bodies[b];
  const double dt = *dtp;
  const double M = B.mass;
  const double mb = kp.mass_b, mi = M / (double)B.count;
  if (s[12] != (double)B.count) set_error(err, SPH_ERR_FLOATING);
  const double g[3] = {kp.gx, kp.gy, kp.gz};
  double F[3] = {0.0, 0.0, 0.0}, T[3] = {0.0, 0.0, 0.0}, A[3] = {0.0, 0.0, 0.0};
  double al[3] = {0.0, 0.0, 0.0};
  // (a 2-D case holds its gravity in components 0 and 1, like its positions)
  for (int d = 0; d < DIM; ++d) {
    F[d] = mb * s[d];
    A[d] = F[d] / M + g[d];
  }
  if (DIM == 2) {
    T[0] = mb * s[3];
    const double I = mi * s[6];
    if (I > 0.0) al[0] = T[0] / I;
    else set_error(err, SPH_ERR_FLOATING);
  } else {
    for (int d = 0; d < 3; ++d) T[d] = mb * s[3 + d];
    const double ixx = mi * s[6], iyy = mi * s[7], izz = mi * s[8];
    const double ixy = mi * s[9], ixz = mi * s[10], iyz = mi * s[11];
    // adjugate of the symmetric inertia tensor
    const double c00 = iyy * izz - iyz * iyz, c01 = ixz * iyz - ixy * izz;
    const double c02 = ixy * iyz - ixz * iyy, c11 = ixx * izz - ixz * ixz;
    const double c12 = ixy * ixz - ixx * iyz, c22 = ixx * iyy - ixy * ixy;
    const double det = ixx * c00 + ixy * c01 + ixz * c02;
    const double tr = ixx + iyy + izz;
    if (det > 1e-12 * tr * tr * tr / 27.0) {
      al[0] = (c00 * T[0] + c01 * T[1] + c02 * T[2]) / det;
      al[1] = (c01 * T[0] + c11 * T[1] + c12 * T[2]) / det;
      al[2] = (c02 * T[0] + c12 * T[1] + c22 * T[2]) / det;
    } else {
      set_error(err, SPH_ERR_FLOATING);
    }
  }
  for (int d = 0; d < 3; ++d) {
    B.force[d] = F[d];
    B.torque[d] = T[d];
  }
  const int nw = DIM == 2 ? 1 : 3;
  double th[3] = {0.0, 0.0, 0.0};
  if (PHASE == 0) {
    for (int d = 0; d < 3; ++d) {
      B.center_n[d] = B.center[d];
      B.vel_n[d] = B.vel[d];
      B.omega_n[d] = B.omega[d];
    }
    for (int d = 0; d < DIM; ++d) {
      B.center[d] = B.center_n[d] + 0.5 * dt * B.vel_n[d];
      B.vel[d] = B.vel_n[d] + 0.5 * dt * A[d];
    }
    for (int d = 0; d < nw; ++d) {
      th[d] = 0.5 * dt * B.omega_n[d];
      B.omega[d] = B.omega_n[d] + 0.5 * dt * al[d];
    }
  } else {
    for (int d = 0; d < DIM; ++d) {
      B.vel[d] = B.vel_n[d] + dt * A[d];
      B.center[d] = B.center_n[d] + dt * 0.5 * (B.vel[d] + B.vel_n[d]);
    }
    for (int d = 0; d < nw; ++d) {
      B.omega[d] = B.omega_n[d] + dt * al[d];
      th[d] = dt * 0.5 * (B.omega[d] + B.omega_n[d]);
    }
  }
  BodyMotion m{};
  rotation_matrix<DIM>(th, m.q);
  for (int d = 0; d < 3; ++d) {
    m.from[d] = B.center_n[d];
    m.to[d] = B.center[d];
    m.vel[d] = B.vel[d];
    m.omega[d] = B.omega[d];
  }
  motion[b] = m;
}

// ------------------------------------------------------ particle motion --
// r_k = R0 + Q (r_k^n - R0^n), v_k = V + Omega x (r_k - R0) (Eq. 50), from
// the saved state n.
// With disp (the predictor), also records the largest distance moved.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_float_move(
    int64_t n, const sph_body* __restrict__ bodies, const uint32_t* __restrict__ map,
    const uint8_t* __restrict__ type, const uint32_t* __restrict__ id,
    const BodyMotion* __restrict__ motion, const double* __restrict__ pos_n,
    double* __restrict__ pos, float* __restrict__ vel, uint32_t* __restrict__ disp) {
  const int b = blockIdx.y, p = blockIdx.x;
  const int64_t base = body_base(bodies, b);
  const int64_t first = bodies[b].id_first, count = bodies[b].count;
  const BodyMotion& m = motion[b];
  double dmax2 = 0.0;
  for (int64_t k = (int64_t)p * kBlock + threadIdx.x; k < count;
       k += (int64_t)kFloatParts * kBlock) {
    const int64_t i = slot_particle(n, map, type, id, base + k, first + k);
    if (i < 0) continue;
    double r0[3] = {0.0, 0.0, 0.0}, r[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < DIM; ++d) r0[d] = pos_n[d * n + i] - m.from[d];
    for (int d = 0; d < DIM; ++d) {
      double v = 0.0;
      for (int e = 0; e < DIM; ++e) v += m.q[d * 3 + e] * r0[e];
      r[d] = v;
    }
    double w[3];
    if (DIM == 2) {
      w[0] = -m.omega[0] * r[1];
      w[1] = m.omega[0] * r[0];
    } else {
      w[0] = m.omega[1] * r[2] - m.omega[2] * r[1];
      w[1] = m.omega[2] * r[0] - m.omega[0] * r[2];
      w[2] = m.omega[0] * r[1] - m.omega[1] * r[0];
    }
    double d2 = 0.0;
    for (int d = 0; d < DIM; ++d) {
      const double x1 = m.to[d] + r[d];
      d2 += (x1 - pos[d * n + i]) * (x1 - pos[d * n + i]);
      pos[d * n + i] = x1;
      vel[d * n + i] = (float)(m.vel[d] + w[d]);
    }
    dmax2 = d2 > dmax2 ? d2 : dmax2;
  }
  if (disp) record_displacement(dmax2, disp);
}

hipError_t launch_floating(const KParams& kp, int64_t n, int phase, const double* dt,
                           sph_body* bodies, int nb, const sph_state& saved, sph_state& s,
                           const float* ace, void* ws, hipStream_t st) {
  const WsLayout L = ws_layout(n);
  uint32_t* err = &ws_ptr<WsHeader>(ws, L.err)->err;
  uint32_t* map = ws_ptr<uint32_t>(ws, L.keyB);
  double* part = ws_ptr<double>(ws, L.fpart);
  BodyMotion* motion = ws_ptr<BodyMotion>(ws, L.fmotion);
  // the predictor's moves count towards the displacement since the binning
  uint32_t* disp = phase == 0 ? ws_ptr<uint32_t>(ws, L.disp) : nullptr;
  if (n > 0) {
    const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_float_map, dim3(grid), dim3(kBlock), 0, st, n, s.type, s.id, bodies, nb,
                       map, err);
  }
  const dim3 g2(kFloatParts, (unsigned)nb);
  if (kp.dim == 2) {
    hipLaunchKernelGGL(k_float_reduce<2>, g2, dim3(kBlock), 0, st, n, bodies, map, s.type, s.id,
                       s.pos, ace, part);
    if (phase == 0)
      hipLaunchKernelGGL((k_float_finish<2, 0>), dim3(1), dim3(64), 0, st, kp, dt, bodies, nb,
                         part, motion, err);
    else
      hipLaunchKernelGGL((k_float_finish<2, 1>), dim3(1), dim3(64), 0, st, kp, dt, bodies, nb,
                         part, motion, err);
    hipLaunchKernelGGL(k_float_move<2>, g2, dim3(kBlock), 0, st, n, bodies, map, s.type, s.id,
                       motion, saved.pos, s.pos, s.vel, disp);
  } else {
    hipLaunchKernelGGL(k_float_reduce<3>, g2, dim3(kBlock), 0, st, n, bodies, map, s.type, s.id,
                       s.pos, ace, part);
    if (phase == 0)
      hipLaunchKernelGGL((k_float_finish<3, 0>), dim3(1), dim3(64), 0, st, kp, dt, bodies, nb,
                         part, motion, err);
    else
      hipLaunchKernelGGL((k_float_finish<3, 1>), dim3(1), dim3(64), 0, st, kp, dt, bodies, nb,
                         part, motion, err);
    hipLaunchKernelGGL(k_float_move<3>, g2, dim3(kBlock), 0, st, n, bodies, map, s.type, s.id,
                       motion, saved.pos, s.pos, s.vel, disp);
  }
  return hipGetLastError();
}

}  // namespace sph
