// Per-particle device routines shared by the single-case and the batched
// kernels: the cell key, the sorted-order gather with its interaction view,
// and the symplectic update (Sections 2.5.2 and 5.1 of the DualSPHysics v5.0
// paper).
#pragma once

#include "sph_internal.h"

namespace sph {

// Along a periodic component k (period L > 0, Section 2.7) a coordinate that
// left [o, o + L) re-enters at the other end: x - L, or x + L (o if that
// rounds to o + L).
__device__ inline double wrap_coord(const KParams& kp, int k, double x) {
  const double L = k == 0 ? kp.px : (k == 1 ? kp.py : kp.pz);
  if (!(L > 0.0)) return x;
  const double o = k == 0 ? kp.ox : (k == 1 ? kp.oy : kp.oz);
  if (x >= o + L) return __dsub_rn(x, L);
  if (x < o) {
    x = __dadd_rn(x, L);
    if (x >= o + L) x = o;
  }
  return x;
}

// Cell index per axis = floor((x - origin) * inv): one FP64 subtraction and
// one FP64 multiplication (no contraction is possible), x fastest; inv is the
// inverse cell size, times x_sub along x.  Outside
// the grid, and for particles excluded earlier, the key is ncell_total, so
// they sort last and lie in no cell range.  Periodic components take the
// wrapped coordinate (and its last cell if the product rounds up to the
// end).
__device__ inline uint32_t cell_key_local(const KParams& kp, const double* __restrict__ pos,
                                          const uint8_t* __restrict__ type, int64_t n,
                                          int64_t i) {
  if (is_excluded(type[i])) return kp.ncell_total;
  const double org[3] = {kp.ox, kp.oy, kp.oz};
  const int nc[3] = {kp.ncx, kp.ncy, kp.ncz};
  int c[3] = {0, 0, 0};
  for (int k = 0; k < kp.dim; ++k) {
    const double d = __dsub_rn(wrap_coord(kp, k, pos[k * n + i]), org[k]);
    const double s = __dmul_rn(d, k == 0 ? kp.inv_csx : kp.inv_cs);
    double f = floor(s);
    if (((kp.periodic >> k) & 1) && f == (double)nc[k]) f -= 1.0;
    if (!(f >= 0.0) || !(f < (double)nc[k])) return kp.ncell_total;
    c[k] = (int)f;
  }
  return (uint32_t)(c[0] + nc[0] * (c[1] + nc[1] * c[2]));
}

// (rho/rho0)^gamma - 1 of the Tait equation (Eq. 28: P = B_t times this), in
// FP64; for gamma = 7 as the expansion of (1+u)^7 - 1 in u = rho/rho0 - 1,
// which keeps the small pressures of a nearly incompressible fluid free of
// cancellation.
__device__ inline double tait_ratio(const KParams& kp, double r) {
  const double u = r / kp.rho0 - 1.0;
  if (kp.gamma == 7.0)
    return u * (7.0 + u * (21.0 + u * (35.0 + u * (35.0 + u * (21.0 + u * (7.0 + u))))));
  return pow(r / kp.rho0, kp.gamma) - 1.0;
}

__device__ inline void write_view(const KParams& kp, int64_t i, const double* x, const float* v,
                                  float rho, uint8_t t, uint32_t lkey, float4* __restrict__ pr,
                                  float4* __restrict__ vp);

// Gathers particle src into sorted slot i and writes the two float4 the
// interaction reads (the "view"):
//   pr = {local position (dim components), 0, +rho fluid / -rho wall}
//   vp = {velocity (dim components), 0, P}
// lkey is the particle's key relative to its case.  Local positions follow
// the precision scheme of Section 5.1 (FP64 positions, short FP32 distances,
// so the error does not grow with the domain): along y and z the FP32 offset
// x - (origin + c cs) from the particle's cell, evaluated in FP64; along x a
// 32-bit fixed-point position modulo kFrameCells cells (the bits are stored
// in the float slot), whose differences are exact modulo that period.  P is the
// Tait pressure of Eq. 28, per particle in FP64 (tait_ratio).  Returns true if
// the particle was excluded by this call (it left the grid).
__device__ inline bool reorder_one(const KParams& kp, int64_t n, int64_t i, int64_t src,
                                   uint32_t lkey, const sph_state& in, const sph_state& out,
                                   const sph_state& cin, const sph_state& cout, int carry,
                                   float4* __restrict__ pr, float4* __restrict__ vp) {
  double x[3] = {0.0, 0.0, 0.0};
  float v[3] = {0.f, 0.f, 0.f};
  const bool live = !(in.type[src] & SPH_EXCLUDED);
  for (int d = 0; d < kp.dim; ++d) {
    x[d] = in.pos[d * n + src];
    if (live) x[d] = wrap_coord(kp, d, x[d]);
    v[d] = in.vel[d * n + src];
    out.pos[d * n + i] = x[d];
    out.vel[d * n + i] = v[d];
  }
  const float rho = in.rho[src];
  out.rho[i] = rho;
  uint8_t t = in.type[src];
  bool newly = false;
  if (lkey == kp.ncell_total && !(t & SPH_EXCLUDED)) {
    t |= SPH_EXCLUDED;
    newly = true;
  }
  out.type[i] = t;
  if (in.id && out.id) out.id[i] = in.id[src];
  if (in.normal && out.normal)
    for (int d = 0; d < kp.dim; ++d) out.normal[d * n + i] = in.normal[d * n + src];
  if (in.vel64 && out.vel64) {  // an all-FP64 state's velocities and densities
    for (int d = 0; d < kp.dim; ++d) out.vel64[d * n + i] = in.vel64[d * n + src];
    out.rho64[i] = in.rho64[src];
  }
  if (carry) {
    for (int d = 0; d < kp.dim; ++d) {
      cout.pos[d * n + i] = cin.pos[d * n + src];
      cout.vel[d * n + i] = cin.vel[d * n + src];
    }
    cout.rho[i] = cin.rho[src];
    if (cin.vel64 && cout.vel64) {
      for (int d = 0; d < kp.dim; ++d) cout.vel64[d * n + i] = cin.vel64[d * n + src];
      cout.rho64[i] = cin.rho64[src];
    }
  }
  if (t & SPH_EXCLUDED) {
    pr[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    vp[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    return newly;
  }
  write_view(kp, i, x, v, rho, t, lkey, pr, vp);
  return newly;
}

// The view entry of sorted slot i (a live particle) from its position x
// (FP64), velocity v, density rho and type t, relative to the cell of key
// lkey (see reorder_one).  The position may lie slightly outside that cell
// (a view refreshed after the particle moved): the offsets then fall
// outside [0, cs), which the interaction handles like any other.
__device__ inline void write_view(const KParams& kp, int64_t i, const double* x, const float* v,
                                  float rho, uint8_t t, uint32_t lkey, float4* __restrict__ pr,
                                  float4* __restrict__ vp) {
  const int c0 = (int)(lkey % (uint32_t)kp.ncx);
  const uint32_t rest = lkey / (uint32_t)kp.ncx;
  const int c[3] = {c0, (int)(rest % (uint32_t)kp.ncy), (int)(rest / (uint32_t)kp.ncy)};
  const double org[3] = {kp.ox, kp.oy, kp.oz};
  float o[3] = {0.f, 0.f, 0.f};
  for (int d = 1; d < kp.dim; ++d) o[d] = (float)(x[d] - (org[d] + (double)c[d] * kp.cs));
  // x: fixed-point position modulo kFrameCells cells, 2^32 units per period
  const double fr = (x[0] - org[0]) * kp.inv_frame;
  const double f = fr - floor(fr);
  o[0] = __uint_as_float((uint32_t)(uint64_t)(f * 4294967296.0));
  const double pw = tait_ratio(kp, (double)rho);
  pr[i] = make_float4(o[0], o[1], o[2], is_fluid(t) ? rho : -rho);
  vp[i] = make_float4(v[0], v[1], v[2], (float)(kp.b_tait * pw));
}

// Imposed wall motion along x: D(t) = (A/w^2)(1 - cos wt), v(t) = (A/w) sin wt.
__device__ inline double motion_disp(const KParams& kp, double t) {
  if (kp.motion_omega == 0.0) return 0.0;
  const double w = kp.motion_omega;
  return kp.motion_amp / (w * w) * (1.0 - cos(w * t));
}
__device__ inline double motion_vel(const KParams& kp, double t) {
  if (kp.motion_omega == 0.0) return 0.0;
  return kp.motion_amp / kp.motion_omega * sin(kp.motion_omega * t);
}

// One particle of the symplectic update: PHASE 0 is the predictor (Eq. 33
// lines 1-2, Eq. 34 line 1) and saves state n; PHASE 1 the corrector (Eq. 33
// lines 3-4, Eq. 34 line 2) from the saved state.  dmove / vmove are the
// imposed wall displacement since t and velocity at the phase's end time.
// Returns true if the new state is not finite or the density not positive.
// disp2 (PHASE 0) receives the squared distance the particle moved.
template <int PHASE>
__device__ inline bool symplectic_one(const KParams& kp, int64_t n, int64_t i, double dt,
                                      double dmove, double vmove, const sph_state& saved,
                                      const sph_state& s, const float* __restrict__ ace,
                                      const float* __restrict__ arho, double& disp2) {
  const uint8_t t = s.type[i];
  if (PHASE == 0) {
    for (int d = 0; d < kp.dim; ++d) {
      saved.pos[d * n + i] = s.pos[d * n + i];
      saved.vel[d * n + i] = s.vel[d * n + i];
    }
    saved.rho[i] = s.rho[i];
  }
  if (is_excluded(t)) return false;
  bool bad = false;
  if (is_fluid(t)) {
    for (int d = 0; d < kp.dim; ++d) {
      const double a = (double)ace[d * n + i];
      if (PHASE == 0) {
        const double v = (double)s.vel[d * n + i];
        const double x0 = s.pos[d * n + i], x1 = x0 + 0.5 * dt * v;
        s.pos[d * n + i] = x1;
        disp2 += (x1 - x0) * (x1 - x0);
        const float v1 = (float)(v + 0.5 * dt * a);
        s.vel[d * n + i] = v1;
        bad |= !isfinite(v1);
      } else {
        const double vn = (double)saved.vel[d * n + i];
        const double v1 = vn + dt * a;
        s.pos[d * n + i] = saved.pos[d * n + i] + dt * 0.5 * (v1 + vn);
        const float v1f = (float)v1;
        s.vel[d * n + i] = v1f;
        bad |= !isfinite(v1f);
      }
    }
  } else if ((t & 0x7f) == SPH_BOUND_MOVING) {
    s.pos[i] = saved.pos[i] + dmove;
    s.vel[i] = (float)vmove;
    if (PHASE == 0) disp2 += dmove * dmove;
  }
  double r;
  if (PHASE == 0) {
    r = (double)s.rho[i] + 0.5 * dt * (double)arho[i];
  } else {
    const double eps = -((double)arho[i] / (double)s.rho[i]) * dt;
    r = (double)saved.rho[i] * (2.0 - eps) / (2.0 + eps);
  }
  const float rf = (float)r;
  s.rho[i] = rf;
  return bad || !(rf > 0.f) || !isfinite(rf);
}

// As symplectic_one for an all-FP64 state (vel64 and rho64 set in s and
// saved): the same update in FP64 from FP64 rates, with the FP32 copies of
// velocity and density rewritten as their roundings.
template <int PHASE>
__device__ inline bool symplectic_one_f64(const KParams& kp, int64_t n, int64_t i, double dt,
                                          double dmove, double vmove, const sph_state& saved,
                                          const sph_state& s, const double* __restrict__ ace,
                                          const double* __restrict__ arho, double& disp2) {
  const uint8_t t = s.type[i];
  if (PHASE == 0) {
    for (int d = 0; d < kp.dim; ++d) {
      saved.pos[d * n + i] = s.pos[d * n + i];
      saved.vel[d * n + i] = s.vel[d * n + i];
      saved.vel64[d * n + i] = s.vel64[d * n + i];
    }
    saved.rho[i] = s.rho[i];
    saved.rho64[i] = s.rho64[i];
  }
  if (is_excluded(t)) return false;
  bool bad = false;
  if (is_fluid(t)) {
    for (int d = 0; d < kp.dim; ++d) {
      const double a = ace[d * n + i];
      double v1;
      if (PHASE == 0) {
        const double v = s.vel64[d * n + i];
        const double x0 = s.pos[d * n + i], x1 = x0 + 0.5 * dt * v;
        s.pos[d * n + i] = x1;
        disp2 += (x1 - x0) * (x1 - x0);
        v1 = v + 0.5 * dt * a;
      } else {
        const double vn = saved.vel64[d * n + i];
        v1 = vn + dt * a;
        s.pos[d * n + i] = saved.pos[d * n + i] + dt * 0.5 * (v1 + vn);
      }
      s.vel64[d * n + i] = v1;
      s.vel[d * n + i] = (float)v1;
      bad |= !isfinite(v1);
    }
  } else if ((t & 0x7f) == SPH_BOUND_MOVING) {
    s.pos[i] = saved.pos[i] + dmove;
    s.vel64[i] = vmove;
    s.vel[i] = (float)vmove;
    if (PHASE == 0) disp2 += dmove * dmove;
  }
  double r;
  if (PHASE == 0) {
    r = s.rho64[i] + 0.5 * dt * arho[i];
  } else {
    const double eps = -(arho[i] / s.rho64[i]) * dt;
    r = saved.rho64[i] * (2.0 - eps) / (2.0 + eps);
  }
  s.rho64[i] = r;
  s.rho[i] = (float)r;
  return bad || !(r > 0.0) || !isfinite(r);
}

// One particle of the Verlet update (Section 2.5.1): MODE 0 is Eq. 30
// (v^{n+1} = v^{n-1} + 2 dt F, rho^{n+1} = rho^{n-1} + 2 dt R), MODE 1 is
// Eq. 31 (v^{n+1} = v^n + dt F, rho^{n+1} = rho^n + dt R, the intermediate
// step); both move fluid particles by r += dt v^n + dt^2/2 F.  `prev` holds
// the velocity and density of step n-1 and receives those of step n.  Moving
// walls take their imposed position and velocity (dmove since t, vmove at
// t + dt).  Returns true if the new state is not finite or the density not
// positive.
template <int MODE>
__device__ inline bool verlet_one(const KParams& kp, int64_t n, int64_t i, double dt,
                                  double dmove, double vmove, const sph_state& prev,
                                  const sph_state& s, const float* __restrict__ ace,
                                  const float* __restrict__ arho) {
  const uint8_t t = s.type[i];
  if (is_excluded(t)) return false;
  bool bad = false;
  const bool fluid = is_fluid(t);
  for (int d = 0; d < kp.dim; ++d) {
    const float vn = s.vel[d * n + i];
    if (fluid) {
      const double a = (double)ace[d * n + i];
      s.pos[d * n + i] = s.pos[d * n + i] + dt * (double)vn + 0.5 * dt * dt * a;
      const double v1 = MODE == 0 ? (double)prev.vel[d * n + i] + 2.0 * dt * a
                                  : (double)vn + dt * a;
      const float v1f = (float)v1;
      s.vel[d * n + i] = v1f;
      bad |= !isfinite(v1f);
    }
    prev.vel[d * n + i] = vn;
  }
  if ((t & 0x7f) == SPH_BOUND_MOVING) {
    s.pos[i] = s.pos[i] + dmove;
    s.vel[i] = (float)vmove;
  }
  const float rn = s.rho[i];
  const double r = MODE == 0 ? (double)prev.rho[i] + 2.0 * dt * (double)arho[i]
                             : (double)rn + dt * (double)arho[i];
  prev.rho[i] = rn;
  const float rf = (float)r;
  s.rho[i] = rf;
  return bad || !(rf > 0.f) || !isfinite(rf);
}

}  // namespace sph
