// Device code shared by the single-case and the batched interaction kernels:
// the pair terms of the WCSPH interaction and the per-lane neighbour walk
// (Section 2.3 of the DualSPHysics v5.0 paper).
#pragma once

#include "sph_internal.h"

namespace sph {

// Per-target sums of the pair loop, each without the factors that are the
// same for every pair of the target (applied once in write_target):
// kfab m_f (the fluid particle's mass with the kernel gradient's constant),
// 1/rho_a and h.
struct PairAcc {
  float ax, ay, az;  // dv/dt = kfab m_f / rho_a * (ax, ay, az)
  float cont;        // drho/dt continuity part = rho_a kfab m_f * cont
  float diff;        // density diffusion sum = kfab m_f * diff
  float vmax;        // visc = h * vmax
  uint32_t cnt;      // pairs evaluated
};

struct TargetData {
  bool fluid;
  float rho, irho, p;
  float vx, vy, vz;
  bool flt;  // a floating particle (general kernels only): Eq. 47
  float ik;  // kvc / rho_a: the viscosity constant's share of the target (see pair_terms)
};

// max(m, |t|) for a running maximum m >= 0 as one instruction: the compiler's
// own maximum first quiets a possible signalling NaN in m (an extra
// instruction per pair), which the values here (finite or quiet) never need.
__device__ __forceinline__ float max_abs(float m, float t) {
  float r;
  asm("v_max_f32_e64 %0, %1, |%2|" : "=v"(r) : "v"(m), "v"(t));
  return r;
}

// The pair terms of Eq. 15, 17-18, 21-22 and 36 for one pair (a, b) with
// r_ab = (dx, dy, dz), |r_ab|^2 = r2 < 4h^2.  pbw is +rho_b for a fluid
// particle and -rho_b for a wall; vb.w is P_b.  The caller has already
// dropped wall-wall pairs (Eq. 36 sums over fluid neighbours only).
//   F_ab = kfab g(q): Wendland C2 (Eq. 11) g = (1 - q/2)^3, or cubic spline
//     (Eq. 10) g = -3 + 9q/4 (q <= 1), -3/4 (2 - q)^2 / q (q > 1);
//   with m_b = mr m_f (mr = 1 for fluid neighbours and with equal masses)
//   and fv = mr g / rho_b, so that V_b F_ab = kfab m_f fv:
//   continuity:  V_b F_ab v_ab.r_ab = kfab m_f fv v_ab.r_ab;
//   momentum:    -m_b [(P_a + P_b)/(rho_a rho_b) + Pi_ab] F_ab r_ab
//              = -(kfab m_f / rho_a) [fv (P_a + P_b) + mr g pi_ab] r_ab,
//   with Pi_ab = -2 alpha c0 mu_ab / (rho_a + rho_b) for approaching pairs
//   (mu_ab = h t, t = v_ab.r_ab / (r^2 + eta^2) < 0) and 0 otherwise (Eq. 21),
//   so pi_ab = rho_a Pi_ab / m_f = min(t, 0) / (rho_b kvc/rho_a + kvc) with
//   kvc = -1 / (2 alpha c0 h) (per case) and kvc/rho_a = T.ik (per target);
//   or, with laminar viscosity (Eq. 23), no Pi_ab and
//     + (kfab m_f / rho_a) mr g r^2 v_ab / ((r^2 + eta^2)(rho_b kvc/rho_a + kvc)),
//   kvc = 1 / (4 nu0);
//   diffusion:   -(rho_b - rho_a) V_b F_ab over fluid b (Eq. 18), or with
//   rho_b - rho_a less its hydrostatic part rho^H_ab (Eq. 19-20).
// The per-target factors kfab m_f, 1/rho_a (and h in visc = max |mu|) are
// applied once in write_target.  With alpha (or nu0) zero kvc is infinite
// and the viscous term is exactly zero (the reciprocal of infinity).
// GEN: any formulation option (read from kp, uniform per slot) and floating
// targets, which take the momentum terms of a fluid target from their fluid
// neighbours (Eq. 47; no viscosity maximum, no diffusion); otherwise the
// default formulation (Wendland C2, artificial viscosity, Eq. 18 or no
// diffusion), whose code keeps the register budget of the production pass.
// EQM: fluid and wall particles have the same mass (mr = 1 for every pair).
template <int DIM, bool EQM, bool GEN>
__device__ __forceinline__ void pair_terms(const KParams& kp, const TargetData& a, float dx,
                                           float dy, float dz, float r2, float pbw,
                                           const float4& vb, PairAcc& acc) {
  const bool fb = pbw > 0.f;
  const float rhob = fabsf(pbw);
  const float dvx = a.vx - vb.x, dvy = a.vy - vb.y, dvz = DIM == 3 ? a.vz - vb.z : 0.f;
  // (explicit fused multiply-adds: the same bits in every kernel)
  const float vr = DIM == 3 ? fmaf(dvz, dz, fmaf(dvy, dy, dvx * dx)) : fmaf(dvy, dy, dvx * dx);
  const float s = __builtin_amdgcn_sqrtf(r2);
  float g;
  if (!GEN || kp.kernel == 0) {
    const float w = fmaf(s, kp.mhalf_inv_h_f, 1.f);  // 1 - q/2
    g = w * w * w;
  } else {
    const float q = s * kp.inv_h_f, u = 2.f - q;
    g = q <= 1.f ? fmaf(2.25f, q, -3.f) : -0.75f * u * u * __builtin_amdgcn_rcpf(q);
  }
  if (!EQM && !fb) g *= kp.mass_ratio_f;  // m_b / m_f for a wall neighbour
  const float fv = g * __builtin_amdgcn_rcpf(rhob);
  acc.cont = fmaf(fv, vr, acc.cont);
  acc.cnt += 1u;
  if (a.fluid || (GEN && a.flt)) {
    const float rr = __builtin_amdgcn_rcpf(r2 + kp.eta2_f);
    const float t = vr * rr;
    if (!GEN || !a.flt) acc.vmax = max_abs(acc.vmax, t);
    const float ivs = __builtin_amdgcn_rcpf(fmaf(rhob, a.ik, kp.kvc_f));
    const float pab = a.p + vb.w;
    if (!GEN || kp.viscosity == 0) {
      const float coef = fmaf(fv, pab, (fminf(t, 0.f) * ivs) * g);
      acc.ax = fmaf(-coef, dx, acc.ax);
      acc.ay = fmaf(-coef, dy, acc.ay);
      if (DIM == 3) acc.az = fmaf(-coef, dz, acc.az);
    } else {
      const float coef = fv * pab;
      const float lam = (rr * ivs) * (g * r2);
      acc.ax = fmaf(lam, dvx, fmaf(-coef, dx, acc.ax));
      acc.ay = fmaf(lam, dvy, fmaf(-coef, dy, acc.ay));
      if (DIM == 3) acc.az = fmaf(lam, dvz, fmaf(-coef, dz, acc.az));
    }
    float drho = rhob - a.rho;
    if (GEN && kp.ddt == 2) {
      const float e = kp.fz_f * (DIM == 3 ? dz : dy);  // vertical z_ab
      drho -= e * fmaf(e, fmaf(e, kp.hc3_f, kp.hc2_f), kp.hc1_f);
    }
    drho = fb ? drho : 0.f;
    acc.diff = fmaf(-drho, fv, acc.diff);
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

// Per-target outputs: dv/dt (with gravity) for fluid targets, dv/dt of
// Eq. 47 (without gravity) for floating ones, drho/dt, visc and the pair
// count; returns |dv/dt|, visc and the fluid flag for the block partial
// results.
template <int DIM>
__device__ __forceinline__ void write_target(const KParams& kp, int64_t n, int64_t a,
                                             const TargetData& t, const PairAcc& acc,
                                             uint32_t count_out, float* ace, float* arho,
                                             float* visc, uint32_t* nbr, float& fmag,
                                             float& vmax_out, uint32_t& nfl) {
  float ax = 0.f, ay = 0.f, az = 0.f;
  // the factors the pair sums leave out (see PairAcc)
  const float km = kp.kfab_mf_f, kma = km * t.irho;
  float ar = (t.rho * km) * acc.cont;
  const float vm = kp.h_f * acc.vmax;
  if (t.fluid) {
    ax = fmaf(kma, acc.ax, kp.gx_f);
    ay = fmaf(kma, acc.ay, kp.gy_f);
    az = DIM == 3 ? fmaf(kma, acc.az, kp.gz_f) : 0.f;
    ar += (kp.ddt_coef_f * km) * acc.diff;
    fmag = sqrtf(ax * ax + ay * ay + az * az);
    vmax_out = vm;
    nfl = 1;
  } else if (t.flt) {
    ax = kma * acc.ax;
    ay = kma * acc.ay;
    az = DIM == 3 ? kma * acc.az : 0.f;
  }
  ace[a] = ax;
  ace[n + a] = ay;
  if (DIM == 3) ace[2 * n + a] = az;
  arho[a] = ar;
  if (visc) visc[a] = vm;
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
// r_ab = (dx, dy, dz) and |r_ab|^2 of candidate pb for a target with
// fixed-point x bits xa and row-shifted offsets (ys, zs) (see gather_group):
// one form for the cell walk and the neighbour-list replay, so that both
// take the same FP32 decisions.
// Written with explicit fused multiply-adds, so that no compiler contraction
// choice can differ between the kernels that inline it.
template <int DIM>
__device__ __forceinline__ float pair_geom(const KParams& kp, uint32_t xa, float ys, float zs,
                                           const float4& pb, float& dx, float& dy, float& dz) {
  dx = (float)(int32_t)(xa - __float_as_uint(pb.x)) * kp.unit_x_f;
  dy = ys - pb.y;
  dz = DIM == 3 ? zs - pb.z : 0.f;
  return DIM == 3 ? fmaf(dz, dz, fmaf(dy, dy, dx * dx)) : fmaf(dy, dy, dx * dx);
}

// The target's offset along y or z shifted to the row d cells away: p - d cs
// as one fused multiply-add (the same bits in every kernel).
__device__ __forceinline__ float row_shift(float p, int d, float cs) {
  return fmaf(-(float)d, cs, p);
}

// Element k of an array at a uniform base, addressed by a 32-bit byte offset
// (k * sizeof(T) < 2^32, which the calls' size limits keep): the load then
// takes the base from scalar registers and the offset from one vector
// register, with no 64-bit address arithmetic per lane.
template <typename T>
__device__ __forceinline__ const T& at32(const T* __restrict__ base, uint32_t k) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                     (uint32_t)(k * (uint32_t)sizeof(T)));
}
// The element U places after byte offset o (U a compile-time constant, folded
// into the load's immediate offset).
template <int U, typename T>
__device__ __forceinline__ const T& at_byte(const T* __restrict__ base, uint32_t o) {
  return *(reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + o) + U);
}

// One group of NU (4, 2 or 1) consecutive candidates j..j+NU-1 of a row for
// one target lane, all before the row's end j1 (o = 16 j and o1 = 16 j1 are
// byte offsets into the views: 32 bits, which the calls' limit of n < 2^28
// keeps exact): the candidate positions are loaded together, tested, then the
// velocities of the hits are loaded together and their pair terms
// accumulated.  Along x the views hold fixed-point offsets (units of
// kFrameCells*cs / 2^32, periodic over kFrameCells cells): the 32-bit
// difference of two offsets, read as signed, is x_a - x_b exactly modulo the
// period, which exceeds twice the reach of the stencil.  Along y and z the
// offsets are cell-relative and (ys, zs) carry the row's cell shift.  Wall
// targets skip wall candidates (Eq. 36).
template <int DIM, bool DIAG, bool EQM, bool GEN, bool PER, int NU = 4>
__device__ __forceinline__ void gather_group(const KParams& kp, int64_t n, int64_t i,
                                             uint32_t xa, float ys, float zs,
                                             const TargetData& T, uint32_t o,
                                             const float4* __restrict__ pr,
                                             const float4* __restrict__ vp,
                                             const double* pa64,
                                             const double* __restrict__ pos64, PairAcc& acc,
                                             uint32_t& c64) {
  float4 pb[NU];
  pb[0] = at_byte<0>(pr, o);
  if (NU > 1) pb[1 % NU] = at_byte<1>(pr, o);
  if (NU > 2) pb[2 % NU] = at_byte<2>(pr, o);
  if (NU > 3) pb[3 % NU] = at_byte<3>(pr, o);
  bool hit[NU];
  float dxs[NU], dys[NU], dzs[NU], r2s[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    r2s[u] = pair_geom<DIM>(kp, xa, ys, zs, pb[u], dxs[u], dys[u], dzs[u]);
    hit[u] = (T.fluid || pb[u].w > 0.f) && r2s[u] < kp.support2_f;
    if (DIAG) {
      const uint32_t jj = (o >> 4) + u;
      // (pb.w == 0: a particle excluded by a view refresh, no neighbour)
      if ((int64_t)jj != i && (T.fluid || pb[u].w > 0.f) && pb[u].w != 0.f) {
        double r2d = 0.0;
        for (int d = 0; d < DIM; ++d) {
          double e = __dsub_rn(pa64[d], pos64[d * n + jj]);
          if (PER && ((kp.periodic >> d) & 1)) {  // nearest image
            const double L = d == 0 ? kp.px : (d == 1 ? kp.py : kp.pz);
            if (e > 0.5 * L) e = __dsub_rn(e, L);
            else if (e < -0.5 * L) e = __dadd_rn(e, L);
          }
          r2d = __dadd_rn(r2d, __dmul_rn(e, e));
        }
        c64 += (r2d < kp.support2) ? 1u : 0u;
      }
    }
  }
  float4 vb[NU];
  if (hit[0]) vb[0] = at_byte<0>(vp, o);
  if (NU > 1 && hit[1 % NU]) vb[1 % NU] = at_byte<1>(vp, o);
  if (NU > 2 && hit[2 % NU]) vb[2 % NU] = at_byte<2>(vp, o);
  if (NU > 3 && hit[3 % NU]) vb[3 % NU] = at_byte<3>(vp, o);
#pragma unroll
  for (int u = 0; u < NU; ++u)
    if (hit[u])
      pair_terms<DIM, EQM, GEN>(kp, T, dxs[u], dys[u], dzs[u], r2s[u], pb[u].w, vb[u], acc);
}

// The candidate walk of one target lane over the rows of its neighbour cells
// (cell indices offset by cbase).  The key cells of a row along x (2R+1
// cells of cs, each split into x_sub key cells) are consecutive in the sorted
// order, so a row is one candidate range; a row is cut to the key cells that
// the support sphere of the target reaches: with e_y,
// e_z the distances from the target to the row's cell extent along y and z,
// only |x_ab| < sqrt(4h^2 - e_y^2 - e_z^2) can hold a neighbour (rows with a
// negative radicand are skipped).  The cut uses a support enlarged by 1e-4
// relative, far above the FP32 error of the offsets, so that no pair within
// 2h is ever cut.  Each range runs as whole groups of 4, then a group of 2
// and a group of 1 for its last candidates.
//
// Periodic components (PER kernels only, Section 2.7): a row index along
// y or z past either end wraps to the other end (the row's shift (ys, zs)
// stays that of the unwrapped cell, which is the nearest image since the
// offsets are cell-relative); along x the cut window may run past either
// end, and the part beyond is walked as a second range of cells at the
// other end, with the target's fixed-point x moved by one period so that
// the 32-bit differences give the nearest image.  Validation keeps every
// periodic component at least 2R+1 cells long, so no cell is walked twice.
//
// Reused cells (an interaction after a view refresh, R one above the
// stencil of the cells): the particles have moved by up to delta since the
// binning, so a neighbour within 2h of the target's current position lies
// in a cell whose binned extent is within 2h + delta of it.  The caller
// passes the culling radius squared accordingly (cull2), and one more cell
// of reach covers the target's own drift out of its cell while 2 delta
// stays below a cell.  Along x the visited candidates then lie within 4
// cells plus delta of the target; one that aliases across the 8-cell
// fixed-point period is at least 4 cells away either way, beyond 2h, so it
// is never a neighbour.
//
// The target is not excluded from its own candidates: its self pair adds
// exactly zero to every sum (v_aa = 0, r_aa = 0 and rho_a - rho_a = 0) and
// the caller takes it off the count (fluid targets meet themselves; wall
// targets skip wall candidates).  DIAG also counts neighbours with an FP64
// test on the FP64 positions (c64, self excluded).
//
// LPT > 1: the rows of the stencil are dealt to LPT lanes (by position in
// the stencil, lane `sub` taking every LPT-th), which shortens each lane's
// chain of dependent loads for cases too small to fill the GPU; the caller
// sums the lanes' partial results (combine_lanes).
template <int DIM, int R, bool DIAG, bool EQM, bool GEN, bool PER, int LPT = 1>
__device__ __forceinline__ void gather_walk(const KParams& kp, uint32_t cbase, int64_t n,
                                            int64_t i, const float4& pa, const TargetData& T,
                                            int cx, int cy, int cz,
                                            const float4* __restrict__ pr,
                                            const float4* __restrict__ vp,
                                            const uint32_t* __restrict__ cstart,
                                            const double* __restrict__ pos64, PairAcc& acc,
                                            uint32_t& c64, float cull2, int sub = 0) {
  static_assert(R <= 3, "the x period (8 cells) must exceed twice the stencil reach");
  static_assert(kFrameCells == 8, "x offsets use 2^29 units per cell");
  double pa64[3] = {0.0, 0.0, 0.0};
  if (DIAG)
    for (int d = 0; d < DIM; ++d) pa64[d] = pos64[d * n + i];
  const float cs = kp.cs_f;
  const uint32_t xa = __float_as_uint(pa.x);
  // the target's offset inside its own key cell along x (key cells of
  // cs/x_sub: 2^(29 - lg x_sub) fixed-point units each)
  const int fcells = kFrameCells << kp.lg_xsub;
  const float fx =
      (float)(int32_t)(xa - ((uint32_t)(cx % fcells) << (29 - kp.lg_xsub))) * kp.unit_x_f;
  const int reach = R * kp.x_sub;  // the stencil's reach in key cells along x
  const bool perx = PER && (kp.periodic & 1);
  const bool pery = PER && (kp.periodic & 2);
  const bool perz = PER && DIM == 3 && (kp.periodic & 4);
  const int xlo = cx - reach < 0 && !perx ? 0 : cx - reach;
  const int xhi = cx + reach >= kp.ncx && !perx ? kp.ncx - 1 : cx + reach;
  const int zlo = DIM == 3 ? -R : 0, zhi = DIM == 3 ? R : 0;
  // one row of the stencil: the key cells (dy, dz) away, cut to the window
  // the support sphere reaches
  auto visit = [&](int dz, int dy) {
    int z = cz + dz;
    if (z < 0 || z >= kp.ncz) {
      if (!perz) return;
      z += z < 0 ? kp.ncz : -kp.ncz;
    }
    const float ez0 = (float)dz * cs - pa.z;  // lower edge of the row's z extent
    const float ez = dz > 0 ? ez0 : (dz < 0 ? -(ez0 + cs) : 0.f);
    int y = cy + dy;
    if (y < 0 || y >= kp.ncy) {
      if (!pery) return;
      y += y < 0 ? kp.ncy : -kp.ncy;
    }
    const float ey0 = (float)dy * cs - pa.y;
    const float ey = dy > 0 ? ey0 : (dy < 0 ? -(ey0 + cs) : 0.f);
    const float w2 = cull2 - ey * ey - ez * ez;
    if (!(w2 > 0.f)) return;
    const float w = __builtin_amdgcn_sqrtf(w2);
    int x0 = cx + (int)floorf((fx - w) * kp.inv_csx_f);
    int x1 = cx + (int)floorf((fx + w) * kp.inv_csx_f);
    x0 = x0 < xlo ? xlo : x0;
    x1 = x1 > xhi ? xhi : x1;
    const uint32_t row =
        cbase + (uint32_t)kp.ncx * ((uint32_t)y + (uint32_t)kp.ncy * (uint32_t)z);
    const float ys = row_shift(pa.y, dy, cs), zs = row_shift(pa.z, dz, cs);
    // the candidates of key cells [c0, c1] of the row, with target x bits xv
    auto walk = [&](int c0, int c1, uint32_t xv) {
      // byte offsets of the range in the views
      uint32_t o = at32(cstart, row + c0) * 16u;
      const uint32_t o1 = at32(cstart, row + c1 + 1) * 16u;
      for (; o + 64u <= o1; o += 64u)
        gather_group<DIM, DIAG, EQM, GEN, PER>(kp, n, i, xv, ys, zs, T, o, pr, vp, pa64, pos64,
                                               acc, c64);
      // the last 0-3 candidates as a group of 2 and a group of 1 (a masked
      // group of 4 would test up to 3 slots past the range)
      if (o + 32u <= o1) {
        gather_group<DIM, DIAG, EQM, GEN, PER, 2>(kp, n, i, xv, ys, zs, T, o, pr, vp, pa64,
                                                  pos64, acc, c64);
        o += 32u;
      }
      if (o < o1)
        gather_group<DIM, DIAG, EQM, GEN, PER, 1>(kp, n, i, xv, ys, zs, T, o, pr, vp, pa64,
                                                  pos64, acc, c64);
    };
    if (perx) {
      if (x0 < 0) {  // cells at the far end, one period below
        walk(kp.ncx + x0, kp.ncx - 1, xa + kp.lu);
        x0 = 0;
      }
      if (x1 >= kp.ncx) {  // cells at the near end, one period above
        walk(0, x1 - kp.ncx, xa - kp.lu);
        x1 = kp.ncx - 1;
      }
    }
    walk(x0, x1, xa);
  };
  if constexpr (LPT == 1) {
    for (int dz = zlo; dz <= zhi; ++dz)
      for (int dy = -R; dy <= R; ++dy) visit(dz, dy);
  } else {
    // the LPT lanes of a target walk different rows at the same time: in
    // round q, lane `sub` takes row q LPT + sub of the stencil
    constexpr int kRowsY = 2 * R + 1;
    constexpr int kRows = kRowsY * (DIM == 3 ? 2 * R + 1 : 1);
    for (int q = 0; q < (kRows + LPT - 1) / LPT; ++q) {
      const int r = q * LPT + sub;
      if (r < kRows) visit(zlo + r / kRowsY, r % kRowsY - R);
    }
  }
}

// Sums the walks of the LPT lanes of each target (adjacent lanes, LPT a
// power of two); every lane of the wave calls this, and every lane of a
// group ends with the group's sums.  Maxima take the maximum.
template <int LPT>
__device__ __forceinline__ void combine_lanes(PairAcc& acc, uint32_t& c64) {
  for (int off = 1; off < LPT; off <<= 1) {
    acc.ax += __shfl_xor(acc.ax, off, 64);
    acc.ay += __shfl_xor(acc.ay, off, 64);
    acc.az += __shfl_xor(acc.az, off, 64);
    acc.cont += __shfl_xor(acc.cont, off, 64);
    acc.diff += __shfl_xor(acc.diff, off, 64);
    acc.vmax = fmaxf(acc.vmax, __shfl_xor(acc.vmax, off, 64));
    acc.cnt += (uint32_t)__shfl_xor((int)acc.cnt, off, 64);
    c64 += (uint32_t)__shfl_xor((int)c64, off, 64);
  }
}

}  // namespace sph
