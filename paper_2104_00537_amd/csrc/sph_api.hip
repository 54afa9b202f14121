// The C ABI of libsph (declared in include/sph.h): argument checks, workspace
// carving and kernel launches.  No call allocates device memory.
#include <math.h>
#include <string.h>

#include "sph_kernels.h"

namespace sph {

KParams make_kparams(const sph_params& p) {
  KParams k{};
  k.dim = p.dim;
  k.cell_div = p.cell_div;
  k.ddt = p.ddt;
  k.ncx = p.ncell[0];
  k.ncy = p.ncell[1];
  k.ncz = p.ncell[2];
  k.ncell_total = (uint32_t)((uint64_t)p.ncell[0] * p.ncell[1] * p.ncell[2]);
  k.ox = p.origin[0];
  k.oy = p.origin[1];
  k.oz = p.origin[2];
  k.cs = p.cell_size;
  k.inv_cs = p.inv_cell_size;
  k.x_sub = p.x_sub;
  k.lg_xsub = p.x_sub == 8 ? 3 : p.x_sub == 4 ? 2 : p.x_sub == 2 ? 1 : 0;
  k.inv_csx = p.inv_cell_size * (double)p.x_sub;
  k.h = p.h;
  k.rho0 = p.rho0;
  k.gamma = p.gamma;
  k.c0 = p.c0;
  k.b_tait = p.c0 * p.c0 * p.rho0 / p.gamma;
  k.cfl = p.cfl;
  k.dt_floor = p.dt_floor;
  k.mass_f = p.mass_fluid;
  k.mass_b = p.mass_bound;
  k.gx = p.gravity[0];
  k.gy = p.gravity[1];
  k.gz = p.gravity[2];
  k.motion_amp = p.motion_amp;
  k.motion_omega = p.motion_omega;
  k.support2 = (2.0 * p.h) * (2.0 * p.h);
  // Kernel gradient grad_a W_ab = kfab g(q) r_ab.  Wendland C2 (Eq. 11):
  // alpha_D = 7/(4 pi h^2) in 2-D, 21/(16 pi h^3) in 3-D, kfab = -5 alpha_D / h^2,
  // g = (1 - q/2)^3.  Cubic spline (Eq. 10): alpha_D = 10/(7 pi h^2), 1/(pi h^3),
  // kfab = alpha_D / h^2, g = -3 + 9q/4 (q <= 1), -3/4 (2 - q)^2 / q (q > 1).
  const double alpha_d = p.kernel == 1
      ? (p.dim == 2 ? 10.0 / (7.0 * M_PI * p.h * p.h) : 1.0 / (M_PI * p.h * p.h * p.h))
      : (p.dim == 2 ? 7.0 / (4.0 * M_PI * p.h * p.h)
                    : 21.0 / (16.0 * M_PI * p.h * p.h * p.h));
  const double kfab = p.kernel == 1 ? alpha_d / (p.h * p.h) : -5.0 * alpha_d / (p.h * p.h);
  k.inv_frame = 1.0 / (kFrameCells * p.cell_size);
  k.kfab = kfab;
  k.inv_h = 1.0 / p.h;
  k.w_alpha = alpha_d;
  k.f_coef = kfab;
  k.alpha_c0 = p.alpha * p.c0;
  k.ddt_coef = p.ddt ? 2.0 * p.delta * p.h * p.c0 : 0.0;
  k.eta2 = p.eta2;
  k.h_f = (float)p.h;
  k.mhalf_inv_h_f = (float)(-0.5 / p.h);
  k.support2_f = (float)k.support2;
  k.kfab_mf_f = (float)(kfab * p.mass_fluid);
  k.kfab_mb_f = (float)(kfab * p.mass_bound);
  k.kpi_mf_f = (float)(-2.0 * p.alpha * p.c0 * kfab * p.mass_fluid);
  k.kpi_mb_f = (float)(-2.0 * p.alpha * p.c0 * kfab * p.mass_bound);
  k.eta2_f = (float)p.eta2;
  k.kernel = p.kernel;
  k.boundary = p.boundary;
  k.floating = p.floating;
  k.periodic = 0;
  for (int d = 0; d < p.dim; ++d)
    if (p.period[d] > 0.0) k.periodic |= 1 << d;
  k.px = p.period[0] > 0.0 ? p.period[0] : 0.0;
  k.py = p.dim > 1 && p.period[1] > 0.0 ? p.period[1] : 0.0;
  k.pz = p.dim > 2 && p.period[2] > 0.0 ? p.period[2] : 0.0;
  // the x period in fixed-point x units (kFrameCells cells = 2^32), mod 2^32
  {
    const double fr = k.px / (kFrameCells * p.cell_size);
    k.lu = (uint32_t)(uint64_t)llround((fr - floor(fr)) * 4294967296.0);
  }
  k.viscosity = p.viscosity;
  k.inv_h_f = (float)(1.0 / p.h);
  k.klam_mf_f = (float)(4.0 * p.visc_nu * kfab * p.mass_fluid);
  k.klam_mb_f = (float)(4.0 * p.visc_nu * kfab * p.mass_bound);
  {
    // Eq. 19-20: rho^H_ab = rho0 [(1 + eps)^(1/gamma) - 1], eps = rho0 g z_ab / B,
    // as its series to eps^3 (|eps| < 0.01 within 2h of any case, so the
    // remainder is below 1e-8 relative)
    const double b = p.c0 * p.c0 * p.rho0 / p.gamma;
    const double g = fabs(p.gravity[p.dim - 1]);
    const double e = 1.0 / p.gamma;
    k.fz_f = (float)(p.rho0 * g / b);
    k.hc1_f = (float)(p.rho0 * e);
    k.hc2_f = (float)(p.rho0 * e * (e - 1.0) / 2.0);
    k.hc3_f = (float)(p.rho0 * e * (e - 1.0) * (e - 2.0) / 6.0);
  }
  k.ddt_coef_f = p.ddt ? (float)(2.0 * p.delta * p.h * p.c0) : 0.f;
  // the viscous term's constant in the pair loop's scaling (infinite when
  // the viscosity is zero: the term is then exactly zero)
  k.kvc_f = p.viscosity == 0 ? (float)(-1.0 / (2.0 * p.alpha * p.c0 * p.h))
                             : (float)(1.0 / (4.0 * p.visc_nu));
  k.mass_ratio_f = (float)(p.mass_bound / p.mass_fluid);
  k.cs_f = (float)p.cell_size;
  k.inv_csx_f = (float)(p.inv_cell_size * (double)p.x_sub);
  k.unit_x_f = (float)(kFrameCells * p.cell_size / 4294967296.0);
  k.w_alpha_f = (float)alpha_d;
  k.shift_k_f = (float)(p.shift_coef * p.h);
  k.shift_fs_f = (float)p.shift_fs;
  k.gx_f = (float)p.gravity[0];
  k.gy_f = (float)p.gravity[1];
  k.gz_f = (float)p.gravity[2];
  return k;
}

// The constants of a case in the batch's 3-D layout: a 2-D case (x, z) is
// stored as (x, 0, z) with a single cell across y centred on y = 0; its kernel
// normalisation stays the 2-D one.
KParams make_slot_kparams(const sph_params& p) {
  KParams k = make_kparams(p);
  if (p.dim == 2) {
    k.dim = 3;
    k.ncx = p.ncell[0];
    k.ncy = 1;
    k.ncz = p.ncell[1];
    k.ox = p.origin[0];
    k.oy = -0.5 * p.cell_size;
    k.oz = p.origin[1];
    k.gx = p.gravity[0];
    k.gy = 0.0;
    k.gz = p.gravity[1];
    k.gx_f = (float)k.gx;
    k.gy_f = 0.f;
    k.gz_f = (float)k.gz;
    // a periodic vertical component moves from the second to the third
    k.periodic = (k.periodic & 1) | ((k.periodic & 2) << 1);
    k.pz = k.py;
    k.py = 0.0;
  }
  return k;
}

// Every periodic component spans at least 2 reach + 1 cells, so that a walk
// of that reach meets no cell twice (params_ok checks the cells' own reach;
// a walk on reused cells reaches one cell further).
static bool periodic_reach_ok(const sph_params* p, int reach) {
  for (int k = 0; k < p->dim; ++k) {
    if (!(p->period[k] > 0.0)) continue;
    const int cells = k == 0 ? p->ncell[0] / p->x_sub : p->ncell[k];
    if (cells < 2 * reach + 1) return false;
  }
  return true;
}

bool params_ok(const sph_params* p) {
  if (!p) return false;
  if (p->dim != 2 && p->dim != 3) return false;
  if (p->cell_div != 1 && p->cell_div != 2) return false;
  if (p->x_sub != 1 && p->x_sub != 2 && p->x_sub != 4 && p->x_sub != 8) return false;
  if (p->ddt < 0 || p->ddt > 2) return false;
  if (p->kernel != 0 && p->kernel != 1) return false;
  if (p->boundary != 0 && p->boundary != 1) return false;
  if (p->floating != 0 && p->floating != 1) return false;
  if (!(p->shift_coef >= 0.0) || !isfinite(p->shift_coef)) return false;
  if (!(p->shift_fs >= 0.0) || !isfinite(p->shift_fs)) return false;
  if (p->floating == 1 && p->boundary != 0) return false;
  // periodic components: the grid spans exactly the period, in whole cells,
  // at least 2 cell_div + 1 of them (so no neighbour cell is reached twice)
  for (int k = 0; k < 3; ++k) {
    const double L = p->period[k];
    if (!(L >= 0.0) || !isfinite(L)) return false;
    if (L == 0.0) continue;
    if (k >= p->dim || p->boundary != 0 || p->floating != 0) return false;
    if (k == 0 && p->ncell[0] % p->x_sub != 0) return false;
    const int cells = k == 0 ? p->ncell[0] / p->x_sub : p->ncell[k];
    if (cells < 2 * p->cell_div + 1) return false;
    if (fabs(L - cells * p->cell_size) > 1e-9 * L) return false;
  }
  if (p->viscosity != 0 && p->viscosity != 1) return false;
  if (!(p->visc_nu >= 0) || !isfinite(p->visc_nu)) return false;
  for (int k = 0; k < 3; ++k)
    if (p->ncell[k] < 1) return false;
  if (p->dim == 2 && p->ncell[2] != 1) return false;
  const uint64_t total = (uint64_t)p->ncell[0] * p->ncell[1] * p->ncell[2];
  if (total + 1 >= 0xffffffffull) return false;
  if (!(p->h > 0) || !(p->rho0 > 0) || !(p->gamma > 0) || !(p->c0 > 0)) return false;
  if (!(p->cell_size > 0) || !(p->inv_cell_size > 0)) return false;
  // the +-cell_div cell stencil must cover the 2h support
  if (p->cell_size * p->cell_div < 2.0 * p->h * (1.0 - 1e-12)) return false;
  // eta^2 > 0 keeps Eq. 21 non-singular (also for coincident particles)
  if (!(p->cfl > 0) || !(p->eta2 > 0) || !(p->mass_fluid > 0) || !(p->mass_bound > 0))
    return false;
  return true;
}

static bool n_ok(int64_t n) { return n >= 0 && n < (int64_t)0xfffffff0ll; }

static bool state_ok(const sph_state* s, bool need_type) {
  return s && s->pos && s->vel && s->rho && (!need_type || s->type) &&
         (s->vel64 == nullptr) == (s->rho64 == nullptr);
}

// an all-FP64 state (the precision study's reference arm)
static bool f64_state(const sph_state* s) { return s && s->vel64 != nullptr; }

static sph_status hip_status(hipError_t e) { return e == hipSuccess ? SPH_OK : SPH_E_HIP; }

}  // namespace sph

using namespace sph;

extern "C" {

size_t sph_workspace_bytes(const sph_params* p, int64_t n) {
  (void)p;
  if (!n_ok(n)) return 0;
  return ws_layout(n).total;
}

sph_status sph_bin_cells(const sph_params* p, int64_t n, const sph_state* in, sph_state* out,
                         const sph_state* carry_in, sph_state* carry_out, uint32_t* key,
                         uint32_t* perm, uint32_t* cell_start, void* ws, size_t ws_bytes,
                         void* stream) {
  if (!params_ok(p) || !n_ok(n) || !cell_start || !ws) return SPH_E_ARG;
  if (n > 0 && (!state_ok(in, true) || !state_ok(out, true) || !key || !perm)) return SPH_E_ARG;
  if (n > 0 && in->pos == out->pos) return SPH_E_ARG;
  if ((carry_in == nullptr) != (carry_out == nullptr)) return SPH_E_ARG;
  if (carry_in && n > 0 && (!state_ok(carry_in, false) || !state_ok(carry_out, false)))
    return SPH_E_ARG;
  if (ws_bytes < ws_layout(n).total) return SPH_E_WORKSPACE;
  const KParams kp = make_kparams(*p);
  sph_state i0 = n > 0 ? *in : sph_state{}, o0 = n > 0 ? *out : sph_state{};
  return hip_status(launch_bin_cells(kp, n, i0, o0, carry_in, carry_out, key, perm, cell_start,
                                     ws, (hipStream_t)stream));
}

// The interaction walk addresses the views and the cell ranges with 32-bit
// byte offsets.
static bool walk_size_ok(const sph_params* p, int64_t n) {
  const uint64_t cells = (uint64_t)p->ncell[0] * p->ncell[1] * p->ncell[2];
  return n < ((int64_t)1 << 28) && cells < ((uint64_t)1 << 30);
}

sph_status sph_interact(const sph_params* p, int64_t n, const sph_state* s, const uint32_t* key,
                        const uint32_t* cell_start, float* ace, float* arho, float* visc,
                        uint32_t* nbr_count, uint32_t flags, void* ws, size_t ws_bytes,
                        void* stream) {
  if (!params_ok(p) || !n_ok(n) || !cell_start || !ws || !walk_size_ok(p, n)) return SPH_E_ARG;
  if (n > 0 && (!state_ok(s, true) || !key || !ace || !arho)) return SPH_E_ARG;
  // none, the FP64 diagnostic count and/or reused cells, or one
  // precision-study arm alone
  const uint32_t reuse = flags & SPH_INTERACT_REUSE_CELLS;
  const uint32_t base =
      flags & ~(uint32_t)(SPH_INTERACT_REUSE_CELLS | SPH_INTERACT_ONE_LANE);
  const bool arm = base == SPH_INTERACT_F64 || base == SPH_INTERACT_ABS_F32 ||
                   base == SPH_INTERACT_F64_STATE;
  if (base != 0 && base != SPH_DIAG_COUNT_F64 && !arm) return SPH_E_ARG;
  if (reuse && (arm || p->boundary != 0 || !periodic_reach_ok(p, p->cell_div + 1)))
    return SPH_E_ARG;
  // the precision-study arms implement the default formulation only
  if (arm && (p->kernel != 0 || p->viscosity != 0 || p->ddt == 2 || p->floating != 0 ||
              p->period[0] > 0.0 || p->period[1] > 0.0 || p->period[2] > 0.0))
    return SPH_E_ARG;
  // the all-FP64 arm reads the state's FP64 copies (not with modified DBC,
  // which writes FP32 wall densities)
  if (base == SPH_INTERACT_F64_STATE && n > 0 && (!f64_state(s) || p->boundary != 0))
    return SPH_E_ARG;
  if (ws_bytes < ws_layout(n).total) return SPH_E_WORKSPACE;
  const KParams kp = make_kparams(*p);
  sph_state s0 = n > 0 ? *s : sph_state{};
  return hip_status(launch_interact(kp, n, s0, key, cell_start, ace, arho, visc, nbr_count, flags,
                                    ws, (hipStream_t)stream));
}

// ------------------------------------------------------- neighbour lists --
// The list kernels run the default formulation (the production pass).
static bool list_params_ok(const sph_params* p, int64_t n) {
  return params_ok(p) && n_ok(n) && walk_size_ok(p, n) && p->kernel == 0 &&
         p->viscosity == 0 && p->ddt != 2 && p->floating == 0 && p->boundary == 0 &&
         !(p->period[0] > 0.0) && !(p->period[1] > 0.0) && !(p->period[2] > 0.0);
}

// Chunks per target that a list buffer of `bytes` holds (0: too small).
static int64_t list_cap(int64_t n, size_t bytes) {
  const ListLayout L0 = list_layout(n, 0);
  if (bytes < L0.total) return 0;
  const size_t nn = (size_t)(n > 0 ? n : 1);
  const int64_t cap = (int64_t)((bytes - L0.total) / (8 * nn));
  return cap < kListCap ? cap : kListCap;
}

size_t sph_list_bytes(const sph_params* p, int64_t n) {
  if (!list_params_ok(p, n)) return 0;
  return list_layout(n, kListCap).total;
}

sph_status sph_build_list(const sph_params* p, int64_t n, const sph_state* s,
                          const uint32_t* key, const uint32_t* cell_start, double skin,
                          uint32_t flags, void* list, size_t list_bytes, void* ws,
                          size_t ws_bytes, void* stream) {
  if (!list_params_ok(p, n) || !cell_start || !ws || !list) return SPH_E_ARG;
  if (flags & ~(uint32_t)SPH_LIST_ADAPTIVE_SKIN) return SPH_E_ARG;
  if (!(skin >= 0.0) || !(skin < 0.5 * p->cell_size)) return SPH_E_ARG;
  if (n > 0 && (!state_ok(s, true) || !key || f64_state(s))) return SPH_E_ARG;
  const int64_t cap = list_cap(n, list_bytes);
  if (cap < 1) return SPH_E_ARG;
  if (ws_bytes < ws_layout(n).total) return SPH_E_WORKSPACE;
  sph_state s0 = n > 0 ? *s : sph_state{};
  return hip_status(launch_build_list(make_kparams(*p), n, s0, key, cell_start, (float)skin,
                                      (flags & SPH_LIST_ADAPTIVE_SKIN) != 0, list, cap, ws,
                                      (hipStream_t)stream));
}

sph_status sph_interact_list(const sph_params* p, int64_t n, const sph_state* s,
                             const uint32_t* key, const uint32_t* cell_start, const void* list,
                             size_t list_bytes, float* ace, float* arho, float* visc,
                             uint32_t* nbr_count, uint32_t flags, void* ws, size_t ws_bytes,
                             void* stream) {
  if (!list_params_ok(p, n) || !cell_start || !ws || !list) return SPH_E_ARG;
  if (flags & ~(uint32_t)(SPH_DIAG_COUNT_F64 | SPH_INTERACT_REUSE_CELLS | SPH_INTERACT_ONE_LANE))
    return SPH_E_ARG;
  if ((flags & SPH_INTERACT_REUSE_CELLS) && !periodic_reach_ok(p, p->cell_div + 1))
    return SPH_E_ARG;
  if (n > 0 && (!state_ok(s, true) || !key || !ace || !arho || f64_state(s))) return SPH_E_ARG;
  const int64_t cap = list_cap(n, list_bytes);
  if (cap < 1) return SPH_E_ARG;
  if (ws_bytes < ws_layout(n).total) return SPH_E_WORKSPACE;
  sph_state s0 = n > 0 ? *s : sph_state{};
  return hip_status(launch_interact_list(make_kparams(*p), n, s0, key, cell_start, list, cap, ace,
                                         arho, visc, nbr_count, flags, ws,
                                         (hipStream_t)stream));
}

int64_t sph_list_walks(const void* ws) {
  if (!ws) return SPH_E_ARG;
  WsHeader h{};
  if (hipDeviceSynchronize() != hipSuccess) return SPH_E_HIP;
  if (hipMemcpy(&h, ws, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return SPH_E_HIP;
  return (int64_t)h.list_walks;
}

sph_status sph_refresh_view(const sph_params* p, int64_t n, sph_state* s, const uint32_t* key,
                            void* ws, size_t ws_bytes, void* stream) {
  if (!params_ok(p) || !n_ok(n) || !ws) return SPH_E_ARG;
  if (n > 0 && (!state_ok(s, true) || !key || f64_state(s))) return SPH_E_ARG;
  if (ws_bytes < ws_layout(n).total) return SPH_E_WORKSPACE;
  sph_state s0 = n > 0 ? *s : sph_state{};
  return hip_status(launch_refresh_view(make_kparams(*p), n, s0, key, ws, (hipStream_t)stream));
}

sph_status sph_reduce_dt(const sph_params* p, int64_t n, double* dt, uint64_t* interactions,
                         float* maxima, void* ws, size_t ws_bytes, void* stream) {
  if (!params_ok(p) || !n_ok(n) || !dt || !ws) return SPH_E_ARG;
  if (ws_bytes < ws_layout(n).total) return SPH_E_WORKSPACE;
  return hip_status(
      launch_reduce_dt(make_kparams(*p), n, dt, interactions, maxima, ws, (hipStream_t)stream));
}

sph_status sph_symplectic_step(const sph_params* p, int64_t n, int32_t phase, const double* dt,
                               double* t, sph_state* saved, sph_state* s, const float* ace,
                               const float* arho, void* ws, size_t ws_bytes, void* stream) {
  if (!params_ok(p) || !n_ok(n) || !dt || !t || !ws) return SPH_E_ARG;
  if (phase != 0 && phase != 1) return SPH_E_ARG;
  if (n > 0 && (!state_ok(s, true) || !state_ok(saved, false) || !ace || !arho))
    return SPH_E_ARG;
  // an all-FP64 state needs an all-FP64 saved state (no floating bodies)
  if (n > 0 && f64_state(s) && (!f64_state(saved) || p->floating != 0)) return SPH_E_ARG;
  if (ws_bytes < ws_layout(n).total) return SPH_E_WORKSPACE;
  sph_state sv = n > 0 ? *saved : sph_state{}, st = n > 0 ? *s : sph_state{};
  return hip_status(launch_symplectic(make_kparams(*p), n, phase, dt, t, sv, st, ace, arho, ws,
                                      (hipStream_t)stream));
}

sph_status sph_verlet_step(const sph_params* p, int64_t n, int32_t mode, const double* dt,
                           double* t, sph_state* prev, sph_state* s, const float* ace,
                           const float* arho, void* ws, size_t ws_bytes, void* stream) {
  if (!params_ok(p) || !n_ok(n) || !dt || !t || !ws) return SPH_E_ARG;
  if (mode != 0 && mode != 1) return SPH_E_ARG;
  if (n > 0 && (!state_ok(s, true) || !prev || !prev->vel || !prev->rho || !ace || !arho ||
                f64_state(s)))
    return SPH_E_ARG;
  if (ws_bytes < ws_layout(n).total) return SPH_E_WORKSPACE;
  sph_state pv = n > 0 ? *prev : sph_state{}, st = n > 0 ? *s : sph_state{};
  return hip_status(launch_verlet(make_kparams(*p), n, mode, dt, t, pv, st, ace, arho, ws,
                                  (hipStream_t)stream));
}

sph_status sph_mdbc(const sph_params* p, int64_t n, sph_state* s, const uint32_t* key,
                    const uint32_t* cell_start, void* ws, size_t ws_bytes, void* stream) {
  if (!params_ok(p) || !n_ok(n) || !cell_start || !ws || p->boundary != 1) return SPH_E_ARG;
  if (n > 0 && (!state_ok(s, true) || !s->normal || !key || f64_state(s))) return SPH_E_ARG;
  if (ws_bytes < ws_layout(n).total) return SPH_E_WORKSPACE;
  if (n == 0) return SPH_OK;
  return hip_status(launch_mdbc(make_kparams(*p), n, *s, key, cell_start, ws, (hipStream_t)stream));
}

sph_status sph_floating_step(const sph_params* p, int64_t n, int32_t phase, const double* dt,
                             sph_body* bodies, int32_t n_bodies, const sph_state* saved,
                             sph_state* s, const float* ace, void* ws, size_t ws_bytes,
                             void* stream) {
  if (!params_ok(p) || !n_ok(n) || !dt || !ws || !bodies || p->floating != 1) return SPH_E_ARG;
  if (phase != 0 && phase != 1) return SPH_E_ARG;
  if (n_bodies < 1 || n_bodies > SPH_MAX_BODIES) return SPH_E_ARG;
  if (n > 0 && (!state_ok(s, true) || !s->id || !saved || !saved->pos || !ace || f64_state(s)))
    return SPH_E_ARG;
  if (ws_bytes < ws_layout(n).total) return SPH_E_WORKSPACE;
  sph_state sv = n > 0 ? *saved : sph_state{}, st = n > 0 ? *s : sph_state{};
  return hip_status(launch_floating(make_kparams(*p), n, phase, dt, bodies, n_bodies, sv, st, ace,
                                    ws, (hipStream_t)stream));
}

sph_status sph_shifting(const sph_params* p, int64_t n, sph_state* s, const uint32_t* key,
                        const uint32_t* cell_start, const double* dt, float* conc,
                        float* shift, uint32_t flags, void* ws, size_t ws_bytes, void* stream) {
  if (!params_ok(p) || !n_ok(n) || !cell_start || !dt || !ws) return SPH_E_ARG;
  if (!(p->shift_coef > 0.0)) return SPH_E_ARG;
  if (flags & ~(uint32_t)SPH_INTERACT_REUSE_CELLS) return SPH_E_ARG;
  if ((flags & SPH_INTERACT_REUSE_CELLS) &&
      (p->boundary != 0 || !periodic_reach_ok(p, p->cell_div + 1)))
    return SPH_E_ARG;
  if (n > 0 && (!state_ok(s, true) || !key || f64_state(s))) return SPH_E_ARG;
  if (ws_bytes < ws_layout(n).total) return SPH_E_WORKSPACE;
  if (n == 0) return SPH_OK;
  return hip_status(launch_shifting(make_kparams(*p), n, *s, key, cell_start, dt, conc, shift,
                                    (flags & SPH_INTERACT_REUSE_CELLS) != 0, ws,
                                    (hipStream_t)stream));
}

int32_t sph_read_error(const void* ws) {
  if (!ws) return SPH_E_ARG;
  uint32_t v = 0;
  if (hipDeviceSynchronize() != hipSuccess) return SPH_E_HIP;
  if (hipMemcpy(&v, ws, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return SPH_E_HIP;
  return (int32_t)(v & 0x7fffffffu);
}

sph_status sph_clear_error(void* ws, void* stream) {
  if (!ws) return SPH_E_ARG;
  return hip_status(launch_clear_error(ws, (hipStream_t)stream));
}

// ---------------------------------------------------------------- batches --
static bool batch_ok(const sph_batch* b) {
  return b && b->n_slots >= 1 && b->n_slots <= SPH_BATCH_MAX_SLOTS && b->table &&
         (b->cell_div == 1 || b->cell_div == 2) && b->n_total >= 0 &&
         b->n_total < ((int64_t)1 << 27) && b->key_cells >= 1 &&
         b->key_cells < (int64_t)0xfffffff0ll;
}

static BatchDesc batch_desc(const sph_batch* b) {
  return BatchDesc{b->n_slots, b->cell_div, b->n_total, b->key_cells, b->table, b->flags,
                   b->lanes};
}

size_t sph_batch_table_bytes(int32_t n_slots) {
  if (n_slots < 1 || n_slots > SPH_BATCH_MAX_SLOTS) return 0;
  return sizeof(SlotEntry) * (size_t)n_slots;
}

sph_status sph_batch_describe(const sph_params* params, const int64_t* offsets, int32_t n_slots,
                              uint32_t options, void* table_host, size_t table_bytes,
                              sph_batch* batch) {
  if (!params || !offsets || !table_host || !batch) return SPH_E_ARG;
  if (options & ~(uint32_t)SPH_BATCH_FOUR_LANES) return SPH_E_ARG;
  if (n_slots < 1 || n_slots > SPH_BATCH_MAX_SLOTS) return SPH_E_ARG;
  if (table_bytes < sph_batch_table_bytes(n_slots)) return SPH_E_ARG;
  if (offsets[0] != 0) return SPH_E_ARG;
  SlotEntry* tab = (SlotEntry*)table_host;
  uint64_t cbase = 0;
  bool general = false, periodic = false;
  for (int s = 0; s < n_slots; ++s) {
    const sph_params* p = &params[s];
    if (!params_ok(p) || p->cell_div != params[0].cell_div) return SPH_E_ARG;
    // the batch takes DBC walls and no floating bodies; formulation options
    // (cubic spline kernel, laminar viscosity, Fourtakas DDT) and periodic
    // components per slot, the latter long enough for the reused-cells pass
    if (p->boundary != 0 || p->floating != 0) return SPH_E_ARG;
    const bool per = p->period[0] > 0.0 || p->period[1] > 0.0 || p->period[2] > 0.0;
    if (per && !periodic_reach_ok(p, p->cell_div + 1)) return SPH_E_ARG;
    general = general || p->kernel != 0 || p->viscosity != 0 || p->ddt == 2;
    periodic = periodic || per;
    if (offsets[s + 1] < offsets[s]) return SPH_E_ARG;
    SlotEntry e{};
    e.kp = make_slot_kparams(*p);
    e.cbase = (uint32_t)cbase;
    e.off = offsets[s];
    e.n = offsets[s + 1] - offsets[s];
    tab[s] = e;
    cbase += (uint64_t)e.kp.ncell_total + 1;
    if (cbase >= 0xfffffff0ull) return SPH_E_ARG;
  }
  if (offsets[n_slots] >= ((int64_t)1 << 27)) return SPH_E_ARG;
  bool aligned = true;
  for (int s = 0; s <= n_slots; ++s) aligned = aligned && offsets[s] % 64 == 0;
  // interaction lanes: with SPH_BATCH_FOUR_LANES and wave-aligned slots,
  // four per target for a slot of at most kLanesMaxN particles (by its own
  // size only), else one
  const bool four = aligned && (options & SPH_BATCH_FOUR_LANES);
  int64_t lanes = 0;
  for (int s = 0; s < n_slots; ++s) {
    tab[s].lpt = four && tab[s].n <= kLanesMaxN ? kMaxLanes : 1;
    tab[s].loff = lanes;
    lanes += tab[s].n * tab[s].lpt;
  }
  batch->n_slots = n_slots;
  batch->flags = (aligned ? SPH_BATCH_WAVE_ALIGNED : 0u) | (four ? SPH_BATCH_FOUR_LANES : 0u) |
                 (general ? SPH_BATCH_GENERAL : 0u) | (periodic ? SPH_BATCH_PERIODIC : 0u);
  batch->lanes = (uint32_t)lanes;
  batch->cell_div = params[0].cell_div;
  batch->n_total = offsets[n_slots];
  batch->key_cells = (int64_t)cbase;
  batch->table = nullptr;
  return SPH_OK;
}

size_t sph_batch_workspace_bytes(const sph_batch* b) {
  if (!b || b->n_slots < 1 || b->n_total < 0) return 0;
  return batch_ws_layout(b->n_slots, b->n_total).total;
}

sph_status sph_batch_bin_cells(const sph_batch* b, const sph_state* in, sph_state* out,
                               const sph_state* carry_in, sph_state* carry_out, uint32_t* key,
                               uint32_t* perm, uint32_t* cell_start, void* ws, size_t ws_bytes,
                               void* stream) {
  if (!batch_ok(b) || !cell_start || !ws) return SPH_E_ARG;
  const int64_t n = b->n_total;
  if (n > 0 && (!state_ok(in, true) || !state_ok(out, true) || !key || !perm)) return SPH_E_ARG;
  if (n > 0 && in->pos == out->pos) return SPH_E_ARG;
  if ((carry_in == nullptr) != (carry_out == nullptr)) return SPH_E_ARG;
  if (carry_in && n > 0 && (!state_ok(carry_in, false) || !state_ok(carry_out, false)))
    return SPH_E_ARG;
  if (n > 0 && (f64_state(in) || f64_state(out) || f64_state(carry_in) || f64_state(carry_out)))
    return SPH_E_ARG;
  if (ws_bytes < batch_ws_layout(b->n_slots, n).total) return SPH_E_WORKSPACE;
  sph_state i0 = n > 0 ? *in : sph_state{}, o0 = n > 0 ? *out : sph_state{};
  return hip_status(launch_batch_bin_cells(batch_desc(b), i0, o0, carry_in, carry_out, key, perm,
                                           cell_start, ws, (hipStream_t)stream));
}

sph_status sph_batch_interact(const sph_batch* b, const sph_state* s, const uint32_t* key,
                              const uint32_t* cell_start, float* ace, float* arho, float* visc,
                              uint32_t* nbr_count, uint32_t flags, void* ws, size_t ws_bytes,
                              void* stream) {
  if (!batch_ok(b) || !cell_start || !ws || b->key_cells >= ((int64_t)1 << 30)) return SPH_E_ARG;
  if (flags & ~(uint32_t)SPH_INTERACT_REUSE_CELLS) return SPH_E_ARG;
  if (b->n_total > 0 && (!state_ok(s, true) || !key || !ace || !arho || f64_state(s)))
    return SPH_E_ARG;
  if (ws_bytes < batch_ws_layout(b->n_slots, b->n_total).total) return SPH_E_WORKSPACE;
  return hip_status(launch_batch_interact(batch_desc(b), key, cell_start, ace, arho, visc,
                                          nbr_count, (flags & SPH_INTERACT_REUSE_CELLS) != 0, ws,
                                          (hipStream_t)stream));
}

sph_status sph_batch_refresh_view(const sph_batch* b, sph_state* s, const uint32_t* key, void* ws,
                                  size_t ws_bytes, void* stream) {
  if (!batch_ok(b) || !ws) return SPH_E_ARG;
  if (b->n_total > 0 && (!state_ok(s, true) || !key || f64_state(s))) return SPH_E_ARG;
  if (ws_bytes < batch_ws_layout(b->n_slots, b->n_total).total) return SPH_E_WORKSPACE;
  sph_state s0 = b->n_total > 0 ? *s : sph_state{};
  return hip_status(launch_batch_refresh_view(batch_desc(b), s0, key, ws, (hipStream_t)stream));
}

sph_status sph_batch_reduce_dt(const sph_batch* b, double* dt, uint64_t* interactions, void* ws,
                               size_t ws_bytes, void* stream) {
  if (!batch_ok(b) || !dt || !ws) return SPH_E_ARG;
  if (ws_bytes < batch_ws_layout(b->n_slots, b->n_total).total) return SPH_E_WORKSPACE;
  return hip_status(
      launch_batch_reduce_dt(batch_desc(b), dt, interactions, ws, (hipStream_t)stream));
}

sph_status sph_batch_symplectic_step(const sph_batch* b, int32_t phase, const double* dt,
                                     double* t, sph_state* saved, sph_state* s, const float* ace,
                                     const float* arho, void* ws, size_t ws_bytes, void* stream) {
  if (!batch_ok(b) || !dt || !t || !ws) return SPH_E_ARG;
  if (phase != 0 && phase != 1) return SPH_E_ARG;
  if (b->n_total > 0 && (!state_ok(s, true) || !state_ok(saved, false) || !ace || !arho ||
                         f64_state(s) || f64_state(saved)))
    return SPH_E_ARG;
  if (ws_bytes < batch_ws_layout(b->n_slots, b->n_total).total) return SPH_E_WORKSPACE;
  sph_state sv = b->n_total > 0 ? *saved : sph_state{}, st = b->n_total > 0 ? *s : sph_state{};
  return hip_status(launch_batch_symplectic(batch_desc(b), phase, dt, t, sv, st, ace, arho, ws,
                                            (hipStream_t)stream));
}

sph_status sph_batch_shifting(const sph_batch* b, sph_state* s, const uint32_t* key,
                              const uint32_t* cell_start, const double* dt, float* conc,
                              float* shift, uint32_t flags, void* ws, size_t ws_bytes,
                              void* stream) {
  if (!batch_ok(b) || !cell_start || !dt || !ws) return SPH_E_ARG;
  if (flags & ~(uint32_t)SPH_INTERACT_REUSE_CELLS) return SPH_E_ARG;
  if (b->n_total > 0 && (!state_ok(s, true) || !key || f64_state(s))) return SPH_E_ARG;
  if (ws_bytes < batch_ws_layout(b->n_slots, b->n_total).total) return SPH_E_WORKSPACE;
  if (b->n_total == 0) return SPH_OK;
  return hip_status(launch_batch_shifting(batch_desc(b), *s, key, cell_start, dt, conc, shift,
                                          (flags & SPH_INTERACT_REUSE_CELLS) != 0, ws,
                                          (hipStream_t)stream));
}

sph_status sph_batch_read_errors(const sph_batch* b, const void* ws, uint32_t* slot_errors) {
  if (!b || b->n_slots < 1 || b->n_slots > SPH_BATCH_MAX_SLOTS || !ws || !slot_errors)
    return SPH_E_ARG;
  const BatchWsLayout W = batch_ws_layout(b->n_slots, b->n_total);
  if (hipDeviceSynchronize() != hipSuccess) return SPH_E_HIP;
  if (hipMemcpy(slot_errors, (const char*)ws + W.slot_err, sizeof(uint32_t) * b->n_slots,
                hipMemcpyDeviceToHost) != hipSuccess)
    return SPH_E_HIP;
  return SPH_OK;
}

sph_status sph_batch_clear_errors(const sph_batch* b, void* ws, void* stream) {
  if (!b || b->n_slots < 1 || b->n_slots > SPH_BATCH_MAX_SLOTS || !ws) return SPH_E_ARG;
  return hip_status(launch_batch_clear_errors(batch_desc(b), ws, (hipStream_t)stream));
}

const char* sph_strerror(sph_status s) {
  switch (s) {
    case SPH_OK: return "ok";
    case SPH_E_ARG: return "invalid argument";
    case SPH_E_WORKSPACE: return "workspace too small";
    case SPH_E_HIP: return "HIP runtime or launch error";
  }
  return "unknown status";
}

}  // extern "C"
