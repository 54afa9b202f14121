/*
 * CPU oracle for the WCSPH particle-interaction step (test infrastructure).
 * FP64, brute-force neighbour search, OpenMP over target particles.  See
 * sph_oracle.h for the conventions.  Each function names the passage of the
 * DualSPHysics v5.0 paper (arXiv 2104.00537) it follows, and the reading
 * taken where the printed formula is garbled or silent.
 *
 * Compile without floating-point contraction (-ffp-contract=off): the cell
 * key and the FP64 neighbour test are specified operation by operation.
 */
#include "sph_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EXCLUDED 0x80u
#define ORC_FLUID 0u
#define ORC_MOVING 2u
#define ORC_FLOATING 3u

static int is_fluid(uint8_t t) { return (t & 0x7fu) == ORC_FLUID; }
static int is_floating(uint8_t t) { return (t & 0x7fu) == ORC_FLOATING; }
static int is_excluded(uint8_t t) { return (t & ORC_EXCLUDED) != 0; }

/* Normalisation alpha_D of the Wendland C2 kernel, Eq. 11: 7/(4 pi h^2) in
 * 2-D and 21/(16 pi h^3) in 3-D (the printed "7/4 pi h^2" read as a single
 * fraction; a unit integral of W pins it). */
static double wendland_alpha(double h, int32_t dim) {
  if (dim == 2) return 7.0 / (4.0 * M_PI * h * h);
  return 21.0 / (16.0 * M_PI * h * h * h);
}

/* Eq. 11: W(r, h) = alpha_D (1 - q/2)^4 (2q + 1) for 0 <= q <= 2, q = r/h. */
double orc_wendland_w(double r, double h, int32_t dim) {
  double q = r / h;
  if (q < 0.0 || q > 2.0) return 0.0;
  double w = 1.0 - 0.5 * q;
  return wendland_alpha(h, dim) * w * w * w * w * (2.0 * q + 1.0);
}

/* Gradient of Eq. 11 written as grad_a W_ab = F_ab r_ab with r_ab = r_a - r_b.
 * d/dq [(1 - q/2)^4 (2q + 1)] = -5 q (1 - q/2)^3, and dq/dr = 1/h, so
 * grad W = alpha_D (1/h) (-5 q (1 - q/2)^3) r_ab / r = -5 alpha_D / h^2
 * (1 - q/2)^3 r_ab, i.e. F_ab = -5 alpha_D (1 - q/2)^3 / h^2 (finite at r=0). */
double orc_wendland_fab(double r, double h, int32_t dim) {
  double q = r / h;
  if (q < 0.0 || q >= 2.0) return 0.0;
  double w = 1.0 - 0.5 * q;
  return -5.0 * wendland_alpha(h, dim) * w * w * w / (h * h);
}

/* Normalisation alpha_D of the cubic spline, Eq. 10: 10/(7 pi h^2) in 2-D and
 * 1/(pi h^3) in 3-D. */
static double cubic_alpha(double h, int32_t dim) {
  if (dim == 2) return 10.0 / (7.0 * M_PI * h * h);
  return 1.0 / (M_PI * h * h * h);
}

/* Eq. 10: W = alpha_D (1 - 3/2 q^2 + 3/4 q^3) for q <= 1, alpha_D (2 - q)^3 / 4
 * for 1 < q <= 2, 0 beyond. */
double orc_cubic_w(double r, double h, int32_t dim) {
  double q = r / h;
  if (q < 0.0 || q > 2.0) return 0.0;
  if (q <= 1.0) return cubic_alpha(h, dim) * (1.0 - 1.5 * q * q + 0.75 * q * q * q);
  double u = 2.0 - q;
  return cubic_alpha(h, dim) * 0.25 * u * u * u;
}

/* Gradient of Eq. 10 as grad_a W_ab = F_ab r_ab: dW/dq = alpha_D (-3q + 9/4 q^2)
 * for q <= 1 and -3/4 alpha_D (2 - q)^2 beyond, times dq/dr / r = 1/(h r) =
 * 1/(h^2 q): F_ab = alpha_D/h^2 (-3 + 9/4 q) and -3/4 alpha_D/h^2 (2-q)^2/q. */
double orc_cubic_fab(double r, double h, int32_t dim) {
  double q = r / h;
  if (q < 0.0 || q >= 2.0) return 0.0;
  double k = cubic_alpha(h, dim) / (h * h);
  if (q <= 1.0) return k * (-3.0 + 2.25 * q);
  double u = 2.0 - q;
  return -0.75 * k * u * u / q;
}

static double kernel_w(const orc_params* p, double r) {
  return p->kernel == 1 ? orc_cubic_w(r, p->h, p->dim) : orc_wendland_w(r, p->h, p->dim);
}

static double kernel_fab(const orc_params* p, double r) {
  return p->kernel == 1 ? orc_cubic_fab(r, p->h, p->dim) : orc_wendland_fab(r, p->h, p->dim);
}

/* Hydrostatic part of the density difference rho_b - rho_a for the DDT of
 * Fourtakas et al., Eq. 19-20: the hydrostatic pressure difference
 * P^H_ab = rho0 g z_ab (z_ab = z_a - z_b along the vertical, the last axis;
 * g the magnitude of gravity along it) turned into a density difference by
 * the inverse of Eq. 28, rho^H_ab = rho0 [(1 + P^H_ab / B)^(1/gamma) - 1]. */
static double hydrostatic_drho(const orc_params* p, double z_ab) {
  const double b = p->c0 * p->c0 * p->rho0 / p->gamma;
  const double g = fabs(p->gravity[p->dim - 1]);
  const double ph = p->rho0 * g * z_ab;
  return p->rho0 * (pow(1.0 + ph / b, 1.0 / p->gamma) - 1.0);
}

/* Eq. 28: P = (c^2 rho0 / gamma) [(rho/rho0)^gamma - 1], with the constant
 * numerical speed of sound c = c0 (Section 2.4). */
double orc_pressure(const orc_params* p, double rho) {
  double b = p->c0 * p->c0 * p->rho0 / p->gamma;
  return b * (pow(rho / p->rho0, p->gamma) - 1.0);
}

/* Periodic boundaries, Section 2.7: along a periodic component k the domain
 * is [origin_k, origin_k + L_k) and repeats with period L_k, so that a
 * particle near one end sees those near the other end as neighbours.
 * Distances take the nearest image: d - L if d > L/2, d + L if d < -L/2
 * (one image suffices while L exceeds twice the support 2h). */
static double min_image(const orc_params* p, int k, double d) {
  const double L = p->period[k];
  if (L > 0.0) {
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
  }
  return d;
}

/* A particle that left [origin, origin + L) along a periodic component
 * re-enters at the other end: x - L, or x + L (and origin if x + L rounds
 * to the end itself).  Excluded particles are left alone. */
void orc_wrap(const orc_params* p, int64_t n, double* pos, const uint8_t* type) {
  for (int k = 0; k < p->dim; ++k) {
    const double L = p->period[k], o = p->origin[k];
    if (!(L > 0.0)) continue;
    for (int64_t a = 0; a < n; ++a) {
      if (type && is_excluded(type[a])) continue;
      double x = pos[k * n + a];
      if (x >= o + L) {
        x = x - L;
      } else if (x < o) {
        x = x + L;
        if (x >= o + L) x = o;
      }
      pos[k * n + a] = x;
    }
  }
}

/* Cell key of Section 5.1's cell-linked list: the cell index along each axis
 * is floor((x - origin) * inv) (an FP64 subtraction, then an FP64
 * multiplication) with inv the inverse cell size of that axis
 * (inv_cell_size, times x_sub along x), and cells are numbered with x
 * fastest, then y, then z.  A particle outside the grid gets the key
 * ncell_total. */
uint32_t orc_cell_key(const orc_params* p, const double* pos, int64_t n, int64_t i) {
  int64_t c[3] = {0, 0, 0};
  for (int k = 0; k < p->dim; ++k) {
    double d = pos[k * n + i] - p->origin[k];
    double inv = p->inv_cell_size * (k == 0 && p->x_sub > 1 ? (double)p->x_sub : 1.0);
    double s = d * inv;
    double f = floor(s);
    /* a wrapped coordinate lies in [origin, origin + L): a product that
     * rounds up to the end is the last cell */
    if (p->period[k] > 0.0 && f == (double)p->ncell[k]) f -= 1.0;
    if (!(f >= 0.0) || !(f < (double)p->ncell[k]))
      return (uint32_t)((int64_t)p->ncell[0] * p->ncell[1] * p->ncell[2]);
    c[k] = (int64_t)f;
  }
  return (uint32_t)(c[0] + (int64_t)p->ncell[0] * (c[1] + (int64_t)p->ncell[1] * c[2]));
}

void orc_cell_keys(const orc_params* p, int64_t n, const double* pos, uint32_t* key) {
  for (int64_t i = 0; i < n; ++i) key[i] = orc_cell_key(p, pos, n, i);
}

/* Stable ascending sort of particles by cell key (ties keep input order):
 * perm[j] is the input index of the j-th particle in sorted order. */
typedef struct { uint32_t key; uint32_t idx; } key_idx;

static int cmp_key_idx(const void* a, const void* b) {
  const key_idx* x = (const key_idx*)a;
  const key_idx* y = (const key_idx*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
  return 0;
}

void orc_sort_perm(int64_t n, const uint32_t* key, uint32_t* perm) {
  key_idx* a = (key_idx*)malloc(sizeof(key_idx) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) { a[i].key = key[i]; a[i].idx = (uint32_t)i; }
  qsort(a, (size_t)n, sizeof(key_idx), cmp_key_idx);
  for (int64_t i = 0; i < n; ++i) perm[i] = a[i].idx;
  free(a);
}

/* First particle of every cell in sorted order (Section 5.1): start[c] is the
 * number of particles whose key is below c, for c = 0..ncell_total, so cell c
 * holds sorted particles [start[c], start[c+1]) and start[ncell_total] counts
 * the particles inside the grid. */
void orc_cell_start(int64_t n, const uint32_t* sorted_key, int64_t ncell_total,
                    uint32_t* start) {
  uint32_t* count = (uint32_t*)calloc((size_t)ncell_total + 2, sizeof(uint32_t));
  for (int64_t i = 0; i < n; ++i) {
    uint32_t k = sorted_key[i];
    if ((int64_t)k > ncell_total) k = (uint32_t)ncell_total;
    count[k]++;
  }
  uint32_t run = 0;
  for (int64_t c = 0; c <= ncell_total; ++c) { start[c] = run; run += count[c]; }
  free(count);
}

static double particle_mass(const orc_params* p, uint8_t t) {
  return is_fluid(t) ? p->mass_fluid : p->mass_bound;
}

/* One particle-interaction pass (Section 2.3) for the listed targets, by
 * brute force over every particle b != a with |r_ab|^2 < (2h)^2 (Eq. 4 with
 * k = 2).  For a target a:
 *
 *  a fluid (Eq. 22 with Eq. 21, Eq. 15 with Eq. 17-18):
 *    dv_a/dt   = g - sum_b m_b [(P_a + P_b)/(rho_a rho_b) + Pi_ab] grad_a W_ab
 *    Pi_ab     = -alpha c0 mu_ab / rhobar_ab   if v_ab . r_ab < 0, else 0
 *    mu_ab     = h v_ab . r_ab / (r_ab^2 + eta^2),  rhobar_ab = (rho_a+rho_b)/2
 *    drho_a/dt = rho_a sum_b (m_b/rho_b) v_ab . grad_a W_ab + D_a
 *    D_a       = delta h c0 sum_{b in F} psi_ab . grad_a W_ab V_b
 *    visc_a    = max_b |mu_ab|          (the per-particle term of Eq. 35)
 *
 *  a wall (Eq. 36): drho_a/dt = rho_a sum_{b in F} (m_b/rho_b) v_ab.grad_a W_ab
 *  and no momentum sum (its motion is imposed, Eq. 37).
 *
 *  a floating particle (type 3, Section 3.2): the density of a wall (Eq. 36)
 *  and, by Eq. 47, the momentum sum of a fluid target taken over its fluid
 *  neighbours only and without gravity (which acts on the whole body, see
 *  orc_body_step):
 *    dv_a/dt = - sum_{b in F} m_b [(P_a + P_b)/(rho_a rho_b) + Pi_ab] grad_a W_ab.
 *  In every sum a floating particle b is a boundary particle of mass
 *  mass_bound (K is a subset of B); then the force m_B dv_a/dt on a floating
 *  particle is exactly opposite to the force its fluid neighbours receive
 *  from it.  visc_a stays 0 (Eq. 35 runs over fluid only).
 *
 * Distances along periodic components take the nearest image (Section
 * 2.7, min_image).
 *
 * Readings: the mean in Eq. 21 is (x_a + x_b)/2; eta^2 = eta2 (the case uses
 * 0.001 h^2); c_a and cbar_ab are the constant c0; psi_ab of Eq. 18 is taken
 * along r_ba = r_b - r_a, the diffusive direction of the Molteni-Colagrossi
 * term, so psi_ab . grad_a W_ab = 2 (rho_b - rho_a)(-F_ab) with F_ab < 0;
 * density diffusion acts between fluid particles only.
 *
 * Options: kernel 1 takes the cubic spline of Eq. 10 for W; viscosity 1
 * replaces Pi_ab by the laminar term of Eq. 23,
 *   dv_a/dt += sum_b m_b 4 nu0 (r_ab . grad_a W_ab) / ((rho_a + rho_b)(r_ab^2 + eta^2)) v_ab,
 * (visc_a and Eq. 35 unchanged); ddt 2 takes psi_ab of Eq. 19, i.e. rho_b -
 * rho_a above becomes (rho_b - rho_a) - rho^H_ab (hydrostatic_drho).
 *
 * nbr[a] counts the pairs evaluated for a: all neighbours of a fluid target,
 * the fluid neighbours of a wall target.  Outputs are indexed by target slot;
 * ace is [dim][ntarget].  Excluded particles take no part and get zeros. */
void orc_interact(const orc_params* p, int64_t n, const double* pos,
                  const double* vel, const double* rho, const uint8_t* type,
                  int64_t ntarget, const int64_t* target, double* ace,
                  double* arho, double* visc, uint32_t* nbr) {
  const int dim = p->dim;
  const double h = p->h;
  const double support2 = (2.0 * h) * (2.0 * h);

#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < ntarget; ++s) {
    const int64_t a = target ? target[s] : s;
    double acc[3] = {0.0, 0.0, 0.0};
    double cont = 0.0, diff = 0.0, vmax = 0.0;
    uint32_t count = 0;
    const uint8_t ta = type[a];
    /* with modified DBC the wall density comes from orc_mdbc (Eq. 38), not
     * from Eq. 36: wall targets get no sums */
    if (!is_excluded(ta) && (is_fluid(ta) || p->boundary == 0)) {
      const int fa = is_fluid(ta);
      const int ka = is_floating(ta);
      const double rho_a = rho[a];
      const double p_a = orc_pressure(p, rho_a);
      for (int64_t b = 0; b < n; ++b) {
        if (b == a) continue;
        const uint8_t tb = type[b];
        if (is_excluded(tb)) continue;
        const int fb = is_fluid(tb);
        if (!fa && !fb) continue;  /* Eq. 36 sums over fluid b only */
        double dx[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
        for (int k = 0; k < dim; ++k) {
          dx[k] = min_image(p, k, pos[k * n + a] - pos[k * n + b]);
          r2 += dx[k] * dx[k];
        }
        if (!(r2 < support2)) continue;
        const double r = sqrt(r2);
        const double fab = kernel_fab(p, r);
        double vr = 0.0;
        for (int k = 0; k < dim; ++k) vr += (vel[k * n + a] - vel[k * n + b]) * dx[k];
        const double rho_b = rho[b];
        const double m_b = particle_mass(p, tb);
        const double vol_b = m_b / rho_b;
        cont += vol_b * vr * fab;  /* (m_b/rho_b) v_ab . grad_a W_ab */
        count++;
        if (fa || ka) {
          const double p_b = orc_pressure(p, rho_b);
          const double mu = h * vr / (r2 + p->eta2);
          const double rhobar = 0.5 * (rho_a + rho_b);
          double pi_ab = 0.0;
          if (p->viscosity == 0) {
            pi_ab = vr < 0.0 ? -p->alpha * p->c0 * mu / rhobar : 0.0;
          } else {
            const double lam =
                m_b * 4.0 * p->visc_nu * (fab * r2) / ((rho_a + rho_b) * (r2 + p->eta2));
            for (int k = 0; k < dim; ++k) acc[k] += lam * (vel[k * n + a] - vel[k * n + b]);
          }
          const double coef = m_b * ((p_a + p_b) / (rho_a * rho_b) + pi_ab);
          for (int k = 0; k < dim; ++k) acc[k] -= coef * fab * dx[k];
          if (fa && fabs(mu) > vmax) vmax = fabs(mu);
          if (fa && p->ddt && fb) {
            double drho = rho_b - rho_a;
            if (p->ddt == 2) drho -= hydrostatic_drho(p, dx[dim - 1]);
            const double psi_dot_grad = 2.0 * drho * (-fab);
            diff += psi_dot_grad * vol_b;
          }
        }
      }
      if (fa) {
        for (int k = 0; k < dim; ++k) acc[k] += p->gravity[k];
        arho[s] = rho_a * cont + p->delta * h * p->c0 * diff;
      } else {
        arho[s] = rho_a * cont;
      }
    } else {
      arho[s] = 0.0;
    }
    for (int k = 0; k < dim; ++k) ace[k * ntarget + s] = acc[k];
    if (visc) visc[s] = vmax;
    if (nbr) nbr[s] = count;
  }
}

/* Eq. 35 with C_CFL = cfl and c_s = c0: dt_f = min_a sqrt(h/|f_a|) and
 * dt_cv = min_a h/(c0 + visc_a) over fluid particles (|f_a| is the full
 * acceleration including gravity); dt = cfl min(dt_f, dt_cv). */
double orc_time_step(const orc_params* p, int64_t n, const uint8_t* type,
                     const double* ace, const double* visc) {
  double dt_f = INFINITY, dt_cv = INFINITY;
  for (int64_t a = 0; a < n; ++a) {
    if (!is_fluid(type[a]) || is_excluded(type[a])) continue;
    double f2 = 0.0;
    for (int k = 0; k < p->dim; ++k) f2 += ace[k * n + a] * ace[k * n + a];
    const double f = sqrt(f2);
    if (f > 0.0) {
      const double t1 = sqrt(p->h / f);
      if (t1 < dt_f) dt_f = t1;
    }
    const double t2 = p->h / (p->c0 + visc[a]);
    if (t2 < dt_cv) dt_cv = t2;
  }
  const double m = dt_f < dt_cv ? dt_f : dt_cv;
  return p->cfl * m;
}

/* Imposed wall motion along x (Eq. 37 with a predefined law): displacement
 * D(t) = (A/w^2)(1 - cos wt) and velocity (A/w) sin wt, so the wall starts at
 * rest and its acceleration is A cos wt. */
static double motion_disp(const orc_params* p, double t) {
  if (p->motion_omega == 0.0) return 0.0;
  const double w = p->motion_omega;
  return p->motion_amp / (w * w) * (1.0 - cos(w * t));
}
static double motion_vel(const orc_params* p, double t) {
  if (p->motion_omega == 0.0) return 0.0;
  const double w = p->motion_omega;
  return p->motion_amp / w * sin(w * t);
}

/* Symplectic predictor, Eq. 33 (first two lines) and Eq. 34 (first line):
 * saves the state at n, then r^{n+1/2} = r^n + dt/2 v^n,
 * v^{n+1/2} = v^n + dt/2 F^n, rho^{n+1/2} = rho^n + dt/2 R^n for fluid;
 * walls update density only, and moving walls take their imposed position
 * and velocity at t + dt/2. */
void orc_predictor(const orc_params* p, int64_t n, double dt, double t,
                   double* pos, double* vel, double* rho, const uint8_t* type,
                   const double* ace, const double* arho, double* pos_n,
                   double* vel_n, double* rho_n) {
  const int dim = p->dim;
  const double hdt = 0.5 * dt;
  const double dmove = motion_disp(p, t + hdt) - motion_disp(p, t);
  const double vmove = motion_vel(p, t + hdt);
  for (int64_t a = 0; a < n; ++a) {
    for (int k = 0; k < dim; ++k) {
      pos_n[k * n + a] = pos[k * n + a];
      vel_n[k * n + a] = vel[k * n + a];
    }
    rho_n[a] = rho[a];
    if (is_excluded(type[a])) continue;
    if (is_fluid(type[a])) {
      for (int k = 0; k < dim; ++k) {
        pos[k * n + a] = pos_n[k * n + a] + hdt * vel_n[k * n + a];
        vel[k * n + a] = vel_n[k * n + a] + hdt * ace[k * n + a];
      }
    } else if ((type[a] & 0x7fu) == ORC_MOVING) {
      pos[a] = pos_n[a] + dmove;
      vel[a] = vmove;
    }
    rho[a] = rho_n[a] + hdt * arho[a];
  }
}

/* Symplectic corrector, Eq. 33 (last two lines) and Eq. 34 (second line):
 * v^{n+1} = v^n + dt F^{n+1/2}, r^{n+1} = r^n + dt (v^{n+1} + v^n)/2 for
 * fluid; for every particle eps = -(R^{n+1/2}/rho^{n+1/2}) dt and
 * rho^{n+1} = rho^n (2 - eps)/(2 + eps); moving walls take their imposed
 * position and velocity at t + dt. */
void orc_corrector(const orc_params* p, int64_t n, double dt, double t,
                   double* pos, double* vel, double* rho, const uint8_t* type,
                   const double* ace, const double* arho, const double* pos_n,
                   const double* vel_n, const double* rho_n) {
  const int dim = p->dim;
  const double dmove = motion_disp(p, t + dt) - motion_disp(p, t);
  const double vmove = motion_vel(p, t + dt);
  for (int64_t a = 0; a < n; ++a) {
    if (is_excluded(type[a])) continue;
    if (is_fluid(type[a])) {
      for (int k = 0; k < dim; ++k) {
        const double v1 = vel_n[k * n + a] + dt * ace[k * n + a];
        pos[k * n + a] = pos_n[k * n + a] + dt * 0.5 * (v1 + vel_n[k * n + a]);
        vel[k * n + a] = v1;
      }
    } else if ((type[a] & 0x7fu) == ORC_MOVING) {
      pos[a] = pos_n[a] + dmove;
      vel[a] = vmove;
    }
    const double eps = -(arho[a] / rho[a]) * dt;
    rho[a] = rho_n[a] * (2.0 - eps) / (2.0 + eps);
  }
}

/* Modified dynamic boundary condition, Section 2.6.2.  For every wall
 * particle B its ghost node G = r_B + normal_B (the mirror image of B across
 * the wall face, inside the fluid) collects the fluid particles b with
 * |r_b - r_G| < 2h.  With r = r_b - r_G, w = W(|r|), grad W = F r (the kernel
 * of the case) and V_b = m_b / rho_b, the first-order corrected SPH
 * approximation (Liu and Liu) of a field f at G solves
 *   [ sum V w      sum V w r^T    ] [ f_G      ]   [ sum V f_b w   ]
 *   [ sum V F r    sum V F r r^T  ] [ grad f_G ] = [ sum V f_b F r ]
 * which every linear f satisfies exactly (Taylor expansion about G); for
 * the density V_b rho_b = m_b.  Then rho_B = rho_G + (r_B - r_G).grad rho_G
 * (Eq. 38).  When |det| of the matrix (dimensionless: about 1 for a full
 * support) is below 1e-3, the zeroth-order Shepard value sum m w / sum V w
 * is used with no gradient.  The ghost velocity is the Shepard sum of
 * Eq. 39, v_G = sum V v_b w / sum V w, and the wall particle takes it
 * reversed about its own velocity, v_B = 2 v_wall - v_G (no slip; v_B = -v_G
 * for a fixed wall).  A wall particle with no fluid around its ghost node
 * gets rho0 and its own velocity.  Fluid and excluded particles are copied
 * unchanged.  rho_out [n], vel_out [dim][n]. */
static int solve_small(int m, double* A, double* b, double* det) {
  /* Gaussian elimination with partial pivoting on the m x m row-major A */
  double d = 1.0;
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (fabs(A[r * m + c]) > fabs(A[piv * m + c])) piv = r;
    if (A[piv * m + c] == 0.0) { *det = 0.0; return 0; }
    if (piv != c) {
      for (int k = 0; k < m; ++k) {
        double t = A[c * m + k]; A[c * m + k] = A[piv * m + k]; A[piv * m + k] = t;
      }
      double t = b[c]; b[c] = b[piv]; b[piv] = t;
      d = -d;
    }
    d *= A[c * m + c];
    for (int r = c + 1; r < m; ++r) {
      const double f = A[r * m + c] / A[c * m + c];
      for (int k = c; k < m; ++k) A[r * m + k] -= f * A[c * m + k];
      b[r] -= f * b[c];
    }
  }
  for (int c = m - 1; c >= 0; --c) {
    double s = b[c];
    for (int k = c + 1; k < m; ++k) s -= A[c * m + k] * b[k];
    b[c] = s / A[c * m + c];
  }
  *det = d;
  return 1;
}

void orc_mdbc(const orc_params* p, int64_t n, const double* pos, const double* vel,
              const double* rho, const uint8_t* type, const double* normal,
              double* rho_out, double* vel_out) {
  const int dim = p->dim;
  const int m = dim + 1;
  const double support2 = (2.0 * p->h) * (2.0 * p->h);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t a = 0; a < n; ++a) {
    rho_out[a] = rho[a];
    for (int k = 0; k < dim; ++k) vel_out[k * n + a] = vel[k * n + a];
    if (is_excluded(type[a]) || is_fluid(type[a])) continue;
    double g[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k) g[k] = pos[k * n + a] + normal[k * n + a];
    double A[16], B[4], s0 = 0.0, sv[3] = {0.0, 0.0, 0.0};
    memset(A, 0, sizeof(A));
    memset(B, 0, sizeof(B));
    for (int64_t b = 0; b < n; ++b) {
      if (is_excluded(type[b]) || !is_fluid(type[b])) continue;
      double r[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
      for (int k = 0; k < dim; ++k) {
        r[k] = min_image(p, k, pos[k * n + b] - g[k]);
        r2 += r[k] * r[k];
      }
      if (!(r2 < support2)) continue;
      const double d = sqrt(r2);
      const double w = kernel_w(p, d), f = kernel_fab(p, d);
      const double mb = particle_mass(p, type[b]);
      const double vb = mb / rho[b];
      double row0[4] = {1.0, r[0], r[1], r[2]};
      for (int k = 0; k < m; ++k) A[0 * m + k] += vb * w * row0[k];
      for (int i = 0; i < dim; ++i)
        for (int k = 0; k < m; ++k) A[(1 + i) * m + k] += vb * f * r[i] * row0[k];
      B[0] += mb * w;
      for (int i = 0; i < dim; ++i) B[1 + i] += mb * f * r[i];
      s0 += vb * w;
      for (int k = 0; k < dim; ++k) sv[k] += vb * w * vel[k * n + b];
    }
    if (!(s0 > 0.0)) {
      rho_out[a] = p->rho0;
      continue;
    }
    double det = 0.0;
    double x[4] = {B[0], B[1], B[2], B[3]};
    double rho_b;
    if (solve_small(m, A, x, &det) && fabs(det) >= 1e-3) {
      rho_b = x[0];
      for (int k = 0; k < dim; ++k) rho_b += (pos[k * n + a] - g[k]) * x[1 + k];
    } else {
      rho_b = B[0] / s0;
    }
    rho_out[a] = rho_b;
    for (int k = 0; k < dim; ++k) vel_out[k * n + a] = 2.0 * vel[k * n + a] - sv[k] / s0;
  }
}

/* Verlet step, Section 2.5.1, from state n (pos, vel, rho) with the state of
 * step n-1 (vel_p, rho_p) and the rates F^n (ace), R^n (arho):
 *   mode 0 (Eq. 30): v^{n+1} = v^{n-1} + 2 dt F^n, rho^{n+1} = rho^{n-1} + 2 dt R^n;
 *   mode 1 (Eq. 31, the intermediate step, also the first step):
 *     v^{n+1} = v^n + dt F^n, rho^{n+1} = rho^n + dt R^n;
 *   both: r^{n+1} = r^n + dt v^n + dt^2/2 F^n.
 * Positions and velocities change for fluid particles only; moving walls
 * take their imposed position and velocity at t + dt; density evolves for
 * every particle.  Afterwards vel_p, rho_p hold state n. */
void orc_verlet(const orc_params* p, int64_t n, double dt, double t, int32_t mode,
                double* pos, double* vel, double* rho, double* vel_p, double* rho_p,
                const uint8_t* type, const double* ace, const double* arho) {
  const int dim = p->dim;
  const double dmove = motion_disp(p, t + dt) - motion_disp(p, t);
  const double vmove = motion_vel(p, t + dt);
  for (int64_t a = 0; a < n; ++a) {
    if (is_excluded(type[a])) continue;
    for (int k = 0; k < dim; ++k) {
      const double vn = vel[k * n + a];
      if (is_fluid(type[a])) {
        const double f = ace[k * n + a];
        pos[k * n + a] = pos[k * n + a] + dt * vn + 0.5 * dt * dt * f;
        vel[k * n + a] = mode == 0 ? vel_p[k * n + a] + 2.0 * dt * f : vn + dt * f;
      }
      vel_p[k * n + a] = vn;
    }
    if ((type[a] & 0x7fu) == ORC_MOVING) {
      pos[a] = pos[a] + dmove;
      vel[a] = vmove;
    }
    const double rn = rho[a];
    rho[a] = mode == 0 ? rho_p[a] + 2.0 * dt * arho[a] : rn + dt * arho[a];
    rho_p[a] = rn;
  }
}

/* Floating bodies, Section 3.2.  A body is a set of floating particles
 * (type 3), here particles [first, first + count) of the arrays, moving as
 * one rigid object of total mass M, centre R0, velocity V and angular
 * velocity Omega.
 *
 * Force, torque and inertia (Eq. 48-49).  Each particle k contributes the
 * force m_B dv_k/dt, with dv_k/dt from orc_interact (Eq. 47) and m_B the
 * boundary particle mass it carries in the SPH sums, so the fluid part of
 * the force is F = sum_k m_B dv_k/dt and its torque about R0 is
 * T = sum_k m_B (r_k - R0) x dv_k/dt.  The body's own mass M sets its
 * inertia: it is shared equally by its particles, so the inertia tensor
 * about R0 is I = sum_k (M/count) (|r'|^2 1 - r' r'^T) with r' = r_k - R0.
 * In 2-D the rotation is about the axis normal to the plane of the two
 * components: Omega, T and I are scalars (stored in [0]), T = sum m_B
 * (r'_0 a_1 - r'_1 a_0) and I = sum (M/count)|r'|^2, so that a positive
 * Omega turns the first axis towards the second.
 * force [dim], torque [3] (2-D: [0]), inertia [9] row-major (2-D: [0]).
 * Excluded particles are left out. */
void orc_body_forces(const orc_params* p, int64_t n, const double* pos, const double* ace,
                     const orc_body* b, double* force, double* torque, double* inertia) {
  const int dim = p->dim;
  const double mb = p->mass_bound;
  const double mi = b->count > 0 ? b->mass / (double)b->count : 0.0;
  for (int k = 0; k < 3; ++k) { force[k] = 0.0; torque[k] = 0.0; }
  for (int k = 0; k < 9; ++k) inertia[k] = 0.0;
  for (int64_t j = b->first; j < b->first + b->count; ++j) {
    double r[3] = {0.0, 0.0, 0.0}, a[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k) {
      r[k] = pos[k * n + j] - b->center[k];
      a[k] = ace[k * n + j];
      force[k] += mb * a[k];
    }
    const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    if (dim == 2) {
      torque[0] += mb * (r[0] * a[1] - r[1] * a[0]);
      inertia[0] += mi * r2;
    } else {
      torque[0] += mb * (r[1] * a[2] - r[2] * a[1]);
      torque[1] += mb * (r[2] * a[0] - r[0] * a[2]);
      torque[2] += mb * (r[0] * a[1] - r[1] * a[0]);
      for (int u = 0; u < 3; ++u)
        for (int v = 0; v < 3; ++v)
          inertia[u * 3 + v] += mi * ((u == v ? r2 : 0.0) - r[u] * r[v]);
    }
  }
}

/* Rotation by the rotation vector th (3-D: axis th/|th|, angle |th|,
 * right-handed) of the vector x, by Rodrigues' formula
 * x' = x cos(phi) + (e x x) sin(phi) + e (e.x)(1 - cos(phi)), e the unit
 * axis; in 2-D the rotation by the angle th[0] in the plane. */
static void rotate(int dim, const double* th, const double* x, double* out) {
  if (dim == 2) {
    const double c = cos(th[0]), s = sin(th[0]);
    out[0] = c * x[0] - s * x[1];
    out[1] = s * x[0] + c * x[1];
    return;
  }
  const double phi = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
  if (phi == 0.0) {
    for (int k = 0; k < 3; ++k) out[k] = x[k];
    return;
  }
  const double e[3] = {th[0] / phi, th[1] / phi, th[2] / phi};
  const double c = cos(phi), s = sin(phi);
  const double ex[3] = {e[1] * x[2] - e[2] * x[1], e[2] * x[0] - e[0] * x[2],
                        e[0] * x[1] - e[1] * x[0]};
  const double ed = e[0] * x[0] + e[1] * x[1] + e[2] * x[2];
  for (int k = 0; k < 3; ++k) out[k] = x[k] * c + ex[k] * s + e[k] * ed * (1.0 - c);
}

/* Omega x r (Eq. 50); 2-D: omega[0] (-r_1, r_0). */
static void omega_cross(int dim, const double* om, const double* r, double* out) {
  if (dim == 2) {
    out[0] = -om[0] * r[1];
    out[1] = om[0] * r[0];
    return;
  }
  out[0] = om[1] * r[2] - om[2] * r[1];
  out[1] = om[2] * r[0] - om[0] * r[2];
  out[2] = om[0] * r[1] - om[1] * r[0];
}

/* One phase of the symplectic update of a floating body (Section 2.5.2
 * applied to Eq. 48-50), after orc_predictor / orc_corrector of the same
 * phase (which leave floating particles in place and update their density
 * as walls).  pos holds the current positions (state n in the predictor,
 * n+1/2 in the corrector) and b the current body state; pos_n and b_n hold
 * state n (phase 0 writes b_n).  With the linear and angular accelerations
 *   A = F/M + g (gravity acts on the body as a whole),
 *   alpha = I^-1 T (Eq. 49 as printed, I of the current configuration),
 * evaluated from the current state:
 *   phase 0: V = V^n + dt/2 A, Omega = Omega^n + dt/2 alpha,
 *            R0 = R0^n + dt/2 V^n, rotation by dt/2 Omega^n;
 *   phase 1: V = V^n + dt A, Omega = Omega^n + dt alpha,
 *            R0 = R0^n + dt (V + V^n)/2, rotation by dt (Omega + Omega^n)/2,
 * the position and velocity updates of Eq. 33 for the centre and the
 * orientation.  Every particle then takes the rigid motion from state n,
 *   r_k = R0 + Rot (r_k^n - R0^n),   v_k = V + Omega x (r_k - R0)  (Eq. 50).
 * force / torque (nullable) receive F and T.  Returns 0, or 1 if the
 * inertia tensor is singular. */
int32_t orc_body_step(const orc_params* p, int64_t n, int32_t phase, double dt, orc_body* b,
                      orc_body* b_n, const double* pos_n, double* pos, double* vel,
                      const uint8_t* type, const double* ace, double* force, double* torque) {
  const int dim = p->dim;
  double F[3], T[3], I[9];
  orc_body_forces(p, n, pos, ace, b, F, T, I);
  if (force) for (int k = 0; k < 3; ++k) force[k] = F[k];
  if (torque) for (int k = 0; k < 3; ++k) torque[k] = T[k];
  double A[3] = {0.0, 0.0, 0.0}, al[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < dim; ++k) A[k] = F[k] / b->mass + p->gravity[k];
  if (dim == 2) {
    if (!(I[0] > 0.0)) return 1;
    al[0] = T[0] / I[0];
  } else {
    double M[9], det = 0.0;
    for (int k = 0; k < 9; ++k) M[k] = I[k];
    for (int k = 0; k < 3; ++k) al[k] = T[k];
    if (!solve_small(3, M, al, &det) || !(fabs(det) > 0.0)) return 1;
  }
  const int nw = dim == 2 ? 1 : 3;
  double th[3] = {0.0, 0.0, 0.0};
  if (phase == 0) {
    *b_n = *b;
    for (int k = 0; k < dim; ++k) {
      b->vel[k] = b_n->vel[k] + 0.5 * dt * A[k];
      b->center[k] = b_n->center[k] + 0.5 * dt * b_n->vel[k];
    }
    for (int k = 0; k < nw; ++k) {
      b->omega[k] = b_n->omega[k] + 0.5 * dt * al[k];
      th[k] = 0.5 * dt * b_n->omega[k];
    }
  } else {
    for (int k = 0; k < dim; ++k) {
      b->vel[k] = b_n->vel[k] + dt * A[k];
      b->center[k] = b_n->center[k] + dt * 0.5 * (b->vel[k] + b_n->vel[k]);
    }
    for (int k = 0; k < nw; ++k) {
      b->omega[k] = b_n->omega[k] + dt * al[k];
      th[k] = dt * 0.5 * (b->omega[k] + b_n->omega[k]);
    }
  }
  for (int64_t j = b->first; j < b->first + b->count; ++j) {
    if (is_excluded(type[j])) continue;
    double r[3] = {0.0, 0.0, 0.0}, q[3], w[3];
    for (int k = 0; k < dim; ++k) r[k] = pos_n[k * n + j] - b_n->center[k];
    rotate(dim, th, r, q);
    omega_cross(dim, b->omega, q, w);
    for (int k = 0; k < dim; ++k) {
      pos[k * n + j] = b->center[k] + q[k];
      vel[k * n + j] = b->vel[k] + w[k];
    }
  }
  return 0;
}

/* Particle shifting, Section 2.8: Eq. 40-41 with the concentration and its
 * gradient of Eq. 53, for fluid particles:
 *   C_a      = sum_{b in P} V_b W_ab, b = a included (the kernel sum of the
 *              particle distribution: about 1 inside the fluid, lower where
 *              the support is truncated),
 *   grad C_a = sum_{b in P} V_b (C_b - C_a) grad_a W_ab,
 *   dr_a     = -D_s grad C_a,  D_s = A_s h |v_a| dt  (A_s = shift_coef),
 * with V_b = m_b / rho_b over every non-excluded particle (fluid, walls,
 * floating).  Particles move from crowded to sparse regions.  With
 * shift_fs > 0 a particle whose C_a < shift_fs (a support truncated by the
 * free surface) keeps only the tangential part of dr_a: its component along
 * n = grad C_a / |grad C_a| is removed (Eq. 54 with a_n = 0, the setting
 * the paper gives for violent flows).  Non-fluid and excluded
 * particles get dr = 0 (their C is still computed).
 * conc [n], grad [dim][n], dr [dim][n]: outputs, each nullable. */
void orc_shift(const orc_params* p, int64_t n, const double* pos, const double* vel,
               const double* rho, const uint8_t* type, double dt, double* conc, double* grad,
               double* dr) {
  const int dim = p->dim;
  const double support2 = (2.0 * p->h) * (2.0 * p->h);
  double* c = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t a = 0; a < n; ++a) {
    if (is_excluded(type[a])) continue;
    double s = 0.0;
    for (int64_t b = 0; b < n; ++b) {
      if (is_excluded(type[b])) continue;
      double r2 = 0.0;
      for (int k = 0; k < dim; ++k) {
        const double d = min_image(p, k, pos[k * n + a] - pos[k * n + b]);
        r2 += d * d;
      }
      if (!(r2 < support2)) continue;
      s += particle_mass(p, type[b]) / rho[b] * kernel_w(p, sqrt(r2));
    }
    c[a] = s;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t a = 0; a < n; ++a) {
    double g[3] = {0.0, 0.0, 0.0}, d[3] = {0.0, 0.0, 0.0};
    if (!is_excluded(type[a]) && is_fluid(type[a])) {
      for (int64_t b = 0; b < n; ++b) {
        if (b == a || is_excluded(type[b])) continue;
        double dx[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
        for (int k = 0; k < dim; ++k) {
          dx[k] = min_image(p, k, pos[k * n + a] - pos[k * n + b]);
          r2 += dx[k] * dx[k];
        }
        if (!(r2 < support2)) continue;
        const double f = kernel_fab(p, sqrt(r2));
        const double w = particle_mass(p, type[b]) / rho[b] * (c[b] - c[a]) * f;
        for (int k = 0; k < dim; ++k) g[k] += w * dx[k];
      }
      double v2 = 0.0;
      for (int k = 0; k < dim; ++k) v2 += vel[k * n + a] * vel[k * n + a];
      const double ds = p->shift_coef * p->h * sqrt(v2) * dt;
      for (int k = 0; k < dim; ++k) d[k] = -ds * g[k];
      if (p->shift_fs > 0.0 && c[a] < p->shift_fs) {
        double g2 = 0.0, dn = 0.0;
        for (int k = 0; k < dim; ++k) g2 += g[k] * g[k];
        if (g2 > 0.0) {
          for (int k = 0; k < dim; ++k) dn += d[k] * g[k];
          for (int k = 0; k < dim; ++k) d[k] -= dn / g2 * g[k];
        }
      }
    }
    for (int k = 0; k < dim; ++k) {
      if (grad) grad[k * n + a] = g[k];
      if (dr) dr[k * n + a] = d[k];
    }
    if (conc) conc[a] = c[a];
  }
  free(c);
}

/* Marks particles outside the cell grid as excluded (they leave the
 * computation for good, as the GPU path's binning does). */
static void mark_excluded(const orc_params* p, int64_t n, const double* pos,
                          uint8_t* type) {
  const uint32_t out = (uint32_t)((int64_t)p->ncell[0] * p->ncell[1] * p->ncell[2]);
  for (int64_t a = 0; a < n; ++a)
    if (orc_cell_key(p, pos, n, a) == out) type[a] |= ORC_EXCLUDED;
}

/* nsteps symplectic steps (Section 2.5.2), each: PI at n -> dt (Eq. 35, from
 * the state at n, used for both half steps) -> predictor -> PI at n+1/2 ->
 * corrector -> t += dt.  dt_hist[s] receives each step's dt (nullable);
 * *interactions accumulates the pair count of every PI (nullable).
 * Returns 0; 1 if a density became non-finite or non-positive; 2 if dt is
 * not a positive finite number (e.g. no fluid particle is left); 3 if a
 * floating body's inertia is singular.  bodies[n_bodies] (nullable): the
 * floating bodies, advanced by orc_body_step after each update phase. */
/* With modified DBC (boundary 1, normal required) each PI is preceded by
 * orc_mdbc: the wall densities it gives replace the state's, and the
 * interaction sees its wall velocities. */
static void mdbc_before_pi(const orc_params* p, int64_t n, const double* pos,
                           const double* vel, double* rho, const uint8_t* type,
                           const double* normal, double* vel_pi) {
  if (p->boundary == 1) {
    double* rho_new = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    orc_mdbc(p, n, pos, vel, rho, type, normal, rho_new, vel_pi);
    memcpy(rho, rho_new, sizeof(double) * (size_t)n);
    free(rho_new);
  } else {
    memcpy(vel_pi, vel, sizeof(double) * (size_t)p->dim * (size_t)n);
  }
}

int32_t orc_run(const orc_params* p, int64_t n, double* pos, double* vel,
                double* rho, uint8_t* type, const double* normal, int32_t nsteps, double* t,
                double* dt_hist, uint64_t* interactions, orc_body* bodies, int32_t n_bodies) {
  const int dim = p->dim;
  size_t nd = (size_t)dim * (size_t)(n > 0 ? n : 1);
  double* ace = (double*)calloc(nd, sizeof(double));
  double* arho = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double* visc = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  uint32_t* nbr = (uint32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
  double* pos_n = (double*)calloc(nd, sizeof(double));
  double* vel_n = (double*)calloc(nd, sizeof(double));
  double* rho_n = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double* vel_pi = (double*)calloc(nd, sizeof(double));
  orc_body* bodies_n =
      (orc_body*)calloc((size_t)(n_bodies > 0 ? n_bodies : 1), sizeof(orc_body));
  double* shift = (double*)calloc(nd, sizeof(double));
  int32_t status = 0;
  for (int32_t s = 0; s < nsteps && status == 0; ++s) {
    orc_wrap(p, n, pos, type);
    mark_excluded(p, n, pos, type);
    mdbc_before_pi(p, n, pos, vel, rho, type, normal, vel_pi);
    orc_interact(p, n, pos, vel_pi, rho, type, n, NULL, ace, arho, visc, nbr);
    uint64_t count = 0;
    for (int64_t a = 0; a < n; ++a) count += nbr[a];
    const double dt = orc_time_step(p, n, type, ace, visc);
    if (dt_hist) dt_hist[s] = dt;
    if (!(dt > 0.0) || !isfinite(dt)) { status = 2; break; }
    orc_predictor(p, n, dt, *t, pos, vel, rho, type, ace, arho, pos_n, vel_n, rho_n);
    for (int32_t k = 0; k < n_bodies; ++k)
      if (orc_body_step(p, n, 0, dt, &bodies[k], &bodies_n[k], pos_n, pos, vel, type, ace,
                        NULL, NULL))
        status = 3;
    orc_wrap(p, n, pos, type);
    mark_excluded(p, n, pos, type);
    mdbc_before_pi(p, n, pos, vel, rho, type, normal, vel_pi);
    orc_interact(p, n, pos, vel_pi, rho, type, n, NULL, ace, arho, visc, nbr);
    for (int64_t a = 0; a < n; ++a) count += nbr[a];
    /* shifting (Section 2.8): computed on the state of the corrector's PI,
     * added to the corrected positions */
    if (p->shift_coef > 0.0) orc_shift(p, n, pos, vel_pi, rho, type, dt, NULL, NULL, shift);
    orc_corrector(p, n, dt, *t, pos, vel, rho, type, ace, arho, pos_n, vel_n, rho_n);
    if (p->shift_coef > 0.0)
      for (int64_t a = 0; a < n; ++a)
        for (int k = 0; k < dim; ++k) pos[k * n + a] += shift[k * n + a];
    for (int32_t k = 0; k < n_bodies; ++k)
      if (orc_body_step(p, n, 1, dt, &bodies[k], &bodies_n[k], pos_n, pos, vel, type, ace,
                        NULL, NULL))
        status = 3;
    *t += dt;
    if (interactions) *interactions += count;
    for (int64_t a = 0; a < n; ++a)
      if (!is_excluded(type[a]) && !(rho[a] > 0.0 && isfinite(rho[a]))) status = 1;
  }
  free(ace); free(arho); free(visc); free(nbr);
  free(pos_n); free(vel_n); free(rho_n); free(vel_pi); free(bodies_n); free(shift);
  return status;
}

/* nsteps Verlet steps (Section 2.5.1), each: PI at n -> dt (Eq. 35) -> the
 * update of Eq. 30, or of Eq. 31 on the first step and on every step whose
 * index is a multiple of ns -> t += dt.  Same outputs and status as orc_run. */
int32_t orc_run_verlet(const orc_params* p, int64_t n, double* pos, double* vel,
                       double* rho, uint8_t* type, const double* normal, int32_t nsteps,
                       int32_t ns, double* t, double* dt_hist, uint64_t* interactions) {
  const int dim = p->dim;
  size_t nd = (size_t)dim * (size_t)(n > 0 ? n : 1);
  double* ace = (double*)calloc(nd, sizeof(double));
  double* arho = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double* visc = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  uint32_t* nbr = (uint32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
  double* vel_p = (double*)calloc(nd, sizeof(double));
  double* rho_p = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double* vel_pi = (double*)calloc(nd, sizeof(double));
  int32_t status = 0;
  for (int32_t s = 0; s < nsteps && status == 0; ++s) {
    orc_wrap(p, n, pos, type);
    mark_excluded(p, n, pos, type);
    mdbc_before_pi(p, n, pos, vel, rho, type, normal, vel_pi);
    orc_interact(p, n, pos, vel_pi, rho, type, n, NULL, ace, arho, visc, nbr);
    uint64_t count = 0;
    for (int64_t a = 0; a < n; ++a) count += nbr[a];
    const double dt = orc_time_step(p, n, type, ace, visc);
    if (dt_hist) dt_hist[s] = dt;
    if (!(dt > 0.0) || !isfinite(dt)) { status = 2; break; }
    const int32_t mode = (ns > 0 && s % ns == 0) ? 1 : 0;
    orc_verlet(p, n, dt, *t, mode, pos, vel, rho, vel_p, rho_p, type, ace, arho);
    *t += dt;
    if (interactions) *interactions += count;
    for (int64_t a = 0; a < n; ++a)
      if (!is_excluded(type[a]) && !(rho[a] > 0.0 && isfinite(rho[a]))) status = 1;
  }
  free(ace); free(arho); free(visc); free(nbr);
  free(vel_p); free(rho_p); free(vel_pi);
  return status;
}
