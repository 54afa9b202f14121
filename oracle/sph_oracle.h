/*
 * CPU oracle for the WCSPH particle-interaction step (test infrastructure).
 *
 * A plain, slow, FP64 implementation of what the GPU path computes, written
 * from Section 2 of the DualSPHysics v5.0 paper (arXiv 2104.00537):
 * Wendland C2 kernel (Eq. 11), continuity with density diffusion (Eq. 15,
 * 17, 18), momentum with artificial viscosity (Eq. 21, 22), Tait equation of
 * state (Eq. 28), symplectic position-Verlet update (Eq. 33, 34), variable
 * time step (Eq. 35), dynamic boundary particles (Eq. 36, 37), and the
 * cell-linked list of Section 5.1 (cell keys, stable sort, cell ranges),
 * and the variants: cubic spline (Eq. 10), laminar viscosity (Eq. 23),
 * Fourtakas diffusion (Eq. 19-20), Verlet (Eq. 30-31), modified DBC
 * (Eq. 38-39) and rigid floating bodies (Eq. 47-50).
 *
 * Neighbours are found by brute force over all particle pairs.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark use this
 * library; the product path never links or calls it.
 *
 * Conventions shared with the inputs (not with any GPU code):
 *  - arrays are component-major: component k of particle i is x[k*n + i];
 *    2-D cases store (x, z), the vertical axis last;
 *  - particle type: 0 fluid, 1 fixed wall, 2 moving wall, 3 floating; bit
 *    0x80 marks a particle excluded from the domain (outside the cell grid);
 *  - the key of a particle outside the grid is ncell_total.
 */
#ifndef SPH_ORACLE_H
#define SPH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_params {
  int32_t dim;             /* 2 or 3 */
  int32_t ddt;             /* 0: no density diffusion, 1: Eq. 18 */
  int32_t ncell[3];        /* cells per axis; ncell[2] = 1 in 2-D */
  int32_t x_sub;           /* key cells per cell along x (cells of
                              1/(inv_cell_size*x_sub) along x) */
  double origin[3];        /* grid origin */
  double inv_cell_size;    /* 1 / cell size, as the case defines it */
  double h, rho0, gamma, c0, alpha, delta, eta2, cfl;
  double mass_fluid, mass_bound;
  double gravity[3];
  double motion_amp, motion_omega;  /* moving walls: x += (A/w^2)(1 - cos wt) */
  int32_t kernel;          /* 0: Wendland C2 (Eq. 11), 1: cubic spline (Eq. 10) */
  int32_t viscosity;       /* 0: artificial (Eq. 21), 1: laminar (Eq. 23) */
  double visc_nu;          /* kinematic viscosity of the laminar term */
  int32_t boundary;        /* 0: DBC (Eq. 36); 1: modified DBC (Eq. 38-39) */
  int32_t pad2;
  double period[3];        /* > 0: the domain is periodic along that component
                              with this length, starting at origin (Section
                              2.7); 0: open */
  double shift_coef;       /* A_s of Eq. 41 (> 0: particle shifting on, 2.8) */
  double shift_fs;         /* > 0: particles with C < shift_fs keep only the
                              tangential part of their shift (Eq. 54, a_n = 0) */
} orc_params;

/* A rigid floating body (Section 3.2): particles [first, first + count) of
 * the arrays, all of type 3.  2-D: omega[0] is the angular velocity in the
 * plane (positive turns the first axis towards the second). */
typedef struct orc_body {
  int64_t first, count;
  double mass;             /* M, the body's total mass */
  double center[3];        /* R0, its centre of mass */
  double vel[3];           /* V, the velocity of R0 */
  double omega[3];         /* Omega, the angular velocity */
} orc_body;

double orc_wendland_w(double r, double h, int32_t dim);
double orc_wendland_fab(double r, double h, int32_t dim);
double orc_cubic_w(double r, double h, int32_t dim);
double orc_cubic_fab(double r, double h, int32_t dim);
double orc_pressure(const orc_params* p, double rho);

uint32_t orc_cell_key(const orc_params* p, const double* pos, int64_t n, int64_t i);
void orc_cell_keys(const orc_params* p, int64_t n, const double* pos, uint32_t* key);
void orc_wrap(const orc_params* p, int64_t n, double* pos, const uint8_t* type);
void orc_sort_perm(int64_t n, const uint32_t* key, uint32_t* perm);
void orc_cell_start(int64_t n, const uint32_t* sorted_key, int64_t ncell_total,
                    uint32_t* start);

void orc_interact(const orc_params* p, int64_t n, const double* pos,
                  const double* vel, const double* rho, const uint8_t* type,
                  int64_t ntarget, const int64_t* target, double* ace,
                  double* arho, double* visc, uint32_t* nbr);
double orc_time_step(const orc_params* p, int64_t n, const uint8_t* type,
                     const double* ace, const double* visc);
void orc_predictor(const orc_params* p, int64_t n, double dt, double t,
                   double* pos, double* vel, double* rho, const uint8_t* type,
                   const double* ace, const double* arho, double* pos_n,
                   double* vel_n, double* rho_n);
void orc_corrector(const orc_params* p, int64_t n, double dt, double t,
                   double* pos, double* vel, double* rho, const uint8_t* type,
                   const double* ace, const double* arho, const double* pos_n,
                   const double* vel_n, const double* rho_n);
int32_t orc_run(const orc_params* p, int64_t n, double* pos, double* vel,
                double* rho, uint8_t* type, const double* normal, int32_t nsteps, double* t,
                double* dt_hist, uint64_t* interactions, orc_body* bodies, int32_t n_bodies);
void orc_body_forces(const orc_params* p, int64_t n, const double* pos, const double* ace,
                     const orc_body* b, double* force, double* torque, double* inertia);
int32_t orc_body_step(const orc_params* p, int64_t n, int32_t phase, double dt, orc_body* b,
                      orc_body* b_n, const double* pos_n, double* pos, double* vel,
                      const uint8_t* type, const double* ace, double* force, double* torque);

void orc_verlet(const orc_params* p, int64_t n, double dt, double t, int32_t mode,
                double* pos, double* vel, double* rho, double* vel_p, double* rho_p,
                const uint8_t* type, const double* ace, const double* arho);
void orc_shift(const orc_params* p, int64_t n, const double* pos, const double* vel,
               const double* rho, const uint8_t* type, double dt, double* conc, double* grad,
               double* dr);
void orc_mdbc(const orc_params* p, int64_t n, const double* pos, const double* vel,
              const double* rho, const uint8_t* type, const double* normal,
              double* rho_out, double* vel_out);
int32_t orc_run_verlet(const orc_params* p, int64_t n, double* pos, double* vel,
                       double* rho, uint8_t* type, const double* normal, int32_t nsteps,
                       int32_t ns, double* t, double* dt_hist, uint64_t* interactions);

#ifdef __cplusplus
}
#endif
#endif
