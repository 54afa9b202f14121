/*
 * sph.h -- C ABI of the MI355X (gfx950) WCSPH particle-interaction hot path.
 *
 * One simulation step of a weakly compressible SPH solver is split, as in
 * Section 5.1 of the DualSPHysics v5.0 paper (arXiv 2104.00537), into a
 * neighbour list (NL), a particle interaction (PI) and a system update (SU):
 *
 *   sph_bin_cells        NL: cell keys, stable radix sort, cell ranges, and the
 *                        particle arrays reordered into sorted SoA (plus the
 *                        per-particle data the interaction reads).
 *   sph_interact         PI: continuity and momentum sums over the neighbours
 *                        within 2h (Eq. 11, 15, 17-18, 21-22, 28, 36), plus the
 *                        per-particle maxima that set the time step.
 *   sph_reduce_dt        SU: the variable time step of Eq. 35, kept on the GPU.
 *   sph_verlet_step      SU: the Verlet scheme (Eq. 30-31), one PI per step.
 *   sph_mdbc             wall densities and velocities of the modified
 *                        dynamic boundary condition (Eq. 38-39), before a PI.
 *   sph_symplectic_step  SU: symplectic predictor / corrector (Eq. 33-34), with
 *                        imposed motion of moving walls (Eq. 37).
 *   sph_floating_step    SU of rigid floating bodies (Section 3.2, Eq. 47-50),
 *                        after each phase of sph_symplectic_step.
 *   sph_shifting         particle shifting (Section 2.8, Eq. 40-41, 53) after
 *                        the corrector.
 *   sph_refresh_view     the interaction's view of the half state on the cells
 *                        of the last binning (the n+1/2 PI without a second NL).
 *   sph_build_list,      per-target neighbour lists with a skin, built once per
 *   sph_interact_list    NL and replayed by both PIs of a step (opt-in).
 *   sph_interact_noalloc sph_interact for callers that cannot allocate.
 *   sph_batch_*          the same steps over many independent cases at once
 *                        (continuous batching).
 *
 * A full step is: bin, interact, reduce_dt, predictor, bin (carrying the saved
 * state along), interact, corrector; or, with one NL per step: bin, interact,
 * reduce_dt, predictor, refresh_view, interact (SPH_INTERACT_REUSE_CELLS),
 * corrector.
 *
 * Conventions
 *  - Every array argument is a DEVICE pointer to memory the caller owns (the
 *    library allocates nothing and keeps no pointer after a call returns).
 *  - Arrays are structure-of-arrays and component-major: component k of
 *    particle i is x[k*n + i].  Positions are FP64, velocity and density FP32.
 *    2-D cases store (x, z) -- the vertical axis is always the last component.
 *  - Particle type (uint8): 0 fluid, 1 fixed wall, 2 moving wall, 3 floating
 *    (a particle of a rigid body, see sph_body); bit 0x80 is set by
 *    sph_bin_cells on particles outside the cell grid, which then take no
 *    part in the interaction or the update ("excluded").
 *  - All work is enqueued asynchronously on `stream` (a hipStream_t; NULL means
 *    the default stream).  Calls on distinct workspaces are independent.
 *  - Every call returns an sph_status synchronously for argument and launch
 *    errors.  Data-dependent failures (a non-finite or non-positive density,
 *    a particle leaving the grid, dt below dt_floor) set bits of a device
 *    error word in the workspace, read with sph_read_error after the stream
 *    has finished.  No call aborts the process or throws.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sph_status {
  SPH_OK = 0,
  SPH_E_ARG = -1,        /* a bad argument: null pointer, size, parameter */
  SPH_E_WORKSPACE = -2,  /* workspace smaller than sph_workspace_bytes() */
  SPH_E_HIP = -3         /* a HIP launch or runtime error */
} sph_status;

enum {
  SPH_FLUID = 0,
  SPH_BOUND_FIXED = 1,
  SPH_BOUND_MOVING = 2,
  SPH_FLOATING = 3,
  SPH_EXCLUDED = 0x80
};

/* bits of the device error word */
enum {
  SPH_ERR_NONFINITE = 1u,   /* non-finite velocity, or density not in (0, inf) */
  SPH_ERR_EXCLUDED = 2u,    /* a particle left the cell grid and was excluded */
  SPH_ERR_DT_FLOOR = 4u,    /* dt fell below dt_floor, or is not finite */
  SPH_ERR_FLOATING = 8u,    /* sph_floating_step: a floating particle whose id is
                               in no body's range, a body whose particles are
                               not all present, body counts summing above n,
                               or a singular inertia */
  SPH_ERR_MARGIN = 16u,     /* an interaction or shifting with
                               SPH_INTERACT_REUSE_CELLS after particles moved
                               half a cell or more since the binning, or one
                               without that flag after particles moved at all
                               since the binning (a predictor ran): neighbours
                               may have been missed */
  SPH_ERR_LIST = 32u        /* sph_interact_list with a list built on another
                               binning or with another list_bytes: the pass
                               walked the cells instead (the results are
                               right, the list was not used) */
};

/* flags of sph_interact */
enum {
  /* nbr_count uses an FP64 distance test on the FP64 positions (bit-exact
   * neighbour counts); the sums always use the FP32 cell-relative test. */
  SPH_DIAG_COUNT_F64 = 1u,
  /* Precision-study arms (Section 5.1), not the production path and several
   * times slower; at most one flag may be given.  F64: every pair in FP64
   * from the FP64 positions, pressure recomputed in FP64 from the density.
   * ABS_F32: distances from positions rounded to FP32 as absolute
   * coordinates, the rest FP32 (the scheme that cell-relative positions
   * replace).  Velocities and densities are the stored FP32 values in both;
   * the outputs and the workspace partials are as in the production pass.
   * The arms take the default formulation only (Wendland kernel, artificial
   * viscosity, ddt 0 or 1, no floating bodies, no periodic components);
   * other options are rejected with SPH_E_ARG. */
  SPH_INTERACT_F64 = 2u,
  SPH_INTERACT_ABS_F32 = 4u,
  /* The cells of the last sph_bin_cells are reused for a state whose
   * particles have moved since (the second interaction of a symplectic
   * step, after sph_refresh_view): the search reaches one cell further and
   * widens its cut by the largest distance a particle moved since the
   * binning, which sph_symplectic_step's predictor and sph_floating_step's
   * predictor phase record in the workspace.  The same pairs within 2h are
   * found as after a new binning (only the summation order differs).  Sets
   * SPH_ERR_MARGIN if a particle moved half a cell or more.  Combines with
   * SPH_DIAG_COUNT_F64; not with the precision-study arms or modified DBC;
   * a periodic component must then span at least 2 (cell_div + 1) + 1 cells
   * (else SPH_E_ARG), so that the longer walk meets no cell twice. */
  SPH_INTERACT_REUSE_CELLS = 8u,
  /* One lane per target particle.  By default a case too small to fill the
   * GPU (at most 131,072 particles) with the default formulation (Wendland
   * kernel, artificial viscosity, ddt 0 or 1, no floating bodies or periodic
   * components) deals each target's neighbour rows to four lanes and sums
   * their results, which shortens each lane's chain of dependent loads;
   * results agree up to the order of the FP32 sums (FP64 counts are
   * identical).  Combines with every other flag. */
  SPH_INTERACT_ONE_LANE = 16u,
  /* The all-FP64 arm of the precision study (Section 5.1): as
   * SPH_INTERACT_F64, but velocities and densities come from the state's
   * FP64 copies (s->vel64, s->rho64, required) instead of the stored FP32
   * values, and the rates are written in FP64: `ace` and `arho` then point to
   * double arrays ([dim][n] and [n]) that sph_symplectic_step reads for an
   * all-FP64 state.  visc stays FP32.  Same restrictions as SPH_INTERACT_F64;
   * not with SPH_INTERACT_REUSE_CELLS. */
  SPH_INTERACT_F64_STATE = 32u
};

/* Case constants, passed by pointer to host memory and copied by value into
 * the launches. */
typedef struct sph_params {
  int32_t dim;            /* 2 or 3 */
  int32_t cell_div;       /* 1: cells of size 2h, search +-1 cell (Section 5.1);
                             2: cells of size h, search +-2 cells (Section 5.3) */
  int32_t ddt;            /* density diffusion: 0 none; 1 Eq. 17 with Eq. 18
                             (Molteni-Colagrossi); 2 Eq. 17 with Eq. 19-20
                             (Fourtakas et al., hydrostatic part removed) */
  int32_t ncell[3];       /* key cells per axis; ncell[2] = 1 in 2-D.  Keys are
                             cx + ncell[0]*(cy + ncell[1]*cz) (x fastest); the
                             key of a particle outside the grid is the total
                             cell count.  total + 1 must be < 2^32. */
  int32_t x_sub;          /* 1, 2, 4 or 8: key cells per cell along x (cells
                             of cs/x_sub along x, cs along y and z); finer x
                             cells let the interaction cut each row of
                             neighbour cells closer to the support sphere */
  int32_t boundary;       /* 0: dynamic boundary condition, walls evolve their
                             density by Eq. 36; 1: modified DBC (Eq. 38-39,
                             sph_mdbc before every sph_interact; the state
                             then needs the wall ghost vectors, `normal`) */
  double origin[3];       /* grid origin (components beyond dim ignored) */
  double cell_size;       /* cs = 2h / cell_div */
  double inv_cell_size;   /* 1/cs, computed once by the caller; the cell index
                             is floor((x - origin) * inv_cell_size) in FP64
                             along y and z, and floor((x - origin) *
                             (inv_cell_size * x_sub)) along x */
  double h;               /* smoothing length; support radius 2h */
  double rho0;            /* reference density (Eq. 28) */
  double gamma;           /* polytropic index (Eq. 28) */
  double c0;              /* numerical speed of sound (Section 2.4) */
  double alpha;           /* artificial viscosity coefficient (Eq. 21) */
  double delta;           /* density diffusion coefficient (Eq. 17) */
  double eta2;            /* eta^2 > 0 in the denominators of Eq. 21 and 35 */
  double cfl;             /* Courant number C_CFL (Eq. 35) */
  double mass_fluid;      /* particle masses of fluid / wall particles */
  double mass_bound;
  double gravity[3];      /* body force f of Eq. 13 */
  double motion_amp;      /* moving walls: x(t) = x0 + (A/w^2)(1 - cos wt),   */
  double motion_omega;    /*   A = motion_amp, w = motion_omega (0: no motion) */
  double dt_floor;        /* smallest acceptable dt (error bit below it) */
  int32_t kernel;         /* 0: Wendland C2 (Eq. 11); 1: cubic spline (Eq. 10) */
  int32_t viscosity;      /* 0: artificial viscosity (Eq. 21); 1: laminar
                             viscosity (Eq. 23) with kinematic viscosity
                             visc_nu, in place of Pi_ab (Eq. 35 unchanged) */
  double visc_nu;         /* kinematic viscosity of the laminar term (>= 0) */
  int32_t floating;       /* 1: the state holds floating particles (type 3);
                             sph_interact then gives them the momentum sum of
                             Eq. 47.  Needs boundary 0; with 0, particles of
                             type 3 take the fixed-wall path. */
  int32_t pad0;
  double period[3];       /* periodic boundaries (Section 2.7): period[k] > 0
                             makes component k periodic with this length; the
                             grid along k must start at the periodic boundary
                             (origin[k]) and span exactly the period: period
                             = cells * cell_size within 1e-9 relative, cells
                             = ncell[k] (ncell[0] / x_sub along x, which must
                             divide), and at least 2 cell_div + 1 cells.
                             Particles leaving [origin, origin + period) along
                             k re-enter at the other end (sph_bin_cells wraps
                             the positions it writes) and pairs take the
                             nearest image.  0: open.  Needs boundary 0 and
                             no floating bodies. */
  double shift_coef;      /* A_s of Eq. 41 (>= 0; see sph_shifting) */
  double shift_fs;        /* >= 0: fluid particles whose concentration C is
                             below it (a support truncated by the free
                             surface) keep only the tangential part of their
                             shift (Eq. 54 with a_n = 0); 0: none */
} sph_params;

/* Particle state (SoA device arrays of n particles). */
typedef struct sph_state {
  double* pos;      /* [dim][n] FP64 positions */
  float* vel;       /* [dim][n] velocities */
  float* rho;       /* [n] densities */
  uint8_t* type;    /* [n] particle type, see SPH_FLUID ... */
  uint32_t* id;     /* [n] particle identity, carried through the sort
                       (nullable: then not carried) */
  float* normal;    /* [dim][n] for wall particles the vector to the ghost
                       node (mirror image across the wall face), 0 for
                       fluid; carried through the sort (nullable; needed by
                       sph_mdbc) */
  double* vel64;    /* [dim][n] and [n], nullable as a pair: an all-FP64     */
  double* rho64;    /* state (the precision study's reference arm).  When
                       set they are the velocities and densities, carried
                       through the sort (in and out, and the carried pair,
                       when both sides have them), advanced in FP64 by
                       sph_symplectic_step, which also writes their FP32
                       roundings to vel and rho; read by sph_interact with
                       SPH_INTERACT_F64_STATE.  Not with sph_verlet_step,
                       sph_refresh_view, floating bodies or the batch calls. */
} sph_state;

/* Bytes of workspace the calls need for a case of n particles. */
size_t sph_workspace_bytes(const sph_params* p, int64_t n);

/* NL (Section 5.1).  For every particle of `in`: the cell key (see
 * sph_params.ncell), a stable ascending sort of the keys (ties keep input
 * order), the index of the first sorted particle of every cell, and the state
 * gathered into sorted order.
 *   key[n]            out: sorted keys (particles outside the grid, or already
 *                     excluded, get the key C = total cells and sort last)
 *   perm[n]           out: perm[j] = input index of the j-th sorted particle
 *   cell_start[C+1]   out: C = total cells; cell c holds sorted particles
 *                     [cell_start[c], cell_start[c+1]); cell_start[C] is the
 *                     number of particles inside the grid
 *   out               out: `in` gathered by perm (pos, vel, rho, type, id);
 *                     newly excluded particles get the 0x80 type bit; along
 *                     periodic components positions are first brought back
 *                     into [origin, origin + period): x - period if beyond,
 *                     x + period if below (origin if that rounds to the end)
 *   carry_in/out      nullable pair: a second state (pos, vel, rho only)
 *                     gathered by the same perm -- the saved state n during
 *                     the corrector's NL.
 * `in` and `out` must not alias. */
sph_status sph_bin_cells(const sph_params* p, int64_t n, const sph_state* in,
                         sph_state* out, const sph_state* carry_in,
                         sph_state* carry_out, uint32_t* key, uint32_t* perm,
                         uint32_t* cell_start, void* ws, size_t ws_bytes,
                         void* stream);

/* PI (Section 2.3, Eq. 11, 15, 17-18, 21-22, 28, 36) on a state that
 * sph_bin_cells sorted (s, key, cell_start from the same call; the call also
 * left in the workspace the per-particle data this pass reads -- cell-relative
 * FP32 positions, velocities, densities and Tait pressures -- so nothing may
 * change the state in between, and the workspace must be the same).  For every
 * non-excluded particle a, over neighbours b != a with |r_ab| < 2h:
 *   fluid a:  ace[a]  = g - sum_b m_b [(P_a+P_b)/(rho_a rho_b) + Pi_ab] grad_a W_ab
 *             arho[a] = rho_a sum_b (m_b/rho_b) v_ab.grad_a W_ab + D_a
 *             with D_a = 2 delta h c0 sum_{b fluid} (rho_b - rho_a)|F_ab| m_b/rho_b
 *             (the diffusive reading of Eq. 18) and P from Eq. 28;
 *   wall a:   arho[a] = rho_a sum_{b fluid} (m_b/rho_b) v_ab.grad_a W_ab, ace = 0;
 *   floating a (p->floating = 1): arho as a wall, and (Eq. 47)
 *             ace[a] = - sum_{b fluid} m_b [(P_a+P_b)/(rho_a rho_b) + Pi_ab] grad_a W_ab
 *             (no gravity; visc[a] = 0).
 *   ace[dim][n], arho[n]   out (FP32, sorted order; excluded particles get 0)
 *   visc[n]                out, nullable: max_b |h v_ab.r_ab|/(r_ab^2+eta^2)
 *   nbr_count[n]           out, nullable: pairs evaluated for a (all neighbours
 *                          of a fluid target, fluid neighbours of a wall)
 * Along periodic components (p->period) pairs take the nearest image.
 * Arithmetic is FP32 on cell-relative FP32 positions (Section 5.1, precision
 * paragraph).  Per-block maxima of |ace| and visc over fluid targets and the
 * interaction count go to the workspace for sph_reduce_dt.  n must be below
 * 2^28 and the grid below 2^30 cells (the walk addresses the view and the
 * cell ranges with 32-bit byte offsets), else SPH_E_ARG. */
sph_status sph_interact(const sph_params* p, int64_t n, const sph_state* s,
                        const uint32_t* key, const uint32_t* cell_start,
                        float* ace, float* arho, float* visc,
                        uint32_t* nbr_count, uint32_t flags, void* ws,
                        size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory: code recorded into a HIP
 * graph under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc.  sph_interact without a workspace: the regions the pass needs
 * besides its inputs and outputs (the interaction view, built here from s;
 * the per-block partial results; an error word) live in one device array of
 * the library, 68 MB (for SPH_NOALLOC_MAX_N particles), which each GPU the
 * library runs on holds until the process ends.
 *   s, key, cell_start   as sph_bin_cells left them (s sorted; positions,
 *                        velocities, densities and types not changed since)
 *   ace, arho, visc, nbr_count, flags   as sph_interact (the same kernels:
 *                        the same results), except SPH_INTERACT_REUSE_CELLS
 * n must be at most SPH_NOALLOC_MAX_N and p->boundary 0 (modified DBC takes
 * its wall entries from sph_mdbc), else SPH_E_ARG.  Nothing is allocated:
 * the array's device address is looked up on the first call on each device
 * (the current device, to which `stream` must belong); do one call before a
 * capture.  The array keeps the last call's contents and each call clears
 * what must start at zero; its partial results and error word cannot be read
 * (sph_reduce_dt does not apply).  Calls that overlap on one GPU (other
 * streams or threads) race on the array: serialise them. */
#define SPH_NOALLOC_MAX_N 2097152
sph_status sph_interact_noalloc(const sph_params* p, int64_t n, const sph_state* s,
                                const uint32_t* key, const uint32_t* cell_start, float* ace,
                                float* arho, float* visc, uint32_t* nbr_count, uint32_t flags,
                                void* stream);

/* Neighbour lists (Section 2.3 sums, Section 5.1 NL): per target particle,
 * the candidates of its cells that lie within the list radius 2h (1 + 1e-4)
 * + skin of it, found by one walk of the cells after sph_bin_cells
 * (sph_build_list) and replayed by both interactions of a symplectic step
 * (sph_interact_list): the pass at state n on the binning's view, and the
 * pass at n+1/2 after sph_refresh_view.  A pair within 2h at n+1/2 was
 * within 2h + 2 delta at the binning (delta the largest displacement since,
 * which the predictor records), so while 2 delta stays within the skin the
 * list holds every pair.  The replay gives the pairs, sums and counts of
 * sph_interact on the same view bit for bit (same FP32 test and pair terms,
 * same order); it only runs the wavefront's lanes through their own lists
 * instead of through common cell steps.  Default formulation only (Wendland
 * kernel, artificial viscosity, ddt 0 or 1, DBC walls, no floating bodies or
 * periodic components), FP32 state (no vel64/rho64) and n below 2^28; else
 * SPH_E_ARG.
 *
 * The list is a caller-owned DEVICE buffer of sph_list_bytes(p, n) bytes (or
 * less: a smaller buffer holds fewer chunks per target, and targets whose
 * chunks do not fit walk their cells in both passes). */
size_t sph_list_bytes(const sph_params* p, int64_t n);

/* flags of sph_build_list */
enum {
  /* skin = max(skin argument, the skin that the last sph_interact_list with
   * SPH_INTERACT_REUSE_CELLS on this workspace asked for: 1.5 times twice the
   * displacement it saw), at most half a cell */
  SPH_LIST_ADAPTIVE_SKIN = 1u
};

/* Builds the list of the state that the last sph_bin_cells on this workspace
 * sorted (its view, key and cell_start), with the given skin (metres, >= 0;
 * see SPH_LIST_ADAPTIVE_SKIN).  Records the binning it belongs to. */
sph_status sph_build_list(const sph_params* p, int64_t n, const sph_state* s,
                          const uint32_t* key, const uint32_t* cell_start, double skin,
                          uint32_t flags, void* list, size_t list_bytes, void* ws,
                          size_t ws_bytes, void* stream);

/* sph_interact over a list from sph_build_list (same list_bytes): outputs
 * and workspace partials as sph_interact's.  flags: SPH_DIAG_COUNT_F64,
 * SPH_INTERACT_REUSE_CELLS (the pass after sph_refresh_view: if twice the
 * displacement exceeds the list's skin, every target walks its cells as
 * sph_interact with that flag does -- same results -- and the workspace
 * counts the fallback), SPH_INTERACT_ONE_LANE (no effect: one lane per
 * target).  A list built on another binning, or with another list_bytes,
 * is not used (the pass walks the cells) and sets SPH_ERR_LIST. */
sph_status sph_interact_list(const sph_params* p, int64_t n, const sph_state* s,
                             const uint32_t* key, const uint32_t* cell_start, const void* list,
                             size_t list_bytes, float* ace, float* arho, float* visc,
                             uint32_t* nbr_count, uint32_t flags, void* ws, size_t ws_bytes,
                             void* stream);

/* The number of sph_interact_list passes with SPH_INTERACT_REUSE_CELLS on this
 * workspace that walked the cells because the displacement exceeded the
 * skin (or whose list was stale).  Synchronises the device.  Negative
 * sph_status on failure. */
int64_t sph_list_walks(const void* ws);

/* Rewrites the interaction view that sph_bin_cells left in the workspace
 * from the state's current positions, velocities and densities, keeping the
 * sorted order and the cells of that binning (key, cell_start unchanged),
 * for an interaction with SPH_INTERACT_REUSE_CELLS: the second interaction
 * of a symplectic step, whose particles moved by dt/2 v since the binning,
 * without sorting again.  Positions are not wrapped along periodic
 * components (they stay relative to their binned cells; the next
 * sph_bin_cells wraps them).  A particle now outside the grid along an open
 * component is excluded as sph_bin_cells would exclude it (type bit,
 * SPH_ERR_EXCLUDED); it stays in its slot but meets no target. */
sph_status sph_refresh_view(const sph_params* p, int64_t n, sph_state* s, const uint32_t* key,
                            void* ws, size_t ws_bytes, void* stream);

/* SU, Eq. 35: dt = cfl * min(sqrt(h / max_a |f_a|), h / (c0 + max_a visc_a))
 * over fluid particles, reduced from the last sph_interact on this workspace.
 *   dt[1]            out: FP64, device
 *   interactions[2]  in/out, nullable: the pass's pair count is ADDED to [0],
 *                    the part of it with a wall target (continuity only) to [1]
 *   maxima[2]        out, nullable: {max |f_a|, max visc_a} (FP32)
 * Sets SPH_ERR_DT_FLOOR if dt < dt_floor or dt is not finite. */
sph_status sph_reduce_dt(const sph_params* p, int64_t n, double* dt,
                         uint64_t* interactions, float* maxima, void* ws,
                         size_t ws_bytes, void* stream);

/* SU, Eq. 33-34, symplectic position Verlet, on the sorted state.
 *   phase 0 (predictor): saves s into `saved` (pos, vel, rho), then for fluid
 *     r += dt/2 v, v += dt/2 ace, and for all rho += dt/2 arho;
 *   phase 1 (corrector): with ace, arho evaluated at n+1/2 and `saved` holding
 *     state n (in the current sorted order): fluid v = v_n + dt ace,
 *     r = r_n + dt (v + v_n)/2; all: eps = -(arho/rho) dt,
 *     rho = rho_n (2 - eps)/(2 + eps); then *t += dt.
 *   Moving walls take x = x_n + D(t') - D(t), v_x = (A/w) sin(w t') at
 *   t' = t + dt/2 (predictor) or t + dt (corrector), D(t) = (A/w^2)(1-cos wt).
 *   dt, t: device FP64 scalars (t is read by both phases, advanced by phase 1).
 * Position arithmetic is FP64; velocity and density are stored in FP32.  An
 * all-FP64 state (s->vel64 and s->rho64 set; then `saved` needs them too)
 * is advanced in FP64 from FP64 rates: ace and arho are then double arrays
 * (those of sph_interact with SPH_INTERACT_F64_STATE). */
sph_status sph_symplectic_step(const sph_params* p, int64_t n, int32_t phase,
                               const double* dt, double* t, sph_state* saved,
                               sph_state* s, const float* ace,
                               const float* arho, void* ws, size_t ws_bytes,
                               void* stream);

/* SU, Section 2.5.1: the Verlet scheme, one interaction per step, on the
 * sorted state.
 *   mode 0 (Eq. 30): fluid v = v_prev + 2 dt ace; all rho = rho_prev + 2 dt arho;
 *   mode 1 (Eq. 31, the intermediate step, also the first step when no
 *     previous state exists): fluid v += dt ace; all rho += dt arho;
 *   both: fluid r += dt v^n + dt^2/2 ace (v^n the velocity before the call).
 *   prev: velocity and density of step n-1 in the current sorted order (carry
 *     it through sph_bin_cells as the carried state); on return it holds
 *     those of step n.  prev->pos is not used.
 *   Moving walls take x = x + D(t + dt) - D(t) and v_x = (A/w) sin(w (t + dt));
 *   fixed walls keep position and velocity.  Then *t += dt.
 *   The paper recommends mode 1 every ~40 steps (the caller chooses).
 * Sets SPH_ERR_NONFINITE for a non-finite velocity or a density not in
 * (0, inf). */
sph_status sph_verlet_step(const sph_params* p, int64_t n, int32_t mode, const double* dt,
                           double* t, sph_state* prev, sph_state* s, const float* ace,
                           const float* arho, void* ws, size_t ws_bytes, void* stream);

/* Modified dynamic boundary condition (Section 2.6.2, Eq. 38-39), on the
 * sorted state and the view left by sph_bin_cells, before sph_interact:
 * for every wall particle B, the fluid particles within 2h of its ghost node
 * G = r_B + normal_B give (FP64 sums, positions from s->pos, kernel of the
 * case, V_b = m_b/rho_b) the first-order corrected approximation of the
 * density and its gradient at G, i.e. the solution of
 *   [sum V w, sum V w r^T; sum V F r, sum V F r r^T] [rho_G; grad] =
 *   [sum m w; sum m F r]   (r = r_b - r_G, w = W, grad W = F r),
 * and rho_B = rho_G + (r_B - r_G).grad (Eq. 38); with |det| < 1e-3 the
 * Shepard value sum m w / sum V w and no gradient.  The ghost velocity is the
 * Shepard sum of Eq. 39 and the wall takes v_B = 2 v_wall - v_G (no slip
 * about its own velocity).  With no fluid near G: rho0 and v_wall.
 * Writes rho_B to s->rho and rho_B, v_B, P(rho_B) to the interaction view
 * (the state velocity keeps the wall's own motion).  p->boundary must be 1
 * and s->normal set. */
sph_status sph_mdbc(const sph_params* p, int64_t n, sph_state* s, const uint32_t* key,
                    const uint32_t* cell_start, void* ws, size_t ws_bytes, void* stream);

/* Particle shifting (Section 2.8: Eq. 40-41 with the concentration and its
 * gradient of Eq. 53), called right after the corrector (sph_symplectic_step
 * phase 1) on the same state, before the next sph_bin_cells.  It reads the
 * interaction view that the last sph_bin_cells / sph_interact pair left in
 * the workspace (state n+1/2; with modified DBC, its wall densities):
 *   C_a      = sum_b V_b W_ab over every non-excluded b within 2h, b = a
 *              included (V_b = m_b / rho_b, the kernel of the case),
 *   grad C_a = sum_b V_b (C_b - C_a) grad_a W_ab,
 *   dr_a     = -A_s h |v_a| dt grad C_a   (A_s = p->shift_coef, |v_a| at
 *              n+1/2, dt the step's),
 * for every fluid particle a; if p->shift_fs > 0 and C_a < shift_fs, the
 * component of dr_a along grad C_a is removed (Eq. 54 with a_n = 0).  dr_a
 * is added to s->pos (the corrected positions, FP64).  Along periodic
 * components distances take the nearest image.
 *   conc[n]       out, nullable: C of every particle (FP32, sorted order;
 *                 0 for excluded particles)
 *   shift[dim][n] out, nullable: the dr applied (FP32; 0 for non-fluid)
 * Arithmetic is FP32 on the view's offsets, as in sph_interact.  Needs
 * p->shift_coef > 0.  Without conc the concentrations live in the
 * workspace's sort buffers during the call.  flags: 0, or
 * SPH_INTERACT_REUSE_CELLS when the view is a refreshed one on the cells of
 * an earlier binning (after sph_refresh_view and an interaction with that
 * flag): the search then reaches one cell further and widens its cut by the
 * recorded displacement, as in sph_interact (SPH_ERR_MARGIN past half a
 * cell; not with modified DBC).  Other bits: SPH_E_ARG. */
sph_status sph_shifting(const sph_params* p, int64_t n, sph_state* s, const uint32_t* key,
                        const uint32_t* cell_start, const double* dt, float* conc,
                        float* shift, uint32_t flags, void* ws, size_t ws_bytes, void* stream);

/* Floating bodies (Section 3.2).  A body is a rigid object whose particles
 * are the particles of type SPH_FLOATING with id in [id_first, id_first +
 * count) (sph_state.id is required).  In every SPH sum its particles are
 * boundary particles of mass mass_bound (Eq. 36 gives their density); each
 * gets from sph_interact the momentum sum of a fluid particle over its fluid
 * neighbours only, without gravity (Eq. 47), so that m_B dv_k/dt is exactly
 * the reaction of the fluid to it.  The body moves as one rigid object
 * (Eq. 48-50): its own mass M sets its inertia, gravity acts on it as a
 * whole, and contact with walls or other bodies is not modelled.
 * The table is an array of sph_body in DEVICE memory owned by the caller;
 * sph_floating_step reads and advances it.  FP64 throughout; 2-D cases use
 * components (x, z) in [0], [1] and the rotation in the plane is the scalar
 * in [0] of omega and torque (positive turns the first axis towards the
 * second). */
#define SPH_MAX_BODIES 64

typedef struct sph_body {
  int64_t id_first;     /* first particle id of the body */
  int64_t count;        /* its particle count (> 0) */
  double mass;          /* M, the total mass of the body (> 0) */
  double center[3];     /* R0, centre of mass */
  double vel[3];        /* V, velocity of R0 */
  double omega[3];      /* Omega, angular velocity */
  double center_n[3];   /* state n, written by the predictor (phase 0) */
  double vel_n[3];
  double omega_n[3];
  double force[3];      /* out: sum_k m_B dv_k/dt, the fluid force (Eq. 48) */
  double torque[3];     /* out: sum_k m_B (r_k - R0) x dv_k/dt (Eq. 49) */
} sph_body;

/* One phase of the rigid-body update of n_bodies floating bodies, called
 * right after sph_symplectic_step of the same phase on the same state (that
 * call saved state n and advanced the floating particles' density as walls'
 * but left their position and velocity).  ace is the interaction's output
 * that the symplectic phase used.  Per body, from its particles in the
 * current (sorted) state:
 *   F = sum_k m_B ace_k, T = sum_k m_B (r_k - R0) x ace_k, and the inertia
 *   tensor about R0, I = sum_k (M/count)(|r'|^2 1 - r' r'^T), r' = r_k - R0;
 *   A = F/M + g, alpha = I^-1 T (Eq. 48-49);
 *   phase 0: saves (R0, V, Omega) as state n, then V += dt/2 A,
 *     Omega += dt/2 alpha, R0 += dt/2 V^n, rotation by dt/2 Omega^n;
 *   phase 1: V = V^n + dt A, Omega = Omega^n + dt alpha,
 *     R0 = R0^n + dt (V + V^n)/2, rotation by dt (Omega + Omega^n)/2;
 *   each particle: r_k = R0 + Rot (r_k^n - R0^n) from saved->pos (state n),
 *     v_k = V + Omega x (r_k - R0) (Eq. 50).
 * Sums are taken in a fixed order (by particle id), so results do not
 * depend on the particle order.  Sets SPH_ERR_FLOATING on the conditions
 * listed with it.  The workspace's sort buffers hold the id map between the
 * kernels of one call.  p->floating must be 1 and p->boundary 0;
 * 1 <= n_bodies <= SPH_MAX_BODIES. */
sph_status sph_floating_step(const sph_params* p, int64_t n, int32_t phase, const double* dt,
                             sph_body* bodies, int32_t n_bodies, const sph_state* saved,
                             sph_state* s, const float* ace, void* ws, size_t ws_bytes,
                             void* stream);

/* ---------------------------------------------------------------- batches --
 * Continuous batching: n_slots independent cases packed into one set of
 * arrays advance together through the calls below, each case ("slot") with
 * its own constants, dt and t.  Slot s owns particles [offsets[s],
 * offsets[s+1]) of the packed arrays and the cell keys [cbase_s, cbase_s +
 * C_s] (C_s = its total cells; the last key is for its particles outside its
 * grid), with cbase_s the sum of C + 1 over the slots before it.  So one
 * radix sort, one set of cell ranges, one interaction launch and one update
 * serve every case, and every slot keeps its particle range through every
 * sort; results of a case do not depend on the other cases in the batch.
 * Packed arrays always have three components: a 2-D case (x, z) is stored as
 * (x, 0, z) and gets one cell across y.  All slots share cell_div; at most
 * 2^27 - 1 particles in total.  With one lane per target (no
 * SPH_BATCH_FOUR_LANES, and SPH_INTERACT_ONE_LANE on the single-case side)
 * a slot's results are those of the single-case calls on the same case, bit
 * for bit.
 */
#define SPH_BATCH_MAX_SLOTS 4096

/* sph_batch.flags, set by sph_batch_describe (callers do not change them) */
enum {
  /* every slot's particle range starts and ends at a multiple of 64 (whole
   * wavefronts): the interaction then runs a leaner kernel in which each
   * wavefront lies in one slot.  Pad a case's range with excluded particles
   * (type SPH_EXCLUDED) to get it. */
  SPH_BATCH_WAVE_ALIGNED = 1u,
  /* also an option of sph_batch_describe: in a wave-aligned batch, a slot of
   * at most 131,072 particles gets four lanes per target (as the
   * single-case pass for a small case), the others one.  The choice depends
   * on the option and the slot's own size only, so a case's results do not
   * depend on the other slots.  It shortens each target's chain of loads,
   * which pays when the batch is too small to fill the GPU; when it fills
   * the GPU, one lane per target does the same work in fewer instructions. */
  SPH_BATCH_FOUR_LANES = 2u,
  /* some slot takes a formulation option (kernel 1, viscosity 1 or ddt 2):
   * the interaction then runs the general pair terms, each slot with its own
   * options.  A slot of the default formulation gets the same results there
   * as in the default kernel (the same operations), so a case's results
   * still do not depend on the other slots. */
  SPH_BATCH_GENERAL = 4u,
  /* some slot has periodic components (Section 2.7): the interaction and
   * shifting then take the nearest image along each slot's own periodic
   * components; slots without any see no difference. */
  SPH_BATCH_PERIODIC = 8u
};

typedef struct sph_batch {
  int32_t n_slots;
  int32_t cell_div;
  int64_t n_total;      /* offsets[n_slots] */
  int64_t key_cells;    /* sum over slots of (cells + 1): cell_start has
                           key_cells + 1 entries */
  const void* table;    /* DEVICE copy of the slot table (see below) */
  uint32_t flags;       /* SPH_BATCH_* flags */
  uint32_t lanes;       /* interaction lanes over all slots (set by
                           sph_batch_describe) */
} sph_batch;

/* Bytes of the slot table for n_slots cases. */
size_t sph_batch_table_bytes(int32_t n_slots);

/* Host only (no device call): writes the slot table of the cases params[s]
 * with particle ranges offsets[0..n_slots] (offsets[0] = 0, non-decreasing)
 * to table_host and fills *batch except batch->table.  The caller copies the
 * table to device memory and sets batch->table before the calls below.  The
 * table stays valid while the slots keep their ranges.  Every slot must use
 * the same cell_div, DBC walls (boundary 0) and no floating bodies;
 * otherwise SPH_E_ARG.  Each slot may take its own formulation options
 * (kernel, viscosity, ddt; see SPH_BATCH_GENERAL) and periodic components
 * (see SPH_BATCH_PERIODIC), each of them at least 2 (cell_div + 1) + 1
 * cells long so that the reused-cells pass can serve it (else SPH_E_ARG).
 * options: 0 or SPH_BATCH_FOUR_LANES (else SPH_E_ARG); batch->flags gets
 * SPH_BATCH_WAVE_ALIGNED when every range is whole wavefronts,
 * SPH_BATCH_FOUR_LANES when it was asked for and the batch is wave-aligned,
 * SPH_BATCH_GENERAL when some slot takes a formulation option and
 * SPH_BATCH_PERIODIC when some slot has periodic components. */
sph_status sph_batch_describe(const sph_params* params, const int64_t* offsets, int32_t n_slots,
                              uint32_t options, void* table_host, size_t table_bytes,
                              sph_batch* batch);

/* Bytes of workspace for a batch (the single-case workspace of n_total
 * particles plus per-slot accumulators, motion and error words). */
size_t sph_batch_workspace_bytes(const sph_batch* b);

/* As sph_bin_cells, over all slots (keys offset per slot, see above). */
sph_status sph_batch_bin_cells(const sph_batch* b, const sph_state* in, sph_state* out,
                               const sph_state* carry_in, sph_state* carry_out, uint32_t* key,
                               uint32_t* perm, uint32_t* cell_start, void* ws, size_t ws_bytes,
                               void* stream);

/* As sph_interact, over all slots in one launch (ace is [3][n_total]);
 * per-slot maxima and pair counts go to the workspace.  flags: 0 or
 * SPH_INTERACT_REUSE_CELLS (after sph_batch_refresh_view: each slot's search
 * widened by its own recorded displacement, which the batched predictor
 * records per slot; SPH_ERR_MARGIN in the global word and the word of each
 * slot whose particles moved half a cell or more); other bits: SPH_E_ARG. */
sph_status sph_batch_interact(const sph_batch* b, const sph_state* s, const uint32_t* key,
                              const uint32_t* cell_start, float* ace, float* arho, float* visc,
                              uint32_t* nbr_count, uint32_t flags, void* ws, size_t ws_bytes,
                              void* stream);

/* As sph_refresh_view, over all slots: the view of the current state
 * relative to the cells of the last sph_batch_bin_cells (the second
 * interaction of a symplectic step without a second binning).  A particle
 * now outside its slot's grid is excluded (SPH_ERR_EXCLUDED in the global
 * word and its slot's word).  Like sph_batch_bin_cells it clears the
 * per-slot maxima and pair counts that the next sph_batch_interact
 * accumulates. */
sph_status sph_batch_refresh_view(const sph_batch* b, sph_state* s, const uint32_t* key, void* ws,
                                  size_t ws_bytes, void* stream);

/* Eq. 35 per slot: dt[n_slots] out (device); interactions[n_slots][2]
 * in/out, nullable: each slot's pair count and wall-target count are added. */
sph_status sph_batch_reduce_dt(const sph_batch* b, double* dt, uint64_t* interactions, void* ws,
                               size_t ws_bytes, void* stream);

/* As sph_symplectic_step with per-slot dt[n_slots] and t[n_slots] (device). */
sph_status sph_batch_symplectic_step(const sph_batch* b, int32_t phase, const double* dt,
                                     double* t, sph_state* saved, sph_state* s, const float* ace,
                                     const float* arho, void* ws, size_t ws_bytes, void* stream);

/* sph_shifting over a batch, right after sph_batch_symplectic_step phase 1:
 * every slot whose shift_coef is positive is shifted with its own A_s,
 * surface threshold, dt[n_slots] (device) and, with
 * SPH_INTERACT_REUSE_CELLS, its own recorded displacement; other slots are
 * left as they are (C = 0 and no shift in conc and shift).  conc[n_total]
 * and shift[3][n_total] (packed layout) are nullable outputs as in
 * sph_shifting.  A slot's results do not depend on the other slots.
 * flags: 0 or SPH_INTERACT_REUSE_CELLS (else SPH_E_ARG). */
sph_status sph_batch_shifting(const sph_batch* b, sph_state* s, const uint32_t* key,
                              const uint32_t* cell_start, const double* dt, float* conc,
                              float* shift, uint32_t flags, void* ws, size_t ws_bytes,
                              void* stream);

/* Per-slot error words (SPH_ERR_* bits) to host slot_errors[n_slots], after
 * synchronising the device; the workspace's global error word (read with
 * sph_read_error) holds their union. */
sph_status sph_batch_read_errors(const sph_batch* b, const void* ws, uint32_t* slot_errors);

/* Enqueues clearing of the global and the per-slot error words. */
sph_status sph_batch_clear_errors(const sph_batch* b, void* ws, void* stream);

/* Reads the device error word (SPH_ERR_* bits) of a workspace.  Synchronises
 * the device.  Returns a negative sph_status on failure. */
int32_t sph_read_error(const void* ws);

/* Enqueues clearing of the workspace's error word (a fill kernel). */
sph_status sph_clear_error(void* ws, void* stream);

/* Static description of a status code. */
const char* sph_strerror(sph_status s);

#ifdef __cplusplus
}
#endif
#endif /* SPH_H */
