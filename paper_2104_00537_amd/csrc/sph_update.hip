// System update (Section 5.1): the variable time step of Eq. 35, the
// symplectic position-Verlet update of Eq. 33-34 and the Verlet update of
// Eq. 30-31, with the imposed motion of moving walls (Eq. 37).
#include "sph_dev.h"
#include "sph_kernels.h"

namespace sph {

// Eq. 35 from the per-block partials of the last interaction pass; one block.
constexpr int kRedThreads = 1024;

__global__ __launch_bounds__(kRedThreads) void k_reduce_dt(KParams kp, const BlockRed* __restrict__ red,
                            WsHeader* __restrict__ hdr, double* __restrict__ dt,
                            uint64_t* __restrict__ inter, float* __restrict__ maxima) {
  uint32_t* err = &hdr->err;
  const int64_t nblk = hdr->nred;
  __shared__ float sf[kRedThreads / 64], sv[kRedThreads / 64];
  __shared__ unsigned long long sc[kRedThreads / 64], sw[kRedThreads / 64], sn[kRedThreads / 64];
  float fmax = 0.f, vmax = 0.f;
  unsigned long long cnt = 0, cntw = 0, nfl = 0;
  for (int64_t b = threadIdx.x; b < nblk; b += kRedThreads) {
    const BlockRed r = red[b];
    fmax = fmaxf(fmax, r.fmax);
    vmax = fmaxf(vmax, r.vmax);
    cnt += r.count;
    cntw += r.count_wall;
    nfl += r.nfluid;
  }
  fmax = wave_max(fmax);
  vmax = wave_max(vmax);
  for (int off = 32; off > 0; off >>= 1) {
    cnt += __shfl_xor(cnt, off, 64);
    cntw += __shfl_xor(cntw, off, 64);
    nfl += __shfl_xor(nfl, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { sf[wave] = fmax; sv[wave] = vmax; sc[wave] = cnt; sw[wave] = cntw; sn[wave] = nfl; }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < kRedThreads / 64; ++w) {
    sf[0] = fmaxf(sf[0], sf[w]);
    sv[0] = fmaxf(sv[0], sv[w]);
    sc[0] += sc[w];
    sw[0] += sw[w];
    sn[0] += sn[w];
  }
  const double f = (double)sf[0], v = (double)sv[0];
  double d = INFINITY;
  if (sn[0] > 0) {
    const double dtf = f > 0.0 ? sqrt(kp.h / f) : INFINITY;
    const double dtcv = kp.h / (kp.c0 + v);
    d = kp.cfl * (dtf < dtcv ? dtf : dtcv);
  }
  *dt = d;
  if (!(d >= kp.dt_floor) || !isfinite(d)) set_error(err, SPH_ERR_DT_FLOOR);
  if (inter) {
    inter[0] += (uint64_t)sc[0];
    inter[1] += (uint64_t)sw[0];
  }
  if (maxima) { maxima[0] = sf[0]; maxima[1] = sv[0]; }
}

// phase 0: predictor, saving state n; phase 1: corrector from the saved state.
// The predictor also records the largest distance a particle moved (for an
// interaction that reuses the cells of the last binning).  F64S: an all-FP64
// state, whose rates ace and arho are FP64 arrays.
template <int PHASE, bool F64S>
__global__ __launch_bounds__(kBlock) void k_symplectic(KParams kp, int64_t n,
                                                       const double* __restrict__ dtp,
                                                       const double* __restrict__ tp,
                                                       sph_state saved, sph_state s,
                                                       const void* __restrict__ ace,
                                                       const void* __restrict__ arho,
                                                       uint32_t* __restrict__ err,
                                                       uint32_t* __restrict__ disp) {
  __shared__ double shm[3];
  if (threadIdx.x == 0) {
    const double dt = *dtp, t = *tp;
    const double t1 = PHASE == 0 ? t + 0.5 * dt : t + dt;
    shm[0] = dt;
    shm[1] = motion_disp(kp, t1) - motion_disp(kp, t);
    shm[2] = motion_vel(kp, t1);
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double disp2 = 0.0;
  bool bad = false;
  if (i < n) {
    if constexpr (F64S)
      bad = symplectic_one_f64<PHASE>(kp, n, i, shm[0], shm[1], shm[2], saved, s,
                                      static_cast<const double*>(ace),
                                      static_cast<const double*>(arho), disp2);
    else
      bad = symplectic_one<PHASE>(kp, n, i, shm[0], shm[1], shm[2], saved, s,
                                  static_cast<const float*>(ace),
                                  static_cast<const float*>(arho), disp2);
  }
  if (bad) set_error(err, SPH_ERR_NONFINITE);
  if (PHASE == 0) record_displacement(disp2, disp);
}

// Verlet update (Eq. 30 for MODE 0, Eq. 31 for MODE 1) of the sorted state.
template <int MODE>
__global__ void k_verlet(KParams kp, int64_t n, const double* __restrict__ dtp,
                         const double* __restrict__ tp, sph_state prev, sph_state s,
                         const float* __restrict__ ace, const float* __restrict__ arho,
                         uint32_t* __restrict__ err) {
  __shared__ double shm[3];
  if (threadIdx.x == 0) {
    const double dt = *dtp, t = *tp;
    shm[0] = dt;
    shm[1] = motion_disp(kp, t + dt) - motion_disp(kp, t);
    shm[2] = motion_vel(kp, t + dt);
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (verlet_one<MODE>(kp, n, i, shm[0], shm[1], shm[2], prev, s, ace, arho))
    set_error(err, SPH_ERR_NONFINITE);
}

__global__ void k_advance_time(const double* __restrict__ dt, double* __restrict__ t) {
  if (threadIdx.x == 0) *t = *t + *dt;
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t len, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) p[i] = v;
}

hipError_t launch_reduce_dt(const KParams& kp, int64_t n, double* dt, uint64_t* interactions,
                            float* maxima, void* ws, hipStream_t st) {
  const WsLayout L = ws_layout(n);
  hipLaunchKernelGGL(k_reduce_dt, dim3(1), dim3(kRedThreads), 0, st, kp, ws_ptr<BlockRed>(ws, L.red),
                     ws_ptr<WsHeader>(ws, L.err), dt, interactions, maxima);
  return hipGetLastError();
}

hipError_t launch_symplectic(const KParams& kp, int64_t n, int phase, const double* dt, double* t,
                             sph_state& saved, sph_state& s, const float* ace, const float* arho,
                             void* ws, hipStream_t st) {
  const WsLayout L = ws_layout(n);
  WsHeader* hdr = ws_ptr<WsHeader>(ws, L.err);
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  if (n > 0) {
    uint32_t* disp = ws_ptr<uint32_t>(ws, L.disp);
    const bool f64s = s.vel64 != nullptr;
#define SPH_SYMP(PH, F)                                                                      \
  hipLaunchKernelGGL((k_symplectic<PH, F>), dim3(grid), dim3(kBlock), 0, st, kp, n, dt, t, \
                     saved, s, (const void*)ace, (const void*)arho, &hdr->err, disp)
    if (phase == 0) {
      if (f64s) SPH_SYMP(0, true); else SPH_SYMP(0, false);
    } else {
      if (f64s) SPH_SYMP(1, true); else SPH_SYMP(1, false);
    }
#undef SPH_SYMP
  }
  if (phase == 1) hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(64), 0, st, dt, t);
  return hipGetLastError();
}

hipError_t launch_verlet(const KParams& kp, int64_t n, int mode, const double* dt, double* t,
                          sph_state& prev, sph_state& s, const float* ace, const float* arho,
                          void* ws, hipStream_t st) {
  const WsLayout L = ws_layout(n);
  uint32_t* err = ws_ptr<uint32_t>(ws, L.err);
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  if (n > 0) {
    if (mode == 0)
      hipLaunchKernelGGL(k_verlet<0>, dim3(grid), dim3(kBlock), 0, st, kp, n, dt, t, prev, s,
                         ace, arho, err);
    else
      hipLaunchKernelGGL(k_verlet<1>, dim3(grid), dim3(kBlock), 0, st, kp, n, dt, t, prev, s,
                         ace, arho, err);
  }
  hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(64), 0, st, dt, t);
  return hipGetLastError();
}

hipError_t launch_clear_error(void* ws, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, ws_ptr<uint32_t>(ws, 0), (int64_t)1, 0u);
  return hipGetLastError();
}

}  // namespace sph
