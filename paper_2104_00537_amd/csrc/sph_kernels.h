// Host-side launchers of the libsph kernels (one per ABI call).
#pragma once

#include "sph_internal.h"

namespace sph {

KParams make_kparams(const sph_params& p);
int key_bits(uint32_t ncell_total);
void exclusive_scan(uint32_t* data, int64_t len, uint32_t* part, hipStream_t st);

hipError_t launch_bin_cells(const KParams& kp, int64_t n, const sph_state& in, sph_state& out,
                            const sph_state* cin, sph_state* cout, uint32_t* key,
                            uint32_t* perm, uint32_t* cell_start, void* ws, hipStream_t st);
hipError_t launch_interact(const KParams& kp, int64_t n, const sph_state& s, const uint32_t* key,
                           const uint32_t* cell_start, float* ace, float* arho, float* visc,
                           uint32_t* nbr, uint32_t flags, void* ws, hipStream_t st);
hipError_t launch_reduce_dt(const KParams& kp, int64_t n, double* dt, uint64_t* interactions,
                            float* maxima, void* ws, hipStream_t st);
hipError_t launch_symplectic(const KParams& kp, int64_t n, int phase, const double* dt, double* t,
                             sph_state& saved, sph_state& s, const float* ace, const float* arho,
                             void* ws, hipStream_t st);
hipError_t launch_clear_error(void* ws, hipStream_t st);

}  // namespace sph
