// Host-side launchers of the libsph kernels (one per ABI call).
#pragma once

#include "sph_internal.h"

namespace sph {

KParams make_kparams(const sph_params& p);
KParams make_slot_kparams(const sph_params& p);

// Host view of a batch (see sph_batch in sph.h).
struct BatchDesc {
  int n_slots;
  int cell_div;
  int64_t n_total;
  int64_t key_cells;
  const void* table;  // device SlotEntry[n_slots]
  uint32_t flags;     // SPH_BATCH_* flags of sph_batch_describe
  uint32_t lanes;     // interaction lanes over all slots
};
int key_bits(uint32_t ncell_total);
void exclusive_scan(uint32_t* data, int64_t len, uint32_t* part, hipStream_t st);
hipError_t radix_sort(int64_t n, uint32_t max_key, uint32_t* key_out, uint32_t* perm_out,
                      void* ws, hipStream_t st);
void launch_cell_start(const uint32_t* key, int64_t n, uint32_t last_key, uint32_t* cell_start,
                       hipStream_t st);

hipError_t launch_bin_cells(const KParams& kp, int64_t n, const sph_state& in, sph_state& out,
                            const sph_state* cin, sph_state* cout, uint32_t* key,
                            uint32_t* perm, uint32_t* cell_start, void* ws, hipStream_t st);
hipError_t launch_refresh_view(const KParams& kp, int64_t n, const sph_state& s,
                               const uint32_t* key, void* ws, hipStream_t st);
hipError_t launch_interact(const KParams& kp, int64_t n, const sph_state& s, const uint32_t* key,
                           const uint32_t* cell_start, float* ace, float* arho, float* visc,
                           uint32_t* nbr, uint32_t flags, void* ws, hipStream_t st);
// The device regions an interaction pass reads and writes besides its inputs
// and outputs: the view, the per-block partial results, the header with the
// error word and the displacement record.
struct InteractScratch {
  const float4* pr;
  const float4* vp;
  BlockRed* red;
  WsHeader* hdr;
  const uint32_t* disp;
};
hipError_t launch_interact_on(const KParams& kp, int64_t n, const sph_state& s,
                              const uint32_t* key, const uint32_t* cell_start, float* ace,
                              float* arho, float* visc, uint32_t* nbr, uint32_t flags,
                              const InteractScratch& w, hipStream_t st);
bool params_ok(const sph_params* p);
hipError_t launch_build_list(const KParams& kp, int64_t n, const sph_state& s,
                             const uint32_t* key, const uint32_t* cell_start, float skin_min,
                             bool adaptive, void* list, int64_t cap, void* ws, hipStream_t st);
hipError_t launch_interact_list(const KParams& kp, int64_t n, const sph_state& s,
                                const uint32_t* key, const uint32_t* cell_start,
                                const void* list, int64_t cap, float* ace, float* arho,
                                float* visc, uint32_t* nbr, uint32_t flags, void* ws,
                                hipStream_t st);
hipError_t launch_reduce_dt(const KParams& kp, int64_t n, double* dt, uint64_t* interactions,
                            float* maxima, void* ws, hipStream_t st);
hipError_t launch_symplectic(const KParams& kp, int64_t n, int phase, const double* dt, double* t,
                             sph_state& saved, sph_state& s, const float* ace, const float* arho,
                             void* ws, hipStream_t st);
hipError_t launch_verlet(const KParams& kp, int64_t n, int mode, const double* dt, double* t,
                         sph_state& prev, sph_state& s, const float* ace, const float* arho,
                         void* ws, hipStream_t st);
hipError_t launch_mdbc(const KParams& kp, int64_t n, const sph_state& s, const uint32_t* key,
                       const uint32_t* cell_start, void* ws, hipStream_t st);
hipError_t launch_floating(const KParams& kp, int64_t n, int phase, const double* dt,
                           sph_body* bodies, int nb, const sph_state& saved, sph_state& s,
                           const float* ace, void* ws, hipStream_t st);
hipError_t launch_shifting(const KParams& kp, int64_t n, const sph_state& s, const uint32_t* key,
                           const uint32_t* cell_start, const double* dt, float* conc,
                           float* shift, bool reuse, void* ws, hipStream_t st);
hipError_t launch_clear_error(void* ws, hipStream_t st);

hipError_t launch_batch_bin_cells(const BatchDesc& B, const sph_state& in, sph_state& out,
                                  const sph_state* cin, sph_state* cout, uint32_t* key,
                                  uint32_t* perm, uint32_t* cell_start, void* ws, hipStream_t st);
hipError_t launch_batch_interact(const BatchDesc& B, const uint32_t* key,
                                 const uint32_t* cell_start, float* ace, float* arho, float* visc,
                                 uint32_t* nbr, bool reuse, void* ws, hipStream_t st);
hipError_t launch_batch_refresh_view(const BatchDesc& B, const sph_state& s, const uint32_t* key,
                                     void* ws, hipStream_t st);
hipError_t launch_batch_reduce_dt(const BatchDesc& B, double* dt, uint64_t* interactions, void* ws,
                                  hipStream_t st);
hipError_t launch_batch_symplectic(const BatchDesc& B, int phase, const double* dt, double* t,
                                   sph_state& saved, sph_state& s, const float* ace,
                                   const float* arho, void* ws, hipStream_t st);
hipError_t launch_batch_clear_errors(const BatchDesc& B, void* ws, hipStream_t st);
hipError_t launch_batch_shifting(const BatchDesc& B, const sph_state& s, const uint32_t* key,
                                 const uint32_t* cell_start, const double* dt, float* conc,
                                 float* shift, bool reuse, void* ws, hipStream_t st);

}  // namespace sph
