// sph_interact_noalloc: the interaction of sph_interact for callers that
// cannot allocate device memory, with every region the pass needs besides its
// inputs and outputs (the view, the per-block partial results, the header and
// the displacement record) in one file-scope device array.
//
// Host code never passes the array's name to a kernel: in host code that name
// is a host-side stand-in.  Each device's address of its copy comes from
// hipGetSymbolAddress, once per device (with that device current), and only
// that address is used afterwards.
#include <mutex>

#include "sph_kernels.h"
#include "sph_dev.h"

namespace sph {
namespace {

constexpr int64_t kNaMaxN = SPH_NOALLOC_MAX_N;
constexpr int64_t kNaBlocks = (kNaMaxN + kBlock - 1) / kBlock;
constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }
// layout of the array (offsets in bytes)
constexpr size_t kNaHdr = 0;
constexpr size_t kNaDisp = align256(kNaHdr + sizeof(WsHeader));
constexpr size_t kNaRed = align256(kNaDisp + sizeof(uint32_t) * kDispSlots);
constexpr size_t kNaPr = align256(kNaRed + sizeof(BlockRed) * kNaBlocks * kMaxLanes);
constexpr size_t kNaVp = align256(kNaPr + 16 * (size_t)(kNaMaxN + kViewPad));
constexpr size_t kNaTotal = align256(kNaVp + 16 * (size_t)(kNaMaxN + kViewPad));

__device__ __align__(256) unsigned char scratch[kNaTotal];

constexpr int kNaMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_scratch[kNaMaxDevices] = {};

// The current device's address of `scratch` (looked up on the first call on
// that device), or nullptr on failure.
unsigned char* scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNaMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  return g_scratch[dev];
}

// Clears the header (error word, partial-result count) and the displacement
// record: a call starts from nothing that an earlier call left.
__global__ void k_na_clear(WsHeader* __restrict__ hdr, uint32_t* __restrict__ disp) {
  const int t = threadIdx.x;
  if (t < kDispSlots) disp[t] = 0u;
  if (t == 0) {
    hdr->err = 0u;
    hdr->nred = 0u;
  }
}

// The view entry of every sorted slot from the state, relative to the cell of
// its key (as the binning writes it); excluded particles get zero entries.
__global__ void k_na_view(KParams kp, int64_t n, const uint32_t* __restrict__ key, sph_state s,
                          float4* __restrict__ pr, float4* __restrict__ vp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint8_t t = s.type[i];
  if (t & SPH_EXCLUDED) {
    pr[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    vp[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  double x[3] = {0.0, 0.0, 0.0};
  float v[3] = {0.f, 0.f, 0.f};
  for (int d = 0; d < kp.dim; ++d) {
    x[d] = s.pos[d * n + i];
    v[d] = s.vel[d * n + i];
  }
  write_view(kp, i, x, v, s.rho[i], t, key[i], pr, vp);
}

}  // namespace
}  // namespace sph

using namespace sph;

extern "C" sph_status sph_interact_noalloc(const sph_params* p, int64_t n, const sph_state* s,
                                           const uint32_t* key, const uint32_t* cell_start,
                                           float* ace, float* arho, float* visc,
                                           uint32_t* nbr_count, uint32_t flags, void* stream) {
  if (!params_ok(p) || !cell_start) return SPH_E_ARG;
  if ((uint64_t)p->ncell[0] * p->ncell[1] * p->ncell[2] >= ((uint64_t)1 << 30)) return SPH_E_ARG;
  if (n < 0 || n > kNaMaxN) return SPH_E_ARG;
  // the view is built from the state: not with modified DBC, whose wall
  // entries come from sph_mdbc, nor on reused cells
  if (p->boundary != 0) return SPH_E_ARG;
  const uint32_t base = flags & ~(uint32_t)SPH_INTERACT_ONE_LANE;
  if (base != 0 && base != SPH_DIAG_COUNT_F64 && base != SPH_INTERACT_F64 &&
      base != SPH_INTERACT_ABS_F32)
    return SPH_E_ARG;
  if ((base == SPH_INTERACT_F64 || base == SPH_INTERACT_ABS_F32) &&
      (p->kernel != 0 || p->viscosity != 0 || p->ddt == 2 || p->floating != 0 ||
       p->period[0] > 0.0 || p->period[1] > 0.0 || p->period[2] > 0.0))
    return SPH_E_ARG;
  if (n > 0 && (!s || !s->pos || !s->vel || !s->rho || !s->type || !key || !ace || !arho))
    return SPH_E_ARG;
  unsigned char* w = scratch_ptr();
  if (!w) return SPH_E_HIP;
  const hipStream_t st = (hipStream_t)stream;
  const KParams kp = make_kparams(*p);
  WsHeader* hdr = reinterpret_cast<WsHeader*>(w + kNaHdr);
  uint32_t* disp = reinterpret_cast<uint32_t*>(w + kNaDisp);
  float4* pr = reinterpret_cast<float4*>(w + kNaPr);
  float4* vp = reinterpret_cast<float4*>(w + kNaVp);
  hipLaunchKernelGGL(k_na_clear, dim3(1), dim3(kDispSlots), 0, st, hdr, disp);
  sph_state s0 = n > 0 ? *s : sph_state{};
  if (n > 0)
    hipLaunchKernelGGL(k_na_view, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       st, kp, n, key, s0, pr, vp);
  if (hipGetLastError() != hipSuccess) return SPH_E_HIP;
  const InteractScratch sc{pr, vp, reinterpret_cast<BlockRed*>(w + kNaRed), hdr, disp};
  return launch_interact_on(kp, n, s0, key, cell_start, ace, arho, visc, nbr_count, flags, sc,
                            st) == hipSuccess
             ? SPH_OK
             : SPH_E_HIP;
}
