// Internal definitions shared by the gfx950 kernels of libsph: the launch
// parameter block, the workspace layout and small device helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sph.h"

namespace sph {

constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kSortItems = 8;      // keys per thread per radix tile
constexpr int kSortTile = kBlock * kSortItems;
constexpr int kScanTile = kBlock * 8;
constexpr int kViewPad = 8;        // spare float4 entries after each interaction view
constexpr int kFrameCells = 8;     // x offsets in the views are taken per block of 8 cells
constexpr uint32_t kXcds = 8;      // accelerator complex dies of the MI355X
constexpr int kFloatParts = 32;    // blocks per floating body in its reductions
constexpr int kFloatSums = 16;     // FP64 partial sums per block (force, torque, inertia, count)
constexpr int kFloatMotion = 24;   // FP64 words of a body's rigid motion of one phase

// Per-launch constants derived once on the host from sph_params.
struct KParams {
  int dim, cell_div, ddt, x_sub;   // x_sub: key cells per cell along x
  int lg_xsub;
  int periodic;                    // bit k: component k is periodic (Section 2.7)
  int kernel, viscosity;           // 0 Wendland / 1 cubic spline; 0 artificial / 1 laminar
  int boundary;                    // 0 DBC (Eq. 36) / 1 modified DBC (Eq. 38-39)
  int floating;                    // 1: floating particles (type 3) get Eq. 47
  int ncx, ncy, ncz;
  uint32_t ncell_total;          // also the key of particles outside the grid
  double ox, oy, oz;             // grid origin
  double cs, inv_cs, inv_csx;     // cell size, its inverse, inverse along x (times x_sub)
  double h, rho0, gamma, c0, b_tait, cfl, dt_floor;
  double mass_f, mass_b;
  double gx, gy, gz;
  double motion_amp, motion_omega;
  double px, py, pz;             // periods (0: open)
  double support2;               // (2h)^2 in FP64, for the diagnostic count
  // FP32 copies for the interaction kernel
  double inv_frame;               // 1 / (kFrameCells cs)
  double kfab, alpha_c0, ddt_coef, eta2;  // FP64 copies for the precision-study arms
  double inv_h, w_alpha, f_coef;          // FP64 kernel: 1/h, alpha_D, gradient factor
  float h_f, mhalf_inv_h_f, support2_f;      // h, -1/(2h), 4h^2
  float kfab_mf_f, kfab_mb_f;                // kfab m_fluid, kfab m_wall; kfab = -5 alpha_D / h^2
  float kpi_mf_f, kpi_mb_f;                  // -2 alpha c0 kfab m (Eq. 21 with Eq. 22)
  float inv_h_f;                             // 1/h (cubic spline)
  float klam_mf_f, klam_mb_f;                // 4 nu0 kfab m (Eq. 23)
  float fz_f, hc1_f, hc2_f, hc3_f;           // Eq. 19-20: eps = fz z_ab, rho^H = eps(c1 + eps(c2 + eps c3))
  float eta2_f, ddt_coef_f;                  // eta^2 ; 2 delta h c0
  float kvc_f;                               // -1/(2 alpha c0 h) (Eq. 21), or 1/(4 nu0) (Eq. 23)
  float mass_ratio_f;                        // m_wall / m_fluid
  float cs_f, inv_csx_f, unit_x_f;           // cell size, inverse key-cell size along x, x offset unit
  float gx_f, gy_f, gz_f;
  uint32_t lu;                   // the x period in x-offset units, modulo 2^32
  float w_alpha_f;               // alpha_D of the kernel (shifting's W)
  float shift_k_f, shift_fs_f;   // A_s h (Eq. 41); surface threshold on C
};

// Per-block partial results of the interaction (reduced by sph_reduce_dt).
struct BlockRed {
  float fmax;          // max |dv/dt| over fluid targets of the block
  float vmax;          // max visc over fluid targets of the block
  uint32_t count;      // interactions evaluated by the block
  uint32_t count_wall; // ... of which with a wall target (continuity only)
  uint32_t nfluid;     // fluid targets in the block
  uint32_t pad;
};

// Fixed header at offset 0 of the workspace.
struct WsHeader {
  uint32_t err;      // SPH_ERR_* bits
  uint32_t nred;     // BlockRed entries written by the last interaction pass
  uint32_t nwall;    // wall particles listed by the last sph_mdbc (its work list)
  uint32_t bin_gen;  // binnings so far (modulo 2^32): a neighbour list records
                     // the binning it was built on
  uint32_t list_walks;  // list passes that walked the cells instead (every
                        // target: the displacement exceeded the list's skin)
  uint32_t skin_hint;   // bits of the skin the last list pass on reused
                        // cells asks for (a float: 1.5 times twice the
                        // displacement it saw)
  uint32_t pad[58];
};

// ------------------------------------------------------- neighbour lists --
// A neighbour list (sph_build_list) holds, per target, the candidates of its
// cells within the list radius as chunks: x = first candidate (sorted index),
// y = a mask of the kListSpan candidates from there (bit k: candidate x + k)
// in its low bits and the row of the stencil in the high bits, (dy + 3) +
// 7 (dz + 3).  Chunks follow the stencil's row order, ascending within a row.
constexpr int kListSpan = 26;
constexpr uint32_t kListSpanMask = (1u << kListSpan) - 1u;
constexpr int kListCap = 40;              // chunks per target
constexpr uint32_t kListWalk = 0xffffffffu;  // count of a target whose chunks did not fit

struct ListHeader {
  float skin;        // the list radius is (2h (1 + 1e-4) + skin)
  uint32_t bin_gen;  // the binning the list was built on
  uint32_t cap;      // chunks per target in this buffer
  uint32_t pad[61];
};

struct ListLayout {
  size_t header, count, chunks, total;
};

inline ListLayout list_layout(int64_t n, int64_t cap) {
  ListLayout L{};
  const size_t nn = (size_t)(n > 0 ? n : 1);
  size_t off = 0;
  L.header = off; off += 256;
  L.count = off; off = (off + 4 * nn + 255) / 256 * 256;
  L.chunks = off; off += 8 * nn * (size_t)cap;
  L.total = off;
  return L;
}

// The largest distance a particle moved since the last binning, kept as the
// bits of non-negative floats in kDispSlots words (blocks record into the
// slot of their index modulo kDispSlots, which keeps the atomics apart); the
// value is the maximum over the slots.  The binning sets them to 0.
constexpr int kDispSlots = 64;

// ---------------------------------------------------------------- batches --
// One case ("slot") of a batch: its constants (in 3-D geometry: a 2-D case
// is stored as (x, 0, z) with one cell across y), its first cell key and its
// particle range in the packed arrays.
struct SlotEntry {
  KParams kp;
  uint32_t cbase;    // keys of the slot: cbase .. cbase + kp.ncell_total
  int32_t lpt;       // interaction lanes per target particle (1 or kMaxLanes)
  int64_t off;       // first particle of the slot
  int64_t n;         // particles of the slot
  int64_t loff;      // first interaction lane of the slot (lanes in slot order)
};

// Per-slot results of one interaction pass (cleared by each binning);
// maxima of non-negative floats are kept as their bit patterns.  Each slot
// has kAccCopies copies (blocks add into the copy of their index modulo
// kAccCopies, which keeps the atomics of a large slot apart); the slot's
// value combines the copies.
constexpr int kAccCopies = 64;
struct SlotAccum {
  uint32_t fmax_bits, vmax_bits, nfluid, pad;
  unsigned long long count, count_wall;
};

// Per-slot time step and imposed wall motion of the current update phase.
struct SlotMotion {
  double dt, dmove, vmove, pad;
};

// Most lanes that share one target particle in the interaction, and the
// largest case that gets them (n * kMaxLanes / 64 wavefronts at most).
constexpr int kMaxLanes = 4;
constexpr int64_t kLanesMaxN = 131072;

// Workspace layout (offsets in bytes, each region 256-aligned).
struct WsLayout {
  size_t err;        // the WsHeader (offset 0)
  size_t keyA, valA, keyB, valB;   // radix sort ping-pong buffers, n each
  size_t hist;       // uint32 [bins * nblk_sort] digit counts / offsets
  size_t scan_part;  // uint32 partial sums of the offset scan
  size_t view_pr;    // float4 [n]: cell-relative position, signed density
  size_t view_vp;    // float4 [n]: velocity, pressure
  size_t red;        // BlockRed [nblk_interact]
  size_t disp;       // uint32 [kDispSlots]: displacement record
  size_t fpart;      // double [SPH_MAX_BODIES][kFloatParts][kFloatSums]: body partial sums
  size_t fmotion;    // double [SPH_MAX_BODIES][kFloatMotion]: rigid motion of each body
  size_t total;
  int64_t nblk_sort, nblk_interact, hist_len, scan_parts;
};

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

inline WsLayout ws_layout(int64_t n) {
  WsLayout L{};
  const size_t nn = (size_t)(n > 0 ? n : 1);
  L.nblk_sort = (n + kSortTile - 1) / kSortTile;
  if (L.nblk_sort < 1) L.nblk_sort = 1;
  // one per-block partial result per interaction block of kBlock targets
  L.nblk_interact = (n + kBlock - 1) / kBlock;
  if (L.nblk_interact < 1) L.nblk_interact = 1;
  L.hist_len = 256 * L.nblk_sort;
  L.scan_parts = (L.hist_len + kScanTile - 1) / kScanTile;
  size_t off = 0;
  L.err = off; off = align_up(off + sizeof(WsHeader));
  L.keyA = off; off = align_up(off + 4 * nn);
  L.valA = off; off = align_up(off + 4 * nn);
  L.keyB = off; off = align_up(off + 4 * nn);
  L.valB = off; off = align_up(off + 4 * nn);
  L.hist = off; off = align_up(off + 4 * (size_t)L.hist_len);
  L.scan_part = off; off = align_up(off + 4 * (size_t)L.scan_parts + 4);
  // the views carry kViewPad spare entries: the interaction reads candidates
  // in groups of 4 with scalar loads that may run past the last particle
  L.view_pr = off; off = align_up(off + 16 * (nn + kViewPad));
  L.view_vp = off; off = align_up(off + 16 * (nn + kViewPad));
  // (room for the blocks of kMaxLanes lanes per target)
  L.red = off; off = align_up(off + sizeof(BlockRed) * (size_t)L.nblk_interact * kMaxLanes);
  L.disp = off; off = align_up(off + sizeof(uint32_t) * kDispSlots);
  L.fpart = off;
  off = align_up(off + sizeof(double) * SPH_MAX_BODIES * kFloatParts * kFloatSums);
  L.fmotion = off; off = align_up(off + sizeof(double) * SPH_MAX_BODIES * kFloatMotion);
  L.total = off;
  return L;
}

// A batch workspace: the single-case layout for all packed particles, then
// per-slot accumulators, motion table, error words and displacement records
// (kDispSlots words per slot, as the single-case record).
struct BatchWsLayout {
  WsLayout base;
  size_t accum, motion, slot_err, disp, total;
};

inline BatchWsLayout batch_ws_layout(int32_t n_slots, int64_t n) {
  BatchWsLayout B{};
  B.base = ws_layout(n);
  const size_t ns = (size_t)(n_slots > 0 ? n_slots : 1);
  size_t off = B.base.total;
  B.accum = off; off = align_up(off + sizeof(SlotAccum) * kAccCopies * ns);
  B.motion = off; off = align_up(off + sizeof(SlotMotion) * ns);
  B.slot_err = off; off = align_up(off + sizeof(uint32_t) * ns);
  B.disp = off; off = align_up(off + sizeof(uint32_t) * kDispSlots * ns);
  B.total = off;
  return B;
}

template <typename T>
inline T* ws_ptr(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// ---------------------------------------------------------------- device ----
__device__ inline bool is_excluded(uint8_t t) { return (t & SPH_EXCLUDED) != 0; }
__device__ inline bool is_fluid(uint8_t t) { return (t & 0x7f) == SPH_FLUID; }
__device__ inline bool is_floating(uint8_t t) { return (t & 0x7f) == SPH_FLOATING; }

__device__ inline void set_error(uint32_t* err, uint32_t bits) {
  atomicOr(err, bits);
}

// The dispatcher hands workgroup b to XCD b % kXcds.  Returns the logical
// block index that deals chunks of kXcdChunk consecutive blocks to the XCDs
// in turn (XCD x runs chunks x, x + kXcds, ...; a last incomplete round keeps
// the identity), so that blocks working on neighbouring data mostly share
// one L2 while every XCD gets a share of every part of the domain: the work
// per target varies across the domain (walls, free surface), and one
// contiguous share per XCD leaves some XCDs idle at the end.  A bijection of
// [0, nb).
constexpr uint32_t kXcdChunk = 16;
__device__ inline uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t full = nb / (kXcds * kXcdChunk) * (kXcds * kXcdChunk);
  if (b >= full) return b;
  const uint32_t x = b % kXcds, k = b / kXcds;
  return ((k / kXcdChunk) * kXcds + x) * kXcdChunk + k % kXcdChunk;
}

// Wave-wide reductions over the 64 lanes of a wavefront.
__device__ inline float wave_max(float v) {
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline uint32_t wave_max_u32(uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor(v, off, 64));
  return v;
}

// Raises the recorded largest displacement since the binning to cover the
// distance sqrt(d2) (d2 >= 0, FP64) for the calling block: one atomic per
// block, into its slot.  Every thread of the block calls this (threads
// without a displacement pass 0).
__device__ inline void record_displacement(double d2, uint32_t* disp) {
  __shared__ uint32_t wmax[kBlock / 64];
  // d2 rounded up to a float, its root to nearest then one ulp up: the
  // recorded float is never below the distance
  const float r = __fsqrt_rn(__double2float_ru(d2));
  uint32_t b = __float_as_uint(r) + (r > 0.f ? 1u : 0u);
  b = wave_max_u32(b);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) wmax[wave] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = max(m, wmax[w]);
    if (m) atomicMax(&disp[blockIdx.x % kDispSlots], m);
  }
}

// The recorded displacement (max over the slots; uniform loads).
__device__ inline float read_displacement(const uint32_t* __restrict__ disp) {
  uint32_t m = 0;
  for (int k = 0; k < kDispSlots; ++k) m = max(m, disp[k]);
  return __uint_as_float(m);
}

__device__ inline uint32_t wave_sum(uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace sph
