// Neighbour list (Section 5.1 of the DualSPHysics v5.0 paper): cell keys,
// an in-house stable LSD radix sort in LDS, cell ranges and the reorder of
// the particle state into sorted structure-of-arrays.
#include "sph_dev.h"
#include "sph_kernels.h"

namespace sph {

// -------------------------------------------------------------- cell keys --
// (a new binning also restarts the record of the largest displacement)
__global__ void k_cell_keys(KParams kp, int64_t n, const double* __restrict__ pos,
                            const uint8_t* __restrict__ type, uint32_t* __restrict__ key,
                            uint32_t* __restrict__ disp, WsHeader* __restrict__ hdr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (i == 0) {
    for (int k = 0; k < kDispSlots; ++k) disp[k] = 0u;
    hdr->bin_gen = hdr->bin_gen + 1u;
  }
  key[i] = cell_key_local(kp, pos, type, n, i);
}

// ------------------------------------------------------- exclusive scans --
// Exclusive prefix sum of one value per thread over a 256-thread block.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  uint32_t base = 0, all = 0;
  for (int w = 0; w < kBlock / 64; ++w) {
    if (w < wave) base += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  if (total) *total = all;
  return base + x - v;
}

// Tile-local exclusive scan of kScanTile values; the tile total goes to part[].
__global__ void k_scan_tiles(uint32_t* __restrict__ data, int64_t len,
                             uint32_t* __restrict__ part) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
  uint32_t v[8], s = 0;
  for (int k = 0; k < 8; ++k) {
    v[k] = (base + k < len) ? data[base + k] : 0u;
    s += v[k];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(s, &total);
  for (int k = 0; k < 8; ++k) {
    if (base + k < len) data[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Exclusive scan of the tile totals in one block (loops over chunks).
__global__ void k_scan_parts(uint32_t* __restrict__ part, int64_t parts) {
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t c = 0; c < parts; c += kBlock) {
    const int64_t i = c + threadIdx.x;
    const uint32_t v = i < parts ? part[i] : 0u;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(v, &total);
    const uint32_t cin = carry;
    if (i < parts) part[i] = cin + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry = cin + total;
    __syncthreads();
  }
}

__global__ void k_scan_add(uint32_t* __restrict__ data, int64_t len,
                           const uint32_t* __restrict__ part) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
  const uint32_t add = part[blockIdx.x];
  for (int k = 0; k < 8; ++k)
    if (base + k < len) data[base + k] += add;
}

void exclusive_scan(uint32_t* data, int64_t len, uint32_t* part, hipStream_t st) {
  const int64_t parts = (len + kScanTile - 1) / kScanTile;
  if (parts == 0) return;

  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)parts), dim3(kBlock), 0, st, data, len, part);
  hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kBlock), 0, st, part, parts);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)parts), dim3(kBlock), 0, st, data, len, part);
}

// ------------------------------------------------------------ radix sort --
// One LSD pass over digit (key >> shift) & (2^bits - 1), bits <= 8.  Tiles of
// kSortTile keys; inside a tile the keys are visited in rounds of 256, round
// by round, wave by wave, lane by lane, which is the input order -- so the
// ranks below are stable.
__global__ void k_radix_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                             int bits, uint32_t* __restrict__ hist, int64_t nblk) {
  __shared__ uint32_t h[256];
  const int bins = 1 << bits;
  for (int b = threadIdx.x; b < bins; b += kBlock) h[b] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const uint32_t mask = (uint32_t)bins - 1u;
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + r * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < bins; b += kBlock) hist[(int64_t)b * nblk + blockIdx.x] = h[b];
}

// Scatter of one pass.  Wave w of a block owns keys [w*512, (w+1)*512) of the
// block's tile (8 rounds of 64); a wave ranks the keys of a round among
// themselves with ballots (lanes holding the same digit, in lane order) and
// keeps a running count per digit in its own LDS row, so each key gets its
// position within the wave's digit run without block barriers.  The tile is
// then sorted by digit in LDS (digit-major, then wave, then position) and
// written out from there, so that consecutive threads store consecutive
// addresses of a digit's run.  Tile order is wave-major, round, lane -- the
// input order -- so the pass is stable.
//
// offs holds the digit-major per-tile offsets; with part != nullptr they are
// scanned only within scan tiles of kScanTile entries and part[] holds the
// scan tiles' totals (at most kFusedParts of them), whose prefix each block
// forms itself.
constexpr int kFusedParts = 2 * kBlock;

__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, int64_t n, int shift, int bits,
    const uint32_t* __restrict__ offs, int64_t nblk, const uint32_t* __restrict__ part,
    int64_t parts) {
  __shared__ uint32_t wrun[kBlock / 64][256];  // per-wave digit counts, then local bases
  __shared__ uint32_t dstart[256];             // first local position of each digit
  __shared__ uint32_t gbase[256];              // global position of each digit's run
  __shared__ uint32_t pp[kFusedParts];
  __shared__ uint32_t sk[kSortTile], sv[kSortTile];
  if (part) {
    const int64_t p0 = 2 * (int64_t)threadIdx.x;
    const uint32_t v0 = p0 < parts ? part[p0] : 0u;
    const uint32_t v1 = p0 + 1 < parts ? part[p0 + 1] : 0u;
    const uint32_t ex = block_exclusive_scan(v0 + v1, nullptr);
    pp[p0] = ex;
    pp[p0 + 1] = ex + v0;
  }
  const int bins = 1 << bits;
  const uint32_t mask = (uint32_t)bins - 1u;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int b = lane; b < 256; b += 64) wrun[wave][b] = 0;
  const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
  const int64_t base = tile0 + (int64_t)wave * (64 * kSortItems);
  uint32_t kk[kSortItems], vv[kSortItems], pos[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + r * 64 + lane;
    const bool valid = i < n;
    const uint32_t key = valid ? kin[i] : 0u;
    const uint32_t d = (key >> shift) & mask;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(valid && bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    const uint32_t prior = wrun[wave][d];
    pos[r] = prior + rank;
    // the first lane of each digit group advances the wave's running count
    // (this wave's reads of the round came first, in program order)
    if (valid && rank == 0) wrun[wave][d] = prior + (uint32_t)__popcll(peers);
    kk[r] = key;
    vv[r] = valid ? (vin ? vin[i] : (uint32_t)i) : 0u;
  }
  __syncthreads();
  // digit totals of the tile, their exclusive scan, and the per-wave bases
  const int b = threadIdx.x;  // one digit per thread (bins <= kBlock)
  uint32_t tot = 0;
  if (b < bins)
    for (int w = 0; w < kBlock / 64; ++w) tot += wrun[w][b];
  const uint32_t ds = block_exclusive_scan(b < bins ? tot : 0u, nullptr);
  if (b < bins) {
    dstart[b] = ds;
    const int64_t o = (int64_t)b * nblk + blockIdx.x;
    gbase[b] = offs[o] + (part ? pp[o / kScanTile] : 0u);
    uint32_t s = ds;
    for (int w = 0; w < kBlock / 64; ++w) {
      const uint32_t c = wrun[w][b];
      wrun[w][b] = s;
      s += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    if (base + r * 64 + lane < n) {
      const uint32_t lp = wrun[wave][(kk[r] >> shift) & mask] + pos[r];
      sk[lp] = kk[r];
      sv[lp] = vv[r];
    }
  }
  __syncthreads();
  const int64_t cnt = n - tile0 < kSortTile ? n - tile0 : kSortTile;
  for (int p = threadIdx.x; p < cnt; p += kBlock) {
    const uint32_t key = sk[p];
    const uint32_t d = (key >> shift) & mask;
    const uint32_t dst = gbase[d] + ((uint32_t)p - dstart[d]);
    kout[dst] = key;
    vout[dst] = sv[p];
  }
}

// ------------------------------------------------------------ cell ranges --
// cell_start[c] = first sorted index whose key is >= c (lower bound), for
// c = 0..ncell_total.  A block takes kCsCells consecutive cells: two of its
// waves find the lower bounds of its first cell and of the next block's first
// cell in the whole key array; the keys between them (the block's particles)
// are staged in LDS when they fit, and each cell's lower bound is then found
// there; otherwise within that range in global memory.  Writes are coalesced.
constexpr int kCsCells = 2048;
constexpr int kCsKeys = 4096;

__device__ inline int64_t lower_bound_u32(const uint32_t* __restrict__ a, int64_t lo, int64_t hi,
                                          int64_t v) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kBlock) void k_cell_start(const uint32_t* __restrict__ key,
                                                       int64_t n, uint32_t ncell_total,
                                                       uint32_t* __restrict__ start) {
  __shared__ uint32_t sk[kCsKeys];
  __shared__ int64_t bound[2];
  const int64_t c0 = (int64_t)blockIdx.x * kCsCells;
  const int64_t c1 = c0 + kCsCells < (int64_t)ncell_total + 1 ? c0 + kCsCells
                                                               : (int64_t)ncell_total + 1;
  // waves 0 and 1 find the lower bounds of c0 and c1 by a 64-ary search:
  // each round probes 64 evenly spaced keys of the current range, and the
  // probes below the target (a prefix, the keys being sorted) narrow it to
  // one gap between probes
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (wave < 2) {
    const int64_t c = wave == 0 ? c0 : c1;
    int64_t lo = 0, hi = n;
    while (hi > lo) {
      const int64_t step = (hi - lo + 63) / 64;
      const int64_t p = lo + (int64_t)lane * step;
      const bool below = p < hi && (int64_t)key[p] < c;
      const int64_t cnt = __popcll(__ballot(below));
      const int64_t pc = lo + cnt * step;
      const int64_t nlo = cnt == 0 ? lo : lo + (cnt - 1) * step + 1;
      hi = pc < hi ? pc : hi;
      lo = nlo;
    }
    if (lane == 0) bound[wave] = lo;
  }
  __syncthreads();
  const int64_t lo = bound[0], hi = bound[1];
  const int64_t m = hi - lo;
  if (m <= kCsKeys) {
    for (int64_t k = threadIdx.x; k < m; k += kBlock) sk[k] = key[lo + k];
    __syncthreads();
    for (int64_t c = c0 + threadIdx.x; c < c1; c += kBlock) {
      int a = 0, b = (int)m;
      while (a < b) {
        const int mid = (a + b) >> 1;
        if ((int64_t)sk[mid] < c) a = mid + 1;
        else b = mid;
      }
      start[c] = (uint32_t)(lo + a);
    }
  } else {
    for (int64_t c = c0 + threadIdx.x; c < c1; c += kBlock)
      start[c] = (uint32_t)lower_bound_u32(key, lo, hi, c);
  }
}

// --------------------------------------------------------------- reorder --
__global__ void k_reorder(KParams kp, int64_t n, const uint32_t* __restrict__ perm,
                          const uint32_t* __restrict__ key, sph_state in, sph_state out,
                          sph_state cin, sph_state cout, int carry, float4* __restrict__ pr,
                          float4* __restrict__ vp, uint32_t* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (reorder_one(kp, n, i, perm[i], key[i], in, out, cin, cout, carry, pr, vp))
    set_error(err, SPH_ERR_EXCLUDED);
}

// ------------------------------------------------------------ view refresh --
// Rewrites the view of sorted slot i from the state's current position,
// velocity and density, relative to the cell its key (from the last
// binning) names; positions are not wrapped (they stay relative to that
// cell).  A particle that is now outside the grid along an open component
// is excluded, as a binning would; its view entry gets NaN offsets and zero
// density, so it meets no target in the cell range it still sits in.
__global__ void k_refresh_view(KParams kp, int64_t n, const uint32_t* __restrict__ key,
                               sph_state s, float4* __restrict__ pr, float4* __restrict__ vp,
                               uint32_t* __restrict__ err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint8_t t = s.type[i];
  if (t & SPH_EXCLUDED) return;  // its entry was written by the binning
  if (cell_key_local(kp, s.pos, s.type, n, i) == kp.ncell_total) {
    s.type[i] = t | SPH_EXCLUDED;
    set_error(err, SPH_ERR_EXCLUDED);
    const float nan = __builtin_nanf("");
    pr[i] = make_float4(0.f, nan, nan, 0.f);
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

hipError_t launch_refresh_view(const KParams& kp, int64_t n, const sph_state& s,
                               const uint32_t* key, void* ws, hipStream_t st) {
  const WsLayout L = ws_layout(n);
  if (n > 0)
    hipLaunchKernelGGL(k_refresh_view, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock),
                       0, st, kp, n, key, s, ws_ptr<float4>(ws, L.view_pr),
                       ws_ptr<float4>(ws, L.view_vp), ws_ptr<uint32_t>(ws, L.err));
  return hipGetLastError();
}

// ------------------------------------------------------------------ host --
int key_bits(uint32_t ncell_total) {
  int bits = 1;
  while (bits < 32 && ((uint64_t)1 << bits) <= (uint64_t)ncell_total) ++bits;
  return bits;  // enough bits for keys 0..ncell_total
}

// Stable LSD radix sort of the keys in the workspace's keyA buffer (values
// 0..max_key): sorted keys to key_out, the permutation to perm_out.
hipError_t radix_sort(int64_t n, uint32_t max_key, uint32_t* key_out, uint32_t* perm_out,
                      void* ws, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const WsLayout L = ws_layout(n);
  uint32_t* kA = ws_ptr<uint32_t>(ws, L.keyA);
  uint32_t* vA = ws_ptr<uint32_t>(ws, L.valA);
  uint32_t* kB = ws_ptr<uint32_t>(ws, L.keyB);
  uint32_t* vB = ws_ptr<uint32_t>(ws, L.valB);
  uint32_t* hist = ws_ptr<uint32_t>(ws, L.hist);
  uint32_t* part = ws_ptr<uint32_t>(ws, L.scan_part);
  const int total_bits = key_bits(max_key);
  const int passes = (total_bits + 7) / 8;
  const int per = (total_bits + passes - 1) / passes;
  if (per < 1 || per > 8 || (passes - 1) * per >= total_bits) return hipErrorInvalidValue;
  const uint32_t* ksrc = kA;
  const uint32_t* vsrc = nullptr;  // identity on the first pass
  for (int p = 0; p < passes; ++p) {
    const int shift = p * per;
    const int bits = (shift + per <= total_bits) ? per : (total_bits - shift);
    const bool last = (p == passes - 1);
    uint32_t* kdst = last ? key_out : ((p & 1) ? kA : kB);
    uint32_t* vdst = last ? perm_out : ((p & 1) ? vA : vB);
    const int64_t nblk = L.nblk_sort;
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nblk), dim3(kBlock), 0, st, ksrc, n, shift,
                       bits, hist, nblk);
    const int64_t hlen = (int64_t)(1 << bits) * nblk;
    const int64_t hparts = (hlen + kScanTile - 1) / kScanTile;
    if (hparts <= kFusedParts) {
      // tile-local scans here; the scatter adds the tiles' prefix itself
      hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)hparts), dim3(kBlock), 0, st, hist, hlen,
                         part);
      hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nblk), dim3(kBlock), 0, st, ksrc, vsrc,
                         kdst, vdst, n, shift, bits, hist, nblk, part, hparts);
    } else {
      exclusive_scan(hist, hlen, part, st);
      hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nblk), dim3(kBlock), 0, st, ksrc, vsrc,
                         kdst, vdst, n, shift, bits, hist, nblk, nullptr, (int64_t)0);
    }
    ksrc = kdst;
    vsrc = vdst;
  }
  return hipSuccess;
}

void launch_cell_start(const uint32_t* key, int64_t n, uint32_t last_key, uint32_t* cell_start,
                       hipStream_t st) {
  const int64_t nc1 = (int64_t)last_key + 1;
  hipLaunchKernelGGL(k_cell_start, dim3((unsigned)((nc1 + kCsCells - 1) / kCsCells)),
                     dim3(kBlock), 0, st, key, n, last_key, cell_start);
}

hipError_t launch_bin_cells(const KParams& kp, int64_t n, const sph_state& in, sph_state& out,
                            const sph_state* cin, sph_state* cout, uint32_t* key,
                            uint32_t* perm, uint32_t* cell_start, void* ws, hipStream_t st) {
  const WsLayout L = ws_layout(n);
  uint32_t* err = ws_ptr<uint32_t>(ws, L.err);
  const unsigned gridn = (unsigned)((n + kBlock - 1) / kBlock);
  if (n > 0) {
    hipLaunchKernelGGL(k_cell_keys, dim3(gridn), dim3(kBlock), 0, st, kp, n, in.pos, in.type,
                       ws_ptr<uint32_t>(ws, L.keyA), ws_ptr<uint32_t>(ws, L.disp),
                       ws_ptr<WsHeader>(ws, L.err));
    const hipError_t e = radix_sort(n, kp.ncell_total, key, perm, ws, st);
    if (e != hipSuccess) return e;
  }
  launch_cell_start(key, n, kp.ncell_total, cell_start, st);
  if (n > 0) {
    sph_state ci{}, co{};
    const int carry = (cin && cout) ? 1 : 0;
    if (carry) {
      ci = *cin;
      co = *cout;
    }
    hipLaunchKernelGGL(k_reorder, dim3(gridn), dim3(kBlock), 0, st, kp, n, perm, key, in, out,
                       ci, co, carry, ws_ptr<float4>(ws, L.view_pr), ws_ptr<float4>(ws, L.view_vp),
                       err);
  }
  return hipGetLastError();
}

}  // namespace sph
