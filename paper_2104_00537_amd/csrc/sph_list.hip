// Neighbour lists for the particle interaction (Section 2.3 of the DualSPHysics
// v5.0 paper): the candidates of each target's cells within 2h plus a skin,
// found once per binning by a walk of the cells (k_build_list), and replayed
// by both interaction passes of a symplectic step (k_interact_list): the
// pass at state n on the view of the binning, and the pass at n+1/2 on the
// view refreshed on the same cells, whose particles have moved by at most
// the recorded displacement delta since the binning.
//
// The replay takes every listed candidate through the same FP32 test and
// pair terms as the cell walk and in the same order (the stencil's rows in
// turn, ascending within a row), so it finds the walk's pairs and sums them
// identically, while its lanes stay busy: a lane runs through its own list,
// where the walk makes every lane of a wavefront take the same row and group
// steps and the pair arithmetic of a candidate slot whenever any lane hits
// there.  A pair within 2h at n+1/2 was within 2h + 2 delta at the binning;
// while 2 delta stays within the skin the list holds it, otherwise the pass
// walks the cells as the reused-cells interaction does (same results).
#include "sph_kernels.h"
#include "sph_dev.h"
#include "sph_pair.h"

namespace sph {

// The row code of stencil row (dy, dz) (|dy|, |dz| <= 3) in a chunk's high
// bits, and back.
__device__ __forceinline__ uint32_t row_code(int dy, int dz) {
  return (uint32_t)((dy + 3) + 7 * (dz + 3)) << kListSpan;
}
__device__ __forceinline__ void row_of(uint32_t y, int& dy, int& dz) {
  const int rc = (int)(y >> kListSpan);
  dz = rc / 7 - 3;
  dy = rc - 7 * (dz + 3) - 3;
}

// ---------------------------------------------------------------- build --
// One lane per target: the rows of its stencil of reach R (one cell beyond
// the cells' own: the list also serves the pass at n+1/2) cut to the list
// radius rl, every candidate tested against rl (eligible: a fluid target
// takes every particle, a wall target fluid ones; not itself), the hits of a
// row collected in 64-candidate masks over the row's window and written as
// chunks of kListSpan.  More chunks than the buffer holds make the target's
// count kListWalk (the passes then walk its cells).
template <int DIM, int R>
__global__ __launch_bounds__(kBlock) void k_build_list(
    KParams kp, int64_t n, const float4* __restrict__ pr, const uint32_t* __restrict__ key,
    const uint32_t* __restrict__ cstart, const uint8_t* __restrict__ type,
    const ListHeader* __restrict__ lh, uint32_t cap, uint32_t* __restrict__ count,
    uint2* __restrict__ chunks) {
  const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  // the list radius: the support with the walk's margin, plus the skin
  const float rl = __builtin_amdgcn_sqrtf(kp.support2_f) * 1.0001f + lh->skin;
  const float rl2 = rl * rl;
  if (is_excluded(type[i])) {
    count[i] = 0u;
    return;
  }
  const float4 pa = pr[i];
  const bool fa = pa.w > 0.f;
  int cx, cy, cz;
  {
    const uint32_t k = key[i];
    cx = (int)(k % (uint32_t)kp.ncx);
    const uint32_t rest = k / (uint32_t)kp.ncx;
    cy = (int)(rest % (uint32_t)kp.ncy);
    cz = (int)(rest / (uint32_t)kp.ncy);
  }
  const float cs = kp.cs_f;
  const uint32_t xa = __float_as_uint(pa.x);
  const int fcells = kFrameCells << kp.lg_xsub;
  const float fx =
      (float)(int32_t)(xa - ((uint32_t)(cx % fcells) << (29 - kp.lg_xsub))) * kp.unit_x_f;
  const int reach = R * kp.x_sub;
  const int xlo = cx - reach < 0 ? 0 : cx - reach;
  const int xhi = cx + reach >= kp.ncx ? kp.ncx - 1 : cx + reach;
  const uint32_t oi = (uint32_t)i * 16u;  // the target's own byte offset
  // chunk c of target i sits at c n + i: a wave's chunk accesses are coalesced
  uint2* out = chunks + i;
  uint32_t nc = 0;
  const int zlo = DIM == 3 ? -R : 0, zhi = DIM == 3 ? R : 0;
  for (int dz = zlo; dz <= zhi; ++dz) {
    const int z = cz + dz;
    if (z < 0 || z >= kp.ncz) continue;
    const float ez0 = (float)dz * cs - pa.z;
    const float ez = dz > 0 ? ez0 : (dz < 0 ? -(ez0 + cs) : 0.f);
    for (int dy = -R; dy <= R; ++dy) {
      const int y = cy + dy;
      if (y < 0 || y >= kp.ncy) continue;
      const float ey0 = (float)dy * cs - pa.y;
      const float ey = dy > 0 ? ey0 : (dy < 0 ? -(ey0 + cs) : 0.f);
      const float w2 = rl2 - ey * ey - ez * ez;
      if (!(w2 > 0.f)) continue;
      const float w = __builtin_amdgcn_sqrtf(w2);
      int x0 = cx + (int)floorf((fx - w) * kp.inv_csx_f);
      int x1 = cx + (int)floorf((fx + w) * kp.inv_csx_f);
      x0 = x0 < xlo ? xlo : x0;
      x1 = x1 > xhi ? xhi : x1;
      const uint32_t row = (uint32_t)kp.ncx * ((uint32_t)y + (uint32_t)kp.ncy * (uint32_t)z);
      const float ys = row_shift(pa.y, dy, cs), zs = row_shift(pa.z, dz, cs);
      const uint32_t r0 = at32(cstart, row + x0) * 16u;
      const uint32_t r1 = at32(cstart, row + x1 + 1) * 16u;
      const uint32_t rc = row_code(dy, dz);
      // the row's window in segments of up to 64 candidates, each tested in
      // groups of 4 with their loads in flight together (the views are
      // padded, so a group may read up to 3 entries past the window)
      for (uint32_t o0 = r0; o0 < r1; o0 += 64u * 16u) {
        const uint32_t o1 = r1 - o0 > 64u * 16u ? o0 + 64u * 16u : r1;
        uint64_t m = 0;
        for (uint32_t o = o0; o < o1; o += 64u) {
          float4 pb[4];
          pb[0] = at_byte<0>(pr, o);
          pb[1] = at_byte<1>(pr, o);
          pb[2] = at_byte<2>(pr, o);
          pb[3] = at_byte<3>(pr, o);
          uint32_t nib = 0;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            float dx, ddy, ddz;
            const float r2 = pair_geom<DIM>(kp, xa, ys, zs, pb[u], dx, ddy, ddz);
            const uint32_t ou = o + 16u * u;
            const bool hit = (fa || pb[u].w > 0.f) && r2 < rl2 && ou != oi && ou < o1;
            nib |= (hit ? 1u : 0u) << u;
          }
          m |= (uint64_t)nib << ((o - o0) >> 4);
        }
        const uint32_t jw = o0 >> 4;
        while (m) {
          const uint32_t f = (uint32_t)__builtin_ctzll(m);
          const uint32_t bits = (uint32_t)(m >> f) & kListSpanMask;
          m &= ~((uint64_t)kListSpanMask << f);
          if (nc < cap) out[(size_t)nc * n] = make_uint2(jw + f, bits | rc);
          ++nc;
        }
      }
    }
  }
  count[i] = nc > cap ? kListWalk : nc;
}

// ------------------------------------------------------------------ replay --
// The interaction over the list.  REUSE: the view was refreshed on the cells
// of the list's binning (the pass at n+1/2): rows of the whole reach R =
// cell_div + 1 are replayed, and if twice the recorded displacement exceeds
// the skin, or the list belongs to another binning, every target walks its
// cells with reach R and the cut widened by the displacement.  Otherwise
// (the pass on the binning's own view) chunks of rows beyond the cells'
// reach cell_div are skipped -- they hold no pair within 2h -- so the pairs
// and their order are those of the cell walk of reach cell_div.  Targets
// whose list did not fit walk their cells in either pass.
template <int DIM, int RW, bool DIAG, bool EQM, bool REUSE>
__global__ __launch_bounds__(kBlock) void k_interact_list(
    KParams kp, int64_t n, const float4* __restrict__ pr, const float4* __restrict__ vp,
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ cstart,
    const uint8_t* __restrict__ type, const double* __restrict__ pos64, float* __restrict__ ace,
    float* __restrict__ arho, float* __restrict__ visc, uint32_t* __restrict__ nbr,
    BlockRed* __restrict__ red, WsHeader* __restrict__ hdr, const uint32_t* __restrict__ disp,
    const uint32_t* __restrict__ count, const uint2* __restrict__ chunks,
    const ListHeader* __restrict__ lh, uint32_t cap) {
  const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  float fmag = 0.f, vmax_out = 0.f;
  uint32_t cnt_out = 0, cnt_wall = 0, nfl = 0;
  const float skin = lh->skin;
  // a list of another binning, or built for a buffer of another capacity,
  // is not used
  const bool stale = lh->bin_gen != hdr->bin_gen || lh->cap != cap;
  const float delta = read_displacement(disp);
  bool walk_all = stale;
  float cull2 = kp.support2_f * 1.0002f;
  if (REUSE) {
    const float rc = __builtin_amdgcn_sqrtf(kp.support2_f) * 1.0001f + delta;
    cull2 = rc * rc;
    walk_all = walk_all || !(2.f * delta <= skin);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (!(2.f * delta < kp.cs_f)) set_error(&hdr->err, SPH_ERR_MARGIN);
      if (walk_all) atomicAdd(&hdr->list_walks, 1u);
      // the skin the next list should have: 1.5 times what this pass needed
      hdr->skin_hint = __float_as_uint(3.f * delta);
    }
  } else if (blockIdx.x == 0 && threadIdx.x == 0) {
    // the binning's view, but particles moved since (a predictor ran)
    if (delta > 0.f) set_error(&hdr->err, SPH_ERR_MARGIN);
    if (stale) atomicAdd(&hdr->list_walks, 1u);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && stale) set_error(&hdr->err, SPH_ERR_LIST);
  if (i < n) {
    if (!is_excluded(type[i]) && (kp.boundary == 0 || is_fluid(type[i]))) {
      PairAcc acc{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0u};
      TargetData T{false, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, false, 0.f};
      uint32_t c64 = 0;
      const float4 pa = pr[i], va = vp[i];
      T.fluid = pa.w > 0.f;
      T.rho = fabsf(pa.w);
      T.irho = __builtin_amdgcn_rcpf(T.rho);
      T.ik = kp.kvc_f * T.irho;
      T.p = va.w;
      T.vx = va.x;
      T.vy = va.y;
      T.vz = va.z;
      const uint32_t nch = count[i];
      if (walk_all || nch == kListWalk) {
        const uint32_t k = key[i];
        const int cx = (int)(k % (uint32_t)kp.ncx);
        const uint32_t rest = k / (uint32_t)kp.ncx;
        const int cy = (int)(rest % (uint32_t)kp.ncy);
        const int cz = (int)(rest / (uint32_t)kp.ncy);
        gather_walk<DIM, RW, DIAG, EQM, false, false>(kp, 0u, n, i, pa, T, cx, cy, cz, pr, vp,
                                                      cstart, pos64, acc, c64, cull2);
        if (T.fluid) acc.cnt -= 1u;  // the walk's self pair: counted, added nothing
      } else {
        double pa64[3] = {0.0, 0.0, 0.0};
        if (DIAG)
          for (int d = 0; d < DIM; ++d) pa64[d] = pos64[d * n + i];
        const uint32_t xa = __float_as_uint(pa.x);
        const float cs = kp.cs_f;
        const uint2* L = chunks + i;
        // the chunk stream: `nx` is the next chunk, loaded one step ahead
        uint32_t c = 0, m = 0, jb = 0;
        float ys = 0.f, zs = 0.f;
        uint2 nx = nch > 0 ? L[0] : make_uint2(0u, 0u);
        const size_t ls = (size_t)n;
        // up to 4 listed candidates per round, their loads in flight together
        while (true) {
          uint32_t js[4];
          float ysu[4], zsu[4];
          bool vu[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            while (m == 0 && c < nch) {
              // take the prefetched chunk, fetch the one after it
              const uint2 ch = nx;
              ++c;
              if (c < nch) nx = L[c * ls];
              int dy, dz;
              row_of(ch.y, dy, dz);
              if (!REUSE && (dy > kp.cell_div || dy < -kp.cell_div || dz > kp.cell_div ||
                             dz < -kp.cell_div))
                continue;  // a row beyond the cells' reach: no pair within 2h
              jb = ch.x;
              m = ch.y & kListSpanMask;
              ys = row_shift(pa.y, dy, cs);
              zs = row_shift(pa.z, dz, cs);
            }
            vu[u] = m != 0;
            js[u] = jb + (uint32_t)__builtin_ctz(m | 0x80000000u);
            m &= m - 1u;
            m = vu[u] ? m : 0u;
            ysu[u] = ys;
            zsu[u] = zs;
          }
          if (!vu[0]) break;
          float4 pb[4], vb[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t o = (vu[u] ? js[u] : js[0]) * 16u;
            pb[u] = at_byte<0>(pr, o);
            vb[u] = at_byte<0>(vp, o);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (!vu[u]) continue;
            float dx, dy, dz;
            const float r2 = pair_geom<DIM>(kp, xa, ysu[u], zsu[u], pb[u], dx, dy, dz);
            if (r2 < kp.support2_f) pair_terms<DIM, EQM, false>(kp, T, dx, dy, dz, r2, pb[u].w,
                                                                vb[u], acc);
            if (DIAG && pb[u].w != 0.f) {
              double r2d = 0.0;
              for (int d = 0; d < DIM; ++d) {
                const double e = __dsub_rn(pa64[d], pos64[d * n + js[u]]);
                r2d = __dadd_rn(r2d, __dmul_rn(e, e));
              }
              c64 += (r2d < kp.support2) ? 1u : 0u;
            }
          }
        }
      }
      const uint32_t nout = DIAG ? c64 : acc.cnt;
      write_target<DIM>(kp, n, i, T, acc, nout, ace, arho, visc, nbr, fmag, vmax_out, nfl);
      cnt_out = acc.cnt;
      cnt_wall = T.fluid ? 0u : acc.cnt;
    } else {
      write_zero<DIM>(n, i, ace, arho, visc, nbr);
    }
  }
  write_block_red<kBlock / 64>(fmag, vmax_out, cnt_out, cnt_wall, nfl, red, hdr);
}

// The list header before a build: the skin (the caller's minimum, or with
// `adaptive` the larger of it and the last reused-cells list pass's request,
// at most skin_max), the binning and the capacity; one thread.
__global__ void k_list_prep(ListHeader* __restrict__ lh, const WsHeader* __restrict__ hdr,
                            float skin_min, int adaptive, float skin_max, uint32_t cap) {
  if (threadIdx.x != 0) return;
  float s = skin_min;
  if (adaptive) s = fmaxf(s, fminf(__uint_as_float(hdr->skin_hint), skin_max));
  lh->skin = s;
  lh->bin_gen = hdr->bin_gen;
  lh->cap = cap;
}

hipError_t launch_build_list(const KParams& kp, int64_t n, const sph_state& s,
                             const uint32_t* key, const uint32_t* cell_start, float skin_min,
                             bool adaptive, void* list, int64_t cap, void* ws, hipStream_t st) {
  const WsLayout L = ws_layout(n);
  const ListLayout LL = list_layout(n, cap);
  WsHeader* hdr = ws_ptr<WsHeader>(ws, L.err);
  ListHeader* lh = reinterpret_cast<ListHeader*>(static_cast<char*>(list) + LL.header);
  // beyond half a cell the pass at n+1/2 could not use the cells anyway
  const float skin_max = 0.5f * kp.cs_f;
  hipLaunchKernelGGL(k_list_prep, dim3(1), dim3(64), 0, st, lh, hdr, skin_min, adaptive ? 1 : 0,
                     skin_max, (uint32_t)cap);
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  uint32_t* count = reinterpret_cast<uint32_t*>(static_cast<char*>(list) + LL.count);
  uint2* chunks = reinterpret_cast<uint2*>(static_cast<char*>(list) + LL.chunks);
  if (n > 0) {
    // the stencil of the pass at n+1/2: one cell beyond the cells' own
#define SPH_BUILD(D, RR)                                                                    \
  hipLaunchKernelGGL((k_build_list<D, RR>), dim3(grid), dim3(kBlock), 0, st, kp, n,          \
                     ws_ptr<float4>(ws, L.view_pr), key, cell_start, s.type, lh,             \
                     (uint32_t)cap, count, chunks)
    if (kp.dim == 2) {
      if (kp.cell_div == 1) SPH_BUILD(2, 2); else SPH_BUILD(2, 3);
    } else {
      if (kp.cell_div == 1) SPH_BUILD(3, 2); else SPH_BUILD(3, 3);
    }
#undef SPH_BUILD
  }
  return hipGetLastError();
}

hipError_t launch_interact_list(const KParams& kp, int64_t n, const sph_state& s,
                                const uint32_t* key, const uint32_t* cell_start,
                                const void* list, int64_t cap, float* ace, float* arho,
                                float* visc, uint32_t* nbr, uint32_t flags, void* ws,
                                hipStream_t st) {
  const WsLayout L = ws_layout(n);
  const ListLayout LL = list_layout(n, cap);
  const float4* pr = ws_ptr<float4>(ws, L.view_pr);
  const float4* vp = ws_ptr<float4>(ws, L.view_vp);
  BlockRed* red = ws_ptr<BlockRed>(ws, L.red);
  WsHeader* hdr = ws_ptr<WsHeader>(ws, L.err);
  const uint32_t* disp = ws_ptr<uint32_t>(ws, L.disp);
  const ListHeader* lh =
      reinterpret_cast<const ListHeader*>(static_cast<const char*>(list) + LL.header);
  const uint32_t* count =
      reinterpret_cast<const uint32_t*>(static_cast<const char*>(list) + LL.count);
  const uint2* chunks = reinterpret_cast<const uint2*>(static_cast<const char*>(list) + LL.chunks);
  const unsigned grid = (unsigned)L.nblk_interact;
  const bool diag = (flags & SPH_DIAG_COUNT_F64) != 0;
  const bool reuse = (flags & SPH_INTERACT_REUSE_CELLS) != 0;
  const bool eqm = kp.mass_f == kp.mass_b;
#define SPH_LIST(D, RW, G, PP, RU)                                                           \
  hipLaunchKernelGGL((k_interact_list<D, RW, G, PP, RU>), dim3(grid), dim3(kBlock), 0, st, kp, \
                     n, pr, vp, key, cell_start, s.type, s.pos, ace, arho, visc, nbr, red, hdr, \
                     disp, count, chunks, lh, (uint32_t)cap)
#define SPH_LIST_P(D, RW, G, RU) \
  if (eqm) SPH_LIST(D, RW, G, true, RU); else SPH_LIST(D, RW, G, false, RU)
#define SPH_LIST_G(D, RW, RU) \
  if (diag) SPH_LIST_P(D, RW, true, RU); else SPH_LIST_P(D, RW, false, RU)
  // the walk of targets that fall back: the cells' own reach, one more on
  // reused cells
  if (kp.dim == 2) {
    if (kp.cell_div == 1) {
      if (reuse) { SPH_LIST_G(2, 2, true); } else { SPH_LIST_G(2, 1, false); }
    } else {
      if (reuse) { SPH_LIST_G(2, 3, true); } else { SPH_LIST_G(2, 2, false); }
    }
  } else {
    if (kp.cell_div == 1) {
      if (reuse) { SPH_LIST_G(3, 2, true); } else { SPH_LIST_G(3, 1, false); }
    } else {
      if (reuse) { SPH_LIST_G(3, 3, true); } else { SPH_LIST_G(3, 2, false); }
    }
  }
#undef SPH_LIST_G
#undef SPH_LIST_P
#undef SPH_LIST
  return hipGetLastError();
}

}  // namespace sph
