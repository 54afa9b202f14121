// Slot lookups of batched cases (continuous batching): slot s owns the packed
// particles [off_s, off_s + n_s) and, in the interaction, the lanes
// [loff_s, loff_s + n_s lpt_s); slots are in particle (and lane) order.
#pragma once
#include "sph_internal.h"

namespace sph {

// The slot owning packed particle i: the last slot with off <= i (slots are
// in particle order; an empty slot shares its offset with the next one).
__device__ inline int find_slot(const SlotEntry* __restrict__ tab, int ns, int64_t i) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].off <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The slot owning interaction lane t (slots are in lane order as well).
__device__ inline int find_slot_lane(const SlotEntry* __restrict__ tab, int ns, int64_t t) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].loff <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The slots of the block's first and last particle (LANES: interaction
// lane) -- uniform over the block; -1, -1 for a block wholly past n.  Slots
// are in particle (and lane) order, so equal values mean the whole block
// lies in one slot.
template <bool LANES = false>
__device__ inline int2 block_slots(const SlotEntry* __restrict__ tab, int ns, int64_t n,
                                   int64_t first) {
  if (first >= n) return make_int2(-1, -1);
  const int64_t last = first + kBlock - 1 < n ? first + kBlock - 1 : n - 1;
  const int s0 = LANES ? find_slot_lane(tab, ns, first) : find_slot(tab, ns, first);
  const int s1 = LANES ? find_slot_lane(tab, ns, last) : find_slot(tab, ns, last);
  return make_int2(__builtin_amdgcn_readfirstlane(s0), __builtin_amdgcn_readfirstlane(s1));
}

}  // namespace sph
