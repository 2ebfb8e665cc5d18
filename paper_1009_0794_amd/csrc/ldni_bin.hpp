// ldni_bin.hpp -- LDS tables for binning work into lists with few global
// atomics (included by the kernel sources).
//
// Global atomics are the scarce resource of binning on this GPU (a few tens
// of G per second on the whole chip against hundreds of G plain stores), so a
// workgroup adds its (item, key) pairs into an LDS table keyed by the list
// they go to and touches each list's global counter once per key.
#pragma once

#include "ldni_internal.hpp"

namespace ldni {

constexpr uint32_t kBinEmpty = 0xffffffffu;
constexpr int kBinProbe = 16;
constexpr int kBinSlotBits = 10;
static_assert((1 << kBinSlotBits) == kBinSlots, "table size");

struct BinLds {
  uint32_t key[kBinSlots];  // the list (a key below 2^31), or kBinEmpty
  uint32_t a[kBinSlots];    // pairs counted; or the list position of the slot's range
  uint32_t b[kBinSlots];    // candidates counted; or pairs placed so far
  uint32_t n_rec;
};

// A wave's lanes split into runs of consecutive lanes with equal keys (key
// < 0: no entry, never in a run).  For a lane with an entry: leader = first
// lane of its run, rank = lane - leader; group = lanes in the run (valid at
// the leader).
struct LaneRuns {
  int leader;
  uint32_t rank, group;
};
__device__ __forceinline__ LaneRuns lane_runs(int key) {
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(key, 1, 64);
  const bool live = key >= 0;
  const uint64_t heads = __ballot(live && (lane == 0 || prev != key));
  const uint64_t breaks = heads | __ballot(!live);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);  // lanes 0..lane
  const uint64_t mine = heads & upto;
  LaneRuns r;
  r.leader = mine ? 63 - __clzll((long long)mine) : lane;
  r.rank = (uint32_t)(lane - r.leader);
  const uint64_t above = breaks & ~upto;
  r.group = (uint32_t)((above ? __ffsll((unsigned long long)above) - 1 : 64) - lane);
  return r;
}

__device__ __forceinline__ uint32_t bin_home(uint32_t hk) { return (hk * 2654435761u) >> (32 - kBinSlotBits); }

// The slot of key hk (claimed if new) within kBinProbe probes, else -1.
__device__ __forceinline__ int bin_insert(BinLds& h, uint32_t hk) {
  uint32_t s = bin_home(hk);
  for (int i = 0; i < kBinProbe; ++i) {
    const uint32_t prev = atomicCAS(&h.key[s], kBinEmpty, hk);
    if (prev == kBinEmpty || prev == hk) return (int)s;
    s = (s + 1) & (kBinSlots - 1);
  }
  return -1;
}

// The slot of key hk within kBinProbe probes, else -1.
__device__ __forceinline__ int bin_find(const BinLds& h, uint32_t hk) {
  uint32_t s = bin_home(hk);
  for (int i = 0; i < kBinProbe; ++i) {
    const uint32_t k = h.key[s];
    if (k == hk) return (int)s;
    if (k == kBinEmpty) return -1;
    s = (s + 1) & (kBinSlots - 1);
  }
  return -1;
}

}  // namespace ldni
