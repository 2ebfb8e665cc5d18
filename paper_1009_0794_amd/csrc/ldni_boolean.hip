// ldni_boolean.hip -- gfx950 kernels of Boolean operations on two LDNIs.
//
// Sec. 4.1 (with Fig. 5) reduces a Boolean operation of two solids sampled on
// one grid to 1D work per pixel: each solid's samples bound its volumes as
// consecutive (enter, exit) pairs, and the result keeps the volumes where the
// operation holds; Sec. 4.1.1 then drops volumes thinner than eps.
//
// Each pixel is swept as a merge of its two sorted sample lists.  Events of
// equal depth form one group; a group flips a solid's inside state once per
// sample of that solid in it, and the result state is the operation of the two
// states after the group.  A group that changes the result state contributes
// one end point: A's first sample of the group if it has one, else B's (with
// its normal reversed for the difference).  So touching pieces merge, no
// zero-thickness gap or sliver can appear, and a pair's unpaired last sample
// (an odd count) is left out.  A volume is kept when its thickness
// (double)exit - (double)enter is positive and at least eps.
//
// Passes: count (the sweep: kept end points per pixel and the source of each),
// then the library's exclusive scan turns the counts into the result offsets
// in place (and finds the largest count), then write (a copy of each kept
// sample to its offset).  A wave owns 64 consecutive pixels, whose samples
// are contiguous ranges of both inputs and of the output: the count pass
// stages the depths in LDS with coalesced loads, and the write pass stores
// the output range with coalesced stores.  Nothing is a contraction; the
// passes stream the two inputs and the output (HBM).
#pragma clang fp contract(off)

#include "ldni_internal.hpp"

namespace ldni {
namespace {

constexpr int kBoolBlock = 256;
constexpr int kBoolWaves = kBoolBlock / 64;
constexpr int kBoolCap = 1024;  // depths of a wave's 64 pixels held in LDS (both inputs)
constexpr uint32_t kFromB = 0x80000000u;

__device__ __forceinline__ bool op_holds(int op, bool a, bool b) {
  return op == kBoolUnion ? (a | b) : op == kBoolIntersection ? (a & b) : (a & !b);
}

// The sweep of one pixel over na (even) depths of A and nb of B; emit(enter,
// exit) receives the two end points of each kept volume as the index of the
// sample in its pixel list, | kFromB for B's.  Returns the kept samples.
template <class Emit>
__device__ __forceinline__ uint32_t sweep(const float* da, uint32_t na, const float* db, uint32_t nb,
                                          int op, double eps, Emit&& emit) {
  uint32_t ia = 0, ib = 0, n = 0;
  bool in_a = false, in_b = false, in_r = false;
  float enter = 0.0f;
  uint32_t enter_ref = 0;
  float za = na > 0 ? da[0] : 0.0f, zb = nb > 0 ? db[0] : 0.0f;
  while (ia < na || ib < nb) {
    // the group's depth: the smaller next depth (A first on ties and for
    // values that do not compare); its first event is always taken, so
    // every pass of the loop makes progress (when B's sample comes first,
    // A has none at its depth)
    const bool take_a = ia < na && (ib >= nb || !(zb < za));
    const float d = take_a ? za : zb;
    const uint32_t ref = take_a ? ia : (ib | kFromB);  // A's first sample of the group wins
    if (take_a) {
      in_a = !in_a;
      za = ++ia < na ? da[ia] : 0.0f;
    } else {
      in_b = !in_b;
      zb = ++ib < nb ? db[ib] : 0.0f;
    }
    while (ia < na && za == d) {
      in_a = !in_a;
      za = ++ia < na ? da[ia] : 0.0f;
    }
    while (ib < nb && zb == d) {
      in_b = !in_b;
      zb = ++ib < nb ? db[ib] : 0.0f;
    }
    const bool r = op_holds(op, in_a, in_b);
    if (r == in_r) continue;
    in_r = r;
    if (r) {
      enter = d;
      enter_ref = ref;
      continue;
    }
    const double th = (double)d - (double)enter;
    if (!(th > 0.0 && th >= eps)) continue;  // small interval removal
    emit(n, enter_ref, ref);
    n += 2;
  }
  return n;
}

// One input sample of A or B, read whole before anything is stored (the
// compiler cannot reorder loads past stores to other arrays, so reading and
// storing field by field would wait for each load in turn).
struct Sample {
  float d, nx, ny, nz;
  int32_t t;
};
__device__ __forceinline__ Sample get(const BooleanArgs& g, bool from_b, uint64_t src) {
  const AxisArrays& in = from_b ? g.b : g.a;
  Sample x;
  x.d = in.depth[src];
  x.nx = in.normal[3 * src];
  x.ny = in.normal[3 * src + 1];
  x.nz = in.normal[3 * src + 2];
  x.t = in.tri[src];
  return x;
}

// Stores result sample at (output index) from a sample of A or B.
__device__ __forceinline__ void put(const BooleanArgs& g, uint64_t at, bool from_b, const Sample& x) {
  const float sign = (from_b && g.op == kBoolDifference) ? -1.0f : 1.0f;
  g.out_depth[at] = x.d;
  g.out_normal[3 * at] = sign * x.nx;
  g.out_normal[3 * at + 1] = sign * x.ny;
  g.out_normal[3 * at + 2] = sign * x.nz;
  g.out_tri[at] = from_b ? -1 - x.t : x.t;
}

// A wave takes 64 consecutive pixels.  Their samples are contiguous in both
// inputs (and their results in the output), so the wave works through them in
// batches of consecutive pixels whose samples fit in LDS: it loads a batch's
// depths of both inputs with coalesced loads (all issued before any is waited
// for) and every lane of the batch sweeps its pixel from LDS.  A single pixel
// with more samples than LDS holds is swept straight from global memory.
// Offsets that decrease, pass the sample count, or do not chain from one pixel
// to the next raise the mismatch bit and empty the wave's pixels.
struct WavePixels {
  int64_t p;        // this lane's pixel
  bool live;        // p < npix
  bool ok;          // the whole wave's offsets are a valid prefix
  int nlive;        // live lanes (a prefix of the wave)
  uint32_t a0, a1, b0, b1;
};

__device__ __forceinline__ WavePixels wave_pixels(const BooleanArgs& g, int64_t p0, bool count_pass) {
  WavePixels w;
  const int lane = threadIdx.x & 63;
  w.p = p0 + lane;
  w.live = w.p < g.npix;
  w.nlive = (int)min<int64_t>(g.npix - p0, 64);
  w.a0 = w.a1 = w.b0 = w.b1 = 0;
  bool ok = true;
  if (w.live) {
    w.a0 = g.a.offsets[w.p];
    w.a1 = g.a.offsets[w.p + 1];
    w.b0 = g.b.offsets[w.p];
    w.b1 = g.b.offsets[w.p + 1];
    ok = w.a0 <= w.a1 && w.a1 <= g.a.n && w.b0 <= w.b1 && w.b1 <= g.b.n;
    if (!ok && count_pass) atomicOr(g.status, kStatusMismatch);
  }
  // consecutive pixels must also chain (each starts where the previous ends)
  const uint32_t pa1 = (uint32_t)__shfl_up((int)w.a1, 1, 64), pb1 = (uint32_t)__shfl_up((int)w.b1, 1, 64);
  const bool chained = lane == 0 || !w.live || (pa1 == w.a0 && pb1 == w.b0);
  w.ok = __ballot(!(ok && chained)) == 0;
  return w;
}

// The next batch from lane `first`: the lanes whose samples, counted from
// lane first's, fit in kBoolCap.  Returns its last lane, or first - 1 when
// lane first alone does not fit; sets the batch's first samples and counts.
struct Batch {
  int first, last;
  uint32_t A0, B0, nA, nB;
};
__device__ __forceinline__ Batch next_batch(const WavePixels& w, int first) {
  const int lane = threadIdx.x & 63;
  Batch bt;
  bt.first = first;
  bt.A0 = (uint32_t)__shfl((int)w.a0, first, 64);
  bt.B0 = (uint32_t)__shfl((int)w.b0, first, 64);
  const uint64_t need = (uint64_t)(w.a1 - bt.A0) + (w.b1 - bt.B0);
  const uint64_t fits = __ballot(lane >= first && lane < w.nlive && need <= (uint64_t)kBoolCap);
  bt.last = fits ? 63 - __clzll((long long)fits) : first - 1;
  const int l = bt.last >= first ? bt.last : first;
  bt.nA = (uint32_t)__shfl((int)w.a1, l, 64) - bt.A0;
  bt.nB = (uint32_t)__shfl((int)w.b1, l, 64) - bt.B0;
  return bt;
}

// Loads a batch's depths (A's, then B's) into s; every load is issued before
// the stores to LDS wait for them.
__device__ __forceinline__ void load_batch(const BooleanArgs& g, const Batch& bt, float* s) {
  const int lane = threadIdx.x & 63;
  const uint32_t tot = bt.nA + bt.nB;  // <= kBoolCap
  float v[kBoolCap / 64];
#pragma unroll
  for (int k = 0; k < kBoolCap / 64; ++k) {
    const uint32_t i = (uint32_t)lane + 64u * k;
    v[k] = i < bt.nA ? g.a.depth[(uint64_t)bt.A0 + i]
                     : (i < tot ? g.b.depth[(uint64_t)bt.B0 + (i - bt.nA)] : 0.0f);
  }
#pragma unroll
  for (int k = 0; k < kBoolCap / 64; ++k) {
    const uint32_t i = (uint32_t)lane + 64u * k;
    if (i < tot) s[i] = v[k];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The count pass sweeps every pixel once: it counts the kept samples and
// records each one's source (its index in the pixel's list of A, or of B |
// kFromB) at refs[a0 + b0 + k] -- pixel p's kept samples are at most its
// input samples, so these ranges never overlap.
__global__ void __launch_bounds__(kBoolBlock) boolean_count_kernel(BooleanArgs g) {
  __shared__ float s_dep[kBoolWaves][kBoolCap];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p0 = ((int64_t)blockIdx.x * kBoolWaves + wave) * 64;
  if (p0 >= g.npix) return;
  const WavePixels w = wave_pixels(g, p0, true);
  uint32_t n = 0;
  if (w.ok) {
    const uint32_t na = (w.a1 - w.a0) & ~1u, nb = (w.b1 - w.b0) & ~1u;  // whole pairs only
    uint32_t* refs = g.refs + (uint64_t)w.a0 + w.b0;
    auto record = [&](uint32_t k, uint32_t e, uint32_t x) {
      refs[k] = e;
      refs[k + 1] = x;
    };
    float* s = s_dep[wave];
    for (int first = 0; first < w.nlive;) {
      const Batch bt = next_batch(w, first);
      if (bt.last < first) {  // one pixel deeper than LDS
        if (lane == first) n = sweep(g.a.depth + w.a0, na, g.b.depth + w.b0, nb, g.op, g.eps, record);
        first += 1;
        continue;
      }
      load_batch(g, bt, s);
      if (lane >= first && lane <= bt.last)
        n = sweep(s + (w.a0 - bt.A0), na, s + bt.nA + (w.b0 - bt.B0), nb, g.op, g.eps, record);
      wave_sync();  // before the next batch replaces the depths
      first = bt.last + 1;
    }
  }
  if (w.live) g.counts[w.p] = n;
}

// The write pass copies: the wave's output range [R0, R1) is contiguous;
// output k belongs to the last of the wave's pixels whose offset is <= k
// (binary search over the 64 offsets in LDS), its source comes from refs,
// and the stores are coalesced.
__global__ void __launch_bounds__(kBoolBlock) boolean_write_kernel(BooleanArgs g) {
  __shared__ uint32_t s_o[kBoolWaves][65];
  __shared__ uint32_t s_a0[kBoolWaves][64];
  __shared__ uint32_t s_b0[kBoolWaves][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p0 = ((int64_t)blockIdx.x * kBoolWaves + wave) * 64;
  if (p0 >= g.npix) return;
  const WavePixels w = wave_pixels(g, p0, false);
  if (!w.ok) {  // inputs that changed between the passes: the call fails
    if (lane == 0) atomicOr(g.status, kStatusMismatch);
    return;
  }
  uint32_t* so = s_o[wave];
  const uint32_t o = w.live ? g.counts[w.p] : 0u;
  const uint32_t R1 = g.counts[p0 + w.nlive];
  so[lane] = w.live ? o : R1;
  if (lane == 0) so[64] = R1;
  s_a0[wave][lane] = w.a0;
  s_b0[wave][lane] = w.b0;
  wave_sync();
  const uint32_t R0 = so[0];
  for (uint32_t k0 = R0; k0 < R1; k0 += 4 * 64) {
    // four outputs per lane at a time: their loads are issued together
    uint32_t src[4];
    bool from_b[4], any[4];
    uint32_t base[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t k = k0 + (uint32_t)lane + 64u * u;
      any[u] = k < R1;
      int lo = 0, hi = w.nlive - 1;  // the pixel: last q with so[q] <= k
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (so[mid] <= k) lo = mid; else hi = mid - 1;
      }
      const uint32_t rf = any[u] ? g.refs[(uint64_t)s_a0[wave][lo] + s_b0[wave][lo] + (k - so[lo])] : 0u;
      from_b[u] = (rf & kFromB) != 0;
      base[u] = from_b[u] ? s_b0[wave][lo] : s_a0[wave][lo];
      src[u] = rf & ~kFromB;
    }
    // the four samples' reads, all issued before the stores
    Sample x[4];
    bool ok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t si = (uint64_t)base[u] + src[u];
      ok[u] = any[u] && si < (from_b[u] ? g.b.n : g.a.n);
      if (any[u] && !ok[u]) atomicOr(g.status, kStatusMismatch);  // inputs changed between the passes
      if (ok[u]) x[u] = get(g, from_b[u], si);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (ok[u]) put(g, k0 + (uint32_t)lane + 64u * u, from_b[u], x[u]);
  }
}

}  // namespace

hipError_t launch_boolean(const BooleanArgs& g, bool write, hipStream_t s) {
  if (g.npix <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((g.npix + kBoolBlock - 1) / kBoolBlock);  // 64 pixels per wave
  if (write)
    hipLaunchKernelGGL(boolean_write_kernel, dim3(blocks), dim3(kBoolBlock), 0, s, g);
  else
    hipLaunchKernelGGL(boolean_count_kernel, dim3(blocks), dim3(kBoolBlock), 0, s, g);
  return hipGetLastError();
}

}  // namespace ldni
