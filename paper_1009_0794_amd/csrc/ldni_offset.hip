// ldni_offset.hip -- gfx950 kernels offsetting a solid given by its LDNIs.
//
// Sec. 4.2 approximates the offset of a solid H by a distance r by the
// Minkowski sum of H with a sphere of radius r: a sphere is centred at every
// depth-normal sample of H's LDNIs, sampled into LDNIs on the same grid, and
// united with H (an inner offset, r < 0, subtracts spheres of radius |r|),
// with the Boolean operations of Sec. 4.1 and the small interval removal of
// Sec. 4.1.1.
//
// Fixed readings: the spheres of all samples of the three LDNIs are applied
// at once; a sphere hits a ray when rho^2 < r^2 (float64), at centre -/+
// sqrt(r^2 - rho^2); per ray the events are H's paired samples and the
// spheres' chord ends; events of equal float32 depth form one group, after
// which H's state is the parity of its samples so far and the spheres' state
// is "some sphere entered and not left"; a group that changes the result
// (H or S, resp. H and not S) contributes its first event (H's samples by
// index, then spheres by generating sample, enter before exit); volumes with
// (double)exit - (double)enter <= 0 or < eps are removed.  Generating samples
// are numbered over the x-, y-, z-LDNI in storage order; a sphere's sample
// gets id -1 - g.
//
// Passes: the sphere centres (one thread per pixel); binning of the spheres
// into the lists of the rays they hit (count, scan, scatter); then one wave
// per ray, twice (count, write): the ray's events go to a wave-private LDS
// buffer as 64-bit keys (orderable depth, order), window by window in depth
// when they do not fit, a bitonic sort orders them, and a sweep in chunks of
// 64 (wave prefix sums of H's parity and of the open spheres, group starts by
// a max-scan) finds the result's end points.
// Nothing is a contraction: the work is the exact chord tests and the sorts.
#pragma clang fp contract(off)

#include "ldni_internal.hpp"
#include "ldni_bin.hpp"

namespace ldni {
namespace {

constexpr int kOffBlock = 256;  // four waves, one ray each at a time
constexpr int kOffWaves = kOffBlock / 64;
constexpr uint32_t kSphereOrder = 0x80000000u;

__device__ __forceinline__ uint32_t orderable(float d) {
  uint32_t u = __float_as_uint(d);
  if (u == 0x80000000u) u = 0u;  // -0 groups with +0
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ double centre_of(const OffsetArgs& g, int b, int i) {
  return (double)(float)(g.lo[b] + ((double)i + 0.5) * g.h[b]);
}

// Centres of the spheres: one thread per pixel of each LDNI writes the
// centres of the pixel's samples (world order) at the sample's number.
__global__ __launch_bounds__(kOffBlock) void offset_centres_kernel(OffsetArgs g) {
  const int64_t npix = (int64_t)g.w * g.w;
  const int64_t t = (int64_t)blockIdx.x * kOffBlock + threadIdx.x;
  if (t >= 3 * npix) return;
  const int a = (int)(t / npix);
  const int64_t p = t - a * npix;
  const int u = (a + 1) % 3, v = (a + 2) % 3;
  const AxisArrays& ax = g.in[a];
  const uint32_t o0 = ax.offsets[p], o1 = ax.offsets[p + 1];
  if (o1 < o0 || (uint64_t)o1 > ax.n) {
    atomicOr(g.status, kStatusMismatch);
    return;
  }
  const double cu = centre_of(g, u, (int)(p % g.w)), cv = centre_of(g, v, (int)(p / g.w));
  for (uint32_t q = o0; q < o1; ++q) {
    double* c = g.centres + 3 * (g.base[a] + q);
    c[a] = g.lo[a] + (double)ax.depth[q];
    c[u] = cu;
    c[v] = cv;
  }
}

// Pixel range [i0, i1] of an image axis whose centres may lie within r of x:
// a centre c_i with |c_i - x| < r has i within [t0 - m, t1 + m] for
// t = (x -+ r - lo) / h - 0.5 and m the axis's rounding margin in pixels;
// i0 > i1 if none.
__device__ __forceinline__ void pixel_range(const OffsetArgs& g, int b, double x, int& i0, int& i1) {
  const double t0 = (x - g.r - g.lo[b]) / g.h[b] - 0.5, t1 = (x + g.r - g.lo[b]) / g.h[b] - 0.5;
  const double f0 = floor(t0 - g.margin[b]), f1 = ceil(t1 + g.margin[b]);
  i0 = f0 < 0.0 ? 0 : f0 > (double)(g.w - 1) ? g.w : (int)f0;
  i1 = f1 < 0.0 ? -1 : f1 > (double)(g.w - 1) ? g.w - 1 : (int)f1;
}

// Binning: for sphere s and image a, the rays of the pixels in its range
// that the sphere hits (rho^2 < r^2, the test of the ray pass); count
// (kScatter false) or write the sphere into those rays' lists.  A workgroup
// (256 consecutive spheres of one image, which mostly hit the same rays)
// first adds its (sphere, ray) pairs per ray into an LDS table, one addition
// per run of lanes holding the same ray, and then touches each ray's global
// counter once: the count pass adds its pairs to ray_count; the scatter pass
// reserves a range of the ray's list from ray_cursor and, in a second sweep
// over the same pairs, places each run in its slot's range with an LDS
// atomic.  A ray that finds no free slot (kBinProbe probes) is counted and
// placed run by run with global atomics; slots never free, so it misses the
// table in the second sweep as well.
template <bool kScatter>
__global__ __launch_bounds__(kOffBlock) void offset_bin_kernel(OffsetArgs g) {
  __shared__ BinLds h;
  for (int i = threadIdx.x; i < kBinSlots; i += kOffBlock) {
    h.key[i] = kBinEmpty;
    h.a[i] = 0u;
    h.b[i] = 0u;
  }
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * kOffBlock + threadIdx.x;
  const int lane = (int)__lane_id();
  int a = 0, u = 0, v = 0, ni = 0, n_my = 0, iu0 = 0, iv0 = 0;
  uint32_t s = 0;
  double pu = 0.0, pv = 0.0;
  if (t < 3 * (int64_t)g.n_spheres) {
    a = (int)(t / g.n_spheres);
    s = (uint32_t)(t - (int64_t)a * g.n_spheres);
    u = (a + 1) % 3;
    v = (a + 2) % 3;
    const double* c = g.centres + 3 * (size_t)s;
    pu = c[u];
    pv = c[v];
    int iu1, iv1;
    pixel_range(g, u, pu, iu0, iu1);
    pixel_range(g, v, pv, iv0, iv1);
    if (iu0 <= iu1 && iv0 <= iv1) {
      ni = iu1 - iu0 + 1;
      n_my = ni * (iv1 - iv0 + 1);
    }
  }
  const double r2 = g.r * g.r;
  const int64_t npix = (int64_t)g.w * g.w;
  // every lane's j-th pixel, j = 0, 1, ... while any lane has one; the ray
  // it hits (or -1) and the runs of equal rays
  auto sweep = [&](auto&& on_run) {
    for (int j = 0; __ballot(j < n_my) != 0; ++j) {
      int my = -1;
      if (j < n_my) {
        const int iu = iu0 + j % ni, iv = iv0 + j / ni;
        const double du = centre_of(g, u, iu) - pu, dv = centre_of(g, v, iv) - pv;
        if (du * du + dv * dv < r2) my = (int)(a * npix + (int64_t)iv * g.w + iu);
      }
      on_run(my, lane_runs(my));
    }
  };
  sweep([&](int my, const LaneRuns& r) {
    if (my >= 0 && r.leader == lane) {
      const int sl = bin_insert(h, (uint32_t)my);
      if (sl >= 0) atomicAdd(&h.a[sl], r.group);
      else if (!kScatter) atomicAdd(&g.ray_count[my], r.group);
    }
  });
  __syncthreads();
  for (int i = threadIdx.x; i < kBinSlots; i += kOffBlock) {
    const uint32_t k = h.key[i];
    if (k == kBinEmpty) continue;
    if (!kScatter) atomicAdd(&g.ray_count[k], h.a[i]);
    else h.a[i] = g.ray_start[k] + atomicAdd(&g.ray_cursor[k], h.a[i]);
  }
  if (!kScatter) return;
  __syncthreads();
  sweep([&](int my, const LaneRuns& r) {
    uint32_t lead_base = 0;
    if (my >= 0 && r.leader == lane) {
      const int sl = bin_find(h, (uint32_t)my);
      lead_base = sl >= 0 ? h.a[sl] + atomicAdd(&h.b[sl], r.group)
                          : g.ray_start[my] + atomicAdd(&g.ray_cursor[my], r.group);
    }
    const uint32_t base = (uint32_t)__shfl((int)lead_base, r.leader, 64);
    if (my >= 0) g.list[base + r.rank] = s;
  });
}

// One event's world-order normal and depth for a sphere g on the ray of axis
// a through (cu, cv) (exactly the arithmetic of the hit test).
struct SphereHit {
  float depth;
  float n[3];
};
// the depth alone (the count pass's small-volume test needs no normal)
__device__ __forceinline__ float sphere_depth(const OffsetArgs& g, int a, double cu, double cv, uint32_t s,
                                              bool is_exit) {
  const int u = (a + 1) % 3, v = (a + 2) % 3;
  const double* c = g.centres + 3 * (size_t)s;
  const double du = cu - c[u], dv = cv - c[v];
  const double rho2 = du * du + dv * dv;
  const double t = sqrt(g.r * g.r - rho2);
  const double z = is_exit ? c[a] + t : c[a] - t;
  return (float)(z - g.lo[a]);
}
__device__ __forceinline__ SphereHit sphere_sample(const OffsetArgs& g, int a, double cu, double cv, uint32_t s,
                                                   bool is_exit) {
  const int u = (a + 1) % 3, v = (a + 2) % 3;
  const double* c = g.centres + 3 * (size_t)s;
  const double du = cu - c[u], dv = cv - c[v];
  const double rho2 = du * du + dv * dv;
  const double t = sqrt(g.r * g.r - rho2);
  const double z = is_exit ? c[a] + t : c[a] - t;
  const double sign = g.union_op ? 1.0 : -1.0;
  const float nu = (float)(sign * (du / g.r)), nv = (float)(sign * (dv / g.r)),
              na = (float)(sign * ((z - c[a]) / g.r));
  // to world order by selects (an array indexed by the axis would live in
  // scratch memory): x, y, z are (a, u, v) for a = 0, (v, a, u) for a = 1
  // and (u, v, a) for a = 2
  SphereHit h;
  h.depth = (float)(z - g.lo[a]);
  h.n[0] = a == 0 ? na : (a == 1 ? nv : nu);
  h.n[1] = a == 0 ? nu : (a == 1 ? na : nv);
  h.n[2] = a == 0 ? nv : (a == 1 ? nu : na);
  return h;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Inclusive wave prefix sum.
__device__ __forceinline__ int wave_scan_add(int x) {
  const int lane = (int)lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  return x;
}

__device__ __forceinline__ int wave_scan_max(int x) {
  const int lane = (int)lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x = max(x, y);
  }
  return x;
}

// Sort of key[0..n) ascending by one wave: a bitonic network over the next
// power of two in which every comparator puts the smaller key first (each
// merge of blocks of k starts with a mirrored stage, pairing blk + r with
// blk + k - 1 - r, followed by half-cleaners).  Keys beyond n count as
// larger than all, so no comparator ever moves them: comparators that reach
// beyond n are skipped, blocks wholly beyond n are not visited, and nothing
// beyond n is read or written.  A lane takes up to four comparators of a
// stage at a time, loading all of them before storing any (the comparators
// of a stage are disjoint), so their LDS round trips overlap.
__device__ __forceinline__ void wave_sort(uint64_t* key, uint32_t n) {
  const uint32_t lane = lane_id();
  constexpr int kPairs = 4;
  auto stage = [&](uint32_t pairs, auto&& pair_of) {
    for (uint32_t h0 = lane; h0 < pairs; h0 += 64 * kPairs) {
      uint64_t x[kPairs], y[kPairs];
      uint32_t lo[kPairs], hi[kPairs];
      bool act[kPairs];
#pragma unroll
      for (int j = 0; j < kPairs; ++j) {
        const uint32_t h = h0 + 64u * j;
        pair_of(h, lo[j], hi[j]);
        act[j] = h < pairs && hi[j] < n;
        if (act[j]) {
          x[j] = key[lo[j]];
          y[j] = key[hi[j]];
        }
      }
#pragma unroll
      for (int j = 0; j < kPairs; ++j) {
        if (act[j] && x[j] > y[j]) {
          key[lo[j]] = y[j];
          key[hi[j]] = x[j];
        }
      }
    }
    wave_sync();
  };
  for (uint32_t lk = 1; (1u << (lk - 1)) < n; ++lk) {  // blocks of k = 2^lk
    const uint32_t k = 1u << lk, hk = k >> 1;
    stage(((n + k - 1) >> lk) << (lk - 1), [&](uint32_t h, uint32_t& lo, uint32_t& hi) {
      const uint32_t blk = (h >> (lk - 1)) << lk, r = h & (hk - 1);
      lo = blk + r;
      hi = blk + k - 1 - r;
    });
    for (uint32_t lj = lk - 1; lj-- > 0;) {  // half-cleaners, j = 2^lj = k/4 .. 1
      const uint32_t jj = 1u << lj;
      stage(((n + 2 * jj - 1) >> (lj + 1)) << lj, [&](uint32_t h, uint32_t& lo, uint32_t& hi) {
        lo = ((h >> lj) << (lj + 1)) + (h & (jj - 1));
        hi = lo + jj;
      });
    }
  }
}

// The orderable depth of the event of the given rank (0-based) among
// key[0..n) by one wave: a radix select over the 32 depth bits, five bits a
// pass, with a 32-bin histogram in hist (32 words of the wave's own).
// A cut window keeps fewer than kOffsetKeep events and then takes one more
// step of the sphere loop (two events per lane).
static_assert(kOffsetKeep + 128 <= kOffsetBuf, "a cut window takes one more step of 128 events");
// a sweep step appends up to 64 end points after a flush that leaves one
static_assert(kOffsetEmit >= 65, "the emit buffer takes one step after a flush");
// a ray's kept end points are expanded by one wave, one per lane
static_assert(kOffsetSavedMax <= 64, "kept end points are written one per lane");
__device__ __forceinline__ uint32_t select_depth(const uint64_t* key, uint32_t n, uint32_t rank, uint32_t* hist) {
  const uint32_t lane = lane_id();
  uint32_t prefix = 0, mask = 0;
  for (int hi = 32; hi > 0; hi -= 5) {
    const int lo = hi > 5 ? hi - 5 : 0;
    const uint32_t digit_mask = (1u << (hi - lo)) - 1u;
    if (lane < 32) hist[lane] = 0;
    wave_sync();
    for (uint32_t q = lane; q < n; q += 64) {
      const uint32_t d = (uint32_t)(key[q] >> 32);
      if ((d & mask) == prefix) atomicAdd(&hist[(d >> lo) & digit_mask], 1u);
    }
    wave_sync();
    const uint32_t c = lane < 32 ? hist[lane] : 0u;
    const uint32_t cum = (uint32_t)wave_scan_add((int)c);
    const uint64_t over = __ballot(cum > rank);
    const int bucket = __ffsll((unsigned long long)over) - 1;
    rank -= __shfl(cum - c, bucket);
    prefix |= (uint32_t)bucket << lo;
    mask |= digit_mask << lo;
    wave_sync();
  }
  return prefix;
}

// Writes the result sample of event key k (a sample of the solid, or a
// sphere's chord end) of ray (a, p) at output position o.
__device__ __forceinline__ void write_event(const OffsetArgs& g, int a, int64_t p, double cu, double cv, uint64_t k,
                                            size_t o) {
  if (!(k & kSphereOrder)) {
    const uint32_t hq = g.in[a].offsets[p] + (uint32_t)(k & 0x7fffffffu);
    g.out_depth[a][o] = g.in[a].depth[hq];
    g.out_normal[a][3 * o] = g.in[a].normal[3 * (size_t)hq];
    g.out_normal[a][3 * o + 1] = g.in[a].normal[3 * (size_t)hq + 1];
    g.out_normal[a][3 * o + 2] = g.in[a].normal[3 * (size_t)hq + 2];
    g.out_tri[a][o] = g.in[a].tri[hq];
  } else {
    const uint32_t sph = (uint32_t)((k & 0x7fffffffu) >> 1);
    const SphereHit h = sphere_sample(g, a, cu, cv, sph, (k & 1u) != 0);
    g.out_depth[a][o] = h.depth;
    g.out_normal[a][3 * o] = h.n[0];
    g.out_normal[a][3 * o + 1] = h.n[1];
    g.out_normal[a][3 * o + 2] = h.n[2];
    g.out_tri[a][o] = -1 - (int32_t)sph;
  }
}

// The per-ray pass: counts (kWrite false) or writes the ray's result.  The
// ray's events are taken in windows of depth: a window collects the events
// at or after its lower depth bound into a buffer of kOffsetBuf keys; when a
// chunk would not fit, the buffer is sorted and cut back to the events
// before the depth of its kOffsetKeep-th smallest, which becomes the
// window's (exclusive) upper bound.  Windows end between groups of equal
// depth, and the sweep carries H's parity, the open spheres and the result
// state from one window to the next.
template <bool kWrite>
__global__ __launch_bounds__(kOffBlock) void offset_ray_kernel(OffsetArgs g) {
  __shared__ uint64_t s_key[kOffWaves][kOffsetBuf];
  __shared__ uint64_t s_emit[kOffWaves][kOffsetEmit];
  __shared__ uint32_t s_rbit[kOffWaves][kOffsetBuf / 32];
  __shared__ uint32_t s_hist[kOffWaves][32];

  const int wv = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  const int64_t npix = (int64_t)g.w * g.w;
  // Waves take the deep rays first (workgroups start in index order, so the
  // longest rays do not end up as the launch's tail), then every ray in
  // order, skipping the deep ones.
  const int64_t wave_no = (int64_t)blockIdx.x * kOffWaves + wv;
  int64_t ray;
  if (wave_no < (int64_t)g.n_deep) {
    ray = g.deep[wave_no];
  } else {
    ray = wave_no - g.n_deep;
    if (ray >= 3 * npix) return;
    if (g.n_deep > 0 && g.ray_start[ray + 1] - g.ray_start[ray] > (uint32_t)kOffsetDeep) return;
  }
  const int a = (int)(ray / npix);
  const int64_t p = ray - a * npix;
  const int u = (a + 1) % 3, v = (a + 2) % 3;
  const int iu = (int)(p % g.w), iv = (int)(p / g.w);
  const double cu = centre_of(g, u, iu), cv = centre_of(g, v, iv);
  uint64_t* key = s_key[wv];
  uint64_t* emit = s_emit[wv];
  uint32_t* rbit = s_rbit[wv];
  const AxisArrays& H = g.in[a];

  // the write pass's slot of the ray: out .. out + cnt
  uint32_t out = 0, cnt = 0;
  if (kWrite) {
    out = g.out_offsets[a][p];
    cnt = g.out_offsets[a][p + 1] - out;
    if (cnt == 0) return;
    // a ray whose end points the count pass kept: expand them
    if (g.saved && cnt <= g.n_saved) {
      if (lane < cnt) write_event(g, a, p, cu, cv, g.saved[(size_t)ray * g.n_saved + lane], (size_t)out + lane);
      return;
    }
  }
  const uint32_t o0 = H.offsets[p], o1 = H.offsets[p + 1];
  uint32_t nh = 0;
  if (o1 < o0 || (uint64_t)o1 > H.n) {
    if (lane == 0) atomicOr(g.status, kStatusMismatch);
  } else {
    nh = (o1 - o0) & ~1u;
  }
  const uint32_t l0 = g.ray_start[ray], l1 = g.ray_start[ray + 1];
  const double r2 = g.r * g.r;

  uint32_t lower = 0;        // window: orderable depth >= lower ...
  bool more = true;          // ... and, if bounded, < upper
  int carry_h = 0, carry_s = 0;
  bool prev_res = false;
  uint32_t n_emit = 0;
  uint32_t kept = 0;         // end-point pairs kept so far
  uint32_t big = 0xffffffffu;  // a depth whose group was found larger than a window
  auto depth_of = [&](uint64_t k) -> float {
    if (!(k & kSphereOrder)) return H.depth[o0 + (uint32_t)(k & 0x7fffffffu)];
    return sphere_depth(g, a, cu, cv, (uint32_t)((k & 0x7fffffffu) >> 1), (k & 1u) != 0);
  };
  // Small interval removal over the first np end-point pairs of emit, which
  // are then counted or written (pairs are independent volumes, so the
  // emitted end points are taken in batches); an unpaired last end point
  // moves to the front.
  auto flush = [&](uint32_t np) {
    for (uint32_t m0 = 0; m0 < np; m0 += 64) {
      const uint32_t m = m0 + lane;
      bool keep = false;
      uint64_t ea = 0, eb = 0;
      if (m < np) {
        ea = emit[2 * m];
        eb = emit[2 * m + 1];
        const double th = (double)depth_of(eb) - (double)depth_of(ea);
        keep = th > 0.0 && th >= g.eps;
      }
      const uint64_t km = __ballot(keep);
      const uint32_t rank = kept + (uint32_t)__popcll(km & ((1ull << lane) - 1ull));
      // the sweep is deterministic, so the write pass keeps what the count
      // pass counted; a disagreement (checked at the end) never writes
      // outside the ray's slot
      if (kWrite && keep && 2 * rank + 1 < cnt) {
        write_event(g, a, p, cu, cv, ea, (size_t)out + 2 * rank);
        write_event(g, a, p, cu, cv, eb, (size_t)out + 2 * rank + 1);
      }
      if (!kWrite && keep && g.saved && 2 * rank + 1 < g.n_saved) {
        g.saved[(size_t)ray * g.n_saved + 2 * rank] = ea;
        g.saved[(size_t)ray * g.n_saved + 2 * rank + 1] = eb;
      }
      kept += (uint32_t)__popcll(km);
    }
    wave_sync();
    const uint32_t rest = n_emit - 2 * np;
    if (rest > 0 && lane == 0) emit[0] = emit[2 * np];
    n_emit = rest;
    wave_sync();
  };
  while (more) {
    if (big == lower) {
      // The group of equal depth `big`, from its sums over all the ray's
      // events: H's samples in it, the spheres entering minus those leaving
      // in it, and its first event (the smallest key).  The result state
      // after the group against the one before decides whether it emits,
      // exactly as the sweep decides for a group inside a window.
      uint32_t ch = 0;
      int cs = 0;
      uint64_t first = ~0ull;
      for (uint32_t k0 = 0; k0 < nh; k0 += 64) {
        const uint32_t k = k0 + lane;
        if (k < nh && orderable(H.depth[o0 + k]) == big) {
          ++ch;
          first = min(first, ((uint64_t)big << 32) | k);
        }
      }
      for (uint32_t base = l0; base < l1; base += 64) {
        const uint32_t e = base + lane;
        if (e < l1) {
          const uint32_t sph = g.list[e];
          const double* c = g.centres + 3 * (size_t)sph;
          const double du = cu - c[u], dv = cv - c[v];
          const double rho2 = du * du + dv * dv;
          if (rho2 < r2) {
            const double t = sqrt(r2 - rho2);
            const float d0 = (float)((c[a] - t) - g.lo[a]), d1 = (float)((c[a] + t) - g.lo[a]);
            if (orderable(d0) == big) {
              ++cs;
              first = min(first, ((uint64_t)big << 32) | kSphereOrder | (sph << 1));
            }
            if (orderable(d1) == big) {
              --cs;
              first = min(first, ((uint64_t)big << 32) | kSphereOrder | (sph << 1) | 1u);
            }
          }
        }
      }
      for (int d = 32; d >= 1; d >>= 1) {
        ch += (uint32_t)__shfl_xor((int)ch, d, 64);
        cs += __shfl_xor(cs, d, 64);
        const uint64_t o = __shfl_xor(first, d, 64);
        first = min(first, o);
      }
      carry_h += (int)ch;
      carry_s += cs;
      const bool res = g.union_op ? ((carry_h & 1) != 0 || carry_s > 0) : ((carry_h & 1) != 0 && carry_s <= 0);
      if (res != prev_res) {
        if (n_emit + 1 > (uint32_t)kOffsetEmit) flush(n_emit / 2);
        if (lane == 0) emit[n_emit] = first;
        ++n_emit;
        wave_sync();
      }
      prev_res = res;
      more = big != 0xffffffffu;
      lower = big + 1u;
      big = 0xffffffffu;
      continue;
    }
    uint32_t upper = 0;
    bool bounded = false;
    uint32_t n = 0;
    // append up to two events per lane (keys k0, k1; has0, has1) after filtering
    auto append = [&](uint64_t k0, bool has0, uint64_t k1, bool has1) {
      auto in_window = [&](uint64_t k) {
        const uint32_t d = (uint32_t)(k >> 32);
        return d >= lower && (!bounded || d < upper);
      };
      bool h0 = has0 && in_window(k0), h1 = has1 && in_window(k1);
      uint32_t total = (uint32_t)__popcll(__ballot(h0)) + (uint32_t)__popcll(__ballot(h1));
      if (n + total > (uint32_t)kOffsetBuf) {
        // the depth of the kOffsetKeep-th smallest event becomes the bound;
        // the events before it are compacted to the front (unsorted)
        const uint32_t cut = select_depth(key, n, (uint32_t)kOffsetKeep, s_hist[wv]);
        uint32_t m = 0;
        for (uint32_t c0 = 0; c0 < n; c0 += 64) {
          const uint32_t q = c0 + lane;
          const uint64_t kq = q < n ? key[q] : 0ull;
          const bool keep = q < n && (uint32_t)(kq >> 32) < cut;
          const uint64_t bal = __ballot(keep);
          if (keep) key[m + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull))] = kq;
          m += (uint32_t)__popcll(bal);
        }
        bounded = true;
        upper = cut;
        n = m;
        // one group of equal depth fills the window: the window ends before
        // it and the group is taken whole, by its sums, when it is reached
        if (m == 0) big = cut;
        h0 = has0 && in_window(k0);
        h1 = has1 && in_window(k1);
        wave_sync();
      }
      const uint64_t m0 = __ballot(h0), m1 = __ballot(h1);
      const uint64_t below = (1ull << lane) - 1ull;
      uint32_t pos = n + (uint32_t)__popcll(m0 & below) + (uint32_t)__popcll(m1 & below);
      if (h0) key[pos++] = k0;
      if (h1) key[pos] = k1;
      n += (uint32_t)__popcll(m0) + (uint32_t)__popcll(m1);
    };
    for (uint32_t k0 = 0; k0 < nh; k0 += 64) {
      const uint32_t k = k0 + lane;
      const bool has = k < nh;
      const uint64_t kk = has ? (((uint64_t)orderable(H.depth[o0 + k]) << 32) | k) : 0ull;
      append(kk, has, 0ull, false);
    }
    // the ray's spheres, 64 at a time; loads run ahead (list entries two
    // chunks, centres one chunk) so that a chunk's tests do not wait for them
    uint32_t sph1 = 0, sph2 = 0;
    double cu1 = 0.0, cv1 = 0.0, ca1 = 0.0;
    if (l0 + lane < l1) {
      sph1 = g.list[l0 + lane];
      const double* c = g.centres + 3 * (size_t)sph1;
      cu1 = c[u];
      cv1 = c[v];
      ca1 = c[a];
    }
    if (l0 + 64 + lane < l1) sph2 = g.list[l0 + 64 + lane];
    for (uint32_t base = l0; base < l1; base += 64) {
      const uint32_t e = base + lane;
      const uint32_t sph = sph1;
      const double pu = cu1, pv = cv1, pa = ca1;
      if (e + 64 < l1) {
        const double* c = g.centres + 3 * (size_t)sph2;
        cu1 = c[u];
        cv1 = c[v];
        ca1 = c[a];
      }
      sph1 = sph2;
      if (e + 128 < l1) sph2 = g.list[e + 128];
      bool hit = false;
      uint64_t ka = 0, kb = 0;
      if (e < l1) {
        const double du = cu - pu, dv = cv - pv;
        const double rho2 = du * du + dv * dv;
        if (rho2 < r2) {
          hit = true;
          const double t = sqrt(r2 - rho2);
          const float d0 = (float)((pa - t) - g.lo[a]), d1 = (float)((pa + t) - g.lo[a]);
          ka = ((uint64_t)orderable(d0) << 32) | kSphereOrder | (sph << 1);
          kb = ((uint64_t)orderable(d1) << 32) | kSphereOrder | (sph << 1) | 1u;
        }
      }
      append(ka, hit, kb, hit);
    }
    wave_sync();
    if (n > 0) {
      wave_sort(key, n);
      // sweep: per event H's parity and the open spheres after it; at the
      // last event of each group the result state against the one after the
      // previous group; a change emits the group's first event
      int carry_first = -1;
      const bool window_prev = prev_res;  // result state before this window
      for (uint32_t c0 = 0; c0 < n; c0 += 64) {
        const uint32_t q = c0 + lane;
        const bool valid = q < n;
        const uint64_t kq = valid ? key[q] : ~0ull;
        const bool is_h = valid && !(kq & kSphereOrder);
        const int ph = carry_h + wave_scan_add(is_h ? 1 : 0);
        const int ps = carry_s + wave_scan_add((valid && !is_h) ? ((kq & 1u) ? -1 : 1) : 0);
        const uint32_t dq = (uint32_t)(kq >> 32);
        const bool first = valid && (q == 0 || (uint32_t)(key[q - 1] >> 32) != dq);
        const bool last = valid && (q + 1 == n || (uint32_t)(key[q + 1] >> 32) != dq);
        const int fq = max(carry_first, wave_scan_max(first ? (int)q : -1));
        const bool res = g.union_op ? ((ph & 1) != 0 || ps > 0) : ((ph & 1) != 0 && ps <= 0);
        const uint64_t rm = __ballot(valid && res);
        if (lane == 0) rbit[c0 >> 5] = (uint32_t)rm;
        if (lane == 32) rbit[(c0 >> 5) + 1] = (uint32_t)(rm >> 32);
        wave_sync();
        bool e = false;
        if (last) {
          const bool prev = fq > 0 ? ((rbit[(fq - 1) >> 5] >> ((fq - 1) & 31)) & 1u) != 0 : window_prev;
          e = prev != res;
        }
        const uint64_t em = __ballot(e);
        const uint32_t ne = (uint32_t)__popcll(em);
        if (n_emit + ne > (uint32_t)kOffsetEmit) flush(n_emit / 2);  // (then at most one is left)
        if (e) emit[n_emit + (uint32_t)__popcll(em & ((1ull << lane) - 1ull))] = key[fq];
        n_emit += ne;
        carry_h = __shfl(ph, 63);
        carry_s = __shfl(ps, 63);
        carry_first = __shfl(fq, 63);
        // state after the last event so far (after the window: the next one's start)
        const int last_q = (int)min(c0 + 63, n - 1);
        const uint64_t rm_last = __shfl(rm, 0);
        prev_res = ((rm_last >> (last_q - (int)c0)) & 1ull) != 0;
      }
      wave_sync();
    }
    more = bounded;
    lower = upper;
  }
  flush(n_emit / 2);
  if (!kWrite && lane == 0) g.counts[a][p] = 2 * kept;
  // more or fewer end points than the count pass kept: slots unwritten or
  // surplus ones dropped, so the call fails
  if (kWrite && lane == 0 && 2 * kept != cnt) atomicOr(g.status, kStatusMismatch);
}

}  // namespace

hipError_t launch_offset_centres(const OffsetArgs& g, hipStream_t s) {
  const int64_t n = 3 * (int64_t)g.w * g.w;
  hipLaunchKernelGGL(offset_centres_kernel, dim3((unsigned)((n + kOffBlock - 1) / kOffBlock)), dim3(kOffBlock), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_offset_bin(const OffsetArgs& g, bool scatter, hipStream_t s) {
  const int64_t n = 3 * (int64_t)g.n_spheres;
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + kOffBlock - 1) / kOffBlock));
  if (scatter) hipLaunchKernelGGL(offset_bin_kernel<true>, grid, dim3(kOffBlock), 0, s, g);
  else hipLaunchKernelGGL(offset_bin_kernel<false>, grid, dim3(kOffBlock), 0, s, g);
  return hipGetLastError();
}

__global__ __launch_bounds__(kOffBlock) void offset_deep_kernel(OffsetArgs g) {
  const int64_t ray = (int64_t)blockIdx.x * kOffBlock + threadIdx.x;
  if (ray >= 3 * (int64_t)g.w * g.w) return;
  if (g.ray_start[ray + 1] - g.ray_start[ray] > (uint32_t)kOffsetDeep) g.deep[atomicAdd(&g.status[16], 1u)] = (uint32_t)ray;
}

hipError_t launch_offset_deep(const OffsetArgs& g, hipStream_t s) {
  const int64_t rays = 3 * (int64_t)g.w * g.w;
  hipLaunchKernelGGL(offset_deep_kernel, dim3((unsigned)((rays + kOffBlock - 1) / kOffBlock)), dim3(kOffBlock), 0, s,
                     g);
  return hipGetLastError();
}

hipError_t launch_offset_rays(const OffsetArgs& g, bool write, hipStream_t s) {
  const int64_t rays = 3 * (int64_t)g.w * g.w + g.n_deep;
  const dim3 grid((unsigned)((rays + kOffWaves - 1) / kOffWaves));
  if (write) hipLaunchKernelGGL(offset_ray_kernel<true>, grid, dim3(kOffBlock), 0, s, g);
  else hipLaunchKernelGGL(offset_ray_kernel<false>, grid, dim3(kOffBlock), 0, s, g);
  return hipGetLastError();
}

}  // namespace ldni
