// ldni_kernels.hip -- gfx950 kernels of the LDNI sampler.
//
// Pipeline per call (every kernel covers all requested axes in one launch):
//   setup      triangle-parallel: gather and validate vertices, float64 face
//              normal, candidate pixel rectangle on each image, and the count
//              of entries and candidate pixels of every screen tile it meets
//   tile scan  entry counts -> tile-list offsets; candidate counts -> each
//              tile's region of the staging buffer
//   bin_scatter  triangle ids into per-tile lists
//   sample     one workgroup per tile: exact coverage test of every candidate
//              (triangle, pixel centre); the hits' float64 depth, (depth,
//              triangle) key and arrival slot in their pixel are staged in the
//              tile's region, per-pixel counts -> counts[w*w]
//   scan       counts -> offsets[w*w+1]
//   plan       place items (a tile's pixels split into runs that fit in LDS)
//   place      one workgroup per item: the staged keys of a run are put at
//              their pixel slots in LDS, ranked within the pixel and stored as
//              depth, normal and triangle id; a pixel deeper than LDS is
//              stored unsorted and sorted in place
//   walk       tiles whose hits did not fit their region: walked again and
//              written directly
// Nothing here is a dense contraction, so there is no MFMA: the work is
// integer/FP64 ALU plus HBM traffic.
#pragma clang fp contract(off)

#include <type_traits>

#include "ldni_internal.hpp"
#include "ldni_bin.hpp"

namespace ldni {
namespace {

constexpr int kBlock = 256;          // 4 wave64 per workgroup
// runs of place items per XCD (xcd_runs): the items of a tile split into
// several read the same staged lines.  (Runs of neighbouring tiles in the
// sampling pass line up with the rows of tiles and give some XCDs the dense
// columns of an image.)
constexpr uint32_t kPlaceRun = 16;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxTilePix = 1024;    // tw * th
constexpr int kMaxTileW = 256;
constexpr int kMaxTileH = 64;
// Two builds of the tile kernels: tiles of up to 256 pixels (less LDS, more
// workgroups per CU) and of up to 1024 pixels; the stage holds the (depth,
// triangle) keys of one run of pixels.
constexpr int kSmallTilePix = 256;
__host__ __device__ constexpr int stage_cap(int tile_pix) { return tile_pix <= 256 ? 2048 : 4096; }

// ---------------------------------------------------------------------------
// pixel centres and candidate rectangles
// ---------------------------------------------------------------------------
__device__ __forceinline__ float pixel_centre(double lo, double h, int i) {
  return (float)(lo + ((double)i + 0.5) * h);
}

// Smallest i in [0, w] whose centre is >= x (centres are non-decreasing in i).
// The float64 estimate is exact when it is farther than slack from every
// integer; otherwise it is corrected against the exact float32 centres.
__device__ int first_centre_at_or_above(double lo, double h, double inv_h, double slack, int w, float x) {
  const double t = ((double)x - lo) * inv_h - 0.5;
  if (t > 0.0 && t < (double)w) {
    const double c = ceil(t);
    if (c - t > slack && c - t < 1.0 - slack) return (int)c;
  }
  int i;
  if (!(t > 0.0)) i = 0;
  else if (t >= (double)w) i = w;
  else i = (int)ceil(t);
  while (i > 0 && pixel_centre(lo, h, i - 1) >= x) --i;
  while (i < w && pixel_centre(lo, h, i) < x) ++i;
  return i;
}

// ---------------------------------------------------------------------------
// exact coverage
// ---------------------------------------------------------------------------
// Orientation of the ray with respect to the directed edge P->Q, both
// endpoints already translated into the ray frame.  The two products of
// float32 values are exact in float64, so the sign of the difference is exact.
// A ray exactly on the edge line is decided as if displaced by (+eps, +eps^2).
__device__ __forceinline__ int orient(float pu, float pv, float qu, float qv, double& e) {
  e = (double)pu * (double)qv - (double)pv * (double)qu;
  int s = (e > 0.0) - (e < 0.0);
  if (s == 0) s = (pv > qv) - (pv < qv);
  if (s == 0) s = (qu > pu) - (qu < pu);
  return s;
}

// Approximate normal sampling (Sec. 3): each component c of the unit normal
// becomes one byte, the 8-bit colour (c + 1) / 2 rounded to nearest,
// floor((c + 1) * 127.5 + 0.5) clamped to [0, 255] with float64 operations in
// that order; x | y << 8 | z << 16.
__device__ __forceinline__ uint32_t encode_rgb8(float x, float y, float z) {
  auto q = [](float c) -> uint32_t {
    const double t = floor(((double)c + 1.0) * 127.5 + 0.5);
    return (uint32_t)fmin(fmax(t, 0.0), 255.0);
  };
  return q(x) | (q(y) << 8) | (q(z) << 16);
}

// The normal of output sample o, as three floats or as its 8-bit code.
__device__ __forceinline__ void store_normal(const Image& im, size_t o, float x, float y, float z) {
  if (im.normal_rgb8 != nullptr) {
    im.normal_rgb8[o] = encode_rgb8(x, y, z);
  } else {
    float* dst = im.normal + 3 * o;
    dst[0] = x;
    dst[1] = y;
    dst[2] = z;
  }
}

// (depth, triangle) as one unsigned key whose order is depth, then id.
__device__ __forceinline__ uint64_t sample_key(float d, int32_t t) {
  uint32_t b = __float_as_uint(d);
  b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return ((uint64_t)b << 32) | (uint32_t)t;
}

__device__ __forceinline__ float key_depth(uint64_t k) {
  const uint32_t b = (uint32_t)(k >> 32);
  return __uint_as_float((b & 0x80000000u) ? (b & 0x7fffffffu) : ~b);
}

// ---------------------------------------------------------------------------
// block-level helpers
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    T y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  return x;
}

// Exclusive scan over the workgroup; returns the prefix and sets total.
template <class T>
__device__ __forceinline__ T block_exclusive_scan(T x, T* s_wave, T& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T inc = wave_inclusive_scan(x);
  if (lane == 63) s_wave[wave] = inc;
  __syncthreads();
  T before = 0, sum = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    const T v = s_wave[k];
    if (k < wave) before += v;
    sum += v;
  }
  total = sum;
  __syncthreads();
  return before + inc - x;
}

__device__ __forceinline__ uint32_t block_max(uint32_t x, uint32_t* s_wave) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, d, 64));
  if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = x;
  __syncthreads();
  uint32_t m = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) m = max(m, s_wave[k]);
  __syncthreads();
  return m;
}

// Index of the segment of a prefix array (n+1 entries) that contains x.
template <class T>
__device__ __forceinline__ int segment_of(const T* start, int n, T x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Map a workgroup to (image, tile).
// Workgroups are dealt to the 8 XCDs round robin (block b to XCD b mod 8),
// each with its own L2.  This renumbering gives every XCD runs of R
// consecutive work items, the runs themselves dealt round robin: items that
// read the same lines share an L2 while the load stays spread.  A bijection
// on [0, n).
template <uint32_t R>
__device__ __forceinline__ uint32_t xcd_runs(uint32_t b, uint32_t n) {
  const uint32_t full = n - n % (8u * R);
  if (b >= full) return b;
  const uint32_t x = b & 7u, s = b >> 3;
  return ((s / R) * 8u + x) * R + s % R;
}

__device__ __forceinline__ int image_of_block(const ImageSet& set, uint32_t b) {
  int k = 0;
  while (k + 1 < set.n && b >= set.tile_start[k + 1]) ++k;
  return k;
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------

// One triangle (live: t is a triangle of the mesh): gather and validate its
// vertices, store them and its unit face normal, and its candidate rectangle
// on every image (also returned in r).
template <class ImageAt>
__device__ void setup_one(const MeshSetup& m, int nimg, ImageAt&& image_at, int64_t t, bool live,
                          Rect* r) {
  int32_t ia = 0, ib = 0, ic = 0;
  if (live) {
    ia = m.tris[3 * t];
    ib = m.tris[3 * t + 1];
    ic = m.tris[3 * t + 2];
  }
  float P[9];
  const bool idx_ok = live && ia >= 0 && ia < m.n_verts && ib >= 0 && ib < m.n_verts && ic >= 0 &&
                      ic < m.n_verts;
  bool ok = idx_ok;
  if (idx_ok) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      P[c] = m.verts[3 * (int64_t)ia + c];
      P[3 + c] = m.verts[3 * (int64_t)ib + c];
      P[6 + c] = m.verts[3 * (int64_t)ic + c];
    }
    bool fin = true;
#pragma unroll
    for (int c = 0; c < 9; ++c) fin &= isfinite(P[c]);
    if (!fin) {
      atomicOr(m.status, kStatusNonFinite);
      ok = false;
    }
  } else if (live) {
    atomicOr(m.status, kStatusBadIndex);
  }
  if (!ok) {
    // an invalid triangle becomes a point: never hit, and the call fails
#pragma unroll
    for (int c = 0; c < 9; ++c) P[c] = 0.0f;
  }
  if (live) {
    float* soup = m.soup + 9 * t;
#pragma unroll
    for (int c = 0; c < 9; ++c) soup[c] = P[c];
  }

  // unit face normal (B-A)x(C-A) in float64
  const double e1x = (double)P[3] - (double)P[0], e1y = (double)P[4] - (double)P[1],
               e1z = (double)P[5] - (double)P[2];
  const double e2x = (double)P[6] - (double)P[0], e2y = (double)P[7] - (double)P[1],
               e2z = (double)P[8] - (double)P[2];
  const double nx = e1y * e2z - e1z * e2y;
  const double ny = e1z * e2x - e1x * e2z;
  const double nz = e1x * e2y - e1y * e2x;
  const double len = sqrt((nx * nx + ny * ny) + nz * nz);
  if (live) {
    float4 tn = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (len > 0.0) {
      tn.x = (float)(nx / len);
      tn.y = (float)(ny / len);
      tn.z = (float)(nz / len);
    }
    m.tnorm[t] = tn;
  }

  // The images of one mesh share its box and w, so a world axis has the
  // same pixel centres in both images that use it: the first centre at or
  // above the triangle's min and max on each world axis serves both.
  int lo_c[3] = {0, 0, 0}, hi_c[3] = {0, 0, 0};
  {
    uint32_t need = 0;
    for (int k = 0; k < nimg; ++k) need |= (1u << image_at(k).u) | (1u << image_at(k).v);
    for (int d = 0; d < 3; ++d) {
      if (!((need >> d) & 1u)) continue;
      int k = 0;  // an image that images axis d, with its centre formula for it
      while (image_at(k).u != d && image_at(k).v != d) ++k;
      const Image& im = image_at(k);
      const bool as_u = im.u == d;
      const double lo = as_u ? im.lo_u : im.lo_v, h = as_u ? im.h_u : im.h_v;
      const double inv_h = as_u ? im.inv_h_u : im.inv_h_v, slack = as_u ? im.slack_u : im.slack_v;
      const float mn = fminf(fminf(P[d], P[3 + d]), P[6 + d]);
      const float mx = fmaxf(fmaxf(P[d], P[3 + d]), P[6 + d]);
      lo_c[d] = first_centre_at_or_above(lo, h, inv_h, slack, im.w, mn);
      hi_c[d] = first_centre_at_or_above(lo, h, inv_h, slack, im.w, mx);
    }
  }
  // (loops over the images are unrolled so that r stays in registers)
#pragma unroll
  for (int k = 0; k < kMaxImages; ++k) {
    if (k >= nimg) break;
    const Image& im = image_at(k);
    const int i0 = lo_c[im.u], i1 = hi_c[im.u], j0 = lo_c[im.v], j1 = hi_c[im.v];
    if (i0 < i1 && j0 < j1) {
      r[k].i0 = (int16_t)i0; r[k].i1 = (int16_t)i1; r[k].j0 = (int16_t)j0; r[k].j1 = (int16_t)j1;
    } else {
      r[k].i0 = r[k].i1 = r[k].j0 = r[k].j1 = 0;
    }
    if (live) m.rect[k][t] = r[k];
  }
}

// ---------------------------------------------------------------------------
// setup and binning by chunks of triangles
// ---------------------------------------------------------------------------
// A workgroup takes kBinChunkTris consecutive triangles; mesh order is
// spatially coherent for most meshes, so a chunk meets few tiles.  Global
// atomics are the scarce resource here (a few tens of G per second on the
// whole chip against hundreds of G plain stores), so they are spent per
// (chunk, tile), not per (triangle, tile) or (wave, tile):
//   count    every (triangle, tile) pair is added into an LDS table keyed by
//            (image, tile), one addition per group of a wave's lanes that
//            share the tile; at the end the chunk reserves a range of each
//            tile's list with one global atomic per table slot and records
//            (key, slot, base of the range)
//   scatter  the table is rebuilt slot for slot from the records; a pair's
//            list position is its slot's range start plus a rank from an LDS
//            atomic
// A key that finds no free slot within kBinProbe probes of its home slot is
// counted in tile_ovf and scattered with a global cursor in front of the
// tile's reserved ranges.  Slots never free, so every pair of such a key
// overflows, and in the rebuilt table (the same slots) its kBinProbe probe
// slots hold other keys: it misses there too, while a recorded key is found
// within kBinProbe probes, as when it was inserted.
constexpr int kBinBlock = 512;  // 8 waves per workgroup, one triangle per thread
static_assert(kBinChunkTris % kBinBlock == 0, "whole sub-chunks");

// The (triangle, tile) pairs of one image for one triangle per lane, counted
// into (kScatter false) or placed from (true) the chunk table.  All 64 lanes
// of every wave call this (t beyond the chunk = no tiles).
template <bool kScatter>
__device__ void bin_rect_chunk(const Image& im, uint32_t kimg, int64_t t, bool live, const Rect& r, BinLds& h) {
  const int lane = threadIdx.x & 63;
  auto tile_x = [&](int i) { return im.tw_shift >= 0 ? i >> im.tw_shift : i / im.tw; };
  auto tile_y = [&](int j) { return im.th_shift >= 0 ? j >> im.th_shift : j / im.th; };
  int tx0 = 0, ty0 = 0, nx = 1, n = 0;
  if (live && r.i0 < r.i1 && r.j0 < r.j1) {
    tx0 = tile_x(r.i0);
    ty0 = tile_y(r.j0);
    nx = tile_x(r.i1 - 1) - tx0 + 1;
    n = nx * (tile_y(r.j1 - 1) - ty0 + 1);
  }
  int qx = 0, qy = 0;
  for (int q = 0; __ballot(q < n) != 0; ++q) {
    int key = -1;
    uint32_t cand = 0, geom = 0;
    if (q < n) {
      const int tx = tx0 + qx, ty = ty0 + qy;
      if (++qx == nx) {
        qx = 0;
        ++qy;
      }
      key = ty * im.ntx + tx;
      const int x0 = tx * im.tw, y0 = ty * im.th;
      const int lx0 = max((int)r.i0, x0) - x0, lx1 = min((int)r.i1, x0 + im.tw) - x0;
      const int ly0 = max((int)r.j0, y0) - y0, ly1 = min((int)r.j1, y0 + im.th) - y0;
      if (kScatter)
        geom = (uint32_t)lx0 | ((uint32_t)ly0 << 8) | ((uint32_t)(lx1 - lx0 - 1) << 16) |
               ((uint32_t)(ly1 - ly0 - 1) << 24);
      else
        cand = ((uint32_t)((lx1 - lx0) * (ly1 - ly0)) + 3u) & ~3u;
    }
    // groups: runs of consecutive lanes with the same tile (neighbouring
    // triangles mostly share theirs); a tile may form several runs
    const LaneRuns g = lane_runs(key);
    const int my_leader = g.leader;
    const uint32_t my_rank = g.rank, group = g.group;
    const bool lead = key >= 0 && my_leader == lane;
    const uint32_t hk = (kimg << 30) | (uint32_t)key;
    if (!kScatter) {
      // the run's candidates: inclusive prefix at its last lane minus the
      // prefix before its leader
      const uint32_t incl = wave_inclusive_scan<uint32_t>(cand);
      const uint32_t at_end = (uint32_t)__shfl((int)incl, lead ? lane + (int)group - 1 : lane, 64);
      if (lead) {
        const uint32_t c = at_end - incl + cand;
        const int sl = bin_insert(h, hk);
        if (sl >= 0) {
          atomicAdd(&h.a[sl], group);
          atomicAdd(&h.b[sl], c);
        } else {
          atomicAdd(&im.tile_ovf[key], group);
          atomicAdd(&im.tile_pack[key], (uint64_t)c << 32);
        }
      }
    } else {
      uint32_t lead_base = 0;
      if (lead) {
        const int sl = bin_find(h, hk);
        lead_base = sl >= 0 ? h.a[sl] + atomicAdd(&h.b[sl], group)
                            : im.tile_cnt[key] + atomicAdd(&im.tile_cur[key], group);
      }
      const uint32_t base = (uint32_t)__shfl((int)lead_base, my_leader, 64);
      if (key >= 0) {
        const uint64_t pos = (uint64_t)base + my_rank;
        if (pos < im.list_cap) im.tile_list[pos] = make_int2((int32_t)t, (int32_t)geom);
      }
    }
  }
}

// Counting pass of one chunk [t0, t1): setup of every triangle, its pairs
// into the table, then the reservations and their records.
template <class ImageAt>
__device__ void setup_count_chunk(const MeshSetup& m, int nimg, ImageAt&& image_at, int64_t t0, int64_t t1,
                                  uint32_t chunk) {
  __shared__ BinLds h;
  for (int i = threadIdx.x; i < kBinSlots; i += kBinBlock) {
    h.key[i] = kBinEmpty;
    h.a[i] = 0u;
    h.b[i] = 0u;
  }
  if (threadIdx.x == 0) h.n_rec = 0u;
  __syncthreads();
  for (int64_t tb = t0; tb < t1; tb += kBinBlock) {
    const int64_t t = tb + threadIdx.x;
    const bool live = t < t1;
    Rect r[kMaxImages];
    setup_one(m, nimg, image_at, t, live, r);
#pragma unroll
    for (int k = 0; k < kMaxImages; ++k)
      if (k < nimg) bin_rect_chunk<false>(image_at(k), (uint32_t)k, t, live, r[k], h);
  }
  __syncthreads();
  uint4* rec = m.bin_rec + (size_t)chunk * kBinSlots;
  for (int i = threadIdx.x; i < kBinSlots; i += kBinBlock) {
    const uint32_t hk = h.key[i];
    if (hk == kBinEmpty) continue;
    const Image& im = image_at((int)(hk >> 30));
    const uint32_t key = hk & 0x3fffffffu;
    // one 64-bit atomic adds both and returns the entries reserved before
    const uint32_t base = (uint32_t)atomicAdd(&im.tile_pack[key], ((uint64_t)h.b[i] << 32) | h.a[i]);
    rec[atomicAdd(&h.n_rec, 1u)] = make_uint4(hk, (uint32_t)i, base, 0u);
  }
  __syncthreads();
  if (threadIdx.x == 0) m.bin_nrec[chunk] = h.n_rec;
}

// Scatter pass of one chunk (after the tile scan turned tile_cnt into list
// offsets).
template <class ImageAt>
__device__ void scatter_chunk(const MeshSetup& m, int nimg, ImageAt&& image_at, int64_t t0, int64_t t1,
                              uint32_t chunk) {
  __shared__ BinLds h;
  for (int i = threadIdx.x; i < kBinSlots; i += kBinBlock) h.key[i] = kBinEmpty;
  __syncthreads();
  const uint32_t n = min(m.bin_nrec[chunk], (uint32_t)kBinSlots);
  const uint4* rec = m.bin_rec + (size_t)chunk * kBinSlots;
  for (uint32_t i = threadIdx.x; i < n; i += kBinBlock) {
    const uint4 q = rec[i];
    const Image& im = image_at((int)(q.x >> 30));
    const uint32_t key = q.x & 0x3fffffffu;
    const uint32_t sl = q.y & (kBinSlots - 1);
    h.key[sl] = q.x;
    h.a[sl] = im.tile_cnt[key] + im.tile_ovf[key] + q.z;
    h.b[sl] = 0u;
  }
  __syncthreads();
  for (int64_t tb = t0; tb < t1; tb += kBinBlock) {
    const int64_t t = tb + threadIdx.x;
    const bool live = t < t1;
    for (int k = 0; k < nimg; ++k) {
      const Image& im = image_at(k);
      Rect r{0, 0, 0, 0};
      if (live) r = im.rect[t];
      bin_rect_chunk<true>(im, (uint32_t)k, t, live, r, h);
    }
  }
}

__global__ void __launch_bounds__(kBinBlock) setup_kernel(MeshSetup m, ImageSet set) {
  const int64_t t0 = (int64_t)blockIdx.x * kBinChunkTris;
  setup_count_chunk(m, set.n, [&](int k) -> const Image& { return set.img[k]; }, t0,
                    min(t0 + kBinChunkTris, m.n_tris), blockIdx.x);
}

__global__ void __launch_bounds__(kBinBlock) bin_kernel(MeshSetup m, ImageSet set) {
  const int64_t t0 = (int64_t)blockIdx.x * kBinChunkTris;
  scatter_chunk(m, set.n, [&](int k) -> const Image& { return set.img[k]; }, t0,
                min(t0 + kBinChunkTris, m.n_tris), blockIdx.x);
}

// ---------------------------------------------------------------------------
// candidate enumeration inside one tile
// ---------------------------------------------------------------------------
// A chunk of up to kBlock tile-list entries is loaded into LDS with the
// prefix sum of their candidate counts (pixels of the triangle's rectangle
// inside the tile rows being processed).  Each thread then walks a contiguous
// run of kRun flattened candidates: one binary search finds the first owner,
// after which pixels advance incrementally along the rows of the rectangle.
constexpr int kRun = 16;

template <bool kDepth>
struct ChunkLds {
  float4 ab[kBlock];                   // au, av, bu, bv
  float2 c[kBlock];                    // cu, cv
  float4 z[kDepth ? kBlock : 1];       // az, bz, cz, triangle id (bits)
  int32_t geom[kBlock];                // px0 | py0 << 8 | (width - 1) << 16
  int32_t start[kBlock + 1];           // exclusive prefix of candidates, start[m] = total
  int32_t wave_tmp[kWaves];
};

// Per-entry data of one chunk of a tile list for the sampling walk; an
// entry's candidates end where cg.w says (an exclusive prefix over the chunk),
// so its start is the end of the entry before it.
struct SampleChunk {
  float4 ab[kBlock];        // au, av, bu, bv
  float4 cg[kBlock];        // cu, cv, px0 | py0 << 8 | (width - 1) << 16 (bits), end of candidates (bits)
  float4 z[kBlock];         // az, bz, cz, triangle id (bits)
  int32_t wave_tmp[kWaves];
};

struct TileGeom {
  int x0, y0, cw, ch;  // tile origin and extent in pixels
  int tile;            // tile index within its image
};

// Exact coverage of the ray (ru, rv) by the triangle whose vertices are
// (au,av), (bu,bv), (cu,cv); tav/tbv/tcv are the v-translations of the row.
// Each edge function is one exact product plus one fused multiply-add: since
// both products of float32 values are exact in float64, the FMA returns the
// same correctly rounded difference as two products and a subtraction.
struct Edges {
  double ab, bc, ca;
};

__device__ __forceinline__ bool covered(float au, float bu, float cu, float tav, float tbv,
                                        float tcv, float ru, Edges& e) {
  const float tau = au - ru, tbu = bu - ru, tcu = cu - ru;
  const double dau = tau, dbu = tbu, dcu = tcu, dav = tav, dbv = tbv, dcv = tcv;
  e.ab = fma(dau, dbv, -(dav * dbu));
  e.bc = fma(dbu, dcv, -(dbv * dcu));
  e.ca = fma(dcu, dav, -(dcv * dau));
  const double mn = fmin(fmin(e.ab, e.bc), e.ca), mx = fmax(fmax(e.ab, e.bc), e.ca);
  if ((mn > 0.0) | (mx < 0.0)) return true;   // one strict sign
  if ((mn < 0.0) & (mx > 0.0)) return false;  // two strictly opposite signs: no tie can help
  // the ray meets an edge line: decide as if moved to (+eps, +eps^2)
  double tmp;
  const int s0 = orient(tau, tav, tbu, tbv, tmp);
  const int s1 = orient(tbu, tbv, tcu, tcv, tmp);
  const int s2 = orient(tcu, tcv, tau, tav, tmp);
  return (s0 != 0) & (s0 == s1) & (s1 == s2);
}

// The same decision as covered(), first from float32 edge functions: the
// product tav * tbu is rounded once (error at most 2^-24 of it, or 2^-150
// below the normal range) and the FMA once more, so an edge value larger
// in magnitude than 2^-22 |tav * tbu| + 2^-100 has the sign of the exact
// edge function.  When all three are that large their signs decide (all
// equal: covered); otherwise covered() decides in float64.
__device__ __forceinline__ bool covered_sign(float au, float bu, float cu, float tav, float tbv, float tcv,
                                             float ru) {
  const float tau = au - ru, tbu = bu - ru, tcu = cu - ru;
  const float p0 = tav * tbu, p1 = tbv * tcu, p2 = tcv * tau;
  const float e0 = fmaf(tau, tbv, -p0), e1 = fmaf(tbu, tcv, -p1), e2 = fmaf(tcu, tav, -p2);
  const bool sure = ((int)(fabsf(e0) > fmaf(fabsf(p0), 0x1p-22f, 0x1p-100f)) &
                     (int)(fabsf(e1) > fmaf(fabsf(p1), 0x1p-22f, 0x1p-100f)) &
                     (int)(fabsf(e2) > fmaf(fabsf(p2), 0x1p-22f, 0x1p-100f))) != 0;
  if (__builtin_expect(sure, 1)) {
    const int32_t x0 = __float_as_int(e0), x1 = __float_as_int(e1), x2 = __float_as_int(e2);
    return ((x0 ^ x1) | (x1 ^ x2)) >= 0;
  }
  Edges ed;
  return covered(au, bu, cu, tav, tbv, tcv, ru, ed);
}

// Candidate rectangle of a tile-list entry in tile pixels, rows [y0, y1)
// and columns [x0, x0 + width).  An entry that is not a triangle of the mesh
// or does not fit the tile (the lists were not written as counted) raises the
// mismatch bit and has no candidates (y1 = y0).
struct EntryRect {
  int x0, y0, width, y1;
};
__device__ __forceinline__ EntryRect entry_rect(const Image& im, const TileGeom& g, int2 ent) {
  const uint32_t gm = (uint32_t)ent.y;
  EntryRect r;
  r.x0 = gm & 255;
  r.y0 = (gm >> 8) & 255;
  r.width = ((gm >> 16) & 255) + 1;
  r.y1 = r.y0 + (int)(gm >> 24) + 1;
  if ((uint32_t)ent.x >= (uint64_t)im.n_tris || r.x0 + r.width > g.cw || r.y1 > g.ch) {
    atomicOr(im.status, kStatusMismatch);
    r.x0 = 0;
    r.y0 = 0;
    r.width = 1;
    r.y1 = 0;
  }
  return r;
}

struct NoChunkHook {
  __device__ void operator()(bool, int) const {}
};

// Calls on_hit(k, px, py, edges) for every covered candidate of rows
// [r0, r1) of the tile; k indexes the chunk arrays in L.  Thread 0 calls
// on_chunk(first, candidates) once the candidate count of a chunk is known,
// before the barrier that precedes its walk (first: the tile's first chunk).
template <bool kDepth, class OnHit, class OnChunk = NoChunkHook>
__device__ void tile_candidates(const Image& im, const TileGeom& g, int r0, int r1,
                                ChunkLds<kDepth>& L, const float* s_cu, const float* s_cv,
                                OnHit&& on_hit, OnChunk&& on_chunk = OnChunk()) {
  const uint64_t cap = im.list_cap;
  const uint32_t e_begin = (uint32_t)min((uint64_t)im.tile_cnt[g.tile], cap);
  const uint32_t e_end = (uint32_t)min((uint64_t)im.tile_cnt[g.tile + 1], cap);
  for (uint32_t base = e_begin; base < e_end; base += kBlock) {
    const int m = (int)min((uint32_t)kBlock, e_end - base);
    const int k = threadIdx.x;
    int nc = 0;
    if (k < m) {
      const int2 ent = im.tile_list[base + k];
      const int32_t t = ent.x;
      const EntryRect r = entry_rect(im, g, ent);
      const int py0 = max(r.y0, r0), py1 = min(r.y1, r1);
      const int width = r.width;
      if (py1 > py0) nc = width * (py1 - py0);
      L.geom[k] = r.x0 | (max(py0, 0) << 8) | ((width - 1) << 16);
      if (nc > 0) {  // vertex data only for entries with candidates in these rows
        const float* s = im.soup + 9 * (int64_t)t;
        L.ab[k] = make_float4(s[im.u], s[im.v], s[3 + im.u], s[3 + im.v]);
        L.c[k] = make_float2(s[6 + im.u], s[6 + im.v]);
        if constexpr (kDepth) L.z[k] = make_float4(s[im.a], s[3 + im.a], s[6 + im.a], __int_as_float(t));
      }
    }
    int total;
    const int excl = block_exclusive_scan<int>(nc, L.wave_tmp, total);
    if (k < m) L.start[k] = excl;
    if (k == 0) {
      L.start[m] = total;
      on_chunk(base == e_begin, total);
    }
    __syncthreads();
    for (int wb = 0; wb < total; wb += kBlock * kRun) {
      int c = wb + threadIdx.x * kRun;
      const int cend = min(c + kRun, total);
      if (c < cend) {
        // owner of c: the last entry whose start is <= c
        int lo = 0, hi = m - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (L.start[mid] <= c) lo = mid; else hi = mid - 1;
        }
        int e = lo;
        int gm = L.geom[e];
        int width = ((gm >> 16) & 255) + 1;
        int local = c - L.start[e];
        int row = local / width;
        int col = local - row * width;
        int kend = L.start[e + 1];
        float4 ab = L.ab[e];
        float2 cc = L.c[e];
        int px0 = gm & 255, py0 = (gm >> 8) & 255;
        float rv = s_cv[py0 + row];
        float tav = ab.y - rv, tbv = ab.w - rv, tcv = cc.y - rv;
        for (; c < cend; ++c) {
          if (c == kend) {  // next entry that has candidates
            ++e;
            while (L.start[e + 1] <= c) ++e;
            gm = L.geom[e];
            width = ((gm >> 16) & 255) + 1;
            px0 = gm & 255;
            py0 = (gm >> 8) & 255;
            row = 0;
            col = 0;
            kend = L.start[e + 1];
            ab = L.ab[e];
            cc = L.c[e];
            rv = s_cv[py0];
            tav = ab.y - rv; tbv = ab.w - rv; tcv = cc.y - rv;
          }
          Edges ed;
          if (covered(ab.x, ab.z, cc.x, tav, tbv, tcv, s_cu[px0 + col], ed))
            on_hit(e, px0 + col, py0 + row, ed);
          if (++col == width) {
            col = 0;
            ++row;
            rv = s_cv[py0 + row];
            tav = ab.y - rv; tbv = ab.w - rv; tcv = cc.y - rv;
          }
        }
      }
    }
    __syncthreads();
  }
}

__device__ __forceinline__ TileGeom tile_geom(const Image& im, int tile) {
  TileGeom g;
  g.tile = tile;
  const int tx = tile % im.ntx, ty = tile / im.ntx;
  g.x0 = tx * im.tw;
  g.y0 = ty * im.th;
  g.cw = min(im.tw, im.w - g.x0);
  g.ch = min(im.th, im.w - g.y0);
  return g;
}

// Depth of the hit from lo_a: the axis coordinate interpolated with the
// barycentric weights E_BC, E_CA, E_AB over their sum, in float64.
__device__ __forceinline__ float depth_of(const Edges& e, float az, float bz, float cz,
                                          double lo_a) {
  const double den = (e.ab + e.bc) + e.ca;
  const double num = e.ca * ((double)bz - (double)az) + e.ab * ((double)cz - (double)az);
  const double z = (double)az + num / den;
  float d = (float)(z - lo_a);
  if (d == 0.0f) d = 0.0f;
  return d;
}

// ---------------------------------------------------------------------------
// sampling pass: count and stage every hit
// ---------------------------------------------------------------------------
// A tile's staging region holds at most im.stage_layers hits per tile pixel
// (and never more than the tile's candidates); a tile with more hits than its
// region is walked again by the write pass.
constexpr uint32_t kMinStageLayers = 64, kMaxStageLayers = 1024;

// Workgroups per CU the sampling kernels are built for: seven for small
// tiles, five for large ones (their LDS: 32-bit hit descriptors, larger
// count and centre arrays).
template <int kTilePix>
constexpr int sample_wgs_per_cu() { return kTilePix <= kSmallTilePix ? 7 : 5; }

// Hits found by a wave in one window of its walk, waiting for their depth:
// at most kRun candidates per thread per window (12 for large tiles, so that
// five of their workgroups fit a CU's LDS).
template <int kTilePix>
struct SampleLds {
  // descriptor: tile pixel q | chunk entry << kQBits
  static constexpr int kQBits = kTilePix <= 256 ? 8 : 10;
  static constexpr int kRun = kTilePix <= kSmallTilePix ? 16 : 12;
  using Desc = typename std::conditional<(kTilePix <= 256), uint16_t, uint32_t>::type;
  Desc hit[kWaves][64 * kRun];
};

// One walk of the tile.  Candidates are split into runs of equal length
// over all threads of the workgroup (one binary search per run, then
// incremental pixel steps).  A covered candidate only appends its (entry,
// pixel) descriptor to its wave's list; after each window the wave takes its
// hits 64 at a time, recomputes their edge functions, and computes depth,
// key and arrival slot with every lane busy, storing them to consecutive
// entries of the tile's staging region.  The region is sized by the tile's
// candidate count (pixels of the clipped rectangles), which bounds its hits.
template <int kTilePix>
__device__ void sample_tile(const Image& im, int tile, uint32_t gtile, uint32_t* plan, uint32_t n_total,
                            int place_cap) {
  using Lds = SampleLds<kTilePix>;
  constexpr int kQBits = Lds::kQBits;
  __shared__ uint32_t s_cnt[kTilePix];
  __shared__ float s_cu[kMaxTileW];
  __shared__ float s_cv[kMaxTileH + 1];
  __shared__ SampleChunk L;
  __shared__ Lds H;
  __shared__ uint32_t s_red[kWaves];
  __shared__ uint32_t s_fill;

  const TileGeom g = tile_geom(im, tile);
  const int npix = g.cw * g.ch;
  const int cw = g.cw;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t cap = im.list_cap;
  const uint32_t e_begin = (uint32_t)min((uint64_t)im.tile_cnt[tile], cap);
  const uint32_t e_end = (uint32_t)min((uint64_t)im.tile_cnt[tile + 1], cap);

  if (e_begin == e_end) {
    // no triangle meets the tile: zero counts, no hits, nothing to place
    for (int q = threadIdx.x; q < npix; q += kBlock) {
      const int py = q / cw, px = q - py * cw;
      im.counts[(size_t)(g.y0 + py) * im.w + g.x0 + px] = 0u;
    }
    if (threadIdx.x == 0) {
      im.tile_hits[tile] = 0u;
      im.tile_stage[tile] = 0u;
      if (im.tile_max) im.tile_max[tile] = 0u;
      if (plan) {
        plan[gtile] = 0u;
        plan[n_total + gtile] = 0u;
      }
    }
    return;
  }

  for (int q = threadIdx.x; q < npix; q += kBlock) s_cnt[q] = 0;
  for (int q = threadIdx.x; q < g.cw; q += kBlock) s_cu[q] = pixel_centre(im.lo_u, im.h_u, g.x0 + q);
  for (int q = threadIdx.x; q <= g.ch; q += kBlock)
    s_cv[q] = pixel_centre(im.lo_v, im.h_v, min(g.y0 + q, im.w - 1));

  // The tile's staging region comes from the tile scan (whole 4-entry
  // groups, so the place pass reads 16-byte vectors); a region that ends
  // beyond the buffer is not used and the tile is walked again.
  const uint32_t region_first = im.tile_region[tile];
  const uint32_t region_end = im.tile_region[tile + 1];
  const uint32_t region_size =
      (im.stage_key != nullptr && region_end <= im.stage_cap) ? region_end - region_first : 0u;
  if (threadIdx.x == 0) s_fill = 0;
  __syncthreads();
  const double lo_a = im.lo_a;
  const float inv_cw = 1.0f / (float)cw;
  typename Lds::Desc* my_hits = H.hit[wave];

  for (uint32_t cbase = e_begin; cbase < e_end; cbase += kBlock) {
    // ---- load a chunk of entries with their candidate counts
    const int m = (int)min((uint32_t)kBlock, e_end - cbase);
    int total;
    {
      const int k = threadIdx.x;
      int nc = 0, gm = 0;
      float4 ab = make_float4(0.f, 0.f, 0.f, 0.f), z = ab;
      float2 cc = make_float2(0.f, 0.f);
      if (k < m) {
        const int2 ent = im.tile_list[cbase + k];
        const EntryRect r = entry_rect(im, g, ent);
        if (r.y1 > r.y0) {
          nc = r.width * (r.y1 - r.y0);
          gm = r.x0 | (r.y0 << 8) | ((r.width - 1) << 16);
          const float* sp = im.soup + 9 * (int64_t)ent.x;
          ab = make_float4(sp[im.u], sp[im.v], sp[3 + im.u], sp[3 + im.v]);
          cc = make_float2(sp[6 + im.u], sp[6 + im.v]);
          z = make_float4(sp[im.a], sp[3 + im.a], sp[6 + im.a], __int_as_float(ent.x));
        } else {
          // an entry that does not fit (already reported): one candidate,
          // pixel (0, 0), with all vertices at the origin, which covers
          // nothing, so that every entry of the walk has candidates
          nc = 1;
        }
      }
      const int excl = block_exclusive_scan<int>(nc, L.wave_tmp, total);
      if (k < m) {
        L.ab[k] = ab;
        L.cg[k] = make_float4(cc.x, cc.y, __int_as_float(gm), __int_as_float(excl + nc));
        L.z[k] = z;
      }
      __syncthreads();
    }
    const int run = min(max((total + kBlock - 1) / kBlock, 2), Lds::kRun);

    for (int wb = 0; wb < total; wb += kBlock * run) {
      // ---- walk: covered candidates append their descriptor
      uint32_t nh = 0;  // hits of this wave in the window (wave-uniform)
      int c = wb + threadIdx.x * run;
      const int cend = min(c + run, total);
      if (c < cend) {
        int lo = 0, hi = m - 1;  // owner of c: the first entry whose candidates end after c
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (__float_as_int(L.cg[mid].w) > c) hi = mid; else lo = mid + 1;
        }
        int e = lo;
        const int first = e > 0 ? __float_as_int(L.cg[e - 1].w) : 0;
        float4 ab = L.ab[e];
        float4 cg = L.cg[e];
        int gm = __float_as_int(cg.z);
        int width = ((gm >> 16) & 255) + 1;
        int px0 = gm & 255;
        int kend = __float_as_int(cg.w);
        const int local = c - first;
        const int row = local / width;
        int col = local - row * width;
        int py = ((gm >> 8) & 255) + row;
        for (; c < cend; ++c) {
          const float rv = s_cv[py];
          const int px = px0 + col;
          const bool hit = covered_sign(ab.x, ab.z, cg.x, ab.y - rv, ab.w - rv, cg.y - rv, s_cu[px]);
          const uint64_t mask = __ballot(hit);
          if (hit) {
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
            const uint32_t q = __umul24((uint32_t)py, (uint32_t)cw) + (uint32_t)px;
            my_hits[nh + rank] = (typename Lds::Desc)(q | ((uint32_t)e << kQBits));
          }
          nh += (uint32_t)__popcll(mask);
          // the next candidate: the next column, row or entry, without
          // branches (the entry's data is read again either way)
          ++col;
          const bool next_entry = c + 1 == kend;
          const bool next_row = col == width;
          e = min(e + (next_entry ? 1 : 0), m - 1);
          ab = L.ab[e];
          cg = L.cg[e];
          gm = __float_as_int(cg.z);
          col = (next_entry || next_row) ? 0 : col;
          py = next_entry ? ((gm >> 8) & 255) : py + (next_row ? 1 : 0);
          px0 = gm & 255;
          width = ((gm >> 16) & 255) + 1;
          kend = __float_as_int(cg.w);
        }
      }
      // lanes that left the walk early did not see the later ballots: the
      // wave's count is the largest
      for (int d = 32; d >= 1; d >>= 1) nh = max(nh, (uint32_t)__shfl_xor((int)nh, d, 64));
      nh = __builtin_amdgcn_readfirstlane(nh);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

      // ---- the wave's hits, 64 at a time: depth, key, slot, stage
      uint32_t first = 0;
      if (lane == 0 && nh > 0) first = atomicAdd(&s_fill, nh);
      first = __shfl((int)first, 0, 64);
      for (uint32_t i = lane; i < nh; i += 64) {
        const uint32_t d = my_hits[i];
        const int q = (int)(d & ((1u << kQBits) - 1u));
        const int e = (int)(d >> kQBits);
        const int py = (int)(((float)q + 0.5f) * inv_cw);
        const int px = q - py * cw;
        const float4 ab = L.ab[e];
        const float4 cc = L.cg[e];
        const float4 z = L.z[e];
        const float rv = s_cv[py];
        Edges ed;
        (void)covered(ab.x, ab.z, cc.x, ab.y - rv, ab.w - rv, cc.y - rv, s_cu[px], ed);
        const float dep = depth_of(ed, z.x, z.y, z.z, lo_a);
        const uint32_t slot = atomicAdd(&s_cnt[q], 1u);
        const uint32_t pos = first + i;
        if (pos < region_size) {
          const size_t at = (size_t)region_first + pos;
          im.stage_key[at] = sample_key(dep, __float_as_int(z.w));
          im.stage_qs[at] = (uint32_t)q | (slot << 10);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();  // before the next chunk replaces L
  }

  uint32_t mx = 0;
  for (int q = threadIdx.x; q < npix; q += kBlock) {
    const int py = q / cw, px = q - py * cw;
    const uint32_t c = s_cnt[q];
    mx = max(mx, c);
    im.counts[(size_t)(g.y0 + py) * im.w + g.x0 + px] = c;
  }
  // The largest count: per tile for a later reduction (batches), else one
  // atomic per tile if asked (the single-mesh path takes it from the pixel
  // scan): atomics from every tile to one address would queue up.
  if (im.tile_max != nullptr || im.max_layers != nullptr) mx = block_max(mx, s_red);
  if (threadIdx.x == 0) {
    if (im.tile_max != nullptr) im.tile_max[tile] = mx;
    else if (im.max_layers != nullptr && mx > 0) atomicMax(im.max_layers, mx);
    const uint32_t hits = s_fill;
    const bool staged = hits <= region_size;
    im.tile_hits[tile] = hits;
    if (hits == 0) {
      im.tile_stage[tile] = 0;
    } else if (staged) {
      im.tile_stage[tile] = region_first;
    } else {
      im.tile_stage[tile] = kNoStage;
      im.walk_list[atomicAdd(im.walk_count, 1u)] = gtile;
    }
    // place items: ceil(hits / stage) for a staged tile with hits
    if (plan) {
      const uint32_t K = (hits == 0 || !staged) ? 0u : (hits + place_cap - 1) / (uint32_t)place_cap;
      plan[gtile] = K >= 2 ? K : 0u;
      plan[n_total + gtile] = K == 1 ? 1u : 0u;
    }
  }
}

// (small tiles: at most 72 VGPRs, seven workgroups per CU)
template <int kTilePix>
__global__ void __launch_bounds__(kBlock, sample_wgs_per_cu<kTilePix>()) sample_kernel(ImageSet set) {
  const int k = image_of_block(set, blockIdx.x);
  sample_tile<kTilePix>(set.img[k], (int)(blockIdx.x - set.tile_start[k]), blockIdx.x, set.plan,
                        set.tile_start[set.n], set.place_cap);
}

// ---------------------------------------------------------------------------
// write pass
// ---------------------------------------------------------------------------
// Output of one run of staged keys: each key finds its rank among its
// pixel's keys and is stored at its sorted position; four keys per thread at
// a time, their normal gathers in flight while the ranks are counted.
template <int kTilePix>
__device__ __forceinline__ void write_staged_run(const Image& im, const uint64_t* s_keys,
                                                 const uint16_t* s_pix, const uint32_t* s_pre,
                                                 const uint32_t* s_off, uint32_t run_base, int run_total) {
  constexpr int kU = 4;
  for (int s0 = threadIdx.x; s0 < run_total; s0 += kBlock * kU) {
    uint64_t key[kU];
    int qq[kU];
    float nx[kU], ny[kU], nz[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int s2 = s0 + u * kBlock;
      qq[u] = -1;
      if (s2 < run_total) {
        key[u] = s_keys[s2];
        qq[u] = s_pix[s2];
        const float4 nrm = im.tnorm[(int32_t)(uint32_t)key[u]];  // one 16-byte gather
        nx[u] = nrm.x;
        ny[u] = nrm.y;
        nz[u] = nrm.z;
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (qq[u] < 0) continue;
      const int q = qq[u];
      const uint32_t b = s_pre[q] - run_base;
      const uint32_t n = s_pre[q + 1] - s_pre[q];
      // four independent LDS reads per step (the loop is bound by their latency)
      uint32_t rank = 0, j = 0;
      for (; j + 4 <= n; j += 4) {
        const uint64_t k0 = s_keys[b + j], k1 = s_keys[b + j + 1], k2 = s_keys[b + j + 2],
                       k3 = s_keys[b + j + 3];
        rank += (uint32_t)(k0 < key[u]) + (uint32_t)(k1 < key[u]) + (uint32_t)(k2 < key[u]) +
                (uint32_t)(k3 < key[u]);
      }
      for (; j < n; ++j) rank += (s_keys[b + j] < key[u]) ? 1u : 0u;
      const size_t o = (size_t)s_off[q] + rank;
      im.depth[o] = key_depth(key[u]);
      im.tri[o] = (int32_t)(uint32_t)key[u];
      store_normal(im, o, nx[u], ny[u], nz[u]);
    }
  }
}

// Output offsets (s_off) and exclusive prefix of the sample counts (s_pre,
// npix + 1 entries) of the tile's pixels, q = py * cw + px; s_cur (if given)
// is cleared.  Ends with a barrier.
__device__ void tile_prefix(const Image& im, const TileGeom& g, uint32_t* s_off, uint32_t* s_pre,
                            uint32_t* s_cur, uint32_t* s_wave) {
  const int npix = g.cw * g.ch;
  uint32_t carry = 0;
  for (int base = 0; base < npix; base += kBlock) {
    const int q = base + threadIdx.x;
    uint32_t n = 0;
    if (q < npix) {
      const int py = q / g.cw, px = q - py * g.cw;
      const size_t gp = (size_t)(g.y0 + py) * im.w + g.x0 + px;
      const uint32_t o = im.offsets[gp];
      n = im.offsets[gp + 1] - o;
      s_off[q] = o;
      if (s_cur) s_cur[q] = 0;
    }
    uint32_t total;
    const uint32_t ex = block_exclusive_scan<uint32_t>(n, s_wave, total);
    if (q < npix) s_pre[q] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) s_pre[npix] = carry;
  __syncthreads();
}

// The next run of pixels from q0: the longest whose samples fit in cap
// (at least one pixel).  Returns its end; direct is set when that one pixel
// alone holds more than cap samples.  Ends with a barrier.
__device__ int next_run(const uint32_t* s_pre, int q0, int npix, int cap, int* s_run, bool& direct) {
  if (threadIdx.x == 0) {
    int lo = q0 + 1, hi = npix;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_pre[mid] - s_pre[q0] <= (uint32_t)cap) lo = mid; else hi = mid - 1;
    }
    s_run[0] = lo;
    s_run[1] = (s_pre[q0 + 1] - s_pre[q0] > (uint32_t)cap) ? 1 : 0;
  }
  __syncthreads();
  direct = s_run[1] != 0;
  return s_run[0];
}

// The n samples of one pixel were stored unsorted from output offset o:
// sorted in place by (depth, triangle) key with the whole workgroup, a
// bitonic network over the next power of two N >= n in global memory whose
// compare-exchanges all put the smaller key first (each merge starts by
// comparing mirrored positions), so the virtual +inf keys at positions >= n
// never move and those pairs are skipped; then their normals.
__device__ void finish_deep_pixel(const Image& im, size_t o, uint32_t n) {
  uint32_t N = 1;
  while (N < n) N <<= 1;
  auto cx = [&](uint32_t i, uint32_t j) {  // i < j
    if (j >= n) return;
    const float d0 = im.depth[o + i], d1 = im.depth[o + j];
    const int32_t t0 = im.tri[o + i], t1 = im.tri[o + j];
    if (sample_key(d1, t1) < sample_key(d0, t0)) {
      im.depth[o + i] = d1;
      im.depth[o + j] = d0;
      im.tri[o + i] = t1;
      im.tri[o + j] = t0;
    }
  };
  for (uint32_t k = 2; k <= N; k <<= 1) {
    for (uint32_t h = threadIdx.x; h < N / 2; h += kBlock) {  // mirrored pairs in blocks of k
      const uint32_t blk = h / (k / 2) * k, r = h % (k / 2);
      cx(blk + r, blk + k - 1 - r);
    }
    __threadfence_block();
    __syncthreads();
    for (uint32_t j = k / 4; j >= 1; j >>= 1) {  // half-cleaners in blocks of 2j
      for (uint32_t h = threadIdx.x; h < N / 2; h += kBlock) {
        const uint32_t i = h / j * 2 * j + h % j;
        cx(i, i + j);
      }
      __threadfence_block();
      __syncthreads();
    }
  }
  for (uint32_t s2 = threadIdx.x; s2 < n; s2 += kBlock) {
    const int32_t t = im.tri[o + s2];
    const float4 nrm = im.tnorm[t];
    store_normal(im, o + s2, nrm.x, nrm.y, nrm.z);
  }
}

// The tile's pixels are taken in runs (row-major within the tile) whose
// samples fit in LDS.  Hits of a run are staged at their pixel's slots as
// (depth, triangle) keys with the pixel alongside; each staged key then finds
// its rank among its pixel's keys and is stored straight to its sorted
// position, so sorting and storing are one pass over the staged keys.  Only a
// single pixel with more samples than the LDS capacity is written directly to
// its output range and sorted there.
// Runs of the tile's greedy split with index = part (mod parts) are written
// by this call; the split is the same for every part.
template <int kTilePix>
__device__ void write_tile(const Image& im, int tile, int part = 0, int parts = 1) {
  constexpr int kStageCap = stage_cap(kTilePix);
  __shared__ uint64_t s_keys[kStageCap];
  __shared__ uint16_t s_pix[kStageCap];       // tile pixel index of each staged key
  __shared__ uint32_t s_off[kTilePix];        // output offset of each tile pixel
  __shared__ uint32_t s_pre[kTilePix + 1];    // prefix of samples over tile pixels
  __shared__ uint32_t s_cur[kTilePix];        // fill cursor of each tile pixel
  __shared__ float s_cu[kMaxTileW];
  __shared__ float s_cv[kMaxTileH + 1];
  __shared__ ChunkLds<true> L;
  __shared__ uint32_t s_wave[kWaves];
  __shared__ int s_run[2];                    // end pixel of the run, direct mode

  const TileGeom g = tile_geom(im, tile);
  const int npix = g.cw * g.ch;  // tile pixels, q = py * cw + px

  for (int q = threadIdx.x; q < g.cw; q += kBlock) s_cu[q] = pixel_centre(im.lo_u, im.h_u, g.x0 + q);
  for (int q = threadIdx.x; q <= g.ch; q += kBlock)
    s_cv[q] = pixel_centre(im.lo_v, im.h_v, min(g.y0 + q, im.w - 1));
  tile_prefix(im, g, s_off, s_pre, s_cur, s_wave);

  int q0 = 0;
  for (int run = 0; q0 < npix; ++run) {
    bool direct;
    const int q1 = next_run(s_pre, q0, npix, kStageCap, s_run, direct);
    const uint32_t run_base = s_pre[q0];
    const int run_total = (int)(s_pre[q1] - run_base);
    if (run_total > 0 && run % parts == part) {
      const int r0 = q0 / g.cw, r1 = (q1 - 1) / g.cw + 1;
      const double lo_a = im.lo_a;
      const int cw = g.cw;
      tile_candidates<true>(im, g, r0, r1, L, s_cu, s_cv,
                            [&](int e, int px, int py, const Edges& ed) {
                              const int q = py * cw + px;
                              if (q < q0 || q >= q1) return;
                              const uint32_t slot = atomicAdd(&s_cur[q], 1u);
                              if (slot >= s_pre[q + 1] - s_pre[q]) {  // count/write disagree
                                atomicOr(im.status, kStatusMismatch);
                                return;
                              }
                              const float4 z = L.z[e];
                              const float d = depth_of(ed, z.x, z.y, z.z, lo_a);
                              const int32_t t = __float_as_int(z.w);
                              if (!direct) {
                                const uint32_t at = s_pre[q] - run_base + slot;
                                s_keys[at] = sample_key(d, t);
                                s_pix[at] = (uint16_t)q;
                              } else {
                                const size_t o = (size_t)s_off[q] + slot;
                                im.depth[o] = d;
                                im.tri[o] = t;
                              }
                            });
      // tile_candidates ends with a barrier
      if (!direct) {
        write_staged_run<kTilePix>(im, s_keys, s_pix, s_pre, s_off, run_base, run_total);
      } else {
        finish_deep_pixel(im, s_off[q0], s_pre[q0 + 1] - s_pre[q0]);
      }
    }
    __syncthreads();
    q0 = q1;
  }
}

// Work items of the place pass: a staged tile with S hits gets
// K = ceil(S / stage) items; tiles without hits or walked again get none.
// The sampling pass writes K to the plan ([0, n) for K >= 2, [n, 2n) for
// K = 1), so after one scan of the plan the long tiles come first.
// K <= stage_layers * tile pixels / stage.
// One work item of the place pass.
struct PlaceItem {
  uint32_t gtile;       // set-wide tile number
  uint32_t part_parts;  // part | parts << 16
  uint32_t first;       // first staged entry of the tile
  uint32_t hits;        // staged entries of the tile
};

// Items in launch order (dense tiles first), from the scanned plan.
__global__ void __launch_bounds__(kBlock) plan_items_kernel(ImageSet set, PlaceItem* items) {
  const uint32_t gt = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t n_tiles = set.tile_start[set.n];
  if (gt >= n_tiles) return;
  const int k = image_of_block(set, gt);
  const Image& im = set.img[k];
  const int tile = (int)(gt - set.tile_start[k]);
  const uint32_t* plan = set.plan;
  const uint32_t kd = plan[gt + 1] - plan[gt];
  const uint32_t ks = plan[n_tiles + gt + 1] - plan[n_tiles + gt];
  const uint32_t K = kd + ks;
  if (K == 0) return;
  const uint32_t at = kd ? plan[gt] : plan[n_tiles + gt];
  PlaceItem it;
  it.gtile = gt;
  it.first = im.tile_stage[tile];
  it.hits = im.tile_hits[tile];
  for (uint32_t j = 0; j < K; ++j) {
    it.part_parts = j | (K << 16);
    items[at + j] = it;
  }
}

// ---------------------------------------------------------------------------
// place pass: write the hits staged by the sampling pass
// ---------------------------------------------------------------------------
// The tile's pixels are split into the same runs as in write_tile.  A run
// reads the tile's staged entries, keeps those of its pixels and puts each key
// at its pixel's slot in LDS (the slot came with the hit), then ranks and
// stores the keys like write_tile.  A single pixel deeper than the stage is
// stored unsorted straight to its output range and sorted there.
template <int kTilePix>
__device__ void place_tile(const Image& im, int tile, uint32_t first, uint32_t hits, int part,
                           int parts) {
  constexpr int kStageCap = stage_cap(kTilePix);
  constexpr int kPer = kStageCap / kBlock;  // staged entries per thread of a one-run tile
  __shared__ uint64_t s_keys[kStageCap];
  __shared__ uint16_t s_pix[kStageCap];
  __shared__ uint32_t s_off[kTilePix];
  __shared__ uint32_t s_pre[kTilePix + 1];
  __shared__ uint32_t s_wave[kWaves];
  __shared__ int s_run[2];

  const TileGeom g = tile_geom(im, tile);
  const int npix = g.cw * g.ch;
  const uint64_t* keys = im.stage_key + first;
  const uint32_t* qs = im.stage_qs + first;

  if (hits <= (uint32_t)kStageCap) {
    // One run holds the whole tile: the staged entries are loaded before the
    // pixel offsets are scanned, so the two reads overlap.
    uint32_t rq[kPer];
    uint64_t rk[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const uint32_t i = threadIdx.x + u * kBlock;
      rq[u] = i < hits ? qs[i] : 0xffffffffu;
      rk[u] = i < hits ? keys[i] : 0;
    }
    tile_prefix(im, g, s_off, s_pre, nullptr, s_wave);
    if (s_pre[npix] != hits) {  // staging and counts disagree
      if (threadIdx.x == 0) atomicOr(im.status, kStatusMismatch);
      return;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      if (rq[u] == 0xffffffffu) continue;
      const int q = (int)(rq[u] & 1023u);
      const uint32_t slot = rq[u] >> 10;
      if (q >= npix || slot >= s_pre[q + 1] - s_pre[q]) {
        atomicOr(im.status, kStatusMismatch);
        continue;
      }
      s_keys[s_pre[q] + slot] = rk[u];
      s_pix[s_pre[q] + slot] = (uint16_t)q;
    }
    __syncthreads();
    write_staged_run<kTilePix>(im, s_keys, s_pix, s_pre, s_off, 0u, (int)hits);
    return;
  }

  tile_prefix(im, g, s_off, s_pre, nullptr, s_wave);
  if (s_pre[npix] != hits) {
    if (threadIdx.x == 0) atomicOr(im.status, kStatusMismatch);
    return;
  }
  int q0 = 0;
  for (int run = 0; q0 < npix; ++run) {
    bool direct;
    const int q1 = next_run(s_pre, q0, npix, kStageCap, s_run, direct);
    const uint32_t run_base = s_pre[q0];
    const int run_total = (int)(s_pre[q1] - run_base);
    if (run_total > 0 && run % parts == part) {
      // Eight entries per thread per step: two 16-byte loads (regions are
      // whole 4-entry groups) issued together, then the keys of the run's
      // entries, also together, so a step costs two round trips.
      for (uint32_t b0 = 0; b0 < hits; b0 += 8 * kBlock) {
        uint32_t xs[8];
        uint64_t ks[8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const uint32_t i0 = b0 + 4 * (h * kBlock + threadIdx.x);
          uint4 x4 = make_uint4(0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu);
          if (i0 < hits) x4 = *reinterpret_cast<const uint4*>(qs + i0);
          xs[4 * h] = x4.x; xs[4 * h + 1] = x4.y; xs[4 * h + 2] = x4.z; xs[4 * h + 3] = x4.w;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint32_t i = b0 + 4 * ((u >> 2) * kBlock + threadIdx.x) + (u & 3);
          const int q = (int)(xs[u] & 1023u);
          const bool mine = i < hits && q >= q0 && q < q1;
          ks[u] = mine ? keys[i] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint32_t i = b0 + 4 * ((u >> 2) * kBlock + threadIdx.x) + (u & 3);
          const int q = (int)(xs[u] & 1023u);
          const uint32_t slot = xs[u] >> 10;
          if (i >= hits || q < q0 || q >= q1) continue;
          if (slot >= s_pre[q + 1] - s_pre[q]) {
            atomicOr(im.status, kStatusMismatch);
            continue;
          }
          const uint64_t key = ks[u];
          if (!direct) {
            const uint32_t at = s_pre[q] - run_base + slot;
            s_keys[at] = key;
            s_pix[at] = (uint16_t)q;
          } else {
            const size_t o = (size_t)s_off[q] + slot;
            im.depth[o] = key_depth(key);
            im.tri[o] = (int32_t)(uint32_t)key;
          }
        }
      }
      __syncthreads();
      if (!direct) {
        write_staged_run<kTilePix>(im, s_keys, s_pix, s_pre, s_off, run_base, run_total);
      } else {
        finish_deep_pixel(im, s_off[q0], s_pre[q0 + 1] - s_pre[q0]);
      }
    }
    __syncthreads();
    q0 = q1;
  }
}

// One workgroup per place item.
template <int kTilePix>
__global__ void __launch_bounds__(kBlock) place_kernel(ImageSet set, const PlaceItem* items) {
  const PlaceItem it = items[xcd_runs<kPlaceRun>(blockIdx.x, gridDim.x)];
  const int k = image_of_block(set, it.gtile);
  place_tile<kTilePix>(set.img[k], (int)(it.gtile - set.tile_start[k]), it.first, it.hits,
                       (int)(it.part_parts & 0xffffu), (int)(it.part_parts >> 16));
}

// Tiles whose hits did not fit their staging region: walked and written
// again, one workgroup per tile.
template <int kTilePix>
__global__ void __launch_bounds__(kBlock) walk_kernel(ImageSet set, const uint32_t* list, uint32_t n,
                                                      uint32_t* counter) {
  __shared__ uint32_t s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1u);
    __syncthreads();
    const uint32_t item = s_item;
    __syncthreads();
    if (item >= n) break;
    const uint32_t gt = list[item];
    const int k = image_of_block(set, gt);
    write_tile<kTilePix>(set.img[k], (int)(gt - set.tile_start[k]));
  }
}

// ---------------------------------------------------------------------------
// fill
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) fill_u32_kernel(uint32_t* p, uint32_t value, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * kBlock)
    p[q] = value;
}

// ---------------------------------------------------------------------------
// exclusive scan of u32 with u64 accumulation
// ---------------------------------------------------------------------------
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;  // 4096 values per workgroup

__device__ __forceinline__ void load16_raw(const uint32_t* in, int64_t n, int64_t i, uint32_t v[16]) {
  if (i + 16 <= n) {
    const uint4* p = reinterpret_cast<const uint4*>(in + i);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint4 q = p[k];
      v[4 * k] = q.x; v[4 * k + 1] = q.y; v[4 * k + 2] = q.z; v[4 * k + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = (i + k < n) ? in[i + k] : 0u;
  }
}

// 16 values of in, each capped at cap
__device__ __forceinline__ void load16(const uint32_t* in, int64_t n, int64_t i, uint32_t cap, uint32_t v[16]) {
  load16_raw(in, n, i, v);
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = min(v[k], cap);
}

// 16 values of a packed tile count (entries in the low half, candidates in
// the high half) plus the entries counted apart (add): seg 0 the entries
// (saturating), seg 1 the candidates.  A tile's candidates (at most 1024 per
// entry) fit the high half while it has fewer than 2^22 entries; beyond, the
// candidates count as 2^32 - 1.  Each value is capped at cap.
__device__ __forceinline__ void load16_pack(const uint64_t* pack, const uint32_t* add, int64_t n, int64_t i,
                                            int seg, uint32_t cap, uint32_t v[16]) {
  uint32_t w[16];
  load16_raw(add, n, i, w);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const uint64_t q = (i + k < n) ? pack[i + k] : 0ull;
    const uint64_t cnt = (uint64_t)(uint32_t)q + w[k];
    const uint32_t x = seg == 0 ? (uint32_t)min(cnt, 0xffffffffull)
                                : (cnt >= (1ull << 22) ? 0xffffffffu : (uint32_t)(q >> 32));
    v[k] = min(x, cap);
  }
}

// Up to kMaxImages scans of n values each (input, output and where the
// total goes per segment), nb workgroups per segment.  Every value is first
// capped at the segment's cap; a saturating segment (bit in sat) clamps its
// prefixes at 2^32 - 1 instead of raising the overflow bit.
struct ScanSegs {
  const uint32_t* in[kMaxImages];
  // or, when pack is set, two segments read from packed tile counts (see
  // load16_pack)
  const uint64_t* pack;
  const uint32_t* pack_add;
  uint32_t* out[kMaxImages];
  uint32_t* total[kMaxImages];
  uint32_t* max_out[kMaxImages];  // largest value of the segment, or null
  uint32_t cap[kMaxImages];
  uint32_t sat;
  int64_t n;
  int64_t nb;
  int32_t nseg;
};

__global__ void __launch_bounds__(kBlock) scan_reduce_kernel(ScanSegs sg, uint64_t* partial) {
  __shared__ uint64_t s_w[kWaves];
  const int seg = (int)(blockIdx.x / sg.nb);
  const int64_t b = (int64_t)blockIdx.x - (int64_t)seg * sg.nb;
  const int64_t i = b * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[16];
  if (sg.pack)
    load16_pack(sg.pack, sg.pack_add, sg.n, i, seg, sg.cap[seg], v);
  else
    load16(sg.in[seg], sg.n, i, sg.cap[seg], v);
  uint64_t s = 0;
  uint32_t m = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    s += v[k];
    m = max(m, v[k]);
  }
  uint64_t total;
  block_exclusive_scan<uint64_t>(s, s_w, total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
  if (sg.max_out[seg] != nullptr) {  // the spine takes the largest of these
    __shared__ uint32_t s_m[kWaves];
    m = block_max(m, s_m);
    if (threadIdx.x == 0) partial[(int64_t)sg.nb * sg.nseg + 2 + blockIdx.x] = m;
  }
}

// One workgroup per segment: exclusive scan of its per-tile partial sums,
// and the segment total (2^32 or more raises the overflow bit).
__global__ void __launch_bounds__(kBlock) scan_spine_kernel(ScanSegs sg, uint64_t* partial,
                                                             uint32_t* status) {
  __shared__ uint64_t s_w[kWaves];
  __shared__ uint32_t s_m[kWaves];
  uint64_t* part = partial + (int64_t)blockIdx.x * sg.nb;
  const uint64_t* pmax = partial + (int64_t)sg.nb * sg.nseg + 2 + (int64_t)blockIdx.x * sg.nb;
  const bool want_max = sg.max_out[blockIdx.x] != nullptr;
  uint64_t carry = 0;
  uint32_t m = 0;
  for (int64_t base = 0; base < sg.nb; base += kBlock) {
    const int64_t q = base + threadIdx.x;
    const uint64_t x = q < sg.nb ? part[q] : 0;
    if (want_max && q < sg.nb) m = max(m, (uint32_t)pmax[q]);
    uint64_t total;
    const uint64_t e = block_exclusive_scan<uint64_t>(x, s_w, total);
    if (q < sg.nb) part[q] = carry + e;
    carry += total;
  }
  if (want_max) {
    m = block_max(m, s_m);
    if (threadIdx.x == 0) *sg.max_out[blockIdx.x] = m;
  }
  if (threadIdx.x == 0) {
    const bool sat = (sg.sat >> blockIdx.x) & 1u;
    *sg.total[blockIdx.x] = (uint32_t)min(carry, 0xffffffffull);
    if (carry > 0xffffffffull && status && !sat) atomicOr(status, kStatusOverflow);
  }
}

__global__ void __launch_bounds__(kBlock) scan_apply_kernel(ScanSegs sg, const uint64_t* partial) {
  __shared__ uint64_t s_w[kWaves];
  const int seg = (int)(blockIdx.x / sg.nb);
  const int64_t b = (int64_t)blockIdx.x - (int64_t)seg * sg.nb;
  const int64_t i = b * kScanTile + (int64_t)threadIdx.x * kScanItems;
  const int64_t n = sg.n;
  uint32_t* out = sg.out[seg];
  uint32_t v[16];
  if (sg.pack)
    load16_pack(sg.pack, sg.pack_add, n, i, seg, sg.cap[seg], v);
  else
    load16(sg.in[seg], n, i, sg.cap[seg], v);
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += v[k];
  uint64_t total;
  uint64_t run = block_exclusive_scan<uint64_t>(s, s_w, total) + partial[blockIdx.x];
  const uint64_t top = ((sg.sat >> seg) & 1u) ? 0xffffffffull : ~0ull;
  uint32_t o[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    o[k] = (uint32_t)min(run, top);
    run += v[k];
  }
  if (i + 16 <= n) {
    uint4* p = reinterpret_cast<uint4*>(out + i);
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = make_uint4(o[4 * k], o[4 * k + 1], o[4 * k + 2], o[4 * k + 3]);
  } else {
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (i + k < n) out[i + k] = o[k];
  }
}

// ---------------------------------------------------------------------------
// batched sampling
// ---------------------------------------------------------------------------
// The setup and scatter chunks of all meshes, numbered mesh after mesh.
__global__ void __launch_bounds__(kBinBlock) batch_setup_kernel(BatchDevice B) {
  const int mi = segment_of(B.tri_block_start, B.n_meshes, (uint32_t)blockIdx.x);
  const BatchMesh& bm = B.meshes[mi];
  const uint32_t chunk = blockIdx.x - B.tri_block_start[mi];
  const int64_t t0 = (int64_t)chunk * kBinChunkTris;
  setup_count_chunk(bm.m, bm.nimg, [&](int k) -> const Image& { return B.images[bm.img[k]]; }, t0,
                    min(t0 + kBinChunkTris, bm.m.n_tris), chunk);
}

__global__ void __launch_bounds__(kBinBlock) batch_bin_kernel(BatchDevice B) {
  const int mi = segment_of(B.tri_block_start, B.n_meshes, (uint32_t)blockIdx.x);
  const BatchMesh& bm = B.meshes[mi];
  const uint32_t chunk = blockIdx.x - B.tri_block_start[mi];
  const int64_t t0 = (int64_t)chunk * kBinChunkTris;
  scatter_chunk(bm.m, bm.nimg, [&](int k) -> const Image& { return B.images[bm.img[k]]; }, t0,
                min(t0 + kBinChunkTris, bm.m.n_tris), chunk);
}

// Persistent workgroups take items from a counter, kGrab at a time, until
// none are left; every workgroup reaches the exit.
constexpr uint32_t kGrab = 4;

struct ItemGrabber {
  uint32_t next = 0, left = 0;
  // the next item for the whole workgroup (all threads call it)
  __device__ uint32_t operator()(uint32_t* counter, uint32_t* s_item) {
    if (left == 0) {
      if (threadIdx.x == 0) *s_item = atomicAdd(counter, kGrab);
      __syncthreads();
      next = __builtin_amdgcn_readfirstlane(*s_item);  // uniform: scalar table loads
      __syncthreads();
      left = kGrab;
    }
    --left;
    return next++;
  }
};

// Tiles [t0, t1) of the batch (the images of one tile class), work counter
// `counter`, place runs of at most place_cap keys.
// (the occupancy of sample_kernel)
template <int kTilePix>
__global__ void __launch_bounds__(kBlock, sample_wgs_per_cu<kTilePix>())
    batch_sample_kernel(BatchDevice B, uint32_t n_tiles, uint32_t t0, uint32_t t1, int counter, int place_cap) {
  __shared__ uint32_t s_item;
  ItemGrabber grab;
  for (;;) {
    const uint32_t item = t0 + grab(&B.work[counter], &s_item);
    if (item >= t1) break;
    const int k = __builtin_amdgcn_readfirstlane(segment_of(B.tile_start, B.n_images, item));
    sample_tile<kTilePix>(B.images[k], (int)(item - B.tile_start[k]), item, B.plan, n_tiles, place_cap);
    __syncthreads();  // the next item reuses the tile's LDS
  }
}

// Place items of the batch, in launch order, from the scanned plan.
__global__ void __launch_bounds__(kBlock) batch_plan_items_kernel(BatchDevice B, uint32_t n_tiles) {
  const uint32_t gt = blockIdx.x * kBlock + threadIdx.x;
  if (gt >= n_tiles) return;
  const uint32_t kd = B.plan[gt + 1] - B.plan[gt];
  const uint32_t ks = B.plan[n_tiles + gt + 1] - B.plan[n_tiles + gt];
  const uint32_t K = kd + ks;
  if (K == 0) return;
  const int k = segment_of(B.tile_start, B.n_images, gt);
  const Image& im = B.images[k];
  const int tile = (int)(gt - B.tile_start[k]);
  const uint32_t at = kd ? B.plan[gt] : B.plan[n_tiles + gt];
  PlaceItem it;
  it.gtile = gt;
  it.first = im.tile_stage[tile];
  it.hits = im.tile_hits[tile];
  PlaceItem* items = static_cast<PlaceItem*>(B.items);
  for (uint32_t j = 0; j < K; ++j) {
    it.part_parts = j | (K << 16);
    items[at + j] = it;
  }
}

// The place items of tiles [t0, t1): in launch order the items of tiles
// with several items come first, then those of single-item tiles, each part
// in tile order, so the class's items are two ranges.
// (the occupancy the persistent grid is sized for: seven workgroups per CU
// for small tiles, three for large ones)
template <int kTilePix>
__global__ void __launch_bounds__(kBlock, kTilePix <= kSmallTilePix ? 7 : 3)
    batch_place_kernel(BatchDevice B, uint32_t n_tiles, uint32_t t0, uint32_t t1, int counter) {
  __shared__ uint32_t s_item;
  const uint32_t a0 = B.plan[t0], a1 = B.plan[t1];
  const uint32_t b0 = B.plan[n_tiles + t0], b1 = B.plan[n_tiles + t1];
  const uint32_t n_items = (a1 - a0) + (b1 - b0);
  const PlaceItem* items = static_cast<const PlaceItem*>(B.items);
  ItemGrabber grab;
  for (;;) {
    const uint32_t q = grab(&B.work[counter], &s_item);
    if (q >= n_items) break;
    const uint32_t item = q < a1 - a0 ? a0 + q : b0 + (q - (a1 - a0));
    const PlaceItem it = items[item];
    const int k = __builtin_amdgcn_readfirstlane(segment_of(B.tile_start, B.n_images, it.gtile));
    const Image& im = B.images[k];
    if (im.depth == nullptr) continue;  // the image did not fit the output arena
    place_tile<kTilePix>(im, (int)(it.gtile - B.tile_start[k]), it.first, it.hits,
                         (int)(it.part_parts & 0xffffu), (int)(it.part_parts >> 16));
    // place_tile may return with waves still storing from its LDS stage
    // (one-run tiles): the next item reuses it
    __syncthreads();
  }
}

template <int kTilePix>
__global__ void __launch_bounds__(kBlock) batch_walk_kernel(BatchDevice B) {
  __shared__ uint32_t s_item;
  const uint32_t n = *B.walk_count;
  ItemGrabber grab;
  for (;;) {
    const uint32_t item = grab(&B.work[2], &s_item);
    if (item >= n) break;
    const uint32_t gt = B.walk_list[item];
    const int k = __builtin_amdgcn_readfirstlane(segment_of(B.tile_start, B.n_images, gt));
    const Image& im = B.images[k];
    if (im.depth == nullptr) continue;
    write_tile<kTilePix>(im, (int)(gt - B.tile_start[k]));
    __syncthreads();  // the next item reuses the tile's LDS
  }
}

// Start of every segment in the global exclusive prefix: partial sum of the
// segment's scan tile before its first slot.  One workgroup per segment.
__global__ void __launch_bounds__(kBlock) segment_base_kernel(const uint32_t* in, const uint64_t* partial,
                                                              const uint64_t* seg_start, uint64_t* seg_base) {
  __shared__ uint64_t s_w[kWaves];
  const uint64_t pos = seg_start[blockIdx.x];
  const uint64_t b = pos / kScanTile;
  uint64_t acc = 0;
  for (uint64_t i = b * kScanTile + threadIdx.x; i < pos; i += kBlock) acc += in[i];
  uint64_t total;
  block_exclusive_scan<uint64_t>(acc, s_w, total);
  if (threadIdx.x == 0) seg_base[blockIdx.x] = partial[b] + total;
}

// The workgroup finds the segment of its first value once; a thread whose 16
// values lie in one segment stores them as four 16-byte vectors.
__global__ void __launch_bounds__(kBlock) scan_apply_segmented_kernel(
    const uint32_t* in, int64_t n, const uint64_t* partial, const uint64_t* seg_start,
    const uint64_t* seg_base, int n_seg, uint32_t* out) {
  __shared__ uint64_t s_w[kWaves];
  __shared__ int s_seg;
  const int64_t i = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  if (threadIdx.x == 0) s_seg = segment_of(seg_start, n_seg, (uint64_t)blockIdx.x * kScanTile);
  uint32_t v[16];
  load16(in, n, i, 0xffffffffu, v);
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += v[k];
  uint64_t total;
  uint64_t run = block_exclusive_scan<uint64_t>(s, s_w, total) + partial[blockIdx.x];  // (barriers)
  if (i >= n) return;
  int seg = s_seg;
  while (seg + 1 < n_seg && seg_start[seg + 1] <= (uint64_t)i) ++seg;
  if (i + 16 <= n && (seg + 1 >= n_seg || seg_start[seg + 1] >= (uint64_t)(i + 16))) {
    const uint64_t base = seg_base[seg];
    uint32_t o[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      o[k] = (uint32_t)(run - base);
      run += v[k];
    }
    uint4* p = reinterpret_cast<uint4*>(out + i);
#pragma unroll
    for (int k = 0; k < 4; ++k) p[k] = make_uint4(o[4 * k], o[4 * k + 1], o[4 * k + 2], o[4 * k + 3]);
    return;
  }
  for (int k = 0; k < 16 && i + k < n; ++k) {
    while (seg + 1 < n_seg && seg_start[seg + 1] <= (uint64_t)(i + k)) ++seg;
    out[i + k] = (uint32_t)(run - seg_base[seg]);
    run += v[k];
  }
}

// One workgroup per image: its largest count (from its tiles' largest),
// sample count, placement in the output arena (or the capacity flag), host
// summary.
__global__ void __launch_bounds__(kBlock) batch_finish_counts_kernel(BatchDevice B) {
  __shared__ uint32_t s_m[kWaves];
  const int k = blockIdx.x;
  if (k >= B.n_images) return;
  Image& im = B.images[k];
  uint32_t m = 0;
  for (uint32_t t = B.tile_start[k] + threadIdx.x; t < B.tile_start[k + 1]; t += kBlock)
    m = max(m, B.tile_max[t]);
  m = block_max(m, s_m);
  if (threadIdx.x != 0) return;
  *im.max_layers = m;
  if (k == 0) {
    B.host_out[0] = *B.status;
    B.host_out[1] = *B.tile_total;
    uint32_t* tail = B.host_out + 4 + 4 * (size_t)B.n_images;
    tail[0] = *B.region_total;
    tail[1] = 0u;
    tail[2] = *B.walk_count;
  }
  {
    const uint64_t n = im.offsets[(size_t)im.w * im.w];
    const uint64_t base = B.sample_base[k];
    const bool fits = base + n <= B.sample_cap && (uint64_t)*B.tile_total <= B.list_cap;
    im.depth = fits ? B.depth + base : nullptr;
    im.normal = (fits && B.normal) ? B.normal + 3 * base : nullptr;
    im.normal_rgb8 = (fits && B.normal_rgb8) ? B.normal_rgb8 + base : nullptr;
    im.tri = fits ? B.tri + base : nullptr;
    uint32_t* h = B.host_out + 4 + 4 * (size_t)k;
    h[0] = (uint32_t)n;
    h[1] = (uint32_t)base;
    h[2] = (uint32_t)(base >> 32);
    h[3] = m;  // the host compares n and base with the capacities
  }
  __threadfence_system();
}

struct GatherArgs {
  const uint32_t* src[kMaxGather];
  int n;
};

// Copies a few scattered device words into pinned host memory in one launch.
__global__ void gather_kernel(GatherArgs g, uint32_t* dst) {
  const int k = threadIdx.x;
  if (k < g.n) dst[k] = *g.src[k];
  __threadfence_system();
}

inline unsigned grid_for(int64_t n, int per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static unsigned persistent_grid(uint32_t n_items, int per_cu) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  const uint32_t g = (uint32_t)(cus * per_cu);
  return n_items < g ? (n_items > 0 ? n_items : 1) : g;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  unsigned g = grid_for(n, kBlock);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(g), dim3(kBlock), 0, s, p, value, n);
  return hipGetLastError();
}

hipError_t launch_setup(const MeshSetup& m, const ImageSet& set, hipStream_t s) {
  if (m.n_tris <= 0) return hipSuccess;
  hipLaunchKernelGGL(setup_kernel, dim3(grid_for(m.n_tris, kBinChunkTris)), dim3(kBinBlock), 0, s, m, set);
  return hipGetLastError();
}

hipError_t launch_bin_scatter(const MeshSetup& m, const ImageSet& set, hipStream_t s) {
  if (set.n == 0 || m.n_tris <= 0) return hipSuccess;
  hipLaunchKernelGGL(bin_kernel, dim3(grid_for(m.n_tris, kBinChunkTris)), dim3(kBinBlock), 0, s, m, set);
  return hipGetLastError();
}

static bool small_tiles(const ImageSet& set) {
  for (int k = 0; k < set.n; ++k)
    if (set.img[k].tw * set.img[k].th > kSmallTilePix) return false;
  return true;
}

hipError_t launch_sample(const ImageSet& set, hipStream_t s) {
  const uint32_t blocks = set.tile_start[set.n];
  if (blocks == 0) return hipSuccess;
  if (small_tiles(set))
    hipLaunchKernelGGL(sample_kernel<kSmallTilePix>, dim3(blocks), dim3(kBlock), 0, s, set);
  else
    hipLaunchKernelGGL(sample_kernel<kMaxTilePix>, dim3(blocks), dim3(kBlock), 0, s, set);
  return hipGetLastError();
}

int place_stage_cap(int tile_pix) {
  return stage_cap(tile_pix <= kSmallTilePix ? kSmallTilePix : kMaxTilePix);
}

int max_place_items_per_tile(int tile_pix, uint32_t stage_layers) {
  const int pix = tile_pix <= kSmallTilePix ? kSmallTilePix : kMaxTilePix;
  return (int)(((uint64_t)stage_layers * pix + stage_cap(pix) - 1) / stage_cap(pix));
}

uint32_t stage_layers_for(uint32_t max_layers_seen) {
  uint32_t l = kMinStageLayers;
  while (l < max_layers_seen && l < kMaxStageLayers) l <<= 1;
  return l;
}

hipError_t launch_plan_items(const ImageSet& set, void* items, void* scratch, uint32_t* status,
                             hipStream_t s) {
  const uint32_t n = set.tile_start[set.n];
  if (n == 0) return hipSuccess;
  hipError_t e = launch_scan(set.plan, set.plan, 2 * (int64_t)n, scratch, status, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(plan_items_kernel, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, set,
                     static_cast<PlaceItem*>(items));
  return hipGetLastError();
}

hipError_t launch_place(const ImageSet& set, const void* items, uint32_t n_items, uint32_t* counter,
                        uint32_t n_walk, hipStream_t s) {
  const bool small = small_tiles(set);
  const PlaceItem* it = static_cast<const PlaceItem*>(items);
  if (n_items > 0) {
    if (small)
      hipLaunchKernelGGL(place_kernel<kSmallTilePix>, dim3(n_items), dim3(kBlock), 0, s, set, it);
    else
      hipLaunchKernelGGL(place_kernel<kMaxTilePix>, dim3(n_items), dim3(kBlock), 0, s, set, it);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (n_walk == 0) return hipSuccess;
  hipError_t e = launch_fill_u32(counter, 0u, 1, s);
  if (e != hipSuccess) return e;
  const unsigned wgrid = persistent_grid(n_walk, small ? 4 : 2);
  const uint32_t* list = set.img[0].walk_list;
  if (small)
    hipLaunchKernelGGL(walk_kernel<kSmallTilePix>, dim3(wgrid), dim3(kBlock), 0, s, set, list, n_walk, counter);
  else
    hipLaunchKernelGGL(walk_kernel<kMaxTilePix>, dim3(wgrid), dim3(kBlock), 0, s, set, list, n_walk, counter);
  return hipGetLastError();
}

hipError_t launch_gather(const uint32_t* const* src, int n, uint32_t* host_dst, hipStream_t s) {
  if (n < 0 || n > kMaxGather) return hipErrorInvalidValue;
  GatherArgs g;
  g.n = n;
  for (int k = 0; k < kMaxGather; ++k) g.src[k] = k < n ? src[k] : nullptr;
  hipLaunchKernelGGL(gather_kernel, dim3(1), dim3(64), 0, s, g, host_dst);
  return hipGetLastError();
}

hipError_t launch_batch_setup(const BatchDevice& b, uint32_t chunks, hipStream_t s) {
  if (chunks == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_setup_kernel, dim3(chunks), dim3(kBinBlock), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_batch_scatter(const BatchDevice& b, uint32_t chunks, hipStream_t s) {
  if (chunks == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_bin_kernel, dim3(chunks), dim3(kBinBlock), 0, s, b);
  return hipGetLastError();
}

hipError_t launch_batch_sample(const BatchDevice& b, uint32_t n_tiles, uint32_t n_small, hipStream_t s) {
  if (n_small > 0)
    hipLaunchKernelGGL(batch_sample_kernel<kSmallTilePix>, dim3(persistent_grid(n_small, sample_wgs_per_cu<kSmallTilePix>())), dim3(kBlock), 0, s,
                       b, n_tiles, 0u, n_small, 0, place_stage_cap(kSmallTilePix));
  if (n_tiles > n_small)
    hipLaunchKernelGGL(batch_sample_kernel<kMaxTilePix>, dim3(persistent_grid(n_tiles - n_small, sample_wgs_per_cu<kMaxTilePix>())), dim3(kBlock),
                       0, s, b, n_tiles, n_small, n_tiles, 3, place_stage_cap(kMaxTilePix));
  return hipGetLastError();
}

hipError_t launch_batch_place(const BatchDevice& b, uint32_t n_tiles, uint32_t n_small, void* scratch,
                              hipStream_t s) {
  if (n_tiles == 0) return hipSuccess;
  hipError_t e = launch_scan(b.plan, b.plan, 2 * (int64_t)n_tiles, scratch, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batch_plan_items_kernel, dim3(grid_for(n_tiles, kBlock)), dim3(kBlock), 0, s, b, n_tiles);
  if (n_small > 0)
    hipLaunchKernelGGL(batch_place_kernel<kSmallTilePix>, dim3(persistent_grid(2 * n_small, 7)), dim3(kBlock), 0,
                       s, b, n_tiles, 0u, n_small, 1);
  if (n_tiles > n_small)
    hipLaunchKernelGGL(batch_place_kernel<kMaxTilePix>, dim3(persistent_grid(2 * (n_tiles - n_small), 3)),
                       dim3(kBlock), 0, s, b, n_tiles, n_small, n_tiles, 4);
  // tiles walked again: one build for all (the large one as soon as any
  // image has large tiles)
  if (n_tiles == n_small)
    hipLaunchKernelGGL(batch_walk_kernel<kSmallTilePix>, dim3(persistent_grid(n_tiles, 4)), dim3(kBlock), 0,
                       s, b);
  else
    hipLaunchKernelGGL(batch_walk_kernel<kMaxTilePix>, dim3(persistent_grid(n_tiles, 2)), dim3(kBlock), 0,
                       s, b);
  return hipGetLastError();
}

hipError_t launch_batch_pixel_scan(const BatchDevice& b, const uint32_t* counts, uint32_t* offsets,
                                   int64_t n_slots, void* scratch, hipStream_t s) {
  uint64_t* partial = static_cast<uint64_t*>(scratch);
  const int64_t nb = (n_slots + kScanTile - 1) / kScanTile;
  if (nb == 0 || b.n_images == 0) return hipSuccess;
  ScanSegs sg{};
  sg.in[0] = counts;
  sg.cap[0] = 0xffffffffu;
  sg.n = n_slots;
  sg.nb = nb;
  sg.nseg = 1;
  hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, sg, partial);
  // the spine's grand total goes one past the partial sums; its overflow
  // check does not apply to a batch, whose images are checked one by one
  sg.total[0] = reinterpret_cast<uint32_t*>(partial + nb);
  hipLaunchKernelGGL(scan_spine_kernel, dim3(1), dim3(kBlock), 0, s, sg, partial, (uint32_t*)nullptr);
  hipLaunchKernelGGL(segment_base_kernel, dim3((unsigned)b.n_images), dim3(kBlock), 0, s, counts, partial,
                     b.seg_start, b.sample_base);
  hipLaunchKernelGGL(scan_apply_segmented_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, counts, n_slots,
                     partial, b.seg_start, b.sample_base, b.n_images, offsets);
  return hipGetLastError();
}

hipError_t launch_batch_finish_counts(const BatchDevice& b, hipStream_t s) {
  if (b.n_images == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_finish_counts_kernel, dim3((unsigned)b.n_images), dim3(kBlock), 0, s, b);
  return hipGetLastError();
}

// partial sums of the workgroups, two spare words, then their largest values
size_t scan_scratch_bytes(int64_t n, int nseg) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  return (size_t)(2 * (nb > 0 ? nb : 1) * (nseg > 0 ? nseg : 1) + 2) * sizeof(uint64_t);
}

static hipError_t run_scan(const ScanSegs& sg, void* scratch, uint32_t* status, hipStream_t s) {
  uint64_t* partial = static_cast<uint64_t*>(scratch);
  const unsigned blocks = (unsigned)(sg.nb * sg.nseg);
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(blocks), dim3(kBlock), 0, s, sg, partial);
  hipLaunchKernelGGL(scan_spine_kernel, dim3((unsigned)sg.nseg), dim3(kBlock), 0, s, sg, partial, status);
  hipLaunchKernelGGL(scan_apply_kernel, dim3(blocks), dim3(kBlock), 0, s, sg, partial);
  return hipGetLastError();
}

hipError_t launch_scan_segments(const uint32_t* const* in, uint32_t* const* out, int nseg, int64_t n,
                                void* scratch, uint32_t* status, hipStream_t s, uint32_t* const* max_out) {
  if (nseg < 1 || nseg > kMaxImages) return hipErrorInvalidValue;
  if (n <= 0) {
    for (int k = 0; k < nseg; ++k) {
      hipError_t e = launch_fill_u32(out[k], 0u, 1, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  ScanSegs sg{};
  for (int k = 0; k < nseg; ++k) {
    sg.in[k] = in[k];
    sg.out[k] = out[k];
    sg.total[k] = out[k] + n;
    sg.max_out[k] = max_out ? max_out[k] : nullptr;
    sg.cap[k] = 0xffffffffu;
  }
  sg.n = n;
  sg.nb = (n + kScanTile - 1) / kScanTile;
  sg.nseg = nseg;
  return run_scan(sg, scratch, status, s);
}

hipError_t launch_tile_scan(const uint64_t* tile_pack, const uint32_t* tile_ovf, uint32_t* tile_cnt,
                            uint32_t* tile_region, int64_t n, uint32_t region_cap, void* scratch, uint32_t* status,
                            hipStream_t s) {
  if (n <= 0) {
    hipError_t e = launch_fill_u32(tile_cnt, 0u, 1, s);
    return e != hipSuccess ? e : launch_fill_u32(tile_region, 0u, 1, s);
  }
  ScanSegs sg{};
  sg.in[0] = tile_cnt;
  sg.pack = tile_pack;
  sg.pack_add = tile_ovf;
  sg.out[0] = tile_cnt;
  sg.total[0] = tile_cnt + n;
  sg.cap[0] = 0xffffffffu;
  sg.in[1] = tile_region;
  sg.out[1] = tile_region;
  sg.total[1] = tile_region + n;
  sg.cap[1] = region_cap;
  sg.sat = 2u;
  sg.n = n;
  sg.nb = (n + kScanTile - 1) / kScanTile;
  sg.nseg = 2;
  return run_scan(sg, scratch, status, s);
}

hipError_t launch_scan(const uint32_t* in, uint32_t* out, int64_t n, void* scratch,
                       uint32_t* status, hipStream_t s, uint32_t* max_out) {
  return launch_scan_segments(&in, &out, 1, n, scratch, status, s, max_out ? &max_out : nullptr);
}

}  // namespace ldni
