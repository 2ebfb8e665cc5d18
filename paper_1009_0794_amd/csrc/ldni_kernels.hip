// ldni_kernels.hip -- gfx950 kernels of the LDNI sampler.
//
// Pipeline per call (every kernel covers all requested axes in one launch):
//   setup      triangle-parallel: gather and validate vertices, float64 face
//              normal, candidate pixel rectangle on each image
//   bin_count  triangle-parallel: entries per screen tile (global atomics)
//   scan       tile counts -> tile offsets
//   bin_scatter  triangle ids into per-tile lists
//   count      one workgroup per tile: exact coverage test of every candidate
//              (triangle, pixel centre), LDS per-pixel atomic counters ->
//              counts[w*w] and the largest per-pixel count
//   scan       counts -> offsets[w*w+1]
//   write      one workgroup per tile: the same coverage test, float64 depth,
//              (depth, triangle) keys staged in LDS at their pixel's slots,
//              per-pixel sort, then contiguous row-range stores of depth,
//              normal and triangle id.  A tile row whose samples do not fit
//              in LDS is written straight to its output range and sorted
//              there.
// Nothing here is a dense contraction, so there is no MFMA: the work is
// integer/FP64 ALU plus HBM traffic.
#pragma clang fp contract(off)

#include "ldni_internal.hpp"

namespace ldni {
namespace {

constexpr int kBlock = 256;          // 4 wave64 per workgroup
constexpr int kWaves = kBlock / 64;
constexpr int kMaxTilePix = 1024;    // tw * th
constexpr int kMaxTileW = 256;
constexpr int kMaxTileH = 64;
constexpr int kStageCap = 6144;      // (depth, tri) keys staged per tile chunk

// ---------------------------------------------------------------------------
// pixel centres and candidate rectangles
// ---------------------------------------------------------------------------
__device__ __forceinline__ float pixel_centre(double lo, double h, int i) {
  return (float)(lo + ((double)i + 0.5) * h);
}

// Smallest i in [0, w] whose centre is >= x (centres are non-decreasing in i).
// The float64 estimate is corrected against the exact float32 centres.
__device__ int first_centre_at_or_above(double lo, double h, int w, float x) {
  double t = ((double)x - lo) / h - 0.5;
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

struct Coverage {
  double e_ab, e_bc, e_ca;
  bool hit;
};

__device__ __forceinline__ Coverage cover(float au, float av, float bu, float bv, float cu,
                                          float cv, float ru, float rv) {
  Coverage c;
  const float pau = au - ru, pav = av - rv;
  const float pbu = bu - ru, pbv = bv - rv;
  const float pcu = cu - ru, pcv = cv - rv;
  const int s0 = orient(pau, pav, pbu, pbv, c.e_ab);
  const int s1 = orient(pbu, pbv, pcu, pcv, c.e_bc);
  const int s2 = orient(pcu, pcv, pau, pav, c.e_ca);
  c.hit = (s0 != 0) & (s0 == s1) & (s1 == s2);
  return c;
}

// Depth of the hit from lo_a: the axis coordinate interpolated with the
// barycentric weights E_BC, E_CA, E_AB over their sum, in float64.
__device__ __forceinline__ float hit_depth(const Coverage& c, float az, float bz, float cz,
                                           double lo_a) {
  const double den = (c.e_ab + c.e_bc) + c.e_ca;
  const double num = c.e_ca * ((double)bz - (double)az) + c.e_ab * ((double)cz - (double)az);
  const double z = (double)az + num / den;
  float d = (float)(z - lo_a);
  if (d == 0.0f) d = 0.0f;
  return d;
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

// Map a workgroup to (image, tile).
__device__ __forceinline__ int image_of_block(const ImageSet& set, uint32_t b) {
  int k = 0;
  while (k + 1 < set.n && b >= set.tile_start[k + 1]) ++k;
  return k;
}

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) setup_kernel(MeshSetup m, ImageSet set) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= m.n_tris) return;
  const int32_t ia = m.tris[3 * t], ib = m.tris[3 * t + 1], ic = m.tris[3 * t + 2];
  float P[9];
  const bool idx_ok = ia >= 0 && ia < m.n_verts && ib >= 0 && ib < m.n_verts && ic >= 0 &&
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
  } else {
    atomicOr(m.status, kStatusBadIndex);
  }
  if (!ok) {
    // an invalid triangle becomes a point: never hit, and the call fails
#pragma unroll
    for (int c = 0; c < 9; ++c) P[c] = 0.0f;
  }
  float* soup = m.soup + 9 * t;
#pragma unroll
  for (int c = 0; c < 9; ++c) soup[c] = P[c];

  // unit face normal (B-A)x(C-A) in float64
  const double e1x = (double)P[3] - (double)P[0], e1y = (double)P[4] - (double)P[1],
               e1z = (double)P[5] - (double)P[2];
  const double e2x = (double)P[6] - (double)P[0], e2y = (double)P[7] - (double)P[1],
               e2z = (double)P[8] - (double)P[2];
  const double nx = e1y * e2z - e1z * e2y;
  const double ny = e1z * e2x - e1x * e2z;
  const double nz = e1x * e2y - e1y * e2x;
  const double len = sqrt((nx * nx + ny * ny) + nz * nz);
  float* tn = m.tnorm + 3 * t;
  if (len > 0.0) {
    tn[0] = (float)(nx / len);
    tn[1] = (float)(ny / len);
    tn[2] = (float)(nz / len);
  } else {
    tn[0] = tn[1] = tn[2] = 0.0f;
  }

  for (int k = 0; k < set.n; ++k) {
    const Image& im = set.img[k];
    const float umin = fminf(fminf(P[im.u], P[3 + im.u]), P[6 + im.u]);
    const float umax = fmaxf(fmaxf(P[im.u], P[3 + im.u]), P[6 + im.u]);
    const float vmin = fminf(fminf(P[im.v], P[3 + im.v]), P[6 + im.v]);
    const float vmax = fmaxf(fmaxf(P[im.v], P[3 + im.v]), P[6 + im.v]);
    Rect r;
    const int i0 = first_centre_at_or_above(im.lo_u, im.h_u, im.w, umin);
    const int i1 = first_centre_at_or_above(im.lo_u, im.h_u, im.w, umax);
    const int j0 = first_centre_at_or_above(im.lo_v, im.h_v, im.w, vmin);
    const int j1 = first_centre_at_or_above(im.lo_v, im.h_v, im.w, vmax);
    if (i0 < i1 && j0 < j1) {
      r.i0 = (int16_t)i0; r.i1 = (int16_t)i1; r.j0 = (int16_t)j0; r.j1 = (int16_t)j1;
    } else {
      r.i0 = r.i1 = r.j0 = r.j1 = 0;
    }
    m.rect[k][t] = r;
  }
}

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------
template <bool kScatter>
__global__ void __launch_bounds__(kBlock) bin_kernel(ImageSet set) {
  const Image& im = set.img[blockIdx.y];
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= im.n_tris) return;
  const Rect r = im.rect[t];
  if (r.i0 >= r.i1 || r.j0 >= r.j1) return;
  const int tx0 = r.i0 / im.tw, tx1 = (r.i1 - 1) / im.tw;
  const int ty0 = r.j0 / im.th, ty1 = (r.j1 - 1) / im.th;
  for (int ty = ty0; ty <= ty1; ++ty)
    for (int tx = tx0; tx <= tx1; ++tx) {
      const int tile = ty * im.ntx + tx;
      if (kScatter) {
        const uint32_t slot = atomicAdd(&im.tile_cur[tile], 1u);
        im.tile_list[(size_t)im.tile_cnt[tile] + slot] = (int32_t)t;
      } else {
        atomicAdd(&im.tile_cnt[tile], 1u);
      }
    }
}

// ---------------------------------------------------------------------------
// candidate enumeration inside one tile
// ---------------------------------------------------------------------------
// A chunk of up to kBlock tile-list entries is loaded into LDS together with
// the prefix sum of their candidate counts; every thread then walks the
// flattened (entry, pixel) candidates with a stride of kBlock, so large and
// small triangles share the work evenly.
template <int kNV>
struct ChunkLds {
  int32_t tri[kBlock];
  int32_t start[kBlock];
  int32_t box[kBlock];          // px0 | width << 10 | py0 << 20
  float vtx[kNV][kBlock];       // (au, av, bu, bv, cu, cv[, az, bz, cz])
  int32_t wave_tmp[kWaves];
};

struct TileGeom {
  int x0, y0, cw, ch;  // tile origin and extent in pixels
  int tile;            // tile index within its image
};

// Calls on_hit(k, px, py, cov) for every candidate of rows [r0, r1) of the
// tile that is covered; k indexes the chunk arrays in L.
template <int kNV, class OnHit>
__device__ void tile_candidates(const Image& im, const TileGeom& g, int r0, int r1,
                                ChunkLds<kNV>& L, const float* s_cu, const float* s_cv,
                                OnHit&& on_hit) {
  const uint32_t e_begin = im.tile_cnt[g.tile], e_end = im.tile_cnt[g.tile + 1];
  const int ya = g.y0 + r0, yb = g.y0 + r1;
  for (uint32_t base = e_begin; base < e_end; base += kBlock) {
    const int m = (int)min((uint32_t)kBlock, e_end - base);
    const int k = threadIdx.x;
    int nc = 0;
    if (k < m) {
      const int32_t t = im.tile_list[base + k];
      const Rect r = im.rect[t];
      const int px0 = max((int)r.i0, g.x0) - g.x0, px1 = min((int)r.i1, g.x0 + g.cw) - g.x0;
      const int py0 = max((int)r.j0, ya) - g.y0, py1 = min((int)r.j1, yb) - g.y0;
      if (px1 > px0 && py1 > py0) nc = (px1 - px0) * (py1 - py0);
      L.tri[k] = t;
      L.box[k] = px0 | ((px1 - px0) << 10) | (py0 << 20);
      const float* s = im.soup + 9 * (int64_t)t;
      L.vtx[0][k] = s[im.u];
      L.vtx[1][k] = s[im.v];
      L.vtx[2][k] = s[3 + im.u];
      L.vtx[3][k] = s[3 + im.v];
      L.vtx[4][k] = s[6 + im.u];
      L.vtx[5][k] = s[6 + im.v];
      if (kNV == 9) {
        L.vtx[kNV == 9 ? 6 : 0][k] = s[im.a];
        L.vtx[kNV == 9 ? 7 : 0][k] = s[3 + im.a];
        L.vtx[kNV == 9 ? 8 : 0][k] = s[6 + im.a];
      }
    }
    int total;
    const int excl = block_exclusive_scan<int>(nc, L.wave_tmp, total);
    if (k < m) L.start[k] = excl;
    __syncthreads();
    for (int c = threadIdx.x; c < total; c += kBlock) {
      // owner: the last entry whose start is <= c
      int lo = 0, hi = m - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.start[mid] <= c) lo = mid; else hi = mid - 1;
      }
      const int e = lo;
      const int bx = L.box[e];
      const int px0 = bx & 1023, width = (bx >> 10) & 1023, py0 = bx >> 20;
      const int local = c - L.start[e];
      const int row = local / width;
      const int px = px0 + (local - row * width);
      const int py = py0 + row;
      const Coverage cov = cover(L.vtx[0][e], L.vtx[1][e], L.vtx[2][e], L.vtx[3][e],
                                 L.vtx[4][e], L.vtx[5][e], s_cu[px], s_cv[py]);
      if (cov.hit) on_hit(e, px, py, cov);
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

// ---------------------------------------------------------------------------
// count pass
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) count_kernel(ImageSet set) {
  __shared__ uint32_t s_cnt[kMaxTilePix];
  __shared__ float s_cu[kMaxTileW];
  __shared__ float s_cv[kMaxTileH];
  __shared__ ChunkLds<6> L;
  __shared__ uint32_t s_red[kWaves];

  const int k_img = image_of_block(set, blockIdx.x);
  const Image& im = set.img[k_img];
  const TileGeom g = tile_geom(im, (int)(blockIdx.x - set.tile_start[k_img]));
  const int npix = g.cw * g.ch;

  for (int q = threadIdx.x; q < im.tw * im.th; q += kBlock) s_cnt[q] = 0;
  for (int q = threadIdx.x; q < g.cw; q += kBlock) s_cu[q] = pixel_centre(im.lo_u, im.h_u, g.x0 + q);
  for (int q = threadIdx.x; q < g.ch; q += kBlock) s_cv[q] = pixel_centre(im.lo_v, im.h_v, g.y0 + q);
  __syncthreads();

  const int tw = im.tw;
  tile_candidates<6>(im, g, 0, g.ch, L, s_cu, s_cv,
                     [&](int, int px, int py, const Coverage&) {
                       atomicAdd(&s_cnt[py * tw + px], 1u);
                     });

  uint32_t mx = 0;
  for (int q = threadIdx.x; q < npix; q += kBlock) {
    const int py = q / g.cw, px = q - py * g.cw;
    const uint32_t c = s_cnt[py * tw + px];
    mx = max(mx, c);
    im.counts[(size_t)(g.y0 + py) * im.w + g.x0 + px] = c;
  }
  mx = block_max(mx, s_red);
  if (threadIdx.x == 0 && mx > 0) atomicMax(im.max_layers, mx);
}

// ---------------------------------------------------------------------------
// write pass
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) write_kernel(ImageSet set) {
  __shared__ uint64_t s_keys[kStageCap];
  __shared__ uint32_t s_rel[kMaxTilePix];   // pixel start within its row's range
  __shared__ uint32_t s_pcnt[kMaxTilePix];  // samples of the pixel
  __shared__ uint32_t s_cur[kMaxTilePix];   // fill cursor of the pixel
  __shared__ uint32_t s_rowbase[kMaxTileH]; // global offset of the row's first sample
  __shared__ uint32_t s_rowtot[kMaxTileH];
  __shared__ uint32_t s_stage[kMaxTileH + 1];  // LDS start of each row of the chunk
  __shared__ float s_cu[kMaxTileW];
  __shared__ float s_cv[kMaxTileH];
  __shared__ ChunkLds<9> L;
  __shared__ int s_chunk[3];                 // r1, global mode, chunk total

  const int k_img = image_of_block(set, blockIdx.x);
  const Image& im = set.img[k_img];
  const TileGeom g = tile_geom(im, (int)(blockIdx.x - set.tile_start[k_img]));
  const int tw = im.tw;
  const int npix = g.cw * g.ch;

  for (int q = threadIdx.x; q < g.cw; q += kBlock) s_cu[q] = pixel_centre(im.lo_u, im.h_u, g.x0 + q);
  for (int q = threadIdx.x; q < g.ch; q += kBlock) s_cv[q] = pixel_centre(im.lo_v, im.h_v, g.y0 + q);
  for (int q = threadIdx.x; q < g.ch; q += kBlock) {
    const size_t row0 = (size_t)(g.y0 + q) * im.w + g.x0;
    const uint32_t b = im.offsets[row0];
    s_rowbase[q] = b;
    s_rowtot[q] = im.offsets[row0 + g.cw] - b;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < npix; q += kBlock) {
    const int py = q / g.cw, px = q - py * g.cw;
    const size_t gp = (size_t)(g.y0 + py) * im.w + g.x0 + px;
    const uint32_t o = im.offsets[gp];
    s_rel[py * tw + px] = o - s_rowbase[py];
    s_pcnt[py * tw + px] = im.offsets[gp + 1] - o;
    s_cur[py * tw + px] = 0;
  }
  __syncthreads();

  int r0 = 0;
  while (r0 < g.ch) {
    if (threadIdx.x == 0) {
      int r1 = r0 + 1;
      uint64_t acc = s_rowtot[r0];
      const int global_mode = acc > (uint64_t)kStageCap;
      if (!global_mode)
        while (r1 < g.ch && acc + s_rowtot[r1] <= (uint64_t)kStageCap) acc += s_rowtot[r1++];
      uint32_t st = 0;
      for (int q = r0; q < r1; ++q) {
        s_stage[q - r0] = st;
        st += s_rowtot[q];
      }
      s_stage[r1 - r0] = st;
      s_chunk[0] = r1;
      s_chunk[1] = global_mode;
      s_chunk[2] = (int)st;
    }
    __syncthreads();
    const int r1 = s_chunk[0];
    const bool global_mode = s_chunk[1] != 0;
    const int chunk_total = s_chunk[2];
    if (chunk_total == 0) {  // nothing to write in these rows
      r0 = r1;
      __syncthreads();
      continue;
    }

    const double lo_a = im.lo_a;
    tile_candidates<9>(im, g, r0, r1, L, s_cu, s_cv,
                       [&](int e, int px, int py, const Coverage& cov) {
                         const int p = py * tw + px;
                         const uint32_t slot = atomicAdd(&s_cur[p], 1u);
                         if (slot >= s_pcnt[p]) {  // count and write passes disagree
                           atomicOr(im.status, kStatusOverflow);
                           return;
                         }
                         const float d = hit_depth(cov, L.vtx[6][e], L.vtx[7][e], L.vtx[8][e], lo_a);
                         const int32_t t = L.tri[e];
                         if (!global_mode) {
                           s_keys[s_stage[py - r0] + s_rel[p] + slot] = sample_key(d, t);
                         } else {
                           const size_t o = (size_t)s_rowbase[py] + s_rel[p] + slot;
                           im.depth[o] = d;
                           im.tri[o] = t;
                         }
                       });
    // tile_candidates ends with a barrier

    const int ncol = g.cw;
    const int nchunkpix = (r1 - r0) * ncol;
    if (!global_mode) {
      // per-pixel insertion sort of the staged keys
      for (int q = threadIdx.x; q < nchunkpix; q += kBlock) {
        const int py = r0 + q / ncol, px = q % ncol;
        const int p = py * tw + px;
        uint64_t* seg = s_keys + s_stage[py - r0] + s_rel[p];
        const uint32_t n = s_pcnt[p];
        for (uint32_t x = 1; x < n; ++x) {
          const uint64_t key = seg[x];
          uint32_t y = x;
          while (y > 0 && seg[y - 1] > key) {
            seg[y] = seg[y - 1];
            --y;
          }
          seg[y] = key;
        }
      }
      __syncthreads();
      // contiguous stores, row range by row range
      for (int s = threadIdx.x; s < chunk_total; s += kBlock) {
        int lo = 0, hi = r1 - r0 - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_stage[mid] <= (uint32_t)s) lo = mid; else hi = mid - 1;
        }
        const size_t o = (size_t)s_rowbase[r0 + lo] + (s - s_stage[lo]);
        const uint64_t key = s_keys[s];
        const int32_t t = (int32_t)(uint32_t)key;
        im.depth[o] = key_depth(key);
        im.tri[o] = t;
        const float* n = im.tnorm + 3 * (int64_t)t;
        float* dst = im.normal + 3 * o;
        dst[0] = n[0];
        dst[1] = n[1];
        dst[2] = n[2];
      }
    } else {
      // one oversized row: sort each pixel's range in place in global memory
      for (int q = threadIdx.x; q < ncol; q += kBlock) {
        const int p = r0 * tw + q;
        const size_t o = (size_t)s_rowbase[r0] + s_rel[p];
        const uint32_t n = s_pcnt[p];
        for (uint32_t x = 1; x < n; ++x) {
          const float dk = im.depth[o + x];
          const int32_t tk = im.tri[o + x];
          const uint64_t key = sample_key(dk, tk);
          uint32_t y = x;
          while (y > 0 && sample_key(im.depth[o + y - 1], im.tri[o + y - 1]) > key) {
            im.depth[o + y] = im.depth[o + y - 1];
            im.tri[o + y] = im.tri[o + y - 1];
            --y;
          }
          im.depth[o + y] = dk;
          im.tri[o + y] = tk;
        }
      }
      __syncthreads();
      for (int s = threadIdx.x; s < chunk_total; s += kBlock) {
        const size_t o = (size_t)s_rowbase[r0] + s;
        const int32_t t = im.tri[o];
        const float* n = im.tnorm + 3 * (int64_t)t;
        float* dst = im.normal + 3 * o;
        dst[0] = n[0];
        dst[1] = n[1];
        dst[2] = n[2];
      }
    }
    __syncthreads();
    r0 = r1;
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

__device__ __forceinline__ void load16(const uint32_t* in, int64_t n, int64_t i, uint32_t v[16]) {
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

__global__ void __launch_bounds__(kBlock) scan_reduce_kernel(const uint32_t* in, int64_t n,
                                                              uint64_t* partial) {
  __shared__ uint64_t s_w[kWaves];
  const int64_t i = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[16];
  load16(in, n, i, v);
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += v[k];
  uint64_t total;
  block_exclusive_scan<uint64_t>(s, s_w, total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the per-tile partial sums, total to out[n].
__global__ void __launch_bounds__(kBlock) scan_spine_kernel(uint64_t* partial, int64_t nb,
                                                             uint32_t* out, int64_t n,
                                                             uint32_t* status) {
  __shared__ uint64_t s_w[kWaves];
  uint64_t carry = 0;
  for (int64_t base = 0; base < nb; base += kBlock) {
    const int64_t q = base + threadIdx.x;
    const uint64_t x = q < nb ? partial[q] : 0;
    uint64_t total;
    const uint64_t e = block_exclusive_scan<uint64_t>(x, s_w, total);
    if (q < nb) partial[q] = carry + e;
    carry += total;
  }
  if (threadIdx.x == 0) {
    out[n] = (uint32_t)carry;
    if (carry > 0xffffffffull) atomicOr(status, kStatusOverflow);
  }
}

__global__ void __launch_bounds__(kBlock) scan_apply_kernel(const uint32_t* in, int64_t n,
                                                            const uint64_t* partial,
                                                            uint32_t* out) {
  __shared__ uint64_t s_w[kWaves];
  const int64_t i = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[16];
  load16(in, n, i, v);
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += v[k];
  uint64_t total;
  uint64_t run = block_exclusive_scan<uint64_t>(s, s_w, total) + partial[blockIdx.x];
  uint32_t o[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    o[k] = (uint32_t)run;
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

inline unsigned grid_for(int64_t n, int per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  unsigned g = grid_for(n, kBlock);
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(g), dim3(kBlock), 0, s, p, value, n);
  return hipGetLastError();
}

hipError_t launch_setup(const MeshSetup& m, const ImageSet& set, hipStream_t s) {
  if (m.n_tris <= 0) return hipSuccess;
  hipLaunchKernelGGL(setup_kernel, dim3(grid_for(m.n_tris, kBlock)), dim3(kBlock), 0, s, m, set);
  return hipGetLastError();
}

hipError_t launch_bin_count(const ImageSet& set, hipStream_t s) {
  if (set.n == 0 || set.img[0].n_tris <= 0) return hipSuccess;
  dim3 grid(grid_for(set.img[0].n_tris, kBlock), set.n);
  hipLaunchKernelGGL(bin_kernel<false>, grid, dim3(kBlock), 0, s, set);
  return hipGetLastError();
}

hipError_t launch_bin_scatter(const ImageSet& set, hipStream_t s) {
  if (set.n == 0 || set.img[0].n_tris <= 0) return hipSuccess;
  dim3 grid(grid_for(set.img[0].n_tris, kBlock), set.n);
  hipLaunchKernelGGL(bin_kernel<true>, grid, dim3(kBlock), 0, s, set);
  return hipGetLastError();
}

hipError_t launch_count(const ImageSet& set, hipStream_t s) {
  const uint32_t blocks = set.tile_start[set.n];
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(count_kernel, dim3(blocks), dim3(kBlock), 0, s, set);
  return hipGetLastError();
}

hipError_t launch_write(const ImageSet& set, hipStream_t s) {
  const uint32_t blocks = set.tile_start[set.n];
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(write_kernel, dim3(blocks), dim3(kBlock), 0, s, set);
  return hipGetLastError();
}

size_t scan_scratch_bytes(int64_t n) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  return (size_t)(nb > 0 ? nb : 1) * sizeof(uint64_t);
}

hipError_t launch_scan(const uint32_t* in, uint32_t* out, int64_t n, void* scratch,
                       uint32_t* status, hipStream_t s) {
  uint64_t* partial = static_cast<uint64_t*>(scratch);
  if (n <= 0) return launch_fill_u32(out, 0u, 1, s);
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, partial);
  hipLaunchKernelGGL(scan_spine_kernel, dim3(1), dim3(kBlock), 0, s, partial, nb, out, n, status);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, in, n, partial, out);
  return hipGetLastError();
}

}  // namespace ldni
