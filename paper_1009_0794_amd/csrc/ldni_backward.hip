// ldni_backward.hip -- gfx950 kernels of the sampler's backward pass: the
// vertex gradient of a loss on the samples (depth and normal) of an LDNI,
// with the sample set held fixed.
#pragma clang fp contract(off)

#include <cmath>

#include "ldni_internal.hpp"

namespace ldni {
namespace {

constexpr int kBlock = 256;  // 4 wave64 per workgroup

inline unsigned grid_for(int64_t n, int per_block) { return (unsigned)((n + per_block - 1) / per_block); }

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// For a sample on triangle (A,B,C) at pixel centre c, with barycentric
// weights lambda of c in the projected triangle and unit normal n:
//   depth:  moving vertex X moves the hit along the fixed ray by
//           lambda_X (n . dX) / n_a, so dL/dX += gd * lambda_X * n / n_a;
//   normal: n = N/|N|, N = (B-A)x(C-A): dL/dN = (gn - n (n.gn)) / |N| and
//           dL/dA = (B-C) x dL/dN, dL/dB = (C-A) x dL/dN, dL/dC = (A-B) x dL/dN.
// n / n_a and the normal Jacobian are constant per triangle, so the
// sample-parallel kernel only accumulates, per (triangle, image), the sums of
// gd * lambda_X and of gn; the triangle-parallel kernel applies the
// per-triangle factors and adds to the three vertices.
struct BackwardImage {
  int32_t a, u, v, w;
  double lo_u, h_u, lo_v, h_v;
  // bound, in pixels, on the distance between a float32 pixel centre and
  // its float64 position estimate (x - lo) / h - 0.5 for x within the image
  double margin_u, margin_v;
  const uint32_t* offsets;  // [w*w+1]
  const int32_t* tri;       // [n]
  const float* gd;          // [n] or null
  const float* gn;          // [n][3] or null
  float* acc;               // [T][6] sums of gd * lambda per vertex, then of gn
};

struct BackwardSet {
  BackwardImage img[kMaxImages];
  int32_t n;
  uint32_t block_start[kMaxImages + 1];  // pixel blocks per image
  const float* verts;
  int64_t n_verts;
  const int32_t* tris;
  int64_t n_tris;
};

// One workgroup per kBwdTile x kBwdTile pixel tile.  The tile's samples (one
// contiguous range per pixel row) are spread over the threads; each sample's
// six values (gd * lambda per vertex, gn) are summed per triangle in an LDS
// hash table, and every triangle of the tile then writes its sums once: with
// plain stores when every pixel centre its projection can cover lies in the
// tile (no other tile has samples of it on this image: the common case, and
// stores cost far less than global atomics), else with atomic additions.  A
// sample that finds no free slot adds its own directly (its triangle then has
// no slot in this tile, so nothing stores over it).
constexpr int kBwdTile = 16;
constexpr int kBwdSlots = 1024;
constexpr int kBwdProbe = 32;

// Whether every pixel whose centre can lie in the projection of triangle t
// on image im is a pixel of the tile (x0, y0, cw, ch): the centres within the
// projection's bounding box, its index range widened by the image's rounding
// margin.  Only then does the tile hold all of t's samples on im.
__device__ __forceinline__ bool projection_in_tile(const BackwardSet& bs, const BackwardImage& im, int64_t t,
                                                   int x0, int y0, int cw, int ch) {
  const int32_t* fv = bs.tris + 3 * t;
  double umin = HUGE_VAL, umax = -HUGE_VAL, vmin = HUGE_VAL, vmax = -HUGE_VAL;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const float* P = bs.verts + 3 * (int64_t)min(max(fv[q], 0), (int32_t)(bs.n_verts - 1));
    umin = fmin(umin, (double)P[im.u]);
    umax = fmax(umax, (double)P[im.u]);
    vmin = fmin(vmin, (double)P[im.v]);
    vmax = fmax(vmax, (double)P[im.v]);
  }
  // pixel i has centre f32(lo + (i + 0.5) h); a centre in [mn, mx] has i
  // within [tmn - m, tmx + m] for t = (x - lo) / h - 0.5 and m the margin
  const double iu0 = floor((umin - im.lo_u) / im.h_u - 0.5 - im.margin_u),
               iu1 = ceil((umax - im.lo_u) / im.h_u - 0.5 + im.margin_u);
  const double iv0 = floor((vmin - im.lo_v) / im.h_v - 0.5 - im.margin_v),
               iv1 = ceil((vmax - im.lo_v) / im.h_v - 0.5 + im.margin_v);
  return iu0 >= (double)x0 && iu1 < (double)(x0 + cw) && iv0 >= (double)y0 && iv1 < (double)(y0 + ch);
}

__global__ void __launch_bounds__(kBlock) backward_samples_kernel(BackwardSet bs) {
  __shared__ uint32_t s_row[kBwdTile + 1][kBwdTile + 1];  // offsets of the tile's rows
  __shared__ uint32_t s_pre[kBwdTile + 1];                // samples before each row
  __shared__ uint32_t s_key[kBwdSlots];                   // triangle + 1, 0 = free
  __shared__ float s_val[kBwdSlots][6];
  int k = 0;
  while (k + 1 < bs.n && blockIdx.x >= bs.block_start[k + 1]) ++k;
  const BackwardImage& im = bs.img[k];
  const int ntx = (im.w + kBwdTile - 1) / kBwdTile;
  const int tile = (int)(blockIdx.x - bs.block_start[k]);
  const int x0 = (tile % ntx) * kBwdTile, y0 = (tile / ntx) * kBwdTile;
  const int cw = min(kBwdTile, im.w - x0), ch = min(kBwdTile, im.w - y0);

  for (int q = threadIdx.x; q < kBwdSlots; q += kBlock) {
    s_key[q] = 0;
#pragma unroll
    for (int c = 0; c < 6; ++c) s_val[q][c] = 0.0f;
  }
  for (int q = threadIdx.x; q < ch * (cw + 1); q += kBlock) {
    const int r = q / (cw + 1), x = q - r * (cw + 1);
    s_row[r][x] = im.offsets[(int64_t)(y0 + r) * im.w + x0 + x];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int r = 0; r < ch; ++r) {
      s_pre[r] = acc;
      acc += s_row[r][cw] - s_row[r][0];
    }
    s_pre[ch] = acc;
  }
  __syncthreads();
  const uint32_t S = s_pre[ch];
  float* const accp = im.acc;

  for (uint32_t f = threadIdx.x; f < S; f += kBlock) {
    int r = 0;  // row of f: the last r with s_pre[r] <= f (binary search)
    for (int hi = ch - 1; r < hi;) {
      const int mid = (r + hi + 1) >> 1;
      if (s_pre[mid] <= f) r = mid; else hi = mid - 1;
    }
    const uint32_t s = s_row[r][0] + (f - s_pre[r]);
    const int32_t t = im.tri[s];
    if (t < 0 || t >= bs.n_tris) continue;  // not a triangle of this mesh
    float v[6] = {0, 0, 0, 0, 0, 0};
    const float g = im.gd ? im.gd[s] : 0.0f;
    if (g != 0.0f) {
      int lo = 0, hi = cw - 1;  // pixel of s in the row: the last x with s_row[r][x] <= s
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_row[r][mid] <= s) lo = mid; else hi = mid - 1;
      }
      const double cu = im.lo_u + ((double)(x0 + lo) + 0.5) * im.h_u;
      const double cv = im.lo_v + ((double)(y0 + r) + 0.5) * im.h_v;
      const int32_t* fv = bs.tris + 3 * (int64_t)t;
      double xu[3], xv[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const float* P = bs.verts + 3 * (int64_t)min(max(fv[q], 0), (int32_t)(bs.n_verts - 1));
        xu[q] = (double)P[im.u] - cu;
        xv[q] = (double)P[im.v] - cv;
      }
      const double e_bc = xu[1] * xv[2] - xv[1] * xu[2];
      const double e_ca = xu[2] * xv[0] - xv[2] * xu[0];
      const double e_ab = xu[0] * xv[1] - xv[0] * xu[1];
      const double den = e_ab + e_bc + e_ca;
      if (den != 0.0) {
        const double gs = (double)g / den;
        v[0] = (float)(gs * e_bc);
        v[1] = (float)(gs * e_ca);
        v[2] = (float)(gs * e_ab);
      }
    }
    if (im.gn) {
      const float* gv = im.gn + 3 * (int64_t)s;
      v[3] = gv[0];
      v[4] = gv[1];
      v[5] = gv[2];
    }
    if (v[0] == 0.0f && v[1] == 0.0f && v[2] == 0.0f && v[3] == 0.0f && v[4] == 0.0f && v[5] == 0.0f)
      continue;
    // slot of t in the table (linear probing, a bounded number of steps)
    const uint32_t key = (uint32_t)t + 1u;
    uint32_t h = ((uint32_t)t * 2654435761u) >> 22;  // 10 bits
    int slot = -1;
    for (int step = 0; step < kBwdProbe; ++step) {
      const uint32_t old = atomicCAS(&s_key[h], 0u, key);
      if (old == 0u || old == key) {
        slot = (int)h;
        break;
      }
      h = (h + 1) & (kBwdSlots - 1);
    }
    if (slot >= 0) {
#pragma unroll
      for (int c = 0; c < 6; ++c)
        if (v[c] != 0.0f) atomicAdd(&s_val[slot][c], v[c]);
    } else {
      float* a6 = accp + 6 * (int64_t)t;
#pragma unroll
      for (int c = 0; c < 6; ++c)
        if (v[c] != 0.0f) atomicAdd(a6 + c, v[c]);
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kBwdSlots; q += kBlock) {
    const uint32_t key = s_key[q];
    if (key == 0u) continue;
    const int64_t t = (int64_t)(key - 1u);
    float* a6 = accp + 6 * t;
    if (projection_in_tile(bs, im, t, x0, y0, cw, ch)) {
#pragma unroll
      for (int c = 0; c < 6; ++c) a6[c] = s_val[q][c];
    } else {
#pragma unroll
      for (int c = 0; c < 6; ++c)
        if (s_val[q][c] != 0.0f) atomicAdd(a6 + c, s_val[q][c]);
    }
  }
}

// The gradient of triangle t's three vertices (false: t is not a valid
// triangle, or degenerate, and adds nothing).
__device__ bool triangle_gradient(const BackwardSet& bs, int64_t t, int32_t (&vid)[3], double (&g)[3][3]) {
  const int32_t* f = bs.tris + 3 * t;
  for (int q = 0; q < 3; ++q) {
    vid[q] = f[q];
    if (f[q] < 0 || f[q] >= bs.n_verts) return false;  // not a valid triangle
  }
  double P[3][3];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) P[q][c] = (double)bs.verts[3 * (int64_t)f[q] + c];
  double e1[3], e2[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    e1[c] = P[1][c] - P[0][c];
    e2[c] = P[2][c] - P[0][c];
  }
  const double N[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                       e1[0] * e2[1] - e1[1] * e2[0]};
  const double len = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
  if (!(len > 0.0)) return false;
  const double n[3] = {N[0] / len, N[1] / len, N[2] / len};
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) g[q][c] = 0.0;
  double G[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < bs.n; ++k) {
    const BackwardImage& im = bs.img[k];
    const float* acc = im.acc + 6 * t;
#pragma unroll
    for (int c = 0; c < 3; ++c) G[c] += (double)acc[3 + c];
    if (n[im.a] == 0.0) continue;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double s = (double)acc[q] / n[im.a];
#pragma unroll
      for (int c = 0; c < 3; ++c) g[q][c] += s * n[c];
    }
  }
  if (G[0] != 0.0 || G[1] != 0.0 || G[2] != 0.0) {
    const double dot = n[0] * G[0] + n[1] * G[1] + n[2] * G[2];
    double gN[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) gN[c] = (G[c] - n[c] * dot) / len;
    double ed[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ed[0][c] = P[1][c] - P[2][c];
      ed[1][c] = P[2][c] - P[0][c];
      ed[2][c] = P[0][c] - P[1][c];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      g[q][0] += ed[q][1] * gN[2] - ed[q][2] * gN[1];
      g[q][1] += ed[q][2] * gN[0] - ed[q][0] * gN[2];
      g[q][2] += ed[q][0] * gN[1] - ed[q][1] * gN[0];
    }
  }
  return true;
}

// One thread per triangle, adding to its three vertices with global atomics.
// (Neighbouring lanes add to neighbouring vertices, so a wave's atomics meet
// few cache lines; summing per vertex in an LDS table first was slower:
// 80 against 30 us on the flower.)
__global__ void __launch_bounds__(kBlock) backward_triangles_kernel(BackwardSet bs, int64_t n_tris,
                                                                    float* grad) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  int32_t vid[3];
  double g[3][3];
  if (t >= n_tris || !triangle_gradient(bs, t, vid, g)) return;
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (g[q][c] != 0.0) atomicAdd(grad + 3 * (int64_t)vid[q] + c, (float)g[q][c]);
}

}  // namespace

hipError_t launch_backward(const BackwardArgs& args, hipStream_t s) {
  BackwardSet bs{};
  bs.n = args.n;
  bs.verts = args.verts;
  bs.n_verts = args.n_verts;
  bs.tris = args.tris;
  bs.n_tris = args.n_tris;
  bs.block_start[0] = 0;
  for (int k = 0; k < args.n; ++k) {
    const BackwardAxis& a = args.axis[k];
    BackwardImage& im = bs.img[k];
    im.a = a.a;
    im.u = (a.a + 1) % 3;
    im.v = (a.a + 2) % 3;
    im.w = args.w;
    im.lo_u = args.bbox[im.u];
    im.h_u = (args.bbox[3 + im.u] - args.bbox[im.u]) / (double)args.w;
    im.lo_v = args.bbox[im.v];
    im.h_v = (args.bbox[3 + im.v] - args.bbox[im.v]) / (double)args.w;
    // a centre's float32 rounding (2^-24 of its magnitude, at most
    // |lo| + (w + 1) h) plus the float64 rounding of the estimate, doubled
    const auto margin = [&](double lo, double h) {
      return 2.0 * (std::ldexp(std::fabs(lo) + ((double)args.w + 1.0) * h, -24) / h +
                    std::ldexp((double)args.w + 1.0, -48)) + 1e-6;
    };
    im.margin_u = margin(im.lo_u, im.h_u);
    im.margin_v = margin(im.lo_v, im.h_v);
    im.offsets = a.offsets;
    im.tri = a.tri;
    im.gd = a.gd;
    im.gn = a.gn;
    im.acc = a.acc;
    const uint32_t nt = (uint32_t)((args.w + kBwdTile - 1) / kBwdTile);
    bs.block_start[k + 1] = bs.block_start[k] + nt * nt;
  }
  if (args.n > 0 && bs.block_start[args.n] > 0)
    hipLaunchKernelGGL(backward_samples_kernel, dim3(bs.block_start[args.n]), dim3(kBlock), 0, s, bs);
  if (args.n_tris > 0)
    hipLaunchKernelGGL(backward_triangles_kernel, dim3(grid_for(args.n_tris, kBlock)), dim3(kBlock), 0, s,
                       bs, args.n_tris, args.grad);
  return hipGetLastError();
}

}  // namespace ldni
