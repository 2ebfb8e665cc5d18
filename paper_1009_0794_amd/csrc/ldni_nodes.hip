// ldni_nodes.hip -- gfx950 kernel classifying the grid nodes of three LDNIs.
//
// The rays of the x-, y- and z-LDNI of one box and resolution w meet at the
// nodes of a w x w x w grid (Definition 3).  Along each of its rays a node is
// inside the solid when it lies in one of the ray's volumes (from a sample of
// odd rank to the next; Sec. 2 after Proposition 1); step 1 of the contouring
// algorithm (Sec. 5.1) classifies a node inside when at least two of its
// three LDNIs say so, which repairs disagreements caused by numerical error.
//
// Fixed readings: node t of an axis sits at the pixel centre
// f32(lo + (t + 0.5) h) and has depth f32(centre - lo) on that axis's LDNI
// (the depth a sample exactly there would get); a node is inside along a ray
// when an odd number of the ray's paired samples have depth <= its depth
// (half-open volumes [enter, exit); an unpaired last sample is ignored).
//
// Output: one bit per node in 32 x 32 x 32 bricks of 1024 words (4 KiB).
// Brick (bi, bj, bk) = (i/32, j/32, k/32) is brick number (bk*nb + bj)*nb + bi
// with nb = ceil(w/32); in a brick, word (k%32)*32 + (j%32) holds the nodes
// i = 32 bi .. 32 bi + 31 of row (j, k), node i in bit i%32.  Bits of nodes
// beyond w are zero.
//
// Work decomposition.  A workgroup owns the 64 x 64 rows (j, k) of a block of
// 2 x 2 brick columns and walks along i one brick (32 nodes) at a time:
//  * its 4096 x-rays run along i, so each is streamed once: per thread 16 ray
//    states (next sample, end, parity) in registers, advanced a brick per step;
//  * the y-rays (i, k) and z-rays (i, j) of the step are cut to the block's
//    64 nodes along j (resp. k): each such span is a 64-bit mask built from the
//    samples at or before its last node (a parity fill toggled at each sample),
//    2 x 2048 spans per step;
//  * the spans come out with bits along j (resp. k), the output wants bits
//    along i: each thread transposes one 32 x 32 bit matrix in registers
//    (five block-swap stages), the blocks exchanged through LDS;
//  * majority of the three words, stored as 2 x 128 contiguous bytes per wave.
// The output write (w^3 / 8 bytes) is the dominant HBM traffic; the inputs
// are read once (x) or a few times through the caches (y, z spans of the
// step's 32 rays of each column).  No contraction: nothing for MFMA.
#pragma clang fp contract(off)

#include "ldni_internal.hpp"

namespace ldni {
namespace {

constexpr int kNodeBlock = 256;
constexpr int kSpan = 64;     // nodes of a workgroup's block along j and along k
constexpr int kStep = 32;     // nodes along i per step (one brick)
constexpr int kRow = 33;      // LDS stride of a 32-word bit matrix (no bank conflicts)
constexpr int kVoteBlock = 512;  // threads of a classification workgroup
constexpr int kXRays = kSpan * kSpan / kVoteBlock;       // 8 x-rays per thread
constexpr int kVisits = kStep * kSpan / kVoteBlock;      // 4 y- and 4 z-spans per thread per step
constexpr int kMaxSpans = 16384 / kSpan;

// Depth of node t on an axis with origin lo and pixel size h; nodes past the
// grid get +inf so that the tables stay sorted.
__device__ __forceinline__ float node_depth(double lo, double h, int t, int w) {
  if (t >= w) return __int_as_float(0x7f800000);
  const float c = (float)(lo + ((double)t + 0.5) * h);
  return (float)((double)c - lo);
}

// Number of entries of the sorted table T[0..n) below s, given T[0] < s.
template <int N>
__device__ __forceinline__ int count_below(const float* T, float s) {
  int lo = 1, hi = N;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (T[mid] < s) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Inside mask of the 64 nodes whose depths are T[0..64) along the ray of
// pixel p (bit t = node t): parity of the paired samples at or before each
// node.  Offsets outside [0, n] or decreasing set *bad and give an empty ray.
__device__ __forceinline__ uint64_t span_mask(const AxisArrays& ax, size_t p, const float* T, float t_first,
                                              float t_last, bool& bad) {
  const uint32_t o0 = ax.offsets[p], o1 = ax.offsets[p + 1];
  if (o1 < o0 || (uint64_t)o1 > ax.n) {
    bad = true;
    return 0;
  }
  const uint32_t end = o0 + ((o1 - o0) & ~1u);
  uint64_t m = 0;
  for (uint32_t q = o0; q < end; ++q) {
    const float s = ax.depth[q];
    if (!(s <= t_last)) break;  // this and every later sample lies beyond the span
    const int c = s <= t_first ? 0 : count_below<kSpan>(T, s);
    m ^= c >= 64 ? 0ull : (~0ull << c);
  }
  return m;
}

// 32 x 32 bit matrix transpose in registers: afterwards a[j] bit i is the
// former a[i] bit j.  Stage s swaps the off-diagonal s x s blocks of every
// 2s x 2s block.
template <int S, uint32_t M>
__device__ __forceinline__ void swap_stage(uint32_t (&a)[32]) {
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    if ((i & S) == 0) {
      const uint32_t t = ((a[i] >> S) ^ a[i + S]) & M;
      a[i + S] ^= t;
      a[i] ^= t << S;
    }
  }
}

__device__ __forceinline__ void transpose32(uint32_t* row) {
  uint32_t a[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) a[i] = row[i];
  swap_stage<16, 0x0000ffffu>(a);
  swap_stage<8, 0x00ff00ffu>(a);
  swap_stage<4, 0x0f0f0f0fu>(a);
  swap_stage<2, 0x33333333u>(a);
  swap_stage<1, 0x55555555u>(a);
#pragma unroll
  for (int i = 0; i < 32; ++i) row[i] = a[i];
}

// Ranks of the spans of every y- and z-ray: for span s (nodes 64 s .. 64 s + 63
// along the ray) the number of the ray's paired samples at or before the
// span's first node, i.e. the parity of that node and the position of the
// first sample that can fall inside the span; entry n_spans holds the
// paired count.  One byte each, 255 meaning 255 or more.  ranks[f][s][p]:
// f = 0 for the y-LDNI, 1 for the z-LDNI, p the pixel.  One thread per ray.
__global__ __launch_bounds__(kNodeBlock) void node_ranks_kernel(NodeArgs g) {
  __shared__ float s_start[2][kMaxSpans + 1];
  const int S = g.n_spans;
  for (int q = threadIdx.x; q < 2 * (S + 1); q += kNodeBlock) {
    const int f = q / (S + 1), s = q - f * (S + 1);
    s_start[f][s] = s < S ? node_depth(g.lo[1 + f], g.h[1 + f], s * kSpan, g.w) : __int_as_float(0x7f800000);
  }
  __syncthreads();
  const int64_t npix = (int64_t)g.w * g.w;
  const int64_t t = (int64_t)blockIdx.x * kNodeBlock + threadIdx.x;
  if (t >= 2 * npix) return;
  const int f = t >= npix ? 1 : 0;
  const size_t p = (size_t)(t - f * npix);
  const AxisArrays& ax = g.axis[1 + f];
  uint8_t* R = g.ranks + (size_t)f * (size_t)(S + 1) * (size_t)npix + p;
  const uint32_t o0 = ax.offsets[p], o1 = ax.offsets[p + 1];
  uint32_t cnt = 0;
  if (o1 < o0 || (uint64_t)o1 > ax.n) atomicOr(g.status, kStatusMismatch);
  else cnt = (o1 - o0) & ~1u;
  uint32_t q = 0;
  float d = cnt > 0 ? ax.depth[o0] : 0.0f;
  for (int s = 0; s <= S; ++s) {
    const float T = s_start[f][s];
    while (q < cnt && d <= T) {
      ++q;
      d = q < cnt ? ax.depth[o0 + q] : 0.0f;
    }
    R[(size_t)s * npix] = (uint8_t)(q < 255u ? q : 255u);
  }
}

// Inside mask of a span from its ranks: the parity at its first node, then a
// toggle at each sample inside it (samples o0 + ra .. o0 + rb - 1 are the
// ones after the first node and at or before the next span's first node).
// Saturated ranks walk the ray from its start instead.
__device__ __forceinline__ uint64_t span_from_ranks(const AxisArrays& ax, size_t p, uint32_t o0, uint32_t ra,
                                                    uint32_t rb, const float* T, float t_first, float t_last,
                                                    bool& bad) {
  if (ra == 255u || rb == 255u) return span_mask(ax, p, T, t_first, t_last, bad);
  uint64_t m = (ra & 1u) ? ~0ull : 0ull;
  for (uint32_t q = o0 + ra; q < o0 + rb; ++q) {
    const float s = ax.depth[q];
    if (!(s <= t_last)) break;
    const int c = s <= t_first ? 0 : count_below<kSpan>(T, s);
    m ^= c >= 64 ? 0ull : (~0ull << c);
  }
  return m;
}

__global__ __launch_bounds__(kVoteBlock, 4) void classify_nodes_kernel(NodeArgs g) {
  __shared__ float s_tx[2][kStep];  // node depths of the current and the next step along i
  __shared__ float s_ty[kSpan];
  __shared__ float s_tz[kSpan];
  __shared__ uint32_t s_y[2 * kSpan * kRow];  // matrix (k, j-half): rows i, bits j; then rows j, bits i
  __shared__ uint32_t s_z[2 * kSpan * kRow];  // matrix (j, k-half): rows i, bits k; then rows k, bits i
  __shared__ uint64_t s_sum[2][kVoteBlock / 64];

  const int tid = threadIdx.x;
  const int w = g.w, nb = g.nb;
  const int blocks_j = (nb + 1) >> 1;
  const int bj0 = 2 * (int)(blockIdx.x % blocks_j), bk0 = 2 * (int)(blockIdx.x / blocks_j);
  const int j0 = bj0 * kStep, k0 = bk0 * kStep;
  const AxisArrays& X = g.axis[0];
  const AxisArrays& Y = g.axis[1];
  const AxisArrays& Z = g.axis[2];
  const size_t npix = (size_t)w * w;
  // ranks of this block's span along j (y-rays) and along k (z-rays)
  const uint8_t* ry = g.ranks + (size_t)(j0 / kSpan) * npix;
  const uint8_t* rz = g.ranks + (size_t)(g.n_spans + 1) * npix + (size_t)(k0 / kSpan) * npix;
  bool bad = false;

  if (tid < kSpan) s_ty[tid] = node_depth(g.lo[1], g.h[1], j0 + tid, w);
  else if (tid < 2 * kSpan) s_tz[tid - kSpan] = node_depth(g.lo[2], g.h[2], k0 + tid - kSpan, w);
  else if (tid < 2 * kSpan + kStep) s_tx[0][tid - 2 * kSpan] = node_depth(g.lo[0], g.h[0], tid - 2 * kSpan, w);

  // x-ray states: ray r = tid + 512 m is row (j0 + r % 64, k0 + r / 64); the
  // depth of its next sample is kept loaded
  uint32_t xq[kXRays], xe[kXRays];
  float xs[kXRays];
  uint32_t xpar = 0;
#pragma unroll
  for (int m = 0; m < kXRays; ++m) {
    const int r = tid + kVoteBlock * m;
    const int j = j0 + (r & (kSpan - 1)), k = k0 + (r >> 6);
    xq[m] = xe[m] = 0;
    xs[m] = 0.0f;
    if (j < w && k < w) {
      const size_t p = (size_t)k * w + j;
      const uint32_t o0 = X.offsets[p], o1 = X.offsets[p + 1];
      if (o1 < o0 || (uint64_t)o1 > X.n) {
        bad = true;
      } else {
        xq[m] = o0;
        xe[m] = o0 + ((o1 - o0) & ~1u);
        if (o0 < xe[m]) xs[m] = X.depth[o0];
      }
    }
  }
  __syncthreads();
  const float ty_first = s_ty[0], ty_last = s_ty[kSpan - 1];
  const float tz_first = s_tz[0], tz_last = s_tz[kSpan - 1];
  uint32_t n_inside = 0, n_split = 0;

  for (int bi = 0; bi < nb; ++bi) {
    const int i0 = bi * kStep;
    const float* TX = s_tx[bi & 1];
    const float tx_first = TX[0], tx_last = TX[kStep - 1];
    // (1) offsets and ranks of the step's spans: y-rays (i, k) along j,
    // z-rays (i, j) along k; all issued before any is used
    uint32_t vo[2 * kVisits], vr[2 * kVisits];
#pragma unroll
    for (int m = 0; m < kVisits; ++m) {
      const int v = tid + kVoteBlock * m;
      const int i_y = i0 + (v >> 6), k = k0 + (v & (kSpan - 1));
      const int i_z = i0 + (v & (kStep - 1)), j = j0 + (v >> 5);
      vo[m] = vr[m] = vo[kVisits + m] = vr[kVisits + m] = 0;
      if (i_y < w && k < w) {
        const size_t p = (size_t)i_y * w + k;
        vo[m] = Y.offsets[p];
        vr[m] = (uint32_t)ry[p] | ((uint32_t)ry[npix + p] << 8);
      }
      if (i_z < w && j < w) {
        const size_t p = (size_t)j * w + i_z;
        vo[kVisits + m] = Z.offsets[p];
        vr[kVisits + m] = (uint32_t)rz[p] | ((uint32_t)rz[npix + p] << 8);
      }
    }
    // (2) x-rays, first round: the kept depths decide; the next samples'
    // loads are issued without waiting
    uint32_t xw[kXRays];
    bool more = false;
#pragma unroll
    for (int m = 0; m < kXRays; ++m) {
      xw[m] = ((xpar >> m) & 1u) ? 0xffffffffu : 0u;
      if (xq[m] < xe[m] && xs[m] <= tx_last) {
        const float sd = xs[m];
        const int c = sd <= tx_first ? 0 : count_below<kStep>(TX, sd);
        xw[m] ^= c >= 32 ? 0u : (0xffffffffu << c);
        xpar ^= 1u << m;
        ++xq[m];
        xs[m] = xq[m] < xe[m] ? X.depth[xq[m]] : 0.0f;
        more = true;
      }
    }
    // (3) spans: the parity at the first node goes to LDS; the first sample
    // that may lie inside has its load issued now
    uint32_t vq[2 * kVisits], vn[2 * kVisits];
    float vd[2 * kVisits];
#pragma unroll
    for (int m = 0; m < 2 * kVisits; ++m) {
      const bool is_y = m < kVisits;
      const int v = tid + kVoteBlock * (is_y ? m : m - kVisits);
      const AxisArrays& A = is_y ? Y : Z;
      const uint32_t ra = vr[m] & 255u, rb = vr[m] >> 8;
      uint32_t* row = is_y ? s_y + (2 * (v & (kSpan - 1))) * kRow + (v >> 6)
                           : s_z + (2 * (v >> 5)) * kRow + (v & (kStep - 1));
      uint64_t mask = 0;
      vn[m] = 0;
      vq[m] = 0;
      vd[m] = 0.0f;
      if (ra == 255u || rb == 255u) {  // saturated ranks: walk from the ray's start
        const int i = i0 + (is_y ? (v >> 6) : (v & (kStep - 1)));
        const int o = is_y ? k0 + (v & (kSpan - 1)) : j0 + (v >> 5);
        if (i < w && o < w) {
          const size_t p = is_y ? (size_t)i * w + o : (size_t)o * w + i;
          mask = is_y ? span_mask(Y, p, s_ty, ty_first, ty_last, bad) : span_mask(Z, p, s_tz, tz_first, tz_last, bad);
        }
      } else {
        mask = (ra & 1u) ? ~0ull : 0ull;
        vq[m] = vo[m] + ra;
        vn[m] = rb - ra;
        if (vn[m] > 0) vd[m] = A.depth[vq[m]];
      }
      row[0] = (uint32_t)mask;
      row[kRow] = (uint32_t)(mask >> 32);
    }
    // (4) x-rays, further rounds (two or more samples of a ray in one step)
    while (more) {
      more = false;
#pragma unroll
      for (int m = 0; m < kXRays; ++m) {
        if (xq[m] < xe[m] && xs[m] <= tx_last) {
          const float sd = xs[m];
          const int c = sd <= tx_first ? 0 : count_below<kStep>(TX, sd);
          xw[m] ^= c >= 32 ? 0u : (0xffffffffu << c);
          xpar ^= 1u << m;
          ++xq[m];
          xs[m] = xq[m] < xe[m] ? X.depth[xq[m]] : 0.0f;
          more = true;
        }
      }
    }
    // (5) spans: toggles of the samples inside (each thread owns its LDS words)
#pragma unroll
    for (int m = 0; m < 2 * kVisits; ++m) {
      if (vn[m] == 0) continue;
      const bool is_y = m < kVisits;
      const int v = tid + kVoteBlock * (is_y ? m : m - kVisits);
      const AxisArrays& A = is_y ? Y : Z;
      const float* T = is_y ? s_ty : s_tz;
      const float t_first = is_y ? ty_first : tz_first, t_last = is_y ? ty_last : tz_last;
      uint32_t* row = is_y ? s_y + (2 * (v & (kSpan - 1))) * kRow + (v >> 6)
                           : s_z + (2 * (v >> 5)) * kRow + (v & (kStep - 1));
      uint64_t mask = (uint64_t)row[0] | ((uint64_t)row[kRow] << 32);
      while (vn[m] > 0) {
        const float sd = vd[m];
        if (!(sd <= t_last)) break;
        const int c = sd <= t_first ? 0 : count_below<kSpan>(T, sd);
        mask ^= c >= 64 ? 0ull : (~0ull << c);
        ++vq[m];
        --vn[m];
        if (vn[m] > 0) vd[m] = A.depth[vq[m]];
      }
      row[0] = (uint32_t)mask;
      row[kRow] = (uint32_t)(mask >> 32);
    }
    __syncthreads();
    // (6) one 32 x 32 transpose per thread of the first half: 128 y matrices,
    // then 128 z matrices; the second half prepares the next step's depths
    if (tid < 4 * kSpan) transpose32(tid < 2 * kSpan ? s_y + tid * kRow : s_z + (tid - 2 * kSpan) * kRow);
    else if (tid < 4 * kSpan + kStep) s_tx[(bi + 1) & 1][tid - 4 * kSpan] = node_depth(g.lo[0], g.h[0], i0 + kStep + tid - 4 * kSpan, w);
    __syncthreads();
    // (7) majority of the three words, stored to the brick
    const uint32_t valid = (w - i0 >= 32) ? 0xffffffffu : ((1u << (w - i0)) - 1u);
#pragma unroll
    for (int m = 0; m < kXRays; ++m) {
      const int r = tid + kVoteBlock * m;
      const int jl = r & (kSpan - 1), kl = r >> 6;
      const uint32_t xw_ = xw[m];
      const uint32_t yw = s_y[(2 * kl + (jl >> 5)) * kRow + (jl & 31)];
      const uint32_t zw = s_z[(2 * jl + (kl >> 5)) * kRow + (kl & 31)];
      const uint32_t in = ((xw_ & yw) | (xw_ & zw) | (yw & zw)) & valid;
      const uint32_t split = ((xw_ | yw | zw) & ~(xw_ & yw & zw)) & valid;
      const int bj = bj0 + (jl >> 5), bk = bk0 + (kl >> 5);
      if (bj < nb && bk < nb) {
        g.bits[(((size_t)bk * nb + bj) * nb + bi) * 1024 + (kl & 31) * 32 + (jl & 31)] = in;
        n_inside += __popc(in);
        n_split += __popc(split);
      }
    }
    __syncthreads();  // the next step rewrites s_y and s_z
  }

  if (bad) atomicOr(g.status, kStatusMismatch);
  uint64_t a = n_inside, b = n_split;
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if ((tid & 63) == 0) {
    s_sum[0][tid >> 6] = a;
    s_sum[1][tid >> 6] = b;
  }
  __syncthreads();
  if (tid == 0) {
    uint64_t sa = 0, sb = 0;
    for (int q = 0; q < kVoteBlock / 64; ++q) {
      sa += s_sum[0][q];
      sb += s_sum[1][q];
    }
    g.partial[2 * blockIdx.x] = sa;
    g.partial[2 * blockIdx.x + 1] = sb;
  }
}

// Sums the workgroups' (inside, split) counts into stats[0..1] (one block).
__global__ __launch_bounds__(kNodeBlock) void node_stats_kernel(const uint64_t* partial, uint32_t n, uint64_t* stats) {
  __shared__ uint64_t s_sum[2][kNodeBlock / 64];
  uint64_t a = 0, b = 0;
  for (uint32_t q = threadIdx.x; q < n; q += kNodeBlock) {
    a += partial[2 * q];
    b += partial[2 * q + 1];
  }
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if ((threadIdx.x & 63) == 0) {
    s_sum[0][threadIdx.x >> 6] = a;
    s_sum[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t sa = 0, sb = 0;
    for (int q = 0; q < kNodeBlock / 64; ++q) {
      sa += s_sum[0][q];
      sb += s_sum[1][q];
    }
    stats[0] = sa;
    stats[1] = sb;
  }
}

}  // namespace

uint32_t node_workgroups(int32_t w) {
  const uint32_t nb = (uint32_t)((w + kStep - 1) / kStep);
  const uint32_t per = (nb + 1) / 2;
  return per * per;
}

hipError_t launch_node_ranks(const NodeArgs& g, hipStream_t s) {
  const int64_t rays = 2 * (int64_t)g.w * g.w;
  hipLaunchKernelGGL(node_ranks_kernel, dim3((unsigned)((rays + kNodeBlock - 1) / kNodeBlock)), dim3(kNodeBlock), 0,
                     s, g);
  return hipGetLastError();
}

hipError_t launch_classify_nodes(const NodeArgs& g, hipStream_t s) {
  hipLaunchKernelGGL(classify_nodes_kernel, dim3(node_workgroups(g.w)), dim3(kVoteBlock), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_node_stats(const NodeArgs& g, hipStream_t s) {
  hipLaunchKernelGGL(node_stats_kernel, dim3(1), dim3(kNodeBlock), 0, s, g.partial, node_workgroups(g.w), g.stats);
  return hipGetLastError();
}

}  // namespace ldni
