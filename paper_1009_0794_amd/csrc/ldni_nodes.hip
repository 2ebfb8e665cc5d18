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
// a vote step covers 2 x 32 nodes along i (two bricks) for the block's 64 x 64 (j, k) nodes
constexpr int kRow = 33;      // LDS stride of a 32-word bit matrix (no bank conflicts)
constexpr int kVoteBlock = 512;  // threads of a classification workgroup
static_assert(kSpan * kSpan / kVoteBlock == 8, "the vote kernel gives each thread 8 x-rays of its block");

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

// Span codes.  For every ray of the three LDNIs and every span of 64 nodes
// along it (span s holds nodes 64 s .. 64 s + 63), one 16-bit code:
//   bit 12      parity of the ray's paired samples at or before the span's
//               first node (inside at that node),
//   bits 0..5   t1, bits 6..11 t2: the samples after the first node and at or
//               before the span's last node flip the nodes from position
//               t (1..63) on; 0 means none,
//   bit 13      more than two such samples: bits 0..11 then hold the number
//               of the ray's paired samples before them (4095: that many or
//               more), and the vote pass walks the span's samples.
// Codes are grouped so that one step of one vote workgroup reads 4096
// consecutive codes per axis (index = block * 4096 + v):
//   x-ray (j, k), span s along i:  block ((s*S + k/64)*S + j/64),  v = (k%64)*64 + j%64
//   y-ray (i, k), span s along j:  block ((s*S + k/64)*S + i/64),  v = (i%64)*64 + k%64
//   z-ray (i, j), span s along k:  block ((s*S + j/64)*S + i/64),  v = (j%64)*64 + i%64
// with S = ceil(w/64) spans per axis; one axis's codes fill S^3 * 4096 words.
constexpr uint32_t kCodeParity = 1u << 12;
constexpr uint32_t kCodeWalk = 1u << 13;
constexpr uint32_t kRankMax = 4095u;  // bits 0..11 of a walk code: samples before the span (4095: or more)

__device__ __forceinline__ size_t code_index(int f, int iu, int iv, int s, int S) {
  // (iu, iv) = pixel of the f-LDNI; the frame is cyclic: x (j, k), y (k, i), z (i, j)
  const int a = f == 1 ? iv : iu;  // the coordinate whose 64-block is the inner block index
  const int b = f == 1 ? iu : iv;  // the other one (outer block index, and the row of v)
  // x: a = j, b = k -> v = (k%64)*64 + j%64, block (s, k/64, j/64)
  // y: a = i, b = k -> v = (i%64)*64 + k%64, block (s, k/64, i/64)
  // z: a = i, b = j -> v = (j%64)*64 + i%64, block (s, j/64, i/64)
  const size_t block = ((size_t)s * S + (b >> 6)) * S + (a >> 6);
  const uint32_t v = f == 1 ? (uint32_t)((a & 63) * 64 + (b & 63)) : (uint32_t)((b & 63) * 64 + (a & 63));
  return block * 4096 + v;
}

// One thread per ray: walks the ray's paired samples once and writes the
// code of each of its spans.  Grid (ceil(w*w/256), 3): blockIdx.y is the axis.
__global__ __launch_bounds__(kNodeBlock) void node_codes_kernel(NodeArgs g) {
  extern __shared__ float s_t[];  // the w node depths along this axis
  const int f = blockIdx.y;
  const int w = g.w, S = g.n_spans;
  for (int t = threadIdx.x; t < w; t += kNodeBlock) s_t[t] = node_depth(g.lo[f], g.h[f], t, w);
  __syncthreads();
  const size_t npix = (size_t)w * w;
  const size_t p = (size_t)blockIdx.x * kNodeBlock + threadIdx.x;
  if (p >= npix) return;
  const int iu = (int)(p % (size_t)w), iv = (int)(p / (size_t)w);
  const AxisArrays& ax = g.axis[f];
  uint16_t* C = g.codes + (size_t)f * ((size_t)S * S * S * 4096);
  const uint32_t o0 = ax.offsets[p], o1 = ax.offsets[p + 1];
  uint32_t cnt = 0;
  if (o1 < o0 || (uint64_t)o1 > ax.n) atomicOr(g.status, kStatusMismatch);
  else cnt = (o1 - o0) & ~1u;
  // the samples are read four at a time (independent loads), q indexes them
  const float* dep = ax.depth + o0;
  float b0 = 0.0f, b1 = 0.0f, b2 = 0.0f, b3 = 0.0f;
  auto fill = [&](uint32_t from) {
    if (from < cnt) b0 = dep[from];
    if (from + 1 < cnt) b1 = dep[from + 1];
    if (from + 2 < cnt) b2 = dep[from + 2];
    if (from + 3 < cnt) b3 = dep[from + 3];
  };
  uint32_t q = 0, parity = 0;
  fill(0);
  float d = b0;
  auto next = [&]() {
    ++q;
    if ((q & 3u) == 0) fill(q);
    const uint32_t r = q & 3u;
    d = r == 0 ? b0 : r == 1 ? b1 : r == 2 ? b2 : b3;
  };
  // consecutive spans of one ray are S*S blocks apart
  uint16_t* c = C + code_index(f, iu, iv, 0, S);
  const size_t span_step = (size_t)S * S * 4096;
  for (int s = 0; s < S; ++s, c += span_step) {
    const int base = s * kSpan, last = min(base + kSpan - 1, w - 1);
    const float t_first = s_t[base], t_last = s_t[last];
    while (q < cnt && d <= t_first) {
      parity ^= 1u;
      next();
    }
    uint32_t code = parity ? kCodeParity : 0u;
    if (q < cnt && d <= t_last) {
      const uint32_t rank = q;
      int n_t = 0;
      do {
        // d lies after node base and at or before node last: it flips nodes c.. (c in 1..last-base)
        int lo = 1, hi = last - base;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (s_t[base + mid] < d) lo = mid + 1; else hi = mid;
        }
        if (n_t == 0) code |= (uint32_t)lo;
        else if (n_t == 1) code |= (uint32_t)lo << 6;
        ++n_t;
        parity ^= 1u;
        next();
      } while (q < cnt && d <= t_last);
      // more than two: the code keeps the rank of the span's first sample instead
      if (n_t > 2) code = (code & kCodeParity) | kCodeWalk | (rank < kRankMax ? rank : kRankMax);
    }
    *c = (uint16_t)code;
  }
}

// The rare span with more than two samples inside: from its code's rank, the
// parity at its first node and a walk over its own samples (from the ray's
// start when the rank saturated).
__device__ __forceinline__ uint64_t span_walk(const AxisArrays* ax, size_t p, uint32_t code, const float* T,
                                              uint32_t* bad) {
  const uint32_t rank = code & kRankMax;
  if (rank == kRankMax) {
    bool b = false;
    const uint64_t m = span_mask(*ax, p, T, T[0], T[kSpan - 1], b);
    if (b) *bad = 1u;
    return m;
  }
  const uint32_t o0 = ax->offsets[p], o1 = ax->offsets[p + 1];
  if (o1 < o0 || (uint64_t)o1 > ax->n) {
    *bad = 1u;
    return 0;
  }
  const uint32_t end = o0 + ((o1 - o0) & ~1u);
  const float t_first = T[0], t_last = T[kSpan - 1];
  uint64_t m = (code & kCodeParity) ? ~0ull : 0ull;
  for (uint32_t q = o0 + rank; q < end; ++q) {
    const float s = ax->depth[q];
    if (!(s <= t_last)) break;
    const int c = s <= t_first ? 0 : count_below<kSpan>(T, s);
    m ^= c >= 64 ? 0ull : (~0ull << c);
  }
  return m;
}

// Inside mask of a span from its code (bit t = node t of the span).
__device__ __forceinline__ uint64_t decode_span(uint32_t code) {
  uint64_t m = (code & kCodeParity) ? ~0ull : 0ull;
  const uint32_t t1 = code & 63u, t2 = (code >> 6) & 63u;
  if (t1) m ^= ~0ull << t1;
  if (t2) m ^= ~0ull << t2;
  return m;
}

__device__ __forceinline__ uint32_t code_at(const uint4& c, int m) {
  const uint32_t word = m < 2 ? c.x : m < 4 ? c.y : m < 6 ? c.z : c.w;
  return (m & 1) ? word >> 16 : word & 0xffffu;
}

// LDS bit matrices of one step: y matrix (k, j-half, i-half) and z matrix
// (j, k-half, i-half), 32 rows of kRow words.
__device__ __forceinline__ int ymat(int kl, int jh, int ih) { return (ih * 2 + jh) * kSpan + kl; }
__device__ __forceinline__ int zmat(int jl, int kh, int ih) { return 4 * kSpan + (ih * 2 + kh) * kSpan + jl; }

// The vote.  A workgroup owns the 64 x 64 rows (j, k) of one block and walks
// along i one span (two bricks) per step.  Thread t handles the 8 consecutive
// codes v = 8t .. 8t + 7 of each axis (one 16-byte load each, issued a step
// ahead).
__global__ __launch_bounds__(kVoteBlock, 4) void classify_nodes_kernel(NodeArgs g) {
  __shared__ uint32_t s_m[8 * kSpan * kRow];  // 256 y and 256 z matrices
  __shared__ float s_ty[kSpan], s_tz[kSpan];
  __shared__ float s_tx[2][kSpan];  // node depths of the current and the next span along i
  __shared__ uint64_t s_sum[2][kVoteBlock / 64];

  const int tid = threadIdx.x;
  const int w = g.w, nb = g.nb, S = g.n_spans;
  const int J = (int)(blockIdx.x % S), K = (int)(blockIdx.x / S);
  const int j0 = J * kSpan, k0 = K * kSpan;
  const AxisArrays& X = g.axis[0];
  const AxisArrays& Y = g.axis[1];
  const AxisArrays& Z = g.axis[2];
  const size_t per_axis = (size_t)S * S * S * 4096;
  // x codes of this block: v = kl*64 + jl; thread t takes jl = t % 64 and kl = (t / 64)*8 + m
  const uint16_t* cx = g.codes + ((size_t)K * S + J) * 4096 + (size_t)(tid >> 6) * 512 + (tid & 63);
  const uint4* cy = reinterpret_cast<const uint4*>(g.codes + per_axis) + ((size_t)J * S + K) * S * 512 + tid;
  const uint4* cz = reinterpret_cast<const uint4*>(g.codes + 2 * per_axis) + ((size_t)K * S + J) * S * 512 + tid;
  const size_t x_step = (size_t)S * S * 4096;  // codes per x span step

  if (tid < kSpan) s_ty[tid] = node_depth(g.lo[1], g.h[1], j0 + tid, w);
  else if (tid < 2 * kSpan) s_tz[tid - kSpan] = node_depth(g.lo[2], g.h[2], k0 + tid - kSpan, w);
  else if (tid < 3 * kSpan) s_tx[0][tid - 2 * kSpan] = node_depth(g.lo[0], g.h[0], tid - 2 * kSpan, w);
  // this thread's rays: 8 consecutive v = 8 tid + m
  const int hi6 = tid >> 3, lo6 = (tid & 7) * 8;  // v / 64, v % 64 - m
  uint32_t nx[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) nx[m] = cx[m * 64];
  uint4 ny = cy[0], nz = cz[0];
  __syncthreads();
  uint32_t n_inside = 0, n_split = 0;
  uint32_t bad = 0;

  for (int it = 0; it < S; ++it) {
    uint32_t ux[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) ux[m] = nx[m];
    const uint4 uy = ny, uz = nz;
    if (it + 1 < S) {
#pragma unroll
      for (int m = 0; m < 8; ++m) nx[m] = cx[(size_t)(it + 1) * x_step + m * 64];
      ny = cy[(size_t)(it + 1) * 512];
      nz = cz[(size_t)(it + 1) * 512];
    }
    const int i0 = it * kSpan;
    const float* TX = s_tx[it & 1];
    // y spans: v = il*64 + kl (il = hi6, kl = lo6 + m); z spans: v = jl*64 + il (jl = hi6, il = lo6 + m)
#pragma unroll 1
    for (int m = 0; m < 8; ++m) {
      {
        const int il = hi6, kl = lo6 + m;
        const int i = i0 + il, k = k0 + kl;
        uint64_t mk = 0;
        if (i < w && k < w) {
          const uint32_t c = code_at(uy, m);
          mk = (c & kCodeWalk) ? span_walk(&Y, (size_t)i * w + k, c, s_ty, &bad) : decode_span(c);
        }
        s_m[ymat(kl, 0, il >> 5) * kRow + (il & 31)] = (uint32_t)mk;
        s_m[ymat(kl, 1, il >> 5) * kRow + (il & 31)] = (uint32_t)(mk >> 32);
      }
      {
        const int jl = hi6, il = lo6 + m;
        const int i = i0 + il, j = j0 + jl;
        uint64_t mk = 0;
        if (i < w && j < w) {
          const uint32_t c = code_at(uz, m);
          mk = (c & kCodeWalk) ? span_walk(&Z, (size_t)j * w + i, c, s_tz, &bad) : decode_span(c);
        }
        s_m[zmat(jl, 0, il >> 5) * kRow + (il & 31)] = (uint32_t)mk;
        s_m[zmat(jl, 1, il >> 5) * kRow + (il & 31)] = (uint32_t)(mk >> 32);
      }
    }
    __syncthreads();
    // one 32 x 32 transpose per thread; a spare wave fills the next span's depths
    transpose32(s_m + tid * kRow);
    __syncthreads();
    if (tid >= kVoteBlock - kSpan)
      s_tx[(it + 1) & 1][tid - (kVoteBlock - kSpan)] = node_depth(g.lo[0], g.h[0], i0 + kSpan + tid - (kVoteBlock - kSpan), w);
    // majority of the three words: x-ray (jl, kl), jl = t % 64, kl = (t / 64)*8 + m;
    // a wave stores 64 consecutive words of two brick rows per instruction.
    // For m = 0..7 the y word moves by one matrix (kRow words), the z word by
    // one row and the output by one brick row (32 words).
    const int jl = tid & 63, j = j0 + jl;
    const int kl0 = (tid >> 6) * 8;
    const uint32_t* yp = s_m + ymat(kl0, jl >> 5, 0) * kRow + (jl & 31);
    const uint32_t* zp = s_m + zmat(jl, kl0 >> 5, 0) * kRow + (kl0 & 31);
    constexpr int kYHalf = 2 * kSpan * kRow;  // the i-half step of a y matrix index (ih * 2 * 64 matrices)
    const int bj = 2 * J + (jl >> 5), bk = 2 * K + (kl0 >> 5);
    uint32_t valid[2];
#pragma unroll
    for (int ih = 0; ih < 2; ++ih) {
      const int ib = i0 + 32 * ih;
      valid[ih] = (ib >= w || j >= w) ? 0u : (w - ib >= 32) ? 0xffffffffu : ((1u << (w - ib)) - 1u);
    }
    const bool store[2] = {2 * it < nb && bj < nb && bk < nb, 2 * it + 1 < nb && bj < nb && bk < nb};
    uint32_t* op[2] = {g.bits + (((size_t)bk * nb + bj) * nb + 2 * it) * 1024 + (kl0 & 31) * 32 + (jl & 31),
                       g.bits + (((size_t)bk * nb + bj) * nb + 2 * it + 1) * 1024 + (kl0 & 31) * 32 + (jl & 31)};
#pragma unroll 1
    for (int m = 0; m < 8; ++m) {
      const int k = k0 + kl0 + m;
      uint64_t xm = 0;
      if (j < w && k < w) {
        const uint32_t c = ux[m];
        xm = (c & kCodeWalk) ? span_walk(&X, (size_t)k * w + j, c, TX, &bad) : decode_span(c);
      }
      const bool krow = k < w;
#pragma unroll
      for (int ih = 0; ih < 2; ++ih) {
        const uint32_t xw = (uint32_t)(xm >> (32 * ih));
        const uint32_t yw = yp[m * kRow + ih * kYHalf];
        const uint32_t zw = zp[m + ih * kYHalf];
        // rows past the grid hold no node (their y or z words may carry fill bits)
        const uint32_t row = krow ? valid[ih] : 0u;
        const uint32_t in = ((xw & yw) | (xw & zw) | (yw & zw)) & row;
        n_inside += __popc(in);
        n_split += __popc(((xw | yw | zw) & ~(xw & yw & zw)) & row);
        if (store[ih]) op[ih][m * 32] = in;
      }
    }
    __syncthreads();  // the next step rewrites the matrices
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
  const uint32_t S = (uint32_t)((w + kSpan - 1) / kSpan);
  return S * S;
}

size_t node_code_bytes(int32_t w) {
  const size_t S = (size_t)((w + kSpan - 1) / kSpan);
  return 3 * S * S * S * 4096 * sizeof(uint16_t);
}

hipError_t launch_node_codes(const NodeArgs& g, hipStream_t s) {
  const int64_t npix = (int64_t)g.w * g.w;
  hipLaunchKernelGGL(node_codes_kernel, dim3((unsigned)((npix + kNodeBlock - 1) / kNodeBlock), 3), dim3(kNodeBlock),
                     sizeof(float) * (size_t)g.w, s, g);
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
