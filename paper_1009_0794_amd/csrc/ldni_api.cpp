// ldni_api.cpp -- host side of the C ABI declared in include/ldni.h:
// argument validation (before any GPU call), workspace and output allocation
// from the device's stream-ordered pool, launch sequencing and the readbacks
// of the data-dependent sizes.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ldni.h"
#include "ldni_internal.hpp"

using namespace ldni;

namespace {

thread_local std::string g_last_error;
std::atomic<int> g_tile_w{32};
std::atomic<int> g_tile_h{32};

ldni_status fail(ldni_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

ldni_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(LDNI_ERR_OUT_OF_MEMORY, std::string(what) + ": " + hipGetErrorString(e));
  return fail(LDNI_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                     \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Keep freed pool memory cached on the device instead of returning it to the
// driver at every synchronisation.
void prepare_pool(int device) {
  static std::mutex mu;
  static bool done[64] = {};
  std::lock_guard<std::mutex> lk(mu);
  if (device < 0 || device >= 64 || done[device]) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  done[device] = true;
}

// Small pinned host buffer per thread for the size readbacks.
uint32_t* pinned_readback() {
  thread_local uint32_t* p = nullptr;
  if (!p) {
    if (hipHostMalloc(reinterpret_cast<void**>(&p), 4096, hipHostMallocDefault) != hipSuccess)
      p = nullptr;
  }
  return p;
}

bool env_fault(const char* what) {
  const char* f = std::getenv("LDNI_FAULT");
  return f && std::strstr(f, what) != nullptr;
}

hipError_t pool_alloc(void** p, size_t bytes, hipStream_t s) {
  if (env_fault("alloc")) return hipErrorOutOfMemory;
  if (bytes == 0) bytes = 256;
  return hipMallocAsync(p, bytes, s);
}

ldni_status validate(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                     const float bbox[6], int32_t w, uint32_t axis_mask) {
  if (w < 1 || w > 16384) return fail(LDNI_ERR_INVALID_ARG, "w must be in [1, 16384]");
  if (axis_mask == 0 || axis_mask > 7) return fail(LDNI_ERR_INVALID_ARG, "axis_mask must be in [1, 7]");
  if (n_verts < 0 || n_tris < 0) return fail(LDNI_ERR_INVALID_ARG, "negative vertex or triangle count");
  if (n_tris >= (int64_t(1) << 31)) return fail(LDNI_ERR_INVALID_ARG, "n_tris must be < 2^31");
  if (n_verts >= (int64_t(1) << 40)) return fail(LDNI_ERR_INVALID_ARG, "n_verts too large");
  if (n_tris > 0 && (!tris || !verts || n_verts == 0))
    return fail(LDNI_ERR_INVALID_ARG, "NULL vertex/triangle pointer with triangles present");
  if (!bbox) return fail(LDNI_ERR_INVALID_ARG, "bbox is NULL");
  for (int d = 0; d < 3; ++d) {
    if (!std::isfinite(bbox[d]) || !std::isfinite(bbox[3 + d]))
      return fail(LDNI_ERR_INVALID_ARG, "bbox must be finite");
    if (!(bbox[d] < bbox[3 + d])) return fail(LDNI_ERR_INVALID_ARG, "bbox needs lo < hi on every axis");
  }
  return LDNI_OK;
}

// ---- optional kernel timing ----
struct ProfRecord {
  const char* name;
  hipEvent_t start, stop;
};
std::mutex g_prof_mu;
std::atomic<bool> g_prof_on{false};
std::vector<ProfRecord> g_prof;

template <class F>
hipError_t timed(const char* name, hipStream_t s, F&& launch) {
  if (!g_prof_on.load(std::memory_order_relaxed)) return launch();
  ProfRecord r{name, nullptr, nullptr};
  if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess)
    return launch();
  (void)hipEventRecord(r.start, s);
  const hipError_t e = launch();
  (void)hipEventRecord(r.stop, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof.push_back(r);
  return e;
}

}  // namespace

// ---------------------------------------------------------------------------
// opaque handles
// ---------------------------------------------------------------------------
struct ldni_plan {
  hipStream_t stream = nullptr;
  int32_t w = 0;
  uint32_t mask = 0;
  int64_t n_tris = 0;
  ImageSet set{};
  int axis_of[kMaxImages] = {0, 0, 0};  // image k samples axis axis_of[k]
  void* ws = nullptr;     // workspace
  void* lists = nullptr;  // tile lists
  uint64_t n[3] = {0, 0, 0};
  uint32_t max_layers[3] = {0, 0, 0};
};

struct ldni_result {
  hipStream_t stream = nullptr;
  void* offsets_buf = nullptr;
  void* samples_buf = nullptr;
  ldni_axis_view view[3];
};

namespace {

void release_plan(ldni_plan* p) {
  if (!p) return;
  if (p->lists) hipFreeAsync(p->lists, p->stream);
  if (p->ws) hipFreeAsync(p->ws, p->stream);
  delete p;
}

}  // namespace

extern "C" {

const char* ldni_status_string(ldni_status s) {
  switch (s) {
    case LDNI_OK: return "LDNI_OK";
    case LDNI_ERR_INVALID_ARG: return "LDNI_ERR_INVALID_ARG";
    case LDNI_ERR_INDEX: return "LDNI_ERR_INDEX";
    case LDNI_ERR_OUT_OF_MEMORY: return "LDNI_ERR_OUT_OF_MEMORY";
    case LDNI_ERR_OVERFLOW: return "LDNI_ERR_OVERFLOW";
    case LDNI_ERR_DEVICE: return "LDNI_ERR_DEVICE";
    case LDNI_ERR_NONFINITE: return "LDNI_ERR_NONFINITE";
  }
  return "LDNI_ERR_UNKNOWN";
}

const char* ldni_last_error(void) { return g_last_error.c_str(); }

ldni_status ldni_set_tile_shape(int32_t tw, int32_t th) {
  if (tw < 8 || tw > 256 || th < 1 || th > 64 || tw * th > 1024)
    return fail(LDNI_ERR_INVALID_ARG, "tile shape needs 8<=tw<=256, 1<=th<=64, tw*th<=1024");
  g_tile_w.store(tw);
  g_tile_h.store(th);
  return LDNI_OK;
}

ldni_status ldni_sample_begin(const float* verts, int64_t n_verts, const int32_t* tris,
                              int64_t n_tris, const float bbox[6], int32_t w, uint32_t axis_mask,
                              uint32_t* const offsets[3], void* hip_stream, ldni_plan** plan_out,
                              uint64_t n_samples[3]) {
  if (plan_out) *plan_out = nullptr;
  if (!plan_out || !n_samples || !offsets) return fail(LDNI_ERR_INVALID_ARG, "NULL output argument");
  ldni_status st = validate(verts, n_verts, tris, n_tris, bbox, w, axis_mask);
  if (st != LDNI_OK) return st;
  for (int a = 0; a < 3; ++a)
    if ((axis_mask >> a) & 1u)
      if (!offsets[a]) return fail(LDNI_ERR_INVALID_ARG, "NULL offsets buffer for a requested axis");
  for (int a = 0; a < 3; ++a) n_samples[a] = 0;
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);

  int device = 0;
  HIP_TRY(hipGetDevice(&device), "hipGetDevice");
  prepare_pool(device);
  uint32_t* rb = pinned_readback();
  if (!rb) return fail(LDNI_ERR_OUT_OF_MEMORY, "pinned readback buffer");

  ldni_plan* p = new (std::nothrow) ldni_plan();
  if (!p) return fail(LDNI_ERR_OUT_OF_MEMORY, "plan");
  p->stream = stream;
  p->w = w;
  p->mask = axis_mask;
  p->n_tris = n_tris;

  const int tw = g_tile_w.load(), th = g_tile_h.load();
  const int ntx = (w + tw - 1) / tw, nty = (w + th - 1) / th;
  const int64_t n_tiles = (int64_t)ntx * nty;
  const int64_t npix = (int64_t)w * w;

  // ---- workspace layout ----
  size_t off = 0;
  const size_t o_status = off; off += 256;
  const size_t o_soup = off; off = align_up(off + sizeof(float) * 9 * (size_t)n_tris);
  const size_t o_tnorm = off; off = align_up(off + sizeof(float) * 3 * (size_t)n_tris);
  size_t o_rect[kMaxImages], o_tcnt[kMaxImages], o_tcur[kMaxImages], o_counts[kMaxImages];
  int nimg = 0;
  for (int a = 0; a < 3; ++a)
    if ((axis_mask >> a) & 1u) p->axis_of[nimg++] = a;
  for (int k = 0; k < nimg; ++k) {
    o_rect[k] = off; off = align_up(off + sizeof(Rect) * (size_t)n_tris);
    o_tcnt[k] = off; off = align_up(off + sizeof(uint32_t) * (size_t)(n_tiles + 1));
    o_tcur[k] = off; off = align_up(off + sizeof(uint32_t) * (size_t)n_tiles);
    o_counts[k] = off; off = align_up(off + sizeof(uint32_t) * (size_t)npix);
  }
  const size_t o_scan = off;
  off = align_up(off + std::max(scan_scratch_bytes(npix), scan_scratch_bytes(n_tiles)));

  hipError_t e = pool_alloc(&p->ws, off, stream);
  if (e != hipSuccess) {
    p->ws = nullptr;
    release_plan(p);
    return hip_fail(e, "workspace allocation");
  }
  char* ws = static_cast<char*>(p->ws);
  uint32_t* status = reinterpret_cast<uint32_t*>(ws + o_status);  // [0]=status, [1..3]=max layers

  MeshSetup ms{};
  ms.verts = verts;
  ms.n_verts = n_verts;
  ms.tris = tris;
  ms.n_tris = n_tris;
  ms.soup = reinterpret_cast<float*>(ws + o_soup);
  ms.tnorm = reinterpret_cast<float*>(ws + o_tnorm);
  ms.status = status;

  ImageSet& set = p->set;
  set.n = nimg;
  set.tile_start[0] = 0;
  for (int k = 0; k < nimg; ++k) {
    const int a = p->axis_of[k];
    Image& im = set.img[k];
    im.a = a;
    im.u = (a + 1) % 3;
    im.v = (a + 2) % 3;
    im.w = w;
    im.lo_u = (double)bbox[im.u];
    im.h_u = ((double)bbox[3 + im.u] - (double)bbox[im.u]) / (double)w;
    im.lo_v = (double)bbox[im.v];
    im.h_v = ((double)bbox[3 + im.v] - (double)bbox[im.v]) / (double)w;
    im.lo_a = (double)bbox[a];
    im.tw = tw;
    im.th = th;
    im.ntx = ntx;
    im.nty = nty;
    im.soup = ms.soup;
    im.tnorm = ms.tnorm;
    im.rect = reinterpret_cast<const Rect*>(ws + o_rect[k]);
    ms.rect[k] = reinterpret_cast<Rect*>(ws + o_rect[k]);
    im.n_tris = n_tris;
    im.tile_cnt = reinterpret_cast<uint32_t*>(ws + o_tcnt[k]);
    im.tile_cur = reinterpret_cast<uint32_t*>(ws + o_tcur[k]);
    im.tile_list = nullptr;
    im.counts = reinterpret_cast<uint32_t*>(ws + o_counts[k]);
    im.max_layers = status + 1 + k;
    im.offsets = offsets[a];
    im.status = status;
    set.tile_start[k + 1] = set.tile_start[k] + (uint32_t)n_tiles;
  }
  void* scan_scratch = ws + o_scan;

  auto bail = [&](ldni_status s) {
    release_plan(p);
    return s;
  };
#define STEP(expr, what)                              \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return bail(hip_fail(e_, what)); \
  } while (0)

  STEP(launch_fill_u32(status, 0u, 64, stream), "fill");
  for (int k = 0; k < nimg; ++k) {
    STEP(launch_fill_u32(set.img[k].tile_cnt, 0u, n_tiles + 1, stream), "fill");
    STEP(launch_fill_u32(set.img[k].tile_cur, 0u, n_tiles, stream), "fill");
  }
  STEP(timed("setup", stream, [&] { return launch_setup(ms, set, stream); }), "setup kernel");
  STEP(timed("bin_count", stream, [&] { return launch_bin_count(set, stream); }), "bin count kernel");
  for (int k = 0; k < nimg; ++k)
    STEP(timed("scan_tiles", stream, [&] {
           return launch_scan(set.img[k].tile_cnt, set.img[k].tile_cnt, n_tiles, scan_scratch, status, stream);
         }), "tile scan");
  // readback 1: tile-list sizes and input validity
  STEP(hipMemcpyAsync(rb, status, sizeof(uint32_t), hipMemcpyDeviceToHost, stream), "readback");
  for (int k = 0; k < nimg; ++k)
    STEP(hipMemcpyAsync(rb + 4 + k, set.img[k].tile_cnt + n_tiles, sizeof(uint32_t),
                        hipMemcpyDeviceToHost, stream), "readback");
  STEP(hipStreamSynchronize(stream), "synchronise");
  if (rb[0] & kStatusBadIndex) return bail(fail(LDNI_ERR_INDEX, "triangle index outside [0, n_verts)"));
  if (rb[0] & kStatusNonFinite) return bail(fail(LDNI_ERR_NONFINITE, "non-finite vertex coordinate"));
  size_t list_off[kMaxImages];
  size_t lbytes = 0;
  for (int k = 0; k < nimg; ++k) {
    list_off[k] = lbytes;
    lbytes = align_up(lbytes + sizeof(int32_t) * (size_t)rb[4 + k]);
  }
  e = pool_alloc(&p->lists, lbytes, stream);
  if (e != hipSuccess) {
    p->lists = nullptr;
    return bail(hip_fail(e, "tile list allocation"));
  }
  for (int k = 0; k < nimg; ++k)
    set.img[k].tile_list = reinterpret_cast<int32_t*>(static_cast<char*>(p->lists) + list_off[k]);

  STEP(timed("bin_scatter", stream, [&] { return launch_bin_scatter(set, stream); }), "bin scatter kernel");
  STEP(timed("count", stream, [&] { return launch_count(set, stream); }), "count kernel");
  for (int k = 0; k < nimg; ++k)
    STEP(timed("scan_pixels", stream, [&] {
           return launch_scan(set.img[k].counts, set.img[k].offsets, npix, scan_scratch, status, stream);
         }), "pixel scan");
  // readback 2: sample totals
  STEP(hipMemcpyAsync(rb, status, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, stream), "readback");
  for (int k = 0; k < nimg; ++k)
    STEP(hipMemcpyAsync(rb + 4 + k, set.img[k].offsets + npix, sizeof(uint32_t),
                        hipMemcpyDeviceToHost, stream), "readback");
  STEP(hipStreamSynchronize(stream), "synchronise");
  if (rb[0] & kStatusOverflow) return bail(fail(LDNI_ERR_OVERFLOW, "2^32 or more samples on one axis"));
  for (int k = 0; k < nimg; ++k) {
    const int a = p->axis_of[k];
    p->n[a] = rb[4 + k];
    p->max_layers[a] = rb[1 + k];
    n_samples[a] = p->n[a];
  }
#undef STEP
  *plan_out = p;
  return LDNI_OK;
}

ldni_status ldni_plan_max_layers(const ldni_plan* plan, uint32_t max_layers[3]) {
  if (!plan || !max_layers) return fail(LDNI_ERR_INVALID_ARG, "NULL argument");
  for (int a = 0; a < 3; ++a) max_layers[a] = plan->max_layers[a];
  return LDNI_OK;
}

ldni_status ldni_sample_finish(ldni_plan* p, float* const depth[3], float* const normal[3],
                               int32_t* const tri[3]) {
  if (!p) return fail(LDNI_ERR_INVALID_ARG, "NULL plan");
  if (!depth || !normal || !tri) {
    release_plan(p);
    return fail(LDNI_ERR_INVALID_ARG, "NULL output array");
  }
  for (int k = 0; k < p->set.n; ++k) {
    const int a = p->axis_of[k];
    if (p->n[a] > 0 && (!depth[a] || !normal[a] || !tri[a])) {
      release_plan(p);
      return fail(LDNI_ERR_INVALID_ARG, "NULL output buffer for an axis with samples");
    }
    p->set.img[k].depth = depth[a];
    p->set.img[k].normal = normal[a];
    p->set.img[k].tri = tri[a];
  }
  hipError_t e = hipSuccess;
  if (p->n_tris > 0) e = timed("write", p->stream, [&] { return launch_write(p->set, p->stream); });
  release_plan(p);
  if (e != hipSuccess) return hip_fail(e, "write kernel");
  return LDNI_OK;
}

void ldni_plan_free(ldni_plan* plan) { release_plan(plan); }

ldni_status ldni_profile_enable(int enable) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (enable) {
    for (auto& r : g_prof) {
      (void)hipEventDestroy(r.start);
      (void)hipEventDestroy(r.stop);
    }
    g_prof.clear();
  }
  g_prof_on.store(enable != 0);
  return LDNI_OK;
}

ldni_status ldni_profile_read(ldni_kernel_stat* stats, int32_t max, int32_t* n) {
  if (!n || (max > 0 && !stats)) return fail(LDNI_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  std::vector<ldni_kernel_stat> acc;
  for (auto& r : g_prof) {
    if (hipEventSynchronize(r.stop) != hipSuccess) return fail(LDNI_ERR_DEVICE, "event wait");
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return fail(LDNI_ERR_DEVICE, "event time");
    size_t k = 0;
    while (k < acc.size() && std::strcmp(acc[k].name, r.name) != 0) ++k;
    if (k == acc.size()) acc.push_back(ldni_kernel_stat{r.name, 0, 0.0});
    acc[k].launches += 1;
    acc[k].total_ms += ms;
  }
  *n = (int32_t)acc.size();
  for (int32_t k = 0; k < max && k < (int32_t)acc.size(); ++k) stats[k] = acc[k];
  return LDNI_OK;
}

ldni_status ldni_sample(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                        const float bbox[6], int32_t w, uint32_t axis_mask, void* hip_stream,
                        ldni_result** out) {
  if (out) *out = nullptr;
  if (!out) return fail(LDNI_ERR_INVALID_ARG, "NULL result pointer");
  ldni_status st = validate(verts, n_verts, tris, n_tris, bbox, w, axis_mask);
  if (st != LDNI_OK) return st;
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  int device = 0;
  HIP_TRY(hipGetDevice(&device), "hipGetDevice");
  prepare_pool(device);

  ldni_result* r = new (std::nothrow) ldni_result();
  if (!r) return fail(LDNI_ERR_OUT_OF_MEMORY, "result");
  std::memset(r->view, 0, sizeof(r->view));
  r->stream = stream;
  const size_t per_axis = align_up(sizeof(uint32_t) * ((size_t)w * w + 1));
  hipError_t e = pool_alloc(&r->offsets_buf, 3 * per_axis, stream);
  if (e != hipSuccess) {
    delete r;
    return hip_fail(e, "offsets allocation");
  }
  uint32_t* offs[3] = {nullptr, nullptr, nullptr};
  for (int a = 0; a < 3; ++a)
    if ((axis_mask >> a) & 1u)
      offs[a] = reinterpret_cast<uint32_t*>(static_cast<char*>(r->offsets_buf) + a * per_axis);

  ldni_plan* plan = nullptr;
  uint64_t n[3];
  st = ldni_sample_begin(verts, n_verts, tris, n_tris, bbox, w, axis_mask, offs, hip_stream, &plan, n);
  if (st != LDNI_OK) {
    ldni_free(r);
    return st;
  }
  size_t o_depth[3], o_normal[3], o_tri[3];
  size_t bytes = 0;
  for (int a = 0; a < 3; ++a) {
    o_depth[a] = bytes; bytes = align_up(bytes + sizeof(float) * n[a]);
    o_normal[a] = bytes; bytes = align_up(bytes + sizeof(float) * 3 * n[a]);
    o_tri[a] = bytes; bytes = align_up(bytes + sizeof(int32_t) * n[a]);
  }
  e = pool_alloc(&r->samples_buf, bytes, stream);
  if (e != hipSuccess) {
    r->samples_buf = nullptr;
    ldni_plan_free(plan);
    ldni_free(r);
    return hip_fail(e, "sample allocation");
  }
  char* sb = static_cast<char*>(r->samples_buf);
  float* dp[3];
  float* np_[3];
  int32_t* tp[3];
  uint32_t ml[3];
  ldni_plan_max_layers(plan, ml);
  for (int a = 0; a < 3; ++a) {
    dp[a] = reinterpret_cast<float*>(sb + o_depth[a]);
    np_[a] = reinterpret_cast<float*>(sb + o_normal[a]);
    tp[a] = reinterpret_cast<int32_t*>(sb + o_tri[a]);
    if ((axis_mask >> a) & 1u) {
      ldni_axis_view& v = r->view[a];
      v.w = w;
      v.max_layers = ml[a];
      v.n_samples = n[a];
      v.offsets = offs[a];
      v.depth = dp[a];
      v.normal = np_[a];
      v.tri = tp[a];
    }
  }
  st = ldni_sample_finish(plan, dp, np_, tp);
  if (st != LDNI_OK) {
    ldni_free(r);
    return st;
  }
  *out = r;
  return LDNI_OK;
}

ldni_status ldni_result_axis(const ldni_result* r, int axis, ldni_axis_view* view) {
  if (!r || !view || axis < 0 || axis > 2) return fail(LDNI_ERR_INVALID_ARG, "bad result/axis/view");
  *view = r->view[axis];
  return LDNI_OK;
}

void ldni_free(ldni_result* r) {
  if (!r) return;
  if (r->samples_buf) hipFreeAsync(r->samples_buf, r->stream);
  if (r->offsets_buf) hipFreeAsync(r->offsets_buf, r->stream);
  delete r;
}

}  // extern "C"
