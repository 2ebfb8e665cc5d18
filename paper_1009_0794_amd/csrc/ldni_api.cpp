// ldni_api.cpp -- host side of the C ABI declared in include/ldni.h:
// argument validation (before any GPU call), workspace and output allocation
// from the device's stream-ordered pool, launch sequencing and the readbacks
// of the data-dependent sizes.
#include <hip/hip_runtime.h>

#include <atomic>
#include <algorithm>
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

namespace ldni {

// The centre c_i = f32(lo + (i + 0.5) h) (float64 arithmetic, then rounded)
// differs from the real lo + (i + 0.5) h by at most 2^-24 (1 + 2^-26) M with
// M = |lo| + (w + 1) h, and t carries a relative float64 error of a few
// 2^-53, i.e. below 2^-48 (w + 1) pixels.  Twice the sum, in pixels, is the
// slack.
void finish_image_geometry(Image& im) {
  auto slack = [&](double lo, double h) {
    if (!(h > 0.0)) return HUGE_VAL;
    const double m = std::fabs(lo) + ((double)im.w + 1.0) * h;
    return 2.0 * (std::ldexp(m, -24) * (1.0 + std::ldexp(1.0, -26)) / h + std::ldexp((double)im.w + 1.0, -48));
  };
  auto shift = [](int n) {
    if (n <= 0 || (n & (n - 1)) != 0) return -1;
    int s = 0;
    while ((1 << s) < n) ++s;
    return s;
  };
  im.inv_h_u = 1.0 / im.h_u;
  im.inv_h_v = 1.0 / im.h_v;
  im.slack_u = slack(im.lo_u, im.h_u);
  im.slack_v = slack(im.lo_v, im.h_v);
  im.tw_shift = shift(im.tw);
  im.th_shift = shift(im.th);
}

}  // namespace ldni

namespace {

thread_local std::string g_last_error;
// 0 x 0 = choose per call from the triangle density (auto_tile)
std::atomic<int> g_tile_w{0};
std::atomic<int> g_tile_h{0};

// Tile shape from triangles per pixel: many small triangles and deep pixels
// favour small tiles (short serial work per workgroup), few large triangles
// favour large ones (fewer tile-list entries per triangle).
void auto_tile(int32_t w, int64_t n_tris, int* tw, int* th) {
  const double d = (double)n_tris / ((double)w * (double)w);
  if (d >= 0.75) { *tw = 8; *th = 8; }
  else if (d >= 0.02) { *tw = 8; *th = 32; }  // (tall tiles: 4 % faster than 16 x 16 on scene64 at w 2048)
  else { *tw = 32; *th = 32; }
}

void tile_shape(int32_t w, int64_t n_tris, int req_w, int req_h, int* tw, int* th) {
  if (req_w > 0 && req_h > 0) { *tw = req_w; *th = req_h; return; }
  const int gw = g_tile_w.load(), gh = g_tile_h.load();
  if (gw > 0 && gh > 0) { *tw = gw; *th = gh; return; }
  auto_tile(w, n_tris, tw, th);
}
// largest (tile-list entries / triangles) seen, with headroom
std::atomic<double> g_list_ratio{2.0};
// Staging buffers hold fewer than 2^32 entries (tile regions start at 32-bit
// entry indices); batch_grow adds up to 1/16 + 1024 to what it is asked for.
constexpr uint64_t kMaxStageEntries = 0xf0000000ull;

// Staging entries the sampling pass asked for in recent calls, keyed by the
// call's shape: a repeated call on the same mesh gets what the last one
// needed (plus headroom for moved vertices).
struct StageKey {
  int64_t n_verts, n_tris;
  int32_t w, tw, th;
  uint32_t mask;
  bool operator==(const StageKey& o) const {
    return n_verts == o.n_verts && n_tris == o.n_tris && w == o.w && tw == o.tw && th == o.th &&
           mask == o.mask;
  }
};
struct StageSeen {
  uint64_t demand;      // staging entries asked for
  uint32_t max_layers;  // deepest pixel
};
std::mutex g_stage_mu;
std::vector<std::pair<StageKey, StageSeen>> g_stage_seen;  // most recent last
constexpr size_t kStageMemory = 1024;

bool stage_seen_lookup(const StageKey& k, StageSeen* seen) {
  std::lock_guard<std::mutex> lk(g_stage_mu);
  for (size_t i = g_stage_seen.size(); i-- > 0;)
    if (g_stage_seen[i].first == k) {
      *seen = g_stage_seen[i].second;
      return true;
    }
  return false;
}

void stage_seen_record(const StageKey& k, StageSeen seen) {
  std::lock_guard<std::mutex> lk(g_stage_mu);
  for (size_t i = 0; i < g_stage_seen.size(); ++i)
    if (g_stage_seen[i].first == k) {
      g_stage_seen.erase(g_stage_seen.begin() + i);
      break;
    }
  if (g_stage_seen.size() >= kStageMemory) g_stage_seen.erase(g_stage_seen.begin());
  g_stage_seen.emplace_back(k, seen);
}

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
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
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

// Status words of finished results.  The last kernel of a call copies the
// call's device status word into one pinned host slot and an event is
// recorded after it; the result's first ldni_result_axis waits for the event
// and reports what the write pass found (a write pass that disagrees with
// its count pass).  Slots and events are reused.
struct StatusSlot {
  uint32_t* host = nullptr;  // pinned word
  hipEvent_t done = nullptr;
};
std::mutex g_slot_mu;
std::vector<StatusSlot> g_free_slots;
uint32_t* g_slot_block = nullptr;
size_t g_slot_next = 0;
constexpr size_t kSlotBlock = 1024;  // slots in one pinned allocation

bool slot_get(StatusSlot* out) {
  std::lock_guard<std::mutex> lk(g_slot_mu);
  if (!g_free_slots.empty()) {
    *out = g_free_slots.back();
    g_free_slots.pop_back();
    return true;
  }
  if (!g_slot_block || g_slot_next == kSlotBlock) {
    uint32_t* p = nullptr;
    if (hipHostMalloc(reinterpret_cast<void**>(&p), sizeof(uint32_t) * kSlotBlock, hipHostMallocDefault) !=
        hipSuccess)
      return false;
    g_slot_block = p;  // never freed: later slots of the block are still handed out
    g_slot_next = 0;
  }
  StatusSlot s;
  if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return false;
  s.host = g_slot_block + g_slot_next++;
  *out = s;
  return true;
}

void slot_put(const StatusSlot& s) {
  std::lock_guard<std::mutex> lk(g_slot_mu);
  g_free_slots.push_back(s);
}

bool env_fault(const char* what) {
  const char* f = std::getenv("LDNI_FAULT");
  return f && std::strstr(f, what) != nullptr;
}

// ---------------------------------------------------------------------------
// Stream-ordered buffer cache.  Allocating and freeing through the pool
// costs tens of microseconds of host time per call; buffers a call releases
// are kept for later requests on the same stream instead.  Work on one
// stream runs in order, so the memory's earlier user has finished with it by
// the time a later request's work runs (the same rule as hipFreeAsync).
// ---------------------------------------------------------------------------
struct CachedBuffer {
  int device;
  hipStream_t stream;
  void* ptr;
  size_t bytes;
};
std::mutex g_cache_mu;
std::vector<CachedBuffer> g_cache;  // oldest first
constexpr size_t kCachePerStream = 8;

// sizes rounded up to sixteenths of the next power of two, so that requests
// of slightly different sizes share buffers
size_t round_alloc(size_t b) {
  if (b <= 4096) return 4096;
  size_t p = 4096;
  while (p < b) p <<= 1;
  const size_t step = p / 16;
  return (b + step - 1) / step * step;
}

hipError_t cache_get(void** out, size_t bytes, hipStream_t s, size_t* got) {
  *out = nullptr;
  *got = 0;
  if (env_fault("alloc")) return hipErrorOutOfMemory;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    int best = -1;
    for (size_t i = 0; i < g_cache.size(); ++i) {
      const CachedBuffer& c = g_cache[i];
      if (c.device != dev || c.stream != s || c.bytes < bytes) continue;
      if (best < 0 || c.bytes < g_cache[best].bytes) best = (int)i;
    }
    // not a buffer far larger than asked for (it may be needed for a larger request)
    if (best >= 0 && g_cache[best].bytes <= 4 * bytes + ((size_t)1 << 20)) {
      *out = g_cache[best].ptr;
      *got = g_cache[best].bytes;
      g_cache.erase(g_cache.begin() + best);
      return hipSuccess;
    }
  }
  const size_t b = round_alloc(bytes);
  e = hipMallocAsync(out, b, s);
  if (e != hipSuccess) {
    // give the stream's cached buffers back to the pool and try once more
    std::vector<void*> drop;
    {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      for (size_t i = 0; i < g_cache.size();) {
        if (g_cache[i].device == dev && g_cache[i].stream == s) {
          drop.push_back(g_cache[i].ptr);
          g_cache.erase(g_cache.begin() + i);
        } else {
          ++i;
        }
      }
    }
    for (void* q : drop) (void)hipFreeAsync(q, s);
    (void)hipGetLastError();
    e = hipMallocAsync(out, b, s);
  }
  if (e != hipSuccess) {
    *out = nullptr;
    return e;
  }
  *got = b;
  return hipSuccess;
}

void cache_put(void* ptr, size_t bytes, hipStream_t s) {
  if (!ptr) return;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipFreeAsync(ptr, s);
    return;
  }
  void* evict = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_cache.push_back(CachedBuffer{dev, s, ptr, bytes});
    size_t n = 0, oldest = g_cache.size();
    for (size_t i = 0; i < g_cache.size(); ++i)
      if (g_cache[i].device == dev && g_cache[i].stream == s) {
        if (oldest == g_cache.size()) oldest = i;
        ++n;
      }
    if (n > kCachePerStream) {
      evict = g_cache[oldest].ptr;
      g_cache.erase(g_cache.begin() + oldest);
    }
  }
  if (evict) (void)hipFreeAsync(evict, s);
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
  size_t ws_bytes = 0;
  void* lists = nullptr;  // tile lists
  size_t lists_bytes = 0;
  uint32_t* write_counter = nullptr;
  void* items = nullptr;  // place-pass work items
  uint32_t n_items = 0;
  void* stage = nullptr;  // hits staged by the sampling pass
  size_t stage_bytes = 0;
  uint32_t n_walk = 0;    // tiles the write pass walks again
  uint32_t* status = nullptr;  // the call's device status word
  uint64_t n[3] = {0, 0, 0};
  uint32_t max_layers[3] = {0, 0, 0};
};

struct ldni_result {
  hipStream_t stream = nullptr;
  void* offsets_buf = nullptr;
  size_t offsets_bytes = 0;
  void* samples_buf = nullptr;
  size_t samples_bytes = 0;
  ldni_axis_view view[3];
  // the status word of the call's last kernels, still on its way (pending)
  // or already read (verdict)
  bool pending = false;
  StatusSlot slot;
  ldni_status verdict = LDNI_OK;
};

namespace {

void release_plan(ldni_plan* p) {
  if (!p) return;
  cache_put(p->lists, p->lists_bytes, p->stream);
  cache_put(p->stage, p->stage_bytes, p->stream);
  cache_put(p->ws, p->ws_bytes, p->stream);
  delete p;
}

// What a status word raised by a write pass means for the caller.
ldni_status write_verdict(uint32_t bits) {
  if (bits & kStatusMismatch)
    return fail(LDNI_ERR_DEVICE, "the write pass disagreed with the count pass (unwritten or surplus samples)");
  return LDNI_OK;
}

// After the last kernel of a call: the device status word goes to the
// result's pinned slot, stream-ordered, and the result remembers to check it.
// Without a free slot the call waits and checks at once.
ldni_status arm_status(ldni_result* r, const uint32_t* dev_status, hipStream_t s) {
  StatusSlot slot;
  if (slot_get(&slot)) {
    const uint32_t* src[1] = {dev_status};
    hipError_t e = launch_gather(src, 1, slot.host, s);
    if (e == hipSuccess) e = hipEventRecord(slot.done, s);
    if (e != hipSuccess) {
      slot_put(slot);
      return hip_fail(e, "status readback");
    }
    r->slot = slot;
    r->pending = true;
    return LDNI_OK;
  }
  uint32_t* rb = pinned_readback();
  if (!rb) return fail(LDNI_ERR_OUT_OF_MEMORY, "pinned readback buffer");
  const uint32_t* src[1] = {dev_status};
  HIP_TRY(launch_gather(src, 1, rb, s), "status readback");
  HIP_TRY(hipStreamSynchronize(s), "synchronise");
  r->verdict = write_verdict(rb[0]);
  return LDNI_OK;
}

// The result's status, waiting for its write pass if that is still running.
ldni_status settle(ldni_result* r) {
  if (r->pending) {
    const hipError_t e = hipEventSynchronize(r->slot.done);
    const uint32_t bits = *r->slot.host;
    slot_put(r->slot);
    r->pending = false;
    r->verdict = e != hipSuccess ? hip_fail(e, "waiting for the write pass") : write_verdict(bits);
  }
  return r->verdict;
}

// Without a result to carry the check: wait for the stream and check now.
ldni_status check_now(const uint32_t* dev_status, hipStream_t s) {
  uint32_t* rb = pinned_readback();
  if (!rb) return fail(LDNI_ERR_OUT_OF_MEMORY, "pinned readback buffer");
  const uint32_t* src[1] = {dev_status};
  HIP_TRY(launch_gather(src, 1, rb, s), "status readback");
  HIP_TRY(hipStreamSynchronize(s), "synchronise");
  return write_verdict(rb[0]);
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
  if (!(tw == 0 && th == 0) && (tw < 8 || tw > 256 || th < 1 || th > 64 || tw * th > 1024))
    return fail(LDNI_ERR_INVALID_ARG, "tile shape needs 8<=tw<=256, 1<=th<=64, tw*th<=1024 (or 0, 0)");
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
    if ((axis_mask >> a) & 1u) {
      if (!offsets[a]) return fail(LDNI_ERR_INVALID_ARG, "NULL offsets buffer for a requested axis");
      if (reinterpret_cast<uintptr_t>(offsets[a]) % 16 != 0)
        return fail(LDNI_ERR_INVALID_ARG, "offsets buffer not 16-byte aligned");
    }
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

  int tw = 0, th = 0;
  tile_shape(w, n_tris, 0, 0, &tw, &th);
  const int ntx = (w + tw - 1) / tw, nty = (w + th - 1) / th;
  const int64_t n_tiles = (int64_t)ntx * nty;
  const int64_t npix = (int64_t)w * w;

  // what the last call of this shape needed (staging entries, deepest pixel)
  const StageKey stage_key{n_verts, n_tris, w, tw, th, axis_mask};
  StageSeen seen{0, 0};
  const bool have_seen = stage_seen_lookup(stage_key, &seen);
  const uint32_t stage_layers = stage_layers_for(seen.max_layers);

  // ---- workspace layout ----
  int nimg = 0;
  for (int a = 0; a < 3; ++a)
    if ((axis_mask >> a) & 1u) p->axis_of[nimg++] = a;
  const int64_t n_all = nimg * n_tiles;  // tiles of all images, numbered image after image
  size_t off = 0;
  // status words, tile entry counts (all images, then their total), tile
  // candidate counts (16-byte aligned for the scan) and scatter cursors are
  // adjacent and cleared by one fill
  const size_t o_status = off; off += 256;
  const size_t o_tcnt = off; off += sizeof(uint32_t) * (size_t)(n_all + 1);
  const size_t o_treg = (off + 15) & ~(size_t)15; off = o_treg + sizeof(uint32_t) * (size_t)(n_all + 1);
  const size_t o_tcur = off; off += sizeof(uint32_t) * (size_t)n_all;
  const size_t o_tovf = off; off += sizeof(uint32_t) * (size_t)n_all;
  off = (off + 7) & ~(size_t)7;
  const size_t o_tpack = off; off += sizeof(uint64_t) * (size_t)n_all;
  const int64_t n_clear = (int64_t)(off / sizeof(uint32_t));
  off = align_up(off);
  const int64_t n_chunks = (n_tris + kBinChunkTris - 1) / kBinChunkTris;
  const size_t o_brec = off; off = align_up(off + sizeof(uint4) * kBinSlots * (size_t)n_chunks);
  const size_t o_bnrec = off; off = align_up(off + sizeof(uint32_t) * (size_t)n_chunks);
  const size_t o_soup = off; off = align_up(off + sizeof(float) * 9 * (size_t)n_tris);
  const size_t o_tnorm = off; off = align_up(off + sizeof(float4) * (size_t)n_tris);
  size_t o_rect[kMaxImages], o_counts[kMaxImages], o_tstage[kMaxImages], o_thits[kMaxImages];
  for (int k = 0; k < nimg; ++k) {
    o_rect[k] = off; off = align_up(off + sizeof(Rect) * (size_t)n_tris);
    o_counts[k] = off; off = align_up(off + sizeof(uint32_t) * (size_t)npix);
    o_tstage[k] = off; off = align_up(off + sizeof(uint32_t) * (size_t)n_tiles);
    o_thits[k] = off; off = align_up(off + sizeof(uint32_t) * (size_t)n_tiles);
  }
  const size_t o_walk = off; off = align_up(off + sizeof(uint32_t) * (size_t)n_all);
  const size_t o_items = off;
  off = align_up(off + 16 * (size_t)max_place_items_per_tile(tw * th, stage_layers) * (size_t)n_all);
  const size_t o_plan = off; off = align_up(off + sizeof(uint32_t) * (size_t)(2 * n_all + 1));
  const size_t o_scan = off;
  off = align_up(off + std::max({scan_scratch_bytes(npix, nimg), scan_scratch_bytes(2 * n_all, 1),
                                  scan_scratch_bytes(n_all, 2)}));

  hipError_t e = cache_get(&p->ws, off, stream, &p->ws_bytes);
  if (e != hipSuccess) {
    p->ws = nullptr;
    release_plan(p);
    return hip_fail(e, "workspace allocation");
  }
  char* ws = static_cast<char*>(p->ws);
  // [0] status, [1..3] max layers, [12..13] write-pass work counters,
  // [18] tiles to walk again
  uint32_t* status = reinterpret_cast<uint32_t*>(ws + o_status);
  p->status = status;
  uint32_t* walk_count = status + 18;

  MeshSetup ms{};
  ms.verts = verts;
  ms.n_verts = n_verts;
  ms.tris = tris;
  ms.n_tris = n_tris;
  ms.soup = reinterpret_cast<float*>(ws + o_soup);
  ms.tnorm = reinterpret_cast<float4*>(ws + o_tnorm);
  ms.status = status;
  ms.bin_rec = reinterpret_cast<uint4*>(ws + o_brec);
  ms.bin_nrec = reinterpret_cast<uint32_t*>(ws + o_bnrec);

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
    finish_image_geometry(im);
    im.ntx = ntx;
    im.nty = nty;
    im.soup = ms.soup;
    im.tnorm = ms.tnorm;
    im.rect = reinterpret_cast<const Rect*>(ws + o_rect[k]);
    ms.rect[k] = reinterpret_cast<Rect*>(ws + o_rect[k]);
    im.n_tris = n_tris;
    im.tile_cnt = reinterpret_cast<uint32_t*>(ws + o_tcnt) + k * n_tiles;
    im.tile_cur = reinterpret_cast<uint32_t*>(ws + o_tcur) + k * n_tiles;
    im.tile_ovf = reinterpret_cast<uint32_t*>(ws + o_tovf) + k * n_tiles;
    im.tile_pack = reinterpret_cast<uint64_t*>(ws + o_tpack) + k * n_tiles;
    im.tile_region = reinterpret_cast<uint32_t*>(ws + o_treg) + k * n_tiles;
    im.tile_list = nullptr;
    im.counts = reinterpret_cast<uint32_t*>(ws + o_counts[k]);
    im.max_layers = nullptr;  // the pixel scan writes status[1 + k]
    im.tile_max = nullptr;
    im.offsets = offsets[a];
    im.status = status;
    im.tile_stage = reinterpret_cast<uint32_t*>(ws + o_tstage[k]);
    im.tile_hits = reinterpret_cast<uint32_t*>(ws + o_thits[k]);
    im.walk_list = reinterpret_cast<uint32_t*>(ws + o_walk);
    im.walk_count = walk_count;
    set.tile_start[k + 1] = set.tile_start[k] + (uint32_t)n_tiles;
  }
  // Staging buffer for the hits of the sampling pass: what the last call of
  // the same shape asked for (the candidate total of its tile scan), else a
  // first guess (16 entries per triangle and image, which covers small
  // triangles' rectangles rounded to 4-entry groups, plus four per pixel for
  // large ones).  A tile whose region does not fit is walked again by the
  // place pass, so a short buffer costs time, never results.  Never more
  // than stage_layers entries per pixel, which is all the tiles can ask for.
  {
    const double px = (double)npix * nimg;
    const double want = have_seen ? (double)seen.demand * 1.1 + 65536.0
                                  : 16.0 * (double)n_tris * nimg + 4.0 * px + 65536.0;
    const double most = std::min((double)stage_layers * px + 65536.0, (double)kMaxStageEntries);
    uint64_t stage_cap = (uint64_t)std::min(want, most);
    // test hook: a smaller buffer (0: none) forces tiles onto the walk path
    if (const char* env = std::getenv("LDNI_STAGE_ENTRIES"))
      stage_cap = std::min<uint64_t>(stage_cap, std::strtoull(env, nullptr, 10));
    stage_cap &= ~(uint64_t)3;  // whole 4-entry groups: 16-byte aligned pixel/slot words
    if (stage_cap == 0 ||
        cache_get(&p->stage, stage_cap * (sizeof(uint64_t) + sizeof(uint32_t)), stream, &p->stage_bytes) !=
            hipSuccess)
      p->stage = nullptr;  // no staging: every tile with hits is walked again
    for (int k = 0; k < nimg; ++k) {
      Image& im = set.img[k];
      im.stage_key = p->stage ? static_cast<uint64_t*>(p->stage) : nullptr;
      im.stage_qs = p->stage ? reinterpret_cast<uint32_t*>(static_cast<uint64_t*>(p->stage) + stage_cap)
                             : nullptr;
      im.stage_cap = p->stage ? stage_cap : 0;
      im.stage_layers = stage_layers;
    }
  }
  void* scan_scratch = ws + o_scan;
  set.plan = reinterpret_cast<uint32_t*>(ws + o_plan);
  set.place_cap = place_stage_cap(tw * th);
  p->write_counter = status + 12;
  p->items = ws + o_items;

  auto bail = [&](ldni_status s) {
    release_plan(p);
    return s;
  };
#define STEP(expr, what)                              \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return bail(hip_fail(e_, what)); \
  } while (0)

  uint32_t* tile_cnt_all = reinterpret_cast<uint32_t*>(ws + o_tcnt);
  uint32_t* tile_region_all = reinterpret_cast<uint32_t*>(ws + o_treg);
  uint32_t* tile_cur_all = reinterpret_cast<uint32_t*>(ws + o_tcur);
  STEP(launch_fill_u32(status, 0u, n_clear, stream), "fill");
  // setup also counts every triangle's tiles and their candidate pixels
  STEP(timed("setup", stream, [&] { return launch_setup(ms, set, stream); }), "setup kernel");
  // one scan over the tile counts of all images (the images' lists follow
  // each other in one array), and over their candidate counts (the images'
  // staging regions follow each other in the staging buffer)
  STEP(timed("scan_tiles", stream, [&] {
         return launch_tile_scan(reinterpret_cast<const uint64_t*>(ws + o_tpack),
                                 reinterpret_cast<const uint32_t*>(ws + o_tovf), tile_cnt_all, tile_region_all,
                                 n_all, stage_layers * (uint32_t)(tw * th),
                                 scan_scratch, status, stream);
       }), "tile scan");
  // Tile lists are sized from the largest entries-per-triangle ratio seen so
  // far; the scatter drops entries beyond the capacity and the call is redone
  // with the exact size when that happens (the entry total is read back below).
  // (capped per triangle: a mesh of few large triangles is covered by the
  // per-tile term, and anything beyond is caught by the retry)
  uint64_t cap = (uint64_t)std::ceil((double)n_tris * nimg * std::min(g_list_ratio.load(), 8.0)) +
                 4 * (uint64_t)n_all + 1024;
  auto alloc_lists = [&](uint64_t c) -> hipError_t {
    cache_put(p->lists, p->lists_bytes, stream);
    p->lists = nullptr;
    hipError_t ea = cache_get(&p->lists, sizeof(int2) * (size_t)c, stream, &p->lists_bytes);
    if (ea != hipSuccess) {
      p->lists = nullptr;
      return ea;
    }
    for (int k = 0; k < nimg; ++k) {
      set.img[k].tile_list = static_cast<int2*>(p->lists);
      set.img[k].list_cap = c;
    }
    return hipSuccess;
  };
  STEP(alloc_lists(cap), "tile list allocation");
  const uint32_t* gather_src[kMaxGather];
  int n_gather = 0;
  gather_src[n_gather++] = status;      // rb[0]: status, rb[1..3]: max layers
  gather_src[n_gather++] = status + 1;
  gather_src[n_gather++] = status + 2;
  gather_src[n_gather++] = status + 3;
  for (int k = 0; k < nimg; ++k) gather_src[n_gather++] = set.img[k].offsets + npix;  // rb[4+k]
  const int rb_more = n_gather;
  gather_src[n_gather++] = tile_cnt_all + n_all;     // list entries
  gather_src[n_gather++] = tile_region_all + n_all;  // staging demand (saturated)
  gather_src[n_gather++] = status + 18;              // tiles to walk again
  gather_src[n_gather++] = set.plan + 2 * n_all;     // place items
  const uint32_t* counts_k[kMaxImages];
  uint32_t* offsets_k[kMaxImages];
  uint32_t* max_k[kMaxImages];  // largest count of each image
  for (int k = 0; k < nimg; ++k) {
    counts_k[k] = set.img[k].counts;
    offsets_k[k] = set.img[k].offsets;
    max_k[k] = status + 1 + k;
  }
  for (int attempt = 0; attempt < 2; ++attempt) {
    STEP(timed("bin_scatter", stream, [&] { return launch_bin_scatter(ms, set, stream); }), "bin scatter kernel");
    STEP(timed("sample", stream, [&] { return launch_sample(set, stream); }), "sampling kernel");
    STEP(timed("scan_pixels", stream, [&] {
           return launch_scan_segments(counts_k, offsets_k, nimg, npix, scan_scratch, status, stream, max_k);
         }), "pixel scan");
    STEP(timed("plan_items", stream, [&] {
           return launch_plan_items(set, p->items, scan_scratch, status, stream);
         }), "place plan");
    // the single readback: status, max layers, sample and entry totals
    STEP(launch_gather(gather_src, n_gather, rb, stream), "readback");
    STEP(hipStreamSynchronize(stream), "synchronise");
    if (rb[0] & kStatusBadIndex) return bail(fail(LDNI_ERR_INDEX, "triangle index outside [0, n_verts)"));
    if (rb[0] & kStatusNonFinite) return bail(fail(LDNI_ERR_NONFINITE, "non-finite vertex coordinate"));
    if (rb[0] & kStatusMismatch) return bail(fail(LDNI_ERR_DEVICE, "tile lists disagree with their counts"));
    const uint64_t need = rb[rb_more];
    {
      const uint64_t demand = rb[rb_more + 1];
      uint32_t ml = 0;
      for (int k = 0; k < nimg; ++k) ml = std::max(ml, rb[1 + k]);
      stage_seen_record(stage_key, StageSeen{demand, ml});
      p->n_walk = rb[rb_more + 2];
      p->n_items = rb[rb_more + 3];
    }
    if (n_tris > 0) {
      const double ratio = std::min(8.0, (double)need / ((double)n_tris * nimg) * 1.1);
      double cur = g_list_ratio.load();
      while (ratio > cur && !g_list_ratio.compare_exchange_weak(cur, ratio)) {
      }
    }
    if (need <= cap) break;
    if (attempt == 1) return bail(fail(LDNI_ERR_DEVICE, "tile list sizing failed"));
    cap = need;
    STEP(alloc_lists(cap), "tile list allocation");
    // cursors, max layers and walk count start again
    STEP(launch_fill_u32(tile_cur_all, 0u, n_all, stream), "fill");
    STEP(launch_fill_u32(status + 1, 0u, 3, stream), "fill");
    STEP(launch_fill_u32(walk_count, 0u, 1, stream), "fill");
  }
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

}  // extern "C"

namespace {

// Second half of a call: the place pass into the caller's buffers (float
// normals, or 8-bit codes when rgb8 is given), then the plan is released.
// With owner, the result checks the place pass's status when it is first
// read; without, the call waits for it here.
ldni_status finish_plan(ldni_plan* p, float* const depth[3], float* const normal[3],
                        uint32_t* const rgb8[3], int32_t* const tri[3], ldni_result* owner) {
  if (!p) return fail(LDNI_ERR_INVALID_ARG, "NULL plan");
  if (!depth || !(normal || rgb8) || !tri) {
    release_plan(p);
    return fail(LDNI_ERR_INVALID_ARG, "NULL output array");
  }
  for (int k = 0; k < p->set.n; ++k) {
    const int a = p->axis_of[k];
    const bool have_normal = rgb8 ? rgb8[a] != nullptr : normal[a] != nullptr;
    if (p->n[a] > 0 && (!depth[a] || !have_normal || !tri[a])) {
      release_plan(p);
      return fail(LDNI_ERR_INVALID_ARG, "NULL output buffer for an axis with samples");
    }
    p->set.img[k].depth = depth[a];
    p->set.img[k].normal = rgb8 ? nullptr : normal[a];
    p->set.img[k].normal_rgb8 = rgb8 ? rgb8[a] : nullptr;
    p->set.img[k].tri = tri[a];
  }
  hipError_t e = hipSuccess;
  if (p->n_tris > 0)
    e = timed("place", p->stream, [&] {
      return launch_place(p->set, p->items, p->n_items, p->write_counter, p->n_walk, p->stream);
    });
  ldni_status st = LDNI_OK;
  if (e != hipSuccess) st = hip_fail(e, "write kernel");
  else if (owner) st = arm_status(owner, p->status, p->stream);
  else st = check_now(p->status, p->stream);
  release_plan(p);
  return st;
}

}  // namespace

extern "C" {

ldni_status ldni_sample_finish(ldni_plan* p, float* const depth[3], float* const normal[3],
                               int32_t* const tri[3]) {
  if (!normal) {
    release_plan(p);
    return fail(LDNI_ERR_INVALID_ARG, "NULL output array");
  }
  return finish_plan(p, depth, normal, nullptr, tri, nullptr);
}

ldni_status ldni_sample_finish_rgb8(ldni_plan* p, float* const depth[3], uint32_t* const normal_rgb8[3],
                                    int32_t* const tri[3]) {
  if (!normal_rgb8) {
    release_plan(p);
    return fail(LDNI_ERR_INVALID_ARG, "NULL output array");
  }
  return finish_plan(p, depth, nullptr, normal_rgb8, tri, nullptr);
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
  const bool rgb8 = (axis_mask & LDNI_NORMAL_RGB8) != 0;
  axis_mask &= ~(uint32_t)LDNI_NORMAL_RGB8;
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
  hipError_t e = cache_get(&r->offsets_buf, 3 * per_axis, stream, &r->offsets_bytes);
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
    o_normal[a] = bytes; bytes = align_up(bytes + (rgb8 ? sizeof(uint32_t) : 3 * sizeof(float)) * n[a]);
    o_tri[a] = bytes; bytes = align_up(bytes + sizeof(int32_t) * n[a]);
  }
  e = cache_get(&r->samples_buf, bytes, stream, &r->samples_bytes);
  if (e != hipSuccess) {
    r->samples_buf = nullptr;
    ldni_plan_free(plan);
    ldni_free(r);
    return hip_fail(e, "sample allocation");
  }
  char* sb = static_cast<char*>(r->samples_buf);
  float* dp[3];
  float* np_[3];
  uint32_t* cp[3];
  int32_t* tp[3];
  uint32_t ml[3];
  ldni_plan_max_layers(plan, ml);
  for (int a = 0; a < 3; ++a) {
    dp[a] = reinterpret_cast<float*>(sb + o_depth[a]);
    np_[a] = rgb8 ? nullptr : reinterpret_cast<float*>(sb + o_normal[a]);
    cp[a] = rgb8 ? reinterpret_cast<uint32_t*>(sb + o_normal[a]) : nullptr;
    tp[a] = reinterpret_cast<int32_t*>(sb + o_tri[a]);
    if ((axis_mask >> a) & 1u) {
      ldni_axis_view& v = r->view[a];
      v.w = w;
      v.max_layers = ml[a];
      v.n_samples = n[a];
      v.offsets = offs[a];
      v.depth = dp[a];
      v.normal = np_[a];
      v.normal_rgb8 = cp[a];
      v.tri = tp[a];
    }
  }
  st = rgb8 ? finish_plan(plan, dp, nullptr, cp, tp, r) : finish_plan(plan, dp, np_, nullptr, tp, r);
  if (st != LDNI_OK) {
    ldni_free(r);
    return st;
  }
  *out = r;
  return LDNI_OK;
}

}  // extern "C"

namespace {

// Checks the arguments of a backward call and fills args (every field but
// the workspace).  *n_img = 0: nothing to do.
ldni_status backward_args(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                          const float bbox[6], int32_t w, uint32_t axis_mask, const ldni_axis_view views[3],
                          const float* const grad_depth[3], const float* const grad_normal[3],
                          float* grad_verts, BackwardArgs& args, int* n_img) {
  *n_img = 0;
  ldni_status st = validate(verts, n_verts, tris, n_tris, bbox, w, axis_mask);
  if (st != LDNI_OK) return st;
  if (!views) return fail(LDNI_ERR_INVALID_ARG, "views is NULL");
  if (n_verts > 0 && !grad_verts) return fail(LDNI_ERR_INVALID_ARG, "grad_verts is NULL");
  for (int a = 0; a < 3; ++a) {
    if (!((axis_mask >> a) & 1u)) continue;
    const ldni_axis_view& v = views[a];
    if (v.w != w) return fail(LDNI_ERR_INVALID_ARG, "view resolution differs from w");
    if (!v.offsets || (v.n_samples > 0 && !v.tri))
      return fail(LDNI_ERR_INVALID_ARG, "view of a requested axis lacks offsets or triangle ids");
  }
  if (n_tris == 0) return LDNI_OK;
  args = BackwardArgs{};
  args.w = w;
  for (int d = 0; d < 6; ++d) args.bbox[d] = (double)bbox[d];
  args.verts = verts;
  args.n_verts = n_verts;
  args.tris = tris;
  args.n_tris = n_tris;
  args.grad = grad_verts;
  int nimg = 0;
  for (int a = 0; a < 3; ++a)
    if ((axis_mask >> a) & 1u) {
      const float* gd = grad_depth ? grad_depth[a] : nullptr;
      const float* gn = grad_normal ? grad_normal[a] : nullptr;
      if (views[a].n_samples == 0 || (!gd && !gn)) continue;
      BackwardAxis& ax = args.axis[nimg++];
      ax.a = a;
      ax.offsets = views[a].offsets;
      ax.tri = views[a].tri;
      ax.gd = gd;
      ax.gn = gn;
    }
  args.n = nimg;
  *n_img = nimg;
  return LDNI_OK;
}

// The no-allocation backward's scratch: per triangle 6 floats for each image
// (18 floats), for up to kNoAllocTris triangles.
// Each device holds its own copy from the library's load to the process
// end; host code uses only the address hipGetSymbolAddress gives per device.
constexpr int64_t kNoAllocTris = 262144;
__device__ __align__(256) float scratch[18 * kNoAllocTris];
std::mutex g_scratch_mu;
float* g_scratch_ptr[64] = {};

// The scratch array's device address on the current device (looked up once
// per device, with that device current).
ldni_status scratch_address(float** out) {
  int device = 0;
  HIP_TRY(hipGetDevice(&device), "hipGetDevice");
  if (device < 0 || device >= 64) return fail(LDNI_ERR_DEVICE, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
    if (!p) return fail(LDNI_ERR_DEVICE, "scratch address");
    g_scratch_ptr[device] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[device];
  return LDNI_OK;
}

}  // namespace

extern "C" {

ldni_status ldni_backward(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                          const float bbox[6], int32_t w, uint32_t axis_mask,
                          const ldni_axis_view views[3], const float* const grad_depth[3],
                          const float* const grad_normal[3], float* grad_verts, void* hip_stream) {
  BackwardArgs args{};
  int nimg = 0;
  ldni_status st = backward_args(verts, n_verts, tris, n_tris, bbox, w, axis_mask, views, grad_depth,
                                 grad_normal, grad_verts, args, &nimg);
  if (st != LDNI_OK || nimg == 0) return st;
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  int device = 0;
  HIP_TRY(hipGetDevice(&device), "hipGetDevice");
  prepare_pool(device);
  void* ws = nullptr;
  size_t ws_bytes = 0;
  const size_t per = align_up(sizeof(float) * 6 * (size_t)n_tris);
  hipError_t e = cache_get(&ws, per * nimg, stream, &ws_bytes);
  if (e != hipSuccess) return hip_fail(e, "backward workspace");
  char* base = static_cast<char*>(ws);
  for (int k = 0; k < nimg; ++k) args.axis[k].acc = reinterpret_cast<float*>(base + k * per);
  e = launch_fill_u32(reinterpret_cast<uint32_t*>(ws), 0u, (int64_t)(per * nimg / 4), stream);
  if (e == hipSuccess) e = timed("backward", stream, [&] { return launch_backward(args, stream); });
  cache_put(ws, ws_bytes, stream);
  if (e != hipSuccess) return hip_fail(e, "backward kernels");
  return LDNI_OK;
}

ldni_status ldni_backward_noalloc(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                                  const float bbox[6], int32_t w, uint32_t axis_mask,
                                  const ldni_axis_view views[3], const float* const grad_depth[3],
                                  const float* const grad_normal[3], float* grad_verts, void* hip_stream) {
  if (n_tris > kNoAllocTris)
    return fail(LDNI_ERR_INVALID_ARG, "n_tris beyond the 262144 triangles of the no-allocation scratch");
  BackwardArgs args{};
  int nimg = 0;
  ldni_status st = backward_args(verts, n_verts, tris, n_tris, bbox, w, axis_mask, views, grad_depth,
                                 grad_normal, grad_verts, args, &nimg);
  if (st != LDNI_OK || nimg == 0) return st;
  float* ws = nullptr;
  st = scratch_address(&ws);
  if (st != LDNI_OK) return st;
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  // the same layout as ldni_backward's workspace, without the 256-byte
  // rounding: the sums of image k at k * 6T
  const int64_t per = 6 * n_tris;
  for (int k = 0; k < nimg; ++k) args.axis[k].acc = ws + k * per;
  // the last call's sums are still there: cleared by a fill kernel
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ws), 0u, per * nimg, stream);
  if (e == hipSuccess) e = launch_backward(args, stream);
  if (e != hipSuccess) return hip_fail(e, "backward kernels");
  return LDNI_OK;
}

ldni_status ldni_result_axis(const ldni_result* r, int axis, ldni_axis_view* view) {
  if (!r || !view || axis < 0 || axis > 2) return fail(LDNI_ERR_INVALID_ARG, "bad result/axis/view");
  const ldni_status st = settle(const_cast<ldni_result*>(r));
  if (st != LDNI_OK) return st;
  *view = r->view[axis];
  return LDNI_OK;
}

ldni_status ldni_trim(void) {
  std::vector<CachedBuffer> all;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    all.swap(g_cache);
  }
  int cur = 0;
  const bool have_cur = hipGetDevice(&cur) == hipSuccess;
  bool ok = true;
  for (const CachedBuffer& c : all) {
    ok &= hipSetDevice(c.device) == hipSuccess;
    ok &= hipStreamSynchronize(c.stream) == hipSuccess;
    ok &= hipFree(c.ptr) == hipSuccess;
  }
  if (have_cur) (void)hipSetDevice(cur);
  return ok ? LDNI_OK : fail(LDNI_ERR_DEVICE, "releasing cached buffers");
}

ldni_status ldni_boolean(const ldni_axis_view* a, const ldni_axis_view* b, int32_t op, float eps,
                         int32_t axis, void* hip_stream, ldni_result** out) {
  if (out) *out = nullptr;
  if (!out || !a || !b) return fail(LDNI_ERR_INVALID_ARG, "NULL argument");
  if (op < LDNI_UNION || op > LDNI_DIFFERENCE)
    return fail(LDNI_ERR_INVALID_ARG, "op must be LDNI_UNION, LDNI_INTERSECTION or LDNI_DIFFERENCE");
  if (axis < 0 || axis > 2) return fail(LDNI_ERR_INVALID_ARG, "axis must be 0, 1 or 2");
  if (!(eps >= 0.0f) || !std::isfinite(eps)) return fail(LDNI_ERR_INVALID_ARG, "eps must be finite and >= 0");
  if (a->w < 1 || a->w > 16384 || a->w != b->w)
    return fail(LDNI_ERR_INVALID_ARG, "both views need the same w in [1, 16384]");
  for (const ldni_axis_view* v : {a, b}) {
    if (!v->offsets) return fail(LDNI_ERR_INVALID_ARG, "NULL offsets");
    if (v->n_samples > 0 && (!v->depth || !v->normal || !v->tri))
      return fail(LDNI_ERR_INVALID_ARG, "NULL sample array of a view with samples");
    if (v->n_samples > 0xffffffffull) return fail(LDNI_ERR_INVALID_ARG, "a view has 2^32 or more samples");
  }
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  int device = 0;
  HIP_TRY(hipGetDevice(&device), "hipGetDevice");
  prepare_pool(device);
  uint32_t* rb = pinned_readback();
  if (!rb) return fail(LDNI_ERR_OUT_OF_MEMORY, "pinned readback buffer");
  const int32_t w = a->w;
  const int64_t npix = (int64_t)w * w;

  ldni_result* r = new (std::nothrow) ldni_result();
  if (!r) return fail(LDNI_ERR_OUT_OF_MEMORY, "result");
  std::memset(r->view, 0, sizeof(r->view));
  r->stream = stream;
  hipError_t e = cache_get(&r->offsets_buf, sizeof(uint32_t) * (size_t)(npix + 1), stream, &r->offsets_bytes);
  if (e != hipSuccess) {
    r->offsets_buf = nullptr;
    ldni_free(r);
    return hip_fail(e, "offsets allocation");
  }
  // workspace: status words ([0] status, [1] max layers), scan partials, the
  // kept samples' sources (one word per input sample)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  const size_t o_refs = align_up(256 + scan_scratch_bytes(npix, 1));
  e = cache_get(&ws, o_refs + sizeof(uint32_t) * (size_t)(a->n_samples + b->n_samples), stream, &ws_bytes);
  if (e != hipSuccess) {
    ldni_free(r);
    return hip_fail(e, "workspace allocation");
  }
  auto bail = [&](ldni_status st) {
    cache_put(ws, ws_bytes, stream);
    ldni_free(r);
    return st;
  };
  uint32_t* status = static_cast<uint32_t*>(ws);
  uint32_t* counts = static_cast<uint32_t*>(r->offsets_buf);
  BooleanArgs g{};
  g.a = AxisArrays{a->n_samples, static_cast<const uint32_t*>(a->offsets), static_cast<const float*>(a->depth),
                   static_cast<const float*>(a->normal), static_cast<const int32_t*>(a->tri)};
  g.b = AxisArrays{b->n_samples, static_cast<const uint32_t*>(b->offsets), static_cast<const float*>(b->depth),
                   static_cast<const float*>(b->normal), static_cast<const int32_t*>(b->tri)};
  g.npix = npix;
  g.op = op;
  g.eps = (double)eps;
  g.counts = counts;
  g.refs = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + o_refs);
  g.status = status;
#define BSTEP(expr, what)                                  \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return bail(hip_fail(e_, what)); \
  } while (0)
  BSTEP(launch_fill_u32(status, 0u, 64, stream), "fill");
  BSTEP(timed("boolean_count", stream, [&] { return launch_boolean(g, false, stream); }), "Boolean count kernel");
  BSTEP(timed("boolean_scan", stream, [&] {
          return launch_scan(counts, counts, npix, static_cast<char*>(ws) + 256, status, stream, status + 1);
        }), "Boolean scan");
  const uint32_t* src[3] = {status, status + 1, counts + npix};
  BSTEP(launch_gather(src, 3, rb, stream), "readback");
  BSTEP(hipStreamSynchronize(stream), "synchronise");
  if (rb[0] & kStatusMismatch) return bail(fail(LDNI_ERR_INVALID_ARG, "the offsets of an input view are not a prefix of its samples"));
  if (rb[0] & kStatusOverflow) return bail(fail(LDNI_ERR_OVERFLOW, "2^32 or more result samples"));
  const uint64_t n = rb[2];
  size_t o_normal = align_up(sizeof(float) * n), o_tri = align_up(o_normal + sizeof(float) * 3 * n);
  e = cache_get(&r->samples_buf, o_tri + sizeof(int32_t) * n, stream, &r->samples_bytes);
  if (e != hipSuccess) {
    r->samples_buf = nullptr;
    return bail(hip_fail(e, "sample allocation"));
  }
  char* sb = static_cast<char*>(r->samples_buf);
  g.out_depth = reinterpret_cast<float*>(sb);
  g.out_normal = reinterpret_cast<float*>(sb + o_normal);
  g.out_tri = reinterpret_cast<int32_t*>(sb + o_tri);
  BSTEP(timed("boolean_write", stream, [&] { return launch_boolean(g, true, stream); }), "Boolean write kernel");
  {
    const ldni_status st = arm_status(r, status, stream);
    if (st != LDNI_OK) return bail(st);
  }
#undef BSTEP
  cache_put(ws, ws_bytes, stream);
  ldni_axis_view& v = r->view[axis];
  v.w = w;
  v.max_layers = rb[1];
  v.n_samples = n;
  v.offsets = counts;
  v.depth = g.out_depth;
  v.normal = g.out_normal;
  v.tri = g.out_tri;
  *out = r;
  return LDNI_OK;
}

ldni_status ldni_node_words(int32_t w, uint64_t* n_words) {
  if (!n_words) return fail(LDNI_ERR_INVALID_ARG, "NULL n_words");
  *n_words = 0;
  if (w < 1 || w > 8192) return fail(LDNI_ERR_INVALID_ARG, "w must be in [1, 8192]");
  const uint64_t nb = (uint64_t)(w + 31) / 32;
  *n_words = nb * nb * nb * 1024;
  return LDNI_OK;
}

ldni_status ldni_classify_nodes(const ldni_axis_view views[3], const float bbox[6], uint32_t* bits,
                                uint64_t n_words, uint64_t stats[2], void* hip_stream) {
  if (!views || !bbox || !bits) return fail(LDNI_ERR_INVALID_ARG, "NULL argument");
  const int32_t w = views[0].w;
  if (w < 1 || w > 8192 || views[1].w != w || views[2].w != w)
    return fail(LDNI_ERR_INVALID_ARG, "the three views need the same w in [1, 8192]");
  for (int d = 0; d < 3; ++d) {
    if (!std::isfinite(bbox[d]) || !std::isfinite(bbox[3 + d]))
      return fail(LDNI_ERR_INVALID_ARG, "bbox must be finite");
    if (!(bbox[d] < bbox[3 + d])) return fail(LDNI_ERR_INVALID_ARG, "bbox needs lo < hi on every axis");
    const ldni_axis_view& v = views[d];
    if (!v.offsets) return fail(LDNI_ERR_INVALID_ARG, "NULL offsets");
    if (v.n_samples > 0 && !v.depth) return fail(LDNI_ERR_INVALID_ARG, "NULL depth of a view with samples");
    if (v.n_samples > 0xffffffffull) return fail(LDNI_ERR_INVALID_ARG, "a view has 2^32 or more samples");
  }
  uint64_t need = 0;
  (void)ldni_node_words(w, &need);
  if (n_words < need) return fail(LDNI_ERR_INVALID_ARG, "bits holds fewer words than ldni_node_words(w)");
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  int device = 0;
  HIP_TRY(hipGetDevice(&device), "hipGetDevice");
  prepare_pool(device);
  uint32_t* rb = pinned_readback();
  if (!rb) return fail(LDNI_ERR_OUT_OF_MEMORY, "pinned readback buffer");
  // workspace: [0] status word, [64..80) the two totals, [256..) per-workgroup
  // sums, then the span codes of the three axes
  const uint32_t n_wg = node_workgroups(w);
  const int32_t n_spans = (w + 63) / 64;
  const size_t o_codes = align_up(256 + 16 * (size_t)n_wg);
  void* ws = nullptr;
  size_t ws_bytes = 0;
  hipError_t e = cache_get(&ws, o_codes + node_code_bytes(w), stream, &ws_bytes);
  if (e != hipSuccess) return hip_fail(e, "workspace allocation");
  char* wb = static_cast<char*>(ws);
  NodeArgs g{};
  for (int d = 0; d < 3; ++d) {
    const ldni_axis_view& v = views[d];
    g.axis[d] = AxisArrays{v.n_samples, v.offsets, v.depth, nullptr, nullptr};
    g.lo[d] = (double)bbox[d];
    g.h[d] = ((double)bbox[3 + d] - (double)bbox[d]) / (double)w;
  }
  g.w = w;
  g.nb = (w + 31) / 32;
  g.bits = bits;
  g.status = reinterpret_cast<uint32_t*>(wb);
  g.stats = reinterpret_cast<uint64_t*>(wb + 64);
  g.partial = reinterpret_cast<uint64_t*>(wb + 256);
  g.codes = reinterpret_cast<uint16_t*>(wb + o_codes);
  g.n_spans = n_spans;
  auto run = [&]() -> ldni_status {
#define NSTEP(expr, what)                       \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)
    NSTEP(launch_fill_u32(g.status, 0u, 1, stream), "fill");
    NSTEP(timed("node_codes", stream, [&] { return launch_node_codes(g, stream); }), "span code kernel");
    NSTEP(timed("classify_nodes", stream, [&] { return launch_classify_nodes(g, stream); }), "classify kernel");
    NSTEP(launch_node_stats(g, stream), "node totals");
    const uint32_t* words = reinterpret_cast<const uint32_t*>(g.stats);
    const uint32_t* src[5] = {g.status, words, words + 1, words + 2, words + 3};
    NSTEP(launch_gather(src, 5, rb, stream), "readback");
    NSTEP(hipStreamSynchronize(stream), "synchronise");
#undef NSTEP
    if (rb[0] & kStatusMismatch)
      return fail(LDNI_ERR_INVALID_ARG, "the offsets of an input view are not a prefix of its samples");
    if (stats) {
      stats[0] = (uint64_t)rb[1] | ((uint64_t)rb[2] << 32);
      stats[1] = (uint64_t)rb[3] | ((uint64_t)rb[4] << 32);
    }
    return LDNI_OK;
  };
  const ldni_status st = run();
  cache_put(ws, ws_bytes, stream);
  return st;
}

ldni_status ldni_offset(const ldni_axis_view views[3], const float bbox[6], float r, float eps, void* hip_stream,
                        ldni_result** out) {
  if (out) *out = nullptr;
  if (!out || !views || !bbox) return fail(LDNI_ERR_INVALID_ARG, "NULL argument");
  if (!std::isfinite(r) || r == 0.0f) return fail(LDNI_ERR_INVALID_ARG, "r must be finite and not zero");
  if (!(eps >= 0.0f) || !std::isfinite(eps)) return fail(LDNI_ERR_INVALID_ARG, "eps must be finite and >= 0");
  const int32_t w = views[0].w;
  if (w < 1 || w > 16384 || views[1].w != w || views[2].w != w)
    return fail(LDNI_ERR_INVALID_ARG, "the three views need the same w in [1, 16384]");
  uint64_t n_total = 0;
  for (int d = 0; d < 3; ++d) {
    if (!std::isfinite(bbox[d]) || !std::isfinite(bbox[3 + d]))
      return fail(LDNI_ERR_INVALID_ARG, "bbox must be finite");
    if (!(bbox[d] < bbox[3 + d])) return fail(LDNI_ERR_INVALID_ARG, "bbox needs lo < hi on every axis");
    const ldni_axis_view& v = views[d];
    if (!v.offsets) return fail(LDNI_ERR_INVALID_ARG, "NULL offsets");
    if (v.n_samples > 0 && (!v.depth || !v.normal || !v.tri))
      return fail(LDNI_ERR_INVALID_ARG, "NULL sample array of a view with samples");
    if (v.n_samples > 0xffffffffull) return fail(LDNI_ERR_INVALID_ARG, "a view has 2^32 or more samples");
    n_total += v.n_samples;
  }
  if (n_total >= kMaxSpheres) return fail(LDNI_ERR_INVALID_ARG, "2^30 or more samples in the three views");
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  int device = 0;
  HIP_TRY(hipGetDevice(&device), "hipGetDevice");
  prepare_pool(device);
  uint32_t* rb = pinned_readback();
  if (!rb) return fail(LDNI_ERR_OUT_OF_MEMORY, "pinned readback buffer");
  const int64_t npix = (int64_t)w * w;
  const int64_t n_rays = 3 * npix;

  ldni_result* res = new (std::nothrow) ldni_result();
  if (!res) return fail(LDNI_ERR_OUT_OF_MEMORY, "result");
  std::memset(res->view, 0, sizeof(res->view));
  res->stream = stream;
  hipError_t e = cache_get(&res->offsets_buf, 3 * sizeof(uint32_t) * (size_t)(npix + 1), stream, &res->offsets_bytes);
  if (e != hipSuccess) {
    res->offsets_buf = nullptr;
    ldni_free(res);
    return hip_fail(e, "offsets allocation");
  }
  // workspace: status, ray counts and cursors, ray starts, scan scratch, centres
  const size_t o_count = 256;
  const size_t o_cursor = align_up(o_count + sizeof(uint32_t) * (size_t)n_rays);
  const size_t o_start = align_up(o_cursor + sizeof(uint32_t) * (size_t)n_rays);
  const size_t o_scratch = align_up(o_start + sizeof(uint32_t) * (size_t)(n_rays + 1));
  const size_t scratch = std::max(scan_scratch_bytes(n_rays, 1), scan_scratch_bytes(npix, 3));
  const size_t o_deep = align_up(o_scratch + scratch);
  const size_t o_centres = align_up(o_deep + sizeof(uint32_t) * (size_t)n_rays);
  // the end points the count pass keeps for the write pass: as many per ray
  // (64, 32 or 16) as fit in 1 GiB, else none (the write pass recomputes)
  size_t saved_cap = (size_t)1 << 30;
  // test hook: a smaller budget for them (0: none kept)
  if (const char* env = std::getenv("LDNI_OFFSET_KEEP_BYTES")) saved_cap = std::strtoull(env, nullptr, 10);
  uint32_t n_saved = kOffsetSavedMax;
  while (n_saved >= 16 && sizeof(uint64_t) * n_saved * 3 * (size_t)npix > saved_cap) n_saved /= 2;
  const bool use_saved = n_saved >= 16;
  const size_t saved_bytes = use_saved ? sizeof(uint64_t) * n_saved * 3 * (size_t)npix : 0;
  const size_t o_saved = align_up(o_centres + 3 * sizeof(double) * (size_t)std::max<uint64_t>(n_total, 1));
  void* ws = nullptr;
  size_t ws_bytes = 0;
  e = cache_get(&ws, o_saved + (use_saved ? saved_bytes : 0), stream, &ws_bytes);
  if (e != hipSuccess) {
    ldni_free(res);
    return hip_fail(e, "workspace allocation");
  }
  void* list = nullptr;
  size_t list_bytes = 0;
  auto bail = [&](ldni_status st) {
    cache_put(list, list_bytes, stream);
    cache_put(ws, ws_bytes, stream);
    ldni_free(res);
    return st;
  };
  char* wb = static_cast<char*>(ws);
  OffsetArgs g{};
  uint64_t base = 0;
  for (int d = 0; d < 3; ++d) {
    const ldni_axis_view& v = views[d];
    g.in[d] = AxisArrays{v.n_samples, v.offsets, v.depth, v.normal, v.tri};
    g.lo[d] = (double)bbox[d];
    g.h[d] = ((double)bbox[3 + d] - (double)bbox[d]) / (double)w;
    // a centre f32(lo + (i + 0.5) h) is within 2^-24 (|lo| + (w + 1) h) of
    // the real value, and the index estimate carries a float64 error of a
    // few 2^-53 (w + 1); twice their sum in pixels, plus a millionth
    g.margin[d] = 2.0 * (std::ldexp(std::fabs(g.lo[d]) + ((double)w + 1.0) * g.h[d], -24) / g.h[d] +
                         std::ldexp((double)w + 1.0, -48)) + 1e-6;
    g.base[d] = base;
    base += v.n_samples;
    g.counts[d] = static_cast<uint32_t*>(res->offsets_buf) + d * (npix + 1);
    g.out_offsets[d] = g.counts[d];
  }
  g.w = w;
  g.n_spheres = (uint32_t)n_total;
  g.r = std::fabs((double)r);
  g.eps = (double)eps;
  g.union_op = r > 0.0f ? 1 : 0;
  g.status = reinterpret_cast<uint32_t*>(wb);
  g.ray_count = reinterpret_cast<uint32_t*>(wb + o_count);
  g.ray_cursor = reinterpret_cast<uint32_t*>(wb + o_cursor);
  g.ray_start = reinterpret_cast<uint32_t*>(wb + o_start);
  g.centres = reinterpret_cast<double*>(wb + o_centres);
  g.saved = use_saved ? reinterpret_cast<uint64_t*>(wb + o_saved) : nullptr;
  g.n_saved = use_saved ? n_saved : 0u;
  g.deep = reinterpret_cast<uint32_t*>(wb + o_deep);
  g.n_deep = 0;
  void* scr = wb + o_scratch;
#define OSTEP(expr, what)                                  \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return bail(hip_fail(e_, what)); \
  } while (0)
  OSTEP(launch_fill_u32(g.status, 0u, 64, stream), "fill");
  OSTEP(launch_fill_u32(g.ray_count, 0u, 2 * n_rays + 64, stream), "fill");  // counts and cursors
  OSTEP(timed("offset_centres", stream, [&] { return launch_offset_centres(g, stream); }), "centre kernel");
  OSTEP(timed("offset_bin", stream, [&] { return launch_offset_bin(g, false, stream); }), "binning kernel");
  OSTEP(launch_scan(g.ray_count, g.ray_start, n_rays, scr, g.status, stream), "ray list scan");
  OSTEP(launch_offset_deep(g, stream), "deep ray list");
  {
    const uint32_t* src[3] = {g.status, g.ray_start + n_rays, g.status + 16};
    OSTEP(launch_gather(src, 3, rb, stream), "readback");
    OSTEP(hipStreamSynchronize(stream), "synchronise");
  }
  g.n_deep = std::min<uint32_t>(rb[2], (uint32_t)n_rays);
  if (rb[0] & kStatusMismatch)
    return bail(fail(LDNI_ERR_INVALID_ARG, "the offsets of an input view are not a prefix of its samples"));
  if (rb[0] & kStatusOverflow) return bail(fail(LDNI_ERR_OVERFLOW, "2^32 or more sphere hits on the rays"));
  e = cache_get(&list, sizeof(uint32_t) * (size_t)std::max<uint32_t>(rb[1], 1), stream, &list_bytes);
  if (e != hipSuccess) {
    list = nullptr;
    return bail(hip_fail(e, "ray list allocation"));
  }
  g.list = static_cast<uint32_t*>(list);
  OSTEP(timed("offset_bin", stream, [&] { return launch_offset_bin(g, true, stream); }), "binning kernel");
  OSTEP(timed("offset_count", stream, [&] { return launch_offset_rays(g, false, stream); }), "offset count kernel");
  uint32_t* max_slot = g.status + 8;  // [8..10]: largest count per axis
  uint32_t* maxes[3] = {max_slot, max_slot + 1, max_slot + 2};
  OSTEP(launch_scan_segments(g.counts, g.counts, 3, npix, scr, g.status, stream, maxes), "offset scan");
  {
    const uint32_t* src[7] = {g.status, g.counts[0] + npix, g.counts[1] + npix, g.counts[2] + npix,
                              maxes[0], maxes[1], maxes[2]};
    OSTEP(launch_gather(src, 7, rb, stream), "readback");
    OSTEP(hipStreamSynchronize(stream), "synchronise");
  }
  if (rb[0] & kStatusMismatch)
    return bail(fail(LDNI_ERR_INVALID_ARG, "the offsets of an input view are not a prefix of its samples"));
  if (rb[0] & kStatusOverflow) return bail(fail(LDNI_ERR_OVERFLOW, "2^32 or more result samples on one axis"));
  const uint64_t n_out[3] = {rb[1], rb[2], rb[3]};
  const uint32_t max_layers[3] = {rb[4], rb[5], rb[6]};
  size_t o_ax[3][3], total = 0;
  for (int d = 0; d < 3; ++d) {
    o_ax[d][0] = total;
    o_ax[d][1] = align_up(o_ax[d][0] + sizeof(float) * n_out[d]);
    o_ax[d][2] = align_up(o_ax[d][1] + 3 * sizeof(float) * n_out[d]);
    total = align_up(o_ax[d][2] + sizeof(int32_t) * n_out[d]);
  }
  e = cache_get(&res->samples_buf, std::max<size_t>(total, 256), stream, &res->samples_bytes);
  if (e != hipSuccess) {
    res->samples_buf = nullptr;
    return bail(hip_fail(e, "sample allocation"));
  }
  char* sb = static_cast<char*>(res->samples_buf);
  for (int d = 0; d < 3; ++d) {
    g.out_depth[d] = reinterpret_cast<float*>(sb + o_ax[d][0]);
    g.out_normal[d] = reinterpret_cast<float*>(sb + o_ax[d][1]);
    g.out_tri[d] = reinterpret_cast<int32_t*>(sb + o_ax[d][2]);
  }
  OSTEP(timed("offset_write", stream, [&] { return launch_offset_rays(g, true, stream); }), "offset write kernel");
  {
    const ldni_status st = arm_status(res, g.status, stream);
    if (st != LDNI_OK) return bail(st);
  }
#undef OSTEP
  cache_put(list, list_bytes, stream);
  cache_put(ws, ws_bytes, stream);
  for (int d = 0; d < 3; ++d) {
    ldni_axis_view& v = res->view[d];
    v.w = w;
    v.max_layers = max_layers[d];
    v.n_samples = n_out[d];
    v.offsets = g.counts[d];
    v.depth = g.out_depth[d];
    v.normal = g.out_normal[d];
    v.tri = g.out_tri[d];
  }
  *out = res;
  return LDNI_OK;
}

void ldni_free(ldni_result* r) {
  if (!r) return;
  if (r->pending) {  // the slot is reused only once its copy has landed
    (void)hipEventSynchronize(r->slot.done);
    slot_put(r->slot);
    r->pending = false;
  }
  cache_put(r->samples_buf, r->samples_bytes, r->stream);
  cache_put(r->offsets_buf, r->offsets_bytes, r->stream);
  delete r;
}

}  // extern "C"

// ===========================================================================
// batched sampling
// ===========================================================================
struct ldni_batch {
  int32_t n_meshes = 0;
  uint32_t mask = 0;
  int32_t n_img = 0;
  std::vector<ldni_mesh_desc> desc;
  std::vector<int32_t> img_mesh, img_axis;
  std::vector<uint32_t> tri_block_start, tile_start;
  std::vector<uint64_t> seg_start;
  hipStream_t cs = nullptr;  // private stream the graph is captured on
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* lists = nullptr;
  uint64_t list_cap = 0;
  void* samples = nullptr;
  uint64_t sample_cap = 0;
  void* stage = nullptr;  // hits staged by the sampling pass
  uint64_t stage_cap = 0;
  uint32_t stage_layers = 64;  // staging entries per tile pixel (grows with the deepest pixel)
  void* items = nullptr;  // place items, sized for stage_layers
  uint64_t items_cap = 0;
  bool rgb8 = false;      // 8-bit normal codes instead of float normals
  bool small = true;      // every image's tiles have at most 256 pixels
  uint64_t small_tiles = 0;  // tiles of the images with small tiles (numbered first)
  uint32_t* host_out = nullptr;
  BatchDevice dev{};
  uint32_t* offsets_arena = nullptr;
  uint32_t* counts_arena = nullptr;
  uint32_t* tile_arena = nullptr;
  uint32_t* region_arena = nullptr;  // candidate counts -> staging regions (after tile_arena)
  uint32_t* cur_arena = nullptr;     // scatter cursors of the entries counted apart
  uint32_t* ovf_arena = nullptr;     // entries counted apart (outside the chunk tables)
  uint64_t* pack_arena = nullptr;    // chunk reservations and candidates, packed
  uint32_t* max_layers = nullptr;
  void* scan_scratch = nullptr;
  uint64_t total_tiles = 0, total_slots = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<Image> images_h;
  std::vector<BatchMesh> meshes_h;
  // results of the last run
  std::vector<uint32_t> n, ml;
  std::vector<uint64_t> base;
};

namespace {

void batch_release_graph(ldni_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

void batch_destroy(ldni_batch* b) {
  if (!b) return;
  batch_release_graph(b);
  if (b->cs) (void)hipStreamSynchronize(b->cs);
  if (b->samples) (void)hipFree(b->samples);
  if (b->stage) (void)hipFree(b->stage);
  if (b->items) (void)hipFree(b->items);
  if (b->lists) (void)hipFree(b->lists);
  if (b->ws) (void)hipFree(b->ws);
  if (b->host_out) (void)hipHostFree(b->host_out);
  if (b->cs) (void)hipStreamDestroy(b->cs);
  delete b;
}

// Points the image table at the current list and sample buffers and uploads it.
hipError_t batch_upload(ldni_batch* b) {
  for (int k = 0; k < b->n_img; ++k) {
    b->images_h[k].tile_list = static_cast<int2*>(b->lists);
    b->images_h[k].list_cap = b->list_cap;
  }
  b->dev.list_cap = b->list_cap;
  // sample arena: depth [cap], normals [cap][3] (or codes [cap]), tri [cap]
  const uint64_t nw = b->rgb8 ? 1 : 3;
  b->dev.depth = static_cast<float*>(b->samples);
  b->dev.normal = (b->samples && !b->rgb8) ? static_cast<float*>(b->samples) + b->sample_cap : nullptr;
  b->dev.normal_rgb8 =
      (b->samples && b->rgb8) ? reinterpret_cast<uint32_t*>(static_cast<float*>(b->samples) + b->sample_cap) : nullptr;
  b->dev.tri = b->samples ? reinterpret_cast<int32_t*>(static_cast<float*>(b->samples) + (1 + nw) * b->sample_cap)
                          : nullptr;
  b->dev.sample_cap = b->sample_cap;
  for (int k = 0; k < b->n_img; ++k) {
    Image& im = b->images_h[k];
    im.stage_key = b->stage ? static_cast<uint64_t*>(b->stage) : nullptr;
    im.stage_qs = b->stage ? reinterpret_cast<uint32_t*>(static_cast<uint64_t*>(b->stage) + b->stage_cap)
                           : nullptr;
    im.stage_cap = b->stage ? b->stage_cap : 0;
    im.stage_layers = b->stage_layers;
  }
  b->dev.items = b->items;
  hipError_t e = hipMemcpy(b->dev.images, b->images_h.data(), sizeof(Image) * b->n_img, hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  return hipMemcpy(b->dev.meshes, b->meshes_h.data(), sizeof(BatchMesh) * b->n_meshes, hipMemcpyHostToDevice);
}

// The whole batch, as launched on one stream (and captured).
hipError_t batch_enqueue(ldni_batch* b, hipStream_t s) {
  hipError_t e;
#define Q(x) do { e = (x); if (e != hipSuccess) return e; } while (0)
  Q(launch_fill_u32(b->dev.status, 0u, 20, s));  // status, work counters, walk count
  Q(launch_fill_u32(b->max_layers, 0u, b->n_img, s));
  // tile entry counts and (after them) candidate counts
  // scatter cursors, entries counted apart and packed tile counts (adjacent)
  Q(launch_fill_u32(b->cur_arena, 0u, 4 * (int64_t)b->total_tiles, s));
  Q(launch_batch_setup(b->dev, b->tri_block_start.back(), s));  // also counts tiles and candidates
  Q(launch_tile_scan(b->pack_arena, b->ovf_arena, b->tile_arena, b->region_arena, (int64_t)b->total_tiles,
                     b->stage_layers * (uint32_t)(b->small ? 256 : 1024), b->scan_scratch, b->dev.status, s));
  Q(launch_batch_scatter(b->dev, b->tri_block_start.back(), s));
  Q(launch_batch_sample(b->dev, (uint32_t)b->total_tiles, (uint32_t)b->small_tiles, s));
  Q(launch_batch_pixel_scan(b->dev, b->counts_arena, b->offsets_arena, (int64_t)b->total_slots,
                            b->scan_scratch, s));
  Q(launch_batch_finish_counts(b->dev, s));
  Q(launch_batch_place(b->dev, (uint32_t)b->total_tiles, (uint32_t)b->small_tiles, b->scan_scratch, s));
#undef Q
  return hipSuccess;
}

hipError_t batch_capture(ldni_batch* b) {
  batch_release_graph(b);
  hipError_t e = hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const hipError_t eq = batch_enqueue(b, b->cs);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cs, &g);
  if (eq != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return eq;
  }
  if (e != hipSuccess) return e;
  b->graph = g;
  return hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
}

ldni_status batch_grow(ldni_batch* b, void** buf, uint64_t* cap, uint64_t need, size_t bytes_per) {
  const uint64_t c = (need + need / 16 + 1024) & ~(uint64_t)3;  // whole 4-entry groups
  if (*buf) (void)hipFree(*buf);
  *buf = nullptr;
  hipError_t e = env_fault("alloc") ? hipErrorOutOfMemory : hipMalloc(buf, (size_t)c * bytes_per);
  if (e != hipSuccess) {
    *buf = nullptr;
    *cap = 0;
    return hip_fail(e, "batch buffer");
  }
  *cap = c;
  return LDNI_OK;
}

}  // namespace

extern "C" {

ldni_status ldni_batch_run(ldni_batch* b, void* hip_stream) {
  if (!b) return fail(LDNI_ERR_INVALID_ARG, "NULL batch");
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  for (int attempt = 0; attempt < 3; ++attempt) {
    if (!b->exec) {
      hipError_t e = batch_upload(b);
      if (e == hipSuccess) e = batch_capture(b);
      if (e != hipSuccess) return hip_fail(e, "batch graph capture");
    }
    HIP_TRY(hipGraphLaunch(b->exec, stream), "batch graph launch");
    HIP_TRY(hipStreamSynchronize(stream), "synchronise");
    const uint32_t* h = b->host_out;
    if (h[0] & kStatusBadIndex) return fail(LDNI_ERR_INDEX, "triangle index outside [0, n_verts)");
    if (h[0] & kStatusNonFinite) return fail(LDNI_ERR_NONFINITE, "non-finite vertex coordinate");
    if (h[0] & kStatusMismatch) return fail(LDNI_ERR_DEVICE, "tile lists disagree with their counts");
    bool regrow = false;
    const uint64_t entries = h[1];
    if (entries > b->list_cap) {
      ldni_status st = batch_grow(b, &b->lists, &b->list_cap, entries, sizeof(int2));
      if (st != LDNI_OK) return st;
      regrow = true;
    }
    uint64_t need = 0;
    for (int k = 0; k < b->n_img; ++k) {
      const uint32_t* r = h + 4 + 4 * (size_t)k;
      const uint64_t n = r[0];
      const uint64_t base = (uint64_t)r[1] | ((uint64_t)r[2] << 32);
      b->n[k] = r[0];
      b->base[k] = base;
      b->ml[k] = r[3];
      need = std::max(need, base + n);
    }
    if (regrow) {  // counts were made from truncated lists: sizes are not final
      batch_release_graph(b);
      continue;
    }
    if (need > b->sample_cap) {
      // per sample: depth, normal[3] (or one code), tri
      ldni_status st = batch_grow(b, &b->samples, &b->sample_cap, need, (b->rgb8 ? 3 : 5) * sizeof(float));
      if (st != LDNI_OK) return st;
      batch_release_graph(b);
      continue;
    }
    // Tiles that found no room in the staging buffer were walked again, so
    // the results stand; the buffer and the per-pixel cap grow for the next run.
    uint32_t ml = 0;
    for (int k = 0; k < b->n_img; ++k) ml = std::max(ml, b->ml[k]);
    const uint32_t layers = stage_layers_for(ml);
    if (layers > b->stage_layers) {
      // a larger item buffer first; without one the batch keeps its cap
      const uint64_t need_items =
          (uint64_t)max_place_items_per_tile(b->small ? 256 : 1024, layers) * b->total_tiles;
      void* grown = nullptr;
      if (!env_fault("alloc") && hipMalloc(&grown, (size_t)need_items * 16) == hipSuccess) {
        (void)hipStreamSynchronize(b->cs);
        (void)hipFree(b->items);
        b->items = grown;
        b->items_cap = need_items;
        b->stage_layers = layers;
        batch_release_graph(b);
      } else {
        (void)hipGetLastError();
      }
    }
    const uint32_t* tail = h + 4 + 4 * (size_t)b->n_img;
    // (tile regions start at 32-bit entry indices)
    const uint64_t demand = std::min<uint64_t>((uint64_t)tail[0] | ((uint64_t)tail[1] << 32), kMaxStageEntries);
    if (demand > b->stage_cap) {
      // 12 bytes per entry: key and pixel/slot
      if (batch_grow(b, &b->stage, &b->stage_cap, demand, sizeof(uint64_t) + sizeof(uint32_t)) != LDNI_OK) {
        b->stage = nullptr;  // no staging: every tile is walked again
        b->stage_cap = 0;
      }
      batch_release_graph(b);
    }
    return LDNI_OK;
  }
  return fail(LDNI_ERR_DEVICE, "batch sizing did not converge");
}

ldni_status ldni_batch_create(int32_t n_meshes, const ldni_mesh_desc* meshes, uint32_t axis_mask,
                              void* hip_stream, ldni_batch** out) {
  if (out) *out = nullptr;
  if (!out || !meshes || n_meshes < 1) return fail(LDNI_ERR_INVALID_ARG, "need meshes and an output handle");
  const bool rgb8 = (axis_mask & LDNI_NORMAL_RGB8) != 0;
  axis_mask &= ~(uint32_t)LDNI_NORMAL_RGB8;
  if (axis_mask == 0 || axis_mask > 7) return fail(LDNI_ERR_INVALID_ARG, "axis_mask must be in [1, 7]");
  const int naxes = __builtin_popcount(axis_mask);
  if ((int64_t)n_meshes * naxes > 65536) return fail(LDNI_ERR_INVALID_ARG, "too many images in one batch");
  for (int m = 0; m < n_meshes; ++m) {
    const ldni_mesh_desc& d = meshes[m];
    ldni_status st = validate(d.verts, d.n_verts, d.tris, d.n_tris, d.bbox, d.w, axis_mask);
    if (st != LDNI_OK) return fail(st, "mesh " + std::to_string(m) + ": " + g_last_error);
    if (d.tile_w != 0 || d.tile_h != 0) {
      const int tw = d.tile_w, th = d.tile_h;
      if (tw < 8 || tw > 256 || th < 1 || th > 64 || tw * th > 1024)
        return fail(LDNI_ERR_INVALID_ARG, "mesh " + std::to_string(m) + ": bad tile shape");
    }
  }
  int device = 0;
  HIP_TRY(hipGetDevice(&device), "hipGetDevice");
  ldni_batch* b = new (std::nothrow) ldni_batch();
  if (!b) return fail(LDNI_ERR_OUT_OF_MEMORY, "batch");
  auto bail = [&](ldni_status s) {
    batch_destroy(b);
    return s;
  };
  b->n_meshes = n_meshes;
  b->mask = axis_mask;
  b->rgb8 = rgb8;
  b->desc.assign(meshes, meshes + n_meshes);
  hipError_t e = hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(hip_fail(e, "stream"));
  e = hipHostMalloc(reinterpret_cast<void**>(&b->host_out),
                    sizeof(uint32_t) * (4 + 4 * (size_t)n_meshes * naxes + 4), hipHostMallocCoherent);
  if (e != hipSuccess) {
    b->host_out = nullptr;
    return bail(hip_fail(e, "pinned summary"));
  }

  // ---- tables ----
  b->tri_block_start.push_back(0);
  b->tile_start.push_back(0);
  b->seg_start.push_back(0);
  uint64_t tris_total = 0, rect_total = 0;
  std::vector<uint64_t> tri_off(n_meshes), rect_off;
  for (int m = 0; m < n_meshes; ++m) {
    const ldni_mesh_desc& d = meshes[m];
    tri_off[m] = tris_total;
    tris_total += (uint64_t)d.n_tris;
    const uint32_t tb = (uint32_t)((d.n_tris + kBinChunkTris - 1) / kBinChunkTris);
    b->tri_block_start.push_back(b->tri_block_start.back() + tb);
  }
  // images of meshes with small tiles (at most 256 pixels) first, so that
  // each tile class is one range of the batch's tiles
  for (int cls = 0; cls < 2; ++cls) {
    for (int m = 0; m < n_meshes; ++m) {
      const ldni_mesh_desc& d = meshes[m];
      int tw = 0, th = 0;
      tile_shape(d.w, d.n_tris, d.tile_w, d.tile_h, &tw, &th);
      if ((tw * th > 256) != (cls == 1)) continue;
      const uint64_t tiles = (uint64_t)((d.w + tw - 1) / tw) * ((d.w + th - 1) / th);
      for (int a = 0; a < 3; ++a) {
        if (!((axis_mask >> a) & 1u)) continue;
        b->img_mesh.push_back(m);
        b->img_axis.push_back(a);
        rect_off.push_back(rect_total);
        rect_total += (uint64_t)d.n_tris;
        b->tile_start.push_back((uint32_t)(b->tile_start.back() + tiles));
        b->seg_start.push_back(b->seg_start.back() + (uint64_t)d.w * d.w + 1);
      }
    }
    if (cls == 0) b->small_tiles = b->tile_start.back();
  }
  b->n_img = (int32_t)b->img_mesh.size();
  b->total_tiles = b->tile_start.back();
  b->total_slots = b->seg_start.back();
  if (b->total_tiles >= 0xffffffffull) return bail(fail(LDNI_ERR_INVALID_ARG, "too many tiles in one batch"));
  const int n_img = b->n_img;
  b->n.assign(n_img, 0);
  b->ml.assign(n_img, 0);
  b->base.assign(n_img, 0);

  // ---- workspace ----
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t o_status = take(sizeof(uint32_t) * 64);
  const size_t o_meshes = take(sizeof(BatchMesh) * n_meshes);
  const size_t o_images = take(sizeof(Image) * n_img);
  const size_t o_tbs = take(sizeof(uint32_t) * (n_meshes + 1));
  const size_t o_ts = take(sizeof(uint32_t) * (n_img + 1));
  const size_t o_ss = take(sizeof(uint64_t) * (n_img + 1));
  const size_t o_sb = take(sizeof(uint64_t) * n_img);
  const size_t o_ml = take(sizeof(uint32_t) * n_img);
  const size_t o_soup = take(sizeof(float) * 9 * tris_total);
  const size_t o_tnorm = take(sizeof(float4) * tris_total);
  const size_t o_rect = take(sizeof(Rect) * rect_total);
  // tile entry counts, then (16-byte aligned) tile candidate counts
  const uint64_t region_at = (b->total_tiles + 1 + 3) & ~(uint64_t)3;
  const size_t o_tile = take(sizeof(uint32_t) * (region_at + b->total_tiles + 1));
  // scatter cursors, entries counted apart, packed counts: cleared by one fill
  const size_t o_cur = take(sizeof(uint32_t) * 4 * b->total_tiles);
  const size_t o_brec = take(sizeof(uint4) * kBinSlots * (size_t)b->tri_block_start.back());
  const size_t o_bnrec = take(sizeof(uint32_t) * (size_t)b->tri_block_start.back());
  const size_t o_counts = take(sizeof(uint32_t) * b->total_slots);
  const size_t o_offs = take(sizeof(uint32_t) * b->total_slots);
  b->small = true;
  for (int m = 0; m < n_meshes; ++m)
    for (int a = 0; a < 3; ++a) {
      if (!((axis_mask >> a) & 1u)) continue;
      int tw = 0, th = 0;
      tile_shape(meshes[m].w, meshes[m].n_tris, meshes[m].tile_w, meshes[m].tile_h, &tw, &th);
      b->small = b->small && tw * th <= 256;
    }
  const size_t o_tstage = take(sizeof(uint32_t) * b->total_tiles);
  const size_t o_thits = take(sizeof(uint32_t) * b->total_tiles);
  const size_t o_tmax = take(sizeof(uint32_t) * b->total_tiles);
  const size_t o_walk = take(sizeof(uint32_t) * b->total_tiles);
  const size_t o_plan = take(sizeof(uint32_t) * (2 * b->total_tiles + 1));
  const size_t o_scan = take(std::max({scan_scratch_bytes(2 * (int64_t)b->total_tiles),
                                       scan_scratch_bytes((int64_t)b->total_tiles, 2),
                                       scan_scratch_bytes((int64_t)b->total_slots)}));
  e = env_fault("alloc") ? hipErrorOutOfMemory : hipMalloc(&b->ws, off);
  if (e != hipSuccess) {
    b->ws = nullptr;
    return bail(hip_fail(e, "batch workspace"));
  }
  b->ws_bytes = off;
  char* ws = static_cast<char*>(b->ws);
  BatchDevice& D = b->dev;
  D.status = reinterpret_cast<uint32_t*>(ws + o_status);
  D.work = D.status + 8;
  D.meshes = reinterpret_cast<BatchMesh*>(ws + o_meshes);
  D.n_meshes = n_meshes;
  D.images = reinterpret_cast<Image*>(ws + o_images);
  D.n_images = n_img;
  D.tri_block_start = reinterpret_cast<uint32_t*>(ws + o_tbs);
  D.tile_start = reinterpret_cast<uint32_t*>(ws + o_ts);
  D.seg_start = reinterpret_cast<uint64_t*>(ws + o_ss);
  D.sample_base = reinterpret_cast<uint64_t*>(ws + o_sb);
  D.host_out = b->host_out;
  b->max_layers = reinterpret_cast<uint32_t*>(ws + o_ml);
  b->tile_arena = reinterpret_cast<uint32_t*>(ws + o_tile);
  b->region_arena = b->tile_arena + region_at;
  b->cur_arena = reinterpret_cast<uint32_t*>(ws + o_cur);
  b->ovf_arena = b->cur_arena + b->total_tiles;
  b->pack_arena = reinterpret_cast<uint64_t*>(b->cur_arena + 2 * b->total_tiles);
  b->counts_arena = reinterpret_cast<uint32_t*>(ws + o_counts);
  b->offsets_arena = reinterpret_cast<uint32_t*>(ws + o_offs);
  b->scan_scratch = ws + o_scan;
  D.tile_total = b->tile_arena + b->total_tiles;
  D.plan = reinterpret_cast<uint32_t*>(ws + o_plan);
  D.walk_list = reinterpret_cast<uint32_t*>(ws + o_walk);
  D.walk_count = D.status + 18;
  D.region_total = b->region_arena + b->total_tiles;
  uint32_t* tstage = reinterpret_cast<uint32_t*>(ws + o_tstage);
  uint32_t* thits = reinterpret_cast<uint32_t*>(ws + o_thits);
  uint32_t* tmax = reinterpret_cast<uint32_t*>(ws + o_tmax);
  D.tile_max = tmax;

  b->meshes_h.assign(n_meshes, BatchMesh{});
  b->images_h.assign(n_img, Image{});
  float* soup = reinterpret_cast<float*>(ws + o_soup);
  float4* tnorm = reinterpret_cast<float4*>(ws + o_tnorm);
  Rect* rect = reinterpret_cast<Rect*>(ws + o_rect);
  for (int m = 0; m < n_meshes; ++m) {
    BatchMesh& bm = b->meshes_h[m];
    bm.m.verts = meshes[m].verts;
    bm.m.n_verts = meshes[m].n_verts;
    bm.m.tris = meshes[m].tris;
    bm.m.n_tris = meshes[m].n_tris;
    bm.m.soup = soup + 9 * tri_off[m];
    bm.m.tnorm = tnorm + tri_off[m];
    bm.m.status = D.status;
    bm.m.bin_rec = reinterpret_cast<uint4*>(ws + o_brec) + (size_t)kBinSlots * b->tri_block_start[m];
    bm.m.bin_nrec = reinterpret_cast<uint32_t*>(ws + o_bnrec) + b->tri_block_start[m];
    bm.nimg = 0;
  }
  for (int k = 0; k < n_img; ++k) {
    const int m = b->img_mesh[k], a = b->img_axis[k];
    const ldni_mesh_desc& d = meshes[m];
    BatchMesh& bm = b->meshes_h[m];
    Image& im = b->images_h[k];
    im.a = a;
    im.u = (a + 1) % 3;
    im.v = (a + 2) % 3;
    im.w = d.w;
    im.lo_u = (double)d.bbox[im.u];
    im.h_u = ((double)d.bbox[3 + im.u] - (double)d.bbox[im.u]) / (double)d.w;
    im.lo_v = (double)d.bbox[im.v];
    im.h_v = ((double)d.bbox[3 + im.v] - (double)d.bbox[im.v]) / (double)d.w;
    im.lo_a = (double)d.bbox[a];
    tile_shape(d.w, d.n_tris, d.tile_w, d.tile_h, &im.tw, &im.th);
    finish_image_geometry(im);
    im.ntx = (d.w + im.tw - 1) / im.tw;
    im.nty = (d.w + im.th - 1) / im.th;
    im.soup = bm.m.soup;
    im.tnorm = bm.m.tnorm;
    im.rect = rect + rect_off[k];
    bm.m.rect[bm.nimg] = rect + rect_off[k];
    bm.img[bm.nimg++] = k;
    im.n_tris = d.n_tris;
    im.tile_cnt = b->tile_arena + b->tile_start[k];
    im.tile_cur = b->cur_arena + b->tile_start[k];
    im.tile_ovf = b->ovf_arena + b->tile_start[k];
    im.tile_pack = b->pack_arena + b->tile_start[k];
    im.counts = b->counts_arena + b->seg_start[k];
    im.max_layers = b->max_layers + k;
    im.offsets = b->offsets_arena + b->seg_start[k];
    im.status = D.status;
    im.tile_region = b->region_arena + b->tile_start[k];
    im.tile_stage = tstage + b->tile_start[k];
    im.tile_hits = thits + b->tile_start[k];
    im.tile_max = tmax + b->tile_start[k];
    im.walk_list = D.walk_list;
    im.walk_count = D.walk_count;
  }
  e = hipMemcpy(const_cast<uint32_t*>(D.tri_block_start), b->tri_block_start.data(),
                sizeof(uint32_t) * (n_meshes + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(const_cast<uint32_t*>(D.tile_start), b->tile_start.data(), sizeof(uint32_t) * (n_img + 1),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(const_cast<uint64_t*>(D.seg_start), b->seg_start.data(), sizeof(uint64_t) * (n_img + 1),
                  hipMemcpyHostToDevice);
  // the last slot of every image's counts stays zero for the segmented scan
  if (e == hipSuccess) e = launch_fill_u32(b->counts_arena, 0u, (int64_t)b->total_slots, b->cs);
  if (e == hipSuccess) e = hipStreamSynchronize(b->cs);
  if (e != hipSuccess) return bail(hip_fail(e, "batch tables"));

  // tile lists sized like the single-mesh path; outputs sized by the first run
  uint64_t cap = 1024;
  for (int k = 0; k < n_img; ++k)
    cap += (uint64_t)std::ceil((double)meshes[b->img_mesh[k]].n_tris * std::min(g_list_ratio.load(), 8.0)) +
           4 * (uint64_t)(b->tile_start[k + 1] - b->tile_start[k]);
  ldni_status st = batch_grow(b, &b->lists, &b->list_cap, cap, sizeof(int2));
  if (st != LDNI_OK) return bail(st);
  // staging: a first guess (24 entries per triangle and image plus one per pixel),
  // grown to the demand after the first run if it was short
  {
    uint64_t guess = 65536;
    for (int k = 0; k < n_img; ++k)
      guess += 24 * (uint64_t)meshes[b->img_mesh[k]].n_tris +
               (uint64_t)meshes[b->img_mesh[k]].w * meshes[b->img_mesh[k]].w;
    guess = std::min<uint64_t>(guess, kMaxStageEntries);
    if (batch_grow(b, &b->stage, &b->stage_cap, guess, sizeof(uint64_t) + sizeof(uint32_t)) != LDNI_OK) {
      b->stage = nullptr;
      b->stage_cap = 0;
    }
  }
  st = batch_grow(b, &b->items, &b->items_cap,
                  (uint64_t)max_place_items_per_tile(b->small ? 256 : 1024, b->stage_layers) * b->total_tiles,
                  16);
  if (st != LDNI_OK) return bail(st);
  st = ldni_batch_run(b, hip_stream);
  if (st != LDNI_OK) return bail(st);
  *out = b;
  return LDNI_OK;
}

ldni_status ldni_batch_axis(const ldni_batch* b, int32_t mesh, int axis, ldni_axis_view* view) {
  if (!b || !view || mesh < 0 || mesh >= b->n_meshes || axis < 0 || axis > 2)
    return fail(LDNI_ERR_INVALID_ARG, "bad batch/mesh/axis/view");
  std::memset(view, 0, sizeof(*view));
  for (int k = 0; k < b->n_img; ++k) {
    if (b->img_mesh[k] != mesh || b->img_axis[k] != axis) continue;
    view->w = b->desc[mesh].w;
    view->max_layers = b->ml[k];
    view->n_samples = b->n[k];
    view->offsets = b->offsets_arena + b->seg_start[k];
    const uint64_t nw = b->rgb8 ? 1 : 3;
    const float* arena = static_cast<const float*>(b->samples);
    view->depth = arena + b->base[k];
    if (b->rgb8)
      view->normal_rgb8 = reinterpret_cast<const uint32_t*>(arena + b->sample_cap) + b->base[k];
    else
      view->normal = arena + b->sample_cap + 3 * b->base[k];
    view->tri = reinterpret_cast<const int32_t*>(arena + (1 + nw) * b->sample_cap) + b->base[k];
  }
  return LDNI_OK;
}

void ldni_batch_free(ldni_batch* b) { batch_destroy(b); }

ldni_status ldni_sample_batch(int32_t n_meshes, const ldni_mesh_desc* meshes, uint32_t axis_mask,
                              void* hip_stream, ldni_batch** out) {
  return ldni_batch_create(n_meshes, meshes, axis_mask, hip_stream, out);
}

}  // extern "C"
