// ldni_internal.hpp -- types shared by the gfx950 kernels (ldni_kernels.hip)
// and the host orchestration behind the C ABI (ldni_api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ldni {

// Pixel rectangle of a triangle on one image: columns [i0, i1), rows [j0, j1).
// Only pixels whose centre satisfies min <= c < max in both image
// coordinates can be hit, so this is exactly the candidate set.
struct Rect {
  int16_t i0, i1, j0, j1;
};

// Status bits raised by the device.
enum : uint32_t {
  kStatusBadIndex = 1u,
  kStatusNonFinite = 2u,
  kStatusOverflow = 4u,
  kStatusMismatch = 8u,  // write pass found more hits than the count pass
  kStatusListFull = 16u, // batch: tile lists longer than their capacity
  kStatusOutFull = 32u,  // batch: samples beyond the output capacity
};

// Everything one image (one axis of one mesh) needs on the device.
struct Image {
  // geometry
  int32_t a, u, v;   // sampled axis and image axes (cyclic)
  int32_t w;         // resolution
  double lo_u, h_u;  // pixel centre c_u[i] = f32(lo_u + (i + 0.5) * h_u)
  double lo_v, h_v;
  double inv_h_u, inv_h_v;  // 1 / h (first estimates of pixel indices only)
  // An estimate t = (x - lo) / h - 0.5 farther than this from every integer
  // gives the first centre at or above x as ceil(t), float32 rounding of the
  // centres included; nearer, the centres are compared one by one.
  double slack_u, slack_v;
  double lo_a;       // depth origin
  // tiling
  int32_t tw, th;    // tile shape in pixels
  int32_t tw_shift, th_shift;  // log2 of tw, th when a power of two, else -1
  int32_t ntx, nty;  // tiles along u and v
  // mesh (shared by the images of one mesh)
  const float* soup;   // [T][9] vertex coordinates A,B,C (x,y,z each)
  const float4* tnorm;  // [T] unit face normals (x, y, z, 0): one 16-byte load each
  const Rect* rect;    // [T] candidate rectangle on this image
  int64_t n_tris;
  // workspace
  uint32_t* tile_cnt;   // [n_tiles + 1] entries per tile -> exclusive offsets
  uint32_t* tile_cur;   // [n_tiles] scatter cursors (of the entries counted in tile_ovf)
  uint32_t* tile_ovf;   // [n_tiles] entries counted outside the chunk tables (listed
                        // first in the tile), or null where binning is per triangle
  uint64_t* tile_pack;  // [n_tiles] chunk binning: entries reserved by the chunk
                        // tables (low half) and candidates (high half), or null
  int2* tile_list;      // entries grouped by tile: (triangle id, its candidate
                        // rectangle in the tile: x0 | y0 << 8 | (width - 1) << 16
                        // | (height - 1) << 24, tile-local pixels)
  uint64_t list_cap;    // capacity of tile_list (entries beyond it are dropped)
  uint32_t* counts;     // [w*w] samples per pixel
  uint32_t* max_layers; // [1] largest per-pixel count (atomic max per tile unless
                        // tile_max is given), or null when the pixel scan takes it
  uint32_t* tile_max;   // [n_tiles] largest count of each tile, or null
  // outputs
  uint32_t* offsets;  // [w*w + 1]
  float* depth;       // [n]
  float* normal;      // [n][3] (unused when normal_rgb8 is set)
  uint32_t* normal_rgb8;  // [n] 8-bit normal codes, or null for float normals
  int32_t* tri;       // [n]
  uint32_t* status;   // shared status word
  // Hits of the sampling pass, grouped by tile.  With stage_key null every
  // tile with hits is walked again by the place pass.
  uint64_t* stage_key;               // (depth key, triangle) of each hit
  uint32_t* stage_qs;                // tile pixel | (slot within the pixel << 10)
  uint64_t stage_cap;                // entries in the buffer (below 2^32 - 1)
  uint32_t stage_layers;             // a tile's region holds at most this many entries per pixel
  // [n_tiles + 1] the tile's candidates, each triangle's rounded up to whole
  // 4-entry groups (counted by setup); the region scan turns them into the
  // tile's staging region [tile_region[t], tile_region[t + 1]) (capped at
  // stage_layers entries per tile pixel, saturating at 2^32 - 1)
  uint32_t* tile_region;
  uint32_t* tile_stage;              // [n_tiles] first entry of the tile's hits (a multiple
                                     // of 4; regions are whole 4-entry groups), or kNoStage
  uint32_t* tile_hits;               // [n_tiles] hits of the tile
  uint32_t* walk_list;               // set-wide tile numbers the write pass walks again
  uint32_t* walk_count;              // entries of walk_list (shared by the set)
};

// tile_stage value of a tile whose hits did not fit its staging region
constexpr uint32_t kNoStage = 0xffffffffu;

constexpr int kMaxImages = 3;

// Up to three images launched together; tile blocks are numbered through the
// images in order.
struct ImageSet {
  Image img[kMaxImages];
  int32_t n;
  uint32_t tile_start[kMaxImages + 1];  // prefix of tile counts
  // place-pass plan written by the sampling pass (null: none): items per
  // tile, [0, n_tiles) for tiles of two or more items, [n_tiles, 2 n_tiles)
  // for tiles of one, scanned in place into item positions
  uint32_t* plan;
  int32_t place_cap;  // stage capacity of the place pass
};

// Mesh-level setup: per triangle gather, validate, face normal, candidate
// rectangles for every image in the set.
struct MeshSetup {
  const float* verts;
  int64_t n_verts;
  const int32_t* tris;
  int64_t n_tris;
  float* soup;
  float4* tnorm;  // [T] unit face normals (x, y, z, 0)
  Rect* rect[kMaxImages];
  uint32_t* status;
  // binning by chunks of kBinChunkTris triangles: per chunk up to kBinSlots
  // records (image << 30 | tile, table slot, first list entry reserved in the
  // tile, 0) and their number
  uint4* bin_rec;
  uint32_t* bin_nrec;
};

// Triangles per binning chunk and the size of its LDS table of tiles.
constexpr int kBinChunkTris = 512;
constexpr int kBinSlots = 1024;

// Fills the derived fields of an image (inverse steps, centre slack, tile
// shifts) from w, the tile shape and lo/h of both image axes.
void finish_image_geometry(Image& im);

// ---- launchers (ldni_kernels.hip) ----
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, int64_t n, hipStream_t s);
// per chunk of triangles: gather, validate, normal, candidate rectangles,
// and the entries and candidates of every tile met, reserved per chunk
// (tile_cnt, tile_region, tile_ovf cleared before; m.bin_rec/bin_nrec
// written)
hipError_t launch_setup(const MeshSetup& m, const ImageSet& set, hipStream_t s);
// per chunk: the tile-list entries at the ranges launch_setup reserved (after
// the tile scan; tile_cur cleared before)
hipError_t launch_bin_scatter(const MeshSetup& m, const ImageSet& set, hipStream_t s);
// Sampling pass: per-pixel counts, and every hit staged by tile (see Image).
hipError_t launch_sample(const ImageSet& set, hipStream_t s);
// Work items of the place pass: scans the plan the sampling pass wrote and
// writes the item records (16 bytes each, at most
// max_place_items_per_tile(tw * th, stage_layers) per tile) in launch order.
int max_place_items_per_tile(int tile_pix, uint32_t stage_layers);
// Entries per pixel a tile may reserve in the staging buffer: the deepest
// pixel seen, rounded up to a power of two, within [64, 1024].
uint32_t stage_layers_for(uint32_t max_layers_seen);
int place_stage_cap(int tile_pix);
hipError_t launch_plan_items(const ImageSet& set, void* items, void* scratch, uint32_t* status,
                             hipStream_t s);
// Place pass: n_items workgroups place the staged tiles; the n_walk tiles of
// walk_list are then walked again (persistent, counter[0]).
hipError_t launch_place(const ImageSet& set, const void* items, uint32_t n_items, uint32_t* counter,
                        uint32_t n_walk, hipStream_t s);

// ---- batched sampling: many meshes, each with its own w and tile shape ----
struct BatchMesh {
  MeshSetup m;
  int32_t nimg;
  int32_t img[kMaxImages];  // indices into the image table
};

struct BatchDevice {
  BatchMesh* meshes;
  int32_t n_meshes;
  Image* images;
  int32_t n_images;
  const uint32_t* tri_block_start;  // [n_meshes+1] binning chunks per mesh (prefix)
  const uint32_t* tile_start;       // [n_images+1] tiles per image (prefix)
  const uint32_t* tile_max;         // [total tiles] largest count of each tile
  const uint64_t* seg_start;        // [n_images+1] first slot of each image in counts/offsets
  uint64_t* sample_base;            // [n_images] first sample of each image in the outputs
  uint32_t* work;                   // [2] work counters of the persistent kernels
  uint32_t* status;
  float* depth;                     // output arenas, sample_cap samples
  float* normal;                    // float normals, or null
  uint32_t* normal_rgb8;            // 8-bit normal codes, or null
  int32_t* tri;
  uint64_t sample_cap;
  uint32_t* tile_total;             // entries of all tile lists (end of the tile scan)
  uint64_t list_cap;
  uint32_t* host_out;               // pinned: [0] status, [1] list entries, then per image
                                    // (n, base lo, base hi, max layers), then staging
                                    // demand (lo, hi) and tiles walked again
  // staged sampling (see Image): place plan over all tiles of the batch,
  // item records, tiles walked again
  uint32_t* plan;                   // [2 * total tiles + 1]
  void* items;                      // place items
  uint32_t* walk_list;
  uint32_t* walk_count;
  const uint32_t* region_total;     // staging entries the regions of the batch ask for
};

// setup and tile counts, then (after the tile scan) the scatter: chunks of
// kBinChunkTris triangles of all meshes (tri_block_start.back() of them)
hipError_t launch_batch_setup(const BatchDevice& b, uint32_t chunks, hipStream_t s);
hipError_t launch_batch_scatter(const BatchDevice& b, uint32_t chunks, hipStream_t s);
// n_tiles: tiles of the batch, the first n_small of them those of the
// images whose tiles have at most 256 pixels (each class runs its own build of
// the tile kernels).  Sampling pass (counts, staged hits, place plan), then
// after the pixel scan and the placement of the images: the place items, the
// place pass and the walk of the tiles whose hits were not staged.
hipError_t launch_batch_sample(const BatchDevice& b, uint32_t n_tiles, uint32_t n_small, hipStream_t s);
hipError_t launch_batch_place(const BatchDevice& b, uint32_t n_tiles, uint32_t n_small, void* scratch,
                              hipStream_t s);
// Segmented exclusive scan of the per-image counts (segments of w*w+1 slots,
// the last slot of each zero) into per-image offsets starting at 0, with the
// u64 start of every segment in sample_base.
hipError_t launch_batch_pixel_scan(const BatchDevice& b, const uint32_t* counts, uint32_t* offsets,
                                   int64_t n_slots, void* scratch, hipStream_t s);
// Places every image in the output arena (or flags kStatusOutFull) and
// writes the host summary.
hipError_t launch_batch_finish_counts(const BatchDevice& b, hipStream_t s);

// Vertex gradient of sum(gd * depth) + sum(gn . normal) over the images of
// one forward result.
struct BackwardAxis {
  int32_t a;
  const uint32_t* offsets;
  const int32_t* tri;
  const float* gd;  // may be null
  const float* gn;  // may be null
  float* acc;       // workspace [T][6], zeroed
};
struct BackwardArgs {
  BackwardAxis axis[kMaxImages];
  int32_t n;
  int32_t w;
  double bbox[6];
  const float* verts;
  int64_t n_verts;
  const int32_t* tris;
  int64_t n_tris;
  float* grad;   // [V][3], accumulated
};
hipError_t launch_backward(const BackwardArgs& args, hipStream_t s);

// ---- Boolean operations on two LDNIs of one axis (ldni_boolean.hip) ----
constexpr int kBoolUnion = 0, kBoolIntersection = 1, kBoolDifference = 2;
struct AxisArrays {
  uint64_t n;               // samples
  const uint32_t* offsets;  // [npix + 1]
  const float* depth;
  const float* normal;      // [n][3]
  const int32_t* tri;
};
struct BooleanArgs {
  AxisArrays a, b;
  int64_t npix;
  int32_t op;
  double eps;             // volumes thinner than this are removed
  uint32_t* counts;       // [npix + 1]: kept samples per pixel (count pass),
                          // scanned in place into the result offsets (write pass)
  uint32_t* refs;         // [a.n + b.n]: sources of the kept samples (count pass)
  uint32_t* status;       // kStatusMismatch: offsets of an input out of order
  float* out_depth;
  float* out_normal;
  int32_t* out_tri;
};
hipError_t launch_boolean(const BooleanArgs& g, bool write, hipStream_t s);

// Copies n (<= 16) device words into pinned, device-visible host memory.
// Grid-node classification of three LDNIs of one box and resolution
// (ldni_nodes.hip).  axis[a] is the a-LDNI; lo/h the node origin and
// spacing per world axis; bits holds nb^3 bricks of 1024 words (nb =
// ceil(w/32)); partial 2 words per workgroup (node_workgroups); stats[0..1]
// = nodes inside, nodes whose three votes differ.
struct NodeArgs {
  AxisArrays axis[3];
  int32_t w, nb;
  double lo[3], h[3];
  uint32_t* bits;
  uint32_t* status;   // kStatusMismatch: offsets of an input out of order
  uint64_t* partial;
  uint64_t* stats;
  uint16_t* codes;    // node_code_bytes(w): span codes of the three axes (launch_node_codes)
  int32_t n_spans;    // ceil(w / 64)
};
uint32_t node_workgroups(int32_t w);
size_t node_code_bytes(int32_t w);
hipError_t launch_node_codes(const NodeArgs& g, hipStream_t s);
hipError_t launch_classify_nodes(const NodeArgs& g, hipStream_t s);
hipError_t launch_node_stats(const NodeArgs& g, hipStream_t s);

// Offsetting (ldni_offset.hip): the three input LDNIs, their box (lo, h per
// world axis), |r| and eps, the sphere centres (3 doubles per sample,
// numbered over x, y, z with base[a] the first number of axis a), the
// binning of spheres into the lists of the rays they hit (ray_count over the
// 3 w^2 rays, scanned into ray_start[3 w^2 + 1], ray_cursor, list), the
// per-ray result counts (scanned in place into the output offsets) and the
// output arrays of the write pass.
constexpr int kOffsetBuf = 1024;              // events of one depth window of one ray, in LDS
constexpr int kOffsetKeep = 896;              // a full window is cut back to fewer events than this
constexpr int kOffsetEmit = 128;              // end points of one ray's result before small volumes go
constexpr int kOffsetSavedMax = 64;           // most end points per ray the count pass keeps for the write pass
constexpr int kOffsetDeep = 512;              // a ray with more spheres than this is started first
constexpr uint32_t kMaxSpheres = 1u << 30;    // sphere numbers fit 30 bits of the sort key
struct OffsetArgs {
  AxisArrays in[3];
  int32_t w;
  uint32_t n_spheres;
  uint64_t base[3];
  double lo[3], h[3];
  // per axis, the pixels by which a centre index can differ from the real
  // (x - lo) / h - 0.5 for the float32 rounding of the centres
  double margin[3];
  double r, eps;
  int32_t union_op;
  double* centres;
  uint32_t *ray_count, *ray_start, *ray_cursor, *list;
  uint32_t* counts[3];
  const uint32_t* out_offsets[3];
  float* out_depth[3];
  float* out_normal[3];
  int32_t* out_tri[3];
  uint64_t* saved;   // [3 * w * w][n_saved] kept end-point keys, or null (the write pass recomputes)
  uint32_t n_saved;  // end points kept per ray (at most kOffsetSavedMax)
  // rays with more than kOffsetDeep spheres, listed (any order) so that the
  // ray passes start them first; n_deep of them (known to the host before
  // the ray passes; status[16] counts them on the device)
  uint32_t* deep;
  uint32_t n_deep;
  uint32_t* status;  // kStatusMismatch: bad input offsets; kStatusOutFull: a ray's window or end points overflow
};
hipError_t launch_offset_centres(const OffsetArgs& g, hipStream_t s);
hipError_t launch_offset_bin(const OffsetArgs& g, bool scatter, hipStream_t s);
// the list of deep rays (after the ray-list scan)
hipError_t launch_offset_deep(const OffsetArgs& g, hipStream_t s);
hipError_t launch_offset_rays(const OffsetArgs& g, bool write, hipStream_t s);

// Copies n <= kMaxGather scattered device words to pinned host memory.
constexpr int kMaxGather = 32;
hipError_t launch_gather(const uint32_t* const* src, int n, uint32_t* host_dst, hipStream_t s);

// Exclusive scan of n u32 values into out[0..n] (out[n] = total).  Totals of
// 2^32 or more raise kStatusOverflow.  scratch: scan_scratch_bytes(n, 1).
// max_out (if given) receives the largest value.
size_t scan_scratch_bytes(int64_t n, int nseg = 1);
hipError_t launch_scan(const uint32_t* in, uint32_t* out, int64_t n, void* scratch,
                       uint32_t* status, hipStream_t s, uint32_t* max_out = nullptr);
// nseg <= kMaxImages such scans of n values each, in one set of launches
// (in place allowed); scratch: scan_scratch_bytes(n, nseg); max_out[k] as
// above per segment.
hipError_t launch_scan_segments(const uint32_t* const* in, uint32_t* const* out, int nseg, int64_t n,
                                void* scratch, uint32_t* status, hipStream_t s,
                                uint32_t* const* max_out = nullptr);
// The tile scan: entry counts -> list offsets (as launch_scan, into
// tile_cnt), and in the same launches candidate counts -> staging regions
// (tile_region), each tile's count capped at region_cap and the prefix
// saturating at 2^32 - 1 (n + 1 slots each).  The counts come from tile_pack
// and tile_ovf when tile_pack is given, else from tile_cnt and tile_region
// themselves (in place).  scratch: scan_scratch_bytes(n, 2).
hipError_t launch_tile_scan(const uint64_t* tile_pack, const uint32_t* tile_ovf, uint32_t* tile_cnt,
                            uint32_t* tile_region, int64_t n, uint32_t region_cap, void* scratch, uint32_t* status,
                            hipStream_t s);

}  // namespace ldni
