/*
 * ldni.h -- C ABI of the MI355X (gfx950) Layered Depth-Normal Image sampler.
 *
 * Implements the sampling step of Wang & Chen, "Layered Depth-Normal Images:
 * a Sparse Implicit Representation of Solid Models": a closed triangle mesh
 * is turned into three LDNIs, one per world axis (Sec. 2, Definitions 1-3;
 * Sec. 3 builds them by rasterisation).  For axis a, a w x w grid of rays
 * parallel to a passes through the pixel centres (Sec. 3, "centre of
 * pixel"); every intersection of a ray with a triangle, except with faces
 * parallel to the ray (the note after Definition 1), becomes a Hermite
 * sample (depth, unit face normal) (Definition 2; accurate normal sampling
 * in Sec. 3), and each pixel's samples are stored in ascending depth order
 * (Definition 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  Frame.   Axis a images the two other axes cyclically:
 *           a=x -> (u,v)=(y,z), a=y -> (z,x), a=z -> (x,y).  Pixel (i,j) is
 *           p = j*w + i, i along u, j along v.
 *  Centres. c_u[i] = f32(lo_u + (i + 0.5) * h_u) evaluated in float64 with
 *           h_u = (hi_u - lo_u) / w; the same formula on every axis, so the
 *           rays of the three images meet at the nodes of one w^3 grid
 *           (Definition 3).  Boxes need not be cubic.
 *  Hits.    Vertices are translated into the ray frame in float32 and the
 *           three edge functions are evaluated with exact signs; a ray that
 *           meets an edge or vertex exactly is decided as if moved to
 *           (+eps, +eps^2) in (u,v).  A non-silhouette edge or vertex is thus
 *           owned by exactly one triangle and a silhouette gives 0 or 2 hits,
 *           so every ray through a closed mesh has an even count
 *           (Remark 1, Definition 4).  Rays are infinite lines: hits outside
 *           the box along the axis are kept.
 *  Depth.   float32 distance from lo_a along +a, from a float64 barycentric
 *           interpolation of the hit triangle's axis coordinates; a zero
 *           depth is stored as +0.
 *  Normal.  float32 unit normal of the hit face, (B-A)x(C-A) normalised in
 *           float64, in world (x,y,z) order, never flipped toward the ray
 *           (outward for counter-clockwise-outward meshes).
 *  Order.   Per pixel by depth, equal depths by ascending triangle id.
 *  Layout.  Per axis, compact rows: offsets[w*w+1] (u32, exclusive prefix
 *           sums, offsets[w*w] = n), then depth[n], normal[n][3], tri[n].
 *  Device.  All pointers named "device" refer to memory of the current HIP
 *           device.  All work is ordered on the given hipStream_t (NULL =
 *           the null stream).  Inputs are read-only and stay owned by the
 *           caller; they must stay valid until the call (or the plan) ends.
 *  Errors.  Every call returns an ldni_status and never throws; on error
 *           every output handle is set to NULL.  Argument errors are found
 *           on the host before any GPU work; index, non-finite and overflow
 *           errors are found on the device and reported at the call's
 *           synchronisation point.  ldni_last_error() gives a thread-local
 *           message for the last failing call.
 *  Limits.  1 <= w <= 16384; fewer than 2^32 samples per axis; triangle
 *           indices in [0, n_verts); 0 <= n_tris < 2^31.
 */
#ifndef LDNI_H
#define LDNI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LDNI_OK = 0,
  LDNI_ERR_INVALID_ARG = 1,   /* host-detected bad argument */
  LDNI_ERR_INDEX = 2,         /* a triangle index outside [0, n_verts) */
  LDNI_ERR_OUT_OF_MEMORY = 3, /* device or host allocation failed */
  LDNI_ERR_OVERFLOW = 4,      /* 2^32 or more samples on one axis */
  LDNI_ERR_DEVICE = 5,        /* a HIP runtime call failed */
  LDNI_ERR_NONFINITE = 6      /* a referenced vertex has a NaN/Inf coordinate */
} ldni_status;

enum { LDNI_AXIS_X = 1u, LDNI_AXIS_Y = 2u, LDNI_AXIS_Z = 4u, LDNI_AXIS_ALL = 7u };

/* Option bit for the axis_mask of ldni_sample, ldni_batch_create and
 * ldni_sample_batch: store each sample's normal as the 8-bit colour code of
 * Sec. 3's approximate normal sampling (one u32: x | y << 8 | z << 16, each
 * byte the rounded colour (c + 1) / 2 * 255) in the view's normal_rgb8
 * instead of three floats in normal.  Every other entry point rejects it. */
enum { LDNI_NORMAL_RGB8 = 256u };

/* Read-only view of one axis of a result (borrowed; valid until the result
 * is freed). */
typedef struct {
  int32_t w;
  uint32_t max_layers;     /* largest per-pixel sample count (the paper's n_max) */
  uint64_t n_samples;
  const uint32_t *offsets; /* device [w*w+1] */
  const float *depth;      /* device [n_samples] */
  const float *normal;     /* device [n_samples][3] */
  const int32_t *tri;      /* device [n_samples], id of the hit triangle */
  const uint32_t *normal_rgb8; /* device [n_samples] 8-bit normal codes of a
                                  result made with LDNI_NORMAL_RGB8 (normal is
                                  then NULL), else NULL; ignored in inputs */
} ldni_axis_view;

typedef struct ldni_result ldni_result; /* opaque; owns its device buffers */
typedef struct ldni_plan ldni_plan;     /* opaque; a sampling call split in two */

/*
 * ldni_sample -- build the LDNIs of one mesh (Sec. 2 Definitions 1-3; Sec. 3).
 *   verts     device f32 [n_verts][3], row-major.
 *   tris      device i32 [n_tris][3], counter-clockwise seen from outside.
 *   bbox      HOST f32 {xlo, ylo, zlo, xhi, yhi, zhi}, lo < hi, finite.  The
 *             paper's working envelope (Sec. 3): it fixes the pixel grid
 *             and the depth origin; it does not clip.
 *   w         resolution, 1..16384.
 *   axis_mask any non-empty subset of LDNI_AXIS_{X,Y,Z}, optionally with
 *             LDNI_NORMAL_RGB8 (8-bit normal codes instead of float normals).
 *   out       receives a result that owns every output buffer (device memory
 *             from the stream-ordered pool of the current device); release it
 *             with ldni_free.  Axes not in the mask have empty views.
 * One host synchronisation per call (a second only when a first estimate of
 * the tile-list size was too small): the per-axis sample counts, after the
 * count pass.  The write pass then runs behind the call on hip_stream; the
 * result's first ldni_result_axis waits for it and reports LDNI_ERR_DEVICE if
 * it disagreed with the count pass.  n_tris == 0 is valid (no samples).
 */
ldni_status ldni_sample(const float *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                        const float bbox[6], int32_t w, uint32_t axis_mask, void *hip_stream,
                        ldni_result **out);

/* View of axis 0 (x), 1 (y) or 2 (z): one of the three LDNIs of
 * Definition 3, each an LDI whose depths carry unit normals (Definitions 1
 * and 2).  LDNI_ERR_INVALID_ARG for a NULL result or view, or an axis
 * outside 0..2.  The first call on a result waits for the kernels that
 * wrote it; LDNI_ERR_DEVICE (here and in every later call on the result)
 * when a write pass stored more or fewer samples of a pixel than its count
 * pass counted -- the result must then not be used. */
ldni_status ldni_result_axis(const ldni_result *r, int axis, ldni_axis_view *view);

/* Release a result -- the LDNIs of Definition 3 it holds (NULL-safe).  Its
 * buffers are kept by the library for later calls on the stream the result
 * was made on (reused in that stream's order, like hipFreeAsync), which must
 * still exist.  A result whose kernels may still run is waited for first. */
void ldni_free(ldni_result *r);

/* Device memory the library keeps between calls: the buffers of released
 * results and each call's workspace, per (device, stream), at most 8 per
 * stream.  ldni_trim hands all of it back to the device (synchronous; no
 * call may be in flight, and every stream the library was used on must
 * still exist).  Returns LDNI_OK or LDNI_ERR_DEVICE. */
ldni_status ldni_trim(void);

/*
 * ldni_sample_begin / ldni_sample_finish -- the same sampling with
 * caller-owned outputs, split at the point where the sample counts become
 * known.
 *   offsets   device u32 [w*w+1] per axis in the mask (entries of other axes
 *             are ignored and may be NULL), 16-byte aligned (written with
 *             16-byte stores; LDNI_ERR_INVALID_ARG otherwise); filled by begin.
 *   n_samples HOST u64 [3]; begin writes the count of every axis (0 for
 *             axes not in the mask).
 *   plan      receives the state that finish needs (workspace on the device).
 * Then finish writes, for every axis in the mask, depth f32 [n], normal f32
 * [n][3] and tri i32 [n] into caller device buffers of at least n_samples[a]
 * elements, waits for the write pass (LDNI_ERR_DEVICE if it disagreed with
 * the count pass), and releases the plan whether or not it succeeds.  A plan not
 * finished must be released with ldni_plan_free.  verts/tris must stay
 * unchanged until finish returns.
 */
ldni_status ldni_sample_begin(const float *verts, int64_t n_verts, const int32_t *tris,
                              int64_t n_tris, const float bbox[6], int32_t w, uint32_t axis_mask,
                              uint32_t *const offsets[3], void *hip_stream, ldni_plan **plan,
                              uint64_t n_samples[3]);
ldni_status ldni_sample_finish(ldni_plan *plan, float *const depth[3], float *const normal[3],
                               int32_t *const tri[3]);
/*
 * ldni_sample_finish_rgb8 -- ldni_sample_finish with the paper's approximate
 * normal sampling (Sec. 3, "Approximate Surface Normal Sampling"; the
 * accuracy trade-off under "Balance between time and accuracy"): each
 * component c of a sample's unit normal is stored as the 8-bit colour of
 * (c + 1) / 2, b = floor((c + 1) * 127.5 + 0.5) clamped to [0, 255]
 * (float64 operations in that order), packed as x | y << 8 | z << 16 in one
 * 32-bit word per sample (decode: c ~ b / 127.5 - 1, within 1/255).  Depth,
 * triangle id, order and counts are those of ldni_sample_finish.
 *   normal_rgb8  HOST array of 3 device u32 [n] pointers (entries of axes not
 *                in the mask ignored).  Same ownership and errors as
 *                ldni_sample_finish; the plan is released either way.
 */
ldni_status ldni_sample_finish_rgb8(ldni_plan *plan, float *const depth[3], uint32_t *const normal_rgb8[3],
                                    int32_t *const tri[3]);
void ldni_plan_free(ldni_plan *plan);

/*
 * ldni_backward -- vertex gradient of a loss through the sampling (not in the
 * paper; the differentiation of its Definition 2 samples).  For upstream
 * gradients gd = dL/d depth and gn = dL/d normal of every sample of a
 * forward result, adds to grad_verts the gradient of
 *   sum_s gd[s] * depth[s] + gn[s] . normal[s]
 * with respect to the vertex positions: a sample moves along its fixed ray
 * with its triangle's plane (d depth / dX = lambda_X n / n_a for barycentric
 * weight lambda_X of vertex X), and its face normal n = N/|N| with
 * N = (B-A)x(C-A).  The sample set is held fixed (piecewise-smooth
 * derivative; it does not see samples appearing or vanishing).
 *   verts..axis_mask  the same arguments as the forward call (device mesh,
 *             host bbox, w, mask); the mesh must be the one that was sampled.
 *   views     HOST array of 3 views; for each axis in the mask, w, n_samples,
 *             offsets (device) and tri (device) of the forward result (depth
 *             and normal are not read).
 *   grad_depth, grad_normal  HOST arrays of 3 device pointers, f32 [n] and
 *             f32 [n][3] per axis, or NULL (the array or an entry) for zero.
 *   grad_verts device f32 [n_verts][3]; accumulated with +=, not cleared.
 * Sums use float atomics, so the last bits vary from run to run.  Triangle
 * ids outside [0, n_tris) in a view are ignored.  No host synchronisation.
 */
ldni_status ldni_backward(const float *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                          const float bbox[6], int32_t w, uint32_t axis_mask,
                          const ldni_axis_view views[3], const float *const grad_depth[3],
                          const float *const grad_normal[3], float *grad_verts, void *hip_stream);

/*
 * ldni_backward_noalloc -- ldni_backward for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The same arguments, result and errors
 * as ldni_backward, computed by the same kernels; the per-triangle partial
 * sums live in a fixed scratch array of the library (18 floats per triangle
 * for up to 262,144 triangles, 18 MiB, held on each device the library runs
 * on until the process ends) instead of pool memory, and the call makes no
 * allocation of any kind (no hipMalloc or hipFree, no allocating library
 * routine).  n_tris above 262,144 gives LDNI_ERR_INVALID_ARG.  Every call on
 * one device shares that device's scratch, cleared by a kernel at the start
 * of each call: calls that overlap on one device (different streams or host
 * threads) race and must be ordered by the caller.  No host
 * synchronisation.
 */
ldni_status ldni_backward_noalloc(const float *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                                  const float bbox[6], int32_t w, uint32_t axis_mask,
                                  const ldni_axis_view views[3], const float *const grad_depth[3],
                                  const float *const grad_normal[3], float *grad_verts, void *hip_stream);

/*
 * ldni_boolean -- Boolean operation of two solids given as LDNIs of one axis
 * sampled on the same grid (same box and w), Sec. 4.1 and Fig. 5: in every
 * pixel a solid's samples, read as consecutive (enter, exit) pairs, bound its
 * 1D volumes, and the result keeps the volumes where the operation holds
 *   LDNI_UNION         inside A or inside B,
 *   LDNI_INTERSECTION  inside A and inside B,
 *   LDNI_DIFFERENCE    inside A and not inside B (end points that come from
 *                      B get their normal reversed);
 * then every volume thinner than eps is removed (small interval removal,
 * Sec. 4.1.1; the paper uses eps = 1e-5).
 * Readings fixed here: an unpaired last sample of a pixel (odd count) bounds
 * nothing and is ignored; volumes that touch merge, so the result never
 * holds a zero-thickness gap or sliver (thickness (double)exit -
 * (double)enter must be > 0 and >= eps); an end point at depth d is A's first
 * sample at d if A has one, else B's first sample at d.
 *   a, b    HOST views (ldni_axis_view) of the two inputs: w, n_samples and
 *           device offsets/depth/normal/tri as a sampling result lays them
 *           out (per pixel ascending depth).  Offsets must be a prefix of the
 *           samples (non-decreasing, at most n_samples); the call fails with
 *           LDNI_ERR_INVALID_ARG when the device finds they are not.
 *   op      LDNI_UNION, LDNI_INTERSECTION or LDNI_DIFFERENCE.
 *   eps     finite, >= 0.
 *   axis    0..2: which view of *out holds the result (the others are empty).
 *   out     a new result owned by the caller (ldni_free); samples are copies
 *           of input samples (a B normal negated for the difference), and
 *           tri holds A's triangle id t as t and B's as -1 - t.
 * One host synchronisation (the result size); inputs must stay valid until
 * the work queued on hip_stream has run.
 */
enum { LDNI_UNION = 0, LDNI_INTERSECTION = 1, LDNI_DIFFERENCE = 2 };
ldni_status ldni_boolean(const ldni_axis_view *a, const ldni_axis_view *b, int32_t op, float eps,
                         int32_t axis, void *hip_stream, ldni_result **out);

/*
 * ldni_classify_nodes -- inside/outside of the w x w x w grid nodes where the
 * rays of the three LDNIs of one solid meet (Definition 3; Sec. 5.1, step 1
 * of the contouring algorithm).  Along each of its three rays a node is
 * inside when it lies in one of the ray's volumes (from a sample of odd rank
 * to the next, Sec. 2 after Proposition 1); the node is classified inside
 * when at least two of its three LDNIs say so.
 * Readings fixed here: node (i, j, k) lies at the pixel centres
 * (c_x[i], c_y[j], c_z[k]) (the Centres convention above) and its depth on
 * the a-LDNI is f32(c_a - lo_a) in float64, the depth a sample exactly there
 * would get; along a ray it is inside when an odd number of the ray's
 * samples have depth <= its depth (half-open volumes [enter, exit); an
 * unpaired last sample of an odd count is ignored).
 *   views   HOST array of the x-, y- and z-LDNI views (ldni_result_axis
 *           order), one w in 1..8192; offsets and depth are read (depth ascending per
 *           pixel, as sampled); offsets must be a prefix of the samples
 *           (non-decreasing, at most n_samples), else LDNI_ERR_INVALID_ARG
 *           (found on the device; bits are then unspecified).
 *   bbox    HOST f32 box the views were sampled with (as ldni_sample).
 *   bits    device u32 [n_words], caller-owned, fully written: nb^3 bricks
 *           of 32 x 32 x 32 nodes, nb = ceil(w/32); brick (i/32, j/32, k/32)
 *           starts at word ((k/32 * nb + j/32) * nb + i/32) * 1024; inside a
 *           brick word (k%32)*32 + (j%32) holds nodes i/32*32 .. +31 of row
 *           (j, k), node i in bit i%32.  Bits of nodes beyond w are zero.
 *   n_words at least ldni_node_words(w).
 *   stats   HOST u64 [2] or NULL: nodes inside, and nodes whose three
 *           votes are not all equal (the disagreements the vote repairs).
 * Workspace: about 3 w^3 / 32 bytes (w = 2048: 0.8 GB) of span codes from
 * the stream-ordered pool, kept for reuse like the other calls' buffers.
 * One host synchronisation (the totals and the status).
 */
ldni_status ldni_classify_nodes(const ldni_axis_view views[3], const float bbox[6], uint32_t *bits,
                                uint64_t n_words, uint64_t stats[2], void *hip_stream);

/* Words of the bit volume of ldni_classify_nodes at resolution w (1..8192). */
ldni_status ldni_node_words(int32_t w, uint64_t *n_words);

/*
 * ldni_offset -- offset of a solid given by its three LDNIs by a distance r
 * (Sec. 4.2): the Minkowski sum with a sphere of radius r, approximated by
 * uniting the solid with a sphere centred at every sample of its LDNIs, each
 * sphere sampled on the same grid (r > 0); an inner offset (r < 0) subtracts
 * spheres of radius |r| instead.  The Boolean operations are those of Sec.
 * 4.1 with the small interval removal of Sec. 4.1.1.
 * Readings fixed here: the spheres of all samples of the three LDNIs are
 * applied at once; the centre of a sample of the a-LDNI at pixel (i, j) is
 * (lo_a + depth, c_u[i], c_v[j]) in float64 (placed by axis); a sphere hits
 * a ray when rho^2 < r^2 (float64, rho the distance of the centre from the
 * ray), at centre -/+ sqrt(r^2 - rho^2), depths rounded to float32, normal
 * (x - centre)/|r| in float64 rounded to float32 (negated for r < 0); per
 * ray, events of equal float32 depth form one group, the solid's state after
 * a group is the parity of its (paired) samples so far, the spheres' state is
 * whether one is entered and not left; a group that changes the result
 * contributes its first event: the solid's samples by index, then spheres by
 * generating sample, an enter before its exit; volumes with (double)exit -
 * (double)enter <= 0 or < eps are removed.  Generating samples are numbered
 * over the x-, y-, z-view in storage order; a result sample from the sphere
 * of sample g has tri = -1 - g, one from the solid keeps its id.
 *   views   HOST array of the x-, y- and z-LDNI (ldni_result_axis order), one
 *           w; offsets must be a prefix of the samples (else
 *           LDNI_ERR_INVALID_ARG, found on the device); fewer than 2^30
 *           samples in all.
 *   bbox    HOST f32 box the views were sampled with.
 *   r       finite, not zero (world units).
 *   eps     finite, >= 0 (the paper uses 1e-5).
 *   out     a new three-axis result owned by the caller (ldni_free).
 * A ray may meet any number of events (its paired samples plus two per
 * sphere that hits it) and have any number of end points: events are swept
 * in depth windows of 1024, a group of equal float32 depth too large for a
 * window is taken whole by its sums, and end points are passed to the small
 * volume removal in batches of 512.  Fewer than 2^32 sphere hits over all
 * rays and result samples per axis (else LDNI_ERR_OVERFLOW).  Two host
 * synchronisations (the size of the per-ray sphere lists, the result
 * size).
 */
ldni_status ldni_offset(const ldni_axis_view views[3], const float bbox[6], float r, float eps,
                        void *hip_stream, ldni_result **out);

/* Largest per-pixel count of each axis of a plan (after begin). */
ldni_status ldni_plan_max_layers(const ldni_plan *plan, uint32_t max_layers[3]);

/* Status name ("LDNI_OK", ...), never NULL.  The statuses enforce the input
 * contract of Sec. 2: triangles of a polygonal mesh whose indices name
 * vertices (Remark 2), finite coordinates, and the limits above; a closed,
 * non-self-intersecting mesh (Definition 4) is assumed, not checked. */
const char *ldni_status_string(ldni_status s);

/* Thread-local detail of the last error ("" if none). */
const char *ldni_last_error(void);

/* Tile shape of the sampling kernels (pixels per tile along u and v).
 * tw*th <= 1024, 8 <= tw <= 256, 1 <= th <= 64; or 0, 0 (the default): chosen
 * per call from the triangles per pixel (8x8 from 0.75, 16x16 from 0.02,
 * else 32x32).  Process-wide.  Results do not depend on it. */
ldni_status ldni_set_tile_shape(int32_t tw, int32_t th);

/*
 * Batched sampling -- many meshes, each with its own resolution, box and
 * tile shape, sampled by one captured HIP graph (the same definitions as
 * ldni_sample, applied mesh by mesh; results are bit-identical to separate
 * ldni_sample calls).  A batch keeps the mesh pointers: a run samples the
 * current contents of the same device buffers.
 */
typedef struct {
  const float *verts;   /* device f32 [n_verts][3] */
  int64_t n_verts;
  const int32_t *tris;  /* device i32 [n_tris][3] */
  int64_t n_tris;
  float bbox[6];        /* xlo, ylo, zlo, xhi, yhi, zhi */
  int32_t w;            /* 1..16384 */
  int32_t tile_w, tile_h; /* tile shape for this mesh; 0, 0 = the process default */
} ldni_mesh_desc;

typedef struct ldni_batch ldni_batch; /* opaque; owns its device memory and graph */

/*
 * ldni_batch_create -- validate the descriptors (host array of n_meshes >= 1;
 * the same argument rules as ldni_sample for each), allocate the batch's
 * workspace, capture the whole pipeline (setup, binning, count, segmented
 * scan, placement, write) into a HIP graph on a private stream, and run it
 * once on hip_stream, sizing the tile-list and output buffers.  Device
 * memory is held until ldni_batch_free.  Errors as ldni_sample; on error
 * *out is NULL.
 */
ldni_status ldni_batch_create(int32_t n_meshes, const ldni_mesh_desc *meshes, uint32_t axis_mask,
                              void *hip_stream, ldni_batch **out);

/* Replay the batch's graph on hip_stream and wait for it (one host
 * synchronisation); if the meshes now need larger tile lists or outputs,
 * the buffers grow, the graph is captured again and replayed.  Views from
 * before are invalid afterwards. */
ldni_status ldni_batch_run(ldni_batch *b, void *hip_stream);

/* View of one mesh's axis (0..2) after the last run (empty for axes not in
 * the mask); borrowed, valid until the next run or ldni_batch_free. */
ldni_status ldni_batch_axis(const ldni_batch *b, int32_t mesh, int axis, ldni_axis_view *view);

void ldni_batch_free(ldni_batch *b); /* NULL-safe; synchronous */

/* ldni_batch_create under the name of the batched entry point: Definitions
 * 1-3 applied mesh by mesh, every mesh's geometry sent to the device once
 * and kept (as Sec. 3 keeps it in a display list).  The results come as one
 * ldni_batch handle, not one ldni_result per mesh: ldni_batch_axis gives
 * each mesh's views, valid until the next run or ldni_batch_free. */
ldni_status ldni_sample_batch(int32_t n_meshes, const ldni_mesh_desc *meshes, uint32_t axis_mask,
                              void *hip_stream, ldni_batch **out);

/*
 * Kernel timing (tracing support, not part of the paper's method).
 * ldni_profile_enable(1) starts recording a pair of HIP events around every
 * kernel the library launches from the calling process (on the stream the
 * kernel runs on); ldni_profile_enable(0) stops.  Enabling clears earlier
 * records.  ldni_profile_read waits for the recorded events, then writes up
 * to max entries (one per kernel name, in first-launch order) and sets *n to
 * the number of distinct kernels; names are static strings.
 */
typedef struct {
  const char *name;
  uint64_t launches;
  double total_ms;
} ldni_kernel_stat;

ldni_status ldni_profile_enable(int enable);
ldni_status ldni_profile_read(ldni_kernel_stat *stats, int32_t max, int32_t *n);


#ifdef __cplusplus
}
#endif
#endif /* LDNI_H */
