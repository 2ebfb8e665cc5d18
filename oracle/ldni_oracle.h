/*
 * ldni_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU oracle for Layered Depth-Normal Image (LDNI) sampling
 * (Wang & Chen, "Layered Depth-Normal Images: a Sparse Implicit
 * Representation of Solid Models").  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it; the product library never
 * links, calls or includes it, and it shares no code with the HIP path.
 *
 * What it computes (Sec. 2, Definitions 1-3): for one axis a and a w x w grid
 * of rays through pixel centres (Sec. 3, "centre of pixel"), the sorted list
 * of every intersection of the ray with the mesh triangles, excluding faces
 * parallel to the ray (the note after Definition 1), each paired with the unit
 * normal of the hit face (Sec. 3, "accurate surface normal sampling").
 *
 * Readings fixed here (the paper leaves them open):
 *   frame     a=x -> (u,v)=(y,z); a=y -> (z,x); a=z -> (x,y); p = j*w + i.
 *   centres   c_u[i] = f32(f64(lo_u) + (f64(i) + 0.5) * h_u),
 *             h_u = (f64(hi_u) - f64(lo_u)) / w.
 *   coverage  vertices translated into the ray frame in f32; edge functions
 *             E_XY = X'_u*Y'_v - X'_v*Y'_u in f64 (both products exact, so the
 *             sign is exact); a zero E is resolved by perturbing the ray to
 *             (+eps, +eps^2): sign(X'_v - Y'_v), then sign(Y'_u - X'_u).
 *             Hit iff the three signs are equal and non-zero.
 *   depth     den = (E_AB + E_BC) + E_CA,
 *             z = A_a + (E_CA*(B_a - A_a) + E_AB*(C_a - A_a)) / den,
 *             depth = f32(z - lo_a), a zero depth stored as +0.
 *   normal    N = (B-A) x (C-A) in f64, n = f32(N / sqrt((Nx^2+Ny^2)+Nz^2)),
 *             outward (never flipped toward the viewer).
 *   order     per pixel by depth (f32 compare), ties by triangle id.
 *   layout    offsets[w*w+1] exclusive prefix sums (u32), then depth[n],
 *             normal[n][3], tri[n].
 */
#ifndef LDNI_ORACLE_H
#define LDNI_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* one axis of an oracle LDNI; arrays are malloc'd by the oracle */
typedef struct {
  int32_t w;
  uint64_t n;          /* number of samples */
  uint32_t *offsets;   /* [w*w+1] */
  float *depth;        /* [n] */
  float *normal;       /* [n][3] */
  int32_t *tri;        /* [n] */
} oracle_axis;

/* float64 variant (no f32 rounding anywhere), used for finite differences */
typedef struct {
  int32_t w;
  uint64_t n;
  uint32_t *offsets;   /* [w*w+1] */
  double *depth;       /* [n] */
  double *normal;      /* [n][3] */
  int32_t *tri;        /* [n] */
} oracle_axis64;

/* return codes */
#define ORACLE_OK 0
#define ORACLE_ERR_ARG 1
#define ORACLE_ERR_INDEX 2
#define ORACLE_ERR_NOMEM 3
#define ORACLE_ERR_OVERFLOW 4
#define ORACLE_ERR_NONFINITE 6

/*
 * Sample one axis (0=x, 1=y, 2=z).  verts f32 [nv][3], tris i32 [nt][3],
 * bbox = {xlo,ylo,zlo,xhi,yhi,zhi}.  brute=1 tests every (pixel, triangle)
 * pair; brute=0 tests only pixels in a conservative rectangle around each
 * triangle's projection (same result).  Only pixels with i0<=i<i1, j0<=j<j1
 * are sampled (others get no samples); pass 0,w,0,w for the whole image.
 * nthreads<=0 uses every online core.
 */
int oracle_sample_axis(const float *verts, int64_t nv, const int32_t *tris, int64_t nt,
                       const double bbox[6], int32_t w, int axis, int brute, int nthreads,
                       int32_t i0, int32_t i1, int32_t j0, int32_t j1, oracle_axis *out);
void oracle_axis_free(oracle_axis *a);

/* Same definition evaluated entirely in float64 (translation, edge functions,
 * depth, normal), for central finite differences.  Culled mode only. */
int oracle_sample_axis_f64(const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                           const double bbox[6], int32_t w, int axis,
                           int32_t i0, int32_t i1, int32_t j0, int32_t j1, oracle_axis64 *out);
void oracle_axis64_free(oracle_axis64 *a);

/*
 * Analytic gradient of L = sum_s gd[s]*depth[s] + gn[s].normal[s] over the
 * samples of one axis, with respect to the vertex positions, accumulated in
 * float64 into grad[nv][3].  offsets/tri describe the samples (as produced by
 * oracle_sample_axis); gd or gn may be NULL (zero).
 */
int oracle_backward_axis(const float *verts, int64_t nv, const int32_t *tris, int64_t nt,
                         const double bbox[6], int32_t w, int axis,
                         const uint32_t *offsets, const int32_t *tri, uint64_t n,
                         const float *gd, const float *gn, double *grad);

/* pixel-centre coordinates of one axis: cu[w], cv[w] */
int oracle_pixel_centres(const double bbox[6], int32_t w, int axis, float *cu, float *cv);

#ifdef __cplusplus
}
#endif
#endif
