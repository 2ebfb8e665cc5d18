/*
 * ldni_oracle.c -- TEST INFRASTRUCTURE ONLY: the plain CPU oracle for LDNI
 * sampling.  It is loaded by the tests, the smoke check and the benchmark's
 * CPU-baseline leg, never by the product library, and shares no code with the
 * HIP path.  Build: gcc -O2 -ffp-contract=off -fno-fast-math (no FMA, no
 * x87, IEEE double, denormals kept).
 *
 * Each function states the passage of the paper it follows; the readings
 * taken where the paper is silent are listed in ldni_oracle.h.
 */
#include "ldni_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------------ */
/* frame: the axis a and the two image axes (u, v), cyclic                    */
/* ------------------------------------------------------------------------ */
static void axis_frame(int a, int *u, int *v) {
  /* a=x -> (y,z), a=y -> (z,x), a=z -> (x,y) */
  *u = (a + 1) % 3;
  *v = (a + 2) % 3;
}

/* Pixel centres (Sec. 3: coordinates of a pixel are taken at its centre):
 * c[i] = f32(lo + (i + 0.5) * h), h = (hi - lo) / w, all in f64, one final
 * rounding to f32.  The same formula for every axis, so the three images'
 * rays meet at the nodes of one w^3 grid (Definition 3). */
static void centres_1d(double lo, double hi, int32_t w, float *c) {
  double h = (hi - lo) / (double)w;
  for (int32_t i = 0; i < w; ++i) c[i] = (float)(lo + ((double)i + 0.5) * h);
}

int oracle_pixel_centres(const double bbox[6], int32_t w, int axis, float *cu, float *cv) {
  int u, v;
  if (w < 1 || axis < 0 || axis > 2) return ORACLE_ERR_ARG;
  axis_frame(axis, &u, &v);
  centres_1d(bbox[u], bbox[3 + u], w, cu);
  centres_1d(bbox[v], bbox[3 + v], w, cv);
  return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* exact coverage (the note after Definition 1; Remark 1; Definition 4)     */
/* ------------------------------------------------------------------------ */

/* Sign of the edge function of the directed edge X->Y seen from the ray,
 * where X' and Y' are the vertices translated into the ray frame (f32).
 * E = X'_u*Y'_v - X'_v*Y'_u is evaluated in f64: each product of two f32
 * values is exact in f64, so the rounded difference has the exact sign.
 * E == 0 (the ray meets the edge line) is resolved as if the ray were moved
 * to (+eps, +eps^2): the eps term is X'_v - Y'_v, the eps^2 term Y'_u - X'_u. */
static int edge_sign(float xu, float xv, float yu, float yv, double *e_out) {
  double e = (double)xu * (double)yv - (double)xv * (double)yu;
  *e_out = e;
  if (e > 0.0) return 1;
  if (e < 0.0) return -1;
  if (xv > yv) return 1;
  if (xv < yv) return -1;
  if (yu > xu) return 1;
  if (yu < xu) return -1;
  return 0;
}

/* One ray (pixel centre cu, cv on axis a) against one triangle.  Returns 1 on
 * a hit and writes the canonical f32 depth measured from lo_a. */
static int ray_triangle(const float *A, const float *B, const float *C, int a, int u, int v,
                        float cu, float cv, double lo_a, float *depth) {
  float au = A[u] - cu, av = A[v] - cv;
  float bu = B[u] - cu, bv = B[v] - cv;
  float qu = C[u] - cu, qv = C[v] - cv;
  double e_ab, e_bc, e_ca;
  int s_ab = edge_sign(au, av, bu, bv, &e_ab);
  int s_bc = edge_sign(bu, bv, qu, qv, &e_bc);
  int s_ca = edge_sign(qu, qv, au, av, &e_ca);
  if (s_ab == 0 || s_ab != s_bc || s_bc != s_ca) return 0;
  /* barycentric interpolation of the axis coordinate: the weight of B is
   * E_CA/den, of C is E_AB/den (areas opposite each vertex) */
  double den = (e_ab + e_bc) + e_ca;
  double num = e_ca * ((double)B[a] - (double)A[a]) + e_ab * ((double)C[a] - (double)A[a]);
  double z = (double)A[a] + num / den;
  float d = (float)(z - lo_a);
  if (d == 0.0f) d = 0.0f; /* store +0 */
  *depth = d;
  return 1;
}

/* Unit face normal (Sec. 3, accurate normal sampling: the normal of the face
 * the sample lies on), outward for a counter-clockwise-outward mesh. */
static void face_normal(const float *A, const float *B, const float *C, float n[3]) {
  double e1x = (double)B[0] - (double)A[0], e1y = (double)B[1] - (double)A[1],
         e1z = (double)B[2] - (double)A[2];
  double e2x = (double)C[0] - (double)A[0], e2y = (double)C[1] - (double)A[1],
         e2z = (double)C[2] - (double)A[2];
  double nx = e1y * e2z - e1z * e2y;
  double ny = e1z * e2x - e1x * e2z;
  double nz = e1x * e2y - e1y * e2x;
  double len = sqrt((nx * nx + ny * ny) + nz * nz);
  if (len > 0.0) {
    n[0] = (float)(nx / len);
    n[1] = (float)(ny / len);
    n[2] = (float)(nz / len);
  } else {
    n[0] = n[1] = n[2] = 0.0f;
  }
}

/* ------------------------------------------------------------------------ */
/* candidate pixels of a triangle                                             */
/* ------------------------------------------------------------------------ */

/* first index k in [0,w) with c[k] >= x (w if none); c is non-decreasing */
static int32_t first_ge(const float *c, int32_t w, double x) {
  int32_t lo = 0, hi = w;
  while (lo < hi) {
    int32_t mid = lo + (hi - lo) / 2;
    if ((double)c[mid] >= x) hi = mid; else lo = mid + 1;
  }
  return lo;
}

/* last index k in [0,w) with c[k] <= x (-1 if none) */
static int32_t last_le(const float *c, int32_t w, double x) {
  int32_t lo = 0, hi = w;
  while (lo < hi) {
    int32_t mid = lo + (hi - lo) / 2;
    if ((double)c[mid] > x) hi = mid; else lo = mid + 1;
  }
  return lo - 1;
}

/* ------------------------------------------------------------------------ */
/* the sampler                                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
  const float *verts;
  const int32_t *tris;
  int64_t nt;
  int32_t w;
  int a, u, v;
  double lo_a;
  const float *cu, *cv;
  int brute;
  int32_t i0, i1;        /* pixel window in i */
  int32_t jb, je;        /* this worker's rows */
  int pass;              /* 0 = count, 1 = fill */
  uint32_t *counts;      /* [w*w], pass 0 */
  const uint32_t *offsets;
  uint32_t *cursor;      /* [w*w], pass 1 */
  float *depth;
  int32_t *tri;
  int overflow;
} worker_t;

static void record(worker_t *k, int64_t p, float d, int32_t t) {
  if (k->pass == 0) {
    if (k->counts[p] == 0xffffffffu) { k->overflow = 1; return; }
    k->counts[p] += 1;
  } else {
    uint64_t slot = (uint64_t)k->offsets[p] + k->cursor[p];
    k->cursor[p] += 1;
    k->depth[slot] = d;
    k->tri[slot] = t;
  }
}

static void *worker_run(void *arg) {
  worker_t *k = (worker_t *)arg;
  const int32_t w = k->w;
  if (k->brute) {
    for (int32_t j = k->jb; j < k->je; ++j)
      for (int32_t i = k->i0; i < k->i1; ++i)
        for (int64_t t = 0; t < k->nt; ++t) {
          const int32_t *f = k->tris + 3 * t;
          float d;
          if (ray_triangle(k->verts + 3 * (int64_t)f[0], k->verts + 3 * (int64_t)f[1],
                           k->verts + 3 * (int64_t)f[2], k->a, k->u, k->v, k->cu[i], k->cv[j],
                           k->lo_a, &d))
            record(k, (int64_t)j * w + i, d, (int32_t)t);
        }
    return NULL;
  }
  for (int64_t t = 0; t < k->nt; ++t) {
    const int32_t *f = k->tris + 3 * t;
    const float *A = k->verts + 3 * (int64_t)f[0];
    const float *B = k->verts + 3 * (int64_t)f[1];
    const float *C = k->verts + 3 * (int64_t)f[2];
    /* a hit needs min <= centre < max in both image coordinates; take the
     * pixels whose centres lie in the closed projected bounding rectangle */
    double umin = fmin(fmin(A[k->u], B[k->u]), C[k->u]);
    double umax = fmax(fmax(A[k->u], B[k->u]), C[k->u]);
    double vmin = fmin(fmin(A[k->v], B[k->v]), C[k->v]);
    double vmax = fmax(fmax(A[k->v], B[k->v]), C[k->v]);
    int32_t ib = first_ge(k->cu, w, umin), ie = last_le(k->cu, w, umax);
    int32_t jb = first_ge(k->cv, w, vmin), je = last_le(k->cv, w, vmax);
    if (ib < k->i0) ib = k->i0;
    if (ie > k->i1 - 1) ie = k->i1 - 1;
    if (jb < k->jb) jb = k->jb;
    if (je > k->je - 1) je = k->je - 1;
    for (int32_t j = jb; j <= je; ++j)
      for (int32_t i = ib; i <= ie; ++i) {
        float d;
        if (ray_triangle(A, B, C, k->a, k->u, k->v, k->cu[i], k->cv[j], k->lo_a, &d))
          record(k, (int64_t)j * w + i, d, (int32_t)t);
      }
  }
  return NULL;
}

static int run_workers(worker_t *base, int nthreads) {
  int32_t rows = base->je - base->jb;
  if (nthreads > rows) nthreads = rows > 0 ? rows : 1;
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  worker_t *ks = (worker_t *)calloc((size_t)nthreads, sizeof(worker_t));
  if (!th || !ks) { free(th); free(ks); return ORACLE_ERR_NOMEM; }
  int overflow = 0;
  for (int q = 0; q < nthreads; ++q) {
    ks[q] = *base;
    ks[q].jb = base->jb + (int32_t)((int64_t)rows * q / nthreads);
    ks[q].je = base->jb + (int32_t)((int64_t)rows * (q + 1) / nthreads);
    if (nthreads == 1) worker_run(&ks[q]);
    else pthread_create(&th[q], NULL, worker_run, &ks[q]);
  }
  for (int q = 0; q < nthreads; ++q) {
    if (nthreads > 1) pthread_join(th[q], NULL);
    overflow |= ks[q].overflow;
  }
  free(th);
  free(ks);
  return overflow ? ORACLE_ERR_OVERFLOW : ORACLE_OK;
}

/* sort one pixel's samples by (depth, triangle id): insertion sort */
static void sort_pixel(float *d, int32_t *t, uint32_t n) {
  for (uint32_t x = 1; x < n; ++x) {
    float dk = d[x];
    int32_t tk = t[x];
    uint32_t y = x;
    while (y > 0 && (d[y - 1] > dk || (d[y - 1] == dk && t[y - 1] > tk))) {
      d[y] = d[y - 1];
      t[y] = t[y - 1];
      --y;
    }
    d[y] = dk;
    t[y] = tk;
  }
}

static int check_inputs(const float *verts, int64_t nv, const int32_t *tris, int64_t nt,
                        const double bbox[6], int32_t w, int axis) {
  if (w < 1 || w > 16384 || axis < 0 || axis > 2 || nv < 0 || nt < 0) return ORACLE_ERR_ARG;
  if ((nv > 0 && !verts) || (nt > 0 && !tris)) return ORACLE_ERR_ARG;
  for (int d = 0; d < 3; ++d)
    if (!isfinite(bbox[d]) || !isfinite(bbox[3 + d]) || !(bbox[d] < bbox[3 + d]))
      return ORACLE_ERR_ARG;
  for (int64_t t = 0; t < 3 * nt; ++t)
    if (tris[t] < 0 || (int64_t)tris[t] >= nv) return ORACLE_ERR_INDEX;
  for (int64_t t = 0; t < 3 * nt; ++t) {
    const float *p = verts + 3 * (int64_t)tris[t];
    if (!isfinite(p[0]) || !isfinite(p[1]) || !isfinite(p[2])) return ORACLE_ERR_NONFINITE;
  }
  return ORACLE_OK;
}

int oracle_sample_axis(const float *verts, int64_t nv, const int32_t *tris, int64_t nt,
                       const double bbox[6], int32_t w, int axis, int brute, int nthreads,
                       int32_t i0, int32_t i1, int32_t j0, int32_t j1, oracle_axis *out) {
  memset(out, 0, sizeof(*out));
  int rc = check_inputs(verts, nv, tris, nt, bbox, w, axis);
  if (rc) return rc;
  if (i0 < 0) i0 = 0;
  if (j0 < 0) j0 = 0;
  if (i1 > w) i1 = w;
  if (j1 > w) j1 = w;
  if (nthreads <= 0) nthreads = (int)sysconf(_SC_NPROCESSORS_ONLN);
  if (nthreads < 1) nthreads = 1;

  const uint64_t npix = (uint64_t)w * (uint64_t)w;
  float *cu = (float *)malloc(sizeof(float) * (size_t)w);
  float *cv = (float *)malloc(sizeof(float) * (size_t)w);
  uint32_t *counts = (uint32_t *)calloc((size_t)npix, sizeof(uint32_t));
  uint32_t *offsets = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(npix + 1));
  if (!cu || !cv || !counts || !offsets) {
    free(cu); free(cv); free(counts); free(offsets);
    return ORACLE_ERR_NOMEM;
  }
  oracle_pixel_centres(bbox, w, axis, cu, cv);

  worker_t base;
  memset(&base, 0, sizeof(base));
  base.verts = verts;
  base.tris = tris;
  base.nt = nt;
  base.w = w;
  base.a = axis;
  axis_frame(axis, &base.u, &base.v);
  base.lo_a = bbox[axis];
  base.cu = cu;
  base.cv = cv;
  base.brute = brute;
  base.i0 = i0;
  base.i1 = i1;
  base.jb = j0;
  base.je = j1 > j0 ? j1 : j0;
  base.i1 = i1 > i0 ? i1 : i0;

  /* pass 1: count the hits of every pixel */
  base.pass = 0;
  base.counts = counts;
  rc = run_workers(&base, nthreads);
  if (rc) { free(cu); free(cv); free(counts); free(offsets); return rc; }

  /* exclusive prefix sum -> offsets; totals must fit in u32 */
  uint64_t acc = 0;
  for (uint64_t p = 0; p < npix; ++p) {
    offsets[p] = (uint32_t)acc;
    acc += counts[p];
    if (acc > 0xffffffffull) { free(cu); free(cv); free(counts); free(offsets); return ORACLE_ERR_OVERFLOW; }
  }
  offsets[npix] = (uint32_t)acc;
  const uint64_t n = acc;

  float *depth = (float *)malloc(sizeof(float) * (size_t)(n ? n : 1));
  int32_t *tri = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
  float *normal = (float *)malloc(sizeof(float) * 3 * (size_t)(n ? n : 1));
  if (!depth || !tri || !normal) {
    free(cu); free(cv); free(counts); free(offsets); free(depth); free(tri); free(normal);
    return ORACLE_ERR_NOMEM;
  }

  /* pass 2: the same tests again, each hit stored in its pixel's next slot */
  memset(counts, 0, sizeof(uint32_t) * (size_t)npix);
  base.pass = 1;
  base.offsets = offsets;
  base.cursor = counts;
  base.depth = depth;
  base.tri = tri;
  rc = run_workers(&base, nthreads);

  /* Definition 1: each pixel's depths in ascending order */
  for (uint64_t p = 0; p < npix; ++p)
    sort_pixel(depth + offsets[p], tri + offsets[p], offsets[p + 1] - offsets[p]);

  /* the normal of the hit face */
  for (uint64_t s = 0; s < n; ++s) {
    const int32_t *f = tris + 3 * (int64_t)tri[s];
    face_normal(verts + 3 * (int64_t)f[0], verts + 3 * (int64_t)f[1], verts + 3 * (int64_t)f[2],
                normal + 3 * s);
  }
  free(cu);
  free(cv);
  free(counts);
  out->w = w;
  out->n = n;
  out->offsets = offsets;
  out->depth = depth;
  out->normal = normal;
  out->tri = tri;
  return rc;
}

void oracle_axis_free(oracle_axis *a) {
  if (!a) return;
  free(a->offsets);
  free(a->depth);
  free(a->normal);
  free(a->tri);
  memset(a, 0, sizeof(*a));
}

/* ------------------------------------------------------------------------ */
/* float64 evaluation, for finite differences                                */
/* ------------------------------------------------------------------------ */
static int edge_sign64(double xu, double xv, double yu, double yv, double *e_out) {
  double e = xu * yv - xv * yu;
  *e_out = e;
  if (e > 0.0) return 1;
  if (e < 0.0) return -1;
  if (xv > yv) return 1;
  if (xv < yv) return -1;
  if (yu > xu) return 1;
  if (yu < xu) return -1;
  return 0;
}

static int ray_triangle64(const double *A, const double *B, const double *C, int a, int u, int v,
                          double cu, double cv, double lo_a, double *depth) {
  double au = A[u] - cu, av = A[v] - cv, bu = B[u] - cu, bv = B[v] - cv;
  double qu = C[u] - cu, qv = C[v] - cv;
  double e_ab, e_bc, e_ca;
  int s_ab = edge_sign64(au, av, bu, bv, &e_ab);
  int s_bc = edge_sign64(bu, bv, qu, qv, &e_bc);
  int s_ca = edge_sign64(qu, qv, au, av, &e_ca);
  if (s_ab == 0 || s_ab != s_bc || s_bc != s_ca) return 0;
  double den = (e_ab + e_bc) + e_ca;
  double num = e_ca * (B[a] - A[a]) + e_ab * (C[a] - A[a]);
  *depth = (A[a] + num / den) - lo_a;
  return 1;
}

static void face_normal64(const double *A, const double *B, const double *C, double n[3]) {
  double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
  double e2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
  double nx = e1[1] * e2[2] - e1[2] * e2[1];
  double ny = e1[2] * e2[0] - e1[0] * e2[2];
  double nz = e1[0] * e2[1] - e1[1] * e2[0];
  double len = sqrt((nx * nx + ny * ny) + nz * nz);
  if (len > 0.0) { n[0] = nx / len; n[1] = ny / len; n[2] = nz / len; }
  else { n[0] = n[1] = n[2] = 0.0; }
}

int oracle_sample_axis_f64(const double *verts, int64_t nv, const int32_t *tris, int64_t nt,
                           const double bbox[6], int32_t w, int axis,
                           int32_t i0, int32_t i1, int32_t j0, int32_t j1, oracle_axis64 *out) {
  memset(out, 0, sizeof(*out));
  if (w < 1 || axis < 0 || axis > 2 || nv < 0 || nt < 0) return ORACLE_ERR_ARG;
  for (int64_t t = 0; t < 3 * nt; ++t)
    if (tris[t] < 0 || (int64_t)tris[t] >= nv) return ORACLE_ERR_INDEX;
  if (i0 < 0) i0 = 0;
  if (j0 < 0) j0 = 0;
  if (i1 > w) i1 = w;
  if (j1 > w) j1 = w;
  int u, v;
  axis_frame(axis, &u, &v);
  const uint64_t npix = (uint64_t)w * (uint64_t)w;
  double hu = (bbox[3 + u] - bbox[u]) / (double)w, hv = (bbox[3 + v] - bbox[v]) / (double)w;
  uint32_t *counts = (uint32_t *)calloc((size_t)npix, sizeof(uint32_t));
  uint32_t *offsets = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(npix + 1));
  if (!counts || !offsets) { free(counts); free(offsets); return ORACLE_ERR_NOMEM; }
  double *dep = NULL, *nrm = NULL;
  int32_t *tri = NULL;
  uint64_t n = 0;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      uint64_t acc = 0;
      for (uint64_t p = 0; p < npix; ++p) { offsets[p] = (uint32_t)acc; acc += counts[p]; }
      offsets[npix] = (uint32_t)acc;
      n = acc;
      dep = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
      nrm = (double *)malloc(sizeof(double) * 3 * (size_t)(n ? n : 1));
      tri = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
      if (!dep || !nrm || !tri) {
        free(counts); free(offsets); free(dep); free(nrm); free(tri);
        return ORACLE_ERR_NOMEM;
      }
      memset(counts, 0, sizeof(uint32_t) * (size_t)npix);
    }
    for (int64_t t = 0; t < nt; ++t) {
      const double *A = verts + 3 * (int64_t)tris[3 * t];
      const double *B = verts + 3 * (int64_t)tris[3 * t + 1];
      const double *C = verts + 3 * (int64_t)tris[3 * t + 2];
      double umin = fmin(fmin(A[u], B[u]), C[u]), umax = fmax(fmax(A[u], B[u]), C[u]);
      double vmin = fmin(fmin(A[v], B[v]), C[v]), vmax = fmax(fmax(A[v], B[v]), C[v]);
      int32_t ib = (int32_t)floor((umin - bbox[u]) / hu - 0.5) - 1;
      int32_t ie = (int32_t)floor((umax - bbox[u]) / hu - 0.5) + 1;
      int32_t jb = (int32_t)floor((vmin - bbox[v]) / hv - 0.5) - 1;
      int32_t je = (int32_t)floor((vmax - bbox[v]) / hv - 0.5) + 1;
      if (ib < i0) ib = i0;
      if (ie > i1 - 1) ie = i1 - 1;
      if (jb < j0) jb = j0;
      if (je > j1 - 1) je = j1 - 1;
      for (int32_t j = jb; j <= je; ++j)
        for (int32_t i = ib; i <= ie; ++i) {
          double cu = bbox[u] + ((double)i + 0.5) * hu;
          double cv = bbox[v] + ((double)j + 0.5) * hv;
          double d;
          if (!ray_triangle64(A, B, C, axis, u, v, cu, cv, bbox[axis], &d)) continue;
          uint64_t p = (uint64_t)j * (uint64_t)w + (uint64_t)i;
          if (pass == 0) { counts[p] += 1; continue; }
          uint64_t slot = (uint64_t)offsets[p] + counts[p]++;
          dep[slot] = d;
          tri[slot] = (int32_t)t;
        }
    }
  }
  /* sort by (depth, tri) and attach normals */
  for (uint64_t p = 0; p < npix; ++p) {
    double *d = dep + offsets[p];
    int32_t *t = tri + offsets[p];
    uint32_t m = offsets[p + 1] - offsets[p];
    for (uint32_t x = 1; x < m; ++x) {
      double dk = d[x];
      int32_t tk = t[x];
      uint32_t y = x;
      while (y > 0 && (d[y - 1] > dk || (d[y - 1] == dk && t[y - 1] > tk))) {
        d[y] = d[y - 1]; t[y] = t[y - 1]; --y;
      }
      d[y] = dk; t[y] = tk;
    }
  }
  for (uint64_t s = 0; s < n; ++s) {
    const int32_t *f = tris + 3 * (int64_t)tri[s];
    face_normal64(verts + 3 * (int64_t)f[0], verts + 3 * (int64_t)f[1], verts + 3 * (int64_t)f[2],
                  nrm + 3 * s);
  }
  free(counts);
  out->w = w;
  out->n = n;
  out->offsets = offsets;
  out->depth = dep;
  out->normal = nrm;
  out->tri = tri;
  return ORACLE_OK;
}

void oracle_axis64_free(oracle_axis64 *a) {
  if (!a) return;
  free(a->offsets);
  free(a->depth);
  free(a->normal);
  free(a->tri);
  memset(a, 0, sizeof(*a));
}

/* ------------------------------------------------------------------------ */
/* analytic gradient (float64)                                                */
/* ------------------------------------------------------------------------ */

/* For a sample on triangle (A,B,C) at pixel centre (cu,cv):
 *   depth: the hit point is the barycentric combination lambda_A A + lambda_B B
 *   + lambda_C C constrained to the fixed ray, so moving vertex X moves the
 *   depth by lambda_X * (n . dX) / n_a  ->  dL/dX += gd * lambda_X * n / n_a;
 *   normal: n = N/|N|, N = (B-A)x(C-A); dL/dN = (gn - n (n.gn)) / |N|, and
 *   dL/dA = (B-C) x dL/dN, dL/dB = (C-A) x dL/dN, dL/dC = (A-B) x dL/dN. */
int oracle_backward_axis(const float *verts, int64_t nv, const int32_t *tris, int64_t nt,
                         const double bbox[6], int32_t w, int axis,
                         const uint32_t *offsets, const int32_t *tri, uint64_t n,
                         const float *gd, const float *gn, double *grad) {
  if (w < 1 || axis < 0 || axis > 2 || nv < 0 || nt < 0) return ORACLE_ERR_ARG;
  int u, v;
  axis_frame(axis, &u, &v);
  const uint64_t npix = (uint64_t)w * (uint64_t)w;
  if (offsets[npix] != n) return ORACLE_ERR_ARG;
  /* the ray positions of the float64 definition (no f32 rounding), the same
   * function that oracle_sample_axis_f64 differentiates */
  double hu = (bbox[3 + u] - bbox[u]) / (double)w, hv = (bbox[3 + v] - bbox[v]) / (double)w;
  int rc = ORACLE_OK;
  for (uint64_t p = 0; p < npix && rc == ORACLE_OK; ++p) {
    int32_t i = (int32_t)(p % (uint64_t)w), j = (int32_t)(p / (uint64_t)w);
    double cu = bbox[u] + ((double)i + 0.5) * hu;
    double cv = bbox[v] + ((double)j + 0.5) * hv;
    for (uint32_t s = offsets[p]; s < offsets[p + 1]; ++s) {
      int32_t t = tri[s];
      if (t < 0 || t >= nt) { rc = ORACLE_ERR_INDEX; break; }
      const int32_t *f = tris + 3 * (int64_t)t;
      double P[3][3];
      for (int q = 0; q < 3; ++q)
        for (int c = 0; c < 3; ++c) P[q][c] = (double)verts[3 * (int64_t)f[q] + c];
      double e1[3], e2[3], N[3];
      for (int c = 0; c < 3; ++c) { e1[c] = P[1][c] - P[0][c]; e2[c] = P[2][c] - P[0][c]; }
      N[0] = e1[1] * e2[2] - e1[2] * e2[1];
      N[1] = e1[2] * e2[0] - e1[0] * e2[2];
      N[2] = e1[0] * e2[1] - e1[1] * e2[0];
      double len = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
      if (!(len > 0.0)) continue;
      double nn[3] = {N[0] / len, N[1] / len, N[2] / len};
      if (gd && gd[s] != 0.0f && nn[axis] != 0.0) {
        /* barycentric weights of the pixel centre in the projected triangle */
        double xu[3], xv[3];
        for (int q = 0; q < 3; ++q) { xu[q] = P[q][u] - cu; xv[q] = P[q][v] - cv; }
        double e_bc = xu[1] * xv[2] - xv[1] * xu[2];
        double e_ca = xu[2] * xv[0] - xv[2] * xu[0];
        double e_ab = xu[0] * xv[1] - xv[0] * xu[1];
        double den = e_ab + e_bc + e_ca;
        double lam[3] = {e_bc / den, e_ca / den, e_ab / den};
        for (int q = 0; q < 3; ++q)
          for (int c = 0; c < 3; ++c)
            grad[3 * (int64_t)f[q] + c] += (double)gd[s] * lam[q] * nn[c] / nn[axis];
      }
      if (gn) {
        double g[3] = {gn[3 * s], gn[3 * s + 1], gn[3 * s + 2]};
        double dot = nn[0] * g[0] + nn[1] * g[1] + nn[2] * g[2];
        double gN[3];
        for (int c = 0; c < 3; ++c) gN[c] = (g[c] - nn[c] * dot) / len;
        /* dL/dX = (edge opposite, in cyclic order) x gN */
        double ed[3][3];
        for (int c = 0; c < 3; ++c) {
          ed[0][c] = P[1][c] - P[2][c]; /* A: B - C */
          ed[1][c] = P[2][c] - P[0][c]; /* B: C - A */
          ed[2][c] = P[0][c] - P[1][c]; /* C: A - B */
        }
        for (int q = 0; q < 3; ++q) {
          double cx = ed[q][1] * gN[2] - ed[q][2] * gN[1];
          double cy = ed[q][2] * gN[0] - ed[q][0] * gN[2];
          double cz = ed[q][0] * gN[1] - ed[q][1] * gN[0];
          grad[3 * (int64_t)f[q] + 0] += cx;
          grad[3 * (int64_t)f[q] + 1] += cy;
          grad[3 * (int64_t)f[q] + 2] += cz;
        }
      }
    }
  }
  return rc;
}
