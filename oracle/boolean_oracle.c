/*
 * boolean_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Boolean operations on two LDNIs of one axis sampled on the same grid
 * (Sec. 4.1 and Fig. 5 of the paper; small interval removal, Sec. 4.1.1),
 * pixel by pixel, in plain C so that whole w = 2048 images finish in
 * seconds.  It restates, step by step and with the same readings, what
 * oracle/boolean.py computes (that module's header lists them):
 *   1. A's samples, read as consecutive pairs, are its segments; B's paired
 *      samples likewise (an unpaired last sample is ignored).
 *   2. Each segment of A is sliced at every sample of B strictly inside it.
 *   3. A slice is inside B when its midpoint lies strictly inside a segment
 *      of B.  Union keeps the slices outside B and adds B's segments;
 *      intersection keeps the slices inside B; difference keeps the slices
 *      outside B.
 *   4. Kept pieces that overlap or touch are merged (sorted by start).
 *   5. Volumes of thickness (double)exit - (double)enter that is zero or
 *      below eps are removed.
 *   6. An end point at depth d is A's first paired sample at d, else B's
 *      first paired sample at d (its normal reversed for the difference);
 *      A's ids stay, B's id t becomes -1 - t.
 * Only the test suite may load it (it is built into the oracle's library);
 * the product library shares no code with it.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  double s, e;
} piece_t;

static int piece_cmp(const void *x, const void *y) {
  const piece_t *a = (const piece_t *)x, *b = (const piece_t *)y;
  if (a->s < b->s) return -1;
  if (a->s > b->s) return 1;
  if (a->e < b->e) return -1;
  if (a->e > b->e) return 1;
  return 0;
}

static int dbl_cmp(const void *x, const void *y) {
  const double a = *(const double *)x, b = *(const double *)y;
  return (a > b) - (a < b);
}

/* The result of one pixel as (solid, index, reversed) triples in depth order
 * (solid 0 = A, 1 = B); returns how many.  Scratch buffers are sized by the
 * caller for na + nb samples. */
static int boolean_pixel(const float *da, int na_all, const float *db, int nb_all, int op, double eps,
                         piece_t *pieces, piece_t *vols, double *cuts, int *out_solid, int *out_index) {
  const int na = na_all / 2 * 2, nb = nb_all / 2 * 2;
  int np = 0;
  /* 2. slice A's segments at B's samples strictly inside them */
  for (int i = 0; i < na; i += 2) {
    const double a0 = da[i], a1 = da[i + 1];
    int nc = 0;
    for (int j = 0; j < nb; ++j) {
      const double z = db[j];
      if (a0 < z && z < a1) cuts[nc++] = z;
    }
    qsort(cuts, (size_t)nc, sizeof(double), dbl_cmp);
    double prev = a0;
    for (int k = 0; k < nc; ++k) {
      if (k > 0 && cuts[k] == cuts[k - 1]) continue; /* equal cuts slice once */
      pieces[np].s = prev;
      pieces[np].e = cuts[k];
      ++np;
      prev = cuts[k];
    }
    pieces[np].s = prev;
    pieces[np].e = a1;
    ++np;
  }
  /* 3. classify the slices against B at their midpoints, select per op */
  int nk = 0;
  for (int k = 0; k < np; ++k) {
    const double mid = 0.5 * (pieces[k].s + pieces[k].e);
    int in_b = 0;
    for (int j = 0; j < nb; j += 2)
      if ((double)db[j] < mid && mid < (double)db[j + 1]) in_b = 1;
    const int keep = (op == 1) ? in_b : !in_b;
    if (keep) vols[nk++] = pieces[k];
  }
  if (op == 0)
    for (int j = 0; j < nb; j += 2) {
      vols[nk].s = db[j];
      vols[nk].e = db[j + 1];
      ++nk;
    }
  /* 4. merge pieces that overlap or touch */
  qsort(vols, (size_t)nk, sizeof(piece_t), piece_cmp);
  int nv = 0;
  for (int k = 0; k < nk; ++k) {
    if (nv > 0 && vols[k].s <= vols[nv - 1].e) {
      if (vols[k].e > vols[nv - 1].e) vols[nv - 1].e = vols[k].e;
    } else {
      vols[nv++] = vols[k];
    }
  }
  /* 5. small interval removal; 6. the samples that supply the end points */
  int n = 0;
  for (int k = 0; k < nv; ++k) {
    const double th = vols[k].e - vols[k].s;
    if (!(th > 0.0 && th >= eps)) continue;
    for (int end = 0; end < 2; ++end) {
      const double z = end ? vols[k].e : vols[k].s;
      int solid = -1, index = -1;
      for (int i = 0; i < na && solid < 0; ++i)
        if ((double)da[i] == z) { solid = 0; index = i; }
      for (int j = 0; j < nb && solid < 0; ++j)
        if ((double)db[j] == z) { solid = 1; index = j; }
      if (solid < 0) return -1; /* an end point that is no sample: cannot happen */
      out_solid[n] = solid;
      out_index[n] = index;
      ++n;
    }
  }
  return n;
}

/* The operation (0 union, 1 intersection, 2 difference) over npix pixels.
 * Inputs in the compact layout (offsets[npix+1], depth, normal[3], tri).
 * Outputs are malloc'd: *out_offsets [npix+1], then *out_n samples of depth,
 * normal, tri; free them with oracle_boolean_free.  Returns 0, or 3 when
 * memory runs out, 5 on an end point that is not a sample. */
int oracle_boolean(int64_t npix, const uint32_t *a_off, const float *a_dep, const float *a_nrm,
                   const int32_t *a_tri, const uint32_t *b_off, const float *b_dep, const float *b_nrm,
                   const int32_t *b_tri, int op, double eps, uint32_t **out_offsets, float **out_depth,
                   float **out_normal, int32_t **out_tri, uint64_t *out_n) {
  *out_offsets = NULL;
  *out_depth = NULL;
  *out_normal = NULL;
  *out_tri = NULL;
  *out_n = 0;
  uint64_t cap = 0;
  uint32_t maxp = 0;
  for (int64_t p = 0; p < npix; ++p) {
    const uint32_t na = a_off[p + 1] - a_off[p], nb = b_off[p + 1] - b_off[p];
    cap += na + nb;
    if (na + nb > maxp) maxp = na + nb;
  }
  uint32_t *off = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(npix + 1));
  float *dep = (float *)malloc(sizeof(float) * (size_t)(cap + 1));
  float *nrm = (float *)malloc(3 * sizeof(float) * (size_t)(cap + 1));
  int32_t *tri = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap + 1));
  const size_t m = (size_t)maxp + 2;
  piece_t *pieces = (piece_t *)malloc(sizeof(piece_t) * m * m);
  piece_t *vols = (piece_t *)malloc(sizeof(piece_t) * m * m);
  double *cuts = (double *)malloc(sizeof(double) * m);
  int *sol = (int *)malloc(sizeof(int) * m);
  int *idx = (int *)malloc(sizeof(int) * m);
  if (!off || !dep || !nrm || !tri || !pieces || !vols || !cuts || !sol || !idx) {
    free(off); free(dep); free(nrm); free(tri); free(pieces); free(vols); free(cuts); free(sol); free(idx);
    return 3;
  }
  uint64_t n = 0;
  off[0] = 0;
  for (int64_t p = 0; p < npix; ++p) {
    const uint32_t a0 = a_off[p], a1 = a_off[p + 1], b0 = b_off[p], b1 = b_off[p + 1];
    const int k = boolean_pixel(a_dep + a0, (int)(a1 - a0), b_dep + b0, (int)(b1 - b0), op, eps, pieces, vols,
                                cuts, sol, idx);
    if (k < 0) {
      free(off); free(dep); free(nrm); free(tri); free(pieces); free(vols); free(cuts); free(sol); free(idx);
      return 5;
    }
    for (int q = 0; q < k; ++q) {
      const int from_b = sol[q] == 1;
      const uint64_t src = (uint64_t)(from_b ? b0 : a0) + (uint64_t)idx[q];
      const float *sn = from_b ? b_nrm + 3 * src : a_nrm + 3 * src;
      const float sign = (from_b && op == 2) ? -1.0f : 1.0f;
      dep[n] = from_b ? b_dep[src] : a_dep[src];
      for (int c = 0; c < 3; ++c) nrm[3 * n + c] = sign * sn[c];
      tri[n] = from_b ? -1 - b_tri[src] : a_tri[src];
      ++n;
    }
    off[p + 1] = (uint32_t)n;
  }
  free(pieces); free(vols); free(cuts); free(sol); free(idx);
  *out_offsets = off;
  *out_depth = dep;
  *out_normal = nrm;
  *out_tri = tri;
  *out_n = n;
  return 0;
}

void oracle_boolean_free(uint32_t *offsets, float *depth, float *normal, int32_t *tri) {
  free(offsets);
  free(depth);
  free(normal);
  free(tri);
}
