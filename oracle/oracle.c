/*
 * FP64 CPU oracle for the EFIE Galerkin impedance-matrix fill with adaptive
 * Green-function tables (S. Yang, D. Su, "Fast Green Function Evaluation for
 * Method of Moment").
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no
 * source with the GPU library.  Everything is written the plain way: one
 * matrix entry at a time as the sum of its four triangle-pair integrals,
 * tables built in the order the paper describes them.
 *
 * Discretisation (the paper cites the method-of-moments literature for it
 * rather than writing it out; Section II-A, Section IV-B):
 *   Z_mn = jk eta/(4 pi) sum_{sigma,tau} s_sigma s_tau l_m l_n
 *            int_p int_q [ (r - v_a).(r' - v_b)/4 - 1/k^2 ] g(|r - r'|) dS' dS
 *                      / (A_p A_q),
 *   g(R) = exp(-jkR)/R (Eq. (1)), time convention exp(+j omega t), RWG basis
 *   functions f = s l/(2A) (r - v) on the two triangles of each edge.
 * Regular (vertex-disjoint) triangle pairs use the product quadrature rule;
 * touching pairs (sharing at least one vertex, including p = q) subtract 1/R
 * and integrate it in closed form ("classical singularity cancellation",
 * Section II-C), then are symmetrised.
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define OR_ETA0 376.730313668 /* free-space wave impedance, ohm */

/* ------------------------------------------------------------------------ */
/* Quadrature rules (symmetric rules of degree 2, 4 and 5).                  */
/* ------------------------------------------------------------------------ */

static void put3(double *b, int i, double l0, double l1, double l2) {
  b[3 * i + 0] = l0;
  b[3 * i + 1] = l1;
  b[3 * i + 2] = l2;
}

int or_quad_rule(int q, double *bary, double *w) {
  if (q == 3) {
    const double a = 2.0 / 3.0, b = 1.0 / 6.0;
    put3(bary, 0, a, b, b);
    put3(bary, 1, b, a, b);
    put3(bary, 2, b, b, a);
    w[0] = w[1] = w[2] = 1.0 / 3.0;
    return 3;
  }
  if (q == 6) {
    /* degree 4: two orbits of three points, closed forms of the weights and
     * coordinates of the classical six-point rule */
    const double s10 = sqrt(10.0);
    const double rt = sqrt(38.0 - 44.0 * sqrt(2.0 / 5.0));
    const double a1 = (8.0 - s10 + rt) / 18.0; /* 0.4459... */
    const double a2 = (8.0 - s10 - rt) / 18.0; /* 0.0915... */
    const double wr = sqrt(213125.0 - 53320.0 * s10);
    const double w1 = (620.0 + wr) / 3720.0;
    const double w2 = (620.0 - wr) / 3720.0;
    const double b1 = 1.0 - 2.0 * a1, b2 = 1.0 - 2.0 * a2;
    put3(bary, 0, b1, a1, a1);
    put3(bary, 1, a1, b1, a1);
    put3(bary, 2, a1, a1, b1);
    put3(bary, 3, b2, a2, a2);
    put3(bary, 4, a2, b2, a2);
    put3(bary, 5, a2, a2, b2);
    w[0] = w[1] = w[2] = w1;
    w[3] = w[4] = w[5] = w2;
    return 6;
  }
  if (q == 7) {
    /* degree 5 (Radon) */
    const double s15 = sqrt(15.0);
    const double a = (6.0 - s15) / 21.0, b = (9.0 + 2.0 * s15) / 21.0;
    const double c = (6.0 + s15) / 21.0, d = (9.0 - 2.0 * s15) / 21.0;
    put3(bary, 0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0);
    put3(bary, 1, b, a, a);
    put3(bary, 2, a, b, a);
    put3(bary, 3, a, a, b);
    put3(bary, 4, d, c, c);
    put3(bary, 5, c, d, c);
    put3(bary, 6, c, c, d);
    w[0] = 9.0 / 40.0;
    w[1] = w[2] = w[3] = (155.0 - s15) / 1200.0;
    w[4] = w[5] = w[6] = (155.0 + s15) / 1200.0;
    return 7;
  }
  return -1;
}

/* ------------------------------------------------------------------------ */
/* RWG unknowns.                                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
  int lo, hi, t, a, up; /* up = 1 if the triangle runs lo -> hi */
} halfedge;

static int he_cmp(const void *x, const void *y) {
  const halfedge *u = (const halfedge *)x, *v = (const halfedge *)y;
  if (u->lo != v->lo) return u->lo < v->lo ? -1 : 1;
  if (u->hi != v->hi) return u->hi < v->hi ? -1 : 1;
  if (u->t != v->t) return u->t < v->t ? -1 : 1;
  return u->a - v->a;
}

typedef struct {
  long key; /* first appearance: 3*t + a */
  int g;    /* group start in the sorted half-edge list */
} firstseen;

static int fs_cmp(const void *x, const void *y) {
  const firstseen *u = (const firstseen *)x, *v = (const firstseen *)y;
  return (u->key > v->key) - (u->key < v->key);
}

int or_rwg(int nv, int nt, const int32_t *tri, int32_t *n_edges, int32_t *edges) {
  if (nv <= 0 || nt <= 0 || !tri || !n_edges || !edges) return -1;
  halfedge *h = (halfedge *)malloc(sizeof(halfedge) * 3 * (size_t)nt);
  firstseen *fs = (firstseen *)malloc(sizeof(firstseen) * 3 * (size_t)nt);
  if (!h || !fs) {
    free(h);
    free(fs);
    return -4;
  }
  int rc = 0;
  for (int t = 0; t < nt && rc == 0; ++t) {
    const int32_t *v = tri + 3 * t;
    for (int c = 0; c < 3; ++c)
      if (v[c] < 0 || v[c] >= nv) rc = -2;
    if (v[0] == v[1] || v[1] == v[2] || v[2] == v[0]) rc = -2;
    for (int a = 0; a < 3 && rc == 0; ++a) {
      /* local edge a is opposite vertex a and runs v[a+1] -> v[a+2] */
      int from = v[(a + 1) % 3], to = v[(a + 2) % 3];
      halfedge *e = &h[3 * t + a];
      e->lo = from < to ? from : to;
      e->hi = from < to ? to : from;
      e->t = t;
      e->a = a;
      e->up = (from == e->lo);
    }
  }
  int ne = 0;
  if (rc == 0) {
    qsort(h, 3 * (size_t)nt, sizeof(halfedge), he_cmp);
    int nfs = 0;
    for (int i = 0; i < 3 * nt && rc == 0;) {
      int j = i;
      while (j < 3 * nt && h[j].lo == h[i].lo && h[j].hi == h[i].hi) ++j;
      int cnt = j - i;
      if (cnt > 2) rc = -2; /* non-manifold edge */
      if (cnt == 2) {
        if (h[i].up == h[i + 1].up) rc = -2; /* inconsistent orientation */
        long k0 = 3L * h[i].t + h[i].a, k1 = 3L * h[i + 1].t + h[i + 1].a;
        fs[nfs].key = k0 < k1 ? k0 : k1;
        fs[nfs].g = i;
        ++nfs;
      }
      i = j;
    }
    if (rc == 0) {
      qsort(fs, (size_t)nfs, sizeof(firstseen), fs_cmp);
      for (int m = 0; m < nfs; ++m) {
        const halfedge *x = &h[fs[m].g], *y = &h[fs[m].g + 1];
        const halfedge *pl = x->up ? x : y, *mi = x->up ? y : x;
        int32_t *E = edges + 6 * (size_t)m;
        E[0] = x->lo;
        E[1] = x->hi;
        E[2] = pl->t;
        E[3] = mi->t;
        E[4] = pl->a;
        E[5] = mi->a;
      }
      ne = nfs;
    }
  }
  free(h);
  free(fs);
  *n_edges = ne;
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Small vector helpers.                                                     */
/* ------------------------------------------------------------------------ */

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(const double *a, const double *b, double *c) {
  c[0] = a[0] - b[0];
  c[1] = a[1] - b[1];
  c[2] = a[2] - b[2];
}
static void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }
static double dist3(const double *a, const double *b) {
  double d[3];
  sub3(a, b, d);
  return norm3(d);
}

/* ------------------------------------------------------------------------ */
/* Closed-form potentials of a flat triangle (singularity cancellation).     */
/* The observation point is projected onto the triangle's plane; each edge   */
/* contributes a logarithm and, off the plane, an arctangent (Wilton et al., */
/* IEEE TAP 32(3) 1984; Graglia, IEEE TAP 41(10) 1993).                      */
/* ------------------------------------------------------------------------ */

void or_tri_potentials(const double *x0, const double *x1, const double *x2,
                       const double *r, double *S, double *V) {
  const double *x[3] = {x0, x1, x2};
  double e1[3], e2[3], n[3];
  sub3(x1, x0, e1);
  sub3(x2, x0, e2);
  cross3(e1, e2, n);
  double nn = norm3(n);
  n[0] /= nn;
  n[1] /= nn;
  n[2] /= nn;
  double rx0[3];
  sub3(r, x0, rx0);
  const double d = dot3(n, rx0), ad = fabs(d);
  double rho[3] = {r[0] - d * n[0], r[1] - d * n[1], r[2] - d * n[2]};
  double s = 0.0, vin[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 3; ++i) {
    const double *xm = x[i], *xp = x[(i + 1) % 3];
    double L[3], lh[3], uh[3], pm[3], pp[3];
    sub3(xp, xm, L);
    double len = norm3(L);
    lh[0] = L[0] / len;
    lh[1] = L[1] / len;
    lh[2] = L[2] / len;
    cross3(lh, n, uh); /* outward in-plane edge normal */
    sub3(xp, rho, pp);
    sub3(xm, rho, pm);
    const double lp = dot3(pp, lh), lm = dot3(pm, lh);
    const double p0 = dot3(pm, uh); /* signed distance, positive inside */
    const double r0sq = p0 * p0 + d * d;
    const double Rp = dist3(r, xp), Rm = dist3(r, xm);
    double f = 0.0, beta = 0.0;
    if (r0sq > 0.0) {
      /* ln((R+ + l+)/(R- + l-)) with R + l written as r0^2/(R - l) for l < 0 */
      const double psp = lp >= 0.0 ? Rp + lp : r0sq / (Rp - lp);
      const double psm = lm >= 0.0 ? Rm + lm : r0sq / (Rm - lm);
      f = log(psp / psm);
      beta = atan(p0 * lp / (r0sq + ad * Rp)) - atan(p0 * lm / (r0sq + ad * Rm));
    }
    s += p0 * f - ad * beta;
    const double cv = 0.5 * (r0sq * f + lp * Rp - lm * Rm);
    vin[0] += cv * uh[0];
    vin[1] += cv * uh[1];
    vin[2] += cv * uh[2];
  }
  *S = s;
  /* r' - r = (rho' - rho) - d n */
  V[0] = vin[0] - d * n[0] * s;
  V[1] = vin[1] - d * n[1] * s;
  V[2] = vin[2] - d * n[2] * s;
}

/* (exp(-jkR) - 1)/R = (-2 sin^2(kR/2) - j sin kR)/R, series for small kR. */
static cplx ghat(double k, double R) {
  const double x = k * R;
  if (x < 1e-4) return -I * k - 0.5 * k * k * R + I * (k * k * k * R * R / 6.0);
  const double sh = sin(0.5 * x);
  return (-2.0 * sh * sh - I * sin(x)) / R;
}

void or_ghat(double k, double R, double *re, double *im) {
  cplx g = ghat(k, R);
  *re = creal(g);
  *im = cimag(g);
}

/* ------------------------------------------------------------------------ */
/* Mesh geometry.                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
  int nv, nt, nq;
  const double *V;
  const int32_t *tri;
  const double *bary, *w;
  double *area; /* nt */
  double *qp;   /* nt * nq * 3 absolute quadrature points */
} mesh;

static const double *vtx(const mesh *m, int t, int a) { return m->V + 3 * (size_t)m->tri[3 * t + a]; }

static int mesh_init(mesh *m, int nv, const double *V, int nt, const int32_t *tri, int nq,
                     const double *bary, const double *w) {
  m->nv = nv;
  m->nt = nt;
  m->nq = nq;
  m->V = V;
  m->tri = tri;
  m->bary = bary;
  m->w = w;
  m->area = (double *)malloc(sizeof(double) * (size_t)nt);
  m->qp = (double *)malloc(sizeof(double) * 3 * (size_t)nt * (size_t)nq);
  if (!m->area || !m->qp) return -4;
  for (int t = 0; t < nt; ++t) {
    for (int c = 0; c < 3; ++c)
      if (tri[3 * t + c] < 0 || tri[3 * t + c] >= nv) return -2;
    const double *x0 = vtx(m, t, 0), *x1 = vtx(m, t, 1), *x2 = vtx(m, t, 2);
    double e1[3], e2[3], n[3];
    sub3(x1, x0, e1);
    sub3(x2, x0, e2);
    cross3(e1, e2, n);
    m->area[t] = 0.5 * norm3(n);
    if (!(m->area[t] > 0.0)) return -2;
    for (int i = 0; i < nq; ++i) {
      const double *b = bary + 3 * i;
      double *P = m->qp + 3 * ((size_t)t * nq + i);
      for (int c = 0; c < 3; ++c) P[c] = b[0] * x0[c] + b[1] * x1[c] + b[2] * x2[c];
    }
  }
  return 0;
}

static void mesh_free(mesh *m) {
  free(m->area);
  free(m->qp);
}

static const double *qpt(const mesh *m, int t, int i) { return m->qp + 3 * ((size_t)t * m->nq + i); }

static int touching(const mesh *m, int p, int q) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      if (m->tri[3 * p + a] == m->tri[3 * q + b]) return 1;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Adaptive interpolation tables (Section II-B, II-C).                       */
/* ------------------------------------------------------------------------ */

struct ortable {
  int kind;
  double k, rmin, rmax, tol, t;
  int n;
  double *r;
  cplx *f;
  double delta; /* minimum sampling interval = hash bucket width, Eq. (6) */
  int m;
  int32_t *hash;
  double probe_err;
  int iters;
};

static cplx exact_value(int kind, double k, double r) {
  cplx e = cexp(-I * k * r); /* Eq. (1) */
  return kind == OR_TABLE_EXP ? e : e / r;
}

/* Hash array of Eq. (6): bucket b holds the largest node index whose bucket
 * is <= b; buckets without a node take their predecessor's entry, filled
 * from the low end (Section II-C). */
static int build_hash(ortable *T) {
  double dmin = INFINITY;
  for (int i = 0; i + 1 < T->n; ++i) {
    double g = T->r[i + 1] - T->r[i];
    if (g < dmin) dmin = g;
  }
  if (!(dmin > 0.0)) return -1;
  T->delta = dmin;
  T->m = (int)floor((T->rmax - T->rmin) / dmin) + 1;
  T->hash = (int32_t *)malloc(sizeof(int32_t) * (size_t)T->m);
  if (!T->hash) return -4;
  for (int b = 0; b < T->m; ++b) T->hash[b] = -1;
  for (int i = 0; i < T->n; ++i) {
    int b = (int)floor((T->r[i] - T->rmin) / dmin);
    if (b > T->m - 1) b = T->m - 1;
    T->hash[b] = i;
  }
  if (T->hash[0] < 0) T->hash[0] = 0;
  for (int b = 1; b < T->m; ++b)
    if (T->hash[b] < 0) T->hash[b] = T->hash[b - 1];
  return 0;
}

int or_table_lookup(const ortable *T, double r, int32_t *idx) {
  if (!(r >= T->rmin && r <= T->rmax)) return -3;
  int b = (int)floor((r - T->rmin) / T->delta);
  if (b > T->m - 1) b = T->m - 1;
  int i = T->hash[b];
  if (T->r[i] > r) --i;
  if (i + 1 < T->n && r >= T->r[i + 1]) ++i;
  if (i > T->n - 2) i = T->n - 2;
  if (i < 0) i = 0;
  *idx = i;
  return 0;
}

/* Linear interpolation, Eq. (4), or cubic Lagrange on the four nodes around
 * the interval (shifted at the ends), Eq. (5). */
static cplx interp_at(const ortable *T, int i, double r) {
  if (T->kind == OR_TABLE_EXP) {
    const double r0 = T->r[i], r1 = T->r[i + 1];
    return T->f[i] * ((r - r1) / (r0 - r1)) + T->f[i + 1] * ((r - r0) / (r1 - r0));
  }
  int s = i - 1;
  if (s > T->n - 4) s = T->n - 4;
  if (s < 0) s = 0;
  cplx acc = 0.0;
  for (int j = s; j < s + 4; ++j) {
    double P = 1.0;
    for (int mm = s; mm < s + 4; ++mm)
      if (mm != j) P *= (r - T->r[mm]) / (T->r[j] - T->r[mm]);
    acc += T->f[j] * P;
  }
  return acc;
}

static int table_value(const ortable *T, double r, cplx *v) {
  int32_t i;
  int rc = or_table_lookup(T, r, &i);
  if (rc) return rc;
  *v = interp_at(T, i, r);
  return 0;
}

int or_table_eval(const ortable *T, int n, const double *r, double *out) {
  for (int s = 0; s < n; ++s) {
    cplx v;
    int rc = table_value(T, r[s], &v);
    if (rc) return rc;
    out[2 * s] = creal(v);
    out[2 * s + 1] = cimag(v);
  }
  return 0;
}

static int cmp_double(const void *x, const void *y) {
  double a = *(const double *)x, b = *(const double *)y;
  return (a > b) - (a < b);
}

/* Sampling points for one uniform interval t (Section II-B): uniform samples,
 * local refinement around the zeros of the real and imaginary parts, and the
 * zeros themselves, which win over nearby samples.  Candidates are taken in
 * the order zeros, end points, refined samples, uniform samples; a candidate
 * is kept only if no kept sample lies closer than mu*t. */
static int place_nodes(double k, double rmin, double rmax, double t, int refine, int zeros, double mu,
                       double win, double ratio, double **out, int *nout) {
  const double c = M_PI / (2.0 * k); /* zeros of cos(kr) and sin(kr): r = m c */
  long mz0 = (long)floor(rmin / c) + 1, nz = 0;
  while ((double)(mz0 + nz) * c < rmax) ++nz;
  if (!zeros && !refine) nz = 0;
  const long nu = (long)floor((rmax - rmin) / t) + 2;
  const int nref = (int)floor(win / ratio + 1e-9);
  const long cap = nz + 2 + (refine ? nz * (2 * nref) : 0) + nu + 4;
  double *cand = (double *)malloc(sizeof(double) * (size_t)cap);
  int *cls = (int *)malloc(sizeof(int) * (size_t)cap);
  double *acc = (double *)malloc(sizeof(double) * (size_t)cap);
  if (!cand || !cls || !acc) {
    free(cand);
    free(cls);
    free(acc);
    return -4;
  }
  long nc = 0;
  if (zeros)
    for (long j = 0; j < nz; ++j) {
      cand[nc] = (double)(mz0 + j) * c;
      cls[nc++] = 0;
    }
  cand[nc] = rmin;
  cls[nc++] = 1;
  cand[nc] = rmax;
  cls[nc++] = 1;
  if (refine)
    for (long j = 0; j < nz; ++j) {
      const double z = (double)(mz0 + j) * c;
      for (int s = -nref; s <= nref; ++s) {
        if (s == 0) continue;
        const double x = z + (double)s * (ratio * t);
        if (x > rmin && x < rmax) {
          cand[nc] = x;
          cls[nc++] = 2;
        }
      }
    }
  for (long i = 0;; ++i) {
    const double x = rmin + (double)i * t;
    if (!(x < rmax)) break;
    int inside = 0;
    if (refine) {
      /* dropped if it falls inside an open refinement window */
      long mm = (long)floor(x / c + 0.5);
      for (long d = mm - 1; d <= mm + 1; ++d) {
        if (d < mz0 || d >= mz0 + nz) continue;
        if (fabs(x - (double)d * c) < win * t) inside = 1;
      }
    }
    if (!inside) {
      cand[nc] = x;
      cls[nc++] = 3;
    }
  }
  /* greedy merge by class priority: within a class candidates are at least
   * ratio*t > mu*t apart, so only earlier classes can reject a candidate */
  long na = 0;
  const double mind = mu * t;
  /* kept samples are at least mu*t apart, so a cell of width mu*t holds one
   * of them (two slots allow for rounding in the cell index) */
  const long ncell = (long)floor((rmax - rmin) / mind) + 3;
  double *cell = (double *)malloc(sizeof(double) * 2 * (size_t)ncell);
  if (!cell) {
    free(cand);
    free(cls);
    free(acc);
    return -4;
  }
  for (long i = 0; i < 2 * ncell; ++i) cell[i] = NAN;
  for (int klass = 0; klass < 4; ++klass) {
    for (long i = 0; i < nc; ++i) {
      if (cls[i] != klass) continue;
      const double x = cand[i];
      long ci = (long)floor((x - rmin) / mind) + 1;
      if (ci < 1) ci = 1;
      if (ci > ncell - 2) ci = ncell - 2;
      int ok = 1;
      for (long d = 2 * (ci - 1); d < 2 * (ci + 2); ++d)
        if (!isnan(cell[d]) && fabs(cell[d] - x) < mind) ok = 0;
      if (ok) {
        cell[2 * ci + (isnan(cell[2 * ci]) ? 0 : 1)] = x;
        acc[na++] = x;
      }
    }
  }
  free(cell);
  free(cand);
  free(cls);
  qsort(acc, (size_t)na, sizeof(double), cmp_double);
  *out = acc;
  *nout = (int)na;
  return 0;
}

static double probe_error(const ortable *T) {
  double e = 0.0;
  for (int i = 0; i + 1 < T->n; ++i)
    for (int s = 1; s <= 8; ++s) {
      const double x = T->r[i] + (double)s / 9.0 * (T->r[i + 1] - T->r[i]);
      cplx ex = exact_value(T->kind, T->k, x), v = interp_at(T, i, x);
      double rel = cabs(v - ex) / cabs(ex);
      if (rel > e) e = rel;
    }
  {
    int32_t i;
    if (or_table_lookup(T, T->rmax, &i) == 0) {
      cplx ex = exact_value(T->kind, T->k, T->rmax), v = interp_at(T, i, T->rmax);
      double rel = cabs(v - ex) / cabs(ex);
      if (rel > e) e = rel;
    }
  }
  return e;
}

static void table_release(ortable *T) {
  if (!T) return;
  free(T->r);
  free(T->f);
  free(T->hash);
  T->r = NULL;
  T->f = NULL;
  T->hash = NULL;
}

void or_table_free(ortable *T) {
  table_release(T);
  free(T);
}

/* Uniform interval from the error bound of Eq. (10): linear, n = 1, with
 * |E''| = k^2 |E| and the widest merged gap (1+mu)t; cubic, n = 3, with
 * |G''''|/|G| <= k^4 + 4k^3/r + 12k^2/r^2 + 24k/r^3 + 24/r^4 taken at rmin.
 * Capped at a 32nd of a wavelength so refinement windows never overlap. */
static double interval_from_tol(int kind, double k, double rmin, double tol, double mu) {
  double t;
  if (kind == OR_TABLE_EXP) {
    t = sqrt(8.0 * tol) / (k * (1.0 + mu));
  } else {
    const double r = rmin;
    const double b4 = k * k * k * k + 4.0 * k * k * k / r + 12.0 * k * k / (r * r) +
                      24.0 * k / (r * r * r) + 24.0 / (r * r * r * r);
    t = pow(16.0 * tol / b4, 0.25);
  }
  const double cap = (2.0 * M_PI / k) / 32.0;
  return t < cap ? t : cap;
}

static int table_fill(ortable *T, double t, int refine, int zeros, double mu, double win, double ratio) {
  table_release(T);
  T->t = t;
  int rc = place_nodes(T->k, T->rmin, T->rmax, t, refine, zeros, mu, win, ratio, &T->r, &T->n);
  if (rc) return rc;
  if (T->n < (T->kind == OR_TABLE_EXP ? 2 : 4)) return -1;
  T->f = (cplx *)malloc(sizeof(cplx) * (size_t)T->n);
  if (!T->f) return -4;
  for (int i = 0; i < T->n; ++i) T->f[i] = exact_value(T->kind, T->k, T->r[i]);
  rc = build_hash(T);
  if (rc) return rc;
  T->probe_err = probe_error(T);
  return 0;
}

int or_table_build(int kind, double k, double rmin, double rmax, double tol, double t, int refine,
                   int zeros, double mu, double win, double ratio, ortable **out) {
  if (!out || (kind != OR_TABLE_EXP && kind != OR_TABLE_GREEN)) return -1;
  /* Exp(-jkr) has no singularity at the origin (Section II-B): its table may
   * start at r = 0; the Green function's may not */
  if (!(k > 0.0) || !isfinite(k) || !(kind == OR_TABLE_EXP ? rmin >= 0.0 : rmin > 0.0) ||
      !(rmax > rmin))
    return -1;
  if (!(mu > 0.0) || !(win > 0.0) || !(ratio > mu)) return -1;
  if (!(t > 0.0) && !(tol >= 1e-12 && tol <= 1e-1)) return -1;
  ortable *T = (ortable *)calloc(1, sizeof(ortable));
  if (!T) return -4;
  T->kind = kind;
  T->k = k;
  T->rmin = rmin;
  T->rmax = rmax;
  T->tol = tol;
  int rc;
  if (t > 0.0) {
    rc = table_fill(T, t, refine, zeros, mu, win, ratio);
    T->iters = 0;
  } else {
    double tt = interval_from_tol(kind, k, rmin, tol, mu);
    rc = -6;
    for (int it = 0; it <= 8; ++it) {
      int r2 = table_fill(T, tt, refine, zeros, mu, win, ratio);
      if (r2) {
        rc = r2;
        break;
      }
      T->iters = it;
      if (T->probe_err <= tol) {
        rc = 0;
        break;
      }
      tt = tt / sqrt(2.0);
    }
  }
  if (rc) {
    or_table_free(T);
    return rc;
  }
  *out = T;
  return 0;
}

int or_table_from_nodes(int kind, int n, const double *r, const double *fre, const double *fim,
                        ortable **out) {
  if (!out || n < (kind == OR_TABLE_EXP ? 2 : 4)) return -1;
  for (int i = 0; i + 1 < n; ++i)
    if (!(r[i + 1] > r[i])) return -1;
  ortable *T = (ortable *)calloc(1, sizeof(ortable));
  if (!T) return -4;
  T->kind = kind;
  T->rmin = r[0];
  T->rmax = r[n - 1];
  T->n = n;
  T->r = (double *)malloc(sizeof(double) * (size_t)n);
  T->f = (cplx *)malloc(sizeof(cplx) * (size_t)n);
  if (!T->r || !T->f) {
    or_table_free(T);
    return -4;
  }
  for (int i = 0; i < n; ++i) {
    T->r[i] = r[i];
    T->f[i] = fre[i] + I * fim[i];
  }
  int rc = build_hash(T);
  if (rc) {
    or_table_free(T);
    return rc;
  }
  *out = T;
  return 0;
}

void or_table_info(const ortable *T, int32_t *n, int32_t *m, double *t_used, double *delta,
                   double *probe_err, int32_t *iters) {
  *n = T->n;
  *m = T->m;
  *t_used = T->t;
  *delta = T->delta;
  *probe_err = T->probe_err;
  *iters = T->iters;
}

void or_table_get(const ortable *T, double *r, double *f, int32_t *hash) {
  for (int i = 0; i < T->n; ++i) {
    if (r) r[i] = T->r[i];
    if (f) {
      f[2 * i] = creal(T->f[i]);
      f[2 * i + 1] = cimag(T->f[i]);
    }
  }
  if (hash)
    for (int b = 0; b < T->m; ++b) hash[b] = T->hash[b];
}

/* ------------------------------------------------------------------------ */
/* Distance range over regular quadrature-point pairs (abstract: "maximum     */
/* and minimum distance between any two integration points").               */
/* ------------------------------------------------------------------------ */

int or_r_range(int nv, const double *V, int nt, const int32_t *tri, int nq, const double *bary,
               const double *w, double *rmin, double *rmax) {
  mesh M;
  int rc = mesh_init(&M, nv, V, nt, tri, nq, bary, w);
  if (rc) {
    mesh_free(&M);
    return rc;
  }
  double lo = INFINITY, hi = 0.0;
#pragma omp parallel for schedule(dynamic, 4) reduction(min : lo) reduction(max : hi)
  for (int p = 0; p < nt; ++p)
    for (int q = 0; q < nt; ++q) {
      if (touching(&M, p, q)) continue;
      for (int i = 0; i < nq; ++i)
        for (int j = 0; j < nq; ++j) {
          const double R = dist3(qpt(&M, p, i), qpt(&M, q, j));
          if (R < lo) lo = R;
          if (R > hi) hi = R;
        }
    }
  mesh_free(&M);
  if (!isfinite(lo)) return -1; /* no regular pair */
  *rmin = lo;
  *rmax = hi;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Triangle-pair integrals.                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
  const mesh *M;
  double k;
  int mode, part;
  const ortable *G;
  int force_touching; /* test hook: singularity-subtracted rule on any pair */
} fillctx;

/* Regular pair: both integrals by the product rule,
 * X = sum_i sum_j w_i w_j g(R_ij) [ (r_i - v_a).(r_j - v_b)/4 - 1/k^2 ]. */
static int pair_regular(const fillctx *C, int p, int q, int a, int b, cplx *X) {
  const mesh *M = C->M;
  const double *va = vtx(M, p, a), *vb = vtx(M, q, b);
  const double k = C->k;
  cplx acc = 0.0;
  for (int i = 0; i < M->nq; ++i) {
    const double *ri = qpt(M, p, i);
    double ua[3];
    sub3(ri, va, ua);
    for (int j = 0; j < M->nq; ++j) {
      const double *rj = qpt(M, q, j);
      double ub[3];
      sub3(rj, vb, ub);
      const double R = dist3(ri, rj);
      cplx g;
      if (C->mode == OR_MODE_DIRECT) {
        g = cexp(-I * k * R) / R;
      } else {
        int rc = table_value(C->G, R, &g);
        if (rc) return rc;
      }
      double br = 0.0;
      if (C->part != OR_PART_PHI) br += 0.25 * dot3(ua, ub);
      if (C->part != OR_PART_A) br -= 1.0 / (k * k);
      acc += M->w[i] * M->w[j] * g * br;
    }
  }
  *X = acc;
  return 0;
}

/* Touching pair, inner integral over q done as closed-form 1/R part plus the
 * quadrature of the smooth remainder g - 1/R:
 *   Phi(r)   = int_q g dS'          = S_q(r) + A_q sum_j w_j ghat(R_j)
 *   Psi_b(r) = int_q (r'-v_b) g dS' = V_q(r) + (r - v_b) S_q(r)
 *                                      + A_q sum_j w_j (r_j - v_b) ghat(R_j)
 *   X = (1/A_q) sum_i w_i [ (r_i - v_a).Psi_b(r_i)/4 - Phi(r_i)/k^2 ]. */
static void pair_touching_oneway(const fillctx *C, int p, int q, int a, int b, cplx *X) {
  const mesh *M = C->M;
  const double k = C->k, Aq = M->area[q];
  const double *va = vtx(M, p, a), *vb = vtx(M, q, b);
  cplx acc = 0.0;
  for (int i = 0; i < M->nq; ++i) {
    const double *ri = qpt(M, p, i);
    double S, Vv[3];
    or_tri_potentials(vtx(M, q, 0), vtx(M, q, 1), vtx(M, q, 2), ri, &S, Vv);
    cplx phi = S, psi[3];
    double rb[3];
    sub3(ri, vb, rb);
    for (int c = 0; c < 3; ++c) psi[c] = Vv[c] + rb[c] * S;
    for (int j = 0; j < M->nq; ++j) {
      const double *rj = qpt(M, q, j);
      const cplx gh = ghat(k, dist3(ri, rj));
      phi += Aq * M->w[j] * gh;
      for (int c = 0; c < 3; ++c) psi[c] += Aq * M->w[j] * (rj[c] - vb[c]) * gh;
    }
    double ua[3];
    sub3(ri, va, ua);
    cplx br = 0.0;
    if (C->part != OR_PART_PHI) br += 0.25 * (ua[0] * psi[0] + ua[1] * psi[1] + ua[2] * psi[2]);
    if (C->part != OR_PART_A) br -= phi / (k * k);
    acc += M->w[i] * br;
  }
  *X = acc / Aq;
}

static int pair_value(const fillctx *C, int p, int q, int a, int b, cplx *X) {
  if (C->force_touching || touching(C->M, p, q)) {
    cplx x1, x2;
    pair_touching_oneway(C, p, q, a, b, &x1);
    pair_touching_oneway(C, q, p, b, a, &x2);
    *X = 0.5 * (x1 + x2);
    return 0;
  }
  return pair_regular(C, p, q, a, b, X);
}

int or_pair_block(int nv, const double *V, int nt, const int32_t *tri, int p, int q, double k, int nq,
                  const double *bary, const double *w, int mode, int part, const ortable *gtable,
                  double *out18) {
  const int force = (mode & OR_FORCE_TOUCHING) != 0;
  mode &= ~OR_FORCE_TOUCHING;
  if (p < 0 || q < 0 || p >= nt || q >= nt || !(k > 0.0)) return -1;
  if (mode == OR_MODE_TABLE && !gtable) return -1;
  mesh M;
  int rc = mesh_init(&M, nv, V, nt, tri, nq, bary, w);
  if (rc == 0) {
    fillctx C = {&M, k, mode, part, gtable, force};
    for (int a = 0; a < 3 && rc == 0; ++a)
      for (int b = 0; b < 3 && rc == 0; ++b) {
        cplx X;
        rc = pair_value(&C, p, q, a, b, &X);
        out18[2 * (3 * a + b)] = creal(X);
        out18[2 * (3 * a + b) + 1] = cimag(X);
      }
  }
  mesh_free(&M);
  return rc;
}

/* One matrix entry: four triangle pairs, RWG signs and lengths, prefactor
 * j k eta / (4 pi). */
static int entry_value(const fillctx *C, const int32_t *em, const int32_t *en, cplx *Z) {
  const mesh *M = C->M;
  const double lm = dist3(M->V + 3 * (size_t)em[0], M->V + 3 * (size_t)em[1]);
  const double ln = dist3(M->V + 3 * (size_t)en[0], M->V + 3 * (size_t)en[1]);
  cplx acc = 0.0;
  for (int s = 0; s < 2; ++s)
    for (int u = 0; u < 2; ++u) {
      const int p = em[2 + s], a = em[4 + s], q = en[2 + u], b = en[4 + u];
      const double sg = (s == 0 ? 1.0 : -1.0) * (u == 0 ? 1.0 : -1.0);
      cplx X;
      int rc = pair_value(C, p, q, a, b, &X);
      if (rc) return rc;
      acc += sg * X;
    }
  *Z = (I * C->k * OR_ETA0 / (4.0 * M_PI)) * lm * ln * acc;
  return 0;
}

int or_fill_entries(int nv, const double *V, int nt, const int32_t *tri, int ne, const int32_t *edges,
                    double k, int nq, const double *bary, const double *w, int mode, int part,
                    const ortable *gtable, int64_t ns, const int64_t *rows, const int64_t *cols,
                    double *out) {
  if (!(k > 0.0) || !isfinite(k) || ne <= 0) return -1;
  if (mode != OR_MODE_DIRECT && mode != OR_MODE_TABLE) return -1;
  if (mode == OR_MODE_TABLE && (!gtable || gtable->kind != OR_TABLE_GREEN)) return -1;
  for (int64_t s = 0; s < ns; ++s)
    if (rows[s] < 0 || rows[s] >= ne || cols[s] < 0 || cols[s] >= ne) return -1;
  mesh M;
  int rc = mesh_init(&M, nv, V, nt, tri, nq, bary, w);
  if (rc) {
    mesh_free(&M);
    return rc;
  }
  fillctx C = {&M, k, mode, part, gtable, 0};
  int err = 0;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t s = 0; s < ns; ++s) {
    cplx Z = 0.0;
    int r2 = entry_value(&C, edges + 6 * rows[s], edges + 6 * cols[s], &Z);
    if (r2) {
#pragma omp atomic write
      err = r2;
    }
    out[2 * s] = creal(Z);
    out[2 * s + 1] = cimag(Z);
  }
  mesh_free(&M);
  return err;
}

/* ------------------------------------------------------------------------ */
/* Row block of Z in triangle-pair order (the CPU baseline of the fill): each */
/* triangle pair evaluates its kernel values once and forms all nine local   */
/* entries from them, by the same rules as pair_value; the entries are then  */
/* scattered with the RWG signs and lengths.                                 */
/* ------------------------------------------------------------------------ */

/* Regular pair, all (a, b): one g(R_ij) per point pair. */
static int regular_block9(const fillctx *C, int p, int q, cplx X[3][3]) {
  const mesh *M = C->M;
  const double k = C->k;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) X[a][b] = 0.0;
  for (int i = 0; i < M->nq; ++i) {
    const double *ri = qpt(M, p, i);
    double ua[3][3]; /* r_i - v_a */
    for (int a = 0; a < 3; ++a) sub3(ri, vtx(M, p, a), ua[a]);
    for (int j = 0; j < M->nq; ++j) {
      const double *rj = qpt(M, q, j);
      double ub[3][3]; /* r_j - v_b */
      for (int b = 0; b < 3; ++b) sub3(rj, vtx(M, q, b), ub[b]);
      const double R = dist3(ri, rj);
      cplx g;
      if (C->mode == OR_MODE_DIRECT) {
        g = cexp(-I * k * R) / R;
      } else {
        int rc = table_value(C->G, R, &g);
        if (rc) return rc;
      }
      const cplx wg = M->w[i] * M->w[j] * g;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double br = 0.0;
          if (C->part != OR_PART_PHI) br += 0.25 * dot3(ua[a], ub[b]);
          if (C->part != OR_PART_A) br -= 1.0 / (k * k);
          X[a][b] += wg * br;
        }
    }
  }
  return 0;
}

/* Touching pair, one way, all (a, b): the closed-form potentials and the
 * remainder sums once per outer point (pair_touching_oneway's rule). */
static void touching_block9(const fillctx *C, int p, int q, cplx X[3][3]) {
  const mesh *M = C->M;
  const double k = C->k, Aq = M->area[q];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) X[a][b] = 0.0;
  for (int i = 0; i < M->nq; ++i) {
    const double *ri = qpt(M, p, i);
    double S, Vv[3];
    or_tri_potentials(vtx(M, q, 0), vtx(M, q, 1), vtx(M, q, 2), ri, &S, Vv);
    cplx phi = S, s1[3] = {0.0, 0.0, 0.0}; /* s1 = A_q sum_j w_j r_j ghat */
    cplx s0 = 0.0;                        /* s0 = A_q sum_j w_j ghat */
    for (int j = 0; j < M->nq; ++j) {
      const double *rj = qpt(M, q, j);
      const cplx gh = ghat(k, dist3(ri, rj));
      s0 += Aq * M->w[j] * gh;
      for (int c = 0; c < 3; ++c) s1[c] += Aq * M->w[j] * rj[c] * gh;
    }
    phi += s0;
    for (int b = 0; b < 3; ++b) {
      const double *vb = vtx(M, q, b);
      double rb[3];
      sub3(ri, vb, rb);
      cplx psi[3];
      for (int c = 0; c < 3; ++c) psi[c] = Vv[c] + rb[c] * S + (s1[c] - vb[c] * s0);
      for (int a = 0; a < 3; ++a) {
        double ua[3];
        sub3(ri, vtx(M, p, a), ua);
        cplx br = 0.0;
        if (C->part != OR_PART_PHI) br += 0.25 * (ua[0] * psi[0] + ua[1] * psi[1] + ua[2] * psi[2]);
        if (C->part != OR_PART_A) br -= phi / (k * k);
        X[a][b] += M->w[i] * br;
      }
    }
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) X[a][b] /= Aq;
}

static int pair_block9(const fillctx *C, int p, int q, cplx X[3][3]) {
  if (touching(C->M, p, q)) {
    cplx A[3][3], B[3][3];
    touching_block9(C, p, q, A);
    touching_block9(C, q, p, B);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) X[a][b] = 0.5 * (A[a][b] + B[b][a]);
    return 0;
  }
  return regular_block9(C, p, q, X);
}

int or_fill_rows(int nv, const double *V, int nt, const int32_t *tri, int ne, const int32_t *edges,
                 double k, int nq, const double *bary, const double *w, int mode, int part,
                 const ortable *gtable, int r0, int r1, double *out) {
  if (!(k > 0.0) || !isfinite(k) || ne <= 0 || r0 < 0 || r1 > ne || r0 >= r1) return -1;
  if (mode != OR_MODE_DIRECT && mode != OR_MODE_TABLE) return -1;
  if (mode == OR_MODE_TABLE && (!gtable || gtable->kind != OR_TABLE_GREEN)) return -1;
  mesh M;
  int rc = mesh_init(&M, nv, V, nt, tri, nq, bary, w);
  /* per triangle and local vertex a: the edge opposite a (-1: none) and its sign */
  int32_t *ted = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)nt);
  int8_t *tsg = (int8_t *)malloc(3 * (size_t)nt);
  int32_t *plist = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(r1 - r0));
  char *seen = (char *)calloc((size_t)nt, 1);
  if (!rc && (!ted || !tsg || !plist || !seen)) rc = -4;
  int np = 0;
  if (!rc) {
    for (size_t i = 0; i < 3 * (size_t)nt; ++i) {
      ted[i] = -1;
      tsg[i] = 0;
    }
    for (int m = 0; m < ne; ++m)
      for (int s = 0; s < 2; ++s) {
        const int t = edges[6 * (size_t)m + 2 + s], a = edges[6 * (size_t)m + 4 + s];
        ted[3 * (size_t)t + a] = m;
        tsg[3 * (size_t)t + a] = s == 0 ? 1 : -1;
      }
    for (int m = r0; m < r1; ++m)
      for (int s = 0; s < 2; ++s) {
        const int t = edges[6 * (size_t)m + 2 + s];
        if (!seen[t]) {
          seen[t] = 1;
          plist[np++] = t;
        }
      }
    for (size_t i = 0; i < 2 * (size_t)(r1 - r0) * (size_t)ne; ++i) out[i] = 0.0;
  }
  int err = rc;
  if (!rc) {
    fillctx C = {&M, k, mode, part, gtable, 0};
    const cplx pref = I * k * OR_ETA0 / (4.0 * M_PI);
#pragma omp parallel for schedule(dynamic, 1)
    for (int ip = 0; ip < np; ++ip) {
      const int p = plist[ip];
      for (int q = 0; q < nt; ++q) {
        cplx X[3][3];
        int r2 = pair_block9(&C, p, q, X);
        if (r2) {
#pragma omp atomic write
          err = r2;
          continue;
        }
        for (int a = 0; a < 3; ++a) {
          const int m = ted[3 * (size_t)p + a];
          if (m < r0 || m >= r1) continue;
          const double lm = dist3(V + 3 * (size_t)edges[6 * (size_t)m], V + 3 * (size_t)edges[6 * (size_t)m + 1]);
          for (int b = 0; b < 3; ++b) {
            const int n = ted[3 * (size_t)q + b];
            if (n < 0) continue;
            const double ln = dist3(V + 3 * (size_t)edges[6 * (size_t)n], V + 3 * (size_t)edges[6 * (size_t)n + 1]);
            const cplx v = pref * (tsg[3 * (size_t)p + a] * tsg[3 * (size_t)q + b]) * lm * ln * X[a][b];
            double *o = out + 2 * ((size_t)(m - r0) * ne + n);
#pragma omp atomic
            o[0] += creal(v);
#pragma omp atomic
            o[1] += cimag(v);
          }
        }
      }
    }
  }
  free(ted);
  free(tsg);
  free(plist);
  free(seen);
  mesh_free(&M);
  return err;
}

/* ------------------------------------------------------------------------ */
/* Loss L = Re sum_mn conj(W_mn) Z_mn (direct mode), for finite differences   */
/* of the adjoint: the full sum, or only the entries whose row or column     */
/* edge lies on a triangle containing vertex v (the only entries that move   */
/* when v moves).                                                            */
/* ------------------------------------------------------------------------ */

static int loss_impl(int nv, const double *V, int nt, const int32_t *tri, int ne,
                     const int32_t *edges, double k, int nq, const double *bary, const double *w,
                     const double *W, int vsel, double *L) {
  if (!(k > 0.0) || ne <= 0) return -1;
  mesh M;
  int rc = mesh_init(&M, nv, V, nt, tri, nq, bary, w);
  if (rc) {
    mesh_free(&M);
    return rc;
  }
  fillctx C = {&M, k, OR_MODE_DIRECT, OR_PART_ALL, NULL, 0};
  /* mark the edges that lie on a triangle containing vsel */
  char *mark = (char *)calloc((size_t)ne, 1);
  if (!mark) {
    mesh_free(&M);
    return -4;
  }
  for (int m = 0; m < ne; ++m) {
    if (vsel < 0) {
      mark[m] = 1;
      continue;
    }
    for (int s = 0; s < 2; ++s) {
      const int t = edges[6 * m + 2 + s];
      for (int c = 0; c < 3; ++c)
        if (tri[3 * t + c] == vsel) mark[m] = 1;
    }
  }
  double acc = 0.0;
  int err = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : acc)
  for (int m = 0; m < ne; ++m)
    for (int n = 0; n < ne; ++n) {
      if (vsel >= 0 && !mark[m] && !mark[n]) continue;
      cplx Z;
      int r2 = entry_value(&C, edges + 6 * (size_t)m, edges + 6 * (size_t)n, &Z);
      if (r2) {
#pragma omp atomic write
        err = r2;
      }
      const double wr = W[2 * ((size_t)m * ne + n)], wi = W[2 * ((size_t)m * ne + n) + 1];
      acc += wr * creal(Z) + wi * cimag(Z); /* Re(conj(W) Z) */
    }
  free(mark);
  mesh_free(&M);
  *L = acc;
  return err;
}

int or_loss(int nv, const double *V, int nt, const int32_t *tri, int ne, const int32_t *edges,
            double k, int nq, const double *bary, const double *w, const double *W, double *L) {
  return loss_impl(nv, V, nt, tri, ne, edges, k, nq, bary, w, W, -1, L);
}

int or_loss_local(int nv, const double *V, int nt, const int32_t *tri, int ne,
                  const int32_t *edges, double k, int nq, const double *bary, const double *w,
                  const double *W, int v, double *L) {
  if (v < 0 || v >= nv) return -1;
  return loss_impl(nv, V, nt, tri, ne, edges, k, nq, bary, w, W, v, L);
}

/* Sets the threads of the OpenMP loops (a timing hook; no effect without
 * OpenMP). */
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* Threads the OpenMP loops of this library use (1 without OpenMP). */
int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* MFIE K operator (the magnetic-field formulation the paper fills beside    */
/* the EFIE, Section IV-B), FP64, direct exponential.                        */
/*                                                                          */
/*   K_mn = <f_m, n x PV int grad G x f_n dS'>                              */
/*        = -(1/4pi) int int f_m . n x (d x f_n) (1 + jkR) exp(-jkR)/R^3    */
/* with d = r - r', n the outward normal at r.  With a = r - v_a,           */
/* b = r' - v_b and t = a x n the integrand is b.(t x d) K(R).  The MFIE    */
/* matrix is Z_mn = <f_m, f_n>/2 - K_mn.                                     */
/* ------------------------------------------------------------------------ */

/* Gradient of S(r) = int dS'/|r - r'| over the triangle:
 *   grad S = -sum_i uh_i f_i - sign(d) Omega n,
 * uh_i the outward in-plane edge normals, f_i the edge logarithms of S and
 * Omega the solid angle (sum of the arctangent pairs of S). */
void or_grad_potential(const double *x0, const double *x1, const double *x2, const double *r,
                       double *g) {
  const double *x[3] = {x0, x1, x2};
  double e1[3], e2[3], n[3];
  sub3(x1, x0, e1);
  sub3(x2, x0, e2);
  cross3(e1, e2, n);
  const double nn = norm3(n);
  n[0] /= nn;
  n[1] /= nn;
  n[2] /= nn;
  double rx0[3];
  sub3(r, x0, rx0);
  const double d = dot3(n, rx0), ad = fabs(d);
  const double rho[3] = {r[0] - d * n[0], r[1] - d * n[1], r[2] - d * n[2]};
  double gi[3] = {0.0, 0.0, 0.0}, omega = 0.0;
  for (int i = 0; i < 3; ++i) {
    const double *xm = x[i], *xp = x[(i + 1) % 3];
    double L[3], lh[3], uh[3], pm[3], pp[3];
    sub3(xp, xm, L);
    const double len = norm3(L);
    lh[0] = L[0] / len;
    lh[1] = L[1] / len;
    lh[2] = L[2] / len;
    cross3(lh, n, uh);
    sub3(xp, rho, pp);
    sub3(xm, rho, pm);
    const double lp = dot3(pp, lh), lm = dot3(pm, lh);
    const double p0 = dot3(pm, uh);
    const double r0sq = p0 * p0 + d * d;
    const double Rp = dist3(r, xp), Rm = dist3(r, xm);
    if (r0sq > 0.0) {
      const double psp = lp >= 0.0 ? Rp + lp : r0sq / (Rp - lp);
      const double psm = lm >= 0.0 ? Rm + lm : r0sq / (Rm - lm);
      const double f = log(psp / psm);
      for (int c = 0; c < 3; ++c) gi[c] -= uh[c] * f;
      omega += atan(p0 * lp / (r0sq + ad * Rp)) - atan(p0 * lm / (r0sq + ad * Rm));
    }
  }
  const double sg = d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0);
  for (int c = 0; c < 3; ++c) g[c] = gi[c] - sg * omega * n[c];
}

/* (1 + jkR) exp(-jkR)/R^3 */
static cplx kkernel(double k, double R) {
  return (1.0 + I * k * R) * cexp(-I * k * R) / (R * R * R);
}

/* K(R) - 1/R^3 - k^2/(2R), bounded; Taylor series for kR < 1e-2 */
static cplx kkernel_rem(double k, double R) {
  const double x = k * R;
  if (x < 1e-2) {
    const double k3 = k * k * k;
    return -I * k3 / 3.0 - k3 * x / 8.0 + I * k3 * x * x / 30.0 + k3 * x * x * x / 144.0;
  }
  return kkernel(k, R) - 1.0 / (R * R * R) - 0.5 * k * k / R;
}

static void unit_normal(const mesh *M, int t, double *n) {
  double e1[3], e2[3];
  sub3(vtx(M, t, 1), vtx(M, t, 0), e1);
  sub3(vtx(M, t, 2), vtx(M, t, 0), e2);
  cross3(e1, e2, n);
  const double nn = norm3(n);
  n[0] /= nn;
  n[1] /= nn;
  n[2] /= nn;
}

/* X = (1/4) sum_i sum_j w_i w_j b_j.(t_i x d_ij) K(R_ij), t_i = (r_i - v_a) x n_p.
 * With a Green table G (table mode) the kernel is K = (1/R + jk) G(R)/R. */
static int mfie_regular(const mesh *M, double k, const ortable *G, int p, int q, int a, int b,
                        cplx *X) {
  const double *va = vtx(M, p, a), *vb = vtx(M, q, b);
  double n[3];
  unit_normal(M, p, n);
  cplx acc = 0.0;
  for (int i = 0; i < M->nq; ++i) {
    const double *ri = qpt(M, p, i);
    double ua[3], t[3];
    sub3(ri, va, ua);
    cross3(ua, n, t);
    for (int j = 0; j < M->nq; ++j) {
      const double *rj = qpt(M, q, j);
      double ub[3], d[3], td[3];
      sub3(rj, vb, ub);
      sub3(ri, rj, d);
      cross3(t, d, td);
      const double R = norm3(d);
      cplx K;
      if (G) {
        cplx g;
        int rc = table_value(G, R, &g);
        if (rc) return rc;
        K = (1.0 / R + I * k) * g / R;
      } else {
        K = kkernel(k, R);
      }
      acc += M->w[i] * M->w[j] * dot3(ub, td) * K;
    }
  }
  *X = 0.25 * acc;
  return 0;
}

/* Touching pair p != q: the inner integral of b.(t x d)[1/R^3 + k^2/(2R)]
 * in closed form, t.[(-grad S - (k^2/2) V) x (r - v_b)] (d x (r' - v_b) =
 * d x (r - v_b), int d/R^3 = -grad S, int d/R = -V), the bounded remainder
 * by the rule. */
static void mfie_touching(const mesh *M, double k, int p, int q, int a, int b, cplx *X) {
  const double *va = vtx(M, p, a), *vb = vtx(M, q, b);
  const double Aq = M->area[q];
  double n[3];
  unit_normal(M, p, n);
  cplx acc = 0.0;
  for (int i = 0; i < M->nq; ++i) {
    const double *ri = qpt(M, p, i);
    double ua[3], t[3], gS[3], S, Vq[3], rb[3], w3[3], cr[3];
    sub3(ri, va, ua);
    cross3(ua, n, t);
    or_grad_potential(vtx(M, q, 0), vtx(M, q, 1), vtx(M, q, 2), ri, gS);
    or_tri_potentials(vtx(M, q, 0), vtx(M, q, 1), vtx(M, q, 2), ri, &S, Vq);
    sub3(ri, vb, rb);
    for (int c = 0; c < 3; ++c) w3[c] = -gS[c] - 0.5 * k * k * Vq[c];
    cross3(w3, rb, cr);
    cplx inner = dot3(t, cr) / Aq;
    for (int j = 0; j < M->nq; ++j) {
      const double *rj = qpt(M, q, j);
      double ub[3], d[3], td[3];
      sub3(rj, vb, ub);
      sub3(ri, rj, d);
      cross3(t, d, td);
      inner += M->w[j] * dot3(ub, td) * kkernel_rem(k, norm3(d));
    }
    acc += M->w[i] * inner;
  }
  *X = 0.25 * acc;
}

static int mfie_pair(const mesh *M, double k, const ortable *G, int p, int q, int a, int b,
                     int force, cplx *X) {
  if (p == q) {
    *X = 0.0; /* flat triangle: the integrand vanishes (principal value) */
    return 0;
  }
  if (force || touching(M, p, q)) {
    mfie_touching(M, k, p, q, a, b, X);
    return 0;
  }
  return mfie_regular(M, k, G, p, q, a, b, X);
}

int or_mfie_pair_block(int nv, const double *V, int nt, const int32_t *tri, int p, int q, double k,
                       int nq, const double *bary, const double *w, int force_touching,
                       double *out18) {
  if (p < 0 || q < 0 || p >= nt || q >= nt || !(k > 0.0)) return -1;
  mesh M;
  int rc = mesh_init(&M, nv, V, nt, tri, nq, bary, w);
  if (rc == 0)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        cplx X;
        mfie_pair(&M, k, NULL, p, q, a, b, force_touching, &X);
        out18[2 * (3 * a + b)] = creal(X);
        out18[2 * (3 * a + b) + 1] = cimag(X);
      }
  mesh_free(&M);
  return rc;
}

/* Z_mn = l_m l_n sum over the four triangle pairs s s' [ [p = q] (1/(8 A_p))
 * sum_i w_i (r_i - v_a).(r_i - v_b) + X(p,q;a,b)/(4 pi) ]. */
int or_mfie_entries(int nv, const double *V, int nt, const int32_t *tri, int ne,
                    const int32_t *edges, double k, int nq, const double *bary, const double *w,
                    int mode, const ortable *gtable, int64_t ns, const int64_t *rows,
                    const int64_t *cols, double *out) {
  if (!(k > 0.0) || !isfinite(k) || ne <= 0) return -1;
  if (mode != OR_MODE_DIRECT && mode != OR_MODE_TABLE) return -1;
  if (mode == OR_MODE_TABLE && (!gtable || gtable->kind != OR_TABLE_GREEN)) return -1;
  const ortable *G = mode == OR_MODE_TABLE ? gtable : NULL;
  for (int64_t s = 0; s < ns; ++s)
    if (rows[s] < 0 || rows[s] >= ne || cols[s] < 0 || cols[s] >= ne) return -1;
  mesh M;
  int rc = mesh_init(&M, nv, V, nt, tri, nq, bary, w);
  if (rc) {
    mesh_free(&M);
    return rc;
  }
  int err = 0;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t s = 0; s < ns; ++s) {
    const int32_t *em = edges + 6 * rows[s], *en = edges + 6 * cols[s];
    const double lm = dist3(V + 3 * (size_t)em[0], V + 3 * (size_t)em[1]);
    const double ln = dist3(V + 3 * (size_t)en[0], V + 3 * (size_t)en[1]);
    cplx acc = 0.0;
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) {
        const int p = em[2 + u], a = em[4 + u], q = en[2 + v], b = en[4 + v];
        const double sg = (u == 0 ? 1.0 : -1.0) * (v == 0 ? 1.0 : -1.0);
        cplx X = 0.0;
        int r2 = mfie_pair(&M, k, G, p, q, a, b, 0, &X);
        if (r2) {
#pragma omp atomic write
          err = r2;
        }
        cplx val = X / (4.0 * M_PI);
        if (p == q) {
          double gram = 0.0;
          for (int i = 0; i < M.nq; ++i) {
            double ua[3], ub[3];
            sub3(qpt(&M, p, i), vtx(&M, p, a), ua);
            sub3(qpt(&M, p, i), vtx(&M, p, b), ub);
            gram += M.w[i] * dot3(ua, ub);
          }
          val += gram / (8.0 * M.area[p]);
        }
        acc += sg * val;
      }
    const cplx Z = lm * ln * acc;
    out[2 * s] = creal(Z);
    out[2 * s + 1] = cimag(Z);
  }
  mesh_free(&M);
  return err;
}

/* ------------------------------------------------------------------------ */
/* EFIE inner integrals by the angular transformation (Section II-A: n      */
/* points on each of the three source edges, 3mn Exp evaluations per source  */
/* triangle and m outer points).                                             */
/*                                                                          */
/* Observation point r, source triangle q with unit normal n, r = rho0 + h n */
/* (rho0 in the plane).  Edge i runs from x_i to x_{i+1}; t_i is its unit    */
/* tangent, m_i = t_i x n its outward in-plane normal, p_i = m_i.(x_i -      */
/* rho0) the signed distance from rho0 (positive on the triangle's side),    */
/* l runs along the edge from the foot of the perpendicular, and on the edge */
/* R(l)^2 = d^2 + l^2 with d^2 = p_i^2 + h^2.                                */
/*                                                                          */
/*   I0 = int_q exp(-jkR)/R dS'                                              */
/*   In polar coordinates about rho0 (the angular transformation), R dR =    */
/*   rho drho makes the radial integral exact: int_0^{rho_e} exp(-jkR)/R     */
/*   rho drho = (exp(-jk|h|) - exp(-jkR_e))/(jk).  The triangle is the       */
/*   signed sum of the triangles (rho0, edge i), and the edge is seen under  */
/*   dphi = |p_i| dl/(p_i^2 + l^2):                                          */
/*   I0 = (1/jk) sum_i p_i int_edge [exp(-jk|h|) - exp(-jkR)] dl/(p_i^2 + l^2). */
/*                                                                          */
/*   I1 = int_q (r' - rho0) exp(-jkR)/R dS'                                  */
/*   The in-plane gradient of exp(-jkR) is -jk exp(-jkR)(r' - rho0)/R, so    */
/*   I1 = (j/k) int_q grad' exp(-jkR) dS' = (j/k) sum_i m_i int_edge          */
/*   exp(-jkR) dl (surface divergence theorem).                              */
/*                                                                          */
/* Both edge integrals take the same n Gauss-Legendre points in u, l = d    */
/* sinh(u), R = d cosh(u), dl = R du: the map is smooth through the foot of  */
/* the perpendicular, where R(l) has its kink and the angular weight its    */
/* peak, and exp(-jkR) is computed (or read from the linear Exp table, mode  */
/* OR_MODE_TABLE) once per point for both integrals; exp(-jk|h|) comes from */
/* the same source.  An edge with d = 0 (r on the edge's line) takes the    */
/* points in l and adds nothing to I0.                                       */
/* ------------------------------------------------------------------------ */

/* Legendre polynomial P_n(z) and its derivative (three-term recurrence). */
static void legendre(int n, double z, double *pn, double *dpn) {
  double p0 = 1.0, p1 = z;
  for (int j = 2; j <= n; ++j) {
    const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;
  *dpn = n * (z * p1 - p0) / (z * z - 1.0);
}

/* Gauss-Legendre nodes and weights on [0, 1] (Newton's method on P_n). */
static void gauss01(int n, double *x, double *w) {
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5)), pn, dp;
    for (int it = 0; it < 100; ++it) {
      legendre(n, z, &pn, &dp);
      const double dz = pn / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    legendre(n, z, &pn, &dp);
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
  }
}

static int exp_value(const ortable *E, double k, double R, cplx *v) {
  if (!E) {
    *v = cexp(-I * k * R);
    return 0;
  }
  return table_value(E, R, v);
}

#define OR_MAX_EDGE_PTS 16

/* I0 (one complex) and I1 (three complex) at r for the triangle x0 x1 x2. */
static int angular_inner(const double *x0, const double *x1, const double *x2, const double *r,
                         double k, int n, const double *gx, const double *gw, const ortable *E,
                         cplx *I0, cplx *I1) {
  const double *x[3] = {x0, x1, x2};
  double e1[3], e2[3], nrm[3];
  sub3(x1, x0, e1);
  sub3(x2, x0, e2);
  cross3(e1, e2, nrm);
  const double nn = norm3(nrm);
  for (int c = 0; c < 3; ++c) nrm[c] /= nn;
  double rx0[3];
  sub3(r, x0, rx0);
  const double h = dot3(nrm, rx0), ah = fabs(h);
  const double rho0[3] = {r[0] - h * nrm[0], r[1] - h * nrm[1], r[2] - h * nrm[2]};
  /* exp(-jk|h|) from the same source as the edge values, so that the
   * differences exp(-jk|h|) - exp(-jkR) carry one interpolant, not two */
  cplx eh;
  int rc0 = exp_value(E, k, ah, &eh);
  if (rc0) return rc0;
  cplx a0 = 0.0, a1[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 3; ++i) {
    const double *xa = x[i], *xb = x[(i + 1) % 3];
    double t[3], m[3], da[3], db[3];
    sub3(xb, xa, t);
    const double len = norm3(t);
    for (int c = 0; c < 3; ++c) t[c] /= len;
    cross3(t, nrm, m);
    sub3(xa, rho0, da);
    sub3(xb, rho0, db);
    const double p = dot3(m, da), lm = dot3(t, da), lp = dot3(t, db);
    const double d = sqrt(p * p + h * h);
    cplx s0 = 0.0, s1 = 0.0; /* the two edge integrals */
    if (d > 0.0) {
      const double u0 = asinh(lm / d), du = asinh(lp / d) - u0;
      for (int j = 0; j < n; ++j) {
        const double u = u0 + du * gx[j];
        const double l = d * sinh(u), R = d * cosh(u);
        cplx ev;
        int rc = exp_value(E, k, R, &ev);
        if (rc) return rc;
        s0 += gw[j] * du * R * (eh - ev) / (p * p + l * l);
        s1 += gw[j] * du * R * ev;
      }
    } else {
      for (int j = 0; j < n; ++j) {
        const double l = lm + (lp - lm) * gx[j];
        cplx ev;
        int rc = exp_value(E, k, fabs(l), &ev);
        if (rc) return rc;
        s1 += gw[j] * (lp - lm) * ev;
      }
    }
    a0 += p * s0;
    for (int c = 0; c < 3; ++c) a1[c] += m[c] * s1;
  }
  *I0 = a0 / (I * k);
  for (int c = 0; c < 3; ++c) I1[c] = (I / k) * a1[c];
  return 0;
}

int or_angular_inner(const double *x0, const double *x1, const double *x2, const double *r,
                     double k, int n, int mode, const ortable *etable, double *out8) {
  if (!(k > 0.0) || n < 1 || n > OR_MAX_EDGE_PTS) return -1;
  if (mode == OR_MODE_TABLE && (!etable || etable->kind != OR_TABLE_EXP)) return -1;
  double gx[OR_MAX_EDGE_PTS], gw[OR_MAX_EDGE_PTS];
  gauss01(n, gx, gw);
  cplx I0, I1[3];
  int rc = angular_inner(x0, x1, x2, r, k, n, gx, gw, mode == OR_MODE_TABLE ? etable : NULL, &I0,
                         I1);
  if (rc) return rc;
  out8[0] = creal(I0);
  out8[1] = cimag(I0);
  for (int c = 0; c < 3; ++c) {
    out8[2 + 2 * c] = creal(I1[c]);
    out8[3 + 2 * c] = cimag(I1[c]);
  }
  return 0;
}

/* X(p,q;a,b) = (1/A_q) sum_i w_i [ (r_i - v_a).Psi_b(r_i)/4 - Phi(r_i)/k^2 ],
 * Phi = I0, Psi_b = I1 + (rho0 - v_b) I0, for every pair (touching or not). */
static int angular_pair(const mesh *M, double k, int n, const double *gx, const double *gw,
                        const ortable *E, int p, int q, int a, int b, cplx *X) {
  const double *va = vtx(M, p, a), *vb = vtx(M, q, b);
  double e1[3], e2[3], nrm[3];
  sub3(vtx(M, q, 1), vtx(M, q, 0), e1);
  sub3(vtx(M, q, 2), vtx(M, q, 0), e2);
  cross3(e1, e2, nrm);
  const double nn = norm3(nrm);
  for (int c = 0; c < 3; ++c) nrm[c] /= nn;
  cplx acc = 0.0;
  for (int i = 0; i < M->nq; ++i) {
    const double *ri = qpt(M, p, i);
    cplx I0, I1[3];
    int rc = angular_inner(vtx(M, q, 0), vtx(M, q, 1), vtx(M, q, 2), ri, k, n, gx, gw, E, &I0, I1);
    if (rc) return rc;
    double rx0[3];
    sub3(ri, vtx(M, q, 0), rx0);
    const double h = dot3(nrm, rx0);
    cplx dotv = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double rho0 = ri[c] - h * nrm[c];
      dotv += (ri[c] - va[c]) * (I1[c] + (rho0 - vb[c]) * I0);
    }
    acc += M->w[i] * (0.25 * dotv - I0 / (k * k));
  }
  *X = acc / M->area[q];
  return 0;
}

int or_angular_entries(int nv, const double *V, int nt, const int32_t *tri, int ne,
                       const int32_t *edges, double k, int nq, const double *bary, const double *w,
                       int n_edge, int mode, const ortable *etable, int64_t ns,
                       const int64_t *rows, const int64_t *cols, double *out) {
  if (!(k > 0.0) || !isfinite(k) || ne <= 0 || n_edge < 1 || n_edge > OR_MAX_EDGE_PTS) return -1;
  if (mode != OR_MODE_DIRECT && mode != OR_MODE_TABLE) return -1;
  if (mode == OR_MODE_TABLE && (!etable || etable->kind != OR_TABLE_EXP)) return -1;
  for (int64_t s = 0; s < ns; ++s)
    if (rows[s] < 0 || rows[s] >= ne || cols[s] < 0 || cols[s] >= ne) return -1;
  mesh M;
  int rc = mesh_init(&M, nv, V, nt, tri, nq, bary, w);
  if (rc) {
    mesh_free(&M);
    return rc;
  }
  double gx[OR_MAX_EDGE_PTS], gw[OR_MAX_EDGE_PTS];
  gauss01(n_edge, gx, gw);
  const ortable *E = mode == OR_MODE_TABLE ? etable : NULL;
  int err = 0;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < ns; ++s) {
    const int32_t *em = edges + 6 * rows[s], *en = edges + 6 * cols[s];
    const double lm = dist3(V + 3 * (size_t)em[0], V + 3 * (size_t)em[1]);
    const double ln = dist3(V + 3 * (size_t)en[0], V + 3 * (size_t)en[1]);
    cplx acc = 0.0;
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) {
        const int p = em[2 + u], a = em[4 + u], q = en[2 + v], b = en[4 + v];
        const double sg = (u == 0 ? 1.0 : -1.0) * (v == 0 ? 1.0 : -1.0);
        cplx X = 0.0;
        int r2 = angular_pair(&M, k, n_edge, gx, gw, E, p, q, a, b, &X);
        if (r2) {
#pragma omp atomic write
          err = r2;
        }
        acc += sg * X;
      }
    const cplx Z = (I * k * OR_ETA0 / (4.0 * M_PI)) * lm * ln * acc;
    out[2 * s] = creal(Z);
    out[2 * s + 1] = cimag(Z);
  }
  mesh_free(&M);
  return err;
}

/* Largest distance from a quadrature point to a vertex of another triangle:
 * the upper end of the Exp table for the angular scheme (the distance to a
 * point of an edge never exceeds the distance to one of its ends). */
int or_angular_rmax(int nv, const double *V, int nt, const int32_t *tri, int nq,
                    const double *bary, const double *w, double *rmax) {
  mesh M;
  int rc = mesh_init(&M, nv, V, nt, tri, nq, bary, w);
  if (rc) {
    mesh_free(&M);
    return rc;
  }
  double best = 0.0;
#pragma omp parallel for reduction(max : best) schedule(dynamic, 64)
  for (int p = 0; p < nt; ++p)
    for (int i = 0; i < nq; ++i) {
      const double *ri = qpt(&M, p, i);
      for (int v = 0; v < nv; ++v) {
        const double d = dist3(ri, V + 3 * (size_t)v);
        if (d > best) best = d;
      }
    }
  *rmax = best;
  mesh_free(&M);
  return 0;
}
