/*
 * FP64 CPU oracle for the EFIE Galerkin impedance-matrix fill accelerated by
 * adaptive one-dimensional interpolation tables of Exp(-jkr) and Exp(-jkr)/r
 * (S. Yang, D. Su, "Fast Green Function Evaluation for Method of Moment").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the smoke
 * check and the benchmark's CPU-baseline leg can check the GPU library against
 * a plain, slow, obviously correct implementation.  The product path never
 * links, loads or calls it, and it shares no source with the GPU library.
 *
 * All arithmetic is IEEE double, round to nearest, no FMA contraction.
 * Return codes: 0 ok, -1 bad argument, -2 bad mesh, -3 distance outside the
 * table range, -4 out of memory, -6 table probe check did not converge.
 */
#ifndef MOMFILL_ORACLE_H
#define MOMFILL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Symmetric triangle rule with q in {3,6,7} points: barycentrics (q*3) and
 * weights summing to one. Returns q, or -1 for an unsupported q. */
int or_quad_rule(int q, double *bary, double *w);

/* RWG unknowns of a triangle mesh.  Interior edges (exactly two triangles)
 * are numbered in order of first appearance when triangles are scanned in
 * index order and, inside a triangle, local edges a = 0,1,2 (local edge a is
 * the one opposite vertex a).  Per edge, 6 ints: v_lo, v_hi, T+, T-, a+, a-
 * (a+- = local index of the edge in T+- = index of the free vertex).  T+ is
 * the triangle that runs v_lo -> v_hi in its cyclic vertex order.
 * edges must hold 6*floor(3*nt/2) ints. */
int or_rwg(int nv, int nt, const int32_t *tri, int32_t *n_edges, int32_t *edges);

/* Potentials of a flat triangle with unit density at point r:
 * S = int 1/|r-r'| dS',  V = int (r'-r)/|r-r'| dS'. */
void or_tri_potentials(const double *x0, const double *x1, const double *x2,
                       const double *r, double *S, double *V);

/* (exp(-jkR) - 1)/R, the smooth remainder after removing 1/R. */
void or_ghat(double k, double R, double *re, double *im);

/* Exact FP64 min/max of |r_{p,i} - r_{q,j}| over all regular (vertex-disjoint)
 * triangle pairs and all quadrature-point pairs of the given rule. */
int or_r_range(int nv, const double *V, int nt, const int32_t *tri, int nq,
               const double *bary, const double *w, double *rmin, double *rmax);

/* ---- adaptive tables (Section II-B/C, Eqs. (2)-(6), (10)) ---- */
typedef struct ortable ortable;

#define OR_TABLE_EXP   0   /* Exp(-jkr), linear interpolation, Eq. (4)     */
#define OR_TABLE_GREEN 1   /* Exp(-jkr)/r, cubic Lagrange, Eq. (5)         */

/* Build a table over [rmin, rmax].  If t > 0 that uniform interval is used
 * as given and no probe loop runs; otherwise t comes from tol and the probe
 * check shrinks it by sqrt(2) up to 8 times.  refine != 0 enables the local
 * refinement windows around zeros and zeros != 0 forces zero samples.
 * mu: merge distance in units of t; win: window half width in units of t;
 * ratio: refined interval in units of t. */
int or_table_build(int kind, double k, double rmin, double rmax, double tol,
                   double t, int refine, int zeros, double mu, double win,
                   double ratio, ortable **out);
/* Test hook: a table over the given ascending nodes and complex values. */
int or_table_from_nodes(int kind, int n, const double *r, const double *fre,
                        const double *fim, ortable **out);
void or_table_free(ortable *t);
/* n, number of hash buckets, t, bucket width, probe error, iterations. */
void or_table_info(const ortable *t, int32_t *n, int32_t *m, double *t_used,
                   double *delta, double *probe_err, int32_t *iters);
/* Copies node positions (n), values (2n, re/im interleaved), hash (m). */
void or_table_get(const ortable *t, double *r, double *f, int32_t *hash);
/* Interval index by the hash of Eq. (6) with the fix-ups; -3 if r outside. */
int or_table_lookup(const ortable *t, double r, int32_t *idx);
/* Interpolated values at n points (2n doubles out). */
int or_table_eval(const ortable *t, int n, const double *r, double *out);

/* ---- impedance matrix ---- */
#define OR_MODE_TABLE  0
#define OR_MODE_DIRECT 1
#define OR_PART_ALL    0
#define OR_PART_A      1   /* vector-potential term only  */
#define OR_PART_PHI    2   /* scalar-potential term only  */
#define OR_FORCE_TOUCHING 4 /* or_pair_block only: singular rule on any pair */

/* Entries Z[rows[s], cols[s]] (complex, 2 doubles each), defined per entry
 * as the sum of four triangle-pair integrals.  gtable may be NULL for
 * direct mode. */
int or_fill_entries(int nv, const double *V, int nt, const int32_t *tri,
                    int ne, const int32_t *edges, double k, int nq,
                    const double *bary, const double *w, int mode, int part,
                    const ortable *gtable, int64_t ns, const int64_t *rows,
                    const int64_t *cols, double *out);

/* Rows [r0, r1) of Z (out: (r1-r0) x ne complex, interleaved) in triangle-
 * pair order: every pair's kernel values are evaluated once for its nine
 * local entries (the CPU baseline of the fill; same values as
 * or_fill_entries up to rounding order). */
int or_fill_rows(int nv, const double *V, int nt, const int32_t *tri, int ne,
                 const int32_t *edges, double k, int nq, const double *bary,
                 const double *w, int mode, int part, const ortable *gtable, int r0,
                 int r1, double *out);

/* Normalised local 3x3 block of one ordered triangle pair (p,q):
 * X[a][b] = (1/(A_p A_q)) int_p int_q [(r-v_a).(r'-v_b)/4 - 1/k^2] g dS' dS
 * by the quadrature of the fill (symmetrised for touching pairs). */
int or_pair_block(int nv, const double *V, int nt, const int32_t *tri, int p,
                  int q, double k, int nq, const double *bary, const double *w,
                  int mode, int part, const ortable *gtable, double *out18);

/* L = Re sum_mn conj(W_mn) Z_mn in direct mode, W row-major complex
 * (2*ne*ne doubles).  or_loss_local sums only the entries whose row or
 * column edge lies on a triangle containing vertex v: moving v changes no
 * other entry, so differences of it in v equal differences of L. */
int or_loss(int nv, const double *V, int nt, const int32_t *tri, int ne, const int32_t *edges,
            double k, int nq, const double *bary, const double *w, const double *W, double *L);
int or_loss_local(int nv, const double *V, int nt, const int32_t *tri, int ne,
                  const int32_t *edges, double k, int nq, const double *bary, const double *w,
                  const double *W, int v, double *L);

/* Number of threads the OpenMP loops use. */
void or_set_threads(int n);
int or_max_threads(void);

/* MFIE (magnetic-field) operator, FP64 direct exponential.
 * Gradient of the triangle potential S at r (g: 3 doubles). */
void or_grad_potential(const double *x0, const double *x1, const double *x2, const double *r,
                       double *g);
/* Pair block X[a][b] of the K operator (see oracle.c), 9 complex; a
 * non-zero force_touching applies the singularity-subtracted rule to any
 * pair (test hook). */
int or_mfie_pair_block(int nv, const double *V, int nt, const int32_t *tri, int p, int q, double k,
                       int nq, const double *bary, const double *w, int force_touching,
                       double *out18);
/* MFIE matrix entries Z = <f_m, f_n>/2 - K_mn at (rows[s], cols[s]). */
int or_mfie_entries(int nv, const double *V, int nt, const int32_t *tri, int ne,
                    const int32_t *edges, double k, int nq, const double *bary, const double *w,
                    int mode, const ortable *gtable, int64_t ns, const int64_t *rows,
                    const int64_t *cols, double *out);

#ifdef __cplusplus
}
#endif

/* EFIE inner integrals by the angular transformation (Section II-A):
 * out8 = I0 = int_q exp(-jkR)/R dS' (re, im) and I1 = int_q (r' - rho0)
 * exp(-jkR)/R dS' (three complex), rho0 the projection of r on the plane,
 * n Gauss-Legendre points per edge (1..16); mode OR_MODE_TABLE reads
 * exp(-jkR) from the linear Exp table etable. */
int or_angular_inner(const double *x0, const double *x1, const double *x2, const double *r,
                     double k, int n, int mode, const ortable *etable, double *out8);
/* EFIE entries with every inner integral by the angular transformation. */
int or_angular_entries(int nv, const double *V, int nt, const int32_t *tri, int ne,
                       const int32_t *edges, double k, int nq, const double *bary, const double *w,
                       int n_edge, int mode, const ortable *etable, int64_t ns,
                       const int64_t *rows, const int64_t *cols, double *out);
/* Largest quadrature-point-to-vertex distance (the Exp table's upper end). */
int or_angular_rmax(int nv, const double *V, int nt, const int32_t *tri, int nq,
                    const double *bary, const double *w, double *rmax);
#endif
