/*
 * momfill: EFIE impedance-matrix fill on RWG basis functions for one MI355X
 * (gfx950), with the adaptive interpolation tables of Exp(-jkr) and
 * Exp(-jkr)/r of S. Yang and D. Su, "Fast Green Function Evaluation for
 * Method of Moment" (Section II), beside a direct complex-exponential fill.
 *
 * Conventions
 *  - Time convention exp(+j omega t); free-space impedance eta0 = 376.730313668.
 *  - Z_mn = j k eta0/(4 pi) sum over the two triangles of m and of n of
 *      s s' l_m l_n /(A A') int int [ (r-v).(r'-v')/4 - 1/k^2 ] g(|r-r'|),
 *    g(R) = exp(-jkR)/R (Eq. (1)), with the symmetric triangle rule of
 *    quad_order points on both triangles.  Triangle pairs that share a vertex
 *    ("touching", including a triangle with itself) integrate 1/R in closed
 *    form and the remainder g - 1/R by the rule, then are symmetrised: this
 *    is the singularity cancellation the paper keeps for r < r_min
 *    (Section II-C).
 *  - RWG unknowns are the interior edges numbered in order of first
 *    appearance when triangles are scanned in index order and, inside a
 *    triangle, local edges 0,1,2 (local edge a is opposite vertex a).  T+ of
 *    an edge is the triangle running v_lo -> v_hi in its cyclic vertex order.
 *  - Z is row-major with leading dimension ldz (row = test edge), complex
 *    values as interleaved (re, im) pairs: MF_C64 (float) or MF_C128
 *    (double).  The arithmetic of regular triangle pairs is FP32; tables,
 *    distance range and touching pairs are FP64.
 *
 * Memory and streams
 *  - Arguments named *_dev are device pointers on the current HIP device;
 *    the others are host pointers.  The caller owns every byte of device
 *    memory: vertices, Z, gradients, and one workspace per mesh, per table
 *    set, per batch and per near-field pattern, each sized by its
 *    *_workspace_bytes query and handed over 256-byte aligned.  The library
 *    never allocates or frees device memory; a handle is host memory that
 *    views its workspace, which must outlive the handle's use, and its
 *    destroy call frees only the handle.
 *  - Every call enqueues its kernels on `stream` and returns without
 *    synchronising, except where it says it copies a result to the host.
 *
 * Errors: functions return MF_OK or a negative code and never throw;
 * mf_last_error() gives a message for the calling thread's last error.
 */
#ifndef MOMFILL_H
#define MOMFILL_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MF_OK = 0,
  MF_EINVAL = -1,    /* bad argument                                     */
  MF_EMESH = -2,     /* degenerate / non-manifold / inconsistent mesh     */
  MF_ERANGE = -3,    /* a regular-pair distance outside the table range   */
  MF_ENOMEM = -4,    /* device or host allocation failed                 */
  MF_EHIP = -5,      /* HIP runtime error                                */
  MF_ENOTCONV = -6   /* table probe check failed after 8 refinements      */
};

enum { MF_MODE_TABLE = 0, MF_MODE_DIRECT = 1 };
/* Debug bits OR-ed into mode: keep only the vector-potential term (A) or
 * only the scalar-potential term (PHI) of the bracket. */
enum { MF_PART_A = 0x10, MF_PART_PHI = 0x20 };
enum { MF_C64 = 0, MF_C128 = 1 };

typedef struct mf_mesh mf_mesh;
typedef struct mf_tables mf_tables;

/* Message for the last error of the calling thread ("" if none). */
const char *mf_last_error(void);

/* ---- mesh -------------------------------------------------------------
 * Validates the triangle list (host, n_triangles*3 vertex indices) and
 * builds the RWG edge table, the touching-pair lists and the tile plan on
 * the host (mf_mesh_set_workspace uploads them).  Only topology is fixed
 * here: vertex coordinates are
 * passed to every fill call (device, FP64), so one handle serves perturbed
 * geometries.  MF_EMESH for a repeated or out-of-range vertex index, an edge
 * shared by more than two triangles or two triangles running an edge the
 * same way. */
int mf_mesh_create(int32_t n_vertices, int32_t n_triangles, const int32_t *triangles,
                   mf_mesh **out);
void mf_mesh_destroy(mf_mesh *mesh);
/* Number of RWG unknowns (interior edges). */
int mf_mesh_n_edges(const mf_mesh *mesh, int32_t *n_edges);
/* Copies the edge table to the host: 6 ints per edge,
 * v_lo, v_hi, T+, T-, a+, a- (a = local index of the edge in T+/T-). */
int mf_mesh_edges(const mf_mesh *mesh, int32_t *edges);
/* Number of ordered touching triangle pairs (p, q sharing a vertex). */
int mf_mesh_n_touching(const mf_mesh *mesh, int64_t *n_pairs);
/* The tile plan of the regular fill: the RWG edges are cut into n_blocks
 * blocks of consecutive edges (at most 80 edges and 64 carrying triangles
 * each); every block pair I <= J is one tile, n_tiles = n_blocks (n_blocks
 * + 1)/2, and an off-diagonal tile also writes its transpose (Z = Z^T).
 * max_block_triangles is the largest number of triangles one block needs. */
int mf_mesh_plan(const mf_mesh *mesh, int32_t *n_blocks, int64_t *n_tiles,
                 int32_t *max_block_triangles);
/* The triangle-block plan of the table-mode fill (mf_fill_Z with
 * MF_MODE_TABLE and no MF_PART_ flag): blocks of at most 64 consecutive
 * triangles and 112 edges with a triangle in the block, one tile per block
 * pair I <= J (each unordered triangle pair evaluated once), the source
 * triangles of a block in rounds of at most 32 of which no two share an
 * edge.  n_cut edges have their two triangles in different blocks: their
 * entries are completed from a side buffer in the mesh workspace.  All four
 * outputs are 0 when the mesh has no such plan (then the edge-block plan
 * above serves table mode too). */
int mf_mesh_tb_plan(const mf_mesh *mesh, int32_t *n_blocks, int64_t *n_tiles, int32_t *n_cut,
                    int32_t *max_rounds);

/* Device workspace of a mesh: the topology, the tile plan, the per-triangle
 * records and FP64 quadrature points the kernels read, the touching-pair
 * blocks and small reduction and status words.  mf_mesh_set_workspace binds
 * workspace_dev (at least mf_mesh_workspace_bytes bytes, 256-byte aligned,
 * owned by the caller and kept until the mesh is destroyed or rebound) and
 * uploads the plan on `stream` (synchronises it).  Every call below that
 * runs on the GPU needs a bound workspace: MF_EINVAL otherwise, and for a
 * workspace that is too small or misaligned. */
int mf_mesh_workspace_bytes(const mf_mesh *mesh, size_t *bytes);
int mf_mesh_set_workspace(mf_mesh *mesh, void *workspace_dev, size_t bytes, hipStream_t stream);

/* ---- distance range (abstract; Section II-C) ---------------------------
 * Exact FP64 minimum and maximum of |r_{p,i} - r_{q,j}| over all vertex-
 * disjoint triangle pairs (p,q) and all pairs of quadrature points of the
 * quad_order rule; these bound every distance the regular fill looks up.
 * Copies the two values to the host (synchronises `stream`).  MF_EINVAL if
 * quad_order is not 3, 6 or 7 or the mesh has no vertex-disjoint pair;
 * MF_EMESH for a zero-area triangle. */
int mf_r_range(mf_mesh *mesh, const double *vertices_dev, int quad_order, double *r_min,
               double *r_max, hipStream_t stream);
/* For callers that cannot allocate device memory or hand over scratch: the
 * same range (bit-identical results) with the scan's scratch (four reduction
 * words and 32 bytes per run of 32 triangles) in a 4 MiB array the library
 * holds on each GPU it runs on until the process ends, so no workspace
 * beyond the mesh's inputs is touched and nothing is allocated.  Meshes of
 * more than 4,194,048 triangles are refused with MF_EINVAL.  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (two host
 * threads, or two streams) race and must be serialised by the caller. */
int mf_r_range_static(mf_mesh *mesh, const double *vertices_dev, int quad_order, double *r_min,
                      double *r_max, hipStream_t stream);

/* ---- tables (Section II-B, II-C; Eqs. (2), (4)-(6), (10)) --------------
 * Builds on the device, in FP64, the adaptive tables of Exp(-jkr) (linear
 * interpolation) and Exp(-jkr)/r (cubic Lagrange) over [r_min, r_max]:
 * uniform interval t from the error bound of Eq. (10) for relative error
 * tol (capped at a 32nd of a wavelength), refinement windows of half width
 * 2t with interval t/2 around every zero of the real or imaginary part,
 * forced samples at those zeros, a sample dropped when a higher-priority
 * one is closer than t/4, the hash of Eq. (6) with bucket width equal to the
 * smallest sample interval, and a probe check (8 points per interval and
 * r_max) that halves t^2 and rebuilds, at most 8 times, until the maximum
 * relative error is below tol.  Synchronises `stream` (the probe result
 * decides the loop).  The tables and the build's temporaries live in
 * workspace_dev (caller-owned, 256-byte aligned, at least
 * mf_tables_workspace_bytes(k, r_min, r_max, tol) bytes: a bound over the
 * eight possible refinements, a few MB for the benchmark sphere), which must
 * outlive the handle's use.  MF_EINVAL: k <= 0 or not finite, r_min <= 0,
 * r_max <= r_min, tol outside [1e-12, 1e-1], a NULL or misaligned workspace;
 * MF_ENOMEM if the workspace is smaller than the build needs; MF_ENOTCONV if
 * the probe check still fails. */
int mf_tables_workspace_bytes(double k, double r_min, double r_max, double tol, size_t *bytes);
int mf_build_tables(double k, double r_min, double r_max, double tol, void *workspace_dev,
                    size_t bytes, mf_tables **out, hipStream_t stream);
/* Frees the handle; the workspace is the caller's. */
void mf_tables_destroy(mf_tables *tables);
/* Sizes and parameters: samples of the Exp and Green tables, hash buckets
 * of each, their uniform intervals and the probe errors reached. */
int mf_tables_info(const mf_tables *tables, int32_t *n_exp, int32_t *n_green,
                   int32_t *m_exp, int32_t *m_green, double *t_exp, double *t_green,
                   double *err_exp, double *err_green);
/* Copies a table to the host: which = 0 Exp, 1 Green.  r: n doubles,
 * values: 2n doubles (re, im), hash: m ints (Eq. (6) array).  Any pointer
 * may be NULL.  Synchronises `stream`. */
int mf_tables_get(const mf_tables *tables, int which, double *r, double *values, int32_t *hash,
                  hipStream_t stream);
/* Interpolated values of a table at n device points r_dev (FP64 in, FP64
 * complex out, 2n doubles), through the same FP32 lookup and polynomial
 * evaluation the fill uses.  Points outside [r_min, r_max] give NaN. */
int mf_tables_eval(const mf_tables *tables, int which, int64_t n, const double *r_dev,
                   double *out_dev, hipStream_t stream);

/* ---- fill (Section II-A: the MoM matrix fill the tables accelerate) ------
 * Z (device) receives all n_edges x n_edges entries of the EFIE matrix in
 * the convention above: every regular point pair takes exp(-jkR)/R (Eq. (1))
 * from the cubic Lagrange table of Eq. (5), located through the hash of
 * Eq. (6) (MF_MODE_TABLE), or computed (MF_MODE_DIRECT, the plain method the
 * paper compares against); touching pairs use singularity cancellation in
 * FP64 (Section II-C).  Direct mode keeps the cancellation of the four
 * triangle-pair terms of distant entries exact: each pair's phase is split
 * about its FP64 centroid distance d and the reference exp(-jkd)/d of the
 * div-div term is summed over the four pairs in FP64.  mode: MF_MODE_TABLE
 * (Green function from `tables`, which must cover the mesh's distance
 * range) or MF_MODE_DIRECT (exp(-jkR)/R evaluated per point pair; tables
 * may be NULL), optionally OR-ed with MF_PART_A or MF_PART_PHI.  A regular
 * distance outside the table range by more than FP32 rounding is reported
 * as MF_ERANGE by mf_sync_status. */
int mf_fill_Z(mf_mesh *mesh, const double *vertices_dev, double k, int quad_order, int mode,
              const mf_tables *tables, void *Z_dev, int z_dtype, int64_t ldz,
              hipStream_t stream);

/* ---- tuner ---------------------------------------------------------------
 * A full EFIE fill (table or direct mode, no MF_PART_ flags) can run on three
 * kernels: 0, the triangle-block tiling
 * (mf_mesh_tb_plan) with 1024 threads per workgroup (16 waves, two source
 * triangles per wave and round); 1, the same tiling with 512 threads (8 waves,
 * four source triangles per wave and round, twice the registers per lane);
 * 2, the edge-block tiling (mf_mesh_plan), which repeats the pairs its blocks
 * share but needs no cut-edge fix-up (partial fills always run on it).  In
 * direct mode the fix-up also adds, in FP64, the reference part of the
 * entries of cut edges.  mf_fill_tune runs the fill of its
 * arguments (those of mf_fill_Z, MF_PART_ flags excluded) once per kernel to
 * warm up and once timed with HIP events, keeps the fastest for later
 * mf_fill_Z calls on this mesh in that mode and records it under (triangles, edges,
 * rule, mode, output type, table placement) for the process and, when the
 * environment variable MOMFILL_TUNE_CACHE names a file, in that file, so that
 * later processes take the choice without timing.  *choice receives the
 * kernel; ms (3 floats, may be NULL) the timings in milliseconds, zeros when
 * the cache answered.  Z holds the fill when the call returns (synchronous).
 * A mesh without a triangle-block plan has one kernel (choice 2, no timing).
 * mf_fill_Z on a mesh that was not tuned takes the cached choice for its key,
 * else kernel 0. */
int mf_fill_tune(mf_mesh *mesh, const double *vertices_dev, double k, int quad_order, int mode,
                 const mf_tables *tables, void *Z_dev, int z_dtype, int64_t ldz,
                 hipStream_t stream, int32_t *choice, float *ms);
/* Description of a kernel choice (static string). */
const char *mf_fill_choice_name(int32_t choice);
/* Pins the kernel of this mesh's full mf_fill_Z calls (both modes) to `choice`
 * (0, 1 or 2 as above; for callers that tune by their own measurements or
 * reproduce a given kernel), or with -1 returns to the cached choice or
 * kernel 0.  A mesh without a triangle-block plan runs kernel 2 whatever is
 * pinned.  MF_EINVAL for another value. */
int mf_mesh_set_fill_choice(mf_mesh *mesh, int32_t choice);

/* ---- MFIE fill (Section IV-B: the K operator beside the EFIE) -----------
 * Z_dev receives the MFIE matrix of the closed PEC surface, tested with the
 * RWG functions themselves (n the unit normal (x1 - x0) x (x2 - x0) of each
 * triangle, outward for counter-clockwise triangles seen from outside):
 *   Z_mn = <f_m, f_n>/2 + (1/4 pi) int int f_m . n x (f_n x grad' G) ...
 *        = <f_m, f_n>/2 - <f_m, n x PV int grad G x f_n dS'>,
 * G = exp(-jkR)/(4 pi R), so that Z I = <f_m, n x H_inc> (mf_rhs_planewave_mfie).
 * Regular pairs use the kernel (1 + jkR) exp(-jkR)/R^3 = (1/R + jk) g/R
 * with g from the Green table (MF_MODE_TABLE) or computed (MF_MODE_DIRECT);
 * touching pairs take their singular part in closed form in FP64.  The
 * matrix is not symmetric: every entry is computed.  mode is MF_MODE_TABLE
 * or MF_MODE_DIRECT (no MF_PART_ flags); the other arguments, the checks
 * and the MF_ERANGE report are those of mf_fill_Z. */
int mf_fill_mfie(mf_mesh *mesh, const double *vertices_dev, double k, int quad_order, int mode,
                 const mf_tables *tables, void *Z_dev, int z_dtype, int64_t ldz,
                 hipStream_t stream);

/* ---- angular-transformation fill (Section II-A) --------------------------
 * The paper's own inner scheme: for every test point r (the quad_order rule
 * on the test triangle) and every source triangle, touching or not, the
 * inner integrals I0 = int_q exp(-jkR)/R dS' and I1 = int_q (r' - rho0)
 * exp(-jkR)/R dS' (rho0 the projection of r on the source plane) become sums
 * over the three source edges: polar coordinates about rho0 make the radial
 * integral exact (R dR = rho drho), and I1 is (j/k) times the boundary
 * integral of exp(-jkR) times the outward edge normal.  Each edge takes
 * n_edge (4, 6 or 8) Gauss-Legendre points in u, l = d sinh u along the edge
 * (d the distance from r to the edge's line), and one exp(-jkR) per point
 * serves both integrals: from the linear Exp table (MF_MODE_TABLE; built by
 * mf_build_exp_table over [0, r_max] with r_max from mf_angular_rmax) or
 * computed (MF_MODE_DIRECT; tables may be NULL).  The integrals are FP64;
 * entries are accumulated in FP32 and written as z_dtype.  Z_dev receives all
 * n_edges x n_edges entries of the EFIE matrix in the units of mf_fill_Z
 * (the scheme is not symmetric, every entry is computed).  A distance beyond
 * the table's r_max is reported as MF_ERANGE by mf_sync_status. */
int mf_fill_angular(mf_mesh *mesh, const double *vertices_dev, double k, int quad_order,
                    int n_edge, int mode, const mf_tables *exp_table, void *Z_dev, int z_dtype,
                    int64_t ldz, hipStream_t stream);
/* Largest distance (FP64, exact) from a quadrature point of the quad_order
 * rule to a mesh vertex: every distance the angular fill evaluates is at
 * most this (the distance to a point of an edge never exceeds that to one of
 * its ends).  *r_max is host memory; synchronises `stream`. */
int mf_angular_rmax(mf_mesh *mesh, const double *vertices_dev, int quad_order, double *r_max,
                    hipStream_t stream);
/* The linear Exp(-jkr) table alone (Sections II-B, II-C) over [0, r_max]:
 * Exp(-jkr) has no singularity at the origin, so the table starts at 0.
 * Same placement, hash and probe check as mf_build_tables; the Green table
 * is not built (mf_fill_Z, mf_fill_mfie, the batch, the near field and the
 * adjoint reject such tables). */
int mf_exp_table_workspace_bytes(double k, double r_max, double tol, size_t *bytes);
int mf_build_exp_table(double k, double r_max, double tol, void *workspace_dev, size_t bytes,
                       mf_tables **out, hipStream_t stream);

/* ---- batched fill (frequency sweeps, several meshes) --------------------
 * One persistent fill launch over n items, item i being (meshes[i],
 * vertices_dev[i], k[i], tables[i], Z_dev[i] with leading dimension
 * ldz[i]): the workgroups walk one tile list spanning every item, so items
 * of uneven size share the GPU without a tail per item.  All items share
 * quad_order, mode and z_dtype; items that share a mesh handle must share
 * its vertex pointer (one geometry pass per mesh).  mf_batch_create checks
 * the items as mf_fill_Z does, places the per-item touching-pair blocks and
 * the item list in workspace_dev (caller-owned, 256-byte aligned, at least
 * mf_batch_workspace_bytes(n, meshes) bytes) and copies the item list there
 * (synchronous); the meshes, tables, vertices, outputs and workspace must
 * outlive the batch.  MF_EINVAL for n < 1, a NULL array, a short or
 * misaligned workspace or any item mf_fill_Z would reject. */
typedef struct mf_batch mf_batch;
int mf_batch_workspace_bytes(int32_t n, mf_mesh *const *meshes, size_t *bytes);
int mf_batch_create(int32_t n, mf_mesh *const *meshes, const double *const *vertices_dev,
                    const double *k, const mf_tables *const *tables, int quad_order, int mode,
                    void *const *Z_dev, int z_dtype, const int64_t *ldz, void *workspace_dev,
                    size_t workspace_bytes, mf_batch **out);
/* Enqueues the batch on `stream`: geometry once per distinct mesh, the
 * touching-pair blocks of every item, then the single fill launch.  It
 * allocates nothing and copies nothing, so a HIP graph can capture it. */
int mf_batch_fill(mf_batch *batch, hipStream_t stream);
/* Tile-shape tuner.  mf_batch_create, before returning, fills the batch once
 * on the null stream and times the persistent launch with each candidate
 * tile shape: edge-block tiles (runs of at most 80 edges, the tiles of
 * neighbouring blocks sharing triangles) with 512, 768 and 1024 threads per
 * workgroup (2, 3 or 4 waves per SIMD: each lane's register budget against
 * the latency hiding of the table gathers), and, when every item's mesh has
 * a triangle-block plan (mf_mesh_tb_plan), triangle-block tiles (each
 * unordered triangle pair evaluated once, cut edges completed by a fix-up
 * per item) with 1024 and 512 threads (two or four source triangles per
 * wave and round).  It keeps the fastest; the choice is cached per (quad_order,
 * mode, table placement, z_dtype, plan availability) for the process and
 * in the MOMFILL_TUNE_CACHE file when it is set (as for mf_fill_tune), so
 * later batches of the same kind skip the timing.  The outputs hold the
 * batch's result when mf_batch_create returns.  mf_batch_info reports the
 * choice (*threads, *tile_shape: 0 edge blocks, 1 triangle blocks) and the
 * five timings in milliseconds in the order above (tune_ms5; zeros for the
 * candidates not run and when the cache answered); any pointer may be
 * NULL.  With triangle-block plans the workspace holds a cut-edge side
 * buffer per item, 8 n_cut (E + n_cut) bytes. */
int mf_batch_info(const mf_batch *batch, int32_t *threads, int32_t *tile_shape,
                  float *tune_ms5);
/* Pins the batch's launch to candidate `choice` of the tuner's list (0-2:
 * edge blocks at 512, 768, 1024 threads; 3, 4: triangle blocks at 1024, 512
 * threads) for its later mf_batch_fill calls, for tests and measurements.
 * MF_EINVAL for an index out of range or triangle blocks without plans. */
int mf_batch_set_choice(mf_batch *batch, int32_t choice);
void mf_batch_destroy(mf_batch *batch);

/* ---- near-field fill (Section II-A) --------------------------------------
 * With a fast method (MLFMA, pFFT, AIM) only the near-field interactions
 * are filled directly.  Here two RWG unknowns are near when the midpoints
 * of their edges are at most r_near apart (every unknown is near itself).
 * mf_near_create builds, on the host, the CSR pattern of those pairs from
 * the host vertex array (n_vertices*3 doubles) and the list of edge-block
 * tiles that hold a near pair; mf_near_set_workspace uploads the tile lists
 * into workspace_dev (caller-owned, 256-byte aligned, at least
 * mf_near_workspace_bytes bytes; synchronises `stream`) before the first
 * mf_fill_near.  The pattern keeps the mesh handle, which must outlive it.
 * MF_EINVAL for r_near <= 0 or more than 2^31 pairs. */
typedef struct mf_near mf_near;
int mf_near_create(mf_mesh *mesh, const double *vertices_host, double r_near, mf_near **out);
int mf_near_workspace_bytes(const mf_near *pattern, size_t *bytes);
int mf_near_set_workspace(mf_near *pattern, void *workspace_dev, size_t bytes,
                          hipStream_t stream);
/* Number of near pairs and of tiles the near fill runs over. */
int mf_near_info(const mf_near *pattern, int64_t *nnz, int64_t *n_tiles);
/* Host copy of the pattern: row_ptr (n_edges + 1 int64), col (nnz int32,
 * ascending within a row). */
int mf_near_pattern(const mf_near *pattern, int64_t *row_ptr, int32_t *col);
/* values_dev[i] (nnz complex values, MF_C64 or MF_C128) receives Z at the
 * i-th CSR position: the same entries mf_fill_Z computes, from the same
 * kernels run over the near tiles only.  Arguments as for mf_fill_Z; the
 * pattern must belong to `mesh`. */
int mf_fill_near(mf_mesh *mesh, mf_near *pattern, const double *vertices_dev, double k,
                 int quad_order, int mode, const mf_tables *tables, void *values_dev,
                 int z_dtype, hipStream_t stream);
void mf_near_destroy(mf_near *pattern);

/* ---- plane-wave scattering (Section IV-B) --------------------------------
 * Excitation of the EFIE system for E_inc(r) = E0 exp(-j k khat.r):
 *   out_dev[m] = int f_m . E_inc dS,
 * with the quad_order rule on each triangle, in FP64 (stored as z_dtype).
 * khat: host, 3 doubles (unit vector); E0: host, 3 complex as (re, im)
 * pairs.  k = 0 gives the static excitation. */
int mf_rhs_planewave(mf_mesh *mesh, const double *vertices_dev, double k, int quad_order,
                     const double *khat, const double *E0, void *out_dev, int z_dtype,
                     hipStream_t stream);
/* MFIE excitation (FP64): out_dev[m] = int f_m . (n x H_inc) dS with
 * H_inc = (khat x E0) exp(-j k khat.r) / eta0 and n the unit normal
 * (x1 - x0) x (x2 - x0) of each triangle; arguments as mf_rhs_planewave. */
int mf_rhs_planewave_mfie(mf_mesh *mesh, const double *vertices_dev, double k, int quad_order,
                          const double *khat, const double *E0, void *out_dev, int z_dtype,
                          hipStream_t stream);
/* Far field of the currents I_dev (n_edges values of z_dtype) in the
 * n_dirs unit directions dirs_dev (device, n_dirs*3 doubles), in FP64:
 *   F_dev[d] = sum_n I_n int f_n exp(+j k rhat_d.r') dS'   (3 complex, (re, im) pairs)
 * and, when sigma_dev is not NULL, the bistatic cross-section
 *   sigma_dev[d] = (k eta0)^2/(4 pi) |F - rhat (rhat.F)|^2 / e0_norm^2
 * (the scattered field being E = -j k eta0 exp(-jkr)/(4 pi r) (F - rhat (rhat.F))). */
int mf_far_field(mf_mesh *mesh, const double *vertices_dev, double k, int quad_order,
                 const void *I_dev, int z_dtype, int32_t n_dirs, const double *dirs_dev,
                 double e0_norm, double *F_dev, double *sigma_dev, hipStream_t stream);

/* ---- adjoint ------------------------------------------------------------
 * Gradient of L = Re sum_mn conj(W_mn) Z_mn, W = dLdZ_dev (same dtype and
 * layout as Z), with respect to the vertex coordinates (dL_dvertices_dev,
 * n_vertices*3 doubles, overwritten) and k (dL_dk_dev, one double,
 * overwritten).  Table mode uses the tables as constants: dG/dR from the
 * derivative of the cubic and dG/dk = -j Exp(-jkR) from the linear Exp
 * table; direct mode differentiates exp(-jkR)/R. */
int mf_fill_Z_backward(mf_mesh *mesh, const double *vertices_dev, double k, int quad_order,
                       int mode, const mf_tables *tables, const void *dLdZ_dev, int z_dtype,
                       int64_t ldz, double *dL_dvertices_dev, double *dL_dk_dev,
                       hipStream_t stream);

/* Phase timing.  With mf_set_timing(1), every mf_fill_Z records HIP events
 * on its stream around its phases; mf_mesh_timings waits for the last fill
 * on `mesh` and writes milliseconds: ms[0] geometry preparation, ms[1]
 * touching pairs (FP64), ms[2] regular-pair tile fill.  MF_EINVAL if no
 * timed fill has run on the mesh. */
void mf_set_timing(int on);
int mf_mesh_timings(mf_mesh *mesh, float *ms3);
/* The regular-fill phase of the last timed fill split in two: ms2[0] the
 * tile kernel, ms2[1] the cut-edge fix-up of the triangle-block plan (0 when
 * the fill ran on another kernel, then ms2[0] is the whole phase). */
int mf_mesh_fill_timings(mf_mesh *mesh, float *ms2);

/* Synchronises `stream` and returns a deferred device-side status of the
 * last fill on this mesh (MF_ERANGE) or MF_OK. */
int mf_sync_status(mf_mesh *mesh, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
