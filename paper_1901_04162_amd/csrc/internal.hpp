// Internal declarations shared by the host and device sources of libmomfill.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "momfill.h"

namespace mf {

constexpr double kEta0 = 376.730313668;  // free-space wave impedance
constexpr int kMaxQ = 7;
// Operator of a fill: the EFIE (L operator) or the MFIE (K operator plus the
// identity term).  kModeMfie marks an MFIE fill in the internal mode word.
enum { MF_OP_EFIE = 0, MF_OP_MFIE = 1 };
constexpr int kModeMfie = 0x100;
constexpr int kMaxBlockEdges = 80;  // RWG edges per row/column block of a tile
constexpr int kMaxBlockTris = 64;   // triangles carrying a block's edges (one per lane)
// Triangle-block plan (table-mode fill): blocks of at most 64 consecutive
// triangles and 112 block edges (edges with a triangle in the block), the
// source triangles of a block in rounds of at most 32 pairwise non-adjacent
// triangles, at most kTBMaxRounds rounds.
constexpr int kTBTris = 64;
constexpr int kTBEdges = 112;
constexpr int kTBRound = 32;
constexpr int kTBMaxRounds = 12;
// The MFIE tile (edge blocks, 8 waves) walks each block's source triangles
// in rounds of at most kEBRound pairwise non-adjacent triangles.
constexpr int kEBRound = 8;
constexpr int kEBMaxRounds = 16;

// Per-triangle record read by the regular-pair kernel (72 floats, 288 B):
//  [0,21)  rho_i = r_i - c      (i-major, xyz)           FP32
//  [21,42) w_i rho_i                                       FP32
//  [42,51) alpha_a = c - v_a   (a-major, xyz)             FP32
//  [51,54) sigma_a = s_a l_a  (0 for a boundary edge)    FP32
//  [54,60) centroid c as three doubles                    FP64
//  [60,63) vertex indices                                 int32
//  63      radius of the quadrature points about c, rounded up  FP32
//  [64,71) |rho_i|^2, the squared offsets (a source triangle's, read by the
//          table-mode moments through scalar loads)                 FP32
constexpr int kRecFloats = 72;
constexpr int kRecRho = 0, kRecWRho = 21, kRecAlpha = 42, kRecSigma = 51, kRecCent = 54,
              kRecVid = 60, kRecRad = 63, kRecRho2 = 64;

// Carves a caller-owned device workspace into arrays: `bottom` takes space
// from the low end (arrays that outlive a call), `top` from the high end
// (temporaries, released by restoring `hi`).  Every array starts on a
// 256-byte boundary of the workspace (whose base must be 256-byte aligned).
// With base == nullptr and size == SIZE_MAX it only counts: `lo` then ends
// as the bytes a workspace needs for the same sequence of bottom calls.
struct Arena {
  char *base = nullptr;
  size_t size = 0, lo = 0, hi = 0;
  Arena() = default;
  Arena(void *b, size_t n) : base((char *)b), size(n), lo(0), hi(n) {}
  static Arena counter() { return Arena(nullptr, SIZE_MAX); }
  static size_t up(size_t x) { return (x + 255) & ~(size_t)255; }
  template <class T>
  bool bottom(T **p, size_t count) {
    const size_t a = up(lo), b = up(sizeof(T) * (count ? count : 1));
    if (a > hi || b > hi - a) return false;
    lo = a + b;
    *p = base ? (T *)(base + a) : nullptr;
    return true;
  }
  template <class T>
  bool top(T **p, size_t count) {
    const size_t b = up(sizeof(T) * (count ? count : 1));
    if (b > hi || hi - b < up(lo)) return false;
    hi = (hi - b) & ~(size_t)255;
    *p = base ? (T *)(base + hi) : nullptr;
    return true;
  }
};

struct Rule {
  int nq = 0;
  double bary[kMaxQ][3] = {};
  double w[kMaxQ] = {};
};
bool make_rule(int q, Rule *r);

}  // namespace mf

struct mf_tables {
  double k = 0, rmin = 0, rmax = 0, tol = 0;
  mf::Arena arena;  // over the caller's workspace; the arrays below live in it
  struct One {
    int n = 0, m = 0, iters = 0;
    double t = 0, delta = 0, err = 0;
    double *r = nullptr;     // FP64 nodes (device)
    double *f = nullptr;     // FP64 values, 2n (device)
    int32_t *hash = nullptr; // Eq. (6) array (device)
    // FP32 lookup (device): mb bucket records of 16 bytes (lookup.hpp) with
    // bucket coordinate x = r*binv + bbias clamped to [0, btop], and the
    // interval coefficients: Green 2(n-1) records, (c0,c1) then (c2,c3)
    // about each interval's first sample; Exp n-1 records {E_i, slope}.
    int4 *look = nullptr;
    int mb = 0;
    float binv = 0.0f, bbias = 0.0f, btop = 0.0f;
    // Green table only: the one-sample bucket records the fill kernels read
    // (look_offset1 in lookup.hpp), width just under the smallest interval
    int4 *look1 = nullptr;
    int mb1 = 0;
    float binv1 = 0.0f, bbias1 = 0.0f, btop1 = 0.0f;
    float4 *coef = nullptr;
    // FP64 lookup of the Exp table: m64 bucket records of 64 bytes, bucket
    // b = (int)(r * inv64) of width just under the smallest sample interval,
    // so at most one sample (split) lies inside a bucket: {split, x_b, the
    // value at x_b of the interval left of split and of the one right of it
    // (2 + 2 doubles), then the two intervals' slopes as 4 floats}; a lookup
    // evaluates E + slope (r - x_b)
    double *look64 = nullptr;
    int m64 = 0;
    double inv64 = 0.0;
  } e, g;
};

struct mf_mesh {
  int nv = 0, nt = 0, ne = 0;
  std::vector<int32_t> tri;        // nt*3
  std::vector<int32_t> edges;      // ne*6
  std::vector<int32_t> tedge;      // nt*3 global edge of local edge a, -1 if boundary
  std::vector<int8_t> tsign;       // nt*3 +1 (T+), -1 (T-), 0
  std::vector<int32_t> touch_off;  // nt+1 CSR of touching q per p (sorted)
  std::vector<int32_t> touch_q;
  std::vector<int32_t> touch_rev;  // index of (q,p) for pair (p,q)
  std::vector<int32_t> touch_p;    // p of each touching pair
  std::vector<int32_t> touch_u;    // the pairs with p <= q (each unordered pair once)
  std::vector<int32_t> blk_e0;     // nblk+1: first edge of each block
  std::vector<int32_t> blk_off;    // nblk+1: triangles needed by each edge block
  std::vector<int32_t> blk_tri;
  std::vector<int32_t> blk_pos;    // packed local-edge positions inside the block
  // nblk*kMaxBlockEdges: for row r of block b, the positions in the block's
  // triangle list of the row edge's T+ (bits 0-7) and T- (bits 8-15)
  std::vector<int32_t> blk_rt;
  // per block, positions in its triangle list in round order (block_rounds),
  // and nblk*(kEBMaxRounds+1) round starts
  std::vector<int32_t> blk_ord, blk_rounds;
  std::vector<int32_t> tiles;      // (I << 16) | J for every block pair I <= J
  int nblk = 0, max_blk_tris = 0;

  // Triangle-block plan: block b holds triangles [tb_t0[b], tb_t0[b+1]) and
  // owns the edges [tb_e0[b], tb_e0[b+1]) (those first seen in its
  // triangles); its block edges are the owned edges (local index e - e0)
  // followed by the non-owner halves of cut edges owned by earlier blocks.
  bool tb_ok = false;
  int fill_choice[2] = {-1, -1};   // tuned kernel of single fills per mode (-1: cache/default)
  int tb_nblk = 0, n_cut = 0;
  std::vector<int32_t> tb_t0, tb_e0;
  std::vector<int32_t> tb_nbe;       // block edges per block
  std::vector<int32_t> tb_be_off;    // nblk+1 CSR of the non-owner halves' cut indices
  std::vector<int32_t> tb_be_cut;
  std::vector<int32_t> tb_pos;       // nt: packed local block-edge index of local edges 0..2
  std::vector<int32_t> tb_order;     // nt: triangles of each block in round order
  std::vector<int32_t> tb_rounds;    // nblk*(kTBMaxRounds+1) round starts in the block's order
  std::vector<int32_t> tb_tiles;     // (I << 16) | J, I <= J
  std::vector<int32_t> cut_idx;      // ne: index of a cut edge, -1 if interior to a block
  std::vector<int32_t> cut_edge;     // n_cut: edge of each cut index

  // device copies
  int32_t *d_tri = nullptr, *d_tedge = nullptr;
  int32_t *d_edges = nullptr;      // ne*6, as edges
  int8_t *d_tsign = nullptr;
  int32_t *d_touch_off = nullptr, *d_touch_q = nullptr, *d_touch_rev = nullptr;
  int32_t *d_touch_p = nullptr;    // p of each touching pair
  int32_t *d_touch_u = nullptr;    // touch_u
  int32_t *d_blk_off = nullptr, *d_blk_tri = nullptr, *d_blk_pos = nullptr;
  int32_t *d_tiles = nullptr, *d_blk_e0 = nullptr, *d_blk_rt = nullptr;
  int32_t *d_blk_ord = nullptr, *d_blk_rounds = nullptr;
  float *d_elen = nullptr;         // ne edge lengths (FP32, from the FP64 vertices)
  float *d_rec = nullptr;          // nt * kRecFloats
  double *d_qp64 = nullptr;        // nt * kMaxQ * 3 quadrature points (FP64)
  double *d_brad = nullptr;        // nt*4: radius of the quadrature points about the centroid, unit normal
  double *d_sing1 = nullptr;       // one-way touching blocks: npairs*9*2
  float *d_sing = nullptr;         // symmetrised, FP32 complex: npairs*9*2
  unsigned long long *d_scratch = nullptr;  // small reductions and flags
  int *d_status = nullptr;
  double *d_sph = nullptr;         // range scan: bounding spheres of 32-triangle runs
  int32_t *d_tb_t0 = nullptr, *d_tb_e0 = nullptr, *d_tb_nbe = nullptr, *d_tb_be_off = nullptr,
          *d_tb_be_cut = nullptr, *d_tb_pos = nullptr, *d_tb_order = nullptr,
          *d_tb_rounds = nullptr, *d_tb_tiles = nullptr, *d_cut_idx = nullptr,
          *d_cut_edge = nullptr;
  float *d_side = nullptr;         // n_cut x (ne + n_cut) complex: cut-edge partial entries
  void *ws = nullptr;              // the caller's device workspace (mf_mesh_set_workspace)
  size_t ws_bytes = 0;
  // phase events of a timed fill: ev[0..3] around geometry, touching pairs
  // and the regular fill; ev[4] inside the regular fill, between the tile
  // kernel and the cut-edge fix-up (recorded when `split` is set)
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  bool timed = false, timing_now = false, split = false;
};

namespace mf {
void set_error(const std::string &msg);
int hip_fail(hipError_t e, const char *what);
#define MF_HIP(call)                                             \
  do {                                                           \
    hipError_t e_ = (call);                                      \
    if (e_ != hipSuccess) return ::mf::hip_fail(e_, #call);      \
  } while (0)


struct RuleArg;
RuleArg rule_arg(const Rule &r);

// Runs of 32 triangles the range scan bounds by spheres (4 doubles each).
int range_runs(int nt);
int launch_geometry(mf_mesh *m, const double *V, const Rule &r, hipStream_t s);
int launch_r_range(mf_mesh *m, const double *V, const Rule &r, double *rmin, double *rmax,
                   hipStream_t s);
// The same scan with its scratch in a static device array (no workspace).
int launch_r_range_static(mf_mesh *m, const double *V, const Rule &r, double *rmin,
                          double *rmax, hipStream_t s);
int max_static_range_triangles();
// Touching-pair blocks into out (m->d_sing when out is null).
int launch_singular(mf_mesh *m, const double *V, const Rule &r, double k, int part,
                    hipStream_t s, float *out = nullptr);
int launch_fill(mf_mesh *m, const Rule &r, double k, int mode, const mf_tables *tab, void *Z,
                int z_dtype, int64_t ldz, hipStream_t s);
// Kernels a table-mode single fill can run (the tuner's candidates).
enum { kFillTB1024 = 0, kFillTB512 = 1, kFillEB1024 = 2, kFillChoices = 3 };
const char *fill_choice_name(int c);
// Tuning cache: per process, and in the file named by MOMFILL_TUNE_CACHE
// when it is set (read once, appended to).  Keys are text.
bool tune_cache_get(const std::string &key, int *value);
void tune_cache_put(const std::string &key, int value);
std::string fill_tune_key(const mf_mesh *m, int nq, int mode, int z_dtype, const mf_tables *tab);
// The cached choice for this fill, or the default (kFillTB1024).
int cached_fill_choice(const mf_mesh *m, int nq, int mode, int z_dtype, const mf_tables *tab);
// MFIE: touching-pair blocks (FP64, one-way, with the identity term on the
// self pairs) into m->d_sing; then the fill with mode | kModeMfie.
int launch_singular_mfie(mf_mesh *m, const double *V, const Rule &r, double k, hipStream_t s);
// Plane-wave excitation (E0: 3 complex as re/im pairs) and far field.
int launch_rhs(mf_mesh *m, const double *V, const Rule &r, double k, const double *khat,
               const double *E0, void *out, int z_dtype, hipStream_t s, bool mfie = false);
int launch_far_field(mf_mesh *m, const double *V, const Rule &r, double k, const void *I,
                     int z_dtype, int n_dirs, const double *dirs, double e0n2, double *F,
                     double *sigma, hipStream_t s);
// Near-field fill: only the listed tiles, scattered into CSR values.
int launch_fill_near(mf_mesh *m, const Rule &r, double k, int mode, const mf_tables *tab,
                     const int32_t *tiles, int ntiles, const int32_t *sp_off, const int4 *sp_ent,
                     void *values, int z_dtype, hipStream_t s);
// Several items (meshes x wavenumbers) in one persistent fill launch.
struct FillLaunch;
// items_dev: device memory of fill_items_bytes(n) for the item list of a
// batched launch (n > 1), owned by the caller; may be null for one item.
size_t fill_items_bytes(int n);
// side: per-item side buffers (2 n_cut (ne + n_cut) floats each) that let a
// batch of EFIE items run on the triangle-block plan; may be null.
int fill_launch_create(int n, mf_mesh *const *m, const double *k, const mf_tables *const *tab,
                       const Rule &r, int mode, void *const *Z, int z_dtype, const int64_t *ldz,
                       const float *const *sing, void *items_dev, FillLaunch **out,
                       float *const *side = nullptr);
int fill_launch_run(FillLaunch *L, hipStream_t s);
// Candidates of the batch tuner: edge-block tiles at 512, 768, 1024 threads,
// then triangle-block tiles at 1024 and 512 threads.
constexpr int kBatchChoices = 5;
// Times the tile-shape variants of a batched launch (running it), keeps the
// fastest; ms (may be NULL) receives the kBatchChoices timings (zeros for
// candidates not run), *threads and *shape (0 edge blocks, 1 triangle
// blocks) the choice.
int fill_launch_autotune(FillLaunch *L, hipStream_t s, float *ms, int *threads, int *shape);
// Pins candidate c (index into the tuner's list) for later runs.
int fill_launch_set_choice(FillLaunch *L, int c);
void fill_launch_destroy(FillLaunch *L);
int build_tables_device(mf_tables *t, double tol, hipStream_t s, bool green = true);
// Upper bound of the device workspace a table build needs (both tables, or
// the Exp table alone).
size_t tables_workspace_bytes(double k, double rmin, double rmax, double tol, bool green);
// Frees every device array of both tables (safe on partly built ones).
void release_tables(mf_tables *t);
// Angular-transformation fill (FP64 inner integrals on every pair).
int launch_range_angular(mf_mesh *m, const double *V, const Rule &r, double *rmax,
                         hipStream_t s);
int launch_fill_angular(mf_mesh *m, const double *V, const Rule &r, double k, int n_edge,
                        int mode, const mf_tables *tab, void *Z, int z_dtype, int64_t ldz,
                        hipStream_t s);
int launch_table_eval(const mf_tables *t, int which, int64_t n, const double *r, double *out,
                      hipStream_t s);
int launch_backward(mf_mesh *m, const double *V, const Rule &r, double k, int mode,
                    const mf_tables *tab, const void *W, int z_dtype, int64_t ldz, double *dV,
                    double *dk, hipStream_t s);
}  // namespace mf
