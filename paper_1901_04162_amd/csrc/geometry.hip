// Geometry preparation, exact distance range and touching-pair blocks (FP64).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "internal.hpp"
#include "singular.hpp"

namespace mf {

RuleArg rule_arg(const Rule &r) {
  RuleArg a{};
  a.nq = r.nq;
  for (int i = 0; i < r.nq; ++i) {
    for (int c = 0; c < 3; ++c) a.b[i][c] = r.bary[i][c];
    a.w[i] = r.w[i];
  }
  return a;
}

// Quadrature point i of triangle (x0,x1,x2): b0 x0 + b1 x1 + b2 x2, evaluated
// left to right without contraction so that every distance derived from it
// is reproducible bit for bit.
__device__ inline void quad_point(const RuleArg &R, int i, const double *x0, const double *x1,
                                  const double *x2, double *P) {
#pragma clang fp contract(off)
  for (int c = 0; c < 3; ++c) P[c] = R.b[i][0] * x0[c] + R.b[i][1] * x1[c] + R.b[i][2] * x2[c];
}

__device__ inline double exact_dist(const double *a, const double *b) {
#pragma clang fp contract(off)
  const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
  return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
}

// ---- K0: per-triangle record for the regular-pair kernel ------------------

__global__ void k_geometry(const double *__restrict__ V, const int32_t *__restrict__ tri,
                           const int32_t *__restrict__ tedge, const int8_t *__restrict__ tsign,
                           int nt, RuleArg R, float *__restrict__ rec, double *__restrict__ qp64,
                           double *__restrict__ brad, float *__restrict__ elen,
                           int *__restrict__ status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  double x[3][3];
  int vid[3];
  for (int a = 0; a < 3; ++a) {
    vid[a] = tri[3 * t + a];
    for (int c = 0; c < 3; ++c) x[a][c] = V[3 * (size_t)vid[a] + c];
  }
  double c[3];
  for (int d = 0; d < 3; ++d) c[d] = (x[0][d] + x[1][d] + x[2][d]) / 3.0;
  const double e1[3] = {x[1][0] - x[0][0], x[1][1] - x[0][1], x[1][2] - x[0][2]};
  const double e2[3] = {x[2][0] - x[0][0], x[2][1] - x[0][1], x[2][2] - x[0][2]};
  const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                       e1[0] * e2[1] - e1[1] * e2[0]};
  const double area2 = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  if (!(area2 > 0.0)) atomicOr(&status[1], 1);
  float *o = rec + (size_t)t * kRecFloats;
  double rb = 0.0;
  for (int i = 0; i < kMaxQ; ++i) {
    float rr[3] = {0.0f, 0.0f, 0.0f};  // the FP32 offsets as stored
    double P[3] = {0.0, 0.0, 0.0};
    if (i < R.nq) quad_point(R, i, x[0], x[1], x[2], P);
    for (int d = 0; d < 3; ++d) {
      const double rho = i < R.nq ? P[d] - c[d] : 0.0;
      o[kRecRho + 3 * i + d] = (float)rho;
      o[kRecWRho + 3 * i + d] = (float)(i < R.nq ? R.w[i] * rho : 0.0);
      rr[d] = (float)rho;
      if (qp64 && i < R.nq) qp64[((size_t)t * kMaxQ + i) * 3 + d] = P[d];
    }
    // |rho_i|^2 from the stored FP32 offsets, with the fill's own FP32 formula
    o[kRecRho2 + i] = fmaf(rr[0], rr[0], fmaf(rr[1], rr[1], rr[2] * rr[2]));
    if (i < R.nq) {
      const double dd[3] = {P[0] - c[0], P[1] - c[1], P[2] - c[2]};
      rb = fmax(rb, sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]));
    }
  }
  if (brad) {
    brad[4 * t] = rb;
    for (int d = 0; d < 3; ++d) brad[4 * t + 1 + d] = area2 > 0.0 ? n[d] / area2 : 0.0;
  }
  for (int a = 0; a < 3; ++a) {
    for (int d = 0; d < 3; ++d) o[kRecAlpha + 3 * a + d] = (float)(c[d] - x[a][d]);
    const double *u = x[(a + 1) % 3], *v = x[(a + 2) % 3];
    const double l = sqrt((u[0] - v[0]) * (u[0] - v[0]) + (u[1] - v[1]) * (u[1] - v[1]) +
                          (u[2] - v[2]) * (u[2] - v[2]));
    o[kRecSigma + a] = tedge[3 * t + a] >= 0 ? (float)(tsign[3 * t + a] * l) : 0.0f;
    if (elen && tedge[3 * t + a] >= 0 && tsign[3 * t + a] > 0) elen[tedge[3 * t + a]] = (float)l;
  }
  double *cd = reinterpret_cast<double *>(o + kRecCent);
  cd[0] = c[0];
  cd[1] = c[1];
  cd[2] = c[2];
  int *vi = reinterpret_cast<int *>(o + kRecVid);
  vi[0] = vid[0];
  vi[1] = vid[1];
  vi[2] = vid[2];
  float rf = (float)rb;
  if ((double)rf < rb) rf = nextafterf(rf, INFINITY);
  o[kRecRho2 + kMaxQ] = 0.0f;
  o[kRecRad] = rf;
}

int launch_geometry(mf_mesh *m, const double *V, const Rule &r, hipStream_t s) {
  RuleArg R = rule_arg(r);
  hipLaunchKernelGGL(k_geometry, dim3((m->nt + 127) / 128), dim3(128), 0, s, V, m->d_tri,
                     m->d_tedge, m->d_tsign, m->nt, R, m->d_rec, m->d_qp64, m->d_brad, m->d_elen,
                     m->d_status);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

// ---- K1: exact distance range over regular pairs --------------------------
// Every unordered vertex-disjoint pair (p,q) is bounded from its centroid
// offset D (d = |D|), the radii rb of the quadrature points about the
// centroids and the reach h of those points along D (points lie in the
// triangle's plane, so h <= rb sin(angle(D, normal))): with delta the
// offset between two points, |delta| <= rb_p + rb_q = rr and
// |D.delta|/d <= h_p + h_q = hh, so every squared point distance lies in
// [d^2 - 2 d hh, d^2 + 2 d hh + rr^2].  The exact FP64 point-pair distances
// are evaluated only for pairs whose bounds can still lower the running
// minimum or raise the running maximum; the running values start from
// witnesses (exact distances of a sample of pairs), so the result is the
// exact extreme whatever the order of evaluation.  Squared distances are
// compared and the square root taken once: sqrt is correctly rounded and
// monotone, so this gives the same extreme as comparing distances.

constexpr int kRangeBlock = 256;
constexpr int kRangeChunk = 256;  // equal to kRangeBlock (the run tests assume it)
constexpr int kRangeScreen = 32;  // source triangles screened per round

struct RangeTri {
  double c[3];
  double rb;
  double n[3];
  int v[3];
};

__device__ inline void load_range_tri(const double *brad, const float *rec, int t, RangeTri &o) {
  const double *cd = reinterpret_cast<const double *>(rec + (size_t)t * kRecFloats + kRecCent);
  const int *vi = reinterpret_cast<const int *>(rec + (size_t)t * kRecFloats + kRecVid);
  for (int d = 0; d < 3; ++d) {
    o.c[d] = cd[d];
    o.v[d] = vi[d];
    o.n[d] = brad[4 * t + 1 + d];
  }
  o.rb = brad[4 * t];
}

__device__ inline double sq_dist(const double *a, const double *b) {
#pragma clang fp contract(off)
  const double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
  return d0 * d0 + d1 * d1 + d2 * d2;
}

__device__ inline bool share_vertex(const int *a, const int *b) {
  bool s = false;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) s |= a[i] == b[j];
  return s;
}

__device__ inline double dist3(const double *a, const double *b) { return exact_dist(a, b); }

__device__ inline unsigned long long wave_min_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long w = __shfl_xor(v, o);
    v = w < v ? w : v;
  }
  return v;
}
__device__ inline unsigned long long wave_max_u64(unsigned long long v) {
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long w = __shfl_xor(v, o);
    v = w > v ? w : v;
  }
  return v;
}

// lo, hi: running extremes of the squared distance.  Both triangles' points
// are loaded once into registers (nq is uniform; slots past it are neither
// loaded nor used).
__device__ inline void pair_extremes(const double *qp64, int nq, int p, int q, double &lo,
                                     double &hi) {
  double P[kMaxQ][3], Qp[kMaxQ][3];
  const double *pp = qp64 + (size_t)p * kMaxQ * 3, *qq = qp64 + (size_t)q * kMaxQ * 3;
#pragma unroll
  for (int a = 0; a < kMaxQ; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      P[a][c] = a < nq ? pp[3 * a + c] : 0.0;
      Qp[a][c] = a < nq ? qq[3 * a + c] : 0.0;
    }
#pragma unroll
  for (int a = 0; a < kMaxQ; ++a)
#pragma unroll
    for (int b = 0; b < kMaxQ; ++b)
      if (a < nq && b < nq) {
        const double R2 = sq_dist(P[a], Qp[b]);
        lo = fmin(lo, R2);
        hi = fmax(hi, R2);
      }
}

// Farthest centroid from the centroid of triangle `from` (or, when from < 0,
// of the triangle whose index sits in the low half of *from_slot): *out keeps
// the maximum of (float bits of the squared distance) << 32 | index.  Two
// such sweeps give an approximate diameter pair of the mesh, the witnesses
// for the largest distance.
__global__ void k_range_far(const float *__restrict__ rec, int nt, int from,
                            const unsigned long long *__restrict__ from_slot,
                            unsigned long long *__restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int f = from >= 0 ? from : (int)(unsigned)(*from_slot & 0xffffffffull);
  const double *fc = reinterpret_cast<const double *>(rec + (size_t)f * kRecFloats + kRecCent);
  unsigned long long v = 0ull;
  if (t < nt) {
    const double *tc = reinterpret_cast<const double *>(rec + (size_t)t * kRecFloats + kRecCent);
    const float d2 = (float)sq_dist(tc, fc);
    v = ((unsigned long long)__float_as_uint(d2) << 32) | (unsigned)t;
  }
  v = wave_max_u64(v);
  if ((threadIdx.x & 63) == 0) atomicMax(out, v);
}

// Witnesses: each triangle against a few index neighbours (close in space for
// meshes numbered with locality), a few pseudo-random partners and the two
// ends of the approximate diameter (far[0], far[1]).  One thread per
// (triangle, witness): blockIdx.y is the witness, so the grid holds
// kRangeWitnesses times as many threads as triangles and fills the chip; the
// extremes are reduced over the workgroup before its two atomics.
constexpr int kRangeWitnesses = 26;
constexpr int kSeedThreads = 256;

__global__ __launch_bounds__(kSeedThreads) void k_range_seed(
    const double *__restrict__ qp64, const float *__restrict__ rec, int nt, int nq,
    unsigned long long *__restrict__ out, const unsigned long long *__restrict__ far) {
  const int p = blockIdx.x * kSeedThreads + threadIdx.x;
  const int j = blockIdx.y;
  double lo = INFINITY, hi = 0.0;
  if (p < nt) {
    const int *pv = reinterpret_cast<const int *>(rec + (size_t)p * kRecFloats + kRecVid);
    const int q = j < 16   ? (p + 2 + j) % nt
                  : j < 24 ? (int)(((long long)p * 7919 + (long long)j * 104729) % nt)
                  : (int)(unsigned)(far[j - 24] & 0xffffffffull);
    const int *qv = reinterpret_cast<const int *>(rec + (size_t)q * kRecFloats + kRecVid);
    if (q != p && !share_vertex(pv, qv)) pair_extremes(qp64, nq, p, q, lo, hi);
  }
  unsigned long long l = lo < INFINITY ? (unsigned long long)__double_as_longlong(lo) : ~0ull;
  unsigned long long h = (unsigned long long)__double_as_longlong(hi);
  l = wave_min_u64(l);
  h = wave_max_u64(h);
  __shared__ unsigned long long red[2][kSeedThreads / 64];
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = l;
    red[1][threadIdx.x >> 6] = h;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kSeedThreads / 64; ++w) {
      l = red[0][w] < l ? red[0][w] : l;
      h = red[1][w] > h ? red[1][w] : h;
    }
    if (l != ~0ull) atomicMin(&out[0], l);
    atomicMax(&out[1], h);
  }
}

// Bounding sphere of every run of kRun triangles (centre, radius covering all
// their quadrature points), for skipping whole block pairs and, per test
// triangle, whole rounds of sources.
template <int kRun>
__global__ __launch_bounds__(kRun) void k_range_spheres(const double *__restrict__ brad,
                                                        const float *__restrict__ rec, int nt,
                                                        double *__restrict__ sph) {
  __shared__ double red[kRun][3];
  __shared__ double cen[3];
  const int t = blockIdx.x * kRun + threadIdx.x;
  const int n = min(kRun, nt - (int)blockIdx.x * kRun);
  RangeTri T{};
  if (t < nt) load_range_tri(brad, rec, t, T);
  for (int d = 0; d < 3; ++d) red[threadIdx.x][d] = t < nt ? T.c[d] : 0.0;
  __syncthreads();
  for (int h = kRun / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int d = 0; d < 3; ++d) red[threadIdx.x][d] += red[threadIdx.x + h][d];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int d = 0; d < 3; ++d) cen[d] = red[0][d] / n;
  __syncthreads();
  double r = 0.0;
  if (t < nt) r = sqrt(sq_dist(T.c, cen)) + T.rb;
  __syncthreads();
  red[threadIdx.x][0] = r;
  __syncthreads();
  for (int h = kRun / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x][0] = fmax(red[threadIdx.x][0], red[threadIdx.x + h][0]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double *o = sph + 4 * blockIdx.x;
    o[0] = cen[0];
    o[1] = cen[1];
    o[2] = cen[2];
    o[3] = red[0][0] * (1.0 + 1e-12) + 1e-300;
  }
}

__global__ __launch_bounds__(kRangeBlock) void k_range(const double *__restrict__ qp64,
                                                       const double *__restrict__ brad,
                                                       const float *__restrict__ rec, int nt,
                                                       int nq, const double *__restrict__ sph_round,
                                                       unsigned long long *out) {
  const int p0 = blockIdx.x * kRangeBlock, q0 = blockIdx.y * kRangeChunk;
  if (q0 + kRangeChunk <= p0) return;  // unordered pairs: q > p only
  // Skip the block pair when no point pair in it can lower the running
  // minimum or raise the running maximum: 64 threads test the 8 x 8 pairs of
  // its 32-triangle runs' bounding spheres.
  // The running extremes are read once per workgroup (a relaxed agent-scope
  // load, not a read-modify-write on the two contended words) and shared
  // through LDS; an older value only keeps more pairs, never fewer.
  __shared__ int keep;
  __shared__ unsigned long long extb[2];
  __shared__ double ext[2];
  if (threadIdx.x == 0) {
    keep = 0;
    extb[0] = __hip_atomic_load(&out[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    extb[1] = __hip_atomic_load(&out[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // no minimum yet (~0): +inf, so that every pair is screened in
    ext[0] = extb[0] == ~0ull ? INFINITY : __longlong_as_double((long long)extb[0]);
    ext[1] = __longlong_as_double((long long)extb[1]);
  }
  __syncthreads();
  constexpr int kRuns = kRangeBlock / kRangeScreen;
  if (threadIdx.x < kRuns * kRuns) {
    const int ra = p0 / kRangeScreen + (int)threadIdx.x / kRuns;
    const int rb = q0 / kRangeScreen + (int)threadIdx.x % kRuns;
    const int nr = (nt + kRangeScreen - 1) / kRangeScreen;
    if (ra < nr && rb < nr && rb >= ra) {
      const double *a = sph_round + 4 * ra, *b = sph_round + 4 * rb;
      const double dc = sqrt(sq_dist(a, b)), rr = a[3] + b[3];
      const double dmin = fmax(0.0, dc - rr), dmax = dc + rr;
      if (!(dmin * dmin * (1.0 - 1e-9) > ext[0] && dmax * dmax * (1.0 + 1e-9) < ext[1]))
        atomicOr(&keep, 1);
    }
  }
  __syncthreads();
  if (!keep) return;
  __shared__ RangeTri sq[kRangeChunk];
  // pairs that pass the screen, {test lane << 16 | source index}, evaluated
  // by the whole block so that no wave idles behind a few passing lanes
  __shared__ int list[kRangeBlock * kRangeScreen];
  __shared__ int nlist;
  const int p = p0 + threadIdx.x;
  const int nqc = min(kRangeChunk, nt - q0);
  for (int i = threadIdx.x; i < nqc; i += kRangeBlock) load_range_tri(brad, rec, q0 + i, sq[i]);
  double lo = ext[0], hi = ext[1];
  RangeTri P{};
  if (p < nt) load_range_tri(brad, rec, p, P);
  // The pair bounds are screened in FP32 and made conservative: the centre
  // offset is formed in FP64 before rounding, the sine of each normal angle
  // is bounded from above (+1e-5 under the root), the bounds are widened by
  // 1e-5 of their size and the running extremes by 1e-6, all far above the
  // FP32 rounding, so a pair that could move an extreme is never screened
  // out.  The pairs that pass are evaluated exactly in FP64.
  const float pn[3] = {(float)P.n[0], (float)P.n[1], (float)P.n[2]};
  const float prb = (float)P.rb;
  for (int jc = 0; jc < nqc; jc += kRangeScreen) {
    if (threadIdx.x == 0) nlist = 0;
    __syncthreads();
    // this round's sources lie in one bounding sphere: skip them when no
    // point of them can move an extreme against this test triangle
    bool near_or_far = p < nt;
    if (near_or_far) {
      const double *b = sph_round + 4 * ((q0 + jc) / kRangeScreen);
      const double dc = sqrt(sq_dist(P.c, b)), rr = P.rb + b[3];
      const double dmin = fmax(0.0, dc - rr), dmax = dc + rr;
      near_or_far = !(dmin * dmin * (1.0 - 1e-9) > lo && dmax * dmax * (1.0 + 1e-9) < hi);
    }
    if (near_or_far) {
      const float lo_f = (float)lo * 1.000001f, hi_f = (float)hi * 0.999999f;
      const int j1 = min(jc + kRangeScreen, nqc);
      for (int j = max(jc, p + 1 - q0); j < j1; ++j) {
        const RangeTri &Q = sq[j];
        if (share_vertex(P.v, Q.v)) continue;
        const float D[3] = {(float)(Q.c[0] - P.c[0]), (float)(Q.c[1] - P.c[1]),
                            (float)(Q.c[2] - P.c[2])};
        const float d2 = fmaf(D[0], D[0], fmaf(D[1], D[1], D[2] * D[2]));
        const float qrb = (float)Q.rb;
        const float d = sqrtf(d2), rr = prb + qrb;
        // Bounds from the two radii alone: with sp, sqq <= sqrt(1 + 1e-5) below,
        // (d + rr)^2 * 1.00002 lies above hi_b and 0.99998 d2 - 2.0001 d rr
        // below lo_b, with margins far above their FP32 rounding; a pair
        // outside both cannot move an extreme and skips the normal terms.
        if ((d + rr) * (d + rr) * 1.00002f < hi_f && fmaf(d2, 0.99998f, -2.0001f * d * rr) > lo_f)
          continue;
        const float id2 = 1.0f / fmaxf(d2, 1e-30f);
        const float dp = D[0] * pn[0] + D[1] * pn[1] + D[2] * pn[2];
        const float dq = D[0] * (float)Q.n[0] + D[1] * (float)Q.n[1] + D[2] * (float)Q.n[2];
        const float sp = sqrtf(fmaxf(0.0f, 1.0f - dp * dp * id2) + 1e-5f);
        const float sqq = sqrtf(fmaxf(0.0f, 1.0f - dq * dq * id2) + 1e-5f);
        const float dh = 2.0f * d * (prb * sp + qrb * sqq);
        const float lo_b = (d2 - dh) - 1e-5f * (d2 + dh);
        const float hi_b = (d2 + dh + rr * rr) * 1.00001f;
        if (lo_b <= lo_f || hi_b >= hi_f) list[atomicAdd(&nlist, 1)] = (threadIdx.x << 16) | j;
      }
    }
    __syncthreads();
    const int n = nlist;
    for (int e = threadIdx.x; e < n; e += kRangeBlock)
      pair_extremes(qp64, nq, p0 + (list[e] >> 16), q0 + (list[e] & 0xffff), lo, hi);
    __syncthreads();
  }
  // Reduce over the workgroup; touch the two contended words only when the
  // workgroup improves on the extremes it read at its start (bit patterns of
  // non-negative doubles order as unsigned integers; ~0 is "none yet").
  unsigned long long l = lo < INFINITY ? (unsigned long long)__double_as_longlong(lo) : ~0ull;
  unsigned long long h = (unsigned long long)__double_as_longlong(hi);
  l = wave_min_u64(l);
  h = wave_max_u64(h);
  __shared__ unsigned long long red[2][kRangeBlock / 64];
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = l;
    red[1][threadIdx.x >> 6] = h;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kRangeBlock / 64; ++w) {
      l = red[0][w] < l ? red[0][w] : l;
      h = red[1][w] > h ? red[1][w] : h;
    }
    if (l < extb[0]) atomicMin(&out[0], l);
    if (h > extb[1]) atomicMax(&out[1], h);
  }
}

int range_runs(int nt) { return (nt + kRangeScreen - 1) / kRangeScreen; }

// The scan with its scratch at `words` (4 reduction words) and `sph` (the
// run spheres): the mesh's workspace, or the static array below.
static int range_scan(mf_mesh *m, const Rule &r, unsigned long long *words, double *sph,
                      double *rmin, double *rmax, hipStream_t s) {
  unsigned long long init[4] = {~0ull, 0ull, 0ull, 0ull};
  MF_HIP(hipMemcpyAsync(words, init, sizeof(init), hipMemcpyHostToDevice, s));
  const dim3 tgrid((m->nt + 255) / 256);
  hipLaunchKernelGGL(k_range_far, tgrid, dim3(256), 0, s, m->d_rec, m->nt, 0, words, words + 2);
  hipLaunchKernelGGL(k_range_far, tgrid, dim3(256), 0, s, m->d_rec, m->nt, -1, words + 2,
                     words + 3);
  hipLaunchKernelGGL(k_range_seed, dim3((m->nt + kSeedThreads - 1) / kSeedThreads, kRangeWitnesses),
                     dim3(kSeedThreads), 0, s, m->d_qp64, m->d_rec, m->nt, r.nq, words, words + 2);
  MF_HIP(hipGetLastError());
  const int nb = (m->nt + kRangeBlock - 1) / kRangeBlock;
  const int nr = range_runs(m->nt);
  hipLaunchKernelGGL(k_range_spheres<kRangeScreen>, dim3(nr), dim3(kRangeScreen), 0, s,
                     m->d_brad, m->d_rec, m->nt, sph);
  dim3 grid(nb, (m->nt + kRangeChunk - 1) / kRangeChunk);
  hipLaunchKernelGGL(k_range, grid, dim3(kRangeBlock), 0, s, m->d_qp64, m->d_brad, m->d_rec,
                     m->nt, r.nq, sph, words);
  MF_HIP(hipGetLastError());
  unsigned long long res[2];
  int st[4];
  MF_HIP(hipMemcpyAsync(res, words, sizeof(res), hipMemcpyDeviceToHost, s));
  MF_HIP(hipMemcpyAsync(st, m->d_status, sizeof(st), hipMemcpyDeviceToHost, s));
  MF_HIP(hipStreamSynchronize(s));
  if (st[1]) {
    MF_HIP(hipMemset(m->d_status, 0, sizeof(int) * 4));
    set_error("mf_r_range: zero-area triangle");
    return MF_EMESH;
  }
  if (res[0] == ~0ull) {
    set_error("mf_r_range: the mesh has no vertex-disjoint triangle pair");
    return MF_EINVAL;
  }
  double lo2, hi2;
  std::memcpy(&lo2, &res[0], 8);
  std::memcpy(&hi2, &res[1], 8);
  *rmin = std::sqrt(lo2);
  *rmax = std::sqrt(hi2);
  return MF_OK;
}

int launch_r_range(mf_mesh *m, const double *V, const Rule &r, double *rmin, double *rmax,
                   hipStream_t s) {
  (void)V;
  return range_scan(m, r, m->d_scratch, m->d_sph, rmin, rmax, s);
}

// ---- the range scan without a scratch workspace ---------------------------
// For callers that cannot allocate: the scan's scratch (4 reduction words,
// then 4 doubles per run of 32 triangles) lives in this file-scope array,
// one copy per GPU for the life of the process.  Host code reaches it only
// through the address hipGetSymbolAddress gives for the current device.
constexpr size_t kStaticScratchBytes = (size_t)4 << 20;
constexpr size_t kStaticSphOffset = 256;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

static int static_scratch(void **out) {
  int dev = 0;
  MF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("mf_r_range_static: device index beyond the library's table");
    return MF_EINVAL;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    MF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MF_OK;
}

int max_static_range_triangles() {
  return (int)((kStaticScratchBytes - kStaticSphOffset) / (4 * sizeof(double))) * kRangeScreen;
}

int launch_r_range_static(mf_mesh *m, const double *V, const Rule &r, double *rmin,
                          double *rmax, hipStream_t s) {
  (void)V;
  if (m->nt > max_static_range_triangles()) {
    set_error("mf_r_range_static: more triangles than the static scratch holds (" +
              std::to_string(max_static_range_triangles()) + ")");
    return MF_EINVAL;
  }
  void *p = nullptr;
  int rc = static_scratch(&p);
  if (rc) return rc;
  auto *words = reinterpret_cast<unsigned long long *>(p);
  auto *sph = reinterpret_cast<double *>(reinterpret_cast<char *>(p) + kStaticSphOffset);
  return range_scan(m, r, words, sph, rmin, rmax, s);
}

// ---- K5: touching pairs (FP64 singularity cancellation) -------------------

// Eight lanes per touching pair: lane i takes the terms of the outer
// quadrature point i (lanes past the rule's points add nothing), and the
// lanes' partial blocks are summed with cross-lane shuffles.  The groups of
// eight are aligned in the wave and share one pair, so a group is either
// wholly past the end or wholly live, and every lane reaches the shuffles.
// Workgroups of 256 with two waves per SIMD give it 256 VGPRs: the default
// bound of 128 spills most of the FP64 state (0.72 against 0.28 ms on the
// 30,720-unknown sphere).
constexpr int kSingLanes = 8;
constexpr int kSingThreads = 256;
static_assert(kMaxQ <= kSingLanes, "one lane per outer quadrature point");

__global__ __launch_bounds__(kSingThreads, 2) void k_singular(const double *__restrict__ V, const int32_t *__restrict__ tri,
                           const int32_t *__restrict__ tp, const int32_t *__restrict__ tq,
                           int64_t npair, RuleArg R, double k, int part, double *__restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t s = g / kSingLanes;
  const int i = (int)(g % kSingLanes);
  const bool live = s < npair;
  double accr[9], acci[9];
  for (int t = 0; t < 9; ++t) accr[t] = acci[t] = 0.0;
  double Aq = 1.0;
  if (live) {
    const int p = tp[s], q = tq[s];
    double xp[3][3], xq[3][3];
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) {
        xp[a][c] = V[3 * (size_t)tri[3 * p + a] + c];
        xq[a][c] = V[3 * (size_t)tri[3 * q + a] + c];
      }
    Aq = oneway_terms(
        xp, xq, R, k, part,
        [&](int a, int b, double re, double im) {
          accr[3 * a + b] += re;
          acci[3 * a + b] += im;
        },
        i, i + 1);
  }
  for (int t = 0; t < 9; ++t)
    for (int d = 1; d < kSingLanes; d <<= 1) {
      accr[t] += __shfl_xor(accr[t], d, kSingLanes);
      acci[t] += __shfl_xor(acci[t], d, kSingLanes);
    }
  if (live && i == 0) {
    double *o = out + (size_t)s * 18;
    for (int t = 0; t < 9; ++t) {
      o[2 * t] = accr[t] / Aq;
      o[2 * t + 1] = acci[t] / Aq;
    }
  }
}

// X_sym(p,q)[a][b] = (X(p,q)[a][b] + X(q,p)[b][a]) / 2, stored as FP32.
__global__ void k_symmetrise(const double *__restrict__ one, const int32_t *__restrict__ rev,
                             int64_t npair, float *__restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= npair) return;
  const double *x = one + (size_t)s * 18, *y = one + (size_t)rev[s] * 18;
  float *o = out + (size_t)s * 18;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      o[2 * (3 * a + b)] = (float)(0.5 * (x[2 * (3 * a + b)] + y[2 * (3 * b + a)]));
      o[2 * (3 * a + b) + 1] = (float)(0.5 * (x[2 * (3 * a + b) + 1] + y[2 * (3 * b + a) + 1]));
    }
}

int launch_singular(mf_mesh *m, const double *V, const Rule &r, double k, int part,
                    hipStream_t s, float *out) {
  const int64_t np = (int64_t)m->touch_q.size();
  if (np == 0) return MF_OK;
  RuleArg R = rule_arg(r);
  hipLaunchKernelGGL(k_singular, dim3((unsigned)((np * kSingLanes + kSingThreads - 1) / kSingThreads)),
                     dim3(kSingThreads), 0, s, V, m->d_tri, m->d_touch_p, m->d_touch_q, np, R, k,
                     part, m->d_sing1);
  MF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_symmetrise, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s,
                     m->d_sing1, m->d_touch_rev, np, out ? out : m->d_sing);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

}  // namespace mf
