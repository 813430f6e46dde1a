// Regular-pair impedance fill (FP32), table and direct modes.
//
// Z is symmetric (Galerkin reciprocity of the EFIE with the same rule on
// test and source triangles, and symmetrised touching pairs), so only the
// block pairs I <= J of the edge blocks (runs of consecutive edges, at most
// kMaxBlockEdges long) are computed; an off-diagonal tile is written to
// Z[I,J] and, transposed, to Z[J,I].
//
// One workgroup owns a tile at a time (persistent grid) and accumulates it
// in LDS, without atomics (fill_tile).  A tile needs every triangle carrying
// one of its row edges (list I) against every triangle carrying one of its
// column edges (list J).  Lane l of a wave takes test triangle I[l] (its
// record read where used); the wave walks the source triangles of J, whose
// records are wave-uniform and so come through scalar loads into SGPRs.  Per triangle pair the Q x Q point pairs are reduced to four
// moments of g = exp(-jkR)/R,
//   S0 = sum w_i w_j g, Srho = sum w_i w_j g rho_i, Srho' = sum w_i w_j g rho'_j,
//   Srr = sum w_i w_j g rho_i.rho'_j,
// from which the nine local entries follow with alpha_a = c_p - v_a and
// beta_b = c_q - v_b:
//   X_ab = (Srr + alpha_a.Srho' + beta_b.Srho + alpha_a.beta_b S0)/4 - S0/k^2.
// Touching pairs take their FP64 blocks from the singular kernel.  The
// Green-function table's interval coefficients sit in LDS when they fit (read
// from global memory otherwise); its bucket records are read from global
// memory through the vector L1.
//
// Distances: D = c_p - c_q is formed in FP64 and split into FP32 hi + lo;
// each test point's offset hi + (lo + rho_i) is rounded once in FP32, then
// the source offsets are subtracted: R carries a few FP32 roundings at its
// own size and no cancellation error of the centroids.
//
// Direct mode keeps FP64 accuracy where the RWG sum cancels.  For distant
// edges the four triangle-pair terms of an entry are tens of times larger
// than their sum (the div-div terms of the two charge dipoles cancel), so
// FP32 rounding of the terms, and the FP32 phase error k dR ~ 1e-6 of each
// point pair at kR ~ 30, would reach the entry at the 1e-6 level.  The
// direct tile therefore splits every phase about the FP64 centroid distance
// d (exp(-jkR) = exp(-jkd) exp(-jku), u = R - d formed without
// cancellation), accumulates the moments as deviations from the reference
// exp(-jkd)/d of the pair, and keeps that reference (rounded to FP32) per
// triangle pair in LDS; the write-out adds the second difference of the
// references over the four triangle pairs of each entry in FP64, where the
// cancellation is exact.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <type_traits>
#include <vector>

#include "internal.hpp"
#include "lookup.hpp"
#include "uniform.hpp"

namespace mf {

constexpr int kBM = kMaxBlockEdges;
constexpr int kAccStride = 2 * kBM + 1;  // odd stride: rows fall in different banks
constexpr int kAccFloats = kBM * kAccStride;
// The EFIE kernels run 1024 threads (4 waves per SIMD, at most 128 VGPRs):
// the source records sit in SGPRs and the test triangle's data is read from
// its record where it is used.  Sixteen waves also split a block's source
// triangles (at most 64) evenly.
template <int MODE>
constexpr int fill_threads() {
  return 1024;
}
// The MFIE kernel holds both directions' moments and two accumulators: 512
// threads (2 waves per SIMD, 256 VGPRs per lane), one workgroup per CU.
template <int MODE, int OP>
constexpr int fill_threads_op() {
  return OP == MF_OP_MFIE ? 512 : fill_threads<MODE>();
}

// One fill item: a mesh, a wavenumber, its table and its output.  A launch
// walks the global tile list of one or more items (tiles tile_begin ..
// tile_end - 1 belong to this item).
struct FillItem {
  int tile_begin, tile_end;
  int tb_begin, tb_end;  // the item's range in the batch's triangle-block tile list
  int ne;
  double kd;  // wavenumber (FP64: the per-pair reference phase of direct mode)
  float k, ik2;
  float pref;  // k eta0 / (4 pi)
  int tn, tm;
  float tinv, tbias, tmax;  // bucket coordinate x = r*tinv + tbias, clamped to [0, tmax]
  float lo_ok, hi_ok;
  long long ldz;
  const float *rec;
  const int32_t *tiles, *blk_e0, *blk_off, *blk_tri, *blk_pos, *touch_off, *touch_q, *touch_rev;
  const int32_t *blk_rt;  // per block row: positions of its T+ and T- in the block's list
  const int32_t *blk_ord, *blk_rounds;  // round order of each block's triangles (MFIE)
  const float *elen;      // edge lengths
  // triangle-block plan (table mode, see fill_tile_tb)
  const int32_t *tb_t0, *tb_e0, *tb_nbe, *tb_be_off, *tb_be_cut, *tb_pos, *tb_order, *tb_rounds,
      *tb_tiles;
  float2 *side;           // cut-edge partial entries, rows of lside complex values
  long long lside;
  const int32_t *edges;   // ne x 6: v_lo, v_hi, T+, T-, a+, a-
  const int32_t *cut_idx; // ne: cut index of an edge, -1 inside a block
  const int32_t *cut_edge;  // n_cut: edge of each cut index
  int n_cut;
  const float *sing;
  const int4 *look;
  const float4 *coef;
  void *Z;
  int *status;
  // near-field fill: entries of tile t are sp_ent[sp_off[t] .. sp_off[t+1]),
  // each {r << 8 | c, position of (row, col), position of the mirror or -1}
  const int32_t *sp_off;
  const int4 *sp_ent;
};
typedef FillItem FillScalars;

// Quadrature weights, common to every item of a launch, and the rule in a
// triangle's own frame: point j is rho_j = s_j e1 + t_j e2 with e1 = v0 - c,
// e2 = v1 - c and (s_j, t_j) = (l0 - l2, l1 - l2) from its barycentric
// coordinates (sum l = 1, sum (v - c) = 0), the same for every triangle.
struct FillRule {
  float w[kMaxQ];
  float s2[kMaxQ], t2[kMaxQ];  // 2 s_j, 2 t_j
  float ws[kMaxQ], wt[kMaxQ];  // w_j s_j, w_j t_j
};

// Which of s_j, t_j vanish in the symmetric rules (the orbit order of the
// rule's definition): 0 both (the centroid), 1 t = 0, 2 s = 0, 3 s = t.
// Orbit points (x, y, y), (y, x, y), (y, y, x) give kinds 1, 2, 3.
__host__ __device__ constexpr int bary_kind(int Q, int j) {
  return Q == 7 ? (j == 0 ? 0 : 1 + (j - 1) % 3) : 1 + j % 3;
}

struct TabPtrs {
  const int4 *look;     // one-sample bucket records {i0, x(i0), x(i0 + 1), -}
  const float4 *c01;    // per interval (c0, c1) about its first sample
  const float4 *c23;    // per interval (c2, c3)
};

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// In LDS the (c2, c3) array starts a fixed kLdsCoefHalf records after the
// (c0, c1) array, so that one address serves both reads of a lookup (the
// second through the instruction's offset field).
constexpr int kLdsCoefHalf = 1899;  // with the two accumulator halves: 163,824 B of LDS

// Direct mode: the per-triangle-pair references exp(-jkd)/d of a tile,
// indexed [source position][test position] with an odd stride of float2.
constexpr int kRefStride = kMaxBlockTris + 1;
constexpr int kRefFloat2 = kMaxBlockTris * kRefStride;


// The four moments of one triangle pair (S0, Srho, Srho', Srr), complex.
struct Moments {
  float s0r, s0i, srr, sri;
  float spr[3], spi[3];  // Srho
  float sqr[3], sqi[3];  // Srho'
};

// Adds w_i T0 and w_i T1 of test point i (rho_i = pri) into the moments.
__device__ __forceinline__ void add_point(Moments &M, float wi, const float *pri, float t0r,
                                          float t0i, const float *t1r, const float *t1i) {
  t0r *= wi;
  t0i *= wi;
  M.s0r += t0r;
  M.s0i += t0i;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float ar = t1r[c] * wi, ai = t1i[c] * wi;
    M.spr[c] = fmaf(pri[c], t0r, M.spr[c]);
    M.spi[c] = fmaf(pri[c], t0i, M.spi[c]);
    M.sqr[c] += ar;
    M.sqi[c] += ai;
    M.srr = fmaf(pri[c], ar, M.srr);
    M.sri = fmaf(pri[c], ai, M.sri);
  }
}

__device__ __forceinline__ void zero(Moments &M) {
  M.s0r = M.s0i = M.srr = M.sri = 0.0f;
#pragma unroll
  for (int c = 0; c < 3; ++c) M.spr[c] = M.spi[c] = M.sqr[c] = M.sqi[c] = 0.0f;
}

// MFIE (K operator).  The kernel is K = (1 + jkR) exp(-jkR)/R^3 =
// (1/R + jk) g/R, taken from the same Green table, and the integrand of the
// local entry (a, b) is (r' - v_b).(t_a,i x d) K with t_a,i = (r_i - v_a) x n
// and d = r - r'.  Writing r_i - v_a = alpha_a + rho_i, r' - v_b = beta_b +
// rho'_j, a_i = c_p - c_q + rho_i (so d = a_i - rho'_j), tau_a = alpha_a x n,
// sigma_i = rho_i x n, and per test point T0 = sum_j w_j K, T1 = sum_j w_j K
// rho'_j (the EFIE's inner sums with K in place of g), the entry needs four
// moments over the test points:
//   Md = sum w_i (a_i T0 - T1),       Mx = sum w_i a_i x T1,
//   Ms = sum w_i sigma_i x (a_i T0 - T1),  M0 = sum w_i sigma_i.(a_i x T1),
//   X_ab = (beta_b.(tau_a x Md + Ms) + tau_a.Mx + M0)/4.
// The operator is not symmetric, but K(R) is: the same kernel values give the
// reverse block (test triangle q, source p) too.  With n' the unit normal of
// q, tau'_b = beta_b x n' and the third inner sum T2 = sum_j w_j K |rho'_j|^2
// (rho'_j lies in q's plane, so the terms quadratic in rho'_j reduce to it),
//   Md' = -Md,   Mx' = -sum w_i (a_i T0 - T1) x rho_i,
//   Ms' = -sum w_i [ (T1 x n') x a_i - n' T2 ],
//   M0' = -sum w_i [ (T1 x n').(a_i x rho_i) - T2 (n'.rho_i) ],
//   X'_ba = (alpha_a.(tau'_b x Md' + Ms') + tau'_b.Mx' + M0')/4.
struct MomentsM {
  float dr[3], di[3], xr[3], xi[3], sr[3], si[3], m0r, m0i;  // p tested against q
  float qxr[3], qxi[3], qsr[3], qsi[3], q0r, q0i;             // q tested against p
};

__device__ __forceinline__ void zero(MomentsM &M) {
  M.m0r = M.m0i = M.q0r = M.q0i = 0.0f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    M.dr[c] = M.di[c] = M.xr[c] = M.xi[c] = M.sr[c] = M.si[c] = 0.0f;
    M.qxr[c] = M.qxi[c] = M.qsr[c] = M.qsi[c] = 0.0f;
  }
}

__device__ __forceinline__ void cross3(const float *u, const float *v, float *o) {
  o[0] = fmaf(u[1], v[2], -u[2] * v[1]);
  o[1] = fmaf(u[2], v[0], -u[0] * v[2]);
  o[2] = fmaf(u[0], v[1], -u[1] * v[0]);
}

__device__ __forceinline__ float dot3(const float *u, const float *v) {
  return fmaf(u[0], v[0], fmaf(u[1], v[1], u[2] * v[2]));
}

__device__ __forceinline__ void add_point(MomentsM &M, float wi, const float *pri, const float *a,
                                          const float *nrm, const float *nq, float t0r, float t0i,
                                          const float *t1r, const float *t1i, float t2r,
                                          float t2i) {
  float vr[3], vi[3], cr[3], ci[3], sg[3], u[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    vr[c] = wi * fmaf(a[c], t0r, -t1r[c]);
    vi[c] = wi * fmaf(a[c], t0i, -t1i[c]);
    M.dr[c] += vr[c];
    M.di[c] += vi[c];
  }
  float wt[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) wt[c] = wi * t1r[c];
  cross3(a, wt, cr);
#pragma unroll
  for (int c = 0; c < 3; ++c) wt[c] = wi * t1i[c];
  cross3(a, wt, ci);
  cross3(pri, nrm, sg);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    M.xr[c] += cr[c];
    M.xi[c] += ci[c];
  }
  M.m0r += dot3(sg, cr);
  M.m0i += dot3(sg, ci);
  cross3(sg, vr, u);
#pragma unroll
  for (int c = 0; c < 3; ++c) M.sr[c] += u[c];
  cross3(sg, vi, u);
#pragma unroll
  for (int c = 0; c < 3; ++c) M.si[c] += u[c];
  // reverse direction
  cross3(vr, pri, u);
#pragma unroll
  for (int c = 0; c < 3; ++c) M.qxr[c] -= u[c];
  cross3(vi, pri, u);
#pragma unroll
  for (int c = 0; c < 3; ++c) M.qxi[c] -= u[c];
  float axr[3], cw[3];
  cross3(a, pri, axr);
  const float nr = dot3(nq, pri), w2r = wi * t2r, w2i = wi * t2i;
#pragma unroll
  for (int c = 0; c < 3; ++c) wt[c] = wi * t1r[c];
  cross3(wt, nq, cw);
  cross3(cw, a, u);
#pragma unroll
  for (int c = 0; c < 3; ++c) M.qsr[c] -= fmaf(-nq[c], w2r, u[c]);
  M.q0r -= fmaf(-w2r, nr, dot3(cw, axr));
#pragma unroll
  for (int c = 0; c < 3; ++c) wt[c] = wi * t1i[c];
  cross3(wt, nq, cw);
  cross3(cw, a, u);
#pragma unroll
  for (int c = 0; c < 3; ++c) M.qsi[c] -= fmaf(-nq[c], w2i, u[c]);
  M.q0i -= fmaf(-w2i, nr, dot3(cw, axr));
}

// g -> K = (1/R + jk) g / R (MFIE kernel from the Green-function value).
__device__ __forceinline__ void green_to_k(float k, float ri, float &gr, float &gi) {
  const float ur = fmaf(gr, ri, -k * gi), ui = fmaf(gi, ri, k * gr);
  gr = ur * ri;
  gi = ui * ri;
}

template <int OP>
using MomentsOf = typename std::conditional<OP == MF_OP_MFIE, MomentsM, Moments>::type;

// MFIE table mode.  The test-point loop stays rolled and reads rho_i from
// the record; the lookups of one test point go in three steps over all
// source points at once (distances and bucket-record reads, then
// coefficient reads, then the cubic and the sums), so that the dependent
// reads overlap.  The interval search is the bucket lookup of Eq. (6) in the
// record form of lookup.hpp (one gather gives the interval and its first
// sample), and the cubic of Eq. (5) is evaluated in Horner form about that
// sample; K = (1/R + jk) g/R follows from the same value.  As in the EFIE's
// table mode (moments_bary) the distances and the inner sum T1 use the
// rule's own frame: R^2 = |a|^2 + 2 s_j a.beta_0 + 2 t_j a.beta_1 +
// |rho'_j|^2, and T1 = sum_j w_j K rho'_j = -(beta_0 T_s + beta_1 T_t) with
// T_s = sum w_j s_j K, T_t = sum w_j t_j K (the zero terms skipped); the
// weights w_j |rho'_j|^2 of the third inner sum T2 are formed once per pair.
template <int Q, bool kLDS>
__device__ __forceinline__ void moments_table_mfie(MomentsM &M, const TabPtrs &tab,
                                                   const FillScalars &S, const FillRule &W,
                                                   const float *pr, const float *nrm,
                                                   const float *nq, float hx, float hy, float hz,
                                                   float lx, float ly, float lz, cfloat *qr,
                                                   float &rlo, float &rhi) {
  zero(M);
  float n2[Q], wr2[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const float qx = qr[kRecRho + 3 * j], qy = qr[kRecRho + 3 * j + 1],
                qz = qr[kRecRho + 3 * j + 2];
    n2[j] = fmaf(qx, qx, fmaf(qy, qy, qz * qz));
    wr2[j] = W.w[j] * n2[j];
  }
  float b0[3], b1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    b0[c] = qr[kRecAlpha + c];
    b1[c] = qr[kRecAlpha + 3 + c];
  }
#pragma unroll 1
  for (int i = 0; i < Q; ++i) {
    float pri[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) pri[c] = pr[kRecRho + 3 * i + c];
    const float ax = hx + (pri[0] + lx), ay = hy + (pri[1] + ly), az = hz + (pri[2] + lz);
    const float A2 = fmaf(ax, ax, fmaf(ay, ay, az * az));
    const float B0 = fmaf(ax, b0[0], fmaf(ay, b0[1], az * b0[2]));
    const float B1 = fmaf(ax, b1[0], fmaf(ay, b1[1], az * b1[2]));
    const float B01 = B0 + B1;
    float r[Q];
    int4 w[Q];
    __builtin_amdgcn_s_setprio(1);  // gathers and coefficient reads ahead of arithmetic
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int kind = bary_kind(Q, j);
      const float r2 = kind == 0   ? A2
                       : kind == 1 ? fmaf(W.s2[j], B0, A2 + n2[j])
                       : kind == 2 ? fmaf(W.t2[j], B1, A2 + n2[j])
                                   : fmaf(W.s2[j], B01, A2 + n2[j]);
      r[j] = __builtin_amdgcn_sqrtf(r2);
      w[j] = look_record(tab.look, look_bucket(r[j], S.tinv, S.tbias, S.tmax));
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      rlo = fminf(rlo, r[j]);
      rhi = fmaxf(rhi, r[j]);
    }
    float u[Q];
    float4 A[Q], B[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int off = look_offset1(w[j], r[j], u[j]);
      A[j] = at_offset(tab.c01, off);
      // in LDS the (c2, c3) half sits a constant distance after (c0, c1): one
      // address, the distance in the read's offset field
      B[j] = kLDS ? at_offset(tab.c01, off + 16 * kLdsCoefHalf) : at_offset(tab.c23, off);
    }
    __builtin_amdgcn_s_setprio(0);
    float t0r = 0.f, t0i = 0.f, tsr = 0.f, tsi = 0.f, ttr = 0.f, tti = 0.f;
    float t2r = 0.f, t2i = 0.f;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int kind = bary_kind(Q, j);
      const float2 g = cubic(A[j], B[j], u[j]);
      float gr = g.x, gi = g.y;
      green_to_k(S.k, __builtin_amdgcn_rcpf(r[j]), gr, gi);
      t0r = fmaf(W.w[j], gr, t0r);
      t0i = fmaf(W.w[j], gi, t0i);
      if (kind == 1 || kind == 3) {
        tsr = fmaf(W.ws[j], gr, tsr);
        tsi = fmaf(W.ws[j], gi, tsi);
      }
      if (kind == 2 || kind == 3) {
        ttr = fmaf(W.wt[j], gr, ttr);
        tti = fmaf(W.wt[j], gi, tti);
      }
      if (kind != 0) {  // the centroid's |rho'_j|^2 is zero up to rounding
        t2r = fmaf(wr2[j], gr, t2r);
        t2i = fmaf(wr2[j], gi, t2i);
      }
    }
    float t1r[3], t1i[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      t1r[c] = -fmaf(b0[c], tsr, b1[c] * ttr);
      t1i[c] = -fmaf(b0[c], tsi, b1[c] * tti);
    }
    const float a[3] = {ax, ay, az};
    add_point(M, W.w[i], pri, a, nrm, nq, t0r, t0i, t1r, t1i, t2r, t2i);
  }
}

// Output written once and never read back by the fill: non-temporal stores
// stream it past the caches, which keep the reused triangle and bucket
// records instead.
template <typename T>
__device__ __forceinline__ void store_stream(T *dst, T v) {
  if constexpr (sizeof(T) == 8) {
    __builtin_nontemporal_store(__builtin_bit_cast(double, v), reinterpret_cast<double *>(dst));
  } else {
    __builtin_nontemporal_store(v.x, &dst->x);
    __builtin_nontemporal_store(v.y, &dst->y);
  }
}

// EFIE table mode in the rule's own frame.  With rho_i = -(s_i alpha_0 +
// t_i alpha_1) on the test triangle and rho'_j = -(s_j beta_0 + t_j beta_1)
// on the source triangle (alpha_a = c_p - v_a, beta_b = c_q - v_b), and the
// rule's three weight vectors u^0 = w, u^s = w s, u^t = w t, the four
// moments of a pair come from nine bilinear forms of g,
//   N_xy = sum_ij u^x_i u^y_j g_ij,        x, y in {0, s, t},
// through the dot products D_ab = alpha_a.beta_b:
//   S0 = N_00,   alpha_a.Srho' = -(D_a0 N_0s + D_a1 N_0t),
//   beta_b.Srho = -(D_0b N_s0 + D_1b N_t0),
//   Srr = D_00 N_ss + D_01 N_st + D_10 N_ts + D_11 N_tt.
// The inner sums over the source points skip the terms where s_j or t_j is
// zero (bary_kind).  The distances use the same frame: with a_i = D + rho_i,
// A = |a_i|^2 and B_b = a_i.beta_b,
//   R^2 = A + 2 s_j B_0 + 2 t_j B_1 + |rho'_j|^2,
// two operations per point pair instead of six.
struct Bary {
  float r[9], i[9];  // N_00, N_0s, N_0t, N_s0, N_ss, N_st, N_t0, N_ts, N_tt
};

template <int Q, bool kLDS>
__device__ __forceinline__ void moments_bary(Bary &N, const TabPtrs &tab, const FillScalars &S,
                                             const FillRule &W, const float *pr, float hx,
                                             float hy, float hz, float lx, float ly, float lz,
                                             cfloat *qr, bool &oor, bool range = true) {
#pragma unroll
  for (int x = 0; x < 9; ++x) N.r[x] = N.i[x] = 0.0f;
  // |rho'_j|^2 from the source record (scalar loads, formed by k_geometry)
  cfloat *nq = qr + kRecRho2;
  const float b0x = qr[kRecAlpha], b0y = qr[kRecAlpha + 1], b0z = qr[kRecAlpha + 2];
  const float b1x = qr[kRecAlpha + 3], b1y = qr[kRecAlpha + 4], b1z = qr[kRecAlpha + 5];
#pragma unroll 1
  for (int i = 0; i < Q; ++i) {
    const float ax = hx + (pr[kRecRho + 3 * i] + lx), ay = hy + (pr[kRecRho + 3 * i + 1] + ly),
                az = hz + (pr[kRecRho + 3 * i + 2] + lz);
    const float A = fmaf(ax, ax, fmaf(ay, ay, az * az));
    const float B0 = fmaf(ax, b0x, fmaf(ay, b0y, az * b0z));
    const float B1 = fmaf(ax, b1x, fmaf(ay, b1y, az * b1z));
    const float B01 = B0 + B1;
    float r[Q];
    int4 w[Q];
    // the distances, their gathers and the coefficient reads at raised wave
    // priority, so that a wave about to start its memory latency issues ahead
    // of waves doing arithmetic
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int kind = bary_kind(Q, j);
      // the centroid's rho'_j is zero up to the rounding of its FP64 mean
      const float r2 = kind == 0   ? A
                       : kind == 1 ? fmaf(W.s2[j], B0, A + nq[j])
                       : kind == 2 ? fmaf(W.t2[j], B1, A + nq[j])
                                   : fmaf(W.s2[j], B01, A + nq[j]);
      r[j] = __builtin_amdgcn_sqrtf(r2);
      w[j] = look_record(tab.look, look_bucket(r[j], S.tinv, S.tbias, S.tmax));
    }
    if (range) {
      // a distance outside the table's range sets the lane's flag; the
      // smallest and largest of the Q distances decide it without branches
      float rmin = r[0], rmax = r[0];
#pragma unroll
      for (int j = 1; j < Q; ++j) {
        rmin = fminf(rmin, r[j]);
        rmax = fmaxf(rmax, r[j]);
      }
      oor = oor | (rmin < S.lo_ok) | (rmax > S.hi_ok);
    }
    float u[Q];
    float4 Ac[Q], Bc[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int off = look_offset1(w[j], r[j], u[j]);
      Ac[j] = at_offset(tab.c01, off);
      Bc[j] = kLDS ? at_offset(tab.c01, off + 16 * kLdsCoefHalf) : at_offset(tab.c23, off);
    }
    __builtin_amdgcn_s_setprio(0);
    float t0r = 0.f, t0i = 0.f, tsr = 0.f, tsi = 0.f, ttr = 0.f, tti = 0.f;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int kind = bary_kind(Q, j);
      const float2 g = cubic(Ac[j], Bc[j], u[j]);
      t0r = fmaf(W.w[j], g.x, t0r);
      t0i = fmaf(W.w[j], g.y, t0i);
      if (kind == 1 || kind == 3) {
        tsr = fmaf(W.ws[j], g.x, tsr);
        tsi = fmaf(W.ws[j], g.y, tsi);
      }
      if (kind == 2 || kind == 3) {
        ttr = fmaf(W.wt[j], g.x, ttr);
        tti = fmaf(W.wt[j], g.y, tti);
      }
    }
    const float u3[3] = {W.w[i], W.ws[i], W.wt[i]};
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      N.r[3 * x] = fmaf(u3[x], t0r, N.r[3 * x]);
      N.i[3 * x] = fmaf(u3[x], t0i, N.i[3 * x]);
      N.r[3 * x + 1] = fmaf(u3[x], tsr, N.r[3 * x + 1]);
      N.i[3 * x + 1] = fmaf(u3[x], tsi, N.i[3 * x + 1]);
      N.r[3 * x + 2] = fmaf(u3[x], ttr, N.r[3 * x + 2]);
      N.i[3 * x + 2] = fmaf(u3[x], tti, N.i[3 * x + 2]);
    }
  }
}

// The nine local entries of a regular pair from its bilinear forms:
//   X_ab = (Srr + alpha_a.Srho' + beta_b.Srho + D_ab S0)/4 - S0/k^2;
// PART drops the vector part (MF_PART_PHI) or the scalar part (MF_PART_A).
template <int PART>
__device__ __forceinline__ void entries_bary(const Bary &N, const float (&al)[3][3],
                                             const float (&be)[3][3], float ik2,
                                             float (&Xr)[3][3], float (&Xi)[3][3]) {
  constexpr bool vec = !(PART & MF_PART_PHI), sca = !(PART & MF_PART_A);
  float D[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      D[a][b] = fmaf(al[a][0], be[b][0], fmaf(al[a][1], be[b][1], al[a][2] * be[b][2]));
  float c0r = 0.f, c0i = 0.f;
  if (vec) {
    c0r = 0.25f * fmaf(D[0][0], N.r[4], fmaf(D[0][1], N.r[5], fmaf(D[1][0], N.r[7],
                                                                      D[1][1] * N.r[8])));
    c0i = 0.25f * fmaf(D[0][0], N.i[4], fmaf(D[0][1], N.i[5], fmaf(D[1][0], N.i[7],
                                                                      D[1][1] * N.i[8])));
  }
  if (sca) {
    c0r = fmaf(-ik2, N.r[0], c0r);
    c0i = fmaf(-ik2, N.i[0], c0i);
  }
  const float q0r = 0.25f * N.r[0], q0i = 0.25f * N.i[0];
  float Ar[3], Ai[3], Br[3], Bi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Ar[a] = c0r;
    Ai[a] = c0i;
    Br[a] = Bi[a] = 0.0f;
    if (vec) {
      // alpha_a.Srho' / 4 and beta_a.Srho / 4
      Ar[a] -= 0.25f * fmaf(D[a][0], N.r[1], D[a][1] * N.r[2]);
      Ai[a] -= 0.25f * fmaf(D[a][0], N.i[1], D[a][1] * N.i[2]);
      Br[a] = -0.25f * fmaf(D[0][a], N.r[3], D[1][a] * N.r[6]);
      Bi[a] = -0.25f * fmaf(D[0][a], N.i[3], D[1][a] * N.i[6]);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      float vr = Ar[a] + Br[b], vi = Ai[a] + Bi[b];
      if (vec) {
        vr = fmaf(D[a][b], q0r, vr);
        vi = fmaf(D[a][b], q0i, vi);
      }
      Xr[a][b] = vr;
      Xi[a][b] = vi;
    }
}

// Direct mode: exp(-jkR)/R from rsqrt and sincos; the test-point loop stays
// rolled (the inlined sincos is long) and reads rho_i from the record.
template <int Q, int OP>
__device__ __forceinline__ void moments_direct(MomentsOf<OP> &M, const FillScalars &S,
                                               const FillRule &W, const float *pr,
                                               const float *nrm, const float *nq, float hx, float hy, float hz, float lx, float ly,
                                               float lz, cfloat *qr) {
  zero(M);
  // the third inner sum's weights w_j |rho'_j|^2, once per pair (MFIE)
  float wr2[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j)
    wr2[j] = OP == MF_OP_MFIE
                 ? fmaf(qr[kRecWRho + 3 * j], qr[kRecRho + 3 * j],
                        fmaf(qr[kRecWRho + 3 * j + 1], qr[kRecRho + 3 * j + 1],
                             qr[kRecWRho + 3 * j + 2] * qr[kRecRho + 3 * j + 2]))
                 : 0.0f;
#pragma unroll 1
  for (int i = 0; i < Q; ++i) {
    float pri[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) pri[c] = pr[kRecRho + 3 * i + c];
    const float ax = hx + (pri[0] + lx), ay = hy + (pri[1] + ly), az = hz + (pri[2] + lz);
    float t0r = 0.f, t0i = 0.f, t1r[3] = {0.f, 0.f, 0.f}, t1i[3] = {0.f, 0.f, 0.f};
    float t2r = 0.f, t2i = 0.f;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const float dx = ax - qr[kRecRho + 3 * j + 0];
      const float dy = ay - qr[kRecRho + 3 * j + 1];
      const float dz = az - qr[kRecRho + 3 * j + 2];
      const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
      const float ri = __builtin_amdgcn_rsqf(r2);
      float sn, cs;
      sincosf(S.k * (r2 * ri), &sn, &cs);
      float gr = cs * ri, gi = -sn * ri;
      if constexpr (OP == MF_OP_MFIE) green_to_k(S.k, ri, gr, gi);
      t0r = fmaf(W.w[j], gr, t0r);
      t0i = fmaf(W.w[j], gi, t0i);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float wq = qr[kRecWRho + 3 * j + c];
        t1r[c] = fmaf(wq, gr, t1r[c]);
        t1i[c] = fmaf(wq, gi, t1i[c]);
      }
      if constexpr (OP == MF_OP_MFIE) {
        t2r = fmaf(wr2[j], gr, t2r);
        t2i = fmaf(wr2[j], gi, t2i);
      }
    }
    if constexpr (OP == MF_OP_MFIE) {
      const float a[3] = {ax, ay, az};
      add_point(M, W.w[i], pri, a, nrm, nq, t0r, t0i, t1r, t1i, t2r, t2i);
    } else {
      add_point(M, W.w[i], pri, t0r, t0i, t1r, t1i);
    }
  }
}

// Direct mode, EFIE, with the phase split about the centroid distance d of
// the pair (FP64, passed as dn = d, d2 = d^2, rd = 1/d rounded to FP32).
// With delta = rho_i - rho'_j, R^2 = d^2 + num, num = 2 D.delta + |delta|^2,
// and u = R - d = num/(R + d) has no cancellation.  The moments accumulate
// g'' = exp(-jku)/R - 1/d = (cos ku - 1)/R - u/(R d) - j sin(ku)/R; the
// caller rotates them by exp(-jkd) and adds exp(-jkd)/d to S0.  With
// one = 1 and rd = 0 (a pair whose centroids coincide) g'' is exp(-jku)/R
// and u = R: no reference.
template <int Q>
__device__ __forceinline__ void moments_direct_split(Moments &M, const FillScalars &S,
                                                     const FillRule &W, const float *pr, float hx,
                                                     float hy, float hz, float dn, float d2,
                                                     float rd, float one, cfloat *qr) {
  zero(M);
#pragma unroll 1
  for (int i = 0; i < Q; ++i) {
    float pri[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) pri[c] = pr[kRecRho + 3 * i + c];
    float t0r = 0.f, t0i = 0.f, t1r[3] = {0.f, 0.f, 0.f}, t1i[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const float ex = pri[0] - qr[kRecRho + 3 * j + 0];
      const float ey = pri[1] - qr[kRecRho + 3 * j + 1];
      const float ez = pri[2] - qr[kRecRho + 3 * j + 2];
      const float ee = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
      const float de = fmaf(hx, ex, fmaf(hy, ey, hz * ez));
      const float num = fmaf(2.0f, de, ee);
      const float r2 = d2 + num;
      const float ri = __builtin_amdgcn_rsqf(r2);
      const float u = num * __builtin_amdgcn_rcpf(fmaf(r2, ri, dn));
      float sn, cs;
      sincosf(S.k * u, &sn, &cs);
      const float gr = fmaf((cs - 1.0f) + one, ri, -(u * ri) * rd), gi = -sn * ri;
      t0r = fmaf(W.w[j], gr, t0r);
      t0i = fmaf(W.w[j], gi, t0i);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float wq = qr[kRecWRho + 3 * j + c];
        t1r[c] = fmaf(wq, gr, t1r[c]);
        t1i[c] = fmaf(wq, gi, t1i[c]);
      }
    }
    add_point(M, W.w[i], pri, t0r, t0i, t1r, t1i);
  }
}

// The reference of direct mode for a triangle pair with FP64 centroid offset
// D: d = |D|, 1/d (0 when the centroids coincide) and exp(-jkd).  Evaluated
// without contraction, so that the fill and the cut-edge fix-up, which
// recompute it, round it identically (the sign of D does not matter).
struct PairRef {
  double d, d2, id, sn, cs;
};
__device__ __forceinline__ PairRef pair_ref(double Dx, double Dy, double Dz, double kd) {
#pragma clang fp contract(off)
  PairRef P;
  P.d2 = Dx * Dx + Dy * Dy + Dz * Dz;
  P.d = sqrt(P.d2);
  P.id = P.d > 0.0 ? 1.0 / P.d : 0.0;
  sincos(kd * P.d, &P.sn, &P.cs);
  return P;
}

// FP32 rounding of the reference exp(-jkd)/d.
__device__ __forceinline__ float2 pair_ref_g(const PairRef &P) {
#pragma clang fp contract(off)
  return make_float2((float)(P.cs * P.id), (float)(-P.sn * P.id));
}

// Complex product (xr + j xi)(er + j ei) in place.
__device__ __forceinline__ void crot(float &xr, float &xi, float er, float ei) {
  const float yr = fmaf(xr, er, -xi * ei);
  xi = fmaf(xr, ei, xi * er);
  xr = yr;
}

// Second difference of the per-pair references over the four triangle pairs
// of entry (row r of block I, column c of block J), in FP64, times
// -l_m l_n / k^2: the reference part of the entry's div-div term.
// The second difference a - b - c + d of the references of an entry's four
// triangle pairs (+m +n, +m -n, -m +n, -m -n), in FP64, times -l_m l_n / k^2.
__device__ __forceinline__ void ref_second_difference(const FillItem &S, float2 a, float2 b,
                                                      float2 c2, float2 d, int em, int en,
                                                      float &vr, float &vi) {
  const double sr = ((double)a.x - (double)b.x) - ((double)c2.x - (double)d.x);
  const double si = ((double)a.y - (double)b.y) - ((double)c2.y - (double)d.y);
  const double f = -((double)S.elen[em] * (double)S.elen[en]) / (S.kd * S.kd);
  vr = (float)(f * sr);
  vi = (float)(f * si);
}

__device__ __forceinline__ void ref_part(const FillItem &S, const float2 *gref, int I, int J,
                                         int r, int c, int em, int en, float &vr, float &vi) {
  const int rtI = S.blk_rt[I * kMaxBlockEdges + r], rtJ = S.blk_rt[J * kMaxBlockEdges + c];
  const int pp = rtI & 0xff, pm = (rtI >> 8) & 0xff, qp = rtJ & 0xff, qm = (rtJ >> 8) & 0xff;
  ref_second_difference(S, gref[qp * kRefStride + pp], gref[qm * kRefStride + pp],
                        gref[qp * kRefStride + pm], gref[qm * kRefStride + pm], em, en, vr, vi);
}

// Direct-mode moments of one regular pair: the split-phase moments rotated
// by exp(-jkd), the FP32 reference g = fl(exp(-jkd)/d) and, in scr/sci, S0
// less g (the remainder of the reference kept, g added back in FP64 at
// write-out).
template <int Q>
__device__ __forceinline__ void direct_pair(Moments &M, const FillScalars &S, const FillRule &W,
                                            const float *pr, cfloat *qr, double Dx, double Dy,
                                            double Dz, float hx, float hy, float hz, float &gr,
                                            float &gi, float &scr, float &sci) {
  // everything the pair needs from its FP64 reference, in FP32, before the
  // long point-pair loop: the doubles do not stay live across it
  float er, ei, dgr, dgi, fd, fd2, fid, one;
  {
    const PairRef P = pair_ref(Dx, Dy, Dz, S.kd);
    er = (float)P.cs;  // exp(-jkd)
    ei = (float)-P.sn;
    const double gcr = P.cs * P.id, gci = -P.sn * P.id;
    const float2 g = pair_ref_g(P);
    gr = g.x;
    gi = g.y;
    dgr = (float)(gcr - (double)gr);
    dgi = (float)(gci - (double)gi);
    fd = (float)P.d;
    fd2 = (float)P.d2;
    fid = (float)P.id;
    one = P.d > 0.0 ? 0.0f : 1.0f;
  }
  moments_direct_split<Q>(M, S, W, pr, hx, hy, hz, fd, fd2, fid, one, qr);
  crot(M.s0r, M.s0i, er, ei);
  crot(M.srr, M.sri, er, ei);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    crot(M.spr[c], M.spi[c], er, ei);
    crot(M.sqr[c], M.sqi[c], er, ei);
  }
  scr = M.s0r + dgr;
  sci = M.s0i + dgi;
}

// The item's Green table: the interval coefficients are copied into LDS
// after the accumulator when they fit, the bucket records stay in global
// memory (read through the vector L1).  Splitting the two gathers of a lookup
// between the LDS and the vector-memory path measured 5 % faster than both in
// LDS, whose bank conflicts bind the kernel (and 9 % faster than the bucket
// records in LDS with the coefficients in global memory).
template <bool kLDS, int kThreads>
__device__ __forceinline__ TabPtrs load_table(const FillItem &S, float4 *lds_coef) {
  const int ne = S.tn - 1;
  if (!kLDS) return TabPtrs{S.look, S.coef, S.coef + ne};
  for (int i = threadIdx.x; i < 2 * ne; i += kThreads)
    lds_coef[i < ne ? i : kLdsCoefHalf + (i - ne)] = S.coef[i];
  return TabPtrs{S.look, lds_coef, lds_coef + kLdsCoefHalf};
}

// One tile of one item: accumulate it in LDS, then write it and its mirror.
// The item's arrays come in as separate __restrict__ parameters: once the
// function is inlined they carry no-alias scopes, which lets the
// wave-uniform source records go through scalar loads into SGPRs.
template <int Q, int MODE, int PART, typename ZT, int kFillThreads, bool kSparse = false,
          bool kLDS = false>
__device__ __forceinline__ void fill_tile(
    const FillItem &S, const FillRule &W, const TabPtrs &tab, float *acc, float2 *gref, int local,
    bool &oor, const float *__restrict__ rec, const int32_t *__restrict__ tiles,
    const int32_t *__restrict__ blk_e0, const int32_t *__restrict__ blk_off,
    const int32_t *__restrict__ blk_tri, const int32_t *__restrict__ blk_pos,
    const int32_t *__restrict__ touch_off, const int32_t *__restrict__ touch_q,
    const float *__restrict__ sing, ZT *__restrict__ Z) {
  constexpr int kWaves = kFillThreads / 64;
  // direct mode: reference of the div-div term per triangle pair (see top)
  constexpr bool kRef = MODE == MF_MODE_DIRECT && !(PART & MF_PART_A);
  const int lane = threadIdx.x & 63;
  const int wave = uniform(threadIdx.x >> 6);
  const int tij = tiles[local];
  const int I = (int)((unsigned)tij >> 16), J = tij & 0xffff;
  for (int i = threadIdx.x; i < 2 * kAccFloats; i += kFillThreads) acc[i] = 0.0f;
  __syncthreads();
  const int p0 = blk_off[I], np = blk_off[I + 1] - p0;
  const int q0 = blk_off[J], nq = blk_off[J + 1] - q0;
  for (int pc = 0; pc < np; pc += 64) {
    const bool pv = pc + lane < np;
    const int pidx = pv ? pc + lane : pc;
    const int p = blk_tri[p0 + pidx];
    const int prow = pv ? blk_pos[p0 + pidx] : -1;
    const float *pr = rec + (size_t)p * kRecFloats;
    float palpha[3][3], psig[3];  // read from the record where they are used
    const double *pcd = reinterpret_cast<const double *>(pr + kRecCent);
    const double pcx = pcd[0], pcy = pcd[1], pcz = pcd[2];
    const int *pvi = reinterpret_cast<const int *>(pr + kRecVid);
    const int pv0 = pvi[0], pv1 = pvi[1], pv2 = pvi[2];

    for (int qi = wave; qi < nq; qi += kWaves) {
      const int q = uniform(as_const(blk_tri)[q0 + qi]);
      const int qcol = uniform(as_const(blk_pos)[q0 + qi]);
      cfloat *qr = as_const(rec) + (size_t)q * kRecFloats;
      cint32 *qvi = (cint32 *)(qr + kRecVid);
      const int qv0 = qvi[0], qv1 = qvi[1], qv2 = qvi[2];
      const bool touch = pv0 == qv0 || pv0 == qv1 || pv0 == qv2 || pv1 == qv0 || pv1 == qv1 ||
                         pv1 == qv2 || pv2 == qv0 || pv2 == qv1 || pv2 == qv2;
      float Xr[3][3], Xi[3][3];
      if (!touch) {
        cdouble *qcd = (cdouble *)(qr + kRecCent);
        const double Dx = pcx - qcd[0], Dy = pcy - qcd[1], Dz = pcz - qcd[2];
        const float hx = (float)Dx, hy = (float)Dy, hz = (float)Dz;
        const float lx = (float)(Dx - (double)hx), ly = (float)(Dy - (double)hy),
                    lz = (float)(Dz - (double)hz);
        if (MODE == MF_MODE_TABLE) {
          Bary N;
          moments_bary<Q, kLDS>(N, tab, S, W, pr, hx, hy, hz, lx, ly, lz, qr, oor);
          float al[3][3], be[3][3];
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              al[a][c] = pr[kRecAlpha + 3 * a + c];
              be[a][c] = qr[kRecAlpha + 3 * a + c];
            }
          entries_bary<PART>(N, al, be, S.ik2, Xr, Xi);
        } else {
          Moments M;
          // s0r/s0i: S0 for the vector terms; scr/sci: S0 for the div-div term,
          // less the reference the write-out adds back in FP64 (direct mode)
          float s0r, s0i, scr, sci;
          {
            float gr, gi;
            direct_pair<Q>(M, S, W, pr, qr, Dx, Dy, Dz, hx, hy, hz, gr, gi, scr, sci);
            if (kRef) {
              if (pv) gref[qi * kRefStride + pidx] = make_float2(gr, gi);
              s0r = gr + scr;
              s0i = gi + sci;
            } else {
              s0r = scr = gr + scr;
              s0i = sci = gi + sci;
            }
          }
          const float srr = M.srr, sri = M.sri;
          const float *spr = M.spr, *spi = M.spi, *sqr = M.sqr, *sqi = M.sqi;
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) palpha[a][c] = pr[kRecAlpha + 3 * a + c];
          // X_ab = (Srr + alpha_a.Srho' + beta_b.Srho + (alpha_a.beta_b) S0)/4 - S0/k^2,
          // with the parts that depend on a or b alone formed once
          float c0r = 0.f, c0i = 0.f;
          if (!(PART & MF_PART_PHI)) {
            c0r = 0.25f * srr;
            c0i = 0.25f * sri;
          }
          if (!(PART & MF_PART_A)) {
            c0r = fmaf(-S.ik2, scr, c0r);
            c0i = fmaf(-S.ik2, sci, c0i);
          }
          float Ar[3], Ai[3], Br[3], Bi[3], beta[3][3];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            Ar[a] = c0r;
            Ai[a] = c0i;
            Br[a] = Bi[a] = 0.f;
#pragma unroll
            for (int c = 0; c < 3; ++c) beta[a][c] = qr[kRecAlpha + 3 * a + c];
            if (!(PART & MF_PART_PHI)) {
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                Ar[a] = fmaf(0.25f * palpha[a][c], sqr[c], Ar[a]);
                Ai[a] = fmaf(0.25f * palpha[a][c], sqi[c], Ai[a]);
                Br[a] = fmaf(0.25f * beta[a][c], spr[c], Br[a]);
                Bi[a] = fmaf(0.25f * beta[a][c], spi[c], Bi[a]);
              }
            }
          }
          const float q0r = 0.25f * s0r, q0i = 0.25f * s0i;
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              float vr = Ar[a] + Br[b], vi = Ai[a] + Bi[b];
              if (!(PART & MF_PART_PHI)) {
                const float ab = palpha[a][0] * beta[b][0] + palpha[a][1] * beta[b][1] +
                                 palpha[a][2] * beta[b][2];
                vr = fmaf(ab, q0r, vr);
                vi = fmaf(ab, q0i, vi);
              }
              Xr[a][b] = vr;
              Xi[a][b] = vi;
            }
        }
      } else {
        int s = touch_off[p];
        const int s1 = touch_off[p + 1];
        while (s < s1 && touch_q[s] != q) ++s;
        const bool found = s < s1;  // always: touching pairs are listed both ways
        const float *x = sing + (size_t)(found ? s : 0) * 18;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            Xr[a][b] = found ? x[2 * (3 * a + b)] : 0.0f;
            Xi[a][b] = found ? x[2 * (3 * a + b) + 1] : 0.0f;
          }
        if (kRef && pv) gref[qi * kRefStride + pidx] = make_float2(0.0f, 0.0f);
      }
      if (pv) {
#pragma unroll
        for (int a = 0; a < 3; ++a) psig[a] = pr[kRecSigma + a];
        // Accumulation without atomics.  Each entry is kept in two halves,
        // by the sign of the source triangle in the column's RWG function;
        // a source triangle belongs to one wave, so no other wave writes the
        // halves it adds to.  Within the wave the two triangles of a row's
        // RWG function are two lanes: rows of the plus triangle are added in
        // a first pass and rows of the minus triangle in a second, so no two
        // lanes of one instruction share an address.
#pragma unroll
        for (int pass = 0; pass < 2; ++pass)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const int row = (prow >> (8 * a)) & 0xff;
            if (row == 0xff || (psig[a] < 0.0f) != (pass == 1)) continue;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              const int col = (qcol >> (8 * b)) & 0xff;
              if (col == 0xff) continue;
              const float qs = qr[kRecSigma + b];
              const float sg = psig[a] * qs;
              float *dst = acc + (qs < 0.0f ? kAccFloats : 0) + row * kAccStride + 2 * col;
              dst[0] += sg * Xr[a][b];
              dst[1] += sg * Xi[a][b];
            }
          }
      }
    }
  }
  __syncthreads();
  const int i0 = blk_e0[I], ni = blk_e0[I + 1] - i0;
  const int j0 = blk_e0[J], nj = blk_e0[J + 1] - j0;
  if (kSparse) {
    // near-field entries only, into the CSR values (Z) at their positions
    for (int e = S.sp_off[local] + threadIdx.x; e < S.sp_off[local + 1]; e += kFillThreads) {
      const int4 en = S.sp_ent[e];
      const int r = en.x >> 8, c = en.x & 0xff;
      const int o = r * kAccStride + 2 * c;
      float ar = acc[o] + acc[kAccFloats + o], ai = acc[o + 1] + acc[kAccFloats + o + 1];
      if (kRef) {
        float vr, vi;
        ref_part(S, gref, I, J, r, c, i0 + r, j0 + c, vr, vi);
        ar += vr;
        ai += vi;
      }
      ZT v;
      v.x = -S.pref * ai;
      v.y = S.pref * ar;
      store_stream(Z + en.y, v);
      if (en.z >= 0) store_stream(Z + en.z, v);
    }
  } else {
    if (kRef) {
      // the reference part of every entry, into the first half
      for (int e = threadIdx.x; e < ni * nj; e += kFillThreads) {
        const int r = e / nj, c = e % nj;
        const int o = r * kAccStride + 2 * c;
        float vr, vi;
        ref_part(S, gref, I, J, r, c, i0 + r, j0 + c, vr, vi);
        acc[o] += vr;
        acc[o + 1] += vi;
      }
      __syncthreads();
    }
    // Z = j k eta/(4 pi) * acc, and its transpose below the diagonal
    for (int e = threadIdx.x; e < ni * nj; e += kFillThreads) {
      const int r = e / nj, c = e % nj;
      const int o = r * kAccStride + 2 * c;
      const float ar = acc[o] + acc[kAccFloats + o], ai = acc[o + 1] + acc[kAccFloats + o + 1];
      ZT v;
      v.x = -S.pref * ai;
      v.y = S.pref * ar;
      store_stream(Z + (size_t)(i0 + r) * S.ldz + (j0 + c), v);
    }
    if (I != J) {
      for (int e = threadIdx.x; e < ni * nj; e += kFillThreads) {
        const int c = e / ni, r = e % ni;
        const int o = r * kAccStride + 2 * c;
        const float ar = acc[o] + acc[kAccFloats + o], ai = acc[o + 1] + acc[kAccFloats + o + 1];
        ZT v;
        v.x = -S.pref * ai;
        v.y = S.pref * ar;
        store_stream(Z + (size_t)(j0 + c) * S.ldz + (i0 + r), v);
      }
    }
  }
  __syncthreads();
}

// One MFIE tile.  The operator is not symmetric: a tile (I, J) with I != J
// accumulates rows I against columns J in acc and, from the same kernel
// values, rows J against columns I in acc2, each written once.  The test
// points are read from the record per test point (the moments of both
// directions hold the registers the EFIE tile gives to them).
template <int Q, int MODE, typename ZT, int kFillThreads, bool kLDS = false>
__device__ __forceinline__ void fill_tile_mfie(
    const FillItem &S, const FillRule &W, const TabPtrs &tab, float *acc, float *acc2, int local,
    float &rlo, float &rhi, const float *__restrict__ rec, const int32_t *__restrict__ tiles,
    const int32_t *__restrict__ blk_e0, const int32_t *__restrict__ blk_off,
    const int32_t *__restrict__ blk_tri, const int32_t *__restrict__ blk_pos,
    const int32_t *__restrict__ touch_off, const int32_t *__restrict__ touch_q,
    const int32_t *__restrict__ touch_rev, const float *__restrict__ sing, ZT *__restrict__ Z) {
  constexpr int kWaves = kFillThreads / 64;
  const int lane = threadIdx.x & 63;
  const int wave = uniform(threadIdx.x >> 6);
  const int tij = tiles[local];
  const int I = (int)((unsigned)tij >> 16), J = tij & 0xffff;
  const bool rev = I != J;  // also the block (J, I)
  for (int i = threadIdx.x; i < kAccFloats; i += kFillThreads) acc[i] = 0.0f;
  if (rev)
    for (int i = threadIdx.x; i < kAccFloats; i += kFillThreads) acc2[i] = 0.0f;
  __syncthreads();
  const int p0 = blk_off[I], np = blk_off[I + 1] - p0;
  const int q0 = blk_off[J], nq = blk_off[J + 1] - q0;
  for (int pc = 0; pc < np; pc += 64) {
    const bool pv = pc + lane < np;
    const int pidx = pv ? pc + lane : pc;
    const int p = blk_tri[p0 + pidx];
    const int prow = pv ? blk_pos[p0 + pidx] : -1;
    const float *pr = rec + (size_t)p * kRecFloats;
    float palpha[3][3], psig[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int c = 0; c < 3; ++c) palpha[a][c] = pr[kRecAlpha + 3 * a + c];
      psig[a] = pr[kRecSigma + a];
    }
    // unit normal of p (alpha_0 - alpha_a = v_a - v_0)
    float nrm[3];
    {
      float e1[3], e2[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        e1[c] = palpha[0][c] - palpha[1][c];
        e2[c] = palpha[0][c] - palpha[2][c];
      }
      cross3(e1, e2, nrm);
      const float inv = __builtin_amdgcn_rsqf(dot3(nrm, nrm));
#pragma unroll
      for (int c = 0; c < 3; ++c) nrm[c] *= inv;
    }
    const double *pcd = reinterpret_cast<const double *>(pr + kRecCent);
    const double pcx = pcd[0], pcy = pcd[1], pcz = pcd[2];
    const int *pvi = reinterpret_cast<const int *>(pr + kRecVid);
    const int pv0 = pvi[0], pv1 = pvi[1], pv2 = pvi[2];

    // the source triangles in rounds of pairwise non-adjacent triangles, one
    // per wave, with a barrier after each round: no two waves add to one
    // column of the forward block or one row of the reverse block at once
    const int32_t *rs = S.blk_rounds + (size_t)J * (kEBMaxRounds + 1);
    for (int rd = 0; rd < kEBMaxRounds; ++rd) {
      const int r0 = uniform(rs[rd]), r1 = uniform(rs[rd + 1]);
      if (r0 == r1) break;
      for (int j = r0 + wave; j < r1; j += kWaves) {
        const int qi = uniform(as_const(S.blk_ord)[q0 + j]);
        const int q = uniform(as_const(blk_tri)[q0 + qi]);
        const int qcol = uniform(as_const(blk_pos)[q0 + qi]);
        cfloat *qr = as_const(rec) + (size_t)q * kRecFloats;
        cint32 *qvi = (cint32 *)(qr + kRecVid);
        const int qv0 = qvi[0], qv1 = qvi[1], qv2 = qvi[2];
        const bool touch = pv0 == qv0 || pv0 == qv1 || pv0 == qv2 || pv1 == qv0 || pv1 == qv1 ||
                           pv1 == qv2 || pv2 == qv0 || pv2 == qv1 || pv2 == qv2;
        float Xr[3][3], Xi[3][3];
        float Rr[3][3], Ri[3][3];  // reverse block [b][a] (q tested against p)
        if (!touch) {
          cdouble *qcd = (cdouble *)(qr + kRecCent);
          const double Dx = pcx - qcd[0], Dy = pcy - qcd[1], Dz = pcz - qcd[2];
          const float hx = (float)Dx, hy = (float)Dy, hz = (float)Dz;
          const float lx = (float)(Dx - (double)hx), ly = (float)(Dy - (double)hy),
                      lz = (float)(Dz - (double)hz);
          // unit normal of q (from its record, wave-uniform)
          float qn[3];
          {
            float e1[3], e2[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              e1[c] = qr[kRecAlpha + c] - qr[kRecAlpha + 3 + c];
              e2[c] = qr[kRecAlpha + c] - qr[kRecAlpha + 6 + c];
            }
            cross3(e1, e2, qn);
            const float inv = __builtin_amdgcn_rsqf(dot3(qn, qn));
#pragma unroll
            for (int c = 0; c < 3; ++c) qn[c] *= inv;
          }
          MomentsM M;
          if (MODE == MF_MODE_TABLE)
            moments_table_mfie<Q, kLDS>(M, tab, S, W, pr, nrm, qn, hx, hy, hz, lx, ly, lz, qr,
                                        rlo, rhi);
          else
            moments_direct<Q, MF_OP_MFIE>(M, S, W, pr, nrm, qn, hx, hy, hz, lx, ly, lz, qr);
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            float tau[3], Yr[3], Yi[3];
            cross3(palpha[a], nrm, tau);
            cross3(tau, M.dr, Yr);
            cross3(tau, M.di, Yi);
            const float yr = dot3(tau, M.xr) + M.m0r;
            const float yi = dot3(tau, M.xi) + M.m0i;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              Yr[c] += M.sr[c];
              Yi[c] += M.si[c];
            }
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              const float beta[3] = {qr[kRecAlpha + 3 * b], qr[kRecAlpha + 3 * b + 1],
                                     qr[kRecAlpha + 3 * b + 2]};
              Xr[a][b] = 0.25f * (dot3(beta, Yr) + yr);
              Xi[a][b] = 0.25f * (dot3(beta, Yi) + yi);
            }
          }
          if (rev) {
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              float tau[3], Yr[3], Yi[3];
              const float beta[3] = {qr[kRecAlpha + 3 * b], qr[kRecAlpha + 3 * b + 1],
                                     qr[kRecAlpha + 3 * b + 2]};
              cross3(beta, qn, tau);
              cross3(M.dr, tau, Yr);  // tau x Md' = Md x tau (Md' = -Md)
              cross3(M.di, tau, Yi);
              const float yr = dot3(tau, M.qxr) + M.q0r;
              const float yi = dot3(tau, M.qxi) + M.q0i;
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                Yr[c] += M.qsr[c];
                Yi[c] += M.qsi[c];
              }
#pragma unroll
              for (int a = 0; a < 3; ++a) {
                Rr[b][a] = 0.25f * (dot3(palpha[a], Yr) + yr);
                Ri[b][a] = 0.25f * (dot3(palpha[a], Yi) + yi);
              }
            }
          }
        } else {
          int s = touch_off[p];
          const int s1 = touch_off[p + 1];
          while (s < s1 && touch_q[s] != q) ++s;
          const bool found = s < s1;  // always: touching pairs are listed both ways
          const float *x = sing + (size_t)(found ? s : 0) * 18;
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              Xr[a][b] = found ? x[2 * (3 * a + b)] : 0.0f;
              Xi[a][b] = found ? x[2 * (3 * a + b) + 1] : 0.0f;
            }
          if (rev) {  // the pair (q, p), block [b][a]
            const float *y = sing + (size_t)(found ? touch_rev[s] : 0) * 18;
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
              for (int a = 0; a < 3; ++a) {
                Rr[b][a] = found ? y[2 * (3 * b + a)] : 0.0f;
                Ri[b][a] = found ? y[2 * (3 * b + a) + 1] : 0.0f;
              }
          }
        }
        if (pv) {
          // Plain adds: the rounds keep the waves apart, and within the wave
          // the rows of an edge's plus and minus triangles (two lanes) are
          // added in two passes, in both blocks.
#pragma unroll
          for (int pass = 0; pass < 2; ++pass)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              const int row = (prow >> (8 * a)) & 0xff;
              if (row == 0xff || (psig[a] < 0.0f) != (pass == 1)) continue;
#pragma unroll
              for (int b = 0; b < 3; ++b) {
                const int col = (qcol >> (8 * b)) & 0xff;
                if (col == 0xff) continue;
                const float sg = psig[a] * qr[kRecSigma + b];
                float *dst = acc + row * kAccStride + 2 * col;
                dst[0] += sg * Xr[a][b];
                dst[1] += sg * Xi[a][b];
                if (rev) {
                  float *dst2 = acc2 + col * kAccStride + 2 * row;
                  dst2[0] += sg * Rr[b][a];
                  dst2[1] += sg * Ri[b][a];
                }
              }
            }
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  // Z = acc/(4 pi): rows of block I, columns of block J; and the reverse
  const int i0 = blk_e0[I], ni = blk_e0[I + 1] - i0;
  const int j0 = blk_e0[J], nj = blk_e0[J + 1] - j0;
  for (int e = threadIdx.x; e < ni * nj; e += kFillThreads) {
    const int r = e / nj, c = e % nj;
    ZT v;
    const int o = r * kAccStride + 2 * c;
    v.x = S.pref * acc[o];
    v.y = S.pref * acc[o + 1];
    store_stream(Z + (size_t)(i0 + r) * S.ldz + (j0 + c), v);
  }
  if (rev) {
    for (int e = threadIdx.x; e < ni * nj; e += kFillThreads) {
      const int r = e / ni, c = e % ni;
      ZT v;
      v.x = S.pref * acc2[r * kAccStride + 2 * c];
      v.y = S.pref * acc2[r * kAccStride + 2 * c + 1];
      store_stream(Z + (size_t)(j0 + r) * S.ldz + (i0 + c), v);
    }
  }
  __syncthreads();
}

template <int Q, int MODE, bool kLDS, int PART, typename ZT, bool kSparse, int OP = MF_OP_EFIE>
__global__ __launch_bounds__((fill_threads_op<MODE, OP>()))
__attribute__((amdgpu_waves_per_eu(fill_threads_op<MODE, OP>() / 256,
                                   fill_threads_op<MODE, OP>() / 256))) void k_fill(
    FillItem S, FillRule W) {
  constexpr int kFillThreads = fill_threads_op<MODE, OP>();
  // the EFIE's two halves; the MFIE's forward and reverse blocks
  constexpr int kAccs = 2;
  extern __shared__ float4 smem4[];
  float *acc = reinterpret_cast<float *>(smem4);
  float *acc2 = OP == MF_OP_MFIE ? acc + kAccFloats : nullptr;
  const TabPtrs tab = load_table<MODE == MF_MODE_TABLE && kLDS, kFillThreads>(
      S, smem4 + kAccs * kAccFloats / 4 + 1);
  float2 *gref = reinterpret_cast<float2 *>(acc + 2 * kAccFloats + 4);  // direct mode
  float rlo = INFINITY, rhi = 0.0f;  // the MFIE's distance extremes
  bool oor = false;                   // the EFIE's out-of-range flag
  const int ntiles = S.tile_end - S.tile_begin;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    if constexpr (OP == MF_OP_MFIE)
      fill_tile_mfie<Q, MODE, ZT, kFillThreads, MODE == MF_MODE_TABLE && kLDS>(
          S, W, tab, acc, acc2, t, rlo, rhi, S.rec, S.tiles, S.blk_e0, S.blk_off, S.blk_tri,
          S.blk_pos, S.touch_off, S.touch_q, S.touch_rev, S.sing, reinterpret_cast<ZT *>(S.Z));
    else
      fill_tile<Q, MODE, PART, ZT, kFillThreads, kSparse, MODE == MF_MODE_TABLE && kLDS>(
          S, W, tab, acc, gref, t, oor, S.rec, S.tiles, S.blk_e0, S.blk_off, S.blk_tri, S.blk_pos,
          S.touch_off, S.touch_q, S.sing, reinterpret_cast<ZT *>(S.Z));
  }
  if (MODE == MF_MODE_TABLE && (oor || rlo < S.lo_ok || rhi > S.hi_ok)) atomicOr(S.status, 1);
}

// ---- triangle-block tiles (table mode) -------------------------------------
// The halo-free tiling: blocks of at most 64 consecutive triangles, and one
// tile per block pair I <= J evaluates every triangle pair (p in I, q in J)
// exactly once.  The tile accumulates, in one LDS array without atomics,
// the entries between the block edges of I (rows) and of J (columns): the
// edges I and J own (first seen in their triangles) and the non-owner halves
// of edges cut between blocks.  Lane l takes test triangle l of I; the
// waves take the source triangles of J in rounds of pairwise non-adjacent
// triangles with a barrier after each round, so no two waves ever add to
// one column at once, and within a wave the rows of an edge's plus and
// minus triangles are added in two passes.  Write-out: the owned x owned
// rectangle goes to Z (and, transposed, below the diagonal); entries with a
// non-owner half go to the side buffer, whose rows are the cut edges'
// non-owner halves and whose columns are the edges (owned parts) followed by
// the non-owner halves; k_cut_rows and k_cut_cols add them in afterwards.
constexpr int kTBStride = 2 * kTBEdges + 1;  // odd: rows fall in different banks
constexpr int kTBAccFloats = kTBEdges * kTBStride;
// Test-point offsets of a tile's test triangles staged in LDS (21 floats per
// triangle, odd stride), read there by the test-point loop instead of from
// the triangle records.
constexpr int kRhoFloats = 3 * kMaxQ;
// and the fields every triangle pair reads: alpha [0, 9), sigma [9, 12), the
// radius 12, the vertex ids [13, 16) and the FP64 centroid [16, 22) (22
// floats, so each centroid is 8-byte aligned); held in LDS rather than in
// registers across the pair loop
constexpr int kAuxFloats = 22;
constexpr int kAuxVid = 13, kAuxCent = 16;
template <int Q, int MODE, typename ZT, bool kLDS, bool kRhoLDS, int kTBThreads>
__device__ __forceinline__ void fill_tile_tb(
    const FillItem &S, const FillRule &W, const TabPtrs &tab, float *acc, float2 *gref,
    float *rho_lds, float *aux_lds, int local, bool &oor, const float *__restrict__ rec,
    const int32_t *__restrict__ tb_pos,
    const int32_t *__restrict__ tb_order, const int32_t *__restrict__ touch_off,
    const int32_t *__restrict__ touch_q, const float *__restrict__ sing, ZT *__restrict__ Z,
    float2 *__restrict__ side) {
  constexpr int kWaves = kTBThreads / 64;
  const int lane = threadIdx.x & 63;
  const int wave = uniform(threadIdx.x >> 6);
  const int tij = S.tb_tiles[local];
  const int I = (int)((unsigned)tij >> 16), J = tij & 0xffff;
  const int nbeI = S.tb_nbe[I], nbeJ = S.tb_nbe[J];
  const int tI0 = S.tb_t0[I], npI = S.tb_t0[I + 1] - tI0;
  const int tJ0 = S.tb_t0[J];
  for (int i = threadIdx.x; i < nbeI * kTBStride; i += kTBThreads) acc[i] = 0.0f;
  if (kRhoLDS) {
    for (int x = threadIdx.x; x < npI * kRhoFloats; x += kTBThreads) {
      const int l = x / kRhoFloats, e = x - l * kRhoFloats;
      rho_lds[x] = rec[(size_t)(tI0 + l) * kRecFloats + kRecRho + e];
    }
    for (int x = threadIdx.x; x < npI * kAuxFloats; x += kTBThreads) {
      const int l = x / kAuxFloats, e = x - l * kAuxFloats;
      const int f = e < 12         ? kRecAlpha + e
                    : e == 12      ? kRecRad
                    : e < kAuxCent ? kRecVid + (e - kAuxVid)
                                   : kRecCent + (e - kAuxCent);
      aux_lds[x] = rec[(size_t)(tI0 + l) * kRecFloats + f];
    }
  }
  __syncthreads();
  const bool pv = lane < npI;
  const int p = tI0 + (pv ? lane : 0);
  const int prow = pv ? tb_pos[p] : -1;
  const float *pr = rec + (size_t)p * kRecFloats;
  // the test points' offsets (kRecRho = 0 in both layouts)
  const float *prho = kRhoLDS ? rho_lds + (pv ? lane : 0) * kRhoFloats : pr;
  // alpha at [0, 9), sigma at [9, 12) in both layouts (kRecSigma = kRecAlpha + 9)
  const float *paux = kRhoLDS ? aux_lds + (pv ? lane : 0) * kAuxFloats : pr + kRecAlpha;
  // the centroid and vertex ids: read per pair from LDS when staged there
  const double *pcd = reinterpret_cast<const double *>(kRhoLDS ? paux + kAuxCent : pr + kRecCent);
  const int *pvi = reinterpret_cast<const int *>(kRhoLDS ? paux + kAuxVid : pr + kRecVid);
  const int32_t *rs = S.tb_rounds + (size_t)J * (kTBMaxRounds + 1);
  for (int k = 0; k < kTBMaxRounds; ++k) {
    const int s0 = uniform(rs[k]), s1 = uniform(rs[k + 1]);
    if (s0 == s1) break;
    for (int j = s0 + wave; j < s1; j += kWaves) {
      const int q = uniform(as_const(tb_order)[tJ0 + j]);
      const int qcol = uniform(as_const(tb_pos)[q]);
      cfloat *qr = as_const(rec) + (size_t)q * kRecFloats;
      cint32 *qvi = (cint32 *)(qr + kRecVid);
      const int qv0 = qvi[0], qv1 = qvi[1], qv2 = qvi[2];
      const int pv0 = pvi[0], pv1 = pvi[1], pv2 = pvi[2];
      const bool touch = pv0 == qv0 || pv0 == qv1 || pv0 == qv2 || pv1 == qv0 || pv1 == qv1 ||
                         pv1 == qv2 || pv2 == qv0 || pv2 == qv1 || pv2 == qv2;
      float Xr[3][3], Xi[3][3];
      if (!touch) {
        cdouble *qcd = (cdouble *)(qr + kRecCent);
        const double Dx = pcd[0] - qcd[0], Dy = pcd[1] - qcd[1], Dz = pcd[2] - qcd[2];
        const float hx = (float)Dx, hy = (float)Dy, hz = (float)Dz;
        float palpha[3][3], beta[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            palpha[a][c] = paux[3 * a + c];
            beta[a][c] = qr[kRecAlpha + 3 * a + c];
          }
        if (MODE == MF_MODE_TABLE) {
          const float lx = (float)(Dx - (double)hx), ly = (float)(Dy - (double)hy),
                      lz = (float)(Dz - (double)hz);
          // Every point distance of the pair lies within d -+ (radius p +
          // radius q); only waves where that interval leaves the table's range
          // for some lane check each distance (the slack covers rounding).
          const float dd = __builtin_amdgcn_sqrtf(fmaf(hx, hx, fmaf(hy, hy, hz * hz)));
          // the test triangle's radius read where used (LDS when staged)
          const float rr = (kRhoLDS ? paux[12] : pr[kRecRad]) + qr[kRecRad];
          const float sl = 1e-5f * (dd + rr);
          const bool near_end = pv && (dd - rr - sl < S.lo_ok || dd + rr + sl > S.hi_ok);
          Bary N;
          moments_bary<Q, kLDS>(N, tab, S, W, prho, hx, hy, hz, lx, ly, lz, qr, oor,
                                __any(near_end) != 0);
          entries_bary<0>(N, palpha, beta, S.ik2, Xr, Xi);
        } else {
          Moments M;
          // s0r/s0i: S0 of the vector terms; scr/sci: S0 of the div-div term
          // less the reference that the write-out adds in FP64
          float gr, gi, scr, sci;
          direct_pair<Q>(M, S, W, prho, qr, Dx, Dy, Dz, hx, hy, hz, gr, gi, scr, sci);
          if (pv) gref[(q - tJ0) * kRefStride + lane] = make_float2(gr, gi);
          const float s0r = gr + scr, s0i = gi + sci;
          const float *spr = M.spr, *spi = M.spi, *sqr = M.sqr, *sqi = M.sqi;
          // X_ab = (Srr + alpha_a.Srho' + beta_b.Srho + (alpha_a.beta_b) S0)/4 - S0/k^2
          const float c0r = fmaf(-S.ik2, scr, 0.25f * M.srr);
          const float c0i = fmaf(-S.ik2, sci, 0.25f * M.sri);
          float Ar[3], Ai[3], Br[3], Bi[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            Ar[a] = c0r;
            Ai[a] = c0i;
            Br[a] = Bi[a] = 0.f;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              Ar[a] = fmaf(0.25f * palpha[a][c], sqr[c], Ar[a]);
              Ai[a] = fmaf(0.25f * palpha[a][c], sqi[c], Ai[a]);
              Br[a] = fmaf(0.25f * beta[a][c], spr[c], Br[a]);
              Bi[a] = fmaf(0.25f * beta[a][c], spi[c], Bi[a]);
            }
          }
          const float q0r = 0.25f * s0r, q0i = 0.25f * s0i;
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              const float ab = palpha[a][0] * beta[b][0] + palpha[a][1] * beta[b][1] +
                               palpha[a][2] * beta[b][2];
              Xr[a][b] = fmaf(ab, q0r, Ar[a] + Br[b]);
              Xi[a][b] = fmaf(ab, q0i, Ai[a] + Bi[b]);
            }
        }
      } else {
        // touching pairs carry no reference
        if (MODE != MF_MODE_TABLE && pv) gref[(q - tJ0) * kRefStride + lane] = make_float2(0.f, 0.f);
        int s = touch_off[p];
        const int s1t = touch_off[p + 1];
        while (s < s1t && touch_q[s] != q) ++s;
        const bool found = s < s1t;  // always: touching pairs are listed both ways
        const float *x = sing + (size_t)(found ? s : 0) * 18;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            Xr[a][b] = found ? x[2 * (3 * a + b)] : 0.0f;
            Xi[a][b] = found ? x[2 * (3 * a + b) + 1] : 0.0f;
          }
      }
      if (pv) {
        float psig[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) psig[a] = paux[9 + a];
        // rows of plus triangles first, then minus: the two triangles of an
        // edge interior to the block are two lanes of this wave
#pragma unroll
        for (int pass = 0; pass < 2; ++pass)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const int row = (prow >> (8 * a)) & 0xff;
            if (row == 0xff || (psig[a] < 0.0f) != (pass == 1)) continue;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              const int col = (qcol >> (8 * b)) & 0xff;
              if (col == 0xff) continue;
              const float sg = psig[a] * qr[kRecSigma + b];
              float *dst = acc + row * kTBStride + 2 * col;
              dst[0] += sg * Xr[a][b];
              dst[1] += sg * Xi[a][b];
            }
          }
      }
    }
    __syncthreads();
  }
  const int e0I = S.tb_e0[I], nownI = S.tb_e0[I + 1] - e0I;
  const int e0J = S.tb_e0[J], nownJ = S.tb_e0[J + 1] - e0J;
  if (MODE != MF_MODE_TABLE) {
    // direct mode: the reference part of every owned entry whose edges are
    // both inside their blocks (the cut-edge fix-up adds it to the others)
    for (int e = threadIdx.x; e < nownI * nownJ; e += kTBThreads) {
      const int r = e / nownJ, c = e % nownJ;
      const int em = e0I + r, en = e0J + c;
      if (S.cut_idx[em] >= 0 || S.cut_idx[en] >= 0) continue;
      const int pp = S.edges[6 * em + 2] - tI0, pm = S.edges[6 * em + 3] - tI0;
      const int qp = S.edges[6 * en + 2] - tJ0, qm = S.edges[6 * en + 3] - tJ0;
      float vr, vi;
      ref_second_difference(S, gref[qp * kRefStride + pp], gref[qm * kRefStride + pp],
                            gref[qp * kRefStride + pm], gref[qm * kRefStride + pm], em, en, vr,
                            vi);
      float *a = acc + r * kTBStride + 2 * c;
      a[0] += vr;
      a[1] += vi;
    }
    __syncthreads();
  }
  // write-out: Z = j k eta/(4 pi) acc; a wave per row, lanes along it
  const int32_t *cutI = S.tb_be_cut + S.tb_be_off[I], *cutJ = S.tb_be_cut + S.tb_be_off[J];
  const float pref = S.pref;
  for (int r = wave; r < nownI; r += kWaves) {
    ZT *zr = Z + (size_t)(e0I + r) * S.ldz + e0J;
    for (int c = lane; c < nownJ; c += 64) {
      const float *a = acc + r * kTBStride + 2 * c;
      ZT v;
      v.x = -pref * a[1];
      v.y = pref * a[0];
      store_stream(zr + c, v);
    }
  }
  if (I != J)
    for (int c = wave; c < nownJ; c += kWaves) {
      ZT *zc = Z + (size_t)(e0J + c) * S.ldz + e0I;
      for (int r = lane; r < nownI; r += 64) {
        const float *a = acc + r * kTBStride + 2 * c;
        ZT v;
        v.x = -pref * a[1];
        v.y = pref * a[0];
        store_stream(zc + r, v);
      }
    }
  // rows that are non-owner halves: side[cut row][column of the J part]
  for (int r = nownI + wave; r < nbeI; r += kWaves) {
    float2 *sr = side + (size_t)cutI[r - nownI] * S.lside;
    for (int c = lane; c < nbeJ; c += 64) {
      const float *a = acc + r * kTBStride + 2 * c;
      const long long col = c < nownJ ? (long long)(e0J + c) : (long long)S.ne + cutJ[c - nownJ];
      store_stream(sr + col, make_float2(-pref * a[1], pref * a[0]));
    }
  }
  // columns that are non-owner halves, as rows of the side buffer (the
  // diagonal tile has them among its rows already)
  if (I != J)
    for (int c = nownJ + wave; c < nbeJ; c += kWaves) {
      float2 *sr = side + (size_t)cutJ[c - nownJ] * S.lside;
      for (int r = lane; r < nbeI; r += 64) {
        const float *a = acc + r * kTBStride + 2 * c;
        const long long col = r < nownI ? (long long)(e0I + r) : (long long)S.ne + cutI[r - nownI];
        store_stream(sr + col, make_float2(-pref * a[1], pref * a[0]));
      }
    }
  __syncthreads();
}

template <int Q, int MODE, bool kLDS, bool kRhoLDS, typename ZT, int kTBThreads>
__global__ __launch_bounds__(kTBThreads)
__attribute__((amdgpu_waves_per_eu(kTBThreads / 256, kTBThreads / 256))) void k_fill_tb(
    FillItem S, FillRule W, int ntiles) {
  extern __shared__ float4 smem4[];
  float *acc = reinterpret_cast<float *>(smem4);
  // after the accumulator: the table's coefficients (table mode; the test
  // points' offsets in the gap between their two halves) or the tile's
  // per-pair references and then the offsets (direct mode)
  const TabPtrs tab =
      load_table<MODE == MF_MODE_TABLE && kLDS, kTBThreads>(S, smem4 + kTBAccFloats / 4 + 1);
  float2 *gref = reinterpret_cast<float2 *>(smem4 + kTBAccFloats / 4 + 1);
  // table mode with the coefficients in LDS: the offsets in the gap after
  // (c0, c1), the per-pair fields in the gap after (c2, c3)
  float *rho_lds =
      MODE != MF_MODE_TABLE ? reinterpret_cast<float *>(gref + kRefFloat2)
      : kLDS               ? reinterpret_cast<float *>(smem4 + kTBAccFloats / 4 + 1 + (S.tn - 1))
                           : reinterpret_cast<float *>(smem4 + kTBAccFloats / 4 + 1);
  float *aux_lds = MODE == MF_MODE_TABLE && kLDS
                       ? reinterpret_cast<float *>(smem4 + kTBAccFloats / 4 + 1 + kLdsCoefHalf +
                                                   (S.tn - 1))
                       : rho_lds + kRhoFloats * kTBTris;
  bool oor = false;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x)
    fill_tile_tb<Q, MODE, ZT, kLDS, kRhoLDS, kTBThreads>(
        S, W, tab, acc, gref, rho_lds, aux_lds, t, oor, S.rec, S.tb_pos, S.tb_order, S.touch_off,
        S.touch_q, S.sing, reinterpret_cast<ZT *>(S.Z), S.side);
  if (MODE == MF_MODE_TABLE && oor) atomicOr(S.status, 1);
}

// Several items on the triangle-block plan in one persistent launch: the
// workgroups stride through the items' concatenated triangle-block tile
// lists (as k_fill_batch does over edge-block tiles), loading each item's
// table once; every item has its own side buffer, and its cut-edge fix-up
// follows the launch.
template <int Q, int MODE, bool kLDS, bool kRhoLDS, typename ZT, int kTBThreads>
__global__ __launch_bounds__(kTBThreads)
__attribute__((amdgpu_waves_per_eu(kTBThreads / 256, kTBThreads / 256))) void k_fill_tb_batch(
    const FillItem *__restrict__ items, int n_items, FillRule W) {
  extern __shared__ float4 smem4[];
  float *acc = reinterpret_cast<float *>(smem4);
  float2 *gref = reinterpret_cast<float2 *>(smem4 + kTBAccFloats / 4 + 1);
  const int G = gridDim.x;
  for (int it = 0; it < n_items; ++it) {
    const FillItem &S = items[it];
    int t = S.tb_begin + (((int)blockIdx.x - S.tb_begin) % G + G) % G;
    if (t >= S.tb_end) continue;
    const TabPtrs tab =
        load_table<MODE == MF_MODE_TABLE && kLDS, kTBThreads>(S, smem4 + kTBAccFloats / 4 + 1);
    float *rho_lds =
        MODE != MF_MODE_TABLE ? reinterpret_cast<float *>(gref + kRefFloat2)
        : kLDS ? reinterpret_cast<float *>(smem4 + kTBAccFloats / 4 + 1 + (S.tn - 1))
               : reinterpret_cast<float *>(smem4 + kTBAccFloats / 4 + 1);
    float *aux_lds = MODE == MF_MODE_TABLE && kLDS
                         ? reinterpret_cast<float *>(smem4 + kTBAccFloats / 4 + 1 +
                                                     kLdsCoefHalf + (S.tn - 1))
                         : rho_lds + kRhoFloats * kTBTris;
    bool oor = false;
    for (; t < S.tb_end; t += G)
      fill_tile_tb<Q, MODE, ZT, kLDS, kRhoLDS, kTBThreads>(
          S, W, tab, acc, gref, rho_lds, aux_lds, t - S.tb_begin, oor, S.rec, S.tb_pos,
          S.tb_order, S.touch_off, S.touch_q, S.sing, reinterpret_cast<ZT *>(S.Z), S.side);
    if (MODE == MF_MODE_TABLE && oor) atomicOr(S.status, 1);
    // the next item's table overwrites this one's in LDS
    __syncthreads();
  }
}

// Cut-edge fix-up, one 64 x 64 tile per workgroup: 64 cut edges c (rows) by
// 64 consecutive edges n (columns).  Each entry Z[c][n] is completed from
// the owned part the fill wrote and the side buffer, (c^ x own n), and for a
// cut n also (own c x n^) and (c^ x n^), and written back along the row.
// The completed tile is then transposed through LDS into the columns c of
// the rows n that are not cut (Z = Z^T; cut rows are completed by their own
// tiles), so every column write of one row falls within the tile's span.
constexpr int kFixTile = 64;

// The reference of triangle pair (p, q) as the fill rounded it: zero for a
// touching pair.
__device__ __forceinline__ float2 tri_pair_ref(const FillItem &S, int p, int q) {
  const float *pr = S.rec + (size_t)p * kRecFloats, *qr = S.rec + (size_t)q * kRecFloats;
  const int *pv = reinterpret_cast<const int *>(pr + kRecVid);
  const int *qv = reinterpret_cast<const int *>(qr + kRecVid);
  bool touch = false;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) touch = touch || pv[a] == qv[b];
  if (touch) return make_float2(0.f, 0.f);
  const double *pc = reinterpret_cast<const double *>(pr + kRecCent);
  const double *qc = reinterpret_cast<const double *>(qr + kRecCent);
  return pair_ref_g(pair_ref(pc[0] - qc[0], pc[1] - qc[1], pc[2] - qc[2], S.kd));
}

template <typename ZT, bool kRef>
__global__ __launch_bounds__(256) void k_cut_fix(ZT *__restrict__ Z, long long ldz, int ne,
                                                 int ncut, const int32_t *__restrict__ cut_edge,
                                                 const int32_t *__restrict__ cut_idx,
                                                 const float2 *__restrict__ side,
                                                 long long lside, FillItem S) {
  __shared__ ZT tile[kFixTile][kFixTile + 1];
  const int n0 = blockIdx.x * kFixTile, ci0 = blockIdx.y * kFixTile;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 4 waves
  const int n = n0 + tx;
  const int cn = n < ne ? cut_idx[n] : -1;
  for (int i = ty; i < kFixTile; i += 4) {
    const int ci = ci0 + i;
    if (ci >= ncut || n >= ne) continue;
    const int c = cut_edge[ci];
    const float2 a = side[(size_t)ci * lside + n];
    ZT z = Z[(size_t)c * ldz + n];
    z.x += a.x;
    z.y += a.y;
    if (cn >= 0) {
      const float2 b = side[(size_t)cn * lside + c];
      const float2 d = side[(size_t)ci * lside + ne + cn];
      z.x += b.x + d.x;
      z.y += b.y + d.y;
    }
    if (kRef) {
      // direct mode: the reference part of the completed entry
      const int cp = S.edges[6 * c + 2], cm = S.edges[6 * c + 3];
      const int np = S.edges[6 * n + 2], nm = S.edges[6 * n + 3];
      float vr, vi;
      ref_second_difference(S, tri_pair_ref(S, cp, np), tri_pair_ref(S, cp, nm),
                            tri_pair_ref(S, cm, np), tri_pair_ref(S, cm, nm), c, n, vr, vi);
      z.x += -S.pref * vi;
      z.y += S.pref * vr;
    }
    store_stream(Z + (size_t)c * ldz + n, z);
    tile[i][tx] = z;
  }
  __syncthreads();
  // columns: row n0 + j (if not cut) receives the 64 values at columns c
  const int ci = ci0 + tx;
  const int c = ci < ncut ? cut_edge[ci] : 0;
  for (int j = ty; j < kFixTile; j += 4) {
    const int m = n0 + j;
    if (m >= ne || ci >= ncut || cut_idx[m] >= 0) continue;
    // an isolated entry per line: streamed past the caches
    store_stream(Z + (size_t)m * ldz + c, tile[tx][j]);
  }
}

// Several items in one persistent launch: the workgroups stride through the
// concatenated tile list, so every workgroup visits the items in order and
// loads each item's table once.
template <int Q, int MODE, bool kLDS, typename ZT, int kFillThreads>
__global__ __launch_bounds__(kFillThreads)
__attribute__((amdgpu_waves_per_eu(kFillThreads / 256, kFillThreads / 256))) void k_fill_batch(
    const FillItem *__restrict__ items, int n_items, FillRule W) {
  extern __shared__ float4 smem4[];
  float *acc = reinterpret_cast<float *>(smem4);
  float2 *gref = reinterpret_cast<float2 *>(acc + 2 * kAccFloats + 4);  // direct mode
  const int G = gridDim.x;
  for (int it = 0; it < n_items; ++it) {
    const FillItem &S = items[it];
    // first tile of this item that falls to this workgroup
    int t = S.tile_begin + (((int)blockIdx.x - S.tile_begin) % G + G) % G;
    if (t >= S.tile_end) continue;
    const TabPtrs tab =
        load_table<MODE == MF_MODE_TABLE && kLDS, kFillThreads>(S, smem4 + 2 * kAccFloats / 4 + 1);
    bool oor = false;
    for (; t < S.tile_end; t += G)
      fill_tile<Q, MODE, 0, ZT, kFillThreads, false, MODE == MF_MODE_TABLE && kLDS>(
          S, W, tab, acc, gref, t - S.tile_begin, oor, S.rec, S.tiles, S.blk_e0, S.blk_off,
          S.blk_tri, S.blk_pos, S.touch_off, S.touch_q, S.sing, reinterpret_cast<ZT *>(S.Z));
    if (MODE == MF_MODE_TABLE && oor) atomicOr(S.status, 1);
  }
}

// A prepared launch over one or more items: the first item travels as a
// kernel argument, the full list (when there are several) in device memory.
struct FillLaunch {
  FillItem first;
  FillRule rule;
  FillItem *d_items = nullptr;  // in the batch's workspace; null for a single item
  int total_tiles = 0, n = 0;
  size_t lds = 0;
  int nq = 0, base = 0, part = 0, z_dtype = 0, op = MF_OP_EFIE;
  int threads = 0;  // workgroup size of a batched launch (0: the mode's default)
  bool lds_tab = false, sparse = false;
  long long grid = 0;
  // Batched launch on the triangle-block plan (every item's mesh has one and
  // a side buffer of its own): shape 1 selects it.
  bool tb_ok = false, tb_in_lds = false, tb_rho_lds = true;
  int shape = 0, tb_total = 0;
  size_t tb_lds = 0;
  std::vector<FillItem> host_items;  // for the per-item cut-edge fix-ups
};

template <typename K>
static int plan_grid(FillLaunch &L, K kern, int threads) {
  if (L.lds > 65536)
    MF_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)L.lds));
  int dev = 0, ncu = 0, per = 0;
  MF_HIP(hipGetDevice(&dev));
  MF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  MF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, threads, L.lds));
  if (per < 1) {
    set_error("mf_fill_Z: fill kernel does not fit on a compute unit");
    return MF_EINVAL;
  }
  L.grid = (long long)ncu * per;
  if (L.grid > L.total_tiles) L.grid = L.total_tiles;
  if (getenv("MOMFILL_VERBOSE"))
    fprintf(stderr, "[momfill] k_fill Q=%d mode=%d lds_table=%d items=%d grid=%lld x %d lds=%zu B\n",
            L.nq, L.base, (int)L.lds_tab, L.n, L.grid, threads, L.lds);
  return MF_OK;
}

// Batched launch with a given workgroup size (the variants the tuner times).
template <int Q, int MODE, bool kLDS, typename ZT, int kThreads>
static int launch_batch(FillLaunch &L, bool plan_only, hipStream_t s) {
  auto kern = k_fill_batch<Q, MODE, kLDS, ZT, kThreads>;
  if (L.grid == 0) {
    const int rc = plan_grid(L, kern, kThreads);
    if (rc) return rc;
  }
  if (plan_only || L.total_tiles == 0) return MF_OK;
  hipLaunchKernelGGL(kern, dim3((unsigned)L.grid), dim3(kThreads), L.lds, s, L.d_items, L.n,
                     L.rule);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <int Q, int MODE, bool kLDS, int PART, typename ZT>
static int launch_t(FillLaunch &L, bool plan_only, hipStream_t s) {
  constexpr int kFillThreads = fill_threads<MODE>();
  if (L.op == MF_OP_MFIE) {
    if constexpr (PART == 0) {
      constexpr int kThr = fill_threads_op<MODE, MF_OP_MFIE>();
      auto kern = k_fill<Q, MODE, kLDS, 0, ZT, false, MF_OP_MFIE>;
      if (L.grid == 0) {
        const int rc = plan_grid(L, kern, kThr);
        if (rc) return rc;
      }
      if (plan_only || L.total_tiles == 0) return MF_OK;
      hipLaunchKernelGGL(kern, dim3((unsigned)L.grid), dim3(kThr), L.lds, s, L.first, L.rule);
    } else {
      set_error("the MFIE fill has no partial modes");
      return MF_EINVAL;
    }
  } else if (L.n == 1 && L.sparse) {
    auto kern = k_fill<Q, MODE, kLDS, PART, ZT, true>;
    if (L.grid == 0) {
      const int rc = plan_grid(L, kern, kFillThreads);
      if (rc) return rc;
    }
    if (plan_only || L.total_tiles == 0) return MF_OK;
    hipLaunchKernelGGL(kern, dim3((unsigned)L.grid), dim3(kFillThreads), L.lds, s, L.first,
                       L.rule);
  } else if (L.n == 1) {
    auto kern = k_fill<Q, MODE, kLDS, PART, ZT, false>;
    if (L.grid == 0) {
      const int rc = plan_grid(L, kern, kFillThreads);
      if (rc) return rc;
    }
    if (plan_only || L.total_tiles == 0) return MF_OK;
    hipLaunchKernelGGL(kern, dim3((unsigned)L.grid), dim3(kFillThreads), L.lds, s, L.first,
                       L.rule);
  } else {
    switch (L.threads ? L.threads : kFillThreads) {
      case 512: return launch_batch<Q, MODE, kLDS, ZT, 512>(L, plan_only, s);
      case 1024: return launch_batch<Q, MODE, kLDS, ZT, 1024>(L, plan_only, s);
      default: return launch_batch<Q, MODE, kLDS, ZT, 768>(L, plan_only, s);
    }
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <int Q, int MODE, bool kLDS, typename ZT>
static int launch_part(FillLaunch &L, bool plan_only, hipStream_t s) {
  if (L.part == MF_PART_A) return launch_t<Q, MODE, kLDS, MF_PART_A, ZT>(L, plan_only, s);
  if (L.part == MF_PART_PHI) return launch_t<Q, MODE, kLDS, MF_PART_PHI, ZT>(L, plan_only, s);
  return launch_t<Q, MODE, kLDS, 0, ZT>(L, plan_only, s);
}

template <int Q, typename ZT>
static int launch_q(FillLaunch &L, bool plan_only, hipStream_t s) {
  if (L.base == MF_MODE_DIRECT) return launch_part<Q, MF_MODE_DIRECT, false, ZT>(L, plan_only, s);
  if (L.lds_tab) return launch_part<Q, MF_MODE_TABLE, true, ZT>(L, plan_only, s);
  return launch_part<Q, MF_MODE_TABLE, false, ZT>(L, plan_only, s);
}

template <typename ZT>
static int launch_z(FillLaunch &L, bool plan_only, hipStream_t s) {
  switch (L.nq) {
    case 3: return launch_q<3, ZT>(L, plan_only, s);
    case 6: return launch_q<6, ZT>(L, plan_only, s);
    default: return launch_q<7, ZT>(L, plan_only, s);
  }
}

// Batched launch on the triangle-block plan, then each item's cut-edge
// fix-up (as launch_tb_t does for one item).
template <int Q, int MODE, bool kLDS, bool kRhoLDS, typename ZT, int kThr>
static int launch_tb_batch(FillLaunch &L, bool plan_only, hipStream_t s) {
  auto kern = k_fill_tb_batch<Q, MODE, kLDS, kRhoLDS, ZT, kThr>;
  if (L.grid == 0) {
    int dev = 0, ncu = 0, per = 0;
    MF_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)L.tb_lds));
    MF_HIP(hipGetDevice(&dev));
    MF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    MF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kThr, L.tb_lds));
    if (per < 1) {
      set_error("batched triangle-block fill kernel does not fit on a compute unit");
      return MF_EINVAL;
    }
    L.grid = std::min<long long>((long long)ncu * per, std::max(L.tb_total, 1));
    if (getenv("MOMFILL_VERBOSE"))
      fprintf(stderr, "[momfill] k_fill_tb_batch Q=%d mode=%d lds_table=%d items=%d grid=%lld x %d lds=%zu B\n",
              Q, MODE, (int)kLDS, L.n, L.grid, kThr, L.tb_lds);
  }
  if (plan_only || L.tb_total == 0) return MF_OK;
  hipLaunchKernelGGL(kern, dim3((unsigned)L.grid), dim3(kThr), L.tb_lds, s, L.d_items, L.n,
                     L.rule);
  MF_HIP(hipGetLastError());
  for (const FillItem &S : L.host_items) {
    if (S.n_cut <= 0) continue;
    const dim3 fg((unsigned)((S.ne + kFixTile - 1) / kFixTile),
                  (unsigned)((S.n_cut + kFixTile - 1) / kFixTile));
    hipLaunchKernelGGL((k_cut_fix<ZT, MODE != MF_MODE_TABLE>), fg, dim3(256), 0, s,
                       reinterpret_cast<ZT *>(S.Z), S.ldz, S.ne, S.n_cut, S.cut_edge, S.cut_idx,
                       reinterpret_cast<const float2 *>(S.side), S.lside, S);
    MF_HIP(hipGetLastError());
  }
  return MF_OK;
}

template <int Q, int MODE, bool kLDS, bool kRhoLDS, typename ZT>
static int launch_tb_batch_t(FillLaunch &L, bool plan_only, hipStream_t s) {
  if (L.threads == 512) return launch_tb_batch<Q, MODE, kLDS, kRhoLDS, ZT, 512>(L, plan_only, s);
  return launch_tb_batch<Q, MODE, kLDS, kRhoLDS, ZT, 1024>(L, plan_only, s);
}

template <int Q, typename ZT>
static int launch_tb_batch_q(FillLaunch &L, bool plan_only, hipStream_t s) {
  if (L.base == MF_MODE_DIRECT)
    return launch_tb_batch_t<Q, MF_MODE_DIRECT, false, true, ZT>(L, plan_only, s);
  if (!L.tb_in_lds) return launch_tb_batch_t<Q, MF_MODE_TABLE, false, true, ZT>(L, plan_only, s);
  return L.tb_rho_lds ? launch_tb_batch_t<Q, MF_MODE_TABLE, true, true, ZT>(L, plan_only, s)
                      : launch_tb_batch_t<Q, MF_MODE_TABLE, true, false, ZT>(L, plan_only, s);
}

template <typename ZT>
static int launch_tb_batch_z(FillLaunch &L, bool plan_only, hipStream_t s) {
  switch (L.nq) {
    case 3: return launch_tb_batch_q<3, ZT>(L, plan_only, s);
    case 6: return launch_tb_batch_q<6, ZT>(L, plan_only, s);
    default: return launch_tb_batch_q<7, ZT>(L, plan_only, s);
  }
}

static int dispatch(FillLaunch &L, bool plan_only, hipStream_t s) {
  if (L.shape == 1) {
    if (L.z_dtype == MF_C64) return launch_tb_batch_z<float2>(L, plan_only, s);
    return launch_tb_batch_z<double2>(L, plan_only, s);
  }
  if (L.z_dtype == MF_C64) return launch_z<float2>(L, plan_only, s);
  return launch_z<double2>(L, plan_only, s);
}

static size_t table_lds_bytes(const mf_tables *tab) {
  // the coefficients (load_table); longer tables stay in global memory
  return tab->g.n - 1 <= kLdsCoefHalf ? sizeof(float4) * 2 * (size_t)kLdsCoefHalf
                                      : ((size_t)1 << 30);
}

static FillItem make_item(const mf_mesh *m, const Rule &r, double k, int base,
                          const mf_tables *tab, void *Z, int64_t ldz, const float *sing,
                          int tile_begin, int tb_begin = 0, float *side = nullptr) {
  FillItem S{};
  S.tile_begin = tile_begin;
  S.tile_end = tile_begin + (int)m->tiles.size();
  S.tb_begin = tb_begin;
  S.tb_end = tb_begin + (m->tb_ok ? (int)m->tb_tiles.size() : 0);
  S.ne = m->ne;
  S.kd = k;
  S.k = (float)k;
  S.ik2 = (float)(1.0 / (k * k));
  S.pref = (float)(k * kEta0 / (4.0 * M_PI));
  S.ldz = ldz;
  S.rec = m->d_rec;
  S.tiles = m->d_tiles;
  S.blk_e0 = m->d_blk_e0;
  S.blk_ord = m->d_blk_ord;
  S.blk_rounds = m->d_blk_rounds;
  S.blk_off = m->d_blk_off;
  S.blk_tri = m->d_blk_tri;
  S.blk_pos = m->d_blk_pos;
  S.blk_rt = m->d_blk_rt;
  S.elen = m->d_elen;
  S.tb_t0 = m->d_tb_t0;
  S.tb_e0 = m->d_tb_e0;
  S.tb_nbe = m->d_tb_nbe;
  S.tb_be_off = m->d_tb_be_off;
  S.tb_be_cut = m->d_tb_be_cut;
  S.tb_pos = m->d_tb_pos;
  S.tb_order = m->d_tb_order;
  S.tb_rounds = m->d_tb_rounds;
  S.tb_tiles = m->d_tb_tiles;
  S.side = reinterpret_cast<float2 *>(side ? side : m->d_side);
  S.lside = (long long)m->ne + m->n_cut;
  S.edges = m->d_edges;
  S.cut_idx = m->d_cut_idx;
  S.cut_edge = m->d_cut_edge;
  S.n_cut = m->tb_ok ? m->n_cut : 0;
  S.touch_off = m->d_touch_off;
  S.touch_q = m->d_touch_q;
  S.touch_rev = m->d_touch_rev;
  S.sing = sing;
  S.Z = Z;
  S.status = m->d_status;
  if (base == MF_MODE_TABLE) {
    const mf_tables::One &g = tab->g;
    S.look = g.look1;
    S.coef = g.coef;
    S.tn = g.n;
    S.tm = g.mb1;
    S.tinv = g.binv1;
    S.tbias = g.bbias1;
    S.tmax = g.btop1;
    S.lo_ok = (float)(tab->rmin * (1.0 - 1e-6));
    S.hi_ok = (float)(tab->rmax * (1.0 + 1e-6));
  }
  return S;
}

// The rule's weights and frame coefficients (FillRule).  The kernels take the
// zero pattern of s_j, t_j from bary_kind; it is checked here against the
// rule's barycentric coordinates.
static bool fill_rule(const Rule &r, FillRule *W) {
  *W = FillRule{};
  for (int j = 0; j < r.nq; ++j) {
    const double s = r.bary[j][0] - r.bary[j][2], t = r.bary[j][1] - r.bary[j][2];
    const int kind = bary_kind(r.nq, j);
    const bool ok = kind == 0   ? (s == 0.0 && t == 0.0)
                    : kind == 1 ? (s != 0.0 && t == 0.0)
                    : kind == 2 ? (s == 0.0 && t != 0.0)
                                : (s != 0.0 && s == t);
    if (!ok) {
      set_error("fill: quadrature rule does not have the orbit layout of the kernels");
      return false;
    }
    W->w[j] = (float)r.w[j];
    W->s2[j] = (float)(2.0 * s);
    W->t2[j] = (float)(2.0 * t);
    W->ws[j] = (float)(r.w[j] * s);
    W->wt[j] = (float)(r.w[j] * t);
  }
  return true;
}

// Builds the launch of n items (all with the same rule, mode and Z type).
// With more than one item the item list is copied to the device here
// (synchronously); running the launch afterwards only enqueues the kernel.
size_t fill_items_bytes(int n) { return sizeof(FillItem) * (size_t)n; }

int fill_launch_create(int n, mf_mesh *const *m, const double *k, const mf_tables *const *tab,
                       const Rule &r, int mode, void *const *Z, int z_dtype, const int64_t *ldz,
                       const float *const *sing, void *items_dev, FillLaunch **out,
                       float *const *side) {
  FillLaunch *L = new (std::nothrow) FillLaunch;
  if (!L) {
    set_error("out of host memory");
    return MF_ENOMEM;
  }
  L->n = n;
  L->nq = r.nq;
  L->base = mode & 0xf;
  L->part = mode & (MF_PART_A | MF_PART_PHI);
  L->op = (mode & kModeMfie) ? MF_OP_MFIE : MF_OP_EFIE;
  L->z_dtype = z_dtype;
  if (!fill_rule(r, &L->rule)) {
    delete L;
    return MF_EINVAL;
  }
  L->lds = sizeof(float) * kAccFloats * 2 + 16;
  // direct EFIE: the per-pair references of the div-div term
  if (L->op == MF_OP_EFIE && L->base == MF_MODE_DIRECT && !(L->part & MF_PART_A))
    L->lds += sizeof(float2) * kRefFloat2;
  // triangle-block tiles for a batch: EFIE, no partial mode, every mesh with a
  // triangle-block plan and every item with a side buffer of its own
  bool tb = n > 1 && L->op == MF_OP_EFIE && L->part == 0 && side != nullptr;
  for (int i = 0; i < n && tb; ++i) tb = m[i]->tb_ok && side[i] != nullptr;
  std::vector<FillItem> items(n);
  size_t tmax = 0;
  int tiles = 0, tb_tiles = 0, tn_max = 0;
  for (int i = 0; i < n; ++i) {
    items[i] = make_item(m[i], r, k[i], L->base, tab ? tab[i] : nullptr, Z[i], ldz[i], sing[i],
                         tiles, tb_tiles, tb ? side[i] : nullptr);
    if (L->op == MF_OP_MFIE) items[i].pref = (float)(1.0 / (4.0 * M_PI));
    tiles = items[i].tile_end;
    tb_tiles = items[i].tb_end;
    if (L->base == MF_MODE_TABLE) {
      tmax = std::max(tmax, table_lds_bytes(tab[i]));
      tn_max = std::max(tn_max, tab[i]->g.n);
    }
  }
  L->total_tiles = tiles;
  L->first = items[0];
  int rc = MF_OK;
  int dev = 0, maxlds = 0;
  {
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
      e = hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) rc = hip_fail(e, "device attributes");
  }
  if (!rc && L->base == MF_MODE_TABLE) {
    if (L->lds + tmax <= (size_t)maxlds) {
      L->lds_tab = true;
      L->lds += tmax;
    }
  }
  if (!rc && tb) {
    // LDS of the triangle-block tile as for a single fill (launch_fill_tb)
    const size_t base = sizeof(float) * kTBAccFloats + 16;
    const size_t rho_bytes = sizeof(float) * kRhoFloats * kTBTris;
    const size_t aux_bytes = sizeof(float) * kAuxFloats * kTBTris;
    size_t lds = base;
    if (L->base == MF_MODE_TABLE) {
      L->tb_in_lds = base + tmax <= (size_t)maxlds;
      if (L->tb_in_lds) {
        lds += tmax;
        L->tb_rho_lds = (size_t)(tn_max - 1) * sizeof(float4) + std::max(rho_bytes, aux_bytes) <=
                        sizeof(float4) * (size_t)kLdsCoefHalf;
      } else {
        lds += rho_bytes + aux_bytes;
      }
    } else {
      lds += sizeof(float2) * kRefFloat2 + rho_bytes + aux_bytes;
    }
    L->tb_ok = lds <= (size_t)maxlds;
    L->tb_lds = lds;
    L->tb_total = tb_tiles;
  }
  L->host_items = items;
  if (!rc && n > 1 && L->op == MF_OP_MFIE) {
    set_error("the MFIE fill takes one item");
    rc = MF_EINVAL;
  }
  if (!rc && n > 1) {
    if (!items_dev) {
      set_error("internal: a batched launch needs device memory for its item list");
      rc = MF_EINVAL;
    } else {
      L->d_items = reinterpret_cast<FillItem *>(items_dev);
      hipError_t e =
          hipMemcpy(L->d_items, items.data(), sizeof(FillItem) * n, hipMemcpyHostToDevice);
      if (e != hipSuccess) rc = hip_fail(e, "fill item list");
    }
  }
  if (!rc) rc = dispatch(*L, true, nullptr);
  if (rc) {
    fill_launch_destroy(L);
    return rc;
  }
  *out = L;
  return MF_OK;
}

int fill_launch_run(FillLaunch *L, hipStream_t s) { return dispatch(*L, false, s); }

// Tile-shape tuner of batched launches.  Candidates: edge-block tiles with
// 512, 768 or 1024 threads per workgroup (2, 3 or 4 waves per SIMD, trading
// each lane's register budget against the latency hiding of the table
// gathers) and, when every item has a triangle-block plan and a side buffer,
// triangle-block tiles with 1024 or 512 threads (one or two source
// triangles per wave and round).  Each candidate runs the whole launch once
// to warm up and once timed with HIP events; the fastest is kept for every
// later launch with the same rule, mode, table placement, output type and
// plan availability in this process (and in the MOMFILL_TUNE_CACHE file).
static const int kBatchCand[kBatchChoices][2] = {
    {0, 512}, {0, 768}, {0, 1024}, {1, 1024}, {1, 512}};

int fill_launch_autotune(FillLaunch *L, hipStream_t s, float *ms, int *threads, int *shape) {
  if (ms)
    for (int i = 0; i < kBatchChoices; ++i) ms[i] = 0.0f;
  if (shape) *shape = 0;
  if (L->n < 2 || L->op != MF_OP_EFIE || L->sparse) {  // single fills keep the defaults
    if (threads)
      *threads = L->threads ? L->threads
                            : (L->op == MF_OP_MFIE ? fill_threads_op<MF_MODE_TABLE, MF_OP_MFIE>()
                                                   : fill_threads<MF_MODE_TABLE>());
    return MF_OK;
  }
  const int nc = L->tb_ok ? kBatchChoices : 3;
  const std::string key = "batch q=" + std::to_string(L->nq) + " mode=" + std::to_string(L->base) +
                          " ldstable=" + std::to_string((int)L->lds_tab) +
                          " z=" + std::to_string(L->z_dtype) + " tb=" + std::to_string((int)L->tb_ok);
  auto apply = [&](int c) {
    L->shape = kBatchCand[c][0];
    L->threads = kBatchCand[c][1];
    L->grid = 0;
    if (threads) *threads = L->threads;
    if (shape) *shape = L->shape;
  };
  {
    int cached = -1;
    if (tune_cache_get(key, &cached) && cached >= 0 && cached < nc) {
      apply(cached);
      return dispatch(*L, true, nullptr);
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MF_HIP(hipEventCreate(&e0));
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(he, "tuner events");
  }
  int rc = MF_OK, best = 1;
  float best_ms = INFINITY;
  for (int c = 0; c < nc && !rc; ++c) {
    apply(c);
    rc = dispatch(*L, false, s);  // warm-up (and grid plan)
    if (rc) break;
    he = hipEventRecord(e0, s);
    if (he == hipSuccess) rc = dispatch(*L, false, s);
    if (!rc && he == hipSuccess) he = hipEventRecord(e1, s);
    if (!rc && he == hipSuccess) he = hipEventSynchronize(e1);
    float t = 0.0f;
    if (!rc && he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
    if (he != hipSuccess) rc = hip_fail(he, "tuner timing");
    if (ms) ms[c] = t;
    if (!rc && t < best_ms) {
      best_ms = t;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  apply(best);
  tune_cache_put(key, best);
  return dispatch(*L, true, nullptr);
}

int fill_launch_set_choice(FillLaunch *L, int c) {
  if (L->n < 2 || L->op != MF_OP_EFIE || L->sparse || c < 0 || c >= kBatchChoices ||
      (kBatchCand[c][0] == 1 && !L->tb_ok)) {
    set_error("mf_batch_set_choice: no such candidate for this batch");
    return MF_EINVAL;
  }
  L->shape = kBatchCand[c][0];
  L->threads = kBatchCand[c][1];
  L->grid = 0;
  return dispatch(*L, true, nullptr);
}

void fill_launch_destroy(FillLaunch *L) { delete L; }

int launch_fill_near(mf_mesh *m, const Rule &r, double k, int mode, const mf_tables *tab,
                     const int32_t *tiles, int ntiles, const int32_t *sp_off, const int4 *sp_ent,
                     void *values, int z_dtype, hipStream_t s) {
  FillLaunch *L = nullptr;
  const float *sing = m->d_sing;
  int64_t ld = m->ne;
  int rc = fill_launch_create(1, &m, &k, &tab, r, mode, &values, z_dtype, &ld, &sing, nullptr, &L);
  if (rc) return rc;
  L->sparse = true;
  L->first.tiles = tiles;
  L->first.tile_begin = 0;
  L->first.tile_end = ntiles;
  L->first.sp_off = sp_off;
  L->first.sp_ent = sp_ent;
  L->total_tiles = ntiles;
  L->grid = 0;  // plan again for the sparse kernel and this tile count
  rc = fill_launch_run(L, s);
  fill_launch_destroy(L);
  return rc;
}

template <int Q, int MODE, bool kLDS, bool kRhoLDS, typename ZT, int kTBThreads>
static int launch_tb_t(mf_mesh *m, const FillItem &S, const FillRule &W, size_t lds,
                       hipStream_t s) {
  auto kern = k_fill_tb<Q, MODE, kLDS, kRhoLDS, ZT, kTBThreads>;
  static std::once_flag once;
  static long long grid = 0;
  static hipError_t ge = hipSuccess;
  std::call_once(once, [&]() {
    int dev = 0, ncu = 0, per = 0;
    ge = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
    if (ge == hipSuccess) ge = hipGetDevice(&dev);
    if (ge == hipSuccess) ge = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ge == hipSuccess)
      ge = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kTBThreads, lds);
    grid = (long long)ncu * per;
  });
  if (ge != hipSuccess) return hip_fail(ge, "triangle-block fill set-up");
  if (grid < 1) {
    set_error("mf_fill_Z: triangle-block fill kernel does not fit on a compute unit");
    return MF_EINVAL;
  }
  const int ntiles = (int)m->tb_tiles.size();
  const long long g = std::min<long long>(grid, ntiles);
  if (getenv("MOMFILL_VERBOSE"))
    fprintf(stderr,
            "[momfill] k_fill_tb Q=%d mode=%d lds_table=%d tiles=%d grid=%lld lds=%zu B cut=%d\n",
            Q, MODE, (int)kLDS, ntiles, g, lds, m->n_cut);
  hipLaunchKernelGGL(kern, dim3((unsigned)g), dim3(kTBThreads), lds, s, S, W, ntiles);
  MF_HIP(hipGetLastError());
  if (m->timing_now) {
    MF_HIP(hipEventRecord(m->ev[4], s));
    m->split = true;
  }
  if (m->n_cut > 0) {
    const dim3 fg((unsigned)((m->ne + kFixTile - 1) / kFixTile),
                  (unsigned)((m->n_cut + kFixTile - 1) / kFixTile));
    hipLaunchKernelGGL((k_cut_fix<ZT, MODE != MF_MODE_TABLE>), fg, dim3(256), 0, s,
                       reinterpret_cast<ZT *>(S.Z), S.ldz, m->ne, m->n_cut, m->d_cut_edge,
                       m->d_cut_idx, reinterpret_cast<const float2 *>(m->d_side), S.lside, S);
    MF_HIP(hipGetLastError());
  }
  return MF_OK;
}

template <int MODE, bool kLDS, bool kRhoLDS, typename ZT, int kTBThreads>
static int launch_tb_q(mf_mesh *m, int nq, const FillItem &S, const FillRule &W, size_t lds,
                       hipStream_t s) {
  switch (nq) {
    case 3: return launch_tb_t<3, MODE, kLDS, kRhoLDS, ZT, kTBThreads>(m, S, W, lds, s);
    case 6: return launch_tb_t<6, MODE, kLDS, kRhoLDS, ZT, kTBThreads>(m, S, W, lds, s);
    default: return launch_tb_t<7, MODE, kLDS, kRhoLDS, ZT, kTBThreads>(m, S, W, lds, s);
  }
}

template <typename ZT, int kTBThreads>
static int launch_tb_z(mf_mesh *m, int nq, int mode, bool in_lds, bool rho_lds, const FillItem &S,
                       const FillRule &W, size_t lds, hipStream_t s) {
  if (mode == MF_MODE_DIRECT)
    return launch_tb_q<MF_MODE_DIRECT, false, true, ZT, kTBThreads>(m, nq, S, W, lds, s);
  if (!in_lds) return launch_tb_q<MF_MODE_TABLE, false, true, ZT, kTBThreads>(m, nq, S, W, lds, s);
  return rho_lds ? launch_tb_q<MF_MODE_TABLE, true, true, ZT, kTBThreads>(m, nq, S, W, lds, s)
                 : launch_tb_q<MF_MODE_TABLE, true, false, ZT, kTBThreads>(m, nq, S, W, lds, s);
}

// EFIE fill on the triangle-block plan (k_fill_tb and the cut-edge fix-up),
// one item, table or direct mode.
static int launch_fill_tb(mf_mesh *m, const Rule &r, double k, int mode, const mf_tables *tab,
                          void *Z, int z_dtype, int64_t ldz, hipStream_t s, int threads) {
  FillItem S = make_item(m, r, k, mode, tab, Z, ldz, m->d_sing, 0);
  FillRule W;
  if (!fill_rule(r, &W)) return MF_EINVAL;
  int dev = 0, maxlds = 0;
  MF_HIP(hipGetDevice(&dev));
  MF_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  const size_t base = sizeof(float) * kTBAccFloats + 16;
  const size_t rho_bytes = sizeof(float) * kRhoFloats * kTBTris;
  const size_t aux_bytes = sizeof(float) * kAuxFloats * kTBTris;
  bool in_lds = false, rho_lds = true;
  size_t lds = base;
  if (mode == MF_MODE_TABLE) {
    const size_t tbytes = table_lds_bytes(tab);
    in_lds = base + tbytes <= (size_t)maxlds;
    if (in_lds) {
      // the offsets go in the gap between the two coefficient halves
      lds += tbytes;
      rho_lds = (size_t)(tab->g.n - 1) * sizeof(float4) + std::max(rho_bytes, aux_bytes) <=
                sizeof(float4) * (size_t)kLdsCoefHalf;
    } else {
      lds += rho_bytes + aux_bytes;
    }
  } else {
    // the tile's per-pair references, then the staged fields
    lds += sizeof(float2) * kRefFloat2 + rho_bytes + aux_bytes;
  }
  if (threads == 512)
    return z_dtype == MF_C64
               ? launch_tb_z<float2, 512>(m, r.nq, mode, in_lds, rho_lds, S, W, lds, s)
               : launch_tb_z<double2, 512>(m, r.nq, mode, in_lds, rho_lds, S, W, lds, s);
  return z_dtype == MF_C64
             ? launch_tb_z<float2, 1024>(m, r.nq, mode, in_lds, rho_lds, S, W, lds, s)
             : launch_tb_z<double2, 1024>(m, r.nq, mode, in_lds, rho_lds, S, W, lds, s);
}

const char *fill_choice_name(int c) {
  switch (c) {
    case kFillTB1024: return "triangle blocks of 64, 1024 threads (16 waves, two source triangles per wave and round)";
    case kFillTB512: return "triangle blocks of 64, 512 threads (8 waves, four source triangles per wave and round)";
    case kFillEB1024: return "edge blocks of 80 edges / 64 triangles, 1024 threads";
    default: return "unknown";
  }
}

int launch_fill(mf_mesh *m, const Rule &r, double k, int mode, const mf_tables *tab, void *Z,
                int z_dtype, int64_t ldz, hipStream_t s) {
  if ((mode == MF_MODE_TABLE || mode == MF_MODE_DIRECT) && m->tb_ok) {
    int c = m->fill_choice[mode];
    if (c < 0) c = cached_fill_choice(m, r.nq, mode, z_dtype, tab);
    if (c == kFillTB512) return launch_fill_tb(m, r, k, mode, tab, Z, z_dtype, ldz, s, 512);
    if (c != kFillEB1024) return launch_fill_tb(m, r, k, mode, tab, Z, z_dtype, ldz, s, 1024);
  }
  FillLaunch *L = nullptr;
  const float *sing = m->d_sing;
  int rc = fill_launch_create(1, &m, &k, &tab, r, mode, &Z, z_dtype, &ldz, &sing, nullptr, &L);
  if (rc) return rc;
  rc = fill_launch_run(L, s);
  fill_launch_destroy(L);
  return rc;
}

}  // namespace mf
