// Adjoint of the fill: gradient of L = Re sum_mn conj(W_mn) Z_mn with respect
// to the vertex coordinates and k.
//
// Regular triangle pairs (FP32, analytic).  Writing
//   Omega_ab = conj(W[e(p,a), e(q,b)]) s_a l_a s_b l_b      (zero off the tile)
// the pair's share of L is Re[c sum_ij w_i w_j g(R_ij) B_ij], c = j k eta/(4 pi),
//   B_ij = sum_ab Omega_ab [ (r_i - v_a).(r_j - v_b)/4 - 1/k^2 ]
//        = (O rho_i.rho'_j + rho_i.P + Qv.rho'_j + Gamma)/4 - O/k^2
// with O = sum Omega, P = sum Omega_ab beta_b, Qv = sum Omega_ab alpha_a,
// Gamma = sum Omega_ab alpha_a.beta_b.  Differentiating:
//   d/dr_i : w_i w_j [ g'(R) B (r_i - r_j)/R + g (O rho'_j + P)/4 ]   (and the
//            mirror for r_j), chained to the vertices through the barycentric
//            weights of the rule;
//   d/dv_a : -(c/4) [ Omega_a. Srho' + P_a S0 ]   (v_a = free vertex a of p);
//   d/dl_a : Re[c sum_b Omega_ab X_ab] / l_a, chained through l_a = |edge a|;
//   d/dk   : Re[(c/k) sum w w g B + c sum w w (dg/dk) B + c (2 O/k^3) S0],
//            dg/dk = -j exp(-jkR) = -j R g.
// Table mode treats the Green table as a fixed function of R: dg/dR is the
// derivative of the interval's cubic (Eq. (5)) and dg/dk is -j R times the
// interpolated g; direct mode differentiates exp(-jkR)/R.
//
// Tiles.  With a triangle-block plan (the table-mode fill's) a tile (I, J),
// I <= J, evaluates every triangle pair of its two blocks once; an
// off-diagonal tile stands for Z[I,J] and its mirror Z[J,I], so its weight is
// W[I,J] + W[J,I]^T, gathered from the full W over the blocks' edges (owned
// edges and non-owner halves alike: the adjoint needs no cut-edge fix-up).
// Meshes without that plan take the edge-block tiles, which repeat the
// triangle pairs their blocks share and skip the repeats' weights.
//
// Touching pairs (FP64): each unordered pair (p, q) carries the share
//   Re[c sum_ab Omega'_ab (X(p,q)[a][b] + X(q,p)[b][a]) / 2],
// Omega' from W[e(p,a), e(q,b)] + W[e(q,b), e(p,a)] (W alone for p = q),
// with X the singularity-cancelled blocks of the forward fill.  Its
// derivatives with respect to the coordinates of the pair's distinct vertices
// but one (at most 12) are carried through that FP64 evaluation in forward
// mode (dual.hpp), one tangent per thread; the first vertex and k follow from
// the share's translation invariance and homogeneity.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "dual.hpp"
#include "internal.hpp"
#include "lookup.hpp"
#include "singular.hpp"

namespace mf {

constexpr int kBwdThreads = 256;    // edge-block tiles
constexpr int kBwdBM = kMaxBlockEdges;
constexpr int kBwdTBThreads = 512;  // triangle-block tiles: 8 waves

struct BwdScalars {
  int ntiles;
  float k, ik2, pref;  // pref = k eta0 / (4 pi)
  float w[kMaxQ];
  float bary[kMaxQ][3];
  // Green table (cubic): one-sample bucket records (lookup.hpp) and the
  // interval coefficients, (c0, c1) then (c2, c3), gn intervals
  const int4 *gl;
  const float4 *g01, *g23;
  float ginv, gbias, gmax;
  int gn;
  long long ldz;
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Omega_ab = conj(W[row(a), col(b)]) sigma_a sigma_b from the tile's weights
// (row stride ldw), zero where the local edge is a boundary edge or lies
// outside the tile's blocks.
__device__ __forceinline__ void omega(const float2 *Wt, int ldw, int prow, int qcol, int a, int b,
                                      float sg, float &re, float &im) {
  const int row = (prow >> (8 * a)) & 0xff, col = (qcol >> (8 * b)) & 0xff;
  float2 w = make_float2(0.f, 0.f);
  if (row != 0xff && col != 0xff) w = Wt[row * ldw + col];
  re = w.x * sg;
  im = -w.y * sg;
}

// The adjoint of one regular pair (test p, source q): adds to p's vertex
// gradient Gv and edge-length derivatives Gl, to q's vertex gradient gq
// (9: vertex-major) and to the k derivative gk.
template <int Q, int MODE>
__device__ __forceinline__ void bwd_pair(const BwdScalars &S, const float *__restrict__ pr,
                                         const float (&pal)[3][3], const float (&psig)[3],
                                         const double *pcd, const float *__restrict__ qr,
                                         int prow, int qcol, const float2 *Wt, int ldw,
                                         const float4 *g01, const float4 *g23,
                                         float (&Gv)[3][3], float (&Gl)[3], float (&gq)[9],
                                         float &gk) {
  float beta[3][3], qsig[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
#pragma unroll
    for (int c = 0; c < 3; ++c) beta[b][c] = qr[kRecAlpha + 3 * b + c];
    qsig[b] = qr[kRecSigma + b];
  }
  // O = sum Omega, P = sum Omega_ab beta_b, Qv = sum Omega_ab alpha_a,
  // Gamma = sum Omega_ab alpha_a.beta_b
  float O_r = 0.f, O_i = 0.f, Gm_r = 0.f, Gm_i = 0.f;
  float P_r[3] = {0.f, 0.f, 0.f}, P_i[3] = {0.f, 0.f, 0.f};
  float Qv_r[3] = {0.f, 0.f, 0.f}, Qv_i[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      float wr, wi;
      omega(Wt, ldw, prow, qcol, a, b, psig[a] * qsig[b], wr, wi);
      O_r += wr;
      O_i += wi;
      const float ab = pal[a][0] * beta[b][0] + pal[a][1] * beta[b][1] + pal[a][2] * beta[b][2];
      Gm_r = fmaf(wr, ab, Gm_r);
      Gm_i = fmaf(wi, ab, Gm_i);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        P_r[c] = fmaf(wr, beta[b][c], P_r[c]);
        P_i[c] = fmaf(wi, beta[b][c], P_i[c]);
        Qv_r[c] = fmaf(wr, pal[a][c], Qv_r[c]);
        Qv_i[c] = fmaf(wi, pal[a][c], Qv_i[c]);
      }
    }
  const double *qcd = reinterpret_cast<const double *>(qr + kRecCent);
  const double Dx = pcd[0] - qcd[0], Dy = pcd[1] - qcd[1], Dz = pcd[2] - qcd[2];
  const float hx = (float)Dx, hy = (float)Dy, hz = (float)Dz;
  const float lx = (float)(Dx - (double)hx), ly = (float)(Dy - (double)hy),
              lz = (float)(Dz - (double)hz);
  // moments of w w g: S0, Srho.rho', Srho, Srho'
  float s0r = 0.f, s0i = 0.f, srr = 0.f, sri = 0.f;
  float spr[3] = {0.f, 0.f, 0.f}, spi[3] = {0.f, 0.f, 0.f};
  float sqr_[3] = {0.f, 0.f, 0.f}, sqi_[3] = {0.f, 0.f, 0.f};
  float kg_i = 0.f, ke_r = 0.f;  // Im sum w w g B, Re sum w w exp(-jkR) B
  // Only imaginary parts survive Re[c z] with c = j pref.
  float Fq[Q][3];
#pragma unroll
  for (int j = 0; j < Q; ++j) Fq[j][0] = Fq[j][1] = Fq[j][2] = 0.f;
#pragma unroll 1
  for (int i = 0; i < Q; ++i) {
    const float prho[3] = {pr[kRecRho + 3 * i], pr[kRecRho + 3 * i + 1], pr[kRecRho + 3 * i + 2]};
    const float ax = prho[0] + lx, ay = prho[1] + ly, az = prho[2] + lz;
    // the j sums of this test point: sum w w g (t0) and sum w w g rho'_j (t1);
    // sum hi (r_i - r_j) (Fp)
    float t0r = 0.f, t0i = 0.f, t1r[3] = {0.f, 0.f, 0.f}, t1i[3] = {0.f, 0.f, 0.f};
    float Fp[3] = {0.f, 0.f, 0.f};
    // B_ij pieces that do not depend on j
    const float bpr =
        0.25f * (P_r[0] * prho[0] + P_r[1] * prho[1] + P_r[2] * prho[2] + Gm_r) - S.ik2 * O_r;
    const float bpi =
        0.25f * (P_i[0] * prho[0] + P_i[1] * prho[1] + P_i[2] * prho[2] + Gm_i) - S.ik2 * O_i;
    float tq_r[3], tq_i[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      tq_r[c] = 0.25f * fmaf(O_r, prho[c], Qv_r[c]);
      tq_i[c] = 0.25f * fmaf(O_i, prho[c], Qv_i[c]);
    }
    // table mode: the bucket records of every source point are gathered
    // first, so that their latencies overlap
    float Rj[Q], rij[Q];
    int4 wj[Q];
    if (MODE == MF_MODE_TABLE) {
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const float d0 = hx + (ax - qr[kRecRho + 3 * j]), d1 = hy + (ay - qr[kRecRho + 3 * j + 1]),
                    d2 = hz + (az - qr[kRecRho + 3 * j + 2]);
        const float R2 = fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
        rij[j] = __builtin_amdgcn_rsqf(R2);
        Rj[j] = R2 * rij[j];
        wj[j] = look_record(S.gl, look_bucket(Rj[j], S.ginv, S.gbias, S.gmax));
      }
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const float rq0 = qr[kRecRho + 3 * j], rq1 = qr[kRecRho + 3 * j + 1],
                  rq2 = qr[kRecRho + 3 * j + 2];
      const float d0 = hx + (ax - rq0), d1 = hy + (ay - rq1), d2 = hz + (az - rq2);
      float ri, R;
      if (MODE == MF_MODE_TABLE) {
        ri = rij[j];
        R = Rj[j];
      } else {
        const float R2 = fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
        ri = __builtin_amdgcn_rsqf(R2);
        R = R2 * ri;
      }
      float gr, gi, dgr, dgi;  // g, dg/dR
      if (MODE == MF_MODE_TABLE) {
        float u;
        const int off = look_offset1(wj[j], R, u);
        const float4 A = at_offset(g01, off), B = at_offset(g23, off);
        // g = c0 + c1 u + c2 u^2 + c3 u^3, g' = c1 + 2 c2 u + 3 c3 u^2
        const float der = fmaf(3.0f * B.z, u, 2.0f * B.x);
        const float dei = fmaf(3.0f * B.w, u, 2.0f * B.y);
        dgr = fmaf(der, u, A.z);
        dgi = fmaf(dei, u, A.w);
        const float2 g = cubic(A, B, u);
        gr = g.x;
        gi = g.y;
      } else {
        float sn, cs;
        sincosf(S.k * R, &sn, &cs);
        gr = cs * ri;
        gi = -sn * ri;
        // dg/dR = -(jk + 1/R) g
        dgr = fmaf(S.k, gi, -ri * gr);
        dgi = fmaf(-S.k, gr, -ri * gi);
      }
      const float rr = prho[0] * rq0 + prho[1] * rq1 + prho[2] * rq2;
      const float qdot_r = Qv_r[0] * rq0 + Qv_r[1] * rq1 + Qv_r[2] * rq2;
      const float qdot_i = Qv_i[0] * rq0 + Qv_i[1] * rq1 + Qv_i[2] * rq2;
      const float Br = fmaf(0.25f, fmaf(O_r, rr, qdot_r), bpr);
      const float Bi = fmaf(0.25f, fmaf(O_i, rr, qdot_i), bpi);
      const float ww = S.w[i] * S.w[j];
      const float hi = (ww * ri) * (dgr * Bi + dgi * Br);  // Im(w w g' B / R)
      const float wgr = ww * gr, wgi = ww * gi;
      const float rq[3] = {rq0, rq1, rq2}, d[3] = {d0, d1, d2};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Fp[c] = fmaf(hi, d[c], Fp[c]);
        Fq[j][c] = fmaf(-hi, d[c], fmaf(wgr, tq_i[c], fmaf(wgi, tq_r[c], Fq[j][c])));
        t1r[c] = fmaf(wgr, rq[c], t1r[c]);
        t1i[c] = fmaf(wgi, rq[c], t1i[c]);
      }
      t0r += wgr;
      t0i += wgi;
      // exp(-jkR) = R g
      kg_i = fmaf(wgr, Bi, fmaf(wgi, Br, kg_i));
      ke_r = fmaf(R, fmaf(wgr, Br, -wgi * Bi), ke_r);
    }
    // the moments, and the j sums of w w g (O rho'_j + P)/4 in Fp
    s0r += t0r;
    s0i += t0i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      spr[c] = fmaf(t0r, prho[c], spr[c]);
      spi[c] = fmaf(t0i, prho[c], spi[c]);
      sqr_[c] += t1r[c];
      sqi_[c] += t1i[c];
      srr = fmaf(prho[c], t1r[c], srr);
      sri = fmaf(prho[c], t1i[c], sri);
      Fp[c] += 0.25f * (fmaf(O_i, t1r[c], P_i[c] * t0r) + fmaf(O_r, t1i[c], P_r[c] * t0i));
    }
    // Re[c z] = -pref Im z, chained to the vertices through r_i's weights
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int c = 0; c < 3; ++c) Gv[v][c] = fmaf(-S.pref * S.bary[i][v], Fp[c], Gv[v][c]);
  }
  // source points to q's vertices
#pragma unroll
  for (int j = 0; j < Q; ++j)
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int c = 0; c < 3; ++c) gq[3 * v + c] -= S.bary[j][v] * S.pref * Fq[j][c];
  // d/dk
  gk += -(S.pref / S.k) * kg_i + S.pref * ke_r -
        S.pref * 2.0f * S.ik2 / S.k * (O_r * s0i + O_i * s0r);
  // free-vertex and edge-length terms, Omega re-read from the tile
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      float wr, wi;
      omega(Wt, ldw, prow, qcol, a, b, psig[a] * qsig[b], wr, wi);
      const float ab = pal[a][0] * beta[b][0] + pal[a][1] * beta[b][1] + pal[a][2] * beta[b][2];
      // X_ab = (Srr + alpha_a.Srho' + beta_b.Srho + alpha_a.beta_b S0)/4 - S0/k^2
      float xr = fmaf(ab, s0r, srr), xi = fmaf(ab, s0i, sri);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        xr += pal[a][c] * sqr_[c] + beta[b][c] * spr[c];
        xi += pal[a][c] * sqi_[c] + beta[b][c] * spi[c];
        // d/dv_a: -(1/4) Omega_ab (Srho' + beta_b S0); d/dv_b: -(1/4) Omega_ab (Srho + alpha_a S0)
        const float ya = (wr * fmaf(beta[b][c], s0i, sqi_[c]) + wi * fmaf(beta[b][c], s0r, sqr_[c]));
        const float yb = (wr * fmaf(pal[a][c], s0i, spi[c]) + wi * fmaf(pal[a][c], s0r, spr[c]));
        Gv[a][c] = fmaf(0.25f * S.pref, ya, Gv[a][c]);
        gq[3 * b + c] = fmaf(0.25f * S.pref, yb, gq[3 * b + c]);
      }
      xr = fmaf(0.25f, xr, -S.ik2 * s0r);
      xi = fmaf(0.25f, xi, -S.ik2 * s0i);
      const float im = wr * xi + wi * xr;  // Im(Omega X)
      const float la = fabsf(psig[a]), lb = fabsf(qsig[b]);
      if (la > 0.f) Gl[a] -= S.pref * im / la;
      if (lb > 0.f) {
        // l_b = |x_{b+1} - x_{b+2}| and x_{b+1} - x_{b+2} = beta_{b+2} - beta_{b+1}
        const int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
        const float g = -S.pref * im / (lb * lb);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float e = beta[b2][c] - beta[b1][c];
          gq[3 * b1 + c] = fmaf(g, e, gq[3 * b1 + c]);
          gq[3 * b2 + c] = fmaf(-g, e, gq[3 * b2 + c]);
        }
      }
    }
}

// p's vertex gradient from Gv and the edge-length derivatives Gl
// (l_a = |x_{a+1} - x_{a+2}|, x_{a+1} - x_{a+2} = alpha_{a+2} - alpha_{a+1}).
__device__ __forceinline__ void p_gradient(const float (&pal)[3][3], const float (&psig)[3],
                                           const float (&Gv)[3][3], const float (&Gl)[3],
                                           float (&gpv)[9]) {
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int c = 0; c < 3; ++c) gpv[3 * v + c] = Gv[v][c];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float la = fabsf(psig[a]);
    if (la > 0.f) {
      const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float e = pal[a2][c] - pal[a1][c];
        gpv[3 * a1 + c] += Gl[a] * e / la;
        gpv[3 * a2 + c] -= Gl[a] * e / la;
      }
    }
  }
}

__device__ __forceinline__ bool touching(int pv0, int pv1, int pv2, const int *qvi) {
  return pv0 == qvi[0] || pv0 == qvi[1] || pv0 == qvi[2] || pv1 == qvi[0] || pv1 == qvi[1] ||
         pv1 == qvi[2] || pv2 == qvi[0] || pv2 == qvi[1] || pv2 == qvi[2];
}

template <int Q, int MODE, typename ZT>
__global__ __launch_bounds__(kBwdThreads) void k_bwd_regular(
    BwdScalars S, const float *__restrict__ rec, const int32_t *__restrict__ tiles,
    const int32_t *__restrict__ blk_e0, const int32_t *__restrict__ blk_off,
    const int32_t *__restrict__ blk_tri, const int32_t *__restrict__ blk_pos,
    const ZT *__restrict__ W, double *__restrict__ dV, double *__restrict__ dk) {
  __shared__ float2 Wt[kBwdBM * kBwdBM];
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  constexpr int kWaves = kBwdThreads / 64;
  float gk = 0.0f;

  for (int tile = blockIdx.x; tile < S.ntiles; tile += gridDim.x) {
    const int tij = tiles[tile];
    const int I = (int)((unsigned)tij >> 16), J = tij & 0xffff;
    const int i0 = blk_e0[I], ni = blk_e0[I + 1] - i0;
    const int j0 = blk_e0[J], nj = blk_e0[J + 1] - j0;
    __syncthreads();
    for (int e = threadIdx.x; e < ni * nj; e += kBwdThreads) {
      const int r = e / nj, c = e % nj;
      const ZT v = W[(size_t)(i0 + r) * S.ldz + (j0 + c)];
      Wt[r * kBwdBM + c] = make_float2((float)v.x, (float)v.y);
    }
    __syncthreads();
    if (I != J) {
      for (int e = threadIdx.x; e < ni * nj; e += kBwdThreads) {
        const int c = e / ni, r = e % ni;
        const ZT v = W[(size_t)(j0 + c) * S.ldz + (i0 + r)];
        float2 &t = Wt[r * kBwdBM + c];
        t.x += (float)v.x;
        t.y += (float)v.y;
      }
      __syncthreads();
    }
    const int p0 = blk_off[I], np = blk_off[I + 1] - p0;
    const int q0 = blk_off[J], nq = blk_off[J + 1] - q0;
    for (int pc = 0; pc < np; pc += 64) {
      const bool pv = pc + lane < np;
      const int pidx = pv ? pc + lane : pc;
      const int p = blk_tri[p0 + pidx];
      const int prow = pv ? blk_pos[p0 + pidx] : -1;
      const float *pr = rec + (size_t)p * kRecFloats;
      float pal[3][3], psig[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int c = 0; c < 3; ++c) pal[a][c] = pr[kRecAlpha + 3 * a + c];
        psig[a] = pr[kRecSigma + a];
      }
      const double *pcd = reinterpret_cast<const double *>(pr + kRecCent);
      const int *pvi = reinterpret_cast<const int *>(pr + kRecVid);
      const int pv0 = pvi[0], pv1 = pvi[1], pv2 = pvi[2];
      float Gv[3][3], Gl[3];  // gradient on p's vertices; d/dl_a
#pragma unroll
      for (int a = 0; a < 3; ++a) Gv[a][0] = Gv[a][1] = Gv[a][2] = Gl[a] = 0.f;

      for (int qi = wave; qi < nq; qi += kWaves) {
        const int q = uni(blk_tri[q0 + qi]);
        const int qcol = uni(blk_pos[q0 + qi]);
        const float *qr = rec + (size_t)q * kRecFloats;
        const int *qvi = reinterpret_cast<const int *>(qr + kRecVid);
        float gq[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // q vertex gradient
        if (!touching(pv0, pv1, pv2, qvi) && pv)
          bwd_pair<Q, MODE>(S, pr, pal, psig, pcd, qr, prow, qcol, Wt, kBwdBM, S.g01, S.g23, Gv,
                            Gl, gq, gk);
        // sum over lanes, one atomic per coordinate of q
#pragma unroll
        for (int c = 0; c < 9; ++c) {
          const float v = wave_sum(gq[c]);
          if (lane == 0 && v != 0.0f) atomicAdd(&dV[3 * (size_t)qvi[c / 3] + c % 3], (double)v);
        }
      }
      if (pv) {
        float gpv[9];
        p_gradient(pal, psig, Gv, Gl, gpv);
        const int vids[3] = {pv0, pv1, pv2};
#pragma unroll
        for (int c = 0; c < 9; ++c)
          if (gpv[c] != 0.0f) atomicAdd(&dV[3 * (size_t)vids[c / 3] + c % 3], (double)gpv[c]);
      }
    }
  }
  const float s = wave_sum(gk);
  if (lane == 0) atomicAdd(dk, (double)s);
}

// Triangle-block tiles.  Lane l of every wave takes test triangle l of block
// I (at most 64); the waves share out the source triangles of J.  The tile's
// weights Wt[r][c] (block edges of I by those of J, stride kTBEdges) come
// from W through each block edge's global edge: owned edges e0 + r, then the
// edges of the non-owner halves.  p's gradient is summed over the waves in
// LDS (in the weights' space, once the pairs are done) before its atomics;
// q's over the lanes of its wave.  With kLDS the Green table's coefficients
// follow the weights in LDS.
struct BwdTB {
  const int32_t *tiles, *t0, *e0, *nbe, *be_off, *be_cut, *pos, *cut_edge;
};
constexpr int kBwdTBWt = kTBEdges * kTBEdges;  // float2
// Green intervals whose coefficients fit in LDS beside the weights
constexpr int kBwdLdsCoef = (160 * 1024 - 8 * kBwdTBWt) / 32;

__device__ __forceinline__ int block_edge(const BwdTB &B, int blk, int e0, int nown, int r) {
  return r < nown ? e0 + r : B.cut_edge[B.be_cut[B.be_off[blk] + r - nown]];
}

template <int Q, int MODE, bool kLDS, typename ZT>
__global__ __launch_bounds__(kBwdTBThreads) void k_bwd_tb(BwdScalars S, BwdTB B,
                                                          const float *__restrict__ rec,
                                                          const ZT *__restrict__ W,
                                                          double *__restrict__ dV,
                                                          double *__restrict__ dk) {
  constexpr int kWaves = kBwdTBThreads / 64;
  extern __shared__ float4 bsm4[];
  float2 *Wt = reinterpret_cast<float2 *>(bsm4);
  float *red = reinterpret_cast<float *>(bsm4);  // [9][kWaves][64], over Wt after the pairs
  const float4 *g01 = S.g01, *g23 = S.g23;
  if (kLDS) {
    float4 *c = bsm4 + kBwdTBWt / 2;
    for (int i = threadIdx.x; i < 2 * S.gn; i += kBwdTBThreads) c[i] = S.g01[i];
    g01 = c;
    g23 = c + S.gn;
  }
  const int lane = threadIdx.x & 63;
  const int wave = uni(threadIdx.x >> 6);
  float gk = 0.0f;
  for (int tile = blockIdx.x; tile < S.ntiles; tile += gridDim.x) {
    const int tij = B.tiles[tile];
    const int I = (int)((unsigned)tij >> 16), J = tij & 0xffff;
    const int e0I = B.e0[I], nownI = B.e0[I + 1] - e0I, nbeI = B.nbe[I];
    const int e0J = B.e0[J], nownJ = B.e0[J + 1] - e0J, nbeJ = B.nbe[J];
    __syncthreads();
    // W[I,J] along rows of W, then W[J,I]^T along rows of W
    for (int e = threadIdx.x; e < nbeI * nbeJ; e += kBwdTBThreads) {
      const int r = e / nbeJ, c = e % nbeJ;
      const int m = block_edge(B, I, e0I, nownI, r), n = block_edge(B, J, e0J, nownJ, c);
      const ZT v = W[(size_t)m * S.ldz + n];
      Wt[r * kTBEdges + c] = make_float2((float)v.x, (float)v.y);
    }
    __syncthreads();
    if (I != J) {
      for (int e = threadIdx.x; e < nbeI * nbeJ; e += kBwdTBThreads) {
        const int c = e / nbeI, r = e % nbeI;
        const int m = block_edge(B, I, e0I, nownI, r), n = block_edge(B, J, e0J, nownJ, c);
        const ZT v = W[(size_t)n * S.ldz + m];
        float2 &t = Wt[r * kTBEdges + c];
        t.x += (float)v.x;
        t.y += (float)v.y;
      }
      __syncthreads();
    }
    const int tI0 = B.t0[I], npI = B.t0[I + 1] - tI0;
    const int tJ0 = B.t0[J], npJ = B.t0[J + 1] - tJ0;
    const bool pv = lane < npI;
    const int p = tI0 + (pv ? lane : 0);
    const int prow = pv ? B.pos[p] : -1;
    const float *pr = rec + (size_t)p * kRecFloats;
    float pal[3][3], psig[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int c = 0; c < 3; ++c) pal[a][c] = pr[kRecAlpha + 3 * a + c];
      psig[a] = pr[kRecSigma + a];
    }
    const double *pcd = reinterpret_cast<const double *>(pr + kRecCent);
    const int *pvi = reinterpret_cast<const int *>(pr + kRecVid);
    const int pv0 = pvi[0], pv1 = pvi[1], pv2 = pvi[2];
    float Gv[3][3], Gl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) Gv[a][0] = Gv[a][1] = Gv[a][2] = Gl[a] = 0.f;
    for (int j = wave; j < npJ; j += kWaves) {
      const int q = tJ0 + j;
      const int qcol = uni(B.pos[q]);
      const float *qr = rec + (size_t)q * kRecFloats;
      const int *qvi = reinterpret_cast<const int *>(qr + kRecVid);
      float gq[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (pv && !touching(pv0, pv1, pv2, qvi))
        bwd_pair<Q, MODE>(S, pr, pal, psig, pcd, qr, prow, qcol, Wt, kTBEdges, g01, g23, Gv,
                          Gl, gq, gk);
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const float v = wave_sum(gq[c]);
        if (lane == 0 && v != 0.0f) atomicAdd(&dV[3 * (size_t)qvi[c / 3] + c % 3], (double)v);
      }
    }
    float gpv[9];
    p_gradient(pal, psig, Gv, Gl, gpv);
    __syncthreads();  // every wave is done with Wt
#pragma unroll
    for (int c = 0; c < 9; ++c) red[(c * kWaves + wave) * 64 + lane] = pv ? gpv[c] : 0.0f;
    __syncthreads();
    for (int e = threadIdx.x; e < 9 * 64; e += kBwdTBThreads) {
      const int c = e / 64, l = e % 64;
      if (l >= npI) continue;
      float v = 0.0f;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) v += red[(c * kWaves + w) * 64 + l];
      const int *vi = reinterpret_cast<const int *>(rec + (size_t)(tI0 + l) * kRecFloats + kRecVid);
      if (v != 0.0f) atomicAdd(&dV[3 * (size_t)vi[c / 3] + c % 3], (double)v);
    }
  }
  const float s = wave_sum(gk);
  if (lane == 0) atomicAdd(dk, (double)s);
}

// ---- touching pairs -------------------------------------------------------

// Share of L carried by the unordered touching pair (p,q), from the weights
// Wr + j Wi (already W + W^T for p != q) of its local edge pairs:
//   Re[c sum_ab conj(W_ab) s_a s_b l_a l_b (X(p,q)[a][b] + X(q,p)[b][a]) / 2],
// contracted term by term so no 3x3 block is held.
template <class T>
__device__ T touching_share(const T xp[3][3], const T xq[3][3], const RuleArg &R, T k,
                            const double (&Wr)[9], const double (&Wi)[9],
                            const signed char *sp, const signed char *sq) {
  T Or[9], Oi[9];  // conj(W_ab) s_a s_b l_a l_b
  for (int a = 0; a < 3; ++a) {
    const T *u = xp[(a + 1) % 3], *v = xp[(a + 2) % 3];
    const T la = d_sqrt((u[0] - v[0]) * (u[0] - v[0]) + (u[1] - v[1]) * (u[1] - v[1]) +
                        (u[2] - v[2]) * (u[2] - v[2]));
    for (int b = 0; b < 3; ++b) {
      const T *s = xq[(b + 1) % 3], *t = xq[(b + 2) % 3];
      const T lb = d_sqrt((s[0] - t[0]) * (s[0] - t[0]) + (s[1] - t[1]) * (s[1] - t[1]) +
                          (s[2] - t[2]) * (s[2] - t[2]));
      const T f = ((double)sp[a] * (double)sq[b]) * (la * lb);
      Or[3 * a + b] = f * Wr[3 * a + b];
      Oi[3 * a + b] = f * (-Wi[3 * a + b]);
    }
  }
  // only the imaginary part of the contraction enters Re[j c (sr + j si)]
  T s1i = 0.0, s2i = 0.0;
  const T A1 = oneway_terms(xp, xq, R, k, 0, [&](int a, int b, const T &re, const T &im) {
    s1i += Or[3 * a + b] * im + Oi[3 * a + b] * re;
  });
  const T A2 = oneway_terms(xq, xp, R, k, 0, [&](int b, int a, const T &re, const T &im) {
    s2i += Or[3 * a + b] * im + Oi[3 * a + b] * re;
  });
  const T si = 0.5 * (s1i / A1 + s2i / A2);
  // Re[j k eta/(4 pi) (sr + j si)]
  return (-kEta0 / (4.0 * M_PI)) * (k * si);
}

// Thread (pair u, group g) carries tangents g*N .. g*N + N - 1 of the pair's
// list: x, y, z of its distinct vertices after the first (p's second and
// third, then q's others).  The rest follows from two invariances of the
// share: it does not change when the pair is translated, so the first
// vertex's gradient is minus the sum of the others'; and it is homogeneous,
// share(a V, k / a) = a^2 share(V, k), so
//   k d/dk = sum_v x_v . d/dx_v - 2 share = sum_{v > 0} (x_v - x_0) . d/dx_v - 2 share.
constexpr int kTouchTangents = 12;  // at most 4 vertices besides the first
constexpr int kTouchN = 1;
constexpr int kTouchGroups = (kTouchTangents + kTouchN - 1) / kTouchN;

template <typename ZT>
__global__ __launch_bounds__(256) void k_bwd_touching(
    const double *__restrict__ V, const int32_t *__restrict__ tri,
    const int32_t *__restrict__ tp, const int32_t *__restrict__ tq,
    const int32_t *__restrict__ tu, const int32_t *__restrict__ tedge,
    const signed char *__restrict__ tsign, int64_t nu, RuleArg R, double k,
    const ZT *__restrict__ W, long long ldz, double *__restrict__ dV, double *__restrict__ dk) {
  using T = Dual<kTouchN>;
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nu * kTouchGroups) return;
  const int64_t u = s / kTouchGroups;
  const int g = (int)(s % kTouchGroups);
  const int pair = tu[u];
  const int p = tp[pair], q = tq[pair];
  int vp[3], vq[3], dv[5];
  signed char sp[3], sq[3];
  double Wr[9], Wi[9];
  for (int a = 0; a < 3; ++a) {
    vp[a] = tri[3 * p + a];
    vq[a] = tri[3 * q + a];
    sp[a] = tsign[3 * p + a];
    sq[a] = tsign[3 * q + a];
  }
  int nd = 3;
  for (int a = 0; a < 3; ++a) {
    dv[a] = vp[a];
    if (vq[a] != vp[0] && vq[a] != vp[1] && vq[a] != vp[2]) dv[nd++] = vq[a];
  }
  const int ntan = 3 * (nd - 1), t0 = g * kTouchN;
  if (t0 >= ntan) return;
  for (int a = 0; a < 3; ++a) {
    const int ea = tedge[3 * p + a];
    for (int b = 0; b < 3; ++b) {
      const int eb = tedge[3 * q + b];
      double wr = 0.0, wi = 0.0;
      if (ea >= 0 && eb >= 0) {
        const ZT w = W[(size_t)ea * ldz + eb];
        wr = (double)w.x;
        wi = (double)w.y;
        if (p != q) {
          const ZT w2 = W[(size_t)eb * ldz + ea];
          wr += (double)w2.x;
          wi += (double)w2.y;
        }
      }
      Wr[3 * a + b] = wr;
      Wi[3 * a + b] = wi;
    }
  }
  // seed: tangent t moves coordinate t % 3 of distinct vertex 1 + t / 3
  T xp[3][3], xq[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      xp[a][c] = T(V[3 * (size_t)vp[a] + c]);
      xq[a][c] = T(V[3 * (size_t)vq[a] + c]);
      for (int j = 0; j < kTouchN; ++j) {
        const int t = t0 + j;
        const bool on = t < ntan && t % 3 == c;
        xp[a][c].d[j] = on && dv[1 + t / 3] == vp[a] ? 1.0 : 0.0;
        xq[a][c].d[j] = on && dv[1 + t / 3] == vq[a] ? 1.0 : 0.0;
      }
    }
  const T share = touching_share(xp, xq, R, T(k), Wr, Wi, sp, sq);
  double gk = g == 0 ? -2.0 * share.v : 0.0;
  for (int j = 0; j < kTouchN; ++j) {
    const int t = t0 + j;
    if (t >= ntan) break;
    const int v = dv[1 + t / 3], c = t % 3;
    const double d = share.d[j];
    atomicAdd(&dV[3 * (size_t)v + c], d);
    atomicAdd(&dV[3 * (size_t)dv[0] + c], -d);
    gk += (V[3 * (size_t)v + c] - V[3 * (size_t)dv[0] + c]) * d;
  }
  atomicAdd(dk, gk / k);
}

__global__ void k_zero(double *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

static int grid_for(const void *kern, int threads, size_t lds, int ntiles, long long *grid) {
  int dev = 0, ncu = 0, per = 0;
  MF_HIP(hipGetDevice(&dev));
  MF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  MF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, threads, lds));
  if (per < 1) per = 1;
  *grid = std::min<long long>((long long)ncu * per, std::max(ntiles, 1));
  return MF_OK;
}

template <int Q, int MODE, bool kLDS, typename ZT>
static int launch_bwd_tb(mf_mesh *m, BwdScalars S, const ZT *W, double *dV, double *dk,
                         hipStream_t s) {
  long long grid = 0;
  int rc;
  {
    auto kern = k_bwd_tb<Q, MODE, kLDS, ZT>;
    static_assert(sizeof(float) * 9 * kBwdTBThreads <= sizeof(float2) * kBwdTBWt,
                  "the wave reduction lives in the weights' space");
    const size_t lds_max =
        sizeof(float2) * kBwdTBWt + (kLDS ? sizeof(float4) * 2 * kBwdLdsCoef : 0);
    const size_t lds = sizeof(float2) * kBwdTBWt + (kLDS ? sizeof(float4) * 2 * S.gn : 0);
    static std::once_flag once;  // per instantiation
    static hipError_t ge = hipSuccess;
    std::call_once(once, [&]() {
      ge = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_max);
    });
    if (ge != hipSuccess) return hip_fail(ge, "adjoint set-up");
    S.ntiles = (int)m->tb_tiles.size();
    if ((rc = grid_for(reinterpret_cast<const void *>(kern), kBwdTBThreads, lds, S.ntiles, &grid)))
      return rc;
    BwdTB B{m->d_tb_tiles, m->d_tb_t0,  m->d_tb_e0,  m->d_tb_nbe,
            m->d_tb_be_off, m->d_tb_be_cut, m->d_tb_pos, m->d_cut_edge};
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kBwdTBThreads), lds, s, S, B, m->d_rec, W,
                       dV, dk);
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <int Q, int MODE, typename ZT>
static int launch_bwd_t(mf_mesh *m, BwdScalars S, const ZT *W, double *dV, double *dk,
                        hipStream_t s) {
  long long grid = 0;
  int rc;
  if (m->tb_ok) {
    if (MODE == MF_MODE_TABLE && S.gn <= kBwdLdsCoef)
      return launch_bwd_tb<Q, MODE, true, ZT>(m, S, W, dV, dk, s);
    return launch_bwd_tb<Q, MODE, false, ZT>(m, S, W, dV, dk, s);
  } else {
    auto kern = k_bwd_regular<Q, MODE, ZT>;
    S.ntiles = (int)m->tiles.size();
    if ((rc = grid_for(reinterpret_cast<const void *>(kern), kBwdThreads, 0, S.ntiles, &grid)))
      return rc;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kBwdThreads), 0, s, S, m->d_rec,
                       m->d_tiles, m->d_blk_e0, m->d_blk_off, m->d_blk_tri, m->d_blk_pos, W, dV,
                       dk);
  }
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <typename ZT>
static int launch_bwd_z(mf_mesh *m, const Rule &r, int mode, const BwdScalars &S, const void *W,
                        double *dV, double *dk, hipStream_t s) {
  const ZT *w = reinterpret_cast<const ZT *>(W);
  if (mode == MF_MODE_TABLE)
    return r.nq == 3   ? launch_bwd_t<3, MF_MODE_TABLE, ZT>(m, S, w, dV, dk, s)
           : r.nq == 6 ? launch_bwd_t<6, MF_MODE_TABLE, ZT>(m, S, w, dV, dk, s)
                       : launch_bwd_t<7, MF_MODE_TABLE, ZT>(m, S, w, dV, dk, s);
  return r.nq == 3   ? launch_bwd_t<3, MF_MODE_DIRECT, ZT>(m, S, w, dV, dk, s)
         : r.nq == 6 ? launch_bwd_t<6, MF_MODE_DIRECT, ZT>(m, S, w, dV, dk, s)
                     : launch_bwd_t<7, MF_MODE_DIRECT, ZT>(m, S, w, dV, dk, s);
}

template <typename ZT>
static int launch_bwd_touch(mf_mesh *m, const double *V, const Rule &r, double k, const void *W,
                            int64_t ldz, double *dV, double *dk, hipStream_t s) {
  const int64_t nu = (int64_t)m->touch_u.size();
  if (nu == 0) return MF_OK;
  RuleArg R = rule_arg(r);
  const int64_t nthreads = nu * kTouchGroups;
  hipLaunchKernelGGL(k_bwd_touching<ZT>, dim3((unsigned)((nthreads + 255) / 256)), dim3(256), 0,
                     s, V, m->d_tri, m->d_touch_p, m->d_touch_q, m->d_touch_u, m->d_tedge,
                     reinterpret_cast<const signed char *>(m->d_tsign), nu, R, k,
                     reinterpret_cast<const ZT *>(W), (long long)ldz, dV, dk);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int launch_backward(mf_mesh *m, const double *V, const Rule &r, double k, int mode,
                    const mf_tables *tab, const void *W, int z_dtype, int64_t ldz, double *dV,
                    double *dk, hipStream_t s) {
  const int64_t nvc = 3 * (int64_t)m->nv;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((nvc + 255) / 256)), dim3(256), 0, s, dV, nvc);
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, s, dk, (int64_t)1);
  MF_HIP(hipGetLastError());
  BwdScalars S{};
  S.k = (float)k;
  S.ik2 = (float)(1.0 / (k * k));
  S.pref = (float)(k * kEta0 / (4.0 * M_PI));
  for (int i = 0; i < kMaxQ; ++i) {
    S.w[i] = i < r.nq ? (float)r.w[i] : 0.0f;
    for (int c = 0; c < 3; ++c) S.bary[i][c] = i < r.nq ? (float)r.bary[i][c] : 0.0f;
  }
  S.ldz = ldz;
  if (mode == MF_MODE_TABLE) {
    const mf_tables::One &g = tab->g;
    S.gl = g.look1;
    S.g01 = g.coef;
    S.g23 = g.coef + (g.n - 1);
    S.ginv = g.binv1;
    S.gbias = g.bbias1;
    S.gmax = g.btop1;
    S.gn = g.n - 1;
  }
  int rc = z_dtype == MF_C64 ? launch_bwd_z<float2>(m, r, mode, S, W, dV, dk, s)
                             : launch_bwd_z<double2>(m, r, mode, S, W, dV, dk, s);
  if (rc) return rc;
  return z_dtype == MF_C64 ? launch_bwd_touch<float2>(m, V, r, k, W, ldz, dV, dk, s)
                           : launch_bwd_touch<double2>(m, V, r, k, W, ldz, dV, dk, s);
}

}  // namespace mf
