// EFIE fill with every inner integral taken by the angular transformation
// (Section II-A: the singular-cancellation-plus-angular-transformation scheme
// whose inner surface integral becomes n points on each of the three source
// edges, 3mn Exp(-jkr) evaluations per source triangle and m outer points).
// FP64 throughout the integrals: for distant pairs both edge sums below
// cancel to a small remainder, which FP32 would not resolve.
//
// Test point r, source triangle q (unit normal n, r = rho0 + h n), edge i
// from x_i to x_{i+1} with unit tangent t_i, outward in-plane normal m_i =
// t_i x n, signed distance p_i = m_i.(x_i - rho0) (positive on the
// triangle's side), l along the edge from the foot of the perpendicular,
// R^2 = d^2 + l^2, d^2 = p_i^2 + h^2:
//   I0 = int_q exp(-jkR)/R dS'
//      = (1/jk) sum_i p_i int_edge [exp(-jk|h|) - exp(-jkR)] dl/(p_i^2 + l^2)
//     (polar coordinates about rho0, the radial integral exact since
//      R dR = rho drho, each edge seen under dphi = |p_i| dl/(p_i^2 + l^2));
//   I1 = int_q (r' - rho0) exp(-jkR)/R dS' = (j/k) sum_i m_i int_edge exp(-jkR) dl
//     ((r' - rho0) exp(-jkR)/R is (j/k) times the in-plane gradient of exp(-jkR)).
// Both edge integrals use the same n Gauss-Legendre points in u, l = d sinh u,
// R = d cosh u, dl = R du, one Exp(-jkR) per point: read from the linear Exp
// table through the hash of Eq. (6) (table mode) or computed (direct mode).
//
// Per test point, J = I1 + (rho0 - c_q) I0 and four moments over the test
// points (rho_i = r_i - c_p, alpha_a = c_p - v_a, beta_b = c_q - v_b):
//   S0 = sum w I0, SJ = sum w J, SrJ = sum w rho_i.J, Sr0 = sum w rho_i I0,
//   X_ab = [ (alpha_a.SJ + SrJ + (alpha_a.beta_b) S0 + beta_b.Sr0)/4 - S0/k^2 ] / A_q,
// the same normalisation as the regular-pair kernel, Z = j k eta0/(4 pi) sum
// s s' l l X.  The scheme is not symmetric in the two triangles, so every
// ordered tile is accumulated.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "internal.hpp"

namespace mf {

constexpr int kAngThreads = 256;
constexpr int kAngAccStride = 2 * kMaxBlockEdges + 1;
constexpr int kAngAccFloats = kMaxBlockEdges * kAngAccStride;

struct AngArgs {
  const double *V, *qp64, *brad;
  const int32_t *tri;
  const float *rec;
  const int32_t *tiles, *blk_e0, *blk_off, *blk_tri, *blk_pos;
  int ntiles, nq;
  long long ldz;
  double w[kMaxQ];
  double k, ik2, pref;
  // Exp table (FP64 bucket records, see mf_tables) and its range [0, rmax]
  const double *elook;
  int em;
  double einv, ermax;
  void *Z;
  int *status;
};

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// exp(-jkR): the linear table of Eq. (4), one 64-byte bucket record per
// lookup (the bucket of a coarsened Eq. (6) hash holds both candidate
// intervals and the sample between them), or sincos.  A table distance
// beyond r_max (by more than rounding) raises the status flag.
template <int MODE>
__device__ __forceinline__ void exp_jkr(const AngArgs &A, double R, double &re, double &im,
                                        bool &bad) {
  if (MODE == MF_MODE_DIRECT) {
    double s, c;
    sincos(A.k * R, &s, &c);
    re = c;
    im = -s;
    return;
  }
  bad |= !(R <= A.ermax * (1.0 + 1e-12));
  int b = (int)(R * A.einv);
  b = b < 0 ? 0 : (b > A.em - 1 ? A.em - 1 : b);
  const double2 *o = reinterpret_cast<const double2 *>(A.elook + 8 * (size_t)b);
  const double2 h = o[0], lv = o[1], rv = o[2];
  const float4 sl = *reinterpret_cast<const float4 *>(o + 3);
  const bool right = R >= h.x;
  const double u = R - h.y;
  re = fma((double)(right ? sl.z : sl.x), u, right ? rv.x : lv.x);
  im = fma((double)(right ? sl.w : sl.y), u, right ? rv.y : lv.y);
}

// Gauss-Legendre nodes and weights on [0, 1] by Newton iteration on P_n,
// one node per call.
__device__ inline void gauss_node(int n, int i, double &x, double &w) {
  double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
  for (int it = 0; it < 100; ++it) {
    double a = 1.0, b = z;
    for (int j = 2; j <= n; ++j) {
      const double c = ((2.0 * j - 1.0) * z * b - (j - 1.0) * a) / j;
      a = b;
      b = c;
    }
    dp = n * (z * b - a) / (z * z - 1.0);
    const double step = b / dp;
    z -= step;
    if (fabs(step) < 1e-16) break;
  }
  double a = 1.0, b = z;
  for (int j = 2; j <= n; ++j) {
    const double c = ((2.0 * j - 1.0) * z * b - (j - 1.0) * a) / j;
    a = b;
    b = c;
  }
  dp = n * (z * b - a) / (z * z - 1.0);
  x = 0.5 * (1.0 - z);
  w = 1.0 / ((1.0 - z * z) * dp * dp);
}

// One point of an edge: both edge integrands at u = u0 + du x.
template <int MODE>
__device__ __forceinline__ void edge_point(const AngArgs &A, double u0, double du, double gx,
                                           double gw, double d, double p, double ehr, double ehi,
                                           double &s0r, double &s0i, double &s1r, double &s1i,
                                           bool &bad) {
  const double ex = exp(u0 + du * gx), exi = 1.0 / ex;
  const double R = 0.5 * d * (ex + exi), l = 0.5 * d * (ex - exi);
  double er, ei;
  exp_jkr<MODE>(A, R, er, ei, bad);
  const double g = gw * du * R;
  const double g0 = g / (p * p + l * l);
  s0r += g0 * (ehr - er);
  s0i += g0 * (ehi - ei);
  s1r += g * er;
  s1i += g * ei;
}

template <int MODE, int NE>
__device__ void inner_integrals(const AngArgs &A, const double *gxs, const double *gws,
                                const double (&x)[3][3], const double *nrm,
                                const double *r, double &i0r, double &i0i, double (&i1r)[3],
                                double (&i1i)[3], double (&rho0)[3], bool &bad) {
  const double h = nrm[0] * (r[0] - x[0][0]) + nrm[1] * (r[1] - x[0][1]) + nrm[2] * (r[2] - x[0][2]);
  for (int c = 0; c < 3; ++c) rho0[c] = r[c] - h * nrm[c];
  double ehr, ehi;
  exp_jkr<MODE>(A, fabs(h), ehr, ehi, bad);
  double a0r = 0.0, a0i = 0.0, a1r[3] = {0.0, 0.0, 0.0}, a1i[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
  for (int e = 0; e < 3; ++e) {
    const double *xa = x[e], *xb = x[(e + 1) % 3];
    double t[3] = {xb[0] - xa[0], xb[1] - xa[1], xb[2] - xa[2]};
    const double len = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    for (int c = 0; c < 3; ++c) t[c] /= len;
    const double m[3] = {t[1] * nrm[2] - t[2] * nrm[1], t[2] * nrm[0] - t[0] * nrm[2],
                         t[0] * nrm[1] - t[1] * nrm[0]};
    const double da[3] = {xa[0] - rho0[0], xa[1] - rho0[1], xa[2] - rho0[2]};
    const double p = m[0] * da[0] + m[1] * da[1] + m[2] * da[2];
    const double lm = t[0] * da[0] + t[1] * da[1] + t[2] * da[2];
    const double lp = lm + len;
    const double d = sqrt(p * p + h * h);
    double s0r = 0.0, s0i = 0.0, s1r = 0.0, s1i = 0.0;
    if (d > 0.0) {
      const double u0 = asinh(lm / d), du = asinh(lp / d) - u0;
      if (MODE == MF_MODE_TABLE) {
        // pairs of points: two table reads in flight
#pragma unroll 2
        for (int j = 0; j < NE; ++j)
          edge_point<MODE>(A, u0, du, gxs[j], gws[j], d, p, ehr, ehi, s0r, s0i, s1r, s1i, bad);
      } else {
#pragma unroll 1
        for (int j = 0; j < NE; ++j)
          edge_point<MODE>(A, u0, du, gxs[j], gws[j], d, p, ehr, ehi, s0r, s0i, s1r, s1i, bad);
      }
    } else {  // r on the edge's line: no angle, the line integral in l
#pragma unroll 1
      for (int j = 0; j < NE; ++j) {
        const double l = lm + len * gxs[j];
        double er, ei;
        exp_jkr<MODE>(A, fabs(l), er, ei, bad);
        s1r += gws[j] * len * er;
        s1i += gws[j] * len * ei;
      }
    }
    a0r += p * s0r;
    a0i += p * s0i;
    for (int c = 0; c < 3; ++c) {
      a1r[c] += m[c] * s1r;
      a1i[c] += m[c] * s1i;
    }
  }
  // I0 = a0/(jk), I1 = (j/k) a1
  const double ik = 1.0 / A.k;
  i0r = a0i * ik;
  i0i = -a0r * ik;
  for (int c = 0; c < 3; ++c) {
    i1r[c] = -a1i[c] * ik;
    i1i[c] = a1r[c] * ik;
  }
}

template <int MODE, typename ZT, int NE>
__global__ __launch_bounds__(kAngThreads) void k_fill_angular(AngArgs A) {
  constexpr int kWaves = kAngThreads / 64;
  extern __shared__ float acc[];
  __shared__ double gxs[NE], gws[NE];
  if (threadIdx.x < NE) gauss_node(NE, threadIdx.x, gxs[threadIdx.x], gws[threadIdx.x]);
  const int lane = threadIdx.x & 63;
  const int wave = uniform_i(threadIdx.x >> 6);
  bool bad = false;
  ZT *Z = reinterpret_cast<ZT *>(A.Z);
  for (int tl = blockIdx.x; tl < A.ntiles; tl += gridDim.x) {
    const int tij = A.tiles[tl];
    const int I0 = (int)((unsigned)tij >> 16), J0 = tij & 0xffff;
    for (int dir = 0; dir < (I0 != J0 ? 2 : 1); ++dir) {
      const int I = dir ? J0 : I0, J = dir ? I0 : J0;
      for (int i = threadIdx.x; i < kAngAccFloats; i += kAngThreads) acc[i] = 0.0f;
      __syncthreads();
      const int p0 = A.blk_off[I], np = A.blk_off[I + 1] - p0;
      const int q0 = A.blk_off[J], nqt = A.blk_off[J + 1] - q0;
      for (int pc = 0; pc < np; pc += 64) {
        const bool pv = pc + lane < np;
        const int pidx = pv ? pc + lane : pc;
        const int p = A.blk_tri[p0 + pidx];
        const int prow = pv ? A.blk_pos[p0 + pidx] : -1;
        const float *pr = A.rec + (size_t)p * kRecFloats;
        const double *pcd = reinterpret_cast<const double *>(pr + kRecCent);
        const double cp[3] = {pcd[0], pcd[1], pcd[2]};
        for (int qi = wave; qi < nqt; qi += kWaves) {
          const int q = uniform_i(A.blk_tri[q0 + qi]);
          const int qcol = uniform_i(A.blk_pos[q0 + qi]);
          const float *qr = A.rec + (size_t)q * kRecFloats;
          const double *qcd = reinterpret_cast<const double *>(qr + kRecCent);
          const double cq[3] = {qcd[0], qcd[1], qcd[2]};
          double x[3][3];
          for (int a = 0; a < 3; ++a) {
            const int v = A.tri[3 * q + a];
            for (int c = 0; c < 3; ++c) x[a][c] = A.V[3 * (size_t)v + c];
          }
          const double nrm[3] = {A.brad[4 * q + 1], A.brad[4 * q + 2], A.brad[4 * q + 3]};
          const double e1[3] = {x[1][0] - x[0][0], x[1][1] - x[0][1], x[1][2] - x[0][2]};
          const double e2[3] = {x[2][0] - x[0][0], x[2][1] - x[0][1], x[2][2] - x[0][2]};
          const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                                e1[0] * e2[1] - e1[1] * e2[0]};
          const double iAq = 2.0 / sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
          double s0r = 0.0, s0i = 0.0, srjr = 0.0, srji = 0.0;
          double sjr[3] = {0.0, 0.0, 0.0}, sji[3] = {0.0, 0.0, 0.0};
          double s0pr[3] = {0.0, 0.0, 0.0}, s0pi[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
          for (int i = 0; i < A.nq; ++i) {
            const double *ri = A.qp64 + ((size_t)p * kMaxQ + i) * 3;
            const double r[3] = {ri[0], ri[1], ri[2]};
            double i0r, i0i, i1r[3], i1i[3], rho0[3];
            inner_integrals<MODE, NE>(A, gxs, gws, x, nrm, r, i0r, i0i, i1r, i1i, rho0, bad);
            const double w = A.w[i];
            double jr[3], ji[3], rh[3];
            for (int c = 0; c < 3; ++c) {
              jr[c] = i1r[c] + (rho0[c] - cq[c]) * i0r;
              ji[c] = i1i[c] + (rho0[c] - cq[c]) * i0i;
              rh[c] = r[c] - cp[c];
            }
            s0r += w * i0r;
            s0i += w * i0i;
            for (int c = 0; c < 3; ++c) {
              sjr[c] += w * jr[c];
              sji[c] += w * ji[c];
              s0pr[c] += w * rh[c] * i0r;
              s0pi[c] += w * rh[c] * i0i;
            }
            srjr += w * (rh[0] * jr[0] + rh[1] * jr[1] + rh[2] * jr[2]);
            srji += w * (rh[0] * ji[0] + rh[1] * ji[1] + rh[2] * ji[2]);
          }
          if (pv) {
            for (int a = 0; a < 3; ++a) {
              const int row = (prow >> (8 * a)) & 0xff;
              if (row == 0xff) continue;
              const int va = A.tri[3 * p + a];
              double alpha[3];
              for (int c = 0; c < 3; ++c) alpha[c] = cp[c] - A.V[3 * (size_t)va + c];
              const double ajr = alpha[0] * sjr[0] + alpha[1] * sjr[1] + alpha[2] * sjr[2];
              const double aji = alpha[0] * sji[0] + alpha[1] * sji[1] + alpha[2] * sji[2];
              for (int b = 0; b < 3; ++b) {
                const int col = (qcol >> (8 * b)) & 0xff;
                if (col == 0xff) continue;
                const double beta[3] = {cq[0] - x[b][0], cq[1] - x[b][1], cq[2] - x[b][2]};
                const double ab = alpha[0] * beta[0] + alpha[1] * beta[1] + alpha[2] * beta[2];
                const double bsr = beta[0] * s0pr[0] + beta[1] * s0pr[1] + beta[2] * s0pr[2];
                const double bsi = beta[0] * s0pi[0] + beta[1] * s0pi[1] + beta[2] * s0pi[2];
                const double xr = (0.25 * (ajr + srjr + ab * s0r + bsr) - A.ik2 * s0r) * iAq;
                const double xi = (0.25 * (aji + srji + ab * s0i + bsi) - A.ik2 * s0i) * iAq;
                const float sg = pr[kRecSigma + a] * qr[kRecSigma + b];
                float *dst = acc + row * kAngAccStride + 2 * col;
                atomicAdd(dst, sg * (float)xr);
                atomicAdd(dst + 1, sg * (float)xi);
              }
            }
          }
        }
      }
      __syncthreads();
      // Z = j k eta0/(4 pi) acc, rows of block I, columns of block J
      const int i0 = A.blk_e0[I], ni = A.blk_e0[I + 1] - i0;
      const int j0 = A.blk_e0[J], nj = A.blk_e0[J + 1] - j0;
      const float pref = (float)A.pref;
      for (int e = threadIdx.x; e < ni * nj; e += kAngThreads) {
        const int rr = e / nj, c = e % nj;
        ZT v;
        v.x = -pref * acc[rr * kAngAccStride + 2 * c + 1];
        v.y = pref * acc[rr * kAngAccStride + 2 * c];
        Z[(size_t)(i0 + rr) * A.ldz + (j0 + c)] = v;
      }
      __syncthreads();
    }
  }
  if (bad) atomicOr(A.status, 1);
}

// Largest distance from a quadrature point to a vertex (FP64, the upper end
// of the Exp table): one thread per quadrature point, vertices staged through
// LDS, the maximum of the non-negative distances kept as its bit pattern.
constexpr int kRangeThreads = 256;

__global__ __launch_bounds__(kRangeThreads) void k_range_angular(const double *__restrict__ qp64,
                                                                 const double *__restrict__ V,
                                                                 int nt, int nq, int nv,
                                                                 unsigned long long *out) {
#pragma clang fp contract(off)
  __shared__ double sv[kRangeThreads * 3];
  const int g = blockIdx.x * kRangeThreads + threadIdx.x;
  const bool ok = g < nt * nq;
  double r[3] = {0.0, 0.0, 0.0};
  if (ok) {
    const int t = g / nq, i = g % nq;
    for (int c = 0; c < 3; ++c) r[c] = qp64[((size_t)t * kMaxQ + i) * 3 + c];
  }
  double best = 0.0;
  for (int v0 = 0; v0 < nv; v0 += kRangeThreads) {
    __syncthreads();
    const int v = v0 + threadIdx.x;
    for (int c = 0; c < 3; ++c) sv[3 * threadIdx.x + c] = v < nv ? V[3 * (size_t)v + c] : 0.0;
    __syncthreads();
    const int nb = min(kRangeThreads, nv - v0);
    if (ok)
      for (int j = 0; j < nb; ++j) {
        const double d0 = r[0] - sv[3 * j], d1 = r[1] - sv[3 * j + 1], d2 = r[2] - sv[3 * j + 2];
        const double dd = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        best = dd > best ? dd : best;
      }
  }
  unsigned long long bits = (unsigned long long)__double_as_longlong(best);
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(bits, o);
    bits = y > bits ? y : bits;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(out, bits);
}

int launch_range_angular(mf_mesh *m, const double *V, const Rule &r, double *rmax,
                         hipStream_t s) {
  unsigned long long *d = m->d_scratch + 8;  // one word of the mesh's scratch
  hipError_t e = hipMemsetAsync(d, 0, sizeof(unsigned long long), s);
  const int npts = m->nt * r.nq;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_range_angular, dim3((npts + kRangeThreads - 1) / kRangeThreads),
                       dim3(kRangeThreads), 0, s, m->d_qp64, V, m->nt, r.nq, m->nv, d);
    e = hipGetLastError();
  }
  unsigned long long h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "angular distance range");
  double v;
  static_assert(sizeof(v) == sizeof(h), "bit pattern");
  __builtin_memcpy(&v, &h, sizeof(v));
  *rmax = v;
  return MF_OK;
}

template <int MODE, typename ZT, int NE>
static int launch_ang_t(const AngArgs &A, hipStream_t s) {
  auto kern = k_fill_angular<MODE, ZT, NE>;
  const size_t lds = sizeof(float) * kAngAccFloats;
  MF_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds));
  int dev = 0, ncu = 0, per = 0;
  MF_HIP(hipGetDevice(&dev));
  MF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  MF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kAngThreads, lds));
  if (per < 1) {
    set_error("mf_fill_angular: kernel does not fit on a compute unit");
    return MF_EINVAL;
  }
  long long grid = (long long)ncu * per;
  if (grid > A.ntiles) grid = A.ntiles;
  if (getenv("MOMFILL_VERBOSE"))
    fprintf(stderr, "[momfill] k_fill_angular mode=%d n=%d grid=%lld x %d lds=%zu B\n", MODE, NE,
            grid, kAngThreads, lds);
  if (grid == 0) return MF_OK;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kAngThreads), lds, s, A);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <int MODE, typename ZT>
static int launch_ang_n(const AngArgs &A, int n, hipStream_t s) {
  switch (n) {
    case 4: return launch_ang_t<MODE, ZT, 4>(A, s);
    case 6: return launch_ang_t<MODE, ZT, 6>(A, s);
    default: return launch_ang_t<MODE, ZT, 8>(A, s);
  }
}

int launch_fill_angular(mf_mesh *m, const double *V, const Rule &r, double k, int n_edge,
                        int mode, const mf_tables *tab, void *Z, int z_dtype, int64_t ldz,
                        hipStream_t s) {
  AngArgs A{};
  A.V = V;
  A.qp64 = m->d_qp64;
  A.brad = m->d_brad;
  A.tri = m->d_tri;
  A.rec = m->d_rec;
  A.tiles = m->d_tiles;
  A.blk_e0 = m->d_blk_e0;
  A.blk_off = m->d_blk_off;
  A.blk_tri = m->d_blk_tri;
  A.blk_pos = m->d_blk_pos;
  A.ntiles = (int)m->tiles.size();
  A.nq = r.nq;
  A.ldz = ldz;
  for (int i = 0; i < kMaxQ; ++i) A.w[i] = i < r.nq ? r.w[i] : 0.0;
  A.k = k;
  A.ik2 = 1.0 / (k * k);
  A.pref = k * kEta0 / (4.0 * M_PI);
  if (mode == MF_MODE_TABLE) {
    const mf_tables::One &e = tab->e;
    A.elook = e.look64;
    A.em = e.m64;
    A.einv = e.inv64;
    A.ermax = tab->rmax;
  }
  A.Z = Z;
  A.status = m->d_status;
  if (mode == MF_MODE_TABLE)
    return z_dtype == MF_C64 ? launch_ang_n<MF_MODE_TABLE, float2>(A, n_edge, s)
                             : launch_ang_n<MF_MODE_TABLE, double2>(A, n_edge, s);
  return z_dtype == MF_C64 ? launch_ang_n<MF_MODE_DIRECT, float2>(A, n_edge, s)
                           : launch_ang_n<MF_MODE_DIRECT, double2>(A, n_edge, s);
}

}  // namespace mf
