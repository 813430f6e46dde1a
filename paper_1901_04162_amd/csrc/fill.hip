// Regular-pair impedance fill (FP32), table and direct modes.
//
// The output is cut into tiles of kTileEdges x kTileEdges RWG edges.  One
// workgroup owns a tile at a time (persistent grid, tiles strided by the
// grid size) and accumulates its entries in LDS.  A tile needs every
// triangle carrying one of its row edges (list I) against every triangle
// carrying one of its column edges (list J); lane l of a wave takes test
// triangle I[l] (its record in registers) and the wave walks source
// triangles of J (records loaded once per wave through the scalar cache).
// Per triangle pair the Q x Q point pairs are reduced to four moments of
// g = exp(-jkR)/R,
//   S0 = sum w_i w_j g, Srho = sum w_i w_j g rho_i, Srho' = sum w_i w_j g rho'_j,
//   Srr = sum w_i w_j g rho_i.rho'_j,
// from which the nine local entries follow with alpha_a = c_p - v_a and
// beta_b = c_q - v_b:
//   X_ab = (Srr + alpha_a.Srho' + beta_b.Srho + alpha_a.beta_b S0)/4 - S0/k^2.
// Touching pairs take their FP64 blocks from the singular kernel.  The
// Green-function table sits in LDS when it fits and is read from global
// memory otherwise.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.hpp"

namespace mf {

constexpr int kBM = kTileEdges;
constexpr int kAccStride = 2 * kBM + 1;  // odd stride: rows land in different banks
constexpr int kAccFloats = kBM * kAccStride;
constexpr int kFillThreads = 512;

struct FillArgs {
  const float *rec;
  const int32_t *blk_off, *blk_tri, *blk_pos;
  const int32_t *touch_off, *touch_q;
  const float *sing;
  int nblk, ne;
  long long ntiles;
  float k, ik2;
  float pref;  // k eta0 / (4 pi)
  float w[kMaxQ];
  // table (global memory copy)
  const int2 *bucket;
  const float *node;
  const float4 *coef;
  int tn, tm;
  float trmin, tinv, lo_ok, hi_ok;
  void *Z;
  long long ldz;
  int *status;
};

template <bool kLDS>
struct Tab {
  const int2 *bucket;
  const float *node;
  const float4 *coef;
  int m;
  float rmin, inv;
  __device__ __forceinline__ float2 operator()(float r) const {
    int b = (int)((r - rmin) * inv);
    b = min(max(b, 0), m - 1);
    const int2 w = bucket[b];
    const int i = w.x + (r >= __int_as_float(w.y) ? 1 : 0);
    const float u = r - node[i];
    const float4 c01 = coef[2 * i], c23 = coef[2 * i + 1];
    float re = fmaf(c23.z, u, c23.x), im = fmaf(c23.w, u, c23.y);
    re = fmaf(re, u, c01.z);
    im = fmaf(im, u, c01.w);
    re = fmaf(re, u, c01.x);
    im = fmaf(im, u, c01.y);
    return make_float2(re, im);
  }
};

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <int Q, int MODE, bool kLDS, int PART, typename ZT>
__global__ __launch_bounds__(kFillThreads) void k_fill(FillArgs A) {
  extern __shared__ float4 smem4[];
  float *acc = reinterpret_cast<float *>(smem4);
  const int lane = threadIdx.x & 63;
  const int wave = uniform(threadIdx.x >> 6);
  const int nwave = kFillThreads / 64;

  Tab<kLDS> tab;
  if (MODE == MF_MODE_TABLE) {
    tab.m = A.tm;
    tab.rmin = A.trmin;
    tab.inv = A.tinv;
    if (kLDS) {
      float4 *c = smem4 + kAccFloats / 4 + 1;
      int2 *b = reinterpret_cast<int2 *>(c + 2 * (A.tn - 1));
      float *nd = reinterpret_cast<float *>(b + A.tm);
      for (int i = threadIdx.x; i < 2 * (A.tn - 1); i += kFillThreads) c[i] = A.coef[i];
      for (int i = threadIdx.x; i < A.tm; i += kFillThreads) b[i] = A.bucket[i];
      for (int i = threadIdx.x; i < A.tn; i += kFillThreads) nd[i] = A.node[i];
      tab.coef = c;
      tab.bucket = b;
      tab.node = nd;
    } else {
      tab.coef = A.coef;
      tab.bucket = A.bucket;
      tab.node = A.node;
    }
  }
  float rlo = INFINITY, rhi = 0.0f;

  for (long long tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    const int I = (int)(tile / A.nblk), J = (int)(tile % A.nblk);
    for (int i = threadIdx.x; i < kAccFloats; i += kFillThreads) acc[i] = 0.0f;
    __syncthreads();
    const int p0 = A.blk_off[I], np = A.blk_off[I + 1] - p0;
    const int q0 = A.blk_off[J], nq = A.blk_off[J + 1] - q0;
    for (int pc = 0; pc < np; pc += 64) {
      const bool pv = pc + lane < np;
      const int pidx = pv ? pc + lane : pc;
      const int p = A.blk_tri[p0 + pidx];
      const int prow = pv ? A.blk_pos[p0 + pidx] : -1;
      const float *pr = A.rec + (size_t)p * kRecFloats;
      float prho[Q][3], pwrho[Q][3], palpha[3][3], psig[3];
      if (MODE == MF_MODE_TABLE) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            prho[i][c] = pr[kRecRho + 3 * i + c];
            pwrho[i][c] = pr[kRecWRho + 3 * i + c];
          }
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int c = 0; c < 3; ++c) palpha[a][c] = pr[kRecAlpha + 3 * a + c];
        psig[a] = pr[kRecSigma + a];
      }
      const double *pcd = reinterpret_cast<const double *>(pr + kRecCent);
      const double pcx = pcd[0], pcy = pcd[1], pcz = pcd[2];
      const int *pvi = reinterpret_cast<const int *>(pr + kRecVid);
      const int pv0 = pvi[0], pv1 = pvi[1], pv2 = pvi[2];

      for (int qi = wave; qi < nq; qi += nwave) {
        const int q = uniform(A.blk_tri[q0 + qi]);
        const int qcol = uniform(A.blk_pos[q0 + qi]);
        const float *qr = A.rec + (size_t)q * kRecFloats;
        const int *qvi = reinterpret_cast<const int *>(qr + kRecVid);
        const int qv0 = qvi[0], qv1 = qvi[1], qv2 = qvi[2];
        const bool touch = pv0 == qv0 || pv0 == qv1 || pv0 == qv2 || pv1 == qv0 || pv1 == qv1 ||
                           pv1 == qv2 || pv2 == qv0 || pv2 == qv1 || pv2 == qv2;
        float Xr[3][3], Xi[3][3];
        if (!touch) {
          const double *qcd = reinterpret_cast<const double *>(qr + kRecCent);
          const double Dx = pcx - qcd[0], Dy = pcy - qcd[1], Dz = pcz - qcd[2];
          const float hx = (float)Dx, hy = (float)Dy, hz = (float)Dz;
          const float lx = (float)(Dx - (double)hx), ly = (float)(Dy - (double)hy),
                      lz = (float)(Dz - (double)hz);
          float qrho[Q][3], qwrho[Q][3];
#pragma unroll
          for (int j = 0; j < Q; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              qrho[j][c] = qr[kRecRho + 3 * j + c];
              qwrho[j][c] = qr[kRecWRho + 3 * j + c];
            }
          float s0r = 0.f, s0i = 0.f, srr = 0.f, sri = 0.f;
          float spr[3] = {0.f, 0.f, 0.f}, spi[3] = {0.f, 0.f, 0.f};  // Srho
          float sqr[3] = {0.f, 0.f, 0.f}, sqi[3] = {0.f, 0.f, 0.f};  // Srho'
          // direct mode keeps the outer loop rolled (the inlined sincos is long)
          // and reads the test point from the record each time
#pragma unroll(MODE == MF_MODE_TABLE ? Q : 1)
          for (int i = 0; i < Q; ++i) {
            float pri[3], pwi[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              pri[c] = MODE == MF_MODE_TABLE ? prho[i][c] : pr[kRecRho + 3 * i + c];
              pwi[c] = MODE == MF_MODE_TABLE ? pwrho[i][c] : pr[kRecWRho + 3 * i + c];
            }
            const float ax = pri[0] + lx, ay = pri[1] + ly, az = pri[2] + lz;
            float t0r = 0.f, t0i = 0.f;
            float t1r[3] = {0.f, 0.f, 0.f}, t1i[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int j = 0; j < Q; ++j) {
              const float dx = hx + (ax - qrho[j][0]);
              const float dy = hy + (ay - qrho[j][1]);
              const float dz = hz + (az - qrho[j][2]);
              const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
              float gr, gi;
              if (MODE == MF_MODE_TABLE) {
                const float r = __builtin_amdgcn_sqrtf(r2);
                rlo = fminf(rlo, r);
                rhi = fmaxf(rhi, r);
                const float2 g = tab(r);
                gr = g.x;
                gi = g.y;
              } else {
                const float ri = __builtin_amdgcn_rsqf(r2);
                const float r = r2 * ri;
                float sn, cs;
                sincosf(A.k * r, &sn, &cs);
                gr = cs * ri;
                gi = -sn * ri;
              }
              t0r = fmaf(A.w[j], gr, t0r);
              t0i = fmaf(A.w[j], gi, t0i);
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                t1r[c] = fmaf(qwrho[j][c], gr, t1r[c]);
                t1i[c] = fmaf(qwrho[j][c], gi, t1i[c]);
              }
            }
            s0r = fmaf(A.w[i], t0r, s0r);
            s0i = fmaf(A.w[i], t0i, s0i);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              spr[c] = fmaf(pwi[c], t0r, spr[c]);
              spi[c] = fmaf(pwi[c], t0i, spi[c]);
              sqr[c] = fmaf(A.w[i], t1r[c], sqr[c]);
              sqi[c] = fmaf(A.w[i], t1i[c], sqi[c]);
              srr = fmaf(pwi[c], t1r[c], srr);
              sri = fmaf(pwi[c], t1i[c], sri);
            }
          }
          float beta[3][3];
#pragma unroll
          for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) beta[b][c] = qr[kRecAlpha + 3 * b + c];
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              float vr = 0.f, vi = 0.f;
              if (!(PART & MF_PART_PHI)) {
                const float ab = palpha[a][0] * beta[b][0] + palpha[a][1] * beta[b][1] +
                                 palpha[a][2] * beta[b][2];
                vr = srr + ab * s0r;
                vi = sri + ab * s0i;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                  vr = fmaf(palpha[a][c], sqr[c], fmaf(beta[b][c], spr[c], vr));
                  vi = fmaf(palpha[a][c], sqi[c], fmaf(beta[b][c], spi[c], vi));
                }
                vr *= 0.25f;
                vi *= 0.25f;
              }
              if (!(PART & MF_PART_A)) {
                vr = fmaf(-A.ik2, s0r, vr);
                vi = fmaf(-A.ik2, s0i, vi);
              }
              Xr[a][b] = vr;
              Xi[a][b] = vi;
            }
        } else {
          int s = A.touch_off[p];
          const int s1 = A.touch_off[p + 1];
          while (s < s1 && A.touch_q[s] != q) ++s;
          const bool found = s < s1;  // always, touching pairs are listed both ways
          const float *x = A.sing + (size_t)(found ? s : 0) * 18;
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              Xr[a][b] = found ? x[2 * (3 * a + b)] : 0.0f;
              Xi[a][b] = found ? x[2 * (3 * a + b) + 1] : 0.0f;
            }
        }
        if (pv) {
          float qsig[3];
#pragma unroll
          for (int b = 0; b < 3; ++b) qsig[b] = qr[kRecSigma + b];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const int row = (prow >> (8 * a)) & 0xff;
            if (row == 0xff) continue;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              const int col = (qcol >> (8 * b)) & 0xff;
              if (col == 0xff) continue;
              const float sg = psig[a] * qsig[b];
              float *dst = acc + row * kAccStride + 2 * col;
              atomicAdd(dst, sg * Xr[a][b]);
              atomicAdd(dst + 1, sg * Xi[a][b]);
            }
          }
        }
      }
    }
    __syncthreads();
    // Z = j k eta/(4 pi) * acc
    const int i0 = I * kBM, j0 = J * kBM;
    for (int e = threadIdx.x; e < kBM * kBM; e += kFillThreads) {
      const int r = e / kBM, c = e % kBM;
      if (i0 + r < A.ne && j0 + c < A.ne) {
        const float ar = acc[r * kAccStride + 2 * c], ai = acc[r * kAccStride + 2 * c + 1];
        ZT v;
        v.x = -A.pref * ai;
        v.y = A.pref * ar;
        reinterpret_cast<ZT *>(A.Z)[(size_t)(i0 + r) * A.ldz + (j0 + c)] = v;
      }
    }
    __syncthreads();
  }
  if (MODE == MF_MODE_TABLE && (rlo < A.lo_ok || rhi > A.hi_ok)) atomicOr(A.status, 1);
}

template <int Q, int MODE, bool kLDS, int PART, typename ZT>
static int launch_t(const FillArgs &A, size_t lds, hipStream_t s) {
  auto kern = k_fill<Q, MODE, kLDS, PART, ZT>;
  if (lds > 65536) MF_HIP(hipFuncSetAttribute((const void *)kern,
                                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int dev = 0, ncu = 0, per = 0;
  MF_HIP(hipGetDevice(&dev));
  MF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  MF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kFillThreads, lds));
  if (per < 1) {
    set_error("mf_fill_Z: fill kernel does not fit on a compute unit");
    return MF_EINVAL;
  }
  long long grid = (long long)ncu * per;
  if (grid > A.ntiles) grid = A.ntiles;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kFillThreads), lds, s, A);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

template <int Q, int MODE, bool kLDS, typename ZT>
static int launch_part(const FillArgs &A, int part, size_t lds, hipStream_t s) {
  if (part == MF_PART_A) return launch_t<Q, MODE, kLDS, MF_PART_A, ZT>(A, lds, s);
  if (part == MF_PART_PHI) return launch_t<Q, MODE, kLDS, MF_PART_PHI, ZT>(A, lds, s);
  return launch_t<Q, MODE, kLDS, 0, ZT>(A, lds, s);
}

template <int Q, typename ZT>
static int launch_q(const FillArgs &A, int mode, int part, bool lds_tab, size_t lds,
                    hipStream_t s) {
  if (mode == MF_MODE_DIRECT) return launch_part<Q, MF_MODE_DIRECT, false, ZT>(A, part, lds, s);
  if (lds_tab) return launch_part<Q, MF_MODE_TABLE, true, ZT>(A, part, lds, s);
  return launch_part<Q, MF_MODE_TABLE, false, ZT>(A, part, lds, s);
}

template <typename ZT>
static int launch_z(const FillArgs &A, int nq, int mode, int part, bool lds_tab, size_t lds,
                    hipStream_t s) {
  switch (nq) {
    case 3: return launch_q<3, ZT>(A, mode, part, lds_tab, lds, s);
    case 6: return launch_q<6, ZT>(A, mode, part, lds_tab, lds, s);
    default: return launch_q<7, ZT>(A, mode, part, lds_tab, lds, s);
  }
}

int launch_fill(mf_mesh *m, const Rule &r, double k, int mode, const mf_tables *tab, void *Z,
                int z_dtype, int64_t ldz, hipStream_t s) {
  FillArgs A{};
  A.rec = m->d_rec;
  A.blk_off = m->d_blk_off;
  A.blk_tri = m->d_blk_tri;
  A.blk_pos = m->d_blk_pos;
  A.touch_off = m->d_touch_off;
  A.touch_q = m->d_touch_q;
  A.sing = m->d_sing;
  A.nblk = m->nblk;
  A.ne = m->ne;
  A.ntiles = (long long)m->nblk * m->nblk;
  A.k = (float)k;
  A.ik2 = (float)(1.0 / (k * k));
  A.pref = (float)(k * kEta0 / (4.0 * M_PI));
  for (int i = 0; i < kMaxQ; ++i) A.w[i] = i < r.nq ? (float)r.w[i] : 0.0f;
  A.Z = Z;
  A.ldz = ldz;
  A.status = m->d_status;
  const int base = mode & 0xf, part = mode & (MF_PART_A | MF_PART_PHI);
  size_t lds = sizeof(float) * kAccFloats + 16;
  bool lds_tab = false;
  if (base == MF_MODE_TABLE) {
    const mf_tables::One &g = tab->g;
    A.bucket = g.bucket;
    A.node = g.node;
    A.coef = g.coef;
    A.tn = g.n;
    A.tm = g.m;
    A.trmin = (float)tab->rmin;
    A.tinv = (float)(1.0 / g.delta);
    A.lo_ok = (float)(tab->rmin * (1.0 - 1e-6));
    A.hi_ok = (float)(tab->rmax * (1.0 + 1e-6));
    const size_t tbytes = sizeof(float4) * 2 * (size_t)(g.n - 1) + sizeof(int2) * (size_t)g.m +
                          sizeof(float) * (size_t)g.n;
    int dev = 0, maxlds = 0;
    MF_HIP(hipGetDevice(&dev));
    MF_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (lds + tbytes <= (size_t)maxlds) {
      lds_tab = true;
      lds += tbytes;
    }
  }
  if (z_dtype == MF_C64) return launch_z<float2>(A, r.nq, base, part, lds_tab, lds, s);
  return launch_z<double2>(A, r.nq, base, part, lds_tab, lds, s);
}

int launch_backward(mf_mesh *, const double *, const Rule &, double, int, const mf_tables *,
                    const void *, int, int64_t, double *, double *, hipStream_t) {
  set_error("mf_fill_Z_backward: not available in this build");
  return MF_EINVAL;
}

}  // namespace mf
