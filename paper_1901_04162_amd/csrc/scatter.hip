// Plane-wave excitation and far field of the RWG currents (FP64), for
// scattering from the filled EFIE system (Section IV-B: PEC sphere under a
// plane wave).
//
//   V_m = int f_m . E0 exp(-j k khat.r) dS
//       = sum over the two triangles of m of s l/2 sum_i w_i (r_i - v).E0 exp(-j k khat.r_i)
//   MFIE: E0 replaced on each triangle by n x H0, H0 = khat x E0 / eta0
//       (the tested n x H_inc; n the unit normal (x1 - x0) x (x2 - x0))
//   F(rhat) = sum_n I_n int f_n exp(+j k rhat.r') dS'
//   sigma(rhat) = (k eta0)^2/(4 pi) |F - rhat (rhat.F)|^2 / |E0|^2
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "singular.hpp"

namespace mf {

struct Vec3d {
  double v[3];
};

// One thread per RWG edge.
template <typename ZT, bool kMfie>
__global__ void k_rhs(const double *__restrict__ V, const int32_t *__restrict__ tri,
                      const int32_t *__restrict__ edges, int ne, RuleArg R, double k, Vec3d kh,
                      Vec3d e0r, Vec3d e0i, ZT *__restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int32_t *E = edges + 6 * (size_t)e;
  double l = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double d = V[3 * (size_t)E[0] + c] - V[3 * (size_t)E[1] + c];
    l += d * d;
  }
  l = sqrt(l);
  double sr = 0.0, si = 0.0;
  for (int h = 0; h < 2; ++h) {
    const int t = E[2 + h], a = E[4 + h];
    const double s = h == 0 ? 1.0 : -1.0;
    double x[3][3];
    for (int v = 0; v < 3; ++v)
      for (int c = 0; c < 3; ++c) x[v][c] = V[3 * (size_t)tri[3 * t + v] + c];
    // the field the edge function is tested with on this triangle
    double fr[3], fi[3];
    if (kMfie) {
      const double e1[3] = {x[1][0] - x[0][0], x[1][1] - x[0][1], x[1][2] - x[0][2]};
      const double e2[3] = {x[2][0] - x[0][0], x[2][1] - x[0][1], x[2][2] - x[0][2]};
      double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                     e1[0] * e2[1] - e1[1] * e2[0]};
      const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      for (int c = 0; c < 3; ++c) n[c] /= nn;
      double hr[3], hi[3];  // khat x E0 / eta0
      for (int c = 0; c < 3; ++c) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        hr[c] = (kh.v[c1] * e0r.v[c2] - kh.v[c2] * e0r.v[c1]) / kEta0;
        hi[c] = (kh.v[c1] * e0i.v[c2] - kh.v[c2] * e0i.v[c1]) / kEta0;
      }
      for (int c = 0; c < 3; ++c) {
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        fr[c] = n[c1] * hr[c2] - n[c2] * hr[c1];
        fi[c] = n[c1] * hi[c2] - n[c2] * hi[c1];
      }
    } else {
      for (int c = 0; c < 3; ++c) {
        fr[c] = e0r.v[c];
        fi[c] = e0i.v[c];
      }
    }
    for (int i = 0; i < R.nq; ++i) {
      double r[3];
      for (int c = 0; c < 3; ++c)
        r[c] = R.b[i][0] * x[0][c] + R.b[i][1] * x[1][c] + R.b[i][2] * x[2][c];
      double dr = 0.0, di = 0.0;  // (r - v) . field
      for (int c = 0; c < 3; ++c) {
        dr += (r[c] - x[a][c]) * fr[c];
        di += (r[c] - x[a][c]) * fi[c];
      }
      double sn, cs;
      sincos(k * (kh.v[0] * r[0] + kh.v[1] * r[1] + kh.v[2] * r[2]), &sn, &cs);
      // exp(-j phase) (dr + j di)
      const double f = s * l * 0.5 * R.w[i];
      sr += f * (cs * dr + sn * di);
      si += f * (cs * di - sn * dr);
    }
  }
  out[e].x = sr;
  out[e].y = si;
}

constexpr int kFarThreads = 256;

// One workgroup per direction; threads stride over the edges.
template <typename ZT>
__global__ __launch_bounds__(kFarThreads) void k_far_field(
    const double *__restrict__ V, const int32_t *__restrict__ tri,
    const int32_t *__restrict__ edges, int ne, RuleArg R, double k,
    const ZT *__restrict__ I, const double *__restrict__ dirs, double e0n2,
    double *__restrict__ F, double *__restrict__ sigma) {
  __shared__ double red[kFarThreads][6];
  const int d = blockIdx.x;
  const double ux = dirs[3 * d], uy = dirs[3 * d + 1], uz = dirs[3 * d + 2];
  double acc[6] = {0, 0, 0, 0, 0, 0};  // re/im of the three components
  for (int e = threadIdx.x; e < ne; e += kFarThreads) {
    const int32_t *E = edges + 6 * (size_t)e;
    double l = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double q = V[3 * (size_t)E[0] + c] - V[3 * (size_t)E[1] + c];
      l += q * q;
    }
    l = sqrt(l);
    const double Ir = (double)I[e].x, Ii = (double)I[e].y;
    for (int h = 0; h < 2; ++h) {
      const int t = E[2 + h], a = E[4 + h];
      const double s = h == 0 ? 1.0 : -1.0;
      double x[3][3];
      for (int v = 0; v < 3; ++v)
        for (int c = 0; c < 3; ++c) x[v][c] = V[3 * (size_t)tri[3 * t + v] + c];
      for (int i = 0; i < R.nq; ++i) {
        double r[3];
        for (int c = 0; c < 3; ++c)
          r[c] = R.b[i][0] * x[0][c] + R.b[i][1] * x[1][c] + R.b[i][2] * x[2][c];
        double sn, cs;
        sincos(k * (ux * r[0] + uy * r[1] + uz * r[2]), &sn, &cs);
        // I exp(+j phase) s l/2 w
        const double f = s * l * 0.5 * R.w[i];
        const double pr = f * (Ir * cs - Ii * sn), pi = f * (Ir * sn + Ii * cs);
        for (int c = 0; c < 3; ++c) {
          const double q = r[c] - x[a][c];
          acc[2 * c] += pr * q;
          acc[2 * c + 1] += pi * q;
        }
      }
    }
  }
  for (int c = 0; c < 6; ++c) red[threadIdx.x][c] = acc[c];
  __syncthreads();
  for (int h = kFarThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int c = 0; c < 6; ++c) red[threadIdx.x][c] += red[threadIdx.x + h][c];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int c = 0; c < 6; ++c) F[6 * (size_t)d + c] = red[0][c];
    if (sigma) {
      const double u[3] = {ux, uy, uz};
      double pr = 0.0, pi = 0.0;  // rhat . F
      for (int c = 0; c < 3; ++c) {
        pr += u[c] * red[0][2 * c];
        pi += u[c] * red[0][2 * c + 1];
      }
      double t2 = 0.0;
      for (int c = 0; c < 3; ++c) {
        const double tr = red[0][2 * c] - u[c] * pr, ti = red[0][2 * c + 1] - u[c] * pi;
        t2 += tr * tr + ti * ti;
      }
      sigma[d] = (k * kEta0) * (k * kEta0) / (4.0 * M_PI) * t2 / e0n2;
    }
  }
}

template <bool kMfie>
static void launch_rhs_t(mf_mesh *m, const double *V, const RuleArg &R, double k, const Vec3d &kh,
                         const Vec3d &er, const Vec3d &ei, void *out, int z_dtype,
                         hipStream_t s) {
  const dim3 grid((m->ne + 127) / 128);
  if (z_dtype == MF_C64)
    hipLaunchKernelGGL((k_rhs<float2, kMfie>), grid, dim3(128), 0, s, V, m->d_tri, m->d_edges,
                       m->ne, R, k, kh, er, ei, reinterpret_cast<float2 *>(out));
  else
    hipLaunchKernelGGL((k_rhs<double2, kMfie>), grid, dim3(128), 0, s, V, m->d_tri, m->d_edges,
                       m->ne, R, k, kh, er, ei, reinterpret_cast<double2 *>(out));
}

int launch_rhs(mf_mesh *m, const double *V, const Rule &r, double k, const double *khat,
               const double *E0, void *out, int z_dtype, hipStream_t s, bool mfie) {
  RuleArg R = rule_arg(r);
  const Vec3d kh{{khat[0], khat[1], khat[2]}};
  const Vec3d er{{E0[0], E0[2], E0[4]}}, ei{{E0[1], E0[3], E0[5]}};
  if (mfie)
    launch_rhs_t<true>(m, V, R, k, kh, er, ei, out, z_dtype, s);
  else
    launch_rhs_t<false>(m, V, R, k, kh, er, ei, out, z_dtype, s);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

int launch_far_field(mf_mesh *m, const double *V, const Rule &r, double k, const void *I,
                     int z_dtype, int n_dirs, const double *dirs, double e0n2, double *F,
                     double *sigma, hipStream_t s) {
  RuleArg R = rule_arg(r);
  if (z_dtype == MF_C64)
    hipLaunchKernelGGL(k_far_field<float2>, dim3(n_dirs), dim3(kFarThreads), 0, s, V, m->d_tri,
                       m->d_edges, m->ne, R, k, reinterpret_cast<const float2 *>(I), dirs, e0n2,
                       F, sigma);
  else
    hipLaunchKernelGGL(k_far_field<double2>, dim3(n_dirs), dim3(kFarThreads), 0, s, V, m->d_tri,
                       m->d_edges, m->ne, R, k, reinterpret_cast<const double2 *>(I), dirs, e0n2,
                       F, sigma);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

}  // namespace mf
