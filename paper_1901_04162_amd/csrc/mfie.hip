// MFIE touching-pair blocks (FP64).  The MFIE tests n x H with the RWG
// functions themselves (Section IV-B fills the K operator beside the EFIE's
// L operator):
//   Z_mn = <f_m, f_n>/2 - <f_m, n x PV int grad G x f_n dS'>
//        = <f_m, f_n>/2 + (1/4 pi) int int (r' - v_b).(t x d) K(R) dS' dS,
// t = (r - v_a) x n_p, d = r - r', K = (1 + jkR) exp(-jkR)/R^3.  In the
// units of the regular blocks (Z = (1/4 pi) sum s s' l l X) a pair of
// triangles gives
//   p = q:  X_ab = (pi/(2 A_p)) sum_i w_i (r_i - v_a).(r_i - v_b)   (identity term;
//           the K integrand vanishes on a flat triangle)
//   p != q touching: the inner integral of K's singular part 1/R^3 + k^2/(2R)
//           in closed form and the bounded remainder by the rule,
//     X_ab = (1/4) sum_i w_i t_a,i . (W_i x (r_i - v_b)),
//     W_i  = (-grad S_q - (k^2/2) V_q)/A_q + sum_j w_j Krem(R_ij) (r_i - r_j),
//   using d x (r' - v_b) = d x (r - v_b), int d/R^3 dS' = -grad S and
//   int d/R dS' = -V.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "singular.hpp"

namespace mf {

// K(R) - 1/R^3 - k^2/(2R), bounded (-j k^3/3 at R = 0).  From the series of
// (1 + jx) exp(-jx) = 1 + x^2/2 - j x^3/3 - x^4/8 + j x^5/30 + x^6/144 - ...
// for x = kR < 1e-2; otherwise in closed form, with cos x - 1 = -2 sin^2(x/2).
__device__ inline void krem(double k, double R, double &re, double &im) {
  const double x = k * R, k3 = k * k * k;
  if (x < 1e-2) {
    re = k3 * x * (-1.0 / 8.0 + x * x / 144.0);
    im = k3 * (-1.0 / 3.0 + x * x / 30.0);
    return;
  }
  double sh, ch, sx, cx;
  sincos(0.5 * x, &sh, &ch);
  sx = 2.0 * sh * ch;
  cx = 1.0 - 2.0 * sh * sh;
  const double r3 = R * R * R;
  re = (-2.0 * sh * sh + x * sx - 0.5 * x * x) / r3;
  im = (x * cx - sx) / r3;
}

// 255 VGPRs at two waves per SIMD; the default bound of 128 spills the FP64
// state of the pair.
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2))) void k_singular_mfie(
    const double *__restrict__ V, const int32_t *__restrict__ tri, const int32_t *__restrict__ tp,
    const int32_t *__restrict__ tq, int64_t npair, RuleArg R, double k, float *__restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= npair) return;
  const int p = tp[s], q = tq[s];
  double xp[3][3], xq[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      xp[a][c] = V[3 * (size_t)tri[3 * p + a] + c];
      xq[a][c] = V[3 * (size_t)tri[3 * q + a] + c];
    }
  double Xr[9], Xi[9];
  for (int i = 0; i < 9; ++i) Xr[i] = Xi[i] = 0.0;
  const double e1[3] = {xp[1][0] - xp[0][0], xp[1][1] - xp[0][1], xp[1][2] - xp[0][2]};
  const double e2[3] = {xp[2][0] - xp[0][0], xp[2][1] - xp[0][1], xp[2][2] - xp[0][2]};
  double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                 e1[0] * e2[1] - e1[1] * e2[0]};
  const double n2 = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  if (p == q) {
    const double f = M_PI / n2;  // pi/(2 A_p), 2 A_p = |e1 x e2|
    for (int i = 0; i < R.nq; ++i) {
      double ri[3];
      for (int c = 0; c < 3; ++c)
        ri[c] = R.b[i][0] * xp[0][c] + R.b[i][1] * xp[1][c] + R.b[i][2] * xp[2][c];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double d = 0.0;
          for (int c = 0; c < 3; ++c) d += (ri[c] - xp[a][c]) * (ri[c] - xq[b][c]);
          Xr[3 * a + b] += f * R.w[i] * d;
        }
    }
  } else {
    for (int c = 0; c < 3; ++c) n[c] /= n2;
    const double f1[3] = {xq[1][0] - xq[0][0], xq[1][1] - xq[0][1], xq[1][2] - xq[0][2]};
    const double f2[3] = {xq[2][0] - xq[0][0], xq[2][1] - xq[0][1], xq[2][2] - xq[0][2]};
    const double cx = f1[1] * f2[2] - f1[2] * f2[1], cy = f1[2] * f2[0] - f1[0] * f2[2],
                 cz = f1[0] * f2[1] - f1[1] * f2[0];
    const double iAq = 2.0 / sqrt(cx * cx + cy * cy + cz * cz);
    for (int i = 0; i < R.nq; ++i) {
      double ri[3];
      for (int c = 0; c < 3; ++c)
        ri[c] = R.b[i][0] * xp[0][c] + R.b[i][1] * xp[1][c] + R.b[i][2] * xp[2][c];
      double S, Vv[3], G[3];
      tri_field(xq, ri, &S, Vv, G);
      double wr[3], wi[3];
      for (int c = 0; c < 3; ++c) {
        wr[c] = (-G[c] - 0.5 * k * k * Vv[c]) * iAq;
        wi[c] = 0.0;
      }
      for (int j = 0; j < R.nq; ++j) {
        double d[3];
        for (int c = 0; c < 3; ++c)
          d[c] = ri[c] - (R.b[j][0] * xq[0][c] + R.b[j][1] * xq[1][c] + R.b[j][2] * xq[2][c]);
        double kr, ki;
        krem(k, sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), kr, ki);
        for (int c = 0; c < 3; ++c) {
          wr[c] += R.w[j] * kr * d[c];
          wi[c] += R.w[j] * ki * d[c];
        }
      }
      for (int b = 0; b < 3; ++b) {
        const double u[3] = {ri[0] - xq[b][0], ri[1] - xq[b][1], ri[2] - xq[b][2]};
        const double cr[3] = {wr[1] * u[2] - wr[2] * u[1], wr[2] * u[0] - wr[0] * u[2],
                              wr[0] * u[1] - wr[1] * u[0]};
        const double ci[3] = {wi[1] * u[2] - wi[2] * u[1], wi[2] * u[0] - wi[0] * u[2],
                              wi[0] * u[1] - wi[1] * u[0]};
        for (int a = 0; a < 3; ++a) {
          const double ua[3] = {ri[0] - xp[a][0], ri[1] - xp[a][1], ri[2] - xp[a][2]};
          const double t[3] = {ua[1] * n[2] - ua[2] * n[1], ua[2] * n[0] - ua[0] * n[2],
                               ua[0] * n[1] - ua[1] * n[0]};
          const double f = 0.25 * R.w[i];
          Xr[3 * a + b] += f * (t[0] * cr[0] + t[1] * cr[1] + t[2] * cr[2]);
          Xi[3 * a + b] += f * (t[0] * ci[0] + t[1] * ci[1] + t[2] * ci[2]);
        }
      }
    }
  }
  float *o = out + (size_t)s * 18;
  for (int i = 0; i < 9; ++i) {
    o[2 * i] = (float)Xr[i];
    o[2 * i + 1] = (float)Xi[i];
  }
}

int launch_singular_mfie(mf_mesh *m, const double *V, const Rule &r, double k, hipStream_t s) {
  const int64_t np = (int64_t)m->touch_q.size();
  if (np == 0) return MF_OK;
  RuleArg R = rule_arg(r);
  hipLaunchKernelGGL(k_singular_mfie, dim3((unsigned)((np + 127) / 128)), dim3(128), 0, s, V,
                     m->d_tri, m->d_touch_p, m->d_touch_q, np, R, k, m->d_sing);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

}  // namespace mf
