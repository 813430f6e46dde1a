// FP64 touching-pair block (singularity cancellation), shared by the fill
// and the adjoint.
#pragma once

#include <hip/hip_runtime.h>

#include "dual.hpp"
#include "internal.hpp"

namespace mf {

struct RuleArg {
  int nq;
  double b[kMaxQ][3];
  double w[kMaxQ];
};

// Potentials of a flat triangle with unit density at r:
//   S = int dS'/|r-r'|,  V = int (r'-r)/|r-r'| dS'
// from the edge formulas of Wilton et al. (IEEE TAP 32(3), 1984) and Graglia
// (IEEE TAP 41(10), 1993): project r onto the plane, sum one logarithm per
// edge and, off the plane, one arctangent pair per edge.
// T is double, or Dual<N> for the adjoint's derivatives (dual.hpp).
template <class T>
__device__ inline void tri_potentials(const T x[3][3], const T *r, T *S, T *Vv) {
  const T e1[3] = {x[1][0] - x[0][0], x[1][1] - x[0][1], x[1][2] - x[0][2]};
  const T e2[3] = {x[2][0] - x[0][0], x[2][1] - x[0][1], x[2][2] - x[0][2]};
  T n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
            e1[0] * e2[1] - e1[1] * e2[0]};
  const T nn = d_sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  n[0] /= nn;
  n[1] /= nn;
  n[2] /= nn;
  const T h = n[0] * (r[0] - x[0][0]) + n[1] * (r[1] - x[0][1]) + n[2] * (r[2] - x[0][2]);
  const T ah = d_fabs(h);
  const T pr[3] = {r[0] - h * n[0], r[1] - h * n[1], r[2] - h * n[2]};
  T s = 0.0, vin[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 3; ++i) {
    const T *a = x[i], *b = x[(i + 1) % 3];
    T t[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const T len = d_sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    t[0] /= len;
    t[1] /= len;
    t[2] /= len;
    const T m[3] = {t[1] * n[2] - t[2] * n[1], t[2] * n[0] - t[0] * n[2],
                    t[0] * n[1] - t[1] * n[0]};
    const T ap[3] = {a[0] - pr[0], a[1] - pr[1], a[2] - pr[2]};
    const T bp[3] = {b[0] - pr[0], b[1] - pr[1], b[2] - pr[2]};
    const T sa = ap[0] * t[0] + ap[1] * t[1] + ap[2] * t[2];
    const T sb = bp[0] * t[0] + bp[1] * t[1] + bp[2] * t[2];
    const T p0 = ap[0] * m[0] + ap[1] * m[1] + ap[2] * m[2];
    const T q2 = p0 * p0 + h * h;
    const T Ra = d_sqrt((r[0] - a[0]) * (r[0] - a[0]) + (r[1] - a[1]) * (r[1] - a[1]) +
                        (r[2] - a[2]) * (r[2] - a[2]));
    const T Rb = d_sqrt((r[0] - b[0]) * (r[0] - b[0]) + (r[1] - b[1]) * (r[1] - b[1]) +
                        (r[2] - b[2]) * (r[2] - b[2]));
    T lg = 0.0, at = 0.0;
    if (val(q2) > 0.0) {
      // log((Rb + sb)/(Ra + sa)); R + s = q2/(R - s) when s < 0 avoids cancellation
      const T fb = val(sb) >= 0.0 ? Rb + sb : q2 / (Rb - sb);
      const T fa = val(sa) >= 0.0 ? Ra + sa : q2 / (Ra - sa);
      lg = d_log(fb / fa);
      at = d_atan(p0 * sb / (q2 + ah * Rb)) - d_atan(p0 * sa / (q2 + ah * Ra));
    }
    s += p0 * lg - ah * at;
    const T cv = 0.5 * (q2 * lg + sb * Rb - sa * Ra);
    vin[0] += cv * m[0];
    vin[1] += cv * m[1];
    vin[2] += cv * m[2];
  }
  *S = s;
  Vv[0] = vin[0] - h * n[0] * s;
  Vv[1] = vin[1] - h * n[1] * s;
  Vv[2] = vin[2] - h * n[2] * s;
}

// S, V and grad S = int (r'-r)/|r-r'|^3 dS' of a flat triangle at r.  The
// gradient has one in-plane term per edge (its outward normal m times the
// edge logarithm, negated) and a normal term from the solid angle the
// triangle subtends at r (the arctangent pairs of S): grad S = -sum m_i L_i
// - sign(h) Omega n, which also follows from differentiating the edge
// formulas of S.
__device__ inline void tri_field(const double x[3][3], const double *r, double *S, double *Vv,
                                 double *G) {
  const double e1[3] = {x[1][0] - x[0][0], x[1][1] - x[0][1], x[1][2] - x[0][2]};
  const double e2[3] = {x[2][0] - x[0][0], x[2][1] - x[0][1], x[2][2] - x[0][2]};
  double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                 e1[0] * e2[1] - e1[1] * e2[0]};
  const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  n[0] /= nn;
  n[1] /= nn;
  n[2] /= nn;
  const double h = n[0] * (r[0] - x[0][0]) + n[1] * (r[1] - x[0][1]) + n[2] * (r[2] - x[0][2]);
  const double ah = fabs(h);
  const double pr[3] = {r[0] - h * n[0], r[1] - h * n[1], r[2] - h * n[2]};
  double s = 0.0, om = 0.0, vin[3] = {0.0, 0.0, 0.0}, gin[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < 3; ++i) {
    const double *a = x[i], *b = x[(i + 1) % 3];
    double t[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double len = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    t[0] /= len;
    t[1] /= len;
    t[2] /= len;
    const double m[3] = {t[1] * n[2] - t[2] * n[1], t[2] * n[0] - t[0] * n[2],
                         t[0] * n[1] - t[1] * n[0]};
    const double ap[3] = {a[0] - pr[0], a[1] - pr[1], a[2] - pr[2]};
    const double bp[3] = {b[0] - pr[0], b[1] - pr[1], b[2] - pr[2]};
    const double sa = ap[0] * t[0] + ap[1] * t[1] + ap[2] * t[2];
    const double sb = bp[0] * t[0] + bp[1] * t[1] + bp[2] * t[2];
    const double p0 = ap[0] * m[0] + ap[1] * m[1] + ap[2] * m[2];
    const double q2 = p0 * p0 + h * h;
    const double Ra = sqrt((r[0] - a[0]) * (r[0] - a[0]) + (r[1] - a[1]) * (r[1] - a[1]) +
                           (r[2] - a[2]) * (r[2] - a[2]));
    const double Rb = sqrt((r[0] - b[0]) * (r[0] - b[0]) + (r[1] - b[1]) * (r[1] - b[1]) +
                           (r[2] - b[2]) * (r[2] - b[2]));
    double lg = 0.0, at = 0.0;
    if (q2 > 0.0) {
      const double fb = sb >= 0.0 ? Rb + sb : q2 / (Rb - sb);
      const double fa = sa >= 0.0 ? Ra + sa : q2 / (Ra - sa);
      lg = log(fb / fa);
      at = atan(p0 * sb / (q2 + ah * Rb)) - atan(p0 * sa / (q2 + ah * Ra));
    }
    s += p0 * lg - ah * at;
    om += at;
    const double cv = 0.5 * (q2 * lg + sb * Rb - sa * Ra);
    for (int c = 0; c < 3; ++c) {
      vin[c] += cv * m[c];
      gin[c] -= lg * m[c];
    }
  }
  const double sg = h > 0.0 ? 1.0 : (h < 0.0 ? -1.0 : 0.0);
  *S = s;
  for (int c = 0; c < 3; ++c) {
    Vv[c] = vin[c] - h * n[c] * s;
    G[c] = gin[c] - sg * om * n[c];
  }
}

// (exp(-jkR) - 1)/R, with its Taylor series for kR < 1e-4.
template <class T>
__device__ inline void ghat(T k, T R, T &re, T &im) {
  const T x = k * R;
  if (val(x) < 1e-4) {
    re = -0.5 * k * k * R;
    im = -k + k * k * k * R * R / 6.0;
    return;
  }
  T sh, ch;
  d_sincos(0.5 * x, &sh, &ch);
  const T s1 = 2.0 * sh * ch;
  re = -2.0 * sh * sh / R;
  im = -s1 / R;
}


// One ordered touching pair (p,q) given by its vertices: the inner integral
// over q is S_q + the rule applied to g - 1/R, the outer one the rule over p;
// normalised by A_p A_q like the regular blocks:
//   X[a][b] = (1/A_q) sum_i w_i [ (r_i - v_a).Psi_b(r_i)/4 - Phi(r_i)/k^2 ],
//   Phi = S_q + A_q sum_j w_j ghat(R_ij),
//   Psi_b = V_q + (r_i - v_b) S_q + A_q sum_j w_j (r_j - v_b) ghat(R_ij).
// Quadrature points are b0 x0 + b1 x1 + b2 x2 as in the rest of the path.
// oneway_terms hands every term w_i [...] of the sum to sink(a, b, re, im)
// and returns A_q; the caller applies the 1/A_q.  Only the outer points
// i_begin <= i < i_end are taken (all of them by default).
template <class T, class Sink>
__device__ inline T oneway_terms(const T xp[3][3], const T xq[3][3], const RuleArg &R, T k,
                                 int part, Sink &&sink, int i_begin = 0, int i_end = kMaxQ) {
  const T e1[3] = {xq[1][0] - xq[0][0], xq[1][1] - xq[0][1], xq[1][2] - xq[0][2]};
  const T e2[3] = {xq[2][0] - xq[0][0], xq[2][1] - xq[0][1], xq[2][2] - xq[0][2]};
  const T cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
          cz = e1[0] * e2[1] - e1[1] * e2[0];
  const T Aq = 0.5 * d_sqrt(cx * cx + cy * cy + cz * cz);
  const T ik2 = 1.0 / (k * k);
  for (int i = i_begin; i < R.nq && i < i_end; ++i) {
    T ri[3];
    for (int c = 0; c < 3; ++c)
      ri[c] = R.b[i][0] * xp[0][c] + R.b[i][1] * xp[1][c] + R.b[i][2] * xp[2][c];
    T S, Vv[3];
    tri_potentials(xq, ri, &S, Vv);
    T m1r[3] = {0.0, 0.0, 0.0}, m1i[3] = {0.0, 0.0, 0.0};  // Aq sum_j w_j r_j ghat
    T g0r = 0.0, g0i = 0.0;                                // Aq sum_j w_j ghat
    for (int j = 0; j < R.nq; ++j) {
      T rq[3];
      for (int c = 0; c < 3; ++c)
        rq[c] = R.b[j][0] * xq[0][c] + R.b[j][1] * xq[1][c] + R.b[j][2] * xq[2][c];
      const T d0 = ri[0] - rq[0], d1 = ri[1] - rq[1], d2 = ri[2] - rq[2];
      T gr, gi;
      ghat(k, d_sqrt(d0 * d0 + d1 * d1 + d2 * d2), gr, gi);
      const T wa = Aq * R.w[j];
      g0r += wa * gr;
      g0i += wa * gi;
      for (int c = 0; c < 3; ++c) {
        m1r[c] += wa * rq[c] * gr;
        m1i[c] += wa * rq[c] * gi;
      }
    }
    const T phr = S + g0r, phi = g0i;
    for (int b = 0; b < 3; ++b) {
      T psr[3], psi[3];
      for (int c = 0; c < 3; ++c) {
        psr[c] = Vv[c] + (ri[c] - xq[b][c]) * S + m1r[c] - xq[b][c] * g0r;
        psi[c] = m1i[c] - xq[b][c] * g0i;
      }
      for (int a = 0; a < 3; ++a) {
        const T ua[3] = {ri[0] - xp[a][0], ri[1] - xp[a][1], ri[2] - xp[a][2]};
        T br = 0.0, bi = 0.0;
        if (!(part & MF_PART_PHI)) {
          br += 0.25 * (ua[0] * psr[0] + ua[1] * psr[1] + ua[2] * psr[2]);
          bi += 0.25 * (ua[0] * psi[0] + ua[1] * psi[1] + ua[2] * psi[2]);
        }
        if (!(part & MF_PART_A)) {
          br -= phr * ik2;
          bi -= phi * ik2;
        }
        sink(a, b, R.w[i] * br, R.w[i] * bi);
      }
    }
  }
  return Aq;
}

}  // namespace mf
