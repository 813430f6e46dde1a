// Adaptive interpolation tables of Exp(-jkr) and Exp(-jkr)/r, built on the
// device in FP64 (Section II-B, II-C) and packed to FP32 for the fill.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"
#include "lookup.hpp"

namespace mf {

constexpr double kMu = 0.25;    // merge distance, units of t
constexpr double kWin = 2.0;    // refinement window half width, units of t
constexpr double kRatio = 0.5;  // refined interval, units of t
constexpr int kNRef = 4;        // refined samples on each side of a zero
constexpr int kScanThreads = 1024;

enum { kExp = 0, kGreen = 1 };

// ---- sample placement -----------------------------------------------------
// Candidates come in four classes taken in priority order: zeros of the real
// and imaginary parts (r = m pi/(2k)), the end points, refined samples around
// each zero, uniform samples.  A candidate is kept unless a kept sample of an
// earlier class lies closer than mu*t.  Samples of one class are at least
// t/2 > mu*t apart, so each class is decided in parallel after the classes
// before it.  Kept samples go to cells of width mu*t (two slots each), which
// also sorts them.

struct Plan {
  double rmin, rmax, t, c, mind, win_t, step_ref;
  long mz0, nz, nu, ncell;
};

__device__ inline long cell_of(const Plan &P, double x) {
#pragma clang fp contract(off)
  long ci = (long)floor((x - P.rmin) / P.mind) + 1;
  if (ci < 1) ci = 1;
  if (ci > P.ncell - 2) ci = P.ncell - 2;
  return ci;
}

__device__ inline void try_keep(const Plan &P, double *cells, double x) {
  const long ci = cell_of(P, x);
  for (long d = 2 * (ci - 1); d < 2 * (ci + 2); ++d) {
    const double y = cells[d];
    if (!isnan(y) && fabs(y - x) < P.mind) return;
  }
  cells[2 * ci + (isnan(cells[2 * ci]) ? 0 : 1)] = x;
}

__global__ void k_fill_nan(double *p, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = __longlong_as_double(0x7ff8000000000000ll);
}

__global__ void k_place(Plan P, int klass, double *cells) {
#pragma clang fp contract(off)
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (klass == 0) {
    if (i < P.nz) try_keep(P, cells, (double)(P.mz0 + i) * P.c);
  } else if (klass == 1) {
    if (i == 0) try_keep(P, cells, P.rmin);
    if (i == 1) try_keep(P, cells, P.rmax);
  } else if (klass == 2) {
    const long j = i / (2 * kNRef), k = i % (2 * kNRef);
    if (j >= P.nz) return;
    const int s = k < kNRef ? (int)k - kNRef : (int)k - kNRef + 1;  // -4..-1, 1..4
    const double z = (double)(P.mz0 + j) * P.c;
    const double x = z + (double)s * P.step_ref;
    if (x > P.rmin && x < P.rmax) try_keep(P, cells, x);
  } else {
    if (i >= P.nu) return;
    const double x = P.rmin + (double)i * P.t;
    if (!(x < P.rmax)) return;
    const long mm = (long)floor(x / P.c + 0.5);
    for (long d = mm - 1; d <= mm + 1; ++d) {
      if (d < P.mz0 || d >= P.mz0 + P.nz) continue;
      if (fabs(x - (double)d * P.c) < P.win_t) return;  // inside an open window
    }
    try_keep(P, cells, x);
  }
}

// Single-block compaction of the cells into the ascending sample list.
__global__ __launch_bounds__(kScanThreads) void k_compact(const double *cells, long ncell,
                                                          double *out, int *count) {
  __shared__ int part[kScanThreads];
  const long per = (ncell + kScanThreads - 1) / kScanThreads;
  const long c0 = threadIdx.x * per, c1 = min(ncell, c0 + per);
  int cnt = 0;
  for (long c = c0; c < c1; ++c) cnt += !isnan(cells[2 * c]) + !isnan(cells[2 * c + 1]);
  part[threadIdx.x] = cnt;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    int v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int pos = part[threadIdx.x] - cnt;
  if (out) {
    for (long c = c0; c < c1; ++c) {
      double a = cells[2 * c], b = cells[2 * c + 1];
      if (!isnan(a) && !isnan(b) && b < a) {
        double t = a;
        a = b;
        b = t;
      }
      if (!isnan(a)) out[pos++] = a;
      if (!isnan(b)) out[pos++] = b;
    }
  }
  if (threadIdx.x == kScanThreads - 1) *count = part[kScanThreads - 1];
}

__global__ void k_values(const double *r, int n, double k, int kind, double *f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s, c;
  sincos(k * r[i], &s, &c);
  double re = c, im = -s;  // Eq. (1): exp(-jkr)
  if (kind == kGreen) {
    re /= r[i];
    im /= r[i];
  }
  f[2 * i] = re;
  f[2 * i + 1] = im;
}

__global__ void k_min_gap(const double *r, int n, unsigned long long *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long v = ~0ull;
  if (i + 1 < n) v = (unsigned long long)__double_as_longlong(r[i + 1] - r[i]);
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long w = __shfl_xor(v, o);
    v = w < v ? w : v;
  }
  if ((threadIdx.x & 63) == 0 && v != ~0ull) atomicMin(out, v);
}

// Hash array of Eq. (6): the node of each occupied bucket, then a prefix
// maximum fills empty buckets from their predecessor.
__global__ void k_hash_init(int32_t *h, int m) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < m) h[b] = -1;
}

__global__ void k_hash_scatter(const double *r, int n, double rmin, double delta, int m,
                               int32_t *h) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int b = (int)floor((r[i] - rmin) / delta);
  if (b > m - 1) b = m - 1;
  atomicMax(&h[b], i);
}

__global__ __launch_bounds__(kScanThreads) void k_hash_fill(int32_t *h, int m) {
  __shared__ int part[kScanThreads];
  const int per = (m + kScanThreads - 1) / kScanThreads;
  const int b0 = threadIdx.x * per, b1 = min(m, b0 + per);
  int mx = -1;
  for (int b = b0; b < b1; ++b) mx = max(mx, h[b]);
  part[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    int v = threadIdx.x >= o ? part[threadIdx.x - o] : -1;
    __syncthreads();
    part[threadIdx.x] = max(part[threadIdx.x], v);
    __syncthreads();
  }
  int run = threadIdx.x > 0 ? part[threadIdx.x - 1] : -1;
  if (run < 0) run = 0;
  for (int b = b0; b < b1; ++b) {
    run = max(run, h[b]);
    h[b] = run;
  }
}

// ---- FP64 interpolation (linear, Eq. (4); cubic Lagrange, Eq. (5)) --------

__device__ inline void interp64(int kind, const double *r, const double *f, int n, int i, double x,
                                double &re, double &im) {
  if (kind == kExp) {
    const double r0 = r[i], r1 = r[i + 1];
    const double a = (x - r1) / (r0 - r1), b = (x - r0) / (r1 - r0);
    re = f[2 * i] * a + f[2 * i + 2] * b;
    im = f[2 * i + 1] * a + f[2 * i + 3] * b;
    return;
  }
  int s = i - 1;
  if (s > n - 4) s = n - 4;
  if (s < 0) s = 0;
  re = im = 0.0;
  for (int j = s; j < s + 4; ++j) {
    double P = 1.0;
    for (int m = s; m < s + 4; ++m)
      if (m != j) P *= (x - r[m]) / (r[j] - r[m]);
    re += f[2 * j] * P;
    im += f[2 * j + 1] * P;
  }
}

__device__ inline void exact64(int kind, double k, double x, double &re, double &im) {
  double s, c;
  sincos(k * x, &s, &c);
  re = c;
  im = -s;
  if (kind == kGreen) {
    re /= x;
    im /= x;
  }
}

__global__ void k_probe(const double *r, const double *f, int n, int kind, double k,
                        unsigned long long *err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (i + 1 < n) {
    for (int s = 1; s <= 8; ++s) {
      const double x = r[i] + (double)s / 9.0 * (r[i + 1] - r[i]);
      double vr, vi, er, ei;
      interp64(kind, r, f, n, i, x, vr, vi);
      exact64(kind, k, x, er, ei);
      e = fmax(e, hypot(vr - er, vi - ei) / hypot(er, ei));
    }
  }
  if (i == n - 1 && n >= 2) {  // r_max, in the last interval
    const double x = r[n - 1];
    double vr, vi, er, ei;
    interp64(kind, r, f, n, n - 2, x, vr, vi);
    exact64(kind, k, x, er, ei);
    e = fmax(e, hypot(vr - er, vi - ei) / hypot(er, ei));
  }
  unsigned long long v = (unsigned long long)__double_as_longlong(e);
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long w = __shfl_xor(v, o);
    v = w > v ? w : v;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(err, v);
}

// ---- FP32 packing --------------------------------------------------------
// Bucket of every sample, by the FP32 formula of the lookup itself.
__global__ void k_node_bucket(const double *r, int n, float inv, float bias, float top, int *nb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) nb[i] = look_bucket((float)r[i], inv, bias, top);
}

// Bucket records of the FP32 lookup (layout in lookup.hpp).  The bucket's
// samples are found by binary search over the samples' buckets; the first
// sample (r_min) and the last (r_max) are never splits, so the interval
// index stays in [0, n - 2].  More than two samples in a bucket sets *bad.
__global__ void k_pack_look(const double *r, const int *nb, int n, int mb, int4 *look, int *bad) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= mb) return;
  int lo = 0, hi = n;  // first sample whose bucket is >= b
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (nb[mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  int i0 = lo - 1, c = lo;
  if (i0 < 0) {
    i0 = 0;
    c = 1;
  }
  if (i0 > n - 2) i0 = n - 2;
  const float inf = __int_as_float(0x7f800000);
  float s1 = inf, s2 = inf;
  if (c < n - 1 && nb[c] == b) {
    s1 = (float)r[c];
    if (c + 1 < n - 1 && nb[c + 1] == b) {
      s2 = (float)r[c + 1];
      if (c + 2 < n - 1 && nb[c + 2] == b) atomicOr(bad, 1);
    }
  }
  look[b] = make_int4(i0, __float_as_int((float)r[i0]), __float_as_int(s1), __float_as_int(s2));
}

// One-sample bucket records (look_offset1 in lookup.hpp): the byte offset
// 16 i0 of the coefficients of the interval i0 containing the bucket's first
// point, its first sample and the next sample (+inf after the last
// interval).  Two samples in one bucket set *bad.
__global__ void k_pack_look1(const double *r, const int *nb, int n, int mb, int4 *look,
                             int *bad) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= mb) return;
  int lo = 0, hi = n;  // first sample whose bucket is >= b
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (nb[mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  int i0 = lo - 1, c = lo;
  if (i0 < 0) {
    i0 = 0;
    c = 1;
  }
  if (i0 > n - 2) i0 = n - 2;
  if (c < n - 1 && nb[c] == b && c + 1 < n - 1 && nb[c + 1] == b) atomicOr(bad, 1);
  const float x1 = i0 + 1 < n - 1 ? (float)r[i0 + 1] : __int_as_float(0x7f800000);
  look[b] = make_int4(16 * i0, __float_as_int((float)r[i0]), __float_as_int(x1), 0);
}

// Cubic Lagrange polynomial of interval i (stencil s..s+3) re-expanded in
// powers of u = r - float(r_i): sum_k c_k u^k, coefficients in FP64, stored
// as two arrays of n-1 records, (c0, c1) then (c2, c3).
__global__ void k_pack_green(const double *r, const double *f, int n, float4 *coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  int s = i - 1;
  if (s > n - 4) s = n - 4;
  if (s < 0) s = 0;
  const double base = (double)(float)r[i];
  double cr[4] = {0, 0, 0, 0}, ci[4] = {0, 0, 0, 0};
  for (int j = s; j < s + 4; ++j) {
    double d[3], den = 1.0;
    int q = 0;
    for (int mm = s; mm < s + 4; ++mm) {
      if (mm == j) continue;
      d[q++] = r[mm] - base;
      den *= r[j] - r[mm];
    }
    // (u - d0)(u - d1)(u - d2) = u^3 - e1 u^2 + e2 u - e3
    const double e1 = d[0] + d[1] + d[2];
    const double e2 = d[0] * d[1] + d[0] * d[2] + d[1] * d[2];
    const double e3 = d[0] * d[1] * d[2];
    const double pr = f[2 * j] / den, pi = f[2 * j + 1] / den;
    cr[3] += pr;
    ci[3] += pi;
    cr[2] -= e1 * pr;
    ci[2] -= e1 * pi;
    cr[1] += e2 * pr;
    ci[1] += e2 * pi;
    cr[0] -= e3 * pr;
    ci[0] -= e3 * pi;
  }
  coef[i] = make_float4((float)cr[0], (float)ci[0], (float)cr[1], (float)ci[1]);
  coef[(n - 1) + i] = make_float4((float)cr[2], (float)ci[2], (float)cr[3], (float)ci[3]);
}

// Linear interpolant of interval i written about float(r_i).
__global__ void k_pack_exp(const double *r, const double *f, int n, float4 *coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  const double h = r[i + 1] - r[i];
  const double sr = (f[2 * i + 2] - f[2 * i]) / h, si = (f[2 * i + 3] - f[2 * i + 1]) / h;
  const double base = (double)(float)r[i];
  const double vr = f[2 * i] + sr * (base - r[i]), vi = f[2 * i + 1] + si * (base - r[i]);
  coef[i] = make_float4((float)vr, (float)vi, (float)sr, (float)si);
}

// FP64 bucket records of the linear Exp table (a coarsened form of the hash
// of Eq. (6) for a table that starts at r = 0): bucket b = (int)(r * inv)
// with width just under the smallest sample interval holds at most one
// sample; its record carries that sample (split, +inf if none), the bucket
// start x_b and both candidate intervals as value-at-x_b (FP64) and slope
// (FP32: the slope only multiplies r - x_b, less than one bucket), so one
// 64-byte read answers a lookup.  Sample buckets use the lookup's own formula.
__global__ void k_node_bucket64(const double *r, int n, double inv, int *nb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) nb[i] = (int)(r[i] * inv);
}

__device__ inline void linear_at(const double *r, const double *f, int i, double x, double *o) {
  const double h = r[i + 1] - r[i];
  const double sr = (f[2 * i + 2] - f[2 * i]) / h, si = (f[2 * i + 3] - f[2 * i + 1]) / h;
  o[0] = f[2 * i] + sr * (x - r[i]);
  o[1] = f[2 * i + 1] + si * (x - r[i]);
  o[2] = sr;
  o[3] = si;
}

__global__ void k_pack_look64(const double *r, const double *f, const int *nb, int n, int m,
                              double inv, double *look, int *bad) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= m) return;
  int lo = 0, hi = n;  // first sample whose bucket is >= b
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (nb[mid] < b)
      lo = mid + 1;
    else
      hi = mid;
  }
  const int c = lo;
  int iL = c - 1, iR = c;
  double split = __longlong_as_double(0x7ff0000000000000ll);
  if (c < n && nb[c] == b) {
    split = r[c];
    if (c + 1 < n && nb[c + 1] == b) atomicOr(bad, 1);
  } else {
    iR = iL;
  }
  iL = iL < 0 ? 0 : (iL > n - 2 ? n - 2 : iL);
  iR = iR < 0 ? 0 : (iR > n - 2 ? n - 2 : iR);
  const double xb = (double)b / inv;
  double *o = look + 8 * (size_t)b;
  double L[4], Rr[4];
  linear_at(r, f, iL, xb, L);
  linear_at(r, f, iR, xb, Rr);
  o[0] = split;
  o[1] = xb;
  o[2] = L[0];
  o[3] = L[1];
  o[4] = Rr[0];
  o[5] = Rr[1];
  float *sl = reinterpret_cast<float *>(o + 6);
  sl[0] = (float)L[2];
  sl[1] = (float)L[3];
  sl[2] = (float)Rr[2];
  sl[3] = (float)Rr[3];
}

// ---- host driver ---------------------------------------------------------

static unsigned blocks(long n, int t) { return (unsigned)((n + t - 1) / t); }

// Uniform interval from Eq. (10): linear (n = 1) with |E''| = k^2 |E| and the
// widest merged gap (1 + mu) t; cubic (n = 3) with |G''''|/|G| bounded by
// k^4 + 4k^3/r + 12k^2/r^2 + 24k/r^3 + 24/r^4 at r_min.  Capped at a 32nd of
// a wavelength so that refinement windows never overlap.
static double interval_from_tol(int kind, double k, double rmin, double tol) {
  double t;
  if (kind == kExp) {
    t = std::sqrt(8.0 * tol) / (k * (1.0 + kMu));
  } else {
    const double r = rmin;
    const double b4 = k * k * k * k + 4.0 * k * k * k / r + 12.0 * k * k / (r * r) +
                      24.0 * k / (r * r * r) + 24.0 / (r * r * r * r);
    t = std::pow(16.0 * tol / b4, 0.25);
  }
  const double cap = (2.0 * M_PI / k) / 32.0;
  return t < cap ? t : cap;
}

static void release(mf_tables::One &o) {
  // the arrays live in the caller's workspace: forget them
  o.r = o.f = nullptr;
  o.hash = nullptr;
  o.look = nullptr;
  o.look1 = nullptr;
  o.coef = nullptr;
  o.look64 = nullptr;
}

static Plan make_plan(double k, double rmin, double rmax, double t) {
  Plan P{};
  P.rmin = rmin;
  P.rmax = rmax;
  P.t = t;
  P.c = M_PI / (2.0 * k);
  P.mind = kMu * t;
  P.win_t = kWin * t;
  P.step_ref = kRatio * t;
  P.mz0 = (long)std::floor(P.rmin / P.c) + 1;
  P.nz = 0;
  while ((double)(P.mz0 + P.nz) * P.c < P.rmax) ++P.nz;
  P.nu = (long)std::floor((P.rmax - P.rmin) / t) + 2;
  P.ncell = (long)std::floor((P.rmax - P.rmin) / P.mind) + 3;
  return P;
}

// Arrays of one table in the workspace arena: samples and values, hash
// (bottom) and the placement cells and counters (top, released on return).
static int build_one(mf_tables *T, int kind, double t, mf_tables::One &o, hipStream_t s) {
  release(o);
  const Plan P = make_plan(T->k, T->rmin, T->rmax, t);
  Arena &A = T->arena;
  const size_t top0 = A.hi;
  double *cells = nullptr;
  int *d_count = nullptr;
  unsigned long long *d_u = nullptr;
  auto out_of_space = [&]() {
    A.hi = top0;
    set_error("mf_build_tables: table workspace too small");
    return MF_ENOMEM;
  };
  if (!A.top(&cells, 2 * (size_t)P.ncell) || !A.top(&d_count, 1) || !A.top(&d_u, 2))
    return out_of_space();
#define CK(call)                   \
  do {                             \
    hipError_t e_ = (call);        \
    if (e_ != hipSuccess) {        \
      A.hi = top0;                 \
      return hip_fail(e_, #call);  \
    }                              \
  } while (0)
  hipLaunchKernelGGL(k_fill_nan, dim3(blocks(2 * P.ncell, 256)), dim3(256), 0, s, cells,
                     2 * P.ncell);
  const long ncand[4] = {P.nz, 2, P.nz * 2 * kNRef, P.nu};
  for (int klass = 0; klass < 4; ++klass)
    if (ncand[klass] > 0)
      hipLaunchKernelGGL(k_place, dim3(blocks(ncand[klass], 256)), dim3(256), 0, s, P, klass,
                         cells);
  CK(hipGetLastError());
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(kScanThreads), 0, s, cells, P.ncell, nullptr,
                     d_count);
  int n = 0;
  CK(hipMemcpyAsync(&n, d_count, sizeof(int), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  if (n < (kind == kExp ? 2 : 4)) {
    A.hi = top0;
    set_error("mf_build_tables: range too short for the interpolation stencil");
    return MF_EINVAL;
  }
  o.n = n;
  // samples and values in one array, the values 256-byte aligned
  const size_t n_pad = ((size_t)n + 31) & ~(size_t)31;
  if (!A.bottom(&o.r, n_pad + 2 * (size_t)n)) return out_of_space();
  o.f = o.r + n_pad;
  hipLaunchKernelGGL(k_compact, dim3(1), dim3(kScanThreads), 0, s, cells, P.ncell, o.r, d_count);
  hipLaunchKernelGGL(k_values, dim3(blocks(n, 256)), dim3(256), 0, s, o.r, n, T->k, kind, o.f);
  unsigned long long init[2] = {~0ull, 0ull};
  CK(hipMemcpyAsync(d_u, init, sizeof(init), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_min_gap, dim3(blocks(n, 256)), dim3(256), 0, s, o.r, n, d_u);
  hipLaunchKernelGGL(k_probe, dim3(blocks(n, 256)), dim3(256), 0, s, o.r, o.f, n, kind, T->k,
                     d_u + 1);
  CK(hipGetLastError());
  unsigned long long res[2];
  CK(hipMemcpyAsync(res, d_u, sizeof(res), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  std::memcpy(&o.delta, &res[0], 8);
  std::memcpy(&o.err, &res[1], 8);
  o.t = t;
  o.m = (int)std::floor((T->rmax - T->rmin) / o.delta) + 1;
  if (!A.bottom(&o.hash, (size_t)o.m)) return out_of_space();
  hipLaunchKernelGGL(k_hash_init, dim3(blocks(o.m, 256)), dim3(256), 0, s, o.hash, o.m);
  hipLaunchKernelGGL(k_hash_scatter, dim3(blocks(n, 256)), dim3(256), 0, s, o.r, n, T->rmin,
                     o.delta, o.m, o.hash);
  hipLaunchKernelGGL(k_hash_fill, dim3(1), dim3(kScanThreads), 0, s, o.hash, o.m);
  CK(hipGetLastError());
  // the caller's stream has used the temporaries; later work on it may reuse them
  A.hi = top0;
#undef CK
  return MF_OK;
}

// Bucket width of the FP32 lookup: just under twice the smallest sample
// interval, so that FP32 rounding of the bucket coordinate can never put
// three samples in one bucket.
constexpr double kBucketWidth = 1.99;
// the fill's one-sample buckets: just under the smallest interval
constexpr double kBucketWidth1 = 0.99;

static int pack(mf_tables *T, int kind, mf_tables::One &o, hipStream_t s) {
  Arena &A = T->arena;
  const size_t top0 = A.hi;
  auto out_of_space = [&]() {
    A.hi = top0;
    set_error("mf_build_tables: table workspace too small");
    return MF_ENOMEM;
  };
  const double bw = kBucketWidth * o.delta;
  o.mb = (int)std::floor((T->rmax - T->rmin) / bw) + 1;
  o.binv = (float)(1.0 / bw);
  o.bbias = (float)(-T->rmin / bw);
  o.btop = (float)(o.mb - 1);
  int *nb = nullptr, *bad = nullptr;
  if (!A.bottom(&o.look, (size_t)o.mb) ||
      !A.bottom(&o.coef, (kind == kGreen ? 2 : 1) * (size_t)(o.n - 1)) ||
      !A.top(&nb, (size_t)o.n + 1) || !A.top(&bad, 1))
    return out_of_space();
  hipError_t e = hipMemsetAsync(bad, 0, sizeof(int), s);
  if (e != hipSuccess) {
    A.hi = top0;
    return hip_fail(e, "table packing");
  }
  hipLaunchKernelGGL(k_node_bucket, dim3(blocks(o.n, 256)), dim3(256), 0, s, o.r, o.n, o.binv,
                     o.bbias, o.btop, nb);
  hipLaunchKernelGGL(k_pack_look, dim3(blocks(o.mb, 256)), dim3(256), 0, s, o.r, nb, o.n, o.mb,
                     o.look, bad);
  if (kind == kGreen) {
    hipLaunchKernelGGL(k_pack_green, dim3(blocks(o.n, 256)), dim3(256), 0, s, o.r, o.f, o.n,
                       o.coef);
    const double bw1 = kBucketWidth1 * o.delta;
    o.mb1 = (int)std::floor((T->rmax - T->rmin) / bw1) + 1;
    o.binv1 = (float)(1.0 / bw1);
    o.bbias1 = (float)(-T->rmin / bw1);
    o.btop1 = (float)(o.mb1 - 1);
    if (!A.bottom(&o.look1, (size_t)o.mb1)) return out_of_space();
    hipLaunchKernelGGL(k_node_bucket, dim3(blocks(o.n, 256)), dim3(256), 0, s, o.r, o.n, o.binv1,
                       o.bbias1, o.btop1, nb);
    hipLaunchKernelGGL(k_pack_look1, dim3(blocks(o.mb1, 256)), dim3(256), 0, s, o.r, nb, o.n,
                       o.mb1, o.look1, bad);
  } else {
    hipLaunchKernelGGL(k_pack_exp, dim3(blocks(o.n, 256)), dim3(256), 0, s, o.r, o.f, o.n,
                       o.coef);
  }
  if (kind == kExp && T->rmin == 0.0) {
    const double w = 0.999 * o.delta;
    o.inv64 = 1.0 / w;
    o.m64 = (int)(T->rmax * o.inv64) + 1;
    if (!A.bottom(&o.look64, 8 * (size_t)o.m64)) return out_of_space();
    hipLaunchKernelGGL(k_node_bucket64, dim3(blocks(o.n, 256)), dim3(256), 0, s, o.r, o.n,
                       o.inv64, nb);
    hipLaunchKernelGGL(k_pack_look64, dim3(blocks(o.m64, 256)), dim3(256), 0, s, o.r, o.f, nb,
                       o.n, o.m64, o.inv64, o.look64, bad);
  }
  int hbad = 0;
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  A.hi = top0;
  if (e != hipSuccess) return hip_fail(e, "table packing");
  if (hbad) {
    set_error("mf_build_tables: a lookup bucket holds more samples than its record");
    return MF_EINVAL;
  }
  return MF_OK;
}

// Workspace bound of one table: every array at the largest size the probe
// loop can reach (t down to t0/16 after eight refinements).  Counts of a
// plan never grow with t, and kept samples are at least mu t apart, so the
// bucket counts are bounded through the smallest interval mu t.
static void count_table(Arena &A, int kind, double k, double rmin, double rmax, double tol,
                        size_t &top_max) {
  const double t0 = interval_from_tol(kind, k, rmin, tol);
  const double tmin = t0 / 16.0 * (1.0 - 1e-9);
  const Plan P = make_plan(k, rmin, rmax, tmin);
  const size_t n = (size_t)(P.nz * (1 + 2 * kNRef) + 2 + P.nu) + 2;
  const double dmin = kMu * tmin;
  const size_t m = (size_t)std::floor((rmax - rmin) / dmin) + 3;
  double *r = nullptr;
  int32_t *h = nullptr;
  int4 *look = nullptr;
  float4 *coef = nullptr;
  A.bottom(&r, ((n + 31) & ~(size_t)31) + 2 * n);
  A.bottom(&h, m);
  A.bottom(&look, (size_t)std::floor((rmax - rmin) / (kBucketWidth * dmin)) + 3);
  A.bottom(&coef, (kind == kGreen ? 2 : 1) * n);
  if (kind == kGreen)
    A.bottom(&look, (size_t)std::floor((rmax - rmin) / (kBucketWidth1 * dmin)) + 3);
  if (kind == kExp && rmin == 0.0) A.bottom(&r, 8 * ((size_t)(rmax / (0.999 * dmin)) + 3));
  // temporaries: placement cells and counters, or the packing's bucket list
  const size_t place = Arena::up(sizeof(double) * 2 * (size_t)P.ncell) + 2 * 256;
  const size_t packing = Arena::up(sizeof(int) * (n + 1)) + 256;
  top_max = std::max(top_max, std::max(place, packing) + 256);
}

size_t tables_workspace_bytes(double k, double rmin, double rmax, double tol, bool green) {
  Arena A = Arena::counter();
  size_t top = 0;
  if (green) count_table(A, kGreen, k, rmin, rmax, tol, top);
  count_table(A, kExp, k, rmin, rmax, tol, top);
  return A.lo + top + 512;
}

void release_tables(mf_tables *t) {
  release(t->e);
  release(t->g);
  t->arena.lo = 0;
  t->arena.hi = t->arena.size;
}

int build_tables_device(mf_tables *T, double tol, hipStream_t s, bool green) {
  for (int kind : {kGreen, kExp}) {
    if (kind == kGreen && !green) continue;
    mf_tables::One &o = kind == kGreen ? T->g : T->e;
    double t = interval_from_tol(kind, T->k, T->rmin, tol);
    bool ok = false;
    const size_t mark = T->arena.lo;  // each attempt reuses this table's space
    for (int it = 0; it <= 8; ++it) {
      T->arena.lo = mark;
      int rc = build_one(T, kind, t, o, s);
      if (rc) return rc;
      o.iters = it;
      if (o.err <= tol) {
        ok = true;
        break;
      }
      t = t / std::sqrt(2.0);
    }
    if (!ok) {
      set_error("mf_build_tables: probe check above tol after 8 refinements");
      return MF_ENOTCONV;
    }
    int rc = pack(T, kind, o, s);
    if (rc) return rc;
  }
  return MF_OK;
}

// ---- FP32 evaluation (the lookup and polynomial the fill uses) ------------

__global__ void k_table_eval(const int4 *look, const float4 *coef, int tn, float binv,
                             float bbias, float btop, double lo, double hi, int kind, int64_t n,
                             const double *r, double *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = r[i];
  if (!(x >= lo && x <= hi)) {
    out[2 * i] = out[2 * i + 1] = __longlong_as_double(0x7ff8000000000000ll);
    return;
  }
  const float rf = (float)x;
  float u;
  const int ii = look_interval(look_record(look, look_bucket(rf, binv, bbias, btop)), rf, u);
  float2 v;
  if (kind == kGreen) {
    v = cubic(coef[ii], coef[(tn - 1) + ii], u);
  } else {
    const float4 c = coef[ii];
    v = make_float2(fmaf(c.z, u, c.x), fmaf(c.w, u, c.y));
  }
  out[2 * i] = v.x;
  out[2 * i + 1] = v.y;
}

int launch_table_eval(const mf_tables *T, int which, int64_t n, const double *r, double *out,
                      hipStream_t s) {
  const mf_tables::One &o = which == 0 ? T->e : T->g;
  hipLaunchKernelGGL(k_table_eval, dim3(blocks(n, 256)), dim3(256), 0, s, o.look, o.coef, o.n,
                     o.binv, o.bbias, o.btop, T->rmin, T->rmax, which == 0 ? kExp : kGreen, n,
                     r, out);
  MF_HIP(hipGetLastError());
  return MF_OK;
}

}  // namespace mf
