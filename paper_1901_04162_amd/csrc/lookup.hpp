// FP32 interval search of the tables (Section II-C), shared by every kernel
// that reads a table so that all of them take the same FP32 decisions.
//
// The buckets are a coarsened form of the hash of Eq. (6): their width is
// just under twice the smallest sample interval, so a bucket holds at most
// two samples.  Each bucket stores one 16-byte record
//   { i0, x(i0), s1, s2 }
// with i0 the interval that contains the bucket's first point, x(i0) that
// interval's first sample and s1, s2 the positions of the samples inside the
// bucket (+inf where there are fewer; the last sample is never a split, so
// the interval index stays at most n - 2).  The interval of r is then
//   i0 + [r >= s1] + [r >= s2]
// and its first sample comes from the same record, so one gather gives both
// the interval and the origin u = r - x(i) of its polynomial: the paper's
// bucket read, compare-with-the-sample fix-up and sample read in one step.
// Bucket membership of every sample is decided with the very FP32 formula
// the lookup uses, so the comparisons agree with it exactly.
#pragma once

#include <hip/hip_runtime.h>

namespace mf {

// Bucket of r: x = r * inv + bias, clamped to [0, top], truncated.
__device__ __forceinline__ int look_bucket(float r, float inv, float bias, float top) {
  return (int)__builtin_amdgcn_fmed3f(fmaf(r, inv, bias), 0.0f, top);
}

// Bucket record b; the 32-bit byte offset lets the load take its base from
// scalar registers.
__device__ __forceinline__ int4 look_record(const int4 *look, int b) {
  return *reinterpret_cast<const int4 *>(reinterpret_cast<const char *>(look) +
                                         ((unsigned)b << 4));
}

// Interval of r from its bucket record; u receives r minus the interval's
// first sample.
__device__ __forceinline__ int look_interval(const int4 &w, float r, float &u) {
  const float s1 = __int_as_float(w.z), s2 = __int_as_float(w.w);
  const bool a1 = r >= s1, a2 = r >= s2;
  u = r - (a2 ? s2 : (a1 ? s1 : __int_as_float(w.y)));
  return w.x + (int)a1 + (int)a2;
}

// The fill kernels read a second set of records whose buckets are just
// narrower than the smallest sample interval, the width of the paper's hash:
// such a bucket holds at most one sample, and its record
//   { 16 i0, x(i0), x(i0 + 1), unused }
// gives the interval as i0 + [r >= x(i0 + 1)] (x(i0 + 1) = +inf when i0 is the
// last interval).  Either x(i0 + 1) lies in the bucket, or beyond it and then
// no r of the bucket reaches it.  One compare and one select fewer per lookup,
// for twice the records.  The interval comes back as the byte offset of its
// 16-byte coefficient record, which the gather takes as it is.
__device__ __forceinline__ int look_offset1(const int4 &w, float r, float &u) {
  const float x1 = __int_as_float(w.z);
  const bool a1 = r >= x1;
  u = r - (a1 ? x1 : __int_as_float(w.y));
  return w.x + (a1 ? 16 : 0);
}

// The float4 at byte offset off from base.
__device__ __forceinline__ float4 at_offset(const float4 *base, int off) {
  return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(base) + off);
}

// Cubic of interval i in Horner form, (c0, c1) and (c2, c3) complex.
__device__ __forceinline__ float2 cubic(const float4 &A, const float4 &B, float u) {
  float re = fmaf(B.z, u, B.x), im = fmaf(B.w, u, B.y);
  re = fmaf(re, u, A.z);
  im = fmaf(im, u, A.w);
  return make_float2(fmaf(re, u, A.x), fmaf(im, u, A.y));
}

}  // namespace mf
