// Wave-uniform read-only data (a source triangle's record, the block lists)
// is read through the constant address space: the loads then go to the scalar
// unit and the values live in SGPRs.  Through plain pointers the compiler
// keeps them as vector loads of one address, which costs VGPRs and a memory
// round trip per triangle pair.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mf {

typedef __attribute__((address_space(4))) const float cfloat;
typedef __attribute__((address_space(4))) const int32_t cint32;
typedef __attribute__((address_space(4))) const double cdouble;
__device__ __forceinline__ cfloat *as_const(const float *p) { return (cfloat *)p; }
__device__ __forceinline__ cint32 *as_const(const int32_t *p) { return (cint32 *)p; }

}  // namespace mf
