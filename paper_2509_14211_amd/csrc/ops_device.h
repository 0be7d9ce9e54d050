// Device-side evaluation of the library's operands and closed operator set,
// shared by the dense kernels and the kernels of vectors with missing
// entries.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.h"

namespace nbgrb {

template <typename T>
__device__ __forceinline__ T load_as(const Operand& o, int64_t i) {
  if (!o.p) return (T)o.iso;
  switch (o.type) {
    case T_BOOL: return (T)(((const uint8_t*)o.p)[i]);
    case T_INT32: return (T)(((const int*)o.p)[i]);
    case T_FP32: return (T)(((const float*)o.p)[i]);
    default: return (T)(((const double*)o.p)[i]);
  }
}

__device__ __forceinline__ bool nonzero_at(const Operand& o, int64_t i) {
  if (!o.p) return o.iso != 0.0;
  switch (o.type) {
    case T_BOOL: return ((const uint8_t*)o.p)[i] != 0;
    case T_INT32: return ((const int*)o.p)[i] != 0;
    case T_FP32: return ((const float*)o.p)[i] != 0.0f;
    default: return ((const double*)o.p)[i] != 0.0;
  }
}

template <typename T>
__device__ __forceinline__ void store_as(void* p, int type, int64_t i, T v) {
  switch (type) {
    case T_BOOL: ((uint8_t*)p)[i] = (uint8_t)(v != (T)0); break;
    case T_INT32: ((int*)p)[i] = (int)v; break;
    case T_FP32: ((float*)p)[i] = (float)v; break;
    default: ((double*)p)[i] = (double)v; break;
  }
}

// Called by thread 0 of the block that produced a guarded residual (and,
// for the fused pass, the dangling mass of the same pass, 0 when none is
// computed).  A residual or mass that is not finite ends the loop and marks
// the guard bad, which the drivers report as an execution error: a NaN
// compares false with the tolerance and would otherwise read as converged.
__device__ __forceinline__ void guard_advance(GuardDev* g, double rho, double D = 0.0) {
  g->rho_prev = g->rho;
  g->rho = rho;
  const int it = g->iters + 1;
  g->iters = it;
  const bool finite = __builtin_isfinite(rho) && __builtin_isfinite(D);
  if (!finite) g->bad = 1;
  g->active = (finite && rho > g->tol && it < g->itermax) ? 1 : 0;
}

// alpha * s + beta with one rounding (generated kernels use the same form).
__device__ __forceinline__ double scalar_value(const ScalarArg& s) {
  return s.dev ? fma(s.alpha, *s.dev, s.beta) : s.beta;
}

template <typename T>
__device__ __forceinline__ T apply_binop(int op, T x, T y) {
  switch (op) {
    case B_PLUS: return x + y;
    case B_MINUS: return x - y;
    case B_TIMES: return x * y;
    case B_DIV: return x / y;
    case B_MAX: return x > y ? x : y;
    case B_MIN: return x < y ? x : y;
    case B_FIRST: return x;
    case B_SECOND: return y;
    default: return fabs(x - y);  // B_ABSDIFF
  }
}

template <typename T>
__device__ __forceinline__ T apply_unop(int op, T x) {
  switch (op) {
    case U_IDENTITY: return x;
    case U_ABS: return fabs(x);
    case U_AINV: return -x;
    case U_MINV: return (T)1 / x;
    default: return x != (T)0 ? (T)1 / x : (T)0;  // U_MINV_OR_ZERO
  }
}

}  // namespace nbgrb
