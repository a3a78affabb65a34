// Device helpers shared by the stage kernels (the plane-marching kernel and
// the WENO5 kernel): the CFL limit of one cell and its reduction.
#pragma once

#include "device_common.h"
#include "foap4_internal.h"

namespace f4 {

// CFL inverse time step sum_d (|v_d| + c) / dx of one cell.  FP64 states use
// the operation order of the definition without contraction (equal to a plain
// evaluation); FP32 states evaluate it in FP32 with the hardware reciprocal
// and square root, and the maximum over cells is reduced in FP64 (an FP32
// maximum converts exactly, so a kernel may keep its running maximum in FP32).
template <int NDIM>
__device__ __forceinline__ double cell_inv_dt(const double *U, double gamma, double dx, bool &bad) {
#pragma clang fp contract(off)
  const double r = U[0];
  double ke = 0.0, v[3];
#pragma unroll
  for (int d = 0; d < NDIM; d++) {
    v[d] = U[1 + d] / r;
    ke += U[1 + d] * v[d];
  }
  const double p = (gamma - 1.0) * (U[NDIM + 1] - 0.5 * ke);
  const double cs = sqrt(gamma * p / r);
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < NDIM; d++) s += (fabs(v[d]) + cs) / dx;
  bad |= !(r > 0.0) || !(p > 0.0) || !isfinite(s);
  return s;
}

template <int NDIM>
__device__ __forceinline__ float cell_inv_dt(const float *U, float gamma, float idx, bool &bad) {
  const float r = U[0];
  const float ir = __builtin_amdgcn_rcpf(r);
  float ke = 0.0f, sv = 0.0f;
#pragma unroll
  for (int d = 0; d < NDIM; d++) {
    const float v = U[1 + d] * ir;
    ke += U[1 + d] * v;
    sv += fabsf(v);
  }
  const float p = (gamma - 1.0f) * (U[NDIM + 1] - 0.5f * ke);
  const float cs = __builtin_amdgcn_sqrtf(gamma * p * ir);
  const float s = (sv + NDIM * cs) * idx;
  bad |= !(r > 0.0f) || !(p > 0.0f) || !isfinite(s);
  return s;
}

// Wave-level maximum of the CFL limits and the unphysical flag of the
// cells a wave updated, folded into the mesh's scalars by one atomic each.
__device__ __forceinline__ void flush_dt(const MeshDev &M, double &vmax, bool &bad) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, o));
  const bool anybad = __ballot(bad) != 0;
  if ((threadIdx.x & 63) == 0) {
    if (vmax > 0.0) atomic_max_pos_if_larger(&M.scal[kMaxInv], vmax);
    if (anybad) atomic_max_pos(&M.scal[kBad], 1.0);
  }
  vmax = 0.0;
  bad = false;
}

}  // namespace f4
