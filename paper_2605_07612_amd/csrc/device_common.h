// Device-side physics and limiter helpers shared by the library's kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace f4 {

// Global-memory access through address-space-1 pointers.  Pointers read out
// of a descriptor are generic, and the compiler would use FLAT instructions,
// which count against the LDS wait counter too: every wait for an LDS result
// would then also wait for all outstanding prefetch loads.
template <typename T>
__device__ __forceinline__ T gload(const T *p) {
  return *(const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ void gstore(T *p, T v) {
  *(__attribute__((address_space(1))) T *)p = v;
}
// Raw buffer access: a descriptor in scalar registers for a wave-uniform
// base address, then per access the lane's 32-bit byte offset and a scalar
// byte offset, so no per-lane 64-bit address arithmetic runs.  Every offset
// used with these stays far below the descriptor's 2^31 - 1 byte range.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, 0x7fffffff, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <typename T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
  } else {
    using U64 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U64, v), r, voff, soff, 0);
  }
}

// Generalized minmod G(a, b, theta = 1) (eq. gminmod): zero unless a and b
// have the same strict sign, else the one of smaller magnitude.  That value is
// the median of {0, a, b}: for equal signs the argument closer to zero, for
// opposite signs zero.  FP32: one v_med3_f32; FP64: min/max of the median.
__device__ __forceinline__ float minmod(float a, float b) { return __builtin_amdgcn_fmed3f(0.0f, a, b); }
__device__ __forceinline__ double minmod(double a, double b) {
  return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}

// FP64 reciprocal of a normal, finite x: the hardware estimate refined by
// two Newton-Raphson steps r <- r + r (1 - x r), each of which squares the
// relative error, so the result is within a few ulp of 1/x at about half the
// instructions of an IEEE division.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// sqrt(r) and 1/sqrt(r) of a positive, normal density: one reciprocal
// square root and s = r q.  FP64 refines the hardware estimate of 1/sqrt(r)
// by two Newton-Raphson steps q <- q + (q/2)(1 - r q^2), each of which about
// doubles the correct bits, so q and s are within a few ulp (the IEEE square
// root and a refined reciprocal of it cost about twice the instructions).
__device__ __forceinline__ void sqrt_and_rsq(float r, float &s, float &q) {
  q = __builtin_amdgcn_rsqf(r);
  s = r * q;
}
__device__ __forceinline__ void sqrt_and_rsq(double r, double &s, double &q) {
  double y = __builtin_amdgcn_rsq(r);
  double e = fma(-(r * y), y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-(r * y), y, 1.0);
  q = fma(0.5 * y, e, y);
  s = r * q;
}

// Reciprocal and square root: the hardware approximations (about 1 ulp) for
// FP32 states; for FP64 states the refined reciprocal (a few ulp) and IEEE
// square root.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return rcp_nr(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double fdiv(double a, double b) { return a * rcp_nr(b); }

// Primitive state (rho, v[0..NDIM-1], p) packed as NV = NDIM + 2 values.
// Conservative -> primitive (Sec. 3.5): v = m / rho, p = (gamma-1)(E - m.v/2).
template <typename T, int NDIM>
__device__ __forceinline__ void to_prim(const T *U, T gamma, T *W) {
  const T r = U[0];
  const T ir = frcp(r);
  T ke = T(0);
  W[0] = r;
#pragma unroll
  for (int d = 0; d < NDIM; d++) {
    const T v = U[1 + d] * ir;
    W[1 + d] = v;
    ke += U[1 + d] * v;
  }
  W[NDIM + 1] = (gamma - T(1)) * (U[NDIM + 1] - T(0.5) * ke);
}

// van Leer limiter (Sec. 3.2 limiter list): the harmonic mean 2ab/(a+b) of
// the one-sided slopes when their product is positive, else zero.
template <typename T>
__device__ __forceinline__ T vanleer(T a, T b) {
  const T ab = a * b;
  return ab > T(0) ? fdiv(T(2) * ab, a + b) : T(0);
}

// Slope of the reconstruction: LIM 0 minmod, 1 van Leer.
template <int LIM, typename T>
__device__ __forceinline__ T limit(T a, T b) {
  if constexpr (LIM == 1) return vanleer(a, b);
  else return minmod(a, b);
}

// Numerical flux (Sec. 3.2) along axis AX between reconstructed primitive
// states WL and WR from the Einfeldt speeds (Sec. 3.5): sqrt(rho)-weighted
// mean velocity u_bar and
// d_bar^2 = (sL cL^2 + sR cR^2)/(sL + sR) + sL sR/(2 (sL+sR)^2) (vR - vL)^2.
// Rusanov (HLL false): a = max(|u_bar - d_bar|, |u_bar + d_bar|) = |u_bar| + d_bar,
//   F = (FL+FR)/2 - a (UR-UL)/2.
// HLL: with s0 = min(u_bar - d_bar, 0), s1 = max(u_bar + d_bar, 0),
//   F = (s1 FL - s0 FR + s0 s1 (UR - UL)) / (s1 - s0), which is FL when every
//   signal moves right (s0 = 0), FR when every signal moves left (s1 = 0),
//   and the HLL intermediate-state flux otherwise.
// Both are evaluated as al UL + ar UR + wl PL + wr PR with the pressure terms
// P = (0, p e_AX, p v_AX) of each side.
template <typename T, int NDIM, int AX, bool HLL = false>
__device__ __forceinline__ void riemann(const T *WL, const T *WR, T gamma, T *F) {
  constexpr int NV = NDIM + 2;
  const T rl = WL[0], rr = WR[0];
  const T pl = WL[NV - 1], pr = WR[NV - 1];
  const T vl = WL[1 + AX], vr = WR[1 + AX];
  // wave speeds first, so the per-component flux needs few live registers;
  // with the weights w = sqrt(rho) / (sL + sR) of each side,
  // u_bar = wL vL + wR vR and d_bar^2 = gamma (pL / sL + pR / sR) / (sL + sR)
  // + wL wR dv^2 / 2 (s c^2 = gamma p / s = gamma p / sqrt(rho))
  T sl, sr, ql, qr;  // sqrt(rho) and 1 / sqrt(rho) of each side
  sqrt_and_rsq(rl, sl, ql);
  sqrt_and_rsq(rr, sr, qr);
  const T is = frcp(sl + sr);
  const T wlw = sl * is, wrw = sr * is;
  const T ubar = wlw * vl + wrw * vr;
  const T dv = vr - vl;
  const T d2 = gamma * (pl * ql + pr * qr) * is + (T(0.5) * wlw * wrw) * (dv * dv);
  const T db = fsqrt(d2);
  T al, ar, wl, wr;
  if constexpr (!HLL) {
    // max(|u_bar - d_bar|, |u_bar + d_bar|) with d_bar >= 0 is |u_bar| + d_bar,
    // bit for bit: the rounding of u_bar - d_bar and u_bar + d_bar is
    // symmetric in the sign of u_bar, so the larger magnitude is the
    // rounded |u_bar| + d_bar
    const T ha = T(0.5) * (fabs(ubar) + db);
    // (F_L + F_R)/2 - ha (U_R - U_L) with F = U v_n + pressure terms:
    // al = vl/2 + ha, ar = vr/2 - ha, both pressure weights 1/2
    al = T(0.5) * vl + ha;
    ar = T(0.5) * vr - ha;
    wl = wr = T(0.5);
  } else {
    const T m0 = ubar - db, m1 = ubar + db;
    const T s0 = m0 < T(0) ? m0 : T(0), s1 = m1 > T(0) ? m1 : T(0);
    const T iD = frcp(s1 - s0);
    wl = s1 * iD;
    wr = -s0 * iD;
    al = wl * (vl - s0);
    ar = wr * (vr - s1);
  }
  // With A = al rho_L and B = ar rho_R: mass A + B, momentum A v_L + B v_R
  // (plus the pressure weights on the normal component), and energy
  // al E_L + ar E_R + wl pL vL + wr pR vR with E = p / (gamma - 1) + rho |v|^2 / 2,
  // grouped as (A |v_L|^2 + B |v_R|^2) / 2 + pL (al / (gamma-1) + wl vL)
  // + pR (ar / (gamma-1) + wr vR)
  const T A = al * rl, B = ar * rr;
  F[0] = A + B;
  T ql2 = T(0), qr2 = T(0);
#pragma unroll
  for (int d = 0; d < NDIM; d++) {
    const T ul = WL[1 + d], ur = WR[1 + d];
    F[1 + d] = A * ul + B * ur;
    if (d == AX) F[1 + d] += wl * pl + wr * pr;
    ql2 += ul * ul;
    qr2 += ur * ur;
  }
  const T igm1 = frcp(gamma - T(1));
  const T cl = al * igm1 + wl * vl, cr = ar * igm1 + wr * vr;
  F[NV - 1] = T(0.5) * (A * ql2 + B * qr2) + (pl * cl + pr * cr);
}

// Scheme of a stage kernel, a bit mask: limiter (bit 0: van Leer, else
// minmod), flux (bit 1: HLL, else Rusanov), gravity source (bit 2).
constexpr int kSchVanLeer = 1, kSchHLL = 2, kSchGravity = 4, kNSchemes = 8;

// Face flux from four primitive states along the face normal: limited
// linear reconstruction (Sec. 3.2) W_L = W1 + s1/2, W_R = W2 - s2/2.
template <typename T, int NDIM, int AX, int SCH = 0>
__device__ __forceinline__ void face_flux(const T *W0, const T *W1, const T *W2, const T *W3, T gamma,
                                          T *F) {
  constexpr int NV = NDIM + 2;
  T L[NV], R[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) {
    const T s1 = limit<SCH & kSchVanLeer>(W1[v] - W0[v], W2[v] - W1[v]);
    const T s2 = limit<SCH & kSchVanLeer>(W2[v] - W1[v], W3[v] - W2[v]);
    L[v] = W1[v] + T(0.5) * s1;
    R[v] = W2[v] - T(0.5) * s2;
  }
  riemann<T, NDIM, AX, (SCH & kSchHLL) != 0>(L, R, gamma, F);
}

// Atomic max of a non-negative double through its bit pattern (IEEE order of
// non-negative doubles equals the order of their bit patterns).
__device__ __forceinline__ void atomic_max_pos(double *addr, double v) {
  __hip_atomic_fetch_max((__attribute__((address_space(1))) unsigned long long *)addr,
                         (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The same, skipped when the stored value is already at least v: a maximum
// that only grows during a launch is read at device scope first, so the
// thousands of waves of a launch do not all queue on one address (a stale
// read can only be smaller, which costs one unneeded atomic).  The result is
// the same maximum.
__device__ __forceinline__ void atomic_max_pos_if_larger(double *addr, double v) {
  const unsigned long long cur = __hip_atomic_load((__attribute__((address_space(1))) unsigned long long *)addr,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((unsigned long long)__double_as_longlong(v) > cur) atomic_max_pos(addr, v);
}

}  // namespace f4
