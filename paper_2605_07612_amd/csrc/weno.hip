// WENO5 stage kernel (Sec. 3.2 limiter list: the fifth-order WENO
// reconstruction of Jiang and Shu, three ghost layers).
//
// One thread per interior cell.  Along each axis the thread converts the
// seven cells i-3 .. i+3 of its line to primitive variables, reconstructs
// the left and right states of its -face (cells i-3 .. i+2) and of its +face
// (cells i-2 .. i+3), and evaluates both face fluxes; the neighbouring cell
// evaluates the shared face again.  Every stencil cell lies in the block
// itself or in its face ghosts, which the ghost rounds fill (the plain form's
// stored ghosts), so no halo staging is needed.  The update, the refinement-
// face flux capture, the gravity source and the CFL epilogue follow the
// plane-marching stage kernel: stage 1 / 2 Heun's stages, 3 the generic
// sub-step, 4 the generic sub-step with three earlier states.  The
// reconstruction carries ~3x the arithmetic of the MUSCL one and each face is
// evaluated twice, so this kernel is bound by its VALU work.
#include "device_common.h"
#include "foap4_internal.h"
#include "stage_common.h"

namespace f4 {

// Value at the right face of cell 2 of v0 .. v4 (cells i-2 .. i+2): the
// convex combination of the three third-order candidates with weights
// alpha_k / sum alpha, alpha_k = d_k / (eps + beta_k)^2, d = (1, 6, 3)/10,
// eps = 1e-6, beta_k the candidates' smoothness indicators.
template <typename T>
__device__ __forceinline__ T weno5(T v0, T v1, T v2, T v3, T v4) {
  const T s6 = T(1) / T(6);
  const T q0 = (T(2) * v0 - T(7) * v1 + T(11) * v2) * s6;
  const T q1 = (-v1 + T(5) * v2 + T(2) * v3) * s6;
  const T q2 = (T(2) * v2 + T(5) * v3 - v4) * s6;
  const T c13 = T(13) / T(12), c14 = T(0.25);
  T a = v0 - T(2) * v1 + v2, b = v0 - T(4) * v1 + T(3) * v2;
  const T b0 = c13 * a * a + c14 * b * b;
  a = v1 - T(2) * v2 + v3;
  b = v1 - v3;
  const T b1 = c13 * a * a + c14 * b * b;
  a = v2 - T(2) * v3 + v4;
  b = T(3) * v2 - T(4) * v3 + v4;
  const T b2 = c13 * a * a + c14 * b * b;
  const T eps = T(1e-6);
  const T e0 = eps + b0, e1 = eps + b1, e2 = eps + b2;
  const T a0 = fdiv(T(0.1), e0 * e0), a1 = fdiv(T(0.6), e1 * e1), a2 = fdiv(T(0.3), e2 * e2);
  return fdiv(a0 * q0 + a1 * q1 + a2 * q2, a0 + a1 + a2);
}

// Fluxes of the -face (Fm) and +face (Fp) of cell c of block data u along AX.
template <typename T, int NDIM, int AX, int SCH>
__device__ __forceinline__ void weno_axis(const T *u, int64_t sv, int N, int g, const int c[3], T gamma, T *Fm,
                                          T *Fp) {
  constexpr int NV = NDIM + 2;
  T W[7][NV];
#pragma unroll
  for (int s = 0; s < 7; s++) {
    int q[3] = {c[0], c[1], c[2]};
    q[AX] += s - 3;
    const int o = cell_off<NDIM>(q[0], q[1], q[2], N, g);
    T U[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) U[v] = gload(u + v * sv + o);
    to_prim<T, NDIM>(U, gamma, W[s]);
  }
  T L[NV], R[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) {
    L[v] = weno5(W[0][v], W[1][v], W[2][v], W[3][v], W[4][v]);
    R[v] = weno5(W[5][v], W[4][v], W[3][v], W[2][v], W[1][v]);
  }
  riemann<T, NDIM, AX, (SCH & kSchHLL) != 0>(L, R, gamma, Fm);
#pragma unroll
  for (int v = 0; v < NV; v++) {
    L[v] = weno5(W[1][v], W[2][v], W[3][v], W[4][v], W[5][v]);
    R[v] = weno5(W[6][v], W[5][v], W[4][v], W[3][v], W[2][v]);
  }
  riemann<T, NDIM, AX, (SCH & kSchHLL) != 0>(L, R, gamma, Fp);
}

template <typename T, int NDIM, int SCH, int STG>
__global__ __launch_bounds__(256) void weno_stage_kernel(const MeshDev *__restrict__ Mp, int64_t total, SubStep ss) {
  const MeshDev &M = *Mp;
  constexpr int NV = NDIM + 2, NF = 2 * NDIM;
  constexpr int stage = STG;
  const int N = M.N, g = M.g, P = N + 2 * g;
  const int64_t sv = (NDIM == 3) ? (int64_t)P * P * P : (int64_t)P * P;
  const int64_t bel = sv * NV;
  const int64_t cpb = (NDIM == 3) ? (int64_t)N * N * N : (int64_t)N * N;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double vmax = 0.0;
  bool bad = false;
  if (id < total) {
    const int64_t b = id / cpb;
    const int cc = (int)(id % cpb);
    const int c[3] = {cc % N, (cc / N) % N, (NDIM == 3) ? cc / (N * N) : 0};
    const int cur = M.cur;
    const T *ud = (const T *)M.s[stage >= 3 ? role_buffer(ss.deriv, cur) : (stage == 1 ? cur : 1 - cur)] + b * bel;
    T *uo = (T *)M.s[stage >= 3 ? role_buffer(ss.out, cur) : (stage == 1 ? 1 - cur : cur)] + b * bel;
    const T *up = (const T *)M.s[stage >= 3 ? role_buffer(ss.prev, cur) : cur] + b * bel;
    const T gamma = (T)M.gamma;
    const double dx = ldexp(M.dx0, -gload(M.level + b));
    const T idx = (T)(1.0 / dx);
    const double dt = gload(M.scal + kDt);
    const T dts = (T)(stage >= 3 ? ss.c * dt : (stage == 1 ? dt : 0.5 * dt));
    int finfo[NF];
#pragma unroll
    for (int f = 0; f < NF; f++) finfo[f] = gload(M.face_info + b * NF + f);
    // refinement-face fluxes, in the layout of the plane-marching kernel
    auto store_bflux = [&](int f, int t1, int t2, const T *F) {
      const int info = finfo[f];
      if (info < 0) return;
      T *buf = (T *)((info & 1) ? M.bflux_c : M.bflux_f);
      const int64_t slot = info >> 1;
#pragma unroll
      for (int v = 0; v < NV; v++) {
        const int64_t o = (NDIM == 3) ? ((slot * NV + v) * N + t2) * N + t1 : (slot * NV + v) * N + t1;
        gstore(buf + o, F[v]);
      }
    };
    T div[NV], Fm[NV], Fp[NV];
    weno_axis<T, NDIM, 0, SCH>(ud, sv, N, g, c, gamma, Fm, Fp);
#pragma unroll
    for (int v = 0; v < NV; v++) div[v] = Fp[v] - Fm[v];
    if (c[0] == 0) store_bflux(0, c[1], c[2], Fm);
    if (c[0] == N - 1) store_bflux(1, c[1], c[2], Fp);
    weno_axis<T, NDIM, 1, SCH>(ud, sv, N, g, c, gamma, Fm, Fp);
#pragma unroll
    for (int v = 0; v < NV; v++) div[v] += Fp[v] - Fm[v];
    if (c[1] == 0) store_bflux(2, c[0], c[2], Fm);
    if (c[1] == N - 1) store_bflux(3, c[0], c[2], Fp);
    if constexpr (NDIM == 3) {
      weno_axis<T, NDIM, 2, SCH>(ud, sv, N, g, c, gamma, Fm, Fp);
#pragma unroll
      for (int v = 0; v < NV; v++) div[v] += Fp[v] - Fm[v];
      if (c[2] == 0) store_bflux(4, c[0], c[1], Fm);
      if (c[2] == N - 1) store_bflux(5, c[0], c[1], Fp);
    }
    const int o = cell_off<NDIM>(c[0], c[1], c[2], N, g);
    T U0[NV], Up[NV], Uout[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
      U0[v] = gload(ud + v * sv + o);
      Up[v] = (stage >= 2) ? gload(up + v * sv + o) : T(0);
    }
    [[maybe_unused]] T src[NV];
    if constexpr ((SCH & kSchGravity) != 0) {
      T gm = T(0);
      src[0] = T(0);
#pragma unroll
      for (int d = 0; d < NDIM; d++) {
        src[1 + d] = U0[0] * (T)M.grav[d];
        gm += (T)M.grav[d] * U0[1 + d];
      }
      src[NV - 1] = gm;
    }
    const T cdt = dts * idx;
#pragma unroll
    for (int v = 0; v < NV; v++) {
      T base;
      if (stage == 1) base = U0[v];
      else if (stage == 2) base = T(0.5) * (Up[v] + U0[v]);
      else if (stage == 3) base = (T)ss.wp * Up[v] + (T)ss.wd * U0[v];
      else {
        const T *up2 = (const T *)M.s[role_buffer(ss.prev2, cur)] + b * bel;
        const T *up3 = (const T *)M.s[role_buffer(ss.prev3, cur)] + b * bel;
        base = (((T)ss.wp * Up[v] + (T)ss.wp2 * gload(up2 + v * sv + o)) + (T)ss.wp3 * gload(up3 + v * sv + o)) +
               (T)ss.wd * U0[v];
      }
      if constexpr ((SCH & kSchGravity) != 0) Uout[v] = (base + dts * src[v]) - cdt * div[v];
      else Uout[v] = base - cdt * div[v];
      gstore(uo + v * sv + o, Uout[v]);
    }
    if (stage == 2 || (stage >= 3 && ss.epi)) {
      // cells next to F2C faces are finished (and their dt taken) by the flux fix
      auto is_f2c = [&](int f) { return finfo[f] >= 0 && (finfo[f] & 1); };
      bool skip = (is_f2c(0) && c[0] == 0) || (is_f2c(1) && c[0] == N - 1) || (is_f2c(2) && c[1] == 0) ||
                  (is_f2c(3) && c[1] == N - 1);
      if constexpr (NDIM == 3) skip = skip || (is_f2c(4) && c[2] == 0) || (is_f2c(5) && c[2] == N - 1);
      if (!skip) {
        if constexpr (sizeof(T) == 8) vmax = cell_inv_dt<NDIM>((const double *)Uout, M.gamma, dx, bad);
        else vmax = cell_inv_dt<NDIM>((const float *)Uout, (float)gamma, (float)idx, bad);
      }
    }
  }
  if (stage == 2 || (stage >= 3 && ss.epi)) flush_dt(M, vmax, bad);
}

template <typename T, int NDIM, int SCH>
static void launch_weno_t(unsigned nblk, const MeshDev *d, int64_t total, int stage, const SubStep &ss, hipStream_t s) {
  switch (stage) {
    case 1: weno_stage_kernel<T, NDIM, SCH, 1><<<nblk, 256, 0, s>>>(d, total, ss); break;
    case 2: weno_stage_kernel<T, NDIM, SCH, 2><<<nblk, 256, 0, s>>>(d, total, ss); break;
    case 3: weno_stage_kernel<T, NDIM, SCH, 3><<<nblk, 256, 0, s>>>(d, total, ss); break;
    default: weno_stage_kernel<T, NDIM, SCH, 4><<<nblk, 256, 0, s>>>(d, total, ss); break;
  }
}

template <typename T, int NDIM>
static void launch_weno_nd(unsigned nblk, const MeshDev *d, int64_t total, int stage, int scheme, const SubStep &ss,
                           hipStream_t s) {
  switch (scheme & (kSchHLL | kSchGravity)) {
    case 0: launch_weno_t<T, NDIM, 0>(nblk, d, total, stage, ss, s); break;
    case kSchHLL: launch_weno_t<T, NDIM, kSchHLL>(nblk, d, total, stage, ss, s); break;
    case kSchGravity: launch_weno_t<T, NDIM, kSchGravity>(nblk, d, total, stage, ss, s); break;
    default: launch_weno_t<T, NDIM, kSchHLL | kSchGravity>(nblk, d, total, stage, ss, s); break;
  }
}

hipError_t launch_weno_stage(const MeshDev *d_mesh, int64_t cells, int stage, int ndim, bool f64, int scheme,
                             hipStream_t s, const SubStep &ss) {
  if (cells <= 0) return hipSuccess;
  const unsigned nblk = (unsigned)((cells + 255) / 256);
  if (f64) {
    if (ndim == 3) launch_weno_nd<double, 3>(nblk, d_mesh, cells, stage, scheme, ss, s);
    else launch_weno_nd<double, 2>(nblk, d_mesh, cells, stage, scheme, ss, s);
  } else {
    if (ndim == 3) launch_weno_nd<float, 3>(nblk, d_mesh, cells, stage, scheme, ss, s);
    else launch_weno_nd<float, 2>(nblk, d_mesh, cells, stage, scheme, ss, s);
  }
  return hipGetLastError();
}

}  // namespace f4
