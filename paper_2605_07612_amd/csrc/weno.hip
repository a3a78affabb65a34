// WENO5 stage kernels (Sec. 3.2 limiter list: the fifth-order WENO
// reconstruction of Jiang and Shu, three ghost layers).  Every stencil cell
// lies in the block itself or in its face ghosts, which the ghost rounds fill
// (the stored ghosts of the plain form).
//
// 3-D blocks of 8^3 or 16^3 cells take the marching kernel: one workgroup per
// block, primitives converted once per cell, each face evaluated once (x- and
// y-faces shared through LDS, z-faces through a register window).  Other
// shapes take the per-cell kernel: one thread per interior cell converts the
// seven cells of its line along each axis and evaluates both faces of its
// cell, so every face is evaluated twice.  The update, the refinement-face
// flux capture, the gravity source and the CFL epilogue follow the
// plane-marching stage kernel: stage 1 / 2 Heun's stages, 3 the generic
// sub-step, 4 the generic sub-step with three earlier states.  The
// reconstruction carries ~3x the arithmetic of the MUSCL one, so both are
// bound by their VALU work.
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

// FP64: the same weights with one (refined) reciprocal.  Numerator and denominator of
// sum(alpha_k q_k) / sum(alpha_k) are multiplied by the product of the three
// (eps + beta_k)^2, so alpha_k becomes d_k times the other two squares; the
// products stay finite for beta_k below ~1e75.
template <>
__device__ __forceinline__ double weno5<double>(double v0, double v1, double v2, double v3, double v4) {
  const double s6 = 1.0 / 6.0;
  const double q0 = (2.0 * v0 - 7.0 * v1 + 11.0 * v2) * s6;
  const double q1 = (-v1 + 5.0 * v2 + 2.0 * v3) * s6;
  const double q2 = (2.0 * v2 + 5.0 * v3 - v4) * s6;
  const double c13 = 13.0 / 12.0, c14 = 0.25;
  double a = v0 - 2.0 * v1 + v2, b = v0 - 4.0 * v1 + 3.0 * v2;
  const double b0 = c13 * a * a + c14 * b * b;
  a = v1 - 2.0 * v2 + v3;
  b = v1 - v3;
  const double b1 = c13 * a * a + c14 * b * b;
  a = v2 - 2.0 * v3 + v4;
  b = 3.0 * v2 - 4.0 * v3 + v4;
  const double b2 = c13 * a * a + c14 * b * b;
  const double e0 = 1e-6 + b0, e1 = 1e-6 + b1, e2 = 1e-6 + b2;
  const double E0 = e0 * e0, E1 = e1 * e1, E2 = e2 * e2;
  const double a0 = 0.1 * (E1 * E2), a1 = 0.6 * (E0 * E2), a2 = 0.3 * (E0 * E1);
  return (a0 * q0 + a1 * q1 + a2 * q2) * rcp_nr(a0 + a1 + a2);
}

// Flux along AX through the face between cells 2 and 3 of the six primitive
// states c[0..5] (cells f-3 .. f+2 of face f-1/2): left state reconstructed
// from c[0..4], right state from c[5..1].
template <typename T, int NDIM, int AX, int SCH>
__device__ __forceinline__ void weno_face(const T (*c)[NDIM + 2], T gamma, T *F) {
  constexpr int NV = NDIM + 2;
  T L[NV], R[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) {
    L[v] = weno5(c[0][v], c[1][v], c[2][v], c[3][v], c[4][v]);
    R[v] = weno5(c[5][v], c[4][v], c[3][v], c[2][v], c[1][v]);
  }
  riemann<T, NDIM, AX, (SCH & kSchHLL) != 0>(L, R, gamma, F);
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
  weno_face<T, NDIM, AX, SCH>(W, gamma, Fm);
  weno_face<T, NDIM, AX, SCH>(W + 1, gamma, Fp);
}

// Update of cell c (offset o in the block) from its flux divergence: the
// stage's base state, the gravity source, and for the last (sub-)step the
// maximum of vmax and the cell's CFL limit, except next to F2C faces, whose
// cells the flux fix finishes.
template <typename T, int NDIM, int SCH, int STG>
__device__ __forceinline__ void weno_update(const MeshDev &M, const SubStep &ss, int64_t boff, int64_t sv,
                                            const T *ud, const T *up, T *uo, int o, const int c[3], const T *div,
                                            T dts, T idx, double dx, const int *finfo, double &vmax, bool &bad) {
  constexpr int NV = NDIM + 2;
  constexpr int stage = STG;
  const int N = M.N;
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
      const T *up2 = (const T *)M.s[role_buffer(ss.prev2, M.cur)] + boff;
      const T *up3 = (const T *)M.s[role_buffer(ss.prev3, M.cur)] + boff;
      base = (((T)ss.wp * Up[v] + (T)ss.wp2 * gload(up2 + v * sv + o)) + (T)ss.wp3 * gload(up3 + v * sv + o)) +
             (T)ss.wd * U0[v];
    }
    if constexpr ((SCH & kSchGravity) != 0) Uout[v] = (base + dts * src[v]) - cdt * div[v];
    else Uout[v] = base - cdt * div[v];
    gstore(uo + v * sv + o, Uout[v]);
  }
  if (stage == 2 || (stage >= 3 && ss.epi)) {
    auto is_f2c = [&](int f) { return finfo[f] >= 0 && (finfo[f] & 1); };
    bool skip = (is_f2c(0) && c[0] == 0) || (is_f2c(1) && c[0] == N - 1) || (is_f2c(2) && c[1] == 0) ||
                (is_f2c(3) && c[1] == N - 1);
    if constexpr (NDIM == 3) skip = skip || (is_f2c(4) && c[2] == 0) || (is_f2c(5) && c[2] == N - 1);
    if (!skip) {
      double s;
      if constexpr (sizeof(T) == 8) s = cell_inv_dt<NDIM>((const double *)Uout, M.gamma, dx, bad);
      else s = cell_inv_dt<NDIM>((const float *)Uout, (float)M.gamma, (float)idx, bad);
      vmax = fmax(vmax, s);
    }
  }
}

// Refinement-face flux F of face f of block b at in-face position (t1, t2),
// in the layout of the plane-marching stage kernel.
template <typename T, int NDIM>
__device__ __forceinline__ void weno_bflux(const MeshDev &M, const int *finfo, int f, int t1, int t2, const T *F) {
  constexpr int NV = NDIM + 2;
  const int info = finfo[f];
  if (info < 0) return;
  const int N = M.N;
  T *buf = (T *)((info & 1) ? M.bflux_c : M.bflux_f);
  const int64_t slot = info >> 1;
#pragma unroll
  for (int v = 0; v < NV; v++) {
    const int64_t o = (NDIM == 3) ? ((slot * NV + v) * N + t2) * N + t1 : (slot * NV + v) * N + t1;
    gstore(buf + o, F[v]);
  }
}

// Per-block constants of one stage: source, output and previous-state
// blocks, the step fraction and the inverse cell width.
template <typename T, int NDIM, int STG>
struct WenoBlock {
  const T *ud, *up;
  T *uo;
  int64_t boff;
  double dx;
  T idx, dts;
  int finfo[2 * NDIM];
  __device__ __forceinline__ WenoBlock(const MeshDev &M, const SubStep &ss, int64_t b, int64_t bel) {
    constexpr int stage = STG;
    const int cur = M.cur;
    boff = b * bel;
    ud = (const T *)M.s[stage >= 3 ? role_buffer(ss.deriv, cur) : (stage == 1 ? cur : 1 - cur)] + boff;
    uo = (T *)M.s[stage >= 3 ? role_buffer(ss.out, cur) : (stage == 1 ? 1 - cur : cur)] + boff;
    up = (const T *)M.s[stage >= 3 ? role_buffer(ss.prev, cur) : cur] + boff;
    dx = ldexp(M.dx0, -gload(M.level + b));
    idx = (T)(1.0 / dx);
    const double dt = gload(M.scal + kDt);
    dts = (T)(stage >= 3 ? ss.c * dt : (stage == 1 ? dt : 0.5 * dt));
#pragma unroll
    for (int f = 0; f < 2 * NDIM; f++) finfo[f] = gload(M.face_info + b * 2 * NDIM + f);
  }
};

// One thread per interior cell, any block size and dimension.
template <typename T, int NDIM, int SCH, int STG>
__global__ __launch_bounds__(256) void weno_stage_kernel(const MeshDev *__restrict__ Mp, int64_t total, SubStep ss) {
  const MeshDev &M = *Mp;
  constexpr int NV = NDIM + 2;
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
    const WenoBlock<T, NDIM, STG> B(M, ss, b, bel);
    const T gamma = (T)M.gamma;
    T div[NV], Fm[NV], Fp[NV];
    weno_axis<T, NDIM, 0, SCH>(B.ud, sv, N, g, c, gamma, Fm, Fp);
#pragma unroll
    for (int v = 0; v < NV; v++) div[v] = Fp[v] - Fm[v];
    if (c[0] == 0) weno_bflux<T, NDIM>(M, B.finfo, 0, c[1], c[2], Fm);
    if (c[0] == N - 1) weno_bflux<T, NDIM>(M, B.finfo, 1, c[1], c[2], Fp);
    weno_axis<T, NDIM, 1, SCH>(B.ud, sv, N, g, c, gamma, Fm, Fp);
#pragma unroll
    for (int v = 0; v < NV; v++) div[v] += Fp[v] - Fm[v];
    if (c[1] == 0) weno_bflux<T, NDIM>(M, B.finfo, 2, c[0], c[2], Fm);
    if (c[1] == N - 1) weno_bflux<T, NDIM>(M, B.finfo, 3, c[0], c[2], Fp);
    if constexpr (NDIM == 3) {
      weno_axis<T, NDIM, 2, SCH>(B.ud, sv, N, g, c, gamma, Fm, Fp);
#pragma unroll
      for (int v = 0; v < NV; v++) div[v] += Fp[v] - Fm[v];
      if (c[2] == 0) weno_bflux<T, NDIM>(M, B.finfo, 4, c[0], c[1], Fm);
      if (c[2] == N - 1) weno_bflux<T, NDIM>(M, B.finfo, 5, c[0], c[1], Fp);
    }
    const int o = cell_off<NDIM>(c[0], c[1], c[2], N, g);
    weno_update<T, NDIM, SCH, STG>(M, ss, B.boff, sv, B.ud, B.up, B.uo, o, c, div, B.dts, B.idx, B.dx, B.finfo, vmax,
                                   bad);
  }
  if (STG == 2 || (STG >= 3 && ss.epi)) flush_dt(M, vmax, bad);
}

// LDS elements of the marching kernel for block size N: one primitive plane
// with three halo cells a side, and the x- and y-face fluxes of one plane.
__host__ __device__ constexpr int weno_march_lds(int N) { return 5 * ((N + 6) * (N + 6) + 2 * N * (N + 1)); }

// 3-D blocks with N * N a multiple of 64 and at most 256 (N = 8, 16): one
// workgroup per block, thread (i, j) owns column (i, j) and marches it in z.
// Each plane's primitives (with their x and y halos, read from the block's
// stored ghosts) are staged in LDS once; every x- and y-face of the plane is
// evaluated once into LDS and read by the two cells that share it; the
// z-faces come from a seven-cell register window of the column, the upper
// face of one plane being the lower face of the next.  Per plane that is
// 2N(N+1) + N^2 face evaluations instead of the per-cell kernel's 6 N^2;
// the x- and y-faces share one loop, so its last round is the only partial one.
template <typename T, int SCH, int STG>
__global__ __launch_bounds__(256) void weno_march_kernel(const MeshDev *__restrict__ Mp, SubStep ss) {
  constexpr int NV = 5;
  extern __shared__ __align__(16) unsigned char weno_lds[];
  const MeshDev &M = *Mp;
  const int N = M.N, g = M.g, P = N + 2 * g, Q = N + 6;
  const int64_t sv = (int64_t)P * P * P, bel = sv * NV;
  const int64_t b = blockIdx.x;
  const int t = threadIdx.x, nt = N * N;
  const int i = t % N, j = t / N;
  T *Ws = (T *)weno_lds;               // [NV][Q][Q], cell (x, y) at column x + 3, row y + 3
  T *Fx = Ws + NV * Q * Q;             // [NV][N][N + 1]: face fi - 1/2 of row fj
  T *Fy = Fx + NV * N * (N + 1);       // [NV][N + 1][N]: face fj - 1/2 of column fi
  const WenoBlock<T, 3, STG> B(M, ss, b, bel);
  const T gamma = (T)M.gamma;
  auto load_prim = [&](int x, int y, int z, T *W) {
    const int o = cell_off<3>(x, y, z, N, g);
    T U[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) U[v] = gload(B.ud + v * sv + o);
    to_prim<T, 3>(U, gamma, W);
  };
  double vmax = 0.0;
  bool bad = false;
  T w[7][NV];  // column cells k-3 .. k+3
#pragma unroll
  for (int s = 1; s < 7; s++) load_prim(i, j, s - 4, w[s]);
  T Fzm[NV];
  for (int k = 0; k < N; k++) {
#pragma unroll
    for (int s = 0; s < 6; s++)
#pragma unroll
      for (int v = 0; v < NV; v++) w[s][v] = w[s + 1][v];
    load_prim(i, j, k + 3, w[6]);
    if (k == 0) {
      weno_face<T, 3, 2, SCH>(w, gamma, Fzm);
      weno_bflux<T, 3>(M, B.finfo, 4, i, j, Fzm);
    }
    __syncthreads();  // the previous plane's LDS readers are done
#pragma unroll
    for (int v = 0; v < NV; v++) Ws[(v * Q + j + 3) * Q + i + 3] = w[3][v];
    for (int h = t; h < 12 * N; h += nt) {  // halo strips x-, x+, y-, y+, each 3 deep
      const int strip = h / (3 * N), r = h % (3 * N), d = r / N, e = r % N;
      const int x = strip == 0 ? d - 3 : strip == 1 ? N + d : e;
      const int y = strip == 2 ? d - 3 : strip == 3 ? N + d : e;
      T W[NV];
      load_prim(x, y, k, W);
#pragma unroll
      for (int v = 0; v < NV; v++) Ws[(v * Q + y + 3) * Q + x + 3] = W[v];
    }
    __syncthreads();
    // x- and y-faces in one loop of uniform work: a y-face's primitives are
    // read with the first two velocity components swapped, so every face
    // evaluates the x-normal flux, and its momentum fluxes are swapped back.
    const int nxf = (N + 1) * N;
    for (int f = t; f < 2 * nxf; f += nt) {
      const bool ya = f >= nxf;
      const int ff = ya ? f - nxf : f;
      const int fi = ya ? ff % N : ff % (N + 1), fj = ya ? ff / N : ff / (N + 1);
      const int base = ya ? fj * Q + fi + 3 : (fj + 3) * Q + fi;  // stencil cell 0, variable 0
      const int step = ya ? Q : 1;
      T c6[6][NV], F[NV];
#pragma unroll
      for (int s = 0; s < 6; s++)
#pragma unroll
        for (int v = 0; v < NV; v++) {
          const int vv = (v == 1 || v == 2) && ya ? 3 - v : v;
          c6[s][v] = Ws[vv * Q * Q + base + s * step];
        }
      weno_face<T, 3, 0, SCH>(c6, gamma, F);
      if (!ya) {
#pragma unroll
        for (int v = 0; v < NV; v++) Fx[(v * N + fj) * (N + 1) + fi] = F[v];
        if (fi == 0) weno_bflux<T, 3>(M, B.finfo, 0, fj, k, F);
        if (fi == N) weno_bflux<T, 3>(M, B.finfo, 1, fj, k, F);
      } else {
        const T f1 = F[1];
        F[1] = F[2];
        F[2] = f1;
#pragma unroll
        for (int v = 0; v < NV; v++) Fy[(v * (N + 1) + fj) * N + fi] = F[v];
        if (fj == 0) weno_bflux<T, 3>(M, B.finfo, 2, fi, k, F);
        if (fj == N) weno_bflux<T, 3>(M, B.finfo, 3, fi, k, F);
      }
    }
    T Fzp[NV];
    weno_face<T, 3, 2, SCH>(w + 1, gamma, Fzp);
    if (k == N - 1) weno_bflux<T, 3>(M, B.finfo, 5, i, j, Fzp);
    __syncthreads();
    T div[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) div[v] = Fx[(v * N + j) * (N + 1) + i + 1] - Fx[(v * N + j) * (N + 1) + i];
#pragma unroll
    for (int v = 0; v < NV; v++) div[v] += Fy[(v * (N + 1) + j + 1) * N + i] - Fy[(v * (N + 1) + j) * N + i];
#pragma unroll
    for (int v = 0; v < NV; v++) {
      div[v] += Fzp[v] - Fzm[v];
      Fzm[v] = Fzp[v];
    }
    const int c[3] = {i, j, k};
    weno_update<T, 3, SCH, STG>(M, ss, B.boff, sv, B.ud, B.up, B.uo, cell_off<3>(i, j, k, N, g), c, div, B.dts, B.idx,
                                B.dx, B.finfo, vmax, bad);
  }
  if (STG == 2 || (STG >= 3 && ss.epi)) flush_dt(M, vmax, bad);
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

template <typename T, int SCH>
static void launch_march_t(unsigned nblocks, int N, const MeshDev *d, int stage, const SubStep &ss, hipStream_t s) {
  const unsigned nt = (unsigned)(N * N);
  const size_t lds = sizeof(T) * (size_t)weno_march_lds(N);
  switch (stage) {
    case 1: weno_march_kernel<T, SCH, 1><<<nblocks, nt, lds, s>>>(d, ss); break;
    case 2: weno_march_kernel<T, SCH, 2><<<nblocks, nt, lds, s>>>(d, ss); break;
    case 3: weno_march_kernel<T, SCH, 3><<<nblocks, nt, lds, s>>>(d, ss); break;
    default: weno_march_kernel<T, SCH, 4><<<nblocks, nt, lds, s>>>(d, ss); break;
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

template <typename T>
static void launch_march(unsigned nblocks, int N, const MeshDev *d, int stage, int scheme, const SubStep &ss,
                         hipStream_t s) {
  switch (scheme & (kSchHLL | kSchGravity)) {
    case 0: launch_march_t<T, 0>(nblocks, N, d, stage, ss, s); break;
    case kSchHLL: launch_march_t<T, kSchHLL>(nblocks, N, d, stage, ss, s); break;
    case kSchGravity: launch_march_t<T, kSchGravity>(nblocks, N, d, stage, ss, s); break;
    default: launch_march_t<T, kSchHLL | kSchGravity>(nblocks, N, d, stage, ss, s); break;
  }
}

hipError_t launch_weno_stage(const MeshDev *d_mesh, int64_t nblocks, int block_n, int stage, int ndim, bool f64,
                             int scheme, hipStream_t s, const SubStep &ss) {
  if (nblocks <= 0) return hipSuccess;
  if (ndim == 3 && (block_n == 8 || block_n == 16)) {
    if (f64) launch_march<double>((unsigned)nblocks, block_n, d_mesh, stage, scheme, ss, s);
    else launch_march<float>((unsigned)nblocks, block_n, d_mesh, stage, scheme, ss, s);
    return hipGetLastError();
  }
  const int64_t cells = nblocks * block_n * block_n * (ndim == 3 ? block_n : 1);
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
