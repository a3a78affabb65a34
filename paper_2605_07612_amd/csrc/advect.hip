// Stage kernel of scalar advection (Sec. 3.4): one conserved variable rho
// carried by a uniform velocity v, rho_t + div(rho v) = 0.  The face values
// come from the mesh's reconstruction (minmod or van Leer MUSCL, WENO5), the
// physical flux on either side of a face is rho v_d, and the numerical flux
// (Rusanov or HLL) takes the wave speeds min(v_d, 0) and max(v_d, 0).
//
// One workgroup per block and one thread per (i, j) column, which marches
// along k.  Per plane the workgroup stages the plane with its x and y face
// ghosts in LDS (the interior from the threads' own z windows, the ghosts
// from the block's stored ghost cells, filled by the ghost rounds), double
// buffered so that one barrier per plane suffices; every thread then
// evaluates the two x faces and two y faces of its cell from LDS and the
// upper z face from its register window of the column (the lower one is the
// upper face of the previous plane).  The update, the refinement-face flux
// capture and the CFL epilogue follow the Euler stage kernels: stage 1 / 2
// Heun's stages, 3 the generic sub-step, 4 the generic sub-step with three
// earlier states.  With a single variable the work per cell is small, so the
// kernel is bound by its HBM traffic: the state is read once per stage (plus
// the face ghosts, and Heun's second stage reads U^n) and written once.
#include "device_common.h"
#include "foap4_internal.h"

namespace f4 {

// Reconstruction of an advection stage: LIM 0 minmod, 1 van Leer, 2 WENO5.
// R = cells on either side of a face that the stencil reaches.
template <int LIM>
struct AdvStencil {
  static constexpr int R = (LIM == 2) ? 3 : 2;
};

// Value at the right face of cell c2 of c0 .. c4 (WENO5 of Jiang and Shu,
// eps 1e-6, ideal weights 1/10, 6/10, 3/10).
template <typename T>
__device__ __forceinline__ T adv_weno5(T v0, T v1, T v2, T v3, T v4) {
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
  const T e0 = T(1e-6) + b0, e1 = T(1e-6) + b1, e2 = T(1e-6) + b2;
  const T a0 = fdiv(T(0.1), e0 * e0), a1 = fdiv(T(0.6), e1 * e1), a2 = fdiv(T(0.3), e2 * e2);
  return fdiv(a0 * q0 + a1 * q1 + a2 * q2, a0 + a1 + a2);
}

// Numerical flux through the face between cells w[R-1] and w[R] of the 2R
// cells w[0 .. 2R-1] along the face normal, velocity component v.
// Rusanov: (v L + v R)/2 - |v| (R - L)/2 (the largest of |min(v, 0)| and
// |max(v, 0)| is |v|).  HLL with s0 = min(v, 0), s1 = max(v, 0): the left
// flux v L when s0 >= 0, else (s1 = 0) the right flux v R.
template <typename T, int LIM, bool HLL>
__device__ __forceinline__ T adv_flux(const T *w, T v) {
  T L, R;
  if constexpr (LIM == 2) {
    L = adv_weno5(w[0], w[1], w[2], w[3], w[4]);
    R = adv_weno5(w[5], w[4], w[3], w[2], w[1]);
  } else {
    const T s1 = limit<LIM>(w[1] - w[0], w[2] - w[1]);
    const T s2 = limit<LIM>(w[2] - w[1], w[3] - w[2]);
    L = w[1] + T(0.5) * s1;
    R = w[2] - T(0.5) * s2;
  }
  if constexpr (HLL) return v >= T(0) ? L * v : R * v;
  else return T(0.5) * (L * v + R * v) - T(0.5) * fabs(v) * (R - L);
}

// Stores the refinement-face flux F of face f at in-face position (t1, t2)
// (layout [slot][t2][t1], one variable).
template <typename T, int NDIM>
__device__ __forceinline__ void adv_bflux(const MeshDev &M, int info, int t1, int t2, T F) {
  if (info < 0) return;
  const int N = M.N;
  T *buf = (T *)((info & 1) ? M.bflux_c : M.bflux_f);
  const int64_t slot = info >> 1;
  const int64_t o = (NDIM == 3) ? (slot * N + t2) * N + t1 : slot * N + t1;
  gstore(buf + o, F);
}

// LDS elements: two planes of (N + 2g)^2 cells.
__host__ __device__ constexpr int adv_lds(int N, int g) { return 2 * (N + 2 * g) * (N + 2 * g); }

template <typename T, int NDIM, int LIM, bool HLL, int STG>
__global__ __launch_bounds__(1024) void advect_kernel(const MeshDev *__restrict__ Mp, SubStep ss) {
  constexpr int R = AdvStencil<LIM>::R;
  extern __shared__ __align__(16) unsigned char adv_smem[];
  const MeshDev &M = *Mp;
  const int N = M.N, g = M.g, P = N + 2 * g, Q = P;
  const int rows = (NDIM == 3) ? P * P : P;  // rows (k, j) of the row part of a block
  const int64_t sv = (NDIM == 3) ? (int64_t)P * P * P : (int64_t)P * P;
  const int64_t b = blockIdx.x;
  const int t = threadIdx.x, i = t % N, j = t / N;
  const int cur = M.cur;
  const int64_t boff = b * sv;
  const T *ud = (const T *)M.s[STG >= 3 ? role_buffer(ss.deriv, cur) : (STG == 1 ? cur : 1 - cur)] + boff;
  T *uo = (T *)M.s[STG >= 3 ? role_buffer(ss.out, cur) : (STG == 1 ? 1 - cur : cur)] + boff;
  const T *up = (const T *)M.s[STG >= 3 ? role_buffer(ss.prev, cur) : cur] + boff;
  const double dx = ldexp(M.dx0, -gload(M.level + b));
  const T idx = (T)(1.0 / dx);
  const double dt = gload(M.scal + kDt);
  const T dts = (T)(STG >= 3 ? ss.c * dt : (STG == 1 ? dt : 0.5 * dt));
  const T cdt = dts * idx;
  int finfo[2 * NDIM];
#pragma unroll
  for (int f = 0; f < 2 * NDIM; f++) finfo[f] = gload(M.face_info + b * 2 * NDIM + f);
  const T vx = (T)M.vel[0], vy = (T)M.vel[1], vz = (T)M.vel[2];
  T *lds = (T *)adv_smem;
  // halo cells of one plane: the 2g y-ghost rows (x inside) and the 2g
  // x-ghosts of the N interior rows
  const int nhalo = 4 * g * N;
  auto row_of = [&](int jj, int kk) { return (NDIM == 3) ? (kk + g) * P + (jj + g) : (jj + g); };
  // the z window of column (i, j): cells k - R + 1 .. k + R (3-D)
  T w[2 * R];
  if constexpr (NDIM == 3) {
#pragma unroll
    for (int s = 1; s < 2 * R; s++) w[s] = gload(ud + row_of(j, s - R) * N + i);
  }
  T Fz = T(0);  // flux through the lower z face of the current plane
  const int nk = (NDIM == 3) ? N : 1;
  for (int k = 0; k < nk; k++) {
    T *pl = lds + (k & 1) * Q * Q;  // cell (x, y) at (y + g) Q + x + g
    T c;
    if constexpr (NDIM == 3) {
#pragma unroll
      for (int s = 0; s < 2 * R - 1; s++) w[s] = w[s + 1];
      w[2 * R - 1] = gload(ud + row_of(j, k + R) * N + i);
      c = w[R - 1];
    } else {
      c = gload(ud + row_of(j, 0) * N + i);
    }
    pl[(j + g) * Q + i + g] = c;
    for (int h = t; h < nhalo; h += N * N) {
      if (h < 2 * g * N) {  // y ghost rows: y = -g .. -1, N .. N + g - 1
        const int x = h % N, r = h / N;
        const int y = r < g ? r - g : N + r - g;
        pl[(y + g) * Q + x + g] = gload(ud + row_of(y, k) * N + x);
      } else {              // x ghosts of rows 0 .. N-1, c = 0 .. 2g-1
        const int e = h - 2 * g * N, cc = e % (2 * g), y = e / (2 * g);
        const int x = cc < g ? cc - g : N + cc - g;
        pl[(y + g) * Q + x + g] = gload(ud + rows * N + row_of(y, k) * 2 * g + cc);
      }
    }
    __syncthreads();
    // x faces i - 1/2 and i + 1/2, then y faces, from the staged plane
    T sx[2 * R + 1], sy[2 * R + 1];
#pragma unroll
    for (int s = 0; s < 2 * R + 1; s++) {
      sx[s] = pl[(j + g) * Q + i + g + s - R];
      sy[s] = pl[(j + g + s - R) * Q + i + g];
    }
    const T fxm = adv_flux<T, LIM, HLL>(sx, vx), fxp = adv_flux<T, LIM, HLL>(sx + 1, vx);
    T div = fxp - fxm;
    if (i == 0) adv_bflux<T, NDIM>(M, finfo[0], j, k, fxm);
    if (i == N - 1) adv_bflux<T, NDIM>(M, finfo[1], j, k, fxp);
    const T fym = adv_flux<T, LIM, HLL>(sy, vy), fyp = adv_flux<T, LIM, HLL>(sy + 1, vy);
    div += fyp - fym;
    if (j == 0) adv_bflux<T, NDIM>(M, finfo[2], i, k, fym);
    if (j == N - 1) adv_bflux<T, NDIM>(M, finfo[3], i, k, fyp);
    if constexpr (NDIM == 3) {
      if (k == 0) {  // the block's lower z face, from cells -R .. R-1
        T w0[2 * R];
        w0[0] = gload(ud + row_of(j, -R) * N + i);
#pragma unroll
        for (int s = 1; s < 2 * R; s++) w0[s] = w[s - 1];
        Fz = adv_flux<T, LIM, HLL>(w0, vz);
        adv_bflux<T, NDIM>(M, finfo[4], i, j, Fz);
      }
      const T fzp = adv_flux<T, LIM, HLL>(w, vz);
      div += fzp - Fz;
      if (k == N - 1) adv_bflux<T, NDIM>(M, finfo[5], i, j, fzp);
      Fz = fzp;
    }
    const int64_t o = row_of(j, k) * N + i;
    T base;
    if constexpr (STG == 1) base = c;
    else if constexpr (STG == 2) base = T(0.5) * (gload(up + o) + c);
    else if constexpr (STG == 3) base = (T)ss.wp * gload(up + o) + (T)ss.wd * c;
    else {
      const T *up2 = (const T *)M.s[role_buffer(ss.prev2, cur)] + boff;
      const T *up3 = (const T *)M.s[role_buffer(ss.prev3, cur)] + boff;
      base = (((T)ss.wp * gload(up + o) + (T)ss.wp2 * gload(up2 + o)) + (T)ss.wp3 * gload(up3 + o)) + (T)ss.wd * c;
    }
    const T out = base - cdt * div;
    gstore(uo + o, out);
    if (STG == 2 || (STG >= 3 && ss.epi)) {
      // the CFL limit of advection is the same in every cell of the block;
      // only the state's finiteness is per cell (cells next to F2C faces
      // are checked after the flux fix)
      if (!isfinite(out)) atomic_max_pos(&M.scal[kBad], 1.0);
    }
  }
  if ((STG == 2 || (STG >= 3 && ss.epi)) && t == 0) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; d++) s += fabs(M.vel[d]) / dx;
    atomic_max_pos_if_larger(&M.scal[kMaxInv], s);
  }
}

template <typename T, int NDIM, int LIM, bool HLL>
static void launch_adv(unsigned nb, int N, int g, const MeshDev *d, int stage, const SubStep &ss, hipStream_t s) {
  const unsigned threads = (unsigned)(N * N);
  const size_t lds = (size_t)adv_lds(N, g) * sizeof(T);
  switch (stage) {
    case 1: advect_kernel<T, NDIM, LIM, HLL, 1><<<nb, threads, lds, s>>>(d, ss); break;
    case 2: advect_kernel<T, NDIM, LIM, HLL, 2><<<nb, threads, lds, s>>>(d, ss); break;
    case 3: advect_kernel<T, NDIM, LIM, HLL, 3><<<nb, threads, lds, s>>>(d, ss); break;
    default: advect_kernel<T, NDIM, LIM, HLL, 4><<<nb, threads, lds, s>>>(d, ss); break;
  }
}

template <typename T, int NDIM>
static void launch_adv_scheme(unsigned nb, int N, int g, const MeshDev *d, int stage, int limiter, bool hll,
                              const SubStep &ss, hipStream_t s) {
  if (limiter == FOAP4_LIM_WENO5) {
    if (hll) launch_adv<T, NDIM, 2, true>(nb, N, g, d, stage, ss, s);
    else launch_adv<T, NDIM, 2, false>(nb, N, g, d, stage, ss, s);
  } else if (limiter == FOAP4_LIM_VANLEER) {
    if (hll) launch_adv<T, NDIM, 1, true>(nb, N, g, d, stage, ss, s);
    else launch_adv<T, NDIM, 1, false>(nb, N, g, d, stage, ss, s);
  } else {
    if (hll) launch_adv<T, NDIM, 0, true>(nb, N, g, d, stage, ss, s);
    else launch_adv<T, NDIM, 0, false>(nb, N, g, d, stage, ss, s);
  }
}

hipError_t launch_advect_stage(const MeshDev *d_mesh, int64_t nblocks, int block_n, int n_ghost, int stage, int ndim,
                               bool f64, int limiter, bool hll, hipStream_t s, const SubStep &ss) {
  if (nblocks <= 0) return hipSuccess;
  const unsigned nb = (unsigned)nblocks;
  if (f64) {
    if (ndim == 3) launch_adv_scheme<double, 3>(nb, block_n, n_ghost, d_mesh, stage, limiter, hll, ss, s);
    else launch_adv_scheme<double, 2>(nb, block_n, n_ghost, d_mesh, stage, limiter, hll, ss, s);
  } else {
    if (ndim == 3) launch_adv_scheme<float, 3>(nb, block_n, n_ghost, d_mesh, stage, limiter, hll, ss, s);
    else launch_adv_scheme<float, 2>(nb, block_n, n_ghost, d_mesh, stage, limiter, hll, ss, s);
  }
  return hipGetLastError();
}

}  // namespace f4
