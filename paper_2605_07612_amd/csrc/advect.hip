// Stage kernel of scalar advection (Sec. 3.4): one conserved variable rho
// carried by a uniform velocity v, rho_t + div(rho v) = 0.  The face values
// come from the mesh's reconstruction (minmod or van Leer MUSCL, WENO5), the
// physical flux on either side of a face is rho v_d, and the numerical flux
// (Rusanov or HLL) takes the wave speeds min(v_d, 0) and max(v_d, 0).
//
// One workgroup per block and one thread per (i, j) column, which marches
// along k.  Per plane the workgroup stages the plane with its x and y face
// halos in LDS (the interior from the threads' own z windows; the halo of a
// same-level face straight from the neighbouring block's interior when the
// mesh gathers halos, else - and always across refinement and boundary
// faces - from the block's stored ghosts, filled by the ghost rounds),
// double buffered so that one barrier per plane suffices; every thread then
// evaluates the two x faces and two y faces of its cell from LDS and the
// upper z face from its register window of the column (the lower one is the
// upper face of the previous plane).  The update, the refinement-face flux
// capture and the CFL epilogue follow the Euler stage kernels: stage 1 / 2
// Heun's stages, 3 the generic sub-step, 4 the generic sub-step with three
// earlier states.  With a single variable the work per cell is small, so the
// kernel is bound by its HBM traffic: the state is read once per stage (plus
// the face halos, and Heun's second stage reads U^n) and written once.
#include <type_traits>

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

// MAXT: the largest workgroup (N^2 threads) the instantiation serves: 1024
// for 32^2 columns, 256 for 8^2 and 16^2 (which leaves the compiler up to 512
// registers per thread instead of 128).  HS: halo cells per thread and
// plane, ceil(4 g N / N^2): 1, or 2 for 8^2 columns with g >= 3 (N >= 2 g
// bounds it by 2).  Every register saved is worth it here: the kernel waits
// on its loads, and more waves per SIMD hide more of that.
template <typename T, int NDIM, int LIM, bool HLL, int STG, int MAXT, int HS>
__global__ __launch_bounds__(MAXT) void advect_kernel(const MeshDev *__restrict__ Mp, SubStep ss) {
  constexpr int R = AdvStencil<LIM>::R;
  extern __shared__ __align__(16) unsigned char adv_smem[];
  const MeshDev &M = *Mp;
  const int N = M.N, g = M.g, P = N + 2 * g, Q = P;
  const int rows = (NDIM == 3) ? P * P : P;  // rows (k, j) of the row part of a block
  const int64_t sv = (NDIM == 3) ? (int64_t)P * P * P : (int64_t)P * P;
  // XCD-aware block order: workgroup w runs on XCD w mod 8, so XCD x is
  // given the contiguous range of blocks [x q + min(x, r), ...) of q or q + 1
  // blocks (nb = 8 q + r): blocks that are neighbours in Morton order, whose
  // face halos each reads, share that XCD's L2.  A bijection onto 0 .. nb-1.
  const int64_t nbk = M.nb, xq = nbk / 8, xr = nbk % 8;
  const int64_t xid = blockIdx.x % 8, xi = blockIdx.x / 8;
  const int64_t b = xid * xq + (xid < xr ? xid : xr) + xi;
  const int t = threadIdx.x, i = t % N, j = t / N;
  const int cur = M.cur;
  const int64_t boff = b * sv;
  const T *ud0 = (const T *)M.s[STG >= 3 ? role_buffer(ss.deriv, cur) : (STG == 1 ? cur : 1 - cur)];
  const T *ud = ud0 + boff;
  T *uo = (T *)M.s[STG >= 3 ? role_buffer(ss.out, cur) : (STG == 1 ? 1 - cur : cur)] + boff;
  const T *up = (const T *)M.s[STG >= 3 ? role_buffer(ss.prev, cur) : cur] + boff;
  const double dx = ldexp(M.dx0, -gload(M.level + b));
  const T idx = (T)(1.0 / dx);
  const double dt = gload(M.scal + kDt);
  const T dts = (T)(STG >= 3 ? ss.c * dt : (STG == 1 ? dt : 0.5 * dt));
  const T cdt = dts * idx;
  int finfo[2 * NDIM];
  // with gathered halos, the block data of the same-level neighbour across
  // each face (null: the face's halo comes from this block's stored ghosts)
  const T *nbp[2 * NDIM];
#pragma unroll
  for (int f = 0; f < 2 * NDIM; f++) {
    finfo[f] = gload(M.face_info + b * 2 * NDIM + f);
    nbp[f] = (M.gather && finfo[f] <= -2) ? ud0 + (int64_t)(-2 - finfo[f]) * sv : nullptr;
  }
  const T vx = (T)M.vel[0], vy = (T)M.vel[1], vz = (T)M.vel[2];
  T *lds = (T *)adv_smem;
  // halo cells of one plane: the 2g y-ghost rows (x inside) and the 2g
  // x-ghosts of the N interior rows
  const int nhalo = 4 * g * N;
  auto row_of = [&](int jj, int kk) { return (NDIM == 3) ? (kk + g) * P + (jj + g) : (jj + g); };
  // a cell of the block or of its face halo (at most one coordinate outside
  // 0 .. N-1): across a same-level face from the neighbour's interior when
  // gathering, else from the stored ghosts
  auto cell = [&](int x, int y, int kk) -> T {
    if (x < 0) return nbp[0] ? gload(nbp[0] + row_of(y, kk) * N + x + N) : gload(ud + rows * N + row_of(y, kk) * 2 * g + x + g);
    if (x >= N) return nbp[1] ? gload(nbp[1] + row_of(y, kk) * N + x - N) : gload(ud + rows * N + row_of(y, kk) * 2 * g + x - N + g);
    const T *src = ud;
    if (y < 0 && nbp[2]) { src = nbp[2]; y += N; }
    else if (y >= N && nbp[3]) { src = nbp[3]; y -= N; }
    if constexpr (NDIM == 3) {
      if (kk < 0 && nbp[4]) { src = nbp[4]; kk += N; }
      else if (kk >= N && nbp[5]) { src = nbp[5]; kk -= N; }
    }
    return gload(src + row_of(y, kk) * N + x);
  };
  // this thread's halo cells of a plane (the same (x, y) in every plane)
  constexpr int HMAX = HS;
  int hx[HMAX], hy[HMAX];
  bool hv[HMAX];
#pragma unroll
  for (int q = 0; q < HMAX; q++) {
    const int h = t + q * N * N;
    hv[q] = h < nhalo;
    if (h < 2 * g * N) {  // y ghost rows: y = -g .. -1, N .. N + g - 1
      const int r = h / N;
      hx[q] = h % N;
      hy[q] = r < g ? r - g : N + r - g;
    } else {              // x ghosts of rows 0 .. N-1, c = 0 .. 2g-1
      const int e = h - 2 * g * N, cc = e % (2 * g);
      hy[q] = e / (2 * g);
      hx[q] = cc < g ? cc - g : N + cc - g;
    }
  }
  // Loads run D planes ahead of use: with one variable a plane holds little
  // work, so the window cells, halo cells and earlier-state cells of the next
  // D planes are in flight together (in register slots: plane kk in slot
  // kk % D; the plane loop is unrolled by D so that every slot is named by a
  // constant).  FP64 workgroups of 1024 threads (128 registers) keep D = 2,
  // or D = 1 with WENO5.
  constexpr int D = (sizeof(T) == 8 && MAXT > 256) ? (LIM == 2 ? 1 : 2) : 4;
  const T *up2 = (const T *)M.s[STG == 4 ? role_buffer(ss.prev2, cur) : cur] + boff;
  const T *up3 = (const T *)M.s[STG == 4 ? role_buffer(ss.prev3, cur) : cur] + boff;
  // Addresses: cell (i, j, kk) of the own column is at the wave-uniform
  // plane base wbase(kk) (this block, or across -z / +z the neighbour's when
  // gathering) plus the lane's byte offset lo, read and written through
  // buffer descriptors; a halo cell of this thread is at hp[q] + kk hs[q].
  const int pstride = (NDIM == 3) ? P * N : 0;  // elements per plane of the row part
  const uint32_t lo = (uint32_t)(row_of(j, 0) * N + i) * (uint32_t)sizeof(T);
  auto wbase = [&](int kk) -> const T * {
    if constexpr (NDIM == 3) {
      if (kk < 0 && nbp[4]) return nbp[4] + (kk + N) * pstride;
      if (kk >= N && nbp[5]) return nbp[5] + (kk - N) * pstride;
    }
    return ud + kk * pstride;
  };
  const T *hp[HMAX];
  int hs[HMAX];
#pragma unroll
  for (int q = 0; q < HMAX; q++) {
    const int x = hx[q], y = hy[q];
    hp[q] = ud;
    hs[q] = 0;
    if (!hv[q]) continue;
    if (x < 0 || x >= N) {
      const T *nb = nbp[x < 0 ? 0 : 1];
      if (nb) {
        hp[q] = nb + row_of(y, 0) * N + (x < 0 ? x + N : x - N);
        hs[q] = pstride;
      } else {  // stored x ghosts: rows of 2 g after the row part
        hp[q] = ud + rows * N + row_of(y, 0) * 2 * g + (x < 0 ? x + g : x - N + g);
        hs[q] = (NDIM == 3) ? P * 2 * g : 0;
      }
    } else {
      const T *src = ud;
      int yy = y;
      if (y < 0 && nbp[2]) { src = nbp[2]; yy += N; }
      else if (y >= N && nbp[3]) { src = nbp[3]; yy -= N; }
      hp[q] = src + row_of(yy, 0) * N + x;
      hs[q] = pstride;
    }
  }
  T hq[D][HMAX], pq[D], pq2[D], pq3[D], wq[D];
  auto fetch = [&](int kk, auto slot) {  // the values plane kk needs beyond the window
    constexpr int S = decltype(slot)::value;
#pragma unroll
    for (int q = 0; q < HMAX; q++)
      if (hv[q]) hq[S][q] = gload(hp[q] + kk * hs[q]);
    if constexpr (STG >= 2) pq[S] = buf_load<T>(buf_rsrc(up + kk * pstride), lo, 0);
    if constexpr (STG == 4) {
      pq2[S] = buf_load<T>(buf_rsrc(up2 + kk * pstride), lo, 0);
      pq3[S] = buf_load<T>(buf_rsrc(up3 + kk * pstride), lo, 0);
    }
    wq[S] = buf_load<T>(buf_rsrc(wbase((NDIM == 3) ? kk + R : 0)), lo, 0);
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  // the z window of column (i, j): cells k - R + 1 .. k + R (3-D)
  T w[2 * R];
  if constexpr (NDIM == 3) {
#pragma unroll
    for (int s = 1; s < 2 * R; s++) w[s] = cell(i, j, s - R);
  }
  const int nk = (NDIM == 3) ? N : 1;
  fetch(0, I0{});
  if constexpr (D > 1) {
    if (1 < nk) fetch(1, I1{});
  }
  if constexpr (D > 2) {
    if (2 < nk) fetch(2, I2{});
    if (3 < nk) fetch(3, I3{});
  }
  T Fz = T(0);  // flux through the lower z face of the current plane
  auto plane = [&](const int k, auto slot) __attribute__((always_inline)) {
    constexpr int S = decltype(slot)::value;
    T *pl = lds + (k & 1) * Q * Q;  // cell (x, y) at (y + g) Q + x + g
    T c;
    if constexpr (NDIM == 3) {
#pragma unroll
      for (int s = 0; s < 2 * R - 1; s++) w[s] = w[s + 1];
      w[2 * R - 1] = wq[S];
      c = w[R - 1];
    } else {
      c = wq[S];
    }
    pl[(j + g) * Q + i + g] = c;
#pragma unroll
    for (int q = 0; q < HMAX; q++)
      if (hv[q]) pl[(hy[q] + g) * Q + hx[q] + g] = hq[S][q];
    const T cp = (STG >= 2) ? pq[S] : T(0);
    const T cp2 = (STG == 4) ? pq2[S] : T(0), cp3 = (STG == 4) ? pq3[S] : T(0);
    if (k + D < nk) fetch(k + D, slot);
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
        w0[0] = cell(i, j, -R);
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
    T base;
    if constexpr (STG == 1) base = c;
    else if constexpr (STG == 2) base = T(0.5) * (cp + c);
    else if constexpr (STG == 3) base = (T)ss.wp * cp + (T)ss.wd * c;
    else base = (((T)ss.wp * cp + (T)ss.wp2 * cp2) + (T)ss.wp3 * cp3) + (T)ss.wd * c;
    const T out = base - cdt * div;
    buf_store<T>(out, buf_rsrc(uo + k * pstride), lo, 0);
    if (STG == 2 || (STG >= 3 && ss.epi)) {
      // the CFL limit of advection is the same in every cell of the block;
      // only the state's finiteness is per cell (cells next to F2C faces
      // are checked after the flux fix)
      if (!isfinite(out)) atomic_max_pos(&M.scal[kBad], 1.0);
    }
  };
  for (int k = 0; k < nk; k += D) {
    plane(k, I0{});
    if constexpr (D > 1) {
      if (k + 1 >= nk) break;
      plane(k + 1, I1{});
    }
    if constexpr (D > 2) {
      if (k + 2 >= nk) break;
      plane(k + 2, I2{});
      if (k + 3 >= nk) break;
      plane(k + 3, I3{});
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
#define F4_ADV(STG, MAXT, HS) advect_kernel<T, NDIM, LIM, HLL, STG, MAXT, HS><<<nb, threads, lds, s>>>(d, ss)
#define F4_ADV_STAGES(MAXT, HS)                \
  switch (stage) {                             \
    case 1: F4_ADV(1, MAXT, HS); break;        \
    case 2: F4_ADV(2, MAXT, HS); break;        \
    case 3: F4_ADV(3, MAXT, HS); break;        \
    default: F4_ADV(4, MAXT, HS); break;       \
  }
  // halo cells of a plane: 4 g N (2-D: also 4 g N per row of planes)
  const bool two_halo = 4 * g * N > N * N;
  if (threads > 256) {
    F4_ADV_STAGES(1024, 1)  // N = 32 with g <= 4: 4 g N <= N^2
  } else if (two_halo) {
    F4_ADV_STAGES(256, 2)
  } else {
    F4_ADV_STAGES(256, 1)
  }
#undef F4_ADV_STAGES
#undef F4_ADV
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
