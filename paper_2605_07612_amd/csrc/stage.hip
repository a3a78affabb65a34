// Fused flux/update stage kernel (Sec. 3.2 step list, eq. feuler / eq. heun).
//
// Work decomposition (gfx950, wave64): a workgroup of 256 threads processes
// one work item.  An item is a TILE x TILE column of cells of one block
// (TILE = 16 for N = 16, 32; for N = 8 four 8 x 8 blocks share the workgroup,
// one per wave) that marches along k over a slab of N / ks planes.  Per
// plane the primitive variables of the tile and of its +-2 ring are staged in
// LDS for the x/y stencils, while each thread keeps its own column's k-2..k+2
// window in registers for the z stencil.  Every face flux is computed once.
// Fluxes on refinement-boundary faces are stored for flux fixing (Sec. 2.7).
// In stage 2 an FP64 epilogue reduces the CFL limit of the new state.
#include "device_common.h"
#include "foap4_internal.h"

namespace f4 {

template <int N>
struct TileCfg {
  static constexpr int TILE = (N == 8) ? 8 : 16;
  static constexpr int SUB = 256 / (TILE * TILE);       // sub-tiles per workgroup
  static constexpr int TPB = (N / TILE) * (N / TILE);   // tiles per block plane
};

// LDS elements per workgroup: SUB * (plane + x faces + y faces) * NV, maximum
// over the block sizes (TILE 16: 400 + 272 + 272; TILE 8: 4 * (144 + 72 + 72)).
template <int NDIM>
constexpr int smem_cells() { return 1152 * (NDIM + 2); }

// CFL inverse time step of one cell, sum_d (|v_d| + c) / dx, in FP64 with the
// operation order of the definition (no contraction).
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

template <typename T, int NDIM, int N>
__device__ __forceinline__ void stage_item(const MeshDev &M, int stage, int64_t local, T *smem,
                                           double &vmax, bool &bad) {
  using C = TileCfg<N>;
  constexpr int TILE = C::TILE, SUB = C::SUB, TPB = C::TPB;
  constexpr int NV = NDIM + 2;
  constexpr int LP = TILE + 4;
  constexpr int PLANE = LP * LP;
  constexpr int NFX = (TILE + 1) * TILE;
  constexpr int TT = TILE * TILE;
  constexpr int NF = 2 * NDIM;

  const int tid = threadIdx.x;
  const int sub = tid / TT, lt = tid % TT;
  const int ti = lt % TILE, tj = lt / TILE;
  const int ks = (NDIM == 3) ? M.ks : 1;
  const int kslab = (int)(local % ks);
  const int64_t s = (local / ks) * SUB + sub;
  const bool valid = (s / TPB) < M.nb;
  const int64_t b = valid ? s / TPB : M.nb - 1;
  const int tile = (int)(s % TPB);
  const int i0 = (tile % (N / TILE)) * TILE, j0 = (tile / (N / TILE)) * TILE;
  const int kd = (NDIM == 3) ? N / ks : 1;
  const int k0 = (NDIM == 3) ? kslab * kd : 0, k1 = k0 + kd;
  const int g = M.g, P = N + 2 * g;
  const int64_t sj = P, sk = (int64_t)P * P, sv = (NDIM == 3) ? sk * P : sk;
  const int64_t bel = sv * NV;
  const int cur = M.cur;
  const T *__restrict__ ud = (const T *)M.s[stage == 1 ? cur : 1 - cur] + b * bel;
  T *uo = (T *)M.s[stage == 1 ? 1 - cur : cur] + b * bel;
  const T *up = (const T *)M.s[cur] + b * bel;
  const T gamma = (T)M.gamma;
  const double dx = ldexp(M.dx0, -M.level[b]);
  const T idx = (T)(1.0 / dx);
  const double dt = M.scal[kDt];
  const T dts = (T)(stage == 1 ? dt : 0.5 * dt);

  int finfo[NF];
#pragma unroll
  for (int f = 0; f < NF; f++) finfo[f] = M.face_info[b * NF + f];

  T *Wp = smem + sub * (PLANE + 2 * NFX) * NV;  // [v][PLANE]
  T *FX = Wp + PLANE * NV;                      // [v][TILE][TILE + 1]
  T *FY = FX + NFX * NV;                        // [v][TILE + 1][TILE]

  auto off = [&](int ii, int jj, int kk) -> int64_t {
    return (NDIM == 3 ? (int64_t)(kk + g) * sk : 0) + (int64_t)(jj + g) * sj + (ii + g);
  };
  auto load = [&](const T *base, int64_t o, T *U) {
#pragma unroll
    for (int v = 0; v < NV; v++) U[v] = base[v * sv + o];
  };
  auto store_bflux = [&](int f, int t1, int t2, const T *F) {
    const int info = finfo[f];
    if (info < 0 || !valid) return;
    T *buf = (T *)((info & 1) ? M.bflux_c : M.bflux_f);
    const int64_t slot = info >> 1;
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const int64_t o = (NDIM == 3) ? ((slot * NV + v) * N + t2) * N + t1 : (slot * NV + v) * N + t1;
      buf[o] = F[v];
    }
  };

  // ring cell of this thread (x ghosts: 4 per row; y ghosts: 4 rows)
  const bool ring = lt < 8 * TILE;
  int ri = 0, rj = 0;
  if (lt < 4 * TILE) {
    const int c = lt & 3;
    rj = lt >> 2;
    ri = (c < 2) ? c - 2 : TILE + c - 2;
  } else if (ring) {
    const int r = lt - 4 * TILE, c = r / TILE;
    ri = r % TILE;
    rj = (c < 2) ? c - 2 : TILE + c - 2;
  }
  const int ring_lds = (rj + 2) * LP + (ri + 2);
  const int own_lds = (tj + 2) * LP + (ti + 2);
  const int I = i0 + ti, J = j0 + tj;

  // F2C faces of this block: the cells next to them are finished by the flux fix
  bool f2c_adj = false;
  {
    const bool xm = finfo[0] >= 0 && (finfo[0] & 1), xp = finfo[1] >= 0 && (finfo[1] & 1);
    const bool ym = finfo[2] >= 0 && (finfo[2] & 1), yp = finfo[3] >= 0 && (finfo[3] & 1);
    f2c_adj = (xm && I == 0) || (xp && I == N - 1) || (ym && J == 0) || (yp && J == N - 1);
  }

  T U0[NV], U1[NV], U2[NV], Un[NV], Ur[NV];
  T Wm1[NV], W0[NV], W1[NV], W2[NV], Fz[NV];

  if constexpr (NDIM == 3) {
    T Wm2[NV], tmp[NV];
    load(ud, off(I, J, k0 - 2), tmp);
    to_prim<T, NDIM>(tmp, gamma, Wm2);
    load(ud, off(I, J, k0 - 1), tmp);
    to_prim<T, NDIM>(tmp, gamma, Wm1);
    load(ud, off(I, J, k0), U0);
    load(ud, off(I, J, k0 + 1), U1);
    load(ud, off(I, J, k0 + 2), U2);
    if (ring) load(ud, off(i0 + ri, j0 + rj, k0), Ur);
    if (k0 + 3 <= k1 + 1) load(ud, off(I, J, k0 + 3), Un);
    to_prim<T, NDIM>(U0, gamma, W0);
    to_prim<T, NDIM>(U1, gamma, W1);
    to_prim<T, NDIM>(U2, gamma, W2);
    face_flux<T, NDIM, NDIM - 1>(Wm2, Wm1, W0, W1, gamma, Fz);
    if (k0 == 0) store_bflux(4, I, J, Fz);
  } else {
    load(ud, off(I, J, 0), U0);
    if (ring) load(ud, off(i0 + ri, j0 + rj, 0), Ur);
    to_prim<T, NDIM>(U0, gamma, W0);
  }

  for (int k = k0; k < k1; k++) {
    // stage the primitive plane k (own cell + ring) in LDS
#pragma unroll
    for (int v = 0; v < NV; v++) Wp[v * PLANE + own_lds] = W0[v];
    if (ring) {
      T Wr[NV];
      to_prim<T, NDIM>(Ur, gamma, Wr);
#pragma unroll
      for (int v = 0; v < NV; v++) Wp[v * PLANE + ring_lds] = Wr[v];
      if (k + 1 < k1) load(ud, off(i0 + ri, j0 + rj, k + 1), Ur);
    }
    T Uprev[NV];
    if (stage == 2) load(up, off(I, J, k), Uprev);
    __syncthreads();

    T Fz1[NV];
    if constexpr (NDIM == 3) {
      face_flux<T, NDIM, 2>(Wm1, W0, W1, W2, gamma, Fz1);
      if (k == N - 1) store_bflux(5, I, J, Fz1);
    }

    // x and y faces of the plane, flattened over the sub-tile's threads
#pragma unroll
    for (int pass = 0; pass < (2 * NFX + TT - 1) / TT; pass++) {
      const int e = lt + pass * TT;
      if (e < NFX) {
        const int fi = e % (TILE + 1), fj = e / (TILE + 1);
        T A0[NV], A1[NV], A2[NV], A3[NV], F[NV];
        const int base = (fj + 2) * LP + fi;  // cell fi - 2
#pragma unroll
        for (int v = 0; v < NV; v++) {
          A0[v] = Wp[v * PLANE + base];
          A1[v] = Wp[v * PLANE + base + 1];
          A2[v] = Wp[v * PLANE + base + 2];
          A3[v] = Wp[v * PLANE + base + 3];
        }
        face_flux<T, NDIM, 0>(A0, A1, A2, A3, gamma, F);
#pragma unroll
        for (int v = 0; v < NV; v++) FX[(v * TILE + fj) * (TILE + 1) + fi] = F[v];
        if (fi == 0 && i0 == 0) store_bflux(0, j0 + fj, k, F);
        if (fi == TILE && i0 + TILE == N) store_bflux(1, j0 + fj, k, F);
      } else if (e < 2 * NFX) {
        const int e2 = e - NFX;
        const int fi = e2 % TILE, fj = e2 / TILE;
        T A0[NV], A1[NV], A2[NV], A3[NV], F[NV];
        const int base = fj * LP + fi + 2;  // cell fj - 2
#pragma unroll
        for (int v = 0; v < NV; v++) {
          A0[v] = Wp[v * PLANE + base];
          A1[v] = Wp[v * PLANE + base + LP];
          A2[v] = Wp[v * PLANE + base + 2 * LP];
          A3[v] = Wp[v * PLANE + base + 3 * LP];
        }
        face_flux<T, NDIM, 1>(A0, A1, A2, A3, gamma, F);
#pragma unroll
        for (int v = 0; v < NV; v++) FY[(v * (TILE + 1) + fj) * TILE + fi] = F[v];
        if (fj == 0 && j0 == 0) store_bflux(2, i0 + fi, k, F);
        if (fj == TILE && j0 + TILE == N) store_bflux(3, i0 + fi, k, F);
      }
    }
    __syncthreads();

    // conservative update of the own cell (eq. feuler with Heun weights)
    T Uout[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const T dfx = FX[(v * TILE + tj) * (TILE + 1) + ti + 1] - FX[(v * TILE + tj) * (TILE + 1) + ti];
      const T dfy = FY[(v * (TILE + 1) + tj + 1) * TILE + ti] - FY[(v * (TILE + 1) + tj) * TILE + ti];
      T rhs = -(dfx * idx);
      rhs -= dfy * idx;
      if constexpr (NDIM == 3) rhs -= (Fz1[v] - Fz[v]) * idx;
      if (stage == 1)
        Uout[v] = dts * rhs + U0[v];
      else
        Uout[v] = dts * rhs + T(0.5) * (Uprev[v] + U0[v]);
    }
    const int64_t o = off(I, J, k);
    if (valid) {
#pragma unroll
      for (int v = 0; v < NV; v++) uo[v * sv + o] = Uout[v];
    }
    if (stage == 2 && valid) {
      const bool skip = f2c_adj || (NDIM == 3 && ((finfo[4 % NF] >= 0 && (finfo[4 % NF] & 1) && k == 0) ||
                                                  (finfo[5 % NF] >= 0 && (finfo[5 % NF] & 1) && k == N - 1)));
      if (!skip) {
        double Ud[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) Ud[v] = (double)Uout[v];
        const double sv_ = cell_inv_dt<NDIM>(Ud, M.gamma, dx, bad);
        vmax = fmax(vmax, sv_);
      }
    }

    if constexpr (NDIM == 3) {
#pragma unroll
      for (int v = 0; v < NV; v++) {
        Fz[v] = Fz1[v];
        Wm1[v] = W0[v];
        W0[v] = W1[v];
        W1[v] = W2[v];
        U0[v] = U1[v];
        U1[v] = U2[v];
      }
      if (k + 3 <= k1 + 1) {
#pragma unroll
        for (int v = 0; v < NV; v++) U2[v] = Un[v];
        to_prim<T, NDIM>(U2, gamma, W2);
        if (k + 4 <= k1 + 1) load(ud, off(I, J, k + 4), Un);
      }
    }
  }
}

__device__ __forceinline__ void flush_dt(const MeshDev &M, double &vmax, bool &bad) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, o));
  const bool anybad = __ballot(bad) != 0;
  if ((threadIdx.x & 63) == 0) {
    if (vmax > 0.0) atomic_max_pos(&M.scal[kMaxInv], vmax);
    if (anybad) atomic_max_pos(&M.scal[kBad], 1.0);
  }
  vmax = 0.0;
  bad = false;
}

template <typename T, int NDIM>
__global__ __launch_bounds__(256) void stage_kernel(const MeshDev *__restrict__ meshes, int n_meshes,
                                                    int64_t total, int stage) {
  __shared__ T smem[smem_cells<NDIM>()];
  double vmax = 0.0;
  bool bad = false;
  int mprev = -1;
  for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
    int lo = 0, hi = n_meshes - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (meshes[mid].item_begin <= item) lo = mid; else hi = mid - 1;
    }
    if (stage == 2 && mprev >= 0 && lo != mprev) flush_dt(meshes[mprev], vmax, bad);
    mprev = lo;
    const MeshDev &M = meshes[lo];
    const int64_t local = item - M.item_begin;
    switch (M.N) {
      case 8: stage_item<T, NDIM, 8>(M, stage, local, smem, vmax, bad); break;
      case 16: stage_item<T, NDIM, 16>(M, stage, local, smem, vmax, bad); break;
      default: stage_item<T, NDIM, 32>(M, stage, local, smem, vmax, bad); break;
    }
    __syncthreads();
  }
  if (stage == 2 && mprev >= 0) flush_dt(meshes[mprev], vmax, bad);
}

int64_t stage_items_for(int ndim, int N, int64_t nb, int ks) {
  const int tile = (N == 8) ? 8 : 16;
  const int sub = 256 / (tile * tile);
  const int tpb = (N / tile) * (N / tile);
  const int64_t tiles = nb * tpb;
  return ((tiles + sub - 1) / sub) * (ndim == 3 ? ks : 1);
}

hipError_t launch_stage(const MeshDev *d_meshes, int n_meshes, int64_t total_items, int stage,
                        int ndim, bool f64, int grid, hipStream_t s) {
  if (total_items <= 0) return hipSuccess;
  const unsigned nblk = (unsigned)((grid > 0 && grid < total_items) ? grid : total_items);
  if (f64) {
    if (ndim == 3)
      stage_kernel<double, 3><<<nblk, 256, 0, s>>>(d_meshes, n_meshes, total_items, stage);
    else
      stage_kernel<double, 2><<<nblk, 256, 0, s>>>(d_meshes, n_meshes, total_items, stage);
  } else {
    if (ndim == 3)
      stage_kernel<float, 3><<<nblk, 256, 0, s>>>(d_meshes, n_meshes, total_items, stage);
    else
      stage_kernel<float, 2><<<nblk, 256, 0, s>>>(d_meshes, n_meshes, total_items, stage);
  }
  return hipGetLastError();
}

}  // namespace f4
