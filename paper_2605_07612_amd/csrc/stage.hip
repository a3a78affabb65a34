// Fused flux/update stage kernel (Sec. 3.2 step list, eq. feuler / eq. heun).
//
// Work decomposition (gfx950, wave64): a workgroup of 256 threads processes
// one work item.  An item is a TILE x TILE column of cells of one block
// (TILE = 16 for N = 16, 32; for N = 8 four 8 x 8 blocks share the workgroup,
// one per wave) that marches along k over a slab of N / ks planes.  Per
// plane the primitive variables of the tile and of its +-2 ring are staged in
// LDS for the x/y stencils, while each thread keeps its own column's k-2..k+2
// window in registers for the z stencil; global loads run ahead of use.
// Every face flux is computed once.  Halo cells across a same-level face are
// read straight from the neighbouring block ("gather"); across refinement
// faces they come from the ghost cells that the ghost rounds filled.  Fluxes
// on refinement-boundary faces are stored for flux fixing (Sec. 2.7).  In
// stage 2 an epilogue evaluates the CFL limit of every new cell and reduces
// its maximum in FP64.  Items can be visited in an XCD-aware order:
// workgroup w runs on XCD w mod 8, so each XCD is given a contiguous range of
// items (neighbouring blocks in Morton order then share that XCD's L2).
// The kernel is specialised on the set of block sizes present in a launch.
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

// CFL inverse time step sum_d (|v_d| + c) / dx of one cell.  FP64 states use
// the operation order of the definition without contraction (equal to a plain
// evaluation); FP32 states evaluate it in FP32 with the hardware reciprocal
// and square root, and the maximum over cells is reduced in FP64.
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
__device__ __forceinline__ double cell_inv_dt(const float *U, float gamma, float idx, bool &bad) {
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
  return (double)s;
}

template <typename T, int NV>
__device__ __forceinline__ void copyv(T *dst, const T *src) {
#pragma unroll
  for (int v = 0; v < NV; v++) dst[v] = src[v];
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
  const int sj = P, sk = P * P;
  const int sv = (NDIM == 3) ? sk * P : sk;
  const int64_t bel = (int64_t)sv * NV;
  const int cur = M.cur;
  const T *__restrict__ ud0 = (const T *)M.s[stage == 1 ? cur : 1 - cur];
  T *uo = (T *)M.s[stage == 1 ? 1 - cur : cur] + b * bel;
  const T *up = (const T *)M.s[cur] + b * bel;
  const T gamma = (T)M.gamma;
  const double dx = ldexp(M.dx0, -M.level[b]);
  const T idx = (T)(1.0 / dx);
  const double dt = M.scal[kDt];
  const T dts = (T)(stage == 1 ? dt : 0.5 * dt);

  // per face: refinement-face flux slot (>= 0), same-level neighbour (-2 - n) or -1
  int finfo[NF];
#pragma unroll
  for (int f = 0; f < NF; f++) finfo[f] = M.face_info[b * NF + f];
  auto nbr_of = [&](int f) -> int64_t { return (M.gather && finfo[f] <= -2) ? (int64_t)(-2 - finfo[f]) : -1; };

  T *Wp = smem + sub * (PLANE + 2 * NFX) * NV;  // [v][PLANE]
  T *FX = Wp + PLANE * NV;                      // [v][TILE][TILE + 1]
  T *FY = FX + NFX * NV;                        // [v][TILE + 1][TILE]

  auto off = [&](int ii, int jj, int kk) -> int {
    return (NDIM == 3 ? (kk + g) * sk : 0) + (jj + g) * sj + (ii + g);
  };
  auto load = [&](const T *p, T *U) {
#pragma unroll
    for (int v = 0; v < NV; v++) U[v] = p[v * sv];
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

  // Source pointers, fixed for the whole item: the ring cell's column (its
  // block does not change with k) and the own column inside the block and
  // across the -z / +z faces.  Plane k of a column is at + k * sk.
  const T *ring_p;
  {
    int RI = i0 + ri, RJ = j0 + rj;
    int64_t blk = b;
    int f = -1;
    if (RI < 0) f = 0; else if (RI >= N) f = 1; else if (RJ < 0) f = 2; else if (RJ >= N) f = 3;
    if (f >= 0) {
      const int64_t n = nbr_of(f);
      if (n >= 0) {
        blk = n;
        if (f == 0) RI += N; else if (f == 1) RI -= N; else if (f == 2) RJ += N; else RJ -= N;
      }
    }
    ring_p = ud0 + blk * bel + off(RI, RJ, 0);
  }
  const T *own_p = ud0 + b * bel + off(I, J, 0);
  const T *zlo_p = nullptr, *zhi_p = nullptr;  // neighbour columns across -z / +z (gather)
  if constexpr (NDIM == 3) {
    const int64_t nlo = nbr_of(4 % NF), nhi = nbr_of(5 % NF);
    if (nlo >= 0) zlo_p = ud0 + nlo * bel + off(I, J, 0);
    if (nhi >= 0) zhi_p = ud0 + nhi * bel + off(I, J, 0);
  }
  auto col = [&](int kk) -> const T * {
    if (kk < 0 && zlo_p) return zlo_p + (kk + N) * sk;
    if (kk >= N && zhi_p) return zhi_p + (kk - N) * sk;
    return own_p + kk * sk;
  };

  // cells next to F2C faces are finished (and their dt taken) by the flux fix
  auto is_f2c = [&](int f) { return f < NF && finfo[f] >= 0 && (finfo[f] & 1); };
  const bool f2c_adj = (is_f2c(0) && I == 0) || (is_f2c(1) && I == N - 1) || (is_f2c(2) && J == 0) ||
                       (is_f2c(3) && J == N - 1);
  const bool f2c_zlo = NDIM == 3 && is_f2c(4), f2c_zhi = NDIM == 3 && is_f2c(5);

  T U0[NV], U1[NV], U2[NV], Q1[NV], R0[NV];
  T Wm1[NV], W0[NV], W1[NV], W2[NV], Fz[NV];

  if constexpr (NDIM == 3) {
    T tmp[NV], Wm2[NV];
    load(col(k0 - 2), tmp);
    to_prim<T, NDIM>(tmp, gamma, Wm2);
    load(col(k0 - 1), tmp);
    to_prim<T, NDIM>(tmp, gamma, Wm1);
    load(col(k0), U0);
    load(col(k0 + 1), U1);
    load(col(k0 + 2), U2);
    if (ring) load(ring_p + k0 * sk, R0);
    if (k0 + 3 <= k1 + 1) load(col(k0 + 3), Q1);
    to_prim<T, NDIM>(U0, gamma, W0);
    to_prim<T, NDIM>(U1, gamma, W1);
    to_prim<T, NDIM>(U2, gamma, W2);
    face_flux<T, NDIM, 2>(Wm2, Wm1, W0, W1, gamma, Fz);
    if (k0 == 0) store_bflux(4, I, J, Fz);
  } else {
    load(own_p, U0);
    if (ring) load(ring_p, R0);
    to_prim<T, NDIM>(U0, gamma, W0);
  }
  T Up[NV];
  if (stage == 2) load(up + off(I, J, k0), Up);

  for (int k = k0; k < k1; k++) {
    // stage the primitive plane k (own cell + ring) in LDS
#pragma unroll
    for (int v = 0; v < NV; v++) Wp[v * PLANE + own_lds] = W0[v];
    if (ring) {
      T Wr[NV];
      to_prim<T, NDIM>(R0, gamma, Wr);
#pragma unroll
      for (int v = 0; v < NV; v++) Wp[v * PLANE + ring_lds] = Wr[v];
      if (k + 1 < k1) load(ring_p + (k + 1) * sk, R0);
    }
    __syncthreads();

    T Fz1[NV];
    if constexpr (NDIM == 3) {
      face_flux<T, NDIM, 2>(Wm1, W0, W1, W2, gamma, Fz1);
      if (k == N - 1) store_bflux(5, I, J, Fz1);
    }

    // x and y faces of the plane: every thread computes the -x and the -y
    // face of its cell; the TILE extra +x faces of the last column go to the
    // first TILE lanes and the TILE extra +y faces of the last row to the
    // lanes of the next wave (TILE 16), so that no wave mixes x and y faces.
    auto xface = [&](int fi, int fj) {
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
    };
    auto yface = [&](int fi, int fj) {
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
    };
    xface(ti, tj);
    yface(ti, tj);
    constexpr int YX = (TT >= 64 + TILE && TILE == 16) ? 64 : TILE;  // first lane of the extra y faces
    if (lt < TILE) xface(TILE, lt);
    else if (lt >= YX && lt < YX + TILE) yface(lt - YX, TILE);
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
        Uout[v] = dts * rhs + T(0.5) * (Up[v] + U0[v]);
    }
    if (stage == 2 && k + 1 < k1) load(up + off(I, J, k + 1), Up);
    const int o = off(I, J, k);
    if (valid) {
#pragma unroll
      for (int v = 0; v < NV; v++) uo[v * sv + o] = Uout[v];
    }
    if (stage == 2 && valid) {
      const bool skip = f2c_adj || (f2c_zlo && k == 0) || (f2c_zhi && k == N - 1);
      if (!skip) {
        if constexpr (sizeof(T) == 8) {
          vmax = fmax(vmax, cell_inv_dt<NDIM>((const double *)Uout, M.gamma, dx, bad));
        } else {
          vmax = fmax(vmax, cell_inv_dt<NDIM>((const float *)Uout, (float)gamma, (float)idx, bad));
        }
      }
    }

    if constexpr (NDIM == 3) {
      copyv<T, NV>(Fz, Fz1);
      copyv<T, NV>(Wm1, W0);
      copyv<T, NV>(W0, W1);
      copyv<T, NV>(W1, W2);
      copyv<T, NV>(U0, U1);
      copyv<T, NV>(U1, U2);
      if (k + 3 <= k1 + 1) {
        copyv<T, NV>(U2, Q1);
        to_prim<T, NDIM>(U2, gamma, W2);
        if (k + 4 <= k1 + 1) load(col(k + 4), Q1);
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

// Item visited by iteration `it` of workgroup w: with xcd != 0, XCD x = w mod 8
// walks the x-th eighth of the item range; else plain striding.
__device__ __forceinline__ int64_t item_of(int64_t w, int64_t it, int64_t grid, int64_t total, int xcd) {
  if (!xcd) return w + it * grid;
  const int64_t per_xcd = (total + 7) / 8;
  const int64_t lanes = (grid + 7 - (w & 7)) / 8;  // workgroups on this XCD
  const int64_t j = (w >> 3) + it * lanes;         // position inside the XCD's range
  return j < per_xcd ? (w & 7) * per_xcd + j : total;
}

// Target waves per SIMD: 3 for single-size FP32 kernels (167 VGPRs, no
// spills); the mixed-size and FP64 kernels keep what their registers allow.
template <typename T, int NM>
constexpr int stage_waves() { return (sizeof(T) == 4 && NM != 7) ? 3 : 1; }

// NM: bit mask of the block sizes present (1: N = 8, 2: N = 16, 4: N = 32)
template <typename T, int NDIM, int NM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(stage_waves<T, NM>())))
void stage_kernel(const MeshDev *__restrict__ meshes, int n_meshes, int64_t total, int stage, int xcd) {
  __shared__ T smem[smem_cells<NDIM>()];
  double vmax = 0.0;
  bool bad = false;
  int mprev = -1;
  const int64_t grid = gridDim.x;
  const int64_t lanes = grid / 8 > 0 ? grid / 8 : 1;
  const int64_t iters = xcd ? ((total + 7) / 8 + lanes - 1) / lanes : (total + grid - 1) / grid;
  for (int64_t it = 0; it < iters; it++) {
    const int64_t item = item_of(blockIdx.x, it, grid, total, xcd);
    if (item >= total) break;
    int lo = 0, hi = n_meshes - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (meshes[mid].item_begin <= item) lo = mid; else hi = mid - 1;
    }
    if (stage == 2 && mprev >= 0 && lo != mprev) flush_dt(meshes[mprev], vmax, bad);
    mprev = lo;
    const MeshDev &M = meshes[lo];
    const int64_t local = item - M.item_begin;
    if constexpr (NM == 1) {
      stage_item<T, NDIM, 8>(M, stage, local, smem, vmax, bad);
    } else if constexpr (NM == 2) {
      stage_item<T, NDIM, 16>(M, stage, local, smem, vmax, bad);
    } else if constexpr (NM == 4) {
      stage_item<T, NDIM, 32>(M, stage, local, smem, vmax, bad);
    } else {
      switch (M.N) {
        case 8: stage_item<T, NDIM, 8>(M, stage, local, smem, vmax, bad); break;
        case 16: stage_item<T, NDIM, 16>(M, stage, local, smem, vmax, bad); break;
        default: stage_item<T, NDIM, 32>(M, stage, local, smem, vmax, bad); break;
      }
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

template <typename T, int NDIM>
static void launch_t(unsigned nblk, int nmask, const MeshDev *d, int n, int64_t total, int stage, int xcd,
                     hipStream_t s) {
  switch (nmask) {
    case 1: stage_kernel<T, NDIM, 1><<<nblk, 256, 0, s>>>(d, n, total, stage, xcd); break;
    case 2: stage_kernel<T, NDIM, 2><<<nblk, 256, 0, s>>>(d, n, total, stage, xcd); break;
    case 4: stage_kernel<T, NDIM, 4><<<nblk, 256, 0, s>>>(d, n, total, stage, xcd); break;
    default: stage_kernel<T, NDIM, 7><<<nblk, 256, 0, s>>>(d, n, total, stage, xcd); break;
  }
}

hipError_t launch_stage(const MeshDev *d_meshes, int n_meshes, int64_t total_items, int stage,
                        int ndim, bool f64, int grid, hipStream_t s, int xcd, int nmask) {
  if (total_items <= 0) return hipSuccess;
  int64_t nblk = (grid > 0 && grid < total_items) ? grid : total_items;
  if (xcd) nblk = (nblk + 7) / 8 * 8;  // every XCD gets the same number of workgroups
  if (f64) {
    if (ndim == 3) launch_t<double, 3>((unsigned)nblk, nmask, d_meshes, n_meshes, total_items, stage, xcd, s);
    else launch_t<double, 2>((unsigned)nblk, nmask, d_meshes, n_meshes, total_items, stage, xcd, s);
  } else {
    if (ndim == 3) launch_t<float, 3>((unsigned)nblk, nmask, d_meshes, n_meshes, total_items, stage, xcd, s);
    else launch_t<float, 2>((unsigned)nblk, nmask, d_meshes, n_meshes, total_items, stage, xcd, s);
  }
  return hipGetLastError();
}

}  // namespace f4
