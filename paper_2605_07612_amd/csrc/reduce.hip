// FP64 reductions and flux fixing: CFL time step, step finalisation,
// conserved totals, and the flux correction at refinement boundaries
// (Sec. 2.7).
#include "device_common.h"
#include "foap4_internal.h"

#include <mutex>

namespace f4 {

// sum_d (|v_d| + c) / dx of one cell in FP64, operation order of the
// definition, no contraction (bit-identical to a plain evaluation).
template <int NDIM>
__device__ __forceinline__ double inv_dt_cell(const double *U, double gamma, double dx, bool &bad) {
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

// Scalar advection (Sec. 3.4): the fastest wave along d is |v_d| in every
// cell, so the CFL limit is sum_d |v_d| / dx (the definition's operation
// order); a non-finite rho marks the state bad.
template <int NDIM>
__device__ __forceinline__ double inv_dt_adv(const MeshDev &M, double rho, double dx, bool &bad) {
#pragma clang fp contract(off)
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < NDIM; d++) s += fabs(M.vel[d]) / dx;
  bad |= !isfinite(rho);
  return s;
}

__device__ __forceinline__ void wave_flush(double *scal, double vmax, bool bad) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, o));
  const bool anybad = __ballot(bad) != 0;
  if ((threadIdx.x & 63) == 0) {
    if (vmax > 0.0) atomic_max_pos_if_larger(&scal[kMaxInv], vmax);
    if (anybad) atomic_max_pos(&scal[kBad], 1.0);
  }
}

// CFL limit of every interior cell of the current state (one workgroup per block)
template <typename T, int NDIM, int NV>
__global__ __launch_bounds__(256) void dt_full_kernel(const MeshDev *__restrict__ Mp) {
  const MeshDev &M = *Mp;
  const int64_t b = blockIdx.x;
  const int N = M.N, g = M.g, P = N + 2 * g;
  const int64_t sv = (NDIM == 3) ? (int64_t)P * P * P : (int64_t)P * P;
  const T *u = (const T *)M.s[M.cur] + b * sv * NV;
  const double dx = ldexp(M.dx0, -M.level[b]);
  const int cells = (NDIM == 3) ? N * N * N : N * N;
  double vmax = 0.0;
  bool bad = false;
  for (int c = threadIdx.x; c < cells; c += blockDim.x) {
    const int i = c % N, j = (c / N) % N, k = (NDIM == 3) ? c / (N * N) : 0;
    const int64_t o = cell_off<NDIM>(i, j, k, N, g);
    double U[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) U[v] = (double)u[v * sv + o];
    if constexpr (NV == 1) vmax = fmax(vmax, inv_dt_adv<NDIM>(M, U[0], dx, bad));
    else vmax = fmax(vmax, inv_dt_cell<NDIM>(U, M.gamma, dx, bad));
  }
  wave_flush(M.scal, vmax, bad);
}

// dt_next = cfl / max_cells(inv dt); advance: t += dt (of the finished step)
__global__ void finalize_kernel(const MeshDev *__restrict__ meshes, int n_meshes, int advance) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_meshes) return;
  double *sc = meshes[m].scal;
  const double mx = sc[kMaxInv];
  const double next = mx > 0.0 ? meshes[m].cfl * (1.0 / mx) : 0.0;
  if (advance) sc[kTime] += sc[kDt];
  sc[kDt] = next;
  sc[kMaxInv] = 0.0;
}

// Flux fixing (Sec. 2.7): one workgroup per coarse block with F2C faces.
// Faces are applied in face order; each coarse face cell is corrected by
// dt_s (F_c - <F_f>) / dx on a + face, dt_s (<F_f> - F_c) / dx on a - face,
// with <F_f> the FP64 pairwise mean of the 2^(d-1) fine fluxes.  In stage 2
// the CFL limit of the corrected cells is then added to the reduction.
template <typename T, int NDIM, int NV>
__global__ __launch_bounds__(256) void fluxfix_kernel(const MeshDev *__restrict__ Mp, int stage, SubStep ss) {
  const MeshDev &M = *Mp;
  constexpr int NF = 2 * NDIM;
  constexpr int PER = 1 << (NDIM - 1);
  const int32_t cb = M.fix_list[blockIdx.x];
  const int N = M.N, H = N / 2, g = M.g, P = N + 2 * g;
  const int64_t sv = (NDIM == 3) ? (int64_t)P * P * P : (int64_t)P * P;
  const int ob = stage >= 3 ? role_buffer(ss.out, M.cur) : (stage == 1 ? 1 - M.cur : M.cur);
  T *uo = (T *)M.s[ob] + (int64_t)cb * sv * NV;
  const double dx = ldexp(M.dx0, -M.level[cb]);
  const double dts = stage >= 3 ? ss.c * M.scal[kDt] : (stage == 1 ? M.scal[kDt] : 0.5 * M.scal[kDt]);
  const int N2 = (NDIM == 3) ? N : 1;
  const int64_t fv = (int64_t)N * N2;  // face values per variable
  const T *bf = (const T *)M.bflux_f;
  const T *bc = (const T *)M.bflux_c;
  // the fine-side flux slots of the face's 2^(d-1) F2C records, read once
  __shared__ int32_t kfs[PER];
  constexpr int B = 2;  // face cells in flight per thread: loads first, then updates
  for (int f = 0; f < NF; f++) {
    const int info = M.face_info[(int64_t)cb * NF + f];
    if (info < 0 || !(info & 1)) continue;
    const int ax = f / 2, side = f % 2;
    const int t1 = (ax == 0) ? 1 : 0, t2 = (NDIM == 3) ? ((ax == 2) ? 1 : 2) : -1;
    const int64_t grp = info >> 1;
    if (threadIdx.x < PER) kfs[threadIdx.x] = M.f2c[4 * (grp * PER + threadIdx.x) + 3];
    __syncthreads();
    const int total = NV * (int)fv;
    for (int e0 = threadIdx.x; e0 < total; e0 += B * blockDim.x) {
      double Fc[B], f0[B], f1[B], f2[B], f3[B], uv[B];
      int64_t o[B];
#pragma unroll
      for (int k = 0; k < B; k++) {
        const int e = e0 + k * blockDim.x;
        o[k] = -1;
        if (e >= total) continue;
        const int p1 = e % N, p2 = (e / N) % N2, v = e / (int)fv;
        const int bt1 = p1 >= H, bt2 = (NDIM == 3) ? (p2 >= H) : 0;
        const int32_t kf = kfs[bt1 + 2 * bt2];
        Fc[k] = (double)bc[(grp * NV + v) * fv + (int64_t)p2 * N + p1];
        const int q1 = 2 * (p1 - bt1 * H), q2 = (NDIM == 3) ? 2 * (p2 - bt2 * H) : 0;
        const T *ff = bf + ((int64_t)kf * NV + v) * fv;
        if (NDIM == 3) {
          f0[k] = (double)ff[(int64_t)q2 * N + q1];
          f1[k] = (double)ff[(int64_t)q2 * N + q1 + 1];
          f2[k] = (double)ff[(int64_t)(q2 + 1) * N + q1];
          f3[k] = (double)ff[(int64_t)(q2 + 1) * N + q1 + 1];
        } else {
          f0[k] = (double)ff[q1];
          f1[k] = (double)ff[q1 + 1];
          f2[k] = f3[k] = 0.0;
        }
        int c[3] = {0, 0, 0};
        c[ax] = side ? N - 1 : 0;
        c[t1] = p1;
        if (t2 >= 0) c[t2] = p2;
        o[k] = (int64_t)v * sv + cell_off<NDIM>(c[0], c[1], c[2], N, g);
        uv[k] = (double)uo[o[k]];
      }
#pragma unroll
      for (int k = 0; k < B; k++) {
        if (o[k] < 0) continue;
        double mean;
        if (NDIM == 3) {
          const double s0 = f0[k] + f1[k];
          const double s1 = f2[k] + f3[k];
          mean = (s0 + s1) * 0.25;
        } else {
          mean = (f0[k] + f1[k]) * 0.5;
        }
        const double corr = side ? dts * (Fc[k] - mean) / dx : dts * (mean - Fc[k]) / dx;
        uo[o[k]] = (T)(uv[k] + corr);
      }
    }
    __syncthreads();
  }
  if (stage != 2 && !(stage >= 3 && ss.epi)) return;
  double vmax = 0.0;
  bool bad = false;
  for (int f = 0; f < NF; f++) {
    const int info = M.face_info[(int64_t)cb * NF + f];
    if (info < 0 || !(info & 1)) continue;
    const int ax = f / 2, side = f % 2;
    const int t1 = (ax == 0) ? 1 : 0, t2 = (NDIM == 3) ? ((ax == 2) ? 1 : 2) : -1;
    for (int e = threadIdx.x; e < (int)fv; e += blockDim.x) {
      const int p1 = e % N, p2 = e / N;
      int c[3] = {0, 0, 0};
      c[ax] = side ? N - 1 : 0;
      c[t1] = p1;
      if (t2 >= 0) c[t2] = p2;
      const int64_t o = cell_off<NDIM>(c[0], c[1], c[2], N, g);
      double U[NV];
#pragma unroll
      for (int v = 0; v < NV; v++) U[v] = (double)uo[v * sv + o];
      if constexpr (NV == 1) vmax = fmax(vmax, inv_dt_adv<NDIM>(M, U[0], dx, bad));
      else vmax = fmax(vmax, inv_dt_cell<NDIM>(U, M.gamma, dx, bad));
    }
  }
  wave_flush(M.scal, vmax, bad);
}

// per-block interior sums of every variable in FP64 times the cell volume
template <typename T, int NDIM, int NV>
__global__ __launch_bounds__(256) void totals_kernel(const MeshDev *__restrict__ Mp, double *part) {
  const MeshDev &M = *Mp;
  __shared__ double red[4][NV];
  const int64_t b = blockIdx.x;
  const int N = M.N, g = M.g, P = N + 2 * g;
  const int64_t sv = (NDIM == 3) ? (int64_t)P * P * P : (int64_t)P * P;
  const T *u = (const T *)M.s[M.cur] + b * sv * NV;
  const int cells = (NDIM == 3) ? N * N * N : N * N;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) acc[v] = 0.0;
  for (int c = threadIdx.x; c < cells; c += blockDim.x) {
    const int i = c % N, j = (c / N) % N, k = (NDIM == 3) ? c / (N * N) : 0;
    const int64_t o = cell_off<NDIM>(i, j, k, N, g);
#pragma unroll
    for (int v = 0; v < NV; v++) acc[v] += (double)u[v * sv + o];
  }
#pragma unroll
  for (int v = 0; v < NV; v++)
    for (int o = 32; o > 0; o >>= 1) acc[v] += __shfl_xor(acc[v], o);
  if ((threadIdx.x & 63) == 0)
    for (int v = 0; v < NV; v++) red[threadIdx.x >> 6][v] = acc[v];
  __syncthreads();
  if (threadIdx.x < NV) {
    const double dx = ldexp(M.dx0, -M.level[b]);
    const double vol = (NDIM == 3) ? dx * dx * dx : dx * dx;
    const int v = threadIdx.x;
    part[b * NV + v] = (((red[0][v] + red[1][v]) + red[2][v]) + red[3][v]) * vol;
  }
}

// fixed-order sum over blocks (one workgroup, deterministic)
__global__ __launch_bounds__(256) void totals_sum_kernel(const double *part, int64_t nb, int nv, double *out) {
  __shared__ double red[256];
  for (int v = 0; v < nv; v++) {
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += 256) s += part[b * nv + v];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = red[0];
    __syncthreads();
  }
}

// Instantiation by (element type, dimension, variables): the Euler system
// (ndim + 2 variables) or scalar advection (one).
#define F4_BY_TYPE(KERNEL, GRID, ...)                                                        \
  do {                                                                                       \
    if (nv == 1) {                                                                           \
      if (ndim == 3) {                                                                       \
        if (f64) KERNEL<double, 3, 1><<<(GRID), 256, 0, s>>>(__VA_ARGS__);                   \
        else KERNEL<float, 3, 1><<<(GRID), 256, 0, s>>>(__VA_ARGS__);                        \
      } else {                                                                               \
        if (f64) KERNEL<double, 2, 1><<<(GRID), 256, 0, s>>>(__VA_ARGS__);                   \
        else KERNEL<float, 2, 1><<<(GRID), 256, 0, s>>>(__VA_ARGS__);                        \
      }                                                                                      \
    } else if (ndim == 3) {                                                                  \
      if (f64) KERNEL<double, 3, 5><<<(GRID), 256, 0, s>>>(__VA_ARGS__);                     \
      else KERNEL<float, 3, 5><<<(GRID), 256, 0, s>>>(__VA_ARGS__);                          \
    } else {                                                                                 \
      if (f64) KERNEL<double, 2, 4><<<(GRID), 256, 0, s>>>(__VA_ARGS__);                     \
      else KERNEL<float, 2, 4><<<(GRID), 256, 0, s>>>(__VA_ARGS__);                          \
    }                                                                                        \
  } while (0)

hipError_t launch_dt_full(const foap4_mesh *m, hipStream_t s) {
  if (m->topo.leaves.empty()) return hipSuccess;
  const unsigned nb = (unsigned)m->topo.leaves.size();
  const bool f64 = m->d.prec == FOAP4_F64;
  const int ndim = m->d.ndim, nv = m->nvar;
  F4_BY_TYPE(dt_full_kernel, nb, m->d_dev);
  return hipGetLastError();
}

hipError_t launch_finalize(const MeshDev *d_meshes, int n_meshes, int advance, hipStream_t s) {
  finalize_kernel<<<(n_meshes + 63) / 64, 64, 0, s>>>(d_meshes, n_meshes, advance);
  return hipGetLastError();
}

hipError_t launch_fluxfix(const MeshDev *d_mesh, int ndim, int nv, bool f64, int n_fix, int stage, hipStream_t s,
                          const SubStep &ss) {
  if (n_fix <= 0) return hipSuccess;
  F4_BY_TYPE(fluxfix_kernel, n_fix, d_mesh, stage, ss);
  return hipGetLastError();
}

// Fixed device scratch of foap4_conserved_totals_noalloc: the per-block
// partial sums of launch_totals.  One copy per GPU, held until the process
// ends; its address on a device comes from hipGetSymbolAddress with that
// device current (the array's name is not a device address in host code).
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  double *p = nullptr;
  const hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

double *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t launch_totals(const foap4_mesh *m, double *d_part, double *d_out, hipStream_t s) {
  const int64_t nb = (int64_t)m->topo.leaves.size();
  if (nb == 0) return hipSuccess;
  const bool f64 = m->d.prec == FOAP4_F64;
  const int ndim = m->d.ndim, nv = m->nvar;
  F4_BY_TYPE(totals_kernel, (unsigned)nb, m->d_dev, d_part);
  totals_sum_kernel<<<1, 256, 0, s>>>(d_part, nb, m->nvar, d_out);
  return hipGetLastError();
}

#undef F4_BY_TYPE

}  // namespace f4
