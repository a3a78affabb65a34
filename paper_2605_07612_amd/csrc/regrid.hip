// Refinement flags (Sec. 3.3) and the data remap after a mesh change (Sec. 2.2).
#include "foap4_internal.h"

namespace f4 {

// Lohner-type criterion of eq. lohner-simple on the density, in FP64 with
// the operation order of the definition and no contraction, so that the
// flags equal a plain evaluation bit for bit.  One workgroup per block.
template <typename T, int NDIM, int NV>
__global__ __launch_bounds__(256) void lohner_kernel(const MeshDev *__restrict__ Mp, double cr2, double cd2,
                                                     double eps, double eps_abs, int8_t *flags,
                                                     const int8_t *skip) {
#pragma clang fp contract(off)
  const MeshDev &M = *Mp;
  const int64_t b = blockIdx.x;
  if (skip && skip[b]) return;
  const int N = M.N, g = M.g, P = N + 2 * g;
  const int64_t sv = (NDIM == 3) ? (int64_t)P * P * P : (int64_t)P * P;
  const T *u = (const T *)M.s[M.cur] + b * sv * NV;  // variable 0 = density
  const int cells = (NDIM == 3) ? N * N * N : N * N;
  bool any_ref = false, all_deref = true;
  for (int c = threadIdx.x; c < cells; c += blockDim.x) {
    const int i = c % N, j = (c / N) % N, k = (NDIM == 3) ? c / (N * N) : 0;
    const double uc = u[cell_off<NDIM>(i, j, k, N, g)];
    double S = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; d++) {
      const int dm[3] = {d == 0, d == 1, d == 2};
      const double um = u[cell_off<NDIM>(i - dm[0], j - dm[1], k - dm[2], N, g)];
      const double up = u[cell_off<NDIM>(i + dm[0], j + dm[1], k + dm[2], N, g)];
      const double num = fabs((um - 2.0 * uc) + up);
      const double den = ((eps_abs + fabs(uc - um)) + fabs(up - uc)) + eps * ((fabs(um) + 2.0 * fabs(uc)) + fabs(up));
      const double E = num / den;
      S = (d == 0) ? E * E : S + E * E;
    }
    any_ref |= S > cr2;
    all_deref &= S < cd2;
  }
  const int r = __syncthreads_or(any_ref ? 1 : 0);
  const int dall = __syncthreads_and(all_deref ? 1 : 0);
  if (threadIdx.x == 0) flags[b] = r ? 1 : (dall ? -1 : 0);
}

// One workgroup per new block: map[n] = (op, src, arg) with op 0 copy old
// block src, op 1 prolong child arg (bits x + 2y + 4z) of old block src with
// limited slopes (old ghosts filled), op 2 restrict old children src..src+2^d-1.
template <typename T, int NDIM, int NV>
__global__ __launch_bounds__(256) void remap_kernel(const T *__restrict__ uold, T *unew, const int32_t *map, int N,
                                                    int g) {
  // FP64 in the operation order of the definitions, no contraction (the
  // prolonged value u_P + corr / 4 stays bit-exact when corr / 4 is subnormal)
#pragma clang fp contract(off)
  const int64_t n = blockIdx.x;
  const int P = N + 2 * g, H = N / 2;
  const int64_t sv = (NDIM == 3) ? (int64_t)P * P * P : (int64_t)P * P;
  const int64_t bel = sv * NV;
  const int op = map[3 * n], src = map[3 * n + 1], arg = map[3 * n + 2];
  const int cells = (NDIM == 3) ? N * N * N : N * N;
  auto at = [&](const int c[3]) -> int64_t { return cell_off<NDIM>(c[0], c[1], c[2], N, g); };
  for (int e = threadIdx.x; e < NV * cells; e += blockDim.x) {
    const int v = e / cells, c0 = e % cells;
    const int c[3] = {c0 % N, (c0 / N) % N, (NDIM == 3) ? c0 / (N * N) : 0};
    double val;
    if (op == 0) {
      val = uold[(int64_t)src * bel + v * sv + at(c)];
    } else if (op == 1) {
      const T *uc = uold + (int64_t)src * bel + v * sv;
      int Pc[3] = {0, 0, 0}, sig[3] = {0, 0, 0};
#pragma unroll
      for (int d = 0; d < NDIM; d++) {
        Pc[d] = ((arg >> d) & 1) * H + (c[d] >> 1);
        sig[d] = (c[d] & 1) ? 1 : -1;
      }
      const double up = uc[at(Pc)];
      double corr = 0.0;
#pragma unroll
      for (int d = 0; d < NDIM; d++) {
        int lo[3] = {Pc[0], Pc[1], Pc[2]}, hi[3] = {Pc[0], Pc[1], Pc[2]};
        lo[d] -= 1;
        hi[d] += 1;
        const double a = up - (double)uc[at(lo)], bb = (double)uc[at(hi)] - up;
        double delta = 0.0;
        if (a > 0.0 && bb > 0.0) delta = a < bb ? a : bb;
        else if (a < 0.0 && bb < 0.0) delta = a > bb ? a : bb;
        const double term = sig[d] > 0 ? delta : -delta;
        corr = (d == 0) ? term : corr + term;
      }
      val = up + 0.25 * corr;
    } else {
      int ch = 0, base[3] = {0, 0, 0};
#pragma unroll
      for (int d = 0; d < NDIM; d++) {
        const int bit = c[d] >= H;
        ch |= bit << d;
        base[d] = 2 * (c[d] - bit * H);
      }
      const T *uq = uold + (int64_t)(src + ch) * bel + v * sv;
      if (NDIM == 2) {
        int q[3] = {base[0], base[1], 0};
        const double f00 = uq[at(q)];
        q[0]++; const double f10 = uq[at(q)];
        q[1]++; const double f11 = uq[at(q)];
        q[0]--; const double f01 = uq[at(q)];
        val = ((f00 + f10) + (f01 + f11)) * 0.25;
      } else {
        double f[2][2][2];
        for (int oz = 0; oz < 2; oz++)
          for (int oy = 0; oy < 2; oy++)
            for (int ox = 0; ox < 2; ox++) {
              const int q[3] = {base[0] + ox, base[1] + oy, base[2] + oz};
              f[oz][oy][ox] = uq[at(q)];
            }
        const double a0 = f[0][0][0] + f[0][0][1], a1 = f[0][1][0] + f[0][1][1];
        const double a2 = f[1][0][0] + f[1][0][1], a3 = f[1][1][0] + f[1][1][1];
        val = ((a0 + a1) + (a2 + a3)) * 0.125;
      }
    }
    unew[n * bel + v * sv + at(c)] = (T)val;
  }
}

// Instantiation by (element type, dimension, variables): the Euler system
// (ndim + 2 variables) or scalar advection (one).
#define F4_BY_TYPE(KERNEL, T_, GRID, ...)                                                 \
  do {                                                                                    \
    if (f64) {                                                                            \
      using T_ = double;                                                                  \
      if (nv == 1) {                                                                      \
        if (ndim == 3) KERNEL<T_, 3, 1><<<(GRID), 256, 0, s>>>(__VA_ARGS__);              \
        else KERNEL<T_, 2, 1><<<(GRID), 256, 0, s>>>(__VA_ARGS__);                        \
      } else if (ndim == 3) KERNEL<T_, 3, 5><<<(GRID), 256, 0, s>>>(__VA_ARGS__);         \
      else KERNEL<T_, 2, 4><<<(GRID), 256, 0, s>>>(__VA_ARGS__);                          \
    } else {                                                                              \
      using T_ = float;                                                                   \
      if (nv == 1) {                                                                      \
        if (ndim == 3) KERNEL<T_, 3, 1><<<(GRID), 256, 0, s>>>(__VA_ARGS__);              \
        else KERNEL<T_, 2, 1><<<(GRID), 256, 0, s>>>(__VA_ARGS__);                        \
      } else if (ndim == 3) KERNEL<T_, 3, 5><<<(GRID), 256, 0, s>>>(__VA_ARGS__);         \
      else KERNEL<T_, 2, 4><<<(GRID), 256, 0, s>>>(__VA_ARGS__);                          \
    }                                                                                     \
  } while (0)

hipError_t launch_lohner(const foap4_mesh *m, int8_t *d_flags, const int8_t *skip, hipStream_t s) {
  const int64_t nb = (int64_t)m->topo.leaves.size();
  if (nb == 0) return hipSuccess;
  const double cr = 5e-2, cd = 6.25e-3;  // c_refine, c_derefine of the AMR runs (Sec. 5.4)
  const double cr2 = cr * cr, cd2 = cd * cd, eps = 1e-2, eps_abs = 1e-10;
  const bool f64 = m->d.prec == FOAP4_F64;
  const int ndim = m->d.ndim, nv = m->nvar;
  F4_BY_TYPE(lohner_kernel, T, (unsigned)nb, m->d_dev, cr2, cd2, eps, eps_abs, d_flags, skip);
  return hipGetLastError();
}

hipError_t launch_remap(const foap4_mesh *m, const void *src_state, void *dst_state, const int32_t *d_map,
                        int64_t nb_new, hipStream_t s) {
  if (nb_new == 0) return hipSuccess;
  const bool f64 = m->d.prec == FOAP4_F64;
  const int N = m->d.block_n, g = m->d.n_ghost;
  const int ndim = m->d.ndim, nv = m->nvar;
  F4_BY_TYPE(remap_kernel, T, (unsigned)nb_new, (const T *)src_state, (T *)dst_state, d_map, N, g);
  return hipGetLastError();
}

#undef F4_BY_TYPE

}  // namespace f4
