// Execution of the stored ghost pattern (Sec. 2.6), one workgroup per record.
//   round R1: SRL records (copy g layers both ways across a face pair),
//             F2C records (coarse ghost = mean of the 2^d fine cells, FP64)
//             and physical boundary faces (Sec. 2.4: Dirichlet / Neumann
//             values reflected through the face, FP64)
//   round R2: C2F records (fine ghost = limited prolongation from the coarse
//             block, FP64 slopes; reads the coarse block's R1 ghosts)
// Work items of several meshes are concatenated (r1_begin / r2_begin).
// NV, the number of variables per cell, is a template parameter: ndim + 2
// for the Euler system, 1 for scalar advection.
#include "foap4_internal.h"

namespace f4 {

template <int NDIM>
struct Geo {
  int N, g, P;
  int64_t sv;  // values per variable
  __device__ Geo(int N_, int g_) : N(N_), g(g_), P(N_ + 2 * g_), sv(NDIM == 3 ? (int64_t)(N_ + 2 * g_) * (N_ + 2 * g_) * (N_ + 2 * g_)
                                                                     : (int64_t)(N_ + 2 * g_) * (N_ + 2 * g_)) {}
  __device__ __forceinline__ int64_t at(const int c[3]) const { return cell_off<NDIM>(c[0], c[1], c[2], N, g); }
};

// Tangential axes of a face with normal AX, in increasing order.  The face
// axis is a template parameter of every record routine, so the small
// coordinate arrays below are indexed statically and stay in registers.
template <int NDIM, int AX>
struct Tang {
  static constexpr int t1 = (AX == 0) ? 1 : 0;
  static constexpr int t2 = (NDIM == 3) ? ((AX == 2) ? 1 : 2) : -1;
};

__device__ __forceinline__ double mm(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

template <typename T, int NDIM, int NV, int N, int ax>
__device__ void srl_record(const MeshDev &M, T *u, int32_t a, int32_t b) {
  constexpr int N2 = (NDIM == 3) ? N : 1;
  const Geo<NDIM> G(N, M.g);
  const int g = M.g;
  constexpr int t1 = Tang<NDIM, ax>::t1, t2 = Tang<NDIM, ax>::t2;
  const int64_t bel = G.sv * NV;
  const int total = 2 * NV * N2 * N * g;
  constexpr int B = 8;  // elements in flight per thread: loads first, then stores
  for (int e0 = threadIdx.x; e0 < total; e0 += B * blockDim.x) {
    T val[B];
    int64_t dsto[B];
#pragma unroll
    for (int q = 0; q < B; q++) {
      const int e = e0 + q * blockDim.x;
      dsto[q] = -1;
      if (e >= total) continue;
      int l, p1, p2, v, side, r = e;
      if (ax == 0) {         // x ghost layers of a row are contiguous in memory: layer fastest
        l = r % g; r /= g;
        p1 = r % N; r /= N;
        p2 = r % N2; r /= N2;
      } else if (ax == 1) {  // rows along x are contiguous, the g ghost rows adjacent
        p1 = r % N; r /= N;
        l = r % g; r /= g;
        p2 = r % N2; r /= N2;
      } else {               // a z ghost plane is N^2 contiguous values: x, then y
        p1 = r % N; r /= N;
        p2 = r % N2; r /= N2;
        l = r % g; r /= g;
      }
      v = r % NV; side = r / NV;
      int src[3] = {0, 0, 0}, dst[3] = {0, 0, 0};
      src[t1] = dst[t1] = p1;
      if constexpr (t2 >= 0) src[t2] = dst[t2] = p2;
      int64_t sb, db;
      if (side == 0) {  // b's -ax ghosts from a's last layers
        src[ax] = N - 1 - l; dst[ax] = -1 - l; sb = a; db = b;
      } else {          // a's +ax ghosts from b's first layers
        src[ax] = l; dst[ax] = N + l; sb = b; db = a;
      }
      val[q] = u[sb * bel + v * G.sv + G.at(src)];
      dsto[q] = db * bel + v * G.sv + G.at(dst);
    }
#pragma unroll
    for (int q = 0; q < B; q++)
      if (dsto[q] >= 0) u[dsto[q]] = val[q];
  }
}

// x faces with two ghost layers: a row's two ghost layers are one aligned
// pair of values on both sides of the copy (the last or first two interior
// cells of the source row, the two x-ghost slots of the destination row), so
// each thread moves pairs with one vector load and one vector store.  Every
// offset is even (N, P, the variable and block strides are even), and state
// buffers are 16-byte aligned.
template <typename T>
struct Pair {
  typedef T type __attribute__((ext_vector_type(2)));
};

template <typename T, int NDIM, int NV, int N>
__device__ void srl_record_x2(const MeshDev &M, T *u, int32_t a, int32_t b) {
  using PT = typename Pair<T>::type;
  constexpr int N2 = (NDIM == 3) ? N : 1;
  constexpr int P = N + 4;
  constexpr int64_t SV = (NDIM == 3) ? (int64_t)P * P * P : (int64_t)P * P;
  constexpr int ROWS = (NDIM == 3) ? P * P : P;
  constexpr int64_t BEL = SV * NV;
  constexpr int total = 2 * NV * N2 * N;
  constexpr int B = 4;  // pairs in flight per thread (8 values): loads first, then stores
  for (int e0 = threadIdx.x; e0 < total; e0 += B * blockDim.x) {
    PT val[B];
    int64_t dsto[B];
#pragma unroll
    for (int q = 0; q < B; q++) {
      const int e = e0 + q * blockDim.x;
      dsto[q] = -1;
      if (e >= total) continue;
      int r = e;
      const int p1 = r % N;  // y: consecutive threads take consecutive rows
      r /= N;
      const int p2 = r % N2;
      r /= N2;
      const int v = r % NV, side = r / NV;
      const int row = (NDIM == 3) ? (p2 + 2) * P + (p1 + 2) : (p1 + 2);
      int64_t src, dst;
      if (side == 0) {  // b's -x ghosts (slots 0, 1) from a's last two cells
        src = a * BEL + v * SV + row * N + (N - 2);
        dst = b * BEL + v * SV + ROWS * N + row * 4;
      } else {          // a's +x ghosts (slots 2, 3) from b's first two cells
        src = b * BEL + v * SV + row * N;
        dst = a * BEL + v * SV + ROWS * N + row * 4 + 2;
      }
      val[q] = *(const PT *)(u + src);
      dsto[q] = dst;
    }
#pragma unroll
    for (int q = 0; q < B; q++)
      if (dsto[q] >= 0) *(PT *)(u + dsto[q]) = val[q];
  }
}

// mean of the 2^d fine cells base + {0,1}^d of block q, summed in pairs
// along x, then y, then z, in FP64
template <typename T, int NDIM>
__device__ __forceinline__ double fine_mean(const T *uq, const Geo<NDIM> &G, const int base[3]) {
  int c[3] = {base[0], base[1], base[2]};
  if (NDIM == 2) {
    const double f00 = uq[G.at(c)];
    c[0]++; const double f10 = uq[G.at(c)];
    c[1]++; const double f11 = uq[G.at(c)];
    c[0]--; const double f01 = uq[G.at(c)];
    return ((f00 + f10) + (f01 + f11)) * 0.25;
  } else {
    double f[2][2][2];
#pragma unroll
    for (int oz = 0; oz < 2; oz++)
#pragma unroll
      for (int oy = 0; oy < 2; oy++)
#pragma unroll
        for (int ox = 0; ox < 2; ox++) {
          const int cc[3] = {base[0] + ox, base[1] + oy, base[2] + oz};
          f[oz][oy][ox] = uq[G.at(cc)];
        }
    const double a0 = f[0][0][0] + f[0][0][1], a1 = f[0][1][0] + f[0][1][1];
    const double a2 = f[1][0][0] + f[1][0][1], a3 = f[1][1][0] + f[1][1][1];
    return ((a0 + a1) + (a2 + a3)) * 0.125;
  }
}

template <typename T, int NDIM, int NV, int N, int ax>
__device__ void f2c_record(const MeshDev &M, T *u, int side, int32_t cb, int32_t q, int32_t h) {
  constexpr int H = N / 2;
  constexpr int H2 = (NDIM == 3) ? H : 1;
  const Geo<NDIM> G(N, M.g);
  const int g = M.g;
  constexpr int t1 = Tang<NDIM, ax>::t1, t2 = Tang<NDIM, ax>::t2;
  const int bt1 = h & 1, bt2 = (h >> 1) & 1;
  const int64_t bel = G.sv * NV;
  const int total = NV * H2 * H * g;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int l, p1, p2, v, r = e;
    if (ax == 0) {
      l = r % g; r /= g;
      p1 = r % H; r /= H;
    } else {
      p1 = r % H; r /= H;
      l = r % g; r /= g;
    }
    p2 = r % H2; v = r / H2;
    const int L = l + 1;
    int cc[3] = {0, 0, 0}, base[3] = {0, 0, 0};
    cc[ax] = side ? N - 1 + L : -L;
    base[ax] = side ? 2 * (L - 1) : N - 2 * L;
    cc[t1] = bt1 * H + p1;
    base[t1] = 2 * p1;
    if constexpr (t2 >= 0) {
      cc[t2] = bt2 * H + p2;
      base[t2] = 2 * p2;
    }
    const double mean = fine_mean<T, NDIM>(u + (int64_t)q * bel + v * G.sv, G, base);
    u[(int64_t)cb * bel + v * G.sv + G.at(cc)] = (T)mean;
  }
}

// limited prolongation (Sec. 2.2) of coarse cell P of block data uc for the
// child whose position is sig (+-1 per axis); slopes and sum in FP64, axes
// summed in order x, y, z.  The stencil (P and its two neighbours per axis)
// is loaded first, so that a thread can keep several in flight.
template <typename T, int NDIM>
struct Stencil {
  T c, lo[NDIM], hi[NDIM];
};

template <typename T, int NDIM>
__device__ __forceinline__ void load_stencil(const T *uc, const Geo<NDIM> &G, const int P[3], Stencil<T, NDIM> &s) {
  s.c = uc[G.at(P)];
#pragma unroll
  for (int d = 0; d < NDIM; d++) {
    int lo[3] = {P[0], P[1], P[2]}, hi[3] = {P[0], P[1], P[2]};
    lo[d] -= 1;
    hi[d] += 1;
    s.lo[d] = uc[G.at(lo)];
    s.hi[d] = uc[G.at(hi)];
  }
}

template <typename T, int NDIM>
__device__ __forceinline__ double prolong(const Stencil<T, NDIM> &s, const int sig[3]) {
  // no contraction: u_P + corr / 4 rounded twice as written, which also
  // holds when corr / 4 is subnormal (where a fused multiply-add would differ)
#pragma clang fp contract(off)
  const double up = s.c;
  double corr = 0.0;
#pragma unroll
  for (int d = 0; d < NDIM; d++) {
    const double delta = mm(up - (double)s.lo[d], (double)s.hi[d] - up);
    const double term = sig[d] > 0 ? delta : -delta;
    corr = (d == 0) ? term : corr + term;
  }
  return up + 0.25 * corr;
}

template <typename T, int NDIM, int NV, int N, int ax>
__device__ void c2f_record(const MeshDev &M, T *u, int side, int32_t q, int32_t cb, int32_t h) {
  constexpr int N2 = (NDIM == 3) ? N : 1;
  constexpr int H = N / 2;
  const Geo<NDIM> G(N, M.g);
  const int g = M.g;
  constexpr int t1 = Tang<NDIM, ax>::t1, t2 = Tang<NDIM, ax>::t2;
  const int bt1 = h & 1, bt2 = (h >> 1) & 1;
  const int64_t bel = G.sv * NV;
  const int total = NV * N2 * N * g;
  // elements in flight per thread, stencils first, then values: two in FP32;
  // in FP64 a second stencil would cost the ghost kernel a wave per SIMD
  constexpr int B = sizeof(T) == 4 ? 2 : 1;
  for (int e0 = threadIdx.x; e0 < total; e0 += B * blockDim.x) {
    Stencil<T, NDIM> st[B];
    int sg[B][3];
    int64_t dsto[B];
#pragma unroll
    for (int k = 0; k < B; k++) {
      const int e = e0 + k * blockDim.x;
      dsto[k] = -1;
      if (e >= total) continue;
      int l, p1, p2, v, r = e;
      if (ax == 0) {
        l = r % g; r /= g;
        p1 = r % N; r /= N;
      } else {
        p1 = r % N; r /= N;
        l = r % g; r /= g;
      }
      p2 = r % N2; v = r / N2;
      const int L = l + 1;
      int fc[3] = {0, 0, 0}, P[3] = {0, 0, 0};
      sg[k][0] = sg[k][1] = sg[k][2] = 0;
      fc[ax] = side ? N - 1 + L : -L;
      const int fn = side ? (L - 1) : (2 * N - L);
      P[ax] = fn >> 1;
      sg[k][ax] = (fn & 1) ? 1 : -1;
      fc[t1] = p1;
      P[t1] = bt1 * H + (p1 >> 1);
      sg[k][t1] = (p1 & 1) ? 1 : -1;
      if constexpr (t2 >= 0) {
        fc[t2] = p2;
        P[t2] = bt2 * H + (p2 >> 1);
        sg[k][t2] = (p2 & 1) ? 1 : -1;
      }
      load_stencil<T, NDIM>(u + (int64_t)cb * bel + v * G.sv, G, P, st[k]);
      dsto[k] = (int64_t)q * bel + v * G.sv + G.at(fc);
    }
#pragma unroll
    for (int k = 0; k < B; k++)
      if (dsto[k] >= 0) u[dsto[k]] = (T)prolong<T, NDIM>(st[k], sg[k]);
  }
}

// Physical boundary face f of block b: ghost layer L = 1..g outside the face
// from the L-th cell inside, 2 u_b - u_in (Dirichlet value u_b) or
// u_in + (2L - 1) dx u'_b (Neumann, outward derivative u'_b); FP64 without
// contraction, rounded once.  u_b / u'_b come from the per-face-cell array
// bc_data (record rec, variable, face cell p1 + N p2) when it is set, else
// from the uniform per-face values.  Each thread keeps B elements in flight
// (loads first, then stores); only the loaded values and the element indices
// stay live between the two passes (the cell coordinates are decoded again),
// which keeps this routine from setting the ghost kernel's register count.
template <typename T, int NDIM, int NV, int N, int ax>
__device__ void bc_record(const MeshDev &M, T *u, int side, int64_t rec, int32_t b) {
#pragma clang fp contract(off)
  constexpr int N2 = (NDIM == 3) ? N : 1;
  const Geo<NDIM> G(N, M.g);
  const int g = M.g, f = 2 * ax + side;
  constexpr int t1 = Tang<NDIM, ax>::t1, t2 = Tang<NDIM, ax>::t2;
  T *ub = u + (int64_t)b * G.sv * NV;
  const double dx = ldexp(M.dx0, -M.level[b]);
  const int total = NV * N2 * N * g;
  // element e -> layer l, face cell (p1, p2), variable v (the SRL copy's orders)
  auto decode = [&](int e, int &l, int &p1, int &p2, int &v) {
    int r = e;
    if (ax == 0) {
      l = r % g; r /= g;
      p1 = r % N; r /= N;
      p2 = r % N2; r /= N2;
    } else if (ax == 1) {
      p1 = r % N; r /= N;
      l = r % g; r /= g;
      p2 = r % N2; r /= N2;
    } else {
      p1 = r % N; r /= N;
      p2 = r % N2; r /= N2;
      l = r % g; r /= g;
    }
    v = r;
  };
  constexpr int B = 4;
  for (int e0 = threadIdx.x; e0 < total; e0 += B * blockDim.x) {
    double uin[B];
#pragma unroll
    for (int q = 0; q < B; q++) {
      const int e = e0 + q * blockDim.x;
      if (e >= total) continue;
      int l, p1, p2, v;
      decode(e, l, p1, p2, v);
      int ic[3] = {0, 0, 0};
      ic[ax] = side ? N - 1 - l : l;
      ic[t1] = p1;
      if constexpr (t2 >= 0) ic[t2] = p2;
      uin[q] = (double)ub[v * G.sv + G.at(ic)];
    }
#pragma unroll
    for (int q = 0; q < B; q++) {
      const int e = e0 + q * blockDim.x;
      if (e >= total) continue;
      int l, p1, p2, v;
      decode(e, l, p1, p2, v);
      const int L = l + 1;
      int gc[3] = {0, 0, 0};
      gc[ax] = side ? N - 1 + L : -L;
      gc[t1] = p1;
      if constexpr (t2 >= 0) gc[t2] = p2;
      const double val = M.bc_data ? M.bc_data[(rec * NV + v) * (N * N2) + p1 + N * p2] : M.bc_val[f][v];
      const double out = (M.bc_type[f][v] == 0) ? 2.0 * val - uin[q] : uin[q] + ((double)(2 * L - 1) * dx) * val;
      ub[v * G.sv + G.at(gc)] = (T)out;
    }
  }
}

// y and z faces: the ghost rows (y) and planes (z) are whole row parts of N
// interior x cells, so each thread moves 16 bytes (4 FP32 or 2 FP64 values
// along x) with one vector load and one vector store.  Every offset is a
// multiple of 16 bytes: N is a multiple of 4, the row part of a row starts
// at row N, the variable stride P^d and the block stride NV P^d are
// multiples of 4 (P = N + 2g is even), and state buffers are 16-byte aligned.
template <typename T>
struct Quad {  // one 16-byte chunk: W values of T (four FP32, two FP64)
  static constexpr int W = 16 / (int)sizeof(T);
  typedef T type __attribute__((ext_vector_type(W)));
};

template <typename T, int NDIM, int NV, int N, int ax>
__device__ void srl_record_rows(const MeshDev &M, T *u, int32_t a, int32_t b) {
  static_assert(ax >= 1 && ax < NDIM, "row copies serve the y and z faces");
  using VT = typename Quad<T>::type;
  constexpr int W = Quad<T>::W, NW = N / W;
  static_assert(N % W == 0, "rows hold whole 16-byte chunks");
  constexpr int N2 = (NDIM == 3) ? N : 1;
  const Geo<NDIM> G(N, M.g);
  const int g = M.g;
  constexpr int t2 = Tang<NDIM, ax>::t2;
  const int64_t bel = G.sv * NV;
  const int total = 2 * NV * N2 * NW * g;
  constexpr int B = 4;  // chunks in flight per thread: loads first, then stores
  for (int e0 = threadIdx.x; e0 < total; e0 += B * blockDim.x) {
    VT val[B];
    int64_t dsto[B];
#pragma unroll
    for (int q = 0; q < B; q++) {
      const int e = e0 + q * blockDim.x;
      dsto[q] = -1;
      if (e >= total) continue;
      int l, p2, r = e;
      const int c = r % NW;  // 16-byte chunk of the row part
      r /= NW;
      if (ax == 1) {  // the g ghost rows of a plane are adjacent
        l = r % g; r /= g;
        p2 = r % N2; r /= N2;
      } else {        // a z ghost plane is N^2 contiguous values
        p2 = r % N2; r /= N2;
        l = r % g; r /= g;
      }
      const int v = r % NV, side = r / NV;
      int src[3] = {c * W, 0, 0}, dst[3] = {c * W, 0, 0};
      if constexpr (t2 >= 0) src[t2] = dst[t2] = p2;
      int64_t sb, db;
      if (side == 0) {  // b's -ax ghosts from a's last layers
        src[ax] = N - 1 - l; dst[ax] = -1 - l; sb = a; db = b;
      } else {          // a's +ax ghosts from b's first layers
        src[ax] = l; dst[ax] = N + l; sb = b; db = a;
      }
      val[q] = *(const VT *)(u + sb * bel + v * G.sv + G.at(src));
      dsto[q] = db * bel + v * G.sv + G.at(dst);
    }
#pragma unroll
    for (int q = 0; q < B; q++)
      if (dsto[q] >= 0) *(VT *)(u + dsto[q]) = val[q];
  }
}

template <typename T, int NDIM, int NV, int N>
__device__ void ghost_item(const MeshDev &M, int round, int64_t r, int which) {
  T *u = (T *)M.s[role_buffer(which, M.cur)];
  // the record's face f = 2 axis + side; the axis selects the routine
#define F4_BY_AXIS(CALL)                           \
  switch (f >> 1) {                                \
    case 0: CALL(0); break;                        \
    case 1: CALL(1); break;                        \
    default: if constexpr (NDIM == 3) CALL(2);     \
  }
  if (round == 1) {
    if (r < M.r1_srl) {
      r = M.srl_sub ? M.srl_sub[r] : r + M.srl_first;
      int f = 1;
      while (r >= M.poff[kSRL][f + 1]) f += 2;
#define F4_SRL(A)                                                          \
  do {                                                                     \
    if constexpr ((A) > 0)                                                 \
      srl_record_rows<T, NDIM, NV, N, A>(M, u, M.srl[2 * r], M.srl[2 * r + 1]); \
    else if (M.g == 2)                                                     \
      srl_record_x2<T, NDIM, NV, N>(M, u, M.srl[2 * r], M.srl[2 * r + 1]); \
    else                                                                   \
      srl_record<T, NDIM, NV, N, A>(M, u, M.srl[2 * r], M.srl[2 * r + 1]); \
  } while (0)
      F4_BY_AXIS(F4_SRL)
#undef F4_SRL
    } else if (r < M.r1_srl + M.pn[kF2C]) {
      r -= M.r1_srl;
      int f = 0;
      while (r >= M.poff[kF2C][f + 1]) f++;
#define F4_F2C(A) f2c_record<T, NDIM, NV, N, A>(M, u, f & 1, M.f2c[4 * r], M.f2c[4 * r + 1], M.f2c[4 * r + 2])
      F4_BY_AXIS(F4_F2C)
#undef F4_F2C
    } else {
      r -= M.r1_srl + M.pn[kF2C];
      int f = 0;
      while (r >= M.poff[kBC][f + 1]) f++;
#define F4_BC(A) bc_record<T, NDIM, NV, N, A>(M, u, f & 1, r, M.bc[r])
      F4_BY_AXIS(F4_BC)
#undef F4_BC
    }
  } else {
    int f = 0;
    while (r >= M.poff[kC2F][f + 1]) f++;
#define F4_C2F(A) c2f_record<T, NDIM, NV, N, A>(M, u, f & 1, M.c2f[3 * r], M.c2f[3 * r + 1], M.c2f[3 * r + 2])
    F4_BY_AXIS(F4_C2F)
#undef F4_C2F
  }
#undef F4_BY_AXIS
}

template <typename T, int NDIM, int NV>
__global__ __launch_bounds__(256) void ghost_kernel(const MeshDev *__restrict__ meshes, int n_meshes,
                                                    int64_t total, int round, int which) {
  // one workgroup per record (grid = total): XCD-aware record order, as
  // workgroup w runs on XCD w mod 8; XCD x takes the contiguous range of
  // records [x q + min(x, r), ...) (total = 8 q + r), so consecutive records,
  // which touch the same blocks (the +x copies of (a, b) and (b, c) both read
  // rows of b), share that XCD's L2.  A bijection onto 0 .. total-1.
  const bool one_each = (int64_t)gridDim.x == total;
  const int64_t xq = total / 8, xr = total % 8, xid = blockIdx.x % 8;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int64_t item = one_each ? xid * xq + (xid < xr ? xid : xr) + w / 8 : w;
    int lo = 0, hi = n_meshes - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      const int64_t b = round == 1 ? meshes[mid].r1_begin : meshes[mid].r2_begin;
      if (b <= item) lo = mid; else hi = mid - 1;
    }
    const MeshDev &M = meshes[lo];
    const int64_t r = item - (round == 1 ? M.r1_begin : M.r2_begin);
    switch (M.N) {
      case 8: ghost_item<T, NDIM, NV, 8>(M, round, r, which); break;
      case 16: ghost_item<T, NDIM, NV, 16>(M, round, r, which); break;
      default: ghost_item<T, NDIM, NV, 32>(M, round, r, which); break;
    }
  }
}

// The x-face SRL copies of one mesh with stored ghosts, by block.  An SRL
// record (a, b) fills b's -x ghosts from a's last g columns and a's +x
// ghosts from b's first g columns; the records that use block b read its rows
// at different times (they are sorted by their first block), so the line or
// lines of a row were fetched twice for 2 g of its cells.  Here one
// workgroup reads each row of its block once, the first and last g cells in
// adjacent lanes, and writes them to the two same-level x neighbours
// (coarse-fine and boundary faces keep their own records).  Each face pair is
// still written exactly once per side.  Used for 3D blocks of 16^3 and 32^3:
// an 8^3 block is too little work for a workgroup, and its records measure
// faster.
template <typename T, int NV, int N>
__device__ void srl_x_block(const MeshDev &M, T *u, int64_t b) {
  constexpr int NF = 6;
  // the block's same-level -x and +x neighbours (-1: none)
  __shared__ int64_t nbr[2];
  if (threadIdx.x < 2) {
    const int32_t f = M.face_info[b * NF + threadIdx.x];
    nbr[threadIdx.x] = f <= -2 ? (int64_t)(-2 - f) : -1;
  }
  __syncthreads();
  if (nbr[0] < 0 && nbr[1] < 0) return;
  const int g = M.g;
  const Geo<3> G(N, g);
  const int64_t bel = G.sv * NV;
  const int per_row = 2 * g;  // the row's first g cells, then its last g
  const int total = NV * N * N * per_row;
  constexpr int B = 8;  // elements in flight per thread: loads first, then stores
  for (int e0 = threadIdx.x; e0 < total; e0 += B * blockDim.x) {
    T val[B];
    int64_t dsto[B];
#pragma unroll
    for (int q = 0; q < B; q++) {
      const int e = e0 + q * blockDim.x;
      dsto[q] = -1;
      if (e >= total) continue;
      int r = e;
      const int c = r % per_row;
      r /= per_row;
      const int p1 = r % N;  // y
      r /= N;
      const int p2 = r % N;  // z
      const int v = r / N;
      const bool lo = c < g;
      const int64_t db = nbr[lo ? 0 : 1];
      if (db < 0) continue;
      const int l = lo ? c : c - g;
      const int src[3] = {lo ? l : N - 1 - l, p1, p2};   // the block's column l, or N - 1 - l
      const int dst[3] = {lo ? N + l : -1 - l, p1, p2};  // the neighbour's ghost across its face
      val[q] = u[b * bel + v * G.sv + G.at(src)];
      dsto[q] = db * bel + v * G.sv + G.at(dst);
    }
#pragma unroll
    for (int q = 0; q < B; q++)
      if (dsto[q] >= 0) u[dsto[q]] = val[q];
  }
}

template <typename T, int NV>
__global__ __launch_bounds__(256) void srl_x_blocks_kernel(const MeshDev *__restrict__ Mp, int64_t nb, int which) {
  const MeshDev &M = *Mp;
  T *u = (T *)M.s[role_buffer(which, M.cur)];
  // XCD-aware block order (workgroup w runs on XCD w mod 8; XCD x takes the
  // contiguous blocks [x q + min(x, r), ...), nb = 8 q + r)
  const int64_t xq = nb / 8, xr = nb % 8, xid = blockIdx.x % 8;
  const int64_t b = xid * xq + (xid < xr ? xid : xr) + blockIdx.x / 8;
  if (M.N == 16) srl_x_block<T, NV, 16>(M, u, b);
  else srl_x_block<T, NV, 32>(M, u, b);
}

hipError_t launch_srl_x_blocks(const MeshDev *d_mesh, int64_t nblocks, int which, int ndim, bool f64, hipStream_t s,
                               int nv) {
  if (nblocks <= 0) return hipSuccess;
  if (ndim != 3) return hipErrorInvalidValue;
  const unsigned nblk = (unsigned)nblocks;
#define F4_XB(T, V) srl_x_blocks_kernel<T, V><<<nblk, 256, 0, s>>>(d_mesh, nblocks, which)
  if (nv == 1) {  // scalar advection
    if (f64) F4_XB(double, 1);
    else F4_XB(float, 1);
  } else if (f64) {
    F4_XB(double, 5);
  } else {
    F4_XB(float, 5);
  }
#undef F4_XB
  return hipGetLastError();
}

hipError_t launch_ghost(const MeshDev *d_meshes, int n_meshes, int64_t total, int round, int which,
                        int ndim, bool f64, int grid, hipStream_t s, int nv) {
  if (total <= 0) return hipSuccess;
  const unsigned nblk = (unsigned)((grid > 0 && grid < total) ? grid : total);
#define F4_GHOST(T, D, V) ghost_kernel<T, D, V><<<nblk, 256, 0, s>>>(d_meshes, n_meshes, total, round, which)
  if (nv == 1) {  // scalar advection
    if (f64) {
      if (ndim == 3) F4_GHOST(double, 3, 1);
      else F4_GHOST(double, 2, 1);
    } else {
      if (ndim == 3) F4_GHOST(float, 3, 1);
      else F4_GHOST(float, 2, 1);
    }
  } else if (f64) {
    if (ndim == 3) F4_GHOST(double, 3, 5);
    else F4_GHOST(double, 2, 4);
  } else {
    if (ndim == 3) F4_GHOST(float, 3, 5);
    else F4_GHOST(float, 2, 4);
  }
#undef F4_GHOST
  return hipGetLastError();
}

}  // namespace f4
