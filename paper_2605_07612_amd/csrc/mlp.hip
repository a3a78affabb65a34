// Learned refinement indicator, an addition to the paper's method that is
// taught by its gradient criterion (Sec. 3.3): per-block features of the
// current state, a 16-64-64-3 MLP whose matrix products run on the gfx950
// matrix cores (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32 accumulation),
// the gradient of its class-weighted cross-entropy, and Adam.
//
// MFMA operand layout (16x32 A times 32x16 B into 16x16 D, 64 lanes, l =
// lane, r = l % 16, q = l / 16): lane l holds A[r][8q + i] and B[8q + i][r]
// for i = 0..7 and receives D[4q + i][r] for i = 0..3.
#include <algorithm>
#include <cmath>

#include "device_common.h"
#include "foap4_internal.h"

namespace f4 {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// fragment ids: forward B operands, then the transposed weights of the
// back-propagation products
enum {
  kFragW1 = 0,    // [nt]      B[k][n] = W1[k][16nt + n], k < 16
  kFragW2 = 4,    // [kt][nt]  B[k][n] = W2[32kt + k][16nt + n]
  kFragW3 = 12,   // [kt]      B[k][n] = W3[32kt + k][n], n < 3
  kFragW3T = 14,  // [nt]      B[k][n] = W3[16nt + n][k], k < 3
  kFragW2T = 18   // [kt][nt]  B[k][n] = W2[16nt + n][32kt + k]
};
static_assert(kFragW2T + 8 == kMlpFrags, "fragment count");

// BF16 bits of x, rounded to nearest even
__device__ inline uint32_t bf16_bits(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return b >> 16;
}
__device__ inline uint32_t pack2(float lo, float hi) { return bf16_bits(lo) | (bf16_bits(hi) << 16); }

__device__ inline f4v mma(u32x4 a, u32x4 b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

// eight BF16 values from a u16 array at stride st, packed as an operand
__device__ inline u32x4 gather8(const uint16_t *p, int st) {
  u32x4 r;
#pragma unroll
  for (int i = 0; i < 4; i++) r[i] = (uint32_t)p[(2 * i) * st] | ((uint32_t)p[(2 * i + 1) * st] << 16);
  return r;
}

// ------------------------------------------------------------------ features

// Density and pressure of one cell: FP64 states in the operation order of the
// definition (v = m / rho, ke = sum m v, p = (gamma-1)(E - ke/2), no
// contraction), FP32 states in FP32 with the hardware reciprocal.
template <typename T, int NDIM>
__device__ __forceinline__ void rho_p(const T *u, int64_t sv, int64_t o, double gm1, T &rho, T &p) {
#pragma clang fp contract(off)
  constexpr int NV = NDIM + 2;
  rho = gload(u + o);
  T ke = T(0);
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int d = 0; d < NDIM; d++) {
      const T md = gload(u + (1 + d) * sv + o);
      const T v = md / rho;
      ke = ke + md * v;
    }
    p = (T)gm1 * (gload(u + (NV - 1) * sv + o) - T(0.5) * ke);
  } else {
    const T ir = __builtin_amdgcn_rcpf(rho);
#pragma unroll
    for (int d = 0; d < NDIM; d++) {
      const T md = gload(u + (1 + d) * sv + o);
      ke = ke + md * (md * ir);
    }
    p = (T)gm1 * (gload(u + (NV - 1) * sv + o) - T(0.5) * ke);
  }
}

// r0, r1 of every block: one workgroup per block marches over the planes;
// density and pressure of plane k (interior and the one-cell face ring from
// the ghost cells) go to LDS for the x/y differences, each thread keeps its
// own cells' planes k-1, k, k+1 in registers for the z differences, so every
// cell is converted once.  Differences, squares (summed x, y, z) and the
// maxima follow the definition; FP64 states give the plain evaluation's
// values bit for bit.
template <typename T, int NDIM>
__global__ __launch_bounds__(256) void raw_features_kernel(const MeshDev *__restrict__ Mp, double *raw) {
#pragma clang fp contract(off)
  const MeshDev &M = *Mp;
  constexpr int NV = NDIM + 2;
  constexpr int CPT = 4;      // own cells per thread (N <= 32)
  constexpr int LW = 34;      // LDS row: N + 2 <= 34
  __shared__ T pl[2][2][LW * LW];  // [buffer][rho, p][cell]
  __shared__ double red[2][256];
  const int64_t b = blockIdx.x;
  const int N = M.N, g = M.g, P = N + 2 * g, L = N + 2;
  const int64_t sv = (NDIM == 3) ? (int64_t)P * P * P : (int64_t)P * P;
  const T *u = (const T *)M.s[M.cur] + b * sv * NV;
  const double gm1 = M.gamma - 1.0;
  const int nk = (NDIM == 3) ? N : 1;
  auto at = [&](int i, int j, int k) -> int64_t { return cell_off<NDIM>(i, j, k, N, g); };
  const int ncell = N * N;
  // own cells c = tid + 256 m, m < CPT, c < N*N
  T r0[CPT], p0[CPT], r1[CPT], p1[CPT], r2[CPT], p2[CPT];  // planes k-1, k, k+1
#pragma unroll
  for (int m = 0; m < CPT; m++) {
    const int c = threadIdx.x + 256 * m;
    r0[m] = p0[m] = r1[m] = p1[m] = T(1);
    if (c < ncell) {
      if (NDIM == 3) rho_p<T, NDIM>(u, sv, at(c % N, c / N, -1), gm1, r0[m], p0[m]);
      rho_p<T, NDIM>(u, sv, at(c % N, c / N, 0), gm1, r1[m], p1[m]);
    }
  }
  double best_r = 0.0, best_p = 0.0;
  for (int k = 0; k < nk; k++) {
    T *R = pl[k & 1][0], *Pp = pl[k & 1][1];
    // plane k into LDS: own cells, then the face ring (ghost cells)
#pragma unroll
    for (int m = 0; m < CPT; m++) {
      const int c = threadIdx.x + 256 * m;
      if (c < ncell) {
        const int o = (c / N + 1) * L + (c % N + 1);
        R[o] = r1[m];
        Pp[o] = p1[m];
      }
    }
    if ((int)threadIdx.x < 4 * N) {
      const int side = threadIdx.x / N, t = threadIdx.x % N;
      const int i = side == 0 ? -1 : side == 1 ? N : t, j = side < 2 ? t : (side == 2 ? -1 : N);
      T rr, pp;
      rho_p<T, NDIM>(u, sv, at(i, j, k), gm1, rr, pp);
      R[(j + 1) * L + (i + 1)] = rr;
      Pp[(j + 1) * L + (i + 1)] = pp;
    }
    // own cells of plane k + 1 for the z differences
    if constexpr (NDIM == 3) {
#pragma unroll
      for (int m = 0; m < CPT; m++) {
        const int c = threadIdx.x + 256 * m;
        r2[m] = p2[m] = T(1);
        if (c < ncell) rho_p<T, NDIM>(u, sv, at(c % N, c / N, k + 1), gm1, r2[m], p2[m]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < CPT; m++) {
      const int c = threadIdx.x + 256 * m;
      if (c < ncell) {
        const int o = (c / N + 1) * L + (c % N + 1);
        const T hf = T(0.5);
        const T drx = hf * (R[o + 1] - R[o - 1]), dpx = hf * (Pp[o + 1] - Pp[o - 1]);
        const T dry = hf * (R[o + L] - R[o - L]), dpy = hf * (Pp[o + L] - Pp[o - L]);
        T sr = drx * drx, sp = dpx * dpx;
        sr = sr + dry * dry;
        sp = sp + dpy * dpy;
        if constexpr (NDIM == 3) {
          const T drz = hf * (r2[m] - r0[m]), dpz = hf * (p2[m] - p0[m]);
          sr = sr + drz * drz;
          sp = sp + dpz * dpz;
        }
        double gr, gp;
        if constexpr (sizeof(T) == 8) {
          gr = sqrt(sr) / r1[m];
          gp = sqrt(sp) / p1[m];
        } else {
          gr = (double)(__builtin_amdgcn_sqrtf(sr) * __builtin_amdgcn_rcpf(r1[m]));
          gp = (double)(__builtin_amdgcn_sqrtf(sp) * __builtin_amdgcn_rcpf(p1[m]));
        }
        if (gr > best_r) best_r = gr;
        if (gp > best_p) best_p = gp;
      }
    }
    if constexpr (NDIM == 3) {
#pragma unroll
      for (int m = 0; m < CPT; m++) {
        r0[m] = r1[m];
        p0[m] = p1[m];
        r1[m] = r2[m];
        p1[m] = p2[m];
      }
    }
    // the other LDS buffer is written next; this one is reused two planes on
  }
  red[0][threadIdx.x] = best_r;
  red[1][threadIdx.x] = best_p;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      const double a = red[0][threadIdx.x + h], q = red[1][threadIdx.x + h];
      if (a > red[0][threadIdx.x]) red[0][threadIdx.x] = a;
      if (q > red[1][threadIdx.x]) red[1][threadIdx.x] = q;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    raw[2 * b] = red[0][0];
    raw[2 * b + 1] = red[1][0];
  }
}

// 16 features per block from the raw maxima of the block and of its face
// neighbours (face_info: -2 - n same level, 2 slot coarser neighbour = the
// coarse block of C2F record slot, 2 slot + 1 finer neighbours = the fine
// blocks of F2C records slot * 2^(d-1) ...).  One thread per block.
__global__ void assemble_features_kernel(const MeshDev *__restrict__ Mp, int ndim, double lmax,
                                         const double *__restrict__ raw, float *feat) {
  const MeshDev &M = *Mp;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= M.nb) return;
  const int nf = 2 * ndim, per = 1 << (ndim - 1);
  float F[16];
  F[0] = (float)log1p(raw[2 * b]);
  F[1] = (float)log1p(raw[2 * b + 1]);
  F[2] = (float)((double)M.level[b] / lmax);
#pragma unroll
  for (int f = 0; f < 6; f++) {
    double a0 = 0.0, a1 = 0.0;
    if (f < nf) {
      const int32_t info = M.face_info[b * nf + f];
      if (info <= -2) {
        const int64_t n = -2 - (int64_t)info;
        a0 = log1p(raw[2 * n]);
        a1 = log1p(raw[2 * n + 1]);
      } else if (info >= 0 && !(info & 1)) {
        const int64_t c = M.c2f[3 * (int64_t)(info >> 1) + 1];
        a0 = log1p(raw[2 * c]);
        a1 = log1p(raw[2 * c + 1]);
      } else if (info >= 0) {
        const int64_t base = (int64_t)(info >> 1) * per;
        for (int h = 0; h < per; h++) {
          const int64_t q = M.f2c[4 * (base + h) + 1];
          const double l0 = log1p(raw[2 * q]), l1 = log1p(raw[2 * q + 1]);
          a0 = (h == 0 || l0 > a0) ? l0 : a0;
          a1 = (h == 0 || l1 > a1) ? l1 : a1;
        }
      }
    }
    F[3 + 2 * f] = (float)a0;
    F[4 + 2 * f] = (float)a1;
  }
  F[15] = 0.0f;
  float4 *o = (float4 *)(feat + 16 * b);
#pragma unroll
  for (int v = 0; v < 4; v++) o[v] = make_float4(F[4 * v], F[4 * v + 1], F[4 * v + 2], F[4 * v + 3]);
}

// ---------------------------------------------------------------- the network

// B operand value k, n of fragment id (see the enum above)
__device__ inline float frag_value(const float *w, int id, int k, int n) {
  if (id < kFragW2) return k < 16 ? w[kOffW1 + k * 64 + 16 * id + n] : 0.0f;
  if (id < kFragW3) {
    const int kt = (id - kFragW2) >> 2, nt = (id - kFragW2) & 3;
    return w[kOffW2 + (32 * kt + k) * 64 + 16 * nt + n];
  }
  if (id < kFragW3T) return n < 3 ? w[kOffW3 + (32 * (id - kFragW3) + k) * 3 + n] : 0.0f;
  if (id < kFragW2T) return k < 3 ? w[kOffW3 + (16 * (id - kFragW3T) + n) * 3 + k] : 0.0f;
  const int kt = (id - kFragW2T) >> 2, nt = (id - kFragW2T) & 3;
  return w[kOffW2 + (16 * nt + n) * 64 + 32 * kt + k];
}

// BF16 operand fragments of the current FP32 weights: thread = (id, lane)
__global__ void pack_kernel(const float *__restrict__ w, u32x4 *frag) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kMlpFrags * 64) return;
  const int id = t >> 6, lane = t & 63, r = lane & 15, q = lane >> 4;
  u32x4 v;
#pragma unroll
  for (int i = 0; i < 4; i++)
    v[i] = pack2(frag_value(w, id, 8 * q + 2 * i, r), frag_value(w, id, 8 * q + 2 * i + 1, r));
  frag[t] = v;
}

struct MlpArgs {
  const float *x;        // [n][16] features
  const int8_t *y;       // [n] labels -1, 0, +1 (training)
  int64_t n;
  const u32x4 *frag;     // [kMlpFrags][64]
  const float *w;        // FP32 parameters (biases)
  const float *cls;      // per-class sample weight (training)
  float *logits;         // [n][3] or null
  int8_t *flags;         // decisions or null
  int8_t *decided;
  float thr;
  float *part;           // [gridDim.x][kMlpPartStride] (training)
};

constexpr int kRow = 72;  // LDS row stride (u16) of a 32 x 64 activation tile

struct WaveTiles {
  uint16_t xs[32 * 16];    // BF16 input rows
  uint16_t ha[32 * kRow];  // h1, then dz1
  uint16_t hb[32 * kRow];  // h2, then dz2
  uint16_t d3[32 * 16];    // BF16 dz3, classes 3..15 zero
  float zf[32 * 4];        // logits
};
constexpr int kMlpSmem = (4 * (int)sizeof(WaveTiles) > (kMlpPartStride * 4)) ? 4 * (int)sizeof(WaveTiles)
                                                                              : kMlpPartStride * 4;

// Each wave takes chunks of 32 rows; the workgroup's four waves take four
// consecutive chunks per round, and every wave of a workgroup runs the same
// number of rounds (rows past n carry zero weight), so the barriers between
// phases are uniform.  TRAIN: forward, softmax cross-entropy, backward with
// the gradient accumulated in registers, then the workgroup's partial
// gradient written to part[blockIdx.x] (waves summed in a fixed order).
template <bool TRAIN>
__global__ __launch_bounds__(256) void mlp_kernel(MlpArgs A) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[kMlpSmem];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  WaveTiles &L = ((WaveTiles *)smem)[wv];
  const int64_t nchunk = (A.n + 31) / 32;
  const u32x4 *Fg = A.frag + lane;

  for (int e = lane; e < 32 * 16; e += 64) L.d3[e] = 0;
  f4v gw1[4], gw2[16], gw3[4];
  float gb1[4], gb2[4], gb3[3] = {0.0f, 0.0f, 0.0f}, gloss = 0.0f;
#pragma unroll
  for (int t = 0; t < 4; t++) {
    gw1[t] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
    gw3[t] = gw1[t];
    gb1[t] = gb2[t] = 0.0f;
  }
#pragma unroll
  for (int t = 0; t < 16; t++) gw2[t] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
  __syncthreads();

  for (int64_t grp = blockIdx.x; grp * 4 < nchunk; grp += gridDim.x) {
    const int64_t s0 = (grp * 4 + wv) * 32;
    // ---- layer 1: A from the input rows (columns 16..31 are zero padding)
    u32x4 ax[2];
#pragma unroll
    for (int mt = 0; mt < 2; mt++) {
      const int64_t s = s0 + 16 * mt + r;
      u32x4 a = {0u, 0u, 0u, 0u};
      if (q < 2 && s < A.n) {
        const float4 *p = (const float4 *)(A.x + s * 16 + 8 * q);
        const float4 v0 = p[0], v1 = p[1];
        a = u32x4{pack2(v0.x, v0.y), pack2(v0.z, v0.w), pack2(v1.x, v1.y), pack2(v1.z, v1.w)};
      }
      ax[mt] = a;
      if (TRAIN && q < 2) *(u32x4 *)&L.xs[(16 * mt + r) * 16 + 8 * q] = a;
    }
    f4v z1[2][4];
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      const u32x4 bw = Fg[(kFragW1 + nt) * 64];
      const float bias = A.w[kOffB1 + 16 * nt + r];
#pragma unroll
      for (int mt = 0; mt < 2; mt++) {
        z1[mt][nt] = mma(ax[mt], bw, f4v{0.0f, 0.0f, 0.0f, 0.0f});
#pragma unroll
        for (int i = 0; i < 4; i++) {
          z1[mt][nt][i] += bias;
          L.ha[(16 * mt + 4 * q + i) * kRow + 16 * nt + r] = (uint16_t)bf16_bits(fmaxf(z1[mt][nt][i], 0.0f));
        }
      }
    }
    __syncthreads();
    // ---- layer 2
    f4v z2[2][4];
#pragma unroll
    for (int mt = 0; mt < 2; mt++)
#pragma unroll
      for (int nt = 0; nt < 4; nt++) z2[mt][nt] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kt = 0; kt < 2; kt++) {
      u32x4 bw[4];
#pragma unroll
      for (int nt = 0; nt < 4; nt++) bw[nt] = Fg[(kFragW2 + 4 * kt + nt) * 64];
#pragma unroll
      for (int mt = 0; mt < 2; mt++) {
        const u32x4 a = *(const u32x4 *)&L.ha[(16 * mt + r) * kRow + 32 * kt + 8 * q];
#pragma unroll
        for (int nt = 0; nt < 4; nt++) z2[mt][nt] = mma(a, bw[nt], z2[mt][nt]);
      }
    }
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      const float bias = A.w[kOffB2 + 16 * nt + r];
#pragma unroll
      for (int mt = 0; mt < 2; mt++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          z2[mt][nt][i] += bias;
          L.hb[(16 * mt + 4 * q + i) * kRow + 16 * nt + r] = (uint16_t)bf16_bits(fmaxf(z2[mt][nt][i], 0.0f));
        }
    }
    __syncthreads();
    // ---- layer 3 (classes padded to 16)
    {
      f4v z3[2] = {f4v{0.0f, 0.0f, 0.0f, 0.0f}, f4v{0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
      for (int kt = 0; kt < 2; kt++) {
        const u32x4 bw = Fg[(kFragW3 + kt) * 64];
#pragma unroll
        for (int mt = 0; mt < 2; mt++)
          z3[mt] = mma(*(const u32x4 *)&L.hb[(16 * mt + r) * kRow + 32 * kt + 8 * q], bw, z3[mt]);
      }
      if (r < 3) {
        const float bias = A.w[kOffB3 + r];
#pragma unroll
        for (int mt = 0; mt < 2; mt++)
#pragma unroll
          for (int i = 0; i < 4; i++) L.zf[(16 * mt + 4 * q + i) * 4 + r] = z3[mt][i] + bias;
      }
    }
    __syncthreads();
    // ---- softmax per row, lanes 0..31
    if (lane < 32) {
      const int64_t s = s0 + lane;
      const float za = L.zf[lane * 4], zb = L.zf[lane * 4 + 1], zc = L.zf[lane * 4 + 2];
      const float zm = fmaxf(za, fmaxf(zb, zc));
      const float ea = expf(za - zm), eb = expf(zb - zm), ec = expf(zc - zm);
      const float sum = ea + eb + ec;
      if (!TRAIN) {
        if (s < A.n) {
          if (A.logits) {
            A.logits[3 * s] = za;
            A.logits[3 * s + 1] = zb;
            A.logits[3 * s + 2] = zc;
          }
          if (A.flags) {
            int c = 0;
            float best = za;
            if (zb > best) { c = 1; best = zb; }
            if (zc > best) c = 2;
            const bool ok = 1.0f / sum >= A.thr;
            A.decided[s] = ok ? 1 : 0;
            if (ok) A.flags[s] = (int8_t)(c - 1);
          }
        }
      } else {
        int c = 0;
        float wt = 0.0f;
        if (s < A.n) {
          const int lab = A.y[s] + 1;
          if (lab >= 0 && lab <= 2) {
            c = lab;
            wt = A.cls[c];
          }
        }
        const float inv = 1.0f / sum;
        const float d0 = (ea * inv - (c == 0 ? 1.0f : 0.0f)) * wt;
        const float d1 = (eb * inv - (c == 1 ? 1.0f : 0.0f)) * wt;
        const float d2 = (ec * inv - (c == 2 ? 1.0f : 0.0f)) * wt;
        const float zt = c == 0 ? za : (c == 1 ? zb : zc);
        gloss += wt * (logf(sum) - (zt - zm));
        gb3[0] += d0;
        gb3[1] += d1;
        gb3[2] += d2;
        L.d3[lane * 16] = (uint16_t)bf16_bits(d0);
        L.d3[lane * 16 + 1] = (uint16_t)bf16_bits(d1);
        L.d3[lane * 16 + 2] = (uint16_t)bf16_bits(d2);
      }
    }
    if (!TRAIN) {
      __syncthreads();
      continue;
    }
    __syncthreads();
    // ---- dW3 += H2^T dZ3 (M = hidden, N = class, K = row)
    {
      const u32x4 bd = gather8(&L.d3[(8 * q) * 16 + r], 16);
#pragma unroll
      for (int mt = 0; mt < 4; mt++) gw3[mt] = mma(gather8(&L.hb[(8 * q) * kRow + 16 * mt + r], kRow), bd, gw3[mt]);
    }
    // ---- dH2 = dZ3 W3^T (K = class, only 0..2 non-zero), dZ2 = dH2 where z2 > 0
    f4v dz[2][4];
#pragma unroll
    for (int mt = 0; mt < 2; mt++) {
      const u32x4 a = (q == 0) ? *(const u32x4 *)&L.d3[(16 * mt + r) * 16] : u32x4{0u, 0u, 0u, 0u};
#pragma unroll
      for (int nt = 0; nt < 4; nt++) {
        const f4v dh = mma(a, Fg[(kFragW3T + nt) * 64], f4v{0.0f, 0.0f, 0.0f, 0.0f});
#pragma unroll
        for (int i = 0; i < 4; i++) {
          dz[mt][nt][i] = z2[mt][nt][i] > 0.0f ? dh[i] : 0.0f;
          gb2[nt] += dz[mt][nt][i];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < 2; mt++)
#pragma unroll
      for (int nt = 0; nt < 4; nt++)
#pragma unroll
        for (int i = 0; i < 4; i++) L.hb[(16 * mt + 4 * q + i) * kRow + 16 * nt + r] = (uint16_t)bf16_bits(dz[mt][nt][i]);
    __syncthreads();
    // ---- dW2 += H1^T dZ2 (M = hidden 1, N = hidden 2, K = row)
    {
      u32x4 bd[4];
#pragma unroll
      for (int nt = 0; nt < 4; nt++) bd[nt] = gather8(&L.hb[(8 * q) * kRow + 16 * nt + r], kRow);
#pragma unroll
      for (int mt = 0; mt < 4; mt++) {
        const u32x4 a = gather8(&L.ha[(8 * q) * kRow + 16 * mt + r], kRow);
#pragma unroll
        for (int nt = 0; nt < 4; nt++) gw2[4 * mt + nt] = mma(a, bd[nt], gw2[4 * mt + nt]);
      }
    }
    // ---- dH1 = dZ2 W2^T, dZ1 = dH1 where z1 > 0
#pragma unroll
    for (int mt = 0; mt < 2; mt++)
#pragma unroll
      for (int nt = 0; nt < 4; nt++) dz[mt][nt] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kt = 0; kt < 2; kt++) {
      u32x4 bw[4];
#pragma unroll
      for (int nt = 0; nt < 4; nt++) bw[nt] = Fg[(kFragW2T + 4 * kt + nt) * 64];
#pragma unroll
      for (int mt = 0; mt < 2; mt++) {
        const u32x4 a = *(const u32x4 *)&L.hb[(16 * mt + r) * kRow + 32 * kt + 8 * q];
#pragma unroll
        for (int nt = 0; nt < 4; nt++) dz[mt][nt] = mma(a, bw[nt], dz[mt][nt]);
      }
    }
#pragma unroll
    for (int mt = 0; mt < 2; mt++)
#pragma unroll
      for (int nt = 0; nt < 4; nt++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          dz[mt][nt][i] = z1[mt][nt][i] > 0.0f ? dz[mt][nt][i] : 0.0f;
          gb1[nt] += dz[mt][nt][i];
        }
    __syncthreads();
#pragma unroll
    for (int mt = 0; mt < 2; mt++)
#pragma unroll
      for (int nt = 0; nt < 4; nt++)
#pragma unroll
        for (int i = 0; i < 4; i++) L.ha[(16 * mt + 4 * q + i) * kRow + 16 * nt + r] = (uint16_t)bf16_bits(dz[mt][nt][i]);
    __syncthreads();
    // ---- dW1 += X^T dZ1 (M = feature, N = hidden 1, K = row)
    {
      const u32x4 a = gather8(&L.xs[(8 * q) * 16 + r], 16);
#pragma unroll
      for (int nt = 0; nt < 4; nt++) gw1[nt] = mma(a, gather8(&L.ha[(8 * q) * kRow + 16 * nt + r], kRow), gw1[nt]);
    }
    __syncthreads();
  }
  if (!TRAIN) return;

  // bias sums over the four row groups of a column, class sums and the loss
  // over all lanes; xor butterflies leave the same value in every lane
#pragma unroll
  for (int t = 0; t < 4; t++) {
    gb1[t] += __shfl_xor(gb1[t], 16);
    gb1[t] += __shfl_xor(gb1[t], 32);
    gb2[t] += __shfl_xor(gb2[t], 16);
    gb2[t] += __shfl_xor(gb2[t], 32);
  }
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    gb3[0] += __shfl_xor(gb3[0], m);
    gb3[1] += __shfl_xor(gb3[1], m);
    gb3[2] += __shfl_xor(gb3[2], m);
    gloss += __shfl_xor(gloss, m);
  }
  float *red = (float *)smem;
  for (int w = 0; w < 4; w++) {
    if (wv == w) {
      auto put = [&](int idx, float v) { red[idx] = (w == 0) ? v : red[idx] + v; };
#pragma unroll
      for (int nt = 0; nt < 4; nt++)
#pragma unroll
        for (int i = 0; i < 4; i++) put(kOffW1 + (4 * q + i) * 64 + 16 * nt + r, gw1[nt][i]);
#pragma unroll
      for (int mt = 0; mt < 4; mt++)
#pragma unroll
        for (int nt = 0; nt < 4; nt++)
#pragma unroll
          for (int i = 0; i < 4; i++) put(kOffW2 + (16 * mt + 4 * q + i) * 64 + 16 * nt + r, gw2[4 * mt + nt][i]);
      if (r < 3) {
#pragma unroll
        for (int mt = 0; mt < 4; mt++)
#pragma unroll
          for (int i = 0; i < 4; i++) put(kOffW3 + (16 * mt + 4 * q + i) * 3 + r, gw3[mt][i]);
      }
      if (q == 0) {
#pragma unroll
        for (int nt = 0; nt < 4; nt++) {
          put(kOffB1 + 16 * nt + r, gb1[nt]);
          put(kOffB2 + 16 * nt + r, gb2[nt]);
        }
      }
      if (lane == 0) {
        put(kOffB3, gb3[0]);
        put(kOffB3 + 1, gb3[1]);
        put(kOffB3 + 2, gb3[2]);
        put(kMlpParams, gloss);
      }
    }
    __syncthreads();
  }
  for (int p = threadIdx.x; p <= kMlpParams; p += blockDim.x) A.part[(int64_t)blockIdx.x * kMlpPartStride + p] = red[p];
}

// Sum of the workgroup partials in FP64 in workgroup order, then (update)
// one Adam step on the FP32 master weights with FP64 moments.
__global__ void reduce_adam_kernel(const float *__restrict__ part, int groups, float *w, double *mv, float *grad,
                                   double *loss, int update, double lr, double bc1, double bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kMlpParams) return;
  double s = 0.0;
  for (int g = 0; g < groups; g++) s += (double)part[(int64_t)g * kMlpPartStride + p];
  if (p == kMlpParams) {
    if (loss) *loss = s;
    return;
  }
  if (grad) grad[p] = (float)s;
  if (!update) return;
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const double m = b1 * mv[p] + (1.0 - b1) * s;
  const double v = b2 * mv[kMlpParams + p] + (1.0 - b2) * s * s;
  mv[p] = m;
  mv[kMlpParams + p] = v;
  const double mh = m / bc1, vh = v / bc2;
  w[p] = (float)((double)w[p] - lr * mh / (sqrt(vh) + eps));
}

__global__ void count_labels_kernel(const int8_t *__restrict__ y, int64_t n, unsigned long long *cnt) {
  unsigned long long c[4] = {0, 0, 0, 0};
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
    const int lab = y[s] + 1;
    c[(lab >= 0 && lab <= 2) ? lab : 3]++;
  }
#pragma unroll
  for (int k = 0; k < 4; k++) {
    unsigned long long v = c[k];
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(&cnt[k], v);
  }
}

// ------------------------------------------------------------------ launchers

hipError_t launch_block_features(const foap4_mesh *m, double *d_raw, float *d_feat, hipStream_t s) {
  const int64_t nb = (int64_t)m->topo.leaves.size();
  if (nb == 0) return hipSuccess;
  const bool f64 = m->d.prec == FOAP4_F64;
  if (m->d.ndim == 3) {
    if (f64) raw_features_kernel<double, 3><<<(unsigned)nb, 256, 0, s>>>(m->d_dev, d_raw);
    else raw_features_kernel<float, 3><<<(unsigned)nb, 256, 0, s>>>(m->d_dev, d_raw);
  } else {
    if (f64) raw_features_kernel<double, 2><<<(unsigned)nb, 256, 0, s>>>(m->d_dev, d_raw);
    else raw_features_kernel<float, 2><<<(unsigned)nb, 256, 0, s>>>(m->d_dev, d_raw);
  }
  const hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch_assemble_features(m, d_raw, d_feat, s);
}

hipError_t launch_assemble_features(const foap4_mesh *m, const double *d_raw, float *d_feat, hipStream_t s) {
  const int64_t nb = (int64_t)m->topo.leaves.size();
  if (nb == 0) return hipSuccess;
  const double lmax = (double)(m->d.max_level > 1 ? m->d.max_level : 1);
  assemble_features_kernel<<<(unsigned)((nb + 255) / 256), 256, 0, s>>>(m->d_dev, m->d.ndim, lmax, d_raw, d_feat);
  return hipGetLastError();
}

static MlpArgs base_args(const foap4_mlp *net, const float *x, int64_t n) {
  MlpArgs A{};
  A.x = x;
  A.n = n;
  A.frag = (const u32x4 *)net->d_frag;
  A.w = net->d_w;
  A.cls = net->d_cls;
  return A;
}

static unsigned forward_grid(int64_t n) {
  const int64_t groups = (n + 127) / 128;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(groups, 2048));
}

hipError_t launch_mlp_decide(const foap4_mlp *net, const float *d_feat, int64_t n, int8_t *d_flags,
                             int8_t *d_decided, hipStream_t s) {
  if (n == 0) return hipSuccess;
  MlpArgs A = base_args(net, d_feat, n);
  A.flags = d_flags;
  A.decided = d_decided;
  A.thr = net->threshold;
  mlp_kernel<false><<<forward_grid(n), 256, 0, s>>>(A);
  return hipGetLastError();
}

}  // namespace f4

using namespace f4;

static foap4_status mlp_fail(foap4_mlp *net, foap4_status st, const std::string &msg) {
  fail(nullptr, st, msg);
  if (net) net->err = msg;
  return st;
}
#define M_HIP(net, call)                                                                          \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess) return mlp_fail((net), FOAP4_E_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

extern "C" {

foap4_status foap4_mlp_create(void *hip_stream, foap4_mlp **out) {
  if (!out) return mlp_fail(nullptr, FOAP4_E_INVALID, "null output pointer");
  *out = nullptr;
  foap4_mlp *net = new foap4_mlp();
  net->stream = (hipStream_t)hip_stream;
  if (hipMalloc((void **)&net->d_w, kMlpParams * 4) != hipSuccess ||
      hipMalloc((void **)&net->d_mv, 2 * kMlpParams * 8) != hipSuccess ||
      hipMalloc((void **)&net->d_grad, kMlpParams * 4) != hipSuccess ||
      hipMalloc(&net->d_frag, kMlpFrags * 64 * 16) != hipSuccess ||
      hipMalloc((void **)&net->d_cls, 4 * 4) != hipSuccess ||
      hipMalloc((void **)&net->d_cnt, 4 * 8) != hipSuccess) {
    foap4_mlp_destroy(net);
    return mlp_fail(nullptr, FOAP4_E_HIP, "device allocation failed");
  }
  *out = net;
  return FOAP4_OK;
}

foap4_status foap4_mlp_destroy(foap4_mlp *net) {
  if (!net) return FOAP4_OK;
  (void)hipStreamSynchronize(net->stream);
  void *ptrs[] = {net->d_w, net->d_mv, net->d_grad, net->d_frag, net->d_cls, net->d_cnt, net->d_part, net->d_loss};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete net;
  return FOAP4_OK;
}

static foap4_status repack(foap4_mlp *net) {
  pack_kernel<<<(kMlpFrags * 64 + 255) / 256, 256, 0, net->stream>>>(net->d_w, (u32x4 *)net->d_frag);
  M_HIP(net, hipGetLastError());
  return FOAP4_OK;
}

foap4_status foap4_mlp_set_params(foap4_mlp *net, const float *w_host, int64_t n) {
  if (!net || !w_host) return mlp_fail(net, FOAP4_E_INVALID, "null argument");
  if (n != kMlpParams) return mlp_fail(net, FOAP4_E_INVALID, "expected FOAP4_MLP_NPARAM parameters");
  M_HIP(net, hipMemcpyAsync(net->d_w, w_host, kMlpParams * 4, hipMemcpyHostToDevice, net->stream));
  M_HIP(net, hipMemsetAsync(net->d_mv, 0, 2 * kMlpParams * 8, net->stream));
  foap4_status st = repack(net);
  if (st != FOAP4_OK) return st;
  M_HIP(net, hipStreamSynchronize(net->stream));
  net->t = 0;
  net->has_weights = true;
  return FOAP4_OK;
}

foap4_status foap4_mlp_get_params(foap4_mlp *net, float *w_host, int64_t n) {
  if (!net || !w_host) return mlp_fail(net, FOAP4_E_INVALID, "null argument");
  if (n != kMlpParams) return mlp_fail(net, FOAP4_E_INVALID, "expected FOAP4_MLP_NPARAM parameters");
  if (!net->has_weights) return mlp_fail(net, FOAP4_E_ORDER, "network has no weights");
  M_HIP(net, hipMemcpyAsync(w_host, net->d_w, kMlpParams * 4, hipMemcpyDeviceToHost, net->stream));
  M_HIP(net, hipStreamSynchronize(net->stream));
  return FOAP4_OK;
}

foap4_status foap4_mlp_set_threshold(foap4_mlp *net, float threshold) {
  if (!net) return mlp_fail(nullptr, FOAP4_E_INVALID, "null network");
  if (!(threshold >= 0.0f && threshold <= 1.0f)) return mlp_fail(net, FOAP4_E_INVALID, "threshold must be in [0, 1]");
  net->threshold = threshold;
  return FOAP4_OK;
}

foap4_status foap4_mlp_forward(foap4_mlp *net, const float *feat_dev, int64_t n, float *logits_dev) {
  if (!net) return mlp_fail(nullptr, FOAP4_E_INVALID, "null network");
  if (n < 0 || (n > 0 && (!feat_dev || !logits_dev))) return mlp_fail(net, FOAP4_E_INVALID, "bad rows or buffers");
  if (!aligned16(feat_dev)) return mlp_fail(net, FOAP4_E_INVALID, "features must be 16-byte aligned");
  if (!net->has_weights) return mlp_fail(net, FOAP4_E_ORDER, "network has no weights");
  if (n == 0) return FOAP4_OK;
  MlpArgs A = base_args(net, feat_dev, n);
  A.logits = logits_dev;
  mlp_kernel<false><<<forward_grid(n), 256, 0, net->stream>>>(A);
  M_HIP(net, hipGetLastError());
  return FOAP4_OK;
}

// label counts (checked on the host) and the per-class sample weights
static foap4_status prepare_loss(foap4_mlp *net, const int8_t *y, int64_t n, const float *class_w) {
  for (int c = 0; c < 3; c++)
    if (!(class_w[c] >= 0.0f) || !std::isfinite(class_w[c]))
      return mlp_fail(net, FOAP4_E_INVALID, "class weights must be finite and >= 0");
  M_HIP(net, hipMemsetAsync(net->d_cnt, 0, 4 * 8, net->stream));
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024));
  count_labels_kernel<<<grid, 256, 0, net->stream>>>(y, n, net->d_cnt);
  M_HIP(net, hipGetLastError());
  unsigned long long cnt[4];
  M_HIP(net, hipMemcpyAsync(cnt, net->d_cnt, sizeof(cnt), hipMemcpyDeviceToHost, net->stream));
  M_HIP(net, hipStreamSynchronize(net->stream));
  if (cnt[3]) return mlp_fail(net, FOAP4_E_INVALID, "labels must be -1, 0 or +1");
  const double tot = (double)class_w[0] * cnt[0] + (double)class_w[1] * cnt[1] + (double)class_w[2] * cnt[2];
  if (!(tot > 0.0)) return mlp_fail(net, FOAP4_E_INVALID, "total sample weight is zero");
  float cls[4] = {(float)(class_w[0] / tot), (float)(class_w[1] / tot), (float)(class_w[2] / tot), 0.0f};
  M_HIP(net, hipMemcpyAsync(net->d_cls, cls, sizeof(cls), hipMemcpyHostToDevice, net->stream));
  return FOAP4_OK;
}

static foap4_status ensure_part(foap4_mlp *net, size_t groups) {
  if (net->cap_part >= groups) return FOAP4_OK;
  if (net->d_part) M_HIP(net, hipFree(net->d_part));
  net->d_part = nullptr;
  net->cap_part = 0;
  M_HIP(net, hipMalloc((void **)&net->d_part, groups * kMlpPartStride * 4));
  net->cap_part = groups;
  return FOAP4_OK;
}

static unsigned train_grid(int64_t n) {
  const int64_t groups = (n + 127) / 128;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(groups, 512));
}

// one gradient evaluation, then the reduction (and an Adam step if update)
static foap4_status grad_step(foap4_mlp *net, const float *x, const int8_t *y, int64_t n, double *d_loss,
                              int update, double lr) {
  const unsigned grid = train_grid(n);
  MlpArgs A = base_args(net, x, n);
  A.y = y;
  A.part = net->d_part;
  mlp_kernel<true><<<grid, 256, 0, net->stream>>>(A);
  M_HIP(net, hipGetLastError());
  double bc1 = 1.0, bc2 = 1.0;
  if (update) {
    const int64_t t = net->t + 1;
    bc1 = 1.0 - std::pow(0.9, (double)t);
    bc2 = 1.0 - std::pow(0.999, (double)t);
  }
  reduce_adam_kernel<<<(kMlpParams + 1 + 255) / 256, 256, 0, net->stream>>>(net->d_part, (int)grid, net->d_w,
                                                                              net->d_mv, net->d_grad, d_loss,
                                                                              update, lr, bc1, bc2);
  M_HIP(net, hipGetLastError());
  if (update) {
    net->t++;
    foap4_status st = repack(net);
    if (st != FOAP4_OK) return st;
  }
  return FOAP4_OK;
}

static foap4_status check_rows(foap4_mlp *net, const float *x, const int8_t *y, int64_t n, const float *class_w) {
  if (!net) return mlp_fail(nullptr, FOAP4_E_INVALID, "null network");
  if (n <= 0 || !x || !y || !class_w) return mlp_fail(net, FOAP4_E_INVALID, "need n > 0 rows, labels and class weights");
  if (!aligned16(x)) return mlp_fail(net, FOAP4_E_INVALID, "features must be 16-byte aligned");
  if (!net->has_weights) return mlp_fail(net, FOAP4_E_ORDER, "network has no weights");
  return ensure_part(net, train_grid(n));
}

foap4_status foap4_mlp_loss_grad(foap4_mlp *net, const float *feat_dev, const int8_t *label_dev, int64_t n,
                                 const float *class_w, double *loss_host, float *grad_host) {
  foap4_status st;
  if ((st = check_rows(net, feat_dev, label_dev, n, class_w)) != FOAP4_OK) return st;
  if (net->cap_loss < 1) {
    M_HIP(net, hipMalloc((void **)&net->d_loss, 8));
    net->cap_loss = 1;
  }
  if ((st = prepare_loss(net, label_dev, n, class_w)) != FOAP4_OK) return st;
  if ((st = grad_step(net, feat_dev, label_dev, n, net->d_loss, 0, 0.0)) != FOAP4_OK) return st;
  if (loss_host) M_HIP(net, hipMemcpyAsync(loss_host, net->d_loss, 8, hipMemcpyDeviceToHost, net->stream));
  if (grad_host) M_HIP(net, hipMemcpyAsync(grad_host, net->d_grad, kMlpParams * 4, hipMemcpyDeviceToHost, net->stream));
  M_HIP(net, hipStreamSynchronize(net->stream));
  return FOAP4_OK;
}

foap4_status foap4_mlp_train(foap4_mlp *net, const float *feat_dev, const int8_t *label_dev, int64_t n,
                             const float *class_w, int32_t iters, float lr, double *loss_host) {
  foap4_status st;
  if ((st = check_rows(net, feat_dev, label_dev, n, class_w)) != FOAP4_OK) return st;
  if (iters < 0 || !(lr > 0.0f)) return mlp_fail(net, FOAP4_E_INVALID, "need iters >= 0 and lr > 0");
  if (iters == 0) return FOAP4_OK;
  if (net->cap_loss < (size_t)iters) {
    if (net->d_loss) M_HIP(net, hipFree(net->d_loss));
    net->d_loss = nullptr;
    net->cap_loss = 0;
    M_HIP(net, hipMalloc((void **)&net->d_loss, (size_t)iters * 8));
    net->cap_loss = (size_t)iters;
  }
  if ((st = prepare_loss(net, label_dev, n, class_w)) != FOAP4_OK) return st;
  for (int32_t it = 0; it < iters; it++)
    if ((st = grad_step(net, feat_dev, label_dev, n, net->d_loss + it, 1, (double)lr)) != FOAP4_OK) return st;
  if (loss_host) M_HIP(net, hipMemcpyAsync(loss_host, net->d_loss, (size_t)iters * 8, hipMemcpyDeviceToHost, net->stream));
  M_HIP(net, hipStreamSynchronize(net->stream));
  return FOAP4_OK;
}

}  // extern "C"
