// Device-side construction of the ghost-cell pattern (Sec. 2.6).
//
// 1. classify: one thread per (block, face) locates the leaf covering the
//    neighbouring region by binary search in the sorted leaf keys and
//    classifies the face as SRL / finer neighbours (F2C into this block) /
//    coarser neighbour (C2F into this block) / physical boundary (the end of
//    a bounded axis).
// 2. count rows [type][face][block] and a row marking blocks with F2C faces.
// 3. exclusive scan of every row (one workgroup per row) -> stable order
//    "face, receiving block, hanging offset" without a sort.
// 4. scatter the records, the per-face flux slots and the flux-fix list.
// Only the row totals travel back to the host (to size the arrays and the
// later launches).
#include <algorithm>

#include "foap4_internal.h"
#include "morton.h"

namespace f4 {

enum { kKindSRL = 0, kKindFine = 1, kKindCoarse = 2, kKindBC = 3 };

struct TopoDev {
  const uint64_t *keys;
  const int32_t *level;
  const int32_t *gc;  // [nb][3]
  int64_t nb;
  int32_t nt[3];
  int32_t ndim;
  int32_t periodic[3];
};

__device__ int64_t locate(const TopoDev &T, int32_t l, const int32_t G[3]) {
  const uint64_t k = leaf_key(T.ndim, T.nt, l, G);
  int64_t lo = 0, hi = T.nb - 1;
  while (lo < hi) {  // last leaf with key <= k
    const int64_t mid = (lo + hi + 1) >> 1;
    if (T.keys[mid] <= k) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ inline void tang_axes(int ndim, int ax, int &t1, int &t2) {
  t1 = (ax == 0) ? 1 : 0;
  t2 = (ndim == 3) ? ((ax == 2) ? 1 : 2) : -1;
}

// kind[b*nf+f], nbr[(b*nf+f)*4 + i], hh[b*nf+f]; err set on unbalanced meshes
__global__ void classify_kernel(TopoDev T, int8_t *kind, int32_t *nbr, int8_t *hh, int32_t *err) {
  const int nf = 2 * T.ndim;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= T.nb * nf) return;
  const int64_t b = id / nf;
  const int f = (int)(id % nf), ax = f / 2, side = f % 2;
  const int32_t l = T.level[b];
  int32_t G[3] = {T.gc[3 * b], T.gc[3 * b + 1], T.gc[3 * b + 2]};
  int32_t H[3] = {G[0], G[1], G[2]};
  const int32_t E = T.nt[ax] << l;
  H[ax] += side ? 1 : -1;
  int32_t *nb4 = nbr + id * 4;
  nb4[0] = nb4[1] = nb4[2] = nb4[3] = -1;
  hh[id] = 0;
  if ((H[ax] < 0 || H[ax] >= E) && !T.periodic[ax]) {
    kind[id] = kKindBC;
    return;
  }
  if (H[ax] < 0) H[ax] += E;
  if (H[ax] >= E) H[ax] -= E;
  int t1, t2;
  tang_axes(T.ndim, ax, t1, t2);
  const int64_t n = locate(T, l, H);
  const int32_t ln = T.level[n];
  if (ln == l) {
    kind[id] = kKindSRL;
    nb4[0] = (int32_t)n;
  } else if (ln < l) {
    if (ln != l - 1) atomicExch(err, 1);
    kind[id] = kKindCoarse;
    nb4[0] = (int32_t)n;
    hh[id] = (int8_t)((G[t1] & 1) + (t2 >= 0 ? 2 * (G[t2] & 1) : 0));
  } else {
    kind[id] = kKindFine;
    const int per = 1 << (T.ndim - 1);
    for (int h = 0; h < per; h++) {
      int32_t C[3] = {2 * H[0], 2 * H[1], 2 * H[2]};
      if (T.ndim == 2) C[2] = 0;
      C[ax] += side ? 0 : 1;
      C[t1] += h & 1;
      if (t2 >= 0) C[t2] += (h >> 1) & 1;
      const int64_t m = locate(T, l + 1, C);
      if (T.level[m] != l + 1) atomicExch(err, 1);
      nb4[h] = (int32_t)m;
    }
  }
}

// rows: r = type * nf + f for the 4 record types, r = 4 * nf for the fix list
__global__ void count_kernel(int64_t nb, int ndim, const int8_t *kind, int32_t *cnt) {
  const int nf = 2 * ndim;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  int anyfine = 0;
  for (int f = 0; f < nf; f++) {
    const int k = kind[b * nf + f];
    cnt[(int64_t)(kSRL * nf + f) * nb + b] = (k == kKindSRL && (f & 1)) ? 1 : 0;
    cnt[(int64_t)(kF2C * nf + f) * nb + b] = (k == kKindFine) ? (1 << (ndim - 1)) : 0;
    cnt[(int64_t)(kC2F * nf + f) * nb + b] = (k == kKindCoarse) ? 1 : 0;
    cnt[(int64_t)(kBC * nf + f) * nb + b] = (k == kKindBC) ? 1 : 0;
    anyfine |= (k == kKindFine);
  }
  cnt[(int64_t)(4 * nf) * nb + b] = anyfine;
}

// In-place exclusive scan of one row per workgroup (1024 threads, 4 values
// per thread per chunk, running carry across chunks); totals to tot[row].
__global__ __launch_bounds__(1024) void scan_rows_kernel(int32_t *cnt, int64_t nb, int32_t *tot) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t carry_s;
  int32_t *row = cnt + (int64_t)blockIdx.x * nb;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) carry_s = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += 4096) {
    int32_t v[4], s = 0;
    for (int q = 0; q < 4; q++) {
      const int64_t i = base + (int64_t)tid * 4 + q;
      v[q] = (i < nb) ? row[i] : 0;
      s += v[q];
    }
    // inclusive scan of s across the wave
    int32_t x = s;
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    if (wid == 0) {
      int32_t w = (lane < 16) ? wsum[lane] : 0;
      for (int o = 1; o < 16; o <<= 1) {
        const int32_t y = __shfl_up(w, o);
        if (lane >= o) w += y;
      }
      if (lane < 16) wsum[lane] = w;
    }
    __syncthreads();
    const int32_t carry = carry_s;
    int32_t ex = carry + (wid > 0 ? wsum[wid - 1] : 0) + x - s;
    for (int q = 0; q < 4; q++) {
      const int64_t i = base + (int64_t)tid * 4 + q;
      if (i < nb) row[i] = ex;
      ex += v[q];
    }
    __syncthreads();
    if (tid == 0) carry_s = carry + wsum[15];
    __syncthreads();
  }
  if (tid == 0) tot[blockIdx.x] = carry_s;
}

struct ScatterArgs {
  int64_t nb;
  int32_t ndim;
  int32_t off[4][7];  // CSR offsets per type
  const int8_t *kind;
  const int32_t *nbr;
  const int8_t *hh;
  const int32_t *cnt;
  int32_t *srl, *f2c, *c2f, *bc, *face_info, *fix_list;
};

__global__ void scatter_kernel(ScatterArgs A) {
  const int nf = 2 * A.ndim;
  const int per = 1 << (A.ndim - 1);
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= A.nb * nf) return;
  const int64_t b = id / nf;
  const int f = (int)(id % nf);
  const int k = A.kind[id];
  const int32_t *nb4 = A.nbr + id * 4;
  int32_t info = -1;
  if (k == kKindSRL) {
    info = -2 - nb4[0];  // same-level neighbour, read directly by the gathering stage kernel
    if (f & 1) {
      const int64_t pos = A.off[kSRL][f] + A.cnt[(int64_t)(kSRL * nf + f) * A.nb + b];
      A.srl[2 * pos] = (int32_t)b;
      A.srl[2 * pos + 1] = nb4[0];
    }
  } else if (k == kKindFine) {
    const int64_t base = A.off[kF2C][f] + A.cnt[(int64_t)(kF2C * nf + f) * A.nb + b];
    const int fo = f ^ 1;
    for (int h = 0; h < per; h++) {
      const int32_t q = nb4[h];
      const int64_t pos = base + h;
      A.f2c[4 * pos] = (int32_t)b;
      A.f2c[4 * pos + 1] = q;
      A.f2c[4 * pos + 2] = h;
      A.f2c[4 * pos + 3] = A.off[kC2F][fo] + A.cnt[(int64_t)(kC2F * nf + fo) * A.nb + q];
    }
    info = (int32_t)(2 * (base / per) + 1);
  } else if (k == kKindCoarse) {
    const int64_t pos = A.off[kC2F][f] + A.cnt[(int64_t)(kC2F * nf + f) * A.nb + b];
    A.c2f[3 * pos] = (int32_t)b;
    A.c2f[3 * pos + 1] = nb4[0];
    A.c2f[3 * pos + 2] = A.hh[id];
    info = (int32_t)(2 * pos);
  } else {
    const int64_t pos = A.off[kBC][f] + A.cnt[(int64_t)(kBC * nf + f) * A.nb + b];
    A.bc[pos] = (int32_t)b;
  }
  A.face_info[id] = info;
  if (f == 0) {
    bool anyfine = false;
    for (int ff = 0; ff < nf; ff++) anyfine |= (A.kind[b * nf + ff] == kKindFine);
    if (anyfine) A.fix_list[A.cnt[(int64_t)(4 * nf) * A.nb + b]] = (int32_t)b;
  }
}

// SRL records whose ghosts a coarse-to-fine prolongation reads: those with a
// side that is the coarse block of some C2F record (its stencils reach into
// the ghosts of that block's other faces).  Meshes that read same-level halos
// straight from the neighbours run only these in round R1.
__global__ void mark_c2f_coarse_kernel(const int32_t *c2f, int64_t n_c2f, int8_t *coarse) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_c2f) coarse[c2f[3 * r + 1]] = 1;
}

__global__ void srl_need_kernel(const int32_t *srl, int64_t n_srl, const int8_t *coarse, int32_t *need) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_srl) need[r] = (coarse[srl[2 * r]] | coarse[srl[2 * r + 1]]) ? 1 : 0;
}

// need[] holds the exclusive prefix sums of the flags (recomputed here)
__global__ void srl_compact_kernel(const int32_t *srl, int64_t n_srl, const int8_t *coarse, const int32_t *pos,
                                   int32_t *sub) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_srl && (coarse[srl[2 * r]] | coarse[srl[2 * r + 1]])) sub[pos[r]] = (int32_t)r;
}

static foap4_status ensure(foap4_mesh *m, void **p, size_t &cap, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (cap >= bytes) return FOAP4_OK;
  if (*p) F4_HIP(m, hipFree(*p));
  *p = nullptr;
  cap = 0;
  F4_HIP(m, hipMalloc(p, bytes));
  cap = bytes;
  return FOAP4_OK;
}

foap4_status build_pattern(foap4_mesh *m) {
  Pattern &P = m->pat;
  const int nf = m->nf, ndim = m->d.ndim, per = 1 << (ndim - 1);
  const int64_t nb = (int64_t)m->topo.leaves.size();
  const int rows = 4 * nf + 1;
  hipStream_t s = m->stream;
  foap4_status st;
  // workspace: kind (int8), nbr (4 int32), hh (int8) per (block, face); count rows
  static_assert(sizeof(int32_t) == 4, "");
  const size_t nbf = (size_t)nb * nf;
  const size_t ws_bytes = nbf * (1 + 16 + 1) + 64;
  if ((st = ensure(m, (void **)&P.cnt, P.cap[0], (size_t)rows * nb * 4 + ws_bytes)) != FOAP4_OK) return st;
  // row totals, the balance error flag, the count of SRL records C2F needs
  if ((st = ensure(m, (void **)&P.tot, P.cap[1], (size_t)(rows + 2) * 4)) != FOAP4_OK) return st;
  int32_t *cnt = P.cnt;
  int32_t *nbr = cnt + (size_t)rows * nb;
  int8_t *kind = (int8_t *)(nbr + nbf * 4);
  int8_t *hh = kind + nbf;
  int32_t *err = P.tot + rows;

  TopoDev T{m->d_keys, m->d_level, m->d_gc, nb, {m->topo.nt[0], m->topo.nt[1], m->topo.nt[2]}, ndim,
            {m->topo.periodic[0], m->topo.periodic[1], m->topo.periodic[2]}};
  F4_HIP(m, hipMemsetAsync(err, 0, 4, s));
  const unsigned g1 = (unsigned)((nbf + 255) / 256);
  classify_kernel<<<g1, 256, 0, s>>>(T, kind, nbr, hh, err);
  F4_HIP(m, hipGetLastError());
  count_kernel<<<(unsigned)((nb + 255) / 256), 256, 0, s>>>(nb, ndim, kind, cnt);
  F4_HIP(m, hipGetLastError());
  scan_rows_kernel<<<rows, 1024, 0, s>>>(cnt, nb, P.tot);
  F4_HIP(m, hipGetLastError());
  int32_t tot[4 * 6 + 1 + 1] = {};
  F4_HIP(m, hipMemcpyAsync(tot, P.tot, (size_t)(rows + 1) * 4, hipMemcpyDeviceToHost, s));
  F4_HIP(m, hipStreamSynchronize(s));
  if (tot[rows]) return fail(m, FOAP4_E_INVALID, "mesh is not 2:1 balanced");
  for (int t = 0; t < kTypes; t++) {
    P.off[t][0] = 0;
    for (int f = 0; f < 6; f++) P.off[t][f + 1] = P.off[t][f] + (f < nf ? tot[t * nf + f] : 0);
    P.n[t] = P.off[t][nf];
  }
  P.n_fix = tot[4 * nf];
  if ((st = ensure(m, (void **)&P.srl, P.cap[2], (size_t)P.n[kSRL] * 8)) != FOAP4_OK) return st;
  if ((st = ensure(m, (void **)&P.f2c, P.cap[3], (size_t)P.n[kF2C] * 16)) != FOAP4_OK) return st;
  if ((st = ensure(m, (void **)&P.c2f, P.cap[4], (size_t)P.n[kC2F] * 12)) != FOAP4_OK) return st;
  if ((st = ensure(m, (void **)&P.bc, P.cap[5], (size_t)P.n[kBC] * 4)) != FOAP4_OK) return st;
  if ((st = ensure(m, (void **)&P.face_info, P.cap[6], nbf * 4)) != FOAP4_OK) return st;
  if ((st = ensure(m, (void **)&P.fix_list, P.cap[7], (size_t)P.n_fix * 4)) != FOAP4_OK) return st;
  // refinement-boundary flux buffers, one N^(d-1) x nvar face per slot
  const int64_t face_vals = (int64_t)m->nvar * (ndim == 3 ? m->d.block_n * m->d.block_n : m->d.block_n);
  if ((st = ensure(m, &P.bflux_f, P.cap_bflux[0], (size_t)P.n[kC2F] * face_vals * m->elem)) != FOAP4_OK) return st;
  if ((st = ensure(m, &P.bflux_c, P.cap_bflux[1], (size_t)(P.n[kF2C] / per) * face_vals * m->elem)) != FOAP4_OK)
    return st;
  ScatterArgs A;
  A.nb = nb;
  A.ndim = ndim;
  for (int t = 0; t < 4; t++)
    for (int f = 0; f < 7; f++) A.off[t][f] = P.off[t][f];
  A.kind = kind;
  A.nbr = nbr;
  A.hh = hh;
  A.cnt = cnt;
  A.srl = P.srl;
  A.f2c = P.f2c;
  A.c2f = P.c2f;
  A.bc = P.bc;
  A.face_info = P.face_info;
  A.fix_list = P.fix_list;
  scatter_kernel<<<g1, 256, 0, s>>>(A);
  F4_HIP(m, hipGetLastError());
  // the SRL records that C2F prolongation depends on (ordered by record);
  // the classification workspace is free again and holds the flags and sums
  P.n_srl_c2f = 0;
  if (P.n[kC2F] > 0 && P.n[kSRL] > 0) {
    int8_t *coarse = (int8_t *)(cnt + 3 * (size_t)nb + 64);
    int32_t *pos = cnt;  // n[kSRL] <= 3 nb entries
    F4_HIP(m, hipMemsetAsync(coarse, 0, (size_t)nb, s));
    mark_c2f_coarse_kernel<<<(unsigned)((P.n[kC2F] + 255) / 256), 256, 0, s>>>(P.c2f, P.n[kC2F], coarse);
    srl_need_kernel<<<(unsigned)((P.n[kSRL] + 255) / 256), 256, 0, s>>>(P.srl, P.n[kSRL], coarse, pos);
    scan_rows_kernel<<<1, 1024, 0, s>>>(pos, P.n[kSRL], P.tot + rows + 1);
    F4_HIP(m, hipGetLastError());
    int32_t n_sub = 0;
    F4_HIP(m, hipMemcpyAsync(&n_sub, P.tot + rows + 1, 4, hipMemcpyDeviceToHost, s));
    F4_HIP(m, hipStreamSynchronize(s));
    if ((st = ensure(m, (void **)&P.srl_c2f, P.cap_srl_c2f, (size_t)n_sub * 4)) != FOAP4_OK) return st;
    srl_compact_kernel<<<(unsigned)((P.n[kSRL] + 255) / 256), 256, 0, s>>>(P.srl, P.n[kSRL], coarse, pos,
                                                                            P.srl_c2f);
    F4_HIP(m, hipGetLastError());
    P.n_srl_c2f = n_sub;
  }
  m->pat_valid = true;
  return FOAP4_OK;
}

}  // namespace f4
