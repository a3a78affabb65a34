// Fused flux/update stage kernel (Sec. 3.2 step list, eq. feuler / eq. heun).
//
// Work decomposition (gfx950, wave64): a workgroup of 256 threads processes
// one work item.  An item is a TX x TY column of cells of one block (16 x 16
// for N = 16 and 32; 32 x 8 for 3-D FP32 N = 32, so that no two items share
// the cache line of a row; for N = 8 four 8 x 8 blocks share the workgroup,
// one per wave) that marches along k over a slab of N / ks planes.  The
// primitive variables of the tile and of its +-2 ring are staged in LDS, in a
// ring of three planes (k, k+1, k+2) that serves both the x/y stencils of
// plane k and the z stencil of each thread's own column; global loads run a
// plane ahead of use.
// Every face flux is computed once.  Halo cells across a same-level face are
// read straight from the neighbouring block ("gather"); across refinement
// faces they come from the ghost cells that the ghost rounds filled.  Fluxes
// on refinement-boundary faces are stored for flux fixing (Sec. 2.7).  In
// stage 2 an epilogue evaluates the CFL limit of every new cell and reduces
// its maximum in FP64.  Items can be visited in an XCD-aware order:
// workgroup w runs on XCD w mod 8, so each XCD is given a contiguous range of
// items (neighbouring blocks in Morton order then share that XCD's L2).
// The kernel is specialised on the set of block sizes present in a launch and
// on the scheme (limiter, flux, gravity source).  This file is compiled once
// per scheme with F4_SCHEME set to that scheme's bit mask; the compile with
// F4_SCHEME = 0 also holds the dispatcher over all schemes.
#include <type_traits>

#include "device_common.h"
#include "foap4_internal.h"
#include "stage_common.h"

namespace f4 {

// Tile of a work item: TX cells along x by TY along y (TB: bytes per value).
// A 3-D FP32 32^3 block is split along y only: an interior row of 32 FP32
// values is one 128-byte line, so two items that split rows along x would
// each fetch every line (their k-marches are not synchronised) and each
// write half lines.  In FP64 a 16-cell half row is a whole line already, and
// the 16 x 16 tile keeps its paired edge faces.
template <int N, int NDIM, int TB = 4>
struct TileCfg {
  static constexpr bool WIDE = N == 32 && NDIM == 3 && TB == 4;
  static constexpr int TX = (N == 8) ? 8 : WIDE ? 32 : 16;
  static constexpr int TY = (N == 8) ? 8 : WIDE ? 8 : 16;
  static constexpr int SUB = 256 / (TX * TY);        // sub-tiles per workgroup
  static constexpr int TPB = (N / TX) * (N / TY);    // tiles per block plane
};
// the host counts items without the value type: both tilings give the same
static_assert(TileCfg<32, 3, 4>::TPB == TileCfg<32, 3, 8>::TPB && TileCfg<32, 3, 4>::SUB == TileCfg<32, 3, 8>::SUB,
              "item counts must not depend on the value type");

// Primitive planes held in LDS: k, k+1, k+2 in a ring of three slots (3D).
template <int NDIM>
constexpr int lds_planes() { return NDIM == 3 ? 3 : 1; }

// LDS elements of one work item: SUB * (planes + x faces + y faces + the
// edge fluxes of the next plane) * NV.
template <int NDIM, int N, int TB>
constexpr int item_cells() {
  using C = TileCfg<N, NDIM, TB>;
  return C::SUB * (lds_planes<NDIM>() * (C::TX + 4) * (C::TY + 4) + 2 * (C::TY + 1) * (C::TX + 4) + 2 * C::TX) *
         (NDIM + 2);
}

// LDS elements per workgroup: the maximum over the block sizes in NM.
template <int NDIM, int NM, int TB>
constexpr int smem_cells() {
  int c = 0;
  if (NM & 1) c = item_cells<NDIM, 8, TB>() > c ? item_cells<NDIM, 8, TB>() : c;
  if (NM & 2) c = item_cells<NDIM, 16, TB>() > c ? item_cells<NDIM, 16, TB>() : c;
  if (NM & 4) c = item_cells<NDIM, 32, TB>() > c ? item_cells<NDIM, 32, TB>() : c;
  return c;
}

// Variable slot of v when the velocity components x and y are exchanged
// (sw): a y face is evaluated as the x face of the exchanged state, so x and
// y faces run the same instructions and the flux components are exchanged
// back on store.
__device__ __forceinline__ int xy_slot(int v, bool sw) { return (sw && (v == 1 || v == 2)) ? 3 - v : v; }

// Flux of one x or y face of the LDS plane Wp ([v][PLANE]) from the four cells
// base + m * step (m = 0..3) along the face normal; F is in natural variable
// order.  sw may differ between lanes.
template <typename T, int NDIM, int PLANE, int SCH>
__device__ __forceinline__ void plane_face(const T *Wp, int base, int step, bool sw, T gamma, T *F) {
  constexpr int NV = NDIM + 2;
  T A0[NV], A1[NV], A2[NV], A3[NV], G[NV];
#pragma unroll
  for (int v = 0; v < NV; v++) {
    const T *p = Wp + xy_slot(v, sw) * PLANE + base;
    A0[v] = p[0];
    A1[v] = p[step];
    A2[v] = p[2 * step];
    A3[v] = p[3 * step];
  }
  face_flux<T, NDIM, 0, SCH>(A0, A1, A2, A3, gamma, G);
#pragma unroll
  for (int v = 0; v < NV; v++) F[v] = (v == 1) ? (sw ? G[2] : G[1]) : (v == 2) ? (sw ? G[1] : G[2]) : G[v];
}

// FEAT (stage 1 only): also reduce, per block, r0 = max |grad rho| / rho and
// r1 = max |grad p| / p over the interior cells of the stage's input state
// (undivided central differences, squares summed x, y, z) into feat_raw[b][2]
// by an atomic maximum; the primitive planes are already in LDS.
template <typename T, int NDIM, int N, int SCH, bool FEAT = false>
__device__ __forceinline__ void stage_item(const MeshDev &M, int stage, int64_t local, T *smem,
                                           double &vmax, bool &bad, double *feat_raw = nullptr,
                                           const SubStep &ss = SubStep{}) {
  using C = TileCfg<N, NDIM, (int)sizeof(T)>;
  constexpr int TX = C::TX, TY = C::TY, SUB = C::SUB, TPB = C::TPB;
  constexpr int NV = NDIM + 2;
  constexpr int LP = TX + 4;            // LDS row stride
  constexpr int PLANE = LP * (TY + 4);
  constexpr int NFX = (TY + 1) * LP;  // x (and y) face flux slots per variable (rows of LP)
  constexpr int TT = TX * TY;
  constexpr int NF = 2 * NDIM;

  const int tid = threadIdx.x;
  // a sub-tile is one or more whole waves (TT >= 64): its block, tile and
  // slab are wave-uniform, and so are the base addresses derived from them
  const int sub = __builtin_amdgcn_readfirstlane(tid / TT), lt = tid % TT;
  // Lanes to cells: LDS has 32 banks of 4 bytes and serves a wave in two
  // halves of 32 lanes.  With the row stride LP = TX + 4 (20, or 12 for
  // 8 x 8 tiles), rows r and r + 4 (r + 2) start 16 (24) banks apart, so a
  // half wave that holds two rows of 16 (four rows of 8) spaced that way
  // reads and writes every plane and face array without bank conflicts;
  // adjacent rows would share 4 banks.  Each wave thus holds the rows
  // w, w + 4, w + 8, w + 12 of a 16 x 16 tile (w the wave), or the even rows
  // then the odd rows of an 8 x 8 tile.  In a 32 x 8 tile a half wave is one
  // whole row (the wave holds rows w and w + 4).
  int ti, tj;
  if constexpr (TX == 16) {
    const int w = lt >> 6, l = lt & 63;
    ti = l & 15;
    tj = w + 4 * (l >> 4);
  } else if constexpr (TX == 32) {
    const int w = lt >> 6, l = lt & 63;
    ti = l & 31;
    tj = w + 4 * (l >> 5);
  } else {
    const int q = lt >> 3;
    ti = lt & 7;
    tj = 2 * (q & 3) + (q >> 2);
  }
  const int ks = (NDIM == 3) ? M.ks : 1;
  const int kslab = (int)(local % ks);
  const int64_t s = (local / ks) * SUB + sub;
  const bool valid = (s / TPB) < M.nb;
  const int64_t b = valid ? s / TPB : M.nb - 1;
  const int tile = (int)(s % TPB);
  const int i0 = (tile % (N / TX)) * TX, j0 = (tile / (N / TX)) * TY;
  const int kd = (NDIM == 3) ? N / ks : 1;
  const int k0 = (NDIM == 3) ? kslab * kd : 0, k1 = k0 + kd;
  const int g = M.g, P = N + 2 * g;
  const int sk = P * N;  // plane stride of a row-part column (cell_off: a plane is P rows of N)
  const int sv = (NDIM == 3) ? P * P * P : P * P;
  const int64_t bel = (int64_t)sv * NV;
  const int cur = M.cur;
  // stage 1 / 2: Heun's stages; stage 3: the generic sub-step ss (states by role)
  const T *__restrict__ ud0 = (const T *)M.s[stage >= 3 ? role_buffer(ss.deriv, cur) : (stage == 1 ? cur : 1 - cur)];
  T *uo = (T *)M.s[stage >= 3 ? role_buffer(ss.out, cur) : (stage == 1 ? 1 - cur : cur)] + b * bel;
  const T *up = (const T *)M.s[stage >= 3 ? role_buffer(ss.prev, cur) : cur] + b * bel;
  [[maybe_unused]] const T *up2 = nullptr, *up3 = nullptr;
  if (stage == 4) {
    up2 = (const T *)M.s[role_buffer(ss.prev2, cur)] + b * bel;
    up3 = (const T *)M.s[role_buffer(ss.prev3, cur)] + b * bel;
  }
  const T gamma = (T)M.gamma;
  const double dx = ldexp(M.dx0, -gload(M.level + b));
  const T idx = (T)(1.0 / dx);
  const double dt = gload(M.scal + kDt);
  const T dts = (T)(stage >= 3 ? ss.c * dt : (stage == 1 ? dt : 0.5 * dt));
  [[maybe_unused]] const T wd = (T)ss.wd, wp = (T)ss.wp, wp2 = (T)ss.wp2, wp3 = (T)ss.wp3;
  [[maybe_unused]] T grav[NDIM];
  if constexpr ((SCH & kSchGravity) != 0) {
#pragma unroll
    for (int d = 0; d < NDIM; d++) grav[d] = (T)M.grav[d];
  }

  // per face: refinement-face flux slot (>= 0), same-level neighbour (-2 - n) or -1
  int finfo[NF];
#pragma unroll
  for (int f = 0; f < NF; f++) finfo[f] = gload(M.face_info + b * NF + f);
  auto nbr_of = [&](int f) -> int64_t { return (M.gather && finfo[f] <= -2) ? (int64_t)(-2 - finfo[f]) : -1; };

  constexpr int NS = lds_planes<NDIM>();
  T *Wring = smem + sub * (NS * PLANE + 2 * NFX + 2 * TX) * NV;  // [slot][v][PLANE]
  T *FX = Wring + NS * PLANE * NV;                                // [v][TY (+ 1)][LP]: TX + 1 x faces a row
  T *FY = FX + NFX * NV;                                          // [v][TY + 1][LP]: TX y faces a row
  T *XE = FY + NFX * NV;  // [v][2 TX]: edge fluxes (+x column, +y row) of plane k + 1 (square tiles)
  auto slot = [&](int kk) -> T * { return NS == 1 ? Wring : Wring + (kk % NS) * (PLANE * NV); };

  auto off = [&](int ii, int jj, int kk) -> int { return cell_off<NDIM>(ii, jj, kk, N, g); };
  auto load = [&](const T *p, T *U) {
#pragma unroll
    for (int v = 0; v < NV; v++) U[v] = gload(p + v * sv);
  };
  auto store_bflux = [&](int f, int t1, int t2, const T *F) {
    const int info = finfo[f];
    if (info < 0 || !valid) return;
    T *buf = (T *)((info & 1) ? M.bflux_c : M.bflux_f);
    const int64_t slot = info >> 1;
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const int64_t o = (NDIM == 3) ? ((slot * NV + v) * N + t2) * N + t1 : (slot * NV + v) * N + t1;
      gstore(buf + o, F[v]);
    }
  };

  // ring cell of this thread (x ghosts: 4 per row; y ghosts: 4 rows)
  const bool ring = lt < 4 * (TX + TY);
  int ri = 0, rj = 0;
  if (lt < 4 * TY) {
    const int c = lt & 3;
    rj = lt >> 2;
    ri = (c < 2) ? c - 2 : TX + c - 2;
  } else if (ring) {
    const int r = lt - 4 * TY, c = r / TX;
    ri = r % TX;
    rj = (c < 2) ? c - 2 : TY + c - 2;
  }
  const int ring_lds = (rj + 2) * LP + (ri + 2);
  const int own_lds = (tj + 2) * LP + (ti + 2);
  const int I = i0 + ti, J = j0 + tj;

  // Source pointers, fixed for the whole item: the ring cell's column (its
  // block does not change with k) and the own column inside the block and
  // across the -z / +z faces.  Plane k of a column is at + k * sk, of the
  // ring column at + k * ring_sk (an own x ghost column steps by P 2g).
  const T *ring_p;
  int ring_sk;
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
    ring_sk = ((unsigned)RI < (unsigned)N) ? sk : P * 2 * g;
  }
  // The own column: plane kk of variable v of block B at the wave-uniform
  // base B + v sv + kk sk plus the lane's byte offset own_ob (interior cells:
  // the offset of (I, J, kk) is that of (I, J, 0) plus kk sk).  colb(kk) is
  // the base of plane kk, in the neighbour block across -z / +z (gather).
  const T *own_b = ud0 + b * bel;
  const uint32_t own_ob = (uint32_t)off(I, J, 0) * (uint32_t)sizeof(T);
  const T *zlo_b = nullptr, *zhi_b = nullptr;
  if constexpr (NDIM == 3) {
    const int64_t nlo = nbr_of(4 % NF), nhi = nbr_of(5 % NF);
    if (nlo >= 0) zlo_b = ud0 + nlo * bel;
    if (nhi >= 0) zhi_b = ud0 + nhi * bel;
  }
  auto colb = [&](int kk) -> const T * {
    if (kk < 0 && zlo_b) return zlo_b + (kk + N) * sk;
    if (kk >= N && zhi_b) return zhi_b + (kk - N) * sk;
    return own_b + kk * sk;
  };
  auto loadc = [&](const T *base, T *U) {
    const auto r = buf_rsrc(base);
#pragma unroll
    for (int v = 0; v < NV; v++) U[v] = buf_load<T>(r, own_ob, (uint32_t)(v * sv * (int)sizeof(T)));
  };

  // cells next to F2C faces are finished (and their dt taken) by the flux fix
  auto is_f2c = [&](int f) { return f < NF && finfo[f] >= 0 && (finfo[f] & 1); };
  const bool f2c_adj = (is_f2c(0) && I == 0) || (is_f2c(1) && I == N - 1) || (is_f2c(2) && J == 0) ||
                       (is_f2c(3) && J == N - 1);
  const bool f2c_zlo = NDIM == 3 && is_f2c(4), f2c_zhi = NDIM == 3 && is_f2c(5);

  // Primitive planes live in a ring of LDS slots (plane kk in slot kk % 3):
  // at iteration k the slots hold planes k, k+1, k+2; the own column's z
  // stencil reads them there, so only the conserved state of the own column
  // (cells k .. k+2, needed by the update, and the prefetched k+3) is kept in
  // registers.  Those four states rotate through the register sets X (plane
  // kk in set (kk - k0) % 4), the fluxes of faces k -+ 1/2 through Fz2 and
  // the prefetched U^n through P1: the plane loop is unrolled by four, so
  // every set is named by a constant and no state is copied between planes.
  T X[4][NV], Fz2[2][NV], R[NV], Sk[NV];  // ..., ring prefetch, z slope of cell k
  auto put = [&](T *S, int at, const T *U) {
    T W[NV];
    to_prim<T, NDIM>(U, gamma, W);
#pragma unroll
    for (int v = 0; v < NV; v++) S[v * PLANE + at] = W[v];
  };

  [[maybe_unused]] T fr = T(0), fp = T(0);  // this thread's feature maxima
  [[maybe_unused]] T zr = T(1), zp = T(1);  // rho, p of own cell k0 - 1
  // features of plane q of the own column; planes q-1 / q+1 from lo / hi
  [[maybe_unused]] auto feat_cell = [&](const T *Sq, T rlo, T plo, T rhi, T phi) {
    const T *c = Sq + own_lds, *cp = Sq + (NV - 1) * PLANE + own_lds;
    const T hf = T(0.5);
    const T drx = hf * (c[1] - c[-1]), dpx = hf * (cp[1] - cp[-1]);
    const T dry = hf * (c[LP] - c[-LP]), dpy = hf * (cp[LP] - cp[-LP]);
    T sr = drx * drx, sp = dpx * dpx;
    sr = sr + dry * dry;
    sp = sp + dpy * dpy;
    if constexpr (NDIM == 3) {
      const T drz = hf * (rhi - rlo), dpz = hf * (phi - plo);
      sr = sr + drz * drz;
      sp = sp + dpz * dpz;
    }
    const T gr = fsqrt(sr) * frcp(c[0]), gp = fsqrt(sp) * frcp(cp[0]);
    fr = gr > fr ? gr : fr;
    fp = gp > fp ? gp : fp;
  };

  if constexpr (NDIM == 3) {
    T tmp[NV], Wm2[NV], Wm1[NV], W0[NV], W1[NV];
    loadc(colb(k0 - 2), tmp);
    to_prim<T, NDIM>(tmp, gamma, Wm2);
    loadc(colb(k0 - 1), tmp);
    to_prim<T, NDIM>(tmp, gamma, Wm1);
    loadc(colb(k0), X[0]);
    to_prim<T, NDIM>(X[0], gamma, W0);
    loadc(colb(k0 + 1), X[1]);
    to_prim<T, NDIM>(X[1], gamma, W1);
#pragma unroll
    for (int v = 0; v < NV; v++) {
      slot(k0)[v * PLANE + own_lds] = W0[v];
      slot(k0 + 1)[v * PLANE + own_lds] = W1[v];
    }
    if (ring) {
      load(ring_p + k0 * ring_sk, tmp);
      put(slot(k0), ring_lds, tmp);
      load(ring_p + (k0 + 1) * ring_sk, tmp);
      put(slot(k0 + 1), ring_lds, tmp);
    }
    // face k0 - 1/2; the slope of cell k0 is carried into the plane loop
    T L[NV], Rt[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const T s1 = limit<SCH & kSchVanLeer>(Wm1[v] - Wm2[v], W0[v] - Wm1[v]);
      Sk[v] = limit<SCH & kSchVanLeer>(W0[v] - Wm1[v], W1[v] - W0[v]);
      L[v] = Wm1[v] + T(0.5) * s1;
      Rt[v] = W0[v] - T(0.5) * Sk[v];
    }
    riemann<T, NDIM, 2, (SCH & kSchHLL) != 0>(L, Rt, gamma, Fz2[0]);
    if (k0 == 0) store_bflux(4, I, J, Fz2[0]);
    if constexpr (FEAT) {
      zr = Wm1[0];
      zp = Wm1[NV - 1];
    }
    loadc(colb(k0 + 2), X[2]);
    if (ring) load(ring_p + (k0 + 2) * ring_sk, R);
  } else {
    T tmp[NV];
    loadc(own_b, X[0]);
    put(slot(0), own_lds, X[0]);
    if (ring) {
      load(ring_p, tmp);
      put(slot(0), ring_lds, tmp);
    }
  }

  // U^n (stage >= 2) and the two earlier states of RK4's last sub-step of
  // the own cell, loaded one plane ahead (plane kk in set (kk - k0) % 2)
  [[maybe_unused]] T P1[2][NV], P2[2][NV], P3[2][NV];
  if (stage >= 2) loadc(up + k0 * sk, P1[0]);
  if (stage == 4) {
    loadc(up2 + k0 * sk, P2[0]);
    loadc(up3 + k0 * sk, P3[0]);
  }

  T vloc = T(0);  // running maximum of the CFL limits of the item's cells

  // plane k, PH = (k - k0) % 4
  auto plane = [&](auto phase, const int k) __attribute__((always_inline)) {
    constexpr int PH = decltype(phase)::value;
    if constexpr (NDIM == 3) {
      // plane k + 2 into the slot plane k - 1 used; prefetch plane k + 3
      put(slot(k + 2), own_lds, X[(PH + 2) & 3]);
      if (ring && k + 2 < k1) put(slot(k + 2), ring_lds, R);
      if (k + 3 <= k1 + 1) loadc(colb(k + 3), X[(PH + 3) & 3]);
      if (ring && k + 3 < k1) load(ring_p + (k + 3) * ring_sk, R);
    }
    const T *U0 = X[PH & 3];
    [[maybe_unused]] const T *Up = P1[PH & 1], *Up2 = P2[PH & 1], *Up3 = P3[PH & 1];
    if (stage == 4 && k + 1 < k1) {
      loadc(up2 + (k + 1) * sk, P2[(PH + 1) & 1]);
      loadc(up3 + (k + 1) * sk, P3[(PH + 1) & 1]);
    }
    if (stage >= 2 && k + 1 < k1) loadc(up + (k + 1) * sk, P1[(PH + 1) & 1]);
    const T *Wp = slot(k);
    __syncthreads();

    if constexpr (FEAT) {
      if (valid) {
        if constexpr (NDIM == 3) {
          const T *S1 = slot(k + 1), *S2 = slot(k + 2);
          constexpr int PV = (NV - 1) * PLANE;
          if (k == k0) feat_cell(Wp, zr, zp, S1[own_lds], S1[PV + own_lds]);
          if (k + 1 < k1) feat_cell(S1, Wp[own_lds], Wp[PV + own_lds], S2[own_lds], S2[PV + own_lds]);
        } else {
          feat_cell(Wp, T(0), T(0), T(0), T(0));
        }
      }
    }

    [[maybe_unused]] const T *Fz = Fz2[PH & 1];
    [[maybe_unused]] T *Fz1 = Fz2[(PH + 1) & 1];
    if constexpr (NDIM == 3) {
      // face k + 1/2 with the carried slope of cell k
      const T *A = Wp + own_lds, *B = slot(k + 1) + own_lds, *Cc = slot(k + 2) + own_lds;
      T L[NV], Rt[NV];
#pragma unroll
      for (int v = 0; v < NV; v++) {
        const T w0 = A[v * PLANE], w1 = B[v * PLANE], w2 = Cc[v * PLANE];
        const T sn = limit<SCH & kSchVanLeer>(w1 - w0, w2 - w1);
        L[v] = w0 + T(0.5) * Sk[v];
        Rt[v] = w1 - T(0.5) * sn;
        Sk[v] = sn;
      }
      riemann<T, NDIM, 2, (SCH & kSchHLL) != 0>(L, Rt, gamma, Fz1);
      if (k == N - 1) store_bflux(5, I, J, Fz1);
    }

    // x and y faces of the plane: every thread computes the -x and the -y
    // face of its cell (FX[v][fj][fi], FY[v][fj][fi], rows of LP, both NFX per
    // variable).
    // The TY extra +x faces of the last column and the TX extra +y faces
    // of the last row run together in lanes of one wave (the y ones on
    // exchanged velocities); with 4 waves per tile the wave rotates with the
    // plane (pair) so that every SIMD gets its share.
    {
      T F[NV];
      plane_face<T, NDIM, PLANE, SCH>(Wp, (tj + 2) * LP + ti, 1, false, gamma, F);  // cells ti-2 .. ti+1
#pragma unroll
      for (int v = 0; v < NV; v++) FX[v * NFX + tj * LP + ti] = F[v];
      if (ti == 0 && i0 == 0) store_bflux(0, j0 + tj, k, F);
      plane_face<T, NDIM, PLANE, SCH>(Wp, tj * LP + ti + 2, LP, true, gamma, F);  // cells tj-2 .. tj+1
#pragma unroll
      for (int v = 0; v < NV; v++) FY[v * NFX + tj * LP + ti] = F[v];
      if (tj == 0 && j0 == 0) store_bflux(2, i0 + ti, k, F);
    }
    if constexpr (NDIM == 3 && TT == 256 && TX == TY) {
      constexpr int TILE = TX;
      // 3D tiles of 16 x 16: the edge faces of planes k and k + 1 together,
      // every other plane, in the 64 lanes of one wave (one plane's 2 TILE
      // edge faces would leave half of it idle); the fluxes of plane k + 1
      // wait in XE and are put in place on the next plane (the planes of a
      // slab come in pairs: N / kslabs is even).  For 8^3 blocks each wave
      // keeps its own plane's 16 edge faces: pairing them there costs more
      // registers (and occupancy) than it saves.  A 32 x 8 tile has 40 edge
      // faces a plane, too many to pair in 64 lanes: one wave takes them on
      // every plane.
      const int pair = (k - k0) >> 1;
      const int e = lt - 64 * ((pair + (int)local) & 3);
      if (((k - k0) & 1) == 0) {
        if (e >= 0 && e < 4 * TILE) {
          const int pk = e >= 2 * TILE ? 1 : 0;  // plane k + pk
          const int ee = e - 2 * TILE * pk;
          const bool sw = ee >= TILE;
          const int m = sw ? ee - TILE : ee;
          if (pk == 0 || k + 1 < k1) {
            T F[NV];
            plane_face<T, NDIM, PLANE, SCH>(pk ? slot(k + 1) : Wp, sw ? TILE * LP + m + 2 : (m + 2) * LP + TILE,
                                       sw ? LP : 1, sw, gamma, F);
            T *out = pk ? XE + ee : (sw ? FY + TILE * LP + m : FX + m * LP + TILE);
            const int ost = pk ? 2 * TILE : NFX;
#pragma unroll
            for (int v = 0; v < NV; v++) out[v * ost] = F[v];
            if (!sw && i0 + TILE == N) store_bflux(1, j0 + m, k + pk, F);
            if (sw && j0 + TILE == N) store_bflux(3, i0 + m, k + pk, F);
          }
        }
      } else if (e >= 0 && e < 2 * TILE) {
        const bool sw = e >= TILE;
        const int m = sw ? e - TILE : e;
        T *out = sw ? FY + TILE * LP + m : FX + m * LP + TILE;
#pragma unroll
        for (int v = 0; v < NV; v++) out[v * NFX] = XE[v * 2 * TILE + e];
      }
    } else {
      const int e = (TT == 256) ? lt - 64 * ((k + (int)local) & 3) : lt;
      if (e >= 0 && e < TX + TY) {
        const bool sw = e >= TY;
        const int m = sw ? e - TY : e;
        T F[NV];
        plane_face<T, NDIM, PLANE, SCH>(Wp, sw ? TY * LP + m + 2 : (m + 2) * LP + TX, sw ? LP : 1, sw, gamma, F);
        T *out = sw ? FY + TY * LP + m : FX + m * LP + TX;
#pragma unroll
        for (int v = 0; v < NV; v++) out[v * NFX] = F[v];
        if (!sw && i0 + TX == N) store_bflux(1, j0 + m, k, F);
        if (sw && j0 + TY == N) store_bflux(3, i0 + m, k, F);
      }
    }
    __syncthreads();

    // conservative update of the own cell (eq. feuler with Heun weights):
    // U_out = base - (dt_s / dx) sum_d (F_d(+) - F_d(-)) [+ dt_s S(U0)]
    T Uout[NV];
    const T cdt = dts * idx;
    [[maybe_unused]] T src[NV];
    if constexpr ((SCH & kSchGravity) != 0) {
      // gravity source of the cell's stage input (Sec. 4.2): (0, rho g, g.m)
      T gm = T(0);
      src[0] = T(0);
#pragma unroll
      for (int d = 0; d < NDIM; d++) {
        src[1 + d] = U0[0] * grav[d];
        gm += grav[d] * U0[1 + d];
      }
      src[NV - 1] = gm;
    }
#pragma unroll
    for (int v = 0; v < NV; v++) {
      const T dfx = FX[v * NFX + tj * LP + ti + 1] - FX[v * NFX + tj * LP + ti];
      const T dfy = FY[v * NFX + (tj + 1) * LP + ti] - FY[v * NFX + tj * LP + ti];
      T div = dfx + dfy;
      if constexpr (NDIM == 3) div += Fz1[v] - Fz[v];
      T base;
      if (stage == 1) base = U0[v];
      else if (stage == 2) base = T(0.5) * (Up[v] + U0[v]);
      else if (stage == 3) base = wp * Up[v] + wd * U0[v];
      else base = ((wp * Up[v] + wp2 * Up2[v]) + wp3 * Up3[v]) + wd * U0[v];
      if constexpr ((SCH & kSchGravity) != 0) Uout[v] = (base + dts * src[v]) - cdt * div;
      else Uout[v] = base - cdt * div;
    }
    // a tile's rows are contiguous runs of the block's row part; the tiles
    // of a block together write each interior plane as one contiguous range
    if (valid) {
      const auto r = buf_rsrc(uo + k * sk);
#pragma unroll
      for (int v = 0; v < NV; v++) buf_store<T>(Uout[v], r, own_ob, (uint32_t)(v * sv * (int)sizeof(T)));
    }
    if ((stage == 2 || (stage >= 3 && ss.epi)) && valid) {
      const bool skip = f2c_adj || (f2c_zlo && k == 0) || (f2c_zhi && k == N - 1);
      if (!skip) {
        if constexpr (sizeof(T) == 8) {
          vloc = fmax(vloc, cell_inv_dt<NDIM>((const double *)Uout, M.gamma, dx, bad));
        } else {
          vloc = fmaxf(vloc, cell_inv_dt<NDIM>((const float *)Uout, (float)gamma, (float)idx, bad));
        }
      }
    }
  };
  for (int k = k0; k < k1; k += 4) {
    plane(std::integral_constant<int, 0>{}, k);
    if (k + 1 >= k1) break;
    plane(std::integral_constant<int, 1>{}, k + 1);
    if (k + 2 >= k1) break;
    plane(std::integral_constant<int, 2>{}, k + 2);
    if (k + 3 >= k1) break;
    plane(std::integral_constant<int, 3>{}, k + 3);
  }
  vmax = fmax(vmax, (double)vloc);
  if constexpr (FEAT) {
    double dr = (double)fr, dp = (double)fp;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      dr = fmax(dr, __shfl_xor(dr, o));
      dp = fmax(dp, __shfl_xor(dp, o));
    }
    if ((threadIdx.x & 63) == 0 && valid) {
      atomic_max_pos(feat_raw + 2 * b, dr);
      atomic_max_pos(feat_raw + 2 * b + 1, dp);
    }
  }
}

// Item visited by iteration `it` of workgroup w.  order 0: plain striding;
// 1: XCD x = w mod 8 walks the x-th eighth of the item range; 2: workgroup w
// takes the w-th contiguous chunk, so a block and its Morton neighbours (the
// x neighbour first) run back to back on one CU and the neighbour rows that a
// halo read pulls into the cache are used again by the next item.
__device__ __forceinline__ int64_t item_of(int64_t w, int64_t it, int64_t grid, int64_t total, int xcd) {
  if (!xcd) return w + it * grid;
  if (xcd == 2) return w * ((total + grid - 1) / grid) + it;
  const int64_t per_xcd = (total + 7) / 8;
  const int64_t lanes = (grid + 7 - (w & 7)) / 8;  // workgroups on this XCD
  const int64_t j = (w >> 3) + it * lanes;         // position inside the XCD's range
  return j < per_xcd ? (w & 7) * per_xcd + j : total;
}

// Target waves per SIMD: single-size FP32 kernels 4 (4 resident workgroups
// of 4 waves per CU: stage 2 then spills a few values per lane at 128
// registers, which ran faster than 3 waves without spills); the mixed-size
// FP32 kernel 3 (its LDS allows 3 workgroups per CU; at 168 registers it
// spills a little and ran ~14 % faster than at 2 waves); FP64 kernels keep
// what their registers allow.
template <typename T, int NM, int STG = 2>
constexpr int stage_waves() { return sizeof(T) == 4 ? (NM != 7 ? 4 : 3) : 1; }

// NM: bit mask of the block sizes present (1: N = 8, 2: N = 16, 4: N = 32)
// STG: the Heun stage (compiled separately: stage 1 needs no U^n stream and
// no dt epilogue, so it runs with fewer registers), or 3: the generic
// sub-step ss of the other Runge-Kutta schemes (weights at run time), 4: the
// same with three earlier states (classical RK4's last sub-step)
template <typename T, int NDIM, int NM, int STG, int SCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(stage_waves<T, NM, STG>())))
void stage_kernel(const MeshDev *__restrict__ meshes, int n_meshes, int64_t total, int xcd, SubStep ss) {
  constexpr int stage = STG;
  __shared__ T smem[smem_cells<NDIM, NM, (int)sizeof(T)>()];
  double vmax = 0.0;
  bool bad = false;
  int mprev = -1;
  const int64_t grid = gridDim.x;
  const int64_t lanes = grid / 8 > 0 ? grid / 8 : 1;
  const int64_t iters = xcd == 1 ? ((total + 7) / 8 + lanes - 1) / lanes : (total + grid - 1) / grid;
  for (int64_t it = 0; it < iters; it++) {
    const int64_t item = item_of(blockIdx.x, it, grid, total, xcd);
    if (item >= total) break;
    int lo = 0, hi = n_meshes - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (meshes[mid].item_begin <= item) lo = mid; else hi = mid - 1;
    }
    if (stage >= 2 && mprev >= 0 && lo != mprev) flush_dt(meshes[mprev], vmax, bad);
    mprev = lo;
    const MeshDev &M = meshes[lo];
    const int64_t local = item - M.item_begin;
    if constexpr (NM == 1) {
      stage_item<T, NDIM, 8, SCH>(M, stage, local, smem, vmax, bad, nullptr, ss);
    } else if constexpr (NM == 2) {
      stage_item<T, NDIM, 16, SCH>(M, stage, local, smem, vmax, bad, nullptr, ss);
    } else if constexpr (NM == 4) {
      stage_item<T, NDIM, 32, SCH>(M, stage, local, smem, vmax, bad, nullptr, ss);
    } else {
      switch (M.N) {
        case 8: stage_item<T, NDIM, 8, SCH>(M, stage, local, smem, vmax, bad, nullptr, ss); break;
        case 16: stage_item<T, NDIM, 16, SCH>(M, stage, local, smem, vmax, bad, nullptr, ss); break;
        default: stage_item<T, NDIM, 32, SCH>(M, stage, local, smem, vmax, bad, nullptr, ss); break;
      }
    }
    __syncthreads();
  }
  if (stage >= 2 && mprev >= 0) flush_dt(meshes[mprev], vmax, bad);
}

template <typename T, int NDIM, int SCH>
static void launch_t(unsigned nblk, int nmask, const MeshDev *d, int n, int64_t total, int stage, int xcd,
                     hipStream_t s, const SubStep &ss) {
#define F4_STAGE_LAUNCH(NM)                                                                     \
  if (stage == 1) stage_kernel<T, NDIM, NM, 1, SCH><<<nblk, 256, 0, s>>>(d, n, total, xcd, ss); \
  else if (stage == 2) stage_kernel<T, NDIM, NM, 2, SCH><<<nblk, 256, 0, s>>>(d, n, total, xcd, ss); \
  else if (stage == 3) stage_kernel<T, NDIM, NM, 3, SCH><<<nblk, 256, 0, s>>>(d, n, total, xcd, ss); \
  else stage_kernel<T, NDIM, NM, 4, SCH><<<nblk, 256, 0, s>>>(d, n, total, xcd, ss);
  switch (nmask) {
    case 1: F4_STAGE_LAUNCH(1) break;
    case 2: F4_STAGE_LAUNCH(2) break;
    case 4: F4_STAGE_LAUNCH(4) break;
    default: F4_STAGE_LAUNCH(7) break;
  }
#undef F4_STAGE_LAUNCH
}

// Stage 1 of one mesh (one workgroup per work item) that also reduces the
// per-block features of its input state into feat_raw (zeroed by the caller).
template <typename T, int NDIM, int NM, int SCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(stage_waves<T, NM, 1>())))
void stage1_feat_kernel(const MeshDev *__restrict__ Mp, int64_t total, double *feat_raw) {
  __shared__ T smem[smem_cells<NDIM, NM, (int)sizeof(T)>()];
  constexpr int N = (NM == 1) ? 8 : (NM == 2) ? 16 : 32;
  double vmax = 0.0;
  bool bad = false;
  if ((int64_t)blockIdx.x >= total) return;
  stage_item<T, NDIM, N, SCH, true>(*Mp, 1, blockIdx.x, smem, vmax, bad, feat_raw);
}

template <typename T, int NDIM, int SCH>
static void launch_feat_t(unsigned nblk, int nmask, const MeshDev *d, int64_t total, double *fr, hipStream_t s) {
  switch (nmask) {
    case 1: stage1_feat_kernel<T, NDIM, 1, SCH><<<nblk, 256, 0, s>>>(d, total, fr); break;
    case 2: stage1_feat_kernel<T, NDIM, 2, SCH><<<nblk, 256, 0, s>>>(d, total, fr); break;
    default: stage1_feat_kernel<T, NDIM, 4, SCH><<<nblk, 256, 0, s>>>(d, total, fr); break;
  }
}

// Launchers of one scheme; each compile of this file instantiates those of
// its own F4_SCHEME.
template <int SCH>
hipError_t launch_stage_sch(const MeshDev *d_meshes, int n_meshes, int64_t total_items, int stage, int ndim,
                            bool f64, int grid, hipStream_t s, int xcd, int nmask, const SubStep &ss) {
  int64_t nblk = (grid > 0 && grid < total_items) ? grid : total_items;
  if (xcd == 1) nblk = (nblk + 7) / 8 * 8;  // every XCD gets the same number of workgroups
  if (f64) {
    if (ndim == 3) launch_t<double, 3, SCH>((unsigned)nblk, nmask, d_meshes, n_meshes, total_items, stage, xcd, s, ss);
    else launch_t<double, 2, SCH>((unsigned)nblk, nmask, d_meshes, n_meshes, total_items, stage, xcd, s, ss);
  } else {
    if (ndim == 3) launch_t<float, 3, SCH>((unsigned)nblk, nmask, d_meshes, n_meshes, total_items, stage, xcd, s, ss);
    else launch_t<float, 2, SCH>((unsigned)nblk, nmask, d_meshes, n_meshes, total_items, stage, xcd, s, ss);
  }
  return hipGetLastError();
}

template <int SCH>
hipError_t launch_feat_sch(const MeshDev *d_mesh, int64_t total_items, int ndim, bool f64, int nmask,
                           double *feat_raw, hipStream_t s) {
  const unsigned nblk = (unsigned)total_items;
  if (f64) {
    if (ndim == 3) launch_feat_t<double, 3, SCH>(nblk, nmask, d_mesh, total_items, feat_raw, s);
    else launch_feat_t<double, 2, SCH>(nblk, nmask, d_mesh, total_items, feat_raw, s);
  } else {
    if (ndim == 3) launch_feat_t<float, 3, SCH>(nblk, nmask, d_mesh, total_items, feat_raw, s);
    else launch_feat_t<float, 2, SCH>(nblk, nmask, d_mesh, total_items, feat_raw, s);
  }
  return hipGetLastError();
}

#ifndef F4_SCHEME
#define F4_SCHEME 0
#endif
static_assert(F4_SCHEME >= 0 && F4_SCHEME < kNSchemes, "F4_SCHEME is a scheme bit mask");

template hipError_t launch_stage_sch<F4_SCHEME>(const MeshDev *, int, int64_t, int, int, bool, int, hipStream_t,
                                                int, int, const SubStep &);
template hipError_t launch_feat_sch<F4_SCHEME>(const MeshDev *, int64_t, int, bool, int, double *, hipStream_t);

#if F4_SCHEME == 0
template <int N, int NDIM>
static int64_t items_of(int64_t nb, int ks) {
  using C = TileCfg<N, NDIM>;
  const int64_t tiles = nb * C::TPB;
  return ((tiles + C::SUB - 1) / C::SUB) * (NDIM == 3 ? ks : 1);
}

int64_t stage_items_for(int ndim, int N, int64_t nb, int ks) {
  if (ndim == 3) return N == 8 ? items_of<8, 3>(nb, ks) : N == 16 ? items_of<16, 3>(nb, ks) : items_of<32, 3>(nb, ks);
  return N == 8 ? items_of<8, 2>(nb, ks) : N == 16 ? items_of<16, 2>(nb, ks) : items_of<32, 2>(nb, ks);
}

// the other schemes' launchers live in the other compiles of this file
#define F4_EXTERN_SCHEME(S)                                                                                    \
  extern template hipError_t launch_stage_sch<S>(const MeshDev *, int, int64_t, int, int, bool, int,          \
                                                 hipStream_t, int, int, const SubStep &);                      \
  extern template hipError_t launch_feat_sch<S>(const MeshDev *, int64_t, int, bool, int, double *, hipStream_t);
F4_EXTERN_SCHEME(1)
F4_EXTERN_SCHEME(2)
F4_EXTERN_SCHEME(3)
F4_EXTERN_SCHEME(4)
F4_EXTERN_SCHEME(5)
F4_EXTERN_SCHEME(6)
F4_EXTERN_SCHEME(7)
#undef F4_EXTERN_SCHEME

hipError_t launch_stage(const MeshDev *d_meshes, int n_meshes, int64_t total_items, int stage,
                        int ndim, bool f64, int grid, hipStream_t s, int xcd, int nmask, int scheme,
                        const SubStep &ss) {
  if (total_items <= 0) return hipSuccess;
  switch (scheme) {
#define F4_CASE(S) \
    case S: return launch_stage_sch<S>(d_meshes, n_meshes, total_items, stage, ndim, f64, grid, s, xcd, nmask, ss);
    F4_CASE(0) F4_CASE(1) F4_CASE(2) F4_CASE(3) F4_CASE(4) F4_CASE(5) F4_CASE(6) F4_CASE(7)
#undef F4_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stage1_features(const MeshDev *d_mesh, int64_t total_items, int ndim, bool f64, int nmask,
                                  double *feat_raw, hipStream_t s, int scheme) {
  if (total_items <= 0) return hipSuccess;
  if (nmask != 1 && nmask != 2 && nmask != 4) return hipErrorInvalidValue;
  switch (scheme) {
#define F4_CASE(S) case S: return launch_feat_sch<S>(d_mesh, total_items, ndim, f64, nmask, feat_raw, s);
    F4_CASE(0) F4_CASE(1) F4_CASE(2) F4_CASE(3) F4_CASE(4) F4_CASE(5) F4_CASE(6) F4_CASE(7)
#undef F4_CASE
    default: return hipErrorInvalidValue;
  }
}
#endif

}  // namespace f4
