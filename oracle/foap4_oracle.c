/*
 * Plain FP64 CPU oracle for the block-AMR Euler step of foap4
 * (Teunissen et al., arXiv 2605.07612).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP library under
 * paper_2605_07612_amd/csrc, and the HIP library never calls it.
 *
 * Every routine works one cell or one face at a time in double precision, in
 * the order the paper describes, with no blocking or fusion:
 *   ghost filling          Sec. 2.6 (two rounds R1, R2), Sec. 2.2 (restriction,
 *                          limited prolongation, eq. gminmod with theta = 1),
 *                          Sec. 2.4 (Dirichlet / Neumann physical boundaries,
 *                          filled in R1)
 *   stage operator L(U)    Sec. 3.2 (primitive MUSCL reconstruction with the
 *                          minmod or van Leer limiter, Rusanov or HLL flux,
 *                          source term first, then the flux divergence),
 *                          Sec. 3.5 (eq. euler, Einfeldt speeds), Sec. 4.2
 *                          (gravity source S = (0, rho g, rho g.u))
 *   Runge-Kutta stages     Sec. 3.1, eq. feuler and eq. heun; the SSP
 *                          schemes with three and four stages (Sec. 3.1);
 *                          classical RK4, eq. rk4
 *   flux fixing            Sec. 2.7
 *   CFL time step          Sec. 3.1 / Sec. 3.2 step list
 *   refinement criterion   Sec. 3.3, eq. lohner-simple
 *   regrid data remap      Sec. 2.2 (copy / prolong / restrict lists)
 *   scalar advection       Sec. 3.4 (one conserved variable rho, uniform
 *                          velocity v, flux rho v, wave speeds min(v_d, 0)
 *                          and max(v_d, 0)); the same reconstructions, fluxes,
 *                          integrators, ghost filling and flux fixing
 * Readings of points the paper leaves open are listed in the design notes:
 * the Einfeldt speed formula (Toro's form), the CFL formula
 * dt = CFL * min_cells 1 / sum_d (|v_d| + c) / dx, the placement of the flux
 * fix after every stage, the pairwise order of restriction sums, and the
 * Lohner comparison on squares.
 *
 * Layout: state arrays are [block][var][k][j][i] with every spatial index
 * padded by g ghost layers (i fastest), the paper's uu(i,j,k,ivar,iblock)
 * (eq. array-structure) with 0-based indices running from -g to N+g-1.
 * Variables are (rho, m_x, m_y[, m_z], E) for the Euler system and the
 * single variable rho for scalar advection.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t ndim, N, g, nvar;
  int64_t nb;
  const int32_t *level; /* [nb] refinement level of each block                */
  double dx0;           /* cell width at level 0                                */
  double gamma, cfl;
  /* ghost pattern (Sec. 2.6); records grouped by receiving face f = 2*axis+side */
  const int32_t *srl;     /* (a, b): b is the +axis neighbour of a, stored under f = 2*axis+1 */
  const int32_t *srl_off; /* [2*ndim+1]                                         */
  const int32_t *f2c;     /* (c, q, h, c2f_index): coarse c receives from fine q */
  const int32_t *f2c_off;
  const int32_t *c2f;     /* (q, c, h): fine q receives from coarse c            */
  const int32_t *c2f_off;
  const int32_t *bc;      /* (b): face f of block b is a physical boundary         */
  const int32_t *bc_off;
  int32_t bc_type[6][5];  /* per face direction and variable: 0 Dirichlet, 1 Neumann */
  double bc_val[6][5];    /* boundary value u_b, or outward normal derivative u'_b */
  const double *bc_data;  /* optional spatially varying values (eq. bc-data):
                             [boundary record][var][face cell p1 + N p2], replacing
                             bc_val where given                                   */
  int32_t limiter;        /* reconstruction: 0 minmod, 1 van Leer, 2 WENO5 (g >= 3) */
  int32_t flux;           /* numerical flux: 0 Rusanov, 1 HLL                     */
  double grav[3];         /* gravitational acceleration; all zero: no source term */
  int32_t rk;             /* time integrator: 0 Heun (SSP-RK2), 1 SSP-RK3, 2 SSP-RK(4,3),
                             3 classical RK4 (eq. rk4)                          */
  int32_t phys;           /* 0: Euler system (nvar = ndim + 2); 1: scalar advection
                             (Sec. 3.4, nvar = 1)                               */
  double vel[3];          /* uniform advection velocity (phys = 1)             */
} om_mesh;

/* ---------------------------------------------------------------- indexing */

static inline int64_t cells_per_var(const om_mesh *m) {
  int64_t P = m->N + 2 * m->g;
  return m->ndim == 2 ? P * P : P * P * P;
}

/* offset of cell c = (i, j, k) of variable v in block b */
static inline int64_t ix(const om_mesh *m, int64_t b, int v, const int c[3]) {
  int64_t P = m->N + 2 * m->g;
  int64_t o = (b * m->nvar + v) * cells_per_var(m);
  if (m->ndim == 3) o += (int64_t)(c[2] + m->g) * P * P;
  return o + (int64_t)(c[1] + m->g) * P + (c[0] + m->g);
}

static inline double dx_of(const om_mesh *m, int64_t b) {
  return ldexp(m->dx0, -m->level[b]);
}

/* tangential axes of a face with normal axis ax, in increasing order */
static void tangential_axes(int ndim, int ax, int *t1, int *t2) {
  int t[2] = {0, 0}, n = 0;
  for (int d = 0; d < ndim; d++)
    if (d != ax) t[n++] = d;
  *t1 = t[0];
  *t2 = (ndim == 3) ? t[1] : -1;
}

/* minmod = generalized minmod G(a, b, theta = 1) of eq. gminmod: zero unless
 * a and b have the same strict sign, else the one of smaller magnitude. */
static inline double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

/* van Leer limiter (Sec. 3.2 limiter list, van Leer 1977): the harmonic mean
 * 2ab/(a+b) of the two one-sided slopes when they have the same strict sign,
 * else zero; phi(r) = (r + |r|)/(1 + |r|) times b with r = a/b. */
static inline double vanleer(double a, double b) {
  if ((a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0)) return 2.0 * a * b / (a + b);
  return 0.0;
}

/* slope of a cell from its backward (a) and forward (b) differences */
static inline double limited_slope(const om_mesh *m, double a, double b) {
  return m->limiter == 1 ? vanleer(a, b) : minmod(a, b);
}

double om_limiter(int32_t kind, double a, double b) {
  return kind == 1 ? vanleer(a, b) : minmod(a, b);
}

/* WENO5 (Sec. 3.2 limiter list; Jiang and Shu 1996): the value at the right
 * face of cell 2 of the five values v[0..4] (cells i-2 .. i+2), a convex
 * combination of the three third-order candidates
 *   q0 = (2 v0 - 7 v1 + 11 v2)/6, q1 = (-v1 + 5 v2 + 2 v3)/6,
 *   q2 = (2 v2 + 5 v3 - v4)/6
 * with weights alpha_k / sum alpha, alpha_k = d_k / (eps + beta_k)^2,
 * d = (1/10, 6/10, 3/10), eps = 1e-6 and the smoothness indicators
 *   beta_0 = 13/12 (v0 - 2 v1 + v2)^2 + 1/4 (v0 - 4 v1 + 3 v2)^2
 *   beta_1 = 13/12 (v1 - 2 v2 + v3)^2 + 1/4 (v1 - v3)^2
 *   beta_2 = 13/12 (v2 - 2 v3 + v4)^2 + 1/4 (3 v2 - 4 v3 + v4)^2 */
double om_weno5(const double *v) {
  double q0 = (2.0 * v[0] - 7.0 * v[1] + 11.0 * v[2]) / 6.0;
  double q1 = (-v[1] + 5.0 * v[2] + 2.0 * v[3]) / 6.0;
  double q2 = (2.0 * v[2] + 5.0 * v[3] - v[4]) / 6.0;
  double a = v[0] - 2.0 * v[1] + v[2], b = v[0] - 4.0 * v[1] + 3.0 * v[2];
  double b0 = 13.0 / 12.0 * a * a + 0.25 * b * b;
  a = v[1] - 2.0 * v[2] + v[3];
  b = v[1] - v[3];
  double b1 = 13.0 / 12.0 * a * a + 0.25 * b * b;
  a = v[2] - 2.0 * v[3] + v[4];
  b = 3.0 * v[2] - 4.0 * v[3] + v[4];
  double b2 = 13.0 / 12.0 * a * a + 0.25 * b * b;
  double eps = 1e-6;
  double a0 = 0.1 / ((eps + b0) * (eps + b0));
  double a1 = 0.6 / ((eps + b1) * (eps + b1));
  double a2 = 0.3 / ((eps + b2) * (eps + b2));
  return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

/* ------------------------------------------------------- ghost cells, R1/R2 */

/* SRL record: copy g layers across the +axis face of a into b's -axis ghosts
 * and b's first layers into a's +axis ghosts (both sides from one record). */
static void fill_srl(const om_mesh *m, double *u, int ax, int32_t a, int32_t b) {
  int N = m->N, g = m->g, t1, t2;
  tangential_axes(m->ndim, ax, &t1, &t2);
  int n2 = (t2 >= 0) ? N : 1;
  for (int v = 0; v < m->nvar; v++)
    for (int p2 = 0; p2 < n2; p2++)
      for (int p1 = 0; p1 < N; p1++)
        for (int l = 1; l <= g; l++) {
          int src[3] = {0, 0, 0}, dst[3] = {0, 0, 0};
          src[t1] = dst[t1] = p1;
          if (t2 >= 0) src[t2] = dst[t2] = p2;
          src[ax] = N - l; dst[ax] = -l;
          u[ix(m, b, v, dst)] = u[ix(m, a, v, src)];
          src[ax] = l - 1; dst[ax] = N - 1 + l;
          u[ix(m, a, v, dst)] = u[ix(m, b, v, src)];
        }
}

/* F2C record: the coarse ghost cells of face f of c that lie over fine block q
 * (hanging offset h) get the mean of the 2^d fine cells they cover
 * (restriction, Sec. 2.2).  The fine cells are summed in pairs along x, then
 * y, then z, and the sum is scaled by 2^-d. */
static double restrict_mean(const om_mesh *m, const double *u, int64_t q, int v, const int base[3]) {
  int c[3];
  if (m->ndim == 2) {
    double s0, s1;
    c[2] = 0;
    c[0] = base[0]; c[1] = base[1];     double f00 = u[ix(m, q, v, c)];
    c[0] = base[0] + 1;                 double f10 = u[ix(m, q, v, c)];
    c[0] = base[0]; c[1] = base[1] + 1; double f01 = u[ix(m, q, v, c)];
    c[0] = base[0] + 1;                 double f11 = u[ix(m, q, v, c)];
    s0 = f00 + f10;
    s1 = f01 + f11;
    return (s0 + s1) * 0.25;
  } else {
    double f[2][2][2];
    for (int oz = 0; oz < 2; oz++)
      for (int oy = 0; oy < 2; oy++)
        for (int ox = 0; ox < 2; ox++) {
          c[0] = base[0] + ox; c[1] = base[1] + oy; c[2] = base[2] + oz;
          f[oz][oy][ox] = u[ix(m, q, v, c)];
        }
    double a0 = f[0][0][0] + f[0][0][1];
    double a1 = f[0][1][0] + f[0][1][1];
    double a2 = f[1][0][0] + f[1][0][1];
    double a3 = f[1][1][0] + f[1][1][1];
    double b0 = a0 + a1;
    double b1 = a2 + a3;
    return (b0 + b1) * 0.125;
  }
}

static void fill_f2c(const om_mesh *m, double *u, int f, int32_t cb, int32_t q, int32_t h) {
  int N = m->N, g = m->g, half = N / 2, ax = f / 2, side = f % 2, t1, t2;
  tangential_axes(m->ndim, ax, &t1, &t2);
  int bt1 = h & 1, bt2 = (h >> 1) & 1;
  int n2lo = (t2 >= 0) ? bt2 * half : 0, n2hi = (t2 >= 0) ? (bt2 + 1) * half : 1;
  for (int v = 0; v < m->nvar; v++)
    for (int p2 = n2lo; p2 < n2hi; p2++)
      for (int p1 = bt1 * half; p1 < (bt1 + 1) * half; p1++)
        for (int l = 1; l <= g; l++) {
          int cc[3] = {0, 0, 0}, base[3] = {0, 0, 0};
          cc[ax] = side ? N - 1 + l : -l;
          cc[t1] = p1;
          base[ax] = side ? 2 * (l - 1) : N - 2 * l;
          base[t1] = 2 * (p1 - bt1 * half);
          if (t2 >= 0) {
            cc[t2] = p2;
            base[t2] = 2 * (p2 - bt2 * half);
          }
          u[ix(m, cb, v, cc)] = restrict_mean(m, u, q, v, base);
        }
}

/* Limited prolongation (Sec. 2.2): the fine cell that is child sig (+-1 per
 * axis) of coarse cell P of block cb gets u_P + 1/4 sum_d sig_d delta_d with
 * delta_d = minmod(u_P - u_{P-e_d}, u_{P+e_d} - u_P), summed over x, y, z. */
static double prolong_value(const om_mesh *m, const double *u, int64_t cb, int v, const int P[3],
                            const int sig[3]) {
  double uP = u[ix(m, cb, v, P)];
  double corr = 0.0;
  for (int d = 0; d < m->ndim; d++) {
    int lo[3] = {P[0], P[1], P[2]}, hi[3] = {P[0], P[1], P[2]};
    lo[d] -= 1;
    hi[d] += 1;
    double delta = minmod(uP - u[ix(m, cb, v, lo)], u[ix(m, cb, v, hi)] - uP);
    double term = (sig[d] > 0) ? delta : -delta;
    corr = (d == 0) ? term : corr + term;
  }
  return uP + 0.25 * corr;
}

/* C2F record: the g ghost layers of face f of fine block q are prolonged from
 * coarse block c (q sits at hanging offset h on c's face).  Reads c's interior
 * and the face ghosts that R1 filled. */
static void fill_c2f(const om_mesh *m, double *u, int f, int32_t q, int32_t cb, int32_t h) {
  int N = m->N, g = m->g, half = N / 2, ax = f / 2, side = f % 2, t1, t2;
  tangential_axes(m->ndim, ax, &t1, &t2);
  int bt1 = h & 1, bt2 = (h >> 1) & 1;
  int n2 = (t2 >= 0) ? N : 1;
  for (int v = 0; v < m->nvar; v++)
    for (int p2 = 0; p2 < n2; p2++)
      for (int p1 = 0; p1 < N; p1++)
        for (int l = 1; l <= g; l++) {
          int fc[3] = {0, 0, 0}, P[3] = {0, 0, 0}, sig[3] = {0, 0, 0};
          fc[ax] = side ? N - 1 + l : -l;
          int fn = side ? (l - 1) : (2 * N - l); /* fine index inside c along ax */
          P[ax] = fn >> 1;
          sig[ax] = (fn & 1) ? 1 : -1;
          fc[t1] = p1;
          P[t1] = bt1 * half + (p1 >> 1);
          sig[t1] = (p1 & 1) ? 1 : -1;
          if (t2 >= 0) {
            fc[t2] = p2;
            P[t2] = bt2 * half + (p2 >> 1);
            sig[t2] = (p2 & 1) ? 1 : -1;
          }
          u[ix(m, q, v, fc)] = prolong_value(m, u, cb, v, P, sig);
        }
}

/* One round of ghost filling: round 1 = SRL copies and F2C restriction,
 * round 2 = C2F prolongation (which reads round 1's ghosts). */
/* Physical boundary face f of block b (Sec. 2.4): ghost layer l = 1..g
 * outside the face takes, per variable, the value of its mirror cell, the
 * l-th cell inside, reflected through the boundary condition at the face:
 *   Dirichlet (u = u_b on the face):        2 u_b - u_in
 *   Neumann (du/dn = u'_b, n outward):      u_in + (2l - 1) dx u'_b
 * (the face lies (l - 1/2) dx from both cells).  With bc_data, u_b / u'_b
 * are given per face cell (p1, p2) of every boundary record r. */
static void fill_bc(const om_mesh *m, double *u, int f, int32_t r, int32_t b) {
  int N = m->N, ax = f / 2, side = f % 2, t1, t2;
  tangential_axes(m->ndim, ax, &t1, &t2);
  double dx = dx_of(m, b);
  int n2 = (t2 >= 0) ? N : 1;
  for (int v = 0; v < m->nvar; v++)
    for (int l = 1; l <= m->g; l++)
      for (int p2 = 0; p2 < n2; p2++)
        for (int p1 = 0; p1 < N; p1++) {
          int gc[3] = {0, 0, 0}, ic[3] = {0, 0, 0};
          gc[ax] = side ? N - 1 + l : -l;
          ic[ax] = side ? N - l : l - 1;
          gc[t1] = ic[t1] = p1;
          if (t2 >= 0) gc[t2] = ic[t2] = p2;
          double uin = u[ix(m, b, v, ic)];
          double ub = m->bc_data ? m->bc_data[((int64_t)r * m->nvar + v) * (N * n2) + p1 + N * p2] : m->bc_val[f][v];
          u[ix(m, b, v, gc)] = (m->bc_type[f][v] == 0) ? 2.0 * ub - uin : uin + ((2 * l - 1) * dx) * ub;
        }
}

void om_ghost_round(const om_mesh *m, double *u, int round) {
  int nf = 2 * m->ndim;
  if (round == 2) {
    for (int f = 0; f < nf; f++) {
#pragma omp parallel for schedule(static)
      for (int32_t r = m->c2f_off[f]; r < m->c2f_off[f + 1]; r++)
        fill_c2f(m, u, f, m->c2f[3 * r], m->c2f[3 * r + 1], m->c2f[3 * r + 2]);
    }
    return;
  }
  for (int f = 0; f < nf; f++) {
    int ax = f / 2;
#pragma omp parallel for schedule(static)
    for (int32_t r = m->srl_off[f]; r < m->srl_off[f + 1]; r++)
      fill_srl(m, u, ax, m->srl[2 * r], m->srl[2 * r + 1]);
  }
  for (int f = 0; f < nf; f++) {
#pragma omp parallel for schedule(static)
    for (int32_t r = m->f2c_off[f]; r < m->f2c_off[f + 1]; r++)
      fill_f2c(m, u, f, m->f2c[4 * r], m->f2c[4 * r + 1], m->f2c[4 * r + 2]);
  }
  if (m->bc)
    for (int f = 0; f < nf; f++) {
#pragma omp parallel for schedule(static)
      for (int32_t r = m->bc_off[f]; r < m->bc_off[f + 1]; r++) fill_bc(m, u, f, r, m->bc[r]);
    }
}

/* Round R1 (SRL copies, F2C restriction), then round R2 (C2F prolongation). */
void om_ghost_fill(const om_mesh *m, double *u) {
  om_ghost_round(m, u, 1);
  om_ghost_round(m, u, 2);
}

/* ------------------------------------------------------------ Euler physics */

typedef struct { double rho, v[3], p; } prim_t;

/* conservative -> primitive (Sec. 3.5): v = m / rho, p = (gamma-1)(E - m.v/2) */
static prim_t to_primitive(const om_mesh *m, const double *u, int64_t b, const int c[3]) {
  prim_t w;
  w.rho = u[ix(m, b, 0, c)];
  double ke = 0.0;
  w.v[0] = w.v[1] = w.v[2] = 0.0;
  for (int d = 0; d < m->ndim; d++) {
    double md = u[ix(m, b, 1 + d, c)];
    w.v[d] = md / w.rho;
    ke += md * w.v[d];
  }
  double E = u[ix(m, b, m->nvar - 1, c)];
  w.p = (m->gamma - 1.0) * (E - 0.5 * ke);
  return w;
}

/* conserved state and physical flux along axis ax of a primitive state */
static void state_and_flux(const om_mesh *m, const prim_t *w, int ax, double *U, double *F) {
  int nv = m->nvar;
  double vn = w->v[ax];
  double ke = 0.0;
  U[0] = w->rho;
  F[0] = w->rho * vn;
  for (int d = 0; d < m->ndim; d++) {
    double md = w->rho * w->v[d];
    U[1 + d] = md;
    F[1 + d] = md * vn + (d == ax ? w->p : 0.0);
    ke += md * w->v[d];
  }
  double E = w->p / (m->gamma - 1.0) + 0.5 * ke;
  U[nv - 1] = E;
  F[nv - 1] = (E + w->p) * vn;
}

/* Einfeldt wave speeds (Sec. 3.5) of the face between wl and wr along ax:
 * Roe-type averages with sqrt(rho) weights, u_bar = (sL vL + sR vR)/(sL+sR),
 * d_bar^2 = (sL cL^2 + sR cR^2)/(sL+sR) + eta2 (vR - vL)^2,
 * eta2 = sL sR / (2 (sL+sR)^2); the slowest and fastest signals are
 * u_bar - d_bar and u_bar + d_bar. */
static void einfeldt_speeds(const om_mesh *m, const prim_t *wl, const prim_t *wr, int ax, double *smin,
                            double *smax) {
  double sl = sqrt(wl->rho), sr = sqrt(wr->rho);
  double cl2 = m->gamma * wl->p / wl->rho, cr2 = m->gamma * wr->p / wr->rho;
  double vl = wl->v[ax], vr = wr->v[ax];
  double ssum = sl + sr;
  double ubar = (sl * vl + sr * vr) / ssum;
  double eta2 = 0.5 * sl * sr / (ssum * ssum);
  double dv = vr - vl;
  double d2 = (sl * cl2 + sr * cr2) / ssum + eta2 * dv * dv;
  double dbar = sqrt(d2);
  *smin = ubar - dbar;
  *smax = ubar + dbar;
}

/* Rusanov (local Lax-Friedrichs) flux (Sec. 3.2):
 * F = (FL+FR)/2 - a (UR-UL)/2 with a the largest |Einfeldt speed|. */
static void rusanov(const om_mesh *m, const prim_t *wl, const prim_t *wr, int ax, double *F) {
  double UL[5], UR[5], FL[5], FR[5];
  state_and_flux(m, wl, ax, UL, FL);
  state_and_flux(m, wr, ax, UR, FR);
  double smin, smax;
  einfeldt_speeds(m, wl, wr, ax, &smin, &smax);
  double lm = fabs(smin), lp = fabs(smax);
  double a = lm > lp ? lm : lp;
  for (int v = 0; v < m->nvar; v++) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * a * (UR[v] - UL[v]);
}

/* HLL flux (Sec. 3.2; Harten, Lax and van Leer) with the Einfeldt speeds
 * sL <= sR as the fastest signals: the left flux when sL >= 0, the right one
 * when sR <= 0, else the flux of the single intermediate state,
 * (sR FL - sL FR + sL sR (UR - UL)) / (sR - sL). */
static void hll(const om_mesh *m, const prim_t *wl, const prim_t *wr, int ax, double *F) {
  double UL[5], UR[5], FL[5], FR[5];
  state_and_flux(m, wl, ax, UL, FL);
  state_and_flux(m, wr, ax, UR, FR);
  double sl, sr;
  einfeldt_speeds(m, wl, wr, ax, &sl, &sr);
  for (int v = 0; v < m->nvar; v++) {
    if (sl >= 0.0)
      F[v] = FL[v];
    else if (sr <= 0.0)
      F[v] = FR[v];
    else
      F[v] = (sr * FL[v] - sl * FR[v] + sl * sr * (UR[v] - UL[v])) / (sr - sl);
  }
}

static void riemann_flux(const om_mesh *m, const prim_t *wl, const prim_t *wr, int ax, double *F) {
  if (m->flux == 1)
    hll(m, wl, wr, ax, F);
  else
    rusanov(m, wl, wr, ax, F);
}

/* The numerical flux of the mesh's scheme between two primitive states
 * (rho, v_x, v_y, v_z, p) along axis ax. */
void om_riemann_flux(const om_mesh *m, const double *wl, const double *wr, int32_t ax, double *F) {
  prim_t a = {wl[0], {wl[1], wl[2], wl[3]}, wl[4]}, b = {wr[0], {wr[1], wr[2], wr[3]}, wr[4]};
  riemann_flux(m, &a, &b, ax, F);
}

/* ---------------------------------------------------------- scalar advection */

/* Scalar advection (Sec. 3.4): rho_t + div(rho v) = 0 with a uniform velocity
 * v, so the conserved and the primitive variable are both rho.  The face
 * values come from the reconstruction of the mesh's limiter, exactly as for
 * one primitive variable of the Euler system (Sec. 3.2); the physical flux
 * on either side is rho v_ax, and the numerical flux (Rusanov or HLL) takes
 * the slowest and fastest wave speeds min(v_ax, 0) and max(v_ax, 0) that
 * Sec. 3.4 gives. */
static double advection_face_flux(const om_mesh *m, const double *u, int64_t b, const int c[3], int ax) {
  double L, R;
  if (m->limiter == 2) {
    double a[6];
    for (int s = 0; s < 6; s++) {
      int cs[3] = {c[0], c[1], c[2]};
      cs[ax] += s - 2;
      a[s] = u[ix(m, b, 0, cs)];
    }
    double vl[5] = {a[0], a[1], a[2], a[3], a[4]};
    double vr[5] = {a[5], a[4], a[3], a[2], a[1]};
    L = om_weno5(vl);
    R = om_weno5(vr);
  } else {
    int cm[3] = {c[0], c[1], c[2]}, cp[3] = {c[0], c[1], c[2]}, cpp[3] = {c[0], c[1], c[2]};
    cm[ax] -= 1;
    cp[ax] += 1;
    cpp[ax] += 2;
    double r0 = u[ix(m, b, 0, cm)], r1 = u[ix(m, b, 0, c)], r2 = u[ix(m, b, 0, cp)], r3 = u[ix(m, b, 0, cpp)];
    double s1 = limited_slope(m, r1 - r0, r2 - r1);
    double s2 = limited_slope(m, r2 - r1, r3 - r2);
    L = r1 + 0.5 * s1;
    R = r2 - 0.5 * s2;
  }
  double v = m->vel[ax];
  double smin = v < 0.0 ? v : 0.0, smax = v > 0.0 ? v : 0.0;
  double FL = L * v, FR = R * v;
  if (m->flux == 1) {
    if (smin >= 0.0) return FL;
    if (smax <= 0.0) return FR;
    return (smax * FL - smin * FR + smin * smax * (R - L)) / (smax - smin);
  }
  double lm = fabs(smin), lp = fabs(smax);
  double a = lm > lp ? lm : lp;
  return 0.5 * (FL + FR) - 0.5 * a * (R - L);
}

/* Numerical flux through the face between cell c and c + e_ax of block b,
 * from limited linear reconstruction of primitives (Sec. 3.2). */
static void face_flux(const om_mesh *m, const double *u, int64_t b, const int c[3], int ax, double *F) {
  if (m->phys == 1) {
    F[0] = advection_face_flux(m, u, b, c, ax);
    return;
  }
  if (m->limiter == 2) {
    /* WENO5: the left state from cells c-2 .. c+2, the right state from
     * c+3 .. c-1 (the same formula mirrored) */
    double a[6][5];
    for (int s = 0; s < 6; s++) {
      int cs[3] = {c[0], c[1], c[2]};
      cs[ax] += s - 2;
      prim_t w = to_primitive(m, u, b, cs);
      a[s][0] = w.rho;
      a[s][1] = w.v[0];
      a[s][2] = w.v[1];
      a[s][3] = w.v[2];
      a[s][4] = w.p;
    }
    double L[5], R[5];
    for (int k = 0; k < 5; k++) {
      double vl[5] = {a[0][k], a[1][k], a[2][k], a[3][k], a[4][k]};
      double vr[5] = {a[5][k], a[4][k], a[3][k], a[2][k], a[1][k]};
      L[k] = om_weno5(vl);
      R[k] = om_weno5(vr);
    }
    prim_t wl = {L[0], {L[1], L[2], L[3]}, L[4]};
    prim_t wr = {R[0], {R[1], R[2], R[3]}, R[4]};
    riemann_flux(m, &wl, &wr, ax, F);
    return;
  }
  int cm[3] = {c[0], c[1], c[2]}, cp[3] = {c[0], c[1], c[2]}, cpp[3] = {c[0], c[1], c[2]};
  cm[ax] -= 1;
  cp[ax] += 1;
  cpp[ax] += 2;
  prim_t w0 = to_primitive(m, u, b, cm), w1 = to_primitive(m, u, b, c);
  prim_t w2 = to_primitive(m, u, b, cp), w3 = to_primitive(m, u, b, cpp);
  double a0[5] = {w0.rho, w0.v[0], w0.v[1], w0.v[2], w0.p};
  double a1[5] = {w1.rho, w1.v[0], w1.v[1], w1.v[2], w1.p};
  double a2[5] = {w2.rho, w2.v[0], w2.v[1], w2.v[2], w2.p};
  double a3[5] = {w3.rho, w3.v[0], w3.v[1], w3.v[2], w3.p};
  double L[5], R[5];
  for (int k = 0; k < 5; k++) {
    double s1 = limited_slope(m, a1[k] - a0[k], a2[k] - a1[k]);
    double s2 = limited_slope(m, a2[k] - a1[k], a3[k] - a2[k]);
    L[k] = a1[k] + 0.5 * s1;
    R[k] = a2[k] - 0.5 * s2;
  }
  prim_t wl = {L[0], {L[1], L[2], L[3]}, L[4]};
  prim_t wr = {R[0], {R[1], R[2], R[3]}, R[4]};
  riemann_flux(m, &wl, &wr, ax, F);
}

/* One Runge-Kutta sub-step of eq. feuler for Heun's method (eq. heun):
 *   stage 1: uo = dt L(ud) + ud
 *   stage 2: uo = (dt/2) L(ud) + (up + ud)/2
 * with L(U)_c = S_c - sum_d (F_{c+1/2} - F_{c-1/2}) / dx, the source S of the
 * cell's own state first (Sec. 3.2 step list): with gravity g (Sec. 4.2)
 * S = (0, rho g, rho g.u), else zero.  uo may alias up but never ud. */
void om_stage(const om_mesh *m, const double *ud, const double *up, double *uo, int stage, double dt) {
  int N = m->N, nv = m->nvar;
  int nk = (m->ndim == 3) ? N : 1;
  double hdt = 0.5 * dt;
  int has_src = m->phys == 0 && (m->grav[0] != 0.0 || m->grav[1] != 0.0 || m->grav[2] != 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < m->nb; b++) {
    double dx = dx_of(m, b);
    for (int k = 0; k < nk; k++)
      for (int j = 0; j < N; j++)
        for (int i = 0; i < N; i++) {
          int c[3] = {i, j, k};
          double rhs[5] = {0, 0, 0, 0, 0};
          if (has_src) {
            prim_t w = to_primitive(m, ud, b, c);
            double gu = 0.0;
            for (int d = 0; d < m->ndim; d++) {
              rhs[1 + d] = w.rho * m->grav[d];
              gu += m->grav[d] * w.v[d];
            }
            rhs[nv - 1] = w.rho * gu;
          }
          for (int ax = 0; ax < m->ndim; ax++) {
            double Fp[5], Fm[5];
            int cl[3] = {i, j, k};
            cl[ax] -= 1;
            face_flux(m, ud, b, c, ax, Fp);
            face_flux(m, ud, b, cl, ax, Fm);
            for (int v = 0; v < nv; v++) rhs[v] -= (Fp[v] - Fm[v]) / dx;
          }
          for (int v = 0; v < nv; v++) {
            int64_t o = ix(m, b, v, c);
            if (stage == 1)
              uo[o] = dt * rhs[v] + ud[o];
            else
              uo[o] = hdt * rhs[v] + 0.5 * (up[o] + ud[o]);
          }
        }
  }
}

/* One sub-step of the Runge-Kutta framework (eq. feuler) with up to three
 * earlier states:
 *   uo = c dt L(ud) + wd ud + sum_i wp[i] up[i]
 * with L as in om_stage (source first, then the flux divergence); up[i] may
 * be NULL when wp[i] = 0.  uo may alias an up[i] but never ud. */
void om_substep_n(const om_mesh *m, const double *ud, const double *const *up, const double *wp, int np, double *uo,
                  double c, double wd, double dt) {
  int N = m->N, nv = m->nvar;
  int nk = (m->ndim == 3) ? N : 1;
  int has_src = m->phys == 0 && (m->grav[0] != 0.0 || m->grav[1] != 0.0 || m->grav[2] != 0.0);
  double cdt = c * dt;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < m->nb; b++) {
    double dx = dx_of(m, b);
    for (int k = 0; k < nk; k++)
      for (int j = 0; j < N; j++)
        for (int i = 0; i < N; i++) {
          int c3[3] = {i, j, k};
          double rhs[5] = {0, 0, 0, 0, 0};
          if (has_src) {
            prim_t w = to_primitive(m, ud, b, c3);
            double gu = 0.0;
            for (int d = 0; d < m->ndim; d++) {
              rhs[1 + d] = w.rho * m->grav[d];
              gu += m->grav[d] * w.v[d];
            }
            rhs[nv - 1] = w.rho * gu;
          }
          for (int ax = 0; ax < m->ndim; ax++) {
            double Fp[5], Fm[5];
            int cl[3] = {i, j, k};
            cl[ax] -= 1;
            face_flux(m, ud, b, c3, ax, Fp);
            face_flux(m, ud, b, cl, ax, Fm);
            for (int v = 0; v < nv; v++) rhs[v] -= (Fp[v] - Fm[v]) / dx;
          }
          for (int v = 0; v < nv; v++) {
            int64_t o = ix(m, b, v, c3);
            double acc = wd * ud[o];
            for (int q = 0; q < np; q++)
              if (wp[q] != 0.0) acc += wp[q] * up[q][o];
            uo[o] = cdt * rhs[v] + acc;
          }
        }
  }
}

/* Flux fixing (Sec. 2.7): every coarse cell next to a refinement boundary is
 * corrected by dt_s (F_coarse - mean F_fine) / dx_c on its +axis face and by
 * dt_s (mean F_fine - F_coarse) / dx_c on its -axis face.  Fluxes are the
 * ones the stage used (recomputed here from ud).  The 2^(d-1) fine fluxes are
 * averaged in pairs along the lower tangential axis first.  Faces of one
 * coarse block are applied in face order. */
void om_flux_fix(const om_mesh *m, const double *ud, double *uo, double dt_s) {
  int N = m->N, half = N / 2, nv = m->nvar, nf = 2 * m->ndim;
  for (int f = 0; f < nf; f++) {
    int ax = f / 2, side = f % 2, t1, t2;
    tangential_axes(m->ndim, ax, &t1, &t2);
    int32_t r0 = m->f2c_off[f], r1 = m->f2c_off[f + 1];
    int per = (m->ndim == 3) ? 4 : 2;
    for (int32_t r = r0; r < r1; r += per) {
      int32_t cb = m->f2c[4 * r];
      double dxc = dx_of(m, cb);
      int n2 = (t2 >= 0) ? N : 1;
      for (int p2 = 0; p2 < n2; p2++)
        for (int p1 = 0; p1 < N; p1++) {
          int bt1 = p1 >= half, bt2 = (t2 >= 0) ? (p2 >= half) : 0;
          int h = bt1 + 2 * bt2;
          int32_t q = -1;
          for (int s = 0; s < per; s++)
            if (m->f2c[4 * (r + s) + 2] == h) q = m->f2c[4 * (r + s) + 1];
          int cc[3] = {0, 0, 0};
          cc[ax] = side ? N - 1 : -1; /* the face lies between cc and cc + e_ax */
          cc[t1] = p1;
          if (t2 >= 0) cc[t2] = p2;
          double Fc[5];
          face_flux(m, ud, cb, cc, ax, Fc);
          /* fine faces on q's opposite face */
          double Ff[2][2][5];
          for (int o2 = 0; o2 < (t2 >= 0 ? 2 : 1); o2++)
            for (int o1 = 0; o1 < 2; o1++) {
              int fc[3] = {0, 0, 0};
              fc[ax] = side ? -1 : N - 1;
              fc[t1] = 2 * (p1 - bt1 * half) + o1;
              if (t2 >= 0) fc[t2] = 2 * (p2 - bt2 * half) + o2;
              face_flux(m, ud, q, fc, ax, Ff[o2][o1]);
            }
          int cell[3] = {0, 0, 0};
          cell[ax] = side ? N - 1 : 0;
          cell[t1] = p1;
          if (t2 >= 0) cell[t2] = p2;
          for (int v = 0; v < nv; v++) {
            double mean;
            if (t2 >= 0) {
              double s0 = Ff[0][0][v] + Ff[0][1][v];
              double s1 = Ff[1][0][v] + Ff[1][1][v];
              mean = (s0 + s1) * 0.25;
            } else {
              mean = (Ff[0][0][v] + Ff[0][1][v]) * 0.5;
            }
            int64_t o = ix(m, cb, v, cell);
            if (side)
              uo[o] += dt_s * (Fc[v] - mean) / dxc;
            else
              uo[o] += dt_s * (mean - Fc[v]) / dxc;
          }
        }
    }
  }
}

/* CFL time step: dt = cfl * min over interior cells of
 * 1 / sum_d (|v_d| + c) / dx,  c = sqrt(gamma p / rho); for scalar
 * advection (Sec. 3.4) the largest wave speed along d is |v_d|, so every
 * cell of a block gives 1 / sum_d |v_d| / dx. */
double om_dt(const om_mesh *m, const double *u) {
  int N = m->N, nk = (m->ndim == 3) ? N : 1;
  double best = INFINITY;
  for (int64_t b = 0; b < m->nb; b++) {
    double dx = dx_of(m, b);
    for (int k = 0; k < nk; k++)
      for (int j = 0; j < N; j++)
        for (int i = 0; i < N; i++) {
          int c[3] = {i, j, k};
          if (m->phys == 1) {
            double s = 0.0;
            for (int d = 0; d < m->ndim; d++) s += fabs(m->vel[d]) / dx;
            double dtc = 1.0 / s;
            if (dtc < best) best = dtc;
            continue;
          }
          prim_t w = to_primitive(m, u, b, c);
          double cs = sqrt(m->gamma * w.p / w.rho);
          double s = 0.0;
          for (int d = 0; d < m->ndim; d++) s += (fabs(w.v[d]) + cs) / dx;
          double dtc = 1.0 / s;
          if (dtc < best) best = dtc;
        }
  }
  return m->cfl * best;
}

/* Returns the number of interior cells with rho <= 0, p <= 0 or a
 * non-finite variable (scalar advection: a non-finite rho; its rho may
 * take any sign). */
int64_t om_count_unphysical(const om_mesh *m, const double *u) {
  int N = m->N, nk = (m->ndim == 3) ? N : 1;
  int64_t bad = 0;
  for (int64_t b = 0; b < m->nb; b++)
    for (int k = 0; k < nk; k++)
      for (int j = 0; j < N; j++)
        for (int i = 0; i < N; i++) {
          int c[3] = {i, j, k};
          int ok = 1;
          for (int v = 0; v < m->nvar; v++)
            if (!isfinite(u[ix(m, b, v, c)])) ok = 0;
          if (ok && m->phys == 0) {
            prim_t w = to_primitive(m, u, b, c);
            if (!(w.rho > 0.0) || !(w.p > 0.0)) ok = 0;
          }
          bad += !ok;
        }
  return bad;
}

/* One Heun step (eq. heun) with ghost filling before each evaluation of L
 * and flux fixing after each stage: u0 holds U^n on entry and U^{n+1} on
 * exit, u1 is scratch.  Returns the dt that was used. */
void om_substep(const om_mesh *m, const double *ud, const double *up, double *uo, double c, double wd,
                double wp, double dt) {
  const double *ups[1] = {up};
  om_substep_n(m, ud, ups, &wp, 1, uo, c, wd, dt);
}

/* One sub-step of a step with its ghost fill before and flux fix after. */
static void substep(const om_mesh *m, double *ud, double *up, double *uo, double c, double wd, double wp,
                    double dt) {
  om_ghost_fill(m, ud);
  om_substep(m, ud, up, uo, c, wd, wp, dt);
  om_flux_fix(m, ud, uo, c * dt);
}

double om_step(const om_mesh *m, double *u0, double *u1) {
  double dt = om_dt(m, u0);
  if (m->rk == 1 || m->rk == 2) {
    /* a third state: the SSP schemes with three and four stages (Sec. 3.1) */
    size_t n = (size_t)m->nb * m->nvar * cells_per_var(m);
    double *u2 = (double *)calloc(n ? n : 1, sizeof(double));
    if (m->rk == 1) {
      /* SSP-RK3: u1 = u + dt L(u); u2 = 3/4 u + 1/4 (u1 + dt L(u1));
       * u' = 1/3 u + 2/3 (u2 + dt L(u2)) */
      substep(m, u0, NULL, u1, 1.0, 1.0, 0.0, dt);
      substep(m, u1, u0, u2, 0.25, 0.25, 0.75, dt);
      substep(m, u2, u0, u0, 2.0 / 3.0, 2.0 / 3.0, 1.0 / 3.0, dt);
    } else {
      /* SSP-RK(4,3): u1 = u + dt/2 L(u); u2 = u1 + dt/2 L(u1);
       * u3 = 2/3 u + 1/3 u2 + dt/6 L(u2); u' = u3 + dt/2 L(u3) */
      substep(m, u0, NULL, u1, 0.5, 1.0, 0.0, dt);
      substep(m, u1, NULL, u2, 0.5, 1.0, 0.0, dt);
      substep(m, u2, u0, u1, 1.0 / 6.0, 1.0 / 3.0, 2.0 / 3.0, dt);
      substep(m, u1, NULL, u0, 0.5, 1.0, 0.0, dt);
    }
    free(u2);
    return dt;
  }
  if (m->rk == 3) {
    /* classical RK4 (eq. rk4): u1 = u + dt/2 L(u); u2 = u + dt/2 L(u1);
     * u3 = u + dt L(u2); u' = dt/6 L(u3) + (-u + u1 + 2 u2 + u3)/3 */
    size_t n = (size_t)m->nb * m->nvar * cells_per_var(m);
    double *u2 = (double *)calloc(n ? n : 1, sizeof(double));
    double *u3 = (double *)calloc(n ? n : 1, sizeof(double));
    substep(m, u0, NULL, u1, 0.5, 1.0, 0.0, dt);
    substep(m, u1, u0, u2, 0.5, 0.0, 1.0, dt);
    substep(m, u2, u0, u3, 1.0, 0.0, 1.0, dt);
    om_ghost_fill(m, u3);
    const double *ups[3] = {u0, u1, u2};
    const double wps[3] = {-1.0 / 3.0, 1.0 / 3.0, 2.0 / 3.0};
    om_substep_n(m, u3, ups, wps, 3, u0, 1.0 / 6.0, 1.0 / 3.0, dt);
    om_flux_fix(m, u3, u0, dt / 6.0);
    free(u2);
    free(u3);
    return dt;
  }
  om_ghost_fill(m, u0);
  om_stage(m, u0, NULL, u1, 1, dt);
  om_flux_fix(m, u0, u1, dt);
  om_ghost_fill(m, u1);
  om_stage(m, u1, u0, u0, 2, dt);
  om_flux_fix(m, u1, u0, 0.5 * dt);
  return dt;
}

/* Runs n steps; writes the dt of each step to dts (may be NULL).  Stops and
 * returns the failing step + 1 if the state becomes unphysical, else 0. */
int32_t om_run(const om_mesh *m, double *u0, double *u1, int32_t n, double *dts) {
  for (int32_t s = 0; s < n; s++) {
    double dt = om_step(m, u0, u1);
    if (dts) dts[s] = dt;
    if (om_count_unphysical(m, u0) != 0) return s + 1;
  }
  return 0;
}

/* Conserved totals M_v = sum over leaves and interior cells of U_v dx^d,
 * summed per block then over blocks in block order. */
void om_totals(const om_mesh *m, const double *u, double *out) {
  int N = m->N, nk = (m->ndim == 3) ? N : 1;
  for (int v = 0; v < m->nvar; v++) out[v] = 0.0;
  for (int64_t b = 0; b < m->nb; b++) {
    double dx = dx_of(m, b), vol = (m->ndim == 3) ? dx * dx * dx : dx * dx;
    for (int v = 0; v < m->nvar; v++) {
      double s = 0.0;
      for (int k = 0; k < nk; k++)
        for (int j = 0; j < N; j++)
          for (int i = 0; i < N; i++) {
            int c[3] = {i, j, k};
            s += u[ix(m, b, v, c)] * vol;
          }
      out[v] += s;
    }
  }
}

/* ------------------------------------------------------ refinement criterion */

/* Lohner-type indicator of eq. lohner-simple on the density, per interior
 * cell and axis:
 *   E_n = |u_- - 2u + u_+| / (eps_abs + |u - u_-| + |u_+ - u| + eps (|u_-| + 2|u| + |u_+|)).
 * |E|^2 = E_x^2 + E_y^2 (+ E_z^2) is compared with c_refine^2 and
 * c_derefine^2: +1 if some cell exceeds c_refine, -1 if every cell is below
 * c_derefine, else 0.  Needs the face ghosts of u. */
void om_lohner_flags(const om_mesh *m, const double *u, double c_ref, double c_deref, double eps,
                     double eps_abs, int8_t *flags) {
  int N = m->N, nk = (m->ndim == 3) ? N : 1;
  double cr2 = c_ref * c_ref, cd2 = c_deref * c_deref;
  for (int64_t b = 0; b < m->nb; b++) {
    int any_ref = 0, all_deref = 1;
    for (int k = 0; k < nk; k++)
      for (int j = 0; j < N; j++)
        for (int i = 0; i < N; i++) {
          int c[3] = {i, j, k};
          double uc = u[ix(m, b, 0, c)];
          double S = 0.0;
          for (int d = 0; d < m->ndim; d++) {
            int lo[3] = {i, j, k}, hi[3] = {i, j, k};
            lo[d] -= 1;
            hi[d] += 1;
            double um = u[ix(m, b, 0, lo)], up = u[ix(m, b, 0, hi)];
            double num = fabs((um - 2.0 * uc) + up);
            double den = ((eps_abs + fabs(uc - um)) + fabs(up - uc)) +
                         eps * ((fabs(um) + 2.0 * fabs(uc)) + fabs(up));
            double E = num / den;
            S = (d == 0) ? E * E : S + E * E;
          }
          if (S > cr2) any_ref = 1;
          if (!(S < cd2)) all_deref = 0;
        }
    flags[b] = any_ref ? 1 : (all_deref ? -1 : 0);
  }
}

/* --------------------------------------------- learned-indicator features */

/* Per-block raw inputs of the learned refinement indicator: r[2b] = max over
 * interior cells of |grad_c rho| / rho and r[2b+1] = max of |grad_c p| / p,
 * with grad_c the undivided central difference (u_+ - u_-)/2 along each axis
 * (norm over the axes, summed in axis order).  Needs the face ghosts. */
void om_block_raw_features(const om_mesh *m, const double *u, double *r) {
  int N = m->N, nk = (m->ndim == 3) ? N : 1;
  for (int64_t b = 0; b < m->nb; b++) {
    double best_r = 0.0, best_p = 0.0;
    for (int k = 0; k < nk; k++)
      for (int j = 0; j < N; j++)
        for (int i = 0; i < N; i++) {
          int c[3] = {i, j, k};
          prim_t w = to_primitive(m, u, b, c);
          double sr = 0.0, sp = 0.0;
          for (int d = 0; d < m->ndim; d++) {
            int lo[3] = {i, j, k}, hi[3] = {i, j, k};
            lo[d] -= 1;
            hi[d] += 1;
            prim_t wl = to_primitive(m, u, b, lo), wh = to_primitive(m, u, b, hi);
            double dr = 0.5 * (wh.rho - wl.rho), dp = 0.5 * (wh.p - wl.p);
            sr = (d == 0) ? dr * dr : sr + dr * dr;
            sp = (d == 0) ? dp * dp : sp + dp * dp;
          }
          double gr = sqrt(sr) / w.rho, gp = sqrt(sp) / w.p;
          if (gr > best_r) best_r = gr;
          if (gp > best_p) best_p = gp;
        }
    r[2 * b] = best_r;
    r[2 * b + 1] = best_p;
  }
}

/* ------------------------------------------------------------ regrid remap */

/* Data transfer after a mesh change (Sec. 2.2): for each new block n,
 * op[n] = 0 copies old block src[n]; op[n] = 1 prolongs child arg[n]
 * (child bits x + 2y + 4z) of old block src[n] with the limited slopes of
 * prolong_value (old ghosts must be filled); op[n] = 2 restricts the 2^d old
 * children src[n] .. src[n] + 2^d - 1 (child order x + 2y + 4z).  Only
 * interior cells of the new blocks are written. */
void om_remap(const om_mesh *mold, const double *uold, const om_mesh *mnew, double *unew,
              const int32_t *op, const int32_t *src, const int32_t *arg) {
  int N = mnew->N, half = N / 2, nk = (mnew->ndim == 3) ? N : 1;
  for (int64_t n = 0; n < mnew->nb; n++) {
    for (int v = 0; v < mnew->nvar; v++)
      for (int k = 0; k < nk; k++)
        for (int j = 0; j < N; j++)
          for (int i = 0; i < N; i++) {
            int c[3] = {i, j, k};
            double val;
            if (op[n] == 0) {
              val = uold[ix(mold, src[n], v, c)];
            } else if (op[n] == 1) {
              int P[3] = {0, 0, 0}, sig[3] = {0, 0, 0};
              for (int d = 0; d < mnew->ndim; d++) {
                int bit = (arg[n] >> d) & 1;
                P[d] = bit * half + (c[d] >> 1);
                sig[d] = (c[d] & 1) ? 1 : -1;
              }
              val = prolong_value(mold, uold, src[n], v, P, sig);
            } else {
              int ch = 0, base[3] = {0, 0, 0};
              for (int d = 0; d < mnew->ndim; d++) {
                int bit = c[d] >= half;
                ch |= bit << d;
                base[d] = 2 * (c[d] - bit * half);
              }
              val = restrict_mean(mold, uold, src[n] + ch, v, base);
            }
            unew[ix(mnew, n, v, c)] = val;
          }
  }
}
