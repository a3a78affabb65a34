// extern "C" entry points of include/foap4.h and the host-side drivers:
// the plain per-kernel step, the batched persistent step captured in a HIP
// graph, regrid, and the work-decomposition autotuner.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>

#include "foap4_internal.h"

namespace {
thread_local std::string g_last_err;
}

namespace f4 {

foap4_status fail(foap4_mesh *m, foap4_status s, const std::string &msg) {
  g_last_err = msg;
  if (m) m->err = msg;
  return s;
}

// The single-mesh fill copies the x-face SRL records by block for 3D blocks of
// 16^3 and 32^3; an 8^3 block is too little work for a workgroup, and its
// records measure faster.
static bool srl_x_by_block(const foap4_mesh *m) { return m->d.ndim == 3 && m->d.block_n >= 16; }

MeshDev make_dev(const foap4_mesh *m, int ks, int gather, bool x_by_block) {
  MeshDev d{};
  d.s[0] = m->state[0];
  d.s[1] = m->state[1];
  d.s[2] = m->state[2];
  d.s[3] = m->state[3];
  d.level = m->d_level;
  d.face_info = m->pat.face_info;
  d.srl = m->pat.srl;
  d.f2c = m->pat.f2c;
  d.c2f = m->pat.c2f;
  d.bc = m->pat.bc;
  d.bc_data = m->bc_data;
  d.fix_list = m->pat.fix_list;
  d.bflux_f = m->pat.bflux_f;
  d.bflux_c = m->pat.bflux_c;
  d.scal = m->d_scal;
  d.nb = (int64_t)m->topo.leaves.size();
  d.item_begin = 0;
  d.r1_begin = 0;
  d.r2_begin = 0;
  d.dx0 = m->d.tree_size / m->d.block_n;
  d.gamma = m->d.gamma;
  d.cfl = m->d.cfl;
  for (int a = 0; a < 3; a++) d.grav[a] = (a < m->d.ndim) ? m->d.gravity[a] : 0.0;
  d.nv = m->nvar;
  for (int a = 0; a < 3; a++)
    d.vel[a] = (m->d.physics == FOAP4_PHYS_ADVECTION && a < m->d.ndim) ? m->d.velocity[a] : 0.0;
  for (int f = 0; f < 6; f++)
    for (int v = 0; v < 5; v++) {
      d.bc_val[f][v] = m->d.bc_value[f][v];
      d.bc_type[f][v] = m->d.bc_type[f][v];
    }
  for (int t = 0; t < kTypes; t++) {
    d.pn[t] = m->pat.n[t];
    for (int f = 0; f < 7; f++) d.poff[t][f] = m->pat.off[t][f];
  }
  d.n_fix = m->pat.n_fix;
  d.cur = m->cur;
  d.N = m->d.block_n;
  d.g = m->d.n_ghost;
  d.ks = std::max(1, std::min(ks, m->d.block_n / 8));
  d.gather = gather;
  // with gathered halos the SRL ghosts are needed only as input of the C2F
  // prolongation stencils: the SRL records with a side that is the coarse
  // block of a C2F record
  d.r1_srl = gather ? m->pat.n_srl_c2f : m->pat.n[kSRL];
  d.srl_sub = gather ? m->pat.srl_c2f : nullptr;
  // with stored ghosts, the single mesh's fill copies the x faces by block
  // (launch_srl_x_blocks) and R1 runs the SRL records from the first y face on
  // (records are grouped by face direction, the x faces first)
  d.srl_first = (!gather && x_by_block && srl_x_by_block(m)) ? m->pat.off[kSRL][2] : 0;
  d.r1_srl -= d.srl_first;
  return d;
}

foap4_status upload_dev(foap4_mesh *m) {
  MeshDev d = make_dev(m, 1, 0, true);
  F4_HIP(m, hipMemcpyAsync(m->d_dev, &d, sizeof(d), hipMemcpyHostToDevice, m->stream));
  F4_HIP(m, hipStreamSynchronize(m->stream));
  return FOAP4_OK;
}

static foap4_status upload_leaves(foap4_mesh *m) {
  const size_t nb = m->topo.leaves.size();
  std::vector<int32_t> lev(nb), gc(3 * nb);
  std::vector<uint64_t> keys(nb);
  for (size_t i = 0; i < nb; i++) {
    const Leaf &L = m->topo.leaves[i];
    lev[i] = L.level;
    for (int d = 0; d < 3; d++) gc[3 * i + d] = L.g[d];
    keys[i] = m->topo.key(L);
  }
  if (nb) {
    F4_HIP(m, hipMemcpyAsync(m->d_level, lev.data(), nb * 4, hipMemcpyHostToDevice, m->stream));
    F4_HIP(m, hipMemcpyAsync(m->d_gc, gc.data(), nb * 12, hipMemcpyHostToDevice, m->stream));
    F4_HIP(m, hipMemcpyAsync(m->d_keys, keys.data(), nb * 8, hipMemcpyHostToDevice, m->stream));
  }
  F4_HIP(m, hipStreamSynchronize(m->stream));
  return FOAP4_OK;
}

static foap4_status check_bad(foap4_mesh *m) {
  double bad = 0.0;
  F4_HIP(m, hipMemcpyAsync(&bad, m->d_scal + kBad, 8, hipMemcpyDeviceToHost, m->stream));
  F4_HIP(m, hipStreamSynchronize(m->stream));
  if (bad != 0.0) return fail(m, FOAP4_E_UNPHYSICAL, "unphysical state (rho <= 0, p <= 0 or non-finite)");
  return FOAP4_OK;
}

// Ghost rounds R1 and R2 of the single mesh (its own descriptor m->d_dev, with
// the x-face SRL copies done by block): the x faces by block and the other
// R1 records, then R2, which reads what R1 wrote.
static foap4_status fill(foap4_mesh *m, const MeshDev *dd, int which) {
  const bool f64 = m->d.prec == FOAP4_F64;
  // x-face SRL records, copied by block where srl_x_by_block holds
  const int64_t nx = srl_x_by_block(m) ? m->pat.off[kSRL][2] : 0;
  const int64_t r1 = m->pat.n[kSRL] - nx + m->pat.n[kF2C] + m->pat.n[kBC], r2 = m->pat.n[kC2F];
  if (nx) F4_HIP(m, launch_srl_x_blocks(dd, (int64_t)m->topo.leaves.size(), which, m->d.ndim, f64, m->stream,
                                        m->nvar));
  F4_HIP(m, launch_ghost(dd, 1, r1, 1, which, m->d.ndim, f64, 0, m->stream, m->nvar));
  if (r2) F4_HIP(m, launch_ghost(dd, 1, r2, 2, which, m->d.ndim, f64, 0, m->stream, m->nvar));
  return FOAP4_OK;
}

static foap4_status ensure_dt(foap4_mesh *m) {
  if (m->dt_valid) return FOAP4_OK;
  F4_HIP(m, launch_dt_full(m, m->stream));
  F4_HIP(m, launch_finalize(m->d_dev, 1, 0, m->stream));
  m->dt_valid = true;
  return FOAP4_OK;
}

}  // namespace f4

using namespace f4;

// ------------------------------------------------------------------ batch type
struct foap4_batch {
  std::vector<foap4_mesh *> meshes;
  std::vector<int64_t> revs, serials;
  int ndim = 3;
  int nv = 5;          // variables per cell, shared by all meshes
  bool f64 = false;
  int ks = 1, wg1 = 0, wg2 = 0, gather = 1, xcd = 1;  // wg1 / wg2: workgroups per CU of stage 1 / 2
  MeshDev *d_devs = nullptr;
  int64_t total_items = 0, r1_total = 0, r2_total = 0;
  int nmask = 0;
  int scheme = 0;  // scheme_of() shared by all meshes
  int integrator = 0;  // shared time integrator
  bool weno = false;   // WENO5 meshes: their own stage kernel per mesh, stored ghosts
  bool adv = false;    // scalar advection meshes: the advection kernel per mesh, stored ghosts
  hipStream_t stream = nullptr, cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool graph_valid = false;
  int n_cu = 256;
  std::string err;
};

extern "C" {

const char *foap4_last_error(const foap4_mesh *mesh) {
  return mesh ? mesh->err.c_str() : g_last_err.c_str();
}

foap4_status foap4_mesh_create(const foap4_mesh_desc *desc, void *state0, void *state1, size_t state_bytes_each,
                               void *hip_stream, foap4_mesh **out) {
  if (!desc || !out) return fail(nullptr, FOAP4_E_INVALID, "null descriptor or output pointer");
  *out = nullptr;
  const foap4_mesh_desc &d = *desc;
  if (d.ndim != 2 && d.ndim != 3) return fail(nullptr, FOAP4_E_INVALID, "ndim must be 2 or 3");
  if (d.block_n != 8 && d.block_n != 16 && d.block_n != 32)
    return fail(nullptr, FOAP4_E_INVALID, "block_n must be 8, 16 or 32");
  if (d.n_ghost < 2 || d.n_ghost > 4 || d.block_n < 2 * d.n_ghost)
    return fail(nullptr, FOAP4_E_INVALID, "n_ghost must be in 2..4 with block_n >= 2 n_ghost");
  int64_t ntrees = 1;
  for (int a = 0; a < d.ndim; a++) {
    if (d.n_trees[a] < 1) return fail(nullptr, FOAP4_E_INVALID, "n_trees must be >= 1");
    if (d.periodic[a] != 0 && d.periodic[a] != 1) return fail(nullptr, FOAP4_E_INVALID, "periodic must be 0 or 1");
    if (!d.periodic[a])
      for (int f = 2 * a; f < 2 * a + 2; f++)
        for (int v = 0; v < (d.physics == FOAP4_PHYS_ADVECTION ? 1 : d.ndim + 2); v++) {
          if (d.bc_type[f][v] != 0 && d.bc_type[f][v] != 1)
            return fail(nullptr, FOAP4_E_INVALID, "bc_type must be 0 (Dirichlet) or 1 (Neumann)");
          if (!std::isfinite(d.bc_value[f][v])) return fail(nullptr, FOAP4_E_INVALID, "bc_value must be finite");
        }
    ntrees *= d.n_trees[a];
  }
  if (ntrees >= 65536) return fail(nullptr, FOAP4_E_INVALID, "at most 65535 trees");
  if (d.init_level < 0 || d.min_level < 0 || d.max_level > kMaxLevel || d.min_level > d.max_level ||
      d.init_level > d.max_level)
    return fail(nullptr, FOAP4_E_INVALID, "levels must satisfy 0 <= min <= max <= 14, init <= max");
  if (!(d.tree_size > 0) || !(d.gamma > 1) || !(d.cfl > 0)) return fail(nullptr, FOAP4_E_INVALID, "tree_size, gamma, cfl");
  if (d.prec != FOAP4_F32 && d.prec != FOAP4_F64) return fail(nullptr, FOAP4_E_INVALID, "prec");
  if (d.limiter != FOAP4_LIM_MINMOD && d.limiter != FOAP4_LIM_VANLEER && d.limiter != FOAP4_LIM_WENO5)
    return fail(nullptr, FOAP4_E_INVALID, "limiter must be minmod, van Leer or WENO5");
  if (d.limiter == FOAP4_LIM_WENO5 && d.n_ghost < 3)
    return fail(nullptr, FOAP4_E_INVALID, "WENO5 needs n_ghost >= 3");
  if (d.flux != FOAP4_FLUX_RUSANOV && d.flux != FOAP4_FLUX_HLL)
    return fail(nullptr, FOAP4_E_INVALID, "flux must be Rusanov or HLL");
  if (d.integrator != FOAP4_RK_HEUN && d.integrator != FOAP4_RK_SSP3 && d.integrator != FOAP4_RK_SSP43 &&
      d.integrator != FOAP4_RK_RK4)
    return fail(nullptr, FOAP4_E_INVALID, "integrator must be Heun, SSP-RK3, SSP-RK(4,3) or RK4");
  for (int a = 0; a < 3; a++)
    if (!std::isfinite(d.gravity[a])) return fail(nullptr, FOAP4_E_INVALID, "gravity must be finite");
  if (d.physics != FOAP4_PHYS_EULER && d.physics != FOAP4_PHYS_ADVECTION)
    return fail(nullptr, FOAP4_E_INVALID, "physics must be Euler or advection");
  if (d.physics == FOAP4_PHYS_ADVECTION) {
    bool moving = false;
    for (int a = 0; a < d.ndim; a++) {
      if (!std::isfinite(d.velocity[a])) return fail(nullptr, FOAP4_E_INVALID, "velocity must be finite");
      moving |= d.velocity[a] != 0.0;
    }
    if (!moving) return fail(nullptr, FOAP4_E_INVALID, "scalar advection needs a non-zero velocity");
    if (scheme_of(d) & 4) return fail(nullptr, FOAP4_E_INVALID, "scalar advection takes no gravity");
  }
  if (!state0 || !state1 || state0 == state1) return fail(nullptr, FOAP4_E_INVALID, "two distinct state buffers needed");
  if ((((uintptr_t)state0) | ((uintptr_t)state1)) & 15u)
    return fail(nullptr, FOAP4_E_INVALID, "state buffers must be 16-byte aligned");
  foap4_mesh *m = new foap4_mesh();
  m->d = d;
  m->nvar = d.physics == FOAP4_PHYS_ADVECTION ? 1 : d.ndim + 2;
  m->P = d.block_n + 2 * d.n_ghost;
  m->nf = 2 * d.ndim;
  m->elem = d.prec == FOAP4_F64 ? 8 : 4;
  m->block_elems = (int64_t)m->nvar * m->P * m->P * (d.ndim == 3 ? m->P : 1);
  m->state[0] = state0;
  m->state[1] = state1;
  m->state_bytes = state_bytes_each;
  m->stream = (hipStream_t)hip_stream;
  if ((size_t)d.max_blocks * m->block_elems * m->elem > state_bytes_each || d.max_blocks < 1) {
    delete m;
    return fail(nullptr, FOAP4_E_INVALID, "state buffers smaller than max_blocks blocks");
  }
  m->topo.init_uniform(d.ndim, d.n_trees, d.init_level);
  for (int a = 0; a < 3; a++) m->topo.periodic[a] = (a < d.ndim) ? d.periodic[a] : 1;
  if ((int64_t)m->topo.leaves.size() > d.max_blocks) {
    delete m;
    return fail(nullptr, FOAP4_E_CAPACITY, "initial mesh exceeds max_blocks");
  }
  auto bail = [&](foap4_status s) {
    std::string msg = m->err;
    foap4_mesh_destroy(m);
    g_last_err = msg;
    return s;
  };
  const size_t cap = (size_t)d.max_blocks;
  if (hipMalloc((void **)&m->d_level, cap * 4) != hipSuccess || hipMalloc((void **)&m->d_gc, cap * 12) != hipSuccess ||
      hipMalloc((void **)&m->d_keys, cap * 8) != hipSuccess || hipMalloc((void **)&m->d_scal, kNScal * 8) != hipSuccess ||
      hipMalloc((void **)&m->d_dev, sizeof(MeshDev)) != hipSuccess) {
    m->err = "device allocation failed";
    return bail(FOAP4_E_HIP);
  }
  m->cap_blocks = cap;
  // set-up of the allocation-free totals on this device (once per device)
  if (hipGetDevice(&m->device) != hipSuccess || noalloc_scratch_init(m->device) != hipSuccess) {
    m->err = "device scratch lookup failed";
    return bail(FOAP4_E_HIP);
  }
  if (hipMemsetAsync(m->d_scal, 0, kNScal * 8, m->stream) != hipSuccess) {
    m->err = "memset failed";
    return bail(FOAP4_E_HIP);
  }
  foap4_status st;
  if ((st = upload_leaves(m)) != FOAP4_OK) return bail(st);
  if ((st = build_pattern(m)) != FOAP4_OK) return bail(st);
  if ((st = upload_dev(m)) != FOAP4_OK) return bail(st);
  *out = m;
  return FOAP4_OK;
}

foap4_status foap4_mesh_destroy(foap4_mesh *m) {
  if (!m) return FOAP4_OK;
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  void *ptrs[] = {m->d_level, m->d_gc, m->d_keys, m->d_scal, m->d_dev, m->d_item_begin,
                  m->pat.srl, m->pat.f2c, m->pat.c2f, m->pat.bc, m->pat.face_info, m->pat.fix_list,
                  m->pat.cnt, m->pat.tot, m->pat.bflux_f, m->pat.bflux_c, m->pat.srl_c2f, m->d_ind, m->d_featcap};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete m;
  return FOAP4_OK;
}

foap4_status foap4_mesh_info(const foap4_mesh *m, int64_t *n_blocks, int64_t *revision, int32_t *cur_state) {
  if (!m) return fail(nullptr, FOAP4_E_INVALID, "null mesh");
  if (n_blocks) *n_blocks = (int64_t)m->topo.leaves.size();
  if (revision) *revision = m->revision;
  if (cur_state) *cur_state = m->cur;
  return FOAP4_OK;
}

foap4_status foap4_mesh_export(const foap4_mesh *m, int32_t *level, int32_t *tree, int32_t *anchor) {
  if (!m) return fail(nullptr, FOAP4_E_INVALID, "null mesh");
  for (size_t i = 0; i < m->topo.leaves.size(); i++) {
    const Leaf &L = m->topo.leaves[i];
    if (level) level[i] = L.level;
    if (tree) tree[i] = m->topo.tree_id(L);
    if (anchor)
      for (int d = 0; d < 3; d++) anchor[3 * i + d] = (d < m->d.ndim) ? L.g[d] - ((L.g[d] >> L.level) << L.level) : 0;
  }
  return FOAP4_OK;
}

foap4_status foap4_ghost_pattern_build(foap4_mesh *m) {
  if (!m) return fail(nullptr, FOAP4_E_INVALID, "null mesh");
  foap4_status st = build_pattern(m);
  if (st != FOAP4_OK) return st;
  return upload_dev(m);
}

foap4_status foap4_ghost_pattern_counts(const foap4_mesh *m, int32_t counts[24]) {
  if (!m || !counts) return fail(nullptr, FOAP4_E_INVALID, "null argument");
  for (int t = 0; t < 4; t++)
    for (int f = 0; f < 6; f++) counts[t * 6 + f] = m->pat.off[t][f + 1] - m->pat.off[t][f];
  return FOAP4_OK;
}

foap4_status foap4_ghost_pattern_export(const foap4_mesh *mc, int32_t *srl, int32_t *f2c, int32_t *c2f,
                                        int32_t *bc) {
  foap4_mesh *m = const_cast<foap4_mesh *>(mc);
  if (!m) return fail(nullptr, FOAP4_E_INVALID, "null mesh");
  const Pattern &P = m->pat;
  if (srl && P.n[kSRL]) F4_HIP(m, hipMemcpyAsync(srl, P.srl, (size_t)P.n[kSRL] * 8, hipMemcpyDeviceToHost, m->stream));
  if (f2c && P.n[kF2C]) F4_HIP(m, hipMemcpyAsync(f2c, P.f2c, (size_t)P.n[kF2C] * 16, hipMemcpyDeviceToHost, m->stream));
  if (c2f && P.n[kC2F]) F4_HIP(m, hipMemcpyAsync(c2f, P.c2f, (size_t)P.n[kC2F] * 12, hipMemcpyDeviceToHost, m->stream));
  if (bc && P.n[kBC]) F4_HIP(m, hipMemcpyAsync(bc, P.bc, (size_t)P.n[kBC] * 4, hipMemcpyDeviceToHost, m->stream));
  F4_HIP(m, hipStreamSynchronize(m->stream));
  return FOAP4_OK;
}

foap4_status foap4_ghost_fill(foap4_mesh *m, int32_t state) {
  if (!m || (state != 0 && state != 1)) return fail(m, FOAP4_E_INVALID, "bad mesh or state index");
  if (!m->pat_valid) return fail(m, FOAP4_E_ORDER, "no ghost pattern");
  return fill(m, m->d_dev, state == m->cur ? 0 : 1);
}

foap4_status foap4_compute_dt(foap4_mesh *m) {
  if (!m) return fail(nullptr, FOAP4_E_INVALID, "null mesh");
  m->dt_valid = false;
  return ensure_dt(m);
}

// Sub-steps of the integrators with extra states (Sec. 3.1, eq. feuler):
// {c, wd, wp, deriv, prev, out, epi[, wp2, wp3, prev2, prev3]}, states by
// role (0 U^n, 1 the other creation buffer, 2 and 3 the extra states);
// U^{n+1} lands in role 0 again.
static const SubStep kSSP3[3] = {{1.0, 1.0, 0.0, 0, 0, 1, 0},
                                 {0.25, 0.25, 0.75, 1, 0, 2, 0},
                                 {2.0 / 3.0, 2.0 / 3.0, 1.0 / 3.0, 2, 0, 0, 1}};
static const SubStep kSSP43[4] = {{0.5, 1.0, 0.0, 0, 0, 1, 0},
                                  {0.5, 1.0, 0.0, 1, 1, 2, 0},
                                  {1.0 / 6.0, 1.0 / 3.0, 2.0 / 3.0, 2, 0, 1, 0},
                                  {0.5, 1.0, 0.0, 1, 1, 0, 1}};
// classical RK4 (eq. rk4): u1 = u + dt/2 L(u), u2 = u + dt/2 L(u1),
// u3 = u + dt L(u2), u' = dt/6 L(u3) + (-u + u1 + 2 u2 + u3)/3 (the last with
// three earlier states: roles 0, 1, 2 with weights -1/3, 1/3, 2/3)
static const SubStep kRK4[4] = {{0.5, 1.0, 0.0, 0, 0, 1, 0, 0.0, 0.0, 0, 0},
                                {0.5, 0.0, 1.0, 1, 0, 2, 0, 0.0, 0.0, 0, 0},
                                {1.0, 0.0, 1.0, 2, 0, 3, 0, 0.0, 0.0, 0, 0},
                                {1.0 / 6.0, 1.0 / 3.0, -1.0 / 3.0, 3, 0, 0, 1, 1.0 / 3.0, 2.0 / 3.0, 1, 2}};
static int substeps_of(int integrator, const SubStep **ss) {
  if (integrator == FOAP4_RK_SSP3) { *ss = kSSP3; return 3; }
  if (integrator == FOAP4_RK_SSP43) { *ss = kSSP43; return 4; }
  if (integrator == FOAP4_RK_RK4) { *ss = kRK4; return 4; }
  *ss = nullptr;
  return 0;
}
// the stage kernel's form of a sub-step: 4 with three earlier states, else 3
static int substep_form(const SubStep &ss) { return (ss.wp2 != 0.0 || ss.wp3 != 0.0) ? 4 : 3; }
// extra states an integrator needs (indices 2 .. 1 + n)
static int extra_states_of(int integrator) {
  return integrator == FOAP4_RK_RK4 ? 2 : (integrator == FOAP4_RK_HEUN ? 0 : 1);
}
static bool extra_states_set(const foap4_mesh *m) {
  for (int i = 0; i < extra_states_of(m->d.integrator); i++)
    if (!m->state[2 + i]) return false;
  return true;
}

foap4_status foap4_mesh_set_extra_state(foap4_mesh *m, int32_t index, void *state, size_t bytes) {
  if (!m || !state) return fail(m, FOAP4_E_INVALID, "null argument");
  if (index != 2 && index != 3) return fail(m, FOAP4_E_INVALID, "extra state index must be 2 or 3");
  if (((uintptr_t)state) & 15u) return fail(m, FOAP4_E_INVALID, "state buffers must be 16-byte aligned");
  if ((size_t)m->d.max_blocks * m->block_elems * m->elem > bytes)
    return fail(m, FOAP4_E_INVALID, "extra state buffer smaller than max_blocks blocks");
  for (int i = 0; i < 4; i++)
    if (i != index && state == m->state[i]) return fail(m, FOAP4_E_INVALID, "state buffers must be distinct");
  m->state[index] = state;
  m->dev_serial++;
  return upload_dev(m);
}

// One stage or sub-step of the plain form: the advection kernel for scalar
// advection, the WENO5 kernel for a WENO5 mesh, else the plane-marching
// kernel (one workgroup per work item).
static hipError_t mesh_stage(foap4_mesh *m, int64_t items, int stage, const SubStep &ss = SubStep{}) {
  const bool f64 = m->d.prec == FOAP4_F64;
  const int ndim = m->d.ndim;
  if (m->d.physics == FOAP4_PHYS_ADVECTION)
    return launch_advect_stage(m->d_dev, (int64_t)m->topo.leaves.size(), m->d.block_n, m->d.n_ghost, stage, ndim, f64,
                               m->d.limiter, m->d.flux == FOAP4_FLUX_HLL, m->stream, ss);
  if (m->d.limiter == FOAP4_LIM_WENO5) {
    return launch_weno_stage(m->d_dev, (int64_t)m->topo.leaves.size(), m->d.block_n, stage, ndim, f64, scheme_of(m->d),
                             m->stream, ss);
  }
  return launch_stage(m->d_dev, 1, items, stage, ndim, f64, 0, m->stream, 0, nmask_of(m->d.block_n), scheme_of(m->d),
                      ss);
}

foap4_status foap4_step(foap4_mesh *m, int32_t n_steps, double *t_out, double *dt_out) {
  if (!m || n_steps < 0) return fail(m, FOAP4_E_INVALID, "bad mesh or step count");
  if (!m->pat_valid) return fail(m, FOAP4_E_ORDER, "no ghost pattern");
  const SubStep *subs = nullptr;
  const int nsub = substeps_of(m->d.integrator, &subs);
  if (nsub && !extra_states_set(m)) return fail(m, FOAP4_E_ORDER, "this integrator needs its extra state buffers");
  if ((nsub || m->d.limiter == FOAP4_LIM_WENO5 || m->nvar == 1) && m->capture && n_steps > 0)
    return fail(m, FOAP4_E_INVALID, "feature capture needs the Heun integrator and a two-ghost limiter");
  if (nsub) {
    const bool f64 = m->d.prec == FOAP4_F64;
    const int ndim = m->d.ndim;
    const int64_t items = stage_items_for(ndim, m->d.block_n, (int64_t)m->topo.leaves.size(), 1);
    foap4_status st;
    if ((st = ensure_dt(m)) != FOAP4_OK) return st;
    for (int32_t s = 0; s < n_steps; s++) {
      for (int k = 0; k < nsub; k++) {
        if ((st = fill(m, m->d_dev, subs[k].deriv)) != FOAP4_OK) return st;
        const int form = substep_form(subs[k]);
        F4_HIP(m, mesh_stage(m, items, form, subs[k]));
        F4_HIP(m, launch_fluxfix(m->d_dev, ndim, m->nvar, f64, m->pat.n_fix, form, m->stream, subs[k]));
      }
      F4_HIP(m, launch_finalize(m->d_dev, 1, 1, m->stream));
    }
    m->steps_done += n_steps;
    if (t_out || dt_out) return foap4_time(m, t_out, dt_out);
    return FOAP4_OK;
  }
  const bool f64 = m->d.prec == FOAP4_F64;
  const int ndim = m->d.ndim;
  const int64_t items = stage_items_for(ndim, m->d.block_n, (int64_t)m->topo.leaves.size(), 1);
  foap4_status st;
  if ((st = ensure_dt(m)) != FOAP4_OK) return st;
  const size_t nb = m->topo.leaves.size();
  const bool capture = m->capture && n_steps > 0 && nb > 0;
  if (capture && m->cap_featcap < nb) {
    if (m->d_featcap) F4_HIP(m, hipFree(m->d_featcap));
    m->d_featcap = nullptr;
    m->cap_featcap = 0;
    F4_HIP(m, hipMalloc((void **)&m->d_featcap, nb * 16));
    m->cap_featcap = nb;
  }
  for (int32_t s = 0; s < n_steps; s++) {
    if ((st = fill(m, m->d_dev, 0)) != FOAP4_OK) return st;
    if (capture && s == n_steps - 1) {
      // last step: stage 1 also reduces the features of its input state
      F4_HIP(m, hipMemsetAsync(m->d_featcap, 0, nb * 16, m->stream));
      F4_HIP(m, launch_stage1_features(m->d_dev, items, ndim, f64, nmask_of(m->d.block_n), m->d_featcap, m->stream,
                                       scheme_of(m->d)));
    } else {
      F4_HIP(m, mesh_stage(m, items, 1));
    }
    F4_HIP(m, launch_fluxfix(m->d_dev, ndim, m->nvar, f64, m->pat.n_fix, 1, m->stream));
    if ((st = fill(m, m->d_dev, 1)) != FOAP4_OK) return st;
    F4_HIP(m, mesh_stage(m, items, 2));
    F4_HIP(m, launch_fluxfix(m->d_dev, ndim, m->nvar, f64, m->pat.n_fix, 2, m->stream));
    F4_HIP(m, launch_finalize(m->d_dev, 1, 1, m->stream));
  }
  m->steps_done += n_steps;
  if (capture) {
    m->cap_at = m->steps_done;
    m->cap_rev = m->revision;
  }
  if (t_out || dt_out) return foap4_time(m, t_out, dt_out);
  return FOAP4_OK;
}

foap4_status foap4_mesh_capture_features(foap4_mesh *m, int32_t on) {
  if (!m) return fail(nullptr, FOAP4_E_INVALID, "null mesh");
  if (on && m->nvar == 1) return fail(m, FOAP4_E_INVALID, "the indicator features are defined for the Euler system");
  m->capture = on != 0;
  return FOAP4_OK;
}

static bool capture_fresh(const foap4_mesh *m) {
  return m->cap_at >= 0 && m->cap_at == m->steps_done && m->cap_rev == m->revision;
}

foap4_status foap4_captured_features(foap4_mesh *m, float *feat_dev, double *raw_dev) {
  if (!m || !feat_dev) return fail(m, FOAP4_E_INVALID, "null argument");
  if (((uintptr_t)feat_dev & 15u) != 0) return fail(m, FOAP4_E_INVALID, "features must be 16-byte aligned");
  if (!capture_fresh(m)) return fail(m, FOAP4_E_ORDER, "no features captured by the last step of this mesh");
  const size_t nb = m->topo.leaves.size();
  F4_HIP(m, launch_assemble_features(m, m->d_featcap, feat_dev, m->stream));
  if (raw_dev) F4_HIP(m, hipMemcpyAsync(raw_dev, m->d_featcap, nb * 16, hipMemcpyDeviceToDevice, m->stream));
  return FOAP4_OK;
}

foap4_status foap4_time(foap4_mesh *m, double *t_out, double *dt_out) {
  if (!m) return fail(nullptr, FOAP4_E_INVALID, "null mesh");
  double sc[kNScal];
  F4_HIP(m, hipMemcpyAsync(sc, m->d_scal, sizeof(sc), hipMemcpyDeviceToHost, m->stream));
  F4_HIP(m, hipStreamSynchronize(m->stream));
  if (t_out) *t_out = sc[kTime];
  if (dt_out) *dt_out = sc[kDt];
  if (sc[kBad] != 0.0) return fail(m, FOAP4_E_UNPHYSICAL, "unphysical state (rho <= 0, p <= 0 or non-finite)");
  return FOAP4_OK;
}

foap4_status foap4_conserved_totals(foap4_mesh *m, double *out) {
  if (!m || !out) return fail(m, FOAP4_E_INVALID, "null argument");
  const size_t nb = m->topo.leaves.size();
  double *d_part = nullptr;
  F4_HIP(m, hipMalloc((void **)&d_part, (nb * m->nvar + m->nvar) * 8));
  hipError_t e = launch_totals(m, d_part, d_part + nb * m->nvar, m->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_part + nb * m->nvar, m->nvar * 8, hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  (void)hipFree(d_part);
  if (e != hipSuccess) return fail(m, FOAP4_E_HIP, std::string("totals: ") + hipGetErrorString(e));
  return FOAP4_OK;
}

foap4_status foap4_conserved_totals_noalloc(foap4_mesh *m, double *out_dev) {
  if (!m || !out_dev) return fail(m, FOAP4_E_INVALID, "null argument");
  const int64_t nb = (int64_t)m->topo.leaves.size();
  if (nb * m->nvar > kNoAllocScratchDoubles)
    return fail(m, FOAP4_E_CAPACITY, "foap4_conserved_totals_noalloc: n_blocks * nvar = " + std::to_string(nb * m->nvar) +
                                         " exceeds its fixed scratch of " + std::to_string(kNoAllocScratchDoubles) +
                                         " values");
  int dev = -1;
  F4_HIP(m, hipGetDevice(&dev));
  if (dev != m->device) return fail(m, FOAP4_E_INVALID, "the mesh's device must be current");
  double *part = noalloc_scratch(dev);
  if (!part) return fail(m, FOAP4_E_ORDER, "device scratch not set up");
  F4_HIP(m, launch_totals(m, part, out_dev, m->stream));
  return FOAP4_OK;
}

// indicator scratch of nb blocks: raw [nb][2] FP64, features [nb][16] FP32,
// flags [nb] directly followed by decisions [nb] (one copy to the host)
struct IndScratch {
  double *raw;
  float *feat;
  int8_t *flags, *decided;
};

static foap4_status ind_scratch(foap4_mesh *m, IndScratch &S) {
  const size_t nb = std::max<size_t>(1, m->topo.leaves.size());
  const size_t a = (nb * 16 + 255) & ~(size_t)255, b = (nb * 64 + 255) & ~(size_t)255, c = nb;
  const size_t bytes = a + b + 2 * c;
  if (m->cap_ind < bytes) {
    if (m->d_ind) F4_HIP(m, hipFree(m->d_ind));
    m->d_ind = nullptr;
    m->cap_ind = 0;
    F4_HIP(m, hipMalloc(&m->d_ind, bytes));
    m->cap_ind = bytes;
  }
  char *p = (char *)m->d_ind;
  S.raw = (double *)p;
  S.feat = (float *)(p + a);
  S.flags = (int8_t *)(p + a + b);
  S.decided = (int8_t *)(p + a + b + c);
  return FOAP4_OK;
}

foap4_status foap4_block_features(foap4_mesh *m, float *feat_dev, double *raw_dev) {
  if (!m || !feat_dev) return fail(m, FOAP4_E_INVALID, "null argument");
  if (m->nvar == 1) return fail(m, FOAP4_E_INVALID, "the indicator features are defined for the Euler system");
  if (((uintptr_t)feat_dev & 15u) != 0) return fail(m, FOAP4_E_INVALID, "features must be 16-byte aligned");
  foap4_status st;
  IndScratch S;
  if (!raw_dev && (st = ind_scratch(m, S)) != FOAP4_OK) return st;
  if ((st = fill(m, m->d_dev, 0)) != FOAP4_OK) return st;
  F4_HIP(m, launch_block_features(m, raw_dev ? raw_dev : S.raw, feat_dev, m->stream));
  return FOAP4_OK;
}

foap4_status foap4_mesh_set_indicator(foap4_mesh *m, foap4_indicator ind, const foap4_mlp *net) {
  if (!m) return fail(nullptr, FOAP4_E_INVALID, "null mesh");
  if (ind != FOAP4_IND_LOHNER && ind != FOAP4_IND_MLP) return fail(m, FOAP4_E_INVALID, "unknown indicator");
  if (ind == FOAP4_IND_MLP && !net) return fail(m, FOAP4_E_INVALID, "the MLP indicator needs a network");
  if (ind == FOAP4_IND_MLP && m->nvar == 1)
    return fail(m, FOAP4_E_INVALID, "the MLP indicator's features are defined for the Euler system");
  m->ind = ind;
  m->mlp = net;
  return FOAP4_OK;
}

foap4_status foap4_indicator_fallbacks(const foap4_mesh *m, int64_t *n_fallback) {
  if (!m || !n_fallback) return fail(nullptr, FOAP4_E_INVALID, "null argument");
  *n_fallback = m->n_fallback;
  return FOAP4_OK;
}

foap4_status foap4_refine_flags(foap4_mesh *m, foap4_indicator ind, int8_t *flags_host) {
  if (!m || !flags_host) return fail(m, FOAP4_E_INVALID, "null argument");
  if (ind != FOAP4_IND_LOHNER && ind != FOAP4_IND_MLP) return fail(m, FOAP4_E_INVALID, "unknown indicator");
  if (ind == FOAP4_IND_MLP && m->nvar == 1)
    return fail(m, FOAP4_E_INVALID, "the MLP indicator's features are defined for the Euler system");
  if (ind == FOAP4_IND_MLP && (!m->mlp || !m->mlp->has_weights))
    return fail(m, FOAP4_E_ORDER, "no MLP with weights attached to this mesh");
  const size_t nb = m->topo.leaves.size();
  if (nb == 0) return FOAP4_OK;
  foap4_status st;
  IndScratch S;
  if ((st = ind_scratch(m, S)) != FOAP4_OK) return st;
  if (ind == FOAP4_IND_MLP && capture_fresh(m)) {
    // features captured by the last step: the network first; ghosts and the
    // criterion only if some block falls back to it
    F4_HIP(m, launch_assemble_features(m, m->d_featcap, S.feat, m->stream));
    F4_HIP(m, launch_mlp_decide(m->mlp, S.feat, (int64_t)nb, S.flags, S.decided, m->stream));
    std::vector<int8_t> both(2 * nb);
    F4_HIP(m, hipMemcpyAsync(both.data(), S.flags, 2 * nb, hipMemcpyDeviceToHost, m->stream));
    F4_HIP(m, hipStreamSynchronize(m->stream));
    m->n_fallback = (int64_t)std::count(both.begin() + nb, both.end(), (int8_t)0);
    if (m->n_fallback > 0) {
      if ((st = fill(m, m->d_dev, 0)) != FOAP4_OK) return st;
      F4_HIP(m, launch_lohner(m, S.flags, S.decided, m->stream));
      F4_HIP(m, hipMemcpyAsync(both.data(), S.flags, nb, hipMemcpyDeviceToHost, m->stream));
      F4_HIP(m, hipStreamSynchronize(m->stream));
    }
    std::memcpy(flags_host, both.data(), nb);
    return FOAP4_OK;
  }
  if ((st = fill(m, m->d_dev, 0)) != FOAP4_OK) return st;
  if (ind == FOAP4_IND_MLP) {
    F4_HIP(m, launch_block_features(m, S.raw, S.feat, m->stream));
    F4_HIP(m, launch_mlp_decide(m->mlp, S.feat, (int64_t)nb, S.flags, S.decided, m->stream));
    F4_HIP(m, launch_lohner(m, S.flags, S.decided, m->stream));
  } else {
    F4_HIP(m, launch_lohner(m, S.flags, nullptr, m->stream));
  }
  if (ind == FOAP4_IND_MLP) {
    std::vector<int8_t> both(2 * nb);
    F4_HIP(m, hipMemcpyAsync(both.data(), S.flags, 2 * nb, hipMemcpyDeviceToHost, m->stream));
    F4_HIP(m, hipStreamSynchronize(m->stream));
    std::memcpy(flags_host, both.data(), nb);
    m->n_fallback = (int64_t)std::count(both.begin() + nb, both.end(), (int8_t)0);
  } else {
    F4_HIP(m, hipMemcpyAsync(flags_host, S.flags, nb, hipMemcpyDeviceToHost, m->stream));
    F4_HIP(m, hipStreamSynchronize(m->stream));
  }
  return FOAP4_OK;
}

foap4_status foap4_regrid(foap4_mesh *m, const int8_t *flags_host, int32_t *changed) {
  if (!m) return fail(nullptr, FOAP4_E_INVALID, "null mesh");
  if (changed) *changed = 0;
  const size_t nb = m->topo.leaves.size();
  std::vector<int8_t> fl(nb);
  foap4_status st;
  if (flags_host) {
    std::memcpy(fl.data(), flags_host, nb);
  } else if ((st = foap4_refine_flags(m, m->ind, fl.data())) != FOAP4_OK) {
    return st;
  }
  std::vector<Leaf> nl;
  std::vector<int32_t> op, src, arg;
  if (!m->topo.regrid(fl.data(), m->d.min_level, m->d.max_level, nl, op, src, arg)) return FOAP4_OK;
  if ((int64_t)nl.size() > m->d.max_blocks) return fail(m, FOAP4_E_CAPACITY, "regrid would exceed max_blocks");
  // old ghosts feed the prolongation stencils
  if ((st = fill(m, m->d_dev, 0)) != FOAP4_OK) return st;
  std::vector<int32_t> map(3 * nl.size());
  for (size_t i = 0; i < nl.size(); i++) {
    map[3 * i] = op[i];
    map[3 * i + 1] = src[i];
    map[3 * i + 2] = arg[i];
  }
  int32_t *d_map = nullptr;
  F4_HIP(m, hipMalloc((void **)&d_map, map.size() * 4 + 4));
  hipError_t e = hipMemcpyAsync(d_map, map.data(), map.size() * 4, hipMemcpyHostToDevice, m->stream);
  if (e == hipSuccess) e = launch_remap(m, m->state[m->cur], m->state[1 - m->cur], d_map, (int64_t)nl.size(), m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  (void)hipFree(d_map);
  if (e != hipSuccess) return fail(m, FOAP4_E_HIP, std::string("remap: ") + hipGetErrorString(e));
  m->cur = 1 - m->cur;
  m->topo.leaves.swap(nl);
  m->topo.sort_and_index();
  m->revision++;
  m->bc_data = nullptr;  // its records belong to the old mesh
  if ((st = upload_leaves(m)) != FOAP4_OK) return st;
  if ((st = build_pattern(m)) != FOAP4_OK) return st;
  if ((st = upload_dev(m)) != FOAP4_OK) return st;
  m->dt_valid = false;
  if (changed) *changed = 1;
  if (m->bc_cb) m->bc_cb(m, m->bc_user);  // may set new boundary data (Sec. 2.4)
  return FOAP4_OK;
}

foap4_status foap4_set_bc_data(foap4_mesh *m, const double *data, int64_t n_values, foap4_bc_callback on_change,
                               void *user) {
  if (!m) return fail(nullptr, FOAP4_E_INVALID, "null mesh");
  const int64_t per = (int64_t)m->nvar * (m->d.ndim == 3 ? m->d.block_n * m->d.block_n : m->d.block_n);
  if (data && n_values != (int64_t)m->pat.n[kBC] * per)
    return fail(m, FOAP4_E_INVALID, "bc_data must hold n_bc * nvar * N^(ndim-1) values");
  m->bc_data = data;
  m->bc_cb = on_change;
  m->bc_user = user;
  m->dev_serial++;
  return upload_dev(m);
}

// -------------------------------------------------------------------- batch

static foap4_status batch_fail(foap4_batch *b, foap4_status s, const std::string &msg) {
  g_last_err = msg;
  if (b) b->err = msg;
  return s;
}
#define B_HIP(b, call)                                                                          \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) return batch_fail((b), FOAP4_E_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

static void drop_graph(foap4_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_valid = false;
}

static foap4_status batch_upload(foap4_batch *b) {
  std::vector<MeshDev> devs;
  int64_t it = 0, r1 = 0, r2 = 0;
  for (foap4_mesh *m : b->meshes) {
    MeshDev d = make_dev(m, b->ks, b->weno ? 0 : b->gather);
    d.item_begin = it;
    d.r1_begin = r1;
    d.r2_begin = r2;
    it += stage_items_for(b->ndim, m->d.block_n, d.nb, d.ks);
    r1 += d.r1_srl + m->pat.n[kF2C] + m->pat.n[kBC];
    r2 += m->pat.n[kC2F];
    devs.push_back(d);
  }
  b->total_items = it;
  b->nmask = 0;
  for (foap4_mesh *m : b->meshes) b->nmask |= nmask_of(m->d.block_n);
  b->r1_total = r1;
  b->r2_total = r2;
  B_HIP(b, hipMemcpyAsync(b->d_devs, devs.data(), devs.size() * sizeof(MeshDev), hipMemcpyHostToDevice, b->stream));
  B_HIP(b, hipStreamSynchronize(b->stream));
  return FOAP4_OK;
}

// one step of every mesh: per stage or sub-step two ghost rounds, the stage
// launch and the flux fix of each mesh with refinement boundaries; then finalize
static int stage_grid(const foap4_batch *b, int stage) {
  const int wg = stage == 1 ? b->wg1 : b->wg2;
  return wg > 0 ? wg * b->n_cu : 0;
}

// One stage or sub-step of every mesh of a batch: one persistent launch of
// the plane-marching kernel over all work items, or for WENO5 meshes and
// scalar advection one launch of their own kernel per mesh.
static hipError_t batch_stage(foap4_batch *b, int stage, int grid, hipStream_t s, const SubStep &ss = SubStep{}) {
  const int n = (int)b->meshes.size();
  if (b->adv) {
    for (int i = 0; i < n; i++) {
      const foap4_mesh *m = b->meshes[i];
      hipError_t e = launch_advect_stage(b->d_devs + i, (int64_t)m->topo.leaves.size(), m->d.block_n, m->d.n_ghost,
                                         stage, b->ndim, b->f64, m->d.limiter, m->d.flux == FOAP4_FLUX_HLL, s, ss);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (!b->weno)
    return launch_stage(b->d_devs, n, b->total_items, stage, b->ndim, b->f64, grid, s, b->xcd, b->nmask, b->scheme, ss);
  for (int i = 0; i < n; i++) {
    const foap4_mesh *m = b->meshes[i];
    hipError_t e = launch_weno_stage(b->d_devs + i, (int64_t)m->topo.leaves.size(), m->d.block_n, stage, b->ndim,
                                     b->f64, b->scheme, s, ss);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static hipError_t batch_enqueue_step(foap4_batch *b, hipStream_t s) {
  const int n = (int)b->meshes.size();
  hipError_t e;
  const SubStep *subs = nullptr;
  const int nsub = substeps_of(b->integrator, &subs);
  for (int k = 0; k < nsub; k++) {  // integrators with extra states: generic sub-steps
    const int which = subs[k].deriv;
    if ((e = launch_ghost(b->d_devs, n, b->r1_total, 1, which, b->ndim, b->f64, 0, s, b->nv)) != hipSuccess) return e;
    if (b->r2_total && (e = launch_ghost(b->d_devs, n, b->r2_total, 2, which, b->ndim, b->f64, 0, s, b->nv)) != hipSuccess)
      return e;
    const int form = substep_form(subs[k]);
    if ((e = batch_stage(b, form, stage_grid(b, 2), s, subs[k])) != hipSuccess) return e;
    for (int i = 0; i < n; i++)
      if (b->meshes[i]->pat.n_fix > 0 &&
          (e = launch_fluxfix(b->d_devs + i, b->ndim, b->nv, b->f64, b->meshes[i]->pat.n_fix, form, s, subs[k])) != hipSuccess)
        return e;
  }
  if (nsub) return launch_finalize(b->d_devs, n, 1, s);
  for (int stage = 1; stage <= 2; stage++) {
    const int which = stage - 1;
    const int grid = stage_grid(b, stage);
    if ((e = launch_ghost(b->d_devs, n, b->r1_total, 1, which, b->ndim, b->f64, 0, s, b->nv)) != hipSuccess) return e;
    if (b->r2_total && (e = launch_ghost(b->d_devs, n, b->r2_total, 2, which, b->ndim, b->f64, 0, s, b->nv)) != hipSuccess)
      return e;
    if ((e = batch_stage(b, stage, grid, s)) != hipSuccess) return e;
    for (int i = 0; i < n; i++)
      if (b->meshes[i]->pat.n_fix > 0 &&
          (e = launch_fluxfix(b->d_devs + i, b->ndim, b->nv, b->f64, b->meshes[i]->pat.n_fix, stage, s)) != hipSuccess)
        return e;
  }
  return launch_finalize(b->d_devs, n, 1, s);
}

static foap4_status batch_prepare(foap4_batch *b) {
  bool stale = !b->graph_valid;
  for (size_t i = 0; i < b->meshes.size(); i++)
    if (b->meshes[i]->revision != b->revs[i] || b->meshes[i]->dev_serial != b->serials[i]) stale = true;
  for (foap4_mesh *m : b->meshes)
    if (!m->dt_valid) {
      foap4_status st = ensure_dt(m);
      if (st != FOAP4_OK) return batch_fail(b, st, m->err);
      B_HIP(b, hipStreamSynchronize(m->stream));
    }
  if (!stale) return FOAP4_OK;
  drop_graph(b);
  for (size_t i = 0; i < b->meshes.size(); i++) {
    b->revs[i] = b->meshes[i]->revision;
    b->serials[i] = b->meshes[i]->dev_serial;
  }
  foap4_status st = batch_upload(b);
  if (st != FOAP4_OK) return st;
  B_HIP(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = batch_enqueue_step(b, b->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return batch_fail(b, FOAP4_E_HIP, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
  }
  b->graph = g;
  B_HIP(b, hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  b->graph_valid = true;
  return FOAP4_OK;
}

foap4_status foap4_batch_create(foap4_mesh *const *meshes, int32_t n, foap4_batch **out) {
  if (!meshes || n < 1 || !out) return fail(nullptr, FOAP4_E_INVALID, "need at least one mesh");
  *out = nullptr;
  foap4_batch *b = new foap4_batch();
  for (int i = 0; i < n; i++) {
    if (!meshes[i]) {
      delete b;
      return fail(nullptr, FOAP4_E_INVALID, "null mesh in batch");
    }
    b->meshes.push_back(meshes[i]);
    b->revs.push_back(-1);
    b->serials.push_back(-1);
  }
  b->ndim = meshes[0]->d.ndim;
  b->f64 = meshes[0]->d.prec == FOAP4_F64;
  b->scheme = scheme_of(meshes[0]->d);
  b->integrator = meshes[0]->d.integrator;
  b->weno = meshes[0]->d.limiter == FOAP4_LIM_WENO5;
  b->adv = meshes[0]->d.physics == FOAP4_PHYS_ADVECTION;
  b->nv = meshes[0]->nvar;
  for (foap4_mesh *m : b->meshes)
    if (m->d.physics != meshes[0]->d.physics) {
      delete b;
      return fail(nullptr, FOAP4_E_INVALID, "batch meshes must share the system (Euler or advection)");
    } else if (m->d.ndim != b->ndim || (m->d.prec == FOAP4_F64) != b->f64) {
      delete b;
      return fail(nullptr, FOAP4_E_INVALID, "batch meshes must share ndim and precision");
    } else if (scheme_of(m->d) != b->scheme) {
      delete b;
      return fail(nullptr, FOAP4_E_INVALID, "batch meshes must share limiter, flux and gravity on/off");
    } else if (m->d.integrator != b->integrator) {
      delete b;
      return fail(nullptr, FOAP4_E_INVALID, "batch meshes must share the time integrator");
    } else if ((m->d.limiter == FOAP4_LIM_WENO5) != b->weno) {
      delete b;
      return fail(nullptr, FOAP4_E_INVALID, "batch meshes must all use WENO5 or none");
    }
  b->stream = meshes[0]->stream;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) b->n_cu = prop.multiProcessorCount;
  if (hipMalloc((void **)&b->d_devs, sizeof(MeshDev) * n) != hipSuccess ||
      hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    foap4_batch_destroy(b);
    return fail(nullptr, FOAP4_E_HIP, "batch allocation failed");
  }
  *out = b;
  return FOAP4_OK;
}

foap4_status foap4_batch_destroy(foap4_batch *b) {
  if (!b) return FOAP4_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  if (b->d_devs) (void)hipFree(b->d_devs);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
  return FOAP4_OK;
}

foap4_status foap4_batch_set_config(foap4_batch *b, int32_t kslabs, int32_t wg_stage1, int32_t wg_stage2,
                                    int32_t xcd_order, int32_t gather_halos) {
  if (!b || (kslabs != 1 && kslabs != 2 && kslabs != 4) || wg_stage1 < 0 || wg_stage1 > 64 || wg_stage2 < 0 ||
      wg_stage2 > 64 || xcd_order < 0 || xcd_order > 2 || (gather_halos != 0 && gather_halos != 1))
    return batch_fail(b, FOAP4_E_INVALID,
                      "kslabs must be 1, 2 or 4, 0 <= workgroups per CU <= 64, xcd_order 0, 1 or 2, gather_halos 0 or 1");
  if (b->ks != kslabs || b->wg1 != wg_stage1 || b->wg2 != wg_stage2 || b->xcd != xcd_order || b->gather != gather_halos)
    drop_graph(b);
  b->ks = kslabs;
  b->wg1 = wg_stage1;
  b->wg2 = wg_stage2;
  b->xcd = xcd_order;
  b->gather = gather_halos;
  return FOAP4_OK;
}

foap4_status foap4_batch_step(foap4_batch *b, int32_t n_steps) {
  if (!b || n_steps < 0) return batch_fail(b, FOAP4_E_INVALID, "bad batch or step count");
  for (foap4_mesh *m : b->meshes) {
    if (!m->pat_valid) return batch_fail(b, FOAP4_E_ORDER, "mesh without ghost pattern");
    if (!extra_states_set(m)) return batch_fail(b, FOAP4_E_ORDER, "this integrator needs its extra state buffers");
  }
  foap4_status st = batch_prepare(b);
  if (st != FOAP4_OK) return st;
  for (int32_t s = 0; s < n_steps; s++) B_HIP(b, hipGraphLaunch(b->exec, b->stream));
  return FOAP4_OK;
}

// ------------------------------------------------------------- phase timing

foap4_status foap4_batch_phase_times(foap4_batch *b, int32_t n_steps, double *out_ms) {
  if (!b || n_steps < 1 || !out_ms) return batch_fail(b, FOAP4_E_INVALID, "bad arguments");
  if (b->integrator != FOAP4_RK_HEUN || b->weno)
    return batch_fail(b, FOAP4_E_INVALID, "phase timing and autotuning time the Heun stages of the plane kernel");
  if (b->adv && b->ks != 1)
    return batch_fail(b, FOAP4_E_INVALID, "the advection kernel has no k-slabs");
  foap4_status st = batch_prepare(b);
  if (st != FOAP4_OK) return st;
  const int n = (int)b->meshes.size();
  hipStream_t s = b->stream;
  // events: per step 2 x (R1, R2, stage, fix) + finalize = 9 intervals
  const int per = 9;
  std::vector<hipEvent_t> ev((size_t)n_steps * per + 1);
  for (auto &e : ev) B_HIP(b, hipEventCreate(&e));
  B_HIP(b, hipEventRecord(ev[0], s));
  int k = 0;
  for (int it = 0; it < n_steps; it++) {
    for (int stage = 1; stage <= 2; stage++) {
      const int which = stage - 1;
      B_HIP(b, launch_ghost(b->d_devs, n, b->r1_total, 1, which, b->ndim, b->f64, 0, s, b->nv));
      B_HIP(b, hipEventRecord(ev[++k], s));
      if (b->r2_total) B_HIP(b, launch_ghost(b->d_devs, n, b->r2_total, 2, which, b->ndim, b->f64, 0, s, b->nv));
      B_HIP(b, hipEventRecord(ev[++k], s));
      B_HIP(b, batch_stage(b, stage, stage_grid(b, stage), s));
      B_HIP(b, hipEventRecord(ev[++k], s));
      for (int i = 0; i < n; i++)
        if (b->meshes[i]->pat.n_fix > 0)
          B_HIP(b, launch_fluxfix(b->d_devs + i, b->ndim, b->nv, b->f64, b->meshes[i]->pat.n_fix, stage, s));
      B_HIP(b, hipEventRecord(ev[++k], s));
    }
    B_HIP(b, launch_finalize(b->d_devs, n, 1, s));
    B_HIP(b, hipEventRecord(ev[++k], s));
  }
  B_HIP(b, hipEventSynchronize(ev[k]));
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int it = 0; it < n_steps; it++) {
    const int base = it * per;
    float ms[9];
    for (int j = 0; j < per; j++) B_HIP(b, hipEventElapsedTime(&ms[j], ev[base + j], ev[base + j + 1]));
    acc[0] += ms[0] + ms[4];  // R1
    acc[1] += ms[1] + ms[5];  // R2
    acc[6] += ms[2];          // stage 1
    acc[7] += ms[6];          // stage 2
    acc[3] += ms[3] + ms[7];  // flux fix
    acc[4] += ms[8];          // finalize
    for (int j = 0; j < per; j++) acc[5] += ms[j];
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  out_ms[0] = acc[0] / (2.0 * n_steps);
  out_ms[1] = acc[1] / (2.0 * n_steps);
  out_ms[2] = (acc[6] + acc[7]) / (2.0 * n_steps);
  out_ms[3] = acc[3] / n_steps;
  out_ms[4] = acc[4] / n_steps;
  out_ms[5] = acc[5] / n_steps;
  out_ms[6] = acc[6] / n_steps;
  out_ms[7] = acc[7] / n_steps;
  return FOAP4_OK;
}

// ---------------------------------------------------------------- autotune

static std::string batch_key(const foap4_batch *b) {
  std::map<int, int64_t> mix;
  int64_t total = 0;
  for (foap4_mesh *m : b->meshes) {
    mix[m->d.block_n] += (int64_t)m->topo.leaves.size();
    total += (int64_t)m->topo.leaves.size();
  }
  char arch[64] = "gfx";
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    std::snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
  for (char *c = arch; *c; c++)
    if (*c == ':' || *c == '"') *c = '_';
  std::ostringstream k;
  k << arch << "|" << (b->f64 ? "f64" : "f32") << "|" << b->ndim << "d|scheme" << b->scheme << "|meshes"
    << b->meshes.size();
  for (auto &kv : mix) {
    // block counts rounded to two significant digits so that nearby sizes share an entry
    const double share = (double)kv.second / (double)std::max<int64_t>(total, 1);
    k << "|N" << kv.first << ":" << (int)std::lround(share * 100.0);
  }
  const int mag = total > 0 ? (int)std::floor(std::log2((double)total)) : 0;
  k << "|log2blocks" << mag;
  return k.str();
}

// cache entries: "key": [kslabs, workgroups per CU of stage 1, of stage 2, xcd_order]
static bool cache_lookup(const char *path, const std::string &key, int cfg[4]) {
  if (!path) return false;
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  while (std::getline(f, line)) {
    const size_t q0 = line.find('"'), q1 = line.find('"', q0 + 1);
    if (q0 == std::string::npos || q1 == std::string::npos) continue;
    if (line.substr(q0 + 1, q1 - q0 - 1) != key) continue;
    int a = 0, c1 = 0, c2 = 0, x = 0;
    if (std::sscanf(line.c_str() + q1 + 1, " : [%d , %d , %d , %d]", &a, &c1, &c2, &x) == 4) {
      cfg[0] = a;
      cfg[1] = c1;
      cfg[2] = c2;
      cfg[3] = x;
      return true;
    }
  }
  return false;
}

static void cache_store(const char *path, const std::string &key, const int cfg[4]) {
  if (!path) return;
  std::vector<std::string> keep;
  {
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
      const size_t q0 = line.find('"'), q1 = line.find('"', q0 + 1);
      if (q0 == std::string::npos || q1 == std::string::npos) continue;
      if (line.substr(q0 + 1, q1 - q0 - 1) == key) continue;
      std::string l = line;
      while (!l.empty() && (l.back() == ',' || l.back() == ' ')) l.pop_back();
      keep.push_back(l);
    }
  }
  char buf[512];
  std::snprintf(buf, sizeof(buf), "  \"%s\": [%d, %d, %d, %d]", key.c_str(), cfg[0], cfg[1], cfg[2], cfg[3]);
  keep.push_back(buf);
  std::ofstream o(path);
  o << "{\n";
  for (size_t i = 0; i < keep.size(); i++) o << keep[i] << (i + 1 < keep.size() ? ",\n" : "\n");
  o << "}\n";
}

foap4_status foap4_batch_autotune(foap4_batch *b, const char *cache_path, int32_t *cfg_out) {
  if (!b) return batch_fail(nullptr, FOAP4_E_INVALID, "null batch");
  if (b->adv) return batch_fail(b, FOAP4_E_INVALID, "the advection kernel has no launch configuration to tune");
  const std::string key = batch_key(b);
  int cached[4] = {1, 0, 0, 1};
  if (cache_lookup(cache_path, key, cached)) {
    foap4_status st = foap4_batch_set_config(b, cached[0], cached[1], cached[2], cached[3], b->gather);
    if (cfg_out)
      for (int i = 0; i < 4; i++) cfg_out[i] = cached[i];
    return st;
  }
  // save the current states and scalars; restored after timing.  The time
  // step of every mesh is computed first, so that the saved scalars hold a
  // valid dt (restoring the scalars of a mesh whose dt is still pending would
  // leave dt = 0 behind a mesh that counts its dt as computed)
  {
    foap4_status st = batch_prepare(b);
    if (st != FOAP4_OK) return st;
  }
  std::vector<void *> saved;
  std::vector<std::array<double, kNScal>> scal(b->meshes.size());
  for (size_t i = 0; i < b->meshes.size(); i++) {
    foap4_mesh *m = b->meshes[i];
    void *p = nullptr;
    const size_t bytes = m->topo.leaves.size() * m->block_elems * m->elem;
    B_HIP(b, hipMalloc(&p, bytes + 16));
    saved.push_back(p);
    B_HIP(b, hipMemcpyAsync(p, m->state[m->cur], bytes, hipMemcpyDeviceToDevice, b->stream));
    B_HIP(b, hipMemcpyAsync(scal[i].data(), m->d_scal, kNScal * 8, hipMemcpyDeviceToHost, b->stream));
  }
  B_HIP(b, hipStreamSynchronize(b->stream));
  auto restore = [&]() -> hipError_t {
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < b->meshes.size() && e == hipSuccess; i++) {
      foap4_mesh *m = b->meshes[i];
      const size_t bytes = m->topo.leaves.size() * m->block_elems * m->elem;
      e = hipMemcpyAsync(m->state[m->cur], saved[i], bytes, hipMemcpyDeviceToDevice, b->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(m->d_scal, scal[i].data(), kNScal * 8, hipMemcpyHostToDevice, b->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    return e;
  };
  const int ks_cand[3] = {1, 2, 4};
  // workgroups per CU of the persistent grid: the stage kernels hold 2-4 per
  // CU, so every count up to 4 and two oversubscribed grids are tried
  constexpr int kWg = 7;
  const int wg_cand[kWg] = {0, 1, 2, 3, 4, 6, 8};
  int max_ks = 1;
  for (foap4_mesh *m : b->meshes) max_ks = std::max(max_ks, m->d.block_n / 8);
  if (b->ndim == 2) max_ks = 1;
  foap4_status result = FOAP4_OK;
  // warm-up in the default configuration (clocks ramp up during the first
  // launches), then two passes over the candidates
  if ((result = foap4_batch_step(b, 8)) == FOAP4_OK && restore() != hipSuccess) result = FOAP4_E_HIP;
  // The two Heun stages are separate launches with the same work items, so
  // each (kslabs, xcd_order) pair takes, per stage, the workgroup count that
  // runs that stage fastest; the rest of a step does not depend on the grid.
  struct Cand {
    int ks, wg, x;
    float s1, s2, rest;
  };
  std::vector<Cand> cands;
  for (int a = 0; a < 3; a++)
    if (ks_cand[a] <= max_ks)
      for (int c = 0; c < kWg; c++)
        for (int x = 0; x < 3; x++) cands.push_back({ks_cand[a], wg_cand[c], x, 3.4e38f, 3.4e38f, 3.4e38f});
  auto choose = [&](int &ks, int &w1, int &w2, int &x) {
    float best = 3.4e38f;
    for (const Cand &p : cands) {
      // best stage-1 and stage-2 grids for this (kslabs, xcd_order)
      float b1 = 3.4e38f, b2 = 3.4e38f, rest = 3.4e38f;
      int g1 = 0, g2 = 0;
      for (const Cand &q : cands) {
        if (q.ks != p.ks || q.x != p.x) continue;
        if (q.s1 < b1) { b1 = q.s1; g1 = q.wg; }
        if (q.s2 < b2) { b2 = q.s2; g2 = q.wg; }
        rest = std::min(rest, q.rest);
      }
      const float t = b1 + b2 + rest;
      if (t < best) {
        best = t;
        ks = p.ks; w1 = g1; w2 = g2; x = p.x;
      }
    }
    return best;
  };
  // pass 1 times every candidate; pass 2 times again those whose stage 1 or
  // stage 2 is within 10 % of the best of that stage (each keeps its fastest
  // run: single runs jitter by a few %)
  for (int pass = 0; pass < 2 && result == FOAP4_OK; pass++) {
    float best1 = 3.4e38f, best2 = 3.4e38f;
    for (const Cand &c : cands) {
      best1 = std::min(best1, c.s1);
      best2 = std::min(best2, c.s2);
    }
    for (Cand &cd : cands) {
      if (pass == 1 && cd.s1 > 1.1f * best1 && cd.s2 > 1.1f * best2) continue;
      if ((result = foap4_batch_set_config(b, cd.ks, cd.wg, cd.wg, cd.x, b->gather)) != FOAP4_OK) break;
      if ((result = foap4_batch_step(b, 1)) != FOAP4_OK) break;  // warm-up
      for (int rep = 0; rep < 2 && result == FOAP4_OK; rep++) {
        double ph[8];
        if ((result = foap4_batch_phase_times(b, 2, ph)) != FOAP4_OK) break;
        cd.s1 = std::min(cd.s1, (float)ph[6]);
        cd.s2 = std::min(cd.s2, (float)ph[7]);
        cd.rest = std::min(cd.rest, (float)(ph[5] - ph[6] - ph[7]));
      }
      if (result != FOAP4_OK) break;
      if (restore() != hipSuccess) { result = FOAP4_E_HIP; break; }
    }
  }
  int best_cfg[4] = {1, 0, 0, 1};
  if (result == FOAP4_OK) choose(best_cfg[0], best_cfg[1], best_cfg[2], best_cfg[3]);
  // pass 3: a minimum over two short runs favours a lucky outlier, so for the
  // chosen (kslabs, xcd_order) the three fastest grids of each stage are
  // timed again (three runs of three steps) and compared by their medians
  for (int stage = 1; stage <= 2 && result == FOAP4_OK; stage++) {
    std::vector<const Cand *> top;
    for (const Cand &q : cands)
      if (q.ks == best_cfg[0] && q.x == best_cfg[3]) top.push_back(&q);
    std::sort(top.begin(), top.end(), [&](const Cand *u, const Cand *v) {
      return stage == 1 ? u->s1 < v->s1 : u->s2 < v->s2;
    });
    if (top.size() > 3) top.resize(3);
    float best_med = 3.4e38f;
    int best_wg = stage == 1 ? best_cfg[1] : best_cfg[2];
    for (const Cand *q : top) {
      const int w1 = stage == 1 ? q->wg : best_cfg[1], w2 = stage == 2 ? q->wg : best_cfg[2];
      if ((result = foap4_batch_set_config(b, best_cfg[0], w1, w2, best_cfg[3], b->gather)) != FOAP4_OK) break;
      if ((result = foap4_batch_step(b, 1)) != FOAP4_OK) break;  // warm-up
      float t[3];
      for (int rep = 0; rep < 3 && result == FOAP4_OK; rep++) {
        double ph[8];
        result = foap4_batch_phase_times(b, 3, ph);
        t[rep] = (float)ph[stage == 1 ? 6 : 7];
      }
      if (result != FOAP4_OK) break;
      std::sort(t, t + 3);
      if (t[1] < best_med) {
        best_med = t[1];
        best_wg = q->wg;
      }
      if (restore() != hipSuccess) { result = FOAP4_E_HIP; break; }
    }
    if (result == FOAP4_OK) (stage == 1 ? best_cfg[1] : best_cfg[2]) = best_wg;
  }
  const hipError_t re = restore();
  for (void *p : saved) (void)hipFree(p);
  if (result != FOAP4_OK) return result;
  if (re != hipSuccess) return batch_fail(b, FOAP4_E_HIP, "autotune restore failed");
  cache_store(cache_path, key, best_cfg);
  if (cfg_out)
    for (int i = 0; i < 4; i++) cfg_out[i] = best_cfg[i];
  return foap4_batch_set_config(b, best_cfg[0], best_cfg[1], best_cfg[2], best_cfg[3], b->gather);
}

}  // extern "C"
