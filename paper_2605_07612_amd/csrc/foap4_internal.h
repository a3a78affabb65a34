// Internal declarations of the foap4 MI355X library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "foap4.h"

namespace f4 {

constexpr int kMaxLevel = 14;     // finest level accepted in a descriptor
constexpr int kKeyLevel = 16;     // Morton key resolution per tree
constexpr int kTypes = 4;         // SRL, F2C, C2F, BC
enum { kSRL = 0, kF2C = 1, kC2F = 2, kBC = 3 };

// learned indicator: 16 features -> 64 -> 64 -> 3 classes
constexpr int kMlpIn = 16, kMlpHid = 64, kMlpOut = 3;
constexpr int kOffW1 = 0, kOffB1 = 1024, kOffW2 = 1088, kOffB2 = 5184, kOffW3 = 5248, kOffB3 = 5440;
constexpr int kMlpParams = 5443;
constexpr int kMlpPartStride = 5448;  // partial gradient row: parameters, loss, padding
constexpr int kMlpFrags = 26;         // 16x32 / 32x16 BF16 weight operand tiles

// scal[] slots of a mesh (FP64, device)
enum { kDt = 0, kTime = 1, kMaxInv = 2, kBad = 3, kNScal = 8 };

// Offset of cell (i, j, k), -g <= i, j, k < N + g, inside the P^d values
// (P = N + 2g) that one variable of one block occupies.  The rows [k][j]
// (z ghost planes and y ghost rows included) hold the N interior x cells
// only, so the interior of a plane is N^2 contiguous values; the 2g x ghosts
// of every row follow all rows, as [k][j][c] with c = i + g for i < 0 and
// c = i - N + g for i >= N.  The block stride (nvar P^d) and the variable
// stride (P^d) are those of a padded cube.
template <int NDIM>
__host__ __device__ __forceinline__ int cell_off(int i, int j, int k, int N, int g) {
  const int P = N + 2 * g;
  const int row = (NDIM == 3) ? (k + g) * P + (j + g) : (j + g);
  if ((unsigned)i < (unsigned)N) return row * N + i;
  const int rows = (NDIM == 3) ? P * P : P;
  return rows * N + row * 2 * g + (i < 0 ? i + g : i - N + g);
}

struct Leaf {
  int32_t level;
  int32_t g[3];  // global integer coordinates at `level` (tree * 2^level + anchor)
};

struct LeafHash {
  size_t operator()(const std::array<int32_t, 4> &k) const {
    uint64_t h = 1469598103934665603ull;
    for (int32_t v : k) { h ^= (uint32_t)v; h *= 1099511628211ull; }
    return (size_t)h;
  }
};

// Host-side forest of trees: leaf table, lookup, regrid (refine, 2:1 corner
// balance, coarsen) and the old -> new remap lists.
class Topology {
 public:
  int ndim = 3;
  int nt[3] = {1, 1, 1};
  int periodic[3] = {1, 1, 1};  // 0: bounded axis (no neighbours across its ends)
  std::vector<Leaf> leaves;

  void init_uniform(int ndim_, const int32_t nt_[3], int level);
  uint64_t key(const Leaf &l) const;
  int32_t tree_id(const Leaf &l) const;
  void sort_and_index();
  int64_t find(int32_t level, const int32_t g[3]) const;
  // Returns false (and leaves the mesh unchanged) when nothing changes.
  // On success fills op/src/arg for every new block (0 copy, 1 prolong child
  // arg of old src, 2 restrict old children src..src+2^d-1).
  bool regrid(const int8_t *flags, int lmin, int lmax, std::vector<Leaf> &out,
              std::vector<int32_t> &op, std::vector<int32_t> &src, std::vector<int32_t> &arg) const;

 private:
  std::unordered_map<std::array<int32_t, 4>, int64_t, LeafHash> index_;
};

// Device descriptor of one mesh as the kernels see it (copied to the device).
// One sub-step of the Runge-Kutta framework (eq. feuler) in its generic
// form: u(out) = c dt L(u(deriv)) + wd u(deriv) + wp u(prev) [+ wp2 u(prev2)
// + wp3 u(prev3), the form with three earlier states].  States are named by
// role: 0 the current state, 1 the other of the two creation buffers, 2 and
// 3 the extra state buffers.  epi: the last sub-step of a step, which
// evaluates the CFL limit of its output.
struct SubStep {
  double c, wd, wp;
  int32_t deriv, prev, out, epi;
  double wp2, wp3;
  int32_t prev2, prev3;
};
__host__ __device__ __forceinline__ int role_buffer(int role, int cur) {
  return role == 0 ? cur : (role == 1 ? 1 - cur : role);
}

struct MeshDev {
  void *s[4];                 // state buffers: the two of creation and the optional extra two
  const int32_t *level;       // [nb]
  // [nb][2*ndim]: -2 - n for a same-level neighbour n, -1 for a boundary,
  // 2*slot for a C2F face (fine-side flux slot), 2*slot+1 for an F2C face
  const int32_t *face_info;
  const int32_t *srl, *f2c, *c2f, *bc, *fix_list;  // ghost pattern records
  const double *bc_data;      // per-face-cell boundary values [bc record][var][N^(d-1)], or null
  void *bflux_f;              // fine-side face fluxes [n_c2f][nvar][N^(d-1)]
  void *bflux_c;              // coarse-side face fluxes [n_f2c/2^(d-1)][nvar][N^(d-1)]
  double *scal;               // kDt, kTime, kMaxInv, kBad ...
  int64_t nb;
  int64_t item_begin;         // first stage work item of this mesh in its launch
  int64_t r1_begin, r2_begin; // first ghost record of this mesh in R1 / R2 launches
  double dx0;                 // cell width at level 0
  double gamma, cfl;
  double grav[3];             // gravitational acceleration (source term on)
  double vel[3];              // scalar advection: the uniform velocity
  int32_t nv;                 // variables per cell: ndim + 2 (Euler) or 1 (advection)
  double bc_val[6][5];        // physical boundary values per face direction and variable
  int32_t bc_type[6][5];      // 0 Dirichlet, 1 Neumann
  int32_t pn[4];              // record totals per type
  int32_t poff[4][7];         // CSR offsets per type and face
  int32_t n_fix;
  int32_t cur;                // current state buffer
  int32_t N, g, ks;           // block size, ghost layers, k-slabs per tile
  int32_t gather;             // stage reads same-level halos from the neighbours
  int32_t r1_srl;             // SRL records executed in round R1: all pn[kSRL] with stored
                              // ghosts, with gathered halos only those C2F prolongation
                              // reads (indices in srl_sub); R1 then runs pn[kF2C]
                              // restrictions and pn[kBC] boundary faces
  const int32_t *srl_sub;     // with gathered halos: the SRL records R1 runs, else null
  int32_t srl_first;          // without srl_sub: the first SRL record R1 runs (the
                              // records before it, the x faces, are copied by block in
                              // launch_srl_x_blocks)
};

struct Pattern {
  int32_t off[kTypes][7] = {};  // CSR offsets per face (host copy)
  int32_t n[kTypes] = {};       // totals
  int32_t n_fix = 0;            // coarse blocks with at least one F2C face
  int32_t *srl = nullptr, *f2c = nullptr, *c2f = nullptr, *bc = nullptr;
  int32_t *face_info = nullptr, *fix_list = nullptr;
  int32_t *cnt = nullptr;       // classification and scan workspace
  int32_t *tot = nullptr;       // row totals + error flag (device)
  void *bflux_f = nullptr, *bflux_c = nullptr;
  size_t cap[8] = {};           // capacities in bytes of the buffers above
  size_t cap_bflux[2] = {};
  int32_t *srl_c2f = nullptr;   // SRL record indices whose ghosts C2F prolongation reads
  int32_t n_srl_c2f = 0;
  size_t cap_srl_c2f = 0;
};

}  // namespace f4

struct foap4_mesh {
  foap4_mesh_desc d{};
  int nvar = 0, P = 0, nf = 0;
  size_t elem = 0;             // bytes per value
  int64_t block_elems = 0;     // nvar * P^ndim
  void *state[4] = {nullptr, nullptr, nullptr, nullptr};  // extra states of the longer integrators
  size_t state_bytes = 0;
  hipStream_t stream = nullptr;
  int device = 0;              // HIP device current at creation
  int32_t cur = 0;
  f4::Topology topo;
  int64_t revision = 0;
  // device copies of the leaf table
  int32_t *d_level = nullptr, *d_gc = nullptr;
  uint64_t *d_keys = nullptr;
  size_t cap_blocks = 0;
  f4::Pattern pat;
  bool pat_valid = false;
  double *d_scal = nullptr;
  bool dt_valid = false;
  f4::MeshDev *d_dev = nullptr;  // single-mesh descriptor for the plain path
  int64_t *d_item_begin = nullptr;
  // refinement indicator: default for regrid, attached MLP, scratch
  foap4_indicator ind = FOAP4_IND_LOHNER;
  const foap4_mlp *mlp = nullptr;
  void *d_ind = nullptr;       // raw features, features, flags, decisions
  size_t cap_ind = 0;
  int64_t n_fallback = 0;      // blocks of the last MLP flag call that took the Lohner flag
  // features captured by the stage-1 pass of the last step of a foap4_step call
  bool capture = false;
  double *d_featcap = nullptr; // [nb][2] raw maxima of the state at the start of that step
  size_t cap_featcap = 0;      // in blocks
  int64_t steps_done = 0;      // steps taken by foap4_step since creation
  int64_t cap_at = -1, cap_rev = -1;  // steps_done and revision when captured
  // spatially varying boundary values (caller-owned) and the mesh-change callback
  const double *bc_data = nullptr;
  foap4_bc_callback bc_cb = nullptr;
  void *bc_user = nullptr;
  int64_t dev_serial = 0;      // bumped when the device descriptor changes without a regrid
  std::string err;
};

// Learned refinement indicator: FP32 master weights, FP64 Adam moments,
// BF16 MFMA operand fragments and the gradient workspace, all on the device.
struct foap4_mlp {
  hipStream_t stream = nullptr;
  float *d_w = nullptr;        // [kMlpParams] flat W1 b1 W2 b2 W3 b3
  double *d_mv = nullptr;      // [2][kMlpParams] Adam first and second moments
  float *d_grad = nullptr;     // [kMlpParams] last gradient
  void *d_frag = nullptr;      // [kMlpFrags][64] 16-byte operand fragments
  float *d_cls = nullptr;      // [4] per-class sample weight of the loss
  unsigned long long *d_cnt = nullptr;  // [4] label counts (classes, invalid)
  float *d_part = nullptr;     // [groups][kMlpPartStride] per-workgroup partial gradients
  size_t cap_part = 0;         // in workgroups
  double *d_loss = nullptr;    // [cap_loss] loss per iteration
  size_t cap_loss = 0;
  int64_t t = 0;               // Adam steps taken since the last set_params
  bool has_weights = false;
  float threshold = 0.5f;
  std::string err;
};

namespace f4 {

// error helpers
foap4_status fail(foap4_mesh *m, foap4_status s, const std::string &msg);
#define F4_HIP(m, call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::f4::fail((m), FOAP4_E_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

// ks: k-slabs per tile; gather: same-level halos read from the neighbours,
// so round R1 runs its SRL copies only where R2's prolongation needs them;
// x_by_block (a mesh's own descriptor, stored ghosts): for 3D blocks of 16^3
// and 32^3, R1 skips the x-face SRL records, which the single-mesh fill copies
// by block
MeshDev make_dev(const foap4_mesh *m, int ks, int gather, bool x_by_block = false);
foap4_status upload_dev(foap4_mesh *m);

// pattern.hip
foap4_status build_pattern(foap4_mesh *m);
// ghost.hip: round 1 = SRL + F2C + boundary, round 2 = C2F; which = state role
// (0 current, 1 other, 2 third)
// nv: variables per cell (ndim + 2 for the Euler system, 1 for scalar advection)
hipError_t launch_ghost(const MeshDev *d_meshes, int n_meshes, int64_t total, int round, int which,
                        int ndim, bool f64, int grid, hipStream_t s, int nv);
// Same-level x faces of a single 3D mesh with stored ghosts, by block: block
// b's first g columns into its -x neighbour's +x ghosts, its last g columns
// into its +x neighbour's -x ghosts (the x-face SRL records, done by block).
// Blocks of 16^3 or 32^3 only; ndim other than 3 returns hipErrorInvalidValue.
hipError_t launch_srl_x_blocks(const MeshDev *d_mesh, int64_t nblocks, int which, int ndim, bool f64, hipStream_t s,
                               int nv);
// stage.hip
int64_t stage_items_for(int ndim, int N, int64_t nb, int ks);
// nmask: block sizes present in the launch (1: N = 8, 2: N = 16, 4: N = 32);
// scheme: scheme_of() of the meshes in the launch; stage 1 / 2: Heun's stages,
// stage 3: the generic sub-step ss, stage 4: the same with three earlier states
hipError_t launch_stage(const MeshDev *d_meshes, int n_meshes, int64_t total_items, int stage,
                        int ndim, bool f64, int grid, hipStream_t s, int xcd, int nmask, int scheme,
                        const SubStep &ss = SubStep{});
// weno.hip: the WENO5 stage (one thread per interior cell, stored ghosts)
hipError_t launch_weno_stage(const MeshDev *d_mesh, int64_t nblocks, int block_n, int stage, int ndim, bool f64,
                             int scheme, hipStream_t s, const SubStep &ss = SubStep{});
// advect.hip: the scalar advection stage (one workgroup per block, stored ghosts)
hipError_t launch_advect_stage(const MeshDev *d_mesh, int64_t nblocks, int block_n, int n_ghost, int stage, int ndim,
                               bool f64, int limiter, bool hll, hipStream_t s, const SubStep &ss = SubStep{});
// stage 1 of one mesh that also reduces the raw features of its input state
// (feat_raw [nb][2], zeroed by the caller) by atomic maxima
hipError_t launch_stage1_features(const MeshDev *d_mesh, int64_t total_items, int ndim, bool f64, int nmask,
                                  double *feat_raw, hipStream_t s, int scheme);
// scheme bit mask of a mesh: 1 van Leer limiter, 2 HLL flux, 4 gravity source
inline int scheme_of(const foap4_mesh_desc &d) {
  const bool grav = d.gravity[0] != 0.0 || d.gravity[1] != 0.0 || (d.ndim == 3 && d.gravity[2] != 0.0);
  return (d.limiter == FOAP4_LIM_VANLEER ? 1 : 0) | (d.flux == FOAP4_FLUX_HLL ? 2 : 0) | (grav ? 4 : 0);
}
inline int nmask_of(int N) { return N == 8 ? 1 : (N == 16 ? 2 : 4); }
// reduce.hip
hipError_t launch_dt_full(const foap4_mesh *m, hipStream_t s);
hipError_t launch_finalize(const MeshDev *d_meshes, int n_meshes, int advance, hipStream_t s);
hipError_t launch_fluxfix(const MeshDev *d_mesh, int ndim, int nv, bool f64, int n_fix, int stage, hipStream_t s,
                          const SubStep &ss = SubStep{});
hipError_t launch_totals(const foap4_mesh *m, double *d_part, double *d_out, hipStream_t s);
// The allocation-free totals: a fixed device array of kNoAllocScratchDoubles
// FP64 values (2 MiB) per GPU, looked up once per device (with that device
// current) by noalloc_scratch_init; noalloc_scratch returns the looked-up
// device address (null before the lookup).
constexpr int64_t kNoAllocScratchDoubles = 262144;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch_init(int device);
double *noalloc_scratch(int device);
// regrid.hip
// skip (may be null): blocks whose flag is already set are left alone
hipError_t launch_lohner(const foap4_mesh *m, int8_t *d_flags, const int8_t *skip, hipStream_t s);
hipError_t launch_remap(const foap4_mesh *m, const void *src_state, void *dst_state,
                        const int32_t *d_map, int64_t nb_new, hipStream_t s);
// mlp.hip: features of the current state (ghosts filled), raw [nb][2] FP64 and
// feat [nb][16] FP32; MLP decisions: flags[b] = argmax - 1 and decided[b] = 1
// where the largest class probability reaches the threshold, else decided 0
hipError_t launch_block_features(const foap4_mesh *m, double *d_raw, float *d_feat, hipStream_t s);
hipError_t launch_assemble_features(const foap4_mesh *m, const double *d_raw, float *d_feat, hipStream_t s);
hipError_t launch_mlp_decide(const foap4_mlp *net, const float *d_feat, int64_t n, int8_t *d_flags,
                             int8_t *d_decided, hipStream_t s);

}  // namespace f4
