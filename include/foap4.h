/*
 * foap4 on MI355X: C ABI of the block-structured quadtree/octree AMR Euler
 * hot path (Teunissen et al., "foap4: adaptive mesh refinement with OpenACC,
 * MPI, and p4est", arXiv 2605.07612).
 *
 * One library call = one of the paper's public operations (Sec. 2.1, the
 * f4_ routines of the architecture figure): create a mesh, build the ghost
 * pattern (Sec. 2.6), fill ghost cells (Sec. 2.6), advance in time (Sec. 3.1),
 * adapt the mesh (Sec. 2.2), plus the batched multi-problem form.
 *
 * Conventions shared by every entry point:
 *  - Every call returns foap4_status; no C++ exception crosses this ABI.
 *    On an error the mesh is left unchanged and foap4_last_error() holds a
 *    message.
 *  - Device pointers are HIP device addresses on the current device; host
 *    pointers are ordinary CPU memory.  Sizes are in elements unless noted.
 *  - The two state buffers are owned by the caller and passed at creation.
 *    Each holds [max_blocks][nvar] groups of P^ndim values, P = N + 2g (the
 *    paper's uu(i,j,k,ivar,iblock) of eq. array-structure, one padded block
 *    per group), nvar = ndim + 2, variables (rho, m_x, m_y[, m_z], E), for
 *    the Euler system; nvar = 1 (rho) for scalar advection.
 *    Inside a group the rows (j, k) = (-g .. N+g-1)^(ndim-1), k slowest,
 *    hold the N interior x cells each (i fastest), so a plane's interior is
 *    N^2 contiguous values; then the 2g x ghosts of every row, in the same
 *    row order.  Cell (i,j,k), -g <= i,j,k < N + g, is at offset
 *      row * N + i                          if 0 <= i < N,
 *      P^(ndim-1) * N + row * 2g + c        otherwise,
 *    with row = (k+g) P + (j+g) (2D: j+g) and c = i+g (i < 0) or
 *    i-N+g (i >= N).
 *  - Everything else (pattern, flux buffers, time step, scratch) is owned by
 *    the library and freed by foap4_mesh_destroy().
 *  - A mesh is not thread-safe; all its work runs on the HIP stream given at
 *    creation, in stream order.  Calls that return host data synchronize
 *    that stream; the others only enqueue work.
 */
#ifndef FOAP4_H
#define FOAP4_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct foap4_mesh foap4_mesh;   /* opaque, library-owned */
typedef struct foap4_batch foap4_batch; /* opaque, library-owned */
typedef struct foap4_mlp foap4_mlp;     /* opaque, library-owned */

typedef enum {
  FOAP4_OK = 0,
  FOAP4_E_INVALID = -1,    /* bad argument or descriptor                         */
  FOAP4_E_CAPACITY = -2,   /* more blocks than max_blocks                         */
  FOAP4_E_HIP = -3,        /* a HIP runtime call failed                           */
  FOAP4_E_ORDER = -4,      /* call sequence misuse (e.g. step before a pattern)   */
  FOAP4_E_UNPHYSICAL = -5  /* rho <= 0, p <= 0 or a non-finite value was produced */
} foap4_status;

typedef enum { FOAP4_F32 = 0, FOAP4_F64 = 1 } foap4_prec;
typedef enum { FOAP4_IND_LOHNER = 0, FOAP4_IND_MLP = 1 } foap4_indicator;
/* Slope limiter of the primitive reconstruction and numerical flux of the
 * stage (Sec. 3.2): minmod = the generalized minmod of eq. gminmod with
 * theta = 1; van Leer = the harmonic mean 2ab/(a+b) of the one-sided slopes
 * a, b when they share a strict sign, else 0; WENO5 = the fifth-order WENO
 * reconstruction of Jiang and Shu (eps 1e-6), which needs n_ghost >= 3 and
 * runs without feature capture; in a batch (all meshes WENO5) its kernel is
 * launched once per mesh inside the captured step.  Rusanov = local Lax-Friedrichs
 * with the largest Einfeldt speed; HLL = Harten-Lax-van Leer with the
 * Einfeldt speeds u_bar -+ d_bar as the slowest and fastest signals. */
typedef enum { FOAP4_LIM_MINMOD = 0, FOAP4_LIM_VANLEER = 1, FOAP4_LIM_WENO5 = 2 } foap4_limiter;
typedef enum { FOAP4_FLUX_RUSANOV = 0, FOAP4_FLUX_HLL = 1 } foap4_flux;
/* Time integrators (Sec. 3.1), each a sequence of sub-steps of eq. feuler:
 * Heun (SSP-RK2, eq. heun); SSP-RK3 (u1 = u + dt L(u), u2 = 3/4 u + 1/4 (u1 +
 * dt L(u1)), u' = 1/3 u + 2/3 (u2 + dt L(u2))); SSP-RK(4,3) (u1 = u + dt/2
 * L(u), u2 = u1 + dt/2 L(u1), u3 = 2/3 u + 1/3 u2 + dt/6 L(u2), u' = u3 +
 * dt/2 L(u3)); classical RK4 (eq. rk4).  SSP-RK3 and SSP-RK(4,3) need the
 * extra state 2, RK4 the extra states 2 and 3 (foap4_mesh_set_extra_state). */
typedef enum { FOAP4_RK_HEUN = 0, FOAP4_RK_SSP3 = 1, FOAP4_RK_SSP43 = 2, FOAP4_RK_RK4 = 3 } foap4_integrator;
/* The system of conservation laws (Sec. 3): the Euler equations of gas
 * dynamics (Sec. 3.5; nvar = ndim + 2 variables rho, m_x, m_y[, m_z], E) or
 * scalar advection (Sec. 3.4; nvar = 1, the variable rho carried by a
 * uniform velocity v: rho_t + div(rho v) = 0, physical flux rho v_d, wave
 * speeds min(v_d, 0) and max(v_d, 0) along axis d, so the CFL limit of every
 * cell is sum_d |v_d| / dx).  Advection uses the same reconstructions,
 * fluxes, integrators, ghost rounds, flux fixing and regrid as the Euler
 * system; gamma is unused, gravity must be zero, and the learned indicator
 * (whose features need a pressure) is refused. */
typedef enum { FOAP4_PHYS_EULER = 0, FOAP4_PHYS_ADVECTION = 1 } foap4_physics;

/* Mesh descriptor.  A brick of n_trees[0] x n_trees[1] (x n_trees[2]) trees
 * (the paper's p4est brick, Sec. 2.2), periodic or bounded per axis; cubic
 * cells with dx_l = tree_size / (N * 2^l) at refinement level l. */
typedef struct {
  int32_t ndim;        /* 2 or 3                                                     */
  int32_t n_trees[3];  /* trees per axis (n_trees[2] ignored in 2D); product < 65536 */
  int32_t periodic[3]; /* 1: periodic axis; 0: bounded, by bc_type / bc_value          */
  double origin[3];    /* coordinates of the brick's low corner                      */
  double tree_size;    /* edge length of one tree                                    */
  int32_t block_n;     /* N, cells per block edge: 8, 16 or 32                        */
  int32_t n_ghost;     /* g, ghost layers: 2 .. 4 with N >= 2g                         */
  int32_t init_level;  /* uniform level of the initial mesh                          */
  int32_t min_level;   /* coarsest level regrid may produce                          */
  int32_t max_level;   /* finest level regrid may produce (<= 14)                     */
  int64_t max_blocks;  /* capacity of each state buffer, in blocks (Sec. 2.3)        */
  foap4_prec prec;     /* element type of the state buffers                          */
  double gamma;        /* ratio of specific heats (Sec. 3.5)                          */
  double cfl;          /* CFL number of the time step                                 */
  foap4_limiter limiter; /* reconstruction limiter (zero-initialised: minmod)         */
  foap4_flux flux;     /* numerical flux (zero-initialised: Rusanov)                  */
  double gravity[3];   /* uniform gravitational acceleration g (Sec. 4.2): the stage
                          adds the source S = (0, rho g, rho g.u) of each cell's own
                          state to its right-hand side; all zero (the default): no
                          source.  gravity[2] is ignored in 2D.  The time step stays
                          the wave-speed CFL limit. */
  /* Physical boundaries (Sec. 2.4) of the non-periodic axes, per face direction
   * f (0..5: -x, +x, -y, +y, -z, +z) and variable v (rho, m_x, m_y[, m_z], E):
   * bc_type 0 = Dirichlet, u = bc_value on the face; 1 = Neumann, outward
   * normal derivative du/dn = bc_value.  Ghost layer l = 1..g outside the face
   * takes 2 u_b - u_in (Dirichlet) or u_in + (2l - 1) dx u'_b (Neumann), u_in
   * the l-th cell inside, in FP64 rounded once; filled in ghost round R1.  A
   * reflecting wall is Dirichlet 0 on the normal momentum and Neumann 0 on the
   * other variables.  Entries of periodic axes are ignored. */
  int32_t bc_type[6][5];
  double bc_value[6][5];
  foap4_integrator integrator; /* time integrator (zero-initialised: Heun)          */
  foap4_physics physics; /* system (zero-initialised: Euler)                            */
  double velocity[3];    /* scalar advection: the uniform velocity, finite and not zero
                            on every axis at once (velocity[2] ignored in 2D)             */
} foap4_mesh_desc;

/* Creates a mesh at the uniform level desc->init_level (Sec. 2.2) and its
 * leaf table in Morton order per tree (block n = leaf n).  state0/state1 are
 * caller-owned device buffers of state_bytes_each bytes each (>= max_blocks *
 * nvar * P^ndim * element size), 16-byte aligned (256-byte alignment, as
 * torch gives, keeps every block's rows on whole cache lines where the
 * layout allows); the caller writes the initial condition into
 * the interior cells of state0.  hip_stream is a hipStream_t (NULL: default
 * stream).  Builds the ghost pattern.  Errors: FOAP4_E_INVALID (descriptor),
 * FOAP4_E_CAPACITY (initial blocks > max_blocks), FOAP4_E_HIP. */
foap4_status foap4_mesh_create(const foap4_mesh_desc *desc, void *state0, void *state1,
                               size_t state_bytes_each, void *hip_stream, foap4_mesh **out);
foap4_status foap4_mesh_destroy(foap4_mesh *mesh);

/* Number of blocks, mesh revision (changes only when regrid changes the
 * mesh, Sec. 2.2) and which state buffer (0 or 1) holds the current solution. */
foap4_status foap4_mesh_info(const foap4_mesh *mesh, int64_t *n_blocks, int64_t *revision,
                             int32_t *cur_state);

/* Spatially varying boundary values (Sec. 2.4, eq. bc-data).  bc_data_dev
 * is a caller-owned FP64 device array of n_values = n_bc * nvar * N^(ndim-1)
 * values, [boundary record][variable][face cell], the boundary records in the
 * order foap4_ghost_pattern_export returns them (grouped by face direction),
 * face cells p1 + N p2 over the face's tangential axes in increasing order
 * (p1 fastest).  Where given, these values replace bc_value (the types stay
 * those of bc_type).  NULL restores the uniform values.  The array must stay
 * valid while the mesh (or a batch holding it) uses it.  When a regrid changes
 * the mesh, the library drops the array (its records no longer match) and, if
 * on_change is set, calls on_change(mesh, user) on the host from inside
 * foap4_regrid once the new pattern exists; the callback may call
 * foap4_set_bc_data with data for the new records.  Errors: FOAP4_E_INVALID
 * (n_values does not match). */
/* Extra state buffer `index` (2 or 3) of the integrators with more than two
 * sub-steps: caller-owned, device, at least max_blocks * nvar * P^ndim
 * elements (state_bytes bytes), 16-byte aligned, with the layout of the other
 * two, distinct from them.  It holds intermediate stages only.  foap4_step
 * returns FOAP4_E_ORDER for an integrator whose extra states are not set.
 * Errors: FOAP4_E_INVALID (index, size, alignment, aliasing). */
foap4_status foap4_mesh_set_extra_state(foap4_mesh *mesh, int32_t index, void *state, size_t state_bytes);

typedef void (*foap4_bc_callback)(foap4_mesh *mesh, void *user);
foap4_status foap4_set_bc_data(foap4_mesh *mesh, const double *bc_data_dev, int64_t n_values,
                               foap4_bc_callback on_change, void *user);

/* Host copies of the leaf table: level[n_blocks], tree[n_blocks] (tree id
 * t_x + n_x (t_y + n_y t_z)) and anchor[n_blocks][3] (integer position of the
 * block inside its tree at its level).  Any pointer may be NULL. */
foap4_status foap4_mesh_export(const foap4_mesh *mesh, int32_t *level, int32_t *tree, int32_t *anchor);

/* Builds the ghost pattern on the device (Sec. 2.6): for every block face a
 * binary search in the sorted leaf keys classifies the neighbour as same
 * level (SRL), finer (this block receives F2C restriction), coarser (this
 * block receives C2F prolongation) or boundary; records are grouped by face
 * direction (-x,+x,-y,+y,-z,+z) and sorted by receiving block and hanging
 * offset with a stable count/scan/scatter.  Called by create and regrid;
 * callable again at any time (idempotent). */
foap4_status foap4_ghost_pattern_build(foap4_mesh *mesh);

/* Record counts: counts[t * 6 + f] for type t (0 SRL, 1 F2C, 2 C2F, 3 BC)
 * and face f.  SRL records are stored once per face pair under the + face. */
foap4_status foap4_ghost_pattern_counts(const foap4_mesh *mesh, int32_t counts[24]);

/* Host copies of the pattern records, each array sized by the counts above
 * and ordered by face, then receiving block, then hanging offset:
 *   srl[n][2] (a, b)           b is the + neighbour of a
 *   f2c[n][4] (c, q, h, k)     coarse c receives restricted data from fine q
 *                              at hanging offset h; k indexes q's C2F record
 *   c2f[n][3] (q, c, h)        fine q receives prolonged data from coarse c
 *   bc[n]     (b)              physical boundary face of b on a bounded
 *                              axis (grouped by face direction)
 * Any pointer may be NULL. */
foap4_status foap4_ghost_pattern_export(const foap4_mesh *mesh, int32_t *srl, int32_t *f2c,
                                        int32_t *c2f, int32_t *bc);

/* Executes the stored pattern on state buffer `state` (0 or 1): round R1
 * (SRL copies and F2C restriction), then round R2 (C2F limited
 * prolongation, which reads R1's ghosts) (Sec. 2.6).  Only face ghosts are
 * written; corner and edge ghosts are never touched (Sec. 2.1). */
foap4_status foap4_ghost_fill(foap4_mesh *mesh, int32_t state);

/* Computes the CFL time step of the current state on the device:
 * dt = cfl * min over interior cells of 1 / sum_d (|v_d| + c) / dx_l, in
 * FP64.  Done automatically by the first foap4_step after create/regrid. */
foap4_status foap4_compute_dt(foap4_mesh *mesh);

/* Advances n_steps steps of the mesh's time integrator (Heun, eq. heun, by
 * default; SSP-RK3 or SSP-RK(4,3), Sec. 3.1) on the current state: per
 * sub-step ghost fill, fused flux/update stage, flux fix at refinement
 * boundaries (Sec. 2.7); the next dt comes from the new state (FP64
 * reduction on the device).  The result is in the current state buffer.
 * FOAP4_E_ORDER if the integrator needs extra state buffers that are not set;
 * FOAP4_E_INVALID if feature capture is on with an integrator other than
 * Heun.  Enqueues only; if t_out/dt_out are non-NULL
 * the stream is synchronized and the simulation time / the dt of the next
 * step are returned, and FOAP4_E_UNPHYSICAL is reported if the state went
 * bad.  This is the plain form: one kernel launch per operation and one
 * workgroup per block tile.  Ghost cells of both state buffers are
 * unspecified after a step (the stages may overwrite them); every call that
 * reads ghosts fills them first. */
foap4_status foap4_step(foap4_mesh *mesh, int32_t n_steps, double *t_out, double *dt_out);

/* Reads back the simulation time and the dt of the next step (synchronizes). */
foap4_status foap4_time(foap4_mesh *mesh, double *t_out, double *dt_out);

/* Conserved totals sum over leaves and cells of U_v dx_l^d in FP64
 * (out[nvar], host).  Synchronizes. */
foap4_status foap4_conserved_totals(foap4_mesh *mesh, double *out);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the totals of
 * foap4_conserved_totals, computed by the same kernels in the same order
 * (bit-identical), written to out_dev[nvar] (FP64, device, caller-owned) on
 * the mesh's stream.  Enqueue only; allocates nothing and synchronizes
 * nothing.  Its per-block partial sums live in a fixed device array of
 * 262144 FP64 values (2 MiB) per GPU, set up by foap4_mesh_create on that
 * GPU and held until the process ends.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (several streams, several threads)
 * race and must be ordered by the caller.  The mesh's device must be
 * current.  Errors: FOAP4_E_CAPACITY if n_blocks * nvar > 262144 (nothing
 * is enqueued), FOAP4_E_INVALID (null pointer, another device current),
 * FOAP4_E_HIP (launch failure). */
foap4_status foap4_conserved_totals_noalloc(foap4_mesh *mesh, double *out_dev);

/* Per-block refinement flags (+1 refine, 0 keep, -1 derefine; Sec. 2.2) of
 * the current state, written to flags_host[n_blocks].  Both indicators fill
 * ghosts first.  FOAP4_IND_LOHNER is the paper's criterion (Sec. 3.3, eq.
 * lohner-simple, constants of Sec. 5.4) on the density, in FP64.
 * FOAP4_IND_MLP needs an MLP attached with foap4_mesh_set_indicator and
 * holding weights (else FOAP4_E_ORDER): features (foap4_block_features), the
 * network, flag = argmax class - 1 where the largest class probability is
 * at least the MLP's threshold, and the Lohner flag elsewhere (computed only
 * for those blocks). */
foap4_status foap4_refine_flags(foap4_mesh *mesh, foap4_indicator ind, int8_t *flags_host);

/* Adapts the mesh (Sec. 2.2): refine every +1 block below max_level, then
 * restore 2:1 balance across faces, edges and corners, then coarsen every
 * complete family of old blocks that are all -1, lie above min_level and
 * whose parent stays within one level of its neighbours.  The state is
 * remapped on the device (copy, limited prolongation, restriction) into the
 * other buffer, which becomes current; the pattern is rebuilt.  flags_host
 * may be NULL (then the indicator chosen with foap4_mesh_set_indicator,
 * Lohner by default, computes them).  *changed (may be NULL)
 * is 1 if the mesh changed.  FOAP4_E_CAPACITY (mesh unchanged) if the new
 * mesh would exceed max_blocks. */
foap4_status foap4_regrid(foap4_mesh *mesh, const int8_t *flags_host, int32_t *changed);

/* ----------------------------------------------- learned refinement indicator
 * Not part of the paper's method: a small network that predicts the flags of
 * its gradient criterion (Sec. 3.3) from per-block features, with that
 * criterion kept as fallback.  Features, 16 per block, all computed on the
 * device from the current state with ghosts filled, with r0 = max over the
 * block's interior cells of |(rho(x+e_d) - rho(x-e_d)) / 2|_2 / rho(x) (norm
 * over the axes d, undivided central differences) and r1 the same for the
 * pressure p:
 *   f0 = log(1 + r0), f1 = log(1 + r1), f2 = level / max(max_level, 1),
 *   f(3+2k), f(4+2k) = f0, f1 of the neighbour across face k (order -x, +x,
 *   -y, +y, -z, +z; maximum over the finer blocks of a refined face; 0 in 2D
 *   for k >= 4), f15 = 0.
 * Network: 16 -> 64 (ReLU) -> 64 (ReLU) -> 3 logits of the classes -1, 0, +1.
 * Parameters, FP32, flat in this order (row-major matrices, input index
 * first): W1[16][64], b1[64], W2[64][64], b2[64], W3[64][3], b3[3].  The
 * three products run on the matrix cores with BF16 operands (weights,
 * inputs, activations and back-propagated errors rounded to nearest even)
 * and FP32 accumulation; biases stay FP32. */
#define FOAP4_MLP_NIN 16
#define FOAP4_MLP_NHID 64
#define FOAP4_MLP_NOUT 3
#define FOAP4_MLP_NPARAM 5443

/* Features of the current state: fills ghosts, then writes feat_dev
 * [n_blocks][16] FP32 and, if raw_dev is non-NULL, raw_dev[n_blocks][2] =
 * (r0, r1) in FP64 (evaluated in FP64 in the operation order of the
 * definition above, with v = m / rho and p = (gamma - 1)(E - m.v / 2)).
 * Device buffers owned by the caller; feat_dev 16-byte aligned.  Enqueue only. */
foap4_status foap4_block_features(foap4_mesh *mesh, float *feat_dev, double *raw_dev);

/* on != 0: every later foap4_step call also evaluates r0, r1 of the state at
 * the start of its last step, inside that step's first stage (the primitive
 * planes the stage stages in LDS give the central differences; FP32 states
 * in FP32), so that no separate pass over the state is needed at a regrid.
 * The captured values stay valid until the next step or regrid. */
foap4_status foap4_mesh_capture_features(foap4_mesh *mesh, int32_t on);

/* The 16 features (layout as foap4_block_features) assembled from the values
 * captured by the last foap4_step call, and (raw_dev non-NULL) the captured
 * r0, r1 [n_blocks][2].  They describe the state one step before the current
 * one.  FOAP4_E_ORDER if that call did not capture (capture off, or a step
 * or regrid came after it).  Enqueue only.  FOAP4_IND_MLP flags use them
 * whenever they are valid; then ghosts are filled and the criterion runs
 * only if some block falls back to it. */
foap4_status foap4_captured_features(foap4_mesh *mesh, float *feat_dev, double *raw_dev);

/* Chooses the indicator foap4_regrid uses when flags_host is NULL, and
 * attaches net (may be NULL for FOAP4_IND_LOHNER) for FOAP4_IND_MLP.  The
 * network is referenced, not copied: it must outlive the attachment, and its
 * work must be ordered with the mesh's stream by the caller. */
foap4_status foap4_mesh_set_indicator(foap4_mesh *mesh, foap4_indicator ind, const foap4_mlp *net);

/* Number of blocks of the last FOAP4_IND_MLP flag computation that fell back
 * to the Lohner flag. */
foap4_status foap4_indicator_fallbacks(const foap4_mesh *mesh, int64_t *n_fallback);

/* A network with no weights yet, working on hip_stream (a hipStream_t, NULL:
 * default stream).  Holds the FP32 master weights, FP64 Adam moments and the
 * training workspace in device memory. */
foap4_status foap4_mlp_create(void *hip_stream, foap4_mlp **out);
foap4_status foap4_mlp_destroy(foap4_mlp *net);

/* Copies n = FOAP4_MLP_NPARAM FP32 parameters from w_host (layout above),
 * resets the Adam moments and step count.  Synchronizes. */
foap4_status foap4_mlp_set_params(foap4_mlp *net, const float *w_host, int64_t n);

/* Copies the current FP32 parameters to w_host[n], n = FOAP4_MLP_NPARAM.
 * Synchronizes. */
foap4_status foap4_mlp_get_params(foap4_mlp *net, float *w_host, int64_t n);

/* Smallest largest-class probability at which the network's flag is used
 * (default 0.5; 0 never falls back). */
foap4_status foap4_mlp_set_threshold(foap4_mlp *net, float threshold);

/* Logits of n feature rows: feat_dev[n][16] -> logits_dev[n][3] (FP32,
 * device, caller-owned, feat_dev 16-byte aligned).  Enqueue only. */
foap4_status foap4_mlp_forward(foap4_mlp *net, const float *feat_dev, int64_t n, float *logits_dev);

/* Class-weighted cross-entropy sum_s w(c_s) CE_s / sum_s w(c_s) of n rows
 * with labels label_dev[n] in {-1, 0, +1} (class = label + 1, weights
 * class_w[3] on the host, each >= 0 with a positive total) and its gradient
 * with respect to the parameters, written to loss_host and grad_host
 * [FOAP4_MLP_NPARAM] (either may be NULL).  The sum over rows is
 * deterministic: per-workgroup partials reduced in a fixed order in FP64.
 * FOAP4_E_INVALID for a label outside {-1, 0, +1}.  Synchronizes. */
foap4_status foap4_mlp_loss_grad(foap4_mlp *net, const float *feat_dev, const int8_t *label_dev, int64_t n,
                                 const float *class_w, double *loss_host, float *grad_host);

/* iters full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning
 * rate lr) on the loss above, all on the device; loss_host[iters] (may be
 * NULL) receives the loss before each step.  Synchronizes once at the start
 * (label check) and once at the end. */
foap4_status foap4_mlp_train(foap4_mlp *net, const float *feat_dev, const int8_t *label_dev, int64_t n,
                             const float *class_w, int32_t iters, float lr, double *loss_host);

/* ------------------------------------------------------------------ batch
 * Many independent meshes of one precision advanced together: one
 * persistent launch per stage over the concatenated (mesh, block tile,
 * k-slab) work items of all meshes, one launch per ghost round, steps
 * captured once in a HIP graph and replayed.  Each mesh keeps its own dt.
 * The meshes must share ndim, precision, limiter, flux and whether gravity
 * is on (its value may differ); FOAP4_E_INVALID otherwise. */
foap4_status foap4_batch_create(foap4_mesh *const *meshes, int32_t n_meshes, foap4_batch **out);
foap4_status foap4_batch_destroy(foap4_batch *batch);

/* Work decomposition of the batched stage kernel: kslabs = 1, 2 or 4 k-slabs
 * per block tile (the LDS tile depth is N / kslabs planes), wg_stage1 and
 * wg_stage2 = workgroups per compute unit of the persistent grid of the
 * first and the second Heun stage (0: one workgroup per work item, no
 * persistence; the two stages differ in registers and traffic, so their
 * best grids differ), xcd_order = 0 for plain
 * striding of the work items over the workgroups, 1 to give each of the 8
 * XCDs a contiguous range of work items (Morton neighbours share an L2), 2 to
 * give each workgroup a contiguous chunk (a block and its Morton neighbours
 * run back to back on one CU), gather_halos = 1 to read same-level halo cells straight from the
 * neighbouring blocks instead of copying them into ghost cells first (the
 * results are identical; round R1 then runs only the SRL copies whose ghosts
 * a coarse-to-fine prolongation reads: the records with a side that is the
 * coarse block of a C2F record).  Defaults: 1, 0, 0, 1, 1.
 * FOAP4_E_INVALID outside those ranges (workgroups per CU: 0 .. 64). */
foap4_status foap4_batch_set_config(foap4_batch *batch, int32_t kslabs, int32_t wg_stage1,
                                    int32_t wg_stage2, int32_t xcd_order, int32_t gather_halos);

/* Times the candidate configurations (kslabs x workgroups per CU x
 * xcd_order, each stage timed on its own) on the batch itself and keeps, per
 * (kslabs, xcd_order), the fastest grid of each stage, then the fastest
 * whole step; results are cached in the JSON file cache_path (may be NULL)
 * keyed by GPU architecture, precision and the batch's block-size mix.  The
 * meshes' states are restored afterwards.  Writes the chosen {kslabs,
 * wg_stage1, wg_stage2, xcd_order} to cfg_out[4] (may be NULL). */
foap4_status foap4_batch_autotune(foap4_batch *batch, const char *cache_path, int32_t *cfg_out);
/* (Phase timing and the autotuner time Heun's two stages: FOAP4_E_INVALID for
 * a batch with another integrator, whose generic sub-steps use the stage-2
 * grid of foap4_batch_set_config.) */

/* Advances every mesh of the batch by n_steps Heun steps (enqueue only). */
foap4_status foap4_batch_step(foap4_batch *batch, int32_t n_steps);

/* Runs n_steps steps of the batch with the same launches as the captured
 * graph but launched one by one, with HIP events recorded on the batch's
 * stream around every launch, and writes average durations in ms to
 * out_ms[8]: [0] ghost round R1 per launch, [1] ghost round R2 per launch,
 * [2] stage kernel per launch (both stages), [3] flux fixing per step,
 * [4] dt finalisation per step, [5] whole step, [6] stage 1, [7] stage 2.
 * Synchronizes.  Advances the meshes like foap4_batch_step. */
foap4_status foap4_batch_phase_times(foap4_batch *batch, int32_t n_steps, double *out_ms);

/* Last error message of a mesh (NULL: of the most recent failing call). */
const char *foap4_last_error(const foap4_mesh *mesh);

#ifdef __cplusplus
}
#endif
#endif /* FOAP4_H */
