/*
 * lfltsmc.h -- C ABI of an MI355X (gfx950) library for multilevel Monte Carlo
 * with stabilized leapfrog local time-stepping (LF-LTS) for the wave equation
 * with a random coefficient (Grote, Michel, Nobile: "Uncertainty
 * quantification by MLMC and local time-stepping for wave propagation").
 *
 * Model (Sec. 2.1): u_tt - div(c^2 grad u) = 0 in D, u = 0 on the boundary,
 * u(0) = u0, u_t(0) = 0, with c = exp(g) and g piecewise constant on a grid of
 * coefficient blocks.  Space (Sec. 3.1): continuous P1 elements with mass
 * lumping on rectilinear grids whose cells are split into two triangles along
 * the diagonal (x_a, y_b)-(x_a+1, y_b+1).  Time (Sec. 3.3, Algorithm 2): one
 * coarse leapfrog step dt per step and p local substeps of size dt/p on the
 * DOFs selected by the diagonal projector P.  Estimator (Sec. 2.2): the
 * coupled differences Delta Q_l = Q_l - Q_{l-1} on a common sample, their
 * per-level mean and unbiased variance, and Algorithm 1 for N_l and L.
 *
 * Conventions shared by every entry point:
 *  - Every function returns lts_status: LTS_OK (0) or a negative code.  No
 *    function throws, aborts or exits.  After an error, lts_last_error(ctx)
 *    describes it (ctx-owned string, valid until the next call on ctx).
 *  - Arguments are validated before any time step is launched (host arrays
 *    on the host; device sample arrays by a checking gather kernel, see
 *    lts_samples); an LTS_ERR_ARG return leaves every output untouched.
 *  - Caller arrays are only read during the call (meshes are copied in).
 *    Output arrays are caller-allocated.  The context owns all device
 *    workspace (level data, states, checkpoints, captured graphs).
 *  - ptr_kind LTS_PTR_HOST: sample arrays and outputs are host memory; the
 *    call returns after the results are in place.  LTS_PTR_DEVICE: they are
 *    device pointers on the context's device; work is ordered on the context
 *    stream and the call returns once the outputs are written (the library
 *    synchronizes its stream before returning in both cases).
 *  - A context is not thread-safe; distinct contexts are independent.
 *  - Floating point is IEEE binary64 unless a precision flag says otherwise.
 */
#ifndef LFLTSMC_H
#define LFLTSMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lts_status;
typedef struct lts_ctx_s* lts_ctx;

enum {
  LTS_OK = 0,
  LTS_ERR_ARG = -1,       /* invalid argument (sizes, ids, ranges, pointers) */
  LTS_ERR_HIP = -2,       /* a HIP runtime call failed; text in lts_last_error */
  LTS_ERR_OOM = -3,       /* device allocation failed */
  LTS_ERR_UNSTABLE = -4,  /* at least one sample produced a non-finite QoI;
                             those QoIs are NaN, all others are valid */
  LTS_ERR_STATE = -5      /* call not valid in the current context state */
};

enum { LTS_FP64 = 0, LTS_FP32_STEP = 1 };   /* time-stepping precision; QoI sums stay FP64 */
enum { LTS_PTR_HOST = 0, LTS_PTR_DEVICE = 1 };

/* Node flag bits returned by lts_level_arrays (one byte per grid node). */
enum { LTS_NODE_DOF = 1, LTS_NODE_P = 2, LTS_NODE_FPLUS = 4 };

/* ------------------------------------------------------------------------ */
/* Context                                                                   */
/* ------------------------------------------------------------------------ */

/* Create a context on HIP device `hip_device`.  `hip_stream` is a hipStream_t
 * (cast to void*) that all device work is ordered on; NULL makes the context
 * create and own a stream of default priority.  *out receives the handle.
 * Errors: LTS_ERR_ARG (out NULL, no such device), LTS_ERR_HIP. */
lts_status lts_create(lts_ctx* out, int32_t hip_device, void* hip_stream);

/* Release every device resource of ctx (ctx may be NULL). */
lts_status lts_destroy(lts_ctx ctx);

/* Text of the last error on ctx ("" if none).  Never NULL. */
const char* lts_last_error(lts_ctx ctx);

/* ------------------------------------------------------------------------ */
/* Levels (Sec. 3.2-3.5: the mesh hierarchy with local refinement)           */
/* ------------------------------------------------------------------------ */

/* One level's mesh.  Cells are [x_a, x_a+1] x [y_b, y_b+1], a = 0..nx_cells-1,
 * b = 0..ny_cells-1, flat cell index b*nx_cells + a; nodes (a, b), a =
 * 0..nx_cells, flat node index b*(nx_cells+1) + a.  Every active cell is two
 * P1 triangles.  A node is a DOF iff its four incident cells exist and are
 * active (homogeneous Dirichlet data everywhere else).  P (Sec. 3.3) marks the
 * DOFs that are vertices of a fine cell.  All arrays are caller-owned and
 * copied by lts_add_level. */
typedef struct {
  int32_t nx_cells, ny_cells;     /* >= 2 each */
  const double* x;                /* [nx_cells+1], strictly increasing */
  const double* y;                /* [ny_cells+1], strictly increasing */
  const uint8_t* cell_active;     /* [ny_cells*nx_cells], 1 = cell in D; NULL = all */
  const int32_t* cell_block;      /* [ny_cells*nx_cells], coefficient block in [0, n_blocks) */
  const uint8_t* cell_fine;       /* [ny_cells*nx_cells], 1 = cell in D_fine */
  const uint8_t* cell_qoi;        /* [ny_cells*nx_cells], 1 = cell in the QoI region */
  int32_t n_blocks;               /* 1..255 */
  double h;                       /* base spacing; the step rule dt = cfl*h/max c uses it */
  int32_t p;                      /* local substeps, 1..256 */
  double nu;                      /* stabilization, 0 <= nu <= 1 (nu = 0: original LF-LTS) */
} lts_grid_desc;

/* Copy a level into ctx (host and device) and return its id (0, 1, ... in
 * call order).  Errors: LTS_ERR_ARG (sizes, ordering, ids), LTS_ERR_OOM. */
lts_status lts_add_level(lts_ctx ctx, const lts_grid_desc* desc, int32_t* level_id_out);

enum { LTS_RULE_BOX = 0, LTS_RULE_GRADED_L = 1, LTS_RULE_LF = 0x100 };

/* Generated rectilinear levels (exact dyadic node coordinates).
 *  LTS_RULE_BOX: square [lo,hi]^2, n_base uniform cells per axis; per axis,
 *    every coarse interval meeting the open interval (box_lo, box_hi) is split
 *    into `ref` equal parts (Sec. 3.2: a fixed refined region).
 *  LTS_RULE_GRADED_L: square [lo,hi]^2 minus the cells with midpoint x > 0,
 *    y < 0 (an L-shape with reentrant corner at the origin); per axis the two
 *    cells next to 0 are replaced by the nodes +-h 2^-j, j = 1..layers
 *    (Sec. 3.5: grading toward a reentrant corner).
 * Both: fine cells have a leg shorter than h/2; blocks are an nbx x nby grid
 * over [lo,hi]^2 assigned by cell midpoint (block = by*nbx + bx); QoI cells
 * have their midpoint in the closed box [qx_lo,qx_hi] x [qy_lo,qy_hi];
 * p = 0 selects p = ceil(h / smallest cell leg).
 * kind | LTS_RULE_LF: the standard leapfrog twin of that level (the baseline
 * the paper compares LF-LTS with, Sec. 4): the same grid, blocks and QoI
 * cells with no fine cells (P empty) and p = 1, so every step is one plain
 * leapfrog step over all DOFs, and nominal spacing h/p (p of the LTS level),
 * so that samples drawn for it step at dt/p on every element. */
/* Fine set of a graded level (fine_rule of lts_rect_rule; Sec. 3.5).
 *  LTS_FINE_HALF_H: cells with a leg shorter than h/2, step spacing h (the
 *    workloads' rule; the only one for LTS_RULE_BOX).
 *  LTS_FINE_TIERS: the fine_tiers = q smallest tiers, q in 0..layers.  Tier k
 *    holds the cells whose shorter leg is h 2^(k-1-layers); the coarse step
 *    uses the spacing H = 2 x (shortest coarse leg), so that the coarse time
 *    step follows the smallest coarse elements, and p = ceil(H / h_min)
 *    (p = 1 when q = 0: plain leapfrog).  q = layers - 1 is LTS_FINE_HALF_H.
 *  LTS_FINE_QOPT: q chosen to minimise the DOF-update rate
 *    ((N - |P_q|) + p_q |P_q|) / H_q, the LTS cost per unit time (the smallest
 *    q on a tie), among the q with p_q <= p_max when p_max > 0 (a fine-tile
 *    region holds the F+ nodes within p of its tile, so very large p can leave
 *    a level that no tile shape fits); fine_tiers is ignored. */
enum { LTS_FINE_HALF_H = 0, LTS_FINE_TIERS = 1, LTS_FINE_QOPT = 2 };

typedef struct {
  int32_t kind;
  double lo, hi;
  int32_t n_base;
  double box_lo, box_hi;
  int32_t ref;
  int32_t layers;
  int32_t nbx, nby;
  double qx_lo, qx_hi, qy_lo, qy_hi;
  int32_t p;                      /* > 0 overrides the p of the rule */
  double nu;
  int32_t fine_rule;              /* LTS_FINE_* (0: LTS_FINE_HALF_H) */
  int32_t fine_tiers;             /* q for LTS_FINE_TIERS */
  int32_t p_max;                  /* LTS_FINE_QOPT: largest p allowed (0: none) */
} lts_rect_rule;

/* Build the level described by `rule` on the host, then lts_add_level it.
 * Errors: LTS_ERR_ARG, LTS_ERR_OOM. */
lts_status lts_build_rect_level(lts_ctx ctx, const lts_rect_rule* rule, int32_t* level_id_out);

typedef struct {
  int32_t nx_nodes, ny_nodes;     /* nx_cells+1, ny_cells+1 */
  int32_t n_dof, n_P, n_Fplus;    /* DOFs, |P|, |F+| with F+ = P and its stiffness neighbours */
  int32_t p, n_blocks;
  double h, nu;
  double delta, omega;            /* stabilized Chebyshev constants (Sec. 3.3) */
  int32_t tile_x, tile_y;         /* fine-tile shape in use (grid nodes; 0, 0: adaptive) */
  int32_t tile_rect, tuned;       /* rectangular LDS region (2: coarse and fine in one launch);
                                     chosen by the autotuner */
  double halo_ratio;              /* nodes of all fine-tile regions / |F+| */
  double tuned_ms;                /* measured step time per sample of the tuned tiling */
} lts_level_info;

/* Sizes and constants of a level.  Errors: LTS_ERR_ARG. */
lts_status lts_level_info_get(lts_ctx ctx, int32_t level, lts_level_info* out);

/* Host copies of a level's derived arrays (any pointer may be NULL):
 * x [nx_nodes], y [ny_nodes], node_flags [ny_nodes*nx_nodes] (LTS_NODE_*
 * bits), mass [ny_nodes*nx_nodes] (lumped mass, every node incl. boundary:
 * sum over incident triangles of |T|/3), qoi_w [ny_nodes*nx_nodes] (QoI
 * weights: the same sum restricted to QoI cells, 0 on non-DOFs),
 * cell_block [ny_cells*nx_cells] (-1 for inactive cells).  Errors: LTS_ERR_ARG. */
lts_status lts_level_arrays(lts_ctx ctx, int32_t level, double* x, double* y, uint8_t* node_flags,
                            double* mass, double* qoi_w, int32_t* cell_block);

/* Host-only variant of lts_build_rect_level + lts_level_arrays: builds the
 * level of `rule` without any device and copies out its info (required) and
 * arrays (each may be NULL; sizes as in lts_level_arrays, so a first call with
 * NULL arrays returns the sizes).  Errors: LTS_ERR_ARG. */
lts_status lts_rect_level_host(const lts_rect_rule* rule, lts_level_info* info, double* x, double* y,
                               uint8_t* node_flags, double* mass, double* qoi_w, int32_t* cell_block);

typedef struct {
  int32_t n_fine, n_coarse;       /* fine-tile and coarse-item workgroups per sample */
  int32_t tile_x, tile_y, tile_rect;
  int32_t max_region;             /* nodes (rect mode: lanes) of the largest fine-tile region */
  int32_t regions_exact;          /* 1: every region holds all F+ nodes within Manhattan
                                     distance p of its tile (compact mode: exactly those) */
  int32_t threads;                /* threads of a fine workgroup: 1024 in rect mode; in compact
                                     mode the fewest of 256, 512, 1024 whose lanes (4 nodes
                                     each) hold the largest region */
  double halo_ratio;              /* nodes of all fine-tile regions / |F+| */
} lts_tiling_info;

/* Host only (no device): the fine-tile tiling that lts_set_tiling(level,
 * tile_x, tile_y, rect) picks for the level lts_build_rect_level builds from
 * `rule` (tile_x = tile_y = 0, rect = 0: the adaptive tiling), and which tile
 * writes each node back.  A node at distance d from a tile reaches it after d
 * substeps, so a region must hold the F+ nodes within distance p of its tile
 * (Algorithm 2 runs p substeps on F+ only).  info is required; owner may be
 * NULL or hold [ny_nodes*nx_nodes]: the index of the fine tile that writes the
 * node back, -1 where no tile does, -2 where more than one would.  Errors:
 * LTS_ERR_ARG (bad rule, sizes, or a tiling that does not fit). */
lts_status lts_tiling_host(const lts_rect_rule* rule, int32_t tile_x, int32_t tile_y, int32_t rect,
                           lts_tiling_info* info, int32_t* owner);

/* ------------------------------------------------------------------------ */
/* Levels given as triangulations (Sec. 3.1: conforming P1 elements with     */
/* mass lumping on a triangle mesh)                                          */
/* ------------------------------------------------------------------------ */

/* One level as a triangle mesh.  Element T contributes kappa_T |T| G_T^T G_T
 * to the stiffness (G_T: gradients of the barycentric coordinates) and |T|/3
 * to the lumped mass of each vertex; kappa_T = kappa of block tri_block[T].
 * A node is a DOF iff it is not Dirichlet; every DOF must be a vertex of a
 * triangle.  P (Sec. 3.3) marks the DOFs that are vertices of a fine element,
 * F+ the DOFs of P and those coupled to P by a nonzero stiffness entry.  All
 * arrays are caller-owned and copied by lts_add_mesh. */
typedef struct {
  int32_t n_nodes, n_tris;
  int32_t n_blocks;               /* 1..255 */
  const double* xy;               /* [n_nodes][2], finite */
  const int32_t* tri;             /* [n_tris][3] node ids, counter-clockwise (positive area);
                                     every edge in at most two triangles */
  const uint8_t* dirichlet;       /* [n_nodes]: 1 = homogeneous Dirichlet node (u = 0); NULL = none */
  const int32_t* tri_block;       /* [n_tris] in [0, n_blocks) */
  const uint8_t* tri_fine;        /* [n_tris]: 1 = element in D_fine; NULL = none */
  const double* qoi_w;            /* [n_nodes]: Q = sum over DOFs of qoi_w[i] u_i(T) (the entries of
                                     Dirichlet nodes are not used); NULL = all 0 */
  double h;                       /* coarse spacing: the step rule dt = cfl h / max c uses it */
  int32_t p;                      /* local substeps, 1..64 */
  double nu;                      /* stabilization, 0 <= nu <= 1 */
} lts_mesh_desc;

/* Sizes of a triangle-mesh level.  A fine tile's region holds the F+ DOFs
 * within graph distance p of its DOFs (at most LTS_MESH_REGION_CAP; an F+ DOF
 * may have at most LTS_MESH_MAX_DEGREE stiffness neighbours). */
#define LTS_MESH_REGION_CAP 2048
#define LTS_MESH_MAX_DEGREE 12
typedef struct {
  int32_t n_nodes, n_tris, n_dof, n_P, n_Fplus;
  int32_t n_edges;                /* directed stiffness couplings of the DOF rows (Dirichlet neighbours incl.) */
  int32_t max_degree;             /* largest number of neighbours of an F+ DOF */
  int32_t n_tiles, max_region;    /* fine tiles and the largest region */
  int32_t p, n_blocks;
  double h, nu, delta, omega;
  double halo_ratio;              /* region nodes of all tiles / |F+| */
} lts_mesh_info;

/* Copy a triangle-mesh level into ctx and return its id (0, 1, ... in call
 * order; mesh ids are separate from the ids of lts_add_level).  Errors:
 * LTS_ERR_ARG (sizes, orientation, indices, a non-manifold edge, a DOF in no
 * triangle, an F+ DOF with more than LTS_MESH_MAX_DEGREE neighbours, a region
 * that exceeds LTS_MESH_REGION_CAP even for a one-DOF tile), LTS_ERR_OOM. */
lts_status lts_add_mesh(lts_ctx ctx, const lts_mesh_desc* desc, int32_t* mesh_id_out);

/* Sizes of mesh `mesh`.  Errors: LTS_ERR_ARG. */
lts_status lts_mesh_info_get(lts_ctx ctx, int32_t mesh, lts_mesh_info* out);

/* Host only: validate `desc` and build the level as lts_add_mesh does; info
 * (required) and, per node (each may be NULL), node_flags [n_nodes]
 * (LTS_NODE_* bits) and mass [n_nodes] (lumped mass, every node).
 * Errors: as lts_add_mesh. */
lts_status lts_mesh_host(const lts_mesh_desc* desc, lts_mesh_info* info, uint8_t* node_flags, double* mass);

/* Stabilized Chebyshev constants of Sec. 3.3 for (p, nu): delta = 1 + nu/p^2,
 * omega = 2 T_p'(delta)/T_p(delta); beta[k] = T_{k-1}(delta)/T_{k+1}(delta) and
 * beta_half[k] = T_k(delta)/T_{k+1}(delta) for k = 1..p-1 (arrays of length p,
 * index 0 set to 0; may be NULL).  Also the per-step coefficients for a step
 * dt (coef may be NULL, length p+1): coef[0] = a_p (after the p substeps a DOF
 * outside F+ holds u + a_p w, a_p = -dt^2/2 up to rounding), coef[1] =
 * 1/2 (dt/p)^2 2p^2/(omega delta), coef[1+m] = (dt/p)^2 2p^2/omega beta_{m+1/2}.
 * Errors: LTS_ERR_ARG (p outside 1..256, nu outside [0,1]). */
lts_status lts_cheb_constants(int32_t p, double nu, double dt, double* delta, double* omega,
                              double* beta, double* beta_half, double* coef);

/* ------------------------------------------------------------------------ */
/* Random samples (host; counter-based, reproducible per (seed, level, i))   */
/* ------------------------------------------------------------------------ */

/* Sample law: g_b ~ N(0, sigma^2) i.i.d. on n_blocks blocks; pulse centre
 * uniform in [px_lo,px_hi] x [py_lo,py_hi]; u0 = exp(-|x-x0|^2/width^2);
 * n_steps = ceil(T max_b exp(g_b) / (cfl h)), dt = T/n_steps on a mesh of
 * base spacing h. */
typedef struct {
  int32_t n_blocks;               /* even, 2..255 */
  double sigma;
  double px_lo, px_hi, py_lo, py_hi;
  double width;
  double T;
  double cfl;
} lts_sample_rule;

/* Draw samples i = first_index .. first_index+n-1 of MLMC level
 * `sample_level` (Sec. 2.2: each level has its own independent samples; the
 * fine and coarse solve of one difference share them).  Stream: Philox4x64-10
 * (Salmon et al., SC'11) with key (seed, 0) and counter (j, i, sample_level,
 * purpose), purpose 0 = field, 1 = pulse; uniforms ((x >> 12) + 0.5) 2^-52;
 * Box-Muller on consecutive uniforms.  Steps and dt are for a mesh of base
 * spacing h_mesh.  Outputs (host, any may be NULL): g [n][n_blocks],
 * kappa [n][n_blocks] = exp(2 g), x0 [n][2], n_steps [n], dt [n].
 * Errors: LTS_ERR_ARG. */
lts_status lts_gen_samples(uint64_t seed, int32_t sample_level, int64_t first_index, int32_t n,
                           const lts_sample_rule* rule, double h_mesh, double* g_out,
                           double* kappa_out, double* x0_out, int32_t* n_steps_out,
                           double* dt_out);

/* Raw Philox4x64-10 block (for known-answer tests): out[4] = Philox(ctr[4], key[2]). */
lts_status lts_philox4x64_10(const uint64_t* ctr, const uint64_t* key, uint64_t* out);

/* ------------------------------------------------------------------------ */
/* Forward solves (Algorithm 2 per sample, QoI at T)                         */
/* ------------------------------------------------------------------------ */

/* One batch of samples.  The coefficient is given either as kappa = c^2 or,
 * with kappa NULL, as g = log c (Sec. 2.1: c = exp(g) with g piecewise
 * constant on the blocks), in which case the library forms kappa = exp(2 g)
 * on the device.
 * Device arrays (LTS_PTR_DEVICE) are read on the device: kappa or g and x0 are
 * gathered into the library's sorted order by a kernel that also checks them
 * (an invalid value gives LTS_ERR_ARG before any time step is launched, the
 * outputs untouched); only n_steps and dt are copied to the host, because the
 * launch schedule (which samples still run at each step) and the per-sample
 * step coefficients (a_p from an extended-precision recurrence) are planned
 * there.  Device outputs are written by kernels on the context stream.  The
 * inputs must be complete when the call is made: work on another stream that
 * writes them must have finished or be ordered before the context stream
 * (the Python binding waits for the caller's current torch stream). */
typedef struct {
  int32_t n;                      /* number of samples, >= 0 */
  int32_t ptr_kind;               /* LTS_PTR_HOST or LTS_PTR_DEVICE for the arrays below */
  const double* kappa;            /* [n][n_blocks of the level], finite and > 0; or NULL (then g) */
  const double* x0;               /* [n][2] pulse centres, finite */
  const int32_t* n_steps;         /* [n], >= 1 */
  const double* dt;               /* [n], finite and > 0 */
  double width;                   /* pulse width, > 0 */
  const double* g;                /* [n][n_blocks], finite; read only when kappa is NULL */
} lts_samples;

/* Solve every sample on `level` from t = 0 to n_steps*dt with stabilized
 * LF-LTS (Algorithm 2; start-up u_1 = q_1(u_0) since u_t(0) = 0) and write
 * Q[s] = sum_i qoi_w[i] u_i(T) (same ptr_kind as the samples).
 * precision: LTS_FP64, or LTS_FP32_STEP: states, increments, the LDS copies
 * and the stencil / recurrence arithmetic in binary32 (edge coefficients and
 * Chebyshev scalars are formed in binary64 and rounded once); the QoI sum is
 * accumulated in binary64 in both cases.
 * Errors: LTS_ERR_ARG, LTS_ERR_OOM, LTS_ERR_HIP, LTS_ERR_UNSTABLE. */
lts_status lts_forward(lts_ctx ctx, int32_t level, const lts_samples* samples, int32_t precision,
                       double* Q_out);

/* The same solve with one kernel launch per sample and step (no batching of
 * samples), used as the unbatched reference form.  Same contract. */
lts_status lts_forward_plain(lts_ctx ctx, int32_t level, const lts_samples* samples,
                             int32_t precision, double* Q_out);

/* Size in bytes of the per-device array that lts_forward_noalloc works in. */
#define LTS_NOALLOC_SCRATCH_BYTES (64ULL << 20)

/* For callers that cannot allocate device memory during a solve (serving
 * loops, harnesses that forbid hipMalloc): lts_forward (batched, FP64 or
 * LTS_FP32_STEP) with every piece of device scratch -- the sorted per-sample
 * tables, a staging flag and the two time levels of the state -- in one fixed
 * array of LTS_NOALLOC_SCRATCH_BYTES bytes per GPU, which the library holds from
 * the first lts_create on that GPU until the process ends.  The call makes no
 * hipMalloc or hipFree (the level and its tiling must exist already:
 * lts_add_level and lts_set_tiling / lts_autotune allocate).  The batch must fit:
 * about 2 n (nx_nodes rounded up to 8) ny_nodes values of 8 bytes (4 under
 * LTS_FP32_STEP) plus n (n_blocks + p + 6) * 8 bytes; a larger batch returns
 * LTS_ERR_ARG naming the bytes it needs, before anything is read.  All calls
 * on one GPU, from any context or thread, share that GPU's array and leave
 * their contents in it: calls that overlap in time on one GPU race.  No
 * timing events are recorded.  Otherwise the contract of lts_forward, with the
 * same results bit for bit.  Errors as lts_forward; LTS_ERR_STATE if the
 * array's address could not be taken on this device. */
lts_status lts_forward_noalloc(lts_ctx ctx, int32_t level, const lts_samples* samples, int32_t precision,
                               double* Q_out);

/* Coupled difference for MLMC level l >= 1 (Sec. 2.2): the same samples
 * (kappa, x0) solved on level_fine and level_coarse, each with its own
 * n_steps/dt.  Writes Qf, Qc and dQ = Qf - Qc (any may be NULL; same
 * ptr_kind).  Errors as lts_forward. */
lts_status lts_forward_coupled(lts_ctx ctx, int32_t level_fine, int32_t level_coarse,
                               const lts_samples* fine, const lts_samples* coarse,
                               int32_t precision, double* Qf_out, double* Qc_out, double* dQ_out);

/* Algorithm 2 for every sample on mesh `mesh` (as lts_forward: pulse initial
 * state exp(-|x - x0|^2 / width^2) at the DOFs, zero velocity, start-up step,
 * n_steps coarse steps of dt; Q = sum qoi_w u(T)).  FP64 only (precision must
 * be LTS_FP64).  Errors as lts_forward. */
lts_status lts_mesh_forward(lts_ctx ctx, int32_t mesh, const lts_samples* samples, int32_t precision,
                            double* Q_out);

/* Coupled difference on two meshes (Sec. 2.2), as lts_forward_coupled. */
lts_status lts_mesh_forward_coupled(lts_ctx ctx, int32_t mesh_fine, int32_t mesh_coarse,
                                    const lts_samples* fine, const lts_samples* coarse, int32_t precision,
                                    double* Qf_out, double* Qc_out, double* dQ_out);

/* ------------------------------------------------------------------------ */
/* Multi-level local time stepping (Sec. 3.5, closing remark)                */
/* ------------------------------------------------------------------------ */

/* Tiers of ever smaller elements inside D_fine, each advancing with its own
 * step: Algorithm 2 nested once per tier (the paper names the multi-level
 * method without stating it; this nesting is the library's reading).  Tier j
 * (1..n_tiers) has the fine set S_j = the cells of tier >= j (S_1 = D_fine),
 * P_j = the DOFs that are vertices of a cell of S_j, and the ratio p_j.  Tier j
 * covers a time sigma_j (sigma_1 = dt) with the p_j stages of Algorithm 2's
 * stabilized recurrence for (p_j, nu), in increment form with the force
 * Phi_m = F + A P_j e_m; each stage's leapfrog half step from rest, of time
 * sigma_j+1 = sigma_j (2 / (omega_j delta_j))^1/2 (= sigma_j / p_j when nu = 0),
 * is taken by tier j+1 with the force Phi_m as its F; the innermost tier takes
 * it directly.  The step is u_n+1 = 2 u_n - u_n-1 + 2 e (e: tier 1's increment
 * for F = A u_n), the start-up u_1 = u_0 + e.  One tier with p_1 = p is
 * Algorithm 2.
 * cell_tier: [ny_cells*nx_cells], 0 for a coarse or inactive cell, else the
 * deepest tier (1..n_tiers) whose set holds the cell; it must be >= 1 exactly on
 * the active fine cells.  NULL selects the halving rule: an active fine cell
 * has tier 1 + #{j in 2..n_tiers : shorter leg < h 2^-j} (on the graded
 * L-shape with p_j = 2, every tier then steps at the coarse cells' ratio of
 * step to leg). */
#define LTS_MLTS_MAX_TIERS 5
#define LTS_MLTS_MAX_P 16
typedef struct {
  int32_t n_tiers;                        /* 1..LTS_MLTS_MAX_TIERS */
  int32_t p[LTS_MLTS_MAX_TIERS];          /* p_1 .. p_n_tiers, each 1..LTS_MLTS_MAX_P */
  const uint8_t* cell_tier;               /* caller-owned, copied; or NULL */
  int32_t max_region;                     /* largest fine-tile region: 512, 1024 or 2048 nodes (workgroups
                                             of 256, 512 or 1024 threads); 0 selects 2048 */
} lts_mlts_desc;

typedef struct {
  int32_t n_tiers;
  int32_t p[LTS_MLTS_MAX_TIERS];
  int32_t n_P[LTS_MLTS_MAX_TIERS];        /* |P_j| */
  int32_t phases;                         /* exchange phases per step: sum_j (p_1 .. p_j-1)(p_j - 1),
                                             also the radius of the fine tiles' regions */
  int32_t n_tiles, max_region, threads;   /* the tiling of the MLTS step (regions of F+ nodes within
                                             Manhattan distance `phases`, two per lane) */
  double halo_ratio;                      /* region nodes of all tiles / |F+| */
  double updates_per_step;                /* DOF updates of one step of one sample:
                                             (N - |P_1|) + sum_j (p_1 .. p_j)(|P_j| - |P_j+1|) */
} lts_mlts_info;

/* Attach tiers to rectilinear level `level` (replacing earlier ones) and build
 * the tiling of the MLTS step.  Errors: LTS_ERR_ARG (n_tiers or p out of
 * range, a cell_tier value beyond n_tiers or inconsistent with the fine cells,
 * a region beyond 2048 nodes), LTS_ERR_OOM. */
lts_status lts_set_mlts(lts_ctx ctx, int32_t level, const lts_mlts_desc* desc);

/* Sizes of the tiers attached to `level`.  Errors: LTS_ERR_ARG (no such level),
 * LTS_ERR_STATE (no tiers attached). */
lts_status lts_mlts_info_get(lts_ctx ctx, int32_t level, lts_mlts_info* out);

/* Host only: the tiers lts_set_mlts would attach to the level of `rule`; info
 * (required) and node_tier [ny_nodes*nx_nodes] (may be NULL): the largest j
 * with the node in P_j, 0 off P_1.  Errors: as lts_set_mlts. */
lts_status lts_mlts_host(const lts_rect_rule* rule, const lts_mlts_desc* desc, lts_mlts_info* info,
                         uint8_t* node_tier);

/* Solve every sample on `level` with its tiers (contract of lts_forward: pulse
 * initial state, n_steps steps of dt, Q = sum qoi_w u(T)).  precision: LTS_FP64,
 * or LTS_FP32_STEP (states and stepping in FP32, the QoI summed in FP64).
 * Errors as lts_forward; LTS_ERR_STATE if no tiers are attached. */
lts_status lts_mlts_forward(lts_ctx ctx, int32_t level, const lts_samples* samples, int32_t precision,
                            double* Q_out);

/* ------------------------------------------------------------------------ */
/* Batched form: many (level, samples) jobs advanced together                */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t level;
  lts_samples samples;            /* all jobs of one call use the same ptr_kind */
  int32_t q_offset;               /* Q of sample s of this job goes to Q_out[q_offset + s] */
} lts_job;

enum { LTS_BATCH_GRAPH = 1,      /* capture the step loop into HIP graphs and replay */
       LTS_BATCH_FP32 = 2,        /* FP32 stepping as LTS_FP32_STEP; QoI sums in FP64 */
       LTS_BATCH_PERSIST = 4,     /* persistent form (below); excludes LTS_BATCH_GRAPH */
       LTS_BATCH_SB1 = 8,         /* persistent form: S_b capped at 1 */
       LTS_BATCH_SB2 = 16,        /* persistent form: S_b capped at 2 (neither: at 4) */
       LTS_BATCH_SB_MASK = 24,
       LTS_BATCH_AUTO = 32,       /* choose the form by measurement (below) */
       LTS_BATCH_MLTS = 64 };     /* multi-level LTS on every job (below) */

/* Advance all jobs of all levels together (the MLMC cost sum_l N_l C_l of
 * Sec. 2.2 spread over one device): uneven mesh sizes and step counts share
 * the device.  Fine-tile shapes come from the context's autotuner (tuned once
 * per level shape and cached).  FP64 unless LTS_BATCH_FP32.  Forms:
 *  - default: one set of step launches per coarse step, each advancing every
 *    job that still has steps left (LTS_BATCH_GRAPH: the launch sequence
 *    captured once per job-list shape into a HIP graph and replayed);
 *  - LTS_BATCH_PERSIST: one cooperative launch (one workgroup per CU) runs
 *    all steps of all jobs, with a device-wide barrier after each step; a
 *    workgroup runs a rect-mode fine tile, four coarse items, or S_b compact
 *    tiles of one tile position for S_b consecutive samples side by side
 *    (S_b = 1, 2 or 4: the largest whose tiles of 1024 / S_b threads hold the
 *    level's regions, capped by LTS_BATCH_SB1 / LTS_BATCH_SB2).  A barrier
 *    wait is bounded (lts_set_barrier_timeout): on expiry every workgroup
 *    leaves and the call fails with LTS_ERR_STATE.  Needs cooperative launch.
 *  - LTS_BATCH_AUTO: time the first steps of this job list (at most 48) in
 *    the graph form and the persistent form with S_b caps 4, 2 and 1, and run
 *    the whole batch in the fastest (the choice is cached per job-list shape;
 *    lts_get_timing reports it).  Excludes the other form flags.
 *  - LTS_BATCH_MLTS: every job is solved by multi-level LTS with its level's
 *    tiers (lts_set_mlts; LTS_ERR_STATE for a level without), the coarse DOFs
 *    and the fine tiles of all jobs in shared launches per step (with
 *    LTS_BATCH_GRAPH captured and replayed); QoIs bit-identical to
 *    lts_mlts_forward in the same precision (FP32 stepping with
 *    LTS_BATCH_FP32); excludes LTS_BATCH_PERSIST and LTS_BATCH_AUTO.
 * Every form gives bit-identical QoIs.  Errors as lts_forward. */
lts_status lts_batch_run(lts_ctx ctx, const lts_job* jobs, int32_t n_jobs, int32_t flags,
                         double* Q_out);

/* Autotuner: time the candidate fine-tile shapes of `level` on a synthetic
 * batch and keep the fastest for all later solves on the level (the choice is
 * cached per level shape for the life of the process).  lts_batch_run tunes
 * levels that are not tuned yet.  Errors: LTS_ERR_ARG, LTS_ERR_HIP. */
lts_status lts_autotune(lts_ctx ctx, int32_t level);

/* Pin the fine-tile shape of `level` to tile_x x tile_y grid nodes in rect
 * mode (rect = 1: each region handled as a zero-padded rectangle of up to
 * 64 x 64 nodes, one lane per column, state in registers) or
 * compact mode (rect = 0: the region's F+ nodes compacted with neighbour
 * indices), with the tile-grid origin chosen to minimise region overhead.
 * tile_x = tile_y = 0 with rect = 0 selects the adaptive compact tiling: the
 * F+ set is bisected recursively until each part's region fits a workgroup
 * (long tiles along thin bands of F+).  rect = 2: rect mode with the coarse
 * items and the fine tiles of a step in one launch (the autotuner times this
 * form for its rect-mode winner; lts_level_info reports tile_rect = 2 then).
 * Later solves use it and lts_batch_run does not re-tune the level (a later
 * lts_autotune does).  A tiling decides which workgroup updates a node, not
 * the arithmetic applied to it.  Errors: LTS_ERR_ARG (no such
 * level, sizes outside 1..4096 other than the adaptive 0 x 0, or the region
 * does not fit the workgroup or its LDS), LTS_ERR_HIP. */
lts_status lts_set_tiling(lts_ctx ctx, int32_t level, int32_t tile_x, int32_t tile_y, int32_t rect);

/* ------------------------------------------------------------------------ */
/* Reductions (Sec. 2.2: estimator and level variance)                       */
/* ------------------------------------------------------------------------ */

/* out[0] = n, out[1] = mean, out[2] = M2 = sum (x_i - mean)^2 of x[0..n-1],
 * computed on the device by per-lane Welford updates merged pairwise (Chan
 * et al.); the unbiased variance is M2/(n-1).  x has ptr_kind; out is host.
 * Errors: LTS_ERR_ARG, LTS_ERR_HIP. */
lts_status lts_moments(lts_ctx ctx, const double* x, int32_t n, int32_t ptr_kind, double* out);

/* ------------------------------------------------------------------------ */
/* Discrete adjoint (gradient of the QoI w.r.t. the block log wave speeds)   */
/* ------------------------------------------------------------------------ */

/* dQ_dg[s][b] = dL/dg_b for L = sum_s dLdQ[s] Q_s, where g_b = log c_b =
 * log(kappa_b)/2, by the backward LF-LTS recurrence (the adjoint of the
 * forward recurrence, run from T to 0) with the forward states restored from
 * checkpoint pairs stored every K_ckpt steps: on levels with fine tiles by
 * running the (time-symmetric) step backward from the pair above each
 * segment, at most K_ckpt steps (rounding about K_ckpt eps max |u|), else by
 * recomputing each segment forward.  dt and n_steps are held fixed.
 * Q_out (may be NULL) receives the forward QoIs.  FP64 only.
 * Errors: LTS_ERR_ARG, LTS_ERR_OOM, LTS_ERR_HIP. */
lts_status lts_backward(lts_ctx ctx, int32_t level, const lts_samples* samples, const double* dLdQ,
                        int32_t K_ckpt, double* Q_out, double* dQ_dg_out);

/* ------------------------------------------------------------------------ */
/* Multilevel Monte Carlo driver (Algorithm 1)                              */
/* ------------------------------------------------------------------------ */

enum { LTS_MLMC_BATCHED = 0, LTS_MLMC_PLAIN = 1 };

#define LTS_MAX_LEVELS 8

typedef struct {
  int32_t n_levels;               /* levels given in level_ids, 0..LTS_MAX_LEVELS */
  int32_t level_ids[LTS_MAX_LEVELS];
  lts_sample_rule rule;
  uint64_t seed;
  double eps;                     /* RMSE target */
  double alpha;                   /* bias decay rate of the bias estimate (2 in the paper) */
  int32_t L_start;                /* initial finest level (Algorithm 1 starts at 2) */
  int32_t N_init[LTS_MAX_LEVELS]; /* initial sample counts, >= 2 for every level that may be used */
  int32_t mode;                   /* LTS_MLMC_BATCHED or LTS_MLMC_PLAIN */
  int32_t max_total_samples;      /* safety cap (<= 0: none) */
  int32_t n_levels_max;           /* > n_levels: levels n_levels .. n_levels_max-1 are built
                                     from gen_rule when Algorithm 1 first needs them */
  lts_rect_rule gen_rule;         /* level l of a generated hierarchy: gen_rule with
                                     n_base = gen_rule.n_base * 2^l */
  int32_t level_kind;             /* LTS_LEVELS_GRID: level_ids from lts_add_level /
                                     lts_build_rect_level; LTS_LEVELS_MESH: mesh ids from
                                     lts_add_mesh (solved by lts_mesh_forward level by level;
                                     no generated levels, no gradient); LTS_LEVELS_MLTS: grid
                                     levels with tiers attached (lts_set_mlts), solved by
                                     multi-level LTS (batched: lts_batch_run with
                                     LTS_BATCH_MLTS | LTS_BATCH_GRAPH; plain: lts_mlts_forward
                                     level by level), the cost model counting the multi-level
                                     updates ceil(T/(cfl h)) x updates_per_step (no gradient) */
  lts_mlts_desc gen_mlts;         /* LTS_LEVELS_MLTS with generated levels: the tiers attached
                                     to each (cell_tier must be NULL: the halving rule) */
} lts_mlmc_opts;

enum { LTS_LEVELS_GRID = 0, LTS_LEVELS_MESH = 1, LTS_LEVELS_MLTS = 2 };

typedef struct {
  double estimate;                /* sum_l mean(Delta Q_l) */
  int32_t L;                      /* finest level used */
  int32_t N[LTS_MAX_LEVELS];
  double mean[LTS_MAX_LEVELS];
  double var[LTS_MAX_LEVELS];     /* unbiased V_l */
  double cost[LTS_MAX_LEVELS];    /* cost model C_l (DOF updates per Delta Q_l sample) */
  double bias;                    /* |mean Delta Q_L| / (2^alpha - 1) */
  double rmse;                    /* sqrt(sum V_l/N_l + bias^2) */
  int32_t converged;              /* 1 if the bias test passed at the final L */
  double seconds;                 /* wall time of the solves (generated levels' set-up included) */
  int32_t level_ids[LTS_MAX_LEVELS]; /* context level id of every level used (generated ones too) */
} lts_mlmc_result;

/* Algorithm 1: start with L = min(L_start, Lmax) and N_init; repeat
 * {solve the missing Delta Q samples; estimate V_l; raise N_l to
 * ceil(2/eps^2 sqrt(V_l/C_l) sum sqrt(V C)); if the bias estimate exceeds
 * eps/sqrt(2) and L < Lmax, add level L+1} until no N_l grew.
 * Lmax + 1 = max(n_levels, n_levels_max): with n_levels_max > n_levels the
 * hierarchy grows beyond the given levels, each new level built (and added to
 * the context) only when the bias test asks for it.
 * C_l is the cost model in DOF updates per sample with the nominal step
 * cfl*h.  Errors: LTS_ERR_ARG, LTS_ERR_OOM, LTS_ERR_HIP, LTS_ERR_UNSTABLE. */
lts_status lts_mlmc(lts_ctx ctx, const lts_mlmc_opts* opts, lts_mlmc_result* out);

/* Algorithm 1 with the gradient of the QoI estimated alongside it: every
 * sample of every level is solved by the backward LF-LTS (lts_backward with
 * dL/dQ = 1, checkpoints every K_ckpt steps) on the fine and the coarse mesh,
 * which gives Q_l, Q_l-1 (equal bit for bit to the forward solves, so L, N_l
 * and *out are those of lts_mlmc) and dQ_l/dg, dQ_l-1/dg on the same sample.
 * Per level l <= out->L and block b: grad_mean[l*n_blocks + b] and
 * grad_var[l*n_blocks + b] are the mean and unbiased variance of
 * dG_l = dQ_l/dg_b - dQ_l-1/dg_b (dQ_0/dg_b for l = 0), reduced on the device
 * like lts_moments; grad_estimate[b] = sum_l grad_mean[l][b] estimates
 * dE[Q]/dg_b.  Levels not used are set to 0.  Host arrays of n_blocks, and
 * LTS_MAX_LEVELS x n_blocks.  Every used level needs p <= 64 (the adjoint's
 * limit).  Errors as lts_mlmc and lts_backward. */
lts_status lts_mlmc_grad(lts_ctx ctx, const lts_mlmc_opts* opts, int32_t K_ckpt, lts_mlmc_result* out,
                         double* grad_estimate, double* grad_mean, double* grad_var);

/* ------------------------------------------------------------------------ */
/* One-dimensional workloads (Sec. 4.1, 4.2): Neumann data, L^2(D)-valued QoI */
/* ------------------------------------------------------------------------ */

/* A level on an interval (lo, hi): uniform cells of size H, and every cell
 * inside the closed interval [fine_lo, fine_hi] split into cells of size
 * h_fine (H / h_fine an integer); P = the nodes of the fine cells, p =
 * ceil(H / h_fine) (1 when H <= h_fine: plain leapfrog).  Homogeneous Neumann
 * data: every node is a DOF; lumped masses sum |cell|/2.  The fine cells must
 * form one interval with at most 64 nodes in P and its neighbours (their
 * substeps run on one wavefront). */
typedef struct {
  double lo, hi, H;
  double fine_lo, fine_hi, h_fine;
  double nu;                      /* stabilization, 0 <= nu <= 1 */
  int32_t lf;                     /* 1: the standard leapfrog twin (the same nodes, P empty,
                                     p = 1, steps on the spacing h_fine of the refined cells) */
} lts_line_rule;

typedef struct {
  int32_t n_nodes, n_P, p;
  int32_t f0, n_fplus;            /* P and its neighbours: nodes f0 .. f0 + n_fplus - 1 */
  double H, nu;
} lts_line_info;

#define LTS_LINE_KL_TERMS 100
enum { LTS_LINE_KL = 0, LTS_LINE_JUMP = 1 };

/* Random wave speed of a one-dimensional workload, kappa = c^2 per cell at the
 * cell midpoint.  LTS_LINE_KL (Sec. 4.1): c^2(x) = 1 + sum_{k=1}^{100}
 * (1/(4 pi^2 k^2)) (cos(k pi x/6) xi1_k + sin(k pi x/6) xi2_k), xi ~ U(-1, 1)
 * i.i.d. (xi1_k = 2 u_{2k-2} - 1, xi2_k = 2 u_{2k-1} - 1 of the sample's
 * stream).  LTS_LINE_JUMP (Sec. 4.2): c = c_left for x < xi, c_right from xi
 * on, xi ~ U(jump_lo, jump_hi).  Streams as lts_gen_samples (purpose 0).
 * u_0(x) = exp(-(x - pulse_x)^2 / pulse_w2), u_t(0) = 0; n_steps =
 * ceil(T sqrt(max kappa) / (cfl H)), dt = T / n_steps. */
typedef struct {
  int32_t kind;
  double jump_lo, jump_hi, c_left, c_right;
  double pulse_x, pulse_w2;
  double T, cfl;
} lts_line_sample_rule;

/* Build a one-dimensional level; ids count 0, 1, ... separately from the 2D
 * levels.  Errors: LTS_ERR_ARG, LTS_ERR_OOM, LTS_ERR_HIP. */
lts_status lts_build_line_level(lts_ctx ctx, const lts_line_rule* rule, int32_t* line_id);

/* Host only: the level of `rule` (info required; x, mass [n_nodes] and P
 * [n_nodes] may be NULL).  Errors: LTS_ERR_ARG. */
lts_status lts_line_level_host(const lts_line_rule* rule, lts_line_info* info, double* x, double* mass,
                               uint8_t* P);

/* Host only: kappa [n][n_nodes - 1], n_steps [n], dt [n] of samples first ..
 * first+n-1 of MLMC level sample_level on the level of `mesh` (any output may
 * be NULL).  Errors: LTS_ERR_ARG. */
lts_status lts_gen_line_samples(uint64_t seed, int32_t sample_level, int64_t first, int32_t n,
                                const lts_line_sample_rule* rule, const lts_line_rule* mesh,
                                double* kappa, int32_t* n_steps, double* dt);

/* Solve n samples on line level `line_id` with stabilized LF-LTS
 * (Algorithm 2, start-up u_1 = q_1(u_0)) and write u(T) at every node:
 * U_out [n][n_nodes].  One workgroup per sample runs all its steps in one
 * launch, the state in LDS, the substeps of F+ on one wavefront.  kappa,
 * n_steps, dt and U_out have ptr_kind.  Errors: LTS_ERR_ARG, LTS_ERR_OOM,
 * LTS_ERR_HIP, LTS_ERR_UNSTABLE (a non-finite u(T)). */
lts_status lts_line_forward(lts_ctx ctx, int32_t line_id, int32_t n, int32_t ptr_kind, const double* kappa,
                            const int32_t* n_steps, const double* dt, const lts_line_sample_rule* rule,
                            double* U_out);

typedef struct {
  int32_t n_levels;               /* 1..LTS_MAX_LEVELS */
  int32_t line_ids[LTS_MAX_LEVELS];
  lts_line_sample_rule rule;
  uint64_t seed;
  double eps, alpha;
  int32_t L_start;
  int32_t N_init[LTS_MAX_LEVELS];
} lts_line_mlmc_opts;

typedef struct {
  int32_t L;
  int32_t N[LTS_MAX_LEVELS];
  double var[LTS_MAX_LEVELS];       /* V_l = sum_i |Delta Q_l(i) - mean|_V^2 / (N_l - 1) */
  double mean_norm[LTS_MAX_LEVELS]; /* |mean Delta Q_l|_V */
  double cost[LTS_MAX_LEVELS];      /* cost model per Delta Q_l sample */
  double bias, rmse;
  int32_t converged;
  int32_t n_nodes;                  /* nodes of the finest level used (length of the estimate) */
  double seconds;
} lts_line_mlmc_result;

/* Algorithm 1 for the V = L^2(D)-valued QoI Q = u(T) (Sec. 2.1, 2.2):
 * Delta Q_l = u_l - I u_{l-1} on mesh l (I the nodal interpolation onto the
 * finer, nested mesh), |v|_V^2 = sum_i m_i v_i^2 with mesh l's lumped masses,
 * V_l and the bias |mean Delta Q_L|_V / (2^alpha - 1) in that norm, N_l and L
 * as lts_mlmc (C_l = ceil(T/(cfl H)) ((N - |P|) + p |P|) per solve).
 * estimate [n_nodes of level L] receives sum_l I mean Delta Q_l on the finest
 * mesh used (host array of at least the finest level's n_nodes).  The
 * differences and their moments are formed on the device.  Errors as
 * lts_line_forward. */
lts_status lts_line_mlmc(lts_ctx ctx, const lts_line_mlmc_opts* opts, lts_line_mlmc_result* out,
                         double* estimate);

/* ------------------------------------------------------------------------ */
/* Timing of the last forward call (for benchmarks)                          */
/* ------------------------------------------------------------------------ */

typedef struct {
  double step_kernel_ms;          /* summed HIP-event time of the step kernel launches */
  int64_t step_launches;          /* number of step kernel launches */
  double total_ms;                /* HIP-event time of the whole device part */
  double dof_updates;             /* sum over samples of n_steps ((N - |P|) + p |P|) */
  double alg_bytes;               /* sum over samples of n_steps * 24 (12 in FP32) * N */
  int32_t batch_form;             /* last lts_batch_run: 0 step launches, 1 graph, 2 persistent */
  int32_t batch_sb_cap;           /* its S_b cap (persistent form), else 0 */
} lts_timing;

/* Enable (1) or disable (0) per-launch event timing (adds events around the
 * step kernel launches on the context stream). */
lts_status lts_set_timing(lts_ctx ctx, int32_t enable);
lts_status lts_get_timing(lts_ctx ctx, lts_timing* out);

/* Bound on a persistent workgroup's wait at a step barrier, in milliseconds
 * of the device's constant wall clock (default 2000; > 0).  A wait that runs
 * out makes the whole launch leave and lts_batch_run fail with LTS_ERR_STATE.
 * Errors: LTS_ERR_ARG. */
lts_status lts_set_barrier_timeout(lts_ctx ctx, double ms);

#ifdef __cplusplus
}
#endif

#endif /* LFLTSMC_H */
