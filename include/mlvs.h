/*
 * mlvs.h -- C ABI of the MI355X (gfx950) multi-level adaptive velocity-space
 * DUGKS library (libmlvs.so).
 *
 * The library advances the reduced BGK-Shakhov distributions g~, h~ of a
 * structured 2-D (or 1-D) finite-volume mesh with the discrete unified
 * gas-kinetic scheme (Sec. 2.2 of the paper, Eqs. phi_update .. recover_phi),
 * on one uniform velocity space or on a few representative velocity levels
 * built from per-cell requirements (Sec. 3.2) with conservative inter-level
 * coupling (Secs. 3.3-3.4).  Every hot-path step runs in HIP kernels on the
 * device; the host only builds geometry and level tables.
 *
 * Conventions
 *  - Every call returns mlvs_status (0 = MLVS_OK, negative = error).  No C++
 *    exception crosses the ABI.  mlvs_last_error() returns a thread-local,
 *    NUL-terminated message describing the last failure on that thread; it
 *    stays valid until the next call on that thread.
 *  - Arguments are checked before any device work; a failed check returns
 *    MLVS_E_ARG (bad argument) or MLVS_E_STATE (call not valid now) and leaves
 *    the context unchanged.  HIP runtime failures return MLVS_E_HIP.
 *  - Host arrays passed in are read during the call and copied; the caller
 *    keeps ownership.  Output arrays are caller-owned host buffers of the
 *    stated size.  Device memory is obtained only through the allocator in
 *    mlvs_device (or hipMalloc when none is given) and is owned by the context
 *    until mlvs_destroy.
 *  - All device work is ordered on the stream given in mlvs_device (the null
 *    stream when NULL).  mlvs_step is asynchronous; calls that return data to
 *    the host synchronise that stream.
 *  - Cells are numbered c = i + ni * j.  Velocity points of the base grid are
 *    numbered b = ix + nx * iy.  Points of a level follow the ascending order
 *    of their first (smallest) base index.
 */
#ifndef MLVS_H
#define MLVS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlvs_ctx_s* mlvs_ctx;
typedef int mlvs_status;

enum {
    MLVS_OK = 0,
    MLVS_E_ARG = -1,      /* invalid argument                              */
    MLVS_E_HIP = -2,      /* HIP runtime or kernel launch failure          */
    MLVS_E_OOM = -3,      /* device allocation failed                      */
    MLVS_E_STATE = -4,    /* call not valid in the current context state   */
    MLVS_E_NUMERIC = -5   /* non-finite or non-physical state (strict mode) */
};

/* Boundary kinds (Sec. 4 workloads; the wall is the isothermal diffuse wall). */
enum { MLVS_BC_WALL = 1, MLVS_BC_FARFIELD = 2, MLVS_BC_OUTFLOW = 3 };

typedef struct {
    int kind;          /* MLVS_BC_*                                                */
    double rho, u, v;  /* FARFIELD: incoming Maxwellian state; WALL: wall velocity */
    double T;          /* WALL: wall temperature; FARFIELD: temperature            */
} mlvs_bc;

/* Physical and numerical parameters.
 *  dim        1 or 2 (D of the paper); K internal degrees of freedom (0).
 *  R, Pr      gas constant and Prandtl number (Pr = 1 gives BGK).
 *  mu = mu_ref (T / T_ref)^omega  (power-law viscosity, Sec. 4 opening).
 *  dt > 0     fixed time step; dt <= 0: dt = cfl * hmin / max|xi| with hmin
 *             twice the smallest centre-to-face distance.
 *  precision  64 (g~, h~ stored in double) or 32 (stored in float; moment
 *             sums, corrections and totals in double).
 *  compat     0, 4 or 8: compatibility correction of the Shakhov target
 *             (Sec. 3.3.1): four moments (mass, momentum, energy; Eq.
 *             eq_four_moment_constraint) or eight (also the heat flux (1-Pr) q
 *             and a zero deviatoric stress; Eqs. eq_eight_basis,
 *             eq_eight_moment_constraint).  8 needs dim = 2.
 *  face_compat 1: also correct the face target used in Eq. recover_phi.
 *  map_moments 0, 4 or 9: linear mapping correction for level switches,
 *             neighbour mapping and cross-level states and fluxes (Sec. 3.3.2):
 *             four moments (mass, momentum, energy; Eqs. raw_four_g_basis,
 *             raw_four_gh_coupling) or nine (also the second g moments and the
 *             energy flux; Eqs. raw_six_g_basis, raw_three_h_basis,
 *             mapping_h_residual_correction).  9 needs dim = 2.
 *  positivity 0 or 1: what a level switch or a neighbour row does when its
 *             linear mapping correction turns a nonnegative provisional g
 *             negative somewhere (Sec. 3.3, the positivity check after the
 *             correction): 0 keeps the linear result (counted, see
 *             mlvs_neg_count); 1 replaces it by the exponential
 *             moment-constrained correction g* = g^p exp(a . phi), h* = h^p
 *             exp(a . phi), phi = [1, xi_x, xi_y, |xi|^2], with a from Newton's
 *             method on the four conserved moments (Eq.
 *             exponential_moment_correction; see mlvs_positivity_counts).
 *             1 needs map_moments = 4. */
typedef struct {
    int dim, K;
    double R, Pr, omega, mu_ref, T_ref;
    double dt, cfl;
    int precision, compat, face_compat, map_moments;
    int positivity;
} mlvs_physics;

/* Structured mesh: node coordinates row-major by j, (nj+1) x (ni+1) values
 * each; cells must be counter-clockwise.  1-D: nj = 1 and only x-faces are
 * used.  bc_* hold ids into bcs for the faces on each side (ignored on a
 * periodic side): bc_imin/bc_imax have nj entries, bc_jmin/bc_jmax ni. */
typedef struct {
    int ni, nj;
    const double *node_x, *node_y;
    int periodic_i, periodic_j;
    const int32_t *bc_imin, *bc_imax, *bc_jmin, *bc_jmax;
    int n_bc;
    const mlvs_bc* bcs;
} mlvs_mesh;

/* Unstructured 2-D mesh (Sec. 2.2; the paper's two-cavity expansion runs on
 * one).  Cells are counter-clockwise triangles or quadrilaterals: cell c has
 * the nodes cell_node[cell_ptr[c] .. cell_ptr[c+1]-1] (3 or 4 of them,
 * cell_ptr[0] = 0).  An edge shared by two cells is an interior face; an edge
 * of one cell only is a boundary face and must appear in bedge as (node a,
 * node b, boundary id into bcs), in either node order.  An edge of three or
 * more cells, a clockwise or degenerate cell, an unlisted boundary edge or an
 * id out of range is MLVS_E_ARG.  Every array is read during the call only.
 * Slopes: least squares over the face neighbours (a boundary face adds a
 * zero-gradient ghost at the mirror point), limited with Venkatakrishnan's
 * function at the face centres, eps^2 = |V_c|^(3/2) phi_ref^2 with phi_ref the
 * largest |phi| of the cell and its neighbours (Eq. reconstruction). */
typedef struct {
    int n_nodes, n_cells;
    const double *node_x, *node_y;    /* [n_nodes] */
    const int32_t *cell_ptr;          /* [n_cells + 1] */
    const int32_t *cell_node;         /* [cell_ptr[n_cells]] */
    int n_bedges;
    const int32_t* bedge;             /* [n_bedges][3] */
    int n_bc;
    const mlvs_bc* bcs;
} mlvs_umesh;

/* Tensor base velocity grid V_base: xi_b = (x[ix], y[iy]), w_b = wx[ix] * wy[iy].
 * 1-D: ny = 1, y = {0}, wy = {1}. */
typedef struct {
    int nx, ny;
    const double *x, *wx, *y, *wy;
} mlvs_vgrid;

/* Adaptation parameters (Sec. 3.2, Eqs. block-hysteresis-rule and
 * combined-merge-condition; tau_clust of the clustering).  interval > 0:
 * mlvs_step adapts at step 0 and every interval steps, before the step. */
typedef struct {
    double C_split, C_merge, eps_merge, tau_clust;
    int flux_test, interval;
} mlvs_adapt_params;

/* Device allocator hooks.  alloc returns device memory of at least `bytes`
 * (256-byte aligned) or NULL; free releases it.  NULL hooks use hipMalloc. */
typedef struct {
    void* stream;
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} mlvs_device;

typedef struct {
    int n_levels;          /* levels after the adaptation                   */
    int64_t n_unique;      /* distinct per-cell masks                       */
    int64_t n_changed;     /* cells whose velocity space changed (remapped) */
    int64_t n_cross;       /* cross-level faces                             */
    double nbar;           /* cell-weighted mean number of velocity points  */
    int64_t neg_count;     /* corrections that produced negative g          */
    int64_t n_fallback;    /* learned adaptation: cells sent to the criterion */
    /* host wall time of the parts of a criterion adaptation (ms): criterion
     * kernel (stream synchronised after it), deduplication of the masks,
     * clustering, level installation (remap, work lists); 0 for learned ones */
    double ms_criterion, ms_dedupe, ms_cluster, ms_install;
} mlvs_adapt_report;

/* Quadrature helpers (Sec. 2.3).  Newton-Cotes on [-a, a]: composite Boole
 * when (n-1) % 4 == 0, composite Simpson when (n-1) is even, composite
 * midpoint (cell-centred nodes) when n is even.  Gauss-Hermite: nodes
 * sqrt(2 R T0) x_k, weights sqrt(2 R T0) w_k exp(x_k^2).  x, w: n doubles. */
mlvs_status mlvs_vgrid_newton_cotes(int n, double a, double* x, double* w);
mlvs_status mlvs_vgrid_gauss_hermite(int n, double R, double T0, double* x, double* w);

/* mu_ref from a Knudsen number with the VHS relation
 * mu = 15 sqrt(pi) / (2 (5 - 2 omega)(7 - 2 omega)) Kn rho sqrt(2 R T) L. */
mlvs_status mlvs_mu_ref_from_kn(double Kn, double rho, double T, double R, double L,
                                double omega, double* mu_out);

/* Create a context on the current HIP device.  adapt may be NULL (uniform
 * velocity space).  Multi-level mode needs dim == 2. */
mlvs_status mlvs_create(const mlvs_physics* phys, const mlvs_mesh* mesh, const mlvs_vgrid* vgrid,
                        const mlvs_adapt_params* adapt, const mlvs_device* dev, mlvs_ctx* out);

/* The same on an unstructured mesh (dim = 2).  Cells keep their input ids in
 * every per-cell array of the ABI.  The learned selector's density-gradient
 * feature is the least-squares gradient over the face neighbours here. */
mlvs_status mlvs_create_unstructured(const mlvs_physics* phys, const mlvs_umesh* mesh, const mlvs_vgrid* vgrid,
                                     const mlvs_adapt_params* adapt, const mlvs_device* dev, mlvs_ctx* out);

/* Initial state: g~ = g_eq, h~ = h_eq at (rho, u, v, T) per cell, with the
 * compatibility correction when enabled.  rho_u_v_T: [n_cells][4] host. */
mlvs_status mlvs_init_equilibrium(mlvs_ctx ctx, const double* rho_u_v_T);

/* Install a level catalogue: kappa [n_levels][N_b] coarsening indices on the
 * 2x2 blocks of V_base (Sec. 3.2), cell_level [n_cells].  Cells whose space
 * changes are remapped (projection + mapping correction, Eq.
 * level_switch_conservation). */
mlvs_status mlvs_set_levels(mlvs_ctx ctx, int n_levels, const uint8_t* kappa, const int32_t* cell_level);

/* Advance n_steps time steps (stream-ordered, asynchronous).  Cross-level
 * faces run on a second stream of the context (default priority), forked
 * from the context stream after the neighbour mapping and joined back before
 * the update of the same step, so every step stays ordered on the caller's
 * stream.  In strict mode (mlvs_set_strict) the call synchronises and can
 * return MLVS_E_NUMERIC; the state is then left as computed. */
mlvs_status mlvs_step(mlvs_ctx ctx, int n_steps);

/* Strict mode (Sec. 3.3: the positivity check after every correction, here
 * made an error instead of a count).  flags is a bit set:
 *  1  before the first step of each mlvs_step call and after every step, the
 *     state of every cell is formed from the moments of its g~, h~ (Eqs.
 *     W_from_tilde, discrete_W); a moment that is not finite, or rho <= 0 or
 *     T <= 0, makes mlvs_step return MLVS_E_NUMERIC at that step, with the
 *     number of such cells and the first one's index, rho and T in
 *     mlvs_last_error().  Each step then synchronises the context stream.
 *  2  a mapping correction that makes a nonnegative provisional g negative
 *     (mlvs_neg_count), or an exponential correction whose Newton iteration
 *     does not converge, during an mlvs_step call makes that call return
 *     MLVS_E_NUMERIC after its last step.
 * 0 (the default) turns both off: such events are only counted.  Other
 * values are MLVS_E_ARG. */
mlvs_status mlvs_set_strict(mlvs_ctx ctx, int flags);

/* Replace the adaptation parameters (meaning as at create).  They apply from
 * the next adaptation on; mlvs_step adapts before every step whose index,
 * counted from create, is a multiple of the new interval.  MLVS_E_STATE if
 * the context was created without adaptation parameters; MLVS_E_ARG for
 * interval < 0 or C_merge > C_split. */
mlvs_status mlvs_set_adapt(mlvs_ctx ctx, const mlvs_adapt_params* adapt);

/* Criterion + grouping + remap now (Secs. 3.2, 3.4).  report may be NULL. */
mlvs_status mlvs_adapt(mlvs_ctx ctx, mlvs_adapt_report* report);

/* Per-cell coarsening masks of the criterion on the current state, without
 * changing levels: out [n_cells][N_b] host bytes.  Synchronises. */
mlvs_status mlvs_criterion(mlvs_ctx ctx, uint8_t* out);

/* Per-cell (rho, u, v, T, qx, qy) from g~, h~ (q as in Eq. discrete_q):
 * out [n_cells][6] host.  Synchronises. */
mlvs_status mlvs_moments(mlvs_ctx ctx, double* out);

/* Per-cell deviatoric stress (sigma_xx, sigma_xy, sigma_yy) = (P_xx - p,
 * P_xy, P_yy - p), P_ab = sum w c_a c_b g~ with c = xi - u and p = rho R T
 * (the viscous stress of the paper's cavity and cylinder results): out
 * [n_cells][3] host.  dim = 2 only.  Synchronises. */
mlvs_status mlvs_stress(mlvs_ctx ctx, double* out);

/* sum_cells |V| (rho, rho u, rho v, rho E), FP64, fixed-order tree sum. */
mlvs_status mlvs_totals(mlvs_ctx ctx, double out[4]);

/* Levels: n_levels; npts [n_levels]; ncells [n_levels]; n_cross.  Arrays may
 * be NULL; when given they must hold at least *n_levels entries (call once
 * with NULL arrays to size them). */
mlvs_status mlvs_level_info(mlvs_ctx ctx, int* n_levels, int32_t* npts, int32_t* ncells, int64_t* n_cross);

/* kappa of a level: out [N_b]. */
mlvs_status mlvs_level_kappa(mlvs_ctx ctx, int level, uint8_t* out);

/* Cell -> level map: out [n_cells]. */
mlvs_status mlvs_cell_levels(mlvs_ctx ctx, int32_t* out);

/* Read / write one cell's g~, h~ on its level (FP64 host values, npts of the
 * cell's level; g, h may be NULL to query npts).  Synchronises. */
mlvs_status mlvs_get_f(mlvs_ctx ctx, int64_t cell, double* g, double* h, int32_t* npts);
mlvs_status mlvs_set_f(mlvs_ctx ctx, int64_t cell, const double* g, const double* h);

/* Bulk read / write of every cell's g~, h~ in cell order, each cell's
 * values on its level: g, h hold sum over cells of npts(level(cell)). */
mlvs_status mlvs_get_state(mlvs_ctx ctx, double* g, double* h);
mlvs_status mlvs_set_state(mlvs_ctx ctx, const double* g, const double* h);

/* Time step in use, mesh hmin, and counts: n_cells, N_b (2x2 blocks). */
mlvs_status mlvs_info(mlvs_ctx ctx, double* dt, int64_t* n_cells, int32_t* n_blocks, int32_t* n_base);

/* Launch variants of a stage (kernels instantiated for several pairs of
 * velocity points per lane per load batch and minimum occupancy): *count
 * variants exist for `stage` (numbering as in mlvs_time_stage);
 * mlvs_set_variant selects one for subsequent launches.  Used by the
 * autotuner; results do not depend on the variant. */
mlvs_status mlvs_variants(int stage, int* count);
mlvs_status mlvs_set_variant(mlvs_ctx ctx, int stage, int variant);

/* Replay each step as a HIP graph (on = 1): the launches of one step are
 * captured once per level set (again after every adaptation or level
 * change) and replayed with hipGraphLaunch.  Needs a non-default stream
 * (MLVS_E_STATE otherwise).  Results are identical to direct launches. */
mlvs_status mlvs_set_graph(mlvs_ctx ctx, int on);

/* Persistent step (the batched form of the step, north of Sec. 4.4's remark
 * on kernel organisation and synchronisation): on = 1 runs each time step as
 * ONE launch of a persistent kernel over the context's work lists (neighbour
 * rows, then cross-level and same-level faces, then update with the next
 * step's cell stage, stages separated by grid-wide barriers; velocity rows
 * whole), preceded by a one-thread kernel that clears its barrier counter.
 * The kernel reads every work-list pointer and item count from a device
 * block the context rewrites in place at each level install, so with
 * mlvs_set_graph(ctx, 1) the captured step survives adaptations (captured
 * again only when the mode or the launch variant changes; see
 * mlvs_graph_info).  Results equal the fused step's.  on = 0 restores the
 * staged launches.  Synchronises. */
mlvs_status mlvs_set_persistent(mlvs_ctx ctx, int on);

/* Step launch statistics: *persistent the mode, *captures the number of step
 * graphs captured since creation, *launches the graph launches, *grid the
 * persistent kernel's workgroup count (0 before its first launch), *error the
 * persistent kernel's sticky error flag (1: a grid barrier gave up waiting,
 * the step that set it is invalid).  Any pointer may be NULL; reading *error
 * synchronises. */
mlvs_status mlvs_graph_info(mlvs_ctx ctx, int* persistent, int64_t* captures, int64_t* launches, int* grid,
                            int* error);

/* Traversal tiles of a 2-D structured mesh: cells (and the faces, by their
 * left cells) are visited tw x th cells at a time, row-major inside a tile and
 * over tiles, and each level stores its cells' rows in that order, so a run
 * of consecutive work items reads a compact patch of rows and its stencil halo
 * (L2 reuse on one XCD).  tw = th = 0: row-major.  The default is 16 x 8
 * (environment MLVS_TILE=WxH at creation overrides it).  Changing the tiles
 * reorders every level's state rows on the device (a copy, values unchanged)
 * and drops a captured step graph; results of later steps do not depend on
 * the tiles.  Errors: MLVS_E_ARG for tw or th outside [0, 4096] or only one of
 * them 0; MLVS_E_STATE for unstructured or 1-D meshes. */
mlvs_status mlvs_set_tiling(mlvs_ctx ctx, int tw, int th);
/* The current traversal tiles (0, 0: row-major or an unstructured mesh's
 * Morton order).  Either pointer may be NULL. */
mlvs_status mlvs_tiling(mlvs_ctx ctx, int* tw, int* th);

/* Work counters since creation: steps taken, cell-velocity updates on the
 * cells' own levels (sum over steps of sum over cells of the level size),
 * interface-space points processed on cross-level faces, adaptations. */
mlvs_status mlvs_counters(mlvs_ctx ctx, int64_t* steps, double* cell_updates, double* iface_points,
                          int64_t* adaptations);

/* Profiling: launch one stage of the step `reps` times on the context stream,
 * bracketed by two HIP events recorded on that stream, and return the mean
 * duration per launch in milliseconds.  stage: 0 cell, 1 neighbour mapping,
 * 2 face reconstruction (same-level and boundary faces), 3 face target (same
 * faces: face state, corrected target, recovery weights), 4 cross-level
 * faces, 5 update (fluxes and new state; the state is saved before and put
 * back after the timed launches), 6 criterion, and the fused forms of the
 * step whose levels have at most 1024 points: 7 face reconstruction and target
 * in one launch, 8 update followed by the next step's cell stage (state, rows
 * and parameters saved and put back as for 5; MLVS_E_STATE when the step is
 * not fused), 9 the persistent step (state saved and put back as for 8;
 * MLVS_E_STATE when it is off).  Needs a step taken since the last level
 * change for meaningful inputs.  Synchronises. */
mlvs_status mlvs_time_stage(mlvs_ctx ctx, int stage, int reps, double* ms_per_launch);

/* The stages one step launches, in order (numbering as in mlvs_time_stage):
 * 0 1 2 3 4 5, or 1 7 4 8 when every level has at most 1024 points (the
 * fused step; MLVS_FUSE=0 in the environment at create turns it off), or 9
 * with the persistent step on.
 * stages: caller-owned array of at least 8 ints, or null to query *count. */
mlvs_status mlvs_step_stages(mlvs_ctx ctx, int* stages, int* count);

/* Item counts of a stage's launch (cells, ghost rows, faces, ...) and the
 * total number of velocity points the launch processes. */
mlvs_status mlvs_stage_size(mlvs_ctx ctx, int stage, int64_t* items, double* points);

/* Device bytes held by the context. */
mlvs_status mlvs_memory(mlvs_ctx ctx, size_t* device_bytes);

/* Number of corrections since creation whose result had a negative g where
 * the provisional distribution had none (positivity check; values kept). */
mlvs_status mlvs_neg_count(mlvs_ctx ctx, int64_t* count);

/* Exponential fallbacks (positivity = 1) since creation: maps that took the
 * exponential correction, and maps whose Newton iteration did not converge
 * (those keep the linear result). */
mlvs_status mlvs_positivity_counts(mlvs_ctx ctx, int64_t* applied, int64_t* failed);

/* ---- learned level selector ------------------------------------------------
 * Network 10 -> 64 -> 64 -> K (ReLU, softmax), parameters as float in the
 * layout W1 [64][10], b1 [64], W2 [64][64], b2 [64], W3 [K][64], b3 [K],
 * mean [10], std [10] (inputs are standardised by mean/std); 2 <= K <= 16.
 * Features per cell: log rho, u/sqrt(R T_ref), v/sqrt(R T_ref), log(T/T_ref),
 * q_x/(p sqrt(RT)), q_y/(p sqrt(RT)), sigma_xx/p, sigma_xy/p,
 * log(1 + dx |grad rho|/rho), log10(lambda/dx) with lambda = (mu/p)
 * sqrt(pi R T/2), dx = sqrt(|V|); grad rho by central differences per index
 * direction (structured meshes) or least squares over the face neighbours
 * (unstructured meshes).  Labels: the fewest-point level of the
 * current catalogue whose enclosing mask is no coarser than the cell's own
 * criterion mask anywhere (the criterion decides), -1 if none. */
typedef struct {
    int epochs, batch;
    double lr, beta1, beta2, eps;
    double val_frac;       /* last fraction of the samples (in given order) held out */
    uint64_t seed;         /* shuffling */
} mlvs_train_cfg;

typedef struct {
    double loss_first, loss_last;   /* mean training loss of the first / last epoch */
    double train_acc, val_acc;      /* FP32 inference accuracy                     */
    int64_t n_train, n_val, steps;
    double ms;                      /* device time of the training loop            */
} mlvs_train_report;

/* Number of float parameters for K classes. */
mlvs_status mlvs_mlp_nparams(int K, int64_t* n);

/* Features of every cell from the current state: out [n_cells][10] floats. */
mlvs_status mlvs_features(mlvs_ctx ctx, float* out);

/* Criterion-judged catalogue labels of every cell: out [n_cells] (needs
 * adaptation parameters; the catalogue is the current level set). */
mlvs_status mlvs_labels(mlvs_ctx ctx, int32_t* out);

/* Train on the device (FP32 forward/backward/Adam kernels).  params: in the
 * initial values, out the trained ones (the mean/std block is set from the
 * training samples).  X [n][10], y [n] host arrays.  Uses hipMalloc and the
 * null stream; synchronous. */
mlvs_status mlvs_mlp_train(float* params, int K, const float* X, const int32_t* y, int64_t n,
                           const mlvs_train_cfg* cfg, mlvs_train_report* report);

/* One forward/backward pass on the device (no update): probs [B][K], grad
 * [n_params] (zero on the mean/std block), *loss the mean cross-entropy.
 * Host arrays; synchronous. */
mlvs_status mlvs_mlp_eval(const float* params, int K, const float* X, const int32_t* y, int B,
                          float* probs, float* grad, double* loss);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid hipMalloc):
 * mlvs_mlp_eval on caller-owned device buffers, with no allocation.  The
 * partial gradients and loss sums of the batch's workgroups live in a fixed
 * device array of the library of about 6.0 MB, which each GPU the library
 * runs on holds until the process ends.  d_params [mlvs_mlp_nparams(K)], d_X [B][10] and d_y [B]
 * (labels in [0, K), not checked) are device inputs; d_probs [B][K],
 * d_grad [mlvs_mlp_nparams(K)] (zero on the mean/std block) and d_loss_sum
 * (one double: the SUM of the per-sample cross-entropies; the mean is it / B)
 * are device outputs, each may be NULL.  1 <= B <= 4096 (MLVS_E_ARG
 * otherwise).  Asynchronous on `stream` (a hipStream_t; NULL = null stream),
 * no synchronisation and no memset, so the call can be captured in a graph.
 * Calls that overlap on one GPU share the array and race: order them on one
 * stream. */
mlvs_status mlvs_mlp_eval_noalloc(const float* d_params, int K, const float* d_X, const int32_t* d_y, int B,
                                  float* d_probs, float* d_grad, double* d_loss_sum, void* stream);

/* Inference: classes [B] (argmax, the lowest class on a tie) and optional
 * probs [B][K]; bf16 = 1 rounds the standardised inputs, weights and hidden
 * activations to bfloat16 (nearest even) and accumulates in FP32 on the matrix
 * cores; bf16 = 0 computes in FP32. */
mlvs_status mlvs_mlp_predict(const float* params, int K, const float* X, int B, int bf16,
                             int32_t* classes, float* probs);

/* Install a trained selector for the current catalogue (K == number of
 * levels) and enable learned adaptation.  Afterwards adaptations (mlvs_adapt,
 * and those mlvs_step runs at its interval) keep this catalogue frozen: each
 * cell's level is predicted from its features (BF16 inference); a prediction
 * is rejected when a block the predicted level merges has I_B > C_split on
 * the cell's distribution (tail-mass check); rejected cells take the
 * criterion's label.  params NULL removes the selector (and disables learned
 * adaptation). */
mlvs_status mlvs_selector_set(mlvs_ctx ctx, const float* params, int K);

/* Record one training snapshot from the context's own state: the features of
 * every cell and its criterion-judged label against the current catalogue
 * (as mlvs_features and mlvs_labels), appended to a host-side store owned by
 * the context.  reset = 1 empties the store first.  The store belongs to one
 * catalogue: a snapshot taken after the catalogue changed is MLVS_E_STATE
 * unless reset = 1.  *n_samples (may be NULL) receives the stored sample
 * count.  Synchronises. */
mlvs_status mlvs_selector_snapshot(mlvs_ctx ctx, int reset, int64_t* n_samples);

/* Train the selector on the recorded snapshots (samples whose label is -1
 * are skipped; the last val_frac of the rest, in recording order, is held
 * out) with the device training kernels, starting from He-normal weights
 * drawn from cfg->seed (splitmix64 stream, Box-Muller), and install the
 * result for the current catalogue, which must be the one the snapshots
 * refer to (MLVS_E_STATE otherwise, or when no snapshot was recorded).
 * Learned adaptation stays as mlvs_selector_enable left it (off after
 * create).  rep may be NULL.  Uses hipMalloc and the null stream;
 * synchronous. */
mlvs_status mlvs_selector_train(mlvs_ctx ctx, const mlvs_train_cfg* cfg, mlvs_train_report* rep);

/* on = 1: adaptations use the installed network (as described for
 * mlvs_selector_set); MLVS_E_STATE when none is installed or its class count
 * differs from the catalogue's level count.  on = 0: adaptations run the
 * criterion and rebuild the catalogue (the network stays installed). */
mlvs_status mlvs_selector_enable(mlvs_ctx ctx, int on);

/* The tail-mass check of learned adaptation on its own (Sec. 3.2 indicator,
 * Eq. block-contribution-indicator, applied to a proposed level): levels [n]
 * is a catalogue level index per cell, proposed for it; accept [n] receives
 * 1 where no block that level's mask merges carries I_B > C_split on the
 * cell's current distribution refined to V_base, else 0.  Host arrays, one
 * entry per cell.  MLVS_E_ARG for a level outside [0, number of levels);
 * MLVS_E_STATE for dim != 2.  Synchronous on the context's stream. */
mlvs_status mlvs_selector_check(mlvs_ctx ctx, const int32_t* levels, int32_t* accept);

/* The installed network: *K its class count (0: none); out (may be NULL)
 * receives mlvs_mlp_nparams(*K) floats in the layout above.  Synchronises. */
mlvs_status mlvs_selector_params(mlvs_ctx ctx, float* out, int* K);

void        mlvs_destroy(mlvs_ctx ctx);
const char* mlvs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MLVS_H */
