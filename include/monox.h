/*
 * monox.h -- C ABI of the MI355X monodomain finite-element hot path.
 *
 * The library advances the monodomain model of TorchCor (arXiv 2510.12011):
 * Eq. (1) discretised with P1 finite elements in space and the theta-method
 * in time (Eq. 2 and the definitions of A and b after Eq. 3), one step being
 *   1. ionic update at every node (states by forward Euler, gating variables
 *      by Rush-Larsen), I_ion = I_ion(V^k, u^{k+1});
 *   2. b = chi M (Cm V^k - dt I_ion + dt I_stim) - (1-theta) dt K V^k;
 *   3. A V^{k+1} = b, A = chi Cm M + theta dt K, solved by Jacobi-PCG
 *      (Algorithm 1) from a warm start (2V^k - V^{k-1} by default);
 *   4. activation (LAT) and repolarisation (LRT) times.
 * The problem statement follows the "Software functionality" section: a mesh
 * with fibres and element regions, per-region longitudinal/transverse
 * conductivities, an ionic model with editable parameters, any number of
 * timed stimuli on node sets, solver tolerances, V saved at a fixed interval.
 *
 * Units (Table 1): mm, ms, mV, uA/mm^2, uF/mm^2, 1/mm, S/m.
 * Node and element ids are 0-based int32.  Every array crossing this
 * interface is in the caller's ORIGINAL node order; the library reorders
 * nodes internally (reverse Cuthill-McKee) and undoes it on output.
 *
 * Ownership: the caller owns every host array; the library copies inputs
 * before returning and keeps no pointer to them.  Device memory comes from
 * the caller: a persistent workspace bound with mdx_bind_workspace (it must
 * outlive the context) and a setup scratch passed to mdx_prepare (free to
 * reuse once mdx_prepare has returned).  The library itself allocates only
 * pinned host staging buffers (flags and one snapshot of V).
 *
 * Errors: every call returns an mdx_status.  Negative: the call had no
 * effect; mdx_last_error() describes it.  Positive: a warning, results are
 * valid (e.g. some PCG solves reached max_iter).  No C++ exception crosses
 * this interface.  A context is bound to one device and one HIP stream and
 * is not thread-safe.
 */
#ifndef MONOX_H
#define MONOX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#ifndef MDX_API
#define MDX_API __attribute__((visibility("default")))
#endif

typedef enum {
    MDX_OK = 0,
    MDX_WARN_NOT_CONVERGED = 1,   /* some solves hit max_iter; see mdx_stats */
    MDX_ERR_INVALID_ARG = -1,     /* bad pointer, size, range or value       */
    MDX_ERR_BAD_MESH = -2,        /* out-of-range id, degenerate element     */
    MDX_ERR_DEVICE = -3,          /* a HIP call failed                       */
    MDX_ERR_NO_WORKSPACE = -4,    /* workspace missing or too small          */
    MDX_ERR_NONFINITE = -5,       /* NaN/Inf appeared in V                   */
    MDX_ERR_STATE = -6,           /* call out of order (e.g. run before prepare) */
    MDX_ERR_UNSUPPORTED = -7
} mdx_status;

typedef struct mdx_ctx mdx_ctx;

/* ionic models: none (diffusion only), Mitchell-Schaeffer two-variable,
 * ten Tusscher-Panfilov 2006 (endocardial), Courtemanche-Ramirez-Nattel
 * 1998 (human atrial) */
enum { MDX_IONIC_NONE = 0, MDX_IONIC_MS = 1, MDX_IONIC_TT = 2, MDX_IONIC_CRN = 3 };
/* PCG warm start: previous step V^k, extrapolation 2V^k - V^{k-1} (paper),
 * or the learned per-node network (see mdx_set_mlp), which corrects the
 * extrapolation and falls back to it whenever its initial residual is not
 * the smaller of the two */
enum { MDX_WS_PREV = 0, MDX_WS_EXTRAP = 1, MDX_WS_MLP = 2 };
/* relative stopping test: ||z|| / ||z_0|| (paper) or ||z|| / ||D^-1 b|| */
enum { MDX_REL_INITIAL = 0, MDX_REL_RHS = 1 };
/* which assembled matrix mdx_get_matrix returns */
enum { MDX_MAT_M = 0, MDX_MAT_K = 1, MDX_MAT_A = 2 };

/* arithmetic of the step:
 *   MDX_PREC_FP64          plain FP64 throughout;
 *   MDX_PREC_MIXED         PCG iterations in FP32 (matrix values and vectors
 *                          of the SpMV and vector updates) with FP64 dot
 *                          products, FP64 right-hand side, solution and
 *                          residual replacement; ionic model in FP64;
 *   MDX_PREC_MIXED_GATES32 as MIXED, and the ionic gating variables stored
 *                          and advanced in FP32 (concentrations FP64).  On the
 *                          ten Tusscher-Panfilov slab this alone moves V by
 *                          ~1e-5 relative L2 over 50 ms. */
enum { MDX_PREC_FP64 = 0, MDX_PREC_MIXED = 1, MDX_PREC_MIXED_GATES32 = 2 };

typedef struct {
    double atol;          /* absolute tolerance on ||z|| (0: off)           */
    double rtol;          /* relative tolerance, see rel_mode               */
    int32_t rel_mode;     /* MDX_REL_*                                      */
    int32_t max_iter;     /* iteration cap per solve (>= 1)                 */
    int32_t warm_start;   /* MDX_WS_*                                       */
    int32_t precision;    /* MDX_PREC_*                                     */
    int32_t rr_interval;  /* mixed: FP64 residual replacement every this   */
                          /* many iterations (0: only at convergence / cap) */
    int32_t reserved;     /* must be 0                                      */
} mdx_solver_opts;

typedef struct {
    int64_t steps;            /* steps advanced since prepare / reset        */
    int64_t cg_iters_total;
    int64_t cg_iters_max;
    int64_t not_converged;    /* solves that reached max_iter                */
    int64_t n_nodes, nnz, n_sell_slots, bandwidth;
    double step_loop_seconds; /* host wall time inside mdx_run               */
    int64_t spmv_timed;       /* PCG SpMV-kernel launches timed (profiling on) */
    double spmv_seconds;      /* their summed device duration (HIP events)   */
    int64_t spmv_work;        /* of those, launches that did the SpMV (the   */
                              /* others only applied the stopping test)      */
    double spmv_bytes;        /* algorithmic bytes moved by those launches   */
    double host_wait_seconds; /* host time blocked on the stream in mdx_run  */
    int64_t fallbacks;        /* learned warm start: steps that used V^k     */
    int64_t col_index_bytes;  /* bytes per stored column index the per-step  */
                              /* kernels of a single mesh read: 2 (16-bit    */
                              /* offsets, MDX_TUNE_COMPACT_COLUMNS) or 4     */
} mdx_stats;

/* ---- context -------------------------------------------------------- */
/* device: HIP device ordinal; stream: a hipStream_t (NULL = null stream).
 * device -1 creates a host-only context that accepts the problem statement
 * (validation, reordering, workspace sizing) but no device work. */
MDX_API mdx_status mdx_create(mdx_ctx **out, int device, void *stream);
MDX_API void mdx_destroy(mdx_ctx *ctx);
/* message of the last failing call on ctx (never NULL) */
MDX_API const char *mdx_last_error(const mdx_ctx *ctx);
/* library version, for the binding's sanity check */
MDX_API int mdx_version(void);

/* ---- problem statement ------------------------------------------------ */
/* Mesh (P1 tetrahedra).  xyz: n_nodes*3 doubles, divided by unit_conversion
 * to give mm (1000 for micrometre input).  tets: n_tets*4 ids.  region:
 * n_tets region tags or NULL (all 0).  fibre: n_tets*3 directions (any
 * length, normalised inside) or NULL (isotropic: transverse value used).
 * Rejects non-finite coordinates, ids out of range and elements with
 * |det J| <= 1e-14 h^3 (h: the element's longest edge). */
MDX_API mdx_status mdx_set_mesh(mdx_ctx *ctx, int64_t n_nodes, const double *xyz,
                        double unit_conversion, int64_t n_tets, const int32_t *tets,
                        const int32_t *region, const double *fibre);
/* Surface mesh (P1 triangles in 3D, the triangular elements the paper's
 * "Software functionality" section admits beside tetrahedra).  The same
 * arguments as mdx_set_mesh with tris: n_tris*3 ids (any orientation),
 * region and fibre per triangle.  M and K are the P1 matrices of the
 * surface: M_e = area/12 (1 + d_ab), K_e = area grad(phi_a) . sigma
 * grad(phi_b) with gradients along the triangle and sigma built on the
 * fibre's projection onto the triangle's plane (isotropic where that
 * projection vanishes).  Rejects non-finite coordinates, ids out of range
 * and triangles with |(x1 - x0) x (x2 - x0)| <= 1e-14 h^2.  Batches of
 * surfaces: mdx_set_surface_mesh_batch. */
MDX_API mdx_status mdx_set_surface_mesh(mdx_ctx *ctx, int64_t n_nodes, const double *xyz,
                                        double unit_conversion, int64_t n_tris,
                                        const int32_t *tris, const int32_t *region,
                                        const double *fibre);
/* Conductivities (S/m) along (il) and across (it) the fibre for every
 * element whose region tag is in region_ids[0..n_ids).  Later calls override
 * earlier ones for the same tag.  Every tag present must be covered before
 * mdx_prepare. */
MDX_API mdx_status mdx_add_conductivity(mdx_ctx *ctx, int32_t n_ids, const int32_t *region_ids,
                                double il, double it);
/* The same from intracellular (il, it) and extracellular (el, et)
 * conductivities (S/m, all > 0), as the paper's add_conductivity takes them
 * (its usage listing): the monodomain conductivity in each direction is the
 * series combination s_i s_e / (s_i + s_e) (Table 2's 0.1334177 and
 * 0.0173515 S/m are those of (0.17, 0.62) and (0.019, 0.20)). */
MDX_API mdx_status mdx_add_conductivity_ie(mdx_ctx *ctx, int32_t n_ids, const int32_t *region_ids,
                                   double il, double it, double el, double et);
/* chi (1/mm) > 0, Cm (uF/mm^2) > 0, theta in [0, 1] (the paper's table of
 * schemes: 0 forward Euler, 0.5 Crank-Nicolson, 2/3 Galerkin, 1 backward
 * Euler) */
MDX_API mdx_status mdx_set_tissue(mdx_ctx *ctx, double chi, double cm, double theta);
/* Mass matrix M of A and b (Eq. 2): 0 (default) the consistent P1 mass, 1
 * the lumped mass (each row's sum on the diagonal).  Takes effect at the next
 * mdx_prepare. */
MDX_API mdx_status mdx_set_mass_lumping(mdx_ctx *ctx, int32_t lumped);
/* Ionic model and its editable parameters (NULL: defaults).
 * MDX_IONIC_MS, 7 params: tau_in, tau_out, tau_open, tau_close, u_gate,
 *   v_rest, v_amp (defaults 0.3, 6, 120, 150, 0.13, -80, 100).
 * MDX_IONIC_TT, 12 params: maximal conductances GNa, GK1, Gto, GKr, GKs,
 *   GCaL, GbNa, GbCa, GpCa, GpK and pump/exchanger scales PNaK, kNaCa.
 * MDX_IONIC_CRN, 13 params: gNa, gK1, gto, gKr, gKs, gCaL, gbNa, gbCa
 *   (nS/pF; defaults 7.8, 0.09, 0.1652, 0.029411765, 0.12941176, 0.12375,
 *   6.744375e-4, 1.131e-3), INaK_max, INaCa_max, IpCa_max (pA/pF; 0.59933874,
 *   1600, 0.275), Iup_max (mM/ms; 0.005) and a scale of gKur(V) (1).  Its
 *   gating variables always advance in FP64 (MDX_PREC_MIXED_GATES32 is
 *   MDX_ERR_UNSUPPORTED with this model). */
MDX_API mdx_status mdx_set_ionic(mdx_ctx *ctx, int32_t kind, int32_t n_params, const double *params);
/* number of ionic states per node (excluding V) and of parameters */
MDX_API int32_t mdx_ionic_nstates(int32_t kind);
MDX_API int32_t mdx_ionic_nparams(int32_t kind);
/* Stimulus: intensity (uA/mm^2) on node_idx[0..n_idx) for steps k with
 * round(start/dt) <= k < round((start+duration)/dt).  Stimuli add. */
MDX_API mdx_status mdx_add_stimulus(mdx_ctx *ctx, int64_t n_idx, const int32_t *node_idx,
                            double start, double duration, double intensity);
MDX_API mdx_status mdx_set_solver(mdx_ctx *ctx, const mdx_solver_opts *opts);

/* ---- device memory ---------------------------------------------------- */
/* Bytes of persistent workspace and of one-off setup scratch that
 * mdx_prepare needs for the current mesh and model (256-byte aligned). */
MDX_API mdx_status mdx_workspace_size(mdx_ctx *ctx, size_t *persistent_bytes, size_t *scratch_bytes);
/* device_ptr: device memory on ctx's device, at least persistent_bytes. */
MDX_API mdx_status mdx_bind_workspace(mdx_ctx *ctx, void *device_ptr, size_t bytes);

/* ---- setup and time stepping ------------------------------------------ */
/* Assemble M, K and A = chi Cm M + theta dt K on the device, build the
 * Jacobi preconditioner and set V, states to the ionic model's rest values
 * (V^{-1} := V^0), LAT/LRT to +inf, step counter to 0.  scratch: device
 * memory of at least scratch_bytes.  Blocks until the device is done. */
MDX_API mdx_status mdx_prepare(mdx_ctx *ctx, double dt, void *scratch, size_t scratch_bytes);
/* Advance n_steps.  Every out_every steps (0: never) the current V is
 * written to v_out (host, [n_steps/out_every][n_nodes] doubles, may be
 * NULL).  Returns MDX_WARN_NOT_CONVERGED if a solve hit max_iter,
 * MDX_ERR_NONFINITE (state left as is, step counter at the failing step)
 * if V stopped being finite. */
MDX_API mdx_status mdx_run(mdx_ctx *ctx, int64_t n_steps, int64_t out_every, double *v_out);
/* LAT and LRT (ms; +inf where not reached), host arrays of n_nodes or NULL.
 * LAT_i: the first step time t^{k+1} at which V_i > 0; LRT_i: the first later
 * step time at which V_i < -70 mV and falling ("Software functionality"). */
MDX_API mdx_status mdx_get_times(mdx_ctx *ctx, double *lat, double *lrt);
/* Action potential duration per node, APD_i = LRT_i - LAT_i (ms), +inf where
 * the node has not both activated and repolarised; host array of n_nodes. */
MDX_API mdx_status mdx_get_apd(mdx_ctx *ctx, double *apd);
/* PCG iteration count of each of the last n steps (n <= steps run so far
 * in the last mdx_run call), -1 where max_iter was hit. */
MDX_API mdx_status mdx_get_iterations(mdx_ctx *ctx, int64_t n, int32_t *iters);
MDX_API mdx_status mdx_get_stats(mdx_ctx *ctx, mdx_stats *out);
/* Profiling: every_n > 0 attaches HIP start/stop events (on the context's
 * stream) to every launch of the PCG kernel that computes q = A p during
 * every every_n-th step of mdx_run; their durations are summed into
 * mdx_stats.spmv_seconds (count spmv_timed, of which spmv_work did the
 * product, moving spmv_bytes algorithmic bytes).  0 (default) turns it off.
 * Events cost time: sample (e.g. every 10th step) to keep the step loop's
 * timing representative. */
MDX_API mdx_status mdx_set_profiling(mdx_ctx *ctx, int32_t every_n);

/* Launch-shape tuning (no effect on results beyond rounding order):
 *   MDX_TUNE_MAX_GROUPS  cap on workgroups of the row-tiled kernels
 *                        (16..65536, default 2048);
 *   MDX_TUNE_SPMV_MAX_GROUPS cap on workgroups of the PCG iteration's SpMV
 *                        kernel (16..65536, default 65536: one 256-row tile
 *                        per workgroup up to 16.7M rows);
 *   MDX_TUNE_ITER_SCHEME plain FP64 PCG iteration as three kernels (0:
 *                        SpMV, update, direction) or two kernels (1: the
 *                        SpMV kernel forms q = A p = A z + beta q and
 *                        p = z + beta p, A being linear, so its gathers
 *                        read z only).  The mixed-precision iteration
 *                        always takes the two-kernel form;
 *   MDX_TUNE_FORMAT      batched context: storage the iteration's FP32 SpMV
 *                        reads, 0 sliced ELL (default; 1 lane per row),
 *                        1 CSR (no padding; 8 lanes per row), 2 sliced
 *                        ELL with 4 consecutive entries per lane and
 *                        16-byte loads (1 lane per row), or 3 the same
 *                        with non-temporal loads of the matrix;
 *   MDX_TUNE_LANES_PER_ROW   batched context: lanes of a wavefront per row in
 *                        that SpMV: 1, 2 or 4 for sliced ELL (64, 32 or 16
 *                        rows per wavefront), 4, 8 or 16 for CSR;
 *   MDX_TUNE_TILES_PER_GROUP batched context: 256-row tiles per workgroup
 *                        (default 1);
 *   MDX_TUNE_GRAPH       batched context: 1 to replay each time step's work
 *                        up to the convergence check as a captured HIP graph
 *                        (one per iteration count and buffer rotation), 0 to
 *                        launch it kernel by kernel (default 0).
 *   MDX_TUNE_PERSISTENT  batched context: 1 to run each step's CG iterations
 *                        of all instances in one persistent launch (every
 *                        workgroup resident, the workgroups of an instance
 *                        meeting at barriers of their own, each instance
 *                        iterating until its next residual replacement),
 *                        0 (default) as five launches per iteration.  A
 *                        barrier that waits longer than about 60 ms (its
 *                        workgroups could not all be resident) ends the
 *                        launch and mdx_run returns MDX_ERR_DEVICE; a
 *                        batch with more instances than workgroups that can
 *                        be resident at once is refused (MDX_ERR_UNSUPPORTED);
 *   MDX_TUNE_NONTEMPORAL matrix streams (values, column indices) read with the
 *                        non-temporal cache hint: -1 (default) for each
 *                        kernel whose streams exceed 256 MiB (larger than
 *                        the Infinity Cache can keep between products), 0
 *                        never, 1 always.
 *   MDX_TUNE_COMPACT_COLUMNS  1 (default): where every 64-row slice's
 *                        columns span fewer than 2^16 indices (RCM keeps
 *                        them within about twice the matrix bandwidth), the
 *                        per-step kernels of a single mesh read the column
 *                        indices as 16-bit offsets from a per-slice base,
 *                        2 bytes per stored entry instead of 4; 0 reads the
 *                        32-bit indices.  Results are bitwise the same.
 * MAX_GROUPS, SPMV_MAX_GROUPS and ITER_SCHEME take effect at the next
 * mdx_prepare / mdx_run;
 * the batched keys need a prepared batched context and act at once. */
enum {
    MDX_TUNE_MAX_GROUPS = 1,
    MDX_TUNE_ITER_SCHEME = 2,
    MDX_TUNE_LANES_PER_ROW = 3,
    MDX_TUNE_TILES_PER_GROUP = 4,
    MDX_TUNE_GRAPH = 5,
    MDX_TUNE_FORMAT = 6,
    MDX_TUNE_NONTEMPORAL = 7,
    MDX_TUNE_COMPACT_COLUMNS = 8,
    MDX_TUNE_SPMV_MAX_GROUPS = 9,
    MDX_TUNE_PERSISTENT = 10
};
MDX_API mdx_status mdx_set_tuning(mdx_ctx *ctx, int32_t key, int64_t value);

/* ---- batched form ------------------------------------------------------- */
/* Many independent meshes ("instances") in one context, each its own
 * monodomain problem (Eq. 1, discretised as Eq. 2-3, its own conductivities
 * through region tags and its own stimuli), advanced together as one
 * block-diagonal system.  node_ptr: HOST [n_inst + 1], instance i owns the
 * nodes [node_ptr[i], node_ptr[i+1]) of the concatenated xyz (node_ptr[0] =
 * 0, strictly increasing, node_ptr[n_inst] = n_nodes); every element's nodes
 * must lie in one instance (else MDX_ERR_BAD_MESH).  The remaining arguments
 * and checks are those of mdx_set_mesh over the concatenation.  Inside, each
 * instance is ordered by reverse Cuthill-McKee and starts on a 256-row
 * boundary.  A batched context solves with the mixed-precision form
 * (MDX_PREC_MIXED or MDX_PREC_MIXED_GATES32; MDX_PREC_FP64 and MDX_WS_MLP
 * return MDX_ERR_UNSUPPORTED from mdx_run), with its own CG scalars,
 * stopping test and iteration count per instance: finished instances stop
 * iterating while the others continue.  All other calls work on the
 * concatenated node numbering. */
MDX_API mdx_status mdx_set_mesh_batch(mdx_ctx *ctx, int32_t n_inst, const int64_t *node_ptr,
                                      int64_t n_nodes, const double *xyz,
                                      double unit_conversion, int64_t n_tets,
                                      const int32_t *tets, const int32_t *region,
                                      const double *fibre);
/* The same for a batch of triangle surface meshes (the paper's cohort of
 * atrial surfaces run one after another, here advanced together): tris
 * n_tris*3 ids in the concatenated numbering, element rules as
 * mdx_set_surface_mesh, batch rules as mdx_set_mesh_batch. */
MDX_API mdx_status mdx_set_surface_mesh_batch(mdx_ctx *ctx, int32_t n_inst,
                                              const int64_t *node_ptr, int64_t n_nodes,
                                              const double *xyz, double unit_conversion,
                                              int64_t n_tris, const int32_t *tris,
                                              const int32_t *region, const double *fibre);
/* PCG iterations of the last n steps of a batched context, per instance:
 * iters[s * n_inst + i] (HOST, n * n_inst; -1: the solve hit max_iter). */
MDX_API mdx_status mdx_get_instance_iterations(mdx_ctx *ctx, int64_t n, int32_t *iters);

#define MDX_TUNE_MAX_CANDIDATES 32
typedef struct {
    int32_t format;             /* installed choice: MDX_TUNE_FORMAT value    */
    int32_t lanes_per_row;
    int32_t tiles_per_group;
    int32_t n_candidates;
    double seconds;             /* its mean SpMV time                        */
    double bytes;               /* algorithmic bytes per SpMV: 8 nnz + 8 n    */
    int32_t cand_format[MDX_TUNE_MAX_CANDIDATES];
    int32_t cand_lanes_per_row[MDX_TUNE_MAX_CANDIDATES];
    int32_t cand_tiles_per_group[MDX_TUNE_MAX_CANDIDATES];
    double cand_seconds[MDX_TUNE_MAX_CANDIDATES];
} mdx_tune_report;
/* Autotuner of a prepared batched context: times reps launches (1..1000) of
 * the iteration's FP32 SpMV on the context's own matrix for sliced ELL with
 * 1, 2, 4 lanes per row (64, 32, 16 rows per wavefront), sliced ELL with
 * 4-entry vector loads (plain or non-temporal), and CSR with 4, 8, 16 lanes
 * per row (16, 8, 4 rows
 * per wavefront), each with 1, 2, 4, 8 tiles
 * per workgroup, and installs the fastest (as the MDX_TUNE_FORMAT,
 * MDX_TUNE_LANES_PER_ROW and MDX_TUNE_TILES_PER_GROUP keys would).  Results
 * of later steps change only by the FP32 summation order of the SpMV.
 * report (HOST, may be NULL) receives every candidate's time. */
MDX_API mdx_status mdx_autotune(mdx_ctx *ctx, int32_t reps, mdx_tune_report *report);

/* ---- state (checkpoint / resume, parity checks) ----------------------- */
/* V^k, V^{k-1}, states u (SoA, [nstates][n_nodes]), LAT, LRT and the step
 * index, all host arrays in original node order; any pointer may be NULL
 * on get.  set requires all of V, Vprev, u (if nstates > 0), each finite
 * (else MDX_ERR_INVALID_ARG); LAT and LRT may hold +inf. */
MDX_API mdx_status mdx_get_state(mdx_ctx *ctx, double *V, double *Vprev, double *u,
                         double *lat, double *lrt, int64_t *step);
MDX_API mdx_status mdx_set_state(mdx_ctx *ctx, const double *V, const double *Vprev,
                         const double *u, const double *lat, const double *lrt,
                         int64_t step);

/* ---- inspection -------------------------------------------------------- */
/* Assembled matrix `which` (MDX_MAT_*) as COO triplets in original node
 * numbering, structural zeros of the padded layout omitted.  Call with
 * rows == NULL to get *nnz; then with arrays of *nnz entries. */
MDX_API mdx_status mdx_get_matrix(mdx_ctx *ctx, int32_t which, int64_t *nnz, int32_t *rows,
                          int32_t *cols, double *vals);
/* y = which * x with the library's SpMV kernel; host x, y in original order */
MDX_API mdx_status mdx_spmv(mdx_ctx *ctx, int32_t which, const double *x, double *y);
/* One Jacobi-preconditioned CG solve (Algorithm 1) of A x = b with the
 * context's system matrix A = chi Cm M + theta dt K, outside the time loop:
 * host b and x0 (n values, original order) in, host x out; *iters (may be
 * NULL) receives the iterations taken, or -1 if max_iter ran out.  Non-finite
 * b or x0: MDX_ERR_INVALID_ARG.  Uses the
 * solver options' atol, rtol, rel_mode and max_iter with the FP64 kernels
 * of the time step (three per iteration), whatever the precision setting.
 * Needs mdx_prepare; leaves the simulation state untouched.  Single-mesh
 * contexts only (MDX_ERR_UNSUPPORTED on a batch); MDX_ERR_NONFINITE if the
 * iteration produced a non-finite value.  Blocks until done. */
MDX_API mdx_status mdx_solve(mdx_ctx *ctx, const double *b, const double *x0, double *x,
                             int32_t *iters);
/* One ionic update of the model set by mdx_set_ionic on n independent cells,
 * DEVICE arrays on ctx's device and stream: V[n]; u[nstates][n] (SoA)
 * advanced in place; iion[n] receives I_ion(V, u^{k+1}) / Cm in mV/ms.
 * Needs no mesh and no workspace; does not touch the simulation state.
 * Blocks until the device is done. */
MDX_API mdx_status mdx_ionic_step(mdx_ctx *ctx, double dt, int64_t n, const double *V,
                          double *u, double *iion);

/* ---- learned warm start: the network ---------------------------------- */
/* A per-node MLP 4 -> 64 -> 64 -> 64 -> 1 (ReLU) predicts the normalised
 * departure of V^{n+1} from the extrapolation 2V^n - V^{n-1} (the paper's
 * warm start, after Algorithm 1) from node-local features; the network is
 * not part of the paper.
 * Parameters: FP32, MDX_MLP_NPARAM values laid out
 *   W1[64][4] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64] b4
 * (W[out][in]).  Kernels use BF16 weights and activations with FP32
 * accumulation (BF16 MFMA).  All arrays below are DEVICE arrays on ctx's
 * device; calls are queued on ctx's stream and return without waiting. */
#define MDX_MLP_NPARAM 8705
MDX_API int32_t mdx_mlp_nparams(void);
/* y[i] = net(X[i]) for i < n; X is [n][4] FP32 (16-byte aligned), y [n]. */
MDX_API mdx_status mdx_mlp_forward(mdx_ctx *ctx, const float *params, int64_t n, const float *X,
                                   float *y);
/* bytes of scratch mdx_mlp_grad needs for n samples */
MDX_API size_t mdx_mlp_grad_scratch(int64_t n);
/* grad = d/dparams of L = (1/n) sum_i (net(X[i]) - T[i])^2 and loss = L
 * (loss may be NULL).  Deterministic: per-workgroup partials in scratch are
 * summed in a fixed order. */
MDX_API mdx_status mdx_mlp_grad(mdx_ctx *ctx, const float *params, int64_t n, const float *X,
                                const float *T, float *grad, float *loss, void *scratch,
                                size_t scratch_bytes);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid hipMalloc):
 * the gradient and loss of mdx_mlp_grad with no scratch argument.  The
 * per-workgroup partials live in a file-scope device array of the library,
 * 256 workgroups x (MDX_MLP_NPARAM + 1) floats = 8.9 MB, held by every device
 * the library runs on until the process ends; its address is resolved per
 * device at mdx_create.  Any n in [1, 2^31 - 1] fits (each workgroup takes
 * ceil(n / 8192) tiles of 32 samples); a larger n is rejected with
 * MDX_ERR_INVALID_ARG.  For n <= 8192 the samples are partitioned as in
 * mdx_mlp_grad and the results are bitwise the same; above, they differ by
 * the FP32 summation order of the partials.  Allocates nothing and calls no
 * allocating routine.  All calls on one device share its array (each call
 * overwrites it): calls queued on one stream are safe, calls that overlap on
 * one GPU (other streams or contexts) race. */
MDX_API mdx_status mdx_mlp_grad_noalloc(mdx_ctx *ctx, const float *params, int64_t n,
                                        const float *X, const float *T, float *grad,
                                        float *loss);
/* one Adam step (Kingma & Ba) on params with moments m, v; t >= 1 */
MDX_API mdx_status mdx_mlp_adam(mdx_ctx *ctx, float *params, float *m, float *v, const float *grad,
                                int32_t t, double lr, double beta1, double beta2, double eps);

/* ---- learned warm start: use in the time step ------------------------- */
/* Install the network for MDX_WS_MLP.  params: HOST FP32 [MDX_MLP_NPARAM];
 * norm: HOST [9] = feature means (4), feature standard deviations (4),
 * output scale.  Features of node i at step n: V^n, V^n - V^{n-1},
 * (I_stim - I_ion)/Cm (mV/ms), (K V^{n-1})_i / K_ii (the neighbour aggregate
 * of the previous step's right-hand side).  The network predicts the
 * departure from the paper's extrapolation: guess x0 = 2V^n - V^{n-1} +
 * scale y, used when its initial residual ||D^-1 r0|| is below that of the
 * extrapolation itself (the fallback; a network with zero output is the
 * paper's warm start).  Requires a prepared context; the network lives in
 * the workspace. */
MDX_API mdx_status mdx_set_mlp(mdx_ctx *ctx, const float *params, const double *norm);
/* Training samples for mdx_mlp_grad (the network's training data plumbing,
 * on the device): for i < n_idx, row j = idx[i] of the recorder's output
 * (X: [n_rows][4] raw features, dV: [n_rows] increments V^{n+1} - V^n) is
 * written to Xo[i][0..3] and To[i], either raw (norm NULL) or as the network
 * trains on it (norm: HOST double[9] as mdx_set_mlp takes it): Xo = (X -
 * mean) / std, To = (dV - X[1]) / out_scale, i.e. the departure of V^{n+1}
 * from the extrapolation 2V^n - V^{n-1} in units of out_scale.  idx, X, dV,
 * Xo, To are DEVICE arrays (idx int64; X and Xo 16-byte aligned); an index
 * outside [0, n_rows) gives a zero feature row and a NaN target.  Queued on
 * ctx's stream.  Errors: MDX_ERR_INVALID_ARG for a negative count, a null
 * or misaligned array, a non-finite norm or a std or out_scale <= 0. */
MDX_API mdx_status mdx_mlp_samples(mdx_ctx *ctx, int64_t n_idx, const int64_t *idx, int64_t n_rows,
                                   const float *X, const float *dV, const double *norm, float *Xo,
                                   float *To);
/* Training-data recorder: when non-NULL, every step of mdx_run writes the
 * raw features of node i (internal node order, i < n_nodes) to X[i][0..3]
 * and, after the solve, V^{n+1}_i - V^n_i to dV[i] (DEVICE arrays of
 * n_nodes float4 / float, overwritten each step); y (DEVICE, n_nodes floats,
 * may be NULL; needs X and dV) receives the network's output of the step
 * when the warm start is MDX_WS_MLP.  The permutation from internal to
 * original order is node_order[i] (mdx_get_node_order).  Pass NULLs to stop
 * recording. */
MDX_API mdx_status mdx_set_recorder(mdx_ctx *ctx, float *X, float *dV, float *y);
/* original node id of internal row i, i < n_nodes (host array) */
MDX_API mdx_status mdx_get_node_order(mdx_ctx *ctx, int32_t *order);

#ifdef __cplusplus
}
#endif
#endif /* MONOX_H */
