// Internal interface between the host library (mdx_host.h and the sources
// that include it) and the gfx950 kernels (mdx_assembly.hip, mdx_ionic.hip,
// mdx_solver.hip and the forms' files).
//
// Matrix layout on the device: sliced ELL with slices of 64 consecutive rows
// (one wavefront, one lane per row), column-major inside a slice:
//   entry j of row r lives at slice_ptr[r / 64] + j * 64 + (r % 64)
// so the j-th loads of the 64 rows of a wavefront are one contiguous 512-byte
// (f64) or 256-byte (f32/i32) segment.  Rows are in reverse Cuthill-McKee
// order, each row's columns ascending; short rows are padded with (col = row,
// value = 0).  The row count is padded to a multiple of TILE with empty rows
// whose vectors stay zero.  M, K and A share one pattern (slice_ptr, col).
// When every slice's columns span fewer than 2^16 indices (RCM keeps a
// slice's columns within about twice the bandwidth), the per-step kernels
// read the columns as 16-bit offsets from a per-slice base instead: 2 bytes
// per stored entry instead of 4.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace mdx {

constexpr int SLICE = 64;   // rows per slice = wavefront width
constexpr int TILE = 256;   // rows per workgroup pass = 4 slices
constexpr int NXCD = 8;     // accelerator complex dies on MI355X

// Row tiles owned by each workgroup.  Workgroup b (logical, after the XCD
// remap) owns tiles [b*tpb, min((b+1)*tpb, n_tiles)).  A reduction kernel
// writes one partial per workgroup; consumers re-reduce the `groups`
// partials in a fixed order, so every result is deterministic.
struct Tiling {
    int64_t n_rows;   // padded row count, multiple of TILE
    int n_tiles;      // n_rows / TILE
    int tpb;          // tiles per workgroup
    int groups;       // workgroups launched = ceil(n_tiles / tpb)
};
Tiling make_tiling(int64_t n_rows_padded, int max_groups);

// Device-side solver scalars, written by kernels, read by kernels and by the
// host (copied to pinned memory).  Double-buffered rho avoids a read/write
// race between workgroups of one kernel.
struct alignas(256) Scalars {
    double rho[2];      // r^T z of the current iteration (index k & 1)
    double ref;         // denominator of the relative stopping test
    double floor_;      // rounding floor 1e-15 * ||D^-1 b||
    double z0, znorm;   // ||z_0|| and the last ||z||
    double atol, rtol;
    int32_t done;       // solve finished (converged)
    int32_t iters;      // iterations taken by the finished solve
    int32_t nonfinite;  // a non-finite V was produced
    int32_t zero;       // always 0 (for launches that must not early-exit)
    // mixed-precision form: residual replacement protocol
    int32_t replace;    // a replacement is pending (iteration kernels idle): 1 the
                        // recursive residual passed the test, 2 periodic or cap
    int32_t nonfinite_v;  // a non-finite V found by the activation-time update
                          // (kept across solves; cleared with the state)
    int32_t it_next;    // iterations completed (index of the next one)
    int32_t use_mlp;    // learned warm start: the MLP guess was chosen this step
    double beta;        // beta of the next iteration (0: restart with p = z)
    double alpha;       // alpha of the current iteration
};

// Scalars as published to host memory (coherent pinned): the host spins on
// seq, written after the copy of s
struct Published {
    Scalars s;
    alignas(64) volatile int32_t seq;
};

// standardisation of the learned warm start's features and output scale
struct MlpNorm {
    float mean[4];
    float inv_std[4];
    float out_scale;
};

struct SellView {
    const int64_t *slice_ptr;
    const int32_t *col;
    const uint16_t *col16 = nullptr;   // 16-bit column offsets (null: read col)
    const int32_t *cbase = nullptr;    // per-slice base of col16
};

// Column stream of the sliced ELL as a kernel reads it: CI = int32_t (the
// columns themselves) or uint16_t (offsets from base[slice]).
template <typename CI>
struct Cols {
    using index_type = CI;
    const CI *idx;
    const int32_t *base;
};

// Calls f(std::integral_constant<bool, NT>{}, Cols<CI>{...}) for the column
// stream P provides and the non-temporal choice nt.
template <class F>
void with_cols(const SellView &P, bool nt, F &&f)
{
    if (P.col16) {
        const Cols<uint16_t> c{P.col16, P.cbase};
        if (nt) f(std::true_type{}, c); else f(std::false_type{}, c);
    } else {
        const Cols<int32_t> c{P.col, nullptr};
        if (nt) f(std::true_type{}, c); else f(std::false_type{}, c);
    }
}

// ---- assembly (mdx_assembly.hip) -----------------------------------------
// npe: 4 tetrahedra, 3 surface triangles (elements as 4-id records)
void launch_element(hipStream_t s, int npe, int64_t m, const double *xyz, const int32_t *tets,
                    const double *fibre, const double *sig, double *elem_vol, double *elem_k);
void launch_gather(hipStream_t s, int npe, int64_t n_slots, const int64_t *cptr,
                   const int32_t *contrib, const double *elem_vol, const double *elem_k,
                   double *Mv, double *Kv);
void launch_system(hipStream_t s, int64_t n_slots, const double *Mv, const double *Kv,
                   double cM, double cK, double *Av);
// mass lumping in place: row sums onto the diagonal, other entries zero
void launch_lump(hipStream_t s, int64_t n_rows, SellView A, double *Mv);
void launch_dinv(hipStream_t s, int64_t n_rows, int64_t n_real, SellView A, const double *Av,
                 double *dinv);

// ---- ionic models (mdx_ionic.hip) -----------------------------------------
int ionic_nstates(int kind);
int ionic_nparams(int kind);
void ionic_defaults(int kind, double *params);
// params: host array of ionic_nparams(kind) values (passed by value to kernels)
// tile_real (optional): per-tile count of real rows of the batched layout;
// rows beyond it are padding (no cell; out = 0, state untouched)
void launch_ionic_init(hipStream_t s, int kind, const double *params, int64_t n, int64_t ld,
                       double *V, double *Vprev, double *u, const int32_t *tile_real = nullptr);
// u advanced in place from V; out[i] = istim[i] - cm * I_ion/Cm if raw == 0,
// or I_ion/Cm (mV/ms) if raw != 0.  istim may be null (no active stimulus).
// With a guard, the kernel does nothing unless *guard is non-zero when it
// runs (a step's update queued before its predecessor's solve is known to be
// done).
// The previous step's activation and repolarisation times, carried by the
// kernel that reads the state they are taken from: t1 is the time of V (the
// kernel's input, V^{k+1}), Vold is V^k; lat == nullptr carries nothing.
struct StepTimes {
    double t1 = 0.0;
    const double *Vold = nullptr;
    double *lat = nullptr, *lrt = nullptr;
    Scalars *sc = nullptr;   // its nonfinite_v flag
};
void launch_ionic_step(hipStream_t s, int kind, const double *params, int64_t n, int64_t ld,
                       double dt, double cm, const double *V, double *u, const double *istim,
                       double *out, int raw, const int32_t *tile_real = nullptr,
                       const int32_t *guard = nullptr, const StepTimes &times = StepTimes{});

// Mixed-precision form: gates in FP32 (g32, ionic_gate_rows(kind) rows of ld
// floats), concentrations and the current in FP64 (u).  The FP64 array u
// keeps the full state layout; launch_gates_to_f32 / _to_f64 move the gate
// rows between u and g32.
int ionic_gate_rows(int kind);
int ionic_gate_row0(int kind);
void launch_ionic_step_mixed(hipStream_t s, int kind, const double *params, int64_t n, int64_t ld,
                             double dt, double cm, const double *V, double *u, float *g32,
                             const double *istim, double *out,
                             const int32_t *tile_real = nullptr,
                             const int32_t *guard = nullptr,
                             const StepTimes &times = StepTimes{});
void launch_gates_to_f32(hipStream_t s, int kind, int64_t ld, const double *u, float *g32);
void launch_gates_to_f64(hipStream_t s, int kind, int64_t ld, const float *g32, double *u);

struct StepParams {
    double chi, cm, theta, dt;
    int warm_start;    // 0: x0 = V^k, 1: x0 = 2V^k - V^{k-1}
    int rel_mode;      // 0: relative to ||z_0||, 1: relative to ||D^-1 b||
};

// ---- mixed-precision solver (mdx_mixed.hip) -----------------------------
void launch_to_f32(hipStream_t s, int64_t n, const double *a, float *b);
void launch_rhs_init_mixed(hipStream_t s, const Tiling &t, SellView P, const double *Mv,
                           const double *Kv, const double *dinv, const float *dinv32,
                           const StepParams &sp, const double *V, const double *Vprev,
                           const double *src, double *x, double *r64, float *r32, float *z32,
                           float *delta, double *partial, const double *kdiag, float *kvp, bool nt,
                           const int32_t *skip = nullptr);
// PCG iteration k of the FP32 form: SpMV on the tiling ts (q = A z + beta q,
// p = z + beta p, partial p.q), alpha, update on t (delta, r, z, partials
// r.z, z.z), stopping test of ||z_{k+1}|| and beta.  Events (optional) are
// recorded around the SpMV dispatch.
void launch_cg_iteration32(hipStream_t s, const Tiling &ts, const Tiling &t, int k, int rr,
                           int max_iter, SellView P, const float *A32, const float *dinv32,
                           float *z, float *p, float *q, float *delta, float *r,
                           double *partial_pq, double *partial_rz, Scalars *sc,
                           hipEvent_t ev_start, hipEvent_t ev_stop, bool nt);
// true residual update (r64 -= A32 delta), flush, finalize (all no-ops
// unless a replacement is pending)
void launch_replacement(hipStream_t s, const Tiling &t, SellView P, int max_iter, const float *A32,
                        double *x, float *delta, double *r64, const double *dinv,
                        const float *dinv32, float *r32, float *z32, double *partial, Scalars *sc,
                        bool nt);

// ---- learned warm start network (mdx_mlp.hip) ------------------------------
int mlp_nparams();
// gradient partials: one row of NPARAM + 1 floats per workgroup, at most
// kGradGroups (caller's scratch) or kNoAllocGroups (the library's array)
constexpr int kGradGroups = 2048;
constexpr int kNoAllocGroups = 256;
int mlp_grad_groups(int64_t n, int max_groups);
size_t mlp_grad_scratch_bytes(int64_t n);
// device address of the library's partials array on `device`, which must be
// current; resolved on the first call per device (null if that fails)
float *mlp_noalloc_scratch(int device);
void launch_mlp_forward(hipStream_t s, const float *P, int64_t n, const float *X, float *y);
// the same with the features formed from the state (no feature pass)
void launch_mlp_forward_state(hipStream_t s, const float *P, int64_t n, const double *V,
                              const double *Vprev, const double *src, const float *kvp, double cm,
                              const MlpNorm &nm, float *y);
void launch_mlp_grad(hipStream_t s, const float *P, int64_t n, const float *X, const float *T,
                     float *grad, float *loss, float *partials, int max_groups);
void launch_adam(hipStream_t s, float *P, float *m, float *v, const float *g, int t, double lr,
                 double b1, double b2, double eps);

// ---- learned warm start in the step (mdx_learned.hip) ----------------------
void launch_kdiag(hipStream_t s, int64_t n_rows, int64_t n_real, SellView K, const double *Kv,
                  double *kdiag);
// kvp = (K v)_i / K_ii in FP32 (the learned warm start's neighbour feature)
void launch_kv_feature(hipStream_t s, const Tiling &t, SellView P, const double *Kv,
                       const double *kdiag, const double *v, float *kvp);
// features of step n: V^n, V^n - V^{n-1}, s / Cm, kvp = (K V^{n-1})_i / K_ii;
// standardised into feat and raw into raw (either may be null), rows < n_real
void launch_features(hipStream_t s, int64_t n_real, int64_t n_rows, const double *V,
                     const double *Vprev, const double *src, const float *kvp, double cm,
                     const MlpNorm &nm, float *feat, float *raw);
// one pass over M and K: x = 2V - V_prev + scale y and its residual r = b - A x,
// the FP32 residual, z and zero correction (r32 non-null: FP32 iteration) or
// p0 = D^-1 r (FP64, p0 may be null), kvp = (K V)_i / K_ii for the next step;
// partials (five rows of t.groups) r.z, z.z of x and of 2V - V_prev
// (FP32-rounded in the FP32 iteration) and |D^-1 b|^2 into part5
void launch_rhs_learned(hipStream_t s, const Tiling &t, SellView P, const double *Mv,
                        const double *Kv, const double *kdiag, const double *dinv,
                        const float *dinv32, const StepParams &sp, float out_scale,
                        const double *V, const double *Vprev, const double *src, const float *y,
                        double *x, double *r, double *p0, float *r32, float *z32, float *delta,
                        float *kvp, double *part5, bool nt);
// chooses the guess (sc->use_mlp) and sets the scalars of its PCG start
void launch_init_finalize_ws(hipStream_t s, const Tiling &t, const double *p5, int rel_mode,
                             Scalars *sc);
void launch_record_dv(hipStream_t s, int64_t n, const double *Vold, const double *Vnew, float *dv);
void launch_mlp_samples(hipStream_t s, int64_t n_idx, const int64_t *idx, int64_t n_rows,
                        const float *X, const float *dV, bool stdz, const MlpNorm &nm, float *Xo,
                        float *To);

// ---- batched form (mdx_batch.hip) -----------------------------------------
// Several independent systems ("instances") share one block-diagonal matrix.
// Each instance's rows form a contiguous range that starts on a TILE
// boundary; the rows between its last real row and the next boundary are
// padding (empty rows, zero vectors, excluded from the ionic update by the
// per-tile count of real rows).  Every workgroup works for exactly one
// instance: entry g of the group table is {instance, first tile, end tile}
// and the groups of instance i are [inst_grp[i], inst_grp[i+1]), so a
// producer's per-group partials of one instance are contiguous and one
// finalize workgroup per instance reduces them in a fixed order.
struct SegTiling {
    int groups;                 // workgroups launched
    int n_inst;
    const int4 *grp;            // [groups] {instance, tile begin, tile end, 0}
    const int32_t *inst_grp;    // [n_inst + 1] first group of each instance
};

// Per-instance solver state of the batched mixed-precision PCG.  Only the
// finalize kernels (one workgroup per instance) write it; every other kernel
// reads it, so kernel boundaries order all accesses.
struct alignas(128) BScalars {
    double rho;         // r.z of the current iteration
    double alpha, beta;
    double ref;         // denominator of the relative stopping test
    double floor_;      // rounding floor 1e-15 ||D^-1 b||
    double z0, znorm;
    int32_t done;       // finished: converged, failed or non-finite
    int32_t iters;      // iterations of the finished solve
    int32_t it;         // iterations completed so far
    int32_t replace;    // replacement pending (iteration kernels idle): 1 after the
                        // recursive residual passed the test, 2 periodic or cap
    int32_t redirect;   // replacement did not stop: p = z + beta p pending
    int32_t nonfinite;  // a non-finite value reached a reduction
    int32_t failed;     // iteration cap reached without convergence
    int32_t pad_;
};

struct BParams {
    double atol, rtol;
    int max_iter;       // per step
    int rr;             // replacement interval (0: only at the stopping test and the cap)
    int rel_mode;       // 0: relative to ||z_0||, 1: relative to ||D^-1 b||
};

// Alternative layout of the iteration matrix for lpr lanes per row
// (lpr in {1, 2, 4}; 64 / lpr rows per wavefront): slices of 64/lpr rows;
// step j of the row in slice position s and sub-lane u holds entry
// j*lpr + u of that row at slice_ptr[slice] + 64*j + s*lpr + u.  lpr = 1 is
// the base layout.  sell_width(lpr) gives slice widths (steps) from row
// lengths; launch_relayout fills col / FP32 values from the base layout.
void launch_relayout(hipStream_t s, int lpr, int64_t n_slices, const int64_t *sptr_new,
                     SellView base, const float *A32, int32_t *col_new, float *A32_new);

// The iteration matrix as the SpMV reads it: sliced ELL (format 0, lpr in
// {1, 2, 4}, slice pointers sptr), CSR (format 1, lpr in {4, 8, 16} lanes
// reading each row's contiguous entries, row pointers rptr) or sliced ELL
// with 4-entry lane chunks (format 2, lpr 1), all in the internal row order
// with the FP32 values.
struct IterMatrix {
    int format;
    int lpr;
    bool nt;            // formats 0, 1: matrix streams read with the non-temporal hint
    const int64_t *sptr;
    const int32_t *rptr;
    const int32_t *col;
    const float *val;
};
// format 2: sliced ELL whose lanes load 4 consecutive entries of their row
// (entry k of slice position l at sptr[slice] + 256 (k / 4) + 4 l + k % 4)
void launch_relayout_v4(hipStream_t s, int64_t n_slices, const int64_t *sptr_new, SellView base,
                        const float *A32, int32_t *col_new, float *A32_new);
// CSR copy of the FP32 iteration matrix from the base sliced layout (rptr:
// row pointers of the real entries, already on the device)
void launch_build_csr(hipStream_t s, int64_t n_rows, SellView base, const float *A32,
                      const int32_t *rptr, int32_t *col_csr, float *val_csr);

// gv: scratch of 3 doubles per row (the gathered per-node values)
void launch_b_rhs_init(hipStream_t s, const SegTiling &t, SellView P, const double *Mv,
                       const double *Kv, const double *dinv, const float *dinv32,
                       const StepParams &sp, int64_t n_rows, const double *V, const double *Vprev,
                       const double *src, double *gv, double *x, double *b, float *r32,
                       float *delta, double *partial, bool nt);
void launch_b_init_finalize(hipStream_t s, const SegTiling &t, const double *partial,
                            const BParams &bp, BScalars *sc);
void launch_b_set_direction(hipStream_t s, const SegTiling &t, const float *dinv32,
                            const float *r32, float *p32, const BScalars *sc);
// one PCG iteration of every running instance: q = A p (+p.q), alpha,
// update (+r.z, z.z), test / beta, direction
void launch_b_iteration(hipStream_t s, const SegTiling &t, const IterMatrix &A,
                        const BParams &bp, const float *dinv32, float *p32, float *q32,
                        float *delta, float *r32, double *part_pq, double *part_rz, BScalars *sc,
                        hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// flush, true residual, finalize, redirect for instances with a pending replacement
// Persistent iteration: every running instance iterates in one launch until
// its next replacement point (see mdx_batch.hip); t must be a group table
// whose workgroups can all be resident (persistent_capacity: the most that
// can, 0 if the query fails).  bar: t.n_inst + 1 words (counters, then the
// fault flag at bar[t.n_inst], viewed as fault), cleared by the launch.
int persistent_capacity(int device);
void launch_b_persistent(hipStream_t s, const SegTiling &t, SellView P, const float *A32,
                         const float *dinv32, const BParams &bp, float *p32, float *q32,
                         float *delta, float *r32, double *part_pq, double *part_rz,
                         BScalars *sc, unsigned *bar, int *fault, int spin_cap);
void launch_b_replacement(hipStream_t s, const SegTiling &t, SellView P, const BParams &bp,
                          const double *Av, double *x, float *delta, const double *b,
                          const double *dinv, const float *dinv32, float *r32, float *p32,
                          double *partial, BScalars *sc, bool nt);
// the SpMV of the iteration alone (timing by the autotuner): q = A p, partial p.q
void launch_b_spmv(hipStream_t s, const SegTiling &t, const IterMatrix &A,
                   const float *p32, float *q32, double *part_pq, const BScalars *sc,
                   hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);

// ---- solver (mdx_solver.hip) ---------------------------------------------
void launch_fill(hipStream_t s, int64_t n, double v, double *x);
void launch_stim_add(hipStream_t s, int64_t n_idx, const int32_t *idx, double amp, double *istim);
// b, x0, r0 = b - A x0 and the partials (r.z, z.z, |D^-1 b|^2), z = D^-1 r
// skip (optional): the kernels return at once while *skip is non-zero (the
// learned warm start's fallback pass, run only where the network lost)
void launch_rhs_init(hipStream_t s, const Tiling &t, SellView P, const double *Mv,
                     const double *Kv, const double *dinv, const StepParams &sp,
                     const double *V, const double *Vprev, const double *src, double *x,
                     double *r, double *partial, const double *kdiag, float *kvp, double *p0,
                     bool nt, const int32_t *skip = nullptr);
// standalone solve: r = b - A x, p0 = z = D^-1 r, partials as the RHS pass
void launch_residual_init(hipStream_t s, const Tiling &t, SellView P, const double *Av,
                          const double *dinv, const double *b, const double *x, double *r,
                          double *p0, double *partial);
void launch_init_finalize(hipStream_t s, const Tiling &t, const double *partial, int rel_mode,
                          Scalars *sc, const int32_t *skip = nullptr);
// q = A p with partial p.q (no convergence logic; `done` non-zero skips it).
// ev_start/ev_stop: optional events recorded around the dispatch
void launch_spmv_dot(hipStream_t s, const Tiling &t, SellView P, const double *Av,
                     const double *p, double *q, double *partial, const int32_t *done,
                     hipEvent_t ev_start, hipEvent_t ev_stop, bool nt);
// PCG iteration k of the FP64 form: scheme 1 (two streaming kernels:
// q = A z + beta q and p = z + beta p on the tiling ts, then x, r, z) or 0
// (three: q = A p on ts, then x and r, then p = D^-1 r + beta p), each with
// the alpha and the stopping-test/beta finalize kernels.  Events (optional)
// are recorded around the SpMV dispatch.
void launch_cg_iteration(hipStream_t s, const Tiling &ts, const Tiling &t, int k, int max_iter,
                         int scheme, SellView P, const double *Av, const double *dinv, double *r,
                         double *z, double *p, double *q, double *x, double *partial_pq,
                         double *partial_rz, Scalars *sc, hipEvent_t ev_start, hipEvent_t ev_stop,
                         bool nt);
void launch_set_direction(hipStream_t s, int64_t n, const double *dinv, const double *r, double *p,
                          const Scalars *sc);
// activation / repolarisation times at t1 and the non-finite check; with a
// guard, only once *guard is non-zero (idempotent: it may be queued after
// every chunk of a solve)
void launch_epilogue(hipStream_t s, int64_t n, double t1, const double *Vold, const double *Vnew,
                     double *lat, double *lrt, Scalars *sc, const int32_t *guard = nullptr);
// the scalars copied to host-visible memory, then seq (after a system fence)
void launch_publish(hipStream_t s, const Scalars *sc, Published *pub, int32_t seq);

}  // namespace mdx
