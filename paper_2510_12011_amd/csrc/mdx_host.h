// Host side of the monodomain library, shared by its source files: the
// context behind the C ABI's opaque handle (problem statement, ordering and
// layout, device workspace offsets, solver and form state) and the internal
// helpers each part of the host code provides:
//   mdx_order.hip        node adjacency, reverse Cuthill-McKee, Hilbert order
//   mdx_layout.hip       sliced-ELL pattern and workspace layout, batched
//                        group tables and iteration layouts, mesh intake
//   mdx_batched_run.hip  the batched form's time loop
//   mdx_run.hip          mdx_run: the single-mesh time loop
//   mdx_api.hip          the remaining entry points of include/monox.h
#pragma once

#include <hip/hip_runtime.h>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <new>
#include <string>
#include <vector>
#include "../../include/monox.h"
#include "mdx_internal.h"

namespace mdx {
namespace host {


constexpr int kMaxGroups = 2048;      // default cap on row-tiled workgroups
// matrix streams above this size are read with the non-temporal hint (they do
// not stay in the 256 MB Infinity Cache between products anyway)
constexpr double kStreamCacheBytes = 256.0 * 1024 * 1024;
constexpr int kPartialCap = 65536;    // partial slots per reduction (>= any cap)
constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Stim {
    std::vector<int32_t> nodes;   // original ids, sorted, unique
    double start, duration, amp;
};

// byte offsets of every array inside the persistent workspace / setup scratch
struct Layout {
    size_t slice_ptr, col, col16, cbase, Mv, Kv, Av, dinv, vec[3], r, p, p2, q, b, s, istim, u, lat,
        lrt, stim_idx, partial, scalars;
    size_t A32, dinv32, r32, z32, p32, q32, delta, g32;   // mixed-precision form
    size_t kdiag, kvp, feat, mlp_y, mlp_params;       // learned warm start
    size_t tile_real, grp, inst_grp, bsc, sptr_t, col_t, A32_t;   // batched form
    size_t pgrp, pinst_grp, pbar;   // batched form, persistent iteration
    size_t csr_ptr, csr_col, csr_val, gv;
    size_t total;
    size_t x_xyz, x_tets, x_fibre, x_sig, x_vol, x_ek, x_cptr, x_contrib, x_total;
};


}  // namespace host
}  // namespace mdx

using namespace mdx;
using namespace mdx::host;

struct mdx_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // problem statement (host copies, original numbering)
    int64_t n = 0, m = 0;
    int npe = 4;                   // vertex ids per element: 4 tetrahedra, 3 surface triangles
    std::vector<double> xyz;       // mm
    std::vector<int32_t> tets, region;   // tets: 4 ids per element (-1 after a triangle's 3)
    std::vector<double> fibre;     // empty: isotropic
    std::map<int32_t, std::pair<double, double>> cond;
    double chi = 140.0, cm = 0.01, theta = 0.5;
    bool lumped = false;   // mass lumping (row sums on the diagonal)
    int ionic_kind = 0;
    std::vector<double> ionic_params;
    std::vector<Stim> stims;
    mdx_solver_opts opts{1e-5, 1e-5, MDX_REL_INITIAL, 100, MDX_WS_EXTRAP, MDX_PREC_FP64, 50, 0};

    // ordering and layout (host)
    std::vector<int32_t> perm, iperm;   // perm[new] = old, iperm[old] = new
    int64_t npad = 0, nslices = 0, nslots = 0, nnz = 0, bandwidth = 0;
    std::vector<int64_t> slice_ptr;
    std::vector<int32_t> col_sell, rowlen;
    // compact columns: col_sell[e] = cbase[slice] + col16[e] when every
    // slice's columns span fewer than 2^16 indices (else both empty)
    std::vector<uint16_t> col16;
    std::vector<int32_t> cbase;
    std::vector<int64_t> stim_off;      // offsets of each stimulus in the device list

    // device memory
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Layout L{};
    float *grad_scratch = nullptr;   // library-owned partials of mdx_mlp_grad_noalloc
    // the model's gates have no FP32 form (MDX_PREC_MIXED_GATES32 unsupported)
    bool ionic_gates64_only() const { return ionic_kind == MDX_IONIC_CRN; }
    Tiling tiling{};        // vector and right-hand-side kernels
    Tiling tiling_spmv{};   // the PCG iteration's SpMV kernel
    bool prepared = false;
    double dt = 0.0;
    int64_t step = 0;
    int vb[3] = {0, 1, 2};   // which vec[] holds V^k, V^{k-1}, x
    std::vector<char> active;  // stimuli currently summed into istim

    Scalars *sc_host = nullptr;   // pinned
    // end-of-chunk scalars: coherent pinned memory the device writes and the
    // host polls (pub_dev: its device address)
    Published *pub = nullptr, *pub_dev = nullptr;
    int32_t pub_seq = 0;
    double *stage = nullptr;      // pinned, npad doubles

    // learned warm start
    bool mlp_set = false;
    MlpNorm mlp_norm{{0.f, 0.f, 0.f, 0.f}, {1.f, 1.f, 1.f, 1.f}, 0.f};
    float *rec_X = nullptr, *rec_dV = nullptr;   // training-data recorder
    float *rec_y = nullptr;                      // and the network's in-step output
    bool kvp_valid = false;   // kvp holds (K V^{n-1})_i / K_ii of the current state

    // launch-shape tuning
    int max_groups = kMaxGroups;
    int spmv_max_groups = kPartialCap;   // one 256-row tile per workgroup up to 16.7M rows
    int iter_scheme = 0;
    int nt_mode = -1;   // non-temporal matrix loads: -1 by stream size, 0 never, 1 always
    bool compact_cols = true;   // per-step kernels read col16 when it exists

    // batched form: instances, each a contiguous row range starting on a
    // TILE boundary (a single-mesh context has one instance, rows [0, n))
    bool batched = false;
    int n_inst = 1;
    std::vector<int64_t> inst_node_ptr;   // original numbering, n_inst + 1
    std::vector<int64_t> inst_row0;       // internal rows, n_inst + 1 (last: npad)
    std::vector<int64_t> inst_nnz;
    std::vector<int32_t> tile_real;       // real rows of each tile
    int64_t nslots_lpr[4] = {0, 0, 0, 0}; // slots of the layouts lpr 1, 2, 4 and 4-entry chunks
    int fmt = 0;                          // iteration SpMV format: 0 sliced ELL, 1 CSR
    bool csr_built = false;
    int lpr = 1;                          // lanes per row of the iteration SpMV
    int lpr_built = 0;                    // layout in sptr_t / col_t / A32_t: 2, 4 (lanes
                                          // per row), 5 (4-entry chunks), 0 none
    int tpb_b = 1;                        // tiles per workgroup
    bool persistent = false;              // CG iterations in one persistent launch
    SegTiling pseg{};                     // its group table (all groups resident)
    SegTiling seg{};
    BScalars *bsc_host = nullptr;         // pinned, n_inst
    std::vector<int32_t> inst_iters_hist; // per step, n_inst each
    bool use_graph = false;
    hipStream_t own_stream = nullptr;
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;   // (iterations, rotation)

    // profiling: event pairs around the SpMV launches of every
    // `profile_every`-th step (0: off)
    int profile_every = 0;
    bool profiling = false;   // this step carries events
    std::vector<hipEvent_t> ev;

    // statistics
    int last_iters = 0;
    std::vector<int32_t> iters_hist;
    mdx_stats stats{};

    template <class T>
    T *dev(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    double *vec(int role) const { return dev<double>(L.vec[vb[role]]); }
};

namespace mdx {
namespace host {

struct BatchPtrs {
    SellView P;
    IterMatrix IM;
    const double *Mv, *Kv, *Av, *dinv;
    const float *dinv32;
    double *b, *s, *u, *part0, *part_pq, *part_rz;
    float *r32, *p32, *q32, *delta, *g32;
    BScalars *bsc;
};

mdx_status fail(mdx_ctx *c, mdx_status st, const char *fmt, ...);

void node_graph(int64_t n, int64_t m, int npe, const int32_t *tets, std::vector<int64_t> &ptr,
                std::vector<int32_t> &adj);
std::vector<int32_t> rcm(int64_t n, const std::vector<int64_t> &ptr, const std::vector<int32_t> &adj);
uint64_t hilbert_key(uint32_t x0, uint32_t x1, uint32_t x2, int bits);
void hilbert_order(const std::vector<double> &xyz, int64_t p0, int64_t p1,
                   std::vector<int32_t> &out);
void compact_columns(mdx_ctx *c);
SellView step_view(const mdx_ctx *c);
int64_t sell_slot(const mdx_ctx *c, int64_t r, int32_t colv);
void compute_layout(mdx_ctx *c);
mdx_status require_mesh(mdx_ctx *ctx);
mdx_status copy_vec_out(mdx_ctx *ctx, const double *dsrc, double *host);
mdx_status copy_vec_in(mdx_ctx *ctx, const double *host, double *ddst);
StepParams step_params(const mdx_ctx *c);
mdx_status wait_published(mdx_ctx *ctx, hipStream_t st, int32_t seq);
mdx_status update_stimulus(mdx_ctx *ctx, hipStream_t st, int64_t k, bool &any);
void release_graphs(mdx_ctx *ctx);
bool use_nt(const mdx_ctx *c, double bytes);
double slots(const mdx_ctx *c);
int64_t span_rows(const mdx_ctx *c);
const int32_t *row_mask(const mdx_ctx *c);
mdx_status build_groups(mdx_ctx *c, int tpb, std::vector<int4> &grp, std::vector<int32_t> &ig);
mdx_status install_persistent_groups(mdx_ctx *c);
mdx_status install_groups(mdx_ctx *c, int tpb);
std::vector<int64_t> lpr_slices(const mdx_ctx *c, int lpr);
mdx_status build_lpr_layout(mdx_ctx *c, int lpr);
std::vector<int64_t> v4_slices(const mdx_ctx *c);
mdx_status build_v4_layout(mdx_ctx *c);
mdx_status build_csr(mdx_ctx *c);
mdx_status set_iter_layout(mdx_ctx *c, int fmt, int lpr);
IterMatrix iter_matrix(const mdx_ctx *c);
mdx_status set_mesh_impl(mdx_ctx *ctx, int32_t n_inst, const int64_t *node_ptr, bool batched,
                         int64_t n_nodes, const double *xyz, double unit_conversion,
                         int64_t n_tets, const int32_t *elems, const int32_t *region,
                         const double *fibre, int npe = 4);
BatchPtrs batch_ptrs(mdx_ctx *c);
BParams batch_params(const mdx_ctx *c);
void launch_persistent(mdx_ctx *c, hipStream_t st, const BatchPtrs &q, const BParams &bp);
mdx_status persistent_fault(mdx_ctx *c);
void enqueue_batched_step(mdx_ctx *c, hipStream_t st, int iters, const double *istim, bool timed);
mdx_status fetch_bscalars(mdx_ctx *c, hipStream_t st);
bool all_done(const mdx_ctx *c);
mdx_status run_batched(mdx_ctx *ctx, int64_t n_steps, int64_t out_every, double *v_out);

}  // namespace host
}  // namespace mdx

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, MDX_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define GUARD_BEGIN try {
#define GUARD_END                                                              \
    }                                                                          \
    catch (const std::bad_alloc &) {                                           \
        return fail(ctx, MDX_ERR_INVALID_ARG, "host allocation failed");       \
    }                                                                          \
    catch (...) {                                                              \
        return fail(ctx, MDX_ERR_INVALID_ARG, "unexpected host exception");    \
    }
