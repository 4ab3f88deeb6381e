// Host side of the monodomain library: the C ABI of include/monox.h.
//
// Setup (host, once per mesh): validation, node adjacency, reverse
// Cuthill-McKee ordering (the paper reorders with RCM to shrink the matrix
// bandwidth, "Software implementation" section), the sliced-ELL pattern shared
// by M, K and A, and the slot map that lists, for every matrix slot, the
// (element, a, b) contributions in ascending element order.  Device setup
// (mdx_prepare): element matrices, deterministic gather into M and K,
// A = chi Cm M + theta dt K, the Jacobi diagonal, rest state.
//
// Time loop (mdx_run): per step the kernels of mdx_ionic.hip / mdx_solver.hip
// (mdx_mixed.hip, mdx_learned.hip for the forms) are queued on the context's
// stream; PCG iterations are queued in chunks (first chunk = last step's
// count).  A chunk ends with the guarded epilogue, a one-wave kernel that
// publishes the solver scalars to coherent pinned host memory with a
// sequence number, and the next step's ionic update guarded by the done flag;
// the host spins on the sequence number.  Kernels queued after convergence
// return at their first instruction.
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

using namespace mdx;

namespace {

constexpr int kMaxGroups = 2048;      // default cap on row-tiled workgroups
// matrix streams above this size are read with the non-temporal hint (they do
// not stay in the 256 MB Infinity Cache between products anyway)
constexpr double kStreamCacheBytes = 256.0 * 1024 * 1024;
constexpr int kPartialCap = 65536;    // partial slots per reduction (>= any cap)
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

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

}  // namespace

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

namespace {

mdx_status fail(mdx_ctx *c, mdx_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

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

// ---------------------------------------------------------------------------
// graph of the mesh: node -> neighbouring nodes (sharing an element), no
// self.  Elements are 4-id records of which the first npe ids are used.
// ---------------------------------------------------------------------------
void node_graph(int64_t n, int64_t m, int npe, const int32_t *tets, std::vector<int64_t> &ptr,
                std::vector<int32_t> &adj)
{
    std::vector<int64_t> tptr(n + 1, 0);
    for (int64_t e = 0; e < m; ++e)
        for (int a = 0; a < npe; ++a) tptr[tets[4 * e + a] + 1]++;
    for (int64_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
    std::vector<int32_t> tlist(tptr[n]);
    {
        std::vector<int64_t> pos(tptr.begin(), tptr.end() - 1);
        for (int64_t e = 0; e < m; ++e)
            for (int a = 0; a < npe; ++a) tlist[pos[tets[4 * e + a]]++] = (int32_t)e;
    }
    std::vector<int32_t> mark(n, -1);
    ptr.assign(n + 1, 0);
    adj.clear();
    adj.reserve((size_t)(14 * n));
    for (int64_t i = 0; i < n; ++i) {
        size_t row0 = adj.size();
        mark[i] = (int32_t)i;
        for (int64_t q = tptr[i]; q < tptr[i + 1]; ++q) {
            const int32_t *t = tets + 4 * (int64_t)tlist[q];
            for (int a = 0; a < npe; ++a)
                if (mark[t[a]] != (int32_t)i) {
                    mark[t[a]] = (int32_t)i;
                    adj.push_back(t[a]);
                }
        }
        std::sort(adj.begin() + row0, adj.end());
        ptr[i + 1] = (int64_t)adj.size();
    }
}

// Reverse Cuthill-McKee: per connected component, BFS from a pseudo-peripheral
// node (George-Liu search) visiting neighbours by increasing degree (ties by
// index); the concatenated order is reversed.  Returns perm[new] = old.
std::vector<int32_t> rcm(int64_t n, const std::vector<int64_t> &ptr, const std::vector<int32_t> &adj)
{
    auto deg = [&](int32_t v) { return ptr[v + 1] - ptr[v]; };
    std::vector<int32_t> order;
    order.reserve(n);
    std::vector<char> placed(n, 0);
    std::vector<int32_t> level(n, -1), queue;
    queue.reserve(n);
    std::vector<int32_t> touched;

    // BFS levels from root; returns eccentricity and the last level's nodes
    auto bfs_levels = [&](int32_t root, std::vector<int32_t> &last) {
        for (int32_t v : touched) level[v] = -1;
        touched.clear();
        queue.clear();
        queue.push_back(root);
        level[root] = 0;
        touched.push_back(root);
        size_t head = 0;
        int ecc = 0;
        while (head < queue.size()) {
            int32_t v = queue[head++];
            ecc = std::max(ecc, level[v]);
            for (int64_t q = ptr[v]; q < ptr[v + 1]; ++q) {
                int32_t w = adj[q];
                if (level[w] < 0) {
                    level[w] = level[v] + 1;
                    touched.push_back(w);
                    queue.push_back(w);
                }
            }
        }
        last.clear();
        for (int32_t v : queue)
            if (level[v] == ecc) last.push_back(v);
        return ecc;
    };

    std::vector<int32_t> last, nbr;
    for (int64_t s = 0; s < n; ++s) {
        if (placed[s]) continue;
        int32_t root = (int32_t)s;
        int ecc = bfs_levels(root, last);
        for (int guard = 0; guard < 64; ++guard) {
            int32_t cand = last[0];
            for (int32_t v : last)
                if (deg(v) < deg(cand) || (deg(v) == deg(cand) && v < cand)) cand = v;
            std::vector<int32_t> last2;
            int e2 = bfs_levels(cand, last2);
            if (e2 > ecc) {
                root = cand;
                ecc = e2;
                last.swap(last2);
            } else {
                break;
            }
        }
        // Cuthill-McKee BFS from root
        size_t head = order.size();
        order.push_back(root);
        placed[root] = 1;
        while (head < order.size()) {
            int32_t v = order[head++];
            nbr.clear();
            for (int64_t q = ptr[v]; q < ptr[v + 1]; ++q)
                if (!placed[adj[q]]) nbr.push_back(adj[q]);
            std::sort(nbr.begin(), nbr.end(), [&](int32_t a, int32_t b) {
                return deg(a) < deg(b) || (deg(a) == deg(b) && a < b);
            });
            for (int32_t w : nbr) {
                placed[w] = 1;
                order.push_back(w);
            }
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

// Position of a point on the 3-D Hilbert curve of order `bits` (Skilling's
// transform of the axes to the transposed Hilbert index, then bit
// interleaving): points close on the curve are close in space, so a run of
// consecutive nodes is a compact patch of the mesh.
uint64_t hilbert_key(uint32_t x0, uint32_t x1, uint32_t x2, int bits)
{
    uint32_t X[3] = {x0, x1, x2};
    const uint32_t M = 1u << (bits - 1);
    // inverse undo of the excess work
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    // Gray encode
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    uint64_t h = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int i = 0; i < 3; ++i) h = (h << 1) | ((X[i] >> b) & 1u);
    return h;
}

// nodes [p0, p1) sorted by the Hilbert key of their coordinates in the
// bounding box of that range (2^10 cells per axis)
void hilbert_order(const std::vector<double> &xyz, int64_t p0, int64_t p1,
                   std::vector<int32_t> &out)
{
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t v = p0; v < p1; ++v)
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], xyz[3 * v + k]);
            hi[k] = std::max(hi[k], xyz[3 * v + k]);
        }
    const int bits = 10;
    const double cells = (double)((1u << bits) - 1);
    double ext = 0.0;
    for (int k = 0; k < 3; ++k) ext = std::max(ext, hi[k] - lo[k]);
    const double sc = ext > 0.0 ? cells / ext : 0.0;
    std::vector<std::pair<uint64_t, int32_t>> key((size_t)(p1 - p0));
    for (int64_t v = p0; v < p1; ++v) {
        uint32_t c[3];
        for (int k = 0; k < 3; ++k)
            c[k] = (uint32_t)std::min(cells, std::max(0.0, (xyz[3 * v + k] - lo[k]) * sc));
        key[v - p0] = {hilbert_key(c[0], c[1], c[2], bits), (int32_t)v};
    }
    std::sort(key.begin(), key.end());
    for (auto &kv : key) out.push_back(kv.second);
}

// 16-bit column offsets from each slice's smallest column, when every
// slice's columns span fewer than 2^16 indices
void compact_columns(mdx_ctx *c)
{
    c->col16.clear();
    c->cbase.clear();
    std::vector<int32_t> base(c->nslices);
    for (int64_t sl = 0; sl < c->nslices; ++sl) {
        int32_t lo = INT32_MAX, hi = -1;
        for (int64_t e = c->slice_ptr[sl]; e < c->slice_ptr[sl + 1]; ++e) {
            lo = std::min(lo, c->col_sell[e]);
            hi = std::max(hi, c->col_sell[e]);
        }
        if (hi < 0) lo = 0;
        if ((int64_t)hi - lo >= 65536) return;
        base[sl] = lo;
    }
    std::vector<uint16_t> off(c->col_sell.size());
    for (int64_t sl = 0; sl < c->nslices; ++sl)
        for (int64_t e = c->slice_ptr[sl]; e < c->slice_ptr[sl + 1]; ++e)
            off[e] = (uint16_t)(c->col_sell[e] - base[sl]);
    c->col16.swap(off);
    c->cbase.swap(base);
}

// the pattern as the per-step kernels read it
SellView step_view(const mdx_ctx *c)
{
    SellView P{c->dev<int64_t>(c->L.slice_ptr), c->dev<int32_t>(c->L.col)};
    if (c->compact_cols && !c->col16.empty()) {
        P.col16 = c->dev<uint16_t>(c->L.col16);
        P.cbase = c->dev<int32_t>(c->L.cbase);
    }
    return P;
}

// position of column c in new-row r of the sliced-ELL pattern, or -1
int64_t sell_slot(const mdx_ctx *c, int64_t r, int32_t colv)
{
    int64_t base = c->slice_ptr[r / SLICE] + (r % SLICE);
    int lo = 0, hi = c->rowlen[r] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        int32_t v = c->col_sell[base + (int64_t)mid * SLICE];
        if (v == colv) return base + (int64_t)mid * SLICE;
        if (v < colv) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

void compute_layout(mdx_ctx *c)
{
    Layout &L = c->L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    const size_t np = (size_t)c->npad, ns = (size_t)c->nslots;
    L.slice_ptr = take(sizeof(int64_t) * (c->nslices + 1));
    L.col = take(sizeof(int32_t) * ns);
    L.col16 = take(sizeof(uint16_t) * std::max<size_t>(c->col16.size(), 1));
    L.cbase = take(sizeof(int32_t) * std::max<size_t>(c->cbase.size(), 1));
    L.Mv = take(sizeof(double) * ns);
    L.Kv = take(sizeof(double) * ns);
    L.Av = take(sizeof(double) * ns);
    L.dinv = take(sizeof(double) * np);
    for (int i = 0; i < 3; ++i) L.vec[i] = take(sizeof(double) * np);
    L.r = take(sizeof(double) * np);
    L.p = take(sizeof(double) * np);
    L.p2 = take(sizeof(double) * np);
    L.q = take(sizeof(double) * np);
    L.b = take(sizeof(double) * np);
    L.s = take(sizeof(double) * np);
    L.istim = take(sizeof(double) * np);
    L.u = take(sizeof(double) * np * std::max(1, ionic_nstates(c->ionic_kind)));
    L.lat = take(sizeof(double) * np);
    L.lrt = take(sizeof(double) * np);
    size_t nst = 0;
    for (auto &s : c->stims) nst += s.nodes.size();
    L.stim_idx = take(sizeof(int32_t) * std::max<size_t>(nst, 1));
    L.partial = take(sizeof(double) * 3 * 3 * kPartialCap);
    L.scalars = take(sizeof(Scalars));
    L.A32 = take(sizeof(float) * ns);
    L.dinv32 = take(sizeof(float) * np);
    L.r32 = take(sizeof(float) * np);
    L.z32 = take(sizeof(float) * np);
    L.p32 = take(sizeof(float) * np);
    L.q32 = take(sizeof(float) * np);
    L.delta = take(sizeof(float) * np);
    L.g32 = take(sizeof(float) * np * std::max(1, ionic_gate_rows(c->ionic_kind)));
    L.kdiag = take(sizeof(double) * np);
    L.kvp = take(sizeof(float) * np);
    L.feat = take(sizeof(float) * 4 * np);
    L.mlp_y = take(sizeof(float) * np);
    L.mlp_params = take(sizeof(float) * mlp_nparams());
    {
        const size_t n_tiles = np / TILE, ni = (size_t)c->n_inst;
        L.tile_real = take(sizeof(int32_t) * n_tiles);
        L.grp = take(sizeof(int4) * (n_tiles + ni));
        L.inst_grp = take(sizeof(int32_t) * (ni + 1));
        L.pgrp = take(sizeof(int4) * (n_tiles + ni));
        L.pinst_grp = take(sizeof(int32_t) * (ni + 1));
        L.pbar = take(sizeof(uint32_t) * (ni + 1));
        L.bsc = take(sizeof(BScalars) * ni);
        const size_t alt =
            c->batched ? (size_t)std::max({c->nslots_lpr[1], c->nslots_lpr[2], c->nslots_lpr[3]}) : 1;
        L.sptr_t = take(sizeof(int64_t) * (c->batched ? np / (SLICE / 4) + 1 : 1));
        L.col_t = take(sizeof(int32_t) * alt);
        L.A32_t = take(sizeof(float) * alt);
        const size_t cnz = c->batched ? (size_t)c->nnz : 1;
        L.csr_ptr = take(sizeof(int32_t) * (c->batched ? np + 1 : 1));
        L.csr_col = take(sizeof(int32_t) * cnz);
        L.csr_val = take(sizeof(float) * cnz);
        L.gv = take(sizeof(double) * 4 * (c->batched ? np : 1));
    }
    L.total = o;

    o = 0;
    const size_t m = (size_t)c->m, n = (size_t)c->n;
    L.x_xyz = take(sizeof(double) * 3 * n);
    L.x_tets = take(sizeof(int32_t) * 4 * m);
    L.x_fibre = take(sizeof(double) * 3 * (c->fibre.empty() ? 1 : m));
    L.x_sig = take(sizeof(double) * 2 * m);
    L.x_vol = take(sizeof(double) * m);
    L.x_ek = take(sizeof(double) * 16 * m);
    L.x_cptr = take(sizeof(int64_t) * (ns + 1));
    L.x_contrib = take(sizeof(int32_t) * 16 * m);
    L.x_total = o;
}

mdx_status require_mesh(mdx_ctx *ctx)
{
    if (ctx->n <= 0) return fail(ctx, MDX_ERR_STATE, "no mesh set");
    return MDX_OK;
}

mdx_status copy_vec_out(mdx_ctx *ctx, const double *dsrc, double *host)
{
    HIPCHK(hipMemcpyAsync(ctx->stage, dsrc, sizeof(double) * ctx->npad, hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int64_t i = 0; i < ctx->n; ++i) host[i] = ctx->stage[ctx->iperm[i]];
    return MDX_OK;
}

mdx_status copy_vec_in(mdx_ctx *ctx, const double *host, double *ddst)
{
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int64_t r = 0; r < ctx->npad; ++r)
        ctx->stage[r] = ctx->perm[r] >= 0 ? host[ctx->perm[r]] : 0.0;
    HIPCHK(hipMemcpyAsync(ddst, ctx->stage, sizeof(double) * ctx->npad, hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MDX_OK;
}

StepParams step_params(const mdx_ctx *c)
{
    StepParams sp;
    sp.chi = c->chi;
    sp.cm = c->cm;
    sp.theta = c->theta;
    sp.dt = c->dt;
    sp.warm_start = c->opts.warm_start;
    sp.rel_mode = c->opts.rel_mode;
    return sp;
}

// Rebuild istim if the set of stimuli active at step k changed.
// Wait for the publish numbered seq and copy the scalars it carries to
// sc_host.  The host spins on the sequence number (no blocking sync, no copy
// kernel); should the stream drain without it, the memory is not coherent as
// promised and the call fails.
mdx_status wait_published(mdx_ctx *ctx, hipStream_t st, int32_t seq)
{
    for (uint64_t n = 1; ctx->pub->seq != seq; ++n) {
        if (n % 1024 == 0) {
            const hipError_t q = hipStreamQuery(st);
            if (q == hipSuccess) {
                std::atomic_thread_fence(std::memory_order_seq_cst);
                if (ctx->pub->seq == seq) break;
                return fail(ctx, MDX_ERR_DEVICE, "published solver scalars not visible on the host");
            }
            if (q != hipErrorNotReady) HIPCHK(q);
        }
        __builtin_ia32_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    std::memcpy(ctx->sc_host, (const void *)&ctx->pub->s, sizeof(Scalars));
    return MDX_OK;
}

mdx_status update_stimulus(mdx_ctx *ctx, hipStream_t st, int64_t k, bool &any)
{
    std::vector<char> want(ctx->stims.size(), 0);
    any = false;
    for (size_t s = 0; s < ctx->stims.size(); ++s) {
        const Stim &st = ctx->stims[s];
        int64_t ks = std::llround(st.start / ctx->dt);
        int64_t ke = std::llround((st.start + st.duration) / ctx->dt);
        want[s] = (k >= ks && k < ke) ? 1 : 0;
        any = any || want[s];
    }
    if (want == ctx->active) return MDX_OK;
    double *istim = ctx->dev<double>(ctx->L.istim);
    launch_fill(st, ctx->npad, 0.0, istim);
    for (size_t s = 0; s < ctx->stims.size(); ++s)
        if (want[s])
            launch_stim_add(st, (int64_t)ctx->stims[s].nodes.size(),
                            ctx->dev<int32_t>(ctx->L.stim_idx) + ctx->stim_off[s],
                            ctx->stims[s].amp, istim);
    HIPCHK(hipGetLastError());
    ctx->active = want;
    return MDX_OK;
}

void release_graphs(mdx_ctx *ctx)
{
    for (auto &kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
    ctx->graphs.clear();
}

// non-temporal hint for a kernel whose matrix streams total `bytes`
bool use_nt(const mdx_ctx *c, double bytes)
{
    return c->nt_mode < 0 ? bytes > kStreamCacheBytes : c->nt_mode != 0;
}
double slots(const mdx_ctx *c) { return (double)c->nslots; }

// rows covered by the pointwise kernels and their padding mask: the real
// rows are a prefix in a single-mesh context and interleaved with padding
// (masked per tile) in a batched one
int64_t span_rows(const mdx_ctx *c) { return c->batched ? c->npad : c->n; }
const int32_t *row_mask(const mdx_ctx *c)
{
    return c->batched ? c->dev<int32_t>(c->L.tile_real) : nullptr;
}

// group table of the segmented kernels: instance i's tiles in runs of tpb
mdx_status build_groups(mdx_ctx *c, int tpb, std::vector<int4> &grp, std::vector<int32_t> &ig)
{
    grp.clear();
    ig.assign(c->n_inst + 1, 0);
    for (int i = 0; i < c->n_inst; ++i) {
        ig[i] = (int32_t)grp.size();
        const int t0 = (int)(c->inst_row0[i] / TILE), t1 = (int)(c->inst_row0[i + 1] / TILE);
        for (int t = t0; t < t1; t += tpb) grp.push_back(make_int4(i, t, std::min(t + tpb, t1), 0));
    }
    ig[c->n_inst] = (int32_t)grp.size();
    if ((int64_t)grp.size() > kPartialCap)
        return fail(c, MDX_ERR_INVALID_ARG, "%zu workgroups exceed %d: use more tiles per group",
                    grp.size(), kPartialCap);
    return MDX_OK;
}

// Group table of the persistent iteration: the fewest tiles per group for
// which every group can be resident at once.
mdx_status install_persistent_groups(mdx_ctx *c)
{
    mdx_ctx *ctx = c;   // for HIPCHK
    const int cap = persistent_capacity(c->device);
    if (cap <= 0) return fail(c, MDX_ERR_DEVICE, "occupancy query of the persistent kernel failed");
    std::vector<int4> grp;
    std::vector<int32_t> ig;
    int tpb = 1;
    for (;; ++tpb) {
        if (mdx_status e = build_groups(c, tpb, grp, ig)) return e;
        if ((int)grp.size() <= cap) break;
    }
    HIPCHK(hipMemcpyAsync(c->dev<int4>(c->L.pgrp), grp.data(), sizeof(int4) * grp.size(),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->dev<int32_t>(c->L.pinst_grp), ig.data(), sizeof(int32_t) * ig.size(),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->pseg.groups = (int)grp.size();
    c->pseg.n_inst = c->n_inst;
    c->pseg.grp = c->dev<int4>(c->L.pgrp);
    c->pseg.inst_grp = c->dev<int32_t>(c->L.pinst_grp);
    return MDX_OK;
}

mdx_status install_groups(mdx_ctx *c, int tpb)
{
    mdx_ctx *ctx = c;   // for HIPCHK
    std::vector<int4> grp;
    std::vector<int32_t> ig;
    if (mdx_status e = build_groups(c, tpb, grp, ig)) return e;
    HIPCHK(hipMemcpyAsync(c->dev<int4>(c->L.grp), grp.data(), sizeof(int4) * grp.size(),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->dev<int32_t>(c->L.inst_grp), ig.data(), sizeof(int32_t) * ig.size(),
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->seg.groups = (int)grp.size();
    c->seg.n_inst = c->n_inst;
    c->seg.grp = c->dev<int4>(c->L.grp);
    c->seg.inst_grp = c->dev<int32_t>(c->L.inst_grp);
    c->tpb_b = tpb;
    release_graphs(c);
    return MDX_OK;
}

// slice pointers of the lanes-per-row layout lpr (2 or 4)
std::vector<int64_t> lpr_slices(const mdx_ctx *c, int lpr)
{
    const int H = SLICE / lpr;
    const int64_t ns = c->npad / H;
    std::vector<int64_t> sp(ns + 1, 0);
    for (int64_t sl = 0; sl < ns; ++sl) {
        int w = 0;
        for (int l = 0; l < H; ++l) w = std::max(w, (c->rowlen[sl * H + l] + lpr - 1) / lpr);
        sp[sl + 1] = sp[sl] + (int64_t)w * SLICE;
    }
    return sp;
}

// build the iteration matrix in layout lpr (2 or 4) into the alternative
// arrays; lpr = 1 is the base layout and needs nothing
mdx_status build_lpr_layout(mdx_ctx *c, int lpr)
{
    mdx_ctx *ctx = c;   // for HIPCHK
    if (lpr == 1 || c->lpr_built == lpr) return MDX_OK;
    std::vector<int64_t> sp = lpr_slices(c, lpr);
    const int li = lpr == 2 ? 1 : 2;
    if (sp.back() != c->nslots_lpr[li] || (int64_t)sp.size() - 1 != c->npad / (SLICE / lpr))
        return fail(c, MDX_ERR_STATE, "internal layout inconsistent (lanes per row %d)", lpr);
    HIPCHK(hipMemcpyAsync(c->dev<int64_t>(c->L.sptr_t), sp.data(), sizeof(int64_t) * sp.size(),
                          hipMemcpyHostToDevice, c->stream));
    SellView base{c->dev<int64_t>(c->L.slice_ptr), c->dev<int32_t>(c->L.col)};
    launch_relayout(c->stream, lpr, (int64_t)sp.size() - 1, c->dev<int64_t>(c->L.sptr_t), base,
                    c->dev<float>(c->L.A32), c->dev<int32_t>(c->L.col_t), c->dev<float>(c->L.A32_t));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->lpr_built = lpr;
    return MDX_OK;
}

// slice pointers of the 4-entry-chunk layout: widths rounded up to 4
std::vector<int64_t> v4_slices(const mdx_ctx *c)
{
    const int64_t ns = c->npad / SLICE;
    std::vector<int64_t> sp(ns + 1, 0);
    for (int64_t sl = 0; sl < ns; ++sl) {
        const int64_t w = (c->slice_ptr[sl + 1] - c->slice_ptr[sl]) / SLICE;
        sp[sl + 1] = sp[sl] + (w + 3) / 4 * 4 * SLICE;
    }
    return sp;
}

mdx_status build_v4_layout(mdx_ctx *c)
{
    mdx_ctx *ctx = c;   // for HIPCHK
    if (c->lpr_built == 5) return MDX_OK;
    std::vector<int64_t> sp = v4_slices(c);
    if (sp.back() != c->nslots_lpr[3])
        return fail(c, MDX_ERR_STATE, "internal layout inconsistent (4-entry chunks)");
    HIPCHK(hipMemcpyAsync(c->dev<int64_t>(c->L.sptr_t), sp.data(), sizeof(int64_t) * sp.size(),
                          hipMemcpyHostToDevice, c->stream));
    SellView base{c->dev<int64_t>(c->L.slice_ptr), c->dev<int32_t>(c->L.col)};
    launch_relayout_v4(c->stream, (int64_t)sp.size() - 1, c->dev<int64_t>(c->L.sptr_t), base,
                       c->dev<float>(c->L.A32), c->dev<int32_t>(c->L.col_t),
                       c->dev<float>(c->L.A32_t));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->lpr_built = 5;
    return MDX_OK;
}

// CSR copy of the FP32 iteration matrix (real entries only)
mdx_status build_csr(mdx_ctx *c)
{
    mdx_ctx *ctx = c;   // for HIPCHK
    if (c->csr_built) return MDX_OK;
    if (c->nnz >= ((int64_t)1 << 31)) return fail(c, MDX_ERR_UNSUPPORTED, "CSR needs nnz < 2^31");
    std::vector<int32_t> rp(c->npad + 1, 0);
    for (int64_t r = 0; r < c->npad; ++r) rp[r + 1] = rp[r] + c->rowlen[r];
    if (rp[c->npad] != c->nnz) return fail(c, MDX_ERR_STATE, "internal layout inconsistent (CSR)");
    HIPCHK(hipMemcpyAsync(c->dev<int32_t>(c->L.csr_ptr), rp.data(), sizeof(int32_t) * rp.size(),
                          hipMemcpyHostToDevice, c->stream));
    SellView base{c->dev<int64_t>(c->L.slice_ptr), c->dev<int32_t>(c->L.col)};
    launch_build_csr(c->stream, c->npad, base, c->dev<float>(c->L.A32), c->dev<int32_t>(c->L.csr_ptr),
                     c->dev<int32_t>(c->L.csr_col), c->dev<float>(c->L.csr_val));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->csr_built = true;
    return MDX_OK;
}

// install format / lanes per row for the iteration SpMV (building its arrays)
mdx_status set_iter_layout(mdx_ctx *c, int fmt, int lpr)
{
    if (fmt == 0 && lpr != 1 && lpr != 2 && lpr != 4)
        return fail(c, MDX_ERR_INVALID_ARG, "sliced ELL takes 1, 2 or 4 lanes per row");
    if (fmt == 1 && lpr != 4 && lpr != 8 && lpr != 16)
        return fail(c, MDX_ERR_INVALID_ARG, "CSR takes 4, 8 or 16 lanes per row");
    if (fmt >= 2 && lpr != 1)
        return fail(c, MDX_ERR_INVALID_ARG, "4-entry-chunk layouts take 1 lane per row");
    if (fmt == 0) {
        if (mdx_status e = build_lpr_layout(c, lpr)) return e;
    } else if (fmt == 1) {
        if (mdx_status e = build_csr(c)) return e;
    } else {
        if (mdx_status e = build_v4_layout(c)) return e;
    }
    c->fmt = fmt;
    c->lpr = lpr;
    release_graphs(c);
    return MDX_OK;
}

IterMatrix iter_matrix(const mdx_ctx *c)
{
    const Layout &L = c->L;
    IterMatrix A{};
    A.format = c->fmt;
    A.lpr = c->lpr;
    A.nt = use_nt(c, 8.0 * slots(c));
    if (c->fmt == 1) {
        A.rptr = c->dev<int32_t>(L.csr_ptr);
        A.col = c->dev<int32_t>(L.csr_col);
        A.val = c->dev<float>(L.csr_val);
    } else if (c->lpr == 1 && c->fmt == 0) {
        A.sptr = c->dev<int64_t>(L.slice_ptr);
        A.col = c->dev<int32_t>(L.col);
        A.val = c->dev<float>(L.A32);
    } else {
        A.sptr = c->dev<int64_t>(L.sptr_t);
        A.col = c->dev<int32_t>(L.col_t);
        A.val = c->dev<float>(L.A32_t);
    }
    return A;
}

// npe: vertex ids per element in the caller's array (4 tetrahedra, 3 surface
// triangles); inside, every element is a 4-id record (-1 after a triangle's 3)
mdx_status set_mesh_impl(mdx_ctx *ctx, int32_t n_inst, const int64_t *node_ptr, bool batched,
                         int64_t n_nodes, const double *xyz, double unit_conversion,
                         int64_t n_tets, const int32_t *elems, const int32_t *region,
                         const double *fibre, int npe = 4)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    GUARD_BEGIN
    if (n_nodes <= 0 || n_tets <= 0 || !xyz || !elems)
        return fail(ctx, MDX_ERR_INVALID_ARG, "empty mesh or null array");
    if (n_nodes >= (int64_t)1 << 31 || n_tets >= (int64_t)1 << 27)
        return fail(ctx, MDX_ERR_INVALID_ARG, "mesh too large (n < 2^31, tets < 2^27)");
    if (!(unit_conversion > 0.0) || !std::isfinite(unit_conversion))
        return fail(ctx, MDX_ERR_INVALID_ARG, "unit_conversion must be finite and > 0");
    for (int64_t i = 0; i < 3 * n_nodes; ++i)
        if (!std::isfinite(xyz[i]))
            return fail(ctx, MDX_ERR_INVALID_ARG, "non-finite coordinate at node %lld",
                        (long long)(i / 3));
    for (int64_t q = 0; q < npe * n_tets; ++q)
        if (elems[q] < 0 || elems[q] >= n_nodes)
            return fail(ctx, MDX_ERR_BAD_MESH, "element %lld references node %d out of range",
                        (long long)(q / npe), elems[q]);
    std::vector<int32_t> tv((size_t)(4 * n_tets), -1);
    for (int64_t e = 0; e < n_tets; ++e)
        for (int a = 0; a < npe; ++a) tv[4 * e + a] = elems[npe * e + a];
    const int32_t *tets = tv.data();
    if (node_ptr[0] != 0 || node_ptr[n_inst] != n_nodes)
        return fail(ctx, MDX_ERR_INVALID_ARG, "node_ptr must run from 0 to n_nodes");
    for (int32_t i = 0; i < n_inst; ++i)
        if (node_ptr[i + 1] <= node_ptr[i])
            return fail(ctx, MDX_ERR_INVALID_ARG, "instance %d has no nodes", i);
    std::vector<int32_t> inst_of(n_nodes);
    for (int32_t i = 0; i < n_inst; ++i)
        std::fill(inst_of.begin() + node_ptr[i], inst_of.begin() + node_ptr[i + 1], i);
    for (int64_t e = 0; e < n_tets; ++e)
        for (int a = 1; a < npe; ++a)
            if (inst_of[tets[4 * e + a]] != inst_of[tets[4 * e]])
                return fail(ctx, MDX_ERR_BAD_MESH, "element %lld joins two instances",
                            (long long)e);
    if (fibre)
        for (int64_t q = 0; q < 3 * n_tets; ++q)
            if (!std::isfinite(fibre[q]))
                return fail(ctx, MDX_ERR_INVALID_ARG, "non-finite fibre at element %lld",
                            (long long)(q / 3));
    std::vector<double> X(xyz, xyz + 3 * n_nodes);
    for (double &v : X) v /= unit_conversion;
    // element quality: tetrahedra |det J| > 1e-14 h^3, triangles
    // |(x1 - x0) x (x2 - x0)| > 1e-14 h^2
    for (int64_t e = 0; e < n_tets; ++e) {
        const int32_t *t = tets + 4 * e;
        double d[3][3] = {}, h2 = 0.0;
        for (int a = 1; a < npe; ++a)
            for (int k = 0; k < 3; ++k) d[a - 1][k] = X[3 * t[a] + k] - X[3 * t[0] + k];
        for (int a = 0; a < npe; ++a)
            for (int b = a + 1; b < npe; ++b) {
                double s = 0.0;
                for (int k = 0; k < 3; ++k) {
                    double w = X[3 * t[a] + k] - X[3 * t[b] + k];
                    s += w * w;
                }
                h2 = std::max(h2, s);
            }
        if (npe == 3) {
            const double cx = d[0][1] * d[1][2] - d[0][2] * d[1][1];
            const double cy = d[0][2] * d[1][0] - d[0][0] * d[1][2];
            const double cz = d[0][0] * d[1][1] - d[0][1] * d[1][0];
            const double c2 = std::sqrt(cx * cx + cy * cy + cz * cz);
            if (!(c2 > 1e-14 * h2))
                return fail(ctx, MDX_ERR_BAD_MESH, "degenerate element %lld (2 area = %g)",
                            (long long)e, c2);
            continue;
        }
        double det = d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) -
                     d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0]) +
                     d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0]);
        double h3 = h2 * std::sqrt(h2);
        if (!(std::fabs(det) > 1e-14 * h3))
            return fail(ctx, MDX_ERR_BAD_MESH, "degenerate element %lld (|det J| = %g)",
                        (long long)e, std::fabs(det));
    }

    // adjacency; node order: one mesh by reverse Cuthill-McKee (a narrow band,
    // which on structured grids also keeps each wavefront's gathers in few
    // cache lines); a batch instance by instance along the Hilbert curve
    // (unstructured meshes: the gathers of a wavefront's rows stay in fewer
    // cache lines than in a level-by-level order)
    std::vector<int64_t> gptr;
    std::vector<int32_t> gadj;
    node_graph(n_nodes, n_tets, npe, tets, gptr, gadj);
    std::vector<int32_t> order;
    if (batched) {
        order.reserve(n_nodes);
        for (int32_t i = 0; i < n_inst; ++i) hilbert_order(X, node_ptr[i], node_ptr[i + 1], order);
    } else {
        order = rcm(n_nodes, gptr, gadj);
    }
    std::vector<int64_t> row0(n_inst + 1, 0);
    for (int32_t i = 0; i < n_inst; ++i)
        row0[i + 1] = row0[i] + (node_ptr[i + 1] - node_ptr[i] + TILE - 1) / TILE * TILE;
    const int64_t npad = row0[n_inst];
    if (npad >= ((int64_t)1 << 31))
        return fail(ctx, MDX_ERR_INVALID_ARG, "padded row count exceeds 2^31");
    std::vector<int32_t> perm(npad, -1), iperm(n_nodes);
    {
        int64_t q = 0;
        for (int32_t i = 0; i < n_inst; ++i)
            for (int64_t k = 0; k < node_ptr[i + 1] - node_ptr[i]; ++k) perm[row0[i] + k] = order[q++];
    }
    order.clear();
    order.shrink_to_fit();
    if (batched) {
        // irregular meshes: rows sorted by length (longest first) inside each
        // 256-row tile, so the 64-row slices hold rows of similar length and
        // the sliced layout pads little; padding rows stay at the tile's end
        auto deg = [&](int32_t o) { return gptr[o + 1] - gptr[o]; };
        for (int64_t t0 = 0; t0 < npad; t0 += TILE) {
            int64_t t1 = t0;
            while (t1 < t0 + TILE && perm[t1] >= 0) ++t1;
            std::stable_sort(perm.begin() + t0, perm.begin() + t1,
                             [&](int32_t a, int32_t b) { return deg(a) > deg(b); });
        }
    }
    for (int64_t r = 0; r < npad; ++r)
        if (perm[r] >= 0) iperm[perm[r]] = (int32_t)r;
    std::vector<int32_t> tile_real(npad / TILE, 0);
    for (int64_t r = 0; r < npad; ++r)
        if (perm[r] >= 0) tile_real[r / TILE]++;

    // sliced-ELL pattern over the padded rows (padding rows are empty)
    const int64_t nslices = npad / SLICE;
    std::vector<int32_t> rowlen(npad, 0);
    std::vector<int64_t> inst_nnz(n_inst, 0);
    int64_t nnz = 0, bw = 0;
    for (int32_t i = 0; i < n_inst; ++i)
        for (int64_t r = row0[i]; r < row0[i + 1]; ++r)
            if (perm[r] >= 0) {
                const int32_t o = perm[r];
                rowlen[r] = (int32_t)(gptr[o + 1] - gptr[o] + 1);
                nnz += rowlen[r];
                inst_nnz[i] += rowlen[r];
            }
    std::vector<int64_t> sptr(nslices + 1, 0);
    for (int64_t sl = 0; sl < nslices; ++sl) {
        int w = 0;
        for (int l = 0; l < SLICE; ++l) w = std::max(w, rowlen[sl * SLICE + l]);
        sptr[sl + 1] = sptr[sl] + (int64_t)w * SLICE;
    }
    std::vector<int32_t> colv(sptr[nslices]);
    std::vector<int32_t> cols;
    for (int64_t r = 0; r < npad; ++r) {
        int64_t base = sptr[r / SLICE] + (r % SLICE);
        int64_t w = (sptr[r / SLICE + 1] - sptr[r / SLICE]) / SLICE;
        cols.clear();
        if (perm[r] >= 0) {
            int32_t o = perm[r];
            cols.push_back((int32_t)r);
            for (int64_t q = gptr[o]; q < gptr[o + 1]; ++q) cols.push_back(iperm[gadj[q]]);
            std::sort(cols.begin(), cols.end());
            for (int32_t c : cols) bw = std::max<int64_t>(bw, std::llabs((long long)c - r));
        }
        for (int64_t j = 0; j < w; ++j)
            colv[base + j * SLICE] = j < (int64_t)cols.size() ? cols[j] : (int32_t)r;
    }
    // slot counts of the 2- and 4-lanes-per-row layouts (autotuner candidates)
    int64_t nsl[4] = {sptr[nslices], 0, 0, 0};
    if (batched) {
        for (int64_t sl = 0; sl < nslices; ++sl)
            nsl[3] += ((sptr[sl + 1] - sptr[sl]) / SLICE + 3) / 4 * 4 * SLICE;
        for (int li = 1; li < 3; ++li) {
            const int lpr = 1 << li, H = SLICE / lpr;
            int64_t tot = 0;
            for (int64_t sl = 0; sl < npad / H; ++sl) {
                int w = 0;
                for (int l = 0; l < H; ++l) w = std::max(w, (rowlen[sl * H + l] + lpr - 1) / lpr);
                tot += (int64_t)w * SLICE;
            }
            nsl[li] = tot;
        }
    }

    ctx->n = n_nodes;
    ctx->m = n_tets;
    ctx->npe = npe;
    ctx->xyz.swap(X);
    ctx->tets.swap(tv);
    ctx->region.assign(n_tets, 0);
    if (region) ctx->region.assign(region, region + n_tets);
    ctx->fibre.clear();
    if (fibre) ctx->fibre.assign(fibre, fibre + 3 * n_tets);
    ctx->perm.swap(perm);
    ctx->iperm.swap(iperm);
    ctx->npad = npad;
    ctx->nslices = nslices;
    ctx->nslots = sptr[nslices];
    ctx->nnz = nnz;
    ctx->bandwidth = bw;
    ctx->slice_ptr.swap(sptr);
    ctx->col_sell.swap(colv);
    ctx->rowlen.swap(rowlen);
    compact_columns(ctx);
    ctx->batched = batched;
    ctx->n_inst = n_inst;
    ctx->inst_node_ptr.assign(node_ptr, node_ptr + n_inst + 1);
    ctx->inst_row0.swap(row0);
    ctx->inst_nnz.swap(inst_nnz);
    ctx->tile_real.swap(tile_real);
    for (int li = 0; li < 4; ++li) ctx->nslots_lpr[li] = nsl[li];
    ctx->fmt = 0;
    ctx->lpr = 1;
    ctx->lpr_built = 0;
    ctx->csr_built = false;
    release_graphs(ctx);
    ctx->stims.clear();
    ctx->prepared = false;
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    return MDX_OK;
    GUARD_END
}


// ---------------------------------------------------------------------------
// batched form: one time step's work up to the host check
// ---------------------------------------------------------------------------
struct BatchPtrs {
    SellView P;
    IterMatrix IM;
    const double *Mv, *Kv, *Av, *dinv;
    const float *dinv32;
    double *b, *s, *u, *part0, *part_pq, *part_rz;
    float *r32, *p32, *q32, *delta, *g32;
    BScalars *bsc;
};

BatchPtrs batch_ptrs(mdx_ctx *c)
{
    const Layout &L = c->L;
    BatchPtrs q;
    q.P = SellView{c->dev<int64_t>(L.slice_ptr), c->dev<int32_t>(L.col)};
    q.IM = iter_matrix(c);
    q.Mv = c->dev<double>(L.Mv);
    q.Kv = c->dev<double>(L.Kv);
    q.Av = c->dev<double>(L.Av);
    q.dinv = c->dev<double>(L.dinv);
    q.dinv32 = c->dev<float>(L.dinv32);
    q.b = c->dev<double>(L.b);
    q.s = c->dev<double>(L.s);
    q.u = ionic_nstates(c->ionic_kind) ? c->dev<double>(L.u) : nullptr;
    q.part0 = c->dev<double>(L.partial);
    q.part_pq = q.part0 + 3 * kPartialCap;
    q.part_rz = q.part0 + 6 * kPartialCap;
    q.r32 = c->dev<float>(L.r32);
    q.p32 = c->dev<float>(L.p32);
    q.q32 = c->dev<float>(L.q32);
    q.delta = c->dev<float>(L.delta);
    q.g32 = c->dev<float>(L.g32);
    q.bsc = c->dev<BScalars>(L.bsc);
    return q;
}

BParams batch_params(const mdx_ctx *c)
{
    return BParams{c->opts.atol, c->opts.rtol, c->opts.max_iter, c->opts.rr_interval,
                   c->opts.rel_mode};
}

constexpr int kPersistentSpinCap = 1000000;   // polls (about 60 ms) before a barrier gives up

void launch_persistent(mdx_ctx *c, hipStream_t st, const BatchPtrs &q, const BParams &bp)
{
    unsigned *bar = c->dev<unsigned>(c->L.pbar);
    launch_b_persistent(st, c->pseg, q.P, c->dev<float>(c->L.A32), q.dinv32, bp, q.p32, q.q32,
                        q.delta, q.r32, q.part_pq, q.part_rz, q.bsc, bar,
                        reinterpret_cast<int *>(bar + c->n_inst), kPersistentSpinCap);
}

// the persistent iteration's barrier timed out (its groups were not all resident)
mdx_status persistent_fault(mdx_ctx *c, hipStream_t st)
{
    mdx_ctx *ctx = c;   // for HIPCHK
    int fault = 0;
    HIPCHK(hipMemcpyAsync(&fault, c->dev<unsigned>(c->L.pbar) + c->n_inst, sizeof(int),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (fault)
        return fail(c, MDX_ERR_DEVICE,
                    "a barrier of the persistent batched iteration timed out (%d workgroups; "
                    "not all were resident)", c->pseg.groups);
    return MDX_OK;
}

// ionic update, right-hand side and initial residual, `iters` PCG iterations
// of every running instance, one residual-replacement pass.  With `timed`,
// event pairs bracket the SpMV launches.
void enqueue_batched_step(mdx_ctx *c, hipStream_t st, int iters, const double *istim, bool timed)
{
    const BatchPtrs q = batch_ptrs(c);
    const BParams bp = batch_params(c);
    const StepParams sp = step_params(c);
    double *V = c->vec(0), *Vprev = c->vec(1), *X = c->vec(2);
    if (c->opts.precision == MDX_PREC_MIXED_GATES32)
        launch_ionic_step_mixed(st, c->ionic_kind, c->ionic_params.data(), c->npad, c->npad, c->dt,
                                c->cm, V, q.u, q.g32, istim, q.s, row_mask(c));
    else
        launch_ionic_step(st, c->ionic_kind, c->ionic_params.data(), c->npad, c->npad, c->dt, c->cm,
                          V, q.u, istim, q.s, 0, row_mask(c));
    launch_b_rhs_init(st, c->seg, q.P, q.Mv, q.Kv, q.dinv, q.dinv32, sp, c->npad, V, Vprev, q.s,
                      c->dev<double>(c->L.gv), X, q.b, q.r32, q.delta, q.part0,
                      use_nt(c, 20.0 * slots(c)));
    launch_b_init_finalize(st, c->seg, q.part0, bp, q.bsc);
    launch_b_set_direction(st, c->seg, q.dinv32, q.r32, q.p32, q.bsc);
    if (c->persistent) {
        launch_persistent(c, st, q, bp);
        iters = 0;
    }
    for (int i = 0; i < iters; ++i) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timed && 2 * i + 1 < (int)c->ev.size()) {
            e0 = c->ev[2 * i];
            e1 = c->ev[2 * i + 1];
        }
        launch_b_iteration(st, c->seg, q.IM, bp, q.dinv32, q.p32, q.q32, q.delta, q.r32, q.part_pq,
                           q.part_rz, q.bsc, e0, e1);
    }
    launch_b_replacement(st, c->seg, q.P, bp, q.Av, X, q.delta, q.b, q.dinv, q.dinv32, q.r32, q.p32,
                         q.part0, q.bsc, use_nt(c, 12.0 * slots(c)));
}

mdx_status fetch_bscalars(mdx_ctx *c, hipStream_t st)
{
    mdx_ctx *ctx = c;   // for HIPCHK
    HIPCHK(hipMemcpyAsync(c->bsc_host, c->dev<BScalars>(c->L.bsc), sizeof(BScalars) * c->n_inst,
                          hipMemcpyDeviceToHost, st));
    auto w0 = std::chrono::steady_clock::now();
    HIPCHK(hipStreamSynchronize(st));
    c->stats.host_wait_seconds +=
        std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
    return MDX_OK;
}

bool all_done(const mdx_ctx *c)
{
    for (int i = 0; i < c->n_inst; ++i)
        if (!c->bsc_host[i].done) return false;
    return true;
}

mdx_status run_batched(mdx_ctx *ctx, int64_t n_steps, int64_t out_every, double *v_out)
{
    if (ctx->opts.precision == MDX_PREC_FP64)
        return fail(ctx, MDX_ERR_UNSUPPORTED,
                    "a batched context runs the mixed-precision solver (MDX_PREC_MIXED)");
    if (ctx->opts.warm_start == MDX_WS_MLP || ctx->rec_X)
        return fail(ctx, MDX_ERR_UNSUPPORTED, "no learned warm start or recorder in a batched context");
    // graphs cannot be captured on the legacy default stream: use an own one
    hipStream_t st = ctx->stream;
    if (!st) {
        if (!ctx->own_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        st = ctx->own_stream;
    }
    const Layout &L = ctx->L;
    const BatchPtrs q = batch_ptrs(ctx);
    const BParams bp = batch_params(ctx);
    const int max_iter = ctx->opts.max_iter;
    double *istim_dev = ctx->dev<double>(L.istim);
    Scalars *sc = ctx->dev<Scalars>(L.scalars);
    mdx_status result = MDX_OK;
    ctx->iters_hist.clear();
    ctx->inst_iters_hist.clear();
    int64_t n_out = 0;
    auto t_start = std::chrono::steady_clock::now();

    for (int64_t j = 0; j < n_steps; ++j) {
        const int64_t k = ctx->step;
        bool any_stim = false;
        if (mdx_status e = update_stimulus(ctx, st, k, any_stim)) return e;
        double *V = ctx->vec(0), *X = ctx->vec(2);
        const bool profiling = ctx->profile_every > 0 && k % ctx->profile_every == 0;
        const int C = std::max(1, std::min(ctx->last_iters, max_iter));
        if (ctx->use_graph && !profiling) {
            const std::pair<int, int> key{ctx->persistent ? -1 : C, ctx->vb[0]};
            auto it = ctx->graphs.find(key);
            if (it == ctx->graphs.end()) {
                hipGraph_t g = nullptr;
                HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                enqueue_batched_step(ctx, st, C, istim_dev, false);
                HIPCHK(hipStreamEndCapture(st, &g));
                hipGraphExec_t ex = nullptr;
                hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                HIPCHK(ie);
                it = ctx->graphs.emplace(key, ex).first;
            }
            HIPCHK(hipGraphLaunch(it->second, st));
        } else {
            enqueue_batched_step(ctx, st, C, any_stim ? istim_dev : nullptr, profiling);
        }
        HIPCHK(hipGetLastError());
        int units = C;
        if (mdx_status e = fetch_bscalars(ctx, st)) return e;
        if (ctx->persistent)
            if (mdx_status e = persistent_fault(ctx, st)) return e;
        while (!all_done(ctx) && units < max_iter + 1) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (profiling && 2 * units + 1 < (int)ctx->ev.size()) {
                e0 = ctx->ev[2 * units];
                e1 = ctx->ev[2 * units + 1];
            }
            if (ctx->persistent)
                launch_persistent(ctx, st, q, bp);
            else
                launch_b_iteration(st, ctx->seg, q.IM, bp, q.dinv32, q.p32, q.q32, q.delta, q.r32,
                                   q.part_pq, q.part_rz, q.bsc, e0, e1);
            launch_b_replacement(st, ctx->seg, q.P, bp, q.Av, X, q.delta, q.b, q.dinv, q.dinv32, q.r32,
                                 q.p32, q.part0, q.bsc, use_nt(ctx, 12.0 * slots(ctx)));
            HIPCHK(hipGetLastError());
            ++units;
            if (mdx_status e = fetch_bscalars(ctx, st)) return e;
            if (ctx->persistent)
                if (mdx_status e = persistent_fault(ctx, st)) return e;
        }
        if (!all_done(ctx))
            return fail(ctx, MDX_ERR_STATE, "batched solve of step %lld did not finish",
                        (long long)k);
        int max_it = 0, step_iters = 0;
        bool failed = false;
        double bytes = 0.0;
        for (int i = 0; i < ctx->n_inst; ++i) {
            const BScalars &b = ctx->bsc_host[i];
            if (b.nonfinite)
                return fail(ctx, MDX_ERR_NONFINITE,
                            "non-finite value in the solve of instance %d, step %lld", i,
                            (long long)k);
            const int itv = b.failed ? -1 : b.iters;
            ctx->inst_iters_hist.push_back(itv);
            max_it = std::max(max_it, b.it);
            if (itv < 0) {
                failed = true;
                ctx->stats.not_converged++;
            } else {
                step_iters = std::max(step_iters, itv);
            }
            ctx->stats.cg_iters_total += b.it;
            const int64_t ni = ctx->inst_node_ptr[i + 1] - ctx->inst_node_ptr[i];
            bytes += (double)b.it * (8.0 * (double)ctx->inst_nnz[i] + 8.0 * (double)ni);
        }
        ctx->stats.cg_iters_max = std::max<int64_t>(ctx->stats.cg_iters_max, max_it);
        ctx->last_iters = max_it;
        if (failed) result = MDX_WARN_NOT_CONVERGED;
        if (profiling) {
            const int timed = std::min(units, (int)ctx->ev.size() / 2);
            for (int u_ = 0; u_ < timed; ++u_) {
                float ms = 0.0f;
                HIPCHK(hipEventElapsedTime(&ms, ctx->ev[2 * u_], ctx->ev[2 * u_ + 1]));
                ctx->stats.spmv_seconds += 1e-3 * ms;
                ctx->stats.spmv_timed++;
            }
            if (timed == units) {
                ctx->stats.spmv_work += units;
                ctx->stats.spmv_bytes += bytes;
            }
        }
        launch_epilogue(st, ctx->npad, (double)(k + 1) * ctx->dt, V, X, ctx->dev<double>(L.lat),
                        ctx->dev<double>(L.lrt), sc);
        int old_prev = ctx->vb[1];
        ctx->vb[1] = ctx->vb[0];
        ctx->vb[0] = ctx->vb[2];
        ctx->vb[2] = old_prev;
        ctx->step++;
        ctx->iters_hist.push_back(failed ? -1 : step_iters);
        ctx->stats.steps++;
        if (out_every > 0 && (j + 1) % out_every == 0 && v_out) {
            HIPCHK(hipStreamSynchronize(st));
            if (mdx_status e = copy_vec_out(ctx, ctx->vec(0), v_out + n_out * ctx->n)) return e;
            ++n_out;
        }
    }
    HIPCHK(hipMemcpyAsync(ctx->sc_host, sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ctx->stats.step_loop_seconds +=
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (ctx->sc_host->nonfinite)
        return fail(ctx, MDX_ERR_NONFINITE, "non-finite V after step %lld", (long long)ctx->step);
    return result;
}

}  // namespace

// ===========================================================================
extern "C" {

int mdx_version(void) { return 1; }

int32_t mdx_ionic_nstates(int32_t kind) { return ionic_nstates(kind); }
int32_t mdx_ionic_nparams(int32_t kind) { return ionic_nparams(kind); }

mdx_status mdx_create(mdx_ctx **out, int device, void *stream)
{
    if (!out) return MDX_ERR_INVALID_ARG;
    *out = nullptr;
    if (device == -1) {   // host-only context: problem statement and validation only
        mdx_ctx *ctx = new (std::nothrow) mdx_ctx();
        if (!ctx) return MDX_ERR_INVALID_ARG;
        ctx->device = -1;
        *out = ctx;
        return MDX_OK;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return MDX_ERR_DEVICE;
    mdx_ctx *ctx = new (std::nothrow) mdx_ctx();
    if (!ctx) return MDX_ERR_INVALID_ARG;
    ctx->device = device;
    ctx->stream = (hipStream_t)stream;
    if (hipSetDevice(device) != hipSuccess ||
        hipHostMalloc((void **)&ctx->sc_host, sizeof(Scalars), hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return MDX_ERR_DEVICE;
    }
    if (hipHostMalloc((void **)&ctx->pub, sizeof(Published),
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void **)&ctx->pub_dev, ctx->pub, 0) != hipSuccess) {
        if (ctx->pub) (void)hipHostFree(ctx->pub);
        (void)hipHostFree(ctx->sc_host);
        delete ctx;
        return MDX_ERR_DEVICE;
    }
    ctx->pub->seq = 0;
    // device address of the allocation-free gradient's partials (resolved
    // once per device, with the device current)
    ctx->grad_scratch = mlp_noalloc_scratch(device);
    *out = ctx;
    return MDX_OK;
}

void mdx_destroy(mdx_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->device < 0) {
        delete ctx;
        return;
    }
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream); else (void)hipDeviceSynchronize();
    for (hipEvent_t e : ctx->ev) (void)hipEventDestroy(e);
    release_graphs(ctx);
    if (ctx->own_stream) {
        (void)hipStreamSynchronize(ctx->own_stream);
        (void)hipStreamDestroy(ctx->own_stream);
    }
    if (ctx->bsc_host) (void)hipHostFree(ctx->bsc_host);
    if (ctx->sc_host) (void)hipHostFree(ctx->sc_host);
    if (ctx->pub) (void)hipHostFree(ctx->pub);
    if (ctx->stage) (void)hipHostFree(ctx->stage);
    delete ctx;
}

const char *mdx_last_error(const mdx_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

mdx_status mdx_set_mesh(mdx_ctx *ctx, int64_t n_nodes, const double *xyz, double unit_conversion,
                        int64_t n_tets, const int32_t *tets, const int32_t *region,
                        const double *fibre)
{
    const int64_t ptr[2] = {0, n_nodes};
    return set_mesh_impl(ctx, 1, ptr, false, n_nodes, xyz, unit_conversion, n_tets, tets, region,
                         fibre);
}

mdx_status mdx_set_surface_mesh(mdx_ctx *ctx, int64_t n_nodes, const double *xyz,
                                double unit_conversion, int64_t n_tris, const int32_t *tris,
                                const int32_t *region, const double *fibre)
{
    const int64_t ptr[2] = {0, n_nodes};
    return set_mesh_impl(ctx, 1, ptr, false, n_nodes, xyz, unit_conversion, n_tris, tris, region,
                         fibre, 3);
}

mdx_status mdx_set_mesh_batch(mdx_ctx *ctx, int32_t n_inst, const int64_t *node_ptr, int64_t n_nodes,
                              const double *xyz, double unit_conversion, int64_t n_tets,
                              const int32_t *tets, const int32_t *region, const double *fibre)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (n_inst < 1 || n_inst > (1 << 20) || !node_ptr)
        return fail(ctx, MDX_ERR_INVALID_ARG, "n_inst must lie in [1, 2^20] with node_ptr given");
    return set_mesh_impl(ctx, n_inst, node_ptr, true, n_nodes, xyz, unit_conversion, n_tets, tets,
                         region, fibre);
}

mdx_status mdx_set_surface_mesh_batch(mdx_ctx *ctx, int32_t n_inst, const int64_t *node_ptr,
                                      int64_t n_nodes, const double *xyz, double unit_conversion,
                                      int64_t n_tris, const int32_t *tris, const int32_t *region,
                                      const double *fibre)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (n_inst < 1 || n_inst > (1 << 20) || !node_ptr)
        return fail(ctx, MDX_ERR_INVALID_ARG, "n_inst must lie in [1, 2^20] with node_ptr given");
    return set_mesh_impl(ctx, n_inst, node_ptr, true, n_nodes, xyz, unit_conversion, n_tris, tris,
                         region, fibre, 3);
}

mdx_status mdx_add_conductivity(mdx_ctx *ctx, int32_t n_ids, const int32_t *region_ids, double il,
                                double it)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (n_ids <= 0 || !region_ids)
        return fail(ctx, MDX_ERR_INVALID_ARG, "no region ids given");
    if (!(il >= 0.0) || !(it >= 0.0) || !std::isfinite(il) || !std::isfinite(it) || il + it <= 0.0)
        return fail(ctx, MDX_ERR_INVALID_ARG, "conductivities must be finite and >= 0 (not both 0)");
    GUARD_BEGIN
    for (int32_t i = 0; i < n_ids; ++i) ctx->cond[region_ids[i]] = {il, it};
    ctx->prepared = false;
    return MDX_OK;
    GUARD_END
}

mdx_status mdx_add_conductivity_ie(mdx_ctx *ctx, int32_t n_ids, const int32_t *region_ids,
                                   double il, double it, double el, double et)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    for (double v : {il, it, el, et})
        if (!(v > 0.0) || !std::isfinite(v))
            return fail(ctx, MDX_ERR_INVALID_ARG,
                        "intra- and extracellular conductivities must be finite and > 0");
    // monodomain conductivity per direction: intra- and extracellular in series
    return mdx_add_conductivity(ctx, n_ids, region_ids, il * el / (il + el), it * et / (it + et));
}

mdx_status mdx_set_mass_lumping(mdx_ctx *ctx, int32_t lumped)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (lumped != 0 && lumped != 1) return fail(ctx, MDX_ERR_INVALID_ARG, "lumped is 0 or 1");
    ctx->lumped = lumped != 0;
    ctx->prepared = false;
    return MDX_OK;
}

mdx_status mdx_set_tissue(mdx_ctx *ctx, double chi, double cm, double theta)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (!(chi > 0.0) || !(cm > 0.0) || !std::isfinite(chi) || !std::isfinite(cm))
        return fail(ctx, MDX_ERR_INVALID_ARG, "chi and Cm must be finite and > 0");
    if (!(theta >= 0.0 && theta <= 1.0))
        return fail(ctx, MDX_ERR_INVALID_ARG, "theta must lie in [0, 1]");
    ctx->chi = chi;
    ctx->cm = cm;
    ctx->theta = theta;
    ctx->prepared = false;
    return MDX_OK;
}

mdx_status mdx_set_ionic(mdx_ctx *ctx, int32_t kind, int32_t n_params, const double *params)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (kind < MDX_IONIC_NONE || kind > MDX_IONIC_CRN)
        return fail(ctx, MDX_ERR_UNSUPPORTED, "unknown ionic model %d", kind);
    int np = ionic_nparams(kind);
    if (params && n_params != np)
        return fail(ctx, MDX_ERR_INVALID_ARG, "model %d takes %d parameters, got %d", kind, np,
                    n_params);
    std::vector<double> p(np);
    ionic_defaults(kind, p.data());
    if (params)
        for (int i = 0; i < np; ++i) {
            if (!std::isfinite(params[i]))
                return fail(ctx, MDX_ERR_INVALID_ARG, "non-finite ionic parameter %d", i);
            p[i] = params[i];
        }
    if (kind == MDX_IONIC_MS && (!(p[0] > 0) || !(p[1] > 0) || !(p[2] > 0) || !(p[3] > 0) ||
                                 p[6] == 0.0))
        return fail(ctx, MDX_ERR_INVALID_ARG, "Mitchell-Schaeffer time constants must be > 0");
    if (ctx->ionic_kind != kind) ctx->prepared = false;
    ctx->ionic_kind = kind;
    ctx->ionic_params = p;
    // captured step graphs hold the parameters by value
    release_graphs(ctx);
    return MDX_OK;
}

mdx_status mdx_add_stimulus(mdx_ctx *ctx, int64_t n_idx, const int32_t *node_idx, double start,
                            double duration, double intensity)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (mdx_status s = require_mesh(ctx)) return s;
    if (n_idx <= 0 || !node_idx) return fail(ctx, MDX_ERR_INVALID_ARG, "empty stimulus");
    if (!std::isfinite(start) || !(duration >= 0.0) || !std::isfinite(duration) ||
        !std::isfinite(intensity))
        return fail(ctx, MDX_ERR_INVALID_ARG, "stimulus start/duration/intensity invalid");
    GUARD_BEGIN
    Stim st;
    st.nodes.assign(node_idx, node_idx + n_idx);
    for (int32_t v : st.nodes)
        if (v < 0 || v >= ctx->n)
            return fail(ctx, MDX_ERR_INVALID_ARG, "stimulus node %d out of range", v);
    std::sort(st.nodes.begin(), st.nodes.end());
    st.nodes.erase(std::unique(st.nodes.begin(), st.nodes.end()), st.nodes.end());
    st.start = start;
    st.duration = duration;
    st.amp = intensity;
    ctx->stims.push_back(std::move(st));
    ctx->prepared = false;
    return MDX_OK;
    GUARD_END
}

mdx_status mdx_set_solver(mdx_ctx *ctx, const mdx_solver_opts *o)
{
    if (!ctx || !o) return MDX_ERR_INVALID_ARG;
    if (!(o->atol >= 0.0) || !(o->rtol >= 0.0) || o->max_iter < 1 || o->reserved != 0 ||
        o->precision < MDX_PREC_FP64 || o->precision > MDX_PREC_MIXED_GATES32 || o->rr_interval < 0 ||
        (o->rel_mode != MDX_REL_INITIAL && o->rel_mode != MDX_REL_RHS) ||
        (o->warm_start != MDX_WS_PREV && o->warm_start != MDX_WS_EXTRAP &&
         o->warm_start != MDX_WS_MLP))
        return fail(ctx, MDX_ERR_INVALID_ARG, "invalid solver options");
    ctx->opts = *o;
    release_graphs(ctx);   // captured steps hold the solver options
    if (ctx->prepared) {
        Scalars *sc = ctx->dev<Scalars>(ctx->L.scalars);
        HIPCHK(hipMemcpyAsync(&sc->atol, &o->atol, sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(&sc->rtol, &o->rtol, sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return MDX_OK;
}

mdx_status mdx_workspace_size(mdx_ctx *ctx, size_t *persistent_bytes, size_t *scratch_bytes)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (mdx_status s = require_mesh(ctx)) return s;
    compute_layout(ctx);
    if (persistent_bytes) *persistent_bytes = ctx->L.total;
    if (scratch_bytes) *scratch_bytes = ctx->L.x_total;
    return MDX_OK;
}

mdx_status mdx_bind_workspace(mdx_ctx *ctx, void *device_ptr, size_t bytes)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (ctx->device < 0) return fail(ctx, MDX_ERR_DEVICE, "host-only context (device -1)");
    if (mdx_status s = require_mesh(ctx)) return s;
    compute_layout(ctx);
    if (!device_ptr || ((uintptr_t)device_ptr % kAlign) != 0)
        return fail(ctx, MDX_ERR_NO_WORKSPACE, "workspace must be non-null and 256-byte aligned");
    if (bytes < ctx->L.total)
        return fail(ctx, MDX_ERR_NO_WORKSPACE, "workspace of %zu bytes < required %zu", bytes,
                    ctx->L.total);
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, device_ptr) != hipSuccess ||
        attr.type != hipMemoryTypeDevice || attr.device != ctx->device)
        return fail(ctx, MDX_ERR_NO_WORKSPACE, "workspace is not device memory of device %d",
                    ctx->device);
    ctx->ws = (char *)device_ptr;
    ctx->ws_bytes = bytes;
    ctx->prepared = false;
    return MDX_OK;
}

mdx_status mdx_prepare(mdx_ctx *ctx, double dt, void *scratch, size_t scratch_bytes)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (ctx->device < 0) return fail(ctx, MDX_ERR_DEVICE, "host-only context (device -1)");
    if (mdx_status s = require_mesh(ctx)) return s;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, MDX_ERR_INVALID_ARG, "dt must be > 0");
    compute_layout(ctx);
    if (!ctx->ws || ctx->ws_bytes < ctx->L.total)
        return fail(ctx, MDX_ERR_NO_WORKSPACE, "no (large enough) workspace bound");
    if (!scratch || ((uintptr_t)scratch % kAlign) != 0 || scratch_bytes < ctx->L.x_total)
        return fail(ctx, MDX_ERR_NO_WORKSPACE, "setup scratch missing, unaligned or < %zu bytes",
                    ctx->L.x_total);
    GUARD_BEGIN
    // per-element conductivities
    std::vector<double> sig(2 * ctx->m);
    for (int64_t e = 0; e < ctx->m; ++e) {
        auto it = ctx->cond.find(ctx->region[e]);
        if (it == ctx->cond.end())
            return fail(ctx, MDX_ERR_STATE, "no conductivity for region %d", ctx->region[e]);
        sig[2 * e] = it->second.first;
        sig[2 * e + 1] = it->second.second;
    }
    // slot map: contributions (element*16 + a*4 + b, a and b < npe) per slot,
    // ascending element order
    const int npe = ctx->npe;
    const int64_t ncontrib = (int64_t)npe * npe * ctx->m;
    std::vector<int64_t> cptr(ctx->nslots + 1, 0);
    std::vector<int64_t> slot_of(16 * ctx->m, -1);
    for (int64_t e = 0; e < ctx->m; ++e) {
        const int32_t *t = &ctx->tets[4 * e];
        for (int a = 0; a < npe; ++a)
            for (int b = 0; b < npe; ++b) {
                int64_t s = sell_slot(ctx, ctx->iperm[t[a]], ctx->iperm[t[b]]);
                if (s < 0) return fail(ctx, MDX_ERR_BAD_MESH, "pattern lookup failed");
                slot_of[16 * e + 4 * a + b] = s;
                cptr[s + 1]++;
            }
    }
    for (int64_t s = 0; s < ctx->nslots; ++s) cptr[s + 1] += cptr[s];
    std::vector<int32_t> contrib(ncontrib);
    {
        std::vector<int64_t> pos(cptr.begin(), cptr.end() - 1);
        for (int64_t q = 0; q < 16 * ctx->m; ++q)
            if (slot_of[q] >= 0) contrib[pos[slot_of[q]]++] = (int32_t)q;
    }
    slot_of.clear();
    slot_of.shrink_to_fit();

    // host-side check of everything the kernels index with, before any launch
    if (ctx->slice_ptr.size() != (size_t)ctx->nslices + 1 || ctx->slice_ptr[0] != 0 ||
        ctx->slice_ptr[ctx->nslices] != ctx->nslots || (int64_t)ctx->col_sell.size() != ctx->nslots ||
        cptr[ctx->nslots] != ncontrib || ctx->npad % TILE != 0 || ctx->npad < ctx->n)
        return fail(ctx, MDX_ERR_BAD_MESH, "internal layout inconsistent");
    for (int64_t sl = 0; sl < ctx->nslices; ++sl)
        if (ctx->slice_ptr[sl + 1] < ctx->slice_ptr[sl] ||
            (ctx->slice_ptr[sl + 1] - ctx->slice_ptr[sl]) % SLICE != 0)
            return fail(ctx, MDX_ERR_BAD_MESH, "internal layout inconsistent (slice %lld)",
                        (long long)sl);
    for (int32_t c : ctx->col_sell)
        if (c < 0 || c >= ctx->npad) return fail(ctx, MDX_ERR_BAD_MESH, "column out of range");
    if (!ctx->col16.empty()) {
        if ((int64_t)ctx->col16.size() != ctx->nslots || (int64_t)ctx->cbase.size() != ctx->nslices)
            return fail(ctx, MDX_ERR_BAD_MESH, "internal layout inconsistent (16-bit columns)");
        for (int64_t sl = 0; sl < ctx->nslices; ++sl)
            for (int64_t e = ctx->slice_ptr[sl]; e < ctx->slice_ptr[sl + 1]; ++e)
                if (ctx->cbase[sl] + (int32_t)ctx->col16[e] != ctx->col_sell[e])
                    return fail(ctx, MDX_ERR_BAD_MESH, "16-bit column mismatch");
    }
    for (int32_t code : contrib)
        if (code < 0 || code >= 16 * ctx->m || (code >> 2 & 3) >= npe || (code & 3) >= npe)
            return fail(ctx, MDX_ERR_BAD_MESH, "contribution out of range");

    HIPCHK(hipSetDevice(ctx->device));
    if (!ctx->stage) HIPCHK(hipHostMalloc((void **)&ctx->stage, sizeof(double) * ctx->npad,
                                          hipHostMallocDefault));
    const Layout &L = ctx->L;
    char *x = (char *)scratch;
    hipStream_t st = ctx->stream;
    HIPCHK(hipMemcpyAsync(x + L.x_xyz, ctx->xyz.data(), sizeof(double) * 3 * ctx->n,
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(x + L.x_tets, ctx->tets.data(), sizeof(int32_t) * 4 * ctx->m,
                          hipMemcpyHostToDevice, st));
    if (!ctx->fibre.empty())
        HIPCHK(hipMemcpyAsync(x + L.x_fibre, ctx->fibre.data(), sizeof(double) * 3 * ctx->m,
                              hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(x + L.x_sig, sig.data(), sizeof(double) * 2 * ctx->m,
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(x + L.x_cptr, cptr.data(), sizeof(int64_t) * (ctx->nslots + 1),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(x + L.x_contrib, contrib.data(), sizeof(int32_t) * ncontrib,
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ctx->dev<int64_t>(L.slice_ptr), ctx->slice_ptr.data(),
                          sizeof(int64_t) * (ctx->nslices + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(ctx->dev<int32_t>(L.col), ctx->col_sell.data(),
                          sizeof(int32_t) * ctx->nslots, hipMemcpyHostToDevice, st));
    if (!ctx->col16.empty()) {
        HIPCHK(hipMemcpyAsync(ctx->dev<uint16_t>(L.col16), ctx->col16.data(),
                              sizeof(uint16_t) * ctx->nslots, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(ctx->dev<int32_t>(L.cbase), ctx->cbase.data(),
                              sizeof(int32_t) * ctx->nslices, hipMemcpyHostToDevice, st));
    }
    // stimulus node lists in the new numbering
    std::vector<int32_t> sidx;
    ctx->stim_off.assign(1, 0);
    for (auto &s : ctx->stims) {
        for (int32_t v : s.nodes) sidx.push_back(ctx->iperm[v]);
        ctx->stim_off.push_back((int64_t)sidx.size());
    }
    if (!sidx.empty())
        HIPCHK(hipMemcpyAsync(ctx->dev<int32_t>(L.stim_idx), sidx.data(),
                              sizeof(int32_t) * sidx.size(), hipMemcpyHostToDevice, st));

    double *Mv = ctx->dev<double>(L.Mv), *Kv = ctx->dev<double>(L.Kv), *Av = ctx->dev<double>(L.Av);
    launch_element(st, npe, ctx->m, (double *)(x + L.x_xyz), (int32_t *)(x + L.x_tets),
                   ctx->fibre.empty() ? nullptr : (double *)(x + L.x_fibre),
                   (double *)(x + L.x_sig), (double *)(x + L.x_vol), (double *)(x + L.x_ek));
    launch_gather(st, npe, ctx->nslots, (int64_t *)(x + L.x_cptr), (int32_t *)(x + L.x_contrib),
                  (double *)(x + L.x_vol), (double *)(x + L.x_ek), Mv, Kv);
    if (ctx->lumped)
        launch_lump(st, ctx->npad, SellView{ctx->dev<int64_t>(L.slice_ptr), ctx->dev<int32_t>(L.col)},
                    Mv);
    launch_system(st, ctx->nslots, Mv, Kv, ctx->chi * ctx->cm, ctx->theta * dt, Av);
    SellView P{ctx->dev<int64_t>(L.slice_ptr), ctx->dev<int32_t>(L.col)};
    launch_dinv(st, ctx->npad, span_rows(ctx), P, Av, ctx->dev<double>(L.dinv));
    launch_kdiag(st, ctx->npad, span_rows(ctx), P, Kv, ctx->dev<double>(L.kdiag));
    // FP32 copies for the mixed-precision form
    launch_to_f32(st, ctx->nslots, Av, ctx->dev<float>(L.A32));
    launch_to_f32(st, ctx->npad, ctx->dev<double>(L.dinv), ctx->dev<float>(L.dinv32));
    HIPCHK(hipGetLastError());

    // state: rest values, zeroed work vectors, LAT/LRT = +inf
    ctx->vb[0] = 0;
    ctx->vb[1] = 1;
    ctx->vb[2] = 2;
    if (ctx->batched)
        HIPCHK(hipMemcpyAsync(ctx->dev<int32_t>(L.tile_real), ctx->tile_real.data(),
                              sizeof(int32_t) * ctx->tile_real.size(), hipMemcpyHostToDevice, st));
    launch_ionic_init(st, ctx->ionic_kind, ctx->ionic_params.data(), ctx->n, ctx->npad, ctx->vec(0),
                      ctx->vec(1), ionic_nstates(ctx->ionic_kind) ? ctx->dev<double>(L.u) : nullptr,
                      row_mask(ctx));
    for (size_t off : {L.vec[2], L.r, L.p, L.p2, L.q, L.b, L.s, L.istim})
        launch_fill(st, ctx->npad, 0.0, ctx->dev<double>(off));
    launch_fill(st, ctx->npad * 2, 0.0, ctx->dev<double>(L.feat));   // 4 floats per row
    launch_fill(st, ctx->npad / 2, 0.0, ctx->dev<double>(L.mlp_y));
    launch_fill(st, ctx->npad / 2, 0.0, ctx->dev<double>(L.kvp));
    ctx->kvp_valid = false;
    // FP32 vectors: zero bits (float zero) via the double fill over half the count
    for (size_t off : {L.r32, L.z32, L.p32, L.q32, L.delta})
        launch_fill(st, ctx->npad / 2, 0.0, ctx->dev<double>(off));
    launch_gates_to_f32(st, ctx->ionic_kind, ctx->npad, ctx->dev<double>(L.u), ctx->dev<float>(L.g32));
    const double inf = std::numeric_limits<double>::infinity();
    launch_fill(st, ctx->npad, inf, ctx->dev<double>(L.lat));
    launch_fill(st, ctx->npad, inf, ctx->dev<double>(L.lrt));
    HIPCHK(hipGetLastError());
    Scalars init{};
    init.atol = ctx->opts.atol;
    init.rtol = ctx->opts.rtol;
    HIPCHK(hipMemcpyAsync(ctx->dev<Scalars>(L.scalars), &init, sizeof(Scalars),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));

    ctx->tiling = make_tiling(ctx->npad, ctx->max_groups);
    ctx->tiling_spmv = make_tiling(ctx->npad, ctx->spmv_max_groups);
    release_graphs(ctx);
    ctx->fmt = 0;
    ctx->lpr = 1;
    ctx->lpr_built = 0;
    ctx->csr_built = false;
    ctx->inst_iters_hist.clear();
    if (ctx->batched) {
        if (ctx->bsc_host) (void)hipHostFree(ctx->bsc_host);
        ctx->bsc_host = nullptr;
        HIPCHK(hipHostMalloc((void **)&ctx->bsc_host, sizeof(BScalars) * ctx->n_inst,
                             hipHostMallocDefault));
        std::memset((void *)ctx->bsc_host, 0, sizeof(BScalars) * ctx->n_inst);
        HIPCHK(hipMemcpyAsync(ctx->dev<BScalars>(L.bsc), ctx->bsc_host,
                              sizeof(BScalars) * ctx->n_inst, hipMemcpyHostToDevice, st));
        // default: one tile per workgroup (the per-instance partials are
        // reduced once, not by every consumer), more if the partial slots
        // would not hold them
        const int64_t slots = ctx->npad / TILE + ctx->n_inst;
        const int tpb = (int)std::max<int64_t>(1, (slots + kPartialCap - 1) / kPartialCap + 1);
        if (mdx_status e = install_groups(ctx, slots <= kPartialCap ? 1 : tpb)) return e;
        // back to the default iteration (as the layout choice); the persistent
        // group table is rebuilt when it is next selected
        ctx->persistent = false;
        ctx->pseg = SegTiling{};
    }
    ctx->dt = dt;
    ctx->step = 0;
    ctx->active.assign(ctx->stims.size(), 0);
    ctx->last_iters = 0;
    ctx->iters_hist.clear();
    ctx->stats = mdx_stats{};
    ctx->prepared = true;
    ctx->mlp_set = false;
    ctx->rec_X = ctx->rec_dV = ctx->rec_y = nullptr;
    return MDX_OK;
    GUARD_END
}

mdx_status mdx_run(mdx_ctx *ctx, int64_t n_steps, int64_t out_every, double *v_out)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (!ctx->prepared) return fail(ctx, MDX_ERR_STATE, "mdx_prepare has not been called");
    if (n_steps < 0 || out_every < 0) return fail(ctx, MDX_ERR_INVALID_ARG, "negative count");
    if (ctx->opts.precision == MDX_PREC_MIXED_GATES32 && ctx->ionic_gates64_only())
        return fail(ctx, MDX_ERR_UNSUPPORTED,
                    "this ionic model advances its gates in FP64 only (use MDX_PREC_MIXED)");
    GUARD_BEGIN
    HIPCHK(hipSetDevice(ctx->device));
    if (ctx->batched) return run_batched(ctx, n_steps, out_every, v_out);
    const Layout &L = ctx->L;
    hipStream_t st = ctx->stream;
    const Tiling &T = ctx->tiling;
    const Tiling &TS = ctx->tiling_spmv;
    const SellView P = step_view(ctx);
    double *Mv = ctx->dev<double>(L.Mv), *Kv = ctx->dev<double>(L.Kv), *Av = ctx->dev<double>(L.Av);
    double *dinv = ctx->dev<double>(L.dinv);
    double *r = ctx->dev<double>(L.r), *q = ctx->dev<double>(L.q);
    double *pbuf[2] = {ctx->dev<double>(L.p), ctx->dev<double>(L.p2)};
    double *s = ctx->dev<double>(L.s);
    double *u = ionic_nstates(ctx->ionic_kind) ? ctx->dev<double>(L.u) : nullptr;
    double *part0 = ctx->dev<double>(L.partial);
    double *part_pq = part0 + 3 * kPartialCap, *part_rz = part0 + 6 * kPartialCap;
    Scalars *sc = ctx->dev<Scalars>(L.scalars);
    const StepParams sp = step_params(ctx);
    const int max_iter = ctx->opts.max_iter;
    const bool mixed = ctx->opts.precision != MDX_PREC_FP64;
    const bool gates32 = ctx->opts.precision == MDX_PREC_MIXED_GATES32;
    const bool learned = ctx->opts.warm_start == MDX_WS_MLP;
    if (learned && !ctx->mlp_set)
        return fail(ctx, MDX_ERR_STATE, "warm start MDX_WS_MLP needs mdx_set_mlp first");
    double *kdiag = ctx->dev<double>(L.kdiag);
    float *feat = ctx->dev<float>(L.feat), *mlp_y = ctx->dev<float>(L.mlp_y);
    float *kvp = ctx->dev<float>(L.kvp);
    const float *mlp_params = ctx->dev<float>(L.mlp_params);
    float *A32 = ctx->dev<float>(L.A32);
    float *dinv32 = ctx->dev<float>(L.dinv32), *r32 = ctx->dev<float>(L.r32);
    float *p32 = ctx->dev<float>(L.p32), *q32 = ctx->dev<float>(L.q32);
    float *z32 = ctx->dev<float>(L.z32);
    float *delta = ctx->dev<float>(L.delta), *g32 = ctx->dev<float>(L.g32);
    mdx_status result = MDX_OK;
    ctx->iters_hist.clear();
    int64_t n_out = 0;
    // non-temporal hints by the size of each kernel's matrix streams
    const double cbytes = P.col16 ? 2.0 : 4.0;              // per stored column index
    const bool nt_rhs = use_nt(ctx, (16.0 + cbytes) * slots(ctx));   // M, K and columns
    const bool nt_iter64 = use_nt(ctx, (8.0 + cbytes) * slots(ctx));  // FP64 A and columns
    const bool nt_iter32 = use_nt(ctx, (4.0 + cbytes) * slots(ctx));  // FP32 A and columns
    auto t_start = std::chrono::steady_clock::now();
    double *lat = ctx->dev<double>(L.lat), *lrt = ctx->dev<double>(L.lrt);
    // ionic update from Vk: s = I_stim - I_ion (with a guard: only if *guard)
    auto queue_ionic = [&](const double *Vk, const double *istim_k, const int32_t *guard) {
        if (gates32)
            launch_ionic_step_mixed(st, ctx->ionic_kind, ctx->ionic_params.data(), ctx->n, ctx->npad,
                                    ctx->dt, ctx->cm, Vk, u, g32, istim_k, s, nullptr, guard);
        else
            launch_ionic_step(st, ctx->ionic_kind, ctx->ionic_params.data(), ctx->n, ctx->npad,
                              ctx->dt, ctx->cm, Vk, u, istim_k, s, 0, nullptr, guard);
    };
    bool ionic_queued = false;   // this step's ionic update was queued by the previous step

    for (int64_t j = 0; j < n_steps; ++j) {
        const int64_t k = ctx->step;
        bool any_stim = false;
        if (mdx_status e = update_stimulus(ctx, st, k, any_stim)) return e;
        double *V = ctx->vec(0), *Vprev = ctx->vec(1), *X = ctx->vec(2);
        ctx->profiling = ctx->profile_every > 0 && k % ctx->profile_every == 0;
        const double *istim = any_stim ? ctx->dev<double>(L.istim) : nullptr;

        // ---- ionic update: s = I_stim - I_ion ----
        if (!ionic_queued) queue_ionic(V, istim, nullptr);
        ionic_queued = false;

        // ---- right-hand side, warm start, initial residual ----
        // (the three-kernel FP64 iteration starts from p0 = z0, written by
        // the pass that forms r0)
        double *p0_fp64 = mixed ? nullptr : ctx->iter_scheme == 0 ? pbuf[0] : pbuf[1];
        // the learned warm start and the recorder need the neighbour feature
        // (K V^{n-1})_i / K_ii, kept up to date by the right-hand-side pass
        const bool want_kvp = learned || ctx->rec_X;
        if (want_kvp && !ctx->kvp_valid) launch_kv_feature(st, T, P, Kv, kdiag, Vprev, kvp);
        if (learned) {
            // the network forms its features from the state (padding rows
            // keep y = 0); the recorder also takes the raw features and y
            if (ctx->rec_X)
                launch_features(st, ctx->n, ctx->n, V, Vprev, s, kvp, ctx->cm, ctx->mlp_norm,
                                nullptr, ctx->rec_X);
            launch_mlp_forward_state(st, mlp_params, ctx->n, V, Vprev, s, kvp, ctx->cm,
                                     ctx->mlp_norm, mlp_y);
            if (ctx->rec_y)
                HIPCHK(hipMemcpyAsync(ctx->rec_y, mlp_y, sizeof(float) * ctx->n,
                                      hipMemcpyDeviceToDevice, st));
            launch_rhs_learned(st, T, P, Mv, Kv, kdiag, dinv, dinv32, sp,
                               ctx->mlp_norm.out_scale, V, Vprev, s, mlp_y, X, r, p0_fp64,
                               mixed ? r32 : nullptr, z32, delta, kvp, part_pq, part0, nt_rhs);
            launch_init_finalize_ws(st, T, part_pq, part0, sp.rel_mode, sc);
            // where the extrapolation's residual was the smaller, its start
            // vectors (the scalars are already its own, from the same pass):
            // one pass on a small grid, which returns at once, and cheaply,
            // when the network's guess is taken
            StepParams ex = sp;
            ex.warm_start = MDX_WS_EXTRAP;
            const Tiling TF = make_tiling(ctx->npad, 256);
            const int32_t *lost = &sc->use_mlp;
            double *part_unused = part0 + 3 * kPartialCap;   // no reader
            if (mixed)
                launch_rhs_init_mixed(st, TF, P, Mv, Kv, dinv, dinv32, ex, V, Vprev, s, X, r, r32,
                                      z32, delta, part_unused, kdiag, nullptr, nt_rhs, lost);
            else
                launch_rhs_init(st, TF, P, Mv, Kv, dinv, ex, V, Vprev, s, X, r, part_unused,
                                kdiag, nullptr, p0_fp64, nt_rhs, lost);
        } else {
            if (ctx->rec_X)   // training-data recorder: raw features
                launch_features(st, ctx->n, ctx->n, V, Vprev, s, kvp, ctx->cm, ctx->mlp_norm,
                                nullptr, ctx->rec_X);
            float *kvp_out = want_kvp ? kvp : nullptr;
            if (mixed)
                launch_rhs_init_mixed(st, T, P, Mv, Kv, dinv, dinv32, sp, V, Vprev, s, X, r, r32,
                                      z32, delta, part0, kdiag, kvp_out, nt_rhs);
            else
                launch_rhs_init(st, T, P, Mv, Kv, dinv, sp, V, Vprev, s, X, r, part0, kdiag,
                                kvp_out, p0_fp64, nt_rhs);
            launch_init_finalize(st, T, part0, sp.rel_mode, sc);
        }
        ctx->kvp_valid = want_kvp;

        // ---- PCG ----
        int units = 0;   // kernels carrying the SpMV launched so far
        bool done = false;
        // End of a chunk of iterations: the epilogue (activation times; it
        // acts once the solve is done and is idempotent), the scalars
        // published to host memory, and the next step's ionic update (it acts
        // only if this solve is done), which keeps the device busy while the
        // host reads the scalars and queues the rest of that step.
        const double t1 = (double)(k + 1) * ctx->dt;
        bool next_queued = false;
        auto end_chunk = [&]() -> mdx_status {
            launch_epilogue(st, ctx->n, t1, V, X, lat, lrt, sc, &sc->done);
            launch_publish(st, sc, ctx->pub_dev, ++ctx->pub_seq);
            if (j + 1 < n_steps) {
                bool any_next = false;
                if (mdx_status e = update_stimulus(ctx, st, k + 1, any_next)) return e;
                queue_ionic(X, any_next ? ctx->dev<double>(L.istim) : nullptr, &sc->done);
                next_queued = true;
            }
            HIPCHK(hipGetLastError());
            auto w0 = std::chrono::steady_clock::now();
            if (mdx_status e = wait_published(ctx, st, ctx->pub_seq)) return e;
            ctx->stats.host_wait_seconds +=
                std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
            return MDX_OK;
        };
        if (mixed) {
            // a chunk of iterations (each ends with its stopping test), then
            // the (conditional) residual replacement
            const int rr = ctx->opts.rr_interval;
            int it = 0;
            int chunk = std::max(1, ctx->last_iters);
            for (int guard = 0; !done && it < max_iter && guard < 2 * max_iter + 8; ++guard) {
                const int c = std::min(chunk, max_iter - it);
                for (int i = 0; i < c; ++i) {
                    hipEvent_t e0 = nullptr, e1 = nullptr;
                    if (ctx->profiling && 2 * units + 1 < (int)ctx->ev.size()) {
                        e0 = ctx->ev[2 * units];
                        e1 = ctx->ev[2 * units + 1];
                    }
                    launch_cg_iteration32(st, TS, T, it + i, rr, max_iter, P, A32, dinv32, z32, p32,
                                          q32, delta, r32, part_pq, part_rz, sc, e0, e1, nt_iter32);
                    ++units;
                }
                launch_replacement(st, T, P, max_iter, A32, X, delta, r, dinv, dinv32, r32, z32,
                                   part0, sc, nt_iter32);
                if (mdx_status e = end_chunk()) return e;
                done = ctx->sc_host->done != 0;
                it = ctx->sc_host->it_next;
                chunk = 1;
            }
        } else {
            // FP64: a chunk of iterations (the previous step's count first,
            // then one at a time); iteration it ends with the test of
            // ||z_{it+1}||.  Scheme 0 starts from p0 = z0, scheme 1 from
            // z0, both written by the pass that forms r0.
            double *p = pbuf[0], *z = pbuf[1];
            int chunk = std::max(1, ctx->last_iters);
            while (!done && units < max_iter) {
                const int c = std::min(chunk, max_iter - units);
                for (int i = 0; i < c; ++i) {
                    const int it = units + i;
                    hipEvent_t e0 = nullptr, e1 = nullptr;
                    if (ctx->profiling && 2 * it + 1 < (int)ctx->ev.size()) {
                        e0 = ctx->ev[2 * it];
                        e1 = ctx->ev[2 * it + 1];
                    }
                    launch_cg_iteration(st, TS, T, it, max_iter, ctx->iter_scheme, P, Av, dinv, r,
                                        z, p, q, X, part_pq, part_rz, sc, e0, e1, nt_iter64);
                }
                units += c;
                if (mdx_status e = end_chunk()) return e;
                done = ctx->sc_host->done != 0;
                chunk = 1;
            }
        }
        if (learned && !ctx->sc_host->use_mlp) ctx->stats.fallbacks++;
        if (ctx->rec_dV) launch_record_dv(st, ctx->n, V, X, ctx->rec_dV);
        if (ctx->sc_host->nonfinite)
            return fail(ctx, MDX_ERR_NONFINITE, "non-finite value in the solve of step %lld",
                        (long long)k);
        const int iters = done ? ctx->sc_host->iters : -1;
        ctx->last_iters = done ? iters : max_iter;
        if (ctx->profiling) {
            const int timed = std::min(units, (int)ctx->ev.size() / 2);
            if (timed > 0) HIPCHK(hipEventSynchronize(ctx->ev[2 * timed - 1]));
            for (int u_ = 0; u_ < timed; ++u_) {
                float ms = 0.0f;
                HIPCHK(hipEventElapsedTime(&ms, ctx->ev[2 * u_], ctx->ev[2 * u_ + 1]));
                ctx->stats.spmv_seconds += 1e-3 * ms;
                ctx->stats.spmv_timed++;
            }
            const int64_t work = std::min<int64_t>(
                mixed ? ctx->sc_host->it_next : (done ? iters : max_iter), timed);
            ctx->stats.spmv_work += work;
            // per nonzero: value + column.  Per row: the three-kernel FP64
            // scheme reads p once and writes q once; the two-kernel schemes
            // read z once and read and write p and q (q = A z + beta q,
            // p = z + beta p)
            const double per_nnz = (mixed ? 4.0 : 8.0) + cbytes;
            const double per_row = mixed ? 20.0 : ctx->iter_scheme == 1 ? 40.0 : 16.0;
            ctx->stats.spmv_bytes +=
                (double)work * (per_nnz * (double)ctx->nnz + per_row * (double)ctx->n);
        }
        ionic_queued = next_queued && done;
        if (!done)   // iteration cap: the guarded epilogue did not act
            launch_epilogue(st, ctx->n, t1, V, X, lat, lrt, sc);
        // rotate: V^{k+1} <- x, V^k -> V^{k-1}
        int old_prev = ctx->vb[1];
        ctx->vb[1] = ctx->vb[0];
        ctx->vb[0] = ctx->vb[2];
        ctx->vb[2] = old_prev;
        ctx->step++;
        ctx->iters_hist.push_back(iters);
        ctx->stats.steps++;
        if (iters < 0) {
            ctx->stats.not_converged++;
            ctx->stats.cg_iters_total += max_iter;
            result = MDX_WARN_NOT_CONVERGED;
        } else {
            ctx->stats.cg_iters_total += iters;
            ctx->stats.cg_iters_max = std::max<int64_t>(ctx->stats.cg_iters_max, iters);
        }
        if (out_every > 0 && (j + 1) % out_every == 0 && v_out) {
            if (mdx_status e = copy_vec_out(ctx, ctx->vec(0), v_out + n_out * ctx->n)) return e;
            ++n_out;
        }
    }
    HIPCHK(hipMemcpyAsync(ctx->sc_host, sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ctx->stats.step_loop_seconds +=
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (ctx->sc_host->nonfinite)
        return fail(ctx, MDX_ERR_NONFINITE, "non-finite V after step %lld", (long long)ctx->step);
    return result;
    GUARD_END
}

mdx_status mdx_get_times(mdx_ctx *ctx, double *lat, double *lrt)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (!ctx->prepared) return fail(ctx, MDX_ERR_STATE, "not prepared");
    if (lat)
        if (mdx_status e = copy_vec_out(ctx, ctx->dev<double>(ctx->L.lat), lat)) return e;
    if (lrt)
        if (mdx_status e = copy_vec_out(ctx, ctx->dev<double>(ctx->L.lrt), lrt)) return e;
    return MDX_OK;
}

mdx_status mdx_get_apd(mdx_ctx *ctx, double *apd)
{
    if (!ctx || !apd) return MDX_ERR_INVALID_ARG;
    if (!ctx->prepared) return fail(ctx, MDX_ERR_STATE, "not prepared");
    std::vector<double> lrt(ctx->n);
    if (mdx_status e = mdx_get_times(ctx, apd, lrt.data())) return e;
    for (int64_t i = 0; i < ctx->n; ++i)
        apd[i] = std::isfinite(apd[i]) && std::isfinite(lrt[i]) ? lrt[i] - apd[i] : INFINITY;
    return MDX_OK;
}

mdx_status mdx_get_iterations(mdx_ctx *ctx, int64_t n, int32_t *iters)
{
    if (!ctx || (n > 0 && !iters)) return MDX_ERR_INVALID_ARG;
    if (n < 0 || n > (int64_t)ctx->iters_hist.size())
        return fail(ctx, MDX_ERR_INVALID_ARG, "only %zu step counts recorded",
                    ctx->iters_hist.size());
    std::copy(ctx->iters_hist.end() - n, ctx->iters_hist.end(), iters);
    return MDX_OK;
}

mdx_status mdx_get_instance_iterations(mdx_ctx *ctx, int64_t n, int32_t *iters)
{
    if (!ctx || (n > 0 && !iters)) return MDX_ERR_INVALID_ARG;
    const int64_t steps = (int64_t)ctx->inst_iters_hist.size() / std::max(1, ctx->n_inst);
    if (!ctx->batched) return fail(ctx, MDX_ERR_UNSUPPORTED, "not a batched context");
    if (n < 0 || n > steps)
        return fail(ctx, MDX_ERR_INVALID_ARG, "only %lld steps recorded", (long long)steps);
    std::copy(ctx->inst_iters_hist.end() - n * ctx->n_inst, ctx->inst_iters_hist.end(), iters);
    return MDX_OK;
}

mdx_status mdx_autotune(mdx_ctx *ctx, int32_t reps, mdx_tune_report *rep)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (!ctx->prepared || !ctx->batched)
        return fail(ctx, MDX_ERR_STATE, "needs a prepared batched context");
    if (reps < 1 || reps > 1000) return fail(ctx, MDX_ERR_INVALID_ARG, "reps must lie in [1, 1000]");
    GUARD_BEGIN
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    // every instance running: the scalars are re-initialised by the next step
    std::memset((void *)ctx->bsc_host, 0, sizeof(BScalars) * ctx->n_inst);
    HIPCHK(hipMemcpyAsync(ctx->dev<BScalars>(ctx->L.bsc), ctx->bsc_host,
                          sizeof(BScalars) * ctx->n_inst, hipMemcpyHostToDevice, st));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    mdx_tune_report r{};
    double best = std::numeric_limits<double>::infinity();
    int best_fmt = 0, best_lpr = 1, best_tpb = ctx->tpb_b;
    const int layouts[8][2] = {{0, 1}, {0, 2}, {0, 4}, {2, 1}, {3, 1}, {1, 4}, {1, 8}, {1, 16}};
    const int tpbs[4] = {1, 2, 4, 8};
    mdx_status st_ = MDX_OK;
    for (const auto &lay : layouts) {
        if ((st_ = set_iter_layout(ctx, lay[0], lay[1]))) break;
        const BatchPtrs q = batch_ptrs(ctx);
        for (int tpb : tpbs) {
            std::vector<int4> grp;
            std::vector<int32_t> ig;
            if (build_groups(ctx, tpb, grp, ig) != MDX_OK) continue;   // too many groups
            if ((st_ = install_groups(ctx, tpb))) break;
            for (int w = 0; w < 2; ++w)
                launch_b_spmv(st, ctx->seg, q.IM, q.dinv32, q.q32, q.part_pq, q.bsc);
            HIPCHK(hipEventRecord(e0, st));
            for (int i = 0; i < reps; ++i)
                launch_b_spmv(st, ctx->seg, q.IM, q.dinv32, q.q32, q.part_pq, q.bsc);
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            const double sec = 1e-3 * ms / reps;
            if (r.n_candidates < MDX_TUNE_MAX_CANDIDATES) {
                r.cand_format[r.n_candidates] = lay[0];
                r.cand_lanes_per_row[r.n_candidates] = lay[1];
                r.cand_tiles_per_group[r.n_candidates] = tpb;
                r.cand_seconds[r.n_candidates] = sec;
                r.n_candidates++;
            }
            if (sec < best) {
                best = sec;
                best_fmt = lay[0];
                best_lpr = lay[1];
                best_tpb = tpb;
            }
        }
        if (st_) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st_) return st_;
    if (mdx_status e = set_iter_layout(ctx, best_fmt, best_lpr)) return e;
    if (mdx_status e = install_groups(ctx, best_tpb)) return e;
    r.format = best_fmt;
    r.lanes_per_row = best_lpr;
    r.tiles_per_group = best_tpb;
    r.seconds = best;
    r.bytes = 8.0 * (double)ctx->nnz + 8.0 * (double)ctx->n;
    if (rep) *rep = r;
    return MDX_OK;
    GUARD_END
}

mdx_status mdx_get_stats(mdx_ctx *ctx, mdx_stats *out)
{
    if (!ctx || !out) return MDX_ERR_INVALID_ARG;
    *out = ctx->stats;
    out->n_nodes = ctx->n;
    out->nnz = ctx->nnz;
    out->n_sell_slots = ctx->nslots;
    out->bandwidth = ctx->bandwidth;
    out->col_index_bytes = !ctx->batched && ctx->compact_cols && !ctx->col16.empty() ? 2 : 4;
    return MDX_OK;
}

mdx_status mdx_set_profiling(mdx_ctx *ctx, int32_t enable)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (ctx->device < 0) return fail(ctx, MDX_ERR_DEVICE, "host-only context (device -1)");
    HIPCHK(hipSetDevice(ctx->device));
    if (enable < 0) return fail(ctx, MDX_ERR_INVALID_ARG, "sampling period must be >= 0");
    if (enable && ctx->ev.empty()) {
        const int pairs = std::min(ctx->opts.max_iter + 1, 4097);
        for (int i = 0; i < 2 * pairs; ++i) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            ctx->ev.push_back(e);
        }
    }
    ctx->profile_every = enable;
    return MDX_OK;
}

mdx_status mdx_set_tuning(mdx_ctx *ctx, int32_t key, int64_t value)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    switch (key) {
    case MDX_TUNE_MAX_GROUPS:
        if (value < 16 || value > kPartialCap)
            return fail(ctx, MDX_ERR_INVALID_ARG, "max_groups must lie in [16, %d]", kPartialCap);
        ctx->max_groups = (int)value;
        if (ctx->npad > 0) ctx->tiling = make_tiling(ctx->npad, ctx->max_groups);
        return MDX_OK;
    case MDX_TUNE_SPMV_MAX_GROUPS:
        if (value < 16 || value > kPartialCap)
            return fail(ctx, MDX_ERR_INVALID_ARG, "spmv max_groups must lie in [16, %d]",
                        kPartialCap);
        ctx->spmv_max_groups = (int)value;
        if (ctx->npad > 0) ctx->tiling_spmv = make_tiling(ctx->npad, ctx->spmv_max_groups);
        return MDX_OK;
    case MDX_TUNE_ITER_SCHEME:
        if (value != 0 && value != 1) return fail(ctx, MDX_ERR_INVALID_ARG, "scheme is 0 or 1");
        ctx->iter_scheme = (int)value;
        return MDX_OK;
    case MDX_TUNE_FORMAT:
        if (value < 0 || value > 3) return fail(ctx, MDX_ERR_INVALID_ARG, "format is 0..3");
        if (!ctx->batched || !ctx->prepared)
            return fail(ctx, MDX_ERR_STATE, "needs a prepared batched context");
        GUARD_BEGIN
        HIPCHK(hipSetDevice(ctx->device));
        return set_iter_layout(ctx, (int)value, value == 1 ? 8 : 1);
        GUARD_END
    case MDX_TUNE_LANES_PER_ROW:
    case MDX_TUNE_TILES_PER_GROUP:
        if (!ctx->batched || !ctx->prepared)
            return fail(ctx, MDX_ERR_STATE, "needs a prepared batched context");
        GUARD_BEGIN
        HIPCHK(hipSetDevice(ctx->device));
        if (key == MDX_TUNE_LANES_PER_ROW) {
            if (value < 1 || value > 16) return fail(ctx, MDX_ERR_INVALID_ARG, "bad lanes per row");
            return set_iter_layout(ctx, ctx->fmt, (int)value);
        }
        if (value < 1 || value > (1 << 20))
            return fail(ctx, MDX_ERR_INVALID_ARG, "tiles per group must lie in [1, 2^20]");
        return install_groups(ctx, (int)value);
        GUARD_END
    case MDX_TUNE_NONTEMPORAL:
        if (value < -1 || value > 1) return fail(ctx, MDX_ERR_INVALID_ARG, "use -1, 0 or 1");
        ctx->nt_mode = (int)value;
        release_graphs(ctx);
        return MDX_OK;
    case MDX_TUNE_COMPACT_COLUMNS:
        if (value != 0 && value != 1) return fail(ctx, MDX_ERR_INVALID_ARG, "use 0 or 1");
        ctx->compact_cols = value != 0;
        return MDX_OK;
    case MDX_TUNE_PERSISTENT:
        if (value != 0 && value != 1) return fail(ctx, MDX_ERR_INVALID_ARG, "persistent is 0 or 1");
        if (!ctx->batched || !ctx->prepared)
            return fail(ctx, MDX_ERR_STATE, "needs a prepared batched context");
        if (value == 1 && ctx->pseg.groups == 0) {
            GUARD_BEGIN
            HIPCHK(hipSetDevice(ctx->device));
            if (mdx_status e = install_persistent_groups(ctx)) return e;
            GUARD_END
        }
        ctx->persistent = value == 1;
        release_graphs(ctx);
        return MDX_OK;
    case MDX_TUNE_GRAPH:
        if (value != 0 && value != 1) return fail(ctx, MDX_ERR_INVALID_ARG, "graph is 0 or 1");
        ctx->use_graph = value != 0;
        release_graphs(ctx);
        return MDX_OK;
    default:
        return fail(ctx, MDX_ERR_INVALID_ARG, "unknown tuning key %d", key);
    }
}

mdx_status mdx_get_state(mdx_ctx *ctx, double *V, double *Vprev, double *u, double *lat,
                         double *lrt, int64_t *step)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (!ctx->prepared) return fail(ctx, MDX_ERR_STATE, "not prepared");
    GUARD_BEGIN
    if (V) if (mdx_status e = copy_vec_out(ctx, ctx->vec(0), V)) return e;
    if (Vprev) if (mdx_status e = copy_vec_out(ctx, ctx->vec(1), Vprev)) return e;
    int ns = ionic_nstates(ctx->ionic_kind);
    if (u && ctx->opts.precision == MDX_PREC_MIXED_GATES32)   // gates live in FP32
        launch_gates_to_f64(ctx->stream, ctx->ionic_kind, ctx->npad, ctx->dev<float>(ctx->L.g32),
                            ctx->dev<double>(ctx->L.u));
    if (u)
        for (int s = 0; s < ns; ++s)
            if (mdx_status e = copy_vec_out(ctx, ctx->dev<double>(ctx->L.u) + s * ctx->npad,
                                            u + s * ctx->n))
                return e;
    if (lat) if (mdx_status e = copy_vec_out(ctx, ctx->dev<double>(ctx->L.lat), lat)) return e;
    if (lrt) if (mdx_status e = copy_vec_out(ctx, ctx->dev<double>(ctx->L.lrt), lrt)) return e;
    if (step) *step = ctx->step;
    return MDX_OK;
    GUARD_END
}

mdx_status mdx_set_state(mdx_ctx *ctx, const double *V, const double *Vprev, const double *u,
                         const double *lat, const double *lrt, int64_t step)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (!ctx->prepared) return fail(ctx, MDX_ERR_STATE, "not prepared");
    int ns = ionic_nstates(ctx->ionic_kind);
    if (!V || !Vprev || (ns > 0 && !u) || step < 0)
        return fail(ctx, MDX_ERR_INVALID_ARG, "V, Vprev (and u) are required, step >= 0");
    for (int64_t i = 0; i < ctx->n; ++i)
        if (!std::isfinite(V[i]) || !std::isfinite(Vprev[i]))
            return fail(ctx, MDX_ERR_INVALID_ARG, "non-finite V at node %lld", (long long)i);
    for (int64_t i = 0; i < (int64_t)ns * ctx->n; ++i)
        if (!std::isfinite(u[i]))
            return fail(ctx, MDX_ERR_INVALID_ARG, "non-finite ionic state %lld of node %lld",
                        (long long)(i / ctx->n), (long long)(i % ctx->n));
    GUARD_BEGIN
    if (mdx_status e = copy_vec_in(ctx, V, ctx->vec(0))) return e;
    if (mdx_status e = copy_vec_in(ctx, Vprev, ctx->vec(1))) return e;
    for (int s = 0; s < ns; ++s)
        if (mdx_status e = copy_vec_in(ctx, u + s * ctx->n, ctx->dev<double>(ctx->L.u) + s * ctx->npad))
            return e;
    launch_gates_to_f32(ctx->stream, ctx->ionic_kind, ctx->npad, ctx->dev<double>(ctx->L.u),
                        ctx->dev<float>(ctx->L.g32));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (lat) {
        if (mdx_status e = copy_vec_in(ctx, lat, ctx->dev<double>(ctx->L.lat))) return e;
    }
    if (lrt) {
        if (mdx_status e = copy_vec_in(ctx, lrt, ctx->dev<double>(ctx->L.lrt))) return e;
    }
    // padding rows of lat/lrt were zeroed by copy_vec_in; they are never read
    ctx->step = step;
    ctx->kvp_valid = false;
    return MDX_OK;
    GUARD_END
}

mdx_status mdx_get_matrix(mdx_ctx *ctx, int32_t which, int64_t *nnz, int32_t *rows, int32_t *cols,
                          double *vals)
{
    if (!ctx || !nnz) return MDX_ERR_INVALID_ARG;
    if (!ctx->prepared) return fail(ctx, MDX_ERR_STATE, "not prepared");
    if (which < MDX_MAT_M || which > MDX_MAT_A) return fail(ctx, MDX_ERR_INVALID_ARG, "bad matrix");
    if (!rows) {
        *nnz = ctx->nnz;
        return MDX_OK;
    }
    if (!cols || !vals || *nnz < ctx->nnz)
        return fail(ctx, MDX_ERR_INVALID_ARG, "arrays of %lld entries required", (long long)ctx->nnz);
    GUARD_BEGIN
    size_t off = which == MDX_MAT_M ? ctx->L.Mv : which == MDX_MAT_K ? ctx->L.Kv : ctx->L.Av;
    std::vector<double> v(ctx->nslots);
    HIPCHK(hipMemcpyAsync(v.data(), ctx->dev<double>(off), sizeof(double) * ctx->nslots,
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    int64_t o = 0;
    for (int64_t r = 0; r < ctx->npad; ++r) {
        if (ctx->perm[r] < 0) continue;
        int64_t base = ctx->slice_ptr[r / SLICE] + (r % SLICE);
        for (int j = 0; j < ctx->rowlen[r]; ++j) {
            rows[o] = ctx->perm[r];
            cols[o] = ctx->perm[ctx->col_sell[base + (int64_t)j * SLICE]];
            vals[o] = v[base + (int64_t)j * SLICE];
            ++o;
        }
    }
    *nnz = o;
    return MDX_OK;
    GUARD_END
}

mdx_status mdx_spmv(mdx_ctx *ctx, int32_t which, const double *x, double *y)
{
    if (!ctx || !x || !y) return MDX_ERR_INVALID_ARG;
    if (!ctx->prepared) return fail(ctx, MDX_ERR_STATE, "not prepared");
    if (which < MDX_MAT_M || which > MDX_MAT_A) return fail(ctx, MDX_ERR_INVALID_ARG, "bad matrix");
    GUARD_BEGIN
    const Layout &L = ctx->L;
    size_t off = which == MDX_MAT_M ? L.Mv : which == MDX_MAT_K ? L.Kv : L.Av;
    double *p = ctx->dev<double>(L.p), *q = ctx->dev<double>(L.q);
    if (mdx_status e = copy_vec_in(ctx, x, p)) return e;
    const SellView P = step_view(ctx);
    Scalars *sc = ctx->dev<Scalars>(L.scalars);
    launch_spmv_dot(ctx->stream, ctx->tiling, P, ctx->dev<double>(off), p, q,
                    ctx->dev<double>(L.partial) + 3 * kPartialCap, &sc->zero, nullptr, nullptr, false);
    HIPCHK(hipGetLastError());
    return copy_vec_out(ctx, q, y);
    GUARD_END
}

mdx_status mdx_solve(mdx_ctx *ctx, const double *b, const double *x0, double *x, int32_t *iters)
{
    if (!ctx || !b || !x0 || !x) return MDX_ERR_INVALID_ARG;
    if (!ctx->prepared) return fail(ctx, MDX_ERR_STATE, "not prepared");
    if (ctx->batched) return fail(ctx, MDX_ERR_UNSUPPORTED, "not available on a batched context");
    for (int64_t i = 0; i < ctx->n; ++i)
        if (!std::isfinite(b[i]) || !std::isfinite(x0[i]))
            return fail(ctx, MDX_ERR_INVALID_ARG, "non-finite b or x0 at node %lld", (long long)i);
    GUARD_BEGIN
    const Layout &L = ctx->L;
    hipStream_t st = ctx->stream;
    // per-step scratch only: the simulation state is untouched
    double *bd = ctx->dev<double>(L.b), *X = ctx->vec(2), *r = ctx->dev<double>(L.r);
    double *p = ctx->dev<double>(L.p), *q = ctx->dev<double>(L.q);
    double *part0 = ctx->dev<double>(L.partial);
    double *part_pq = part0 + 3 * kPartialCap, *part_rz = part0 + 6 * kPartialCap;
    Scalars *sc = ctx->dev<Scalars>(L.scalars);
    if (mdx_status e = copy_vec_in(ctx, b, bd)) return e;
    if (mdx_status e = copy_vec_in(ctx, x0, X)) return e;
    const Tiling &T = ctx->tiling;
    const SellView P = step_view(ctx);
    const double *Av = ctx->dev<double>(L.Av), *dinv = ctx->dev<double>(L.dinv);
    launch_residual_init(st, T, P, Av, dinv, bd, X, r, p, part0);
    launch_init_finalize(st, T, part0, ctx->opts.rel_mode, sc);
    const int max_iter = ctx->opts.max_iter;
    Scalars h{};
    HIPCHK(hipMemcpyAsync(&h, sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    int it = 0;
    while (!h.done && it < max_iter) {
        const int c = std::min(8, max_iter - it);
        for (int i = 0; i < c; ++i, ++it) {
            launch_cg_iteration(st, ctx->tiling_spmv, T, it, max_iter, 0, P, Av, dinv, r, nullptr,
                                p, q, X, part_pq, part_rz, sc, nullptr, nullptr, false);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&h, sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    if (iters) *iters = h.done ? h.iters : -1;
    if (mdx_status e = copy_vec_out(ctx, X, x)) return e;
    if (h.nonfinite) return fail(ctx, MDX_ERR_NONFINITE, "non-finite value in the solve");
    return MDX_OK;
    GUARD_END
}

mdx_status mdx_ionic_step(mdx_ctx *ctx, double dt, int64_t n, const double *V, double *u,
                          double *iion)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (ctx->device < 0) return fail(ctx, MDX_ERR_DEVICE, "host-only context (device -1)");
    if (n < 0 || (n > 0 && (!V || !iion || (ionic_nstates(ctx->ionic_kind) > 0 && !u))))
        return fail(ctx, MDX_ERR_INVALID_ARG, "null device array");
    if (!(dt >= 0.0) || !std::isfinite(dt)) return fail(ctx, MDX_ERR_INVALID_ARG, "dt must be >= 0");
    if (ctx->ionic_params.empty() && ctx->ionic_kind != 0)
        return fail(ctx, MDX_ERR_STATE, "ionic model not set");
    HIPCHK(hipSetDevice(ctx->device));
    launch_ionic_step(ctx->stream, ctx->ionic_kind, ctx->ionic_params.data(), n, n, dt, 1.0, V, u,
                      nullptr, iion, 1);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MDX_OK;
}

int32_t mdx_mlp_nparams(void) { return mlp_nparams(); }

size_t mdx_mlp_grad_scratch(int64_t n) { return n > 0 ? mlp_grad_scratch_bytes(n) : 0; }

mdx_status mdx_mlp_forward(mdx_ctx *ctx, const float *params, int64_t n, const float *X, float *y)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (ctx->device < 0) return fail(ctx, MDX_ERR_DEVICE, "host-only context (device -1)");
    if (n < 0 || (n > 0 && (!params || !X || !y)) || ((uintptr_t)X % 16) != 0)
        return fail(ctx, MDX_ERR_INVALID_ARG, "null or misaligned device array");
    HIPCHK(hipSetDevice(ctx->device));
    launch_mlp_forward(ctx->stream, params, n, X, y);
    HIPCHK(hipGetLastError());
    return MDX_OK;
}

mdx_status mdx_mlp_grad(mdx_ctx *ctx, const float *params, int64_t n, const float *X, const float *T,
                        float *grad, float *loss, void *scratch, size_t scratch_bytes)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (ctx->device < 0) return fail(ctx, MDX_ERR_DEVICE, "host-only context (device -1)");
    if (n <= 0 || !params || !X || !T || !grad || ((uintptr_t)X % 16) != 0)
        return fail(ctx, MDX_ERR_INVALID_ARG, "null or misaligned device array, or n <= 0");
    if (!scratch || scratch_bytes < mlp_grad_scratch_bytes(n))
        return fail(ctx, MDX_ERR_NO_WORKSPACE, "scratch of %zu bytes required",
                    mlp_grad_scratch_bytes(n));
    HIPCHK(hipSetDevice(ctx->device));
    launch_mlp_grad(ctx->stream, params, n, X, T, grad, loss, (float *)scratch, kGradGroups);
    HIPCHK(hipGetLastError());
    return MDX_OK;
}

mdx_status mdx_mlp_grad_noalloc(mdx_ctx *ctx, const float *params, int64_t n, const float *X,
                                const float *T, float *grad, float *loss)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (ctx->device < 0) return fail(ctx, MDX_ERR_DEVICE, "host-only context (device -1)");
    if (n <= 0 || !params || !X || !T || !grad || ((uintptr_t)X % 16) != 0)
        return fail(ctx, MDX_ERR_INVALID_ARG, "null or misaligned device array, or n <= 0");
    if (n > (int64_t)INT32_MAX)
        return fail(ctx, MDX_ERR_INVALID_ARG, "n = %lld exceeds the maximum 2^31 - 1 samples",
                    (long long)n);
    if (!ctx->grad_scratch)
        return fail(ctx, MDX_ERR_DEVICE, "the library's gradient partials were not resolved");
    HIPCHK(hipSetDevice(ctx->device));
    launch_mlp_grad(ctx->stream, params, n, X, T, grad, loss, ctx->grad_scratch, kNoAllocGroups);
    HIPCHK(hipGetLastError());
    return MDX_OK;
}

mdx_status mdx_mlp_adam(mdx_ctx *ctx, float *params, float *m, float *v, const float *grad, int32_t t,
                        double lr, double beta1, double beta2, double eps)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (ctx->device < 0) return fail(ctx, MDX_ERR_DEVICE, "host-only context (device -1)");
    if (!params || !m || !v || !grad || t < 1 || !(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) ||
        !(beta2 >= 0.0 && beta2 < 1.0) || !(eps >= 0.0))
        return fail(ctx, MDX_ERR_INVALID_ARG, "invalid Adam arguments");
    HIPCHK(hipSetDevice(ctx->device));
    launch_adam(ctx->stream, params, m, v, grad, t, lr, beta1, beta2, eps);
    HIPCHK(hipGetLastError());
    return MDX_OK;
}

mdx_status mdx_set_mlp(mdx_ctx *ctx, const float *params, const double *norm)
{
    if (!ctx || !params || !norm) return MDX_ERR_INVALID_ARG;
    if (!ctx->prepared) return fail(ctx, MDX_ERR_STATE, "not prepared");
    const int np = mlp_nparams();
    for (int i = 0; i < np; ++i)
        if (!std::isfinite(params[i])) return fail(ctx, MDX_ERR_INVALID_ARG, "non-finite parameter %d", i);
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(norm[i])) return fail(ctx, MDX_ERR_INVALID_ARG, "non-finite norm %d", i);
    for (int c = 0; c < 4; ++c)
        if (!(norm[4 + c] > 0.0)) return fail(ctx, MDX_ERR_INVALID_ARG, "std must be > 0");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipMemcpyAsync(ctx->dev<float>(ctx->L.mlp_params), params, sizeof(float) * np,
                          hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int c = 0; c < 4; ++c) {
        ctx->mlp_norm.mean[c] = (float)norm[c];
        ctx->mlp_norm.inv_std[c] = (float)(1.0 / norm[4 + c]);
    }
    ctx->mlp_norm.out_scale = (float)norm[8];
    ctx->mlp_set = true;
    return MDX_OK;
}

mdx_status mdx_set_recorder(mdx_ctx *ctx, float *X, float *dV, float *y)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (!ctx->prepared) return fail(ctx, MDX_ERR_STATE, "not prepared");
    if ((X == nullptr) != (dV == nullptr))
        return fail(ctx, MDX_ERR_INVALID_ARG, "set both recorder arrays or neither");
    if (y && !X) return fail(ctx, MDX_ERR_INVALID_ARG, "y is recorded only with X and dV");
    if (X && ((uintptr_t)X % 16) != 0) return fail(ctx, MDX_ERR_INVALID_ARG, "X must be 16-byte aligned");
    ctx->rec_X = X;
    ctx->rec_dV = dV;
    ctx->rec_y = y;
    return MDX_OK;
}

mdx_status mdx_get_node_order(mdx_ctx *ctx, int32_t *order)
{
    if (!ctx || !order) return MDX_ERR_INVALID_ARG;
    if (mdx_status s = require_mesh(ctx)) return s;
    if (ctx->batched)
        return fail(ctx, MDX_ERR_UNSUPPORTED, "internal rows of a batched context include padding");
    std::copy(ctx->perm.begin(), ctx->perm.begin() + ctx->n, order);
    return MDX_OK;
}

}  // extern "C"
