// Host-side layout: compact column indices, the sliced-ELL pattern shared by
// M, K and A and its slot map, offsets of every array in the workspace,
// small helpers of the time loops, the batched form's group tables and
// iteration layouts (lanes per row, 4-entry chunks, CSR), and the intake of
// a mesh or a batch of meshes.
#include "mdx_host.h"

namespace mdx {
namespace host {

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
        L.gv = take(sizeof(double) * 3 * (c->batched ? np : 1));
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
    // every instance needs a group of its own; from there on, more tiles per
    // group always end with one group per instance
    if (c->n_inst > cap)
        return fail(c, MDX_ERR_UNSUPPORTED,
                    "%d instances exceed the %d workgroups the persistent iteration can keep "
                    "resident", c->n_inst, cap);
    std::vector<int4> grp;
    std::vector<int32_t> ig;
    const int64_t tiles = c->npad / TILE;
    int tpb = (int)std::max<int64_t>(1, (tiles + cap - 1) / cap);
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
                         const double *fibre, int npe)
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

}  // namespace host
}  // namespace mdx
