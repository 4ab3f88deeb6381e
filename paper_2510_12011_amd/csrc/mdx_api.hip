// Host side of the monodomain library: the entry points of include/monox.h
// other than mdx_run (mdx_run.hip).
//
// Setup (host, once per mesh): validation, ordering (mdx_order.hip), the
// sliced-ELL pattern shared by M, K and A and the slot map that lists, for
// every matrix slot, the (element, a, b) contributions in ascending element
// order (mdx_layout.hip).  Device setup (mdx_prepare): element matrices,
// deterministic gather into M and K, A = chi Cm M + theta dt K, the Jacobi
// diagonal, rest state.
#include "mdx_host.h"

namespace mdx {
namespace host {

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

}  // namespace host
}  // namespace mdx

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
        // one record more: its first word receives the persistent iteration's
        // fault flag with the same synchronisation
        HIPCHK(hipHostMalloc((void **)&ctx->bsc_host, sizeof(BScalars) * (ctx->n_inst + 1),
                             hipHostMallocDefault));
        std::memset((void *)ctx->bsc_host, 0, sizeof(BScalars) * (ctx->n_inst + 1));
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
    const int32_t zero = 0;   // a non-finite V of the replaced state no longer stands
    HIPCHK(hipMemcpyAsync(reinterpret_cast<char *>(ctx->dev<Scalars>(ctx->L.scalars)) +
                              offsetof(Scalars, nonfinite_v),
                          &zero, sizeof zero, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
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

mdx_status mdx_mlp_samples(mdx_ctx *ctx, int64_t n_idx, const int64_t *idx, int64_t n_rows,
                           const float *X, const float *dV, const double *norm, float *Xo,
                           float *To)
{
    if (!ctx) return MDX_ERR_INVALID_ARG;
    if (ctx->device < 0) return fail(ctx, MDX_ERR_DEVICE, "host-only context (device -1)");
    if (n_idx < 0 || n_rows < 0) return fail(ctx, MDX_ERR_INVALID_ARG, "negative count");
    if (n_idx == 0) return MDX_OK;
    if (!idx || !X || !dV || !Xo || !To) return fail(ctx, MDX_ERR_INVALID_ARG, "null array");
    if (reinterpret_cast<uintptr_t>(X) % 16 || reinterpret_cast<uintptr_t>(Xo) % 16)
        return fail(ctx, MDX_ERR_INVALID_ARG, "X and Xo must be 16-byte aligned");
    MlpNorm nm{{0.f, 0.f, 0.f, 0.f}, {1.f, 1.f, 1.f, 1.f}, 1.f};
    if (norm) {
        for (int i = 0; i < 9; ++i)
            if (!std::isfinite(norm[i])) return fail(ctx, MDX_ERR_INVALID_ARG, "non-finite norm %d", i);
        for (int c = 0; c < 4; ++c) {
            if (!(norm[4 + c] > 0.0)) return fail(ctx, MDX_ERR_INVALID_ARG, "std must be > 0");
            nm.mean[c] = (float)norm[c];
            nm.inv_std[c] = (float)(1.0 / norm[4 + c]);
        }
        if (!(norm[8] > 0.0)) return fail(ctx, MDX_ERR_INVALID_ARG, "out_scale must be > 0");
        nm.out_scale = (float)norm[8];
    }
    HIPCHK(hipSetDevice(ctx->device));
    launch_mlp_samples(ctx->stream, n_idx, idx, n_rows, X, dV, norm != nullptr, nm, Xo, To);
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
