// The batched form's time loop: per step the ionic update, right-hand side
// and initial residual of every instance, chunks of PCG iterations (five
// launches per iteration, or one persistent launch) and the residual
// replacement, replayed as HIP graphs when enabled; the host reads the
// per-instance records once per chunk.
#include "mdx_host.h"

namespace mdx {
namespace host {

// ---------------------------------------------------------------------------
// batched form: one time step's work up to the host check
// ---------------------------------------------------------------------------

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

// the persistent iteration's barrier timed out (its groups were not all
// resident); the flag arrives with the instance records (fetch_bscalars)
mdx_status persistent_fault(mdx_ctx *c)
{
    if (*reinterpret_cast<const int *>(c->bsc_host + c->n_inst))
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
    if (c->persistent)
        HIPCHK(hipMemcpyAsync(c->bsc_host + c->n_inst, c->dev<unsigned>(c->L.pbar) + c->n_inst,
                              sizeof(int), hipMemcpyDeviceToHost, st));
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
            if (mdx_status e = persistent_fault(ctx)) return e;
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
                if (mdx_status e = persistent_fault(ctx)) return e;
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
        // the persistent iteration has no separate SpMV launches to time
        if (profiling && !ctx->persistent) {
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

}  // namespace host
}  // namespace mdx
