// mdx_run: the single-mesh time loop (plain FP64, precision and learned
// forms).  Per step the kernels of mdx_ionic.hip / mdx_solver.hip
// (mdx_mixed.hip, mdx_learned.hip for the forms) are queued on the
// context's stream; PCG iterations are queued in chunks (first chunk = last
// step's count).  A chunk ends with a one-wave kernel that publishes the
// solver scalars to coherent pinned host memory with a sequence number and
// the next step's ionic update guarded by the done flag (it also records
// this step's activation and repolarisation times); the host spins on the
// sequence number.  Kernels queued after convergence return at their first
// instruction.
#include "mdx_host.h"

extern "C" {

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
    // (the learned right-hand-side pass writes five rows from part_pq on, into
    // part_rz's space, which is unused until the iteration)
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
    float *mlp_y = ctx->dev<float>(L.mlp_y);
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
    // (and, with times, the previous step's activation and repolarisation
    // times from the same read of Vk)
    auto queue_ionic = [&](const double *Vk, const double *istim_k, const int32_t *guard,
                           const StepTimes &times) {
        if (gates32)
            launch_ionic_step_mixed(st, ctx->ionic_kind, ctx->ionic_params.data(), ctx->n, ctx->npad,
                                    ctx->dt, ctx->cm, Vk, u, g32, istim_k, s, nullptr, guard,
                                    times);
        else
            launch_ionic_step(st, ctx->ionic_kind, ctx->ionic_params.data(), ctx->n, ctx->npad,
                              ctx->dt, ctx->cm, Vk, u, istim_k, s, 0, nullptr, guard, times);
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
        if (!ionic_queued) queue_ionic(V, istim, nullptr, StepTimes{});
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
                               mixed ? r32 : nullptr, z32, delta, kvp, part_pq, nt_rhs);
            launch_init_finalize_ws(st, T, part_pq, sp.rel_mode, sc);
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
        // End of a chunk of iterations: the scalars published to host
        // memory and the next step's ionic update (it acts only if this solve
        // is done), which keeps the device busy while the host reads the
        // scalars and queues the rest of that step.  This step's activation
        // and repolarisation times ride in that update (it reads V^{k+1}
        // anyway; idempotent, so the chunk's copy that finds the solve done
        // acts once); the last step of the run has an epilogue kernel instead.
        const double t1 = (double)(k + 1) * ctx->dt;
        bool next_queued = false;
        auto end_chunk = [&]() -> mdx_status {
            const bool carry = j + 1 < n_steps;
            if (!carry) launch_epilogue(st, ctx->n, t1, V, X, lat, lrt, sc, &sc->done);
            launch_publish(st, sc, ctx->pub_dev, ++ctx->pub_seq);
            if (carry) {
                bool any_next = false;
                if (mdx_status e = update_stimulus(ctx, st, k + 1, any_next)) return e;
                queue_ionic(X, any_next ? ctx->dev<double>(L.istim) : nullptr, &sc->done,
                            StepTimes{t1, V, lat, lrt, sc});
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
        if (ctx->sc_host->nonfinite_v)   // found while reading V^k in this step's ionic update
            return fail(ctx, MDX_ERR_NONFINITE, "non-finite V after step %lld", (long long)k - 1);
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
            // p = z + beta p), except the solve's first iteration (beta = 0),
            // which reads neither the old p nor the old q
            const double per_nnz = (mixed ? 4.0 : 8.0) + cbytes;
            const double per_row = mixed ? 20.0 : ctx->iter_scheme == 1 ? 40.0 : 16.0;
            const double fresh_saving = mixed ? 8.0 : ctx->iter_scheme == 1 ? 16.0 : 0.0;
            ctx->stats.spmv_bytes +=
                (double)work * (per_nnz * (double)ctx->nnz + per_row * (double)ctx->n) -
                (work > 0 ? fresh_saving * (double)ctx->n : 0.0);
        }
        ionic_queued = next_queued && done;
        if (!done)   // iteration cap: the guarded update carrying the times did not act
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
    if (ctx->sc_host->nonfinite || ctx->sc_host->nonfinite_v)
        return fail(ctx, MDX_ERR_NONFINITE, "non-finite V after step %lld", (long long)ctx->step);
    return result;
    GUARD_END
}

}  // extern "C"
