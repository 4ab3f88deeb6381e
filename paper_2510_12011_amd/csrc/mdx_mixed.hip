// Mixed-precision form of the PCG step: FP32 matrix values and FP32 vectors
// in the SpMV and the vector updates of every iteration, FP64 dot products,
// FP64 right-hand side and solution, FP64 residual replacement.
//
// b, r0 = b - A x0 and every replaced residual use the FP64 matrices, so the
// solve converges to the solution of the FP64 system: FP32-rounded K loses
// its zero row sums (K 1 = 0 is what conserves charge) and a rounded A is not
// the combination of rounded M and K, and either would add a small spurious
// source at every step that accumulates over a run.
//
// The FP32 iteration solves for a correction: x64 stays fixed while
// delta32 accumulates alpha p.  A replacement, triggered every rr
// iterations, when the recursive residual passes the stopping test, or at
// the iteration cap, flushes x64 += delta32 and recomputes the true residual
// r64 = b - A x64 in FP64 -- the stopping test
// is then applied to that true residual, so the solve stops on the same
// criterion as the FP64 path.  If the true residual does not pass, the
// iteration continues from r = r64: after a periodic replacement with
// beta = rho_new / rho_old (the search direction is kept), after one
// triggered by the recursive residual passing the test with p = z (the
// recursion had drifted from the true residual; restart).
//
// Kernels queued after convergence or while a replacement is pending return
// at their first instruction; the replacement kernels return unless one is
// pending.  Reductions are the deterministic two-level scheme of
// mdx_device.h.
#include "mdx_device.h"
#include "mdx_internal.h"

#include <hip/hip_ext.h>

namespace mdx {

namespace {

__device__ __forceinline__ bool halted(const Scalars *sc) { return sc->done || sc->replace; }

__global__ __launch_bounds__(256) void k_to_f32(int64_t n, const double *__restrict__ a,
                                                float *__restrict__ b)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// b, x0 and r0 = b - A x0 in FP64 (FP64 M and K); r32 = r0; delta = 0;
// partials: r32.z32 (FP64 accumulation), |D^-1 r0|^2, |D^-1 b|^2.
template <bool NT, typename CI>
__global__ __launch_bounds__(256) void k_rhs_init_mixed(
    Tiling t, const int64_t *__restrict__ slice_ptr, Cols<CI> col,
    const double *__restrict__ Mv, const double *__restrict__ Kv, const double *__restrict__ dinv,
    const float *__restrict__ dinv32, StepParams sp, const double *__restrict__ V,
    const double *__restrict__ Vprev, const double *__restrict__ src, double *__restrict__ x,
    double *__restrict__ b, float *__restrict__ r32, float *__restrict__ delta,
    double *__restrict__ partial, const double *__restrict__ kdiag, float *__restrict__ kvp)
{
    const int g = logical_group(t.groups);
    const int lane = threadIdx.x & (SLICE - 1);
    const double cK_old = (1.0 - sp.theta) * sp.dt;
    const double cM_new = sp.chi * sp.cm;
    const double cK_new = sp.theta * sp.dt;
    const bool extrap = sp.warm_start == 1;
    double acc[3] = {0.0, 0.0, 0.0};
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t row = (int64_t)tile * TILE + threadIdx.x;
        const int64_t sl = row / SLICE;
        const int64_t beg = slice_ptr[sl] + lane, end = slice_ptr[sl + 1];
        const int32_t cb = slice_base(col, sl);
        double mv = 0.0, kv = 0.0, mx = 0.0, kx = 0.0;
        for (int64_t e = beg; e < end; e += SLICE) {
            const int32_t c = cb + (int32_t)ld_stream<NT>(col.idx + e);
            const double m = ld_stream<NT>(Mv + e), kk = ld_stream<NT>(Kv + e);
            const double vj = V[c];
            const double x0j = extrap ? 2.0 * vj - Vprev[c] : vj;
            mv += m * (sp.cm * vj + sp.dt * src[c]);
            kv += kk * vj;
            mx += m * x0j;
            kx += kk * x0j;
        }
        const double bi = sp.chi * mv - cK_old * kv;
        const double ri = bi - (cM_new * mx + cK_new * kx);
        const double vi = V[row];
        x[row] = extrap ? 2.0 * vi - Vprev[row] : vi;
        b[row] = bi;
        if (kvp) kvp[row] = kdiag[row] != 0.0 ? (float)(kv / kdiag[row]) : 0.0f;
        const float rf = (float)ri;
        r32[row] = rf;
        delta[row] = 0.0f;
        const float zf = dinv32[row] * rf;
        const double zi = dinv[row] * ri, di = dinv[row] * bi;
        acc[0] += (double)rf * (double)zf;
        acc[1] += zi * zi;
        acc[2] += di * di;
    }
    write_partials<3>(acc, partial, t.groups, g);
}

__global__ __launch_bounds__(256) void k_set_direction32(int64_t n, const float *__restrict__ dinv32,
                                                         const float *__restrict__ r32,
                                                         float *__restrict__ p32,
                                                         const Scalars *__restrict__ sc)
{
    if (sc->done) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p32[i] = dinv32[i] * r32[i];
}

// q = A p in FP32; partial p.q in FP64
template <bool NT, typename CI>
__global__ __launch_bounds__(256) void k_spmv32_dot(Tiling t, const int64_t *__restrict__ slice_ptr,
                                                    Cols<CI> col,
                                                    const float *__restrict__ A32,
                                                    const float *__restrict__ p,
                                                    float *__restrict__ q,
                                                    double *__restrict__ partial,
                                                    Scalars *__restrict__ sc)
{
    if (halted(sc)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->redirect = 0;   // consumed by now
    const int g = logical_group(t.groups);
    const int lane = threadIdx.x & (SLICE - 1);
    double acc[1] = {0.0};
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t row = (int64_t)tile * TILE + threadIdx.x;
        const int64_t sl = row / SLICE;
        const int64_t beg = slice_ptr[sl] + lane, end = slice_ptr[sl + 1];
        const int32_t cb = slice_base(col, sl);
        float sum = 0.0f;
#pragma unroll 4
        for (int64_t e = beg; e < end; e += SLICE) sum += ld_stream<NT>(A32 + e) * p[cb + (int32_t)ld_stream<NT>(col.idx + e)];
        q[row] = sum;
        acc[0] += (double)p[row] * (double)sum;
    }
    write_partials<1>(acc, partial, t.groups, g);
}

__global__ __launch_bounds__(256) void k_cg_update32(Tiling t, int k,
                                                     const double *__restrict__ partial_pq,
                                                     const float *__restrict__ dinv32,
                                                     const float *__restrict__ p,
                                                     const float *__restrict__ q,
                                                     float *__restrict__ delta,
                                                     float *__restrict__ r,
                                                     double *__restrict__ partial_rz,
                                                     Scalars *__restrict__ sc)
{
    if (halted(sc)) return;
    double pq[1];
    reduce_partials<1>(partial_pq, t.groups, pq);
    const float alpha = (float)(sc->rho[k & 1] / pq[0]);
    const int g = logical_group(t.groups);
    double acc[2] = {0.0, 0.0};
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t i = (int64_t)tile * TILE + threadIdx.x;
        delta[i] += alpha * p[i];
        const float ri = r[i] - alpha * q[i];
        r[i] = ri;
        const float zi = dinv32[i] * ri;
        acc[0] += (double)ri * (double)zi;
        acc[1] += (double)zi * (double)zi;
    }
    write_partials<2>(acc, partial_rz, t.groups, g);
}

// test of the recursive residual; request a replacement when it passes, every
// rr iterations, or at the cap; otherwise beta and p = z + beta p
__global__ __launch_bounds__(256) void k_cg_direction32(Tiling t, int k, int rr, int max_iter,
                                                        const double *__restrict__ partial_rz,
                                                        const float *__restrict__ dinv32,
                                                        const float *__restrict__ r,
                                                        float *__restrict__ p,
                                                        Scalars *__restrict__ sc)
{
    if (halted(sc)) return;
    double v[2];
    reduce_partials<2>(partial_rz, t.groups, v);
    const double zn = sqrt(v[1]);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (!(zn == zn)) {
        if (lead) {
            sc->nonfinite = 2;
            sc->done = 1;
            sc->iters = k + 1;
            sc->it_next = k + 1;
            sc->znorm = zn;
        }
        return;
    }
    const bool pass = zn < sc->atol || zn < sc->rtol * sc->ref || zn <= sc->floor_;
    if (pass || (rr > 0 && (k + 1) % rr == 0) || k + 1 >= max_iter) {
        if (lead) {
            sc->replace = pass ? 1 : 2;   // 1: the recursive residual passed the test
            sc->it_next = k + 1;
            sc->znorm = zn;
        }
        return;
    }
    const double beta = v[0] / sc->rho[k & 1];
    if (lead) {
        sc->rho[(k + 1) & 1] = v[0];
        sc->it_next = k + 1;
        sc->znorm = zn;
    }
    const float bf = (float)beta;
    const int g = logical_group(t.groups);
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t i = (int64_t)tile * TILE + threadIdx.x;
        p[i] = dinv32[i] * r[i] + bf * p[i];
    }
}

// replacement, part 1: x64 += delta, delta = 0
__global__ __launch_bounds__(256) void k_flush(int64_t n, double *__restrict__ x,
                                               float *__restrict__ delta,
                                               const Scalars *__restrict__ sc)
{
    if (!sc->replace || sc->done) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        x[i] += (double)delta[i];
        delta[i] = 0.0f;
    }
}

// replacement, part 2: r64 = b - A x64 in FP64, r32 = r64; partials r32.z32
// and |D^-1 r64|^2
template <bool NT, typename CI>
__global__ __launch_bounds__(256) void k_true_residual(
    Tiling t, const int64_t *__restrict__ slice_ptr, Cols<CI> col,
    const double *__restrict__ Av, const double *__restrict__ x, const double *__restrict__ b,
    const double *__restrict__ dinv, const float *__restrict__ dinv32, float *__restrict__ r32,
    double *__restrict__ partial, const Scalars *__restrict__ sc)
{
    if (!sc->replace || sc->done) return;
    const int g = logical_group(t.groups);
    const int lane = threadIdx.x & (SLICE - 1);
    double acc[2] = {0.0, 0.0};
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t row = (int64_t)tile * TILE + threadIdx.x;
        const int64_t sl = row / SLICE;
        const int64_t beg = slice_ptr[sl] + lane, end = slice_ptr[sl + 1];
        const int32_t cb = slice_base(col, sl);
        double ax = 0.0;
#pragma unroll 4
        for (int64_t e = beg; e < end; e += SLICE) ax += ld_stream<NT>(Av + e) * x[cb + (int32_t)ld_stream<NT>(col.idx + e)];
        const double ri = b[row] - ax;
        const float rf = (float)ri;
        r32[row] = rf;
        const float zf = dinv32[row] * rf;
        const double zi = dinv[row] * ri;
        acc[0] += (double)rf * (double)zf;
        acc[1] += zi * zi;
    }
    write_partials<2>(acc, partial, t.groups, g);
}

// replacement, part 3 (one workgroup): stopping test on the true residual;
// if it fails, rho and beta for continuing
__global__ __launch_bounds__(256) void k_replace_finalize(int groups, int max_iter,
                                                          const double *__restrict__ partial,
                                                          Scalars *__restrict__ sc)
{
    if (!sc->replace || sc->done) return;
    double v[2];
    reduce_partials<2>(partial, groups, v);
    if (threadIdx.x != 0) return;
    const double zn = sqrt(v[1]);
    const int it = sc->it_next;
    const int why = sc->replace;
    sc->znorm = zn;
    sc->replace = 0;
    if (!(zn == zn)) {
        sc->nonfinite = 2;
        sc->done = 1;
        sc->iters = it;
        return;
    }
    if (zn < sc->atol || zn < sc->rtol * sc->ref || zn <= sc->floor_) {
        sc->done = 1;
        sc->iters = it;
        return;
    }
    if (it >= max_iter || it < 1) return;   // cap: the host reports no convergence
    // The recursive FP32 residual passed but the true one did not: the two have
    // drifted apart, rho of the recursion is no measure of the true residual,
    // and CG restarts from it (p = z).  A periodic replacement keeps the
    // recurrence (beta = rho_new / rho_old).
    sc->beta = why == 1 ? 0.0 : v[0] / sc->rho[(it - 1) & 1];
    sc->rho[it & 1] = v[0];
    sc->redirect = 1;
}

// replacement, part 4: p = z + beta p after a replacement that did not stop
__global__ __launch_bounds__(256) void k_redirect(int64_t n, const float *__restrict__ dinv32,
                                                  const float *__restrict__ r,
                                                  float *__restrict__ p,
                                                  const Scalars *__restrict__ sc)
{
    if (!sc->redirect || sc->done) return;
    const float bf = (float)sc->beta;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = dinv32[i] * r[i] + bf * p[i];
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void launch_to_f32(hipStream_t s, int64_t n, const double *a, float *b)
{
    if (n > 0) hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(n)), dim3(256), 0, s, n, a, b);
}

void launch_rhs_init_mixed(hipStream_t s, const Tiling &t, SellView P, const double *Mv,
                           const double *Kv, const double *dinv, const float *dinv32,
                           const StepParams &sp, const double *V, const double *Vprev,
                           const double *src, double *x, double *b, float *r32, float *delta,
                           double *partial, const double *kdiag, float *kvp, bool nt)
{
    MDX_LAUNCH_SELL(P, nt, k_rhs_init_mixed, dim3(t.groups), dim3(TILE), 0, s, t, P.slice_ptr, cols,
                    Mv, Kv, dinv, dinv32, sp, V, Vprev, src, x, b, r32, delta, partial, kdiag, kvp);
}

void launch_set_direction32(hipStream_t s, int64_t n, const float *dinv32, const float *r32,
                            float *p32, const Scalars *sc)
{
    hipLaunchKernelGGL(k_set_direction32, dim3(blocks_for(n)), dim3(256), 0, s, n, dinv32, r32, p32,
                       sc);
}

void launch_spmv32_dot(hipStream_t s, const Tiling &t, SellView P, const float *A32,
                       const float *p, float *q, double *partial, Scalars *sc,
                       hipEvent_t ev_start, hipEvent_t ev_stop, bool nt)
{
    MDX_LAUNCH_SELL_EV(P, nt, ev_start, ev_stop, k_spmv32_dot, dim3(t.groups), dim3(TILE), 0, s, t,
                       P.slice_ptr, cols, A32, p, q, partial, sc);
}

void launch_cg_update32(hipStream_t s, const Tiling &t, int k, const double *partial_pq,
                        const float *dinv32, const float *p, const float *q, float *delta,
                        float *r, double *partial_rz, Scalars *sc)
{
    hipLaunchKernelGGL(k_cg_update32, dim3(t.groups), dim3(TILE), 0, s, t, k, partial_pq, dinv32, p,
                       q, delta, r, partial_rz, sc);
}

void launch_cg_direction32(hipStream_t s, const Tiling &t, int k, int rr, int max_iter,
                           const double *partial_rz, const float *dinv32, const float *r, float *p,
                           Scalars *sc)
{
    hipLaunchKernelGGL(k_cg_direction32, dim3(t.groups), dim3(TILE), 0, s, t, k, rr, max_iter,
                       partial_rz, dinv32, r, p, sc);
}

void launch_replacement(hipStream_t s, const Tiling &t, SellView P, int max_iter, const double *Av,
                        double *x, float *delta, const double *b, const double *dinv,
                        const float *dinv32, float *r32, float *p32, double *partial, Scalars *sc,
                        bool nt)
{
    const int64_t n = t.n_rows;
    hipLaunchKernelGGL(k_flush, dim3(blocks_for(n)), dim3(256), 0, s, n, x, delta, sc);
    MDX_LAUNCH_SELL(P, nt, k_true_residual, dim3(t.groups), dim3(TILE), 0, s, t, P.slice_ptr, cols,
                    Av, x, b, dinv, dinv32, r32, partial, sc);
    hipLaunchKernelGGL(k_replace_finalize, dim3(1), dim3(TILE), 0, s, t.groups, max_iter, partial,
                       sc);
    hipLaunchKernelGGL(k_redirect, dim3(blocks_for(n)), dim3(256), 0, s, n, dinv32, r32, p32, sc);
}

}  // namespace mdx
