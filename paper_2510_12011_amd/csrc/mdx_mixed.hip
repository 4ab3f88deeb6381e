// Mixed-precision form of the PCG step: FP32 matrix values and FP32 vectors
// in the SpMV and the vector updates of every iteration, FP64 dot products,
// FP64 right-hand side and solution, FP64 residual replacement.
//
// b and r0 = b - A x0 are formed with the FP64 matrices, so the solve
// converges to the solution of the FP64 system: FP32-rounded K loses its zero
// row sums (K 1 = 0 is what conserves charge) and a rounded A is not the
// combination of rounded M and K, and either, applied to V itself, would add
// a small spurious source at every step that accumulates over a run.
//
// The FP32 iteration solves for a correction: x64 stays fixed while
// delta32 accumulates alpha p.  A replacement, triggered every rr
// iterations, when the recursive residual passes the stopping test, or at
// the iteration cap, brings the true residual up to date in FP64,
// r64 -= A delta32 (A's FP32 values, products exact in FP64: the rounding of
// A enters only through the correction, about 6e-8 |delta| / |x| relative),
// then flushes x64 += delta32 -- the stopping test
// is then applied to that true residual, so the solve stops on the same
// criterion as the FP64 path.  If the true residual does not pass, the
// iteration continues from r = r64: after a periodic replacement with
// beta = rho_new / rho_old (the search direction is kept), after one
// triggered by the recursive residual passing the test with p = z (the
// recursion had drifted from the true residual; restart).
//
// Per iteration k (Algorithm 1's recurrences, regrouped), two streaming
// kernels and two single-workgroup finalize kernels:
//   cg_spmv32    beta_k from the scalars; q = A p_k = A z_k + beta_k q_{k-1}
//                and p_k = z_k + beta_k p_{k-1} by linearity of A: the gathers
//                read z, the own rows update p and q; partial p_k . q
//   cg_alpha32   alpha_k = rho_k / p_k.q (fixed-order sum of the partials)
//   cg_update32  delta += alpha p; r -= alpha q; z = D^-1 r (stored);
//                partials r.z, z.z
//   cg_beta32    stopping test of ||z_{k+1}||; beta_{k+1}, rho_{k+1}
// The SpMV kernel runs on its own tiling (one 256-row tile per workgroup by
// default: many short-lived workgroups hide the latency of the gathers), the
// vector kernels on the shared one.  Only the finalize kernels read the
// partials, so the count of SpMV workgroups costs no re-reduction.
//
// Kernels queued after convergence or while a replacement is pending return
// at their first instruction; the replacement kernels return unless one is
// pending.  Reductions are deterministic (fixed-order sums, mdx_device.h).
#include "mdx_device.h"
#include "mdx_internal.h"

#include <hip/hip_ext.h>

namespace mdx {

namespace {

// both flags read in one round trip
__device__ __forceinline__ bool halted(const Scalars *sc) { return (sc->done | sc->replace) != 0; }

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
    double *__restrict__ r64, float *__restrict__ r32, float *__restrict__ z32,
    float *__restrict__ delta, double *__restrict__ partial, const double *__restrict__ kdiag,
    float *__restrict__ kvp, const int32_t *__restrict__ skip)
{
    if (skip && *skip) return;   // the learned guess was taken: nothing to redo
    const int g = logical_group(t.groups);
    const int lane = threadIdx.x & (SLICE - 1);
    const double cK_old = (1.0 - sp.theta) * sp.dt;
    const double cM_new = sp.chi * sp.cm;
    const double cK_new = sp.theta * sp.dt;
    const bool extrap = sp.warm_start == 1;
    double acc[3] = {0.0, 0.0, 0.0};
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t sl = wave_slice(tile);
        const int64_t row = sl * SLICE + lane;
        const int64_t b0 = slice_ptr[sl];
        const int w = (int)((slice_ptr[sl + 1] - b0) / SLICE);
        double mv = 0.0, kv = 0.0, mx = 0.0, kx = 0.0;
        sell_row2<8, NT>(w, col.idx + b0 + lane, Mv + b0 + lane, Kv + b0 + lane,
                         slice_base(col, sl), [&](int32_t c, double m, double kk) {
                             const double vj = V[c], vpj = Vprev[c];
                             const double x0j = extrap ? 2.0 * vj - vpj : vj;
                             mv += m * (sp.cm * vj + sp.dt * src[c]);
                             kv += kk * vj;
                             mx += m * x0j;
                             kx += kk * x0j;
                         });
        const double bi = sp.chi * mv - cK_old * kv;
        const double ri = bi - (cM_new * mx + cK_new * kx);
        const double vi = V[row];
        x[row] = extrap ? 2.0 * vi - Vprev[row] : vi;
        r64[row] = ri;
        if (kvp) kvp[row] = kdiag[row] != 0.0 ? (float)(kv / kdiag[row]) : 0.0f;
        const float rf = (float)ri;
        r32[row] = rf;
        delta[row] = 0.0f;
        const float zf = dinv32[row] * rf;
        z32[row] = zf;
        const double zi = dinv[row] * ri, di = dinv[row] * bi;
        acc[0] += (double)rf * (double)zf;
        acc[1] += zi * zi;
        acc[2] += di * di;
    }
    write_partials<3>(acc, partial, t.groups, g);
}

// Stopping test of the mixed iteration on ||z_k|| (zn): 0 continue; 1 the
// recursive residual passes; 2 periodic replacement (every rr iterations)
// or the iteration cap.  A NaN stops the solve and flags it.
__device__ __forceinline__ int test_z(Scalars *sc, const StopTest &st, double zn, int k, int rr,
                                      int max_iter, bool lead)
{
    if (!isfinite(zn)) {
        if (lead) {
            sc->nonfinite = 2;
            sc->done = 1;
            sc->iters = k;
            sc->it_next = k;
            sc->znorm = zn;
        }
        return -1;
    }
    const bool pass = passes(st, zn);
    const int why = pass ? 1 : (rr > 0 && k % rr == 0) || k >= max_iter ? 2 : 0;
    if (why && lead) {
        sc->replace = why;
        sc->it_next = k;
        sc->znorm = zn;
    }
    return why;
}

// Iteration k, SpMV half (see the file comment); beta_k = 0 (the start,
// or a restart after a replacement) takes p = z, q = A z without reading the
// earlier p, q.
template <bool NT, typename CI>
__global__ __launch_bounds__(256) void k_cg_spmv32(Tiling t, const int64_t *__restrict__ slice_ptr,
                                                   Cols<CI> col, const float *__restrict__ A32,
                                                   const float *__restrict__ z,
                                                   float *__restrict__ p, float *__restrict__ q,
                                                   double *__restrict__ partial_pq,
                                                   const Scalars *__restrict__ sc)
{
    if (halted(sc)) return;
    const double beta = sc->beta;
    const bool fresh = beta == 0.0;
    const float bf = (float)beta;
    const int g = logical_group(t.groups);
    const int lane = threadIdx.x & (SLICE - 1);
    double acc[1] = {0.0};
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t sl = wave_slice(tile);
        const int64_t row = sl * SLICE + lane;
        const int64_t b0 = slice_ptr[sl];
        const int w = (int)((slice_ptr[sl + 1] - b0) / SLICE);
        const int32_t cb = slice_base(col, sl);
        const float zi = z[row];
        const float pold = fresh ? 0.0f : p[row], qold = fresh ? 0.0f : q[row];
        const float sum = sell_row<NT, float>(w, col.idx + b0 + lane, A32 + b0 + lane, z, cb);
        const float pi = fresh ? zi : zi + bf * pold;
        const float qi = fresh ? sum : sum + bf * qold;
        p[row] = pi;
        q[row] = qi;
        acc[0] += (double)pi * (double)qi;
    }
    write_partials<1>(acc, partial_pq, t.groups, g);
}

// Iteration k: alpha_k = rho_k / (p_k . q) from the SpMV's partials.
__global__ __launch_bounds__(FIN) void k_cg_alpha32(int groups, int k,
                                                    const double *__restrict__ partial_pq,
                                                    Scalars *__restrict__ sc)
{
    const double rho = sc->rho[k & 1];   // read with the verdict
    if (halted(sc)) return;
    double pq[1];
    finalize_partials<1>(partial_pq, groups, pq);
    if (threadIdx.x == 0) {
        sc->alpha = rho / pq[0];
        sc->it_next = k + 1;
    }
}

// Iteration k, update half: delta += alpha p; r -= alpha q; z = D^-1 r;
// partials r.z and z.z for the next test.
__global__ __launch_bounds__(256) void k_cg_update32(Tiling t, const float *__restrict__ dinv32,
                                                     const float *__restrict__ p,
                                                     const float *__restrict__ q,
                                                     float *__restrict__ delta,
                                                     float *__restrict__ r, float *__restrict__ z,
                                                     double *__restrict__ partial_rz,
                                                     const Scalars *__restrict__ sc)
{
    if (halted(sc)) return;
    const float alpha = (float)sc->alpha;
    const int g = logical_group(t.groups);
    double acc[2] = {0.0, 0.0};
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t i = (int64_t)tile * TILE + threadIdx.x;
        delta[i] += alpha * p[i];
        const float ri = r[i] - alpha * q[i];
        r[i] = ri;
        const float zi = dinv32[i] * ri;
        z[i] = zi;
        acc[0] += (double)ri * (double)zi;
        acc[1] += (double)zi * (double)zi;
    }
    write_partials<2>(acc, partial_rz, t.groups, g);
}

// After iteration k's update (k1 = k + 1): the stopping test of ||z_k1||; if
// the iteration goes on, beta_k1 = rho_k1 / rho_k.
__global__ __launch_bounds__(FIN) void k_cg_beta32(int groups, int k1, int rr, int max_iter,
                                                   const double *__restrict__ partial_rz,
                                                   Scalars *__restrict__ sc)
{
    const StopTest st = stop_test(sc);   // read with the verdict
    const double rho_prev = sc->rho[(k1 - 1) & 1];
    if (halted(sc)) return;
    double v[2];
    finalize_partials<2>(partial_rz, groups, v);
    const bool lead = threadIdx.x == 0;
    const double zn = sqrt(v[1]);
    if (test_z(sc, st, zn, k1, rr, max_iter, lead)) return;
    if (lead) {
        sc->beta = v[0] / rho_prev;
        sc->rho[k1 & 1] = v[0];
        sc->znorm = zn;
    }
}

// replacement, part 2: x64 += delta, delta = 0
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

// replacement, part 1: the true residual of x64 + delta brought up to date
// in FP64, r64 -= A delta, r32 = r64, z32 = D^-1 r32; partials r32.z32 and
// |D^-1 r64|^2.  r64 starts as b - A x0 formed in FP64 by the right-hand-side
// pass; each product of an FP32 value of A and the FP32 correction is exact
// in FP64, so only A's FP32 rounding enters, and only through delta.
template <bool NT, typename CI>
__global__ __launch_bounds__(256) void k_true_residual(
    Tiling t, const int64_t *__restrict__ slice_ptr, Cols<CI> col,
    const float *__restrict__ A32, const float *__restrict__ delta, double *__restrict__ r64,
    const double *__restrict__ dinv, const float *__restrict__ dinv32, float *__restrict__ r32,
    float *__restrict__ z32, double *__restrict__ partial, const Scalars *__restrict__ sc)
{
    if (!sc->replace || sc->done) return;
    const int g = logical_group(t.groups);
    const int lane = threadIdx.x & (SLICE - 1);
    double acc[2] = {0.0, 0.0};
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t sl = wave_slice(tile);
        const int64_t row = sl * SLICE + lane;
        const int64_t b0 = slice_ptr[sl];
        const int w = (int)((slice_ptr[sl + 1] - b0) / SLICE);
        const double ad =
            sell_row<NT, double>(w, col.idx + b0 + lane, A32 + b0 + lane, delta, slice_base(col, sl));
        const double ri = r64[row] - ad;
        r64[row] = ri;
        const float rf = (float)ri;
        r32[row] = rf;
        const float zf = dinv32[row] * rf;
        z32[row] = zf;
        const double zi = dinv[row] * ri;
        acc[0] += (double)rf * (double)zf;
        acc[1] += zi * zi;
    }
    write_partials<2>(acc, partial, t.groups, g);
}

// replacement, part 3 (one workgroup): stopping test on the true residual;
// if it fails, iteration it restarts from it with rho and beta set here
__global__ __launch_bounds__(TILE) void k_replace_finalize(int groups, int max_iter,
                                                          const double *__restrict__ partial,
                                                          Scalars *__restrict__ sc)
{
    // everything read from the scalars is read with the verdict
    const StopTest st = stop_test(sc);
    const int it = sc->it_next;
    const int why = sc->replace;
    const double rho01[2] = {sc->rho[0], sc->rho[1]};
    if (!why || sc->done) return;
    double v[2];
    finalize_partials<2, TILE>(partial, groups, v);
    if (threadIdx.x != 0) return;
    const double zn = sqrt(v[1]);
    sc->znorm = zn;
    sc->replace = 0;
    if (!isfinite(zn)) {
        sc->nonfinite = 2;
        sc->done = 1;
        sc->iters = it;
        return;
    }
    if (passes(st, zn)) {
        sc->done = 1;
        sc->iters = it;
        return;
    }
    if (it >= max_iter || it < 1) return;   // cap: the host reports no convergence
    // The recursive FP32 residual passed but the true one did not: the two have
    // drifted apart, rho of the recursion is no measure of the true residual,
    // and CG restarts from it (p = z).  A periodic replacement keeps the
    // recurrence (beta = rho_new / rho_old).
    sc->beta = why == 1 ? 0.0 : v[0] / rho01[(it - 1) & 1];
    sc->rho[it & 1] = v[0];
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
                           const double *src, double *x, double *r64, float *r32, float *z32,
                           float *delta, double *partial, const double *kdiag, float *kvp, bool nt,
                           const int32_t *skip)
{
    MDX_LAUNCH_SELL(P, nt, k_rhs_init_mixed, dim3(t.groups), dim3(TILE), 0, s, t, P.slice_ptr, cols,
                    Mv, Kv, dinv, dinv32, sp, V, Vprev, src, x, r64, r32, z32, delta, partial, kdiag,
                    kvp, skip);
}

void launch_cg_iteration32(hipStream_t s, const Tiling &ts, const Tiling &t, int k, int rr,
                           int max_iter, SellView P, const float *A32, const float *dinv32,
                           float *z, float *p, float *q, float *delta, float *r,
                           double *partial_pq, double *partial_rz, Scalars *sc,
                           hipEvent_t ev_start, hipEvent_t ev_stop, bool nt)
{
    MDX_LAUNCH_SELL_EV(P, nt, ev_start, ev_stop, k_cg_spmv32, dim3(ts.groups), dim3(TILE), 0, s, ts,
                       P.slice_ptr, cols, A32, z, p, q, partial_pq, sc);
    hipLaunchKernelGGL(k_cg_alpha32, dim3(1), dim3(FIN), 0, s, ts.groups, k, partial_pq, sc);
    hipLaunchKernelGGL(k_cg_update32, dim3(t.groups), dim3(TILE), 0, s, t, dinv32, p, q, delta, r,
                       z, partial_rz, sc);
    hipLaunchKernelGGL(k_cg_beta32, dim3(1), dim3(FIN), 0, s, t.groups, k + 1, rr, max_iter,
                       partial_rz, sc);
}

void launch_replacement(hipStream_t s, const Tiling &t, SellView P, int max_iter, const float *A32,
                        double *x, float *delta, double *r64, const double *dinv,
                        const float *dinv32, float *r32, float *z32, double *partial, Scalars *sc,
                        bool nt)
{
    const int64_t n = t.n_rows;
    MDX_LAUNCH_SELL(P, nt, k_true_residual, dim3(t.groups), dim3(TILE), 0, s, t, P.slice_ptr, cols,
                    A32, delta, r64, dinv, dinv32, r32, z32, partial, sc);
    hipLaunchKernelGGL(k_flush, dim3(blocks_for(n)), dim3(256), 0, s, n, x, delta, sc);
    hipLaunchKernelGGL(k_replace_finalize, dim3(1), dim3(TILE), 0, s, t.groups, max_iter, partial,
                       sc);
}

}  // namespace mdx
