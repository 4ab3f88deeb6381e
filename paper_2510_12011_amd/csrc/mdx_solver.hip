// Per-step solver kernels of the plain FP64 path.
//
// One time step (the paper's Eq. 2 and the definitions of A and b after
// Eq. 3, Jacobi-PCG of Algorithm 1):
//   rhs_init      b = chi M (Cm V^k + dt s) - (1-theta) dt K V^k,  s = I_stim - I_ion
//                 (formed per row, not stored),
//                 x0 = 2V^k - V^{k-1} (or V^k), r0 = b - A x0 with
//                 A x0 = chi Cm (M x0) + theta dt (K x0), p0 = z0 = D^-1 r0,
//                 per-workgroup partials of r.z, z.z, |D^-1 b|^2
//   init_finalize rho_0, ||z_0||, the stopping reference, done if z_0 is at the
//                 rounding floor
//   per iteration k, two streaming kernels (the default: three) and two
//   single-workgroup finalize kernels:
//   cg_spmv       beta_k from the scalars; q = A p_k = A z_k + beta_k q_{k-1}
//                 and p_k = z_k + beta_k p_{k-1} (A is linear: the gathers
//                 read z only); partial p_k . q
//   (or spmv_dot  q = A p_k with partial p_k . q)
//   cg_alpha      alpha_k = rho_k / p_k.q
//   cg_update     x += alpha p_k; r -= alpha q; z = D^-1 r (stored for
//                 cg_spmv); partials r.z, z.z
//   cg_beta       stopping test of ||z_{k+1}|| (< atol, < rtol * ref, or at
//                 the floor); beta_{k+1} = rho_{k+1} / rho_k
//   (cg_direction p_{k+1} = z_{k+1} + beta_{k+1} p_k, with spmv_dot)
//   epilogue      activation / repolarisation times, non-finite check
//
// Matrix traversal: sliced ELL (see mdx_internal.h); one lane per row, so the
// j-th column/value loads of a wavefront are contiguous; a row's loads are
// all issued before its gathers (sell_row).  The SpMV kernels run one 256-row
// tile per workgroup by default: many short-lived workgroups hide the
// gathers' latency.  Workgroups are remapped so that each of the 8 XCDs owns
// a contiguous eighth of the rows: the x-gathers of neighbouring rows (RCM
// keeps them within the bandwidth) then hit that XCD's own L2.
//
// Reductions: wavefront butterfly (shfl_xor) -> LDS across the wavefronts
// -> one partial per workgroup; a single-workgroup finalize kernel sums the
// partials in a fixed order and writes the scalar the next kernel reads, so
// runs are deterministic; no atomics, no grid-wide synchronisation.
#include "mdx_device.h"
#include "mdx_internal.h"

#include <hip/hip_ext.h>

#include <algorithm>

namespace mdx {

Tiling make_tiling(int64_t n_rows_padded, int max_groups)
{
    Tiling t;
    t.n_rows = n_rows_padded;
    t.n_tiles = (int)(n_rows_padded / TILE);
    int g = std::max(1, std::min(t.n_tiles, max_groups));
    t.tpb = (t.n_tiles + g - 1) / g;
    t.groups = (t.n_tiles + t.tpb - 1) / t.tpb;
    return t;
}

namespace {

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fill(int64_t n, double v, double *__restrict__ x)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ __launch_bounds__(256) void k_stim_add(int64_t n_idx, const int32_t *__restrict__ idx,
                                                  double amp, double *__restrict__ istim)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n_idx) istim[idx[j]] += amp;   // node lists are duplicate-free
}

template <bool NT, typename CI>
__global__ __launch_bounds__(256) void k_rhs_init(
    Tiling t, const int64_t *__restrict__ slice_ptr, Cols<CI> col,
    const double *__restrict__ Mv, const double *__restrict__ Kv, const double *__restrict__ dinv,
    StepParams sp, const double *__restrict__ V, const double *__restrict__ Vprev,
    const double *__restrict__ src, double *__restrict__ x, double *__restrict__ r,
    double *__restrict__ partial, const double *__restrict__ kdiag, float *__restrict__ kvp,
    double *__restrict__ p0, const int32_t *__restrict__ skip)
{
    if (skip && *skip) return;   // the learned guess was taken: nothing to redo
    const int g = logical_group(t.groups);
    const int lane = threadIdx.x & (SLICE - 1);
    const double cK_old = (1.0 - sp.theta) * sp.dt;   // weight of K V^k in b
    const double cM_new = sp.chi * sp.cm;             // A = cM_new M + cK_new K
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
        const double ax = cM_new * mx + cK_new * kx;
        const double vi = V[row];
        const double x0i = extrap ? 2.0 * vi - Vprev[row] : vi;
        const double di = dinv[row];
        const double ri = bi - ax;
        const double zi = di * ri;
        x[row] = x0i;
        r[row] = ri;
        if (p0) p0[row] = zi;   // the first direction p0 = z0
        if (kvp) kvp[row] = kdiag[row] != 0.0 ? (float)(kv / kdiag[row]) : 0.0f;
        acc[0] += ri * zi;
        acc[1] += zi * zi;
        acc[2] += (di * bi) * (di * bi);
    }
    write_partials<3>(acc, partial, t.groups, g);
}

// Initial residual of a given system (the standalone solve): r = b - A x,
// z = D^-1 r, p0 = z; partials r.z, z.z and |D^-1 b|^2 in the layout
// k_init_finalize reads.
template <bool NT, typename CI>
__global__ __launch_bounds__(256) void k_residual_init(
    Tiling t, const int64_t *__restrict__ slice_ptr, Cols<CI> col, const double *__restrict__ Av,
    const double *__restrict__ dinv, const double *__restrict__ b, const double *__restrict__ x,
    double *__restrict__ r, double *__restrict__ p0, double *__restrict__ partial)
{
    const int g = logical_group(t.groups);
    const int lane = threadIdx.x & (SLICE - 1);
    double acc[3] = {0.0, 0.0, 0.0};
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t row = (int64_t)tile * TILE + threadIdx.x;
        const int64_t sl = row / SLICE;
        const int64_t beg = slice_ptr[sl] + lane, end = slice_ptr[sl + 1];
        const int32_t cb = slice_base(col, sl);
        double ax = 0.0;
        for (int64_t e = beg; e < end; e += SLICE)
            ax += ld_stream<NT>(Av + e) * x[cb + (int32_t)ld_stream<NT>(col.idx + e)];
        const double di = dinv[row], bi = b[row];
        const double ri = bi - ax, zi = di * ri;
        r[row] = ri;
        p0[row] = zi;
        acc[0] += ri * zi;
        acc[1] += zi * zi;
        acc[2] += (di * bi) * (di * bi);
    }
    write_partials<3>(acc, partial, t.groups, g);
}

__global__ __launch_bounds__(TILE) void k_init_finalize(int groups, const double *__restrict__ partial,
                                                       int rel_mode, Scalars *__restrict__ sc,
                                                       const int32_t *__restrict__ skip)
{
    if (skip && *skip) return;
    const double atol = sc->atol;
    double v[3];
    finalize_partials<3, TILE>(partial, groups, v);
    if (threadIdx.x == 0) {
        const double z0 = sqrt(v[1]);
        const double db = sqrt(v[2]);
        sc->rho[0] = v[0];
        sc->z0 = z0;
        sc->znorm = z0;
        sc->ref = rel_mode == 1 ? db : z0;
        const double floor_ = 1e-15 * db;
        sc->floor_ = floor_;
        // a non-finite start (NaN, or a norm that overflowed) ends the solve
        // and is reported; a finite one clears the flag of an earlier solve
        const bool finite = isfinite(z0) && isfinite(db) && isfinite(v[0]);
        sc->nonfinite = finite ? 0 : 2;
        sc->done = (!finite || z0 <= floor_ || z0 < atol) ? 1 : 0;
        sc->iters = 0;
        sc->replace = 0;
        sc->beta = 0.0;
        sc->it_next = 0;
    }
}

template <bool NT, typename CI>
__global__ __launch_bounds__(256) void k_spmv_dot(Tiling t, const int64_t *__restrict__ slice_ptr,
                                                  Cols<CI> col,
                                                  const double *__restrict__ Av,
                                                  const double *__restrict__ p,
                                                  double *__restrict__ q,
                                                  double *__restrict__ partial,
                                                  const int32_t *__restrict__ done)
{
    if (*done) return;
    const int g = logical_group(t.groups);
    const int lane = threadIdx.x & (SLICE - 1);
    double acc[1] = {0.0};
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t sl = wave_slice(tile);
        const int64_t row = sl * SLICE + lane;
        const int64_t b0 = slice_ptr[sl];
        const int w = (int)((slice_ptr[sl + 1] - b0) / SLICE);
        const double pi = p[row];
        const double sum =
            sell_row<NT, double>(w, col.idx + b0 + lane, Av + b0 + lane, p, slice_base(col, sl));
        q[row] = sum;
        acc[0] += pi * sum;
    }
    write_partials<1>(acc, partial, t.groups, g);
}

// Iteration k, SpMV half of the two-kernel scheme: beta_k from the
// scalars, then, A being linear,
//   q = A p_k = A z_k + beta_k q_{k-1},   p_k = z_k + beta_k p_{k-1}:
// the gathers read z_k only (z_0 written by the pass that forms r_0), own
// rows update p and q in place; beta_0 = 0 takes p = z, q = A z without
// reading the earlier p, q; partial p_k . q.
template <bool NT, typename CI>
__global__ __launch_bounds__(256) void k_cg_spmv(Tiling t, const int64_t *__restrict__ slice_ptr,
                                                 Cols<CI> col, const double *__restrict__ Av,
                                                 const double *__restrict__ z,
                                                 double *__restrict__ p, double *__restrict__ q,
                                                 double *__restrict__ partial_pq,
                                                 const Scalars *__restrict__ sc)
{
    if (sc->done) return;
    const double beta = sc->beta;
    const bool fresh = beta == 0.0;
    const int g = logical_group(t.groups);
    const int lane = threadIdx.x & (SLICE - 1);
    double acc[1] = {0.0};
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t sl = wave_slice(tile);
        const int64_t row = sl * SLICE + lane;
        const int64_t b0 = slice_ptr[sl];
        const int w = (int)((slice_ptr[sl + 1] - b0) / SLICE);
        const double zi = z[row];
        const double pold = fresh ? 0.0 : p[row], qold = fresh ? 0.0 : q[row];
        const double sum =
            sell_row<NT, double>(w, col.idx + b0 + lane, Av + b0 + lane, z, slice_base(col, sl));
        const double pi = fresh ? zi : zi + beta * pold;
        const double qi = fresh ? sum : sum + beta * qold;
        p[row] = pi;
        q[row] = qi;
        acc[0] += pi * qi;
    }
    write_partials<1>(acc, partial_pq, t.groups, g);
}

// Iteration k: alpha_k = rho_k / (p_k . q) from the SpMV's partials.
__global__ __launch_bounds__(FIN) void k_cg_alpha(int groups, int k,
                                                  const double *__restrict__ partial_pq,
                                                  Scalars *__restrict__ sc)
{
    const double rho = sc->rho[k & 1];   // read with the verdict
    if (sc->done) return;
    double pq[1];
    finalize_partials<1>(partial_pq, groups, pq);
    if (threadIdx.x == 0) sc->alpha = rho / pq[0];
}

// Iteration k, update half: x += alpha_k p_k; r -= alpha_k q; z = D^-1 r
// (stored when z is given); partials r.z and z.z for the next test.
__global__ __launch_bounds__(256) void k_cg_update(Tiling t, const double *__restrict__ dinv,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ q,
                                                   double *__restrict__ x, double *__restrict__ r,
                                                   double *__restrict__ z,
                                                   double *__restrict__ partial_rz,
                                                   const Scalars *__restrict__ sc)
{
    if (sc->done) return;
    const double alpha = sc->alpha;
    const int g = logical_group(t.groups);
    double acc[2] = {0.0, 0.0};
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t i = (int64_t)tile * TILE + threadIdx.x;
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        const double zi = dinv[i] * ri;
        if (z) z[i] = zi;
        acc[0] += ri * zi;
        acc[1] += zi * zi;
    }
    write_partials<2>(acc, partial_rz, t.groups, g);
}

// After iteration k's update (k1 = k + 1): Algorithm 1's stopping test on
// ||z_k1|| (the solve ends after k1 iterations), else beta_k1 =
// rho_k1 / rho_k.  At k1 == max_iter it only tests: the cap is reached and the
// host reports no convergence.
__global__ __launch_bounds__(FIN) void k_cg_beta(int groups, int k1, int max_iter,
                                                 const double *__restrict__ partial_rz,
                                                 Scalars *__restrict__ sc)
{
    const StopTest st = stop_test(sc);   // read with the verdict
    const double rho_prev = sc->rho[(k1 - 1) & 1];
    if (sc->done) return;
    double v[2];
    finalize_partials<2>(partial_rz, groups, v);
    if (threadIdx.x != 0) return;
    const double zn = sqrt(v[1]);
    sc->znorm = zn;
    if (!isfinite(zn)) {   // NaN or overflow: stop the solve and flag it
        sc->nonfinite = 2;
        sc->done = 1;
        sc->iters = k1;
        return;
    }
    if (passes(st, zn)) {
        sc->done = 1;
        sc->iters = k1;
        return;
    }
    if (k1 >= max_iter) return;
    sc->beta = v[0] / rho_prev;
    sc->rho[k1 & 1] = v[0];
}

// Three-kernel scheme, last kernel of iteration k: p = z + beta p in place
// (p and the SpMV input are the same buffer), z = D^-1 r formed here.
__global__ __launch_bounds__(256) void k_cg_direction(Tiling t, const double *__restrict__ dinv,
                                                      const double *__restrict__ r,
                                                      double *__restrict__ p,
                                                      const Scalars *__restrict__ sc)
{
    if (sc->done) return;
    const double beta = sc->beta;
    const int g = logical_group(t.groups);
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t i = (int64_t)tile * TILE + threadIdx.x;
        p[i] = dinv[i] * r[i] + beta * p[i];
    }
}

// z_0 -> p (three-kernel scheme starts from p_0 = z_0)
__global__ __launch_bounds__(256) void k_set_direction(int64_t n, const double *__restrict__ dinv,
                                                       const double *__restrict__ r,
                                                       double *__restrict__ p,
                                                       const Scalars *__restrict__ sc)
{
    if (sc->done) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = dinv[i] * r[i];
}

__global__ __launch_bounds__(256) void k_epilogue(int64_t n, double t1, const double *__restrict__ Vold,
                                                  const double *__restrict__ Vnew,
                                                  double *__restrict__ lat, double *__restrict__ lrt,
                                                  Scalars *__restrict__ sc,
                                                  const int32_t *__restrict__ guard)
{
    if (guard && !*guard) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!update_times(i, t1, Vold[i], Vnew[i], lat, lrt)) sc->nonfinite = 1;
}

// One wavefront: the scalars (whole 4-byte words) into host-visible memory,
// a system-scope fence, then the sequence number the host waits for.
__global__ __launch_bounds__(64) void k_publish(const Scalars *__restrict__ sc, Published *pub,
                                                int32_t seq)
{
    static_assert(sizeof(Scalars) % 4 == 0, "whole words");
    constexpr int words = (int)(sizeof(Scalars) / 4);
    const int32_t *src = reinterpret_cast<const int32_t *>(sc);
    int32_t *dst = reinterpret_cast<int32_t *>(&pub->s);
    for (int w = threadIdx.x; w < words; w += 64) dst[w] = src[w];
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) pub->seq = seq;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void launch_fill(hipStream_t s, int64_t n, double v, double *x)
{
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(256), 0, s, n, v, x);
}

void launch_stim_add(hipStream_t s, int64_t n_idx, const int32_t *idx, double amp, double *istim)
{
    if (n_idx > 0)
        hipLaunchKernelGGL(k_stim_add, dim3(blocks_for(n_idx)), dim3(256), 0, s, n_idx, idx, amp,
                           istim);
}

void launch_rhs_init(hipStream_t s, const Tiling &t, SellView P, const double *Mv,
                     const double *Kv, const double *dinv, const StepParams &sp, const double *V,
                     const double *Vprev, const double *src, double *x, double *r,
                     double *partial, const double *kdiag, float *kvp, double *p0, bool nt,
                     const int32_t *skip)
{
    MDX_LAUNCH_SELL(P, nt, k_rhs_init, dim3(t.groups), dim3(TILE), 0, s, t, P.slice_ptr, cols, Mv,
                    Kv, dinv, sp, V, Vprev, src, x, r, partial, kdiag, kvp, p0, skip);
}

void launch_residual_init(hipStream_t s, const Tiling &t, SellView P, const double *Av,
                          const double *dinv, const double *b, const double *x, double *r,
                          double *p0, double *partial)
{
    MDX_LAUNCH_SELL(P, false, k_residual_init, dim3(t.groups), dim3(TILE), 0, s, t, P.slice_ptr,
                    cols, Av, dinv, b, x, r, p0, partial);
}

void launch_init_finalize(hipStream_t s, const Tiling &t, const double *partial, int rel_mode,
                          Scalars *sc, const int32_t *skip)
{
    hipLaunchKernelGGL(k_init_finalize, dim3(1), dim3(TILE), 0, s, t.groups, partial, rel_mode, sc,
                       skip);
}

void launch_spmv_dot(hipStream_t s, const Tiling &t, SellView P, const double *Av, const double *p,
                     double *q, double *partial, const int32_t *done, hipEvent_t ev_start,
                     hipEvent_t ev_stop, bool nt)
{
    MDX_LAUNCH_SELL_EV(P, nt, ev_start, ev_stop, k_spmv_dot, dim3(t.groups), dim3(TILE), 0, s, t,
                       P.slice_ptr, cols, Av, p, q, partial, done);
}

void launch_cg_iteration(hipStream_t s, const Tiling &ts, const Tiling &t, int k, int max_iter,
                         int scheme, SellView P, const double *Av, const double *dinv, double *r,
                         double *z, double *p, double *q, double *x, double *partial_pq,
                         double *partial_rz, Scalars *sc, hipEvent_t ev_start, hipEvent_t ev_stop,
                         bool nt)
{
    if (scheme == 1)
        MDX_LAUNCH_SELL_EV(P, nt, ev_start, ev_stop, k_cg_spmv, dim3(ts.groups), dim3(TILE), 0, s,
                           ts, P.slice_ptr, cols, Av, z, p, q, partial_pq, sc);
    else
        MDX_LAUNCH_SELL_EV(P, nt, ev_start, ev_stop, k_spmv_dot, dim3(ts.groups), dim3(TILE), 0, s,
                           ts, P.slice_ptr, cols, Av, p, q, partial_pq, &sc->done);
    hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(FIN), 0, s, ts.groups, k, partial_pq, sc);
    hipLaunchKernelGGL(k_cg_update, dim3(t.groups), dim3(TILE), 0, s, t, dinv, p, q, x, r,
                       scheme == 1 ? z : nullptr, partial_rz, sc);
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(FIN), 0, s, t.groups, k + 1, max_iter, partial_rz,
                       sc);
    if (scheme != 1)
        hipLaunchKernelGGL(k_cg_direction, dim3(t.groups), dim3(TILE), 0, s, t, dinv, r, p, sc);
}

void launch_set_direction(hipStream_t s, int64_t n, const double *dinv, const double *r, double *p,
                          const Scalars *sc)
{
    hipLaunchKernelGGL(k_set_direction, dim3(blocks_for(n)), dim3(256), 0, s, n, dinv, r, p, sc);
}

void launch_epilogue(hipStream_t s, int64_t n, double t1, const double *Vold, const double *Vnew,
                     double *lat, double *lrt, Scalars *sc, const int32_t *guard)
{
    if (n > 0)
        hipLaunchKernelGGL(k_epilogue, dim3(blocks_for(n)), dim3(256), 0, s, n, t1, Vold, Vnew, lat,
                           lrt, sc, guard);
}

void launch_publish(hipStream_t s, const Scalars *sc, Published *pub, int32_t seq)
{
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, sc, pub, seq);
}

}  // namespace mdx
