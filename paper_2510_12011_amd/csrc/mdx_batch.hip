// Batched form: many independent monodomain systems in one block-diagonal
// matrix, solved together by the mixed-precision PCG (FP32 matrix values and
// vectors in the iteration, FP64 right-hand side, solution, dot products and
// residual replacement), with one set of CG scalars per instance.
//
// Per time step (after the pointwise ionic update over all rows):
//   b_rhs_init        b, x0, r0 = b - A x0 (FP64 M and K), r32, delta = 0;
//                     per-group partials r.z, |D^-1 r0|^2, |D^-1 b|^2
//   b_init_finalize   one workgroup per instance: rho_0, ||z_0||, stopping
//                     reference and rounding floor
//   b_set_direction   p_0 = z_0
//   per iteration:    spmv (q = A p, p.q), alpha (per instance), update
//                     (x, r, z; r.z, z.z), beta (per instance: test, replacement
//                     trigger, beta), direction (p = z + beta p)
//   replacement       flush (x64 += delta), true residual in FP64, finalize
//                     (stop or continue), redirect
// Every kernel returns at once for the workgroups of an instance that has
// finished (or, for the iteration kernels, waits for a replacement), so
// converged instances cost no memory traffic while the others iterate; the
// host stops when every instance is done.
//
// The iteration's SpMV takes the matrix in the layout chosen by the
// autotuner: sliced ELL with lpr lanes per row (64/lpr rows per wavefront,
// the lanes of a row summed by a butterfly over adjacent lanes), sliced ELL
// read with 16-byte vector loads (4 entries per lane and load), or CSR with
// 4-16 lanes per row.
//
// Optionally (k_b_persistent) a chunk of iterations runs as one launch whose
// workgroups are all resident: the workgroups of an instance meet at
// barriers of their own (a generation counter per instance, a bounded wait
// that raises a fault flag instead of hanging) between the SpMV, the update
// and the direction, and each instance iterates until its next residual
// replacement.
#include "mdx_device.h"
#include "mdx_internal.h"

#include <hip/hip_ext.h>

namespace mdx {

namespace {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bool stopped(const BScalars &s) { return s.done != 0; }
__device__ __forceinline__ bool idle(const BScalars &s) { return (s.done | s.replace) != 0; }

// Sum NV per-group partials of groups [g0, g1) (layout partial[k * groups + g]):
// thread t adds g0 + t, g0 + t + TILE, ... in turn, then the workgroup sum.
// Up to U of a thread's loads are issued before its first add.
template <int NV>
__device__ __forceinline__ void reduce_range(const double *__restrict__ partial, int groups, int g0,
                                             int g1, double (&v)[NV])
{
    constexpr int U = 8;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    for (int gb = g0 + (int)threadIdx.x; gb < g1; gb += U * TILE) {
        double t[U][NV];
#pragma unroll
        for (int j = 0; j < U; ++j)
#pragma unroll
            for (int k = 0; k < NV; ++k)
                t[j][k] = gb + j * TILE < g1 ? partial[k * groups + gb + j * TILE] : 0.0;
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (gb + j * TILE < g1)
#pragma unroll
                for (int k = 0; k < NV; ++k) v[k] += t[j][k];
    }
    group_sum<NV>(v);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_relayout(int lpr, int64_t n_slices,
                                                  const int64_t *__restrict__ sptr_new,
                                                  const int64_t *__restrict__ sptr,
                                                  const int32_t *__restrict__ col,
                                                  const float *__restrict__ A32,
                                                  int32_t *__restrict__ col_new,
                                                  float *__restrict__ A32_new)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t sl = tid / SLICE;
    if (sl >= n_slices) return;
    const int lane = (int)(tid % SLICE);
    const int H = SLICE / lpr;
    const int64_t row = sl * H + lane / lpr;
    const int sub = lane % lpr;
    const int64_t bsl = row / SLICE;
    const int64_t bbase = sptr[bsl] + (row % SLICE);
    const int64_t bw = (sptr[bsl + 1] - sptr[bsl]) / SLICE;   // base width of the row's slice
    const int64_t w = (sptr_new[sl + 1] - sptr_new[sl]) / SLICE;
    for (int64_t j = 0; j < w; ++j) {
        const int64_t k = j * lpr + sub;   // entry of the row
        const int64_t e = sptr_new[sl] + j * SLICE + lane;
        if (k < bw) {
            col_new[e] = col[bbase + k * SLICE];
            A32_new[e] = A32[bbase + k * SLICE];
        } else {
            col_new[e] = (int32_t)row;
            A32_new[e] = 0.0f;
        }
    }
}

// base layout -> 64-row slices whose lanes hold 4 consecutive entries of
// their row per 256-slot step (entry k of the row in slice position l at
// sptr_new[slice] + 256 (k / 4) + 4 l + k % 4), for 16-byte vector loads
__global__ __launch_bounds__(256) void k_relayout_v4(int64_t n_slices,
                                                     const int64_t *__restrict__ sptr_new,
                                                     const int64_t *__restrict__ sptr,
                                                     const int32_t *__restrict__ col,
                                                     const float *__restrict__ A32,
                                                     int32_t *__restrict__ col_new,
                                                     float *__restrict__ A32_new)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t sl = tid / SLICE;
    if (sl >= n_slices) return;
    const int lane = (int)(tid % SLICE);
    const int64_t row = sl * SLICE + lane;
    const int64_t bbase = sptr[sl] + lane;
    const int64_t bw = (sptr[sl + 1] - sptr[sl]) / SLICE;
    const int64_t w4 = (sptr_new[sl + 1] - sptr_new[sl]) / (4 * SLICE);
    for (int64_t c = 0; c < w4; ++c)
        for (int i = 0; i < 4; ++i) {
            const int64_t k = 4 * c + i;
            const int64_t e = sptr_new[sl] + c * 4 * SLICE + 4 * lane + i;
            if (k < bw) {
                col_new[e] = col[bbase + k * SLICE];
                A32_new[e] = A32[bbase + k * SLICE];
            } else {
                col_new[e] = (int32_t)row;
                A32_new[e] = 0.0f;
            }
        }
}

__global__ __launch_bounds__(256) void k_build_csr(int64_t n_rows, const int64_t *__restrict__ sptr,
                                                   const int32_t *__restrict__ col,
                                                   const float *__restrict__ A32,
                                                   const int32_t *__restrict__ rptr,
                                                   int32_t *__restrict__ col_csr,
                                                   float *__restrict__ val_csr)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const int64_t base = sptr[r / SLICE] + (r % SLICE);
    const int32_t b = rptr[r], len = rptr[r + 1] - b;
    for (int k = 0; k < len; ++k) {
        col_csr[b + k] = col[base + (int64_t)k * SLICE];
        val_csr[b + k] = A32[base + (int64_t)k * SLICE];
    }
}

// Per node, the three values the right-hand-side pass gathers, as one
// 32-byte record: {Cm V + dt s, V, x0, 0} (x0 = 2 V - V_prev or V), so each
// nonzero costs one gather instead of three scattered ones.
// The per-node values the right-hand-side pass gathers at each column: a =
// Cm V + dt s (for M), V (for K) and the warm start x0 (for A); 24 bytes
// (a 32-byte record measured 1.4% more step time on the 12M-node cohort).
struct GV3 {
    double a, v, x;
};
__global__ __launch_bounds__(256) void k_b_gather_prep(int64_t n, StepParams sp,
                                                       const double *__restrict__ V,
                                                       const double *__restrict__ Vprev,
                                                       const double *__restrict__ src,
                                                       GV3 *__restrict__ gv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = V[i];
    GV3 r;
    r.a = sp.cm * v + sp.dt * src[i];
    r.v = v;
    r.x = sp.warm_start == 1 ? 2.0 * v - Vprev[i] : v;
    gv[i] = r;
}

// ---------------------------------------------------------------------------
template <bool NT>
__global__ __launch_bounds__(256) void k_b_rhs_init(
    SegTiling t, const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ col,
    const double *__restrict__ Mv, const double *__restrict__ Kv, const double *__restrict__ dinv,
    const float *__restrict__ dinv32, StepParams sp, const GV3 *__restrict__ gv,
    double *__restrict__ x, double *__restrict__ b, float *__restrict__ r32,
    float *__restrict__ delta, double *__restrict__ partial)
{
    const int g = logical_group(t.groups);
    const int4 gr = t.grp[g];
    const int lane = threadIdx.x & (SLICE - 1);
    const double cK_old = (1.0 - sp.theta) * sp.dt;
    const double cM_new = sp.chi * sp.cm;
    const double cK_new = sp.theta * sp.dt;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int tile = gr.y; tile < gr.z; ++tile) {
        const int64_t sl = wave_slice(tile);
        const int64_t row = sl * SLICE + lane;
        const int64_t b0 = slice_ptr[sl];
        const int w = (int)((slice_ptr[sl + 1] - b0) / SLICE);
        double mv = 0.0, kv = 0.0, mx = 0.0, kx = 0.0;
        sell_row2<8, NT>(w, col + b0 + lane, Mv + b0 + lane, Kv + b0 + lane, 0,
                         [&](int32_t c, double m, double kk) {
                             const GV3 gj = gv[c];
                             mv += m * gj.a;
                             kv += kk * gj.v;
                             mx += m * gj.x;
                             kx += kk * gj.x;
                         });
        const double bi = sp.chi * mv - cK_old * kv;
        const double ri = bi - (cM_new * mx + cK_new * kx);
        x[row] = gv[row].x;
        b[row] = bi;
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

__global__ __launch_bounds__(256) void k_b_init_finalize(int groups,
                                                         const int32_t *__restrict__ inst_grp,
                                                         const double *__restrict__ partial,
                                                         BParams bp, BScalars *__restrict__ sc)
{
    const int i = blockIdx.x;
    double v[3];
    reduce_range<3>(partial, groups, inst_grp[i], inst_grp[i + 1], v);
    if (threadIdx.x != 0) return;
    BScalars &s = sc[i];
    const double z0 = sqrt(v[1]), db = sqrt(v[2]);
    s.rho = v[0];
    s.alpha = 0.0;
    s.beta = 0.0;
    s.z0 = z0;
    s.znorm = z0;
    s.ref = bp.rel_mode == 1 ? db : z0;
    s.floor_ = 1e-15 * db;
    s.iters = 0;
    s.it = 0;
    s.replace = 0;
    s.redirect = 0;
    s.failed = 0;
    const bool finite = isfinite(z0) && isfinite(db) && isfinite(v[0]);
    s.nonfinite = finite ? 0 : 1;
    s.done = (!finite || z0 <= s.floor_ || z0 < bp.atol) ? 1 : 0;
}

// p = D^-1 r for the groups of running instances
__global__ __launch_bounds__(256) void k_b_set_direction(SegTiling t,
                                                         const float *__restrict__ dinv32,
                                                         const float *__restrict__ r32,
                                                         float *__restrict__ p32,
                                                         const BScalars *__restrict__ sc)
{
    const int4 gr = t.grp[logical_group(t.groups)];
    if (stopped(sc[gr.x])) return;
    for (int tile = gr.y; tile < gr.z; ++tile) {
        const int64_t i = (int64_t)tile * TILE + threadIdx.x;
        p32[i] = dinv32[i] * r32[i];
    }
}

// q = A p (FP32, lpr lanes per row), partial p.q (FP64 accumulation)
template <int LPR, bool NT>
__global__ __launch_bounds__(256) void k_b_spmv(SegTiling t, const int64_t *__restrict__ sptr,
                                                const int32_t *__restrict__ col,
                                                const float *__restrict__ A,
                                                const float *__restrict__ p,
                                                float *__restrict__ q, double *__restrict__ partial,
                                                const BScalars *__restrict__ sc)
{
    const int g = logical_group(t.groups);
    const int4 gr = t.grp[g];
    if (idle(sc[gr.x])) return;
    constexpr int H = SLICE / LPR;   // rows per wavefront
    const int lane = threadIdx.x & (SLICE - 1);
    const int w = threadIdx.x >> 6;
    double acc[1] = {0.0};
    for (int tile = gr.y; tile < gr.z; ++tile) {
#pragma unroll
        for (int pass = 0; pass < LPR; ++pass) {
            const int64_t row = (int64_t)tile * TILE + pass * (TILE / LPR) + w * H + lane / LPR;
            const int64_t sl = row / H;
            const int64_t b0 = sptr[sl];
            const int wl = (int)((sptr[sl + 1] - b0) / SLICE);   // entries per lane
            float sum = sell_row<NT, float>(wl, col + b0 + lane, A + b0 + lane, p, 0);
            if constexpr (LPR >= 4) sum += __shfl_xor(sum, 2, 64);
            if constexpr (LPR >= 2) sum += __shfl_xor(sum, 1, 64);
            if ((lane & (LPR - 1)) == 0) {
                q[row] = sum;
                acc[0] += (double)p[row] * (double)sum;
            }
        }
    }
    write_partials<1>(acc, partial, t.groups, g);
}

// Row of the vector-load sliced layout (chunk k of a lane at 4k * SLICE):
// for a fixed chunk count all chunk loads are issued before the gathers;
// entries are summed in column order as a loop would.
template <int NC, bool NT>
__device__ __forceinline__ float v4_row_n(const int32_t *__restrict__ col, const float *__restrict__ A,
                                          const float *__restrict__ p)
{
    i32x4 c[NC];
    f32x4 a[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        if constexpr (NT) {
            c[k] = __builtin_nontemporal_load(reinterpret_cast<const i32x4 *>(col + 4 * k * SLICE));
            a[k] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(A + 4 * k * SLICE));
        } else {
            c[k] = *reinterpret_cast<const i32x4 *>(col + 4 * k * SLICE);
            a[k] = *reinterpret_cast<const f32x4 *>(A + 4 * k * SLICE);
        }
    }
    float x[NC][4];
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) x[k][j] = p[c[k][j]];
    float sum = 0.0f;
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) sum += a[k][j] * x[k][j];
    return sum;
}

template <bool NT>
__device__ __forceinline__ float v4_row(int nc, const int32_t *__restrict__ col,
                                        const float *__restrict__ A, const float *__restrict__ p)
{
    switch (nc) {
    case 0: return 0.0f;
    case 1: return v4_row_n<1, NT>(col, A, p);
    case 2: return v4_row_n<2, NT>(col, A, p);
    case 3: return v4_row_n<3, NT>(col, A, p);
    case 4: return v4_row_n<4, NT>(col, A, p);
    case 5: return v4_row_n<5, NT>(col, A, p);
    case 6: return v4_row_n<6, NT>(col, A, p);
    default: {
        float sum = 0.0f;
        for (int k = 0; k < nc; ++k) {
            i32x4 c;
            f32x4 a;
            if constexpr (NT) {
                c = __builtin_nontemporal_load(reinterpret_cast<const i32x4 *>(col + 4 * k * SLICE));
                a = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(A + 4 * k * SLICE));
            } else {
                c = *reinterpret_cast<const i32x4 *>(col + 4 * k * SLICE);
                a = *reinterpret_cast<const f32x4 *>(A + 4 * k * SLICE);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) sum += a[j] * p[c[j]];
        }
        return sum;
    }
    }
}

// q = A p, vector-load sliced layout: one lane per row, 4 entries per load.
// NT: the matrix streams are read with the non-temporal hint (each value is
// read once per product), leaving the caches to the gathered vector.
template <bool NT>
__global__ __launch_bounds__(256) void k_b_spmv_v4(SegTiling t, const int64_t *__restrict__ sptr,
                                                   const int32_t *__restrict__ col,
                                                   const float *__restrict__ A,
                                                   const float *__restrict__ p,
                                                   float *__restrict__ q,
                                                   double *__restrict__ partial,
                                                   const BScalars *__restrict__ sc)
{
    const int g = logical_group(t.groups);
    const int4 gr = t.grp[g];
    if (idle(sc[gr.x])) return;
    const int lane = threadIdx.x & (SLICE - 1);
    double acc[1] = {0.0};
    for (int tile = gr.y; tile < gr.z; ++tile) {
        const int64_t sl = wave_slice(tile);
        const int64_t row = sl * SLICE + lane;
        const int64_t b0 = sptr[sl];
        const int nc = (int)((sptr[sl + 1] - b0) / (4 * SLICE));   // 4-entry chunks per lane
        const float sum = v4_row<NT>(nc, col + b0 + 4 * lane, A + b0 + 4 * lane, p);
        q[row] = sum;
        acc[0] += (double)p[row] * (double)sum;
    }
    write_partials<1>(acc, partial, t.groups, g);
}

// q = A p with A in CSR: LPR lanes per row stride through the row's
// contiguous entries, then a butterfly over the row's lanes
template <int LPR, bool NT>
__global__ __launch_bounds__(256) void k_b_spmv_csr(SegTiling t, const int32_t *__restrict__ rptr,
                                                    const int32_t *__restrict__ col,
                                                    const float *__restrict__ A,
                                                    const float *__restrict__ p,
                                                    float *__restrict__ q,
                                                    double *__restrict__ partial,
                                                    const BScalars *__restrict__ sc)
{
    const int g = logical_group(t.groups);
    const int4 gr = t.grp[g];
    if (idle(sc[gr.x])) return;
    constexpr int H = SLICE / LPR;   // rows per wavefront
    const int lane = threadIdx.x & (SLICE - 1);
    const int w = threadIdx.x >> 6;
    const int sub = lane & (LPR - 1);
    double acc[1] = {0.0};
    for (int tile = gr.y; tile < gr.z; ++tile) {
        for (int pass = 0; pass < LPR; ++pass) {
            const int64_t row = (int64_t)tile * TILE + pass * (TILE / LPR) + w * H + lane / LPR;
            const int32_t end = rptr[row + 1];
            float sum = 0.0f;
            for (int32_t e = rptr[row] + sub; e < end; e += LPR)
                sum += ld_stream<NT>(A + e) * p[ld_stream<NT>(col + e)];
#pragma unroll
            for (int off = LPR / 2; off >= 1; off >>= 1) sum += __shfl_xor(sum, off, 64);
            if (sub == 0) {
                q[row] = sum;
                acc[0] += (double)p[row] * (double)sum;
            }
        }
    }
    write_partials<1>(acc, partial, t.groups, g);
}

__global__ __launch_bounds__(256) void k_b_alpha(int groups, const int32_t *__restrict__ inst_grp,
                                                 const double *__restrict__ partial,
                                                 BScalars *__restrict__ sc)
{
    const int i = blockIdx.x;
    BScalars &s = sc[i];
    // what is read besides the partials is read with the verdict
    const int g0 = inst_grp[i], g1 = inst_grp[i + 1];
    const double rho = s.rho;
    if (idle(s)) return;
    double v[1];
    reduce_range<1>(partial, groups, g0, g1, v);
    if (threadIdx.x != 0) return;
    s.alpha = rho / v[0];
    s.redirect = 0;
}

// delta += alpha p; r -= alpha q; z = D^-1 r; partials r.z, z.z
__global__ __launch_bounds__(256) void k_b_update(SegTiling t, const float *__restrict__ dinv32,
                                                  const float *__restrict__ p,
                                                  const float *__restrict__ q,
                                                  float *__restrict__ delta, float *__restrict__ r,
                                                  double *__restrict__ partial,
                                                  const BScalars *__restrict__ sc)
{
    const int g = logical_group(t.groups);
    const int4 gr = t.grp[g];
    const BScalars &s = sc[gr.x];
    if (idle(s)) return;
    const float alpha = (float)s.alpha;
    double acc[2] = {0.0, 0.0};
    for (int tile = gr.y; tile < gr.z; ++tile) {
        const int64_t i = (int64_t)tile * TILE + threadIdx.x;
        delta[i] += alpha * p[i];
        const float ri = r[i] - alpha * q[i];
        r[i] = ri;
        const float zi = dinv32[i] * ri;
        acc[0] += (double)ri * (double)zi;
        acc[1] += (double)zi * (double)zi;
    }
    write_partials<2>(acc, partial, t.groups, g);
}

// stopping test of the recursive residual; a replacement is requested when it
// passes, every rr iterations and at the cap; otherwise beta
__global__ __launch_bounds__(256) void k_b_beta(int groups, const int32_t *__restrict__ inst_grp,
                                                const double *__restrict__ partial, BParams bp,
                                                BScalars *__restrict__ sc)
{
    const int i = blockIdx.x;
    BScalars &s = sc[i];
    const int g0 = inst_grp[i], g1 = inst_grp[i + 1];
    const int it = s.it + 1;
    const double ref = s.ref, floor_ = s.floor_, rho = s.rho;
    if (idle(s)) return;
    double v[2];
    reduce_range<2>(partial, groups, g0, g1, v);
    if (threadIdx.x != 0) return;
    const double zn = sqrt(v[1]);
    s.it = it;
    s.znorm = zn;
    if (!isfinite(zn) || !isfinite(v[0])) {
        s.nonfinite = 1;
        s.done = 1;
        s.iters = it;
        return;
    }
    const bool pass = zn < bp.atol || zn < bp.rtol * ref || zn <= floor_;
    if (pass || (bp.rr > 0 && it % bp.rr == 0) || it >= bp.max_iter) {
        s.replace = pass ? 1 : 2;   // 1: the recursive residual passed the test
        return;
    }
    s.beta = v[0] / rho;
    s.rho = v[0];
}

// p = D^-1 r + beta p
__global__ __launch_bounds__(256) void k_b_direction(SegTiling t, const float *__restrict__ dinv32,
                                                     const float *__restrict__ r,
                                                     float *__restrict__ p,
                                                     const BScalars *__restrict__ sc)
{
    const int4 gr = t.grp[logical_group(t.groups)];
    const BScalars &s = sc[gr.x];
    if (idle(s)) return;
    const float bf = (float)s.beta;
    for (int tile = gr.y; tile < gr.z; ++tile) {
        const int64_t i = (int64_t)tile * TILE + threadIdx.x;
        p[i] = dinv32[i] * r[i] + bf * p[i];
    }
}

// ---- residual replacement --------------------------------------------------
__device__ __forceinline__ bool replacing(const BScalars &s) { return s.replace && !s.done; }

__global__ __launch_bounds__(256) void k_b_flush(SegTiling t, double *__restrict__ x,
                                                 float *__restrict__ delta,
                                                 const BScalars *__restrict__ sc)
{
    const int4 gr = t.grp[logical_group(t.groups)];
    if (!replacing(sc[gr.x])) return;
    for (int tile = gr.y; tile < gr.z; ++tile) {
        const int64_t i = (int64_t)tile * TILE + threadIdx.x;
        x[i] += (double)delta[i];
        delta[i] = 0.0f;
    }
}

// r64 = b - A x64 (FP64 values), r32 = r64; partials r32.z32, |D^-1 r64|^2
template <bool NT>
__global__ __launch_bounds__(256) void k_b_true_residual(
    SegTiling t, const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ col,
    const double *__restrict__ Av, const double *__restrict__ x, const double *__restrict__ b,
    const double *__restrict__ dinv, const float *__restrict__ dinv32, float *__restrict__ r32,
    double *__restrict__ partial, const BScalars *__restrict__ sc)
{
    const int g = logical_group(t.groups);
    const int4 gr = t.grp[g];
    if (!replacing(sc[gr.x])) return;
    const int lane = threadIdx.x & (SLICE - 1);
    double acc[2] = {0.0, 0.0};
    for (int tile = gr.y; tile < gr.z; ++tile) {
        const int64_t sl = wave_slice(tile);
        const int64_t row = sl * SLICE + lane;
        const int64_t beg = slice_ptr[sl] + lane, end = slice_ptr[sl + 1];
        // a loop, not the fixed-width body: with FP64 values and the batch's
        // long rows the unrolled body's registers cost more occupancy than
        // its early loads gain (751 vs 677 us on the 12M-node cohort)
        double ax = 0.0;
#pragma unroll 4
        for (int64_t e = beg; e < end; e += SLICE) ax += ld_stream<NT>(Av + e) * x[ld_stream<NT>(col + e)];
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

__global__ __launch_bounds__(256) void k_b_replace_finalize(int groups,
                                                            const int32_t *__restrict__ inst_grp,
                                                            const double *__restrict__ partial,
                                                            BParams bp, BScalars *__restrict__ sc)
{
    const int i = blockIdx.x;
    BScalars &s = sc[i];
    const int g0 = inst_grp[i], g1 = inst_grp[i + 1];
    const int it = s.it;
    const int why = s.replace;
    const double ref = s.ref, floor_ = s.floor_, rho = s.rho;
    if (!replacing(s)) return;
    double v[2];
    reduce_range<2>(partial, groups, g0, g1, v);
    if (threadIdx.x != 0) return;
    const double zn = sqrt(v[1]);
    s.znorm = zn;
    s.replace = 0;
    if (!isfinite(zn) || !isfinite(v[0])) {
        s.nonfinite = 1;
        s.done = 1;
        s.iters = it;
        return;
    }
    if (zn < bp.atol || zn < bp.rtol * ref || zn <= floor_) {
        s.done = 1;
        s.iters = it;
        return;
    }
    if (it >= bp.max_iter) {
        s.failed = 1;
        s.done = 1;
        s.iters = it;
        return;
    }
    // restart (p = z) after the recursive residual passed but the true one did
    // not; keep the recurrence after a periodic replacement
    s.beta = why == 1 ? 0.0 : v[0] / rho;
    s.rho = v[0];
    s.redirect = 1;
}

__global__ __launch_bounds__(256) void k_b_redirect(SegTiling t, const float *__restrict__ dinv32,
                                                    const float *__restrict__ r,
                                                    float *__restrict__ p,
                                                    const BScalars *__restrict__ sc)
{
    const int4 gr = t.grp[logical_group(t.groups)];
    const BScalars &s = sc[gr.x];
    if (!s.redirect || s.done) return;
    const float bf = (float)s.beta;
    for (int tile = gr.y; tile < gr.z; ++tile) {
        const int64_t i = (int64_t)tile * TILE + threadIdx.x;
        p[i] = dinv32[i] * r[i] + bf * p[i];
    }
}

// ---- persistent iteration --------------------------------------------------
// All CG iterations of every running instance in one launch: each workgroup
// owns a fixed range of one instance's tiles (its own group table, sized so
// that every workgroup is resident at once) and the workgroups of an
// instance meet at a barrier of their own after the product, after the
// update and after the direction.  Every workgroup of an instance sums that
// instance's partials in the same fixed order and so takes the same
// decisions; the instance's first workgroup records them in its scalars.
// An instance leaves the loop when its recursive residual passes the test,
// every rr iterations and at the cap (the residual replacement kernels then
// run), or when a value is not finite.
//
// Barrier: a counter per instance, raised once per workgroup and barrier;
// the n-th barrier of an instance with G workgroups ends when the counter
// reaches n G.  Device-scope fences order the partials around it.  The wait
// is bounded: after `spin_cap` polls the workgroup records a timeout in
// *fault and leaves (the host reports an error), so a launch whose
// workgroups could not all be resident ends instead of hanging.
__device__ __forceinline__ bool inst_barrier(unsigned *__restrict__ counter, unsigned target,
                                             int *__restrict__ fault, int spin_cap)
{
    __shared__ int flag;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(counter, 1u);
        int spins = 0, f = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > spin_cap ||
                __hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                atomicOr(fault, 1);
                f = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
        flag = f;
    }
    __syncthreads();
    return flag == 0;
}

__global__ __launch_bounds__(256) void k_b_zero_u32(int n, unsigned *__restrict__ a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0u;
}

__global__ __launch_bounds__(256) void k_b_persistent(
    SegTiling t, const int64_t *__restrict__ slice_ptr, const int32_t *__restrict__ col,
    const float *__restrict__ A32, const float *__restrict__ dinv32, BParams bp,
    float *__restrict__ p, float *__restrict__ q, float *__restrict__ delta,
    float *__restrict__ r, double *__restrict__ part_pq, double *__restrict__ part_rz,
    BScalars *__restrict__ sc, unsigned *__restrict__ bar, int *__restrict__ fault, int spin_cap)
{
    const int g = blockIdx.x;   // instance-major order: an instance's groups are adjacent
    const int4 gr = t.grp[g];
    const int inst = gr.x;
    const int g0 = t.inst_grp[inst], g1 = t.inst_grp[inst + 1];
    const unsigned G = (unsigned)(g1 - g0);
    const bool lead = g == g0 && threadIdx.x == 0;
    BScalars &s = sc[inst];
    if (idle(s)) return;   // every group of the instance reads the same state
    const int lane = threadIdx.x & (SLICE - 1);
    double rho = s.rho, beta = s.beta;
    int it = s.it;
    if (lead) s.redirect = 0;   // p holds the direction (set before the launch)
    unsigned n_bar = 0;
    for (;;) {
        // ---- q = A p, partial p.q ----
        double acc1[1] = {0.0};
        for (int tile = gr.y; tile < gr.z; ++tile) {
            const int64_t sl = wave_slice(tile);
            const int64_t row = sl * SLICE + lane;
            const int64_t b0 = slice_ptr[sl];
            const int w = (int)((slice_ptr[sl + 1] - b0) / SLICE);
            const float sum = sell_row<false, float>(w, col + b0 + lane, A32 + b0 + lane, p, 0);
            q[row] = sum;
            acc1[0] += (double)p[row] * (double)sum;
        }
        write_partials<1>(acc1, part_pq, t.groups, g);
        if (!inst_barrier(bar + inst, ++n_bar * G, fault, spin_cap)) return;
        // ---- alpha; delta += alpha p, r -= alpha q; partials r.z, z.z ----
        double pq[1];
        reduce_range<1>(part_pq, t.groups, g0, g1, pq);
        const double alpha = rho / pq[0];
        const float af = (float)alpha;
        double acc2[2] = {0.0, 0.0};
        for (int tile = gr.y; tile < gr.z; ++tile) {
            const int64_t i = (int64_t)tile * TILE + threadIdx.x;
            delta[i] += af * p[i];
            const float ri = r[i] - af * q[i];
            r[i] = ri;
            const float zi = dinv32[i] * ri;
            acc2[0] += (double)ri * (double)zi;
            acc2[1] += (double)zi * (double)zi;
        }
        write_partials<2>(acc2, part_rz, t.groups, g);
        if (!inst_barrier(bar + inst, ++n_bar * G, fault, spin_cap)) return;
        // ---- stopping test, beta ----
        double v[2];
        reduce_range<2>(part_rz, t.groups, g0, g1, v);
        const double zn = sqrt(v[1]);
        ++it;
        int why = 0;
        if (!isfinite(zn) || !isfinite(v[0])) {
            why = -1;
        } else {
            const bool pass = zn < bp.atol || zn < bp.rtol * s.ref || zn <= s.floor_;
            why = pass ? 1 : ((bp.rr > 0 && it % bp.rr == 0) || it >= bp.max_iter) ? 2 : 0;
        }
        if (why != 0) {
            if (lead) {
                s.it = it;
                s.znorm = zn;
                s.alpha = alpha;
                if (why < 0) {
                    s.nonfinite = 1;
                    s.done = 1;
                    s.iters = it;
                } else {
                    s.replace = why;
                }
            }
            return;
        }
        beta = v[0] / rho;
        rho = v[0];
        // ---- p = D^-1 r + beta p ----
        const float bf = (float)beta;
        for (int tile = gr.y; tile < gr.z; ++tile) {
            const int64_t i = (int64_t)tile * TILE + threadIdx.x;
            p[i] = dinv32[i] * r[i] + bf * p[i];
        }
        if (lead) {
            s.it = it;
            s.znorm = zn;
            s.rho = rho;
            s.beta = beta;
            s.alpha = alpha;
        }
        if (!inst_barrier(bar + inst, ++n_bar * G, fault, spin_cap)) return;
    }
}

template <class Ptr, class Kernel>
void spmv_launch(Kernel k, hipStream_t s, const SegTiling &t, const Ptr *ptr, const IterMatrix &A,
                 const float *p32, float *q32, double *part_pq, const BScalars *sc, hipEvent_t e0,
                 hipEvent_t e1)
{
    if (e0)
        hipExtLaunchKernelGGL(k, dim3(t.groups), dim3(TILE), 0, s, e0, e1, 0, t, ptr, A.col, A.val,
                              p32, q32, part_pq, sc);
    else
        hipLaunchKernelGGL(k, dim3(t.groups), dim3(TILE), 0, s, t, ptr, A.col, A.val, p32, q32,
                           part_pq, sc);
}

}  // namespace

void launch_relayout(hipStream_t s, int lpr, int64_t n_slices, const int64_t *sptr_new,
                     SellView base, const float *A32, int32_t *col_new, float *A32_new)
{
    const int64_t threads = n_slices * SLICE;
    if (threads > 0)
        hipLaunchKernelGGL(k_relayout, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, lpr,
                           n_slices, sptr_new, base.slice_ptr, base.col, A32, col_new, A32_new);
}

void launch_b_rhs_init(hipStream_t s, const SegTiling &t, SellView P, const double *Mv,
                       const double *Kv, const double *dinv, const float *dinv32,
                       const StepParams &sp, int64_t n_rows, const double *V, const double *Vprev,
                       const double *src, double *gv, double *x, double *b, float *r32,
                       float *delta, double *partial, bool nt)
{
    hipLaunchKernelGGL(k_b_gather_prep, dim3((unsigned)((n_rows + 255) / 256)), dim3(256), 0, s,
                       n_rows, sp, V, Vprev, src, (GV3 *)gv);
    MDX_LAUNCH_NT(nt, k_b_rhs_init, dim3(t.groups), dim3(TILE), 0, s, t, P.slice_ptr, P.col, Mv, Kv,
                  dinv, dinv32, sp, (const GV3 *)gv, x, b, r32, delta, partial);
}

void launch_b_init_finalize(hipStream_t s, const SegTiling &t, const double *partial,
                            const BParams &bp, BScalars *sc)
{
    hipLaunchKernelGGL(k_b_init_finalize, dim3(t.n_inst), dim3(TILE), 0, s, t.groups, t.inst_grp,
                       partial, bp, sc);
}

void launch_b_set_direction(hipStream_t s, const SegTiling &t, const float *dinv32,
                            const float *r32, float *p32, const BScalars *sc)
{
    hipLaunchKernelGGL(k_b_set_direction, dim3(t.groups), dim3(TILE), 0, s, t, dinv32, r32, p32, sc);
}

void launch_relayout_v4(hipStream_t s, int64_t n_slices, const int64_t *sptr_new, SellView base,
                        const float *A32, int32_t *col_new, float *A32_new)
{
    const int64_t threads = n_slices * SLICE;
    if (threads > 0)
        hipLaunchKernelGGL(k_relayout_v4, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                           n_slices, sptr_new, base.slice_ptr, base.col, A32, col_new, A32_new);
}

void launch_build_csr(hipStream_t s, int64_t n_rows, SellView base, const float *A32,
                      const int32_t *rptr, int32_t *col_csr, float *val_csr)
{
    if (n_rows > 0)
        hipLaunchKernelGGL(k_build_csr, dim3((unsigned)((n_rows + 255) / 256)), dim3(256), 0, s,
                           n_rows, base.slice_ptr, base.col, A32, rptr, col_csr, val_csr);
}

void launch_b_spmv(hipStream_t s, const SegTiling &t, const IterMatrix &A, const float *p32,
                   float *q32, double *part_pq, const BScalars *sc, hipEvent_t e0, hipEvent_t e1)
{
    if (A.format == 2) {
        spmv_launch(k_b_spmv_v4<false>, s, t, A.sptr, A, p32, q32, part_pq, sc, e0, e1);
    } else if (A.format == 3) {
        spmv_launch(k_b_spmv_v4<true>, s, t, A.sptr, A, p32, q32, part_pq, sc, e0, e1);
    } else if (A.format == 1) {
        if (A.lpr == 16)
            spmv_launch(A.nt ? k_b_spmv_csr<16, true> : k_b_spmv_csr<16, false>, s, t, A.rptr, A, p32,
                        q32, part_pq, sc, e0, e1);
        else if (A.lpr == 8)
            spmv_launch(A.nt ? k_b_spmv_csr<8, true> : k_b_spmv_csr<8, false>, s, t, A.rptr, A, p32,
                        q32, part_pq, sc, e0, e1);
        else
            spmv_launch(A.nt ? k_b_spmv_csr<4, true> : k_b_spmv_csr<4, false>, s, t, A.rptr, A, p32,
                        q32, part_pq, sc, e0, e1);
    } else {
        if (A.lpr == 4)
            spmv_launch(A.nt ? k_b_spmv<4, true> : k_b_spmv<4, false>, s, t, A.sptr, A, p32, q32,
                        part_pq, sc, e0, e1);
        else if (A.lpr == 2)
            spmv_launch(A.nt ? k_b_spmv<2, true> : k_b_spmv<2, false>, s, t, A.sptr, A, p32, q32,
                        part_pq, sc, e0, e1);
        else
            spmv_launch(A.nt ? k_b_spmv<1, true> : k_b_spmv<1, false>, s, t, A.sptr, A, p32, q32,
                        part_pq, sc, e0, e1);
    }
}

void launch_b_iteration(hipStream_t s, const SegTiling &t, const IterMatrix &A, const BParams &bp,
                        const float *dinv32, float *p32, float *q32, float *delta, float *r32,
                        double *part_pq, double *part_rz, BScalars *sc, hipEvent_t ev_start,
                        hipEvent_t ev_stop)
{
    launch_b_spmv(s, t, A, p32, q32, part_pq, sc, ev_start, ev_stop);
    hipLaunchKernelGGL(k_b_alpha, dim3(t.n_inst), dim3(TILE), 0, s, t.groups, t.inst_grp, part_pq,
                       sc);
    hipLaunchKernelGGL(k_b_update, dim3(t.groups), dim3(TILE), 0, s, t, dinv32, p32, q32, delta, r32,
                       part_rz, sc);
    hipLaunchKernelGGL(k_b_beta, dim3(t.n_inst), dim3(TILE), 0, s, t.groups, t.inst_grp, part_rz, bp,
                       sc);
    hipLaunchKernelGGL(k_b_direction, dim3(t.groups), dim3(TILE), 0, s, t, dinv32, r32, p32, sc);
}

int persistent_capacity(int device)
{
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_b_persistent, TILE, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return 0;
    return per_cu * cus;
}

void launch_b_persistent(hipStream_t s, const SegTiling &t, SellView P, const float *A32,
                         const float *dinv32, const BParams &bp, float *p32, float *q32,
                         float *delta, float *r32, double *part_pq, double *part_rz,
                         BScalars *sc, unsigned *bar, int *fault, int spin_cap)
{
    const int n = t.n_inst + 1;   // the counters and the fault flag
    hipLaunchKernelGGL(k_b_zero_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, bar);
    hipLaunchKernelGGL(k_b_persistent, dim3(t.groups), dim3(TILE), 0, s, t, P.slice_ptr, P.col, A32,
                       dinv32, bp, p32, q32, delta, r32, part_pq, part_rz, sc, bar, fault, spin_cap);
}

void launch_b_replacement(hipStream_t s, const SegTiling &t, SellView P, const BParams &bp,
                          const double *Av, double *x, float *delta, const double *b,
                          const double *dinv, const float *dinv32, float *r32, float *p32,
                          double *partial, BScalars *sc, bool nt)
{
    hipLaunchKernelGGL(k_b_flush, dim3(t.groups), dim3(TILE), 0, s, t, x, delta, sc);
    MDX_LAUNCH_NT(nt, k_b_true_residual, dim3(t.groups), dim3(TILE), 0, s, t, P.slice_ptr, P.col, Av,
                  x, b, dinv, dinv32, r32, partial, sc);
    hipLaunchKernelGGL(k_b_replace_finalize, dim3(t.n_inst), dim3(TILE), 0, s, t.groups, t.inst_grp,
                       partial, bp, sc);
    hipLaunchKernelGGL(k_b_redirect, dim3(t.groups), dim3(TILE), 0, s, t, dinv32, r32, p32, sc);
}

}  // namespace mdx
