// Learned warm start for the PCG solve of each step.
//
// Per-node features at step n (after the ionic update):
//   f0 = V^n,  f1 = V^n - V^{n-1},  f2 = s / Cm = (I_stim - I_ion) / Cm,
//   f3 = (K V^{n-1})_i / K_ii  (one neighbour aggregate: the stiffness SpMV
//        the previous step's right-hand side already formed)
// are standardised and fed to the per-node MLP (mdx_mlp.hip), whose output
// y predicts the departure of V^{n+1} from the paper's extrapolation:
// x_mlp = x_ex + out_scale * y, x_ex = 2V^n - V^{n-1}.  Because the
// aggregate is the previous step's, the network runs before the right-hand
// side, and one pass over M and K then forms the initial residual of x_mlp
// (with the vectors the iteration starts from), the norms of both x_mlp's and
// x_ex's residuals, and the next step's aggregate.  The MLP guess is used
// only if its ||D^-1 r0|| is smaller (and finite), otherwise the
// extrapolation is (the fallback, whose vectors a guarded pass then forms):
// the network can only lower the initial residual of the method without it.
//
// k_features also serves as the recorder of training data: raw features of
// every node, and after the solve the increment V^{n+1} - V^n.
#include "mdx_device.h"
#include "mdx_internal.h"

namespace mdx {

namespace {

// kvp = (K v)_i / K_ii
template <bool NT, typename CI>
__global__ __launch_bounds__(256) void k_kv_feature(Tiling t, const int64_t *__restrict__ slice_ptr,
                                                    Cols<CI> col,
                                                    const double *__restrict__ Kv,
                                                    const double *__restrict__ kdiag,
                                                    const double *__restrict__ v,
                                                    float *__restrict__ kvp)
{
    const int g = logical_group(t.groups);
    const int lane = threadIdx.x & (SLICE - 1);
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t sl = wave_slice(tile);
        const int64_t row = sl * SLICE + lane;
        const int64_t b0 = slice_ptr[sl];
        const int w = (int)((slice_ptr[sl + 1] - b0) / SLICE);
        const double kv =
            sell_row<NT, double>(w, col.idx + b0 + lane, Kv + b0 + lane, v, slice_base(col, sl));
        const double kd = kdiag[row];
        kvp[row] = kd != 0.0 ? (float)(kv / kd) : 0.0f;
    }
}

__global__ __launch_bounds__(256) void k_features(int64_t n_real, int64_t n_rows,
                                                  const double *__restrict__ V,
                                                  const double *__restrict__ Vprev,
                                                  const double *__restrict__ src,
                                                  const float *__restrict__ kvp, double inv_cm,
                                                  MlpNorm nm, float4 *__restrict__ feat,
                                                  float4 *__restrict__ raw)
{
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n_rows) return;
    const double vi = V[row];
    float4 f;
    f.x = (float)vi;
    f.y = (float)(vi - Vprev[row]);
    f.z = (float)(src[row] * inv_cm);
    f.w = kvp[row];
    if (raw && row < n_real) raw[row] = f;
    if (feat) {
        float4 h;
        h.x = (f.x - nm.mean[0]) * nm.inv_std[0];
        h.y = (f.y - nm.mean[1]) * nm.inv_std[1];
        h.z = (f.z - nm.mean[2]) * nm.inv_std[2];
        h.w = (f.w - nm.mean[3]) * nm.inv_std[3];
        feat[row] = h;
    }
}

// b = chi M (Cm V + dt s) - (1-theta) dt K V;  the extrapolation
// x_ex = 2V - V_prev has A x_ex = chi Cm M x_ex + theta dt K x_ex and
// r_ex = b - A x_ex;  the network's guess x = x_ex + scale y has
// r = r_ex - scale A y, which is what the pass stores, with what the
// iteration starts from: the FP32 residual, z and correction (FP32
// iteration) or z0 = D^-1 r (FP64 iteration; p0 may be null).  Partials:
// r.z, |z|^2 of the guess and of the extrapolation (FP32-rounded residuals
// when the iteration runs in FP32), |D^-1 b|^2.  Where the extrapolation
// wins, a guarded pass recomputes its x and r (k_rhs_init*).
template <bool NT, typename CI>
__global__ __launch_bounds__(256) void k_rhs_learned(
    Tiling t, const int64_t *__restrict__ slice_ptr, Cols<CI> col,
    const double *__restrict__ Mv, const double *__restrict__ Kv, const double *__restrict__ kdiag,
    const double *__restrict__ dinv, const float *__restrict__ dinv32, StepParams sp,
    float out_scale, const double *__restrict__ V, const double *__restrict__ Vprev,
    const double *__restrict__ src, const float *__restrict__ y, double *__restrict__ x,
    double *__restrict__ r, double *__restrict__ p0, float *__restrict__ r32,
    float *__restrict__ z32, float *__restrict__ delta, float *__restrict__ kvp,
    double *__restrict__ part5)
{
    const int g = logical_group(t.groups);
    const int lane = threadIdx.x & (SLICE - 1);
    const double cK_old = (1.0 - sp.theta) * sp.dt;
    const double cM_new = sp.chi * sp.cm;
    const double cK_new = sp.theta * sp.dt;
    const double scale = (double)out_scale;
    const bool fp32_iter = r32 != nullptr;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int t_end = min((g + 1) * t.tpb, t.n_tiles);
    for (int tile = g * t.tpb; tile < t_end; ++tile) {
        const int64_t sl = wave_slice(tile);
        const int64_t row = sl * SLICE + lane;
        const int64_t b0 = slice_ptr[sl];
        const int w = (int)((slice_ptr[sl + 1] - b0) / SLICE);
        // M (Cm V + dt s), K V, M x_ex, K x_ex, M y, K y
        double mb = 0.0, kv = 0.0, mx = 0.0, kx = 0.0, my = 0.0, ky = 0.0;
        // chunks of 4 entries: with six accumulators and four gathered
        // vectors, chunks of 8 need 128 registers (4 waves per SIMD), of 4
        // 94 (5 waves), which measured 2.5% faster per step on the shell
        sell_row2<4, NT>(w, col.idx + b0 + lane, Mv + b0 + lane, Kv + b0 + lane,
                         slice_base(col, sl), [&](int32_t c, double m, double kk) {
                             const double vj = V[c], xj = 2.0 * vj - Vprev[c];
                             const double yj = (double)y[c];
                             mb += m * (sp.cm * vj + sp.dt * src[c]);
                             kv += kk * vj;
                             mx += m * xj;
                             kx += kk * xj;
                             my += m * yj;
                             ky += kk * yj;
                         });
        const double bi = sp.chi * mb - cK_old * kv;
        const double rx = bi - (cM_new * mx + cK_new * kx);
        const double rm = rx - scale * (cM_new * my + cK_new * ky);
        const double vi = V[row];
        x[row] = (2.0 * vi - Vprev[row]) + scale * (double)y[row];
        r[row] = rm;
        const double kd = kdiag[row];
        kvp[row] = kd != 0.0 ? (float)(kv / kd) : 0.0f;
        const double di = dinv[row];
        if (fp32_iter) {
            const float rmf = (float)rm, rxf = (float)rx, df = dinv32[row];
            const float zmf = df * rmf, zxf = df * rxf;
            r32[row] = rmf;
            z32[row] = zmf;
            delta[row] = 0.0f;
            acc[0] += (double)rmf * (double)zmf;
            acc[1] += (double)zmf * (double)zmf;
            acc[2] += (double)rxf * (double)zxf;
            acc[3] += (double)zxf * (double)zxf;
        } else {
            const double zm = di * rm, zx = di * rx;
            if (p0) p0[row] = zm;
            acc[0] += rm * zm;
            acc[1] += zm * zm;
            acc[2] += rx * zx;
            acc[3] += zx * zx;
        }
        acc[4] += (di * bi) * (di * bi);
    }
    write_partials<5>(acc, part5, t.groups, g);
}

// choose the guess; scalars of the PCG initialisation.  The pass's partials
// are five rows: r.z and |z|^2 of the guess, of the extrapolation, |D^-1 b|^2.
__global__ __launch_bounds__(TILE) void k_init_finalize_ws(int groups, const double *__restrict__ p5,
                                                          int rel_mode, Scalars *__restrict__ sc)
{
    const double atol = sc->atol;
    double v[5];
    finalize_partials<5, TILE>(p5, groups, v);
    if (threadIdx.x != 0) return;
    const bool finite = v[1] == v[1] && v[1] < 1e300;
    const bool use = finite && v[1] < v[3];
    const double rz = use ? v[0] : v[2];
    const double z0 = sqrt(use ? v[1] : v[3]);
    const double db = sqrt(v[4]);
    const double floor_ = 1e-15 * db;
    sc->use_mlp = use ? 1 : 0;
    sc->rho[0] = rz;
    sc->z0 = z0;
    sc->znorm = z0;
    sc->ref = rel_mode == 1 ? db : z0;
    sc->floor_ = floor_;
    // a non-finite start ends the solve and is reported; a finite one clears
    // the flag of an earlier solve
    const bool ok = isfinite(z0) && isfinite(db) && isfinite(rz);
    sc->nonfinite = ok ? 0 : 2;
    sc->done = (!ok || z0 <= floor_ || z0 < atol) ? 1 : 0;
    sc->iters = 0;
    sc->replace = 0;
    sc->beta = 0.0;
    sc->it_next = 0;
}

__global__ __launch_bounds__(256) void k_record_dv(int64_t n, const double *__restrict__ Vold,
                                                   const double *__restrict__ Vnew,
                                                   float *__restrict__ dv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dv[i] = (float)(Vnew[i] - Vold[i]);
}

__global__ __launch_bounds__(256) void k_kdiag(int64_t n_rows, int64_t n_real,
                                               const int64_t *__restrict__ slice_ptr,
                                               const int32_t *__restrict__ col,
                                               const double *__restrict__ Kv,
                                               double *__restrict__ kdiag)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    double d = 0.0;
    if (r < n_real) {
        const int64_t sl = r / SLICE;
        const int lane = (int)(r % SLICE);
        for (int64_t e = slice_ptr[sl] + lane; e < slice_ptr[sl + 1]; e += SLICE)
            if (col[e] == r) d += Kv[e];
    }
    kdiag[r] = d;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

// Training samples: row idx[i] of the recorded features X and increments dV,
// raw or as the network trains on them (standardised features; target the
// departure of the increment from the previous one, in units of out_scale).
// An index outside [0, n_rows) gives a zero feature row and a NaN target.
__global__ __launch_bounds__(256) void k_mlp_samples(int64_t n_idx, const int64_t *__restrict__ idx,
                                                     int64_t n_rows, const float4 *__restrict__ X,
                                                     const float *__restrict__ dV, int stdz,
                                                     MlpNorm nm, float4 *__restrict__ Xo,
                                                     float *__restrict__ To)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_idx) return;
    const int64_t j = idx[i];
    if (j < 0 || j >= n_rows) {
        Xo[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        To[i] = __builtin_nanf("");
        return;
    }
    const float4 x = X[j];
    const float d = dV[j];
    if (stdz) {
        Xo[i] = make_float4((x.x - nm.mean[0]) * nm.inv_std[0], (x.y - nm.mean[1]) * nm.inv_std[1],
                            (x.z - nm.mean[2]) * nm.inv_std[2], (x.w - nm.mean[3]) * nm.inv_std[3]);
        To[i] = (d - x.y) / nm.out_scale;
    } else {
        Xo[i] = x;
        To[i] = d;
    }
}

}  // namespace

void launch_kdiag(hipStream_t s, int64_t n_rows, int64_t n_real, SellView K, const double *Kv,
                  double *kdiag)
{
    hipLaunchKernelGGL(k_kdiag, dim3(blocks_for(n_rows)), dim3(256), 0, s, n_rows, n_real,
                       K.slice_ptr, K.col, Kv, kdiag);
}

void launch_kv_feature(hipStream_t s, const Tiling &t, SellView P, const double *Kv,
                       const double *kdiag, const double *v, float *kvp)
{
    MDX_LAUNCH_SELL(P, false, k_kv_feature, dim3(t.groups), dim3(TILE), 0, s, t, P.slice_ptr, cols,
                    Kv, kdiag, v, kvp);
}

void launch_features(hipStream_t s, int64_t n_real, int64_t n_rows, const double *V,
                     const double *Vprev, const double *src, const float *kvp, double cm,
                     const MlpNorm &nm, float *feat, float *raw)
{
    if (n_rows > 0)
        hipLaunchKernelGGL(k_features, dim3(blocks_for(n_rows)), dim3(256), 0, s, n_real, n_rows, V,
                           Vprev, src, kvp, 1.0 / cm, nm, (float4 *)feat, (float4 *)raw);
}

void launch_rhs_learned(hipStream_t s, const Tiling &t, SellView P, const double *Mv,
                        const double *Kv, const double *kdiag, const double *dinv,
                        const float *dinv32, const StepParams &sp, float out_scale,
                        const double *V, const double *Vprev, const double *src, const float *y,
                        double *x, double *r, double *p0, float *r32, float *z32, float *delta,
                        float *kvp, double *part5, bool nt)
{
    MDX_LAUNCH_SELL(P, nt, k_rhs_learned, dim3(t.groups), dim3(TILE), 0, s, t, P.slice_ptr, cols, Mv,
                    Kv, kdiag, dinv, dinv32, sp, out_scale, V, Vprev, src, y, x, r, p0, r32, z32,
                    delta, kvp, part5);
}

void launch_init_finalize_ws(hipStream_t s, const Tiling &t, const double *p5,
                             int rel_mode, Scalars *sc)
{
    hipLaunchKernelGGL(k_init_finalize_ws, dim3(1), dim3(TILE), 0, s, t.groups, p5, rel_mode, sc);
}

void launch_mlp_samples(hipStream_t s, int64_t n_idx, const int64_t *idx, int64_t n_rows,
                        const float *X, const float *dV, bool stdz, const MlpNorm &nm, float *Xo,
                        float *To)
{
    if (n_idx > 0)
        hipLaunchKernelGGL(k_mlp_samples, dim3(blocks_for(n_idx)), dim3(256), 0, s, n_idx, idx,
                           n_rows, reinterpret_cast<const float4 *>(X), dV, stdz ? 1 : 0, nm,
                           reinterpret_cast<float4 *>(Xo), To);
}

void launch_record_dv(hipStream_t s, int64_t n, const double *Vold, const double *Vnew, float *dv)
{
    if (n > 0)
        hipLaunchKernelGGL(k_record_dv, dim3(blocks_for(n)), dim3(256), 0, s, n, Vold, Vnew, dv);
}

}  // namespace mdx
