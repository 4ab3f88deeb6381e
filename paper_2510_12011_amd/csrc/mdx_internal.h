// Internal interface between the host library (mdx_api.hip) and the gfx950
// kernels (mdx_assembly.hip, mdx_ionic.hip, mdx_solver.hip).
//
// Matrix layout on the device: sliced ELL with slices of 64 consecutive rows
// (one wavefront, one lane per row), column-major inside a slice:
//   entry j of row r lives at slice_ptr[r / 64] + j * 64 + (r % 64)
// so the j-th loads of the 64 rows of a wavefront are one contiguous 512-byte
// (f64) or 256-byte (f32/i32) segment.  Rows are in reverse Cuthill-McKee
// order, each row's columns ascending; short rows are padded with (col = row,
// value = 0).  The row count is padded to a multiple of TILE with empty rows
// whose vectors stay zero.  M, K and A share one pattern (slice_ptr, col).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mdx {

constexpr int SLICE = 64;   // rows per slice = wavefront width
constexpr int TILE = 256;   // rows per workgroup pass = 4 slices
constexpr int NXCD = 8;     // accelerator complex dies on MI355X

// Row tiles owned by each workgroup.  Workgroup b (logical, after the XCD
// remap) owns tiles [b*tpb, min((b+1)*tpb, n_tiles)).  A reduction kernel
// writes one partial per workgroup; consumers re-reduce the `groups`
// partials in a fixed order, so every result is deterministic.
struct Tiling {
    int64_t n_rows;   // padded row count, multiple of TILE
    int n_tiles;      // n_rows / TILE
    int tpb;          // tiles per workgroup
    int groups;       // workgroups launched = ceil(n_tiles / tpb)
};
Tiling make_tiling(int64_t n_rows_padded, int max_groups);

// Device-side solver scalars, written by kernels, read by kernels and by the
// host (copied to pinned memory).  Double-buffered rho avoids a read/write
// race between workgroups of one kernel.
struct alignas(256) Scalars {
    double rho[2];      // r^T z of the current iteration (index k & 1)
    double ref;         // denominator of the relative stopping test
    double floor_;      // rounding floor 1e-15 * ||D^-1 b||
    double z0, znorm;   // ||z_0|| and the last ||z||
    double atol, rtol;
    int32_t done;       // solve finished (converged)
    int32_t iters;      // iterations taken by the finished solve
    int32_t nonfinite;  // a non-finite V was produced
    int32_t zero;       // always 0 (for launches that must not early-exit)
};

struct SellView {
    const int64_t *slice_ptr;
    const int32_t *col;
};

// ---- assembly (mdx_assembly.hip) -----------------------------------------
void launch_element(hipStream_t s, int64_t m, const double *xyz, const int32_t *tets,
                    const double *fibre, const double *sig, double *elem_vol, double *elem_k);
void launch_gather(hipStream_t s, int64_t n_slots, const int64_t *cptr, const int32_t *contrib,
                   const double *elem_vol, const double *elem_k, double *Mv, double *Kv);
void launch_system(hipStream_t s, int64_t n_slots, const double *Mv, const double *Kv,
                   double cM, double cK, double *Av);
void launch_dinv(hipStream_t s, int64_t n_rows, int64_t n_real, SellView A, const double *Av,
                 double *dinv);

// ---- ionic models (mdx_ionic.hip) -----------------------------------------
int ionic_nstates(int kind);
int ionic_nparams(int kind);
void ionic_defaults(int kind, double *params);
// params: host array of ionic_nparams(kind) values (passed by value to kernels)
void launch_ionic_init(hipStream_t s, int kind, const double *params, int64_t n, int64_t ld,
                       double *V, double *Vprev, double *u);
// u advanced in place from V; out[i] = istim[i] - cm * I_ion/Cm if raw == 0,
// or I_ion/Cm (mV/ms) if raw != 0.  istim may be null (no active stimulus).
void launch_ionic_step(hipStream_t s, int kind, const double *params, int64_t n, int64_t ld,
                       double dt, double cm, const double *V, double *u, const double *istim,
                       double *out, int raw);

// ---- solver (mdx_solver.hip) ---------------------------------------------
struct StepParams {
    double chi, cm, theta, dt;
    int warm_start;    // 0: x0 = V^k, 1: x0 = 2V^k - V^{k-1}
    int rel_mode;      // 0: relative to ||z_0||, 1: relative to ||D^-1 b||
};
void launch_fill(hipStream_t s, int64_t n, double v, double *x);
void launch_stim_add(hipStream_t s, int64_t n_idx, const int32_t *idx, double amp, double *istim);
// b, x0, r0 = b - A x0, p0 = z0 = D^-1 r0 and the partials (r.z, z.z, |D^-1 b|^2)
void launch_rhs_init(hipStream_t s, const Tiling &t, SellView P, const double *Mv,
                     const double *Kv, const double *dinv, const StepParams &sp,
                     const double *V, const double *Vprev, const double *src, double *x,
                     double *r, double *p, double *b, double *partial);
void launch_init_finalize(hipStream_t s, const Tiling &t, const double *partial, int rel_mode,
                          Scalars *sc);
// ev_start/ev_stop: optional events recorded around the dispatch
void launch_spmv_dot(hipStream_t s, const Tiling &t, SellView P, const double *Av,
                     const double *p, double *q, double *partial, const int32_t *done,
                     hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
void launch_cg_update(hipStream_t s, const Tiling &t, int k, const double *partial_pq,
                      const double *dinv, const double *p, const double *q, double *x, double *r,
                      double *partial_rz, Scalars *sc);
void launch_cg_direction(hipStream_t s, const Tiling &t, int k, const double *partial_rz,
                         const double *dinv, const double *r, double *p, Scalars *sc);
void launch_epilogue(hipStream_t s, int64_t n, double t1, const double *Vold, const double *Vnew,
                     double *lat, double *lrt, Scalars *sc);

}  // namespace mdx
