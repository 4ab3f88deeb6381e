// Assembly of the P1 mass and stiffness matrices on the device (setup only).
//
// Element stage: one thread per tetrahedron computes its volume and the 4x4
// stiffness block K_e[a][b] = vol * grad(phi_a) . sigma grad(phi_b), with
// sigma = st I + (sl - st) f f^T for the unit fibre f (transversely isotropic
// conductivity from the element's longitudinal and transverse values; the
// "Software functionality" section).  Barycentric gradients come from face
// normals: grad(phi_a) = n_a / (n_a . (x_a - x_b)), n_a the normal of the
// face opposite vertex a.  The consistent P1 mass block is vol/20 (1 + d_ab).
//
// Surface triangles (P1 triangles in 3D, the "Software functionality"
// section's triangular elements): one thread per triangle, with the normal
// n = (x1 - x0) x (x2 - x0), area |n| / 2 and surface gradients
// grad(phi_a) = n x (x_c - x_b) / |n|^2 for (a, b, c) cyclic; sigma is built
// on the fibre's projection onto the triangle's plane, normalised (isotropic
// where the projection vanishes).  The consistent mass is area/12 (1 + d_ab).
//
// Gather stage: one thread per matrix slot sums the contributions listed for
// that slot (element id * 16 + a * 4 + b), in ascending element order.  No
// atomics, so assembly is deterministic.
#include "mdx_internal.h"

namespace mdx {

namespace {

struct v3 {
    double x, y, z;
};
__device__ __forceinline__ v3 sub(v3 a, v3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double dot3(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ v3 cross(v3 a, v3 b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

__global__ __launch_bounds__(256) void k_element(int64_t m, const double *__restrict__ xyz,
                                                 const int32_t *__restrict__ tets,
                                                 const double *__restrict__ fibre,
                                                 const double *__restrict__ sig,
                                                 double *__restrict__ elem_vol,
                                                 double *__restrict__ elem_k)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    v3 X[4];
    for (int a = 0; a < 4; ++a) {
        int64_t v = tets[4 * e + a];
        X[a] = {xyz[3 * v], xyz[3 * v + 1], xyz[3 * v + 2]};
    }
    double six_vol = fabs(dot3(sub(X[1], X[0]), cross(sub(X[2], X[0]), sub(X[3], X[0]))));
    v3 g[4];
    for (int a = 0; a < 4; ++a) {
        v3 xb = X[(a + 1) & 3], xc = X[(a + 2) & 3], xd = X[(a + 3) & 3];
        v3 nrm = cross(sub(xc, xb), sub(xd, xb));
        double h = dot3(nrm, sub(X[a], xb));
        g[a] = {nrm.x / h, nrm.y / h, nrm.z / h};
    }
    double sl = sig[2 * e], st = sig[2 * e + 1];
    v3 f = {0.0, 0.0, 0.0};
    if (fibre) {
        v3 fr = {fibre[3 * e], fibre[3 * e + 1], fibre[3 * e + 2]};
        double len = sqrt(dot3(fr, fr));
        if (len > 0.0) f = {fr.x / len, fr.y / len, fr.z / len};
    }
    double gf[4];
    for (int a = 0; a < 4; ++a) gf[a] = dot3(g[a], f);
    double vol = six_vol / 6.0;
    elem_vol[e] = vol;
    double *out = elem_k + 16 * e;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            out[4 * a + b] = vol * (st * dot3(g[a], g[b]) + (sl - st) * gf[a] * gf[b]);
}

// elements given as 4-id records; the 3x3 block of the 16-entry record
__global__ __launch_bounds__(256) void k_element_tri(int64_t m, const double *__restrict__ xyz,
                                                     const int32_t *__restrict__ tris,
                                                     const double *__restrict__ fibre,
                                                     const double *__restrict__ sig,
                                                     double *__restrict__ elem_area,
                                                     double *__restrict__ elem_k)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    v3 X[3];
    for (int a = 0; a < 3; ++a) {
        int64_t v = tris[4 * e + a];
        X[a] = {xyz[3 * v], xyz[3 * v + 1], xyz[3 * v + 2]};
    }
    const v3 nrm = cross(sub(X[1], X[0]), sub(X[2], X[0]));
    const double n2 = dot3(nrm, nrm);
    v3 g[3];
    for (int a = 0; a < 3; ++a) {
        const v3 c = cross(nrm, sub(X[(a + 2) % 3], X[(a + 1) % 3]));
        g[a] = {c.x / n2, c.y / n2, c.z / n2};
    }
    double sl = sig[2 * e], st = sig[2 * e + 1];
    v3 f = {0.0, 0.0, 0.0};
    if (fibre) {
        const v3 fr = {fibre[3 * e], fibre[3 * e + 1], fibre[3 * e + 2]};
        const double fn = dot3(fr, nrm) / n2;
        const v3 ft = {fr.x - fn * nrm.x, fr.y - fn * nrm.y, fr.z - fn * nrm.z};
        const double len = sqrt(dot3(ft, ft));
        if (len > 1e-12 * sqrt(dot3(fr, fr))) f = {ft.x / len, ft.y / len, ft.z / len};
    }
    double gf[3];
    for (int a = 0; a < 3; ++a) gf[a] = dot3(g[a], f);
    const double area = 0.5 * sqrt(n2);
    elem_area[e] = area;
    double *out = elem_k + 16 * e;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            out[4 * a + b] = area * (st * dot3(g[a], g[b]) + (sl - st) * gf[a] * gf[b]);
}

// mass_den: 20 for tetrahedra (vol/20 (1 + d_ab)), 12 for triangles
__global__ __launch_bounds__(256) void k_gather(int64_t n_slots, const int64_t *__restrict__ cptr,
                                                const int32_t *__restrict__ contrib,
                                                const double *__restrict__ elem_vol,
                                                const double *__restrict__ elem_k, double mass_den,
                                                double *__restrict__ Mv, double *__restrict__ Kv)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_slots) return;
    double msum = 0.0, ksum = 0.0;
    for (int64_t c = cptr[s]; c < cptr[s + 1]; ++c) {
        uint32_t code = (uint32_t)contrib[c];
        int64_t e = code >> 4;
        int ab = code & 15;
        bool diag = (ab >> 2) == (ab & 3);
        msum += elem_vol[e] * (diag ? 2.0 : 1.0) / mass_den;
        ksum += elem_k[16 * e + ab];
    }
    Mv[s] = msum;
    Kv[s] = ksum;
}

__global__ __launch_bounds__(256) void k_system(int64_t n_slots, const double *__restrict__ Mv,
                                                const double *__restrict__ Kv, double cM,
                                                double cK, double *__restrict__ Av)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n_slots) Av[s] = cM * Mv[s] + cK * Kv[s];
}

// Lumped mass: each row's entries summed onto its diagonal, every other
// entry zero.  The diagonal is the row's first slot with col == row (the
// padding slots after a row's real entries also carry col == row).
__global__ __launch_bounds__(256) void k_lump(int64_t n_rows, const int64_t *__restrict__ slice_ptr,
                                              const int32_t *__restrict__ col,
                                              double *__restrict__ Mv)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const int64_t sl = r / SLICE;
    const int lane = (int)(r % SLICE);
    double sum = 0.0;
    for (int64_t e = slice_ptr[sl] + lane; e < slice_ptr[sl + 1]; e += SLICE) sum += Mv[e];
    bool placed = false;
    for (int64_t e = slice_ptr[sl] + lane; e < slice_ptr[sl + 1]; e += SLICE) {
        const bool diag = !placed && col[e] == r;
        Mv[e] = diag ? sum : 0.0;
        placed = placed || diag;
    }
}

// dinv[r] = 1 / A_rr; the padding entries carry col = row and value 0, so the
// sum over all entries with col == row is the diagonal.  Padding rows: 0.
__global__ __launch_bounds__(256) void k_dinv(int64_t n_rows, int64_t n_real,
                                              const int64_t *__restrict__ slice_ptr,
                                              const int32_t *__restrict__ col,
                                              const double *__restrict__ Av,
                                              double *__restrict__ dinv)
{
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    if (r >= n_real) {
        dinv[r] = 0.0;
        return;
    }
    int64_t sl = r / SLICE;
    int lane = (int)(r % SLICE);
    double d = 0.0;
    for (int64_t e = slice_ptr[sl] + lane; e < slice_ptr[sl + 1]; e += SLICE)
        if (col[e] == r) d += Av[e];
    // a padding row of the batched layout has only zero-valued self entries
    dinv[r] = d != 0.0 ? 1.0 / d : 0.0;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

void launch_element(hipStream_t s, int npe, int64_t m, const double *xyz, const int32_t *tets,
                    const double *fibre, const double *sig, double *elem_vol, double *elem_k)
{
    if (m <= 0) return;
    if (npe == 3)
        hipLaunchKernelGGL(k_element_tri, dim3(blocks_for(m)), dim3(256), 0, s, m, xyz, tets,
                           fibre, sig, elem_vol, elem_k);
    else
        hipLaunchKernelGGL(k_element, dim3(blocks_for(m)), dim3(256), 0, s, m, xyz, tets, fibre,
                           sig, elem_vol, elem_k);
}

void launch_gather(hipStream_t s, int npe, int64_t n_slots, const int64_t *cptr,
                   const int32_t *contrib, const double *elem_vol, const double *elem_k,
                   double *Mv, double *Kv)
{
    if (n_slots > 0)
        hipLaunchKernelGGL(k_gather, dim3(blocks_for(n_slots)), dim3(256), 0, s, n_slots, cptr,
                           contrib, elem_vol, elem_k, npe == 3 ? 12.0 : 20.0, Mv, Kv);
}

void launch_system(hipStream_t s, int64_t n_slots, const double *Mv, const double *Kv, double cM,
                   double cK, double *Av)
{
    if (n_slots > 0)
        hipLaunchKernelGGL(k_system, dim3(blocks_for(n_slots)), dim3(256), 0, s, n_slots, Mv, Kv,
                           cM, cK, Av);
}

void launch_lump(hipStream_t s, int64_t n_rows, SellView A, double *Mv)
{
    if (n_rows > 0)
        hipLaunchKernelGGL(k_lump, dim3(blocks_for(n_rows)), dim3(256), 0, s, n_rows, A.slice_ptr,
                           A.col, Mv);
}

void launch_dinv(hipStream_t s, int64_t n_rows, int64_t n_real, SellView A, const double *Av,
                 double *dinv)
{
    if (n_rows > 0)
        hipLaunchKernelGGL(k_dinv, dim3(blocks_for(n_rows)), dim3(256), 0, s, n_rows, n_real,
                           A.slice_ptr, A.col, Av, dinv);
}

}  // namespace mdx
