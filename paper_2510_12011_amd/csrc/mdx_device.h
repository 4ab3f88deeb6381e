// Device helpers shared by the row-tiled solver kernels: XCD-aware
// workgroup remap and deterministic two-level reductions.
#pragma once
#include "mdx_internal.h"

namespace mdx {

// Hardware dispatches workgroup i to XCD i % 8; return the logical workgroup
// so that XCD x owns the contiguous logical range of its share.
static __device__ __forceinline__ int logical_group(int nb)
{
    int i = blockIdx.x;
    int x = i % NXCD, j = i / NXCD;
    int q = nb / NXCD, rem = nb % NXCD;
    return x * q + min(x, rem) + j;
}

// Load of a matrix stream (values, column indices).  With NT the load carries
// the non-temporal hint: a matrix larger than the Infinity Cache is read once
// per product and would only evict the gathered vectors; a smaller one is
// better left to stay cache-resident across products (NT = false).  The host
// picks NT per kernel from the size of the streams it reads.
template <bool NT, class T>
static __device__ __forceinline__ T ld_stream(const T *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// first column of slice sl for 16-bit offsets, 0 for 32-bit columns
template <typename CI>
static __device__ __forceinline__ int32_t slice_base(const Cols<CI> &c, int64_t sl)
{
    if constexpr (sizeof(CI) == 2)
        return c.base[sl];
    else
        return 0;
}

#define MDX_LAUNCH_NT(nt, kernel, ...)                                                       \
    do {                                                                                     \
        if (nt)                                                                              \
            hipLaunchKernelGGL(kernel<true>, __VA_ARGS__);                                   \
        else                                                                                 \
            hipLaunchKernelGGL(kernel<false>, __VA_ARGS__);                                  \
    } while (0)

// Launch kernel<NT, CI> on the column stream of SellView P: the launch
// arguments name that stream `cols`.
#define MDX_LAUNCH_SELL(P, nt, kernel, ...)                                                  \
    with_cols((P), (nt), [&](auto ntc_, auto cols) {                                         \
        auto kern_ = &kernel<decltype(ntc_)::value, typename decltype(cols)::index_type>;    \
        hipLaunchKernelGGL(kern_, __VA_ARGS__);                                              \
    })

// the same with start/stop events recorded around the launch
#define MDX_LAUNCH_SELL_EV(P, nt, e0, e1, kernel, grid, block, shm, st, ...)                 \
    with_cols((P), (nt), [&](auto ntc_, auto cols) {                                         \
        auto kern_ = &kernel<decltype(ntc_)::value, typename decltype(cols)::index_type>;    \
        if (e0)                                                                              \
            hipExtLaunchKernelGGL(kern_, grid, block, shm, st, e0, e1, 0, __VA_ARGS__);       \
        else                                                                                 \
            hipLaunchKernelGGL(kern_, grid, block, shm, st, __VA_ARGS__);                    \
    })

static __device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum NV values over the 256 threads of the workgroup; the totals are
// returned to every thread.
template <int NV>
__device__ __forceinline__ void group_sum(double (&v)[NV])
{
    __shared__ double lds[4][NV];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) lds[w][k] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = ((lds[0][k] + lds[1][k]) + lds[2][k]) + lds[3][k];
    __syncthreads();
}

// Sum NV values over a workgroup of any whole number of wavefronts (up to
// 1024 threads); the totals are returned to every thread.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV])
{
    __shared__ double lds[16][NV];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = wave_sum(v[k]);
        if (lane == 0) lds[w][k] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int i = 0; i < nw; ++i) s += lds[i][k];
        v[k] = s;
    }
    __syncthreads();
}

// Activation and repolarisation times of row i after a step to time t1 with
// V^k = vo, V^{k+1} = vn: LAT = the first t^{k+1} with V > 0; LRT = the first
// later t^{k+1} with V < -70 mV while V falls.  Returns false for a
// non-finite vn.
__device__ __forceinline__ bool update_times(int64_t i, double t1, double vo, double vn,
                                             double *__restrict__ lat, double *__restrict__ lrt)
{
    if (!isfinite(vn)) return false;
    double l = lat[i];
    if (isinf(l) && vn > 0.0) {
        l = t1;
        lat[i] = t1;
    }
    if (!isinf(l) && l < t1 && isinf(lrt[i]) && vn < -70.0 && vn < vo) lrt[i] = t1;
    return true;
}

// One workgroup of NT threads (the finalize kernels) sums the `groups`
// partials of a producer kernel, laid out partial[k * groups + g], in a fixed
// order: thread t adds g = t, t + NT, t + 2 NT, ... in turn, then the
// workgroup sum.  The loads of up to FIN_U of a thread's partials are all
// issued before its first add, so the partials cost one memory round trip
// (a loop that added as it loaded waited on each load in turn).  The
// iteration's finalize kernels reduce one partial per SpMV workgroup (4,905
// on the 1.26M-node shell) with FIN threads; those that reduce one per
// vector-kernel workgroup (at most 2,048) are faster with 256.
constexpr int FIN = 1024;
constexpr int FIN_U = 8;
template <int NV, int NT = FIN>
__device__ __forceinline__ void finalize_partials(const double *__restrict__ partial, int groups,
                                                  double (&v)[NV])
{
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    for (int g0 = threadIdx.x; g0 < groups; g0 += FIN_U * NT) {
        double t[FIN_U][NV];
#pragma unroll
        for (int j = 0; j < FIN_U; ++j)
#pragma unroll
            for (int k = 0; k < NV; ++k)
                t[j][k] = g0 + j * NT < groups ? partial[k * groups + g0 + j * NT] : 0.0;
#pragma unroll
        for (int j = 0; j < FIN_U; ++j)
            if (g0 + j * NT < groups)
#pragma unroll
                for (int k = 0; k < NV; ++k) v[k] += t[j][k];
    }
    block_sum<NV>(v);
}

// Product of one sliced-ELL row with a gathered vector x: the row's entries
// are c[j * SLICE], a[j * SLICE] for j < w, where w is its slice's width
// (uniform over the wavefront).  For a fixed width every column and value
// load is issued before the first gather, so a row costs one memory round
// trip for the streams and one for the gathers; entries are summed in
// column order j = 0, 1, ... as a loop would.
template <int W, bool NT, typename ACC, typename CI, typename TA, typename TX>
__device__ __forceinline__ ACC sell_row_w(const CI *__restrict__ c, const TA *__restrict__ a,
                                          const TX *__restrict__ x, int32_t cb)
{
    CI cc[W];
    TA aa[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        cc[j] = ld_stream<NT>(c + j * SLICE);
        aa[j] = ld_stream<NT>(a + j * SLICE);
    }
    TX xx[W];
#pragma unroll
    for (int j = 0; j < W; ++j) xx[j] = x[cb + (int32_t)cc[j]];
    ACC s = 0;
#pragma unroll
    for (int j = 0; j < W; ++j) s += (ACC)aa[j] * (ACC)xx[j];
    return s;
}

constexpr int SELL_UNROLLED = 24;   // widest slice with a fixed-width body
template <bool NT, typename ACC, typename CI, typename TA, typename TX>
__device__ __forceinline__ ACC sell_row(int w, const CI *__restrict__ c, const TA *__restrict__ a,
                                        const TX *__restrict__ x, int32_t cb)
{
    switch (w) {
#define MDX_SELL_CASE(n) \
    case n: return sell_row_w<n, NT, ACC>(c, a, x, cb);
        MDX_SELL_CASE(1) MDX_SELL_CASE(2) MDX_SELL_CASE(3) MDX_SELL_CASE(4)
        MDX_SELL_CASE(5) MDX_SELL_CASE(6) MDX_SELL_CASE(7) MDX_SELL_CASE(8)
        MDX_SELL_CASE(9) MDX_SELL_CASE(10) MDX_SELL_CASE(11) MDX_SELL_CASE(12)
        MDX_SELL_CASE(13) MDX_SELL_CASE(14) MDX_SELL_CASE(15) MDX_SELL_CASE(16)
        MDX_SELL_CASE(17) MDX_SELL_CASE(18) MDX_SELL_CASE(19) MDX_SELL_CASE(20)
        MDX_SELL_CASE(21) MDX_SELL_CASE(22) MDX_SELL_CASE(23) MDX_SELL_CASE(24)
#undef MDX_SELL_CASE
    default: {
        ACC s = 0;
        for (int j = 0; j < w; ++j)
            s += (ACC)ld_stream<NT>(a + j * SLICE) * (ACC)x[cb + (int32_t)ld_stream<NT>(c + j * SLICE)];
        return s;
    }
    }
}

// A row of two matrices sharing the pattern (M and K values at a0, a1):
// f(column, m, k) is applied to its entries in column order, in chunks of
// up to C entries whose column and value loads are all issued before the
// chunk's first gather (f does the gathers).
template <int W, bool NT, typename CI, typename F>
__device__ __forceinline__ void sell_chunk2(const CI *__restrict__ c, const double *__restrict__ a0,
                                            const double *__restrict__ a1, int32_t cb, F &f)
{
    CI cc[W];
    double m[W], k[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        cc[j] = ld_stream<NT>(c + j * SLICE);
        m[j] = ld_stream<NT>(a0 + j * SLICE);
        k[j] = ld_stream<NT>(a1 + j * SLICE);
    }
#pragma unroll
    for (int j = 0; j < W; ++j) f(cb + (int32_t)cc[j], m[j], k[j]);
}

template <int C, bool NT, typename CI, typename F>
__device__ __forceinline__ void sell_row2(int w, const CI *__restrict__ c,
                                          const double *__restrict__ a0,
                                          const double *__restrict__ a1, int32_t cb, F &&f)
{
    static_assert(C >= 2 && C <= 8, "remainder cases below cover chunks of up to 8");
    int j = 0;
    for (; j + C <= w; j += C)
        sell_chunk2<C, NT>(c + j * SLICE, a0 + j * SLICE, a1 + j * SLICE, cb, f);
    c += j * SLICE;
    a0 += j * SLICE;
    a1 += j * SLICE;
    // the remainder (fewer than C entries); cases of C entries or more are
    // not instantiated, so they cost no registers
    switch (w - j) {
    case 1: sell_chunk2<1, NT>(c, a0, a1, cb, f); break;
    case 2: if constexpr (C > 2) sell_chunk2<2, NT>(c, a0, a1, cb, f); break;
    case 3: if constexpr (C > 3) sell_chunk2<3, NT>(c, a0, a1, cb, f); break;
    case 4: if constexpr (C > 4) sell_chunk2<4, NT>(c, a0, a1, cb, f); break;
    case 5: if constexpr (C > 5) sell_chunk2<5, NT>(c, a0, a1, cb, f); break;
    case 6: if constexpr (C > 6) sell_chunk2<6, NT>(c, a0, a1, cb, f); break;
    case 7: if constexpr (C > 7) sell_chunk2<7, NT>(c, a0, a1, cb, f); break;
    default: break;
    }
}

// Slice handled by wavefront `wv` (0..3) of tile `tile`, as a scalar: its
// header loads then go through the scalar cache.
__device__ __forceinline__ int64_t wave_slice(int tile)
{
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    return (int64_t)tile * (TILE / SLICE) + wv;
}

// The stopping test's constants, read by a finalize kernel together with its
// verdict, so that they arrive with the first round trip rather than after
// the partials' sum.
struct StopTest {
    double atol, rtol, ref, floor_;
};
__device__ __forceinline__ StopTest stop_test(const Scalars *sc)
{
    return {sc->atol, sc->rtol, sc->ref, sc->floor_};
}
__device__ __forceinline__ bool passes(const StopTest &t, double zn)
{
    return zn < t.atol || zn < t.rtol * t.ref || zn <= t.floor_;
}

// A producer kernel's workgroup g stores its NV sums at partial[k * groups + g].
template <int NV>
__device__ __forceinline__ void write_partials(double (&v)[NV], double *__restrict__ partial,
                                               int groups, int g)
{
    group_sum<NV>(v);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) partial[k * groups + g] = v[k];
}

}  // namespace mdx
