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

// Every workgroup reduces the `groups` partials of a producer kernel, laid
// out partial[k * groups + g], in the same order.
template <int NV>
__device__ __forceinline__ void reduce_partials(const double *__restrict__ partial, int groups,
                                                double (&v)[NV])
{
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    for (int g = threadIdx.x; g < groups; g += TILE)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += partial[k * groups + g];
    group_sum<NV>(v);
}

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
