// Per-node MLP of the learned warm start: 4 -> 64 -> 64 -> 64 -> 1, ReLU,
// BF16 weights and activations, FP32 accumulation, on the 32x32x8 BF16 MFMA
// of gfx950.  Forward (inference), gradient of the mean-squared error
// (training) and Adam.
//
// Parameter vector (FP32 master copy, 8,705 values):
//   W1[64][4] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[64] b4
//
// Arithmetic: layer 1 in FP32 VALU with BF16-rounded W1 on FP32 features;
// h1 = bf16(relu(z1)); layers 2 and 3 on MFMA (BF16 operands, FP32
// accumulators) plus FP32 bias; h2 = bf16(relu(z2)); h3 = relu(z3) in FP32;
// y = sum bf16(W4) h3 + b4 in FP32.
//
// One wavefront handles a tile of 32 nodes.  Hidden layers are computed as
// transposed products Z^T = W H^T (M = output unit, N = node, K = input
// unit).  With v_mfma_f32_32x32x8_bf16 the accumulator element held in
// register v of lane l is Z^T[8(v/4) + 4(l/32) + v%4][l%32]; the B operand
// of the next layer's K-step s in lane l is H^T[8s + 4(l/32) + i][l%32],
// i = 0..3.  These coincide (s = v/4 within a 32-row output tile), so each
// layer's output feeds the next MFMA from registers with no data exchange.
#include "mdx_device.h"
#include "mdx_internal.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

namespace mdx {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 256, OFF_W2 = 320, OFF_B2 = 4416, OFF_W3 = 4480,
              OFF_B3 = 8576, OFF_W4 = 8640, OFF_B4 = 8704;
constexpr int NPARAM = 8705;
constexpr int WSTRIDE = 68;   // LDS row stride (bf16) of W2/W3: 8-byte aligned, fewer conflicts

__device__ __forceinline__ unsigned short f2bf(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ __forceinline__ float round_bf(float f) { return bf2f(f2bf(f)); }

__device__ __forceinline__ f32x16 mfma(bf16x4 a, bf16x4 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}

// weights staged in LDS once per workgroup
struct MlpLds {
    float w1[NH][4];       // BF16-rounded
    float b1[NH];
    unsigned short w2[NH * WSTRIDE];
    float b2[NH];
    unsigned short w3[NH * WSTRIDE];
    float b3[NH];
    float w4[NH];          // BF16-rounded
    float b4;
};

__device__ void load_weights(const float *__restrict__ P, MlpLds &w)
{
    for (int i = threadIdx.x; i < NH * 4; i += blockDim.x) w.w1[i / 4][i % 4] = round_bf(P[OFF_W1 + i]);
    for (int i = threadIdx.x; i < NH * NH; i += blockDim.x) {
        const int o = i / NH, k = i % NH;
        w.w2[o * WSTRIDE + k] = f2bf(P[OFF_W2 + i]);
        w.w3[o * WSTRIDE + k] = f2bf(P[OFF_W3 + i]);
    }
    for (int i = threadIdx.x; i < NH; i += blockDim.x) {
        w.b1[i] = P[OFF_B1 + i];
        w.b2[i] = P[OFF_B2 + i];
        w.b3[i] = P[OFF_B3 + i];
        w.w4[i] = round_bf(P[OFF_W4 + i]);
    }
    if (threadIdx.x == 0) w.b4 = P[OFF_B4];
}

// A fragment of W (rows = output units): lane holds W[32 ot + l%32][8 ks + 4 half + 0..3]
__device__ __forceinline__ bf16x4 frag_w(const unsigned short *w, int ot, int ks, int lane)
{
    const int o = 32 * ot + (lane & 31), k = 8 * ks + 4 * (lane >> 5);
    return *reinterpret_cast<const bf16x4 *>(w + o * WSTRIDE + k);
}

// A fragment of W^T (rows = input units): lane holds W[8 s + 4 half + i][32 kt + l%32]
__device__ __forceinline__ bf16x4 frag_wt(const unsigned short *w, int kt, int s, int lane)
{
    const int k = 32 * kt + (lane & 31), o = 8 * s + 4 * (lane >> 5);
    bf16x4 a;
    a[0] = (short)w[(o + 0) * WSTRIDE + k];
    a[1] = (short)w[(o + 1) * WSTRIDE + k];
    a[2] = (short)w[(o + 2) * WSTRIDE + k];
    a[3] = (short)w[(o + 3) * WSTRIDE + k];
    return a;
}

// unit index held in accumulator register v of output tile ot by this lane
__device__ __forceinline__ int unit_of(int ot, int v, int half) { return 32 * ot + 8 * (v / 4) + 4 * half + (v % 4); }

struct Tile {
    bf16x4 h1[8];      // B fragments: h1 for units 8t + 4 half + i
    bf16x4 h2[8];      // B fragments: h2 for units 8t + 4 half + i
    float z1[32];      // layer-1 pre-activations (same units as h1, t*4 + i)
    float z2[32];      // layer-2 pre-activations, index 16 ot + v
    float z3[32];      // layer-3 pre-activations, index 16 ot + v
    float y;
};

__device__ __forceinline__ void forward_tile(const MlpLds &w, float4 x, Tile &T, bool keep)
{
    const int lane = threadIdx.x & 63, half = lane >> 5;
    // layer 1 (VALU)
#pragma unroll
    for (int t = 0; t < 8; ++t) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = 8 * t + 4 * half + i;
            float z = w.b1[o] + w.w1[o][0] * x.x + w.w1[o][1] * x.y + w.w1[o][2] * x.z + w.w1[o][3] * x.w;
            if (keep) T.z1[4 * t + i] = z;
            T.h1[t][i] = (short)f2bf(fmaxf(z, 0.0f));
        }
    }
    // layer 2 (MFMA)
#pragma unroll
    for (int ot = 0; ot < 2; ++ot) {
        f32x16 acc = {0};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) acc = mfma(frag_w(w.w2, ot, ks, lane), T.h1[ks], acc);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const float z = acc[v] + w.b2[unit_of(ot, v, half)];
            if (keep) T.z2[16 * ot + v] = z;
            T.h2[4 * ot + v / 4][v % 4] = (short)f2bf(fmaxf(z, 0.0f));
        }
    }
    // layer 3 (MFMA) and output layer (VALU)
    float s = 0.0f;
#pragma unroll
    for (int ot = 0; ot < 2; ++ot) {
        f32x16 acc = {0};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) acc = mfma(frag_w(w.w3, ot, ks, lane), T.h2[ks], acc);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int o = unit_of(ot, v, half);
            const float z = acc[v] + w.b3[o];
            T.z3[16 * ot + v] = z;
            s += w.w4[o] * fmaxf(z, 0.0f);
        }
    }
    s += __shfl_xor(s, 32, 64);
    T.y = s + w.b4;
}

// ---------------------------------------------------------------------------
// Inference (the warm start of every time step).  Same function as
// forward_tile with every layer on v_mfma_f32_32x32x16_bf16 (K = 16, twice
// the K of the training kernels' instruction per issue):
//   layer 1: the FP32 features enter as a BF16 pair hi + lo (x = hi + lo to
//            about 2^-17 relative): B rows 0..3 hi, 4..7 lo, 8..15 zero and
//            A columns W1, W1, 0, so one MFMA gives BF16(W1) x in FP32;
//   layers 2, 3: K-step s of a 64-unit layer reads, in lane half h, the
//            accumulator registers 8 (s % 2) .. + 7 of the previous layer's
//            output tile s / 2 -- units 16 s + 8 (j / 4) + 4 h + j % 4 for
//            j = 0..7 -- so the weight fragment takes those columns (two
//            8-byte LDS reads) and no data moves between lanes;
//   biases:  FP32, loaded as the accumulators' initial values;
//   BF16 rounding of the activations by the hardware conversion
//   (round to nearest even, as f2bf).
// No pre-activations are kept, so several wavefronts share a SIMD.
// ---------------------------------------------------------------------------
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8n __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x16 mfma16(s16x8 a, s16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8n, a),
                                                    __builtin_bit_cast(bf16x8n, b), c, 0, 0, 0);
}

__device__ __forceinline__ s16x8 cat8(bf16x4 lo, bf16x4 hi)
{
    return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

// A fragment of a hidden layer's W (64 x 64, LDS row stride WSTRIDE) for
// output tile ot and K-step s: row 32 ot + l % 32, the columns listed above
__device__ __forceinline__ s16x8 frag_w16(const unsigned short *w, int ot, int s, int lane)
{
    const unsigned short *row = w + (32 * ot + (lane & 31)) * WSTRIDE + 16 * s + 4 * (lane >> 5);
    return cat8(*reinterpret_cast<const bf16x4 *>(row), *reinterpret_cast<const bf16x4 *>(row + 8));
}
typedef __bf16 bf16x2n __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ unsigned pack_bf16(float a, float b)
{
    f32x2 v = {a, b};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2n));
}
__device__ __forceinline__ bf16x4 pack_bf16x4(float a, float b, float c, float d)
{
    u32x2 u = {pack_bf16(a, b), pack_bf16(c, d)};
    return __builtin_bit_cast(bf16x4, u);
}
// bf16(relu(a)), ... for four values: ReLU after the rounding, on the packed
// pairs as signed 16-bit integers (a BF16 value is negative exactly when its
// bit pattern is, and rounding to nearest keeps the sign, so max(bits, 0)
// maps negatives, -0 included, to +0 and keeps the rest)
typedef short s16x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned relu_bf16x2(float a, float b)
{
    const s16x2v zero = {0, 0};
    const s16x2v v = __builtin_bit_cast(s16x2v, pack_bf16(a, b));
    return __builtin_bit_cast(unsigned, __builtin_elementwise_max(v, zero));
}
__device__ __forceinline__ bf16x4 relu_pack_bf16x4(float a, float b, float c, float d)
{
    u32x2 u = {relu_bf16x2(a, b), relu_bf16x2(c, d)};
    return __builtin_bit_cast(bf16x4, u);
}

// ReLU in FP32 as a signed-integer max on the bit pattern: values with the
// sign bit set (negatives, -0) become +0, the rest are kept.  fmaxf would
// add a canonicalising max per value.
__device__ __forceinline__ float relu_bits(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

struct alignas(16) InferLds {
    float b1[NH], b2[NH], b3[NH], w4[NH];   // FP32 biases, BF16-rounded w4
    unsigned short w1[NH * 16];             // BF16 [W1 W1 0]: columns 0..3, 4..7, 8..15
    unsigned short w2[NH * WSTRIDE];
    unsigned short w3[NH * WSTRIDE];
    float b4;
};

// bias (or w4) values of the units held by this lane in output tile ot, in
// accumulator order: v = 4 g + j -> unit 32 ot + 8 g + 4 half + j
__device__ __forceinline__ f32x16 unit_frag(const float *v, int ot, int half)
{
    f32x16 r;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const float4 q = *reinterpret_cast<const float4 *>(v + 32 * ot + 8 * g + 4 * half);
        r[4 * g + 0] = q.x;
        r[4 * g + 1] = q.y;
        r[4 * g + 2] = q.z;
        r[4 * g + 3] = q.w;
    }
    return r;
}

// The network's input per node: stored standardised features (X), or the
// features formed from the state as the feature pass forms them (same
// expressions, so the same bits): V, V - V_prev, s / Cm, the neighbour
// aggregate, standardised.
// fetch() issues a node's loads (zeros past n, or for lanes that hold no
// node), form() turns them into the network's input, so that the loads of
// the next nodes can be in flight while the current ones are computed.
template <bool STATE>
struct FeatRaw;
template <>
struct FeatRaw<false> {
    float4 x;
};
template <>
struct FeatRaw<true> {
    double v, vp, s;
    float k;
};

struct FeatIn {
    const float4 *X;
    const double *V, *Vprev, *src;
    const float *kvp;
    double inv_cm;   // 1 / Cm
    MlpNorm nm;
    template <bool STATE>
    __device__ __forceinline__ FeatRaw<STATE> fetch(int64_t i, bool ok) const
    {
        if constexpr (STATE) {
            FeatRaw<true> r{0.0, 0.0, 0.0, 0.0f};
            if (ok) r = {V[i], Vprev[i], src[i], kvp[i]};
            return r;
        } else {
            FeatRaw<false> r{make_float4(0.f, 0.f, 0.f, 0.f)};
            if (ok) r.x = X[i];
            return r;
        }
    }
    template <bool STATE>
    __device__ __forceinline__ float4 form(const FeatRaw<STATE> &r, bool ok) const
    {
        if (!ok) return make_float4(0.f, 0.f, 0.f, 0.f);
        if constexpr (STATE) {
            const float fx = (float)r.v, fy = (float)(r.v - r.vp), fz = (float)(r.s * inv_cm);
            return make_float4((fx - nm.mean[0]) * nm.inv_std[0],
                               (fy - nm.mean[1]) * nm.inv_std[1],
                               (fz - nm.mean[2]) * nm.inv_std[2],
                               (r.k - nm.mean[3]) * nm.inv_std[3]);
        } else {
            return r.x;
        }
    }
};

template <bool STATE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_mlp_forward(const float *__restrict__ P, int64_t n,
                                                     FeatIn in, float *__restrict__ y)
{
    __shared__ InferLds w;
    {
        // the weights into LDS, every load issued before the first
        // conversion: a fixed stride of 256 threads (the launch's size),
        // fully unrolled (a loop over blockDim.x waited on each load in turn)
        constexpr int NT = 256, R = NH * NH / NT;
        const int t = threadIdx.x;
        float a2[R], a3[R], a1[4];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            a2[j] = P[OFF_W2 + t + NT * j];
            a3[j] = P[OFF_W3 + t + NT * j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = t + NT * j, o = i / 16, k = i % 16;
            a1[j] = k < 8 ? P[OFF_W1 + 4 * o + (k & 3)] : 0.0f;
        }
        float bb[4] = {0.0f, 0.0f, 0.0f, 0.0f}, b4 = 0.0f;
        if (t < NH) {
            bb[0] = P[OFF_B1 + t];
            bb[1] = P[OFF_B2 + t];
            bb[2] = P[OFF_B3 + t];
            bb[3] = P[OFF_W4 + t];
        }
        if (t == 0) b4 = P[OFF_B4];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int i = t + NT * j, o = i / NH, k = i % NH;
            w.w2[o * WSTRIDE + k] = f2bf(a2[j]);
            w.w3[o * WSTRIDE + k] = f2bf(a3[j]);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) w.w1[t + NT * j] = f2bf(a1[j]);
        if (t < NH) {
            w.b1[t] = bb[0];
            w.b2[t] = bb[1];
            w.b3[t] = bb[2];
            w.w4[t] = round_bf(bb[3]);
        }
        if (t == 0) w.b4 = b4;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, half = lane >> 5;
    // two 32-node tiles per pass share every weight and bias fragment read
    // from LDS and give each wavefront two independent MFMA chains to
    // interleave (one tile per pass took 44-49 us on 1.26M nodes, two 26-28)
    const int64_t n_pairs = ((n + 31) / 32 + 1) / 2;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    const int64_t pr0 = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    FeatRaw<STATE> raw[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int64_t nd = (2 * pr0 + b) * 32 + (lane & 31);
        raw[b] = in.fetch<STATE>(nd, pr0 < n_pairs && half == 0 && nd < n);
    }
    for (int64_t pr = pr0; pr < n_pairs; pr += waves) {
        // weights are re-read from LDS for every pair: held in registers
        // across pairs they would take ~200 VGPRs and leave one wavefront
        // per SIMD to hide the latency of the layer chain
        asm volatile("" ::: "memory");
        int64_t node[2];
        s16x8 xb[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            node[b] = (2 * pr + b) * 32 + (lane & 31);
            const float4 x = in.form<STATE>(raw[b], half == 0 && node[b] < n);
            const bf16x4 xh = pack_bf16x4(x.x, x.y, x.z, x.w);
            const float4 xr = make_float4(x.x - bf2f((unsigned short)xh[0]),
                                          x.y - bf2f((unsigned short)xh[1]),
                                          x.z - bf2f((unsigned short)xh[2]),
                                          x.w - bf2f((unsigned short)xh[3]));
            xb[b] = cat8(xh, pack_bf16x4(xr.x, xr.y, xr.z, xr.w));
        }
        // the next pair's loads, issued once this pair's inputs are formed
        // (loads retire in order) and in flight during its layers
        const int64_t pn = pr + waves;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t nd = (2 * pn + b) * 32 + (lane & 31);
            raw[b] = in.fetch<STATE>(nd, pn < n_pairs && half == 0 && nd < n);
        }
        // layer 1
        bf16x4 h1[2][8];
#pragma unroll
        for (int ot = 0; ot < 2; ++ot) {
            const s16x8 a =
                *reinterpret_cast<const s16x8 *>(w.w1 + (32 * ot + (lane & 31)) * 16 + 8 * half);
            const f32x16 bias = unit_frag(w.b1, ot, half);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const f32x16 acc = mfma16(a, xb[b], bias);
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    h1[b][4 * ot + g] = relu_pack_bf16x4(acc[4 * g], acc[4 * g + 1],
                                                         acc[4 * g + 2], acc[4 * g + 3]);
            }
        }
        // layer 2
        bf16x4 h2[2][8];
#pragma unroll
        for (int ot = 0; ot < 2; ++ot) {
            f32x16 acc[2];
            acc[0] = acc[1] = unit_frag(w.b2, ot, half);
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const s16x8 wf = frag_w16(w.w2, ot, ks, lane);
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[b] = mfma16(wf, cat8(h1[b][2 * ks], h1[b][2 * ks + 1]), acc[b]);
            }
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    h2[b][4 * ot + g] = relu_pack_bf16x4(acc[b][4 * g], acc[b][4 * g + 1],
                                                         acc[b][4 * g + 2], acc[b][4 * g + 3]);
        }
        // layer 3 and the output unit
        float sum[2] = {0.0f, 0.0f};
#pragma unroll
        for (int ot = 0; ot < 2; ++ot) {
            f32x16 acc[2];
            acc[0] = acc[1] = unit_frag(w.b3, ot, half);
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const s16x8 wf = frag_w16(w.w3, ot, ks, lane);
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[b] = mfma16(wf, cat8(h2[b][2 * ks], h2[b][2 * ks + 1]), acc[b]);
            }
            const f32x16 w4 = unit_frag(w.w4, ot, half);
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 16; ++v) sum[b] += w4[v] * relu_bits(acc[b][v]);
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const float t = sum[b] + __shfl_xor(sum[b], 32, 64);
            if (half == 0 && node[b] < n) y[node[b]] = t + w.b4;
        }
    }
}

// ---------------------------------------------------------------------------
// Training: gradient of L = (1/n) sum_i (y_i - t_i)^2.  One wavefront per
// workgroup; each workgroup accumulates its samples' gradient into its own
// slice of `partial` (NPARAM values + its loss sum), reduced afterwards in a
// fixed order by k_mlp_reduce -- no atomics, deterministic.
// Weight gradients dW = dZ H^T are MFMA products over the tile's 32 nodes:
// activations and deltas are staged in LDS as [unit][node] BF16 so that the
// A fragments (lane = output unit) and B fragments (lane = input unit) are
// 8-byte reads.  An extra row of ones in each staged input gives the bias
// gradients as one more column of the same products.
// ---------------------------------------------------------------------------
constexpr int SSTRIDE = 36;   // staged row stride (bf16): 32 nodes + pad

struct TrainLds {
    MlpLds w;
    unsigned short xs[32 * SSTRIDE];    // rows 0..3 features, 4 ones, rest 0
    unsigned short h1s[96 * SSTRIDE];   // rows 0..63 h1, 64 ones, rest 0
    unsigned short h2s[96 * SSTRIDE];
    unsigned short h3s[96 * SSTRIDE];
    unsigned short d1s[64 * SSTRIDE];   // dz1 [unit][node]
    unsigned short d2s[64 * SSTRIDE];
    unsigned short d3s[64 * SSTRIDE];
    unsigned short dys[32 * SSTRIDE];   // row 0: dL/dy, rest 0
};

__device__ __forceinline__ bf16x4 frag_rows(const unsigned short *s, int row, int ks, int lane)
{
    return *reinterpret_cast<const bf16x4 *>(s + row * SSTRIDE + 8 * ks + 4 * (lane >> 5));
}

// acc[v] -> partial for output tile (mt, nt) of dW = D S^T where D rows are
// output units m and S rows are inputs n; map(m, n) gives the parameter
// index or -1.
template <class Map>
__device__ __forceinline__ void product_to_partial(const unsigned short *D, int mt,
                                                   const unsigned short *S, int nt, float *part,
                                                   Map map)
{
    const int lane = threadIdx.x & 63, half = lane >> 5;
    f32x16 acc = {0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
        acc = mfma(frag_rows(D, 32 * mt + (lane & 31), ks, lane),
                   frag_rows(S, 32 * nt + (lane & 31), ks, lane), acc);
    const int n = 32 * nt + (lane & 31);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int m = 32 * mt + 8 * (v / 4) + 4 * half + (v % 4);
        const int idx = map(m, n);
        if (idx >= 0) part[idx] += acc[v];
    }
}

__global__ __launch_bounds__(64) void k_mlp_grad(const float *__restrict__ P, int64_t n,
                                                 const float *__restrict__ X,
                                                 const float *__restrict__ Tgt,
                                                 int tiles_per_group, float *__restrict__ partials)
{
    __shared__ TrainLds L;
    load_weights(P, L.w);
    const int lane = threadIdx.x;
    const int half = lane >> 5;
    const int j = lane & 31;
    // constant rows: ones and zero padding
    for (int i = lane; i < 32 * SSTRIDE; i += 64) {
        const int row = i / SSTRIDE;
        L.xs[i] = row == 4 ? (unsigned short)0x3f80 : 0;
        L.dys[i] = 0;
    }
    for (int i = lane; i < 96 * SSTRIDE; i += 64) {
        const int row = i / SSTRIDE;
        const unsigned short v = row == 64 ? (unsigned short)0x3f80 : 0;
        L.h1s[i] = v;
        L.h2s[i] = v;
        L.h3s[i] = v;
    }
    float *part = partials + (int64_t)blockIdx.x * (NPARAM + 1);
    for (int i = lane; i < NPARAM + 1; i += 64) part[i] = 0.0f;
    __syncthreads();

    const double inv_n = 1.0 / (double)n;
    float loss = 0.0f;
    Tile T;
    const int64_t t0 = (int64_t)blockIdx.x * tiles_per_group;
    const int64_t n_tiles = (n + 31) / 32;
    for (int64_t tile = t0; tile < min(t0 + tiles_per_group, n_tiles); ++tile) {
        const int64_t node = tile * 32 + j;
        const bool valid = node < n;
        float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
        float tg = 0.0f;
        if (valid) {
            x = reinterpret_cast<const float4 *>(X)[node];
            tg = Tgt[node];
        }
        forward_tile(L.w, x, T, true);
        const float r = valid ? T.y - tg : 0.0f;
        if (half == 0) loss += r * r;
        const float dy = (float)(2.0 * inv_n) * r;

        // output layer: dz3 = dy W4 (z3 > 0); stage h3 and dz3
        bf16x4 d3f[8];
#pragma unroll
        for (int ot = 0; ot < 2; ++ot)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int o = unit_of(ot, v, half);
                const float z = T.z3[16 * ot + v];
                const float dz = z > 0.0f ? dy * L.w.w4[o] : 0.0f;
                d3f[4 * ot + v / 4][v % 4] = (short)f2bf(dz);
                L.d3s[o * SSTRIDE + j] = f2bf(dz);
                L.h3s[o * SSTRIDE + j] = f2bf(fmaxf(z, 0.0f));
            }
        if (half == 0) L.dys[j] = f2bf(dy);
        // dh2 = W3^T dz3 -> dz2 = dh2 (z2 > 0); stage h2 and dz2
        bf16x4 d2f[8];
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            f32x16 acc = {0};
#pragma unroll
            for (int s = 0; s < 8; ++s) acc = mfma(frag_wt(L.w.w3, kt, s, lane), d3f[s], acc);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int k = unit_of(kt, v, half);
                const float z = T.z2[16 * kt + v];
                const float dz = z > 0.0f ? acc[v] : 0.0f;
                d2f[4 * kt + v / 4][v % 4] = (short)f2bf(dz);
                L.d2s[k * SSTRIDE + j] = f2bf(dz);
                L.h2s[k * SSTRIDE + j] = (unsigned short)T.h2[4 * kt + v / 4][v % 4];
            }
        }
        // dh1 = W2^T dz2 -> dz1 = dh1 (z1 > 0); stage h1, dz1, x
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            f32x16 acc = {0};
#pragma unroll
            for (int s = 0; s < 8; ++s) acc = mfma(frag_wt(L.w.w2, kt, s, lane), d2f[s], acc);
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int k = unit_of(kt, v, half);   // = 8 t + 4 half + i, t = 4 kt + v / 4
                const int t = 4 * kt + v / 4, i = v % 4;
                const float z = T.z1[4 * t + i];
                L.d1s[k * SSTRIDE + j] = f2bf(z > 0.0f ? acc[v] : 0.0f);
                L.h1s[k * SSTRIDE + j] = (unsigned short)T.h1[t][i];
            }
        }
        if (half == 0) {
            L.xs[0 * SSTRIDE + j] = f2bf(x.x);
            L.xs[1 * SSTRIDE + j] = f2bf(x.y);
            L.xs[2 * SSTRIDE + j] = f2bf(x.z);
            L.xs[3 * SSTRIDE + j] = f2bf(x.w);
        }
        __syncthreads();
        // weight and bias gradients: MFMA over the tile's 32 nodes
#pragma unroll
        for (int nt = 0; nt < 3; ++nt) {
            product_to_partial(L.dys, 0, L.h3s, nt, part, [](int m, int c) {
                return m == 0 ? (c < NH ? OFF_W4 + c : c == NH ? OFF_B4 : -1) : -1;
            });
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                product_to_partial(L.d3s, mt, L.h2s, nt, part, [](int m, int c) {
                    return c < NH ? OFF_W3 + m * NH + c : c == NH ? OFF_B3 + m : -1;
                });
                product_to_partial(L.d2s, mt, L.h1s, nt, part, [](int m, int c) {
                    return c < NH ? OFF_W2 + m * NH + c : c == NH ? OFF_B2 + m : -1;
                });
            }
        }
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
            product_to_partial(L.d1s, mt, L.xs, 0, part, [](int m, int c) {
                return c < 4 ? OFF_W1 + m * 4 + c : c == 4 ? OFF_B1 + m : -1;
            });
        __syncthreads();
    }
    loss = wave_sum((double)loss);
    if (lane == 0) part[NPARAM] = loss;
}

__global__ __launch_bounds__(256) void k_mlp_reduce(int groups, const float *__restrict__ partials,
                                                    int64_t n, float *__restrict__ grad,
                                                    float *__restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > NPARAM) return;
    float s = 0.0f;
    for (int g = 0; g < groups; ++g) s += partials[(int64_t)g * (NPARAM + 1) + p];
    if (p < NPARAM)
        grad[p] = s;
    else if (loss)
        loss[0] = (float)((double)s / (double)n);
}

__global__ __launch_bounds__(256) void k_adam(float *__restrict__ P, float *__restrict__ m,
                                              float *__restrict__ v, const float *__restrict__ g,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.0f - b1) * gi;
    const float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    P[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace

int mlp_nparams() { return NPARAM; }

int mlp_grad_groups(int64_t n, int max_groups)
{
    const int64_t tiles = (n + 31) / 32;
    const int64_t tpg = std::max<int64_t>(1, (tiles + max_groups - 1) / max_groups);
    return (int)((tiles + tpg - 1) / tpg);
}

size_t mlp_grad_scratch_bytes(int64_t n)
{
    return sizeof(float) * (size_t)(NPARAM + 1) * (size_t)mlp_grad_groups(n, kGradGroups);
}

// Partials of the allocation-free gradient entry point: at most
// kNoAllocGroups workgroups of NPARAM + 1 floats (8.9 MB).  Every device the
// library runs on holds its own copy until the process ends; host code never
// names this array directly (its host-side symbol is not a device address)
// but only the address that mlp_noalloc_scratch resolves per device.
static __device__ __align__(256) float scratch[(size_t)kNoAllocGroups * (NPARAM + 1)];

float *mlp_noalloc_scratch(int device)
{
    static std::mutex mu;
    static std::vector<float *> table;
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0) return nullptr;
    if ((size_t)device >= table.size()) table.resize((size_t)device + 1, nullptr);
    if (!table[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != device) return nullptr;
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        table[device] = static_cast<float *>(ptr);
    }
    return table[device];
}

// inference grid: 160 registers per lane leave three wavefronts per SIMD,
// i.e. three 256-thread workgroups per CU on 256 CUs, all resident at once
constexpr int64_t kInferGroups = 768;

void launch_mlp_forward(hipStream_t s, const float *P, int64_t n, const float *X, float *y)
{
    if (n <= 0) return;
    const int64_t pairs = ((n + 31) / 32 + 1) / 2;
    const int blocks = (int)std::min<int64_t>((pairs + 3) / 4, kInferGroups);
    const FeatIn in{reinterpret_cast<const float4 *>(X), nullptr, nullptr, nullptr, nullptr, 1.0,
                    MlpNorm{}};
    hipLaunchKernelGGL(k_mlp_forward<false>, dim3(blocks), dim3(256), 0, s, P, n, in, y);
}

void launch_mlp_forward_state(hipStream_t s, const float *P, int64_t n, const double *V,
                              const double *Vprev, const double *src, const float *kvp, double cm,
                              const MlpNorm &nm, float *y)
{
    if (n <= 0) return;
    const int64_t pairs = ((n + 31) / 32 + 1) / 2;
    const int blocks = (int)std::min<int64_t>((pairs + 3) / 4, kInferGroups);
    const FeatIn in{nullptr, V, Vprev, src, kvp, 1.0 / cm, nm};
    hipLaunchKernelGGL(k_mlp_forward<true>, dim3(blocks), dim3(256), 0, s, P, n, in, y);
}

void launch_mlp_grad(hipStream_t s, const float *P, int64_t n, const float *X, const float *T,
                     float *grad, float *loss, float *partials, int max_groups)
{
    const int64_t tiles = (n + 31) / 32;
    const int groups = mlp_grad_groups(n, max_groups);
    const int tpg = (int)((tiles + groups - 1) / groups);
    hipLaunchKernelGGL(k_mlp_grad, dim3(groups), dim3(64), 0, s, P, n, X, T, tpg, partials);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NPARAM + 1 + 255) / 256), dim3(256), 0, s, groups,
                       partials, n, grad, loss);
}

void launch_adam(hipStream_t s, float *P, float *m, float *v, const float *g, int t, double lr,
                 double b1, double b2, double eps)
{
    const double c1 = 1.0 - std::pow(b1, (double)t), c2 = 1.0 - std::pow(b2, (double)t);
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, s, P, m, v, g, (float)lr,
                       (float)b1, (float)b2, (float)eps, (float)c1, (float)c2);
}

}  // namespace mdx
