// Learned bandwidth proposal: a 4-layer perceptron 32 -> 128 -> 128 -> 128 -> 16
// (24 summary features and 3 Cholesky coordinates of H, zero padded) with
// ReLU, trained by mean squared error with Adam.
//
// Every matrix product runs on the gfx950 matrix cores: v_mfma_f32_16x16x16
// with BF16 operands and FP32 accumulation. Master parameters, biases, the
// loss and the optimizer state are FP32; the operands of each product
// (weights, layer inputs, and in the backward pass the output gradients) are
// rounded to BF16 (nearest, ties to even) where they enter the product.
// A workgroup (4 wavefronts) owns 64 rows; wavefront w owns rows 16w..16w+15
// of every layer, so the forward pass needs no exchange between wavefronts.
// Gradients are summed per workgroup and then over workgroups in a fixed
// order: results do not depend on scheduling. Built without floating-point
// contraction.

#include "kde_internal.h"

namespace kde {
namespace {

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kRows = kMlpRows;           // rows per workgroup
constexpr int kThreads = 256;
constexpr int kLds = 136;                 // LDS row pitch (bf16 elements)

__device__ __forceinline__ f4 mfma(bf4 a, bf4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }

// FP32 -> BF16, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

struct Lane {
    int lane, wave, i16, q;
    __device__ Lane() {
        lane = threadIdx.x & 63;
        wave = threadIdx.x >> 6;
        i16 = lane & 15;
        q = (lane >> 4) * 4;
    }
};

// out rows of this wavefront = relu(in rows x W + b), W given n-major (Wt[n][k]).
template <int K, int N, bool LAST>
__device__ __forceinline__ void fwd_layer(const uint16_t (*in)[kLds], uint16_t (*out)[kLds], const uint16_t* Wt,
                                          const float* bias, uint16_t* gact, float* y, int64_t row0, int64_t B) {
    const Lane L;
    const int r0 = 16 * L.wave;
    f4 acc[N / 16];
#pragma unroll
    for (int j = 0; j < N / 16; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < K / 16; ++kt) {
        const bf4 a = *reinterpret_cast<const bf4*>(&in[r0 + L.i16][16 * kt + L.q]);
#pragma unroll
        for (int j = 0; j < N / 16; ++j) {
            const bf4 b = *reinterpret_cast<const bf4*>(Wt + (16 * j + L.i16) * K + 16 * kt + L.q);
            acc[j] = mfma(a, b, acc[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < N / 16; ++j) {
        const int col = 16 * j + L.i16;
        const float bj = bias[col];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = r0 + L.q + v;
            const float z = acc[j][v] + bj;
            if constexpr (LAST) {
                if (col < kMlpOut && row0 + row < B) y[(row0 + row) * kMlpOut + col] = z;
            } else {
                const uint16_t h = to_bf16(z > 0.f ? z : 0.f);
                out[row][col] = h;
                if (gact && row0 + row < B) gact[(row0 + row) * N + col] = h;
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) void mlp_fwd_kernel(MlpArgs a) {
    __shared__ uint16_t act[2][kRows][kLds];
    const int tid = threadIdx.x;
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kRows;
    const uint16_t* Wt = a.Wt;
    const float* P = a.P;
    {
        // 64 rows x 32 inputs: 8 per thread
        const int r = tid >> 2, c0 = (tid & 3) * 8;
        const int64_t gr = row0 + r;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int col = c0 + c;
            const float v = (gr < a.B && col < kMlpIn) ? a.X[gr * kMlpIn + col] : 0.f;
            const uint16_t h = to_bf16(v);
            act[0][r][col] = h;
            if (a.acts && gr < a.B) a.acts[gr * kMlpInPad + col] = h;
        }
    }
    __syncthreads();
    uint16_t* g1 = a.acts ? a.acts + a.B * kMlpInPad : nullptr;
    uint16_t* g2 = a.acts ? g1 + a.B * kMlpHid : nullptr;
    uint16_t* g3 = a.acts ? g2 + a.B * kMlpHid : nullptr;
    fwd_layer<kMlpInPad, kMlpHid, false>(act[0], act[1], Wt + kMlpWt1, P + kMlpB1, g1, nullptr, row0, a.B);
    __syncthreads();
    fwd_layer<kMlpHid, kMlpHid, false>(act[1], act[0], Wt + kMlpWt2, P + kMlpB2, g2, nullptr, row0, a.B);
    __syncthreads();
    fwd_layer<kMlpHid, kMlpHid, false>(act[0], act[1], Wt + kMlpWt3, P + kMlpB3, g3, nullptr, row0, a.B);
    __syncthreads();
    fwd_layer<kMlpHid, kMlpOutPad, true>(act[1], nullptr, Wt + kMlpWt4, P + kMlpB4, nullptr, a.Y, row0, a.B);
}

// Stage rows [row0, row0 + 64) x K of a global BF16 activation array into LDS.
template <int K>
__device__ __forceinline__ void stage(uint16_t (*dst)[kLds], const uint16_t* src, int64_t row0, int64_t B) {
    for (int e = threadIdx.x; e < kRows * K; e += kThreads) {
        const int r = e / K, c = e % K;
        dst[r][c] = row0 + r < B ? src[(row0 + r) * K + c] : 0;
    }
}

// Gradient of one layer with input width K and output width N, for this
// workgroup's rows: bias and weight gradients into part, and (PREV) the
// next output gradient dz_prev = (dz W') * (a > 0) into dzf / dzb.
template <int K, int N, bool PREV>
__device__ __forceinline__ void bwd_layer(const uint16_t (*sa)[kLds], uint16_t (*sdz)[kLds], float (*sdzf)[kMlpHid + 4],
                                          const uint16_t* Wk, float* part_W, float* part_b) {
    const Lane L;
    const int tid = threadIdx.x;
    // bias gradient: column sums of the FP32 output gradient, fixed order
    for (int j = tid; j < N; j += kThreads) {
        float s = 0.f;
        for (int r = 0; r < kRows; ++r) s += sdzf[r][j];
        part_b[j] = s;
    }
    // weight gradient dW[k][n] = sum_rows a[r][k] dz[r][n]: (K/16) x (N/16) tiles over the wavefronts
    constexpr int kTiles = (K / 16) * (N / 16);
    for (int t = L.wave; t < kTiles; t += 4) {
        const int kt = t / (N / 16), nt = t % (N / 16);
        f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int it = 0; it < kRows / 16; ++it) {
            bf4 av, bv;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                av[v] = static_cast<short>(sa[16 * it + L.q + v][16 * kt + L.i16]);
                bv[v] = static_cast<short>(sdz[16 * it + L.q + v][16 * nt + L.i16]);
            }
            acc = mfma(av, bv, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) part_W[(16 * kt + L.q + v) * N + 16 * nt + L.i16] = acc[v];
    }
    if constexpr (PREV) {
        // da[r][k] = sum_n dz[r][n] W[k][n]; this wavefront's 16 rows, K/16 column tiles
        const int r0 = 16 * L.wave;
        f4 acc[K / 16];
#pragma unroll
        for (int j = 0; j < K / 16; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int nt = 0; nt < N / 16; ++nt) {
            const bf4 av = *reinterpret_cast<const bf4*>(&sdz[r0 + L.i16][16 * nt + L.q]);
#pragma unroll
            for (int j = 0; j < K / 16; ++j) {
                const bf4 bv = *reinterpret_cast<const bf4*>(Wk + (16 * j + L.i16) * N + 16 * nt + L.q);
                acc[j] = mfma(av, bv, acc[j]);
            }
        }
        __syncthreads();   // every wavefront is done reading sdz / sdzf of this layer
#pragma unroll
        for (int j = 0; j < K / 16; ++j) {
            const int col = 16 * j + L.i16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = r0 + L.q + v;
                const float g = sa[row][col] != 0 ? acc[j][v] : 0.f;   // a = relu(z) > 0 exactly where z > 0
                sdzf[row][col] = g;
                sdz[row][col] = to_bf16(g);
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) void mlp_bwd_kernel(MlpArgs a) {
    __shared__ uint16_t sa[kRows][kLds];
    __shared__ uint16_t sdz[kRows][kLds];
    __shared__ float sdzf[kRows][kMlpHid + 4];
    __shared__ float red[kThreads];
    const int tid = threadIdx.x;
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kRows;
    float* part = a.partial + static_cast<int64_t>(blockIdx.x) * kMlpParams;
    // output gradient of the mean squared error, and this group's share of the loss
    float lsum = 0.f;
    for (int e = tid; e < kRows * kMlpOutPad; e += kThreads) {
        const int r = e / kMlpOutPad, c = e % kMlpOutPad;
        const int64_t gr = row0 + r;
        float g = 0.f;
        if (c < kMlpOut && gr < a.B) {
            const float d = a.Y[gr * kMlpOut + c] - a.T[gr * kMlpOut + c];
            lsum += d * d;
            g = 2.f * d / static_cast<float>(a.B);
        }
        sdzf[r][c] = g;
        sdz[r][c] = to_bf16(g);
    }
    red[tid] = lsum;
    const uint16_t* A0 = a.acts;
    const uint16_t* A1 = A0 + a.B * kMlpInPad;
    const uint16_t* A2 = A1 + a.B * kMlpHid;
    const uint16_t* A3 = A2 + a.B * kMlpHid;
    stage<kMlpHid>(sa, A3, row0, a.B);
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = red[tid] + red[tid + s];
        __syncthreads();
    }
    if (tid == 0) a.loss_partial[blockIdx.x] = red[0];
    bwd_layer<kMlpHid, kMlpOutPad, true>(sa, sdz, sdzf, a.Wk + kMlpWk4, part + kMlpW4, part + kMlpB4);
    __syncthreads();
    stage<kMlpHid>(sa, A2, row0, a.B);
    __syncthreads();
    bwd_layer<kMlpHid, kMlpHid, true>(sa, sdz, sdzf, a.Wk + kMlpWk3, part + kMlpW3, part + kMlpB3);
    __syncthreads();
    stage<kMlpHid>(sa, A1, row0, a.B);
    __syncthreads();
    bwd_layer<kMlpHid, kMlpHid, true>(sa, sdz, sdzf, a.Wk + kMlpWk2, part + kMlpW2, part + kMlpB2);
    __syncthreads();
    stage<kMlpInPad>(sa, A0, row0, a.B);
    __syncthreads();
    bwd_layer<kMlpInPad, kMlpHid, false>(sa, sdz, sdzf, a.Wk + kMlpWk1, part + kMlpW1, part + kMlpB1);
}

// grad[p] = sum over groups of partial[g][p] (group order); loss = sum of the loss partials / B.
__global__ __launch_bounds__(kThreads) void mlp_reduce_kernel(MlpArgs a) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (p < kMlpParams) {
        float s = 0.f;
        for (int64_t g = 0; g < a.groups; ++g) s += a.partial[g * kMlpParams + p];
        a.grad[p] = s;
    }
    if (p == 0 && a.loss) {
        float s = 0.f;
        for (int64_t g = 0; g < a.groups; ++g) s += a.loss_partial[g];
        a.loss[0] = s / static_cast<float>(a.B);
    }
}

// BF16 copies of weight element p (k-major and n-major) from the FP32 master value.
__device__ __forceinline__ void write_bf16(uint16_t* Wk, uint16_t* Wt, int64_t p, float w) {
    const int64_t starts[4] = {kMlpW1, kMlpW2, kMlpW3, kMlpW4};
    const int Ks[4] = {kMlpInPad, kMlpHid, kMlpHid, kMlpHid};
    const int Ns[4] = {kMlpHid, kMlpHid, kMlpHid, kMlpOutPad};
    const int64_t wk[4] = {kMlpWk1, kMlpWk2, kMlpWk3, kMlpWk4};
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const int64_t o = p - starts[l];
        if (o >= 0 && o < static_cast<int64_t>(Ks[l]) * Ns[l]) {
            const int k = static_cast<int>(o / Ns[l]), n = static_cast<int>(o % Ns[l]);
            const uint16_t h = to_bf16(w);
            Wk[wk[l] + static_cast<int64_t>(k) * Ns[l] + n] = h;
            Wt[wk[l] + static_cast<int64_t>(n) * Ks[l] + k] = h;
        }
    }
}

__global__ __launch_bounds__(kThreads) void mlp_adam_kernel(MlpArgs a) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (p >= kMlpParams) return;
    const float g = a.grad[p];
    const float m = a.b1 * a.m[p] + (1.f - a.b1) * g;
    const float v = a.b2 * a.v[p] + (1.f - a.b2) * g * g;
    a.m[p] = m;
    a.v[p] = v;
    const float mh = m / a.c1, vh = v / a.c2;
    const float w = a.Pw[p] - a.lr * mh / (sqrtf(vh) + a.eps);
    a.Pw[p] = w;
    write_bf16(a.Wkw, a.Wtw, p, w);
}

// Load: master parameters from params, moments zeroed, BF16 copies written.
__global__ __launch_bounds__(kThreads) void mlp_load_kernel(MlpArgs a, const float* __restrict__ params) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (p >= kMlpParams) return;
    const float w = params[p];
    a.Pw[p] = w;
    a.m[p] = 0.f;
    a.v[p] = 0.f;
    write_bf16(a.Wkw, a.Wtw, p, w);
}

}  // namespace

hipError_t launch_mlp(int op, const MlpArgs& a, const float* params, hipStream_t s) {
    const dim3 blk(kThreads);
    const unsigned pblocks = static_cast<unsigned>((kMlpParams + kThreads - 1) / kThreads);
    switch (op) {
        case kMlpOpLoad: KDE_LAUNCH(mlp_load_kernel, dim3(pblocks), blk, 0, s, a, params); break;
        case kMlpOpForward:
            KDE_LAUNCH(mlp_fwd_kernel, dim3(static_cast<unsigned>(a.groups)), blk, 0, s, a);
            break;
        case kMlpOpBackward:
            KDE_LAUNCH(mlp_bwd_kernel, dim3(static_cast<unsigned>(a.groups)), blk, 0, s, a);
            break;
        case kMlpOpReduce: KDE_LAUNCH(mlp_reduce_kernel, dim3(pblocks), blk, 0, s, a); break;
        case kMlpOpAdam: KDE_LAUNCH(mlp_adam_kernel, dim3(pblocks), blk, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace kde
