// Learned warm start for the Newmark solve: a per-edge 4 -> 64 -> 64 -> 1 ReLU network on
// gfx950 matrix cores.  Layer 2 (64 x 64) runs as v_mfma_f32_16x16x32_bf16 tiles (BF16
// operands, FP32 accumulation); layer 1 (K = 4) is computed on the vector ALUs straight
// into the MFMA operand layout; layer 3 is a 64-wide dot reduced across lanes.  Training
// uses the same tiles for the backward products dW2 = dZ2^T H1 (reduction over the batch
// rows) and dH1 = dZ2 W2, staged through per-wave LDS tiles; Adam keeps FP32 masters.
//
// Operand layout of v_mfma_f32_16x16x32_bf16 (wave64), lane l, g = l / 16:
//   A (16 x 32):  row l % 16, 8 consecutive k starting at 8 g
//   B (32 x 16):  column l % 16, the same 8 k
//   D (16 x 16):  rows 4 g + i (i = 0..3), column l % 16
// Only the pairing of A's and B's k entries within a lane matters for the sum, and both
// operands are always built with the same k order.
#include <algorithm>

#include "fepic_internal.h"

namespace fepic {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kH = 64;           // hidden width
constexpr int kIn = 4;           // inputs per edge
// flat parameter layout: W1[64][4], b1[64], W2[64][64], b2[64], W3[64], b3
constexpr int oW1 = 0, ob1 = 256, oW2 = 320, ob2 = 4416, oW3 = 4480, ob3 = 4544, kNP = 4545;
static_assert(kNP == FEPIC_MLP_N_PARAMS, "parameter layout");

constexpr int kMlpBlock = 256;   // 4 waves

__device__ __forceinline__ floatx4 mfma(const bf16x8& a, const bf16x8& b, const floatx4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

struct MlpLds {
    float W1[kH * kIn];
    float b1[kH], b2[kH], W3[kH];
    float b3;
    alignas(16) __bf16 W2[kH * kH];    // [n][k]
    alignas(16) __bf16 W2T[kH * kH];   // [k][n]
};

__device__ __forceinline__ void load_params(MlpLds& L, const float* __restrict__ P) {
    for (int i = threadIdx.x; i < kH * kIn; i += blockDim.x) L.W1[i] = P[oW1 + i];
    for (int i = threadIdx.x; i < kH; i += blockDim.x) {
        L.b1[i] = P[ob1 + i];
        L.b2[i] = P[ob2 + i];
        L.W3[i] = P[oW3 + i];
    }
    for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) {
        const __bf16 w = (__bf16)P[oW2 + i];
        L.W2[i] = w;
        L.W2T[(i % kH) * kH + i / kH] = w;
    }
    if (threadIdx.x == 0) L.b3 = P[ob3];
    __syncthreads();
}

// Layer 1 for one row into the A-operand layout: h1[k] = relu(W1[k] . x + b1[k]) for
// k = 32 kb + 8 g + j.
__device__ __forceinline__ bf16x8 layer1_operand(const MlpLds& L, const float x[4], int kb, int g) {
    bf16x8 a;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = 32 * kb + 8 * g + j;
        float z = L.b1[k] + L.W1[4 * k] * x[0] + L.W1[4 * k + 1] * x[1] + L.W1[4 * k + 2] * x[2] + L.W1[4 * k + 3] * x[3];
        a[j] = (__bf16)fmaxf(z, 0.0f);
    }
    return a;
}

// B operand for the forward product: B[k][n] = W2[n][k], n = 16 nt + l % 16,
// k = 32 kb + 8 g + j (8 contiguous entries of row n of W2).
__device__ __forceinline__ bf16x8 w2_operand(const MlpLds& L, int nt, int kb, int lane) {
    const int n = 16 * nt + (lane & 15), g = lane >> 4;
    return *reinterpret_cast<const bf16x8*>(&L.W2[n * kH + 32 * kb + 8 * g]);
}

__device__ __forceinline__ float group16_sum(float v) {
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

// y = network(X) for n rows (X [n][4] FP32, y [n]).  Waves take 16-row tiles.
__global__ __launch_bounds__(kMlpBlock) void k_mlp_forward(int64_t n, const float4* __restrict__ X,
                                                           const float* __restrict__ P, float* __restrict__ y) {
    __shared__ MlpLds L;
    load_params(L, P);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
    bf16x8 B[4][2];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) B[nt][kb] = w2_operand(L, nt, kb, lane);
    const int64_t n_tiles = (n + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < n_tiles; t += (int64_t)gridDim.x * 4) {
        const int64_t row = 16 * t + c;
        float x[4] = {0.f, 0.f, 0.f, 0.f};
        if (row < n) {
            const float4 v = X[row];
            x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
        }
        const bf16x8 a0 = layer1_operand(L, x, 0, g), a1 = layer1_operand(L, x, 1, g);
        float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma(a0, B[nt][0], acc);
            acc = mfma(a1, B[nt][1], acc);
            const int nn = 16 * nt + c;
#pragma unroll
            for (int i = 0; i < 4; ++i) part[i] += fmaxf(acc[i] + L.b2[nn], 0.0f) * L.W3[nn];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float s = group16_sum(part[i]);
            const int64_t r = 16 * t + 4 * g + i;
            if (c == 0 && r < n) y[r] = s + L.b3;
        }
    }
}

// Minibatch source: explicit rows, or rows drawn from a recorded set by a counter-based
// hash of (seed, step, position).
struct BatchSrc {
    const float4* X;
    const float* T;
    int64_t n;            // rows in this minibatch
    int64_t n_all;        // rows in the recorded set (0 = explicit rows)
    uint64_t seed;
};

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int64_t batch_row(const BatchSrc& s, int64_t i) {
    return s.n_all ? (int64_t)(mix64(s.seed ^ (uint64_t)i * 0xD1B54A32D192ED03ull) % (uint64_t)s.n_all) : i;
}

// Gradient of L = (1/N) sum (y - t)^2 over a minibatch; every workgroup writes the sum of
// its rows' gradients (4545 values) and of its squared errors to part[blockIdx].
// Waves take 32-row tiles (two 16-row halves for the forward product, one K = 32 block
// for dW2).
__global__ __launch_bounds__(kMlpBlock) void k_mlp_grad(BatchSrc src, float inv_n, const float* __restrict__ P,
                                                        float* __restrict__ part, double* __restrict__ loss_part) {
    __shared__ MlpLds L;
    // per-wave tiles: dZ2 [row][n] and H1 [row][k] (BF16); after the main loop the same
    // memory holds the cross-wave reduction of dW2 (FP32 [n][k])
    __shared__ alignas(16) __bf16 sTiles[2][4][32 * kH];
    __bf16 (*sZ)[32 * kH] = sTiles[0];
    __bf16 (*sH)[32 * kH] = sTiles[1];
    float* sRed = reinterpret_cast<float*>(&sTiles[0][0][0]);
    __shared__ float sX[4][32 * 4];
    __shared__ float sVec[4][4 * kH + 1];
    __shared__ double sLoss[4];
    load_params(L, P);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;

    floatx4 dW2[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) dW2[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    float dW1[4][4] = {}, db1[4] = {}, db2[4] = {}, dW3[4] = {};
    float db3 = 0.f;
    double loss = 0.0;

    const int64_t n_tiles = (src.n + 31) / 32;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < n_tiles; t += (int64_t)gridDim.x * 4) {
        // ---- forward and the output-layer backward, per 16-row half
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t i0 = 32 * t + 16 * h;
            float x[4] = {0.f, 0.f, 0.f, 0.f};
            {
                const int64_t i = i0 + c;
                if (i < src.n) {
                    const float4 v = src.X[batch_row(src, i)];
                    x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
                }
            }
            if (g == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) sX[wave][(16 * h + c) * 4 + q] = x[q];
            }
            const bf16x8 a0 = layer1_operand(L, x, 0, g), a1 = layer1_operand(L, x, 1, g);
            // H1 tile (row c of this half, k = 32 kb + 8 g + j)
            *reinterpret_cast<bf16x8*>(&sH[wave][(16 * h + c) * kH + 8 * g]) = a0;
            *reinterpret_cast<bf16x8*>(&sH[wave][(16 * h + c) * kH + 32 + 8 * g]) = a1;
            floatx4 z2[4];
            float part_y[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                floatx4 acc = {0.f, 0.f, 0.f, 0.f};
                acc = mfma(a0, w2_operand(L, nt, 0, lane), acc);
                acc = mfma(a1, w2_operand(L, nt, 1, lane), acc);
                const int nn = 16 * nt + c;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    acc[i] += L.b2[nn];
                    part_y[i] += fmaxf(acc[i], 0.0f) * L.W3[nn];
                }
                z2[nt] = acc;
            }
            float dy[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float yv = group16_sum(part_y[i]) + L.b3;
                const int64_t r = i0 + 4 * g + i;
                float e = 0.f;
                if (r < src.n) e = yv - src.T[batch_row(src, r)];
                dy[i] = 2.0f * inv_n * e;
                if (c == 0) {
                    loss += (double)e * e;
                    db3 += dy[i];
                }
            }
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int nn = 16 * nt + c;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float z = z2[nt][i];
                    const float h2 = fmaxf(z, 0.0f);
                    dW3[nt] += dy[i] * h2;
                    const float dz = (z > 0.0f) ? dy[i] * L.W3[nn] : 0.0f;
                    db2[nt] += dz;
                    sZ[wave][(16 * h + 4 * g + i) * kH + nn] = (__bf16)dz;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // ---- dW2[n][k] += sum over the 32 rows of dZ2[m][n] H1[m][k] (K = rows)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            bf16x8 a;
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = sZ[wave][(8 * g + j) * kH + 16 * nt + c];
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) {
                bf16x8 b;
#pragma unroll
                for (int j = 0; j < 8; ++j) b[j] = sH[wave][(8 * g + j) * kH + 16 * kt + c];
                dW2[nt][kt] = mfma(a, b, dW2[nt][kt]);
            }
        }
        // ---- dH1 = dZ2 W2 per 16-row half, then through the first ReLU
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(&sZ[wave][(16 * h + c) * kH + 8 * g]);
            const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(&sZ[wave][(16 * h + c) * kH + 32 + 8 * g]);
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) {
                const int k = 16 * kt + c;
                // B[n][k] = W2[n][k], n = 32 nb + 8 g + j: contiguous in W2^T row k
                const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(&L.W2T[k * kH + 8 * g]);
                const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(&L.W2T[k * kH + 32 + 8 * g]);
                floatx4 acc = {0.f, 0.f, 0.f, 0.f};
                acc = mfma(a0, b0, acc);
                acc = mfma(a1, b1, acc);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int m = 16 * h + 4 * g + i;
                    const float* xr = &sX[wave][m * 4];
                    const float z1 = L.b1[k] + L.W1[4 * k] * xr[0] + L.W1[4 * k + 1] * xr[1] +
                                     L.W1[4 * k + 2] * xr[2] + L.W1[4 * k + 3] * xr[3];
                    const float dz1 = (z1 > 0.0f) ? acc[i] : 0.0f;
                    db1[kt] += dz1;
#pragma unroll
                    for (int q = 0; q < 4; ++q) dW1[kt][q] += dz1 * xr[q];
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }

    // ---- block reduction into part[blockIdx.x][0..4544]
    float* out = part + (size_t)blockIdx.x * kNP;
    __syncthreads();  // every wave is done with its tiles before they become sRed
    for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) sRed[i] = 0.f;
    __syncthreads();
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int kt = 0; kt < 4; ++kt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) sRed[(16 * nt + 4 * g + i) * kH + 16 * kt + c] += dW2[nt][kt][i];
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) out[oW2 + i] = sRed[i];
    // per-k / per-n vectors: sum over the 4 lane groups, then over waves
    float vec[4 * 4 + 4 + 4 + 4];
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
#pragma unroll
        for (int q = 0; q < 4; ++q) vec[4 * kt + q] = dW1[kt][q];
        vec[16 + kt] = db1[kt];
        vec[20 + kt] = db2[kt];
        vec[24 + kt] = dW3[kt];
    }
#pragma unroll
    for (int v = 0; v < 28; ++v) {
        vec[v] += __shfl_xor(vec[v], 16);
        vec[v] += __shfl_xor(vec[v], 32);
    }
    float b3s = db3;
    for (int off = 32; off > 0; off >>= 1) b3s += __shfl_xor(b3s, off);
    for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off);
    if (g == 0) {
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            const int k = 16 * kt + c;
#pragma unroll
            for (int q = 0; q < 4; ++q) sVec[wave][4 * k + q] = vec[4 * kt + q];
        }
    }
    __syncthreads();
    if (threadIdx.x < 4 * kH) {
        float a = 0.f;
        for (int w = 0; w < 4; ++w) a += sVec[w][threadIdx.x];
        out[oW1 + threadIdx.x] = a;
    }
    __syncthreads();
    if (g == 0) {
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            const int k = 16 * kt + c;
            sVec[wave][k] = vec[16 + kt];
            sVec[wave][kH + k] = vec[20 + kt];
            sVec[wave][2 * kH + k] = vec[24 + kt];
        }
    }
    if (lane == 0) {
        sVec[wave][4 * kH] = b3s;
        sLoss[wave] = loss;
    }
    __syncthreads();
    if (threadIdx.x < 3 * kH) {
        float a = 0.f;
        for (int w = 0; w < 4; ++w) a += sVec[w][threadIdx.x];
        const int which = threadIdx.x / kH, k = threadIdx.x % kH;
        out[(which == 0 ? ob1 : which == 1 ? ob2 : oW3) + k] = a;
    }
    if (threadIdx.x == 0) {
        out[ob3] = sVec[0][4 * kH] + sVec[1][4 * kH] + sVec[2][4 * kH] + sVec[3][4 * kH];
        loss_part[blockIdx.x] = sLoss[0] + sLoss[1] + sLoss[2] + sLoss[3];
    }
}

// grad[p] = sum over blocks (fixed order); optional Adam update of the FP32 masters.
__global__ __launch_bounds__(256) void k_mlp_reduce_adam(const float* __restrict__ part, int n_blocks,
                                                         float* __restrict__ grad, float* __restrict__ P,
                                                         float* __restrict__ m, float* __restrict__ v, int adam,
                                                         float lr, float b1, float b2, float eps, float bc1,
                                                         float bc2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNP) return;
    float s = 0.f;
    for (int b = 0; b < n_blocks; ++b) s += part[(size_t)b * kNP + p];
    if (grad) grad[p] = s;
    if (adam) {
        const float mm = b1 * m[p] + (1.f - b1) * s;
        const float vv = b2 * v[p] + (1.f - b2) * s * s;
        m[p] = mm;
        v[p] = vv;
        P[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
    }
}

// Mean squared error from the per-workgroup sums of k_mlp_grad (fixed order, one thread).
__global__ __launch_bounds__(64) void k_mlp_loss_sum(const double* __restrict__ loss_part, int n_blocks, double inv_n,
                                                     double* __restrict__ loss) {
    if (threadIdx.x != 0) return;
    double a = 0.0;
    for (int b = 0; b < n_blocks; ++b) a += loss_part[b];
    loss[0] = a * inv_n;
}

// Per-edge features over the interior edges: e / s_e, (e - e_prev) / s_d,
// (e_prev - e_prev2) / s_d (differences in FP64, before the rounding), dG / s_g.
__global__ __launch_bounds__(256) void k_mlp_features(int64_t n_int, const int32_t* __restrict__ ie,
                                                      const double* __restrict__ e, const double* __restrict__ ep,
                                                      const double* __restrict__ ep2, const double* __restrict__ dg,
                                                      const double* __restrict__ scales, float4* __restrict__ X) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n_int) return;
    const int k = ie[j];
    const double se = 1.0 / scales[4], sd = 1.0 / scales[0], sg = 1.0 / scales[1];
    const double en = e[k], e1 = ep[k];
    X[j] = make_float4((float)(en * se), (float)((en - e1) * sd), (float)((e1 - ep2[k]) * sd), (float)(dg[k] * sg));
}

// The scales of the inputs over interior edges (each 1 where zero): s_d = RMS of
// e^n - e^{n-1} into scales[0], s_g = RMS of dG into scales[1], s_e = RMS of e^n into
// scales[4]; per-workgroup sums of squares (grid-stride), then one workgroup adds them in
// a fixed order.
constexpr int kRmsBlocks = 256;

__global__ __launch_bounds__(256) void k_mlp_rms_part(int64_t n_int, const int32_t* __restrict__ ie,
                                                      const double* __restrict__ e, const double* __restrict__ ep,
                                                      const double* __restrict__ dg, double* __restrict__ part) {
    __shared__ double s[3][4];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n_int; j += (int64_t)gridDim.x * 256) {
        const int k = ie[j];
        const double en = e[k], d = en - ep[k], g = dg[k];
        a += en * en;
        b += d * d;
        c += g * g;
    }
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
        c += __shfl_xor(c, off);
    }
    if ((threadIdx.x & 63) == 0) {
        s[0][threadIdx.x >> 6] = a;
        s[1][threadIdx.x >> 6] = b;
        s[2][threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int q = threadIdx.x;
        part[q * kRmsBlocks + blockIdx.x] = (s[q][0] + s[q][1]) + (s[q][2] + s[q][3]);
    }
}

__global__ __launch_bounds__(256) void k_mlp_rms_fin(int64_t n_int, int nb, const double* __restrict__ part,
                                                     double* __restrict__ scales) {
    __shared__ double s[3][4];
    double v[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) v[q] = threadIdx.x < nb ? part[q * kRmsBlocks + threadIdx.x] : 0.0;
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int q = 0; q < 3; ++q) v[q] += __shfl_xor(v[q], off);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < 3; ++q) s[q][threadIdx.x >> 6] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        double r[3];
        for (int q = 0; q < 3; ++q) {
            const double sum = (s[q][0] + s[q][1]) + (s[q][2] + s[q][3]);
            r[q] = n_int ? sqrt(sum / (double)n_int) : 0.0;
            if (!(r[q] > 0.0)) r[q] = 1.0;
        }
        scales[4] = r[0];
        scales[0] = r[1];
        scales[1] = r[2];
    }
}

// Rows r0, r0 + stride, ... (n of them) of X [rows][4] into dst: the subsample of edges a
// snapshot records.
__global__ __launch_bounds__(256) void k_mlp_pick(const float4* __restrict__ X, int64_t r0, int64_t stride, int64_t n,
                                                  float4* __restrict__ dst) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < n) dst[j] = X[r0 + j * stride];
}

// Predicted increment as an edge vector: d[ie] = s_d y (d is zero elsewhere).
__global__ __launch_bounds__(256) void k_mlp_direction(int64_t n_int, const int32_t* __restrict__ ie,
                                                       const float* __restrict__ y, const double* __restrict__ scales,
                                                       double* __restrict__ d) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n_int) return;
    d[ie[j]] = scales[0] * (double)y[j];
}

// Training target, first pass: the increments e^{n+1} - e^n on interior edges r0,
// r0 + stride, ... (n rows) into d (FP64) and per-workgroup sums of their squares.
__global__ __launch_bounds__(256) void k_mlp_target(int64_t n, int64_t r0, int64_t stride,
                                                    const int32_t* __restrict__ ie, const double* __restrict__ e_new,
                                                    const double* __restrict__ e, double* __restrict__ d,
                                                    double* __restrict__ part) {
    __shared__ double s[4];
    double a = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
        const int k = ie[r0 + j * stride];
        const double v = e_new[k] - e[k];
        d[j] = v;
        a += v * v;
    }
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

// Second pass: t = d / s_d, and (workgroup 0) the RMS of t into scales[3], by which the host
// leaves out steps where the history is near zero (a neutral start) and the increment
// dwarfs it.
__global__ __launch_bounds__(256) void k_mlp_target_scale(int64_t n, int nb, const double* __restrict__ part,
                                                          const double* __restrict__ d, double* __restrict__ scales,
                                                          float* __restrict__ t) {
    const double inv = 1.0 / scales[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double a = 0.0;
        for (int b = 0; b < nb; ++b) a += part[b];
        scales[3] = n ? sqrt(a / (double)n) * inv : 0.0;
    }
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256)
        t[j] = (float)(d[j] * inv);
}

}  // namespace

// ------------------------------------------------------------------------- launchers
int mlp_grad_blocks(int64_t n) {
    const int64_t tiles = (n + 31) / 32;
    int64_t b = (tiles + 15) / 16;  // about 4 tiles per wave
    if (b < 1) b = 1;
    if (b > 512) b = 512;
    return (int)b;
}

void mlp_launch_rms(hipStream_t s, int64_t n_int, const int32_t* ie, const double* e, const double* ep,
                    const double* dg, double* part, double* scales) {
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kRmsBlocks, (n_int + 1023) / 1024));
    hipLaunchKernelGGL(k_mlp_rms_part, dim3(nb), dim3(256), 0, s, n_int, ie, e, ep, dg, part);
    hipLaunchKernelGGL(k_mlp_rms_fin, dim3(1), dim3(256), 0, s, n_int, nb, part, scales);
}

void mlp_launch_features(hipStream_t s, int64_t n_int, const int32_t* ie, const double* e, const double* ep,
                         const double* ep2, const double* dg, const double* scales, float* X) {
    if (n_int <= 0) return;
    hipLaunchKernelGGL(k_mlp_features, dim3(grid_1d(n_int, 256)), dim3(256), 0, s, n_int, ie, e, ep, ep2, dg, scales,
                       (float4*)X);
}

void mlp_launch_forward(hipStream_t s, int64_t n, const float* X, const float* P, float* y) {
    if (n <= 0) return;
    const int64_t tiles = (n + 15) / 16;
    int64_t blocks = (tiles + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(kMlpBlock), 0, s, n, (const float4*)X, P, y);
}

void mlp_launch_direction(hipStream_t s, int64_t n_int, const int32_t* ie, const float* y, const double* scales,
                          double* d) {
    if (n_int <= 0) return;
    hipLaunchKernelGGL(k_mlp_direction, dim3(grid_1d(n_int, 256)), dim3(256), 0, s, n_int, ie, y, scales, d);
}

void mlp_launch_target(hipStream_t s, int64_t n, int64_t r0, int64_t stride, const int32_t* ie, const double* e_new,
                       const double* e, double* work, double* part, double* scales, float* t) {
    if (n <= 0) return;
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kRmsBlocks, (n + 1023) / 1024));
    hipLaunchKernelGGL(k_mlp_target, dim3(nb), dim3(256), 0, s, n, r0, stride, ie, e_new, e, work, part);
    hipLaunchKernelGGL(k_mlp_target_scale, dim3(nb), dim3(256), 0, s, n, nb, part, work, scales, t);
}

void mlp_launch_pick(hipStream_t s, const float* X, int64_t r0, int64_t stride, int64_t n, float* dst) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_pick, dim3(grid_1d(n, 256)), dim3(256), 0, s, (const float4*)X, r0, stride, n,
                       (float4*)dst);
}

void mlp_launch_grad(hipStream_t s, const float* X, const float* T, int64_t n, int64_t n_all, uint64_t seed,
                     const float* P, float* part, double* loss_part, int blocks) {
    BatchSrc src{(const float4*)X, T, n, n_all, seed};
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(kMlpBlock), 0, s, src, 1.0f / (float)n, P, part, loss_part);
}

void mlp_launch_loss_sum(hipStream_t s, const double* loss_part, int blocks, double inv_n, double* loss) {
    hipLaunchKernelGGL(k_mlp_loss_sum, dim3(1), dim3(64), 0, s, loss_part, blocks, inv_n, loss);
}

void mlp_launch_reduce_adam(hipStream_t s, const float* part, int blocks, float* grad, float* P, float* m, float* v,
                            int adam, float lr, float b1, float b2, float eps, float bc1, float bc2) {
    hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((kNP + 255) / 256), dim3(256), 0, s, part, blocks, grad, P, m, v, adam,
                       lr, b1, b2, eps, bc1, bc2);
}

}  // namespace fepic
