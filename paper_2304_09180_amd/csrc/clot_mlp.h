// BF16 MFMA multilayer perceptron of the reaction surrogate (gfx950).
//
// Network: 32 inputs -> 64 tanh -> 64 tanh -> 16 outputs (14 used), BF16 weights and
// activations, FP32 accumulation, every layer on v_mfma_f32_16x16x16_bf16 (a wave
// multiplies 16x16 tiles; a group of 16 cells is the N dimension).
//
// Operand layout of the 16x16x16 BF16 MFMA (lane l in 0..63, element e in 0..3):
//   A (M x K): row l%16,  k = 4*(l/16) + e
//   B (K x N): col l%16,  k = 4*(l/16) + e
//   D (M x N): col l%16,  row = 4*(l/16) + e
// so the D tile of one 16-row block of a layer is, lane for lane, the B tile of the
// matching 16-k block of the next layer.  k_mfma_selftest checks this layout.
#pragma once
#include "clot_common.h"

namespace clot {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MLP_IN = 32, MLP_H = 64, MLP_OUT = 16, MLP_NSP = 14;
// float32 parameter block: W1[64][32] b1[64] W2[64][64] b2[64] W3[16][64] b3[16]
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * MLP_IN, MLP_OFF_W2 = MLP_OFF_B1 + MLP_H,
              MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H, MLP_OFF_W3 = MLP_OFF_B2 + MLP_H,
              MLP_OFF_B3 = MLP_OFF_W3 + MLP_OUT * MLP_H, MLP_NPARAM = MLP_OFF_B3 + MLP_OUT;

// Round-to-nearest-even float -> bf16 bits (finite inputs).
__host__ __device__ inline uint16_t f2bf(float f) {
    union {
        float f;
        uint32_t u;
    } v;
    v.f = f;
    const uint32_t r = 0x7FFFu + ((v.u >> 16) & 1u);
    return (uint16_t)((v.u + r) >> 16);
}
__host__ __device__ inline float bf2f(uint16_t h) {
    union {
        float f;
        uint32_t u;
    } v;
    v.u = (uint32_t)h << 16;
    return v.f;
}

// Four floats to bf16 with the hardware round-to-nearest-even conversion
// (v_cvt_pk_bf16_f32; the same rounding as f2bf for finite values).
__device__ inline bf16x4 pack4_bf16(float a, float b, float c, float d) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    typedef __bf16 h4 __attribute__((ext_vector_type(4)));
    const h4 h = __builtin_convertvector((f4){a, b, c, d}, h4);
    return __builtin_bit_cast(bf16x4, h);
}

__device__ inline f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// A operand from a row-major bf16 matrix M[rows][ld], tile (r0, k0).
__device__ inline bf16x4 load_a(const uint16_t* M, int ld, int r0, int k0) {
    const int l = threadIdx.x & 63;
    const uint16_t* p = M + (r0 + (l & 15)) * ld + k0 + 4 * (l >> 4);
    bf16x4 a;
    a[0] = (short)p[0];
    a[1] = (short)p[1];
    a[2] = (short)p[2];
    a[3] = (short)p[3];
    return a;
}
// A operand of the transpose of M (M row-major [rows][ld]): A[i][k] = M[k][i].
__device__ inline bf16x4 load_at(const uint16_t* M, int ld, int r0, int k0) {
    const int l = threadIdx.x & 63;
    const int i = r0 + (l & 15), k = k0 + 4 * (l >> 4);
    bf16x4 a;
    a[0] = (short)M[(k + 0) * ld + i];
    a[1] = (short)M[(k + 1) * ld + i];
    a[2] = (short)M[(k + 2) * ld + i];
    a[3] = (short)M[(k + 3) * ld + i];
    return a;
}
// B operand from a "cell-major" bf16 matrix X[n][ldx] holding B[k][n] = X[n][k].
__device__ inline bf16x4 load_b_cm(const uint16_t* X, int ldx, int k0, int n0) {
    const int l = threadIdx.x & 63;
    const uint16_t* p = X + (n0 + (l & 15)) * ldx + k0 + 4 * (l >> 4);
    bf16x4 b;
    b[0] = (short)p[0];
    b[1] = (short)p[1];
    b[2] = (short)p[2];
    b[3] = (short)p[3];
    return b;
}

// Layout self-test: D = A (16x16) * B (16x16), A, B row-major bf16, D row-major f32.
__global__ void k_mfma_selftest(const uint16_t* A, const uint16_t* B, float* D) {
    const int l = threadIdx.x;
    __shared__ uint16_t Bt[16 * 16];   // cell-major copy of B: Bt[n][k] = B[k][n]
    for (int q = l; q < 256; q += 64) Bt[(q % 16) * 16 + q / 16] = B[q];
    __syncthreads();
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = mfma16(load_a(A, 16, 0, 0), load_b_cm(Bt, 16, 0, 0), c);
    for (int e = 0; e < 4; ++e) D[(4 * (l >> 4) + e) * 16 + (l & 15)] = c[e];
}

// ---------------------------------------------------------------------------------
// Wave-level MLP forward for 16 cells, chained through registers: the D tile of one
// layer's 16-unit block is the B operand of the next layer's matching k block, so
// only the inputs and the outputs pass through memory.
// ---------------------------------------------------------------------------------
struct MLPWeights {
    const uint16_t* W1;
    const uint16_t* W2;
    const uint16_t* W3;
    const float* b1;
    const float* b2;
    const float* b3;
};

// tanh(x) = 1 - 2/(1 + e^{2x}), with the hardware exp2 and reciprocal: absolute
// error a few 1e-7, far below the bf16 rounding the activations then take; +-inf
// saturate to +-1.
__device__ inline float fast_tanh(float x) {
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);   // 2 log2(e)
    return fmaf(-2.f, __builtin_amdgcn_rcpf(1.f + e), 1.f);
}

__device__ inline bf16x4 act_bf16(f32x4 c, const float* b, int u0) {
    const float4 bb = *reinterpret_cast<const float4*>(b + u0);
    return pack4_bf16(fast_tanh(c[0] + bb.x), fast_tanh(c[1] + bb.y), fast_tanh(c[2] + bb.z), fast_tanh(c[3] + bb.w));
}

// The A operands of all three layers for one wave (28 x 4 bf16 per lane).
struct MLPRegs {
    bf16x4 w1[4][2], w2[4][4], w3[4];
    __device__ inline void load(const MLPWeights& w) {
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) w1[rb][kb] = load_a(w.W1, MLP_IN, 16 * rb, 16 * kb);
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) w2[rb][kb] = load_a(w.W2, MLP_H, 16 * rb, 16 * kb);
        }
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) w3[kb] = load_a(w.W3, MLP_H, 0, 16 * kb);
    }
};

// x[kb]: B operands of the 16 cells' inputs (k block kb of 32).  Returns lane l's
// outputs 4*(l/16)+e of cell l%16; h1/h2 receive the bf16 activations of units
// 16*rb + 4*(l/16) + e of that cell.
__device__ inline f32x4 mlp_chain16(const MLPRegs& R, const MLPWeights& w, const bf16x4 (&x)[2], bf16x4 (&h1)[4],
                                    bf16x4 (&h2)[4]) {
    const int rq = 4 * ((threadIdx.x & 63) >> 4);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
        c = mfma16(R.w1[rb][0], x[0], c);
        c = mfma16(R.w1[rb][1], x[1], c);
        h1[rb] = act_bf16(c, w.b1, 16 * rb + rq);
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) c = mfma16(R.w2[rb][kb], h1[kb], c);
        h2[rb] = act_bf16(c, w.b2, 16 * rb + rq);
    }
    const float4 b3 = *reinterpret_cast<const float4*>(w.b3 + rq);
    f32x4 c = {b3.x, b3.y, b3.z, b3.w};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) c = mfma16(R.w3[kb], h2[kb], c);
    return c;
}

// Forward over a batch: x bf16 [n][32] (cell-major), y f32 [n][16]; cache (optional)
// bf16 [n][128] = h1, h2.  One wave per 64 samples (four groups of 16); 4 waves per
// block.
__global__ __launch_bounds__(256) void k_mlp_forward(MLPWeights w, const uint16_t* x, int64_t n, float* y,
                                                     uint16_t* cache) {
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int rq = 4 * (l >> 4);
    MLPRegs R;
    R.load(w);
    for (int grp = 0; grp < 4; ++grp) {
        const int64_t c = ((int64_t)blockIdx.x * 4 + wv) * 64 + 16 * grp + (l & 15);
        const bool in = c < n;
        bf16x4 xb[2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            if (in) {
                const uint2 v = *reinterpret_cast<const uint2*>(x + c * MLP_IN + 16 * kb + rq);
                xb[kb][0] = (short)(v.x & 0xFFFF);
                xb[kb][1] = (short)(v.x >> 16);
                xb[kb][2] = (short)(v.y & 0xFFFF);
                xb[kb][3] = (short)(v.y >> 16);
            } else {
                xb[kb] = bf16x4{0, 0, 0, 0};
            }
        }
        bf16x4 h1[4], h2[4];
        const f32x4 o = mlp_chain16(R, w, xb, h1, h2);
        if (in) {
            *reinterpret_cast<float4*>(y + c * MLP_OUT + rq) = make_float4(o[0], o[1], o[2], o[3]);
            if (cache) {
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    *reinterpret_cast<bf16x4*>(cache + c * 2 * MLP_H + 16 * rb + rq) = h1[rb];
                    *reinterpret_cast<bf16x4*>(cache + c * 2 * MLP_H + MLP_H + 16 * rb + rq) = h2[rb];
                }
            }
        }
    }
}

// Backward over a batch.  dy f32 [n][16] = dLoss/dy.  Each wave back-propagates 16
// samples with MFMA (delta2 = W3^T dy (.) (1-h2^2), delta1 = W2^T delta2 (.) (1-h1^2))
// and forms its weight-gradient contributions with MFMA, the 16 samples being the
// contraction dimension; block partials go to part[block][MLP_NPARAM] (float),
// reduced in a fixed order by k_mlp_reduce.
__global__ __launch_bounds__(256) void k_mlp_backward(MLPWeights w, const uint16_t* x, const uint16_t* cache,
                                                      const float* dy, int64_t n, float* part) {
    __shared__ uint16_t sX[4][16 * MLP_IN];
    __shared__ uint16_t sH1[4][16 * MLP_H];
    __shared__ uint16_t sH2[4][16 * MLP_H];
    __shared__ uint16_t sD3[4][16 * MLP_OUT];   // cell-major bf16 deltas
    __shared__ uint16_t sD2[4][16 * MLP_H];
    __shared__ uint16_t sD1[4][16 * MLP_H];
    __shared__ float sG[MLP_NPARAM];
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int col = l & 15, rq = 4 * (l >> 4);
    for (int q = threadIdx.x; q < MLP_NPARAM; q += 256) sG[q] = 0.f;
    const int64_t c0 = ((int64_t)blockIdx.x * 4 + wv) * 16;
    for (int q = l; q < 16 * MLP_IN; q += 64) {
        const int64_t c = c0 + q / MLP_IN;
        sX[wv][q] = c < n ? x[c * MLP_IN + q % MLP_IN] : (uint16_t)0;
    }
    for (int q = l; q < 16 * MLP_H; q += 64) {
        const int64_t c = c0 + q / MLP_H;
        sH1[wv][q] = c < n ? cache[c * 2 * MLP_H + q % MLP_H] : (uint16_t)0;
        sH2[wv][q] = c < n ? cache[c * 2 * MLP_H + MLP_H + q % MLP_H] : (uint16_t)0;
    }
    for (int q = l; q < 16 * MLP_OUT; q += 64) {
        const int64_t c = c0 + q / MLP_OUT;
        sD3[wv][q] = f2bf(c < n ? dy[c * MLP_OUT + q % MLP_OUT] : 0.f);
    }
    __syncthreads();
    // delta2 (64 x 16) = W3^T (64 x 16) dy^T (16 x 16) (.) (1 - h2^2)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
        c = mfma16(load_at(w.W3, MLP_H, 16 * rb, 0), load_b_cm(sD3[wv], MLP_OUT, 0, 0), c);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int u = 16 * rb + rq + e;
            const float h = bf2f(sH2[wv][col * MLP_H + u]);
            sD2[wv][col * MLP_H + u] = f2bf(c[e] * (1.f - h * h));
        }
    }
    __syncthreads();
    // delta1 (64 x 16) = W2^T delta2 (.) (1 - h1^2)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) c = mfma16(load_at(w.W2, MLP_H, 16 * rb, 16 * kb), load_b_cm(sD2[wv], MLP_H, 16 * kb, 0), c);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int u = 16 * rb + rq + e;
            const float h = bf2f(sH1[wv][col * MLP_H + u]);
            sD1[wv][col * MLP_H + u] = f2bf(c[e] * (1.f - h * h));
        }
    }
    __syncthreads();
    // weight gradients: dW = Delta (out x 16 samples) * Act^T (16 samples x in), the
    // A operand is the transpose of the cell-major delta, B the cell-major activation
    // read as B[k=sample][n=unit] = Act[sample][unit].
    auto gemm_acc = [&](const uint16_t* Dl, int ldd, int nout, const uint16_t* Act, int lda, int nin, int off) {
        for (int rb = 0; rb < nout / 16; ++rb)
            for (int cb = 0; cb < nin / 16; ++cb) {
                f32x4 c = {0.f, 0.f, 0.f, 0.f};
                // A[i][k] = Dl[k][16rb+i]  (k = sample)
                bf16x4 a;
                {
                    const int i = 16 * rb + (l & 15), k = 4 * (l >> 4);
                    a[0] = (short)Dl[(k + 0) * ldd + i];
                    a[1] = (short)Dl[(k + 1) * ldd + i];
                    a[2] = (short)Dl[(k + 2) * ldd + i];
                    a[3] = (short)Dl[(k + 3) * ldd + i];
                }
                // B[k][j] = Act[k][16cb+j]
                bf16x4 b;
                {
                    const int j = 16 * cb + (l & 15), k = 4 * (l >> 4);
                    b[0] = (short)Act[(k + 0) * lda + j];
                    b[1] = (short)Act[(k + 1) * lda + j];
                    b[2] = (short)Act[(k + 2) * lda + j];
                    b[3] = (short)Act[(k + 3) * lda + j];
                }
                c = mfma16(a, b, c);
#pragma unroll
                for (int e = 0; e < 4; ++e) atomicAdd(&sG[off + (16 * rb + rq + e) * nin + 16 * cb + col], c[e]);
            }
    };
    gemm_acc(sD3[wv], MLP_OUT, MLP_OUT, sH2[wv], MLP_H, MLP_H, MLP_OFF_W3);
    gemm_acc(sD2[wv], MLP_H, MLP_H, sH1[wv], MLP_H, MLP_H, MLP_OFF_W2);
    gemm_acc(sD1[wv], MLP_H, MLP_H, sX[wv], MLP_IN, MLP_IN, MLP_OFF_W1);
    // bias gradients: sums of the deltas over the samples
    for (int u = l; u < MLP_H; u += 64) {
        float s1 = 0.f, s2 = 0.f;
        for (int c = 0; c < 16; ++c) {
            s1 += bf2f(sD1[wv][c * MLP_H + u]);
            s2 += bf2f(sD2[wv][c * MLP_H + u]);
        }
        atomicAdd(&sG[MLP_OFF_B1 + u], s1);
        atomicAdd(&sG[MLP_OFF_B2 + u], s2);
    }
    if (l < MLP_OUT) {
        float s3 = 0.f;
        for (int c = 0; c < 16; ++c) s3 += bf2f(sD3[wv][c * MLP_OUT + l]);
        atomicAdd(&sG[MLP_OFF_B3 + l], s3);
    }
    __syncthreads();
    float* out = part + (int64_t)blockIdx.x * MLP_NPARAM;
    for (int q = threadIdx.x; q < MLP_NPARAM; q += 256) out[q] = sG[q];
}

// Sum of the block partials in block order: dw[q] = sum_b part[b][q].
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* part, int nblk, float* dw) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= MLP_NPARAM) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * MLP_NPARAM + q];
    dw[q] = (float)s;
}

// Adam on the FP32 master weights; refreshes the BF16 copy.
__global__ __launch_bounds__(256) void k_mlp_adam(float* wm, uint16_t* wb, const float* g, float* m, float* v,
                                                  int64_t np, float lr, float b1, float b2, float eps, float bc1,
                                                  float bc2) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= np) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    const float w = wm[q] - lr * (mq / bc1) / (sqrtf(vq / bc2) + eps);
    wm[q] = w;
    wb[q] = f2bf(w);
}

// Mean-squared error on the first nuse outputs: dy = 2 (y - t) / (n nuse); loss partials.
__global__ __launch_bounds__(256) void k_mlp_mse(const float* y, const float* t, int64_t n, int nuse, float* dy,
                                                 double* lpart) {
    __shared__ double lds[5];
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double acc[1] = {0.0};
    if (c < n) {
        for (int o = 0; o < MLP_OUT; ++o) {
            const float d = o < nuse ? y[c * MLP_OUT + o] - t[c * MLP_OUT + o] : 0.f;
            dy[c * MLP_OUT + o] = 2.f * d / (float)(n * nuse);
            acc[0] += (double)d * d;
        }
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) lpart[blockIdx.x] = acc[0];
}

}  // namespace clot
