// learned.hip -- the learned tail compositor's network on gfx950 matrix cores.
//
// A 9 -> 64 -> 64 -> 5 MLP (GELU, tanh form) predicts a pixel's tail
// composite (premultiplied RGBA) and a confidence logit from 9 tail features.
// Inference, loss, backward and the Adam update are hand-written on the
// matrix cores with FP32 accumulation; the master weights and their
// gradients stay FP32.  Products over the 64 hidden units use gfx950's
// v_mfma_f32_16x16x32_bf16, those over 16 (the 9 inputs, the 16 rows of a
// tile) v_mfma_f32_16x16x16_bf16.
//
// All products are written transposed: Z^T (units x rows) = W^T (units x in)
// * X^T (in x rows).  The D tile of an MFMA holds D[4*(l/16)+i][l%16] in
// lane l, i < 4: units 16*mt + 4*(l/16) + i of row l%16.  In the 16x16x16
// form that is exactly the B operand (4 consecutive k per lane) of the next
// layer's k-step mt; in the 16x16x32 form a lane supplies 8 k, and two D
// tiles side by side (mt = 2ks, 2ks + 1) give them without any lane
// exchange, provided the weights' k axis is stored in the same order: k-step
// ks, lane group g, slot j < 4 is unit 32ks + 4g + j and slot 4 + j is unit
// 32ks + 16 + 4g + j (the sum over k does not depend on the order).  So
// forward activations never leave registers.  The weight gradients (sums
// over rows) need the row index as the reduction axis and go through small
// per-wave LDS transposes.
#include "kern.h"

namespace hexfc {

typedef __attribute__((ext_vector_type(4))) short bf4;
typedef __attribute__((ext_vector_type(8))) short bf8;
typedef __attribute__((ext_vector_type(8))) __bf16 bf8v;
typedef __attribute__((ext_vector_type(4))) float f4;

constexpr int NF = 9, NH = 64, NO = 5;
constexpr int P_MU = 0, P_IS = 9, P_W1 = 18, P_B1 = P_W1 + NF * NH, P_W2 = P_B1 + NH, P_B2 = P_W2 + NH * NH,
              P_W3 = P_B2 + NH, P_B3 = P_W3 + NH * NO, P_END = P_B3 + NO;
static_assert(P_END == MLP_PARAMS, "parameter layout");
constexpr float LAMBDA = 0.1f;

__device__ __forceinline__ unsigned short f2bf(float x) {  // round to nearest even
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ f4 mfma(bf4 a, bf4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
__device__ __forceinline__ f4 mfma32(bf8 a, bf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a), __builtin_bit_cast(bf8v, b), c, 0, 0, 0);
}
__device__ __forceinline__ bf4 ld4(const unsigned short *p) { return *reinterpret_cast<const bf4 *>(p); }
__device__ __forceinline__ bf8 ld8(const unsigned short *p) { return *reinterpret_cast<const bf8 *>(p); }
// the B operand of k-step ks over 64 units: D tiles 2ks and 2ks + 1 side by side
__device__ __forceinline__ bf8 cat8(bf4 lo, bf4 hi) { return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7); }
// hidden unit stored at column c of a weight's 64-unit k axis (see the top)
__host__ __device__ constexpr int kunit(int c) {
    return 32 * (c / 32) + ((c % 8) < 4 ? 4 * ((c % 32) / 8) + c % 8 : 16 + 4 * ((c % 32) / 8) + c % 8 - 4);
}
__device__ __forceinline__ bf4 pack4(float a, float b, float c, float d) {
    bf4 r;
    r[0] = (short)f2bf(a);
    r[1] = (short)f2bf(b);
    r[2] = (short)f2bf(c);
    r[3] = (short)f2bf(d);
    return r;
}

constexpr float GC = 0.7978845608028654f;  // sqrt(2/pi)
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.f + tanhf(GC * (x + 0.044715f * x * x * x))); }
__device__ __forceinline__ float gelu_d(float x) {
    const float t = tanhf(GC * (x + 0.044715f * x * x * x));
    return 0.5f * (1.f + t) + 0.5f * x * (1.f - t * t) * GC * (1.f + 3.f * 0.044715f * x * x);
}

// BF16 weights in LDS, each in the layout its MFMA operand reads (4 or 8
// consecutive k values per lane; a 64-unit k axis in kunit order); FP32
// biases and input standardisation.
struct MlpLds {
    unsigned short w1t[NH][16];  // [unit][in]       (in >= 9 zero)
    unsigned short w2t[NH][NH];  // [out unit][in unit, kunit order]
    unsigned short w3t[16][NH];  // [out][unit, kunit order]  (out >= 5 zero)
    unsigned short w3[NH][16];   // [unit][out]
    unsigned short w2[NH][NH];   // [in unit][out unit, kunit order]
    float b1[NH], b2[NH], b3[16], mu[16], is[16];
};

template <bool BWD>
__device__ void mlp_load(MlpLds &L, const float *__restrict__ p) {
    for (int i = threadIdx.x; i < NH * 16; i += blockDim.x) {
        const int u = i / 16, k = i % 16;
        L.w1t[u][k] = k < NF ? f2bf(p[P_W1 + k * NH + u]) : 0;
        if (BWD) L.w3[u][k] = k < NO ? f2bf(p[P_W3 + u * NO + k]) : 0;
        const int o = i / NH, c = i % NH;
        L.w3t[o][c] = o < NO ? f2bf(p[P_W3 + kunit(c) * NO + o]) : 0;
    }
    for (int i = threadIdx.x; i < NH * NH; i += blockDim.x) {
        const int a = i / NH, c = i % NH;
        L.w2t[a][c] = f2bf(p[P_W2 + kunit(c) * NH + a]);
        if (BWD) L.w2[a][c] = f2bf(p[P_W2 + a * NH + kunit(c)]);
    }
    for (int i = threadIdx.x; i < NH; i += blockDim.x) {
        L.b1[i] = p[P_B1 + i];
        L.b2[i] = p[P_B2 + i];
    }
    for (int i = threadIdx.x; i < 16; i += blockDim.x) {
        L.b3[i] = i < NO ? p[P_B3 + i] : 0.f;
        L.mu[i] = i < NF ? p[P_MU + i] : 0.f;
        L.is[i] = i < NF ? p[P_IS + i] : 0.f;
    }
}

// Standardised inputs of row `row` as the layer-1 B operand (features 4q..4q+3).
__device__ __forceinline__ bf4 input_operand(const MlpLds &L, const float *__restrict__ X, int64_t row, bool valid,
                                             int q, float (&xs)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = 4 * q + i;
        xs[i] = (valid && k < NF) ? (X[row * NF + k] - L.mu[k]) * L.is[k] : 0.f;
    }
    return pack4(xs[0], xs[1], xs[2], xs[3]);
}

struct Fwd {
    f4 z1[4], z2[4], y;
};

// Forward of one 16-row tile (4 + 8 + 2 MFMAs).  Lane l: row l%16; z1/z2
// hold units 16*mt + 4*(l/16) + i, y holds outputs 4*(l/16) + i.
__device__ __forceinline__ void mlp_fwd16(const MlpLds &L, bf4 xb, Fwd &f) {
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const f4 zero = {0.f, 0.f, 0.f, 0.f};
    bf4 hb[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f4 z = mfma(ld4(&L.w1t[16 * mt + r][4 * q]), xb, zero);
#pragma unroll
        for (int i = 0; i < 4; ++i) z[i] += L.b1[16 * mt + 4 * q + i];
        f.z1[mt] = z;
        hb[mt] = pack4(gelu(z[0]), gelu(z[1]), gelu(z[2]), gelu(z[3]));
    }
    bf4 hb2[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f4 z = zero;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
            z = mfma32(ld8(&L.w2t[16 * mt + r][32 * ks + 8 * q]), cat8(hb[2 * ks], hb[2 * ks + 1]), z);
#pragma unroll
        for (int i = 0; i < 4; ++i) z[i] += L.b2[16 * mt + 4 * q + i];
        f.z2[mt] = z;
        hb2[mt] = pack4(gelu(z[0]), gelu(z[1]), gelu(z[2]), gelu(z[3]));
    }
    f4 y = zero;
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) y = mfma32(ld8(&L.w3t[r][32 * ks + 8 * q]), cat8(hb2[2 * ks], hb2[2 * ks + 1]), y);
#pragma unroll
    for (int i = 0; i < 4; ++i) y[i] += L.b3[4 * q + i];
    f.y = y;
}

// ------------------------------------------------------------------ forward (outputs only)
__global__ void __launch_bounds__(256) k_mlp_forward(const float *__restrict__ params, const float *__restrict__ X,
                                                     int64_t n, float *__restrict__ Y) {
    __shared__ MlpLds L;
    mlp_load<false>(L, params);
    __syncthreads();
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t t = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); t * 16 < n; t += waves) {
        const int64_t row = t * 16 + r;
        float xs[4];
        const bf4 xb = input_operand(L, X, row, row < n, q, xs);
        Fwd f;
        mlp_fwd16(L, xb, f);
        if (row < n) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (4 * q + i < NO) Y[row * NO + 4 * q + i] = f.y[i];
        }
    }
}

// ------------------------------------------------------------------ loss
__global__ void __launch_bounds__(256) k_mlp_loss(const float *__restrict__ Y, const float *__restrict__ T, int64_t n,
                                                  float conf_tol, float *__restrict__ dY,
                                                  float *__restrict__ loss_sum) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (i < n) {
        const float inv_n = 1.f / (float)n;
        float e[4], emax = 0.f, se = 0.f;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            e[c] = Y[i * NO + c] - T[i * 4 + c];
            emax = fmaxf(emax, fabsf(e[c]));
            se += e[c] * e[c];
            dY[i * NO + c] = 0.5f * e[c] * inv_n;
        }
        const float label = emax < conf_tol ? 1.f : 0.f;
        const float yc = Y[i * NO + 4];
        const float s = 1.f / (1.f + expf(-yc));
        // BCE with logits, stable form: max(y,0) - y*label + log(1 + exp(-|y|))
        const float bce = fmaxf(yc, 0.f) - yc * label + log1pf(expf(-fabsf(yc)));
        dY[i * NO + 4] = LAMBDA * (s - label) * inv_n;
        l = 0.25f * se + LAMBDA * bce;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o);
    if ((threadIdx.x & 63) == 0 && l != 0.f) atomicAdd(loss_sum, l);
}

// ------------------------------------------------------------------ backward
// Per wave: 16-row tiles; forward recomputed, then dZ3 -> dW3, db3, dH2 ->
// dZ2 -> dW2, db2, dH1 -> dZ1 -> dW1, db1.  Weight-gradient accumulators
// live in registers for the wave's whole row range and are added to the
// FP32 gradient with atomics at the end.
struct BwdLds {
    unsigned short t3[16][16];   // dZ3^T [out][row]
    unsigned short h2[NH][16];   // H2^T  [unit][row]
    unsigned short d2[NH][16];   // dZ2^T [unit][row]
    unsigned short h1[NH][16];   // H1^T  [unit][row]
    unsigned short d1[NH][16];   // dZ1^T [unit][row]
    unsigned short xs[16][16];   // Xs^T  [in][row]
};

__global__ void __launch_bounds__(64) k_mlp_backward(const float *__restrict__ params, const float *__restrict__ X,
                                                     const float *__restrict__ dY, int64_t n,
                                                     float *__restrict__ grad) {
    __shared__ MlpLds L;
    __shared__ BwdLds B;
    mlp_load<true>(L, params);
    __syncthreads();
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const f4 zero = {0.f, 0.f, 0.f, 0.f};
    f4 gw3[4], gw2[4][4], gw1[4];
    float gb1[4][4], gb2[4][4], gb3[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gw3[a] = zero;
        gw1[a] = zero;
        gb3[a] = 0.f;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            gw2[a][b] = zero;
            gb1[a][b] = 0.f;
            gb2[a][b] = 0.f;
        }
    }
    for (int64_t t = blockIdx.x; t * 16 < n; t += gridDim.x) {
        const int64_t row = t * 16 + r;
        const bool valid = row < n;
        float xs[4];
        const bf4 xb = input_operand(L, X, row, valid, q, xs);
        Fwd f;
        mlp_fwd16(L, xb, f);
        // dZ3^T in the D layout (outputs 4q+i, row r)
        f4 d3;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = 4 * q + i;
            d3[i] = (valid && o < NO) ? dY[row * NO + o] : 0.f;
            gb3[i] += d3[i];
            B.t3[o][r] = f2bf(d3[i]);
            B.xs[o][r] = f2bf(xs[i]);  // (in = 4q + i)
        }
        // H1^T, H2^T (bf16, as used by the forward) to LDS
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                B.h1[16 * mt + 4 * q + i][r] = f2bf(gelu(f.z1[mt][i]));
                B.h2[16 * mt + 4 * q + i][r] = f2bf(gelu(f.z2[mt][i]));
            }
        __syncthreads();
        // dW3^T[out][unit] += dZ3^T[out][row] * H2[row][unit]
        const bf4 a3 = ld4(&B.t3[r][4 * q]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) gw3[nt] = mfma(a3, ld4(&B.h2[16 * nt + r][4 * q]), gw3[nt]);
        // dH2^T = W3 * dZ3^T;  dZ2^T = dH2^T * gelu'(Z2^T)
        const bf4 b3 = pack4(d3[0], d3[1], d3[2], d3[3]);
        f4 dz2[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f4 h = mfma(ld4(&L.w3[16 * mt + r][4 * q]), b3, zero);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                h[i] *= gelu_d(f.z2[mt][i]);
                gb2[mt][i] += h[i];
                B.d2[16 * mt + 4 * q + i][r] = f2bf(h[i]);
            }
            dz2[mt] = h;
        }
        __syncthreads();
        // dW2^T[u2][u1] += dZ2^T[u2][row] * H1[row][u1]
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const bf4 a = ld4(&B.d2[16 * mt + r][4 * q]);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) gw2[mt][nt] = mfma(a, ld4(&B.h1[16 * nt + r][4 * q]), gw2[mt][nt]);
        }
        // dH1^T = W2 * dZ2^T;  dZ1^T = dH1^T * gelu'(Z1^T)
        bf4 bz2[4];
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) bz2[ks] = pack4(dz2[ks][0], dz2[ks][1], dz2[ks][2], dz2[ks][3]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f4 h = zero;
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
                h = mfma32(ld8(&L.w2[16 * mt + r][32 * ks + 8 * q]), cat8(bz2[2 * ks], bz2[2 * ks + 1]), h);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                h[i] *= gelu_d(f.z1[mt][i]);
                gb1[mt][i] += h[i];
                B.d1[16 * mt + 4 * q + i][r] = f2bf(h[i]);
            }
        }
        __syncthreads();
        // dW1^T[unit][in] += dZ1^T[unit][row] * Xs[row][in]
        const bf4 bx = ld4(&B.xs[r][4 * q]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) gw1[mt] = mfma(ld4(&B.d1[16 * mt + r][4 * q]), bx, gw1[mt]);
        __syncthreads();
    }
    // bias sums: reduce over the 16 rows (lanes with equal q)
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            gb3[i] += __shfl_xor(gb3[i], o);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                gb1[mt][i] += __shfl_xor(gb1[mt][i], o);
                gb2[mt][i] += __shfl_xor(gb2[mt][i], o);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (r == 0) {
            if (4 * q + i < NO) atomicAdd(&grad[P_B3 + 4 * q + i], gb3[i]);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                atomicAdd(&grad[P_B1 + 16 * mt + 4 * q + i], gb1[mt][i]);
                atomicAdd(&grad[P_B2 + 16 * mt + 4 * q + i], gb2[mt][i]);
            }
        }
        // weight tiles in the D layout: row index 4q+i of the tile, column r
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int o = 4 * q + i, u = 16 * nt + r;
            if (o < NO) atomicAdd(&grad[P_W3 + u * NO + o], gw3[nt][i]);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)  // dW2^T[u2 = 16mt+4q+i][u1 = 16nt+r]
                atomicAdd(&grad[P_W2 + u * NH + 16 * mt + 4 * q + i], gw2[mt][nt][i]);
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)  // dW1^T[unit = 16mt+4q+i][in = r]
            if (r < NF) atomicAdd(&grad[P_W1 + r * NH + 16 * mt + 4 * q + i], gw1[mt][i]);
    }
}

// ------------------------------------------------------------------ Adam (FP32 master weights)
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v, const float *__restrict__ g,
                       int count, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count || i < P_W1) return;  // the input standardisation is not trained
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------------ inference in the learned resolve
// Row j: pixel pix[j] (global tile-major id; PIX_SKIP for a row the head
// already resolved) with head composite head[j] and features feat[j].  The
// network's tail is composed under the head when the list is longer than K
// and the pixel confidence 1 - (1 - A_head) (1 - sigmoid(y_4)) reaches
// conf_min; else the pixel is appended to the fallback list of its length
// class c, fb[fb_base.b[c] + i] with i counted in stats[ST_FB + c] (at most
// the class's row count), for the exact resolve.  mask (nullable, preset to
// 1 = exact) gets 0 where the learned tail was used.
__global__ void __launch_bounds__(256) k_mlp_apply(const float *__restrict__ params, const float *__restrict__ feat,
                                                   const float *__restrict__ head, const uint32_t *__restrict__ pix,
                                                   int64_t n, ResolveArgs a, int t_sort, int K, float conf_min,
                                                   uint32_t *__restrict__ fb, FallbackBase fb_base,
                                                   uint64_t *__restrict__ stats, uint8_t *__restrict__ mask) {
    __shared__ MlpLds L;
    mlp_load<false>(L, params);
    __syncthreads();
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t below = (1ull << lane) - 1;  // lanes under this one
    for (int64_t t = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); t * 16 < n; t += waves) {
        const int64_t row = t * 16 + r;
        const bool valid = row < n;
        float xs[4];
        const bf4 xb = input_operand(L, feat, row, valid, q, xs);
        Fwd f;
        mlp_fwd16(L, xb, f);
        const float logit = __shfl(f.y[0], 16 + r);  // output 4 of row r lives in lane 16 + r
        // lanes 0..15 own the 16 rows of the tile
        uint32_t p = PIX_SKIP, cnt = 0;
        float4 h = make_float4(0.f, 0.f, 0.f, 0.f);
        if (q == 0 && valid) p = pix[row];
        const bool active = p != PIX_SKIP;
        if (active) {
            cnt = a.count[p];
            h = reinterpret_cast<const float4 *>(head)[row];
        }
        // pixel confidence: the tail is either predicted well (network
        // confidence) or hidden behind the head
        const float conf = 1.f - (1.f - h.w) * (1.f - 1.f / (1.f + __expf(-logit)));
        // exact resolve for lists of at most K fragments and low (or NaN) confidence
        const bool fallback = active && (cnt <= (uint32_t)K || !(conf >= conf_min));
        const int c = fallback ? length_class(cnt, t_sort) : -1;
#pragma unroll
        for (int cc = 1; cc < NCLASS - 1; ++cc) {
            const uint64_t b = __ballot(c == cc);
            if (!b) continue;
            const int leader = __builtin_ctzll(b);
            uint64_t at = 0;
            if (lane == leader) at = atomicAdd((unsigned long long *)&stats[ST_FB + cc], (unsigned long long)__popcll(b));
            at = __shfl(at, leader);
            if (c == cc) fb[fb_base.b[cc] + at + __popcll(b & below)] = p;
        }
        if (!active || fallback) continue;
        const PixelRef pr = pixel_ref(a.tl, p);
        const int64_t o = (pr.view * a.tl.H + pr.y) * (int64_t)a.tl.W + pr.x;
        const float4 tail = make_float4(fminf(fmaxf(f.y[0], 0.f), 1.f), fminf(fmaxf(f.y[1], 0.f), 1.f),
                                        fminf(fmaxf(f.y[2], 0.f), 1.f), fminf(fmaxf(f.y[3], 0.f), 1.f));
        if (mask) mask[o] = 0;
        const float T = 1.f - h.w;
        const float C0 = h.x + T * tail.x, C1 = h.y + T * tail.y, C2 = h.z + T * tail.z, A = h.w + T * tail.w;
        const float Tb = 1.f - A;
        const ShadeParams &sp = view_params(a.views, pr.view).sp;
        reinterpret_cast<float4 *>(a.rgba)[o] =
            make_float4(C0 + Tb * sp.bg[0], C1 + Tb * sp.bg[1], C2 + Tb * sp.bg[2], A);
    }
}

__global__ void k_fill_u8(uint8_t *__restrict__ p, int64_t n, uint8_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ launchers
static unsigned grid_for(int64_t tiles16, int waves_per_block) {
    int64_t b = (tiles16 + waves_per_block - 1) / waves_per_block;
    return (unsigned)std::min<int64_t>(std::max<int64_t>(b, 1), 1024);
}

void launch_mlp_forward(const float *params, const float *X, int64_t n, float *Y, hipStream_t s) {
    if (n <= 0) return;
    k_mlp_forward<<<grid_for((n + 15) / 16, 4), 256, 0, s>>>(params, X, n, Y);
}
void launch_mlp_loss(const float *Y, const float *T, int64_t n, float conf_tol, float *dY, float *loss_sum,
                     hipStream_t s) {
    if (n <= 0) return;
    k_mlp_loss<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(Y, T, n, conf_tol, dY, loss_sum);
}
void launch_mlp_backward(const float *params, const float *X, const float *dY, int64_t n, float *grad,
                         hipStream_t s) {
    if (n <= 0) return;
    k_mlp_backward<<<grid_for((n + 15) / 16, 1), 64, 0, s>>>(params, X, dY, n, grad);
}
void launch_adam(float *w, float *m, float *v, const float *g, int count, float lr, float b1, float b2, float eps,
                 int step, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    k_adam<<<(count + 255) / 256, 256, 0, s>>>(w, m, v, g, count, lr, b1, b2, eps, c1, c2);
}
void launch_mlp_apply(const float *params, const float *feat, const float *head, const uint32_t *pix, int64_t n,
                      const ResolveArgs &a, int t_sort, int K, float conf_min, uint32_t *fb,
                      const FallbackBase &fb_base, uint64_t *stats, uint8_t *mask, hipStream_t s) {
    if (n <= 0) return;
    k_mlp_apply<<<grid_for((n + 15) / 16, 4), 256, 0, s>>>(params, feat, head, pix, n, a, t_sort, K, conf_min, fb,
                                                            fb_base, stats, mask);
}
void launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s) {
    if (n <= 0) return;
    k_fill_u8<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n, v);
}

}  // namespace hexfc

// ------------------------------------------------------------------ C ABI (context-free)
#include "../../include/hexfc.h"

namespace {
hexfc_status launched() { return hipGetLastError() == hipSuccess ? HEXFC_OK : HEXFC_EDEVICE; }
}  // namespace

extern "C" {

int64_t hexfc_mlp_param_count(void) { return hexfc::MLP_PARAMS; }

hexfc_status hexfc_mlp_forward(const float *params, const float *x, int64_t n, float *y, void *stream) {
    if (n < 0 || (n > 0 && (!params || !x || !y))) return HEXFC_EINVAL;
    hexfc::launch_mlp_forward(params, x, n, y, (hipStream_t)stream);
    return launched();
}

hexfc_status hexfc_mlp_loss(const float *y, const float *target, int64_t n, float conf_tol, float *dy,
                            float *loss_sum, void *stream) {
    if (n < 0 || (n > 0 && (!y || !target || !dy || !loss_sum))) return HEXFC_EINVAL;
    if (!(conf_tol > 0.f)) return HEXFC_ERANGE;
    hexfc::launch_mlp_loss(y, target, n, conf_tol, dy, loss_sum, (hipStream_t)stream);
    return launched();
}

hexfc_status hexfc_mlp_backward(const float *params, const float *x, const float *dy, int64_t n, float *grad,
                                void *stream) {
    if (n < 0 || (n > 0 && (!params || !x || !dy || !grad))) return HEXFC_EINVAL;
    hexfc::launch_mlp_backward(params, x, dy, n, grad, (hipStream_t)stream);
    return launched();
}

hexfc_status hexfc_mlp_adam_step(float *params, float *m, float *v, const float *grad, float lr, float beta1,
                                 float beta2, float eps, int step, void *stream) {
    if (!params || !m || !v || !grad) return HEXFC_EINVAL;
    if (step < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return HEXFC_ERANGE;
    hexfc::launch_adam(params, m, v, grad, hexfc::MLP_PARAMS, lr, beta1, beta2, eps, step, (hipStream_t)stream);
    return launched();
}

}  // extern "C"
