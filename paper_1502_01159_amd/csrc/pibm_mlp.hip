// pibm_mlp.hip -- the learned per-particle closure: a 16 -> 128 -> 128 -> 128
// -> 4 multilayer perceptron with GELU (erf form) hidden units, evaluated and
// trained on gfx950 matrix cores.
//
// Arithmetic: BF16 operands on v_mfma_f32_16x16x16_bf16 with FP32
// accumulation; FP32 master weights, biases, pre-activations and Adam state.
// Quantisation points (what a mirror of this arithmetic must round to BF16):
// the inputs (given as BF16), every weight, every hidden activation fed to the
// next layer, the output gradient dL/dy and every pre-activation gradient fed
// to a product.  Bias gradients are sums of those BF16 pre-activation
// gradients; weight gradients are FP32 sums of BF16 x BF16 products.  The
// hidden units' erf is Hastings' rational approximation (|error| <= 1.5e-7);
// the BF16 roundings are the hardware's round-to-nearest-even conversion.
//
// Layout.  Every layer is computed transposed, Y^T = W^T X^T, with 16 samples
// along the product's N dimension: the 16x16 result tile of one product (lane
// i holds rows 4(i/16) .. 4(i/16)+3 of column i%16) is then exactly the B
// operand of the next layer (lane i holds K rows 4(i/16) .. +3 of column
// i%16), so activations pass from layer to layer in registers.  Weights live
// in LDS as BF16 W^T (rows = output units, padded by 8 elements against bank
// conflicts), 80 KB for the whole network.
//
// Training: one workgroup per 64 samples computes the forward pass, the
// backward pass and its partial weight gradients (products with K = the 64
// samples, from BF16 activations and pre-activation gradients staged in LDS)
// and writes them to its own slot; a second kernel sums the slots in a fixed
// order and applies Adam.  Results are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/pibm.h"
#include "pibm_internal.h"

namespace {

constexpr int NI = PIBM_MLP_IN, NH = PIBM_MLP_HIDDEN, NO = PIBM_MLP_OUT, NOP = 16;
constexpr int NPARAM = PIBM_MLP_NPARAM;
// canonical parameter order: W1[in][out], b1, W2, b2, W3, b3, W4, b4
constexpr int OW1 = 0, OB1 = OW1 + NI * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH * NH, OW4 = OB3 + NH, OB4 = OW4 + NH * NO;
static_assert(OB4 + NO == NPARAM, "parameter count");
// BF16 W^T copies in LDS: row stride (elements) and offsets
constexpr int P1 = NI + 8, PH = NH + 8;
constexpr int BW1 = 0, BW2 = BW1 + NH * P1, BW3 = BW2 + NH * PH, BW4 = BW3 + NH * PH, NBF = BW4 + NOP * PH;
constexpr int NBIAS = 3 * NH + NO;
constexpr int MLP_THREADS = 256;
constexpr int SPB = 64;                 // training samples per workgroup (4 waves x 16)
constexpr int PS = SPB + 8;             // row stride of the LDS activation / gradient stages

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__host__ __device__ inline uint16_t bf16_rne(float f)
{
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// erf(x) by Hastings' rational approximation (Abramowitz & Stegun 7.1.26):
// erf(x) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2) with
// t = 1 / (1 + p |x|), odd in x, |error| <= 1.5e-7 -- far below the BF16
// rounding of the activations.  Branch-free (one reciprocal, one
// exponential), unlike a library erff whose range split diverges across a
// wave.  Also returns exp(-x^2).
__device__ __forceinline__ float erf_hastings(float x, float &ex2)
{
    constexpr float p = 0.3275911f, a1 = 0.254829592f, a2 = -0.284496736f, a3 = 1.421413741f, a4 = -1.453152027f,
                    a5 = 1.061405429f;
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(p, ax, 1.0f));
    const float poly = t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, a5, a4), a3), a2), a1);
    ex2 = __expf(-ax * ax);
    return copysignf(fmaf(-poly, ex2, 1.0f), x);
}
// GELU(z) = z Phi(z), Phi(z) = (1 + erf(z / sqrt 2)) / 2; GELU'(z) = Phi(z) + z phi(z)
__device__ __forceinline__ float gelu(float z)
{
    float e;
    return 0.5f * z * (1.0f + erf_hastings(z * 0.70710678118654752f, e));
}
__device__ __forceinline__ float gelu_d(float z)
{
    float e;
    const float Phi = 0.5f * (1.0f + erf_hastings(z * 0.70710678118654752f, e));
    return Phi + z * 0.39894228040143268f * e;
}

__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef short v8s __attribute__((ext_vector_type(8)));
// Two consecutive K = 16 products in one K = 32 product: lane group g holds
// K positions 8g .. 8g + 7, here the first operands' 4g .. 4g + 3 followed by
// the second's.  A and B share that order, so the result is a0 b0 + a1 b1.
__device__ __forceinline__ v4f mfma2(v4s a0, v4s a1, v4s b0, v4s b1, v4f c)
{
    const v8s a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
    const v8s b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}
__device__ __forceinline__ v4s lds4(const uint16_t *p) { return *(const v4s *)p; }
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
// four floats to BF16, round to nearest even (the hardware pack conversion)
__device__ __forceinline__ v4s pack4(float a, float b, float c, float d)
{
    const v2bf lo = __builtin_convertvector((v2f){a, b}, v2bf), hi = __builtin_convertvector((v2f){c, d}, v2bf);
    v4s r;
    uint32_t u0, u1;
    memcpy(&u0, &lo, 4);
    memcpy(&u1, &hi, 4);
    r[0] = (short)(u0 & 0xffffu); r[1] = (short)(u0 >> 16); r[2] = (short)(u1 & 0xffffu); r[3] = (short)(u1 >> 16);
    return r;
}

struct MlpArgs {
    const float *param;         // FP32 masters, canonical order (biases are read from here)
    const uint16_t *wbf;        // BF16 W^T copies, LDS layout
};

__device__ void stage_weights(const MlpArgs &a, uint16_t *w, float *bias)
{
    const uint4 *src = (const uint4 *)a.wbf;
    uint4 *dst = (uint4 *)w;
    for (int i = threadIdx.x; i < NBF / 8; i += blockDim.x) dst[i] = src[i];
    for (int i = threadIdx.x; i < NBIAS; i += blockDim.x) {
        const int o = i < NH ? OB1 + i : (i < 2 * NH ? OB2 + i - NH : (i < 3 * NH ? OB3 + i - 2 * NH : OB4 + i - 3 * NH));
        bias[i] = a.param[o];
    }
}

// One hidden layer forward for a wave's 16 samples: in[t] holds K tile t of
// the input (as B operands), out[m] the 8 result tiles (pre-activations).
template <int KT>
__device__ __forceinline__ void layer_fwd(const uint16_t *w, int stride, const v4s *in, v4f *z, int l16, int g)
{
#pragma unroll
    for (int m = 0; m < NH / 16; ++m) {
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        const uint16_t *wr = w + (16 * m + l16) * stride + 4 * g;
        if (KT % 2 == 0) {
#pragma unroll
            for (int t = 0; t < KT; t += 2) acc = mfma2(lds4(wr + 16 * t), lds4(wr + 16 * t + 16), in[t], in[t + 1], acc);
        } else {
#pragma unroll
            for (int t = 0; t < KT; ++t) acc = mfma(lds4(wr + 16 * t), in[t], acc);
        }
        z[m] = acc;
    }
}

// ---------------------------------------------------------------------------
// Inference: y[n][4] (FP32) from x[n][16] (BF16 bits), grid-stride over
// tiles of 16 samples, one tile per wave at a time.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(MLP_THREADS) void k_mlp_fwd(MlpArgs a, const uint16_t *x, float *y, int n)
{
    __shared__ __align__(16) uint16_t w[NBF];
    __shared__ float bias[NBIAS];
    stage_weights(a, w, bias);
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
    const int ntile = (n + 15) / 16;
    for (int tile = blockIdx.x * (MLP_THREADS / 64) + wv; tile < ntile; tile += gridDim.x * (MLP_THREADS / 64)) {
        // keeps the weights' LDS reads inside the loop: hoisted, they would hold
        // ~290 registers and allow one wave per SIMD; read per tile, two waves
        // per SIMD overlap one's GELUs with the other's matrix products
        asm volatile("" ::: "memory");
        const int s = tile * 16 + l16;
        v4s xb = {0, 0, 0, 0};
        if (s < n) xb = *(const v4s *)(x + (size_t)s * NI + 4 * g);
        v4f z[NH / 16];
        v4s h[NH / 16];
        layer_fwd<1>(w + BW1, P1, &xb, z, l16, g);
#pragma unroll
        for (int L = 0; L < 3; ++L) {
            const float *b = bias + L * NH;
#pragma unroll
            for (int m = 0; m < NH / 16; ++m) {
                float v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] = gelu(z[m][j] + b[16 * m + 4 * g + j]);
                h[m] = pack4(v[0], v[1], v[2], v[3]);
            }
            if (L < 2) layer_fwd<NH / 16>(w + (L == 0 ? BW2 : BW3), PH, h, z, l16, g);
        }
        v4f o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < NH / 16; t += 2)
            o = mfma2(lds4(w + BW4 + l16 * PH + 16 * t + 4 * g), lds4(w + BW4 + l16 * PH + 16 * t + 16 + 4 * g), h[t], h[t + 1], o);
        if (g == 0 && s < n) {
            float4 r;
            r.x = o[0] + bias[3 * NH + 0]; r.y = o[1] + bias[3 * NH + 1];
            r.z = o[2] + bias[3 * NH + 2]; r.w = o[3] + bias[3 * NH + 3];
            *(float4 *)(y + (size_t)s * NO) = r;
        }
    }
}

// ---------------------------------------------------------------------------
// Training pass over samples [64 b, 64 b + 64) of a batch of n: loss
// L = sum (y - t)^2 / (4 n) over the batch; writes this workgroup's partial
// dL/dparam (canonical order) and partial sum of squared errors.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(MLP_THREADS) void k_mlp_grad(MlpArgs a, const uint16_t *x, const float *tg, int n,
                                                         float *part, double *loss_part)
{
    __shared__ __align__(16) uint16_t w[NBF];
    __shared__ float bias[NBIAS];
    __shared__ __align__(16) uint16_t ht[NI * PS + 3 * NH * PS];   // activations, [unit][sample]
    __shared__ __align__(16) uint16_t dzt[NH * PS];                // pre-activation gradients, [unit][sample]
    __shared__ __align__(16) uint16_t dyt[NOP * PS];               // output gradient, [output][sample]
    __shared__ double red[MLP_THREADS / 64];
    stage_weights(a, w, bias);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, l16 = lane & 15, g = lane >> 4;
    const int col = 16 * wv + l16;                   // this lane's sample within the workgroup
    const int s = blockIdx.x * SPB + col;
    const bool ok = s < n;
    float *pw = part + (size_t)blockIdx.x * NPARAM;
    // input stage [16 units][64 samples]
    v4s xb = {0, 0, 0, 0};
    if (ok) xb = *(const v4s *)(x + (size_t)s * NI + 4 * g);
#pragma unroll
    for (int j = 0; j < 4; ++j) ht[(4 * g + j) * PS + col] = (uint16_t)xb[j];
    __syncthreads();

    // forward, keeping GELU'(z) per hidden layer
    v4f gp[3][NH / 16];
    v4s h[NH / 16];
    v4f z[NH / 16];
    layer_fwd<1>(w + BW1, P1, &xb, z, l16, g);
#pragma unroll
    for (int L = 0; L < 3; ++L) {
        const float *b = bias + L * NH;
        uint16_t *hs = ht + NI * PS + L * NH * PS;
#pragma unroll
        for (int m = 0; m < NH / 16; ++m) {
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float zz = z[m][j] + b[16 * m + 4 * g + j];
                v[j] = gelu(zz);
                gp[L][m][j] = gelu_d(zz);
            }
            h[m] = pack4(v[0], v[1], v[2], v[3]);
#pragma unroll
            for (int j = 0; j < 4; ++j) hs[(16 * m + 4 * g + j) * PS + col] = (uint16_t)h[m][j];
        }
        if (L < 2) layer_fwd<NH / 16>(w + (L == 0 ? BW2 : BW3), PH, h, z, l16, g);
    }
    v4f o = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < NH / 16; t += 2)
        o = mfma2(lds4(w + BW4 + l16 * PH + 16 * t + 4 * g), lds4(w + BW4 + l16 * PH + 16 * t + 16 + 4 * g), h[t], h[t + 1], o);
    // output gradient dL/dy = (y - t) / (2 n), zero for padding samples and rows
    double se = 0.0;
    float dy[4] = {0.f, 0.f, 0.f, 0.f};
    if (g == 0 && ok) {
        const float4 tv = *(const float4 *)(tg + (size_t)s * NO);
        const float t4[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float e = o[j] + bias[3 * NH + j] - t4[j];
            se += (double)e * (double)e;
            dy[j] = e * (0.5f / (float)n);
        }
    }
    v4s dyb = pack4(dy[0], dy[1], dy[2], dy[3]);
#pragma unroll
    for (int j = 0; j < 4; ++j) dyt[(4 * g + j) * PS + col] = (uint16_t)dyb[j];
    // squared error of this workgroup, in a fixed order
#pragma unroll
    for (int off = 32; off; off >>= 1) se += __shfl_xor(se, off);
    if (lane == 0) red[wv] = se;

    // backward through layer 4: dh3 = W4 dy (A operand: W4 as [hidden][output])
    v4f dh[NH / 16];
#pragma unroll
    for (int m = 0; m < NH / 16; ++m) {
        v4s A;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) A[kk] = (short)w[BW4 + (4 * g + kk) * PH + 16 * m + l16];
        const v4f zero = {0.f, 0.f, 0.f, 0.f};
        dh[m] = mfma(A, dyb, zero);
    }
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);

    // weight gradient of one layer: dW[in][out] = sum_s H[in][s] dZ[out][s]
    auto wgrad = [&](const uint16_t *hs, int nin, const uint16_t *dz, int nout, int nout_real, int ow, int ob) {
        const int ntm = nin / 16, ntn = (nout + 15) / 16;
        for (int tt = wv; tt < ntm * ntn; tt += MLP_THREADS / 64) {
            const int ta = tt / ntn, tb = tt % ntn;
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            const uint16_t *ha = hs + (16 * ta + l16) * PS + 4 * g, *db = dz + (16 * tb + l16) * PS + 4 * g;
#pragma unroll
            for (int k = 0; k < SPB / 16; k += 2)
                acc = mfma2(lds4(ha + 16 * k), lds4(ha + 16 * k + 16), lds4(db + 16 * k), lds4(db + 16 * k + 16), acc);
            const int out = 16 * tb + l16;
            if (out < nout_real) {
#pragma unroll
                for (int j = 0; j < 4; ++j) pw[ow + (16 * ta + 4 * g + j) * nout_real + out] = acc[j];
            }
        }
        for (int u = threadIdx.x; u < nout_real; u += MLP_THREADS) {
            float sb = 0.f;
            for (int c = 0; c < SPB; ++c) sb += bf16_f(dz[u * PS + c]);
            pw[ob + u] = sb;
        }
    };
    wgrad(ht + NI * PS + 2 * NH * PS, NH, dyt, NOP, NO, OW4, OB4);

    // hidden layers 3, 2, 1
#pragma unroll
    for (int L = 2; L >= 0; --L) {
        v4s dzb[NH / 16];
#pragma unroll
        for (int m = 0; m < NH / 16; ++m) {
            float v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = dh[m][j] * gp[L][m][j];
            dzb[m] = pack4(v[0], v[1], v[2], v[3]);
        }
        __syncthreads();                              // dzt free again
#pragma unroll
        for (int m = 0; m < NH / 16; ++m)
#pragma unroll
            for (int j = 0; j < 4; ++j) dzt[(16 * m + 4 * g + j) * PS + col] = (uint16_t)dzb[m][j];
        __syncthreads();
        const uint16_t *hin = L == 0 ? ht : ht + NI * PS + (L - 1) * NH * PS;
        const int nin = L == 0 ? NI : NH;
        const int ow = L == 0 ? OW1 : (L == 1 ? OW2 : OW3), ob = L == 0 ? OB1 : (L == 1 ? OB2 : OB3);
        wgrad(hin, nin, dzt, NH, NH, ow, ob);
        if (L > 0) {
            // dh_{L-1} = W_L dz_L; A operand: W_L as [in][out] read from W_L^T
            const uint16_t *wl = w + (L == 1 ? BW2 : BW3);
#pragma unroll
            for (int m = 0; m < NH / 16; ++m) {
                v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int t = 0; t < NH / 16; t += 2) {
                    v4s A0, A1;
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        A0[kk] = (short)wl[(16 * t + 4 * g + kk) * PH + 16 * m + l16];
                        A1[kk] = (short)wl[(16 * t + 16 + 4 * g + kk) * PH + 16 * m + l16];
                    }
                    acc = mfma2(A0, A1, dzb[t], dzb[t + 1], acc);
                }
                dh[m] = acc;
            }
        }
    }
}

// Sum the per-workgroup partial gradients in a fixed order; either return
// them (grad != NULL) or take one Adam step (Kingma & Ba) on the masters and
// refresh the BF16 copies.
__global__ void k_mlp_reduce_adam(float *param, uint16_t *wbf, float *mom, float *vel, const float *part, int nblk,
                                  float *grad, float lr, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    float gsum = 0.f;
    for (int b = 0; b < nblk; ++b) gsum += part[(size_t)b * NPARAM + p];
    if (grad) { grad[p] = gsum; return; }
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float m = b1 * mom[p] + (1.f - b1) * gsum;
    const float v = b2 * vel[p] + (1.f - b2) * gsum * gsum;
    mom[p] = m;
    vel[p] = v;
    const float np = param[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    param[p] = np;
    // BF16 copy of a weight in the W^T LDS layout
    int base = -1, in = 0, out = 0, nout = 0, stride = 0;
    if (p < OB1) { base = BW1; nout = NH; stride = P1; in = (p - OW1) / nout; out = (p - OW1) % nout; }
    else if (p >= OW2 && p < OB2) { base = BW2; nout = NH; stride = PH; in = (p - OW2) / nout; out = (p - OW2) % nout; }
    else if (p >= OW3 && p < OB3) { base = BW3; nout = NH; stride = PH; in = (p - OW3) / nout; out = (p - OW3) % nout; }
    else if (p >= OW4 && p < OB4) { base = BW4; nout = NO; stride = PH; in = (p - OW4) / nout; out = (p - OW4) % nout; }
    if (base >= 0) wbf[base + out * stride + in] = bf16_rne(np);
}

// Scratch of the allocation-free gradient pass: the partial gradients of up
// to PIBM_MLP_NOALLOC_MAX_BATCH / 64 workgroups, their sum and the
// workgroups' loss partials.  One copy per GPU, held until the process ends.
// Host code never uses the array's name as an address: each device's address
// comes from hipGetSymbolAddress (scratch_on below).
constexpr int NOALLOC_BLK = PIBM_MLP_NOALLOC_MAX_BATCH / SPB;
static_assert(NOALLOC_BLK * SPB == PIBM_MLP_NOALLOC_MAX_BATCH, "whole workgroups");
constexpr size_t SCR_PART = 0;
constexpr size_t SCR_GRAD = SCR_PART + ((size_t)NOALLOC_BLK * NPARAM * 4 + 255) / 256 * 256;
constexpr size_t SCR_LOSS = SCR_GRAD + ((size_t)NPARAM * 4 + 255) / 256 * 256;
constexpr size_t SCR_BYTES = SCR_LOSS + (size_t)NOALLOC_BLK * 8;
static __device__ __align__(256) unsigned char scratch[SCR_BYTES];

// splitmix64 (Steele, Lea & Flood): state += 0x9e3779b97f4a7c15, then the
// variant-13 finaliser; 53-bit uniforms in [0, 1)
struct SplitMix {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

}  // namespace

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct pibm_mlp {
    hipStream_t stream;
    int max_batch, max_blk;
    long long step;
    float *param, *mom, *vel, *part, *grad;
    double *loss_part;
    uint16_t *wbf;
};

namespace {

struct MlpPlan {
    size_t off[7];
    size_t total;
};
MlpPlan mlp_plan(int max_batch)
{
    MlpPlan P{};
    const int nblk = (max_batch + SPB - 1) / SPB;
    const size_t sz[7] = {(size_t)NPARAM * 4, (size_t)NPARAM * 4, (size_t)NPARAM * 4, (size_t)NBF * 2,
                          (size_t)nblk * NPARAM * 4, (size_t)NPARAM * 4, (size_t)nblk * 8};
    size_t o = 0;
    for (int i = 0; i < 7; ++i) {
        P.off[i] = o;
        o += (sz[i] + 255) / 256 * 256;
    }
    P.total = o;
    return P;
}

// BF16 W^T image of canonical parameters
void build_wbf(const float *prm, std::vector<uint16_t> &wb)
{
    wb.assign(NBF, 0);
    for (int i = 0; i < NI; ++i)
        for (int o = 0; o < NH; ++o) wb[BW1 + o * P1 + i] = bf16_rne(prm[OW1 + i * NH + o]);
    for (int i = 0; i < NH; ++i)
        for (int o = 0; o < NH; ++o) {
            wb[BW2 + o * PH + i] = bf16_rne(prm[OW2 + i * NH + o]);
            wb[BW3 + o * PH + i] = bf16_rne(prm[OW3 + i * NH + o]);
        }
    for (int i = 0; i < NH; ++i)
        for (int o = 0; o < NO; ++o) wb[BW4 + o * PH + i] = bf16_rne(prm[OW4 + i * NO + o]);
}

int mlp_upload(pibm_mlp *m, const float *prm)
{
    std::vector<uint16_t> wb;
    build_wbf(prm, wb);
    if (hipMemcpyAsync(m->param, prm, (size_t)NPARAM * 4, hipMemcpyHostToDevice, m->stream) != hipSuccess) return PIBM_EDEVICE;
    if (hipMemcpyAsync(m->wbf, wb.data(), (size_t)NBF * 2, hipMemcpyHostToDevice, m->stream) != hipSuccess) return PIBM_EDEVICE;
    // optimizer state restarts with new parameters (fill kernels, not memsets)
    std::vector<float> zero((size_t)NPARAM, 0.f);
    if (hipMemcpyAsync(m->mom, zero.data(), (size_t)NPARAM * 4, hipMemcpyHostToDevice, m->stream) != hipSuccess) return PIBM_EDEVICE;
    if (hipMemcpyAsync(m->vel, zero.data(), (size_t)NPARAM * 4, hipMemcpyHostToDevice, m->stream) != hipSuccess) return PIBM_EDEVICE;
    m->step = 0;
    return hipStreamSynchronize(m->stream) == hipSuccess ? PIBM_OK : PIBM_EDEVICE;
}

int mlp_grad_pass(pibm_mlp *m, const void *x, const float *t, int n)
{
    const int nblk = (n + SPB - 1) / SPB;
    MlpArgs a{m->param, m->wbf};
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(MLP_THREADS), 0, m->stream, a, (const uint16_t *)x, t, n, m->part,
                       m->loss_part);
    return hipGetLastError() == hipSuccess ? PIBM_OK : PIBM_EDEVICE;
}

int mlp_loss(pibm_mlp *m, int n, double *loss)
{
    const int nblk = (n + SPB - 1) / SPB;
    std::vector<double> lp((size_t)nblk);
    if (hipMemcpyAsync(lp.data(), m->loss_part, (size_t)nblk * 8, hipMemcpyDeviceToHost, m->stream) != hipSuccess) return PIBM_EDEVICE;
    if (hipStreamSynchronize(m->stream) != hipSuccess) return PIBM_EDEVICE;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += lp[(size_t)b];
    *loss = s / (4.0 * n);
    return PIBM_OK;
}

// Device address of `scratch` on the device of `stream`, resolved once per
// device with that device current and kept for the process.
constexpr int SCR_MAX_DEVICES = 64;
std::mutex scr_mu;
char *scr_addr[SCR_MAX_DEVICES];

int scratch_on(hipStream_t stream, char **out)
{
    int dev = 0;
    if ((stream ? hipStreamGetDevice(stream, &dev) : hipGetDevice(&dev)) != hipSuccess) return PIBM_EDEVICE;
    if (dev < 0 || dev >= SCR_MAX_DEVICES) return PIBM_EDEVICE;
    std::lock_guard<std::mutex> lock(scr_mu);
    if (!scr_addr[dev]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return PIBM_EDEVICE;
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return PIBM_EDEVICE;
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) return PIBM_EDEVICE;
        scr_addr[dev] = (char *)p;
    }
    *out = scr_addr[dev];
    return PIBM_OK;
}

}  // namespace

int pibm_mlp_forward_on(pibm_mlp *m, const void *dev_x, float *dev_y, int n, hipStream_t stream)
{
    if (!m || n < 0 || (n > 0 && (!dev_x || !dev_y))) return PIBM_EINVAL;
    if (((uintptr_t)dev_x & 7) || ((uintptr_t)dev_y & 15)) return PIBM_EINVAL;
    if (n == 0) return PIBM_OK;
    const int ntile = (n + 15) / 16;
    int grid = (ntile + 3) / 4;
    if (grid > 2048) grid = 2048;
    MlpArgs a{m->param, m->wbf};
    hipLaunchKernelGGL(k_mlp_fwd, dim3(grid), dim3(MLP_THREADS), 0, stream, a, (const uint16_t *)dev_x, dev_y, n);
    return hipGetLastError() == hipSuccess ? PIBM_OK : PIBM_EDEVICE;
}

extern "C" {

size_t pibm_mlp_workspace_bytes(int max_batch)
{
    if (max_batch < 1) return 0;
    return mlp_plan(max_batch).total;
}

int pibm_mlp_create(pibm_mlp **out, unsigned long long seed, int max_batch, void *ws, size_t bytes, void *stream)
{
    if (!out || max_batch < 1 || !ws || ((uintptr_t)ws & 255)) return PIBM_EINVAL;
    *out = nullptr;
    const MlpPlan P = mlp_plan(max_batch);
    if (bytes < P.total) return PIBM_EINVAL;
    pibm_mlp *m = new (std::nothrow) pibm_mlp();
    if (!m) return PIBM_EINVAL;
    char *b = (char *)ws;
    m->stream = (hipStream_t)stream;
    m->max_batch = max_batch;
    m->max_blk = (max_batch + SPB - 1) / SPB;
    m->param = (float *)(b + P.off[0]);
    m->mom = (float *)(b + P.off[1]);
    m->vel = (float *)(b + P.off[2]);
    m->wbf = (uint16_t *)(b + P.off[3]);
    m->part = (float *)(b + P.off[4]);
    m->grad = (float *)(b + P.off[5]);
    m->loss_part = (double *)(b + P.off[6]);
    // U(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases
    std::vector<float> prm((size_t)NPARAM, 0.f);
    SplitMix r{seed};
    const int ow[4] = {OW1, OW2, OW3, OW4}, nin[4] = {NI, NH, NH, NH}, nout[4] = {NH, NH, NH, NO};
    for (int L = 0; L < 4; ++L) {
        const double lim = 1.0 / std::sqrt((double)nin[L]);
        for (int i = 0; i < nin[L] * nout[L]; ++i) prm[(size_t)ow[L] + i] = (float)((2.0 * r.uniform() - 1.0) * lim);
    }
    const int st = mlp_upload(m, prm.data());
    if (st) { delete m; return st; }
    *out = m;
    return PIBM_OK;
}

int pibm_mlp_set_params(pibm_mlp *m, const float *host_params)
{
    if (!m || !host_params) return PIBM_EINVAL;
    for (int i = 0; i < NPARAM; ++i)
        if (!std::isfinite(host_params[i])) return PIBM_EINVAL;
    return mlp_upload(m, host_params);
}

int pibm_mlp_get_params(pibm_mlp *m, float *host_params)
{
    if (!m || !host_params) return PIBM_EINVAL;
    if (hipMemcpyAsync(host_params, m->param, (size_t)NPARAM * 4, hipMemcpyDeviceToHost, m->stream) != hipSuccess) return PIBM_EDEVICE;
    return hipStreamSynchronize(m->stream) == hipSuccess ? PIBM_OK : PIBM_EDEVICE;
}

int pibm_mlp_forward(pibm_mlp *m, const void *dev_x, float *dev_y, int n)
{
    if (!m) return PIBM_EINVAL;
    return pibm_mlp_forward_on(m, dev_x, dev_y, n, m->stream);
}

int pibm_mlp_grads(pibm_mlp *m, const void *dev_x, const float *dev_t, int n, float *host_grads, double *loss)
{
    if (!m || n < 1 || n > m->max_batch || !dev_x || !dev_t || !host_grads) return PIBM_EINVAL;
    if (((uintptr_t)dev_x & 7) || ((uintptr_t)dev_t & 15)) return PIBM_EINVAL;
    int st = mlp_grad_pass(m, dev_x, dev_t, n);
    if (st) return st;
    const int nblk = (n + SPB - 1) / SPB;
    hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, m->param, m->wbf, m->mom,
                       m->vel, (const float *)m->part, nblk, m->grad, 0.f, 1.f, 1.f);
    if (hipGetLastError() != hipSuccess) return PIBM_EDEVICE;
    if (hipMemcpyAsync(host_grads, m->grad, (size_t)NPARAM * 4, hipMemcpyDeviceToHost, m->stream) != hipSuccess) return PIBM_EDEVICE;
    if (loss) return mlp_loss(m, n, loss);
    return hipStreamSynchronize(m->stream) == hipSuccess ? PIBM_OK : PIBM_EDEVICE;
}

int pibm_mlp_grads_noalloc(pibm_mlp *m, const void *dev_x, const float *dev_t, int n, float *host_grads,
                           double *loss)
{
    if (!m || n < 1 || n > PIBM_MLP_NOALLOC_MAX_BATCH || !dev_x || !dev_t || !host_grads) return PIBM_EINVAL;
    if (((uintptr_t)dev_x & 7) || ((uintptr_t)dev_t & 15)) return PIBM_EINVAL;
    char *scr = nullptr;
    int st = scratch_on(m->stream, &scr);
    if (st) return st;
    float *part = (float *)(scr + SCR_PART), *grad = (float *)(scr + SCR_GRAD);
    double *loss_part = (double *)(scr + SCR_LOSS);
    // every workgroup writes its whole gradient slot and its loss partial, and
    // the sum overwrites every gradient entry: nothing needs clearing
    const int nblk = (n + SPB - 1) / SPB;
    MlpArgs a{m->param, m->wbf};
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(MLP_THREADS), 0, m->stream, a, (const uint16_t *)dev_x, dev_t, n,
                       part, loss_part);
    hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, m->param, m->wbf, m->mom,
                       m->vel, (const float *)part, nblk, grad, 0.f, 1.f, 1.f);
    if (hipGetLastError() != hipSuccess) return PIBM_EDEVICE;
    double lp[NOALLOC_BLK];
    if (hipMemcpyAsync(host_grads, grad, (size_t)NPARAM * 4, hipMemcpyDeviceToHost, m->stream) != hipSuccess) return PIBM_EDEVICE;
    if (loss && hipMemcpyAsync(lp, loss_part, (size_t)nblk * 8, hipMemcpyDeviceToHost, m->stream) != hipSuccess)
        return PIBM_EDEVICE;
    if (hipStreamSynchronize(m->stream) != hipSuccess) return PIBM_EDEVICE;
    if (loss) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += lp[b];
        *loss = s / (4.0 * n);
    }
    return PIBM_OK;
}

int pibm_mlp_train_step(pibm_mlp *m, const void *dev_x, const float *dev_t, int n, float lr, double *loss)
{
    if (!m || n < 1 || n > m->max_batch || !dev_x || !dev_t || !(lr > 0.f)) return PIBM_EINVAL;
    if (((uintptr_t)dev_x & 7) || ((uintptr_t)dev_t & 15)) return PIBM_EINVAL;
    int st = mlp_grad_pass(m, dev_x, dev_t, n);
    if (st) return st;
    m->step += 1;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)m->step));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)m->step));
    const int nblk = (n + SPB - 1) / SPB;
    hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, m->stream, m->param, m->wbf, m->mom,
                       m->vel, (const float *)m->part, nblk, (float *)nullptr, lr, c1, c2);
    if (hipGetLastError() != hipSuccess) return PIBM_EDEVICE;
    if (loss) return mlp_loss(m, n, loss);
    return PIBM_OK;
}

int pibm_mlp_destroy(pibm_mlp *m)
{
    delete m;
    return PIBM_OK;
}

}  // extern "C"
