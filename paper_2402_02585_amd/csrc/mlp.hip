// Angle-predictor MLP: 131 -> 256 -> GELU -> 256 -> GELU -> 2, bfloat16
// operands on the matrix cores (v_mfma_f32_16x16x32_bf16), float32 accumulation.
//
// The paper proposes deriving G-QAOA angles from statistics of the density of
// states (Sec. V) and observes that optimized single-angle pairs cluster
// (Sec. III.B); the network maps the normalized level histogram and (n, d, p)
// to one (beta, gamma) pair.
//
// Storage points in bfloat16 (round to nearest even): inputs, weights,
// post-GELU activations, and the pre-activation gradients that enter the
// backward products. Pre-activations z1, z2, outputs and all gradients of
// parameters are float32; the float32 master weights are updated by Adam.
//
// GEMM: 256 threads compute a 64x64 tile of C = A B; each wave owns a 32x32
// quarter as 2x2 MFMA tiles. A and B tiles of 64x32 are staged in LDS with k
// contiguous so a lane fetches its 8 consecutive k values with one 16-byte
// LDS read. Transposed operands (the backward products) are handled by the
// staging loads.
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace gqaoa {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int kDIn = 131, kDInPad = 160, kDH = 256, kDOut = 2;
constexpr size_t kOffW1 = 0;
constexpr size_t kOffB1 = kOffW1 + (size_t)kDInPad * kDH;
constexpr size_t kOffW2 = kOffB1 + kDH;
constexpr size_t kOffB2 = kOffW2 + (size_t)kDH * kDH;
constexpr size_t kOffW3 = kOffB2 + kDH;
constexpr size_t kOffB3 = kOffW3 + (size_t)kDH * kDOut;
constexpr size_t kNParams = kOffB3 + kDOut;
static_assert(kNParams == GQAOA_MLP_NPARAMS, "parameter packing");

// Round a float to bfloat16, nearest with ties to even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
    const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
    const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
    return cdf + z * pdf;
}

// ---- activation cache layout ---------------------------------------------------
struct ActLayout {
    size_t xb, z1, h1, z2, h2, dz, dz1, wb, total;
};
static size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
static ActLayout act_layout(int batch) {
    ActLayout L{};
    const size_t B = (size_t)batch;
    size_t o = 0;
    L.xb = o;  o += al256(B * kDInPad * 2);   // bf16 inputs, padded to 160
    L.z1 = o;  o += al256(B * kDH * 4);       // float z1
    L.h1 = o;  o += al256(B * kDH * 2);       // bf16 h1
    L.z2 = o;  o += al256(B * kDH * 4);       // float z2
    L.h2 = o;  o += al256(B * kDH * 2);       // bf16 h2
    L.dz = o;  o += al256(B * kDH * 2);       // bf16 dz2
    L.dz1 = o; o += al256(B * kDH * 2);       // bf16 dz1
    L.wb = o;  o += al256(kNParams * 2);      // bf16 copies of W1, W2, W3 (same packing)
    L.total = o;
    return L;
}
size_t mlp_act_bytes(int batch) { return act_layout(batch).total; }

// ---- MFMA GEMM -------------------------------------------------------------------
enum Epi { kEpiBiasGelu = 0, kEpiStoreF32 = 1, kEpiGeluGrad = 2 };

struct GemmArgs {
    const uint16_t *A;  // bf16
    const uint16_t *B;  // bf16
    int M, N, K, lda, ldb;
    // epilogue
    const float *bias;  // [N]            (kEpiBiasGelu)
    float *Cf;          // [M][ldc] float (z for kEpiBiasGelu, C for kEpiStoreF32)
    uint16_t *Cb;       // [M][ldc] bf16  (gelu(z) or dz)
    const float *Zin;   // [M][ldc] float pre-activation (kEpiGeluGrad)
    int ldc;
};

constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8;

template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g) {
    __shared__ uint16_t As[kBM][kBK + kPad];
    __shared__ uint16_t Bs[kBN][kBK + kPad];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < g.K; k0 += kBK) {
        // stage A (64 x 32) and B (32 x 64), k contiguous in LDS
        if constexpr (!TA) {
            const int r = tid >> 2, kc = (tid & 3) * 8;
            const int m = m0 + r;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + kc + e;
                As[r][kc + e] = (m < g.M && k < g.K) ? g.A[(size_t)m * g.lda + k] : (uint16_t)0;
            }
        } else {
            const int kk = tid >> 3, mc = (tid & 7) * 8;
            const int k = k0 + kk;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int m = m0 + mc + e;
                As[mc + e][kk] = (m < g.M && k < g.K) ? g.A[(size_t)k * g.lda + m] : (uint16_t)0;
            }
        }
        if constexpr (TB) {
            const int r = tid >> 2, kc = (tid & 3) * 8;
            const int n = n0 + r;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + kc + e;
                Bs[r][kc + e] = (n < g.N && k < g.K) ? g.B[(size_t)n * g.ldb + k] : (uint16_t)0;
            }
        } else {
            const int kk = tid >> 3, nc = (tid & 7) * 8;
            const int k = k0 + kk;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int n = n0 + nc + e;
                Bs[nc + e][kk] = (n < g.N && k < g.K) ? g.B[(size_t)k * g.ldb + n] : (uint16_t)0;
            }
        }
        __syncthreads();
        const int r16 = lane & 15, kg = (lane >> 4) * 8;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const u16x8 av = *reinterpret_cast<const u16x8 *>(&As[wm + i * 16 + r16][kg]);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const u16x8 bv = *reinterpret_cast<const u16x8 *>(&Bs[wn + j * 16 + r16][kg]);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                    __builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv), acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // lane holds C[4*(lane/16) + r][lane % 16] of each 16x16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
                const int n = n0 + wn + j * 16 + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                const float v = acc[i][j][r];
                const size_t o = (size_t)m * g.ldc + n;
                if constexpr (EPI == kEpiBiasGelu) {
                    const float z = v + g.bias[n];
                    g.Cf[o] = z;
                    g.Cb[o] = f2bf(gelu(z));
                } else if constexpr (EPI == kEpiStoreF32) {
                    g.Cf[o] = v;
                } else {
                    g.Cb[o] = f2bf(v * gelu_grad(g.Zin[o]));
                }
            }
}

template <bool TA, bool TB, int EPI>
static int gemm(const GemmArgs &g, hipStream_t st) {
    const dim3 grid((g.N + kBN - 1) / kBN, (g.M + kBM - 1) / kBM);
    hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB, EPI>), grid, dim3(256), 0, st, g);
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

// ---- small kernels -----------------------------------------------------------------
// x (float [B][131]) -> bf16 [B][160] zero padded.
__global__ void pack_inputs_kernel(const float *__restrict__ x, int batch, uint16_t *__restrict__ xb) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)batch * kDInPad) return;
    const int b = (int)(i / kDInPad), c = (int)(i % kDInPad);
    xb[i] = c < kDIn ? f2bf(x[(size_t)b * kDIn + c]) : (uint16_t)0;
}

// bf16 copies of W1, W2, W3 (rows 131..159 of W1 are zero in the master copy).
__global__ void pack_weights_kernel(const float *__restrict__ prm, uint16_t *__restrict__ wb) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kNParams) wb[i] = f2bf(prm[i]);
}

// o[b][c] = sum_j h2[b][j] W3[j][c] + b3[c]; one wave per row.
__global__ void out_layer_kernel(const uint16_t *__restrict__ h2, const uint16_t *__restrict__ w3b,
                                 const float *__restrict__ b3, int batch, float *__restrict__ out) {
    const int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= batch) return;
    float s0 = 0.f, s1 = 0.f;
    for (int j = lane; j < kDH; j += 64) {
        const float h = bf2f(h2[(size_t)row * kDH + j]);
        s0 += h * bf2f(w3b[j * 2]);
        s1 += h * bf2f(w3b[j * 2 + 1]);
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    if (lane == 0) {
        out[(size_t)row * 2] = s0 + b3[0];
        out[(size_t)row * 2 + 1] = s1 + b3[1];
    }
}

// dz2[b][j] = bf16((sum_c dout[b][c] W3[j][c]) * gelu'(z2[b][j])).
__global__ void out_backward_kernel(const float *__restrict__ dout, const uint16_t *__restrict__ w3b,
                                    const float *__restrict__ z2, int batch, uint16_t *__restrict__ dz2) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)batch * kDH) return;
    const int b = (int)(i / kDH), j = (int)(i % kDH);
    const float dh = dout[(size_t)b * 2] * bf2f(w3b[j * 2]) + dout[(size_t)b * 2 + 1] * bf2f(w3b[j * 2 + 1]);
    dz2[i] = f2bf(dh * gelu_grad(z2[i]));
}

// Column sums over the batch, fixed order: one block per column group.
//   mode 0: g[c] = sum_b bf16 dz[b][c]                 (bias gradients)
//   mode 1: gW3[j][c] = sum_b h2[b][j] dout[b][c], gb3 (output layer)
__global__ void __launch_bounds__(256) colsum_bf16_kernel(const uint16_t *__restrict__ dz, int batch,
                                                         int ncol, float *__restrict__ g) {
    __shared__ double red[4];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < batch; b += 256) s += bf2f(dz[(size_t)b * ncol + c]);
    double v[1] = {s};
    block_sum<1, 256>(v, red);
    if (threadIdx.x == 0) g[c] = (float)v[0];
}

__global__ void __launch_bounds__(256) out_grad_kernel(const uint16_t *__restrict__ h2,
                                                       const float *__restrict__ dout, int batch,
                                                       float *__restrict__ gW3, float *__restrict__ gb3) {
    __shared__ double red[8];
    const int j = blockIdx.x;  // 0..255 -> W3 row; 256 -> bias
    double s0 = 0.0, s1 = 0.0;
    for (int b = threadIdx.x; b < batch; b += 256) {
        const double h = j < kDH ? (double)bf2f(h2[(size_t)b * kDH + j]) : 1.0;
        s0 += h * dout[(size_t)b * 2];
        s1 += h * dout[(size_t)b * 2 + 1];
    }
    double v[2] = {s0, s1};
    block_sum<2, 256>(v, red);
    if (threadIdx.x == 0) {
        if (j < kDH) {
            gW3[j * 2] = (float)v[0];
            gW3[j * 2 + 1] = (float)v[1];
        } else {
            gb3[0] = (float)v[0];
            gb3[1] = (float)v[1];
        }
    }
}

// Loss of the angle regression and its gradient with respect to the raw outputs:
// beta = 2 pi sigmoid(o0), gamma = pi sigmoid(o1),
// L = mean_b ((beta-beta*)/(2 pi))^2 + ((gamma-gamma*)/pi)^2.
__global__ void __launch_bounds__(256) loss_kernel(const float *__restrict__ out, const float *__restrict__ tgt,
                                                   int batch, float *__restrict__ dout, float *__restrict__ loss) {
    __shared__ double red[4];
    double s = 0.0;
    const float invB = 1.0f / (float)batch;
    for (int b = threadIdx.x; b < batch; b += 256) {
        const float s0 = 1.f / (1.f + expf(-out[(size_t)b * 2]));
        const float s1 = 1.f / (1.f + expf(-out[(size_t)b * 2 + 1]));
        const float rb = s0 - tgt[(size_t)b * 2] * (0.5f / (float)M_PI);
        const float rg = s1 - tgt[(size_t)b * 2 + 1] * (1.0f / (float)M_PI);
        s += (double)(rb * rb + rg * rg);
        dout[(size_t)b * 2] = 2.f * rb * s0 * (1.f - s0) * invB;
        dout[(size_t)b * 2 + 1] = 2.f * rg * s1 * (1.f - s1) * invB;
    }
    double v[1] = {s};
    block_sum<1, 256>(v, red);
    if (threadIdx.x == 0) *loss = (float)(v[0] / batch);
}

__global__ void adam_kernel(float *__restrict__ prm, const float *__restrict__ grd, float *__restrict__ m,
                            float *__restrict__ v, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParams) return;
    // rows 131..159 of W1 stay zero
    if (i < kOffB1 && (i / kDH) >= (size_t)kDIn) return;
    const float g = grd[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    prm[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Features: w_k = N_k / 2^n for k < 128 (zero beyond m), n/24, d/8, log2(p)/6.
__global__ void features_kernel(const unsigned long long *__restrict__ hists, int hist_stride,
                                const int32_t *__restrict__ n, const int32_t *__restrict__ m,
                                const int32_t *__restrict__ p, int batch, float *__restrict__ x) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)batch * kDIn) return;
    const int b = (int)(i / kDIn), c = (int)(i % kDIn);
    float v;
    if (c < 128) v = c <= m[b] && c < hist_stride ? (float)((double)hists[(size_t)b * hist_stride + c] * ldexp(1.0, -n[b])) : 0.f;
    else if (c == 128) v = (float)n[b] / 24.f;
    else if (c == 129) v = (float)((double)m[b] / (double)n[b] / 8.0);
    else v = (float)(log2((double)p[b]) / 6.0);
    x[i] = v;
}

// ---- host entry points ---------------------------------------------------------------
int run_mlp_forward(const float *prm, int batch, const float *x, float *out, void *act, hipStream_t st) {
    const ActLayout L = act_layout(batch);
    char *a = reinterpret_cast<char *>(act);
    uint16_t *xb = reinterpret_cast<uint16_t *>(a + L.xb);
    uint16_t *wb = reinterpret_cast<uint16_t *>(a + L.wb);
    const size_t nx = (size_t)batch * kDInPad;
    hipLaunchKernelGGL(pack_inputs_kernel, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, st, x, batch, xb);
    GQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(pack_weights_kernel, dim3((unsigned)((kNParams + 255) / 256)), dim3(256), 0, st, prm, wb);
    GQ_LAUNCH_CHECK();
    GemmArgs g{};
    g.A = xb; g.lda = kDInPad;
    g.B = wb + kOffW1; g.ldb = kDH;
    g.M = batch; g.N = kDH; g.K = kDInPad;
    g.bias = prm + kOffB1;
    g.Cf = reinterpret_cast<float *>(a + L.z1);
    g.Cb = reinterpret_cast<uint16_t *>(a + L.h1);
    g.ldc = kDH;
    int s = gemm<false, false, kEpiBiasGelu>(g, st);
    if (s) return s;
    g.A = reinterpret_cast<uint16_t *>(a + L.h1); g.lda = kDH;
    g.B = wb + kOffW2; g.ldb = kDH;
    g.K = kDH;
    g.bias = prm + kOffB2;
    g.Cf = reinterpret_cast<float *>(a + L.z2);
    g.Cb = reinterpret_cast<uint16_t *>(a + L.h2);
    if ((s = gemm<false, false, kEpiBiasGelu>(g, st))) return s;
    hipLaunchKernelGGL(out_layer_kernel, dim3((unsigned)((batch + 3) / 4)), dim3(256), 0, st,
                       reinterpret_cast<uint16_t *>(a + L.h2), wb + kOffW3, prm + kOffB3, batch, out);
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

int run_mlp_backward(const float *prm, int batch, const void *act, const float *dout, float *grads,
                     hipStream_t st) {
    (void)prm;
    const ActLayout L = act_layout(batch);
    char *a = const_cast<char *>(reinterpret_cast<const char *>(act));
    const uint16_t *wb = reinterpret_cast<uint16_t *>(a + L.wb);
    const uint16_t *h1 = reinterpret_cast<uint16_t *>(a + L.h1);
    const uint16_t *h2 = reinterpret_cast<uint16_t *>(a + L.h2);
    uint16_t *dz2 = reinterpret_cast<uint16_t *>(a + L.dz);
    uint16_t *dz1 = reinterpret_cast<uint16_t *>(a + L.dz1);
    const uint16_t *xb = reinterpret_cast<uint16_t *>(a + L.xb);
    // output layer: gW3, gb3, then dz2
    hipLaunchKernelGGL(out_grad_kernel, dim3(kDH + 1), dim3(256), 0, st, h2, dout, batch, grads + kOffW3, grads + kOffB3);
    GQ_LAUNCH_CHECK();
    const size_t nh = (size_t)batch * kDH;
    hipLaunchKernelGGL(out_backward_kernel, dim3((unsigned)((nh + 255) / 256)), dim3(256), 0, st, dout,
                       wb + kOffW3, reinterpret_cast<const float *>(a + L.z2), batch, dz2);
    GQ_LAUNCH_CHECK();
    // gW2 = h1^T dz2  (M = 256, N = 256, K = batch)
    GemmArgs g{};
    g.A = h1; g.lda = kDH;
    g.B = dz2; g.ldb = kDH;
    g.M = kDH; g.N = kDH; g.K = batch;
    g.Cf = grads + kOffW2; g.ldc = kDH;
    int s = gemm<true, false, kEpiStoreF32>(g, st);
    if (s) return s;
    hipLaunchKernelGGL(colsum_bf16_kernel, dim3(kDH), dim3(256), 0, st, dz2, batch, kDH, grads + kOffB2);
    GQ_LAUNCH_CHECK();
    // dz1 = bf16((dz2 W2^T) * gelu'(z1))  (M = batch, N = 256, K = 256)
    GemmArgs d{};
    d.A = dz2; d.lda = kDH;
    d.B = wb + kOffW2; d.ldb = kDH;   // W2[i][j] read as B(k=j, n=i)
    d.M = batch; d.N = kDH; d.K = kDH;
    d.Zin = reinterpret_cast<const float *>(a + L.z1);
    d.Cb = dz1; d.ldc = kDH;
    if ((s = gemm<false, true, kEpiGeluGrad>(d, st))) return s;
    // gW1 = xb^T dz1 (M = 160, N = 256, K = batch)
    GemmArgs w{};
    w.A = xb; w.lda = kDInPad;
    w.B = dz1; w.ldb = kDH;
    w.M = kDInPad; w.N = kDH; w.K = batch;
    w.Cf = grads + kOffW1; w.ldc = kDH;
    if ((s = gemm<true, false, kEpiStoreF32>(w, st))) return s;
    hipLaunchKernelGGL(colsum_bf16_kernel, dim3(kDH), dim3(256), 0, st, dz1, batch, kDH, grads + kOffB1);
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

int run_mlp_adam(float *prm, const float *grads, float *state, int step, float lr, float b1, float b2,
                 float eps, hipStream_t st) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((kNParams + 255) / 256)), dim3(256), 0, st, prm, grads,
                       state, state + kNParams, lr, b1, b2, eps, c1, c2);
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

int run_mlp_loss(int batch, const float *out, const float *tgt, float *dout, float *loss, hipStream_t st) {
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, st, out, tgt, batch, dout, loss);
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

int run_mlp_features(int batch, const uint64_t *hists, int hist_stride, const int32_t *n, const int32_t *m,
                     const int32_t *p, float *x, hipStream_t st) {
    const size_t nx = (size_t)batch * kDIn;
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<const unsigned long long *>(hists), hist_stride, n, m, p, batch, x);
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

// ---- inference: weights stationary in LDS ----------------------------------------------
// A small kernel packs the LDS images of W1^T and W2^T (bfloat16) into the
// workspace; then two persistent kernels of 512 threads (8 waves) run over
// tiles of 128 rows, each block copying its weight image with 16-byte loads; a
// wave owns 16 rows and all 256 hidden units (16 MFMA tiles, 64 accumulator
// registers). Kernel 1 keeps W1^T (bfloat16) in LDS, stages the tile's x rows
// (contiguous in memory) through LDS and writes h1 = bf16(gelu(x W1 + b1)).
// Kernel 2 keeps W2^T in LDS, loads h1 fragments straight into the MFMA
// operand layout and folds the output layer into its epilogue, so h2 never
// leaves registers. The MFMA k-order equals the training GEMM's, so h1 and
// h2 are bit-identical to the training forward; only the output layer's
// 256-term sum is taken in another order.
constexpr int kInfThreads = 512, kInfRows = 128, kWPad = 8;
constexpr int kW1Ld = kDInPad + kWPad, kW2Ld = kDH + kWPad, kXLd = kDInPad + kWPad;

constexpr size_t kW1Image = (size_t)kDH * kW1Ld * 2, kW2Image = (size_t)kDH * kW2Ld * 2;  // bytes

// workspace: [W1^T LDS image | W2^T LDS image | h1 (bfloat16 [batch][256])]
size_t mlp_infer_bytes(int batch) { return al256(kW1Image) + al256(kW2Image) + al256((size_t)batch * kDH * 2); }

// The LDS images of both weight matrices, bfloat16, transposed ([n][k]) and
// padded, so every block of the inference kernels loads them with 16-byte
// copies.
__global__ void mlp_pack_images_kernel(const float *__restrict__ prm, uint16_t *__restrict__ w1t,
                                       uint16_t *__restrict__ w2t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kDH * kW1Ld) {
        const int n = i / kW1Ld, k = i % kW1Ld;
        w1t[i] = k < kDIn ? f2bf(prm[kOffW1 + (size_t)k * kDH + n]) : (uint16_t)0;
    }
    if (i < kDH * kW2Ld) {
        const int n = i / kW2Ld, k = i % kW2Ld;
        w2t[i] = k < kDH ? f2bf(prm[kOffW2 + (size_t)k * kDH + n]) : (uint16_t)0;
    }
}

// 16-byte copy of an LDS image (bytes a multiple of 16) by a whole block.
__device__ __forceinline__ void load_image(uint16_t *dst, const uint16_t *__restrict__ src, size_t bytes) {
    const uint4 *s = reinterpret_cast<const uint4 *>(src);
    uint4 *d = reinterpret_cast<uint4 *>(dst);
    for (size_t i = threadIdx.x; i < bytes / 16; i += blockDim.x) d[i] = s[i];
}

__global__ void __launch_bounds__(kInfThreads) mlp_infer_l1_kernel(const float *__restrict__ prm,
                                                                    const uint16_t *__restrict__ w1t,
                                                                    const float *__restrict__ x, int batch,
                                                                    int x_aligned, uint16_t *__restrict__ h1) {
    __shared__ __attribute__((aligned(16))) uint16_t w[kDH * kW1Ld];        // W1^T: [n][k]
    __shared__ __attribute__((aligned(16))) uint16_t xs[kInfRows * kXLd];   // the tile's inputs: [row][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    load_image(w, w1t, kW1Image);
    const int r16 = lane & 15, kg = (lane >> 4) * 8;
    float b1[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) b1[t] = prm[kOffB1 + t * 16 + r16];
    const int ntiles = (batch + kInfRows - 1) / kInfRows;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int row0 = tile * kInfRows;
        const int rows = min(kInfRows, batch - row0);
        __syncthreads();  // the previous tile's reads of xs (and, first time, the W1 staging) are done
        // the tile's rows are contiguous and, when x is 16-byte aligned, start
        // 16-byte aligned (row0 is a multiple of 4): float4 loads over the
        // valid part, zeros past the batch
        const float *src = x + (size_t)row0 * kDIn;
        const int nvalid = rows * kDIn;
        for (int j = tid; j < (kInfRows * kDIn) / 4; j += kInfThreads) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (x_aligned && 4 * j + 3 < nvalid) {
                v = reinterpret_cast<const float4 *>(src)[j];
            } else {
                if (4 * j < nvalid) v.x = src[4 * j];
                if (4 * j + 1 < nvalid) v.y = src[4 * j + 1];
                if (4 * j + 2 < nvalid) v.z = src[4 * j + 2];
                if (4 * j + 3 < nvalid) v.w = src[4 * j + 3];
            }
            const float e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 4 * j + q, r = i / kDIn, k = i % kDIn;
                xs[r * kXLd + k] = f2bf(e[q]);
            }
        }
        for (int i = tid; i < kInfRows * (kDInPad - kDIn); i += kInfThreads) {
            const int r = i / (kDInPad - kDIn), k = kDIn + i % (kDInPad - kDIn);
            xs[r * kXLd + k] = 0;
        }
        __syncthreads();
        f32x4 acc[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kDInPad / 32; ++ks) {
            const u16x8 av = *reinterpret_cast<const u16x8 *>(&xs[(wave * 16 + r16) * kXLd + ks * 32 + kg]);
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const u16x8 bv = *reinterpret_cast<const u16x8 *>(&w[(t * 16 + r16) * kW1Ld + ks * 32 + kg]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                                 __builtin_bit_cast(bf16x8, bv), acc[t], 0, 0, 0);
            }
        }
        // lane holds C[4*(lane/16) + r][lane % 16] of each 16x16 tile
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = row0 + wave * 16 + 4 * (lane >> 4) + r;
            if (row >= batch) continue;
            uint16_t *dst = h1 + (size_t)row * kDH + r16;
#pragma unroll
            for (int t = 0; t < 16; ++t) dst[t * 16] = f2bf(gelu(acc[t][r] + b1[t]));
        }
    }
}

__global__ void __launch_bounds__(kInfThreads) mlp_infer_l23_kernel(const float *__restrict__ prm,
                                                                     const uint16_t *__restrict__ w2t,
                                                                     const uint16_t *__restrict__ h1, int batch,
                                                                     float *__restrict__ out) {
    __shared__ __attribute__((aligned(16))) uint16_t w[kDH * kW2Ld];        // W2^T: [n][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    load_image(w, w2t, kW2Image);
    const int r16 = lane & 15, kg = (lane >> 4) * 8;
    float b2[16], w30[16], w31[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int n = t * 16 + r16;
        b2[t] = prm[kOffB2 + n];
        w30[t] = bf2f(f2bf(prm[kOffW3 + (size_t)n * kDOut]));
        w31[t] = bf2f(f2bf(prm[kOffW3 + (size_t)n * kDOut + 1]));
    }
    const float b30 = prm[kOffB3], b31 = prm[kOffB3 + 1];
    __syncthreads();
    const int ntiles = (batch + kInfRows - 1) / kInfRows;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int row0 = tile * kInfRows;
        const int arow = row0 + wave * 16 + r16;  // the A-operand row of this lane
        const bool live = arow < batch;
        const uint16_t *src = h1 + (size_t)(live ? arow : 0) * kDH + kg;
        f32x4 acc[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
        for (int ks = 0; ks < kDH / 32; ++ks) {
            u16x8 av = *reinterpret_cast<const u16x8 *>(src + ks * 32);
            if (!live) av = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const u16x8 bv = *reinterpret_cast<const u16x8 *>(&w[(t * 16 + r16) * kW2Ld + ks * 32 + kg]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                                 __builtin_bit_cast(bf16x8, bv), acc[t], 0, 0, 0);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float s0 = 0.f, s1 = 0.f;
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const float h = bf2f(f2bf(gelu(acc[t][r] + b2[t])));
                s0 += h * w30[t];
                s1 += h * w31[t];
            }
            // the 16 lanes of a group hold the same rows, different columns
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                s0 += __shfl_xor(s0, off, kWave);
                s1 += __shfl_xor(s1, off, kWave);
            }
            const int row = row0 + wave * 16 + 4 * (lane >> 4) + r;
            if (r16 == 0 && row < batch) {
                out[(size_t)row * kDOut] = s0 + b30;
                out[(size_t)row * kDOut + 1] = s1 + b31;
            }
        }
    }
}

int run_mlp_infer(const float *prm, int batch, const float *x, float *out, void *ws, hipStream_t st) {
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    char *base = reinterpret_cast<char *>(ws);
    uint16_t *w1t = reinterpret_cast<uint16_t *>(base);
    uint16_t *w2t = reinterpret_cast<uint16_t *>(base + al256(kW1Image));
    uint16_t *h1 = reinterpret_cast<uint16_t *>(base + al256(kW1Image) + al256(kW2Image));
    const int img = std::max(kDH * kW1Ld, kDH * kW2Ld);
    hipLaunchKernelGGL(mlp_pack_images_kernel, dim3((img + 255) / 256), dim3(256), 0, st, prm, w1t, w2t);
    GQ_LAUNCH_CHECK();
    const int ntiles = (batch + kInfRows - 1) / kInfRows;
    const int blocks = std::min(ntiles, dev.num_cus);
    const int x_aligned = (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    hipLaunchKernelGGL(mlp_infer_l1_kernel, dim3(blocks), dim3(kInfThreads), 0, st, prm, w1t, x, batch, x_aligned,
                       h1);
    GQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(mlp_infer_l23_kernel, dim3(blocks), dim3(kInfThreads), 0, st, prm, w2t, h1, batch, out);
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

}  // namespace gqaoa
