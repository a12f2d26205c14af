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

}  // namespace gqaoa
