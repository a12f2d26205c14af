// X-QAOA rounds: phase separator plus the transverse-field mixer
// exp(-i beta sum_q X_q) = prod_q exp(-i beta X_q) (Sec. II.B, the "X" rows of
// Table I), streamed from HBM.
//
// exp(-i beta X_q) mixes the amplitude pairs that differ in bit q:
// (a, b) -> (c a - i s b, c b - i s a), c = cos beta, s = sin beta. A round
// is done in passes over 32 KiB LDS tiles (2^T amplitudes, T = 12 for
// complex64, 11 for complex128):
//   * the low pass takes 2^T consecutive amplitudes, reads out P_sol / E /
//     norm of the incoming state, applies the phase LUT e^{-i gamma C(z)} and
//     then the butterflies of qubits 0..T-1;
//   * each high pass takes 2^C consecutive amplitudes (one 128-byte run:
//     C = 4 for complex64, 3 for complex128) times the 2^K values of qubits
//     q0..q0+K-1 (K = T - C = 8) and applies those K butterfly stages.
// At n = 28, complex64, a round is three passes (qubits 0-11, 12-19, 20-27).
// Butterfly stages are applied two qubits at a time (radix 4) between LDS
// round trips.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace gqaoa {

constexpr int kXThreads = 256;
constexpr int kXTileBytesLog2 = 15;  // 32 KiB of LDS per tile
constexpr int kXRowBytesLog2 = 7;    // 128-byte contiguous runs in the high passes
constexpr int kXMaxBlocks = 4096;
constexpr int kXR = 7;  // partial sums per block, laid out as in the statevector passes

inline int x_tile_bits(int dtype) { return kXTileBytesLog2 - (dtype == GQAOA_C64 ? 3 : 4); }
inline int x_row_bits(int dtype) { return kXRowBytesLog2 - (dtype == GQAOA_C64 ? 3 : 4); }

template <typename T>
struct XC {
    T re, im;
};

template <typename T>
__device__ __forceinline__ XC<T> xmul(XC<T> a, XC<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// (a, b) -> (c a - i s b, c b - i s a)
template <typename T>
__device__ __forceinline__ void xrot(XC<T> &a, XC<T> &b, T c, T s) {
    const XC<T> na{c * a.re + s * b.im, c * a.im - s * b.re};
    const XC<T> nb{c * b.re + s * a.im, c * b.im - s * a.re};
    a = na;
    b = nb;
}

// Butterflies on tile bits [lo, lo + nb) of a tile of 2^tb elements in LDS.
template <typename T>
__device__ __forceinline__ void tile_butterflies(XC<T> *tile, int tb, int lo, int nb, T c, T s) {
    int q = lo;
    const int end = lo + nb;
    for (; q + 1 < end; q += 2) {  // radix 4: bits q and q+1 together
        const int quads = 1 << (tb - 2);
        for (int k = threadIdx.x; k < quads; k += kXThreads) {
            const int lowm = (1 << q) - 1;
            const int i0 = (k & lowm) | ((k & ~lowm) << 2);
            XC<T> v0 = tile[i0], v1 = tile[i0 | (1 << q)], v2 = tile[i0 | (2 << q)], v3 = tile[i0 | (3 << q)];
            xrot(v0, v1, c, s);
            xrot(v2, v3, c, s);
            xrot(v0, v2, c, s);
            xrot(v1, v3, c, s);
            tile[i0] = v0;
            tile[i0 | (1 << q)] = v1;
            tile[i0 | (2 << q)] = v2;
            tile[i0 | (3 << q)] = v3;
        }
        __syncthreads();
    }
    if (q < end) {  // one remaining bit
        const int pairs = 1 << (tb - 1);
        for (int k = threadIdx.x; k < pairs; k += kXThreads) {
            const int lowm = (1 << q) - 1;
            const int i0 = (k & lowm) | ((k & ~lowm) << 1);
            XC<T> a = tile[i0], b = tile[i0 | (1 << q)];
            xrot(a, b, c, s);
            tile[i0] = a;
            tile[i0 | (1 << q)] = b;
        }
        __syncthreads();
    }
}

struct XLowArgs {
    const uint8_t *cost;
    const void *psi_in;
    void *psi_out;
    int n;
    int tile_bits;         // min(n, T)
    const void *lut;       // e^{-i gamma_j k}, 256 entries of complex T
    int mix;               // 0: readout only (no phase, no butterflies, no store)
    int init_uniform;
    double init_amp;
    int target;
    double c, s;           // cos beta_j, sin beta_j
    double *partials;      // [gridDim.x][kXR]
};

template <typename T>
__global__ void __launch_bounds__(kXThreads) x_low_kernel(XLowArgs a) {
    extern __shared__ unsigned char smem[];
    XC<T> *tile = reinterpret_cast<XC<T> *>(smem);
    __shared__ XC<T> lut_s[256];
    __shared__ double red_s[kXR * kXThreads / kWave];
    for (int i = threadIdx.x; i < 256; i += kXThreads) lut_s[i] = reinterpret_cast<const XC<T> *>(a.lut)[i];
    __syncthreads();
    const int tsz = 1 << a.tile_bits;
    const uint64_t ntiles = (1ull << a.n) >> a.tile_bits;
    const XC<T> *src = reinterpret_cast<const XC<T> *>(a.psi_in);
    XC<T> *dst = reinterpret_cast<XC<T> *>(a.psi_out);
    const T c = (T)a.c, s = (T)a.s;
    double aP = 0, aE = 0, aN = 0;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint64_t base = t << a.tile_bits;
        for (int i = threadIdx.x; i < tsz; i += kXThreads) {
            const uint32_t cz = a.cost[base + i];
            XC<T> v = a.init_uniform ? XC<T>{(T)a.init_amp, (T)0} : src[base + i];
            const double pr = (double)v.re * v.re + (double)v.im * v.im;
            aN += pr;
            aE += (double)cz * pr;
            aP += cz == (uint32_t)a.target ? pr : 0.0;
            if (a.mix) tile[i] = xmul(lut_s[cz], v);
        }
        if (!a.mix) continue;  // uniform across the block
        __syncthreads();
        tile_butterflies(tile, a.tile_bits, 0, a.tile_bits, c, s);
        for (int i = threadIdx.x; i < tsz; i += kXThreads) dst[base + i] = tile[i];
        __syncthreads();
    }
    double r[kXR] = {0.0, 0.0, aP, aE, aN, 0.0, 0.0};
    block_sum<kXR, kXThreads>(r, red_s);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < kXR; ++k) a.partials[(size_t)blockIdx.x * kXR + k] = r[k];
}

struct XHighArgs {
    void *psi;
    int n, q0, kbits, cbits;  // qubits q0..q0+kbits-1; 2^cbits consecutive amplitudes per row
    double c, s;
};

template <typename T>
__global__ void __launch_bounds__(kXThreads) x_high_kernel(XHighArgs a) {
    extern __shared__ unsigned char smem[];
    XC<T> *tile = reinterpret_cast<XC<T> *>(smem);
    const int tb = a.cbits + a.kbits;
    const int tsz = 1 << tb;
    const int rest_low_bits = a.q0 - a.cbits;  // bits cbits..q0-1 of z
    const uint64_t ntiles = (1ull << a.n) >> tb;
    XC<T> *psi = reinterpret_cast<XC<T> *>(a.psi);
    const T c = (T)a.c, s = (T)a.s;
    const uint64_t cmask = (1ull << a.cbits) - 1;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint64_t rl = t & ((1ull << rest_low_bits) - 1), rh = t >> rest_low_bits;
        const uint64_t base = (rl << a.cbits) | (rh << (a.q0 + a.kbits));
        for (int i = threadIdx.x; i < tsz; i += kXThreads) {
            const uint64_t z = base | ((uint64_t)i & cmask) | ((uint64_t)(i >> a.cbits) << a.q0);
            tile[i] = psi[z];
        }
        __syncthreads();
        tile_butterflies(tile, tb, a.cbits, a.kbits, c, s);
        for (int i = threadIdx.x; i < tsz; i += kXThreads) {
            const uint64_t z = base | ((uint64_t)i & cmask) | ((uint64_t)(i >> a.cbits) << a.q0);
            psi[z] = tile[i];
        }
        __syncthreads();
    }
}

// ---- host ------------------------------------------------------------------------
struct XPartialFin {
    const double *partials;
    int nblocks;
    double *readout;  // psol, E, norm
};

__global__ void __launch_bounds__(1024) x_finalize_kernel(XPartialFin f) {
    __shared__ double lds[3 * 1024 / kWave];
    double r[3] = {0, 0, 0};
    for (int b = threadIdx.x; b < f.nblocks; b += 1024)
        for (int k = 0; k < 3; ++k) r[k] += f.partials[(size_t)b * kXR + 2 + k];
    block_sum<3, 1024>(r, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) f.readout[k] = r[k];
}

// Workspace: phase LUTs [max(p,1)][256] complex, readouts [p+1][3] doubles,
// block partials [kXMaxBlocks][kXR] doubles (each region 256-byte aligned).
struct XLayout {
    char *lut;
    double *ro, *part;
    size_t bytes;
};

static XLayout x_layout(void *ws, int p, int dtype) {
    const size_t cs = dtype == GQAOA_C64 ? 8 : 16;
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    XLayout L{};
    char *w = reinterpret_cast<char *>(ws);
    size_t off = 0;
    L.lut = w + off;
    off += al((size_t)std::max(p, 1) * 256 * cs);
    L.ro = reinterpret_cast<double *>(w + off);
    off += al(sizeof(double) * 3 * ((size_t)p + 1));
    L.part = reinterpret_cast<double *>(w + off);
    off += al(sizeof(double) * kXR * (size_t)kXMaxBlocks);
    L.bytes = off;
    return L;
}

size_t x_workspace_bytes(int p, int dtype) { return x_layout(nullptr, p, dtype).bytes; }

int run_evolve_x(int n, const uint8_t *cost, int p, const double *beta, const double *gamma, int dtype,
                 int init_uniform, void *psi, int target, double *psol, double *energy, double *norm, void *ws,
                 hipStream_t st) {
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    const size_t cs = dtype == GQAOA_C64 ? 8 : 16;
    const XLayout L = x_layout(ws, p, dtype);
    const int tb = std::min(n, x_tile_bits(dtype));
    const int cbits = x_row_bits(dtype);
    const uint64_t ntiles_low = (1ull << n) >> tb;
    const int blocks = (int)std::min<uint64_t>(ntiles_low, std::min<uint64_t>((uint64_t)dev.num_cus * 8, kXMaxBlocks));
    const size_t smem = cs << tb;
    std::vector<char> tab((size_t)std::max(p, 1) * 256 * cs, 0);
    const double two_pi = 2.0 * M_PI;
    for (int j = 0; j < p; ++j)
        for (int k = 0; k < 256; ++k) {
            const double ang = std::fmod(gamma[j] * (double)k, two_pi);
            if (dtype == GQAOA_C64) {
                float *f = reinterpret_cast<float *>(tab.data()) + 2 * ((size_t)j * 256 + k);
                f[0] = (float)std::cos(ang);
                f[1] = (float)-std::sin(ang);
            } else {
                double *d = reinterpret_cast<double *>(tab.data()) + 2 * ((size_t)j * 256 + k);
                d[0] = std::cos(ang);
                d[1] = -std::sin(ang);
            }
        }
    if (p > 0) GQ_HIP(hipMemcpyAsync(L.lut, tab.data(), (size_t)p * 256 * cs, hipMemcpyHostToDevice, st));
    const double amp0 = 1.0 / std::sqrt((double)(1ull << n));
    // Low pass of round j (mix = 1), or the readout of the final state (mix = 0).
    auto low = [&](int j, bool mix, bool uniform, double c, double sn) -> int {
        XLowArgs a{};
        a.cost = cost;
        a.psi_in = psi;
        a.psi_out = psi;
        a.n = n;
        a.tile_bits = tb;
        a.lut = L.lut + (size_t)(mix ? j : 0) * 256 * cs;
        a.mix = mix ? 1 : 0;
        a.init_uniform = uniform ? 1 : 0;
        a.init_amp = amp0;
        a.target = target;
        a.c = c;
        a.s = sn;
        a.partials = L.part;
        if (dtype == GQAOA_C64)
            hipLaunchKernelGGL(x_low_kernel<float>, dim3(blocks), dim3(kXThreads), smem, st, a);
        else
            hipLaunchKernelGGL(x_low_kernel<double>, dim3(blocks), dim3(kXThreads), smem, st, a);
        GQ_LAUNCH_CHECK();
        XPartialFin f{L.part, blocks, L.ro + 3 * (size_t)j};
        hipLaunchKernelGGL(x_finalize_kernel, dim3(1), dim3(1024), 0, st, f);
        GQ_LAUNCH_CHECK();
        return GQAOA_OK;
    };
    for (int j = 0; j < p; ++j) {
        const double c = std::cos(beta[j]), sn = std::sin(beta[j]);
        ProfScope ps(dtype == GQAOA_C64 ? "x_round_c64" : "x_round_c128", st);
        if ((s = low(j, true, init_uniform && j == 0, c, sn))) return s;
        for (int q0 = tb; q0 < n; q0 += tb - cbits) {
            XHighArgs h{};
            h.psi = psi;
            h.n = n;
            h.q0 = q0;
            h.cbits = cbits;
            h.kbits = std::min(tb - cbits, n - q0);
            h.c = c;
            h.s = sn;
            const int htb = h.cbits + h.kbits;
            const uint64_t nt = (1ull << n) >> htb;
            const int hb = (int)std::min<uint64_t>(nt, (uint64_t)dev.num_cus * 8);
            if (dtype == GQAOA_C64)
                hipLaunchKernelGGL(x_high_kernel<float>, dim3(hb), dim3(kXThreads), cs << htb, st, h);
            else
                hipLaunchKernelGGL(x_high_kernel<double>, dim3(hb), dim3(kXThreads), cs << htb, st, h);
            GQ_LAUNCH_CHECK();
        }
        ps.end();
    }
    if (p == 0 && init_uniform) {
        // the output state is |s>: one low pass with beta = 0 and the phase of
        // gamma = 0 writes it (both are identities) and reads it out
        std::vector<char> id(256 * cs, 0);
        for (int k = 0; k < 256; ++k) {
            if (dtype == GQAOA_C64) reinterpret_cast<float *>(id.data())[2 * k] = 1.0f;
            else reinterpret_cast<double *>(id.data())[2 * k] = 1.0;
        }
        GQ_HIP(hipMemcpyAsync(L.lut, id.data(), id.size(), hipMemcpyHostToDevice, st));
        if ((s = low(0, true, true, 1.0, 0.0))) return s;
    } else if ((s = low(p, false, false, 1.0, 0.0))) {
        return s;
    }
    std::vector<double> out((size_t)3 * (p + 1));
    GQ_HIP(hipMemcpyAsync(out.data(), L.ro, out.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    GQ_HIP(hipStreamSynchronize(st));
    if (prof_on()) prof_collect();
    for (int j = 0; j <= p; ++j) {
        if (psol) psol[j] = out[3 * j];
        if (energy) energy[j] = out[3 * j + 1];
        if (norm) norm[j] = out[3 * j + 2];
    }
    return GQAOA_OK;
}

}  // namespace gqaoa
