// X-QAOA rounds: phase separator plus the transverse-field mixer
// exp(-i beta sum_q X_q) = prod_q exp(-i beta X_q) (Sec. II.B, the "X" rows of
// Table I), streamed from HBM.
//
// exp(-i beta X_q) mixes the amplitude pairs that differ in bit q:
// (a, b) -> (c a - i s b, c b - i s a), c = cos beta, s = sin beta. All
// factors commute, so the qubits of a round can be taken in any grouping
// and order.
//
// Above T qubits (T = 12 for complex64, 11 for complex128: a 32 KiB tile)
// the qubits form groups: group 0 = qubits 0..T-1 (a tile is 2^T consecutive
// amplitudes), then groups of K = 8 qubits (a tile is 2^(T-K) consecutive
// amplitudes, one 128-byte run, times the 2^K values of the group's qubits),
// the last one possibly smaller (its runs are longer). One pass streams the
// state once and applies one group's factors:
//   * each thread holds E = 2^(T-8) amplitudes of a tile in registers and
//     applies the butterflies of the register-resident bits there; the tile
//     is re-distributed through LDS to bring the next bits into registers
//     (two to four exchanges per pass, never a butterfly in LDS);
//   * the group order alternates between rounds (0..g-1, then g-1..0, ...),
//     so the last pass of a round and the first of the next touch the same
//     group and are fused: mixers of round j, readout of the state after
//     round j, phase of round j+1, mixers of round j+1. A round then costs
//     g - 1 passes (two at n = 28, complex64) instead of g.
// The phase and readouts need C(z) in tile order: group 0 reads the cost
// table itself, the last group a tile-ordered copy built once per call.
// Up to T qubits the whole state is one tile, evolved by a simple LDS kernel.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace gqaoa {

constexpr int kXThreads = 256;
constexpr int kXThreadBits = 8;
constexpr int kXTileBytesLog2 = 15;  // 32 KiB of LDS per tile
constexpr int kXGroupBits = 8;       // qubits of a full high group
constexpr int kXMaxBlocks = 8192;
constexpr int kXR = 7;  // partial sums per block of the small-n kernel
constexpr int kXMaxChunks = 6;

inline int x_tile_bits(int dtype) { return kXTileBytesLog2 - (dtype == GQAOA_C64 ? 3 : 4); }

template <typename T>
struct XCfg;
template <>
struct XCfg<float> {
    static constexpr int TB = 12, R = 4;
};
template <>
struct XCfg<double> {
    static constexpr int TB = 11, R = 3;
};

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

// ---- streaming passes for n > T -------------------------------------------------
// Register layout rb: thread t holds tile elements e(t, i) for i < E, with
// bits [rb, rb + R) of e equal to i and the other bits taken from t in order.
__device__ __forceinline__ int x_elem(int t, int i, int rb, int R) {
    return (t & ((1 << rb) - 1)) | (i << rb) | ((t >> rb) << (rb + R));
}
// LDS slot of tile element e: one pad slot per 16 elements spreads the
// strided layouts over the banks.
__device__ __forceinline__ int x_phys(int e) { return e + (e >> 4); }

// The register chunks of one group's mixers: chunk k holds tile bits
// [rb[k], rb[k] + R) in registers and applies the qubits of mask[k].
struct XPlan {
    int nchunks;
    int rb[kXMaxChunks];
    int mask[kXMaxChunks];
};

enum : int {
    XOP_PRE = 1,     // readout, then phase lut_a, before mixer A (first pass)
    XOP_MIX_A = 2,   // mixer A (c_a, s_a)
    XOP_MID = 4,     // after mixer A: readout, phase lut_b, mixer B (c_b, s_b)
    XOP_POST = 8,    // readout after the mixers (last pass)
};

struct XPassArgs {
    void *psi;
    const uint8_t *cost;   // C in tile order: tile t, element e at (t << T) + e
    int n, mlo, q0;        // tile bits [0, mlo) = z bits [0, mlo); [mlo, T) = z bits [q0, ...)
    int contig;            // tile bits that are consecutive in z (T for group 0, else mlo)
    uint64_t ntiles;
    XPlan plan;
    int ops;
    int init_uniform;
    double init_amp;
    int target;
    const void *lut_a, *lut_b;
    double ca, sa, cb, sb;
    double *partials;      // [gridDim.x][3]: P_sol, E, norm of the pass's readout
};

template <typename T>
__device__ __forceinline__ XC<T> x_load(const XC<T> *p) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
    return {v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void x_store(XC<T> a, XC<T> *p) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(v2{a.re, a.im}, reinterpret_cast<v2 *>(p));
}

template <typename T, int R>
__device__ __forceinline__ void x_exchange(XC<T> (&v)[1 << R], XC<T> *lds, int from, int to) {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) lds[x_phys(x_elem(t, i, from, R))] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) v[i] = lds[x_phys(x_elem(t, i, to, R))];
    __syncthreads();
}

template <typename T, int R>
__device__ __forceinline__ void x_stages(XC<T> (&v)[1 << R], int mask, T c, T s) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!((mask >> r) & 1)) continue;  // uniform across the block
#pragma unroll
        for (int i = 0; i < (1 << R); ++i)
            if (!((i >> r) & 1)) xrot(v[i], v[i | (1 << r)], c, s);
    }
}

// Mixers of one group, chunk by chunk, forward (from rb[0]) or backward (from
// the last chunk); rb is the register layout on entry and on exit.
template <typename T, int R>
__device__ __forceinline__ void x_mix(XC<T> (&v)[1 << R], XC<T> *lds, const XPlan &pl, bool forward, int &rb,
                                      T c, T s) {
    for (int k = 0; k < pl.nchunks; ++k) {
        const int kk = forward ? k : pl.nchunks - 1 - k;
        if (pl.rb[kk] != rb) {
            x_exchange<T, R>(v, lds, rb, pl.rb[kk]);
            rb = pl.rb[kk];
        }
        x_stages<T, R>(v, pl.mask[kk], c, s);
    }
}

// Readouts of one tile's register values: sums in the state precision within
// the tile, float64 across tiles.
template <typename T, int R>
__device__ __forceinline__ void x_readout(const XC<T> (&v)[1 << R], const uint32_t (&cz)[1 << R], double &aP,
                                          double &aE, double &aN, int target) {
    T sP = 0, sE = 0, sN = 0;
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        const T pr = v[i].re * v[i].re + v[i].im * v[i].im;
        sN += pr;
        sE += (T)cz[i] * pr;
        sP += cz[i] == (uint32_t)target ? pr : T(0);
    }
    aP += (double)sP;
    aE += (double)sE;
    aN += (double)sN;
}

// OPS: the XOP_* flags of the pass, fixed at compile time so that a pass
// that only mixes carries no readout, cost or phase state.
template <typename T, int OPS>
__global__ void __launch_bounds__(kXThreads) x_pass_kernel(XPassArgs a) {
    constexpr int TB = XCfg<T>::TB, R = XCfg<T>::R, E = 1 << R;
    static_assert(TB - R == kXThreadBits, "one tile per block of 256 threads");
    extern __shared__ unsigned char smem[];
    XC<T> *lds = reinterpret_cast<XC<T> *>(smem);
    __shared__ XC<T> lut_s[2][256];
    __shared__ double red_s[3 * kXThreads / kWave];
    for (int i = threadIdx.x; i < 256; i += kXThreads) {
        if constexpr ((OPS & XOP_PRE) != 0) lut_s[0][i] = reinterpret_cast<const XC<T> *>(a.lut_a)[i];
        if constexpr ((OPS & XOP_MID) != 0) lut_s[1][i] = reinterpret_cast<const XC<T> *>(a.lut_b)[i];
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int rb0 = TB - R;
    const T ca = (T)a.ca, sa = (T)a.sa, cb = (T)a.cb, sb = (T)a.sb;
    constexpr bool store = (OPS & (XOP_MIX_A | XOP_MID)) != 0;
    XC<T> *psi = reinterpret_cast<XC<T> *>(a.psi);
    const int lowbits = a.q0 - a.mlo;         // z bits mlo..q0-1 come from the tile index
    const int hishift = a.q0 + TB - a.mlo;    // z bits above the group
    const uint32_t cmask = (1u << a.mlo) - 1u;
    double aP = 0.0, aE = 0.0, aN = 0.0;
    // z of tile element e is base | zmap(e); zmap is a bit placement, so for
    // e = (thread part) | (register part) it splits into a per-thread offset
    // and a per-register offset that is uniform across the block.
    auto zmap = [&](uint32_t e) -> uint64_t { return (uint64_t)(e & cmask) | ((uint64_t)(e >> a.mlo) << a.q0); };
    const uint64_t zt0 = zmap((uint32_t)x_elem(t, 0, rb0, R));
    auto tile_base = [&](uint64_t tile) -> uint64_t {
        return ((tile & ((1ull << lowbits) - 1)) << a.mlo) | ((tile >> lowbits) << hishift);
    };
    auto load_tile = [&](uint64_t tile, XC<T>(&w)[E]) {
        const XC<T> *src = psi + tile_base(tile) + zt0;
#pragma unroll
        for (int i = 0; i < E; ++i) w[i] = x_load(src + zmap((uint32_t)i << rb0));
    };
    XC<T> v[E];
    if constexpr (OPS == XOP_MIX_A) {
        // Mixing only: light enough in registers to keep the next tile's
        // loads in flight while this tile is mixed and stored.
        XC<T> nxt[E];
        uint64_t tile = blockIdx.x;
        if (tile < a.ntiles) load_tile(tile, nxt);
        for (; tile < a.ntiles; tile += gridDim.x) {
#pragma unroll
            for (int i = 0; i < E; ++i) v[i] = nxt[i];
            if (tile + gridDim.x < a.ntiles) load_tile(tile + gridDim.x, nxt);
            int rb = rb0;
            x_mix<T, R>(v, lds, a.plan, true, rb, ca, sa);
            if ((int)sizeof(XC<T>) << (rb < a.contig ? rb : a.contig) < 128) {
                x_exchange<T, R>(v, lds, rb, rb0);
                rb = rb0;
            }
            XC<T> *dst = psi + tile_base(tile) + zmap((uint32_t)x_elem(t, 0, rb, R));
#pragma unroll
            for (int i = 0; i < E; ++i) x_store(v[i], dst + zmap((uint32_t)i << rb));
        }
        return;
    }
    for (uint64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        XC<T> *tp = psi + tile_base(tile);
        const uint8_t *ct = a.cost + (tile << TB);
        uint32_t cz[E];
        // C of this tile's elements in register layout rb (read where used)
        auto load_cost = [&](int rb) {
            const uint8_t *cc = ct + x_elem(t, 0, rb, R);
#pragma unroll
            for (int i = 0; i < E; ++i) cz[i] = cc[i << rb];
        };
        if (a.init_uniform) {
#pragma unroll
            for (int i = 0; i < E; ++i) v[i] = XC<T>{(T)a.init_amp, (T)0};
        } else {
            load_tile(tile, v);
        }
        int rb = rb0;
        if constexpr ((OPS & XOP_PRE) != 0) {
            load_cost(rb);
            x_readout<T, R>(v, cz, aP, aE, aN, a.target);
#pragma unroll
            for (int i = 0; i < E; ++i) v[i] = xmul(lut_s[0][cz[i]], v[i]);
        }
        if constexpr ((OPS & XOP_MIX_A) != 0) x_mix<T, R>(v, lds, a.plan, true, rb, ca, sa);
        if constexpr ((OPS & XOP_MID) != 0) {
            load_cost(rb);
            x_readout<T, R>(v, cz, aP, aE, aN, a.target);
#pragma unroll
            for (int i = 0; i < E; ++i) v[i] = xmul(lut_s[1][cz[i]], v[i]);
            x_mix<T, R>(v, lds, a.plan, false, rb, cb, sb);
        }
        if constexpr ((OPS & XOP_POST) != 0) {
            load_cost(rb);
            x_readout<T, R>(v, cz, aP, aE, aN, a.target);
        }
        if constexpr (store) {
            // store from a layout whose lanes cover runs of >= 128 bytes
            if ((int)sizeof(XC<T>) << (rb < a.contig ? rb : a.contig) < 128) {
                x_exchange<T, R>(v, lds, rb, rb0);
                rb = rb0;
            }
            XC<T> *dst = tp + zmap((uint32_t)x_elem(t, 0, rb, R));
#pragma unroll
            for (int i = 0; i < E; ++i) x_store(v[i], dst + zmap((uint32_t)i << rb));
        }
    }
    if constexpr ((OPS & (XOP_PRE | XOP_MID | XOP_POST)) != 0) {
        double r[3] = {aP, aE, aN};
        block_sum<3, kXThreads>(r, red_s);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < 3; ++k) a.partials[(size_t)blockIdx.x * 3 + k] = r[k];
    }
}

// Tile-ordered copy of the cost table for one group: out[(t << T) + e] = C(z(t, e)).
__global__ void __launch_bounds__(256) x_cost_tiles_kernel(const uint8_t *__restrict__ cost, uint8_t *__restrict__ out,
                                                          int tb, int mlo, int q0, uint64_t total) {
    const int lowbits = q0 - mlo, hishift = q0 + tb - mlo;
    const uint32_t cmask = (1u << mlo) - 1u;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t tile = k >> tb;
        const uint32_t e = (uint32_t)(k & ((1ull << tb) - 1));
        const uint64_t base = ((tile & ((1ull << lowbits) - 1)) << mlo) | ((tile >> lowbits) << hishift);
        out[k] = cost[base | (e & cmask) | ((uint64_t)(e >> mlo) << q0)];
    }
}

// ---- host ------------------------------------------------------------------------
struct XPartialFin {
    const double *partials;
    int nblocks, stride, off;  // block b's P_sol, E, norm at partials[b*stride + off + 0..2]
    double *readout;           // psol, E, norm
};

__global__ void __launch_bounds__(1024) x_finalize_kernel(XPartialFin f) {
    __shared__ double lds[3 * 1024 / kWave];
    double r[3] = {0, 0, 0};
    for (int b = threadIdx.x; b < f.nblocks; b += 1024)
        for (int k = 0; k < 3; ++k) r[k] += f.partials[(size_t)b * f.stride + f.off + k];
    block_sum<3, 1024>(r, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) f.readout[k] = r[k];
}

// Workspace: phase LUTs [max(p,1)][256] complex, readouts [p+1][3] doubles,
// block partials [kXMaxBlocks][kXR] doubles, and for n > T the tile-ordered
// cost table of the last group (2^n bytes); each region 256-byte aligned.
struct XLayout {
    char *lut;
    double *ro, *part;
    uint8_t *cost_t;
    size_t bytes;
};

static XLayout x_layout(void *ws, int n, int p, int dtype) {
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
    L.cost_t = reinterpret_cast<uint8_t *>(w + off);
    if (n > x_tile_bits(dtype)) off += al(size_t(1) << n);
    L.bytes = off;
    return L;
}

size_t x_workspace_bytes(int n, int p, int dtype) { return x_layout(nullptr, n, p, dtype).bytes; }

template <typename T>
static int launch_pass(int ops, int blocks, size_t smem, hipStream_t st, const XPassArgs &a) {
    switch (ops) {
        case XOP_MIX_A:
            hipLaunchKernelGGL((x_pass_kernel<T, XOP_MIX_A>), dim3(blocks), dim3(kXThreads), smem, st, a);
            break;
        case XOP_PRE | XOP_MIX_A:
            hipLaunchKernelGGL((x_pass_kernel<T, XOP_PRE | XOP_MIX_A>), dim3(blocks), dim3(kXThreads), smem, st, a);
            break;
        case XOP_MIX_A | XOP_MID:
            hipLaunchKernelGGL((x_pass_kernel<T, XOP_MIX_A | XOP_MID>), dim3(blocks), dim3(kXThreads), smem, st, a);
            break;
        case XOP_MIX_A | XOP_POST:
            hipLaunchKernelGGL((x_pass_kernel<T, XOP_MIX_A | XOP_POST>), dim3(blocks), dim3(kXThreads), smem, st, a);
            break;
        case XOP_POST:
            hipLaunchKernelGGL((x_pass_kernel<T, XOP_POST>), dim3(blocks), dim3(kXThreads), smem, st, a);
            break;
        case XOP_PRE | XOP_MIX_A | XOP_POST:
            hipLaunchKernelGGL((x_pass_kernel<T, XOP_PRE | XOP_MIX_A | XOP_POST>), dim3(blocks), dim3(kXThreads), smem,
                               st, a);
            break;
        default:
            return fail(GQAOA_EINVAL, "internal: X pass operations %d", ops);
    }
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

// One group of qubits for the streaming passes (n > T).
struct XGroup {
    int mlo, q0;  // tile bits [mlo, T) are qubits q0 .. q0 + T - mlo - 1
    XPlan plan;
};

static XGroup x_group(int mlo, int q0, int TB, int R) {
    XGroup g{};
    g.mlo = mlo;
    g.q0 = q0;
    uint32_t done = 0;
    const uint32_t want = ((1u << TB) - 1u) & ~((1u << mlo) - 1u);
    int rb = TB - R;
    for (;;) {
        int m = 0;
        for (int r = 0; r < R; ++r) {
            const int bit = rb + r;
            if (bit >= mlo && bit < TB && !((done >> bit) & 1u)) {
                m |= 1 << r;
                done |= 1u << bit;
            }
        }
        g.plan.rb[g.plan.nchunks] = rb;
        g.plan.mask[g.plan.nchunks] = m;
        ++g.plan.nchunks;
        if (done == want) break;
        rb = std::max(mlo, rb - R);
    }
    return g;
}

int run_evolve_x(int n, const uint8_t *cost, int p, const double *beta, const double *gamma, int dtype,
                 int init_uniform, void *psi, int target, double *psol, double *energy, double *norm, void *ws,
                 hipStream_t st) {
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    const size_t cs = dtype == GQAOA_C64 ? 8 : 16;
    const XLayout L = x_layout(ws, n, p, dtype);
    const int TB = x_tile_bits(dtype);
    const int R = dtype == GQAOA_C64 ? XCfg<float>::R : XCfg<double>::R;
    const char *prof = dtype == GQAOA_C64 ? "x_pass_c64" : "x_pass_c128";
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
    if (p == 0) {  // the identity phase, for the p = 0 readout pass
        for (int k = 0; k < 256; ++k) {
            if (dtype == GQAOA_C64) reinterpret_cast<float *>(tab.data())[2 * k] = 1.0f;
            else reinterpret_cast<double *>(tab.data())[2 * k] = 1.0;
        }
    }
    GQ_HIP(hipMemcpyAsync(L.lut, tab.data(), tab.size(), hipMemcpyHostToDevice, st));
    const double amp0 = 1.0 / std::sqrt((double)(1ull << n));
    auto lut = [&](int j) -> const void * { return L.lut + (size_t)j * 256 * cs; };  // phase of round j + 1
    auto finalize = [&](int nblocks, int stride, int off, int j) -> int {
        XPartialFin f{L.part, nblocks, stride, off, L.ro + 3 * (size_t)j};
        hipLaunchKernelGGL(x_finalize_kernel, dim3(1), dim3(1024), 0, st, f);
        GQ_LAUNCH_CHECK();
        return GQAOA_OK;
    };

    if (n <= TB) {
        // the whole state is one tile: one LDS pass per round, then a readout pass
        const size_t smem = cs << n;
        auto low = [&](int j, bool mix, bool uniform, double c, double sn) -> int {
            XLowArgs a{};
            a.cost = cost;
            a.psi_in = psi;
            a.psi_out = psi;
            a.n = n;
            a.tile_bits = n;
            a.lut = lut(mix ? j : 0);
            a.mix = mix ? 1 : 0;
            a.init_uniform = uniform ? 1 : 0;
            a.init_amp = amp0;
            a.target = target;
            a.c = c;
            a.s = sn;
            a.partials = L.part;
            ProfScope ps(prof, st);
            if (dtype == GQAOA_C64)
                hipLaunchKernelGGL(x_low_kernel<float>, dim3(1), dim3(kXThreads), smem, st, a);
            else
                hipLaunchKernelGGL(x_low_kernel<double>, dim3(1), dim3(kXThreads), smem, st, a);
            ps.end();
            GQ_LAUNCH_CHECK();
            return finalize(1, kXR, 2, j);
        };
        for (int j = 0; j < p; ++j)
            if ((s = low(j, true, init_uniform && j == 0, std::cos(beta[j]), std::sin(beta[j])))) return s;
        // p = 0 from |s>: a mixing pass with identity phase and beta = 0 writes |s>
        if (p == 0 && init_uniform) s = low(0, true, true, 1.0, 0.0);
        else s = low(p, false, false, 1.0, 0.0);
        if (s) return s;
    } else {
        // groups: qubits [0, T), then runs of kXGroupBits, the last one shorter
        std::vector<XGroup> groups;
        groups.push_back(x_group(0, 0, TB, R));
        for (int q0 = TB; q0 < n; q0 += kXGroupBits) {
            const int kb = std::min(kXGroupBits, n - q0);
            groups.push_back(x_group(TB - kb, q0, TB, R));
        }
        const int G = (int)groups.size();
        const XGroup &last = groups[G - 1];
        const uint64_t total = 1ull << n;
        const uint64_t ntiles = total >> TB;
        // 32 blocks per CU (about 4 resident at once by LDS): at n = 28 the passes
        // ran 3% faster per round than with 8 per CU, and no faster with more
        const int blocks = (int)std::min<uint64_t>(ntiles, std::min<uint64_t>((uint64_t)dev.num_cus * 32, kXMaxBlocks));
        {
            const int cb = (int)std::min<uint64_t>((total + 255) / 256, (uint64_t)dev.num_cus * 16);
            hipLaunchKernelGGL(x_cost_tiles_kernel, dim3(cb), dim3(256), 0, st, cost, L.cost_t, TB, last.mlo, last.q0,
                               total);
            GQ_LAUNCH_CHECK();
        }
        const size_t smem = (cs << TB) + (cs << TB) / 16;
        auto pass = [&](int gi, int ops, bool uniform, int ja, int jb, int readout_j) -> int {
            const XGroup &gr = groups[gi];
            XPassArgs a{};
            a.psi = psi;
            a.cost = gi == 0 ? cost : L.cost_t;
            a.n = n;
            a.mlo = gr.mlo;
            a.q0 = gr.q0;
            a.contig = gi == 0 ? TB : gr.mlo;
            a.ntiles = ntiles;
            a.plan = gr.plan;
            a.ops = ops;
            a.init_uniform = uniform ? 1 : 0;
            a.init_amp = amp0;
            a.target = target;
            if (ops & XOP_PRE) a.lut_a = lut(ja);          // phase of round ja + 1
            if (ops & XOP_MID) a.lut_b = lut(jb);          // phase of round jb + 1
            a.ca = 1.0;  // p = 0: the mixer of the |s> writing pass is the identity
            if ((ops & XOP_MIX_A) && ja < p) {
                a.ca = std::cos(beta[ja]);
                a.sa = std::sin(beta[ja]);
            }
            if (ops & XOP_MID) {
                a.cb = std::cos(beta[jb]);
                a.sb = std::sin(beta[jb]);
            }
            a.partials = L.part;
            ProfScope ps(prof, st);
            const int rc = dtype == GQAOA_C64 ? launch_pass<float>(ops, blocks, smem, st, a)
                                              : launch_pass<double>(ops, blocks, smem, st, a);
            ps.end();
            if (rc) return rc;
            return readout_j >= 0 ? finalize(blocks, 3, 0, readout_j) : GQAOA_OK;
        };
        if (p == 0) {
            // readout of the initial state (written as |s> when init_uniform):
            // a pass with the identity phase and no mixer on group 0
            if (init_uniform) {
                if ((s = pass(0, XOP_PRE | XOP_MIX_A, true, 0, 0, 0))) return s;
            } else if ((s = pass(0, XOP_POST, false, 0, 0, 0))) {
                return s;
            }
        }
        // Rounds are 0-based here: round j applies phase j and mixer j.
        for (int j = 0; j < p; ++j) {
            const bool fwd = (j % 2) == 0;
            for (int k = 0; k < G; ++k) {
                if (k == 0 && j > 0) continue;  // fused into the previous round's last pass
                const int gi = fwd ? k : G - 1 - k;
                int ops = XOP_MIX_A, readout = -1, jb = 0;
                if (j == 0 && k == 0) {
                    ops |= XOP_PRE;
                    readout = 0;
                }
                if (k == G - 1) {
                    if (j + 1 < p) {
                        ops |= XOP_MID;
                        jb = j + 1;
                        readout = j + 1;
                    } else {
                        ops |= XOP_POST;
                        readout = p;
                    }
                }
                if ((s = pass(gi, ops, init_uniform && j == 0 && k == 0, j, jb, readout))) return s;
            }
        }
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
