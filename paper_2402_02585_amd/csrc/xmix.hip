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
// amplitudes), then groups of K = 8 qubits, the last one possibly smaller.
// A high group's tile is twice as large, 2^(T+1) amplitudes (64 KiB): runs of
// 2^(T+1-K) consecutive amplitudes (256 bytes) times the 2^K values of the
// group's qubits: a high group's passes on them ran 15% faster than on the
// 128-byte runs of 32 KiB tiles (n = 28, complex64), and the GPU holds two
// such tiles per CU in LDS. One
// pass streams the state once and applies one group's factors:
//   * each thread holds E = 2^R amplitudes of a tile in registers (R = 4
//     for complex64, 3 for complex128; 256 threads per group-0 tile, 512 per
//     high-group tile) and applies the butterflies of the register-resident
//     bits there; the tile is re-distributed through LDS to bring the next
//     bits into registers (one to four exchanges per pass, never a butterfly
//     in LDS). For group 0 and the full groups the chunk plan is a template
//     parameter, so the exchanges use fixed LDS offsets and the stages run
//     without branches;
//   * the group order alternates between rounds (o_0..o_{g-1}, then back),
//     so the last pass of a round and the first of the next touch the same
//     group and are fused: mixers of round j, readout of the state after
//     round j, phase of round j+1, mixers of round j+1. A round then costs
//     g - 1 passes (two at n = 28, complex64) instead of g. With three or
//     more groups, group 0 (the most qubits, contiguous tiles) goes second,
//     so it takes a mixing-only pass and the fused passes, which apply two
//     mixers, fall on the high groups.
// The phase and readouts need C(z) in tile order: group 0 reads the cost
// table itself, the other two groups that take the fused passes read
// tile-ordered copies built once per call. After a group's forward mixers
// each thread's costs are consecutive in either, so the streaming passes
// read them with one vector load per tile. Group 0's passes run on a grid of
// 32 blocks per CU, each block keeping its next tile's loads in flight while
// it mixes the current one; the high groups' passes give each block one
// tile. The first pass of a call starts in the cost-copy layout (|s> is the
// same in every layout) and runs its mixers backward.
// Up to T qubits the whole state is one tile, evolved by a simple LDS kernel.
#include "internal.h"
#include "xplan.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace gqaoa {

constexpr int kXThreads = 256;       // blocks of the group-0 and small-state kernels
constexpr int kXMaxRb = 9;           // largest register layout of a pass (TB - R of the high-group tiles)
constexpr int kXTileBytesLog2 = 15;  // 32 KiB group-0 tiles; the high groups' tiles are twice that
constexpr int kXGroupBits = 8;       // qubits of a full high group
constexpr int kXMaxBlocks = 65536;
constexpr int kXR = 7;  // partial sums per block of the small-n kernel

inline int x_tile_bits(int dtype) { return kXTileBytesLog2 - (dtype == GQAOA_C64 ? 3 : 4); }

template <typename T>
struct XCfg;
// TB: tile bits of group 0 (256 threads of 2^R registers); TBW = TB + 1: tile
// bits of the high groups (512 threads), whose rows are then 256 bytes long.
template <>
struct XCfg<float> {
    static constexpr int TB = 12, TBW = 13, R = 4;
};
template <>
struct XCfg<double> {
    static constexpr int TB = 11, TBW = 12, R = 3;
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

enum : int {
    XOP_PRE = 1,     // readout, then phase lut_a, before mixer A (first pass)
    XOP_MIX_A = 2,   // mixer A (c_a, s_a)
    XOP_MID = 4,     // after mixer A: readout, phase lut_b, mixer B (c_b, s_b)
    XOP_POST = 8,    // readout after the mixers (last pass)
};

struct XPassArgs {
    void *psi;
    const uint8_t *cost;   // C of tile t at (t << T), in the order after the group's forward mixers
    const uint8_t *cost_z; // the cost table (z order), for the readout-only pass
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

// Tile element e sits in LDS slot e + (e >> 4): one pad slot per 16
// elements spreads the strided layouts over the banks. The slot of register
// element i of thread t in layout rb splits into a per-thread part and a
// per-element part: the bits of the element index that come from t and from
// i are disjoint, so the pad term e >> 4 splits too.
// With rb fixed at compile time the element part is an instruction's
// immediate offset.
template <int R>
__device__ __forceinline__ int x_slot_t(int t, int rb) {
    const int tp = (t & ((1 << rb) - 1)) | ((t >> rb) << (rb + R));
    return tp + (tp >> 4);
}
constexpr int x_slot_i(int i, int rb) { return (i << rb) + ((i << rb) >> 4); }

template <typename T>
struct XV2 {
    typedef T type __attribute__((ext_vector_type(2)));
};

// Write (PUT) or read the register elements in layout RB.
template <typename T, int R, bool PUT, int RB>
__device__ __forceinline__ void x_lds_at(XC<T> (&v)[1 << R], XC<T> *lds) {
    typedef typename XV2<T>::type v2;
    v2 *p = reinterpret_cast<v2 *>(lds) + x_slot_t<R>(threadIdx.x, RB);
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
        if constexpr (PUT) {
            p[x_slot_i(i, RB)] = v2{v[i].re, v[i].im};
        } else {
            const v2 w = p[x_slot_i(i, RB)];
            v[i] = XC<T>{w.x, w.y};
        }
    }
}
// The same for the runtime rb of a plan (uniform across the block, 0 <= rb <= T - R).
template <typename T, int R, bool PUT, int RB = 0>
__device__ __forceinline__ void x_lds_move(XC<T> (&v)[1 << R], XC<T> *lds, int rb) {
    if constexpr (RB <= kXMaxRb) {
        if (rb == RB) x_lds_at<T, R, PUT, RB>(v, lds);
        else x_lds_move<T, R, PUT, RB + 1>(v, lds, rb);
    }
}

template <typename T, int R>
__device__ __forceinline__ void x_exchange(XC<T> (&v)[1 << R], XC<T> *lds, int from, int to) {
    x_lds_move<T, R, true>(v, lds, from);
    __syncthreads();
    x_lds_move<T, R, false>(v, lds, to);
    __syncthreads();
}
template <typename T, int R, int FROM, int TO>
__device__ __forceinline__ void x_exchange_c(XC<T> (&v)[1 << R], XC<T> *lds) {
    x_lds_at<T, R, true, FROM>(v, lds);
    __syncthreads();
    x_lds_at<T, R, false, TO>(v, lds);
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ T x_fma(T a, T b, T c);
template <>
__device__ __forceinline__ float x_fma<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <>
__device__ __forceinline__ double x_fma<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

// xrot as one multiply and one accumulate per output, with -s in a register
// of its own, so that every instruction is a two-operand form on vector
// registers (these issue at twice the rate of forms with a scalar operand).
template <typename T>
__device__ __forceinline__ void xrot2(XC<T> &a, XC<T> &b, T c, T s, T ns) {
    const XC<T> na{x_fma(s, b.im, c * a.re), x_fma(ns, b.re, c * a.im)};
    const XC<T> nb{x_fma(s, a.im, c * b.re), x_fma(ns, a.re, c * b.im)};
    a = na;
    b = nb;
}

// cos and sin of a mixer angle and -sin, in vector registers.
template <typename T>
struct XF {
    T c, s, ns;
};
template <typename T>
__device__ __forceinline__ XF<T> x_factors(T c, T s) {
    T cv = c, sv = s, nsv = -s;
    asm volatile("" : "+v"(cv), "+v"(sv), "+v"(nsv));
    return XF<T>{cv, sv, nsv};
}

template <typename T, int R>
__device__ __forceinline__ void x_stages(XC<T> (&v)[1 << R], int mask, const XF<T> &f) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!((mask >> r) & 1)) continue;  // uniform across the block
#pragma unroll
        for (int i = 0; i < (1 << R); ++i)
            if (!((i >> r) & 1)) xrot2(v[i], v[i | (1 << r)], f.c, f.s, f.ns);
    }
}

// Mixers of one group, chunk by chunk, forward (from rb[0]) or backward (from
// the last chunk); rb is the register layout on entry and on exit.
template <typename T, int R>
__device__ __forceinline__ void x_mix(XC<T> (&v)[1 << R], XC<T> *lds, const XPlan &pl, bool forward, int &rb,
                                      const XF<T> &f) {
    for (int k = 0; k < pl.nchunks; ++k) {
        const int kk = forward ? k : pl.nchunks - 1 - k;
        if (pl.rb[kk] != rb) {
            x_exchange<T, R>(v, lds, rb, pl.rb[kk]);
            rb = pl.rb[kk];
        }
        x_stages<T, R>(v, pl.mask[kk], f);
    }
}

// The same with the group's plan fixed at compile time (group on tile bits
// [MLO, TB)): exchanges at fixed layouts, no branches between stages.
template <typename T, int R, int MASK>
__device__ __forceinline__ void x_stages_c(XC<T> (&v)[1 << R], const XF<T> &f) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if ((MASK >> r) & 1) {
#pragma unroll
            for (int i = 0; i < (1 << R); ++i)
                if (!((i >> r) & 1)) xrot2(v[i], v[i | (1 << r)], f.c, f.s, f.ns);
        }
    }
}
template <typename T, int R, int TB, int PLAN, bool FWD, int K = 0>
__device__ __forceinline__ void x_mix_c(XC<T> (&v)[1 << R], XC<T> *lds, const XF<T> &f) {
    constexpr XPlan P = x_plan_id(TB, R, PLAN);
    if constexpr (K < P.nchunks) {
        constexpr int kk = FWD ? K : P.nchunks - 1 - K;
        constexpr int from = K == 0 ? (FWD ? P.rb[0] : P.rb[P.nchunks - 1])
                                    : (FWD ? P.rb[K - 1] : P.rb[P.nchunks - K]);
        if constexpr (P.rb[kk] != from) x_exchange_c<T, R, from, P.rb[kk]>(v, lds);
        x_stages_c<T, R, P.mask[kk]>(v, f);
        x_mix_c<T, R, TB, PLAN, FWD, K + 1>(v, lds, f);
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

// The 2^R cost bytes of one thread's elements in the layout after a group's
// forward mixers (register bits at the plan's last chunk): consecutive in
// the cost array for group 0 (z order, last chunk at bit 0) and in the last
// group's tile-ordered copy, which is written in that order.
template <int R>
struct XCostVec {
    typedef uint32_t type __attribute__((ext_vector_type((1 << R) / 4)));
};
template <int R>
__device__ __forceinline__ typename XCostVec<R>::type x_load_costs(const uint8_t *ct) {
    return *reinterpret_cast<const typename XCostVec<R>::type *>(ct + ((size_t)threadIdx.x << R));
}
template <int R>
__device__ __forceinline__ void x_unpack_costs(const typename XCostVec<R>::type &w, uint32_t (&cz)[1 << R]) {
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) cz[i] = (w[i >> 2] >> (8 * (i & 3))) & 0xFFu;
}

// OPS: the XOP_* flags of the pass, fixed at compile time so that a pass
// that only mixes carries no readout, cost or phase state. TB: the tile bits
// (group 0's tiles or the high groups' twice larger ones), one tile per
// 2^(TB - R) threads. MLO >= 0: the group is on tile bits [MLO, TB) and its
// plan is fixed at compile time (group 0 and the full groups of 8 qubits);
// MLO = -1: any group, from the plan in the arguments.
template <typename T, int OPS, int MLO, int TB>
__global__ void __launch_bounds__(1 << (TB - XCfg<T>::R)) x_pass_kernel(XPassArgs a) {
    constexpr int R = XCfg<T>::R, E = 1 << R, kThreads = 1 << (TB - R);
    static_assert(TB - R <= kXMaxRb, "register layouts up to kXMaxRb");
    static_assert(E >= 8, "costs are read as whole 32-bit words");
    // Passes that start with the mixers always read the state and keep the
    // next tile's loads (and its costs, when the pass reads them) in flight
    // while this tile is mixed and stored.
    constexpr bool kStream = (OPS & XOP_MIX_A) != 0 && (OPS & XOP_PRE) == 0;
    constexpr bool kReadout = (OPS & (XOP_PRE | XOP_MID | XOP_POST)) != 0;
    constexpr int kPlan = OPS == XOP_MIX_A && MLO == 0 ? kXPlanMix0 : MLO >= 0 ? MLO : 0;
    constexpr XPlan kP = x_plan_id(TB, R, kPlan);
    extern __shared__ __align__(16) unsigned char smem[];
    XC<T> *lds = reinterpret_cast<XC<T> *>(smem);
    __shared__ XC<T> lut_s[2][256];
    __shared__ double red_s[3 * kThreads / kWave];
    for (int i = threadIdx.x; i < 256; i += kThreads) {
        if constexpr ((OPS & XOP_PRE) != 0) lut_s[0][i] = reinterpret_cast<const XC<T> *>(a.lut_a)[i];
        if constexpr ((OPS & XOP_MID) != 0) lut_s[1][i] = reinterpret_cast<const XC<T> *>(a.lut_b)[i];
    }
    __syncthreads();
    const int t = threadIdx.x;
    constexpr int rb0 = TB - R;
    constexpr bool store = (OPS & (XOP_MIX_A | XOP_MID)) != 0;
    XC<T> *psi = reinterpret_cast<XC<T> *>(a.psi);
    const int mlo = MLO >= 0 ? MLO : a.mlo;
    const int contig = MLO == 0 ? TB : MLO > 0 ? MLO : a.contig;
    const int lowbits = a.q0 - mlo;         // z bits mlo..q0-1 come from the tile index
    const int hishift = a.q0 + TB - mlo;    // z bits above the group
    const uint32_t cmask = (1u << mlo) - 1u;
    double aP = 0.0, aE = 0.0, aN = 0.0;
    // z of tile element e is base | zmap(e); zmap is a bit placement, so for
    // e = (thread part) | (register part) it splits into a per-thread offset
    // and a per-register offset that is uniform across the block.
    auto zmap = [&](uint32_t e) -> uint64_t { return (uint64_t)(e & cmask) | ((uint64_t)(e >> mlo) << a.q0); };
    const uint64_t zt0 = zmap((uint32_t)x_elem(t, 0, rb0, R));
    auto tile_base = [&](uint64_t tile) -> uint64_t {
        return ((tile & ((1ull << lowbits) - 1)) << mlo) | ((tile >> lowbits) << hishift);
    };
    auto load_tile = [&](uint64_t tile, XC<T>(&w)[E]) {
        const XC<T> *src = psi + tile_base(tile) + zt0;
#pragma unroll
        for (int i = 0; i < E; ++i) w[i] = x_load(src + zmap((uint32_t)i << rb0));
    };
    auto store_tile = [&](uint64_t tile, XC<T>(&w)[E], int rb) {
        // store from a layout whose lanes cover runs of >= 128 bytes
        if ((int)sizeof(XC<T>) << (rb < contig ? rb : contig) < 128) {
            x_exchange<T, R>(w, lds, rb, rb0);
            rb = rb0;
        }
        XC<T> *dst = psi + tile_base(tile) + zmap((uint32_t)x_elem(t, 0, rb, R));
#pragma unroll
        for (int i = 0; i < E; ++i) x_store(w[i], dst + zmap((uint32_t)i << rb));
    };
    // mixers forward from rb0 or backward to it; rb: the layout on exit
    auto mix = [&](XC<T>(&w)[E], bool forward, int &rb, const XF<T> &f) {
        if constexpr (MLO >= 0) {
            if (forward) {
                x_mix_c<T, R, TB, kPlan, true>(w, lds, f);
                rb = kP.rb[kP.nchunks - 1];
            } else {
                x_mix_c<T, R, TB, kPlan, false>(w, lds, f);
                rb = rb0;
            }
        } else {
            x_mix<T, R>(w, lds, a.plan, forward, rb, f);
        }
    };
    XC<T> v[E];
    uint32_t cz[E];
    if constexpr (kStream) {
        constexpr bool kCosts = (OPS & (XOP_MID | XOP_POST)) != 0;
        typedef typename XCostVec<R>::type CV;
        XC<T> nxt[E];
        CV cn{};
        uint64_t tile = blockIdx.x;
        if (tile < a.ntiles) {
            load_tile(tile, nxt);
            if constexpr (kCosts) cn = x_load_costs<R>(a.cost + (tile << TB));
        }
        for (; tile < a.ntiles; tile += gridDim.x) {
#pragma unroll
            for (int i = 0; i < E; ++i) v[i] = nxt[i];
            const CV cw = cn;
            if (tile + gridDim.x < a.ntiles) {
                load_tile(tile + gridDim.x, nxt);
                if constexpr (kCosts) cn = x_load_costs<R>(a.cost + ((tile + gridDim.x) << TB));
            }
            int rb = rb0;
            mix(v, true, rb, x_factors((T)a.ca, (T)a.sa));
            if constexpr (kCosts) {
                x_unpack_costs<R>(cw, cz);
                x_readout<T, R>(v, cz, aP, aE, aN, a.target);
            }
            if constexpr ((OPS & XOP_MID) != 0) {
#pragma unroll
                for (int i = 0; i < E; ++i) v[i] = xmul(lut_s[1][cz[i]], v[i]);
                mix(v, false, rb, x_factors((T)a.cb, (T)a.sb));
            }
            store_tile(tile, v, rb);
        }
    } else {
        // The first pass of a call: the tile is taken in the layout its
        // group's costs are stored in (after the forward mixers; |s> needs no
        // load, a given state one exchange), read out and phased there, and
        // mixed backward into the load layout. The readout-only pass (p = 0)
        // gathers its costs from the cost table.
        static_assert((OPS & XOP_PRE) == 0 || (OPS & XOP_MID) == 0, "the first pass is no boundary pass");
        const int rb_end = MLO >= 0 ? kP.rb[kP.nchunks - 1] : a.plan.rb[a.plan.nchunks - 1];
        for (uint64_t tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
            auto load_cost = [&](int rb) {
                const uint8_t *cc = a.cost_z + tile_base(tile) + zmap((uint32_t)x_elem(t, 0, rb, R));
#pragma unroll
                for (int i = 0; i < E; ++i) cz[i] = cc[zmap((uint32_t)i << rb)];
            };
            int rb = rb0;
            if constexpr ((OPS & XOP_PRE) != 0) {
                const typename XCostVec<R>::type cw = x_load_costs<R>(a.cost + (tile << TB));
                if (a.init_uniform) {
#pragma unroll
                    for (int i = 0; i < E; ++i) v[i] = XC<T>{(T)a.init_amp, (T)0};
                } else {
                    load_tile(tile, v);
                    if (rb_end != rb0) x_exchange<T, R>(v, lds, rb0, rb_end);
                }
                rb = rb_end;
                x_unpack_costs<R>(cw, cz);
                x_readout<T, R>(v, cz, aP, aE, aN, a.target);
#pragma unroll
                for (int i = 0; i < E; ++i) v[i] = xmul(lut_s[0][cz[i]], v[i]);
                if constexpr ((OPS & XOP_MIX_A) != 0) mix(v, false, rb, x_factors((T)a.ca, (T)a.sa));
            } else {
                load_tile(tile, v);
                if constexpr ((OPS & XOP_MIX_A) != 0) mix(v, true, rb, x_factors((T)a.ca, (T)a.sa));
            }
            if constexpr ((OPS & XOP_POST) != 0) {
                load_cost(rb);
                x_readout<T, R>(v, cz, aP, aE, aN, a.target);
            }
            if constexpr (store) store_tile(tile, v, rb);
        }
    }
    if constexpr (kReadout) {
        double r[3] = {aP, aE, aN};
        block_sum<3, kThreads>(r, red_s);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < 3; ++k) a.partials[(size_t)blockIdx.x * 3 + k] = r[k];
    }
}

// Tile-ordered copy of the cost table for one high group (tile bits [0, mlo)
// = z bits [0, mlo), mlo >= 3), each tile in the order its streaming passes
// read it after the forward mixers: thread t's 2^R costs are consecutive,
// out[(tile << tb) + (t << R) + i] = C(z(tile, e)) with e = x_elem(t, i, rb, R).
// A block takes kXCopyTiles consecutive tiles: their rows are runs of 2^mlo
// bytes of the table, adjacent for adjacent tiles while the tile index's low
// bits are z bits, so lanes read consecutive 8-byte pieces; the tiles are
// staged in LDS in element order and each thread then gathers its 2^R bytes
// and writes them with one vector store.
constexpr int kXCopyTilesLog2 = 3;
constexpr int kXCopyBytesLog2 = 15;  // LDS of the copy kernel
// Tiles per block of the copy kernel, log2: kXCopyTilesLog2, fewer when the
// tiles are larger than 4 KiB or there are fewer tiles (ntiles is a power of 2).
__host__ __device__ inline int x_copy_ntl(int tb, uint64_t ntiles) {
    int ntl = kXCopyTilesLog2 < kXCopyBytesLog2 - tb ? kXCopyTilesLog2 : kXCopyBytesLog2 - tb;
    while (ntl > 0 && (1ull << ntl) > ntiles) --ntl;
    return ntl;
}
__global__ void __launch_bounds__(256) x_cost_tiles_kernel(const uint8_t *__restrict__ cost, uint8_t *__restrict__ out,
                                                          int tb, int mlo, int q0, int rb, int R, uint64_t ntiles) {
    __shared__ __align__(16) uint8_t st[1 << kXCopyBytesLog2];
    const int lowbits = q0 - mlo, hishift = q0 + tb - mlo;
    const int ntl = x_copy_ntl(tb, ntiles);
    const int runl = mlo - 3;  // 8-byte pieces per row run, log2
    const int E = 1 << R;
    for (uint64_t tile0 = (uint64_t)blockIdx.x << ntl; tile0 < ntiles; tile0 += (uint64_t)gridDim.x << ntl) {
        for (int k = threadIdx.x; k < (1 << (ntl + tb - 3)); k += blockDim.x) {
            const int pb = k & ((1 << runl) - 1);
            const int j = (k >> runl) & ((1 << ntl) - 1);
            const int row = k >> (runl + ntl);
            const uint64_t tile = tile0 + j;
            const uint64_t base = ((tile & ((1ull << lowbits) - 1)) << mlo) | ((tile >> lowbits) << hishift);
            const uint2 v = *reinterpret_cast<const uint2 *>(cost + (base | ((uint64_t)pb << 3) | ((uint64_t)row << q0)));
            *reinterpret_cast<uint2 *>(st + (j << tb) + (row << mlo) + (pb << 3)) = v;
        }
        __syncthreads();
        for (int w0 = threadIdx.x * E; w0 < (1 << (ntl + tb)); w0 += blockDim.x * E) {
            const int j = w0 >> tb, t = (w0 & ((1 << tb) - 1)) >> R;
            const uint8_t *src = st + (j << tb);
            uint32_t wd[4] = {0u, 0u, 0u, 0u};
            for (int i = 0; i < E; ++i) wd[i >> 2] |= (uint32_t)src[x_elem(t, i, rb, R)] << (8 * (i & 3));
            uint8_t *dst = out + (tile0 << tb) + w0;
            if (E == 16) *reinterpret_cast<uint4 *>(dst) = uint4{wd[0], wd[1], wd[2], wd[3]};
            else *reinterpret_cast<uint2 *>(dst) = uint2{wd[0], wd[1]};
        }
        __syncthreads();
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
    // up to one row per pass block (32768 for the high groups at n = 28):
    // unrolled so that several rows' loads are in flight per thread
#pragma unroll 8
    for (int b = threadIdx.x; b < f.nblocks; b += 1024)
        for (int k = 0; k < 3; ++k) r[k] += f.partials[(size_t)b * f.stride + f.off + k];
    block_sum<3, 1024>(r, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) f.readout[k] = r[k];
}

// Workspace: phase LUTs [max(p,1)][256] complex, readouts [p+1][3] doubles,
// block partials [kXMaxBlocks][kXR] doubles, and for n > T the tile-ordered
// cost copies of the groups that take the fused boundary passes, other than
// group 0 (x_copies of 2^n bytes); each region 256-byte aligned.
struct XLayout {
    char *lut;
    double *ro, *part;
    uint8_t *cost_t;
    size_t bytes;
};

// Qubit groups for n > T: group 0 = qubits [0, T), then groups of up to
// kXGroupBits qubits. Group 0, the largest and the only one with contiguous
// tiles, goes second in the order when there are three or more groups, so
// that it takes the mixing-only pass and the fused boundary passes (two
// mixers each) fall on the smaller groups.
static int x_ngroups(int n, int dtype) {
    const int tb = x_tile_bits(dtype);
    return n <= tb ? 1 : 1 + (n - tb + kXGroupBits - 1) / kXGroupBits;
}
static int x_order(int G, int k) { return G >= 3 ? (k == 0 ? 1 : k == 1 ? 0 : k) : k; }
static int x_copies(int n, int dtype) {
    const int G = x_ngroups(n, dtype);
    return G <= 1 ? 0 : (x_order(G, 0) != 0) + (x_order(G, G - 1) != 0);
}

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
    static_assert(kXR <= 3 * kXMaxBlocks, "the small-state kernel's partials fit");
    off += al(sizeof(double) * 3 * (size_t)kXMaxBlocks);
    L.cost_t = reinterpret_cast<uint8_t *>(w + off);
    off += (size_t)x_copies(n, dtype) * al(size_t(1) << n);
    L.bytes = off;
    return L;
}

size_t x_workspace_bytes(int n, int p, int dtype) { return x_layout(nullptr, n, p, dtype).bytes; }

// Group 0 (mlo = 0) on its own tiles; the high groups on the larger ones,
// a full group of 8 qubits with its compile-time plan.
template <typename T, int OPS>
static void launch_group(int mlo, int blocks, size_t smem, hipStream_t st, const XPassArgs &a) {
    constexpr int TB = XCfg<T>::TB, TBW = XCfg<T>::TBW, R = XCfg<T>::R;
    constexpr int kFull = TBW - kXGroupBits;  // high-group tile bits below a full group
    if (mlo == 0)
        hipLaunchKernelGGL((x_pass_kernel<T, OPS, 0, TB>), dim3(blocks), dim3(1 << (TB - R)), smem, st, a);
    else if (mlo == kFull)
        hipLaunchKernelGGL((x_pass_kernel<T, OPS, kFull, TBW>), dim3(blocks), dim3(1 << (TBW - R)), smem, st, a);
    else
        hipLaunchKernelGGL((x_pass_kernel<T, OPS, -1, TBW>), dim3(blocks), dim3(1 << (TBW - R)), smem, st, a);
}

template <typename T>
static int launch_pass(int ops, int blocks, size_t smem, hipStream_t st, const XPassArgs &a) {
    switch (ops) {
        case XOP_MIX_A: launch_group<T, XOP_MIX_A>(a.mlo, blocks, smem, st, a); break;
        case XOP_PRE | XOP_MIX_A: launch_group<T, XOP_PRE | XOP_MIX_A>(a.mlo, blocks, smem, st, a); break;
        case XOP_MIX_A | XOP_MID: launch_group<T, XOP_MIX_A | XOP_MID>(a.mlo, blocks, smem, st, a); break;
        case XOP_MIX_A | XOP_POST: launch_group<T, XOP_MIX_A | XOP_POST>(a.mlo, blocks, smem, st, a); break;
        case XOP_POST: launch_group<T, XOP_POST>(a.mlo, blocks, smem, st, a); break;
        case XOP_PRE | XOP_MIX_A | XOP_POST:
            launch_group<T, XOP_PRE | XOP_MIX_A | XOP_POST>(a.mlo, blocks, smem, st, a);
            break;
        default:
            return fail(GQAOA_EINVAL, "internal: X pass operations %d", ops);
    }
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

// One group of qubits for the streaming passes (n > T).
struct XGroup {
    int tb;       // tile bits of the group's passes
    int mlo, q0;  // tile bits [mlo, tb) are qubits q0 .. q0 + tb - mlo - 1
    XPlan plan;
};

static XGroup x_group(int mlo, int q0, int TB, int R) {
    XGroup g{};
    g.tb = TB;
    g.mlo = mlo;
    g.q0 = q0;
    g.plan = x_plan(TB, R, mlo);
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
    const int TBW = dtype == GQAOA_C64 ? XCfg<float>::TBW : XCfg<double>::TBW;
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
        // the streaming passes read group 0's costs straight from the table:
        // its forward mixers end with the register bits at tile bit 0
        if (groups[0].plan.rb[groups[0].plan.nchunks - 1] != 0)
            return fail(GQAOA_EINVAL, "internal: X group 0 plan ends at tile bit %d",
                        groups[0].plan.rb[groups[0].plan.nchunks - 1]);
        for (int q0 = TB; q0 < n; q0 += kXGroupBits) {
            const int kb = std::min(kXGroupBits, n - q0);
            groups.push_back(x_group(TBW - kb, q0, TBW, R));
        }
        const int G = (int)groups.size();
        if (G != x_ngroups(n, dtype)) return fail(GQAOA_EINVAL, "internal: %d X groups for n=%d", G, n);
        const uint64_t total = 1ull << n;
        // Group 0: 32 blocks per CU looping over tiles with the next one in
        // flight (about 4 resident at once by LDS): at n = 28 its pass ran
        // 1-5% faster than with 4, 8 or 16 per CU, and no faster with up to
        // one tile per block. High groups: one tile per block up to
        // kXMaxBlocks (2 resident per CU by LDS).
        auto ntiles_of = [&](const XGroup &gr) -> uint64_t { return total >> gr.tb; };
        auto blocks_of = [&](const XGroup &gr) -> int {
            const uint64_t want = gr.tb == TB ? (uint64_t)dev.num_cus * 32 : ntiles_of(gr);
            return (int)std::min<uint64_t>(ntiles_of(gr), std::min<uint64_t>(want, kXMaxBlocks));
        };
        auto smem_of = [&](const XGroup &gr) -> size_t { return (cs << gr.tb) + (cs << gr.tb) / 16; };
        for (const XGroup &gr : groups)
            if (gr.tb > TBW || gr.tb - R > kXMaxRb || gr.mlo < 0 || gr.mlo >= gr.tb || gr.q0 + gr.tb - gr.mlo > n ||
                smem_of(gr) + 2 * 256 * cs + 3 * sizeof(double) * (1 << (gr.tb - R)) / kWave > dev.lds_per_block)
                return fail(GQAOA_EINVAL, "internal: X group tb=%d mlo=%d q0=%d for n=%d", gr.tb, gr.mlo, gr.q0, n);
        // cost copies of the boundary groups other than group 0, each in the
        // order its streaming passes read (after the forward mixers)
        std::vector<const uint8_t *> cost_of(G, nullptr);
        cost_of[0] = cost;
        {
            int slot = 0;
            for (int b : {x_order(G, 0), x_order(G, G - 1)}) {
                if (cost_of[b]) continue;
                const XGroup &gr = groups[b];
                if (gr.mlo < 3 || (R != 3 && R != 4) || (1 << (x_copy_ntl(gr.tb, ntiles_of(gr)) + gr.tb)) > (1 << kXCopyBytesLog2))
                    return fail(GQAOA_EINVAL, "internal: X cost copy for tb=%d, mlo=%d, R=%d", gr.tb, gr.mlo, R);
                const int cb = (int)std::max<uint64_t>(
                    1, std::min<uint64_t>(ntiles_of(gr) >> kXCopyTilesLog2, (uint64_t)dev.num_cus * 16));
                uint8_t *dst = L.cost_t + (size_t)slot++ * ((total + 255) & ~uint64_t(255));
                hipLaunchKernelGGL(x_cost_tiles_kernel, dim3(cb), dim3(256), 0, st, cost, dst, gr.tb, gr.mlo, gr.q0,
                                   gr.plan.rb[gr.plan.nchunks - 1], R, ntiles_of(gr));
                GQ_LAUNCH_CHECK();
                cost_of[b] = dst;
            }
            if (slot != x_copies(n, dtype)) return fail(GQAOA_EINVAL, "internal: %d X cost copies", slot);
        }
        auto pass = [&](int gi, int ops, bool uniform, int ja, int jb, int readout_j) -> int {
            const XGroup &gr = groups[gi];
            const int blocks = blocks_of(gr);
            const size_t smem = smem_of(gr);
            XPassArgs a{};
            a.psi = psi;
            a.cost = cost_of[gi];
            a.cost_z = cost;
            a.n = n;
            a.mlo = gr.mlo;
            a.q0 = gr.q0;
            a.contig = gi == 0 ? TB : gr.mlo;
            a.ntiles = ntiles_of(gr);
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
                const int gi = x_order(G, fwd ? k : G - 1 - k);
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
