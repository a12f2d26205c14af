// Statevector G-QAOA rounds (Eq. (3)) and their adjoint, streamed from HBM.
//
// One round is exp(-i gamma_j H_P) followed by the Grover mixer
// exp(-i beta_j |s><s|) = I + (e^{-i beta_j} - 1)|s><s| (Eq. (2)). The mixer
// adds the same scalar to every amplitude, delta_j = (e^{-i beta_j}-1) S_j / 2^n
// with S_j = sum_z phi_z, so it is applied lazily: pass j reads psi (holding
// phi_{j-1}) and the device scalar delta_{j-1}, forms psi' = phi_{j-1} + delta_{j-1}
// (the true state after round j-1), reads out P_sol / E (Eq. (4)) / norm of
// psi', multiplies by the phase LUT entry e^{-i gamma_j C(z)} and stores
// phi_j. One pass = one read and one write of psi plus one byte of cost per
// amplitude. Block partial sums are reduced in a fixed order by a one-block
// finalize kernel per instance, which also forms delta_j on the device, so no
// value crosses to the host between rounds.
//
// The reverse sweep of the adjoint gradient uses the same streaming shape:
// pass k reads lambda_k, phi_k and C, forms mu_k = lambda_k + eps_k
// (eps_k = (e^{+i beta_k}-1) sum lambda_k / 2^n), accumulates
// G_k = sum conj(mu) C phi (dP/dgamma_k = 2 Im G_k), and writes
// lambda_{k-1} = e^{+i gamma_k C} mu_k together with its sum.
//
// All kernels take an instance index in blockIdx.y so that many equally
// sized instances stream in one launch.
#include "internal.h"
#include "stream_pool.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <new>
#include <vector>

namespace gqaoa {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kSvThreads = 256;
constexpr int kFwdR = 7;   // S.re, S.im, psol, energy, norm, T.re, T.im (T = sum over target level)
constexpr int kRevR = 4;   // L.re, L.im (sum of lambda_{k-1}), G.re, G.im

template <typename T>
struct Cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ Cx<T> cmulc(Cx<T> a, Cx<T> b) {  // conj(a) * b
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

// ---- vectorized amplitude and cost I/O ---------------------------------------
// NT = 1: nontemporal loads and stores (streamed data is not kept in the caches).
template <int NT, typename V>
__device__ __forceinline__ V ld(const V *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <int NT, typename V>
__device__ __forceinline__ void st(V v, V *p) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <typename T, int AMP, int NT = 1>
struct AmpIO;

template <int AMP, int NT>
struct AmpIO<float, AMP, NT> {
    static_assert(AMP >= 2 && AMP % 2 == 0, "complex64 chunks hold pairs of amplitudes");
    static __device__ __forceinline__ void load(const void *p, Cx<float> (&a)[AMP]) {
        const f32x4 *q = reinterpret_cast<const f32x4 *>(p);
#pragma unroll
        for (int i = 0; i < AMP / 2; ++i) {
            const f32x4 v = ld<NT>(q + i);
            a[2 * i] = {v.x, v.y};
            a[2 * i + 1] = {v.z, v.w};
        }
    }
    static __device__ __forceinline__ void store(void *p, const Cx<float> (&a)[AMP]) {
        f32x4 *q = reinterpret_cast<f32x4 *>(p);
#pragma unroll
        for (int i = 0; i < AMP / 2; ++i)
            st<NT>(f32x4{a[2 * i].re, a[2 * i].im, a[2 * i + 1].re, a[2 * i + 1].im}, q + i);
    }
};

template <int AMP, int NT>
struct AmpIO<double, AMP, NT> {
    static __device__ __forceinline__ void load(const void *p, Cx<double> (&a)[AMP]) {
        const f64x2 *q = reinterpret_cast<const f64x2 *>(p);
#pragma unroll
        for (int i = 0; i < AMP; ++i) {
            const f64x2 v = ld<NT>(q + i);
            a[i] = {v.x, v.y};
        }
    }
    static __device__ __forceinline__ void store(void *p, const Cx<double> (&a)[AMP]) {
        f64x2 *q = reinterpret_cast<f64x2 *>(p);
#pragma unroll
        for (int i = 0; i < AMP; ++i) st<NT>(f64x2{a[i].re, a[i].im}, q + i);
    }
};

template <int AMP>
__device__ __forceinline__ void load_costs(const uint8_t *p, uint32_t (&c)[AMP]) {
    if constexpr (AMP == 1) {
        c[0] = p[0];
    } else if constexpr (AMP == 2) {
        const uint32_t v = *reinterpret_cast<const uint16_t *>(p);
        c[0] = v & 0xFFu;
        c[1] = v >> 8;
    } else if constexpr (AMP == 4) {
        const uint32_t v = *reinterpret_cast<const uint32_t *>(p);
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = (v >> (8 * i)) & 0xFFu;
    } else if constexpr (AMP == 8) {
        const uint64_t v = *reinterpret_cast<const uint64_t *>(p);
#pragma unroll
        for (int i = 0; i < 8; ++i) c[i] = (uint32_t)(v >> (8 * i)) & 0xFFu;
    } else {
        static_assert(AMP == 16, "unsupported chunk");
        const u32x4 v = *reinterpret_cast<const u32x4 *>(p);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 16; ++i) c[i] = (w[i >> 2] >> (8 * (i & 3))) & 0xFFu;
    }
}

// Accumulator type for per-tile partial sums (float tiles are short).
template <typename T>
struct Acc;
template <>
struct Acc<float> {
    using t = float;
};
template <>
struct Acc<double> {
    using t = double;
};

struct FinArgs {
    const double *partials;  // [inst][nblocks][kFwdR]
    int nblocks;
    double inv_N;
    // per instance (strided by the *_stride fields, all in doubles)
    const double *mixf;      // e^{-i beta_j} - 1 for this round; null in the last pass
    int mixf_stride;
    double *delta_out;       // delta_j
    double *S_out;           // S_j
    double *readout_out;     // psol, E, norm of the state before this pass's phase
    double *T_out;           // sum over the target level (last pass only)
    int stride;              // stride for delta_out/S_out/T_out per instance
    int readout_stride;
    // adjoint set-up after the last forward pass: eps_p and dbeta_p
    const double *mixb;      // e^{+i beta_p} - 1, null: skip
    const double *ebeta;     // e^{-i beta_p}
    const double *S_p;       // S_p
    double *eps_out;
    double *dbeta_out;
    int mix_stride;          // doubles per instance in mixb / ebeta (2p)
    int grad_stride;         // doubles per instance in dbeta (p)
};

// Turn the summed partials of one instance into its readouts and delta_j.
__device__ __forceinline__ void finalize_apply(const FinArgs &a, int inst, const double (&r)[kFwdR]) {
    if (a.readout_out) {
        double *ro = a.readout_out + (size_t)inst * a.readout_stride;
        ro[0] = r[2];
        ro[1] = r[3];
        ro[2] = r[4];
    }
    if (a.mixf) {
        const double *mf = a.mixf + (size_t)inst * a.mixf_stride;
        const double sr = r[0] * a.inv_N, si = r[1] * a.inv_N;
        double *d = a.delta_out + (size_t)inst * a.stride;
        d[0] = mf[0] * sr - mf[1] * si;
        d[1] = mf[0] * si + mf[1] * sr;
        if (a.S_out) {
            double *s = a.S_out + (size_t)inst * a.stride;
            s[0] = r[0];
            s[1] = r[1];
        }
    }
    if (a.T_out) {
        double *t = a.T_out + (size_t)inst * a.stride;
        t[0] = r[5];
        t[1] = r[6];
    }
    if (a.mixb) {
        // eps_p = (e^{+i beta_p}-1) sum(lambda_p)/N, sum(lambda_p) = T
        const double *mb = a.mixb + (size_t)inst * a.mix_stride;
        const double tr = r[5], ti = r[6];
        double *e = a.eps_out + (size_t)inst * 2;
        e[0] = (mb[0] * tr - mb[1] * ti) * a.inv_N;
        e[1] = (mb[0] * ti + mb[1] * tr) * a.inv_N;
        // dbeta_p = 2 Re(-i e^{-i beta_p} conj(T) S_p) / N
        const double *eb = a.ebeta + (size_t)inst * a.mix_stride;
        const double *sp = a.S_p + (size_t)inst * a.stride;
        const double xr = tr * sp[0] + ti * sp[1], xi = tr * sp[1] - ti * sp[0];  // conj(T) S
        const double yi = eb[0] * xi + eb[1] * xr;                                // Im(e^{-i b} x)
        a.dbeta_out[(size_t)inst * a.grad_stride] = 2.0 * yi * a.inv_N;          // Re(-i y) = Im y
    }
}

// Fixed-order sum of the nrows x R partials of one instance by kThreads
// threads (rows strided over threads, then a block reduction).
template <int R, int kThreads>
__device__ __forceinline__ void reduce_rows(const double *p, int nrows, double (&r)[R], double *lds) {
#pragma unroll
    for (int k = 0; k < R; ++k) r[k] = 0.0;
    for (int b0 = threadIdx.x; b0 < nrows; b0 += 4 * kThreads) {
        double v[4][R];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int b = b0 + i * kThreads;
#pragma unroll
            for (int k = 0; k < R; ++k) v[i][k] = b < nrows ? p[(size_t)b * R + k] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int k = 0; k < R; ++k) r[k] += v[i][k];
    }
    block_sum<R, kThreads>(r, lds);
}

// ---- forward pass ---------------------------------------------------------------
struct FwdArgs {
    const uint8_t *cost;     // [inst][N]
    const void *psi_in;      // [inst][N] complex T (ignored if init_uniform)
    void *psi_out;           // [inst][N] complex T (may equal psi_in)
    uint64_t N;
    const void *lut;         // [inst][lut_stride] complex T, e^{-i gamma C}; null: no phase
    int lut_stride;
    int lut_len;
    const double *delta;     // [inst][delta_stride] complex double added before the phase; null: none
    int delta_stride;
    int init_uniform;
    double init_amp;
    const int32_t *target;   // [inst]
    double *partials;        // [inst][gridDim.x][kFwdR]
    unsigned int *counter;   // [inst] blocks finished (fused finalize only; zero between launches)
    FinArgs fin;             // finalize of this round (fused finalize only)
};

// FUSED: the last block of each instance to finish (counted with a device-scope
// atomic after a release fence) sums all partial rows in the fixed row order
// and applies the finalize itself, so a round is a single launch.
template <typename T, bool PHASE, bool WRITE, int AMP, int UNROLL, int NT = 1, bool FUSED = false>
__global__ void __launch_bounds__(kSvThreads) sv_forward_kernel(FwdArgs a) {
    __shared__ Cx<T> lut_s[256];
    __shared__ double red_s[kFwdR * kSvThreads / kWave];
    const int inst = blockIdx.y;
    const uint64_t ioff = (uint64_t)inst * a.N;
    if constexpr (PHASE) {
        const Cx<T> *lut = reinterpret_cast<const Cx<T> *>(a.lut) + (size_t)inst * a.lut_stride;
        for (int i = threadIdx.x; i < a.lut_len; i += kSvThreads) lut_s[i] = lut[i];
        __syncthreads();
    }
    const uint32_t target = (uint32_t)a.target[inst];
    Cx<T> dl{T(0), T(0)};
    if (a.delta) {
        const double *d = a.delta + (size_t)inst * a.delta_stride;
        dl = {T(d[0]), T(d[1])};
    }
    const uint8_t *cost = a.cost + ioff;
    const Cx<T> *src = reinterpret_cast<const Cx<T> *>(a.psi_in) + ioff;
    Cx<T> *dst = reinterpret_cast<Cx<T> *>(a.psi_out) + ioff;
    const T amp0 = T(a.init_amp);

    double accSr = 0, accSi = 0, accP = 0, accE = 0, accN = 0, accTr = 0, accTi = 0;
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t wave = ((uint64_t)blockIdx.x * kSvThreads + threadIdx.x) / kWave;
    const uint64_t nwaves = (uint64_t)gridDim.x * kSvThreads / kWave;
    constexpr uint64_t kTile = (uint64_t)kWave * AMP * UNROLL;
    for (uint64_t base = wave * kTile; base < a.N; base += nwaves * kTile) {
        uint32_t c[UNROLL][AMP];
        Cx<T> v[UNROLL][AMP];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint64_t idx = base + (uint64_t)u * kWave * AMP + (uint64_t)lane * AMP;
            if (idx < a.N) {
                load_costs<AMP>(cost + idx, c[u]);
                if (!a.init_uniform) AmpIO<T, AMP, NT>::load(src + idx, v[u]);
            } else {
#pragma unroll
                for (int i = 0; i < AMP; ++i) c[u][i] = 0xFFFFu;  // never a target level
            }
        }
        typename Acc<T>::t sSr = 0, sSi = 0, sP = 0, sE = 0, sN = 0, sTr = 0, sTi = 0;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint64_t idx = base + (uint64_t)u * kWave * AMP + (uint64_t)lane * AMP;
            const bool ok = idx < a.N;
#pragma unroll
            for (int i = 0; i < AMP; ++i) {
                Cx<T> x = a.init_uniform ? Cx<T>{amp0, T(0)} : v[u][i];
                x.re += dl.re;
                x.im += dl.im;
                const T pr = ok ? x.re * x.re + x.im * x.im : T(0);
                sN += pr;
                sE += T(c[u][i]) * pr;
                const bool hit = c[u][i] == target;
                sP += hit ? pr : T(0);
                sTr += hit ? x.re : T(0);
                sTi += hit ? x.im : T(0);
                if constexpr (PHASE) {
                    x = cmul(lut_s[ok ? c[u][i] : 0], x);
                    sSr += ok ? x.re : T(0);
                    sSi += ok ? x.im : T(0);
                }
                v[u][i] = x;
            }
        }
        accSr += sSr; accSi += sSi; accP += sP; accE += sE; accN += sN; accTr += sTr; accTi += sTi;
        if constexpr (WRITE) {
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const uint64_t idx = base + (uint64_t)u * kWave * AMP + (uint64_t)lane * AMP;
                if (idx < a.N) AmpIO<T, AMP, NT>::store(dst + idx, v[u]);
            }
        }
    }
    double r[kFwdR] = {accSr, accSi, accP, accE, accN, accTr, accTi};
    block_sum<kFwdR, kSvThreads>(r, red_s);
    if (threadIdx.x == 0) {
        double *out = a.partials + ((size_t)inst * gridDim.x + blockIdx.x) * kFwdR;
#pragma unroll
        for (int k = 0; k < kFwdR; ++k) out[k] = r[k];
    }
    if constexpr (FUSED) {
        __shared__ int last_s;
        if (threadIdx.x == 0) {
            __threadfence();
            const unsigned int done = atomicAdd(a.counter + inst, 1u);
            last_s = done == gridDim.x - 1;
        }
        __syncthreads();
        if (last_s) {
            __threadfence();
            double t[kFwdR];
            reduce_rows<kFwdR, kSvThreads>(a.partials + (size_t)inst * gridDim.x * kFwdR, gridDim.x, t, red_s);
            if (threadIdx.x == 0) {
                finalize_apply(a.fin, inst, t);
                a.counter[inst] = 0u;
            }
        }
    }
}

// ---- resident evolution of small states ------------------------------------------
// A state of at most 2^14 (complex64) or 2^13 (complex128) amplitudes fits the
// registers of one block, so all p rounds of one instance run in a single
// launch: each thread owns the PER consecutive amplitudes z = tid PER + i in
// every round, with their costs packed four to a register. Round j: add
// delta_{j-1} (the previous mixer, applied lazily), read out psi_{j-1},
// apply the phase from the round's table (staged in LDS, the next round's
// table loaded while this one is used), sum phi_j; one float64 reduction per
// round gives S_j, delta_j and the readouts, with the same per-element
// arithmetic as the streaming round pass (delta and the table in the state's
// precision, per-thread sums in that precision, float64 across threads). The
// final state is written once, at the end.
struct ResArgs {
    const uint8_t *cost;
    void *psi;             // [N] complex: initial state (unless init_uniform), final state
    const void *lut;       // [p][256] complex, the state's precision
    const double *mixf;    // [p][2]: e^{-i beta_j} - 1
    double *readout;       // [p+1][3]: P_sol, E, norm of psi_0 .. psi_p
    int n, p, init_uniform, target;
};

template <typename T, int THREADS, int PER>
__global__ void __launch_bounds__(THREADS) sv_resident_kernel(ResArgs a) {
    constexpr int kWaves = THREADS / kWave;
    constexpr int kLutPer = (256 + THREADS - 1) / THREADS;
    __shared__ Cx<T> lut_s[2][256];
    __shared__ double red_s[2][kWaves][5];  // per-wave sums, double-buffered by round parity
    const uint32_t N = 1u << a.n;
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const bool owns = (uint32_t)tid * PER < N;
    const Cx<T> *lut = reinterpret_cast<const Cx<T> *>(a.lut);
    const uint32_t target = (uint32_t)a.target;
    const double invN = ldexp(1.0, -a.n);
    uint32_t cpk[(PER + 3) / 4];
#pragma unroll
    for (int w = 0; w < (PER + 3) / 4; ++w) cpk[w] = 0u;
    Cx<T> x[PER];
    if (owns) {
        load_packed_costs<PER>(a.cost + (size_t)tid * PER, cpk);
        const Cx<T> *src = reinterpret_cast<const Cx<T> *>(a.psi) + (size_t)tid * PER;
        const T amp0 = T(sqrt(invN));
#pragma unroll
        for (int i = 0; i < PER; ++i) x[i] = a.init_uniform ? Cx<T>{amp0, T(0)} : src[i];
    }
    for (int k = tid; k < 256; k += THREADS) lut_s[1][k] = lut[k];  // round 1 uses buffer 1
    __syncthreads();
    Cx<T> dl{T(0), T(0)};
    for (int j = 1; j <= a.p + 1; ++j) {
        const bool ph = j <= a.p;
        double mr = 0.0, mi = 0.0;  // this round's mixer factor, loaded before the sweep
        if (ph) {
            mr = a.mixf[2 * (j - 1)];
            mi = a.mixf[2 * (j - 1) + 1];
        }
        Cx<T> next[kLutPer];  // the next round's table, loaded now, stored after the sweep
        if (j < a.p)
#pragma unroll
            for (int r = 0; r < kLutPer; ++r)
                if (tid + r * THREADS < 256) next[r] = lut[(size_t)j * 256 + tid + r * THREADS];
        T sSr = 0, sSi = 0, sP = 0, sE = 0, sN = 0;
        if (owns) {
            const Cx<T> *tab = lut_s[j & 1];
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const uint32_t cz = (cpk[i >> 2] >> (8 * (i & 3))) & 0xFFu;
                Cx<T> v = x[i];
                v.re += dl.re;
                v.im += dl.im;
                const T pr = v.re * v.re + v.im * v.im;
                sN += pr;
                sE += T(cz) * pr;
                sP += cz == target ? pr : T(0);
                if (ph) {
                    v = cmul(tab[cz], v);
                    sSr += v.re;
                    sSi += v.im;
                }
                x[i] = v;
            }
        }
        if (j < a.p)
#pragma unroll
            for (int r = 0; r < kLutPer; ++r)
                if (tid + r * THREADS < 256) lut_s[(j + 1) & 1][tid + r * THREADS] = next[r];
        // one barrier per round: it publishes the per-wave sums and the next
        // table; a buffer is rewritten two rounds later, after the next
        // round's barrier, which every thread passes only once it has read it
        // (DPP wave sums: the block is converged here)
        double r5[5] = {(double)sSr, (double)sSi, (double)sP, (double)sE, (double)sN};
#pragma unroll
        for (int q = 0; q < 5; ++q) r5[q] = wave_sum_dpp(r5[q]);
        double(*buf)[5] = red_s[j & 1];
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < 5; ++q) buf[tid / kWave][q] = r5[q];
        __syncthreads();
        if constexpr (kWaves > 1) {
#pragma unroll
            for (int q = 0; q < 5; ++q) r5[q] = lanes_sum_dpp<kWaves>(lane < kWaves ? buf[lane][q] : 0.0);
        }
        if (tid == 0) {
            double *ro = a.readout + 3 * (size_t)(j - 1);
            ro[0] = r5[2];
            ro[1] = r5[3];
            ro[2] = r5[4];
        }
        if (ph) {
            const double sr = r5[0] * invN, si = r5[1] * invN;
            dl = {T(mr * sr - mi * si), T(mr * si + mi * sr)};
        } else {
            dl = {T(0), T(0)};
        }
    }
    if (owns) {
        Cx<T> *dst = reinterpret_cast<Cx<T> *>(a.psi) + (size_t)tid * PER;
#pragma unroll
        for (int i = 0; i < PER; ++i) dst[i] = x[i];
    }
}

// Largest n of the resident form: the state's registers in one block.
static int resident_max_n(int dtype) { return dtype == GQAOA_C64 ? 14 : 13; }

static bool resident_ok(int n, int dtype, int p) {
    if (p < 1 || n > resident_max_n(dtype)) return false;
    const char *e = getenv("GQAOA_SV_RESIDENT");  // "0": always stream (for comparisons)
    return !(e && e[0] == '0');
}

typedef void (*ResFn)(ResArgs);
template <typename T>
static ResFn resident_fn(int n, int *threads) {
    // one wave of 2^n / 64 amplitudes per lane while that is at most the run
    // length, then 2^n / run threads (complex64: runs of 16, complex128: 8)
    constexpr int kRun = sizeof(T) == 4 ? 16 : 8;
    const int N = 1 << n;
    *threads = std::max(kWave, N / kRun);
    if (*threads == kWave) {
        switch (std::max(1, N / kWave)) {
            case 1: return sv_resident_kernel<T, 64, 1>;
            case 2: return sv_resident_kernel<T, 64, 2>;
            case 4: return sv_resident_kernel<T, 64, 4>;
            case 8: return sv_resident_kernel<T, 64, 8>;
            default: break;
        }
        if constexpr (kRun == 16) return sv_resident_kernel<T, 64, 16>;
    }
    switch (*threads) {
        case 128: return sv_resident_kernel<T, 128, kRun>;
        case 256: return sv_resident_kernel<T, 256, kRun>;
        case 512: return sv_resident_kernel<T, 512, kRun>;
        default: return sv_resident_kernel<T, 1024, kRun>;
    }
}

static int launch_resident(int dtype, const ResArgs &a, hipStream_t st) {
    int threads = 0;
    const ResFn fn = dtype == GQAOA_C64 ? resident_fn<float>(a.n, &threads) : resident_fn<double>(a.n, &threads);
    ProfScope ps(dtype == GQAOA_C64 ? "sv_resident_c64" : "sv_resident_c128", st);
    hipLaunchKernelGGL(fn, dim3(1), dim3(threads), 0, st, a);
    ps.end();
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

// ---- reverse (adjoint) pass -------------------------------------------------------
struct RevArgs {
    const uint8_t *cost;
    const void *phi;        // phi_k, [inst][N]
    const void *lam_in;     // lambda_k, [inst][N]; null on the first reverse step
    void *lam_out;          // lambda_{k-1}, may equal lam_in
    uint64_t N;
    const void *lut;        // forward LUT of round k (the pass uses its conjugate)
    int lut_stride;
    int lut_len;
    const double *eps;      // [inst][eps_stride] complex: eps_k
    int eps_stride;
    const double *delta_p;  // [inst][delta_stride] complex delta_p (first step only)
    int delta_stride;
    const int32_t *target;
    double *partials;       // [inst][gridDim.x][kRevR]
};

template <typename T, bool FIRST, bool WRITE, int AMP, int UNROLL>
__global__ void __launch_bounds__(kSvThreads) sv_reverse_kernel(RevArgs a) {
    __shared__ Cx<T> lut_s[256];
    __shared__ double red_s[kRevR * kSvThreads / kWave];
    const int inst = blockIdx.y;
    const uint64_t ioff = (uint64_t)inst * a.N;
    {
        const Cx<T> *lut = reinterpret_cast<const Cx<T> *>(a.lut) + (size_t)inst * a.lut_stride;
        for (int i = threadIdx.x; i < a.lut_len; i += kSvThreads) lut_s[i] = lut[i];
        __syncthreads();
    }
    const uint32_t target = (uint32_t)a.target[inst];
    const double *e = a.eps + (size_t)inst * a.eps_stride;
    const Cx<T> eps{T(e[0]), T(e[1])};
    Cx<T> dp{T(0), T(0)};
    if constexpr (FIRST) {
        const double *d = a.delta_p + (size_t)inst * a.delta_stride;
        dp = {T(d[0]), T(d[1])};
    }
    const uint8_t *cost = a.cost + ioff;
    const Cx<T> *phi = reinterpret_cast<const Cx<T> *>(a.phi) + ioff;
    const Cx<T> *lin = reinterpret_cast<const Cx<T> *>(a.lam_in) + ioff;
    Cx<T> *lout = reinterpret_cast<Cx<T> *>(a.lam_out) + ioff;

    double accLr = 0, accLi = 0, accGr = 0, accGi = 0;
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t wave = ((uint64_t)blockIdx.x * kSvThreads + threadIdx.x) / kWave;
    const uint64_t nwaves = (uint64_t)gridDim.x * kSvThreads / kWave;
    constexpr uint64_t kTile = (uint64_t)kWave * AMP * UNROLL;
    for (uint64_t base = wave * kTile; base < a.N; base += nwaves * kTile) {
        uint32_t c[UNROLL][AMP];
        Cx<T> f[UNROLL][AMP], l[UNROLL][AMP];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint64_t idx = base + (uint64_t)u * kWave * AMP + (uint64_t)lane * AMP;
            if (idx < a.N) {
                load_costs<AMP>(cost + idx, c[u]);
                AmpIO<T, AMP>::load(phi + idx, f[u]);
                if constexpr (!FIRST) AmpIO<T, AMP>::load(lin + idx, l[u]);
            }
        }
        typename Acc<T>::t sLr = 0, sLi = 0, sGr = 0, sGi = 0;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint64_t idx = base + (uint64_t)u * kWave * AMP + (uint64_t)lane * AMP;
            if (idx < a.N) {
#pragma unroll
                for (int i = 0; i < AMP; ++i) {
                    Cx<T> lam;
                    if constexpr (FIRST) {
                        const bool hit = c[u][i] == target;
                        lam = {hit ? f[u][i].re + dp.re : T(0), hit ? f[u][i].im + dp.im : T(0)};
                    } else {
                        lam = l[u][i];
                    }
                    const Cx<T> mu{lam.re + eps.re, lam.im + eps.im};
                    const Cx<T> g = cmulc(mu, f[u][i]);
                    const T cc = T(c[u][i]);
                    sGr += cc * g.re;
                    sGi += cc * g.im;
                    const Cx<T> nl = cmulc(lut_s[c[u][i]], mu);  // e^{+i gamma C} mu
                    sLr += nl.re;
                    sLi += nl.im;
                    l[u][i] = nl;
                }
            }
        }
        accLr += sLr; accLi += sLi; accGr += sGr; accGi += sGi;
        if constexpr (WRITE) {
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                const uint64_t idx = base + (uint64_t)u * kWave * AMP + (uint64_t)lane * AMP;
                if (idx < a.N) AmpIO<T, AMP>::store(lout + idx, l[u]);
            }
        }
    }
    double r[kRevR] = {accLr, accLi, accGr, accGi};
    block_sum<kRevR, kSvThreads>(r, red_s);
    if (threadIdx.x == 0) {
        double *out = a.partials + ((size_t)inst * gridDim.x + blockIdx.x) * kRevR;
#pragma unroll
        for (int k = 0; k < kRevR; ++k) out[k] = r[k];
    }
}

// ---- finalizers (fixed-order sums of the per-block partial rows) -----------------
// A streaming pass writes one row of partial sums per block. One finalize
// block of kFinThreads threads takes up to kFinThreads rows of an instance,
// one row per thread with every load issued before the first add (the
// finalize sits between two bandwidth-bound passes, so its cost is one memory
// latency, not a chain). A pass with more blocks per instance is folded
// first: fold_partials_kernel sums each run of kFinThreads rows into one row,
// in the same fixed order, so at most kMaxPassBlocks / kFinThreads plus one
// row per instance remain.
constexpr int kFinThreads = 1024;

constexpr int kFinWave = kWave;  // finalize of at most one row per lane: one wave, no barrier

template <int R, int T = kFinThreads>
__device__ __forceinline__ void reduce_partials(const double *p, int nblocks /* <= T */,
                                                double (&r)[R], double *lds) {
    const int b = threadIdx.x;
#pragma unroll
    for (int k = 0; k < R; ++k) r[k] = b < nblocks ? p[(size_t)b * R + k] : 0.0;
    if constexpr (T == kWave) {
#pragma unroll
        for (int k = 0; k < R; ++k) r[k] = wave_sum_dpp(r[k]);
    } else {
        block_sum<R, T>(r, lds);
    }
}

// Block (f, i): rows [f kFinThreads, (f + 1) kFinThreads) of instance i's
// nrows partial rows, summed into row f of the folded rows [inst][nfold][R].
template <int R>
__global__ void __launch_bounds__(kFinThreads) fold_partials_kernel(const double *p, int nrows, double *q, int nfold) {
    __shared__ double lds[R * kFinThreads / kWave];
    const int inst = blockIdx.y;
    const int first = blockIdx.x * kFinThreads;
    double r[R];
    reduce_partials<R>(p + ((size_t)inst * nrows + first) * R, min(kFinThreads, nrows - first), r, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < R; ++k) q[((size_t)inst * nfold + blockIdx.x) * R + k] = r[k];
}

// T threads: kFinThreads, or one wave when the instance has at most kFinWave rows
template <int T>
__global__ void __launch_bounds__(T) sv_finalize_kernel(FinArgs a) {
    __shared__ double lds[kFwdR * T / kWave];
    const int inst = blockIdx.x;
    double r[kFwdR];
    reduce_partials<kFwdR, T>(a.partials + (size_t)inst * a.nblocks * kFwdR, a.nblocks, r, lds);
    if (threadIdx.x == 0) finalize_apply(a, inst, r);
}

struct RevFinArgs {
    const double *partials;  // [inst][nblocks][kRevR]
    int nblocks;
    double inv_N;
    double *dgamma_k;        // [inst * grad_stride]
    // for k > 1: eps_{k-1} and dbeta_{k-1}
    const double *mixb_km1;  // e^{+i beta_{k-1}} - 1
    const double *ebeta_km1; // e^{-i beta_{k-1}}
    const double *S_km1;     // S_{k-1}
    int S_stride;
    double *eps_out;
    double *dbeta_km1;
    int grad_stride;
};

template <int T>
__global__ void __launch_bounds__(T) sv_rev_finalize_kernel(RevFinArgs a) {
    __shared__ double lds[kRevR * T / kWave];
    const int inst = blockIdx.x;
    double r[kRevR];
    reduce_partials<kRevR, T>(a.partials + (size_t)inst * a.nblocks * kRevR, a.nblocks, r, lds);
    if (threadIdx.x != 0) return;
    a.dgamma_k[(size_t)inst * a.grad_stride] = 2.0 * r[3];
    if (a.mixb_km1) {
        const double *mb = a.mixb_km1 + (size_t)inst * a.grad_stride * 2;
        const double lr = r[0], li = r[1];
        double *e = a.eps_out + (size_t)inst * 2;
        e[0] = (mb[0] * lr - mb[1] * li) * a.inv_N;
        e[1] = (mb[0] * li + mb[1] * lr) * a.inv_N;
        const double *eb = a.ebeta_km1 + (size_t)inst * a.grad_stride * 2;
        const double *sp = a.S_km1 + (size_t)inst * a.S_stride;
        const double xr = lr * sp[0] + li * sp[1], xi = lr * sp[1] - li * sp[0];
        const double yi = eb[0] * xi + eb[1] * xr;
        a.dbeta_km1[(size_t)inst * a.grad_stride] = 2.0 * yi * a.inv_N;
    }
}

// ---- launch shapes ------------------------------------------------------------------
struct PassShape {
    int amp, unroll, blocks_x, nt;
};

constexpr int kMaxPassBlocks = 262144;  // partial-sum rows per launch (all instances)

// Launch shape of the streaming passes. A lane moves exactly one 16-byte
// chunk of the state per group (2 complex64 or 1 complex128 amplitudes), so
// each wave-wide load or store instruction covers 1 KiB of contiguous memory;
// UNROLL groups per loop trip keep that many loads in flight per lane. By
// default the grid gives every block one tile (4 groups per lane, up to 1024
// blocks per CU and kMaxPassBlocks rows): at n = 28 (131,072 blocks) that
// streams about 5% faster than a persistent grid of 16 blocks per CU looping
// over 8-group tiles and 1.2% faster than 65,536 blocks of two tiles each,
// and the 256 instances of a batched adjoint of n = 20 get 1024 blocks each
// (3% faster per batch than 256); the extra partial rows are folded before
// the finalize. The fused finalize (the last block sums every row) keeps the
// persistent grid.
// GQAOA_SV_SHAPE="amp,unroll,blocks_per_cu,nt" overrides the round pass (a
// tuning hook; shapes outside the compiled set fall back to the default).
static PassShape pass_shape(uint64_t N, int num_inst, int dtype, const DeviceInfo &dev, bool fused = false) {
    PassShape s;
    int bpc = fused ? 16 : 1024;
    s.nt = 1;
    s.amp = dtype == GQAOA_C64 ? 2 : 1;
    s.unroll = fused ? 8 : 4;
    if (const char *e = getenv("GQAOA_SV_SHAPE")) {
        int a = 0, u = 0, b = 0, t = 1;
        if (sscanf(e, "%d,%d,%d,%d", &a, &u, &b, &t) >= 3 && a > 0 && u > 0 && b > 0) {
            s.amp = a;
            s.unroll = u;
            bpc = b;
            s.nt = t ? 1 : 0;
        }
    }
    if (N < (uint64_t)kWave * s.amp * s.unroll) {  // fewer amplitudes than one tile
        s.amp = dtype == GQAOA_C64 ? 2 : 1;
        s.unroll = 1;
        s.nt = 1;
    }
    const uint64_t per_block = (uint64_t)kSvThreads * s.amp * s.unroll;
    const uint64_t want = (N + per_block - 1) / per_block;
    const uint64_t cap = std::max<uint64_t>(1, (uint64_t)std::min(kMaxPassBlocks, dev.num_cus * bpc) / num_inst);
    static_assert(kMaxPassBlocks / kFinThreads <= kFinThreads, "one fold leaves rows for one finalize block");
    s.blocks_x = (int)std::max<uint64_t>(1, std::min(want, cap));
    return s;
}

#define GQ_FWD_SHAPE(TT, A, U, NTF)                                                                  \
    if (s.amp == A && s.unroll == U && s.nt == NTF) {                                             \
        hipLaunchKernelGGL((sv_forward_kernel<TT, PHASE, WRITE, A, U, NTF>), grid, block, 0, st, a); \
        return;                                                                                    \
    }

template <typename T, bool PHASE, bool WRITE>
static void launch_fwd_t(const PassShape &s, int num_inst, const FwdArgs &a, hipStream_t st) {
    const dim3 grid(s.blocks_x, num_inst), block(kSvThreads);
    if constexpr (sizeof(T) == 4) {
        if constexpr (PHASE && WRITE) {  // the round pass: every compiled tuning shape
            if (a.counter && s.amp == 2 && s.unroll == 8 && s.nt == 1) {
                hipLaunchKernelGGL((sv_forward_kernel<T, true, true, 2, 8, 1, true>), grid, block, 0, st, a);
                return;
            }
            GQ_FWD_SHAPE(T, 2, 4, 1) GQ_FWD_SHAPE(T, 2, 16, 1) GQ_FWD_SHAPE(T, 2, 8, 0) GQ_FWD_SHAPE(T, 2, 16, 0)
            GQ_FWD_SHAPE(T, 4, 4, 1) GQ_FWD_SHAPE(T, 4, 4, 0)
        }
        if (s.unroll == 1) hipLaunchKernelGGL((sv_forward_kernel<T, PHASE, WRITE, 2, 1>), grid, block, 0, st, a);
        else if (s.unroll == 4) hipLaunchKernelGGL((sv_forward_kernel<T, PHASE, WRITE, 2, 4>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((sv_forward_kernel<T, PHASE, WRITE, 2, 8>), grid, block, 0, st, a);
    } else {
        if constexpr (PHASE && WRITE) {
            if (a.counter && s.amp == 1 && s.unroll == 8 && s.nt == 1) {
                hipLaunchKernelGGL((sv_forward_kernel<T, true, true, 1, 8, 1, true>), grid, block, 0, st, a);
                return;
            }
            GQ_FWD_SHAPE(T, 1, 4, 1) GQ_FWD_SHAPE(T, 1, 16, 1) GQ_FWD_SHAPE(T, 1, 8, 0) GQ_FWD_SHAPE(T, 2, 4, 1)
        }
        if (s.unroll == 1) hipLaunchKernelGGL((sv_forward_kernel<T, PHASE, WRITE, 1, 1>), grid, block, 0, st, a);
        else if (s.unroll == 4) hipLaunchKernelGGL((sv_forward_kernel<T, PHASE, WRITE, 1, 4>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((sv_forward_kernel<T, PHASE, WRITE, 1, 8>), grid, block, 0, st, a);
    }
}
#undef GQ_FWD_SHAPE

static void launch_fwd(int dtype, bool phase, bool write, const PassShape &s, int num_inst,
                       const FwdArgs &a, hipStream_t st) {
    if (dtype == GQAOA_C64) {
        if (phase) launch_fwd_t<float, true, true>(s, num_inst, a, st);
        else if (write) launch_fwd_t<float, false, true>(s, num_inst, a, st);
        else launch_fwd_t<float, false, false>(s, num_inst, a, st);
    } else {
        if (phase) launch_fwd_t<double, true, true>(s, num_inst, a, st);
        else if (write) launch_fwd_t<double, false, true>(s, num_inst, a, st);
        else launch_fwd_t<double, false, false>(s, num_inst, a, st);
    }
}

template <typename T, bool FIRST, bool WRITE>
static void launch_rev_t(const PassShape &s, int num_inst, const RevArgs &a, hipStream_t st) {
    const dim3 grid(s.blocks_x, num_inst), block(kSvThreads);
    if constexpr (sizeof(T) == 4) {
        if (s.unroll == 1) hipLaunchKernelGGL((sv_reverse_kernel<T, FIRST, WRITE, 2, 1>), grid, block, 0, st, a);
        else if (s.unroll == 4) hipLaunchKernelGGL((sv_reverse_kernel<T, FIRST, WRITE, 2, 4>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((sv_reverse_kernel<T, FIRST, WRITE, 2, 8>), grid, block, 0, st, a);
    } else {
        if (s.unroll == 1) hipLaunchKernelGGL((sv_reverse_kernel<T, FIRST, WRITE, 1, 1>), grid, block, 0, st, a);
        else if (s.unroll == 4) hipLaunchKernelGGL((sv_reverse_kernel<T, FIRST, WRITE, 1, 4>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((sv_reverse_kernel<T, FIRST, WRITE, 1, 8>), grid, block, 0, st, a);
    }
}

static void launch_rev(int dtype, bool first, bool write, const PassShape &s, int num_inst,
                       const RevArgs &a, hipStream_t st) {
    if (dtype == GQAOA_C64) {
        if (first) {
            if (write) launch_rev_t<float, true, true>(s, num_inst, a, st);
            else launch_rev_t<float, true, false>(s, num_inst, a, st);
        } else {
            if (write) launch_rev_t<float, false, true>(s, num_inst, a, st);
            else launch_rev_t<float, false, false>(s, num_inst, a, st);
        }
    } else {
        if (first) {
            if (write) launch_rev_t<double, true, true>(s, num_inst, a, st);
            else launch_rev_t<double, true, false>(s, num_inst, a, st);
        } else {
            if (write) launch_rev_t<double, false, true>(s, num_inst, a, st);
            else launch_rev_t<double, false, false>(s, num_inst, a, st);
        }
    }
}

// ---- workspace layout ---------------------------------------------------------------
// Small tables first (per instance), then the state slots used by the adjoint.
struct SvLayout {
    size_t lut, mixf, mixb, ebeta, delta, S, readout, T, eps, dbeta, dgamma, angles, target, counter, partials, folded;
    size_t slots, slot_bytes, nslots, total;
};

static size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

static SvLayout sv_layout(int num_inst, int n, int p, int dtype, int ckpt_every, bool grad) {
    SvLayout L{};
    const size_t cs = dtype == GQAOA_C64 ? 8 : 16;
    const size_t I = (size_t)num_inst;
    const size_t P = (size_t)std::max(p, 1);
    size_t o = 0;
    L.lut = o;      o += al256(I * P * 256 * cs);
    L.mixf = o;     o += al256(I * P * 16);
    L.mixb = o;     o += al256(I * P * 16);
    L.ebeta = o;    o += al256(I * P * 16);
    L.delta = o;    o += al256(I * (P + 1) * 16);
    L.S = o;        o += al256(I * (P + 1) * 16);
    L.readout = o;  o += al256(I * (P + 1) * 24);
    L.T = o;        o += al256(I * 16);
    L.eps = o;      o += al256(I * 16);
    L.dbeta = o;    o += al256(I * P * 8);
    L.dgamma = o;   o += al256(I * P * 8);
    L.angles = o;   o += al256(I * P * 16);   // beta[p] then gamma[p], uploaded by graph-plan runs
    L.target = o;   o += al256(I * 4);
    L.counter = o;  o += al256(I * 4);
    L.partials = o; o += al256(std::max<size_t>(kMaxPassBlocks, I) * kFwdR * 8);
    L.folded = o;   o += al256((kMaxPassBlocks / kFinThreads + I) * kFwdR * 8);  // rows left after a fold
    L.slots = o;
    L.slot_bytes = al256(I * ((size_t)1 << n) * cs);
    L.nslots = 0;
    if (grad) {
        const int c = (ckpt_every <= 0 || ckpt_every >= p) ? p : ckpt_every;
        const int nseg = (p + c - 1) / c;
        L.nslots = (size_t)(nseg - 1) /*checkpoints*/ + (size_t)c /*segment*/ +
                   (nseg > 1 ? 1 : 0) /*working*/ + 1 /*lambda*/;
    }
    L.total = o + L.nslots * L.slot_bytes;
    return L;
}

size_t sv_workspace_bytes(int num_inst, int n, int p, int dtype, int ckpt_every, bool grad) {
    return sv_layout(num_inst, n, p, dtype, ckpt_every, grad).total;
}

// Host tables: phase LUTs e^{-i gamma_j k} (k = 0..m, gamma_j k reduced mod 2 pi in
// double, rounded once to the state's precision), mixer factors per round.
static void build_tables(int num_inst, const int32_t *m_of, int p, const double *beta,
                         const double *gamma, int dtype, std::vector<char> &lut,
                         std::vector<double> &mixf, std::vector<double> &mixb,
                         std::vector<double> &ebeta) {
    const size_t cs = dtype == GQAOA_C64 ? 8 : 16;
    lut.assign((size_t)num_inst * p * 256 * cs, 0);
    mixf.assign((size_t)num_inst * p * 2, 0.0);
    mixb.assign((size_t)num_inst * p * 2, 0.0);
    ebeta.assign((size_t)num_inst * p * 2, 0.0);
    const double two_pi = 2.0 * M_PI;
    for (int i = 0; i < num_inst; ++i) {
        for (int j = 0; j < p; ++j) {
            const double g = gamma[(size_t)i * p + j], b = beta[(size_t)i * p + j];
            for (int k = 0; k <= m_of[i]; ++k) {
                const double ang = std::fmod(g * (double)k, two_pi);
                const double re = std::cos(ang), im = -std::sin(ang);
                const size_t e = ((size_t)i * p + j) * 256 + k;
                if (dtype == GQAOA_C64) {
                    float *f = reinterpret_cast<float *>(lut.data()) + 2 * e;
                    f[0] = (float)re;
                    f[1] = (float)im;
                } else {
                    double *d = reinterpret_cast<double *>(lut.data()) + 2 * e;
                    d[0] = re;
                    d[1] = im;
                }
            }
            const size_t q = ((size_t)i * p + j) * 2;
            mixf[q] = std::cos(b) - 1.0;
            mixf[q + 1] = -std::sin(b);
            mixb[q] = std::cos(b) - 1.0;
            mixb[q + 1] = std::sin(b);
            ebeta[q] = std::cos(b);
            ebeta[q + 1] = -std::sin(b);
        }
    }
}

static int upload(void *dst, const void *src, size_t bytes, hipStream_t st) {
    if (!bytes) return GQAOA_OK;
    GQ_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    return GQAOA_OK;
}

// ---- forward evolution (used by evolve and by the adjoint) -----------------------------
struct FwdPlan {
    int dtype, num_inst, n, p;
    uint64_t N;
    char *ws;
    SvLayout L;
    PassShape shape;
    const uint8_t *cost;
    int fuse_mode = 0;  // 0: the GQAOA_SV_FUSE switch decides, 1: fused when the shape allows, -1: never
};

static FwdArgs base_fwd_args(const FwdPlan &P) {
    FwdArgs a{};
    a.cost = P.cost;
    a.N = P.N;
    a.lut_stride = P.p * 256;
    a.lut_len = 256;
    a.delta_stride = 2 * (P.p + 1);
    a.init_amp = 1.0 / std::sqrt((double)P.N);
    a.target = reinterpret_cast<const int32_t *>(P.ws + P.L.target);
    a.partials = reinterpret_cast<double *>(P.ws + P.L.partials);
    return a;
}

static FinArgs base_fin_args(const FwdPlan &P) {
    FinArgs f{};
    f.partials = reinterpret_cast<double *>(P.ws + P.L.partials);
    f.nblocks = P.shape.blocks_x;
    f.inv_N = 1.0 / (double)P.N;
    f.mixf_stride = 2 * P.p;
    f.stride = 2 * (P.p + 1);
    f.readout_stride = 3 * (P.p + 1);
    f.mix_stride = 2 * P.p;
    f.grad_stride = P.p;
    return f;
}

// Finalize of a pass with P.shape.blocks_x partial rows per instance, folded
// first when one finalize block cannot take them all.
template <int R>
static int fold_for_finalize(const FwdPlan &P, const double *rows, const double **out, int *out_rows,
                             hipStream_t st) {
    const int n = P.shape.blocks_x;
    if (n <= kFinThreads) {
        *out = rows;
        *out_rows = n;
        return GQAOA_OK;
    }
    const int nfold = (n + kFinThreads - 1) / kFinThreads;
    double *q = reinterpret_cast<double *>(P.ws + P.L.folded);
    hipLaunchKernelGGL(fold_partials_kernel<R>, dim3(nfold, P.num_inst), dim3(kFinThreads), 0, st, rows, n, q, nfold);
    GQ_LAUNCH_CHECK();
    *out = q;
    *out_rows = nfold;
    return GQAOA_OK;
}

static int launch_finalize(const FwdPlan &P, FinArgs f, hipStream_t st) {
    int s = fold_for_finalize<kFwdR>(P, f.partials, &f.partials, &f.nblocks, st);
    if (s) return s;
    // the smallest block that holds one row per thread (the rows past
    // nblocks add zeros in a larger one, so the sums are the same bits)
    if (f.nblocks <= kFinWave) hipLaunchKernelGGL(sv_finalize_kernel<kFinWave>, dim3(P.num_inst), dim3(kFinWave), 0, st, f);
    else if (f.nblocks <= 2 * kFinWave)
        hipLaunchKernelGGL(sv_finalize_kernel<2 * kFinWave>, dim3(P.num_inst), dim3(2 * kFinWave), 0, st, f);
    else hipLaunchKernelGGL(sv_finalize_kernel<kFinThreads>, dim3(P.num_inst), dim3(kFinThreads), 0, st, f);
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

// GQAOA_SV_FUSE=1 folds the finalize into the last block of the round pass
// (one launch per round, on the persistent grid). It is off by default: the
// release fence each block needs before counting itself done writes back its
// XCD's L2, which costs more bandwidth than the separate finalize launch saves
// (0.99 vs 0.75 ms per round at n = 28, complex64).
static bool fuse_requested() {
    const char *e = getenv("GQAOA_SV_FUSE");
    return e && e[0] == '1';
}

static bool fused_round(const FwdPlan &P) {
    if (P.fuse_mode < 0) return false;
    if (P.fuse_mode == 0 && !fuse_requested()) return false;
    const PassShape &s = P.shape;
    return s.unroll == 8 && s.nt == 1 && s.amp == (P.dtype == GQAOA_C64 ? 2 : 1);
}

// One forward round j (1-based): psi_in holds phi_{j-1} (or |s> if j == 1 and
// uniform), psi_out receives phi_j. With finalize, writes delta_j, S_j and the
// readout of round j-1.
static int forward_round(const FwdPlan &P, int j, const void *psi_in, void *psi_out, bool uniform,
                         bool finalize, hipStream_t st) {
    const size_t cs = P.dtype == GQAOA_C64 ? 8 : 16;
    FwdArgs a = base_fwd_args(P);
    a.psi_in = psi_in;
    a.psi_out = psi_out;
    a.lut = P.ws + P.L.lut + (size_t)(j - 1) * 256 * cs;
    a.delta = j > 1 ? reinterpret_cast<double *>(P.ws + P.L.delta) + 2 * (j - 1) : nullptr;
    a.init_uniform = uniform ? 1 : 0;
    FinArgs f = base_fin_args(P);
    f.mixf = reinterpret_cast<double *>(P.ws + P.L.mixf) + 2 * (j - 1);
    f.delta_out = reinterpret_cast<double *>(P.ws + P.L.delta) + 2 * j;
    f.S_out = reinterpret_cast<double *>(P.ws + P.L.S) + 2 * j;
    f.readout_out = reinterpret_cast<double *>(P.ws + P.L.readout) + 3 * (j - 1);
    const bool fused = finalize && fused_round(P);
    if (fused) {
        a.counter = reinterpret_cast<unsigned int *>(P.ws + P.L.counter);
        a.fin = f;
    }
    ProfScope ps(P.dtype == GQAOA_C64 ? "sv_round_c64" : "sv_round_c128", st);
    launch_fwd(P.dtype, true, true, P.shape, P.num_inst, a, st);
    ps.end();
    GQ_LAUNCH_CHECK();
    if (finalize && !fused) return launch_finalize(P, f, st);
    return GQAOA_OK;
}

// Final pass: psi_out = phi_p + delta_p (if write), readout of round p.
static int final_pass(const FwdPlan &P, const void *psi_in, void *psi_out, bool uniform, bool write,
                      hipStream_t st) {
    FwdArgs a = base_fwd_args(P);
    a.psi_in = psi_in;
    a.psi_out = psi_out;
    a.lut = nullptr;
    a.delta = P.p > 0 ? reinterpret_cast<double *>(P.ws + P.L.delta) + 2 * P.p : nullptr;
    a.init_uniform = uniform ? 1 : 0;
    launch_fwd(P.dtype, false, write, P.shape, P.num_inst, a, st);
    GQ_LAUNCH_CHECK();
    FinArgs f = base_fin_args(P);
    f.readout_out = reinterpret_cast<double *>(P.ws + P.L.readout) + 3 * P.p;
    return launch_finalize(P, f, st);
}

static int prepare_plan(FwdPlan &P, int num_inst, int n, const int32_t *m_of, const uint8_t *cost,
                        int p, const double *beta, const double *gamma, int dtype,
                        const int32_t *targets, void *ws, int ckpt_every, bool grad,
                        hipStream_t st, std::vector<char> &keep_lut, std::vector<double> &keep_f,
                        std::vector<double> &keep_b, std::vector<double> &keep_e,
                        std::vector<int32_t> &keep_t) {
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    P.dtype = dtype;
    P.num_inst = num_inst;
    P.n = n;
    P.p = p;
    P.N = 1ull << n;
    P.ws = reinterpret_cast<char *>(ws);
    P.L = sv_layout(num_inst, n, p, dtype, ckpt_every, grad);
    P.shape = pass_shape(P.N, num_inst, dtype, dev, fuse_requested());
    P.cost = cost;
    if (p > 0) {
        build_tables(num_inst, m_of, p, beta, gamma, dtype, keep_lut, keep_f, keep_b, keep_e);
        // the LUT block is laid out [inst][p][256]; the kernels index it with lut_stride p*256
        if ((s = upload(P.ws + P.L.lut, keep_lut.data(), keep_lut.size(), st))) return s;
        if ((s = upload(P.ws + P.L.mixf, keep_f.data(), keep_f.size() * 8, st))) return s;
        if ((s = upload(P.ws + P.L.mixb, keep_b.data(), keep_b.size() * 8, st))) return s;
        if ((s = upload(P.ws + P.L.ebeta, keep_e.data(), keep_e.size() * 8, st))) return s;
    }
    keep_t.assign(targets, targets + num_inst);
    if ((s = upload(P.ws + P.L.target, keep_t.data(), keep_t.size() * 4, st))) return s;
    GQ_HIP(hipMemsetAsync(P.ws + P.L.delta, 0, (size_t)num_inst * (p + 1) * 16, st));
    GQ_HIP(hipMemsetAsync(P.ws + P.L.counter, 0, (size_t)num_inst * 4, st));
    return GQAOA_OK;
}

// ---- entry points (validated by the ABI layer) ---------------------------------------------
int run_evolve(int n, int m, const uint8_t *cost, int p, const double *beta, const double *gamma,
               int dtype, int init_uniform, void *psi, int target, double *psol, double *energy,
               double *norm, void *ws, hipStream_t st) {
    FwdPlan P;
    std::vector<char> lut;
    std::vector<double> f, b, e;
    std::vector<int32_t> t;
    int32_t m_of[1] = {m};
    int32_t tg[1] = {target};
    int s = prepare_plan(P, 1, n, m_of, cost, p, beta, gamma, dtype, tg, ws, 0, false, st, lut, f, b, e, t);
    if (s) return s;
    if (resident_ok(n, dtype, p)) {
        ResArgs r{cost, psi, P.ws + P.L.lut, reinterpret_cast<const double *>(P.ws + P.L.mixf),
                  reinterpret_cast<double *>(P.ws + P.L.readout), n, p, init_uniform ? 1 : 0, target};
        if ((s = launch_resident(dtype, r, st))) return s;
    } else {
        for (int j = 1; j <= p; ++j)
            if ((s = forward_round(P, j, psi, psi, init_uniform && j == 1, true, st))) return s;
        const bool write = p > 0 || init_uniform;
        if ((s = final_pass(P, psi, psi, init_uniform && p == 0, write, st))) return s;
    }
    std::vector<double> ro((size_t)(p + 1) * 3);
    GQ_HIP(hipMemcpyAsync(ro.data(), P.ws + P.L.readout, ro.size() * 8, hipMemcpyDeviceToHost, st));
    GQ_HIP(hipStreamSynchronize(st));
    if (prof_on()) prof_collect();
    for (int j = 0; j <= p; ++j) {
        if (psol) psol[j] = ro[3 * j];
        if (energy) energy[j] = ro[3 * j + 1];
        if (norm) norm[j] = ro[3 * j + 2];
    }
    return GQAOA_OK;
}

int run_solution_prob(int n, const uint8_t *cost, const void *psi, int dtype, int target,
                      double *out, void *ws, hipStream_t st) {
    FwdPlan P;
    std::vector<char> lut;
    std::vector<double> f, b, e;
    std::vector<int32_t> t;
    int32_t m_of[1] = {255};
    int32_t tg[1] = {target};
    int s = prepare_plan(P, 1, n, m_of, cost, 0, nullptr, nullptr, dtype, tg, ws, 0, false, st, lut, f, b, e, t);
    if (s) return s;
    if ((s = final_pass(P, psi, const_cast<void *>(psi), false, false, st))) return s;
    double ro[3];
    GQ_HIP(hipMemcpyAsync(ro, P.ws + P.L.readout, 24, hipMemcpyDeviceToHost, st));
    GQ_HIP(hipStreamSynchronize(st));
    *out = ro[0];
    return GQAOA_OK;
}

int run_grad(int num_inst, int n, const int32_t *m_of, const uint8_t *cost, int p,
             const double *beta, const double *gamma, int dtype, const int32_t *targets,
             int ckpt_every, double *psol, double *dbeta, double *dgamma, void *ws, hipStream_t st) {
    FwdPlan P;
    std::vector<char> lut;
    std::vector<double> f, b, e;
    std::vector<int32_t> t;
    int s = prepare_plan(P, num_inst, n, m_of, cost, p, beta, gamma, dtype, targets, ws, ckpt_every,
                         true, st, lut, f, b, e, t);
    if (s) return s;
    const int c = (ckpt_every <= 0 || ckpt_every >= p) ? p : ckpt_every;
    const int nseg = (p + c - 1) / c;
    auto slot = [&](size_t k) { return (void *)(P.ws + P.L.slots + k * P.L.slot_bytes); };
    // slots: [0, nseg-1) checkpoints phi_{s c} for s = 1..nseg-1; then c segment
    // slots; then the working slot (if nseg > 1); then lambda.
    const size_t seg0 = (size_t)(nseg - 1);
    const size_t work = seg0 + (size_t)c;
    const size_t lam = work + (nseg > 1 ? 1 : 0);
    const int k0_last = (nseg - 1) * c;
    auto seg_slot = [&](int k, int k0) { return slot(seg0 + (size_t)(k - k0 - 1)); };

    // forward sweep
    const void *prev = nullptr;
    for (int k = 1; k <= p; ++k) {
        void *out;
        if (k > k0_last) out = seg_slot(k, k0_last);
        else if (k % c == 0) out = slot((size_t)(k / c - 1));
        else out = slot(work);
        if ((s = forward_round(P, k, k == 1 ? out : prev, out, k == 1, true, st))) return s;
        prev = out;
    }
    // readout of round p and adjoint set-up (eps_p, dbeta_p); the target sum T
    // is taken from the final state's level-t amplitudes.
    {
        FwdArgs a = base_fwd_args(P);
        a.psi_in = prev;
        a.psi_out = nullptr;
        a.lut = nullptr;
        a.delta = reinterpret_cast<double *>(P.ws + P.L.delta) + 2 * p;
        launch_fwd(P.dtype, false, false, P.shape, P.num_inst, a, st);
        GQ_LAUNCH_CHECK();
        FinArgs fa = base_fin_args(P);
        fa.readout_out = reinterpret_cast<double *>(P.ws + P.L.readout) + 3 * p;
        fa.mixb = reinterpret_cast<double *>(P.ws + P.L.mixb) + 2 * (p - 1);
        fa.ebeta = reinterpret_cast<double *>(P.ws + P.L.ebeta) + 2 * (p - 1);
        fa.S_p = reinterpret_cast<double *>(P.ws + P.L.S) + 2 * p;
        fa.stride = 2 * (p + 1);
        fa.eps_out = reinterpret_cast<double *>(P.ws + P.L.eps);
        fa.dbeta_out = reinterpret_cast<double *>(P.ws + P.L.dbeta) + (p - 1);
        if ((s = launch_finalize(P, fa, st))) return s;
    }
    // reverse sweep, segment by segment
    const size_t cs = dtype == GQAOA_C64 ? 8 : 16;
    for (int sg = nseg - 1; sg >= 0; --sg) {
        const int k0 = sg * c, k1 = std::min(p, k0 + c);
        if (sg != nseg - 1) {  // recompute phi_{k0+1..k1} from the checkpoint
            for (int k = k0 + 1; k <= k1; ++k) {
                const void *in = k == k0 + 1 ? (k0 == 0 ? seg_slot(k, k0) : slot((size_t)(k0 / c - 1)))
                                             : seg_slot(k - 1, k0);
                if ((s = forward_round(P, k, in, seg_slot(k, k0), k == 1, false, st))) return s;
            }
        }
        for (int k = k1; k >= k0 + 1; --k) {
            RevArgs r{};
            r.cost = P.cost;
            r.phi = seg_slot(k, k0);
            r.lam_in = k == p ? nullptr : slot(lam);
            r.lam_out = slot(lam);
            r.N = P.N;
            r.lut = P.ws + P.L.lut + (size_t)(k - 1) * 256 * cs;
            r.lut_stride = p * 256;
            r.lut_len = 256;
            r.eps = reinterpret_cast<double *>(P.ws + P.L.eps);
            r.eps_stride = 2;
            r.delta_p = reinterpret_cast<double *>(P.ws + P.L.delta) + 2 * p;
            r.delta_stride = 2 * (p + 1);
            r.target = reinterpret_cast<const int32_t *>(P.ws + P.L.target);
            r.partials = reinterpret_cast<double *>(P.ws + P.L.partials);
            ProfScope ps(dtype == GQAOA_C64 ? "sv_reverse_c64" : "sv_reverse_c128", st);
            launch_rev(dtype, k == p, k > 1, P.shape, P.num_inst, r, st);
            ps.end();
            GQ_LAUNCH_CHECK();
            RevFinArgs rf{};
            rf.partials = r.partials;
            rf.nblocks = P.shape.blocks_x;
            rf.inv_N = 1.0 / (double)P.N;
            rf.dgamma_k = reinterpret_cast<double *>(P.ws + P.L.dgamma) + (k - 1);
            rf.grad_stride = p;
            if (k > 1) {
                rf.mixb_km1 = reinterpret_cast<double *>(P.ws + P.L.mixb) + 2 * (k - 2);
                rf.ebeta_km1 = reinterpret_cast<double *>(P.ws + P.L.ebeta) + 2 * (k - 2);
                rf.S_km1 = reinterpret_cast<double *>(P.ws + P.L.S) + 2 * (k - 1);
                rf.S_stride = 2 * (p + 1);
                rf.eps_out = reinterpret_cast<double *>(P.ws + P.L.eps);
                rf.dbeta_km1 = reinterpret_cast<double *>(P.ws + P.L.dbeta) + (k - 2);
            }
            if ((s = fold_for_finalize<kRevR>(P, rf.partials, &rf.partials, &rf.nblocks, st))) return s;
            if (rf.nblocks <= kFinWave)
                hipLaunchKernelGGL(sv_rev_finalize_kernel<kFinWave>, dim3(P.num_inst), dim3(kFinWave), 0, st, rf);
            else
                hipLaunchKernelGGL(sv_rev_finalize_kernel<kFinThreads>, dim3(P.num_inst), dim3(kFinThreads), 0, st, rf);
            GQ_LAUNCH_CHECK();
        }
    }
    std::vector<double> ro((size_t)num_inst * (p + 1) * 3), db((size_t)num_inst * p), dg((size_t)num_inst * p);
    GQ_HIP(hipMemcpyAsync(ro.data(), P.ws + P.L.readout, ro.size() * 8, hipMemcpyDeviceToHost, st));
    GQ_HIP(hipMemcpyAsync(db.data(), P.ws + P.L.dbeta, db.size() * 8, hipMemcpyDeviceToHost, st));
    GQ_HIP(hipMemcpyAsync(dg.data(), P.ws + P.L.dgamma, dg.size() * 8, hipMemcpyDeviceToHost, st));
    GQ_HIP(hipStreamSynchronize(st));
    if (prof_on()) prof_collect();
    for (int i = 0; i < num_inst; ++i) {
        if (psol) psol[i] = ro[((size_t)i * (p + 1) + p) * 3];
        for (int k = 0; k < p; ++k) {
            if (dbeta) dbeta[(size_t)i * p + k] = db[(size_t)i * p + k];
            if (dgamma) dgamma[(size_t)i * p + k] = dg[(size_t)i * p + k];
        }
    }
    return GQAOA_OK;
}

// ---- graph-captured evolution ------------------------------------------------------------
// For callers that evolve one instance many times with new angles (angle
// searches at small n, where each round pass is a few microseconds and the
// launches dominate): the whole call — angle tables, p round passes with
// their finalizes, the final readout pass — is captured once into a HIP
// graph. A run uploads the 2p angles, replays the graph and reads back the
// readouts; the tables are computed on the device from the angles, with the
// same float64 reduction and rounding as the host tables of run_evolve.
// Block (j, i): round j of instance i; ang[i] = (beta[p], gamma[p]), the
// instance's m from m_dev (or m_all when m_dev is null); tables [i][p][256]
// and [i][p][2].
template <typename T>
__global__ void __launch_bounds__(256) evolve_tables_kernel(const double *__restrict__ ang, int p,
                                                            const int32_t *__restrict__ m_dev, int m_all,
                                                            T *__restrict__ lut, double *__restrict__ mixf) {
    const int j = blockIdx.x, k = threadIdx.x, i = blockIdx.y;
    const int m = m_dev ? m_dev[i] : m_all;
    ang += (size_t)i * 2 * p;
    lut += (size_t)i * p * 256 * 2;
    mixf += (size_t)i * p * 2;
    T re = 0, im = 0;
    if (k <= m) {
        double sn, cs;
        sincos(fmod(ang[p + j] * (double)k, 2.0 * M_PI), &sn, &cs);
        re = (T)cs;
        im = (T)-sn;
    }
    lut[2 * ((size_t)j * 256 + k)] = re;
    lut[2 * ((size_t)j * 256 + k) + 1] = im;
    if (k == 0) {
        double sb, cb;
        sincos(ang[j], &sb, &cb);
        mixf[2 * j] = cb - 1.0;
        mixf[2 * j + 1] = -sb;
    }
}

struct EvolvePlan {
    FwdPlan P;
    int device = -1, m = 0;
    int target_host[1] = {0};
    double *stage = nullptr;  // pinned: angles [2p], then readouts [(p+1) * 3]
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
};

void evolve_plan_destroy(EvolvePlan *E) {
    if (!E) return;
    if (E->exec) (void)hipGraphExecDestroy(E->exec);
    if (E->graph) (void)hipGraphDestroy(E->graph);
    if (E->cap) {
        // back to the pool once the graph was instantiated (its capture has
        // ended); destroyed after a failed creation
        if (E->exec) stream_pool_give(E->device, {E->cap});
        else (void)hipStreamDestroy(E->cap);
    }
    if (E->stage) (void)hipHostFree(E->stage);
    delete E;
}

struct EvolvePlanGuard {
    EvolvePlan *e;
    hipStream_t st;
    ~EvolvePlanGuard() {
        if (!e) return;
        (void)hipStreamSynchronize(st);
        evolve_plan_destroy(e);
    }
};

static int enqueue_evolve(EvolvePlan *E, int init_uniform, void *psi, hipStream_t st) {
    FwdPlan &P = E->P;
    const double *ang = reinterpret_cast<const double *>(P.ws + P.L.angles);
    double *mixf = reinterpret_cast<double *>(P.ws + P.L.mixf);
    if (P.dtype == GQAOA_C64)
        hipLaunchKernelGGL(evolve_tables_kernel<float>, dim3(P.p), dim3(256), 0, st, ang, P.p, nullptr, E->m,
                           reinterpret_cast<float *>(P.ws + P.L.lut), mixf);
    else
        hipLaunchKernelGGL(evolve_tables_kernel<double>, dim3(P.p), dim3(256), 0, st, ang, P.p, nullptr, E->m,
                           reinterpret_cast<double *>(P.ws + P.L.lut), mixf);
    GQ_LAUNCH_CHECK();
    if (resident_ok(P.n, P.dtype, P.p)) {
        ResArgs r{P.cost, psi, P.ws + P.L.lut, mixf, reinterpret_cast<double *>(P.ws + P.L.readout), P.n, P.p,
                  init_uniform, *E->target_host};
        return launch_resident(P.dtype, r, st);
    }
    int s;
    for (int j = 1; j <= P.p; ++j)
        if ((s = forward_round(P, j, psi, psi, init_uniform && j == 1, true, st))) return s;
    return final_pass(P, psi, psi, false, true, st);
}

int evolve_plan_create(int n, int m, const uint8_t *cost, int p, int dtype, int init_uniform, void *psi, int target,
                       void *ws, hipStream_t st, EvolvePlan **out) {
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    EvolvePlanGuard G{new (std::nothrow) EvolvePlan, st};
    if (!G.e) return fail(GQAOA_EINVAL, "out of host memory");
    EvolvePlan *E = G.e;
    E->device = dev.device;
    E->m = m;
    E->target_host[0] = target;
    FwdPlan &P = E->P;
    P.dtype = dtype;
    P.num_inst = 1;
    P.n = n;
    P.p = p;
    P.N = 1ull << n;
    P.ws = reinterpret_cast<char *>(ws);
    P.L = sv_layout(1, n, p, dtype, 0, false);
    P.cost = cost;
    // The round passes with their separate fold / finalize launches: on the
    // one-tile grid they replay faster than the fused finalize at every size
    // measured (n = 16..22, complex64).
    P.fuse_mode = -1;
    P.shape = pass_shape(P.N, 1, dtype, dev);
    GQ_HIP(hipHostMalloc(reinterpret_cast<void **>(&E->stage), sizeof(double) * (2 * (size_t)p + 3 * ((size_t)p + 1)),
                         hipHostMallocDefault));
    {
        std::vector<hipStream_t> c;
        s = stream_pool_take(1, &c);
        if (!c.empty()) E->cap = c[0];
        if (s) return s;
    }
    const int32_t tg = target;
    GQ_HIP(hipMemcpyAsync(P.ws + P.L.target, &tg, 4, hipMemcpyHostToDevice, st));
    GQ_HIP(hipStreamSynchronize(st));  // tg ends here; the captured work reads the target from the workspace
    GQ_HIP(hipStreamBeginCapture(E->cap, hipStreamCaptureModeThreadLocal));
    s = enqueue_evolve(E, init_uniform, psi, E->cap);
    hipGraph_t graph = nullptr;
    const hipError_t e_end = hipStreamEndCapture(E->cap, &graph);
    E->graph = graph;
    if (s) return s;
    GQ_HIP(e_end);
    GQ_HIP(hipGraphInstantiate(&E->exec, E->graph, nullptr, nullptr, 0));
    *out = E;
    G.e = nullptr;
    return GQAOA_OK;
}

int evolve_plan_run(EvolvePlan *E, const double *beta, const double *gamma, double *psol, double *energy,
                    double *norm, hipStream_t st) {
    int cur = -1;
    GQ_HIP(hipGetDevice(&cur));
    if (cur != E->device) return fail(GQAOA_EINVAL, "plan made on device %d, current device is %d", E->device, cur);
    const int p = E->P.p;
    for (int j = 0; j < p; ++j)
        if (!std::isfinite(beta[j]) || !std::isfinite(gamma[j])) return fail(GQAOA_EINVAL, "non-finite angle in round %d", j + 1);
    double *ang = E->stage, *ro = E->stage + 2 * (size_t)p;
    std::copy(beta, beta + p, ang);
    std::copy(gamma, gamma + p, ang + p);
    const FwdPlan &P = E->P;
    GQ_HIP(hipMemcpyAsync(P.ws + P.L.angles, ang, 16 * (size_t)p, hipMemcpyHostToDevice, st));
    GQ_HIP(hipGraphLaunch(E->exec, st));
    GQ_HIP(hipMemcpyAsync(ro, P.ws + P.L.readout, 24 * ((size_t)p + 1), hipMemcpyDeviceToHost, st));
    GQ_HIP(hipStreamSynchronize(st));
    for (int j = 0; j <= p; ++j) {
        if (psol) psol[j] = ro[3 * j];
        if (energy) energy[j] = ro[3 * j + 1];
        if (norm) norm[j] = ro[3 * j + 2];
    }
    return GQAOA_OK;
}

// ---- streamed statevector work items (states too large for registers) --------------------
// Single-angle-pair items of one size n, evolved together: item k is
// instance k of a batched streaming evolution (its own cost table copy,
// state, tables and target), complex64, p = p_list[num_p-1] rounds from |s>;
// the readouts at p_list go to the items' output rows.
__global__ void gather_costs_kernel(const uint8_t *__restrict__ costs, const uint64_t *__restrict__ off, uint64_t N,
                                    uint8_t *__restrict__ dst) {
    const uint8_t *src = costs + off[blockIdx.y];
    uint8_t *d = dst + (uint64_t)blockIdx.y * N;
    for (uint64_t z = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; z < N; z += (uint64_t)gridDim.x * blockDim.x)
        d[z] = src[z];
}

__global__ void gather_readouts_kernel(const double *__restrict__ ro, int p, int count, const int32_t *__restrict__ out,
                                       const int32_t *__restrict__ p_list, int num_p, float *__restrict__ psol,
                                       float *__restrict__ energy) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count * num_p) return;
    const int k = t / num_p, q = t % num_p;
    const double *r = ro + (size_t)k * 3 * (p + 1) + 3 * (size_t)p_list[q];
    psol[(size_t)out[k] * num_p + q] = (float)r[0];
    if (energy) energy[(size_t)out[k] * num_p + q] = (float)r[1];
}

int sv_items_stream(int n, int count, const int32_t *item_inst, const int32_t *item_out, const double *beta,
                    const double *gamma, const uint8_t *costs, const uint64_t *cost_off, const int32_t *m_host,
                    const int32_t *target_host, int num_p, const int32_t *p_list, float *psol, float *energy,
                    hipStream_t st) {
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    const int p = p_list[num_p - 1];
    const uint64_t N = 1ull << n;
    // chunks of items whose states and cost copies stay within 4 GiB
    const int chunk = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)count, (4ull << 30) / (9 * N)));
    for (int c0 = 0; c0 < count; c0 += chunk) {
        const int cnt = std::min(chunk, count - c0);
        FwdPlan P;
        P.dtype = GQAOA_C64;
        P.num_inst = cnt;
        P.n = n;
        P.p = p;
        P.N = N;
        P.L = sv_layout(cnt, n, p, GQAOA_C64, 0, false);
        P.shape = pass_shape(N, cnt, GQAOA_C64, dev);
        P.fuse_mode = -1;
        auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
        const size_t o_cost = al(P.L.total), o_psi = o_cost + al(cnt * N), o_off = o_psi + al(cnt * N * 8);
        const size_t o_m = o_off + al(8 * (size_t)cnt), o_out = o_m + al(4 * (size_t)cnt);
        const size_t o_pl = o_out + al(4 * (size_t)cnt), total = o_pl + al(4 * (size_t)num_p);
        AsyncScratch guard(st);
        GQ_HIP(guard.alloc(total));
        char *base = reinterpret_cast<char *>(guard.ptr);
        P.ws = base;
        P.cost = reinterpret_cast<const uint8_t *>(base + o_cost);
        std::vector<uint64_t> off(cnt);
        std::vector<int32_t> m(cnt), tg(cnt), out(cnt);
        std::vector<double> ang((size_t)cnt * 2 * p);
        for (int k = 0; k < cnt; ++k) {
            const int i = item_inst[c0 + k];
            off[k] = cost_off[i];
            m[k] = m_host[i];
            tg[k] = target_host ? target_host[i] : 0;
            out[k] = item_out[c0 + k];
            std::fill(ang.begin() + (size_t)k * 2 * p, ang.begin() + (size_t)k * 2 * p + p, beta[c0 + k]);
            std::fill(ang.begin() + (size_t)k * 2 * p + p, ang.begin() + (size_t)(k + 1) * 2 * p, gamma[c0 + k]);
        }
        GQ_HIP(hipMemcpyAsync(base + o_off, off.data(), 8 * (size_t)cnt, hipMemcpyHostToDevice, st));
        GQ_HIP(hipMemcpyAsync(base + o_m, m.data(), 4 * (size_t)cnt, hipMemcpyHostToDevice, st));
        GQ_HIP(hipMemcpyAsync(base + o_out, out.data(), 4 * (size_t)cnt, hipMemcpyHostToDevice, st));
        GQ_HIP(hipMemcpyAsync(base + o_pl, p_list, 4 * (size_t)num_p, hipMemcpyHostToDevice, st));
        GQ_HIP(hipMemcpyAsync(base + P.L.target, tg.data(), 4 * (size_t)cnt, hipMemcpyHostToDevice, st));
        GQ_HIP(hipMemcpyAsync(base + P.L.angles, ang.data(), 8 * ang.size(), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(gather_costs_kernel, dim3((unsigned)std::min<uint64_t>(1024, (N + 255) / 256), cnt),
                           dim3(256), 0, st, costs, reinterpret_cast<const uint64_t *>(base + o_off), N,
                           reinterpret_cast<uint8_t *>(base + o_cost));
        GQ_LAUNCH_CHECK();
        hipLaunchKernelGGL(evolve_tables_kernel<float>, dim3(p, cnt), dim3(256), 0, st,
                           reinterpret_cast<const double *>(base + P.L.angles), p,
                           reinterpret_cast<const int32_t *>(base + o_m), 0, reinterpret_cast<float *>(base + P.L.lut),
                           reinterpret_cast<double *>(base + P.L.mixf));
        GQ_LAUNCH_CHECK();
        void *psi = base + o_psi;
        for (int j = 1; j <= p; ++j)
            if ((s = forward_round(P, j, psi, psi, j == 1, true, st))) return s;
        if ((s = final_pass(P, psi, psi, false, false, st))) return s;
        hipLaunchKernelGGL(gather_readouts_kernel, dim3((cnt * num_p + 255) / 256), dim3(256), 0, st,
                           reinterpret_cast<const double *>(base + P.L.readout), p, cnt,
                           reinterpret_cast<const int32_t *>(base + o_out),
                           reinterpret_cast<const int32_t *>(base + o_pl), num_p, psol, energy);
        GQ_LAUNCH_CHECK();
        GQ_HIP(hipStreamSynchronize(st));  // the host tables of this chunk end here
    }
    return GQAOA_OK;
}

}  // namespace gqaoa
