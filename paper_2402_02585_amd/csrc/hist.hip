// Level-space ("effective space") G-QAOA, App. C "Optimization".
//
// From |s>, every amplitude depends on z only through the level C(z) = k, so
// the state is one amplitude b_k per occupied level with weight
// w_k = N_k / 2^n. A round (Eq. (3)) is b_k <- e^{-i gamma k} b_k, then
// b_k <- b_k + (e^{-i beta} - 1) S with S = sum_k w_k b_k (= <s|psi>).
// Readouts: P_sol = w_t |b_t|^2, E = sum_k k w_k |b_k|^2 (Eq. (4)).
//
// gqaoa_hist_evolve: one instance, float64, one wave; lanes own levels and
// S is a wave reduction per round.
// gqaoa_scan_batched: the single-angle-pair protocol (Eq. (5)) for every
// (instance, gamma, beta) triple, float32. A wave takes one (instance, gamma,
// 64-beta tile) work item from a global counter; gamma is wave-uniform, so the
// phase/weight table lives in LDS and is read as broadcasts, while each lane
// holds its own beta's K level amplitudes in registers. Instances are
// bucketed by padded level count (a register-array size per kernel
// instantiation) and, inside a bucket, ordered by level count descending so
// the dynamic queue ends with the short items.
#include "batch.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

namespace gqaoa {

// ---- single instance, float64 ------------------------------------------------------
// rounds[j] = {cos g_j, -sin g_j, cos b_j - 1, -sin b_j} is not enough for exact
// phases at every level, so the host passes, per round, e^{-i gamma_j 2^t} for
// t = 0..7 (each reduced mod 2 pi in double); level k multiplies the powers
// selected by its bits.
struct HistRound {
    double pw[8][2];   // e^{-i gamma 2^t}
    double mix[2];     // e^{-i beta} - 1
    int same_gamma;    // gamma equal to the previous round's: phases unchanged
    int pad;
};

__global__ void __launch_bounds__(64)
hist_evolve_kernel(const unsigned long long *__restrict__ hist, int m, int n, int p,
                   const HistRound *__restrict__ rounds, int target, double *__restrict__ out) {
    const int lane = threadIdx.x;
    constexpr int kPer = 4;  // levels per lane: k = lane + 64 i
    const double invN = std::ldexp(1.0, -n);
    double w[kPer], br[kPer], bi[kPer], pr[kPer], pi_[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int k = lane + 64 * i;
        w[i] = k <= m ? (double)hist[k] * invN : 0.0;
        br[i] = 1.0;
        bi[i] = 0.0;
        pr[i] = 1.0;
        pi_[i] = 0.0;
    }
    auto readout = [&](int j) {
        double P = 0, E = 0, Nn = 0;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int k = lane + 64 * i;
            const double pb = w[i] * (br[i] * br[i] + bi[i] * bi[i]);
            Nn += pb;
            E += (double)k * pb;
            P += k == target ? pb : 0.0;
        }
        P = wave_sum_dpp(P);  // the one-wave block is converged here
        E = wave_sum_dpp(E);
        Nn = wave_sum_dpp(Nn);
        if (lane == 0) {
            out[3 * j] = P;
            out[3 * j + 1] = E;
            out[3 * j + 2] = Nn;
        }
    };
    readout(0);
    for (int j = 0; j < p; ++j) {
        const HistRound &R = rounds[j];
        if (!R.same_gamma) {
#pragma unroll
            for (int i = 0; i < kPer; ++i) {
                const int k = lane + 64 * i;
                double xr = 1.0, xi = 0.0;
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if ((k >> t) & 1) {
                        const double yr = xr * R.pw[t][0] - xi * R.pw[t][1];
                        xi = xr * R.pw[t][1] + xi * R.pw[t][0];
                        xr = yr;
                    }
                pr[i] = xr;
                pi_[i] = xi;
            }
        }
        double sr = 0, si = 0;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const double nr = pr[i] * br[i] - pi_[i] * bi[i];
            bi[i] = pr[i] * bi[i] + pi_[i] * br[i];
            br[i] = nr;
            sr += w[i] * br[i];
            si += w[i] * bi[i];
        }
        sr = wave_sum_dpp(sr);
        si = wave_sum_dpp(si);
        const double cr = R.mix[0] * sr - R.mix[1] * si, ci = R.mix[0] * si + R.mix[1] * sr;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            br[i] += cr;
            bi[i] += ci;
        }
        readout(j + 1);
    }
}

int run_hist_evolve(int n, int m, const uint64_t *hist, int p, const double *beta,
                    const double *gamma, int target, double *psol, double *energy, double *norm,
                    hipStream_t st) {
    std::vector<HistRound> rounds((size_t)std::max(p, 1));
    const double two_pi = 2.0 * M_PI;
    for (int j = 0; j < p; ++j) {
        HistRound &R = rounds[j];
        for (int t = 0; t < 8; ++t) {
            const double a = std::fmod(gamma[j] * (double)(1 << t), two_pi);
            R.pw[t][0] = std::cos(a);
            R.pw[t][1] = -std::sin(a);
        }
        R.mix[0] = std::cos(beta[j]) - 1.0;
        R.mix[1] = -std::sin(beta[j]);
        R.same_gamma = (j > 0 && gamma[j] == gamma[j - 1]) ? 1 : 0;
        R.pad = 0;
    }
    const size_t rb = sizeof(HistRound) * rounds.size();
    const size_t ob = sizeof(double) * 3 * (size_t)(p + 1);
    AsyncScratch guard(st);
    GQ_HIP(guard.alloc(rb + ob + 256));
    char *base = reinterpret_cast<char *>(guard.ptr);
    double *d_out = reinterpret_cast<double *>(base + ((rb + 255) & ~size_t(255)));
    GQ_HIP(hipMemcpyAsync(base, rounds.data(), rb, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(hist_evolve_kernel, dim3(1), dim3(64), 0, st,
                       reinterpret_cast<const unsigned long long *>(hist), m, n, p,
                       reinterpret_cast<const HistRound *>(base), target, d_out);
    GQ_LAUNCH_CHECK();
    std::vector<double> o((size_t)3 * (p + 1));
    GQ_HIP(hipMemcpyAsync(o.data(), d_out, ob, hipMemcpyDeviceToHost, st));
    GQ_HIP(hipStreamSynchronize(st));
    for (int j = 0; j <= p; ++j) {
        if (psol) psol[j] = o[3 * j];
        if (energy) energy[j] = o[3 * j + 1];
        if (norm) norm[j] = o[3 * j + 2];
    }
    return GQAOA_OK;
}

// ---- batched single-angle-pair scan, float32 -------------------------------------------
constexpr int kScanMaxWaves = 4;
// Tables up to kScanHoist4 levels stay in registers whole (cos, -sin, sin, w:
// every instruction of a level-round has two VGPR operands); up to
// kScanHoist3 levels as (cos, sin, w), with the one negated product of a
// level-round as a three-operand fma, which gives the same value; larger
// tables are re-read from LDS every round.
constexpr int kScanHoist4 = 24;
constexpr int kScanHoist3 = 36;

// Per item, each wave's table in LDS: tab[k] = {cos(gamma l_k), -sin(gamma l_k),
// sin(gamma l_k), w_k}; the energy weights l_k w_k (read only at readouts) go
// from the lanes that compute them to scalar registers. The target level,
// when occupied, is level 0 of the instance's compacted order, so the
// crossing readout reads one amplitude.
//
// A level-round is eight two-operand VALU instructions on VGPR operands (the
// form gfx950 issues at twice the rate of instructions with an SGPR or a third
// source): the phase multiply as two products and two fused accumulates, the
// weighted sum for <s|phi> as two fused accumulates, the mixer as two adds.
// Dual issue needs two waves with VALU work on a SIMD, so an item's loads
// (its descriptor, levels and weights) are issued one item ahead, while the
// previous item's rounds run, instead of stalling the wave between items.

// The work item's coordinates: beta tile, gamma index and slot.
struct ScanItem {
    int tile, g;
    unsigned slot;
};
__device__ __forceinline__ ScanItem scan_decode(const ScanArgs &a, unsigned item) {
    const unsigned rest = item / (unsigned)a.ntiles;
    return ScanItem{(int)(item % (unsigned)a.ntiles), (int)(rest % (unsigned)a.ng), rest / (unsigned)a.ng};
}

// The lane's share of an instance's levels: level k = lane + 64 i.
template <int NL>
__device__ __forceinline__ void scan_load_levels(const ScanArgs &a, const ScanSlot &sl, int lane, int (&lv)[NL],
                                                 float (&wk)[NL]) {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int k = lane + 64 * i;
        lv[i] = k < sl.K ? a.lev[sl.lev_off + k] : 0;
        wk[i] = k < sl.K ? a.w[sl.lev_off + k] : 0.f;
    }
}

// Writes the item's table (phases in float64, rounded once) to LDS.
template <int KMAX, int NL>
__device__ __forceinline__ void scan_table(const ScanArgs &a, const ScanSlot &sl, int g, int lane, const int (&lv)[NL],
                                           const float (&wk)[NL], float4 *tab, float (&kwl)[NL]) {
    const double gam = a.gammas[(a.per_inst ? (size_t)sl.inst * a.ng : 0) + g];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        const int k = lane + 64 * i;
        if (k < KMAX) {
            float4 e = {1.f, 0.f, 0.f, 0.f};
            float ew = 0.f;
            if (k < sl.K) {
                double sn, cs;
                sincos(gam * (double)lv[i], &sn, &cs);
                e = {(float)cs, (float)-sn, (float)sn, wk[i]};
                ew = wk[i] * (float)lv[i];
            }
            tab[k] = e;
            kwl[i] = ew;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The rounds of one item for this lane's beta (mixer e^{-i beta} - 1 = mr + i mi).
template <int KMAX, bool CROSS>
__device__ __forceinline__ void scan_rounds(const ScanArgs &a, const ScanSlot &sl, const ScanItem &it, int lane,
                                            float mr, float mi, const float4 *tab,
                                            const float (&kwl)[(KMAX + 63) / 64]) {
    // l_k w_k of every level, for the energy readout: the same in every lane,
    // so held in scalar registers (read out of the lane that computed it)
    float kw[CROSS ? 1 : KMAX];
    if constexpr (!CROSS) {
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
            kw[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(kwl[k / 64]), k % 64));
    }
    const int b = it.tile * 64 + lane;
    const bool active = b < a.nb;
    const float w0 = sl.t_idx == 0 ? tab[0].w : 0.f;   // weight of the target level (index 0)
    // The lane keeps the phased amplitudes phi_k of the current round and the
    // mixer's correction c of the round before, and forms b_k = phi_k + c at
    // the start of the next round: the same adds on the same operands as
    // applying the mixer at the end of each round, with one level's
    // temporaries live at a time instead of all of them.
    float pr[KMAX], pi[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        pr[k] = 1.f;
        pi[k] = 0.f;
    }
    float cr = 0.f, ci = 0.f;
    int q = 0;
    int found = 0;
    const int pmax = sl.pmax;
    int next_p = CROSS ? 0 : a.p_list[0];   // next readout round, kept in a register
    for (int j = 1; j <= pmax; ++j) {
        // Small tables stay in registers across rounds; larger ones are
        // re-read from LDS (broadcast) each round to bound register use.
        if constexpr (KMAX > kScanHoist3) asm volatile("" ::: "memory");
        float sr = 0.f, si = 0.f;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const float4 e = tab[k];
            const float xr = pr[k] + cr, xi = pi[k] + ci;               // b_k after the last mixer
            const float nr = __builtin_fmaf(e.x, xr, e.z * xi);         // cos br + sin bi
            float ni;                                                    // cos bi - sin br
            if constexpr (KMAX <= kScanHoist4)
                ni = __builtin_fmaf(e.x, xi, e.y * xr);
            else
                ni = __builtin_fmaf(e.x, xi, -(e.z * xr));
            pr[k] = nr;
            pi[k] = ni;
            sr = __builtin_fmaf(e.w, nr, sr);
            si = __builtin_fmaf(e.w, ni, si);
        }
        cr = mr * sr - mi * si;
        ci = mr * si + mi * sr;
        if constexpr (CROSS) {
            const float b0r = pr[0] + cr, b0i = pi[0] + ci;
            const float P = w0 * (b0r * b0r + b0i * b0i);
            if (found == 0 && P >= a.threshold) found = j;
            if (__ballot(active && found == 0) == 0) break;  // wave-uniform
        } else if (j == next_p) {
            float E = 0.f;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const float br = pr[k] + cr, bi = pi[k] + ci;
                E = __builtin_fmaf(kw[k], br * br + bi * bi, E);
            }
            const float b0r = pr[0] + cr, b0i = pi[0] + ci;
            const float P = w0 * (b0r * b0r + b0i * b0i);
            if (active) {
                const size_t o = (((size_t)sl.inst * a.num_p + q) * a.ng + it.g) * a.nb + b;
                a.psol[o] = P;
                if (a.energy) a.energy[o] = E;
            }
            ++q;
            next_p = q < a.num_p ? a.p_list[q] : 0;
        }
    }
    if constexpr (CROSS)
        if (active) a.first_p[((size_t)sl.inst * a.ng + it.g) * a.nb + b] = found;
}

// Mixer factor of this lane's beta, recomputed only when the beta row changes
// (the grid is shared, or the instance's own).
__device__ __forceinline__ void scan_mixer(const ScanArgs &a, const ScanSlot &sl, int tile, int lane, long long &key,
                                           float &mr, float &mi) {
    const long long k = (long long)(a.per_inst ? sl.inst : 0) * a.ntiles + tile;
    if (k == key) return;
    key = k;
    const int b = tile * 64 + lane;
    double sb, cb;
    sincos(a.betas[(a.per_inst ? (size_t)sl.inst * a.nb : 0) + (b < a.nb ? b : 0)], &sb, &cb);
    mr = (float)(cb - 1.0);
    mi = (float)(-sb);
}

// CROSS = false: P_sol (and E) after each p in p_list. Every item of a bucket
// costs the same (same padded level count, same rounds), so wave w of the
// grid takes items w, w + W, w + 2W, ... (W waves), and the next item's
// descriptor and levels are loaded while the current one runs.
// CROSS = true: the first round j <= p_i with P >= threshold; a wave stops
// once every lane has crossed, so items differ in length and come from a
// global queue (the next index is fetched while the current item runs).
template <int KMAX, bool CROSS>
__global__ void __launch_bounds__(kScanMaxWaves * 64) scan_kernel(ScanArgs a) {
    constexpr int NL = (KMAX + 63) / 64;
    __shared__ float4 tab_s[kScanMaxWaves][KMAX];
    const int lane = threadIdx.x & 63;
    float4 *tab = tab_s[threadIdx.x >> 6];
    float kwl[NL];
    long long mix_key = -1;
    float mr = 0.f, mi = 0.f;
    unsigned item;
    if constexpr (CROSS) {
        unsigned v = 0;
        if (lane == 0) v = atomicAdd(a.counter, 1u);
        item = __builtin_amdgcn_readfirstlane(__shfl(v, 0, 64));
    } else {
        item = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    }
    if (item >= a.total_items) return;  // whole waves
    const unsigned W = gridDim.x * (blockDim.x >> 6);
    ScanItem it = scan_decode(a, item);
    ScanSlot sl = a.slots[it.slot];
    int lv[NL];
    float wk[NL];
    scan_load_levels<NL>(a, sl, lane, lv, wk);
    unsigned nxt = CROSS ? 0u : item + W;
    ScanSlot sl_n = sl;
    if constexpr (!CROSS)
        if (nxt < a.total_items) sl_n = a.slots[scan_decode(a, nxt).slot];
    for (;;) {
        scan_table<KMAX, NL>(a, sl, it.g, lane, lv, wk, tab, kwl);
        // loads for the next item, consumed after this item's rounds
        int lv_n[NL];
        float wk_n[NL];
        unsigned nn = 0;
        ScanSlot sl_nn = sl_n;
        if constexpr (CROSS) {
            unsigned v = 0;
            if (lane == 0) v = atomicAdd(a.counter, 1u);
            nxt = __builtin_amdgcn_readfirstlane(__shfl(v, 0, 64));
        } else {
            if (nxt < a.total_items) scan_load_levels<NL>(a, sl_n, lane, lv_n, wk_n);
            nn = nxt + W;
            if (nn < a.total_items) sl_nn = a.slots[scan_decode(a, nn).slot];
        }
        scan_mixer(a, sl, it.tile, lane, mix_key, mr, mi);
        scan_rounds<KMAX, CROSS>(a, sl, it, lane, mr, mi, tab, kwl);
        // the next item rewrites tab: keep every lane's reads of this one first
        __builtin_amdgcn_wave_barrier();
        if (nxt >= a.total_items) break;
        it = scan_decode(a, nxt);
        if constexpr (CROSS) {
            sl = a.slots[it.slot];
            scan_load_levels<NL>(a, sl, lane, lv, wk);
        } else {
            sl = sl_n;
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                lv[i] = lv_n[i];
                wk[i] = wk_n[i];
            }
            sl_n = sl_nn;
            nxt = nn;
        }
    }
}

__global__ void zero_counters_kernel(unsigned int *c, int n) {
    const int i = threadIdx.x;
    if (i < n) c[i] = 0u;
}

// Register-array sizes of the scan kernel instantiations: every multiple of
// 4 up to 64 (an instance pays for at most 3 padding levels, which carry
// weight 0), then steps of 16.
static const int kBuckets[] = {4, 8, 12, 16, 20, 24, 28, 32, 36, 40, 44, 48, 52, 56, 60, 64, 80, 96, 112, 128};
constexpr int kNumBuckets = sizeof(kBuckets) / sizeof(kBuckets[0]);
constexpr int kScanMaxK = 128;

typedef void (*ScanFn)(ScanArgs);
template <bool CROSS, int... KS>
static ScanFn scan_fn_pick(int kmax, std::integer_sequence<int, KS...>) {
    ScanFn f = nullptr;
    ((f = (KS == kmax ? scan_kernel<KS, CROSS> : f)), ...);
    return f;
}
template <bool CROSS>
static ScanFn scan_fn_t(int bucket) {
    return scan_fn_pick<CROSS>(kBuckets[bucket], std::integer_sequence<int, 4, 8, 12, 16, 20, 24, 28, 32, 36, 40, 44, 48,
                                                                       52, 56, 60, 64, 80, 96, 112, 128>{});
}
static ScanFn scan_fn(int bucket, bool cross) { return cross ? scan_fn_t<true>(bucket) : scan_fn_t<false>(bucket); }

int scan_max_levels() { return kScanMaxK; }

// ---- autotuned launch shape -----------------------------------------------------------
// Candidates: waves per block in {1, 2, 4} x blocks per CU in {2, 4, 8, 16}. A
// candidate is timed on the bucket's real work (a prefix of the queue) and
// the best is cached per (device arch, bucket, beta tiles) for the process;
// GQAOA_TUNE_CACHE names an optional text file that persists the choices.
static std::mutex g_tune_mu;
static std::map<std::string, TileChoice> g_tune;
static bool g_tune_loaded = false;

static void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = getenv("GQAOA_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    tune_cache_read(f, g_tune);  // shapes outside the accepted range are dropped and retuned
    fclose(f);
}

static void tune_store_locked() {
    const char *path = getenv("GQAOA_TUNE_CACHE");
    if (!path) return;
    FILE *f = fopen(path, "w");
    if (!f) return;
    tune_cache_write(f, g_tune);
    fclose(f);
}

int scan_launch_bucket(int bucket, const TileChoice &tc, const DeviceInfo &dev, ScanArgs a, unsigned int *counter,
                       hipStream_t st) {
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, st, counter, 1);
    GQ_LAUNCH_CHECK();
    a.counter = counter;
    const unsigned want = (a.total_items + tc.waves - 1) / tc.waves;
    const unsigned blocks = std::max(1u, std::min<unsigned>(want, (unsigned)(dev.num_cus * tc.blocks_per_cu)));
    hipLaunchKernelGGL(scan_fn(bucket, a.first_p != nullptr), dim3(blocks), dim3(64 * tc.waves), 0, st, a);
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

static int tune_bucket(int bucket, const DeviceInfo &dev, const ScanArgs &a, unsigned int *counter,
                       hipStream_t st, TileChoice *out) {
    const std::string plain_key = std::string(dev.arch) + ":k" + std::to_string(kBuckets[bucket]) + ":t" +
                                  std::to_string(a.ntiles) + ":p" +
                                  std::to_string(a.p_list[a.num_p - 1] > 16 ? 64 : 16);
    const std::string key = plain_key + (a.first_p ? ":x" : "");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tune.find(key);
        if (it == g_tune.end() && a.first_p) it = g_tune.find(plain_key);  // same loop, plus a readout
        if (it != g_tune.end()) {
            *out = it->second;
            return GQAOA_OK;
        }
    }
    // time a prefix of the queue that fills the device a few times over; the
    // crossing form's items can run thousands of rounds, so its prefix is a
    // single fill of the device
    ScanArgs t = a;
    t.total_items = std::min<unsigned>(a.total_items, (unsigned)dev.num_cus * (a.first_p ? 8 : 64));
    const int waves_c[] = {1, 2, 4};
    const int bpc_c[] = {2, 4, 8, 16};
    hipEvent_t e0, e1;
    GQ_HIP(hipEventCreate(&e0));
    GQ_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    TileChoice bestc{4, 4};
    for (int wv : waves_c)
        for (int bpc : bpc_c) {
            TileChoice tc{wv, bpc};
            int s = scan_launch_bucket(bucket, tc, dev, t, counter, st);  // warm-up
            if (s) return s;
            GQ_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < 3; ++r)
                if ((s = scan_launch_bucket(bucket, tc, dev, t, counter, st))) return s;
            GQ_HIP(hipEventRecord(e1, st));
            GQ_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            GQ_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                bestc = tc;
            }
        }
    GQ_HIP(hipEventDestroy(e0));
    GQ_HIP(hipEventDestroy(e1));
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = bestc;
    tune_store_locked();
    *out = bestc;
    return GQAOA_OK;
}

size_t scan_workspace_bytes(int num_inst, int hist_stride, int nb, int ng, int num_p, int per_inst) {
    (void)num_p;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t lv = (size_t)num_inst * std::min(hist_stride, kScanMaxK);
    const size_t ga = per_inst ? (size_t)num_inst : 1;
    return al(sizeof(ScanSlot) * (size_t)num_inst) + al(4 * lv) + al(4 * lv) + al(8 * (size_t)nb * ga) +
           al(8 * (size_t)ng * ga) + al(4 * kNumBuckets) + 256;
}

int scan_num_buckets() { return kNumBuckets; }

ScanDev scan_dev_tables(void *ws, int num_inst, int hist_stride, int nb, int ng, int per_inst) {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t lv = (size_t)num_inst * std::min(hist_stride, kScanMaxK);
    const size_t ga = per_inst ? (size_t)num_inst : 1;
    char *p = reinterpret_cast<char *>(ws);
    ScanDev d;
    d.slots = reinterpret_cast<ScanSlot *>(p);
    p += al(sizeof(ScanSlot) * (size_t)num_inst);
    d.lev = reinterpret_cast<int32_t *>(p);
    p += al(4 * lv);
    d.w = reinterpret_cast<float *>(p);
    p += al(4 * lv);
    d.betas = reinterpret_cast<double *>(p);
    p += al(8 * (size_t)nb * ga);
    d.gammas = reinterpret_cast<double *>(p);
    p += al(8 * (size_t)ng * ga);
    d.counters = reinterpret_cast<unsigned int *>(p);
    return d;
}

int scan_host_tables(int num_inst, const int32_t *n_host, const int32_t *m_host, const uint64_t *hists,
                     int hist_stride, const int32_t *target_host, const int32_t *pmax_host, int pmax_all,
                     ScanHost *out) {
    // compact the occupied levels of every instance
    std::vector<int32_t> K(num_inst), tidx(num_inst), off(num_inst);
    out->lev.clear();
    out->w.clear();
    for (int i = 0; i < num_inst; ++i) {
        const uint64_t *h = hists + (size_t)i * hist_stride;
        const int t = target_host ? target_host[i] : 0;
        off[i] = (int32_t)out->lev.size();
        tidx[i] = -1;
        const double invN = std::ldexp(1.0, -n_host[i]);
        // the target level (when occupied) first, then the others in level order
        if (t <= m_host[i] && h[t]) {
            tidx[i] = 0;
            out->lev.push_back(t);
            out->w.push_back((float)((double)h[t] * invN));
        }
        for (int k = 0; k <= m_host[i]; ++k)
            if (h[k] && k != t) {
                out->lev.push_back(k);
                out->w.push_back((float)((double)h[k] * invN));
            }
        K[i] = (int32_t)out->lev.size() - off[i];
        if (K[i] > kScanMaxK) return fail(GQAOA_ERANGE, "instance %d has %d occupied levels (max %d)", i, K[i], kScanMaxK);
    }
    // buckets, each ordered by K descending
    std::vector<std::vector<int>> members(kNumBuckets);
    for (int i = 0; i < num_inst; ++i) {
        int bk = 0;
        while (kBuckets[bk] < std::max(1, K[i])) ++bk;
        members[bk].push_back(i);
    }
    out->slots.clear();
    out->bucket_first.assign(kNumBuckets + 1, 0);
    for (int bk = 0; bk < kNumBuckets; ++bk) {
        auto &mb = members[bk];
        std::stable_sort(mb.begin(), mb.end(), [&](int x, int y) { return K[x] > K[y]; });
        out->bucket_first[bk] = (int)out->slots.size();
        for (int i : mb)
            out->slots.push_back(ScanSlot{i, off[i], K[i], tidx[i], pmax_host ? pmax_host[i] : pmax_all, {0, 0, 0}});
    }
    out->bucket_first[kNumBuckets] = (int)out->slots.size();
    return GQAOA_OK;
}

int scan_choose_tile(int bucket, const DeviceInfo &dev, const ScanArgs &a, unsigned int *counter,
                     const int32_t *tile, hipStream_t st, TileChoice *out) {
    if (tile) {
        *out = TileChoice{tile[0], tile[1]};
        return GQAOA_OK;
    }
    return tune_bucket(bucket, dev, a, counter, st, out);
}

int run_scan(int num_inst, const int32_t *n_host, const int32_t *m_host, const uint64_t *hists,
             int hist_stride, const int32_t *target_host, int nb, const double *betas, int ng,
             const double *gammas, int per_inst, int num_p, const int32_t *p_list, float *psol, float *energy,
             float threshold, int32_t *first_p, const int32_t *pmax_host, const int32_t *tile, void *ws,
             hipStream_t st) {
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    ScanHost H;
    if ((s = scan_host_tables(num_inst, n_host, m_host, hists, hist_stride, target_host, pmax_host,
                              p_list[num_p - 1], &H)))
        return s;
    const ScanDev D = scan_dev_tables(ws, num_inst, hist_stride, nb, ng, per_inst);
    const size_t ga = per_inst ? (size_t)num_inst : 1;
    GQ_HIP(hipMemcpyAsync(D.slots, H.slots.data(), sizeof(ScanSlot) * H.slots.size(), hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(D.lev, H.lev.data(), 4 * H.lev.size(), hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(D.w, H.w.data(), 4 * H.w.size(), hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(D.betas, betas, 8 * (size_t)nb * ga, hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(D.gammas, gammas, 8 * (size_t)ng * ga, hipMemcpyHostToDevice, st));

    ScanArgs a{};
    a.lev = D.lev;
    a.w = D.w;
    a.betas = D.betas;
    a.gammas = D.gammas;
    a.psol = psol;
    a.energy = energy;
    a.first_p = first_p;
    a.threshold = threshold;
    a.nb = nb;
    a.ng = ng;
    a.ntiles = (nb + 63) / 64;
    a.num_p = num_p;
    a.per_inst = per_inst;
    for (int q = 0; q < num_p; ++q) a.p_list[q] = p_list[q];
    for (int bk = 0; bk < kNumBuckets; ++bk) {
        const int nslots = H.bucket_first[bk + 1] - H.bucket_first[bk];
        if (!nslots) continue;
        ScanArgs ab = a;
        ab.slots = D.slots + H.bucket_first[bk];
        ab.total_items = (unsigned)nslots * (unsigned)ng * (unsigned)ab.ntiles;
        TileChoice tc;
        if ((s = scan_choose_tile(bk, dev, ab, D.counters + bk, tile, st, &tc))) return s;
        ProfScope ps("scan", st);
        if ((s = scan_launch_bucket(bk, tc, dev, ab, D.counters + bk, st))) return s;
        ps.end();
    }
    GQ_HIP(hipStreamSynchronize(st));  // host staging vectors end here
    if (prof_on()) prof_collect();
    return GQAOA_OK;
}

}  // namespace gqaoa
