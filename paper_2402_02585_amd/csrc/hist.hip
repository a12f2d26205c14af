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
constexpr int kScanHoistMax = 24;  // largest bucket whose phase table is kept in registers

// CROSS = false: P_sol (and E) after each p in p_list. CROSS = true: the
// first round j <= p_list[0] with P >= threshold; a wave stops once every
// lane has crossed.
template <int KMAX, bool CROSS>
__global__ void __launch_bounds__(kScanMaxWaves * 64) scan_kernel(ScanArgs a) {
    __shared__ float4 tab_s[kScanMaxWaves][KMAX];   // e^{-i gamma k}.re/.im, w_k, k w_k
    const int lane = threadIdx.x & 63;
    float4 *tab = tab_s[threadIdx.x >> 6];
    for (;;) {
        unsigned int item = 0;
        if (lane == 0) item = atomicAdd(a.counter, 1u);
        item = __builtin_amdgcn_readfirstlane(__shfl(item, 0, 64));
        if (item >= a.total_items) break;
        const int tile = (int)(item % (unsigned)a.ntiles);
        const unsigned rest = item / (unsigned)a.ntiles;
        const int g = (int)(rest % (unsigned)a.ng);
        const ScanSlot sl = a.slots[rest / (unsigned)a.ng];
        const int pmax = sl.pmax;
        const double gam = a.gammas[(a.per_inst ? (size_t)sl.inst * a.ng : 0) + g];
        for (int k = lane; k < KMAX; k += 64) {
            float4 e = {1.f, 0.f, 0.f, 0.f};
            if (k < sl.K) {
                const int lv = a.lev[sl.lev_off + k];
                const float wk = a.w[sl.lev_off + k];
                double s, c;
                sincos(fmod(gam * (double)lv, 2.0 * M_PI), &s, &c);
                e = {(float)c, (float)-s, wk, wk * (float)lv};
            }
            tab[k] = e;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        const int b = tile * 64 + lane;
        const bool active = b < a.nb;
        double sb, cb;
        sincos(a.betas[(a.per_inst ? (size_t)sl.inst * a.nb : 0) + (active ? b : 0)], &sb, &cb);
        const float mr = (float)(cb - 1.0), mi = (float)(-sb);
        float br[KMAX], bi[KMAX];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            br[k] = 1.f;
            bi[k] = 0.f;
        }
        int q = 0;
        int found = 0;
        for (int j = 1; j <= pmax; ++j) {
            // Small tables stay in registers across rounds; larger ones are
            // re-read from LDS (broadcast) each round to bound register use.
            if constexpr (KMAX > kScanHoistMax) asm volatile("" ::: "memory");
            float sr = 0.f, si = 0.f;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const float4 e = tab[k];
                const float nr = e.x * br[k] - e.y * bi[k];
                const float ni = e.x * bi[k] + e.y * br[k];
                br[k] = nr;
                bi[k] = ni;
                sr += e.z * nr;
                si += e.z * ni;
            }
            const float cr = mr * sr - mi * si, ci = mr * si + mi * sr;
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                br[k] += cr;
                bi[k] += ci;
            }
            if constexpr (CROSS) {
                float P = 0.f;
#pragma unroll
                for (int k = 0; k < KMAX; ++k)
                    P += k == sl.t_idx ? tab[k].z * (br[k] * br[k] + bi[k] * bi[k]) : 0.f;
                if (found == 0 && P >= a.threshold) found = j;
                if (__ballot(active && found == 0) == 0) break;  // wave-uniform
            } else if (j == a.p_list[q]) {
                float P = 0.f, E = 0.f;
#pragma unroll
                for (int k = 0; k < KMAX; ++k) {
                    const float4 e = tab[k];
                    const float pb = br[k] * br[k] + bi[k] * bi[k];
                    E += e.w * pb;
                    P += k == sl.t_idx ? e.z * pb : 0.f;
                }
                if (active) {
                    const size_t o = (((size_t)sl.inst * a.num_p + q) * a.ng + g) * a.nb + b;
                    a.psol[o] = P;
                    if (a.energy) a.energy[o] = E;
                }
                ++q;
            }
        }
        if constexpr (CROSS)
            if (active) a.first_p[((size_t)sl.inst * a.ng + g) * a.nb + b] = found;
        // the next item rewrites tab: keep every lane's reads of this one first
        __builtin_amdgcn_wave_barrier();
    }
}

__global__ void zero_counters_kernel(unsigned int *c, int n) {
    const int i = threadIdx.x;
    if (i < n) c[i] = 0u;
}

// Register-array sizes of the scan kernel instantiations.
static const int kBuckets[] = {8, 16, 24, 32, 40, 48, 56, 64, 80, 96, 112, 128};
constexpr int kNumBuckets = sizeof(kBuckets) / sizeof(kBuckets[0]);
constexpr int kScanMaxK = 128;

typedef void (*ScanFn)(ScanArgs);
template <bool CROSS>
static ScanFn scan_fn_t(int bucket) {
    switch (kBuckets[bucket]) {
        case 8: return scan_kernel<8, CROSS>;
        case 16: return scan_kernel<16, CROSS>;
        case 24: return scan_kernel<24, CROSS>;
        case 32: return scan_kernel<32, CROSS>;
        case 40: return scan_kernel<40, CROSS>;
        case 48: return scan_kernel<48, CROSS>;
        case 56: return scan_kernel<56, CROSS>;
        case 64: return scan_kernel<64, CROSS>;
        case 80: return scan_kernel<80, CROSS>;
        case 96: return scan_kernel<96, CROSS>;
        case 112: return scan_kernel<112, CROSS>;
        default: return scan_kernel<128, CROSS>;
    }
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
        for (int k = 0; k <= m_host[i]; ++k)
            if (h[k]) {
                if (k == t) tidx[i] = (int32_t)(out->lev.size() - off[i]);
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
