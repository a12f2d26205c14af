// Statevector evaluation of single-angle-pair work items of small instances:
// the independent statevector check of the batched level-space scan (Eq. (5)
// evolved amplitude by amplitude instead of level by level).
//
// One block per item (instance, beta, gamma), sized to the state, each
// thread owning the same PER consecutive amplitudes in every round. Under the
// single-angle-pair protocol the phase table e^{-i gamma k} is the same in
// every round: it sits in LDS, the thread's amplitudes and their costs (four
// to a register) stay in registers. Round j is one sweep over the thread's
// amplitudes: it forms
// psi_{j-1} = phi_{j-1} + delta_{j-1} (the Grover mixer of the previous round
// applied lazily, as in the streaming round pass), reads out P_sol and E
// when j-1 is a requested round, applies the phase and sums phi_j; one
// reduction (float64) gives delta_j = (e^{-i beta} - 1) S_j / 2^n. The
// reduction is the only exchange between threads (wave shuffles alone for a
// one-wave block). Items of larger instances (n > GQAOA_SV_ITEMS_MAX_N) are
// evolved by the streaming round passes, all items of one n in one batch.
#include "batch.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace gqaoa {

// Shape of a block for items of size n: one wave of PER = max(1, 2^n / 64)
// amplitudes per lane up to n = 11 (its sums are pure wave reductions), then
// 2^n / 32 threads of 32 amplitudes (fewer waves per item, so less
// reduction work per amplitude).
static int item_threads(int n) { return n <= 11 ? 64 : (1 << (n - 5)); }

template <int THREADS, int PER>
__global__ void __launch_bounds__(THREADS) sv_items_kernel(SvItemsArgs a) {
    __shared__ float2 lut[256];
    __shared__ double red_s[2][THREADS / kWave][4];  // per-wave sums, double-buffered by round parity
    const uint32_t N = 1u << a.n;
    const int tid = threadIdx.x;
    const double invN = ldexp(1.0, -a.n);
    const float amp0 = (float)sqrt(invN);  // |s> = 2^(-n/2) on every z
    const int pmax = a.p_list[a.num_p - 1];
    for (int item = blockIdx.x; item < a.num_items; item += gridDim.x) {
        const SvItem it = a.items[item];
        const uint8_t *src = a.costs + a.cost_off[it.inst];
        const int m = a.m[it.inst];
        const uint32_t target = (uint32_t)a.target[it.inst];
        for (int k = tid; k <= m; k += THREADS) {
            double s, co;
            sincos(fmod(it.gamma * (double)k, 2.0 * M_PI), &s, &co);
            lut[k] = float2{(float)co, (float)-s};
        }
        double sb, cb;
        sincos(it.beta, &sb, &cb);
        const double mr = cb - 1.0, mi = -sb;
        __syncthreads();
        // this thread's amplitudes z = tid PER + i (a contiguous run): the
        // state in registers, the costs packed four to a register (one
        // vector load when aligned); the phase factor e^{-i gamma C(z)} is
        // read from the LDS table each round. Only the one-amplitude shape
        // (n <= 6) has lanes without amplitudes.
        const bool owns = (uint32_t)tid * PER < N;
        float2 xv[PER];
        uint32_t cpk[(PER + 3) / 4];
#pragma unroll
        for (int w = 0; w < (PER + 3) / 4; ++w) cpk[w] = 0u;
        if (owns) load_packed_costs<PER>(src + (size_t)tid * PER, cpk);
#pragma unroll
        for (int i = 0; i < PER; ++i) xv[i] = float2{amp0, 0.f};
        float dr = 0.f, di = 0.f;
        int q = 0;
        for (int j = 1; j <= pmax + 1; ++j) {
            const bool rd = q < a.num_p && a.p_list[q] == j - 1;
            const bool ph = j <= pmax;
            float sr = 0.f, si = 0.f, sp = 0.f, se = 0.f;
            if (owns) {
                if (j > 1)  // psi_{j-1} = phi_{j-1} + delta_{j-1}: the previous mixer, applied lazily
#pragma unroll
                    for (int i = 0; i < PER; ++i) {
                        xv[i].x += dr;
                        xv[i].y += di;
                    }
                if (rd)
#pragma unroll
                    for (int i = 0; i < PER; ++i) {
                        const uint32_t cz = (cpk[i >> 2] >> (8 * (i & 3))) & 0xFFu;
                        const float pr = xv[i].x * xv[i].x + xv[i].y * xv[i].y;
                        sp += cz == target ? pr : 0.f;
                        se += (float)cz * pr;
                    }
                if (ph)
#pragma unroll
                    for (int i = 0; i < PER; ++i) {
                        const uint32_t cz = (cpk[i >> 2] >> (8 * (i & 3))) & 0xFFu;
                        const float2 e = lut[cz], x = xv[i];
                        const float2 f{e.x * x.x - e.y * x.y, e.x * x.y + e.y * x.x};
                        xv[i] = f;
                        sr += f.x;
                        si += f.y;
                    }
            }
            // S every round; P_sol and E only in the readout rounds
            double r[4] = {sr, si, sp, se};
            const int nq = rd ? 4 : 2;
            // DPP wave sums (nq is uniform, so the whole block is converged)
            if constexpr (THREADS == kWave) {
                // every lane ends with the same totals
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < nq) r[k] = wave_sum_dpp(r[k]);
            } else {
                // wave sums, then a wave sum of the per-wave sums (the same
                // fixed order in every wave, so identical totals in every
                // thread). A buffer is rewritten two rounds later, after the
                // next round's barrier, which every thread passes only once
                // it has read this round's sums.
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < nq) r[k] = wave_sum_dpp(r[k]);
                double(*buf)[4] = red_s[j & 1];
                const int lane = tid & (kWave - 1);
                if (lane == 0)
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (k < nq) buf[tid / kWave][k] = r[k];
                __syncthreads();
                // lane w < waves takes wave w's sums, then one sum over those lanes
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (k < nq) r[k] = lanes_sum_dpp<THREADS / kWave>(lane < THREADS / kWave ? buf[lane][k] : 0.0);
            }
            if (rd) {
                if (tid == 0) {
                    a.psol[(size_t)it.out * a.num_p + q] = (float)r[2];
                    if (a.energy) a.energy[(size_t)it.out * a.num_p + q] = (float)r[3];
                }
                ++q;
            }
            if (ph) {
                const double Sr = r[0] * invN, Si = r[1] * invN;
                dr = (float)(mr * Sr - mi * Si);
                di = (float)(mr * Si + mi * Sr);
            }
        }
        __syncthreads();  // every thread has read lut before the next item rewrites it
    }
}

typedef void (*ItemsFn)(SvItemsArgs);
static ItemsFn items_fn(int n) {
    switch (n <= 6 ? 6 : n) {
        case 6: return sv_items_kernel<64, 1>;
        case 7: return sv_items_kernel<64, 2>;
        case 8: return sv_items_kernel<64, 4>;
        case 9: return sv_items_kernel<64, 8>;
        case 10: return sv_items_kernel<64, 16>;
        case 11: return sv_items_kernel<64, 32>;
        case 12: return sv_items_kernel<128, 32>;
        case 13: return sv_items_kernel<256, 32>;
        default: return sv_items_kernel<512, 32>;
    }
}

uint64_t batched_cost_offset(int i, const int32_t *n_host);

int sv_items_order(const int32_t *n_host, int num_items, const int32_t *item_inst, const DeviceInfo &dev,
                   ItemOrder *out) {
    (void)dev;
    out->order.resize(num_items);
    for (int k = 0; k < num_items; ++k) out->order[k] = k;
    std::stable_sort(out->order.begin(), out->order.end(),
                     [&](int x, int y) { return n_host[item_inst[x]] < n_host[item_inst[y]]; });
    out->first.clear();
    for (int k = 0; k < num_items; ++k)
        if (k == 0 || n_host[item_inst[out->order[k]]] != n_host[item_inst[out->order[k - 1]]]) out->first.push_back(k);
    out->first.push_back(num_items);
    return GQAOA_OK;
}

int sv_items_launch(const SvItemsArgs &a, const DeviceInfo &dev, hipStream_t st) {
    const int threads = item_threads(a.n);
    const ItemsFn fn = items_fn(a.n);
    // exactly the blocks that are resident at once (each takes items in a
    // grid-stride loop, so a second wave of blocks would only wait)
    int per_cu = 0;
    GQ_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(fn), threads, 0));
    const int blocks = std::min(a.num_items, dev.num_cus * std::max(1, per_cu));
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(threads), 0, st, a);
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

int sv_items_stream(int n, int count, const int32_t *item_inst, const int32_t *item_out, const double *beta,
                    const double *gamma, const uint8_t *costs, const uint64_t *cost_off, const int32_t *m_host,
                    const int32_t *target_host, int num_p, const int32_t *p_list, float *psol, float *energy,
                    hipStream_t st);

int run_sv_items(int num_inst, const int32_t *n_host, const int32_t *m_host, const int32_t *target_host,
                 const uint8_t *costs, int num_items, const int32_t *item_inst, const double *beta,
                 const double *gamma, int num_p, const int32_t *p_list, float *psol, float *energy, hipStream_t st) {
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    ItemOrder ord;
    if ((s = sv_items_order(n_host, num_items, item_inst, dev, &ord))) return s;
    std::vector<uint64_t> off(num_inst);
    for (int i = 0; i < num_inst; ++i) off[i] = batched_cost_offset(i, n_host);
    std::vector<int32_t> tg(num_inst, 0);
    if (target_host) tg.assign(target_host, target_host + num_inst);
    std::vector<SvItem> items(num_items);
    for (int k = 0; k < num_items; ++k) {
        const int o = ord.order[k];
        items[k] = SvItem{item_inst[o], o, beta[o], gamma[o]};
    }
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t b_items = sizeof(SvItem) * items.size(), b_off = 8 * (size_t)num_inst, b_i = 4 * (size_t)num_inst;
    AsyncScratch guard(st);
    GQ_HIP(guard.alloc(al(b_items) + al(b_off) + 2 * al(b_i)));
    char *base = reinterpret_cast<char *>(guard.ptr);
    SvItem *d_items = reinterpret_cast<SvItem *>(base);
    uint64_t *d_off = reinterpret_cast<uint64_t *>(base + al(b_items));
    int32_t *d_m = reinterpret_cast<int32_t *>(base + al(b_items) + al(b_off));
    int32_t *d_t = reinterpret_cast<int32_t *>(base + al(b_items) + al(b_off) + al(b_i));
    GQ_HIP(hipMemcpyAsync(d_items, items.data(), b_items, hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(d_off, off.data(), b_off, hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(d_m, m_host, b_i, hipMemcpyHostToDevice, st));
    GQ_HIP(hipMemcpyAsync(d_t, tg.data(), b_i, hipMemcpyHostToDevice, st));
    for (size_t g = 0; g + 1 < ord.first.size(); ++g) {
        const int k0 = ord.first[g], k1 = ord.first[g + 1];
        const int n = n_host[items[k0].inst];
        if (n > GQAOA_SV_ITEMS_MAX_N) {  // too large for registers: streamed, batched per n
            std::vector<int32_t> ii(k1 - k0), io(k1 - k0);
            std::vector<double> bb(k1 - k0), gg(k1 - k0);
            for (int k = k0; k < k1; ++k) {
                ii[k - k0] = items[k].inst;
                io[k - k0] = items[k].out;
                bb[k - k0] = items[k].beta;
                gg[k - k0] = items[k].gamma;
            }
            if ((s = sv_items_stream(n, k1 - k0, ii.data(), io.data(), bb.data(), gg.data(), costs, off.data(), m_host,
                                     target_host, num_p, p_list, psol, energy, st)))
                return s;
            continue;
        }
        SvItemsArgs a{};
        a.items = d_items + k0;
        a.num_items = k1 - k0;
        a.n = n_host[items[k0].inst];
        a.costs = costs;
        a.cost_off = d_off;
        a.m = d_m;
        a.target = d_t;
        a.num_p = num_p;
        for (int q = 0; q < num_p; ++q) a.p_list[q] = p_list[q];
        a.psol = psol;
        a.energy = energy;
        if ((s = sv_items_launch(a, dev, st))) return s;
    }
    GQ_HIP(hipStreamSynchronize(st));  // the host tables above end with this call
    return GQAOA_OK;
}

}  // namespace gqaoa
