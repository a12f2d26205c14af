// Statevector evaluation of single-angle-pair work items of small instances,
// each state held in LDS: the independent statevector check of the batched
// level-space scan (Eq. (5) evolved amplitude by amplitude instead of level
// by level).
//
// One block of 1024 threads per item (instance, beta, gamma). The instance's
// cost table (from gqaoa_cost_batched) and the phase table e^{-i gamma k} are
// staged in LDS beside the complex64 state. Round j is one sweep over the
// state: it forms psi_{j-1} = phi_{j-1} + delta_{j-1} (the Grover mixer of
// the previous round applied lazily, as in the streaming round pass), reads
// out P_sol and E when j-1 is a requested round, applies the phase and sums
// phi_j; one block reduction (float64) gives delta_j = (e^{-i beta} - 1) S_j / 2^n.
// Each thread owns the same amplitudes in every round, so only the reduction
// needs barriers.
#include "batch.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace gqaoa {

constexpr int kItemThreads = 1024;

size_t sv_items_lds_bytes(int n) {
    const size_t N = size_t(1) << n;
    return 8 * N + ((N + 7) & ~size_t(7)) + 8 * 256;
}

__global__ void __launch_bounds__(kItemThreads) sv_items_kernel(SvItemsArgs a) {
    extern __shared__ unsigned char smem[];
    __shared__ double red_s[4 * kItemThreads / kWave];
    __shared__ double bc_s[4];
    const uint32_t N = 1u << a.n;
    float2 *psi = reinterpret_cast<float2 *>(smem);
    uint8_t *c = smem + 8 * (size_t)N;
    float2 *lut = reinterpret_cast<float2 *>(smem + 8 * (size_t)N + ((N + 7) & ~7u));
    const int tid = threadIdx.x;
    const double invN = ldexp(1.0, -a.n);
    const float amp0 = (float)sqrt(invN);  // |s> = 2^(-n/2) on every z
    const int pmax = a.p_list[a.num_p - 1];
    for (int item = blockIdx.x; item < a.num_items; item += gridDim.x) {
        const SvItem it = a.items[item];
        const uint8_t *src = a.costs + a.cost_off[it.inst];
        for (uint32_t z = tid; z < N; z += kItemThreads) c[z] = src[z];
        const int m = a.m[it.inst];
        const uint32_t target = (uint32_t)a.target[it.inst];
        for (int k = tid; k <= m; k += kItemThreads) {
            double s, co;
            sincos(fmod(it.gamma * (double)k, 2.0 * M_PI), &s, &co);
            lut[k] = float2{(float)co, (float)-s};
        }
        double sb, cb;
        sincos(it.beta, &sb, &cb);
        const double mr = cb - 1.0, mi = -sb;
        __syncthreads();
        float dr = 0.f, di = 0.f;
        int q = 0;
        for (int j = 1; j <= pmax + 1; ++j) {
            const bool rd = q < a.num_p && a.p_list[q] == j - 1;
            const bool ph = j <= pmax;
            float sr = 0.f, si = 0.f, sp = 0.f, se = 0.f;
            for (uint32_t z = tid; z < N; z += kItemThreads) {
                float2 x = j == 1 ? float2{amp0, 0.f} : psi[z];
                if (j > 1) {
                    x.x += dr;
                    x.y += di;
                }
                const uint32_t cz = c[z];
                if (rd) {
                    const float pr = x.x * x.x + x.y * x.y;
                    sp += cz == target ? pr : 0.f;
                    se += (float)cz * pr;
                }
                if (ph) {
                    const float2 e = lut[cz];
                    const float2 f{e.x * x.x - e.y * x.y, e.x * x.y + e.y * x.x};
                    psi[z] = f;
                    sr += f.x;
                    si += f.y;
                }
            }
            double r[4] = {sr, si, sp, se};
            block_sum<4, kItemThreads>(r, red_s);
            if (tid == 0)
                for (int k = 0; k < 4; ++k) bc_s[k] = r[k];
            __syncthreads();
            if (rd) {
                if (tid == 0) {
                    a.psol[(size_t)it.out * a.num_p + q] = (float)bc_s[2];
                    if (a.energy) a.energy[(size_t)it.out * a.num_p + q] = (float)bc_s[3];
                }
                ++q;
            }
            if (ph) {
                const double Sr = bc_s[0] * invN, Si = bc_s[1] * invN;
                dr = (float)(mr * Sr - mi * Si);
                di = (float)(mr * Si + mi * Sr);
            }
            __syncthreads();  // bc_s is rewritten by the next reduction
        }
    }
}

uint64_t batched_cost_offset(int i, const int32_t *n_host);

int sv_items_order(const int32_t *n_host, int num_items, const int32_t *item_inst, const DeviceInfo &dev,
                   ItemOrder *out) {
    for (int k = 0; k < num_items; ++k) {
        const size_t need = sv_items_lds_bytes(n_host[item_inst[k]]);
        if (need > dev.lds_per_block)
            return fail(GQAOA_ERANGE, "item %d: n=%d needs %zu bytes of LDS, the device offers %zu per block", k,
                        n_host[item_inst[k]], need, dev.lds_per_block);
    }
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

int sv_items_allow_lds(int n) {
    const size_t lds = sv_items_lds_bytes(n);
    if (lds > 65536)
        GQ_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(sv_items_kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    return GQAOA_OK;
}

int sv_items_launch(const SvItemsArgs &a, const DeviceInfo &dev, hipStream_t st) {
    const size_t lds = sv_items_lds_bytes(a.n);
    const int per_cu = std::max<int>(1, (int)std::min<size_t>(2, dev.lds_per_block / std::max<size_t>(lds, 1)));
    const int blocks = std::min(a.num_items, dev.num_cus * per_cu);
    hipLaunchKernelGGL(sv_items_kernel, dim3(blocks), dim3(kItemThreads), lds, st, a);
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

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
        if ((s = sv_items_allow_lds(a.n)) || (s = sv_items_launch(a, dev, st))) return s;
    }
    GQ_HIP(hipStreamSynchronize(st));  // the host tables above end with this call
    return GQAOA_OK;
}

}  // namespace gqaoa
