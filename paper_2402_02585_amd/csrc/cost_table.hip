// Cost table C(z) and level histogram N_k by bit-sliced clause evaluation.
//
// C(z) is the number of clauses left unsatisfied by assignment z, i.e. the
// diagonal of H_P (Sec. II.A, the clause energy that follows Eq. (1); App. B).
// N_k = #{z : C(z) = k} is the per-level state count of App. C. The word
// layout and clause records are described in cost_bits.h.
//
// Each lane evaluates one 32-assignment word per loop trip. Per wave tile the
// lanes first test the wave-uniform (high) literals of 64 clauses at a time and
// leave each clause's effective lane mask in wave-private LDS; then, per
// clause, one LDS broadcast read and a sign-extended bit extract select the
// low-literal pattern P for this lane, and a carry-save adder tree folds 16
// clauses at a time into eight bit-planes; 8x8 bit transposes turn the planes
// into byte costs. Clauses whose variables all sit in wave-uniform bits add a
// count found by a ballot.
// The histogram is tallied in LDS (one copy per wave) and written as per-block
// rows, which a second kernel sums in a fixed order.
#include "internal.h"
#include "cost_bits.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

namespace gqaoa {

constexpr int kCostThreads = 256;
constexpr int kCostWaves = kCostThreads / kWave;
constexpr int kMaxVec = 256;  // padded clause records per instance (m <= 255)
// LDS histogram copies per block: four per wave (by lane & 3). Copies are
// kHistStride = 257 words apart, so one level in different copies falls in
// different LDS banks: lanes of different copies tallying the same level
// neither share an address nor a bank.
constexpr int kHistCopies = kCostWaves * 4;
constexpr int kHistStride = 257;

// A clause's effective masks for one wave-tile, as each half-wave reads them:
// entry [c][h] = {P, bits 32h..32h+31 of L_eff} with L_eff = L if the clause's
// high literals are all false in this tile, else 0.
struct EffEntry {
    uint32_t P, Lhalf;
};

// Dynamic LDS of a cost block, sized by the padded clause count nvec:
// clause records [nvec], per-wave effective masks [waves][nvec][2], and the
// histogram copies [copies][kHistStride].
struct CostLds {
    ClauseRec *rec;
    EffEntry *eff;
    uint32_t *hist;
    __device__ CostLds(unsigned char *smem, int nvec)
        : rec(reinterpret_cast<ClauseRec *>(smem)),
          eff(reinterpret_cast<EffEntry *>(smem + sizeof(ClauseRec) * nvec)),
          hist(reinterpret_cast<uint32_t *>(smem + sizeof(ClauseRec) * nvec +
                                            sizeof(EffEntry) * 2 * kCostWaves * nvec)) {}
    __device__ EffEntry (*wave_eff(int nvec))[2] {
        return reinterpret_cast<EffEntry(*)[2]>(eff + (size_t)2 * nvec * (threadIdx.x / kWave));
    }
};

size_t cost_lds_bytes(int nvec) {
    return sizeof(ClauseRec) * nvec + sizeof(EffEntry) * 2 * kCostWaves * nvec +
           sizeof(uint32_t) * kHistCopies * kHistStride;
}

// Zero the histogram copies and stage the clause records in LDS.
__device__ __forceinline__ void stage(CostLds &s, const ClauseRec *__restrict__ vec, int nvec) {
    for (int i = threadIdx.x; i < kHistCopies * kHistStride; i += kCostThreads) s.hist[i] = 0;
    for (int i = threadIdx.x; i < nvec; i += kCostThreads) s.rec[i] = vec[i];
    __syncthreads();
}

__device__ __forceinline__ uint32_t *hist_copy(CostLds &s) {
    return s.hist + ((threadIdx.x / kWave) * 4 + (threadIdx.x & 3)) * kHistStride;
}

// Costs of the 32 assignments of word w = tile*64 + lane as bit planes: bit j
// of v[b] is bit b of C(z) for the assignment at word bit j. Every lane of the
// wave must call this with the same tile.
__device__ __forceinline__ void eval_planes(const ClauseRec *vec, int nvec, const UniformRec *uni, int nuni,
                                            uint64_t tile, EffEntry (*eff)[2], uint32_t (&v)[8]) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t zwave = (tile * kWave) << kLowBits;   // z of lane 0, bit 0
    // 1) high-literal test of 64 clauses at a time, one per lane
    for (int c = lane; c < nvec; c += kWave) {
        const ClauseRec r = vec[c];
        const uint64_t L = high_literals_false(zwave, r.hivar, r.hineg) ? r.L : 0ull;
        eff[c][0] = EffEntry{r.P, (uint32_t)L};
        eff[c][1] = EffEntry{r.P, (uint32_t)(L >> 32)};
    }
    uint32_t u = 0;
    for (int c0 = 0; c0 < nuni; c0 += kWave) {
        const int c = c0 + lane;
        const bool f = c < nuni && high_literals_false(zwave, uni[c].hivar, uni[c].hineg);
        u += (uint32_t)__popcll(__ballot(f));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // 2) per clause: the lane's bit of L_eff selects P; 16 clauses per adder tree
    const int half = lane >> 5, bit = lane & 31;
    SlicedCounter cnt;
    cnt.clear();
    for (int g = 0; g < nvec; g += kGroup) {
        uint32_t f[kGroup];
#pragma unroll
        for (int i = 0; i < kGroup; ++i) {
            const EffEntry e = eff[g + i][half];
            f[i] = e.P & (uint32_t)__builtin_amdgcn_sbfe((int)e.Lhalf, bit, 1);
        }
        cnt.add16(f);
    }
    cnt.add_scalar(u);  // no overflow: every count <= m <= 255
#pragma unroll
    for (int b = 0; b < 8; ++b) v[b] = cnt.p[b];
    // the next tile rewrites eff: every lane's reads of this one come first
    __builtin_amdgcn_wave_barrier();
}

// Planes to bytes: out[r] byte q = C of word bit 8q + r, i.e. C(32 w + 4 r + q).
__device__ __forceinline__ void planes_to_bytes(const uint32_t (&v)[8], uint32_t (&out)[8]) {
    SlicedCounter c;
#pragma unroll
    for (int b = 0; b < 8; ++b) c.p[b] = v[b];
    c.transpose_to_bytes();
#pragma unroll
    for (int r = 0; r < 8; ++r) out[r] = c.p[r];
}

// Per-lane level counters for NB aligned blocks of 32 levels starting at
// level 32 a0, fed straight from the bit planes: the assignments of a word at
// level 32 a + k are the word bits where the planes spell a (planes 5..7) and
// k (planes 0..4), found with a shared AND tree and counted with popcounts.
// Levels outside the window are returned as a word-bit mask for the caller.
template <int NB>
struct LevelWindow {
    uint32_t cnt[NB][32];
    int a0;
    __device__ __forceinline__ void clear(int a) {
        a0 = a;
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int k = 0; k < 32; ++k) cnt[i][k] = 0;
    }
    __device__ __forceinline__ uint32_t add(const uint32_t (&v)[8]) {
        uint32_t in = 0;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int a = a0 + i;  // uniform
            const uint32_t hi = (v[5] ^ ((a & 1) ? 0u : ~0u)) & (v[6] ^ ((a & 2) ? 0u : ~0u)) &
                                (v[7] ^ ((a & 4) ? 0u : ~0u));
            in |= hi;
#pragma unroll
            for (int k43 = 0; k43 < 4; ++k43) {
                const uint32_t t3 = hi & ((k43 & 2) ? v[4] : ~v[4]) & ((k43 & 1) ? v[3] : ~v[3]);
#pragma unroll
                for (int b2 = 0; b2 < 2; ++b2) {
                    const uint32_t t2 = t3 & (b2 ? v[2] : ~v[2]);
#pragma unroll
                    for (int k10 = 0; k10 < 4; ++k10) {
                        const uint32_t leaf = t2 & ((k10 & 2) ? v[1] : ~v[1]) & ((k10 & 1) ? v[0] : ~v[0]);
                        cnt[i][(k43 << 3) | (b2 << 2) | k10] += (uint32_t)__builtin_popcount(leaf);
                    }
                }
            }
        }
        return ~in;
    }
    // add the counters into an LDS histogram (levels < 256)
    __device__ __forceinline__ void flush(uint32_t *h) const {
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
            for (int k = 0; k < 32; ++k)
                if (cnt[i][k] && a0 + i < 8) atomicAdd(h + 32 * (a0 + i) + k, cnt[i][k]);
    }
};

// Tally the word bits of `mask` one by one from the cost bytes (the rare
// levels outside the window).
__device__ __forceinline__ void tally_bits(uint32_t *h, const uint32_t (&t)[8], uint32_t mask) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if ((mask >> (8 * q + r)) & 1u) atomicAdd(h + ((t[r] >> (8 * q)) & 0xFFu), 1u);
}

__device__ __forceinline__ void tally(uint32_t *h, uint32_t v) {
    atomicAdd(h + (v & 0xFFu), 1u);
    atomicAdd(h + ((v >> 8) & 0xFFu), 1u);
    atomicAdd(h + ((v >> 16) & 0xFFu), 1u);
    atomicAdd(h + (v >> 24), 1u);
}

__device__ __forceinline__ void tally_word(uint32_t *h, const uint32_t (&t)[8], uint32_t nbits) {
    if (nbits == 32u) {
#pragma unroll
        for (int r = 0; r < 8; ++r) tally(h, t[r]);
    } else {
        for (uint32_t z = 0; z < nbits; ++z) atomicAdd(h + ((t[z >> 2] >> (8 * (z & 3))) & 0xFFu), 1u);
    }
}

template <int NB>
__global__ void __launch_bounds__(kCostThreads)
cost_table_kernel(const ClauseRec *__restrict__ vec, int nvec, const UniformRec *__restrict__ uni,
                  int nuni, int n, uint8_t *__restrict__ cost, uint32_t *__restrict__ block_hist,
                  int hist_len, int win_a0) {
    extern __shared__ unsigned char smem[];
    CostLds lds(smem, nvec);
    stage(lds, vec, nvec);
    uint32_t *h = hist_copy(lds);
    EffEntry(*eff)[2] = lds.wave_eff(nvec);
    const uint64_t N = 1ull << n;
    const uint64_t nwords = n >= kLowBits ? (N >> kLowBits) : 1;
    const uint64_t ntiles = (nwords + kWave - 1) / kWave;
    const uint64_t nwaves = (uint64_t)gridDim.x * kCostWaves;
    const int lane = threadIdx.x & (kWave - 1);
    LevelWindow<NB> win;
    win.clear(win_a0);
    for (uint64_t tile = (uint64_t)blockIdx.x * kCostWaves + threadIdx.x / kWave; tile < ntiles; tile += nwaves) {
        uint32_t v[8], t[8];
        eval_planes(lds.rec, nvec, uni, nuni, tile, eff, v);
        const uint64_t w = tile * kWave + lane;
        if (w >= nwords) continue;
        if (n >= kLowBits) {
            const uint32_t outside = win.add(v);
            planes_to_bytes(v, t);
            typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
            u32x4 *dst = reinterpret_cast<u32x4 *>(cost + (w << kLowBits));
            dst[0] = u32x4{t[0], t[1], t[2], t[3]};
            dst[1] = u32x4{t[4], t[5], t[6], t[7]};
            if (outside) tally_bits(h, t, outside);
        } else {
            planes_to_bytes(v, t);
            for (uint32_t z = 0; z < (uint32_t)N; ++z) cost[z] = (uint8_t)((t[z >> 2] >> (8 * (z & 3))) & 0xFFu);
            tally_word(h, t, (uint32_t)N);
        }
    }
    win.flush(h);
    __syncthreads();
    for (int k = threadIdx.x; k < hist_len; k += kCostThreads) {
        uint32_t s = 0;
        for (int c = 0; c < kHistCopies; ++c) s += lds.hist[c * kHistStride + k];
        block_hist[(size_t)blockIdx.x * hist_len + k] = s;
    }
}

// hist[k] = sum over blocks of block_hist[b][k]: one block per level k, every
// thread sums a strided subset of rows (integer sums, so the order is free).
__global__ void __launch_bounds__(256) hist_reduce_kernel(const uint32_t *__restrict__ block_hist,
                                                          int nblocks, int hist_len,
                                                          unsigned long long *__restrict__ hist) {
    __shared__ unsigned long long red[256];
    const int k = blockIdx.x;
    unsigned long long s = 0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s += block_hist[(size_t)b * hist_len + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) hist[k] = red[0];
}

// ---- many instances, histograms only ---------------------------------------
// Clause ingest runs on the device here: each block builds its instance's
// records from the raw literals straight into LDS (every clause as a vector
// record, padded to the adder-tree group), so the host uploads 12 bytes per
// clause and packs nothing.
struct HistInst {
    uint32_t lit_off;   // first clause of the instance in the literal array
    int32_t n, m;
    int32_t win_a0;     // first 32-level block of the counting window
    uint64_t cost_off;  // byte offset of the instance's cost table (when costs are written)
};
struct HistUnit {
    uint32_t inst, word0, nwords, pad;
};

__global__ void __launch_bounds__(kCostThreads)
hist_batched_kernel(const HistInst *__restrict__ insts, const HistUnit *__restrict__ units,
                    const int32_t *__restrict__ lits, unsigned long long *__restrict__ hists, int hist_stride,
                    uint8_t *__restrict__ costs) {
    extern __shared__ unsigned char smem[];
    const HistUnit unit = units[blockIdx.x];
    const HistInst in = insts[unit.inst];
    const int nvec = (in.m + kGroup - 1) / kGroup * kGroup;
    CostLds lds(smem, nvec);
    const int32_t *L = lits + 3 * (size_t)in.lit_off;
    for (int i = threadIdx.x; i < kHistCopies * kHistStride; i += kCostThreads) lds.hist[i] = 0;
    for (int c = threadIdx.x; c < nvec; c += kCostThreads)
        lds.rec[c] = c < in.m ? make_record(L[3 * c], L[3 * c + 1], L[3 * c + 2], nullptr)
                              : ClauseRec{0u, 0u, 0ull, 0ull, 0ull};
    __syncthreads();
    uint32_t *h = hist_copy(lds);
    EffEntry(*eff)[2] = lds.wave_eff(nvec);
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t nbits = in.n >= kLowBits ? 32u : (1u << in.n);
    const uint32_t ntiles = (unit.nwords + kWave - 1) / kWave;
    LevelWindow<2> win;
    win.clear(in.win_a0);
    for (uint32_t t0 = threadIdx.x / kWave; t0 < ntiles; t0 += kCostWaves) {
        // word0 is a multiple of 64, so tile (word0 / 64 + t0) starts at word0 + 64 t0
        const uint64_t tile = (uint64_t)unit.word0 / kWave + t0;
        uint32_t v[8], t[8];
        eval_planes(lds.rec, nvec, nullptr, 0, tile, eff, v);
        if (t0 * kWave + lane >= unit.nwords) continue;
        if (nbits == 32u) {
            const uint32_t outside = win.add(v);
            if (outside || costs) planes_to_bytes(v, t);
            if (outside) tally_bits(h, t, outside);
            if (costs) {
                typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
                const uint64_t w = (uint64_t)unit.word0 + t0 * kWave + lane;
                u32x4 *dst = reinterpret_cast<u32x4 *>(costs + in.cost_off + (w << kLowBits));
                dst[0] = u32x4{t[0], t[1], t[2], t[3]};
                dst[1] = u32x4{t[4], t[5], t[6], t[7]};
            }
        } else {
            planes_to_bytes(v, t);
            tally_word(h, t, nbits);
            if (costs)
                for (uint32_t z = 0; z < nbits; ++z)
                    costs[in.cost_off + z] = (uint8_t)((t[z >> 2] >> (8 * (z & 3))) & 0xFFu);
        }
    }
    win.flush(h);
    __syncthreads();
    for (int k = threadIdx.x; k <= in.m; k += kCostThreads) {
        uint32_t s = 0;
        for (int c = 0; c < kHistCopies; ++c) s += lds.hist[c * kHistStride + k];
        if (s && hists) atomicAdd(hists + (size_t)unit.inst * hist_stride + k, (unsigned long long)s);
    }
}

// ---- host launchers (arguments already validated) ---------------------------
// Counting window for an instance with m clauses: C has mean m/8 over all
// assignments (each clause is false on 1/8 of them) and, for random clauses,
// a spread of about sqrt(7m/64); the window is the aligned 32-level blocks
// covering mean +- 4 spreads, at most two. Levels outside it are still
// counted exactly, one by one.
static void level_window(int m, int *a0, int *nb) {
    const double mu = m / 8.0, sd = std::sqrt(m * 7.0 / 64.0);
    const int lo = std::max(0, (int)std::floor(mu - 4.0 * sd));
    const int hi = std::min(m, (int)std::ceil(mu + 4.0 * sd));
    *a0 = lo / 32;
    *nb = std::min(2, hi / 32 - *a0 + 1);
}

// Cost kernel and histogram reduce on records already on the device.
static int enqueue_cost_kernels(int n, int m, int nblocks, int nvec, int nuni, const ClauseRec *d_vec,
                                const UniformRec *d_uni, uint32_t *d_bh, uint8_t *cost, uint64_t *hist,
                                hipStream_t stream) {
    const int hist_len = m + 1;
    int a0 = 0, nb = 1;
    level_window(m, &a0, &nb);
    ProfScope ps("cost_table", stream);
    if (nb == 1)
        hipLaunchKernelGGL(cost_table_kernel<1>, dim3(nblocks), dim3(kCostThreads), cost_lds_bytes(nvec), stream,
                           d_vec, nvec, d_uni, nuni, n, cost, d_bh, hist_len, a0);
    else
        hipLaunchKernelGGL(cost_table_kernel<2>, dim3(nblocks), dim3(kCostThreads), cost_lds_bytes(nvec), stream,
                           d_vec, nvec, d_uni, nuni, n, cost, d_bh, hist_len, a0);
    ps.end();
    GQ_LAUNCH_CHECK();
    if (hist) {
        hipLaunchKernelGGL(hist_reduce_kernel, dim3(hist_len), dim3(256), 0, stream, d_bh, nblocks, hist_len,
                           reinterpret_cast<unsigned long long *>(hist));
        GQ_LAUNCH_CHECK();
    }
    return GQAOA_OK;
}

static int cost_grid(int n, const DeviceInfo &dev, int cap) {
    const uint64_t nwords = n >= kLowBits ? (1ull << (n - kLowBits)) : 1;
    const uint64_t want = (nwords + kCostThreads - 1) / kCostThreads;
    return (int)std::min<uint64_t>(want, (uint64_t)std::min(dev.num_cus * 8, cap));
}

int launch_cost_table(int n, int m, const int32_t *lits, uint8_t *cost, uint64_t *hist,
                      hipStream_t stream) {
    DeviceInfo dev;
    int st = device_info(&dev);
    if (st) return st;
    std::vector<ClauseRec> vec;
    std::vector<UniformRec> uni;
    pack_clauses(m, lits, vec, uni);
    const int nblocks = cost_grid(n, dev, 1 << 30);
    const int hist_len = m + 1;
    const size_t rec_bytes = sizeof(ClauseRec) * vec.size() + sizeof(UniformRec) * (uni.size() + 1);
    const size_t bh_bytes = sizeof(uint32_t) * (size_t)nblocks * hist_len;
    AsyncScratch guard(stream);
    GQ_HIP(guard.alloc(rec_bytes + bh_bytes + 256));
    void *scratch = guard.ptr;
    ClauseRec *d_vec = reinterpret_cast<ClauseRec *>(scratch);
    UniformRec *d_uni = reinterpret_cast<UniformRec *>(d_vec + vec.size());
    uint32_t *d_bh = reinterpret_cast<uint32_t *>(
        (reinterpret_cast<uintptr_t>(d_uni + uni.size() + 1) + 255) & ~uintptr_t(255));
    std::vector<char> staging(rec_bytes);
    memcpy(staging.data(), vec.data(), sizeof(ClauseRec) * vec.size());
    if (!uni.empty()) memcpy(staging.data() + sizeof(ClauseRec) * vec.size(), uni.data(), sizeof(UniformRec) * uni.size());
    GQ_HIP(hipMemcpyAsync(scratch, staging.data(), rec_bytes, hipMemcpyHostToDevice, stream));
    GQ_HIP(hipStreamSynchronize(stream));  // staging is host pageable memory owned here
    return enqueue_cost_kernels(n, m, nblocks, (int)vec.size(), (int)uni.size(), d_vec, d_uni, d_bh, cost, hist,
                                stream);
}

// ---- allocation-free form: scratch in a static device array --------------------------------
// The clause records and the per-block histogram rows of gqaoa_cost_table,
// for callers that cannot allocate device memory. The grid is capped at
// kStaticBlocks blocks (the kernel's loop over tiles covers any n), so every
// valid (n, m) fits: 12 KiB of records and at most 2 MiB of rows. Each GPU
// holds its own copy of the array until the process ends; host code reaches it
// only through the address hipGetSymbolAddress returns on that device.
constexpr int kStaticBlocks = 2048;
constexpr size_t kStaticRecBytes =
    (sizeof(ClauseRec) * kMaxVec + sizeof(UniformRec) * kMaxVec + 255) & ~size_t(255);
constexpr size_t kStaticRowBytes = sizeof(uint32_t) * (size_t)kStaticBlocks * kMaxVec;
constexpr size_t kStaticScratchBytes = kStaticRecBytes + kStaticRowBytes;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static std::map<int, unsigned char *> g_scratch_addr;  // device -> device address of `scratch`

// Device address of this device's copy of `scratch`, looked up once per
// device (with that device current).
static int static_scratch(unsigned char **out) {
    int dev = -1;
    GQ_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it == g_scratch_addr.end()) {
        void *ptr = nullptr;
        GQ_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        it = g_scratch_addr.emplace(dev, reinterpret_cast<unsigned char *>(ptr)).first;
    }
    *out = it->second;
    return GQAOA_OK;
}

int launch_cost_table_noalloc(int n, int m, const int32_t *lits, uint8_t *cost, uint64_t *hist,
                              hipStream_t stream) {
    DeviceInfo dev;
    int st = device_info(&dev);
    if (st) return st;
    unsigned char *base = nullptr;
    if ((st = static_scratch(&base))) return st;
    ClauseRec vec[kMaxVec];
    UniformRec uni[kMaxVec];
    int nvec = 0, nuni = 0;
    pack_clauses(m, lits, vec, &nvec, uni, &nuni);
    const int nblocks = cost_grid(n, dev, kStaticBlocks);
    const size_t vec_bytes = sizeof(ClauseRec) * (size_t)nvec, uni_bytes = sizeof(UniformRec) * (size_t)nuni;
    const size_t row_bytes = sizeof(uint32_t) * (size_t)nblocks * (size_t)(m + 1);
    if (vec_bytes + uni_bytes > kStaticRecBytes || row_bytes > kStaticRowBytes)
        return fail(GQAOA_ERANGE, "cost table n=%d m=%d needs %zu + %zu scratch bytes, more than the static %zu + %zu",
                    n, m, vec_bytes + uni_bytes, row_bytes, kStaticRecBytes, kStaticRowBytes);
    ClauseRec *d_vec = reinterpret_cast<ClauseRec *>(base);
    UniformRec *d_uni = reinterpret_cast<UniformRec *>(base + vec_bytes);
    uint32_t *d_bh = reinterpret_cast<uint32_t *>(base + kStaticRecBytes);
    if (nvec) GQ_HIP(hipMemcpyAsync(d_vec, vec, vec_bytes, hipMemcpyHostToDevice, stream));
    if (nuni) GQ_HIP(hipMemcpyAsync(d_uni, uni, uni_bytes, hipMemcpyHostToDevice, stream));
    GQ_HIP(hipStreamSynchronize(stream));  // the records are host stack memory of this call
    // every block writes its whole row of hist_len counts, so no row needs clearing
    return enqueue_cost_kernels(n, m, nblocks, nvec, nuni, d_vec, d_uni, d_bh, cost, hist, stream);
}

// Byte offset of each instance's cost table in the concatenated output: the
// tables follow each other in instance order, each starting at a multiple of
// 64 bytes.
uint64_t batched_cost_offset(int i, const int32_t *n_host) {
    uint64_t off = 0;
    for (int j = 0; j < i; ++j) off += ((1ull << n_host[j]) + 63) & ~63ull;
    return off;
}

int launch_hist_batched(int num_inst, const int32_t *n_host, const int32_t *m_host,
                        const int32_t *lits, uint64_t *hists, int hist_stride, uint8_t *costs, hipStream_t stream) {
    std::vector<HistInst> insts(num_inst);
    std::vector<HistUnit> units;
    constexpr uint32_t kUnitWords = kCostThreads * 4;
    size_t off = 0;
    int max_m = 1;
    for (int i = 0; i < num_inst; ++i) max_m = std::max(max_m, m_host[i]);
    const size_t smem_bytes = cost_lds_bytes((max_m + kGroup - 1) / kGroup * kGroup);
    uint64_t cost_off = 0;
    for (int i = 0; i < num_inst; ++i) {
        int a0 = 0, nb = 1;
        level_window(m_host[i], &a0, &nb);
        insts[i] = HistInst{(uint32_t)off, n_host[i], m_host[i], a0, cost_off};
        cost_off += ((1ull << n_host[i]) + 63) & ~63ull;
        off += (size_t)m_host[i];
        const uint64_t nwords = n_host[i] >= kLowBits ? (1ull << (n_host[i] - kLowBits)) : 1;
        for (uint64_t w0 = 0; w0 < nwords; w0 += kUnitWords)
            units.push_back(HistUnit{(uint32_t)i, (uint32_t)w0,
                                     (uint32_t)std::min<uint64_t>(kUnitWords, nwords - w0), 0u});
    }
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t b_inst = sizeof(HistInst) * insts.size();
    const size_t b_unit = sizeof(HistUnit) * units.size();
    const size_t b_lits = sizeof(int32_t) * 3 * off;
    const size_t o_unit = al(b_inst), o_lits = o_unit + al(b_unit);
    AsyncScratch guard(stream);
    GQ_HIP(guard.alloc(o_lits + al(b_lits)));
    void *scratch = guard.ptr;
    char *base = reinterpret_cast<char *>(scratch);
    GQ_HIP(hipMemcpyAsync(base, insts.data(), b_inst, hipMemcpyHostToDevice, stream));
    GQ_HIP(hipMemcpyAsync(base + o_unit, units.data(), b_unit, hipMemcpyHostToDevice, stream));
    GQ_HIP(hipMemcpyAsync(base + o_lits, lits, b_lits, hipMemcpyHostToDevice, stream));
    if (hists) GQ_HIP(hipMemsetAsync(hists, 0, sizeof(uint64_t) * (size_t)num_inst * hist_stride, stream));
    hipLaunchKernelGGL(hist_batched_kernel, dim3((unsigned)units.size()), dim3(kCostThreads), smem_bytes, stream,
                       reinterpret_cast<const HistInst *>(base), reinterpret_cast<const HistUnit *>(base + o_unit),
                       reinterpret_cast<const int32_t *>(base + o_lits),
                       reinterpret_cast<unsigned long long *>(hists), hist_stride, costs);
    GQ_LAUNCH_CHECK();
    GQ_HIP(hipStreamSynchronize(stream));  // the host tables above end with this call
    return GQAOA_OK;
}

}  // namespace gqaoa
