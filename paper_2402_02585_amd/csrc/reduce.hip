// Small device-side selections the drivers need between library calls, so
// that no host framework computes on device data:
//  * row_best: per row of a matrix, the best entry (largest or smallest
//    float, or least positive int32) and its column, ties to the lowest
//    column - the best grid cell of a scan, the earliest first crossing;
//  * level_probs: the assignments z of one cost level, ascending, and their
//    output probabilities |psi_z|^2 (the solution distribution sampled in
//    Sec. IV), by an ordered three-pass compaction;
//  * mlp_angles: the network's angle map beta = 2 pi sigmoid(o0),
//    gamma = pi sigmoid(o1), in float64;
//  * gather_rows: rows of a table picked by device indices (training batches).
#include "internal.h"

#include <algorithm>
#include <climits>
#include <cmath>

namespace gqaoa {

// ---- per-row best entry -----------------------------------------------------------------
constexpr int kRowThreads = 256;

// (v, i) is better than (bv, bi) for mode 0 (largest float), 1 (smallest
// float), 2 (least positive int, stored as float-free int in iv). A NaN is
// never better than a number; among equal values the lower index wins.
template <int MODE>
struct RowBest {
    float f;
    int32_t iv;
    int32_t idx;  // INT_MAX: no candidate yet
    __device__ __forceinline__ void init() {
        f = 0.f;
        iv = 0;
        idx = INT_MAX;
    }
    __device__ __forceinline__ bool better_than(const RowBest &o) const {
        if (idx == INT_MAX) return false;
        if (o.idx == INT_MAX) return true;
        if constexpr (MODE == 2) {
            if (iv != o.iv) return iv < o.iv;
        } else {
            const bool n0 = f != f, n1 = o.f != o.f;
            if (n0 != n1) return n1;        // a number beats a NaN
            if (!n0 && f != o.f) return MODE == 0 ? f > o.f : f < o.f;
        }
        return idx < o.idx;
    }
};

template <int MODE>
__global__ void __launch_bounds__(kRowThreads) row_best_kernel(int cols, const void *__restrict__ x,
                                                               int32_t *__restrict__ out_idx, void *__restrict__ out_val) {
    __shared__ RowBest<MODE> red[kRowThreads / 64];
    const size_t row = blockIdx.x;
    RowBest<MODE> b;
    b.init();
    for (int c = threadIdx.x; c < cols; c += kRowThreads) {
        RowBest<MODE> cand;
        cand.idx = c;
        if constexpr (MODE == 2) {
            const int32_t v = reinterpret_cast<const int32_t *>(x)[row * cols + c];
            if (v <= 0) continue;   // only positive entries are candidates
            cand.iv = v;
            cand.f = 0.f;
        } else {
            cand.f = reinterpret_cast<const float *>(x)[row * cols + c];
            cand.iv = 0;
        }
        if (cand.better_than(b)) b = cand;
    }
    // wave, then block: the order of the comparisons does not change the result
    // (the best under a strict total order with index tie-break)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        RowBest<MODE> o;
        o.f = __shfl_xor(b.f, off, 64);
        o.iv = __shfl_xor(b.iv, off, 64);
        o.idx = __shfl_xor(b.idx, off, 64);
        if (o.better_than(b)) b = o;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kRowThreads / 64; ++w)
            if (red[w].better_than(b)) b = red[w];
        if constexpr (MODE == 2) {
            out_idx[row] = b.idx == INT_MAX ? 0 : b.idx;
            if (out_val) reinterpret_cast<int32_t *>(out_val)[row] = b.idx == INT_MAX ? 0 : b.iv;
        } else {
            out_idx[row] = b.idx == INT_MAX ? 0 : b.idx;
            if (out_val) reinterpret_cast<float *>(out_val)[row] = b.f;
        }
    }
}

int run_row_best(int rows, int cols, const void *x, int mode, int32_t *idx, void *val, hipStream_t st) {
    const dim3 grid((unsigned)rows), block(kRowThreads);
    if (mode == 0)
        hipLaunchKernelGGL(row_best_kernel<0>, grid, block, 0, st, cols, x, idx, val);
    else if (mode == 1)
        hipLaunchKernelGGL(row_best_kernel<1>, grid, block, 0, st, cols, x, idx, val);
    else
        hipLaunchKernelGGL(row_best_kernel<2>, grid, block, 0, st, cols, x, idx, val);
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

// ---- assignments of one level and their probabilities -------------------------------------
// The state is cut into chunks of kChunk consecutive z (one block each, every
// thread a run of kPerThread). Pass 1 counts the matches per chunk, pass 2
// turns the counts into chunk offsets (one block, in order), pass 3 writes
// every match at its rank: chunk offset + the matches of earlier threads of
// the block + the earlier matches of the thread's own run.
constexpr int kLpThreads = 256;
constexpr int kPerThread = 64;
constexpr uint64_t kChunk = (uint64_t)kLpThreads * kPerThread;

static uint64_t lp_chunks(int n) { return ((1ull << n) + kChunk - 1) / kChunk; }

size_t level_probs_workspace_bytes(int n) { return sizeof(uint64_t) * (size_t)(lp_chunks(n) + 1); }

__device__ __forceinline__ uint32_t run_matches(const uint8_t *__restrict__ cost, uint64_t z0, uint64_t N,
                                                uint8_t level) {
    uint32_t c = 0;
    for (int i = 0; i < kPerThread; ++i) {
        const uint64_t z = z0 + i;
        c += (z < N && cost[z] == level) ? 1u : 0u;
    }
    return c;
}

__global__ void __launch_bounds__(kLpThreads) lp_count_kernel(const uint8_t *__restrict__ cost, uint64_t N,
                                                              uint8_t level, uint64_t *__restrict__ counts) {
    __shared__ uint32_t red[kLpThreads];
    const uint64_t z0 = (uint64_t)blockIdx.x * kChunk + (uint64_t)threadIdx.x * kPerThread;
    red[threadIdx.x] = run_matches(cost, z0, N, level);
    __syncthreads();
    for (int w = kLpThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = red[0];
}

// counts[0..nchunks) -> exclusive offsets, counts[nchunks] = total
__global__ void __launch_bounds__(1024) lp_offsets_kernel(uint64_t *__restrict__ counts, uint64_t nchunks) {
    __shared__ uint64_t part[1024];
    const uint64_t per = (nchunks + 1023) / 1024;
    const uint64_t b0 = threadIdx.x * per, b1 = std::min<uint64_t>(nchunks, b0 + per);
    uint64_t s = 0;
    for (uint64_t b = b0; b < b1; ++b) s += counts[b];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t run = 0;
        for (int t = 0; t < 1024; ++t) {
            const uint64_t v = part[t];
            part[t] = run;
            run += v;
        }
        counts[nchunks] = run;
    }
    __syncthreads();
    uint64_t run = part[threadIdx.x];
    for (uint64_t b = b0; b < b1; ++b) {
        const uint64_t v = counts[b];
        counts[b] = run;
        run += v;
    }
}

template <typename T>
__global__ void __launch_bounds__(kLpThreads) lp_write_kernel(const uint8_t *__restrict__ cost, const T *__restrict__ psi,
                                                              uint64_t N, uint8_t level,
                                                              const uint64_t *__restrict__ offsets, uint64_t max_out,
                                                              int64_t *__restrict__ z_out, double *__restrict__ p_out) {
    __shared__ uint32_t scan[kLpThreads];
    const uint64_t z0 = (uint64_t)blockIdx.x * kChunk + (uint64_t)threadIdx.x * kPerThread;
    const uint32_t mine = run_matches(cost, z0, N, level);
    scan[threadIdx.x] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {  // exclusive prefix over the block's threads, in order
        uint32_t run = 0;
        for (int t = 0; t < kLpThreads; ++t) {
            const uint32_t v = scan[t];
            scan[t] = run;
            run += v;
        }
    }
    __syncthreads();
    if (!mine) return;
    uint64_t pos = offsets[blockIdx.x] + scan[threadIdx.x];
    for (int i = 0; i < kPerThread && pos < max_out; ++i) {
        const uint64_t z = z0 + i;
        if (z < N && cost[z] == level) {
            const double re = (double)psi[2 * z], im = (double)psi[2 * z + 1];
            if (z_out) z_out[pos] = (int64_t)z;
            if (p_out) p_out[pos] = re * re + im * im;
            ++pos;
        }
    }
}

int run_level_probs(int n, const uint8_t *cost, const void *psi, int dtype, int level, int64_t max_out,
                    int64_t *z_out, double *p_out, int64_t *count, void *ws, hipStream_t st) {
    const uint64_t N = 1ull << n, nch = lp_chunks(n);
    uint64_t *counts = reinterpret_cast<uint64_t *>(ws);
    hipLaunchKernelGGL(lp_count_kernel, dim3((unsigned)nch), dim3(kLpThreads), 0, st, cost, N, (uint8_t)level, counts);
    GQ_LAUNCH_CHECK();
    hipLaunchKernelGGL(lp_offsets_kernel, dim3(1), dim3(1024), 0, st, counts, nch);
    GQ_LAUNCH_CHECK();
    if (max_out > 0) {
        if (dtype == GQAOA_C64)
            hipLaunchKernelGGL(lp_write_kernel<float>, dim3((unsigned)nch), dim3(kLpThreads), 0, st, cost,
                               reinterpret_cast<const float *>(psi), N, (uint8_t)level, counts, (uint64_t)max_out,
                               z_out, p_out);
        else
            hipLaunchKernelGGL(lp_write_kernel<double>, dim3((unsigned)nch), dim3(kLpThreads), 0, st, cost,
                               reinterpret_cast<const double *>(psi), N, (uint8_t)level, counts, (uint64_t)max_out,
                               z_out, p_out);
        GQ_LAUNCH_CHECK();
    }
    uint64_t total = 0;
    GQ_HIP(hipMemcpyAsync(&total, counts + nch, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    GQ_HIP(hipStreamSynchronize(st));
    *count = (int64_t)total;
    return GQAOA_OK;
}

// ---- angle map of the network ------------------------------------------------------------
__global__ void mlp_angles_kernel(int batch, const float *__restrict__ out, double *__restrict__ beta,
                                  double *__restrict__ gamma) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const double o0 = (double)out[2 * b], o1 = (double)out[2 * b + 1];
    beta[b] = 2.0 * M_PI / (1.0 + exp(-o0));
    gamma[b] = M_PI / (1.0 + exp(-o1));
}

int run_mlp_angles(int batch, const float *out, double *beta, double *gamma, hipStream_t st) {
    hipLaunchKernelGGL(mlp_angles_kernel, dim3((batch + 255) / 256), dim3(256), 0, st, batch, out, beta, gamma);
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

// ---- row gather ----------------------------------------------------------------------------
// dst row r = src row idx[r] (row_words 32-bit words each); an index outside
// [0, src_rows) gives a row of zeros.
__global__ void gather_rows_kernel(int rows, const int32_t *__restrict__ idx, int src_rows,
                                   const uint32_t *__restrict__ src, int row_words, uint32_t *__restrict__ dst) {
    const int r = blockIdx.x;
    if (r >= rows) return;
    const int32_t s = idx[r];
    const bool ok = s >= 0 && s < src_rows;
    for (int w = threadIdx.x; w < row_words; w += blockDim.x)
        dst[(size_t)r * row_words + w] = ok ? src[(size_t)s * row_words + w] : 0u;
}

int run_gather_rows(int rows, const int32_t *idx, int src_rows, const void *src, int row_bytes, void *dst,
                    hipStream_t st) {
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)rows), dim3(64), 0, st, rows, idx, src_rows,
                       reinterpret_cast<const uint32_t *>(src), row_bytes / 4, reinterpret_cast<uint32_t *>(dst));
    GQ_LAUNCH_CHECK();
    return GQAOA_OK;
}

}  // namespace gqaoa
