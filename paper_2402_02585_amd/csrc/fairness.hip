// Fair-sampling metrics of a solution distribution (Sec. IV, the two
// right-hand columns of Table I), evaluated on noiseless output
// probabilities by Monte Carlo on the device.
//
//   * shots-to-all-solutions: one thread per run draws shots from the output
//     distribution (K solutions with probabilities p_k, the rest of the mass
//     a non-solution outcome) until every solution was seen; a 64-bit mask
//     records the solutions seen.
//   * shots-to-reject-fairness: one wave per trial draws from the
//     distribution conditioned on solutions, 64 draws per step (one per
//     lane); lane k holds the count O_k, and the chi-squared test against the
//     uniform distribution is taken after every draw from N >= n_min on, in
//     the exact integer form K sum O_k^2 - N^2 > crit N.
//
// Random numbers: SplitMix64 (Steele, Lea and Flood, 2014) used
// counter-based, draw d of run r being output r * 2^32 + d of the generator
// started from state `seed`; u = (x >> 11) 2^-53. A draw is the first
// category k with u < cdf[k], cdf being running sums in index order (for
// shots, u past every solution is a non-solution; for conditional draws the
// last solution takes the rest).
#include "internal.h"

#include <vector>

namespace gqaoa {

constexpr int kFairMaxK = 64;
constexpr uint64_t kSmGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * kSmGamma;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double uniform_at(uint64_t seed, uint64_t k) {
    return (double)(splitmix64_at(seed, k) >> 11) * 0x1.0p-53;
}

__global__ void __launch_bounds__(256) shots_all_kernel(const double *__restrict__ cdf, int K, int runs, uint64_t seed,
                                                        int max_shots, int32_t *__restrict__ out) {
    __shared__ double c[kFairMaxK];
    for (int i = threadIdx.x; i < K; i += blockDim.x) c[i] = cdf[i];
    __syncthreads();
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= runs) return;
    const uint64_t full = K == 64 ? ~0ull : ((1ull << K) - 1ull);
    uint64_t seen = 0;
    int res = 0;
    for (int d = 0; d < max_shots; ++d) {
        const double u = uniform_at(seed, ((uint64_t)r << 32) + (uint64_t)d);
        int k = 0;
        while (k < K && !(u < c[k])) ++k;
        if (k < K) {
            seen |= 1ull << k;
            if (seen == full) {
                res = d + 1;
                break;
            }
        }
    }
    out[r] = res;
}

// One wave per trial, 64 consecutive draws per step: lane l takes draw
// N0 + l + 1 (its own SplitMix64 output) and finds its category by binary
// search of the cdf; per-category ballots give each draw the number of
// earlier draws of its category within the step, hence the count O_k just
// before it; the increments 2 O_k + 1 of sum O_k^2, prefix-summed over the
// lanes, give the sum after every draw, so each lane evaluates the test for
// its N exactly as a draw-by-draw loop would (same integers, same double
// comparison) and the first rejecting lane ends the trial.
__global__ void __launch_bounds__(256) reject_kernel(const double *__restrict__ cdf, int K, int trials, uint64_t seed,
                                                     double crit, int n_min, int max_draws, int32_t *__restrict__ out) {
    __shared__ double cs[kFairMaxK];
    for (int i = threadIdx.x; i < K; i += blockDim.x) cs[i] = cdf[i];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int trial = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (trial >= trials) return;  // whole waves, after the block's barrier
    const uint64_t below = (1ull << lane) - 1ull;  // lanes before this one
    int cnt = 0;          // O_lane (lanes < K)
    int64_t sumsq = 0;    // sum_k O_k^2 before the step, the same in every lane
    int res = 0;
    for (int N0 = 0; N0 < max_draws; N0 += kWave) {
        const int N = N0 + lane + 1;  // this lane's draw count
        const double u = uniform_at(seed, ((uint64_t)trial << 32) + (uint64_t)(N - 1));
        // first k < K-1 with u < cdf[k] (cdf nondecreasing), else K-1
        int lo = 0, len = K - 1;
        while (len > 0) {
            const int half = len >> 1;
            if (u < cs[lo + half]) {
                len = half;
            } else {
                lo += half + 1;
                len -= half + 1;
            }
        }
        const int cat = lo;
        int earlier = 0, add = 0;
        for (int k = 0; k < K; ++k) {
            const uint64_t m = __ballot(cat == k);
            if (cat == k) earlier = __popcll(m & below);
            if (lane == k) add = __popcll(m);
        }
        const int ck = __shfl(cnt, cat, kWave) + earlier;  // O_cat just before this draw
        int64_t s = 2 * (int64_t)ck + 1;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {  // inclusive prefix sum over the lanes
            const int64_t t = __shfl_up(s, off, kWave);
            if (lane >= off) s += t;
        }
        const int64_t sq = sumsq + s;
        const bool rej = N <= max_draws && N >= n_min &&
                         (double)((int64_t)K * sq - (int64_t)N * N) > crit * (double)N;
        const uint64_t r = __ballot(rej);
        if (r) {
            res = N0 + __builtin_ctzll(r) + 1;
            break;
        }
        sumsq += __shfl(s, kWave - 1, kWave);
        cnt += add;
    }
    if (lane == 0) out[trial] = res;
}

// cdf of p (running sums in index order), divided by the total when normalize
static std::vector<double> running_cdf(int K, const double *p, bool normalize) {
    std::vector<double> c(K);
    double s = 0.0;
    for (int k = 0; k < K; ++k) c[k] = s = s + p[k];
    if (normalize)
        for (int k = 0; k < K; ++k) c[k] = c[k] / s;
    return c;
}

int run_shots_to_all(int K, const double *p, int runs, uint64_t seed, int max_shots, int32_t *out, hipStream_t st) {
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    const std::vector<double> c = running_cdf(K, p, false);
    AsyncScratch guard(st);
    GQ_HIP(guard.alloc(sizeof(double) * K));
    double *d_c = reinterpret_cast<double *>(guard.ptr);
    GQ_HIP(hipMemcpyAsync(d_c, c.data(), sizeof(double) * K, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(shots_all_kernel, dim3((runs + 255) / 256), dim3(256), 0, st, d_c, K, runs, seed, max_shots, out);
    GQ_LAUNCH_CHECK();
    GQ_HIP(hipStreamSynchronize(st));  // the host cdf ends here
    return GQAOA_OK;
}

int run_draws_to_reject(int K, const double *q, int trials, uint64_t seed, double crit, int n_min, int max_draws,
                        int32_t *out, hipStream_t st) {
    DeviceInfo dev;
    int s = device_info(&dev);
    if (s) return s;
    const std::vector<double> c = running_cdf(K, q, true);
    AsyncScratch guard(st);
    GQ_HIP(guard.alloc(sizeof(double) * K));
    double *d_c = reinterpret_cast<double *>(guard.ptr);
    GQ_HIP(hipMemcpyAsync(d_c, c.data(), sizeof(double) * K, hipMemcpyHostToDevice, st));
    const int waves_per_block = 4;
    hipLaunchKernelGGL(reject_kernel, dim3((trials + waves_per_block - 1) / waves_per_block), dim3(waves_per_block * kWave),
                       0, st, d_c, K, trials, seed, crit, n_min, max_draws, out);
    GQ_LAUNCH_CHECK();
    GQ_HIP(hipStreamSynchronize(st));
    return GQAOA_OK;
}

}  // namespace gqaoa
