// Fair-sampling metrics of a solution distribution (Sec. IV, the two
// right-hand columns of Table I), evaluated on noiseless output
// probabilities by Monte Carlo on the device.
//
//   * shots-to-all-solutions: one thread per run draws shots from the output
//     distribution (K solutions with probabilities p_k, the rest of the mass
//     a non-solution outcome) until every solution was seen; a 64-bit mask
//     records the solutions seen.
//   * shots-to-reject-fairness: one wave per trial draws from the
//     distribution conditioned on solutions; lane k holds the count O_k, a
//     ballot finds the drawn category, and the chi-squared test against the
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

__global__ void __launch_bounds__(256) reject_kernel(const double *__restrict__ cdf, int K, int trials, uint64_t seed,
                                                     double crit, int n_min, int max_draws, int32_t *__restrict__ out) {
    const int lane = threadIdx.x & (kWave - 1);
    const int trial = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (trial >= trials) return;  // whole waves
    // lane k < K-1 draws when u < cdf[k]; lanes from K-1 on always match, so
    // the first match is k, or K-1 when u is past cdf[K-2]
    const double c = lane < K - 1 ? cdf[lane] : __builtin_huge_val();
    int cnt = 0;          // O_lane
    int64_t sumsq = 0;    // sum_k O_k^2, the same in every lane
    int res = 0;
    for (int N = 1; N <= max_draws; ++N) {
        const double u = uniform_at(seed, ((uint64_t)trial << 32) + (uint64_t)(N - 1));
        const uint64_t b = __ballot(u < c);
        const int k = __builtin_ctzll(b);
        const int ck = __shfl(cnt, k, kWave);
        sumsq += 2 * (int64_t)ck + 1;
        if (lane == k) ++cnt;
        if (N >= n_min && (double)((int64_t)K * sumsq - (int64_t)N * N) > crit * (double)N) {
            res = N;
            break;
        }
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
