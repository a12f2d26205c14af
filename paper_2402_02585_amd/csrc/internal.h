// Internal helpers shared by the libgqaoa translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/gqaoa.h"

namespace gqaoa {

// ---- status / error reporting ------------------------------------------------
void set_error(const char *fmt, ...);
void clear_error();
int fail(int status, const char *fmt, ...);

#define GQ_HIP(call)                                                             \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess)                                                    \
            return ::gqaoa::fail(GQAOA_EHIP, "%s failed: %s (%s:%d)", #call,      \
                                 hipGetErrorString(e_), __FILE__, __LINE__);     \
    } while (0)

#define GQ_LAUNCH_CHECK()                                                        \
    do {                                                                         \
        hipError_t e_ = hipGetLastError();                                       \
        if (e_ != hipSuccess)                                                    \
            return ::gqaoa::fail(GQAOA_EHIP, "kernel launch failed: %s (%s:%d)",  \
                                 hipGetErrorString(e_), __FILE__, __LINE__);     \
    } while (0)

// Optional event timing of selected launches (see gqaoa_profile_enable).
bool prof_on();
struct ProfScope {
    // records a start event on construction and an end event on end()
    ProfScope(const char *name, hipStream_t st);
    void end();
    const char *name_;
    hipStream_t st_;
    hipEvent_t e0_ = nullptr;
};
void prof_collect();  // after a stream synchronize: fold finished pairs into totals

// Stream-ordered scratch owned by one call: freed (stream-ordered) on every
// return path, after the work enqueued on the stream before the free.
struct AsyncScratch {
    void *ptr = nullptr;
    hipStream_t st;
    explicit AsyncScratch(hipStream_t s) : st(s) {}
    AsyncScratch(const AsyncScratch &) = delete;
    AsyncScratch &operator=(const AsyncScratch &) = delete;
    hipError_t alloc(size_t bytes) { return hipMallocAsync(&ptr, bytes, st); }
    ~AsyncScratch() {
        if (ptr) (void)hipFreeAsync(ptr, st);
    }
};

// Device properties the launch shapes depend on (cached per device).
struct DeviceInfo {
    int device = -1;
    int num_cus = 0;
    size_t lds_per_block = 0;  // largest LDS allocation one block may use
    char arch[64] = {0};
};
int device_info(DeviceInfo *out);

// ---- device-side helpers -----------------------------------------------------
constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Wave sums without LDS traffic, for per-round reductions inside a loop:
// DPP row shifts (an inclusive scan within each row of 16 lanes) and lane
// reads of the row totals, all on the vector and scalar units. The order of
// the additions is fixed. Every lane of the wave must be active (the lane
// reads do not look at EXEC); every lane receives the total.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_value(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum of lanes 0..K-1 of the wave (K a power of two, at most 16).
template <int K>
__device__ __forceinline__ double lanes_sum_dpp(double v) {
    static_assert(K >= 1 && K <= 16 && (K & (K - 1)) == 0, "row-sized power of two");
    if constexpr (K >= 2) v += dpp_move<0x111>(v);  // row_shr:1
    if constexpr (K >= 4) v += dpp_move<0x112>(v);  // row_shr:2
    if constexpr (K >= 8) v += dpp_move<0x114>(v);  // row_shr:4
    if constexpr (K >= 16) v += dpp_move<0x118>(v); // row_shr:8
    return lane_value(v, K - 1);
}

__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_move<0x111>(v);
    v += dpp_move<0x112>(v);
    v += dpp_move<0x114>(v);
    v += dpp_move<0x118>(v);
    return (lane_value(v, 15) + lane_value(v, 31)) + (lane_value(v, 47) + lane_value(v, 63));
}

// Fixed-order reduction of R doubles across a block of kThreads threads.
// Every thread of the block passes its R values (the block converged: the
// wave sums are the DPP ones); thread 0 receives the block sums.
template <int R, int kThreads>
__device__ __forceinline__ void block_sum(double (&v)[R], double *lds /* R*kThreads/64 */) {
    constexpr int kWaves = kThreads / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = wave_sum_dpp(v[r]);
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) lds[wave * R + r] = v[r];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double s = 0.0;
            for (int w = 0; w < kWaves; ++w) s += lds[w * R + r];
            v[r] = s;
        }
    }
}

// PER consecutive cost bytes from p into cpk (byte i of the run in byte i % 4
// of word i / 4): one 16-byte load per 16 bytes when p is aligned.
template <int PER>
__device__ __forceinline__ void load_packed_costs(const uint8_t *__restrict__ p, uint32_t (&cpk)[(PER + 3) / 4]) {
    static_assert(PER == 1 || PER == 2 || PER == 4 || PER == 8 || PER % 16 == 0, "cost run length");
    if constexpr (PER >= 4) {
        if ((reinterpret_cast<uintptr_t>(p) & (PER >= 16 ? 15 : PER - 1)) == 0) {
            if constexpr (PER >= 16) {
#pragma unroll
                for (int u = 0; u < PER / 16; ++u) {
                    const uint4 v = reinterpret_cast<const uint4 *>(p)[u];
                    cpk[4 * u] = v.x;
                    cpk[4 * u + 1] = v.y;
                    cpk[4 * u + 2] = v.z;
                    cpk[4 * u + 3] = v.w;
                }
            } else if constexpr (PER == 8) {
                const uint2 v = *reinterpret_cast<const uint2 *>(p);
                cpk[0] = v.x;
                cpk[1] = v.y;
            } else {
                cpk[0] = *reinterpret_cast<const uint32_t *>(p);
            }
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) cpk[i >> 2] |= (uint32_t)p[i] << (8 * (i & 3));
}


}  // namespace gqaoa
