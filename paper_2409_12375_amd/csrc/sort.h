// Stable least-significant-digit radix sort of (64-bit key, 32-bit value)
// pairs on the device, 8-bit digits (the tree's Morton codes).
//
// Per pass over one digit:
//   1. every workgroup counts the digits of its tile of 2048 keys in LDS and
//      writes its 256 counts digit-major (count[d][tile]);
//   2. an exclusive prefix sum over that array gives each (digit, tile) its
//      first output position (all smaller digits, then earlier tiles);
//   3. every workgroup ranks its keys stably and scatters them.  A tile is
//      read slot by slot (slot i holds keys 256 i .. 256 i + 255 of the
//      tile, one per thread); within a wave the keys of one digit are
//      ranked by matching the 8 digit bits with ballots, across the waves of
//      a slot by per-wave counts in LDS, across slots by a running count per
//      digit, so equal digits keep their input order.
// The kernels have internal linkage: every source that sorts includes this
// header.
#pragma once

#include "scan.h"

namespace xrl {

constexpr int kSortThreads = 256, kSortSlots = 8, kSortTile = kSortThreads * kSortSlots, kSortWaves = 4;

static __global__ __launch_bounds__(kSortThreads) void k_digit_count(const uint64_t *__restrict__ key, int64_t n, int shift,
                                                              int64_t ntile, int32_t *__restrict__ count)
{
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int i = 0; i < kSortSlots; ++i) {
        const int64_t j = base + i * kSortThreads + threadIdx.x;
        if (j < n) atomicAdd(&h[(key[j] >> shift) & 255], 1);
    }
    __syncthreads();
    count[(int64_t)threadIdx.x * ntile + blockIdx.x] = h[threadIdx.x];
}

static __global__ __launch_bounds__(kSortThreads) void k_digit_scatter(const uint64_t *__restrict__ key,
                                                                const int32_t *__restrict__ val, int64_t n, int shift,
                                                                int64_t ntile, const int64_t *__restrict__ first,
                                                                uint64_t *__restrict__ key_out,
                                                                int32_t *__restrict__ val_out)
{
    __shared__ int64_t pos[256];              // next output position of each digit
    __shared__ int32_t wcnt[kSortWaves][256];  // keys of each digit per wave in this slot
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    pos[t] = first[(int64_t)t * ntile + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const uint64_t below = (1ull << lane) - 1;
    for (int i = 0; i < kSortSlots; ++i) {
        for (int w = 0; w < kSortWaves; ++w) wcnt[w][t] = 0;
        __syncthreads();
        const int64_t j = base + i * kSortThreads + t;
        const bool valid = j < n;
        const uint64_t k = valid ? key[j] : 0;
        const int d = (int)((k >> shift) & 255);
        uint64_t same = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const uint64_t ones = __ballot(valid && ((d >> b) & 1));
            same &= ((d >> b) & 1) ? ones : ~ones;
        }
        const int rank = __popcll(same & below);
        if (valid && rank == 0) wcnt[wave][d] = __popcll(same);
        __syncthreads();
        if (valid) {
            int64_t at = pos[d] + rank;
            for (int w = 0; w < wave; ++w) at += wcnt[w][d];
            key_out[at] = k;
            val_out[at] = val[j];
        }
        __syncthreads();
        pos[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
        // the next slot's counts are cleared only after every thread has
        // read this slot's (the barrier at the top of the next slot)
        __syncthreads();
    }
}

// Sort (key, val) pairs by the low `bits` bits of the key.  key/val are the
// input and hold the sorted result on return; key_tmp/val_tmp are scratch of
// the same length.
inline void radix_sort_pairs(uint64_t *key, int32_t *val, uint64_t *key_tmp, int32_t *val_tmp, int64_t n, int bits,
                             hipStream_t s)
{
    if (n <= 1) return;
    const int64_t ntile = cdiv(n, kSortTile);
    DevBuf<int32_t> count(256 * ntile);
    DevBuf<int64_t> first(256 * ntile), total(1);
    uint64_t *ki = key, *ko = key_tmp;
    int32_t *vi = val, *vo = val_tmp;
    const int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        k_digit_count<<<(unsigned)ntile, kSortThreads, 0, s>>>(ki, n, 8 * p, ntile, count.p);
        XRL_HIP(hipGetLastError());
        exclusive_scan<int32_t, int64_t>(count.p, 256 * ntile, first.p, total.p, s);
        k_digit_scatter<<<(unsigned)ntile, kSortThreads, 0, s>>>(ki, vi, n, 8 * p, ntile, first.p, ko, vo);
        XRL_HIP(hipGetLastError());
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
    if (ki != key) {
        XRL_HIP(hipMemcpyAsync(key, ki, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        XRL_HIP(hipMemcpyAsync(val, vi, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
}

}  // namespace xrl
