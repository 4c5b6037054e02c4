// Exclusive prefix sum on the device (setup work: element offsets, list
// offsets).  Three steps: every workgroup scans its 2048 items and writes
// its total; the totals are scanned the same way (recursively); the scanned
// totals are added back.  Deterministic (fixed order).
#pragma once

#include "common.h"

namespace xrl {

constexpr int kScanThreads = 256, kScanItems = 8;

template <typename TI, typename TO>
__global__ __launch_bounds__(kScanThreads) void k_scan_local(const TI *__restrict__ in, int64_t n,
                                                             TO *__restrict__ out, TO *__restrict__ block_total)
{
    __shared__ TO part[kScanThreads];
    const int64_t base = ((int64_t)blockIdx.x * kScanThreads + threadIdx.x) * kScanItems;
    TO v[kScanItems];
    TO own = 0;
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < n ? (TO)in[base + i] : TO(0);
        own += v[i];
    }
    part[threadIdx.x] = own;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const TO add = threadIdx.x >= off ? part[threadIdx.x - off] : TO(0);
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    TO run = part[threadIdx.x] - own;
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == kScanThreads - 1) block_total[blockIdx.x] = part[kScanThreads - 1];
}

template <typename TO>
__global__ void k_scan_add(TO *__restrict__ out, int64_t n, const TO *__restrict__ block_off)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] += block_off[i / ((int64_t)kScanThreads * kScanItems)];
}

// out[i] = in[0] + ... + in[i-1]; *total (device) = the sum of all n.
template <typename TI, typename TO>
void exclusive_scan(const TI *in, int64_t n, TO *out, TO *total, hipStream_t s)
{
    if (n <= 0) {
        XRL_HIP(hipMemsetAsync(total, 0, sizeof(TO), s));
        return;
    }
    const int64_t per = (int64_t)kScanThreads * kScanItems;
    const int64_t nb = cdiv(n, per);
    DevBuf<TO> bt(nb);
    k_scan_local<TI, TO><<<(unsigned)nb, kScanThreads, 0, s>>>(in, n, out, bt.p);
    XRL_HIP(hipGetLastError());
    if (nb == 1) {
        XRL_HIP(hipMemcpyAsync(total, bt.p, sizeof(TO), hipMemcpyDeviceToDevice, s));
        return;
    }
    DevBuf<TO> bo(nb);
    exclusive_scan<TO, TO>(bt.p, nb, bo.p, total, s);
    k_scan_add<TO><<<(unsigned)cdiv(n, 256), 256, 0, s>>>(out, n, bo.p);
    XRL_HIP(hipGetLastError());
}

}  // namespace xrl
