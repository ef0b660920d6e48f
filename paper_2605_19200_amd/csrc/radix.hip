// Stable LSD radix sort of (64-bit key, 32-bit value) pairs: the space-
// filling-curve sort of the queries before a launch, and the Morton sort of
// the LBVH build.
//
// Each pass sorts on one 8-bit digit, in three kernels over tiles of
// kRadixTile keys (256 threads x 8 keys, the keys of a thread kRadixBlock
// apart so every load is coalesced):
//   k_radix_hist     per-tile digit counts (LDS atomics), stored digit-major
//                    (hist[d * tiles + t]);
//   k_radix_scan     one workgroup per digit turns its row of hist into
//                    exclusive offsets within the digit (keys with digit d
//                    in earlier tiles) and stores the row total;
//   k_radix_scatter  each tile again, 256 keys at a time in input order: a
//                    key's rank among the equal digits of its wave comes
//                    from eight ballots (one per digit bit), the waves
//                    before it add their counts, and the tile's running
//                    offset per digit advances after every 256 keys, so
//                    equal digits keep their input order.  A tile's start
//                    for digit d is the number of keys with a smaller digit
//                    (the scan of the 256 row totals, done in LDS by each
//                    tile) plus its offset within the digit.
// Passes alternate between the two buffers of each pair; nothing needs to
// start at zero (hist is written whole by each pass), so the sort can run
// in a captured graph.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "radix.h"

namespace gwn {

namespace {

constexpr int kRadixBlock = 256;
constexpr int kRadixItems = 8;
constexpr int kRadixTile = kRadixBlock * kRadixItems;
constexpr int kRadixDigits = 256;
constexpr int kRadixWaves = kRadixBlock / 64;

__global__ __launch_bounds__(kRadixBlock) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                            uint32_t *__restrict__ hist, int tiles)
{
    __shared__ uint32_t h[kRadixDigits];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll 4
    for (int i = 0; i < kRadixItems; ++i) {
        const int64_t idx = base + (int64_t)i * kRadixBlock + t;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & (kRadixDigits - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)t * tiles + blockIdx.x] = h[t];
}

// Exclusive scan, in place, of the row hist[d * tiles .. (d + 1) * tiles)
// of digit d = blockIdx.x, in steps of 4 counts per thread; the row's total
// goes to total[d].
__global__ __launch_bounds__(kRadixBlock) void k_radix_scan(uint32_t *__restrict__ hist, int tiles,
                                                            uint32_t *__restrict__ total)
{
    __shared__ uint32_t part[kRadixBlock];
    const int t = threadIdx.x;
    uint32_t *__restrict__ row = hist + (int64_t)blockIdx.x * tiles;
    uint32_t carry = 0;
    for (int base = 0; base < tiles; base += 4 * kRadixBlock) {
        uint32_t v[4];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = base + 4 * t + k;
            v[k] = i < tiles ? row[i] : 0u;
            s += v[k];
        }
        part[t] = s;
        __syncthreads();
        for (int off = 1; off < kRadixBlock; off <<= 1) {
            const uint32_t x = t >= off ? part[t - off] : 0u;
            __syncthreads();
            part[t] += x;
            __syncthreads();
        }
        uint32_t run = carry + (t ? part[t - 1] : 0u);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = base + 4 * t + k;
            if (i < tiles) row[i] = run;
            run += v[k];
        }
        carry += part[kRadixBlock - 1];
        __syncthreads();
    }
    if (t == 0) total[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kRadixBlock) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                               const int32_t *__restrict__ vin,
                                                               uint64_t *__restrict__ kout, int32_t *__restrict__ vout,
                                                               int64_t n, int shift, const uint32_t *__restrict__ hist,
                                                               const uint32_t *__restrict__ total, int tiles)
{
    __shared__ uint32_t next[kRadixDigits];                 // next output position per digit
    __shared__ uint32_t wcount[kRadixWaves][kRadixDigits];  // per-wave digit counts of a 256-key step
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const uint64_t below = (1ull << lane) - 1ull;           // lanes before this one
    // start of digit t: keys with a smaller digit (exclusive scan of the
    // row totals), then this tile's offset within the digit
    next[t] = total[t];
    __syncthreads();
    for (int off = 1; off < kRadixDigits; off <<= 1) {
        const uint32_t x = t >= off ? next[t - off] : 0u;
        __syncthreads();
        next[t] += x;
        __syncthreads();
    }
    const uint32_t start = (t ? next[t - 1] : 0u) + hist[(int64_t)t * tiles + blockIdx.x];
    __syncthreads();
    next[t] = start;
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    for (int i = 0; i < kRadixItems; ++i) {
#pragma unroll
        for (int k = 0; k < kRadixWaves; ++k) wcount[k][t] = 0;
        __syncthreads();
        const int64_t idx = base + (int64_t)i * kRadixBlock + t;
        const bool valid = idx < n;
        uint64_t key = 0;
        int32_t val = 0;
        int d = 0;
        if (valid) {
            key = kin[idx];
            val = vin[idx];
            d = (int)((key >> shift) & (kRadixDigits - 1));
        }
        // lanes of this wave with the same digit
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1;
            const uint64_t bal = __ballot(valid && on);
            same &= on ? bal : ~bal;
        }
        const int rank = __popcll(same & below);
        if (valid && rank == 0) wcount[w][d] = (uint32_t)__popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t pos = next[d] + (uint32_t)rank;
            for (int k = 0; k < w; ++k) pos += wcount[k][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int k = 0; k < kRadixWaves; ++k) add += wcount[k][t];
        next[t] += add;
    }
}

int radix_tiles(int64_t n) { return (int)((n + kRadixTile - 1) / kRadixTile); }

}  // namespace

size_t radix_temp_bytes(int64_t n)
{
    return (size_t)kRadixDigits * ((size_t)(n > 0 ? radix_tiles(n) : 1) + 1) * sizeof(uint32_t);
}

hipError_t radix_sort_pairs(uint64_t *keys[2], int32_t *vals[2], int64_t n, int lo_bit, int hi_bit, void *temp,
                            hipStream_t stream, int &sel)
{
    sel = 0;
    if (n <= 1) return hipSuccess;
    const int tiles = radix_tiles(n);
    uint32_t *hist = (uint32_t *)temp;
    uint32_t *total = hist + (size_t)kRadixDigits * tiles;
    for (int shift = lo_bit; shift < hi_bit; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3(tiles), dim3(kRadixBlock), 0, stream, (const uint64_t *)keys[sel], n,
                           shift, hist, tiles);
        hipLaunchKernelGGL(k_radix_scan, dim3(kRadixDigits), dim3(kRadixBlock), 0, stream, hist, tiles, total);
        hipLaunchKernelGGL(k_radix_scatter, dim3(tiles), dim3(kRadixBlock), 0, stream, (const uint64_t *)keys[sel],
                           (const int32_t *)vals[sel], keys[sel ^ 1], vals[sel ^ 1], n, shift, (const uint32_t *)hist,
                           (const uint32_t *)total, tiles);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        sel ^= 1;
    }
    return hipSuccess;
}

}  // namespace gwn
