// Launch structures shared by the 2D and 3D query kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "gwn_internal.h"

namespace gwn {

// A pair of events around a launch of one of the timed kernels, on its
// stream, while recording is on (query.hip).
void prof_begin(hipStream_t s, hipEvent_t &a);
void prof_end(hipStream_t s, hipEvent_t a, int kernel);

constexpr int kMaxSeg = 32;
constexpr int kMaxModels = 8;
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kMaxBisectIter = 16384;

struct LaunchTable {
    int32_t n_seg;
    int32_t n_waves;
    int32_t qpw;        // queries per wave (64; 8..64 for small launches)
    int32_t pad;
    int32_t seg_model[kMaxSeg];
    int32_t woff[kMaxSeg + 1];
    int64_t qoff[kMaxSeg + 1];
    DevModel models[kMaxModels];
};

struct Ctr {
    long long v[GWN_NCOUNTERS];
};

// Near-field leaves recorded per query by the 3D traversal (at most
// kNearSlots; more sets the overflow count and gives NaN).
constexpr int kNearSlots = 64;

// Byte sizes of the 3D near-field pass's per-query records (one slot per
// query position of the wave grid, n_waves x queries per wave), each part
// 256-byte aligned: the far-field and node-set sum, the near-leaf count,
// kNearSlots leaf indices, the reclassify flag.
struct NearBytes {
    size_t part = 0, cnt = 0, list = 0, need = 0, total = 0;
};

inline NearBytes near_scratch_bytes(int64_t slots)
{
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t ns = (size_t)slots;
    NearBytes b;
    b.part = al(ns * sizeof(double));
    b.cnt = al(ns * sizeof(int32_t));
    b.list = al(ns * kNearSlots * sizeof(int32_t));
    b.need = al(ns);
    b.total = b.part + b.cnt + b.list + b.need;
    return b;
}

__device__ __forceinline__ int uniform_i(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Workgroup -> sorted-query range.  The dispatcher deals workgroups to the 8
// XCDs round robin (block b runs on XCD b % 8), so with the identity map an
// XCD's L2 serves waves from the whole range.  Handing each XCD runs of C
// consecutive blocks, the runs themselves dealt round robin, keeps C
// neighbouring regions' tree nodes in one L2 while the XCDs still share out
// cheap and expensive regions evenly (one contiguous eighth per XCD was far
// slower: the cost per wave varies strongly across a scene).  Blocks past
// the last whole round of 8 C keep their own index.  A bijection on
// [0, gridDim.x); values do not depend on it.
template <int C>
__device__ __forceinline__ int xcd_block()
{
    const int nb = gridDim.x, b = blockIdx.x;
    const int full = nb / (8 * C) * (8 * C);
    if (b >= full) return b;
    const int x = b % 8, i = b / 8;
    return ((i / C) * 8 + x) * C + i % C;
}

struct StackLDS {
    int node[kWavesPerBlock][kStackDepth];
    unsigned long long mask[kWavesPerBlock][kStackDepth];
};

template <bool COUNT>
__device__ __forceinline__ void flush_counters(Ctr &ctr, long long *counters)
{
    if (!COUNT) return;
#pragma unroll
    for (int k = 0; k < GWN_NCOUNTERS; ++k) {
        long long v = ctr.v[k];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane_id() == 0 && v) atomicAdd((unsigned long long *)&counters[k], (unsigned long long)v);
    }
}

}  // namespace gwn
