// Stable LSD radix sort of (64-bit key, 32-bit value) pairs (radix.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace gwn {

// Device bytes of the sort's temporary storage for n pairs.
size_t radix_temp_bytes(int64_t n);

// Sort n pairs on key bits [lo_bit, hi_bit), 8 bits per pass, stable.  The
// input is keys[0] / vals[0]; passes alternate between the two buffers of
// each pair, and `sel` returns the buffer (0 or 1) that holds the sorted
// pairs.  temp: radix_temp_bytes(n) bytes; all work is queued on `stream`.
hipError_t radix_sort_pairs(uint64_t *keys[2], int32_t *vals[2], int64_t n, int lo_bit, int hi_bit, void *temp,
                            hipStream_t stream, int &sel);

}  // namespace gwn
