// gwn_sort.h -- device sorting and scanning primitives of the library: a
// stable least-significant-digit radix sort of 32- or 64-bit keys with an
// optional int payload, and prefix scans (sum, max) of int arrays.  Used by the
// mesh build (welding, Morton order, boundary edges, loop offsets) and by the
// Morton order of dense query batches.
//
// All calls are asynchronous on `st` and work in a caller-provided temporary
// buffer of at least the *_temp_bytes() size (device memory, any contents,
// 256-byte aligned).  Inputs are not modified; outputs must not alias inputs.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gwn {

// Bytes of temporary storage for a sort of n keys of key_bytes (4 or 8) bytes,
// with or without an int payload.
size_t sort_temp_bytes(int64_t n, int key_bytes, bool with_values);

// Bytes of temporary storage for a scan of n ints.
size_t scan_temp_bytes(int64_t n);

// Stable sort by bits [begin_bit, end_bit) of the keys (other bits ignored):
// kout receives the keys, vout (when vin is given) the payloads, in ascending
// order of those bits; equal keys keep their input order.  0 <= n < 2^31.
hipError_t radix_sort_u32(const uint32_t* kin, uint32_t* kout, const int* vin, int* vout, int64_t n, int begin_bit,
                          int end_bit, void* temp, hipStream_t st);
hipError_t radix_sort_u64(const uint64_t* kin, uint64_t* kout, const int* vin, int* vout, int64_t n, int begin_bit,
                          int end_bit, void* temp, hipStream_t st);

// out[i] = in[0] + ... + in[i - 1] (exclusive; out[0] = 0).
hipError_t scan_exclusive_sum(const int* in, int* out, int64_t n, void* temp, hipStream_t st);

// out[i] = max(in[0], ..., in[i]) (inclusive).
hipError_t scan_inclusive_max(const int* in, int* out, int64_t n, void* temp, hipStream_t st);

}  // namespace gwn
