/*
 * gwn_prims.h -- device sorting and scanning primitives of the MI355X GWN
 * library, the ones its mesh build uses to cancel interior edges (Sec. 4.1:
 * equal edges meet after a sort by vertex pair), to order triangles along a
 * Morton curve for the BVH, to weld equal positions and to chain boundary
 * loops, and that order dense query batches for the crossing traversal.
 * Exposed for reuse and for testing.
 *
 * All pointers are DEVICE pointers on the current device, owned by the caller;
 * outputs must not alias inputs, inputs are left unchanged.  Each call takes a
 * stream-ordered temporary buffer (hipMallocAsync / hipFreeAsync on `stream`)
 * and is asynchronous on `stream` (NULL = default stream).  n = 0 is a no-op.
 * Errors: GWN_E_INVALID for n outside [0, 2^31), null arrays with n > 0, or a
 * bit range outside 0 <= begin_bit <= end_bit <= key bits; GWN_E_OOM / GWN_E_HIP
 * from the runtime.
 */
#ifndef GWN_PRIMS_H
#define GWN_PRIMS_H

#include <stdint.h>

#include "gwn.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Stable radix sort by bits [begin_bit, end_bit) of the keys (other bits are
 * ignored): keys_out receives the keys and vals_out (when vals_in is not NULL)
 * the payloads in ascending order of those bits; keys with equal bits keep their
 * input order.  Least significant 8-bit digit first, one histogram, scan and
 * scatter per digit.
 */
gwn_status gwn_radix_sort_u32(const uint32_t* keys_in, uint32_t* keys_out, const int32_t* vals_in,
                              int32_t* vals_out, int64_t n, int32_t begin_bit, int32_t end_bit, void* stream);
gwn_status gwn_radix_sort_u64(const uint64_t* keys_in, uint64_t* keys_out, const int32_t* vals_in,
                              int32_t* vals_out, int64_t n, int32_t begin_bit, int32_t end_bit, void* stream);

/* out[i] = in[0] + ... + in[i-1], out[0] = 0 (32-bit two's-complement sums). */
gwn_status gwn_scan_exclusive_sum_i32(const int32_t* in, int32_t* out, int64_t n, void* stream);

/* out[i] = max(in[0], ..., in[i]). */
gwn_status gwn_scan_inclusive_max_i32(const int32_t* in, int32_t* out, int64_t n, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GWN_PRIMS_H */
