/*
 * gwn_test.h -- test hooks of the MI355X GWN library (not needed in normal use).
 *
 * gwn_test_fail_alloc_after(n): the library's device allocations (hipMalloc /
 * hipMallocAsync, made by any call of include/gwn.h or include/gwn_prims.h)
 * succeed n more times, then every further one fails with out-of-memory --
 * without touching the device -- until the hook is reset; n < 0 resets it (the
 * default: no failures).  The failing call returns GWN_E_OOM with a message in
 * gwn_last_error() and releases whatever it had allocated.  Process-wide, for
 * all devices and threads.  Returns the number of allocations made since the
 * previous call (host-side count), so a test can find out how many a call makes.
 */
#ifndef GWN_TEST_H
#define GWN_TEST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int64_t gwn_test_fail_alloc_after(int64_t n);

#ifdef __cplusplus
}
#endif

#endif /* GWN_TEST_H */
