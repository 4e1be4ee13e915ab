// gwn_alloc.h -- the library's device allocations.  Every one goes through
// these wrappers: they call hipMalloc / hipMallocAsync, except when the
// allocation-failure hook (gwn_test_fail_alloc_after, include/gwn_test.h) makes
// this allocation fail, in which case they return hipErrorOutOfMemory without
// allocating (and set *p to null), so that out-of-memory paths can be exercised
// without exhausting the device.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace gwn {

hipError_t dmalloc(void** p, size_t bytes);
hipError_t dmalloc_async(void** p, size_t bytes, hipStream_t st);

}  // namespace gwn
