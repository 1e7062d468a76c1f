// Device helpers shared by the kernel sources.
#pragma once

#include <hip/hip_runtime.h>

namespace dg {

// Store into mapped host memory that the host reads once the kernel's event
// has completed: a system-scope store, then a system-scope release so the
// value is visible at system scope before anything the kernel does later.
template <typename T>
__device__ __forceinline__ void st_host(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
}

}  // namespace dg
