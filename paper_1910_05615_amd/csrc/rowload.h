// Helpers of the kernels that read one row of X per thread.
#pragma once

#include <hip/hip_runtime.h>

namespace rtd {

// X as a global-memory pointer: rows reached through the item table would
// otherwise be read with flat loads (the compiler cannot tell the address
// space of a pointer loaded from memory).
template <typename T>
using gptr_t = const T __attribute__((address_space(1)))*;
template <typename T>
__device__ inline gptr_t<T> as_global(const T* p) {
  return (gptr_t<T>)p;
}

// Every element of the row in a register at this point: all of the row's
// loads are in flight together.  Without it the compiler issues the later
// columns' loads after the first columns' arithmetic (they are not needed
// before), and a wave waits for memory several times (1M x 20 scoring: 20.0
// against 17.7 us).  The empty statements emit no instructions.
template <typename T, int P>
__device__ inline void all_loaded(T (&v)[P]) {
#pragma unroll
  for (int j = 0; j < P; ++j) asm volatile("" : "+v"(v[j]));
}

}  // namespace rtd
