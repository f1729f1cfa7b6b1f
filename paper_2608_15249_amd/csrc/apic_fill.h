// Staging of global data in LDS with the loads of a round issued together,
// shared by the fused field solves and the field update of the
// electromagnetic step.
#pragma once

#include "apic_device.h"

namespace apic {
namespace {

// Fills count entries (count > 0) from global memory, U per thread per
// round: the U loads of a round are issued before the first is waited for.
// load(t) reads entry t < count (the index is clamped into the range); put(t,
// v) stores entry t, and for t >= count must store v somewhere harmless
// (unconditional stores keep the loads ahead of the first wait).
template <typename T, int U, typename Load, typename Put>
__device__ __forceinline__ void fill_batched(int count, Load load, Put put) {
    for (int t0 = 0; t0 < count; t0 += U * kBlock) {
        T v[U];
#pragma unroll
        for (int r = 0; r < U; ++r) v[r] = load(min(t0 + r * kBlock + (int)threadIdx.x, count - 1));
#pragma unroll
        for (int r = 0; r < U; ++r) put(t0 + r * kBlock + (int)threadIdx.x, v[r]);
    }
}

}  // namespace
}  // namespace apic
