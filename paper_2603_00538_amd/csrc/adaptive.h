// Limits of per-element sample counts, shared by their allocation, the
// emission of their points and their consumption, and the check of one
// element's range.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ft {

// largest sample count of one element (Philox counter word 0 is the sample index)
constexpr int64_t kMaxElemSamples = int64_t(1) << 20;
// largest total of an allocation's samples
constexpr int64_t kMaxAllocTotal = int64_t(1) << 40;

// Element t's samples from the allocation offsets: [o0, o1) of the sample block,
// valid when 1 <= o1 - o0 <= kMaxElemSamples and both lie in [0, total].
__device__ __forceinline__ bool element_range(const int64_t* __restrict__ offs, uint32_t t, int64_t total,
                                              int64_t& o0, uint32_t& N) {
    o0 = offs[t];
    const int64_t o1 = offs[t + 1];
    const bool ok = o0 >= 0 && o1 > o0 && o1 <= total && o1 - o0 <= kMaxElemSamples;
    N = ok ? uint32_t(o1 - o0) : 0u;
    return ok;
}

}  // namespace ft
