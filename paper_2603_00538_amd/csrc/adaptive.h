// Limits of per-element sample counts, shared by their allocation, the
// emission of their points and their consumption.
#pragma once

#include <cstdint>

namespace ft {

// largest sample count of one element (Philox counter word 0 is the sample index)
constexpr int64_t kMaxElemSamples = int64_t(1) << 20;
// largest total of an allocation's samples
constexpr int64_t kMaxAllocTotal = int64_t(1) << 40;

}  // namespace ft
