// Batched vector copies for the solvers: one launch moves a list of device
// vectors (dst = src, or dst = 0 where src is null) instead of one copy
// kernel per vector.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace scc {

struct CopyItem {
  double* dst;
  const double* src;  // nullptr: fill dst with zeros
  int64_t n;
};

// Stream-ordered on s; the list is read before the call returns.  Items may
// not overlap one another.
void launch_copy_list(const std::vector<CopyItem>& items, hipStream_t s);

}  // namespace scc
