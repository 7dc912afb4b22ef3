// Batched vector copies for the solvers (see vec.hpp).
#include "vec.hpp"

#include <algorithm>
#include <stdexcept>
#include <string>

namespace scc {

constexpr int COPY_MAX = 64;  // items per launch (kernel-argument list)

struct CopyList {
  const double* src[COPY_MAX];
  double* dst[COPY_MAX];
  int64_t n[COPY_MAX];
};

// blockIdx.y selects the item; the x blocks stride over its elements
__global__ __launch_bounds__(256) void copy_list_kernel(CopyList L) {
  const int i = blockIdx.y;
  const double* s = L.src[i];
  double* d = L.dst[i];
  const int64_t n = L.n[i];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (s) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) d[e] = s[e];
  } else {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) d[e] = 0.0;
  }
}

void launch_copy_list(const std::vector<CopyItem>& items, hipStream_t s) {
  for (size_t b = 0; b < items.size(); b += COPY_MAX) {
    const int cnt = (int)std::min<size_t>(COPY_MAX, items.size() - b);
    CopyList L{};
    int64_t nmax = 0;
    int used = 0;
    for (int i = 0; i < cnt; ++i) {
      const CopyItem& it = items[b + i];
      if (it.n <= 0) continue;
      if (!it.dst) throw std::runtime_error("copy list: null destination");
      L.src[used] = it.src;
      L.dst[used] = it.dst;
      L.n[used] = it.n;
      nmax = std::max(nmax, it.n);
      ++used;
    }
    if (!used) continue;
    // about 4096 blocks in all, at most one element per thread of the longest item
    const int64_t per = std::max<int64_t>(1, std::min<int64_t>((nmax + 255) / 256, 4096 / used));
    hipLaunchKernelGGL(copy_list_kernel, dim3((unsigned)per, (unsigned)used), dim3(256), 0, s, L);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw std::runtime_error(std::string("copy list launch: ") + hipGetErrorString(e));
  }
}

}  // namespace scc
