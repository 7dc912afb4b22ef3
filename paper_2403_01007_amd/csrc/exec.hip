// HIP kernels for gfx950 and the executor of contraction programs.
//
// * gemm_f64: FP64 matrix-core (v_mfma_f64_16x16x4_f64) GEMM over strided
//   operands.  A 64x64 output tile per 256-thread workgroup (4 wave64s, each
//   32x32 = 2x2 MFMA tiles), K staged through LDS in slabs of 32 (16 for
//   short K) with the next slab's global loads in flight during the MFMAs.
//   Global loads are mapped so that consecutive lanes walk the operand's
//   unit-stride dimension.
// * perm: strided N-d gather/scatter with up to four weighted inputs; used
//   for operand packing, output permutation, linear combinations, block
//   slices and embeddings.
// * dot: two-pass deterministic reduction (no floating-point atomics).
#include <algorithm>
#include <cstdio>
#include <stdexcept>
#include <type_traits>

#include "exec.hpp"

namespace scc {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, GEMM_THREADS = 256;

// n / d for n, d < 2^31 as (umulhi(n, m) + n) >> s with s = ceil(log2 d)
// and m = floor(2^32 (2^s - d) / d) + 1
__device__ __forceinline__ uint32_t fast_div(uint32_t n, uint32_t m, uint32_t s) {
  return (__umulhi(n, m) + n) >> s;
}

// element offset of index x of a fused group (one or two runs)
__device__ __forceinline__ int64_t imap(int64_t x, const IdxMap& m, int64_t si) {
  if (m.D == 0) return x * si;
  const int64_t q = (int64_t)fast_div((uint32_t)x, m.mag, m.sh);
  return q * (int64_t)m.so + (x - q * (int64_t)m.D) * si;
}

// the same in 32 bits, for tensors of fewer than 2^31 elements and every
// group given as two runs (a single run as D = 2^31)
__device__ __forceinline__ uint32_t imap32(uint32_t x, const IdxMap& m, int64_t si) {
  const uint32_t q = fast_div(x, m.mag, m.sh);
  return q * m.so + (x - q * m.D) * (uint32_t)si;
}

constexpr int GEMM_BK = 16;  // slab depth of the matrix-core kernels

// Operand tiles are loaded from global memory into registers one K-slab
// ahead: the loads of slab s+1 are in flight while the matrix cores work on
// slab s from LDS.  TF32 selects FP32 products (operands rounded to FP32 on
// the way into LDS, FP32 accumulation) instead of FP64.

template <int BKT, bool F32, bool TWO>
__device__ __forceinline__ void gemm_body(const GemmArgs& a,
                                          typename std::conditional<F32, float, double>::type (*As)[BM + 1],
                                          typename std::conditional<F32, float, double>::type (*Bs)[BN + 1]) {
  typedef typename std::conditional<F32, float, double>::type T;
  typedef T v4 __attribute__((ext_vector_type(4)));
  const int64_t split = a.splits > 1 ? blockIdx.z : 0;
  const int64_t bz = a.splits > 1 ? 0 : blockIdx.z;
  const int64_t m0 = (int64_t)blockIdx.y * BM;
  const int64_t n0 = (int64_t)blockIdx.x * BN;
  const double* A = a.A + bz * a.sAb;
  const double* B = a.B + bz * a.sBb;
  const int64_t kbeg = a.splits > 1 ? split * a.kchunk : 0;
  const int64_t kend = a.splits > 1 ? min(a.K, kbeg + a.kchunk) : a.K;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 32;
  const int wn = (wave & 1) * 32;
  const bool a_kfast = (a.sAk == 1);
  const bool b_nfast = (a.sBn == 1) || (a.sBk != 1);
  constexpr int EA = BM * BKT / GEMM_THREADS, EB = BN * BKT / GEMM_THREADS;
  double ra[EA], rb[EB];
  // element e of this thread: (row, k) of the A slab and (k, col) of the B
  // slab, consecutive threads along each operand's unit-stride index
  auto a_pos = [&](int e, int& mm, int& kk) {
    const int idx = tid + e * GEMM_THREADS;
    if (a_kfast) {
      kk = idx % BKT;
      mm = idx / BKT;
    } else {
      mm = idx % BM;
      kk = idx / BM;
    }
  };
  auto b_pos = [&](int e, int& nn, int& kk) {
    const int idx = tid + e * GEMM_THREADS;
    if (b_nfast) {
      nn = idx % BN;
      kk = idx / BN;
    } else {
      kk = idx % BKT;
      nn = idx / BKT;
    }
  };
  // two-run groups: 32-bit offsets; the row / column offset of each loaded
  // element is fixed across K slabs
  uint32_t aoff[TWO ? EA : 1], boff[TWO ? EB : 1];
  if constexpr (TWO) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int mm, kk;
      a_pos(e, mm, kk);
      const int64_t gm = m0 + mm;
      aoff[e] = gm < a.M ? imap32((uint32_t)gm, a.mAm, a.sAm) : 0u;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int nn, kk;
      b_pos(e, nn, kk);
      const int64_t gn = n0 + nn;
      boff[e] = gn < a.N ? imap32((uint32_t)gn, a.mBn, a.sBn) : 0u;
    }
  }
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int mm, kk;
      a_pos(e, mm, kk);
      const int64_t gm = m0 + mm, gk = k0 + kk;
      if constexpr (TWO)
        ra[e] = (gm < a.M && gk < kend) ? A[aoff[e] + imap32((uint32_t)gk, a.mAk, a.sAk)] : 0.0;
      else
        ra[e] = (gm < a.M && gk < kend) ? A[gm * a.sAm + gk * a.sAk] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int nn, kk;
      b_pos(e, nn, kk);
      const int64_t gn = n0 + nn, gk = k0 + kk;
      if constexpr (TWO)
        rb[e] = (gn < a.N && gk < kend) ? B[boff[e] + imap32((uint32_t)gk, a.mBk, a.sBk)] : 0.0;
      else
        rb[e] = (gn < a.N && gk < kend) ? B[gk * a.sBk + gn * a.sBn] : 0.0;
    }
  };
  v4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = v4{0, 0, 0, 0};
  if (kbeg < kend) load(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += BKT) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int mm, kk;
      a_pos(e, mm, kk);
      As[kk][mm] = (T)ra[e];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int nn, kk;
      b_pos(e, nn, kk);
      Bs[kk][nn] = (T)rb[e];
    }
    __syncthreads();
    if (k0 + BKT < kend) load(k0 + BKT);
#pragma unroll
    for (int kk = 0; kk < BKT; kk += 4) {
      const int kr = kk + (lane >> 4);
      T af[2], bf[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        af[t] = As[kr][wm + t * 16 + (lane & 15)];
        bf[t] = Bs[kr][wn + t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if constexpr (F32)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
          else
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  const bool part = a.splits > 1;
  double* out = part ? a.P + split * a.M * a.N : a.C + bz * a.sCb;
  const double* Cin = (part || !a.Cin) ? nullptr : a.Cin + bz * a.sCb;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // output layout: v_mfma_f64_16x16x4_f64 puts D[4 r + l / 16][l % 16]
        // in lane l, register r; v_mfma_f32_16x16x4_f32 puts D[4 (l / 16) + r][l % 16]
        const int rr = F32 ? (lane >> 4) * 4 + r : r * 4 + (lane >> 4);
        const int64_t row = m0 + wm + i * 16 + rr;
        const int64_t col = n0 + wn + j * 16 + (lane & 15);
        if (row < a.M && col < a.N) {
          double v = a.alpha * (double)acc[i][j][r];
          const int64_t o = part ? row * a.N + col
                            : TWO ? (int64_t)(imap32((uint32_t)row, a.mCm, a.sCm) + imap32((uint32_t)col, a.mCn, a.sCn))
                                  : row * a.sCm + col * a.sCn;
          if (Cin) v += a.beta * Cin[o];
          out[o] = v;
        }
      }
}

// FP64 matrix-core GEMM (the contraction kernel of every device program):
// every operand index group (rows, columns, summed index) is one run of
// dimensions with one stride.  Slabs of 16 and at most 128 registers per
// lane give four waves per SIMD (measured faster than 32-deep slabs at two
// or three waves: the other waves' matrix work covers each wave's loads,
// LDS staging and barriers).
__global__ __launch_bounds__(GEMM_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void gemm_f64_kernel(
    GemmArgs a) {
  __shared__ double As[GEMM_BK][BM + 1];
  __shared__ double Bs[GEMM_BK][BN + 1];
  gemm_body<GEMM_BK, false, false>(a, As, Bs);
}

// The same where some group spans two runs (read in place instead of
// packing the operand, or writing a temporary, in the group's order)
__global__ __launch_bounds__(GEMM_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void gemm_f64_two_kernel(
    GemmArgs a) {
  __shared__ double As[GEMM_BK][BM + 1];
  __shared__ double Bs[GEMM_BK][BN + 1];
  gemm_body<GEMM_BK, false, true>(a, As, Bs);
}

// Reduced-precision variants: FP64 operands are rounded to FP32 as they are
// staged into LDS, multiplied on the FP32 matrix cores
// (v_mfma_f32_16x16x4_f32) with FP32 accumulation, and the result is written
// back in FP64.  Same tiling and operand mapping as the FP64 kernels.
__global__ __launch_bounds__(GEMM_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void gemm_f32acc_kernel(
    GemmArgs a) {
  __shared__ float As[GEMM_BK][BM + 1];
  __shared__ float Bs[GEMM_BK][BN + 1];
  gemm_body<GEMM_BK, true, false>(a, As, Bs);
}

__global__ __launch_bounds__(GEMM_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void gemm_f32acc_two_kernel(
    GemmArgs a) {
  __shared__ float As[GEMM_BK][BM + 1];
  __shared__ float Bs[GEMM_BK][BN + 1];
  gemm_body<GEMM_BK, true, true>(a, As, Bs);
}

// Multi-segment GEMM: the products of every segment accumulate in the same
// registers (one pass over the output), each segment staged through LDS with
// its own operand layout and its coefficient applied on the way in.
template <int BKT, bool F32>
__device__ __forceinline__ void gemm_multi_body(const GemmMulti& G,
                                                typename std::conditional<F32, float, double>::type (*As)[BM + 1],
                                                typename std::conditional<F32, float, double>::type (*Bs)[BN + 1]) {
  typedef typename std::conditional<F32, float, double>::type T;
  typedef T v4 __attribute__((ext_vector_type(4)));
  const GemmArgs& a = G.g;
  const int64_t split = a.splits > 1 ? blockIdx.z : 0;
  const int64_t bz = a.splits > 1 ? 0 : blockIdx.z;
  const int64_t m0 = (int64_t)blockIdx.y * BM;
  const int64_t n0 = (int64_t)blockIdx.x * BN;
  const int64_t kbeg = a.splits > 1 ? split * a.kchunk : 0;
  const int64_t kend = a.splits > 1 ? min(a.K, kbeg + a.kchunk) : a.K;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 32;
  const int wn = (wave & 1) * 32;
  constexpr int EA = BM * BKT / GEMM_THREADS, EB = BN * BKT / GEMM_THREADS;
  v4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = v4{0, 0, 0, 0};
  for (int sg = 0; sg < G.nseg; ++sg) {
    const GemmSeg& S = G.seg[sg];
    const int64_t lb = max(kbeg - S.k0, (int64_t)0), le = min(kend - S.k0, S.K);
    if (lb >= le) continue;  // the same for the whole block
    const double* A = S.A + bz * S.sAb;
    const double* B = S.B + bz * S.sBb;
    const bool a_kfast = (S.sAk == 1);
    const bool b_nfast = (S.sBn == 1) || (S.sBk != 1);
    // the segment's summed-index maps in scalar registers for the whole K
    // loop (read through the dynamic segment index, they would otherwise be
    // fetched again from the argument block before every load)
    auto sreg = [](uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); };
    const IdxMap mAk{sreg(S.mAk.D), sreg(S.mAk.so), sreg(S.mAk.mag), sreg(S.mAk.sh)};
    const IdxMap mBk{sreg(S.mBk.D), sreg(S.mBk.so), sreg(S.mBk.mag), sreg(S.mBk.sh)};
    const int64_t sAk = (int64_t)sreg((uint32_t)S.sAk), sBk = (int64_t)sreg((uint32_t)S.sBk);
    auto a_pos = [&](int e, int& mm, int& kk) {
      const int idx = tid + e * GEMM_THREADS;
      if (a_kfast) {
        kk = idx % BKT;
        mm = idx / BKT;
      } else {
        mm = idx % BM;
        kk = idx / BM;
      }
    };
    auto b_pos = [&](int e, int& nn, int& kk) {
      const int idx = tid + e * GEMM_THREADS;
      if (b_nfast) {
        nn = idx % BN;
        kk = idx / BN;
      } else {
        kk = idx % BKT;
        nn = idx / BKT;
      }
    };
    uint32_t aoff[EA], boff[EB];
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int mm, kk;
      a_pos(e, mm, kk);
      const int64_t gm = m0 + mm;
      aoff[e] = gm < a.M ? imap32((uint32_t)gm, S.mAm, S.sAm) : 0u;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int nn, kk;
      b_pos(e, nn, kk);
      const int64_t gn = n0 + nn;
      boff[e] = gn < a.N ? imap32((uint32_t)gn, S.mBn, S.sBn) : 0u;
    }
    double ra[EA], rb[EB];
    auto load = [&](int64_t k0) {
#pragma unroll
      for (int e = 0; e < EA; ++e) {
        int mm, kk;
        a_pos(e, mm, kk);
        const int64_t gm = m0 + mm, gk = k0 + kk;
        ra[e] = (gm < a.M && gk < le) ? A[aoff[e] + imap32((uint32_t)gk, mAk, sAk)] : 0.0;
      }
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        int nn, kk;
        b_pos(e, nn, kk);
        const int64_t gn = n0 + nn, gk = k0 + kk;
        rb[e] = (gn < a.N && gk < le) ? B[boff[e] + imap32((uint32_t)gk, mBk, sBk)] : 0.0;
      }
    };
    const double alpha = S.alpha;
    load(lb);
    for (int64_t k0 = lb; k0 < le; k0 += BKT) {
#pragma unroll
      for (int e = 0; e < EA; ++e) {
        int mm, kk;
        a_pos(e, mm, kk);
        As[kk][mm] = (T)(alpha * ra[e]);
      }
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        int nn, kk;
        b_pos(e, nn, kk);
        Bs[kk][nn] = (T)rb[e];
      }
      __syncthreads();
      if (k0 + BKT < le) load(k0 + BKT);
#pragma unroll
      for (int kk = 0; kk < BKT; kk += 4) {
        const int kr = kk + (lane >> 4);
        T af[2], bf[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          af[t] = As[kr][wm + t * 16 + (lane & 15)];
          bf[t] = Bs[kr][wn + t * 16 + (lane & 15)];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            if constexpr (F32)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
          }
      }
      __syncthreads();
    }
  }
  const bool part = a.splits > 1;
  double* out = part ? a.P + split * a.M * a.N : a.C + bz * a.sCb;
  const double* Cin = (part || !a.Cin) ? nullptr : a.Cin + bz * a.sCb;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = F32 ? (lane >> 4) * 4 + r : r * 4 + (lane >> 4);
        const int64_t row = m0 + wm + i * 16 + rr;
        const int64_t col = n0 + wn + j * 16 + (lane & 15);
        if (row < a.M && col < a.N) {
          double v = (double)acc[i][j][r];
          const int64_t o = part ? row * a.N + col
                                 : (int64_t)(imap32((uint32_t)row, a.mCm, a.sCm) + imap32((uint32_t)col, a.mCn, a.sCn));
          if (Cin) v += a.beta * Cin[o];
          out[o] = v;
        }
      }
}

__global__ __launch_bounds__(GEMM_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void gemm_f64_multi_kernel(
    GemmMulti m) {
  __shared__ double As[GEMM_BK][BM + 1];
  __shared__ double Bs[GEMM_BK][BN + 1];
  gemm_multi_body<GEMM_BK, false>(m, As, Bs);
}

__global__ __launch_bounds__(GEMM_THREADS) __attribute__((amdgpu_waves_per_eu(4, 4))) void gemm_f32acc_multi_kernel(
    GemmMulti m) {
  __shared__ float As[GEMM_BK][BM + 1];
  __shared__ float Bs[GEMM_BK][BN + 1];
  gemm_multi_body<GEMM_BK, true>(m, As, Bs);
}

// sum_{s < n} p[s * stride] in the order s = 0, 1, ...: the loads are issued
// in batches of eight ahead of the additions (latency, not bandwidth, bounds
// a serial chain of loads)
__device__ __forceinline__ double ordered_sum(const double* p, int64_t n, int64_t stride) {
  double v = 0.0;
  int64_t s = 0;
  for (; s + 8 <= n; s += 8) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = p[(s + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += t[u];
  }
  for (; s < n; ++s) v += p[s * stride];
  return v;
}

__global__ void splitk_reduce_kernel(GemmArgs a) {
  const int64_t mn = a.M * a.N;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < mn; i += stride) {
    const int64_t row = i / a.N, col = i % a.N;
    double v = ordered_sum(a.P + i, a.splits, mn);
    const int64_t o = imap(row, a.mCm, a.sCm) + imap(col, a.mCn, a.sCn);
    if (a.Cin) v += a.beta * a.Cin[o];
    a.C[o] = v;
  }
}

__global__ void perm_kernel(PermArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t lin = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; lin < a.total; lin += stride) {
    int64_t rem = lin, oo = 0;
    int64_t io[4] = {0, 0, 0, 0};
    for (int d = a.nd - 1; d >= 0; --d) {
      const int64_t x = rem % a.dim[d];
      rem /= a.dim[d];
      oo += x * a.ostr[d];
      for (int i = 0; i < a.nin; ++i) io[i] += x * a.istr[i][d];
    }
    double v = 0.0;
    if (a.mul)
      v = a.coef[0] * a.in[0][io[0]] * a.in[1][io[1]];
    else
      for (int i = 0; i < a.nin; ++i) v += a.coef[i] * a.in[i][io[i]];
    if (a.addend) v += a.beta * a.addend[oo];
    a.out[oo] = v;
  }
}

__global__ void fill_kernel(double* p, int64_t n, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

constexpr int RED_THREADS = 256, RED_BLOCKS = 1024;

__device__ double block_sum(double v) {
  __shared__ double sh[RED_THREADS];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

__global__ __launch_bounds__(RED_THREADS) void dot_partial_kernel(const double* x, const double* y, int64_t n,
                                                                  double* partials) {
  double v = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = x[i + u * stride];
      b[u] = y[i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) v += a[u] * b[u];
  }
  for (; i < n; i += stride) v += x[i] * y[i];
  v = block_sum(v);
  if (threadIdx.x == 0) partials[blockIdx.x] = v;
}

__global__ __launch_bounds__(RED_THREADS) void dot_final_kernel(const double* partials, int nblocks, double alpha,
                                                                const double* addend, double beta, double* out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += blockDim.x) v += partials[i];
  v = block_sum(v);
  if (threadIdx.x == 0) out[0] = alpha * v + (addend ? beta * addend[0] : 0.0);
}

__global__ void axpby_kernel(double a, const double* x, double b, double* y, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = a * x[i] + b * y[i];
}

__global__ void precond_kernel(const double* x, const double* d, double shift, double fl, double* y, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double den = d[i] - shift;
    if (fabs(den) < fl) den = den < 0 ? -fl : fl;
    y[i] = x[i] / den;
  }
}

__global__ void sym_pairs_kernel(double* x, int64_t nov) {
  const int64_t total = nov * nov;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
    const int64_t p = i / nov, q = i % nov;
    if (p < q) {
      const double v = 0.5 * (x[p * nov + q] + x[q * nov + p]);
      x[p * nov + q] = v;
      x[q * nov + p] = v;
    }
  }
}

// one block per coordinate: grad[k] = <dh_k, D1> + <dL_k, Z>
__global__ __launch_bounds__(RED_THREADS) void deriv_contract_kernel(const double* dh, int64_t nh, const double* D1,
                                                                     const double* dL, int64_t nl, const double* Z,
                                                                     double* partials, int chunks) {
  const int k = blockIdx.y;
  const int c = blockIdx.x;
  const double* h = dh + (int64_t)k * nh;
  const double* l = dL + (int64_t)k * nl;
  double v = 0.0;
  const int64_t stride = (int64_t)chunks * blockDim.x;
  // four loads of each operand in flight per batch; same summation order
  auto dot = [&](const double* x, const double* y, int64_t n) {
    int64_t i = (int64_t)c * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = x[i + u * stride];
        b[u] = y[i + u * stride];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) v += a[u] * b[u];
    }
    for (; i < n; i += stride) v += x[i] * y[i];
  };
  dot(h, D1, nh);
  dot(l, Z, nl);
  v = block_sum(v);
  if (threadIdx.x == 0) partials[(int64_t)k * chunks + c] = v;
}

__global__ void deriv_final_kernel(const double* partials, int chunks, int ncoord, double* grad) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < ncoord) grad[k] = ordered_sum(partials + (int64_t)k * chunks, chunks, 1);
}

static void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

static unsigned grid_for(int64_t n, int threads = 256) {
  int64_t b = (n + threads - 1) / threads;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

void launch_gemm_main(const GemmArgs& a, hipStream_t s, bool f32) {
  if (a.M <= 0 || a.N <= 0 || a.batch <= 0) return;
  if (a.splits > 1 && (a.batch != 1 || !a.P || a.kchunk <= 0)) throw std::runtime_error("bad split-K plan");
  dim3 grid((unsigned)((a.N + BN - 1) / BN), (unsigned)((a.M + BM - 1) / BM),
            (unsigned)(a.splits > 1 ? a.splits : a.batch));
  if (grid.y > 65535 || grid.z > 65535 || (uint64_t)grid.x * grid.y * grid.z >= ((uint64_t)1 << 32))
    throw std::runtime_error("gemm grid too large");
  switch (gemm_kernel_id(a, f32)) {
    case GEMM_F64: hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(GEMM_THREADS), 0, s, a); break;
    case GEMM_F64_TWO: hipLaunchKernelGGL(gemm_f64_two_kernel, grid, dim3(GEMM_THREADS), 0, s, a); break;
    case GEMM_F32: hipLaunchKernelGGL(gemm_f32acc_kernel, grid, dim3(GEMM_THREADS), 0, s, a); break;
    default: hipLaunchKernelGGL(gemm_f32acc_two_kernel, grid, dim3(GEMM_THREADS), 0, s, a); break;
  }
  check(hipGetLastError(), "gemm launch");
}

void launch_gemm_reduce(const GemmArgs& a, hipStream_t s) {
  if (a.splits <= 1 || a.M <= 0 || a.N <= 0) return;
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid_for(a.M * a.N)), dim3(256), 0, s, a);
  check(hipGetLastError(), "split-K reduce launch");
}

void launch_gemm_multi(const GemmMulti& m, hipStream_t s, bool f32) {
  const GemmArgs& a = m.g;
  if (a.M <= 0 || a.N <= 0 || a.batch <= 0) return;
  if (m.nseg < 1 || m.nseg > MAXSEG) throw std::runtime_error("bad multi-segment GEMM");
  if (a.splits > 1 && (a.batch != 1 || !a.P || a.kchunk <= 0)) throw std::runtime_error("bad split-K plan");
  dim3 grid((unsigned)((a.N + BN - 1) / BN), (unsigned)((a.M + BM - 1) / BM),
            (unsigned)(a.splits > 1 ? a.splits : a.batch));
  if (grid.y > 65535 || grid.z > 65535 || (uint64_t)grid.x * grid.y * grid.z >= ((uint64_t)1 << 32))
    throw std::runtime_error("gemm grid too large");
  if (f32)
    hipLaunchKernelGGL(gemm_f32acc_multi_kernel, grid, dim3(GEMM_THREADS), 0, s, m);
  else
    hipLaunchKernelGGL(gemm_f64_multi_kernel, grid, dim3(GEMM_THREADS), 0, s, m);
  check(hipGetLastError(), "multi gemm launch");
}

void launch_gemm(const GemmArgs& a, hipStream_t s) {
  launch_gemm_main(a, s);
  launch_gemm_reduce(a, s);
}

// coefficients travel as kernel arguments (no host-to-device copy)
constexpr int COMBINE_MAXC = 224;
struct CombineCoef {
  double c[COMBINE_MAXC];
};

__global__ void combine_kernel(const double* __restrict__ X, int k, int64_t n, CombineCoef cf,
                               double* __restrict__ y) {
  const double* coef = cf.c;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double acc = y[i];
    int j = 0;
    for (; j + 8 <= k; j += 8) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = X[(int64_t)(j + u) * n + i];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += coef[j + u] * t[u];
    }
    for (; j < k; ++j) acc += coef[j] * X[(int64_t)j * n + i];
    y[i] = acc;
  }
}

__global__ __launch_bounds__(256) void gemv_rows_kernel(GemvArgs g) {
  // one wave per row; lanes stride over the unit-stride k index
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + wave;
  if (row >= g.R) return;  // the whole wave leaves together (no barriers below)
  const int64_t split = blockIdx.y;
  const int64_t kb = split * g.kchunk;
  const int64_t ke = g.splits > 1 ? min(g.K, kb + g.kchunk) : g.K;
  const double* m = g.Mt + row * g.sr;
  double acc = 0.0;
  int64_t k = kb + lane;
  for (; k + 3 * 64 < ke; k += 4 * 64) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = m[(k + 64 * u) * g.sk];
      b[u] = g.x[(k + 64 * u) * g.sx];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += a[u] * b[u];
  }
  for (; k < ke; k += 64) acc += m[k * g.sk] * g.x[k * g.sx];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) {
    if (g.splits > 1) {
      g.P[split * g.R + row] = acc;
    } else {
      double v = g.alpha * acc;
      if (g.yin) v += g.beta * g.yin[row * g.sy];
      g.y[row * g.sy] = v;
    }
  }
}

__global__ __launch_bounds__(256) void gemv_cols_kernel(GemvArgs g) {
  // one thread per row; neighbouring threads read neighbouring rows
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= g.R) return;
  const int64_t split = blockIdx.y;
  const int64_t kb = split * g.kchunk;
  const int64_t ke = g.splits > 1 ? min(g.K, kb + g.kchunk) : g.K;
  const double* m = g.Mt + row * g.sr;
  double acc = 0.0;
  int64_t k = kb;
  for (; k + 4 <= ke; k += 4) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = m[(k + u) * g.sk];
      b[u] = g.x[(k + u) * g.sx];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += a[u] * b[u];
  }
  for (; k < ke; ++k) acc += m[k * g.sk] * g.x[k * g.sx];
  if (g.splits > 1) {
    g.P[split * g.R + row] = acc;
  } else {
    double v = g.alpha * acc;
    if (g.yin) v += g.beta * g.yin[row * g.sy];
    g.y[row * g.sy] = v;
  }
}

__global__ void gemv_reduce_kernel(GemvArgs g) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < g.R; r += stride) {
    double v = ordered_sum(g.P + r, g.splits, g.R);
    v *= g.alpha;
    if (g.yin) v += g.beta * g.yin[r * g.sy];
    g.y[r * g.sy] = v;
  }
}

void launch_gemv(const GemvArgs& g, hipStream_t s) {
  if (g.R <= 0) return;
  if (g.splits > 1 && (!g.P || g.kchunk <= 0)) throw std::runtime_error("bad split GEMV plan");
  const int64_t bx = g.rows ? (g.R + 3) / 4 : (g.R + 255) / 256;
  if (bx > 0x7fffffff || g.splits > 65535) throw std::runtime_error("GEMV grid too large");
  dim3 grid((unsigned)bx, (unsigned)g.splits);
  if (g.rows)
    hipLaunchKernelGGL(gemv_rows_kernel, grid, dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL(gemv_cols_kernel, grid, dim3(256), 0, s, g);
  check(hipGetLastError(), "gemv launch");
  if (g.splits > 1) {
    hipLaunchKernelGGL(gemv_reduce_kernel, dim3(grid_for(g.R)), dim3(256), 0, s, g);
    check(hipGetLastError(), "gemv reduce launch");
  }
}

void launch_combine(const double* X, int k, int64_t n, const double* coef, double* y, hipStream_t s) {
  if (k <= 0 || n <= 0) return;
  // chunks of vectors in order: the additions keep the serial order
  for (int j0 = 0; j0 < k; j0 += COMBINE_MAXC) {
    const int kc = std::min(COMBINE_MAXC, k - j0);
    CombineCoef cf;
    for (int j = 0; j < kc; ++j) cf.c[j] = coef[j0 + j];
    hipLaunchKernelGGL(combine_kernel, dim3(grid_for(n)), dim3(256), 0, s, X + (int64_t)j0 * n, kc, n, cf, y);
    check(hipGetLastError(), "combine launch");
  }
}

// Index arithmetic of the permutation kernel in 32 bits: n / d for
// n, d < 2^31 as (umulhi(n, m) + n) >> s with s = ceil(log2 d) and
// m = floor(2^32 (2^s - d) / d) + 1 (round-up multiplier).
struct FastPerm {
  PermArgs a;
  uint32_t dim[MAXD], mag[MAXD], sh[MAXD];
};


template <int NIN, bool MUL>
__global__ __launch_bounds__(256) void perm_fast_kernel(FastPerm f) {
  const PermArgs& a = f.a;
  const uint32_t total = (uint32_t)a.total;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t lin = blockIdx.x * blockDim.x + threadIdx.x; lin < total; lin += stride) {
    uint32_t rem = lin;
    int64_t oo = 0;
    int64_t io[NIN];
#pragma unroll
    for (int i = 0; i < NIN; ++i) io[i] = 0;
#pragma unroll
    for (int d = MAXD - 1; d >= 0; --d) {
      if (d < a.nd) {
        const uint32_t q = fast_div(rem, f.mag[d], f.sh[d]);
        const int64_t x = (int64_t)(rem - q * f.dim[d]);
        rem = q;
        oo += x * a.ostr[d];
#pragma unroll
        for (int i = 0; i < NIN; ++i) io[i] += x * a.istr[i][d];
      }
    }
    double v = 0.0;
    if constexpr (MUL) {
      v = a.coef[0] * a.in[0][io[0]] * a.in[1][io[1]];
    } else {
#pragma unroll
      for (int i = 0; i < NIN; ++i) v += a.coef[i] * a.in[i][io[i]];
    }
    if (a.addend) v += a.beta * a.addend[oo];
    a.out[oo] = v;
  }
}

// Transposing copy: the output's unit-stride index x and the input's
// unit-stride index y differ.  32 x 32 tiles of (y, x) go through LDS so that
// both the reads (along y) and the writes (along x) are coalesced; the
// remaining indices of the iteration are decoded once per tile.
struct TransPerm {
  PermArgs a;
  int dx, dy;                    // iteration dims of the output / input unit strides
  uint32_t ntx, nty, nrest;      // tiles along x, y; product of the other dims
  int nr;                        // number of other dims
  int rd[MAXD];                  // their iteration dims (innermost last)
  uint32_t rdim[MAXD], rmag[MAXD], rsh[MAXD];
};

__global__ __launch_bounds__(256) void perm_transpose_kernel(TransPerm t) {
  __shared__ double tile[32][33];
  const PermArgs& a = t.a;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const uint32_t ntiles = t.ntx * t.nty;
  const uint32_t nblk = ntiles * t.nrest;
  for (uint32_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    uint32_t rest = blk / ntiles;
    const uint32_t tt = blk - rest * ntiles;
    const uint32_t by = tt / t.ntx, bx = tt - by * t.ntx;
    int64_t ibase = 0, obase = 0;
    for (int q = t.nr - 1; q >= 0; --q) {
      const uint32_t qd = fast_div(rest, t.rmag[q], t.rsh[q]);
      const int64_t x = (int64_t)(rest - qd * t.rdim[q]);
      rest = qd;
      ibase += x * a.istr[0][t.rd[q]];
      obase += x * a.ostr[t.rd[q]];
    }
    const int64_t X = a.dim[t.dx], Y = a.dim[t.dy];
    const int64_t x0 = (int64_t)bx * 32, y0 = (int64_t)by * 32;
    // read: consecutive lanes along y (unit stride in the input)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t y = y0 + tx, x = x0 + ty + 8 * i;
      if (y < Y && x < X) tile[ty + 8 * i][tx] = a.in[0][ibase + y * a.istr[0][t.dy] + x * a.istr[0][t.dx]];
    }
    __syncthreads();
    // write: consecutive lanes along x (unit stride in the output)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t x = x0 + tx, y = y0 + ty + 8 * i;
      if (y < Y && x < X) {
        const int64_t o = obase + x * a.ostr[t.dx] + y * a.ostr[t.dy];
        double v = a.coef[0] * tile[tx][ty + 8 * i];
        if (a.addend) v += a.beta * a.addend[o];
        a.out[o] = v;
      }
    }
    __syncthreads();
  }
}

void launch_perm(const PermArgs& in, hipStream_t s) {
  if (in.total <= 0) return;
  // merge neighbouring dimensions that are contiguous in the output and in
  // every input (fewer index digits per element)
  PermArgs a = in;
  for (int d = a.nd - 2; d >= 0; --d) {
    bool ok = a.ostr[d] == a.ostr[d + 1] * a.dim[d + 1];
    for (int i = 0; i < a.nin; ++i) ok = ok && a.istr[i][d] == a.istr[i][d + 1] * a.dim[d + 1];
    if (!ok) continue;
    a.dim[d] *= a.dim[d + 1];
    a.ostr[d] = a.ostr[d + 1];
    for (int i = 0; i < a.nin; ++i) a.istr[i][d] = a.istr[i][d + 1];
    for (int e = d + 1; e + 1 < a.nd; ++e) {
      a.dim[e] = a.dim[e + 1];
      a.ostr[e] = a.ostr[e + 1];
      for (int i = 0; i < a.nin; ++i) a.istr[i][e] = a.istr[i][e + 1];
    }
    --a.nd;
  }
  const int64_t lim = (int64_t)1 << 31;
  auto magic = [](uint64_t dd, uint32_t& mag, uint32_t& sh) {
    sh = 0;
    while ((1ull << sh) < dd) ++sh;
    mag = (uint32_t)(((1ull << 32) * ((1ull << sh) - dd)) / dd + 1);
  };
  // single input whose unit-stride index is not the output's: tiled transpose
  if (a.total < lim && a.nin == 1 && !a.mul && a.nd >= 2) {
    int dx = -1, dy = -1;
    for (int d = 0; d < a.nd; ++d) {
      if (a.ostr[d] == 1 && a.dim[d] > 1) dx = d;
      if (a.istr[0][d] == 1 && a.dim[d] > 1) dy = d;
    }
    if (dx >= 0 && dy >= 0 && dx != dy && a.dim[dx] >= 8 && a.dim[dy] >= 8) {
      TransPerm t{};
      t.a = a;
      t.dx = dx;
      t.dy = dy;
      t.ntx = (uint32_t)((a.dim[dx] + 31) / 32);
      t.nty = (uint32_t)((a.dim[dy] + 31) / 32);
      t.nr = 0;
      uint64_t rest = 1;
      for (int d = 0; d < a.nd; ++d) {
        if (d == dx || d == dy) continue;
        t.rd[t.nr] = d;
        t.rdim[t.nr] = (uint32_t)a.dim[d];
        magic((uint64_t)a.dim[d], t.rmag[t.nr], t.rsh[t.nr]);
        rest *= (uint64_t)a.dim[d];
        ++t.nr;
      }
      t.nrest = (uint32_t)rest;
      const uint64_t nblk = (uint64_t)t.ntx * t.nty * rest;
      if (nblk < ((uint64_t)1 << 31)) {
        const unsigned grid = (unsigned)std::min<uint64_t>(nblk, 65536);
        hipLaunchKernelGGL(perm_transpose_kernel, dim3(grid), dim3(256), 0, s, t);
        check(hipGetLastError(), "transpose launch");
        return;
      }
    }
  }
  if (a.total < lim && a.nin >= 1 && a.nin <= 4) {
    FastPerm f{};
    f.a = a;
    for (int d = 0; d < a.nd; ++d) {
      const uint64_t dd = (uint64_t)a.dim[d];
      uint32_t sh = 0;
      while ((1ull << sh) < dd) ++sh;
      f.dim[d] = (uint32_t)dd;
      f.sh[d] = sh;
      f.mag[d] = (uint32_t)(((1ull << 32) * ((1ull << sh) - dd)) / dd + 1);
    }
    const dim3 grid(grid_for(a.total)), block(256);
    if (a.mul) {
      hipLaunchKernelGGL((perm_fast_kernel<2, true>), grid, block, 0, s, f);
    } else {
      switch (a.nin) {
        case 1: hipLaunchKernelGGL((perm_fast_kernel<1, false>), grid, block, 0, s, f); break;
        case 2: hipLaunchKernelGGL((perm_fast_kernel<2, false>), grid, block, 0, s, f); break;
        case 3: hipLaunchKernelGGL((perm_fast_kernel<3, false>), grid, block, 0, s, f); break;
        default: hipLaunchKernelGGL((perm_fast_kernel<4, false>), grid, block, 0, s, f); break;
      }
    }
  } else {
    hipLaunchKernelGGL(perm_kernel, dim3(grid_for(a.total)), dim3(256), 0, s, a);
  }
  check(hipGetLastError(), "perm launch");
}

void launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  check(hipGetLastError(), "fill launch");
}

void launch_dot(const double* x, const double* y, int64_t n, double alpha, const double* addend, double beta,
                double* out, double* partials, hipStream_t s) {
  int nb = (int)std::max<int64_t>(1, std::min<int64_t>(RED_BLOCKS, (n + RED_THREADS * 4 - 1) / (RED_THREADS * 4)));
  hipLaunchKernelGGL(dot_partial_kernel, dim3(nb), dim3(RED_THREADS), 0, s, x, y, n, partials);
  hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(RED_THREADS), 0, s, partials, nb, alpha, addend, beta, out);
  check(hipGetLastError(), "dot launch");
}

void launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(axpby_kernel, dim3(grid_for(n)), dim3(256), 0, s, a, x, b, y, n);
  check(hipGetLastError(), "axpby launch");
}

void launch_precond(const double* x, const double* d, double shift, double fl, double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(precond_kernel, dim3(grid_for(n)), dim3(256), 0, s, x, d, shift, fl, y, n);
  check(hipGetLastError(), "precond launch");
}

void launch_sym_pairs(double* x, int64_t nov, hipStream_t s) {
  hipLaunchKernelGGL(sym_pairs_kernel, dim3(grid_for(nov * nov)), dim3(256), 0, s, x, nov);
  check(hipGetLastError(), "sym launch");
}

void launch_deriv_contract(const double* dh, int64_t nh, const double* D1, const double* dL, int64_t nl,
                           const double* Z, int ncoord, double* grad, double* partials, hipStream_t s) {
  if (ncoord <= 0) return;
  int chunks = (int)std::max<int64_t>(1, std::min<int64_t>(256, (nh + nl + 256 * 64 - 1) / (256 * 64)));
  while ((int64_t)chunks * ncoord > (1 << 18)) chunks /= 2;
  // partials must hold ncoord * chunks doubles
  hipLaunchKernelGGL(deriv_contract_kernel, dim3(chunks, ncoord), dim3(RED_THREADS), 0, s, dh, nh, D1, dL, nl, Z,
                     partials, chunks);
  hipLaunchKernelGGL(deriv_final_kernel, dim3((ncoord + 63) / 64), dim3(64), 0, s, partials, chunks, ncoord, grad);
  check(hipGetLastError(), "deriv launch");
}

// ---------------------------------------------------------------------------
// planning
// ---------------------------------------------------------------------------
// Split-K plan of one unbatched GEMM with `tiles` output tiles and summed
// length K.  The grid holds tiles * sp workgroups, of which GEMM_SLOTS are
// resident at once (256 CUs, four 256-thread workgroups each); the time is
// modelled as (rounds of resident workgroups) x (one workgroup's K chunk)
// plus the partial sums written and read back by the reduction.  A grid just
// above a multiple of the resident slots runs a nearly empty last round, so
// the split is chosen to fill the rounds, not only to reach one full round.
// The partial buffer is capped at 64 Mi doubles.  Returns sp (1: no split).
constexpr int64_t GEMM_SLOTS = 1024;
static int64_t choose_splits(int64_t M, int64_t N, int64_t K, int64_t tiles, int64_t& kchunk) {
  kchunk = K;
  if (K < 128 || M <= 0 || N <= 0) return 1;
  const double slot_rate = 45e12 / GEMM_SLOTS;  // FP64 flop/s of one resident workgroup
  const double red_rate = 5e12;                 // bytes/s of the partial-sum traffic
  const int64_t spmax = std::min<int64_t>({K / 64, (int64_t)1024, std::max<int64_t>(1, (64ll << 20) / (M * N))});
  double best = 0;
  int64_t bsp = 1;
  for (int64_t sp = 1; sp <= spmax; ++sp) {
    int64_t kc = (K + sp - 1) / sp;
    kc = (kc + BK - 1) / BK * BK;
    if ((K + kc - 1) / kc != sp) continue;
    const int64_t rounds = (tiles * sp + GEMM_SLOTS - 1) / GEMM_SLOTS;
    double t = (double)rounds * 2.0 * BM * BN * (double)kc / slot_rate;
    if (sp > 1) t += (double)(sp + 1) * (double)M * (double)N * 8.0 / red_rate;
    if (sp == 1 || t < 0.97 * best) {
      best = t;
      bsp = sp;
      kchunk = kc;
    }
  }
  return bsp;
}

static std::vector<int64_t> row_major_strides(const TensorDesc& d) {
  std::vector<int64_t> s(d.nd, 1);
  for (int i = d.nd - 2; i >= 0; --i) s[i] = s[i + 1] * d.dim[i + 1];
  return s;
}

struct View {
  bool ok;
  int64_t size, stride;
};

// Can indices `order` (a subsequence of labels `l`) of a row-major tensor be
// fused into one dimension (in that order)?
static View fuse(const std::string& l, const TensorDesc& d, const std::string& order) {
  auto st = row_major_strides(d);
  if (order.empty()) return {true, 1, 0};
  int64_t size = 1;
  for (size_t i = 0; i < order.size(); ++i) size *= d.dim[l.find(order[i])];
  for (size_t i = 0; i + 1 < order.size(); ++i) {
    int p = (int)l.find(order[i]), q = (int)l.find(order[i + 1]);
    if (st[p] != st[q] * d.dim[q]) return {false, size, 0};
  }
  return {true, size, st[l.find(order.back())]};
}

// Indices `order` as at most two runs of fusible dimensions: the outer run
// (stride ostride of its last index) and the inner run (size `inner`, stride
// `stride` of its last index); inner = 0 for a single run.
struct View2 {
  bool ok;
  int64_t size, stride, inner, ostride;
};

static View2 fuse2(const std::string& l, const TensorDesc& d, const std::string& order) {
  auto st = row_major_strides(d);
  if (order.empty()) return {true, 1, 0, 0, 0};
  int64_t size = 1;
  for (char c : order) size *= d.dim[l.find(c)];
  int breaks = 0, bpos = -1;
  for (size_t i = 0; i + 1 < order.size(); ++i) {
    int p = (int)l.find(order[i]), q = (int)l.find(order[i + 1]);
    if (st[p] != st[q] * d.dim[q]) {
      ++breaks;
      bpos = (int)i;
    }
  }
  const int64_t last = st[l.find(order.back())];
  if (breaks == 0) return {true, size, last, 0, 0};
  if (breaks > 1 || size >= ((int64_t)1 << 31)) return {false, size, 0, 0, 0};
  int64_t inner = 1;
  for (size_t i = bpos + 1; i < order.size(); ++i) inner *= d.dim[l.find(order[i])];
  return {true, size, last, inner, st[l.find(order[bpos])]};
}

static IdxMap make_map(const View2& v) {
  IdxMap m;
  if (v.inner == 0) return m;
  m.D = (uint32_t)v.inner;
  m.so = (uint32_t)v.ostride;
  uint32_t sh = 0;
  while ((1ull << sh) < (uint64_t)v.inner) ++sh;
  m.sh = sh;
  m.mag = (uint32_t)(((1ull << 32) * ((1ull << sh) - (uint64_t)v.inner)) / (uint64_t)v.inner + 1);
  return m;
}

static std::string filter(const std::string& src, const std::string& keep) {
  std::string r;
  for (char c : src)
    if (keep.find(c) != std::string::npos) r += c;
  return r;
}

// gather-copy tensor (labels l) into a contiguous buffer with index order `order`
static PermArgs pack_args(const TensorDesc& d, const std::string& l, const std::string& order, const double* src,
                          double* dst) {
  PermArgs p{};
  auto st = row_major_strides(d);
  p.nd = (int)order.size();
  p.nin = 1;
  p.in[0] = src;
  p.coef[0] = 1.0;
  p.out = dst;
  p.addend = nullptr;
  p.beta = 0.0;
  int64_t total = 1;
  for (int i = 0; i < p.nd; ++i) {
    int pos = (int)l.find(order[i]);
    p.dim[i] = d.dim[pos];
    p.istr[0][i] = st[pos];
    total *= p.dim[i];
  }
  int64_t s = 1;
  for (int i = p.nd - 1; i >= 0; --i) {
    p.ostr[i] = s;
    s *= p.dim[i];
  }
  p.total = total;
  if (p.nd == 0) {
    p.nd = 1;
    p.dim[0] = 1;
    p.istr[0][0] = 0;
    p.ostr[0] = 0;
    p.total = 1;
  }
  return p;
}

// Plan of a contraction with several products (Op::segs): the output index
// groups (batch, rows from the first operands, columns from the second) are
// common; each product gets its own summed-index order, and an operand that
// no order of up to two runs reads in place is packed.
static ContractPlan plan_multi(const Graph& g, const Op& op, double* arena, double* scratch) {
  ContractPlan P;
  P.kind = ContractKind::Multi;
  const TensorDesc& dO = g.t[op.out];
  const std::string& lo = op.lo;
  std::vector<Seg> ss = {Seg{op.a, op.b, op.la, op.lb, op.alpha}};
  for (const Seg& x : op.segs) ss.push_back(x);
  if ((int)ss.size() > MAXSEG) throw std::runtime_error("too many products in one contraction");
  std::string bat, mi, ni;
  for (char c : lo) {
    const bool ia = ss[0].la.find(c) != std::string::npos, ib = ss[0].lb.find(c) != std::string::npos;
    (ia && ib ? bat : ia ? mi : ni) += c;
  }
  for (const Seg& x : ss)
    for (char c : lo) {
      const bool ia = x.la.find(c) != std::string::npos, ib = x.lb.find(c) != std::string::npos;
      const bool ok = (ia && ib) ? bat.find(c) != std::string::npos
                                 : ia ? mi.find(c) != std::string::npos : ni.find(c) != std::string::npos;
      if (!ok) throw std::runtime_error("products of one contraction split the output differently");
    }
  const std::string bord = filter(lo, bat);
  int64_t M = 1, N = 1, Bt = 1;
  for (char c : mi) M *= dO.dim[lo.find(c)];
  for (char c : ni) N *= dO.dim[lo.find(c)];
  for (char c : bord) Bt *= dO.dim[lo.find(c)];
  constexpr double HBM_RATE = 3e12, LAUNCH_S = 4e-6;
  auto move_s = [&](int64_t elems) { return 16.0 * elems / HBM_RATE + LAUNCH_S; };
  auto kset = [&](const Seg& x) {
    std::string k;
    for (char c : x.la)
      if (x.lb.find(c) != std::string::npos && lo.find(c) == std::string::npos) k += c;
    return k;
  };
  // cost of one product for given row / column orders: best summed order
  auto seg_cost = [&](const Seg& x, const std::string& m, const std::string& n, std::string* kbest) {
    const TensorDesc& dA = g.t[x.a];
    const TensorDesc& dB = g.t[x.b];
    const std::string ki = kset(x);
    double best = -1;
    for (const std::string& k : {filter(x.la, ki), filter(x.lb, ki)}) {
      const bool okA = fuse2(x.la, dA, m).ok && fuse2(x.la, dA, k).ok && fuse(x.la, dA, bord).ok;
      const bool okB = fuse2(x.lb, dB, k).ok && fuse2(x.lb, dB, n).ok && fuse(x.lb, dB, bord).ok;
      const double c = (okA ? 0.0 : move_s(dA.size())) + (okB ? 0.0 : move_s(dB.size()));
      if (best < 0 || c < best) {
        best = c;
        if (kbest) *kbest = k;
      }
    }
    return best;
  };
  std::string bm, bn;
  double best = -1;
  for (const std::string& m : {filter(lo, mi), filter(ss[0].la, mi)})
    for (const std::string& n : {filter(lo, ni), filter(ss[0].lb, ni)}) {
      double c = (fuse2(lo, dO, m).ok && fuse2(lo, dO, n).ok && fuse(lo, dO, bord).ok) ? 0.0 : move_s(dO.size());
      for (const Seg& x : ss) c += seg_cost(x, m, n, nullptr);
      if (best < 0 || c < best) {
        best = c;
        bm = m;
        bn = n;
      }
    }
  const double* pC0 = op.c0 >= 0 ? arena + g.t[op.c0].offset : nullptr;
  double* pO = arena + dO.offset;
  GemmArgs& G = P.g;
  G.M = M;
  G.N = N;
  G.batch = Bt;
  G.alpha = 1.0;
  G.beta = op.beta;
  G.two = true;
  int64_t sc = 0, ktot = 0;
  for (const Seg& x : ss) {
    const TensorDesc& dA = g.t[x.a];
    const TensorDesc& dB = g.t[x.b];
    std::string bk;
    seg_cost(x, bm, bn, &bk);
    int64_t K = 1;
    for (char c : bk) K *= dA.dim[x.la.find(c)];
    GemmSeg q{};
    q.K = K;
    q.k0 = ktot;
    q.alpha = x.alpha;
    ktot += K;
    const double* pA = arena + dA.offset;
    const double* pB = arena + dB.offset;
    View2 vm = fuse2(x.la, dA, bm), vk = fuse2(x.la, dA, bk);
    View vb = fuse(x.la, dA, bord);
    if (vm.ok && vk.ok && vb.ok) {
      q.A = pA;
      q.sAm = vm.stride;
      q.sAk = vk.stride;
      q.sAb = vb.stride;
      q.mAm = make_map(vm);
      q.mAk = make_map(vk);
    } else {
      P.spacks.push_back(pack_args(dA, x.la, bord + bm + bk, pA, scratch + sc));
      q.A = scratch + sc;
      q.sAk = 1;
      q.sAm = K;
      q.sAb = M * K;
      sc += dA.size();
    }
    View2 wk = fuse2(x.lb, dB, bk), wn = fuse2(x.lb, dB, bn);
    View wb = fuse(x.lb, dB, bord);
    if (wk.ok && wn.ok && wb.ok) {
      q.B = pB;
      q.sBk = wk.stride;
      q.sBn = wn.stride;
      q.sBb = wb.stride;
      q.mBk = make_map(wk);
      q.mBn = make_map(wn);
    } else {
      P.spacks.push_back(pack_args(dB, x.lb, bord + bk + bn, pB, scratch + sc));
      q.B = scratch + sc;
      q.sBn = 1;
      q.sBk = N;
      q.sBb = K * N;
      sc += dB.size();
    }
    P.segs.push_back(q);
  }
  G.K = ktot;
  {
    View2 vm = fuse2(lo, dO, bm), vn = fuse2(lo, dO, bn);
    View vb = fuse(lo, dO, bord);
    if (vm.ok && vn.ok && vb.ok) {
      G.C = pO;
      G.Cin = pC0;
      G.sCm = vm.stride;
      G.sCn = vn.stride;
      G.sCb = vb.stride;
      G.mCm = make_map(vm);
      G.mCn = make_map(vn);
    } else {
      P.tmpC = true;
      double* tmp = scratch + sc;
      sc += dO.size();
      G.C = tmp;
      G.Cin = nullptr;
      G.beta = 0.0;
      G.sCn = 1;
      G.sCm = N;
      G.sCb = M * N;
      const std::string tl = bord + bm + bn;
      PermArgs& p = P.pc;
      p = PermArgs{};
      p.nd = (int)lo.size();
      p.nin = 1;
      p.in[0] = tmp;
      p.coef[0] = 1.0;
      p.out = pO;
      p.addend = pC0;
      p.beta = op.beta;
      std::vector<int64_t> tst(tl.size(), 1);
      for (int i = (int)tl.size() - 2; i >= 0; --i) tst[i] = tst[i + 1] * dO.dim[lo.find(tl[i + 1])];
      auto ost = row_major_strides(dO);
      int64_t total = 1;
      for (int i = 0; i < p.nd; ++i) {
        p.dim[i] = dO.dim[i];
        p.ostr[i] = ost[i];
        p.istr[0][i] = tst[tl.find(lo[i])];
        total *= dO.dim[i];
      }
      p.total = total;
    }
  }
  // every group through the branch-free two-run arithmetic
  const IdxMap ident{1u << 31, 0, 1, 31};
  for (IdxMap* m : {&G.mCm, &G.mCn})
    if (m->D == 0) *m = ident;
  for (GemmSeg& q : P.segs)
    for (IdxMap* m : {&q.mAm, &q.mAk, &q.mBk, &q.mBn})
      if (m->D == 0) *m = ident;
  // split-K over the concatenated summed index (fills the resident slots)
  if (Bt == 1) {
    const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
    int64_t kc = 0;
    const int64_t sp = choose_splits(M, N, ktot, tiles, kc);
    if (sp > 1) {
      G.splits = sp;
      G.kchunk = kc;
      G.P = scratch + sc;
      sc += sp * M * N;
    }
  }
  P.scratch = sc;
  return P;
}

ContractPlan plan_contract(const Graph& g, const Op& op, double* arena, double* scratch) {
  if (!op.segs.empty()) return plan_multi(g, op, arena, scratch);
  ContractPlan P;
  const TensorDesc& dA = g.t[op.a];
  const TensorDesc& dB = g.t[op.b];
  const TensorDesc& dO = g.t[op.out];
  const std::string &la = op.la, &lb = op.lb, &lo = op.lo;
  std::string bat, mi, ni, ki;
  for (char c : lo) {
    bool ia = la.find(c) != std::string::npos, ib = lb.find(c) != std::string::npos;
    if (ia && ib)
      bat += c;
    else if (ia)
      mi += c;
    else
      ni += c;
  }
  for (char c : la)
    if (lb.find(c) != std::string::npos && lo.find(c) == std::string::npos) ki += c;
  const double* pA = arena + dA.offset;
  const double* pB = arena + dB.offset;
  double* pO = arena + dO.offset;
  const double* pC0 = op.c0 >= 0 ? arena + g.t[op.c0].offset : nullptr;

  // scalar output: deterministic dot product
  if (lo.empty()) {
    std::string kord = filter(la, ki);
    View vb = fuse(lb, dB, kord);
    P.dot = true;
    int64_t n = dA.size();
    if (!(vb.ok && (vb.stride == 1 || n == 1))) {
      P.packB = true;
      P.pb = pack_args(dB, lb, kord, pB, scratch);
      P.scratch = n;
    }
    P.g.K = n;
    P.g.alpha = op.alpha;
    P.g.beta = op.beta;
    P.g.A = pA;
    P.g.B = P.packB ? scratch : pB;
    P.g.Cin = pC0;
    P.g.C = pO;
    return P;
  }

  // no summed index of extent above one: an elementwise product in the
  // output's order, broadcast through zero strides (no packs, no temporary)
  {
    int64_t kx = 1;
    for (char c : ki) kx *= dA.dim[la.find(c)];
    if (kx == 1) {
      auto sa = row_major_strides(dA), sb = row_major_strides(dB), so = row_major_strides(dO);
      PermArgs& p = P.pc;
      p = PermArgs{};
      p.nd = (int)lo.size();
      p.nin = 2;
      p.mul = 1;
      p.in[0] = pA;
      p.in[1] = pB;
      p.coef[0] = op.alpha;
      p.out = pO;
      p.addend = pC0;
      p.beta = op.beta;
      int64_t total = 1;
      for (int i = 0; i < p.nd; ++i) {
        const char c = lo[i];
        p.dim[i] = dO.dim[i];
        p.ostr[i] = so[i];
        p.istr[0][i] = la.find(c) != std::string::npos ? sa[la.find(c)] : 0;
        p.istr[1][i] = lb.find(c) != std::string::npos ? sb[lb.find(c)] : 0;
        total *= dO.dim[i];
      }
      p.total = total;
      P.kind = ContractKind::Outer;
      P.g.M = total;
      P.g.N = P.g.K = P.g.batch = 1;
      return P;
    }
  }

  // choose fused orders; candidates from each operand's memory order
  std::vector<std::string> mcand = {filter(lo, mi), filter(la, mi)};
  std::vector<std::string> ncand = {filter(lo, ni), filter(lb, ni)};
  std::vector<std::string> kcand = {filter(la, ki), filter(lb, ki)};
  std::string bord = filter(lo, bat);
  // Each candidate order is costed in time: the matrix-core kernel (slower
  // per flop when it reads some group as two runs, from the index
  // arithmetic of every load) plus each pack or output temporary as one
  // read and one write at HBM speed and a launch.  Degenerate shapes
  // (memory-bound kernels) take single-run operands only.
  int64_t Mx = 1, Nx = 1, Kx = 1, Bx = 1;
  for (char c : mi) Mx *= dO.dim[lo.find(c)];
  for (char c : ni) Nx *= dO.dim[lo.find(c)];
  for (char c : ki) Kx *= dA.dim[la.find(c)];
  for (char c : bat) Bx *= dO.dim[lo.find(c)];
  const int64_t lim32 = (int64_t)1 << 31;
  const bool two_ok = !(Bx == 1 && (Mx == 1 || Nx == 1)) && dA.size() < lim32 && dB.size() < lim32 &&
                      dO.size() < lim32;
  constexpr double GEMM_RATE = 40e12, TWO_PENALTY = 1.35, TWO_PENALTY_SHORT = 1.6, HBM_RATE = 3e12, LAUNCH_S = 4e-6;
  const double gemm_s = 2.0 * Mx * Nx * Kx * Bx / GEMM_RATE;
  auto move_s = [&](int64_t elems) { return 16.0 * elems / HBM_RATE + LAUNCH_S; };
  bool two = false;
  auto view = [&](const std::string& l, const TensorDesc& d, const std::string& order) {
    if (two) return fuse2(l, d, order);
    View v = fuse(l, d, order);
    return View2{v.ok, v.size, v.stride, 0, 0};
  };
  double best = -1;
  bool best_two = false;
  std::string bm, bn, bk;
  for (int mode = 0; mode < (two_ok ? 2 : 1); ++mode) {
    two = mode == 1;
    for (auto& m : mcand)
      for (auto& n : ncand)
        for (auto& k : kcand) {
          View2 am = view(la, dA, m), ak = view(la, dA, k), bk_ = view(lb, dB, k), bn_ = view(lb, dB, n);
          View2 cm = view(lo, dO, m), cn = view(lo, dO, n);
          const bool okA = am.ok && ak.ok && fuse(la, dA, bord).ok;
          const bool okB = bk_.ok && bn_.ok && fuse(lb, dB, bord).ok;
          const bool okC = cm.ok && cn.ok && fuse(lo, dO, bord).ok;
          const bool any_two = (okA && (am.inner || ak.inner)) || (okB && (bk_.inner || bn_.inner)) ||
                               (okC && (cm.inner || cn.inner));
          if (two && !any_two) continue;  // the single-run pass has this one
          // a unit-stride group in runs shorter than 16 elements breaks the
          // coalescing of its loads or stores (measured about 25 % slower)
          bool short_runs = false;
          const View2* vs[6] = {&am, &ak, &bk_, &bn_, &cm, &cn};
          const bool oks[6] = {okA, okA, okB, okB, okC, okC};
          for (int q = 0; q < 6; ++q)
            if (oks[q] && vs[q]->inner && vs[q]->stride == 1 && vs[q]->inner < 16) short_runs = true;
          double cost = gemm_s * (any_two ? (short_runs ? TWO_PENALTY_SHORT : TWO_PENALTY) : 1.0);
          if (!okA) cost += move_s(dA.size());
          if (!okB) cost += move_s(dB.size());
          if (!okC) cost += move_s(dO.size());
          if (best < 0 || cost < best) {
            best = cost;
            best_two = two;
            bm = m;
            bn = n;
            bk = k;
          }
        }
  }
  two = best_two;
  int64_t M = 1, N = 1, K = 1, Bt = 1;
  for (char c : bm) M *= dO.dim[lo.find(c)];
  for (char c : bn) N *= dO.dim[lo.find(c)];
  for (char c : bk) K *= dA.dim[la.find(c)];
  for (char c : bord) Bt *= dO.dim[lo.find(c)];
  GemmArgs& G = P.g;
  G.M = M;
  G.N = N;
  G.K = K;
  G.batch = Bt;
  G.alpha = op.alpha;
  G.beta = op.beta;
  int64_t sc = 0;
  // A
  {
    View2 vm = view(la, dA, bm), vk = view(la, dA, bk);
    View vb = fuse(la, dA, bord);
    if (vm.ok && vk.ok && vb.ok) {
      G.A = pA;
      G.sAm = vm.stride;
      G.sAk = vk.stride;
      G.sAb = vb.stride;
      G.mAm = make_map(vm);
      G.mAk = make_map(vk);
    } else {
      P.packA = true;
      P.pa = pack_args(dA, la, bord + bm + bk, pA, scratch + sc);
      G.A = scratch + sc;
      G.sAk = 1;
      G.sAm = K;
      G.sAb = M * K;
      sc += dA.size();
    }
  }
  // B
  {
    View2 vk = view(lb, dB, bk), vn = view(lb, dB, bn);
    View vb = fuse(lb, dB, bord);
    if (vk.ok && vn.ok && vb.ok) {
      G.B = pB;
      G.sBk = vk.stride;
      G.sBn = vn.stride;
      G.sBb = vb.stride;
      G.mBk = make_map(vk);
      G.mBn = make_map(vn);
    } else {
      P.packB = true;
      P.pb = pack_args(dB, lb, bord + bk + bn, pB, scratch + sc);
      G.B = scratch + sc;
      G.sBn = 1;
      G.sBk = N;
      G.sBb = K * N;
      sc += dB.size();
    }
  }
  // C
  {
    View2 vm = view(lo, dO, bm), vn = view(lo, dO, bn);
    View vb = fuse(lo, dO, bord);
    if (vm.ok && vn.ok && vb.ok) {
      G.C = pO;
      G.Cin = pC0;
      G.sCm = vm.stride;
      G.sCn = vn.stride;
      G.sCb = vb.stride;
      G.mCm = make_map(vm);
      G.mCn = make_map(vn);
    } else {
      P.tmpC = true;
      double* tmp = scratch + sc;
      sc += dO.size();
      G.C = tmp;
      G.Cin = nullptr;
      G.beta = 0.0;
      G.sCn = 1;
      G.sCm = N;
      G.sCb = M * N;
      // out[lo] = tmp[bord+bm+bn] + beta c0
      std::string tl = bord + bm + bn;
      PermArgs& p = P.pc;
      p = PermArgs{};
      p.nd = (int)lo.size();
      p.nin = 1;
      p.in[0] = tmp;
      p.coef[0] = 1.0;
      p.out = pO;
      p.addend = pC0;
      p.beta = op.beta;
      std::vector<int64_t> tst(tl.size(), 1);
      for (int i = (int)tl.size() - 2; i >= 0; --i) tst[i] = tst[i + 1] * dO.dim[lo.find(tl[i + 1])];
      auto ost = row_major_strides(dO);
      int64_t total = 1;
      for (int i = 0; i < p.nd; ++i) {
        p.dim[i] = dO.dim[i];
        p.ostr[i] = ost[i];
        p.istr[0][i] = tst[tl.find(lo[i])];
        total *= dO.dim[i];
      }
      p.total = total;
    }
  }
  G.two = G.mAm.D || G.mAk.D || G.mBk.D || G.mBn.D || G.mCm.D || G.mCn.D;
  if (G.two) {
    // the two-run kernel takes every group through the same branch-free
    // arithmetic: a single run is a first run of 2^31 (quotient 0)
    for (IdxMap* m : {&G.mAm, &G.mAk, &G.mBk, &G.mBn, &G.mCm, &G.mCn})
      if (m->D == 0) *m = IdxMap{1u << 31, 0, 1, 31};
  }
  // degenerate shapes are memory-bound: no matrix cores
  if (Bt == 1 && (N == 1 || M == 1)) {
    GemvArgs& v = P.gv;
    v = GemvArgs{};
    v.K = K;
    v.alpha = G.alpha;
    v.beta = G.beta;
    v.y = G.C;
    v.yin = G.Cin;
    if (N == 1) {
      v.R = M;
      v.Mt = G.A;
      v.sr = G.sAm;
      v.sk = G.sAk;
      v.x = G.B;
      v.sx = G.sBk;
      v.sy = G.sCm;
    } else {
      v.R = N;
      v.Mt = G.B;
      v.sr = G.sBn;
      v.sk = G.sBk;
      v.x = G.A;
      v.sx = G.sAk;
      v.sy = G.sCn;
    }
    v.rows = v.sk == 1 && v.sr != 1;
    const int64_t blocks = v.rows ? (v.R + 3) / 4 : (v.R + 255) / 256;
    const int64_t kmin = v.rows ? 512 : 64;
    int64_t sp = std::min<int64_t>((1024 + blocks - 1) / blocks, K / kmin);
    sp = std::min<int64_t>(sp, 4096);
    if (sp > 1) {
      const int64_t kc = (K + sp - 1) / sp;
      v.splits = (K + kc - 1) / kc;
      v.kchunk = kc;
      v.P = scratch + sc;
      sc += v.splits * v.R;
    }
    P.kind = ContractKind::Gemv;
    P.scratch = sc;
    return P;
  }
  // split-K (fills the resident slots; long K with few output tiles)
  if (Bt == 1) {
    const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
    int64_t kc = 0;
    const int64_t sp = choose_splits(M, N, K, tiles, kc);
    if (sp > 1) {
      G.splits = sp;
      G.kchunk = kc;
      G.P = scratch + sc;
      sc += sp * M * N;
    }
  }
  P.scratch = sc;
  return P;
}

int64_t Executor::plan_scratch(Graph& g) {
  int64_t mx = 0;
  for (auto& op : g.ops)
    if (op.kind == OpKind::Contract) {
      ContractPlan p = plan_contract(g, op, nullptr, nullptr);
      mx = std::max(mx, p.scratch);
    }
  return mx;
}

void Executor::plan_all() {
  plans_.assign(g_.ops.size(), ContractPlan{});
  for (size_t k = 0; k < g_.ops.size(); ++k)
    if (g_.ops[k].kind == OpKind::Contract) {
      plans_[k] = plan_contract(g_, g_.ops[k], arena_, scratch_);
      if (plans_[k].scratch > scratch_n_) throw std::runtime_error("scratch too small");
    }
}

Executor::~Executor() {
  for (auto& e : ev_) (void)hipEventDestroy(e);
  for (auto& kv : graphs_cache_) {
    for (auto& e : kv.second.ev) (void)hipEventDestroy(e);
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
  }
}

// algorithmic bytes of one GEMM launch: both operands read once, the output
// written once (and read once when accumulated)
static double gemm_bytes(const GemmArgs& g) {
  return 8.0 * g.batch * ((double)(g.M + g.N) * g.K + (double)g.M * g.N * (g.Cin ? 2 : 1));
}

void Executor::account(double ms, double flops, double bytes, const std::array<int64_t, 5>& shape, int kid) {
  kernel_ms[kid] += ms;
  kernel_flops[kid] += flops;
  kernel_bytes[kid] += bytes;
  ++kernel_launches[kid];
  ShapeStat& st = shapes_[{shape[0], shape[1], shape[2], shape[3], shape[4], kid}];
  st.n += 1;
  st.ms += ms;
  st.flops += flops;
}

void Executor::set_profile(bool on) {
  if (on && ev_.empty()) {
    ev_.resize(2 * 4096);
    for (auto& e : ev_) check(hipEventCreate(&e), "event create");
    ev_flops_.resize(4096);
    ev_bytes_.resize(4096);
    ev_shape_.resize(4096);
    ev_kid_.resize(4096);
  }
  if (!on) flush_profile();
  prof_ = on;
}

void Executor::flush_profile() {
  if (nev_ == 0) return;
  check(hipEventSynchronize(ev_[2 * nev_ - 1]), "event sync");
  for (size_t i = 0; i < nev_; ++i) {
    float ms = 0;
    check(hipEventElapsedTime(&ms, ev_[2 * i], ev_[2 * i + 1]), "event elapsed");
    account(ms, ev_flops_[i], ev_bytes_[i], ev_shape_[i], ev_kid_[i]);
  }
  nev_ = 0;
}

void Executor::timed_gemm(const GemmArgs& g, hipStream_t s, bool f32, const GemmMulti* multi) {
  const int kid = multi ? (f32 ? GEMM_F32_MULTI : GEMM_F64_MULTI) : gemm_kernel_id(g, f32);
  auto main = [&]() {
    if (multi)
      launch_gemm_multi(*multi, s, f32);
    else
      launch_gemm_main(g, s, f32);
  };
  if (cap_) {
    // inside a graph capture: event pairs of the graph's own
    hipEvent_t e0, e1;
    check(hipEventCreate(&e0), "event create");
    check(hipEventCreate(&e1), "event create");
    cap_->ev.push_back(e0);
    cap_->ev.push_back(e1);
    check(hipEventRecord(e0, s), "event record");
    main();
    check(hipEventRecord(e1, s), "event record");
    launch_gemm_reduce(g, s);
    cap_->flops.push_back(2.0 * g.M * g.N * g.K * g.batch);
    cap_->bytes.push_back(gemm_bytes(g));
    cap_->shape.push_back({g.M, g.N, g.K, g.batch, g.splits});
    cap_->kid.push_back((char)kid);
    return;
  }
  if (nev_ == ev_flops_.size()) flush_profile();
  // the events bracket the MFMA kernel alone (a split-K reduction follows)
  check(hipEventRecord(ev_[2 * nev_], s), "event record");
  main();
  ev_kid_[nev_] = (char)kid;
  check(hipEventRecord(ev_[2 * nev_ + 1], s), "event record");
  launch_gemm_reduce(g, s);
  ev_flops_[nev_] = 2.0 * g.M * g.N * g.K * g.batch;
  ev_bytes_[nev_] = gemm_bytes(g);
  ev_shape_[nev_] = {g.M, g.N, g.K, g.batch, g.splits};
  ++nev_;
}

void Executor::shape_report(FILE* f, int top) const {
  static const char* names[NGEMMK] = {"f64", "f64/two", "f32", "f32/two", "f64/sum", "f32/sum"};
  std::vector<std::pair<std::array<int64_t, 6>, ShapeStat>> v(shapes_.begin(), shapes_.end());
  std::sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return a.second.ms > b.second.ms; });
  std::fprintf(f, "gemm shapes by time (M N K batch splits kernel: launches, ms, TFLOP/s)\n");
  for (int i = 0; i < (int)v.size() && i < top; ++i) {
    const auto& k = v[i].first;
    const auto& st = v[i].second;
    std::fprintf(f, "  %7lld %7lld %7lld %4lld %3lld %-7s: %9lld %10.1f %6.2f\n", (long long)k[0], (long long)k[1],
                 (long long)k[2], (long long)k[3], (long long)k[4], names[k[5]], (long long)st.n, st.ms,
                 st.ms > 0 ? st.flops / (st.ms * 1e9) : 0.0);
  }
  for (int q = 0; q < NGEMMK; ++q)
    if (kernel_launches[q])
      std::fprintf(f, "  kernel %-7s: %lld launches, %.1f ms, %.2f TFLOP/s\n", names[q], (long long)kernel_launches[q],
                   kernel_ms[q], kernel_flops[q] / (kernel_ms[q] * 1e9));
}

double Executor::flops(const std::vector<int>& list) const {
  double f = 0;
  for (int k : list)
    if (g_.ops[k].kind == OpKind::Contract) {
      // (multi-segment plans hold the total summed extent in g.K)
      const ContractPlan& p = plans_[k];
      if (p.dot)
        f += 2.0 * p.g.K;
      else
        f += 2.0 * p.g.M * p.g.N * p.g.K * p.g.batch;
    }
  return f;
}

void Executor::run(const std::vector<int>& list, hipStream_t s) {
  if (!graphs_ || prof_ || list.empty()) {
    for (int k : list) run_op(k, s);
    return;
  }
  const std::array<int64_t, 3> key = {(int64_t)(intptr_t)&list, lowp_ ? 1 : 0, prof_ ? 1 : 0};
  auto it = graphs_cache_.find(key);
  if (it == graphs_cache_.end()) {
    flush_profile();
    Captured c;
    cap_ = &c;
    check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "graph capture begin");
    try {
      for (int k : list) run_op(k, s);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(s, &g);
      if (g) (void)hipGraphDestroy(g);
      cap_ = nullptr;
      for (auto& e : c.ev) (void)hipEventDestroy(e);
      throw;
    }
    cap_ = nullptr;
    check(hipStreamEndCapture(s, &c.graph), "graph capture end");
    check(hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0), "graph instantiate");
    it = graphs_cache_.emplace(key, std::move(c)).first;
  }
  Captured& c = it->second;
  check(hipGraphLaunch(c.exec, s), "graph launch");
  if (prof_ && !c.ev.empty()) {
    // the event nodes are re-recorded by the next replay: read them now
    check(hipStreamSynchronize(s), "graph profile sync");
    for (size_t i = 0; i < c.flops.size(); ++i) {
      float ms = 0;
      check(hipEventElapsedTime(&ms, c.ev[2 * i], c.ev[2 * i + 1]), "event elapsed");
      account(ms, c.flops[i], c.bytes[i], c.shape[i], c.kid[i]);
    }
  }
}

void Executor::run_op(int k, hipStream_t s) {
  const Op& op = g_.ops[k];
  if (op.kind == OpKind::Nop) return;
  if (g_.t[op.out].offset < 0) throw std::runtime_error("op without storage (not in any program)");
  switch (op.kind) {
    case OpKind::Nop:
      break;
    case OpKind::Contract: {
      const ContractPlan& p = plans_[k];
      if (p.kind == ContractKind::Multi) {
        for (const PermArgs& pk : p.spacks) launch_perm(pk, s);
        GemmMulti gm{};
        gm.g = p.g;
        gm.nseg = (int)p.segs.size();
        for (int q = 0; q < gm.nseg; ++q) gm.seg[q] = p.segs[q];
        const bool f32 = lowp_ && p.g.M >= 64 && p.g.N >= 64 && p.g.K >= 64;
        if (prof_ && (prof_mask_ >> (f32 ? GEMM_F32_MULTI : GEMM_F64_MULTI) & 1u)) {
          timed_gemm(p.g, s, f32, &gm);
        } else {
          launch_gemm_multi(gm, s, f32);
          launch_gemm_reduce(p.g, s);
        }
        if (p.tmpC) launch_perm(p.pc, s);
        break;
      }
      if (p.packA) launch_perm(p.pa, s);
      if (p.packB) launch_perm(p.pb, s);
      if (p.dot) {
        launch_dot(p.g.A, p.g.B, p.g.K, p.g.alpha, p.g.Cin, p.g.beta, p.g.C, partials_, s);
      } else if (p.kind == ContractKind::Outer) {
        launch_perm(p.pc, s);
      } else if (p.kind == ContractKind::Gemv) {
        launch_gemv(p.gv, s);
        if (p.tmpC) launch_perm(p.pc, s);
      } else {
        const bool f32 = lowp_ && p.g.M >= 64 && p.g.N >= 64 && p.g.K >= 64;
        if (prof_ && (prof_mask_ >> gemm_kernel_id(p.g, f32) & 1u)) {
          timed_gemm(p.g, s, f32);
        } else {
          launch_gemm_main(p.g, s, f32);
          launch_gemm_reduce(p.g, s);
        }
        if (p.tmpC) launch_perm(p.pc, s);
      }
      break;
    }
    case OpKind::Lincomb: {
      const TensorDesc& dO = g_.t[op.out];
      auto ost = row_major_strides(dO);
      size_t i0 = 0;
      const double* prev = nullptr;
      while (i0 < op.ins.size()) {
        PermArgs p{};
        p.nd = dO.nd;
        int64_t total = 1;
        for (int d = 0; d < dO.nd; ++d) {
          p.dim[d] = dO.dim[d];
          p.ostr[d] = ost[d];
          total *= dO.dim[d];
        }
        if (dO.nd == 0) {
          p.nd = 1;
          p.dim[0] = 1;
          p.ostr[0] = 0;
        }
        p.total = total;
        p.out = ptr(op.out);
        p.addend = prev;
        p.beta = prev ? 1.0 : 0.0;
        int cnt = 0;
        for (; i0 < op.ins.size() && cnt < 4; ++i0, ++cnt) {
          const TensorDesc& di = g_.t[op.ins[i0]];
          auto ist = row_major_strides(di);
          p.in[cnt] = ptr(op.ins[i0]);
          p.coef[cnt] = op.coef[i0];
          for (int d = 0; d < dO.nd; ++d) p.istr[cnt][d] = ist[op.lin[i0].find(op.lo[d])];
          if (dO.nd == 0) p.istr[cnt][0] = 0;
        }
        p.nin = cnt;
        launch_perm(p, s);
        prev = p.out;
      }
      break;
    }
    case OpKind::Slice:
    case OpKind::Embed: {
      const TensorDesc& di = g_.t[op.a];
      const TensorDesc& dO = g_.t[op.out];
      auto ist = row_major_strides(di);
      auto ost = row_major_strides(dO);
      PermArgs p{};
      p.nin = 1;
      p.coef[0] = 1.0;
      p.addend = nullptr;
      if (op.kind == OpKind::Slice) {
        int64_t base = 0;
        for (int d = 0; d < di.nd; ++d) base += op.off[d] * ist[d];
        p.nd = dO.nd;
        for (int d = 0; d < dO.nd; ++d) {
          p.dim[d] = dO.dim[d];
          p.istr[0][d] = ist[d];
          p.ostr[d] = ost[d];
        }
        p.in[0] = ptr(op.a) + base;
        p.out = ptr(op.out);
        p.total = dO.size();
      } else {
        launch_fill(ptr(op.out), dO.size(), 0.0, s);
        int64_t base = 0;
        for (int d = 0; d < dO.nd; ++d) base += op.off[d] * ost[d];
        p.nd = di.nd;
        for (int d = 0; d < di.nd; ++d) {
          p.dim[d] = di.dim[d];
          p.istr[0][d] = ist[d];
          p.ostr[d] = ost[d];
        }
        p.in[0] = ptr(op.a);
        p.out = ptr(op.out) + base;
        p.total = di.size();
      }
      launch_perm(p, s);
      break;
    }
  }
}

}  // namespace scc
