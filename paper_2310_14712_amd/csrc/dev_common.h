// Device helpers shared by the HIP kernels of the library: launch width,
// lane exchanges through DPP and wave-level reductions, strided row dots.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace imex {
namespace dev {

constexpr int kThreads = 256;

template <typename T>
__device__ inline double to_d(T v) { return (double)v; }

// within 8 lanes, mirror within 16 lanes.
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

// sums over aligned groups of 4 / 8 / 16 lanes (every lane gets the sum)
__device__ inline double reduce4(double v) {
  v += dpp_move<kDppXor1>(v);
  v += dpp_move<kDppXor2>(v);
  return v;
}
__device__ inline double reduce8(double v) {
  v = reduce4(v);
  v += dpp_move<kDppHalfMirror>(v);
  return v;
}
__device__ inline double reduce16(double v) {
  v = reduce8(v);
  v += dpp_move<kDppMirror>(v);
  return v;
}
__device__ inline double reduce64(double v) {
  v = reduce16(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}
__device__ inline double reduce_max64(double v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Partial dot product of a row M[0..n) with x[0..n) over LANES lanes (lane
// `sub` takes t = sub, sub + LANES, ...): the first LANES * PER entries are
// loaded at once, the rest (if any) in further batches of the same size.
// NT: M is read once per step, with non-temporal loads.
template <int LANES, int PER, bool NT = false, typename XP>
__device__ inline double row_dot(const double* M, XP x, int n, int sub) {
  double acc = 0.0;
  for (int base = 0; base < n; base += LANES * PER) {
    double mv[PER], xv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = base + sub + u * LANES;
      mv[u] = t < n ? (NT ? __builtin_nontemporal_load(&M[t]) : M[t]) : 0.0;
      xv[u] = t < n ? x[t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) acc += mv[u] * xv[u];
  }
  return acc;
}

// The dispatcher hands workgroups to the chip's 8 XCDs in turn (workgroup b
// to XCD b mod 8), and each XCD has its own L2.  Renumbering so that XCD x
// runs one contiguous range of logical ids keeps neighbouring tiles, whose
// halos share cache lines, on one L2.  A bijection of [0, n) for any n.
constexpr int kXcds = 8;
__device__ inline int xcd_contiguous(int b, int n) {
  const int q = n / kXcds, r = n % kXcds, x = b % kXcds, k = b / kXcds;
  return x * q + min(x, r) + k;
}

// Quotient and remainder by a workgroup-uniform divisor 0 < d < 2^22, for
// 0 <= n < 2^22, through one FP32 product with the correctly rounded
// reciprocal: the product carries a relative error below 2^-23, so the
// truncated float quotient is off by at most one, which one integer
// correction removes.  About a third of the instructions of a general
// 32-bit division.
struct SmallDiv {
  int d;
  float r;
  __device__ explicit SmallDiv(int d_) : d(d_), r(1.0f / (float)d_) {}
  __device__ inline int quot(int n, int* rem) const {
    int q = (int)((float)n * r);
    int m = n - q * d;
    if (m < 0) {
      --q;
      m += d;
    } else if (m >= d) {
      ++q;
      m -= d;
    }
    *rem = m;
    return q;
  }
};

inline dim3 grid1d(int64_t n, int t) { return dim3((unsigned)((n + t - 1) / t)); }

// The instance of workgroup b in a batched launch: the i with
// first[i] <= b < first[i + 1] (first: n + 1 ascending block offsets).
__device__ inline int batch_instance(const int32_t* first, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Let kernel k use all the LDS of a workgroup on the current device (less
// its static LDS): contexts with different tiles or factors share the kernel
// functions, so the attribute is not tied to one context's size.
inline hipError_t allow_full_lds(const void* k) {
  int dev = 0, v = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  hipFuncAttributes fa;
  if (e == hipSuccess) e = hipFuncGetAttributes(&fa, k);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, v - (int)fa.sharedSizeBytes);
}

}  // namespace dev
}  // namespace imex
