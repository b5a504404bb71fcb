// Setup-time dense inverses on the device: the dissected factor stores
// A_pp^-1 and Sigma^-1 of every part and separator system (they make each
// step's solve a set of parallel dense products).  Blocks of a few thousand
// rows (3D meshes) are inverted here rather than on the host.
//
// Method: Gauss-Jordan elimination in place without pivoting, one rank-one
// sweep per pivot.  For an SPD matrix every pivot is the diagonal entry of a
// Schur complement and therefore positive, so no pivoting is needed; a
// non-positive pivot reports the matrix as not positive definite.  Each
// sweep reads and writes the matrix once: O(n^3) work in n pairs of
// launches, about a second for n = 7000, once per context.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "internal.h"

namespace imex {

namespace {

// pivot row k scaled by 1/p (entry k: 1/p) and the old column k (entry k: 0)
__global__ void gj_prep_kernel(const double* A, int64_t n, int64_t k, double* r, double* c, int* bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double p = A[k * n + k];
  if (t == k && !(p > 0.0)) bad[0] = 1;
  r[t] = t == k ? 1.0 / p : A[k * n + t] / p;
  c[t] = t == k ? 0.0 : A[t * n + k];
}

// A[k, :] = r; A[i, j] = A[i, j] - c_i r_j (i != k), with A[i, k] taken as 0
__global__ void gj_sweep_kernel(double* A, int64_t n, int64_t k, const double* r, const double* c) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j >= n) return;
  double* Ai = A + i * n;
  if (i == k) Ai[j] = r[j];
  else Ai[j] = (j == k ? 0.0 : Ai[j]) - c[i] * r[j];
}

std::mutex g_inverse_mutex;  // the factor's components are built by several host threads

}  // namespace

bool gpu_spd_inverse(double* A, int64_t n, int device) {
  if (n <= 0) return true;
  if (n > 65535) return false;  // one grid row per matrix row
  std::lock_guard<std::mutex> lock(g_inverse_mutex);
  if (hipSetDevice(device) != hipSuccess) return false;  // the calling host thread may be a worker
  const size_t bytes = sizeof(double) * (size_t)n * (size_t)n;
  double *dA = nullptr, *dr = nullptr, *dc = nullptr;
  int* dbad = nullptr;
  hipStream_t s = nullptr;
  bool ok = hipStreamCreate(&s) == hipSuccess;
  ok = ok && hipMalloc(&dA, bytes) == hipSuccess;
  ok = ok && hipMalloc(&dr, sizeof(double) * n) == hipSuccess;
  ok = ok && hipMalloc(&dc, sizeof(double) * n) == hipSuccess;
  ok = ok && hipMalloc(&dbad, sizeof(int)) == hipSuccess;
  ok = ok && hipMemcpyAsync(dA, A, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
  ok = ok && hipMemsetAsync(dbad, 0, sizeof(int), s) == hipSuccess;
  if (ok) {
    const dim3 blk(256), g1((unsigned)((n + 255) / 256)), g2((unsigned)((n + 255) / 256), (unsigned)n);
    for (int64_t k = 0; k < n && ok; ++k) {
      hipLaunchKernelGGL(gj_prep_kernel, g1, blk, 0, s, dA, n, k, dr, dc, dbad);
      hipLaunchKernelGGL(gj_sweep_kernel, g2, blk, 0, s, dA, n, k, dr, dc);
      ok = hipGetLastError() == hipSuccess;
    }
  }
  int bad = 1;
  ok = ok && hipMemcpyAsync(&bad, dbad, sizeof(int), hipMemcpyDeviceToHost, s) == hipSuccess;
  ok = ok && hipMemcpyAsync(A, dA, bytes, hipMemcpyDeviceToHost, s) == hipSuccess;
  ok = ok && hipStreamSynchronize(s) == hipSuccess;
  if (dA) (void)hipFree(dA);
  if (dr) (void)hipFree(dr);
  if (dc) (void)hipFree(dc);
  if (dbad) (void)hipFree(dbad);
  if (s) (void)hipStreamDestroy(s);
  if (!ok || bad) return false;
  // the exact inverse is symmetric; average the two rounded halves
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < i; ++j) {
      const double v = 0.5 * (A[i * n + j] + A[j * n + i]);
      A[i * n + j] = v;
      A[j * n + i] = v;
    }
  return true;
}

}  // namespace imex
