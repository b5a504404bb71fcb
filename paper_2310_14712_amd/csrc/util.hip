// Small utility kernels of the library: the device step counter, state
// conversions between the grid storage type and FP64, increments.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "device.h"

namespace imex {

namespace {

using namespace dev;

__global__ void set_int_kernel(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}
__global__ void add_int_kernel(int* p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = p[0] + v;
}

template <typename T>
__global__ void scatter_c_kernel(T* grid, const int64_t* c_nodes, const double* src, int64_t nc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc) grid[c_nodes[i]] = T(src[i]);
}
template <typename T>
__global__ void grid_to_f64_kernel(const T* grid, double* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)grid[i];
}
template <typename T>
__global__ void f64_to_grid_kernel(const double* src, T* grid, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) grid[i] = T(src[i]);
}

// receiver r: sum over its cell's nodes of basis value x nodal value
template <typename T>
__global__ void sample_kernel(const T* grid, const int64_t* ids, const double* w, int nb, int64_t n, double* out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double s = 0.0;
  for (int t = 0; t < nb; ++t) s += w[r * nb + t] * (double)grid[ids[r * nb + t]];
  out[r] = s;
}

// receiver r with its basis evaluated on the device: the containing cell
// (the lower one on a face) and the tensor Lagrange basis there, from the
// point's coordinates; the same sum over the cell's nodes as sample_kernel.
// The host has checked that every point lies in the box and in an active cell.
template <typename T>
__global__ void sample_points_kernel(const T* grid, const SamplePointsArgs A, const double* pts, int64_t n,
                                     double* out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int nb1 = A.n;
  double val[3][kMaxN];
  int64_t cidx[3] = {0, 0, 0};
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < kMaxN; ++i) val[k][i] = 1.0;
  for (int k = 0; k < A.dim; ++k) {
    const double x = pts[r * A.dim + k];
    int64_t ci = (int64_t)floor(x / A.h[k]);
    ci = ci < A.ne[k] - 1 ? ci : A.ne[k] - 1;
    cidx[k] = ci;
    const double xi = 2.0 * (x - ci * A.h[k]) / A.h[k] - 1.0;
    for (int i = 0; i < nb1; ++i) {
      double v = 1.0;
      for (int j = 0; j < nb1; ++j) {
        if (j == i) continue;
        v = v * (xi - A.x[j]) * (1.0 / (A.x[i] - A.x[j]));
      }
      val[k][i] = v;
    }
  }
  const int p = nb1 - 1;
  const int64_t g0 = cidx[0] * p + A.nn[0] * (cidx[1] * p + A.nn[1] * (cidx[2] * p));
  const int nz = A.dim == 3 ? nb1 : 1;
  double s = 0.0;
  for (int c = 0; c < nz; ++c)
    for (int b = 0; b < nb1; ++b)
      for (int a = 0; a < nb1; ++a) {
        double w = val[0][a] * val[1][b];
        if (A.dim == 3) w *= val[2][c];
        s += w * (double)grid[g0 + a + A.nn[0] * (b + A.nn[1] * c)];
      }
  out[r] = s;
}

// failure detection: any NaN or Inf among x[0..n) sets *flag (every writer
// stores the same value, so the order of the stores does not matter)
template <typename T>
__global__ void nonfinite_kernel(const T* x, int64_t n, int* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    bad |= !__builtin_isfinite((double)x[i]);
  if (bad) flag[0] = 1;
}

__global__ void sub_f32_kernel(float* d, const float* a, const float* b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = a[i] - b[i];
}


}  // namespace

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}
hipError_t launch_add_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(add_int_kernel, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_check_finite(const void* x, int64_t n, int fp, int* flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const dim3 g((unsigned)std::min<int64_t>((n + 255) / 256, 2048));
  if (fp == 32)
    hipLaunchKernelGGL(nonfinite_kernel<float>, g, dim3(256), 0, s, static_cast<const float*>(x), n, flag);
  else
    hipLaunchKernelGGL(nonfinite_kernel<double>, g, dim3(256), 0, s, static_cast<const double*>(x), n, flag);
  return hipGetLastError();
}

hipError_t launch_scatter_c(void* grid, const int64_t* c_nodes, const double* src, int64_t nc,
                            int fp, hipStream_t s) {
  if (nc == 0) return hipSuccess;
  if (fp == 32)
    hipLaunchKernelGGL(scatter_c_kernel<float>, grid1d(nc, 256), dim3(256), 0, s,
                       static_cast<float*>(grid), c_nodes, src, nc);
  else
    hipLaunchKernelGGL(scatter_c_kernel<double>, grid1d(nc, 256), dim3(256), 0, s,
                       static_cast<double*>(grid), c_nodes, src, nc);
  return hipGetLastError();
}

hipError_t launch_grid_to_f64(const void* grid, double* dst, int64_t n, int fp, hipStream_t s) {
  if (fp == 32)
    hipLaunchKernelGGL(grid_to_f64_kernel<float>, grid1d(n, 256), dim3(256), 0, s,
                       static_cast<const float*>(grid), dst, n);
  else
    hipLaunchKernelGGL(grid_to_f64_kernel<double>, grid1d(n, 256), dim3(256), 0, s,
                       static_cast<const double*>(grid), dst, n);
  return hipGetLastError();
}

hipError_t launch_sub_f32(float* d, const float* a, const float* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(sub_f32_kernel, grid1d(n, 256), dim3(256), 0, s, d, a, b, n);
  return hipGetLastError();
}

hipError_t launch_f64_to_grid(const double* src, void* grid, int64_t n, int fp, hipStream_t s) {
  if (fp == 32)
    hipLaunchKernelGGL(f64_to_grid_kernel<float>, grid1d(n, 256), dim3(256), 0, s, src,
                       static_cast<float*>(grid), n);
  else
    hipLaunchKernelGGL(f64_to_grid_kernel<double>, grid1d(n, 256), dim3(256), 0, s, src,
                       static_cast<double*>(grid), n);
  return hipGetLastError();
}

hipError_t launch_sample(const void* grid, const int64_t* ids, const double* w, int nb, int64_t n, double* out,
                         int fp, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (fp == 32)
    hipLaunchKernelGGL(sample_kernel<float>, grid1d(n, 256), dim3(256), 0, s, static_cast<const float*>(grid), ids, w,
                       nb, n, out);
  else
    hipLaunchKernelGGL(sample_kernel<double>, grid1d(n, 256), dim3(256), 0, s, static_cast<const double*>(grid), ids,
                       w, nb, n, out);
  return hipGetLastError();
}

hipError_t launch_sample_points(const void* grid, const SamplePointsArgs& a, const double* pts, int64_t n,
                                double* out, int fp, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (fp == 32)
    hipLaunchKernelGGL(sample_points_kernel<float>, grid1d(n, 256), dim3(256), 0, s,
                       static_cast<const float*>(grid), a, pts, n, out);
  else
    hipLaunchKernelGGL(sample_points_kernel<double>, grid1d(n, 256), dim3(256), 0, s,
                       static_cast<const double*>(grid), a, pts, n, out);
  return hipGetLastError();
}

}  // namespace imex
