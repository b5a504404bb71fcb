// HIP kernels (gfx950) of the iterative solvers of the implicit block S:
// flexible CG vector kernels, the element-block preconditioner and the
// per-cut-cell MLP preconditioner (BF16 MFMA inference and training).
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "learned.h"
#include <cstdlib>

namespace imex {

namespace {

using namespace dev;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite inputs)
__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------------------------------
// BF16 GEMM: one wave per 16 x 16 tile of C, 4 waves per workgroup.
// v_mfma_f32_16x16x16_bf16 operand layout: lane l holds A[l % 16][4 (l / 16) + j]
// and B[4 (l / 16) + j][l % 16] (j = 0..3); the result lane l holds
// C[4 (l / 16) + j][l % 16].
// ---------------------------------------------------------------------------
__device__ inline bf16x4 load_frag(const uint16_t* p, int ld, int layout, int row, int k) {
  bf16x4 v;
  if (layout == kRowMajor) {
    v = *reinterpret_cast<const bf16x4*>(p + (size_t)row * ld + k);  // 8-byte aligned: ld, k multiples of 4
  } else {
    v[0] = (short)p[(size_t)(k + 0) * ld + row];
    v[1] = (short)p[(size_t)(k + 1) * ld + row];
    v[2] = (short)p[(size_t)(k + 2) * ld + row];
    v[3] = (short)p[(size_t)(k + 3) * ld + row];
  }
  return v;
}

__global__ __launch_bounds__(256) void gemm_bf16_kernel(const GemmArgs g) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tiles_n = g.N / 16, tiles = (g.M / 16) * tiles_n;
  const int t = blockIdx.x * 4 + wave;
  if (t >= tiles) return;
  const int tm = t / tiles_n, tn = t - tm * tiles_n;
  const int kz = blockIdx.y;
  const int k_begin = g.epi == kEpiPartial ? kz * g.ksplit : 0;
  const int k_end = g.epi == kEpiPartial ? min(g.K, k_begin + g.ksplit) : g.K;
  const int r = lane & 15, kq = (lane >> 4) * 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = k_begin; k0 < k_end; k0 += 16) {
    // A operand: A(tm 16 + r, k0 + kq + j);  B operand: B(k0 + kq + j, tn 16 + r)
    const bf16x4 a = load_frag(g.a, g.lda, g.a_layout, tm * 16 + r, k0 + kq);
    const bf16x4 b = load_frag(g.b, g.ldb, g.b_layout, tn * 16 + r, k0 + kq);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  const int n = tn * 16 + r;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int m = tm * 16 + kq + j;
    const size_t o = (size_t)m * g.N + n;
    float v = acc[j];
    switch (g.epi) {
      case kEpiBiasReluBf16:
        g.out_b[o] = f2bf(fmaxf(v + g.bias[n], 0.f));
        break;
      case kEpiBiasF32:
        g.out_f[o] = v + g.bias[n];
        break;
      case kEpiMaskF32Bf16: {
        const bool on = (g.mask[o] & 0x7FFF) != 0 && (g.mask[o] & 0x8000) == 0;
        v = on ? v : 0.f;
        g.out_f[o] = v;
        g.out_b[o] = f2bf(v);
        break;
      }
      default:
        g.out_f[(size_t)kz * g.M * g.N + o] = v;
        break;
    }
  }
}

// The same products by 64 x 64 blocks of C per workgroup: for each k step of
// 16 the block's A (64 x 16) and B (16 x 64) slices are staged in LDS with
// coalesced loads (transposed operands are transposed on the way), and each
// wave takes 2 x 2 tiles of 16 x 16 from there.  Every tile still takes one
// MFMA per k step in increasing k, so the results equal the kernel above.
constexpr int kGemmBlk = 64, kGemmLdsK = 20;  // LDS row: 16 k values and 4 of padding
__global__ __launch_bounds__(256) void gemm_bf16_lds_kernel(const GemmArgs g) {
  __shared__ __align__(16) uint16_t sA[kGemmBlk][kGemmLdsK], sB[kGemmBlk][kGemmLdsK];  // [m][k], [n][k]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int blocks_n = (g.N + kGemmBlk - 1) / kGemmBlk;
  const int m0 = (blockIdx.x / blocks_n) * kGemmBlk, n0 = (blockIdx.x % blocks_n) * kGemmBlk;
  const int kz = blockIdx.y;
  const int k_begin = g.epi == kEpiPartial ? kz * g.ksplit : 0;
  const int k_end = g.epi == kEpiPartial ? min(g.K, k_begin + g.ksplit) : g.K;
  const int r = lane & 15, kq = (lane >> 4) * 4;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;  // the wave's 32 x 32 corner of the block
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jn = 0; jn < 2; ++jn) acc[i][jn] = f32x4{0.f, 0.f, 0.f, 0.f};
  // staging: row-major operands, thread -> (row t / 4, k 4 (t % 4)); transposed
  // ones, thread -> (k t / 16, rows 4 (t % 16) .. + 3)
  auto stage = [&](const uint16_t* p, int ld, int layout, int row0, int rows, int k0, uint16_t (*dst)[kGemmLdsK]) {
    if (layout == kRowMajor) {
      const int row = tid >> 2, k = (tid & 3) * 4;
      bf16x4 v = {0, 0, 0, 0};
      if (row0 + row < rows) v = *reinterpret_cast<const bf16x4*>(p + (size_t)(row0 + row) * ld + k0 + k);
      *reinterpret_cast<bf16x4*>(&dst[row][k]) = v;
    } else {
      const int k = tid >> 4, row = (tid & 15) * 4;
      bf16x4 v = {0, 0, 0, 0};
      if (row0 + row < rows) v = *reinterpret_cast<const bf16x4*>(p + (size_t)(k0 + k) * ld + row0 + row);
#pragma unroll
      for (int i = 0; i < 4; ++i) dst[row + i][k] = (uint16_t)v[i];
    }
  };
  for (int k0 = k_begin; k0 < k_end; k0 += 16) {
    __syncthreads();  // the previous step's fragments have been read
    stage(g.a, g.lda, g.a_layout, m0, g.M, k0, sA);
    stage(g.b, g.ldb, g.b_layout, n0, g.N, k0, sB);
    __syncthreads();
    bf16x4 af[2], bfr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      af[i] = *reinterpret_cast<const bf16x4*>(&sA[wm + 16 * i + r][kq]);
      bfr[i] = *reinterpret_cast<const bf16x4*>(&sB[wn + 16 * i + r][kq]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int jn = 0; jn < 2; ++jn) acc[i][jn] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[i], bfr[jn], acc[i][jn], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jn = 0; jn < 2; ++jn) {
      const int tm0 = m0 + wm + 16 * i, tn0 = n0 + wn + 16 * jn;
      if (tm0 >= g.M || tn0 >= g.N) continue;  // M, N are multiples of 16: whole tiles
      const int n = tn0 + r;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = tm0 + kq + j;
        const size_t o = (size_t)m * g.N + n;
        float v = acc[i][jn][j];
        switch (g.epi) {
          case kEpiBiasReluBf16:
            g.out_b[o] = f2bf(fmaxf(v + g.bias[n], 0.f));
            break;
          case kEpiBiasF32:
            g.out_f[o] = v + g.bias[n];
            break;
          case kEpiMaskF32Bf16: {
            const bool on = (g.mask[o] & 0x7FFF) != 0 && (g.mask[o] & 0x8000) == 0;
            v = on ? v : 0.f;
            g.out_f[o] = v;
            g.out_b[o] = f2bf(v);
            break;
          }
          default:
            g.out_f[(size_t)kz * g.M * g.N + o] = v;
            break;
        }
      }
    }
}

__global__ void sum_slices_kernel(const float* part, int slices, int64_t n, float* out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  float acc = 0.f;
  for (int s = 0; s < slices; ++s) acc += part[(size_t)s * n + j];
  out[j] = acc;
}

// column sums: stage 1 over 256-row chunks, stage 2 over chunks
__global__ void colsum_stage1(const float* m, int64_t rows, int cols, float* work) {
  const int c = blockIdx.y * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  const int64_t r0 = (int64_t)blockIdx.x * 256, r1 = min(rows, r0 + 256);
  float acc = 0.f;
  for (int64_t r = r0; r < r1; ++r) acc += m[r * cols + c];
  work[(size_t)blockIdx.x * cols + c] = acc;
}
__global__ void colsum_stage2(const float* work, int chunks, int cols, float* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float acc = 0.f;
  for (int k = 0; k < chunks; ++k) acc += work[(size_t)k * cols + c];
  out[c] = acc;
}

// ---------------------------------------------------------------------------
// MLP rows: features, targets, loss, scatter
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mlp_features_kernel(const ElemArgs L, const MlpDims d, const double* R,
                                                           const double* BR, const int* vsel, int n_vec,
                                                           int rows_pad, uint16_t* X, double* s, float* valid) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows_pad) return;
  const int nrows = n_vec * L.E;
  uint16_t* x = X + (size_t)row * d.F;
  if (row >= nrows) {
    for (int f = lane; f < d.F; f += 64) x[f] = 0;
    if (lane == 0) {
      s[row] = 0.0;
      valid[row] = 0.f;
    }
    return;
  }
  const int k = row / L.E, e = row - k * L.E;
  const size_t voff = (size_t)(vsel ? vsel[k] : k) * L.nc;
  const double* r = R + voff;
  const double* br = BR + voff;
  const int32_t* idx = L.eidx + (size_t)e * L.ne;
  double ss = 0.0;
  for (int l = lane; l < L.ne; l += 64) {
    const double t = r[idx[l]];
    ss += t * t;
  }
  ss = reduce64(ss);
  const double sn = sqrt(ss);
  for (int f = lane; f < d.F; f += 64) {
    float val = 0.f;
    if (f < L.ne) {
      val = sn > 0.0 ? (float)(r[idx[f]] / sn) : 0.f;
    } else if (f < 2 * L.ne) {
      const int32_t i = idx[f - L.ne];
      val = sn > 0.0 ? (float)(L.diag[i] * br[i] / sn) : 0.f;
    } else if (f < 3 * L.ne) {
      val = L.gfeat[(size_t)e * L.ne + (f - 2 * L.ne)];
    }
    x[f] = f2bf(val);
  }
  if (lane == 0) {
    s[row] = sn;
    valid[row] = sn > 0.0 ? 1.f : 0.f;
  }
}

// Training rows: a cell takes part in the loss of a pair only if its local
// residual norm is at least kTrainRel times the largest over the pair's
// cells.  On cells whose residual is negligible the target (the local
// correction over the local norm) is the response to residuals elsewhere,
// which the cell's features do not see, and unbounded.
constexpr double kTrainRel = 1e-3;
__global__ __launch_bounds__(256) void mlp_train_rows_kernel(int E, int n_vec, int rows_pad, const double* s,
                                                             float* valid) {
  __shared__ double red[4];
  const int k = blockIdx.x;  // one workgroup per pair
  double mx = 0.0;
  for (int e = threadIdx.x; e < E; e += 256) mx = fmax(mx, s[(size_t)k * E + e]);
  mx = reduce_max64(mx);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  for (int e = threadIdx.x; e < E; e += 256) {
    const double v = s[(size_t)k * E + e];
    valid[(size_t)k * E + e] = (v > 0.0 && v >= kTrainRel * mx) ? 1.f : 0.f;
  }
  (void)n_vec;
  (void)rows_pad;
}

__global__ __launch_bounds__(256) void mlp_targets_kernel(const ElemArgs L, const MlpDims d, const double* Xs,
                                                          const double* BR, const int* vsel, int n_vec,
                                                          int rows_pad, const double* s, const float* valid,
                                                          float* T) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows_pad) return;
  float* t = T + (size_t)row * d.O;
  const int nrows = n_vec * L.E;
  const bool on = row < nrows && valid[row] > 0.f;
  if (!on) {
    for (int l = lane; l < d.O; l += 64) t[l] = 0.f;
    return;
  }
  const int k = row / L.E, e = row - k * L.E;
  const size_t voff = (size_t)(vsel ? vsel[k] : k) * L.nc;
  const double* x = Xs + voff;
  const double* br = BR + voff;
  const int32_t* idx = L.eidx + (size_t)e * L.ne;
  for (int l = lane; l < d.O; l += 64) {
    float out = 0.f;
    if (l < L.ne) {
      const int32_t i = idx[l];
      out = (float)(L.diag[i] * (x[i] - br[i]) / s[row]);
    }
    t[l] = out;
  }
}

__global__ __launch_bounds__(256) void mlp_loss_kernel(const MlpDims d, int ne, int rows_pad, const float* Y,
                                                       const float* T, const float* valid, float inv_count,
                                                       float* dY, uint16_t* dYb, double* partial) {
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = blockIdx.x * 4 + wave;
  double ls = 0.0;
  if (row < rows_pad) {
    const float w = valid[row];
    for (int l = lane; l < d.O; l += 64) {
      const size_t o = (size_t)row * d.O + l;
      const float diff = (l < ne) ? (Y[o] - T[o]) * w : 0.f;
      ls += (double)diff * diff;
      const float g = 2.f * diff * inv_count;
      dY[o] = g;
      dYb[o] = f2bf(g);
    }
  }
  ls = reduce64(ls);
  if (lane == 0) red[wave] = ls;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void mlp_scatter_kernel(const ElemArgs L, const MlpDims d, const double* s, const float* Y, double* z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.nc) return;
  double acc = 0.0;
  for (int k = L.inc_ptr[i]; k < L.inc_ptr[i + 1]; ++k) {
    const int e = L.inc[k] / L.ne, l = L.inc[k] - e * L.ne;
    acc += s[e] * (double)Y[(size_t)e * d.O + l];
  }
  z[i] = L.inv_mult[i] * (acc / L.diag[i]);
}

// y = x - y (FP64 vectors)
__global__ void rsub_kernel(const double* x, double* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i] - y[i];
}

// element-block preconditioner: ze = Binv_e r_e (wave per cell), then the
// sum over the cells at every dof
__global__ __launch_bounds__(256) void block_apply_kernel(const ElemArgs L, const double* r, double* ze) {
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (e >= L.E) return;
  const int32_t* idx = L.eidx + (size_t)e * L.ne;
  const double* B = L.binv + (size_t)e * L.ne * L.ne;
  for (int l = lane; l < L.ne; l += 64) {
    double acc = 0.0;
    for (int j = 0; j < L.ne; ++j) acc += B[(size_t)l * L.ne + j] * r[idx[j]];
    ze[(size_t)e * L.ne + l] = acc;
  }
}
__global__ void block_scatter_kernel(const ElemArgs L, const double* ze, double* z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.nc) return;
  double acc = 0.0;
  for (int k = L.inc_ptr[i]; k < L.inc_ptr[i + 1]; ++k) acc += ze[L.inc[k]];
  z[i] = acc;
}

__global__ void adam_kernel(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2, uint16_t* pb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  pb[i] = f2bf(pi);
}
__global__ void to_bf16_kernel(const float* x, uint16_t* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// ---------------------------------------------------------------------------
// flexible CG
// ---------------------------------------------------------------------------
// block-level sum of one double per thread (256 threads) into part[blockIdx.x]
__device__ inline void block_sum_store(double v, double* part) {
  __shared__ double red[4];
  v = reduce64(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
}

// wave per row, grid-stride over the rows; returns this lane's share of y_i
__device__ inline double csr_row(const CsrDev& S, int64_t i, const double* x, int lane) {
  double acc = 0.0;
  for (int64_t k = S.rp[i] + lane; k < S.rp[i + 1]; k += 64) acc += S.val[k] * x[S.col[k]];
  return reduce64(acc);
}

__global__ __launch_bounds__(256) void fcg_init_kernel(const CsrDev S, const double* b, const double* x, double* r,
                                                       double* part) {
  const int lane = threadIdx.x & 63;
  double bb = 0.0, rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < S.n; i += (int64_t)gridDim.x * 4) {
    const double sx = csr_row(S, i, x, lane);
    if (lane == 0) {
      const double ri = b[i] - sx;
      r[i] = ri;
      bb += b[i] * b[i];
      rr += ri * ri;
    }
  }
  block_sum_store(bb, part);
  block_sum_store(rr, part + kFcgBlocks);
}

__global__ __launch_bounds__(256) void fcg_spmv_kernel(const CsrDev S, const double* p, double* q, double* part) {
  const int lane = threadIdx.x & 63;
  double pq = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < S.n; i += (int64_t)gridDim.x * 4) {
    const double qi = csr_row(S, i, p, lane);
    if (lane == 0) {
      q[i] = qi;
      pq += p[i] * qi;
    }
  }
  block_sum_store(pq, part);
}

__global__ __launch_bounds__(256) void fcg_update_kernel(int64_t n, const double* sc, double* x, double* r,
                                                         double* r_old, const double* p, const double* q,
                                                         double* part) {
  const double alpha = sc[kAlpha];
  double rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const double ro = r[i];
    const double rn = ro - alpha * q[i];
    r_old[i] = ro;
    r[i] = rn;
    rr += rn * rn;
  }
  block_sum_store(rr, part);
}

__global__ __launch_bounds__(256) void fcg_dots_kernel(int64_t n, const double* z, const double* r,
                                                       const double* r_old, const double* diag, double* part) {
  double zd = 0.0, rz = 0.0, jd = 0.0, rj = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ri = r[i];
    const double dr = r_old ? ri - r_old[i] : ri;
    const double ji = ri / diag[i];
    zd += z[i] * dr;
    rz += ri * z[i];
    jd += ji * dr;
    rj += ri * ji;
  }
  block_sum_store(zd, part);
  block_sum_store(rz, part + kFcgBlocks);
  block_sum_store(jd, part + 2 * kFcgBlocks);
  block_sum_store(rj, part + 3 * kFcgBlocks);
}

// block k sums partial array k into sc[dst + k]
// partials of br.q2, br.r and c.r (the learned preconditioner's combination)
__global__ __launch_bounds__(256) void combine_dots_kernel(int64_t n, const double* br, const double* q2,
                                                           const double* c, const double* r, double* part) {
  double a12 = 0.0, b1 = 0.0, b2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    a12 += br[i] * q2[i];
    b1 += br[i] * r[i];
    b2 += c[i] * r[i];
  }
  block_sum_store(a12, part);
  block_sum_store(b1, part + kFcgBlocks);
  block_sum_store(b2, part + 2 * kFcgBlocks);
}

// z = beta1 br + beta2 c, (beta1, beta2) minimising the S-norm of the error
// over span{br, c} from sc = [br.S br, c.S c, br.S c, br.r, c.r]; a
// degenerate pair (c = 0 or parallel to br) keeps the scaled br
__global__ void combine_kernel(int64_t n, const double* sc, const double* br, const double* c, double* z) {
  const double a11 = sc[0], a22 = sc[1], a12 = sc[2], b1 = sc[3], b2 = sc[4];
  const double det = a11 * a22 - a12 * a12;
  double be1 = a11 > 0.0 ? b1 / a11 : 0.0, be2 = 0.0;
  if (a22 > 0.0 && det > 1e-12 * a11 * a22) {
    be1 = (b1 * a22 - b2 * a12) / det;
    be2 = (a11 * b2 - a12 * b1) / det;
  }
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = be1 * br[i] + be2 * c[i];
}

__global__ __launch_bounds__(256) void fcg_reduce_kernel(const double* part, double* sc, int dst) {
  const double* p = part + (size_t)blockIdx.x * kFcgBlocks;
  double v = 0.0;
  for (int i = threadIdx.x; i < kFcgBlocks; i += 256) v += p[i];
  __shared__ double red[4];
  v = reduce64(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) sc[dst + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void fcg_scalars_kernel(double* sc, int which) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (which == 1) {
    sc[kAlpha] = sc[kRZ] / sc[kPQ];
    return;
  }
  const bool use_j = !(sc[kRZn] > 0.0);  // also when not finite
  sc[kUseJ] = use_j ? 1.0 : 0.0;
  if (which == 0) {
    sc[kRZ] = use_j ? sc[kRJ] : sc[kRZn];
    sc[kBeta] = 0.0;
  } else {
    sc[kBeta] = (use_j ? sc[kJdR] : sc[kZdR]) / sc[kRZ];
    sc[kRZ] = use_j ? sc[kRJ] : sc[kRZn];
  }
}

__global__ void fcg_direction_kernel(int64_t n, const double* sc, const double* z, const double* r,
                                     const double* diag, double* p, int start) {
  const bool use_j = sc[kUseJ] != 0.0;
  const double beta = sc[kBeta];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double zeta = use_j ? r[i] / diag[i] : z[i];
    p[i] = start ? zeta : zeta + beta * p[i];
  }
}

__global__ void jacobi_kernel(int64_t n, const double* r, const double* diag, double* z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = r[i] / diag[i];
}

}  // namespace

hipError_t launch_gemm_bf16(const GemmArgs& g, hipStream_t s) {
  const int tiles = (g.M / 16) * (g.N / 16);
  if (tiles == 0) return hipSuccess;
  const int slices = g.epi == kEpiPartial ? (g.K + g.ksplit - 1) / g.ksplit : 1;
  const int blocks = ((g.M + kGemmBlk - 1) / kGemmBlk) * ((g.N + kGemmBlk - 1) / kGemmBlk);
  // LDS blocks for products of at least two blocks per CU without split K
  // (the training's forward products on the 48^3 cube: 15 against 40 us);
  // one wave per tile for the smaller ones and the split-K gradient
  // products, where it was faster.  IMEX_GEMM_TILES=1 / IMEX_GEMM_BLOCKS=1
  // force either form (they give the same bits).
  bool lds = g.epi != kEpiPartial && blocks >= 512;
  if (const char* v = std::getenv("IMEX_GEMM_TILES"); v && v[0] == '1') lds = false;
  if (const char* v = std::getenv("IMEX_GEMM_BLOCKS"); v && v[0] == '1') lds = true;
  if (lds)
    hipLaunchKernelGGL(gemm_bf16_lds_kernel, dim3((unsigned)blocks, (unsigned)slices), dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL(gemm_bf16_kernel, dim3((unsigned)((tiles + 3) / 4), (unsigned)slices), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_sum_slices(const float* part, int slices, int64_t n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_slices_kernel, grid1d(n, 256), dim3(256), 0, s, part, slices, n, out);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* m, int64_t rows, int cols, float* work, float* out, hipStream_t s) {
  const int chunks = (int)((rows + 255) / 256);
  if (chunks == 0) return hipSuccess;
  hipLaunchKernelGGL(colsum_stage1, dim3((unsigned)chunks, (unsigned)((cols + 255) / 256)), dim3(256), 0, s, m, rows,
                     cols, work);
  hipLaunchKernelGGL(colsum_stage2, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, s, work, chunks, cols, out);
  return hipGetLastError();
}

hipError_t launch_mlp_features(const ElemArgs& L, const MlpDims& d, const double* R, const double* BR, const int* vsel,
                               int n_vec, int rows_pad, uint16_t* X, double* s, float* valid, hipStream_t st) {
  hipLaunchKernelGGL(mlp_features_kernel, dim3((unsigned)((rows_pad + 3) / 4)), dim3(256), 0, st, L, d, R, BR, vsel,
                     n_vec, rows_pad, X, s, valid);
  return hipGetLastError();
}

hipError_t launch_mlp_targets(const ElemArgs& L, const MlpDims& d, const double* Xs, const double* BR, const int* vsel,
                              int n_vec, int rows_pad, const double* s, float* valid, float* T, hipStream_t st) {
  if (n_vec > 0)
    hipLaunchKernelGGL(mlp_train_rows_kernel, dim3((unsigned)n_vec), dim3(256), 0, st, L.E, n_vec, rows_pad, s, valid);
  hipLaunchKernelGGL(mlp_targets_kernel, dim3((unsigned)((rows_pad + 3) / 4)), dim3(256), 0, st, L, d, Xs, BR, vsel,
                     n_vec, rows_pad, s, valid, T);
  return hipGetLastError();
}

hipError_t launch_rsub(const double* x, double* y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(rsub_kernel, grid1d(n, 256), dim3(256), 0, st, x, y, n);
  return hipGetLastError();
}

hipError_t launch_mlp_loss(const MlpDims& d, int ne, int rows_pad, const float* Y, const float* T, const float* valid,
                           float inv_count, float* dY, uint16_t* dYb, double* partial, int* n_partial,
                           hipStream_t st) {
  const int blocks = (rows_pad + 3) / 4;
  *n_partial = blocks;
  hipLaunchKernelGGL(mlp_loss_kernel, dim3((unsigned)blocks), dim3(256), 0, st, d, ne, rows_pad, Y, T, valid,
                     inv_count, dY, dYb, partial);
  return hipGetLastError();
}

hipError_t launch_mlp_scatter(const ElemArgs& L, const MlpDims& d, const double* s, const float* Y, double* z,
                              hipStream_t st) {
  hipLaunchKernelGGL(mlp_scatter_kernel, grid1d(L.nc, 256), dim3(256), 0, st, L, d, s, Y, z);
  return hipGetLastError();
}

hipError_t launch_combine(const CsrDev& S, const double* r, const double* br, const double* c, double* q1,
                          double* q2, double* part, double* sc, double* z, hipStream_t st) {
  hipLaunchKernelGGL(fcg_spmv_kernel, dim3(kFcgBlocks), dim3(256), 0, st, S, br, q1, part);
  hipLaunchKernelGGL(fcg_reduce_kernel, dim3(1), dim3(256), 0, st, part, sc, 0);
  hipLaunchKernelGGL(fcg_spmv_kernel, dim3(kFcgBlocks), dim3(256), 0, st, S, c, q2, part);
  hipLaunchKernelGGL(fcg_reduce_kernel, dim3(1), dim3(256), 0, st, part, sc, 1);
  hipLaunchKernelGGL(combine_dots_kernel, dim3(kFcgBlocks), dim3(256), 0, st, S.n, br, q2, c, r, part);
  hipLaunchKernelGGL(fcg_reduce_kernel, dim3(3), dim3(256), 0, st, part, sc, 2);
  hipLaunchKernelGGL(combine_kernel, grid1d(S.n, 256), dim3(256), 0, st, S.n, sc, br, c, z);
  return hipGetLastError();
}

hipError_t launch_block_precond(const ElemArgs& L, const double* r, double* ze, double* z, hipStream_t st) {
  hipLaunchKernelGGL(block_apply_kernel, dim3((unsigned)((L.E + 3) / 4)), dim3(256), 0, st, L, r, ze);
  hipLaunchKernelGGL(block_scatter_kernel, grid1d(L.nc, 256), dim3(256), 0, st, L, ze, z);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, uint16_t* pb, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, grid1d(n, 256), dim3(256), 0, st, p, m, v, g, n, lr, b1, b2, eps, c1, c2, pb);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(to_bf16_kernel, grid1d(n, 256), dim3(256), 0, st, x, y, n);
  return hipGetLastError();
}

hipError_t launch_fcg_init(const CsrDev& S, const double* b, const double* x, double* r, double* part,
                           hipStream_t st) {
  hipLaunchKernelGGL(fcg_init_kernel, dim3(kFcgBlocks), dim3(256), 0, st, S, b, x, r, part);
  return hipGetLastError();
}
hipError_t launch_fcg_spmv(const CsrDev& S, const double* p, double* q, double* part, hipStream_t st) {
  hipLaunchKernelGGL(fcg_spmv_kernel, dim3(kFcgBlocks), dim3(256), 0, st, S, p, q, part);
  return hipGetLastError();
}
hipError_t launch_fcg_update(int64_t n, const double* sc, double* x, double* r, double* r_old, const double* p,
                             const double* q, double* part, hipStream_t st) {
  hipLaunchKernelGGL(fcg_update_kernel, dim3(kFcgBlocks), dim3(256), 0, st, n, sc, x, r, r_old, p, q, part);
  return hipGetLastError();
}
hipError_t launch_fcg_dots(int64_t n, const double* z, const double* r, const double* r_old, const double* diag,
                           double* part, hipStream_t st) {
  hipLaunchKernelGGL(fcg_dots_kernel, dim3(kFcgBlocks), dim3(256), 0, st, n, z, r, r_old, diag, part);
  return hipGetLastError();
}
hipError_t launch_fcg_reduce(const double* part, int k, double* sc, int dst, hipStream_t st) {
  hipLaunchKernelGGL(fcg_reduce_kernel, dim3((unsigned)k), dim3(256), 0, st, part, sc, dst);
  return hipGetLastError();
}
hipError_t launch_fcg_scalars(double* sc, int which, hipStream_t st) {
  hipLaunchKernelGGL(fcg_scalars_kernel, dim3(1), dim3(64), 0, st, sc, which);
  return hipGetLastError();
}
hipError_t launch_fcg_direction(int64_t n, const double* sc, const double* z, const double* r, const double* diag,
                                double* p, int start, hipStream_t st) {
  hipLaunchKernelGGL(fcg_direction_kernel, dim3(kFcgBlocks), dim3(256), 0, st, n, sc, z, r, diag, p, start);
  return hipGetLastError();
}
hipError_t launch_jacobi(int64_t n, const double* r, const double* diag, double* z, hipStream_t st) {
  hipLaunchKernelGGL(jacobi_kernel, grid1d(n, 256), dim3(256), 0, st, n, r, diag, z);
  return hipGetLastError();
}

}  // namespace imex
