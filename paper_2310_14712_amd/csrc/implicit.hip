// HIP kernels (gfx950) of the implicit part of the Newmark IMEX step: the
// predictor and right-hand side of the cut block, the dissected Cholesky
// solve of S a^c = rhs (parts, separator systems, correction) and the
// trapezoidal corrector.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "device.h"

namespace imex {

namespace {

using namespace dev;


// ---------------------------------------------------------------------------
// implicit part
// ---------------------------------------------------------------------------
// rhs_i = f_t(t_{n+1}) f_x^c_i - K^cd_i u^d_{n+1} - K^cc_i (u^c + dt v^c + (1/2 - beta) dt^2 a^c):
// L lanes per row (L = 16 or 32: four or two rows per wave); each lane
// keeps the index, value and gather loads of up to four entries of both
// segments in flight.
// the predictor u + dt v + (1/2 - beta) dt^2 a of one c dof, with its
// multiply-adds written out (the per-entry and the first-pass forms agree
// bit for bit)
// Values read once per step (the K^c entries, the factor): non-temporal
// loads, so that they do not evict the two grid buffers, which the next
// step's explicit kernel reads again (a step streams about five times the
// grid's bytes through the caches).  Column indices keep the default policy.
__device__ inline double stream_load(const double* p) { return __builtin_nontemporal_load(p); }

__device__ inline double predict(double u, double v, double a, double dt, double q) {
  return fma(q, a, fma(dt, v, u));
}

__global__ __launch_bounds__(kThreads) void predict_kernel(const RhsArgs A) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < A.nc) A.pred[i] = predict(A.uc[i], A.vc[i], A.ac[i], A.dt, A.qp);
}

template <typename T, int L, bool PRED>
__device__ __forceinline__ void rhs_body(const RhsArgs& A, int blk) {
  constexpr int U = 4, RPW = 64 / L;
  const int lane = threadIdx.x & 63, sub = lane & (L - 1);
  const int64_t row = ((int64_t)blk * (kThreads / 64) + (threadIdx.x >> 6)) * RPW + lane / L;
  const bool live = row < A.nc;
  const T* ug = static_cast<const T*>(A.ugrid);
  const double dt = A.dt, q = A.qp;
  int64_t d0 = 0, d1 = 0, c0 = 0, c1 = 0;
  if (live) {
    d0 = A.rp_d[row];
    d1 = A.rp_d[row + 1];
    c0 = A.rp_c[row];
    c1 = A.rp_c[row + 1];
  }
  double acc_d = 0.0, acc_c = 0.0;
  for (int64_t base = sub;; base += L * U) {
    const bool more = d0 + base < d1 || c0 + base < c1;
    if (!__any(more)) break;
    int32_t jd[U], jc[U];
    double vd[U], vc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t kd = d0 + base + L * u, kc = c0 + base + L * u;
      jd[u] = 0;
      jc[u] = 0;
      vd[u] = 0.0;
      vc[u] = 0.0;
      if (kd < d1) {
        jd[u] = A.col_d[kd];
        vd[u] = stream_load(&A.val_d[kd]);
      }
      if (kc < c1) {
        jc[u] = A.col_c[kc];
        vc[u] = stream_load(&A.val_c[kc]);
      }
    }
    double ud[U], uu[U], uv[U], ua[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ud[u] = 0.0;
      uu[u] = 0.0;
      uv[u] = 0.0;
      ua[u] = 0.0;
      if (d0 + base + L * u < d1) ud[u] = to_d(ug[jd[u]]);
      if (c0 + base + L * u < c1) {
        if constexpr (PRED) {
          uu[u] = A.pred[jc[u]];
        } else {
          uu[u] = A.uc[jc[u]];
          uv[u] = A.vc[jc[u]];
          ua[u] = A.ac[jc[u]];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc_d += vd[u] * ud[u];
      acc_c += vc[u] * (PRED ? uu[u] : predict(uu[u], uv[u], ua[u], dt, q));
    }
  }
  double acc = reduce16(acc_d + acc_c);
  if constexpr (L == 32) acc += __shfl_xor(acc, 16, 64);
  if (sub == 0 && live) A.rhs[row] = A.ft[A.step[0] + 1] * A.fxc[row] - acc;
}

template <typename T, int L, bool PRED>
__global__ __launch_bounds__(kThreads) void rhs_kernel(const RhsArgs A) {
  rhs_body<T, L, PRED>(A, blockIdx.x);
}
template <typename T, int L>
__global__ __launch_bounds__(kThreads) void rhs_batch_kernel(const BatchTable<RhsArgs> B) {
  const int i = batch_instance(B.first, B.n, blockIdx.x);
  rhs_body<T, L, false>(B.args[i], blockIdx.x - B.first[i]);
}

// Forward and backward substitution with one envelope Cholesky factor
// ("chain"), in place on xs (length m, LDS).  Rows are processed in blocks of
// kBlk: z_b = x_b - L_{b,left} y_left (envelope rows), y_b = D_b z_b with D_b
// the inverse of the diagonal block (lower triangle packed by columns);
// backward z_b = y_b - L_{below,b}^T x_below (envelope rows below the block),
// x_b = D_b^T z_b, reading D_b by columns.  Thread mapping: each of
// the 4 waves handles 8 rows of a block with 8 lanes per row (shuffle
// reductions), so a block costs two workgroup barriers.
__device__ __attribute__((always_inline)) inline void chain_solve(const double* V, const int32_t* I, int m, int nb,
                                                                 int nnz, double* xs, double* zsh) {
  const int tid = threadIdx.x;
  const int r = (tid >> 6) * 8 + ((tid & 63) >> 3);
  const int sub = tid & 7;
  const double* L = V;
  const double* Dc = V + nnz;
  const int32_t* first = I;
  const int32_t* rowoff = I + m;
  const int32_t* rmax = I + 2 * m;
  for (int b = 0; b < nb; ++b) {
    const int row0 = b * kBlk;
    const int nr = min(kBlk, m - row0);
    double part = 0.0;
    if (r < nr) {
      const int i = row0 + r;
      const int f = first[i];
      const double* Li = L + rowoff[i] - f;
      int j = f + sub;
      for (; j + 24 < row0; j += 32) {
        const double l0 = Li[j], l1 = Li[j + 8], l2 = Li[j + 16], l3 = Li[j + 24];
        part += l0 * xs[j] + l1 * xs[j + 8] + l2 * xs[j + 16] + l3 * xs[j + 24];
      }
      for (; j < row0; j += 8) part += Li[j] * xs[j];
    }
    part = reduce8(part);
    if (sub == 0) zsh[r] = (r < nr) ? xs[row0 + r] - part : 0.0;
    __syncthreads();
    const double* Db = Dc + (size_t)b * kTri;
    part = 0.0;
    for (int j = sub; j <= r; j += 8) part += Db[j * kBlk - (j * (j - 1)) / 2 + (r - j)] * zsh[j];
    part = reduce8(part);
    if (sub == 0 && r < nr) xs[row0 + r] = part;
    __syncthreads();
  }
  for (int b = nb - 1; b >= 0; --b) {
    const int row0 = b * kBlk;
    const int nr = min(kBlk, m - row0);
    const int rend = row0 + nr;
    double part = 0.0;
    if (r < nr) {
      const int col = row0 + r;
      const int rm = rmax[b];
      for (int j = rend + sub; j <= rm; j += 8) {
        const int f = first[j];
        if (col >= f) part += L[rowoff[j] + col - f] * xs[j];
      }
    }
    part = reduce8(part);
    if (sub == 0) zsh[r] = (r < nr) ? xs[row0 + r] - part : 0.0;
    __syncthreads();
    const double* Db = Dc + (size_t)b * kTri;
    const double* Dcol = Db + r * kBlk - (r * (r - 1)) / 2 - r;  // column r: D(j, r) = Dcol[j], j >= r
    part = 0.0;
    for (int j = r + sub; j < kBlk; j += 8) part += Dcol[j] * zsh[j];
    part = reduce8(part);
    if (sub == 0 && r < nr) xs[row0 + r] = part;
    __syncthreads();
  }
}

// Stage a chain's values and metadata into LDS behind xs when they fit; the
// copy keeps 16 loads per thread in flight.
template <typename X>
__device__ inline void copy_to_lds(X* dst, const X* src, size_t n) {
  constexpr int U = 16;
  for (size_t base = threadIdx.x; base < n; base += (size_t)kThreads * U) {
    X t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t k = base + (size_t)u * kThreads;
      t[u] = k < n ? src[k] : X(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t k = base + (size_t)u * kThreads;
      if (k < n) dst[k] = t[u];
    }
  }
}

__device__ inline bool stage_chain(const ChainMeta& cm, const double* vals, const int32_t* ints, double* sm,
                                   int64_t smem_bytes, const double** V, const int32_t** I) {
  const int m = cm.nrows;
  const size_t nv = (size_t)cm.nnz + (size_t)cm.nblocks * kTri;
  const size_t ni = 2 * (size_t)m + cm.nblocks;
  *V = vals + cm.voff;
  *I = ints + cm.ioff;
  int32_t* Is = reinterpret_cast<int32_t*>(sm + m);
  copy_to_lds(Is, *I, ni);
  *I = Is;
  const size_t ioff = (ni * sizeof(int32_t) + sizeof(double) - 1) / sizeof(double);
  if ((int64_t)((m + ioff + nv) * sizeof(double)) <= smem_bytes) {
    double* Vs = sm + m + ioff;
    copy_to_lds(Vs, *V, nv);
    *V = Vs;
    return true;
  }
  return false;
}

// The c state of one row, loaded ahead of the acceleration it is corrected
// with so that its loads overlap the solve.
struct CState {
  double a0, v0, u0;
  int64_t node;
};
__device__ inline CState load_cstate(const SolveArgs& A, int64_t i) {
  return CState{A.ac[i], A.vc[i], A.uc[i], A.c_nodes[i]};
}

template <typename T>
__device__ inline void correct_loaded(const SolveArgs& A, int64_t i, const CState& cs, double an) {
  const double dt = A.dt;
  const double a0 = cs.a0, v0 = cs.v0, u0 = cs.u0;
  const double up = u0 + dt * v0 + A.qp * a0;
  const double vp = v0 + 0.5 * dt * a0;
  const double un = up + A.qc * an;
  A.uc[i] = un;
  A.vc[i] = vp + 0.5 * dt * an;
  A.ac[i] = an;
  static_cast<T*>(A.ugrid)[cs.node] = T(un);
}

template <typename T>
__device__ inline void correct_row(const SolveArgs& A, int64_t i, double an) {
  correct_loaded<T>(A, i, load_cstate(A, i), an);
}

// corrector of every c row from a given acceleration (iterative solvers)
template <typename T>
__global__ void correct_all_kernel(const SolveArgs A, const double* an, int64_t nc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nc) correct_row<T>(A, i, an[i]);
  if (A.advance_step && i == 0) A.step[0] = A.step[0] + 1;
}

// w_p = A_pp^-1 r_p for one part, and its contribution A_Sp w_p to the
// adjacent separator rows
__global__ __launch_bounds__(kThreads) void part_solve_kernel(const SolveArgs A) {
  extern __shared__ double sm[];
  __shared__ double zsh[kBlk];
  const ChainMeta cm = A.parts[blockIdx.x];
  double* xs = sm;
  for (int i = threadIdx.x; i < cm.nrows; i += kThreads) xs[i] = A.rhs[cm.row0 + i];
  const double* V;
  const int32_t* I;
  const bool staged = stage_chain(cm, A.vals, A.ints, sm, A.smem_part, &V, &I);
  __syncthreads();
  if (staged) {
    const size_t ioff = ((2 * (size_t)cm.nrows + cm.nblocks) * sizeof(int32_t) + sizeof(double) - 1) / sizeof(double);
    chain_solve(sm + cm.nrows + ioff, reinterpret_cast<const int32_t*>(sm + cm.nrows), cm.nrows, cm.nblocks,
                cm.nnz, xs, zsh);
  } else {
    chain_solve(A.vals + cm.voff, reinterpret_cast<const int32_t*>(sm + cm.nrows), cm.nrows, cm.nblocks, cm.nnz,
                xs, zsh);
  }
  for (int i = threadIdx.x; i < cm.nrows; i += kThreads) A.w[cm.row0 + i] = xs[i];
  if (cm.nadj > 0) {
    const int32_t* ptr = A.cp_ptr + A.cp_rowptr[blockIdx.x];
    const int sub = threadIdx.x & 7;
    for (int row = threadIdx.x >> 3; row < ((cm.nadj + 31) / 32) * 32; row += kThreads / 8) {
      double acc = 0.0;
      if (row < cm.nadj)
        for (int k = ptr[row] + sub; k < ptr[row + 1]; k += 8) acc += A.cp_val[k] * xs[A.cp_col[k]];
      acc = reduce8(acc);
      if (sub == 0 && row < cm.nadj) A.cbuf[cm.coff + row] = acc;
    }
  }
}

// Dense form of the part stage: one wave per row of A_pp^-1 (w_p = A_pp^-1 r_p)
// or per column of Z_p (the coupling A_Sp w_p = Z_p^T r_p); a workgroup takes
// four consecutive rows of one chunk of 16.  NT (the batched kernels, whose
// instances stream far more than the caches hold): the dense values are
// read non-temporally, so that the instances' grids stay cached; a single
// plate's solve fits in the caches, where the hint slowed it.
template <bool NT>
__device__ __forceinline__ void part_dense_body(const SolveArgs& A, int blk) {
  const DenseChunk dc = A.pd_chunks[blk >> 2];
  const int r = (int)(blk & 3) * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  const double* M = (dc.kind == 0 ? A.pinv : A.zvals) + dc.moff + (int64_t)r * dc.n;
  double acc = 0.0;
  if (r < dc.rows) acc = row_dot<64, 16, NT>(M, A.rhs + dc.x0, dc.n, lane);
  acc = reduce64(acc);
  if (lane == 0 && r < dc.rows) (dc.kind == 0 ? A.w : A.cbuf)[dc.out0 + r] = acc;
}

__global__ __launch_bounds__(kThreads) void part_dense_kernel(const SolveArgs A) {
  part_dense_body<false>(A, blockIdx.x);
}
__global__ __launch_bounds__(kThreads) void part_dense_batch_kernel(const BatchTable<SolveArgs> B) {
  const int i = batch_instance(B.first, B.n, blockIdx.x);
  part_dense_body<true>(B.args[i], blockIdx.x - B.first[i]);
}

// Parts above 1024 rows keep only the lower triangle of the symmetric A_pp^-1,
// in 64 x 64 blocks (I >= J, row-major, zero-padded), which halves what the
// part stage reads.  One workgroup per stored block B = (A_pp^-1)_{IJ}:
// u = B x_J goes to block row I and, off the diagonal, v = B^T x_I to block
// row J, each into its own slot of the part's partial-sum array
// (partial[I][J][0..63] receives the contribution of block column J to block
// row I); part_sym_sum_kernel adds the slots in a fixed order.
constexpr int kSymB = 64;
__global__ __launch_bounds__(kThreads) void part_sym_kernel(const SolveArgs A) {
  constexpr int ROWS = kSymB / (kThreads / 64);  // rows of the block per wave
  __shared__ double vsum[kThreads / 64][kSymB];
  const SymBlock sb = A.sym_blocks[blockIdx.x];
  const int n = sb.n, I = sb.I, J = sb.J;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double* B = A.pinv + sb.boff;
  const double* x = A.rhs + sb.row0;
  const int cj = J * kSymB + lane;
  const double xj = cj < n ? x[cj] : 0.0;
  double b[ROWS];
#pragma unroll
  for (int t = 0; t < ROWS; ++t) b[t] = B[(wv + 4 * t) * kSymB + lane];  // a row per wave load
  double v = 0.0;
#pragma unroll
  for (int t = 0; t < ROWS; ++t) {
    const int ri = I * kSymB + wv + 4 * t;
    v += b[t] * (ri < n ? x[ri] : 0.0);
  }
  // the wave's 16 row sums of B x_J by a reduce-scatter over the lanes:
  // each exchange halves the rows a lane keeps (17 exchanges instead of 16
  // full reductions of 6); lane l ends with row 8 l5 + 4 l4 + 2 l3 + l2
  static_assert(ROWS == 16, "the reduce-scatter assumes 16 rows per wave");
  double q8[8], q4[4], q2[2];
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8, h2 = lane & 4;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double lo = b[k] * xj, hi = b[8 + k] * xj;
    q8[k] = (h5 ? hi : lo) + __shfl_xor(h5 ? lo : hi, 32, 64);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) q4[k] = (h4 ? q8[4 + k] : q8[k]) + __shfl_xor(h4 ? q8[k] : q8[4 + k], 16, 64);
#pragma unroll
  for (int k = 0; k < 2; ++k) q2[k] = (h3 ? q4[2 + k] : q4[k]) + __shfl_xor(h3 ? q4[k] : q4[2 + k], 8, 64);
  double q = (h2 ? q2[1] : q2[0]) + __shfl_xor(h2 ? q2[0] : q2[1], 4, 64);
  q += __shfl_xor(q, 2, 64);
  q += __shfl_xor(q, 1, 64);
  if ((lane & 3) == 0) {
    const int t = (h5 ? 8 : 0) + (h4 ? 4 : 0) + (h3 ? 2 : 0) + (h2 ? 1 : 0);
    A.sym_partial[sb.prow + wv + 4 * t] = q;
  }
  if (I != J) {  // uniform over the workgroup
    vsum[wv][lane] = v;
    __syncthreads();
    if (wv == 0)
      A.sym_partial[sb.pcol + lane] = ((vsum[0][lane] + vsum[1][lane]) + vsum[2][lane]) + vsum[3][lane];
  }
}

// w_p rows of one 64-row chunk: the sum of the chunk's partial slots over the
// block columns, in increasing order
__global__ __launch_bounds__(kSymB) void part_sym_sum_kernel(const SolveArgs A) {
  const int64_t part = A.part_chunks[2 * blockIdx.x], r0 = A.part_chunks[2 * blockIdx.x + 1];
  const ChainMeta cm = A.parts[part];
  const int n = cm.nrows, nbk = (n + kSymB - 1) / kSymB, I = (int)(r0 / kSymB);
  const int r = (int)r0 + threadIdx.x;
  if (r >= n) return;
  const double* ps = A.sym_partial + A.sym_poff[part] + (int64_t)I * nbk * kSymB + threadIdx.x;
  double y = 0.0;
  for (int Jc = 0; Jc < nbk; ++Jc) y += ps[(int64_t)Jc * kSymB];
  A.w[cm.row0 + r] = y;
}

// Wide form of the coupling: A_Sp w_p for the separator rows of one chunk of
// 16 (the same quantity as Z_p^T r_p, since Z_p = A_pp^-1 A_pS and A_pp^-1 is
// symmetric), from the sparse A_Sp and the w_p just formed instead of the
// dense Z_p: 16 lanes per row, four entries per lane in flight.
__global__ __launch_bounds__(kThreads) void part_coupling_kernel(const SolveArgs A) {
  const int64_t chunk = blockIdx.x;
  const int64_t part = A.dense_chunks[3 * chunk + 1], first = A.dense_chunks[3 * chunk + 2];
  const ChainMeta cm = A.parts[part];
  const int row = (int)first + (threadIdx.x >> 4), sub = threadIdx.x & 15;
  const bool ok = row < cm.nadj && row < first + 16;
  const int32_t* ptr = A.cp_ptr + A.cp_rowptr[part];
  const double* w = A.w + cm.row0;
  double acc = 0.0;
  if (ok) {
    const int end = ptr[row + 1];
    for (int base = ptr[row] + sub; base < end; base += 64) {
      int32_t cj[4];
      double cv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = base + 16 * u;
        cj[u] = k < end ? A.cp_col[k] : 0;
        cv[u] = k < end ? A.cp_val[k] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += cv[u] * w[cj[u]];
    }
  }
  acc = reduce16(acc);
  if (sub == 0 && ok) A.cbuf[cm.coff + row] = acc;
}

// x_S = Sigma^-1 (r_S - sum_p A_Sp w_p): one wave per row of one component's
// Sigma^-1 (four rows per workgroup); corrects those separator rows.  NT as
// in the part stage.
template <typename T, bool NT>
__device__ __forceinline__ void schur_body(const SolveArgs& A, int blk) {
  extern __shared__ double rs[];  // r_S of the component (smem_sep bytes)
  const SepChunk sc = A.sep_chunks[blk >> 2];
  const int m = sc.m;
  const int r = (int)(blk & 3) * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int row = sc.first + r;
  const bool ok = r < sc.rows;
  // this wave's row of Sigma^-1 (its first kPre * 64 entries) and the row's
  // c state are loaded while the right-hand side is formed
  constexpr int kPre = 8;
  const double* Mrow = A.schur_inv + sc.moff + (int64_t)r * m;
  double mv[kPre];
#pragma unroll
  for (int u = 0; u < kPre; ++u) {
    const int t = lane + 64 * u;
    mv[u] = (ok && t < m) ? (NT ? stream_load(&Mrow[t]) : Mrow[t]) : 0.0;
  }
  CState cs{};
  if (ok && lane == 0) cs = load_cstate(A, sc.row0 + row);
  for (int s = threadIdx.x; s < m; s += kThreads) {
    const int64_t i = sc.row0 + s;
    const int64_t s0 = A.sep_src[2 * i], s1 = A.sep_src[2 * i + 1];
    const double c0 = s0 >= 0 ? A.cbuf[s0] : 0.0, c1 = s1 >= 0 ? A.cbuf[s1] : 0.0;
    rs[s] = A.rhs[i] - c0 - c1;
  }
  __syncthreads();
  // the same summation order as a row_dot<64, kPre> over the whole row
  double acc = 0.0;
  if (ok) {
    double xv[kPre];
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      const int t = lane + 64 * u;
      xv[u] = t < m ? rs[t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPre; ++u) acc += mv[u] * xv[u];
    if (m > 64 * kPre)
      acc += row_dot<64, kPre, NT>(Mrow + 64 * kPre, (const double*)rs + 64 * kPre, m - 64 * kPre, lane);
  }
  acc = reduce64(acc);
  if (lane == 0 && ok) {
    A.w[sc.row0 + row] = acc;
    correct_loaded<T>(A, sc.row0 + row, cs, acc);
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void schur_kernel(const SolveArgs A) {
  schur_body<T, false>(A, blockIdx.x);
}
template <typename T>
__global__ __launch_bounds__(kThreads) void schur_batch_kernel(const BatchTable<SolveArgs> B) {
  const int i = batch_instance(B.first, B.n, blockIdx.x);
  schur_body<T, true>(B.args[i], blockIdx.x - B.first[i]);
}

// Wide form of the separator stage (3D meshes, separator systems of
// thousands of rows): r_S - sum_p A_Sp w_p is formed once per row here
// instead of once per workgroup, so that the products below need no LDS
// copy of it.  Four chunks of 16 rows per workgroup.
__global__ __launch_bounds__(64) void schur_rs_kernel(const SolveArgs A, int64_t n_chunks) {
  const int64_t chunk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 4);
  if (chunk >= n_chunks) return;
  const int64_t comp = A.schur_chunks[2 * chunk], r0 = A.schur_chunks[2 * chunk + 1];
  const ChainMeta cm = A.schur[comp];
  const int s = (int)r0 + (threadIdx.x & 15);
  if (s >= cm.nrows) return;
  const int64_t i = cm.row0 + s;
  const int64_t s0 = A.sep_src[2 * i], s1 = A.sep_src[2 * i + 1];
  const double c0 = s0 >= 0 ? A.cbuf[s0] : 0.0, c1 = s1 >= 0 ? A.cbuf[s1] : 0.0;
  A.rs[i] = A.rhs[i] - c0 - c1;
}

// x_S = Sigma^-1 r_S for a 16-row chunk: each wave four rows with the loads
// of all four in flight and every load of r_S shared; corrects those rows.
template <typename T>
__global__ __launch_bounds__(kThreads) void schur_wide_kernel(const SolveArgs A) {
  constexpr int R = 4, PER = 4;
  const int64_t chunk = blockIdx.x;
  const int64_t comp = A.schur_chunks[2 * chunk], first = A.schur_chunks[2 * chunk + 1];
  const ChainMeta cm = A.schur[comp];
  const int m = cm.nrows;
  const int lane = threadIdx.x & 63, r0 = (int)first + (threadIdx.x >> 6) * R;
  const int nout = (int)min((int64_t)m, first + 16);
  const double* M = A.schur_inv + cm.voff;
  const double* x = A.rs + cm.row0;
  CState cs[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (lane == 0 && r0 + r < nout) cs[r] = load_cstate(A, cm.row0 + r0 + r);
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  for (int base = 0; base < m; base += 64 * PER) {
    double xv[PER], mv[R][PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = base + lane + 64 * u;
      xv[u] = t < m ? x[t] : 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) mv[r][u] = (r0 + r < nout && t < m) ? M[(int64_t)(r0 + r) * m + t] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < PER; ++u) acc[r] += mv[r][u] * xv[u];
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double v = reduce64(acc[r]);
    if (lane == 0 && r0 + r < nout) {
      A.w[cm.row0 + r0 + r] = v;
      correct_loaded<T>(A, cm.row0 + r0 + r, cs[r], v);
    }
  }
}

// Separator systems in chain form (large components): one workgroup per
// component solves Sigma x_S = r_S - sum_p A_Sp w_p with the envelope chain
// and corrects the separator rows.
template <typename T>
__global__ __launch_bounds__(kThreads) void schur_chain_kernel(const SolveArgs A) {
  extern __shared__ double sm[];
  __shared__ double zsh[kBlk];
  const ChainMeta cm = A.schur[A.schur_chain[blockIdx.x]];
  const size_t ioff = ((2 * (size_t)cm.nrows + cm.nblocks) * sizeof(int32_t) + sizeof(double) - 1) / sizeof(double);
  // the solution vector lives in LDS when it fits with the metadata, else in
  // the global solution array (rows of this separator system)
  const bool in_lds = (int64_t)((cm.nrows + ioff) * sizeof(double)) <= A.smem_schur;
  double* xg = A.w + cm.row0;
  for (int s = threadIdx.x; s < cm.nrows; s += kThreads) {
    const int64_t i = cm.row0 + s;
    const int64_t s0 = A.sep_src[2 * i], s1 = A.sep_src[2 * i + 1];
    const double c0 = s0 >= 0 ? A.cbuf[s0] : 0.0, c1 = s1 >= 0 ? A.cbuf[s1] : 0.0;
    const double v = A.rhs[i] - c0 - c1;
    if (in_lds) sm[s] = v;
    else xg[s] = v;
  }
  if (in_lds) {
    const double* V;
    const int32_t* I;
    const bool staged = stage_chain(cm, A.vals, A.ints, sm, A.smem_schur, &V, &I);
    __syncthreads();
    if (staged)
      chain_solve(sm + cm.nrows + ioff, reinterpret_cast<const int32_t*>(sm + cm.nrows), cm.nrows, cm.nblocks,
                  cm.nnz, sm, zsh);
    else
      chain_solve(A.vals + cm.voff, reinterpret_cast<const int32_t*>(sm + cm.nrows), cm.nrows, cm.nblocks, cm.nnz,
                  sm, zsh);
  } else {
    __syncthreads();
    chain_solve(A.vals + cm.voff, A.ints + cm.ioff, cm.nrows, cm.nblocks, cm.nnz, xg, zsh);
  }
  for (int s = threadIdx.x; s < cm.nrows; s += kThreads) {
    const double a = in_lds ? sm[s] : xg[s];
    A.w[cm.row0 + s] = a;
    correct_row<T>(A, cm.row0 + s, a);
  }
}

// x_p = w_p - Z_p x_S(adjacent separators): one workgroup of 16 waves per
// 64-row chunk, lane = row, so that every load of the column-major Z_p is a
// contiguous 512-byte segment; wave v takes the columns k = v mod 16, and the
// partial sums are added in wave order.  Corrects those part rows.  NT as in
// the part stage.
constexpr int kCorrectWaves = 16;
template <typename T, bool NT>
__device__ __forceinline__ void part_correct_body(const SolveArgs& A, int blk) {
  __shared__ double part_sum[kCorrectWaves][64];
  const CorrChunk ch = A.part_corr[blk];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool ok = lane < ch.rows;
  // the first wave's rows: solution of the part system and c state, ahead
  CState cs{};
  double wi = 0.0;
  if (wv == 0 && ok) {
    cs = load_cstate(A, ch.row + lane);
    wi = A.w[ch.row + lane];
  }
  double x = 0.0;
  if (ok) {
    const double* Zi = A.zvals + ch.z + lane;
    const double* xs = A.w + ch.adj0;
    constexpr int U = 8;
    for (int base = wv; base < ch.na; base += kCorrectWaves * U) {
      double zv[U], xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = base + kCorrectWaves * u;
        zv[u] = k < ch.na ? (NT ? stream_load(&Zi[(int64_t)k * ch.ld]) : Zi[(int64_t)k * ch.ld]) : 0.0;
        xv[u] = k < ch.na ? xs[k] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) x += zv[u] * xv[u];
    }
  }
  part_sum[wv][lane] = x;
  __syncthreads();
  if (wv == 0 && ok) {
    double z = part_sum[0][lane];
#pragma unroll
    for (int v = 1; v < kCorrectWaves; ++v) z += part_sum[v][lane];
    correct_loaded<T>(A, ch.row + lane, cs, wi - z);
  }
  if (A.advance_step && blk == 0 && threadIdx.x == 0) A.step[0] = A.step[0] + 1;
}

template <typename T>
__global__ __launch_bounds__(64 * kCorrectWaves) void part_correct_kernel(const SolveArgs A) {
  part_correct_body<T, false>(A, blockIdx.x);
}
template <typename T>
__global__ __launch_bounds__(64 * kCorrectWaves) void part_correct_batch_kernel(const BatchTable<SolveArgs> B) {
  const int i = batch_instance(B.first, B.n, blockIdx.x);
  part_correct_body<T, true>(B.args[i], blockIdx.x - B.first[i]);
}

// Wide form of the correction: x_p = w_p - Z_p x_S with Z_p row-major, one
// workgroup per 16-row chunk, each wave four rows with the loads of all four
// in flight and every load of x_S shared; corrects those part rows.
template <typename T>
__global__ __launch_bounds__(kThreads) void part_correct_wide_kernel(const SolveArgs A) {
  constexpr int R = 4, PER = 4;
  const CorrChunk ch = A.corr_chunks[blockIdx.x];
  const int na = ch.na, nout = ch.rows;
  const int lane = threadIdx.x & 63, r0 = (threadIdx.x >> 6) * R;  // rows local to the chunk
  const double* Z = A.zvals + ch.z;
  const double* xs = A.w + ch.adj0;
  CState cs[R];
  double wi[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    wi[r] = 0.0;
    if (lane == 0 && r0 + r < nout) {
      cs[r] = load_cstate(A, ch.row + r0 + r);
      wi[r] = A.w[ch.row + r0 + r];
    }
  }
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  for (int base = 0; base < na; base += 64 * PER) {
    double xv[PER], mv[R][PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = base + lane + 64 * u;
      xv[u] = t < na ? xs[t] : 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) mv[r][u] = (r0 + r < nout && t < na) ? Z[(int64_t)(r0 + r) * na + t] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int u = 0; u < PER; ++u) acc[r] += mv[r][u] * xv[u];
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double z = reduce64(acc[r]);
    if (lane == 0 && r0 + r < nout) correct_loaded<T>(A, ch.row + r0 + r, cs[r], wi[r] - z);
  }
  if (A.advance_step && blockIdx.x == 0 && threadIdx.x == 0) A.step[0] = A.step[0] + 1;
}

// ---------------------------------------------------------------------------
// nested-dissection solve (NdFactor): one launch per level and direction
// ---------------------------------------------------------------------------
constexpr int kNdRows = 4;  // rows per wave; a chunk is 4 waves x kNdRows rows
constexpr int kNdBatch = 4; // rows per thread whose gathers are in flight together

// b'_s = rhs_s - (children's updates at the rows of s) into vec[0..m), the
// gathers of kNdBatch rows per thread in flight together (index, source,
// value: three round trips to memory for the whole fill).  The updates are
// subtracted one by one in slot order.
__device__ inline void nd_fill_rhs(const SolveArgs& A, const NdChunk& ch, double* vec, int tid, int nthr) {
  for (int i0 = tid; i0 < ch.m; i0 += kNdBatch * nthr) {
    int64_t g0[kNdBatch], g1[kNdBatch], s0[kNdBatch], s1[kNdBatch];
    double v[kNdBatch], w0[kNdBatch], w1[kNdBatch];
#pragma unroll
    for (int b = 0; b < kNdBatch; ++b) {
      const int i = i0 + b * nthr;
      g0[b] = g1[b] = 0;
      v[b] = 0.0;
      if (i < ch.m) {
        g0[b] = A.nd_gptr[ch.goff + i];
        g1[b] = A.nd_gptr[ch.goff + i + 1];
        v[b] = A.rhs[ch.c0 + i];
      }
    }
#pragma unroll
    for (int b = 0; b < kNdBatch; ++b) {
      s0[b] = g0[b] < g1[b] ? A.nd_gsrc[g0[b]] : 0;
      s1[b] = g0[b] + 1 < g1[b] ? A.nd_gsrc[g0[b] + 1] : 0;
    }
#pragma unroll
    for (int b = 0; b < kNdBatch; ++b) {
      w0[b] = g0[b] < g1[b] ? A.nd_W[s0[b]] : 0.0;
      w1[b] = g0[b] + 1 < g1[b] ? A.nd_W[s1[b]] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < kNdBatch; ++b) {
      const int i = i0 + b * nthr;
      if (i >= ch.m) break;
      double x = v[b];
      if (g0[b] < g1[b]) x -= w0[b];
      if (g0[b] + 1 < g1[b]) x -= w1[b];
      for (int64_t g = g0[b] + 2; g < g1[b]; ++g) x -= A.nd_W[A.nd_gsrc[g]];
      vec[i] = x;
    }
  }
}

// the children's updates at update row r (>= m) of a chunk's supernode, in
// slot order (the first two sources requested together): added to the row's
// product when it is written into W
__device__ inline double nd_ext_sum(const SolveArgs& A, const NdChunk& ch, int r) {
  const int64_t slot = ch.goff + r;
  const int64_t g0 = A.nd_gptr[slot], g1 = A.nd_gptr[slot + 1];
  const int64_t s0 = g0 < g1 ? A.nd_gsrc[g0] : 0, s1 = g0 + 1 < g1 ? A.nd_gsrc[g0 + 1] : 0;
  const double w0 = g0 < g1 ? A.nd_W[s0] : 0.0, w1 = g0 + 1 < g1 ? A.nd_W[s1] : 0.0;
  double v = 0.0;
  if (g0 < g1) v += w0;
  if (g0 + 1 < g1) v += w1;
  for (int64_t g = g0 + 2; g < g1; ++g) v += A.nd_W[A.nd_gsrc[g]];
  return v;
}

// Forward substitution of one level: b'_s (the right-hand side less the
// children's updates) in LDS, then rows of L_ss^-1 (into y) and of C_s (plus
// the children's updates at struct(s), into W_s).  PER values per lane and
// row are in flight at once (the host picks PER from the level's longest
// row), and the first of them are requested before the gathers of b'_s, so
// that a level waits on about one round trip to memory.
template <int PER>
__global__ __launch_bounds__(kThreads) void nd_forward_kernel(const SolveArgs A, int64_t chunk0, int n) {
  extern __shared__ double vec[];
  const NdChunk ch = A.nd_fchunks[chunk0 + xcd_contiguous(blockIdx.x, n)];
  const int m = ch.m;
  const int lane = threadIdx.x & 63, r0 = ch.first + (threadIdx.x >> 6) * kNdRows;
  const int rend = ch.first + ch.rows;
  const double* row[kNdRows];
  int len[kNdRows];
  int lmax = 0;
#pragma unroll
  for (int u = 0; u < kNdRows; ++u) {
    const int r = r0 + u;
    len[u] = r >= rend ? 0 : (r < m ? r + 1 : m);
    row[u] = A.nd_fwd + ch.moff +
             (r < m ? (int64_t)r * (r + 1) / 2 : (int64_t)m * (m + 1) / 2 + (int64_t)(r - m) * m);
    lmax = max(lmax, len[u]);
  }
  double mv[kNdRows][PER];
#pragma unroll
  for (int v = 0; v < PER; ++v) {
    const int j = lane + 64 * v;
#pragma unroll
    for (int u = 0; u < kNdRows; ++u) mv[u][v] = j < len[u] ? stream_load(&row[u][j]) : 0.0;
  }
  // lane u < kNdRows: the children's updates at update row r0 + u, gathered
  // now, off the path of the products
  double ext = 0.0;
  if (lane < kNdRows && r0 + lane < rend && r0 + lane >= m) ext = nd_ext_sum(A, ch, r0 + lane);
  nd_fill_rhs(A, ch, vec, threadIdx.x, kThreads);
  __syncthreads();
  double acc[kNdRows];
#pragma unroll
  for (int u = 0; u < kNdRows; ++u) acc[u] = 0.0;
  for (int base = 0;;) {
    double xv[PER];
#pragma unroll
    for (int v = 0; v < PER; ++v) {
      const int j = base + lane + 64 * v;
      xv[v] = j < lmax ? vec[j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kNdRows; ++u)
#pragma unroll
      for (int v = 0; v < PER; ++v) acc[u] += mv[u][v] * xv[v];
    base += 64 * PER;
    if (base >= lmax) break;
#pragma unroll
    for (int v = 0; v < PER; ++v) {
      const int j = base + lane + 64 * v;
#pragma unroll
      for (int u = 0; u < kNdRows; ++u) mv[u][v] = j < len[u] ? stream_load(&row[u][j]) : 0.0;
    }
  }
#pragma unroll
  for (int u = 0; u < kNdRows; ++u) {
    const int r = r0 + u;
    if (r >= rend) break;  // uniform over the wave
    const double t = reduce64(acc[u]);
    const double e = __shfl(ext, u);
    if (lane == 0) {
      if (r < m) A.w[ch.c0 + r] = t;
      else A.nd_W[ch.woff + r - m] = t + e;
    }
  }
}

// Forward substitution of one level for small supernodes: one thread per
// output row t of [L_ss^-1; C_s] (64 consecutive rows per wave, four waves
// per workgroup, each wave its own chunk), looping over the columns j of the
// row.  Column j of the stacked matrix is row j of the backward values, where
// the entry of row t sits at t - j (for the L_ss^-1 part, only j <= t), so
// the lanes of a wave read consecutive values for every j.
__global__ __launch_bounds__(kThreads) void nd_forward_cols_kernel(const SolveArgs A, int64_t chunk0, int n) {
  __shared__ double vec[kThreads / 64][kNdColsMaxM];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t ci = (int64_t)blockIdx.x * (kThreads / 64) + wv;
  const bool live = ci < n;
  NdChunk ch{};
  if (live) ch = A.nd_fcchunks[chunk0 + ci];
  const int m = ch.m, k = ch.k;
  const int t = ch.first + lane;
  const bool ok = live && lane < ch.rows;
  // the children's updates at this lane's update row, gathered ahead
  const double ext = ok && t >= m ? nd_ext_sum(A, ch, t) : 0.0;
  nd_fill_rhs(A, ch, vec[wv], lane, 64);
  __syncthreads();
  if (!live) return;
  const int jmax = ok ? (t < m ? t : m - 1) : -1;
  const int tl = ch.first + ch.rows - 1;       // the wave's last row
  const int jend = tl < m ? tl : m - 1;
  const double* col = A.nd_bwd + ch.moff;      // backward row j: (m - j) + k values
  constexpr int U = 16;                        // loads in flight per lane
  double acc0 = 0.0, acc1 = 0.0;
  for (int j0 = 0; j0 <= jend; j0 += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u;
      v[u] = j <= jmax ? stream_load(&col[(int64_t)j * (m + k) - (int64_t)j * (j - 1) / 2 + t - j]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; u += 2) {
      acc0 = fma(v[u], j0 + u <= jend ? vec[wv][j0 + u] : 0.0, acc0);
      acc1 = fma(v[u + 1], j0 + u + 1 <= jend ? vec[wv][j0 + u + 1] : 0.0, acc1);
    }
  }
  const double r = acc0 + acc1;
  if (ok) {
    if (t < m) A.w[ch.c0 + t] = r;
    else A.nd_W[ch.woff + t - m] = r + ext;
  }
}

// Backward substitution of one level: [y_s; -x at struct(s)] in LDS, then
// x_s = L_ss^-T y_s - C_s^T x_struct(s) row by row (columns of the stacked
// forward values), each followed by the trapezoidal corrector of that c row.
// Values in flight as in the forward kernel.
template <typename T, int PER>
__global__ __launch_bounds__(kThreads) void nd_backward_kernel(const SolveArgs A, int64_t chunk0, int n) {
  extern __shared__ double vec[];
  const NdChunk ch = A.nd_bchunks[chunk0 + xcd_contiguous(blockIdx.x, n)];
  const int m = ch.m, k = ch.k;
  const int lane = threadIdx.x & 63, j0 = ch.first + (threadIdx.x >> 6) * kNdRows;
  const int jend = ch.first + ch.rows;
  CState cs[kNdRows];
  const double* row[kNdRows];
  int len[kNdRows];
  int lmax = 0;
#pragma unroll
  for (int u = 0; u < kNdRows; ++u) {
    const int j = j0 + u;
    len[u] = j >= jend ? 0 : m - j + k;
    row[u] = A.nd_bwd + ch.moff + (int64_t)j * (m + k) - (int64_t)j * (j - 1) / 2;
    lmax = max(lmax, len[u]);
  }
  double mv[kNdRows][PER];
#pragma unroll
  for (int v = 0; v < PER; ++v) {
    const int t = lane + 64 * v;
#pragma unroll
    for (int u = 0; u < kNdRows; ++u) mv[u][v] = t < len[u] ? stream_load(&row[u][t]) : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kNdRows; ++u)
    if (lane == 0 && j0 + u < jend) cs[u] = load_cstate(A, ch.c0 + j0 + u);
  // [y_s; -x at struct(s)], kNdBatch entries per thread in flight together
  for (int i0 = threadIdx.x; i0 < m + k; i0 += kNdBatch * kThreads) {
    int64_t idx[kNdBatch];
    double v[kNdBatch];
#pragma unroll
    for (int b = 0; b < kNdBatch; ++b) {
      const int i = i0 + b * kThreads;
      idx[b] = (i >= m && i < m + k) ? A.nd_st[ch.soff + i - m] : 0;
      v[b] = i < m ? A.w[ch.c0 + i] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < kNdBatch; ++b) {
      const int i = i0 + b * kThreads;
      if (i >= m && i < m + k) v[b] = -A.ac[idx[b]];
    }
#pragma unroll
    for (int b = 0; b < kNdBatch; ++b) {
      const int i = i0 + b * kThreads;
      if (i < m + k) vec[i] = v[b];
    }
  }
  __syncthreads();
  double acc[kNdRows];
#pragma unroll
  for (int u = 0; u < kNdRows; ++u) acc[u] = 0.0;
  for (int base = 0;;) {
#pragma unroll
    for (int u = 0; u < kNdRows; ++u)
#pragma unroll
      for (int v = 0; v < PER; ++v) {
        const int t = base + lane + 64 * v;
        acc[u] += mv[u][v] * (t < len[u] ? vec[j0 + u + t] : 0.0);
      }
    base += 64 * PER;
    if (base >= lmax) break;
#pragma unroll
    for (int v = 0; v < PER; ++v) {
      const int t = base + lane + 64 * v;
#pragma unroll
      for (int u = 0; u < kNdRows; ++u) mv[u][v] = t < len[u] ? stream_load(&row[u][t]) : 0.0;
    }
  }
#pragma unroll
  for (int u = 0; u < kNdRows; ++u) {
    const int j = j0 + u;
    if (j >= jend) break;  // uniform over the wave
    const double x = reduce64(acc[u]);
    if (lane == 0) correct_loaded<T>(A, ch.c0 + j, cs[u], x);
  }
  if (A.advance_step && chunk0 == 0 && blockIdx.x == 0 && threadIdx.x == 0) A.step[0] = A.step[0] + 1;
}

// ---------------------------------------------------------------------------
// local time-stepping leap-frog on the fine rows (LtsArgs)
// ---------------------------------------------------------------------------
// one wave per row: partial sums over the row's entries, wave reduction
__device__ inline double csr_row_dot(const int64_t* rp, const int32_t* col, const double* val, const double* x,
                                     int64_t row, int lane) {
  double acc = 0.0;
  for (int64_t k = rp[row] + lane; k < rp[row + 1]; k += 64) acc += val[k] * x[col[k]];
  return reduce64(acc);
}

__global__ __launch_bounds__(kThreads) void lts_pre_kernel(const LtsArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (i >= A.nf) return;
  const double ko = csr_row_dot(A.rp_o, A.col_o, A.val_o, A.un, i, lane);
  if (lane == 0) {
    const int64_t g = A.node[i];
    A.g[i] = A.minv[i] * (ko - A.ft[A.step[0]] * A.fx[i]);
    A.q[0][i] = A.un[g];
    A.uprev[i] = A.uw[g];
  }
}

// substep k (0 <= k < m): q[(k+1) % 3] from q[k % 3] and q[(k-1) % 3]
__global__ __launch_bounds__(kThreads) void lts_substep_kernel(const LtsArgs A, int k) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (i >= A.nf) return;
  const double* qk = A.q[k % 3];
  const double kp = csr_row_dot(A.rp_f, A.col_f, A.val_f, qk, i, lane);
  if (lane == 0) {
    const double acc = A.g[i] + A.minv[i] * kp;
    const double qn = k == 0 ? qk[i] - 0.5 * A.tau2 * acc : 2.0 * qk[i] - A.q[(k + 2) % 3][i] - A.tau2 * acc;
    if (k == A.m - 1) {
      const double u1 = 2.0 * qn - A.uprev[i];
      A.uw[A.node[i]] = u1;
      if (i < A.nc) A.uc[i] = u1;
    } else {
      A.q[(k + 1) % 3][i] = qn;
    }
  }
  if (k == A.m - 1 && blockIdx.x == 0 && threadIdx.x == 0) A.step[0] = A.step[0] + 1;
}

}  // namespace

namespace {
template <bool PRED>
void launch_rhs_rows(const RhsArgs& a, int fp, hipStream_t s) {
  if (a.lanes_per_row == 32) {
    const dim3 g = grid1d(a.nc, 2 * (kThreads / 64));  // two rows per wave
    if (fp == 32) hipLaunchKernelGGL((rhs_kernel<float, 32, PRED>), g, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL((rhs_kernel<double, 32, PRED>), g, dim3(kThreads), 0, s, a);
  } else {
    const dim3 g = grid1d(a.nc, 4 * (kThreads / 64));  // four rows per wave
    if (fp == 32) hipLaunchKernelGGL((rhs_kernel<float, 16, PRED>), g, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL((rhs_kernel<double, 16, PRED>), g, dim3(kThreads), 0, s, a);
  }
}
}  // namespace

hipError_t launch_rhs(const RhsArgs& a, int fp, hipStream_t s) {
  if (a.nc == 0) return hipSuccess;
  if (a.pred) {
    hipLaunchKernelGGL(predict_kernel, grid1d(a.nc, kThreads), dim3(kThreads), 0, s, a);
    launch_rhs_rows<true>(a, fp, s);
  } else {
    launch_rhs_rows<false>(a, fp, s);
  }
  return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs& a, int64_t n_parts, int64_t n_schur_chunks, int64_t n_schur_chain,
                        int64_t n_part_chunks, int64_t n_dense_chunks, int fp, hipStream_t s) {
  if (n_parts == 0) return hipSuccess;
  if (a.dense && a.dense_wide) {
    // symmetric blocked A_pp^-1, then A_Sp w_p over the chunk list of the
    // coupling rows (16 separator rows per chunk)
    if (a.n_sym_blocks > 0)
      hipLaunchKernelGGL(part_sym_kernel, dim3((unsigned)a.n_sym_blocks), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(part_sym_sum_kernel, dim3((unsigned)n_part_chunks), dim3(kSymB), 0, s, a);
    if (n_dense_chunks > 0)
      hipLaunchKernelGGL(part_coupling_kernel, dim3((unsigned)n_dense_chunks), dim3(kThreads), 0, s, a);
  }
  else if (a.dense)
    hipLaunchKernelGGL(part_dense_kernel, dim3((unsigned)(4 * n_dense_chunks)), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(part_solve_kernel, dim3((unsigned)n_parts), dim3(kThreads), (size_t)a.smem_part, s, a);
  if (n_schur_chain > 0) {
    if (fp == 32)
      hipLaunchKernelGGL(schur_chain_kernel<float>, dim3((unsigned)n_schur_chain), dim3(kThreads),
                         (size_t)a.smem_schur, s, a);
    else
      hipLaunchKernelGGL(schur_chain_kernel<double>, dim3((unsigned)n_schur_chain), dim3(kThreads),
                         (size_t)a.smem_schur, s, a);
  }
  if (a.dense_wide && n_schur_chunks > 0) {
    hipLaunchKernelGGL(schur_rs_kernel, dim3((unsigned)((n_schur_chunks + 3) / 4)), dim3(64), 0, s, a, n_schur_chunks);
    if (fp == 32)
      hipLaunchKernelGGL(schur_wide_kernel<float>, dim3((unsigned)n_schur_chunks), dim3(kThreads), 0, s, a);
    else
      hipLaunchKernelGGL(schur_wide_kernel<double>, dim3((unsigned)n_schur_chunks), dim3(kThreads), 0, s, a);
    n_schur_chunks = 0;  // done
  }
  if (a.dense_wide) {
    if (fp == 32)
      hipLaunchKernelGGL(part_correct_wide_kernel<float>, dim3((unsigned)a.n_corr_chunks), dim3(kThreads), 0, s, a);
    else
      hipLaunchKernelGGL(part_correct_wide_kernel<double>, dim3((unsigned)a.n_corr_chunks), dim3(kThreads), 0, s, a);
  } else if (fp == 32) {
    if (n_schur_chunks > 0)
      hipLaunchKernelGGL(schur_kernel<float>, dim3((unsigned)(4 * n_schur_chunks)), dim3(kThreads),
                         (size_t)a.smem_sep, s, a);
    hipLaunchKernelGGL(part_correct_kernel<float>, dim3((unsigned)n_part_chunks), dim3(64 * kCorrectWaves), 0, s, a);
  } else {
    if (n_schur_chunks > 0)
      hipLaunchKernelGGL(schur_kernel<double>, dim3((unsigned)(4 * n_schur_chunks)), dim3(kThreads),
                         (size_t)a.smem_sep, s, a);
    hipLaunchKernelGGL(part_correct_kernel<double>, dim3((unsigned)n_part_chunks), dim3(64 * kCorrectWaves), 0, s, a);
  }
  return hipGetLastError();
}

namespace {
template <int PER>
void nd_forward_level(const SolveArgs& a, int64_t c0, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(nd_forward_kernel<PER>, dim3((unsigned)n), dim3(kThreads), (size_t)a.nd_smem_f, s, a, c0, (int)n);
}
template <typename T, int PER>
void nd_backward_level(const SolveArgs& a, int64_t c0, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((nd_backward_kernel<T, PER>), dim3((unsigned)n), dim3(kThreads), (size_t)a.nd_smem_b, s, a, c0,
                     (int)n);
}
template <typename T>
void nd_backward_level_t(const SolveArgs& a, int per, int64_t c0, int64_t n, hipStream_t s) {
  if (per <= 1) nd_backward_level<T, 1>(a, c0, n, s);
  else if (per == 2) nd_backward_level<T, 2>(a, c0, n, s);
  else if (per <= 4) nd_backward_level<T, 4>(a, c0, n, s);
  else nd_backward_level<T, 8>(a, c0, n, s);
}
}  // namespace

hipError_t launch_nd_solve(const SolveArgs& a, const NdLevels& L, int fp, hipStream_t s) {
  for (int h = 0; h < L.n_levels; ++h) {
    const int64_t n = L.flev[h + 1] - L.flev[h];
    if (n > 0) {
      const int per = L.fper[h];
      if (per <= 1) nd_forward_level<1>(a, L.flev[h], n, s);
      else if (per == 2) nd_forward_level<2>(a, L.flev[h], n, s);
      else if (per <= 4) nd_forward_level<4>(a, L.flev[h], n, s);
      else nd_forward_level<8>(a, L.flev[h], n, s);
    }
    const int64_t nc = L.fclev[h + 1] - L.fclev[h];
    if (nc > 0)
      hipLaunchKernelGGL(nd_forward_cols_kernel, dim3((unsigned)((nc + 3) / 4)), dim3(kThreads), 0, s, a, L.fclev[h],
                         (int)nc);
  }
  for (int h = L.n_levels - 1; h >= 0; --h) {
    const int64_t n = L.blev[h + 1] - L.blev[h];
    if (n == 0) continue;
    if (fp == 32) nd_backward_level_t<float>(a, L.bper[h], L.blev[h], n, s);
    else nd_backward_level_t<double>(a, L.bper[h], L.blev[h], n, s);
  }
  return hipGetLastError();
}

hipError_t launch_lts_step(const LtsArgs& a, hipStream_t s) {
  const dim3 g = grid1d(a.nf, kThreads / 64);
  for (int k = 0; k < a.m; ++k) hipLaunchKernelGGL(lts_substep_kernel, g, dim3(kThreads), 0, s, a, k);
  return hipGetLastError();
}

hipError_t launch_lts_pre(const LtsArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(lts_pre_kernel, grid1d(a.nf, kThreads / 64), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rhs_batch(const BatchTable<RhsArgs>& t, int blocks, int fp, int lanes, hipStream_t s) {
  if (blocks == 0) return hipSuccess;
  if (lanes == 32) {
    if (fp == 32) hipLaunchKernelGGL((rhs_batch_kernel<float, 32>), dim3(blocks), dim3(kThreads), 0, s, t);
    else hipLaunchKernelGGL((rhs_batch_kernel<double, 32>), dim3(blocks), dim3(kThreads), 0, s, t);
  } else {
    if (fp == 32) hipLaunchKernelGGL((rhs_batch_kernel<float, 16>), dim3(blocks), dim3(kThreads), 0, s, t);
    else hipLaunchKernelGGL((rhs_batch_kernel<double, 16>), dim3(blocks), dim3(kThreads), 0, s, t);
  }
  return hipGetLastError();
}

hipError_t launch_solve_batch(const BatchTable<SolveArgs>& dense, int dense_blocks, const BatchTable<SolveArgs>& sep,
                              int sep_blocks, size_t sep_smem, const BatchTable<SolveArgs>& corr, int corr_blocks,
                              int fp, hipStream_t s) {
  if (dense_blocks > 0)
    hipLaunchKernelGGL(part_dense_batch_kernel, dim3(dense_blocks), dim3(kThreads), 0, s, dense);
  if (sep_blocks > 0) {
    if (fp == 32) hipLaunchKernelGGL(schur_batch_kernel<float>, dim3(sep_blocks), dim3(kThreads), sep_smem, s, sep);
    else hipLaunchKernelGGL(schur_batch_kernel<double>, dim3(sep_blocks), dim3(kThreads), sep_smem, s, sep);
  }
  if (corr_blocks > 0) {
    if (fp == 32)
      hipLaunchKernelGGL(part_correct_batch_kernel<float>, dim3(corr_blocks), dim3(64 * kCorrectWaves), 0, s, corr);
    else
      hipLaunchKernelGGL(part_correct_batch_kernel<double>, dim3(corr_blocks), dim3(64 * kCorrectWaves), 0, s, corr);
  }
  return hipGetLastError();
}

hipError_t prepare_solve_batch(int fp) {
  return allow_full_lds(fp == 32 ? (const void*)schur_batch_kernel<float> : (const void*)schur_batch_kernel<double>);
}

hipError_t launch_correct_all(const SolveArgs& a, const double* an, int64_t nc, int fp, hipStream_t s) {
  if (nc == 0) return hipSuccess;
  if (fp == 32)
    hipLaunchKernelGGL(correct_all_kernel<float>, grid1d(nc, 256), dim3(256), 0, s, a, an, nc);
  else
    hipLaunchKernelGGL(correct_all_kernel<double>, grid1d(nc, 256), dim3(256), 0, s, a, an, nc);
  return hipGetLastError();
}

hipError_t prepare_solve(const SolveArgs& a, int fp) {
  (void)a;
  hipError_t e = allow_full_lds((const void*)part_solve_kernel);
  if (e == hipSuccess) e = allow_full_lds((const void*)nd_forward_kernel<1>);
  if (e == hipSuccess) e = allow_full_lds((const void*)nd_forward_kernel<2>);
  if (e == hipSuccess) e = allow_full_lds((const void*)nd_forward_kernel<4>);
  if (e == hipSuccess) e = allow_full_lds((const void*)nd_forward_kernel<8>);
  if (fp == 32) {
    if (e == hipSuccess) e = allow_full_lds((const void*)nd_backward_kernel<float, 1>);
    if (e == hipSuccess) e = allow_full_lds((const void*)nd_backward_kernel<float, 2>);
    if (e == hipSuccess) e = allow_full_lds((const void*)nd_backward_kernel<float, 4>);
    if (e == hipSuccess) e = allow_full_lds((const void*)nd_backward_kernel<float, 8>);
  } else {
    if (e == hipSuccess) e = allow_full_lds((const void*)nd_backward_kernel<double, 1>);
    if (e == hipSuccess) e = allow_full_lds((const void*)nd_backward_kernel<double, 2>);
    if (e == hipSuccess) e = allow_full_lds((const void*)nd_backward_kernel<double, 4>);
    if (e == hipSuccess) e = allow_full_lds((const void*)nd_backward_kernel<double, 8>);
  }
  if (e == hipSuccess) e = allow_full_lds((const void*)schur_kernel<float>);
  if (e == hipSuccess) e = allow_full_lds((const void*)schur_kernel<double>);
  if (e != hipSuccess) return e;
  return allow_full_lds(fp == 32 ? (const void*)schur_chain_kernel<float> : (const void*)schur_chain_kernel<double>);
}

}  // namespace imex
