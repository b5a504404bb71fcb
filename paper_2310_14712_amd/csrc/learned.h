// Device side of the iterative solvers of the implicit block: CSR products
// with S, flexible CG vector kernels, the element-block (additive Schwarz)
// preconditioner and the per-cut-cell MLP preconditioner with its training
// kernels (learned.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace imex {

// Cut cells and their dofs (c order), shared by the block and MLP
// preconditioners.
struct ElemArgs {
  int64_t nc;
  int E, ne;                  // cut cells, dofs per cut cell ((p+1)^d)
  const int32_t* eidx;        // E x ne c indices (local order x fastest)
  const double* diag;         // diag(S), nc
  const double* inv_mult;     // 1 / number of cut cells sharing the dof, nc
  const float* gfeat;         // E x ne: diag(S) over its maximum on the cell
  const int32_t* inc_ptr;     // nc + 1: cut-cell incidences of every dof
  const int32_t* inc;         // e * ne + l
  const double* binv;         // E x ne x ne inverses of the cells' diagonal blocks of S (row-major)
};

// MLP shapes: F = pad16(3 ne) inputs, H hidden, O = pad16(ne) outputs.
struct MlpDims {
  int F, H, O;
};

// Products C = A B in BF16 with FP32 accumulation (16x16x16 MFMA tiles).
enum GemmLayout { kRowMajor = 0, kTransposed = 1 };
enum GemmEpilogue {
  kEpiBiasReluBf16 = 0,  // out_b = bf16(max(C + bias, 0))
  kEpiBiasF32 = 1,       // out_f = C + bias
  kEpiMaskF32Bf16 = 2,   // out_f = C .* (mask > 0), out_b = bf16(out_f)
  kEpiPartial = 3        // out_f[kz] = C over the kz-th slice of K (split K)
};
struct GemmArgs {
  int M, N, K;            // multiples of 16
  const uint16_t* a;      // A(m, k) = a[m lda + k] (kRowMajor) or a[k lda + m] (kTransposed)
  int lda, a_layout;
  const uint16_t* b;      // B(k, n) = b[n ldb + k] (kRowMajor: B stored N x K) or b[k ldb + n] (kTransposed)
  int ldb, b_layout;
  const float* bias;      // N
  const uint16_t* mask;   // M x N (bf16), kEpiMaskF32Bf16
  float* out_f;           // M x N (ldc = N)
  uint16_t* out_b;        // M x N
  int epi;
  int ksplit;             // K per slice (kEpiPartial), multiple of 16
};

hipError_t launch_gemm_bf16(const GemmArgs& g, hipStream_t s);
// out[j] = sum_s part[s][j], j < n
hipError_t launch_sum_slices(const float* part, int slices, int64_t n, float* out, hipStream_t s);
// out[c] = sum_r m[r][c] for a rows x cols FP32 matrix (deterministic two-level sum)
hipError_t launch_colsum(const float* m, int64_t rows, int cols, float* work, float* out, hipStream_t s);

// MLP rows of n_vec residual vectors: row = k * E + e takes vector
// v = vsel[k] (or k when vsel is null) of R and of BR (B r of the same
// vectors; vectors of nc FP64 values).  X: rows_pad x F (BF16) with the
// features [r_e / s, diag_e .* (B r)_e / s, diag_e / max diag_e], s:
// rows_pad (local norms), valid: rows_pad (1 if s > 0)
hipError_t launch_mlp_features(const ElemArgs& L, const MlpDims& d, const double* R, const double* BR, const int* vsel,
                               int n_vec, int rows_pad, uint16_t* X, double* s, float* valid, hipStream_t st);
// training rows and targets: valid = 1 on the cells of each pair whose
// local norm s is positive and at least 1e-3 times the pair's largest
// (written over the features' valid); T (rows_pad x O, FP32) = diag_e .*
// (x - B r)_e / s on the first ne outputs of those rows, zero elsewhere, x
// from Xs (the solutions of the pairs), B r from BR
hipError_t launch_mlp_targets(const ElemArgs& L, const MlpDims& d, const double* Xs, const double* BR, const int* vsel,
                              int n_vec, int rows_pad, const double* s, float* valid, float* T, hipStream_t st);
// y = x - y (FP64)
hipError_t launch_rsub(const double* x, double* y, int64_t n, hipStream_t st);
// dY = 2 (Y - T) valid / count on the first ne outputs (FP32 and BF16), and
// per-block partial sums of valid (Y - T)^2
hipError_t launch_mlp_loss(const MlpDims& d, int ne, int rows_pad, const float* Y, const float* T, const float* valid,
                           float inv_count, float* dY, uint16_t* dYb, double* partial, int* n_partial,
                           hipStream_t st);
// the learned correction c_i = inv_mult_i sum_{(e,l) at i} s_e Y[e][l] / diag_i
hipError_t launch_mlp_scatter(const ElemArgs& L, const MlpDims& d, const double* s, const float* Y, double* z,
                              hipStream_t st);
struct CsrDev;
// z = beta1 br + beta2 c with (beta1, beta2) minimising ||S^-1 r - z||_S over
// span{br, c}: q1 = S br, q2 = S c, five reductions into sc[0..5) (partials
// in part, 3 x kFcgBlocks), then the combination; a degenerate pair keeps
// (br.r / br.S br) br
hipError_t launch_combine(const CsrDev& S, const double* r, const double* br, const double* c, double* q1,
                          double* q2, double* part, double* sc, double* z, hipStream_t st);
// element-block (additive Schwarz) preconditioner z = sum_e P_e^T Binv_e r_e
hipError_t launch_block_precond(const ElemArgs& L, const double* r, double* ze, double* z, hipStream_t st);
// Adam (Kingma and Ba) on FP32 master parameters; writes their BF16 copies
hipError_t launch_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, uint16_t* pb, hipStream_t st);
hipError_t launch_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t st);

// ---- flexible CG on S (CSR, c order) -----------------------------------------
struct CsrDev {
  int64_t n;
  const int64_t* rp;
  const int32_t* col;
  const double* val;
};
// Scalars of the iteration, in device memory (FcgScalar indices)
enum FcgScalar {
  kBB = 0,   // ||b||^2
  kRR,       // ||r||^2
  kRZ,       // r.z
  kPQ,       // p.q
  kAlpha,
  kBeta,
  kZdR,      // z.(r - r_old)
  kRZn,      // r.z of the new z
  kJdR,      // Jacobi z.(r - r_old)
  kRJ,       // r.(r / diag)
  kUseJ,     // 1 when the preconditioned residual is not a descent direction
  kNScalars
};
constexpr int kFcgBlocks = 1024;  // workgroups (and partial sums) of the reductions
// r = b - S x, partials of ||b||^2, ||r||^2
hipError_t launch_fcg_init(const CsrDev& S, const double* b, const double* x, double* r, double* part,
                           hipStream_t st);
// q = S p, partials of p.q
hipError_t launch_fcg_spmv(const CsrDev& S, const double* p, double* q, double* part, hipStream_t st);
// x += alpha p; r_old = r; r -= alpha q; partials of ||r||^2
hipError_t launch_fcg_update(int64_t n, const double* sc, double* x, double* r, double* r_old, const double* p,
                             const double* q, double* part, hipStream_t st);
// partials of z.(r - r_old), r.z, and the same for the Jacobi vector r / diag
hipError_t launch_fcg_dots(int64_t n, const double* z, const double* r, const double* r_old, const double* diag,
                           double* part, hipStream_t st);
// sums `k` interleaved partial arrays into sc[dst .. dst + k)
hipError_t launch_fcg_reduce(const double* part, int k, double* sc, int dst, hipStream_t st);
// scalar steps: which = 0 (start: p.z -> rz, falls back to Jacobi), 1 (alpha), 2 (beta and the new r.z)
hipError_t launch_fcg_scalars(double* sc, int which, hipStream_t st);
// p = zeta + beta p (zeta = z or r / diag when kUseJ); start: p = zeta
hipError_t launch_fcg_direction(int64_t n, const double* sc, const double* z, const double* r, const double* diag,
                                double* p, int start, hipStream_t st);
// z = r / diag
hipError_t launch_jacobi(int64_t n, const double* r, const double* diag, double* z, hipStream_t st);

}  // namespace imex
