// Iterative solvers of the implicit block S a^c = rhs (flexible CG with a
// Jacobi, element-block or learned preconditioner), the per-cut-cell MLP
// preconditioner (weights, collection of training pairs from the method's
// own solves, training with Adam) and their C ABI entry points.
//
// The learned preconditioner is a learned correction on top of the
// element-block (additive Schwarz) step B r = sum_e P_e^T Binv_e r_e (Binv_e
// the inverse of cut cell e's diagonal block of S).  For every cut cell e
// with c dofs idx_e, local residual r_e, s_e = ||r_e|| and d_e = diag(S)_e,
// an MLP maps the features [r_e / s_e, d_e .* (B r)_e / s_e, d_e / max d_e]
// through two ReLU layers of 128 to y_e, and
//   z = B r + w .* sum_e P_e^T (s_e y_e / d_e),
// w = 1 / (cut cells sharing a dof).  It is trained on pairs (r, x = S^-1 r)
// that the method's own implicit solves produce (each step's right-hand
// side with the new acceleration, and the warm-start residual rhs - S a^c_n
// with the change of the acceleration), so that y_e reproduces
// d_e .* (x - B r)_e / s_e.  Each application returns the combination
// beta1 B r + beta2 c of the two parts (c the learned correction) that
// minimises the S-norm of the error over their span, so that exact outputs
// give z = S^-1 r and useless ones the (scaled) element-block step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "ctx.h"
#include "learned.h"

namespace imex {

namespace {
constexpr int kHidden = 128;
int pad16(int n) { return (n + 15) / 16 * 16; }
}  // namespace

struct LearnedState {
  std::vector<void*> allocs;
  // cut cells
  int E = 0, ne = 0, Epad = 0;
  ElemArgs L{};
  MlpDims d{};
  CsrDev S{};
  // parameters: [W1 (H x F) | b1 (H) | W2 (H x H) | b2 (H) | W3 (O x H) | b3 (O)]
  int64_t n_params = 0, oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  uint16_t* pb = nullptr;
  bool weights_set = false;
  int adam_t = 0;
  // one-vector inference buffers
  uint16_t *X1 = nullptr, *H1 = nullptr, *H2 = nullptr;
  double* s1 = nullptr;
  float *valid1 = nullptr, *Y1 = nullptr;
  // flexible CG
  double *x = nullptr, *r = nullptr, *r_old = nullptr, *pv = nullptr, *q = nullptr, *z = nullptr, *ze = nullptr;
  double *part = nullptr, *sc = nullptr;
  double tol = 1e-10;
  int maxit = 1000, check_every = 4, judge_every = 0;
  // training pairs collected from the solves: residuals R, solutions Xs,
  // and B r of the residuals (BR, formed before training)
  int cap = 0, count = 0;
  double *R = nullptr, *Xs = nullptr, *BR = nullptr;
  double* br1 = nullptr;  // B r of the one-vector inference
  double *cvec = nullptr, *cq1 = nullptr, *cq2 = nullptr, *cpart = nullptr, *csc = nullptr;  // the combination
  bool collecting = false, pending = false;
  // statistics
  int64_t solves = 0, iterations = 0, fallbacks = 0, judged = 0;
  int last_iterations = 0;
  double last_relres = 0.0, judge_max = 0.0;

  template <typename X>
  hipError_t alloc(X** ptr, size_t bytes) {
    void* q0 = nullptr;
    hipError_t e = hipMalloc(&q0, std::max<size_t>(bytes, 16));
    if (e == hipSuccess) {
      allocs.push_back(q0);
      *ptr = static_cast<X*>(q0);
    }
    return e;
  }
  ~LearnedState() {
    for (void* a : allocs) (void)hipFree(a);
  }
};

namespace {

#define LCHECK(ctx, expr, what)                                 \
  do {                                                          \
    hipError_t e_ = (expr);                                     \
    if (e_ != hipSuccess) return (ctx)->hipfail(e_, what);      \
  } while (0)

template <typename X>
hipError_t put(LearnedState* ls, X** dst, const std::vector<X>& src, hipStream_t s) {
  hipError_t e = ls->alloc(dst, sizeof(X) * src.size());
  if (e == hipSuccess && !src.empty())
    e = hipMemcpyAsync(*dst, src.data(), sizeof(X) * src.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

// inverse of a small SPD matrix (n x n, row-major) by Cholesky; false if not SPD
bool spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> Lm(A.size(), 0.0);
  for (int j = 0; j < n; ++j) {
    double dsum = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) dsum -= Lm[(size_t)j * n + k] * Lm[(size_t)j * n + k];
    if (!(dsum > 0.0)) return false;
    const double ljj = std::sqrt(dsum);
    Lm[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= Lm[(size_t)i * n + k] * Lm[(size_t)j * n + k];
      Lm[(size_t)i * n + j] = t / ljj;
    }
  }
  // columns of the inverse: solve L L^T x = e_c
  std::vector<double> col(n);
  for (int c = 0; c < n; ++c) {
    std::fill(col.begin(), col.end(), 0.0);
    col[c] = 1.0;
    for (int i = 0; i < n; ++i) {
      double t = col[i];
      for (int k = 0; k < i; ++k) t -= Lm[(size_t)i * n + k] * col[k];
      col[i] = t / Lm[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = col[i];
      for (int k = i + 1; k < n; ++k) t -= Lm[(size_t)k * n + i] * col[k];
      col[i] = t / Lm[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) A[(size_t)i * n + c] = col[i];
  }
  return true;
}

imex_status setup(imex_ctx* c) {
  if (c->learned) return IMEX_OK;
  if (c->host_only || !c->assembled) return c->fail(IMEX_ESTATE, "assemble the implicit block first");
  const HostSetup& hs = c->hs;
  const int64_t nc = (int64_t)hs.c_nodes.size();
  if (nc == 0) return c->fail(IMEX_EINVAL, "the mesh has no implicit block");
  auto* ls = new (std::nothrow) LearnedState();
  if (!ls) return c->fail(IMEX_ENOMEM, "out of host memory");
  const int dim = hs.dim, p = hs.p, n = p + 1;
  const int ne = dim == 3 ? n * n * n : n * n;
  std::vector<int64_t> cells(hs.cut_cells);
  std::sort(cells.begin(), cells.end());
  const int E = (int)cells.size();
  // cells' c indices (local order x fastest) and the diagonal of S
  std::vector<int32_t> eidx((size_t)E * ne);
  for (int e = 0; e < E; ++e) {
    const int64_t cid = cells[e];
    const int64_t ix = cid % hs.ne[0], iy = (cid / hs.ne[0]) % hs.ne[1], iz = cid / (hs.ne[0] * hs.ne[1]);
    int l = 0;
    for (int cz = 0; cz < (dim == 3 ? n : 1); ++cz)
      for (int b = 0; b < n; ++b)
        for (int a = 0; a < n; ++a, ++l) {
          const int64_t gnode = (ix * p + a) + hs.nn[0] * ((iy * p + b) + hs.nn[1] * (iz * p + cz));
          eidx[(size_t)e * ne + l] = (int32_t)hs.c_index[gnode];
          if (hs.c_index[gnode] < 0) {
            delete ls;
            return c->fail(IMEX_EINVAL, "a cut cell node is not a c dof");
          }
        }
  }
  const Csr& S = hs.S;
  std::vector<double> diag(nc, 0.0);
  for (int64_t i = 0; i < nc; ++i)
    for (int64_t k = S.ptr[i]; k < S.ptr[i + 1]; ++k)
      if (S.col[k] == i) diag[i] = S.val[k];
  std::vector<float> gfeat((size_t)E * ne);
  std::vector<int32_t> mult(nc, 0);
  for (int e = 0; e < E; ++e) {
    double mx = 0.0;
    for (int l = 0; l < ne; ++l) mx = std::max(mx, diag[eidx[(size_t)e * ne + l]]);
    for (int l = 0; l < ne; ++l) {
      gfeat[(size_t)e * ne + l] = (float)(diag[eidx[(size_t)e * ne + l]] / mx);
      mult[eidx[(size_t)e * ne + l]]++;
    }
  }
  std::vector<double> inv_mult(nc);
  std::vector<int32_t> inc_ptr(nc + 1, 0), inc((size_t)E * ne);
  for (int64_t i = 0; i < nc; ++i) {
    inv_mult[i] = 1.0 / std::max(1, mult[i]);
    inc_ptr[i + 1] = inc_ptr[i] + mult[i];
  }
  {
    std::vector<int32_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
    for (int e = 0; e < E; ++e)
      for (int l = 0; l < ne; ++l) inc[fill[eidx[(size_t)e * ne + l]]++] = e * ne + l;
  }
  // inverses of the cells' diagonal blocks of S
  std::vector<double> binv((size_t)E * ne * ne);
  bool spd = true;
#pragma omp parallel reduction(&& : spd)
  {
    std::vector<int> pos(nc, -1);  // c index -> local position in the current cell
    std::vector<double> A((size_t)ne * ne);
#pragma omp for schedule(dynamic)
    for (int e = 0; e < E; ++e) {
      const int32_t* idx = &eidx[(size_t)e * ne];
      for (int a = 0; a < ne; ++a) pos[idx[a]] = a;
      std::fill(A.begin(), A.end(), 0.0);
      for (int a = 0; a < ne; ++a) {
        const int64_t i = idx[a];
        for (int64_t k = S.ptr[i]; k < S.ptr[i + 1]; ++k) {
          const int b = pos[S.col[k]];
          if (b >= 0) A[(size_t)a * ne + b] = S.val[k];
        }
      }
      for (int a = 0; a < ne; ++a) pos[idx[a]] = -1;
      spd = spd_inverse(A, ne) && spd;
      std::copy(A.begin(), A.end(), binv.begin() + (size_t)e * ne * ne);
    }
  }
  if (!spd) {
    delete ls;
    return c->fail(IMEX_ENOTSPD, "a cut cell's block of S is not positive definite");
  }
  std::vector<int32_t> col32(S.col.size());
  for (size_t k = 0; k < S.col.size(); ++k) col32[k] = (int32_t)S.col[k];
  hipStream_t st = c->stream;
  hipError_t e = hipSuccess;
  int32_t *d_eidx = nullptr, *d_incp = nullptr, *d_inc = nullptr, *d_col = nullptr;
  double *d_diag = nullptr, *d_invm = nullptr, *d_binv = nullptr, *d_val = nullptr;
  float* d_g = nullptr;
  int64_t* d_rp = nullptr;
  if (e == hipSuccess) e = put(ls, &d_eidx, eidx, st);
  if (e == hipSuccess) e = put(ls, &d_diag, diag, st);
  if (e == hipSuccess) e = put(ls, &d_invm, inv_mult, st);
  if (e == hipSuccess) e = put(ls, &d_g, gfeat, st);
  if (e == hipSuccess) e = put(ls, &d_incp, inc_ptr, st);
  if (e == hipSuccess) e = put(ls, &d_inc, inc, st);
  if (e == hipSuccess) e = put(ls, &d_binv, binv, st);
  if (e == hipSuccess) e = put(ls, &d_rp, S.ptr, st);
  if (e == hipSuccess) e = put(ls, &d_col, col32, st);
  if (e == hipSuccess) e = put(ls, &d_val, S.val, st);
  ls->E = E;
  ls->ne = ne;
  ls->Epad = pad16(std::max(E, 1));
  ls->L = ElemArgs{nc, E, ne, d_eidx, d_diag, d_invm, d_g, d_incp, d_inc, d_binv};
  ls->S = CsrDev{nc, d_rp, d_col, d_val};
  ls->d = MlpDims{pad16(3 * ne), kHidden, pad16(ne)};
  const int F = ls->d.F, H = ls->d.H, O = ls->d.O;
  ls->oW1 = 0;
  ls->ob1 = ls->oW1 + (int64_t)H * F;
  ls->oW2 = ls->ob1 + H;
  ls->ob2 = ls->oW2 + (int64_t)H * H;
  ls->oW3 = ls->ob2 + H;
  ls->ob3 = ls->oW3 + (int64_t)O * H;
  ls->n_params = ls->ob3 + O;
  const size_t np = (size_t)ls->n_params;
  if (e == hipSuccess) e = ls->alloc(&ls->p, 4 * np);
  if (e == hipSuccess) e = ls->alloc(&ls->m, 4 * np);
  if (e == hipSuccess) e = ls->alloc(&ls->v, 4 * np);
  if (e == hipSuccess) e = ls->alloc(&ls->g, 4 * np);
  if (e == hipSuccess) e = ls->alloc(&ls->pb, 2 * np);
  const size_t Ep = (size_t)ls->Epad;
  if (e == hipSuccess) e = ls->alloc(&ls->X1, 2 * Ep * F);
  if (e == hipSuccess) e = ls->alloc(&ls->H1, 2 * Ep * H);
  if (e == hipSuccess) e = ls->alloc(&ls->H2, 2 * Ep * H);
  if (e == hipSuccess) e = ls->alloc(&ls->Y1, 4 * Ep * O);
  if (e == hipSuccess) e = ls->alloc(&ls->s1, 8 * Ep);
  if (e == hipSuccess) e = ls->alloc(&ls->valid1, 4 * Ep);
  for (double** vec : {&ls->x, &ls->r, &ls->r_old, &ls->pv, &ls->q, &ls->z, &ls->br1, &ls->cvec, &ls->cq1, &ls->cq2})
    if (e == hipSuccess) e = ls->alloc(vec, 8 * (size_t)nc);
  if (e == hipSuccess) e = ls->alloc(&ls->ze, 8 * (size_t)E * ne);
  if (e == hipSuccess) e = ls->alloc(&ls->part, 8 * (size_t)4 * kFcgBlocks);
  if (e == hipSuccess) e = ls->alloc(&ls->sc, 8 * (size_t)kNScalars);
  if (e == hipSuccess) e = ls->alloc(&ls->cpart, 8 * (size_t)3 * kFcgBlocks);
  if (e == hipSuccess) e = ls->alloc(&ls->csc, 8 * (size_t)8);
  if (e != hipSuccess) {
    delete ls;
    return c->hipfail(e, "learned setup");
  }
  c->learned = ls;
  return IMEX_OK;
}

// z = P(r) for one vector (device arrays, c order)
imex_status precond(imex_ctx* c, int which, const double* r, double* z, hipStream_t st) {
  LearnedState* ls = c->learned;
  const int64_t nc = ls->L.nc;
  if (which == IMEX_SOLVER_PCG_JACOBI) {
    LCHECK(c, launch_jacobi(nc, r, ls->L.diag, z, st), "jacobi");
    return IMEX_OK;
  }
  if (which == IMEX_SOLVER_PCG_BLOCK) {
    LCHECK(c, launch_block_precond(ls->L, r, ls->ze, z, st), "block preconditioner");
    return IMEX_OK;
  }
  const MlpDims& d = ls->d;
  LCHECK(c, launch_block_precond(ls->L, r, ls->ze, ls->br1, st), "block preconditioner");
  LCHECK(c, launch_mlp_features(ls->L, d, r, ls->br1, nullptr, 1, ls->Epad, ls->X1, ls->s1, ls->valid1, st),
         "features");
  GemmArgs g{};
  g.M = ls->Epad;
  g.N = d.H;
  g.K = d.F;
  g.a = ls->X1;
  g.lda = d.F;
  g.a_layout = kRowMajor;
  g.b = ls->pb + ls->oW1;
  g.ldb = d.F;
  g.b_layout = kRowMajor;
  g.bias = ls->p + ls->ob1;
  g.out_b = ls->H1;
  g.epi = kEpiBiasReluBf16;
  LCHECK(c, launch_gemm_bf16(g, st), "mlp layer 1");
  g.K = d.H;
  g.a = ls->H1;
  g.lda = d.H;
  g.b = ls->pb + ls->oW2;
  g.ldb = d.H;
  g.bias = ls->p + ls->ob2;
  g.out_b = ls->H2;
  LCHECK(c, launch_gemm_bf16(g, st), "mlp layer 2");
  g.N = d.O;
  g.a = ls->H2;
  g.b = ls->pb + ls->oW3;
  g.bias = ls->p + ls->ob3;
  g.out_f = ls->Y1;
  g.out_b = nullptr;
  g.epi = kEpiBiasF32;
  LCHECK(c, launch_gemm_bf16(g, st), "mlp layer 3");
  LCHECK(c, launch_mlp_scatter(ls->L, d, ls->s1, ls->Y1, ls->cvec, st), "mlp scatter");
  LCHECK(c, launch_combine(ls->S, r, ls->br1, ls->cvec, ls->cq1, ls->cq2, ls->cpart, ls->csc, z, st), "combination");
  return IMEX_OK;
}

// reads ||r||^2 and ||b||^2 (waits for the stream)
imex_status read_norms(imex_ctx* c, hipStream_t st, double* rr, double* bb) {
  double h[2];
  LCHECK(c, hipMemcpyAsync(h, c->learned->sc + kBB, 2 * sizeof(double), hipMemcpyDeviceToHost, st), "read norms");
  LCHECK(c, hipStreamSynchronize(st), "sync");
  *bb = h[0];
  *rr = h[1];
  return IMEX_OK;
}

// flexible CG on S x = b from x (device vectors); *iters, *conv
imex_status fcg(imex_ctx* c, int which, const double* b, double* x, hipStream_t st, int* iters, bool* conv,
                double* relres) {
  LearnedState* ls = c->learned;
  const int64_t n = ls->L.nc;
  const double* diag = ls->L.diag;
  *iters = 0;
  *conv = false;
  LCHECK(c, launch_fcg_init(ls->S, b, x, ls->r, ls->part, st), "fcg init");
  LCHECK(c, launch_fcg_reduce(ls->part, 2, ls->sc, kBB, st), "fcg reduce");
  double rr = 0, bb = 0;
  imex_status s0 = read_norms(c, st, &rr, &bb);
  if (s0 != IMEX_OK) return s0;
  const double tol2 = ls->tol * ls->tol * bb;
  *relres = bb > 0 ? std::sqrt(rr / bb) : 0.0;
  if (!(bb > 0) || rr <= tol2) {
    *conv = std::isfinite(rr);
    if (!(bb > 0)) LCHECK(c, hipMemsetAsync(x, 0, 8 * (size_t)n, st), "zero");
    return IMEX_OK;
  }
  imex_status sp = precond(c, which, ls->r, ls->z, st);
  if (sp != IMEX_OK) return sp;
  LCHECK(c, launch_fcg_dots(n, ls->z, ls->r, nullptr, diag, ls->part, st), "fcg dots");
  LCHECK(c, launch_fcg_reduce(ls->part, 4, ls->sc, kZdR, st), "fcg reduce");
  LCHECK(c, launch_fcg_scalars(ls->sc, 0, st), "fcg scalars");
  LCHECK(c, launch_fcg_direction(n, ls->sc, ls->z, ls->r, diag, ls->pv, 1, st), "fcg direction");
  for (int it = 1; it <= ls->maxit; ++it) {
    LCHECK(c, launch_fcg_spmv(ls->S, ls->pv, ls->q, ls->part, st), "fcg spmv");
    LCHECK(c, launch_fcg_reduce(ls->part, 1, ls->sc, kPQ, st), "fcg reduce");
    LCHECK(c, launch_fcg_scalars(ls->sc, 1, st), "fcg alpha");
    LCHECK(c, launch_fcg_update(n, ls->sc, x, ls->r, ls->r_old, ls->pv, ls->q, ls->part, st), "fcg update");
    LCHECK(c, launch_fcg_reduce(ls->part, 1, ls->sc, kRR, st), "fcg reduce");
    if (it % ls->check_every == 0 || it == ls->maxit) {
      s0 = read_norms(c, st, &rr, &bb);
      if (s0 != IMEX_OK) return s0;
      *iters = it;
      *relres = std::sqrt(rr / bb);
      if (!std::isfinite(rr)) return IMEX_OK;
      if (rr <= tol2) {
        *conv = true;
        return IMEX_OK;
      }
    }
    sp = precond(c, which, ls->r, ls->z, st);
    if (sp != IMEX_OK) return sp;
    LCHECK(c, launch_fcg_dots(n, ls->z, ls->r, ls->r_old, diag, ls->part, st), "fcg dots");
    LCHECK(c, launch_fcg_reduce(ls->part, 4, ls->sc, kZdR, st), "fcg reduce");
    LCHECK(c, launch_fcg_scalars(ls->sc, 2, st), "fcg beta");
    LCHECK(c, launch_fcg_direction(n, ls->sc, ls->z, ls->r, diag, ls->pv, 0, st), "fcg direction");
  }
  *iters = ls->maxit;
  return IMEX_OK;
}

// sum of squares of (a - b) and of b (host copies; tests and the judge only)
void host_diff(const std::vector<double>& a, const std::vector<double>& b, double* num, double* den) {
  double s0 = 0, s1 = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    s0 += (a[i] - b[i]) * (a[i] - b[i]);
    s1 += b[i] * b[i];
  }
  *num = s0;
  *den = s1;
}

// one minibatch of rows: features, targets, forward, loss, backward (grads in ls->g)
struct TrainBuffers {
  int rows_cap = 0;
  uint16_t *X = nullptr, *H1 = nullptr, *H2 = nullptr, *dYb = nullptr, *dA2b = nullptr, *dA1b = nullptr;
  float *T = nullptr, *Y = nullptr, *dY = nullptr, *dA2 = nullptr, *dA1 = nullptr, *valid = nullptr;
  float *slices = nullptr, *colwork = nullptr;
  double *s = nullptr, *lpart = nullptr;
  int* vsel = nullptr;
};

imex_status ensure_train_buffers(imex_ctx* c, TrainBuffers& tb, int rows, int max_vec) {
  LearnedState* ls = c->learned;
  if (rows <= tb.rows_cap) return IMEX_OK;
  const MlpDims& d = ls->d;
  const size_t R = (size_t)rows;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = ls->alloc(&tb.X, 2 * R * d.F);
  if (e == hipSuccess) e = ls->alloc(&tb.H1, 2 * R * d.H);
  if (e == hipSuccess) e = ls->alloc(&tb.H2, 2 * R * d.H);
  if (e == hipSuccess) e = ls->alloc(&tb.dYb, 2 * R * d.O);
  if (e == hipSuccess) e = ls->alloc(&tb.dA2b, 2 * R * d.H);
  if (e == hipSuccess) e = ls->alloc(&tb.dA1b, 2 * R * d.H);
  if (e == hipSuccess) e = ls->alloc(&tb.T, 4 * R * d.O);
  if (e == hipSuccess) e = ls->alloc(&tb.Y, 4 * R * d.O);
  if (e == hipSuccess) e = ls->alloc(&tb.dY, 4 * R * d.O);
  if (e == hipSuccess) e = ls->alloc(&tb.dA2, 4 * R * d.H);
  if (e == hipSuccess) e = ls->alloc(&tb.dA1, 4 * R * d.H);
  if (e == hipSuccess) e = ls->alloc(&tb.valid, 4 * R);
  const size_t slices = (R + 1023) / 1024;
  const size_t wmax = (size_t)std::max(d.H * d.F, std::max(d.H * d.H, d.O * d.H));
  if (e == hipSuccess) e = ls->alloc(&tb.slices, 4 * slices * wmax);
  if (e == hipSuccess) e = ls->alloc(&tb.colwork, 4 * ((R + 255) / 256) * (size_t)std::max(d.H, d.O));
  if (e == hipSuccess) e = ls->alloc(&tb.s, 8 * R);
  if (e == hipSuccess) e = ls->alloc(&tb.lpart, 8 * ((R + 3) / 4));
  if (e == hipSuccess) e = ls->alloc(&tb.vsel, sizeof(int) * (size_t)max_vec);
  if (e != hipSuccess) return c->hipfail(e, "training buffers");
  tb.rows_cap = rows;
  return IMEX_OK;
}

// B r of vectors R[0..n) into BR (device)
imex_status block_all(imex_ctx* c, const double* R, double* BR, int n) {
  LearnedState* ls = c->learned;
  for (int k = 0; k < n; ++k)
    LCHECK(c, launch_block_precond(ls->L, R + (size_t)k * ls->L.nc, ls->ze, BR + (size_t)k * ls->L.nc, c->stream),
           "block preconditioner");
  return IMEX_OK;
}

// one Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected) of the FP32
// master parameters with the gradients in ls->g; refreshes the BF16 copies
imex_status adam_update(imex_ctx* c, double lr) {
  LearnedState* ls = c->learned;
  ls->adam_t++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)ls->adam_t), c2 = 1.f - std::pow(b2, (float)ls->adam_t);
  LCHECK(c, launch_adam(ls->p, ls->m, ls->v, ls->g, ls->n_params, (float)lr, b1, b2, 1e-8f, c1, c2, ls->pb,
                        c->stream),
         "adam");
  return IMEX_OK;
}

// loss and gradients of the pairs (R, Xs)[vsel[0..nv)] (host vsel; BR: B r of
// the residuals) into ls->g
imex_status loss_grad(imex_ctx* c, TrainBuffers& tb, const double* R, const double* Xs, const double* BR,
                      const std::vector<int>& vsel, double* loss, int* n_rows) {
  LearnedState* ls = c->learned;
  hipStream_t st = c->stream;
  const MlpDims& d = ls->d;
  const int nv = (int)vsel.size();
  const int rows = pad16(nv * ls->E);
  imex_status s0 = ensure_train_buffers(c, tb, rows, nv);
  if (s0 != IMEX_OK) return s0;
  LCHECK(c, hipMemcpyAsync(tb.vsel, vsel.data(), sizeof(int) * nv, hipMemcpyHostToDevice, st), "vsel");
  LCHECK(c, launch_mlp_features(ls->L, d, R, BR, tb.vsel, nv, rows, tb.X, tb.s, tb.valid, st), "features");
  LCHECK(c, launch_mlp_targets(ls->L, d, Xs, BR, tb.vsel, nv, rows, tb.s, tb.valid, tb.T, st), "targets");
  std::vector<float> valid(rows);
  LCHECK(c, hipMemcpyAsync(valid.data(), tb.valid, 4 * (size_t)rows, hipMemcpyDeviceToHost, st), "valid");
  LCHECK(c, hipStreamSynchronize(st), "sync");
  int count = 0;
  for (float v0 : valid) count += v0 > 0.f;
  *n_rows = count;
  if (count == 0) {
    *loss = 0.0;
    LCHECK(c, hipMemsetAsync(ls->g, 0, 4 * (size_t)ls->n_params, st), "zero grads");
    return IMEX_OK;
  }
  // forward
  GemmArgs g{};
  g.M = rows;
  g.N = d.H;
  g.K = d.F;
  g.a = tb.X;
  g.lda = d.F;
  g.a_layout = kRowMajor;
  g.b = ls->pb + ls->oW1;
  g.ldb = d.F;
  g.b_layout = kRowMajor;
  g.bias = ls->p + ls->ob1;
  g.out_b = tb.H1;
  g.epi = kEpiBiasReluBf16;
  LCHECK(c, launch_gemm_bf16(g, st), "forward 1");
  g.K = d.H;
  g.a = tb.H1;
  g.lda = d.H;
  g.b = ls->pb + ls->oW2;
  g.ldb = d.H;
  g.bias = ls->p + ls->ob2;
  g.out_b = tb.H2;
  LCHECK(c, launch_gemm_bf16(g, st), "forward 2");
  g.N = d.O;
  g.a = tb.H2;
  g.b = ls->pb + ls->oW3;
  g.bias = ls->p + ls->ob3;
  g.out_f = tb.Y;
  g.out_b = nullptr;
  g.epi = kEpiBiasF32;
  LCHECK(c, launch_gemm_bf16(g, st), "forward 3");
  int nlp = 0;
  LCHECK(c, launch_mlp_loss(d, ls->ne, rows, tb.Y, tb.T, tb.valid, 1.0f / (float)count, tb.dY, tb.dYb, tb.lpart,
                            &nlp, st),
         "loss");
  // backward: weight gradients by split-K products, bias gradients by column sums
  const int ksplit = 1024;
  auto wgrad = [&](const uint16_t* dA, int ldA, const uint16_t* act, int ldAct, int M, int N, float* out) {
    GemmArgs w{};
    w.M = M;
    w.N = N;
    w.K = rows;
    w.a = dA;
    w.lda = ldA;
    w.a_layout = kTransposed;
    w.b = act;
    w.ldb = ldAct;
    w.b_layout = kTransposed;
    w.out_f = tb.slices;
    w.epi = kEpiPartial;
    w.ksplit = ksplit;
    hipError_t e = launch_gemm_bf16(w, st);
    if (e == hipSuccess) e = launch_sum_slices(tb.slices, (rows + ksplit - 1) / ksplit, (int64_t)M * N, out, st);
    return e;
  };
  LCHECK(c, wgrad(tb.dYb, d.O, tb.H2, d.H, d.O, d.H, ls->g + ls->oW3), "grad W3");
  LCHECK(c, launch_colsum(tb.dY, rows, d.O, tb.colwork, ls->g + ls->ob3, st), "grad b3");
  GemmArgs bd{};
  bd.M = rows;
  bd.N = d.H;
  bd.K = d.O;
  bd.a = tb.dYb;
  bd.lda = d.O;
  bd.a_layout = kRowMajor;
  bd.b = ls->pb + ls->oW3;
  bd.ldb = d.H;
  bd.b_layout = kTransposed;
  bd.mask = tb.H2;
  bd.out_f = tb.dA2;
  bd.out_b = tb.dA2b;
  bd.epi = kEpiMaskF32Bf16;
  LCHECK(c, launch_gemm_bf16(bd, st), "back 3");
  LCHECK(c, wgrad(tb.dA2b, d.H, tb.H1, d.H, d.H, d.H, ls->g + ls->oW2), "grad W2");
  LCHECK(c, launch_colsum(tb.dA2, rows, d.H, tb.colwork, ls->g + ls->ob2, st), "grad b2");
  bd.K = d.H;
  bd.a = tb.dA2b;
  bd.lda = d.H;
  bd.b = ls->pb + ls->oW2;
  bd.ldb = d.H;
  bd.mask = tb.H1;
  bd.out_f = tb.dA1;
  bd.out_b = tb.dA1b;
  LCHECK(c, launch_gemm_bf16(bd, st), "back 2");
  LCHECK(c, wgrad(tb.dA1b, d.H, tb.X, d.F, d.H, d.F, ls->g + ls->oW1), "grad W1");
  LCHECK(c, launch_colsum(tb.dA1, rows, d.H, tb.colwork, ls->g + ls->ob1, st), "grad b1");
  std::vector<double> lp(nlp);
  LCHECK(c, hipMemcpyAsync(lp.data(), tb.lpart, 8 * (size_t)nlp, hipMemcpyDeviceToHost, st), "loss");
  LCHECK(c, hipStreamSynchronize(st), "sync");
  double l = 0.0;
  for (double v0 : lp) l += v0;
  *loss = l / count;
  return IMEX_OK;
}

}  // namespace

// ---- hooks used by the time loop (capi.cpp) -----------------------------------
imex_status learned_collect(imex_ctx* c, hipStream_t st) {
  LearnedState* ls = c->learned;
  if (!ls || !ls->collecting || ls->count + 2 > ls->cap) return IMEX_OK;
  const int64_t nc = ls->L.nc;
  const double* rhs = c->sa.rhs;
  const double* ac = c->sa.ac;  // a^c_n (before the solve)
  double* R0 = ls->R + (size_t)ls->count * nc;
  double* X0 = ls->Xs + (size_t)ls->count * nc;
  // pair 0: (rhs, a^c_{n+1}); pair 1: (rhs - S a^c_n, a^c_{n+1} - a^c_n)
  LCHECK(c, hipMemcpyAsync(R0, rhs, 8 * (size_t)nc, hipMemcpyDeviceToDevice, st), "collect");
  LCHECK(c, launch_fcg_init(ls->S, rhs, ac, R0 + nc, ls->part, st), "collect residual");
  LCHECK(c, hipMemcpyAsync(X0 + nc, ac, 8 * (size_t)nc, hipMemcpyDeviceToDevice, st), "collect");
  ls->pending = true;
  return IMEX_OK;
}

imex_status learned_collect_after(imex_ctx* c, hipStream_t st) {
  LearnedState* ls = c->learned;
  if (!ls || !ls->pending) return IMEX_OK;
  const int64_t nc = ls->L.nc;
  const double* ac = c->sa.ac;  // a^c_{n+1} (after the solve and corrector)
  double* X0 = ls->Xs + (size_t)ls->count * nc;
  LCHECK(c, hipMemcpyAsync(X0, ac, 8 * (size_t)nc, hipMemcpyDeviceToDevice, st), "collect");
  LCHECK(c, launch_rsub(ac, X0 + nc, nc, st), "collect correction");
  ls->pending = false;
  ls->count += 2;
  return IMEX_OK;
}

imex_status learned_solve_step(imex_ctx* c, const SolveArgs& s, hipStream_t st) {
  LearnedState* ls = c->learned;
  const int64_t nc = ls->L.nc;
  // warm start from a^c_n
  LCHECK(c, hipMemcpyAsync(ls->x, s.ac, 8 * (size_t)nc, hipMemcpyDeviceToDevice, st), "warm start");
  int it = 0;
  bool conv = false;
  double relres = 0.0;
  imex_status r0 = fcg(c, c->solver, s.rhs, ls->x, st, &it, &conv, &relres);
  if (r0 != IMEX_OK) return r0;
  ls->solves++;
  ls->iterations += it;
  ls->last_iterations = it;
  ls->last_relres = relres;
  const bool judge = ls->judge_every > 0 && (ls->solves % ls->judge_every) == 0;
  if (!conv || judge) {
    // the factorised direct solve: fallback, or judge of the iterative result
    if (!conv) ls->fallbacks++;
    hipError_t e = launch_factor_solve(c, s, st);
    if (e != hipSuccess) return c->hipfail(e, "solve kernels");
    if (conv && judge) {
      std::vector<double> a(nc), b(nc);
      LCHECK(c, hipMemcpyAsync(a.data(), ls->x, 8 * (size_t)nc, hipMemcpyDeviceToHost, st), "judge");
      LCHECK(c, hipMemcpyAsync(b.data(), s.ac, 8 * (size_t)nc, hipMemcpyDeviceToHost, st), "judge");
      LCHECK(c, hipStreamSynchronize(st), "sync");
      double num = 0, den = 0;
      host_diff(a, b, &num, &den);
      ls->judged++;
      ls->judge_max = std::max(ls->judge_max, den > 0 ? std::sqrt(num / den) : std::sqrt(num));
    }
    return IMEX_OK;
  }
  LCHECK(c, launch_correct_all(s, ls->x, nc, c->fp, st), "corrector");
  return IMEX_OK;
}

bool learned_needs_eager(const imex_ctx* c) {
  return c->solver != IMEX_SOLVER_CHOLESKY || (c->learned && c->learned->collecting);
}

void learned_free(imex_ctx* c) {
  delete c->learned;
  c->learned = nullptr;
}

}  // namespace imex

using namespace imex;

extern "C" {

imex_status imex_set_solver(imex_ctx* c, int solver, double tol, int max_iter, int judge_every) {
  if (!c) return IMEX_EINVAL;
  if (solver < IMEX_SOLVER_CHOLESKY || solver > IMEX_SOLVER_PCG_MLP) return c->fail(IMEX_EINVAL, "unknown solver");
  if (solver != IMEX_SOLVER_CHOLESKY) {
    if (c->lts_m > 0) return c->fail(IMEX_EINVAL, "the leap-frog substepping has no implicit solve");
    if (!(tol > 0) || max_iter < 1 || judge_every < 0) return c->fail(IMEX_EINVAL, "bad iteration settings");
    imex_status st = setup(c);
    if (st != IMEX_OK) return st;
    if (solver == IMEX_SOLVER_PCG_MLP && !c->learned->weights_set)
      return c->fail(IMEX_ESTATE, "set or train the MLP weights first");
    c->learned->tol = tol;
    c->learned->maxit = max_iter;
    c->learned->judge_every = judge_every;
  }
  c->solver = solver;
  c->drop_graphs();
  return IMEX_OK;
}

imex_status imex_mlp_shape(imex_ctx* c, imex_mlp_info* out) {
  if (!c || !out) return IMEX_EINVAL;
  imex_status st = setup(c);
  if (st != IMEX_OK) return st;
  const LearnedState* ls = c->learned;
  out->n_cells = ls->E;
  out->dofs_per_cell = ls->ne;
  out->inputs = ls->d.F;
  out->hidden = ls->d.H;
  out->outputs = ls->d.O;
  out->n_params = ls->n_params;
  out->collected = ls->count;
  return IMEX_OK;
}

imex_status imex_mlp_set_weights(imex_ctx* c, const float* params, int64_t n) {
  if (!c || !params) return IMEX_EINVAL;
  imex_status st = setup(c);
  if (st != IMEX_OK) return st;
  LearnedState* ls = c->learned;
  if (n != ls->n_params) return c->fail(IMEX_EINVAL, "parameter count mismatch");
  LCHECK(c, hipMemcpyAsync(ls->p, params, 4 * (size_t)n, hipMemcpyHostToDevice, c->stream), "weights");
  LCHECK(c, launch_to_bf16(ls->p, ls->pb, n, c->stream), "bf16 weights");
  LCHECK(c, hipMemsetAsync(ls->m, 0, 4 * (size_t)n, c->stream), "adam");
  LCHECK(c, hipMemsetAsync(ls->v, 0, 4 * (size_t)n, c->stream), "adam");
  LCHECK(c, hipStreamSynchronize(c->stream), "sync");
  ls->adam_t = 0;
  ls->weights_set = true;
  return IMEX_OK;
}

imex_status imex_mlp_get_weights(imex_ctx* c, float* params, int64_t n) {
  if (!c || !params) return IMEX_EINVAL;
  if (!c->learned || !c->learned->weights_set) return c->fail(IMEX_ESTATE, "no weights");
  if (n != c->learned->n_params) return c->fail(IMEX_EINVAL, "parameter count mismatch");
  LCHECK(c, hipMemcpyAsync(params, c->learned->p, 4 * (size_t)n, hipMemcpyDeviceToHost, c->stream), "weights");
  LCHECK(c, hipStreamSynchronize(c->stream), "sync");
  return IMEX_OK;
}

imex_status imex_mlp_collect(imex_ctx* c, int capacity) {
  if (!c || capacity < 0) return IMEX_EINVAL;
  imex_status st = setup(c);
  if (st != IMEX_OK) return st;
  LearnedState* ls = c->learned;
  capacity += capacity & 1;  // whole pairs of vectors per step
  if (capacity > ls->cap) {
    double *R = nullptr, *Xs = nullptr, *BR = nullptr;
    const size_t bytes = 8 * (size_t)capacity * ls->L.nc;
    LCHECK(c, ls->alloc(&R, bytes), "training vectors");
    LCHECK(c, ls->alloc(&Xs, bytes), "training vectors");
    LCHECK(c, ls->alloc(&BR, bytes), "training vectors");
    if (ls->count > 0) {
      const size_t kept = 8 * (size_t)ls->count * ls->L.nc;
      LCHECK(c, hipMemcpyAsync(R, ls->R, kept, hipMemcpyDeviceToDevice, c->stream), "keep vectors");
      LCHECK(c, hipMemcpyAsync(Xs, ls->Xs, kept, hipMemcpyDeviceToDevice, c->stream), "keep vectors");
    }
    LCHECK(c, hipStreamSynchronize(c->stream), "sync");
    ls->R = R;
    ls->Xs = Xs;
    ls->BR = BR;
    ls->cap = capacity;
  }
  ls->collecting = capacity > 0;
  c->drop_graphs();
  return IMEX_OK;
}

imex_status imex_mlp_adam_step(imex_ctx* c, const float* grads, double lr) {
  if (!c || !grads || !(lr > 0)) return IMEX_EINVAL;
  LearnedState* ls = c->learned;
  if (!ls || !ls->weights_set) return c->fail(IMEX_ESTATE, "set the MLP weights first");
  LCHECK(c, hipMemcpyAsync(ls->g, grads, 4 * (size_t)ls->n_params, hipMemcpyHostToDevice, c->stream), "grads");
  imex_status st = adam_update(c, lr);
  if (st != IMEX_OK) return st;
  LCHECK(c, hipStreamSynchronize(c->stream), "sync");
  return IMEX_OK;
}

imex_status imex_mlp_train(imex_ctx* c, int epochs, int vectors_per_batch, double lr, uint64_t seed,
                           double* last_loss) {
  if (!c || epochs < 0 || vectors_per_batch < 1 || !(lr > 0)) return IMEX_EINVAL;
  LearnedState* ls = c->learned;
  if (!ls || !ls->weights_set) return c->fail(IMEX_ESTATE, "set the initial MLP weights first");
  if (ls->count == 0) return c->fail(IMEX_ESTATE, "no training vectors collected");
  TrainBuffers tb;
  imex_status sb = block_all(c, ls->R, ls->BR, ls->count);
  if (sb != IMEX_OK) return sb;
  std::vector<int> order(ls->count);
  std::iota(order.begin(), order.end(), 0);
  std::mt19937_64 rng(seed);
  double ep_loss = 0.0;
  for (int ep = 0; ep < epochs; ++ep) {
    std::shuffle(order.begin(), order.end(), rng);
    double tot = 0.0;
    int nb = 0;
    for (int b0 = 0; b0 < ls->count; b0 += vectors_per_batch) {
      std::vector<int> vsel(order.begin() + b0, order.begin() + std::min(ls->count, b0 + vectors_per_batch));
      double loss = 0.0;
      int rows = 0;
      imex_status st = loss_grad(c, tb, ls->R, ls->Xs, ls->BR, vsel, &loss, &rows);
      if (st != IMEX_OK) return st;
      if (rows == 0) continue;
      st = adam_update(c, lr);
      if (st != IMEX_OK) return st;
      tot += loss;
      ++nb;
    }
    ep_loss = nb ? tot / nb : 0.0;
  }
  LCHECK(c, hipStreamSynchronize(c->stream), "sync");
  if (last_loss) *last_loss = ep_loss;
  return IMEX_OK;
}

imex_status imex_mlp_loss_grad(imex_ctx* c, const double* vectors, const double* solutions, int n_vectors,
                               double* loss, float* grads) {
  if (!c || !vectors || !solutions || n_vectors < 1 || !loss) return IMEX_EINVAL;
  LearnedState* ls = c->learned;
  if (!ls || !ls->weights_set) return c->fail(IMEX_ESTATE, "set the MLP weights first");
  const int64_t nc = ls->L.nc;
  double* R = nullptr;
  const size_t bytes = 8 * (size_t)n_vectors * nc;
  LCHECK(c, hipMalloc(&R, 3 * bytes), "vectors");
  double* Xs = R + (size_t)n_vectors * nc;
  double* BR = Xs + (size_t)n_vectors * nc;
  hipError_t e = hipMemcpyAsync(R, vectors, bytes, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(Xs, solutions, bytes, hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) {
    (void)hipFree(R);
    return c->hipfail(e, "vectors");
  }
  TrainBuffers tb;
  std::vector<int> vsel(n_vectors);
  std::iota(vsel.begin(), vsel.end(), 0);
  int rows = 0;
  imex_status st = block_all(c, R, BR, n_vectors);
  if (st == IMEX_OK) st = loss_grad(c, tb, R, Xs, BR, vsel, loss, &rows);
  if (st == IMEX_OK && grads) {
    e = hipMemcpyAsync(grads, ls->g, 4 * (size_t)ls->n_params, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) st = c->hipfail(e, "grads");
  }
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(R);
  return st;
}

imex_status imex_precond_apply(imex_ctx* c, int which, const double* r, double* z) {
  if (!c || !r || !z) return IMEX_EINVAL;
  if (which < IMEX_SOLVER_PCG_JACOBI || which > IMEX_SOLVER_PCG_MLP) return c->fail(IMEX_EINVAL, "unknown preconditioner");
  imex_status st = setup(c);
  if (st != IMEX_OK) return st;
  LearnedState* ls = c->learned;
  if (which == IMEX_SOLVER_PCG_MLP && !ls->weights_set) return c->fail(IMEX_ESTATE, "set the MLP weights first");
  const int64_t nc = ls->L.nc;
  LCHECK(c, hipMemcpyAsync(ls->r_old, r, 8 * (size_t)nc, hipMemcpyHostToDevice, c->stream), "r");
  st = precond(c, which, ls->r_old, ls->z, c->stream);
  if (st != IMEX_OK) return st;
  LCHECK(c, hipMemcpyAsync(z, ls->z, 8 * (size_t)nc, hipMemcpyDeviceToHost, c->stream), "z");
  LCHECK(c, hipStreamSynchronize(c->stream), "sync");
  return IMEX_OK;
}

imex_status imex_solve_implicit(imex_ctx* c, int which, const double* rhs, double* x, int* iterations) {
  if (!c || !rhs || !x) return IMEX_EINVAL;
  if (which < IMEX_SOLVER_PCG_JACOBI || which > IMEX_SOLVER_PCG_MLP) return c->fail(IMEX_EINVAL, "unknown solver");
  imex_status st = setup(c);
  if (st != IMEX_OK) return st;
  LearnedState* ls = c->learned;
  if (which == IMEX_SOLVER_PCG_MLP && !ls->weights_set) return c->fail(IMEX_ESTATE, "set the MLP weights first");
  const int64_t nc = ls->L.nc;
  double* bd = nullptr;
  LCHECK(c, hipMalloc(&bd, 8 * (size_t)nc), "rhs");
  hipError_t e = hipMemcpyAsync(bd, rhs, 8 * (size_t)nc, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(ls->x, x, 8 * (size_t)nc, hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) {
    (void)hipFree(bd);
    return c->hipfail(e, "upload");
  }
  int it = 0;
  bool conv = false;
  double relres = 0.0;
  st = fcg(c, which, bd, ls->x, c->stream, &it, &conv, &relres);
  if (st == IMEX_OK) {
    e = hipMemcpyAsync(x, ls->x, 8 * (size_t)nc, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) st = c->hipfail(e, "download");
  }
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(bd);
  if (iterations) *iterations = it;
  if (st == IMEX_OK && !conv) return c->fail(IMEX_ENOCONV, "flexible CG did not converge");
  return st;
}

imex_status imex_solver_stats(const imex_ctx* cc, imex_solver_info* out) {
  if (!cc || !out) return IMEX_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->solver = cc->solver;
  const LearnedState* ls = cc->learned;
  if (!ls) return IMEX_OK;
  out->solves = ls->solves;
  out->iterations = ls->iterations;
  out->fallbacks = ls->fallbacks;
  out->judged = ls->judged;
  out->last_iterations = ls->last_iterations;
  out->last_relres = ls->last_relres;
  out->judge_max_rel_diff = ls->judge_max;
  return IMEX_OK;
}

}  // extern "C"
