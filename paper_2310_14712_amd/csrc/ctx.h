// The library context (one Newmark IMEX problem on one device), shared by the
// C ABI (capi.cpp) and the iterative solvers of the implicit block
// (learned_host.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/imex.h"
#include "device.h"
#include "internal.h"

namespace imex {
struct LearnedState;  // iterative solvers and the learned preconditioner (learned_host.cpp)
}
struct imex_ctx;
namespace imex {
// hooks of the time loop into the iterative solvers (learned_host.cpp)
imex_status learned_collect(imex_ctx* c, hipStream_t st);        // after the rhs kernel, before the solve
imex_status learned_collect_after(imex_ctx* c, hipStream_t st);  // after the solve and corrector
imex_status learned_solve_step(imex_ctx* c, const SolveArgs& s, hipStream_t st);
// the factorised solve and corrector of one step (either factor form)
hipError_t launch_factor_solve(const imex_ctx* c, const SolveArgs& s, hipStream_t st);
bool learned_needs_eager(const imex_ctx* c);  // the step runs host-driven (no graphs)
void learned_free(imex_ctx* c);
}  // namespace imex
using namespace imex;  // internal header: the context is built from the imex:: types

struct DevBuf {
  void* p = nullptr;
  bool owned = false;
};

struct imex_ctx {
  std::string err;
  HostSetup hs;
  bool host_only = false;
  int fp = 64;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;

  DevBuf grid[2];
  DevBuf cstate;  // u^c | v^c | a^c
  float* d_delta = nullptr;  // FP32: increment u_n - u_{n-1} on the d nodes
  uint8_t* d_flags = nullptr;
  uint32_t* d_kron_mask = nullptr;  // 3D tensor-product form of the explicit kernel
  int64_t* d_kron_rest = nullptr;
  double* d_src = nullptr;
  int64_t sbox_lo[3] = {0, 0, 0}, sbox_hi[3] = {0, 0, 0};
  // implicit block
  int64_t *d_rp_d = nullptr, *d_rp_c = nullptr;
  int32_t *d_col_d = nullptr, *d_col_c = nullptr;  // 32-bit column ids (grid and c indices)
  double *d_val_d = nullptr, *d_val_c = nullptr, *d_fxc = nullptr;
  int64_t* d_cnodes = nullptr;
  ChainMeta *d_parts = nullptr, *d_schur = nullptr;
  double *d_cvals = nullptr, *d_zvals = nullptr, *d_cpval = nullptr, *d_cbuf = nullptr;
  int32_t *d_cints = nullptr, *d_cpptr = nullptr, *d_cpcol = nullptr;
  int64_t *d_cprowptr = nullptr, *d_sepsrc = nullptr;
  double* d_work = nullptr;  // right-hand side of the implicit solve
  double* d_pred = nullptr;  // predicted u^c of the step (formed once per c dof before the rhs)
  double* d_w = nullptr;     // part / separator solutions
  int64_t n_parts = 0, n_schur_chunks = 0, n_schur_chain = 0, n_part_chunks = 0, n_dense_chunks = 0;
  int64_t* d_schain = nullptr;
  double* d_pinv = nullptr;
  SymBlock* d_symblocks = nullptr;  // symmetric blocked part inverses (parts above 1024 rows)
  int64_t* d_sympoff = nullptr;
  double* d_sympartial = nullptr;
  double* d_rs = nullptr;          // separator right-hand sides (wide form)
  CorrChunk* d_corrchunks = nullptr; // 16-row chunks of the parts (wide form)
  CorrChunk* d_partcorr = nullptr;   // chunk descriptors of the plain form
  DenseChunk* d_pdchunks = nullptr;
  SepChunk* d_sepchunks = nullptr;
  int64_t n_corr_chunks = 0;
  int64_t n_sym_blocks = 0, nnz_part_inv = 0;
  int64_t* d_dchunks = nullptr;
  double* d_sinv = nullptr;
  int64_t *d_schunks = nullptr, *d_pchunks = nullptr;
  double* d_ft = nullptr;
  int64_t ft_cap = 0;
  int* d_step = nullptr;
  int* d_check = nullptr;    // failure detection flag
  bool check_finite = false; // imex_step scans the state for NaN / Inf
  int64_t n_comp = 0;
  // nested-dissection factor (NdFactor) on the device
  double *d_ndf = nullptr, *d_ndb = nullptr, *d_ndW = nullptr;
  NdChunk *d_nd_fch = nullptr, *d_nd_bch = nullptr, *d_nd_fcch = nullptr;
  int32_t *d_nd_st = nullptr, *d_nd_gsrc = nullptr;
  int64_t* d_nd_gptr = nullptr;
  std::vector<int64_t> nd_flev, nd_fclev, nd_blev;  // chunk ranges per level
  std::vector<int8_t> nd_fper, nd_bper;              // values in flight per lane and row, per level
  // local time-stepping leap-frog (m > 0): substeps on the fine rows
  int lts_m = 0;
  LtsArgs la{};
  RhsArgs ra{};
  SolveArgs sa{};

  int cur = 0;  // grid buffer holding u_n
  bool assembled = false, initialized = false;
  int64_t steps_taken = 0;
  ExplicitArgs ea{};
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  // per-kernel timing inside the step (imex_set_step_timing): for each of
  // the last kTimedSteps steps, events before the explicit kernel and after
  // it, after the predictor and right-hand side, and after the solve
  std::vector<hipEvent_t> tev;
  bool timing = false;
  int64_t tev_count = 0;  // timed steps since timing was switched on

  std::vector<void*> allocs;
  // implicit solver of the steps (IMEX_SOLVER_*) and its state
  int solver = IMEX_SOLVER_CHOLESKY;
  imex::LearnedState* learned = nullptr;

  imex_status fail(imex_status s, const std::string& m) {
    err = m;
    return s;
  }
  imex_status hipfail(hipError_t e, const char* what) {
    std::ostringstream os;
    os << what << ": " << hipGetErrorString(e);
    err = os.str();
    return IMEX_EHIP;
  }
  template <typename X>
  hipError_t alloc(X** p, size_t bytes) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(bytes, 16));
    if (e == hipSuccess) {
      allocs.push_back(q);
      *p = static_cast<X*>(q);
    }
    return e;
  }
  void drop_graphs() {
    for (int k = 0; k < 2; ++k)
      if (graph[k]) {
        (void)hipGraphExecDestroy(graph[k]);
        graph[k] = nullptr;
      }
  }
  size_t grid_elem() const { return fp == 32 ? sizeof(float) : sizeof(double); }
};

#define HIPCHECK(ctx, expr, what)            \
  do {                                       \
    hipError_t e_ = (expr);                  \
    if (e_ != hipSuccess) return (ctx)->hipfail(e_, what); \
  } while (0)

