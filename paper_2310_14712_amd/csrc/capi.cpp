// C ABI of the Newmark IMEX library: context lifetime, device uploads,
// initial state, the time loop (HIP graphs of step chunks) and exports.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/imex.h"
#include "ctx.h"
#include "device.h"
#include "internal.h"

using namespace imex;

namespace {
thread_local std::string g_setup_error;

constexpr int kGraphChunk = 32;  // steps per captured graph (even)
constexpr int kTimedSteps = 32;  // event slots of the per-kernel step timing
constexpr int kBatchLanes = 16;  // streams a batch spreads its instances over

}  // namespace

// ---- device scratch of the allocation-free sampling entry point ------------
// A file-scope device array: every device the library runs on holds one copy
// until the process ends.  Host code never passes the array's name to a
// kernel or a copy (in host code it is a host-side stand-in); it uses the
// device address obtained once per device with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[IMEX_SAMPLE_NOALLOC_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// the device address of `scratch` on `device` (the current device), looked
// up once per device
hipError_t scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the lookup needs that device current
    void* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}
}  // namespace

namespace {

template <typename X>
hipError_t upload(imex_ctx* c, X** dst, const std::vector<X>& src) {
  hipError_t e = c->alloc(dst, sizeof(X) * src.size());
  if (e != hipSuccess) return e;
  if (!src.empty()) e = hipMemcpyAsync(*dst, src.data(), sizeof(X) * src.size(), hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(c->stream);
}

// tile choices of the explicit kernel for a grid (2D: tx cells in x per tile
// and lz cell rows per chunk; 3D: tx x ty cells per layer, lz layers)
void choose_tiles(imex_ctx* c) {
  ExplicitArgs& a = c->ea;
  const HostSetup& hs = c->hs;
  const int n = hs.n;
  auto env = [](const char* k, int d) {
    const char* v = std::getenv(k);
    return v ? std::max(1, std::atoi(v)) : d;
  };
  if (hs.dim == 2) {
    // tiles of tx x ty cells: at most kOwnMax owned nodes per thread, and
    // enough workgroups to fill the chip
    a.dim = 2;
    a.p = hs.p;
    int tx = 8, ty = 8;
    auto owned = [&](int x, int y) { return (int64_t)(x * hs.p + 1) * (y * hs.p + 1); };
    while (owned(tx, ty) > 8 * 256) {
      if (ty >= tx) ty /= 2;
      else tx /= 2;
    }
    while (((hs.ne[0] + tx - 1) / tx) * ((hs.ne[1] + ty - 1) / ty) < 512 && (tx > 4 || ty > 2)) {
      if (ty >= tx && ty > 2) ty /= 2;
      else tx /= 2;
    }
    a.tx = env("IMEX_TX", tx);
    a.ty = env("IMEX_TY", ty);
    if (owned(a.tx, a.ty) > 8 * 256) {
      a.tx = tx;
      a.ty = ty;
    }
    a.lz = 1;
    a.mode = 0;
    const char* mv = std::getenv("IMEX_EXPLICIT_MODE");
    if (mv && mv[0] == '3') {
      // LDS tiles on 128-thread workgroups: at most 8 * 128 owned nodes
      a.mode = 3;
      while (owned(a.tx, a.ty) > 8 * 128) {
        if (a.ty >= a.tx) a.ty /= 2;
        else a.tx /= 2;
      }
    }
    // register strips (p <= 5): kStripCells cells per wave, lz rows per wave,
    // about 2048 waves when the grid allows
    if (hs.n <= kStripMaxN && !(mv && (mv[0] == '0' || mv[0] == '3'))) {
      a.mode = (mv && mv[0] == '2') || (!mv && c->fp == 32) ? 2 : 1;
      const int64_t strips = (hs.ne[0] + kStripCells - 1) / kStripCells;
      int64_t lz = (hs.ne[1] * strips + 2047) / 2048;
      lz = std::max<int64_t>(1, std::min<int64_t>(64, lz));
      a.tx = kStripCells;
      a.lz = env("IMEX_LZ", (int)lz);
      a.ty = a.lz;
    }
  } else {
    // largest tile (8 x 8 cells) whose LDS footprint allows two workgroups
    // per CU, shrinking y then x
    a.dim = 3;
    a.p = hs.p;
    a.tx = 8;
    a.ty = 8;
    while (explicit_smem_bytes(a, c->fp) > 80 * 1024 && (a.tx > 1 || a.ty > 1)) {
      if (a.ty >= a.tx && a.ty > 1) a.ty /= 2;
      else a.tx /= 2;
    }
    int lz = 8;
    while (lz > 2 && ((hs.ne[0] + a.tx - 1) / a.tx) * ((hs.ne[1] + a.ty - 1) / a.ty) * ((hs.ne[2] + lz - 1) / lz) < 1024)
      lz /= 2;
    a.tx = env("IMEX_TX", a.tx);
    a.ty = env("IMEX_TY", a.ty);
    a.lz = env("IMEX_LZ", lz);
    // the tensor-product form unless a cell-by-cell form (0: 256-, 4:
    // 512-thread workgroups) is asked for
    const char* mv = std::getenv("IMEX_EXPLICIT_MODE");
    a.mode = mv && mv[0] == '4' ? 4 : (mv && mv[0] == '0' ? 0 : kModeKron);
    if (a.mode == kModeKron) {
      // tiles fixed by the order; chunks of lz layers, at least two
      // workgroups per CU when the grid allows
      a.tx = kKronCX[hs.p];
      a.ty = kKronCY[hs.p];
      const int64_t tiles = ((hs.ne[0] + a.tx - 1) / a.tx) * ((hs.ne[1] + a.ty - 1) / a.ty);
      int kz = 8;
      while (kz > 1 && tiles * ((hs.ne[2] + kz - 1) / kz) < 512) kz /= 2;
      a.lz = env("IMEX_LZ", kz);
    }
  }
  a.ntx = (int)((hs.ne[0] + a.tx - 1) / a.tx);
  a.nty = (int)((hs.ne[1] + a.ty - 1) / a.ty);
  a.nchunk = hs.dim == 3 ? (int)((hs.ne[2] + a.lz - 1) / a.lz) : 1;
}

// state buffers of the explicit kernel for a step from grid[cur]: FP64 writes
// u_{n+1} over u_{n-1}; FP32 updates the increment in place and writes
// u_{n+1} into the other grid buffer
void bind_explicit(const imex_ctx* c, ExplicitArgs& a, int cur) {
  a.un = c->grid[cur].p;
  if (c->fp == 32) {
    a.uw = c->d_delta;
    a.uout = c->grid[1 - cur].p;
    a.write_u = 1;
  } else {
    a.uw = c->grid[1 - cur].p;
    a.uout = nullptr;
    a.write_u = 0;
  }
}

}  // namespace

namespace imex {
hipError_t launch_factor_solve(const imex_ctx* c, const SolveArgs& s, hipStream_t st) {
  if (c->hs.nd)
  {
    const NdLevels L{c->nd_flev.data(), c->nd_fclev.data(), c->nd_blev.data(), c->nd_fper.data(),
                     c->nd_bper.data(), (int)c->nd_flev.size() - 1};
    return launch_nd_solve(s, L, c->fp, st);
  }
  return launch_solve(s, c->n_parts, c->n_schur_chunks, c->n_schur_chain, c->n_part_chunks, c->n_dense_chunks,
                      c->fp, st);
}
}  // namespace imex

namespace {

bool debug_on() {
  const char* v = std::getenv("IMEX_DEBUG");
  return v && v[0] == '1';
}

// whether the steps record the per-kernel timing events: the factorised
// step without leap-frog substeps, launched one by one
bool times_steps(const imex_ctx* c) {
  return c->timing && c->lts_m == 0 && c->solver == IMEX_SOLVER_CHOLESKY && !c->learned;
}

// One step from grid[which_cur].  slot >= 0 records the timing events of that
// slot between the step's launches.
imex_status run_step(imex_ctx* c, int which_cur, hipStream_t stream, int slot = -1) {
  const int fp = c->fp;
  ExplicitArgs a = c->ea;
  bind_explicit(c, a, which_cur);
  hipEvent_t* ev = slot >= 0 ? &c->tev[4 * (size_t)slot] : nullptr;
  auto mark = [&](int i) { return ev ? hipEventRecord(ev[i], stream) : hipSuccess; };
  if (c->lts_m > 0) {
    // leap-frog with substeps on the fine rows: the coarse term and the
    // saved u_{n-1} first, then the explicit kernel, then the substeps
    LtsArgs l = c->la;
    l.un = static_cast<const double*>(c->grid[which_cur].p);
    l.uw = static_cast<double*>(c->grid[1 - which_cur].p);
    hipError_t e = l.nf > 0 ? launch_lts_pre(l, stream) : hipSuccess;
    if (e == hipSuccess) e = launch_explicit(a, fp, stream);
    if (e == hipSuccess) e = l.nf > 0 ? launch_lts_step(l, stream) : launch_add_int(c->d_step, 1, stream);
    if (e != hipSuccess) return c->hipfail(e, "leap-frog step kernels");
    return IMEX_OK;
  }
  if (debug_on())
    std::fprintf(stderr, "[imex] explicit dim=%d p=%d tx=%d ty=%d lz=%d tiles=%dx%d chunks=%d smem=%zu\n", a.dim,
                 a.p, a.tx, a.ty, a.lz, a.ntx, a.nty, a.nchunk, explicit_smem_bytes(a, fp));
  hipError_t e = mark(0);
  if (e == hipSuccess) e = launch_explicit(a, fp, stream);
  if (e == hipSuccess) e = mark(1);
  if (e != hipSuccess) return c->hipfail(e, "explicit step kernel");
  const int64_t nc = (int64_t)c->hs.c_nodes.size();
  if (nc > 0) {
    RhsArgs r = c->ra;
    r.ugrid = c->grid[1 - which_cur].p;
    e = launch_rhs(r, fp, stream);
    if (e == hipSuccess) e = mark(2);
    if (e != hipSuccess) return c->hipfail(e, "rhs kernel");
    SolveArgs s = c->sa;
    s.ugrid = c->grid[1 - which_cur].p;
    s.advance_step = 1;
    if (c->learned) {
      const imex_status st = learned_collect(c, stream);
      if (st != IMEX_OK) return st;
    }
    if (c->solver != IMEX_SOLVER_CHOLESKY) {
      const imex_status st = learned_solve_step(c, s, stream);
      if (st != IMEX_OK || !c->learned) return st;
      return learned_collect_after(c, stream);
    }
    e = launch_factor_solve(c, s, stream);
    if (e == hipSuccess) e = mark(3);
    if (e != hipSuccess) return c->hipfail(e, "solve kernels");
    if (c->learned) return learned_collect_after(c, stream);
  } else {
    e = launch_add_int(c->d_step, 1, stream);
    if (e == hipSuccess) e = mark(2);
    if (e == hipSuccess) e = mark(3);
    if (e != hipSuccess) return c->hipfail(e, "step counter");
  }
  return IMEX_OK;
}

// kGraphChunk steps from grid[start_cur], captured on the context's stream
imex_status capture_chunk(imex_ctx* c, int start_cur, hipGraph_t* out) {
  hipGraph_t g = nullptr;
  HIPCHECK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "begin capture");
  int cur = start_cur;
  imex_status st = IMEX_OK;
  for (int k = 0; k < kGraphChunk && st == IMEX_OK; ++k) {
    st = run_step(c, cur, c->stream);
    cur = 1 - cur;
  }
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (st != IMEX_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return c->hipfail(e, "end capture");
  *out = g;
  return IMEX_OK;
}

imex_status ensure_graph(imex_ctx* c, int start_cur) {
  if (c->graph[start_cur]) return IMEX_OK;
  hipGraph_t g = nullptr;
  imex_status st = capture_chunk(c, start_cur, &g);
  if (st != IMEX_OK) return st;
  hipError_t e = hipGraphInstantiate(&c->graph[start_cur], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return c->hipfail(e, "graph instantiate");
  return IMEX_OK;
}

// Failure detection: scan the state (both grid buffers, the FP32 increment,
// u^c | v^c | a^c) for NaN or Inf and wait for the result.
imex_status check_state(imex_ctx* c) {
  const int64_t ng = c->hs.n_grid, nc = (int64_t)c->hs.c_nodes.size();
  HIPCHECK(c, launch_set_int(c->d_check, 0, c->stream), "finite check");
  for (int k = 0; k < 2; ++k)
    HIPCHECK(c, launch_check_finite(c->grid[k].p, ng, c->fp, c->d_check, c->stream), "finite check");
  if (c->d_delta) HIPCHECK(c, launch_check_finite(c->d_delta, ng, 32, c->d_check, c->stream), "finite check");
  HIPCHECK(c, launch_check_finite(c->cstate.p, 3 * nc, 64, c->d_check, c->stream), "finite check");
  int flag = 0;
  HIPCHECK(c, hipMemcpyAsync(&flag, c->d_check, sizeof(int), hipMemcpyDeviceToHost, c->stream), "finite check");
  HIPCHECK(c, hipStreamSynchronize(c->stream), "finite check");
  if (flag) return c->fail(IMEX_EUNSTABLE, "NaN or Inf in the state after step " + std::to_string(c->steps_taken));
  return IMEX_OK;
}

bool use_graphs() {
  const char* v = std::getenv("IMEX_NO_GRAPH");
  return !(v && v[0] == '1');
}

}  // namespace

extern "C" {

imex_status imex_setup_mesh(const imex_mesh_desc* d, void* hip_stream, imex_ctx** out) {
  if (!d || !out) {
    g_setup_error = "null argument";
    return IMEX_EINVAL;
  }
  *out = nullptr;
  imex_ctx* c = new (std::nothrow) imex_ctx();
  if (!c) {
    g_setup_error = "out of host memory";
    return IMEX_ENOMEM;
  }
  if (d->explicit_fp != 64 && d->explicit_fp != 32) {
    g_setup_error = "explicit_fp must be 64 or 32";
    delete c;
    return IMEX_EINVAL;
  }
  c->fp = d->explicit_fp;
  c->host_only = d->device_mode == IMEX_HOST_ONLY;
  std::string m;
  try {
    m = setup_mesh_host(c->hs, d->dim, d->n_cells, d->extent, d->p, d->rho, d->c, d->alpha_f,
                        d->tree_depth, d->n_holes, d->hole_center, d->hole_radius, d->source,
                        d->dt, d->cfl, d->n_forced_cut, d->forced_cut);
  } catch (const std::bad_alloc&) {
    m = "out of host memory during setup";
  } catch (const std::exception& ex) {
    m = ex.what();
  }
  if (!m.empty()) {
    g_setup_error = m;
    delete c;
    return IMEX_EINVAL;
  }
  if (!c->host_only) {
    const HostSetup& hs = c->hs;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) {
      if (hip_stream) c->stream = static_cast<hipStream_t>(hip_stream);
      else {
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        c->own_stream = (e == hipSuccess);
      }
    }
    // explicit-part tables: cell flags and the point source box
    if (e == hipSuccess) e = upload(c, &c->d_flags, hs.cell_flag);
    if (e == hipSuccess && hs.dim == 3) {
      // IMEX_KRON_REST_ALL=1 sends every d node through the cell-by-cell
      // rest kernel (a check of that kernel on meshes that have no such nodes)
      const char* ra = std::getenv("IMEX_KRON_REST_ALL");
      if (ra && ra[0] == '1') {
        e = upload(c, &c->d_kron_mask, std::vector<uint32_t>(hs.kron_mask.size(), 0u));
        if (e == hipSuccess) e = upload(c, &c->d_kron_rest, hs.d_nodes);
        c->ea.n_rest = (int64_t)hs.d_nodes.size();
      } else {
        e = upload(c, &c->d_kron_mask, hs.kron_mask);
        if (e == hipSuccess) e = upload(c, &c->d_kron_rest, hs.kron_rest);
        c->ea.n_rest = (int64_t)hs.kron_rest.size();
      }
      c->ea.kron_mask = c->d_kron_mask;
      c->ea.kron_rest = c->d_kron_rest;
    }
    if (e == hipSuccess) {
      for (int k = 0; k < 3; ++k) {
        c->sbox_lo[k] = INT64_MAX;
        c->sbox_hi[k] = INT64_MIN;
      }
      for (int64_t g : hs.src_nodes) {
        const int64_t I[3] = {g % hs.nn[0], (g / hs.nn[0]) % hs.nn[1], g / (hs.nn[0] * hs.nn[1])};
        for (int k = 0; k < 3; ++k) {
          c->sbox_lo[k] = std::min(c->sbox_lo[k], I[k]);
          c->sbox_hi[k] = std::max(c->sbox_hi[k], I[k] + 1);
        }
      }
      const int64_t bx = c->sbox_hi[0] - c->sbox_lo[0], by = c->sbox_hi[1] - c->sbox_lo[1];
      const int64_t bz = c->sbox_hi[2] - c->sbox_lo[2];
      std::vector<double> dense((size_t)(bx * by * bz), 0.0);
      for (size_t t = 0; t < hs.src_nodes.size(); ++t) {
        const int64_t g = hs.src_nodes[t];
        const int64_t I[3] = {g % hs.nn[0], (g / hs.nn[0]) % hs.nn[1], g / (hs.nn[0] * hs.nn[1])};
        dense[((I[2] - c->sbox_lo[2]) * by + (I[1] - c->sbox_lo[1])) * bx + (I[0] - c->sbox_lo[0])] =
            hs.src_vals[t];
      }
      e = upload(c, &c->d_src, dense);
    }
    if (e == hipSuccess) {
      void* sp = nullptr;  // device copy of the sampling scratch (once per device)
      e = scratch_address(c->device, &sp);
    }
    if (e == hipSuccess) e = c->alloc(&c->d_step, sizeof(int) * 4);
    if (e == hipSuccess) e = c->alloc(&c->d_check, sizeof(int) * 4);
    if (e != hipSuccess) {
      g_setup_error = std::string("HIP: ") + hipGetErrorString(e);
      imex_destroy(c);
      return IMEX_EHIP;
    }
    ExplicitArgs& a = c->ea;
    a.dim = hs.dim;
    a.p = hs.p;
    for (int k = 0; k < 3; ++k) {
      a.ne[k] = hs.ne[k];
      a.nn[k] = hs.nn[k];
      a.sbox_lo[k] = c->sbox_lo[k];
      a.sbox_hi[k] = c->sbox_hi[k];
    }
    a.flags = c->d_flags;
    a.src_dense = c->d_src;
    a.step = c->d_step;
    double J = 1.0;
    for (int k = 0; k < hs.dim; ++k) J *= 0.5 * hs.h[k];
    a.mass_scale = hs.rho * J;
    if (hs.dim == 2) {
      a.s[0] = hs.kappa * hs.h[1] / hs.h[0];
      a.s[1] = hs.kappa * hs.h[0] / hs.h[1];
      a.s[2] = 0;
    } else {
      a.s[0] = hs.kappa * hs.h[1] * hs.h[2] / (2 * hs.h[0]);
      a.s[1] = hs.kappa * hs.h[0] * hs.h[2] / (2 * hs.h[1]);
      a.s[2] = hs.kappa * hs.h[0] * hs.h[1] / (2 * hs.h[2]);
    }
    a.dt2 = hs.dt * hs.dt;
    if (c->fp == 64) {
      // CDM sum step u_{n+1} = 2 u_n - u_{n-1} + dt^2 a_n (Eq. CDMstep)
      a.c1 = 2.0;
      a.c2 = -1.0;
      a.c3 = 1.0;
    } else {
      // the same step in increment form: d_{n+1/2} = d_{n-1/2} + dt^2 a_n,
      // u_{n+1} = u_n + d_{n+1/2}
      a.c1 = 0.0;
      a.c2 = 1.0;
      a.c3 = 1.0;
    }
    a.ft_offset = 0;
    // the 1D operators and GLL weights are symmetric and centro-symmetric;
    // every entry takes the value at its canonical position (the smallest of
    // the equivalent indices), so the tables are exactly so and the kernels
    // may read any of the equivalent entries
    const int n1 = hs.n, P1 = hs.p;
    for (int r = 0; r < n1; ++r)
      for (int q = 0; q < n1; ++q) {
        const int k = std::min(std::min(r * n1 + q, q * n1 + r),
                               std::min((P1 - r) * n1 + (P1 - q), (P1 - q) * n1 + (P1 - r)));
        a.Kh[r * n1 + q] = hs.ref.Kh[k];
        a.Mh[r * n1 + q] = hs.ref.Mh[k];
      }
    for (int i = 0; i < n1; ++i) a.w[i] = hs.ref.w[std::min(i, P1 - i)];
    choose_tiles(c);
    const size_t smem = explicit_smem_bytes(a, c->fp);
    if (smem > 160 * 1024) {
      g_setup_error = "explicit tile does not fit in LDS";
      imex_destroy(c);
      return IMEX_EINVAL;
    }
    e = prepare_explicit(a, c->fp);
    if (e != hipSuccess) {
      g_setup_error = std::string("HIP: ") + hipGetErrorString(e);
      imex_destroy(c);
      return IMEX_EHIP;
    }
  }
  *out = c;
  return IMEX_OK;
}

imex_status imex_query(const imex_ctx* c, imex_info* o) {
  if (!c || !o) return IMEX_EINVAL;
  const HostSetup& hs = c->hs;
  std::memset(o, 0, sizeof(*o));
  o->n_grid = hs.n_grid;
  o->n_active = hs.n_active;
  o->n_d = (int64_t)hs.d_nodes.size();
  o->n_c = (int64_t)hs.c_nodes.size();
  o->n_cells_empty = hs.counts[kEmpty];
  o->n_cells_cut = hs.counts[kCut];
  o->n_cells_uncut = hs.counts[kUncut];
  o->nnz_kc = (int64_t)hs.Kc.col.size();
  o->nnz_factor = hs.nnz_factor;
  {
    const DissectedFactor& F = hs.fac;
    o->nnz_part_inv = c->assembled && !c->host_only ? c->nnz_part_inv : (F.dense ? (int64_t)F.pinv.size() : 0);
    o->nnz_coupling = (int64_t)F.zvals.size();
    o->nnz_sep_inv = (int64_t)F.schur_inv.size();
    int64_t chain = 0;
    if (!F.dense)
      for (const ChainMeta& cm : F.parts) chain += cm.nnz;
    for (const ChainMeta& cm : F.schur)
      if (cm.coff == -2) chain += cm.nnz;
    o->nnz_chain = chain;
    o->coupling_passes = hs.nd ? 0 : (c->n_sym_blocks > 0 ? 1 : 2);
  }
  o->n_components = (int64_t)hs.layout.size();
  o->factor_form = hs.nd ? 1 : 0;
  if (hs.nd) {
    const NdFactor& N = hs.ndf;
    o->nd_supernodes = (int64_t)N.sn.size();
    o->nd_levels = N.height + 1;
    o->nd_nnz_L = N.nnz_L;
    o->nd_update_rows = N.w_len;
    o->nd_max_m = N.max_m;
    o->nd_max_mk = N.max_mk;
  }
  for (int k = 0; k < 3; ++k) o->grid_dims[k] = hs.nn[k];
  o->steps_taken = c->steps_taken;
  o->dt = hs.dt;
  o->dt_crit_uncut = hs.dt_crit;
  o->field_bytes[0] = o->field_bytes[1] = (size_t)hs.n_grid * c->grid_elem();
  o->field_bytes[2] = 3 * sizeof(double) * hs.c_nodes.size();
  return IMEX_OK;
}

imex_status imex_bind_buffers(imex_ctx* c, void* const* ptrs, const size_t* bytes, int n) {
  if (!c || !ptrs || !bytes || n != 3) return c ? c->fail(IMEX_EINVAL, "bind needs 3 buffers") : IMEX_EINVAL;
  if (c->host_only) return c->fail(IMEX_ESTATE, "host-only context has no device buffers");
  if (c->assembled) return c->fail(IMEX_ESTATE, "bind buffers before imex_assemble_implicit_block");
  imex_info inf;
  imex_query(c, &inf);
  for (int k = 0; k < 3; ++k) {
    if (bytes[k] < inf.field_bytes[k] || (!ptrs[k] && inf.field_bytes[k] > 0))
      return c->fail(IMEX_EINVAL, "bound buffer too small");
  }
  c->grid[0] = {ptrs[0], false};
  c->grid[1] = {ptrs[1], false};
  c->cstate = {ptrs[2], false};
  return IMEX_OK;
}

imex_status imex_set_check_finite(imex_ctx* c, int on) {
  if (!c) return IMEX_EINVAL;
  if (c->host_only) return c->fail(IMEX_ESTATE, "host-only context cannot step");
  c->check_finite = on != 0;
  return IMEX_OK;
}

imex_status imex_set_step_timing(imex_ctx* c, int on) {
  if (!c) return IMEX_EINVAL;
  if (c->host_only) return c->fail(IMEX_ESTATE, "host-only context cannot step");
  if (on && c->tev.empty()) {
    c->tev.assign(4 * (size_t)kTimedSteps, nullptr);
    for (hipEvent_t& ev : c->tev) HIPCHECK(c, hipEventCreate(&ev), "timing events");
  }
  c->timing = on != 0;
  c->tev_count = 0;
  return IMEX_OK;
}

imex_status imex_step_timing(imex_ctx* c, double* ms) {
  if (!c || !ms) return IMEX_EINVAL;
  if (!c->timing || c->tev_count == 0)
    return c->fail(IMEX_ESTATE, "no timed step: enable step timing, then step the factorised method");
  HIPCHECK(c, hipStreamSynchronize(c->stream), "sync");
  const int n = (int)std::min<int64_t>(c->tev_count, kTimedSteps);
  double sum[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < n; ++k)
    for (int g = 0; g < 3; ++g) {
      float t = 0.f;
      HIPCHECK(c, hipEventElapsedTime(&t, c->tev[4 * (size_t)k + g], c->tev[4 * (size_t)k + g + 1]), "event time");
      sum[g] += t;
    }
  for (int g = 0; g < 3; ++g) ms[g] = sum[g] / n;
  return IMEX_OK;
}

imex_status imex_set_newmark_beta(imex_ctx* c, double beta) {
  if (!c) return IMEX_EINVAL;
  if (c->assembled) return c->fail(IMEX_ESTATE, "set beta before imex_assemble_implicit_block");
  if (!(beta >= 0.0 && beta <= 0.5)) return c->fail(IMEX_EINVAL, "beta must lie in [0, 1/2]");
  c->hs.beta = beta;
  return IMEX_OK;
}

imex_status imex_set_leapfrog(imex_ctx* c, int m) {
  if (!c) return IMEX_EINVAL;
  if (c->assembled) return c->fail(IMEX_ESTATE, "set the substeps before imex_assemble_implicit_block");
  if (m < 0 || m > 4096) return c->fail(IMEX_EINVAL, "substeps must lie in [0, 4096]");
  c->lts_m = m;
  if (m > 0) c->hs.beta = 0.0;  // the c block is explicit: S = M^cc for the initial acceleration
  return IMEX_OK;
}

imex_status imex_set_cut_mass(imex_ctx* c, int kind) {
  if (!c) return IMEX_EINVAL;
  if (c->assembled) return c->fail(IMEX_ESTATE, "set the cut-cell mass before imex_assemble_implicit_block");
  if (kind != IMEX_CUT_MASS_CONSISTENT && kind != IMEX_CUT_MASS_HRZ) return c->fail(IMEX_EINVAL, "unknown mass kind");
  c->hs.hrz_cut_mass = kind == IMEX_CUT_MASS_HRZ;
  return IMEX_OK;
}

imex_status imex_global_critical_step(imex_ctx* c, int max_iter, double rel_tol, double* dt_crit) {
  if (!c || !dt_crit || max_iter < 1 || !(rel_tol >= 0.0)) return IMEX_EINVAL;
  if (!c->assembled) return c->fail(IMEX_ESTATE, "assemble the implicit block first");
  try {
    *dt_crit = global_critical_step(c->hs, max_iter, rel_tol);
  } catch (const std::bad_alloc&) {
    return c->fail(IMEX_ENOMEM, "out of host memory in the critical-step iteration");
  }
  return IMEX_OK;
}

imex_status imex_assemble_implicit_block(imex_ctx* c, int solver) {
  if (!c) return IMEX_EINVAL;
  if (solver != IMEX_SOLVER_CHOLESKY) return c->fail(IMEX_EINVAL, "unknown solver");
  if (c->assembled) return c->fail(IMEX_ESTATE, "already assembled");
  if (c->lts_m > 0 && (!c->hs.hrz_cut_mass || c->fp != 64))
    return c->fail(IMEX_EINVAL, "the leap-frog substepping needs the HRZ-lumped cut-cell mass and FP64 state");
  bool notspd = false;
  std::string m;
  if (!c->host_only) {
    // large parts and separator systems are inverted on the device, so they
    // can take the dense form too
    c->hs.dense_inverse = gpu_spd_inverse;
    HIPCHECK(c, hipGetDevice(&c->hs.inverse_device), "device");
    int lds = 0;  // the separator kernel keeps r_S of a whole system in LDS
    HIPCHECK(c, hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->hs.inverse_device),
             "device attribute");
    c->hs.dense_rows = std::min<int64_t>(kDenseRowsDevice, (lds - 1024) / (int64_t)sizeof(double));
    if (const char* v = std::getenv("IMEX_DEVICE_INVERSE_MIN")) c->hs.device_inverse_min = std::max(1, std::atoi(v));
  }
  if (const char* v = std::getenv("IMEX_DENSE_ROWS")) c->hs.dense_rows = std::max(1, std::atoi(v));
  if (const char* v = std::getenv("IMEX_PART_ROWS")) c->hs.part_rows = std::max(1, std::atoi(v));
  if (const char* v = std::getenv("IMEX_FACTOR")) {
    const std::string f(v);
    c->hs.factor_form = f == "dissected" ? 1 : f == "nd" ? 2 : 0;
  }
  if (const char* v = std::getenv("IMEX_ND_LEAF")) c->hs.nd_leaf = std::max(1, std::atoi(v));
  if (c->hs.hrz_cut_mass) {
    // HRZ: each cut cell's mass matrix becomes its diagonal, scaled to keep
    // the cell's total mass (the sum of all entries)
    int64_t nb = 1;
    for (int k = 0; k < c->hs.dim; ++k) nb *= c->hs.n;
    for (size_t e = 0; e < c->hs.cut_cells.size(); ++e) {
      double* Me = &c->hs.Me_cut[e * nb * nb];
      double total = 0.0, diag = 0.0;
      for (int64_t k = 0; k < nb * nb; ++k) total += Me[k];
      for (int64_t i = 0; i < nb; ++i) diag += Me[i * nb + i];
      for (int64_t i = 0; i < nb; ++i)
        for (int64_t j = 0; j < nb; ++j) Me[i * nb + j] = i == j ? Me[i * nb + i] * (total / diag) : 0.0;
    }
  }  // (idempotent: a lumped matrix is left as it is)
  try {
    m = assemble_implicit_host(c->hs, &notspd);
  } catch (const std::bad_alloc&) {
    return c->fail(IMEX_ENOMEM, "out of host memory during assembly");
  }
  if (!m.empty()) return c->fail(notspd ? IMEX_ENOTSPD : IMEX_EINVAL, m);
  c->assembled = true;
  if (c->host_only) return IMEX_OK;
  const HostSetup& hs = c->hs;
  const int64_t nc = (int64_t)hs.c_nodes.size();
  // state buffers
  for (int k = 0; k < 2; ++k)
    if (!c->grid[k].p) {
      HIPCHECK(c, c->alloc(&c->grid[k].p, (size_t)hs.n_grid * c->grid_elem()), "alloc grid");
      c->grid[k].owned = true;
    }
  if (!c->cstate.p) {
    HIPCHECK(c, c->alloc(&c->cstate.p, 3 * sizeof(double) * (size_t)nc), "alloc c state");
    c->cstate.owned = true;
  }
  if (c->fp == 32) {
    HIPCHECK(c, c->alloc(&c->d_delta, sizeof(float) * (size_t)hs.n_grid), "alloc increment");
    HIPCHECK(c, hipMemsetAsync(c->d_delta, 0, sizeof(float) * (size_t)hs.n_grid, c->stream), "clear");
  }
  HIPCHECK(c, hipMemsetAsync(c->grid[0].p, 0, (size_t)hs.n_grid * c->grid_elem(), c->stream), "clear");
  HIPCHECK(c, hipMemsetAsync(c->grid[1].p, 0, (size_t)hs.n_grid * c->grid_elem(), c->stream), "clear");
  HIPCHECK(c, hipMemsetAsync(c->cstate.p, 0, 3 * sizeof(double) * (size_t)nc, c->stream), "clear");
  // implicit block
  if (hs.n_grid >= ((int64_t)1 << 31)) return c->fail(IMEX_EINVAL, "grid has 2^31 nodes or more");
  HIPCHECK(c, upload(c, &c->d_rp_d, hs.Kcd.ptr), "upload Kcd");
  HIPCHECK(c, upload(c, &c->d_col_d, std::vector<int32_t>(hs.Kcd.col.begin(), hs.Kcd.col.end())), "upload Kcd");
  HIPCHECK(c, upload(c, &c->d_val_d, hs.Kcd.val), "upload Kcd");
  HIPCHECK(c, upload(c, &c->d_rp_c, hs.Kcc.ptr), "upload Kcc");
  HIPCHECK(c, upload(c, &c->d_col_c, std::vector<int32_t>(hs.Kcc.col.begin(), hs.Kcc.col.end())), "upload Kcc");
  HIPCHECK(c, upload(c, &c->d_val_c, hs.Kcc.val), "upload Kcc");
  HIPCHECK(c, upload(c, &c->d_fxc, hs.fxc), "upload fxc");
  HIPCHECK(c, upload(c, &c->d_cnodes, hs.c_nodes), "upload c nodes");
  const DissectedFactor& F = hs.fac;
  c->n_parts = (int64_t)F.parts.size();
  c->n_comp = (int64_t)F.schur.size();
  // parts above 1024 rows: A_pp^-1 as the lower triangle in 64 x 64 blocks
  // (row-major, zero-padded), (part, I, J) per block, and the offsets of the
  // parts' partial sums; the dense chunk list keeps the Z_p^T chunks only
  int64_t max_part = 0;
  for (const ChainMeta& cm : F.parts) max_part = std::max<int64_t>(max_part, cm.nrows);
  const bool sym = F.dense && max_part > kDenseRows;
  std::vector<ChainMeta> parts_dev = F.parts;
  std::vector<double> pinv_sym;
  std::vector<SymBlock> sym_blocks;
  std::vector<int64_t> sym_poff, dchunks = F.dense_chunks;
  std::vector<CorrChunk> corr_chunks;
  std::vector<double> zrow;
  int64_t partial_len = 0;
  if (sym) {
    constexpr int B = 64;
    for (size_t p = 0; p < parts_dev.size(); ++p) {
      ChainMeta& cm = parts_dev[p];
      const int64_t n = cm.nrows, nbk = (n + B - 1) / B;
      const double* P = &F.pinv[F.parts[p].doff];
      cm.doff = (int64_t)pinv_sym.size();
      pinv_sym.resize(pinv_sym.size() + (size_t)(nbk * (nbk + 1) / 2) * B * B, 0.0);
      double* dst = &pinv_sym[cm.doff];
      for (int64_t I = 0; I < nbk; ++I)
        for (int64_t J = 0; J <= I; ++J, dst += B * B) {
          sym_blocks.push_back(SymBlock{(int64_t)(dst - pinv_sym.data()), cm.row0, partial_len + (I * nbk + J) * B,
                                        partial_len + (J * nbk + I) * B, (int32_t)n, (int32_t)I, (int32_t)J, 0});
          for (int64_t r = 0; r < B && I * B + r < n; ++r)
            for (int64_t q = 0; q < B && J * B + q < n; ++q) dst[r * B + q] = P[(I * B + r) * n + J * B + q];
        }
      sym_poff.push_back(partial_len);
      partial_len += nbk * nbk * B;
    }
    dchunks.clear();
    for (size_t k = 0; k + 2 < F.dense_chunks.size(); k += 3) {
      if (F.dense_chunks[k] == 1) dchunks.insert(dchunks.end(), F.dense_chunks.begin() + k, F.dense_chunks.begin() + k + 3);
      else {
        const ChainMeta& cm = F.parts[F.dense_chunks[k + 1]];
        const int64_t first = F.dense_chunks[k + 2], na = std::max<int64_t>(cm.nadj, 0);
        corr_chunks.push_back(CorrChunk{na > 0 ? cm.zoff + first * na : 0, cm.row0 + first, cm.adj0, (int32_t)na,
                                        (int32_t)std::min<int64_t>(16, cm.nrows - first), na});
      }
    }
    // Z_p row-major (n x nadj): in the wide form only the correction reads it,
    // four rows per wave along contiguous rows
    zrow.resize(F.zvals.size());
    for (const ChainMeta& cm : F.parts) {
      if (cm.nadj <= 0 || cm.zoff < 0) continue;
      const double* Zc = &F.zvals[cm.zoff];
      double* Zr = &zrow[cm.zoff];
      for (int64_t k = 0; k < cm.nadj; ++k)
        for (int64_t i = 0; i < cm.nrows; ++i) Zr[i * cm.nadj + k] = Zc[k * cm.nrows + i];
    }
  }
  c->n_corr_chunks = (int64_t)corr_chunks.size();
  HIPCHECK(c, upload(c, &c->d_corrchunks, corr_chunks), "upload factor");
  // descriptors of the plain form's chunks (same order as the chunk lists)
  std::vector<DenseChunk> pd_chunks;
  std::vector<CorrChunk> part_corr;
  std::vector<SepChunk> sep_chunks;
  if (!sym) {
    if (F.dense)
      for (size_t k = 0; k + 2 < F.dense_chunks.size(); k += 3) {
        const int64_t kind = F.dense_chunks[k], first = F.dense_chunks[k + 2];
        const ChainMeta& cm = F.parts[F.dense_chunks[k + 1]];
        const int64_t rows = std::min<int64_t>(16, (kind == 0 ? cm.nrows : cm.nadj) - first);
        pd_chunks.push_back(DenseChunk{(kind == 0 ? cm.doff : cm.zoff) + first * cm.nrows, cm.row0,
                                       (kind == 0 ? cm.row0 : cm.coff) + first, cm.nrows, (int32_t)rows,
                                       (int32_t)kind, 0});
      }
    for (size_t k = 0; k + 1 < F.part_chunks.size(); k += 2) {
      const ChainMeta& cm = F.parts[F.part_chunks[k]];
      const int64_t r0 = F.part_chunks[k + 1], na = std::max<int64_t>(cm.nadj, 0);
      part_corr.push_back(CorrChunk{na > 0 ? cm.zoff + r0 : 0, cm.row0 + r0, cm.adj0, (int32_t)na,
                                    (int32_t)std::min<int64_t>(64, cm.nrows - r0), cm.nrows});
    }
    for (size_t k = 0; k + 1 < F.schur_chunks.size(); k += 2) {
      const ChainMeta& cm = F.schur[F.schur_chunks[k]];
      const int64_t r0 = F.schur_chunks[k + 1];
      sep_chunks.push_back(SepChunk{cm.voff + r0 * cm.nrows, cm.row0, cm.nrows, (int32_t)r0,
                                    (int32_t)std::min<int64_t>(16, cm.nrows - r0), 0});
    }
  }
  HIPCHECK(c, upload(c, &c->d_pdchunks, pd_chunks), "upload factor");
  HIPCHECK(c, upload(c, &c->d_partcorr, part_corr), "upload factor");
  HIPCHECK(c, upload(c, &c->d_sepchunks, sep_chunks), "upload factor");
  c->n_sym_blocks = (int64_t)sym_blocks.size();
  c->nnz_part_inv = sym ? (int64_t)pinv_sym.size() : (F.dense ? (int64_t)F.pinv.size() : 0);
  HIPCHECK(c, upload(c, &c->d_symblocks, sym_blocks), "upload factor");
  HIPCHECK(c, upload(c, &c->d_sympoff, sym_poff), "upload factor");
  HIPCHECK(c, c->alloc(&c->d_sympartial, sizeof(double) * std::max<int64_t>(partial_len, 1)), "alloc work");
  HIPCHECK(c, upload(c, &c->d_parts, parts_dev), "upload factor");
  HIPCHECK(c, upload(c, &c->d_schur, F.schur), "upload factor");
  HIPCHECK(c, upload(c, &c->d_cvals, F.vals), "upload factor");
  HIPCHECK(c, upload(c, &c->d_cints, F.ints), "upload factor");
  HIPCHECK(c, upload(c, &c->d_zvals, sym ? zrow : F.zvals), "upload factor");
  for (const ChainMeta& cm : F.schur)
    if (cm.coff != -2 && cm.nrows > std::max<int64_t>(hs.dense_rows, kDenseRows))
      return c->fail(IMEX_EINVAL, "a dense separator system exceeds the dense-row limit");
  HIPCHECK(c, upload(c, &c->d_schain, F.schur_chain), "upload factor");
  c->n_schur_chain = (int64_t)F.schur_chain.size();
  HIPCHECK(c, upload(c, &c->d_sinv, F.schur_inv), "upload factor");
  HIPCHECK(c, upload(c, &c->d_schunks, F.schur_chunks), "upload factor");
  HIPCHECK(c, upload(c, &c->d_pchunks, F.part_chunks), "upload factor");
  c->n_schur_chunks = (int64_t)F.schur_chunks.size() / 2;
  HIPCHECK(c, upload(c, &c->d_pinv, sym ? pinv_sym : F.pinv), "upload factor");
  HIPCHECK(c, upload(c, &c->d_dchunks, dchunks), "upload factor");
  c->n_dense_chunks = (int64_t)dchunks.size() / 3;
  c->n_part_chunks = (int64_t)F.part_chunks.size() / 2;
  HIPCHECK(c, upload(c, &c->d_cprowptr, F.cp_rowptr), "upload factor");
  HIPCHECK(c, upload(c, &c->d_cpptr, F.cp_ptr), "upload factor");
  HIPCHECK(c, upload(c, &c->d_cpcol, F.cp_col), "upload factor");
  HIPCHECK(c, upload(c, &c->d_cpval, F.cp_val), "upload factor");
  HIPCHECK(c, upload(c, &c->d_sepsrc, F.sep_src), "upload factor");
  HIPCHECK(c, c->alloc(&c->d_cbuf, sizeof(double) * std::max<int64_t>(F.coupling_slots, 1)), "alloc work");
  HIPCHECK(c, c->alloc(&c->d_work, sizeof(double) * std::max<int64_t>(nc, 1)), "alloc work");
  HIPCHECK(c, c->alloc(&c->d_pred, sizeof(double) * std::max<int64_t>(nc, 1)), "alloc predictor");
  HIPCHECK(c, c->alloc(&c->d_rs, sizeof(double) * std::max<int64_t>(nc, 1)), "alloc work");
  HIPCHECK(c, c->alloc(&c->d_w, sizeof(double) * std::max<int64_t>(nc, 1)), "alloc work");
  if (hs.nd) {
    // nested-dissection factor: values, struct lists, gather slots, and the
    // chunks of every level (forward: rows of [L_ss^-1; C_s], backward:
    // columns), 4 x kNdRows = 16 rows per chunk
    const NdFactor& N = hs.ndf;
    constexpr int32_t kChunk = 16;
    // forward of small supernodes (m <= 64 by default, IMEX_ND_COLS=<m> up
    // to kNdColsMaxM; 0 keeps every supernode on the row-per-wave form): 64
    // output rows per chunk, one thread per row
    const char* cv = std::getenv("IMEX_ND_COLS");
    const int32_t cols_max = cv ? std::min<int32_t>(std::max(0, std::atoi(cv)), kNdColsMaxM) : 64;
    std::vector<NdChunk> fch, fcch, bch;
    c->nd_flev.assign(N.height + 2, 0);
    c->nd_fclev.assign(N.height + 2, 0);
    c->nd_blev.assign(N.height + 2, 0);
    c->nd_fper.assign(N.height + 1, 1);
    c->nd_bper.assign(N.height + 1, 1);
    // values in flight per lane and row: enough for one pass over the rows
    // of 90 % of the level's chunks (longer rows take more passes), at most
    // 8 forward and 4 backward (register budget of the backward kernel), and
    // at most 2 on levels of more than 1024 chunks (occupancy)
    auto per_of = [](std::vector<int32_t>& len, int cap) -> int8_t {
      if (len.empty()) return 1;
      if (len.size() > 1024) cap = std::min(cap, 2);
      const size_t i = (len.size() * 9) / 10;
      std::nth_element(len.begin(), len.begin() + i, len.end());
      const int32_t q = (len[i] + 63) / 64;
      return (int8_t)std::min(cap, q <= 1 ? 1 : q <= 2 ? 2 : q <= 4 ? 4 : 8);
    };
    for (int32_t h = 0; h <= N.height; ++h) {
      c->nd_flev[h] = (int64_t)fch.size();
      c->nd_fclev[h] = (int64_t)fcch.size();
      c->nd_blev[h] = (int64_t)bch.size();
      std::vector<int32_t> flen, blen;  // longest row of each chunk
      for (const NdSnode& q : N.sn) {
        if (q.height != h) continue;
        for (int32_t j = 0; j < q.m; j += kChunk) blen.push_back(q.m - j + q.k);
        if (q.m > cols_max)
          for (int32_t r = 0; r < q.m + q.k; r += kChunk) flen.push_back(std::min(q.m, r + kChunk));
      }
      c->nd_fper[h] = per_of(flen, 8);
      c->nd_bper[h] = per_of(blen, 4);
      for (const NdSnode& q : N.sn) {
        if (q.height != h) continue;
        if (q.m <= cols_max) {
          for (int32_t r = 0; r < q.m + q.k; r += 64)
            fcch.push_back(NdChunk{q.boff, q.c0, q.woff, q.soff, q.goff, q.m, q.k, r, std::min(64, q.m + q.k - r)});
        } else {
          for (int32_t r = 0; r < q.m + q.k; r += kChunk)
            fch.push_back(NdChunk{q.foff, q.c0, q.woff, q.soff, q.goff, q.m, q.k, r, std::min(kChunk, q.m + q.k - r)});
        }
        for (int32_t j = 0; j < q.m; j += kChunk)
          bch.push_back(NdChunk{q.boff, q.c0, q.woff, q.soff, q.goff, q.m, q.k, j, std::min(kChunk, q.m - j)});
      }
    }
    c->nd_flev[N.height + 1] = (int64_t)fch.size();
    c->nd_fclev[N.height + 1] = (int64_t)fcch.size();
    c->nd_blev[N.height + 1] = (int64_t)bch.size();
    if (N.max_mk * (int64_t)sizeof(double) > 150 * 1024)
      return c->fail(IMEX_EINVAL, "a supernode of the nested dissection is too large for the LDS");
    HIPCHECK(c, upload(c, &c->d_ndf, N.fwd), "upload factor");
    HIPCHECK(c, upload(c, &c->d_ndb, N.bwd), "upload factor");
    HIPCHECK(c, upload(c, &c->d_nd_fch, fch), "upload factor");
    HIPCHECK(c, upload(c, &c->d_nd_fcch, fcch), "upload factor");
    HIPCHECK(c, upload(c, &c->d_nd_bch, bch), "upload factor");
    HIPCHECK(c, upload(c, &c->d_nd_st, N.st), "upload factor");
    HIPCHECK(c, upload(c, &c->d_nd_gptr, N.gptr), "upload factor");
    HIPCHECK(c, upload(c, &c->d_nd_gsrc, N.gsrc), "upload factor");
    HIPCHECK(c, c->alloc(&c->d_ndW, sizeof(double) * std::max<int64_t>(N.w_len, 1)), "alloc work");
  }
  if (c->lts_m > 0) {
    LtsRows rows;
    const std::string lm = build_lts_rows(hs, rows);
    if (!lm.empty()) return c->fail(IMEX_EINVAL, lm);
    LtsArgs& l = c->la;
    l.nf = (int64_t)rows.node.size();
    l.nc = rows.nc;
    std::vector<double> minv(rows.mass.size());
    for (size_t i = 0; i < minv.size(); ++i) minv[i] = 1.0 / rows.mass[i];
    int64_t *rpo = nullptr, *rpf = nullptr, *node = nullptr;
    int32_t *colo = nullptr, *colf = nullptr;
    double *valo = nullptr, *valf = nullptr, *dminv = nullptr, *dfx = nullptr, *bufs = nullptr;
    HIPCHECK(c, upload(c, &rpo, rows.Ko.ptr), "upload leap-frog rows");
    HIPCHECK(c, upload(c, &colo, std::vector<int32_t>(rows.Ko.col.begin(), rows.Ko.col.end())), "upload");
    HIPCHECK(c, upload(c, &valo, rows.Ko.val), "upload leap-frog rows");
    HIPCHECK(c, upload(c, &rpf, rows.Kf.ptr), "upload leap-frog rows");
    HIPCHECK(c, upload(c, &colf, std::vector<int32_t>(rows.Kf.col.begin(), rows.Kf.col.end())), "upload");
    HIPCHECK(c, upload(c, &valf, rows.Kf.val), "upload leap-frog rows");
    HIPCHECK(c, upload(c, &dminv, minv), "upload leap-frog rows");
    HIPCHECK(c, upload(c, &dfx, rows.fx), "upload leap-frog rows");
    HIPCHECK(c, upload(c, &node, rows.node), "upload leap-frog rows");
    HIPCHECK(c, c->alloc(&bufs, sizeof(double) * 5 * (size_t)std::max<int64_t>(l.nf, 1)), "alloc leap-frog");
    l.rp_o = rpo;
    l.col_o = colo;
    l.val_o = valo;
    l.rp_f = rpf;
    l.col_f = colf;
    l.val_f = valf;
    l.minv = dminv;
    l.fx = dfx;
    l.node = node;
    l.step = c->d_step;
    l.g = bufs;
    for (int k = 0; k < 3; ++k) l.q[k] = bufs + (size_t)(k + 1) * std::max<int64_t>(l.nf, 1);
    l.uprev = bufs + 4 * (size_t)std::max<int64_t>(l.nf, 1);
    l.uc = static_cast<double*>(c->cstate.p);
    l.m = c->lts_m;
    l.tau2 = (hs.dt / c->lts_m) * (hs.dt / c->lts_m);
  }
  // LDS of the chain kernels: the solution vector plus, when it fits, the
  // chain's factor data
  // solution vector + metadata always; factor values when they fit in 150 KB
  auto base = [](const ChainMeta& cm) {
    return (int64_t)(cm.nrows * sizeof(double) +
                     ((2LL * cm.nrows + cm.nblocks) * sizeof(int32_t) + sizeof(double) - 1) / sizeof(double) *
                         sizeof(double));
  };
  auto need = [&](const ChainMeta& cm) {
    return base(cm) + (int64_t)((cm.nnz + (int64_t)cm.nblocks * kTri) * sizeof(double));
  };
  const int64_t cap = 150 * 1024;
  int64_t sp = 0, ss = 0;
  if (!F.dense)
    for (const ChainMeta& cm : F.parts) {
      if (base(cm) > cap) return c->fail(IMEX_EINVAL, "an implicit part is too large for the LDS");
      sp = std::max(sp, need(cm) <= cap ? need(cm) : base(cm));
    }
  for (const ChainMeta& cm : F.schur)
    if (cm.coff == -2) ss = std::max(ss, need(cm) <= cap ? need(cm) : std::min(base(cm), cap));
  if (const char* v = std::getenv("IMEX_SCHUR_LDS")) ss = std::min<int64_t>(ss, std::max(64, std::atoi(v)));
  double* cs = static_cast<double*>(c->cstate.p);
  RhsArgs& r = c->ra;
  r.nc = nc;
  r.rp_d = c->d_rp_d;
  r.col_d = c->d_col_d;
  r.val_d = c->d_val_d;
  r.rp_c = c->d_rp_c;
  r.col_c = c->d_col_c;
  r.val_c = c->d_val_c;
  r.uc = cs;
  r.vc = cs + nc;
  r.ac = cs + 2 * nc;
  r.fxc = c->d_fxc;
  r.step = c->d_step;
  r.dt = hs.dt;
  r.qp = (0.5 - hs.beta) * hs.dt * hs.dt;
  r.rhs = c->d_work;
  // the predictor pass pays where the rows are long (hexahedra: about 150
  // to 230 entries, each K^cc entry then gathers one value instead of
  // three); on quadrilaterals the extra launch costs more than it saves
  r.pred = hs.dim == 3 ? c->d_pred : nullptr;
  {
    // rows of p = 3 and p = 4 hexahedra hold about 130 and 230 entries: two
    // rows of 32 lanes per wave were 11% and 5% faster there than four rows
    // of 16 lanes (the 64^3 and 48^3 cubes; 64 lanes per row were slower);
    // quadrilaterals keep 16
    const double avg = nc > 0 ? double(hs.Kcd.ptr.back() + hs.Kcc.ptr.back()) / double(nc) : 0.0;
    r.lanes_per_row = avg > 96.0 ? 32 : 16;
    if (const char* v = std::getenv("IMEX_RHS_LANES")) r.lanes_per_row = std::atoi(v) == 32 ? 32 : 16;
  }
  SolveArgs& sa = c->sa;
  sa.parts = c->d_parts;
  sa.schur = c->d_schur;
  sa.vals = c->d_cvals;
  sa.ints = c->d_cints;
  sa.zvals = c->d_zvals;
  sa.schur_inv = c->d_sinv;
  sa.schur_chunks = c->d_schunks;
  sa.schur_chain = c->d_schain;
  sa.part_chunks = c->d_pchunks;
  sa.pinv = c->d_pinv;
  sa.dense_chunks = c->d_dchunks;
  sa.dense = F.dense ? 1 : 0;
  sa.cp_rowptr = c->d_cprowptr;
  sa.cp_ptr = c->d_cpptr;
  sa.cp_col = c->d_cpcol;
  sa.cp_val = c->d_cpval;
  sa.cbuf = c->d_cbuf;
  sa.sep_src = c->d_sepsrc;
  sa.rhs = c->d_work;
  sa.w = c->d_w;
  sa.uc = cs;
  sa.vc = cs + nc;
  sa.ac = cs + 2 * nc;
  sa.c_nodes = c->d_cnodes;
  sa.step = c->d_step;
  sa.dt = hs.dt;
  sa.qp = (0.5 - hs.beta) * hs.dt * hs.dt;
  sa.qc = hs.beta * hs.dt * hs.dt;
  sa.smem_part = sp;
  sa.smem_schur = ss;
  int64_t max_sep = 0;  // largest separator system in dense form
  for (const ChainMeta& cm : F.schur)
    if (cm.coff != -2) max_sep = std::max<int64_t>(max_sep, cm.nrows);
  sa.smem_sep = (int64_t)sizeof(double) * std::max<int64_t>(max_sep, 1);
  sa.dense_wide = c->n_sym_blocks > 0 ? 1 : 0;
  sa.sym_blocks = c->d_symblocks;
  sa.sym_poff = c->d_sympoff;
  sa.sym_partial = c->d_sympartial;
  sa.n_sym_blocks = c->n_sym_blocks;
  sa.rs = c->d_rs;
  sa.corr_chunks = c->d_corrchunks;
  sa.part_corr = c->d_partcorr;
  sa.pd_chunks = c->d_pdchunks;
  sa.sep_chunks = c->d_sepchunks;
  sa.n_corr_chunks = c->n_corr_chunks;
  sa.nd = hs.nd ? 1 : 0;
  sa.nd_fwd = c->d_ndf;
  sa.nd_bwd = c->d_ndb;
  sa.nd_fchunks = c->d_nd_fch;
  sa.nd_bchunks = c->d_nd_bch;
  sa.nd_fcchunks = c->d_nd_fcch;
  sa.nd_st = c->d_nd_st;
  sa.nd_gptr = c->d_nd_gptr;
  sa.nd_gsrc = c->d_nd_gsrc;
  sa.nd_W = c->d_ndW;
  sa.nd_smem_f = (int64_t)sizeof(double) * std::max<int64_t>(hs.ndf.max_m, 1);
  sa.nd_smem_b = (int64_t)sizeof(double) * std::max<int64_t>(hs.ndf.max_mk, 1);
  if (nc > 0) HIPCHECK(c, prepare_solve(sa, c->fp), "prepare solve");
  HIPCHECK(c, hipStreamSynchronize(c->stream), "sync");
  return IMEX_OK;
}

static imex_status ensure_ft(imex_ctx* c, int64_t n) {
  if (n <= c->ft_cap) return IMEX_OK;
  int64_t cap = std::max<int64_t>(n, 4096);
  double* p = nullptr;
  HIPCHECK(c, c->alloc(&p, sizeof(double) * cap), "alloc ft");
  c->d_ft = p;
  c->ft_cap = cap;
  c->ea.ft = p;
  c->ra.ft = p;
  c->la.ft = p;
  c->drop_graphs();
  return IMEX_OK;
}

imex_status imex_set_initial(imex_ctx* c, const double* u0, const double* v0, double ft0) {
  if (!c) return IMEX_EINVAL;
  if (!c->assembled) return c->fail(IMEX_ESTATE, "assemble the implicit block first");
  if (c->host_only) return c->fail(IMEX_ESTATE, "host-only context cannot hold a state");
  const HostSetup& hs = c->hs;
  const int64_t ng = hs.n_grid, nc = (int64_t)hs.c_nodes.size();
  std::vector<double> u(ng, 0.0), v(ng, 0.0);
  for (int64_t g = 0; g < ng; ++g)
    if (hs.node_kind[g] != kInactive) {
      u[g] = u0 ? u0[g] : 0.0;
      v[g] = v0 ? v0[g] : 0.0;
    }
  // c state: u^c_0, v^c_0 and a^c_0 from M^cc a = f_t(0) f_x^c - K^c u_0
  std::vector<double> cs(3 * nc, 0.0);
  std::vector<double> ku(nc, 0.0);
  kc_apply(hs, u.data(), ku.data());
  for (int64_t i = 0; i < nc; ++i) {
    cs[i] = u[hs.c_nodes[i]];
    cs[nc + i] = v[hs.c_nodes[i]];
    cs[2 * nc + i] = ft0 * hs.fxc[i] - ku[i];
  }
  mcc_solve(hs, cs.data() + 2 * nc);
  imex_status st = ensure_ft(c, 2);
  if (st != IMEX_OK) return st;
  // grid[0] = u_0, grid[1] = v_0 (d entries used by the start step)
  std::vector<double> tmp(ng);
  double* dtmp = nullptr;
  HIPCHECK(c, hipMalloc(&dtmp, sizeof(double) * ng), "alloc tmp");
  auto put = [&](const std::vector<double>& h, void* dst) -> hipError_t {
    hipError_t e = hipMemcpyAsync(dtmp, h.data(), sizeof(double) * ng, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_f64_to_grid(dtmp, dst, ng, c->fp, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e;
  };
  if (c->fp == 32)  // the increment buffer holds v_0 on the d nodes only
    for (int64_t g = 0; g < ng; ++g)
      if (hs.node_kind[g] != kD) v[g] = 0.0;
  hipError_t e = put(u, c->grid[0].p);
  if (e == hipSuccess) e = put(v, c->fp == 32 ? static_cast<void*>(c->d_delta) : c->grid[1].p);
  (void)hipFree(dtmp);
  if (e != hipSuccess) return c->hipfail(e, "upload initial state");
  HIPCHECK(c, hipMemcpyAsync(c->cstate.p, cs.data(), sizeof(double) * 3 * nc, hipMemcpyHostToDevice, c->stream),
           "upload c state");
  HIPCHECK(c, hipMemcpyAsync(c->d_ft, &ft0, sizeof(double), hipMemcpyHostToDevice, c->stream), "upload ft0");
  HIPCHECK(c, launch_set_int(c->d_step, 0, c->stream), "step counter");
  // start value u^d_{-1} = u_0 - dt v_0 + dt^2/2 a^d_0, written over v_0
  // (FP32: the start increment u_0 - u^d_{-1} = dt v_0 - dt^2/2 a^d_0, then
  // u_{-1} = u_0 - that increment)
  ExplicitArgs a = c->ea;
  bind_explicit(c, a, 0);
  a.write_u = 0;
  a.ft_offset = 0;
  a.c1 = c->fp == 32 ? 0.0 : 1.0;
  a.c2 = c->fp == 32 ? hs.dt : -hs.dt;
  a.c3 = c->fp == 32 ? -0.5 : 0.5;
  HIPCHECK(c, launch_explicit(a, c->fp, c->stream), "start step");
  if (c->lts_m > 0 && nc > 0) {
    // leap-frog: the c dofs take the central-difference start value too,
    // u^c_{-1} = u^c_0 - dt v^c_0 + dt^2/2 a^c_0, into the u_{n-1} grid
    std::vector<double> up(nc);
    for (int64_t i = 0; i < nc; ++i) up[i] = cs[i] - hs.dt * cs[nc + i] + 0.5 * hs.dt * hs.dt * cs[2 * nc + i];
    double* dup = nullptr;
    HIPCHECK(c, hipMalloc(&dup, sizeof(double) * nc), "alloc tmp");
    hipError_t e2 = hipMemcpyAsync(dup, up.data(), sizeof(double) * nc, hipMemcpyHostToDevice, c->stream);
    if (e2 == hipSuccess) e2 = launch_scatter_c(c->grid[1].p, c->d_cnodes, dup, nc, c->fp, c->stream);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(c->stream);
    (void)hipFree(dup);
    if (e2 != hipSuccess) return c->hipfail(e2, "leap-frog start value");
  }
  if (c->fp == 32)
    HIPCHECK(c, launch_sub_f32(static_cast<float*>(c->grid[1].p), static_cast<const float*>(c->grid[0].p),
                               c->d_delta, ng, c->stream),
             "start value");
  HIPCHECK(c, hipStreamSynchronize(c->stream), "sync");
  c->cur = 0;
  c->initialized = true;
  c->steps_taken = 0;
  return IMEX_OK;
}

imex_status imex_set_state(imex_ctx* c, int which, const double* src, int64_t len) {
  if (!c || !src) return IMEX_EINVAL;
  if (!c->assembled || c->host_only) return c->fail(IMEX_ESTATE, "no device state");
  const HostSetup& hs = c->hs;
  const int64_t ng = hs.n_grid, nc = (int64_t)hs.c_nodes.size();
  if (which == IMEX_FIELD_U || which == IMEX_FIELD_UPREV) {
    if (len != ng) return c->fail(IMEX_EINVAL, "grid field length mismatch");
    std::vector<double> u(ng, 0.0);
    for (int64_t g = 0; g < ng; ++g)
      if (hs.node_kind[g] != kInactive) u[g] = src[g];
    double* dtmp = nullptr;
    HIPCHECK(c, hipMalloc(&dtmp, sizeof(double) * ng), "alloc tmp");
    const int dst = which == IMEX_FIELD_U ? c->cur : 1 - c->cur;
    hipError_t e = hipMemcpyAsync(dtmp, u.data(), sizeof(double) * ng, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_f64_to_grid(dtmp, c->grid[dst].p, ng, c->fp, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(dtmp);
    if (e != hipSuccess) return c->hipfail(e, "set state");
    if (c->fp == 32) {  // the increment follows u_n - u_{n-1}
      HIPCHECK(c, launch_sub_f32(c->d_delta, static_cast<const float*>(c->grid[c->cur].p),
                                 static_cast<const float*>(c->grid[1 - c->cur].p), ng, c->stream),
               "increment");
      HIPCHECK(c, hipStreamSynchronize(c->stream), "sync");
    }
    if (which == IMEX_FIELD_U) {  // u^c follows u_n
      std::vector<double> uc(nc);
      for (int64_t i = 0; i < nc; ++i) uc[i] = u[hs.c_nodes[i]];
      HIPCHECK(c, hipMemcpy(c->cstate.p, uc.data(), sizeof(double) * nc, hipMemcpyHostToDevice), "set u^c");
    }
  } else if (which == IMEX_FIELD_VC || which == IMEX_FIELD_AC || which == IMEX_FIELD_UC) {
    if (len != nc) return c->fail(IMEX_EINVAL, "c field length mismatch");
    double* base = static_cast<double*>(c->cstate.p) +
                   (which == IMEX_FIELD_UC ? 0 : which == IMEX_FIELD_VC ? nc : 2 * nc);
    HIPCHECK(c, hipMemcpy(base, src, sizeof(double) * nc, hipMemcpyHostToDevice), "set c field");
  } else if (which == IMEX_FIELD_DELTA) {
    if (c->fp != 32) return c->fail(IMEX_EINVAL, "the increment field exists in FP32 contexts only");
    if (len != ng) return c->fail(IMEX_EINVAL, "grid field length mismatch");
    std::vector<float> h(ng, 0.0f);
    for (int64_t g = 0; g < ng; ++g)
      if (hs.node_kind[g] == kD) h[g] = (float)src[g];
    HIPCHECK(c, hipMemcpy(c->d_delta, h.data(), sizeof(float) * ng, hipMemcpyHostToDevice), "set increment");
  } else {
    return c->fail(IMEX_EINVAL, "unknown field");
  }
  c->initialized = true;
  return IMEX_OK;
}

imex_status imex_step(imex_ctx* c, int n_steps, const double* ft, int ft_on_device) {
  if (!c) return IMEX_EINVAL;
  if (c->host_only) return c->fail(IMEX_ESTATE, "host-only context cannot step");
  if (!c->initialized) return c->fail(IMEX_ESTATE, "set the initial state first");
  if (n_steps < 0 || (n_steps > 0 && !ft)) return c->fail(IMEX_EINVAL, "bad step arguments");
  if (n_steps == 0) return IMEX_OK;
  imex_status st = ensure_ft(c, (int64_t)n_steps + 1);
  if (st != IMEX_OK) return st;
  HIPCHECK(c, hipMemcpyAsync(c->d_ft, ft, sizeof(double) * (n_steps + 1),
                             ft_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream),
           "upload ft");
  if (!ft_on_device) HIPCHECK(c, hipStreamSynchronize(c->stream), "sync ft upload");
  HIPCHECK(c, launch_set_int(c->d_step, 0, c->stream), "step counter");
  int left = n_steps;
  const bool timed = times_steps(c);  // events between launches: no graphs then
  if (use_graphs() && !learned_needs_eager(c) && !timed) {
    while (left >= kGraphChunk) {
      st = ensure_graph(c, c->cur);
      if (st != IMEX_OK) return st;
      HIPCHECK(c, hipGraphLaunch(c->graph[c->cur], c->stream), "graph launch");
      left -= kGraphChunk;  // even chunk: parity unchanged
    }
  }
  while (left > 0) {
    st = run_step(c, c->cur, c->stream, timed ? (int)(c->tev_count % kTimedSteps) : -1);
    if (st != IMEX_OK) return st;
    if (timed) ++c->tev_count;
    c->cur = 1 - c->cur;
    --left;
  }
  c->steps_taken += n_steps;
  if (c->check_finite) return check_state(c);
  if (c->own_stream) HIPCHECK(c, hipStreamSynchronize(c->stream), "sync");
  return IMEX_OK;
}

imex_status imex_sample_field(imex_ctx* c, int which, int64_t n, const double* points, double* out) {
  if (!c || n < 0 || (n > 0 && (!points || !out))) return IMEX_EINVAL;
  if (!c->assembled || c->host_only) return c->fail(IMEX_ESTATE, "no device state");
  if (which != IMEX_FIELD_U && which != IMEX_FIELD_UPREV) return c->fail(IMEX_EINVAL, "only grid fields can be sampled");
  if (n == 0) return IMEX_OK;
  std::vector<int64_t> ids;
  std::vector<double> wts;
  const std::string m = sample_weights(c->hs, points, n, ids, wts);
  if (!m.empty()) return c->fail(IMEX_EINVAL, m);
  const int nb = (int)(ids.size() / (size_t)n);
  const void* src = c->grid[which == IMEX_FIELD_U ? c->cur : 1 - c->cur].p;
  int64_t* dids = nullptr;
  double *dw = nullptr, *dout = nullptr;
  hipError_t e = hipMalloc(&dids, sizeof(int64_t) * ids.size());
  if (e == hipSuccess) e = hipMalloc(&dw, sizeof(double) * wts.size());
  if (e == hipSuccess) e = hipMalloc(&dout, sizeof(double) * n);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dids, ids.data(), sizeof(int64_t) * ids.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dw, wts.data(), sizeof(double) * wts.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_sample(src, dids, dw, nb, n, dout, c->fp, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (dids) (void)hipFree(dids);
  if (dw) (void)hipFree(dw);
  if (dout) (void)hipFree(dout);
  if (e != hipSuccess) return c->hipfail(e, "sample field");
  return IMEX_OK;
}

imex_status imex_sample_field_noalloc(imex_ctx* c, int which, int64_t n, const double* points, double* out) {
  if (!c || n < 0 || (n > 0 && (!points || !out))) return IMEX_EINVAL;
  if (!c->assembled || c->host_only) return c->fail(IMEX_ESTATE, "no device state");
  if (which != IMEX_FIELD_U && which != IMEX_FIELD_UPREV) return c->fail(IMEX_EINVAL, "only grid fields can be sampled");
  if (n == 0) return IMEX_OK;
  const HostSetup& hs = c->hs;
  const int64_t max_n = imex_sample_noalloc_max_points(hs.dim);
  if (n > max_n) return c->fail(IMEX_EINVAL, "too many sample points for the allocation-free sampling scratch");
  // the checks of imex_sample_field, without temporary storage
  for (int64_t r = 0; r < n; ++r) {
    int64_t cidx[3] = {0, 0, 0};
    for (int k = 0; k < hs.dim; ++k) {
      const double x = points[r * hs.dim + k];
      if (!(x >= 0.0 && x <= hs.ne[k] * hs.h[k])) return c->fail(IMEX_EINVAL, "a sample point lies outside the box");
      cidx[k] = std::min<int64_t>((int64_t)std::floor(x / hs.h[k]), hs.ne[k] - 1);
    }
    const int64_t cid = cidx[0] + hs.ne[0] * (cidx[1] + hs.ne[1] * cidx[2]);
    if (hs.cell_flag[cid] == kEmpty) return c->fail(IMEX_EINVAL, "a sample point lies in an empty cell");
  }
  void* sp = nullptr;
  HIPCHECK(c, scratch_address(c->device, &sp), "sampling scratch address");
  // scratch layout: points (n x dim doubles) | values (n doubles)
  double* dpts = static_cast<double*>(sp);
  double* dout = dpts + n * hs.dim;
  SamplePointsArgs a{};
  a.dim = hs.dim;
  a.n = hs.n;
  for (int k = 0; k < 3; ++k) {
    a.ne[k] = hs.ne[k];
    a.nn[k] = hs.nn[k];
    a.h[k] = hs.h[k];
  }
  for (int i = 0; i < hs.n; ++i) a.x[i] = hs.ref.x[i];
  const void* src = c->grid[which == IMEX_FIELD_U ? c->cur : 1 - c->cur].p;
  hipError_t e = hipMemcpyAsync(dpts, points, sizeof(double) * (size_t)(n * hs.dim), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_sample_points(src, a, dpts, n, dout, c->fp, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return c->hipfail(e, "sample field (no allocation)");
  return IMEX_OK;
}

int64_t imex_sample_noalloc_max_points(int dim) {
  if (dim != 2 && dim != 3) return 0;
  return (int64_t)(IMEX_SAMPLE_NOALLOC_BYTES / (sizeof(double) * (size_t)(dim + 1)));
}

imex_status imex_read_field(imex_ctx* c, int which, void* dst, int dst_is_device, int64_t len) {
  if (!c || !dst) return IMEX_EINVAL;
  if (!c->assembled || c->host_only) return c->fail(IMEX_ESTATE, "no device state");
  const HostSetup& hs = c->hs;
  const int64_t ng = hs.n_grid, nc = (int64_t)hs.c_nodes.size();
  if (which == IMEX_FIELD_U || which == IMEX_FIELD_UPREV) {
    if (len != ng) return c->fail(IMEX_EINVAL, "grid field length mismatch");
    const void* src = c->grid[which == IMEX_FIELD_U ? c->cur : 1 - c->cur].p;
    if (dst_is_device) {
      HIPCHECK(c, launch_grid_to_f64(src, static_cast<double*>(dst), ng, c->fp, c->stream), "read");
    } else {
      double* dtmp = nullptr;
      HIPCHECK(c, hipMalloc(&dtmp, sizeof(double) * ng), "alloc tmp");
      hipError_t e = launch_grid_to_f64(src, dtmp, ng, c->fp, c->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(dst, dtmp, sizeof(double) * ng, hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      (void)hipFree(dtmp);
      if (e != hipSuccess) return c->hipfail(e, "read field");
    }
  } else if (which == IMEX_FIELD_VC || which == IMEX_FIELD_AC || which == IMEX_FIELD_UC) {
    if (len != nc) return c->fail(IMEX_EINVAL, "c field length mismatch");
    const double* base = static_cast<const double*>(c->cstate.p) +
                         (which == IMEX_FIELD_UC ? 0 : which == IMEX_FIELD_VC ? nc : 2 * nc);
    HIPCHECK(c, hipMemcpyAsync(dst, base, sizeof(double) * nc,
                               dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream),
             "read c field");
    if (!dst_is_device) HIPCHECK(c, hipStreamSynchronize(c->stream), "sync");
  } else if (which == IMEX_FIELD_DELTA) {
    if (c->fp != 32) return c->fail(IMEX_EINVAL, "the increment field exists in FP32 contexts only");
    if (len != ng) return c->fail(IMEX_EINVAL, "grid field length mismatch");
    double* dtmp = static_cast<double*>(dst);
    if (!dst_is_device) HIPCHECK(c, hipMalloc(&dtmp, sizeof(double) * ng), "alloc tmp");
    hipError_t e = launch_grid_to_f64(c->d_delta, dtmp, ng, 32, c->stream);
    if (e == hipSuccess && !dst_is_device)
      e = hipMemcpyAsync(dst, dtmp, sizeof(double) * ng, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (!dst_is_device) (void)hipFree(dtmp);
    if (e != hipSuccess) return c->hipfail(e, "read increment");
  } else {
    return c->fail(IMEX_EINVAL, "unknown field");
  }
  return IMEX_OK;
}

imex_status imex_export_csr(const imex_ctx* cc, int which, int64_t* nrows, int64_t* nnz, int64_t* row_ptr,
                            int64_t* cols, double* vals) {
  imex_ctx* c = const_cast<imex_ctx*>(cc);
  if (!c || !nrows || !nnz) return IMEX_EINVAL;
  if (!c->assembled) return c->fail(IMEX_ESTATE, "assemble first");
  const Csr* A = which == IMEX_CSR_KC ? &c->hs.Kc : which == IMEX_CSR_MCC ? &c->hs.Mcc
               : which == IMEX_CSR_S ? &c->hs.S : nullptr;
  if (!A) return c->fail(IMEX_EINVAL, "unknown matrix");
  *nrows = A->nrows;
  *nnz = (int64_t)A->col.size();
  if (row_ptr) std::copy(A->ptr.begin(), A->ptr.end(), row_ptr);
  if (cols) std::copy(A->col.begin(), A->col.end(), cols);
  if (vals) std::copy(A->val.begin(), A->val.end(), vals);
  return IMEX_OK;
}

imex_status imex_export_index(const imex_ctx* cc, int which, int64_t* dst, int64_t* len) {
  imex_ctx* c = const_cast<imex_ctx*>(cc);
  if (!c || !len) return IMEX_EINVAL;
  const HostSetup& hs = c->hs;
  std::vector<int64_t> v;
  switch (which) {
    case IMEX_INDEX_CELL_FLAGS:
      v.assign(hs.cell_flag.begin(), hs.cell_flag.end());
      break;
    case IMEX_INDEX_C_NODES:
      v = hs.c_nodes;
      break;
    case IMEX_INDEX_D_NODES:
      v = hs.d_nodes;
      break;
    case IMEX_INDEX_COMP_PTR:
      for (const ComponentLayout& L : hs.layout) v.push_back(L.begin);
      v.push_back((int64_t)hs.c_nodes.size());
      break;
    default:
      return c->fail(IMEX_EINVAL, "unknown index");
  }
  if (dst) {
    if (*len < (int64_t)v.size()) return c->fail(IMEX_EINVAL, "destination too small");
    std::copy(v.begin(), v.end(), dst);
  }
  *len = (int64_t)v.size();
  return IMEX_OK;
}

imex_status imex_factor_solve_host(imex_ctx* c, const double* b, double* x) {
  if (!c || !b || !x) return IMEX_EINVAL;
  if (!c->assembled) return c->fail(IMEX_ESTATE, "assemble the implicit block first");
  if (!c->hs.nd) return c->fail(IMEX_EINVAL, "the host solve exists for the nested-dissection factor only");
  nd_solve_host(c->hs.ndf, b, x);
  return IMEX_OK;
}

imex_status imex_time_kernel(imex_ctx* c, int which, int reps, double* avg_ms) {
  if (!c || !avg_ms || reps < 1) return IMEX_EINVAL;
  if (c->host_only || !c->initialized) return c->fail(IMEX_ESTATE, "no device state");
  const int64_t nc = (int64_t)c->hs.c_nodes.size();
  if (which < 0 || which > 2) return c->fail(IMEX_EINVAL, "unknown kernel");
  if (which > 0 && nc == 0) return c->fail(IMEX_EINVAL, "no implicit block");
  imex_status st = ensure_ft(c, 2);
  if (st != IMEX_OK) return st;
  HIPCHECK(c, launch_set_int(c->d_step, 0, c->stream), "step counter");
  ExplicitArgs a = c->ea;
  bind_explicit(c, a, c->cur);
  RhsArgs r = c->ra;
  r.ugrid = c->grid[1 - c->cur].p;
  SolveArgs s = c->sa;
  s.ugrid = c->grid[1 - c->cur].p;
  s.advance_step = 0;
  hipEvent_t e0, e1;
  HIPCHECK(c, hipEventCreate(&e0), "event");
  HIPCHECK(c, hipEventCreate(&e1), "event");
  hipError_t e = hipEventRecord(e0, c->stream);
  for (int k = 0; k < reps && e == hipSuccess; ++k) {
    if (which == 0) e = launch_explicit(a, c->fp, c->stream);
    else if (which == 1) e = launch_rhs(r, c->fp, c->stream);
    else e = launch_factor_solve(c, s, c->stream);
  }
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return c->hipfail(e, "time kernel");
  *avg_ms = (double)ms / reps;
  c->initialized = false;  // the state has been overwritten
  return IMEX_OK;
}

imex_status imex_autotune_tiles(imex_ctx* c, int reps, int* chosen) {
  if (!c || reps < 1) return IMEX_EINVAL;
  if (c->host_only || !c->assembled) return c->fail(IMEX_ESTATE, "assemble the implicit block first");
  const HostSetup& hs = c->hs;
  imex_status st = ensure_ft(c, 2);
  if (st != IMEX_OK) return st;
  const double zero[2] = {0.0, 0.0};
  HIPCHECK(c, hipMemcpyAsync(c->d_ft, zero, sizeof(zero), hipMemcpyHostToDevice, c->stream), "ft");
  HIPCHECK(c, launch_set_int(c->d_step, 0, c->stream), "step counter");
  // candidates: 2D tx x ty cells; 3D tx x ty cells per layer and lz layers per chunk
  struct Cand { int tx, ty, lz, mode; };
  std::vector<Cand> cands;
  const int sizes[] = {16, 8, 4, 2, 1};
  if (hs.dim == 2) {
    for (int tx : sizes)
      for (int ty : sizes)
        for (int mode : {0, 3})  // 256- or 128-thread workgroups
          if ((int64_t)(tx * hs.p + 1) * (ty * hs.p + 1) <= 8 * (mode == 0 ? 256 : 128))
            cands.push_back({tx, ty, 1, mode});
    if (hs.n <= kStripMaxN)
      for (int mode : {1, 2})
        for (int lz : {1, 2, 4, 8, 16, 32, 64})
          if (lz <= 2 * hs.ne[1]) cands.push_back({kStripCells, lz, lz, mode});
  } else if (c->ea.mode == kModeKron) {
    // tensor-product form: tiles fixed by the order, chunks of lz layers
    for (int lz : {1, 2, 4, 8, 16}) cands.push_back({kKronCX[hs.p], kKronCY[hs.p], lz, kModeKron});
  } else {
    for (int tx : {8, 4, 2})
      for (int ty : {8, 4, 2})
        for (int lz : {2, 4, 8})
          for (int mode : {0, 4}) cands.push_back({tx, ty, lz, mode});  // 256- or 512-thread workgroups
  }
  hipEvent_t e0, e1;
  HIPCHECK(c, hipEventCreate(&e0), "event");
  HIPCHECK(c, hipEventCreate(&e1), "event");
  const ExplicitArgs keep = c->ea;
  double best = 1e300;
  Cand bestc{keep.tx, keep.ty, keep.lz, keep.mode};
  hipError_t e = hipSuccess;
  for (const Cand& cd : cands) {
    ExplicitArgs a = keep;
    a.tx = cd.tx;
    a.ty = cd.ty;
    a.lz = cd.lz;
    a.mode = cd.mode;
    a.ntx = (int)((hs.ne[0] + a.tx - 1) / a.tx);
    a.nty = (int)((hs.ne[1] + a.ty - 1) / a.ty);
    a.nchunk = hs.dim == 3 ? (int)((hs.ne[2] + a.lz - 1) / a.lz) : 1;
    if (explicit_smem_bytes(a, c->fp) > 80 * 1024) continue;
    bind_explicit(c, a, c->cur);
    a.write_u = 0;  // the timing runs leave u alone
    e = launch_explicit(a, c->fp, c->stream);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
    for (int k = 0; k < reps && e == hipSuccess; ++k) e = launch_explicit(a, c->fp, c->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) break;
    if (ms < best) {
      best = ms;
      bestc = cd;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return c->hipfail(e, "autotune");
  ExplicitArgs& a = c->ea;
  a.tx = bestc.tx;
  a.ty = bestc.ty;
  a.lz = bestc.lz;
  a.mode = bestc.mode;
  a.ntx = (int)((hs.ne[0] + a.tx - 1) / a.tx);
  a.nty = (int)((hs.ne[1] + a.ty - 1) / a.ty);
  a.nchunk = hs.dim == 3 ? (int)((hs.ne[2] + a.lz - 1) / a.lz) : 1;
  c->drop_graphs();
  c->initialized = false;  // the timing launches overwrote the state
  if (chosen) {
    chosen[0] = a.tx;
    chosen[1] = a.ty;
    chosen[2] = a.lz;
    chosen[3] = a.mode;
  }
  return IMEX_OK;
}

const char* imex_last_error(const imex_ctx* c) { return c ? c->err.c_str() : g_setup_error.c_str(); }

void imex_destroy(imex_ctx* c) {
  if (!c) return;
  if (!c->host_only) {
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    c->drop_graphs();
    for (hipEvent_t ev : c->tev) (void)hipEventDestroy(ev);
    learned_free(c);
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

// ---------------------------------------------------------------------------
// batches of independent instances
// ---------------------------------------------------------------------------
// Device tables of the kernel-batched form: for each kernel type the
// instances' argument blocks (for both grid parities) and the prefix sums of
// their workgroup counts.
struct BatchKernels {
  struct Group {                     // explicit kernel, instances of one order p
    int p = 0, blocks = 0;
    size_t smem = 0;
    ExplicitArgs* args[2] = {nullptr, nullptr};
    int32_t* first = nullptr;
    int n = 0;
  };
  std::vector<Group> groups;
  RhsArgs* rhs[2] = {nullptr, nullptr};
  SolveArgs* solve[2] = {nullptr, nullptr};
  int32_t *rhs_first = nullptr, *dense_first = nullptr, *sep_first = nullptr, *corr_first = nullptr;
  int rhs_blocks = 0, dense_blocks = 0, sep_blocks = 0, corr_blocks = 0, lanes = 16, fp = 64;
  size_t sep_smem = 0;
  std::vector<const double*> ft;     // f_t tables the tables were built on
  std::vector<void*> allocs;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  void release() {
    for (int k = 0; k < 2; ++k)
      if (exec[k]) (void)hipGraphExecDestroy(exec[k]);
    exec[0] = exec[1] = nullptr;
    for (void* q : allocs) (void)hipFree(q);
    allocs.clear();
    groups.clear();
    ft.clear();
  }
};

struct imex_batch {
  std::vector<imex_ctx*> ctx;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  int mode = 0;                      // 0: one graph with a branch per instance; 1: lanes; 2: batched kernels (default)
  BatchKernels bk;
  std::vector<hipStream_t> lanes;    // mode 1: instances' graphs round-robin over these streams
  std::vector<hipEvent_t> lane_done;
  hipEvent_t fork = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int> exec_cur;          // grid parity of every instance the graph was built for
  std::vector<const double*> exec_ft;  // f_t tables the graph was built on
  void drop() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
  }
  void release() {
    drop();
    bk.release();
    for (hipEvent_t e : lane_done) (void)hipEventDestroy(e);
    for (hipStream_t q : lanes) (void)hipStreamDestroy(q);
    if (fork) (void)hipEventDestroy(fork);
    lane_done.clear();
    lanes.clear();
    fork = nullptr;
  }
  imex_status fail(imex_status st, const std::string& m) {
    err = m;
    return st;
  }
};

}  // extern "C"

namespace {

// an instance the kernel-batched form can take: a 2D Newmark IMEX context
// with an implicit block solved by the dense dissected factor
bool batch_kernel_eligible(const imex_ctx* c, int fp) {
  const HostSetup& hs = c->hs;
  return hs.dim == 2 && !hs.nd && c->lts_m == 0 && c->fp == fp && !hs.c_nodes.empty() && c->sa.dense == 1 &&
         c->sa.dense_wide == 0 && c->n_schur_chain == 0 && c->solver == IMEX_SOLVER_CHOLESKY && !c->learned &&
         c->ra.lanes_per_row == 16;
}

// the instance's explicit arguments on 256-thread LDS tiles (its own tile
// shape when the autotuner chose that form, else the default shape)
ExplicitArgs tile_args(const imex_ctx* c) {
  ExplicitArgs a = c->ea;
  if (a.mode == 0) return a;
  const HostSetup& hs = c->hs;
  int tx = 8, ty = 8;
  auto owned = [&](int x, int y) { return (int64_t)(x * hs.p + 1) * (y * hs.p + 1); };
  while (owned(tx, ty) > 8 * 256) {
    if (ty >= tx) ty /= 2;
    else tx /= 2;
  }
  while (((hs.ne[0] + tx - 1) / tx) * ((hs.ne[1] + ty - 1) / ty) < 512 && (tx > 4 || ty > 2)) {
    if (ty >= tx && ty > 2) ty /= 2;
    else tx /= 2;
  }
  a.mode = 0;
  a.tx = tx;
  a.ty = ty;
  a.lz = 1;
  a.ntx = (int)((hs.ne[0] + tx - 1) / tx);
  a.nty = (int)((hs.ne[1] + ty - 1) / ty);
  a.nchunk = 1;
  return a;
}

template <typename X>
hipError_t batch_upload(BatchKernels& bk, X** dst, const std::vector<X>& src, hipStream_t s) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(sizeof(X) * src.size(), 16));
  if (e != hipSuccess) return e;
  bk.allocs.push_back(q);
  *dst = static_cast<X*>(q);
  if (!src.empty()) e = hipMemcpyAsync(q, src.data(), sizeof(X) * src.size(), hipMemcpyHostToDevice, s);
  return e;
}

// builds the device tables of the kernel-batched form (instances' current
// f_t tables and both grid parities)
hipError_t build_batch_kernels(imex_batch* b) {
  BatchKernels& bk = b->bk;
  bk.release();
  const size_t n = b->ctx.size();
  bk.fp = b->ctx[0]->fp;
  hipStream_t s = b->stream;
  hipError_t e = hipSuccess;
  // explicit kernel: one group per order p
  std::vector<int> ps;
  for (imex_ctx* c : b->ctx)
    if (std::find(ps.begin(), ps.end(), c->hs.p) == ps.end()) ps.push_back(c->hs.p);
  std::sort(ps.begin(), ps.end());
  for (int p : ps) {
    BatchKernels::Group g;
    g.p = p;
    std::vector<ExplicitArgs> a0, a1;
    std::vector<int32_t> first{0};
    for (imex_ctx* c : b->ctx) {
      if (c->hs.p != p) continue;
      ExplicitArgs a = tile_args(c);
      g.smem = std::max(g.smem, explicit_smem_bytes(a, c->fp));
      ExplicitArgs x0 = a, x1 = a;
      bind_explicit(c, x0, 0);
      bind_explicit(c, x1, 1);
      a0.push_back(x0);
      a1.push_back(x1);
      first.push_back(first.back() + a.ntx * a.nty * a.nchunk);
    }
    g.n = (int)a0.size();
    g.blocks = first.back();
    if (e == hipSuccess) e = batch_upload(bk, &g.args[0], a0, s);
    if (e == hipSuccess) e = batch_upload(bk, &g.args[1], a1, s);
    if (e == hipSuccess) e = batch_upload(bk, &g.first, first, s);
    if (e == hipSuccess) e = prepare_explicit_batch(p, bk.fp);
    bk.groups.push_back(g);
  }
  // rhs and the three solve stages
  std::vector<RhsArgs> r0, r1;
  std::vector<SolveArgs> s0, s1;
  std::vector<int32_t> rf{0}, df{0}, sf{0}, cf{0};
  for (imex_ctx* c : b->ctx) {
    const int64_t nc = (int64_t)c->hs.c_nodes.size();
    for (int cur = 0; cur < 2; ++cur) {
      RhsArgs r = c->ra;
      r.ugrid = c->grid[1 - cur].p;
      r.pred = nullptr;  // the batched rhs forms the predictor per entry
      SolveArgs sa = c->sa;
      sa.ugrid = c->grid[1 - cur].p;
      sa.advance_step = 1;
      (cur == 0 ? r0 : r1).push_back(r);
      (cur == 0 ? s0 : s1).push_back(sa);
    }
    constexpr int64_t kRowsPerBlock = 16;  // the rhs kernel: four rows per wave, four waves
    rf.push_back(rf.back() + (int32_t)((nc + kRowsPerBlock - 1) / kRowsPerBlock));
    df.push_back(df.back() + (int32_t)(4 * c->n_dense_chunks));
    sf.push_back(sf.back() + (int32_t)(4 * c->n_schur_chunks));
    cf.push_back(cf.back() + (int32_t)c->n_part_chunks);
    bk.sep_smem = std::max<size_t>(bk.sep_smem, (size_t)c->sa.smem_sep);
  }
  bk.rhs_blocks = rf.back();
  bk.dense_blocks = df.back();
  bk.sep_blocks = sf.back();
  bk.corr_blocks = cf.back();
  if (e == hipSuccess) e = batch_upload(bk, &bk.rhs[0], r0, s);
  if (e == hipSuccess) e = batch_upload(bk, &bk.rhs[1], r1, s);
  if (e == hipSuccess) e = batch_upload(bk, &bk.solve[0], s0, s);
  if (e == hipSuccess) e = batch_upload(bk, &bk.solve[1], s1, s);
  if (e == hipSuccess) e = batch_upload(bk, &bk.rhs_first, rf, s);
  if (e == hipSuccess) e = batch_upload(bk, &bk.dense_first, df, s);
  if (e == hipSuccess) e = batch_upload(bk, &bk.sep_first, sf, s);
  if (e == hipSuccess) e = batch_upload(bk, &bk.corr_first, cf, s);
  if (e == hipSuccess) e = prepare_solve_batch(bk.fp);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  for (imex_ctx* c : b->ctx) bk.ft.push_back(c->d_ft);
  (void)n;
  return e;
}

// one step of every instance: one launch per kernel type (instances at grid
// parity cur).  The explicit launches of the orders write disjoint
// instances: with a lane per order they fork from s and join back before the
// right-hand side, so that small launches share the GPU (parallel branches
// when captured).
hipError_t batch_kernels_step(const BatchKernels& bk, int cur, int n_inst, hipStream_t s, const imex_batch* b) {
  hipError_t e = hipSuccess;
  const size_t ng = bk.groups.size();
  const bool side = ng > 1 && b->fork && b->lanes.size() >= ng && b->lane_done.size() >= ng;
  if (side) e = hipEventRecord(b->fork, s);
  for (size_t i = 0; i < ng; ++i) {
    const BatchKernels::Group& g = bk.groups[i];
    const BatchTable<ExplicitArgs> t{g.args[cur], g.first, g.n};
    hipStream_t q = side ? b->lanes[i] : s;
    if (e == hipSuccess && side) e = hipStreamWaitEvent(q, b->fork, 0);
    if (e == hipSuccess) e = launch_explicit_batch(t, g.p, g.blocks, g.smem, bk.fp, q);
    if (e == hipSuccess && side) e = hipEventRecord(b->lane_done[i], q);
  }
  for (size_t i = 0; side && i < ng && e == hipSuccess; ++i) e = hipStreamWaitEvent(s, b->lane_done[i], 0);
  const BatchTable<RhsArgs> rt{bk.rhs[cur], bk.rhs_first, n_inst};
  if (e == hipSuccess) e = launch_rhs_batch(rt, bk.rhs_blocks, bk.fp, bk.lanes, s);
  const BatchTable<SolveArgs> dt{bk.solve[cur], bk.dense_first, n_inst}, st{bk.solve[cur], bk.sep_first, n_inst},
      ct{bk.solve[cur], bk.corr_first, n_inst};
  if (e == hipSuccess)
    e = launch_solve_batch(dt, bk.dense_blocks, st, bk.sep_blocks, bk.sep_smem, ct, bk.corr_blocks, bk.fp, s);
  return e;
}

}  // namespace

extern "C" {

imex_status imex_batch_create(imex_ctx* const* ctxs, int n, void* hip_stream, imex_batch** out) {
  if (!ctxs || n < 1 || !out) {
    g_setup_error = "bad batch arguments";
    return IMEX_EINVAL;
  }
  *out = nullptr;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i] || ctxs[i]->host_only || !ctxs[i]->assembled) {
      g_setup_error = "every instance must be an assembled device context";
      return IMEX_ESTATE;
    }
  imex_batch* b = new (std::nothrow) imex_batch();
  if (!b) {
    g_setup_error = "out of host memory";
    return IMEX_ENOMEM;
  }
  b->ctx.assign(ctxs, ctxs + n);
  int n_lanes = kBatchLanes;
  const char* lv = std::getenv("IMEX_BATCH_LANES");
  if (lv) n_lanes = std::max(0, std::atoi(lv));
  bool kernels = !lv;
  for (int i = 0; i < n && kernels; ++i) kernels = batch_kernel_eligible(ctxs[i], ctxs[0]->fp);
  if (kernels) b->mode = 2;
  if (n_lanes > 0) {
    if (!kernels) b->mode = 1;
    hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int k = 0; k < n_lanes && e == hipSuccess; ++k) {
      hipStream_t q = nullptr;
      hipEvent_t ev = nullptr;
      e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking);
      if (e == hipSuccess) b->lanes.push_back(q);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) b->lane_done.push_back(ev);
    }
    if (e != hipSuccess) {
      g_setup_error = std::string("HIP: ") + hipGetErrorString(e);
      b->release();
      delete b;
      return IMEX_EHIP;
    }
  }
  if (hip_stream) b->stream = static_cast<hipStream_t>(hip_stream);
  else {
    hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      g_setup_error = std::string("HIP: ") + hipGetErrorString(e);
      delete b;
      return IMEX_EHIP;
    }
    b->own_stream = true;
  }
  *out = b;
  return IMEX_OK;
}

imex_status imex_batch_step(imex_batch* b, int n_steps, const double* const* ft, int ft_on_device) {
  if (!b) return IMEX_EINVAL;
  if (n_steps < 0 || (n_steps > 0 && !ft)) return b->fail(IMEX_EINVAL, "bad step arguments");
  if (n_steps == 0) return IMEX_OK;
  const size_t n = b->ctx.size();
  for (size_t i = 0; i < n; ++i) {
    imex_ctx* c = b->ctx[i];
    if (!c->initialized) return b->fail(IMEX_ESTATE, "set the initial state of every instance first");
    if (learned_needs_eager(c)) return b->fail(IMEX_ESTATE, "batched instances use the Cholesky solve");
    if (!ft[i]) return b->fail(IMEX_EINVAL, "missing f_t table");
    if (ensure_ft(c, (int64_t)n_steps + 1) != IMEX_OK) return b->fail(IMEX_EHIP, c->err);
    // work queued on the instance's own stream comes first
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->d_ft, ft[i], sizeof(double) * (n_steps + 1),
                         ft_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = launch_set_int(c->d_step, 0, b->stream);
    if (e != hipSuccess) return b->fail(IMEX_EHIP, std::string("batch upload: ") + hipGetErrorString(e));
  }
  if (!ft_on_device) {
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return b->fail(IMEX_EHIP, std::string("sync: ") + hipGetErrorString(e));
  }
  int left = n_steps;
  if (b->mode == 2) {
    // batched kernels: every instance at one grid parity, one launch per
    // kernel type per step, 32-step chunks captured in one graph
    int cur = b->ctx[0]->cur;
    bool same = true;
    std::vector<const double*> fts;
    for (imex_ctx* c : b->ctx) {
      same = same && c->cur == cur;
      fts.push_back(c->d_ft);
    }
    if (same) {
      if (b->bk.groups.empty() || fts != b->bk.ft) {
        const hipError_t e = build_batch_kernels(b);
        if (e != hipSuccess) return b->fail(IMEX_EHIP, std::string("batch tables: ") + hipGetErrorString(e));
      }
      const int ni = (int)n;
      if (left >= kGraphChunk && use_graphs()) {
        if (!b->bk.exec[cur]) {
          hipGraph_t g = nullptr;
          hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
          hipError_t e2 = hipSuccess;
          for (int k = 0; k < kGraphChunk && e == hipSuccess && e2 == hipSuccess; ++k)
            e2 = batch_kernels_step(b->bk, (cur + k) & 1, ni, b->stream, b);
          if (e == hipSuccess) e = hipStreamEndCapture(b->stream, &g);
          if (e == hipSuccess) e = e2;
          if (e == hipSuccess) e = hipGraphInstantiate(&b->bk.exec[cur], g, nullptr, nullptr, 0);
          if (g) (void)hipGraphDestroy(g);
          if (e != hipSuccess) {
            b->bk.exec[cur] = nullptr;
            return b->fail(IMEX_EHIP, std::string("batch graph: ") + hipGetErrorString(e));
          }
        }
        while (left >= kGraphChunk) {
          const hipError_t e = hipGraphLaunch(b->bk.exec[cur], b->stream);
          if (e != hipSuccess) return b->fail(IMEX_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
          left -= kGraphChunk;  // even chunk: parities unchanged
        }
      }
      for (; left > 0; --left) {
        const hipError_t e = batch_kernels_step(b->bk, cur, ni, b->stream, b);
        if (e != hipSuccess) return b->fail(IMEX_EHIP, std::string("batch step: ") + hipGetErrorString(e));
        cur = 1 - cur;
        for (imex_ctx* c : b->ctx) c->cur = 1 - c->cur;
      }
    }
  }
  if (b->mode == 1 && left >= kGraphChunk && use_graphs()) {
    // every instance's own 32-step graphs, instances spread round-robin over
    // the lanes; the lanes fork from and join back into the batch stream
    for (imex_ctx* c : b->ctx)
      if (ensure_graph(c, c->cur) != IMEX_OK) return b->fail(IMEX_EHIP, c->err);
    const int chunks = left / kGraphChunk;
    const size_t L = b->lanes.size();
    hipError_t e = hipEventRecord(b->fork, b->stream);
    for (size_t k = 0; k < L && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->lanes[k], b->fork, 0);
    for (size_t i = 0; i < n && e == hipSuccess; ++i)
      for (int q = 0; q < chunks && e == hipSuccess; ++q)
        e = hipGraphLaunch(b->ctx[i]->graph[b->ctx[i]->cur], b->lanes[i % L]);
    for (size_t k = 0; k < L && e == hipSuccess; ++k) e = hipEventRecord(b->lane_done[k], b->lanes[k]);
    for (size_t k = 0; k < L && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->stream, b->lane_done[k], 0);
    if (e != hipSuccess) return b->fail(IMEX_EHIP, std::string("lanes: ") + hipGetErrorString(e));
    left -= chunks * kGraphChunk;
  }
  if (b->mode == 0 && left >= kGraphChunk && use_graphs()) {
    // one graph: a child graph of kGraphChunk steps per instance, no edges
    // between them, so the instances' kernels may overlap
    std::vector<int> cur(n);
    std::vector<const double*> fts(n);
    for (size_t i = 0; i < n; ++i) {
      cur[i] = b->ctx[i]->cur;
      fts[i] = b->ctx[i]->d_ft;
    }
    if (!b->exec || cur != b->exec_cur || fts != b->exec_ft) {
      b->drop();
      hipGraph_t parent = nullptr;
      hipError_t e = hipGraphCreate(&parent, 0);
      if (e != hipSuccess) return b->fail(IMEX_EHIP, "graph create");
      for (size_t i = 0; i < n; ++i) {
        hipGraph_t child = nullptr;
        if (capture_chunk(b->ctx[i], cur[i], &child) != IMEX_OK) {
          (void)hipGraphDestroy(parent);
          return b->fail(IMEX_EHIP, b->ctx[i]->err);
        }
        hipGraphNode_t node;
        e = hipGraphAddChildGraphNode(&node, parent, nullptr, 0, child);
        (void)hipGraphDestroy(child);
        if (e != hipSuccess) {
          (void)hipGraphDestroy(parent);
          return b->fail(IMEX_EHIP, std::string("child graph: ") + hipGetErrorString(e));
        }
      }
      e = hipGraphInstantiate(&b->exec, parent, nullptr, nullptr, 0);
      (void)hipGraphDestroy(parent);
      if (e != hipSuccess) {
        b->exec = nullptr;
        return b->fail(IMEX_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
      }
      b->exec_cur = cur;
      b->exec_ft = fts;
    }
    while (left >= kGraphChunk) {
      hipError_t e = hipGraphLaunch(b->exec, b->stream);
      if (e != hipSuccess) return b->fail(IMEX_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
      left -= kGraphChunk;  // even chunk: parities unchanged
    }
  }
  for (; left > 0; --left)
    for (imex_ctx* c : b->ctx) {
      if (run_step(c, c->cur, b->stream) != IMEX_OK) return b->fail(IMEX_EHIP, c->err);
      c->cur = 1 - c->cur;
    }
  for (imex_ctx* c : b->ctx) c->steps_taken += n_steps;
  if (b->own_stream) {
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return b->fail(IMEX_EHIP, std::string("sync: ") + hipGetErrorString(e));
  }
  return IMEX_OK;
}

int imex_batch_form(const imex_batch* b) { return b ? b->mode : -1; }

const char* imex_batch_last_error(const imex_batch* b) { return b ? b->err.c_str() : g_setup_error.c_str(); }

void imex_batch_destroy(imex_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (hipStream_t q : b->lanes) (void)hipStreamSynchronize(q);
  b->release();
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"
