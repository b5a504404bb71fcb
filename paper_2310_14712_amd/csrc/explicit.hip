// HIP kernels (gfx950) of the Newmark IMEX step.
//
// Explicit part (diagonal CDM step, Eqs. CDMacc and CDMstep restricted to
// the d dofs): matrix-free stiffness apply on uncut cells by sum
// factorisation,
//   2D  Y = s_x Kh U Mh^T + s_y Mh U Kh^T                   (4 n^3 MAC / cell)
//   3D  Y = s_x Kh_x (Mh_y Mh_z U) + Mh_x (s_y Kh_y Mh_z U + s_z Mh_y Kh_z U)
//                                                          (7 n^4 MAC / cell)
// with the consistent 1D matrices Mh, Kh (the uncut stiffness is integrated
// exactly, Section "Spatial Discretization", last paragraph) and the
// GLL-lumped mass computed on the fly from the GLL weights of the uncut
// cells around each node.
//
// Work decomposition ("layer march", owner computes): a workgroup owns the
// nodes of a tile of cells in x (and y in 3D) and marches over a chunk of
// cell layers along the last direction.  Per layer it stages the layer's
// node planes in LDS, applies the 1D operators pencil by pencil (one thread
// per pencil, operators from the kernel argument block, i.e. scalar
// registers), and sums each owned node's contributions from its adjacent
// cells in a fixed order; the contribution of a layer to its top node plane
// is carried in LDS to the next layer.  One extra cell on the low side of
// the tile (and one extra layer at the start of a chunk) supplies the
// contributions of neighbouring tiles, so no atomics are used and results
// are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "dev_common.h"
#include "device.h"
#include <type_traits>

namespace imex {

namespace {

using namespace dev;

// The 1D GLL operators are symmetric and centro-symmetric (C[a][b] = C[b][a]
// = C[P-a][P-b]; the host makes the tables exactly so), so every entry is
// read from its canonical position: the smallest of the four equivalent
// (row, column) pairs.  The kernels then keep only the distinct values live.
template <int N>
__host__ __device__ constexpr int canon(int a, int b) {
  const int P = N - 1;
  int best = a * N + b;
  const int alt[3] = {b * N + a, (P - a) * N + (P - b), (P - b) * N + (P - a)};
  for (int k = 0; k < 3; ++k) best = alt[k] < best ? alt[k] : best;
  return best;
}

// row `row` of a 1D operator (n x n, row-major) times v[0..N)
template <int N>
__device__ inline double op_row(const double* C, int row, const double* v) {
  double acc = 0.0;
#pragma unroll
  for (int d = 0; d < N; ++d) acc = fma(C[canon<N>(row, d)], v[d], acc);
  return acc;
}

// The arithmetic shared by the 2D kernels, with every fused multiply-add
// written out, so that both forms round identically whatever the compiler
// would contract: s_x y1 + s_y y2 of a cell, the lumped-mass sum and the
// node update out = c1 u_n + c2 w + c3 dt^2 (f_t f_x - y) / (rho |J| m).
__device__ inline double cell_combine(double sx, double y1, double sy, double y2) { return fma(sx, y1, sy * y2); }
__device__ inline double mass_add(double m, double wa, double wb) { return fma(wa, wb, m); }
__device__ inline double node_update(const ExplicitArgs& A, double ft, double fx, double y, double m, double un,
                                     double w) {
  const double acc = fma(ft, fx, -y) / (A.mass_scale * m);
  return fma(A.c1, un, fma(A.c2, w, (A.c3 * A.dt2) * acc));
}

// Lane exchanges through DPP (data-parallel primitives) on both halves of a
// double: quad_perm [1,0,3,2] (xor 1), quad_perm [2,3,0,1] (xor 2), mirror

// ---------------------------------------------------------------------------
// 2D explicit step: one tile of tx x ty cells per workgroup of TT threads
// (256, or 128 so that every wave has pencils to apply on small tiles)
// ---------------------------------------------------------------------------
// The workgroup stages the tile's nodes plus one cell of halo on the low
// side in x and y, applies the operator to all (tx+1)(ty+1) cells, and
// assembles the owned nodes from their (up to four) adjacent cells.  The
// previous values u_{n-1} of the owned nodes are fetched together with the
// tile, so the kernel makes a single round trip to memory before writing.
constexpr int kOwnMax = 8;  // owned nodes per thread

template <int N, typename S, int TT>
__device__ __forceinline__ void explicit2d_body(const ExplicitArgs& A, int blk, int nblk) {
  using T = double;  // LDS and arithmetic
  constexpr int P = N - 1;
  const int tid = threadIdx.x;
  const int tile = xcd_contiguous(blk, nblk);
  const int tix = tile % A.ntx, tiy = tile / A.ntx;
  const int64_t nex = A.ne[0], ney = A.ne[1], nnx = A.nn[0];
  const int ex0 = tix * A.tx, ey0 = tiy * A.ty;
  const int txn = (int)min((int64_t)A.tx, nex - ex0), tyn = (int)min((int64_t)A.ty, ney - ey0);
  const int NX = txn + 1, NY = tyn + 1;          // local cells incl. the halo cell row / column
  const int WX = NX * P + 1, WY = NY * P + 1;
  const int WXmax = (A.tx + 1) * P + 1;
  const int NEmax = (A.tx + 1) * (A.ty + 1);
  const int WYmax = (A.ty + 1) * P + 1;
  const int64_t I0 = (int64_t)(ex0 - 1) * P, J0 = (int64_t)(ey0 - 1) * P;
  const int OX = txn * P + ((ex0 + txn == nex) ? 1 : 0), OY = tyn * P + ((ey0 + tyn == ney) ? 1 : 0);

  extern __shared__ double smem[];
  T* U = reinterpret_cast<T*>(smem);                 // [WYmax][WXmax]
  T* E1 = U + WYmax * WXmax;                          // [NEmax][N][N]: (a, b) -> T1, then Y
  T* E2 = E1 + NEmax * N * N;                         // [NEmax][N][N]: T2
  uint8_t* fl = reinterpret_cast<uint8_t*>(E2 + NEmax * N * N);

  const S* un = static_cast<const S*>(A.un);
  S* uw = static_cast<S*>(A.uw);
  const SmallDiv dOX(OX), dWX(WX), dNX(NX);
  // the step counter through the vector memory path: a scalar load here
  // would make every later wait on kernel arguments wait for it as well
  const double ft = A.ft[__builtin_nontemporal_load(A.step) + A.ft_offset];
  // cell flags of the first NX*NY / TT pass, issued with the node loads
  // so that the tile needs a single round trip to memory
  auto cell_flag = [&](int le) {
    int lx;
    const int ly = dNX.quot(le, &lx);
    const int64_t ex = ex0 - 1 + lx, ey = ey0 - 1 + ly;
    return (ex >= 0 && ey >= 0) ? A.flags[ey * nex + ex] : uint8_t(kEmpty);
  };
  const uint8_t f0 = tid < NX * NY ? cell_flag(tid) : uint8_t(kEmpty);
  // owned nodes of this thread and their previous values (issued first)
  T wprev[kOwnMax];
#pragma unroll
  for (int k = 0; k < kOwnMax; ++k) {
    const int o = tid + k * TT;
    wprev[k] = T(0);
    if (o < OX * OY) {
      int i;
      const int j = P + dOX.quot(o, &i);
      wprev[k] = uw[(J0 + j) * nnx + I0 + P + i];
    }
  }
  // tile nodes, up to 8 per thread in flight; a tile of at most 8 * TT
  // nodes (all but the largest tiles) takes one straight-line pass, which
  // keeps the loads above from being waited for at a loop header
  auto stage_nodes = [&](int base) {
    T v[8];
    int slot[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + tid + u * TT;
      v[u] = T(0);
      slot[u] = -1;
      if (base + u * TT < WY * WX && idx < WY * WX) {
        int i;
        const int j = dWX.quot(idx, &i);
        const int64_t I = I0 + i, J = J0 + j;
        if (I >= 0 && J >= 0) v[u] = un[J * nnx + I];
        slot[u] = j * WXmax + i;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (slot[u] >= 0) U[slot[u]] = v[u];
  };
  if (WY * WX <= TT * 8) {
    stage_nodes(0);
  } else {
    for (int base = 0; base < WY * WX; base += TT * 8) stage_nodes(base);
  }
  if (tid < NX * NY) fl[tid] = f0;
  for (int le = tid + TT; le < NX * NY; le += TT) fl[le] = cell_flag(le);
  __syncthreads();
  // y pencils of every cell: T1 = U Mh^T, T2 = U Kh^T  (per column a)
  for (int idx = tid; idx < NX * NY * N; idx += TT) {
    const int le = idx / N, a = idx - le * N;
    int lx;
    const int ly = dNX.quot(le, &lx);
    T u[N];
#pragma unroll
    for (int b = 0; b < N; ++b) u[b] = U[(ly * P + b) * WXmax + lx * P + a];
#pragma unroll
    for (int b = 0; b < N; ++b) {
      E1[(le * N + a) * N + b] = op_row<N>(A.Mh, b, u);
      E2[(le * N + a) * N + b] = op_row<N>(A.Kh, b, u);
    }
  }
  __syncthreads();
  // x pencils: Y = s_x Kh T1 + s_y Mh T2, zero for non-uncut cells
  const double sx = A.s[0], sy = A.s[1];
  for (int idx = tid; idx < NX * NY * N; idx += TT) {
    const int le = idx / N, b = idx - le * N;
    const bool on = fl[le] == kUncut;
    T t1[N], t2[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      t1[c] = E1[(le * N + c) * N + b];
      t2[c] = E2[(le * N + c) * N + b];
    }
#pragma unroll
    for (int a = 0; a < N; ++a) {
      const T y1 = op_row<N>(A.Kh, a, t1);
      const T y2 = op_row<N>(A.Mh, a, t2);
      E1[(le * N + a) * N + b] = on ? cell_combine(sx, y1, sy, y2) : T(0);
    }
  }
  __syncthreads();
  // owned nodes: assemble from the adjacent cells, lumped mass, CDM update
#pragma unroll
  for (int k = 0; k < kOwnMax; ++k) {
    const int o = tid + k * TT;
    if (o >= OX * OY) break;
    int i;
    const int j = P + dOX.quot(o, &i);
    i += P;
    int lxs[2], axs[2], nxs = 0, lys[2], ays[2], nys = 0;
    if (i % P == 0) {
      lxs[nxs] = i / P - 1; axs[nxs++] = P;
      if (i / P < NX) { lxs[nxs] = i / P; axs[nxs++] = 0; }
    } else {
      lxs[nxs] = i / P; axs[nxs++] = i % P;
    }
    if (j % P == 0) {
      lys[nys] = j / P - 1; ays[nys++] = P;
      if (j / P < NY) { lys[nys] = j / P; ays[nys++] = 0; }
    } else {
      lys[nys] = j / P; ays[nys++] = j % P;
    }
    T y = T(0);
    double m = 0.0;
    bool has_uncut = false, has_cut = false;
    for (int q = 0; q < nys; ++q)
      for (int p2 = 0; p2 < nxs; ++p2) {
        const int le = lys[q] * NX + lxs[p2];
        y += E1[(le * N + axs[p2]) * N + ays[q]];
        const uint8_t f = fl[le];
        if (f == kUncut) {
          m = mass_add(m, A.w[axs[p2]], A.w[ays[q]]);
          has_uncut = true;
        }
        has_cut |= (f == kCut);
      }
    if (!has_uncut || has_cut) continue;  // not a d node
    const int64_t I = I0 + i, J = J0 + j;
    double fx = 0.0;
    if (I >= A.sbox_lo[0] && I < A.sbox_hi[0] && J >= A.sbox_lo[1] && J < A.sbox_hi[1])
      fx = A.src_dense[(J - A.sbox_lo[1]) * (A.sbox_hi[0] - A.sbox_lo[0]) + (I - A.sbox_lo[0])];
    const double un_g = to_d(U[j * WXmax + i]);
    const double out = node_update(A, ft, fx, to_d(y), m, un_g, to_d(wprev[k]));
    const S outS = S(out);
    uw[J * nnx + I] = outS;
    if (A.write_u) static_cast<S*>(A.uout)[J * nnx + I] = S(un_g + to_d(outS));
  }
}

// ---------------------------------------------------------------------------
// 2D explicit step, register strips: one wave per strip of kStripCells cells
// in x (lane l holds cell strip * kStripCells + l; lane 63 is a halo cell)
// marching over lz cell rows (plus one halo row below).  Every lane keeps its
// cell's nodes and the cell's contributions Y in registers; a node shared
// with the right neighbour receives that neighbour's column by a lane shift,
// and the contributions to the top node row are carried to the next cell row.
// A lane owns the node columns a = 1..P of its cell (a = 0 too for the
// domain's first cell) and the node rows b = 0..P-1 of every cell row (the
// last cell row of the domain also the top node row).  Each node sums its
// cell contributions in the same order as the tile kernel (below-left,
// below-right, left, right), so both kernels give identical results.
// ---------------------------------------------------------------------------
// wave-local ordering of LDS writes before reads by other lanes of the wave
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N, typename S, int TT>
__global__ __launch_bounds__(TT) void explicit2d_kernel(const ExplicitArgs A) {
  explicit2d_body<N, S, TT>(A, blockIdx.x, gridDim.x);
}

// the same for every instance of a batch: workgroup b belongs to the instance
// i with first[i] <= b < first[i + 1]
template <int N, typename S, int TT>
__global__ __launch_bounds__(TT) void explicit2d_batch_kernel(const BatchTable<ExplicitArgs> B) {
  const int i = batch_instance(B.first, B.n, blockIdx.x);
  explicit2d_body<N, S, TT>(B.args[i], blockIdx.x - B.first[i], B.first[i + 1] - B.first[i]);
}

template <int N, typename S, bool STAGED>
__global__ __launch_bounds__(64) void explicit2d_strip_kernel(const ExplicitArgs A) {
  constexpr int P = N - 1;
  constexpr int kSlots = 64 * P;  // one node row of a strip: lane l's columns a = 1..P at l P + a - 1
  constexpr int kRow = kSlots + 1;  // a strip's node row (64 cells + 1 node)
  // one wave per workgroup; its LDS: the node rows of a cell row (u_n rows
  // 0..P, previous-value rows 0..P-1), loaded coalesced, and one staged
  // output row so that stores are contiguous
  __shared__ S stage_in[STAGED ? 2 * N - 1 : 1][kRow];
  __shared__ S stage_w[kSlots], stage_u[kSlots];
  __shared__ uint8_t stage_f[kSlots];
  const int lane = threadIdx.x;
  const int id = xcd_contiguous(blockIdx.x, gridDim.x);
  if (id >= A.ntx * A.nty) return;
  const int strip = id % A.ntx, chunk = id / A.ntx;
  const int64_t nex = A.ne[0], ney = A.ne[1], nnx = A.nn[0];
  const int64_t cx = (int64_t)strip * kStripCells + lane;
  const bool cell_in = cx < nex;
  const bool owner = lane < kStripCells && cell_in;
  const int a_lo = cx == 0 ? 0 : 1;
  const int64_t cy_begin = (int64_t)chunk * A.lz;
  const int64_t cy_end = min(ney, cy_begin + A.lz);
  const S* un = static_cast<const S*>(A.un);
  S* uw = static_cast<S*>(A.uw);
  const double ft = A.ft[A.step[0] + A.ft_offset];
  const double sx = A.s[0], sy = A.s[1];

  double carry[N];   // contributions of the cell row below to this row's bottom nodes
  double utop[N];    // the cell row below's top node row (this row's bottom)
  uint8_t fb = kEmpty, fbr = kEmpty;  // flags of the cells below and below-right
#pragma unroll
  for (int a = 0; a < N; ++a) carry[a] = utop[a] = 0.0;
  bool have_top = false;

  for (int64_t cy = cy_begin > 0 ? cy_begin - 1 : 0; cy <= cy_end; ++cy) {
    const bool pseudo = cy == ney;   // the top node row of the domain, after the last cell row
    if (cy == cy_end && !pseudo) break;
    const bool out_row = cy >= cy_begin;
    const int64_t rowJ = cy * P;
    uint8_t f = kEmpty;
    double U[N][N];
    // all node rows of this cell row at once: staged, 64 consecutive nodes
    // per load instruction through LDS (u_n rows b = 0..P, row 0 from the
    // previous cell row when available, and the previous values of the output
    // rows); direct, each lane loading its own cell's nodes
    const int64_t c0 = (int64_t)strip * kStripCells * P;
    const int64_t cols = min((int64_t)kRow, nnx - c0);
    const int n_out = out_row ? (pseudo ? 1 : P) : 0;
    if (!pseudo) f = cell_in ? A.flags[cy * nex + cx] : uint8_t(kEmpty);
    double wv_all[STAGED ? 1 : N][N];
    if constexpr (STAGED) {
      S v[2 * N - 1][P + 1];
#pragma unroll
      for (int r = 0; r < 2 * N - 1; ++r) {
        const bool is_u = r < N;
        const int b = is_u ? r : r - N;
        const bool need = is_u ? (!pseudo && !(b == 0 && have_top)) : (b < n_out);
        if (!need) continue;
        const S* src = is_u ? un : uw;
#pragma unroll
        for (int k = 0; k <= P; ++k) {
          const int col = k * 64 + lane;
          v[r][k] = col < cols ? src[(rowJ + b) * nnx + c0 + col] : S(0);
        }
      }
#pragma unroll
      for (int r = 0; r < 2 * N - 1; ++r) {
        const bool is_u = r < N;
        const int b = is_u ? r : r - N;
        const bool need = is_u ? (!pseudo && !(b == 0 && have_top)) : (b < n_out);
        if (!need) continue;
#pragma unroll
        for (int k = 0; k <= P; ++k) {
          const int col = k * 64 + lane;
          if (col < kRow) stage_in[r][col] = v[r][k];
        }
      }
      wave_lds_sync();
#pragma unroll
      for (int b = 0; b < N; ++b)
#pragma unroll
        for (int a = 0; a < N; ++a) {
          if (b == 0 && (have_top || pseudo)) U[a][0] = utop[a];
          else U[a][b] = (cell_in && !pseudo) ? to_d(stage_in[b][lane * P + a]) : 0.0;
        }
    } else {
      if (n_out > 0 && owner) {
#pragma unroll
        for (int b = 0; b < P; ++b)
#pragma unroll
          for (int a = 0; a < N; ++a)
            if (b < n_out && a >= a_lo) wv_all[b][a] = to_d(uw[(rowJ + b) * nnx + cx * P + a]);
      }
#pragma unroll
      for (int b = 0; b < N; ++b)
#pragma unroll
        for (int a = 0; a < N; ++a) {
          if (b == 0 && (have_top || pseudo)) U[a][0] = utop[a];
          else U[a][b] = (cell_in && !pseudo) ? to_d(un[(rowJ + b) * nnx + cx * P + a]) : 0.0;
        }
    }
    const uint8_t fr = (uint8_t)__shfl_down((int)f, 1, 64);
    const uint8_t frr = (lane == 63) ? uint8_t(kEmpty) : fr;
    // column b of Y = sx Kh U Mh^T + sy Mh U Kh^T, then node row b; the top
    // column (b = P) is carried to the next cell row
#pragma unroll
    for (int b = 0; b < N; ++b) {
      const bool row_out = out_row && b < P && (!pseudo || b == 0);
      if (!row_out && b != P) continue;
      if (pseudo && b == P) continue;
      // previous values of this row's owned nodes (loaded above)
      double wv[N];
      if (row_out) {
#pragma unroll
        for (int a = 0; a < N; ++a) {
          if constexpr (STAGED) wv[a] = to_d(stage_in[N + b][lane * P + a]);
          else wv[a] = wv_all[b < P ? b : 0][a];
        }
      }
      double Yc[N];
      if (!pseudo) {
        double t1[N], t2[N];
#pragma unroll
        for (int c = 0; c < N; ++c) {
          double u[N];
#pragma unroll
          for (int d = 0; d < N; ++d) u[d] = U[c][d];
          t1[c] = op_row<N>(A.Mh, b, u);
          t2[c] = op_row<N>(A.Kh, b, u);
        }
#pragma unroll
        for (int a = 0; a < N; ++a) {
          const double y1 = op_row<N>(A.Kh, a, t1);
          const double y2 = op_row<N>(A.Mh, a, t2);
          Yc[a] = f == kUncut ? cell_combine(sx, y1, sy, y2) : 0.0;
        }
      } else {
#pragma unroll
        for (int a = 0; a < N; ++a) Yc[a] = 0.0;
      }
      const double Rb = __shfl_down(Yc[0], 1, 64);  // the right neighbour's first column
      if (b == P) {
        // carry the top row (the tile kernel adds below-left, then below-right)
#pragma unroll
        for (int a = 0; a < N; ++a) carry[a] = a == P ? Yc[P] + Rb : Yc[a];
        continue;
      }
      const int64_t J = rowJ + b;
#pragma unroll
      for (int a = 0; a < N; ++a) {
        // the domain's first node column (a = 0 of cell 0) is stored
        // directly; columns a = 1..P go through the staging row
        bool d_node = false;
        S vw = S(0), vu = S(0);
        if (owner && a >= a_lo) {
          // cell contributions in the tile kernel's order
          double y = 0.0, m = 0.0;
          bool has_uncut = false, has_cut = false;
          auto add_flag = [&](uint8_t fl, int la, int lb) {
            if (fl == kUncut) {
              m = mass_add(m, A.w[la < P - la ? la : P - la], A.w[lb < P - lb ? lb : P - lb]);
              has_uncut = true;
            }
            has_cut |= (fl == kCut);
          };
          if (b == 0) {
            y += carry[a];
            add_flag(fb, a, P);
            if (a == P) add_flag(fbr, 0, P);
          }
          y += Yc[a];
          add_flag(f, a, b);
          if (a == P) {
            y += Rb;
            add_flag(frr, 0, b);
          }
          d_node = has_uncut && !has_cut;
          if (d_node) {
            const int64_t I = cx * P + a;
            double fx = 0.0;
            if (I >= A.sbox_lo[0] && I < A.sbox_hi[0] && J >= A.sbox_lo[1] && J < A.sbox_hi[1])
              fx = A.src_dense[(J - A.sbox_lo[1]) * (A.sbox_hi[0] - A.sbox_lo[0]) + (I - A.sbox_lo[0])];
            const double un_g = U[a][b];
            const double outv = node_update(A, ft, fx, y, m, un_g, wv[a]);
            vw = S(outv);
            vu = S(un_g + to_d(vw));
          }
        }
        if (a == 0) {
          if (d_node) {
            uw[J * nnx + cx * P] = vw;
            if (A.write_u) static_cast<S*>(A.uout)[J * nnx + cx * P] = vu;
          }
        } else {
          stage_w[lane * P + a - 1] = vw;
          stage_u[lane * P + a - 1] = vu;
          stage_f[lane * P + a - 1] = d_node ? 1 : 0;
        }
      }
      wave_lds_sync();
      // contiguous write-out of the strip's columns cx0 P + 1 + slot
      const int64_t col0 = (int64_t)strip * kStripCells * P + 1;
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const int slot = k * 64 + lane;
        if (slot < kStripCells * P && stage_f[slot]) {
          const int64_t g = J * nnx + col0 + slot;
          uw[g] = stage_w[slot];
          if (A.write_u) static_cast<S*>(A.uout)[g] = stage_u[slot];
        }
      }
      wave_lds_sync();
    }
    if (pseudo) break;
    if constexpr (STAGED) wave_lds_sync();
#pragma unroll
    for (int a = 0; a < N; ++a) utop[a] = U[a][P];
    have_top = true;
    fb = f;
    fbr = frr;
  }
}

// ---------------------------------------------------------------------------
// 3D explicit step (march along z)
// ---------------------------------------------------------------------------
// LDS layout of the 3D kernel for N = 4 (p = 3), chosen against bank
// conflicts: a cell's 16 pencils fill one 64-lane wave quarter, and with the
// plain layout their strides are multiples of 16 doubles.  A node row of the
// staged planes is padded to a stride of 4 or 12 (mod 16) doubles, so that
// the pencils (a, b) of a cell read 16 different banks; a cell's values
// (c, b, a) sit at 16 c + 4 ((b + c) mod 4) + (a + c) mod 4, a bijection per
// plane c under which each pass's lanes, over (a, b), (a, c) or (b, c), fall
// on different banks as well.  Other orders keep the plain layout (odd row
// strides; measured slower with the skew for N = 5).
__host__ __device__ inline int row_stride3d(int wx, int n) {
  if (n != 4) return wx;
  while ((wx & 7) != 4) ++wx;
  return wx;
}
template <int N>
__device__ inline int skew(int c, int b, int a) {
  if constexpr (N == 4) return 16 * c + 4 * ((b + c) & 3) + ((a + c) & 3);
  else return (c * N + b) * N + a;
}

// The (up to two) local cells along one direction around local node
// coordinate i, in increasing order, with the node's index in each; kept in
// named registers (a dynamically indexed array would live in scratch).
struct Adj2 {
  int l0, a0, l1, a1, n;
};
template <int P>
__device__ inline Adj2 adjacent_cells(int i, int ncell) {
  const int q = i / P, r = i - q * P;
  if (r != 0) return Adj2{q, r, q, r, 1};
  const bool lo = q >= 1, hi = q < ncell;
  return Adj2{lo ? q - 1 : q, lo ? P : 0, q, 0, (lo ? 1 : 0) + (hi ? 1 : 0)};
}

template <int N, typename S, int TT>
__global__ __launch_bounds__(TT) void explicit3d_kernel(const ExplicitArgs A) {
  using T = double;  // LDS and arithmetic
  constexpr int P = N - 1;
  constexpr int N2 = N * N, N3 = N * N * N;
  const int tid = threadIdx.x;
  const int tiles = A.ntx * A.nty;
  const int bid = xcd_contiguous(blockIdx.x, gridDim.x);
  const int tile = bid % tiles;
  const int chunk = bid / tiles;
  const int tix = tile % A.ntx, tiy = tile / A.ntx;
  const int64_t nex = A.ne[0], ney = A.ne[1], nez = A.ne[2];
  const int64_t nnx = A.nn[0], nny = A.nn[1];
  const int ex0 = tix * A.tx, ey0 = tiy * A.ty;
  const int txn = (int)min((int64_t)A.tx, nex - ex0);
  const int tyn = (int)min((int64_t)A.ty, ney - ey0);
  const int NX = txn + 1, NY = tyn + 1;       // local cells incl. the low-side halo
  const int NE = NX * NY;
  const int WX = NX * P + 1, WY = NY * P + 1; // local node columns / rows
  const int NXmax = A.tx + 1, NYmax = A.ty + 1;
  const int WXmax = row_stride3d(NXmax * P + 1, N), WYmax = NYmax * P + 1;
  const int PL = WXmax * WYmax;               // plane stride in LDS
  const int NEmax = NXmax * NYmax;
  const int64_t I0 = (int64_t)(ex0 - 1) * P, J0 = (int64_t)(ey0 - 1) * P;
  const int ez_begin = chunk * A.lz;
  const int ez_end = (int)min((int64_t)ez_begin + A.lz, nez);
  const bool last_x = (ex0 + txn == nex), last_y = (ey0 + tyn == ney);
  const int ox_lo = P, ox_hi = P + txn * P + (last_x ? 1 : 0);
  const int oy_lo = P, oy_hi = P + tyn * P + (last_y ? 1 : 0);
  const int OX = ox_hi - ox_lo, OY = oy_hi - oy_lo;

  extern __shared__ double smem[];
  T* U = reinterpret_cast<T*>(smem);          // [N][WYmax][WXmax]
  T* E1 = U + N * PL;                         // [NEmax][N3], index skew(c, b, a)
  T* E2 = E1 + NEmax * N3;
  T* carry = E2 + NEmax * N3;                 // [2][PL]
  uint8_t* flc = reinterpret_cast<uint8_t*>(carry + 2 * PL);  // [NEmax]
  uint8_t* flp = flc + NEmax;

  const S* un = static_cast<const S*>(A.un);
  S* uw = static_cast<S*>(A.uw);
  const double ft = A.ft[A.step[0] + A.ft_offset];
  const double sx = A.s[0], sy = A.s[1], sz = A.s[2];
  const SmallDiv dPlane(WY * WX), dWX(WX), dNX(NX), dOPlane(OY * OX), dOX(OX);

  for (int i = tid; i < 2 * PL; i += TT) carry[i] = T(0);
  int cur = 0;
  const int ez_start = ez_begin > 0 ? ez_begin - 1 : ez_begin;
  for (int ez = ez_start; ez < ez_end; ++ez) {
    const bool out_layer = ez >= ez_begin;
    const bool top = (ez == nez - 1);
    // the layer's cell flags (first pass) and node planes, with every load
    // in flight before the first LDS store: one round trip to memory per
    // layer (per 8 TT staged values)
    uint8_t fc0 = uint8_t(kEmpty), fp0 = uint8_t(kEmpty);
    if (tid < NE) {
      int lx;
      const int ly = dNX.quot(tid, &lx);
      const int64_t ex = ex0 - 1 + lx, ey = ey0 - 1 + ly;
      const bool ok = ex >= 0 && ex < nex && ey >= 0 && ey < ney;
      if (ok) fc0 = A.flags[((int64_t)ez * ney + ey) * nex + ex];
      if (ok && ez > 0) fp0 = A.flags[((int64_t)(ez - 1) * ney + ey) * nex + ex];
    }
    for (int base = 0; base < N * WY * WX; base += 8 * TT) {
      T v[8];
      int slot[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = base + tid + u * TT;
        v[u] = T(0);
        slot[u] = -1;
        if (idx < N * WY * WX) {
          int rem, i;
          const int c = dPlane.quot(idx, &rem);
          const int j = dWX.quot(rem, &i);
          const int64_t I = I0 + i, J = J0 + j, K = (int64_t)ez * P + c;
          if (I >= 0 && I < nnx && J >= 0 && J < nny) v[u] = un[(K * nny + J) * nnx + I];
          slot[u] = c * PL + j * WXmax + i;
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (slot[u] >= 0) U[slot[u]] = v[u];
    }
    if (tid < NE) {
      flc[tid] = fc0;
      flp[tid] = fp0;
    }
    for (int le = tid + TT; le < NE; le += TT) {
      int lx;
      const int ly = dNX.quot(le, &lx);
      const int64_t ex = ex0 - 1 + lx, ey = ey0 - 1 + ly;
      const bool ok = ex >= 0 && ex < nex && ey >= 0 && ey < ney;
      flc[le] = ok ? A.flags[((int64_t)ez * ney + ey) * nex + ex] : uint8_t(kEmpty);
      flp[le] = (ok && ez > 0) ? A.flags[((int64_t)(ez - 1) * ney + ey) * nex + ex] : uint8_t(kEmpty);
    }
    __syncthreads();
    // z pencils (a, b): A = Mh_z U, B = Kh_z U
    for (int idx = tid; idx < NE * N2; idx += TT) {
      const int le = idx / N2, ab = idx - le * N2;
      const int b = ab / N, a = ab - b * N;
      int lx;
      const int ly = dNX.quot(le, &lx);
      const int base = (ly * P + b) * WXmax + lx * P + a;
      T u[N];
#pragma unroll
      for (int c = 0; c < N; ++c) u[c] = U[c * PL + base];
      T* e1 = E1 + le * N3;
      T* e2 = E2 + le * N3;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        e1[skew<N>(c, b, a)] = op_row<N>(A.Mh, c, u);
        e2[skew<N>(c, b, a)] = op_row<N>(A.Kh, c, u);
      }
    }
    __syncthreads();
    // y pencils (a, c): C = Mh_y A, G = s_y Kh_y A + s_z Mh_y B
    for (int idx = tid; idx < NE * N2; idx += TT) {
      const int le = idx / N2, ac = idx - le * N2;
      const int c = ac / N, a = ac - c * N;
      T* e1 = E1 + le * N3;
      T* e2 = E2 + le * N3;
      T ta[N], tb[N];
#pragma unroll
      for (int e = 0; e < N; ++e) {
        ta[e] = e1[skew<N>(c, e, a)];
        tb[e] = e2[skew<N>(c, e, a)];
      }
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const T cc = op_row<N>(A.Mh, b, ta);
        const T dd = op_row<N>(A.Kh, b, ta);
        const T ee = op_row<N>(A.Mh, b, tb);
        e1[skew<N>(c, b, a)] = cc;
        e2[skew<N>(c, b, a)] = sy * dd + sz * ee;
      }
    }
    __syncthreads();
    // x pencils (b, c): Y = s_x Kh_x C + Mh_x G, zero for non-uncut cells
    for (int idx = tid; idx < NE * N2; idx += TT) {
      const int le = idx / N2, bc = idx - le * N2;
      const int c = bc / N, b = bc - c * N;
      const bool on = flc[le] == kUncut;
      T* e1 = E1 + le * N3;
      const T* e2 = E2 + le * N3;
      T tc[N], tg[N];
#pragma unroll
      for (int f = 0; f < N; ++f) {
        tc[f] = e1[skew<N>(c, b, f)];
        tg[f] = e2[skew<N>(c, b, f)];
      }
#pragma unroll
      for (int a = 0; a < N; ++a) {
        const T y1 = op_row<N>(A.Kh, a, tc);
        const T y2 = op_row<N>(A.Mh, a, tg);
        e1[skew<N>(c, b, a)] = on ? sx * y1 + y2 : T(0);
      }
    }
    __syncthreads();
    T* cin = carry + cur * PL;
    T* cout = carry + (1 - cur) * PL;
    const int nplanes = top ? N : P;
    if (out_layer) {
      for (int idx = tid; idx < nplanes * OY * OX; idx += TT) {
        int rem, i;
        const int c = dOPlane.quot(idx, &rem);
        const int j = oy_lo + dOX.quot(rem, &i);
        i += ox_lo;
        const Adj2 X = adjacent_cells<P>(i, NX), Y = adjacent_cells<P>(j, NY);
        T y = T(0);
        double m = 0.0;
        bool has_uncut = false, has_cut = false;
#pragma unroll
        for (int sy_ = 0; sy_ < 2; ++sy_) {
          if (sy_ >= Y.n) break;
          const int ly = sy_ ? Y.l1 : Y.l0, ay = sy_ ? Y.a1 : Y.a0;
#pragma unroll
          for (int sx_ = 0; sx_ < 2; ++sx_) {
            if (sx_ >= X.n) break;
            const int lx = sx_ ? X.l1 : X.l0, ax = sx_ ? X.a1 : X.a0;
            const int le = ly * NX + lx;
            y += E1[le * N3 + skew<N>(c, ay, ax)];
            const uint8_t f = flc[le];
            if (f == kUncut) { m += A.w[ax] * A.w[ay] * A.w[c]; has_uncut = true; }
            has_cut |= (f == kCut);
            if (c == 0) {
              const uint8_t fp = flp[le];
              if (fp == kUncut) { m += A.w[ax] * A.w[ay] * A.w[P]; has_uncut = true; }
              has_cut |= (fp == kCut);
            }
          }
        }
        if (c == 0) y += cin[j * WXmax + i];
        if (!has_uncut || has_cut) continue;
        const int64_t I = I0 + i, J = J0 + j, K = (int64_t)ez * P + c;
        const int64_t g = (K * nny + J) * nnx + I;
        double fx = 0.0;
        if (I >= A.sbox_lo[0] && I < A.sbox_hi[0] && J >= A.sbox_lo[1] && J < A.sbox_hi[1] &&
            K >= A.sbox_lo[2] && K < A.sbox_hi[2]) {
          const int64_t bx = A.sbox_hi[0] - A.sbox_lo[0], by = A.sbox_hi[1] - A.sbox_lo[1];
          fx = A.src_dense[((K - A.sbox_lo[2]) * by + (J - A.sbox_lo[1])) * bx + (I - A.sbox_lo[0])];
        }
        const double acc = (ft * fx - to_d(y)) / (A.mass_scale * m);
        const double un_g = to_d(U[c * PL + j * WXmax + i]);
        const double out = A.c1 * un_g + A.c2 * to_d(uw[g]) + A.c3 * A.dt2 * acc;
        const S outS = S(out);
        uw[g] = outS;
        if (A.write_u) static_cast<S*>(A.uout)[g] = S(un_g + to_d(outS));
      }
    }
    // contribution of this layer to its top node plane (all local columns)
    for (int idx = tid; idx < WY * WX; idx += TT) {
      int i;
      const int j = dWX.quot(idx, &i);
      const Adj2 X = adjacent_cells<P>(i, NX), Y = adjacent_cells<P>(j, NY);
      T y = T(0);
#pragma unroll
      for (int sy_ = 0; sy_ < 2; ++sy_) {
        if (sy_ >= Y.n) break;
        const int ly = sy_ ? Y.l1 : Y.l0, ay = sy_ ? Y.a1 : Y.a0;
#pragma unroll
        for (int sx_ = 0; sx_ < 2; ++sx_) {
          if (sx_ >= X.n) break;
          const int lx = sx_ ? X.l1 : X.l0, ax = sx_ ? X.a1 : X.a0;
          y += E1[(ly * NX + lx) * N3 + skew<N>(P, ay, ax)];
        }
      }
      cout[j * WXmax + i] = y;
    }
    cur = 1 - cur;
    __syncthreads();
  }
}
// ---------------------------------------------------------------------------
// 3D explicit step, tensor-product form
// ---------------------------------------------------------------------------
// On a node whose adjacent cells are all uncut, the row of the assembled
// stiffness is that of the Kronecker sum
//   s_x Kx (x) My (x) Mz + s_y Mx (x) Ky (x) Mz + s_z Mx (x) My (x) Kz
// of the assembled 1D operators along the three grid lines through the
// node, and its lumped mass is the product of the assembled 1D GLL weights.
// An assembled 1D operator is a band of half-width P: node a (0 < a < P) of
// cell q takes row a of the cell matrix over the nodes of q, and the vertex
// shared by cells q-1 and q takes row P over q-1 plus row 0 over q (only one
// of the two at the ends of a line).  The host marks these nodes in a
// bitmask; the other d nodes (next to an empty cell) are listed and summed
// cell by cell (explicit3d_rest_kernel).
//
// A workgroup owns the node slots of CX x CY cells in x and y (slot q: the P
// nodes of cell q from its low vertex on; the tile with the last cell also
// owns the last vertex) and of a chunk of lz cell layers in z, and marches up
// the chunk one node plane at a time:
//   z pass  A = Mz u, B = Kz u on the node columns of the tile and its halo
//           (one slot below, one node above, in x and y), every thread
//           holding the 2P+1 planes around the current one of its columns
//           in registers;
//   y pass  C = My A, G = s_y Ky A + s_z My B on the halo width in x and the
//           owned rows, one slot (P rows) per thread;
//   x pass  Y = s_x Kx C + Mx G on the owned nodes, one slot per thread, and
//           the CDM update of the marked nodes.
// Every node is computed by the same operations in the same order whatever
// the tile and chunk, so all launch shapes of this form agree bit for bit.

// vertex row of an assembled band: row P of the cell below over v[0..P]
// (nodes i-P..i) and row 0 of the cell above over v[P..2P] (nodes i..i+P)
template <int P>
__device__ inline double band_vertex(const double* C, const double* v, bool below, bool above) {
  constexpr int N = P + 1;
  double l = 0.0, r = 0.0;
#pragma unroll
  for (int d = 0; d <= P; ++d) {
    l = fma(C[canon<N>(P, d)], v[d], l);
    r = fma(C[canon<N>(0, d)], v[P + d], r);
  }
  return (below ? l : 0.0) + (above ? r : 0.0);
}
// row a (0 < a < P) of the cell matrix over the cell's nodes v[0..P]
template <int P>
__device__ inline double band_inner(const double* C, int a, const double* v) {
  constexpr int N = P + 1;
  double acc = 0.0;
#pragma unroll
  for (int d = 0; d <= P; ++d) acc = fma(C[canon<N>(a, d)], v[d], acc);
  return acc;
}
// assembled 1D GLL weight of node i on a line of ne cells
template <int P>
__device__ inline double line_weight(const double* w, int64_t i, int64_t ne) {
  const int64_t q = i / P;
  const int a = (int)(i - q * P);
  if (a != 0) return w[a];
  return (q > 0 ? w[P] : 0.0) + (q < ne ? w[0] : 0.0);
}

// the same weight for node a (0 <= a < P, a = 0 the vertex below) of cell q,
// where the caller's a is a compile-time index: no indexed argument load
template <int P>
__device__ inline double line_weight_at(const double* w, int64_t q, int a, int64_t ne) {
  if (a != 0) return w[a];
  return (q > 0 ? w[P] : 0.0) + (q < ne ? w[0] : 0.0);
}

// P <= 3 fits 128 registers, i.e. two workgroups per CU
template <int P, typename S>
__global__ __attribute__((amdgpu_flat_work_group_size(1, kKronThreads), amdgpu_waves_per_eu(P <= 3 ? 4 : 2)))
void explicit3d_kron_kernel(const ExplicitArgs A) {
  constexpr int W = 2 * P + 1;
  constexpr int CX = kKronCX[P], CY = kKronCY[P];
  constexpr int NXH = (CX + 1) * P + 1, NYH = (CY + 1) * P + 1;  // node columns of the z pass
  constexpr int NCOL = NXH * NYH;
  constexpr int CPT = (NCOL + kKronThreads - 1) / kKronThreads;   // columns per thread
  constexpr int NYO = CY * P + 1;                                 // owned rows, the last vertex row included
  constexpr int NXO = CX + 1;                                     // owned slots in x, the last vertex slot included
  static_assert(NXH * (CY + 1) <= kKronThreads && NXO * NYO <= kKronThreads, "one task per thread and pass");
  __shared__ double sA[NYH * NXH], sB[NYH * NXH], sC[NYO * NXH], sG[NYO * NXH];

  const int tid = threadIdx.x;
  const int tiles = A.ntx * A.nty;
  const int bid = xcd_contiguous(blockIdx.x, gridDim.x);
  const int tile = bid % tiles, chunk = bid / tiles;
  const int tix = tile % A.ntx, tiy = tile / A.ntx;
  const int64_t ne0 = A.ne[0], ne1 = A.ne[1], ne2 = A.ne[2];
  const int64_t nnx = A.nn[0], nny = A.nn[1], nnz = A.nn[2];
  const int64_t plane = nnx * nny;
  const int64_t sx0 = (int64_t)tix * CX, sy0 = (int64_t)tiy * CY, sz0 = (int64_t)chunk * A.lz;
  const int64_t rz_end = sz0 + A.lz >= ne2 ? ne2 + 1 : sz0 + A.lz;  // slots of the chunk in z
  const int64_t X0 = P * sx0 - P, Y0 = P * sy0 - P;                 // first node column / row of the halo
  const S* un = static_cast<const S*>(A.un);
  S* uw = static_cast<S*>(A.uw);
  const double ft = A.ft[A.step[0] + A.ft_offset];
  const double sx = A.s[0], sy = A.s[1], sz = A.s[2];

  // z pass: the thread's columns (grid offset J nnx + I, or -1 outside the grid)
  int col[CPT];
#pragma unroll
  for (int u = 0; u < CPT; ++u) {
    const int c = tid + u * kKronThreads;
    col[u] = -1;
    if (c < NCOL) {
      const int y = c / NXH, x = c - y * NXH;
      const int64_t I = X0 + x, J = Y0 + y;
      if (I >= 0 && I < nnx && J >= 0 && J < nny) col[u] = (int)(J * nnx + I);
    }
  }
  // y pass: column yx of the halo width, owned slot yq
  const int yq = tid / NXH, yx = tid - yq * NXH;
  const int64_t gyq = sy0 + yq;
  const bool ytask = yq <= CY && gyq <= ne1 && (yq < CY || gyq == ne1);
  // x pass: owned slot xs, owned row xr
  const int xr = tid / NXO, xs = tid - xr * NXO;
  const int64_t gxs = sx0 + xs, Jx = P * sy0 + xr;
  const bool xtask = xr < NYO && Jx < nny && (xr < CY * P || Jx == nny - 1) && gxs <= ne0 &&
                     (xs < CX || gxs == ne0);
  const int xoff = xtask ? (int)(Jx * nnx + P * gxs) : 0;  // offset of the slot's first node in a plane
  bool xok[P];
#pragma unroll
  for (int e = 0; e < P; ++e) xok[e] = xtask && (e == 0 || gxs < ne0);
  const double wy = xtask ? line_weight<P>(A.w, Jx, ne1) : 0.0;
  const bool src_y = Jx >= A.sbox_lo[1] && Jx < A.sbox_hi[1];

  // The chunk's slots in z, walked up (odd chunks) or down (even chunks):
  // the chunks on either side of a boundary then read the planes around it
  // at about the same time (both at the start or both at the end), so the
  // second read finds them in L2 when both run on one XCD.  Every plane is
  // computed by the same operations either way.
  const bool down = (chunk & 1) == 0;  // uniform over the workgroup
  const int64_t nslot = rz_end - sz0;
  const int64_t r0 = down ? rz_end - 1 : sz0;
  // the window: planes P r0 - P .. P r0 + P (zero outside the grid)
  double win[CPT][W];
#pragma unroll
  for (int u = 0; u < CPT; ++u)
#pragma unroll
    for (int d = 0; d < W; ++d) {
      const int64_t k = P * r0 - P + d;
      win[u][d] = (col[u] >= 0 && k >= 0 && k < nnz) ? to_d(un[k * plane + col[u]]) : 0.0;
    }

  for (int64_t i = 0; i < nslot; ++i) {
    const int64_t r = down ? r0 - i : r0 + i;
#pragma unroll
    for (int a = 0; a < P; ++a) {
      if (a > 0 && r == ne2) break;  // the top vertex plane alone (uniform)
      const int64_t k = P * r + a;
      const S* un_k = un + k * plane;  // the plane's state, offsets J nnx + I below
      S* uw_k = uw + k * plane;
      const uint32_t bit0 = (uint32_t)((k * plane) & 31);
      const uint32_t* mask_k = A.kron_mask + ((k * plane) >> 5);
      // the plane's state and mask words at the thread's x-pass nodes, loaded
      // ahead of the passes; no load waits on another
      double unv[P], uwv[P];
      uint32_t mw[P];
#pragma unroll
      for (int e = 0; e < P; ++e) {
        const int o = xoff + e;
        mw[e] = xok[e] ? mask_k[(bit0 + (uint32_t)o) >> 5] : 0u;
        unv[e] = xok[e] ? to_d(un_k[o]) : 0.0;
        uwv[e] = xok[e] ? to_d(uw_k[o]) : 0.0;
      }
      // z pass
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
        const int c = tid + u * kKronThreads;
        if (c < NCOL) {
          double av, bv;
          if (a == 0) {
            av = band_vertex<P>(A.Mh, win[u], r > 0, r < ne2);
            bv = band_vertex<P>(A.Kh, win[u], r > 0, r < ne2);
          } else {
            av = band_inner<P>(A.Mh, a, win[u] + P);
            bv = band_inner<P>(A.Kh, a, win[u] + P);
          }
          sA[c] = av;
          sB[c] = bv;
        }
      }
      __syncthreads();
      // y pass
      if (ytask) {
        double va[W], vb[W];
#pragma unroll
        for (int d = 0; d < W; ++d) {
          const bool ok = d <= P || yq < CY;  // the last vertex slot reads no rows above the halo
          const int i = (P * yq + d) * NXH + yx;
          va[d] = ok ? sA[i] : 0.0;
          vb[d] = ok ? sB[i] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < P; ++b) {
          if (b > 0 && gyq == ne1) break;
          double cv, dv, ev;
          if (b == 0) {
            cv = band_vertex<P>(A.Mh, va, gyq > 0, gyq < ne1);
            dv = band_vertex<P>(A.Kh, va, gyq > 0, gyq < ne1);
            ev = band_vertex<P>(A.Mh, vb, gyq > 0, gyq < ne1);
          } else {
            cv = band_inner<P>(A.Mh, b, va + P);
            dv = band_inner<P>(A.Kh, b, va + P);
            ev = band_inner<P>(A.Mh, b, vb + P);
          }
          const int o = (P * yq + b) * NXH + yx;
          sC[o] = cv;
          sG[o] = fma(sy, dv, sz * ev);
        }
      }
      __syncthreads();
      // x pass and the CDM update
      if (xtask) {
        double vc[W], vg[W];
#pragma unroll
        for (int d = 0; d < W; ++d) {
          const bool ok = d <= P || xs < CX;
          const int i = xr * NXH + P * xs + d;
          vc[d] = ok ? sC[i] : 0.0;
          vg[d] = ok ? sG[i] : 0.0;
        }
        const double wz = line_weight_at<P>(A.w, r, a, ne2);
        const bool src_yz = src_y && k >= A.sbox_lo[2] && k < A.sbox_hi[2];
#pragma unroll
        for (int e = 0; e < P; ++e) {
          if (!((mw[e] >> ((bit0 + (uint32_t)(xoff + e)) & 31)) & 1u)) continue;  // not a marked d node
          double y1, y2;
          if (e == 0) {
            y1 = band_vertex<P>(A.Kh, vc, gxs > 0, gxs < ne0);
            y2 = band_vertex<P>(A.Mh, vg, gxs > 0, gxs < ne0);
          } else {
            y1 = band_inner<P>(A.Kh, e, vc + P);
            y2 = band_inner<P>(A.Mh, e, vg + P);
          }
          const double y = fma(sx, y1, y2);
          const int64_t I = P * gxs + e;
          const double m = line_weight_at<P>(A.w, gxs, e, ne0) * wy * wz;
          double fx = 0.0;
          if (src_yz && I >= A.sbox_lo[0] && I < A.sbox_hi[0]) {
            const int64_t bx = A.sbox_hi[0] - A.sbox_lo[0], by = A.sbox_hi[1] - A.sbox_lo[1];
            fx = A.src_dense[((k - A.sbox_lo[2]) * by + (Jx - A.sbox_lo[1])) * bx + (I - A.sbox_lo[0])];
          }
          const S outS = S(node_update(A, ft, fx, y, m, unv[e], uwv[e]));
          uw_k[xoff + e] = outS;
          if (A.write_u) static_cast<S*>(A.uout)[k * plane + xoff + e] = S(unv[e] + to_d(outS));
        }
      }
    }
    // slide the window one slot: planes P r' - P .. P r' + P of the next slot r'
    const bool more = i + 1 < nslot;
    if (down) {
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
#pragma unroll
        for (int d = 2 * P; d >= P; --d) win[u][d] = win[u][d - P];
#pragma unroll
        for (int d = 0; d < P; ++d) {
          const int64_t k = P * r - 2 * P + d;
          win[u][d] = (more && col[u] >= 0 && k >= 0) ? to_d(un[k * plane + col[u]]) : 0.0;
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < CPT; ++u) {
#pragma unroll
        for (int d = 0; d <= P; ++d) win[u][d] = win[u][d + P];
#pragma unroll
        for (int d = 0; d < P; ++d) {
          const int64_t k = P * r + P + 1 + d;
          win[u][P + 1 + d] = (more && col[u] >= 0 && k < nnz) ? to_d(un[k * plane + col[u]]) : 0.0;
        }
      }
    }
  }
}

// The d nodes next to an empty cell: one wave per node sums the rows of its
// adjacent uncut cells' matrices (sum-factorised entries, one cell dof per
// lane) and their GLL weights.
template <typename S>
__global__ __launch_bounds__(kThreads) void explicit3d_rest_kernel(const ExplicitArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (i >= A.n_rest) return;
  const int P = A.p, N = P + 1, N3 = N * N * N;
  const int64_t nnx = A.nn[0], nny = A.nn[1];
  const int64_t g = A.kron_rest[i];
  const int64_t I = g % nnx, J = (g / nnx) % nny, K = g / (nnx * nny);
  const int64_t G[3] = {I, J, K};
  int64_t c0[3];
  int l0[3], nc[3];
  for (int k = 0; k < 3; ++k) {
    const int64_t q = G[k] / P;
    const int a = (int)(G[k] - q * P);
    if (a != 0) {
      c0[k] = q;
      l0[k] = a;
      nc[k] = 1;
    } else {
      c0[k] = q > 0 ? q - 1 : q;  // the cell below first
      l0[k] = q > 0 ? P : 0;
      nc[k] = (q > 0 ? 1 : 0) + (q < A.ne[k] ? 1 : 0);
    }
  }
  const S* un = static_cast<const S*>(A.un);
  double acc = 0.0, m = 0.0;
  for (int tz = 0; tz < nc[2]; ++tz)
    for (int ty = 0; ty < nc[1]; ++ty)
      for (int tx = 0; tx < nc[0]; ++tx) {
        const int64_t cx = c0[0] + tx, cy = c0[1] + ty, cz = c0[2] + tz;
        if (A.flags[(cz * A.ne[1] + cy) * A.ne[0] + cx] != kUncut) continue;
        const int a = tx ? 0 : l0[0], b = ty ? 0 : l0[1], c = tz ? 0 : l0[2];
        for (int t = lane; t < N3; t += 64) {
          const int a2 = t % N, b2 = (t / N) % N, c2 = t / (N * N);
          const double kx = A.Kh[a * N + a2], mx = A.Mh[a * N + a2];
          const double ky = A.Kh[b * N + b2], my = A.Mh[b * N + b2];
          const double kz = A.Kh[c * N + c2], mz = A.Mh[c * N + c2];
          const double coef = A.s[0] * kx * my * mz + A.s[1] * mx * ky * mz + A.s[2] * mx * my * kz;
          acc = fma(coef, to_d(un[((cz * P + c2) * nny + cy * P + b2) * nnx + cx * P + a2]), acc);
        }
        m += A.w[a] * A.w[b] * A.w[c];
      }
  const double y = reduce64(acc);
  if (lane == 0) {
    double fx = 0.0;
    if (I >= A.sbox_lo[0] && I < A.sbox_hi[0] && J >= A.sbox_lo[1] && J < A.sbox_hi[1] && K >= A.sbox_lo[2] &&
        K < A.sbox_hi[2]) {
      const int64_t bx = A.sbox_hi[0] - A.sbox_lo[0], by = A.sbox_hi[1] - A.sbox_lo[1];
      fx = A.src_dense[((K - A.sbox_lo[2]) * by + (J - A.sbox_lo[1])) * bx + (I - A.sbox_lo[0])];
    }
    const double ft = A.ft[A.step[0] + A.ft_offset];
    const double un_g = to_d(un[g]);
    S* uw = static_cast<S*>(A.uw);
    const S outS = S(node_update(A, ft, fx, y, m, un_g, to_d(uw[g])));
    uw[g] = outS;
    if (A.write_u) static_cast<S*>(A.uout)[g] = S(un_g + to_d(outS));
  }
}

// LDS of the explicit kernels (staged in FP64 whatever the storage type)
size_t smem_bytes_explicit(const ExplicitArgs& a) {
  const int N = a.p + 1, P = a.p;
  if (a.dim == 3 && a.mode == kModeKron) return 0;  // static LDS only
  if (a.dim == 2 && (a.mode == 1 || a.mode == 2)) return 0;  // register strips: static LDS only
  if (a.dim == 2) {
    const int NEmax = (a.tx + 1) * (a.ty + 1);
    const int W = (a.tx + 1) * P + 1, H = (a.ty + 1) * P + 1;
    return sizeof(double) * ((size_t)W * H + 2 * (size_t)NEmax * N * N) + NEmax;
  }
  const int NXmax = a.tx + 1, NYmax = a.ty + 1;
  const int PL = row_stride3d(NXmax * P + 1, N) * (NYmax * P + 1);
  const int NEmax = NXmax * NYmax;
  return sizeof(double) * ((size_t)N * PL + 2 * (size_t)NEmax * N * N * N + 2 * (size_t)PL) + 2 * NEmax;
}

template <typename T, int N>
hipError_t launch_explicit_n(const ExplicitArgs& a, hipStream_t s, bool prepare) {
  if constexpr (N <= kStripMaxN) {
    if (a.dim == 2 && (a.mode == 1 || a.mode == 2)) {
      if (prepare) return hipSuccess;
      const int waves = a.ntx * a.nty;
      if (a.mode == 2)
        hipLaunchKernelGGL((explicit2d_strip_kernel<N, T, true>), dim3((unsigned)waves), dim3(64), 0, s, a);
      else
        hipLaunchKernelGGL((explicit2d_strip_kernel<N, T, false>), dim3((unsigned)waves), dim3(64), 0, s, a);
      return hipGetLastError();
    }
  }
  if (a.dim == 3 && a.mode == kModeKron) {
    if (prepare) return hipSuccess;
    hipLaunchKernelGGL((explicit3d_kron_kernel<N - 1, T>), dim3((unsigned)(a.ntx * a.nty * a.nchunk)),
                       dim3(kKronThreads), 0, s, a);
    if (a.n_rest > 0)
      hipLaunchKernelGGL((explicit3d_rest_kernel<T>), dim3((unsigned)((a.n_rest + 3) / 4)), dim3(kThreads), 0, s, a);
    return hipGetLastError();
  }
  const size_t smem = smem_bytes_explicit(a);
  const int blocks = a.ntx * a.nty * a.nchunk;
  if (prepare) {
    if (a.dim != 2) {
      hipError_t e = allow_full_lds((const void*)explicit3d_kernel<N, T, kThreads>);
      if (e == hipSuccess) e = allow_full_lds((const void*)explicit3d_kernel<N, T, 2 * kThreads>);
      return e;
    }
    hipError_t e = allow_full_lds((const void*)explicit2d_kernel<N, T, kThreads>);
    if (e == hipSuccess) e = allow_full_lds((const void*)explicit2d_kernel<N, T, kThreads / 2>);
    return e;
  }
  if (a.dim == 2 && a.mode == 3)
    hipLaunchKernelGGL((explicit2d_kernel<N, T, kThreads / 2>), dim3(blocks), dim3(kThreads / 2), smem, s, a);
  else if (a.dim == 2)
    hipLaunchKernelGGL((explicit2d_kernel<N, T, kThreads>), dim3(blocks), dim3(kThreads), smem, s, a);
  else if (a.mode == 4)
    hipLaunchKernelGGL((explicit3d_kernel<N, T, 2 * kThreads>), dim3(blocks), dim3(2 * kThreads), smem, s, a);
  else
    hipLaunchKernelGGL((explicit3d_kernel<N, T, kThreads>), dim3(blocks), dim3(kThreads), smem, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_explicit_t(const ExplicitArgs& a, hipStream_t s, bool prepare) {
  switch (a.p + 1) {
    case 2: return launch_explicit_n<T, 2>(a, s, prepare);
    case 3: return launch_explicit_n<T, 3>(a, s, prepare);
    case 4: return launch_explicit_n<T, 4>(a, s, prepare);
    case 5: return launch_explicit_n<T, 5>(a, s, prepare);
    case 6: return launch_explicit_n<T, 6>(a, s, prepare);
    case 7: return launch_explicit_n<T, 7>(a, s, prepare);
    case 8: return launch_explicit_n<T, 8>(a, s, prepare);
  }
  return hipErrorInvalidValue;
}

template <typename T, int N>
hipError_t launch_explicit_batch_n(const BatchTable<ExplicitArgs>& t, int blocks, size_t smem, hipStream_t s,
                                   bool prepare) {
  if (prepare) return allow_full_lds((const void*)explicit2d_batch_kernel<N, T, kThreads>);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((explicit2d_batch_kernel<N, T, kThreads>), dim3(blocks), dim3(kThreads), smem, s, t);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_explicit_batch_t(const BatchTable<ExplicitArgs>& t, int p, int blocks, size_t smem, hipStream_t s,
                                   bool prepare) {
  switch (p + 1) {
    case 2: return launch_explicit_batch_n<T, 2>(t, blocks, smem, s, prepare);
    case 3: return launch_explicit_batch_n<T, 3>(t, blocks, smem, s, prepare);
    case 4: return launch_explicit_batch_n<T, 4>(t, blocks, smem, s, prepare);
    case 5: return launch_explicit_batch_n<T, 5>(t, blocks, smem, s, prepare);
    case 6: return launch_explicit_batch_n<T, 6>(t, blocks, smem, s, prepare);
    case 7: return launch_explicit_batch_n<T, 7>(t, blocks, smem, s, prepare);
    case 8: return launch_explicit_batch_n<T, 8>(t, blocks, smem, s, prepare);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_explicit_batch(const BatchTable<ExplicitArgs>& t, int p, int blocks, size_t smem, int fp,
                                 hipStream_t s) {
  return fp == 32 ? launch_explicit_batch_t<float>(t, p, blocks, smem, s, false)
                  : launch_explicit_batch_t<double>(t, p, blocks, smem, s, false);
}

hipError_t prepare_explicit_batch(int p, int fp) {
  const BatchTable<ExplicitArgs> t{};
  return fp == 32 ? launch_explicit_batch_t<float>(t, p, 0, 0, nullptr, true)
                  : launch_explicit_batch_t<double>(t, p, 0, 0, nullptr, true);
}


size_t explicit_smem_bytes(const ExplicitArgs& a, int fp) {
  (void)fp;
  return smem_bytes_explicit(a);
}

hipError_t launch_explicit(const ExplicitArgs& a, int fp, hipStream_t s) {
  return fp == 32 ? launch_explicit_t<float>(a, s, false) : launch_explicit_t<double>(a, s, false);
}

hipError_t prepare_explicit(const ExplicitArgs& a, int fp) {
  return fp == 32 ? launch_explicit_t<float>(a, nullptr, true) : launch_explicit_t<double>(a, nullptr, true);
}

}  // namespace imex
