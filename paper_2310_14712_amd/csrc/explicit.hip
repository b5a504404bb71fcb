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

namespace imex {

namespace {

using namespace dev;

// row `row` of a 1D operator (n x n, row-major) times v[0..N)
template <int N>
__device__ inline double op_row(const double* C, int row, const double* v) {
  double acc = 0.0;
#pragma unroll
  for (int d = 0; d < N; ++d) acc += C[row * N + d] * v[d];
  return acc;
}

// Lane exchanges through DPP (data-parallel primitives) on both halves of a
// double: quad_perm [1,0,3,2] (xor 1), quad_perm [2,3,0,1] (xor 2), mirror

// ---------------------------------------------------------------------------
// 2D explicit step: one tile of tx x ty cells per workgroup
// ---------------------------------------------------------------------------
// The workgroup stages the tile's nodes plus one cell of halo on the low
// side in x and y, applies the operator to all (tx+1)(ty+1) cells, and
// assembles the owned nodes from their (up to four) adjacent cells.  The
// previous values u_{n-1} of the owned nodes are fetched together with the
// tile, so the kernel makes a single round trip to memory before writing.
constexpr int kOwnMax = 8;  // owned nodes per thread

template <int N, typename S>
__global__ __launch_bounds__(kThreads) void explicit2d_kernel(const ExplicitArgs A) {
  using T = double;  // LDS and arithmetic
  constexpr int P = N - 1;
  const int tid = threadIdx.x;
  const int tix = blockIdx.x % A.ntx, tiy = blockIdx.x / A.ntx;
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
  // owned nodes of this thread and their previous values (issued first)
  T wprev[kOwnMax];
#pragma unroll
  for (int k = 0; k < kOwnMax; ++k) {
    const int o = tid + k * kThreads;
    wprev[k] = T(0);
    if (o < OX * OY) {
      const int j = P + o / OX, i = P + o % OX;
      wprev[k] = uw[(J0 + j) * nnx + I0 + i];
    }
  }
  for (int base = 0; base < WY * WX; base += kThreads * 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + tid + u * kThreads;
      const int j = idx / WX, i = idx - j * WX;
      const int64_t I = I0 + i, J = J0 + j;
      v[u] = (idx < WY * WX && I >= 0 && J >= 0) ? un[J * nnx + I] : T(0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + tid + u * kThreads;
      if (idx < WY * WX) U[(idx / WX) * WXmax + idx % WX] = v[u];
    }
  }
  for (int le = tid; le < NX * NY; le += kThreads) {
    const int lx = le % NX, ly = le / NX;
    const int64_t ex = ex0 - 1 + lx, ey = ey0 - 1 + ly;
    fl[le] = (ex >= 0 && ey >= 0) ? A.flags[ey * nex + ex] : uint8_t(kEmpty);
  }
  const double ft = A.ft[A.step[0] + A.ft_offset];
  __syncthreads();
  // y pencils of every cell: T1 = U Mh^T, T2 = U Kh^T  (per column a)
  for (int idx = tid; idx < NX * NY * N; idx += kThreads) {
    const int le = idx / N, a = idx - le * N;
    const int lx = le % NX, ly = le / NX;
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
  for (int idx = tid; idx < NX * NY * N; idx += kThreads) {
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
      E1[(le * N + a) * N + b] = on ? sx * y1 + sy * y2 : T(0);
    }
  }
  __syncthreads();
  // owned nodes: assemble from the adjacent cells, lumped mass, CDM update
#pragma unroll
  for (int k = 0; k < kOwnMax; ++k) {
    const int o = tid + k * kThreads;
    if (o >= OX * OY) break;
    const int j = P + o / OX, i = P + o % OX;
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
          m += A.w[axs[p2]] * A.w[ays[q]];
          has_uncut = true;
        }
        has_cut |= (f == kCut);
      }
    if (!has_uncut || has_cut) continue;  // not a d node
    const int64_t I = I0 + i, J = J0 + j;
    double fx = 0.0;
    if (I >= A.sbox_lo[0] && I < A.sbox_hi[0] && J >= A.sbox_lo[1] && J < A.sbox_hi[1])
      fx = A.src_dense[(J - A.sbox_lo[1]) * (A.sbox_hi[0] - A.sbox_lo[0]) + (I - A.sbox_lo[0])];
    const double acc = (ft * fx - to_d(y)) / (A.mass_scale * m);
    const double un_g = to_d(U[j * WXmax + i]);
    const double out = A.c1 * un_g + A.c2 * to_d(wprev[k]) + A.c3 * A.dt2 * acc;
    const S outS = S(out);
    uw[J * nnx + I] = outS;
    if (A.write_u) static_cast<S*>(A.uout)[J * nnx + I] = S(un_g + to_d(outS));
  }
}

// ---------------------------------------------------------------------------
// 3D explicit step (march along z)
// ---------------------------------------------------------------------------
template <int N, typename S>
__global__ __launch_bounds__(kThreads) void explicit3d_kernel(const ExplicitArgs A) {
  using T = double;  // LDS and arithmetic
  constexpr int P = N - 1;
  constexpr int N2 = N * N, N3 = N * N * N;
  const int tid = threadIdx.x;
  const int tiles = A.ntx * A.nty;
  const int tile = blockIdx.x % tiles;
  const int chunk = blockIdx.x / tiles;
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
  const int WXmax = NXmax * P + 1, WYmax = NYmax * P + 1;
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
  T* E1 = U + N * PL;                         // [NEmax][N3], index (c, b, a) a fastest
  T* E2 = E1 + NEmax * N3;
  T* carry = E2 + NEmax * N3;                 // [2][PL]
  uint8_t* flc = reinterpret_cast<uint8_t*>(carry + 2 * PL);  // [NEmax]
  uint8_t* flp = flc + NEmax;

  const S* un = static_cast<const S*>(A.un);
  S* uw = static_cast<S*>(A.uw);
  const double ft = A.ft[A.step[0] + A.ft_offset];
  const double sx = A.s[0], sy = A.s[1], sz = A.s[2];

  for (int i = tid; i < 2 * PL; i += kThreads) carry[i] = T(0);
  int cur = 0;
  const int ez_start = ez_begin > 0 ? ez_begin - 1 : ez_begin;
  for (int ez = ez_start; ez < ez_end; ++ez) {
    const bool out_layer = ez >= ez_begin;
    const bool top = (ez == nez - 1);
    for (int idx = tid; idx < N * WY * WX; idx += kThreads) {
      const int c = idx / (WY * WX);
      const int rem = idx - c * WY * WX;
      const int j = rem / WX, i = rem - j * WX;
      const int64_t I = I0 + i, J = J0 + j, K = (int64_t)ez * P + c;
      U[c * PL + j * WXmax + i] =
          (I >= 0 && I < nnx && J >= 0 && J < nny) ? un[(K * nny + J) * nnx + I] : T(0);
    }
    for (int le = tid; le < NE; le += kThreads) {
      const int lx = le % NX, ly = le / NX;
      const int64_t ex = ex0 - 1 + lx, ey = ey0 - 1 + ly;
      const bool ok = ex >= 0 && ex < nex && ey >= 0 && ey < ney;
      flc[le] = ok ? A.flags[((int64_t)ez * ney + ey) * nex + ex] : uint8_t(kEmpty);
      flp[le] = (ok && ez > 0) ? A.flags[((int64_t)(ez - 1) * ney + ey) * nex + ex] : uint8_t(kEmpty);
    }
    __syncthreads();
    // z pencils (a, b): A = Mh_z U, B = Kh_z U
    for (int idx = tid; idx < NE * N2; idx += kThreads) {
      const int le = idx / N2, ab = idx - le * N2;
      const int b = ab / N, a = ab - b * N;
      const int lx = le % NX, ly = le / NX;
      const int base = (ly * P + b) * WXmax + lx * P + a;
      T u[N];
#pragma unroll
      for (int c = 0; c < N; ++c) u[c] = U[c * PL + base];
      T* e1 = E1 + le * N3 + b * N + a;
      T* e2 = E2 + le * N3 + b * N + a;
#pragma unroll
      for (int c = 0; c < N; ++c) {
        e1[c * N2] = op_row<N>(A.Mh, c, u);
        e2[c * N2] = op_row<N>(A.Kh, c, u);
      }
    }
    __syncthreads();
    // y pencils (a, c): C = Mh_y A, G = s_y Kh_y A + s_z Mh_y B
    for (int idx = tid; idx < NE * N2; idx += kThreads) {
      const int le = idx / N2, ac = idx - le * N2;
      const int c = ac / N, a = ac - c * N;
      T* e1 = E1 + le * N3 + c * N2 + a;
      T* e2 = E2 + le * N3 + c * N2 + a;
      T ta[N], tb[N];
#pragma unroll
      for (int e = 0; e < N; ++e) {
        ta[e] = e1[e * N];
        tb[e] = e2[e * N];
      }
#pragma unroll
      for (int b = 0; b < N; ++b) {
        const T cc = op_row<N>(A.Mh, b, ta);
        const T dd = op_row<N>(A.Kh, b, ta);
        const T ee = op_row<N>(A.Mh, b, tb);
        e1[b * N] = cc;
        e2[b * N] = sy * dd + sz * ee;
      }
    }
    __syncthreads();
    // x pencils (b, c): Y = s_x Kh_x C + Mh_x G, zero for non-uncut cells
    for (int idx = tid; idx < NE * N2; idx += kThreads) {
      const int le = idx / N2, bc = idx - le * N2;
      const bool on = flc[le] == kUncut;
      T* e1 = E1 + le * N3 + bc * N;
      const T* e2 = E2 + le * N3 + bc * N;
      T tc[N], tg[N];
#pragma unroll
      for (int f = 0; f < N; ++f) {
        tc[f] = e1[f];
        tg[f] = e2[f];
      }
#pragma unroll
      for (int a = 0; a < N; ++a) {
        const T y1 = op_row<N>(A.Kh, a, tc);
        const T y2 = op_row<N>(A.Mh, a, tg);
        e1[a] = on ? sx * y1 + y2 : T(0);
      }
    }
    __syncthreads();
    T* cin = carry + cur * PL;
    T* cout = carry + (1 - cur) * PL;
    const int nplanes = top ? N : P;
    if (out_layer) {
      for (int idx = tid; idx < nplanes * OY * OX; idx += kThreads) {
        const int c = idx / (OY * OX);
        const int rem = idx - c * OY * OX;
        const int j = oy_lo + rem / OX, i = ox_lo + rem % OX;
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
        for (int sy_ = 0; sy_ < nys; ++sy_)
          for (int sx_ = 0; sx_ < nxs; ++sx_) {
            const int le = lys[sy_] * NX + lxs[sx_];
            y += E1[le * N3 + c * N2 + ays[sy_] * N + axs[sx_]];
            const uint8_t f = flc[le];
            if (f == kUncut) { m += A.w[axs[sx_]] * A.w[ays[sy_]] * A.w[c]; has_uncut = true; }
            has_cut |= (f == kCut);
            if (c == 0) {
              const uint8_t fp = flp[le];
              if (fp == kUncut) { m += A.w[axs[sx_]] * A.w[ays[sy_]] * A.w[P]; has_uncut = true; }
              has_cut |= (fp == kCut);
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
    for (int idx = tid; idx < WY * WX; idx += kThreads) {
      const int j = idx / WX, i = idx - j * WX;
      int lxs[2], axs[2], nxs = 0, lys[2], ays[2], nys = 0;
      if (i % P == 0) {
        if (i / P - 1 >= 0) { lxs[nxs] = i / P - 1; axs[nxs++] = P; }
        if (i / P < NX) { lxs[nxs] = i / P; axs[nxs++] = 0; }
      } else {
        lxs[nxs] = i / P; axs[nxs++] = i % P;
      }
      if (j % P == 0) {
        if (j / P - 1 >= 0) { lys[nys] = j / P - 1; ays[nys++] = P; }
        if (j / P < NY) { lys[nys] = j / P; ays[nys++] = 0; }
      } else {
        lys[nys] = j / P; ays[nys++] = j % P;
      }
      T y = T(0);
      for (int sy_ = 0; sy_ < nys; ++sy_)
        for (int sx_ = 0; sx_ < nxs; ++sx_)
          y += E1[(lys[sy_] * NX + lxs[sx_]) * N3 + P * N2 + ays[sy_] * N + axs[sx_]];
      cout[j * WXmax + i] = y;
    }
    cur = 1 - cur;
    __syncthreads();
  }
}
// LDS of the explicit kernels (staged in FP64 whatever the storage type)
size_t smem_bytes_explicit(const ExplicitArgs& a) {
  const int N = a.p + 1, P = a.p;
  if (a.dim == 2) {
    const int NEmax = (a.tx + 1) * (a.ty + 1);
    const int W = (a.tx + 1) * P + 1, H = (a.ty + 1) * P + 1;
    return sizeof(double) * ((size_t)W * H + 2 * (size_t)NEmax * N * N) + NEmax;
  }
  const int NXmax = a.tx + 1, NYmax = a.ty + 1;
  const int PL = (NXmax * P + 1) * (NYmax * P + 1);
  const int NEmax = NXmax * NYmax;
  return sizeof(double) * ((size_t)N * PL + 2 * (size_t)NEmax * N * N * N + 2 * (size_t)PL) + 2 * NEmax;
}

template <typename T, int N>
hipError_t launch_explicit_n(const ExplicitArgs& a, hipStream_t s, bool prepare) {
  const size_t smem = smem_bytes_explicit(a);
  const int blocks = a.ntx * a.nty * a.nchunk;
  const void* k = a.dim == 2 ? (const void*)explicit2d_kernel<N, T> : (const void*)explicit3d_kernel<N, T>;
  if (prepare) return allow_full_lds(k);
  if (a.dim == 2)
    hipLaunchKernelGGL((explicit2d_kernel<N, T>), dim3(blocks), dim3(kThreads), smem, s, a);
  else
    hipLaunchKernelGGL((explicit3d_kernel<N, T>), dim3(blocks), dim3(kThreads), smem, s, a);
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

}  // namespace


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
