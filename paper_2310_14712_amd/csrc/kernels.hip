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

#include "device.h"

namespace imex {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxSep = 4096;  // separator rows of one component (checked on the host)

template <typename T>
__device__ inline double to_d(T v) { return (double)v; }

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
// within 8 lanes, mirror within 16 lanes.
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

// sums over aligned groups of 4 / 8 / 16 lanes (every lane gets the sum)
__device__ inline double reduce4(double v) {
  v += dpp_move<kDppXor1>(v);
  v += dpp_move<kDppXor2>(v);
  return v;
}
__device__ inline double reduce8(double v) {
  v = reduce4(v);
  v += dpp_move<kDppHalfMirror>(v);
  return v;
}
__device__ inline double reduce16(double v) {
  v = reduce8(v);
  v += dpp_move<kDppMirror>(v);
  return v;
}
__device__ inline double reduce64(double v) {
  v = reduce16(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// Partial dot product of a row M[0..n) with x[0..n) over LANES lanes (lane
// `sub` takes t = sub, sub + LANES, ...): the first LANES * PER entries are
// loaded at once, the rest (if any) in further batches of the same size.
template <int LANES, int PER, typename XP>
__device__ inline double row_dot(const double* M, XP x, int n, int sub) {
  double acc = 0.0;
  for (int base = 0; base < n; base += LANES * PER) {
    double mv[PER], xv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int t = base + sub + u * LANES;
      mv[u] = t < n ? M[t] : 0.0;
      xv[u] = t < n ? x[t] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) acc += mv[u] * xv[u];
  }
  return acc;
}


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

// ---------------------------------------------------------------------------
// implicit part
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void rhs_kernel(const RhsArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (row >= A.nc) return;
  const T* ug = static_cast<const T*>(A.ugrid);
  const double dt = A.dt, q = 0.25 * dt * dt;
  double acc = 0.0;
  for (int64_t k = A.rp_d[row] + lane; k < A.rp_d[row + 1]; k += 64)
    acc += A.val_d[k] * to_d(ug[A.col_d[k]]);
  for (int64_t k = A.rp_c[row] + lane; k < A.rp_c[row + 1]; k += 64) {
    const int64_t j = A.col_c[k];
    acc += A.val_c[k] * (A.uc[j] + dt * A.vc[j] + q * A.ac[j]);
  }
  acc = reduce16(acc);
  acc += __shfl_xor(acc, 16, 64);
  acc += __shfl_xor(acc, 32, 64);
  if (lane == 0) A.rhs[row] = A.ft[A.step[0] + 1] * A.fxc[row] - acc;
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

template <typename T>
__device__ inline void correct_row(const SolveArgs& A, int64_t i, double an) {
  const double dt = A.dt, q4 = 0.25 * dt * dt;
  const double a0 = A.ac[i], v0 = A.vc[i], u0 = A.uc[i];
  const double up = u0 + dt * v0 + q4 * a0;
  const double vp = v0 + 0.5 * dt * a0;
  const double un = up + q4 * an;
  A.uc[i] = un;
  A.vc[i] = vp + 0.5 * dt * an;
  A.ac[i] = an;
  static_cast<T*>(A.ugrid)[A.c_nodes[i]] = T(un);
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
// four consecutive rows of one chunk of 16.
__global__ __launch_bounds__(kThreads) void part_dense_kernel(const SolveArgs A) {
  const int64_t chunk = blockIdx.x >> 2;
  const int64_t kind = A.dense_chunks[3 * chunk], part = A.dense_chunks[3 * chunk + 1];
  const int64_t first = A.dense_chunks[3 * chunk + 2];
  const ChainMeta cm = A.parts[part];
  const int n = cm.nrows;
  const int row = (int)first + (int)(blockIdx.x & 3) * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int nout = kind == 0 ? n : cm.nadj;
  const double* M = kind == 0 ? A.pinv + cm.doff + (int64_t)row * n : A.zvals + cm.zoff + (int64_t)row * n;
  double acc = 0.0;
  if (row < nout && row < first + 16) acc = row_dot<64, 16>(M, A.rhs + cm.row0, n, lane);
  acc = reduce64(acc);
  if (lane == 0 && row < nout && row < first + 16) {
    if (kind == 0) A.w[cm.row0 + row] = acc;
    else A.cbuf[cm.coff + row] = acc;
  }
}

// x_S = Sigma^-1 (r_S - sum_p A_Sp w_p): one wave per row of one component's
// Sigma^-1 (four rows per workgroup); corrects those separator rows.
template <typename T>
__global__ __launch_bounds__(kThreads) void schur_kernel(const SolveArgs A) {
  __shared__ double rs[kMaxSep];
  const int64_t chunk = blockIdx.x >> 2;
  const int64_t comp = A.schur_chunks[2 * chunk], r0 = A.schur_chunks[2 * chunk + 1];
  const ChainMeta cm = A.schur[comp];
  const int m = cm.nrows;
  for (int s = threadIdx.x; s < m; s += kThreads) {
    const int64_t i = cm.row0 + s;
    const int64_t s0 = A.sep_src[2 * i], s1 = A.sep_src[2 * i + 1];
    const double c0 = s0 >= 0 ? A.cbuf[s0] : 0.0, c1 = s1 >= 0 ? A.cbuf[s1] : 0.0;
    rs[s] = A.rhs[i] - c0 - c1;
  }
  __syncthreads();
  const int row = (int)r0 + (int)(blockIdx.x & 3) * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  const bool ok = row < m && row < r0 + 16;
  double acc = 0.0;
  if (ok) acc = row_dot<64, 8>(A.schur_inv + cm.voff + (int64_t)row * m, (const double*)rs, m, lane);
  acc = reduce64(acc);
  if (lane == 0 && ok) {
    A.w[cm.row0 + row] = acc;
    correct_row<T>(A, cm.row0 + row, acc);
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

// x_p = w_p - Z_p x_S(adjacent separators): 16 lanes per row, 16 rows per
// workgroup (four workgroups per 64-row chunk); corrects those part rows.
template <typename T>
__global__ __launch_bounds__(kThreads) void part_correct_kernel(const SolveArgs A) {
  const int64_t chunk = blockIdx.x >> 2;
  const int64_t part = A.part_chunks[2 * chunk], r0 = A.part_chunks[2 * chunk + 1];
  const ChainMeta cm = A.parts[part];
  const int i = (int)r0 + (int)(blockIdx.x & 3) * 16 + (threadIdx.x >> 4), sub = threadIdx.x & 15;
  const bool ok = i < cm.nrows && i < r0 + 64;
  double x = 0.0;
  if (ok && cm.nadj > 0) {
    // Z_p is column-major: row i of Z_p is strided by nrows
    const double* Zi = A.zvals + cm.zoff + i;
    const double* xs = A.w + cm.adj0;
    for (int base = 0; base < cm.nadj; base += 16 * 8) {
      double zv[8], xv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = base + sub + 16 * u;
        zv[u] = k < cm.nadj ? Zi[(int64_t)k * cm.nrows] : 0.0;
        xv[u] = k < cm.nadj ? xs[k] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) x += zv[u] * xv[u];
    }
  }
  x = reduce16(x);
  if (sub == 0 && ok) correct_row<T>(A, cm.row0 + i, A.w[cm.row0 + i] - x);
  if (A.advance_step && blockIdx.x == 0 && threadIdx.x == 0) A.step[0] = A.step[0] + 1;
}

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

__global__ void sub_f32_kernel(float* d, const float* a, const float* b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = a[i] - b[i];
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
  if (prepare)
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
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

inline dim3 grid1d(int64_t n, int t) { return dim3((unsigned)((n + t - 1) / t)); }

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

hipError_t launch_rhs(const RhsArgs& a, int fp, hipStream_t s) {
  if (a.nc == 0) return hipSuccess;
  const dim3 g = grid1d(a.nc, kThreads / 64);
  if (fp == 32) hipLaunchKernelGGL(rhs_kernel<float>, g, dim3(kThreads), 0, s, a);
  else hipLaunchKernelGGL(rhs_kernel<double>, g, dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs& a, int64_t n_parts, int64_t n_schur_chunks, int64_t n_schur_chain,
                        int64_t n_part_chunks, int64_t n_dense_chunks, int fp, hipStream_t s) {
  if (n_parts == 0) return hipSuccess;
  if (a.dense)
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
  if (fp == 32) {
    if (n_schur_chunks > 0)
      hipLaunchKernelGGL(schur_kernel<float>, dim3((unsigned)(4 * n_schur_chunks)), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(part_correct_kernel<float>, dim3((unsigned)(4 * n_part_chunks)), dim3(kThreads), 0, s, a);
  } else {
    if (n_schur_chunks > 0)
      hipLaunchKernelGGL(schur_kernel<double>, dim3((unsigned)(4 * n_schur_chunks)), dim3(kThreads), 0, s, a);
    hipLaunchKernelGGL(part_correct_kernel<double>, dim3((unsigned)(4 * n_part_chunks)), dim3(kThreads), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t prepare_solve(const SolveArgs& a, int fp) {
  hipError_t e = hipFuncSetAttribute((const void*)part_solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)std::max<int64_t>(a.smem_part, 1));
  if (e != hipSuccess) return e;
  const void* k = fp == 32 ? (const void*)schur_chain_kernel<float> : (const void*)schur_chain_kernel<double>;
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)std::max<int64_t>(a.smem_schur, 1));
}

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}
hipError_t launch_add_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(add_int_kernel, dim3(1), dim3(64), 0, s, p, v);
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

}  // namespace imex
