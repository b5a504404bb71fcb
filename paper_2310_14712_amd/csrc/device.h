// Argument blocks of the device kernels and the host-side launchers
// (explicit.hip, implicit.hip, util.hip).  Plain structs of device pointers and sizes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace imex {

// Explicit part of one Newmark IMEX step on the uncut cells (the diagonal
// CDM step of the flowchart): for every d node
//   a = (f_t f_x - sum_{uncut e} K_e u_e) / M_ii
//   out = c1 u_n + c2 w + c3 dt^2 a          (written over w)
// FP64 (two-step form): (c1, c2, c3) = (2, -1, 1) with w = u_{n-1} for the CDM
// sum step and (1, -dt, 1/2) with w = v_0 for the start value u_{-1}.
// FP32 storage (increment form): w is the increment d_{n-1/2} = u_n - u_{n-1};
// (0, 1, 1) gives d_{n+1/2} and, with write_u, u_{n+1} = u_n + d_{n+1/2} into
// uout; (0, dt, -1/2) with w = v_0 gives the start increment d_{-1/2}.  The
// arithmetic is FP64 for both storage types: only the grid state is FP32.
// Per-instance argument tables of a batched launch (one launch of a kernel
// type over the instances of a batch): instance i owns workgroups
// [first[i], first[i + 1]) and runs with args[i].
template <typename X>
struct BatchTable {
  const X* args;
  const int32_t* first;
  int n;
};

constexpr int kStripCells = 63;  // cells owned by one wave of the 2D strip kernel (one more as halo)
constexpr int kStripMaxN = 6;    // the strip kernel holds a cell's nodes in registers: p <= 5
struct ExplicitArgs {
  int dim, p;
  int64_t ne[3], nn[3];
  int mode;                // 2D: 0 = LDS tiles; register strips (kStripCells cells wide, lz rows per wave)
                           // with 1 = per-lane loads, 2 = loads staged through LDS; 3 = LDS tiles on 128
                           // threads; 3D: 0 / 4 = cell-by-cell LDS tiles on 256 / 512 threads,
                           // 5 = tensor-product form
  int tx, ty, lz;          // tile (elements in x, y) and element layers per chunk
  int ntx, nty, nchunk;    // tiles per direction, chunks along the march direction
  const void* un;          // u_n (grid)
  void* uw;                // w in, out written over it (grid)
  void* uout;              // FP32: u_{n+1} (grid), written when write_u
  int write_u;
  const uint8_t* flags;    // per cell
  const double* ft;        // f_t table
  const int* step;         // device step counter; f_t index = *step + ft_offset
  int ft_offset;
  double c1, c2, c3, dt2;
  double s[3];             // stiffness term scalings (kappa * area / length)
  double mass_scale;       // rho * |J|
  int64_t sbox_lo[3], sbox_hi[3];  // node box of the point source, [lo, hi)
  const double* src_dense;         // f_x over that box (x fastest)
  double Kh[kMaxN * kMaxN], Mh[kMaxN * kMaxN], w[kMaxN];
  // 3D tensor-product form (mode 5): tiles of kKronCX x kKronCY cells
  const uint32_t* kron_mask;       // bit per grid node: d node whose adjacent cells are all uncut
  const int64_t* kron_rest;        // the other d nodes, summed cell by cell
  int64_t n_rest;
};

// 3D explicit kernel, tensor-product form: workgroup size and tile (cells in
// x and y) per order p, sized so that every pass has at most one task per
// thread and the LDS of the z and y passes stays below 48 KB
constexpr int kKronThreads = 512;
constexpr int kKronCX[kMaxN] = {0, 32, 16, 16, 12, 8, 6, 6};
constexpr int kKronCY[kMaxN] = {0, 14, 8, 8, 5, 5, 4, 3};
constexpr int kModeKron = 5;

// Predictor + right-hand side of the implicit solve (one row per c dof):
//   rhs_i = f_t(t_{n+1}) f_x,i - sum_j Kcd_ij u^d_{n+1,j} - sum_j Kcc_ij u^c_pred,j
struct RhsArgs {
  int64_t nc;
  const int64_t* rp_d;          // K^cd
  const int32_t* col_d;         // columns = grid ids
  const double* val_d;
  const int64_t* rp_c;          // K^cc
  const int32_t* col_c;         // columns = c indices
  const double* val_c;
  const void* ugrid;            // grid holding u^d_{n+1}
  const double *uc, *vc, *ac;   // c state at t_n
  const double* fxc;
  const double* ft;
  const int* step;              // f_t index = *step + 1
  double dt;
  double qp;                    // predictor coefficient (1/2 - beta) dt^2
  double* rhs;
  int lanes_per_row;            // 16 or 32 (four or two rows per wave; long 3D rows)
  double* pred;                 // u^c_pred per c dof, formed by a first pass and gathered by the
                                // rows (3D); null: formed per entry from u^c, v^c, a^c (2D, batches)
};

// One stored 64 x 64 block (I >= J) of a symmetric blocked part inverse with
// all that its workgroup needs, so that the block's loads wait on a single
// descriptor load.
struct SymBlock {
  int64_t boff;   // offset of the block in the stored values
  int64_t row0;   // first c row of the part
  int64_t prow;   // partial-sum slot (I, J): B x_J, one value per block row
  int64_t pcol;   // partial-sum slot (J, I): B^T x_I (written when I != J)
  int32_t n, I, J, pad;  // rows of the part, block row and column
};

// Chunk descriptors: the offsets a chunk's workgroup needs, resolved on the
// host, so that its loads wait on one descriptor load instead of a chunk
// list entry and then the part's or separator's metadata.
// A chunk of part rows for the correction x_p = w_p - Z_p x_S: 16 rows with
// Z_p row-major (wide form, ld = na) or 64 rows with Z_p column-major
// (ld = rows of the part).
struct CorrChunk {
  int64_t z;      // offset of Z_p entry (first row of the chunk, column 0)
  int64_t row;    // c index of the chunk's first row
  int64_t adj0;   // first separator row adjacent to the part
  int32_t na;     // columns of Z_p (adjacent separator rows)
  int32_t rows;   // rows in the chunk (fewer at the end of a part)
  int64_t ld;     // column-major Z_p: distance between adjacent columns (rows of the part)
};
// 16 rows of a dense part product: rows of A_pp^-1 (kind 0, into w) or
// columns of Z_p (kind 1, Z_p^T r_p into the coupling buffer).
struct DenseChunk {
  int64_t moff;   // offset of the chunk's first row in A_pp^-1 or Z_p values
  int64_t x0;     // c index of the part's first row (r_p)
  int64_t out0;   // output index of the chunk's first row (w or coupling buffer)
  int32_t n;      // row length (rows of the part)
  int32_t rows;   // rows in the chunk
  int32_t kind;
  int32_t pad;
};
// 16 rows of a separator system's dense inverse.
struct SepChunk {
  int64_t moff;   // offset of the chunk's first row of Sigma^-1
  int64_t row0;   // c index of the separator system's first row
  int32_t m;      // rows of the system
  int32_t first;  // the chunk's first row within the system
  int32_t rows;   // rows in the chunk
  int32_t pad;
};

// One workgroup's share of a supernode in the nested-dissection solve (see
// NdFactor): `rows` consecutive rows from `first` of the supernode's forward
// values (rows of L_ss^-1, then of C_s) or backward values (columns j of
// [L_ss^-1; C_s]), with the offsets the workgroup needs.
struct NdChunk {
  int64_t moff;   // offset of the supernode's forward (backward) values
  int64_t c0;     // first c index of the supernode
  int64_t woff;   // offset of W_s in the update buffer
  int64_t soff;   // offset of struct(s) in the struct list
  int64_t goff;   // first gather slot of the supernode
  int32_t m, k;   // rows of the supernode and of struct(s)
  int32_t first, rows;
};

// Implicit solve S a^c_{n+1} = rhs with the dissected Cholesky factor (see
// DissectedFactor) or the nested-dissection factor (NdFactor), then the
// trapezoidal correction of the c dofs.
struct SolveArgs {
  const ChainMeta* parts;       // all parts
  const ChainMeta* schur;       // one separator system per component
  const double* vals;           // chain values
  const int32_t* ints;          // chain metadata
  const double* zvals;          // Z_p
  const double* schur_inv;      // Sigma^-1 per component (row-major)
  const int64_t* schur_chunks;  // (component, first row) per 16-row chunk
  const int64_t* schur_chain;   // components whose separator system is a chain
  const int64_t* part_chunks;   // (part, first row) per 64-row chunk
  const double* pinv;           // dense A_pp^-1 (dense form)
  const int64_t* dense_chunks;  // (kind, part, first) per 16-row chunk (dense form)
  int dense;
  const int64_t* cp_rowptr;     // per part: offset of its row pointers in cp_ptr
  const int32_t *cp_ptr, *cp_col;  // A_Sp of every part (local columns)
  const double* cp_val;
  double* cbuf;                 // A_Sp w_p, one slot per (part, adjacent separator row)
  const int64_t* sep_src;       // per c row: the (<= 2) slots summed into a separator row
  const double* rhs;            // right-hand side (c order)
  double* w;                    // part solutions w_p, then the separator solution x_S
  double *uc, *vc, *ac;         // c state, updated in place
  const int64_t* c_nodes;
  void* ugrid;                  // grid that receives u^c_{n+1}
  int* step;                    // incremented once per step
  int advance_step;
  double dt;
  double qp, qc;                // (1/2 - beta) dt^2 and beta dt^2 (predictor, corrector)
  int64_t smem_part, smem_schur;   // dynamic LDS bytes of the two chain kernels
  int64_t smem_sep;                // dynamic LDS bytes of the dense separator kernel (largest system)
  int dense_wide;                  // dense parts above 1024 rows: symmetric blocked A_pp^-1, the
                                   // coupling from the sparse A_Sp, the wide separator stage
  const SymBlock* sym_blocks;      // every stored 64 x 64 block (I >= J)
  const int64_t* sym_poff;         // per part: offset of its nbk x nbk x 64 partial sums
  double* sym_partial;             // partial sums of the symmetric products
  int64_t n_sym_blocks;
  double* rs;                      // r_S - sum_p A_Sp w_p of every separator row (wide form)
  const CorrChunk* corr_chunks;    // 16-row chunks of the parts (wide form; Z_p row-major)
  const CorrChunk* part_corr;      // 64-row chunks of the parts (plain form; Z_p column-major)
  const DenseChunk* pd_chunks;     // dense part products (plain form)
  const SepChunk* sep_chunks;      // separator products (plain form)
  int64_t n_corr_chunks;
  // nested-dissection form
  int nd;
  const double *nd_fwd, *nd_bwd;   // forward and backward values of every supernode
  const NdChunk *nd_fchunks, *nd_bchunks;  // chunks of all levels, level by level
  const NdChunk* nd_fcchunks;      // forward chunks of small supernodes (thread per output), level by level
  const int32_t* nd_st;            // struct lists
  const int64_t* nd_gptr;          // gather slots
  const int32_t* nd_gsrc;
  double* nd_W;                    // update buffer (sum over supernodes of k)
  int64_t nd_smem_f, nd_smem_b;    // dynamic LDS bytes of the two kernels
};

// Local time-stepping leap-frog on the fine rows F (LtsRows): per coarse
// step from (u_{n-1}, u_n) on the grid,
//   g = M^-1 (K (I - P) u_n - f_t(t_n) f_x)                 (lts_pre)
//   q_1 = u_n - tau^2/2 (g + M^-1 K P u_n)                   (substep 0)
//   q_{k+1} = 2 q_k - q_{k-1} - tau^2 (g + M^-1 K P q_k)    (substep k)
//   u_{n+1} = 2 q_m - u_{n-1} on the F rows                  (last substep)
// with P the projection onto the c dofs and tau = dt / m; the explicit
// kernel gives the other d rows (where K P = 0 the recurrence is the
// central difference step).  FP64 grid state.
struct LtsArgs {
  int64_t nf, nc;                                  // F rows, of which the first nc are c dofs
  const int64_t* rp_o; const int32_t* col_o; const double* val_o;  // K over F rows, other columns
  const int64_t* rp_f; const int32_t* col_f; const double* val_f;  // K over F rows, c columns (c index)
  const double* minv;                              // 1 / lumped mass per F row
  const double* fx;                                // f_x per F row
  const int64_t* node;                             // grid id per F row
  const double* ft;
  int* step;
  const double* un;                                // grid u_n
  double* uw;                                      // grid u_{n-1}, receives u_{n+1}
  double* g;                                       // frozen coarse term
  double* q[3];                                    // substep iterates (rotating)
  double* uprev;                                   // u_{n-1} on F rows
  double* uc;                                      // u^c of the c state (first nc rows)
  double tau2;
  int m;
};
hipError_t launch_lts_pre(const LtsArgs& a, hipStream_t s);   // before the explicit kernel
hipError_t launch_lts_step(const LtsArgs& a, hipStream_t s);  // the m substeps, after it

hipError_t launch_explicit(const ExplicitArgs& a, int fp, hipStream_t s);
// one launch of the 2D LDS-tile explicit kernel (256 threads) over the
// instances of a batch of order p; smem = the largest instance's LDS
hipError_t launch_explicit_batch(const BatchTable<ExplicitArgs>& t, int p, int blocks, size_t smem, int fp,
                                 hipStream_t s);
hipError_t prepare_explicit_batch(int p, int fp);
// one launch each of the rhs kernel, and of the dense part, separator and
// correction stages of the dissected solve, over the instances of a batch
hipError_t launch_rhs_batch(const BatchTable<RhsArgs>& t, int blocks, int fp, int lanes, hipStream_t s);
hipError_t launch_solve_batch(const BatchTable<SolveArgs>& dense, int dense_blocks, const BatchTable<SolveArgs>& sep,
                              int sep_blocks, size_t sep_smem, const BatchTable<SolveArgs>& corr, int corr_blocks,
                              int fp, hipStream_t s);
hipError_t prepare_solve_batch(int fp);
// raise the dynamic LDS limit of the explicit kernel (once, outside graph capture)
hipError_t prepare_explicit(const ExplicitArgs& a, int fp);
size_t explicit_smem_bytes(const ExplicitArgs& a, int fp);
hipError_t launch_rhs(const RhsArgs& a, int fp, hipStream_t s);
hipError_t launch_solve(const SolveArgs& a, int64_t n_parts, int64_t n_schur_chunks, int64_t n_schur_chain,
                        int64_t n_part_chunks, int64_t n_dense_chunks, int fp, hipStream_t s);
// the nested-dissection solve: forward levels 0..H, then backward levels
// H..0 with the corrector; level h's chunks are [flev[h], flev[h + 1]) and
// [blev[h], blev[h + 1])
// per level of the nested-dissection solve: chunk ranges of the three
// kernels, and the values per lane and row in flight (1, 2, 4 or 8) of the
// row kernels, from the level's longest row
struct NdLevels {
  const int64_t *flev, *fclev, *blev;  // n_levels + 1 entries each
  const int8_t *fper, *bper;
  int n_levels;
};
hipError_t launch_nd_solve(const SolveArgs& a, const NdLevels& levels, int fp, hipStream_t s);
// the largest supernode that may take the forward pass with one thread per
// output row (reading the backward values); larger ones take one wave per row
constexpr int kNdColsMaxM = 128;
// raise the dynamic LDS limit of the chain kernels (once, outside graph capture)
hipError_t prepare_solve(const SolveArgs& a, int fp);
// trapezoidal corrector of all c rows from a^c_{n+1} = an (and the step counter)
hipError_t launch_correct_all(const SolveArgs& a, const double* an, int64_t nc, int fp, hipStream_t s);
hipError_t launch_set_int(int* p, int v, hipStream_t s);
hipError_t launch_check_finite(const void* x, int64_t n, int fp, int* flag, hipStream_t s);
hipError_t launch_add_int(int* p, int v, hipStream_t s);
// grid[c_nodes[i]] = src[i] (converted to the grid type)
hipError_t launch_scatter_c(void* grid, const int64_t* c_nodes, const double* src, int64_t nc,
                            int fp, hipStream_t s);
// dst[i] = (double) grid[i]
hipError_t launch_grid_to_f64(const void* grid, double* dst, int64_t n, int fp, hipStream_t s);
hipError_t launch_f64_to_grid(const double* src, void* grid, int64_t n, int fp, hipStream_t s);
// d[i] = a[i] - b[i] (FP32 grids)
hipError_t launch_sub_f32(float* d, const float* a, const float* b, int64_t n, hipStream_t s);
// out[r] = sum_t w[r nb + t] grid[ids[r nb + t]] (receiver sampling)
hipError_t launch_sample(const void* grid, const int64_t* ids, const double* w, int nb, int64_t n, double* out,
                         int fp, hipStream_t s);

// out[r] = the field at physical point r (pts: n x dim), basis evaluated on
// the device (sampling without temporary device allocations)
struct SamplePointsArgs {
  int dim, n;              // dimension, nodes per cell edge (p + 1)
  int64_t ne[3], nn[3];    // cells and nodes per direction
  double h[3];             // cell sizes
  double x[kMaxN];         // GLL nodes on [-1, 1]
};
hipError_t launch_sample_points(const void* grid, const SamplePointsArgs& a, const double* pts, int64_t n,
                                double* out, int fp, hipStream_t s);

}  // namespace imex
