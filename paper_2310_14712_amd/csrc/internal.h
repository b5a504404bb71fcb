// Internal declarations shared by the host setup (setup.cpp, basis.cpp),
// the C ABI (capi.cpp) and the kernel launchers (explicit.hip, implicit.hip, util.hip).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace imex {

constexpr int kMaxP = 7;
constexpr int kMaxN = kMaxP + 1;
constexpr int kBlk = 32;  // row block of the blocked triangular solves

enum CellFlag : uint8_t { kEmpty = 0, kCut = 1, kUncut = 2 };
enum NodeKind : uint8_t { kInactive = 0, kD = 1, kC = 2 };

// ---- 1D reference operators on [-1, 1] (basis.cpp) ----------------------
struct Ref1D {
  int p = 0, n = 0;
  std::vector<double> x, w;     // GLL nodes / weights
  std::vector<double> Mh, Kh;   // consistent mass / stiffness, n x n row-major
};
void gll_rule(int p, std::vector<double>& x, std::vector<double>& w);
void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w);
// values and derivatives of the n Lagrange polynomials on `nodes` at xi
void lagrange_eval(const std::vector<double>& nodes, double xi, double* val, double* der);
Ref1D make_ref1d(int p);

// ---- geometry ------------------------------------------------------------
struct Geometry {
  int dim = 2;
  std::vector<double> cx;   // centres [n * 3]
  std::vector<double> r;    // radii
  bool fictitious(const double* x) const;
  // returns 0: box is entirely physical, 1: crossed by some sphere,
  // 2: contained in some ball (entirely fictitious)
  int box_state(const double* lo, const double* hi) const;
  bool crossed(const double* lo, const double* hi) const;
};

// sparse matrix in CSR with 64-bit indices
struct Csr {
  int64_t nrows = 0;
  std::vector<int64_t> ptr, col;
  std::vector<double> val;
};

// One connected component of the implicit block after RCM ordering, with
// its envelope Cholesky factor (row i stores L[i][first[i] .. i]).
struct Component {
  int64_t begin = 0, size = 0;        // range in c order
  std::vector<int64_t> first;         // first stored column of each row (local)
  std::vector<int64_t> rowoff;        // offset of row i in `L`
  std::vector<double> L;
};

// ---- dissected factor for the device (setup.cpp) ---------------------------
// Each connected component of the implicit block is split along level sets of
// a breadth-first search into "parts" separated by single levels
// ("separators"); the rows are ordered [part 1, ..., part P, separators].
// Because graph edges only join adjacent levels, the parts are independent
// once the separator values are known:
//   w_p  = A_pp^-1 r_p                                   (per part)
//   x_S  = Sigma^-1 (r_S - sum_p A_Sp w_p),  Sigma = A_SS - sum_p A_Sp A_pp^-1 A_pS
//   x_p  = w_p - Z_p x_S,  Z_p = A_pp^-1 A_pS            (per part)
// which is the exact Cholesky solve of S in that order.  Every A_pp is
// factorised by envelope Cholesky and stored as a "chain": the envelope rows
// plus the inverses of its kBlk x kBlk diagonal blocks.  The small separator
// system Sigma is applied through its inverse, formed once from its Cholesky
// factor, so that stage is a parallel dense product.
struct ChainMeta {
  int64_t row0;     // first row (global c index)
  int32_t nrows;    // rows in the chain
  int32_t nblocks;  // ceil(nrows / kBlk)
  int64_t voff;     // doubles: [envelope (nnz) | D (nblocks * kTri)]; separator systems:
                    // the dense inverse (nrows x nrows, row-major) in schur_inv
  int64_t ioff;     // int32s: [first (nrows) | rowoff (nrows) | rmax (nblocks)]
  int32_t nnz;      // envelope entries
  int32_t comp;     // component id
  int64_t zoff;     // parts: offset of Z_p (column-major nrows x nadj) in the z values
  int64_t adj0;     // parts: first global c row of the adjacent separator range
  int32_t nadj;     // parts: rows in that range
  int32_t pad;
  int64_t coff;     // parts: offset of A_Sp (CSR over the nadj rows) and of the part's
                    // contribution A_Sp w_p in the coupling arrays
  int64_t doff;     // parts: offset of A_pp^-1 (dense, row-major) in pinv; -1 if not formed
};
constexpr int kTri = kBlk * (kBlk + 1) / 2;  // packed triangle of one diagonal block
constexpr int kDenseRows = 1024;             // largest part / separator system applied through its dense inverse
constexpr int kDenseRowsDevice = 20480;      // the same with the device inverse (contexts on a GPU), at
                                             // most what the separator kernel's LDS holds

// In-place inverse of a dense SPD matrix (n x n; symmetric, so either storage
// order); false when a pivot is not positive.
using DenseInverseFn = bool (*)(double* A, int64_t n, int device);
// Gauss-Jordan inverse on a device (setup_gpu.hip)
bool gpu_spd_inverse(double* A, int64_t n, int device);

struct DissectedFactor {
  std::vector<ChainMeta> parts;     // all parts of all components
  std::vector<ChainMeta> schur;     // one per component (nrows = 0 if no separator)
  std::vector<double> vals;         // chain values
  std::vector<int32_t> ints;        // chain metadata
  std::vector<double> zvals;        // Z_p
  std::vector<double> schur_inv;    // Sigma^-1 of every component (row-major)
  std::vector<int64_t> schur_chunks;  // (component, first row) of every 16-row chunk of Sigma^-1
  std::vector<int64_t> schur_chain;   // components whose separator system is a chain
  std::vector<int64_t> part_chunks;   // (part, first row) of every 64-row chunk of the parts
  // dense form of the part solves (when every part has at most kDenseRows rows):
  // w_p = A_pp^-1 r_p and A_Sp w_p = Z_p^T r_p as dense products
  bool dense = false;
  std::vector<double> pinv;           // A_pp^-1 of every part (row-major)
  std::vector<int64_t> dense_chunks;  // (kind 0: rows of A_pp^-1 | kind 1: columns of Z_p, part, first)
  // A_Sp of every part: rows are its adjacent separator rows, local columns
  std::vector<int32_t> cp_ptr;      // per part: nadj + 1 entries (offsets into cp_col/cp_val)
  std::vector<int32_t> cp_col;
  std::vector<double> cp_val;
  std::vector<int64_t> cp_rowptr;   // per part: offset of its nadj + 1 row pointers in cp_ptr
  // per separator row (c order, -1 elsewhere): the contribution slots of the
  // (at most two) parts on either side of its separator
  std::vector<int64_t> sep_src;     // 2 * n_c entries
  int64_t coupling_slots = 0;       // total contribution slots (sum of nadj)
  int64_t nnz_total = 0;            // stored factor values (chains + Z)
  int64_t max_chain_doubles = 0, max_chain_ints = 0, max_chain_rows = 0;
};

// Builds the dissected factor of S (rows already in the final c order) from
// the component ranges and part ranges chosen in assemble_implicit_host.
struct ComponentLayout {
  int64_t begin, size;
  std::vector<int64_t> part_begin;  // part p rows: [part_begin[p], part_begin[p+1]) local
  int64_t sep_begin;                // separators: [sep_begin, size) local
  std::vector<int64_t> sep_ptr;     // separator k rows: [sep_ptr[k], sep_ptr[k+1]) local (k = 0..P-2)
  std::vector<int64_t> rcm;         // c indices of the component in reverse Cuthill-McKee order
};
struct HostSetup;

// ---- nested-dissection supernodal factor for the device (nd_factor.cpp) ----
// Each connected component of the implicit block is ordered by geometric
// nested dissection: its nodes are split by a grid plane of cell faces (no
// cell straddles it, so the plane's nodes separate the two sides), and the
// sides are split again until they hold at most `leaf` rows.  Every split's
// plane nodes, and every leaf, form one supernode s of m rows, numbered in
// postorder (children before parents), so the supernodes of a subtree are a
// contiguous range of c indices.  struct(s) lists the k rows below s's
// diagonal block in the Cholesky factor S = L L^T (all of them in ancestors
// of s).  With L_ss the diagonal block and L_ts the block below it:
//   forward   b'_s = b_s - (updates of s's children at s's rows)
//             y_s  = L_ss^-1 b'_s,    W_s = C_s b'_s + (children's updates at struct(s)),
//             C_s  = L_ts L_ss^-1
//   backward  x_s  = L_ss^-T y_s - C_s^T x_struct(s)
// which is the forward and backward substitution of L y = b, L^T x = y by
// blocks (W_s carries the sum of L_{struct(s),d} y_d over the subtree of s).
// Both passes run level by level (height of a supernode in its tree), and
// the supernodes of one level are independent.
struct NdSnode {
  int64_t c0;      // first c index
  int32_t m, k;    // rows of the supernode, rows of struct(s)
  int32_t parent;  // supernode id of the parent, -1 for a root
  int32_t height;  // 0 for leaves, 1 + max over children otherwise
  int64_t foff;    // forward values: rows of L_ss^-1 (row r holds r + 1 values) then the k rows of C_s (m each)
  int64_t boff;    // backward values: row j holds column j of L_ss^-1 from row j down, then column j of C_s
  int64_t woff;    // offset of W_s in the update buffer
  int64_t soff;    // offset of struct(s) in the struct list
  int64_t goff;    // first of the m + k gather slots (b' rows, then W rows)
};
struct NdFactor {
  std::vector<NdSnode> sn;
  std::vector<int32_t> st;      // struct lists (c indices, ascending per supernode)
  std::vector<double> fwd, bwd;
  std::vector<int64_t> gptr;    // gather slots: sources [gptr[t], gptr[t + 1])
  std::vector<int32_t> gsrc;    // sources: indices into the update buffer
  int64_t w_len = 0;            // update buffer length (sum of k)
  int32_t height = -1;          // largest height
  int64_t nnz_L = 0;            // entries of L: sum of m (m + 1) / 2 + m k
  int64_t max_m = 0, max_mk = 0;
};
// Supernodes of one component in postorder: rows (c indices before the final
// permutation) and parent (index into the list, -1 for a root).
struct NdTreeNode {
  std::vector<int64_t> rows;
  int32_t parent = -1;
};
// geometric nested dissection of one component (its c indices `verts`)
void nd_dissect(const HostSetup& hs, const std::vector<int64_t>& verts, int64_t leaf,
                std::vector<NdTreeNode>& out);
// the numeric factor of S (rows in the final c order) over the supernodes
// (c0, m, parent set; all other fields are filled in); "" on success
std::string build_nd_factor(const Csr& S, NdFactor& F, int n_threads);
// host execution of the device algorithm (same data, same order of
// operations): x = S^-1 b (c order)
void nd_solve_host(const NdFactor& F, const double* b, double* x);

struct HostSetup {
  // description
  int dim = 2, p = 1, n = 2;
  int64_t ne[3] = {1, 1, 1};     // cells per direction (1 for unused dims)
  int64_t nn[3] = {1, 1, 1};     // nodes per direction
  double h[3] = {1, 1, 1};
  double rho = 1, c = 1, kappa = 1, alpha_f = 1e-5;
  int depth = 0;
  double src[3] = {0, 0, 0};
  double dt = 0, dt_crit = 0;
  Geometry geom;
  Ref1D ref;

  int64_t n_cells = 0, n_grid = 0;
  std::vector<uint8_t> cell_flag;      // per cell
  std::vector<uint8_t> node_kind;      // per grid node
  std::vector<int64_t> c_nodes;        // c order -> grid node
  std::vector<int64_t> c_index;        // grid node -> c index or -1
  std::vector<int64_t> d_nodes;        // ascending
  std::vector<uint32_t> kron_mask;     // 3D: bit per grid node, d nodes with only uncut adjacent cells
  std::vector<int64_t> kron_rest;      // 3D: the other d nodes (next to an empty cell), ascending
  int64_t n_active = 0;
  int64_t counts[3] = {0, 0, 0};       // empty, cut, uncut

  // cut-cell element matrices (dense, n^d x n^d, row-major), by cut id
  std::vector<int64_t> cut_cells;      // cell ids of cut cells
  std::vector<int64_t> cut_id;         // cell -> cut id or -1
  std::vector<double> Me_cut, Ke_cut;
  std::vector<double> Ke_uncut;        // shared uncut stiffness
  std::vector<double> Me_uncut_diag;   // shared uncut lumped mass (diagonal)

  // point source: grid nodes and values of f_x (all nonzeros)
  std::vector<int64_t> src_nodes;
  std::vector<double> src_vals;

  // implicit block (c order after component/RCM permutation)
  Csr Kcd;   // columns: grid ids of d nodes
  Csr Kcc;   // columns: c indices
  Csr Kc;    // full K^c, columns: grid ids (export)
  Csr Mcc, S;
  std::vector<double> fxc;             // f_x on c dofs
  std::vector<Component> comps_m;      // envelope factor of M^cc per component, RCM order (host)
  std::vector<ComponentLayout> layout; // components, parts and separators in c order
  DissectedFactor fac;                 // factor of S for the device (dissected form)
  bool nd = false;                     // the factor is the nested-dissection supernodal one
  int factor_form = 0;                 // 0: automatic (3D: nested dissection), 1: dissected, 2: nested dissection
  int64_t nd_leaf = 64;                // largest leaf of the nested dissection
  NdFactor ndf;                        // factor of S for the device (nested-dissection form)
  int64_t nnz_factor = 0;
  int64_t part_rows = 256;             // target rows per part of the dissection
  int64_t dense_rows = kDenseRows;     // parts / separator systems up to this size use dense inverses
  double beta = 0.25;                  // Newmark beta of the c block (0: central differences)
  bool hrz_cut_mass = false;           // HRZ-lumped cut-cell masses (comparator)
  DenseInverseFn dense_inverse = nullptr;  // device inverse of large blocks (null: host only)
  int inverse_device = 0;                  // the device it runs on
  int64_t device_inverse_min = kDenseRows;  // blocks above this size use dense_inverse
};

std::string setup_mesh_host(HostSetup& hs, int dim, const int* n_cells, const double* extent,
                            int p, double rho, double c, double alpha_f, int depth,
                            int n_holes, const double* centers, const double* radii,
                            const double* source, double dt, double cfl,
                            int n_forced, const int64_t* forced);
// assemble K^c, M^cc, S, permute by components + RCM, factorise.
// returns "" on success, else a message; *notspd set on a bad pivot.
std::string assemble_implicit_host(HostSetup& hs, bool* notspd);
// host solves with the envelope factors (vector in c order, in place)
void envelope_solve(const std::vector<Component>& comps, double* x);
// x <- (M^cc)^-1 x (c order, in place)
void mcc_solve(const HostSetup& hs, double* x);
// y = K^c u for a grid vector u (c order rows)
void kc_apply(const HostSetup& hs, const double* u, double* y);
// receiver weights: for each physical point the (p+1)^dim node ids of its
// cell (the lower one on a face) and the tensor Lagrange basis values there;
// "" on success, else a message (a point outside the box or in an empty cell)
std::string sample_weights(const HostSetup& hs, const double* pts, int64_t n, std::vector<int64_t>& ids,
                           std::vector<double>& wts);
// 2 / sqrt(lambda_max(K, M)) with the block mass (lumped on d, consistent on
// c) by power iteration from a seeded start; after assemble_implicit_host
double global_critical_step(const HostSetup& hs, int max_iter, double rel_tol);

// Rows of K over the dofs that the substeps of the local time-stepping
// leap-frog update (the fine dofs, i.e. the c dofs, and their d neighbours):
// F rows are the c dofs in c order, then the d nodes coupled to them
// (ascending grid id).  Columns are split into the c dofs (F-local index =
// c index) and all others (grid ids).  The mass is the lumped diagonal
// (GLL on uncut cells, HRZ on cut cells); "" on success.
struct LtsRows {
  std::vector<int64_t> node;   // grid id of every F row
  int64_t nc = 0;              // the first nc F rows are the c dofs
  Csr Ko, Kf;                  // K over F rows: other columns (grid ids), c columns (c index)
  std::vector<double> mass, fx;
};
std::string build_lts_rows(const HostSetup& hs, LtsRows& out);

std::string build_dissected_factor(const Csr& S, const std::vector<ComponentLayout>& comps,
                                   DissectedFactor& out, int64_t dense_rows = kDenseRows,
                                   DenseInverseFn inverse = nullptr, int64_t inverse_min = kDenseRows,
                                   int inverse_device = 0);

}  // namespace imex
