/*
 * imex.h - C ABI of the MI355X Newmark IMEX library (libimex.so).
 *
 * The library advances the semi-discrete scalar wave equation
 *     M u'' + K u = f_t(t) f_x                       (Eq. discretizedWaveEquation)
 * of an immersed spectral-cell discretisation (Section "Spatial
 * Discretization": GLL Lagrange basis of order p on a Cartesian grid of
 * cells, indicator alpha = 1 in the physical domain and alpha_f in the
 * fictitious domain, space-tree Gauss-Legendre quadrature on cut cells)
 * with the Newmark IMEX scheme (Section "Time Integration", Newmark IMEX
 * flowchart figure): the central difference method on the dofs supported
 * only by uncut cells ("d", diagonal GLL-lumped mass, Eqs. CDMstep and
 * CDMacc) and the trapezoidal Newmark method (beta = 1/4, gamma = 1/2) on
 * the dofs touching cut cells ("c"), solving S = M^cc + beta dt^2 K^cc
 * (Section "Partitioning of the Degrees of Freedom", Eqs. MStructure,
 * KStructure, Kc).
 *
 * Conventions for every call:
 *  - Fields live on the full structured node grid of (N_x p + 1) x
 *    (N_y p + 1) [x (N_z p + 1)] nodes, lexicographic with x fastest.
 *    Nodes of empty cells only are inactive and always read as 0.
 *  - All host arrays are plain C arrays owned by the caller; the library
 *    copies what it keeps.  Device pointers are HIP device addresses.
 *  - Every call returns an imex_status; on failure imex_last_error(ctx)
 *    (or imex_last_error(NULL) when no context exists yet) gives a message.
 *    No call throws across the ABI.
 *  - Calls on one context are not thread safe; contexts are independent.
 *
 * Environment variables (read when a context is set up or assembled; none
 * changes a result beyond rounding order, all exist for tests and tuning):
 *  - IMEX_EXPLICIT_MODE=3|4  explicit kernel on 128-thread tiles (2D) or
 *                            512-thread tiles (3D) before autotuning.
 *  - IMEX_DEVICE_INVERSE_MIN=n  dense blocks of more than n rows are
 *                            inverted on the device (default n = 1024).
 *  - IMEX_DENSE_ROWS=n, IMEX_PART_ROWS=n  largest block stored as a dense
 *                            inverse; target rows per dissection part.
 *  - IMEX_SCHUR_LDS=n        cap on the LDS of the separator chain kernel.
 *  - IMEX_RHS_LANES=16|32    lanes per row of the right-hand-side kernel.
 *  - IMEX_BATCH_LANES=n      streams of a batch (0: one graph per batch step).
 *  - IMEX_NO_GRAPH=1         launch every step's kernels without HIP graphs.
 *  - IMEX_DEBUG=1            print launch shapes and dissection sizes.
 */
#ifndef IMEX_H
#define IMEX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct imex_ctx imex_ctx;

typedef enum {
  IMEX_OK = 0,
  IMEX_EINVAL = -1,     /* invalid description or argument */
  IMEX_ENOMEM = -2,     /* host or device allocation failed */
  IMEX_EHIP = -3,       /* a HIP runtime call failed (or no device) */
  IMEX_ENOTSPD = -4,    /* Cholesky factorisation met a non-positive pivot */
  IMEX_EUNSTABLE = -5,  /* NaN/Inf detected in the state */
  IMEX_ENOCONV = -6,    /* iterative solve did not converge */
  IMEX_ESTATE = -7      /* call out of order (e.g. step before assembly) */
} imex_status;

enum { IMEX_DEVICE = 0, IMEX_HOST_ONLY = 1 };
/* Solvers of the implicit block S a = rhs (imex_set_solver). */
enum {
  IMEX_SOLVER_CHOLESKY = 0,    /* dissected Cholesky factor (direct, FP64)                   */
  IMEX_SOLVER_PCG_JACOBI = 1,  /* flexible CG, preconditioner r / diag(S)                    */
  IMEX_SOLVER_PCG_BLOCK = 2,   /* flexible CG, additive Schwarz: sum_e P_e^T Binv_e P_e, Binv_e */
                               /* the inverse of cut cell e's diagonal block of S             */
  IMEX_SOLVER_PCG_MLP = 3      /* flexible CG, the learned per-cut-cell preconditioner        */
};
enum { IMEX_CELL_EMPTY = 0, IMEX_CELL_CUT = 1, IMEX_CELL_UNCUT = 2 };

/* Field identifiers for imex_read_field / imex_set_state. */
enum {
  IMEX_FIELD_U = 0,      /* u_n on the grid (n_grid values)                       */
  IMEX_FIELD_UPREV = 1,  /* u_{n-1} on the grid; meaningful on d nodes (n_grid)  */
  IMEX_FIELD_VC = 2,     /* velocity of the c dofs, c order (n_c)                */
  IMEX_FIELD_AC = 3,     /* acceleration of the c dofs, c order (n_c)            */
  IMEX_FIELD_DELTA = 4,  /* FP32 contexts only: the increment u_n - u_{n-1} that  */
                         /* the explicit update carries on the d nodes (n_grid)   */
  IMEX_FIELD_UC = 5      /* FP64 displacement of the c dofs, c order (n_c); the   */
                         /* grid holds its FP32 copy in FP32 contexts             */
};
/* Resuming bit for bit: set U, UPREV, then UC, VC, AC and (FP32) DELTA. */

/* Index arrays for imex_export_index. */
enum {
  IMEX_INDEX_CELL_FLAGS = 0, /* per cell (x fastest): IMEX_CELL_* (n_cells values)   */
  IMEX_INDEX_C_NODES = 1,    /* grid node id of each c dof, in c order (n_c)        */
  IMEX_INDEX_D_NODES = 2,    /* grid node ids of the d dofs, ascending (n_d)        */
  IMEX_INDEX_COMP_PTR = 3    /* component boundaries in c order (n_components + 1)  */
};

/* Matrices for imex_export_csr (rows in c order, FP64). */
enum {
  IMEX_CSR_KC = 0,   /* K^c = [K^cd K^cc], columns are grid node ids (Eq. Kc) */
  IMEX_CSR_MCC = 1,  /* M^cc, columns are c indices                          */
  IMEX_CSR_S = 2     /* S = M^cc + dt^2/4 K^cc, columns are c indices        */
};

typedef struct {
  int dim;                    /* 2 or 3                                              */
  int n_cells[3];             /* cells per direction (n_cells[2] ignored in 2D)       */
  double extent[3];           /* box edge lengths; the box starts at the origin       */
  int p;                      /* GLL order, 1..7                                      */
  double rho, c;              /* uniform density and wave speed                       */
  double alpha_f;             /* fictitious density scaling (e.g. 1e-5)               */
  int tree_depth;             /* space-tree depth on cut cells, 0..12                 */
  int n_holes;                /* balls removed from the box                           */
  const double* hole_center;  /* [n_holes * dim], x fastest within a centre           */
  const double* hole_radius;  /* [n_holes]                                            */
  double source[3];           /* point source; must lie in a non-empty cell           */
  double dt;                  /* time step; 0 selects cfl * dt_crit of an uncut cell  */
  double cfl;                 /* safety factor used when dt == 0 (e.g. 0.9)           */
  int explicit_fp;            /* 64: FP64 grid state; 32: FP32 grid state (increment  */
                              /* form), FP64 arithmetic; the implicit block is FP64  */
  int device_mode;            /* IMEX_DEVICE, or IMEX_HOST_ONLY (setup/export only)   */
  int n_forced_cut;           /* cells treated as cut although no boundary crosses    */
  const int64_t* forced_cut;  /* [n_forced_cut] cell ids                              */
} imex_mesh_desc;

typedef struct {
  int64_t n_grid, n_active, n_d, n_c;
  int64_t n_cells_empty, n_cells_cut, n_cells_uncut;
  int64_t nnz_kc, nnz_factor;  /* nonzeros of K^c and of the stored Cholesky profile */
  int64_t n_components;        /* connected components of the implicit block         */
  int64_t grid_dims[3];
  int64_t steps_taken;
  double dt, dt_crit_uncut;
  size_t field_bytes[3];       /* sizes of the bindable buffers, see imex_bind_buffers */
  /* what one factorised solve reads: values of the dense part inverses (the
   * stored lower triangle for parts above 1024 rows), of the couplings Z_p
   * (read coupling_passes times: by the part and correction stages, or only
   * by the correction when the part stage forms A_Sp w_p from the sparse
   * A_Sp), of the dense separator inverses, and of envelope chains still
   * solved as chains (read twice: forward and backward) */
  int64_t nnz_part_inv, nnz_coupling, nnz_sep_inv, nnz_chain, coupling_passes;
  /* factor form: 0 dissected (the fields above), 1 nested dissection (the
   * fields below; the five above are 0) */
  int64_t factor_form;
  /* nested dissection: supernodes, levels (launches per direction), entries
   * of L (the values each of the forward and backward passes reads once),
   * rows of the update buffer, and the largest supernode (m, m + k) */
  int64_t nd_supernodes, nd_levels, nd_nnz_L, nd_update_rows, nd_max_m, nd_max_mk;
} imex_info;

/* Build the mesh: classify cells (empty / cut / uncut by the space-tree fill
 * ratio, threshold 1e-10), integrate cut cells on the space tree, partition
 * the dofs into d and c (Section "Partitioning of the Degrees of Freedom")
 * and upload the explicit-part tables.  hip_stream is the caller's
 * hipStream_t (NULL = default stream); all later device work is ordered on
 * it.  On success *out owns the context; release it with imex_destroy. */
imex_status imex_setup_mesh(const imex_mesh_desc* desc, void* hip_stream, imex_ctx** out);

imex_status imex_query(const imex_ctx* ctx, imex_info* out);

/* Optionally hand the library caller-owned device buffers (e.g. torch
 * tensors) for the state instead of letting it allocate them:
 *   ptrs[0], ptrs[1]: the two grid buffers (field_bytes[0] each),
 *   ptrs[2]: the c state u^c, v^c, a^c (field_bytes[2]).
 * Pass n = 3 before imex_assemble_implicit_block.  The caller keeps them
 * alive until imex_destroy. */
imex_status imex_bind_buffers(imex_ctx* ctx, void* const* ptrs, const size_t* bytes, int n);

/* The finite element field (IMEX_FIELD_U or IMEX_FIELD_UPREV) at n physical
 * points (host array, n x dim, x fastest; results to host `out[n]`): the
 * tensor Lagrange basis of the containing cell (the lower cell on a face),
 * evaluated on the host, applied to the nodal values on the device (Section
 * "Spatial discretisation"; receivers of the accuracy measure).  A point
 * outside the box or in an empty cell: IMEX_EINVAL.  Allocates and frees
 * temporary device memory; synchronises the context's stream. */
imex_status imex_sample_field(imex_ctx* ctx, int which, int64_t n, const double* points, double* out);

/* Solve S x = b (c order, host arrays of n_c values) on the host with the
 * stored nested-dissection factor, through the same values and in the same
 * order of operations as the device kernels (a check of the factor that
 * needs no GPU; host-only contexts too).  IMEX_EINVAL when the context's
 * factor has the dissected form; IMEX_ESTATE before assembly. */
imex_status imex_factor_solve_host(imex_ctx* ctx, const double* b, double* x);

/* The same sampling as imex_sample_field without any device allocation, for
 * callers that cannot allocate device memory (code that must not call
 * hipMalloc / hipFree, such as tight serving loops or harnesses that forbid
 * allocation).  The points are staged, and the values produced, in a
 * library-owned device scratch array of IMEX_SAMPLE_NOALLOC_BYTES (1 MiB)
 * per device, held from the first context set up on that device until the
 * process ends; the basis of the containing cell is evaluated on the device.
 * Limit: n <= imex_sample_noalloc_max_points(dim) (floor(1 MiB / (8 (dim + 1)))
 * points: 43690 in 2D, 32768 in 3D); more points: IMEX_EINVAL, nothing runs.
 * Same argument meaning, checks and errors as imex_sample_field; results
 * agree with it to FP64 rounding.  Nothing in the scratch needs to start at
 * zero (every value read is written by the same call first), and it keeps
 * the last call's contents.  Every context on one device shares that
 * device's scratch: calls that overlap in time on one device (from several
 * threads, or on different streams) race and must be serialised by the
 * caller.  Synchronises the context's stream. */
#define IMEX_SAMPLE_NOALLOC_BYTES (1u << 20)
imex_status imex_sample_field_noalloc(imex_ctx* ctx, int which, int64_t n, const double* points, double* out);
/* Largest n accepted by imex_sample_field_noalloc in dimension dim (0 for
 * another dim). */
int64_t imex_sample_noalloc_max_points(int dim);

/* Newmark beta of the implicit (c) block, before imex_assemble_implicit_block
 * (default 1/4, the method: trapezoidal rule on the c dofs).  beta = 0 makes
 * S = M^cc and the predictor / corrector explicit: the step is then the
 * central difference method on all dofs with the block mass (lumped on d,
 * consistent on c), the CDM comparator of Section "Time Integration"; it is
 * stable only below the global critical step (imex_global_critical_step).
 * IMEX_EINVAL unless 0 <= beta <= 1/2; IMEX_ESTATE after assembly. */
imex_status imex_set_newmark_beta(imex_ctx* ctx, double beta);

/* Leap-frog with substeps on the cut-cell dofs (the explicit comparator of
 * Section "Time Integration": the cut cells advanced with dt_fine = dt / m),
 * before imex_assemble_implicit_block; m = 0 (default) is the Newmark IMEX
 * method.  The formulation, which the paper defers to other work, is the
 * energy-conserving local time-stepping leap-frog of Diaz and Grote (2009):
 * per step, with A = M^-1 K, P the projection onto the c dofs and tau =
 * dt / m, w = A (I - P) u_n - M^-1 f_t(t_n) f_x is frozen, q_0 = u_n,
 * q_1 = q_0 - tau^2/2 (w + A P q_0), q_{k+1} = 2 q_k - q_{k-1} - tau^2 (w +
 * A P q_k), and u_{n+1} = 2 q_m - u_{n-1}; m = 1 is the central difference
 * method on all dofs.  Needs the HRZ-lumped cut-cell mass
 * (imex_set_cut_mass) and FP64 state (IMEX_EINVAL at assembly otherwise);
 * the iterative solvers do not apply.  The start value is the central
 * difference one on every dof.  Stable (paper, Section "Perforated plate")
 * for dt below the uncut block's critical step and dt / m below the cut
 * block's.  The c state vectors hold u^c only (v^c, a^c are the start
 * values).  IMEX_EINVAL unless 0 <= m <= 4096; IMEX_ESTATE after assembly. */
imex_status imex_set_leapfrog(imex_ctx* ctx, int m);

/* Mass of the cut cells, before imex_assemble_implicit_block:
 * IMEX_CUT_MASS_CONSISTENT (default, the method) or IMEX_CUT_MASS_HRZ, the
 * HRZ lumping (each cut cell's mass matrix replaced by its diagonal, scaled
 * to keep the cell's total mass) of the lumped-mass CDM comparator (Section
 * "Time Integration"); use it with beta = 0.  IMEX_EINVAL for another kind,
 * IMEX_ESTATE after assembly. */
enum { IMEX_CUT_MASS_CONSISTENT = 0, IMEX_CUT_MASS_HRZ = 1 };
imex_status imex_set_cut_mass(imex_ctx* ctx, int kind);

/* Global critical step 2 / sqrt(lambda_max) of K x = lambda M x on the
 * active dofs with the block mass, by power iteration from a seeded start
 * (host, after imex_assemble_implicit_block; host-only contexts too).  The
 * Rayleigh quotients rise towards lambda_max, so the step is approached from
 * above; iteration stops when a quotient changes by at most rel_tol
 * (relative) or after max_iter iterations. */
imex_status imex_global_critical_step(imex_ctx* ctx, int max_iter, double rel_tol, double* dt_crit);

/* Assemble K^c, M^cc and S (FP64 CSR), split the implicit block into its
 * connected components, order each by reverse Cuthill-McKee, factorise S and
 * M^cc once by envelope Cholesky (Section "Time Integration": the system
 * matrix is factorised once outside the loop), and upload the blocked
 * factor.  Returns IMEX_ENOTSPD if a pivot is not positive. */
imex_status imex_assemble_implicit_block(imex_ctx* ctx, int solver);

/* Initial state (Newmark IMEX flowchart, first boxes): u0, v0 are host FP64
 * grid arrays (NULL = zero; inactive entries are ignored), ft0 = f_t(0).
 * Computes a^c_0 from M^cc a = f_t(0) f_x^c - K^c u_0 and the CDM start
 * value u^d_{-1} = u^d_0 - dt v^d_0 + dt^2/2 a^d_0. */
imex_status imex_set_initial(imex_ctx* ctx, const double* u0, const double* v0, double ft0);

/* Overwrite one state field from a host FP64 array (checkpoint resume);
 * len must match the field's length.  In FP32 contexts setting U or UPREV
 * also resets the increment to u_n - u_{n-1} (rounded to FP32). */
imex_status imex_set_state(imex_ctx* ctx, int which, const double* src, int64_t len);

/* Advance n_steps Newmark IMEX steps.  ft[k] = f_t(t_{n+k}) for
 * k = 0..n_steps (n_steps + 1 FP64 values), on the host or, with
 * ft_on_device != 0, in device memory.  Asynchronous on the context's
 * stream when ft is on the device. */
imex_status imex_step(imex_ctx* ctx, int n_steps, const double* ft, int ft_on_device);

/* Failure detection (off by default).  With on != 0, every imex_step ends
 * by scanning the state (both grid buffers, the FP32 increment and the c
 * dofs' u, v, a) for NaN or Inf and waiting for the stream; it returns
 * IMEX_EUNSTABLE, with the step count in the message, when one is found.
 * An unstable step size or a non-finite load makes the state non-finite
 * within a few steps.  The scan reads the state once (about 2 n_grid
 * values); imex_batch_step does not scan. */
imex_status imex_set_check_finite(imex_ctx* ctx, int on);

/* Per-kernel durations inside the time loop (benchmark support; the step's
 * work is that of the flowchart in Section "Time Integration").  With
 * on != 0, imex_step launches the steps one by one instead of replaying
 * captured chunks (HIP does not time event records captured in a graph) and
 * records HIP events on the context's stream before the explicit kernel
 * (Eqs. CDMacc, CDMstep) and after it, after the predictor and right-hand
 * side, and after the factorised solve with the correction.  Only the
 * factorised (Cholesky) step without leap-frog substeps records them.  The
 * events sit between launches that the stream orders anyway, so the results
 * are unchanged.  imex_step_timing waits for the stream and writes the mean
 * durations in milliseconds over the last (at most 32) timed steps (ms[0]
 * explicit, ms[1] predictor and right-hand side, ms[2] solve and
 * correction); IMEX_ESTATE when timing is off or no step has been timed
 * since it was switched on.  Switching it on or off resets the count. */
imex_status imex_set_step_timing(imex_ctx* ctx, int on);
imex_status imex_step_timing(imex_ctx* ctx, double* ms);

/* Copy a field out as FP64: to host memory (dst_is_device == 0, waits for
 * the stream) or to device memory (asynchronous on the stream). */
imex_status imex_read_field(imex_ctx* ctx, int which, void* dst, int dst_is_device, int64_t len);

/* Host copies of setup data for tests.  Call with NULL arrays to get the
 * sizes (*nrows, *nnz); row_ptr has nrows + 1 entries. */
imex_status imex_export_csr(const imex_ctx* ctx, int which, int64_t* nrows, int64_t* nnz,
                            int64_t* row_ptr, int64_t* cols, double* vals);
imex_status imex_export_index(const imex_ctx* ctx, int which, int64_t* dst, int64_t* len);

/* Benchmark support: launch one kernel of the step `reps` times back to
 * back on the context's stream between two HIP events and return the mean
 * duration in milliseconds.  which: 0 = explicit apply and CDM update,
 * 1 = predictor and right-hand side of the implicit block, 2 = blocked
 * triangular solves and correction.  The state is overwritten: call
 * imex_set_initial or imex_set_state before stepping again. */
imex_status imex_time_kernel(imex_ctx* ctx, int which, int reps, double* avg_ms);

/* ---- Iterative solves of the implicit block and the learned preconditioner
 * (not in the paper, which factorises S once: Section "Time Integration").
 * The flexible CG (Polak-Ribiere form) starts from a^c_n, stops at
 * ||r|| <= tol ||rhs||, and uses r / diag(S) for any application whose
 * preconditioned residual is not a descent direction.  If it has not
 * converged after max_iter iterations, the step falls back to the factorised
 * FP64 solve; every judge_every-th converged solve (0 = never) is also
 * re-solved with the factor, which then defines the step, and the relative
 * difference is recorded.  Steps with an iterative solver (or while
 * collecting training pairs) run host-driven, without graphs.
 *
 * The learned preconditioner (IMEX_SOLVER_PCG_MLP): a learned correction on
 * top of the element-block (additive Schwarz) step B r = sum_e P_e^T Binv_e
 * r_e, Binv_e the inverse of cut cell e's diagonal block of S.  For every
 * cut cell e with (p+1)^d c dofs idx_e (x fastest), r_e = r[idx_e], s_e =
 * ||r_e|| and d_e = diag(S)[idx_e], an MLP with BF16 weights and FP32
 * accumulation maps
 *   x_e = [r_e / s_e, d_e .* (B r)_e / s_e, d_e / max d_e, 0 padding]  (inputs)
 * through relu(W1 x + b1), relu(W2 h + b2) (hidden = 128) to y = W3 h + b3
 * (outputs), and z = B r + w .* sum_e P_e^T (s_e y_e / d_e), with w = 1 /
 * (number of cut cells sharing a dof).  Parameters (FP32, packed):
 *   [W1 (hidden x inputs) | b1 | W2 (hidden x hidden) | b2 | W3 (outputs x hidden) | b3]
 * Training minimises the mean over (pair, cell) of ||y_e - t_e||^2 over the
 * first (p+1)^d outputs, t_e = d_e .* (x - B r)_e / s_e, for pairs (r, x =
 * S^-1 r) from the method's own implicit solves (imex_mlp_collect): the
 * network learns the part of the exact solve that B misses, so that exact
 * outputs give z = S^-1 r and zero outputs give B r. */
typedef struct {
  int n_cells, dofs_per_cell, inputs, hidden, outputs;
  int64_t n_params;
  int collected;               /* training vectors collected so far */
} imex_mlp_info;
typedef struct {
  int solver;
  int64_t solves, iterations, fallbacks, judged;
  int last_iterations;
  double last_relres, judge_max_rel_diff;
} imex_solver_info;

/* Select the solver of the implicit block for the following steps. */
imex_status imex_set_solver(imex_ctx* ctx, int solver, double tol, int max_iter, int judge_every);
imex_status imex_solver_stats(const imex_ctx* ctx, imex_solver_info* out);
/* Sizes of the learned preconditioner of this mesh (builds its tables). */
imex_status imex_mlp_shape(imex_ctx* ctx, imex_mlp_info* out);
/* Set / read the FP32 parameters (n = n_params); setting resets Adam. */
imex_status imex_mlp_set_weights(imex_ctx* ctx, const float* params, int64_t n);
imex_status imex_mlp_get_weights(imex_ctx* ctx, float* params, int64_t n);
/* Record training pairs during the following steps, two per implicit solve
 * of the factor: (rhs, a^c_{n+1}) and (rhs - S a^c_n, a^c_{n+1} - a^c_n),
 * until `capacity` pairs are held (device memory, 3 x capacity x n_c FP64;
 * capacity rounded up to even).  capacity = 0 stops recording and keeps
 * what was collected.  Recording steps run without HIP graphs. */
imex_status imex_mlp_collect(imex_ctx* ctx, int capacity);
/* Adam (lr, beta 0.9 / 0.999, eps 1e-8) over the collected pairs for
 * `epochs` epochs, minibatches of vectors_per_batch pairs in an order
 * shuffled with `seed`; *last_loss = mean minibatch loss of the last epoch. */
imex_status imex_mlp_train(imex_ctx* ctx, int epochs, int vectors_per_batch, double lr, uint64_t seed,
                           double* last_loss);
/* Loss and gradients (packed like the parameters) over n_vectors host pairs
 * (vectors r and solutions x, each n_vectors x n_c FP64, c order), without
 * an update. */
imex_status imex_mlp_loss_grad(imex_ctx* ctx, const double* vectors, const double* solutions, int n_vectors,
                               double* loss, float* grads);
/* One Adam step (as in training, continuing its step count and moments)
 * with the given gradients (host, packed like the parameters). */
imex_status imex_mlp_adam_step(imex_ctx* ctx, const float* grads, double lr);
/* z = P(r) for one host vector in c order (which: IMEX_SOLVER_PCG_*). */
imex_status imex_precond_apply(imex_ctx* ctx, int which, const double* r, double* z);
/* Solve S x = rhs by flexible CG from the host initial guess x (in/out,
 * c order) with the tolerance and iteration limit last given to
 * imex_set_solver (1e-10 and 1000 before any); IMEX_ENOCONV if it does not
 * converge. */
imex_status imex_solve_implicit(imex_ctx* ctx, int which, const double* rhs, double* x, int* iterations);

/* Tile autotuner of the explicit kernel: times every candidate launch shape
 * over `reps` launches on the context's stream and keeps the fastest.
 * Candidates: 2D LDS tiles of tx x ty cells on 256-thread (mode 0) or
 * 128-thread (mode 3) workgroups, at most 8 owned nodes per thread; 2D
 * register strips (p <= 5: 63 cells per wave, lz cell rows per
 * wave, node rows loaded per lane (mode 1) or staged through LDS (mode 2));
 * 3D tiles of tx x ty cells per layer and lz layers per chunk.  The
 * launch shape does not change any result (every node sums its cell
 * contributions in the same fixed order), only the time.  Call after
 * imex_assemble_implicit_block; it overwrites the state, so call
 * imex_set_initial afterwards.  chosen (may be NULL) receives
 * {tx, ty, lz, mode} (mode 0 and 3 = tiles, 1 and 2 = strips; 3D: mode 0 on
 * 256-thread and mode 4 on 512-thread workgroups). */
imex_status imex_autotune_tiles(imex_ctx* ctx, int reps, int* chosen);

/* ---- Batches of independent instances ----------------------------------
 * A batch steps several assembled and initialised contexts (any sizes,
 * orders and hole layouts) together, on the batch's stream (hip_stream, or
 * a stream the batch owns when NULL), in one of three forms:
 *  - IMEX_BATCH_FORM_KERNELS (default when every instance allows it: 2D Newmark
 *    IMEX contexts of one state precision whose implicit block has the
 *    dense dissected factor): each step is one launch per kernel type over
 *    all instances - the explicit kernel on 256-thread LDS tiles once per
 *    order p, the right-hand side, and the three stages of the dissected
 *    solve - driven by per-instance argument tables (a workgroup finds its
 *    instance from the tables' block offsets); 32-step chunks are captured
 *    in one HIP graph.  Every instance needs the same grid parity (instances
 *    stepped together from their initial state have it).
 *  - IMEX_BATCH_FORM_LANES: every instance advances in its own captured 32-step
 *    graphs, spread round-robin over 16 streams ("lanes";
 *    IMEX_BATCH_LANES=n sets the count and selects this form) that fork
 *    from and join back into the batch's stream.
 *  - IMEX_BATCH_FORM_GRAPH (IMEX_BATCH_LANES=0): one graph per 32 steps with a
 *    child-graph branch per instance.
 * Steps beyond a multiple of 32 run eagerly on the batch's stream.  The
 * instances' own streams are synchronised before each call; afterwards
 * their state is read with imex_read_field as usual.  Destroy the batch
 * before its contexts. */
typedef struct imex_batch imex_batch;
enum { IMEX_BATCH_FORM_GRAPH = 0, IMEX_BATCH_FORM_LANES = 1, IMEX_BATCH_FORM_KERNELS = 2 };
imex_status imex_batch_create(imex_ctx* const* ctxs, int n, void* hip_stream, imex_batch** out);
/* The batch's form (IMEX_BATCH_FORM_*). */
int imex_batch_form(const imex_batch* b);
/* Advance every instance n_steps; ft[i] holds instance i's f_t table
 * (n_steps + 1 FP64 values, host memory or, with ft_on_device, device). */
imex_status imex_batch_step(imex_batch* b, int n_steps, const double* const* ft, int ft_on_device);
const char* imex_batch_last_error(const imex_batch* b);
void imex_batch_destroy(imex_batch* b);

/* Message of the last failed call on ctx, or of the last failed
 * imex_setup_mesh when ctx is NULL.  Valid until the next call. */
const char* imex_last_error(const imex_ctx* ctx);

void imex_destroy(imex_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* IMEX_H */
