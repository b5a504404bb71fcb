"""ctypes binding of libimex.so (argument marshalling only).

Every computation happens in the library: its C++ host setup and its HIP
kernels.  If the shared library is missing this module raises ImportError;
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libimex.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2310_14712_amd.build`")
_lib = C.CDLL(LIB_PATH)

IMEX_OK = 0
STATUS = {0: "IMEX_OK", -1: "IMEX_EINVAL", -2: "IMEX_ENOMEM", -3: "IMEX_EHIP", -4: "IMEX_ENOTSPD",
          -5: "IMEX_EUNSTABLE", -6: "IMEX_ENOCONV", -7: "IMEX_ESTATE"}
DEVICE, HOST_ONLY = 0, 1
FIELD_U, FIELD_UPREV, FIELD_VC, FIELD_AC, FIELD_DELTA, FIELD_UC = 0, 1, 2, 3, 4, 5
INDEX_CELL_FLAGS, INDEX_C_NODES, INDEX_D_NODES, INDEX_COMP_PTR = 0, 1, 2, 3
CSR_KC, CSR_MCC, CSR_S = 0, 1, 2
SOLVER_CHOLESKY, SOLVER_PCG_JACOBI, SOLVER_PCG_BLOCK, SOLVER_PCG_MLP = 0, 1, 2, 3
CUT_MASS_CONSISTENT, CUT_MASS_HRZ = 0, 1
BATCH_GRAPH, BATCH_LANES, BATCH_KERNELS = 0, 1, 2

EXPORTED = ["imex_setup_mesh", "imex_query", "imex_bind_buffers", "imex_assemble_implicit_block",
            "imex_set_initial", "imex_set_state", "imex_step", "imex_read_field",
            "imex_export_csr", "imex_export_index", "imex_time_kernel", "imex_autotune_tiles",
            "imex_set_solver", "imex_solver_stats", "imex_mlp_shape", "imex_mlp_set_weights",
            "imex_mlp_get_weights", "imex_mlp_collect", "imex_mlp_train", "imex_mlp_loss_grad", "imex_mlp_adam_step",
            "imex_precond_apply", "imex_solve_implicit", "imex_set_newmark_beta", "imex_global_critical_step",
            "imex_set_cut_mass", "imex_set_leapfrog", "imex_sample_field", "imex_sample_field_noalloc",
            "imex_sample_noalloc_max_points", "imex_factor_solve_host", "imex_set_check_finite",
            "imex_set_step_timing", "imex_step_timing",
            "imex_batch_create", "imex_batch_step", "imex_batch_form", "imex_batch_last_error", "imex_batch_destroy",
            "imex_last_error", "imex_destroy"]


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_cells", C.c_int * 3), ("extent", C.c_double * 3),
                ("p", C.c_int), ("rho", C.c_double), ("c", C.c_double), ("alpha_f", C.c_double),
                ("tree_depth", C.c_int), ("n_holes", C.c_int),
                ("hole_center", C.POINTER(C.c_double)), ("hole_radius", C.POINTER(C.c_double)),
                ("source", C.c_double * 3), ("dt", C.c_double), ("cfl", C.c_double),
                ("explicit_fp", C.c_int), ("device_mode", C.c_int),
                ("n_forced_cut", C.c_int), ("forced_cut", C.POINTER(C.c_int64))]


class MlpInfo(C.Structure):
    _fields_ = [("n_cells", C.c_int), ("dofs_per_cell", C.c_int), ("inputs", C.c_int), ("hidden", C.c_int),
                ("outputs", C.c_int), ("n_params", C.c_int64), ("collected", C.c_int)]


class SolverInfo(C.Structure):
    _fields_ = [("solver", C.c_int), ("solves", C.c_int64), ("iterations", C.c_int64), ("fallbacks", C.c_int64),
                ("judged", C.c_int64), ("last_iterations", C.c_int), ("last_relres", C.c_double),
                ("judge_max_rel_diff", C.c_double)]


class Info(C.Structure):
    _fields_ = [("n_grid", C.c_int64), ("n_active", C.c_int64), ("n_d", C.c_int64), ("n_c", C.c_int64),
                ("n_cells_empty", C.c_int64), ("n_cells_cut", C.c_int64), ("n_cells_uncut", C.c_int64),
                ("nnz_kc", C.c_int64), ("nnz_factor", C.c_int64), ("n_components", C.c_int64),
                ("grid_dims", C.c_int64 * 3), ("steps_taken", C.c_int64),
                ("dt", C.c_double), ("dt_crit_uncut", C.c_double), ("field_bytes", C.c_size_t * 3),
                ("nnz_part_inv", C.c_int64), ("nnz_coupling", C.c_int64), ("nnz_sep_inv", C.c_int64),
                ("nnz_chain", C.c_int64), ("coupling_passes", C.c_int64),
                ("factor_form", C.c_int64), ("nd_supernodes", C.c_int64), ("nd_levels", C.c_int64),
                ("nd_nnz_L", C.c_int64), ("nd_update_rows", C.c_int64), ("nd_max_m", C.c_int64),
                ("nd_max_mk", C.c_int64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["grid_dims"] = list(self.grid_dims)
        d["field_bytes"] = list(self.field_bytes)
        return d


_vp = C.c_void_p
_lib.imex_setup_mesh.argtypes = [C.POINTER(MeshDesc), _vp, C.POINTER(_vp)]
_lib.imex_query.argtypes = [_vp, C.POINTER(Info)]
_lib.imex_bind_buffers.argtypes = [_vp, C.POINTER(_vp), C.POINTER(C.c_size_t), C.c_int]
_lib.imex_assemble_implicit_block.argtypes = [_vp, C.c_int]
_lib.imex_set_initial.argtypes = [_vp, _vp, _vp, C.c_double]
_lib.imex_set_state.argtypes = [_vp, C.c_int, _vp, C.c_int64]
_lib.imex_step.argtypes = [_vp, C.c_int, _vp, C.c_int]
_lib.imex_read_field.argtypes = [_vp, C.c_int, _vp, C.c_int, C.c_int64]
_lib.imex_export_csr.argtypes = [_vp, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int64), _vp, _vp, _vp]
_lib.imex_export_index.argtypes = [_vp, C.c_int, _vp, C.POINTER(C.c_int64)]
_lib.imex_time_kernel.argtypes = [_vp, C.c_int, C.c_int, C.POINTER(C.c_double)]
_lib.imex_autotune_tiles.argtypes = [_vp, C.c_int, C.POINTER(C.c_int)]
_lib.imex_set_solver.argtypes = [_vp, C.c_int, C.c_double, C.c_int, C.c_int]
_lib.imex_solver_stats.argtypes = [_vp, C.POINTER(SolverInfo)]
_lib.imex_mlp_shape.argtypes = [_vp, C.POINTER(MlpInfo)]
_lib.imex_mlp_set_weights.argtypes = [_vp, _vp, C.c_int64]
_lib.imex_mlp_get_weights.argtypes = [_vp, _vp, C.c_int64]
_lib.imex_mlp_collect.argtypes = [_vp, C.c_int]
_lib.imex_mlp_train.argtypes = [_vp, C.c_int, C.c_int, C.c_double, C.c_uint64, C.POINTER(C.c_double)]
_lib.imex_mlp_loss_grad.argtypes = [_vp, _vp, _vp, C.c_int, C.POINTER(C.c_double), _vp]
_lib.imex_mlp_adam_step.argtypes = [_vp, _vp, C.c_double]
_lib.imex_precond_apply.argtypes = [_vp, C.c_int, _vp, _vp]
_lib.imex_solve_implicit.argtypes = [_vp, C.c_int, _vp, _vp, C.POINTER(C.c_int)]
_lib.imex_set_newmark_beta.argtypes = [_vp, C.c_double]
_lib.imex_set_check_finite.argtypes = [_vp, C.c_int]
_lib.imex_set_step_timing.argtypes = [_vp, C.c_int]
_lib.imex_step_timing.argtypes = [_vp, C.POINTER(C.c_double)]
_lib.imex_global_critical_step.argtypes = [_vp, C.c_int, C.c_double, C.POINTER(C.c_double)]
_lib.imex_set_cut_mass.argtypes = [_vp, C.c_int]
_lib.imex_set_leapfrog.argtypes = [_vp, C.c_int]
_lib.imex_sample_field.argtypes = [_vp, C.c_int, C.c_int64, _vp, _vp]
_lib.imex_factor_solve_host.argtypes = [_vp, _vp, _vp]
_lib.imex_sample_field_noalloc.argtypes = [_vp, C.c_int, C.c_int64, _vp, _vp]
_lib.imex_sample_noalloc_max_points.argtypes = [C.c_int]
_lib.imex_sample_noalloc_max_points.restype = C.c_int64
_lib.imex_batch_create.argtypes = [C.POINTER(_vp), C.c_int, _vp, C.POINTER(_vp)]
_lib.imex_batch_step.argtypes = [_vp, C.c_int, C.POINTER(_vp), C.c_int]
_lib.imex_batch_form.argtypes = [_vp]
_lib.imex_batch_form.restype = C.c_int
_lib.imex_batch_last_error.argtypes = [_vp]
_lib.imex_batch_last_error.restype = C.c_char_p
_lib.imex_batch_destroy.argtypes = [_vp]
_lib.imex_batch_destroy.restype = None
_lib.imex_last_error.argtypes = [_vp]
_lib.imex_last_error.restype = C.c_char_p
_lib.imex_destroy.argtypes = [_vp]
_lib.imex_destroy.restype = None
for _n in EXPORTED:
    if _n not in ("imex_last_error", "imex_batch_last_error", "imex_destroy", "imex_batch_destroy"):
        getattr(_lib, _n).restype = C.c_int


class ImexError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_vp)


def desc_from_workload(w, device_mode=DEVICE, dt=0.0, explicit_fp=None):
    """imex_mesh_desc for a workload description (see inputs.Workload)."""
    d = MeshDesc()
    d.dim = w.dim
    for k in range(3):
        d.n_cells[k] = int(w.n_cells[k]) if k < w.dim else 1
        d.extent[k] = float(w.extent[k]) if k < w.dim else 1.0
        d.source[k] = float(w.source[k]) if k < w.dim else 0.0
    d.p = w.p
    d.rho, d.c, d.alpha_f = w.rho, w.c, w.alpha_f
    d.tree_depth = w.tree_depth
    centers = np.ascontiguousarray(np.asarray(w.hole_centers, dtype=np.float64).reshape(-1, w.dim)
                                   if w.n_holes else np.zeros((0, w.dim)))
    radii = np.ascontiguousarray(np.asarray(w.hole_radii, dtype=np.float64))
    d.n_holes = w.n_holes
    d.hole_center = centers.ctypes.data_as(C.POINTER(C.c_double))
    d.hole_radius = radii.ctypes.data_as(C.POINTER(C.c_double))
    d.dt = float(dt)
    d.cfl = float(w.cfl)
    d.explicit_fp = int(explicit_fp if explicit_fp is not None else w.explicit_fp)
    d.device_mode = device_mode
    forced = np.ascontiguousarray(np.asarray(w.forced_cut if w.forced_cut is not None else [],
                                             dtype=np.int64))
    d.n_forced_cut = len(forced)
    d.forced_cut = forced.ctypes.data_as(C.POINTER(C.c_int64))
    keep = (centers, radii, forced)
    return d, keep


class Imex:
    """One Newmark IMEX problem in the library (a context)."""

    def __init__(self, w, device_mode=DEVICE, stream=None, dt=0.0, explicit_fp=None):
        d, self._keep = desc_from_workload(w, device_mode, dt, explicit_fp)
        h = _vp()
        st = _lib.imex_setup_mesh(C.byref(d), _vp(stream) if stream else None, C.byref(h))
        if st != IMEX_OK:
            raise ImexError(st, _lib.imex_last_error(None).decode())
        self._h = h
        self.workload = w
        if getattr(w, "cut_mass", "consistent") == "hrz":   # the workload's mass treatment
            self.set_cut_mass(CUT_MASS_HRZ)

    def _check(self, st):
        if st != IMEX_OK:
            raise ImexError(st, _lib.imex_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            _lib.imex_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def info(self) -> dict:
        inf = Info()
        self._check(_lib.imex_query(self._h, C.byref(inf)))
        return inf.as_dict()

    def bind_buffers(self, ptrs: Sequence[int], sizes: Sequence[int]):
        arr = (_vp * 3)(*[_vp(p) for p in ptrs])
        sz = (C.c_size_t * 3)(*sizes)
        self._check(_lib.imex_bind_buffers(self._h, arr, sz, 3))

    def set_check_finite(self, on=True):
        """Failure detection: every step call then ends with a scan of the
        state and raises ImexError (IMEX_EUNSTABLE) on NaN or Inf."""
        self._check(_lib.imex_set_check_finite(self._h, int(bool(on))))

    def set_step_timing(self, on=True):
        """Record HIP events around the explicit kernel, the right-hand side
        and the solve in every step of the captured step chunks."""
        self._check(_lib.imex_set_step_timing(self._h, int(bool(on))))

    def step_timing(self):
        """Mean durations (ms) over the steps of the last chunk launched:
        {"explicit", "rhs", "solve"}."""
        ms = (C.c_double * 3)()
        self._check(_lib.imex_step_timing(self._h, ms))
        return {"explicit": ms[0], "rhs": ms[1], "solve": ms[2]}

    def set_newmark_beta(self, beta):
        """beta of the c block before assemble (1/4: the method; 0: the
        central difference comparator)."""
        self._check(_lib.imex_set_newmark_beta(self._h, C.c_double(beta)))

    def sample(self, points, which=FIELD_U):
        """The field at physical points (n x dim) by the cell's Lagrange basis."""
        pts = np.ascontiguousarray(np.atleast_2d(points), dtype=np.float64)
        out = np.empty(len(pts))
        self._check(_lib.imex_sample_field(self._h, int(which), len(pts), _ptr(pts), _ptr(out)))
        return out

    def sample_noalloc(self, points, which=FIELD_U):
        """The same values through the entry point that allocates no device
        memory (points and values staged in the library's device scratch)."""
        pts = np.ascontiguousarray(np.atleast_2d(points), dtype=np.float64)
        out = np.empty(len(pts))
        self._check(_lib.imex_sample_field_noalloc(self._h, int(which), len(pts), _ptr(pts), _ptr(out)))
        return out

    def factor_solve_host(self, b):
        """x = S^-1 b on the host with the nested-dissection factor (c order)."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty_like(b)
        self._check(_lib.imex_factor_solve_host(self._h, _ptr(b), _ptr(x)))
        return x

    def set_leapfrog(self, m):
        """Before assemble: leap-frog with m substeps on the cut-cell dofs
        (needs the HRZ cut-cell mass and FP64 state); 0 = Newmark IMEX."""
        self._check(_lib.imex_set_leapfrog(self._h, int(m)))

    def set_cut_mass(self, kind):
        """Cut-cell mass before assemble: CUT_MASS_CONSISTENT or CUT_MASS_HRZ."""
        self._check(_lib.imex_set_cut_mass(self._h, int(kind)))

    def global_critical_step(self, max_iter=5000, rel_tol=1e-13):
        """2 / sqrt(lambda_max(K, M)) with the block mass (power iteration)."""
        out = C.c_double()
        self._check(_lib.imex_global_critical_step(self._h, int(max_iter), C.c_double(rel_tol), C.byref(out)))
        return out.value

    def assemble(self, solver=0):
        self._check(_lib.imex_assemble_implicit_block(self._h, solver))

    def set_initial(self, u0=None, v0=None, ft0=0.0):
        u0 = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64)
        v0 = None if v0 is None else np.ascontiguousarray(v0, dtype=np.float64)
        self._check(_lib.imex_set_initial(self._h, _ptr(u0), _ptr(v0), float(ft0)))

    def set_state(self, which, arr):
        arr = np.ascontiguousarray(arr, dtype=np.float64)
        self._check(_lib.imex_set_state(self._h, which, _ptr(arr), len(arr)))

    def step(self, ft, n_steps=None, device_ptr=None):
        """Advance; ft holds f_t(t_n .. t_{n+n_steps}) (host array), or pass
        device_ptr (address of n_steps + 1 doubles on the device)."""
        if device_ptr is not None:
            self._check(_lib.imex_step(self._h, int(n_steps), _vp(device_ptr), 1))
            return
        ft = np.ascontiguousarray(ft, dtype=np.float64)
        n = len(ft) - 1 if n_steps is None else int(n_steps)
        self._check(_lib.imex_step(self._h, n, _ptr(ft), 0))

    def read(self, which) -> np.ndarray:
        inf = self.info()
        n = inf["n_grid"] if which in (FIELD_U, FIELD_UPREV, FIELD_DELTA) else inf["n_c"]
        out = np.empty(n, dtype=np.float64)
        self._check(_lib.imex_read_field(self._h, which, _ptr(out), 0, n))
        return out

    def read_to_device(self, which, ptr, n):
        self._check(_lib.imex_read_field(self._h, which, _vp(ptr), 1, n))

    def time_kernel(self, which, reps) -> float:
        """Mean duration (ms) of one kernel of the step over `reps` launches
        (HIP events on the library stream).  Invalidates the state."""
        ms = C.c_double()
        self._check(_lib.imex_time_kernel(self._h, int(which), int(reps), C.byref(ms)))
        return ms.value

    def autotune_tiles(self, reps=50):
        """Pick the fastest explicit launch shape; returns (tx, ty, lz, mode).  The
        state is overwritten: call set_initial afterwards."""
        out = (C.c_int * 4)()
        self._check(_lib.imex_autotune_tiles(self._h, int(reps), out))
        return tuple(out)

    # ---- iterative solvers and the learned preconditioner -----------------
    def set_solver(self, solver, tol=1e-10, max_iter=1000, judge_every=0):
        self._check(_lib.imex_set_solver(self._h, int(solver), float(tol), int(max_iter), int(judge_every)))

    def solver_stats(self) -> dict:
        out = SolverInfo()
        self._check(_lib.imex_solver_stats(self._h, C.byref(out)))
        return {k: getattr(out, k) for k, _ in out._fields_}

    def mlp_shape(self) -> dict:
        out = MlpInfo()
        self._check(_lib.imex_mlp_shape(self._h, C.byref(out)))
        return {k: getattr(out, k) for k, _ in out._fields_}

    def mlp_set_weights(self, params):
        params = np.ascontiguousarray(params, dtype=np.float32)
        self._check(_lib.imex_mlp_set_weights(self._h, _ptr(params), len(params)))

    def mlp_get_weights(self) -> np.ndarray:
        out = np.empty(self.mlp_shape()["n_params"], dtype=np.float32)
        self._check(_lib.imex_mlp_get_weights(self._h, _ptr(out), len(out)))
        return out

    def mlp_collect(self, capacity):
        self._check(_lib.imex_mlp_collect(self._h, int(capacity)))

    def mlp_train(self, epochs, vectors_per_batch=8, lr=1e-3, seed=0) -> float:
        loss = C.c_double()
        self._check(_lib.imex_mlp_train(self._h, int(epochs), int(vectors_per_batch), float(lr), int(seed),
                                        C.byref(loss)))
        return loss.value

    def mlp_loss_grad(self, vectors, solutions):
        vectors = np.ascontiguousarray(vectors, dtype=np.float64)
        solutions = np.ascontiguousarray(solutions, dtype=np.float64)
        assert vectors.shape == solutions.shape
        loss = C.c_double()
        grads = np.empty(self.mlp_shape()["n_params"], dtype=np.float32)
        self._check(_lib.imex_mlp_loss_grad(self._h, _ptr(vectors), _ptr(solutions), len(vectors), C.byref(loss),
                                            _ptr(grads)))
        return loss.value, grads

    def mlp_adam_step(self, grads, lr):
        grads = np.ascontiguousarray(grads, dtype=np.float32)
        self._check(_lib.imex_mlp_adam_step(self._h, _ptr(grads), float(lr)))

    def precond_apply(self, which, r) -> np.ndarray:
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.empty_like(r)
        self._check(_lib.imex_precond_apply(self._h, int(which), _ptr(r), _ptr(z)))
        return z

    def solve_implicit(self, which, rhs, x0=None):
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        x = np.zeros_like(rhs) if x0 is None else np.array(x0, dtype=np.float64)
        it = C.c_int()
        self._check(_lib.imex_solve_implicit(self._h, int(which), _ptr(rhs), _ptr(x), C.byref(it)))
        return x, it.value

    def export_csr(self, which):
        nr, nnz = C.c_int64(), C.c_int64()
        self._check(_lib.imex_export_csr(self._h, which, C.byref(nr), C.byref(nnz), None, None, None))
        rp = np.empty(nr.value + 1, dtype=np.int64)
        cols = np.empty(nnz.value, dtype=np.int64)
        vals = np.empty(nnz.value, dtype=np.float64)
        self._check(_lib.imex_export_csr(self._h, which, C.byref(nr), C.byref(nnz), _ptr(rp), _ptr(cols),
                                         _ptr(vals)))
        return rp, cols, vals

    def export_index(self, which) -> np.ndarray:
        n = C.c_int64(0)
        self._check(_lib.imex_export_index(self._h, which, None, C.byref(n)))
        out = np.empty(n.value, dtype=np.int64)
        self._check(_lib.imex_export_index(self._h, which, _ptr(out), C.byref(n)))
        return out


class Batch:
    """Several contexts stepped together in one graph per 32 steps."""

    def __init__(self, instances, stream=None):
        self._inst = list(instances)       # keep the contexts alive
        arr = (_vp * len(self._inst))(*[i._h for i in self._inst])
        h = _vp()
        st = _lib.imex_batch_create(arr, len(self._inst), _vp(stream) if stream else None, C.byref(h))
        if st != IMEX_OK:
            raise ImexError(st, _lib.imex_batch_last_error(None).decode())
        self._h = h

    def step(self, n_steps, device_ptrs=None, tables=None):
        """device_ptrs[i]: address of instance i's n_steps + 1 f_t values on the
        device; or tables[i]: host arrays."""
        if device_ptrs is not None:
            arr = (_vp * len(device_ptrs))(*[_vp(p) for p in device_ptrs])
            on_dev = 1
        else:
            keep = [np.ascontiguousarray(t, dtype=np.float64) for t in tables]
            arr = (_vp * len(keep))(*[t.ctypes.data_as(_vp) for t in keep])
            on_dev = 0
        st = _lib.imex_batch_step(self._h, int(n_steps), arr, on_dev)
        if st != IMEX_OK:
            raise ImexError(st, _lib.imex_batch_last_error(self._h).decode())

    def form(self) -> int:
        """BATCH_KERNELS, BATCH_LANES or BATCH_GRAPH."""
        return int(_lib.imex_batch_form(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.imex_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sample_noalloc_max_points(dim: int) -> int:
    """Largest point count of Imex.sample_noalloc in dimension dim."""
    return int(_lib.imex_sample_noalloc_max_points(int(dim)))
