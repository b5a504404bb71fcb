"""Rows of the library's exported K^c and S against rows summed from the
oracle's element matrices of the cells around a node (helpers of the CPU and
GPU tests; no test of its own)."""
import numpy as np
import scipy.sparse as sp

from oracle import fcm


def adjacent_cells(w, g):
    """Non-empty candidate cells around grid node g (index tuples, x first)
    and g's local index in each."""
    grid = w.grid_nodes
    idx = []
    for k in range(w.dim):
        idx.append(g % grid[k])
        g //= grid[k]
    per_dim = []
    for k in range(w.dim):
        i, p = idx[k], w.p
        if i % p == 0:
            per_dim.append([(e, a) for e, a in ((i // p - 1, p), (i // p, 0)) if 0 <= e < w.n_cells[k]])
        else:
            per_dim.append([(i // p, i % p)])
    out = []
    for combo in np.ndindex(*[len(c) for c in per_dim]):
        cidx = tuple(per_dim[k][combo[k]][0] for k in range(w.dim))
        loc = sum(per_dim[k][combo[k]][1] * (w.p + 1) ** k for k in range(w.dim))
        out.append((cidx, loc))
    return out


def oracle_rows(w, g, dt, geom, flag_cache, uncut):
    """Row g of K (grid columns) and of M, from the oracle's element matrices
    of the non-empty cells around node g (dicts column -> value); flag_cache
    keeps cell flags and cut-cell matrices between calls."""
    kappa = w.rho * w.c ** 2
    Mu, Ku = uncut
    krow, mrow = {}, {}
    for cidx, loc in adjacent_cells(w, g):
        if cidx not in flag_cache:
            flag_cache[cidx] = fcm.cell_flag(w, geom, cidx)
        f = flag_cache[cidx]
        if f == fcm.EMPTY:
            continue
        nodes = [int(v) for v in fcm.cell_nodes(tuple(w.grid_nodes), w.p, cidx)]
        if f == fcm.CUT:
            key = ("cut",) + tuple(cidx)
            if key not in flag_cache:
                lo, h = fcm.cell_box(w, cidx)
                flag_cache[key] = fcm.cut_element_matrices(geom, w.p, lo, h, w.tree_depth, w.rho, kappa, w.alpha_f)
            Me, Ke = flag_cache[key]
            for j, nj in enumerate(nodes):
                mrow[nj] = mrow.get(nj, 0.0) + Me[loc, j]
        else:
            Ke = Ku
            mrow[g] = mrow.get(g, 0.0) + Mu[loc, loc]
        for j, nj in enumerate(nodes):
            krow[nj] = krow.get(nj, 0.0) + Ke[loc, j]
    return krow, mrow


def _row_err(got, want):
    keys = set(got) | set(want)
    scale = max(abs(v) for v in want.values())
    return max(abs(got.get(j, 0.0) - want.get(j, 0.0)) for j in keys) / scale


def max_row_error(w, lib, dt, rows, geom=None, beta=0.25):
    """Largest relative difference (max norm of a row, relative to its
    largest entry) between the library's K^c and S rows `rows` (c indices)
    and the oracle's: S = M^cc + beta dt^2 K^cc."""
    from paper_2310_14712_amd import imex
    geom = geom or fcm.geometry_of(w)
    inf = lib.info()
    ng = inf["n_grid"]
    cn = lib.export_index(imex.INDEX_C_NODES)
    rp, cols, vals = lib.export_csr(imex.CSR_KC)
    Kc = sp.csr_matrix((vals, cols, rp), shape=(len(cn), ng))
    rp, cols, vals = lib.export_csr(imex.CSR_S)
    S = sp.csr_matrix((vals, cols, rp), shape=(len(cn), len(cn)))
    cpos = np.full(ng, -1, dtype=np.int64)
    cpos[cn] = np.arange(len(cn))
    uncut = fcm.uncut_element_matrices(w.p, w.h, w.rho, w.rho * w.c ** 2)
    cache = {}
    worst = 0.0
    for i in rows:
        i = int(i)
        krow, mrow = oracle_rows(w, int(cn[i]), dt, geom, cache, uncut)
        want_s = {int(cpos[j]): v for j, v in mrow.items()}
        for j, v in krow.items():
            if cpos[j] >= 0:
                want_s[int(cpos[j])] = want_s.get(int(cpos[j]), 0.0) + beta * dt * dt * v
        lo, hi = Kc.indptr[i], Kc.indptr[i + 1]
        got_k = dict(zip(Kc.indices[lo:hi].tolist(), Kc.data[lo:hi].tolist()))
        lo, hi = S.indptr[i], S.indptr[i + 1]
        got_s = dict(zip(S.indices[lo:hi].tolist(), S.data[lo:hi].tolist()))
        worst = max(worst, _row_err(got_k, krow), _row_err(got_s, want_s))
    return worst
