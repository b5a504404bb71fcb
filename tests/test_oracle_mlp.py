"""Pins of the oracle's iterative-solver and learned-preconditioner parts
(CPU): BF16 rounding, a hand-built network through the forward pass,
back-propagation against finite differences, the element-block
preconditioner against exact solves, the learned assembly at its targets
(the exact solve) and at zero (the element-block preconditioner), and the
flexible CG against a direct solve."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fcm, mlp, newmark
from paper_2310_14712_amd import inputs


def small_case(w=None):
    w = w or inputs.small_2d(n=(6, 5), p=2, holes=((0.55, 0.45, 0.23),), depth=2)
    d = fcm.assemble(w)
    ig = newmark.NewmarkImex(d.M, d.K, d.fx, d.Id, d.Ic, d.dt)
    S = ig.S.tocsr()
    return w, d, S, mlp.element_data(d, S)


def test_bf16_rounding():
    # spacing of BF16 at 1 is 2^-7; halfway cases go to the even mantissa
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -2.5, 3.0e-3, 1 + 2.0 ** -7 + 2.0 ** -9])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -6, -2.5, None, 1 + 2.0 ** -7], dtype=object)
    got = mlp.bf16(x)
    for g, w_ in zip(got, want):
        if w_ is not None:
            assert g == w_, (g, w_)
    bits = np.asarray(got, dtype=np.float32).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)
    assert abs(got[4] - 3.0e-3) <= 3.0e-3 * 2.0 ** -8


def test_element_data():
    w, d, S, ed = small_case()
    assert ed.idx.shape == (int(np.sum(d.flags == fcm.CUT)), (w.p + 1) ** 2)
    # every c dof belongs to a cut cell; the assembly counts every incidence
    assert set(np.unique(ed.idx)) == set(range(S.shape[0]))
    ones = mlp.scatter(np.ones(ed.idx.shape), ed)
    assert np.array_equal(ones, 1.0 / ed.inv_mult)
    assert ones.max() <= 4 and ones.min() >= 1
    assert np.allclose(ed.gfeat.max(axis=1), 1.0)


def test_block_preconditioner_exact_on_one_cell():
    """With a single (forced) cut cell, S is that cell's block and the
    element-block preconditioner is S^-1."""
    w = inputs.Workload(name="onecut", dim=2, n_cells=(4, 3), p=3, tree_depth=0, source=(0.1, 0.1),
                        forced_cut=np.array([5]))
    _, d, S, ed = small_case(w)
    assert ed.idx.shape[0] == 1
    r = np.random.default_rng(1).standard_normal(S.shape[0])
    z = mlp.block_precond(r, ed)
    x = spla.spsolve(S.tocsc(), r)
    assert np.linalg.norm(z - x) <= 1e-12 * np.linalg.norm(x)


def test_learned_assembly_at_targets_is_exact_solve():
    """Targets from a pair (r, S^-1 r) reassemble to the exact solution, and
    zero outputs leave the element-block step scaled by (Br.r)/(Br.S Br):
    the learned form reaches from B to S^-1.  Any outputs give a step at
    least as good as that scaled block step in the S-norm of the error."""
    _, d, S, ed = small_case()
    r = np.random.default_rng(2).standard_normal(S.shape[0])
    x = spla.spsolve(S.tocsc(), r)
    T, ok = mlp.targets(r, x, ed, mlp.pad16(ed.n_e))
    assert ok.all()
    z = mlp.apply_outputs(T, r, ed)
    assert np.linalg.norm(z - x) <= 1e-9 * np.linalg.norm(x)
    zb = mlp.block_precond(r, ed)
    scaled = (zb @ r) / (zb @ (S @ zb)) * zb
    z0 = mlp.apply_outputs(np.zeros_like(T), r, ed)
    assert np.array_equal(z0, scaled)

    def err_s(z_):
        e = x - z_
        return e @ (S @ e)

    y = np.random.default_rng(3).standard_normal(T.shape)
    assert err_s(mlp.apply_outputs(y, r, ed)) <= err_s(scaled) * (1 + 1e-12)


def test_training_rows_leave_out_negligible_residuals():
    """A cell whose local residual is below TRAIN_REL times the pair's
    largest is left out of the loss (its target would answer residuals
    elsewhere), and its target row is zero; the others keep theirs."""
    _, d, S, ed = small_case()
    r = np.random.default_rng(4).standard_normal(S.shape[0])
    r[ed.idx[0]] *= 1e-6
    x = spla.spsolve(S.tocsc(), r)
    T, ok = mlp.targets(r, x, ed, mlp.pad16(ed.n_e))
    s = np.linalg.norm(r[ed.idx], axis=1)
    assert not ok[0] and np.all(T[0] == 0.0)
    assert np.array_equal(ok, s >= mlp.TRAIN_REL * s.max())
    assert ok.sum() >= len(ok) - 4


def test_forward_is_the_hand_built_network():
    """A network whose weights are written down by hand: layer 1 splits every
    input into its positive and negative parts (rows +e_i and -e_i), layer 2
    permutes the hidden units (a non-symmetric permutation, so a transposed
    W2 would be caught), layer 3 recombines them with biases.  It computes
    y_i = x_i + beta_i for i < 8 and y_{8+i} = max(x_i + 1/2, 0) - 1/4 on
    inputs of exactly representable values, with and without the BF16
    rounding points."""
    F, H, O = 16, 32, 16
    rng = np.random.default_rng(8)
    X = rng.integers(-8, 9, size=(20, F)) / 4.0          # multiples of 1/4: exact in BF16
    perm = np.roll(np.arange(H), 3)                       # hidden unit k -> perm[k]
    W1 = np.zeros((H, F))
    b1 = np.zeros(H)
    for i in range(8):
        W1[i, i], W1[8 + i, i] = 1.0, -1.0                # relu(x), relu(-x)
        W1[16 + i, i], b1[16 + i] = 1.0, 0.5              # relu(x + 1/2)
    W2 = np.zeros((H, H))
    W2[perm, np.arange(H)] = 1.0                          # h2[perm[k]] = h1[k]
    W3 = np.zeros((O, H))
    beta = np.arange(8) / 8.0
    b3 = np.zeros(O)
    for i in range(8):
        W3[i, perm[i]], W3[i, perm[8 + i]], b3[i] = 1.0, -1.0, beta[i]
        W3[8 + i, perm[16 + i]], b3[8 + i] = 1.0, -0.25
    P = mlp.Params(W1=W1, b1=b1, W2=W2, b2=np.zeros(H), W3=W3, b3=b3)
    want = np.zeros((len(X), O))
    want[:, :8] = X[:, :8] + beta
    want[:, 8:] = np.maximum(X[:, :8] + 0.5, 0.0) - 0.25
    for bf in (False, True):
        y, _ = mlp.forward(P, X, bf)
        assert np.array_equal(y, want), bf


def random_params(ed, hidden, seed, out_scale=0.3):
    F, O = mlp.pad16(3 * ed.n_e), mlp.pad16(ed.n_e)
    p = inputs.mlp_init(F, hidden, O, seed, out_scale).astype(np.float64)
    W1, b1, W2, b2, W3, b3 = inputs.mlp_unpack(p, F, hidden, O)
    rng = np.random.default_rng(seed + 1)
    return mlp.Params(W1=W1.copy(), b1=rng.standard_normal(hidden) * 0.1, W2=W2.copy(),
                      b2=rng.standard_normal(hidden) * 0.1, W3=W3.copy(), b3=rng.standard_normal(O) * 0.1)


def test_gradients_against_finite_differences():
    """Back-propagation (FP64, no BF16 rounding) against central differences
    of the loss, for sampled entries of every parameter."""
    _, d, S, ed = small_case()
    rng = np.random.default_rng(3)
    vecs = [rng.standard_normal(S.shape[0]) for _ in range(3)]
    vecs[1][ed.idx[0]] = 0.0          # a cell with r_e = 0 is left out
    vecs = [(r, spla.spsolve(S.tocsc(), r)) for r in vecs]
    P = random_params(ed, 16, 7)
    loss, g, B = mlp.loss_and_grads(P, vecs, ed, bf=False)
    assert B == 3 * len(ed.idx) - 1
    h = 1e-6
    for name in P.names():
        arr = getattr(P, name)
        flat = arr.reshape(-1)
        for k in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[k]
            flat[k] = old + h
            lp = mlp.loss_and_grads(P, vecs, ed, bf=False)[0]
            flat[k] = old - h
            lm = mlp.loss_and_grads(P, vecs, ed, bf=False)[0]
            flat[k] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[k]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, k, fd, an)


def test_adam_step_matches_definition():
    """One Adam step from zero moments moves each parameter by lr * sign(g)
    (up to eps), the defining property of the bias-corrected first step."""
    _, d, S, ed = small_case()
    P = random_params(ed, 8, 11)
    g = {k: np.random.default_rng(5).standard_normal(getattr(P, k).shape) for k in P.names()}
    P0 = P.copy()
    mlp.adam_step(P, g, {}, lr=1e-3)
    for k in P.names():
        step = getattr(P0, k) - getattr(P, k)
        # |step - lr sign(g)| = lr eps / (|g| + eps) <= lr eps / |g|
        assert np.all(np.abs(step - 1e-3 * np.sign(g[k])) <= 1e-3 * 1e-8 / np.abs(g[k]) + 1e-15)


@pytest.mark.parametrize("which", ["jacobi", "block", "exact"])
def test_flexible_cg(which):
    _, d, S, ed = small_case()
    b = np.random.default_rng(4).standard_normal(S.shape[0])
    x_ref = spla.spsolve(S.tocsc(), b)
    prec = {"jacobi": lambda r: r / ed.diag, "block": lambda r: mlp.block_precond(r, ed),
            "exact": lambda r: spla.spsolve(S.tocsc(), r)}[which]
    x, it, ok = mlp.flexible_cg(S, b, np.zeros_like(b), prec, tol=1e-10, maxit=5000)
    assert ok
    assert np.linalg.norm(S @ x - b) <= 1e-10 * np.linalg.norm(b)
    if which == "exact":
        assert it == 1
    if which == "block":
        it_j = mlp.flexible_cg(S, b, np.zeros_like(b), lambda r: r / ed.diag, tol=1e-10, maxit=5000)[1]
        assert it < it_j


def test_flexible_cg_fallback_on_bad_preconditioner():
    """A preconditioner that points uphill is replaced by Jacobi for that
    application; the iteration still converges."""
    _, d, S, ed = small_case()
    b = np.random.default_rng(6).standard_normal(S.shape[0])
    x, it, ok = mlp.flexible_cg(S, b, np.zeros_like(b), lambda r: -r, tol=1e-10, maxit=5000,
                                fallback=lambda r: r / ed.diag)
    assert ok and np.linalg.norm(S @ x - b) <= 1e-10 * np.linalg.norm(b)
