"""Pins of the oracle's local time-stepping leap-frog (substepping of the
cut-cell dofs with dt / m; oracle/newmark.py lts_leapfrog_run), on small
meshes with a hole and the HRZ-lumped cut-cell mass:

* m = 1 is the central difference method on all dofs (the Newmark loop with
  beta = 0 on the c block), step for step;
* with no load the scheme conserves the discrete energy
  1/2 |v_{n+1/2}|_M^2 + 1/2 u_{n+1}^T M B u_n (B the scheme's operator,
  u_{n+1} = 2 u_n - u_{n-1} - dt^2 B u_n), which holds only if M B is
  symmetric, i.e. if the substeps are weighted as the definition says;
* stability: the two conditions the paper gives for the substepping scheme
  (Section "Perforated plate"), dt_coarse < dt_crit^uncut and dt_coarse / m
  < dt_crit^cut, taken as the exact critical steps of the uncut and cut
  blocks, bound the stable coarse step: bounded at 0.99 of the smaller one
  and growing at 1.01 of it;
* second-order convergence in dt towards a fine run.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import fcm, newmark
from paper_2310_14712_amd import inputs


def hole_case(n=(6, 5), p=2):
    w = inputs.small_2d(n=n, p=p, holes=((0.55, 0.45, 0.23),), depth=3)
    w.cut_mass = "hrz"
    d = fcm.assemble(w)
    act = d.active
    M = sp.csr_matrix(newmark.imex_mass(d.M, d.Id, d.Ic))[act][:, act]
    K = sp.csr_matrix(d.K)[act][:, act]
    pos = {int(g): i for i, g in enumerate(act)}
    fine = np.array([pos[int(g)] for g in d.Ic])
    coarse = np.array([pos[int(g)] for g in d.Id])
    return w, d, M, K, d.fx[act], fine, coarse


def block_limits(M, K, fine, coarse):
    """Exact critical steps of the uncut (coarse) and cut (fine) blocks."""
    Md, Kd = M.toarray(), K.toarray()
    lam_d = sla.eigh(Kd[np.ix_(coarse, coarse)], Md[np.ix_(coarse, coarse)], eigvals_only=True)[-1]
    lam_c = sla.eigh(Kd[np.ix_(fine, fine)], Md[np.ix_(fine, fine)], eigvals_only=True)[-1]
    return 2.0 / np.sqrt(lam_d), 2.0 / np.sqrt(lam_c)


def test_m1_is_central_differences():
    w, d, M, K, fx, fine, coarse = hole_case()
    dt = 0.9 * block_limits(M, K, fine, coarse)[1]
    n = 60
    ft = inputs.ft_table(dt, n, 10.0) + 0.3
    rng = np.random.default_rng(1)
    u0, v0 = rng.standard_normal(len(fx)), rng.standard_normal(len(fx))
    u = newmark.lts_leapfrog_run(M, K, fx, ft, fine, u0, v0, dt, 1, n)
    # the Newmark loop with beta = 0 on the c block, on the same dofs
    ig = newmark.NewmarkImex(M, K, fx, coarse, fine, dt, beta=0.0)
    st = ig.run(ig.initial_state(u0, v0, ft[0]), ft, n)
    assert np.linalg.norm(u - st.u) <= 1e-12 * np.linalg.norm(st.u)


@pytest.mark.parametrize("m", [1, 3, 8])
def test_energy_conserved(m):
    w, d, M, K, fx, fine, coarse = hole_case()
    dt_d, dt_c = block_limits(M, K, fine, coarse)
    dt = 0.9 * min(dt_d, m * dt_c)
    B = newmark.lts_operator(M, K, fine, dt, m)
    Md = M.toarray()
    MB = Md @ B
    assert np.allclose(MB, MB.T, rtol=0, atol=1e-10 * np.abs(MB).max())
    rng = np.random.default_rng(2)
    u0, v0 = rng.standard_normal(len(fx)), rng.standard_normal(len(fx))
    energies = []

    def cb(k, up, u):
        v = (u - up) / dt
        energies.append(0.5 * v @ (Md @ v) + 0.5 * u @ (MB @ up))

    ft = np.zeros(401)
    newmark.lts_leapfrog_run(M, K, fx, ft, fine, u0, v0, dt, m, 400, callback=cb)
    e = np.array(energies)
    assert np.max(np.abs(e - e[0])) <= 1e-11 * abs(e[0])


@pytest.mark.parametrize("m", [1, 2, 4, 12])
def test_stability_limits(m):
    """Bounded at 0.99 x min(dt_crit^uncut, m dt_crit^cut) over 3000 steps and
    growing at 1.01 x (exact block limits; HRZ-lumped cut cells)."""
    w, d, M, K, fx, fine, coarse = hole_case()
    dt_d, dt_c = block_limits(M, K, fine, coarse)
    dt_lim = min(dt_d, m * dt_c)
    rng = np.random.default_rng(3)
    u0 = rng.standard_normal(len(fx))
    ft = np.zeros(3001)
    amp = {}
    for f in (0.99, 1.01):
        with np.errstate(over="ignore", invalid="ignore"):
            u = newmark.lts_leapfrog_run(M, K, fx, ft, fine, u0, np.zeros_like(u0), f * dt_lim, m, 3000)
            amp[f] = np.linalg.norm(u) / np.linalg.norm(u0)
    assert amp[0.99] < 10.0, amp
    assert not amp[1.01] <= 1e3, amp          # grows (or overflows)


def test_second_order_convergence():
    w, d, M, K, fx, fine, coarse = hole_case()
    dt_d, dt_c = block_limits(M, K, fine, coarse)
    m, T = 4, 0.2
    rng = np.random.default_rng(4)
    u0 = np.zeros(len(fx))
    v0 = np.zeros(len(fx))

    def run(nsteps):
        dt = T / nsteps
        t = np.arange(nsteps + 1) * dt
        ft = np.sin(20.0 * t) ** 2
        return newmark.lts_leapfrog_run(M, K, fx, ft, fine, u0, v0, dt, m, nsteps)

    n0 = int(np.ceil(T / (0.5 * min(dt_d, m * dt_c))))
    ref = run(16 * n0)
    errs = [np.linalg.norm(run(k * n0) - ref) for k in (1, 2, 4)]
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0, errs
