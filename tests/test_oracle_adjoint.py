"""Pins of the oracle's fidelity gradient (oracle.adjoint).

* With Krylov spaces as large as the dimension every Lanczos exponential and
  the projected augmented operator are exact, so the gradient must equal the
  one assembled from dense exponentials and scipy's Frechet derivative
  (scipy.linalg.expm_frechet) of every exponential of the scheme.
* At realistic sizes (m < dim) it must agree with central finite differences
  of the oracle's own forward map (the Krylov CFET propagator), for pieces
  aligned with the steps and for pieces that cut steps.
* F is the fidelity of the forward propagator.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import adjoint as A
from oracle import cfet as O
from oracle import schemes as S
from paper_1102_5071_amd import inputs as I


def small_problem(L, K, T, dt, seed, edges=None):
    rng = np.random.default_rng(seed)
    h = rng.uniform(-0.5, 0.5, L)
    u = rng.uniform(-1, 1, K)
    H0 = I.ising_chain(L, 1.0, h)
    H1 = I.sigma_x_sum(L)
    if edges is None:
        edges = np.linspace(0.0, T, K + 1)
    drives = [{"kind": "pwc", "t_edges": np.asarray(edges, float), "u": u}]
    psi0 = I.random_state(1 << L, rng)
    target = I.random_state(1 << L, rng)
    return H0, H1, drives, psi0, target


def exact_gradient(H0, H1, drives, psi0, target, t0, dt, N, scheme):
    """Dense reference: exact exponentials, scipy's expm_frechet per exponential."""
    sc = S.scheme(scheme)
    H0d, H1d = H0.toarray(), H1.toarray()
    d = drives[0]
    K = len(d["u"])
    states, ops = [], []
    psi = psi0.astype(complex)
    for n in range(N):
        t_n = t0 + n * dt
        a, b = O.step_weights(sc, drives, t_n, dt)
        db = A.weight_derivatives(sc, d, t_n, dt)
        for i in range(sc.s - 1, -1, -1):
            Om = -1j * dt * (a[i] * H0d + b[i, 0] * H1d)
            states.append(psi.copy())
            ops.append((Om, db[i]))
            psi = sla.expm(Om) @ psi
    z = np.vdot(target, psi)
    lam = target.astype(complex)
    dz = np.zeros(K, complex)
    for psi_b, (Om, dbi) in zip(reversed(states), reversed(ops)):
        E, L = sla.expm_frechet(Om, -1j * dt * H1d)
        g = np.vdot(lam, L @ psi_b)
        for p, w in dbi.items():
            dz[p] += w * g
        lam = E.conj().T @ lam
    return abs(z) ** 2, 2 * np.real(np.conj(z) * dz)


@pytest.mark.parametrize("scheme", ["CF4:2", "CF6:5Opt", "CF4:3"])
def test_equals_dense_frechet_when_krylov_is_exact(scheme):
    H0, H1, drives, psi0, target = small_problem(3, 5, 0.6, 0.05, 1)
    N = 12
    F, g = A.fidelity_gradient(H0, [H1], drives, psi0, target, 0.0, 0.05, N, scheme, m=8)
    Fr, gr = exact_gradient(H0, H1, drives, psi0, target, 0.0, 0.05, N, scheme)
    assert abs(F - Fr) < 1e-12
    assert np.linalg.norm(g - gr) <= 1e-11 * np.linalg.norm(gr)


def _fd(H0, H1, drives, psi0, target, t0, dt, N, scheme, m, h=1e-4, idx=None):
    u = drives[0]["u"]
    out = {}
    for p in (range(len(u)) if idx is None else idx):
        vals = []
        for sgn in (+1, -1):
            d2 = dict(drives[0])
            d2["u"] = u.copy()
            d2["u"][p] += sgn * h
            vals.append(A.fidelity(H0, [H1], [d2], psi0, target, t0, dt, N, scheme, m))
        out[p] = (vals[0] - vals[1]) / (2 * h)
    return out


def test_matches_finite_differences_aligned():
    H0, H1, drives, psi0, target = small_problem(5, 8, 0.4, 0.01, 2)
    N, m = 40, 12
    F, g = A.fidelity_gradient(H0, [H1], drives, psi0, target, 0.0, 0.01, N, "CF6:5Opt", m)
    # h = 1e-4 balances the O(h^2) truncation against rounding in F (about
    # 1e-15 after 200 exponentials, divided by h); h = 1e-6 is rounding-limited
    fd = _fd(H0, H1, drives, psi0, target, 0.0, 0.01, N, "CF6:5Opt", m)
    scale = np.max(np.abs(g))
    for p, v in fd.items():
        assert abs(v - g[p]) <= 2e-8 * scale, (p, v, g[p])
    fd6 = _fd(H0, H1, drives, psi0, target, 0.0, 0.01, N, "CF6:5Opt", m, h=1e-6, idx=[0, 5])
    for p, v in fd6.items():
        assert abs(v - g[p]) <= 5e-6 * scale, (p, v, g[p])
    assert abs(F - A.fidelity(H0, [H1], drives, psi0, target, 0.0, 0.01, N, "CF6:5Opt", m)) < 1e-15


def test_matches_finite_differences_pieces_cut_steps():
    # piece edges that fall inside steps, between Gauss points
    edges = [0.0, 0.0137, 0.05, 0.0731, 0.1, 0.2]
    H0, H1, drives, psi0, target = small_problem(4, 5, None, 0.02, 3, edges=edges)
    N, m = 10, 10
    F, g = A.fidelity_gradient(H0, [H1], drives, psi0, target, 0.0, 0.02, N, "CF4:2", m)
    fd = _fd(H0, H1, drives, psi0, target, 0.0, 0.02, N, "CF4:2", m)
    scale = np.max(np.abs(g))
    for p, v in fd.items():
        assert abs(v - g[p]) <= 2e-8 * scale, (p, v, g[p])


def test_pieces_after_the_window_have_zero_gradient():
    edges = [0.0, 0.1, 0.2, 5.0, 6.0]
    H0, H1, drives, psi0, target = small_problem(3, 4, None, 0.05, 4, edges=edges)
    F, g = A.fidelity_gradient(H0, [H1], drives, psi0, target, 0.0, 0.05, 8, "CF4:2", 8)
    assert g[3] == 0.0 and g[0] != 0.0


def test_weight_derivatives_sum_to_a_when_aligned():
    # a step inside one piece: sum_m g_{i,m} = a_i (Sec. 7 with f = 1)
    sc = S.scheme("CF8:11")
    d = {"kind": "pwc", "t_edges": np.array([0.0, 1.0]), "u": np.array([0.3])}
    db = A.weight_derivatives(sc, d, 0.2, 0.05)
    a, _ = O.step_weights(sc, [d], 0.2, 0.05)
    for i in range(sc.s):
        assert abs(db[i][0] - a[i]) < 1e-15


def test_adjoint_config_recipe():
    p = I.config_adjoint(L=6, K=20, T=2.0)
    assert p.nsteps == 200 and p.scheme == "CF6:5Opt" and p.m == 20
    d = p.drives[0]
    assert len(d["u"]) == 20 and np.all(np.abs(d["u"]) <= 1)
    assert abs(np.linalg.norm(p.meta["target"]) - 1) < 1e-14
