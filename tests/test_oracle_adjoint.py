"""Pins of the oracle's fidelity gradient (oracle.adjoint).

* With Krylov spaces as large as the dimension every Lanczos exponential and
  the projected augmented operator are exact, so the gradient must equal the
  one assembled from dense exponentials and scipy's Frechet derivative
  (scipy.linalg.expm_frechet) of every exponential of the scheme.
* At realistic sizes (m < dim) it must agree with central finite differences
  of the oracle's own forward map (the Krylov CFET propagator), for pieces
  aligned with the steps and for pieces that cut steps.
* F is the fidelity of the forward propagator.

The second route (Arnoldi on the 2n-dimensional augmented operator
[[X, D], [0, X]] from [0; psi], route="augmented") is pinned on its own:
* with m_aug = 2 dim it equals scipy's Frechet derivative (dim <= 64);
* for commuting X and D (both diagonal) L(X, D) = D exp(X), a closed form;
* at m_aug < 2 dim its error is within the Arnoldi a-posteriori estimate.
The projected route at m < dim is then held to a bound that follows from its
construction: it is the integral over s of <a~(s)| D |b~(s)> with a~, b~ the
Lanczos approximations (same m) of exp(+i s dt H) lam and exp(-i(1-s) dt H) psi,
so its distance from the exact term is at most
||D|| (||psi|| sup_s |a~ - a| + ||lam|| sup_s |b~ - b|).
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


def _frechet_problem(n, seed, dt):
    rng = np.random.default_rng(seed)
    Hi = I.random_hermitian(n, rng, 0.3, 1.0).to_scipy()
    Hk = I.random_hermitian(n, rng, 0.3, 0.5).to_scipy()
    psi, lam = I.random_state(n, rng), I.random_state(n, rng)
    X, D = -1j * dt * Hi.toarray(), -1j * dt * Hk.toarray()
    _, Lf = sla.expm_frechet(X, D)
    return Hi, Hk, psi, lam, np.vdot(lam, Lf @ psi)


@pytest.mark.parametrize("n,seed,dt", [(8, 1, 0.7), (24, 2, 0.3), (40, 3, -0.5), (64, 4, 0.4)])
def test_augmented_route_equals_expm_frechet(n, seed, dt):
    Hi, Hk, psi, lam, exact = _frechet_problem(n, seed, dt)
    info = {}
    g, lam_b = A.frechet_term_augmented(Hi, Hk, psi, lam, dt, n, m_aug=2 * n, info=info)
    assert abs(g - exact) <= 1e-12 * abs(exact)
    # the adjoint state moves back by exp(+i dt H)
    ref = sla.expm(1j * dt * Hi.toarray()) @ lam
    assert np.linalg.norm(lam_b - ref) <= 1e-12


def test_augmented_route_commuting_closed_form():
    # X = -i dt diag(E), D = -i dt diag(c): L(X, D) = D exp(X) exactly
    rng = np.random.default_rng(9)
    n, dt = 32, 0.6
    E, c = rng.uniform(-2, 2, n), rng.uniform(-1, 1, n)
    Hi, Hk = I.diagonal(E).to_scipy(), I.diagonal(c).to_scipy()
    psi, lam = I.random_state(n, rng), I.random_state(n, rng)
    exact = np.sum(np.conj(lam) * (-1j * dt * c) * np.exp(-1j * dt * E) * psi)
    g, _ = A.frechet_term_augmented(Hi, Hk, psi, lam, dt, n, m_aug=2 * n)
    assert abs(g - exact) <= 1e-13
    g0, _ = A.frechet_term_augmented(Hi, Hk, np.zeros(n, complex), lam, dt, 8)
    assert g0 == 0.0


@pytest.mark.parametrize("m_aug", [10, 14, 18, 22])
def test_augmented_route_within_arnoldi_estimate(m_aug):
    Hi, Hk, psi, lam, exact = _frechet_problem(64, 5, 0.4)
    info = {}
    g, _ = A.frechet_term_augmented(Hi, Hk, psi, lam, 0.4, 12, m_aug=m_aug, info=info)
    assert info["k"] == m_aug
    # |<lam|top(y~ - y)>| <= ||lam|| ||y~ - y||, the estimate being of the latter
    assert abs(g - exact) <= np.linalg.norm(lam) * info["estimate"]
    assert abs(g - exact) > 1e-15        # the truncation is real at this size


@pytest.mark.parametrize("m", [5, 7, 9, 11])
def test_projected_route_within_krylov_bound(m):
    n, dt = 64, 0.4
    Hi, Hk, psi, lam, exact = _frechet_problem(n, 5, dt)
    g_aug, _ = A.frechet_term_augmented(Hi, Hk, psi, lam, dt, n, m_aug=2 * n)
    g_proj, _ = A.frechet_term(Hi, Hk, psi, lam, dt, m)
    Hd = Hi.toarray()
    ss = np.linspace(0.0, 1.0, 65)
    e_psi = max(np.linalg.norm(O.expv(Hi, psi, (1 - s) * dt, m)
                               - sla.expm(-1j * (1 - s) * dt * Hd) @ psi) for s in ss)
    e_lam = max(np.linalg.norm(O.expv(Hi, lam, -s * dt, m)
                               - sla.expm(1j * s * dt * Hd) @ lam) for s in ss)
    bound = abs(dt) * np.linalg.norm(Hk.toarray(), 2) * (
        np.linalg.norm(psi) * e_lam + np.linalg.norm(lam) * e_psi)
    assert 1e-12 < abs(g_proj - g_aug) <= 1.05 * bound
    # and the two routes at the same m agree within both estimates
    info = {}
    g_aug_m, _ = A.frechet_term_augmented(Hi, Hk, psi, lam, dt, m, info=info)
    assert abs(g_proj - g_aug_m) <= 1.05 * bound + np.linalg.norm(lam) * info["estimate"]


@pytest.mark.parametrize("scheme", ["CF4:2", "CF6:5Opt"])
def test_gradient_augmented_route_equals_dense_frechet(scheme):
    H0, H1, drives, psi0, target = small_problem(3, 5, 0.6, 0.05, 1)
    N = 12
    F, g = A.fidelity_gradient(H0, [H1], drives, psi0, target, 0.0, 0.05, N, scheme, m=8,
                               route="augmented", m_aug=16)
    Fr, gr = exact_gradient(H0, H1, drives, psi0, target, 0.0, 0.05, N, scheme)
    assert abs(F - Fr) < 1e-12
    assert np.linalg.norm(g - gr) <= 1e-11 * np.linalg.norm(gr)


def test_gradient_routes_agree_at_realistic_sizes():
    # dim 32, m = 12: both routes far from exact Krylov, both converged
    H0, H1, drives, psi0, target = small_problem(5, 8, 0.4, 0.01, 2)
    N, m = 40, 12
    _, gp = A.fidelity_gradient(H0, [H1], drives, psi0, target, 0.0, 0.01, N, "CF6:5Opt", m)
    _, ga = A.fidelity_gradient(H0, [H1], drives, psi0, target, 0.0, 0.01, N, "CF6:5Opt", m,
                                route="augmented")
    assert np.linalg.norm(gp - ga) <= 1e-11 * np.linalg.norm(ga)
    with pytest.raises(ValueError):
        A.fidelity_gradient(H0, [H1], drives, psi0, target, 0.0, 0.01, 1, "CF4:2", m,
                            route="dense")
