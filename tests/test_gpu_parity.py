"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Bar (relative 2-norm): weighted apply 1e-14, small exponential 1e-13 scaled by
dt*||T||, propagation 1e-10 for the same scheme and Krylov dimension.
Inputs come from the seeded generators; no expected value comes from the HIP
path itself.
"""
import math

import numpy as np
import pytest

from oracle import cfet as O
from oracle import schemes as S
from paper_1102_5071_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_1102_5071_amd.binding")

PROP_TOL = 1e-10
PATHS = ["multi", "single", "coop", "sell", "sell_uniform", "sell_split"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    B.load()
    yield
    torch.cuda.synchronize()


def dev(v):
    return torch.from_numpy(np.ascontiguousarray(v, dtype=np.complex128)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def run_gpu(prob_H0, Hk, drives, psi0, t0, dt, nsteps, scheme, m, path=None):
    with B.Propagator(prob_H0, Hk, drives, path=path) as P:
        psi = dev(psi0)
        P.propagate(psi, t0, dt, nsteps, scheme, m)
        out = host(psi)
        st = P.stats()
    if path is not None:
        # a persistent path whose rows do not fit falls back to the multi-kernel one
        # ("sell", "sell_uniform": the multi-kernel path on the sliced-ELL layouts)
        assert B.PATH_NAMES[st["path"]] in (path, "multi")
        if path.startswith("sell"):
            # the split layout applies to 2^b rows (b >= 8) whose far entries are shared
            want = {"sell": (1,), "sell_uniform": (2,), "sell_split": (2, 3)}[path]
            assert st["layout"] in want
            if path == "sell_split" and prob_H0.n >= 256 and is_spin_operator(prob_H0, Hk):
                assert st["layout"] == 3
        if path in ("single", "coop") and prob_H0.n <= 1024:
            assert B.PATH_NAMES[st["path"]] == path
    assert st["status"] == 0, st
    return out, st


def is_spin_operator(H0, Hk):
    """Operators on 2^L rows built from site terms (every column = row XOR a
    power of two or two adjacent powers, or the diagonal)."""
    n = H0.n
    if n & (n - 1):
        return False
    for h in [H0] + list(Hk):
        rows = np.repeat(np.arange(n), np.diff(h.row_ptr))
        off = rows ^ h.col.astype(np.int64)
        single = (off & (off - 1)) == 0
        pair = ((off // 3) & (off // 3 - 1)) == 0
        pair &= (off % 3 == 0) & (off > 0)
        if not np.all(single | pair):
            return False
    return True


def ragged_hermitian(n, seed):
    """Random sparse Hermitian matrix with empty rows and rows longer than 64."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n), dtype=complex)
    for r in range(n):
        k = rng.integers(0, 6)
        if r % 17 == 0:
            k = 0
        if r % 29 == 3:
            k = min(n, 90)
        cols = rng.choice(n, size=k, replace=False)
        A[r, cols] = rng.standard_normal(k) + 1j * rng.standard_normal(k)
    H = A + A.conj().T
    empty = np.arange(0, n, 17)
    H[empty, :] = 0
    H[:, empty] = 0
    return I._dense_to_csr(H)


# --------------------------------------------------------------------------
# weighted apply y = (a H0 + sum_k b_k H_k) x
# --------------------------------------------------------------------------
def _apply_ref(H0, Hk, a, b, x):
    y = a * (H0.to_scipy() @ x)
    for h, bk in zip(Hk, b):
        y = y + bk * (h.to_scipy() @ x)
    return y


def heisenberg_principal(L, n, seed):
    """Leading n x n block of a disordered Heisenberg chain and of sum sx: spin
    structure with a ragged last slice (flips leaving the block are dropped)."""
    rng = np.random.default_rng(seed)
    H0 = I.heisenberg_chain(L, 1.0, rng.uniform(-1, 1, L)).toarray()[:n, :n]
    H1 = I.sigma_x_sum(L).toarray()[:n, :n]
    return I._dense_to_csr(H0), I._dense_to_csr(H1)


@pytest.mark.parametrize("layout", ["multi", "sell", "sell_uniform", "sell_split"])
@pytest.mark.parametrize("case", ["ising10", "hydrogen_small", "ragged", "two_term", "heis12",
                                  "heis_block"])
def test_apply_matches_reference(case, layout):
    rng = np.random.default_rng(5)
    if case == "ising10":
        p = I.config_ising()
        H0, Hk, drives = p.H0, p.Hk, p.drives
    elif case == "hydrogen_small":
        H0, H1 = I.hydrogen_fd(300, 0.1, 7)
        Hk = [H1]
        drives = [{"kind": "cos", "A": 1.0, "omega": 1.0}]
    elif case == "ragged":
        H0 = ragged_hermitian(700, 1)
        Hk = [ragged_hermitian(700, 2)]
        drives = [{"kind": "cos", "A": 1.0, "omega": 1.0}]
    elif case == "two_term":
        H0, Hk, drives = I.noninteracting_spins(8, 0.3, 0.7, 1.1)
    elif case == "heis_block":
        H0, H1 = heisenberg_principal(10, 1000, 3)
        Hk = [H1]
        drives = [{"kind": "cos", "A": 1.0, "omega": 1.0}]
    else:
        p = I.config_heisenberg(L=12)
        H0, Hk, drives = p.H0, p.Hk, p.drives
    x = I.random_state(H0.n, rng)
    a = -0.37
    b = [0.81, -1.3][:len(Hk)]
    with B.Propagator(H0, Hk, drives, path=layout) as P:
        y = host(P.apply(dev(x), a, b))
    ref = _apply_ref(H0, Hk, a, b, x)
    assert rel(y, ref) < 1e-14


def test_sell_uniform_stores_shared_flips_once():
    # every row of sum sx holds one entry per site at column row ^ (1 << i) with
    # value 1, so each 64-row slice stores those L entries once instead of 64 times
    L = 12
    p = I.config_heisenberg(L=L)
    n, nsl = p.dim, p.dim // 64
    with B.Propagator(p.H0, p.Hk, p.drives, path="sell") as P:
        st1 = P.stats()
    with B.Propagator(p.H0, p.Hk, p.drives, path="sell_uniform") as P:
        st2 = P.stats()
    assert (st1["layout"], st2["layout"]) == (1, 2)
    assert st1["matrix_bytes"] == 20 * (p.H0.nnz + p.Hk[0].nnz) + 4 * n + 12 * nsl
    assert st2["matrix_bytes"] <= st1["matrix_bytes"] - 20 * L * n + (20 * L + 12) * nsl


# --------------------------------------------------------------------------
# small exponential exp(-i dt T) e_1
# --------------------------------------------------------------------------
def _tridiag_cases():
    # theta = |dt| h spans the tiny-theta series (< 1e-6), the expansion on the
    # Gershgorin interval (up to 256), the tightened interval above it, and
    # negative dt; m = 32 and 33 straddle the packed (two halves of one
    # wavefront) and the two-vector forms
    rng = np.random.default_rng(11)
    cases = []
    for k in (1, 2, 3, 7, 16, 24, 30, 31, 32, 33, 47, 63, 64):
        a = rng.standard_normal(k) * 3.0
        b = np.abs(rng.standard_normal(k - 1)) + 0.05
        for dt in (0.01, 1.0, 12.0, 40.0, -12.0):
            cases.append((f"rand{k}_dt{dt}", a, b, dt))
    for k in (2, 30, 33):
        a = rng.standard_normal(k)
        b = np.abs(rng.standard_normal(k - 1)) + 0.05
        cases.append((f"tiny_theta{k}", a, b, 1e-8))
    # Lanczos-like: huge spread, tiny tail couplings, near-degenerate pairs
    k = 30
    a = np.concatenate([np.linspace(-0.5, 2.0e5, k - 4), [1.0, 1.0 + 1e-12, 3.0, 3.0]])
    b = np.abs(rng.standard_normal(k - 1)) * 10 + 1e-9
    b[-3] = 1e-13
    cases.append(("spread_ghosts", a, b, 0.05))
    a = np.zeros(20)
    b = np.ones(19)
    cases.append(("zero_diag", a, b, 0.7))
    # theta = |dt| (lambda_max - lambda_min) / 2 above 7000: the diagonalisation
    # route (implicit QR) instead of the expansion; random spectra up to k = 64
    # and a Lanczos-like one (the hydrogen operator's spread at dt = 0.2)
    for k, spread, dt in ((16, 1.0e4, 0.9), (30, 1.0e4, 2.0), (47, 5.0e4, 2.0),
                          (64, 1.0e6, 1.0), (64, 2.0e4, -1.5)):
        a = rng.uniform(-spread, spread, k)
        b = np.abs(rng.standard_normal(k - 1)) * 0.1 * spread + 1.0
        cases.append((f"qr_rand{k}_s{spread:g}_dt{dt}", a, b, dt))
    k = 30
    a = np.concatenate([np.linspace(-0.5, 2.0e5, k - 4), [1.0, 1.0 + 1e-12, 3.0, 3.0]])
    b = np.abs(rng.standard_normal(k - 1)) * 10 + 1e-9
    cases.append(("qr_spread_lanczos", a, b, 0.2))
    a = np.full(10, 2.5)
    b = np.full(9, 1e-200)
    cases.append(("diagonal_limit", a, b, 0.3))
    return cases


@pytest.mark.parametrize("name,a,b,dt", _tridiag_cases(), ids=[c[0] for c in _tridiag_cases()])
def test_tridiag_exponential(name, a, b, dt):
    if name.startswith("qr_"):
        lam = np.linalg.eigvalsh(np.diag(a) + np.diag(b, 1) + np.diag(b, -1))
        assert abs(dt) * 0.5 * (lam[-1] - lam[0]) > 7000.0   # the QR route is taken
    ta = torch.tensor(a, dtype=torch.float64, device="cuda")
    tb = torch.tensor(b, dtype=torch.float64, device="cuda")
    c, status = B.tridiag_expm(ta, tb, dt)
    assert status == 0
    ref = O.tridiag_expm_e1(a, b, dt)
    scale = 1.0 + abs(dt) * (np.abs(a).max() + (np.abs(b).max() if len(b) else 0.0))
    assert np.linalg.norm(host(c) - ref) < 1e-13 * scale


# --------------------------------------------------------------------------
# full propagation
# --------------------------------------------------------------------------
@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("scheme", list(S.SCHEMES))
def test_propagate_random_all_schemes(scheme, path):
    rng = np.random.default_rng(21)
    n = 64
    H0 = I.random_hermitian(n, rng, density=0.15)
    H1 = I.random_hermitian(n, rng, density=0.15)
    H2 = I.random_hermitian(n, rng, density=0.1, real=True)
    drives = [{"kind": "cos", "A": 0.9, "omega": 1.7, "phi": 0.2},
              {"kind": "sechcos", "A": 0.5, "omega": 0.8, "phi": 0.0, "tc": 0.3, "tau": 0.7}]
    psi0 = I.random_state(n, rng)
    args = (H0, [H1, H2], drives, psi0, 0.1, 0.05, 12, scheme, 10)
    out, st = run_gpu(*args, path=path)
    ref = O.propagate(*args[:8], m=10)
    assert rel(out, ref) < PROP_TOL
    assert st["status"] == 0


def test_step_weights_match_oracle():
    p = I.config_hydrogen(Nr=50, lmax=3)
    with B.Propagator(p.H0, p.Hk, p.drives) as P:
        for scheme in S.SCHEMES:
            a, b = P.step_weights(3.0, 0.05, 7, scheme)
            sc = S.scheme(scheme)
            for n in range(7):
                ra, rb = O.step_weights(sc, p.drives, 3.0 + n * 0.05, 0.05)
                assert np.allclose(a, ra, rtol=0, atol=1e-15)
                assert np.allclose(b[n], rb, rtol=0, atol=1e-15)


@pytest.mark.parametrize("path", PATHS)
def test_ising_full_run(path):
    p = I.config_ising()          # L = 10, CF4:2, dt 0.01, 1000 steps, m 16
    out, st = run_gpu(p.H0, p.Hk, p.drives, p.psi0, 0.0, p.dt, p.nsteps, p.scheme, p.m, path)
    ref = O.propagate(p.H0, p.Hk, p.drives, p.psi0, 0.0, p.dt, p.nsteps, p.scheme, m=p.m)
    assert rel(out, ref) < PROP_TOL
    assert st["exponentials"] == 2 * p.nsteps
    assert st["matvecs"] == 2 * p.nsteps * p.m
    assert abs(np.linalg.norm(out) - 1.0) < 1e-12


@pytest.mark.parametrize("path", PATHS)
def test_hydrogen_full_size_short_run(path):
    # dim 128000, CF8:11, m 30: the benchmark's launch configuration.  The
    # table's dt = 0.05 puts dt*||H|| near 1e4, where the m = 30 Krylov step is
    # not converged and the result moves by 1e-4 under 1e-16 input noise (on
    # the oracle alone), so parity is taken at dt = 0.001, where the map is
    # well conditioned.
    p = I.config_hydrogen()
    nsteps = 6
    t0 = 40.0                     # inside the pulse
    dt = 0.001
    out, st = run_gpu(p.H0, p.Hk, p.drives, p.psi0, t0, dt, nsteps, p.scheme, p.m, path)
    ref = O.propagate(p.H0, p.Hk, p.drives, p.psi0, t0, dt, nsteps, p.scheme, m=p.m)
    assert rel(out, ref) < PROP_TOL
    assert st["matvecs"] == nsteps * 11 * p.m


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("L,nsteps", [(10, 40), (14, 4)])
def test_heisenberg_runs(L, nsteps, path):
    p = I.config_heisenberg(L=L)
    out, st = run_gpu(p.H0, p.Hk, p.drives, p.psi0, 0.0, p.dt, nsteps, p.scheme, p.m, path)
    ref = O.propagate(p.H0, p.Hk, p.drives, p.psi0, 0.0, p.dt, nsteps, p.scheme, m=p.m)
    assert rel(out, ref) < PROP_TOL


# --------------------------------------------------------------------------
# edge cases
# --------------------------------------------------------------------------
@pytest.mark.parametrize("path", PATHS)
def test_two_level_breakdown_and_closed_form(path):
    Delta, V, w = 0.5, 0.5, 1.0
    H0, Hk, drives = I.two_level(Delta, V, w)
    psi0 = np.array([1.0, 0.0], dtype=complex)
    T = 2 * math.pi
    out, st = run_gpu(H0, Hk, drives, psi0, 0.0, T / 200, 200, "CF6:5Opt", 16, path)
    ref = O.propagate(H0, Hk, drives, psi0, 0.0, T / 200, 200, "CF6:5Opt", m=16)
    assert rel(out, ref) < PROP_TOL
    assert st["min_m_eff"] == 2


@pytest.mark.parametrize("path", PATHS)
def test_zero_state_stays_zero(path):
    p = I.config_ising(L=6)
    out, st = run_gpu(p.H0, p.Hk, p.drives, np.zeros(64, complex), 0.0, 0.01, 3, "CF4:2", 8,
                      path)
    assert np.all(out == 0)


@pytest.mark.parametrize("path", PATHS)
def test_eigenvector_start(path):
    H0 = I.diagonal(np.linspace(-1, 1, 32))
    H1 = I.diagonal(np.zeros(32))
    drives = [{"kind": "cos", "A": 1.0, "omega": 1.0}]
    psi0 = np.zeros(32, complex)
    psi0[5] = 0.6 - 0.8j
    out, st = run_gpu(H0, [H1], drives, psi0, 0.0, 0.1, 5, "CF4:3Opt", 12, path)
    lam = np.linspace(-1, 1, 32)[5]
    assert abs(out[5] - psi0[5] * np.exp(-0.5j * lam)) < 1e-14
    assert st["min_m_eff"] == 1


@pytest.mark.parametrize("path", PATHS)
def test_m_larger_than_dim_and_m_one(path):
    rng = np.random.default_rng(3)
    H0 = I.random_hermitian(12, rng)
    H1 = I.random_hermitian(12, rng)
    drives = [{"kind": "cos", "A": 1.0, "omega": 2.0}]
    psi0 = I.random_state(12, rng)
    for m in (1, 40):
        out, st = run_gpu(H0, [H1], drives, psi0, 0.0, 0.02, 5, "CF4:2", m, path)
        ref = O.propagate(H0, [H1], drives, psi0, 0.0, 0.02, 5, "CF4:2", m=m)
        assert rel(out, ref) < PROP_TOL


@pytest.mark.parametrize("path", PATHS)
def test_negative_dt_and_nsteps_zero(path):
    rng = np.random.default_rng(4)
    H0 = I.random_hermitian(16, rng)
    H1 = I.random_hermitian(16, rng)
    drives = [{"kind": "cos", "A": 1.0, "omega": 2.0}]
    psi0 = I.random_state(16, rng)
    with B.Propagator(H0, [H1], drives, path=path) as P:
        psi = dev(psi0)
        P.propagate(psi, 0.0, 0.1, 0, "CF6:5Opt", 16)
        assert np.array_equal(host(psi), psi0)
        P.propagate(psi, 0.0, 0.05, 10, "CF6:5Opt", 16)     # m = n: exact exponentials
        P.propagate(psi, 0.5, -0.05, 10, "CF6:5Opt", 16)
        assert rel(host(psi), psi0) < 1e-11


@pytest.mark.parametrize("path", PATHS)
def test_piecewise_constant_drive(path):
    rng = np.random.default_rng(9)
    H0 = I.random_hermitian(40, rng, density=0.2)
    H1 = I.random_hermitian(40, rng, density=0.2)
    edges = np.linspace(0.0, 1.0, 11)
    drives = [{"kind": "pwc", "t_edges": edges, "u": rng.uniform(-1, 1, 10)}]
    psi0 = I.random_state(40, rng)
    out, _ = run_gpu(H0, [H1], drives, psi0, 0.0, 0.01, 100, "CF6:5Opt", 14, path)
    ref = O.propagate(H0, [H1], drives, psi0, 0.0, 0.01, 100, "CF6:5Opt", m=14)
    assert rel(out, ref) < PROP_TOL


@pytest.mark.parametrize("path", ["single", "coop"])
def test_profile_modes(path):
    # events only: launches timed, segment timers untouched; with segments:
    # block 0's segment times accumulate; the state is the same either way
    p = I.config_ising(L=10)
    with B.Propagator(p.H0, p.Hk, p.drives, path=path) as P:
        out = []
        for segments in (False, True):
            psi = dev(p.psi0)
            s0 = P.stats()
            P.profile(True, 64, segments=segments)
            P.propagate(psi, 0.0, p.dt, 20, p.scheme, p.m)
            s1 = P.stats()
            P.profile(False)
            assert s1["status"] == 0 and s1["timed_launches"] >= 1 and s1["timed_ms"] > 0
            grew = [a - b for a, b in zip(s1["segment_us"], s0["segment_us"])]
            assert (min(grew) > 0) if segments else (max(grew) == 0), grew
            out.append(host(psi))
    assert np.array_equal(out[0], out[1])


# --------------------------------------------------------------------------
# error handling through the ABI
# --------------------------------------------------------------------------
def test_error_codes():
    p = I.config_ising(L=4)
    bad = I.CSR(p.H0.n, p.H0.row_ptr.copy(), p.H0.col.copy(), p.H0.val.copy())
    bad.col[3] = 99
    with pytest.raises(B.CfetError) as e:
        B.Propagator(bad, p.Hk, p.drives)
    assert e.value.code == 1
    nanm = I.CSR(p.H0.n, p.H0.row_ptr.copy(), p.H0.col.copy(), p.H0.val.copy())
    nanm.val[0] = np.nan
    with pytest.raises(B.CfetError) as e:
        B.Propagator(nanm, p.Hk, p.drives)
    assert e.value.code == 4
    with B.Propagator(p.H0, p.Hk, p.drives) as P:
        psi = dev(p.psi0)
        for m in (0, 65):
            with pytest.raises(B.CfetError) as e:
                P.propagate(psi, 0.0, 0.01, 1, "CF4:2", m)
            assert e.value.code == 1
        with pytest.raises(B.CfetError) as e:       # no piecewise-constant drive
            P.gradient(psi, psi, 0.0, 0.01, 1, "CF4:2", 4, u=[0.1])
        assert e.value.code == 1
        lib = B.load()
        code = lib.cfet_propagate(P._ctx, p.psi0.ctypes.data, 0.0, 0.01, 1, 1, 4, None)
        assert code == 1                              # host pointer rejected
        code = lib.cfet_propagate(P._ctx, psi.data_ptr(), 0.0, 0.01, 1, 99, 4, None)
        assert code == 1                              # unknown scheme
