"""GPU parity of the Chebyshev exponential path (cfet_propagate_chebyshev,
Sec. 8.1-8.2) against the oracle's Chebyshev propagator
(oracle.chebyshev.propagate_chebyshev), on every operator layout of the
multi-kernel path, and a full-size closed-form check.

Bar: relative 2-norm <= 1e-10 for the same scheme, time grid and tolerance;
the number of products (the series lengths, decided in FP64 from the same
Gershgorin intervals) equal.  The oracle itself is pinned against scipy's
expm, the harmonic oscillator of Sec. 8.2 and exact CFET exponentials.
"""
import numpy as np
import pytest

from oracle import cfet as O
from oracle import chebyshev as C
from paper_1102_5071_amd import inputs as I
from tests.closed_forms import two_level_U

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_1102_5071_amd.binding")

TOL_PARITY = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    B.load()
    yield
    torch.cuda.synchronize()


def dev(v):
    return torch.from_numpy(np.ascontiguousarray(v, dtype=np.complex128)).to("cuda")


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def case(name):
    if name == "ising8_csr":
        q = I.config_ising(L=8)
        return q.H0, q.Hk, q.drives, q.psi0, "CF4:2", 0.05, 0.0, 10, None, 0
    if name == "hydrogen_reordered":
        H0, H1 = I.hydrogen_fd(400, 0.2, 15)
        psi = I.hydrogen_ground_state(400, 0.2, 15)[0]
        return (H0, [H1], [{"kind": "sin2cos", "A": 0.05, "omega": 0.5, "Tp": 200.0}], psi,
                "CF8:11", 0.002, 40.0, 4, None, 0)
    if name.startswith("heis12_"):
        p = I.config_heisenberg(L=12)
        layout = name[len("heis12_"):]
        code = {"sell": 1, "sell_uniform": 2, "sell_split": 3}[layout]
        return p.H0, p.Hk, p.drives, p.psi0, "CF6:5Opt", 0.05, 0.3, 3, layout, code
    if name == "two_terms_negative":
        rng = np.random.default_rng(41)
        n = 40
        H0 = I.random_hermitian(n, rng, 0.3, 1.0)
        Hk = [I.random_hermitian(n, rng, 0.2, 0.5), I.random_hermitian(n, rng, 0.2, 0.7)]
        drives = [{"kind": "cos", "A": 1.3, "omega": 1.7, "phi": 0.2},
                  {"kind": "cos", "A": -0.9, "omega": 0.6, "phi": 1.0}]
        return H0, Hk, drives, I.random_state(n, rng), "CF6:5Opt", 0.1, 0.0, 5, None, 0
    if name == "two_level":
        H0, Hk, dr = I.two_level(2.0, 0.5, 1.0)
        return H0, Hk, dr, np.array([0.6, 0.8j]), "CF8:11", 0.2, 0.0, 10, None, 0
    raise KeyError(name)


CASES = ["ising8_csr", "hydrogen_reordered", "heis12_sell", "heis12_sell_uniform",
         "heis12_sell_split", "two_terms_negative", "two_level"]


@pytest.mark.parametrize("name", CASES)
def test_chebyshev_matches_oracle(name):
    H0, Hk, drives, psi0, scheme, dt, t0, N, layout, code = case(name)
    tol = 1e-12
    ost = {}
    ref = C.propagate_chebyshev(H0, Hk, drives, psi0, t0, dt, N, scheme, tol, stats=ost)
    with B.Propagator(H0, Hk, drives, layout=layout) as P:
        assert P.stats()["layout"] == code
        psi = dev(psi0)
        print(f"[chebyshev {name}] {N} steps", flush=True)
        P.propagate_chebyshev(psi, t0, dt, N, scheme, tol)
        st = P.stats()
        out = psi.cpu().numpy()
    assert st["status"] == 0 and st["path"] == 1
    assert st["exponentials"] == len(ost["terms"])
    assert st["matvecs"] == ost["n_matvec"]
    assert st["min_m_eff"] == min(ost["terms"])
    assert rel(out, ref) <= TOL_PARITY


def test_chebyshev_agrees_with_lanczos_when_both_converge():
    p = I.config_heisenberg(L=12)
    with B.Propagator(p.H0, p.Hk, p.drives) as P:
        a, b = dev(p.psi0), dev(p.psi0)
        P.propagate_chebyshev(a, 0.0, 0.05, 4, "CF6:5Opt", 1e-13)
        P.propagate(b, 0.0, 0.05, 4, "CF6:5Opt", 30)
        assert P.stats()["status"] == 0
        assert rel(a.cpu().numpy(), b.cpu().numpy()) <= 1e-11


def test_noninteracting_spins_L24_tensor_product():
    # dim 2^24 on the split layout with two driven terms: every exponential
    # factorises over the sites, so the state is the tensor product of the
    # single-spin CFET states (oracle, exact 2 x 2 exponentials); 250
    # exponentials at tol 1e-13 add at most 2.5e-11
    L, Delta, V, w = 24, 0.5, 0.5, 1.0
    dt, nsteps, scheme = 0.02, 50, "CF6:5Opt"
    H0, Hk, drives = I.noninteracting_spins(L, Delta, V, w)
    rng = np.random.default_rng(7)
    sites = []
    for _ in range(L):
        v = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        sites.append(v / np.linalg.norm(v))
    psi0 = I.product_state(sites)
    with B.Propagator(H0, Hk, drives) as P:
        assert P.stats()["layout"] == 3
        psi = dev(psi0)
        del psi0
        P.propagate_chebyshev(psi, 0.0, dt, nsteps, scheme, 1e-13)
        st = P.stats()
        out = psi.cpu().numpy()
    del psi
    assert st["status"] == 0 and st["exponentials"] == nsteps * 5
    h0, hk, dr = I.two_level(Delta, V, w)
    cfet_sites = [O.propagate(h0, hk, dr, phi, 0.0, dt, nsteps, scheme, dense=True)
                  for phi in sites]
    ref = I.product_state(cfet_sites)
    assert rel(out, ref) <= TOL_PARITY


def test_chebyshev_argument_errors():
    q = I.config_ising(L=4)
    with B.Propagator(q.H0, q.Hk, q.drives) as P:
        x = dev(q.psi0)
        for tol in (0.0, 1.0, -1e-3, float("nan")):
            with pytest.raises(B.CfetError) as e:
                P.propagate_chebyshev(x, 0.0, 0.01, 1, "CF4:2", tol)
            assert e.value.code == 1
        P.propagate_chebyshev(x, 0.0, 0.01, 0, "CF4:2", 1e-12)   # no steps: no-op
        assert np.array_equal(x.cpu().numpy(), q.psi0)
