"""The allocation-free entry point cfet_propagate_static against
cfet_propagate on the multi-kernel path (the path it takes), through the C
ABI: same result on two calls in a row, the second on a smaller problem (the
fixed device scratch keeps the first call's contents), on the three operator
stores (CSR with the library's own row order, SELL-64 with shared parts split
in two passes, CSR in the caller's order); free device memory unchanged by a
call; a problem too large for the scratch rejected before any work."""
import numpy as np
import pytest

from paper_1102_5071_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_1102_5071_amd.binding")

PROP_TOL = 1e-10


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


def problems():
    # larger first, then smaller: the second call runs on the scratch the
    # first one left
    H0, H1 = I.hydrogen_fd(400, 0.2, 15)            # 6400 rows: reordered CSR rows
    psi_h = I.hydrogen_ground_state(400, 0.2, 15)[0]
    hyd = (H0, [H1], [{"kind": "sin2cos", "A": 0.05, "omega": 0.5, "Tp": 200.0}], psi_h,
           "CF8:11", 0.002, 40.0, 4, 20, None)
    p = I.config_heisenberg(L=12, nsteps=5)          # split two-pass layout
    heis = (p.H0, p.Hk, p.drives, p.psi0, p.scheme, p.dt, 0.0, 5, p.m, "sell_split")
    q = I.config_ising(L=8, nsteps=10)               # 256 rows, CSR
    ising = (q.H0, q.Hk, q.drives, q.psi0, q.scheme, q.dt, 0.0, 10, q.m, None)
    return [hyd, heis, ising]


@pytest.mark.parametrize("order", ["large_then_small", "small_then_large"])
def test_static_scratch_matches_propagate(order):
    probs = problems()
    if order == "small_then_large":
        probs = probs[::-1]
    for (H0, Hk, drives, psi0, scheme, dt, t0, nsteps, m, layout) in probs:
        with B.Propagator(H0, Hk, drives, path="multi", layout=layout) as P:
            ref = dev(psi0)
            P.propagate(ref, t0, dt, nsteps, scheme, m)
            st_ref = P.stats()
            for call in range(2):
                psi = dev(psi0)
                torch.cuda.synchronize()
                free0 = torch.cuda.mem_get_info()[0]
                P.propagate_static(psi, t0, dt, nsteps, scheme, m)
                torch.cuda.synchronize()
                free1 = torch.cuda.mem_get_info()[0]
                st = P.stats()
                assert st["status"] == 0 and st["path"] == 1
                assert free1 == free0
                assert rel(psi.cpu().numpy(), ref.cpu().numpy()) <= PROP_TOL
            if layout == "sell_split":
                assert st["layout"] == 3
            if H0.n == 6400:
                assert st["reordered"] == 1
        assert st_ref["status"] == 0


def test_static_scratch_rejects_oversize():
    p = I.config_ising(L=20, nsteps=1)               # (64 - 1) 2^20 16 B = 1 GiB > 64 MiB
    with B.Propagator(p.H0, p.Hk, p.drives) as P:
        psi = dev(p.psi0)
        with pytest.raises(B.CfetError) as e:
            P.propagate_static(psi, 0.0, 0.01, 1, "CF4:2", 64)
        assert e.value.code == 1 and "scratch" in str(e.value)
        assert np.array_equal(psi.cpu().numpy(), p.psi0)
        # m = 2 fits (one basis vector of 16 MiB)
        P.propagate_static(psi, 0.0, 0.01, 1, "CF4:2", 2)
        assert P.stats()["status"] == 0
