"""Seeded synthetic inputs: Hamiltonians in CSR, drive parameters, initial states.

This module is the only code shared by the HIP path's tests/benchmarks and the
CPU oracle.  It holds problem *definitions* only (matrix entries of the model
Hamiltonians, drive parameters, initial states) and none of the propagation
method's arithmetic: no coefficient tables, quadrature, Krylov or exponential.

Conventions
-----------
* Spin chains: basis index bit i <-> site i, bit value 0 = spin up
  (sigma_z eigenvalue +1), so "all spins up" is basis vector e_0.  Operators
  are Pauli matrices (sigma, not S = sigma/2), sigma_z = diag(1, -1), as in the
  two-level system of the paper's Sec. 6.2.
* CSR arrays: row_ptr int64[n+1], col int32[nnz], val complex128[nnz].  Entries
  of a row are stored in generation order (diagonal first, then off-diagonal
  terms in site/bond order); columns are not sorted.
* Drives are dicts understood by both sides:
    {'kind': 'cos',     'A', 'omega', 'phi'}
    {'kind': 'sin2cos', 'A', 'omega', 'phi', 'Tp'}
    {'kind': 'pwc',     't_edges', 'u'}
    {'kind': 'sechcos', 'A', 'omega', 'phi', 'tc', 'tau'}
* Random numbers: numpy.random.default_rng(seed); fields h_i are drawn first,
  then any per-instance parameters, then state-related draws.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["CSR", "Problem", "ising_chain", "heisenberg_chain", "sigma_x_sum",
           "sigma_y_sum", "hydrogen_fd", "two_level", "noninteracting_spins",
           "random_hermitian", "diagonal", "product_state", "random_state",
           "config_ising", "config_hydrogen", "config_heisenberg", "CONFIGS"]


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray   # int64[n+1]
    col: np.ndarray       # int32[nnz]
    val: np.ndarray       # complex128[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        """A scipy CSR copy (its arrays share no memory with this container:
        scipy sorts a non-canonical matrix's entries in place on some
        operations, e.g. abs(), which would reorder the values here alone)."""
        import scipy.sparse as sp
        return sp.csr_matrix((self.val.copy(), self.col.astype(np.int64),
                              self.row_ptr.copy()), shape=(self.n, self.n))

    def toarray(self):
        return self.to_scipy().toarray()

    def row(self, r: int):
        a, b = int(self.row_ptr[r]), int(self.row_ptr[r + 1])
        return self.col[a:b], self.val[a:b]


@dataclass
class Problem:
    """H(t) = H0 + sum_k f_k(t) Hk[k], initial state psi0 and run parameters."""
    name: str
    H0: CSR
    Hk: list
    drives: list
    psi0: np.ndarray
    scheme: str = "CF4:2"
    dt: float = 0.01
    nsteps: int = 1
    m: int = 16
    t0: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return self.H0.n


def _from_lists(n, counts, fill):
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.complex128)
    fill(row_ptr, col, val)
    return CSR(n, row_ptr, col, val)


def _spin_z(idx, i):
    # sigma_z eigenvalue of site i: +1 for bit 0, -1 for bit 1
    return (1 - 2 * ((idx >> i) & 1)).astype(np.float64)


def sigma_x_sum(L: int, coeff=None) -> CSR:
    """sum_i c_i sigma_x^(i): one entry per site and row, column = row ^ (1 << i)."""
    n = 1 << L
    c = np.ones(L) if coeff is None else np.asarray(coeff, dtype=np.float64)
    idx = np.arange(n, dtype=np.int64)

    def fill(row_ptr, col, val):
        base = row_ptr[:-1]
        for i in range(L):
            col[base + i] = (idx ^ (1 << i)).astype(np.int32)
            val[base + i] = c[i]
    return _from_lists(n, np.full(n, L, dtype=np.int64), fill)


def sigma_y_sum(L: int, coeff=None) -> CSR:
    """sum_i c_i sigma_y^(i).  <r|sigma_y|c> with c = r ^ (1<<i) is +i when site
    i of r is down (bit 1) and -i when it is up (bit 0)."""
    n = 1 << L
    c = np.ones(L) if coeff is None else np.asarray(coeff, dtype=np.float64)
    idx = np.arange(n, dtype=np.int64)

    def fill(row_ptr, col, val):
        base = row_ptr[:-1]
        for i in range(L):
            col[base + i] = (idx ^ (1 << i)).astype(np.int32)
            bit = (idx >> i) & 1
            val[base + i] = np.where(bit == 1, 1j, -1j) * c[i]
    return _from_lists(n, np.full(n, L, dtype=np.int64), fill)


def ising_chain(L: int, J: float, h) -> CSR:
    """H0 = sum_i J sz_i sz_{i+1} (open chain) + sum_i h_i sz_i (diagonal)."""
    n = 1 << L
    idx = np.arange(n, dtype=np.int64)
    d = np.zeros(n)
    for i in range(L - 1):
        d += J * _spin_z(idx, i) * _spin_z(idx, i + 1)
    for i in range(L):
        d += h[i] * _spin_z(idx, i)

    def fill(row_ptr, col, val):
        col[:] = idx.astype(np.int32)
        val[:] = d
    return _from_lists(n, np.ones(n, dtype=np.int64), fill)


def heisenberg_chain(L: int, J: float, h) -> CSR:
    """H0 = J sum_i (sx sx + sy sy + sz sz)_{i,i+1} (open chain) + sum_i h_i sz_i.
    sx sx + sy sy = 2 (s+ s- + s- s+) couples anti-aligned neighbours with 2J."""
    n = 1 << L
    idx = np.arange(n, dtype=np.int64)
    d = np.zeros(n)
    for i in range(L - 1):
        d += J * _spin_z(idx, i) * _spin_z(idx, i + 1)
    for i in range(L):
        d += h[i] * _spin_z(idx, i)
    counts = np.ones(n, dtype=np.int64)
    for i in range(L - 1):
        counts += ((idx >> i) ^ (idx >> (i + 1))) & 1

    def fill(row_ptr, col, val):
        pos = row_ptr[:-1].copy()
        col[pos] = idx.astype(np.int32)
        val[pos] = d
        pos += 1
        for i in range(L - 1):
            anti = (((idx >> i) ^ (idx >> (i + 1))) & 1).astype(bool)
            p = pos[anti]
            col[p] = (idx[anti] ^ (3 << i)).astype(np.int32)
            val[p] = 2.0 * J
            pos[anti] += 1
    return _from_lists(n, counts, fill)


def diagonal(values) -> CSR:
    v = np.asarray(values, dtype=np.complex128)
    n = len(v)
    return CSR(n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), v.copy())


def _dense_to_csr(Hd) -> CSR:
    Hd = np.asarray(Hd, dtype=np.complex128)
    n = Hd.shape[0]
    rows, cols = np.nonzero(Hd)
    counts = np.bincount(rows, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n, row_ptr, cols.astype(np.int32), Hd[rows, cols].copy())


def random_hermitian(n: int, rng, density: float = 1.0, scale: float = 1.0,
                     real: bool = False) -> CSR:
    """Random Hermitian matrix (complex Gaussian entries, optional sparsity)."""
    if real:
        A = rng.standard_normal((n, n))
    else:
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    if density < 1.0:
        mask = rng.random((n, n)) < density
        mask = mask | mask.T
        np.fill_diagonal(mask, True)
        A = A * mask
    H = 0.5 * scale * (A + A.conj().T)
    return _dense_to_csr(H)


def hydrogen_fd(Nr: int = 2000, dr: float = 0.1, lmax: int = 63):
    """Radial finite-difference hydrogen-like atom, m = 0 sector.

    Index = l*Nr + (i-1), r_i = i*dr (i = 1..Nr), Dirichlet ends.
    H0 (block diagonal in l, tridiagonal blocks):
        diag 1/dr^2 + l(l+1)/(2 r_i^2) - 1/r_i, off-diagonal -1/(2 dr^2).
    H1 = r cos(theta): couples (l, i) <-> (l+1, i) with
        r_i (l+1)/sqrt((2l+1)(2l+3)).
    Returns (H0, H1).
    """
    nl = lmax + 1
    n = nl * Nr
    r = dr * np.arange(1, Nr + 1, dtype=np.float64)
    # H0: per row the diagonal, then left and right neighbours inside the block
    i_loc = np.tile(np.arange(Nr), nl)
    l_of = np.repeat(np.arange(nl), Nr)
    counts0 = 1 + (i_loc > 0) + (i_loc < Nr - 1)
    rr = r[i_loc]
    d = 1.0 / dr ** 2 + l_of * (l_of + 1) / (2.0 * rr * rr) - 1.0 / rr
    off = -0.5 / dr ** 2
    rows = np.arange(n, dtype=np.int64)

    def fill0(row_ptr, col, val):
        pos = row_ptr[:-1].copy()
        col[pos] = rows.astype(np.int32)
        val[pos] = d
        pos += 1
        m = i_loc > 0
        col[pos[m]] = (rows[m] - 1).astype(np.int32)
        val[pos[m]] = off
        pos[m] += 1
        m = i_loc < Nr - 1
        col[pos[m]] = (rows[m] + 1).astype(np.int32)
        val[pos[m]] = off
        pos[m] += 1
    H0 = _from_lists(n, counts0.astype(np.int64), fill0)

    def coup(l):
        return (l + 1) / math.sqrt((2 * l + 1) * (2 * l + 3))
    cl = np.array([coup(l) for l in range(nl)])
    counts1 = (l_of > 0).astype(np.int64) + (l_of < nl - 1)

    def fill1(row_ptr, col, val):
        pos = row_ptr[:-1].copy()
        m = l_of > 0           # coupling to l-1
        col[pos[m]] = (rows[m] - Nr).astype(np.int32)
        val[pos[m]] = rr[m] * cl[l_of[m] - 1]
        pos[m] += 1
        m = l_of < nl - 1      # coupling to l+1
        col[pos[m]] = (rows[m] + Nr).astype(np.int32)
        val[pos[m]] = rr[m] * cl[l_of[m]]
        pos[m] += 1
    H1 = _from_lists(n, counts1, fill1)
    return H0, H1


def hydrogen_ground_state(Nr: int = 2000, dr: float = 0.1, lmax: int = 63):
    """Lowest eigenvector of the l = 0 block, normalised, positive sum."""
    from scipy.linalg import eigh_tridiagonal
    r = dr * np.arange(1, Nr + 1, dtype=np.float64)
    d = 1.0 / dr ** 2 - 1.0 / r
    e = np.full(Nr - 1, -0.5 / dr ** 2)
    w, v = eigh_tridiagonal(d, e, select="i", select_range=(0, 0))
    g = v[:, 0]
    g = g / np.linalg.norm(g)
    if g.sum() < 0:
        g = -g
    psi = np.zeros((lmax + 1) * Nr, dtype=np.complex128)
    psi[:Nr] = g
    return psi, float(w[0])


def two_level(Delta: float, V: float, omega: float):
    """H(t) = [[Delta, V e^{-2iwt}], [V e^{2iwt}, -Delta]]  (Sec. 6.2, eq. TwoLevelH)
    written as Delta sz + V cos(2wt) sx + V sin(2wt) sy."""
    H0 = diagonal([Delta, -Delta])
    Hx = _dense_to_csr(np.array([[0, 1], [1, 0]], dtype=complex))
    Hy = _dense_to_csr(np.array([[0, -1j], [1j, 0]], dtype=complex))
    drives = [{"kind": "cos", "A": V, "omega": 2 * omega, "phi": 0.0},
              {"kind": "cos", "A": V, "omega": 2 * omega, "phi": -math.pi / 2}]
    return H0, [Hx, Hy], drives


def noninteracting_spins(L: int, Delta: float, V: float, omega: float):
    """sum_i [Delta sz_i + V cos(2wt) sx_i + V sin(2wt) sy_i]: L copies of the
    circularly driven two-level system, no coupling."""
    n = 1 << L
    idx = np.arange(n, dtype=np.int64)
    d = np.zeros(n)
    for i in range(L):
        d += Delta * _spin_z(idx, i)

    def fill(row_ptr, col, val):
        col[:] = idx.astype(np.int32)
        val[:] = d
    H0 = _from_lists(n, np.ones(n, dtype=np.int64), fill)
    drives = [{"kind": "cos", "A": V, "omega": 2 * omega, "phi": 0.0},
              {"kind": "cos", "A": V, "omega": 2 * omega, "phi": -math.pi / 2}]
    return H0, [sigma_x_sum(L), sigma_y_sum(L)], drives


def product_state(site_states) -> np.ndarray:
    """Kronecker product with site 0 as the least significant bit."""
    psi = np.ones(1, dtype=np.complex128)
    for phi in site_states:           # site 0 first
        psi = np.kron(np.asarray(phi, dtype=np.complex128), psi)
    return psi


def random_product_state(L: int, rng) -> np.ndarray:
    sites = []
    for _ in range(L):
        v = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        sites.append(v / np.linalg.norm(v))
    return product_state(sites)


def random_state(n: int, rng) -> np.ndarray:
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return v / np.linalg.norm(v)


def basis_state(n: int, k: int = 0) -> np.ndarray:
    v = np.zeros(n, dtype=np.complex128)
    v[k] = 1.0
    return v


# --------------------------------------------------------------------------
# the three plain workloads
# --------------------------------------------------------------------------
def config_ising(L: int = 10, seed: int = 0, nsteps: int = 1000) -> Problem:
    """Driven Ising chain: J = 1, h_i ~ U[-0.5, 0.5], H1 = sum sx,
    f = 0.8 cos(2t), psi0 = all up, CF4:2, dt = 0.01, m = 16."""
    rng = np.random.default_rng(seed)
    h = rng.uniform(-0.5, 0.5, L)
    H0 = ising_chain(L, 1.0, h)
    H1 = sigma_x_sum(L)
    drives = [{"kind": "cos", "A": 0.8, "omega": 2.0, "phi": 0.0}]
    return Problem(f"ising-L{L}", H0, [H1], drives, basis_state(1 << L, 0),
                   scheme="CF4:2", dt=0.01, nsteps=nsteps, m=16,
                   meta={"L": L, "h": h, "seed": seed})


def config_hydrogen(Nr: int = 2000, dr: float = 0.1, lmax: int = 63,
                    nsteps: int = 4000) -> Problem:
    """Hydrogen-like atom on a radial grid in a pulsed field:
    f = 0.05 sin^2(pi t/200) cos(0.5 t), psi0 = 1s, CF8:11, dt = 0.05, m = 30."""
    H0, H1 = hydrogen_fd(Nr, dr, lmax)
    psi0, e0 = hydrogen_ground_state(Nr, dr, lmax)
    drives = [{"kind": "sin2cos", "A": 0.05, "omega": 0.5, "phi": 0.0, "Tp": 200.0}]
    return Problem(f"hydrogen-Nr{Nr}-l{lmax}", H0, [H1], drives, psi0,
                   scheme="CF8:11", dt=0.05, nsteps=nsteps, m=30,
                   meta={"Nr": Nr, "dr": dr, "lmax": lmax, "E0": e0})


def config_heisenberg(L: int = 24, seed: int = 0, nsteps: int = 200) -> Problem:
    """Disordered Heisenberg chain: J = 1, h_i ~ U[-1, 1], H1 = sum sx,
    f = 0.5 sin(1.3 t), random product psi0, CF6:5Opt, dt = 0.02, m = 24."""
    rng = np.random.default_rng(seed)
    h = rng.uniform(-1.0, 1.0, L)
    H0 = heisenberg_chain(L, 1.0, h)
    H1 = sigma_x_sum(L)
    psi0 = random_product_state(L, rng)
    drives = [{"kind": "cos", "A": 0.5, "omega": 1.3, "phi": -math.pi / 2}]
    return Problem(f"heisenberg-L{L}", H0, [H1], drives, psi0,
                   scheme="CF6:5Opt", dt=0.02, nsteps=nsteps, m=24,
                   meta={"L": L, "h": h, "seed": seed})


@dataclass
class Batch:
    """Independent trajectories sharing one scheme, time grid and Krylov
    bound.  ops: list of CSR operators; each instance names its H0 and driven
    terms by index into ops (so a term shared by many instances is stored once)
    and carries its own drives and initial state."""
    name: str
    ops: list
    instances: list          # dicts: h0 (int), hk (list of int), drives, psi0
    scheme: str = "CF4:2"
    dt: float = 0.01
    nsteps: int = 500
    m: int = 32
    tol: float = 1e-10
    t0: float = 0.0
    meta: dict = field(default_factory=dict)

    def dims(self):
        return [self.ops[i["h0"]].n for i in self.instances]

    def oracle_instances(self):
        """The instances with operators resolved (H0, Hk matrices)."""
        return [{"H0": self.ops[i["h0"]], "Hk": [self.ops[k] for k in i["hk"]],
                 "drives": i["drives"], "psi0": i["psi0"]} for i in self.instances]


def config_batched(n_traj: int = 256, L_min: int = 12, L_max: int = 18, seed: int = 0,
                   nsteps: int = 500) -> Batch:
    """Many driven Ising chains in one batch: for each trajectory, in order,
    L ~ U{L_min..L_max}, A ~ U[0.2, 1.5], omega ~ U[0.5, 3], then h_i ~ U[-1, 1]
    (i < L); J = 1, H1 = sum sx (one operator per L, shared), f = A cos(omega t),
    psi0 = all up.  CF4:2, dt = 0.01, adaptive m <= 32 at tol 1e-10."""
    rng = np.random.default_rng(seed)
    ops = []
    sx_index = {}
    instances = []
    for _ in range(n_traj):
        L = int(rng.integers(L_min, L_max + 1))
        A = float(rng.uniform(0.2, 1.5))
        omega = float(rng.uniform(0.5, 3.0))
        h = rng.uniform(-1.0, 1.0, L)
        if L not in sx_index:
            sx_index[L] = len(ops)
            ops.append(sigma_x_sum(L))
        ops.append(ising_chain(L, 1.0, h))
        instances.append({"h0": len(ops) - 1, "hk": [sx_index[L]],
                          "drives": [{"kind": "cos", "A": A, "omega": omega, "phi": 0.0}],
                          "psi0": basis_state(1 << L, 0), "L": L})
    return Batch(f"batched-{n_traj}x-ising-L{L_min}-{L_max}", ops, instances,
                 scheme="CF4:2", dt=0.01, nsteps=nsteps, m=32, tol=1e-10,
                 meta={"seed": seed, "L_min": L_min, "L_max": L_max})


def config_adjoint(L: int = 14, K: int = 200, T: float = 20.0, dt: float = 0.01,
                   seed: int = 0) -> Problem:
    """Control problem for the fidelity gradient: Ising chain (J = 1,
    h_i ~ U[-0.5, 0.5]) driven by sum sx with a piecewise-constant amplitude of
    K equal pieces on [0, T], u_k ~ U[-1, 1]; psi0 = all up; target a
    complex-Gaussian random state, normalised.  CF6:5Opt, dt = 0.01, m = 20.
    Draw order: h, then u, then the target."""
    rng = np.random.default_rng(seed)
    h = rng.uniform(-0.5, 0.5, L)
    u = rng.uniform(-1.0, 1.0, K)
    target = random_state(1 << L, rng)
    H0 = ising_chain(L, 1.0, h)
    H1 = sigma_x_sum(L)
    edges = np.linspace(0.0, T, K + 1)
    drives = [{"kind": "pwc", "t_edges": edges, "u": u}]
    nsteps = int(round(T / dt))
    return Problem(f"adjoint-ising-L{L}-K{K}", H0, [H1], drives, basis_state(1 << L, 0),
                   scheme="CF6:5Opt", dt=dt, nsteps=nsteps, m=20,
                   meta={"L": L, "K": K, "T": T, "h": h, "u": u, "target": target,
                         "seed": seed})


CONFIGS = {"ising": config_ising, "hydrogen": config_hydrogen,
           "heisenberg": config_heisenberg}
