"""CFET coefficient tables and Gauss-Legendre quadrature weights (oracle side).

TEST INFRASTRUCTURE ONLY.  This module belongs to the CPU oracle: it may be
imported by ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py``, never by the product path.  It shares no code with the
HIP library, which carries its own, independently written copy of the tables.

Everything here is typed from the paper (Alvermann & Fehske, "High-order
commutator-free exponential time-propagation of driven quantum systems"):

* the CFET ansatz  U~ = exp(Omega_1) ... exp(Omega_s),
  Omega_i = sum_n f[i,n] A_n                                   (Sec. 4, eqs. Ucf, Omi)
* the time-symmetry rule R1  f[s-i+1,n] = (-1)^(n+1) f[i,n]    (Sec. 4.1, eq. FSymm)
* the coefficient tables 4thCFET, 6thCFET, 8thCoeff, 4thCFETOpt, 6thCFETOpt
* shifted Legendre polynomials on [0,1]                         (Sec. 3.1)
* Gauss-Legendre nodes/weights on [0,1], M = 1..4               (Sec. 7, Table tab:GaussLeg)
* g[i,m] = w_m sum_n (2n-1) P_{n-1}(x_m) f[i,n]                 (Sec. 7, eq. OmGLeg)

Indices in this module are 0-based: ``f[i, n-1]`` holds the paper's f_{i+1,n}.

Readings of the paper taken here (each is listed with its reason in the design
notes):
* CF4:2 is the s = 2 member of the CF4 family with f_{1,1} = 1/2,
  f_{1,2} = 1/3 (Sec. 4.2, eq. UCF4:2); the "f_{2,1} = 0" of Table 4thCFET
  names the dropped middle exponential of the s = 3 ansatz (eq. UCF4:3).
* CF6:4 is the s = 6 family with the central pair (rows 3 and 4) dropped,
  which Table 6thCFET expresses as f_{3,n} = 0.
* The number of quadrature points M equals the highest Legendre index used
  by the scheme (N/2 for the plain schemes, N/2+1 for the optimised ones;
  CF8:11 uses M = 4, the largest rule Table tab:GaussLeg prints).
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction
from math import sqrt

import numpy as np

__all__ = ["Scheme", "SCHEMES", "scheme", "legendre_shifted", "gauss_legendre",
           "gl_weights"]


@dataclass(frozen=True)
class Scheme:
    name: str
    order: int          # N
    f: np.ndarray       # (s, nmax) float64, full table after R1 expansion

    @property
    def s(self) -> int:
        return self.f.shape[0]

    @property
    def nmax(self) -> int:
        return self.f.shape[1]

    @property
    def M(self) -> int:
        """Number of Gauss-Legendre points used to form the Omega_i."""
        return self.nmax


def _expand_r1(first_rows, s: int, nmax: int) -> np.ndarray:
    """Build the full s x nmax table from its first ceil(s/2) rows by rule R1
    (Sec. 4.1, eq. FSymm): f_{s-i+1,n} = (-1)^(n+1) f_{i,n}.

    ``first_rows`` is a list of rows, each a dict {n: value} with 1-based n
    (missing entries are zero).  For odd s the last given row is the central
    exponential; its even-n entries must be zero.
    """
    f = np.zeros((s, nmax), dtype=np.float64)
    half = (s + 1) // 2
    if len(first_rows) != half:
        raise ValueError("need ceil(s/2) rows")
    for i, row in enumerate(first_rows):
        for n, v in row.items():
            f[i, n - 1] = float(v)
    for i in range(half):
        j = s - 1 - i          # 0-based mirror of row i
        if j == i:
            # central row of an odd-s scheme: only odd n may be non-zero
            for n in range(1, nmax + 1):
                if n % 2 == 0 and f[i, n - 1] != 0.0:
                    raise ValueError("central row has an even-n entry")
            continue
        for n in range(1, nmax + 1):
            f[j, n - 1] = (-1) ** (n + 1) * f[i, n - 1]
    return f


def _cf2_1():
    # Sec. 4, eq. UCF2: s = 1, f_{1,1} = 1 (exponential midpoint rule).
    return Scheme("CF2:1", 2, _expand_r1([{1: 1.0}], 1, 1))


def _cf4_2():
    # Sec. 4.2, eq. UCF4:2: exp[A1/2 + A2/3] exp[A1/2 - A2/3].
    return Scheme("CF4:2", 4, _expand_r1([{1: Fraction(1, 2), 2: Fraction(1, 3)}], 2, 2))


def _cf4_3():
    # Table 4thCFET (3 exponentials); the central row carries only f_{2,1}.
    rows = [{1: Fraction(11, 40), 2: Fraction(20, 87)}, {1: Fraction(9, 20)}]
    return Scheme("CF4:3", 4, _expand_r1(rows, 3, 2))


def _cf4_3opt():
    # Table 4thCFETOpt / eq. CF4Optimal.
    rows = [{1: Fraction(11, 40), 2: Fraction(20, 87), 3: Fraction(7, 50)},
            {1: Fraction(9, 20), 3: Fraction(-7, 25)}]
    return Scheme("CF4:3Opt", 4, _expand_r1(rows, 3, 3))


def _cf6_4():
    # Table 6thCFET, CF6:4: closed form with cube roots; the s = 6 ansatz with
    # its central pair (f_{3,n} = 0) removed, leaving exponentials 1, 2, 5, 6.
    f11 = (0.5 + (5400.0 - 600.0 * sqrt(6.0)) ** (1.0 / 3.0) / 60.0
           + ((9.0 + sqrt(6.0)) / 5.0) ** (1.0 / 3.0) / (2.0 * 3.0 ** (2.0 / 3.0)))
    f12 = f11 - 2.0 / 3.0 * f11 * f11
    f13 = 1.0 / (10.0 - 10.0 * f11)
    f21 = 0.5 - f11
    f22 = (1.0 - 4.0 * f11 + 2.0 * f11 * f11) / 3.0
    f23 = -f13
    full6 = _expand_r1([{1: f11, 2: f12, 3: f13}, {1: f21, 2: f22, 3: f23},
                        {}], 6, 3)
    # drop the (zero) central pair, rows 3 and 4 (1-based)
    f = np.delete(full6, [2, 3], axis=0)
    return Scheme("CF6:4", 6, f)


def _cf6_5_family(name, f11, f12, f13, f21, f22, f23, f14=None, f24=None):
    # Table 6thCFET / 6thCFETOpt, s = 5: the central exponential has
    # f_{3,1} = 1 - 2 f_{2,1} - 2 f_{1,1},  f_{3,2} = 0,
    # f_{3,3} = -2 f_{2,3} - 2 f_{1,3},      f_{3,4} = 0.
    r1 = {1: f11, 2: f12, 3: f13}
    r2 = {1: f21, 2: f22, 3: f23}
    nmax = 3
    if f14 is not None:
        r1[4] = f14
        r2[4] = f24
        nmax = 4
    r3 = {1: 1.0 - 2.0 * f21 - 2.0 * f11, 3: -2.0 * f23 - 2.0 * f13}
    return Scheme(name, 6, _expand_r1([r1, r2, r3], 5, nmax))


def _cf6_5():
    return _cf6_5_family("CF6:5", 0.16, 0.14587456942714338561, 0.11762370828143015682,
                         0.38752405202531186588, 0.15089113704380764664,
                         -0.12805075909013044594)


def _cf6_5b():
    return _cf6_5_family("CF6:5b", 0.2, 0.1746879190177786220, 0.12406375705333586606,
                         0.34815492558797391479, 0.1068765450953683,
                         -0.139021313323765096675)


def _cf6_5imp():
    return _cf6_5_family("CF6:5Imp", 0.16, 0.14587456942714338561, 0.11762370828143015682,
                         0.38752405202531186588, 0.15089113704380764664,
                         -0.12805075909013044594,
                         f14=0.074, f24=-0.212530296697694739551)


def _cf6_5opt():
    return _cf6_5_family("CF6:5Opt", 0.1714, 0.15409059414309687213, 0.11947178242929061641,
                         0.37496374319946236513, 0.13813675394387646682,
                         -0.13090674649282935743,
                         f14=0.07195, f24=-0.21123356253315514306)


def _cf6_6():
    # Table 6thCFET, s = 6: f_{3,1} = 1/2 - f_{1,1} - f_{2,1},
    # f_{3,3} = -f_{1,3} - f_{2,3}.
    f11, f12, f13 = 0.16, 0.15101538937746543493, 0.13304616813239630479
    f21, f22, f23 = -0.22738164742696330169, -0.087654259755115431662, 0.069919836812656575583
    r3 = {1: 0.5 - f11 - f21, 2: 0.21035154512209824847, 3: -f13 - f23}
    return Scheme("CF6:6", 6, _expand_r1([{1: f11, 2: f12, 3: f13},
                                          {1: f21, 2: f22, 3: f23}, r3], 6, 3))


def _cf6_6opt():
    # Table 6thCFETOpt, s = 6, with the A_4 row.
    f11, f12, f13, f14 = 0.3952, 0.35629343479227292880, 0.27848030437681878641, 0.1579
    f21, f22, f23, f24 = (-0.22432144875476807927, -0.19935407393749030416,
                          -0.15625650102884866893, -0.09512)
    r3 = {1: 0.5 - f11 - f21, 2: 0.1145, 3: -f13 - f23, 4: -0.16475168057141371958}
    return Scheme("CF6:6Opt", 6, _expand_r1([{1: f11, 2: f12, 3: f13, 4: f14},
                                             {1: f21, 2: f22, 3: f23, 4: f24}, r3], 6, 4))


def _cf8_11():
    # Table 8thCoeff: rows 1..5 with n = 1..4, central row 6 with n = 1, 3.
    rows = [
        {1: 0.169715531043933180094151, 2: 0.152866146944615909929839,
         3: 0.119167378745981369601216, 4: 0.068619226448029559107538},
        {1: 0.379420807516005431504230, 2: 0.148839980923180990943008,
         3: -0.115880829186628075021088, 4: -0.188555246668412628269760},
        {1: 0.469459306644050573017994, 2: -0.379844237839363505173921,
         3: 0.022898814729462898505141, 4: 0.571855043580130805495594},
        {1: -0.448225927391070886302766, 2: 0.362889857410989942809900,
         3: -0.022565582830528472333301, 4: -0.544507517141613383517695},
        {1: -0.293924473106317605373923, 2: -0.026255628265819381983204,
         3: 0.096761509131620390100068, 4: 0.000018330145571671744069},
        {1: 0.447109510586798614120629, 3: -0.200762581179816221704073},
    ]
    return Scheme("CF8:11", 8, _expand_r1(rows, 11, 4))


SCHEMES = {sc.name: sc for sc in (
    _cf2_1(), _cf4_2(), _cf4_3(), _cf4_3opt(), _cf6_4(), _cf6_5(), _cf6_5b(),
    _cf6_6(), _cf6_5imp(), _cf6_5opt(), _cf6_6opt(), _cf8_11())}


def scheme(name: str) -> Scheme:
    return SCHEMES[name]


def legendre_shifted(n: int, x):
    """Shifted Legendre polynomial P_n on [0,1] by the three-term recurrence
    of Sec. 3.1: P_0 = 1, P_1 = 2x-1,
    P_{k+1} = ((2k+1)/(k+1)) (2x-1) P_k - (k/(k+1)) P_{k-1}."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if n == 0:
        return p_prev
    p = 2.0 * x - 1.0
    for k in range(1, n):
        p_prev, p = p, ((2 * k + 1) / (k + 1)) * (2.0 * x - 1.0) * p - (k / (k + 1)) * p_prev
    return p


def gauss_legendre(M: int):
    """Nodes x_m and weights w_m on [0,1], M = 1..4 (Table tab:GaussLeg)."""
    if M == 1:
        x = [0.5]
        w = [1.0]
    elif M == 2:
        d = sqrt(3.0) / 6.0
        x = [0.5 - d, 0.5 + d]
        w = [0.5, 0.5]
    elif M == 3:
        d = sqrt(3.0 / 20.0)
        x = [0.5 - d, 0.5, 0.5 + d]
        w = [5.0 / 18.0, 4.0 / 9.0, 5.0 / 18.0]
    elif M == 4:
        d_out = sqrt((3.0 + 2.0 * sqrt(6.0 / 5.0)) / 28.0)
        d_in = sqrt((3.0 - 2.0 * sqrt(6.0 / 5.0)) / 28.0)
        x = [0.5 - d_out, 0.5 - d_in, 0.5 + d_in, 0.5 + d_out]
        wo = (18.0 - sqrt(30.0)) / 72.0
        wi = (18.0 + sqrt(30.0)) / 72.0
        w = [wo, wi, wi, wo]
    else:
        raise ValueError("Table tab:GaussLeg covers M = 1..4")
    return np.array(x), np.array(w)


def gl_weights(sc: Scheme):
    """Return (x, g) with g[i, m] = w_m sum_n (2n-1) P_{n-1}(x_m) f[i,n]
    (Sec. 7, eq. OmGLeg), so that Omega_i = dt sum_m g[i,m] A(t + x_m dt)."""
    x, w = gauss_legendre(sc.M)
    g = np.zeros((sc.s, sc.M))
    for i in range(sc.s):
        for m in range(sc.M):
            acc = 0.0
            for n in range(1, sc.nmax + 1):
                acc += (2 * n - 1) * legendre_shifted(n - 1, x[m]) * sc.f[i, n - 1]
            g[i, m] = w[m] * acc
    return x, g
