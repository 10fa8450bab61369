"""Closed-form solutions the paper prints, for the tests (no propagation
arithmetic of the method here)."""
import math

import numpy as np


def two_level_U(t, Delta, V, w):
    """Propagator of the circularly driven two-level system
    H(t) = Delta sz + V (cos 2wt sx + sin 2wt sy) from time 0 to t
    (Sec. 6.2, eq. TwoLevelU)."""
    Om = math.sqrt((Delta - w) ** 2 + V ** 2)
    c, s = math.cos(Om * t), math.sin(Om * t)
    e = np.exp(-1j * w * t)
    return np.array([
        [e * (c - 1j * (Delta - w) / Om * s), -1j * V / Om * e * s],
        [-1j * V / Om * np.conj(e) * s, np.conj(e) * (c + 1j * (Delta - w) / Om * s)]])
