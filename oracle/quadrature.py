"""Gauss-Legendre rules (the element rule the paper's reference formation uses, Sect. 4)."""
from __future__ import annotations

import numpy as np


def gauss(n):
    """n-point Gauss-Legendre nodes and weights on (-1, 1) (NumPy's routine)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def gauss_on(n, a, b):
    x, w = gauss(n)
    return a + (b - a) * (x + 1.0) / 2.0, w * (b - a) / 2.0
