"""Manufactured solutions (test infrastructure only).

Paper Section 6, eqs. sin_product_exact and two_peak_exact (u1, u2 with
x01 = 0.3, y01 = 0.4, sigma1 = 0.2, x02 = 0.8, y02 = 0.6, sigma2 = 0.1),
plus the product of sines sin(pi x_i) used for the 3D workloads and the
polynomial x(1-x)y(1-y)(z(1-z)) that lies in Q_p for p >= 2.  The right-hand
sides f = -Laplace(u) are derived symbolically (sympy), so no hand-written
derivative enters the oracle.
"""
from __future__ import annotations

import numpy as np
import sympy as sy

_X = sy.symbols("x0:3", real=True)


def _build(expr, dim):
    xs = _X[:dim]
    lap = sum(sy.diff(expr, x, 2) for x in xs)
    fu = sy.lambdify(xs, expr, "numpy")
    ff = sy.lambdify(xs, -lap, "numpy")

    def u(X):
        X = np.asarray(X)
        return np.broadcast_to(fu(*[X[:, k] for k in range(dim)]), (X.shape[0],)).astype(np.float64)

    def f(X):
        X = np.asarray(X)
        return np.broadcast_to(ff(*[X[:, k] for k in range(dim)]), (X.shape[0],)).astype(np.float64)

    return u, f


def sin_product(dim: int, k: int = 1):
    """u = prod_i sin(k pi x_i); f = -Laplace(u) = dim k^2 pi^2 u."""
    return _build(sy.Mul(*[sy.sin(k * sy.pi * x) for x in _X[:dim]]), dim)


def two_peak():
    """The paper's two-peak solution u2 (2D)."""
    x, y = _X[0], _X[1]
    x01, y01, s1 = sy.Rational(3, 10), sy.Rational(2, 5), sy.Rational(1, 5)
    x02, y02, s2 = sy.Rational(4, 5), sy.Rational(3, 5), sy.Rational(1, 10)
    e = x * (1 - x) * y * (1 - y) * (
        2 * sy.exp(-((x - x01) ** 2 + (y - y01) ** 2) / (2 * s1 ** 2))
        - sy.exp(-((x - x02) ** 2 + (y - y02) ** 2) / (2 * s2 ** 2)))
    return _build(e, 2)


def bubble(dim: int):
    """u = prod_i x_i (1 - x_i): in Q_2 and zero on the boundary."""
    return _build(sy.Mul(*[x * (1 - x) for x in _X[:dim]]), dim)


def constant(value: float = 1.0):
    """f = value everywhere (load for the variable-coefficient workloads)."""
    def f(X):
        return np.full(np.asarray(X).shape[0], float(value))
    return f
