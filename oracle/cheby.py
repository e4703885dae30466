"""Stabilized Chebyshev constants of the LF-LTS scheme (Sec. 3.3), oracle side.

delta = 1 + nu/p^2, omega = 2 T_p'(delta) / T_p(delta),
beta_k = T_{k-1}(delta) / T_{k+1}(delta), beta_{k+1/2} = T_k(delta) / T_{k+1}(delta)
for 1 <= k <= p-1, with T_k the Chebyshev polynomials of the first kind.

Everything is evaluated in exact rational arithmetic (fractions.Fraction of the
double nu) and rounded once to double.  T_p'(x) = p U_{p-1}(x) with U the
Chebyshev polynomials of the second kind.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction


def _cheb_T(x: Fraction, kmax: int):
    T = [Fraction(1), x]
    for _ in range(2, kmax + 1):
        T.append(2 * x * T[-1] - T[-2])
    return T[:kmax + 1]


def _cheb_U(x: Fraction, kmax: int):
    U = [Fraction(1), 2 * x]
    for _ in range(2, kmax + 1):
        U.append(2 * x * U[-1] - U[-2])
    return U[:kmax + 1]


@dataclass
class ChebConsts:
    p: int
    nu: float
    delta: float
    omega: float
    beta: list        # beta[k] for k = 1..p-1 (index 0 unused, None)
    beta_half: list   # beta_half[k] = beta_{k+1/2} for k = 1..p-1 (index 0 unused)


def cheb_consts_from_delta(p: int, delta) -> ChebConsts:
    d = Fraction(delta)
    T = _cheb_T(d, p + 1)
    U = _cheb_U(d, p)
    dT = p * U[p - 1]
    omega = 2 * dT / T[p]
    beta = [None] + [float(T[k - 1] / T[k + 1]) for k in range(1, p)]
    beta_half = [None] + [float(T[k] / T[k + 1]) for k in range(1, p)]
    return ChebConsts(p=p, nu=float("nan"), delta=float(d), omega=float(omega),
                      beta=beta, beta_half=beta_half)


def cheb_consts(p: int, nu: float) -> ChebConsts:
    if p < 1:
        raise ValueError("p >= 1")
    if not (0.0 <= nu <= 1.0):
        raise ValueError("0 <= nu <= 1")
    d = 1 + Fraction(nu) / (p * p)
    c = cheb_consts_from_delta(p, d)
    c.nu = nu
    return c
