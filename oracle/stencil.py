"""Central finite-difference weights of arbitrary even order, in exact rationals.

TEST INFRASTRUCTURE ONLY (part of the oracle): used by tests, the smoke check and
the CPU-baseline leg of the benchmark, never by the product library.

The paper (Sec. "Discretisation schemes") computes central first- and
second-derivative stencil coefficients of arbitrary order symbolically.  Here the
same weights come from their defining property, written out: a symmetric stencil
of radius r is exact on every polynomial up to the highest degree its width
allows.  That is a small linear (Vandermonde) system, solved by Gaussian
elimination over Fractions.

  first derivative   D f_0  = (1/h)   sum_{m=1..r} a_m (f_m - f_-m)
      exact for f = x^(2l+1), l = 0..r-1  ->  sum_m 2 a_m m^(2l+1) = [l == 0]
  second derivative  D2 f_0 = (1/h^2) [c_0 f_0 + sum_{m=1..r} c_m (f_m + f_-m)]
      exact for f = x^(2l),   l = 1..r    ->  sum_m c_m m^(2l)      = [l == 1]
      and for f = 1                        ->  c_0 = -2 sum_m c_m
"""
import functools
from fractions import Fraction


def _solve(mat, rhs):
    """Gaussian elimination with exact Fractions (mat is square)."""
    n = len(mat)
    aug = [list(map(Fraction, row)) + [Fraction(b)] for row, b in zip(mat, rhs)]
    for col in range(n):
        piv = next(r for r in range(col, n) if aug[r][col] != 0)
        aug[col], aug[piv] = aug[piv], aug[col]
        for r in range(n):
            if r != col and aug[r][col] != 0:
                f = aug[r][col] / aug[col][col]
                aug[r] = [x - f * y for x, y in zip(aug[r], aug[col])]
    return [aug[i][n] / aug[i][i] for i in range(n)]


def first_derivative_weights(order):
    """a_1..a_r of the order-`order` central first derivative (order even)."""
    return list(_first_derivative_weights(order))


def second_derivative_weights(order):
    """(c_0, [c_1..c_r]) of the order-`order` central second derivative."""
    c0, c = _second_derivative_weights(order)
    return c0, list(c)


# The exact solves are repeated for every call of the oracle; their results are
# remembered per order (the weights are pure functions of it).
@functools.lru_cache(maxsize=None)
def _first_derivative_weights(order):
    if order < 2 or order % 2:
        raise ValueError("order must be a positive even integer")
    r = order // 2
    mat = [[2 * Fraction(m) ** (2 * l + 1) for m in range(1, r + 1)] for l in range(r)]
    rhs = [1 if l == 0 else 0 for l in range(r)]
    return tuple(_solve(mat, rhs))


@functools.lru_cache(maxsize=None)
def _second_derivative_weights(order):
    if order < 2 or order % 2:
        raise ValueError("order must be a positive even integer")
    r = order // 2
    mat = [[Fraction(m) ** (2 * l) for m in range(1, r + 1)] for l in range(1, r + 1)]
    rhs = [1 if l == 1 else 0 for l in range(1, r + 1)]
    c = _solve(mat, rhs)
    return -2 * sum(c), tuple(c)
