"""Cost of optimal binomial checkpointing for reversing a time loop.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Checkpointing (paper Sec. 1) keeps a few states and recomputes the rest
from the nearest stored one. For l steps whose inputs x_0..x_{l-1} are
needed in reverse order and s state slots (the one holding x_0 included),
the minimal number of forward step evaluations is (Griewank's binomial
result)  t(l, s) = r l - C(s + r, r - 1)  with r the least integer such
that C(s + r, s) >= l. The same optimum satisfies the recursion
  T(l, 1) = l (l - 1) / 2,  T(1, s) = 0,
  T(l, s) = min_{0<j<l} [ j + T(l - j, s - 1) + T(j, s) ]
(advance j steps and store, reverse the tail with one slot fewer, then the
head with all slots), which `dp_table` evaluates by brute force.
"""
from __future__ import annotations

from math import comb

import numpy as np


def repetitions(l: int, s: int) -> int:
    r = 0
    while comb(s + r, s) < l:
        r += 1
    return r


def closed_form(l: int, s: int) -> int:
    if l <= 1:
        return 0
    r = repetitions(l, s)
    return r * l - (comb(s + r, r - 1) if r >= 1 else 0)


def dp_table(lmax: int, smax: int) -> np.ndarray:
    T = np.zeros((lmax + 1, smax + 1), dtype=np.int64)
    for l in range(1, lmax + 1):
        T[l, 1] = l * (l - 1) // 2
    for s in range(2, smax + 1):
        for l in range(2, lmax + 1):
            j = np.arange(1, l)
            T[l, s] = np.min(j + T[l - j, s - 1] + T[j, s])
    return T
