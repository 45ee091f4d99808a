"""Chebyshev polynomials and the Chebyshev filter (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``cheb``: the closed form of the definition in Sec. 3.1.1 (eq. polydef):
  C_m(t) = cos(m acos t) on [-1, 1] and cosh(m acosh t) outside; for t < -1
  the parity C_m(-t) = (-1)^m C_m(t) gives the sign.
* ``rho``: |rho(t)| = max |t +- sqrt(t^2 - 1)| for |t| > 1 (Sec. 3.1.1), and
  1 inside [-1, 1].  The convergence ratio of eq. (ratio) is 1/|rho|.
* ``sigmas``: the scalars of Alg. 2, sigma_1 = e / (gamma - c) and
  sigma_{i+1} = 1 / (2/sigma_1 - sigma_i).
* ``chebyshev_filter``: the filter of Sec. 3.1.1 with a degree per
  column: column j becomes p_{m_j}(H) y_j, p_m(x) = C_m((x - c)/e) /
  C_m((gamma - c)/e), evaluated by the scaled three-term recurrence of
  eq. (3term) (each iterate is built from the two before it).  Alg. 2 is
  the blocked, degree-sorted schedule of the same computation; the oracle
  keeps only the per-column definition.
"""
from __future__ import annotations

import math

import numpy as np


def cheb(m: int, t):
    """C_m(t) from the closed form (eq. polydef)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    inside = np.abs(t) <= 1.0
    out[inside] = np.cos(m * np.arccos(t[inside]))
    pos = t > 1.0
    out[pos] = np.cosh(m * np.arccosh(t[pos]))
    neg = t < -1.0
    out[neg] = (-1.0) ** m * np.cosh(m * np.arccosh(-t[neg]))
    return out


def rho(t):
    """|rho(t)| = max |t +- sqrt(t^2 - 1)| outside [-1, 1], else 1."""
    t = np.asarray(t, dtype=np.float64)
    out = np.ones_like(t)
    big = np.abs(t) > 1.0
    tb = t[big]
    r = np.sqrt(tb * tb - 1.0)
    out[big] = np.maximum(np.abs(tb + r), np.abs(tb - r))
    return out


def sigmas(m_max: int, c: float, e: float, gamma: float):
    """[sigma_1, ..., sigma_{m_max}] of Alg. 2."""
    s = [e / (gamma - c)]
    for _ in range(1, m_max):
        s.append(1.0 / (2.0 / s[0] - s[-1]))
    return s


def chebyshev_filter(h: np.ndarray, y0: np.ndarray, degrees, c: float, e: float,
                     gamma: float) -> np.ndarray:
    """Column j of the result is p_{m_j}(H) y0_j, the filter polynomial of
    Sec. 3.1.1 of degree m_j:

        p_m(x) = C_m((x - c)/e) / C_m((gamma - c)/e),

    evaluated by the scaled three-term recurrence of eq. (3term):

        Y_1     = (sigma_1 / e) (H - cI) Y_0
        Y_{i+1} = (2 sigma_{i+1} / e) (H - cI) Y_i - sigma_{i+1} sigma_i Y_{i-1}

    with the sigmas of ``sigmas``.  Every column runs the recurrence on its
    own for m_j steps; the columns still below their degree at a given step
    are simply advanced together.  Degrees may come in any order (Alg. 2
    sorts them only so that the still-active columns form a contiguous
    window, which changes nothing in the result)."""
    m = np.asarray([int(x) for x in degrees], dtype=np.int64)
    k = m.size
    out = np.array(y0, dtype=np.complex128, copy=True)
    if k == 0:
        return out
    if np.any(m < 1):
        raise ValueError("degrees must be >= 1")
    sig = sigmas(int(m.max()), c, e, gamma)

    def shifted(y):                                 # (H - cI) y
        return h @ y - c * y

    cols = np.arange(k)                             # columns still below their degree
    y_prev = out.copy()
    y_cur = (sig[0] / e) * shifted(y_prev)          # degree-1 iterate of every column
    for i in range(1, int(m.max()) + 1):
        # the columns whose degree is i are finished: their iterate is Y_i
        fin = m[cols] == i
        out[:, cols[fin]] = y_cur[:, fin]
        keep = ~fin
        cols, y_prev, y_cur = cols[keep], y_prev[:, keep], y_cur[:, keep]
        if cols.size == 0:
            break
        # Y_{i+1} from Y_i and Y_{i-1} (sig[i] is sigma_{i+1})
        y_next = (2.0 * sig[i] / e) * shifted(y_cur) - (sig[i] * sig[i - 1]) * y_prev
        y_prev, y_cur = y_cur, y_next
    return out


def filter_matvecs(degrees) -> int:
    """Number of column mat-vecs Alg. 2 performs: sum of the degrees."""
    return int(sum(int(x) for x in degrees))
