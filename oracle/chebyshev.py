"""Chebyshev polynomials and the Chebyshev filter (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``cheb``: the closed form of the definition in Sec. 3.1.1 (eq. polydef):
  C_m(t) = cos(m acos t) on [-1, 1] and cosh(m acosh t) outside; for t < -1
  the parity C_m(-t) = (-1)^m C_m(t) gives the sign.
* ``rho``: |rho(t)| = max |t +- sqrt(t^2 - 1)| for |t| > 1 (Sec. 3.1.1), and
  1 inside [-1, 1].  The convergence ratio of eq. (ratio) is 1/|rho|.
* ``sigmas``: the scalars of Alg. 2, sigma_1 = e / (gamma - c) and
  sigma_{i+1} = 1 / (2/sigma_1 - sigma_i).
* ``chebyshev_filter``: Alg. 2 -- the scaled three-term recurrence
  Y_{i+1} = 2 sigma_{i+1} Ht Y_i - sigma_{i+1} sigma_i Y_{i-1} with
  Ht = (H - cI)/e, over columns sorted by ascending degree; a column whose
  degree is reached is carried forward unchanged.

Readings of Alg. 2 (the printed listing has typos):
  * the subtracted term of the recurrence is Y_{i-1} (as in eq. 3term and
    as the sigma recursion requires), not Y_i;
  * the column range is s..k (columns), not s..n;
  * s is the first column whose degree exceeds the current step.
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
    """Alg. 2.  ``degrees`` must be ascending and >= 1; column j of the
    result is p_{m_j}(Ht) y0_j with p_m(t) = C_m(t) / C_m((gamma - c)/e)."""
    m = [int(x) for x in degrees]
    k = len(m)
    if k == 0:
        return y0.copy()
    if any(x < 1 for x in m) or any(m[j] > m[j + 1] for j in range(k - 1)):
        raise ValueError("degrees must be >= 1 and sorted ascending")
    n = h.shape[0]
    ht = (h - c * np.eye(n)) / e                       # shifted, scaled matrix
    sig1 = e / (gamma - c)
    y_prev = y0.astype(np.complex128, copy=True)
    y_cur = sig1 * (ht @ y_prev)                       # degree-1 iterate
    s = next((j for j in range(k) if m[j] != 1), k)    # first column still active
    sig = sig1
    for i in range(1, m[-1]):
        sig_next = 1.0 / (2.0 / sig1 - sig)
        y_next = np.empty_like(y_cur)
        y_next[:, :s] = y_cur[:, :s]                   # finished columns carried forward
        y_next[:, s:] = (2.0 * sig_next) * (ht @ y_cur[:, s:]) \
            - (sig_next * sig) * y_prev[:, s:]         # three-term recurrence
        s = next((j for j in range(s, k) if m[j] != i + 1), k)
        y_prev, y_cur = y_cur, y_next
        sig = sig_next
    return y_cur


def filter_closed_form(lam, q, y0, degrees, c, e, gamma):
    """Reference value of the filter for H = Q diag(lam) Q^H:
    column j -> Q diag(C_{m_j}(t) / C_{m_j}(tg)) Q^H y0_j, t = (lam - c)/e."""
    t = (np.asarray(lam) - c) / e
    tg = (gamma - c) / e
    coef = q.conj().T @ y0
    out = np.empty_like(y0, dtype=np.complex128)
    for j, mj in enumerate(degrees):
        scale = cheb(mj, t) / cheb(mj, np.array([tg]))[0]
        out[:, j] = q @ (scale * coef[:, j])
    return out


def filter_matvecs(degrees) -> int:
    """Number of column mat-vecs Alg. 2 performs: sum of the degrees."""
    return int(sum(int(x) for x in degrees))
