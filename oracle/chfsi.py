"""Chebyshev Filtered Subspace Iteration, Alg. 1 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A plain complex128 implementation of the paper's method, step by step in
the order of Alg. 1:

  reduction    B = L L^H, H = L^{-1} A L^{-H} (Sec. 3.1; the paper writes a
               plain transpose, read here as the conjugate transpose)
  lanczos      a few Lanczos steps bound the top of the spectrum (Sec. 3.1)
  filter       Alg. 2 with per-vector degrees (oracle.chebyshev)
  qr           Householder QR of [locked | filtered] (Sec. 3.1), done as a
               projection against the locked vectors followed by QR
  rayleigh-ritz  G = Q^H H Q, G W = W diag(mu), Q <- Q W (Alg. 1)
  residuals    ||H q - mu q|| (eq. resl)
  locking      converged pairs move to the locked set (Sec. 3.2)
  degrees      m_j >= ln(Res_j / tol) / ln|rho_j| (Sec. 3.1.1, Single
               Optimization), capped at 40

Readings where the paper is silent or ambiguous (identical on the GPU):
  * alpha (lower end of the damped interval) is the largest Ritz value of
    the current block (alpha_rule 0); alpha_rule 1 takes the literal
    (nev+1)-th Ritz value.  gamma (estimate of lambda_1) is
    min(Lanczos theta_min, smallest Ritz value seen).  beta is the Lanczos
    bound theta_max + |b_s|, fixed for the problem.
  * With the previous problem's Ritz values (``lam0``, the inputs
    lambda_1 and lambda_{nev+1} of Alg. 1) the first filter takes alpha and
    gamma from them and filters the start block directly.  Without them the
    start block first gets one QR + Rayleigh-Ritz with the current H, which
    supplies alpha and gamma.
  * Convergence: lock when ||H q - mu q|| <= tol * N_H with
    N_H = max(|beta|, |theta_min|).  Only the lowest (nev - locked) active
    pairs are candidates; every candidate below the threshold locks.
  * Degrees: the analytic rule above with rho from the interval of the
    next filter; guard vectors and vectors inside the damped interval get
    the largest degree of the wanted vectors; the first filter uses deg0.
  * The block has k = nev + nex columns; only nev must converge.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.linalg

from . import chebyshev, counter_rng, eigh

STATUS_OK, STATUS_INVALID, STATUS_NOT_HPD, STATUS_NO_CONVERGENCE, STATUS_NONFINITE = 0, 1, 2, 3, 4


@dataclasses.dataclass
class Options:
    tol: float = 1e-10
    deg0: int = 10
    deg_max: int = 40
    max_iter: int = 100
    lanczos_steps: int = 20
    alpha_rule: int = 0          # 0: top of the block, 1: literal (nev+1)-th Ritz value
    degree_mode: int = 0         # 0: analytic rule, 1: fixed deg0
    seed: int = 0


@dataclasses.dataclass
class Result:
    lam: np.ndarray              # all k Ritz values, ascending
    x: np.ndarray                # n x k Ritz vectors (B-orthonormal)
    status: int
    iters: int
    converged: int
    matvecs: int
    filter_matvecs: int
    beta: float
    norm_h: float
    log: List[dict]


# ----------------------------------------------------------------------------
# Steps

def reduce_to_standard(a: np.ndarray, b: np.ndarray):
    """B = L L^H (Cholesky), H = L^{-1} A L^{-H}, symmetrised."""
    l = np.linalg.cholesky(b)
    w = scipy.linalg.solve_triangular(l, a, lower=True)                 # L^{-1} A
    h = scipy.linalg.solve_triangular(l, w.conj().T, lower=True)        # L^{-1} (L^{-1} A)^H
    h = h.conj().T
    return 0.5 * (h + h.conj().T), l


def lanczos_bounds(h: np.ndarray, steps: int, v0: np.ndarray):
    """``steps`` Lanczos steps with full reorthogonalisation from v0.

    Returns (upper, theta_min, theta_max) with upper = theta_max + |b_s| the
    estimate of the top of the spectrum (Sec. 3.1, after Zhou & Li)."""
    n = h.shape[0]
    s = min(steps, n)
    v = np.zeros((n, s + 1), dtype=np.complex128)
    v[:, 0] = v0[:, 0] / np.linalg.norm(v0[:, 0])
    alphas, betas = [], []
    for j in range(s):
        w = h @ v[:, j]
        a = np.vdot(v[:, j], w).real
        w = w - a * v[:, j]
        if j > 0:
            w = w - betas[j - 1] * v[:, j - 1]
        for _ in range(2):
            w = w - v[:, :j + 1] @ (v[:, :j + 1].conj().T @ w)
        b = np.linalg.norm(w)
        alphas.append(a)
        betas.append(b)
        if b == 0.0 or j == s - 1:
            break
        v[:, j + 1] = w / b
    theta, _ = eigh.tridiagonal_qr(np.array(alphas), np.array(betas[:-1]))
    tmax, tmin = float(np.max(theta)), float(np.min(theta))
    return tmax + abs(betas[-1]), tmin, tmax


def orthonormalize(y: np.ndarray, q_locked: np.ndarray) -> np.ndarray:
    """Orthonormal basis of the part of y orthogonal to the locked vectors:
    two passes of projection, then Householder QR (numpy's LAPACK QR)."""
    if q_locked.shape[1] > 0:
        for _ in range(2):
            y = y - q_locked @ (q_locked.conj().T @ y)
    q, _ = np.linalg.qr(y)
    return q


def rayleigh_ritz(h: np.ndarray, q: np.ndarray):
    """G = Q^H H Q, G W = W diag(mu) (ascending), Q W and H Q W."""
    z = h @ q
    g = q.conj().T @ z
    g = 0.5 * (g + g.conj().T)
    mu, w = eigh.eigh(g)
    return mu, q @ w, z @ w


def residual_norms(q: np.ndarray, z: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """||H q_j - mu_j q_j||_2 given Z = H Q (columns of Q are unit vectors)."""
    return np.linalg.norm(z - q * mu[None, :], axis=0)


def degree_rule(mu, res, n_wanted: int, alpha: float, beta: float, tol_abs: float,
                deg_max: int) -> np.ndarray:
    """Per-vector degrees m_j = ceil(ln(Res_j / tol) / ln|rho_j|), clamped
    to [1, deg_max]; rho from the interval [alpha, beta] of the next filter.
    Guards (index >= n_wanted) and vectors with |rho| = 1 get the largest
    degree of the wanted vectors."""
    c, e = 0.5 * (alpha + beta), 0.5 * (beta - alpha)
    t = (np.asarray(mu) - c) / e
    r = chebyshev.rho(t)
    k = len(mu)
    deg = np.zeros(k, dtype=np.int64)
    defined = np.zeros(k, dtype=bool)
    for j in range(min(n_wanted, k)):
        if r[j] > 1.0:
            ratio = max(res[j] / tol_abs, 1.0)
            m = math.ceil(math.log(ratio) / math.log(r[j]))
            deg[j] = min(max(m, 1), deg_max)
            defined[j] = True
    fill = int(deg[defined].max()) if defined.any() else deg_max
    deg[~defined] = fill
    return deg


# ----------------------------------------------------------------------------
# Alg. 1

def chfsi(a: np.ndarray, nev: int, nex: int, b: Optional[np.ndarray] = None,
          x0: Optional[np.ndarray] = None, opts: Optional[Options] = None,
          lam0: Optional[np.ndarray] = None) -> Result:
    o = opts or Options()
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[0]
    k = nev + nex
    if n < 1 or nev < 1 or nex < 1 or k > n or o.tol <= 0:
        raise ValueError("invalid arguments")
    if not np.all(np.isfinite(a)) or (x0 is not None and not np.all(np.isfinite(x0))):
        return Result(np.zeros(k), np.zeros((n, k), complex), STATUS_NONFINITE, 0, 0, 0, 0,
                      0.0, 0.0, [])

    # reduction to standard form
    l = None
    if b is not None:
        try:
            h, l = reduce_to_standard(a, np.asarray(b, dtype=np.complex128))
        except np.linalg.LinAlgError:
            return Result(np.zeros(k), np.zeros((n, k), complex), STATUS_NOT_HPD, 0, 0, 0, 0,
                          0.0, 0.0, [])
    else:
        h = a

    # start block
    if x0 is None:
        y = counter_rng.complex_block(o.seed, counter_rng.STREAM_START, n, k)
    else:
        y = np.array(x0, dtype=np.complex128)
        if l is not None:
            y = l.conj().T @ y

    # Lanczos bound (Alg. 1, the LANCZOS step)
    v0 = counter_rng.complex_block(o.seed, counter_rng.STREAM_LANCZOS, n, 1)
    beta, theta_min, theta_max = lanczos_bounds(h, o.lanczos_steps, v0)
    norm_h = max(abs(beta), abs(theta_min))
    tol_abs = o.tol * norm_h
    matvecs = min(o.lanczos_steps, n)

    q_locked = np.zeros((n, 0), dtype=np.complex128)
    lam_locked: List[float] = []
    if x0 is not None and lam0 is not None:
        # Alg. 1 inputs: the previous eigenvalues bound the first filter
        mu = np.asarray(lam0, dtype=np.float64).copy()
        qa = y
    else:
        # start: one QR + Rayleigh-Ritz supplies alpha and gamma
        qa = orthonormalize(y, q_locked)
        mu, qa, za = rayleigh_ritz(h, qa)
        matvecs += k
    alpha = _alpha(mu, nev, 0, o.alpha_rule)
    gamma = min(float(mu[0]), theta_min)
    deg = np.full(k, o.deg0, dtype=np.int64)

    log: List[dict] = []
    filter_mv = 0
    status = STATUS_NO_CONVERGENCE
    it = 0
    while it < o.max_iter:
        it += 1
        c, e = 0.5 * (alpha + beta), 0.5 * (beta - alpha)
        yf = chebyshev.chebyshev_filter(h, qa, deg, c, e, gamma)
        filter_mv += chebyshev.filter_matvecs(deg)
        qa = orthonormalize(yf, q_locked)
        mu, qa, za = rayleigh_ritz(h, qa)
        matvecs += chebyshev.filter_matvecs(deg) + qa.shape[1]
        res = residual_norms(qa, za, mu)
        n_locked = len(lam_locked)
        n_cand = nev - n_locked
        lock = np.zeros(qa.shape[1], dtype=bool)
        lock[:n_cand] = res[:n_cand] <= tol_abs
        log.append(dict(it=it, alpha=alpha, beta=beta, gamma=gamma, c=c, e=e,
                        degrees=deg.tolist(), mu=mu.tolist(), res=res.tolist(),
                        locked_before=n_locked, newly_locked=int(lock.sum())))
        if lock.any():
            q_locked = np.concatenate([q_locked, qa[:, lock]], axis=1)
            lam_locked.extend(mu[lock].tolist())
            qa, mu, res = qa[:, ~lock], mu[~lock], res[~lock]
        if len(lam_locked) >= nev:
            status = STATUS_OK
            break
        alpha = _alpha(mu, nev, len(lam_locked), o.alpha_rule)
        gamma = min(gamma, float(mu[0]))
        if o.degree_mode == 1:
            deg = np.full(qa.shape[1], o.deg0, dtype=np.int64)
        else:
            deg = degree_rule(mu, res, nev - len(lam_locked), alpha, beta, tol_abs, o.deg_max)

    lam_all = np.concatenate([np.array(lam_locked), mu])
    y_all = np.concatenate([q_locked, qa], axis=1)
    order = np.argsort(lam_all, kind="stable")
    lam_all, y_all = lam_all[order], y_all[:, order]
    x = y_all if l is None else scipy.linalg.solve_triangular(l.conj().T, y_all, lower=False)
    return Result(lam_all, x, status, it, min(len(lam_locked), nev), matvecs, filter_mv,
                  beta, norm_h, log)


def _alpha(mu, nev, n_locked, rule):
    if rule == 1:
        j = nev - n_locked
        return float(mu[min(j, len(mu) - 1)])
    return float(mu[-1])


def solve_sequence(problems, nev, nex, b=None, opts=None, warm=True, with_lambda=False):
    """Solve A^(1), A^(2), ... warm-starting each from the previous Ritz
    vectors (Sec. 2.2, Alg. 1 input Y^(l-1)) and, with ``with_lambda``, the
    previous Ritz values."""
    out = []
    x = None
    lam = None
    for a in problems:
        r = chfsi(a, nev, nex, b=b, x0=x if warm else None, opts=opts,
                  lam0=lam if (warm and with_lambda) else None)
        out.append(r)
        x, lam = r.x, r.lam
    return out
