"""Dense Hermitian eigensolver written out step by step (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The result it computes has a plain definition: the eigenvalues (ascending)
and orthonormal eigenvectors of a Hermitian matrix.  The steps are the
textbook ones (Golub & Van Loan, Matrix Computations, 4th ed., Sec. 8.3):

  1. Householder reduction to Hermitian tridiagonal form, T = U^H A U.
  2. A diagonal unitary D that turns T into a real symmetric tridiagonal
     matrix with non-negative off-diagonal: S = D^H T D.
  3. Implicit symmetric QR steps with the Wilkinson shift on S, with
     deflation of negligible off-diagonal entries; the Givens rotations are
     accumulated into Z when eigenvectors are wanted (S = Z diag(w) Z^T).
  4. Eigenvectors of A: V = U D Z.

The paper solves its reduced problems with a parallel MRRR solver
(Section 3.2); any backward-stable Hermitian solver returns the same
eigenvalues up to rounding, which is all the oracle needs.
"""
from __future__ import annotations

import math

import numpy as np

EPS = np.finfo(np.float64).eps


def householder_tridiagonal(a: np.ndarray):
    """Reduce Hermitian ``a`` to tridiagonal form.

    Returns (d, e, vs, taus): real diagonal d (n), complex sub-diagonal e
    (n-1), and the reflectors H_k = I - tau_k v_k v_k^H (acting on rows
    k+1..n-1) with T = H_{n-3} ... H_0 A H_0 ... H_{n-3}.
    """
    t = np.array(a, dtype=np.complex128, copy=True)
    n = t.shape[0]
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 0), dtype=np.complex128)
    vs, taus = [], []
    for k in range(n - 2):
        x = t[k + 1:, k].copy()
        xnorm = np.linalg.norm(x)
        x0 = x[0]
        if xnorm == 0.0:
            vs.append(None)
            taus.append(0.0)
            d[k] = t[k, k].real
            e[k] = 0.0
            continue
        phase = x0 / abs(x0) if abs(x0) > 0 else 1.0
        alpha = -phase * xnorm          # H x = alpha e_1
        v = x
        v[0] = x0 - alpha
        vhv = np.vdot(v, v).real
        tau = 2.0 / vhv
        # Two-sided update of the trailing block: A22 <- H A22 H with
        # H = I - tau v v^H, written as A22 - v w^H - w v^H.
        a22 = t[k + 1:, k + 1:]
        p = tau * (a22 @ v)
        kk = 0.5 * tau * np.vdot(v, p)
        w = p - kk * v
        a22 -= np.outer(v, w.conj()) + np.outer(w, v.conj())
        d[k] = t[k, k].real
        e[k] = alpha
        t[k + 1:, k] = 0.0
        t[k, k + 1:] = 0.0
        vs.append(v)
        taus.append(tau)
    if n >= 2:
        d[n - 2] = t[n - 2, n - 2].real
        e[n - 2] = t[n - 1, n - 2]
    if n >= 1:
        d[n - 1] = t[n - 1, n - 1].real
    return d, e, vs, taus


def tridiagonal_phases(e: np.ndarray):
    """Unit phases phi with conj(phi_{k+1}) e_k phi_k = |e_k| (phi_0 = 1)."""
    n = e.size + 1
    phi = np.ones(n, dtype=np.complex128)
    for k in range(n - 1):
        ak = abs(e[k])
        phi[k + 1] = phi[k] * (e[k] / ak) if ak > 0 else phi[k]
    return phi


def tridiagonal_qr(d, e, want_vectors: bool = False, max_sweeps: int = 60):
    """Eigen-decomposition of the real symmetric tridiagonal matrix with
    diagonal ``d`` and off-diagonal ``e`` by implicit symmetric QR steps with
    the Wilkinson shift (Golub & Van Loan Alg. 8.3.2/8.3.3).

    Returns (w, Z) with w unsorted, Z (n x n, columns = eigenvectors) or None.
    """
    a = [float(x) for x in d]
    b = [float(x) for x in e]
    n = len(a)
    zt = np.eye(n) if want_vectors else None   # rows of zt are columns of Z
    h = n - 1
    steps = 0
    while h > 0:
        # deflate negligible off-diagonal entries at the bottom
        if abs(b[h - 1]) <= EPS * (abs(a[h - 1]) + abs(a[h])):
            b[h - 1] = 0.0
            h -= 1
            continue
        # top of the unreduced block that ends at h
        l = h - 1
        while l > 0 and abs(b[l - 1]) > EPS * (abs(a[l - 1]) + abs(a[l])):
            l -= 1
        if l > 0:
            b[l - 1] = 0.0
        steps += 1
        if steps > max_sweeps * n:
            raise RuntimeError("tridiagonal QR did not converge")
        # Wilkinson shift from the trailing 2x2 block
        dd = 0.5 * (a[h - 1] - a[h])
        bb = b[h - 1]
        den = dd + math.copysign(math.hypot(dd, bb), dd if dd != 0.0 else 1.0)
        mu = a[h] - bb * bb / den
        # implicit QR step: chase the bulge from l to h
        x = a[l] - mu
        z = b[l]
        for k in range(l, h):
            r = math.hypot(x, z)
            if r == 0.0:
                c, s = 1.0, 0.0
            else:
                c, s = x / r, z / r
            if k > l:
                b[k - 1] = r
            ak, bk, ak1 = a[k], b[k], a[k + 1]
            a[k] = c * c * ak + 2.0 * c * s * bk + s * s * ak1
            a[k + 1] = s * s * ak - 2.0 * c * s * bk + c * c * ak1
            b[k] = c * s * (ak1 - ak) + (c * c - s * s) * bk
            if k < h - 1:
                x = b[k]
                z = s * b[k + 1]
                b[k + 1] = c * b[k + 1]
            if zt is not None:
                rk = zt[k].copy()
                zt[k] = c * rk + s * zt[k + 1]
                zt[k + 1] = -s * rk + c * zt[k + 1]
    w = np.array(a)
    return w, (zt.T.copy() if zt is not None else None)


def eigh(a: np.ndarray, want_vectors: bool = True):
    """Eigenvalues (ascending) and, optionally, eigenvectors of Hermitian a."""
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[0]
    if n == 0:
        return np.zeros(0), (np.zeros((0, 0), dtype=np.complex128) if want_vectors else None)
    if n == 1:
        return np.array([a[0, 0].real]), (np.ones((1, 1), dtype=np.complex128) if want_vectors else None)
    d, e, vs, taus = householder_tridiagonal(a)
    phi = tridiagonal_phases(e)
    w, z = tridiagonal_qr(d, np.abs(e), want_vectors)
    order = np.argsort(w, kind="stable")
    w = w[order]
    if not want_vectors:
        return w, None
    v = phi[:, None] * z[:, order]       # D Z
    # apply U = H_0 H_1 ... H_{n-3}: V <- H_0 (H_1 (... (H_{n-3} V)))
    for k in range(len(vs) - 1, -1, -1):
        vk = vs[k]
        if vk is None:
            continue
        blk = v[k + 1:, :]
        blk -= taus[k] * np.outer(vk, vk.conj() @ blk)
    return w, v


def eigvalsh(a: np.ndarray) -> np.ndarray:
    return eigh(a, want_vectors=False)[0]
