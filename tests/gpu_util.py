"""Helpers shared by the GPU tests: numpy <-> column-major device tensors."""
import numpy as np


def torch():
    import torch as t
    return t


def dev(x, device="cuda:0"):
    """numpy (n x k) -> column-major complex128 tensor on the GPU."""
    t = torch()
    a = np.asarray(x, dtype=np.complex128)
    if a.ndim == 1:
        a = a[:, None]
    h = t.from_numpy(np.ascontiguousarray(a.T))
    return h.to(device).transpose(0, 1)


def host(t_):
    """column-major (or any) device tensor -> numpy array."""
    return t_.detach().cpu().numpy()


def rel_col_err(got, ref):
    num = np.linalg.norm(got - ref, axis=0)
    den = np.maximum(np.linalg.norm(ref, axis=0), 1e-300)
    return num / den


def certify(a, b, lam, x, nev, tol, norm_h, b_norm=1.0, chunk=600):
    """Certificate of a computed set of eigenpairs that holds at any size,
    formed with torch's FP64 products on the device (not the library's
    kernels), for A x = lambda B x (B = None: the standard problem):

    * r_j = ||A x_j - lam_j B x_j||_2 for every column; every wanted pair
      (j < nev) must reach 2 tol N_H ||B|| (the solver locks at tol N_H in
      the standard form; x = L^-H y multiplies the residual by at most
      ||L|| = ||B||^1/2);
    * ||X^H B X - I||_max over all k columns;
    * Kato-Temple: each wanted lam_j is within r_j^2 / delta_j of an
      eigenvalue, delta_j = min over i != j of |lam_j - lam_i| - r_i (every
      lam_i is within r_i of an eigenvalue, Weyl; B >= I here, so the
      2-norm of the residual bounds its B^-1 norm).  A wanted pair whose
      delta_j does not exceed r_j gets no Kato-Temple bound (reported).

    Returns a dict of the worst values."""
    t = torch()
    n, k = x.shape
    lam_t = t.as_tensor(np.asarray(lam[:k], dtype=np.float64), device=x.device)
    res = np.empty(k)
    for c0 in range(0, k, chunk):
        c1 = min(k, c0 + chunk)
        xs = x[:, c0:c1]
        bx = xs if b is None else b @ xs
        r = a @ xs - bx * lam_t[c0:c1]
        res[c0:c1] = t.linalg.norm(r, dim=0).cpu().numpy()
        del r, bx
    bx = x if b is None else b @ x
    gram = x.conj().transpose(0, 1) @ bx
    gram.diagonal().sub_(1.0)
    orth = float(gram.abs().max())
    del gram, bx
    lam_h = np.asarray(lam[:k], dtype=np.float64)
    kt = np.full(nev, np.inf)
    for j in range(nev):
        d = np.abs(lam_h[j] - lam_h) - res
        d[j] = np.inf
        delta = d.min()
        if delta > res[j]:
            kt[j] = res[j] ** 2 / delta / abs(lam_h[j])
    bound = 2.0 * tol * norm_h * b_norm
    return {"resid_max": float(res[:nev].max()), "resid_bound": bound,
            "resid_ratio": float(res[:nev].max() / bound), "orth": orth,
            "kato_temple_rel_max": float(kt.max()), "no_kt_bound": int(np.isinf(kt).sum())}


def check_certificate(cert, label=""):
    """Asserts of the certificate: every wanted residual within its bound,
    X^H B X = I to 1e-12, every wanted eigenvalue within 1e-10 relative of
    an eigenvalue by the Kato-Temple bound."""
    print(f"  {label} certificate: residual/bound {cert['resid_ratio']:.2e} "
          f"orth {cert['orth']:.1e} Kato-Temple rel {cert['kato_temple_rel_max']:.1e}",
          flush=True)
    assert cert["resid_ratio"] <= 1.0, (label, cert)
    assert cert["orth"] <= 1e-12, (label, cert)
    assert cert["no_kt_bound"] == 0 and cert["kato_temple_rel_max"] <= 1e-10, (label, cert)
