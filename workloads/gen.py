"""Seeded synthetic inputs for sequences of dense Hermitian (generalized)
eigenproblems.

This module only *builds inputs*; it holds none of the eigensolver's
arithmetic, so both the CPU oracle and the GPU path can take their inputs
from here.  Every random draw comes from numpy's PCG64 with a documented
seed, so the numbers are identical on every machine.  The heavy linear
algebra that turns those draws into matrices (a QR and a few products) can
run on the host (numpy) or on a GPU (torch); the two backends give the same
matrices up to rounding (relative differences near 1e-15).

Workload shapes follow the paper's test problems (Section 4, Table 1):
dense complex Hermitian problems with n in the thousands, a wanted fraction
of the spectrum of a few percent, and small perturbations from one problem
of a sequence to the next so that neighbouring problems are correlated
(Section 2.2).  The paper's FLEUR matrices are not available; these
synthetic spectra stand in for them.

Readings (none of these numbers is fixed by the paper):
  * spectrum: round(0.06 n) values ~ U[-20, -15] (the low cluster) and the
    rest ~ 10 N(0, 1) conditioned on > -15 (resampled), sorted ascending.
  * Q: unitary factor of the QR of a complex Gaussian matrix, with the
    column phases fixed so that diag(R) > 0 (this makes Q unique).
  * A^(1) = Q diag(lambda) Q^H, symmetrised.
  * "random Hermitian of unit norm": H = (G + G^H)/2 for complex Gaussian G
    (E|g|^2 = 1), scaled so that 2 ||H||_F / sqrt(n) = 1.  By the semicircle
    law this is the asymptotic spectral norm, so ||H||_2 is 1 to within a
    few percent at these sizes; it is cheap and deterministic.
  * "random HPD of unit norm": G = M M^H scaled by n / (4 ||M||_F^2), the
    Marchenko-Pastur edge for square M, so ||G||_2 is close to 1.
  * B = I + 0.05 G, fixed along a sequence.
  * A^(l+1) = A^(l) + delta_l H_l with a fresh H_l per step.
Seeds: 1000*cfg + role; role 0 spectrum, 1 Q, 2 B, 3 start block,
100 + l perturbation l.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

ROLE_SPECTRUM, ROLE_Q, ROLE_B, ROLE_START = 0, 1, 2, 3
ROLE_PERTURB = 100


def rng(cfg: int, role: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * cfg + role))


def complex_gaussian(g: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """Complex Gaussian matrix with E|z|^2 = 1 (real and imaginary parts
    N(0, 1/2)), column-major (Fortran order)."""
    re = g.standard_normal((cols, rows))
    im = g.standard_normal((cols, rows))
    z = (re + 1j * im) * math.sqrt(0.5)
    return z.T  # Fortran-ordered view of a C-ordered array


def spectrum(n: int, g: np.random.Generator, lo: float = -20.0, hi: float = -15.0,
             frac: float = 0.06, scale: float = 10.0) -> np.ndarray:
    ncl = int(round(frac * n))
    cluster = g.uniform(lo, hi, size=ncl)
    bulk = np.empty(n - ncl)
    filled = 0
    while filled < bulk.size:
        draw = scale * g.standard_normal(bulk.size - filled)
        keep = draw[draw > hi]
        bulk[filled:filled + keep.size] = keep
        filled += keep.size
    return np.sort(np.concatenate([cluster, bulk]))


# ----------------------------------------------------------------------------
# Backends: the arithmetic that assembles matrices from the draws.

class _NumpyBackend:
    name = "numpy"

    def asarray(self, x):
        return np.asfortranarray(x)

    def qr_unitary(self, z):
        q, r = np.linalg.qr(z)
        d = np.diag(r)
        ph = np.where(np.abs(d) > 0, d / np.abs(d), 1.0)
        return np.asfortranarray(q * ph[None, :])

    def from_spectrum(self, q, lam):
        a = (q * lam[None, :]) @ q.conj().T
        return np.asfortranarray(0.5 * (a + a.conj().T))

    def herm_unit(self, z):
        h = 0.5 * (z + z.conj().T)
        n = h.shape[0]
        return np.asfortranarray(h * (math.sqrt(n) / (2.0 * np.linalg.norm(h))))

    def hpd_unit(self, m):
        n = m.shape[0]
        g = m @ m.conj().T
        g = 0.5 * (g + g.conj().T)
        return g * (n / (4.0 * np.linalg.norm(m) ** 2))

    def identity_plus(self, g, w):
        b = w * g
        b[np.diag_indices_from(b)] += 1.0
        return np.asfortranarray(b)

    def axpy(self, a, d, h):
        return np.asfortranarray(a + d * h)

    def to_numpy(self, x):
        return np.asarray(x)


class _TorchBackend:
    """Same construction on a torch device.  Matrices are returned as
    column-major complex128 tensors (a transposed view of contiguous
    storage)."""
    name = "torch"

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = torch.device(device)

    def _colmajor(self, t):
        return t.transpose(0, 1).contiguous().transpose(0, 1)

    def asarray(self, x):
        t = self.torch.from_numpy(np.ascontiguousarray(np.asarray(x).T)).to(self.device)
        return t.transpose(0, 1)

    def qr_unitary(self, z):
        q, r = self.torch.linalg.qr(z.contiguous())
        d = self.torch.diagonal(r)
        a = d.abs()
        ph = self.torch.where(a > 0, d / self.torch.where(a > 0, a, self.torch.ones_like(a)),
                              self.torch.ones_like(d))
        return self._colmajor(q * ph[None, :])

    def from_spectrum(self, q, lam):
        lt = self.torch.as_tensor(lam, device=self.device, dtype=self.torch.float64)
        qh = q.conj().transpose(0, 1).contiguous()
        a = (q * lt[None, :]).contiguous() @ qh
        a = 0.5 * (a + a.conj().transpose(0, 1))
        return self._colmajor(a)

    def herm_unit(self, z):
        h = 0.5 * (z + z.conj().transpose(0, 1))
        n = h.shape[0]
        nrm = float(self.torch.linalg.norm(h))
        return self._colmajor(h * (math.sqrt(n) / (2.0 * nrm)))

    def hpd_unit(self, m):
        n = m.shape[0]
        mc = m.contiguous()
        g = mc @ mc.conj().transpose(0, 1).contiguous()
        g = 0.5 * (g + g.conj().transpose(0, 1))
        nrm = float(self.torch.linalg.norm(m))
        return g * (n / (4.0 * nrm * nrm))

    def identity_plus(self, g, w):
        b = w * g
        b.diagonal().add_(1.0)
        return self._colmajor(b)

    def axpy(self, a, d, h):
        return self._colmajor(a + d * h)

    def to_numpy(self, x):
        return x.detach().cpu().numpy()


def backend(kind: str = "numpy", device: str = "cuda:0"):
    if kind == "numpy":
        return _NumpyBackend()
    if kind == "torch":
        return _TorchBackend(device)
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# Configurations.

@dataclasses.dataclass
class SequenceConfig:
    name: str
    cfg: int            # seed namespace
    n: int
    nev: int
    nex: int
    generalized: bool
    length: int         # number of problems in the sequence
    delta: Callable[[int], float]   # perturbation size for step l -> l+1 (l >= 1)
    b_weight: float = 0.05
    tol: float = 1e-10
    deg0: int = 10

    @property
    def k(self) -> int:
        return self.nev + self.nex


def _const(d):
    return lambda l: d


def _decay(d0):
    return lambda l: d0 * 0.5 ** l


# Single-GPU workloads: a standard problem at n = 1000 and a generalized one
# at n = 8000 (5% of the spectrum wanted, 1% guard vectors), larger standard
# problems at n = 20000 (the mixed-precision size; perturbations as at
# n = 1000) and at n = 30000 (the learned-degree size, 20 problems).
CONFIGS = {
    "std-n1000": SequenceConfig("std-n1000", 0, 1000, 50, 20, False, 4, _const(1e-3)),
    "gen-n8000": SequenceConfig("gen-n8000", 1, 8000, 400, 80, True, 10, _decay(1e-2)),
    "std-n20000": SequenceConfig("std-n20000", 2, 20000, 1000, 200, False, 6, _const(1e-3)),
    "std-n30000": SequenceConfig("std-n30000", 4, 30000, 1500, 300, False, 20, _const(1e-3)),
}


def small_config(name: str, n: int, nev: int, nex: int, generalized: bool, length: int = 3,
                 cfg: int = 50, delta: float = 1e-3) -> SequenceConfig:
    """Scaled-down sequence with the same recipe (for tests)."""
    return SequenceConfig(name, cfg, n, nev, nex, generalized, length, _const(delta))


class Sequence:
    """Lazily generated sequence A^(1..N) (and the fixed B).

    draw="host" (default) takes every Gaussian draw from numpy's PCG64 as
    documented above.  draw="device" (torch backend only) takes the n x n
    Gaussian draws from torch's generator on the device, seeded with the
    same 1000 cfg + role: much faster for large batches, but not the numbers
    the host draws give (the spectrum is still drawn on the host)."""

    def __init__(self, conf: SequenceConfig, kind: str = "numpy", device: str = "cuda:0",
                 draw: str = "host"):
        self.conf = conf
        self.be = backend(kind, device)
        if draw not in ("host", "device") or (draw == "device" and kind != "torch"):
            raise ValueError("draw='device' needs the torch backend")
        self.draw = draw
        n = conf.n
        self.lam = spectrum(n, rng(conf.cfg, ROLE_SPECTRUM))
        z = self._gauss(ROLE_Q, n, n)
        q = self.be.qr_unitary(z)
        del z
        self._a1 = self.be.from_spectrum(q, self.lam)
        del q
        self.B = None
        if conf.generalized:
            m = self._gauss(ROLE_B, n, n)
            g = self.be.hpd_unit(m)
            del m
            self.B = self.be.identity_plus(g, conf.b_weight)

    def _gauss(self, role, rows, cols):
        if self.draw == "host":
            return self.be.asarray(complex_gaussian(rng(self.conf.cfg, role), rows, cols))
        torch = self.be.torch
        g = torch.Generator(device=self.be.device)
        g.manual_seed(1000 * self.conf.cfg + role)
        z = torch.randn((cols, rows), dtype=torch.complex128, device=self.be.device, generator=g)
        return z.transpose(0, 1)   # column-major view, E|z|^2 = 1

    def problems(self, count: Optional[int] = None):
        """Yield (l, A^(l)) for l = 1..min(N, count); A^(l) is the backend's
        array.  Every call starts again from A^(1) (kept by the object) and
        redraws the perturbations from their seeds, so the same sequence can
        be replayed (e.g. once per solver variant) while only A^(1) and the
        current problem are held."""
        last = self.conf.length if count is None else min(count, self.conf.length)
        a = self._a1
        yield 1, a
        for l in range(1, last):
            h = self.be.herm_unit(self._gauss(ROLE_PERTURB + l, self.conf.n, self.conf.n))
            a = self.be.axpy(a, self.conf.delta(l), h)
            del h
            yield l + 1, a


def start_block(conf: SequenceConfig) -> np.ndarray:
    """Seeded complex Gaussian start block (n x k, column-major)."""
    return np.asfortranarray(complex_gaussian(rng(conf.cfg, ROLE_START), conf.n, conf.k))


def prescribed_problem(n: int, lam: np.ndarray, seed: int) -> np.ndarray:
    """A = Q diag(lam) Q^H with Q Haar-like from a seeded QR (host)."""
    be = _NumpyBackend()
    q = be.qr_unitary(complex_gaussian(np.random.Generator(np.random.PCG64(seed)), n, n))
    return be.from_spectrum(q, np.asarray(lam, dtype=np.float64))


def random_hermitian_unit(n: int, seed: int) -> np.ndarray:
    return _NumpyBackend().herm_unit(complex_gaussian(np.random.Generator(np.random.PCG64(seed)), n, n))


def random_hpd(n: int, seed: int, weight: float = 0.05) -> np.ndarray:
    be = _NumpyBackend()
    g = be.hpd_unit(complex_gaussian(np.random.Generator(np.random.PCG64(seed)), n, n))
    return be.identity_plus(g, weight)


def random_block(n: int, k: int, seed: int) -> np.ndarray:
    return np.asfortranarray(complex_gaussian(np.random.Generator(np.random.PCG64(seed)), n, k))


def variant(conf: SequenceConfig, cfg: int, name: str = None) -> SequenceConfig:
    """The same recipe under another seed namespace (e.g. training data)."""
    return dataclasses.replace(conf, cfg=cfg, name=name or f"{conf.name}@{cfg}")


def kpoint_configs(count: int = 32, nmin: int = 2000, nmax: int = 9000, length: int = 5,
                   cfg_base: int = 300, seed: int = 3) -> List[SequenceConfig]:
    """Independent k-point sequences of one self-consistency run: n uniform
    in [nmin, nmax] (seeded), nev = 5 % and nex = 1 % of n, generalized with
    its own B, perturbations 1e-2 * 0.5^l (the n = 8000 schedule)."""
    g = np.random.Generator(np.random.PCG64(seed))
    ns = g.integers(nmin, nmax + 1, size=count)
    out = []
    for q, n in enumerate(ns):
        n = int(n)
        nev = max(1, int(round(0.05 * n)))
        nex = max(1, int(round(0.01 * n)))
        out.append(SequenceConfig(f"kpoint{q}-n{n}", cfg_base + q, n, nev, nex, True, length,
                                  _decay(1e-2)))
    return out
