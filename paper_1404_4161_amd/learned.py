"""Learned per-vector filter degrees: log collection, data set, training.

The solver writes one convergence record per filtered wanted vector and
loop (chfsi_opts.log; layout in include/chfsi.h).  From a record the
observed speed of convergence relative to the analytic model of
Sec. 3.1.1 / eq. (resl) is

    eff = ln(Res_before / Res_after) / (m ln|rho|)

and the network is trained on y = ln(eff) from the record's features.  The
solver then uses m = ceil(m_a exp(margin - y)) with m_a the analytic
continuous degree (degree_mode 2).  Training runs on the GPU through the
library's own kernels (chfsi_mlp_train); this module only prepares arrays.
"""
from __future__ import annotations

import json
import math

import numpy as np

from . import binding as bd

F = bd.CHFSI_LOG_FIELDS
# record fields
R_LOOP, R_J, R_NW, R_KA, R_MU, R_RES, R_GAP = 0, 1, 2, 3, 4, 5, 6
R_ALPHA, R_BETA, R_GAMMA, R_NORM, R_TOL = 7, 8, 9, 10, 11
R_DEG, R_RULE, R_AFTER, R_FLAGS, R_FEAT = 12, 13, 14, 15, 16

FIELD_NAMES = ["loop", "j", "n_wanted", "ka", "mu", "res", "gap", "alpha", "beta", "gamma",
               "norm_h", "tol_abs", "degree", "rule_degree", "res_after", "flags"] + \
              [f"f{i}" for i in range(8)]

# observed reductions are only trusted down to this fraction of the target
# (below it the residual may sit on a rounding floor)
AFTER_FLOOR = 1e-2
Y_MIN, Y_MAX = math.log(0.05), math.log(8.0)


class LogBuffer:
    """Host buffer of convergence records shared by several solves."""

    def __init__(self, capacity=200_000):
        self.buf = np.zeros((capacity, F), dtype=np.float64)
        self.count = 0

    def view(self):
        """The free tail, to pass as chfsi_solve(log=...)."""
        return self.buf[self.count:]

    def advance(self, info):
        self.count += int(info["log_records"])

    def records(self):
        return self.buf[:self.count].copy()


def solve_sequence_logged(problems, Bm, nev, nex, tol, opts, buf, work=None, warm_values=True):
    """Solve a sequence warm-started from each previous solution (X0 and,
    with warm_values, Lambda0), appending every solve's records to `buf`.
    Returns the list of info dicts."""
    x = lam = None
    infos = []
    for a in problems:
        st, lam, x, info = _solve(a, Bm, nev, nex, tol, x, lam if (x is not None and warm_values)
                                  else None, opts, buf, work)
        infos.append(info)
    return infos


def _solve(a, Bm, nev, nex, tol, x0, lam0, opts, buf, work):
    st, lam, x, info = bd.chfsi_solve(a, Bm, nev, nex, tol, X0=x0, Lambda0=lam0, opts=opts,
                                     log=buf.view() if buf is not None else None, work=work)
    if st != 0:
        raise bd.ChfsiError(st, "chfsi_solve")
    if buf is not None:
        buf.advance(info)
    return st, lam, x, info


def targets(rec, fp64_only=True):
    """(X float32 n x 8, y float32 n, keep mask over rec) from records.
    With fp64_only the loops filtered in FP32 are left out: their residuals
    can stop at the FP32 rounding floor, which measures the precision, not
    the polynomial's convergence."""
    rec = np.asarray(rec, dtype=np.float64)
    feats = rec[:, R_FEAT:R_FEAT + 8]
    ok = np.all(np.isfinite(feats), axis=1)
    if fp64_only:
        ok &= (rec[:, R_FLAGS].astype(np.int64) & 1) == 0
    ok &= np.isfinite(rec[:, R_AFTER]) & (rec[:, R_AFTER] > 0) & (rec[:, R_DEG] >= 1)
    ln_rho = np.exp(np.where(ok, feats[:, 1], 0.0))
    after = np.maximum(rec[:, R_AFTER], AFTER_FLOOR * rec[:, R_TOL])
    with np.errstate(divide="ignore", invalid="ignore"):
        eff = np.log(rec[:, R_RES] / after) / (rec[:, R_DEG] * ln_rho)
    ok &= np.isfinite(eff)
    y = np.log(np.clip(eff, math.exp(Y_MIN), math.exp(Y_MAX)))
    return feats[ok].astype(np.float32), y[ok].astype(np.float32), ok


def holdout_margin(pred, y, z=3.0):
    """mean + z std of the held-out errors pred - y, at least 0 (the margin
    the solver subtracts from the network's output where a loop can finish
    every wanted vector)."""
    d = np.asarray(pred, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    if d.size == 0:
        return 0.0
    return max(0.0, float(np.mean(d) + z * np.std(d)))


def init_blob(X, seed=0):
    """Feature statistics from X and seeded Glorot-uniform weights."""
    g = np.random.default_rng(seed)
    p = np.zeros(bd.CHFSI_MLP_PARAMS, dtype=np.float64)
    p[0:8] = X.mean(axis=0)
    sd = X.std(axis=0)
    p[8:16] = np.where(sd > 1e-6, sd, 1.0)
    o = 16
    for fan_in, fan_out in ((8, 64), (64, 64), (64, 1)):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        p[o:o + fan_in * fan_out] = g.uniform(-lim, lim, fan_in * fan_out)
        o += fan_in * fan_out + fan_out          # biases stay 0
    return p.astype(np.float32)


def fit(rec, steps=1500, lr=3e-3, seed=0, holdout=0.2, z=3.0, device="cuda"):
    """Train the degree network on records with the library's kernels.

    Returns (blob float32 numpy, report dict).  The margin (used by the
    solver in loops that can finish every wanted vector) is
    mean + z * std of (prediction - target) on a held-out share of the
    records, floored at 0: a miss in such a loop costs a whole extra loop,
    far more than the extra degrees, so the margin sits far in the tail."""
    import torch
    X, y, _ = targets(rec)
    n = X.shape[0]
    if n < 16:
        raise ValueError("too few usable records to train on")
    g = np.random.default_rng(seed + 1)
    perm = g.permutation(n)
    nh = max(1, int(holdout * n)) if holdout > 0 else 0
    te, tr = perm[:nh], perm[nh:]
    blob = init_blob(X[tr], seed)
    dev = torch.device(device)
    Xt = torch.from_numpy(np.ascontiguousarray(X[tr])).to(dev)
    yt = torch.from_numpy(np.ascontiguousarray(y[tr])).to(dev)
    pt = torch.from_numpy(blob.copy()).to(dev)
    losses = bd.chfsi_mlp_train(Xt, yt, pt, steps, lr)
    report = {"records": int(len(rec)), "usable": int(n), "train": int(len(tr)),
              "holdout": int(nh), "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
              "target_var": float(np.var(y[tr]))}
    if nh:
        Xh = torch.from_numpy(np.ascontiguousarray(X[te])).to(dev)
        pred = bd.chfsi_mlp_forward(Xh, pt).cpu().numpy().astype(np.float64)
        d = pred - y[te]
        report["holdout_mse"] = float(np.mean(d ** 2))
        report["holdout_var"] = float(np.var(y[te]))
        margin = holdout_margin(pred, y[te], z)
    else:
        margin = 0.0
    out = pt.cpu().numpy().astype(np.float32)
    out[bd.CHFSI_MLP_PARAMS - 1] = margin
    report["margin"] = margin
    return out, report


def write_jsonl(rec, path):
    """One JSON object per record (field names as in include/chfsi.h)."""
    with open(path, "w") as fh:
        for r in np.asarray(rec):
            fh.write(json.dumps({k: float(v) for k, v in zip(FIELD_NAMES, r)}) + "\n")
