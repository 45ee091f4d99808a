"""Write the expected eigenvalues of the generalized n = 8000 sequence.

Runs the CPU oracle (oracle.chfsi) on the ten problems of the seeded
generalized workload (n = 8000, nev = 400, nex = 80, B = I + 0.05 G), each
warm-started from the previous Ritz vectors, and writes the nev lowest
eigenvalues of every problem to gen_n8000_eigs.txt next to this script.

With --certify it also checks each result independently of the oracle's
iteration: every returned pair has residual <= tol * ||H|| (so each value is
within that distance of an eigenvalue of the pencil), and a Sylvester
inertia count of A - sigma B (LDL^H, scipy) at sigma just above the nev-th
value shows that exactly nev eigenvalues lie below sigma, i.e. none was
skipped.

Usage:  python tests/golden/make_gen_n8000.py [--certify] [--problems N]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import chfsi  # noqa: E402
from workloads import gen  # noqa: E402


def inertia_below(a, b, sigma):
    import scipy.linalg
    if b is None:                      # standard problem: A - sigma I
        m = np.array(a, dtype=np.complex128, copy=True)
        m[np.diag_indices_from(m)] -= sigma
    else:
        m = a - sigma * b
    _, d, _ = scipy.linalg.ldl(m, lower=True, hermitian=True)
    del m
    # d is block diagonal with 1x1 and 2x2 blocks: a Hermitian tridiagonal
    w = scipy.linalg.eigvalsh_tridiagonal(np.diag(d).real, np.abs(np.diag(d, -1)))
    return int((w < 0).sum())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--certify", action="store_true")
    ap.add_argument("--problems", type=int, default=None)
    ap.add_argument("--out", default=os.path.join(HERE, "gen_n8000_eigs.txt"))
    args = ap.parse_args()
    conf = gen.CONFIGS["gen-n8000"]
    t0 = time.time()
    seq = gen.Sequence(conf, kind="numpy")
    print(f"generated A(1), B in {time.time() - t0:.1f}s", flush=True)
    rows = []
    x = None
    for l, a in seq.problems():
        if args.problems and l > args.problems:
            break
        t = time.time()
        r = chfsi.chfsi(a, conf.nev, conf.nex, b=seq.B, x0=x, opts=chfsi.Options(tol=conf.tol))
        x = r.x
        line = f"problem {l}: status {r.status} iters {r.iters} matvecs {r.matvecs} " \
               f"time {time.time() - t:.1f}s"
        assert r.status == chfsi.STATUS_OK, line
        if args.certify:
            sigma = r.lam[conf.nev - 1] + 1e-6
            cnt = inertia_below(a, seq.B, sigma)
            line += f" inertia({sigma:.6f})={cnt}"
            assert cnt == conf.nev, line
        print(line, flush=True)
        rows.append((l, r.lam[:conf.nev].copy()))
    with open(args.out, "w") as f:
        f.write("# nev lowest eigenvalues of A x = lambda B x for the generalized n=8000 sequence\n")
        f.write("# (n=8000, nev=400, nex=80, B = I + 0.05 G; seeds 1000+role), written by\n")
        f.write("# tests/golden/make_gen_n8000.py with the CPU oracle (tol 1e-10)"
                + (", inertia-certified" if args.certify else "") + "\n")
        f.write("# columns: problem index, eigenvalue index (0-based), eigenvalue\n")
        for l, lam in rows:
            for j, v in enumerate(lam):
                f.write(f"{l} {j} {v:.17e}\n")
    print(f"wrote {args.out} in {time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    main()
