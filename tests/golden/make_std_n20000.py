"""Write the expected eigenvalues of the first problems of the standard
n = 20000 sequence.

Runs the CPU oracle (oracle.chfsi) on problems 1 and 2 of the seeded
standard workload (n = 20000, nev = 1000, nex = 200, A(2) = A(1) + 1e-3 H_1),
with every Gaussian draw taken on the host (numpy PCG64, as documented in
workloads/gen.py), problem 2 warm-started from problem 1's Ritz vectors,
and writes the nev lowest eigenvalues of each problem to std_n20000_eigs.txt
next to this script.

Problem 1 has the prescribed spectrum; the file records the oracle's values
and the script checks them against it.  With --certify a Sylvester inertia
count of A - sigma I (LDL^H, scipy) at sigma just above the nev-th value
shows that exactly nev eigenvalues lie below sigma (none was skipped).

Usage:  python tests/golden/make_std_n20000.py [--certify] [--problems N]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, HERE)

from oracle import chfsi  # noqa: E402
from workloads import gen  # noqa: E402
from make_gen_n8000 import inertia_below  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--certify", action="store_true")
    ap.add_argument("--problems", type=int, default=2)
    ap.add_argument("--out", default=os.path.join(HERE, "std_n20000_eigs.txt"))
    ap.add_argument("--workload", default="std-n20000",
                    help="another standard workload of the same recipe (for a quick check)")
    args = ap.parse_args()
    conf = gen.CONFIGS[args.workload]
    t0 = time.time()
    seq = gen.Sequence(conf, kind="numpy")
    print(f"generated A(1) in {time.time() - t0:.1f}s", flush=True)
    rows = []
    x = None
    for l, a in seq.problems():
        if l > args.problems:
            break
        t = time.time()
        r = chfsi.chfsi(a, conf.nev, conf.nex, x0=x, opts=chfsi.Options(tol=conf.tol))
        x = r.x
        line = f"problem {l}: status {r.status} iters {r.iters} matvecs {r.matvecs} " \
               f"time {time.time() - t:.1f}s"
        assert r.status == chfsi.STATUS_OK, line
        if l == 1:
            dev = float(np.max(np.abs(r.lam[:conf.nev] - seq.lam[:conf.nev])))
            line += f" max|lam - prescribed| {dev:.2e}"
            assert dev < 1e-10, line
        if args.certify:
            sigma = r.lam[conf.nev - 1] + 1e-6
            cnt = inertia_below(a, None, sigma)
            line += f" inertia({sigma:.6f})={cnt}"
            assert cnt == conf.nev, line
        print(line, flush=True)
        rows.append((l, r.lam[:conf.nev].copy()))
    with open(args.out, "w") as f:
        f.write(f"# nev lowest eigenvalues of the standard sequence {conf.name}, problems 1-"
                f"{len(rows)}\n")
        f.write(f"# (n={conf.n}, nev={conf.nev}, nex={conf.nex}, A(l+1) = A(l) + 1e-3 H_l; "
                f"seeds {1000 * conf.cfg}+role, host draws), written by\n")
        f.write("# tests/golden/make_std_n20000.py with the CPU oracle (tol 1e-10)"
                + (", inertia-certified" if args.certify else "") + "\n")
        f.write("# columns: problem index, eigenvalue index (0-based), eigenvalue\n")
        for l, lam in rows:
            for j, v in enumerate(lam):
                f.write(f"{l} {j} {v:.17e}\n")
    print(f"wrote {args.out} in {time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    main()
