"""Benchmark: ChFSI on a sequence of correlated dense Hermitian eigenproblems.

One step = one chfsi_solve call on the next problem of the sequence
(Lanczos bound, filter / QR / Rayleigh-Ritz / residual / locking loops
until nev pairs reach residual 1e-10, plus the reduction to standard form
and the back-transform for generalized problems), warm-started from the
previous problem's Ritz vectors and values.

Default workload (the learned-degree configuration): the standard complex
Hermitian sequence at n = 30000, nev = 1500, nex = 300, 20 problems,
A(l+1) = A(l) + 1e-3 H_l.  Problem 1 (random start block) is solved once,
untimed, with the mixed-precision filter; every timed variant then solves
problems 2..20 in order from that solution (19 timed steps).  Inputs are
generated on the GPU from seeded draws and are resident in HBM before each
timed solve; generating a problem is outside the timed region.

Timed variants: `fp64` (the paper's method: FP64 filter, analytic
degrees), `mixed-fp16+learned` (FP16-split / FP32 defect filter with the
degree network, trained in this run on convergence logs of the n = 8000
generalized, n = 20000 standard and k-point recipes under other seeds) and
`mixed-fp16` (the same filter with the analytic degrees), plus any
`--variants`.

Printed: one JSON line under 4 KB -- FP64 filter TFLOP/s (algorithmic
8 n^2 flops per column mat-vec / device time of the filter launches) as
`value`, the FP64 wall time per step as `ms_per_step`, the filter kernel's
roofline, the CPU oracle's filter rate on a bounded sample and the
FP64-against-mixed+learned comparison.  Per-step detail goes to stderr
(and to --detail-out).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (matrix and vector)

# Bytes beyond the L2 (HBM and Infinity Cache) of one full-width launch of
# the FP64 filter step kernel, from the two rocprofv3 --pmc passes
# (FETCH_SIZE, WRITE_SIZE) of `bench.py --filter-only`, calibrated on a
# 1 GiB device copy; keyed by (n, N, tile variant).  Valid only for the kernel source they were
# measured on (the hash); otherwise the roofline reports traffic null.
TRAFFIC_MEASURED = {
    "zgemm_sha256": "fc73129498a79014fc6f164424c783167f77c67ee9b9e9de9c0922857e7525cd",
    # the default tile (variant 5, 3M, operands loaded straight into LDS); a
    # full-width step at n = 30000 runs as two K splits (partial sums and
    # cheb_reduce, both counted)
    "bytes_per_full_width_launch": {(8000, 480, 5): 3.234e9, (30000, 1800, 5): 428.1e9},
}


def traffic_entry(n, N, variant):
    """Measured GB beyond the L2 of one full-width filter step at (n, N), or None."""
    import hashlib
    src = os.path.join(ROOT, "paper_1404_4161_amd", "csrc", "zgemm.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    b = TRAFFIC_MEASURED["bytes_per_full_width_launch"].get((int(n), int(N), int(variant)))
    if sha != TRAFFIC_MEASURED["zgemm_sha256"] or b is None:
        return None
    return round(b / 1e9, 3)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(a_host: np.ndarray, k: int, degree: int, seed: int = 0):
    """Time the CPU oracle's Chebyshev filter on a bounded sample: the
    workload's n x n matrix and `k` random columns, each filtered to one
    degree (the oracle as it stands, numpy BLAS on the host's threads)."""
    from oracle import chebyshev
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info if i.get("user_api") == "blas"] or [1])
    except Exception:   # pragma: no cover
        threads = os.cpu_count() or 1
    n = a_host.shape[0]
    g = np.random.default_rng(seed)
    y0 = (g.standard_normal((n, k)) + 1j * g.standard_normal((n, k))) * np.sqrt(0.5)
    t = time.perf_counter()
    chebyshev.chebyshev_filter(a_host, y0, [degree] * k, 12.5, 27.5, -20.0)
    dt = time.perf_counter() - t
    flops = 8.0 * n * n * k * degree
    return {"value": round(flops / dt / 1e12, 4), "unit": "TFLOP/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"oracle filter on problem 1's matrix (n={n}), {k} columns at degree "
                      f"{degree}, {dt:.1f} s on the host"}


def filter_only(conf, degree):
    """One 1 GiB device-to-device copy (counter calibration), then one
    Chebyshev filter of the workload's n x k block at a uniform degree on a
    random Hermitian matrix (the filter's cost does not depend on the
    values)."""
    import torch
    import paper_1404_4161_amd as ch
    dev = "cuda:0"
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)      # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    n, k = conf.n, conf.k
    # the launch variant the benchmark would take for this shape
    v, vtf = ch.chfsi_autotune_filter([n], [k])
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    h = torch.randn(n, n, dtype=torch.complex128, device=dev, generator=g)
    h = ch.colmajor(0.5 * (h + h.conj().transpose(0, 1)))
    y = ch.colmajor(torch.randn(n, k, dtype=torch.complex128, device=dev, generator=g))
    nrm = 1.1 * (2.0 * n) ** 0.5      # semicircle edge of this random Hermitian matrix
    torch.cuda.synchronize()
    t = time.perf_counter()
    flops, launches = ch.chfsi_filter(h, y, [degree] * k, 0.0, nrm, -1.05 * nrm)
    dt = time.perf_counter() - t
    # then the defect filter at the same shape with every step in BF16-split
    # form (the Ritz-pair inputs do not change its cost)
    q = ch.colmajor(y / torch.linalg.vector_norm(y, dim=0, keepdim=True))
    z = ch.colmajor(h @ q)
    mu = np.linspace(-1.2 * nrm, -1.1 * nrm, k)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, f16, _ = ch.chfsi_filter_defect_split(h, q, z, mu, [degree] * k, 0.0, nrm, -1.3 * nrm,
                                             degree)
    dt16 = time.perf_counter() - t
    # and with every step in FP16-split form
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, fh, _ = ch.chfsi_filter_defect_split(h, q, z, mu, [degree] * k, 0.0, nrm, -1.3 * nrm,
                                            degree, fp16=True)
    dth = time.perf_counter() - t
    print(json.dumps({"mode": "filter-only", "n": n, "k": k, "degree": degree,
                      "variant": int(v[0]),
                      "variant_tflops": [round(float(x), 2) for x in vtf[0]],
                      "launches": launches, "seconds": round(dt, 6),
                      "tflops_wall": round(flops / dt / 1e12, 3),
                      "bf16_split_defect_seconds": round(dt16, 6),
                      "bf16_split_defect_tflops_wall": round(f16 / dt16 / 1e12, 3),
                      "fp16_split_defect_seconds": round(dth, 6),
                      "fp16_split_defect_tflops_wall": round(fh / dth / 1e12, 3),
                      "copy_bytes": src.numel() * 8}), flush=True)


def kpoints(args):
    """Batched k-point sequences: 32 independent generalized problems with n
    uniform in [2000, 9000], nev = 5 %, nex = 1 % of n, 5 steps each
    (perturbations 1e-2 * 0.5^l).  Step 1 (random starts) is the warm-up;
    steps 2-5 are timed, every problem warm-started from its previous
    solution.  Variants: one chfsi_solve_batch call per step (grouped filter
    launches: FP64, FP64 with graph capture, mixed precision with the defect
    filters grouped or each on its problem's stream) against 32 chfsi_solve
    calls per step (FP64 and mixed).  Prints one JSON line."""
    import torch
    import paper_1404_4161_amd as ch
    from workloads import gen
    dev = "cuda:0"
    confs = gen.kpoint_configs()[:args.kp_count]
    count = len(confs)
    stream = torch.cuda.Stream(device=dev)
    results = {}
    shapes = sorted({(c.n, c.k) for c in confs} | {(c.n, max(c.k // 4, 16)) for c in confs})
    t0 = time.perf_counter()
    tv, ttf = ch.chfsi_autotune_filter([a for a, _ in shapes], [b for _, b in shapes])
    per_variant = np.bincount(tv, minlength=ttf.shape[1]).tolist()
    log(f"autotune of {len(shapes)} shapes in {time.perf_counter() - t0:.1f}s: "
        f"shapes per variant {per_variant}")

    def run(label, precision, batched, graph, serial=False, own_defect=False):
        t0 = time.perf_counter()
        seqs = [gen.Sequence(c, kind="torch", device=dev, draw="device") for c in confs]
        gens = [s_.problems() for s_ in seqs]
        Bs = [s_.B for s_ in seqs]
        torch.cuda.synchronize()
        log(f"[kpoints {label}] generated the first problems in {time.perf_counter() - t0:.1f}s")
        o = ch.chfsi_default_opts()
        o.precision = precision
        works = [torch.empty(ch.chfsi_workspace_bytes(c.n, c.nev, c.nex, True, o),
                             dtype=torch.uint8, device=dev) for c in confs]
        Xs = [ch.colmajor(torch.empty((c.n, c.k), dtype=torch.complex128, device=dev))
              for c in confs]
        x0s = lam0s = None
        walls, infos_all = [], []
        for step in range(confs[0].length):
            As = [next(g_)[1] for g_ in gens]
            torch.cuda.synchronize()
            ts = time.perf_counter()
            with torch.cuda.stream(stream):
                if batched:
                    st, lams, _, infos, sts = ch.chfsi_solve_batch(
                        As, Bs, [c.nev for c in confs], [c.nex for c in confs], 1e-10,
                        X0s=x0s, Lambda0s=lam0s, opts=o, Xs=Xs, works=works, stream=stream,
                        graph=graph, serial=serial, own_defect=own_defect)
                    if st != 0:
                        raise RuntimeError(f"chfsi_solve_batch status {st} {sts}")
                else:
                    lams, infos = [], []
                    for q, c in enumerate(confs):
                        st, lam, _, info = ch.chfsi_solve(
                            As[q], Bs[q], c.nev, c.nex, 1e-10,
                            X0=None if x0s is None else x0s[q],
                            Lambda0=None if lam0s is None else lam0s[q], opts=o, X=Xs[q],
                            work=works[q], stream=stream)
                        if st != 0:
                            raise RuntimeError(f"chfsi_solve status {st}")
                        lams.append(lam)
                        infos.append(info)
            stream.synchronize()
            wall = time.perf_counter() - ts
            log(f"[kpoints {label}] step {step + 1}: {wall:.3f}s, loops "
                f"{min(i['iters'] for i in infos)}-{max(i['iters'] for i in infos)}")
            if step > 0:
                walls.append(wall)
                infos_all.append(infos)
            x0s, lam0s = Xs, lams
            del As
        fl = sum(i["filter_flops"] for inf in infos_all for i in inf)
        phase_names = ["reduction", "lanczos", "filter", "orthonormalize", "rayleigh_ritz",
                       "residuals", "locking", "back_transform"]
        ph = np.sum([i["step_seconds"] for inf in infos_all for i in inf], axis=0) / len(walls)
        results[label] = {
            "device_seconds_per_step_summed_over_problems": {
                nm: round(float(v), 3) for nm, v in zip(phase_names, ph)},
            "s_per_step": round(statistics.mean(walls), 4),
            "s_per_step_each": [round(w, 4) for w in walls],
            "filter_tflops_over_wall": round(fl / sum(walls) / 1e12, 3),
            "loops_per_step": [sum(i["iters"] for i in inf) for inf in infos_all],
            "lams_last": [l[:c.nev].copy() for l, c in zip(lam0s, confs)],
        }
        del works, Xs, seqs, gens, Bs
        torch.cuda.empty_cache()

    variants = {"batched-fp64": ("batched fp64", 0, True, False),
                "batched-fp64-graph": ("batched fp64 graph", 0, True, True),
                "sequential-fp64": ("sequential fp64", 0, False, False),
                "batched-mixed": ("batched mixed", 1, True, False),
                "batched-mixed-bf16": ("batched mixed bf16", 2, True, False),
                "batched-mixed-fp16": ("batched mixed fp16", 3, True, False),
                "batched-mixed-fp16-own": ("batched mixed fp16 own", 3, True, False, False,
                                           True),
                "sequential-mixed-fp16": ("sequential mixed fp16", 3, False, False),
                "batched-fp64-serial": ("batched fp64 serial", 0, True, False, True)}
    chosen = args.kp_variants.split(",")
    for key in chosen:
        run(*variants[key])
    ref_key = "sequential fp64" if "sequential-fp64" in chosen else variants[chosen[0]][0]
    ref = results[ref_key]["lams_last"]
    for lab, r in results.items():
        r[f"max_rel_eig_diff_vs_{ref_key.replace(' ', '_')}"] = float(max(
            np.max(np.abs(a - b) / np.abs(b)) for a, b in zip(r.pop("lams_last"), ref)))
    out = {
        "metric": "s per batched sequence step (32 k-point problems) at 1e-10 residual",
        "autotune": {"shapes": len(shapes), "shapes_per_variant": per_variant,
                     "mean_tflops_per_variant": [round(float(ttf[:, v][ttf[:, v] > 0].mean()), 2)
                                                 if np.any(ttf[:, v] > 0) else None
                                                 for v in range(ttf.shape[1])]},
        "workload": "kpoints: 32 generalized complex Hermitian sequences, n uniform in "
                    "[2000, 9000], nev 5 %, nex 1 %, 5 steps (step 1 untimed)",
        "n": [c.n for c in confs], "steps": confs[0].length - 1,
        "speedup_batched_vs_sequential_fp64": (round(
            results["sequential fp64"]["s_per_step"] / results["batched fp64"]["s_per_step"], 3)
            if {"sequential fp64", "batched fp64"} <= set(results) else None),
        "speedup_batched_vs_sequential_mixed_fp16": (round(
            results["sequential mixed fp16"]["s_per_step"]
            / results["batched mixed fp16"]["s_per_step"], 3)
            if {"sequential mixed fp16", "batched mixed fp16"} <= set(results) else None),
        "variants": results,
    }
    print(json.dumps(out), flush=True)


# (precision, degree_mode, first_rule) of each solver variant.  precision:
# 0 FP64 filter, 1 FP32 defect filter, 2 with BF16-split steps, 3 with
# FP16-split steps; degree_mode: 0 analytic rule, 2 degree network,
# 3 sequence-calibrated speeds.  FP64 takes the first loop's degrees from
# the residuals of X0 only with the network (first_rule 1).
VARIANTS = {
    "fp64": (0, 0, 0),
    "mixed": (1, 0, 0),
    "mixed-bf16": (2, 0, 0),
    "mixed-fp16": (3, 0, 0),
    "mixed-fp16+learned": (3, 2, 0),
    "mixed+learned": (1, 2, 0),
    "mixed-bf16+learned": (2, 2, 0),
    "fp64+learned": (0, 2, 1),
    "mixed-fp16+seqcal": (3, 3, 0),
    "fp64+seqcal": (0, 3, 1),
}
HEADLINE = "mixed-fp16+learned"      # the metric's mixed+learned form
RULE_TWIN = "mixed-fp16"             # the same filter with the analytic degrees
PHASES = ["reduction", "lanczos", "filter", "orthonormalize", "rayleigh_ritz", "residuals",
          "locking", "back_transform"]


def training_logs(dev, quick=False):
    """Convergence records for the degree network: FP64 solves (first loop
    degrees from X0's residuals, and a second pass with degree jitter 0.3
    for spread) of three recipes under seed namespaces the benchmark does
    not time -- the generalized n = 8000 sequence (10 problems), the
    standard n = 20000 sequence (first 3 problems) and 6 k-point
    sequences (n in [2000, 9000], 5 problems each)."""
    import torch
    import paper_1404_4161_amd as ch
    from paper_1404_4161_amd import learned
    from workloads import gen
    buf = learned.LogBuffer(600_000)
    report = []
    c1 = gen.variant(gen.CONFIGS["gen-n8000"], 101)
    c2 = gen.variant(gen.CONFIGS["std-n20000"], 102)
    kp = gen.kpoint_configs(count=6, cfg_base=500, seed=5)
    plan = [(c1, c1.length, (0.0, 0.3)), (c2, 2 if quick else 3, (0.0,))]
    plan += [(c, c.length, (0.0,)) for c in kp[:2 if quick else 6]]
    for conf, count, jitters in plan:
        t0 = time.perf_counter()
        draw = "device" if conf.n > 10000 else "host"
        seq = gen.Sequence(conf, kind="torch", device=dev, draw=draw)
        probs = [a.clone() for _, a in seq.problems(count)]
        torch.cuda.synchronize()
        before = buf.count
        iters = []
        for jit in jitters:
            o = ch.chfsi_default_opts()
            o.precision, o.first_rule, o.degree_jitter, o.seed = 0, 1, jit, 7
            iters.append([i["iters"] for i in learned.solve_sequence_logged(
                probs, seq.B, conf.nev, conf.nex, conf.tol, o, buf)])
        report.append({"recipe": conf.name, "problems": count, "records": buf.count - before,
                       "seconds": round(time.perf_counter() - t0, 1)})
        log(f"training logs {conf.name}: {count} problems, loops {iters}, "
            f"{buf.count - before} records, {time.perf_counter() - t0:.1f}s")
        del probs, seq
        torch.cuda.empty_cache()
    return buf.records(), report


def run_variant(label, seq, conf, B, x1, lam1, steps, work, X, blob, dev):
    """Solve problems 2..steps+1 of the sequence in order, starting from
    problem 1's solution (x1, lam1).  Each problem is generated (untimed)
    before its solve; the wall time of every chfsi_solve call is kept."""
    import torch
    import paper_1404_4161_amd as ch
    prec, mode, first = VARIANTS[label]
    o = ch.chfsi_default_opts()
    o.precision, o.degree_mode, o.first_rule = prec, mode, first
    rates = np.full(conf.k, np.nan) if mode == 3 else None
    x_prev, lam_prev = x1, lam1
    stream = torch.cuda.current_stream(dev)
    infos, walls, lams = [], [], []
    for l, a in seq.problems(steps + 1):
        if l == 1:
            continue
        torch.cuda.synchronize()
        ts = time.perf_counter()
        st, lam, _, info = ch.chfsi_solve(a, B, conf.nev, conf.nex, conf.tol, X0=x_prev,
                                          Lambda0=lam_prev, opts=o, X=X, work=work,
                                          stream=stream, mlp=blob if mode == 2 else None,
                                          seq_rates=rates)
        walls.append(time.perf_counter() - ts)
        if st != 0:
            raise RuntimeError(f"[{label}] chfsi_solve status {st} on problem {l}")
        x_prev, lam_prev = X, lam
        infos.append(info)
        lams.append(lam[:conf.nev].copy())
        log(f"[{label}] problem {l}: loops {info['iters']} (fp32 {info['filter_iters_fp32']}) "
            f"matvecs {info['filter_matvecs']} filter {info['filter_seconds'] * 1e3:.1f} ms "
            f"step {walls[-1] * 1e3:.1f} ms")
        del a
    return {"infos": infos, "walls": walls, "lams": lams}


def summarize(label, r, ref_lams=None):
    infos, walls = r["infos"], r["walls"]
    steps = len(walls)
    fl = sum(i["filter_flops"] for i in infos)
    fs = sum(i["filter_seconds"] for i in infos)
    d = {"ms_per_step": round(1e3 * sum(walls) / steps, 2),
         "s_per_step_median": round(statistics.median(walls), 4),
         "loops": sum(i["iters"] for i in infos),
         "filter_matvecs": sum(i["filter_matvecs"] for i in infos),
         "filter_ms_per_step": round(1e3 * fs / steps, 2),
         "filter_effective_tflops": round(fl / fs / 1e12, 2) if fs > 0 else None}
    if ref_lams is not None:
        d["max_rel_eig_diff_vs_fp64"] = float(f"{max(float(np.max(np.abs(a - b) / np.abs(b))) for a, b in zip(r['lams'], ref_lams)):.2e}")
    return d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=19,
                    help="timed problems (at most the sequence length minus the untimed first)")
    ap.add_argument("--warmup", type=int, default=1,
                    help="accepted for the harness; the one untimed problem is the sequence's "
                         "cold first problem")
    ap.add_argument("--workload", default="std-n30000",
                    choices=["gen-n8000", "std-n1000", "std-n20000", "std-n30000", "kpoints"])
    ap.add_argument("--variants", default="",
                    help="comma list of extra variants to time after fp64, mixed-fp16+learned "
                         "and mixed-fp16: " + ", ".join(VARIANTS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-degree", type=int, default=40)
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the degree network (and the learned variant)")
    ap.add_argument("--quick-logs", action="store_true",
                    help="fewer training-log problems (for short runs)")
    ap.add_argument("--train-steps", type=int, default=1500)
    ap.add_argument("--budget-s", type=float, default=520.0,
                    help="wall-clock budget: optional phases that would not finish within it "
                         "are skipped (and reported as skipped)")
    ap.add_argument("--detail-out", default="",
                    help="write the per-step detail JSON to this file")
    ap.add_argument("--filter-only", action="store_true",
                    help="time only the Chebyshev filter at the workload shape (n x k block, "
                         "uniform degree) after a 1 GiB device copy used to calibrate "
                         "hardware byte counters; for profiler runs")
    ap.add_argument("--degree", type=int, default=4)
    ap.add_argument("--kp-count", type=int, default=32,
                    help="k-point workload: number of problems (32 in the full workload)")
    ap.add_argument("--kp-variants", default="batched-fp64,sequential-fp64,batched-mixed-fp16,"
                                             "batched-mixed-fp16-own,sequential-mixed-fp16")
    args = ap.parse_args()
    t_start = time.perf_counter()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the library solves "
                                   "each problem (or batch) on one device and has no multi-GPU "
                                   "path", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1404_4161_amd as ch
    from workloads import gen

    ch.lib()   # fail loudly if the HIP library is missing
    if args.workload == "kpoints":
        kpoints(args)
        return
    conf = gen.CONFIGS[args.workload]
    if args.filter_only:
        filter_only(conf, args.degree)
        return
    steps = max(1, min(args.steps, conf.length - 1))
    if steps != args.steps:
        log(f"timing {steps} problems: the sequence has {conf.length} problems and the first "
            f"is the untimed cold start")
    dev = "cuda:0"
    n, nev, nex, k = conf.n, conf.nev, conf.nex, conf.k

    def elapsed():
        return time.perf_counter() - t_start

    # Filter tile autotuner (untimed): the tile variants of the FP64 step on
    # the full window and narrower ones; later launches take the choice of
    # the nearest measured shape.
    tune_shapes = [(n, k), (n, (3 * k) // 4), (n, k // 2), (n, k // 4), (n, max(k // 8, 16))]
    tv, ttf = ch.chfsi_autotune_filter([a for a, _ in tune_shapes], [b for _, b in tune_shapes])
    log("autotune: " + ", ".join(f"N={b}: variant {int(v)} ({max(t):.1f} TFLOP/s)"
                                 for (_, b), v, t in zip(tune_shapes, tv, ttf)))

    # Degree network (untimed), trained with the library's kernels.
    blob, train = None, None
    if not args.no_learned:
        from paper_1404_4161_amd import learned
        t0 = time.perf_counter()
        rec, sources = training_logs(dev, quick=args.quick_logs)
        tc = time.perf_counter()
        blob, rep = learned.fit(rec, steps=args.train_steps)
        train = {"records": rep["records"], "usable": rep["usable"],
                 "holdout_mse": round(rep["holdout_mse"], 4),
                 "target_var": round(rep["target_var"], 4), "margin": round(rep["margin"], 4),
                 "train_s": round(time.perf_counter() - tc, 1), "logs_s": round(tc - t0, 1),
                 "sources": ",".join(f"{s['recipe']}:{s['problems']}" for s in sources)}
        log(f"degree network: {rep}")

    t0 = time.perf_counter()
    draw = "device" if n > 10000 else "host"
    seq = gen.Sequence(conf, kind="torch", device=dev, draw=draw)
    B = seq.B
    torch.cuda.synchronize()
    log(f"generated problem 1 (n={n}) in {time.perf_counter() - t0:.1f}s")

    o3 = ch.chfsi_default_opts()
    o3.precision = 3
    wb = max(ch.chfsi_workspace_bytes(n, nev, nex, B is not None, ch.chfsi_default_opts()),
             ch.chfsi_workspace_bytes(n, nev, nex, B is not None, o3))
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    X = ch.colmajor(torch.empty((n, k), dtype=torch.complex128, device=dev))
    X1 = ch.colmajor(torch.empty((n, k), dtype=torch.complex128, device=dev))

    # Problem 1, cold (random start block), untimed: solved with the rule and
    # (when trained) with the network; the rule's solution starts every
    # timed variant.
    a1 = next(seq.problems(1))[1]
    cold = {}
    for label in ([HEADLINE] if blob is not None else []) + [RULE_TWIN]:
        prec, mode, first = VARIANTS[label]
        o = ch.chfsi_default_opts()
        o.precision, o.degree_mode = prec, mode
        st, lam1, _, info = ch.chfsi_solve(a1, B, nev, nex, conf.tol, opts=o, X=X1, work=work,
                                           mlp=blob if mode == 2 else None)
        if st != 0:
            raise RuntimeError(f"cold solve ({label}) status {st}")
        cold[label] = {"s": round(info["total_seconds"], 2), "loops": info["iters"],
                       "filter_matvecs": info["filter_matvecs"]}
        log(f"cold problem 1 [{label}]: {cold[label]}")
    x1 = X1

    runs = {}
    order = ["fp64"] + ([HEADLINE] if blob is not None else []) + [RULE_TWIN]
    order += [v for v in args.variants.split(",") if v and v not in order
              and (blob is not None or VARIANTS[v][1] != 2)]
    skipped = []
    for label in order:
        if label not in ("fp64", HEADLINE) and runs:
            # optional variants run only if they fit the wall-clock budget
            est = 1.25 * min(sum(r["walls"]) for r in runs.values())
            if elapsed() + est > args.budget_s:
                skipped.append(label)
                log(f"[{label}] skipped: {elapsed():.0f}s elapsed, about {est:.0f}s needed, "
                    f"budget {args.budget_s:.0f}s")
                continue
        runs[label] = run_variant(label, seq, conf, B, x1, lam1, steps, work, X, blob, dev)
        torch.cuda.synchronize()

    r64 = runs["fp64"]
    infos = r64["infos"]
    flops = sum(i["filter_flops"] for i in infos)
    mflops = sum(i["filter_flops_fp64_mfma"] for i in infos)
    fsec = sum(i["filter_seconds"] for i in infos)
    launches = sum(i["filter_launches"] for i in infos)
    # value: complex-equivalent rate (8 real flops per complex multiply-add,
    # the standard count); roofline: the real flops the MFMAs executed (6
    # per complex multiply-add on the 3M tile variants)
    tflops = flops / fsec / 1e12
    mtflops = mflops / fsec / 1e12
    wall64 = sum(r64["walls"])
    phases = np.sum([i["step_seconds"] for i in infos], axis=0) / steps
    summ = {lab: summarize(lab, r, None if lab == "fp64" else r64["lams"])
            for lab, r in runs.items()}
    out = {
        "metric": "filter TFLOP/s + s/sequence-step at 1e-10 residual, FP64 vs mixed+learned",
        "value": round(tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 1,
        "ms_per_step": round(1e3 * wall64 / steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{conf.name}: {'generalized' if B is not None else 'standard'} complex "
                         f"Hermitian sequence of {conf.length} problems, n={n}, nev={nev}, "
                         f"nex={nex}, tol {conf.tol}; problem 1 cold (untimed), problems 2-"
                         f"{steps + 1} timed, each warm-started from the previous solution; "
                         f"value = complex-equivalent TFLOP/s of the FP64 filter (8 real flops "
                         f"per complex multiply-add; the 3M tile variants execute 6 on MFMA)"),
            "n": n, "nev": nev, "nex": nex, "problems": conf.length, "problems_timed": steps,
        },
        "roofline": {
            "bound": "mfma",
            "achieved": round(mtflops, 3),
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(mtflops / PEAK_FP64_TFLOPS, 4),
            "traffic": traffic_entry(n, k, tv[0]),
            "kernel": "FP64 filter step zgemm_dma_kernel<EPI_CHEB,3> (3M split, operands "
                      "loaded straight into LDS; split-K steps: partial sums + cheb_reduce; "
                      "other tile variants where the autotuner picks them)",
            "flops_note": "achieved = real flops executed on MFMA (6 n^2 per column mat-vec "
                          "with the 3M split, 8 with 4M) / filter device time",
            "tile_variant_full_width": int(tv[0]),
            "traffic_note": f"GB beyond the L2 (FETCH_SIZE + WRITE_SIZE, calibrated) of one "
                            f"full-width launch (n={n}, N={k}); algorithmic "
                            f"{(16 * n * n + 48 * n * k) / 1e9:.3f} GB",
            "avg_launch_us": round(fsec / launches * 1e6, 1),
            "launches": launches,
        },
        "s_per_sequence_step_median": round(statistics.median(r64["walls"]), 4),
        "phase_s_per_step": {nm: round(float(v), 3) for nm, v in zip(PHASES, phases)
                             if v > 0},
    }
    if HEADLINE in summ:
        h = summ[HEADLINE]
        cmp_ = {"fp64_ms_per_step": out["ms_per_step"],
                "mixed_learned_ms_per_step": h["ms_per_step"],
                "speedup": round(out["ms_per_step"] / h["ms_per_step"], 3),
                "max_rel_eig_diff_vs_fp64": h["max_rel_eig_diff_vs_fp64"],
                "variant": HEADLINE}
        if RULE_TWIN in summ:
            cmp_["rule_ms_per_step"] = summ[RULE_TWIN]["ms_per_step"]
            cmp_["learned_vs_rule"] = round(summ[RULE_TWIN]["ms_per_step"] / h["ms_per_step"], 3)
        out["fp64_vs_mixed_learned"] = cmp_
    out["variants"] = {lab: {kk: v for kk, v in s.items() if kk in
                             ("ms_per_step", "loops", "filter_matvecs", "filter_ms_per_step",
                              "max_rel_eig_diff_vs_fp64")} for lab, s in summ.items()}
    if skipped:
        out["skipped_for_budget"] = skipped
    out["cold_problem_1"] = cold
    if train is not None:
        out["degree_network"] = train
    detail = {lab: {"walls_s": [round(w, 4) for w in r["walls"]],
                    "loops": [i["iters"] for i in r["infos"]],
                    "fp32_loops": [i["filter_iters_fp32"] for i in r["infos"]],
                    "fp16_steps": [i["filter_steps_fp16"] for i in r["infos"]],
                    "filter_matvecs": [i["filter_matvecs"] for i in r["infos"]],
                    "filter_s": [round(i["filter_seconds"], 4) for i in r["infos"]],
                    "learned_cols": [i["learned_cols"] for i in r["infos"]],
                    "fallback_cols": [i["fallback_cols"] for i in r["infos"]],
                    "rr_refined_dense": [[i["rr_refined"], i["rr_dense"]] for i in r["infos"]],
                    "phase_s_per_step": {nm: round(float(v), 4) for nm, v in zip(
                        PHASES, np.sum([i["step_seconds"] for i in r["infos"]], axis=0) / steps)},
                    **summ[lab]}
              for lab, r in runs.items()}
    detail["autotune"] = [{"N": b, "variant": int(v), "tflops": [round(float(x), 2) for x in t]}
                          for (_, b), v, t in zip(tune_shapes, tv, ttf)]
    if not args.no_cpu_baseline:
        # about 1.2e13 flops of the oracle's filter (10-20 s on a few dozen
        # host cores), on problem 1's matrix copied to the host
        cols = int(max(16, min(k, round(1.2e13 / (8.0 * n * n * args.cpu_degree)))))
        est = 1.2e13 / 0.5e12 + n * n * 16 / 2e9
        if elapsed() + est > args.budget_s + 40:
            out["cpu_baseline"] = None
            del seq, a1, work, X, X1, runs
            log(f"cpu baseline skipped: {elapsed():.0f}s elapsed")
        else:
            a_host = a1.cpu().numpy()
            del seq, a1, work, X, X1, runs
            torch.cuda.empty_cache()
            log(f"timing the CPU oracle's filter on {cols} columns at degree {args.cpu_degree}")
            cb = cpu_baseline(a_host, cols, args.cpu_degree)
            # the oracle's filter alone at this rate, for the FP64 step's mat-vecs
            cb["filter_s_per_step_at_this_rate"] = round(flops / steps / (cb["value"] * 1e12), 1)
            out["cpu_baseline"] = cb
    log("detail " + json.dumps(detail))
    if args.detail_out:
        with open(args.detail_out, "w") as fh:
            json.dump({"line": out, "detail": detail}, fh, indent=1)
    line = json.dumps(out)
    if len(line) > 4000:
        log(f"result line is {len(line)} bytes; dropping the per-variant table")
        out.pop("variants", None)
        line = json.dumps(out)
    log(f"total {elapsed():.1f}s")
    print(line, flush=True)


if __name__ == "__main__":
    main()
