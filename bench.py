"""Benchmark: ChFSI on a sequence of dense generalized Hermitian eigenproblems.

One step = one call of chfsi_solve on the next problem of the sequence
(reduction to standard form, Lanczos bound, filter/QR/Rayleigh-Ritz/
residual/locking loops until nev pairs reach residual 1e-10, back-
transform), warm-started from the previous problem's Ritz vectors.

Default workload: generalized complex Hermitian A x = lambda B x,
n = 8000, nev = 400, nex = 80, B = I + 0.05 G (G random HPD of unit norm),
a 10-problem sequence with perturbations 1e-2 * 0.5^l.  The first problem
(random start) is the warm-up; the timed steps are warm-started problems.
All matrices are generated on the GPU from seeded host draws and are
resident in HBM before timing starts.

Printed (one JSON line): filter TFLOP/s (algorithmic 8 n^2 flops per
column mat-vec / device time of the filter-step kernels) as `value`, the
wall time per sequence step as `ms_per_step`, the roofline of the
filter-step kernel and the CPU oracle's filter rate on a bounded sample.
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

# HBM bytes of one full-width filter step (n = 8000, N = 480), from the two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) calibrated on a 1 GiB
# copy, per tile variant of the step kernel; valid only for the kernel
# source it was measured on.
TRAFFIC_MEASURED = {
    "zgemm_sha256": "8df37dde5efc6e7bda01d1ea51ab5cea363e65cd6970b6f321f9b3caf55a364e",
    "bytes_per_full_width_step": {0: 4.571e9, 1: 2.370e9, 2: 1.697e9},
    "algorithmic_bytes_per_full_width_step": 1.208e9,
}


def traffic_entry(variant):
    import hashlib
    src = os.path.join(ROOT, "paper_1404_4161_amd", "csrc", "zgemm.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if sha != TRAFFIC_MEASURED["zgemm_sha256"]:
        return None
    return round(TRAFFIC_MEASURED["bytes_per_full_width_step"][int(variant)] / 1e9, 3)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(a_host: np.ndarray, k: int, degree: int, seed: int = 0):
    """Time the CPU oracle's Chebyshev filter (Alg. 2) on a bounded sample:
    the n x n matrix of the workload and k columns at one degree."""
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
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle Chebyshev filter (Alg. 2), n={n}, {k} columns, degree {degree}, "
                      f"{dt:.1f} s on the host"}


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
    v, _ = ch.chfsi_autotune_filter([n], [k])
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
    q = ch.colmajor(torch.linalg.qr(y)[0])
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
    launches; FP64, FP64 with graph capture, mixed precision) against 32
    chfsi_solve calls per step (FP64).  Prints one JSON line."""
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
    log(f"autotune of {len(shapes)} shapes in {time.perf_counter() - t0:.1f}s: "
        f"variant 1 chosen for {int(tv.sum())}")

    def run(label, precision, batched, graph, serial=False):
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
                        graph=graph, serial=serial)
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
        "autotune": {"shapes": len(shapes), "variant1_chosen": int(tv.sum()),
                     "mean_tflops_kb8": round(float(ttf[:, 0].mean()), 2),
                     "mean_tflops_kb16": round(float(ttf[:, 1].mean()), 2)},
        "workload": "kpoints: 32 generalized complex Hermitian sequences, n uniform in "
                    "[2000, 9000], nev 5 %, nex 1 %, 5 steps (step 1 untimed)",
        "n": [c.n for c in confs], "steps": confs[0].length - 1,
        "speedup_batched_vs_sequential_fp64": (round(
            results["sequential fp64"]["s_per_step"] / results["batched fp64"]["s_per_step"], 3)
            if {"sequential fp64", "batched fp64"} <= set(results) else None),
        "variants": results,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=9)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gen-n8000",
                    choices=["gen-n8000", "std-n1000", "std-n20000", "std-n30000", "kpoints"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-degree", type=int, default=40)
    ap.add_argument("--filter-only", action="store_true",
                    help="time only the Chebyshev filter at the workload shape (n x k block, "
                         "uniform degree) after a 1 GiB device copy used to calibrate "
                         "hardware byte counters; for profiler runs")
    ap.add_argument("--degree", type=int, default=4)
    ap.add_argument("--kp-count", type=int, default=32,
                    help="k-point workload: number of problems (32 in the full workload)")
    ap.add_argument("--kp-variants", default="batched-fp64,batched-fp64-graph,sequential-fp64,"
                                             "batched-mixed,batched-mixed-bf16,"
                                             "batched-mixed-fp16")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip training the degree network and the learned-degree sequences")
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the sequences with BF16-split defect steps (precision 2)")
    ap.add_argument("--no-fp16", action="store_true",
                    help="skip the sequences with FP16-split defect steps (precision 3)")
    ap.add_argument("--train-steps", type=int, default=1500)
    ap.add_argument("--variants", default="",
                    help="comma list of the extra sequences to time (default all): "
                         "mixed+learned, fp64+learned, mixed+seqcal, fp64+seqcal, mixed-bf16, "
                         "mixed-bf16+seqcal, mixed-bf16+learned, mixed-fp16, mixed-fp16+seqcal, "
                         "mixed-fp16+learned (fp64 and mixed always run)")
    ap.add_argument("--no-lambda0", action="store_true",
                    help="warm-start from the previous Ritz vectors only (one extra QR + "
                         "Rayleigh-Ritz per problem) instead of vectors and values")
    args = ap.parse_args()
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
    total = args.warmup + args.steps
    if total > conf.length:
        log(f"warmup + steps = {total} exceeds the sequence length {conf.length}; "
            f"the sequence is extended with the same perturbation schedule")
        conf = gen.SequenceConfig(conf.name, conf.cfg, conf.n, conf.nev, conf.nex,
                                  conf.generalized, total, conf.delta, conf.b_weight, conf.tol,
                                  conf.deg0)
    dev = "cuda:0"
    t0 = time.perf_counter()
    # large problems draw their Gaussian matrices on the GPU (much faster)
    draw = "device" if conf.n > 10000 else "host"
    seq = gen.Sequence(conf, kind="torch", device=dev, draw=draw)
    problems = []
    for l, a in seq.problems():
        problems.append(a)
        if l >= total:
            break
    B = seq.B
    torch.cuda.synchronize()
    log(f"generated {len(problems)} problems (n={conf.n}) in {time.perf_counter() - t0:.1f}s")
    a1_host = problems[0].cpu().numpy() if not args.no_cpu_baseline else None

    n, nev, nex, k = conf.n, conf.nev, conf.nex, conf.k
    stream = torch.cuda.current_stream(dev)
    opts0 = ch.chfsi_default_opts()
    opts1 = ch.chfsi_default_opts()
    opts1.precision = 1
    opts2 = ch.chfsi_default_opts()
    opts2.precision = 2
    opts3 = ch.chfsi_default_opts()
    opts3.precision = 3
    wb = max(ch.chfsi_workspace_bytes(n, nev, nex, B is not None, o)
             for o in (opts0, opts1, opts2, opts3))
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    X = ch.colmajor(torch.empty((n, k), dtype=torch.complex128, device=dev))

    # Filter tile autotuner (untimed): both K-stage variants of the filter
    # step on the full window and narrower ones; later launches take the
    # choice of the nearest measured shape.
    tune_shapes = [(n, k), (n, (3 * k) // 4), (n, k // 2), (n, k // 4), (n, max(k // 8, 16))]
    tv, ttf = ch.chfsi_autotune_filter([a for a, _ in tune_shapes], [b for _, b in tune_shapes])
    autotune = [{"n": a, "N": b, "variant": int(v), "tflops_kb8": round(float(t[0]), 2),
                 "tflops_kb16": round(float(t[1]), 2), "tflops_wide": round(float(t[2]), 2)}
                for (a, b), v, t in zip(tune_shapes, tv, ttf)]
    log(f"autotune: {autotune}")

    # Degree network (untimed): convergence logs of a sequence with the same
    # recipe under another seed, then training with the library's kernels.
    blob, train_report = None, None
    if not args.no_learned:
        from paper_1404_4161_amd import learned
        t0 = time.perf_counter()
        tconf = gen.variant(conf, conf.cfg + 100)
        tseq = gen.Sequence(tconf, kind="torch", device=dev, draw=draw)
        tprobs = [a.clone() for l, a in tseq.problems() if l <= min(tconf.length, total)]
        buf = learned.LogBuffer(400_000)
        tw = torch.empty(wb, dtype=torch.uint8, device=dev)
        collect = []
        for prec, jit in ((0, 0.0), (0, 0.3)):
            o = ch.chfsi_default_opts()
            o.precision, o.first_rule, o.degree_jitter, o.seed = prec, 1, jit, 7
            its = [i["iters"] for i in learned.solve_sequence_logged(
                tprobs, tseq.B, nev, nex, conf.tol, o, buf, work=tw)]
            collect.append({"precision": prec, "jitter": jit, "iters": its})
        del tprobs, tseq, tw
        torch.cuda.empty_cache()
        tc = time.perf_counter()
        blob, train_report = learned.fit(buf.records(), steps=args.train_steps)
        train_report["train_seconds"] = round(time.perf_counter() - tc, 2)
        train_report["collect_seconds"] = round(tc - t0, 2)
        train_report["log_runs"] = collect
        train_report["training_sequence"] = f"{conf.name} recipe, seed namespace {tconf.cfg}"
        log(f"degree network: {train_report}")

    cold = {}

    def run_sequence(opts, label):
        """Warm-up problem(s), then the timed steps; returns per-step infos,
        wall times, eigenvalues and the elapsed time of the timed region."""
        x_prev, lam_prev = None, None
        rates = np.full(k, np.nan) if opts.degree_mode == 3 else None

        def solve(a):
            st, lam, x, info = ch.chfsi_solve(
                a, B, nev, nex, conf.tol, X0=x_prev, opts=opts, X=X, work=work, stream=stream,
                Lambda0=None if (args.no_lambda0 or x_prev is None) else lam_prev,
                mlp=blob if opts.degree_mode == 2 else None, seq_rates=rates)
            if st != 0:
                raise RuntimeError(f"chfsi_solve status {st}")
            return lam, info

        for w in range(args.warmup):
            lam_prev, info = solve(problems[w])
            x_prev = X
            log(f"[{label}] warmup problem {w + 1}: iters {info['iters']} total "
                f"{info['total_seconds']:.3f}s")
            if w == 0:
                # the cold first problem (random start block), untimed
                cold[label] = {"seconds": round(info["total_seconds"], 4),
                               "iters": info["iters"],
                               "filter_matvecs": info["filter_matvecs"]}
        torch.cuda.synchronize()
        infos, walls, lams = [], [], []
        t_start = time.perf_counter()
        for s_ in range(args.steps):
            ts = time.perf_counter()
            lam_prev, info = solve(problems[args.warmup + s_])
            x_prev = X
            walls.append(time.perf_counter() - ts)
            infos.append(info)
            lams.append(lam_prev[:nev].copy())
            log(f"[{label}] problem {args.warmup + s_ + 1}: iters {info['iters']} "
                f"(fp32 {info['filter_iters_fp32']}) filter {info['filter_seconds'] * 1e3:.1f} ms "
                f"step {walls[-1] * 1e3:.1f} ms")
        torch.cuda.synchronize()
        return infos, walls, lams, time.perf_counter() - t_start

    infos, walls, lams64, elapsed = run_sequence(opts0, "fp64")
    minfos, mwalls, lams32, melapsed = run_sequence(opts1, "mixed")
    # further variants: (label, precision, degree_mode, first_rule).  Mixed
    # precision keeps deg0 in the first loop of a warm start (FP32 defect
    # form); FP64 takes the first loop's degrees from X0's residuals.
    # degree_mode 2: the learned network; 3: Multiple Optimization (each
    # eigenvector's speed measured earlier in the sequence, no training).
    plan = []
    if blob is not None:
        plan += [("mixed+learned", 1, 2, 0), ("fp64+learned", 0, 2, 1)]
    plan += [("mixed+seqcal", 1, 3, 0), ("fp64+seqcal", 0, 3, 1)]
    if not args.no_bf16:
        plan += [("mixed-bf16", 2, 0, 0), ("mixed-bf16+seqcal", 2, 3, 0)]
        if blob is not None:
            plan.append(("mixed-bf16+learned", 2, 2, 0))
    if not args.no_fp16:
        plan += [("mixed-fp16", 3, 0, 0), ("mixed-fp16+seqcal", 3, 3, 0)]
        if blob is not None:
            plan.append(("mixed-fp16+learned", 3, 2, 0))
    if args.variants:
        keep = set(args.variants.split(","))
        plan = [p for p in plan if p[0] in keep]
    learned_runs = {}
    variant_modes = {}
    for label, prec, mode, fr in plan:
        o = ch.chfsi_default_opts()
        o.precision, o.degree_mode, o.first_rule = prec, mode, fr
        learned_runs[label] = run_sequence(o, label)
        variant_modes[label] = (prec, mode)

    flops = sum(i["filter_flops"] for i in infos)
    fsec = sum(i["filter_seconds"] for i in infos)
    launches = sum(i["filter_launches"] for i in infos)
    tflops = flops / fsec / 1e12
    avg_launch = fsec / launches
    phases = np.sum([i["step_seconds"] for i in infos], axis=0) / args.steps
    mphases = np.sum([i["step_seconds"] for i in minfos], axis=0) / args.steps
    phase_names = ["reduction", "lanczos", "filter", "orthonormalize", "rayleigh_ritz",
                   "residuals", "locking", "back_transform"]
    mflops = sum(i["filter_flops"] for i in minfos)
    msec = sum(i["filter_seconds"] for i in minfos)
    f32_flops = sum(i["filter_flops_fp32"] for i in minfos)
    f32_sec = sum(i["filter_seconds_fp32"] for i in minfos)
    eig_diff = [float(np.max(np.abs(a - b) / np.abs(a))) for a, b in zip(lams64, lams32)]
    out = {
        "metric": "filter TFLOP/s + s/sequence-step at 1e-10 residual, FP64 vs mixed+learned",
        "value": round(tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{conf.name}: {'generalized' if B is not None else 'standard'} complex "
                         f"Hermitian sequence, n={n}, nev={nev}, nex={nex}, tol={conf.tol}, "
                         f"FP64 filter (complex, 4M split on MFMA)"),
            "n": n, "nev": nev, "nex": nex, "problems_timed": args.steps,
            "warm_start": "X0 only" if args.no_lambda0 else "X0 and Lambda0",
        },
        "s_per_sequence_step_median": round(statistics.median(walls), 4),
        "filter_tflops_over_wall": round(flops / elapsed / 1e12, 3),
        "filter_share_of_step": round(fsec / elapsed, 3),
        "phase_seconds_per_step": {nm: round(float(v), 4) for nm, v in zip(phase_names, phases)},
        "iters_per_step": [i["iters"] for i in infos],
        "rr_eigensolves_refined_dense": [sum(i["rr_refined"] for i in infos),
                                         sum(i["rr_dense"] for i in infos)],
        "b_factor_reused_per_step": [i["b_factor_reused"] for i in infos],
        "roofline": {
            "kernel": "zgemm_kernel<OP_N, OP_N, EPI_CHEB> (Chebyshev filter step)",
            "bound": "mfma",
            "achieved": round(tflops, 3),
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(tflops / PEAK_FP64_TFLOPS, 4),
            "traffic": traffic_entry(tv[0]),
            "tile_variant_full_width": int(tv[0]),
            "traffic_unit": "GB per full-width step (n=8000, N=480), HBM, from FETCH_SIZE/WRITE_SIZE",
            "algorithmic_bytes_full_width_gb": 1.208,
            "avg_launch_us": round(avg_launch * 1e6, 2),
            "launches": launches,
        },
        "mixed": {
            "precision": "FP32 defect filter where the residuals allow, FP64 QR/RR/residuals",
            "ms_per_step": round(1e3 * melapsed / args.steps, 3),
            "s_per_sequence_step_median": round(statistics.median(mwalls), 4),
            "speedup_vs_fp64_per_step": round(elapsed / melapsed, 3),
            "filter_effective_tflops": round(mflops / msec / 1e12, 3),
            "fp32_gemm_tflops": round(f32_flops / f32_sec / 1e12, 3) if f32_sec > 0 else None,
            "fp32_peak_tflops": 157.3,
            "fp32_filter_loops_per_step": [i["filter_iters_fp32"] for i in minfos],
            "iters_per_step": [i["iters"] for i in minfos],
            "phase_seconds_per_step": {nm: round(float(v), 4) for nm, v in zip(phase_names, mphases)},
            "max_rel_eig_diff_vs_fp64_per_step": eig_diff,
        },
    }
    precision_text = {
        0: "FP64 filter",
        1: "FP32 defect filter where the residuals allow",
        2: ("FP32 defect filter where the residuals allow; its early steps with BF16-split "
            "products (3 BF16 MFMA products, FP32 accumulate) where their rounding is damped "
            "enough"),
        3: ("FP32 defect filter where the residuals allow; its steps with FP16-split products "
            "of power-of-two scaled operands (3 FP16 MFMA products, FP32 accumulate) where "
            "their rounding is damped enough (nearly all)"),
    }
    degree_text = {
        0: "analytic rule (Sec. 3.1.1)",
        2: "learned (network trained on logs of another sequence; rule fallback)",
        3: "sequence-calibrated (speeds measured earlier in the sequence; rule floor)",
    }
    for label, (linfos, lwalls, llams, lelapsed) in learned_runs.items():
        lph = np.sum([i["step_seconds"] for i in linfos], axis=0) / args.steps
        prec, mode = variant_modes[label]
        out[label] = {
            "precision": precision_text[prec],
            "degrees": degree_text[mode],
            "first_loop_degrees": ("deg0" if prec >= 1 else
                                   "from the residuals of X0 (one extra product H X0)"),
            "ms_per_step": round(1e3 * lelapsed / args.steps, 3),
            "s_per_sequence_step_median": round(statistics.median(lwalls), 4),
            "speedup_vs_fp64_per_step": round(elapsed / lelapsed, 3),
            "iters_per_step": [i["iters"] for i in linfos],
            "rr_eigensolves_refined_dense": [sum(i["rr_refined"] for i in linfos),
                                             sum(i["rr_dense"] for i in linfos)],
            "fp32_filter_loops_per_step": [i["filter_iters_fp32"] for i in linfos],
            "filter_matvecs_per_step": [i["filter_matvecs"] for i in linfos],
            "learned_cols": sum(i["learned_cols"] for i in linfos),
            "fallback_cols": sum(i["fallback_cols"] for i in linfos),
            "learned_raised_cols": sum(i["learned_raised"] for i in linfos),
            "phase_seconds_per_step": {nm: round(float(v), 4) for nm, v in zip(phase_names, lph)},
            "max_rel_eig_diff_vs_fp64_per_step": [
                float(np.max(np.abs(a - b) / np.abs(a))) for a, b in zip(lams64, llams)],
        }
        if prec >= 2:
            w = "bf16" if prec == 2 else "fp16"
            f16 = sum(i[f"filter_flops_{w}"] for i in linfos)
            f32 = sum(i["filter_flops_fp32"] for i in linfos)
            out[label][f"{w}_steps_per_step"] = [i[f"filter_steps_{w}"] for i in linfos]
            out[label][f"{w}_share_of_defect_flops"] = round(f16 / max(f16 + f32, 1.0), 3)
            lsec = sum(i["filter_seconds"] for i in linfos)
            out[label]["filter_effective_tflops"] = round(
                sum(i["filter_flops"] for i in linfos) / lsec / 1e12, 3)
    # the metric's comparison: FP64 against the fastest mixed-precision
    # variant with learned degrees
    ml = [lab for lab in learned_runs if lab.startswith("mixed") and lab.endswith("+learned")]
    if ml:
        best = min(ml, key=lambda lab: out[lab]["ms_per_step"])
        out["fp64_vs_mixed_learned"] = {
            "fp64_ms_per_step": out["ms_per_step"],
            "variant": best,
            "ms_per_step": out[best]["ms_per_step"],
            "speedup": out[best]["speedup_vs_fp64_per_step"],
            "max_rel_eig_diff_vs_fp64": max(out[best]["max_rel_eig_diff_vs_fp64_per_step"]),
        }
    out["fp64_filter_matvecs_per_step"] = [i["filter_matvecs"] for i in infos]
    out["cold_first_problem_untimed"] = cold
    out["filter_autotune"] = autotune
    if train_report is not None:
        out["degree_network"] = train_report
    if not args.no_cpu_baseline:
        del problems
        torch.cuda.empty_cache()
        log("timing the CPU oracle's filter on a bounded sample")
        # a bounded sample: about k (8000 / n)^2 columns (all of them at n = 8000)
        cols = max(16, min(k, int(round(k * (8000.0 / n) ** 2))))
        out["cpu_baseline"] = cpu_baseline(a1_host, cols, args.cpu_degree)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
