"""Benchmark of the single-trait IHT hot path on one MI355X.

One step = one complete solve on the n=5000 x p=500,000 workload (2-bit PLINK, 625 MB, k=20):
the per-SNP mean/precision pass over the subject set plus the IHT fit to convergence, starting
from the packed genotypes already resident (re-tiled once) in HBM. The reported value is the
gradient passes' algorithmic bytes (ceil(n/4) * p per pass) divided by the whole-solve wall time.

Further sections on the same JSON line: the 108-solve batched layout on the same matrix (int8
matrix cores), cross-validation, logistic IHT, the continuous-batching server on n=10,000 x
p=1,000,000 (saturated, then Poisson streams at 0.5 / 0.8 / 1.0 of capacity), the n=20,000 x
p=2,000,000 workload (96 batched solves against the plain FP64 loop) and the oracle on the host.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|fp32] [--seed S]
                       [--no-cpu-baseline] [--pass-reps R] [--small] [--copy-calibration]
                       [--no-batched] [--no-serving] [--no-c5] [--serve-requests R]
                       [--passes-only single|batched]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "X'r pass GB/s (% HBM peak); batched solves/s + p99 latency vs plain IHT"
HBM_PEAK_GBS = 8000.0
INT8_PEAK_TOPS = 5000.0  # dense int8 matrix-core peak, TOP/s


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def pass_traffic():
    """HBM bytes per FP64 pass launch at n=5000, p=500,000 from the committed counter summary, or None when
    the pass source has changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_pass_c2_hbm_traffic.txt")
    src = os.path.join(ROOT, "paper_1608_01398_amd", "csrc", "iht_pass.hip")
    try:
        txt = open(path).read()
        cur = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m = re.search(r"iht_pass\.hip sha256 ([0-9a-f]{64})", txt)
    t = re.search(r"traffic_bytes_per_launch_fp64: (\d+)", txt)
    if not m or not t or m.group(1) != cur:
        return None
    return int(t.group(1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--pass-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--small", action="store_true", help="n=1000, p=10,000 workload (the oracle-sized case)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-solves section")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving section (n=10,000, p=1,000,000)")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--no-c5", action="store_true", help="skip the n=20,000 x p=2,000,000 section (10 GB packed)")
    ap.add_argument("--oracle-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--passes-only", choices=["single", "batched"], default=None,
                    help="launch only the gradient passes of the workload (3 FP64 + 3 FP32 single-trait calls, or 3 "
                         "matrix-core calls for 108 random residual rows) and exit: for hardware-counter runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also launch one fill and one device-to-device copy of the packed matrix's size, "
                         "the known-size kernels that scale the HBM byte counters")
    args = ap.parse_args()

    if args.oracle_child:
        oracle_child(args)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on exactly one GPU; multi-GPU runs are not part of it "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    from paper_1608_01398_amd import iht, synth

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    cfg = "c1" if args.small else "c2"
    prec = iht.FP64 if args.precision == "fp64" else iht.FP32

    t = time.time()
    prob = synth.make_problem(cfg, args.seed)
    n, p, k = prob["n"], prob["p"], prob["k"]
    log(f"generated {cfg}: n={n} p={p} k={k} in {time.time() - t:.1f}s")
    row = (n + 3) // 4
    pass_bytes = row * p

    t = time.time()
    geno = iht.Geno(prob["bed"], n)
    torch.cuda.synchronize()
    log(f"upload + re-tile: {time.time() - t:.2f}s (host bytes {prob['bed'].nbytes / 1e6:.0f} MB)")
    y = torch.from_numpy(prob["y"]).cuda()

    if args.copy_calibration:
        src = torch.empty(pass_bytes, dtype=torch.uint8, device="cuda")
        src.fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: fill + copy of {pass_bytes} bytes")
        del src, dst

    if args.passes_only:
        stats = iht.Stats(geno)
        if args.passes_only == "single":
            g = torch.empty(p, dtype=torch.float64, device="cuda")
            for precision in (iht.FP64, iht.FP32):
                for _ in range(3):
                    iht.gradient(geno, stats, y, precision, out=g)
        else:
            T = 108
            R = torch.randn((T, n), dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(1))
            G = torch.empty((T, p), dtype=torch.float64, device="cuda")
            for _ in range(3):
                iht.gradient_batch(geno, [stats] * T, R, out=G)
        torch.cuda.synchronize()
        log(f"passes only ({args.passes_only}): done")
        return

    def solve():
        stats = iht.Stats(geno)
        res = iht.fit(geno, stats, y, k, intercept=True, precision=prec)
        return res

    for w in range(args.warmup):
        res = solve()
        log(f"warmup {w}: status {res['status']} iters {res['n_iter']}")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    passes = 0
    iters = []
    for s in range(args.steps):
        res = solve()
        iters.append(res["n_iter"])
        passes += res["n_iter"] + 1
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"timed {args.steps} solves in {elapsed:.3f}s; iterations {iters}")
    value = passes * pass_bytes / elapsed / 1e9
    gpu_support = res["support"].cpu().numpy()
    gpu_beta = res["beta_S"].cpu().numpy()
    gpu_loss = float(res["loss_trace"][-1].item())

    # Dominant kernel: the gradient pass, timed alone with events on the stream it is launched on.
    stats = iht.Stats(geno)
    r = y.clone()
    g = torch.empty(p, dtype=torch.float64, device="cuda")
    for _ in range(3):
        iht.gradient(geno, stats, r, prec, out=g)
    torch.cuda.synchronize()
    g0_gpu = g.cpu().numpy().copy()  # the gradient at beta = 0 (r = y), for the oracle comparison
    stream = torch.cuda.current_stream()
    # one event between consecutive calls: the mean over the back-to-back run and each call's time
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.pass_reps + 1)]
    ev[0].record(stream)
    for i in range(args.pass_reps):
        iht.gradient(geno, stats, r, prec, out=g)
        ev[i + 1].record(stream)
    ev[-1].synchronize()
    pass_ms = ev[0].elapsed_time(ev[-1]) / args.pass_reps
    per_call_us = np.array([ev[i].elapsed_time(ev[i + 1]) * 1e3 for i in range(args.pass_reps)])
    achieved = pass_bytes / (pass_ms * 1e-3) / 1e9
    log(f"gradient pass: {pass_ms * 1e3:.1f} us, {achieved:.0f} GB/s ({achieved / HBM_PEAK_GBS:.1%} of HBM peak); "
        f"per call p10/p50/p90 {np.percentile(per_call_us, 10):.1f}/{np.percentile(per_call_us, 50):.1f}/"
        f"{np.percentile(per_call_us, 90):.1f} us")

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == iht.FP64 else "f32 table entries, f64 accumulation",
        "data": "synthetic HWE genotypes, MAF~U(0.05,0.5), 1% missing, seeded",
        "config": {
            "workload": f"single-trait IHT solve (per-SNP stats pass + fit to convergence), n={n}, p={p}, "
                        f"packed 2-bit PLINK {n * p / 4e6:.0f} MB resident in HBM, k={k}, intercept",
            "n": n, "p": p, "k": k, "seed": args.seed, "precision": args.precision,
            "gradient_passes": passes, "iterations_per_solve": float(np.mean(iters)),
        },
        "solves_per_s": round(args.steps / elapsed, 3),
        "hbm_frac_whole_solve": round(value / HBM_PEAK_GBS, 4),
        "roofline": {
            "bound": "hbm",
            "kernel": "one iht_gradient call, g = X_st^T r: k_center + k_pass + k_pass_finalize",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": pass_traffic() if (prec == iht.FP64 and cfg == "c2") else None,
            "traffic_unit": "HBM bytes per call (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "launch_us": round(pass_ms * 1e3, 2),
            "launch_us_p10_p50_p90": [round(float(np.percentile(per_call_us, q)), 2) for q in (10, 50, 90)],
            "algorithmic_bytes_per_launch": pass_bytes,
            # residual read, u and v read, g written: not credited to the pass
            "aux_bytes_per_launch": 8 * n + 24 * p,
        },
    }

    if not args.no_batched and not args.small:
        out["batched"] = bench_batched(args, torch, iht, synth, prob, geno, y, pass_bytes)
        out["cv"] = bench_cv(args, torch, iht, synth, prob, geno, y)
    if not args.no_batched and not args.small:
        out["logistic"] = bench_logistic(args, torch, iht, synth, prob, geno)
    if not args.no_serving and not args.small:
        out["serving"] = bench_serving(args, torch, iht, synth)
    if not args.no_c5 and not args.small:
        out["c5"] = bench_c5(args, torch, iht, synth)

    if not args.no_cpu_baseline:
        from oracle import oracle

        cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
        log(f"oracle: one full FP64 solve on the same data ({cores} threads)")
        t = time.perf_counter()
        ref = oracle.fit(prob["bed"], n, prob["y"], k, intercept=True)
        ct = time.perf_counter() - t
        cpasses = ref["n_iter"] + 1
        cval = cpasses * pass_bytes / ct / 1e9
        out["cpu_baseline"] = {
            "value": round(cval, 3), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"one complete oracle solve of the same workload (stats + {ref['n_iter']} iterations, "
                      f"{cpasses} gradient passes) in {ct:.1f}s",
        }
        nproc = os.cpu_count()
        t1 = oracle_timings(args, 1)
        tn = oracle_timings(args, cores)
        out["cpu_baseline"]["host_cpu"] = cpu_model()
        out["cpu_baseline"]["host_logical_cpus"] = nproc
        out["cpu_baseline"]["timings"] = {"threads_1": t1, f"threads_{cores}": tn}
        if t1 and tn:
            log(f"oracle timings ({cpu_model()}, {nproc} logical CPUs): n=1000 fit {t1['c1_fit_s_median_of_5']:.3f} s "
                f"(1 thread) / {tn['c1_fit_s_median_of_5']:.3f} s ({cores}); n=5000 x p=500,000 pass "
                f"{t1['c2_pass_gbs']:.3f} GB/s (1 thread) / {tn['c2_pass_gbs']:.3f} GB/s ({cores})")
        same = bool(np.array_equal(gpu_support, ref["support"]))
        brel = float(np.abs(gpu_beta - ref["beta_S"]).max() / np.abs(ref["beta_S"]).max()) if same else None
        lrel = float(abs(gpu_loss - ref["loss_trace"][-1]) / abs(ref["loss_trace"][-1]))
        # the gradient at beta = 0 (r = y), against the oracle's own stats and pass
        ou, ov = oracle.stats(prob["bed"], n)
        g_ref = oracle.gradient(prob["bed"], n, ou, ov, prob["y"])
        grel = float(np.linalg.norm(g0_gpu - g_ref) / np.linalg.norm(g_ref))
        out["parity"] = {"support_equal": same, "beta_max_rel_err": brel, "loss_rel_diff": lrel,
                         "gradient_rel_l2_err_at_beta0": grel,
                         "iterations_gpu": int(iters[-1]), "iterations_oracle": int(ref["n_iter"]),
                         "delta_iterations": int(iters[-1]) - int(ref["n_iter"])}
        log(f"oracle: {ct:.1f}s, {cval:.2f} GB/s; support equal {same}, beta rel err {brel}, loss rel diff {lrel:.2e}, "
            f"gradient rel L2 err {grel:.2e}")
        if "batched" in out:
            smp = out["batched"]["_sample"]
            t = time.perf_counter()
            rb = oracle.fit(prob["bed"], n, smp["y"], smp["k"], intercept=True, subset=smp["mask"])
            bsame = bool(np.array_equal(smp["support"], rb["support"]))
            bre = (float(np.abs(smp["beta_S"] - rb["beta_S"]).max() / np.abs(rb["beta_S"]).max()) if bsame else None)
            out["batched"]["parity_sample"] = {"solve": smp["t"], "support_equal": bsame, "beta_max_rel_err": bre}
            log(f"oracle, batched solve {smp['t']} (fold 0, k={smp['k']}): {time.perf_counter() - t:.1f}s; "
                f"support equal {bsame}, beta rel err {bre}")

    if "batched" in out:
        out["batched"].pop("_sample", None)
    print(json.dumps(out), flush=True)


def time_gradient(torch, iht, geno, stats, r, reps, precision=0):
    """Mean and per-call times (us) of back-to-back iht_gradient calls, HIP events on the launch stream."""
    g = torch.empty(geno.p, dtype=torch.float64, device="cuda")
    for _ in range(3):
        iht.gradient(geno, stats, r, precision, out=g)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for i in range(reps):
        iht.gradient(geno, stats, r, precision, out=g)
        ev[i + 1].record(stream)
    ev[-1].synchronize()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) * 1e3 for i in range(reps)])
    return ev[0].elapsed_time(ev[-1]) * 1e3 / reps, per


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_child(args):
    """Oracle timings in a process of its own (its OpenMP thread count is fixed at start): one fit on the
    n=1000 x p=10,000 workload (median of 5 after a warm-up) and one gradient pass on n=5000 x p=500,000."""
    from oracle import oracle
    from paper_1608_01398_amd import synth

    c1 = synth.make_problem("c1", args.seed)
    oracle.fit(c1["bed"], c1["n"], c1["y"], c1["k"], intercept=True)
    ts = []
    for _ in range(5):
        t = time.perf_counter()
        oracle.fit(c1["bed"], c1["n"], c1["y"], c1["k"], intercept=True)
        ts.append(time.perf_counter() - t)
    c2 = synth.make_problem("c2", args.seed)
    u, v = oracle.stats(c2["bed"], c2["n"])
    t = time.perf_counter()
    oracle.gradient(c2["bed"], c2["n"], u, v, c2["y"])
    tp = time.perf_counter() - t
    print(json.dumps({"c1_fit_s_median_of_5": float(np.median(ts)), "c2_pass_s": tp,
                      "c2_pass_gbs": (c2["n"] + 3) // 4 * c2["p"] / tp / 1e9}), flush=True)


def oracle_timings(args, threads):
    import subprocess

    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-child", "--seed", str(args.seed)],
                         env=env, capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        log(f"oracle child ({threads} threads) failed: {out.stderr[-500:]}")
        return None
    return json.loads(out.stdout.strip().splitlines()[-1])


def fold_masks(n, q, seed):
    rng = np.random.default_rng(seed)
    fold = rng.permutation(np.arange(n) % q)
    return [(fold != f).astype(np.uint8) for f in range(q)] + [np.ones(n, dtype=np.uint8)]


def bench_batched(args, torch, iht, synth, prob, geno, y, pass_bytes):
    """108 solves on the same resident matrix: 5 training folds x k = 1..20 on the trait, plus 8 more
    traits (same generator, k = 20, all subjects), in one mixed-precision batched call, against the
    plain FP64 per-solve loop (iht_fit once per solve) on the same GPU."""
    n, p = prob["n"], prob["p"]
    masks = fold_masks(n, 5, args.seed)
    traits = [prob["y"]]
    for e in range(8):
        ye, *_ = synth.make_trait(prob["bed"], n, prob["q"], prob["k"], (0.1, 0.4), seed=1000 + e)
        traits.append(ye)
    solves = [(f, 0, k) for f in range(5) for k in range(1, 21)] + [(5, 1 + e, 20) for e in range(8)]
    T = len(solves)
    stats_by_mask = [iht.Stats(geno, m) for m in masks]
    stats = [stats_by_mask[f] for f, _, _ in solves]
    Y = torch.from_numpy(np.stack([traits[tr] for _, tr, _ in solves])).cuda()
    ks = [k for _, _, k in solves]

    res = iht.fit_batch(geno, stats, Y, ks, precision=iht.MIXED_I8)  # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(args.batch_steps):
        t0 = time.perf_counter()
        res = iht.fit_batch(geno, stats, Y, ks, precision=iht.MIXED_I8)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    bt = float(np.median(times))
    iters = np.asarray(res["n_iter"])
    log(f"batched: {T} solves in {bt * 1e3:.1f} ms (median of {len(times)}), statuses "
        f"{np.bincount(np.asarray(res['statuses']) + 4, minlength=7)[4:].tolist()} (ok/not conv/stalled), "
        f"iterations {iters.min()}..{iters.max()}")

    # plain loop: one FP64 iht_fit per solve, one after another
    iht.fit(geno, stats[0], Y[0], ks[0])
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for t in range(T):
        a = time.perf_counter()
        iht.fit(geno, stats[t], Y[t], ks[t])
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t0
    log(f"plain FP64 loop: {T} solves in {plain * 1e3:.1f} ms")
    iht.fit(geno, stats[0], Y[0], ks[0], precision=iht.FP32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(T):
        iht.fit(geno, stats[t], Y[t], ks[t], precision=iht.FP32)
    torch.cuda.synchronize()
    plain32 = time.perf_counter() - t0
    log(f"plain FP32 loop: {T} solves in {plain32 * 1e3:.1f} ms")
    # the matrix-core pass alone, all 108 solves (HIP events on the launch stream)
    R = torch.randn((T, n), dtype=torch.float64, device="cuda")
    G = torch.empty((T, p), dtype=torch.float64, device="cuda")
    for _ in range(2):
        iht.gradient_batch(geno, stats, R, out=G)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record(stream)
    for _ in range(reps):
        iht.gradient_batch(geno, stats, R, out=G)
    e1.record(stream)
    e1.synchronize()
    bpass_ms = e0.elapsed_time(e1) / reps
    # algorithmic work: 2 n p T s int8 operations with s = 3 residual digits (the products with the
    # missing-genotype flags, done on the matrix cores too, are not credited)
    ops = 2.0 * n * p * T * 3
    tops = ops / (bpass_ms * 1e-3) / 1e12
    log(f"batched pass (T={T}): {bpass_ms * 1e3:.1f} us, {tops:.0f} TOP/s int8 credited ({tops / INT8_PEAK_TOPS:.1%} of "
        f"peak; {2 * tops:.0f} TOP/s with the missing-flag products), "
        f"{T * pass_bytes / (bpass_ms * 1e-3) / 1e9:.0f} GB/s-equivalent of single-trait passes")
    return {
        "workload": f"{T} solves on the resident n={n} x p={p} matrix: 5 training folds x k=1..20 on one trait "
                    "+ 8 traits at k=20 on all subjects; int8 matrix-core gradient, FP64 decisions",
        "solves": T,
        "solves_per_s": round(T / bt, 2),
        "ms_per_batch": round(bt * 1e3, 2),
        "ms_per_batch_runs": [round(x * 1e3, 2) for x in times],
        "latency_note": "every solve of a batch completes when the call returns: solve latency = batch time "
                        "(median of the timed batches above); request latency percentiles are in the serving section",
        "plain_fp64_loop_solves_per_s": round(T / plain, 2),
        "plain_fp64_solve_latency_ms_p50": round(float(np.percentile(np.asarray(lat) * 1e3, 50)), 2),
        "plain_fp64_solve_latency_ms_p99": round(float(np.percentile(np.asarray(lat) * 1e3, 99)), 2),
        "speedup_vs_plain_fp64_loop": round(plain / bt, 2),
        "plain_fp32_loop_solves_per_s": round(T / plain32, 2),
        "speedup_vs_plain_fp32_loop": round(plain32 / bt, 2),
        "iterations_mean": round(float(iters.mean()), 2),
        "pass_block_snps_autotuned": iht.batch_tuning(geno, T),
        "statuses": [int(x) for x in np.asarray(res["statuses"])],
        "roofline": {
            "bound": "mfma", "kernel": "k_gradB (int8 matrix-core pass, all 108 solves)",
            "achieved": round(tops, 1), "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
            "frac": round(tops / INT8_PEAK_TOPS, 4), "traffic": None, "launch_us": round(bpass_ms * 1e3, 1),
            "algorithmic_ops_per_launch": ops,
            "ops_note": "2 n p T x 3 residual digits; the missing-flag products (another 2 n p T x 3) not credited",
        },
        "_sample": dict(t=19, mask=masks[solves[19][0]], y=traits[solves[19][1]], k=solves[19][2],
                        support=res["support"][19, :solves[19][2]].cpu().numpy(),
                        beta_S=res["beta_S"][19, :solves[19][2]].cpu().numpy()),
    }


def bench_cv(args, torch, iht, synth, prob, geno, y):
    """Model selection as the paper runs it: 5-fold cross-validation over k = 1..20 (training stats,
    100 training fits as one batch, held-out MSE, refit at the chosen k), timed end to end per
    precision; the refit scored by precision, recall and estimated heritability against the
    generator's causal SNPs."""
    n = prob["n"]
    q, ks = 5, list(range(1, 21))
    folds = synth.make_folds(n, q, args.seed)
    full = iht.Stats(geno)
    causal = np.asarray(prob["causal"], dtype=np.int64)
    vy = float(np.var(prob["y"]))
    # h2 = Var(X_st beta) / Var(y) (Results, "Simulation"); the true model standardised by the sample
    g_true = iht.predict(geno, full, torch.from_numpy(causal).cuda(),
                         torch.from_numpy(np.asarray(prob["beta_true"], dtype=np.float64)).cuda())
    h2_true = float(torch.var(g_true, unbiased=False).item()) / vy
    res = {"workload": f"{q}-fold CV over k=1..{ks[-1]} on the resident n={n} x p={prob['p']} matrix, then the refit",
           "folds": q, "path": [ks[0], ks[-1]], "h2_true": round(h2_true, 4)}
    for name, prec in (("mixed_i8", iht.MIXED_I8), ("fp64", iht.FP64)):
        iht.cv(geno, y, ks, folds, q, precision=prec)  # warm-up
        torch.cuda.synchronize()
        times = []
        for _ in range(args.batch_steps):
            t0 = time.perf_counter()
            cvr = iht.cv(geno, y, ks, folds, q, precision=prec)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        ct = float(np.median(times))
        sup = cvr["refit"]["support"].cpu().numpy()
        hit = int(np.intersect1d(sup, causal).size)
        pred = iht.predict(geno, full, cvr["refit"]["support"], cvr["refit"]["beta_S"])
        h2 = float(torch.var(pred, unbiased=False).item()) / vy
        res[name] = {"ms": round(ct * 1e3, 2), "training_fits_per_s": round(q * len(ks) / ct, 1),
                     "k_best": cvr["k_best"], "precision": round(hit / len(sup), 4),
                     "recall": round(hit / len(causal), 4), "h2_est": round(h2, 4),
                     "mean_mse": [round(float(x), 5) for x in cvr["mse"].mean(1)]}
        log(f"cv {name}: {ct * 1e3:.1f} ms (median of {len(times)}), k_best {cvr['k_best']}, "
            f"precision {hit}/{len(sup)}, recall {hit}/{len(causal)}, h2 est {h2:.3f} (true {h2_true:.3f})")
    res["same_choice"] = res["mixed_i8"]["k_best"] == res["fp64"]["k_best"]
    return res


def bench_logistic(args, torch, iht, synth, prob, geno):
    """Logistic IHT (FP64) on the same resident matrix: a case/control trait with the workload's
    20 causal SNPs, k = 20, timed per solve (statistics included)."""
    n = prob["n"]
    yb, causal, _ = synth.make_binary_trait(prob["bed"], n, prob["q"], 20, (0.1, 0.4), seed=args.seed + 900)
    y = torch.from_numpy(yb).cuda()
    res = iht.fit(geno, iht.Stats(geno), y, 20, family=iht.LOGISTIC)  # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        res = iht.fit(geno, iht.Stats(geno), y, 20, family=iht.LOGISTIC)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ms = float(np.median(times)) * 1e3
    hit = int(np.intersect1d(res["support"].cpu().numpy(), causal).size)
    log(f"logistic: {ms:.2f} ms per solve, {res['n_iter']} iterations, status {res['status']}, "
        f"{hit}/20 causal SNPs recovered")
    return {"workload": f"logistic IHT, n={n} x p={prob['p']}, case/control trait, k=20, FP64",
            "ms_per_solve": round(ms, 2), "iterations": res["n_iter"], "status": res["status"],
            "causal_recovered": hit}


def request_stream(n, count, seed):
    """Seeded serving requests: subject subsets of U{2000..n} subjects, 1..64 traits, k ~ U{5..50}."""
    rng = np.random.default_rng([seed, 77])
    reqs = []
    for i in range(count):
        T = int(rng.integers(1, 65))
        reqs.append(dict(size=int(rng.integers(2000, n + 1)), T=T, ks=rng.integers(5, 51, T).astype(np.int32),
                         row0=int(rng.integers(0, 64 - T + 1)), seed=1000 + i))
    return reqs


def serve(iht, torch, srv, reqs, subsets, pool, arrivals=None):
    """Feeds the requests to the server (all at once, or at the given arrival times in seconds) and
    steps it until every request is done; returns (wall seconds, per-request latencies, ids)."""
    t0 = time.perf_counter()
    pending = list(range(len(reqs)))
    live = {}
    lat = [None] * len(reqs)
    ids = [None] * len(reqs)
    while pending or live:
        now = time.perf_counter() - t0
        while pending and (arrivals is None or arrivals[pending[0]] <= now):
            i = pending.pop(0)
            r = reqs[i]
            ids[i] = srv.submit(pool[r["row0"]:r["row0"] + r["T"]], r["ks"], subsets[i])
            live[ids[i]] = (i, t0 + (0.0 if arrivals is None else arrivals[i]))
        if not live:
            time.sleep(max(0.0, arrivals[pending[0]] - now))
            continue
        if srv.step():
            t = time.perf_counter()
            for rid in [rid for rid in live if srv.done(rid)]:
                i, a = live.pop(rid)
                lat[i] = t - a
    return time.perf_counter() - t0, np.asarray(lat), ids


def bench_serving(args, torch, iht, synth):
    """Continuous-batching server on the n=10,000 x p=1,000,000 matrix (2.5 GB resident): requests
    with their own subject subsets, 1..64 traits and k ~ U{5..50}, int8 matrix-core gradient with the
    FP64 iteration's decisions. Saturated (every request queued at once) for solves/s, then Poisson
    streams at 0.5, 0.8 and 1.0 of that rate for latency; against a plain loop of FP64 iht_fit calls
    on the first solves of the stream. Also: the single-trait gradient pass at this size."""
    t = time.time()
    prob = synth.make_problem("c4", args.seed)
    n, p = prob["n"], prob["p"]
    geno = iht.Geno(prob["bed"], n)
    pool = [prob["y"]] + [synth.make_trait(prob["bed"], n, prob["q"], 20, (0.1, 0.4), seed=5000 + e)[0]
                          for e in range(63)]
    pool = torch.from_numpy(np.stack(pool)).cuda()
    reqs = request_stream(n, args.serve_requests, args.seed)
    subsets = [synth.make_subset(n, r["size"], r["seed"]) if r["size"] < n else None for r in reqs]
    traits = int(sum(r["T"] for r in reqs))
    log(f"serving: c4 n={n} p={p} ({n * p / 4e9:.1f} GB packed) ready in {time.time() - t:.1f}s; "
        f"{len(reqs)} requests, {traits} solves")
    pass_us, _ = time_gradient(torch, iht, geno, iht.Stats(geno), pool[0].contiguous(), 20)
    pass_gbs = (n + 3) // 4 * p / (pass_us * 1e-6) / 1e9
    log(f"gradient pass at n={n} x p={p}: {pass_us:.1f} us = {pass_gbs:.0f} GB/s ({pass_gbs / HBM_PEAK_GBS:.1%} of HBM peak)")
    slots, kmax, budget = 256, 50, 24 << 30
    srv = iht.Server(geno, slots=slots, kmax=kmax, hbm_budget=budget, precision=iht.MIXED_I8)
    info0 = srv.info()
    # warm-up: one small request
    srv.submit(pool[:2], [10, 20], subsets[0])
    srv.run_until_idle()
    wall, lat_sat, ids = serve(iht, torch, srv, reqs, subsets, pool)
    sat_rate = traits / wall
    log(f"serving saturated: {traits} solves in {wall:.2f}s = {sat_rate:.0f} solves/s; request latency "
        f"p50 {np.percentile(lat_sat, 50) * 1e3:.0f} ms p99 {np.percentile(lat_sat, 99) * 1e3:.0f} ms; "
        f"{srv.info()['turns'] - info0['turns']} turns")
    # the served results of a few solves against the same solves alone (bitwise)
    same, fp64_same, fp64_beta_err = True, True, 0.0
    checked = 0
    for i in (0, len(reqs) // 2, len(reqs) - 1):
        res = srv.result(ids[i])
        r = reqs[i]
        j = r["T"] - 1
        st = iht.Stats(geno, subsets[i])
        a = iht.fit(geno, st, pool[r["row0"] + j].contiguous(), int(r["ks"][j]), precision=iht.MIXED_I8)
        k = int(r["ks"][j])
        same &= bool(torch.equal(a["support"], res["support"][j, :k]) and torch.equal(a["beta_S"], res["beta_S"][j, :k])
                     and a["n_iter"] == int(res["n_iter"][j]))
        checked += 1
        # the same solve in plain FP64: the served int8 solve takes the FP64 iteration's decisions
        b = iht.fit(geno, st, pool[r["row0"] + j].contiguous(), k)
        fp64_same &= bool(torch.equal(b["support"], res["support"][j, :k]) and b["n_iter"] == int(res["n_iter"][j]))
        bb = b["beta_S"].cpu().numpy()
        fp64_beta_err = max(fp64_beta_err, float(np.abs(res["beta_S"][j, :k].cpu().numpy() - bb).max() / np.abs(bb).max()))
    log(f"served = alone (bitwise) on {checked} sampled solves: {same}; same supports and iterations as FP64: "
        f"{fp64_same}, beta max rel err {fp64_beta_err:.1e}")
    # Poisson arrivals at 0.5, 0.8 and 1.0 of the saturated request rate
    sweep = []
    for frac in (0.5, 0.8, 1.0):
        rate = frac * len(reqs) / wall
        arr = np.cumsum(np.random.default_rng([args.seed, 78, int(frac * 10)]).exponential(1.0 / rate, len(reqs)))
        wall_p, lat_p, _ = serve(iht, torch, srv, reqs, subsets, pool, arrivals=arr)
        sweep.append({"load": frac, "requests_per_s": round(rate, 2), "solves_per_s": round(traits / wall_p, 1),
                      "latency_ms_p50": round(float(np.percentile(lat_p, 50)) * 1e3, 1),
                      "latency_ms_p99": round(float(np.percentile(lat_p, 99)) * 1e3, 1),
                      "latency_ms_max": round(float(lat_p.max()) * 1e3, 1)})
        log(f"serving Poisson at {frac:.1f} x capacity ({rate:.1f} requests/s): {traits / wall_p:.0f} solves/s; "
            f"request latency p50 {np.percentile(lat_p, 50) * 1e3:.0f} ms p99 {np.percentile(lat_p, 99) * 1e3:.0f} ms "
            f"max {lat_p.max() * 1e3:.0f} ms")
    info = srv.info()
    srv.close()
    # plain loop: FP64 iht_fit per solve (stats per request), on the first 96 solves of the stream
    sample, t_plain, done = 96, 0.0, 0
    for i, r in enumerate(reqs):
        if done >= sample:
            break
        t0 = time.perf_counter()
        st = iht.Stats(geno, subsets[i])
        for j in range(r["T"]):
            if done >= sample:
                break
            iht.fit(geno, st, pool[r["row0"] + j].contiguous(), int(r["ks"][j]))
            done += 1
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
    plain_rate = done / t_plain
    log(f"plain FP64 loop: {done} solves in {t_plain:.2f}s = {plain_rate:.1f} solves/s")
    return {
        "workload": f"continuous-batching server, n={n} x p={p} ({n * p / 4e9:.1f} GB packed) resident; "
                    f"{len(reqs)} requests: subsets U{{2000..{n}}} subjects, 1..64 traits, k~U{{5..50}}; "
                    f"{slots} slots, kmax {kmax}, budget {budget >> 30} GiB; int8 matrix-core gradient, FP64 decisions",
        "solves": traits,
        "saturated_solves_per_s": round(sat_rate, 1),
        "saturated_latency_ms_p50": round(float(np.percentile(lat_sat, 50)) * 1e3, 1),
        "saturated_latency_ms_p99": round(float(np.percentile(lat_sat, 99)) * 1e3, 1),
        "poisson": sweep,
        "latency_ms_p50": sweep[1]["latency_ms_p50"],
        "latency_ms_p99": sweep[1]["latency_ms_p99"],
        "latency_note": "request latency (arrival to the end of the step that wrote it out) at 0.8 x capacity",
        "plain_fp64_loop_solves_per_s": round(plain_rate, 2),
        "speedup_vs_plain_fp64_loop": round(sat_rate / plain_rate, 1),
        "served_equals_alone_bitwise_sampled": same,
        "served_vs_fp64_sampled": {"solves": checked, "same_supports_and_iterations": fp64_same,
                                   "beta_max_rel_err": fp64_beta_err},
        "gradient_pass_us": round(pass_us, 1), "gradient_pass_gbs": round(pass_gbs, 1),
        "gradient_pass_hbm_frac": round(pass_gbs / HBM_PEAK_GBS, 4),
        "server_device_bytes": info["device_bytes"],
        "pass_block_snps_autotuned": iht.batch_tuning(geno, slots),
        "stats_blocks": info["stats_blocks"],
    }


def bench_c5(args, torch, iht, synth):
    """The large workload: n=20,000 x p=2,000,000 (10 GB packed), 100 causal SNPs, 5 covariates +
    intercept unpenalised; 32 traits x k in {50, 100, 150} = 96 solves in one int8 matrix-core batch
    against the plain FP64 iht_fit loop over the same 96 solves; the single-trait pass at this size."""
    t = time.time()
    prob = synth.make_problem("c5", 2)
    n, p = prob["n"], prob["p"]
    geno = iht.Geno(prob["bed"], n)
    traits = [prob["y"]] + [synth.make_trait(prob["bed"], n, prob["q"], 100, (0.05, 0.3), seed=700 + e, Z=prob["Z"],
                                             intercept=1.0)[0] for e in range(31)]
    del prob["bed"]
    Z = torch.from_numpy(np.ascontiguousarray(prob["Z"])).to(device="cuda", dtype=torch.float32)
    s = iht.Stats(geno)
    ks = [k for k in (50, 100, 150) for _ in range(32)]
    Y = torch.from_numpy(np.stack(traits * 3)).cuda()
    torch.cuda.synchronize()
    log(f"c5: n={n} p={p} ({n * p / 4e9:.0f} GB packed) ready in {time.time() - t:.0f}s")
    pass_us, _ = time_gradient(torch, iht, geno, s, Y[0].contiguous(), 10)
    pass_gbs = (n + 3) // 4 * p / (pass_us * 1e-6) / 1e9
    log(f"gradient pass at n={n} x p={p}: {pass_us:.1f} us = {pass_gbs:.0f} GB/s ({pass_gbs / HBM_PEAK_GBS:.1%} of HBM peak)")
    t0 = time.perf_counter()
    res = iht.fit_batch(geno, [s] * 96, Y, ks, Z=Z, precision=iht.MIXED_I8)
    torch.cuda.synchronize()
    bt = time.perf_counter() - t0
    log(f"c5 batched: 96 solves in {bt:.2f}s ({96 / bt:.1f} solves/s), statuses "
        f"{np.bincount(np.asarray(res['statuses']) + 4, minlength=7)[4:].tolist()}")
    t0 = time.perf_counter()
    same, berr, lat = 0, 0.0, []
    for tt in range(96):
        a = time.perf_counter()
        r64 = iht.fit(geno, s, Y[tt].contiguous(), ks[tt], Z=Z)
        lat.append(time.perf_counter() - a)
        k = ks[tt]
        ok = bool(torch.equal(r64["support"], res["support"][tt, :k])) and r64["n_iter"] == int(res["n_iter"][tt])
        same += int(ok)
        bb = r64["beta_S"].cpu().numpy()
        berr = max(berr, float(np.abs(res["beta_S"][tt, :k].cpu().numpy() - bb).max() / np.abs(bb).max()))
    plain = time.perf_counter() - t0
    log(f"c5 plain FP64 loop: 96 solves in {plain:.2f}s ({96 / plain:.1f} solves/s); batched speedup {plain / bt:.1f}x; "
        f"identical supports and iterations {same}/96, beta max rel err {berr:.1e}")
    return {
        "workload": f"n={n} x p={p} ({n * p / 4e9:.0f} GB packed), 100 causal SNPs, 5 covariates + intercept "
                    "unpenalised; 32 traits x k in {50, 100, 150} = 96 solves, int8 matrix-core batch (FP64 "
                    "decisions) against the plain FP64 iht_fit loop",
        "solves": 96, "batched_s": round(bt, 3), "batched_solves_per_s": round(96 / bt, 2),
        "plain_fp64_loop_s": round(plain, 3), "plain_fp64_loop_solves_per_s": round(96 / plain, 2),
        "plain_fp64_solve_latency_ms_p50": round(float(np.median(lat)) * 1e3, 1),
        "speedup_vs_plain_fp64_loop": round(plain / bt, 2),
        "same_supports_and_iterations_as_fp64": same, "beta_max_rel_err_vs_fp64": berr,
        "iterations_mean": round(float(np.mean(res["n_iter"])), 2),
        "gradient_pass_us": round(pass_us, 1), "gradient_pass_gbs": round(pass_gbs, 1),
        "gradient_pass_hbm_frac": round(pass_gbs / HBM_PEAK_GBS, 4),
        "pass_block_snps_autotuned": iht.batch_tuning(geno, 96),
    }


if __name__ == "__main__":
    main()
