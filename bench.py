#!/usr/bin/env python3
"""Benchmark of the isolated Poisson solve (arXiv:1106.0557) on one MI355X.

Headline workload: the 128^3 mesh padded to 256^3 (homogeneous oblate spheroid,
a=0.3, b=0.15 of the box, S = 4 pi inside).  One timed step = one batch of
``--batch`` independent FP32 solves issued through the grouped pass launches
that the serving loop uses (five launches per step, each over every problem of
the batch), with all inputs resident in HBM.  Beside it: the FP64 plain path
(sequential single solves, per-solve HIP events), the continuous-batching
serving loop on a Poisson arrival trace, and the FP64 CPU oracle timed on this
host's cores.

Prints one JSON line.  ``value`` = FP32 served solves/s over the timed steps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
METRIC = "solves/s + effective HBM GB/s at 256^3 (FP32 served vs FP64 plain); p50/p99"
CSRC = "paper_1106_0557_amd/csrc"


def algorithmic_bytes(n: int, real: int) -> int:
    """Pad-aware five-pass model: read S and write Phi, 12 complex n^2 (n+1) of
    workspace traffic, the (n+1)^3 spectrum read once."""
    c = 2 * real
    return 2 * real * n**3 + 12 * c * n * n * (n + 1) + real * (n + 1) ** 3


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    f = math.floor(k)
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def source_hash() -> str:
    """Hash of every kernel and runtime source and of the build script (its
    compile flags), to tie counter data to a build."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, CSRC)
    paths = [os.path.join(d, name) for name in sorted(os.listdir(d)) if name.endswith((".hip", ".h", ".cpp"))]
    paths.append(os.path.join(ROOT, "paper_1106_0557_amd", "build.py"))
    for path in paths:
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, n: int, batch: int):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter
    summary, or None when it is missing or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    if data.get("source_hash") != source_hash():
        return None
    entry = data.get("kernels", {}).get(kernel)
    if not entry or entry.get("n") != n or entry.get("batch") != batch:
        return None
    return entry.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--settle-s", type=float, default=0.25,
                    help="untimed steps for this many seconds before the warmup steps, so that the GPU's clocks "
                         "reach their steady state (measured: a few warm-up steps from idle leave the timed steps "
                         "about 5 %% slow)")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--batch", type=int, default=32, help="FP32 solves per served step")
    ap.add_argument("--fp64-solves", type=int, default=2500, help="sequential FP64 plain solves (paper: 2500)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget for the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests per served trace")
    ap.add_argument("--no-large", action="store_true", help="skip the 512^3 single-solve measurement")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "single-GPU benchmark: --gpus must be 1"}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(2)
    torch.cuda.set_device(0)

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "launches": 3}), flush=True)
        return

    import paper_1106_0557_amd as ps
    from paper_1106_0557_amd import sources

    n = args.n
    B = args.batch
    stream = torch.cuda.current_stream()
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731

    # ---------------------------------------------------------------- inputs
    log(f"[bench] n={n} batch={B}: building plans and sources")
    _, h, S64 = sources.config2(n=n)
    plan32 = ps.Plan(n, n, n, h=h, dtype=torch.float32)
    plan64 = ps.Plan(n, n, n, h=h, dtype=torch.float64)
    S32_dev = S64.to("cuda", torch.float32)
    S64_dev = S64.to("cuda", torch.float64)
    ws = [plan32.workspace() for _ in range(B)]
    S_list = [S32_dev.clone() for _ in range(B)]
    P_list = [torch.empty_like(S32_dev) for _ in range(B)]
    torch.cuda.synchronize()

    # --------------------------------------------- FP32 served batch (timed)
    # a fused plan does its x and y transforms in the x passes and skips the y passes
    active = plan32.active_passes
    pass_names = {p: ps.PASS_NAMES[p] for p in active}
    if plan32.fused:
        pass_names[ps.PASS_X_FWD], pass_names[ps.PASS_X_INV] = "xy_fwd", "yx_inv"

    def step(evs=None):
        for i, p in enumerate(active):
            if evs is not None:
                evs[i].record(stream)
            ps.pass_batched(p, ws, S=S_list, Phi=P_list, stream=stream)
        if evs is not None:
            evs[len(active)].record(stream)

    settle_steps = 0
    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < args.settle_s:
        for _ in range(8):
            step()
        settle_steps += 8
        torch.cuda.synchronize()
    settle_s = time.perf_counter() - t_settle
    log(f"[bench] settled for {settle_s:.2f} s ({settle_steps} untimed steps); warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev_sets = [[torch.cuda.Event(enable_timing=True) for _ in range(len(active) + 1)] for _ in range(args.steps)]
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(ev_sets[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_pass_ms = {p: [evs[i].elapsed_time(evs[i + 1]) for evs in ev_sets] for i, p in enumerate(active)}
    step_ms = [evs[0].elapsed_time(evs[len(active)]) for evs in ev_sets]
    solves32 = B * args.steps / wall
    bytes32 = algorithmic_bytes(n, 4)
    eff32 = bytes32 * solves32 / 1e9
    avg_pass = {p: sum(v) / len(v) for p, v in per_pass_ms.items()}
    dom = max(active, key=lambda p: avg_pass[p])
    dom_bytes = plan32.pass_bytes(dom) * B
    dom_gbs = dom_bytes / (avg_pass[dom] * 1e-3) / 1e9
    log(f"[bench] fp32 served: {solves32:.1f} solves/s, {eff32:.0f} GB/s effective; passes (ms) "
        + ", ".join(f"{pass_names[p]}={avg_pass[p]:.4f}" for p in active))

    # accuracy of the FP32 served result (last step) against the GPU FP64 solve
    phi64 = plan64.solve(S64_dev)
    torch.cuda.synchronize()
    d = (P_list[0].double() - phi64)
    acc32 = {"rel_l2_vs_gpu_fp64": float(d.norm() / phi64.norm()),
             "rel_max_vs_gpu_fp64": float(d.abs().max() / phi64.abs().max())}

    # ------------------------------------------ device copy ceiling (context)
    cbytes = 1 << 30
    ca = torch.empty(cbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    cb = torch.empty_like(ca)
    for _ in range(3):
        cb.copy_(ca)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        cb.copy_(ca)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * cbytes * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del ca, cb

    # ---------------------------------------------------- FP64 plain (timed)
    out64 = torch.empty_like(S64_dev)
    for _ in range(20):
        plan64.solve(S64_dev, out=out64)
    torch.cuda.synchronize()
    R = args.fp64_solves
    evs64 = [torch.cuda.Event(enable_timing=True) for _ in range(R + 1)]
    log(f"[bench] fp64 plain: {R} sequential solves")
    t0 = time.perf_counter()
    evs64[0].record(stream)
    for i in range(R):
        plan64.solve(S64_dev, out=out64)
        evs64[i + 1].record(stream)
    torch.cuda.synchronize()
    wall64 = time.perf_counter() - t0
    lat64 = [evs64[i].elapsed_time(evs64[i + 1]) for i in range(R)]
    solves64 = R / wall64
    eff64 = algorithmic_bytes(n, 8) * solves64 / 1e9
    # one FP64 solve's working set (workspace, source, potential, spectrum) fits
    # the 256 MB Infinity Cache; the same solves rotating over 4 plans and 4
    # source/potential pairs (4 times that) do not
    ws64 = plan64.workspace_bytes + 2 * S64_dev.numel() * 8 + ps.plan_resident_bytes(n, n, n, torch.float64)
    rot_plans = [ps.Plan(n, n, n, h=h, dtype=torch.float64) for _ in range(4)]
    rot_S = [S64_dev.clone() for _ in range(4)]
    rot_P = [torch.empty_like(S64_dev) for _ in range(4)]
    for k in range(8):
        rot_plans[k % 4].solve(rot_S[k % 4], out=rot_P[k % 4])
    torch.cuda.synchronize()
    Rr = max(100, R // 5)
    evr = [torch.cuda.Event(enable_timing=True) for _ in range(Rr + 1)]
    t0 = time.perf_counter()
    evr[0].record(stream)
    for i in range(Rr):
        rot_plans[i % 4].solve(rot_S[i % 4], out=rot_P[i % 4])
        evr[i + 1].record(stream)
    torch.cuda.synchronize()
    wall_r = time.perf_counter() - t0
    lat_r = [evr[i].elapsed_time(evr[i + 1]) for i in range(Rr)]
    for pl in rot_plans:
        pl.close()
    del rot_S, rot_P
    fp64_rot = {"solves_per_s": round(Rr / wall_r, 2),
                "effective_GBps_B_model": round(algorithmic_bytes(n, 8) * Rr / wall_r / 1e9, 1),
                "moved_GBps": round(plan64.solve_bytes() * Rr / wall_r / 1e9, 1),
                "latency_ms_p50": round(percentile(lat_r, 50), 5),
                "latency_ms_p99": round(percentile(lat_r, 99), 5), "solves_timed": Rr,
                "working_set_bytes": 4 * ws64}

    # --------------------------------- single large solve, 512^3 (context)
    large = None
    if not args.no_large:
        nl = 512
        log(f"[bench] single large solve n={nl}")
        _, hl, Sl = sources.config5(n=nl, device="cuda")
        large = {"n": nl, "padded": 2 * nl}
        for dt, tag in ((torch.float32, "fp32"), (torch.float64, "fp64")):
            t0 = time.perf_counter()
            pl = ps.Plan(nl, nl, nl, h=hl, dtype=dt)
            torch.cuda.synchronize()
            t_plan = time.perf_counter() - t0
            src = Sl.to(dt)
            out = torch.empty_like(src)
            pl.solve(src, out=out)
            torch.cuda.synchronize()
            reps = 10
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
            ev[0].record(stream)
            for i in range(reps):
                pl.solve(src, out=out)
                ev[i + 1].record(stream)
            torch.cuda.synchronize()
            lat = [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]
            ms = sum(lat) / reps
            large[tag] = {"ms_per_solve": round(ms, 3), "solves_per_s": round(1e3 / ms, 2),
                          "effective_GBps": round(algorithmic_bytes(nl, 4 if tag == "fp32" else 8) / (ms * 1e-3) / 1e9, 1),
                          "plan_create_s": round(t_plan, 3)}
            if tag == "fp32":
                out32 = out.double()
            else:
                d = out32 - out
                large["fp32_vs_fp64"] = {"rel_l2": float(d.norm() / out.norm()),
                                         "rel_max": float(d.abs().max() / out.abs().max())}
            pl.close()
            del src, out
        del Sl, out32
        torch.cuda.empty_cache()
        log(f"[bench] large: {large}")

    # ------------------------------ config 3: 64 mixed-size sources, one batch
    config3 = None
    if not args.no_serve:
        import paper_1106_0557_amd.sources as srcmod

        log("[bench] config 3: 64 sources of sizes {32..128}^3 in one pspfft_solve_batched call")
        batch = srcmod.config3(device="cuda")
        plans3, ws3, S3, P3 = {}, [], [], []
        for nn, src in batch:
            if nn not in plans3:
                plans3[nn] = ps.Plan(nn, nn, nn, h=1.0 / nn, dtype=torch.float32)
            ws3.append(plans3[nn].workspace())
            S3.append(src.to(torch.float32).contiguous())
            P3.append(torch.empty_like(S3[-1]))
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            for _ in range(3):
                ps.solve_batched(ws3, S3, P3, stream=st)
            st.synchronize()
            reps = 30
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(reps):
                ps.solve_batched(ws3, S3, P3, stream=st)
            e1.record(st)
            e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        alg3 = sum(algorithmic_bytes(nn, 4) for nn, _ in batch)
        counts = {}
        for nn, _ in batch:
            counts[nn] = counts.get(nn, 0) + 1
        config3 = {"problems": len(batch), "sizes": {str(k): v for k, v in sorted(counts.items())},
                   "ms_per_batch": round(ms, 4), "solves_per_s": round(len(batch) / ms * 1e3, 1),
                   "effective_GBps": round(alg3 / ms / 1e6, 1)}
        log(f"[bench] config 3: {config3}")
        for w in ws3:
            w.close()
        for pl3 in plans3.values():
            pl3.close()
        del S3, P3, batch
        torch.cuda.empty_cache()

    # ----------------------------------------------- serving loop (Poisson)
    serve = None
    if not args.no_serve:
        try:
            from paper_1106_0557_amd import serve as serve_mod

            serve = serve_mod.bench_served(n=n, dtype=torch.float32, log=log, count=args.serve_requests)
        except ImportError:
            serve = None

    # -------------------------------------------------------- CPU oracle leg
    cpu = None
    if not args.no_cpu:
        import oracle
        from oracle import norms

        log("[bench] cpu oracle sample")
        S_np = S64.numpy()
        all_threads = oracle.threads()

        def timed(fn, budget_s, min_reps=1, max_reps=20):
            times = []
            t_start = time.perf_counter()
            while len(times) < max_reps:
                t0 = time.perf_counter()
                out = fn()
                times.append(time.perf_counter() - t0)
                if len(times) >= min_reps and time.perf_counter() - t_start + times[-1] > budget_s:
                    break
            return out, times

        ref, times = timed(lambda: oracle.solve_fft(S_np, h), args.cpu_seconds * 0.2, min_reps=2)
        c2_all = len(times) / sum(times)
        n1, h1, S1 = sources.config1()
        S1 = S1.numpy()
        _, t1 = timed(lambda: oracle.solve_fft(S1, h1), 1.0, min_reps=3)
        c1_all = len(t1) / sum(t1)
        batch3 = sources.config3()
        t0 = time.perf_counter()
        for nn, src in batch3:
            oracle.solve_fft(src.numpy(), 1.0 / nn)
        c3_s = time.perf_counter() - t0
        c4 = {}
        trace4 = sources.config4_trace(rate_hz=0, count=40)
        for size in sources.CONFIG4_SIZES:
            r4 = next(r for r in trace4 if r.n == size)
            S4 = sources.blob_field(size, r4.blobs).numpy()
            t0 = time.perf_counter()
            oracle.solve_fft(S4, 1.0 / size)
            c4[str(size)] = round(1.0 / (time.perf_counter() - t0), 4)
        oracle.set_threads(1)
        try:
            _, t1s = timed(lambda: oracle.solve_fft(S1, h1), 1.0, min_reps=2)
            _, t2s = timed(lambda: oracle.solve_fft(S_np, h), 0.0, min_reps=1, max_reps=1)
        finally:
            oracle.set_threads(all_threads)
        model = platform.processor() or platform.machine()
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
        cpu = {"value": round(c2_all, 4), "unit": "solves/s", "cores": all_threads, "kind": "oracle",
               "sample": f"{len(times)} FP64 oracle solves (naive mixed-radix FFT convolution on the {2 * n}^3 "
                         f"padded mesh, OpenMP on {all_threads} threads) of the same {n}^3 spheroid source; "
                         f"beside it the configurations below",
               "cpu_model": model, "os_cpu_count": os.cpu_count(), "omp_threads": all_threads,
               "config2_solves_per_s": {"all_threads": round(c2_all, 4), "one_thread": round(1.0 / t2s[0], 4)},
               "config1_solves_per_s": {"all_threads": round(c1_all, 3), "one_thread": round(len(t1s) / sum(t1s), 3)},
               "config3_batch_s_all_threads": round(c3_s, 3),
               "config3_solves_per_s_all_threads": round(len(batch3) / c3_s, 3),
               "config4_sizes_solves_per_s_all_threads": c4}
        acc32["rel_l2_vs_oracle"] = norms.rel_l2(P_list[0].double().cpu().numpy(), ref)
        acc32["rel_max_vs_oracle"] = norms.rel_max(P_list[0].double().cpu().numpy(), ref)
        o64 = out64.cpu().numpy()
        acc64 = {"rel_l2_vs_oracle": norms.rel_l2(o64, ref), "rel_max_vs_oracle": norms.rel_max(o64, ref)}
    else:
        acc64 = None

    traffic = load_traffic(f"pass_{pass_names[dom]}", n, B)
    result = {
        "metric": METRIC,
        "value": round(solves32, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle": {"seconds": round(settle_s, 3), "steps": settle_steps,
                   "note": "untimed steps before the warmup steps, until the GPU's clocks are steady"},
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"isolated Poisson solve, {n}^3 mesh padded to {2 * n}^3 (homogeneous oblate "
                               f"spheroid a=0.3 b=0.15, S=4pi inside), FP32 served path, {B} solves per step "
                               f"in grouped launches",
                   "n": n, "padded": 2 * n, "batch_per_step": B, "parallelism": "single-gpu"},
        "bytes_moved_per_solve": plan32.solve_bytes(),
        "moved_GBps": round(plan32.solve_bytes() * solves32 / 1e9, 1),
        "moved_frac_of_peak": round(plan32.solve_bytes() * solves32 / 1e9 / HBM_PEAK_GBS, 4),
        "copy_ceiling_GBps": round(copy_gbs, 1),
        "fused_xy_planes": plan32.fused,
        "b_model": {"effective_GBps": round(eff32, 1), "bytes_per_solve": bytes32,
                    "note": "five-pass byte model B(n) = 2r n^3 + 12c n^2(n+1) + r(n+1)^3: a fixed yardstick of "
                            "solves/s, not bytes moved (the fused path moves bytes_moved_per_solve)"},
        "step_ms_p50": round(percentile(step_ms, 50), 5),
        "step_ms_p99": round(percentile(step_ms, 99), 5),
        "pass_ms_avg": {pass_names[p]: round(avg_pass[p], 5) for p in active},
        "fp32_accuracy": acc32,
        "fp64_plain": {"solves_per_s": round(solves64, 2), "effective_GBps_B_model": round(eff64, 1),
                       "moved_GBps": round(plan64.solve_bytes() * solves64 / 1e9, 1),
                       "latency_ms_p50": round(percentile(lat64, 50), 5),
                       "latency_ms_p99": round(percentile(lat64, 99), 5),
                       "solves_timed": R, "accuracy": acc64,
                       "working_set_bytes": ws64,
                       "note": "one plan, one source: the working set fits the 256 MB Infinity Cache (MALL), "
                               "so this is not an HBM figure; rotating_4_plans is",
                       "rotating_4_plans": fp64_rot},
        "roofline": {"bound": "hbm",
                     "kernel": f"{'plane_kernel' if pass_names[dom] in ('xy_fwd', 'yx_inv') else 'pass_kernel'} "
                               f"({pass_names[dom]})",
                     "achieved": round(dom_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
                     "algorithmic_bytes_per_launch": dom_bytes,
                     "avg_launch_ms": round(avg_pass[dom], 5),
                     "traffic": traffic},
        "cpu_baseline": cpu,
        "served": serve,
        "single_large_solve": large,
        "config3_batched": config3,
        "kernel_source_hash": source_hash(),
    }
    print(json.dumps(result), flush=True)
    for w in ws:
        w.close()
    plan32.close()
    plan64.close()


if __name__ == "__main__":
    main()
