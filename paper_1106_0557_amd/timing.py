"""Per-pass timing of single solves on one GPU.

    python -m paper_1106_0557_amd.timing --n 576 1152 --dtype fp32 --reps 3

For each mesh n^3 (unit box, h = 1/n) the source is the 512^3 benchmark's kind:
64 Gaussian blobs plus a sphere of radius 0.2 (sources.config5).  The plan and
one workspace are built, solves run untimed for at least a quarter of a second
(at least two; from idle the GPU's clocks need about that long to settle), and each of `reps` solves runs
pass by pass on one stream with HIP events between the passes.  One line per
mesh: the mean milliseconds of every active pass and of the whole solve, and
the solve's algorithmic bytes (the sum of its passes' bytes, Plan.solve_bytes)
over its time.  The kernels run through the C ABI like any solve.
"""
import argparse
import json
import sys
import time


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, nargs="+", default=[512])
    ap.add_argument("--dtype", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)

    import torch

    import paper_1106_0557_amd as ps
    from paper_1106_0557_amd import sources

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        return 2
    torch.cuda.set_device(0)
    dt = torch.float32 if args.dtype == "fp32" else torch.float64
    stream = torch.cuda.current_stream()
    for n in args.n:
        print(f"[timing] n={n} {args.dtype}: plan and source", file=sys.stderr, flush=True)
        _, h, S = sources.config5(n=n, device="cuda")
        src = S.to(dt)
        del S
        plan = ps.Plan(n, n, n, h=h, dtype=dt)
        w = plan.workspace()
        out = torch.empty_like(src)
        t_settle, k = time.perf_counter(), 0
        while k < 2 or time.perf_counter() - t_settle < 0.25:
            ps.solve_batched([w], [src], [out])
            torch.cuda.synchronize()
            k += 1
        active = plan.active_passes
        tot = {p: 0.0 for p in active}
        for _ in range(args.reps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(active) + 1)]
            for i, p in enumerate(active):
                ev[i].record(stream)
                ps.pass_batched(p, [w], S=[src], Phi=[out], stream=stream)
            ev[-1].record(stream)
            torch.cuda.synchronize()
            for i, p in enumerate(active):
                tot[p] += ev[i].elapsed_time(ev[i + 1]) / args.reps
        solve_ms = sum(tot.values())
        line = {"n": n, "dtype": args.dtype, "reps": args.reps,
                "pass_ms": {ps.PASS_NAMES[p]: round(v, 4) for p, v in tot.items()},
                "solve_ms": round(solve_ms, 4),
                "algorithmic_GBps": round(plan.solve_bytes() / (solve_ms * 1e-3) / 1e9, 1),
                "spectrum_kz_fastest": plan.spectrum_kz_fastest}
        print(json.dumps(line), flush=True)
        w.close()
        plan.close()
        del src, out
        torch.cuda.empty_cache()
    return 0


if __name__ == "__main__":
    sys.exit(main())
