"""Benchmark: D-iteration PageRank on one MI355X.

A step is one plain solve of the 1e6-node web-like graph (about 8e6 links,
damping 0.85, uniform B = 0.15/N) from H = 0 until the exact FP64 residual
||B + P H - H||_1 <= 1e-9 ||B||_1: initialization, all diffusion launches,
the exact residual refreshes and the final check. Graph upload and the
partition plan are built once before the timed region (reported apart).

Prints one JSON line. `value` is diffused edges per second over the timed
steps; `time_to_tol_ms` is the wall time of one solve.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
PROFILE = os.path.join(ROOT, "profiles", "k_part_sweep_headline_n1e6.json")


def profiled_traffic():
    """HBM bytes per k_part_sweep launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the kernel
    source changed since those counters were taken."""
    import hashlib

    try:
        prof = json.load(open(PROFILE))
        src = open(os.path.join(ROOT, prof["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != prof.get("source_sha256"):
        return None
    return prof["traffic_bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", type=int, default=0, help="DITR_MODE_* (0 = default)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy (reference for HBM counters)")
    return ap.parse_args()


def copy_calibration():
    """A plain device-to-device copy of known size: the reference that scales
    the FETCH_SIZE / WRITE_SIZE counters of the solver's kernels."""
    import torch

    nbytes = 512 << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "copies": 3}))


def cpu_baseline(cp, ri, b, tol):
    """The FP64 oracle (single thread) on the same graph, timed on the host."""
    import oracle

    oracle.build(force=False)
    t0 = time.perf_counter()
    runs = []
    while True:
        r = oracle.solve(cp, ri, b, rel_tol=tol)
        runs.append(r)
        if time.perf_counter() - t0 > 10.0 or len(runs) >= 3:
            break
    best = min(runs, key=lambda r: r.seconds)
    return {
        "value": best.edges / best.seconds,
        "unit": "diffused edges/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "full 1e6-node solve to 1e-9 ||B||_1, best of %d runs: %.3f s, %.3e edges"
                  % (len(runs), best.seconds, best.edges),
    }


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU: the solver has no multi-GPU path in this build "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import ditgen
    from paper_1202_6168_amd import ditr

    spec = ditgen.HEADLINE
    cp, ri = ditgen.generate(spec)
    b = ditgen.uniform_b(spec.n)
    dev = torch.device("cuda", 0)
    ctx = ditr.Context(0)
    t0 = time.perf_counter()
    cpt, rit = torch.from_numpy(cp).to(dev), torch.from_numpy(ri).to(dev)
    g = ditr.Graph(ctx, cpt, rit)
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t0)
    K = len(g.partitions()) - 1
    bt = torch.from_numpy(b).to(dev)
    ht = torch.empty(spec.n, dtype=torch.float64, device=dev)
    ft = torch.empty(spec.n, dtype=torch.float32, device=dev)
    opts = ditr.opts_default(mode=args.mode, flags=ditr.FLAG_TIME_KERNELS)

    for _ in range(args.warmup):
        ditr.solve(ctx, g, bt, ht, ft, rel_tol=args.tol, opts=opts, allow=(ditr.OK,))
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats.append(ditr.solve(ctx, g, bt, ht, ft, rel_tol=args.tol, opts=opts,
                                allow=(ditr.OK,)))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    edges = sum(s.edges for s in stats)
    diffs = sum(s.diffusions for s in stats)
    ksec = sum(s.kernel_seconds for s in stats)
    klaunch = sum(s.timed_launches for s in stats)
    ms_step = 1e3 * wall / args.steps
    # algorithmic bytes of a diffusion (no reuse on chip): per out-link 4 B index
    # + 8 B FP32 read-modify-write of the target's fluid; per diffused node 4 B
    # column pointer + 8 B fluid read and zero + 16 B FP64 history update
    bytes_alg = 12.0 * edges + 28.0 * diffs
    achieved = bytes_alg / ksec / 1e9 if ksec > 0 else 0.0
    last = stats[-1]
    h = ht.cpu().numpy()
    out = {
        "metric": "time to ||F||_1<=1e-9||B||_1 + diffused edges/s, N=1e6; plain vs batched/warm-start",
        "value": edges / wall,
        "unit": "diffused edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "time_to_tol_ms": ms_step,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": {
            "workload": "D-iteration PageRank, synthetic web-like graph N=1e6, L=%d (block-1000 "
                        "locality, Zipf out-degree, 10%% dangling), B=0.15/N, tol 1e-9 ||B||_1"
                        % ri.size,
            "n": spec.n,
            "nnz": int(ri.size),
            "tol": args.tol,
            "mode": "partitioned sweep" if args.mode in (0, 3) else "mode %d" % args.mode,
            "partitions": K,
        },
        "edges_per_step": edges / args.steps,
        "normalized_iterations": edges / args.steps / ri.size,
        "final_resid_rel": last.resid_l1 / last.b_l1,
        "h_sum": float(h.sum()),
        "graph_setup_ms": setup_ms,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_part_sweep",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": profiled_traffic(),
            "alg_bytes_per_launch": bytes_alg / klaunch if klaunch else None,
            "bytes_per_edge": bytes_alg / edges if edges else None,
            "avg_launch_us": 1e6 * ksec / klaunch if klaunch else None,
            "launches": klaunch,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cp, ri, b, args.tol)
    print(json.dumps(out))
    g.close()
    ctx.close()


if __name__ == "__main__":
    main()
