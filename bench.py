#!/usr/bin/env python3
"""Throughput of the Phurbas MLS / ideal-MHD hot path on one MI355X.

Workload: the adaptive shear-layer set of 1,048,576 particles (resolution
length varying 4x across two tanh shear layers, sampled at one particle per
lambda^3), spatially ordered once during set-up.  One step = forward
(weighted moment assembly, FP64 factor and solve, operator application,
ideal-MHD right-hand side) + backward (reverse mode of the loss
sum_i w_i |dV/dt|_i^2, w_i ~ U(0,1)).  The neighbor build is timed apart.

Prints one JSON line (rank 0).  Progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLS particle updates/s at 1M particles, mixed vs FP64 plain, fwd+bwd"


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target wall time of the CPU oracle sample")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB three times (a plain "
                         "copy of known size, to calibrate hardware byte counters)")
    ap.add_argument("--tune", default="",
                    help="schedule knobs key=value,... (see phb_tune_set)")
    return ap.parse_args()


def time_gpu(fn, reps, torch):
    """Median ms of fn over reps, bracketed by events on torch's current stream."""
    out = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b))
    out.sort()
    return out[len(out) // 2]


def cpu_baseline(c, perm_np, w_np, seconds):
    """The oracle (as it stands) on a bounded random sample of the same set:
    brute-force rows, forward and reverse mode for those owners."""
    import numpy as np
    import oracle
    pos = c["pos"]
    lam = c["lam"]
    q = c["q"]
    n = lam.shape[0]
    threads = os.cpu_count() or 1
    rng = np.random.default_rng(123)

    def run(m):
        rows = np.sort(rng.choice(n, m, replace=False))
        t0 = time.perf_counter()
        off, idx = oracle.neighbors(pos, lam, rows=rows, threads=threads)
        t1 = time.perf_counter()
        rhs, _, _ = oracle.mhd_rhs(pos, lam, off, idx, q, rows=rows, threads=threads)
        t2 = time.perf_counter()
        gbar = np.zeros((8, n))
        gbar[1:4, rows] = 2 * w_np[None, rows] * rhs[1:4]
        oracle.adjoint_rows(pos, lam, off, idx, q, gbar, rows, threads=threads)
        t3 = time.perf_counter()
        return m, t1 - t0, t2 - t1, t3 - t2

    m, tn, tf, tb = run(256)
    per = (tn + tf + tb) / m
    m2 = int(max(256, min(n, seconds / max(per, 1e-9))))
    m, tn, tf, tb = run(m2)
    return {
        "value": m / (tf + tb), "unit": "particle-updates/s", "cores": threads, "kind": "oracle",
        "sample": f"{m} random particles of the same 1,048,576-particle set: oracle forward "
                  f"({tf:.2f} s) + reverse mode ({tb:.2f} s) with their brute-force neighbor rows "
                  f"({tn:.2f} s, reported apart)",
        "neighbor_rows_per_s": m / tn,
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"metric": METRIC, "error": "this build runs on one GPU only; "
                          "--gpus must be 1 (multi-GPU sharding is a design note, not built)"}))
        sys.exit(2)
    import numpy as np
    import torch
    import paper_1110_0836_amd as P
    from paper_1110_0836_amd import flops as F
    from paper_1110_0836_amd import synth

    log("generating the shear-layer set")
    c = synth.config3(n=args.n)
    n = c["lam"].shape[0]
    rng = np.random.default_rng(4)
    w_np = rng.uniform(0.0, 1.0, n)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s = P.Setup(L=c["L"], periodic=c["periodic"], gamma=c["gamma"],
                precision=P.PHB_MIXED if args.precision == "mixed" else P.PHB_FP64)
    pos0 = torch.from_numpy(c["pos"]).to(dev)
    lam0 = torch.from_numpy(c["lam"]).to(dev)
    q0 = torch.from_numpy(c["q"]).to(dev)
    w0 = torch.from_numpy(w_np).to(dev)

    tune = {}
    for kv in filter(None, args.tune.split(",")):
        k, v = kv.split("=")
        tune[k] = int(v)
    for k, v in tune.items():
        P.phb_tune_set(k, v)

    log("spatial ordering (set-up)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    perm = P.spatial_order(pos0, lam0, s)
    pos = P.permute(perm, pos0)
    lam = P.permute(perm, lam0.view(1, n)).view(n)
    q = P.permute(perm, q0)
    w = P.permute(perm, w0.view(1, n)).view(n)
    torch.cuda.synchronize()
    order_ms = (time.perf_counter() - t0) * 1e3

    log("neighbor build")
    off, idx = P.neighbors(pos, lam, s)
    nnz = idx.shape[0]
    cap = nnz
    off2 = torch.empty_like(off)
    idx2 = torch.empty_like(idx)
    nb_ms = time_gpu(lambda: P.phb_neighbors_build(s, pos, lam, off2, idx2, cap), 5, torch)
    tr_bufs = (torch.empty_like(off), torch.empty_like(idx), torch.empty_like(idx))
    tr_ms = time_gpu(lambda: P.phb_neighbors_transpose(off, idx, *tr_bufs), 5, torch)
    trans = tr_bufs
    counts = torch.diff(off).cpu().numpy()
    log(f"n={n} nnz={nnz} neighbors per particle min/median/max "
        f"{counts.min()}/{int(np.median(counts))}/{counts.max()}  build {nb_ms:.2f} ms "
        f"transpose {tr_ms:.2f} ms")

    rhs = torch.empty((8, n), dtype=torch.float64, device=dev)
    dxdt = torch.empty((3, n), dtype=torch.float64, device=dev)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    tape = torch.empty(P.phb_tape_bytes(n) // 8, dtype=torch.float64, device=dev)
    gbar = torch.zeros((8, n), dtype=torch.float64, device=dev)
    q_bar = torch.empty_like(q)
    pos_bar = torch.empty_like(pos)

    def forward():
        P.phb_mhd_rhs(s, pos, lam, off, idx, q, rhs, dxdt, st, tape)

    def backward():
        torch.mul(rhs[1:4], w, out=gbar[1:4])
        gbar[1:4].mul_(2.0)
        P.phb_mhd_rhs_adjoint(s, pos, lam, off, idx, *trans, q, gbar, None, q_bar, pos_bar, tape)

    def step():
        forward()
        backward()

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    nfail = int((st != 0).sum().item())

    log(f"timing {args.steps} steps (fwd+bwd)")
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for k in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    ms_step = ev0.elapsed_time(ev1) / args.steps
    value = n / (ms_step / 1e3)
    fwd_ms = time_gpu(forward, max(3, args.steps // 2), torch)
    log(f"{ms_step:.3f} ms/step (wall {wall_ms / args.steps:.3f}), forward {fwd_ms:.3f} ms")

    roof = None
    kernels = {}
    if not args.no_profile:
        P.phb_profile(True)
        reps = 3
        for _ in range(reps):
            step()
        prof = P.phb_profile_read()
        P.phb_profile(False)
        for name, (ms, cnt) in prof.items():
            kernels[name] = {"avg_ms": ms / cnt, "launches": cnt,
                             "ms_per_step": ms / reps}
        dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
        fl = F.flops(dom, n, nnz)
        by = F.bytes_moved(dom, n, nnz)
        avg_s = kernels[dom]["avg_ms"] / 1e3
        if fl > 0:
            ach = fl / avg_s / 1e12
            roof = {"kernel": dom, "bound": "alu", "achieved": ach,
                    "peak": F.PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
                    "frac": ach / (F.PEAK_FP64_VALU / 1e12), "traffic": None,
                    "algorithmic_per_launch": fl}
        else:
            ach = by / avg_s / 1e9
            roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": F.PEAK_HBM / 1e9,
                    "unit": "GB/s", "frac": ach / (F.PEAK_HBM / 1e9), "traffic": None,
                    "algorithmic_per_launch": by}
        for name in kernels:
            f = F.flops(name, n, nnz)
            if f:
                kernels[name]["tflops"] = f / (kernels[name]["avg_ms"] / 1e3) / 1e12
        log("kernels: " + ", ".join(f"{k} {v['avg_ms']:.3f} ms" for k, v in kernels.items()))

    if args.copy_mib > 0:
        nbytes = args.copy_mib << 20
        a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.copy_mib} MiB three times (counter calibration)")

    cpu = None
    if not args.no_cpu_baseline:
        log("oracle CPU baseline")
        perm_np = perm.cpu().numpy()
        cp = dict(pos=np.ascontiguousarray(c["pos"][:, perm_np]),
                  lam=np.ascontiguousarray(c["lam"][perm_np]),
                  q=np.ascontiguousarray(c["q"][:, perm_np]))
        cpu = cpu_baseline(cp, perm_np, w_np[perm_np], args.cpu_seconds)
        log(f"oracle {cpu['value']:.1f} particle-updates/s on {cpu['cores']} threads")

    out = {
        "metric": METRIC, "value": value, "unit": "particle-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"shear_layer_adaptive_{n}", "n_particles": n, "nnz": int(nnz),
                   "neighbors_median": int(np.median(counts)), "lambda_range": "4x",
                   "precision": args.precision, "step": "forward + reverse mode",
                   "tuning": {k: P.phb_tune_get(k) for k in P.TUNE_KEYS},
                   "loss": "sum_i w_i |dV/dt|_i^2, w ~ U(0,1)"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": {"forward_ms": fwd_ms, "forward_updates_per_s": n / (fwd_ms / 1e3),
                  "neighbor_build_ms": nb_ms, "transpose_ms": tr_ms,
                  "spatial_order_setup_ms": order_ms, "failed_particles": nfail,
                  "kernels": kernels},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
