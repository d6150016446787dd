"""Throughput of the fused collide-and-stream step on one MI355X.

Workload: rotated Fourier-mode decay, D3Q19, periodic 256^3, u = 0, uniform tensor
R diag(1e-2, 1e-4, 1e-6) R^T with a seeded random rotation, phi0 = 1 + 0.01 sin(k.x),
k = 2 pi (1, 2, 3) / 256; populations stored as FP32 deviations (headline), and as FP64,
BF16 and FP16 (variants). A step is one launch of the step kernel over all 256^3 nodes.

Prints one JSON line: MLUPS (= nodes * steps / 1e6 / s) of the FP32 form, the roofline of
the step kernel (algorithmic bytes per launch / HIP-event launch time vs 8 TB/s), the
variants, the error of every form against the exact discrete solution (the FP64 reference
of this workload), and the FP64 CPU oracle timed on the host (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
Q = 19


KERNEL_SOURCES = ["step.hip", "node.h", "lattice.h", "args.h"]


def kernel_source_hash() -> str:
    """SHA-256 over the step kernel's sources (tags the traffic counters with the code they
    were taken from)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_01774_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(precision: str):
    """HBM bytes per launch of the step kernel on this workload, from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE, copy-calibrated), or None if the
    summary is missing or was taken from different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"step_{precision}_decay256_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return float(vals["traffic_bytes_per_launch"])


def bytes_per_lup(precision: str) -> int:
    """Algorithmic bytes per lattice update: every stored population read once and written
    once (uniform tensor and velocity travel in kernel arguments)."""
    return 2 * Q * {"f64": 8, "f32": 4, "bf16": 2, "fp16": 2}[precision]


def exact_phi(prob, steps):
    """Exact discrete solution of the u = 0 decay workload after `steps` steps (the FP64
    oracle equals it to roundoff; see tests/test_oracle_pins.py)."""
    import numpy as np
    from oracle import symbol as sy
    n = prob.nx
    k = 2 * np.pi * np.array(prob.meta["mode"]) / n
    v = sy.mode_history(k, prob.d6, [steps])[0]
    x = np.arange(n)[None, None, :]
    y = np.arange(n)[None, :, None]
    z = np.arange(n)[:, None, None]
    return prob.meta["c0"] + prob.meta["a0"] * (np.exp(1j * (k[0] * x + k[1] * y + k[2] * z)) * v[0]).imag


def run_form(prob, precision, steps, warmup, exact_cache):
    import numpy as np
    import torch
    from paper_2605_01774_amd import lattice

    lat = lattice.from_problem(prob, precision=precision, device="cuda:0")
    stream = torch.cuda.current_stream()
    lat.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = e0.elapsed_time(e1) / steps
    total = warmup + steps
    if total not in exact_cache:
        exact_cache[total] = exact_phi(prob, total)
    phi, _ = lat.moments()
    err = float(np.abs(phi.cpu().numpy() - exact_cache[total]).max() / prob.meta["a0"])
    mass = lat.reduce()[0]
    del lat
    torch.cuda.empty_cache()
    return dict(wall_s=wall, launch_ms=launch_ms, err=err, mass=mass)


def cpu_baseline(prob, seconds_target=15.0):
    """FP64 oracle on the host cores over a bounded sample of the same workload."""
    import numpy as np
    import oracle
    nth = os.cpu_count() or 1
    f = oracle.init_equilibrium(prob)
    t0 = time.perf_counter()
    f = oracle.run(prob, f, 1, nthreads=nth)
    one = time.perf_counter() - t0
    steps = max(1, min(50, int(seconds_target / max(one, 1e-3))))
    t0 = time.perf_counter()
    oracle.run(prob, f, steps, nthreads=nth)
    dt = time.perf_counter() - t0
    return dict(value=prob.n * steps / dt / 1e6, unit="MLUPS", cores=nth, kind="oracle",
                sample=f"{prob.nx}^3 grid, {steps} steps (+1 untimed), FP64 C++ oracle, OpenMP")


def adjoint_ratio(n=128, steps=500, ckpt=50):
    """Backward (recompute + adjoint steps) over forward wall time, FP32, log-tensor field
    workload n^3 x steps with a checkpoint every `ckpt` steps."""
    import torch
    from paper_2605_01774_amd import inputs, lattice
    from paper_2605_01774_amd.autograd import AdjointRun
    prob = inputs.adjoint_problem(n=n, steps=steps)
    lat = lattice.from_problem(prob, precision="f32", device="cuda:0")
    init = lat.save_state()
    target = torch.ones(lat.shape, dtype=torch.float64, device="cuda:0")
    times = []
    for rep in range(2):  # first repetition warms up allocations
        lat.load_state(*init)
        run = AdjointRun(lat, steps, ckpt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi = run.forward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run.backward(phi - target)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
    fwd, bwd = times[-1]
    plain_t0 = time.perf_counter()
    lat.load_state(*init)
    lat.step(steps)
    torch.cuda.synchronize()
    plain = time.perf_counter() - plain_t0
    return dict(workload=f"log-tensor field {n}^3, {steps} steps, checkpoint every {ckpt}, FP32",
                forward_ms=round(fwd * 1e3, 2), backward_ms=round(bwd * 1e3, 2),
                ratio=round(bwd / fwd, 3), plain_forward_ms=round(plain * 1e3, 2),
                ratio_vs_plain_forward=round(bwd / plain, 3))


def copy_calibration(nbytes, reps=20):
    """Plain device-to-device copies of nbytes (torch copy kernel), for scaling the HBM
    traffic counters: each launch reads and writes exactly nbytes."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_bytes": nbytes, "ms": ms, "gbs": 2 * nbytes / ms / 1e6}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--variants", default="f64,bf16,fp16")
    ap.add_argument("--variant-steps", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run plain copies of this many bytes (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the step kernel runs on one GPU's share; multi-GPU sharding is not built).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_01774_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prob = inputs.fourier_decay(n=args.n, steps=args.steps, precision="f32")
    exact_cache = {}
    print(f"[bench] f32 {args.n}^3: {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr, flush=True)
    main_r = run_form(prob, "f32", args.steps, args.warmup, exact_cache)
    n = prob.n
    mlups = n * args.steps / main_r["wall_s"] / 1e6
    bpl = bytes_per_lup("f32")
    achieved = bpl * n / (main_r["launch_ms"] * 1e-3) / 1e9
    variants = {}
    for prec in [p for p in args.variants.split(",") if p]:
        print(f"[bench] variant {prec}: {args.warmup} + {args.variant_steps} steps", file=sys.stderr, flush=True)
        r = run_form(prob, prec, args.variant_steps, args.warmup, exact_cache)
        b = bytes_per_lup(prec)
        ach = b * n / (r["launch_ms"] * 1e-3) / 1e9
        variants[prec] = dict(mlups=round(n * args.variant_steps / r["wall_s"] / 1e6, 1),
                              ms_per_step=round(r["launch_ms"], 4), bytes_per_lup=b,
                              achieved_gbs=round(ach, 1), frac=round(ach / HBM_PEAK_GBS, 4),
                              traffic=measured_traffic(prec),
                              max_err_vs_fp64_exact=r["err"])
    adj = None
    if not args.no_adjoint:
        print("[bench] adjoint / forward time (128^3 x 500, K = 50)", file=sys.stderr, flush=True)
        adj = adjoint_ratio()
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(prob)
    line = {
        "metric": "D3Q19 MLUPS + % HBM peak (FP32/BF16-store vs FP64); adjoint/forward time",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_r["wall_s"] * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"rotated Fourier-mode decay, D3Q19, periodic {args.n}^3, u=0, "
                               "uniform rotated tensor (1e-2,1e-4,1e-6), FP32 deviation storage",
                   "grid": [args.n] * 3, "nodes": n},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("f32"),
                     "algorithmic_bytes_per_launch": bpl * n,
                     "bytes_per_lup": bpl, "kernel_ms": round(main_r["launch_ms"], 4)},
        "max_err_vs_fp64_exact": main_r["err"],
        "variants": variants,
        "adjoint": adj,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
