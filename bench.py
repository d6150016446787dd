"""Throughput of the fused collide-and-stream step on one MI355X.

Default workload (decay256): rotated Fourier-mode decay, D3Q19, periodic 256^3, u = 0,
uniform tensor R diag(1e-2, 1e-4, 1e-6) R^T with a seeded random rotation,
phi0 = 1 + 0.01 sin(k.x), k = 2 pi (1, 2, 3) / 256; populations stored as FP32 deviations
(headline), and as FP64, BF16 and FP16 (variants). A step is one launch of the step kernel
over all 256^3 nodes.

--workload varfield512 (per-node tensor, velocity and source fields, 512^3, 1000 steps) and
--workload porous384 (spheres, Dirichlet walls, 384^3, 5000 steps; the tensor as a material
table, or with --tensor field per node) time the same kernels with per-node coefficients;
their errors are taken against the GPU FP64 run. The wall workload also reports the
effective-conductivity column K_lx = -<q_l>/G_x over the middle half in x (a transient
value at these step counts: the diffusion time across 384 nodes is ~1e7 steps).

Prints one JSON line: MLUPS (= nodes * steps / 1e6 / s) of the FP32 form, the roofline of
the step kernel (algorithmic bytes per launch / HIP-event launch time vs 8 TB/s), the
variants, the error of every form against the FP64 reference of the workload, the
adjoint/backward cost ratio (decay workload) and the FP64 CPU oracle timed on the host
(cpu_baseline).
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
Q = 19  # velocity set of the run (--q 27 times the D3Q27 build)


KERNEL_SOURCES = ["step_kernels.h", "node.h", "lattice.h", "args.h", "fmath.h"]


def code_without_comments(text: str) -> str:
    """C++ source with // comments removed and blank space collapsed to single spaces."""
    import re
    return " ".join(re.sub(r"//[^\n]*", "", text).split())


def kernel_source_hash() -> str:
    """SHA-256 over the step kernel's sources with comments and blank space removed (tags
    the traffic counters with the code they were taken from; editing a comment keeps it)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_01774_amd", "csrc", name)) as fh:
            h.update(code_without_comments(fh.read()).encode())
    return h.hexdigest()


def measured_traffic(precision: str, workload: str = "decay256"):
    """HBM bytes per launch of the step kernel on this workload, from the committed
    rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE, copy-calibrated), or None if the
    summary is missing or was taken from different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"step_{precision}_{workload}_hbm_traffic.txt")
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


# Storage forms timed by the bench: the library's precision forms, plus the 16-bit forms
# with the FP32 rest population and stochastic rounding ("bf16r", "fp16r").
FORMS = {"f64": ("f64", {}), "f32": ("f32", {}), "bf16": ("bf16", {}), "fp16": ("fp16", {}),
         "bf16r": ("bf16", dict(rest_fp32=True, stochastic_rounding=True)),
         "fp16r": ("fp16", dict(rest_fp32=True, stochastic_rounding=True))}


def bytes_per_lup(precision: str, prob=None, phases: bool = False) -> int:
    """Algorithmic bytes per lattice update: every stored population read once and written
    once, plus one read of each per-node coefficient field the workload has (tensor 6,
    velocity 3, source 1 values in the arithmetic type; a tensor given as a material table
    costs the 1-byte material index, the table itself stays in cache); uniform coefficients
    travel in kernel arguments."""
    if precision.endswith("r"):
        b = 2 * (4 + (Q - 1) * 2)  # FP32 rest plane + 18 16-bit planes
    else:
        b = 2 * Q * {"f64": 8, "f32": 4, "bf16": 2, "fp16": 2}[precision]
    precision = FORMS[precision][0]
    if prob is not None:
        import numpy as np
        rb = 8 if precision == "f64" else 4
        comps = (0 if prob.d_uniform or phases else 6) + (0 if prob.u_uniform else 3)
        comps += 1 if (prob.r is not None and np.ndim(prob.r) > 0) else 0
        b += comps * rb + (1 if phases else 0)
    return b


def exact_phi(prob, steps):
    """Exact discrete solution of the u = 0 decay workload after `steps` steps (the FP64
    oracle equals it to roundoff; see tests/test_oracle_pins.py)."""
    import numpy as np
    from oracle import symbol as sy
    n = prob.nx
    k = 2 * np.pi * np.array(prob.meta["mode"]) / n
    v = sy.mode_history(k, prob.d6, [steps], q=Q)[0]
    x = np.arange(n)[None, None, :]
    y = np.arange(n)[None, :, None]
    z = np.arange(n)[:, None, None]
    return prob.meta["c0"] + prob.meta["a0"] * (np.exp(1j * (k[0] * x + k[1] * y + k[2] * z)) * v[0]).imag


def run_form(prob, precision, steps, warmup, phases=False):
    """Time `steps` launches of the step kernel after `warmup` untimed ones. Returns the
    wall time, the per-launch time from HIP events on the lattice's stream, the final
    scalar field (FP64, host) and the mass."""
    import torch
    from paper_2605_01774_amd import lattice

    base, opts = FORMS[precision]
    lat = lattice.from_problem(prob, precision=base, device="cuda:0", q=Q, phases=phases, **opts)
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
    phi, q = lat.moments()
    k_eff = None
    if prob.bc_x == "dirichlet":
        # effective conductivity column K_lx = -<q_l> / G_x over the middle half in x, with
        # the imposed gradient G_x between the wall planes half a cell outside the domain
        x0, x1 = prob.nx // 4, 3 * prob.nx // 4
        g = (prob.phi_hi - prob.phi_lo) / prob.nx
        k_eff = [float(v) for v in (-q[:, :, :, x0:x1].mean(dim=(1, 2, 3)) / g).cpu()]
    del q
    phi = phi.cpu().numpy()
    mass = lat.reduce()[0]
    del lat
    torch.cuda.empty_cache()
    return dict(wall_s=wall, launch_ms=launch_ms, phi=phi, mass=mass, k_eff=k_eff)


def cpu_baseline(prob, seconds_target=15.0):
    """FP64 oracle on the host cores over a bounded sample of the same workload."""
    import numpy as np
    import oracle
    nth = os.cpu_count() or 1
    f = oracle.init_equilibrium(prob, q=Q)
    t0 = time.perf_counter()
    f = oracle.run(prob, f, 1, nthreads=nth, q=Q)
    one = time.perf_counter() - t0
    steps = max(1, min(50, int(seconds_target / max(one, 1e-3))))
    t0 = time.perf_counter()
    f = oracle.run(prob, f, steps, nthreads=nth, q=Q)
    dt = time.perf_counter() - t0
    # one more step on a single thread
    t0 = time.perf_counter()
    oracle.run(prob, f, 1, nthreads=1, q=Q)
    dt1 = time.perf_counter() - t0
    return dict(value=prob.n * steps / dt / 1e6, unit="MLUPS", cores=nth, kind="oracle",
                sample=f"{prob.nx}^3 grid, D3Q{Q}, {steps} steps (+1 untimed), FP64 C++ oracle, OpenMP",
                value_single_thread=round(prob.n / dt1 / 1e6, 2))


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


WORKLOADS = {
    # name: (description, default steps, default variant forms, error reference)
    "decay256": ("rotated Fourier-mode decay, D3Q19, periodic 256^3, u=0, uniform rotated "
                 "tensor (1e-2,1e-4,1e-6)", 2000, "f64,bf16,fp16,bf16r,fp16r", "exact"),
    "varfield512": ("source-driven transport, D3Q19, periodic 512^3, per-node rotated tensor "
                    "field (contrast up to 3e4), shear velocity field, Gaussian source field",
                    1000, "f64,bf16,fp16,bf16r,fp16r", "gpu_f64"),
    "porous384": ("porous conduction, D3Q19, 384^3, overlapping spheres (fluid 0.4), rotated "
                  "1e4:1 solid tensor, anti-bounce-back Dirichlet x faces", 5000, "f64,bf16,bf16r",
                  "gpu_f64"),
    "plume256": ("advected anisotropic Gaussian on a zero background (shape of Sec. 3.1), "
                 "D3Q19, periodic 256^3, sigma0 = 8, uniform rotated tensor (1e-2,1e-3,1e-4) and "
                 "velocity (0.04,0.02,0.01); positivity fallback at most nodes", 1000,
                 "f64,bf16r", "gpu_f64"),
}
# workloads made of a few materials: the tensor is given as a material table by default
MATERIAL_WORKLOADS = {"porous384"}


def make_problem(workload: str, n: int, steps: int):
    from paper_2605_01774_amd import inputs
    if workload == "decay256":
        return inputs.fourier_decay(n=n or 256, steps=steps, precision="f32")
    if workload == "varfield512":
        return inputs.variable_tensor_source(n=n or 512, steps=steps, precision="f32")
    if workload == "porous384":
        return inputs.porous_spheres(n=n or 384, steps=steps, precision="f32")
    if workload == "plume256":
        return inputs.gaussian_plume(n=n or 256, steps=steps, sigma0=8.0, angles=(120, 90, 135),
                                     u=(0.04, 0.02, 0.01))
    raise SystemExit(f"unknown workload {workload}")


def field_error(prob, phi, ref):
    """max |phi - ref| over the largest deviation of ref from the background phi_ref."""
    import numpy as np
    scale = float(np.abs(ref - prob.phi_ref).max()) or 1.0
    return float(np.abs(phi - ref).max() / scale)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="decay256", choices=sorted(WORKLOADS))
    ap.add_argument("--q", type=int, default=19, choices=(19, 27), help="velocity set")
    ap.add_argument("--steps", type=int, default=None, help="timed steps (workload default)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=0, help="grid edge (workload default)")
    ap.add_argument("--variants", default=None, help="extra precision forms, comma separated")
    ap.add_argument("--variant-steps", type=int, default=None,
                    help="timed steps of the variants (decay workload; default 500)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--tensor", choices=("auto", "field", "phases"), default="auto",
                    help="tensor input form: per-node field, or material table + per-node "
                         "index (auto: table for workloads made of a few materials)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run plain copies of this many bytes (counter calibration)")
    args = ap.parse_args()
    global Q
    Q = args.q
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the step kernel runs on one GPU's share; multi-GPU sharding is not built).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    desc, def_steps, def_variants, ref_kind = WORKLOADS[args.workload]
    phases = args.tensor == "phases" or (args.tensor == "auto" and args.workload in MATERIAL_WORKLOADS)
    if phases and args.workload not in MATERIAL_WORKLOADS:
        raise SystemExit(f"--tensor phases: {args.workload} has no material table")
    # tag of the counter summaries: the workload, the tensor form where it is not the
    # default, and the velocity set where it is not D3Q19
    wl_tag = args.workload + ("_field" if (args.workload in MATERIAL_WORKLOADS and not phases) else "")
    wl_tag += "" if Q == 19 else f"_q{Q}"
    if phases:
        desc += "; tensor as a 2-entry material table + 1-byte index per node"
    steps = args.steps if args.steps is not None else def_steps
    variants_arg = def_variants if args.variants is None else args.variants
    forms = [p for p in variants_arg.split(",") if p and p != "f32"]
    if ref_kind == "exact":
        vsteps = args.variant_steps if args.variant_steps is not None else min(500, steps)
    else:
        vsteps = steps  # every form is compared with the FP64 run at the same time
    print(f"[bench] building the {args.workload} workload", file=sys.stderr, flush=True)
    prob = make_problem(args.workload, args.n, steps)
    n = prob.n
    grid = [prob.nx, prob.ny, prob.nz]

    refs = {}

    def reference(total):
        if ref_kind == "exact":
            if total not in refs:
                refs[total] = exact_phi(prob, total)
            return refs[total]
        return refs.get(total)

    results = {}
    order = (["f64"] if "f64" in forms and ref_kind == "gpu_f64" else []) + ["f32"] + \
        [p for p in forms if not (p == "f64" and ref_kind == "gpu_f64")]
    for prec in order:
        k = steps if prec == "f32" else vsteps
        print(f"[bench] {prec} {grid}: {args.warmup} warmup + {k} timed steps", file=sys.stderr, flush=True)
        r = run_form(prob, prec, k, args.warmup, phases=phases)
        if ref_kind == "gpu_f64" and prec == "f64":
            refs[args.warmup + k] = r["phi"]
        ref = reference(args.warmup + k)
        r["err"] = None if ref is None else field_error(prob, r["phi"], ref)
        # total mass sum(phi) against the reference field's (FP64 sums)
        r["mass_err"] = None if ref is None else float(abs(r["mass"] - ref.sum()) / abs(ref.sum()))
        if ref_kind == "gpu_f64" and prec == "f64":
            r["err"] = None  # the reference itself
            r["mass_err"] = None
        del r["phi"]
        results[prec] = (k, r)

    def summary(prec):
        k, r = results[prec]
        b = bytes_per_lup(prec, prob, phases)
        ach = b * n / (r["launch_ms"] * 1e-3) / 1e9
        return k, r, b, ach

    variants = {}
    for prec in forms:
        k, r, b, ach = summary(prec)
        variants[prec] = dict(mlups=round(n * k / r["wall_s"] / 1e6, 1),
                              ms_per_step=round(r["launch_ms"], 4), bytes_per_lup=b,
                              achieved_gbs=round(ach, 1), frac=round(ach / HBM_PEAK_GBS, 4),
                              traffic=measured_traffic(prec, wl_tag),
                              max_err=r["err"], mass_err=r["mass_err"])
        if r["k_eff"] is not None:
            variants[prec]["k_eff_x"] = [round(v, 8) for v in r["k_eff"]]
    k, main_r, bpl, achieved = summary("f32")
    mlups = n * steps / main_r["wall_s"] / 1e6
    adj = None
    if not args.no_adjoint and args.workload == "decay256" and Q == 19:
        print("[bench] adjoint / forward time (128^3 x 500, K = 50)", file=sys.stderr, flush=True)
        adj = adjoint_ratio()
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(prob)
    err_ref = ("exact discrete solution (u = 0 Fourier symbol, equal to the FP64 oracle to "
               "roundoff), max |phi - exact| / a0" if ref_kind == "exact" else
               "GPU FP64 run of the same workload and step count, max |phi - phi64| / "
               "max |phi64 - phi_ref|")
    line = {
        "metric": "D3Q19 MLUPS + % HBM peak (FP32/BF16-store vs FP64); adjoint/forward time"
                  if Q == 19 else "D3Q27 MLUPS + % HBM peak (FP32/BF16-store vs FP64)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_r["wall_s"] * 1e3 / steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}; FP32 deviation storage",
                   "grid": grid, "nodes": n},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("f32", wl_tag),
                     "algorithmic_bytes_per_launch": bpl * n,
                     "bytes_per_lup": bpl, "kernel_ms": round(main_r["launch_ms"], 4)},
        "max_err": main_r["err"],
        "mass_err": main_r["mass_err"],
        "error_reference": err_ref,
        "k_eff_x": None if main_r["k_eff"] is None else [round(v, 8) for v in main_r["k_eff"]],
        "variants": variants,
        "adjoint": adj,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
