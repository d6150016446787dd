"""Throughput of the fused collide-and-stream step on one MI355X.

Default workload (varfield512): source-driven transport with a spatially varying SPD tensor
field (the shape of Sec. 3.3), D3Q19, periodic 512^3: per node D = R(x) diag(d(x)) R(x)^T
with a smooth seeded rotation field and log10 d in [-4.5, 0] (local contrast up to 3e4),
velocity u = 0.02 sin(2 pi y / 512) e_x per node, Gaussian source field. The headline is the
FP64 form (the precision of the paper's results); the variants store the populations as FP32
deviations, as BF16 / FP16 deviations (round to nearest even), and as BF16 / FP16 with the
FP32 rest population and stochastic rounding ("bf16r", "fp16r"). Every variant's error is
taken after --err-steps steps (200) against the FP64 GPU run of the same input and step
count, in a run of its own after the timing. A step is one launch of the step kernel over
all 512^3 nodes. The headline runs exactly --warmup and --steps steps; the variants and
sub-workloads warm up and are timed for at least --min-ms (150 ms) of GPU time each, since
kernels of a few hundred microseconds run slower for the first tens of milliseconds.

Also reported, each in the same JSON line:
- the roofline of the headline's step kernel (algorithmic bytes per launch over the
  HIP-event launch time on the lattice's stream, against 8 TB/s), with the copy-calibrated
  HBM traffic from the committed counter summary while the kernel code matches it, and the
  rate of the library's streaming copy of 2 GiB in the same run (elbm_stream_copy, the step
  kernels' access style: a reference for the achievable bandwidth on the day, which varies
  by a few per cent between boxes) with the step kernel's ratio to it;
- sub-workloads in every form: decay256 (rotated Fourier-mode decay, 256^3, u = 0, uniform
  tensor; errors against the exact discrete solution) and porous384 (porous spheres,
  Dirichlet x faces, 384^3, tensor as a material table, with the effective conductivity
  column K_lx = -<q_l>/G_x over the middle half in x);
- the adjoint leg: backward (recompute + adjoint steps) over forward time of the FP32
  log-tensor-field inverse problem, 128^3 x 500 steps, checkpoint every 50;
- cpu_baseline: the FP64 CPU oracle on the host cores over a bounded sample of the same
  generator at 128^3 (per-step time from the difference of a K-step and a 1-step call, so
  the oracle's set-up, buffer allocation and array copies are not counted).

--workload decay256 | porous384 | plume256 makes another workload the headline (its
--headline form; FP64 by default).
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


def measured_traffic(precision: str, workload: str):
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
ALL_FORMS = ["f64", "f32", "bf16", "fp16", "bf16r", "fp16r"]


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
    oracle equals it to roundoff; see tests/test_oracle_pins.py), as an FP64 host array."""
    import numpy as np
    from oracle import symbol as sy
    n = prob.nx
    k = 2 * np.pi * np.array(prob.meta["mode"]) / n
    v = sy.mode_history(k, prob.d6, [steps], q=Q)[0]
    x = np.arange(n)[None, None, :]
    y = np.arange(n)[None, :, None]
    z = np.arange(n)[:, None, None]
    return prob.meta["c0"] + prob.meta["a0"] * (np.exp(1j * (k[0] * x + k[1] * y + k[2] * z)) * v[0]).imag


def run_form(prob, form, steps, warmup, err_steps, phases=False, min_ms=0.0):
    """Time `steps` launches of the step kernel after `warmup` untimed ones, then run the
    same lattice again from its initial state for `err_steps` steps for the error and mass
    figures. With min_ms > 0 (the forms other than the headline) the warmup is extended to
    at least min_ms of GPU time, and the timed steps to at least min_ms: kernels of a few
    hundred microseconds run slower for the first tens of milliseconds after the GPU has
    been idle. Returns the wall time and per-launch time (HIP events on the lattice's
    stream) of the timed steps, the steps actually run, the final scalar field (FP64, on
    the GPU), the mass and, with Dirichlet walls, K_eff."""
    import math
    import torch
    from paper_2605_01774_amd import lattice

    base, opts = FORMS[form]
    lat = lattice.from_problem(prob, precision=base, device="cuda:0", q=Q, phases=phases, **opts)
    init = lat.save_state()
    stream = lat.stream

    def timed(k):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        lat.step(k)
        e1.record(stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, e0.elapsed_time(e1)

    n_warm = warmup
    _, warm_ms = timed(warmup) if warmup else (0.0, 0.0)
    if min_ms > 0:
        if warmup:
            est = warm_ms / warmup
        else:
            est = timed(1)[1]
            n_warm += 1
        extra = max(0, math.ceil((min_ms - warm_ms) / max(est, 1e-3)))
        if extra:
            timed(extra)
        n_warm += extra
        steps = max(steps, math.ceil(min_ms / max(est, 1e-3)))
    wall, ev_ms = timed(steps)
    launch_ms = ev_ms / steps
    lat.load_state(*init)
    lat.step(err_steps)
    phi, q = lat.moments()
    k_eff = None
    if prob.bc_x == "dirichlet":
        # effective conductivity column K_lx = -<q_l> / G_x over the middle half in x, with
        # the imposed gradient G_x between the wall planes half a cell outside the domain
        x0, x1 = prob.nx // 4, 3 * prob.nx // 4
        g = (prob.phi_hi - prob.phi_lo) / prob.nx
        k_eff = [float(v) for v in (-q[:, :, :, x0:x1].mean(dim=(1, 2, 3)) / g).cpu()]
    del q
    mass = lat.reduce()[0]
    counters = lat.counters()
    del lat, init
    torch.cuda.empty_cache()
    return dict(wall_s=wall, launch_ms=launch_ms, steps=steps, warmup=n_warm, phi=phi, mass=mass,
                k_eff=k_eff, fallback=int(counters["fallback_nodes"]),
                nonfinite=int(counters["nonfinite"]))


def field_error(prob, phi, ref):
    """max |phi - ref| over the largest deviation of ref from the background phi_ref
    (device tensors, FP64)."""
    scale = float((ref - prob.phi_ref).abs().max()) or 1.0
    return float((phi - ref).abs().max()) / scale


def run_workload(wl, steps, warmup, err_steps, forms, phases, log, headline=None, min_ms=0.0):
    """Every form of one workload: timings, and the errors after err_steps steps against the
    workload's FP64 reference (the GPU FP64 run of the same input and step count, or for
    decay256 the exact discrete solution) with mass errors. The headline form runs exactly
    `warmup` + `steps` steps; the others at least min_ms of warmup and of timed work."""
    import torch
    desc, _, ref_kind = WORKLOADS[wl]
    log(f"building the {wl} workload")
    prob = make_problem(wl, steps)
    ref = None
    if ref_kind == "exact":
        ref = torch.as_tensor(exact_phi(prob, err_steps), device="cuda:0")
    out = {}
    order = (["f64"] if "f64" in forms else []) + [f for f in forms if f != "f64"]
    for form in order:
        log(f"{wl} {form}: timing, then {err_steps} steps for the error")
        r = run_form(prob, form, steps, warmup, err_steps, phases=phases,
                     min_ms=0.0 if form == headline else min_ms)
        phi = r.pop("phi")
        if ref_kind == "gpu_f64" and form == "f64":
            ref = phi
            r["err"], r["mass_err"] = None, None
        elif ref is not None:
            r["err"] = field_error(prob, phi, ref)
            ref_mass = float(ref.sum())
            r["mass_err"] = abs(r["mass"] - ref_mass) / abs(ref_mass)
        else:
            r["err"], r["mass_err"] = None, None
        del phi
        b = bytes_per_lup(form, prob, phases)
        ach = b * prob.n / (r["launch_ms"] * 1e-3) / 1e9
        r.update(bytes_per_lup=b, achieved_gbs=ach, frac=ach / HBM_PEAK_GBS,
                 mlups=prob.n * r["steps"] / r["wall_s"] / 1e6)
        out[form] = r
    del ref
    torch.cuda.empty_cache()
    return prob, out


def form_summary(r, form, wl_tag):
    s = dict(mlups=round(r["mlups"], 1), ms_per_step=round(r["launch_ms"], 4),
             steps=r["steps"], warmup=r["warmup"],
             bytes_per_lup=r["bytes_per_lup"], achieved_gbs=round(r["achieved_gbs"], 1),
             frac=round(r["frac"], 4), traffic=measured_traffic(form, wl_tag),
             max_err=r["err"], mass_err=r["mass_err"], fallback_node_updates=r["fallback"])
    if r["k_eff"] is not None:
        s["k_eff_x"] = [round(v, 8) for v in r["k_eff"]]
    return s


def cpu_baseline(wl, n=128, seconds_target=12.0):
    """FP64 CPU oracle on the host cores over a bounded sample of the workload's generator
    at n^3: per-step time from the difference of a K-step and a 1-step call, so the oracle's
    set-up (S per node), its buffer allocation and the array copies are not counted."""
    import oracle
    nth = os.cpu_count() or 1
    prob = make_problem(wl, 10, n=n)
    f = oracle.init_equilibrium(prob, q=Q)

    def timed(k, threads):
        t0 = time.perf_counter()
        oracle.run(prob, f, k, nthreads=threads, q=Q)
        return time.perf_counter() - t0

    t1 = timed(1, nth)
    t2 = timed(2, nth)
    per = max(t2 - t1, 1e-4)
    k = max(3, min(200, int(seconds_target / per)))
    tk = timed(k, nth)
    per = (tk - t1) / (k - 1)
    # one thread: the difference of a 2-step and a 1-step call
    s1 = timed(1, 1)
    s2 = timed(2, 1)
    return dict(value=round(prob.n / per / 1e6, 2), unit="MLUPS", cores=nth, kind="oracle",
                sample=(f"{wl} generator (same seed) at {n}^3, D3Q{Q}, FP64 C++ oracle with OpenMP: "
                        f"({k}-step call - 1-step call) / {k - 1}; set-up, allocation and copies "
                        "excluded"),
                value_single_thread=round(prob.n / max(s2 - s1, 1e-4) / 1e6, 3))


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
    del lat, run
    torch.cuda.empty_cache()
    return dict(workload=f"log-tensor field {n}^3, {steps} steps, checkpoint every {ckpt}, FP32",
                forward_ms=round(fwd * 1e3, 2), backward_ms=round(bwd * 1e3, 2),
                ratio=round(bwd / fwd, 3), plain_forward_ms=round(plain * 1e3, 2),
                ratio_vs_plain_forward=round(bwd / plain, 3))


def copy_rate(nbytes, reps=20, warm_ms=100.0):
    """Plain device-to-device copies of nbytes (torch copy kernel, each launch reads and
    writes exactly nbytes) after at least warm_ms of warmup copies: ms per copy and GB/s
    moved (2 nbytes per copy)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    spent = 0.0
    while True:
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        spent += ms * reps
        if spent >= warm_ms:
            break
    del a, b
    torch.cuda.empty_cache()
    return ms, 2 * nbytes / ms / 1e6


def stream_copy_rate(nbytes=1 << 30, reps=20, warm_ms=100.0):
    """The library's streaming copy (elbm_stream_copy: 16 bytes per lane, nontemporal loads
    and stores, like the step kernels) of nbytes, after at least warm_ms of warmup copies,
    timed with HIP events on the lattice's stream: GB/s moved (2 nbytes per copy)."""
    import torch
    from paper_2605_01774_amd import lattice
    lat = lattice.Lattice(64, 4, 4, precision="f32", device="cuda:0", q=Q)
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    spent = 0.0
    while True:
        e0.record(lat.stream)
        for _ in range(reps):
            lat.stream_copy(a, b)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        spent += ms * reps
        if spent >= warm_ms:
            break
    if not torch.equal(a, b):
        raise SystemExit("stream copy check failed")
    del a, b, lat
    torch.cuda.empty_cache()
    return 2 * nbytes / ms / 1e6


def copy_calibration(nbytes, reps=20):
    """Plain copies for scaling the HBM traffic counters (see copy_rate)."""
    ms, gbs = copy_rate(nbytes, reps)
    print(json.dumps({"copy_bytes": nbytes, "ms": ms, "gbs": gbs}), flush=True)


WORKLOADS = {
    # name: (description, default timed steps, error reference)
    "varfield512": ("source-driven transport, D3Q19, periodic 512^3, per-node rotated tensor "
                    "field (contrast up to 3e4), shear velocity field, Gaussian source field",
                    20, "gpu_f64"),
    "decay256": ("rotated Fourier-mode decay, D3Q19, periodic 256^3, u=0, uniform rotated "
                 "tensor (1e-2,1e-4,1e-6)", 20, "exact"),
    "porous384": ("porous conduction, D3Q19, 384^3, overlapping spheres (fluid 0.4), rotated "
                  "1e4:1 solid tensor, anti-bounce-back Dirichlet x faces", 20, "gpu_f64"),
    "plume256": ("advected anisotropic Gaussian on a zero background (shape of Sec. 3.1), "
                 "D3Q19, periodic 256^3, sigma0 = 8, uniform rotated tensor (1e-2,1e-3,1e-4) and "
                 "velocity (0.04,0.02,0.01); positivity fallback at most nodes", 20, "gpu_f64"),
}
# workloads made of a few materials: the tensor is given as a material table by default
MATERIAL_WORKLOADS = {"porous384"}
SIZES = {"varfield512": 512, "decay256": 256, "porous384": 384, "plume256": 256}


def make_problem(workload: str, steps: int, n: int = 0):
    """The workload's seeded inputs; the 512^3 field workload is generated on the GPU (FP64,
    torch) when it is timed there, and on the host for the CPU oracle's sample."""
    from paper_2605_01774_amd import inputs
    n = n or SIZES[workload]
    if workload == "decay256":
        return inputs.fourier_decay(n=n, steps=steps, precision="f32")
    if workload == "varfield512":
        on_gpu = n == SIZES[workload]
        return inputs.variable_tensor_source(n=n, steps=steps, precision="f32",
                                             device="cuda:0" if on_gpu else None)
    if workload == "porous384":
        return inputs.porous_spheres(n=n, steps=steps, precision="f32")
    if workload == "plume256":
        return inputs.gaussian_plume(n=n, steps=steps, sigma0=8.0 * n / 256, angles=(120, 90, 135),
                                     u=(0.04, 0.02, 0.01))
    raise SystemExit(f"unknown workload {workload}")


def wl_tag_of(wl, phases):
    """Tag of the counter summaries: the workload, the tensor form where it is not the
    default, and the velocity set where it is not D3Q19."""
    tag = wl + ("_field" if (wl in MATERIAL_WORKLOADS and not phases) else "")
    return tag + ("" if Q == 19 else f"_q{Q}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="varfield512", choices=sorted(WORKLOADS))
    ap.add_argument("--headline", default="f64", choices=ALL_FORMS,
                    help="form whose throughput is the line's value")
    ap.add_argument("--q", type=int, default=19, choices=(19, 27), help="velocity set")
    ap.add_argument("--steps", type=int, default=None, help="timed steps (workload default)")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--err-steps", type=int, default=200,
                    help="steps after which every form's error against the reference is taken")
    ap.add_argument("--min-ms", type=float, default=150.0,
                    help="least warmup and timed GPU time of the forms other than the headline")
    ap.add_argument("--forms", default=",".join(ALL_FORMS), help="forms of the headline workload")
    ap.add_argument("--sub", default="decay256,porous384",
                    help="sub-workloads timed in every form ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--tensor", choices=("auto", "field", "phases"), default="auto",
                    help="tensor input form of the headline workload: per-node field, or "
                         "material table + per-node index (auto: table for workloads made of a "
                         "few materials)")
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

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    wl = args.workload
    desc, def_steps, ref_kind = WORKLOADS[wl]
    phases = args.tensor == "phases" or (args.tensor == "auto" and wl in MATERIAL_WORKLOADS)
    if phases and wl not in MATERIAL_WORKLOADS:
        raise SystemExit(f"--tensor phases: {wl} has no material table")
    if phases:
        desc += "; tensor as a 2-entry material table + 1-byte index per node"
    steps = args.steps if args.steps is not None else def_steps
    forms = [f for f in args.forms.split(",") if f]
    if args.headline not in forms:
        forms.insert(0, args.headline)
    prob, res = run_workload(wl, steps, args.warmup, args.err_steps, forms, phases, log,
                             headline=args.headline, min_ms=args.min_ms)
    n = prob.n
    grid = [prob.nx, prob.ny, prob.nz]
    tag = wl_tag_of(wl, phases)
    head = res[args.headline]
    variants = {f: form_summary(r, f, tag) for f, r in res.items() if f != args.headline}

    subs = {}
    for sw in [s for s in args.sub.split(",") if s and s != wl]:
        sph = sw in MATERIAL_WORKLOADS
        sforms = ["f64", "f32", "bf16", "bf16r"] if sw == "porous384" else ALL_FORMS
        sprob, sres = run_workload(sw, steps, args.warmup, args.err_steps, sforms, sph, log,
                                   min_ms=args.min_ms)
        subs[sw] = dict(description=WORKLOADS[sw][0] + ("; tensor as a material table" if sph else ""),
                        grid=[sprob.nx, sprob.ny, sprob.nz],
                        error_reference=("exact discrete solution" if WORKLOADS[sw][2] == "exact"
                                         else "GPU FP64 run"),
                        forms={f: form_summary(r, f, wl_tag_of(sw, sph)) for f, r in sres.items()})
        del sprob

    adj = None
    if not args.no_adjoint and Q == 19:
        log("adjoint / forward time (128^3 x 500, K = 50)")
        adj = adjoint_ratio()
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(wl)
    log("plain 1 GiB device copy (the box's bandwidth on this run)")
    log("the library's streaming copy, 2 GiB (achievable-bandwidth reference)")
    copy_gbs = stream_copy_rate(2 << 30)
    err_ref = ("exact discrete solution (u = 0 Fourier symbol, equal to the FP64 oracle to "
               "roundoff), max |phi - exact| / a0" if ref_kind == "exact" else
               "GPU FP64 run of the same input and step count, max |phi - phi64| / "
               "max |phi64 - phi_ref|")
    achieved = head["achieved_gbs"]
    bpl = head["bytes_per_lup"]
    line = {
        "metric": "D3Q19 MLUPS + % HBM peak (FP32/BF16-store vs FP64); adjoint/forward time"
                  if Q == 19 else "D3Q27 MLUPS + % HBM peak (FP32/BF16-store vs FP64)",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["wall_s"] * 1e3 / steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": FORMS[args.headline][0] if args.headline in ("f64", "f32") else args.headline,
        "data": "synthetic",
        "config": {"workload": f"{wl}: {desc}; headline form {args.headline}",
                   "grid": grid, "nodes": n},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.headline, tag),
                     "algorithmic_bytes_per_launch": bpl * n,
                     "bytes_per_lup": bpl, "kernel_ms": round(head["launch_ms"], 4),
                     "stream_copy_gbs": round(copy_gbs, 1),
                     "over_stream_copy": round(achieved / copy_gbs, 4)},
        "max_err": head["err"],
        "mass_err": head["mass_err"],
        "error_reference": err_ref,
        "error_steps": args.err_steps,
        "k_eff_x": None if head["k_eff"] is None else [round(v, 8) for v in head["k_eff"]],
        "variants": variants,
        "sub_workloads": subs,
        "adjoint": adj,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
