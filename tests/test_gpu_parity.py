"""GPU path (through the C ABI) against the FP64 CPU oracle, element by element.

FP64 bar: max_{x,i} |g_gpu - g_oracle| / max |g_oracle| <= 1e-12 (same seeded inputs, same
ghost floor). Reduced-precision forms are compared with the FP64 oracle at the tolerances
stated in each test (measured, with margin).
"""
import numpy as np
import pytest

import oracle
from oracle import symbol as sy
from paper_2605_01774_amd import inputs as I
from gpuhelp import banner, gpu_lattice, gpu_pops, rel_err, to_lib_order

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12


def _oracle_run(prob, steps, **kw):
    return oracle.run(prob, oracle.init_equilibrium(prob), steps, **kw)


def _random_fields(n3, rng, u_amp=0.05, ratio=1e3):
    nz, ny, nx = n3
    n = nx * ny * nz
    ds = []
    for _ in range(n):
        d = 1e-2 * 10.0 ** (-np.log10(ratio) * rng.uniform(0, 1, 3))
        ds.append(I.rotated_tensor(tuple(d), I.random_rotation(rng)))
    d6 = np.stack(ds, axis=1).reshape((6,) + n3)
    u = rng.uniform(-u_amp, u_amp, size=(3,) + n3)
    return d6, u


# ------------------------------------------------------------------------------------------
# FP64 parity
# ------------------------------------------------------------------------------------------
def test_f64_gaussian_plume_full_size():
    """Advected anisotropic Gaussian, 32^3, 200 steps (full size of the small workload)."""
    banner("f64 gaussian plume 32^3 x 200")
    prob = I.gaussian_plume(n=32, steps=200)
    lat = gpu_lattice(prob, "f64")
    lat.step(prob.steps)
    err = rel_err(gpu_pops(lat), _oracle_run(prob, prob.steps))
    print(f"f64 gaussian 32^3x200 rel err {err:.3e}")
    assert err <= F64_TOL


@pytest.mark.parametrize("shape", [(37, 29, 23), (5, 3, 2), (64, 1, 1), (1, 7, 9)])
def test_f64_ragged_with_all_fields(shape):
    """Ragged and degenerate grids with per-node tensor, velocity and source fields."""
    banner(f"f64 ragged fields {shape}")
    nx, ny, nz = shape
    n3 = (nz, ny, nx)
    rng = np.random.default_rng(21)
    d6, u = _random_fields(n3, rng)
    phi0 = 1.0 + 0.3 * rng.uniform(-1, 1, n3)
    r = 1e-3 * rng.uniform(-1, 1, n3)
    prob = I.Problem("ragged", nx, ny, nz, d6, u, phi0, steps=30, r=r, phi_ref=1.0)
    lat = gpu_lattice(prob, "f64")
    lat.step(prob.steps)
    err = rel_err(gpu_pops(lat), _oracle_run(prob, prob.steps))
    print(f"f64 ragged {shape} rel err {err:.3e}")
    assert err <= F64_TOL
    # moments at the same time level
    phi, q = lat.moments()
    ph_o, _, q_o = oracle.moments(prob, _oracle_run(prob, prob.steps))
    assert np.abs(phi.cpu().numpy() - ph_o).max() <= F64_TOL * np.abs(ph_o).max()
    assert np.abs(q.cpu().numpy() - q_o).max() <= 1e-10 * max(np.abs(q_o).max(), 1e-300)


def test_f64_uniform_source_and_velocity():
    banner("f64 uniform source + velocity")
    rng = np.random.default_rng(22)
    n3 = (9, 11, 13)
    phi0 = 1.0 + 0.2 * rng.uniform(-1, 1, n3)
    prob = I.Problem("src", 13, 11, 9, I.rotated_tensor((3e-2, 1e-3, 1e-5), I.euler_zyz(10, 20, 30)),
                     np.array([0.03, -0.01, 0.02]), phi0, steps=25, r=2e-4, phi_ref=1.0)
    lat = gpu_lattice(prob, "f64")
    lat.step(prob.steps)
    err = rel_err(gpu_pops(lat), _oracle_run(prob, prob.steps))
    print(f"f64 uniform source rel err {err:.3e}")
    assert err <= F64_TOL


def test_f64_porous_dirichlet_reduced():
    """Porous spheres with anti-bounce-back Dirichlet planes (reduced to 24^3)."""
    banner("f64 porous 24^3 x 60")
    prob = I.porous_spheres(n=24, steps=60)
    lat = gpu_lattice(prob, "f64")
    lat.step(prob.steps)
    err = rel_err(gpu_pops(lat), _oracle_run(prob, prob.steps))
    print(f"f64 porous rel err {err:.3e}")
    assert err <= F64_TOL


def test_f64_variable_tensor_source_reduced():
    banner("f64 variable tensor + source 24^3 x 40")
    prob = I.variable_tensor_source(n=24, steps=40)
    lat = gpu_lattice(prob, "f64")
    lat.step(prob.steps)
    err = rel_err(gpu_pops(lat), _oracle_run(prob, prob.steps))
    print(f"f64 variable tensor rel err {err:.3e}")
    assert err <= F64_TOL


@pytest.mark.parametrize("n", [12, 24])
@pytest.mark.parametrize("q", [19, 27])
def test_f64_time_dependent_source_vs_oracle(q, n):
    """Separable time-dependent source R(x, t) = s(t) R(x) (elbm_set_source_scale): each
    step uses its own midpoint amplitude for both half-steps (Sec. 3.3), a pending half
    keeps its amplitude, and readouts in between include it. Against the oracle stepping
    with R scaled per step; manufactured-source problem (variable tensor, u = 1/n per
    component: |u| = 0.14 on 12^3) for 20 steps. The start is an equilibrium, whose ghost
    parts are rounding-level: the FP64 ghost floor tau = 1e-9 keeps their effect on the
    update near 1e-14 (tests/test_oracle_conditioning.py), so populations match to 1e-12
    of max |g| and phi to 1e-13 absolute (phi lies in [1, 3])."""
    banner(f"f64 time-dependent source, D3Q{q}, {n}^3")
    prob = I.manufactured_source(n=n, t_end=20 / float(n * n))
    F = prob.r.copy()
    lat = gpu_lattice(prob, "f64", q=q)
    f = oracle.init_equilibrium(prob, q=q)
    for m in range(prob.steps):
        sc = 3.0 * prob.meta["scale"](m) * (1.0 + 0.5 * np.sin(m))
        lat.set_source_scale(sc)
        lat.step(1)
        prob.r = F * sc
        f = oracle.run(prob, f, 1, q=q)
        if m in (0, 4, prob.steps - 1):
            err = rel_err(gpu_pops(lat), f)
            phi_err = np.abs(lat.moments()[0].cpu().numpy() - f.sum(0)).max()
            print(f"step {m + 1}: populations {err:.3e}, phi abs {phi_err:.3e}")
            assert err <= F64_TOL and phi_err <= 1e-13


def test_f64_log_tensor_field():
    banner("f64 log tensor 16^3 x 20")
    prob = I.adjoint_problem(n=16, steps=20, u=(0.02, 0.01, -0.01))
    lat = gpu_lattice(prob, "f64")
    lat.step(prob.steps)
    err = rel_err(gpu_pops(lat), _oracle_run(prob, prob.steps))
    print(f"f64 log tensor rel err {err:.3e}")
    assert err <= F64_TOL


def test_f64_fallback_and_exact_root():
    """Strongly non-equilibrium start: the positivity fallback fires at many nodes and the
    exact entropic root is taken at flagged nodes; counts match the oracle's."""
    banner("f64 fallback + exact root")
    rng = np.random.default_rng(23)
    n3 = (6, 7, 8)
    nz, ny, nx = n3
    d6, u = _random_fields(n3, rng, u_amp=0.08, ratio=1e4)
    prob = I.Problem("fb", nx, ny, nz, d6, u, np.ones(n3), steps=3, eps=1e-4)
    f0 = oracle.init_equilibrium(prob) * (1.0 + 0.9 * rng.uniform(-1, 1, (19,) + n3))
    for root in (-1.0, 0.3):
        lat = gpu_lattice(prob, "f64", root_rho=root)
        lat.set_populations(to_lib_order(f0))
        lat.reset_counters()
        lat.step(prob.steps)
        f_ref, _, _, (nfb, nfl) = oracle.run(prob, f0, prob.steps, root_rho=root, want_last=True)
        err = rel_err(gpu_pops(lat), f_ref)
        cnt = lat.counters()
        print(f"root={root}: rel err {err:.3e}, fallback {cnt['fallback_nodes']} vs {nfb}, "
              f"flagged {cnt['flagged_nodes']} vs {nfl}")
        assert err <= F64_TOL
        assert cnt["fallback_nodes"] == nfb and nfb > 0
        assert cnt["flagged_nodes"] == nfl
        if root >= 0:
            assert nfl > 0


def test_f64_decay_matches_symbol_full_size():
    """Rotated Fourier-mode decay at 256^3 for 2000 steps in FP64 equals the exact discrete
    solution from the u = 0 symbol; mass is conserved."""
    banner("f64 fourier decay 256^3 x 2000 vs symbol")
    prob = I.fourier_decay(n=256, steps=2000, precision="f64")
    lat = gpu_lattice(prob, "f64")
    m0 = lat.reduce()[0]
    lat.step(prob.steps)
    phi, _ = lat.moments()
    phi = phi.cpu().numpy()
    k = 2 * np.pi * np.array(prob.meta["mode"]) / 256
    v = sy.mode_history(k, prob.d6, [prob.steps])[0]
    x = np.arange(256)[None, None, :]
    y = np.arange(256)[None, :, None]
    z = np.arange(256)[:, None, None]
    exact = 1.0 + 0.01 * (np.exp(1j * (k[0] * x + k[1] * y + k[2] * z)) * v[0]).imag
    err = np.abs(phi - exact).max() / 0.01
    m1 = lat.reduce()[0]
    print(f"f64 decay vs symbol: max |phi - exact| / A0 = {err:.3e}; mass drift {(m1 - m0) / m0:.3e}")
    assert err < 1e-10
    assert abs(m1 - m0) / m0 < 1e-13


def test_f64_state_roundtrip_and_determinism():
    banner("f64 state roundtrip + determinism")
    prob = I.variable_tensor_source(n=16, steps=10)
    a = gpu_lattice(prob, "f64")
    a.step(5)
    f = a.populations()
    saved, st, pend = a.save_state()
    a.step(5)
    fa = a.populations().cpu().numpy()
    a.load_state(saved, st, pend)
    a.step(5)
    fb = a.populations().cpu().numpy()
    assert np.array_equal(fa, fb)
    b = gpu_lattice(prob, "f64")
    b.step(10)
    assert np.array_equal(b.populations().cpu().numpy(), fa)
    # canonical get/set populations round trip (no source pending after set)
    c = gpu_lattice(prob, "f64")
    c.set_populations(f)
    assert np.abs(c.populations().cpu().numpy() - f.cpu().numpy()).max() == 0.0


# ------------------------------------------------------------------------------------------
# Errors raised by the library
# ------------------------------------------------------------------------------------------
def test_error_codes():
    banner("error codes")
    from paper_2605_01774_amd import lattice
    from paper_2605_01774_amd._lib import ElbmError
    lat = lattice.Lattice(8, 8, 8, precision="f64", device="cuda:0")
    with pytest.raises(ElbmError) as e:
        lat.step(1)
    assert e.value.name == "ESTATE"
    with pytest.raises(ElbmError) as e:
        lat.set_diffusion(np.array([1e-2, 0.5, 0, 1e-2, 0, 1e-2]))
    assert e.value.name == "ENOTSPD"
    bad = np.tile(np.array([1e-2, 0, 0, 1e-2, 0, 1e-2])[:, None, None, None], (1, 8, 8, 8))
    bad[:, 3, 2, 1] = [-1.0, 0, 0, 1e-2, 0, 1e-2]
    with pytest.raises(ElbmError) as e:
        lat.set_diffusion(bad)
    assert e.value.name == "ENOTSPD"
    with pytest.raises(ElbmError) as e:
        lat.set_velocity(np.array([0.9, 0.0, 0.0]))
    assert e.value.name == "EVELOCITY"


# ------------------------------------------------------------------------------------------
# Reduced precision (FP32 arithmetic; FP32 / BF16 / FP16 storage)
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("prec,tol", [("f32", 2e-6), ("bf16", 5e-3), ("fp16", 1e-3)])
def test_reduced_precision_vs_oracle(prec, tol):
    """Errors of the reduced-precision forms against the FP64 oracle on the variable-tensor
    source workload (reduced to 24^3, 40 steps), relative to max |g|."""
    banner(f"{prec} vs oracle, variable tensor 24^3 x 40")
    prob = I.variable_tensor_source(n=24, steps=40)
    lat = gpu_lattice(prob, prec)
    lat.step(prob.steps)
    err = rel_err(gpu_pops(lat), _oracle_run(prob, prob.steps, tau=float(lat.cfg.ghost_floor)))
    print(f"{prec}: rel err vs FP64 oracle {err:.3e} (tol {tol:g})")
    assert err <= tol


@pytest.mark.parametrize("form", ["f32", "bf16", "fp16", "bf16r", "fp16r"])
def test_reduced_precision_vs_fp64_scheme(form):
    """The same workload against the oracle at the FP64 form's ghost floor (1e-9) instead of
    the reduced form's own (1e-4): this error adds the stabilizer change of the floor
    (Sec. 2.5, a smaller lambda - 1 where the ghost part is within a few tau phi of zero) to
    the rounding. Bound: the form's own tolerance above (f32 2e-6, bf16 5e-3, fp16 1e-3,
    with the FP32 rest and stochastic rounding 5e-3 and 1e-3) plus the floor's worst case.
    A node whose ghost norm is near tau phi can move by up to about
    |ln E|_max |Dh|_1 |Dh_i| / (tau^2 phi) ~ 0.06 x 19 tau phi = 1.1 tau phi per step
    (|u| <= 0.02 here), i.e. 3.4e-4 of max |g| ~ phi / 3 per step, 1.4e-2 over 40 steps."""
    banner(f"{form} vs oracle at the FP64 ghost floor, variable tensor 24^3 x 40")
    base = {"f32": "f32", "bf16": "bf16", "fp16": "fp16", "bf16r": "bf16", "fp16r": "fp16"}[form]
    kw = dict(rest_fp32=True, stochastic_rounding=True) if form.endswith("r") else {}
    own_tol = {"f32": 2e-6, "bf16": 5e-3, "fp16": 1e-3, "bf16r": 5e-3, "fp16r": 1e-3}[form]
    prob = I.variable_tensor_source(n=24, steps=40)
    lat = gpu_lattice(prob, base, **kw)
    lat.step(prob.steps)
    g = gpu_pops(lat)
    tau_own = float(lat.cfg.ghost_floor)
    err_own = rel_err(g, _oracle_run(prob, prob.steps, tau=tau_own))
    err64 = rel_err(g, _oracle_run(prob, prob.steps, tau=1e-9))
    print(f"{form}: vs oracle at its own floor {tau_own:g}: {err_own:.3e}; at the FP64 floor 1e-9: "
          f"{err64:.3e}")
    assert err_own <= own_tol
    assert err64 <= own_tol + 40 * 3.4e-4


# ------------------------------------------------------------------------------------------
# Row-vector kernel (rows of 64 V W nodes, DPP rotation for the x shift)
# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "fp16"])
@pytest.mark.parametrize("nx", [64, 128, 192, 256, 320, 384, 448, 512])
def test_vector_kernel_bitwise_equals_scalar(prec, nx, bc):
    """Same node arithmetic, different data movement (V nodes per lane, rows of W <= 8
    wavefronts, wall nodes writing their reflected populations themselves): populations
    must be bitwise equal to the one-node-per-thread kernel for every node width that fits
    the row, with tensor, velocity and source fields."""
    banner(f"vector vs scalar kernel {prec} nx={nx} {bc}")
    rng = np.random.default_rng(41)
    n3 = (5, 7, nx)
    d6, u = _random_fields(n3, rng, u_amp=0.04)
    phi0 = 1.0 + 0.2 * rng.uniform(-1, 1, n3)
    r = 1e-3 * rng.uniform(-1, 1, n3)
    prob = I.Problem("vec", nx, 7, 5, d6, u, phi0, steps=7, r=r, phi_ref=1.0, bc_x=bc,
                     phi_lo=1.3, phi_hi=0.8)
    lat = gpu_lattice(prob, prec, scalar_kernel=True)
    lat.step(prob.steps)
    ref = lat.populations().cpu().numpy()
    for width in (0, 1, 2, 4):
        lat = gpu_lattice(prob, prec, vector_width=width)
        lat.step(prob.steps)
        assert np.array_equal(lat.populations().cpu().numpy(), ref), width


COEF_MODES = [("uniform", "zero", "none"), ("uniform", "uniform", "uniform"), ("field", "zero", "field"),
              ("uniform", "field", "uniform"), ("field", "uniform", "none"), ("table", "field", "field"),
              ("table", "uniform", "uniform")]


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16r"])
@pytest.mark.parametrize("tensor,velocity,source", COEF_MODES)
def test_vector_kernel_coefficient_modes(prec, tensor, velocity, source, bc):
    """Every combination of how the coefficients are given reaches the row-vector kernel
    through its own loads (velocity and source issued before the populations, the tensor
    per node, early, or through the material index): uniform or per-node tensor or a
    material table, zero, uniform or per-node velocity, no, uniform or per-node source.
    States must be bitwise equal to the one-node-per-thread kernel's at every width."""
    banner(f"vector vs scalar {prec} tensor={tensor} u={velocity} source={source} {bc}")
    rng = np.random.default_rng(47)
    n3 = (5, 6, 256)
    nz, ny, nx = n3
    table = np.stack([I.rotated_tensor(d, I.random_rotation(rng))
                      for d in ((1e-2, 1e-3, 1e-4), (5e-3, 5e-3, 1e-5), (2e-3, 1e-4, 1e-4))])
    phase = rng.integers(0, 3, n3).astype(np.uint8)
    if tensor == "field":
        d6, _ = _random_fields(n3, rng)
    elif tensor == "table":
        d6 = np.moveaxis(table[phase], -1, 0)
    else:
        d6 = table[0]
    u = {"zero": np.zeros(3), "uniform": np.array([0.03, -0.02, 0.01]),
         "field": rng.uniform(-0.04, 0.04, (3,) + n3)}[velocity]
    r = {"none": None, "uniform": 2e-4, "field": 1e-3 * rng.uniform(-1, 1, n3)}[source]
    phi0 = 1.0 + 0.2 * rng.uniform(-1, 1, n3)
    prob = I.Problem("coef", nx, ny, nz, d6, u, phi0, steps=5, r=r, phi_ref=1.0, bc_x=bc,
                     phi_lo=1.3, phi_hi=0.8, meta=dict(phase=phase, d6_table=table))
    base, opts = ("bf16", dict(rest_fp32=True, stochastic_rounding=True)) if prec == "bf16r" else (prec, {})
    phases = tensor == "table"
    lat = gpu_lattice(prob, base, scalar_kernel=True, phases=phases, **opts)
    lat.step(prob.steps)
    ref = lat.populations().cpu().numpy()
    for width in (0, 1, 2, 4):
        if (base == "f64" and width == 4) or nx % (64 * max(width, 1)):
            continue
        lat = gpu_lattice(prob, base, vector_width=width, phases=phases, **opts)
        lat.step(prob.steps)
        assert np.array_equal(lat.populations().cpu().numpy(), ref), width


STORAGE_MODES = {"rest32": dict(rest_fp32=True), "sr": dict(stochastic_rounding=True),
                 "rest32+sr": dict(rest_fp32=True, stochastic_rounding=True)}


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("mode", sorted(STORAGE_MODES))
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("nx", [64, 192, 256, 512])
def test_vector_kernel_bitwise_storage_modes(prec, mode, nx, bc):
    """16-bit storage with the FP32 rest population and/or stochastic rounding: the two step
    kernels round the same values with the same random bits (counter = node, direction,
    time step), so their states stay bitwise equal."""
    banner(f"vector vs scalar kernel {prec} {mode} nx={nx} {bc}")
    rng = np.random.default_rng(43)
    n3 = (4, 5, nx)
    d6, u = _random_fields(n3, rng, u_amp=0.04)
    phi0 = 1.0 + 0.2 * rng.uniform(-1, 1, n3)
    r = 1e-3 * rng.uniform(-1, 1, n3)
    prob = I.Problem("vecsm", nx, 5, 4, d6, u, phi0, steps=6, r=r, phi_ref=1.0, bc_x=bc,
                     phi_lo=1.3, phi_hi=0.8)
    lat = gpu_lattice(prob, prec, scalar_kernel=True, **STORAGE_MODES[mode])
    lat.step(prob.steps)
    ref = lat.populations().cpu().numpy()
    for width in (1, 2, 4):
        if nx % (64 * width):
            continue
        lat = gpu_lattice(prob, prec, vector_width=width, **STORAGE_MODES[mode])
        lat.step(prob.steps)
        assert np.array_equal(lat.populations().cpu().numpy(), ref), width


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("kern", ["scalar", "vector"])
@pytest.mark.parametrize("mode", sorted(STORAGE_MODES) + ["plain"])
def test_fp16_state_independent_of_store_scale(mode, kern, bc):
    """FP16 runs the step on the stored values (value / scale) with phi_ref, eps, the source
    and the wall values scaled instead. With two power-of-two scales the physical states
    agree to FP16 rounding: deviations in the FP16 subnormal range at one scale and not at
    the other round differently, which can flip later roundings by an ulp (6e-5 at the
    largest deviations here, about 0.07; bound 1e-3). A source or wall value or phi_ref
    left unscaled would move them by 5e-3 or more. Tensor, velocity and source fields,
    20 steps."""
    banner(f"fp16 store scale independence {mode} {kern} {bc}")
    rng = np.random.default_rng(47)
    n3 = (5, 6, 256)
    d6, u = _random_fields(n3, rng, u_amp=0.04)
    phi0 = 1.0 + 0.2 * rng.uniform(-1, 1, n3)
    r = 1e-3 * rng.uniform(-1, 1, n3)
    prob = I.Problem("scale", 256, 6, 5, d6, u, phi0, steps=20, r=r, phi_ref=1.0, bc_x=bc,
                     phi_lo=1.3, phi_hi=0.8)
    kw = dict(STORAGE_MODES.get(mode, {}))
    kw.update(dict(scalar_kernel=True) if kern == "scalar" else dict(vector_width=2))
    pops = []
    for scale in (2.0 ** -8, 2.0 ** -5):
        lat = gpu_lattice(prob, "fp16", store_scale=scale, **kw)
        lat.step(prob.steps)
        pops.append(lat.populations().cpu().numpy())
        del lat
    diff = np.abs(pops[0] - pops[1]).max()
    print(f"max |state(2^-8) - state(2^-5)| = {diff:.3e}")
    assert diff <= 1e-3


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_rest_fp32_storage_conserves_mass(prec):
    """Periodic grid, no source, tensor and velocity fields: the total stored mass is
    conserved to FP32 rounding when the rest population takes up the node's rounding
    residuals (with and without stochastic rounding), unlike plain 16-bit storage."""
    banner(f"mass conservation of the FP32-rest storage, {prec}")
    rng = np.random.default_rng(44)
    n = 48
    n3 = (n, n, n)
    d6 = I.log_tensor_field(n, seed=9)
    u = 0.04 * np.stack([I.smooth_field(n3, rng) for _ in range(3)])
    phi0 = 1.0 + 0.3 * I.smooth_field(n3, rng)
    prob = I.Problem("mass", n, n, n, d6, u, phi0, steps=200, phi_ref=1.0, tensor_is_log=True)
    drift = {}
    for mode, kw in (("plain", {}), ("rest32", dict(rest_fp32=True)),
                     ("rest32+sr", dict(rest_fp32=True, stochastic_rounding=True))):
        lat = gpu_lattice(prob, prec, **kw)
        m0 = lat.reduce()[0]
        lat.step(prob.steps)
        drift[mode] = abs(lat.reduce()[0] - m0) / m0
    print(f"{prec}: relative mass drift over 200 steps {drift}")
    assert drift["rest32"] <= 1e-6
    assert drift["rest32+sr"] <= 1e-6


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_rest_fp32_stochastic_rounding_accuracy(prec):
    """Porous conduction at 48^3 over 1500 steps (Dirichlet walls, 1e4:1 solid tensor):
    error of phi against the GPU FP64 run, relative to max |phi64 - phi_ref|. Plain BF16
    round-to-nearest storage drifts by several per cent; with the FP32 rest population and
    stochastic rounding the error must stay below 1e-2 and improve at least five-fold."""
    banner(f"16-bit storage accuracy, porous 48^3 x 1500, {prec}")
    prob = I.porous_spheres(n=48, steps=1500)

    def phi(prec_, **kw):
        lat = gpu_lattice(prob, prec_, **kw)
        lat.step(prob.steps)
        return lat.moments()[0].cpu().numpy()

    ref = phi("f64")
    scale = np.abs(ref - prob.phi_ref).max()
    err_plain = np.abs(phi(prec) - ref).max() / scale
    err_good = np.abs(phi(prec, rest_fp32=True, stochastic_rounding=True) - ref).max() / scale
    print(f"{prec}: plain {err_plain:.3e}, FP32 rest + stochastic rounding {err_good:.3e}")
    assert err_good <= 1e-2
    if prec == "bf16":
        assert err_good <= err_plain / 5


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("nx,width", [(64, 1), (128, 1), (192, 1), (320, 1), (128, 2), (256, 2)])
def test_f64_vector_rows_vs_oracle(nx, bc, width):
    """The row-vector kernel (forced: the fields below would otherwise select the
    one-node-per-thread kernel) against the FP64 oracle."""
    banner(f"f64 vector rows nx={nx} {bc} V={width} vs oracle")
    rng = np.random.default_rng(42)
    n3 = (6, 5, nx)
    d6, u = _random_fields(n3, rng)
    phi0 = 1.0 + 0.3 * rng.uniform(-1, 1, n3)
    prob = I.Problem("vrow", nx, 5, 6, d6, u, phi0, steps=15, r=1e-4, phi_ref=1.0, bc_x=bc,
                     phi_lo=1.25, phi_hi=0.9)
    lat = gpu_lattice(prob, "f64", vector_width=width)
    lat.step(prob.steps)
    err = rel_err(gpu_pops(lat), _oracle_run(prob, prob.steps))
    print(f"f64 vector rows nx={nx} {bc}: rel err {err:.3e}")
    assert err <= F64_TOL


# ------------------------------------------------------------------------------------------
# Full-size workloads in the launch configuration the benchmark times: sampled outputs
# ------------------------------------------------------------------------------------------
from gpuhelp import sampled_next_step  # noqa: E402


def _sampled_check(prob, prec, warm, nsamp, seed=51, wall_frac=0.0, **kw):
    import torch
    lat = gpu_lattice(prob, prec, **kw)
    lat.step(warm)
    f_now = lat.populations()
    lat.step(1)
    f_next = lat.populations()
    rng = np.random.default_rng(seed)
    xs = rng.integers(0, prob.nx, nsamp)
    nw = int(wall_frac * nsamp)
    xs[:nw] = rng.choice([0, prob.nx - 1], nw)
    samples = (rng.integers(0, prob.nz, nsamp), rng.integers(0, prob.ny, nsamp), xs)
    want, nodes = sampled_next_step(lat, prob, samples, f_now)
    from gpuhelp import perm_lib_to_oracle
    got = f_next.reshape(lat.q, -1)[:, torch.as_tensor(nodes, device=f_next.device)].cpu().numpy()
    got = got[perm_lib_to_oracle(lat.q)].T
    scale = np.abs(want).max()
    err = np.abs(got - want).max() / scale
    del lat, f_now, f_next
    torch.cuda.empty_cache()
    return err


@pytest.mark.parametrize("prec,tol", [("f64", 1e-14), ("f32", 2e-7), ("bf16", 1e-4), ("fp16", 2e-5),
                                      ("bf16r", 3e-4), ("fp16r", 4e-5)])
def test_full_size_decay_sampled_one_step(prec, tol):
    """256^3 rotated decay (the benchmark workload): one GPU step from the GPU's own state
    after 20 steps, at 4000 sampled nodes, against the oracle's step of the same state.
    The tolerance is the rounding of one step in that form (relative to max |g| = W_0):
    FP32 arithmetic ~1e-8; BF16 / FP16 storage rounding of the deviations, half an ulp
    (2^-8 resp. 2^-11 relative) of |d| <= 0.01 W_0, i.e. 4e-5 resp. 5e-6, doubled. With the
    FP32 rest population and stochastic rounding ("r"), each moving population is off by
    up to one ulp and the rest population carries the 18 residuals of its node:
    18 ulp of |d| <= 0.01 W_1, i.e. 2e-4 (BF16) resp. 3e-5 (FP16) of max |g|."""
    banner(f"full-size sampled step {prec} 256^3")
    base = prec.rstrip("r")
    kw = dict(rest_fp32=True, stochastic_rounding=True) if prec.endswith("r") else {}
    prob = I.fourier_decay(n=256, steps=20, precision=base)
    err = _sampled_check(prob, base, 20, 4000, **kw)
    print(f"{prec}: sampled one-step error {err:.3e} (tol {tol:g})")
    assert err <= tol


def test_full_size_porous_sampled_one_step():
    """384^3 porous spheres with Dirichlet planes (FP32): sampled one-step check, with the
    samples concentrated on the wall-adjacent planes as well."""
    banner("full-size sampled step porous 384^3 f32")
    prob = I.porous_spheres(n=384, steps=5)
    err = _sampled_check(prob, "f32", 5, 4000, wall_frac=0.5)
    print(f"porous 384^3 f32: sampled one-step error {err:.3e}")
    assert err <= 2e-7


@pytest.fixture(scope="module")
def varfield512():
    # generated on the GPU (the fields at the sampled nodes are gathered from there)
    return I.variable_tensor_source(n=512, steps=5, device="cuda:0")


@pytest.mark.parametrize("prec,tol", [("f32", 1e-6), ("bf16", 1e-4), ("fp16", 2e-5)])
def test_full_size_varfield_sampled_one_step(varfield512, prec, tol):
    """512^3 source-driven transport with per-node tensor, velocity and source fields (the
    benchmark's field workload): sampled one-step check after 5 steps. FP32: each stored
    population is a sum of about ten rounded FP32 terms (10 x 2^-24 ~ 6e-7 of max |g|),
    plus the rounding of near-equilibrium ghost parts carried into lambda, which the ghost
    floor tau = 1e-4 keeps below a few 1e-7; the 16-bit forms as in the decay case."""
    banner(f"full-size sampled step varfield 512^3 {prec}")
    err = _sampled_check(varfield512, prec, 5, 4000)
    print(f"varfield 512^3 {prec}: sampled one-step error {err:.3e} (tol {tol:g})")
    assert err <= tol


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("bf16r", 3e-4), ("fp16r", 4e-5)])
def test_full_size_varfield_sampled_one_step_more_forms(varfield512, prec, tol):
    """The field workload's other benchmark forms at 512^3 (sampled one step after 5): FP64,
    and the 16-bit forms with the FP32 rest population and stochastic rounding (tolerances
    as in the decay case: each moving population off by up to one ulp, the rest population
    carrying its node's 18 residuals)."""
    banner(f"full-size sampled step varfield 512^3 {prec}")
    base = prec.rstrip("r")
    kw = dict(rest_fp32=True, stochastic_rounding=True) if prec.endswith("r") else {}
    err = _sampled_check(varfield512, base, 5, 4000, **kw)
    print(f"varfield 512^3 {prec}: sampled one-step error {err:.3e} (tol {tol:g})")
    assert err <= tol


@pytest.mark.parametrize("prec,tol", [("bf16", 1e-3), ("bf16r", 3e-3)])
def test_full_size_porous_phases_sampled_one_step_16bit(prec, tol):
    """The porous workload's 16-bit benchmark forms at 384^3 with the material table. The
    deviations reach |phi - phi_ref| = 0.5 of phi: half a BF16 ulp of W_i / 2 is 5e-4 of
    max |g| = 2 W_0; with the FP32 rest population the rest value also carries up to one
    ulp of each of the 18 moving deviations, about 2e-3 of max |g|."""
    banner(f"full-size sampled step porous 384^3 phases {prec}")
    base = prec.rstrip("r")
    kw = dict(rest_fp32=True, stochastic_rounding=True) if prec.endswith("r") else {}
    prob = I.porous_spheres(n=384, steps=5)
    err = _sampled_check(prob, base, 5, 4000, wall_frac=0.5, phases=True, **kw)
    print(f"porous 384^3 phases {prec}: sampled one-step error {err:.3e} (tol {tol:g})")
    assert err <= tol


@pytest.mark.parametrize("prec,kw", [("f64", {}), ("f32", {}), ("bf16", dict(rest_fp32=True)),
                                     ("fp16", {})])
def test_min_population_matches_readout(prec, kw):
    """elbm_min_population equals the minimum of the population readout (bitwise: the same
    FP64 expression per value), on a ragged grid with tensor, velocity and source fields and
    a pending source half-step; on a zero background, where the positivity fallback is
    active, the FP64 minimum stays at or above eps."""
    banner(f"min population {prec} {sorted(kw)}")
    nx, ny, nz = 37, 29, 23
    rng = np.random.default_rng(23)
    d6, u = _random_fields((nz, ny, nx), rng)
    phi0 = 1.0 + 0.3 * rng.uniform(-1, 1, (nz, ny, nx))
    r = 1e-3 * rng.uniform(-1, 1, (nz, ny, nx))
    prob = I.Problem("ragged", nx, ny, nz, d6, u, phi0, steps=12, r=r, phi_ref=1.0)
    lat = gpu_lattice(prob, prec, **kw)
    lat.step(prob.steps)
    assert lat.min_population() == float(lat.populations().min())
    if prec == "f64":
        plume = I.gaussian_plume(n=16, steps=20, sigma0=2.0)
        lat = gpu_lattice(plume, "f64")
        lat.step(plume.steps)
        assert lat.counters()["fallback_nodes"] > 0
        m = lat.min_population()
        assert m == float(lat.populations().min())
        assert m >= plume.eps - 1e-15


@pytest.mark.parametrize("nx", [64, 37])
def test_step_counters_guard_and_fallback(nx):
    """Step counters, aggregated per wavefront: phi = 0 everywhere takes lambda = 1 by the
    guard at every node update; a positive field never does; on a zero-background plume the
    row-vector and one-node-per-thread kernels (bitwise-equal updates) count the same
    fallback nodes (the latter's counts are checked against the oracle elsewhere)."""
    from paper_2605_01774_amd import lattice
    banner(f"step counters nx={nx}")
    lat = lattice.Lattice(nx, 6, 5, precision="f64", device="cuda:0")
    lat.set_diffusion([1e-2, 0, 0, 1e-2, 0, 1e-2])
    lat.init_equilibrium(np.zeros((5, 6, nx)))
    lat.step(3)
    c = lat.counters()
    assert c["guard_nodes"] == 3 * lat.n and c["fallback_nodes"] == 0 and c["nonfinite"] == 0
    lat.reset_counters()
    lat.init_equilibrium(1.0 + 0.1 * np.random.default_rng(3).uniform(-1, 1, (5, 6, nx)))
    lat.step(3)
    assert lat.counters()["guard_nodes"] == 0
    if nx != 64:
        return
    plume = I.gaussian_plume(n=64, steps=10, sigma0=2.0)
    counts = []
    for scalar in (False, True):
        lp = gpu_lattice(plume, "f64", scalar_kernel=scalar)
        lp.step(plume.steps)
        counts.append(lp.counters())
    assert counts[0]["fallback_nodes"] > 0
    assert counts[0] == counts[1]
