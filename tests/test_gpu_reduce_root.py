"""GPU against the FP64 oracle: the global FP64 reductions (Sec. 2.6 mass, the flux sums
behind the effective conductivity of Sec. 4.2.2), the exact entropic root of Sec. 2.5 at
flagged nodes under FP32 arithmetic (every storage form), and the exact root at every node
as a full FP64 mode."""
import math

import numpy as np
import pytest

import oracle
from paper_2605_01774_amd import inputs as I
from gpuhelp import banner, gpu_lattice, gpu_pops, rel_err, to_lib_order

pytestmark = pytest.mark.gpu

FORMS = {"f64": ("f64", {}), "f32": ("f32", {}), "bf16": ("bf16", {}), "fp16": ("fp16", {}),
         "bf16r": ("bf16", dict(rest_fp32=True, stochastic_rounding=True)),
         "fp16r": ("fp16", dict(rest_fp32=True, stochastic_rounding=True))}


def _random_fields(n3, rng, u_amp=0.05, ratio=1e3):
    nz, ny, nx = n3
    ds = []
    for _ in range(nx * ny * nz):
        d = 1e-2 * 10.0 ** (-np.log10(ratio) * rng.uniform(0, 1, 3))
        ds.append(I.rotated_tensor(tuple(d), I.random_rotation(rng)))
    return np.stack(ds, axis=1).reshape((6,) + n3), rng.uniform(-u_amp, u_amp, size=(3,) + n3)


def _fsums(prob, f):
    """Exact sums (math.fsum) of phi and of the three components of q = (I - S/2) j over
    the oracle's moments of the populations f (oracle order), and sum |q| per component."""
    phi, _, q = oracle.moments(prob, f)
    return (math.fsum(phi.ravel()), [math.fsum(q[a].ravel()) for a in range(3)],
            [float(np.abs(q[a]).sum()) for a in range(3)])


def _reduce_problem(bc):
    nx, ny, nz = 37, 29, 23
    n3 = (nz, ny, nx)
    rng = np.random.default_rng(61)
    d6, u = _random_fields(n3, rng)
    phi0 = 1.0 + 0.3 * rng.uniform(-1, 1, n3)
    r = 1e-3 * rng.uniform(-1, 1, n3)
    return I.Problem("reduce", nx, ny, nz, d6, u, phi0, steps=17, r=r, phi_ref=1.0, bc_x=bc,
                     phi_lo=1.4, phi_hi=0.7)


# Tolerances of the sums along the oracle's FP64 trajectory, relative to |sum phi| and to
# sum |q|, per boundary kind. FP64: rounding of the two runs. FP32 arithmetic: each stored
# value carries one FP32 rounding (2^-24 of |d| <= 0.3 W), ~1e-9 of sum phi over the run.
# Plain 16-bit storage rounds every deviation to 2^-9 (BF16) or 2^-12 (FP16, stored over
# 2^-8) of itself; the same slowly varying values round the same way step after step, so
# the mass errors add up between a random walk (~1e-5 of sum phi for BF16) and the bound
# 17 steps x 2^-9 x mean |d| / phi ~ 1e-2; measured 1.1e-4 (BF16), hence 5e-4 and 1e-4. With
# the FP32 rest population the stored mass is exact to FP32 rounding on a periodic grid
# (1e-7); with Dirichlet planes the mass the walls exchange follows the stored state near
# them, which carries the 16-bit form's error (measured 2.8e-7 BF16, 1.0e-7 FP16), hence
# 2e-6. The flux sums follow the stored state: that form's one-step tolerance times a few.
SUM_TOL = {"f64": (1e-13, 1e-11), "f32": (1e-7, 1e-5), "bf16": (5e-4, 3e-2), "fp16": (1e-4, 5e-3),
           "bf16r": (1e-7, 3e-2), "fp16r": (1e-7, 5e-3)}
SUM_TOL_WALLS = dict(SUM_TOL, bf16r=(2e-6, 3e-2), fp16r=(2e-6, 5e-3))


@pytest.mark.parametrize("bc", ["periodic", "dirichlet"])
@pytest.mark.parametrize("form", sorted(FORMS))
def test_reduce_matches_oracle_sums(form, bc):
    """elbm_reduce (sum phi, sum q in FP64) on a ragged grid with tensor, velocity and source
    fields, a pending source half-step and, for "dirichlet", anti-bounce-back walls:
    (1) against math.fsum of the oracle's moments of the GPU's own populations (the
        reduction alone: the state is the same, so 1e-14 of sum phi; q is formed in the
        form's arithmetic, 1e-12 (FP64) or 1e-6 (FP32) of sum |q|);
    (2) against the oracle's own FP64 trajectory (SUM_TOL). Sec. 2.6: the scalar is
        conserved up to the source and wall fluxes, which both sides add alike."""
    banner(f"reduce vs oracle sums {form} {bc}")
    prob = _reduce_problem(bc)
    base, kw = FORMS[form]
    lat = gpu_lattice(prob, base, **kw)
    lat.step(prob.steps)
    got = lat.reduce()
    # (1) the reduction of the GPU state itself
    mine_phi, mine_q, mine_abs = _fsums(prob, gpu_pops(lat))
    e1_phi = abs(got[0] - mine_phi) / abs(mine_phi)
    q_tol1 = 1e-12 if form == "f64" else 1e-6
    e1_q = max(abs(got[1 + a] - mine_q[a]) / mine_abs[a] for a in range(3))
    # (2) the oracle's trajectory with the lattice's ghost floor
    f_or = oracle.run(prob, oracle.init_equilibrium(prob), prob.steps, tau=float(lat.cfg.ghost_floor))
    or_phi, or_q, or_abs = _fsums(prob, f_or)
    e2_phi = abs(got[0] - or_phi) / abs(or_phi)
    e2_q = max(abs(got[1 + a] - or_q[a]) / or_abs[a] for a in range(3))
    tol_phi, tol_q = (SUM_TOL_WALLS if bc == "dirichlet" else SUM_TOL)[form]
    print(f"{form} {bc}: own state phi {e1_phi:.2e} q {e1_q:.2e}; oracle trajectory phi "
          f"{e2_phi:.2e} (tol {tol_phi:g}) q {e2_q:.2e} (tol {tol_q:g})")
    assert e1_phi <= 1e-14 and e1_q <= q_tol1
    assert e2_phi <= tol_phi and e2_q <= tol_q
    assert all(abs(v) > 0 for v in or_q)  # the flux sums are not trivially zero


def _nonequilibrium(n3=(6, 7, 8), seed=23):
    rng = np.random.default_rng(seed)
    nz, ny, nx = n3
    d6, u = _random_fields(n3, rng, u_amp=0.08, ratio=1e4)
    prob = I.Problem("fb", nx, ny, nz, d6, u, np.ones(n3), steps=3, eps=1e-4)
    f0 = oracle.init_equilibrium(prob) * (1.0 + 0.9 * rng.uniform(-1, 1, (19,) + n3))
    return prob, f0


# Tolerances of the reduced-precision root test, relative to max |g|, for one step from the
# same stored state: the start deviates from equilibrium by up to 90 %, so a stored
# deviation |d| is up to ~0.9 of max |g|, and one store rounds it to 2^-9 (BF16) or 2^-11
# (FP16) of itself, i.e. 1.8e-3 resp. 4.4e-4 of max |g|; FP32 adds the rounding of some tens
# of operations (~1e-6).
ROOT_TOL = {"f32": 2e-6, "bf16": 2.5e-3, "fp16": 6e-4}


@pytest.mark.parametrize("prec", sorted(ROOT_TOL))
def test_exact_root_under_fp32_arithmetic(prec):
    """The FP64 exact entropic root at flagged nodes inside FP32 arithmetic (root_rho = 0.3;
    the precision design where FP64 is kept only for the root and the reductions), on the
    strongly non-equilibrium start where the fallback and the root both fire, for three
    steps. Each step, the oracle steps the GPU's own stored state (so the stores' rounding
    does not move the flag decisions of later steps) with the lattice's ghost floor; that
    step's flagged and fallback counts must equal the oracle's, and its populations must lie
    within ROOT_TOL of the oracle's step."""
    banner(f"exact root under FP32 arithmetic, {prec}")
    prob, f0 = _nonequilibrium()
    lat = gpu_lattice(prob, prec, root_rho=0.3)
    lat.set_populations(to_lib_order(f0))
    tot_fb = tot_fl = 0
    for s in range(prob.steps):
        start = gpu_pops(lat)  # the state as stored in this form
        lat.reset_counters()
        lat.step(1)
        f_ref, _, _, (nfb, nfl) = oracle.run(prob, start, 1, root_rho=0.3, want_last=True,
                                             tau=float(lat.cfg.ghost_floor))
        err = rel_err(gpu_pops(lat), f_ref)
        cnt = lat.counters()
        print(f"{prec} step {s + 1}: rel err {err:.3e} (tol {ROOT_TOL[prec]:g}), fallback "
              f"{cnt['fallback_nodes']} vs {nfb}, flagged {cnt['flagged_nodes']} vs {nfl}")
        assert cnt["flagged_nodes"] == nfl
        assert cnt["fallback_nodes"] == nfb
        assert err <= ROOT_TOL[prec]
        tot_fb += nfb
        tot_fl += nfl
    assert tot_fl > 0 and tot_fb > 0


@pytest.mark.parametrize("q", [19, 27])
def test_exact_root_everywhere_fp64(q):
    """The exact root as a full FP64 mode (root_rho = 1e300 flags every node with phi > 0)
    on a 16^3 grid with a velocity field, against the oracle at 1e-12. The start deviates
    from equilibrium by 20 % at random, so every ghost part is far above rounding level and
    the root is well conditioned (at rounding-level ghosts the root is bounded only by
    positivity)."""
    banner(f"exact root everywhere, D3Q{q}")
    rng = np.random.default_rng(71)
    n = 16
    n3 = (n, n, n)
    u = 0.04 * np.stack([I.smooth_field(n3, rng) for _ in range(3)])
    prob = I.Problem("root_all", n, n, n, I.log_tensor_field(n, seed=72), u,
                     1.0 + 0.3 * I.smooth_field(n3, rng), steps=6, tensor_is_log=True, phi_ref=1.0)
    f0 = oracle.init_equilibrium(prob, q=q) * (1.0 + 0.2 * rng.uniform(-1, 1, (q,) + n3))
    lat = gpu_lattice(prob, "f64", root_rho=1e300, q=q)
    lat.set_populations(to_lib_order(f0))
    lat.reset_counters()
    lat.step(prob.steps)
    f_ref, _, _, (nfb, nfl) = oracle.run(prob, f0, prob.steps, root_rho=1e300, q=q, want_last=True)
    err = rel_err(gpu_pops(lat), f_ref)
    cnt = lat.counters()
    print(f"D3Q{q}: rel err {err:.3e}, flagged {cnt['flagged_nodes']} vs {nfl} (of "
          f"{prob.steps * prob.n}), fallback {cnt['fallback_nodes']} vs {nfb}")
    assert err <= 1e-12
    assert cnt["flagged_nodes"] == nfl == prob.steps * prob.n
    assert cnt["fallback_nodes"] == nfb


def test_exact_root_effect_against_closed_form():
    """How far the exact root at every node moves results from the closed-form lambda of
    Sec. 2.5, in FP64 on the GPU (the paper reports results with the closed form):
    - rotated decay, u = 0, 64^3 x 500: the closed form's numerator vanishes identically
      (lambda = 1), the root differs from 1 only at second order in the ghost part, so the
      two runs stay within 1e-4 of the mode amplitude (bound: the ghost part of a long-wave
      mode is O(k^2) of the amplitude, and the root moves lambda by O(ghost));
    - advected Gaussian on a zero background (u != 0), 32^3 x 100: far from the plume the
      ghost parts are at rounding level. The closed form with its ghost floor conserves the
      mass there to rounding; the root, bounded only by positivity, multiplies the rounding
      residual sum_i Dh_i by an arbitrarily large lambda, which moves phi and the mass by a
      sizeable fraction (the oracle does the same with its own rounding). The changes are
      printed; the root run must stay finite and the closed-form run conserve mass to 1e-12.
      This is why the exact root is taken only at flagged nodes by default."""
    banner("exact root everywhere against the closed form")
    prob = I.fourier_decay(n=64, steps=500, mode=(1, 1, 1), precision="f64")
    phi = {}
    for name, rho in (("closed", -1.0), ("root", 1e300)):
        lat = gpu_lattice(prob, "f64", root_rho=rho)
        lat.step(prob.steps)
        phi[name] = lat.moments()[0].cpu().numpy()
        del lat
    dec = float(np.abs(phi["root"] - phi["closed"]).max()) / prob.meta["a0"]
    print(f"decay 64^3 x 500, u = 0: max |phi_root - phi_closed| / a0 = {dec:.3e}")
    assert dec <= 1e-4
    prob = I.gaussian_plume(n=32, steps=100, sigma0=2.5)
    mass = {}
    for name, rho in (("closed", -1.0), ("root", 1e300)):
        lat = gpu_lattice(prob, "f64", root_rho=rho)
        m_init = math.fsum(lat.moments()[0].cpu().numpy().ravel())
        lat.step(prob.steps)
        phi[name] = lat.moments()[0].cpu().numpy()
        mass[name] = math.fsum(phi[name].ravel())
        del lat
    chg = float(np.abs(phi["root"] - phi["closed"]).max()) / float(np.abs(phi["closed"]).max())
    print(f"zero-background plume 32^3 x 100, u != 0: max |phi_root - phi_closed| / max phi = {chg:.3e}; "
          f"mass change over the run: closed form {mass['closed'] / m_init - 1:+.2e}, "
          f"root everywhere {mass['root'] / m_init - 1:+.2e}")
    assert np.isfinite(phi["root"]).all()
    assert abs(mass["closed"] - m_init) <= 1e-12 * abs(m_init)
