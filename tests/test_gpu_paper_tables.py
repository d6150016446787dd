"""The paper's own printed results reproduced by full-size GPU runs of the D3Q27 build
(FP64), as the paper's lattice and, in the absence of a stated precision, the reference
arithmetic.

- Sec. 3.3 manufactured-source benchmark, 128^3 to t = 3 (49152 steps), four anisotropy
  ratios: the global relative error equals the printed GRE to its last printed digit, the
  L2 errors lie in the printed range and the L-infinity errors below the printed bound
  (tests/golden/manufactured_e3.txt).
- Sec. 3.1 advected Gaussian, 256^3 to tau = 6.25 (40000 steps), first anisotropy set: the
  tensor recovered from the second moments about the exact centroid equals the printed
  "Recovered" row to 1e-6 in D (0.001 in the table's units of 1e-3); the paper's run
  starts from an initial state it does not state, which moves the recovered tensor by
  ~1e-7 per 1e-3 of covariance offset, so this is agreement, not identity
  (tests/golden/gaussian3d_recovered.txt).
- Sec. 4.2.1 rotated anisotropic solid, 128^3 between two fixed-temperature planes x = 0
  and x = L, periodic in y and z, four principal ratios and rotations: the conductivity
  entries K_xx, K_xy, K_xz recovered from the LB heat flux q = (I - S/2) j under the imposed
  x-gradient equal the printed exact entries to their last printed digit (the paper's own
  run recovers them to 1.2e-4..1.5e-4; here the linear profile with its Chapman-Enskog flux
  is an exact steady state of the scheme with halfway anti-bounce-back walls, so the
  recovery is exact to roundoff) (tests/golden/thermal_conductivity.txt).
"""
import numpy as np
import pytest
import torch

from paper_2605_01774_amd import inputs as I
from gpuhelp import banner, gpu_lattice
from conftest import golden

pytestmark = pytest.mark.gpu
Q = 27


@pytest.mark.parametrize("row", golden("manufactured_e3.txt"), ids=lambda r: f"d2={r[1]:g}")
def test_manufactured_source_gre_128(row):
    banner(f"Sec. 3.3 manufactured source 128^3, d = {row[:3]}")
    prob = I.manufactured_source(n=128, d=tuple(row[:3]))
    lat = gpu_lattice(prob, "f64", q=Q)
    for m in range(prob.steps):
        lat.set_source_scale(prob.meta["scale"](m))
        lat.step(1)
    phi = lat.moments()[0].cpu().numpy() - prob.meta["shift"]
    ex = prob.meta["exact"](prob.steps * prob.meta["dt"])
    err = phi - ex
    gre = float(np.sqrt((err ** 2).sum() / (ex ** 2).sum()))
    l2 = float(np.sqrt((err ** 2).mean()))
    linf = float(np.abs(err).max())
    print(f"GRE {gre:.6e} (printed {row[3]:.3e}), L2 {l2:.3e}, Linf {linf:.3e}")
    assert abs(gre - row[3]) <= 0.5e-7          # half a unit of the last printed digit
    assert 1.25e-4 <= l2 <= 4.095e-4            # printed: between 1.26e-4 and 4.09e-4
    assert linf < 1.31e-3                       # printed: below 1.31e-3


def test_advected_gaussian_recovered_tensor_256():
    row = golden("gaussian3d_recovered.txt")[0]
    banner(f"Sec. 3.1 advected Gaussian 256^3 x 40000, d = {row[:3]}")
    n, steps, sig0, u = 256, 40000, 8.0, (0.04, 0.02, 0.01)
    prob = I.gaussian_plume(n=n, steps=steps, sigma0=sig0, d=tuple(row[:3]), angles=(120, 90, 135), u=u)
    lat = gpu_lattice(prob, "f64", q=Q)
    m0 = lat.reduce()[0]
    lat.step(steps)
    m1 = lat.reduce()[0]
    phi = lat.moments()[0]
    mu = prob.meta["mu0"] + np.array(u) * steps
    x1 = torch.arange(n, dtype=torch.float64, device=phi.device)
    # offsets from the exact centroid, minimal periodic image
    dx = [torch.remainder(x1 - mu[a] + n / 2, n) - n / 2 for a in range(3)]
    X, Y, Z = dx[0][None, None, :], dx[1][None, :, None], dx[2][:, None, None]
    M = float(phi.sum())
    first = np.array([float((phi * X).sum()), float((phi * Y).sum()), float((phi * Z).sum())]) / M
    prods = {(0, 0): X * X, (0, 1): X * Y, (0, 2): X * Z, (1, 1): Y * Y, (1, 2): Y * Z, (2, 2): Z * Z}
    S = np.zeros((3, 3))
    for (a, b), f in prods.items():
        S[a, b] = S[b, a] = float((phi * f).sum()) / M
    S -= np.outer(first, first)
    D = (S - sig0 ** 2 * np.eye(3)) / (2 * steps)
    got = np.array([D[0, 0], D[0, 1], D[0, 2], D[1, 1], D[1, 2], D[2, 2]]) * 1e3
    want = np.array(row[3:])
    print(f"recovered x1e3 {np.round(got, 5)}, printed {want}, mass drift {(m1 - m0) / m0:.2e}, "
          f"centroid offset {np.linalg.norm(first):.2e}")
    assert np.abs(got - want).max() <= 1e-3
    assert abs((m1 - m0) / m0) <= 1e-11


@pytest.mark.parametrize("row", golden("thermal_conductivity.txt"), ids=lambda r: f"k2={r[1]:g}")
def test_rotated_conductivity_128(row):
    banner(f"Sec. 4.2.1 rotated conductivity 128^3, k = {row[:3]}, angles {row[3:6]}")
    n = 128
    scale = 1e-3                                    # lattice diffusivity per W/(m K)
    K = I.rotated_tensor(tuple(row[:3]), I.euler_zyz(*row[3:6]))
    d6 = K * scale
    phi_lo, phi_hi = 2.0, 1.0                       # walls half a cell outside x = 0, n - 1
    G = (phi_hi - phi_lo) / n                       # d phi / dx
    xs = np.arange(n, dtype=np.float64)
    phi0 = np.broadcast_to((phi_lo + G * (xs + 0.5))[None, None, :], (n, n, n)).copy()
    D = I.mat3(d6)
    # Chapman-Enskog flux of the linear profile: j = -(1/3) S^-1 grad phi, S^-1 = I/2 + 3 D
    j = -(0.5 * np.eye(3) + 3.0 * D) @ np.array([G, 0.0, 0.0]) / 3.0
    j0 = np.broadcast_to(j[:, None, None, None], (3, n, n, n)).copy()
    prob = I.Problem("conductivity", n, n, n, d6, np.zeros(3), phi0, steps=200, bc_x="dirichlet",
                     phi_lo=phi_lo, phi_hi=phi_hi, phi_ref=0.5 * (phi_lo + phi_hi))
    from paper_2605_01774_amd import lattice
    lat = lattice.Lattice(n, n, n, precision="f64", bc_x="dirichlet", phi_ref=prob.phi_ref,
                          device="cuda:0", q=Q)
    lat.set_diffusion(d6)
    lat.set_dirichlet(phi_lo, phi_hi)
    lat.init_equilibrium(phi0, j0)
    f0 = lat.populations()
    lat.step(prob.steps)
    drift = float((lat.populations() - f0).abs().max() / f0.abs().max())
    phi, q = lat.moments()
    interior = slice(n // 4, 3 * n // 4)
    Krec = (-q[:, :, :, interior].mean(dim=(1, 2, 3)) / G / scale).cpu().numpy()
    qrec = Krec / 128.0                             # heat flux for the table's G_x = 1/128
    print(f"K recovered {Krec}, printed exact {row[9:12]}, steady-state drift {drift:.2e}")
    assert drift < 1e-13
    assert np.allclose(Krec, [K[0], K[1], K[2]], rtol=1e-10, atol=0)
    assert np.all(np.abs(Krec - np.array(row[9:12])) <= 0.5e-3)   # printed to 3 decimals
    assert np.all(np.abs(qrec - np.array(row[6:9])) <= 0.5e-5)    # printed to 5 decimals
