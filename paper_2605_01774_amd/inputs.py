"""Seeded synthetic inputs shaped like the paper's three-dimensional benchmarks.

This module only builds inputs (grids, tensors, velocities, sources, initial scalar fields).
It holds none of the scheme's arithmetic: no equilibrium, no relaxation matrix, no update.
Both the GPU library and the FP64 CPU oracle consume the arrays it returns.

Conventions: a grid point is (x, y, z) with x fastest in memory; scalar fields are numpy
arrays of shape (nz, ny, nx); vector fields (3, nz, ny, nx); symmetric tensors are 6-vectors
(xx, xy, xz, yy, yz, zz), either shape (6,) for a uniform tensor or (6, nz, ny, nx).

Rotations follow the ZYZ Euler convention of Sec. 3.1: R = Rz(a) Ry(b) Rz(g) with the
standard active rotation matrices, and D = R diag(d1, d2, d3) R^T.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Union

import numpy as np

ArrayOrScalar = Union[float, np.ndarray]


# --------------------------------------------------------------------------------------------
# Rotations and tensors
# --------------------------------------------------------------------------------------------
def rot_z(a: float) -> np.ndarray:
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def rot_y(b: float) -> np.ndarray:
    c, s = np.cos(b), np.sin(b)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def euler_zyz(alpha_deg: float, beta_deg: float, gamma_deg: float) -> np.ndarray:
    """R = Rz(alpha) Ry(beta) Rz(gamma), angles in degrees (Sec. 3.1)."""
    a, b, g = np.deg2rad([alpha_deg, beta_deg, gamma_deg])
    return rot_z(a) @ rot_y(b) @ rot_z(g)


def sym6(m: np.ndarray) -> np.ndarray:
    """3x3 symmetric matrix -> (xx, xy, xz, yy, yz, zz)."""
    return np.array([m[0, 0], m[0, 1], m[0, 2], m[1, 1], m[1, 2], m[2, 2]], dtype=np.float64)


def mat3(t6: np.ndarray) -> np.ndarray:
    """(xx, xy, xz, yy, yz, zz) -> 3x3 symmetric matrix."""
    t = np.asarray(t6, dtype=np.float64)
    return np.array([[t[0], t[1], t[2]], [t[1], t[3], t[4]], [t[2], t[4], t[5]]])


def rotated_tensor(d: tuple, rot: np.ndarray) -> np.ndarray:
    """D = R diag(d) R^T as a 6-vector."""
    return sym6(rot @ np.diag(np.asarray(d, dtype=np.float64)) @ rot.T)


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform rotation on SO(3) from a normalised 4-D Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


# --------------------------------------------------------------------------------------------
# Problem description shared by both implementations
# --------------------------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    """Everything that defines one run: grid, coefficients, boundary, initial scalar."""
    name: str
    nx: int
    ny: int
    nz: int
    d6: np.ndarray                      # (6,) uniform or (6, nz, ny, nx)
    u: np.ndarray                       # (3,) uniform or (3, nz, ny, nx)
    phi0: np.ndarray                    # (nz, ny, nx)
    steps: int
    r: Optional[ArrayOrScalar] = None   # None, a float, or (nz, ny, nx)
    bc_x: str = "periodic"              # "periodic" or "dirichlet"
    phi_lo: float = 0.0                 # Dirichlet value on the x = 0 side
    phi_hi: float = 0.0                 # Dirichlet value on the x = nx - 1 side
    tensor_is_log: bool = False         # d6 holds L with D = expm(L)
    eps: float = 0.0                    # positivity threshold of the fallback
    phi_ref: float = 0.0                # background used for shifted (deviation) storage
    precision: str = "f64"              # precision form named by the workload
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def d_uniform(self) -> bool:
        return np.ndim(self.d6) == 1

    @property
    def u_uniform(self) -> bool:
        return np.ndim(self.u) == 1


def _grid(nx: int, ny: int, nz: int):
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    y = np.arange(ny, dtype=np.float64)[None, :, None]
    x = np.arange(nx, dtype=np.float64)[None, None, :]
    return x, y, z


def _torch_grid(nx: int, ny: int, nz: int, device):
    import torch
    z = torch.arange(nz, dtype=torch.float64, device=device)[:, None, None]
    y = torch.arange(ny, dtype=torch.float64, device=device)[None, :, None]
    x = torch.arange(nx, dtype=torch.float64, device=device)[None, None, :]
    return x, y, z


def _smooth_field_t(shape, rng: np.random.Generator, modes: int, kmax: int, amp: float, device):
    """smooth_field evaluated with torch in FP64 on `device` (the random draws, and so the
    field, are the same as smooth_field's up to rounding)."""
    import torch
    nz, ny, nx = shape
    x, y, z = _torch_grid(nx, ny, nz, device)
    # a sin(pz + q) with q = 2 pi (kx x / nx + ky y / ny) + th is expanded as
    # a sin(pz) cos(q) + a cos(pz) sin(q): the sum over modes is then one product of a
    # (nz, 2 modes) matrix with a (2 modes, ny nx) matrix, with no transcendental taken over
    # the full grid.
    zc = torch.empty((nz, 2 * modes), dtype=torch.float64, device=device)
    xy = torch.empty((2 * modes, ny * nx), dtype=torch.float64, device=device)
    for m in range(modes):
        k = rng.integers(-kmax, kmax + 1, size=3)
        while not k.any():
            k = rng.integers(-kmax, kmax + 1, size=3)
        th = rng.uniform(0.0, 2.0 * np.pi)
        a = rng.standard_normal()
        q = (2.0 * np.pi * (float(k[0]) * x / nx + float(k[1]) * y / ny) + th).reshape(-1)
        pz = 2.0 * np.pi * float(k[2]) * z.reshape(-1) / nz
        zc[:, 2 * m], zc[:, 2 * m + 1] = a * torch.sin(pz), a * torch.cos(pz)
        xy[2 * m], xy[2 * m + 1] = torch.cos(q), torch.sin(q)
    out = (zc @ xy).reshape(shape)
    m = float(out.abs().max())
    return out * (amp / m if m > 0 else 0.0)


def smooth_field(shape, rng: np.random.Generator, modes: int = 8, kmax: int = 4,
                 amp: float = 1.0, device=None):
    """Sum of `modes` periodic Fourier modes with |k|_inf <= kmax and random phases, scaled
    so that the field has unit maximum modulus, times amp. shape = (nz, ny, nx). FP64,
    computed with torch on `device` (a torch tensor there), or on the host (numpy) if
    device is None."""
    out = _smooth_field_t(shape, rng, modes, kmax, amp, "cpu" if device is None else device)
    return out.numpy() if device is None else out


# --------------------------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------------------------
def gaussian_plume(n: int = 32, steps: int = 200, sigma0: float = 3.0,
                   d=(1e-2, 1e-3, 1e-4), angles=(30.0, 45.0, 60.0),
                   u=(0.05, 0.02, 0.01)) -> Problem:
    """Advected anisotropic Gaussian plume (shape of Sec. 3.1): periodic n^3, uniform rotated
    tensor, uniform velocity, isotropic Gaussian centred at (n-1)/2, zero background."""
    x, y, z = _grid(n, n, n)
    mu = (n - 1) / 2.0
    r2 = (x - mu) ** 2 + (y - mu) ** 2 + (z - mu) ** 2
    phi0 = np.exp(-0.5 * r2 / sigma0 ** 2)
    return Problem(name="gaussian_plume", nx=n, ny=n, nz=n,
                   d6=rotated_tensor(d, euler_zyz(*angles)), u=np.array(u, dtype=np.float64),
                   phi0=phi0, steps=steps, precision="f64",
                   meta=dict(sigma0=sigma0, mu0=mu, d=d, angles=angles))


def fourier_decay(n: int = 256, steps: int = 2000, mode=(1, 2, 3), c0: float = 1.0,
                  a0: float = 0.01, d=(1e-2, 1e-4, 1e-6), seed: int = 2,
                  rotation: Optional[np.ndarray] = None, use_cos: bool = False,
                  precision: str = "f32") -> Problem:
    """Rotated Fourier-mode decay (shape of Sec. 3.2): periodic n^3, u = 0, uniform tensor
    rotated by a seeded random rotation, phi0 = c0 + a0 sin(k.x), k = 2 pi mode / n."""
    rot = random_rotation(np.random.default_rng(seed)) if rotation is None else rotation
    x, y, z = _grid(n, n, n)
    arg = 2.0 * np.pi * (mode[0] * x + mode[1] * y + mode[2] * z) / n
    phi0 = c0 + a0 * (np.cos(arg) if use_cos else np.sin(arg))
    return Problem(name="fourier_decay", nx=n, ny=n, nz=n,
                   d6=rotated_tensor(d, rot), u=np.zeros(3), phi0=phi0, steps=steps,
                   phi_ref=c0, precision=precision,
                   meta=dict(mode=tuple(mode), c0=c0, a0=a0, d=d, rotation=rot, use_cos=use_cos))


def variable_tensor_source(n: int = 512, steps: int = 1000, seed: int = 3,
                           precision: str = "f32", device=None) -> Problem:
    """Source-driven transport with a smooth SPD tensor field (shape of Sec. 3.3): per node
    D = R(x) diag(d(x)) R(x)^T, R(x) = exp([w(x)]_x) from a smooth random rotation-vector
    field, log10 d_k(x) in [-4.5, 0], u = 0.02 sin(2 pi y / n) e_x, Gaussian source of
    amplitude 1e-4 and width 16 n/512 centred in the box, background phi = 1.

    The fields are evaluated with torch in FP64: on `device` if given (they are then torch
    tensors there, which avoids building the 512^3 inputs on the host), else on the host
    as numpy arrays. Both give the same fields up to rounding."""
    import torch
    dev = "cpu" if device is None else device
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    w = torch.stack([_smooth_field_t(shape, rng, 8, 4, np.pi / 4, dev) for _ in range(3)])
    logd = []
    for _ in range(3):
        f = _smooth_field_t(shape, rng, 8, 4, 1.0, dev)
        lo, hi = float(f.min()), float(f.max())
        logd.append(-4.5 + 4.5 * (f - lo) / (hi - lo))
        del f
    d = [torch.pow(10.0, v) for v in logd]
    del logd
    # Rodrigues: R = I + sin(t) K + (1 - cos(t)) K^2, K the skew matrix of w / |w|.
    t = torch.sqrt((w ** 2).sum(dim=0))
    safe = torch.where(t > 0, t, torch.ones_like(t))
    kx, ky, kz = w[0] / safe, w[1] / safe, w[2] / safe
    st, ct = torch.sin(t), 1.0 - torch.cos(t)
    del w, t, safe
    R = [[None] * 3 for _ in range(3)]
    R[0][0] = 1 + ct * (-(ky ** 2) - kz ** 2)
    R[0][1] = -st * kz + ct * kx * ky
    R[0][2] = st * ky + ct * kx * kz
    R[1][0] = st * kz + ct * kx * ky
    R[1][1] = 1 + ct * (-(kx ** 2) - kz ** 2)
    R[1][2] = -st * kx + ct * ky * kz
    R[2][0] = -st * ky + ct * kx * kz
    R[2][1] = st * kx + ct * ky * kz
    R[2][2] = 1 + ct * (-(kx ** 2) - ky ** 2)
    del kx, ky, kz, st, ct
    d6 = torch.empty((6,) + shape, dtype=torch.float64, device=dev)
    for c, (a, b) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
        d6[c] = (R[a][0] * d[0] * R[b][0] + R[a][1] * d[1] * R[b][1] + R[a][2] * d[2] * R[b][2])
    del R, d
    x, y, z = _torch_grid(n, n, n, dev)
    u = torch.zeros((3,) + shape, dtype=torch.float64, device=dev)
    u[0] = 0.02 * torch.sin(2.0 * np.pi * y / n)
    sig = 16.0 * n / 512.0
    c = n / 2.0
    r = 1e-4 * torch.exp(-((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2) / (2.0 * sig ** 2))
    phi0 = torch.ones(shape, dtype=torch.float64, device=dev)
    if device is None:
        d6, u, r, phi0 = d6.numpy(), u.numpy(), r.numpy(), phi0.numpy()
    return Problem(name="variable_tensor_source", nx=n, ny=n, nz=n, d6=d6, u=u, phi0=phi0,
                   r=r, steps=steps, phi_ref=1.0, precision=precision,
                   meta=dict(seed=seed))


def manufactured_source(n: int = 128, d=(1e-2, 1e-2, 1e-6), shift: float = 2.0,
                        t_end: float = 3.0, precision: str = "f64") -> Problem:
    """Variable-tensor transport with a manufactured source (Sec. 3.3) on the periodic unit
    cube sampled by n^3 nodes x = i / n: K = diag(d1 (2 - s(x)s(y)s(z)), d2, d3) with
    s(.) = sin(2 pi .), u = (1, 1, 1), exact solution phi = exp(A t) s(x)s(y)s(z) with
    A = 1 - 4 pi^2 (2 d1 + d2 + d3) for the source
    R = exp(A t) [sss + 4 d1 pi^2 cos(4 pi x) s(y)^2 s(z)^2 + 2 pi (u_x c(x)s(y)s(z) + ...)].
    Lattice units: dx = 1/n and dt = 1/n^2 make u_lat = 1/n and K_lat = K. The scalar is
    shifted, psi = phi + shift, to keep the populations positive; r holds the spatial part
    of R per step (R dt at unit amplitude), and meta["scale"](m) the amplitude exp(A t) at
    the midpoint of step m."""
    x, y, z = _grid(n, n, n)
    X, Y, Z = x / n, y / n, z / n
    sx, sy, sz = np.sin(2 * np.pi * X), np.sin(2 * np.pi * Y), np.sin(2 * np.pi * Z)
    cx, cy, cz = np.cos(2 * np.pi * X), np.cos(2 * np.pi * Y), np.cos(2 * np.pi * Z)
    sss = sx * sy * sz
    d1, d2, d3 = d
    A = 1.0 - 4.0 * np.pi ** 2 * (2.0 * d1 + d2 + d3)
    d6 = np.zeros((6, n, n, n))
    d6[0] = d1 * (2.0 - sss)
    d6[3] = d2
    d6[5] = d3
    u_phys = np.array([1.0, 1.0, 1.0])
    F = (sss + 4.0 * d1 * np.pi ** 2 * np.cos(4 * np.pi * X) * sy ** 2 * sz ** 2
         + 2.0 * np.pi * (u_phys[0] * cx * sy * sz + u_phys[1] * sx * cy * sz + u_phys[2] * sx * sy * cz))
    dt = 1.0 / n ** 2
    steps = int(round(t_end / dt))
    return Problem(name="manufactured_source", nx=n, ny=n, nz=n, d6=d6, u=u_phys / n,
                   phi0=shift + sss, r=F * dt, steps=steps, phi_ref=shift, precision=precision,
                   meta=dict(A=A, dt=dt, shift=shift, d=d, t_end=t_end,
                             scale=lambda m: float(np.exp(A * (m + 0.5) * dt)),
                             exact=lambda t: np.exp(A * t) * sss))


def porous_spheres(n: int = 384, steps: int = 5000, seed: int = 4, radius: float = 12.0,
                   porosity: float = 0.4, d_solid=(1e-1, 1e-1, 1e-5),
                   angles=(105.0, 50.0, 25.0), d_fluid: float = 1e-2,
                   phi_hot: float = 2.0, phi_cold: float = 1.0,
                   precision: str = "f32") -> Problem:
    """Heterogeneous porous conduction (shape of Sec. 4.2.2 with spheres): overlapping
    spheres of radius `radius` (scaled with n/384), centres uniform, added until the fluid
    fraction reaches `porosity`; rotated anisotropic solid tensor (ratio 1e4:1), isotropic
    fluid; Dirichlet planes phi_hot at x = 0 and phi_cold at x = n-1, periodic in y and z;
    initial linear profile between the two wall values (walls half a cell outside)."""
    rng = np.random.default_rng(seed)
    rad = radius * n / 384.0
    solid = np.zeros((n, n, n), dtype=bool)
    target = int(np.ceil((1.0 - porosity) * n ** 3))
    count = 0
    h = int(np.ceil(rad))
    off = np.arange(-h, h + 1)
    while count < target:
        cx, cy, cz = rng.uniform(0, n, size=3)
        ix = np.floor(cx).astype(int) + off
        iy = np.floor(cy).astype(int) + off
        iz = np.floor(cz).astype(int) + off
        ix = ix[(ix >= 0) & (ix < n)]  # clipped in x
        dx = ix - cx
        dy = iy - cy
        dz = iz - cz
        ball = (dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2) <= rad ** 2
        zz, yy = np.mod(iz, n), np.mod(iy, n)  # periodic in y and z
        box = solid[np.ix_(zz, yy, ix)]
        count += int(np.count_nonzero(ball & ~box))
        solid[np.ix_(zz, yy, ix)] = box | ball
    frac = count / n ** 3
    phase = solid.astype(np.uint8)
    ds = rotated_tensor(d_solid, euler_zyz(*angles))
    df = np.array([d_fluid, 0, 0, d_fluid, 0, d_fluid], dtype=np.float64)
    d6 = np.where(solid[None], ds[:, None, None, None], df[:, None, None, None])
    xs = np.arange(n, dtype=np.float64)
    prof = phi_hot + (phi_cold - phi_hot) * (xs + 0.5) / n
    phi0 = np.broadcast_to(prof[None, None, :], (n, n, n)).copy()
    return Problem(name="porous_spheres", nx=n, ny=n, nz=n, d6=d6, u=np.zeros(3), phi0=phi0,
                   steps=steps, bc_x="dirichlet", phi_lo=phi_hot, phi_hi=phi_cold,
                   phi_ref=0.5 * (phi_hot + phi_cold), precision=precision,
                   meta=dict(phase=phase, solid_fraction=float(frac), d_solid_6=ds,
                             d_fluid_6=df, d6_table=np.stack([df, ds])))


def log_tensor_field(n: int, seed: int, base: float = 1e-2, amp: float = 0.5) -> np.ndarray:
    """Log-diffusivity tensor field L = log(base) I + symmetric smooth fluctuation of
    amplitude `amp` (6 smooth fields). D = expm(L) is SPD for any L."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    L = np.stack([smooth_field(shape, rng, amp=amp) for _ in range(6)])
    for c in (0, 3, 5):
        L[c] += np.log(base)
    return L


def adjoint_problem(n: int = 128, steps: int = 500, seed_l: int = 5, seed_phi: int = 7,
                    u=(0.0, 0.0, 0.0), precision: str = "f32") -> Problem:
    """Adjoint inverse problem inputs: log-diffusivity field (seed_l), initial scalar
    1 + 0.5 * smooth field (seed_phi), u as given (zero by default)."""
    L = log_tensor_field(n, seed_l)
    phi0 = 1.0 + smooth_field((n, n, n), np.random.default_rng(seed_phi), amp=0.5)
    return Problem(name="adjoint", nx=n, ny=n, nz=n, d6=L, u=np.asarray(u, dtype=np.float64),
                   phi0=phi0, steps=steps, tensor_is_log=True, phi_ref=1.0,
                   precision=precision, meta=dict(seed_l=seed_l, seed_phi=seed_phi))


def random_populations(q: int, shape, rng: np.random.Generator, base: np.ndarray,
                       scale: float) -> np.ndarray:
    """Positive random populations base_i * (1 + scale * U(-1, 1)) for node-level tests;
    `base` holds one positive value per direction."""
    nz, ny, nx = shape
    noise = rng.uniform(-1.0, 1.0, size=(q, nz, ny, nx))
    return base[:, None, None, None] * (1.0 + scale * noise)
