"""Closed-form linear Fourier symbol of the scheme at zero velocity (test infrastructure).

At u = 0 the equilibrium is W_i phi, ln(g_eq/W) = ln(phi) is the same in every direction so
the correction C of Sec. 2.5 vanishes (the ghost part has zero mass), and
<Dh|Ds_post>_H = (3/phi) j*. sum_i c_i Dh_i = 0 because the ghost part carries no flux
(Sec. 2.2). Hence lambda = 1 exactly, and the post-collision state is
    post_i = W_i (phi + 3 c_i . (I - S) j),
whatever the ghost content before collision. With streaming g_i(x + c_i, t + 1) = post_i(x, t)
and a single mode exp(i k.x), the pre-collision moments (phi, j) evolve by the 4x4 matrix

    M(k) = [[a, 3 b^T (I - S)], [b, 3 C (I - S)]],
    a = sum_i W_i e^{-i k.c_i},  b = sum_i W_i c_i e^{-i k.c_i},  C = sum_i W_i c_i c_i^T e^{-i k.c_i}.

This is a second, independent derivation of the discrete update from the paper's equations
(it never forms populations), used to pin the oracle and the GPU path: lift, S(D),
equilibrium, streaming and the lambda = 1 property all enter it.
"""
from __future__ import annotations

import itertools

import numpy as np


def lattice(q: int = 19):
    """Velocities and weights from their definitions (Sec. 2.1 for D3Q27; D3Q19 standard)."""
    cs, ws = [], []
    for c in itertools.product((-1, 0, 1), repeat=3):
        m = sum(1 for v in c if v != 0)
        if q == 19 and m == 3:
            continue
        cs.append(c)
        if q == 27:
            ws.append((2.0 / 3.0) ** (3 - m) * (1.0 / 6.0) ** m)
        else:
            ws.append({0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0}[m])
    return np.array(cs, dtype=np.float64), np.array(ws)


def relaxation_matrix(d6) -> np.ndarray:
    """S from D through the principal frame (Sec. 2.3, eigen form): S = Q diag(s_k) Q^T,
    s_k = (1/2 + D_k / cs^2)^-1 with cs^2 = 1/3, dt = 1."""
    d = np.asarray(d6, dtype=np.float64)
    D = np.array([[d[0], d[1], d[2]], [d[1], d[3], d[4]], [d[2], d[4], d[5]]])
    lam, Q = np.linalg.eigh(D)
    s = 1.0 / (0.5 + 3.0 * lam)
    return (Q * s) @ Q.T


def symbol(k: np.ndarray, d6, q: int = 19) -> np.ndarray:
    """4x4 complex matrix M(k) acting on (phi_hat, j_hat)."""
    c, w = lattice(q)
    S = relaxation_matrix(d6)
    IS = np.eye(3) - S
    ph = np.exp(-1j * (c @ np.asarray(k, dtype=np.float64)))
    a = np.sum(w * ph)
    b = (w * ph) @ c
    C = np.einsum("i,ia,ib->ab", w * ph, c, c)
    M = np.zeros((4, 4), dtype=np.complex128)
    M[0, 0] = a
    M[0, 1:] = 3.0 * (b @ IS)
    M[1:, 0] = b
    M[1:, 1:] = 3.0 * (C @ IS)
    return M


def decay_rate(k: np.ndarray, d6, q: int = 19) -> float:
    """-ln |mu_max(k)|: asymptotic per-step decay rate of the mode."""
    mu = np.linalg.eigvals(symbol(k, d6, q))
    return float(-np.log(np.max(np.abs(mu))))


def mode_history(k: np.ndarray, d6, steps, v0=None, q: int = 19) -> np.ndarray:
    """Complex moment vectors M^n v0 for n in `steps` (sorted ints). v0 defaults to an
    equilibrium start (1, 0, 0, 0)."""
    M = symbol(k, d6, q)
    v = np.array([1, 0, 0, 0], dtype=np.complex128) if v0 is None else np.asarray(v0, np.complex128)
    out, n = [], 0
    for s in steps:
        while n < s:
            v = M @ v
            n += 1
        out.append(v.copy())
    return np.array(out)


def populations_after(k: np.ndarray, d6, n: int, shape, c0: float, a0: float,
                      use_cos: bool = False, q: int = 19):
    """Pre-collision populations f_i(x, n) (n >= 1) of the run started from the equilibrium
    of c0 + a0 sin(k.x) (or cos). Returns (velocities c, array (q, nz, ny, nx)):
    f_i(x, n) = post_i(x - c_i, n - 1) = W_i (phi_{n-1} + 3 c_i.(I - S) j_{n-1}) at x - c_i."""
    c, w = lattice(q)
    S = relaxation_matrix(d6)
    IS = np.eye(3) - S
    v = mode_history(k, d6, [n - 1], q=q)[0]
    nz, ny, nx = shape
    z = np.arange(nz)[:, None, None]
    y = np.arange(ny)[None, :, None]
    x = np.arange(nx)[None, None, :]
    out = np.empty((len(w), nz, ny, nx))
    for i in range(len(w)):
        arg = k[0] * (x - c[i, 0]) + k[1] * (y - c[i, 1]) + k[2] * (z - c[i, 2])
        e = np.exp(1j * arg)
        amp = v[0] + 3.0 * (c[i] @ IS) @ v[1:]
        field = (e * amp).real if use_cos else (e * amp).imag
        out[i] = w[i] * (c0 + a0 * field)
    return c, out
