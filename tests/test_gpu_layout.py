"""The documented layout of the library's population buffers, read from raw saved state.

Populations are stored by row: for row r = z * ny + y the Q runs of nx values lie together
([z][y][i][x]), as deviations d_i = g_i - W_i phi_ref in the storage type. With the FP32
rest population of the 16-bit forms, run 0 of each row holds nx FP32 values (the space of
two 16-bit runs) and run i >= 1 starts at 16-bit element (i + 1) nx of the row.
Bit-exact checks (the stored values are roundings of known inputs).
"""
import numpy as np
import pytest
import torch

from paper_2605_01774_amd import _lib, lattice
from gpuhelp import banner

pytestmark = pytest.mark.gpu

NX, NY, NZ = 70, 3, 2  # a ragged row length (not a multiple of 64)


def _lattice_with_pattern(prec, **kw):
    q = kw.pop("q", 19)
    lat = lattice.Lattice(NX, NY, NZ, precision=prec, phi_ref=1.0, device="cuda:0", q=q, **kw)
    lat.set_diffusion([1e-2, 0, 0, 1e-2, 0, 1e-2])
    lat.init_equilibrium(np.ones((NZ, NY, NX)))
    _, w = _lib.velocity_table(q)
    rng = np.random.default_rng(5)
    # populations W_i (1 + small node- and direction-dependent deviations)
    f = w[:, None, None, None] * (1.0 + 0.01 * rng.uniform(-1, 1, (q, NZ, NY, NX)))
    lat.set_populations(f)
    raw = lat.save_state()[0].cpu().numpy()
    d = f - w[:, None, None, None] * 1.0  # deviations around phi_ref = 1
    return lat, raw, d


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("prec,dtype", [("f64", np.float64), ("f32", np.float32)])
def test_row_layout_wide_forms(prec, dtype, q):
    banner(f"row layout {prec} q{q}")
    lat, raw, d = _lattice_with_pattern(prec, q=q)
    got = raw.view(dtype).reshape(NZ, NY, q, NX)            # [z][y][i][x]
    want = np.transpose(d, (1, 2, 0, 3)).astype(dtype)       # (Q, z, y, x) -> (z, y, Q, x)
    assert np.array_equal(got, want)


def _bf16_of(x):
    """Round-to-nearest-even bfloat16 of float32 values, as float32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return (b.astype(np.uint32) << 16).view(np.float32)


def test_row_layout_bf16():
    banner("row layout bf16")
    lat, raw, d = _lattice_with_pattern("bf16")
    bits = raw.view(np.uint16).reshape(NZ, NY, 19, NX).astype(np.uint32) << 16
    got = bits.view(np.float32)
    want = _bf16_of(np.transpose(d, (1, 2, 0, 3)).astype(np.float32))
    assert np.array_equal(got, want)


def test_row_layout_bf16_rest_fp32():
    banner("row layout bf16 + FP32 rest")
    lat, raw, d = _lattice_with_pattern("bf16", rest_fp32=True)
    rows = raw.view(np.uint16).reshape(NZ, NY, 20 * NX)      # one row: 2 nx + 18 nx halves
    rest = rows[:, :, :2 * NX].copy().view(np.float32)         # (z, y, nx) FP32
    moving = (rows[:, :, 2 * NX:].reshape(NZ, NY, 18, NX).astype(np.uint32) << 16).view(np.float32)
    dm = np.transpose(d[1:], (1, 2, 0, 3)).astype(np.float32)  # exact FP32 deviations, i >= 1
    want_m = _bf16_of(dm)
    assert np.array_equal(moving, want_m)
    # the rest value carries the 18 rounding residuals of its node: node mass is kept
    mass_stored = rest.astype(np.float64) + moving.astype(np.float64).sum(axis=2)
    mass_true = d.sum(axis=0)
    assert np.abs(mass_stored - mass_true).max() <= 2e-7 * np.abs(d[0]).max() + 1e-9
