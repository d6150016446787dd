"""elbm_reduce_noalloc, the allocation-free variant of elbm_reduce for callers that cannot
allocate: through the C ABI, its four FP64 sums must equal elbm_reduce's bitwise (the same
kernels with the same block count, the partials in the library's static device array
instead of the handle's scratch), on calls in a row with shrinking inputs: the array keeps
the previous call's partials beyond the ones a smaller lattice writes, and they must not
leak into its sums."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2605_01774_amd import inputs as I
from gpuhelp import banner, gpu_lattice

pytestmark = pytest.mark.gpu


def _ragged(shape, prec, seed):
    nx, ny, nz = shape
    n3 = (nz, ny, nx)
    rng = np.random.default_rng(seed)
    d6 = np.tile(I.rotated_tensor((2e-2, 5e-3, 1e-4), I.euler_zyz(20, 40, 60))[:, None, None, None],
                 (1,) + n3)
    u = 0.03 * rng.uniform(-1, 1, (3,) + n3)
    phi0 = 1.0 + 0.3 * rng.uniform(-1, 1, n3)
    r = 1e-3 * rng.uniform(-1, 1, n3)
    prob = I.Problem("noalloc", nx, ny, nz, d6, u, phi0, steps=7, r=r, phi_ref=1.0)
    return gpu_lattice(prob, prec)


def _noalloc(lat):
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda:0")
    rc = lat.lib.elbm_reduce_noalloc(lat._h, ctypes.c_void_p(out.data_ptr()), 32)
    assert rc == 0, lat.lib.elbm_last_error().decode()
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_reduce_equals_reduce_on_shrinking_inputs():
    cases = [("decay 256^3 f32 (2048 partials)", None, "f32"),
             ("ragged 37x29x23 f64 (97 partials)", (37, 29, 23), "f64"),
             ("ragged 11x7x5 bf16 (2 partials)", (11, 7, 5), "bf16")]
    for name, shape, prec in cases:
        banner(f"no-alloc reduce: {name}")
        if shape is None:
            lat = gpu_lattice(I.fourier_decay(n=256, steps=3, precision=prec), prec)
        else:
            lat = _ragged(shape, prec, 5)
        lat.step(3)
        got = _noalloc(lat)
        want = lat.reduce()
        print(f"{name}: noalloc {got}, reduce {want}")
        assert np.array_equal(got, want)
        # an undersized output buffer is refused before any launch
        small = torch.zeros(3, dtype=torch.float64, device="cuda:0")
        rc = lat.lib.elbm_reduce_noalloc(lat._h, ctypes.c_void_p(small.data_ptr()), 24)
        assert rc == -2 and "out4" in lat.lib.elbm_last_error().decode()
        del lat
        torch.cuda.empty_cache()
