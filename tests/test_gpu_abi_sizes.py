"""Byte sizes at the C ABI: every caller-owned device buffer is passed with its size, and an
entry point given a buffer one byte smaller than what it would read or write returns
ELBM_ESHAPE with a message naming the buffer, before touching anything; a required buffer
that is NULL is ELBM_EINVAL. Called through ctypes directly, as a C caller would."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2605_01774_amd import inputs as I
from gpuhelp import banner, gpu_lattice

pytestmark = pytest.mark.gpu

ESHAPE, EINVAL = -2, -1


def P(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def nb(t):
    return t.numel() * t.element_size()


def _expect(lat, rc, code, name):
    msg = lat.lib.elbm_last_error().decode()
    assert rc == code, (rc, msg)
    assert name in msg, msg


@pytest.fixture(scope="module")
def lat():
    prob = I.adjoint_problem(n=8, steps=4)
    return gpu_lattice(prob, "f32")


def test_population_and_state_buffers(lat):
    banner("ABI sizes: populations and state")
    L = lat.lib
    h = lat._h
    n, q = lat.n, lat.q
    pb = lat.pop_bytes
    a = torch.zeros(pb, dtype=torch.uint8, device="cuda:0")
    b = torch.zeros(pb, dtype=torch.uint8, device="cuda:0")
    _expect(lat, L.elbm_bind_populations(h, P(a), pb - 1, P(b), pb), ESHAPE, "buf_a")
    _expect(lat, L.elbm_bind_populations(h, P(a), pb, P(b), pb - 1), ESHAPE, "buf_b")
    a2 = torch.zeros(pb + 16, dtype=torch.uint8, device="cuda:0")
    _expect(lat, L.elbm_bind_populations(h, ctypes.c_void_p(a2.data_ptr() + 8), pb, P(b), pb), EINVAL,
            "16-byte aligned")
    # the lattice's own binding is still the one in use
    f = torch.full((q * n,), -7.0, dtype=torch.float64, device="cuda:0")
    _expect(lat, L.elbm_get_populations(h, P(f), nb(f) - 1), ESHAPE, "f")
    assert bool((f == -7.0).all())  # untouched
    _expect(lat, L.elbm_get_populations(h, None, 0), EINVAL, "f")
    assert L.elbm_get_populations(h, P(f), nb(f)) == 0
    _expect(lat, L.elbm_set_populations(h, P(f), nb(f) - 8), ESHAPE, "f")
    st = torch.zeros(pb, dtype=torch.uint8, device="cuda:0")
    step, pend = ctypes.c_int64(), ctypes.c_int32()
    _expect(lat, L.elbm_save_state(h, P(st), pb - 1, ctypes.byref(step), ctypes.byref(pend)), ESHAPE, "dst")
    assert int(st.sum()) == 0
    _expect(lat, L.elbm_load_state(h, P(st), pb - 1, 0, 0), ESHAPE, "src")
    dst = torch.zeros(pb, dtype=torch.uint8, device="cuda:0")
    lam = torch.zeros(n, dtype=torch.float32, device="cuda:0")
    br = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
    _expect(lat, L.elbm_step_buffers(h, P(a), pb - 1, 0, P(dst), pb, None, 0, None, 0), ESHAPE, "src")
    _expect(lat, L.elbm_step_buffers(h, P(a), pb, 0, P(dst), pb - 1, None, 0, None, 0), ESHAPE, "dst")
    _expect(lat, L.elbm_step_buffers(h, ctypes.c_void_p(a2.data_ptr() + 8), pb, 0, P(dst), pb, None, 0, None, 0),
            EINVAL, "16-byte aligned")
    _expect(lat, L.elbm_step_buffers(h, P(a), pb, 0, P(dst), pb, P(lam), nb(lam) - 1, P(br), nb(br)),
            ESHAPE, "lambda_rec")
    _expect(lat, L.elbm_step_buffers(h, P(a), pb, 0, P(dst), pb, P(lam), nb(lam), P(br), nb(br) - 1),
            ESHAPE, "branch_rec")
    assert int(dst.sum()) == 0
    t0 = lat.time
    lam3 = torch.zeros(3 * n, dtype=torch.float32, device="cuda:0")
    br3 = torch.zeros(3 * n, dtype=torch.uint8, device="cuda:0")
    _expect(lat, L.elbm_step_record(h, 3, P(lam3), nb(lam3) - 1, P(br3), nb(br3)), ESHAPE, "lambda_rec")
    _expect(lat, L.elbm_step_record(h, 3, P(lam3), nb(lam3), P(br3), nb(br3) - 1), ESHAPE, "branch_rec")
    assert lat.time == t0  # no step was taken


def test_field_buffers(lat):
    banner("ABI sizes: fields and moments")
    L = lat.lib
    h = lat._h
    n = lat.n
    d6 = torch.zeros((6, n), dtype=torch.float64, device="cuda:0")
    d6[0] = d6[3] = d6[5] = 1e-2
    ts = torch.zeros((n, 6), dtype=torch.float32, device="cuda:0")
    bad = ctypes.c_int64(-5)
    _expect(lat, L.elbm_set_diffusion_field(h, P(d6), nb(d6) - 1, 0, P(ts), nb(ts), ctypes.byref(bad)),
            ESHAPE, "d6")
    _expect(lat, L.elbm_set_diffusion_field(h, P(d6), nb(d6), 0, P(ts), nb(ts) - 1, ctypes.byref(bad)),
            ESHAPE, "t_store")
    assert float(ts.abs().sum()) == 0.0
    tab = torch.tensor([[1e-2], [0.0], [0.0], [1e-2], [0.0], [1e-2]], dtype=torch.float64, device="cuda:0")
    ph = torch.zeros(n, dtype=torch.uint8, device="cuda:0")
    t1 = torch.zeros((1, 6), dtype=torch.float32, device="cuda:0")
    _expect(lat, L.elbm_set_diffusion_phases(h, P(tab), nb(tab) - 1, 1, 0, P(ph), nb(ph), P(t1), nb(t1),
                                             ctypes.byref(bad)), ESHAPE, "d6_table")
    _expect(lat, L.elbm_set_diffusion_phases(h, P(tab), nb(tab), 1, 0, P(ph), n - 1, P(t1), nb(t1),
                                             ctypes.byref(bad)), ESHAPE, "phase")
    _expect(lat, L.elbm_set_diffusion_phases(h, P(tab), nb(tab), 1, 0, P(ph), n, P(t1), nb(t1) - 1,
                                             ctypes.byref(bad)), ESHAPE, "t_store")
    u3 = torch.zeros((3, n), dtype=torch.float64, device="cuda:0")
    us = torch.zeros((3, n), dtype=torch.float32, device="cuda:0")
    _expect(lat, L.elbm_set_velocity_field(h, P(u3), nb(u3) - 1, P(us), nb(us), ctypes.byref(bad)),
            ESHAPE, "u3")
    _expect(lat, L.elbm_set_velocity_field(h, P(u3), nb(u3), P(us), nb(us) - 1, ctypes.byref(bad)),
            ESHAPE, "u_store")
    r = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    rs = torch.zeros(n, dtype=torch.float32, device="cuda:0")
    _expect(lat, L.elbm_set_source_field(h, P(r), nb(r) - 1, P(rs), nb(rs)), ESHAPE, "r")
    _expect(lat, L.elbm_set_source_field(h, P(r), nb(r), P(rs), nb(rs) - 1), ESHAPE, "r_store")
    # stores the step kernels read with vector loads must be 16-byte aligned
    us2 = torch.zeros(3 * n + 4, dtype=torch.float32, device="cuda:0")
    _expect(lat, L.elbm_set_velocity_field(h, P(u3), nb(u3), ctypes.c_void_p(us2.data_ptr() + 4), nb(us),
                                           ctypes.byref(bad)), EINVAL, "u_store must be 16-byte aligned")
    rs2 = torch.zeros(n + 4, dtype=torch.float32, device="cuda:0")
    _expect(lat, L.elbm_set_source_field(h, P(r), nb(r), ctypes.c_void_p(rs2.data_ptr() + 8), nb(rs)), EINVAL,
            "r_store must be 16-byte aligned")
    assert float(us2.abs().sum()) == 0.0 and float(rs2.abs().sum()) == 0.0
    phi0 = torch.ones(n, dtype=torch.float64, device="cuda:0")
    j0 = torch.zeros((3, n), dtype=torch.float64, device="cuda:0")
    _expect(lat, L.elbm_init_equilibrium(h, P(phi0), nb(phi0) - 1, None, 0), ESHAPE, "phi0")
    _expect(lat, L.elbm_init_equilibrium(h, P(phi0), nb(phi0), P(j0), nb(j0) - 1), ESHAPE, "j0")
    phi = torch.full((n,), 3.0, dtype=torch.float64, device="cuda:0")
    qv = torch.full((3, n), 3.0, dtype=torch.float64, device="cuda:0")
    _expect(lat, L.elbm_read_moments(h, P(phi), nb(phi) - 1, P(qv), nb(qv)), ESHAPE, "phi")
    _expect(lat, L.elbm_read_moments(h, P(phi), nb(phi), P(qv), nb(qv) - 1), ESHAPE, "q3")
    assert bool((phi == 3.0).all()) and bool((qv == 3.0).all())
    # the same calls with the full sizes succeed (q3 may be NULL)
    assert L.elbm_read_moments(h, P(phi), nb(phi), None, 0) == 0


def test_adjoint_buffers(lat):
    banner("ABI sizes: adjoint")
    L = lat.lib
    h = lat._h
    n, q = lat.n, lat.q
    pb = lat.pop_bytes
    st = lat.save_state()[0]
    lam = torch.zeros(n, dtype=torch.float32, device="cuda:0")
    br = torch.full((n,), 255, dtype=torch.uint8, device="cuda:0")
    ai = torch.zeros((q, n), dtype=torch.float32, device="cuda:0")
    ao = torch.full((q, n), 5.0, dtype=torch.float32, device="cuda:0")
    tg = torch.zeros((n, 6), dtype=torch.float32, device="cuda:0")
    full = [P(st), pb, 0, P(lam), nb(lam), P(br), nb(br), P(ai), nb(ai), P(ao), nb(ao), P(tg), nb(tg)]
    for k, name in ((1, "state"), (4, "lambda_rec"), (6, "branch_rec"), (8, "adj_in"), (10, "adj_out"),
                    (12, "t_grad")):
        args = list(full)
        args[k] -= 1
        _expect(lat, L.elbm_adjoint_step(h, *args), ESHAPE, name)
    assert bool((ao == 5.0).all())
    ws_bytes = lat.gradient_workspace_bytes(4, 2)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda:0")
    _expect(lat, L.elbm_forward_record(h, 4, 2, P(ws), ws_bytes - 1), ESHAPE, "workspace")
    dphi = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    _expect(lat, L.elbm_gradient(h, 4, 2, P(ws), ws_bytes - 1, P(dphi), nb(dphi), P(tg), nb(tg), None, 0, None,
                                 0), ESHAPE, "workspace")
    _expect(lat, L.elbm_gradient(h, 4, 2, P(ws), ws_bytes, P(dphi), nb(dphi) - 1, P(tg), nb(tg), None, 0, None,
                                 0), ESHAPE, "dphi_n")
    _expect(lat, L.elbm_gradient(h, 4, 2, P(ws), ws_bytes, P(dphi), nb(dphi), P(tg), nb(tg) - 1, None, 0, None,
                                 0), ESHAPE, "t_grad")
    d6 = lat._keep["d6"]
    out6 = torch.zeros((6, n), dtype=torch.float64, device="cuda:0")
    _expect(lat, L.elbm_tensor_gradient(h, P(d6), nb(d6) - 1, 1, P(tg), nb(tg), P(out6), nb(out6)), ESHAPE, "d6")
    _expect(lat, L.elbm_tensor_gradient(h, P(d6), nb(d6), 1, P(tg), nb(tg), P(out6), nb(out6) - 1), ESHAPE,
            "out6")
    dphi0 = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    _expect(lat, L.elbm_initial_gradient(h, P(ai), nb(ai) - 1, P(dphi0), nb(dphi0), None, 0), ESHAPE, "adj0")
    _expect(lat, L.elbm_initial_gradient(h, P(ai), nb(ai), P(dphi0), nb(dphi0) - 1, None, 0), ESHAPE, "dphi0")
    _expect(lat, L.elbm_initial_gradient(h, P(ai), nb(ai), None, 0, None, 0), EINVAL, "dphi0")
    assert float(out6.abs().sum()) == 0.0 and float(dphi0.abs().sum()) == 0.0


def test_stream_copy(lat):
    """The bandwidth reference copies bytes exactly (partial last tiles included) and rejects
    bad sizes, misaligned and overlapping buffers (ELBM_EINVAL) and a short destination
    (ELBM_ESHAPE) before launching anything."""
    banner("ABI: stream copy")
    L, h = lat.lib, lat._h
    # 16-byte words: one, one partial tile, 24 tiles (dealt to the XCDs) with a partial last,
    # and 2049 tiles (natural order)
    for n in (4, 4 * 1001, 4 * (24 * 1024 - 5), 4 * (2048 * 1024 + 37)):
        a = torch.arange(n, dtype=torch.float32, device="cuda:0")
        b = torch.zeros_like(a)
        assert L.elbm_stream_copy(h, P(a), nb(a), P(b), nb(b)) == 0, L.elbm_last_error()
        torch.cuda.synchronize()
        assert torch.equal(a, b), n
    a = torch.arange(64, dtype=torch.float32, device="cuda:0")
    b = torch.zeros(64, dtype=torch.float32, device="cuda:0")
    _expect(lat, L.elbm_stream_copy(h, P(a), 12, P(b), nb(b)), EINVAL, "multiple of 16")
    _expect(lat, L.elbm_stream_copy(h, P(a), 0, P(b), nb(b)), EINVAL, "multiple of 16")
    _expect(lat, L.elbm_stream_copy(h, P(a), nb(a), P(b), nb(a) - 16), ESHAPE, "dst smaller")
    _expect(lat, L.elbm_stream_copy(h, ctypes.c_void_p(a.data_ptr() + 4), 16, P(b), nb(b)), EINVAL, "aligned")
    _expect(lat, L.elbm_stream_copy(h, P(a), 64, ctypes.c_void_p(a.data_ptr() + 16), 64), EINVAL, "overlap")
    _expect(lat, L.elbm_stream_copy(h, None, 16, P(b), nb(b)), EINVAL, "null")
    torch.cuda.synchronize()
    assert float(b.abs().sum()) == 0.0
