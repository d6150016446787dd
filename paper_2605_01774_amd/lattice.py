"""Python front end of the lattice: torch provides device memory and the stream; every step
of the scheme runs in the HIP library (libelbm.so) through the C ABI of include/elbm.h.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Union

import numpy as np
import torch

from . import _lib

# Default ghost floor tau per arithmetic precision. The closed-form amplitude divides a
# first-order quantity in the ghost part by a second-order one, so rounding in a ghost part
# near roundoff level is amplified; tau^2 phi added to the denominator removes that
# sensitivity below |Dh| ~ tau. A rounding-level ghost h then moves the update by about
# |ln E| (h / tau)^2 phi: FP64 arithmetic (h ~ 1e-16 phi) takes tau = 1e-9, which keeps that
# near 1e-14; FP32 arithmetic needs 1e-4. At physical nodes the floor changes the update by
# at most |lambda - 1| |Dh|, and by a relative (tau phi / |Dh|)^2 in lambda - 1.
GHOST_FLOOR = {"f64": 1e-9, "f32": 1e-4, "bf16": 1e-4, "fp16": 1e-4}
# Default storage scale of the FP16 form (stored value = deviation / scale).
STORE_SCALE = {"f64": 1.0, "f32": 1.0, "bf16": 1.0, "fp16": 2.0 ** -8}
REAL_DTYPE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.float32, "fp16": torch.float32}

TensorLike = Union[np.ndarray, torch.Tensor]


def _numel(a) -> int:
    """Number of values of a numpy array, torch tensor (any device) or scalar."""
    return a.numel() if isinstance(a, torch.Tensor) else int(np.size(a))


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _nb(t: Optional[torch.Tensor]) -> int:
    """Byte size of a caller buffer as the C ABI takes it next to the pointer (0 for None)."""
    return 0 if t is None else t.numel() * t.element_size()


class Lattice:
    """A D3Q19 (or, with q=27, D3Q27) lattice of nx * ny * nz nodes in one precision form
    on one GPU.

    precision: "f64" | "f32" | "bf16" | "fp16" (storage; arithmetic is FP64 for f64, FP32
    otherwise). bc_x: "periodic" | "dirichlet". scalar_kernel forces the one-node-per-thread
    step kernel; vector_width (1, 2, 4; 0 = automatic) sets the nodes per lane of the
    row-vector kernel. For the 16-bit forms, rest_fp32 stores the rest population in FP32
    with the node's rounding residuals (mass-conserving storage) and stochastic_rounding
    rounds the 16-bit stores stochastically. Arrays follow include/elbm.h: planes
    [component][z][y][x]."""

    def __init__(self, nx: int, ny: int, nz: int, precision: str = "f32",
                 bc_x: str = "periodic", phi_ref: float = 0.0, eps: float = 0.0,
                 ghost_floor: Optional[float] = None, root_rho: float = -1.0,
                 store_scale: Optional[float] = None, device: Union[str, torch.device] = "cuda",
                 scalar_kernel: bool = False, vector_width: int = 0, rest_fp32: bool = False,
                 stochastic_rounding: bool = False, q: int = 19):
        self.q = q
        self.lib = _lib.load(q)
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the lattice lives on a GPU device")
        self.precision = precision
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        self.real = REAL_DTYPE[precision]
        cfg = _lib.Config()
        cfg.nx, cfg.ny, cfg.nz = nx, ny, nz
        cfg.precision = _lib.PRECISIONS[precision]
        cfg.bc_x = _lib.BC[bc_x]
        cfg.flags = ((_lib.FLAG_SCALAR_KERNEL if scalar_kernel else 0) | (int(vector_width) << 4) |
                     (_lib.FLAG_REST_FP32 if rest_fp32 else 0) |
                     (_lib.FLAG_STOCHASTIC_ROUNDING if stochastic_rounding else 0))
        cfg.phi_ref = phi_ref
        cfg.eps = eps
        cfg.ghost_floor = GHOST_FLOOR[precision] if ghost_floor is None else ghost_floor
        cfg.root_rho = root_rho
        cfg.store_scale = STORE_SCALE[precision] if store_scale is None else store_scale
        self.cfg = cfg
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            self._check(self.lib.elbm_create(ctypes.byref(cfg), ctypes.byref(self._h)))
            nbytes = self._check(self.lib.elbm_population_bytes(self._h))
            self.pop_bytes = nbytes
            self.buf_a = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.buf_b = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self._check(self.lib.elbm_bind_populations(self._h, _ptr(self.buf_a), _nb(self.buf_a),
                                                       _ptr(self.buf_b), _nb(self.buf_b)))
        self.set_stream(torch.cuda.current_stream(self.device))
        self._keep = {}   # device stores the library reads while stepping
        self._has_source = False

    # -- lifetime --------------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.elbm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int) -> int:
        return _lib.check(rc, self.lib)

    def set_stream(self, stream: torch.cuda.Stream):
        self.stream = stream
        self._check(self.lib.elbm_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))

    # -- helpers ---------------------------------------------------------------------------
    def _dev64(self, a: TensorLike, comps: Optional[int]) -> torch.Tensor:
        t = torch.as_tensor(a)
        t = t.to(device=self.device, dtype=torch.float64).contiguous()
        want = (self.n,) if comps is None else (comps * self.n,)
        if t.numel() != want[0]:
            raise ValueError(f"expected {want[0]} values, got {t.numel()}")
        return t

    def _need(self, t: Optional[torch.Tensor], name: str, numel: int, dtype: torch.dtype,
              optional: bool = False) -> None:
        """Check a caller buffer before its pointer goes to the library, which cannot see
        sizes: a contiguous tensor on the lattice's device, of `dtype`, with at least `numel`
        elements."""
        if t is None:
            if optional:
                return
            raise ValueError(f"{name} is required")
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"{name} must be a tensor on {self.device}")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() < numel:
            raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")

    def _field(self, comps: int) -> torch.Tensor:
        return torch.empty((comps,) + self.shape, dtype=self.real, device=self.device)

    # -- coefficients ----------------------------------------------------------------------
    def set_diffusion(self, d6: TensorLike, is_log: bool = False) -> None:
        """Uniform tensor (6 values, host) or a per-node field (6, nz, ny, nx); is_log:
        the field holds L with D = expm(L)."""
        if _numel(d6) == 6 and not is_log:
            arr = (ctypes.c_double * 6)(*[float(v) for v in np.asarray(torch.as_tensor(d6).cpu())])
            self._check(self.lib.elbm_set_diffusion_uniform(self._h, arr))
            self._keep.pop("t", None)
            return
        d = self._dev64(d6, 6)
        t = self._field(6)
        bad = ctypes.c_int64(-1)
        rc = self.lib.elbm_set_diffusion_field(self._h, _ptr(d), _nb(d), int(is_log), _ptr(t), _nb(t),
                                               ctypes.byref(bad))
        if rc < 0:
            self._check(rc)
        self._keep["t"] = t
        self._keep["d6"] = d
        self.is_log = is_log

    def set_diffusion_phases(self, table_d6: TensorLike, phase: TensorLike, is_log: bool = False) -> None:
        """Tensor per material: table_d6 (nphase, 6) FP64 tensors (or logs), phase: one
        material index (uint8) per node, shape (nz, ny, nx) or flat."""
        tab = torch.as_tensor(table_d6, dtype=torch.float64).reshape(-1, 6)
        nphase = tab.shape[0]
        d = tab.t().contiguous().to(self.device)  # component planes of nphase entries
        ph = torch.as_tensor(phase)
        if ph.dtype != torch.uint8:
            raise ValueError("phase must be uint8")
        ph = ph.reshape(-1).contiguous().to(self.device)
        if ph.numel() != self.n:
            raise ValueError(f"expected {self.n} material indices, got {ph.numel()}")
        t = torch.empty((nphase, 6), dtype=self.real, device=self.device)
        bad = ctypes.c_int64(-1)
        rc = self.lib.elbm_set_diffusion_phases(self._h, _ptr(d), _nb(d), nphase, int(is_log), _ptr(ph),
                                                _nb(ph), _ptr(t), _nb(t), ctypes.byref(bad))
        if rc < 0:
            self.bad_index = bad.value
            self._check(rc)
        self._keep["t"] = t
        self._keep["phase"] = ph
        self._keep.pop("d6", None)
        self.is_log = is_log

    def set_velocity(self, u: TensorLike) -> None:
        if _numel(u) == 3:
            arr = (ctypes.c_double * 3)(*[float(v) for v in np.asarray(torch.as_tensor(u).cpu())])
            self._check(self.lib.elbm_set_velocity_uniform(self._h, arr))
            self._keep.pop("u", None)
            return
        d = self._dev64(u, 3)
        us = self._field(3)
        bad = ctypes.c_int64(-1)
        self._check(self.lib.elbm_set_velocity_field(self._h, _ptr(d), _nb(d), _ptr(us), _nb(us),
                                                     ctypes.byref(bad)))
        self._keep["u"] = us

    @property
    def has_source(self) -> bool:
        return self._has_source

    def set_source(self, r: Optional[Union[float, TensorLike]]) -> None:
        self._has_source = r is not None
        if r is None:
            self._check(self.lib.elbm_clear_source(self._h))
            self._keep.pop("r", None)
        elif np.ndim(r) == 0:
            self._check(self.lib.elbm_set_source_uniform(self._h, float(r)))
            self._keep.pop("r", None)
        else:
            d = self._dev64(r, None)
            rs = self._field(1)
            self._check(self.lib.elbm_set_source_field(self._h, _ptr(d), _nb(d), _ptr(rs), _nb(rs)))
            self._keep["r"] = rs

    def set_source_scale(self, s: float) -> None:
        """Amplitude s of the source for the following steps: R(x, t_{n+1/2}) = s R(x)."""
        self._check(self.lib.elbm_set_source_scale(self._h, float(s)))

    def set_dirichlet(self, phi_lo: float, phi_hi: float) -> None:
        self._check(self.lib.elbm_set_dirichlet(self._h, float(phi_lo), float(phi_hi)))

    # -- state -----------------------------------------------------------------------------
    def init_equilibrium(self, phi0: TensorLike, j0: Optional[TensorLike] = None) -> None:
        p = self._dev64(phi0, None)
        j = None if j0 is None else self._dev64(j0, 3)
        self._check(self.lib.elbm_init_equilibrium(self._h, _ptr(p), _nb(p), _ptr(j), _nb(j)))

    def step(self, n: int = 1) -> None:
        self._check(self.lib.elbm_step(self._h, int(n)))

    def step_record(self, n: int, lam: torch.Tensor, branch: torch.Tensor) -> None:
        """Step n times recording lambda (n * nodes, working precision) and the fallback
        branch (n * nodes, uint8) into caller tensors."""
        self._need(lam, "lam", n * self.n, self.real)
        self._need(branch, "branch", n * self.n, torch.uint8)
        self._check(self.lib.elbm_step_record(self._h, int(n), _ptr(lam), _nb(lam), _ptr(branch), _nb(branch)))

    def step_buffers(self, src: torch.Tensor, pending: int, dst: torch.Tensor,
                     lam: Optional[torch.Tensor] = None, branch: Optional[torch.Tensor] = None) -> None:
        """One step from the raw buffer src (with its pending flag) into dst; the lattice's
        own state is untouched."""
        self._need(src, "src", self.pop_bytes, torch.uint8)
        self._need(dst, "dst", self.pop_bytes, torch.uint8)
        self._need(lam, "lam", self.n, self.real, optional=True)
        self._need(branch, "branch", self.n, torch.uint8, optional=True)
        self._check(self.lib.elbm_step_buffers(self._h, _ptr(src), _nb(src), int(pending), _ptr(dst), _nb(dst),
                                               _ptr(lam), _nb(lam), _ptr(branch), _nb(branch)))

    @property
    def time(self) -> int:
        return int(self.lib.elbm_time(self._h))

    def moments(self):
        """(phi (nz, ny, nx), q (3, nz, ny, nx)) as FP64 device tensors."""
        phi = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        q = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        self._check(self.lib.elbm_read_moments(self._h, _ptr(phi), _nb(phi), _ptr(q), _nb(q)))
        return phi, q

    def reduce(self) -> np.ndarray:
        """(sum phi, sum q_x, sum q_y, sum q_z) in FP64 (synchronous)."""
        out = (ctypes.c_double * 4)()
        self._check(self.lib.elbm_reduce(self._h, out))
        return np.array(list(out))

    def reduce_noalloc(self, out: torch.Tensor) -> None:
        """The four FP64 sums of reduce() written to the device tensor out (4 doubles) on the
        lattice's stream, without allocating or synchronising."""
        self._need(out, "out", 4, torch.float64)
        self._check(self.lib.elbm_reduce_noalloc(self._h, _ptr(out), _nb(out)))

    def min_population(self) -> float:
        """Smallest current population over all nodes and directions (FP64, synchronous)."""
        out = ctypes.c_double()
        self._check(self.lib.elbm_min_population(self._h, ctypes.byref(out)))
        return float(out.value)

    def stream_copy(self, src: torch.Tensor, dst: torch.Tensor) -> None:
        """The library's streaming copy of src into dst (same byte size, on the lattice's
        device), asynchronous on the lattice's stream: the bandwidth reference."""
        if src.device != self.device or dst.device != self.device or not src.is_contiguous() \
                or not dst.is_contiguous():
            raise ValueError("stream_copy: contiguous buffers on the lattice's device")
        self._check(self.lib.elbm_stream_copy(self._h, _ptr(src), _nb(src), _ptr(dst), _nb(dst)))

    def populations(self) -> torch.Tensor:
        """Pre-collision populations as FP64 (Q, nz, ny, nx), library velocity order."""
        f = torch.empty((self.q,) + self.shape, dtype=torch.float64, device=self.device)
        self._check(self.lib.elbm_get_populations(self._h, _ptr(f), _nb(f)))
        return f

    def set_populations(self, f: TensorLike) -> None:
        t = self._dev64(f, self.q)
        self._check(self.lib.elbm_set_populations(self._h, _ptr(t), _nb(t)))
        torch.cuda.current_stream(self.device).synchronize()

    def save_state(self, dst: Optional[torch.Tensor] = None):
        """Copy of the raw current buffer plus (step, pending) for a bitwise restore."""
        if dst is None:
            dst = torch.empty(self.pop_bytes, dtype=torch.uint8, device=self.device)
        self._need(dst, "dst", self.pop_bytes, torch.uint8)
        step = ctypes.c_int64()
        pend = ctypes.c_int32()
        self._check(self.lib.elbm_save_state(self._h, _ptr(dst), _nb(dst), ctypes.byref(step), ctypes.byref(pend)))
        return dst, int(step.value), int(pend.value)

    def load_state(self, src: torch.Tensor, step: int, pending: int) -> None:
        self._need(src, "src", self.pop_bytes, torch.uint8)
        self._check(self.lib.elbm_load_state(self._h, _ptr(src), _nb(src), int(step), int(pending)))

    # -- adjoint ---------------------------------------------------------------------------
    def adjoint_step(self, state: torch.Tensor, pending: int, lam: torch.Tensor,
                     branch: torch.Tensor, adj_in: torch.Tensor, adj_out: torch.Tensor,
                     t_grad: torch.Tensor) -> None:
        self._need(state, "state", self.pop_bytes, torch.uint8)
        self._need(lam, "lam", self.n, self.real)
        self._need(branch, "branch", self.n, torch.uint8)
        self._need(adj_in, "adj_in", self.q * self.n, self.real)
        self._need(adj_out, "adj_out", self.q * self.n, self.real)
        self._need(t_grad, "t_grad", 6 * self.n, self.real)
        self._check(self.lib.elbm_adjoint_step(self._h, _ptr(state), _nb(state), int(pending), _ptr(lam), _nb(lam),
                                               _ptr(branch), _nb(branch), _ptr(adj_in), _nb(adj_in),
                                               _ptr(adj_out), _nb(adj_out), _ptr(t_grad), _nb(t_grad)))

    def gradient_workspace_bytes(self, steps: int, ckpt: int) -> int:
        return self._check(self.lib.elbm_gradient_workspace_bytes(self._h, int(steps), int(ckpt)))

    def forward_record(self, steps: int, ckpt: int, workspace: torch.Tensor) -> None:
        self._need(workspace, "workspace", self.gradient_workspace_bytes(steps, ckpt), torch.uint8)
        self._check(self.lib.elbm_forward_record(self._h, int(steps), int(ckpt), _ptr(workspace), _nb(workspace)))

    def gradient(self, steps: int, ckpt: int, workspace: torch.Tensor, dphi_n: torch.Tensor,
                 t_grad: torch.Tensor, dphi0: Optional[torch.Tensor] = None,
                 dj0: Optional[torch.Tensor] = None) -> None:
        self._need(workspace, "workspace", self.gradient_workspace_bytes(steps, ckpt), torch.uint8)
        self._need(dphi_n, "dphi_n", self.n, torch.float64)
        self._need(t_grad, "t_grad", 6 * self.n, self.real)
        self._need(dphi0, "dphi0", self.n, torch.float64, optional=True)
        self._need(dj0, "dj0", 3 * self.n, torch.float64, optional=True)
        self._check(self.lib.elbm_gradient(self._h, int(steps), int(ckpt), _ptr(workspace), _nb(workspace),
                                           _ptr(dphi_n), _nb(dphi_n), _ptr(t_grad), _nb(t_grad),
                                           _ptr(dphi0), _nb(dphi0), _ptr(dj0), _nb(dj0)))

    def tensor_gradient(self, t_grad: torch.Tensor) -> torch.Tensor:
        """dL/dD (or dL/dL for a log field) from an accumulated dL/dT, FP64 (6, nz, ny, nx)."""
        if "d6" not in self._keep:
            raise RuntimeError("tensor_gradient needs a per-node tensor field (set_diffusion with a field)")
        self._need(t_grad, "t_grad", 6 * self.n, self.real)
        d6 = self._keep["d6"]
        out = torch.empty((6,) + self.shape, dtype=torch.float64, device=self.device)
        self._check(self.lib.elbm_tensor_gradient(self._h, _ptr(d6), _nb(d6), int(self.is_log), _ptr(t_grad),
                                                  _nb(t_grad), _ptr(out), _nb(out)))
        return out

    def initial_gradient(self, adj0: torch.Tensor, with_flux: bool = False):
        """dL/dphi0 (FP64 (nz, ny, nx)) and, if with_flux, dL/dj0 (FP64 (3, nz, ny, nx)) from
        dL/dg at the initial time (Q planes, working precision), for an equilibrium start
        under the current velocity."""
        adj0 = adj0.contiguous()
        if adj0.dtype != self.real or adj0.numel() != self.q * self.n:
            raise ValueError("adj0 must hold Q planes in the working precision")
        dphi = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        dj = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device) if with_flux else None
        self._check(self.lib.elbm_initial_gradient(self._h, _ptr(adj0), _nb(adj0), _ptr(dphi), _nb(dphi),
                                                   _ptr(dj), _nb(dj)))
        return (dphi, dj) if with_flux else dphi

    def counters(self) -> dict:
        c = _lib.Counters()
        self._check(self.lib.elbm_get_counters(self._h, ctypes.byref(c)))
        return dict(fallback_nodes=c.fallback_nodes, flagged_nodes=c.flagged_nodes,
                    nonfinite=c.nonfinite, guard_nodes=c.guard_nodes)

    def reset_counters(self) -> None:
        self._check(self.lib.elbm_reset_counters(self._h))


def from_problem(prob, precision: Optional[str] = None, device="cuda", phases: bool = False,
                 **kw) -> "Lattice":
    """Lattice set up from an inputs.Problem (tensor, velocity, source, walls, initial
    equilibrium). phases: give the tensor as a material table and per-node material index
    (problems whose meta holds "phase" and "d6_table") instead of a per-node field."""
    prec = precision or prob.precision
    lat = Lattice(prob.nx, prob.ny, prob.nz, precision=prec, bc_x=prob.bc_x,
                  phi_ref=prob.phi_ref, eps=prob.eps, device=device, **kw)
    if phases:
        lat.set_diffusion_phases(prob.meta["d6_table"], prob.meta["phase"], is_log=prob.tensor_is_log)
    else:
        lat.set_diffusion(prob.d6, is_log=prob.tensor_is_log)
    lat.set_velocity(prob.u)
    if prob.r is not None:
        lat.set_source(prob.r)
    if prob.bc_x == "dirichlet":
        lat.set_dirichlet(prob.phi_lo, prob.phi_hi)
    lat.init_equilibrium(prob.phi0)
    return lat
