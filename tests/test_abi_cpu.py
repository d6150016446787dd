"""The C ABI without a GPU: both built libraries (D3Q19 libelbm.so, D3Q27 libelbm27.so)
load and export every entry point that include/elbm.h declares, the ctypes binding agrees
with the header's declarations and struct layouts, the velocity tables are the D3Q19 and
D3Q27 sets (matched by vector against the oracle's own tables), and configuration errors
are rejected before any device call.

These tests need the built library (python __graft_entry__.py build, or
python paper_2605_01774_amd/build.py); no compute call is made.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_2605_01774_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "elbm.h")


def _declared():
    """(name, return type text) of every function prototype in the header."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for m in re.finditer(r"^([A-Za-z_][\w \*]*?)\s*\b(elbm_\w+)\s*\(", text, flags=re.M):
        out[m.group(2)] = m.group(1).strip()
    return out


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libelbm.so is not built: run python __graft_entry__.py or the package build.py")
    return _lib.load()


@pytest.fixture(scope="module", params=[19, 27])
def anylib(request):
    path = _lib.LIB_PATHS[request.param]
    if not os.path.exists(path):
        pytest.fail(f"{path} is not built: run the package build.py")
    return request.param, path


def test_header_declares_the_expected_entry_points():
    names = set(_declared())
    assert len(names) == 40
    for must in ("elbm_create", "elbm_step", "elbm_read_moments", "elbm_reduce", "elbm_min_population",
                 "elbm_adjoint_step", "elbm_tensor_gradient", "elbm_initial_gradient",
                 "elbm_set_diffusion_field", "elbm_set_diffusion_phases",
                 "elbm_set_velocity_field", "elbm_set_source_field", "elbm_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(anylib):
    q, path = anylib
    raw = ctypes.CDLL(path)
    for name in _declared():
        assert hasattr(raw, name), f"{name} declared in elbm.h but not exported"
    # and as C symbols (no C++ mangling), in the dynamic symbol table
    nm = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True,
                        text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in nm.splitlines() if " T " in ln}
    missing = set(_declared()) - exported
    assert not missing, missing


def test_binding_matches_header():
    declared = _declared()
    bound = {name: (res, args) for name, res, args in _lib.SIGNATURES}
    assert set(bound) == set(declared)
    ret_map = {"int": ctypes.c_int, "int64_t": ctypes.c_int64, "const char*": ctypes.c_char_p}
    for name, rtype in declared.items():
        assert bound[name][0] is ret_map[rtype.replace(" *", "*")], name
    # argument counts agree with the prototypes
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    for name in declared:
        m = re.search(rf"\b{name}\s*\(([^)]*)\)", text)
        args = [a for a in m.group(1).split(",") if a.strip() and a.strip() != "void"]
        assert len(args) == len(bound[name][1]), name


# host pointers of the interface (everything else that is a pointer is a caller-owned device
# buffer and must come with its byte size)
HOST_POINTERS = {"elbm_create": {"cfg", "out"}, "elbm_velocity_table": {"c", "w"},
                 "elbm_reduce": {"out4"}, "elbm_min_population": {"out"},
                 "elbm_get_counters": {"out"}, "elbm_set_diffusion_uniform": {"d6"},
                 "elbm_set_velocity_uniform": {"u3"}, "elbm_save_state": {"step", "pending"},
                 "elbm_set_stream": {"stream"}}  # a hipStream_t handle, not a buffer
HOST_OUTPUTS = {"bad_node", "bad"}  # first offending node / entry (host, optional)


def _params(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(rf"\b{name}\s*\(([^)]*)\)", text)
    out = []
    for a in m.group(1).split(","):
        a = " ".join(a.split())
        if not a or a == "void":
            continue
        pname = re.findall(r"\w+", a)[-1]
        out.append((a[: -len(pname)].strip(), pname))
    return out


def test_every_device_buffer_comes_with_its_byte_size():
    """Every caller-owned device buffer in the interface is followed by an int64_t
    <name>_bytes argument, which the library checks (ESHAPE if too small)."""
    checked = 0
    for name in _declared():
        ps = _params(name)
        for k, (ptype, pname) in enumerate(ps):
            if "*" not in ptype or "elbm_lattice" in ptype or "elbm_config" in ptype:
                continue
            if pname in HOST_POINTERS.get(name, ()) or pname in HOST_OUTPUTS:
                continue
            assert k + 1 < len(ps), (name, pname)
            assert ps[k + 1] == ("int64_t", pname + "_bytes"), (name, pname, ps[k + 1])
            checked += 1
    assert checked >= 40


def test_struct_layouts_match_header(tmp_path):
    """sizeof/offsetof of elbm_config and elbm_counters as a C compiler sees the header."""
    fields = [f for f, _ in _lib.Config._fields_]
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "elbm.h"', 'int main(void){',
           'printf("%zu\\n", sizeof(elbm_config));']
    src += [f'printf("%zu\\n", offsetof(elbm_config, {f}));' for f in fields]
    src += ['printf("%zu\\n", sizeof(elbm_counters));', 'return 0;}']
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)],
                   check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(_lib.Config)
    for f, off in zip(fields, vals[1:-1]):
        assert getattr(_lib.Config, f).offset == off, f
    assert vals[-1] == ctypes.sizeof(_lib.Counters)


def test_velocity_table_matches_oracle_set(anylib):
    q, _ = anylib
    c, w = _lib.velocity_table(q)
    assert c.shape == (q, 3)
    c_or, w_or = oracle.velocities(q)
    # the same set of (vector, weight) pairs as the oracle's independent table
    for i in range(q):
        j = np.nonzero((c_or == c[i]).all(axis=1))[0]
        assert len(j) == 1
        assert w[i] == w_or[j[0]]
    # opposite pairs (i, i + 1) for odd i; rest velocity first
    assert (c[0] == 0).all()
    for i in range(1, q, 2):
        assert (c[i] == -c[i + 1]).all()


def _cfg(**kw):
    base = dict(nx=8, ny=8, nz=8, precision=1, bc_x=0, flags=0, phi_ref=1.0, eps=0.0,
                ghost_floor=1e-5, root_rho=-1.0, store_scale=1.0)
    base.update(kw)
    return _lib.Config(**base)


@pytest.mark.parametrize("bad,fragment", [
    (dict(nx=0), "grid sizes"),
    (dict(nz=-3), "grid sizes"),
    (dict(nx=2048, ny=1024, nz=1024), "2^31"),
    (dict(precision=7), "precision"),
    (dict(bc_x=5), "bc_x"),
    (dict(flags=1 << 12), "flag"),
    (dict(flags=3 << 4), "vector width"),
    (dict(eps=-1.0), "eps"),
    (dict(eps=float("nan")), "eps"),
    (dict(ghost_floor=-1e-5), "ghost_floor"),
    (dict(phi_ref=float("inf")), "non-finite"),
    (dict(precision=3, store_scale=0.3), "power of two"),
    (dict(precision=3, store_scale=0.0), "power of two"),
])
def test_create_rejects_bad_config_before_any_device_call(lib, bad, fragment):
    h = ctypes.c_void_p(123)
    cfg = _cfg(**bad)
    rc = lib.elbm_create(ctypes.byref(cfg), ctypes.byref(h))
    assert rc == -1
    assert h.value is None
    assert fragment in lib.elbm_last_error().decode()


def test_null_handles_are_errors_not_crashes(lib):
    assert lib.elbm_destroy(None) == 0
    assert lib.elbm_create(None, None) == -1
    assert lib.elbm_population_bytes(None) == -1
    assert lib.elbm_step(None, 1) == -1
    assert lib.elbm_reduce(None, None) == -1
    assert lib.elbm_velocity_table(None, None) == -1
    assert "null" in lib.elbm_last_error().decode()
