"""MI355X-native entropic lattice Boltzmann solver for full-tensor anisotropic
advection-diffusion (D3Q19), after Feng, Leng, Jiang, Chu, arXiv 2605.01774.

The numerical work runs in the HIP library libelbm.so (C ABI: include/elbm.h); this package
is its Python binding. `inputs` builds seeded synthetic workloads and holds no scheme
arithmetic. Heavy imports (torch, the shared library) happen on first use.
"""
import importlib

__all__ = ["Lattice", "from_problem", "velocity_table", "inputs"]


def __getattr__(name):
    if name in ("Lattice", "from_problem"):
        return getattr(importlib.import_module(".lattice", __name__), name)
    if name == "velocity_table":
        return importlib.import_module("._lib", __name__).velocity_table
    if name in ("inputs", "lattice", "autograd"):
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
