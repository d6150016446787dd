"""Helpers shared by the GPU tests: run a Problem through the HIP library and through the
oracle, and compare populations matched by velocity vector."""
import numpy as np

import oracle


def perm_lib_to_oracle():
    """Index list p with lib_population[p[i]] == oracle_population[i] (matched by c)."""
    from paper_2605_01774_amd import _lib
    c_lib, _ = _lib.velocity_table()
    c_or, _ = oracle.velocities(19)
    return [int(np.nonzero((c_lib == c_or[i]).all(axis=1))[0][0]) for i in range(19)]


def gpu_lattice(prob, precision=None, **kw):
    from paper_2605_01774_amd import lattice
    return lattice.from_problem(prob, precision=precision, device="cuda:0", **kw)


def gpu_pops(lat):
    """Populations in oracle order as FP64 numpy."""
    return lat.populations().cpu().numpy()[perm_lib_to_oracle()]


def to_lib_order(f_or):
    p = perm_lib_to_oracle()
    out = np.empty_like(f_or)
    for i in range(19):
        out[p[i]] = f_or[i]
    return out


def rel_err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def banner(msg):
    print(f"\n[gpu] {msg}", flush=True)
