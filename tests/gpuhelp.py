"""Helpers shared by the GPU tests: run a Problem through the HIP library and through the
oracle, and compare populations matched by velocity vector."""
import numpy as np

import oracle


def perm_lib_to_oracle(q=19):
    """Index list p with lib_population[p[i]] == oracle_population[i] (matched by c)."""
    from paper_2605_01774_amd import _lib
    c_lib, _ = _lib.velocity_table(q)
    c_or, _ = oracle.velocities(q)
    return [int(np.nonzero((c_lib == c_or[i]).all(axis=1))[0][0]) for i in range(q)]


def gpu_lattice(prob, precision=None, **kw):
    from paper_2605_01774_amd import lattice
    return lattice.from_problem(prob, precision=precision, device="cuda:0", **kw)


def gpu_pops(lat):
    """Populations in oracle order as FP64 numpy."""
    return lat.populations().cpu().numpy()[perm_lib_to_oracle(lat.q)]


def to_lib_order(f_or):
    q = f_or.shape[0]
    p = perm_lib_to_oracle(q)
    out = np.empty_like(f_or)
    for i in range(q):
        out[p[i]] = f_or[i]
    return out


def rel_err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def banner(msg):
    print(f"\n[gpu] {msg}", flush=True)


def sampled_next_step(lat, prob, samples, f_now):
    """Oracle prediction of the next-step populations at sampled nodes, from the current
    GPU state f_now (FP64 torch tensor (Q, nz, ny, nx) in library order).

    For each sample x and direction j the oracle collides the upstream node x - c_j (its Q
    populations gathered from f_now, plus the first source half-step) and takes direction
    j, or applies the anti-bounce-back rule at Dirichlet planes, then adds the second
    source half-step. Returns (values (S, Q) in oracle order, node indices)."""
    import torch
    q = lat.q
    c_or, w_or = oracle.velocities(q)
    p = perm_lib_to_oracle(q)
    nz, ny, nx = prob.nz, prob.ny, prob.nx
    sz, sy, sx = samples
    S = len(sx)
    # upstream nodes, periodic in y, z (x handled below)
    ux = sx[:, None] - c_or[None, :, 0]
    uy = (sy[:, None] - c_or[None, :, 1]) % ny
    uz = (sz[:, None] - c_or[None, :, 2]) % nz
    wall = (ux < 0) | (ux >= nx)
    if prob.bc_x == "periodic":
        ux = ux % nx
        wall[:] = False
    uxc = np.clip(ux, 0, nx - 1)
    # gather the upstream nodes' populations (library order -> oracle order)
    idx = torch.as_tensor(((uz * ny + uy) * nx + uxc).reshape(-1), device=f_now.device)
    g = f_now.reshape(q, -1)[:, idx].cpu().numpy()[p].T              # (S*q, q) oracle order
    own = torch.as_tensor(((sz * ny + sy) * nx + sx), device=f_now.device)
    g_own = f_now.reshape(q, -1)[:, own].cpu().numpy()[p].T          # (S, q)

    def field(a, comps, nodes):
        if isinstance(a, torch.Tensor):  # inputs generated on the GPU: gather there
            if a.ndim == 1:
                return a.cpu().numpy()
            idx = torch.as_tensor(np.asarray(nodes), device=a.device)
            return a.reshape(comps, -1)[:, idx].T.cpu().numpy()
        a = np.asarray(a)
        if a.ndim == 1:
            return a
        return a.reshape(comps, -1)[:, nodes].T

    up_nodes = ((uz * ny + uy) * nx + uxc).reshape(-1)
    own_nodes = (sz * ny + sy) * nx + sx

    def with_half_source(gg, nodes):
        if prob.r is None:
            return gg
        R = np.asarray(prob.r) if np.ndim(prob.r) == 0 else field(prob.r, 1, nodes)[:, 0]
        U = field(prob.u, 3, nodes)
        if U.ndim == 1:
            U = np.broadcast_to(U, (len(nodes), 3))
        cu = U @ c_or.T
        uu = (U * U).sum(1)[:, None]
        E = w_or[None, :] * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * uu)
        return gg + 0.5 * np.asarray(R).reshape(-1, 1) * E

    g = with_half_source(g, up_nodes)
    g_own = with_half_source(g_own, own_nodes)
    # the oracle takes the lattice's own ghost floor (a parameter of the scheme)
    kw = dict(eps=prob.eps, tensor_is_log=prob.tensor_is_log, tau=float(lat.cfg.ghost_floor), q=q)
    post_up, _ = oracle.collide(g, field(prob.d6, 6, up_nodes), field(prob.u, 3, up_nodes), **kw)
    post_own, _ = oracle.collide(g_own, field(prob.d6, 6, own_nodes), field(prob.u, 3, own_nodes), **kw)
    post_up = post_up.reshape(S, q, q)
    out = np.empty((S, q))
    opp = [int(np.nonzero((c_or == -c_or[j]).all(axis=1))[0][0]) for j in range(q)]
    for j in range(q):
        out[:, j] = post_up[:, j, j]
        wj = wall[:, j]
        if wj.any():
            phw = np.where(ux[:, j] < 0, prob.phi_lo, prob.phi_hi)
            out[wj, j] = -post_own[wj, opp[j]] + 2.0 * w_or[j] * phw[wj]
    out = with_half_source(out, own_nodes)
    return out, own_nodes
