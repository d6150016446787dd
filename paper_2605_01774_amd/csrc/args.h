// Kernel argument block shared by the step, adjoint and auxiliary kernels, and the
// per-node equilibrium coefficients built from it.
#pragma once

#include <cmath>

#include "internal.h"
#include "node.h"

namespace elbm {

template <class Real>
struct StepArgs {
    const void* src;
    void* dst;
    int nx, ny, nz, abb;
    long long n;
    Real phi_ref, eps, tau2, root_rho;
    Real scale, inv_scale;
    Real T[6];
    const Real* tfield;
    Real u[3];
    const Real* ufield;
    Real E[Q], r[Q], l[Q];
    Real R;
    const Real* rfield;
    Real src_mult;
    int has_src;
    Real phi_lo, phi_hi;
    Real* lam_rec;
    uint8_t* br_rec;
    unsigned long long* counters;
    // adjoint only
    const Real* adj_in;
    Real* adj_out;
    Real* t_grad;
    const Real* lam_in;
    const uint8_t* br_in;
};

// Equilibrium factors at one node: UM = 0 zero velocity (constants fold), 1 uniform
// velocity (host-computed factors), 2 velocity field.
template <class Real, int UM>
__device__ __forceinline__ void node_coef(const StepArgs<Real>& a, int k, NodeCoef<Real>& c) {
    if constexpr (UM == 0) {
        c.u[0] = c.u[1] = c.u[2] = Real(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            c.E[i] = Real(1);
            c.r[i] = Real(1.0 / weight(i));
            c.l[i] = Real(0);
        }
    } else if constexpr (UM == 1) {
        c.u[0] = a.u[0];
        c.u[1] = a.u[1];
        c.u[2] = a.u[2];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            c.E[i] = a.E[i];
            c.r[i] = a.r[i];
            c.l[i] = a.l[i];
        }
    } else {
        c.u[0] = a.ufield[k];
        c.u[1] = a.ufield[a.n + k];
        c.u[2] = a.ufield[2 * a.n + k];
        const Real uu = c.u[0] * c.u[0] + c.u[1] * c.u[1] + c.u[2] * c.u[2];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const Real cu = Real(cx(i)) * c.u[0] + Real(cy(i)) * c.u[1] + Real(cz(i)) * c.u[2];
            c.E[i] = Real(1) + Real(3) * cu + Real(4.5) * cu * cu - Real(1.5) * uu;
            c.r[i] = Real(1) / (Real(weight(i)) * c.E[i]);
            c.l[i] = log(c.E[i]);
        }
    }
    if (a.tfield) {
#pragma unroll
        for (int m = 0; m < 6; ++m) c.T[m] = a.tfield[m * a.n + k];
    } else {
#pragma unroll
        for (int m = 0; m < 6; ++m) c.T[m] = a.T[m];
    }
}

template <class Real>
inline StepArgs<Real> make_args(const elbm_lattice* h, double src_mult) {
    StepArgs<Real> a{};
    a.nx = h->cfg.nx;
    a.ny = h->cfg.ny;
    a.nz = h->cfg.nz;
    a.abb = h->cfg.bc_x == ELBM_DIRICHLET;
    a.n = h->n;
    a.phi_ref = Real(h->cfg.phi_ref);
    a.eps = Real(h->cfg.eps);
    a.tau2 = Real(h->cfg.ghost_floor * h->cfg.ghost_floor);
    a.root_rho = Real(h->cfg.root_rho);
    const bool scaled = h->cfg.precision == ELBM_FP16;
    a.scale = Real(scaled ? h->cfg.store_scale : 1.0);
    a.inv_scale = Real(scaled ? 1.0 / h->cfg.store_scale : 1.0);
    for (int m = 0; m < 6; ++m) a.T[m] = Real(h->T_u[m]);
    a.tfield = h->t_field_mode ? static_cast<const Real*>(h->t_field) : nullptr;
    for (int m = 0; m < 3; ++m) a.u[m] = Real(h->u_mode == 1 ? h->u_u[m] : 0.0);
    a.ufield = h->u_mode == 2 ? static_cast<const Real*>(h->u_field) : nullptr;
    const double* u = h->u_u;
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        const double cu = cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2];
        const double E = (h->u_mode == 1) ? 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu : 1.0;
        a.E[i] = Real(E);
        a.r[i] = Real(1.0 / (weight(i) * E));
        a.l[i] = Real(std::log(E));
    }
    a.has_src = h->r_mode != 0;
    a.R = Real(h->r_mode == 1 ? h->r_u : 0.0);
    a.rfield = h->r_mode == 2 ? static_cast<const Real*>(h->r_field) : nullptr;
    a.src_mult = Real(src_mult);
    a.phi_lo = Real(h->phi_lo);
    a.phi_hi = Real(h->phi_hi);
    a.counters = h->d_cnt;
    return a;
}

inline void grid_for(const elbm_lattice* h, dim3* grid, dim3* block, int max_bx = 512) {
    // A block owns whole x-rows when they fit (up to 512 nodes): the x-shifted pushes then
    // stay inside the block's own cache lines, so no line is written by two blocks (which
    // may sit on different XCDs with separate L2s). Short rows are stacked in y.
    const int nx = h->cfg.nx;
    int bx;
    if (nx <= 32) bx = 32;
    else if (nx <= max_bx) bx = ((nx + 63) / 64) * 64;
    else bx = max_bx;
    int by = bx >= 256 ? 1 : 256 / bx;
    if (by > h->cfg.ny) by = h->cfg.ny;
    *block = dim3(bx, by, 1);
    *grid = dim3((nx + bx - 1) / bx, (h->cfg.ny + by - 1) / by, h->cfg.nz);
}

}  // namespace elbm
