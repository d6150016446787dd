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
    const Real* tfield;     // 6 values per row, node-major
    const uint8_t* phase;   // material index per node (row of tfield), or null: row = node
    int phase_max;          // largest valid material index
    Real u[3];
    const Real* ufield;
    Real ex[Q], r[Q], l[Q];  // E_i - 1, 1 / (W_i E_i), ln E_i of a uniform velocity
    Real R;
    const Real* rfield;
    Real src_mult;
    int has_src;
    Real phi_lo, phi_hi;
    int rest32;     // 16-bit forms: rest population in FP32 absorbing the rounding residuals
    int sround;     // 16-bit forms: stochastic rounding of the stores
    uint32_t tmix;  // hash of the time step, mixed into the rounding counters
    int xcd_remap;  // row-vector kernel: XCD slab block order (xcd_block)
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

// Per-node retention tensor, stored node-major (6 values of node k at 6 k): three
// 2-wide loads per node, so the field is one contiguous stream instead of six planes.
__device__ __forceinline__ void load_t6(const float* tf, long long k, float (&T)[6]) {
    const float2* p = reinterpret_cast<const float2*>(tf + 6 * k);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const float2 v = p[m];
        T[2 * m] = v.x;
        T[2 * m + 1] = v.y;
    }
}
__device__ __forceinline__ void load_t6(const double* tf, long long k, double (&T)[6]) {
    const double2* p = reinterpret_cast<const double2*>(tf + 6 * k);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const double2 v = p[m];
        T[2 * m] = v.x;
        T[2 * m + 1] = v.y;
    }
}

// Accumulate 6 values into node k's slot of a node-major 6-vector field (dL/dT), with the
// same three 2-wide accesses, nontemporal (each slot is read and written once per reverse
// step).
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void add_t6(float* tf, long long k, const float (&v)[6]) {
    nt_f2* p = reinterpret_cast<nt_f2*>(tf + 6 * k);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        nt_f2 w = __builtin_nontemporal_load(p + m);
        w.x += v[2 * m];
        w.y += v[2 * m + 1];
        __builtin_nontemporal_store(w, p + m);
    }
}
__device__ __forceinline__ void add_t6(double* tf, long long k, const double (&v)[6]) {
    nt_d2* p = reinterpret_cast<nt_d2*>(tf + 6 * k);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        nt_d2 w = __builtin_nontemporal_load(p + m);
        w.x += v[2 * m];
        w.y += v[2 * m + 1];
        __builtin_nontemporal_store(w, p + m);
    }
}

// Row of the tensor store that holds node k's T: the node itself for a per-node field, its
// material (clamped to the table) for a material table.
template <class Real>
__device__ __forceinline__ long long tensor_row(const StepArgs<Real>& a, long long k) {
    if (a.phase) return min(int(a.phase[k]), a.phase_max);
    return k;
}

// Equilibrium factors at one node: UM = 0 zero velocity (constants fold), 1 uniform
// velocity (host-computed factors), 2 velocity field (the node's velocity u0, u1, u2).
template <class Real, int UM>
__device__ __forceinline__ void coef_velocity(const StepArgs<Real>& a, Real u0, Real u1, Real u2,
                                              NodeCoef<Real>& c) {
    if constexpr (UM == 0) {
        c.u[0] = c.u[1] = c.u[2] = Real(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            c.ex[i] = Real(0);
            c.r[i] = Real(1.0 / weight(i));
            c.l[i] = Real(0);
        }
    } else if constexpr (UM == 1) {
        c.u[0] = a.u[0];
        c.u[1] = a.u[1];
        c.u[2] = a.u[2];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            c.ex[i] = a.ex[i];
            c.r[i] = a.r[i];
            c.l[i] = a.l[i];
        }
    } else {
        c.u[0] = u0;
        c.u[1] = u1;
        c.u[2] = u2;
        const Real uu = c.u[0] * c.u[0] + c.u[1] * c.u[1] + c.u[2] * c.u[2];
        c.ex[0] = -Real(1.5) * uu;
        rest_factors(c.ex[0], c.r[0], c.l[0]);
#pragma unroll
        for (int P = 1; P < Q; P += 2) {
            // opposite pair: E+- = 1 + a +- b with a = 4.5 (c.u)^2 - 1.5 u.u, b = 3 c.u; the
            // excesses a +- b are formed without the 1 so that they keep their relative
            // precision (the equilibrium only needs E - 1)
            const Real cu = cdot(P, c.u[0], c.u[1], c.u[2]);
            const Real ea = Real(4.5) * cu * cu - Real(1.5) * uu;
            const Real eb = Real(3) * cu;
            c.ex[P] = ea + eb;
            c.ex[P + 1] = ea - eb;
            pair_factors(P, c.ex[P], c.ex[P + 1], c.r[P], c.r[P + 1], c.l[P], c.l[P + 1]);
        }
    }
}

template <class Real, int UM>
__device__ __forceinline__ void node_coef(const StepArgs<Real>& a, int k, NodeCoef<Real>& c) {
    if constexpr (UM == 2)
        coef_velocity<Real, UM>(a, a.ufield[k], a.ufield[a.n + k], a.ufield[2 * a.n + k], c);
    else
        coef_velocity<Real, UM>(a, Real(0), Real(0), Real(0), c);
    if (a.tfield) {
        load_t6(a.tfield, tensor_row(a, k), c.T);
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
    a.phase = h->t_field_mode == 2 ? h->t_phase : nullptr;
    a.phase_max = h->nphase - 1;
    for (int m = 0; m < 3; ++m) a.u[m] = Real(h->u_mode == 1 ? h->u_u[m] : 0.0);
    a.ufield = h->u_mode == 2 ? static_cast<const Real*>(h->u_field) : nullptr;
    const double* u = h->u_u;
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        const double cu = cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2];
        const double ex = (h->u_mode == 1) ? 3.0 * cu + 4.5 * cu * cu - 1.5 * uu : 0.0;
        const double E = 1.0 + ex;
        a.ex[i] = Real(ex);
        a.r[i] = Real(1.0 / (weight(i) * E));
        a.l[i] = Real(std::log(E));
    }
    a.has_src = h->r_mode != 0;
    a.R = Real(h->r_mode == 1 ? h->r_u : 0.0);
    a.rfield = h->r_mode == 2 ? static_cast<const Real*>(h->r_field) : nullptr;
    a.src_mult = Real(src_mult);
    a.rest32 = (h->cfg.flags & ELBM_FLAG_REST_FP32) ? 1 : 0;
    a.sround = (h->cfg.flags & ELBM_FLAG_STOCHASTIC_ROUNDING) ? 1 : 0;
    a.tmix = pcg_hash(uint32_t(h->time) ^ 0x9E3779B9u);
    a.xcd_remap = 0;
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
