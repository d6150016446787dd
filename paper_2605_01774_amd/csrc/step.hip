// Fused collide-and-stream step kernel and its adjoint (reverse) step kernel, D3Q19.
//
// Forward (one launch per time step): each thread owns one node x. It reads the 19
// pre-collision populations of x (coalesced: x is fastest in every plane), adds the
// pending source half-steps, collides in registers (node.h), and pushes post_i to
// x + c_i in the other buffer (periodic in y and z; periodic or anti-bounce-back on the x
// faces). Every stored value is read once and written once per step, so the kernel moves
// exactly 2 * 19 stored values per node plus the per-node fields it is given.
//
// Adjoint (one launch per reverse step): each thread gathers dL/dg_{t+1} from x + c_i (the
// transpose of the push), recomputes the node's collision from the saved state, applies
// the vector-Jacobian product and writes dL/dg_t at x; dL/dT is accumulated per node.
#include <hip/hip_runtime.h>

#include "args.h"

namespace elbm {

template <class ST, int UM, bool ROOT>
__global__ __launch_bounds__(256) void k_step(const StepArgs<typename Store<ST>::Real> a) {
    using Real = typename Store<ST>::Real;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int nxy = nx * ny;
    const int k = z * nxy + y * nx + x;
    const ST* src = static_cast<const ST*>(a.src);
    ST* dst = static_cast<ST*>(a.dst);

    Real d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = Store<ST>::load(src + (size_t)i * a.n + k, a.scale);

    NodeCoef<Real> c;
    node_coef<Real, UM>(a, k, c);
    if (a.has_src) {
        const Real R = (a.rfield ? a.rfield[k] : a.R) * a.src_mult;
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] += R * Real(weight(i)) * c.E[i];
    }

    Real post[Q];
    NodeOut<Real> o;
    collide<Real, ROOT>(d, c, a.phi_ref, a.eps, a.tau2, a.root_rho, post, o);

    if (a.lam_rec) {
        a.lam_rec[k] = o.lam;
        a.br_rec[k] = uint8_t(o.branch);
    }
    if (a.counters) {
        if (o.branch != 255) atomicAdd(a.counters + 0, 1ull);
        if (o.flagged) atomicAdd(a.counters + 1, 1ull);
        Real s = Real(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) s += d[i];
        if (!isfinite(s)) atomicAdd(a.counters + 2, 1ull);
    }

    // push streaming
    const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
    const int zm = (z == 0) ? nz - 1 : z - 1, zp = (z == nz - 1) ? 0 : z + 1;
    const int ox[3] = {xm, x, xp};
    const int oy[3] = {ym * nx, y * nx, yp * nx};
    const int oz[3] = {zm * nxy, z * nxy, zp * nxy};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const bool wall = a.abb && ((cx(i) == 1 && x == nx - 1) || (cx(i) == -1 && x == 0));
        if (wall) {
            // halfway anti-bounce-back: the population leaving through the Dirichlet plane
            // comes back as its opposite, g_opp = -post_i + 2 W_i phi_w
            const Real phw = (cx(i) == -1) ? a.phi_lo : a.phi_hi;
            Store<ST>::put(dst + (size_t)opp(i) * a.n + k,
                           -post[i] + Real(2.0 * weight(i)) * (phw - a.phi_ref), a.inv_scale);
        } else {
            const int dk = oz[cz(i) + 1] + oy[cy(i) + 1] + ox[cx(i) + 1];
            Store<ST>::put(dst + (size_t)i * a.n + dk, post[i], a.inv_scale);
        }
    }
}

template <class ST, int UM>
__global__ __launch_bounds__(256) void k_adjoint(const StepArgs<typename Store<ST>::Real> a) {
    using Real = typename Store<ST>::Real;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= a.nx || y >= a.ny) return;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int nxy = nx * ny;
    const int k = z * nxy + y * nx + x;
    const ST* state = static_cast<const ST*>(a.src);

    // gather dL/dpost from the destinations of the push (transpose of streaming)
    const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
    const int zm = (z == 0) ? nz - 1 : z - 1, zp = (z == nz - 1) ? 0 : z + 1;
    const int ox[3] = {xm, x, xp};
    const int oy[3] = {ym * nx, y * nx, yp * nx};
    const int oz[3] = {zm * nxy, z * nxy, zp * nxy};
    Real ph[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const bool wall = a.abb && ((cx(i) == 1 && x == nx - 1) || (cx(i) == -1 && x == 0));
        if (wall) {
            ph[i] = -a.adj_in[(size_t)opp(i) * a.n + k];
        } else {
            const int dk = oz[cz(i) + 1] + oy[cy(i) + 1] + ox[cx(i) + 1];
            ph[i] = a.adj_in[(size_t)i * a.n + dk];
        }
    }

    Real d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = Store<ST>::load(state + (size_t)i * a.n + k, a.scale);
    NodeCoef<Real> c;
    node_coef<Real, UM>(a, k, c);
    if (a.has_src) {
        const Real R = (a.rfield ? a.rfield[k] : a.R) * a.src_mult;
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] += R * Real(weight(i)) * c.E[i];
    }
    Real dd[Q], tg[6];
    collide_vjp<Real>(d, c, a.phi_ref, a.eps, a.tau2, a.lam_in[k], int(a.br_in[k]), ph, dd, tg);
#pragma unroll
    for (int i = 0; i < Q; ++i) a.adj_out[(size_t)i * a.n + k] = dd[i];
#pragma unroll
    for (int m = 0; m < 6; ++m) a.t_grad[(size_t)m * a.n + k] += tg[m];
}

// ------------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------------
template <class ST, int UM>
static hipError_t step_t(const elbm_lattice* h, const void* src, void* dst, double src_mult,
                         void* lam_rec, uint8_t* br_rec) {
    using Real = typename Store<ST>::Real;
    StepArgs<Real> a = make_args<Real>(h, src_mult);
    a.src = src;
    a.dst = dst;
    a.lam_rec = static_cast<Real*>(lam_rec);
    a.br_rec = br_rec;
    dim3 grid, block;
    grid_for(h, &grid, &block);
    if (h->cfg.root_rho >= 0)
        hipLaunchKernelGGL((k_step<ST, UM, true>), grid, block, 0, h->stream, a);
    else
        hipLaunchKernelGGL((k_step<ST, UM, false>), grid, block, 0, h->stream, a);
    return hipGetLastError();
}

template <class ST>
static hipError_t step_u(const elbm_lattice* h, const void* src, void* dst, double m, void* lr,
                         uint8_t* br) {
    switch (h->u_mode) {
        case 0: return step_t<ST, 0>(h, src, dst, m, lr, br);
        case 1: return step_t<ST, 1>(h, src, dst, m, lr, br);
        default: return step_t<ST, 2>(h, src, dst, m, lr, br);
    }
}

hipError_t launch_step(const elbm_lattice* h, const void* src, void* dst, double src_mult,
                       void* lam_rec, uint8_t* br_rec) {
    switch (h->cfg.precision) {
        case ELBM_F64: return step_u<double>(h, src, dst, src_mult, lam_rec, br_rec);
        case ELBM_F32: return step_u<float>(h, src, dst, src_mult, lam_rec, br_rec);
        case ELBM_BF16: return step_u<bf16s>(h, src, dst, src_mult, lam_rec, br_rec);
        default: return step_u<_Float16>(h, src, dst, src_mult, lam_rec, br_rec);
    }
}

template <class ST, int UM>
static hipError_t adj_t(const elbm_lattice* h, const void* state, double src_mult, const void* lam,
                        const uint8_t* br, const void* adj_in, void* adj_out, void* t_grad) {
    using Real = typename Store<ST>::Real;
    StepArgs<Real> a = make_args<Real>(h, src_mult);
    a.src = state;
    a.counters = nullptr;
    a.lam_in = static_cast<const Real*>(lam);
    a.br_in = br;
    a.adj_in = static_cast<const Real*>(adj_in);
    a.adj_out = static_cast<Real*>(adj_out);
    a.t_grad = static_cast<Real*>(t_grad);
    dim3 grid, block;
    grid_for(h, &grid, &block);
    hipLaunchKernelGGL((k_adjoint<ST, UM>), grid, block, 0, h->stream, a);
    return hipGetLastError();
}

template <class ST>
static hipError_t adj_u(const elbm_lattice* h, const void* s, double m, const void* l,
                        const uint8_t* b, const void* ai, void* ao, void* tg) {
    switch (h->u_mode) {
        case 0: return adj_t<ST, 0>(h, s, m, l, b, ai, ao, tg);
        case 1: return adj_t<ST, 1>(h, s, m, l, b, ai, ao, tg);
        default: return adj_t<ST, 2>(h, s, m, l, b, ai, ao, tg);
    }
}

hipError_t launch_adjoint(const elbm_lattice* h, const void* state, double src_mult,
                          const void* lam_rec, const uint8_t* br_rec, const void* adj_in,
                          void* adj_out, void* t_grad) {
    switch (h->cfg.precision) {
        case ELBM_F64: return adj_u<double>(h, state, src_mult, lam_rec, br_rec, adj_in, adj_out, t_grad);
        case ELBM_F32: return adj_u<float>(h, state, src_mult, lam_rec, br_rec, adj_in, adj_out, t_grad);
        case ELBM_BF16: return adj_u<bf16s>(h, state, src_mult, lam_rec, br_rec, adj_in, adj_out, t_grad);
        default: return adj_u<_Float16>(h, state, src_mult, lam_rec, br_rec, adj_in, adj_out, t_grad);
    }
}

}  // namespace elbm
