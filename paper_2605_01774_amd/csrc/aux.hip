// Set-up, readout and reduction kernels around the step kernel.
//
//  - tensor fields: D (or L with D = expm(L)) -> retention tensor T = 2 I - S = 12 D (I+6D)^-1,
//    with S = (I/2 + D/cs^2)^-1 of Sec. 2.3, in FP64; SPD check per node
//  - velocity and source fields: validation and conversion to the working precision
//  - initialisation g = g_eq(phi0, u) + P(j0)                       (Sec. 2.1, 2.2)
//  - readout phi = sum g, q = (I - S/2) j = T j / 2                  (Sec. 4.2.2)
//  - FP64 global sums with per-thread compensated accumulation
//  - the chain rule dL/dT -> dL/dD (-> dL/dL through the Daleckii-Krein formula)
#include <hip/hip_runtime.h>

#include "args.h"

namespace elbm {

int store_bytes(int precision) {
    switch (precision) {
        case ELBM_F64: return 8;
        case ELBM_F32: return 4;
        default: return 2;
    }
}

static inline unsigned blocks_for(long long n, int bs) { return unsigned((n + bs - 1) / bs); }

// ------------------------------------------------------------------------------------------
// 3x3 symmetric helpers (FP64)
// ------------------------------------------------------------------------------------------
__device__ inline void sym_load(const double* p6, double M[3][3]) {
    M[0][0] = p6[0]; M[0][1] = M[1][0] = p6[1]; M[0][2] = M[2][0] = p6[2];
    M[1][1] = p6[3]; M[1][2] = M[2][1] = p6[4]; M[2][2] = p6[5];
}

__device__ inline void inv3(const double M[3][3], double R[3][3]) {
    const double a0 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
    const double a1 = M[0][2] * M[2][1] - M[0][1] * M[2][2];
    const double a2 = M[0][1] * M[1][2] - M[0][2] * M[1][1];
    const double det = M[0][0] * a0 + M[1][0] * a1 + M[2][0] * a2;
    const double id = 1.0 / det;
    R[0][0] = a0 * id;
    R[0][1] = a1 * id;
    R[0][2] = a2 * id;
    R[1][0] = (M[1][2] * M[2][0] - M[1][0] * M[2][2]) * id;
    R[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) * id;
    R[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) * id;
    R[2][0] = (M[1][0] * M[2][1] - M[1][1] * M[2][0]) * id;
    R[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) * id;
    R[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) * id;
}

__device__ inline void mul3(const double A[3][3], const double B[3][3], double C[3][3]) {
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) C[r][c] = A[r][0] * B[0][c] + A[r][1] * B[1][c] + A[r][2] * B[2][c];
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix: A = V diag(w) V^T.
__device__ inline void eig3(const double Ain[3][3], double V[3][3], double w[3]) {
    double A[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            A[r][c] = Ain[r][c];
            V[r][c] = (r == c) ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 16; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= 1e-36 * dia || off == 0.0) break;
        for (int pq = 0; pq < 3; ++pq) {
            const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
            if (A[p][q] == 0.0) continue;
            const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
            for (int k = 0; k < 3; ++k) {  // A <- A J (columns p, q)
                const double akp = A[k][p], akq = A[k][q];
                A[k][p] = c * akp - s * akq;
                A[k][q] = s * akp + c * akq;
            }
            for (int k = 0; k < 3; ++k) {  // A <- J^T A (rows p, q)
                const double apk = A[p][k], aqk = A[q][k];
                A[p][k] = c * apk - s * aqk;
                A[q][k] = s * apk + c * aqk;
            }
            for (int k = 0; k < 3; ++k) {
                const double vkp = V[k][p], vkq = V[k][q];
                V[k][p] = c * vkp - s * vkq;
                V[k][q] = s * vkp + c * vkq;
            }
        }
    }
    for (int k = 0; k < 3; ++k) w[k] = A[k][k];
}

// D (or D = expm(L)) at one node, FP64, and whether it is SPD and finite.
__device__ inline bool node_tensor(const double* d6, long long n, long long k, int is_log, double D[3][3],
                                   double V[3][3], double ev[3]) {
    double p6[6];
    for (int m = 0; m < 6; ++m) p6[m] = d6[m * n + k];
    double M[3][3];
    sym_load(p6, M);
    bool finite = true;
    for (int m = 0; m < 6; ++m) finite = finite && isfinite(p6[m]);
    if (!finite) return false;
    if (is_log) {
        double l[3];
        eig3(M, V, l);
        for (int a = 0; a < 3; ++a) ev[a] = exp(l[a]);
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                D[r][c] = V[r][0] * ev[0] * V[c][0] + V[r][1] * ev[1] * V[c][1] + V[r][2] * ev[2] * V[c][2];
        return ev[0] > 0 && ev[1] > 0 && ev[2] > 0;
    }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) D[r][c] = M[r][c];
    // Cholesky test of positive definiteness
    const double l00 = M[0][0];
    if (!(l00 > 0)) return false;
    const double l10 = M[1][0] / sqrt(l00), l20 = M[2][0] / sqrt(l00);
    const double p11 = M[1][1] - l10 * l10;
    if (!(p11 > 0)) return false;
    const double l21 = (M[2][1] - l20 * l10) / sqrt(p11);
    const double p22 = M[2][2] - l20 * l20 - l21 * l21;
    return p22 > 0;
}

template <class Real>
__global__ void k_tensor_field(const double* d6, int is_log, long long n, Real* t, long long* bad) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double D[3][3], V[3][3], ev[3];
    const bool ok = node_tensor(d6, n, k, is_log, D, V, ev);
    if (!ok) atomicMin(bad, k);
    // T = 12 D (I + 6 D)^-1 (commuting factors), symmetrised
    double M[3][3], Mi[3][3], T[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[r][c] = (r == c ? 1.0 : 0.0) + 6.0 * D[r][c];
    inv3(M, Mi);
    mul3(D, Mi, T);
    const double t6[6] = {12.0 * T[0][0], 6.0 * (T[0][1] + T[1][0]), 6.0 * (T[0][2] + T[2][0]),
                          12.0 * T[1][1], 6.0 * (T[1][2] + T[2][1]), 12.0 * T[2][2]};
    for (int m = 0; m < 6; ++m) t[6 * k + m] = ok ? Real(t6[m]) : Real(0);  // node-major
}

__global__ void k_phase_check(const uint8_t* phase, long long n, int nphase, long long* bad) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (int(phase[k]) >= nphase) atomicMin(bad, k);
}

template <class Real>
__global__ void k_velocity_field(const double* u3, long long n, Real* us, long long* bad) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double u0 = u3[k], u1 = u3[n + k], u2 = u3[2 * n + k];
    const double uu = u0 * u0 + u1 * u1 + u2 * u2;
    bool ok = isfinite(uu);
    for (int i = 0; i < Q; ++i) {
        const double cu = cx(i) * u0 + cy(i) * u1 + cz(i) * u2;
        ok = ok && (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu > 0.0);
    }
    if (!ok) atomicMin(bad, k);
    us[k] = Real(u0);
    us[n + k] = Real(u1);
    us[2 * n + k] = Real(u2);
}

template <class Real>
__global__ void k_source_field(const double* r, long long n, Real* rs) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    rs[k] = Real(r[k]);
}

// Equilibrium factors of one node in FP64 (for set-up and readout kernels).
template <class Real>
__device__ inline void node_u64(const StepArgs<Real>& a, int umode, long long k, double u[3]) {
    if (umode == 2) {
        u[0] = double(a.ufield[k]);
        u[1] = double(a.ufield[a.n + k]);
        u[2] = double(a.ufield[2 * a.n + k]);
    } else {
        u[0] = double(a.u[0]);
        u[1] = double(a.u[1]);
        u[2] = double(a.u[2]);
    }
}
__device__ inline double eq_factor(int i, const double u[3]) {
    const double cu = cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2];
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
}

// Row and column of node k (x fastest): the population buffers are addressed by row.
struct RowCol {
    long long r;
    int x;
};
__device__ inline RowCol row_col(long long k, int nx) {
    const long long r = k / nx;
    return {r, int(k - r * nx)};
}

// Store the Q FP64 values v (deviations) of node k into a population buffer. With the
// FP32 rest population of the 16-bit forms the rounding residuals of the Q - 1 moving
// populations are added to the rest value, so the stored mass of the node equals sum v to
// FP32 rounding.
template <class ST>
__device__ inline void put_node(const StepArgs<typename Store<ST>::Real>& a, ST* buf, long long k,
                                const double (&v)[Q]) {
    using Real = typename Store<ST>::Real;
    const RowCol p = row_col(k, a.nx);
    if constexpr (sizeof(ST) == 2) {
        if (a.rest32) {
            double res = 0.0;
            for (int i = 1; i < Q; ++i) {
                const float q = quantize16<ST>(float(v[i]), 0u, false, a.scale, a.inv_scale);
                res += v[i] - double(q);
                pop_put<ST>(buf, i, p.r, p.x, a.nx, q, 1, a.inv_scale);
            }
            reinterpret_cast<float*>(buf)[rest_offset(p.r, p.x, a.nx)] = float(v[0] + res);
            return;
        }
    }
    for (int i = 0; i < Q; ++i) pop_put<ST>(buf, i, p.r, p.x, a.nx, Real(v[i]), a.rest32, a.inv_scale);
}

template <class ST>
__global__ void k_init(StepArgs<typename Store<ST>::Real> a, int umode, const double* phi0,
                       const double* j0) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    double u[3];
    node_u64(a, umode, k, u);
    const double p = phi0[k];
    const double jx = j0 ? j0[k] : 0.0, jy = j0 ? j0[a.n + k] : 0.0, jz = j0 ? j0[2 * a.n + k] : 0.0;
    double g[Q];
    for (int i = 0; i < Q; ++i)
        g[i] = weight(i) * (p * eq_factor(i, u) - double(a.phi_ref)) +
               w3(i) * (cx(i) * jx + cy(i) * jy + cz(i) * jz);
    put_node<ST>(a, static_cast<ST*>(a.dst), k, g);
}

// Adjoint of the initialisation: g_i = W_i (phi0 E_i(u) - phi_ref) + 3 W_i c_i . j0, so
// dL/dphi0 = sum_i W_i E_i dL/dg_i and dL/dj0 = 3 sum_i W_i c_i dL/dg_i (FP64 sums).
template <class ST>
__global__ void k_init_grad(StepArgs<typename Store<ST>::Real> a, int umode,
                            const typename Store<ST>::Real* adj, double* dphi0, double* dj0) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    double u[3];
    node_u64(a, umode, k, u);
    double gp = 0.0, gj[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        const double g = double(adj[(size_t)i * a.n + k]);
        gp += weight(i) * eq_factor(i, u) * g;
        gj[0] += w3(i) * cx(i) * g;
        gj[1] += w3(i) * cy(i) * g;
        gj[2] += w3(i) * cz(i) * g;
    }
    dphi0[k] = gp;
    if (dj0) {
        dj0[k] = gj[0];
        dj0[a.n + k] = gj[1];
        dj0[2 * a.n + k] = gj[2];
    }
}

// Adjoint of the scalar readout phi = sum_i g_i (+ terms free of g): dL/dg_i = dL/dphi.
template <class Real>
__global__ void k_fill_adjoint(const double* dphi, long long n, Real* adj) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const Real v = Real(dphi[k]);
    for (int i = 0; i < Q; ++i) adj[(size_t)i * n + k] = v;
}

// Pending source half-step as FP64 increments of one node.
template <class Real>
__device__ inline double pending_r(const StepArgs<Real>& a, long long k) {
    if (!a.has_src) return 0.0;
    return 0.5 * double(a.src_mult) * double(a.rfield ? a.rfield[k] : a.R);
}

template <class ST>
__global__ void k_flush(StepArgs<typename Store<ST>::Real> a, int umode) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    double u[3];
    node_u64(a, umode, k, u);
    const double R = pending_r(a, k);
    ST* buf = static_cast<ST*>(a.dst);
    const RowCol p = row_col(k, a.nx);
    double v[Q];
    for (int i = 0; i < Q; ++i)
        v[i] = double(pop_load<ST>(buf, i, p.r, p.x, a.nx, a.rest32, a.scale)) + R * weight(i) * eq_factor(i, u);
    put_node<ST>(a, buf, k, v);
}

template <class ST>
__global__ void k_get_pops(StepArgs<typename Store<ST>::Real> a, int umode, double* f) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    double u[3];
    node_u64(a, umode, k, u);
    const double R = pending_r(a, k);
    const ST* buf = static_cast<const ST*>(a.src);
    const RowCol p = row_col(k, a.nx);
    for (int i = 0; i < Q; ++i)
        f[(size_t)i * a.n + k] = weight(i) * double(a.phi_ref) +
                                 double(pop_load<ST>(buf, i, p.r, p.x, a.nx, a.rest32, a.scale)) +
                                 R * weight(i) * eq_factor(i, u);
}

template <class ST>
__global__ void k_set_pops(StepArgs<typename Store<ST>::Real> a, const double* f) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    double v[Q];
    for (int i = 0; i < Q; ++i) v[i] = f[(size_t)i * a.n + k] - weight(i) * double(a.phi_ref);
    put_node<ST>(a, static_cast<ST*>(a.dst), k, v);
}

// phi deviation and LB flux q = T j / 2 of one node, FP64, including the pending source.
template <class ST>
__device__ inline void node_moments(const StepArgs<typename Store<ST>::Real>& a, int umode, long long k,
                                    double* dphi, double q[3]) {
    double u[3];
    node_u64(a, umode, k, u);
    const double R = pending_r(a, k);
    const ST* buf = static_cast<const ST*>(a.src);
    const RowCol p = row_col(k, a.nx);
    double s = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
    for (int i = 0; i < Q; ++i) {
        const double d = double(pop_load<ST>(buf, i, p.r, p.x, a.nx, a.rest32, a.scale)) +
                         R * weight(i) * eq_factor(i, u);
        s += d;
        j0 += cx(i) * d;
        j1 += cy(i) * d;
        j2 += cz(i) * d;
    }
    const double phi = double(a.phi_ref) + s;
    j0 -= phi * u[0];
    j1 -= phi * u[1];
    j2 -= phi * u[2];
    double T[6];
    const long long row = tensor_row(a, k);
    for (int m = 0; m < 6; ++m) T[m] = a.tfield ? double(a.tfield[6 * row + m]) : double(a.T[m]);
    q[0] = 0.5 * (T[0] * j0 + T[1] * j1 + T[2] * j2);
    q[1] = 0.5 * (T[1] * j0 + T[3] * j1 + T[4] * j2);
    q[2] = 0.5 * (T[2] * j0 + T[4] * j1 + T[5] * j2);
    *dphi = s;
}

template <class ST>
__global__ void k_moments(StepArgs<typename Store<ST>::Real> a, int umode, double* phi, double* q3) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    double dphi, q[3];
    node_moments<ST>(a, umode, k, &dphi, q);
    if (phi) phi[k] = double(a.phi_ref) + dphi;
    if (q3) {
        q3[k] = q[0];
        q3[a.n + k] = q[1];
        q3[2 * a.n + k] = q[2];
    }
}

// Neumaier-compensated accumulation per thread (grid-stride), then an FP64 block tree.
constexpr int kRedThreads = 256;

template <class ST>
__global__ __launch_bounds__(kRedThreads) void k_reduce_partial(StepArgs<typename Store<ST>::Real> a,
                                                                int umode, double* part) {
    double sum[4] = {0, 0, 0, 0}, comp[4] = {0, 0, 0, 0};
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < a.n;
         k += (long long)gridDim.x * blockDim.x) {
        double v[4];
        node_moments<ST>(a, umode, k, &v[0], &v[1]);
        for (int m = 0; m < 4; ++m) {
            const double t = sum[m] + v[m];
            comp[m] += (fabs(sum[m]) >= fabs(v[m])) ? (sum[m] - t) + v[m] : (v[m] - t) + sum[m];
            sum[m] = t;
        }
    }
    __shared__ double sh[4][kRedThreads];
    for (int m = 0; m < 4; ++m) sh[m][threadIdx.x] = sum[m] + comp[m];
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int m = 0; m < 4; ++m) sh[m][threadIdx.x] += sh[m][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int m = 0; m < 4; ++m) part[4 * blockIdx.x + m] = sh[m][0];
}

// Smallest current population g_i (full value, as the population readout gives it, with
// the pending source half-step) per block, grid-stride; NaN values are skipped by fmin.
template <class ST>
__global__ __launch_bounds__(kRedThreads) void k_min_partial(StepArgs<typename Store<ST>::Real> a,
                                                             int umode, double* part) {
    double m = __builtin_huge_val();
    const ST* buf = static_cast<const ST*>(a.src);
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < a.n;
         k += (long long)gridDim.x * blockDim.x) {
        double u[3];
        node_u64(a, umode, k, u);
        const double R = pending_r(a, k);
        const RowCol p = row_col(k, a.nx);
        for (int i = 0; i < Q; ++i)
            m = fmin(m, weight(i) * double(a.phi_ref) +
                            double(pop_load<ST>(buf, i, p.r, p.x, a.nx, a.rest32, a.scale)) +
                            R * weight(i) * eq_factor(i, u));
    }
    __shared__ double sh[kRedThreads];
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kRedThreads) void k_min_final(const double* part, int nb, double* out) {
    double m = __builtin_huge_val();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) m = fmin(m, part[b]);
    __shared__ double sh[kRedThreads];
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// One block of kRedThreads threads: each thread sums a strided subset of the block
// partials with Neumaier compensation, then the threads' results are added in a tree.
__global__ __launch_bounds__(kRedThreads) void k_reduce_final(const double* part, int nb,
                                                              double add_mass, double* out) {
    double sum[4] = {0, 0, 0, 0}, comp[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
        for (int m = 0; m < 4; ++m) {
            const double v = part[4 * b + m];
            const double t = sum[m] + v;
            comp[m] += (fabs(sum[m]) >= fabs(v)) ? (sum[m] - t) + v : (v - t) + sum[m];
            sum[m] = t;
        }
    __shared__ double sh[4][kRedThreads];
    for (int m = 0; m < 4; ++m) sh[m][threadIdx.x] = sum[m] + comp[m];
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int m = 0; m < 4; ++m) sh[m][threadIdx.x] += sh[m][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = add_mass + sh[0][0];
        for (int m = 1; m < 4; ++m) out[m] = sh[m][0];
    }
}

// dL/dT (6 stored components) -> dL/dD or dL/dL (6 stored components), FP64.
template <class Real>
__global__ void k_tensor_grad(const double* d6, int is_log, long long n, const Real* tg, double* out6) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double D[3][3], V[3][3], ev[3];
    node_tensor(d6, n, k, is_log, D, V, ev);
    // full symmetric gradient of T: off-diagonal stored components appear twice
    double g6[6];
    for (int m = 0; m < 6; ++m) g6[m] = double(tg[6 * k + m]);  // node-major
    double G[3][3] = {{g6[0], 0.5 * g6[1], 0.5 * g6[2]},
                      {0.5 * g6[1], g6[3], 0.5 * g6[4]},
                      {0.5 * g6[2], 0.5 * g6[4], g6[5]}};
    // T = 2 I - S, S = (I/2 + 3 D)^-1 = 2 (I + 6 D)^-1: dT = 3 S dD S  =>  G_D = 3 S G S
    double M[3][3], S[3][3], SG[3][3], GD[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[r][c] = 0.5 * (r == c ? 1.0 : 0.0) + 3.0 * D[r][c];
    inv3(M, S);
    mul3(S, G, SG);
    mul3(SG, S, GD);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) GD[r][c] *= 3.0;
    double GO[3][3];
    if (is_log) {
        // Daleckii-Krein: dD = V (F o (V^T dL V)) V^T, F_ab = (e^la - e^lb)/(la - lb)
        double l[3];
        for (int a = 0; a < 3; ++a) l[a] = log(ev[a]);
        double B[3][3], C[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q) acc += V[p][r] * GD[p][q] * V[q][c];
                const double dl = l[r] - l[c];
                const double F = (fabs(dl) > 1e-8) ? ev[c] * expm1(dl) / dl : exp(0.5 * (l[r] + l[c]));
                B[r][c] = F * acc;
            }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q) acc += V[r][p] * B[p][q] * V[c][q];
                C[r][c] = acc;
            }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) GO[r][c] = C[r][c];
    } else {
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) GO[r][c] = GD[r][c];
    }
    out6[k] = GO[0][0];
    out6[n + k] = GO[0][1] + GO[1][0];
    out6[2 * n + k] = GO[0][2] + GO[2][0];
    out6[3 * n + k] = GO[1][1];
    out6[4 * n + k] = GO[1][2] + GO[2][1];
    out6[5 * n + k] = GO[2][2];
}

// ------------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------------
#define ELBM_DISPATCH(h, BODY)                                   \
    switch ((h)->cfg.precision) {                                \
        case ELBM_F64: { using ST = double; BODY; } break;        \
        case ELBM_F32: { using ST = float; BODY; } break;         \
        case ELBM_BF16: { using ST = bf16s; BODY; } break;        \
        default: { using ST = _Float16; BODY; } break;            \
    }

hipError_t launch_tensor_field(const elbm_lattice* h, const double* d6, long long count, int is_log,
                               void* t_store, long long* bad) {
    const unsigned nb = blocks_for(count, 256);
    if (h->cfg.precision == ELBM_F64)
        hipLaunchKernelGGL(k_tensor_field<double>, dim3(nb), dim3(256), 0, h->stream, d6, is_log,
                           count, static_cast<double*>(t_store), bad);
    else
        hipLaunchKernelGGL(k_tensor_field<float>, dim3(nb), dim3(256), 0, h->stream, d6, is_log,
                           count, static_cast<float*>(t_store), bad);
    return hipGetLastError();
}

hipError_t launch_phase_check(const elbm_lattice* h, const uint8_t* phase, int nphase, long long* bad) {
    const unsigned nb = blocks_for(h->n, 256);
    hipLaunchKernelGGL(k_phase_check, dim3(nb), dim3(256), 0, h->stream, phase, (long long)h->n,
                       nphase, bad);
    return hipGetLastError();
}

hipError_t launch_velocity_field(const elbm_lattice* h, const double* u3, void* u_store, long long* bad) {
    const unsigned nb = blocks_for(h->n, 256);
    if (h->cfg.precision == ELBM_F64)
        hipLaunchKernelGGL(k_velocity_field<double>, dim3(nb), dim3(256), 0, h->stream, u3,
                           (long long)h->n, static_cast<double*>(u_store), bad);
    else
        hipLaunchKernelGGL(k_velocity_field<float>, dim3(nb), dim3(256), 0, h->stream, u3,
                           (long long)h->n, static_cast<float*>(u_store), bad);
    return hipGetLastError();
}

hipError_t launch_source_field(const elbm_lattice* h, const double* r, void* r_store) {
    const unsigned nb = blocks_for(h->n, 256);
    if (h->cfg.precision == ELBM_F64)
        hipLaunchKernelGGL(k_source_field<double>, dim3(nb), dim3(256), 0, h->stream, r,
                           (long long)h->n, static_cast<double*>(r_store));
    else
        hipLaunchKernelGGL(k_source_field<float>, dim3(nb), dim3(256), 0, h->stream, r,
                           (long long)h->n, static_cast<float*>(r_store));
    return hipGetLastError();
}

hipError_t launch_init(const elbm_lattice* h, const double* phi0, const double* j0, void* dst) {
    const unsigned nb = blocks_for(h->n, 256);
    ELBM_DISPATCH(h, {
        auto a = make_args<typename Store<ST>::Real>(h, 0.0);
        a.dst = dst;
        hipLaunchKernelGGL(k_init<ST>, dim3(nb), dim3(256), 0, h->stream, a, h->u_mode, phi0, j0);
    });
    return hipGetLastError();
}

hipError_t launch_fill_adjoint(const elbm_lattice* h, const double* dphi, void* adj) {
    const unsigned nb = blocks_for(h->n, 256);
    if (h->cfg.precision == ELBM_F64)
        hipLaunchKernelGGL(k_fill_adjoint<double>, dim3(nb), dim3(256), 0, h->stream, dphi,
                           (long long)h->n, static_cast<double*>(adj));
    else
        hipLaunchKernelGGL(k_fill_adjoint<float>, dim3(nb), dim3(256), 0, h->stream, dphi,
                           (long long)h->n, static_cast<float*>(adj));
    return hipGetLastError();
}

hipError_t launch_init_gradient(const elbm_lattice* h, const void* adj, double* dphi0, double* dj0) {
    const unsigned nb = blocks_for(h->n, 256);
    ELBM_DISPATCH(h, {
        using Real = typename Store<ST>::Real;
        auto a = make_args<Real>(h, 0.0);
        hipLaunchKernelGGL(k_init_grad<ST>, dim3(nb), dim3(256), 0, h->stream, a, h->u_mode,
                           static_cast<const Real*>(adj), dphi0, dj0);
    });
    return hipGetLastError();
}

hipError_t launch_flush_source(const elbm_lattice* h, void* buf) {
    const unsigned nb = blocks_for(h->n, 256);
    ELBM_DISPATCH(h, {
        auto a = make_args<typename Store<ST>::Real>(h, h->pending_scale);
        a.dst = buf;
        hipLaunchKernelGGL(k_flush<ST>, dim3(nb), dim3(256), 0, h->stream, a, h->u_mode);
    });
    return hipGetLastError();
}

// src_mult in readouts: the amplitude of the pending half-step, 0.5 * s * R * E_i
hipError_t launch_get_pops(const elbm_lattice* h, double* f) {
    const unsigned nb = blocks_for(h->n, 256);
    ELBM_DISPATCH(h, {
        auto a = make_args<typename Store<ST>::Real>(h, h->pending ? h->pending_scale : 0.0);
        a.src = h->buf[h->cur];
        hipLaunchKernelGGL(k_get_pops<ST>, dim3(nb), dim3(256), 0, h->stream, a, h->u_mode, f);
    });
    return hipGetLastError();
}

hipError_t launch_set_pops(const elbm_lattice* h, const double* f, void* dst) {
    const unsigned nb = blocks_for(h->n, 256);
    ELBM_DISPATCH(h, {
        auto a = make_args<typename Store<ST>::Real>(h, 0.0);
        a.dst = dst;
        hipLaunchKernelGGL(k_set_pops<ST>, dim3(nb), dim3(256), 0, h->stream, a, f);
    });
    return hipGetLastError();
}

hipError_t launch_moments(const elbm_lattice* h, double* phi, double* q3) {
    const unsigned nb = blocks_for(h->n, 256);
    ELBM_DISPATCH(h, {
        auto a = make_args<typename Store<ST>::Real>(h, h->pending ? h->pending_scale : 0.0);
        a.src = h->buf[h->cur];
        hipLaunchKernelGGL(k_moments<ST>, dim3(nb), dim3(256), 0, h->stream, a, h->u_mode, phi, q3);
    });
    return hipGetLastError();
}

hipError_t launch_reduce(const elbm_lattice* h, double* out4_dev, double* part) {
    const int nb = h->part_blocks;
    ELBM_DISPATCH(h, {
        auto a = make_args<typename Store<ST>::Real>(h, h->pending ? h->pending_scale : 0.0);
        a.src = h->buf[h->cur];
        hipLaunchKernelGGL(k_reduce_partial<ST>, dim3(nb), dim3(kRedThreads), 0, h->stream, a,
                           h->u_mode, part);
    });
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedThreads), 0, h->stream, part, nb,
                       double(h->n) * h->cfg.phi_ref, out4_dev);
    return hipGetLastError();
}

hipError_t launch_min_population(const elbm_lattice* h, double* out_dev) {
    const int nb = h->part_blocks;
    ELBM_DISPATCH(h, {
        auto a = make_args<typename Store<ST>::Real>(h, h->pending ? h->pending_scale : 0.0);
        a.src = h->buf[h->cur];
        hipLaunchKernelGGL(k_min_partial<ST>, dim3(nb), dim3(kRedThreads), 0, h->stream, a,
                           h->u_mode, h->d_part);
    });
    hipLaunchKernelGGL(k_min_final, dim3(1), dim3(kRedThreads), 0, h->stream, h->d_part, nb, out_dev);
    return hipGetLastError();
}

// Streaming copy, the achievable-bandwidth reference for the step kernels: every byte read
// once and written once, 16 bytes per lane and access, nontemporal loads and stores as in
// the step kernels. One tile of 1024 16-byte words per block, four accesses per lane; with a
// multiple of 8 tiles, the tiles are dealt so that each XCD copies one contiguous eighth
// (blocks go to the XCDs in turn). Measured on MI355X for 2 GiB this was the fastest of the
// simple layouts tried (5.9 TB/s; a grid-stride loop over 2048 blocks: 4.6 TB/s; contiguous
// chunks per persistent block: 5.4-5.5 TB/s).
typedef uint32_t copy_u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyTile = 1024;
__global__ __launch_bounds__(256) void k_stream_copy(const copy_u32x4* __restrict__ src,
                                                     copy_u32x4* __restrict__ dst, size_t n) {
    const unsigned g = gridDim.x, b = blockIdx.x;
    const size_t t = (g % 8u == 0) ? size_t(b % 8u) * (g / 8u) + b / 8u : size_t(b);
    const size_t i = t * kCopyTile + threadIdx.x;
    if (i + 3 * 256 < n) {
        const copy_u32x4 x0 = __builtin_nontemporal_load(src + i);
        const copy_u32x4 x1 = __builtin_nontemporal_load(src + i + 256);
        const copy_u32x4 x2 = __builtin_nontemporal_load(src + i + 512);
        const copy_u32x4 x3 = __builtin_nontemporal_load(src + i + 768);
        __builtin_nontemporal_store(x0, dst + i);
        __builtin_nontemporal_store(x1, dst + i + 256);
        __builtin_nontemporal_store(x2, dst + i + 512);
        __builtin_nontemporal_store(x3, dst + i + 768);
    } else {
        for (int k = 0; k < 4; ++k)
            if (i + 256 * k < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i + 256 * k), dst + i + 256 * k);
    }
}

hipError_t launch_stream_copy(const elbm_lattice* h, const void* src, void* dst, size_t words16) {
    const size_t tiles = (words16 + kCopyTile - 1) / kCopyTile;
    if (tiles > 0x7FFFFFFFu) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy, dim3(unsigned(tiles)), dim3(256), 0, h->stream,
                       static_cast<const copy_u32x4*>(src), static_cast<copy_u32x4*>(dst), words16);
    return hipGetLastError();
}

hipError_t launch_tensor_gradient(const elbm_lattice* h, const double* d6, int is_log,
                                  const void* t_grad, double* out6) {
    const unsigned nb = blocks_for(h->n, 256);
    if (h->cfg.precision == ELBM_F64)
        hipLaunchKernelGGL(k_tensor_grad<double>, dim3(nb), dim3(256), 0, h->stream, d6, is_log,
                           (long long)h->n, static_cast<const double*>(t_grad), out6);
    else
        hipLaunchKernelGGL(k_tensor_grad<float>, dim3(nb), dim3(256), 0, h->stream, d6, is_log,
                           (long long)h->n, static_cast<const float*>(t_grad), out6);
    return hipGetLastError();
}

}  // namespace elbm
