// FP64 CPU oracle of the local entropic lattice Boltzmann scheme for the full-tensor
// anisotropic advection-diffusion equation (Feng, Leng, Jiang, Chu, arXiv 2605.01774).
//
// TEST INFRASTRUCTURE ONLY. This is the independent, slow, plain reference the GPU library
// is checked against. Only the test-suite, the smoke check and the CPU-baseline leg of the
// benchmark may load it; the product path never does. It shares no code, header, table or
// constant with the GPU library: its velocity set, weights, equilibrium, inverse and update
// are written out here from the paper, in the paper's order and notation.
//
// Update per node (Sec. 2.7, algorithmic summary), on pre-collision populations g_i(x, t_n):
//   1. zeroth moment phi and second-order equilibrium g_eq            (Sec. 2.1)
//   2. S = (I/2 + D/(cs^2 dt))^-1, non-equilibrium flux j,
//      flux lift Ds = P(j) and ghost residual Dh = g_neq - Ds           (Secs. 2.2, 2.3)
//   3. tensorial flux relaxation Om^(s) = -P(S j), Ds_post = P((I-S) j) (Sec. 2.3)
//   4. entropic amplitude lambda (closed form, Sec. 2.5 / App. B)
//   5. Om = Om^(s) - lambda Dh, positivity fallback alpha              (Secs. 2.5, 2.6)
//   6. g + alpha Om, then streaming g_i(x + c_i, t + dt)                (Sec. 2.1)
// Source terms use the symmetric midpoint splitting of Sec. 3.3 around the carrier step.
//
// Readings where the paper is silent (all also implemented by the GPU path):
//   * lattice: D3Q19 (weights 1/3, 1/18, 1/36) or the paper's tensor-product D3Q27;
//     both satisfy the quadrature identities that App. A uses. dx = dt = 1, cs^2 = 1/3.
//   * ghost floor: the denominator <Dh|Dh>_H gets + tau^2 phi, so lambda -> 1 continuously
//     when the ghost part is at roundoff level; tau = 0 with an exactly zero ghost is the
//     paper's own "lambda = 1 if Dh == 0" rule. lambda = 1 where phi <= 0 (g_eq must be > 0).
//   * fallback: alpha is clamped to [0, 1].
//     Parity unpinned in one regime: where the ghost part is at roundoff level and u != 0,
//     lambda is fixed only by the ghost-floor convention above. Every function here has a
//     pin; that regime has none beyond the convention itself.
//   * Dirichlet planes on x: halfway anti-bounce-back, g_ibar(x_b) = -post_i(x_b) + 2 W_i phi_w.
//   * exact entropic root (optional): at nodes whose closed-form trial populations fall below
//     rho * g_eq, the stationarity condition of Sec. 2.5 is solved by safeguarded Newton-
//     bisection on the interval where every trial population is positive.
//
// Build: g++ -O2 -fopenmp -shared -fPIC (see oracle/build.py).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ----------------------------------------------------------------------------------------
// Scalar types: plain double, and a forward-mode dual number used only to differentiate
// the same update exactly (derivative = chain rule applied to every operation below).
// ----------------------------------------------------------------------------------------
struct Dual {
    double v, d;
    Dual() : v(0.0), d(0.0) {}
    Dual(double x) : v(x), d(0.0) {}
    Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
    return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
inline Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
inline Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual operator/(double a, Dual b) { return Dual(a / b.v, -a * b.d / (b.v * b.v)); }
inline Dual log(Dual a) { return Dual(std::log(a.v), a.d / a.v); }
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline double dval(double) { return 0.0; }
inline double dval(const Dual& x) { return x.d; }
using std::log;

// ----------------------------------------------------------------------------------------
// Velocity set and weights (Sec. 2.1).
// ----------------------------------------------------------------------------------------
struct Lattice {
    int q;
    int c[27][3];
    double w[27];
    int opp[27];
};

// Velocities are enumerated with c_x outermost over {-1, 0, 1}; D3Q19 keeps those with at
// most two nonzero components. Weights: D3Q27 uses the tensor-product rule
// W = (2/3)^(3-m) (1/6)^m of Sec. 2.1 (m = number of nonzero components); D3Q19 uses
// 1/3, 1/18, 1/36 for m = 0, 1, 2.
Lattice make_lattice(int q) {
    Lattice L;
    L.q = 0;
    for (int cx = -1; cx <= 1; ++cx)
        for (int cy = -1; cy <= 1; ++cy)
            for (int cz = -1; cz <= 1; ++cz) {
                int m = (cx != 0) + (cy != 0) + (cz != 0);
                if (q == 19 && m == 3) continue;
                int k = L.q++;
                L.c[k][0] = cx;
                L.c[k][1] = cy;
                L.c[k][2] = cz;
                if (q == 27) {
                    double wq = 1.0;
                    for (int a = 0; a < 3 - m; ++a) wq *= 2.0 / 3.0;
                    for (int a = 0; a < m; ++a) wq *= 1.0 / 6.0;
                    L.w[k] = wq;
                } else {
                    L.w[k] = (m == 0) ? 1.0 / 3.0 : (m == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
                }
            }
    for (int i = 0; i < L.q; ++i)
        for (int k = 0; k < L.q; ++k)
            if (L.c[k][0] == -L.c[i][0] && L.c[k][1] == -L.c[i][1] && L.c[k][2] == -L.c[i][2])
                L.opp[i] = k;
    return L;
}

const double kCs2 = 1.0 / 3.0;  // cs^2 = c^2 / 3 with c = dx/dt = 1 (Sec. 2.1)
const double kDt = 1.0;

}  // namespace

extern "C" {

// Parameters shared by every oracle entry point. Tensors are 6-vectors (xx, xy, xz, yy, yz,
// zz); fields are SoA planes [component][z][y][x]; populations are [i][z][y][x] in this
// oracle's own velocity order (oracle_velocities).
typedef struct {
    int32_t q, nx, ny, nz;
    int32_t bc_x;           // 0: periodic in x; 1: Dirichlet planes on both x faces
    int32_t d_uniform;      // 1: d6 holds a single tensor used at every node
    int32_t u_uniform;      // 1: u3 holds a single velocity
    int32_t r_mode;         // 0: no source; 1: uniform r[0]; 2: r per node
    int32_t tensor_is_log;  // 1: d6 holds the log-diffusivity L, D = expm(L)
    int32_t nthreads;       // OpenMP threads (<= 0: runtime default)
    double phi_lo, phi_hi;  // Dirichlet values on the x = 0 and x = nx-1 sides
    double eps;             // positivity threshold of the fallback
    double tau;             // ghost floor
    double root_rho;        // exact-root flag threshold; < 0 disables the exact root
} oracle_params;

}  // extern "C"

namespace {

struct NodeInfo {
    double lambda = 1.0;      // amplitude used
    double lambda_lin = 1.0;  // closed-form amplitude
    double alpha = 1.0;       // fallback factor used
    int flagged = 0;          // exact root attempted
};

// ----------------------------------------------------------------------------------------
// D -> S, Sec. 2.3: S = (I/2 + D/(cs^2 dt))^-1, by the adjugate of the symmetric 3x3 matrix.
// ----------------------------------------------------------------------------------------
template <class T>
void s_from_d(const T d6[6], T S[9]) {
    T M[9] = {0.5 + d6[0] / (kCs2 * kDt), d6[1] / (kCs2 * kDt), d6[2] / (kCs2 * kDt),
              d6[1] / (kCs2 * kDt),       0.5 + d6[3] / (kCs2 * kDt), d6[4] / (kCs2 * kDt),
              d6[2] / (kCs2 * kDt),       d6[4] / (kCs2 * kDt), 0.5 + d6[5] / (kCs2 * kDt)};
    T A[9];
    A[0] = M[4] * M[8] - M[5] * M[7];
    A[1] = M[2] * M[7] - M[1] * M[8];
    A[2] = M[1] * M[5] - M[2] * M[4];
    A[3] = M[5] * M[6] - M[3] * M[8];
    A[4] = M[0] * M[8] - M[2] * M[6];
    A[5] = M[2] * M[3] - M[0] * M[5];
    A[6] = M[3] * M[7] - M[4] * M[6];
    A[7] = M[1] * M[6] - M[0] * M[7];
    A[8] = M[0] * M[4] - M[1] * M[3];
    T det = M[0] * A[0] + M[1] * A[3] + M[2] * A[6];
    for (int k = 0; k < 9; ++k) S[k] = A[k] / det;
}

// Matrix exponential of a symmetric 3x3 matrix by scaling and squaring of the Taylor series
// (used when the tensor field is given as a log-diffusivity, D = expm(L)).
template <class T>
void expm_sym(const T l6[6], T D6[6]) {
    T Lm[9] = {l6[0], l6[1], l6[2], l6[1], l6[3], l6[4], l6[2], l6[4], l6[5]};
    double nrm = 0.0;
    for (int k = 0; k < 9; ++k) nrm += val(Lm[k]) * val(Lm[k]);
    nrm = std::sqrt(nrm);
    int s = 0;
    while (nrm > 0.25) {
        nrm *= 0.5;
        ++s;
    }
    double scale = std::ldexp(1.0, -s);
    T A[9], E[9], P[9], tmp[9];
    for (int k = 0; k < 9; ++k) {
        A[k] = Lm[k] * scale;
        E[k] = (k % 4 == 0) ? T(1.0) : T(0.0);
        P[k] = E[k];
    }
    for (int n = 1; n <= 24; ++n) {
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                T acc = 0.0;
                for (int k = 0; k < 3; ++k) acc = acc + P[3 * r + k] * A[3 * k + c];
                tmp[3 * r + c] = acc / double(n);
            }
        for (int k = 0; k < 9; ++k) {
            P[k] = tmp[k];
            E[k] = E[k] + P[k];
        }
    }
    for (int it = 0; it < s; ++it) {
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                T acc = 0.0;
                for (int k = 0; k < 3; ++k) acc = acc + E[3 * r + k] * E[3 * k + c];
                tmp[3 * r + c] = acc;
            }
        for (int k = 0; k < 9; ++k) E[k] = tmp[k];
    }
    D6[0] = E[0];
    D6[1] = 0.5 * (E[1] + E[3]);
    D6[2] = 0.5 * (E[2] + E[6]);
    D6[3] = E[4];
    D6[4] = 0.5 * (E[5] + E[7]);
    D6[5] = E[8];
}

// First-order lift P_i(a) = (W_i / cs^2) c_i . a (Sec. 2.2).
template <class T>
inline T lift(const Lattice& L, int i, const T a[3]) {
    T ca = double(L.c[i][0]) * a[0] + double(L.c[i][1]) * a[1] + double(L.c[i][2]) * a[2];
    return (L.w[i] / kCs2) * ca;
}

// Stationarity function of the entropy along the ghost line (Sec. 2.5):
//   F(lambda) = sum_i Dh_i ln((g_eq_i + Ds_post_i + (1 - lambda) Dh_i) / W_i).
// Solved on the open interval where every trial population is positive. F is strictly
// decreasing there (F' = -sum Dh_i^2 / g*_i < 0) and runs from +inf to -inf, so the root is
// unique. Safeguarded Newton-bisection, FP64. Returns false if the interval is empty.
bool entropic_root(const Lattice& L, const double* A, const double* dh, double start,
                   double* root) {
    double lo = -std::numeric_limits<double>::infinity();
    double hi = std::numeric_limits<double>::infinity();
    for (int i = 0; i < L.q; ++i) {
        if (dh[i] > 0.0) hi = std::fmin(hi, A[i] / dh[i]);
        else if (dh[i] < 0.0) lo = std::fmax(lo, A[i] / dh[i]);
        else if (A[i] <= 0.0) return false;
    }
    if (!(lo < hi) || !std::isfinite(lo) || !std::isfinite(hi)) return false;
    double x = (start > lo && start < hi) ? start : 0.5 * (lo + hi);
    double a = lo, b = hi;
    for (int it = 0; it < 200; ++it) {
        double F = 0.0, dF = 0.0;
        bool ok = true;
        for (int i = 0; i < L.q; ++i) {
            double gs = A[i] - x * dh[i];
            if (!(gs > 0.0)) { ok = false; break; }
            F += dh[i] * std::log(gs / L.w[i]);
            dF -= dh[i] * dh[i] / gs;
        }
        if (!ok) {  // numerically at the edge of the interval: step inward
            x = 0.5 * (a + b);
            continue;
        }
        if (F == 0.0) break;  // x is the root
        const double step = F / dF;
        if (std::fabs(step) <= 1e-15 * std::fmax(1.0, std::fabs(x))) {  // converged
            x -= step;
            break;
        }
        // keep the root bracketed: F > 0 means the root lies to the right of x
        if (F > 0.0) a = x; else b = x;
        double xn = x - step;
        if (!(xn > a && xn < b)) xn = 0.5 * (a + b);
        x = xn;
    }
    *root = x;
    return true;
}

// lambda at the exact root as a function of the inputs (implicit function theorem:
// dlambda = -F_theta / F_lambda); for plain doubles it is just the root.
inline double root_value(double lr, const Lattice&, const double*, const double*) { return lr; }
Dual root_value(double lr, const Lattice& L, const Dual* A, const Dual* dh) {
    Dual F = 0.0;
    double dF = 0.0;
    for (int i = 0; i < L.q; ++i) {
        Dual gs = A[i] - lr * dh[i];
        F = F + dh[i] * log(gs / L.w[i]);
        dF -= dh[i].v * dh[i].v / gs.v;
    }
    return Dual(lr, -F.d / dF);
}

// ----------------------------------------------------------------------------------------
// One collision at one node, Sec. 2.7 steps 1-5 and Eq. (update) g + alpha Om.
// g: pre-collision populations; S: 3x3 relaxation matrix; u: velocity.
// ----------------------------------------------------------------------------------------
template <class T>
void collide_node(const Lattice& L, const oracle_params& P, const T* g, const T* S,
                  const double* u, T* out, NodeInfo* info) {
    const int Q = L.q;
    // Zeroth moment, Sec. 2.1.
    T phi = 0.0;
    for (int i = 0; i < Q; ++i) phi = phi + g[i];
    // Second-order low-Mach equilibrium, Sec. 2.1.
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    T geq[27];
    double E[27];
    for (int i = 0; i < Q; ++i) {
        double cu = L.c[i][0] * u[0] + L.c[i][1] * u[1] + L.c[i][2] * u[2];
        E[i] = 1.0 + cu / kCs2 + cu * cu / (2.0 * kCs2 * kCs2) - uu / (2.0 * kCs2);
        geq[i] = phi * L.w[i] * E[i];
    }
    // Non-equilibrium part and first-order non-equilibrium flux j = sum c_i (g_i - g_eq_i).
    T neq[27];
    T j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        neq[i] = g[i] - geq[i];
        for (int a = 0; a < 3; ++a)
            if (L.c[i][a] != 0) j[a] = j[a] + double(L.c[i][a]) * neq[i];
    }
    // Flux/ghost split, Sec. 2.2: Ds = P(j), Dh = g_neq - Ds.
    T ds[27], dh[27];
    for (int i = 0; i < Q; ++i) {
        ds[i] = lift(L, i, j);
        dh[i] = neq[i] - ds[i];
    }
    // Tensorial flux relaxation, Sec. 2.3: Om^(s) = -P(S j), j* = (I - S) j,
    // Ds_post = Ds + Om^(s) = P(j*) (Sec. 2.5).
    T Sj[3], jst[3];
    for (int a = 0; a < 3; ++a) {
        Sj[a] = S[3 * a + 0] * j[0] + S[3 * a + 1] * j[1] + S[3 * a + 2] * j[2];
        jst[a] = j[a] - Sj[a];
    }
    T oms[27], dsp[27];
    for (int i = 0; i < Q; ++i) {
        oms[i] = -lift(L, i, Sj);
        dsp[i] = lift(L, i, jst);
    }
    // ADE-corrected entropic amplitude, Sec. 2.5 / App. B:
    //   lambda = 1 + (<Dh|Ds_post>_H + C) / <Dh|Dh>_H, <x|y>_H = sum x_i y_i / g_eq_i,
    //   C = sum Dh_i ln(g_eq_i / W_i); with the ghost floor tau^2 phi in the denominator.
    // ln(g_eq_i / W_i) = ln(phi) + ln(E_i), and the ln(phi) part multiplies sum Dh_i, which is
    // zero by construction (Sec. 2.2); C is therefore evaluated as sum Dh_i ln(E_i), which
    // keeps the roundoff of sum Dh_i out of the amplitude.
    T lam = 1.0;
    if (val(phi) > 0.0) {
        T hh = 0.0, hs = 0.0, C = 0.0;
        for (int i = 0; i < Q; ++i) {
            hh = hh + dh[i] * dh[i] / geq[i];
            hs = hs + dh[i] * dsp[i] / geq[i];
            C = C + dh[i] * std::log(E[i]);
        }
        T den = hh + (P.tau * P.tau) * phi;
        if (val(den) > 0.0) lam = 1.0 + (hs + C) / den;
    }
    info->lambda_lin = val(lam);
    info->flagged = 0;
    // Optional exact entropic root at nodes near the positivity bound.
    if (P.root_rho >= 0.0 && val(phi) > 0.0) {
        double mn = std::numeric_limits<double>::infinity();
        for (int i = 0; i < Q; ++i) {
            T gs = geq[i] + dsp[i] + (1.0 - lam) * dh[i];
            mn = std::fmin(mn, val(gs) / val(geq[i]));
        }
        if (mn < P.root_rho) {
            info->flagged = 1;
            T A[27];
            double Av[27], dhv[27];
            for (int i = 0; i < Q; ++i) {
                A[i] = geq[i] + dsp[i] + dh[i];
                Av[i] = val(A[i]);
                dhv[i] = val(dh[i]);
            }
            double lr;
            if (entropic_root(L, Av, dhv, val(lam), &lr)) lam = root_value(lr, L, A, dh);
        }
    }
    info->lambda = val(lam);
    // Unrestricted collision, Sec. 2.5: Om = Om^(s) - lambda Dh.
    T om[27];
    bool all_nonneg = true;
    for (int i = 0; i < Q; ++i) {
        om[i] = oms[i] - lam * dh[i];
        if (val(om[i]) < 0.0) all_nonneg = false;
    }
    // Positivity fallback, Sec. 2.6 (clamped to [0, 1]).
    T alpha = 1.0;
    if (!all_nonneg) {
        for (int i = 0; i < Q; ++i) {
            if (val(om[i]) < 0.0) {
                T r = (g[i] - P.eps) / (-om[i]);
                if (val(r) < val(alpha)) alpha = r;
            }
        }
        if (val(alpha) < 0.0) alpha = 0.0;
    }
    info->alpha = val(alpha);
    // Update, Sec. 2.6: g + alpha Om.
    for (int i = 0; i < Q; ++i) out[i] = g[i] + alpha * om[i];
}

// Source weight E_i(u) at unit density (Sec. 3.3, equilibrium polynomial at phi = 1).
inline double source_weight(const Lattice& L, int i, const double* u) {
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double cu = L.c[i][0] * u[0] + L.c[i][1] * u[1] + L.c[i][2] * u[2];
    return L.w[i] * (1.0 + cu / kCs2 + cu * cu / (2.0 * kCs2 * kCs2) - uu / (2.0 * kCs2));
}

inline int64_t node_index(const oracle_params& P, int x, int y, int z) {
    return (int64_t(z) * P.ny + y) * P.nx + x;
}

template <class T>
struct Fields {
    std::vector<T> S;  // 9 per node (or 9 if uniform)
    bool s_uniform = true;
};

// Relaxation matrices for the whole grid (or the single uniform one).
template <class T>
void build_s(const oracle_params& P, const T* d6in, int64_t n, Fields<T>* F) {
    F->s_uniform = P.d_uniform != 0;
    int64_t m = F->s_uniform ? 1 : n;
    F->S.assign(size_t(m) * 9, T(0.0));
    for (int64_t k = 0; k < m; ++k) {
        T d6[6];
        for (int c = 0; c < 6; ++c) d6[c] = F->s_uniform ? d6in[c] : d6in[c * n + k];
        if (P.tensor_is_log) {
            T l6[6];
            for (int c = 0; c < 6; ++c) l6[c] = d6[c];
            expm_sym(l6, d6);
        }
        s_from_d(d6, &F->S[size_t(k) * 9]);
    }
}

inline void node_u(const oracle_params& P, const double* u3, int64_t n, int64_t k, double u[3]) {
    for (int a = 0; a < 3; ++a) u[a] = P.u_uniform ? u3[a] : u3[a * n + k];
}
inline double node_r(const oracle_params& P, const double* r, int64_t k) {
    return P.r_mode == 0 ? 0.0 : (P.r_mode == 1 ? r[0] : r[k]);
}

// Half source step, Sec. 3.3: g_i += (dt/2) R E_i(u), R frozen in time.
template <class T>
void half_source(const Lattice& L, const oracle_params& P, const double* u3, const double* r,
                 T* f, int64_t n) {
    if (P.r_mode == 0) return;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double u[3];
        node_u(P, u3, n, k, u);
        double R = node_r(P, r, k);
        for (int i = 0; i < L.q; ++i) f[i * n + k] = f[i * n + k] + 0.5 * kDt * R * source_weight(L, i, u);
    }
}

struct Counts {
    int64_t fallback = 0;  // nodes with alpha < 1
    int64_t flagged = 0;   // nodes where the exact root was attempted
};

// One full time step: source half, collide, stream (push), source half.
template <class T>
void step(const Lattice& L, const oracle_params& P, const Fields<T>& F, const double* u3,
          const double* r, T* f, T* fnew, double* lam_out, double* alpha_out, Counts* cnt) {
    const int64_t n = int64_t(P.nx) * P.ny * P.nz;
    const int Q = L.q;
    half_source(L, P, u3, r, f, n);
    int64_t fb = 0, fl = 0;
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : fb, fl)
    for (int z = 0; z < P.nz; ++z)
        for (int y = 0; y < P.ny; ++y)
            for (int x = 0; x < P.nx; ++x) {
                const int64_t k = node_index(P, x, y, z);
                T g[27], post[27];
                for (int i = 0; i < Q; ++i) g[i] = f[i * n + k];
                double u[3];
                node_u(P, u3, n, k, u);
                const T* S = F.s_uniform ? &F.S[0] : &F.S[size_t(k) * 9];
                NodeInfo info;
                collide_node(L, P, g, S, u, post, &info);
                if (info.alpha < 1.0) ++fb;
                if (info.flagged) ++fl;
                if (lam_out) lam_out[k] = info.lambda;
                if (alpha_out) alpha_out[k] = info.alpha;
                // Streaming, Sec. 2.1: g_i(x + c_i, t + dt) = post_i(x).
                for (int i = 0; i < Q; ++i) {
                    int xd = x + L.c[i][0];
                    int yd = (y + L.c[i][1] + P.ny) % P.ny;
                    int zd = (z + L.c[i][2] + P.nz) % P.nz;
                    if (xd < 0 || xd >= P.nx) {
                        if (P.bc_x == 1) {
                            // Halfway anti-bounce-back at the Dirichlet plane: the population
                            // leaving through the wall returns as its opposite.
                            double phw = (xd < 0) ? P.phi_lo : P.phi_hi;
                            fnew[L.opp[i] * n + k] = -post[i] + 2.0 * L.w[i] * phw;
                            continue;
                        }
                        xd = (xd + P.nx) % P.nx;
                    }
                    fnew[i * n + node_index(P, xd, yd, zd)] = post[i];
                }
            }
    if (cnt) {
        cnt->fallback += fb;
        cnt->flagged += fl;
    }
    half_source(L, P, u3, r, fnew, n);
}

bool check_params(const oracle_params* p) {
    if (!p) return false;
    if (p->q != 19 && p->q != 27) return false;
    if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0) return false;
    if (p->bc_x != 0 && p->bc_x != 1) return false;
    if (p->r_mode < 0 || p->r_mode > 2) return false;
    return true;
}

void set_threads(const oracle_params* p) {
#ifdef _OPENMP
    if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#else
    (void)p;
#endif
}

}  // namespace

extern "C" {

// Velocity table of this oracle: c[q][3] and W[q]. Returns q, or -1.
int oracle_velocities(int32_t q, int32_t* c, double* w) {
    if (q != 19 && q != 27) return -1;
    Lattice L = make_lattice(q);
    for (int i = 0; i < L.q; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
        w[i] = L.w[i];
    }
    return L.q;
}

// S = (I/2 + D/(cs^2 dt))^-1 for one tensor (Sec. 2.3). s9 is the full 3x3 matrix.
int oracle_s_from_d(const double* d6, double* s9) {
    s_from_d(d6, s9);
    return 0;
}

// D = expm(L) for one symmetric tensor (6-vectors).
int oracle_expm_sym(const double* l6, double* d6) {
    expm_sym(l6, d6);
    return 0;
}

// Collide a batch of independent nodes (no streaming). g[m][q] in, out[m][q]; d6[m][6]
// (or one tensor if p->d_uniform), u3[m][3] (or one if p->u_uniform). info[m][4] (may be
// NULL) receives (lambda used, closed-form lambda, alpha, flagged).
int oracle_collide(const oracle_params* p, int64_t m, const double* g, const double* d6,
                   const double* u3, double* out, double* info) {
    if (!check_params(p)) return -1;
    Lattice L = make_lattice(p->q);
    for (int64_t k = 0; k < m; ++k) {
        double dd[6], S[9], u[3];
        for (int c = 0; c < 6; ++c) dd[c] = p->d_uniform ? d6[c] : d6[6 * k + c];
        if (p->tensor_is_log) {
            double l6[6];
            for (int c = 0; c < 6; ++c) l6[c] = dd[c];
            expm_sym(l6, dd);
        }
        s_from_d(dd, S);
        for (int a = 0; a < 3; ++a) u[a] = p->u_uniform ? u3[a] : u3[3 * k + a];
        NodeInfo ni;
        collide_node(L, *p, g + k * L.q, S, u, out + k * L.q, &ni);
        if (info) {
            info[4 * k + 0] = ni.lambda;
            info[4 * k + 1] = ni.lambda_lin;
            info[4 * k + 2] = ni.alpha;
            info[4 * k + 3] = ni.flagged;
        }
    }
    return 0;
}

// Advance f (pre-collision populations at t_n, [q][z][y][x]) by nsteps full steps in place.
// lam_last / alpha_last (may be NULL) receive the per-node lambda and alpha of the last step.
// counts (may be NULL) receives {nodes with alpha < 1, nodes flagged for the exact root}
// summed over all steps.
int oracle_run(const oracle_params* p, const double* d6, const double* u3, const double* r,
               double* f, int32_t nsteps, double* lam_last, double* alpha_last,
               int64_t* counts) {
    if (!check_params(p) || nsteps < 0) return -1;
    set_threads(p);
    Lattice L = make_lattice(p->q);
    const int64_t n = int64_t(p->nx) * p->ny * p->nz;
    Fields<double> F;
    build_s(*p, d6, n, &F);
    std::vector<double> tmp(static_cast<size_t>(L.q * n));
    double* a = f;
    double* b = tmp.data();
    Counts cnt;
    for (int s = 0; s < nsteps; ++s) {
        bool last = (s == nsteps - 1);
        step(L, *p, F, u3, r, a, b, last ? lam_last : nullptr, last ? alpha_last : nullptr, &cnt);
        std::swap(a, b);
    }
    if (a != f) std::memcpy(f, a, sizeof(double) * size_t(L.q) * n);
    if (counts) {
        counts[0] = cnt.fallback;
        counts[1] = cnt.flagged;
    }
    return 0;
}

// Forward-mode derivative of oracle_run: advances (f, df) where df is the tangent of the
// populations and dd6 the tangent of the tensor input (same layout as d6; the log tensor
// when p->tensor_is_log). Exact derivative of the discrete map along that direction.
int oracle_run_tangent(const oracle_params* p, const double* d6, const double* dd6,
                       const double* u3, const double* r, double* f, double* df,
                       int32_t nsteps) {
    if (!check_params(p) || nsteps < 0) return -1;
    set_threads(p);
    Lattice L = make_lattice(p->q);
    const int64_t n = int64_t(p->nx) * p->ny * p->nz;
    const int64_t nd = p->d_uniform ? 6 : 6 * n;
    std::vector<Dual> dd(static_cast<size_t>(nd));
    for (int64_t k = 0; k < nd; ++k) dd[k] = Dual(d6[k], dd6 ? dd6[k] : 0.0);
    Fields<Dual> F;
    build_s(*p, dd.data(), n, &F);
    std::vector<Dual> a(static_cast<size_t>(L.q * n)), b(static_cast<size_t>(L.q * n));
    for (int64_t k = 0; k < int64_t(L.q) * n; ++k) a[k] = Dual(f[k], df ? df[k] : 0.0);
    for (int s = 0; s < nsteps; ++s) {
        step(L, *p, F, u3, r, a.data(), b.data(), nullptr, nullptr, nullptr);
        std::swap(a, b);
    }
    for (int64_t k = 0; k < int64_t(L.q) * n; ++k) {
        f[k] = a[k].v;
        if (df) df[k] = a[k].d;
    }
    return 0;
}

// Macroscopic readout at the current time (Secs. 2.1, 4.2.2): phi = sum g_i,
// j = sum c_i (g_i - g_eq_i), q = (I - S/2) j. Outputs are planes [c][z][y][x]; any may be NULL.
int oracle_moments(const oracle_params* p, const double* d6, const double* u3, const double* f,
                   double* phi_out, double* j_out, double* q_out) {
    if (!check_params(p)) return -1;
    set_threads(p);
    Lattice L = make_lattice(p->q);
    const int64_t n = int64_t(p->nx) * p->ny * p->nz;
    Fields<double> F;
    build_s(*p, d6, n, &F);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double u[3];
        node_u(*p, u3, n, k, u);
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        double phi = 0.0;
        for (int i = 0; i < L.q; ++i) phi += f[i * n + k];
        double j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < L.q; ++i) {
            double cu = L.c[i][0] * u[0] + L.c[i][1] * u[1] + L.c[i][2] * u[2];
            double geq = phi * L.w[i] * (1.0 + cu / kCs2 + cu * cu / (2.0 * kCs2 * kCs2) - uu / (2.0 * kCs2));
            for (int a = 0; a < 3; ++a) j[a] += L.c[i][a] * (f[i * n + k] - geq);
        }
        const double* S = F.s_uniform ? &F.S[0] : &F.S[size_t(k) * 9];
        if (phi_out) phi_out[k] = phi;
        for (int a = 0; a < 3; ++a) {
            if (j_out) j_out[a * n + k] = j[a];
            if (q_out)
                q_out[a * n + k] = j[a] - 0.5 * (S[3 * a] * j[0] + S[3 * a + 1] * j[1] + S[3 * a + 2] * j[2]);
        }
    }
    return 0;
}

// Initial populations f = g_eq(phi0, u) (Sec. 2.1 equilibrium), optionally plus the flux lift
// P(j0) of a prescribed non-equilibrium flux j0 (planes [3][z][y][x], may be NULL).
int oracle_init_equilibrium(const oracle_params* p, const double* u3, const double* phi0,
                            const double* j0, double* f) {
    if (!check_params(p)) return -1;
    Lattice L = make_lattice(p->q);
    const int64_t n = int64_t(p->nx) * p->ny * p->nz;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double u[3];
        node_u(*p, u3, n, k, u);
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        double jj[3] = {0.0, 0.0, 0.0};
        if (j0)
            for (int a = 0; a < 3; ++a) jj[a] = j0[a * n + k];
        for (int i = 0; i < L.q; ++i) {
            double cu = L.c[i][0] * u[0] + L.c[i][1] * u[1] + L.c[i][2] * u[2];
            double geq = phi0[k] * L.w[i] * (1.0 + cu / kCs2 + cu * cu / (2.0 * kCs2 * kCs2) - uu / (2.0 * kCs2));
            f[i * n + k] = geq + lift(L, i, jj);
        }
    }
    return 0;
}

}  // extern "C"
