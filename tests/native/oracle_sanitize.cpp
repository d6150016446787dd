// Drives every entry point of the FP64 oracle on small inputs, for a build with the address
// and undefined-behaviour sanitizers (tests/test_oracle_sanitizers_cpu.py). The oracle source
// is compiled into this one translation unit. Exit status 0 and "SANITIZE-DRIVER OK" on
// success; a sanitizer finding aborts the run.
#include "../../oracle/elbm_oracle.cpp"

#include <cstdio>
#include <random>

namespace {

std::mt19937_64 rng(12345);
double uni(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

oracle_params params(int q, int nx, int ny, int nz, int bc, int d_uni, int u_uni, int r_mode, int is_log,
                     double root_rho) {
    oracle_params p{};
    p.q = q;
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.bc_x = bc;
    p.d_uniform = d_uni;
    p.u_uniform = u_uni;
    p.r_mode = r_mode;
    p.tensor_is_log = is_log;
    p.nthreads = 2;
    p.phi_lo = 1.3;
    p.phi_hi = 0.8;
    p.eps = 1e-4;
    p.tau = 1e-9;
    p.root_rho = root_rho;
    return p;
}

// diagonally dominant symmetric tensors (SPD), or logs of them
void tensors(std::vector<double>& d6, int64_t n, bool planes) {
    d6.assign(size_t(6 * n), 0.0);
    for (int64_t k = 0; k < n; ++k) {
        const double v[6] = {uni(1e-3, 1e-2), uni(-1e-4, 1e-4), uni(-1e-4, 1e-4), uni(1e-3, 1e-2),
                             uni(-1e-4, 1e-4), uni(1e-3, 1e-2)};
        for (int c = 0; c < 6; ++c) d6[planes ? size_t(c * n + k) : size_t(6 * k + c)] = v[c];
    }
}

int run_case(int q, int nx, int ny, int nz, int bc, bool fields, int r_mode, bool is_log, double root) {
    const int64_t n = int64_t(nx) * ny * nz;
    oracle_params p = params(q, nx, ny, nz, bc, fields ? 0 : 1, fields ? 0 : 1, r_mode, is_log ? 1 : 0, root);
    std::vector<double> d6, u3(fields ? size_t(3 * n) : 3), r(r_mode == 2 ? size_t(n) : 1), phi0(static_cast<size_t>(n));
    tensors(d6, fields ? n : 1, true);
    if (is_log)
        for (double& v : d6) v = (v > 1e-3 ? std::log(v) : v);
    for (double& v : u3) v = uni(-0.05, 0.05);
    for (double& v : r) v = uni(-1e-3, 1e-3);
    for (double& v : phi0) v = uni(0.7, 1.3);
    std::vector<double> f(size_t(q * n)), df(size_t(q * n)), dd6(d6.size());
    if (oracle_init_equilibrium(&p, u3.data(), phi0.data(), nullptr, f.data()) != 0) return 1;
    for (double& v : f) v *= uni(0.02, 1.98);  // far from equilibrium: fallback and root fire
    for (double& v : df) v = uni(-1.0, 1.0);
    for (double& v : dd6) v = uni(-1e-4, 1e-4);
    std::vector<double> lam(static_cast<size_t>(n)), alpha(static_cast<size_t>(n));
    int64_t counts[2] = {0, 0};
    std::vector<double> g = f;
    if (oracle_run(&p, d6.data(), u3.data(), r_mode ? r.data() : nullptr, g.data(), 4, lam.data(), alpha.data(),
                   counts) != 0)
        return 2;
    std::vector<double> gt = f, dgt = df;
    if (!root && oracle_run_tangent(&p, d6.data(), dd6.data(), u3.data(), r_mode ? r.data() : nullptr, gt.data(),
                                    dgt.data(), 3) != 0)
        return 3;
    std::vector<double> phi(static_cast<size_t>(n)), j(size_t(3 * n)), qf(size_t(3 * n));
    if (oracle_moments(&p, d6.data(), u3.data(), g.data(), phi.data(), j.data(), qf.data()) != 0) return 4;
    // node-level collision of m independent nodes (node-major tensors and velocities)
    const int64_t m = 5;
    oracle_params pc = params(q, 1, 1, 1, 0, 0, 0, 0, is_log ? 1 : 0, root);
    std::vector<double> gc(size_t(m * q)), dc, uc(size_t(3 * m)), out(size_t(m * q)), info(size_t(4 * m));
    for (int64_t k = 0; k < m; ++k)
        for (int i = 0; i < q; ++i) gc[size_t(k * q + i)] = f[size_t(i * n + k % n)];
    tensors(dc, m, false);
    for (double& v : uc) v = uni(-0.05, 0.05);
    if (oracle_collide(&pc, m, gc.data(), dc.data(), uc.data(), out.data(), info.data()) != 0) return 5;
    double sum = 0.0;
    for (double v : g) sum += v;
    for (double v : out) sum += v;
    if (!std::isfinite(sum)) return 6;
    std::printf("case q=%d %dx%dx%d bc=%d fields=%d r=%d log=%d root=%g: fallback %lld flagged %lld\n", q, nx, ny,
                nz, bc, int(fields), r_mode, int(is_log), root, (long long)counts[0], (long long)counts[1]);
    return 0;
}

}  // namespace

int main() {
    int c[81];
    double w[27], s9[9], l6[6] = {-4.0, 0.1, 0.0, -5.0, 0.2, -3.0}, d6[6];
    if (oracle_velocities(19, c, w) != 19 || oracle_velocities(27, c, w) != 27) return 10;
    oracle_expm_sym(l6, d6);
    oracle_s_from_d(d6, s9);
    int rc = 0;
    for (int q : {19, 27}) {
        rc |= run_case(q, 7, 5, 3, 0, true, 2, false, -1.0);
        rc |= run_case(q, 6, 4, 5, 1, true, 1, true, -1.0);
        rc |= run_case(q, 5, 3, 2, 1, false, 0, false, 0.3);
        rc |= run_case(q, 1, 6, 4, 0, true, 2, false, 1e300);
    }
    if (rc) {
        std::printf("SANITIZE-DRIVER FAILED rc=%d\n", rc);
        return rc;
    }
    std::printf("SANITIZE-DRIVER OK\n");
    return 0;
}
