// Per-node collision of the entropic anisotropic ADE scheme and its vector-Jacobian product.
//
// Inputs are deviations d_i = g_i - W_i phi_ref (the scalar phi = phi_ref + sum d_i), the
// node's equilibrium factors E_i(u) (second-order equilibrium, Sec. 2.1), r_i = 1/(W_i E_i),
// l_i = ln E_i, the velocity u and the retention tensor T = 2 I - S (Sec. 2.3 with
// S = (I/2 + 3 D)^-1; T = 12 D (I + 6 D)^-1 keeps the O(D) part exact in FP32).
//
// Algebra used (all exact rewrites of the paper's formulas):
//   g_eq_i - W_i phi_ref = W_i (dphi + phi (E_i - 1))                       (Sec. 2.1)
//   j = sum c_i g_i - phi u                                                 (Sec. 2.1)
//   Ds_i = P_i(j) = 3 W_i c_i.j,  Dh_i = g_i - g_eq_i - Ds_i                 (Sec. 2.2)
//   S j = 2 j - T j,  j* = (I - S) j = T j - j,  Om^(s) = -P(S j) = P(T j - 2 j)  (Sec. 2.3)
//   lambda - 1 = N / Dn with the H-products multiplied through by phi:
//     N  = sum Dh_i Ds*_i / (W_i E_i) + phi sum Dh_i ln E_i     (= phi (<Dh|Ds*>_H + C))
//     Dn = sum Dh_i^2 / (W_i E_i) + (tau phi)^2                 (= phi <Dh|Dh>_H + floor)
//   where C = sum Dh_i ln(g_eq_i / W_i) loses its ln(phi) part because sum Dh_i = 0
//   (Sec. 2.5, App. B); lambda = 1 when phi <= 0 or Dn = 0.
//   Om = Om^(s) - lambda Dh; alpha from the positivity fallback (Sec. 2.6); g + alpha Om.
#pragma once

#include "fmath.h"
#include "lattice.h"

namespace elbm {

template <class Real>
struct NodeCoef {
    Real u[3];
    Real ex[Q];  // E_i - 1 = 3 c_i.u + 4.5 (c_i.u)^2 - 1.5 u.u, kept apart from the 1
    Real r[Q];   // 1 / (W_i E_i)
    Real l[Q];   // ln E_i
    Real T[6];   // xx, xy, xz, yy, yz, zz
};

template <class Real>
struct NodeOut {
    Real dphi;    // sum of the input deviations (finite-input check)
    Real lam;
    Real alpha;
    int branch;   // 255: alpha = 1; 254: alpha clamped to 0; else the limiting direction
    int flagged;  // exact root taken
    int guard;    // lambda = 1 by the guard: phi <= 0 or a zero entropic denominator
};

__host__ __device__ constexpr double w3(int i) { return 3.0 * weight(i); }

// 1 / (W_i E_i) and ln E_i of the rest direction and of an opposite pair (P, P + 1) from
// their excesses E - 1. One reciprocal per pair: 1/E+ = E- / (E+ E-), 1/E- = E+ / (E+ E-).
// The step kernels evaluate these where the entropic sums use them, so that a velocity
// field does not keep 2 Q per-node factors live in registers; the adjoint stores them.
template <class Real>
__device__ __forceinline__ void rest_factors(Real ex0, Real& r0, Real& l0) {
    r0 = recip(Real(weight(0)) * (Real(1) + ex0));
    l0 = log1p_e(ex0);
}
// 1/E+ and 1/E- of an opposite pair from one reciprocal.
template <class Real>
__device__ __forceinline__ void pair_inverse(Real Ep, Real Em, Real& ip, Real& im) {
    const Real r = recip(Ep * Em);
    ip = Em * r;
    im = Ep * r;
}
template <class Real>
__device__ __forceinline__ void pair_factors(int P, Real exp, Real exm, Real& rp_out, Real& rm_out,
                                             Real& lp, Real& lm) {
    const Real Ep = Real(1) + exp, Em = Real(1) + exm;
    const Real rp = recip(Ep * Em) * Real(1.0 / weight(P));
    rp_out = Em * rp;
    rm_out = Ep * rp;
    lp = log1p_e(exp);
    lm = log1p_e(exm);
}

// Stationarity of the entropy along the ghost line (Sec. 2.5), solved in FP64 on the open
// interval where every trial population A_i - lambda h_i is positive. The function
// F(lambda) = sum h_i ln((A_i - lambda h_i) / W_i) decreases strictly from +inf to -inf on
// that interval, so safeguarded Newton steps inside a shrinking bracket converge to the
// unique root. Returns false (closed form kept) if the interval is empty.
__host__ __device__ inline bool entropic_root_fp64(const double (&A)[Q], const double (&h)[Q], double start,
                                          double* root) {
    double lo = -1.0e300, hi = 1.0e300;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (h[i] > 0.0) hi = fmin(hi, A[i] / h[i]);
        else if (h[i] < 0.0) lo = fmax(lo, A[i] / h[i]);
        else if (!(A[i] > 0.0)) return false;
    }
    if (!(lo < hi) || lo <= -1.0e300 || hi >= 1.0e300) return false;
    double x = (start > lo && start < hi) ? start : 0.5 * (lo + hi);
    double a = lo, b = hi;
    for (int it = 0; it < 200; ++it) {
        double F = 0.0, dF = 0.0;
        bool inside = true;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double gs = A[i] - x * h[i];
            inside = inside && (gs > 0.0);
            F += h[i] * log(fmax(gs, 1e-300) / weight(i));
            dF -= h[i] * h[i] / fmax(gs, 1e-300);
        }
        if (!inside) {
            x = 0.5 * (a + b);
            continue;
        }
        if (F == 0.0) break;
        const double newton = F / dF;
        if (fabs(newton) <= 1e-15 * fmax(1.0, fabs(x))) {
            x -= newton;
            break;
        }
        if (F > 0.0) a = x; else b = x;  // the root stays inside (a, b)
        double xn = x - newton;
        if (!(xn > a && xn < b)) xn = 0.5 * (a + b);
        x = xn;
    }
    *root = x;
    return true;
}

// c_i . (a0, a1, a2) using only the nonzero velocity components (i is a compile-time
// constant after unrolling; no multiplications by 0 or +-1 are emitted).
template <class Real>
__host__ __device__ inline Real cdot(int i, Real a0, Real a1, Real a2) {
    Real r = Real(0);
    bool any = false;
    if (cx(i)) {
        r = cx(i) > 0 ? a0 : -a0;
        any = true;
    }
    if (cy(i)) {
        r = any ? (cy(i) > 0 ? r + a1 : r - a1) : (cy(i) > 0 ? a1 : -a1);
        any = true;
    }
    if (cz(i)) r = any ? (cz(i) > 0 ? r + a2 : r - a2) : (cz(i) > 0 ? a2 : -a2);
    return r;
}

// Collision of one node (D3Q19 or D3Q27). d: collision input (deviations, sources already
// added).
// post: output deviations g + alpha Om (not yet streamed). UM = 0 is the zero-velocity
// specialisation (E_i = 1, ln E_i = 0, 1/(W_i E_i) = 1/W_i folded at compile time). ROOT
// selects the variant that takes the exact entropic root at nodes flagged by root_rho (a
// separate instantiation, so the FP64 solver's registers do not weigh on the others).
// Opposite directions come in pairs (P, P + 1) with P odd: their flux parts are opposite.
//
// CMASS (FP32 storage): the mass sum is compensated. Its rounding, not the populations',
// sets the FP32 mass error: the collision keeps the node's computed sum, so each step moves
// the mass by the rounding of dphi (half an ulp of phi, against half an ulp of one
// population for the stores). The 19 FP32 deviations are summed in FP64 and the per-class
// equilibrium terms W_m dphi are rounded once from that sum.
//
// LOGC = false (16-bit storage, UM = 2): the logarithms of the node's factors E_i are taken of
// fl(E_i) without the rounding correction. Each ln E_i moves by at most about 2^-24, which
// changes lambda by at most 2^-24 phi sum_i |Dh_i| / Dn and so, by Cauchy-Schwarz with
// sum_i W_i E_i = 1, each output population by at most 2^-24 phi (W_i E_i)^(1/2): below an
// ulp of phi in FP32, against 2^-9 or 2^-12 of a population for the 16-bit stores.
template <class Real, int UM, bool ROOT, bool CMASS = false, bool LOGC = true>
__host__ __device__ inline void collide(const Real (&d)[Q], const NodeCoef<Real>& c, Real phi_ref,
                                        Real eps, Real tau2, Real root_rho, Real (&post)[Q],
                                        NodeOut<Real>& o) {
    // zeroth moment and non-equilibrium flux from pair sums and differences
    Real pm[Q];
#pragma unroll
    for (int P = 1; P < Q; P += 2) pm[P] = d[P] - d[P + 1];
    // CMASS: the pair sums and their tree in FP64 (exact for FP32 inputs whose magnitudes
    // lie within 2^29 of each other), rounded to FP32 once
    using Acc = typename std::conditional<CMASS, double, Real>::type;
    Acc ps[Q];
#pragma unroll
    for (int P = 1; P < Q; P += 2) ps[P] = Acc(d[P]) + Acc(d[P + 1]);
    Acc psum;
    if constexpr (Q == 19)
        psum = ((ps[1] + ps[3]) + (ps[5] + ps[7])) + ((ps[9] + ps[11]) + (ps[13] + ps[15])) + ps[17];
    else
        psum = (((ps[1] + ps[3]) + (ps[5] + ps[7])) + ((ps[9] + ps[11]) + (ps[13] + ps[15]))) +
               (((ps[17] + ps[19]) + (ps[21] + ps[23])) + ps[25]);
    const Acc dphi_acc = Acc(d[0]) + psum;
    const Real dphi = Real(dphi_acc);
    const Real phi = phi_ref + dphi;
    o.dphi = dphi;
    Real j0 = Real(0), j1 = Real(0), j2 = Real(0);
    bool f0 = false, f1 = false, f2 = false;
#pragma unroll
    for (int P = 1; P < Q; P += 2) {
        if (cx(P)) { j0 = f0 ? (cx(P) > 0 ? j0 + pm[P] : j0 - pm[P]) : (cx(P) > 0 ? pm[P] : -pm[P]); f0 = true; }
        if (cy(P)) { j1 = f1 ? (cy(P) > 0 ? j1 + pm[P] : j1 - pm[P]) : (cy(P) > 0 ? pm[P] : -pm[P]); f1 = true; }
        if (cz(P)) { j2 = f2 ? (cz(P) > 0 ? j2 + pm[P] : j2 - pm[P]) : (cz(P) > 0 ? pm[P] : -pm[P]); f2 = true; }
    }
    if (UM != 0) {
        j0 -= phi * c.u[0];
        j1 -= phi * c.u[1];
        j2 -= phi * c.u[2];
    }
    // ghost residual Dh_i = d_i - P_i(j) - (g_eq_i - W_i phi_ref). At u = 0 the equilibrium
    // term W_m dphi is rounded once per velocity class and subtracted first, so that it
    // cancels exactly in the pair differences Dh_P - Dh_P' (there the entropic numerator is
    // zero up to rounding, which the closed-form lambda divides by the small ghost norm);
    // with a velocity the equilibrium term is W_m dphi + (W_m phi)(E_i - 1), both products
    // formed once per class, one multiply-add per direction.
    Real dh[Q];
    Real wd[NCLASS], wp[NCLASS];
#pragma unroll
    for (int m = 0; m < NCLASS; ++m) {
        wd[m] = CMASS ? Real(class_weight(m) * double(dphi_acc)) : Real(class_weight(m)) * dphi;
        wp[m] = Real(class_weight(m)) * phi;
    }
    if (UM == 0) dh[0] = d[0] - wd[0];
    else dh[0] = d[0] - (wp[0] * c.ex[0] + wd[0]);
#pragma unroll
    for (int P = 1; P < Q; P += 2) {
        const Real B = Real(w3(P)) * cdot(P, j0, j1, j2);
        const int m = vclass(P);
        if (UM == 0) {
            dh[P] = (d[P] - wd[m]) - B;
            dh[P + 1] = (d[P + 1] - wd[m]) + B;
        } else {
            dh[P] = (d[P] - B) - (wp[m] * c.ex[P] + wd[m]);
            dh[P + 1] = (d[P + 1] + B) - (wp[m] * c.ex[P + 1] + wd[m]);
        }
    }
    // tensorial relaxation through T = 2 I - S: j* = T j - j, -S j = T j - 2 j
    const Real t0 = c.T[0] * j0 + c.T[1] * j1 + c.T[2] * j2;
    const Real t1 = c.T[1] * j0 + c.T[3] * j1 + c.T[4] * j2;
    const Real t2 = c.T[2] * j0 + c.T[4] * j1 + c.T[5] * j2;
    const Real s0 = t0 - j0, s1 = t1 - j1, s2 = t2 - j2;
    const Real v0 = s0 - j0, v1 = s1 - j1, v2 = s2 - j2;
    // entropic amplitude: N = sum Dh_i Ds*_i / (W_i E_i) + phi sum Dh_i ln E_i,
    // Dn = sum Dh_i^2 / (W_i E_i) + (tau phi)^2; Ds*_opp = -Ds*
    Real N, Dn;
    if (UM == 0) {
        // Ds*_i / W_i = 3 c_i . j*; sums per velocity class m (weights W_m)
        Real nc[NCLASS], dc[NCLASS];
#pragma unroll
        for (int m = 0; m < NCLASS; ++m) nc[m] = dc[m] = Real(0);
#pragma unroll
        for (int P = 1; P < Q; P += 2) {
            const Real q = cdot(P, s0, s1, s2);
            const Real hd = dh[P] - dh[P + 1];
            nc[vclass(P)] += hd * q;
            dc[vclass(P)] += dh[P] * dh[P] + dh[P + 1] * dh[P + 1];
        }
        Real ns = nc[1] + nc[2];
        Dn = Real(1.0 / class_weight(0)) * dh[0] * dh[0] + Real(1.0 / class_weight(1)) * dc[1] +
             Real(1.0 / class_weight(2)) * dc[2];
        if constexpr (NCLASS == 4) {
            ns += nc[3];
            Dn += Real(1.0 / class_weight(3)) * dc[3];
        }
        N = Real(3) * ns;
    } else {
        // the same sums with 1/E_i and per-class weights: with e_i = 1/E_i,
        //   N  = 3 sum_P (c_P . j*) (Dh_P e_P - Dh_P' e_P') + phi sum_i Dh_i ln E_i,
        //   Dn = sum_m (1 / W_m) sum_{i in class m} Dh_i^2 e_i.
        // UM = 1: the uniform velocity's 1/(W_i E_i) and ln E_i from the kernel arguments;
        // UM = 2: the node's factors, evaluated here pair by pair
        Real nc[NCLASS], dc[NCLASS];
#pragma unroll
        for (int m = 0; m < NCLASS; ++m) nc[m] = dc[m] = Real(0);
        Log1pSum<Real, LOGC> lg;
        Real Lg = Real(0);
        {
            Real e0;
            if constexpr (UM == 2) {
                e0 = recip(Real(1) + c.ex[0]);
                lg.add(dh[0], c.ex[0]);
            } else {
                e0 = c.r[0] * Real(weight(0));
                Lg = dh[0] * c.l[0];
            }
            dc[0] = dh[0] * dh[0] * e0;
        }
#pragma unroll
        for (int P = 1; P < Q; P += 2) {
            Real ep, em;
            if constexpr (UM == 2) {
                pair_inverse(Real(1) + c.ex[P], Real(1) + c.ex[P + 1], ep, em);
                lg.add(dh[P], c.ex[P]);
                lg.add(dh[P + 1], c.ex[P + 1]);
            } else {
                ep = c.r[P] * Real(weight(P));
                em = c.r[P + 1] * Real(weight(P));
                Lg += dh[P] * c.l[P] + dh[P + 1] * c.l[P + 1];
            }
            const Real a = dh[P] * ep, b = dh[P + 1] * em;
            nc[vclass(P)] += cdot(P, s0, s1, s2) * (a - b);
            dc[vclass(P)] += a * dh[P] + b * dh[P + 1];
        }
        if constexpr (UM == 2) Lg = lg.value();
        Real ns = nc[1] + nc[2];
        Dn = Real(1.0 / class_weight(0)) * dc[0] + Real(1.0 / class_weight(1)) * dc[1] +
             Real(1.0 / class_weight(2)) * dc[2];
        if constexpr (NCLASS == 4) {
            ns += nc[3];
            Dn += Real(1.0 / class_weight(3)) * dc[3];
        }
        N = Real(3) * ns + phi * Lg;
    }
    Dn += tau2 * phi * phi;
    o.guard = !(phi > Real(0) && Dn > Real(0));
    Real lam = o.guard ? Real(1) : Real(1) + N / Dn;
    o.flagged = 0;
    if (ROOT && phi > Real(0)) {
        bool flag = false;
        double A[Q], h[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const Real E = (UM == 0) ? Real(1) : Real(1) + c.ex[i];
            const Real geq = Real(weight(i)) * phi * E;
            const Real dsp = (i == 0) ? Real(0) : Real(w3(i)) * cdot(i, s0, s1, s2);
            flag = flag || (dsp + (Real(1) - lam) * dh[i] < (root_rho - Real(1)) * geq);
            A[i] = double(geq) + double(dsp) + double(dh[i]);
            h[i] = double(dh[i]);
        }
        if (flag) {
            o.flagged = 1;
            double lr;
            if (entropic_root_fp64(A, h, double(lam), &lr)) lam = Real(lr);
        }
    }
    // increment Om_i = -3 W_i c_i . (S j) - lam Dh_i and the fallback test:
    // every g_i + Om_i >= eps  <=>  alpha = 1
    Real X[Q];
    X[0] = Real(0);
#pragma unroll
    for (int P = 1; P < Q; P += 2) {
        X[P] = Real(w3(P)) * cdot(P, v0, v1, v2);
        X[P + 1] = -X[P];
    }
    // smallest post-collision deviation per velocity class, against eps - W_m phi_ref (each
    // class minimum starts at the class's first value, so no constant enters the test)
    Real mn[NCLASS];
    bool seen[NCLASS];
#pragma unroll
    for (int m = 0; m < NCLASS; ++m) seen[m] = false;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        post[i] = (d[i] + X[i]) - lam * dh[i];
        const int m = vclass(i);
        mn[m] = seen[m] ? fmin(mn[m], post[i]) : post[i];
        seen[m] = true;
    }
    bool all_ok = true;
#pragma unroll
    for (int m = 0; m < NCLASS; ++m) all_ok = all_ok && (mn[m] >= eps - Real(class_weight(m)) * phi_ref);
    o.lam = lam;
    o.alpha = Real(1);
    o.branch = 255;
    if (!all_ok) {
        // some population would end below eps: alpha = min over Om_i < 0 of (g_i - eps)/(-Om_i).
        // The minimum is found without a division per direction: with positive denominators,
        // num / den < bn / bd exactly when num bd < bn den, so the running best is kept as a
        // fraction (starting at 1 / 1) and divided once. Up to rounding of the two products
        // this is the same choice; where two ratios tie within rounding either direction
        // gives the same alpha to rounding.
        Real bn = Real(1), bd = Real(1);
        int br = 255;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const Real om = X[i] - lam * dh[i];
            if (om < Real(0)) {
                const Real num = d[i] + Real(weight(i)) * phi_ref - eps;
                const Real den = -om;
                if (num * bd < bn * den) {
                    bn = num;
                    bd = den;
                    br = i;
                }
            }
        }
        Real alpha = (br == 255) ? Real(1) : bn / bd;
        if (!(alpha < Real(1))) {
            // a ratio below 1 that rounds to 1: no fallback, as a per-direction division
            // would have found
            alpha = Real(1);
            br = 255;
        }
        if (alpha < Real(0)) {
            alpha = Real(0);
            br = 254;
        }
        o.alpha = alpha;
        o.branch = br;
#pragma unroll
        for (int i = 0; i < Q; ++i) post[i] = d[i] + alpha * (X[i] - lam * dh[i]);
    }
}

// Vector-Jacobian product of `collide` (closed-form lambda). ph: dL/dpost; lam_rec and
// branch: the forward step's recorded amplitude and fallback branch. Outputs dL/dd in dd
// and dL/dT (derivatives with respect to the 6 stored components) in tg.
template <class Real>
__host__ __device__ inline void collide_vjp(const Real (&d)[Q], const NodeCoef<Real>& c, Real phi_ref,
                                   Real eps, Real tau2, Real lam_rec, int branch,
                                   const Real (&ph)[Q], Real (&dd)[Q], Real (&tg)[6]) {
    // ---- forward recomputation ----
    Real dphi = Real(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) dphi += d[i];
    const Real phi = phi_ref + dphi;
    Real j0 = Real(0), j1 = Real(0), j2 = Real(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (cx(i)) j0 += Real(cx(i)) * d[i];
        if (cy(i)) j1 += Real(cy(i)) * d[i];
        if (cz(i)) j2 += Real(cz(i)) * d[i];
    }
    j0 -= phi * c.u[0];
    j1 -= phi * c.u[1];
    j2 -= phi * c.u[2];
    Real dh[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const Real wi = Real(weight(i));
        const Real cj = Real(cx(i)) * j0 + Real(cy(i)) * j1 + Real(cz(i)) * j2;
        dh[i] = d[i] - wi * (dphi + phi * c.ex[i]) - Real(w3(i)) * cj;
    }
    const Real t0 = c.T[0] * j0 + c.T[1] * j1 + c.T[2] * j2;
    const Real t1 = c.T[1] * j0 + c.T[3] * j1 + c.T[4] * j2;
    const Real t2 = c.T[2] * j0 + c.T[4] * j1 + c.T[5] * j2;
    const Real s0 = t0 - j0, s1 = t1 - j1, s2 = t2 - j2;
    const Real v0 = s0 - j0, v1 = s1 - j1, v2 = s2 - j2;
    Real N = Real(0), Lg = Real(0), Dn = Real(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const Real dsp = Real(w3(i)) * (Real(cx(i)) * s0 + Real(cy(i)) * s1 + Real(cz(i)) * s2);
        N += dh[i] * dsp * c.r[i];
        Lg += dh[i] * c.l[i];
        Dn += dh[i] * dh[i] * c.r[i];
    }
    N += phi * Lg;
    Dn += tau2 * phi * phi;
    const bool lam_active = (phi > Real(0) && Dn > Real(0));
    const Real lam = lam_rec;
    Real om[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i)
        om[i] = Real(w3(i)) * (Real(cx(i)) * v0 + Real(cy(i)) * v1 + Real(cz(i)) * v2) - lam * dh[i];
    Real alpha = Real(1);
    if (branch == 254) alpha = Real(0);
    Real omk = Real(-1), gk = Real(0);
    if (branch < Q) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
            if (i == branch) {
                omk = om[i];
                gk = d[i] + Real(weight(i)) * phi_ref - eps;
            }
        alpha = gk / (-omk);
    }
    // ---- reverse sweep ----
    Real ahat = Real(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        ahat += ph[i] * om[i];
        dd[i] = ph[i];
    }
    Real omh[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) omh[i] = alpha * ph[i];
    if (branch < Q) {
        // alpha = (g_k - eps) / (-Om_k)
        const Real inv = Real(1) / (-omk);
#pragma unroll
        for (int i = 0; i < Q; ++i)
            if (i == branch) {
                dd[i] += ahat * inv;
                omh[i] += ahat * alpha * inv;
            }
    }
    // Om_i = 3 W_i c_i . v - lam Dh_i
    Real vh0 = Real(0), vh1 = Real(0), vh2 = Real(0), lamh = Real(0);
    Real dhh[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const Real a = Real(w3(i)) * omh[i];
        vh0 += Real(cx(i)) * a;
        vh1 += Real(cy(i)) * a;
        vh2 += Real(cz(i)) * a;
        lamh -= omh[i] * dh[i];
        dhh[i] = -lam * omh[i];
    }
    // lam = 1 + N / Dn
    Real Nh = Real(0), Dnh = Real(0);
    if (lam_active) {
        const Real rD = Real(1) / Dn;
        Nh = lamh * rD;
        Dnh = -Nh * N * rD;
    }
    Real phih = Real(0), sh0 = Real(0), sh1 = Real(0), sh2 = Real(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const Real dsp = Real(w3(i)) * (Real(cx(i)) * s0 + Real(cy(i)) * s1 + Real(cz(i)) * s2);
        dhh[i] += Nh * (dsp * c.r[i] + phi * c.l[i]) + Dnh * Real(2) * dh[i] * c.r[i];
        const Real dsph = Nh * dh[i] * c.r[i];
        sh0 += Real(cx(i)) * Real(w3(i)) * dsph;
        sh1 += Real(cy(i)) * Real(w3(i)) * dsph;
        sh2 += Real(cz(i)) * Real(w3(i)) * dsph;
    }
    phih += Nh * Lg + Dnh * Real(2) * tau2 * phi;
    // j* = T j - j, v = T j - 2 j
    const Real th0 = vh0 + sh0, th1 = vh1 + sh1, th2 = vh2 + sh2;
    Real jh0 = -Real(2) * vh0 - sh0 + c.T[0] * th0 + c.T[1] * th1 + c.T[2] * th2;
    Real jh1 = -Real(2) * vh1 - sh1 + c.T[1] * th0 + c.T[3] * th1 + c.T[4] * th2;
    Real jh2 = -Real(2) * vh2 - sh2 + c.T[2] * th0 + c.T[4] * th1 + c.T[5] * th2;
    tg[0] = th0 * j0;
    tg[1] = th0 * j1 + th1 * j0;
    tg[2] = th0 * j2 + th2 * j0;
    tg[3] = th1 * j1;
    tg[4] = th1 * j2 + th2 * j1;
    tg[5] = th2 * j2;
    // Dh_i = d_i - W_i E_i dphi - W_i phi_ref (E_i - 1) - 3 W_i c_i . j
    Real dphih = Real(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        dd[i] += dhh[i];
        dphih -= Real(weight(i)) * (Real(1) + c.ex[i]) * dhh[i];
        const Real a = Real(w3(i)) * dhh[i];
        jh0 -= Real(cx(i)) * a;
        jh1 -= Real(cy(i)) * a;
        jh2 -= Real(cz(i)) * a;
    }
    // j = sum c_i d_i - phi u;  phi = phi_ref + dphi;  dphi = sum d_i
    phih -= c.u[0] * jh0 + c.u[1] * jh1 + c.u[2] * jh2;
    dphih += phih;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        dd[i] += Real(cx(i)) * jh0 + Real(cy(i)) * jh1 + Real(cz(i)) * jh2 + dphih;
}

}  // namespace elbm
