// Device code of the third-order BGK flux at one Gauss point (section 2.2).
//
// Frame: x along the face normal (from the left/owner side L to the right
// side R), y along the tangent, origin at the Gauss point (so y = 0).
// States W = (rho, rho U, rho V, E) with U normal, V tangential.
//
// A slope vector a[4] stands for the velocity polynomial
//   a.psi = a0 + a1 u + a2 v + a3 (u^2 + v^2 + xi^2) / 2        (Eq. macroVar)
// i.e. the x-, y- or t-derivative of ln g of Eq. Nomenclature1.
//
// Every flux term of the time-integrated Eqs. 3orderg:2 and 3orderf0:2 (at
// y = 0) has the shape  coefficient(t) x g x (product of at most two slope
// polynomials) x u^i v^j.  Writing r = u a1.psi + v a2.psi and
// s2 = u^2 a11.psi + 2 u v a12.psi + v^2 a22.psi, each of the three
// distributions (equilibrium g_0, left half u > 0, right half u < 0)
// contributes  rho < u psi P >  with
//   P = c0 + cr r + cA A + crr r^2 + crA r A + cs s2 + c1 (u A1 + v A2)
//       + cAA A^2 + cAt At,
// whose coefficients are the time integrals of c_1..c_8 of Eq.
// Nomenclature2 combined as listed in flux_coefficients().  P is held in
// monomials u^a v^b (xi^2)^c (a + b + 2c <= 6) and contracted against the
// factorised Maxwellian moments one factor at a time.
#pragma once

#include <hip/hip_runtime.h>

// Callable from host code too, so a CPU build of this file can be checked
// against the oracle without a GPU.
#define GKS_HD __host__ __device__ __forceinline__

namespace gksdev {

constexpr int PD = 7;   // u and v exponents 0..6
constexpr int PC = 3;   // xi^2 exponents 0..2 (products of two slope polynomials)

struct VPoly {
    double c[PD][PD][PC];
};

// Monomials of a.psi: 1, u, v, u^2, v^2, xi^2 (coefficients a0, a1, a2 and
// a3/2 for the last three).
constexpr int TA[6] = {0, 1, 0, 2, 0, 0};
constexpr int TB[6] = {0, 0, 1, 0, 2, 0};
constexpr int TC[6] = {0, 0, 0, 0, 0, 1};

GKS_HD double psi_coef(const double a[4], int i) {
    return i < 3 ? a[i] : 0.5 * a[3];
}

template <int D>
GKS_HD void vp_zero(VPoly& P) {
#pragma unroll
    for (int a = 0; a <= D; ++a)
#pragma unroll
        for (int b = 0; b <= D - a; ++b)
#pragma unroll
            for (int c = 0; 2 * c <= D - a - b && c < PC; ++c) P.c[a][b][c] = 0.0;
}

// P += s u^EU v^EV (a.psi)
template <int EU, int EV>
GKS_HD void vp_add1(VPoly& P, double s, const double a[4]) {
#pragma unroll
    for (int i = 0; i < 6; ++i) P.c[TA[i] + EU][TB[i] + EV][TC[i]] += s * psi_coef(a, i);
}

// P += s u^EU v^EV (a.psi)(b.psi)
template <int EU, int EV>
GKS_HD void vp_add2(VPoly& P, double s, const double a[4], const double b[4]) {
    double sa[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) sa[i] = s * psi_coef(a, i);
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j)
            P.c[TA[i] + TA[j] + EU][TB[i] + TB[j] + EV][TC[i] + TC[j]] += sa[i] * psi_coef(b, j);
}

// Moments of u, v and xi^2 of a normalised Maxwellian (full line or a half
// line for u).
struct Mom {
    double u[10];
    double v[10];
    double x[4];
};

// <u^n> for n = 0..N on the full line: <u^{n+2}> = U <u^{n+1}> + (n+1)/(2 lam) <u^n>
template <int N>
GKS_HD void line_moments(double* m, double U, double lam, double m0, double m1) {
    const double il = 0.5 / lam;
    m[0] = m0;
    m[1] = m1;
#pragma unroll
    for (int n = 0; n + 2 <= N; ++n) m[n + 2] = U * m[n + 1] + (n + 1) * il * m[n];
}

GKS_HD void xi_moments(double* x, double lam, double K) {
    const double il = 0.5 / lam;
    x[0] = 1.0;
    x[1] = K * il;
    x[2] = K * (K + 2.0) * il * il;
    x[3] = K * (K + 2.0) * (K + 4.0) * il * il * il;
}

struct Prim {
    double rho, U, V, lam;
};

GKS_HD Prim primitives(const double W[4], double K) {
    Prim p;
    p.rho = W[0];
    const double ir = 1.0 / W[0];
    p.U = W[1] * ir;
    p.V = W[2] * ir;
    p.lam = (K + 2.0) * W[0] / (4.0 * (W[3] - 0.5 * W[0] * (p.U * p.U + p.V * p.V)));
    return p;
}

template <int NU>
GKS_HD void full_moments(Mom& M, const Prim& p, double K) {
    line_moments<NU>(M.u, p.U, p.lam, 1.0, p.U);
    line_moments<NU>(M.v, p.V, p.lam, 1.0, p.V);
    xi_moments(M.x, p.lam, K);
}

// half line: u > 0 for sign = +1, u < 0 for sign = -1
template <int NU>
GKS_HD void half_moments(Mom& M, const Prim& p, double K, double sign) {
    const double sl = sqrt(p.lam);
    const double m0 = 0.5 * erfc(-sign * sl * p.U);
    const double m1 = p.U * m0 + sign * exp(-p.lam * p.U * p.U) / (2.0 * sqrt(M_PI * p.lam));
    line_moments<NU>(M.u, p.U, p.lam, m0, m1);
    line_moments<NU>(M.v, p.V, p.lam, 1.0, p.V);
    xi_moments(M.x, p.lam, K);
}

// D_alpha = <psi_alpha P> for a polynomial of degree <= D
template <int D>
GKS_HD void psi_moments(double out[4], const VPoly& P, const Mom& M) {
    double f0 = 0.0, f1 = 0.0, f2 = 0.0, f3 = 0.0;
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        double r0 = 0.0, rv1 = 0.0, rv2 = 0.0, rx = 0.0;
#pragma unroll
        for (int b = 0; b <= D - a; ++b) {
            double q0 = 0.0, q1 = 0.0;
#pragma unroll
            for (int c = 0; 2 * c <= D - a - b && c < PC; ++c) {
                q0 += P.c[a][b][c] * M.x[c];
                q1 += P.c[a][b][c] * M.x[c + 1];
            }
            r0 += q0 * M.v[b];
            rv1 += q0 * M.v[b + 1];
            rv2 += q0 * M.v[b + 2];
            rx += q1 * M.v[b];
        }
        f0 += r0 * M.u[a];
        f1 += r0 * M.u[a + 1];
        f2 += rv1 * M.u[a];
        f3 += r0 * M.u[a + 2] + (rv2 + rx) * M.u[a];
    }
    out[0] = f0;
    out[1] = f1;
    out[2] = f2;
    out[3] = 0.5 * f3;
}

// F_alpha += s <u psi_alpha P> for a polynomial of degree <= D (D <= 6)
template <int D>
GKS_HD void flux_moments(double F[4], double s, const VPoly& P, const Mom& M) {
    double f0 = 0.0, f1 = 0.0, f2 = 0.0, f3 = 0.0;
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        double r0 = 0.0, rv1 = 0.0, rv2 = 0.0, rx = 0.0;
#pragma unroll
        for (int b = 0; b <= D - a; ++b) {
            double q0 = 0.0, q1 = 0.0;
#pragma unroll
            for (int c = 0; 2 * c <= D - a - b && c < PC; ++c) {
                q0 += P.c[a][b][c] * M.x[c];
                q1 += P.c[a][b][c] * M.x[c + 1];
            }
            r0 += q0 * M.v[b];
            rv1 += q0 * M.v[b + 1];
            rv2 += q0 * M.v[b + 2];
            rx += q1 * M.v[b];
        }
        f0 += r0 * M.u[a + 1];
        f1 += r0 * M.u[a + 2];
        f2 += rv1 * M.u[a + 1];
        f3 += r0 * M.u[a + 3] + (rv2 + rx) * M.u[a + 1];
    }
    F[0] += s * f0;
    F[1] += s * f1;
    F[2] += s * f2;
    F[3] += s * 0.5 * f3;
}

// Closed-form solution a of rho <psi (a.psi)> = D for a full Maxwellian.
GKS_HD void slope_solve(double a[4], const double D[4], const Prim& p, double K) {
    const double ir = 1.0 / p.rho;
    const double R2 = (D[1] - p.U * D[0]) * ir;
    const double R3 = (D[2] - p.V * D[0]) * ir;
    const double q = p.U * p.U + p.V * p.V + (K + 2.0) / (2.0 * p.lam);
    const double R4 = 2.0 * D[3] * ir - q * D[0] * ir;
    a[3] = 4.0 * p.lam * p.lam / (K + 2.0) * (R4 - 2.0 * p.U * R2 - 2.0 * p.V * R3);
    a[2] = 2.0 * p.lam * R3 - p.V * a[3];
    a[1] = 2.0 * p.lam * R2 - p.U * a[3];
    a[0] = D[0] * ir - p.U * a[1] - p.V * a[2] - 0.5 * a[3] * q;
}

struct Slopes {
    double a1[4], a2[4], a11[4], a12[4], a22[4], A[4], A1[4], A2[4], At[4];
};

// Derivatives of a side: index 0 = n, 1 = t, 2 = nn, 3 = nt, 4 = tt.
// Slopes of Eq. Nomenclature1: a1, a2 from the first derivatives; a11, a12,
// a22 from d^2 g = g (a a + a_ij); A and its x-, y-, t-derivatives from the
// Euler-level compatibility <psi (u a1 + v a2 + A)> = 0 differentiated.
template <bool WITH_AT>
GKS_HD void side_slopes(Slopes& s, const double d[5][4], const Prim& p, const Mom& M,
                                            double K) {
    VPoly P;
    double D[4];
    slope_solve(s.a1, d[0], p, K);
    slope_solve(s.a2, d[1], p, K);

    vp_zero<4>(P);
    vp_add2<0, 0>(P, 1.0, s.a1, s.a1);
    psi_moments<4>(D, P, M);
#pragma unroll
    for (int q = 0; q < 4; ++q) D[q] = d[2][q] - p.rho * D[q];
    slope_solve(s.a11, D, p, K);

    vp_zero<4>(P);
    vp_add2<0, 0>(P, 1.0, s.a1, s.a2);
    psi_moments<4>(D, P, M);
#pragma unroll
    for (int q = 0; q < 4; ++q) D[q] = d[3][q] - p.rho * D[q];
    slope_solve(s.a12, D, p, K);

    vp_zero<4>(P);
    vp_add2<0, 0>(P, 1.0, s.a2, s.a2);
    psi_moments<4>(D, P, M);
#pragma unroll
    for (int q = 0; q < 4; ++q) D[q] = d[4][q] - p.rho * D[q];
    slope_solve(s.a22, D, p, K);

    vp_zero<3>(P);
    vp_add1<1, 0>(P, 1.0, s.a1);
    vp_add1<0, 1>(P, 1.0, s.a2);
    psi_moments<3>(D, P, M);
#pragma unroll
    for (int q = 0; q < 4; ++q) D[q] = -p.rho * D[q];
    slope_solve(s.A, D, p, K);

    // A1: -<psi [u a11 + v a12 + a1 (u a1 + v a2 + A)]>
    vp_zero<5>(P);
    vp_add1<1, 0>(P, 1.0, s.a11);
    vp_add1<0, 1>(P, 1.0, s.a12);
    vp_add2<1, 0>(P, 1.0, s.a1, s.a1);
    vp_add2<0, 1>(P, 1.0, s.a1, s.a2);
    vp_add2<0, 0>(P, 1.0, s.a1, s.A);
    psi_moments<5>(D, P, M);
#pragma unroll
    for (int q = 0; q < 4; ++q) D[q] = -p.rho * D[q];
    slope_solve(s.A1, D, p, K);

    // A2: -<psi [u a12 + v a22 + a2 (u a1 + v a2 + A)]>
    vp_zero<5>(P);
    vp_add1<1, 0>(P, 1.0, s.a12);
    vp_add1<0, 1>(P, 1.0, s.a22);
    vp_add2<1, 0>(P, 1.0, s.a2, s.a1);
    vp_add2<0, 1>(P, 1.0, s.a2, s.a2);
    vp_add2<0, 0>(P, 1.0, s.a2, s.A);
    psi_moments<5>(D, P, M);
#pragma unroll
    for (int q = 0; q < 4; ++q) D[q] = -p.rho * D[q];
    slope_solve(s.A2, D, p, K);

    if constexpr (WITH_AT) {
        // At: -<psi [u A1 + v A2 + A (u a1 + v a2 + A)]>
        vp_zero<5>(P);
        vp_add1<1, 0>(P, 1.0, s.A1);
        vp_add1<0, 1>(P, 1.0, s.A2);
        vp_add2<1, 0>(P, 1.0, s.A, s.a1);
        vp_add2<0, 1>(P, 1.0, s.A, s.a2);
        vp_add2<0, 0>(P, 1.0, s.A, s.A);
        psi_moments<5>(D, P, M);
#pragma unroll
        for (int q = 0; q < 4; ++q) D[q] = -p.rho * D[q];
        slope_solve(s.At, D, p, K);
    }
}

struct PolyCoef {
    double c0, cr, cA, crr, crA, cs, c1, cAA, cAt;
};

// P of the header comment for one distribution.
template <bool EQ>
GKS_HD void build_poly(VPoly& P, const Slopes& s, const PolyCoef& k) {
    vp_zero<6>(P);
    P.c[0][0][0] = k.c0;
    vp_add1<1, 0>(P, k.cr, s.a1);
    vp_add1<0, 1>(P, k.cr, s.a2);
    vp_add1<0, 0>(P, k.cA, s.A);
    vp_add2<2, 0>(P, k.crr, s.a1, s.a1);
    vp_add2<1, 1>(P, 2.0 * k.crr, s.a1, s.a2);
    vp_add2<0, 2>(P, k.crr, s.a2, s.a2);
    vp_add2<1, 0>(P, k.crA, s.a1, s.A);
    vp_add2<0, 1>(P, k.crA, s.a2, s.A);
    vp_add1<2, 0>(P, k.cs, s.a11);
    vp_add1<1, 1>(P, 2.0 * k.cs, s.a12);
    vp_add1<0, 2>(P, k.cs, s.a22);
    vp_add1<1, 0>(P, k.c1, s.A1);
    vp_add1<0, 1>(P, k.c1, s.A2);
    if constexpr (EQ) {
        vp_add2<0, 0>(P, k.cAA, s.A, s.A);
        vp_add1<0, 0>(P, k.cAt, s.At);
    }
}

// Integrals over [0, dt] of c_1..c_8 (Eq. Nomenclature2) and of c_7 t^2 / 2.
struct TimeInt {
    double T[9];
};

GKS_HD TimeInt time_integrals(double dt, double tau, bool exact) {
    TimeInt r;
    const double e = exp(-dt / tau);
    const double t2 = tau * tau, t3 = t2 * tau, d2 = dt * dt;
    r.T[0] = dt - tau * (1.0 - e);
    r.T[1] = 2.0 * t2 * (1.0 - e) - tau * dt * (1.0 + e);
    r.T[2] = 0.5 * d2 - tau * dt + t2 * (1.0 - e);
    r.T[3] = -4.0 * t3 + e * tau * (d2 + 4.0 * tau * dt + 4.0 * t2);
    r.T[4] = d2 * dt / 3.0 - tau * d2;
    r.T[5] = -0.5 * tau * d2 - t3 * (1.0 - e) + e * dt * t2;
    r.T[6] = tau * (1.0 - e);
    r.T[7] = -t2 + e * tau * (tau + dt);
    r.T[8] = t3 - 0.5 * e * tau * (d2 + 2.0 * dt * tau + 2.0 * t2);
    if (exact) {
        const double add = 2.0 * t2 * r.T[0];
        r.T[3] += add;
        r.T[4] += add;
        r.T[5] += add;
    }
    return r;
}

GKS_HD double pressure(const double W[4], double gamma) {
    return (gamma - 1.0) * (W[3] - 0.5 * (W[1] * W[1] + W[2] * W[2]) / W[0]);
}

struct FluxParams {
    double gamma, K, mu, eps;
    int exact_time;
};

// Time-integrated flux per unit length at one Gauss point (local frame).
// dL / dR: derivatives n, t, nn, nt, tt of each side (local frame).
GKS_HD void gp_flux(double F[4], const double WL[4], const double dL[5][4],
                                        const double WR[4], const double dR[5][4], double dt,
                                        const FluxParams& fp) {
    const double K = fp.K;
    const Prim pL = primitives(WL, K);
    const Prim pR = primitives(WR, K);

    // equilibrium state: collision of the two half streams
    double W0[4];
    {
        const double slL = sqrt(pL.lam), slR = sqrt(pR.lam);
        const double mL0 = 0.5 * erfc(-slL * pL.U);
        const double mL1 = pL.U * mL0 + exp(-pL.lam * pL.U * pL.U) / (2.0 * sqrt(M_PI * pL.lam));
        const double mL2 = pL.U * mL1 + 0.5 / pL.lam * mL0;
        const double mR0 = 0.5 * erfc(slR * pR.U);
        const double mR1 = pR.U * mR0 - exp(-pR.lam * pR.U * pR.U) / (2.0 * sqrt(M_PI * pR.lam));
        const double mR2 = pR.U * mR1 + 0.5 / pR.lam * mR0;
        const double vvL = pL.V * pL.V + 0.5 / pL.lam, vvR = pR.V * pR.V + 0.5 / pR.lam;
        const double xL = 0.5 * K / pL.lam, xR = 0.5 * K / pR.lam;
        W0[0] = pL.rho * mL0 + pR.rho * mR0;
        W0[1] = pL.rho * mL1 + pR.rho * mR1;
        W0[2] = pL.rho * mL0 * pL.V + pR.rho * mR0 * pR.V;
        W0[3] = 0.5 * (pL.rho * (mL2 + mL0 * (vvL + xL)) + pR.rho * (mR2 + mR0 * (vvR + xR)));
    }
    const Prim p0 = primitives(W0, K);

    const double prL = pressure(WL, fp.gamma), prR = pressure(WR, fp.gamma);
    const double jump = fabs(prL - prR) / fabs(prL + prR) * dt;
    double tau;
    if (fp.mu > 0.0)
        tau = fp.mu / pressure(W0, fp.gamma) + jump;
    else
        tau = fp.eps * dt + jump;
    const TimeInt ti = time_integrals(dt, tau, fp.exact_time != 0);
    const double* T = ti.T;

    F[0] = F[1] = F[2] = F[3] = 0.0;
    double d0[5][4];
    Slopes s;
    VPoly P;
    Mom M;

    // left side (u > 0)
    {
        full_moments<7>(M, pL, K);
        side_slopes<false>(s, dL, pL, M, K);
        const PolyCoef k = {T[6], T[7] - tau * T[6], -tau * T[6], T[8] - tau * T[7], -tau * T[7],
                            T[8] - tau * T[7], -tau * T[7], 0.0, 0.0};
        build_poly<false>(P, s, k);
        half_moments<9>(M, pL, K, 1.0);
        flux_moments<6>(F, pL.rho, P, M);
    }
    // right side (u < 0)
    {
        full_moments<7>(M, pR, K);
        side_slopes<false>(s, dR, pR, M, K);
        const PolyCoef k = {T[6], T[7] - tau * T[6], -tau * T[6], T[8] - tau * T[7], -tau * T[7],
                            T[8] - tau * T[7], -tau * T[7], 0.0, 0.0};
        build_poly<false>(P, s, k);
        half_moments<9>(M, pR, K, -1.0);
        flux_moments<6>(F, pR.rho, P, M);
    }
    // equilibrium part: derivatives of W0 are the means of both sides
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) d0[i][q] = 0.5 * (dL[i][q] + dR[i][q]);
    {
        full_moments<9>(M, p0, K);
        side_slopes<true>(s, d0, p0, M, K);
        const PolyCoef k = {T[0], T[1], T[2], 0.5 * T[3], T[5], 0.5 * T[3], T[5], 0.5 * T[4], 0.5 * T[4]};
        build_poly<true>(P, s, k);
        flux_moments<6>(F, p0.rho, P, M);
    }
}

}  // namespace gksdev
