// grmhd_c2p.h -- conserved-to-primitive inversion, floors and ceilings on the device.
//
// Sec. 2.3 of the paper: 2D Newton-Raphson on (W, v^2) for Eqs. inv-1/inv-2, a 1D Brent solve on
// W with v^2(W) from inv-1 as the fallback, and the entropy inversion (W from Eq. W_of_S put in
// inv-1, Brent on v^2) when the previous state has beta = p_g/p_b < 1e-2 or the energy methods
// fail.  Eq. inv-2 is used with -B^2(1+v^2)/2 (the rest-frame limit fixes that sign), the
// entropy density is the normal-frame one, alpha U_S / sqrt(-g).  Sec. 2.4: density/energy
// floors, b^2/rho and b^2/u ceilings by adding mass/energy at rest in the normal frame and
// re-inverting with the energy equation, and the Lorentz-factor cap.
#pragma once
#include "grmhd_dev.h"

namespace grmhd {

constexpr double V2MAX = 1.0 - 1e-12;
constexpr double DEPS = 2.220446049250313e-16;

struct Inv {
    double D, Qt, Q1, Q2, Q3;       // D, Q_mu
    double Qu1, Qu3;                // Q^1, Q^3 (Q^2 = g^22 Q_2 computed on use)
    double Qdotn, Qtsq, QdB, Bsq;
    double Bc1, Bc2, Bc3;           // frak B^i = alpha B^i
    double ent;                     // alpha U_S / sqrt(-g)
    double gam, gg, igam1;          // gamma, (gamma-1)/gamma, 1/(gamma-1)
    double ig;                      // 1/sqrt(-g)
    double n1;                      // n^1 = -alpha g^{t1}  (n^2 = n^3 = 0)
};

__device__ __forceinline__ void inv_setup(const double* U, const Geo& G, const RunDev& R, Inv& q) {
    q.ig = 1.0 / G.gdet;
    const double f = G.alpha * q.ig;
    q.gam = R.gam;
    q.gg = R.gg;
    q.igam1 = R.igam1;
    q.D = f * U[0];
    q.Qt = f * U[1];
    q.Q1 = f * U[2];
    q.Q2 = f * U[3];
    q.Q3 = f * U[4];
    q.Bc1 = f * U[5];
    q.Bc2 = f * U[6];
    q.Bc3 = f * U[7];
    q.ent = f * U[8];
    q.n1 = -G.alpha * G.Gt1;
    // n^t = 1/alpha
    q.Qdotn = q.Qt * G.ialpha + q.Q1 * q.n1;
    const double Qut = G.Gtt * q.Qt + G.Gt1 * q.Q1;
    q.Qu1 = G.Gt1 * q.Qt + G.G11 * q.Q1 + G.G13 * q.Q3;
    const double Qu2 = G.G22 * q.Q2;
    q.Qu3 = G.G13 * q.Q1 + G.G33 * q.Q3;
    const double qsq = Qut * q.Qt + q.Qu1 * q.Q1 + Qu2 * q.Q2 + q.Qu3 * q.Q3;
    q.Qtsq = qsq + q.Qdotn * q.Qdotn;
    q.QdB = q.Q1 * q.Bc1 + q.Q2 * q.Bc2 + q.Q3 * q.Bc3;
    q.Bsq = G.g11 * q.Bc1 * q.Bc1 + 2.0 * G.g13 * q.Bc1 * q.Bc3 + G.g22 * q.Bc2 * q.Bc2 + G.g33 * q.Bc3 * q.Bc3;
}

__device__ __forceinline__ double p_of_w(const Inv& q, double W, double v2) {
    return q.gg * (W * (1.0 - v2) - q.D * sqrt(1.0 - v2));
}
// the same with sq = sqrt(1 - v^2) at hand
__device__ __forceinline__ double p_of_w_sq(const Inv& q, double W, double v2, double sq) {
    return q.gg * (W * (1.0 - v2) - q.D * sq);
}
__device__ __forceinline__ double inv1(const Inv& q, double W, double v2) {
    const double bw = q.Bsq + W;
    return v2 * bw * bw - q.QdB * q.QdB * (q.Bsq + 2.0 * W) / (W * W) - q.Qtsq;
}
__device__ __forceinline__ double inv2(const Inv& q, double W, double v2) {
    return -0.5 * q.Bsq * (1.0 + v2) + q.QdB * q.QdB / (2.0 * W * W) - W + p_of_w(q, W, v2) - q.Qdotn;
}
__device__ __forceinline__ double v2_from_w(const Inv& q, double W) {
    const double bw = q.Bsq + W;
    double v2 = (q.Qtsq + q.QdB * q.QdB * (q.Bsq + 2.0 * W) / (W * W)) / (bw * bw);
    return fmin(fmax(v2, 0.0), V2MAX);
}
__device__ __forceinline__ double w_from_s(const Inv& q, double v2) {
    const double lor = 1.0 / sqrt(1.0 - v2);
    return lor * q.D + lor * (q.gam / (q.gam - 1.0)) * pow(q.D / lor, q.gam - 1.0) * q.ent;
}

// residual of the two 1D problems: which = 0 -> inv-2 at v^2(W) (unknown W);
// which = 1 -> inv-1 at W(v^2) (unknown v^2, entropy)
__device__ __forceinline__ double resid1d(const Inv& q, int which, double x) {
    if (which == 0) return inv2(q, x, v2_from_w(q, x));
    return inv1(q, w_from_s(q, x), x);
}

// Brent's bracketing root finder: inverse quadratic / secant steps accepted only while they
// shrink the bracket fast enough, bisection otherwise; stops when half the bracket is below
// 2 eps |x| + atol/2.  Returns false without a sign change or on a non-finite residual.
__device__ __forceinline__ bool brent1d(const Inv& q, int which, double lo, double hi, double atol, double* root) {
    double a = lo, b = hi;
    double fa = resid1d(q, which, a), fb = resid1d(q, which, b);
    if (!isfinite(fa) || !isfinite(fb)) return false;
    if (fa == 0.0) { *root = a; return true; }
    if (fb == 0.0) { *root = b; return true; }
    if ((fa > 0.0) == (fb > 0.0)) return false;
    double c = a, fc = fa, d = b - a, e = d;
    for (int it = 0; it < 300; ++it) {
        if ((fb > 0.0) == (fc > 0.0)) { c = a; fc = fa; d = b - a; e = d; }
        if (fabs(fc) < fabs(fb)) { a = b; b = c; c = a; fa = fb; fb = fc; fc = fa; }
        const double tol = 2.0 * DEPS * fabs(b) + 0.5 * atol;
        const double m = 0.5 * (c - b);
        if (fabs(m) <= tol || fb == 0.0) { *root = b; return true; }
        if (fabs(e) >= tol && fabs(fa) > fabs(fb)) {
            const double s = fb / fa;
            double p, qq;
            if (a == c) {
                p = 2.0 * m * s;
                qq = 1.0 - s;
            } else {
                const double t = fa / fc, r = fb / fc;
                p = s * (2.0 * m * t * (t - r) - (b - a) * (r - 1.0));
                qq = (t - 1.0) * (r - 1.0) * (s - 1.0);
            }
            if (p > 0.0) qq = -qq; else p = -p;
            if (2.0 * p < fmin(3.0 * m * qq - fabs(tol * qq), fabs(e * qq))) {
                e = d;
                d = p / qq;
            } else { d = m; e = m; }
        } else { d = m; e = m; }
        a = b;
        fa = fb;
        b += fabs(d) > tol ? d : (m > 0.0 ? tol : -tol);
        fb = resid1d(q, which, b);
        if (!isfinite(fb)) return false;
    }
    return false;
}

__device__ __forceinline__ bool is_physical(double W, double v2, double rho, double p) {
    return isfinite(W) && isfinite(v2) && isfinite(rho) && isfinite(p) && W > 0.0 && v2 >= 0.0 &&
           v2 < 1.0 && rho > 0.0 && p > 0.0;
}

// u~^i = Gamma/(W + B^2) (Q~^i + (Q.B) B^i / W), Q~^i = Q^i + n^i (Q.n); lor = Gamma.  Both
// quotients come from one reciprocal of W (W + B^2).
__device__ __forceinline__ void velocity_out(const Inv& q, const Geo& G, double W, double lor, double* P) {
    const double bw = W + q.Bsq;
    const double iw = 1.0 / (W * bw);
    const double f = lor * W * iw;
    const double g = q.QdB * bw * iw;
    P[2] = f * (q.Qu1 + q.n1 * q.Qdotn + g * q.Bc1);
    P[3] = f * (G.G22 * q.Q2 + g * q.Bc2);
    P[4] = f * (q.Qu3 + g * q.Bc3);
}

// 2D Newton-Raphson on (W, v^2); true when |dW| < tol W.  Each lane stops at its own iterate (state
// set), and the wave leaves the loop only when no lane iterates any more: the exit is wave-uniform.
// (Inlined inside an enclosing loop, the form with a return per exit made every lane run to maxit
// and report no convergence; the uniform exit does not depend on how the loop is nested.)
__device__ __forceinline__ bool newton2d(const Inv& q, double tol, int maxit, double& W, double& v2) {
    const double gg = q.gg;
    const double qb2 = q.QdB * q.QdB;
    int state = 0;  // 0: iterating, 1: converged, -1: failed
    for (int it = 0; it < maxit; ++it) {
      if (state == 0) {
        const double bw = q.Bsq + W;
        const double iW = 1.0 / W;
        const double iW2 = iW * iW;
        double sq, isq;
        sqrt_rsqrt(1.0 - v2, sq, isq);  // v2 in [0, 1 - 1e-12]
        const double pg = gg * (W * (1.0 - v2) - q.D * sq);
        const double f1 = v2 * bw * bw - qb2 * (q.Bsq + 2.0 * W) * iW2 - q.Qtsq;
        const double f2 = -0.5 * q.Bsq * (1.0 + v2) + 0.5 * qb2 * iW2 - W + pg - q.Qdotn;
        const double j11 = 2.0 * v2 * bw + 2.0 * qb2 * bw * iW2 * iW;
        const double j12 = bw * bw;
        const double j21 = -qb2 * iW2 * iW - 1.0 + gg * (1.0 - v2);
        const double j22 = -0.5 * q.Bsq + gg * (-W + 0.5 * q.D * isq);
        const double idet = 1.0 / (j11 * j22 - j12 * j21);
        const double dW = -(f1 * j22 - f2 * j12) * idet;
        const double dv = -(j11 * f2 - j21 * f1) * idet;
        W += dW;
        v2 = fmin(fmax(v2 + dv, 0.0), V2MAX);
        if (!isfinite(W) || !isfinite(v2) || W <= 0.0) state = -1;
        else if (fabs(dW) < tol * fabs(W)) state = 1;
      }
      if (!__any(state == 0)) break;
    }
    return state == 1;
}

// Primitives from a root (W, v^2) of the energy equations, v^2 in [0, 1 - 1e-12]; false when the
// state is not physical (P untouched then).
__device__ __forceinline__ bool finish_energy(const Inv& q, const Geo& G, double W, double v2, double* P) {
    double sq, lor;
    sqrt_rsqrt(1.0 - v2, sq, lor);
    const double rho = q.D * sq;
    const double p = p_of_w_sq(q, W, v2, sq);
    if (!is_physical(W, v2, rho, p)) return false;
    P[0] = rho;
    P[1] = p * q.igam1;
    velocity_out(q, G, W, lor, P);
    return true;
}

// Energy-equation inversion: 0 (NR), 1 (Brent on W), -1 (NR converged to a non-physical
// state), -2 (no solution).
__device__ __forceinline__ int invert_energy(const Inv& q, const Geo& G, double W0, double v20, double tol,
                                             int maxit, double* P) {
    double W = W0, v2 = v20;
    if (newton2d(q, tol, maxit, W, v2)) return finish_energy(q, G, W, v2, P) ? 0 : -1;
    if (!(q.D > 0.0)) return -2;
    const double lo = q.D;
    double hi = 2.0 * fmax(q.D, W0);
    const double flo = resid1d(q, 0, lo);
    double fhi = resid1d(q, 0, hi);
    for (int n = 0; n < 60 && isfinite(flo) && isfinite(fhi) && ((flo > 0.0) == (fhi > 0.0)); ++n) {
        hi *= 2.0;
        fhi = resid1d(q, 0, hi);
    }
    if (!brent1d(q, 0, lo, hi, 0.0, &W)) return -2;
    v2 = v2_from_w(q, W);
    return finish_energy(q, G, W, v2, P) ? 1 : -2;
}

__device__ __forceinline__ int invert_entropy(const Inv& q, const Geo& G, double* P) {
    if (!(q.D > 0.0) || !(q.ent > 0.0)) return -1;
    double v2;
    if (!brent1d(q, 1, 0.0, V2MAX, 1e-20, &v2)) return -1;
    const double W = w_from_s(q, v2);
    const double lor = 1.0 / sqrt(1.0 - v2);
    const double rho = q.D / lor;
    const double p = (q.ent / lor) * pow(rho, q.gam - 1.0);
    if (!is_physical(W, v2, rho, p)) return -1;
    P[0] = rho;
    P[1] = p * q.igam1;
    velocity_out(q, G, W, lor, P);
    return 2;
}

// Full inversion of one cell, guess/beta switch from the stage-input primitives Pg.
// P[5..7] receives U_B / sqrt(-g); returns 0/1/2 or -1.
__device__ __forceinline__ int invert_cell(const double* U, const double* Pg, const Geo& G, const RunDev& R,
                                           double* P) {
    Inv q;
    inv_setup(U, G, R, q);
    P[5] = U[5] * q.ig;
    P[6] = U[6] * q.ig;
    P[7] = U[7] * q.ig;
    St s;
    prim_state(Pg, G, R.gam, s);
    if (s.p < R.beta_ent * 0.5 * s.bsq) return invert_entropy(q, G, P);
    const double W0 = s.lor * s.lor * s.w;
    const double qsq = s.lor * s.lor - 1.0;
    const int m = invert_energy(q, G, W0, qsq / (1.0 + qsq), R.c2p_tol, R.c2p_maxit, P);
    if (m >= 0) return m;
    return invert_entropy(q, G, P);
}

// Floors, magnetisation ceilings and the Lorentz cap on an inverted (or fixed) cell.
__device__ __forceinline__ void ceiling_reinvert(const RunDev& R, const Geo& G, double* P, double drho, double du) {
    St s;
    prim_state(P, G, R.gam, s);
    double U[NCS];
    const double ent = s.p / pow(P[0], R.gam - 1.0);
    flux_of<0>(P, s, G, ent, U);
    // material added at rest in the normal frame: u^t = 1/alpha, u_i = 0 -> mass and T^t_t only
    U[0] += G.gdet * drho / G.alpha;
    U[1] -= G.gdet * (drho + du);
    Inv q;
    inv_setup(U, G, R, q);
    const double W0 = s.lor * s.lor * s.w;
    const double qsq = s.lor * s.lor - 1.0;
    double Pn[NPR];
    for (int v = 0; v < NPR; ++v) Pn[v] = P[v];
    const int m = invert_energy(q, G, W0, qsq / (1.0 + qsq), R.c2p_tol, R.c2p_maxit, Pn);
    if (m >= 0) {
        for (int v = 0; v < 5; ++v) P[v] = Pn[v];
    } else {
        P[0] += drho;
        P[1] += du;
    }
}

__device__ __forceinline__ void apply_floors(const RunDev& R, const Geo& G, double rho_fl, double u_fl, double* P) {
    P[0] = fmax(P[0], rho_fl);
    P[1] = fmax(P[1], u_fl);
    St s;
    prim_state(P, G, R.gam, s);
    const double drho = fmax(0.0, s.bsq / R.bsq_rho_max - P[0]);
    const double du = fmax(0.0, s.bsq / R.bsq_u_max - P[1]);
    if (drho > 0.0 || du > 0.0) ceiling_reinvert(R, G, P, drho, du);
    const double q1 = P[2], q2 = P[3], q3 = P[4];
    const double qsq = G.g11 * q1 * q1 + 2.0 * G.g13 * q1 * q3 + G.g22 * q2 * q2 + G.g33 * q3 * q3;
    const double lor = sqrt(1.0 + qsq);
    if (lor > R.gamma_max) {
        const double f = sqrt((R.gamma_max * R.gamma_max - 1.0) / (lor * lor - 1.0));
        P[2] *= f;
        P[3] *= f;
        P[4] *= f;
    }
}

}  // namespace grmhd
