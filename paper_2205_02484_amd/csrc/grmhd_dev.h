// grmhd_dev.h -- device-side data layout and per-point physics of the gfx950 GR-MHD stepper.
//
// Layout (all FP64):
//   cell arrays   [var][i + 3][j + 3][k]   three ghost layers in X1 and X2 (PPM reads three cells
//                                           out, PLM two: a PLM run fills only two); X3 (phi) is
//                                           periodic and handled by index wrap, so rows stay aligned
//   face fluxes   same layout; the flux through face i-1/2 (resp. j-1/2, k-1/2) of cell (i,j,k)
//                 is stored at (i,j,k)
//   geometry      [component][i + 3][j + 3]  per (r, theta) point: the metric is phi-independent
//
// The metric of both supported coordinate systems (MKS Kerr-Schild, flat Cartesian) has
// g_{t2} = g_{12} = g_{23} = 0 and g^{t2} = g^{t3} = g^{12} = g^{23} = 0; only the remaining
// components are stored and used.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace grmhd {

constexpr int NPR = 8;  // rho, u, u~1, u~2, u~3, B1, B2, B3
constexpr int NCS = 9;  // sqrt(-g)(rho u^t, T^t_t, T^t_1, T^t_2, T^t_3, B1, B2, B3, S u^t)
constexpr int NG = 3;   // ghost layers in X1 and X2 held in the layout

// centre geometry components
enum {
    G_TT = 0, G_T1, G_T3, G_11, G_13, G_22, G_33,         // g_{mu nu}
    GI_TT, GI_T1, GI_11, GI_13, GI_22, GI_33,             // g^{mu nu}
    G_DET, G_ALPHA, G_IALPHA,                             // sqrt(-g), lapse, 1/lapse
    G_D1,            // 1/2 sqrt(-g) d_1 g_{mu nu}, 7 entries in the order tt,t1,t3,11,13,22,33
    G_D2 = G_D1 + 7, // 1/2 sqrt(-g) d_2 g_{mu nu}
    G_RHOFL = G_D2 + 7, G_UFL,
    NGC
};
constexpr int NGF = G_IALPHA + 1;  // faces carry the entries up to 1/lapse

// Stored face-flux slots.  The stage chain keeps 7 per face: the 5 fluid components and the two
// field components transverse to the face (flux-CT builds the field update from those alone; the
// flux of B^d through a d-face is never read).  Diagnostic copies also keep that normal field
// component (slot 7) and the entropy component (slot 8); arrays are allocated with NCS slots.
constexpr int NFS = 7;
constexpr int FS_BN = 7, FS_ENT = 8;
// slot of conserved component q < 8 in the X^D flux arrays (-1: the normal field component)
template <int D>
__host__ __device__ constexpr int flux_slot(int q) {
    return q < 5 ? q : (q == 4 + D ? -1 : (q < 4 + D ? q : q - 1));
}

// Division of 0 <= n < 2^31 by a fixed d >= 1 with one high multiply, an add and a shift
// (the round-up method of Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994): l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1,
// n / d = (mulhi(m, n) + n) >> l; the sum stays below 2^32 because n < 2^31.
struct FastDiv {
    uint32_t m, l;
};
__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) { return (__umulhi(n, f.m) + n) >> f.l; }

// Per-run constant description (device copy, read with scalar loads).
struct RunVar;
struct RunDev {
    int32_t n1, n2, n3;
    int32_t act1, act2, act3;
    int32_t mks, riemann;
    int32_t c2p_maxit, fixup_rounds;
    int32_t geo_uniform;        // row path: a wave is 64 lanes of one phi row (its cells share
                                //   (r, theta)), lane l of chunk c at k = (64 c + l) mod n3
    int32_t ppm;                // reconstruction: 0 PLM with the MC limiter, 1 PPM
    int32_t pole_fix;           // MKS: cells next to each pole whose u~2 is interpolated to zero
    int32_t nkc;                // row path: 64-lane chunks per row, ceil(n3 / 64)
    int32_t mseg[2];            // row path: faces per wave segment of the X1 and X2 marches
    int32_t row_ok;             // the row path can serve this run (the engine decides geo_uniform)
    int32_t pad_;
    FastDiv fd_n2, fd_n3, fd_kc;  // divisors n2, n3, nkc (the last only on the row path)
    FastDiv fd_row[4];          // [d]: row length of the flux-face rows: n1 + 1, n2 + 1, n2 + 2 act2
    FastDiv fd_jg[3];           // [l]: number of j groups of 2^l rows, ceil(n2 / 2^l)
    int64_t s1, s2, vs;         // cell strides: i, j (k stride 1); variable stride
    int64_t gs1, gpts;          // geometry: i stride (n2 + 2 NG), total points
    double dx[4], idx[4];
    double gam, cfl;
    double gg, igam1;           // (gam - 1)/gam, 1/(gam - 1)
    double bsq_rho_max, bsq_u_max, gamma_max, beta_ent, c2p_tol;
    double* P;                  // state P^n (updated in place by stage 2)
    double* Ph;                 // P^{n+1/2}
    double* F[4];               // F[1..3]
    const double* gc;           // centre geometry
    const double* gf[3];        // gf[1], gf[2]: X1, X2 faces
    int8_t* code;               // method code per cell (cell layout)
    int32_t* fail_list;         // interior linear indices of failed cells
    int32_t* slow_list;         // cells the fast inversion path hands to the full procedure
    RunVar* var;
};

// Per-run mutable scalars.
struct RunVar {
    unsigned long long cmax[3];  // bits of max c_w per direction (non-negative doubles)
    double dt, t, dt_req;        // dt_req > 0: fixed step; <= 0: CFL
    long long nstep, nfail_total, steps_left;
    int32_t fail_count, active, nfail_last, slow_count;
};

// Global-memory access through a wave-uniform base pointer and a 32-bit element index: the
// compiler then issues global_load/store with an SGPR base and a VGPR byte offset, with no 64-bit
// address arithmetic per access.  Every array is < 4 GiB (checked when a run is created).
typedef __attribute__((address_space(1))) char g_char;
typedef __attribute__((address_space(1))) double g_double;

__device__ __forceinline__ double gld(const double* base, uint32_t e) {
    return *(const g_double*)((const g_char*)base + e * 8u);
}
__device__ __forceinline__ void gst(double* base, uint32_t e, double v) {
    *(g_double*)((g_char*)base + e * 8u) = v;
}

// Streaming forms for data a kernel touches once (non-temporal hint: do not keep it in the caches).
__device__ __forceinline__ double gld_nt(const double* base, uint32_t e) {
    return __builtin_nontemporal_load((const g_double*)((const g_char*)base + e * 8u));
}
__device__ __forceinline__ void gst_nt(double* base, uint32_t e, double v) {
    __builtin_nontemporal_store(v, (g_double*)((g_char*)base + e * 8u));
}

// Wave-uniform read of a table no stage kernel writes (the metric) through the constant address
// space: the load is a scalar load even after vector stores of the same kernel, which a
// global-space load in a loop with stores is not (the compiler cannot rule out a clobber).
typedef __attribute__((address_space(4))) const char k_char;
typedef __attribute__((address_space(4))) const double k_double;

__device__ __forceinline__ double kld(const double* base, uint32_t e) {
    return *(const k_double*)((const k_char*)base + e * 8u);
}

__device__ __forceinline__ int64_t cell_index(const RunDev& R, int i, int j, int k) {
    return (int64_t)(i + NG) * R.s1 + (int64_t)(j + NG) * R.s2 + k;
}
__device__ __forceinline__ int64_t geo_index(const RunDev& R, int i, int j) {
    return (int64_t)(i + NG) * R.gs1 + (j + NG);
}

struct Geo {
    double gtt, gt1, gt3, g11, g13, g22, g33;
    double Gtt, Gt1, G11, G13, G22, G33;
    double gdet, alpha, ialpha;
};

__device__ __forceinline__ void load_geo(const double* __restrict__ g, int64_t np, int64_t gi64, Geo& G) {
    const uint32_t gi = (uint32_t)gi64;
    G.gtt = gld(g + G_TT * np, gi);
    G.gt1 = gld(g + G_T1 * np, gi);
    G.gt3 = gld(g + G_T3 * np, gi);
    G.g11 = gld(g + G_11 * np, gi);
    G.g13 = gld(g + G_13 * np, gi);
    G.g22 = gld(g + G_22 * np, gi);
    G.g33 = gld(g + G_33 * np, gi);
    G.Gtt = gld(g + GI_TT * np, gi);
    G.Gt1 = gld(g + GI_T1 * np, gi);
    G.G11 = gld(g + GI_11 * np, gi);
    G.G13 = gld(g + GI_13 * np, gi);
    G.G22 = gld(g + GI_22 * np, gi);
    G.G33 = gld(g + GI_33 * np, gi);
    G.gdet = gld(g + G_DET * np, gi);
    G.alpha = gld(g + G_ALPHA * np, gi);
    G.ialpha = gld(g + G_IALPHA * np, gi);
}

// load_geo for a wave-uniform point gi, as scalar loads
__device__ __forceinline__ void load_geo_k(const double* __restrict__ g, int64_t np, uint32_t gi, Geo& G) {
    G.gtt = kld(g + G_TT * np, gi);
    G.gt1 = kld(g + G_T1 * np, gi);
    G.gt3 = kld(g + G_T3 * np, gi);
    G.g11 = kld(g + G_11 * np, gi);
    G.g13 = kld(g + G_13 * np, gi);
    G.g22 = kld(g + G_22 * np, gi);
    G.g33 = kld(g + G_33 * np, gi);
    G.Gtt = kld(g + GI_TT * np, gi);
    G.Gt1 = kld(g + GI_T1 * np, gi);
    G.G11 = kld(g + GI_11 * np, gi);
    G.G13 = kld(g + GI_13 * np, gi);
    G.G22 = kld(g + GI_22 * np, gi);
    G.G33 = kld(g + GI_33 * np, gi);
    G.gdet = kld(g + G_DET * np, gi);
    G.alpha = kld(g + G_ALPHA * np, gi);
    G.ialpha = kld(g + G_IALPHA * np, gi);
}

// sqrt(x) and 1/sqrt(x) together, for normal x > 0: the hardware reciprocal-square-root estimate
// refined by two coupled Goldschmidt steps on g ~ sqrt(x), h ~ 1/(2 sqrt(x)) (Goldschmidt's
// iteration as given by Markstein for IA-64 square roots): r = 1/2 - g h, g += g r, h += h r.
// Each step squares the relative error, so from the ~2^-22 estimate the pair is within a few ulp;
// 9 instructions where a correctly rounded sqrt plus a division take ~29.
__device__ __forceinline__ void sqrt_rsqrt(double x, double& s, double& rs) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    s = g;
    rs = 2.0 * h;
}

// sqrt(x) for x >= 0 (0 for x below the smallest normal double): one Goldschmidt step, then a
// Newton correction of g with the refined h.
__device__ __forceinline__ double sqrt_fast(double x) {
    const double xc = fmax(x, 2.2250738585072014e-308);
    const double y = __builtin_amdgcn_rsq(xc);
    double g = xc * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    g = fma(fma(-g, g, xc), h, g);
    return x > 2.2250738585072014e-308 ? g : 0.0;
}

// 4-velocity, field 4-vector and thermodynamics of one primitive state.
struct St {
    double ut, u1, u2, u3;       // u^mu
    double lt, l1, l2, l3;       // u_mu
    double bt, b1, b2, b3;       // b^mu
    double ct, c1, c2, c3;       // b_mu
    double bsq, p, w, lor;
};

__device__ __forceinline__ void lower(const Geo& G, double t, double x1, double x2, double x3,
                                      double& l0, double& l1, double& l2, double& l3) {
    l0 = G.gtt * t + G.gt1 * x1 + G.gt3 * x3;
    l1 = G.gt1 * t + G.g11 * x1 + G.g13 * x3;
    l2 = G.g22 * x2;
    l3 = G.gt3 * t + G.g13 * x1 + G.g33 * x3;
}

// u~^i -> u^mu: Gamma = sqrt(1 + g_ij u~^i u~^j), u^t = Gamma/alpha, u^i = u~^i - Gamma alpha g^{ti};
// b^t = B^i u_i, b^i = (B^i + b^t u^i)/u^t  (Sec. 2.1).
__device__ __forceinline__ void prim_state(const double* P, const Geo& G, double gam, St& s) {
    const double q1 = P[2], q2 = P[3], q3 = P[4];
    const double qsq = G.g11 * q1 * q1 + 2.0 * G.g13 * q1 * q3 + G.g22 * q2 * q2 + G.g33 * q3 * q3;
    double lor, ilor;
    sqrt_rsqrt(1.0 + qsq, lor, ilor);
    s.lor = lor;
    s.ut = lor * G.ialpha;
    s.u1 = q1 - lor * G.alpha * G.Gt1;
    s.u2 = q2;
    s.u3 = q3;
    lower(G, s.ut, s.u1, s.u2, s.u3, s.lt, s.l1, s.l2, s.l3);
    const double B1 = P[5], B2 = P[6], B3 = P[7];
    s.bt = B1 * s.l1 + B2 * s.l2 + B3 * s.l3;
    const double iut = G.alpha * ilor;  // 1/u^t
    s.b1 = (B1 + s.bt * s.u1) * iut;
    s.b2 = (B2 + s.bt * s.u2) * iut;
    s.b3 = (B3 + s.bt * s.u3) * iut;
    lower(G, s.bt, s.b1, s.b2, s.b3, s.ct, s.c1, s.c2, s.c3);
    s.bsq = s.bt * s.ct + s.b1 * s.c1 + s.b2 * s.c2 + s.b3 * s.c3;
    s.p = (gam - 1.0) * P[1];
    s.w = P[0] + P[1] + s.p;
}

// Flux vector along D (D = 0: the conserved vector U).  ent = p / rho^(gam-1).
template <int D>
__device__ __forceinline__ void flux_of(const double* P, const St& s, const Geo& G, double ent, double* F) {
    const double ud = D == 0 ? s.ut : (D == 1 ? s.u1 : (D == 2 ? s.u2 : s.u3));
    const double bd = D == 0 ? s.bt : (D == 1 ? s.b1 : (D == 2 ? s.b2 : s.b3));
    const double wb = s.w + s.bsq;
    const double pt = s.p + 0.5 * s.bsq;
    const double gd = G.gdet;
    F[0] = gd * P[0] * ud;
    F[1] = gd * (wb * ud * s.lt + (D == 0 ? pt : 0.0) - bd * s.ct);
    F[2] = gd * (wb * ud * s.l1 + (D == 1 ? pt : 0.0) - bd * s.c1);
    F[3] = gd * (wb * ud * s.l2 + (D == 2 ? pt : 0.0) - bd * s.c2);
    F[4] = gd * (wb * ud * s.l3 + (D == 3 ? pt : 0.0) - bd * s.c3);
    if (D == 0) {
        F[5] = gd * P[5];
        F[6] = gd * P[6];
        F[7] = gd * P[7];
    } else {
        // induction flux sqrt(-g)(b^i u^d - b^d u^i)
        F[5] = gd * (s.b1 * ud - bd * s.u1);
        F[6] = gd * (s.b2 * ud - bd * s.u2);
        F[7] = gd * (s.b3 * ud - bd * s.u3);
    }
    F[8] = gd * ent * ud;
}

// Roots of the simplified dispersion relation along D: (1-cms2)(k.u)^2 = cms2 k.k with
// k_mu = (-omega, k_D), as c1 >= c2 in omega/k_D.  cms2 = v_a^2 + c_s^2 (1 - v_a^2) with
// v_a^2 = b^2/(b^2 + w), c_s^2 = gam p / w, i.e. cms2 = (b^2 + gam p)/(b^2 + w); the quadratic is
// multiplied through by b^2 + w (its roots do not change), which leaves no division for cms2.
template <int D>
__device__ __forceinline__ void wave_speeds(const St& s, const Geo& G, double gam, double& c1, double& c2) {
    const double num = s.bsq + gam * s.p;      // (b^2 + w) cms2
    const double om = s.w - gam * s.p;         // (b^2 + w)(1 - cms2)
    const double ud = D == 1 ? s.u1 : (D == 2 ? s.u2 : s.u3);
    const double gtd = D == 1 ? G.Gt1 : 0.0;
    const double gdd = D == 1 ? G.G11 : (D == 2 ? G.G22 : G.G33);
    const double A = om * s.ut * s.ut - num * G.Gtt;
    const double B = -2.0 * (om * s.ut * ud - num * gtd);
    const double C = om * ud * ud - num * gdd;
    double disc = B * B - 4.0 * A * C;
    disc = disc < 0.0 ? 0.0 : disc;
    const double sq = sqrt_fast(disc);
    const double i2a = 0.5 / A;
    const double r1 = (-B + sq) * i2a;
    const double r2 = (-B - sq) * i2a;
    c1 = fmax(r1, r2);
    c2 = fmin(r1, r2);
}

// Half of the monotonised-central slope, sign(dc) min(2|dm|, 2|dp|, |dc|/2) / 2, zero at extrema:
// the face value is q0 -/+ this.  Halving inside the min is exact (powers of two), so the face
// values equal q0 -/+ 0.5 * slope bit for bit, with two instructions fewer per slope.
__device__ __forceinline__ double mc_half_slope(double qm, double q0, double qp) {
    const double dm = q0 - qm, dp = qp - q0, dc = qp - qm;
    const double lim = fmin(fmin(fabs(dm), fabs(dp)), 0.25 * fabs(dc));
    return (dm * dp > 0.0) ? copysign(lim, dc) : 0.0;
}

// PPM of Colella & Woodward (1984).  Edge values of the parabola in a cell of average a0 whose
// interface values are l (lower) and r (upper), after their monotonicity constraints: a local
// extremum gives the flat profile, and an edge value that would put the parabola's extremum inside
// the cell is moved so that the extremum sits on the opposite edge.  The two moves exclude each
// other, so each edge is decided on its own.
__device__ __forceinline__ double ppm_upper_edge(double a0, double l, double r) {
    const double da = r - l, a6 = 6.0 * (a0 - 0.5 * (l + r));
    if ((r - a0) * (a0 - l) <= 0.0) return a0;
    return (-da * da > da * a6) ? 3.0 * a0 - 2.0 * l : r;
}
__device__ __forceinline__ double ppm_lower_edge(double a0, double l, double r) {
    const double da = r - l, a6 = 6.0 * (a0 - 0.5 * (l + r));
    if ((r - a0) * (a0 - l) <= 0.0) return a0;
    return (da * a6 > da * da) ? 3.0 * a0 - 2.0 * r : l;
}

// PPM states on the face between cells c and d of six consecutive cells a..f: the interface value
// between cells j and j+1 is a_j + (a_{j+1} - a_j)/2 - (s_{j+1} - s_j)/6 with s the MC slope (here
// from the half slopes h = s/2: (h_{j+1} - h_j)/3); the left state is the upper edge of cell c,
// the right state the lower edge of cell d.
__device__ __forceinline__ void ppm_face(double a, double b, double c, double d, double e, double f, double& ql,
                                         double& qr) {
    constexpr double third = 1.0 / 3.0;
    const double hb = mc_half_slope(a, b, c), hc = mc_half_slope(b, c, d);
    const double hd = mc_half_slope(c, d, e), he = mc_half_slope(d, e, f);
    const double ibc = b + 0.5 * (c - b) - (hc - hb) * third;
    const double icd = c + 0.5 * (d - c) - (hd - hc) * third;
    const double ide = d + 0.5 * (e - d) - (he - hd) * third;
    ql = ppm_upper_edge(c, ibc, icd);
    qr = ppm_lower_edge(d, icd, ide);
}

}  // namespace grmhd
