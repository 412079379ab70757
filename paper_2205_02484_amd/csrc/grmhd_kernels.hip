// grmhd_kernels.hip -- gfx950 kernels of the GR-MHD stage chain.
//
// Every stage kernel runs over a packed block table: block b of a launch belongs to run r with
// boff[r] <= b < boff[r+1], so one launch advances every run of an ensemble (a single run is an
// ensemble of one).  Per-run constants come from RunDev (scalar loads, wave-uniform), per-run
// mutable scalars from RunVar.
//
// Stage chain (RK2 midpoint, Sec. 2.2 of the paper):
//   k_bound -> k_flux<1,2,3> (PLM/MC + LLF/HLL, CFL maxima) -> [k_dt] -> k_update (flux-CT,
//   conservative update with the centred source, inversion, floors) -> k_fixup
#include "grmhd_c2p.h"
#include "grmhd_kernels.h"

namespace grmhd {

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on XCD b mod 8), each
// with its own L2.  Remapping so that every XCD walks a contiguous range of logical blocks keeps
// the rows a stencil shares inside one L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b & 7, m = b >> 3;
    const int q = nb >> 3, rem = nb & 7;
    return x * q + (x < rem ? x : rem) + m;
}

__device__ __forceinline__ int find_run(const int* __restrict__ boff, int nruns, int b) {
    int lo = 0, hi = nruns;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (boff[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------------------------------
// geometry (once per run): closed-form Kerr-Schild metric and inverse carried to MKS, sqrt(-g),
// lapse, analytic d_1, d_2 of g_{mu nu} for the source, floor values
// ------------------------------------------------------------------------------------------

struct MetricPoint {
    double g[7], gi[6], gdet, alpha, d1[7], d2[7], r;
};

// r(X1) of the MKS radial map (Sec. 4.1) with its first two X1 derivatives: exp(X1) below xb,
// exp(X1 + u^nx) with u = X1 - xb beyond
__device__ void radial_map(double X1, double xb, int nx, double& r, double& dr, double& d2r) {
    if (!(X1 >= xb)) {
        r = exp(X1);
        dr = r;
        d2r = r;
        return;
    }
    const double u = X1 - xb;
    double un2 = 1.0;  // u^(nx-2)
    for (int k = 0; k < nx - 2; ++k) un2 *= u;
    const double un1 = un2 * u, un = un1 * u;
    const double f1 = 1.0 + nx * un1, f2 = nx * (nx - 1) * un2;
    r = exp(X1 + un);
    dr = r * f1;
    d2r = r * (f1 * f1 + f2);
}

__device__ void mks_point(double X1, double X2, double a, double hh, double xb, int nx, bool derivs,
                          MetricPoint& m) {
    const double PI = 3.14159265358979323846;
    double r, dr, d2r;
    radial_map(X1, xb, nx, r, dr, d2r);
    const double s2pi = sin(2.0 * PI * X2), c2pi = cos(2.0 * PI * X2);
    const double th = PI * X2 + 0.5 * (1.0 - hh) * s2pi;
    const double dth = PI * (1.0 + (1.0 - hh) * c2pi);
    const double d2th = -2.0 * PI * PI * (1.0 - hh) * s2pi;
    double s, c;
    sincos(th, &s, &c);
    const double s2 = s * s;
    const double a2 = a * a;
    const double sig = r * r + a2 * c * c;
    const double del = r * r - 2.0 * r + a2;
    const double z = 2.0 * r / sig;
    // Kerr-Schild g_{mu nu}: tt, tr, tphi, rr, rphi, thth, phiphi
    const double K[7] = {-(1.0 - z), z, -a * z * s2, 1.0 + z, -a * (1.0 + z) * s2, sig,
                         s2 * (sig + a2 * (1.0 + z) * s2)};
    const double J[7] = {1.0, dr, 1.0, dr * dr, dr, dth * dth, 1.0};
    for (int n = 0; n < 7; ++n) m.g[n] = K[n] * J[n];
    // inverse: tt, tr, rr, rphi, thth, phiphi (KS) over the Jacobian factors
    m.gi[0] = -(1.0 + z);
    m.gi[1] = z / dr;
    m.gi[2] = del / sig / (dr * dr);
    m.gi[3] = a / sig / dr;
    m.gi[4] = 1.0 / sig / (dth * dth);
    m.gi[5] = 1.0 / (sig * s2);
    m.gdet = sig * fabs(s) * dr * dth;
    m.alpha = 1.0 / sqrt(1.0 + z);
    m.r = r;
    if (!derivs) return;
    const double dsig_r = 2.0 * r, dsig_t = -2.0 * a2 * c * s;
    const double dz_r = (2.0 * sig - 4.0 * r * r) / (sig * sig);
    const double dz_t = -2.0 * r * dsig_t / (sig * sig);
    const double ds2 = 2.0 * s * c;
    const double Kr[7] = {dz_r, dz_r, -a * s2 * dz_r, dz_r, -a * s2 * dz_r, dsig_r,
                          s2 * dsig_r + a2 * s2 * s2 * dz_r};
    const double Kt[7] = {dz_t, dz_t, -a * (dz_t * s2 + z * ds2), dz_t, -a * (dz_t * s2 + (1.0 + z) * ds2), dsig_t,
                          ds2 * sig + s2 * dsig_t + a2 * (dz_t * s2 * s2 + (1.0 + z) * 2.0 * s2 * ds2)};
    // d_1 of the Jacobian factors dr/dX1, (dr/dX1)^2, dr/dX1
    const double J1[7] = {0.0, d2r, 0.0, 2.0 * dr * d2r, d2r, 0.0, 0.0};
    const double J2[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 2.0 * dth * d2th, 0.0};
    for (int n = 0; n < 7; ++n) {
        m.d1[n] = Kr[n] * dr * J[n] + K[n] * J1[n];
        m.d2[n] = Kt[n] * dth * J[n] + K[n] * J2[n];
    }
}

__global__ void k_geometry(GeoArgs A) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int gn2 = A.n2 + 2 * NG;
    const int np = (A.n1 + 2 * NG) * gn2;
    if (e >= np) return;
    const int i = e / gn2 - NG, j = e % gn2 - NG;
    for (int pass = 0; pass < 3; ++pass) {  // centre, X1 face, X2 face
        double* out = pass == 0 ? A.gc : (pass == 1 ? A.gf1 : A.gf2);
        const double fi = i + 0.5 - (pass == 1 ? 0.5 : 0.0);
        const double fj = j + 0.5 - (pass == 2 ? 0.5 : 0.0);
        MetricPoint m;
        if (A.mks) {
            mks_point(A.x1lo + fi * A.dx1, fj * A.dx2, A.spin, A.h, A.xb, A.nx, pass == 0, m);
        } else {
            for (int n = 0; n < 7; ++n) m.g[n] = m.d1[n] = m.d2[n] = 0.0;
            m.g[0] = -1.0; m.g[3] = 1.0; m.g[5] = 1.0; m.g[6] = 1.0;
            for (int n = 0; n < 6; ++n) m.gi[n] = 0.0;
            m.gi[0] = -1.0; m.gi[2] = 1.0; m.gi[4] = 1.0; m.gi[5] = 1.0;
            m.gdet = 1.0;
            m.alpha = 1.0;
            m.r = 1.0;
        }
        for (int n = 0; n < 7; ++n) out[(G_TT + n) * (int64_t)np + e] = m.g[n];
        for (int n = 0; n < 6; ++n) out[(GI_TT + n) * (int64_t)np + e] = m.gi[n];
        out[G_DET * (int64_t)np + e] = m.gdet;
        out[G_ALPHA * (int64_t)np + e] = m.alpha;
        out[G_IALPHA * (int64_t)np + e] = 1.0 / m.alpha;
        if (pass == 0) {
            for (int n = 0; n < 7; ++n) {
                out[(G_D1 + n) * (int64_t)np + e] = 0.5 * m.gdet * m.d1[n];
                out[(G_D2 + n) * (int64_t)np + e] = 0.5 * m.gdet * m.d2[n];
            }
            double rfl = A.fl_abs, ufl = A.fl_abs;
            if (A.mks) {
                rfl = fmax(rfl, A.rho_fl_coef * pow(m.r, A.rho_fl_pow));
                ufl = fmax(ufl, A.u_fl_coef * pow(m.r, A.u_fl_pow));
            }
            out[G_RHOFL * (int64_t)np + e] = rfl;
            out[G_UFL * (int64_t)np + e] = ufl;
        }
    }
}

// ------------------------------------------------------------------------------------------
// boundary ghosts (Sec. 4.1): radial copy keeping sqrt(-g) B^1 with no inflow at r_out, polar
// reflection flipping u~2 and B2; flat grids are periodic.  X3 is periodic by index wrap.
// Each ghost is computed directly from its interior source, so one launch covers corners too.
// A run fills as many ghost layers as its reconstruction reads: 2 for PLM, 3 for PPM.  With the
// polar velocity interpolation on (pole_fix = n_p > 0, MKS), u~2 of the n_p interior cells next
// to each pole becomes the straight line in X2 from zero at the pole to the centre of the first
// cell left alone; the same launch writes those cells, and every ghost whose source is one of them
// computes that value from the reference cell itself, so no thread reads a cell being written.
// ------------------------------------------------------------------------------------------

__global__ void k_bound(const RunDev* __restrict__ runs, const int* __restrict__ boff, int nruns, int which,
                        int sched) {
    const int bl = (sched & 1) ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int r = find_run(boff, nruns, bl);
    const RunDev& R = runs[r];
    if (!R.var->active) return;
    const int n1 = R.n1, n2 = R.n2, n3 = R.n3;
    const int64_t e = (int64_t)(bl - boff[r]) * blockDim.x + threadIdx.x;
    const int gd = 2 + R.ppm;                      // ghost layers this run reads
    const int npf = R.pole_fix;                    // 0 unless MKS with the polar interpolation
    const int ncolA = 2 * gd * (n2 + 2 * gd);      // X1 ghost rows, over the X2 ghosts too
    const int ncolB = 2 * gd * n1;                 // X2 ghost rows
    const int64_t total = (int64_t)(ncolA + ncolB + 2 * npf * n1) * n3;
    if (e >= total) return;
    const int k = (int)(e % n3);
    const int c = (int)(e / n3);
    double* __restrict__ P = which ? R.Ph : R.P;
    if (c >= ncolA + ncolB) {
        // interior cell next to a pole: u~2 = (m + 1/2)/(n_p + 1/2) times u~2 of the reference cell
        const int cc = c - ncolA - ncolB;
        const int jj = cc / n1, i = cc % n1;      // jj < 2 n_p
        const bool upper = jj >= npf;
        const int m = upper ? jj - npf : jj;      // cells between this one and the pole
        const int j = upper ? n2 - 1 - m : m;
        const int jr = upper ? n2 - 1 - npf : npf;
        const double f = ((double)m + 0.5) / ((double)npf + 0.5);
        gst(P + 3 * R.vs, (uint32_t)cell_index(R, i, j, k), gld(P + 3 * R.vs, (uint32_t)cell_index(R, i, jr, k)) * f);
        return;
    }
    int i, j;
    if (c < ncolA) {
        const int ii = c / (n2 + 2 * gd);
        i = ii < gd ? ii - gd : n1 + (ii - gd);
        j = c % (n2 + 2 * gd) - gd;
    } else {
        const int cc = c - ncolA;
        const int jj = cc / n1;
        j = jj < gd ? jj - gd : n2 + (jj - gd);
        i = cc % n1;
    }
    int is, js;
    if (R.mks) {
        is = i < 0 ? 0 : (i >= n1 ? n1 - 1 : i);
        js = j < 0 ? -1 - j : (j >= n2 ? 2 * n2 - 1 - j : j);
    } else {
        is = (i + n1) % n1;
        js = (j + n2) % n2;
    }
    const int64_t src = cell_index(R, is, js, k), dst = cell_index(R, i, j, k);
    // a source next to a pole has its u~2 rewritten by this launch: take it from the reference
    const int mp = npf == 0 ? -1 : (js < npf ? js : (js >= n2 - npf ? n2 - 1 - js : -1));
    double v[NPR];
#pragma unroll
    for (int q = 0; q < NPR; ++q)
        if (q != 3 || mp < 0) v[q] = gld(P + q * R.vs, (uint32_t)src);
    if (mp >= 0) {
        const int jr = js < npf ? npf : n2 - 1 - npf;
        const double f = ((double)mp + 0.5) / ((double)npf + 0.5);
        v[3] = gld(P + 3 * R.vs, (uint32_t)cell_index(R, is, jr, k)) * f;
    }
    if (R.mks) {
        if (i != is) {
            const int64_t np = R.gpts;
            v[5] *= R.gc[G_DET * np + geo_index(R, is, js)] / R.gc[G_DET * np + geo_index(R, i, js)];
            if (i >= n1) v[2] = fmax(v[2], 0.0);
        }
        if (j != js) {
            v[3] = -v[3];
            v[6] = -v[6];
        }
    }
#pragma unroll
    for (int q = 0; q < NPR; ++q) gst(P + q * R.vs, (uint32_t)dst, v[q]);
}

// ------------------------------------------------------------------------------------------
// face fluxes (Sec. 2.2): PLM/MC (or PPM) reconstruction of the 8 primitives, states and fluxes
// on both sides, simplified-dispersion wave speeds, LLF (or HLL) flux, per-direction max of c_w.
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Slot where flux_face stores component q (ENT: the diagnostic layout with every component).
template <int D, bool ENT>
__device__ __forceinline__ constexpr int flux_store_slot(int q) {
    return q == NCS - 1 ? FS_ENT : (q == 4 + D ? FS_BN : flux_slot<D>(q));
}

// Riemann flux through one face from its two reconstructed states (Sec. 2.2): the state, conserved
// vector, flux and simplified-dispersion speeds of each side, then LLF (or HLL) into out[q] for
// the NQ components the caller keeps; returns c_w.  The left side is finished before the right
// state is formed, which keeps the live register set to one state plus two flux vectors.  With
// ENT = false the entropy component (read only by the entropy inversion of the slow path, which
// recomputes it for its own faces) is neither computed nor combined: that saves both powers of rho.
template <int D, bool ENT>
__device__ __forceinline__ double riemann_face(const RunDev& R, const double* Pl, const double* Pr, const Geo& G,
                                               double* out) {
    constexpr int NQ = ENT ? NCS : 8;
    const double gam = R.gam;
    double Ul[NCS], Fl[NCS];
    double c1l, c2l;
    {
        St s;
        prim_state(Pl, G, gam, s);
        const double ent = ENT ? s.p * pow(Pl[0], 1.0 - gam) : 0.0;
        wave_speeds<D>(s, G, gam, c1l, c2l);
        flux_of<0>(Pl, s, G, ent, Ul);
        flux_of<D>(Pl, s, G, ent, Fl);
    }
    St s;
    prim_state(Pr, G, gam, s);
    const double entr = ENT ? s.p * pow(Pr[0], 1.0 - gam) : 0.0;
    double c1r, c2r;
    wave_speeds<D>(s, G, gam, c1r, c2r);
    const double cmax = fmax(0.0, fmax(c1r, c1l));
    const double cmin = fmax(0.0, fmax(-c2r, -c2l));
    const double cwf = fmax(cmax, cmin);
    double Ur[NCS], Fr[NCS];
    flux_of<0>(Pr, s, G, entr, Ur);
    flux_of<D>(Pr, s, G, entr, Fr);
    if (R.riemann == 1) {
        const double den = cmax + cmin;
        const double id = den > 0.0 ? 1.0 / den : 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            out[q] = den > 0.0 ? (cmax * Fl[q] + cmin * Fr[q] - cmax * cmin * (Ur[q] - Ul[q])) * id
                               : 0.5 * (Fl[q] + Fr[q]);
    } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) out[q] = 0.5 * (Fl[q] + Fr[q] - cwf * (Ur[q] - Ul[q]));
    }
    return cwf;
}

// One face: reconstruction from the cells on either side, then riemann_face; returns c_w (0 when
// the face does not count for the CFL step).  PPM reads three cells on each side of the face (PLM
// two), which the run's ghost layers cover.
template <int D, bool UNI, bool ENT, bool PPM>
__device__ __forceinline__ double flux_face(const RunDev& R, int i, int j, int k, int which, double* ent_out) {
    constexpr int NQ = ENT ? NCS : 8;
    const int n1 = R.n1, n2 = R.n2, n3 = R.n3;
    const int64_t ci = cell_index(R, i, j, k);
    double* __restrict__ F = R.F[D];
    Geo G;
    if (UNI) {
        // wave-uniform metric: read it ahead of any store of this kernel so that the loads are
        // known not to be clobbered and become scalar loads
        load_geo(D == 3 ? R.gc : R.gf[D], R.gpts, __builtin_amdgcn_readfirstlane((int)geo_index(R, i, j)), G);
    }
    if (D == 2 && R.mks && (j == 0 || j == n2)) {
        if (ent_out) {
            *ent_out = 0.0;
            return 0.0;
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (ENT || q != 4 + D) gst_nt(F + flux_store_slot<D, ENT>(q) * R.vs, (uint32_t)ci, 0.0);
        return 0.0;
    }
    const double* __restrict__ P = which ? R.Ph : R.P;
    int64_t cm3 = 0, cm2, cm1, cp1, cp2 = 0;
    if (D == 1) {
        cm2 = ci - 2 * R.s1; cm1 = ci - R.s1; cp1 = ci + R.s1;
        if (PPM) { cm3 = ci - 3 * R.s1; cp2 = ci + 2 * R.s1; }
    } else if (D == 2) {
        cm2 = ci - 2 * R.s2; cm1 = ci - R.s2; cp1 = ci + R.s2;
        if (PPM) { cm3 = ci - 3 * R.s2; cp2 = ci + 2 * R.s2; }
    } else {
        const int64_t base = ci - k;
        cm2 = base + (k >= 2 ? k - 2 : k - 2 + n3);
        cm1 = base + (k >= 1 ? k - 1 : k - 1 + n3);
        cp1 = base + (k + 1 < n3 ? k + 1 : k + 1 - n3);
        if (PPM) {  // n3 >= 3 for PPM runs (checked when a run is created)
            cm3 = base + (k >= 3 ? k - 3 : k - 3 + n3);
            cp2 = base + (k + 2 < n3 ? k + 2 : k + 2 - n3);
        }
    }
    double Pl[NPR], Pr[NPR];
#pragma unroll
    for (int q = 0; q < NPR; ++q) {
        const double* Pq = P + q * R.vs;
        const double a = gld(Pq, (uint32_t)cm2), b = gld(Pq, (uint32_t)cm1), c = gld(Pq, (uint32_t)ci),
                     d = gld(Pq, (uint32_t)cp1);
        if (PPM) {
            ppm_face(gld(Pq, (uint32_t)cm3), a, b, c, d, gld(Pq, (uint32_t)cp2), Pl[q], Pr[q]);
        } else {
            Pl[q] = b + mc_half_slope(a, b, c);
            Pr[q] = c - mc_half_slope(b, c, d);
        }
    }
    if (!UNI) load_geo(D == 3 ? R.gc : R.gf[D], R.gpts, geo_index(R, i, j), G);
    double out[NCS];
    const double cwf = riemann_face<D, ENT>(R, Pl, Pr, G, out);
    if (ent_out) {
        *ent_out = out[NCS - 1];
        return 0.0;
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (!ENT && q == 4 + D) continue;  // normal field component: not stored by the stage chain
        gst_nt(F + flux_store_slot<D, ENT>(q) * R.vs, (uint32_t)ci, out[q]);
    }
    if (D != 1 && (i < 0 || i >= n1)) return 0.0;
    if (D != 2 && (j < 0 || j >= n2)) return 0.0;
    return cwf;
}

// Entropy component of the Riemann flux through face (i,j,k) along D, recomputed on demand.
template <int D>
__device__ __forceinline__ double entropy_flux(const RunDev& R, int i, int j, int k, int which) {
    double f = 0.0;
    if (R.ppm) flux_face<D, false, true, true>(R, i, j, k, which, &f);
    else flux_face<D, false, true, false>(R, i, j, k, which, &f);
    return f;
}

// CFL bookkeeping of the face kernels: wave and workgroup maximum of c_w, then one atomic max per
// workgroup on the run's slot for direction D (non-negative doubles order like their bit patterns).
template <int D>
__device__ __forceinline__ void cfl_max(const RunDev& R, double cw) {
    __shared__ double red[4];
    cw = wave_max(cw);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = cw;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, red[w]);
        unsigned long long* slot = &R.var->cmax[D - 1];
        const unsigned long long bits = (unsigned long long)__double_as_longlong(m);
        const unsigned long long cur = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (bits > cur) atomicMax(slot, bits);
    }
}

template <int D, bool ENT, bool UNI, bool PPM>
__global__ __launch_bounds__(256) void k_flux(const RunDev* __restrict__ runs, const int* __restrict__ boff,
                                              int nruns, int which, int do_cfl, int sched) {
    const int bl = (sched & 1) ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int r = find_run(boff, nruns, bl);
    const RunDev& R = runs[r];
    if (!R.var->active) return;
    const int n1 = R.n1, n2 = R.n2, n3 = R.n3;
    const int i0 = D == 1 ? 0 : -R.act1;
    const int j0 = D == 2 ? 0 : -R.act2;
    const int ni = D == 1 ? n1 + 1 : n1 + 2 * R.act1;
    const int nj = D == 2 ? n2 + 1 : n2 + 2 * R.act2;
    // rows of n3 faces.  On the row path a wave is one row, and X1-face rows go i fastest so
    // that the stencil planes are read close together in time; otherwise a wave spans several
    // rows, and every direction goes j fastest, since consecutive j rows are adjacent in memory
    // (i-fastest rows would spread a wave over planes ~(n2+6) n3 doubles apart: with n3 = 1 every
    // lane of a load touches its own cache line).  X2 and X3 faces always go j fastest.  Every
    // index fits 31 bits (checked when a run is created); divisions use the run's precomputed
    // multipliers.
    const uint32_t nrows = (uint32_t)ni * (uint32_t)nj;
    uint32_t row, k;
    if (UNI) {
        // row path: a wave is 64 lanes of one row, decomposed once per wave; lanes past the row's
        // end wrap to its start and repeat faces other lanes form (same values stored twice)
        const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane(
            (int)((uint32_t)(bl - boff[r]) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
        row = fdiv(wv, R.fd_kc);
        k = ((wv - row * (uint32_t)R.nkc) << 6) + (threadIdx.x & 63);
        if (k >= (uint32_t)n3) k -= (uint32_t)n3;
    } else {
        const uint32_t e = (uint32_t)(bl - boff[r]) * blockDim.x + threadIdx.x;
        row = fdiv(e, R.fd_n3);
        k = e - row * (uint32_t)n3;
    }
    double cw = 0.0;
    if (row < nrows) {
        constexpr bool IFAST = D == 1 && UNI;
        // fd_row[3] divides by n2 + 2 act2, the X1-face row length in j
        const uint32_t q = fdiv(row, (D == 1 && !UNI) ? R.fd_row[3] : R.fd_row[D]);
        int i, j;
        if (IFAST) {
            j = (int)q + j0;
            i = (int)(row - q * (uint32_t)ni) + i0;
        } else {
            i = (int)q + i0;
            j = (int)(row - q * (uint32_t)nj) + j0;
        }
        cw = flux_face<D, UNI, ENT, PPM>(R, i, j, (int)k, which, nullptr);
    }
    if (do_cfl) cfl_max<D>(R, cw);
}

// Face fluxes along D in {1, 2} for PLM runs on the row path, marched along the face normal: a
// wave holds 64 consecutive k of one transverse row and walks a segment of `seg` faces along D,
// carrying the last two cells and the left state of its next face in registers, so each face
// loads one new cell (8 values) where the one-face kernel loads four, and each cell's MC slope is
// formed once instead of twice.  The arithmetic is that of k_flux<D> face for face (bit for bit).
// Waves are numbered 64-k chunk fastest, then along j: for X1 the transverse row (j) before the
// segment, for X2 the segment (along j) before the row (i), so that workgroups running side by side
// read neighbouring j rows rather than rows an i-plane apart (X2 faces at 256^3: 0.407 against
// 0.445 ms per launch with the row first; X1 faces with the segment first: 0.449 against 0.411).
template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_flux_march(const RunDev* __restrict__ runs, const int* __restrict__ boff,
                                                    int nruns, int which, int do_cfl, int sched) {
    static_assert(D == 1 || D == 2, "marching runs along X1 or X2");
    const int bl = (sched & 1) ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int r = find_run(boff, nruns, bl);
    const RunDev& R = runs[r];
    if (!R.var->active) return;
    const int n1 = R.n1, n2 = R.n2;
    const uint32_t nkc = (uint32_t)R.nkc;
    const int act = D == 1 ? R.act2 : R.act1;             // transverse halo rows for flux-CT
    const int ntr = D == 1 ? n2 : n1;                     // interior transverse rows
    const uint32_t nrow = (uint32_t)(ntr + 2 * act);
    const int nf = (D == 1 ? n1 : n2) + 1;                // faces along D
    const int seg = R.mseg[D - 1];
    const uint32_t nseg = (uint32_t)((nf + seg - 1) / seg);
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)((uint32_t)(bl - boff[r]) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const uint32_t t = wv / nkc, kc = wv - t * nkc;
    uint32_t sg, row;
    if (D == 2) {
        row = t / nseg;
        sg = t - row * nseg;
        if (row >= nrow) sg = nseg;                       // a rounded-up wave: no segment
    } else {
        sg = t / nrow;
        row = t - sg * nrow;
    }
    double cw = 0.0;
    if (sg < nseg) {
        int k = (int)(kc << 6) + (int)(threadIdx.x & 63);
        if (k >= R.n3) k -= R.n3;                         // a repeated face of the row
        const int a = (int)sg * seg, b = min(a + seg, nf);
        const int tr = (int)row - act;                    // j (D = 1) or i (D = 2)
        const bool counts = tr >= 0 && tr < ntr;          // halo rows do not enter the CFL step
        const uint32_t st = (uint32_t)(D == 1 ? R.s1 : R.s2);
        uint32_t c = (uint32_t)(D == 1 ? cell_index(R, a, tr, k) : cell_index(R, tr, a, k));
        const uint32_t vs = (uint32_t)R.vs;
        const double* __restrict__ P = which ? R.Ph : R.P;
        double* __restrict__ F = R.F[D];
        // window: c0 = cell f-1, c1 = cell f, Pl = left state of face f-1/2
        double c0[NPR], c1[NPR], Pl[NPR];
#pragma unroll
        for (int q = 0; q < NPR; ++q) {
            const double* Pq = P + q * vs;
            const double m2 = gld(Pq, c - 2 * st), m1 = gld(Pq, c - st);
            c1[q] = gld(Pq, c);
            c0[q] = m1;
            Pl[q] = m1 + mc_half_slope(m2, m1, c1[q]);
        }
        for (int f = a; f < b; ++f, c += st) {
            double Pr[NPR], Pn[NPR];
#pragma unroll
            for (int q = 0; q < NPR; ++q) {
                const double c2 = gld(P + q * vs, c + st);
                const double h = mc_half_slope(c0[q], c1[q], c2);
                Pr[q] = c1[q] - h;
                Pn[q] = c1[q] + h;
                c0[q] = c1[q];
                c1[q] = c2;
            }
            if (D == 2 && R.mks && (f == 0 || f == n2)) {
                // polar axis: no flux through the pole
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (q != 4 + D) gst_nt(F + flux_slot<D>(q) * vs, c, 0.0);
            } else {
                Geo G;
                load_geo_k(R.gf[D], R.gpts,
                           (uint32_t)__builtin_amdgcn_readfirstlane((int)(D == 1 ? geo_index(R, f, tr) : geo_index(R, tr, f))),
                           G);
                double out[NCS];
                const double cwf = riemann_face<D, false>(R, Pl, Pr, G, out);
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (q != 4 + D) gst_nt(F + flux_slot<D>(q) * vs, c, out[q]);
                if (counts) cw = fmax(cw, cwf);
            }
#pragma unroll
            for (int q = 0; q < NPR; ++q) Pl[q] = Pn[q];
        }
    }
    if (do_cfl) cfl_max<D>(R, cw);
}

// Face fluxes along D in {1, 2} for PPM runs on the row path, two faces per thread: a wave holds 64
// consecutive k of one transverse row and the faces f0 = 2p and f0 + 1 along D.  Face f lies between
// cells f-1 and f and needs cells f-3 .. f+2, so the pair loads cells f0-3 .. f0+3 once (seven
// loads for two faces where the one-face kernel makes twelve) and shares three slopes and two
// interface values (Colella & Woodward, the formulas of ppm_face).  Waves are numbered 64-k chunk
// fastest, then pair, then transverse row, so that the pairs sharing stencil cells run together
// (pair-fastest rather than row-fastest order: 0.68 against 0.71 ms per launch at 256^3).  Held to 128 VGPRs (4 waves per SIMD, 8-12 B of spills):
// at 130 the X1 instantiation ran 3 waves and 14 % slower.
template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_flux_ppm_pair(const RunDev* __restrict__ runs, const int* __restrict__ boff,
                                                       int nruns, int which, int do_cfl, int sched) {
    static_assert(D == 1 || D == 2, "pairs along X1 or X2");
    constexpr double third = 1.0 / 3.0;
    const int bl = (sched & 1) ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int r = find_run(boff, nruns, bl);
    const RunDev& R = runs[r];
    if (!R.var->active) return;
    const int n1 = R.n1, n2 = R.n2;
    const uint32_t nkc = (uint32_t)R.nkc;
    const int act = D == 1 ? R.act2 : R.act1;             // transverse halo rows for flux-CT
    const int ntr = D == 1 ? n2 : n1;                     // interior transverse rows
    const uint32_t nrow = (uint32_t)(ntr + 2 * act);
    const int nf = (D == 1 ? n1 : n2) + 1;                // faces along D
    const uint32_t npair = (uint32_t)((nf + 1) / 2);
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)((uint32_t)(bl - boff[r]) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const uint32_t t = wv / nkc, kc = wv - t * nkc;
    const uint32_t row = t / npair, pr = t - row * npair;
    double cw = 0.0;
    if (row < nrow) {
        int k = (int)(kc << 6) + (int)(threadIdx.x & 63);
        if (k >= R.n3) k -= R.n3;                         // a repeated face of the row
        const int f0 = 2 * (int)pr;
        const bool two = f0 + 1 < nf;                     // the last pair may hold one face
        const int tr = (int)row - act;                    // j (D = 1) or i (D = 2)
        const bool counts = tr >= 0 && tr < ntr;          // halo rows do not enter the CFL step
        const uint32_t st = (uint32_t)(D == 1 ? R.s1 : R.s2);
        const uint32_t c = (uint32_t)(D == 1 ? cell_index(R, f0, tr, k) : cell_index(R, tr, f0, k));
        const uint32_t vs = (uint32_t)R.vs;
        const double* __restrict__ P = which ? R.Ph : R.P;
        double* __restrict__ F = R.F[D];
        double Pl0[NPR], Pr0[NPR], Pl1[NPR], Pr1[NPR];
#pragma unroll
        for (int q = 0; q < NPR; ++q) {
            const double* Pq = P + q * vs;
            const double a = gld(Pq, c - 3 * st), b = gld(Pq, c - 2 * st), cc = gld(Pq, c - st);
            const double d = gld(Pq, c), e = gld(Pq, c + st), f = gld(Pq, c + 2 * st);
            const double g = two ? gld(Pq, c + 3 * st) : f;
            const double hb = mc_half_slope(a, b, cc), hc = mc_half_slope(b, cc, d);
            const double hd = mc_half_slope(cc, d, e), he = mc_half_slope(d, e, f);
            const double ibc = b + 0.5 * (cc - b) - (hc - hb) * third;
            const double icd = cc + 0.5 * (d - cc) - (hd - hc) * third;
            const double ide = d + 0.5 * (e - d) - (he - hd) * third;
            Pl0[q] = ppm_upper_edge(cc, ibc, icd);
            Pr0[q] = ppm_lower_edge(d, icd, ide);
            const double hf = mc_half_slope(e, f, g);
            const double ief = e + 0.5 * (f - e) - (hf - he) * third;
            Pl1[q] = ppm_upper_edge(d, icd, ide);
            Pr1[q] = ppm_lower_edge(e, ide, ief);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h == 1 && !two) break;
            const int fh = f0 + h;
            const uint32_t ch = c + (uint32_t)h * st;
            if (D == 2 && R.mks && (fh == 0 || fh == n2)) {
                // polar axis: no flux through the pole
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (q != 4 + D) gst_nt(F + flux_slot<D>(q) * vs, ch, 0.0);
                continue;
            }
            Geo G;
            load_geo_k(R.gf[D], R.gpts,
                       (uint32_t)__builtin_amdgcn_readfirstlane((int)(D == 1 ? geo_index(R, fh, tr) : geo_index(R, tr, fh))),
                       G);
            double out[NCS];
            const double cwf = riemann_face<D, false>(R, h ? Pl1 : Pl0, h ? Pr1 : Pr0, G, out);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q != 4 + D) gst_nt(F + flux_slot<D>(q) * vs, ch, out[q]);
            if (counts) cw = fmax(cw, cwf);
        }
    }
    if (do_cfl) cfl_max<D>(R, cw);
}

// 64-bit lane shifts across the whole wave (DPP wave_shr:1 and wave_shl:1 on both halves): lane l
// takes the value of lane l - 1 (shr) or l + 1 (shl); the one lane without a source keeps `old`.
__device__ __forceinline__ double lane_shr1(double old, double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_shl1(double old, double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// value of lane l (wave-uniform l) in every lane
__device__ __forceinline__ double lane_read(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// X3 face fluxes of runs on the row path: a wave is 64 lanes of one (i, j) row, lane l of chunk c at
// k = (64 c + l) mod n3, and its face k - 1/2 needs cells k-2 .. k+1 (PLM) or k-3 .. k+2 (PPM).  The
// row is periodic, so adjacent lanes hold neighbouring k also where the lanes wrap past the row's
// end (those lanes repeat faces of the row's start).  Each lane loads its own cell and one edge
// cell (lane 0: k0-1, lane 1: k0-2, lane 63: k0+64, and for PPM lane 2: k0-3, lane 62: k0+65;
// periodic in k; the rest reload their own), and takes its neighbours' cells from the adjacent
// lanes: two loads per primitive instead of four (PLM) or six (PPM).  The PLM arithmetic is that
// of k_flux<3> face for face (bit for bit); the PPM faces agree with it to rounding.
template <bool PPM>
__global__ __launch_bounds__(256) void k_flux3_lanes(const RunDev* __restrict__ runs, const int* __restrict__ boff,
                                                     int nruns, int which, int do_cfl, int sched) {
    const int bl = (sched & 1) ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int r = find_run(boff, nruns, bl);
    const RunDev& R = runs[r];
    if (!R.var->active) return;
    const int n1 = R.n1, n2 = R.n2, n3 = R.n3;
    const uint32_t nkc = (uint32_t)R.nkc;
    const uint32_t nj = (uint32_t)(n2 + 2 * R.act2);
    const uint32_t nrows = (uint32_t)(n1 + 2 * R.act1) * nj;
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)((uint32_t)(bl - boff[r]) * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const uint32_t row = wv / nkc, kc = wv - row * nkc;
    double cw = 0.0;
    if (row < nrows) {
        const uint32_t qi = row / nj;
        const int i = (int)qi - R.act1, j = (int)(row - qi * nj) - R.act2;
        const int lane = (int)(threadIdx.x & 63);
        const int k0 = (int)(kc << 6);
        int k = k0 + lane;
        if (k >= n3) k -= n3;            // past the row's end: the row is periodic, so lane
                                         // neighbours stay k neighbours (repeated faces)
        const uint32_t base = (uint32_t)cell_index(R, i, j, 0);
        int ke = k;
        if (lane == 0) ke = k0 - 1;
        else if (lane == 1) ke = k0 - 2;
        else if (lane == 63) ke = k0 + 64;
        else if (PPM && lane == 2) ke = k0 - 3;
        else if (PPM && lane == 62) ke = k0 + 65;
        ke = ke < 0 ? ke + n3 : (ke >= n3 ? ke - n3 : ke);
        const uint32_t vs = (uint32_t)R.vs;
        const double* __restrict__ P = which ? R.Ph : R.P;
        Geo G;
        load_geo_k(R.gc, R.gpts, (uint32_t)__builtin_amdgcn_readfirstlane((int)geo_index(R, i, j)), G);
        double Pl[NPR], Pr[NPR];
#pragma unroll
        for (int q = 0; q < NPR; ++q) {
            const double* Pq = P + q * vs;
            const double c = gld(Pq, base + (uint32_t)k);
            const double e = gld(Pq, base + (uint32_t)ke);
            const double m1 = lane_shr1(e, c);                                     // cell k-1
            const double m2 = lane_shr1(lane_read(e, 1), m1);                      // cell k-2
            const double p1 = lane_shl1(e, c);                                     // cell k+1
            if (PPM) {
                const double m3 = lane_shr1(lane_read(e, 2), m2);                  // cell k-3
                const double p2 = lane_shl1(lane_read(e, 62), p1);                 // cell k+2
                ppm_face(m3, m2, m1, c, p1, p2, Pl[q], Pr[q]);
            } else {
                Pl[q] = m1 + mc_half_slope(m2, m1, c);
                Pr[q] = c - mc_half_slope(m1, c, p1);
            }
        }
        double out[NCS];
        const double cwf = riemann_face<3, false>(R, Pl, Pr, G, out);
        double* __restrict__ F = R.F[3];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (q != 7) gst_nt(F + flux_slot<3>(q) * vs, base + (uint32_t)k, out[q]);
        if (i >= 0 && i < n1 && j >= 0 && j < n2) cw = cwf;
    }
    if (do_cfl) cfl_max<3>(R, cw);
}

// ------------------------------------------------------------------------------------------
// CFL step and per-step bookkeeping: dt = cfl / sum_d max(c_w)/dX^d (Sec. 2.2)
// ------------------------------------------------------------------------------------------

__global__ void k_dt(const RunDev* __restrict__ runs, int nruns) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nruns) return;
    const RunDev& R = runs[r];
    RunVar* V = R.var;
    if (!V->active) return;
    double dt = V->dt_req;
    if (dt <= 0.0) {
        double inv = 0.0;
        if (R.act1) inv += __longlong_as_double((long long)V->cmax[0]) * R.idx[1];
        if (R.act2) inv += __longlong_as_double((long long)V->cmax[1]) * R.idx[2];
        if (R.act3) inv += __longlong_as_double((long long)V->cmax[2]) * R.idx[3];
        dt = R.cfl / inv;
    }
    V->dt = dt;
    V->t += dt;
    V->nstep += 1;
    V->steps_left -= 1;
    V->cmax[0] = V->cmax[1] = V->cmax[2] = 0ull;
    V->nfail_last = 0;
}

// ------------------------------------------------------------------------------------------
// conservative update: flux-CT (edge EMFs from four face fluxes, B fluxes replaced by the
// average of the two edges bounding each face), U = U(P^n) + c dt (-sum dF/dX + S(P_in)),
// inversion, floors; failed cells go to the run's fail list.
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ void source_terms(const St& s, const double* __restrict__ gc, int64_t np, int64_t gi,
                                             const Geo& G, double* S) {
    const double wb = s.w + s.bsq;
    const double pt = s.p + 0.5 * s.bsq;
    // contravariant T^{kl} for the 7 stored (k,l) pairs: tt, t1, t3, 11, 13, 22, 33
    const double T[7] = {
        wb * s.ut * s.ut + pt * G.Gtt - s.bt * s.bt,
        wb * s.ut * s.u1 + pt * G.Gt1 - s.bt * s.b1,
        wb * s.ut * s.u3 - s.bt * s.b3,
        wb * s.u1 * s.u1 + pt * G.G11 - s.b1 * s.b1,
        wb * s.u1 * s.u3 + pt * G.G13 - s.b1 * s.b3,
        wb * s.u2 * s.u2 + pt * G.G22 - s.b2 * s.b2,
        wb * s.u3 * s.u3 + pt * G.G33 - s.b3 * s.b3,
    };
    const double mult[7] = {1.0, 2.0, 2.0, 1.0, 2.0, 1.0, 1.0};
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int n = 0; n < 7; ++n) {
        s1 += mult[n] * T[n] * gld(gc + (G_D1 + n) * np, (uint32_t)gi);
        s2 += mult[n] * T[n] * gld(gc + (G_D2 + n) * np, (uint32_t)gi);
    }
    S[0] = 0.0;
    S[1] = s1;
    S[2] = s2;
    S[3] = 0.0;
}

// ------------------------------------------------------------------------------------------
// flux-CT edge EMFs (Sec. 2.2): each edge EMF is the average of the four face fluxes of the
// transverse field around the edge, formed once per edge by k_emf and kept, for the rest of the
// stage, in slot FS_EMF of a face array (that slot holds the normal field component only in the
// diagnostic copy, never during a step):
//   E3 at (i-1/2, j-1/2, k) in F[1], E1 at (i, j-1/2, k-1/2) in F[2], E2 at (i-1/2, j, k-1/2) in F[3],
// each at the cell index of (i, j, k).  EMFs on the polar axis (MKS, j' = 0 or n2) are zero.
// ------------------------------------------------------------------------------------------

constexpr int FS_EMF = FS_BN;

__device__ __forceinline__ const double* emf_slot(const RunDev& R, int d) {
    return R.F[d == 3 ? 1 : (d == 1 ? 2 : 3)] + FS_EMF * R.vs;
}

// one thread per edge site (i', j', k) in [0, n1] x [0, n2] x [0, n3): E3 where X1 and X2 are active,
// E2 (j' < n2) where X1 and X3 are, E1 (i' < n1) where X2 and X3 are
__global__ __launch_bounds__(256) void k_emf(const RunDev* __restrict__ runs, const int* __restrict__ boff, int nruns,
                                             int sched) {
    const int bl = (sched & 1) ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int r = find_run(boff, nruns, bl);
    const RunDev& R = runs[r];
    if (!R.var->active) return;
    const int n1 = R.n1, n2 = R.n2, n3 = R.n3;
    const uint32_t e = (uint32_t)(bl - boff[r]) * blockDim.x + threadIdx.x;
    if (e >= (uint32_t)(n1 + 1) * (uint32_t)(n2 + 1) * (uint32_t)n3) return;
    const uint32_t t = fdiv(e, R.fd_n3);
    const int k = (int)(e - t * (uint32_t)n3);
    const uint32_t i = fdiv(t, R.fd_row[2]);   // n2 + 1
    const int j = (int)(t - i * (uint32_t)(n2 + 1));
    const uint32_t c = (uint32_t)cell_index(R, (int)i, j, k);
    const uint32_t s1 = (uint32_t)R.s1, s2 = (uint32_t)R.s2, vs = (uint32_t)R.vs;
    const uint32_t ckm = c - (uint32_t)k + (uint32_t)(k == 0 ? n3 - 1 : k - 1);
    const bool axis = R.mks && (j == 0 || j == n2);
    if (R.act1 && R.act2) {
        const double* F1b2 = R.F[1] + flux_slot<1>(6) * vs;
        const double* F2b1 = R.F[2] + flux_slot<2>(5) * vs;
        const double v = axis ? 0.0 : 0.25 * (gld(F1b2, c - s2) + gld(F1b2, c) - gld(F2b1, c - s1) - gld(F2b1, c));
        gst_nt(R.F[1] + FS_EMF * vs, c, v);
    }
    if (R.act1 && R.act3 && j < n2) {
        const double* F3b1 = R.F[3] + flux_slot<3>(5) * vs;
        const double* F1b3 = R.F[1] + flux_slot<1>(7) * vs;
        gst_nt(R.F[3] + FS_EMF * vs, c, 0.25 * (gld(F3b1, c - s1) + gld(F3b1, c) - gld(F1b3, ckm) - gld(F1b3, c)));
    }
    if (R.act2 && R.act3 && (int)i < n1) {
        const double* F2b3 = R.F[2] + flux_slot<2>(7) * vs;
        const double* F3b2 = R.F[3] + flux_slot<3>(6) * vs;
        const double v = axis ? 0.0 : 0.25 * (gld(F2b3, ckm) + gld(F2b3, c) - gld(F3b2, c - s2) - gld(F3b2, c));
        gst_nt(R.F[2] + FS_EMF * vs, c, v);
    }
}

// Conserved state after the stage update of interior cell (i,j,k): flux-CT, the flux divergence,
// the centred source from the stage-input primitives Pg, U = U(P^n) + c dt L.  With ENT = false
// the entropy component (used only by the entropy inversion) is skipped.
template <bool ENT, bool UNI, int STAGE>
__device__ __forceinline__ void stage_state(const RunDev& R, int i, int j, int k, double* U, double* Pg,
                                            Geo& G, St& sg, int64_t& gi_out) {
    constexpr int stage = STAGE;
    const int n3 = R.n3;
    const uint32_t ci = (uint32_t)cell_index(R, i, j, k);
    const uint32_t vs = (uint32_t)R.vs, s1 = (uint32_t)R.s1, s2 = (uint32_t)R.s2;
    const uint32_t kb = ci - (uint32_t)k;
    const uint32_t ckp = kb + (uint32_t)(k + 1 == n3 ? 0 : k + 1);
    const double* __restrict__ F1 = R.F[1];
    const double* __restrict__ F2 = R.F[2];
    const double* __restrict__ F3 = R.F[3];
    const bool has3 = R.act1 && R.act2, has1 = R.act2 && R.act3, has2 = R.act1 && R.act3;

    // ---- L = -sum_d (F_d(+) - F_d(-)) / dX^d with flux-CT for the field components ----
    double L[NCS];
#pragma unroll
    for (int q = 0; q < NCS; ++q) L[q] = 0.0;
    if (ENT) {
        const int which = stage - 1;
        if (R.act1) L[8] -= (entropy_flux<1>(R, i + 1, j, k, which) - entropy_flux<1>(R, i, j, k, which)) * R.idx[1];
        if (R.act2) L[8] -= (entropy_flux<2>(R, i, j + 1, k, which) - entropy_flux<2>(R, i, j, k, which)) * R.idx[2];
        if (R.act3) {
            const int kp = k + 1 == n3 ? 0 : k + 1;
            L[8] -= (entropy_flux<3>(R, i, j, kp, which) - entropy_flux<3>(R, i, j, k, which)) * R.idx[3];
        }
    }
    if (R.act1) {
#pragma unroll
        for (int q = 0; q < 5; ++q) L[q] -= (gld(F1 + q * vs, ci + s1) - gld(F1 + q * vs, ci)) * R.idx[1];
    }
    if (R.act2) {
#pragma unroll
        for (int q = 0; q < 5; ++q) L[q] -= (gld(F2 + q * vs, ci + s2) - gld(F2 + q * vs, ci)) * R.idx[2];
    }
    if (R.act3) {
#pragma unroll
        for (int q = 0; q < 5; ++q) L[q] -= (gld(F3 + q * vs, ckp) - gld(F3 + q * vs, ci)) * R.idx[3];
    }
    // field components: F^d(B^d) is not used; transverse ones come from the edge EMFs where both
    // directions of the edge are active, from the face fluxes themselves otherwise
    double f1b2m = 0.0, f1b2p = 0.0, f1b3m = 0.0, f1b3p = 0.0;
    double f2b1m = 0.0, f2b1p = 0.0, f2b3m = 0.0, f2b3p = 0.0;
    double f3b1m = 0.0, f3b1p = 0.0, f3b2m = 0.0, f3b2p = 0.0;
    if (has3) {
        // E3 on the four edges (i'-1/2, j'-1/2), i' in {i, i+1}, j' in {j, j+1}
        const double* E3 = emf_slot(R, 3);
        const double e00 = gld(E3, ci), e10 = gld(E3, ci + s1), e01 = gld(E3, ci + s2), e11 = gld(E3, ci + s1 + s2);
        f1b2m = 0.5 * (e00 + e01);
        f1b2p = 0.5 * (e10 + e11);
        f2b1m = -0.5 * (e00 + e10);
        f2b1p = -0.5 * (e01 + e11);
    } else {
        if (R.act1) {
            f1b2m = gld(F1 + flux_slot<1>(6) * vs, ci);
            f1b2p = gld(F1 + flux_slot<1>(6) * vs, ci + s1);
        }
        if (R.act2) {
            f2b1m = gld(F2 + flux_slot<2>(5) * vs, ci);
            f2b1p = gld(F2 + flux_slot<2>(5) * vs, ci + s2);
        }
    }
    if (has1) {
        // E1 on the edges (i, j'-1/2, k'-1/2), j' in {j, j+1}, k' in {k, k+1}
        const double* E1 = emf_slot(R, 1);
        const double e00 = gld(E1, ci), e10 = gld(E1, ci + s2), e01 = gld(E1, ckp), e11 = gld(E1, ckp + s2);
        f2b3m = 0.5 * (e00 + e01);
        f2b3p = 0.5 * (e10 + e11);
        f3b2m = -0.5 * (e00 + e10);
        f3b2p = -0.5 * (e01 + e11);
    } else {
        if (R.act2) {
            f2b3m = gld(F2 + flux_slot<2>(7) * vs, ci);
            f2b3p = gld(F2 + flux_slot<2>(7) * vs, ci + s2);
        }
        if (R.act3) {
            f3b2m = gld(F3 + flux_slot<3>(6) * vs, ci);
            f3b2p = gld(F3 + flux_slot<3>(6) * vs, ckp);
        }
    }
    if (has2) {
        // E2 on the edges (i'-1/2, j, k'-1/2), i' in {i, i+1}, k' in {k, k+1}
        const double* E2 = emf_slot(R, 2);
        const double e00 = gld(E2, ci), e10 = gld(E2, ci + s1), e01 = gld(E2, ckp), e11 = gld(E2, ckp + s1);
        f1b3m = -0.5 * (e00 + e01);
        f1b3p = -0.5 * (e10 + e11);
        f3b1m = 0.5 * (e00 + e10);
        f3b1p = 0.5 * (e01 + e11);
    } else {
        if (R.act1) {
            f1b3m = gld(F1 + flux_slot<1>(7) * vs, ci);
            f1b3p = gld(F1 + flux_slot<1>(7) * vs, ci + s1);
        }
        if (R.act3) {
            f3b1m = gld(F3 + flux_slot<3>(5) * vs, ci);
            f3b1p = gld(F3 + flux_slot<3>(5) * vs, ckp);
        }
    }
    if (R.act1) {
        L[6] -= (f1b2p - f1b2m) * R.idx[1];
        L[7] -= (f1b3p - f1b3m) * R.idx[1];
    }
    if (R.act2) {
        L[5] -= (f2b1p - f2b1m) * R.idx[2];
        L[7] -= (f2b3p - f2b3m) * R.idx[2];
    }
    if (R.act3) {
        L[5] -= (f3b1p - f3b1m) * R.idx[3];
        L[6] -= (f3b2p - f3b2m) * R.idx[3];
    }

    int64_t gi = geo_index(R, i, j);
    if (UNI) gi = __builtin_amdgcn_readfirstlane((int)gi);
    gi_out = gi;
    load_geo(R.gc, R.gpts, gi, G);
    const double gam = R.gam;
    const double* __restrict__ Pn = R.P;
    const double* __restrict__ Pin = stage == 1 ? R.P : R.Ph;
#pragma unroll
    for (int q = 0; q < NPR; ++q) Pg[q] = gld_nt(Pin + q * vs, ci);
    prim_state(Pg, G, gam, sg);
    if (stage == 1) {
        // the stage input is P^n itself: U(P^n) comes from the same state
        flux_of<0>(Pg, sg, G, ENT ? sg.p * pow(Pg[0], 1.0 - gam) : 0.0, U);
    } else {
        double P0[NPR];
#pragma unroll
        for (int q = 0; q < NPR; ++q) P0[q] = gld_nt(Pn + q * vs, ci);
        St s0;
        prim_state(P0, G, gam, s0);
        flux_of<0>(P0, s0, G, ENT ? s0.p * pow(P0[0], 1.0 - gam) : 0.0, U);
    }
    double S[4];
    source_terms(sg, R.gc, R.gpts, gi, G, S);
    L[1] += S[0];
    L[2] += S[1];
    L[3] += S[2];
    L[4] += S[3];
    const double h = (stage == 1 ? 0.5 : 1.0) * R.var->dt;
#pragma unroll
    for (int q = 0; q < NCS; ++q) U[q] += h * L[q];
}

// Fast path of the inversion: Newton-Raphson accepted when converged and physical, floors, and
// the Lorentz cap.  Cells that need the entropy method (beta switch), Brent, or a magnetisation
// ceiling go to the run's slow list and are finished by k_update_slow with the full procedure.
template <bool UNI, int STAGE>
__device__ __forceinline__ void update_fast(const RunDev& R, int i, int j, int k) {
    constexpr int stage = STAGE;
    double U[NCS], Pg[NPR];
    Geo G;
    St sg;
    int64_t gi;
    stage_state<false, UNI, STAGE>(R, i, j, k, U, Pg, G, sg, gi);
    bool slow = sg.p < R.beta_ent * 0.5 * sg.bsq;
    double P[NPR];
    if (!slow) {
        Inv q;
        inv_setup(U, G, R, q);
        double W = sg.lor * sg.lor * sg.w;
        const double qsq = sg.lor * sg.lor - 1.0;
        double v2 = qsq / (1.0 + qsq);
        slow = !newton2d(q, R.c2p_tol, R.c2p_maxit, W, v2);
        if (!slow) {
            slow = !finish_energy(q, G, W, v2, P);
            if (!slow) {
                P[5] = U[5] * q.ig;
                P[6] = U[6] * q.ig;
                P[7] = U[7] * q.ig;
                P[0] = fmax(P[0], gld(R.gc + G_RHOFL * R.gpts, (uint32_t)gi));
                P[1] = fmax(P[1], gld(R.gc + G_UFL * R.gpts, (uint32_t)gi));
                St s;
                prim_state(P, G, R.gam, s);
                slow = (s.bsq / R.bsq_rho_max - P[0] > 0.0) || (s.bsq / R.bsq_u_max - P[1] > 0.0);
                if (!slow && s.lor > R.gamma_max) {
                    const double f = sqrt((R.gamma_max * R.gamma_max - 1.0) / (s.lor * s.lor - 1.0));
                    P[2] *= f;
                    P[3] *= f;
                    P[4] *= f;
                }
            }
        }
    }
    if (slow) {
        const int pos = atomicAdd(&R.var->slow_count, 1);
        R.slow_list[pos] = (int)(((int64_t)i * R.n2 + j) * R.n3 + k);
        return;
    }
    const int64_t ci = cell_index(R, i, j, k);
    double* __restrict__ Pout = stage == 1 ? R.Ph : R.P;
    R.code[ci] = 0;
#pragma unroll
    for (int q = 0; q < NPR; ++q) gst_nt(Pout + q * R.vs, (uint32_t)ci, P[q]);
}

// UNI: the launch covers only row-path runs (a wave's cells share (r, theta), metric by scalar
// loads; lanes past the row's end do nothing); the engine keeps a separate block table for the
// other runs.  One code path per instantiation keeps the register count low.
template <int STAGE, bool UNI>
__global__ __launch_bounds__(256) void k_update(const RunDev* __restrict__ runs, const int* __restrict__ boff,
                                                int nruns, int sched) {
    const int bl = (sched & 1) ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int r = find_run(boff, nruns, bl);
    const RunDev& R = runs[r];
    if (!R.var->active) return;
    if (UNI) {
        // The blockDim/64 waves of a workgroup take consecutive j at the same (i, 64 k), so the X2
        // faces and flux-CT neighbours they share are fetched together.  Block order: 64-k chunk
        // fastest, then j group, then i (n2 padded to a multiple of the group).
        const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        const uint32_t lw = blockDim.x == 256 ? 2u : (blockDim.x == 128 ? 1u : 0u);
        const uint32_t eb = (uint32_t)(bl - boff[r]);
        const uint32_t t = fdiv(eb, R.fd_kc);
        const uint32_t kc = eb - t * (uint32_t)R.nkc;
        const uint32_t i = fdiv(t, R.fd_jg[lw]);
        const int j = (int)(((t - i * (uint32_t)((R.n2 + (1 << lw) - 1) >> lw)) << lw) + wv);
        if (j >= R.n2) return;
        const int k = (int)(kc << 6) + (int)(threadIdx.x & 63);
        if (k >= R.n3) return;                            // lanes past the row's end
        update_fast<UNI, STAGE>(R, (int)i, j, k);
    } else {
        const uint32_t e = (uint32_t)(bl - boff[r]) * blockDim.x + threadIdx.x;
        if (e >= (uint32_t)R.n1 * (uint32_t)R.n2 * (uint32_t)R.n3) return;
        const uint32_t t = fdiv(e, R.fd_n3);
        const uint32_t i = fdiv(t, R.fd_n2);
        const int j = (int)(t - i * (uint32_t)R.n2), k = (int)(e - t * (uint32_t)R.n3);
        update_fast<UNI, STAGE>(R, (int)i, j, k);
    }
}

// Slow path: the full inversion (beta switch, NR, Brent on W, entropy) and the full floors with
// ceilings, for the cells the fast path listed.  SLOWB workgroups per run stride over the list.
constexpr int SLOWB = 64;

__global__ __launch_bounds__(256) void k_update_slow(const RunDev* __restrict__ runs, int nruns, int stage) {
    const int r = blockIdx.x / SLOWB;
    const RunDev& R = runs[r];
    if (!R.var->active) return;
    const int n = R.var->slow_count;
    const int n2 = R.n2, n3 = R.n3;
    for (int x = (blockIdx.x % SLOWB) * blockDim.x + threadIdx.x; x < n; x += SLOWB * blockDim.x) {
        const int e = R.slow_list[x];
        const int k = e % n3, t = e / n3, j = t % n2, i = t / n2;
        double U[NCS], Pg[NPR];
        Geo G;
        St sg;
        int64_t gi;
        if (stage == 1) stage_state<true, false, 1>(R, i, j, k, U, Pg, G, sg, gi);
        else stage_state<true, false, 2>(R, i, j, k, U, Pg, G, sg, gi);
        double P[NPR];
#pragma unroll
        for (int q = 0; q < NPR; ++q) P[q] = Pg[q];
        const int m = invert_cell(U, Pg, G, R, P);
        if (m >= 0) {
            apply_floors(R, G, R.gc[G_RHOFL * R.gpts + gi], R.gc[G_UFL * R.gpts + gi], P);
        } else {
            const int pos = atomicAdd(&R.var->fail_count, 1);
            R.fail_list[pos] = e;
        }
        const int64_t ci = cell_index(R, i, j, k);
        double* __restrict__ Pout = stage == 1 ? R.Ph : R.P;
        R.code[ci] = (int8_t)m;
#pragma unroll
        for (int q = 0; q < NPR; ++q) Pout[q * R.vs + ci] = P[q];
    }
}

// ------------------------------------------------------------------------------------------
// fixups (Sec. 2.3): Jacobi rounds of neighbour averaging of the non-field primitives over the
// failed cells of each run -- the 4-cross average when all four are valid, else the 4-diagonal
// average, else the average of whichever of the 8 are valid; neighbours outside the interior do
// not count.  Cells fixed in a round become valid in the next one; a cell still failed after the
// last round takes rho, u, u~ from the stage input and keeps its field.
// The first round reads only cells that were valid before it, so k_fixup_first (averaging) and
// k_fixup_settle (floors) spread it over FIXB workgroups per run; k_fixup (one workgroup per run)
// runs the later rounds, each of which needs the previous one complete, for the cells still failed.
// Most failures are isolated cells that the first round fixes.
// ------------------------------------------------------------------------------------------

constexpr int FIXB = 64;

// averaging step of one round for failed cell e (code -1): the average goes to Pout and the cell
// is marked pending (4: valid from the next round on); a cell with no valid neighbour stays -1
__device__ __forceinline__ void fixup_average(const RunDev& R, double* __restrict__ Pout, int e) {
    const int n1 = R.n1, n2 = R.n2, n3 = R.n3;
    const int64_t vs = R.vs;
    const int k = e % n3, t = e / n3, j = t % n2, i = t / n2;
    const int64_t ci = cell_index(R, i, j, k);
    if (R.code[ci] != -1) return;
    const int di[8] = {1, -1, 0, 0, 1, 1, -1, -1};
    const int dj[8] = {0, 0, 1, -1, 1, -1, 1, -1};
    bool ok[8];
    int nvalid = 0;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int ii = i + di[s], jj = j + dj[s];
        bool v = ii >= 0 && ii < n1 && jj >= 0 && jj < n2;
        if (v) {
            const int8_t c = R.code[cell_index(R, ii, jj, k)];
            v = c >= 0 && c <= 3;
        }
        ok[s] = v;
        nvalid += v;
    }
    if (nvalid == 0) return;
    const bool cross = ok[0] && ok[1] && ok[2] && ok[3];
    const bool diag = ok[4] && ok[5] && ok[6] && ok[7];
    double avg[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const int s0 = cross ? 0 : 4;
    if (cross || diag) {
        for (int s = s0; s < s0 + 4; ++s) {
            const int64_t cn = cell_index(R, i + di[s], j + dj[s], k);
#pragma unroll
            for (int q = 0; q < 5; ++q) avg[q] += Pout[q * vs + cn];
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) avg[q] *= 0.25;
    } else {
        for (int s = 0; s < 8; ++s) {
            if (!ok[s]) continue;
            const int64_t cn = cell_index(R, i + di[s], j + dj[s], k);
#pragma unroll
            for (int q = 0; q < 5; ++q) avg[q] += Pout[q * vs + cn];
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) avg[q] /= (double)nvalid;
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) Pout[q * vs + ci] = avg[q];
    R.code[ci] = 4;
}

// second step of a round for cell e: a pending cell becomes valid (code 3) after the floors;
// returns whether it was pending
__device__ __forceinline__ bool fixup_settle(const RunDev& R, double* __restrict__ Pout, int e) {
    const int n2 = R.n2, n3 = R.n3;
    const int64_t vs = R.vs;
    const int k = e % n3, t = e / n3, j = t % n2, i = t / n2;
    const int64_t ci = cell_index(R, i, j, k);
    if (R.code[ci] != 4) return false;
    R.code[ci] = 3;
    const int64_t gi = geo_index(R, i, j);
    Geo G;
    load_geo(R.gc, R.gpts, gi, G);
    double P[NPR];
#pragma unroll
    for (int q = 0; q < NPR; ++q) P[q] = Pout[q * vs + ci];
    apply_floors(R, G, R.gc[G_RHOFL * R.gpts + gi], R.gc[G_UFL * R.gpts + gi], P);
#pragma unroll
    for (int q = 0; q < NPR; ++q) Pout[q * vs + ci] = P[q];
    return true;
}

// averaging step of the first round, FIXB workgroups per run striding over its failed cells
__global__ __launch_bounds__(256) void k_fixup_first(const RunDev* __restrict__ runs, int nruns, int stage) {
    const RunDev& R = runs[blockIdx.x / FIXB];
    if (!R.var->active || R.fixup_rounds < 1) return;
    const int nf = R.var->fail_count;
    double* __restrict__ Pout = stage == 1 ? R.Ph : R.P;
    for (int x = (blockIdx.x % FIXB) * blockDim.x + threadIdx.x; x < nf; x += FIXB * blockDim.x)
        fixup_average(R, Pout, R.fail_list[x]);
}

// floors step of the first round, FIXB workgroups per run
__global__ __launch_bounds__(256) void k_fixup_settle(const RunDev* __restrict__ runs, int nruns, int stage) {
    const RunDev& R = runs[blockIdx.x / FIXB];
    if (!R.var->active || R.fixup_rounds < 1) return;
    const int nf = R.var->fail_count;
    double* __restrict__ Pout = stage == 1 ? R.Ph : R.P;
    for (int x = (blockIdx.x % FIXB) * blockDim.x + threadIdx.x; x < nf; x += FIXB * blockDim.x)
        fixup_settle(R, Pout, R.fail_list[x]);
}

__global__ __launch_bounds__(256) void k_fixup(const RunDev* __restrict__ runs, int nruns, int stage) {
    const RunDev& R = runs[blockIdx.x];
    RunVar* V = R.var;
    const bool active = V->active;
    const int nf = active ? V->fail_count : 0;
    __shared__ int left_s;
    if (nf > 0) {
        const int n2 = R.n2, n3 = R.n3;
        const int64_t vs = R.vs;
        double* __restrict__ Pout = stage == 1 ? R.Ph : R.P;
        const double* __restrict__ Pin = stage == 1 ? R.P : R.Ph;
        // the first round ran in k_fixup_first and k_fixup_settle: gather the cells still failed
        // into the slow list (finished with by now); a round's result does not depend on the order
        // of its cells, so the later rounds walk only those
        __shared__ int nleft_s;
        if (threadIdx.x == 0) nleft_s = 0;
        __syncthreads();
        for (int x = threadIdx.x; x < nf; x += blockDim.x) {
            const int e = R.fail_list[x];
            const int k = e % n3, t = e / n3, j = t % n2, i = t / n2;
            if (R.code[cell_index(R, i, j, k)] == -1) R.slow_list[atomicAdd(&nleft_s, 1)] = e;
        }
        __syncthreads();
        const int nl = nleft_s;
        if (threadIdx.x == 0) left_s = nl;
        __syncthreads();
        for (int round = 1; round < R.fixup_rounds; ++round) {
            if (left_s == 0) break;
            for (int x = threadIdx.x; x < nl; x += blockDim.x) fixup_average(R, Pout, R.slow_list[x]);
            __syncthreads();
            for (int x = threadIdx.x; x < nl; x += blockDim.x)
                if (fixup_settle(R, Pout, R.slow_list[x])) atomicSub(&left_s, 1);
            __syncthreads();
        }
        int mine = 0;
        for (int x = threadIdx.x; x < nl; x += blockDim.x) {
            const int e = R.slow_list[x];
            const int k = e % n3, t = e / n3, j = t % n2, i = t / n2;
            const int64_t ci = cell_index(R, i, j, k);
            if (R.code[ci] != -1) continue;
            // the fluid variables fall back to the stage input; the field keeps its flux-CT update
#pragma unroll
            for (int q = 0; q < 5; ++q) Pout[q * vs + ci] = Pin[q * vs + ci];
            ++mine;
        }
        if (mine) {
            atomicAdd((unsigned long long*)&V->nfail_total, (unsigned long long)mine);
            atomicAdd(&V->nfail_last, mine);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        V->fail_count = 0;
        V->slow_count = 0;
        if (stage == 2) V->active = V->steps_left > 0 ? 1 : 0;
    }
}

// ------------------------------------------------------------------------------------------
// layout conversion, inversion-only, prim->cons, diagnostics
// ------------------------------------------------------------------------------------------

__global__ void k_load(RunDev R, const double* __restrict__ in, int to_half) {
    const int64_t n = (int64_t)R.n1 * R.n2 * R.n3;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int k = (int)(e % R.n3);
    const int64_t t = e / R.n3;
    const int j = (int)(t % R.n2), i = (int)(t / R.n2);
    double* P = to_half ? R.Ph : R.P;
    const int64_t ci = cell_index(R, i, j, k);
    for (int q = 0; q < NPR; ++q) P[q * R.vs + ci] = in[q * n + e];
}

__global__ void k_store(RunDev R, double* __restrict__ out, const int8_t* __restrict__ code_in, int8_t* __restrict__ code_out) {
    const int64_t n = (int64_t)R.n1 * R.n2 * R.n3;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int k = (int)(e % R.n3);
    const int64_t t = e / R.n3;
    const int j = (int)(t % R.n2), i = (int)(t / R.n2);
    const int64_t ci = cell_index(R, i, j, k);
    if (out)
        for (int q = 0; q < NPR; ++q) out[q * n + e] = R.P[q * R.vs + ci];
    if (code_out) code_out[e] = code_in[ci];
}

__global__ void k_prim2cons(RunDev R, const double* __restrict__ Pi, double* __restrict__ Uo) {
    const int64_t n = (int64_t)R.n1 * R.n2 * R.n3;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int64_t t = e / R.n3;
    const int j = (int)(t % R.n2), i = (int)(t / R.n2);
    Geo G;
    load_geo(R.gc, R.gpts, geo_index(R, i, j), G);
    double P[NPR], U[NCS];
    for (int q = 0; q < NPR; ++q) P[q] = Pi[q * n + e];
    St s;
    prim_state(P, G, R.gam, s);
    flux_of<0>(P, s, G, s.p * pow(P[0], 1.0 - R.gam), U);
    for (int q = 0; q < NCS; ++q) Uo[q * n + e] = U[q];
}

__global__ void k_cons2prim(RunDev R, const double* __restrict__ Ui, double* __restrict__ Pio, int8_t* __restrict__ code) {
    const int64_t n = (int64_t)R.n1 * R.n2 * R.n3;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int64_t t = e / R.n3;
    const int j = (int)(t % R.n2), i = (int)(t / R.n2);
    Geo G;
    load_geo(R.gc, R.gpts, geo_index(R, i, j), G);
    double U[NCS], Pg[NPR], P[NPR];
    for (int q = 0; q < NCS; ++q) U[q] = Ui[q * n + e];
    for (int q = 0; q < NPR; ++q) Pg[q] = P[q] = Pio[q * n + e];
    const int m = invert_cell(U, Pg, G, R, P);
    if (m >= 0)
        for (int q = 0; q < NPR; ++q) Pio[q * n + e] = P[q];
    if (code) code[e] = (int8_t)m;
}

// Horizon shell sums with a fixed-order tree, one workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_diag(RunDev R, int ih, double* __restrict__ out) {
    __shared__ double sm[256], sf[256];
    const int n2 = R.n2, n3 = R.n3;
    double m = 0.0, f = 0.0;
    for (int e = threadIdx.x; e < n2 * n3; e += 256) {
        const int j = e / n3, k = e % n3;
        Geo G;
        load_geo(R.gc, R.gpts, geo_index(R, ih, j), G);
        const int64_t ci = cell_index(R, ih, j, k);
        double P[NPR];
        for (int q = 0; q < NPR; ++q) P[q] = R.P[q * R.vs + ci];
        St s;
        prim_state(P, G, R.gam, s);
        m += G.gdet * P[0] * s.u1 * R.dx[2] * R.dx[3];
        f += 0.5 * G.gdet * fabs(P[5]) * R.dx[2] * R.dx[3];
    }
    sm[threadIdx.x] = m;
    sf[threadIdx.x] = f;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sm[threadIdx.x] += sm[threadIdx.x + w];
            sf[threadIdx.x] += sf[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sm[0];
        out[1] = sf[0];
    }
}

// Accretion diagnostics (Sec. 4.2) of every radial shell: workgroup i sums over the (j, k) cells
// of radial index i, each term weighted by dX2 dX3, in a fixed order (strided partial sums, then a
// tree), out[q * n1 + i] for q = 0..5:
//   sqrt(-g) rho u^1, 1/2 sqrt(-g) |B^1|, sqrt(-g) T^1_3, -sqrt(-g) T^1_0,
//   sqrt(-g) (rho + u + p + b^2) u^1 u_3, sqrt(-g) b^1 b_3
__global__ __launch_bounds__(256) void k_diag_shells(RunDev R, double* __restrict__ out) {
    __shared__ double sm[6][256];
    const int i = blockIdx.x;
    const int n2 = R.n2, n3 = R.n3;
    const double dA = R.dx[2] * R.dx[3];
    double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int e = threadIdx.x; e < n2 * n3; e += 256) {
        const int j = e / n3, k = e % n3;
        Geo G;
        load_geo(R.gc, R.gpts, geo_index(R, i, j), G);
        const int64_t ci = cell_index(R, i, j, k);
        double P[NPR];
        for (int q = 0; q < NPR; ++q) P[q] = R.P[q * R.vs + ci];
        St st;
        prim_state(P, G, R.gam, st);
        double F[NCS];
        flux_of<1>(P, st, G, 0.0, F);  // F[1..4] = sqrt(-g) T^1_nu
        a[0] += G.gdet * P[0] * st.u1 * R.dx[2] * R.dx[3];
        a[1] += 0.5 * G.gdet * fabs(P[5]) * R.dx[2] * R.dx[3];
        a[2] += F[4] * dA;
        a[3] += -F[1] * dA;
        a[4] += G.gdet * (st.w + st.bsq) * st.u1 * st.l3 * dA;
        a[5] += G.gdet * st.b1 * st.c3 * dA;
    }
    for (int q = 0; q < 6; ++q) sm[q][threadIdx.x] = a[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 6; ++q) sm[q][threadIdx.x] += sm[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x * R.n1 + i] = sm[threadIdx.x][0];
}

// copy raw fluxes of interior faces out in [9][m1][m2][m3] order (diagnostic layout: every
// component stored, by k_flux<d, true>)
__global__ void k_flux_out(RunDev R, int d, double* __restrict__ out) {
    const int m1 = R.n1 + (d == 1), m2 = R.n2 + (d == 2), m3 = R.n3 + (d == 3);
    const int64_t n = (int64_t)m1 * m2 * m3;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int k = (int)(e % m3);
    const int64_t t = e / m3;
    const int j = (int)(t % m2), i = (int)(t / m2);
    const int64_t ci = cell_index(R, i, j, k % R.n3);
    for (int q = 0; q < NCS; ++q) {
        const int slot = d == 1 ? flux_store_slot<1, true>(q) : (d == 2 ? flux_store_slot<2, true>(q)
                                                                        : flux_store_slot<3, true>(q));
        out[q * n + e] = R.F[d][slot * R.vs + ci];
    }
}

__global__ void k_set_var(RunVar* V, double dt_req, long long steps_left, int active) {
    if (threadIdx.x == 0) {
        V->dt_req = dt_req;
        if (steps_left >= 0) V->steps_left = steps_left;
        if (active >= 0) V->active = active;
    }
}

// ------------------------------------------------------------------------------------------
// host-side launchers
// ------------------------------------------------------------------------------------------

void launch_geometry(const GeoArgs& A, hipStream_t st) {
    const int np = (A.n1 + 2 * NG) * (A.n2 + 2 * NG);
    k_geometry<<<(np + 127) / 128, 128, 0, st>>>(A);
}

void launch_bound(const RunDev* runs, const int* boff, int nruns, int nblocks, int which, int bs, int sched,
                  hipStream_t st) {
    if (nblocks > 0) k_bound<<<nblocks, bs, 0, st>>>(runs, boff, nruns, which, sched);
}

template <bool ENT, bool UNI, bool PPM>
static void flux_dir(int d, const RunDev* runs, const int* boff, int nruns, int nblocks, int which, int do_cfl,
                     int bs, int sched, hipStream_t st) {
    if (d == 1) k_flux<1, ENT, UNI, PPM><<<nblocks, bs, 0, st>>>(runs, boff, nruns, which, do_cfl, sched);
    else if (d == 2) k_flux<2, ENT, UNI, PPM><<<nblocks, bs, 0, st>>>(runs, boff, nruns, which, do_cfl, sched);
    else k_flux<3, ENT, UNI, PPM><<<nblocks, bs, 0, st>>>(runs, boff, nruns, which, do_cfl, sched);
}

void launch_flux(int d, const RunDev* runs, const int* boff, int nruns, int nblocks, int which, int do_cfl,
                 int ent, int uni, int ppm, int bs, int sched, hipStream_t st) {
    if (nblocks <= 0) return;
    if (uni && !ppm && !ent) {
        if (d == 1) k_flux_march<1><<<nblocks, bs, 0, st>>>(runs, boff, nruns, which, do_cfl, sched);
        else if (d == 2) k_flux_march<2><<<nblocks, bs, 0, st>>>(runs, boff, nruns, which, do_cfl, sched);
        else k_flux3_lanes<false><<<nblocks, bs, 0, st>>>(runs, boff, nruns, which, do_cfl, sched);
    } else if (uni && ppm && !ent) {
        if (d == 1) k_flux_ppm_pair<1><<<nblocks, bs, 0, st>>>(runs, boff, nruns, which, do_cfl, sched);
        else if (d == 2) k_flux_ppm_pair<2><<<nblocks, bs, 0, st>>>(runs, boff, nruns, which, do_cfl, sched);
        else k_flux3_lanes<true><<<nblocks, bs, 0, st>>>(runs, boff, nruns, which, do_cfl, sched);
    } else if (ent) {
        if (ppm) flux_dir<true, false, true>(d, runs, boff, nruns, nblocks, which, do_cfl, bs, sched, st);
        else flux_dir<true, false, false>(d, runs, boff, nruns, nblocks, which, do_cfl, bs, sched, st);
    } else if (uni) {
        if (ppm) flux_dir<false, true, true>(d, runs, boff, nruns, nblocks, which, do_cfl, bs, sched, st);
        else flux_dir<false, true, false>(d, runs, boff, nruns, nblocks, which, do_cfl, bs, sched, st);
    } else {
        if (ppm) flux_dir<false, false, true>(d, runs, boff, nruns, nblocks, which, do_cfl, bs, sched, st);
        else flux_dir<false, false, false>(d, runs, boff, nruns, nblocks, which, do_cfl, bs, sched, st);
    }
}

void launch_emf(const RunDev* runs, const int* boff, int nruns, int nblocks, int bs, int sched, hipStream_t st) {
    if (nblocks > 0) k_emf<<<nblocks, bs, 0, st>>>(runs, boff, nruns, sched);
}

void launch_dt(const RunDev* runs, int nruns, hipStream_t st) {
    k_dt<<<(nruns + 63) / 64, 64, 0, st>>>(runs, nruns);
}

void launch_update(const RunDev* runs, const int* boff, int nruns, int nblocks, int stage, int uni, int bs,
                   int sched, hipStream_t st) {
    if (nblocks <= 0) return;
    if (uni) {
        if (stage == 1) k_update<1, true><<<nblocks, bs, 0, st>>>(runs, boff, nruns, sched);
        else k_update<2, true><<<nblocks, bs, 0, st>>>(runs, boff, nruns, sched);
    } else {
        if (stage == 1) k_update<1, false><<<nblocks, bs, 0, st>>>(runs, boff, nruns, sched);
        else k_update<2, false><<<nblocks, bs, 0, st>>>(runs, boff, nruns, sched);
    }
}

void launch_update_slow(const RunDev* runs, int nruns, int stage, hipStream_t st) {
    k_update_slow<<<nruns * SLOWB, 256, 0, st>>>(runs, nruns, stage);
}

void launch_fixup(const RunDev* runs, int nruns, int stage, hipStream_t st) {
    k_fixup_first<<<nruns * FIXB, 256, 0, st>>>(runs, nruns, stage);
    k_fixup_settle<<<nruns * FIXB, 256, 0, st>>>(runs, nruns, stage);
    k_fixup<<<nruns, 256, 0, st>>>(runs, nruns, stage);
}

static inline unsigned nb(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_load(const RunDev& R, const double* in, int to_half, hipStream_t st) {
    k_load<<<nb((int64_t)R.n1 * R.n2 * R.n3, 256), 256, 0, st>>>(R, in, to_half);
}
void launch_store(const RunDev& R, double* out, const int8_t* code_in, int8_t* code_out, hipStream_t st) {
    k_store<<<nb((int64_t)R.n1 * R.n2 * R.n3, 256), 256, 0, st>>>(R, out, code_in, code_out);
}
void launch_prim2cons(const RunDev& R, const double* P, double* U, hipStream_t st) {
    k_prim2cons<<<nb((int64_t)R.n1 * R.n2 * R.n3, 256), 256, 0, st>>>(R, P, U);
}
void launch_cons2prim(const RunDev& R, const double* U, double* P, int8_t* code, hipStream_t st) {
    k_cons2prim<<<nb((int64_t)R.n1 * R.n2 * R.n3, 256), 256, 0, st>>>(R, U, P, code);
}
void launch_diag(const RunDev& R, int ih, double* out, hipStream_t st) {
    k_diag<<<1, 256, 0, st>>>(R, ih, out);
}
void launch_diag_shells(const RunDev& R, double* out, hipStream_t st) {
    k_diag_shells<<<R.n1, 256, 0, st>>>(R, out);
}
void launch_flux_out(const RunDev& R, int d, double* out, hipStream_t st) {
    const int64_t n = (int64_t)(R.n1 + (d == 1)) * (R.n2 + (d == 2)) * (R.n3 + (d == 3));
    k_flux_out<<<nb(n, 256), 256, 0, st>>>(R, d, out);
}
void launch_set_var(RunVar* V, double dt_req, long long steps_left, int active, hipStream_t st) {
    k_set_var<<<1, 64, 0, st>>>(V, dt_req, steps_left, active);
}

}  // namespace grmhd
