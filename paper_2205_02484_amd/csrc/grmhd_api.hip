// grmhd_api.hip -- the C ABI (include/grmhd.h): run contexts, the ensemble engine, memory
// footprints and the per-step launch chain (optionally replayed from a captured HIP graph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "grmhd.h"
#include "grmhd_kernels.h"

using namespace grmhd;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(x)                                                                         \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess) return fail(GRMHD_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

// block tables: ghosts; fluxes per direction and update, each once over the row-path runs (a wave
// is one phi row, its cells share (r, theta): scalar metric loads) and once over the other runs; the flux
// tables also split PLM runs (KB_F*) from PPM runs (KB_P*), which have kernels of their own
enum {
    KB_BOUND = 0,
    KB_F1, KB_F2, KB_F3, KB_F1N, KB_F2N, KB_F3N,
    KB_P1, KB_P2, KB_P3, KB_P1N, KB_P2N, KB_P3N,
    KB_UPD, KB_UPDN, KB_EMF, NK
};
// flux table of direction d for runs with (uni, ppm)
constexpr int flux_kind(int d, bool uni, bool ppm) { return KB_F1 + (d - 1) + (uni ? 0 : 3) + (ppm ? 6 : 0); }

// Launch shape of one stage-kernel kind: threads per workgroup, block order (bit 0 set:
// XCD-contiguous) and, for the marching X1/X2 face kernels, faces per wave segment.  The
// autotuner picks one per kind.
struct Shape {
    int bs = 256;
    int sched = 1;
    int seg = 16;
};
const Shape kCandidates[] = {{256, 1, 16}, {128, 1, 16}, {64, 1, 16}, {256, 0, 16}, {128, 0, 16},
                             {128, 1, 8}, {256, 1, 32}, {128, 1, 64}};
constexpr int kNumCandidates = sizeof(kCandidates) / sizeof(kCandidates[0]);
// kernel kinds reported by grmhd_kernel_times
enum { TK_BOUND = 0, TK_FLUX1, TK_FLUX2, TK_FLUX3, TK_DT, TK_UPDATE, TK_FIXUP, TK_SLOW, TK_EMF, NTK };

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

struct Layout {
    int64_t vs, s1, s2, gpts;
    int64_t off_P, off_Ph, off_F[4], off_gc, off_gf1, off_gf2, off_code, off_fail, off_slow, off_var, total;
};

Layout make_layout(const grmhd_grid& g) {
    Layout L{};
    const int act3 = g.n3 > 1;
    L.s2 = g.n3;
    L.s1 = (int64_t)(g.n2 + 2 * NG) * g.n3;
    L.vs = (int64_t)(g.n1 + 2 * NG) * L.s1;
    L.gpts = (int64_t)(g.n1 + 2 * NG) * (g.n2 + 2 * NG);
    int64_t o = 0;
    auto take = [&](int64_t bytes) { int64_t at = o; o += align256(bytes); return at; };
    L.off_P = take(NPR * L.vs * 8);
    L.off_Ph = take(NPR * L.vs * 8);
    L.off_F[0] = -1;
    for (int d = 1; d <= 3; ++d) {
        const int act = d == 1 ? g.n1 > 1 : (d == 2 ? g.n2 > 1 : act3);
        L.off_F[d] = act ? take(NCS * L.vs * 8) : -1;
    }
    L.off_gc = take(NGC * L.gpts * 8);
    L.off_gf1 = take(NGF * L.gpts * 8);
    L.off_gf2 = take(NGF * L.gpts * 8);
    L.off_code = take(L.vs);
    L.off_fail = take((int64_t)g.n1 * g.n2 * g.n3 * 4);
    L.off_slow = take((int64_t)g.n1 * g.n2 * g.n3 * 4);
    L.off_var = take(sizeof(RunVar));
    L.total = o;
    return L;
}

// MKS radial map on the host: r(X1) = exp(X1) below ln r_br, exp(X1 + (X1 - ln r_br)^n_x) beyond.
double host_r_of_x1(const grmhd_grid* g, double X1) {
    if (!(g->r_br > 0.0) || X1 < std::log(g->r_br)) return std::exp(X1);
    const double u = X1 - std::log(g->r_br);
    double p = 1.0;
    for (int k = 0; k < g->n_x; ++k) p *= u;
    return std::exp(X1 + p);
}

// X1 of the outer grid edge, r(X1) = r_out: bisection on [ln r_br, ln r_out] (r increases with X1
// and r(ln r_out) >= r_out) when the map is hyper-exponential there.
double host_x1_out(const grmhd_grid* g) {
    double hi = std::log(g->r_out);
    if (!(g->r_br > 0.0) || g->r_out <= g->r_br) return hi;
    double lo = std::log(g->r_br);
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (host_r_of_x1(g, mid) < g->r_out) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// Multiplier and shift of FastDiv for a divisor 1 <= d < 2^31 (see grmhd_dev.h).
FastDiv make_fastdiv(int32_t d) {
    uint32_t l = 0;
    while ((1ull << l) < (uint64_t)d) ++l;
    FastDiv f;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - (uint64_t)d)) / (uint64_t)d + 1);
    f.l = l;
    return f;
}

int validate(const grmhd_grid* g, const grmhd_params* p) {
    if (!g || !p) return fail(GRMHD_EINVAL, "grid and params are required");
    if (g->n1 < 1 || g->n2 < 1 || g->n3 < 1) return fail(GRMHD_EINVAL, "grid sizes must be >= 1");
    if ((int64_t)g->n1 * g->n2 * g->n3 >= (1ll << 31)) return fail(GRMHD_EINVAL, "grid too large (>= 2^31 cells)");
    // every per-variable array is addressed with 32-bit byte offsets: (n1+6)(n2+6) n3 cells < 2^29
    if ((int64_t)(g->n1 + 2 * NG) * (g->n2 + 2 * NG) * g->n3 >= (1ll << 29))
        return fail(GRMHD_EINVAL, "grid too large for one run (more than 2^29 cells with ghosts)");
    if (g->coords != GRMHD_MKS && g->coords != GRMHD_MINKOWSKI_CART) return fail(GRMHD_EINVAL, "unknown coords");
    if (g->coords == GRMHD_MKS) {
        if (g->n1 < 2 || g->n2 < 2) return fail(GRMHD_EINVAL, "MKS grids need n1, n2 >= 2");
        if (!(g->r_in > 0.0) || !(g->r_out > g->r_in)) return fail(GRMHD_EINVAL, "need 0 < r_in < r_out");
        if (!(g->h > 0.0) || !(g->h <= 2.0)) return fail(GRMHD_EINVAL, "MKS h must be in (0, 2]");
        if (!(std::fabs(p->spin) < 1.0)) return fail(GRMHD_EINVAL, "|spin| must be < 1");
        if (g->r_br > 0.0 && (!(g->r_br > g->r_in) || g->n_x < 2 || g->n_x > 16))
            return fail(GRMHD_EINVAL, "hyper-exponential map needs r_br > r_in and 2 <= n_x <= 16");
        if (g->pole_fix < 0 || 2 * (int64_t)g->pole_fix >= g->n2)
            return fail(GRMHD_EINVAL, "pole_fix needs 0 <= pole_fix and 2 pole_fix < n2");
    } else {
        if (g->pole_fix != 0) return fail(GRMHD_EINVAL, "pole_fix applies to MKS grids only");
        for (int d = 0; d < 3; ++d)
            if (!(g->xmax[d] > g->xmin[d])) return fail(GRMHD_EINVAL, "need xmin < xmax");
    }
    if (!(p->gam > 1.0)) return fail(GRMHD_EINVAL, "gamma must be > 1");
    if (!(p->cfl > 0.0)) return fail(GRMHD_EINVAL, "cfl must be > 0");
    if (p->riemann != GRMHD_LLF && p->riemann != GRMHD_HLL) return fail(GRMHD_EINVAL, "unknown riemann solver");
    if (p->recon != GRMHD_PLM && p->recon != GRMHD_PPM) return fail(GRMHD_EINVAL, "unknown reconstruction");
    // PPM reads three cells out: periodic wraps and polar reflections need that many active cells
    if (p->recon == GRMHD_PPM && ((g->n1 > 1 && g->n1 < 3) || (g->n2 > 1 && g->n2 < 3) || (g->n3 > 1 && g->n3 < 3)))
        return fail(GRMHD_EINVAL, "PPM needs at least 3 cells along every direction with more than one");
    if (!(p->bsq_rho_max > 0.0) || !(p->bsq_u_max > 0.0) || !(p->gamma_max >= 1.0))
        return fail(GRMHD_EINVAL, "ceilings must be positive, gamma_max >= 1");
    if (!(p->c2p_tol > 0.0) || p->c2p_maxit < 0 || p->fixup_max_rounds < 0) return fail(GRMHD_EINVAL, "bad inversion controls");
    return GRMHD_OK;
}

bool host_finite(const double* a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

__global__ void k_count_nonfinite(const double* a, int64_t n, int* flag) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n && !isfinite(a[e])) atomicOr(flag, 1);
}

int device_finite(const double* a, int64_t n, hipStream_t st, bool* ok) {
    int* d = nullptr;
    HIPCHK(hipMalloc(&d, sizeof(int)));
    hipError_t e1 = hipMemsetAsync(d, 0, sizeof(int), st);
    if (e1 == hipSuccess) {
        k_count_nonfinite<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(a, n, d);
        e1 = hipGetLastError();
    }
    int h = 0;
    if (e1 == hipSuccess) e1 = hipMemcpyAsync(&h, d, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e1 == hipSuccess) e1 = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e1 != hipSuccess) return fail(GRMHD_EDEVICE, "finite check: %s", hipGetErrorString(e1));
    *ok = h == 0;
    return GRMHD_OK;
}

// One resident run (a context or an ensemble job).
struct Run {
    grmhd_grid grid{};
    grmhd_params par{};
    Layout L{};
    char* mem = nullptr;
    RunDev h{};        // host copy of the device descriptor
    int ih = -1;       // horizon shell index
    int64_t id = 0;
    int64_t nsteps_req = 0;
    bool reported = false;
};

void free_run(Run* r) {
    if (!r) return;
    if (r->mem) (void)hipFree(r->mem);
    delete r;
}

int create_run(const grmhd_grid* g, const grmhd_params* p, const double* prims, int on_device, hipStream_t st,
               Run** out) {
    int rc = validate(g, p);
    if (rc) return rc;
    if (!prims) return fail(GRMHD_EINVAL, "prims is NULL");
    const int64_t ncell = (int64_t)g->n1 * g->n2 * g->n3;
    if (!on_device && !host_finite(prims, NPR * ncell)) return fail(GRMHD_EINVAL, "prims hold NaN/Inf");
    if (on_device) {
        bool ok = false;
        rc = device_finite(prims, NPR * ncell, st, &ok);
        if (rc) return rc;
        if (!ok) return fail(GRMHD_EINVAL, "prims hold NaN/Inf");
    }
    Run* r = new Run();
    r->grid = *g;
    r->par = *p;
    r->L = make_layout(*g);
    hipError_t e = hipMalloc(&r->mem, r->L.total);
    if (e != hipSuccess) {
        delete r;
        (void)hipGetLastError();
        return fail(GRMHD_ENOMEM, "device allocation of %lld bytes failed", (long long)r->L.total);
    }
    const Layout& L = r->L;
    RunDev& R = r->h;
    R.n1 = g->n1; R.n2 = g->n2; R.n3 = g->n3;
    R.act1 = g->n1 > 1; R.act2 = g->n2 > 1; R.act3 = g->n3 > 1;
    R.mks = g->coords == GRMHD_MKS;
    R.riemann = p->riemann;
    R.ppm = p->recon == GRMHD_PPM;
    R.pole_fix = R.mks ? g->pole_fix : 0;
    R.c2p_maxit = p->c2p_maxit;
    R.fixup_rounds = p->fixup_max_rounds;
    R.s1 = L.s1; R.s2 = L.s2; R.vs = L.vs;
    R.gs1 = g->n2 + 2 * NG;
    R.gpts = L.gpts;
    double x1lo = 0.0;
    R.dx[0] = 0.0;
    if (R.mks) {
        x1lo = std::log(g->r_in);
        R.dx[1] = (host_x1_out(g) - x1lo) / g->n1;
        R.dx[2] = 1.0 / g->n2;
        R.dx[3] = 2.0 * M_PI / g->n3;
    } else {
        for (int d = 1; d <= 3; ++d) {
            const int n = d == 1 ? g->n1 : (d == 2 ? g->n2 : g->n3);
            R.dx[d] = (g->xmax[d - 1] - g->xmin[d - 1]) / n;
        }
    }
    for (int d = 0; d < 4; ++d) R.idx[d] = d ? 1.0 / R.dx[d] : 0.0;
    R.gam = p->gam;
    R.cfl = p->cfl;
    R.gg = (p->gam - 1.0) / p->gam;
    R.igam1 = 1.0 / (p->gam - 1.0);
    R.bsq_rho_max = p->bsq_rho_max;
    R.bsq_u_max = p->bsq_u_max;
    R.gamma_max = p->gamma_max;
    R.beta_ent = p->beta_entropy;
    R.c2p_tol = p->c2p_tol;
    R.P = (double*)(r->mem + L.off_P);
    R.Ph = (double*)(r->mem + L.off_Ph);
    R.F[0] = nullptr;
    for (int d = 1; d <= 3; ++d) R.F[d] = L.off_F[d] >= 0 ? (double*)(r->mem + L.off_F[d]) : nullptr;
    R.gc = (const double*)(r->mem + L.off_gc);
    R.gf[0] = nullptr;
    R.gf[1] = (const double*)(r->mem + L.off_gf1);
    R.gf[2] = (const double*)(r->mem + L.off_gf2);
    R.code = (int8_t*)(r->mem + L.off_code);
    R.fail_list = (int32_t*)(r->mem + L.off_fail);
    R.slow_list = (int32_t*)(r->mem + L.off_slow);
    // the row path (waves of 64 lanes along one phi row, the metric by scalar loads) can serve the
    // run when at most a third of the lanes repeat a cell of the row: every n3 that is a multiple
    // of 64, and other n3 >= 48 close enough above one; the engine decides (Engine::rebuild)
    R.nkc = (g->n3 + 63) / 64;
    R.row_ok = g->n3 >= 48 && 3 * (R.nkc * 64 - g->n3) <= R.nkc * 64;
    R.geo_uniform = R.row_ok && g->n3 % 64 == 0;
    R.var = (RunVar*)(r->mem + L.off_var);
    R.fd_n2 = make_fastdiv(g->n2);
    R.fd_n3 = make_fastdiv(g->n3);
    R.fd_kc = make_fastdiv(R.row_ok ? R.nkc : 1);
    R.fd_row[0] = make_fastdiv(1);
    R.fd_row[1] = make_fastdiv(g->n1 + 1);
    R.fd_row[2] = make_fastdiv(g->n2 + 1);
    R.fd_row[3] = make_fastdiv(g->n2 + 2 * R.act2);
    for (int l = 0; l < 3; ++l) R.fd_jg[l] = make_fastdiv((g->n2 + (1 << l) - 1) >> l);

    auto bail = [&](int code) { free_run(r); return code; };
    if (hipMemsetAsync(r->mem, 0, L.total, st) != hipSuccess) return bail(fail(GRMHD_EDEVICE, "memset failed"));
    GeoArgs A{};
    A.n1 = g->n1; A.n2 = g->n2; A.mks = R.mks;
    A.x1lo = x1lo; A.dx1 = R.dx[1]; A.dx2 = R.dx[2];
    A.xb = g->r_br > 0.0 ? std::log(g->r_br) : INFINITY;
    A.nx = g->n_x;
    A.spin = p->spin; A.h = g->h;
    A.rho_fl_coef = p->rho_fl_coef; A.rho_fl_pow = p->rho_fl_pow;
    A.u_fl_coef = p->u_fl_coef; A.u_fl_pow = p->u_fl_pow; A.fl_abs = p->fl_abs;
    A.gc = (double*)R.gc; A.gf1 = (double*)R.gf[1]; A.gf2 = (double*)R.gf[2];
    launch_geometry(A, st);
    const double* src = prims;
    double* tmp = nullptr;
    if (!on_device) {
        if (hipMalloc(&tmp, NPR * ncell * 8) != hipSuccess) {
            (void)hipGetLastError();
            return bail(fail(GRMHD_ENOMEM, "staging allocation failed"));
        }
        if (hipMemcpyAsync(tmp, prims, NPR * ncell * 8, hipMemcpyHostToDevice, st) != hipSuccess) {
            (void)hipFree(tmp);
            return bail(fail(GRMHD_EDEVICE, "H2D copy failed"));
        }
        src = tmp;
    }
    launch_load(R, src, 0, st);
    RunVar v{};
    v.dt_req = -1.0;
    v.steps_left = (1ll << 60);
    v.active = 1;
    hipError_t e2 = hipMemcpyAsync(R.var, &v, sizeof(v), hipMemcpyHostToDevice, st);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(st);
    if (tmp) (void)hipFree(tmp);
    if (e2 != hipSuccess) return bail(fail(GRMHD_EDEVICE, "init: %s", hipGetErrorString(e2)));
    if (hipGetLastError() != hipSuccess) return bail(fail(GRMHD_EDEVICE, "init kernels failed"));
    // horizon shell: first radial cell centre with r >= 1 + sqrt(1 - a^2)
    if (R.mks) {
        const double rh = 1.0 + std::sqrt(1.0 - p->spin * p->spin);
        for (int i = 0; i < g->n1; ++i)
            if (host_r_of_x1(g, x1lo + (i + 0.5) * R.dx[1]) >= rh) { r->ih = i; break; }
    }
    *out = r;
    return GRMHD_OK;
}

int read_var(const Run* r, hipStream_t st, RunVar* v) {
    HIPCHK(hipMemcpyAsync(v, r->h.var, sizeof(RunVar), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return GRMHD_OK;
}

// Stage-chain engine over a set of runs (one context = one run).
struct Engine {
    hipStream_t st = nullptr;
    bool own_stream = false;
    std::vector<Run*> runs;
    RunDev* d_runs = nullptr;
    int* d_boff = nullptr;
    int cap = 0;
    int nblk[NK] = {0};
    bool dirty = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool use_graph = true;
    // optional per-kernel event timing (plain launches, events around every kernel)
    bool timing = false;
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_kind;
    double t_ms[NTK] = {0};
    long long t_n[NTK] = {0};
    Shape shape[NK];
    // The row-path X2 and X3 face kernels run on side streams 0 and 1, and every general-path
    // kernel (the face kernels and the update of the runs off the row path, small ones in a mixed
    // batch) on side stream 2, forked from and joined back into the run's stream (parallel
    // branches of the captured graph); default priority like the main one.  Made on first need:
    // only when the runs hold >= 2^20 cells (the overlap pays on big grids; a lone small run would
    // pay the streams' creation and gain nothing).
    static constexpr int NSIDE = 3;
    hipStream_t side[NSIDE] = {nullptr, nullptr, nullptr};
    hipEvent_t fork_ev = nullptr, join_ev[NSIDE] = {nullptr, nullptr, nullptr};
    hipEvent_t fork2_ev = nullptr, join2_ev = nullptr;
    bool fork_on = false;
    int64_t cells = 0;

    ~Engine() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        drop_graph();
        for (int x = 0; x < NSIDE; ++x) {
            if (join_ev[x]) (void)hipEventDestroy(join_ev[x]);
            if (side[x]) (void)hipStreamDestroy(side[x]);
        }
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        if (fork2_ev) (void)hipEventDestroy(fork2_ev);
        if (join2_ev) (void)hipEventDestroy(join2_ev);
        if (d_runs) (void)hipFree(d_runs);
        if (d_boff) (void)hipFree(d_boff);
        if (own_stream && st) (void)hipStreamDestroy(st);
    }
    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
    }
    int init(void* stream) {
        if (stream) {
            st = (hipStream_t)stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            own_stream = true;
        }
        const char* ng = std::getenv("GRMHD_NO_GRAPH");
        use_graph = !(ng && ng[0] == '1');
        return GRMHD_OK;
    }
    int make_side_streams() {
        if (side[0]) return GRMHD_OK;
        HIPCHK(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&fork2_ev, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&join2_ev, hipEventDisableTiming));
        for (int x = 0; x < NSIDE; ++x) {
            HIPCHK(hipStreamCreateWithFlags(&side[x], hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&join_ev[x], hipEventDisableTiming));
        }
        return GRMHD_OK;
    }
    static int64_t elems(const RunDev& R, int kind, int bs, int seg) {
        const int64_t n1 = R.n1, n2 = R.n2, n3 = R.n3;
        switch (kind) {
            case KB_BOUND: {
                const int64_t gd = 2 + R.ppm;  // ghost layers the run fills
                return (2 * gd * (n2 + 2 * gd) + 2 * gd * n1 + 2 * (int64_t)R.pole_fix * n1) * n3;
            }
            case KB_F1: case KB_F2: case KB_F3: case KB_F1N: case KB_F2N: case KB_F3N:
            case KB_P1: case KB_P2: case KB_P3: case KB_P1N: case KB_P2N: case KB_P3N: {
                const int x = kind - KB_F1, d = x % 3 + 1;
                const bool uni = (x / 3) % 2 == 0, ppm = x >= 6;
                if (uni != (bool)R.geo_uniform || ppm != (bool)R.ppm) return 0;
                const int64_t kl = uni ? (int64_t)R.nkc * 64 : n3;   // lanes per row
                // marching X1/X2 kernels: one wave per segment of seg faces, 64 k and a row
                if (uni && !ppm && (d == 1 || d == 2)) {
                    if (!(d == 1 ? R.act1 : R.act2)) return 0;
                    RunDev Rs = R;
                    Rs.mseg[d - 1] = seg;
                    return march_waves(Rs, d) * 64;
                }
                // PPM X1/X2 faces on the row path: one thread per pair of faces along d
                if (uni && ppm && (d == 1 || d == 2)) {
                    if (!(d == 1 ? R.act1 : R.act2)) return 0;
                    const int64_t npair = ((d == 1 ? n1 : n2) + 2) / 2;
                    return npair * (d == 1 ? n2 + 2 * R.act2 : n1 + 2 * R.act1) * kl;
                }
                if (d == 1) return R.act1 ? (n1 + 1) * (n2 + 2 * R.act2) * kl : 0;
                if (d == 2) return R.act2 ? (n1 + 2 * R.act1) * (n2 + 1) * kl : 0;
                return R.act3 ? (n1 + 2 * R.act1) * (n2 + 2 * R.act2) * kl : 0;
            }
            // uniform-metric update: workgroups of bs/64 waves on consecutive j (n2 padded to a
            // multiple of that)
            case KB_UPD: return R.geo_uniform ? n1 * ((n2 + bs / 64 - 1) / (bs / 64) * (bs / 64)) * R.nkc * 64 : 0;
            // edge EMFs: runs with at least two active directions
            case KB_EMF: return (R.act1 + R.act2 + R.act3 >= 2) ? (n1 + 1) * (n2 + 1) * n3 : 0;
            default: return R.geo_uniform ? 0 : n1 * n2 * n3;
        }
    }
    // Row path and march segments for the current set of runs.  A run whose n3 is not a multiple
    // of 64 leaves some lanes of its rows repeating cells: worth it when the runs together fill the
    // chip (>= 2^20 cells), not for a lone small run, which the one-face kernels spread over more
    // waves.  Such a PLM run gets the same bits from the row path's marching and lane-shift face
    // kernels as from the one-face kernels it takes alone; a PPM run would take the scalar-metric
    // one-face kernels, whose last bits differ from the per-lane-metric ones in a few cells, so a
    // ragged-n3 PPM run stays on the general path in any company.  The marches keep the launch
    // shape's segment unless the runs together would then get fewer than ~4096 waves (about four
    // per SIMD).
    int mseg_eff[2] = {16, 16};
    void plan_row_path() {
        cells = 0;
        for (Run* r : runs) cells += (int64_t)r->h.n1 * r->h.n2 * r->h.n3;
        for (Run* r : runs) {
            RunDev& R = r->h;
            R.geo_uniform = R.row_ok && (R.n3 % 64 == 0 || (cells >= (int64_t(1) << 20) && !R.ppm));
        }
        for (int d = 1; d <= 2; ++d) {
            const int kind = d == 1 ? KB_F1 : KB_F2;
            int64_t units = 0;
            for (Run* r : runs)
                if (r->h.geo_uniform && !r->h.ppm) units += march_units(r->h, d);
            const int64_t cap = units / 4096;
            const int seg = shape[kind].seg;
            mseg_eff[d - 1] = (int)(seg < cap ? seg : (cap > 1 ? cap : 1));
        }
        for (Run* r : runs) {
            r->h.mseg[0] = mseg_eff[0];
            r->h.mseg[1] = mseg_eff[1];
        }
    }
    int rebuild() {
        drop_graph();
        plan_row_path();
        fork_on = cells >= (int64_t(1) << 20);
        if (fork_on) {
            const int rc = make_side_streams();
            if (rc) return rc;
        }
        const int n = (int)runs.size();
        if (n > cap) {
            if (d_runs) (void)hipFree(d_runs);
            if (d_boff) (void)hipFree(d_boff);
            d_runs = nullptr;
            d_boff = nullptr;
            cap = std::max(n, 8);
            HIPCHK(hipMalloc(&d_runs, sizeof(RunDev) * cap));
            HIPCHK(hipMalloc(&d_boff, sizeof(int) * NK * (cap + 1)));
        }
        std::vector<RunDev> hr(n);
        std::vector<int> boff(NK * (cap + 1), 0);
        for (int kind = 0; kind < NK; ++kind) {
            int acc = 0;
            for (int r = 0; r < n; ++r) {
                boff[kind * (cap + 1) + r] = acc;
                const int64_t ne = elems(runs[r]->h, kind, shape[kind].bs,
                                         kind == KB_F1 ? mseg_eff[0] : (kind == KB_F2 ? mseg_eff[1] : shape[kind].seg));
                acc += (int)((ne + shape[kind].bs - 1) / shape[kind].bs);
            }
            boff[kind * (cap + 1) + n] = acc;
            nblk[kind] = acc;
        }
        for (int r = 0; r < n; ++r) hr[r] = runs[r]->h;
        if (n) HIPCHK(hipMemcpyAsync(d_runs, hr.data(), sizeof(RunDev) * n, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(d_boff, boff.data(), sizeof(int) * NK * (cap + 1), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        dirty = false;
        return GRMHD_OK;
    }
    const int* boff(int kind) const { return d_boff + kind * (cap + 1); }
    // record an event pair around the launch when timing
    int mark(int kind) {
        if (!timing) return GRMHD_OK;
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        HIPCHK(hipEventRecord(e, st));
        ev.push_back(e);
        ev_kind.push_back(kind);
        return GRMHD_OK;
    }
    int harvest() {
        if (ev.empty()) return GRMHD_OK;
        HIPCHK(hipEventSynchronize(ev.back()));
        for (size_t x = 0; x + 1 < ev.size(); x += 2) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ev[x], ev[x + 1]));
            t_ms[ev_kind[x]] += ms;
            t_n[ev_kind[x]] += 1;
        }
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        ev.clear();
        ev_kind.clear();
        return GRMHD_OK;
    }
    int enqueue_step() {
        const int n = (int)runs.size();
        if (!n) return GRMHD_OK;
        for (int stage = 1; stage <= 2; ++stage) {
            const int which = stage - 1;
            mark(TK_BOUND);
            launch_bound(d_runs, boff(KB_BOUND), n, nblk[KB_BOUND], which, shape[KB_BOUND].bs,
                         shape[KB_BOUND].sched, st);
            mark(TK_BOUND);
            // face kernels: one direction after another while timing each kernel, otherwise X1 on
            // the run's stream and X2, X3 on the side streams (independent: each reads the stage
            // input and writes its own face array and CFL slot)
            const bool fork = fork_on && !timing;
            if (fork) {
                HIPCHK(hipEventRecord(fork_ev, st));
                for (int x = 0; x < NSIDE; ++x) HIPCHK(hipStreamWaitEvent(side[x], fork_ev, 0));
            }
            for (int d = 1; d <= 3; ++d) {
                int any = 0;
                for (int v = 0; v < 4; ++v) any += nblk[flux_kind(d, v & 1, v >> 1)] > 0;
                if (!any) continue;
                mark(TK_FLUX1 + d - 1);
                for (int v = 0; v < 4; ++v) {
                    const bool uni = v & 1, ppm = v >> 1;
                    const int k = flux_kind(d, uni, ppm);
                    const hipStream_t sd = !fork ? st : (!uni ? side[2] : (d > 1 ? side[d - 2] : st));
                    launch_flux(d, d_runs, boff(k), n, nblk[k], which, stage == 1, 0, uni, ppm, shape[k].bs,
                                shape[k].sched, sd);
                }
                mark(TK_FLUX1 + d - 1);
            }
            if (fork) {
                for (int x = 0; x < NSIDE; ++x) {
                    HIPCHK(hipEventRecord(join_ev[x], side[x]));
                    HIPCHK(hipStreamWaitEvent(st, join_ev[x], 0));
                }
            }
            if (stage == 1) {
                mark(TK_DT);
                launch_dt(d_runs, n, st);
                mark(TK_DT);
            }
            mark(TK_EMF);
            launch_emf(d_runs, boff(KB_EMF), n, nblk[KB_EMF], shape[KB_EMF].bs, shape[KB_EMF].sched, st);
            mark(TK_EMF);
            mark(TK_UPDATE);
            // the row-path and the other runs' updates touch different runs: two branches
            const bool fork2 = fork && nblk[KB_UPD] > 0 && nblk[KB_UPDN] > 0;
            if (fork2) {
                HIPCHK(hipEventRecord(fork2_ev, st));
                HIPCHK(hipStreamWaitEvent(side[2], fork2_ev, 0));
            }
            launch_update(d_runs, boff(KB_UPD), n, nblk[KB_UPD], stage, 1, shape[KB_UPD].bs, shape[KB_UPD].sched, st);
            launch_update(d_runs, boff(KB_UPDN), n, nblk[KB_UPDN], stage, 0, shape[KB_UPDN].bs, shape[KB_UPDN].sched,
                          fork2 ? side[2] : st);
            if (fork2) {
                HIPCHK(hipEventRecord(join2_ev, side[2]));
                HIPCHK(hipStreamWaitEvent(st, join2_ev, 0));
            }
            mark(TK_UPDATE);
            mark(TK_SLOW);
            launch_update_slow(d_runs, n, stage, st);
            mark(TK_SLOW);
            mark(TK_FIXUP);
            launch_fixup(d_runs, n, stage, st);
            mark(TK_FIXUP);
        }
        HIPCHK(hipGetLastError());
        return GRMHD_OK;
    }
    // Online autotuning: every candidate shape runs `reps` ordinary steps with per-kernel events;
    // each kernel kind then keeps the shape with the smallest average duration.  A cell's
    // arithmetic does not depend on the launch shape, so these are regular steps of the runs.
    int autotune(int reps, std::string* report) {
        if (runs.empty() || reps <= 0) return GRMHD_OK;
        int tk_of[NK];
        for (int k = 0; k < NK; ++k)
            tk_of[k] = k == KB_BOUND ? TK_BOUND
                       : (k == KB_EMF ? TK_EMF : (k >= KB_UPD ? TK_UPDATE : TK_FLUX1 + (k - KB_F1) % 3));
        double best_ms[NK];
        int best[NK];
        for (int k = 0; k < NK; ++k) { best_ms[k] = 1e300; best[k] = 0; }
        const bool was_timing = timing;
        char line[256];
        std::string detail;
        for (int c = 0; c < kNumCandidates; ++c) {
            for (int k = 0; k < NK; ++k) shape[k] = kCandidates[c];
            dirty = true;
            int rc = harvest();
            if (rc) return rc;
            for (int k = 0; k < NTK; ++k) { t_ms[k] = 0.0; t_n[k] = 0; }
            timing = true;
            rc = steps(reps);
            if (rc == GRMHD_OK) rc = harvest();
            timing = was_timing;
            if (rc) return rc;
            for (int k = 0; k < NK; ++k) {
                const int tk = tk_of[k];
                if (!t_n[tk]) continue;
                const double ms = t_ms[tk] / (double)t_n[tk];
                snprintf(line, sizeof(line), "kind %d bs %d sched %d seg %d: %.4f ms\n", k, kCandidates[c].bs,
                         kCandidates[c].sched, kCandidates[c].seg, ms);
                detail += line;
                if (ms < best_ms[k]) { best_ms[k] = ms; best[k] = c; }
            }
        }
        for (int k = 0; k < NK; ++k) shape[k] = kCandidates[best[k]];
        for (int k = 0; k < NTK; ++k) { t_ms[k] = 0.0; t_n[k] = 0; }
        dirty = true;
        if (report) {
            // the choice first, so that a short caller buffer still holds it
            for (int k = 0; k < NK; ++k) {
                snprintf(line, sizeof(line), "chosen kind %d: bs %d sched %d seg %d\n", k, shape[k].bs, shape[k].sched,
                         shape[k].seg);
                *report += line;
            }
            *report += detail;
        }
        return GRMHD_OK;
    }
    int steps(int nsteps) {
        if (dirty) {
            int rc = rebuild();
            if (rc) return rc;
        }
        if (runs.empty() || nsteps <= 0) return GRMHD_OK;
        if (use_graph && !gexec && !timing) {
            HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            int rc = enqueue_step();
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(st, &g);
            if (rc || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                (void)hipGetLastError();
                use_graph = false;  // fall back to plain launches
            } else {
                graph = g;
                e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    drop_graph();
                    use_graph = false;
                }
            }
        }
        if (timing) {
            for (int s = 0; s < nsteps; ++s) {
                int rc = enqueue_step();
                if (rc) return rc;
                if (ev.size() > 4096) {
                    rc = harvest();
                    if (rc) return rc;
                }
            }
            return GRMHD_OK;
        }
        for (int s = 0; s < nsteps; ++s) {
            if (use_graph && gexec) {
                HIPCHK(hipGraphLaunch(gexec, st));
            } else {
                int rc = enqueue_step();
                if (rc) return rc;
            }
        }
        return GRMHD_OK;
    }
};

}  // namespace

// Shell sums of grmhd_diag_full_noalloc: one array per GPU for the life of the process.  On the
// host its name is not a device address; host code uses only the address hipGetSymbolAddress gives
// on each device (scratch_address).
static __device__ __align__(256) double scratch[6 * GRMHD_NOALLOC_MAX_N1];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {nullptr};

// device address of `scratch` on the current device, looked up once per device
int scratch_address(double** out) {
    *out = nullptr;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(GRMHD_EDEVICE, "device %d is beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(GRMHD_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        }
        g_scratch[dev] = (double*)p;
    }
    *out = g_scratch[dev];
    return GRMHD_OK;
}

}  // namespace

struct grmhd_ctx {
    Engine eng;
    Run* run = nullptr;
    double last_dt_req = -1.0;
    double* scratch = nullptr;  // device address of `scratch` on the context's GPU
};

struct grmhd_batch {
    Engine eng;
    std::vector<Run*> jobs;  // resident
    int64_t budget = 0;
    int64_t used = 0;
    int32_t max_jobs = 0;
    int64_t next_id = 1;
};

extern "C" {

void grmhd_params_default(grmhd_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->spin = 0.0;
    p->gam = 4.0 / 3.0;
    p->cfl = 0.45;
    p->riemann = GRMHD_LLF;
    p->rho_fl_coef = 1e-5;
    p->rho_fl_pow = -0.5;
    p->u_fl_coef = 1e-5 / 3.0;
    p->u_fl_pow = -2.5;
    p->fl_abs = 1e-20;
    p->bsq_rho_max = 50.0;
    p->bsq_u_max = 2500.0;
    p->gamma_max = 50.0;
    p->beta_entropy = 1e-2;
    p->c2p_tol = 1e-10;
    p->c2p_maxit = 50;
    p->fixup_max_rounds = 8;
}

const char* grmhd_last_error(void) { return g_err.c_str(); }

int64_t grmhd_footprint_bytes(const grmhd_grid* grid) {
    if (!grid || grid->n1 < 1 || grid->n2 < 1 || grid->n3 < 1) return -1;
    return make_layout(*grid).total;
}

int grmhd_init(grmhd_ctx** out, const grmhd_grid* grid, const grmhd_params* params, const double* prims,
               int32_t prims_on_device, void* hip_stream) {
    if (!out) return fail(GRMHD_EINVAL, "out is NULL");
    *out = nullptr;
    grmhd_ctx* c = new grmhd_ctx();
    int rc = c->eng.init(hip_stream);
    if (rc) { delete c; return rc; }
    rc = create_run(grid, params, prims, prims_on_device, c->eng.st, &c->run);
    if (rc) { delete c; return rc; }
    rc = scratch_address(&c->scratch);
    if (rc) { free_run(c->run); delete c; return rc; }
    c->eng.runs.push_back(c->run);
    c->eng.dirty = true;
    *out = c;
    return GRMHD_OK;
}

static int set_dt_req(grmhd_ctx* c, double dt) {
    if (std::isnan(dt)) return fail(GRMHD_EINVAL, "dt is NaN");
    const double req = dt > 0.0 ? dt : -1.0;
    if (req != c->last_dt_req) {
        launch_set_var(c->run->h.var, req, -1, -1, c->eng.st);
        HIPCHK(hipGetLastError());
        c->last_dt_req = req;
    }
    return GRMHD_OK;
}

int grmhd_steps(grmhd_ctx* c, int32_t nsteps, double dt) {
    if (!c) return fail(GRMHD_EINVAL, "ctx is NULL");
    if (nsteps < 0) return fail(GRMHD_EINVAL, "nsteps < 0");
    int rc = set_dt_req(c, dt);
    if (rc) return rc;
    return c->eng.steps(nsteps);
}

int grmhd_step(grmhd_ctx* c, double dt, double* dt_used) {
    int rc = grmhd_steps(c, 1, dt);
    if (rc) return rc;
    if (dt_used) {
        RunVar v;
        rc = read_var(c->run, c->eng.st, &v);
        if (rc) return rc;
        *dt_used = v.dt;
        if (v.nfail_last > 0) return fail(GRMHD_ENUMERIC, "%d cells left unfixed", v.nfail_last);
    }
    return GRMHD_OK;
}

int grmhd_cons2prim(grmhd_ctx* c, const double* U, double* P, int8_t* code, int32_t on_device) {
    if (!c || !U || !P) return fail(GRMHD_EINVAL, "NULL argument");
    const RunDev& R = c->run->h;
    const int64_t n = (int64_t)R.n1 * R.n2 * R.n3;
    hipStream_t st = c->eng.st;
    if (on_device) {
        launch_cons2prim(R, U, P, code, st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        return GRMHD_OK;
    }
    if (!host_finite(U, NCS * n) || !host_finite(P, NPR * n)) return fail(GRMHD_EINVAL, "inputs hold NaN/Inf");
    double *dU = nullptr, *dP = nullptr;
    int8_t* dc = nullptr;
    HIPCHK(hipMalloc(&dU, NCS * n * 8));
    hipError_t e = hipMalloc(&dP, NPR * n * 8);
    if (e == hipSuccess) e = hipMalloc(&dc, n);
    if (e == hipSuccess) e = hipMemcpyAsync(dU, U, NCS * n * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dP, P, NPR * n * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        launch_cons2prim(R, dU, dP, dc, st);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(P, dP, NPR * n * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && code) e = hipMemcpyAsync(code, dc, n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dU);
    (void)hipFree(dP);
    (void)hipFree(dc);
    if (e != hipSuccess) return fail(GRMHD_EDEVICE, "cons2prim: %s", hipGetErrorString(e));
    return GRMHD_OK;
}

int grmhd_prim2cons(grmhd_ctx* c, const double* P, double* U, int32_t on_device) {
    if (!c || !U || !P) return fail(GRMHD_EINVAL, "NULL argument");
    const RunDev& R = c->run->h;
    const int64_t n = (int64_t)R.n1 * R.n2 * R.n3;
    hipStream_t st = c->eng.st;
    if (on_device) {
        launch_prim2cons(R, P, U, st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        return GRMHD_OK;
    }
    if (!host_finite(P, NPR * n)) return fail(GRMHD_EINVAL, "P holds NaN/Inf");
    double *dU = nullptr, *dP = nullptr;
    HIPCHK(hipMalloc(&dU, NCS * n * 8));
    hipError_t e = hipMalloc(&dP, NPR * n * 8);
    if (e == hipSuccess) e = hipMemcpyAsync(dP, P, NPR * n * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        launch_prim2cons(R, dP, dU, st);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(U, dU, NCS * n * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dU);
    (void)hipFree(dP);
    if (e != hipSuccess) return fail(GRMHD_EDEVICE, "prim2cons: %s", hipGetErrorString(e));
    return GRMHD_OK;
}

int grmhd_diag(grmhd_ctx* c, double* mdot, double* phi_b) {
    if (!c || !mdot || !phi_b) return fail(GRMHD_EINVAL, "NULL argument");
    if (!c->run->h.mks || c->run->ih < 0) return fail(GRMHD_EINVAL, "diagnostics need an MKS grid reaching the horizon");
    double* d = nullptr;
    HIPCHK(hipMalloc(&d, 2 * sizeof(double)));
    launch_diag(c->run->h, c->run->ih, d, c->eng.st);
    double h[2] = {0, 0};
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, c->eng.st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->eng.st);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(GRMHD_EDEVICE, "diag: %s", hipGetErrorString(e));
    *mdot = h[0];
    *phi_b = h[1];
    return GRMHD_OK;
}

// Shell sums of one run (a context's or a batch job's) on the stream its work is enqueued on.
static int diag_full_run(Run* r, hipStream_t st, grmhd_horizon* hz, double* radial) {
    const RunDev& R = r->h;
    if (!R.mks || r->ih < 0) return fail(GRMHD_EINVAL, "diagnostics need an MKS grid reaching the horizon");
    const int n1 = R.n1;
    double* d = nullptr;
    HIPCHK(hipMalloc(&d, 6 * (size_t)n1 * sizeof(double)));
    std::vector<double> h(6 * (size_t)n1);
    launch_diag_shells(R, d, st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, h.size() * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(GRMHD_EDEVICE, "diag_full: %s", hipGetErrorString(e));
    const int ih = r->ih;
    hz->mdot = h[0 * n1 + ih];
    hz->phi_b = h[1 * n1 + ih];
    hz->ldot = h[2 * n1 + ih];
    hz->edot = h[3 * n1 + ih];
    hz->phi_b_norm = hz->mdot != 0.0 ? hz->phi_b / std::sqrt(std::fabs(hz->mdot)) : 0.0;
    hz->i_h = ih;
    hz->reserved_ = 0;
    if (radial) {
        for (int q = 0; q < 4; ++q)
            for (int i = 0; i < n1; ++i) radial[q * n1 + i] = h[q * n1 + i];
        for (int i = 0; i < n1; ++i) {
            const double m = h[i];
            radial[4 * n1 + i] = m != 0.0 ? h[4 * n1 + i] / m : NAN;
            radial[5 * n1 + i] = m != 0.0 ? h[5 * n1 + i] / m : NAN;
        }
    }
    return GRMHD_OK;
}

int grmhd_diag_full(grmhd_ctx* c, grmhd_horizon* hz, double* radial) {
    if (!c || !hz) return fail(GRMHD_EINVAL, "NULL argument");
    return diag_full_run(c->run, c->eng.st, hz, radial);
}

int grmhd_diag_full_noalloc(grmhd_ctx* c, grmhd_horizon* hz, double* radial) {
    if (!c || !hz) return fail(GRMHD_EINVAL, "NULL argument");
    const RunDev& R = c->run->h;
    if (!R.mks || c->run->ih < 0) return fail(GRMHD_EINVAL, "diagnostics need an MKS grid reaching the horizon");
    const int n1 = R.n1, ih = c->run->ih;
    if (n1 > GRMHD_NOALLOC_MAX_N1)
        return fail(GRMHD_EINVAL, "n1 = %d exceeds GRMHD_NOALLOC_MAX_N1 = %d", n1, GRMHD_NOALLOC_MAX_N1);
    if (!c->scratch) return fail(GRMHD_EDEVICE, "no scratch address for this context");
    const hipStream_t st = c->eng.st;
    double* d = c->scratch;
    launch_diag_shells(R, d, st);  // every row of the n1 shells is written: nothing to clear
    hipError_t e = hipGetLastError();
    double hs[4] = {0.0, 0.0, 0.0, 0.0};
    if (radial) {
        if (e == hipSuccess) e = hipMemcpyAsync(radial, d, 6 * (size_t)n1 * sizeof(double), hipMemcpyDeviceToHost, st);
    } else {
        for (int q = 0; q < 4 && e == hipSuccess; ++q)
            e = hipMemcpyAsync(&hs[q], d + (size_t)q * n1 + ih, sizeof(double), hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(GRMHD_EDEVICE, "diag_full_noalloc: %s", hipGetErrorString(e));
    if (radial) {
        for (int q = 0; q < 4; ++q) hs[q] = radial[q * n1 + ih];
        for (int i = 0; i < n1; ++i) {
            const double m = radial[i];
            radial[4 * n1 + i] = m != 0.0 ? radial[4 * n1 + i] / m : NAN;
            radial[5 * n1 + i] = m != 0.0 ? radial[5 * n1 + i] / m : NAN;
        }
    }
    hz->mdot = hs[0];
    hz->phi_b = hs[1];
    hz->ldot = hs[2];
    hz->edot = hs[3];
    hz->phi_b_norm = hz->mdot != 0.0 ? hz->phi_b / std::sqrt(std::fabs(hz->mdot)) : 0.0;
    hz->i_h = ih;
    hz->reserved_ = 0;
    return GRMHD_OK;
}

static int get_prims_run(Run* r, hipStream_t st, double* out, int32_t out_on_device) {
    const RunDev& R = r->h;
    const int64_t n = (int64_t)R.n1 * R.n2 * R.n3;
    if (out_on_device) {
        launch_store(R, out, nullptr, nullptr, st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        return GRMHD_OK;
    }
    double* d = nullptr;
    HIPCHK(hipMalloc(&d, NPR * n * 8));
    launch_store(R, d, nullptr, nullptr, st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(out, d, NPR * n * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(GRMHD_EDEVICE, "get_prims: %s", hipGetErrorString(e));
    return GRMHD_OK;
}

int grmhd_get_prims(grmhd_ctx* c, double* out, int32_t out_on_device) {
    if (!c || !out) return fail(GRMHD_EINVAL, "NULL argument");
    return get_prims_run(c->run, c->eng.st, out, out_on_device);
}

int grmhd_get_time(grmhd_ctx* c, double* t, int64_t* nstep, int64_t* nfail_total) {
    if (!c) return fail(GRMHD_EINVAL, "ctx is NULL");
    RunVar v;
    int rc = read_var(c->run, c->eng.st, &v);
    if (rc) return rc;
    if (t) *t = v.t;
    if (nstep) *nstep = v.nstep;
    if (nfail_total) *nfail_total = v.nfail_total;
    return GRMHD_OK;
}

int grmhd_set_time(grmhd_ctx* c, double t, int64_t nstep) {
    if (!c) return fail(GRMHD_EINVAL, "ctx is NULL");
    if (!std::isfinite(t) || nstep < 0) return fail(GRMHD_EINVAL, "t must be finite and nstep >= 0");
    RunVar v;
    int rc = read_var(c->run, c->eng.st, &v);
    if (rc) return rc;
    v.t = t;
    v.nstep = nstep;
    HIPCHK(hipMemcpyAsync(c->run->h.var, &v, sizeof(RunVar), hipMemcpyHostToDevice, c->eng.st));
    HIPCHK(hipStreamSynchronize(c->eng.st));
    return GRMHD_OK;
}

int grmhd_get_codes(grmhd_ctx* c, int8_t* codes) {
    if (!c || !codes) return fail(GRMHD_EINVAL, "NULL argument");
    const RunDev& R = c->run->h;
    const int64_t n = (int64_t)R.n1 * R.n2 * R.n3;
    int8_t* d = nullptr;
    HIPCHK(hipMalloc(&d, n));
    launch_store(R, nullptr, R.code, d, c->eng.st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(codes, d, n, hipMemcpyDeviceToHost, c->eng.st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->eng.st);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(GRMHD_EDEVICE, "get_codes: %s", hipGetErrorString(e));
    return GRMHD_OK;
}

int grmhd_debug_fixup(grmhd_ctx* c, double* pout, const double* pin, int8_t* code, int64_t* left) {
    if (!c || !pout || !pin || !code) return fail(GRMHD_EINVAL, "NULL argument");
    Run* r = c->run;
    const RunDev& R = r->h;
    Engine& E = c->eng;
    if (E.runs.size() != 1) return fail(GRMHD_EINVAL, "context holds more than one run");
    if (E.dirty) {
        int rc = E.rebuild();
        if (rc) return rc;
    }
    const int64_t n = (int64_t)R.n1 * R.n2 * R.n3;
    if (!host_finite(pin, NPR * n)) return fail(GRMHD_EINVAL, "pin holds NaN/Inf");
    // the run's code array (ghosted layout, ghosts 0) and the list of failed interior cells
    std::vector<int8_t> full((size_t)R.vs, 0);
    std::vector<int32_t> fails;
    for (int i = 0; i < R.n1; ++i)
        for (int j = 0; j < R.n2; ++j)
            for (int k = 0; k < R.n3; ++k) {
                const int64_t e = ((int64_t)i * R.n2 + j) * R.n3 + k;
                const int8_t cd = code[e];
                if (cd < -1 || cd > 3) return fail(GRMHD_EINVAL, "codes must be in [-1, 3]");
                full[(size_t)((i + NG) * R.s1 + (j + NG) * R.s2 + k)] = cd;
                if (cd == -1) fails.push_back((int32_t)e);
            }
    hipStream_t st = E.st;
    double* d = nullptr;
    int8_t* dc = nullptr;
    HIPCHK(hipMalloc(&d, 2 * NPR * n * sizeof(double)));
    if (hipMalloc(&dc, n) != hipSuccess) {
        (void)hipFree(d);
        return fail(GRMHD_ENOMEM, "debug_fixup: staging allocation failed");
    }
    const int32_t nf = (int32_t)fails.size();
    hipError_t e = hipMemcpyAsync(d, pout, NPR * n * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(d + NPR * n, pin, NPR * n * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        launch_load(R, d, 1, st);            // stage output -> P^{n+1/2}
        launch_load(R, d + NPR * n, 0, st);  // stage input  -> P^n
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(R.code, full.data(), full.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nf)
        e = hipMemcpyAsync(R.fail_list, fails.data(), fails.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&R.var->fail_count, &nf, sizeof(nf), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        launch_fixup(E.d_runs, 1, 1, st);     // stage-1 roles: output P^{n+1/2}, input P^n
        e = hipGetLastError();
    }
    // the fixed stage output becomes the context's state
    if (e == hipSuccess) e = hipMemcpyAsync(R.P, R.Ph, (size_t)NPR * R.vs * sizeof(double), hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) {
        launch_store(R, d, R.code, dc, st);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(pout, d, NPR * n * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(code, dc, n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    (void)hipFree(dc);
    if (e != hipSuccess) return fail(GRMHD_EDEVICE, "debug_fixup: %s", hipGetErrorString(e));
    if (left) {
        int64_t m = 0;
        for (int64_t x = 0; x < n; ++x) m += code[x] == -1;
        *left = m;
    }
    return GRMHD_OK;
}

int grmhd_debug_fluxes(grmhd_ctx* c, int32_t d, double* F, double* cmax) {
    if (!c || !F) return fail(GRMHD_EINVAL, "NULL argument");
    Run* r = c->run;
    const RunDev& R = r->h;
    if (d < 1 || d > 3 || !(d == 1 ? R.act1 : (d == 2 ? R.act2 : R.act3)))
        return fail(GRMHD_EINVAL, "direction %d is not active", d);
    Engine& E = c->eng;
    if (E.dirty) {
        int rc = E.rebuild();
        if (rc) return rc;
    }
    hipStream_t st = E.st;
    // the context's one run sits in the uniform-metric or the general table; the entropy-carrying
    // flux kernel used here reads the metric per lane and serves either
    const int kind = flux_kind(d, R.geo_uniform, R.ppm);
    HIPCHK(hipMemsetAsync(R.var->cmax, 0, sizeof(R.var->cmax), st));
    launch_bound(E.d_runs, E.boff(KB_BOUND), 1, E.nblk[KB_BOUND], 0, E.shape[KB_BOUND].bs, E.shape[KB_BOUND].sched, st);
    // one thread per face of the direction (the stage chain's table may count marching waves)
    const int64_t nface = (int64_t)(d == 1 ? R.n1 + 1 : R.n1 + 2 * R.act1) * (d == 2 ? R.n2 + 1 : R.n2 + 2 * R.act2) * R.n3;
    const int fbs = E.shape[kind].bs;
    launch_flux(d, E.d_runs, E.boff(kind), 1, (int)((nface + fbs - 1) / fbs), 0, 1, 1, 0, R.ppm, fbs,
                E.shape[kind].sched, st);
    const int64_t n = (int64_t)NCS * (R.n1 + (d == 1)) * (R.n2 + (d == 2)) * (R.n3 + (d == 3));
    double* dF = nullptr;
    HIPCHK(hipMalloc(&dF, n * 8));
    launch_flux_out(R, d, dF, st);
    unsigned long long bits[3] = {0, 0, 0};
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(F, dF, n * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(bits, R.var->cmax, sizeof(bits), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemsetAsync(R.var->cmax, 0, sizeof(R.var->cmax), st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dF);
    if (e != hipSuccess) return fail(GRMHD_EDEVICE, "debug_fluxes: %s", hipGetErrorString(e));
    if (cmax) std::memcpy(cmax, &bits[d - 1], sizeof(double));
    return GRMHD_OK;
}

static int copy_report(const std::string& r, char* out, int32_t len) {
    if (out && len > 0) {
        const size_t n = std::min((size_t)(len - 1), r.size());
        std::memcpy(out, r.data(), n);
        out[n] = '\0';
    }
    return GRMHD_OK;
}

int grmhd_autotune(grmhd_ctx* c, int32_t steps_per_candidate, char* report, int32_t report_len) {
    if (!c) return fail(GRMHD_EINVAL, "ctx is NULL");
    if (steps_per_candidate < 1) return fail(GRMHD_EINVAL, "steps_per_candidate < 1");
    std::string r;
    int rc = c->eng.autotune(steps_per_candidate, &r);
    if (rc) return rc;
    return copy_report(r, report, report_len);
}

// Per-kernel timing of an engine (a context's or a batch's): switching clears the figures.
static int engine_timing(Engine& E, int32_t on) {
    int rc = E.harvest();
    if (rc) return rc;
    E.timing = on != 0;
    for (int k = 0; k < NTK; ++k) {
        E.t_ms[k] = 0.0;
        E.t_n[k] = 0;
    }
    return GRMHD_OK;
}

static int engine_times(Engine& E, double* avg_ms, int64_t* launches, int32_t n) {
    int rc = E.harvest();
    if (rc) return rc;
    for (int k = 0; k < n && k < NTK; ++k) {
        avg_ms[k] = E.t_n[k] ? E.t_ms[k] / (double)E.t_n[k] : 0.0;
        if (launches) launches[k] = E.t_n[k];
    }
    return GRMHD_OK;
}

int grmhd_kernel_timing(grmhd_ctx* c, int32_t on) {
    if (!c) return fail(GRMHD_EINVAL, "ctx is NULL");
    return engine_timing(c->eng, on);
}

int grmhd_kernel_times(grmhd_ctx* c, double* avg_ms, int64_t* launches, int32_t n) {
    if (!c || !avg_ms || n < 0) return fail(GRMHD_EINVAL, "NULL argument");
    return engine_times(c->eng, avg_ms, launches, n);
}

void grmhd_destroy(grmhd_ctx* c) {
    if (!c) return;
    if (c->eng.st) (void)hipStreamSynchronize(c->eng.st);
    free_run(c->run);
    delete c;
}

/* ---------------------------------------------------------------------------------------- */
/* ensemble                                                                                  */
/* ---------------------------------------------------------------------------------------- */

int grmhd_batch_create(grmhd_batch** out, int64_t hbm_budget_bytes, int32_t max_jobs, void* hip_stream) {
    if (!out) return fail(GRMHD_EINVAL, "out is NULL");
    *out = nullptr;
    grmhd_batch* b = new grmhd_batch();
    int rc = b->eng.init(hip_stream);
    if (rc) { delete b; return rc; }
    if (hbm_budget_bytes <= 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) { delete b; return fail(GRMHD_EDEVICE, "hipMemGetInfo failed"); }
        hbm_budget_bytes = (int64_t)(0.9 * (double)fr);
    }
    b->budget = hbm_budget_bytes;
    b->max_jobs = max_jobs > 0 ? max_jobs : 1024;
    *out = b;
    return GRMHD_OK;
}

int grmhd_batch_admit(grmhd_batch* b, const grmhd_grid* grid, const grmhd_params* params, const double* prims,
                      int32_t prims_on_device, int64_t nsteps, int64_t* job_id) {
    if (!b || !grid || !job_id) return fail(GRMHD_EINVAL, "NULL argument");
    if (nsteps < 0) return fail(GRMHD_EINVAL, "nsteps < 0");
    const int64_t need = grmhd_footprint_bytes(grid);
    if (need < 0) return fail(GRMHD_EINVAL, "bad grid");
    if ((int)b->jobs.size() >= b->max_jobs || b->used + need > b->budget)
        return fail(GRMHD_EAGAIN, "job needs %lld bytes, %lld of %lld in use", (long long)need, (long long)b->used,
                    (long long)b->budget);
    Run* r = nullptr;
    int rc = create_run(grid, params, prims, prims_on_device, b->eng.st, &r);
    if (rc) return rc;
    r->id = b->next_id++;
    r->nsteps_req = nsteps;
    launch_set_var(r->h.var, -1.0, nsteps, nsteps > 0 ? 1 : 0, b->eng.st);
    HIPCHK(hipGetLastError());
    b->jobs.push_back(r);
    b->used += r->L.total;
    b->eng.runs.push_back(r);
    b->eng.dirty = true;
    *job_id = r->id;
    return GRMHD_OK;
}

int grmhd_batch_advance(grmhd_batch* b, int32_t steps) {
    if (!b) return fail(GRMHD_EINVAL, "batch is NULL");
    if (steps < 0) return fail(GRMHD_EINVAL, "steps < 0");
    return b->eng.steps(steps);
}

int grmhd_batch_kernel_timing(grmhd_batch* b, int32_t on) {
    if (!b) return fail(GRMHD_EINVAL, "batch is NULL");
    return engine_timing(b->eng, on);
}

int grmhd_batch_kernel_times(grmhd_batch* b, double* avg_ms, int64_t* launches, int32_t n) {
    if (!b || !avg_ms || n < 0) return fail(GRMHD_EINVAL, "NULL argument");
    return engine_times(b->eng, avg_ms, launches, n);
}

int grmhd_batch_autotune(grmhd_batch* b, int32_t steps_per_candidate, char* report, int32_t report_len) {
    if (!b) return fail(GRMHD_EINVAL, "batch is NULL");
    if (steps_per_candidate < 1) return fail(GRMHD_EINVAL, "steps_per_candidate < 1");
    std::string r;
    int rc = b->eng.autotune(steps_per_candidate, &r);
    if (rc) return rc;
    return copy_report(r, report, report_len);
}

int grmhd_batch_poll(grmhd_batch* b, int64_t* done_ids, int32_t cap, int32_t* n_done) {
    if (!b || !n_done) return fail(GRMHD_EINVAL, "NULL argument");
    *n_done = 0;
    HIPCHK(hipStreamSynchronize(b->eng.st));
    bool changed = false;
    for (Run* r : b->jobs) {
        if (r->reported) continue;
        RunVar v;
        int rc = read_var(r, b->eng.st, &v);
        if (rc) return rc;
        if (v.steps_left <= 0) {
            if (*n_done < cap && done_ids) {
                done_ids[(*n_done)++] = r->id;
                r->reported = true;
                // finished jobs leave the launch tables
                auto it = std::find(b->eng.runs.begin(), b->eng.runs.end(), r);
                if (it != b->eng.runs.end()) { b->eng.runs.erase(it); changed = true; }
            }
        }
    }
    if (changed) b->eng.dirty = true;
    return GRMHD_OK;
}

static Run* find_job(grmhd_batch* b, int64_t id) {
    for (Run* r : b->jobs)
        if (r->id == id) return r;
    return nullptr;
}

int grmhd_batch_fetch(grmhd_batch* b, int64_t job_id, double* prims, double* t, int64_t* nstep) {
    if (!b) return fail(GRMHD_EINVAL, "batch is NULL");
    Run* r = find_job(b, job_id);
    if (!r) return fail(GRMHD_ENOTFOUND, "no job %lld", (long long)job_id);
    if (prims) {
        int rc = get_prims_run(r, b->eng.st, prims, 0);
        if (rc) return rc;
    }
    if (t || nstep) {
        RunVar v;
        int rc = read_var(r, b->eng.st, &v);
        if (rc) return rc;
        if (t) *t = v.t;
        if (nstep) *nstep = v.nstep;
    }
    return GRMHD_OK;
}

int grmhd_batch_get_time(grmhd_batch* b, int64_t job_id, double* t, int64_t* nstep, int64_t* nfail_total) {
    if (!b) return fail(GRMHD_EINVAL, "batch is NULL");
    Run* r = find_job(b, job_id);
    if (!r) return fail(GRMHD_ENOTFOUND, "no job %lld", (long long)job_id);
    RunVar v;
    int rc = read_var(r, b->eng.st, &v);
    if (rc) return rc;
    if (t) *t = v.t;
    if (nstep) *nstep = v.nstep;
    if (nfail_total) *nfail_total = v.nfail_total;
    return GRMHD_OK;
}

int grmhd_batch_diag_full(grmhd_batch* b, int64_t job_id, grmhd_horizon* hz, double* radial) {
    if (!b || !hz) return fail(GRMHD_EINVAL, "NULL argument");
    Run* r = find_job(b, job_id);
    if (!r) return fail(GRMHD_ENOTFOUND, "no job %lld", (long long)job_id);
    return diag_full_run(r, b->eng.st, hz, radial);
}

int grmhd_batch_release(grmhd_batch* b, int64_t job_id) {
    if (!b) return fail(GRMHD_EINVAL, "batch is NULL");
    Run* r = find_job(b, job_id);
    if (!r) return fail(GRMHD_ENOTFOUND, "no job %lld", (long long)job_id);
    HIPCHK(hipStreamSynchronize(b->eng.st));
    auto it = std::find(b->eng.runs.begin(), b->eng.runs.end(), r);
    if (it != b->eng.runs.end()) {
        b->eng.runs.erase(it);
        b->eng.dirty = true;
    }
    b->jobs.erase(std::find(b->jobs.begin(), b->jobs.end(), r));
    b->used -= r->L.total;
    free_run(r);
    return GRMHD_OK;
}

int grmhd_batch_usage(grmhd_batch* b, int64_t* bytes, int32_t* jobs) {
    if (!b) return fail(GRMHD_EINVAL, "batch is NULL");
    if (bytes) *bytes = b->used;
    if (jobs) *jobs = (int32_t)b->jobs.size();
    return GRMHD_OK;
}

void grmhd_batch_destroy(grmhd_batch* b) {
    if (!b) return;
    if (b->eng.st) (void)hipStreamSynchronize(b->eng.st);
    for (Run* r : b->jobs) free_run(r);
    delete b;
}

}  // extern "C"
