// grmhd_kernels.h -- host-side launchers of the stage kernels (internal to the library).
#pragma once
#include "grmhd_dev.h"

namespace grmhd {

struct GeoArgs {
    int n1, n2, mks;
    int nx;          // power of the hyper-exponential radial term
    double xb;       // ln r_br: X1 where r(X1) turns hyper-exponential (+inf: never)
    double x1lo, dx1, dx2, spin, h;
    double rho_fl_coef, rho_fl_pow, u_fl_coef, u_fl_pow, fl_abs;
    double* gc;
    double* gf1;
    double* gf2;
};

void launch_geometry(const GeoArgs& A, hipStream_t st);
// bs: threads per workgroup (64, 128 or 256); sched bit 0: XCD-contiguous block order
void launch_bound(const RunDev* runs, const int* boff, int nruns, int nblocks, int which, int bs, int sched,
                  hipStream_t st);
// ent = 1 also computes and stores the entropy component (diagnostics); the stage chain uses 0.
// uni = 1 (with ent = 0): the block table covers only row-path runs (scalar metric loads)
// ppm = 1: the block table covers only PPM runs (0: only PLM runs)
// uni = 1, ppm = 0, ent = 0: X1 and X2 faces are marched along the normal in segments of each
// run's mseg faces per wave (march_waves gives the wave count), X3 faces take neighbouring cells
// from lanes; uni = 1, ppm = 1, ent = 0: X3 faces from lanes, X1 and X2 faces two per thread
void launch_flux(int d, const RunDev* runs, const int* boff, int nruns, int nblocks, int which, int do_cfl,
                 int ent, int uni, int ppm, int bs, int sched, hipStream_t st);
// faces x rows x chunks of the march along d in {1, 2}: its waves with one-face segments
inline int64_t march_units(const RunDev& R, int d) {
    const int64_t nf = (d == 1 ? R.n1 : R.n2) + 1;
    const int64_t nrow = d == 1 ? R.n2 + 2 * R.act2 : R.n1 + 2 * R.act1;
    return nf * nrow * R.nkc;
}
// waves of the marching face kernel along d in {1, 2} for a run on the row path (segments of
// R.mseg[d - 1] faces)
inline int64_t march_waves(const RunDev& R, int d) {
    const int64_t nf = (d == 1 ? R.n1 : R.n2) + 1;
    const int64_t nrow = d == 1 ? R.n2 + 2 * R.act2 : R.n1 + 2 * R.act1;
    const int64_t seg = R.mseg[d - 1];
    return (nf + seg - 1) / seg * nrow * R.nkc;
}
// flux-CT edge EMFs of every run with two or more active directions, over (n1+1)(n2+1)n3 sites
void launch_emf(const RunDev* runs, const int* boff, int nruns, int nblocks, int bs, int sched, hipStream_t st);
void launch_dt(const RunDev* runs, int nruns, hipStream_t st);
// uni = 1: the block table covers only row-path runs (scalar metric loads)
void launch_update(const RunDev* runs, const int* boff, int nruns, int nblocks, int stage, int uni, int bs,
                   int sched, hipStream_t st);
void launch_update_slow(const RunDev* runs, int nruns, int stage, hipStream_t st);
void launch_fixup(const RunDev* runs, int nruns, int stage, hipStream_t st);
void launch_load(const RunDev& R, const double* in, int to_half, hipStream_t st);
void launch_store(const RunDev& R, double* out, const int8_t* code_in, int8_t* code_out, hipStream_t st);
void launch_prim2cons(const RunDev& R, const double* P, double* U, hipStream_t st);
void launch_cons2prim(const RunDev& R, const double* U, double* P, int8_t* code, hipStream_t st);
void launch_diag(const RunDev& R, int ih, double* out, hipStream_t st);
// per radial shell: the six accretion sums of Sec. 4.2, out[6][n1] (device)
void launch_diag_shells(const RunDev& R, double* out, hipStream_t st);
void launch_flux_out(const RunDev& R, int d, double* out, hipStream_t st);
void launch_set_var(RunVar* V, double dt_req, long long steps_left, int active, hipStream_t st);

}  // namespace grmhd
