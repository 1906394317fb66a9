// launch.hpp -- host-side launchers of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace mhd {

struct MhdParams {
    double gamma, gm1inv, rho_floor, p_floor, hlld_eps;
    double gacc[3];
};

struct DustParams {
    int nd;
    double cs, rho_floor, dust_floor;
    double gacc[3];
    double ts[kMaxDust];
};

// ---- adiabatic MHD (z-marching tile kernels) ----
struct FusedGrid {
    int kz;                       // z planes per workgroup
    unsigned int ntx, nty, ntz;   // tiles along x, y, z
    unsigned int nblk;            // workgroups of the flux kernel
    unsigned int nty2, nblk2;     // tiles along y and workgroups of the CT/update kernel
};
FusedGrid fused_grid(const Geo& g, int kz);
// U: 8 fields (rho, M1..3, E, b1..3) of the stage input.
// F: 7 fields per direction, dir-major (mass, Mx, My, Mz, energy, E_t1, E_t2); Rc: 3
// fields of the cell E = -v x B.
hipError_t launch_mhd_flux3(const Geo& g, const MhdParams& p, const FusedGrid& fg, int recon,
                            int riemann, const double* U, double* F, double* Rc, hipStream_t s);
// out = g0 in + g1 base + bdt L; out must not alias in or base.  With dt_out the CFL
// step of out (times cfl_scale) is reduced into dt_out via one partial per workgroup.
hipError_t launch_mhd_ct_update(const Geo& g, const MhdParams& p, const FusedGrid& fg,
                                const double* in, const double* base, const double* F,
                                const double* Rc, double* out, StageCoef coef, double* partial,
                                double* dt_out, double cfl_scale, hipStream_t s);

// ---- CFL and diagnostics ----
// partial: ceil(n/kBlock) doubles; dt_out: 1 double on the device.
hipError_t launch_cfl_mhd(const Geo& g, const MhdParams& p, const double* U, double* partial,
                          double* dt_out, double scale, hipStream_t s);
hipError_t launch_cfl_dust(const Geo& g, const DustParams& p, const double* U,
                           double* partial, double* dt_out, double scale, hipStream_t s);
// out[0] = scale * (NaN-propagating) min of partial[0..m)
hipError_t launch_min_final(const double* partial, long long m, double scale, double* out,
                            hipStream_t s);
// partial: ceil(n/kBlock) * nq doubles; out: nq doubles on the device.
int diag_count(int ndust);
hipError_t launch_diag(const Geo& g, int mhd, int ndust, const double* U, double* partial,
                       double* out, hipStream_t s);

// ---- isothermal gas + dust (IMEX2P) ----
hipError_t launch_dust_prims(const Geo& g, const DustParams& p, const double* U, double* W,
                             hipStream_t s);
hipError_t launch_dust_fluxes(const Geo& g, const DustParams& p, int recon, const double* W,
                              double* F, hipStream_t s);
// stage 1: U1 = S_h(u + lam dt F(u)); stage 2: u <- S_h(RHS2) in place.
hipError_t launch_imex_stage1(const Geo& g, const DustParams& p, const double* u,
                              const double* F, double* U1, double dt, hipStream_t s);
hipError_t launch_imex_stage2(const Geo& g, const DustParams& p, double* u, const double* U1,
                              const double* F, double dt, hipStream_t s);

inline unsigned int blocks_for(long long n) { return (unsigned int)((n + kBlock - 1) / kBlock); }

}  // namespace mhd
