// launch.hpp -- host-side launchers of the device kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

struct mhd_ctx;

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
    int kz;                       // z planes per workgroup (both kernels)
    unsigned int ntx, nty, ntz;   // tiles of the flux/update kernel along x, y, z
    unsigned int nblk;            // workgroups of the flux/update kernel
    unsigned int ctx, cty4, cty8; // tiles of the CT kernel along x, and along y for 4 / 8 rows
};
FusedGrid fused_grid(const Geo& g, int kz);
int flux_tile_cells();  // cells per z plane of a flux/update tile

// A state register of the MHD path by role.  FP64 form (R = double): the 8 canonical
// fields rho, M1..3, E, b1..3.  FP32-bulk form (R = float): E (double) first, then
// rho, M1..3, b1..3 as float.
template <class R>
struct RegView {
    R* rho;
    R* m[3];
    R* b[3];
    double* E;
};
template <class R>
__host__ __device__ inline RegView<R> reg_view(void* base, long long n)
{
    RegView<R> v;
    if constexpr (sizeof(R) == sizeof(double)) {
        R* f = (R*)base;
        v.rho = f;
        for (int a = 0; a < 3; ++a) v.m[a] = f + (1 + a) * n;
        v.E = (double*)(f + 4 * n);
        for (int a = 0; a < 3; ++a) v.b[a] = f + (5 + a) * n;
    } else {
        v.E = (double*)base;
        R* f = (R*)(v.E + n);
        v.rho = f;
        for (int a = 0; a < 3; ++a) v.m[a] = f + (1 + a) * n;
        for (int a = 0; a < 3; ++a) v.b[a] = f + (4 + a) * n;
    }
    return v;
}
inline size_t register_bytes(long long n, bool fp32)
{
    return fp32 ? (size_t)n * (sizeof(double) + 7 * sizeof(float)) : (size_t)n * 8 * sizeof(double);
}

// Fluxes of the stage input `in` and the cell fields of out = g0 in + g1 base + bdt L
// (out must not alias in or base).  F: the 9 face fields the edge EMFs need (per
// direction the mass flux and the two face values of E, see FaceField); Rc: 3 fields of
// the cell E = -v x B (both in the path's real).
hipError_t launch_mhd_flux3(const Geo& g, const MhdParams& p, const FusedGrid& fg, bool fp32, int recon,
                            int riemann, void* in, void* base, void* out, void* F, void* Rc, StageCoef coef,
                            hipStream_t s);
// The face fields of out = g0 in + g1 base + bdt L from the edge EMFs.  With dt_out the
// CFL step of out (times cfl_scale) is reduced into dt_out via one partial per workgroup.
hipError_t launch_mhd_ct_update(const Geo& g, const MhdParams& p, const FusedGrid& fg, bool fp32,
                                void* in, void* base, const void* F, const void* Rc, void* out,
                                StageCoef coef, double* partial, double* dt_out, double cfl_scale,
                                hipStream_t s);
// FP32-bulk register <-> canonical FP64 state (8 fields).
hipError_t launch_pack_fp32(const Geo& g, const double* canon, void* reg, hipStream_t s);
hipError_t launch_unpack_fp32(const Geo& g, const void* reg, double* canon, hipStream_t s);

// ---- CFL and diagnostics ----
// partial: ceil(n/kBlock) doubles; dt_out: 1 double on the device.
hipError_t launch_cfl_mhd(const Geo& g, const MhdParams& p, const double* U, double* partial,
                          double* dt_out, double scale, hipStream_t s);
// The same over the interior cells of nb equal padded FP64 blocks of grid pg (ghost
// layers on every side, interior bx x by x bz, block b's register at reg + 8 off[b]
// doubles); partial: min(ceil(nb bx by bz / kBlock), 4096) doubles.
hipError_t launch_cfl_blocks(const Geo& pg, const MhdParams& p, const double* reg, const unsigned long long* off,
                             int nb, int ghost, int bx, int by, int bz, double* partial, double* dt_out,
                             double scale, hipStream_t s);
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
// Tiling of the fluid passes: one workgroup per (fluid, 64 x 8 tile, chunk of kz planes).
struct DustGrid {
    int kz;
    unsigned int ntx, nty, ntz, ntiles, nblk;
};
DustGrid dust_grid(const Geo& g, int nfluids);
// Explicit parts: stage 1 writes X = u + lam dt L(u) into U1; stage 2 writes
// X = cu u + c1 U1 + (1 - delta) dt L(U1) over u in place.  fp32: the registers hold
// FP32 fields (explicit part in FP32, drag solve in FP64).
hipError_t launch_fluid_pass1(const Geo& g, const DustParams& p, const DustGrid& d, bool fp32, int recon,
                              const void* u, void* U1, double dt, hipStream_t s);
hipError_t launch_fluid_pass2(const Geo& g, const DustParams& p, const DustGrid& d, bool fp32, int recon,
                              void* u, const void* U1, double dt, hipStream_t s);
// Drag solves in place on the explicit part; stage 2 adds the stage-1 drag rates first
// and reduces the CFL step of the new state into dt_out (partial: ceil(n/kBlock) doubles).
hipError_t launch_drag1(const Geo& g, const DustParams& p, bool fp32, void* U1, double dt, hipStream_t s);
hipError_t launch_drag2_cfl(const Geo& g, const DustParams& p, bool fp32, void* u, const void* U1, double dt,
                            double* partial, double* dt_out, double cfl_scale, hipStream_t s);
// FP32 dust register <-> canonical FP64 state, m = nv * n values
hipError_t launch_dust_pack(long long m, const double* canon, void* reg, hipStream_t s);
hipError_t launch_dust_unpack(long long m, const void* reg, double* canon, hipStream_t s);

inline unsigned int blocks_for(long long n) { return (unsigned int)((n + kBlock - 1) / kBlock); }

// ---- what the closure step needs of a single-grid context (api.hip) ----
struct CtxView {
    Geo geo;
    MhdParams mp;
    hipStream_t stream;
    double* state;  // the current state in the canonical FP64 layout (FP64 adiabatic MHD only, else null)
};
CtxView ctx_view(mhd_ctx* c);
// Recompute the context's CFL step from its current state (after a change in place).
hipError_t ctx_refresh_cfl(mhd_ctx* c);

}  // namespace mhd
