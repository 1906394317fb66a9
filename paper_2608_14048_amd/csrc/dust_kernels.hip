// dust_kernels.hip -- IMEX2P step of isothermal gas + N pressureless dust fluids.
//
// Explicit part F(u): minus the flux divergence (isothermal HLLE for the gas, the
// pressureless Rusanov flux for each species; Sec. "Multifluid Dust") plus the gas
// acceleration rho_g g as an unsplit source.  Implicit part G(u): the linear drag of
// eq. (dust_momentum) and its reaction on the gas.  The ARS(2,2,2) pair with the
// diagonal weight lam = 1 + 1/sqrt(2) (Sec. "Time Integration"):
//   U1    = S_h(u + lam dt F(u)),                                   h = lam dt
//   u_new = S_h(u + dt[delta F(u) + (1-delta) F(U1)] + (1-lam) dt G(U1))
// with delta = 1 - 1/(2 lam).  Stage 2 recovers dt F(u) from stage 1's own output,
// dt F(u) = (U1 - u)/lam - dt G(U1), so only the two registers u and U1 exist:
//   u_new = S_h((1 - delta/lam) u + (delta/lam) U1 + (1-delta) dt F(U1)
//               + (1 - lam - delta) dt G(U1)).
// S_h is the closed-form solve of the arrowhead drag system: with w_k = h/(t_k + h),
//   v_g' = (p_g + sum_k w_k p_k) / (rho_g + sum_k w_k rho_k),
//   p_k' = (t_k p_k + h rho_k v_g') / (t_k + h),   p_g' = rho_g v_g',
// exact, O(N) and momentum conserving.
#include "launch.hpp"
#include "physics.hpp"

namespace mhd {

namespace {
constexpr double kLam = 1.7071067811865475244;    // 1 + 1/sqrt(2)
constexpr double kDelta = 0.70710678118654752440;  // 1 - 1/(2 lam) = 1/sqrt(2)
}

// Primitives of fluid s at cell c: gas density floor; dust below its floor reads as
// the floor at rest.
__device__ __forceinline__ void fluid_prim(const DustParams& p, int s, const double* __restrict__ U,
                                           long long n, long long c, double w[4])
{
    const double* u = U + 4LL * s * n;
    double d = u[c];
    if (s == 0) {
        if (d < p.rho_floor) d = p.rho_floor;
    } else if (d < p.dust_floor) {
        w[0] = p.dust_floor;
        w[1] = w[2] = w[3] = 0.0;
        return;
    }
    w[0] = d;
    w[1] = u[n + c] / d;
    w[2] = u[2 * n + c] / d;
    w[3] = u[3 * n + c] / d;
}

__global__ __launch_bounds__(kBlock) void k_dust_prims(Geo g, DustParams p, const double* __restrict__ U,
                                                       double* __restrict__ W)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.n) return;
    const long long n = g.n;
    for (int s = 0; s <= p.nd; ++s) {
        double w[4];
        fluid_prim(p, s, U, n, c, w);
#pragma unroll
        for (int q = 0; q < 4; ++q) W[(4LL * s + q) * n + c] = w[q];
    }
}

// Face fluxes of every fluid on the left face of each cell along D; F holds
// 4(1+nd) fields in the global frame (mass, Mx, My, Mz per fluid).
template <int D, int RECON>
__global__ __launch_bounds__(kBlock) void k_dust_flux(Geo g, DustParams p, const double* __restrict__ W,
                                                      double* __restrict__ F)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.n) return;
    int i, j, k;
    cell_ijk(g, c, i, j, k);
    constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
    const long long n = g.n;
    long long at[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) at[s] = shifted(g, i, j, k, D, s - 3);
    for (int s = 0; s <= p.nd; ++s) {
        const double* w = W + 4LL * s * n;
        double st[6];
        Prim4 L, R;
#pragma unroll
        for (int m = 0; m < 6; ++m) st[m] = w[at[m]];
        face_states<RECON>(st, L.d, R.d);
#pragma unroll
        for (int m = 0; m < 6; ++m) st[m] = w[(1 + D) * n + at[m]];
        face_states<RECON>(st, L.vn, R.vn);
#pragma unroll
        for (int m = 0; m < 6; ++m) st[m] = w[(1 + T1) * n + at[m]];
        face_states<RECON>(st, L.vt1, R.vt1);
#pragma unroll
        for (int m = 0; m < 6; ++m) st[m] = w[(1 + T2) * n + at[m]];
        face_states<RECON>(st, L.vt2, R.vt2);
        Flux4 f;
        if (s == 0)
            riemann_iso_hlle(L, R, p.cs, f);
        else
            riemann_dust(L, R, f);
        double* o = F + 4LL * s * n;
        o[c] = f.d;
        o[(1 + D) * n + c] = f.mn;
        o[(1 + T1) * n + c] = f.mt1;
        o[(1 + T2) * n + c] = f.mt2;
    }
}

// -flux divergence of variable v at cell c (F: 3 direction blocks of nv fields).
__device__ __forceinline__ double neg_div(const Geo& g, const double* __restrict__ F, long long nv,
                                          int v, long long c, long long cx, long long cy, long long cz)
{
    const long long n = g.n;
    const double* Fx = F;
    const double* Fy = F + nv * n;
    const double* Fz = F + 2 * nv * n;
    const double fx = (Fx[v * n + cx] - Fx[v * n + c]) * g.inv_dx[0];
    const double fy = (Fy[v * n + cy] - Fy[v * n + c]) * g.inv_dx[1];
    const double fz = (Fz[v * n + cz] - Fz[v * n + c]) * g.inv_dx[2];
    return -((fx + fy) + fz);
}

// Closed-form drag solve of one momentum component, in place on p[0..nd].
__device__ __forceinline__ void drag_solve(const DustParams& p, const double* rho, double* mom,
                                           double h)
{
    double num = mom[0], den = rho[0];
    for (int s = 1; s <= p.nd; ++s) {
        const double w = h / (p.ts[s - 1] + h);
        num += w * mom[s];
        den += w * rho[s];
    }
    const double vg = num / den;
    for (int s = 1; s <= p.nd; ++s) {
        const double t = p.ts[s - 1];
        mom[s] = (t * mom[s] + h * rho[s] * vg) / (t + h);
    }
    mom[0] = rho[0] * vg;
}

__global__ __launch_bounds__(kBlock) void k_imex_stage1(Geo g, DustParams p, const double* __restrict__ u,
                                                        const double* __restrict__ F,
                                                        double* __restrict__ U1, double dt)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.n) return;
    int i, j, k;
    cell_ijk(g, c, i, j, k);
    const long long n = g.n;
    const long long nv = 4LL * (p.nd + 1);
    const long long cx = shifted(g, i, j, k, 0, 1), cy = shifted(g, i, j, k, 1, 1),
                    cz = shifted(g, i, j, k, 2, 1);
    const double h = kLam * dt;
    double rho[kMaxDust + 1];
    for (int s = 0; s <= p.nd; ++s) {
        const int v = 4 * s;
        rho[s] = u[v * n + c] + h * neg_div(g, F, nv, v, c, cx, cy, cz);
        U1[v * n + c] = rho[s];
    }
    const double rg = u[c];
    for (int a = 0; a < 3; ++a) {
        double mom[kMaxDust + 1];
        for (int s = 0; s <= p.nd; ++s) {
            const int v = 4 * s + 1 + a;
            double L = neg_div(g, F, nv, v, c, cx, cy, cz);
            if (s == 0) L += rg * p.gacc[a];
            mom[s] = u[v * n + c] + h * L;
        }
        drag_solve(p, rho, mom, h);
        for (int s = 0; s <= p.nd; ++s) U1[(4 * s + 1 + a) * n + c] = mom[s];
    }
}

__global__ __launch_bounds__(kBlock) void k_imex_stage2(Geo g, DustParams p, double* __restrict__ u,
                                                        const double* __restrict__ U1,
                                                        const double* __restrict__ F, double dt)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.n) return;
    int i, j, k;
    cell_ijk(g, c, i, j, k);
    const long long n = g.n;
    const long long nv = 4LL * (p.nd + 1);
    const long long cx = shifted(g, i, j, k, 0, 1), cy = shifted(g, i, j, k, 1, 1),
                    cz = shifted(g, i, j, k, 2, 1);
    const double h = kLam * dt;
    const double cu = 1.0 - kDelta / kLam, c1 = kDelta / kLam;
    const double cf = (1.0 - kDelta) * dt, cg = (1.0 - kLam - kDelta) * dt;
    double rho[kMaxDust + 1];
    for (int s = 0; s <= p.nd; ++s) {
        const int v = 4 * s;
        rho[s] = (cu * u[v * n + c] + c1 * U1[v * n + c]) + cf * neg_div(g, F, nv, v, c, cx, cy, cz);
    }
    // drag rates of the stage-1 state: velocities through the same primitive recovery
    double wg[4];
    fluid_prim(p, 0, U1, n, c, wg);
    const double rg1 = U1[c];
    for (int a = 0; a < 3; ++a) {
        double mom[kMaxDust + 1];
        double gsum = 0.0;
        for (int s = 1; s <= p.nd; ++s) {
            double wd[4];
            fluid_prim(p, s, U1, n, c, wd);
            const double fk = U1[4LL * s * n + c] * (wg[1 + a] - wd[1 + a]) / p.ts[s - 1];
            const int v = 4 * s + 1 + a;
            const double L = neg_div(g, F, nv, v, c, cx, cy, cz);
            mom[s] = ((cu * u[v * n + c] + c1 * U1[v * n + c]) + cf * L) + cg * fk;
            gsum -= fk;
        }
        const int v0 = 1 + a;
        const double L0 = neg_div(g, F, nv, v0, c, cx, cy, cz) + rg1 * p.gacc[a];
        mom[0] = ((cu * u[v0 * n + c] + c1 * U1[v0 * n + c]) + cf * L0) + cg * gsum;
        drag_solve(p, rho, mom, h);
        for (int s = 0; s <= p.nd; ++s) u[(4 * s + 1 + a) * n + c] = mom[s];
    }
    for (int s = 0; s <= p.nd; ++s) u[4LL * s * n + c] = rho[s];
}

// ----------------------------------------------------------------------------------

hipError_t launch_dust_prims(const Geo& g, const DustParams& p, const double* U, double* W,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_dust_prims, dim3(blocks_for(g.n)), dim3(kBlock), 0, s, g, p, U, W);
    return hipGetLastError();
}

template <int RECON>
static hipError_t dust_flux_all(const Geo& g, const DustParams& p, const double* W, double* F,
                                hipStream_t s)
{
    const long long nvn = 4LL * (p.nd + 1) * g.n;
    const dim3 gr(blocks_for(g.n)), bl(kBlock);
    hipLaunchKernelGGL((k_dust_flux<0, RECON>), gr, bl, 0, s, g, p, W, F);
    hipLaunchKernelGGL((k_dust_flux<1, RECON>), gr, bl, 0, s, g, p, W, F + nvn);
    hipLaunchKernelGGL((k_dust_flux<2, RECON>), gr, bl, 0, s, g, p, W, F + 2 * nvn);
    return hipGetLastError();
}

hipError_t launch_dust_fluxes(const Geo& g, const DustParams& p, int recon, const double* W,
                              double* F, hipStream_t s)
{
    if (recon == 0) return dust_flux_all<0>(g, p, W, F, s);
    return dust_flux_all<1>(g, p, W, F, s);
}

hipError_t launch_imex_stage1(const Geo& g, const DustParams& p, const double* u,
                              const double* F, double* U1, double dt, hipStream_t s)
{
    hipLaunchKernelGGL(k_imex_stage1, dim3(blocks_for(g.n)), dim3(kBlock), 0, s, g, p, u, F, U1, dt);
    return hipGetLastError();
}

hipError_t launch_imex_stage2(const Geo& g, const DustParams& p, double* u, const double* U1,
                              const double* F, double dt, hipStream_t s)
{
    hipLaunchKernelGGL(k_imex_stage2, dim3(blocks_for(g.n)), dim3(kBlock), 0, s, g, p, u, U1, F, dt);
    return hipGetLastError();
}

}  // namespace mhd
