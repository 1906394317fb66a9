// mhd_kernels.hip -- one stage of the adiabatic CT-MHD Godunov update on gfx950.
//
// A stage is L(u) of eq. (fv_update) plus the face-field rate of eq. (ct), combined
// into the two-register form of eq. (two_register):
//   k_mhd_prims   cons -> prims (floors on the primitives), B_cc = mean of the faces
//   k_mhd_flux<d> reconstruction of primitives along d, rotation to the face frame,
//                 HLLE/HLLD, rotation back; also the face values of E from the
//                 induction fluxes (E_t2 = -F(B_t1), E_t1 = +F(B_t2))
//   k_mhd_edges   Gardiner-Stone upwind edge EMFs from the face values, the cell
//                 field E = -v x B and the mass-flux signs
//   k_mhd_update  out = g0 in + g1 base + bdt (L_U, -curl E)
// Every kernel is cell parallel over the x-fastest layout, so consecutive lanes of a
// wavefront touch consecutive addresses in every sweep direction.
#include "launch.hpp"
#include "physics.hpp"

namespace mhd {

__global__ __launch_bounds__(kBlock) void k_mhd_prims(Geo g, MhdParams p,
                                                      const double* __restrict__ U,
                                                      double* __restrict__ W)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.n) return;
    int i, j, k;
    cell_ijk(g, c, i, j, k);
    const long long n = g.n;
    const double bx = 0.5 * (U[5 * n + c] + U[5 * n + shifted(g, i, j, k, 0, 1)]);
    const double by = 0.5 * (U[6 * n + c] + U[6 * n + shifted(g, i, j, k, 1, 1)]);
    const double bz = 0.5 * (U[7 * n + c] + U[7 * n + shifted(g, i, j, k, 2, 1)]);
    double d = U[c];
    if (d < p.rho_floor) d = p.rho_floor;
    const double vx = U[n + c] / d, vy = U[2 * n + c] / d, vz = U[3 * n + c] / d;
    const double ke = 0.5 * d * ((vx * vx + vy * vy) + vz * vz);
    const double me = 0.5 * ((bx * bx + by * by) + bz * bz);
    double pr = (p.gamma - 1.0) * ((U[4 * n + c] - ke) - me);
    if (pr < p.p_floor) pr = p.p_floor;
    W[c] = d;
    W[n + c] = vx;
    W[2 * n + c] = vy;
    W[3 * n + c] = vz;
    W[4 * n + c] = pr;
    W[5 * n + c] = bx;
    W[6 * n + c] = by;
    W[7 * n + c] = bz;
}

template <int D, int RECON, int RS>
__global__ __launch_bounds__(kBlock) void k_mhd_flux(Geo g, MhdParams p,
                                                     const double* __restrict__ W,
                                                     const double* __restrict__ bface,
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
    double st[6];
    Prim7 L, R;
#define MHD_RECON(comp, fld)                                           \
    _Pragma("unroll") for (int s = 0; s < 6; ++s) st[s] = W[(comp) * n + at[s]]; \
    face_states<RECON>(st, L.fld, R.fld);
    MHD_RECON(0, d)
    MHD_RECON(1 + D, vn)
    MHD_RECON(1 + T1, vt1)
    MHD_RECON(1 + T2, vt2)
    MHD_RECON(4, p)
    MHD_RECON(5 + T1, bt1)
    MHD_RECON(5 + T2, bt2)
#undef MHD_RECON
    const double bn = bface[c];
    Flux7 f;
    if (RS == 1)
        riemann_hlld(L, R, bn, p.gamma, p.gm1inv, p.hlld_eps, f);
    else
        riemann_hlle(L, R, bn, p.gamma, p.gm1inv, f);
    F[c] = f.d;
    F[(1 + D) * n + c] = f.mn;
    F[(1 + T1) * n + c] = f.mt1;
    F[(1 + T2) * n + c] = f.mt2;
    F[4 * n + c] = f.e;
    F[5 * n + c] = f.bt2;   // E_{t1}
    F[6 * n + c] = -f.bt1;  // E_{t2}
}

__device__ __forceinline__ double upwind(double m, double pos, double neg)
{
    return m > 0.0 ? pos : (m < 0.0 ? neg : 0.5 * (pos + neg));
}

// Component a of the cell-centred E = -v x B from the primitives.
__device__ __forceinline__ double cell_emf(const double* __restrict__ W, long long n, long long c, int a)
{
    const int b = (a + 1) % 3, e = (a + 2) % 3;
    return W[(1 + e) * n + c] * W[(5 + b) * n + c] - W[(1 + b) * n + c] * W[(5 + e) * n + c];
}

// Edge E_a at (p-1/2, q-1/2) (p = a+1, q = a+2 cyclic), stored at the cell index.
__global__ __launch_bounds__(kBlock) void k_mhd_edges(Geo g, const double* __restrict__ W,
                                                      const double* __restrict__ F,
                                                      double* __restrict__ E)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.n) return;
    int i, j, k;
    cell_ijk(g, c, i, j, k);
    const long long n = g.n;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int pa = (a + 1) % 3, qa = (a + 2) % 3;
        const double* Fp = F + (long long)pa * 7 * n;
        const double* Fq = F + (long long)qa * 7 * n;
        const long long cp = shifted(g, i, j, k, pa, -1);
        const long long cq = shifted(g, i, j, k, qa, -1);
        int ip, jp, kp;
        cell_ijk(g, cp, ip, jp, kp);
        const long long cpq = shifted(g, ip, jp, kp, qa, -1);
        // E_a is E_{t2} of the p-sweep (slot 6) and E_{t1} of the q-sweep (slot 5)
        const double X0 = Fp[6 * n + c], Xm = Fp[6 * n + cq];
        const double Y0 = Fq[5 * n + c], Ym = Fq[5 * n + cp];
        const double R00 = cell_emf(W, n, c, a), Rm0 = cell_emf(W, n, cp, a);
        const double R0m = cell_emf(W, n, cq, a), Rmm = cell_emf(W, n, cpq, a);
        const double dqp = upwind(Fp[c], Rm0 - Ym, R00 - Y0);
        const double dqm = upwind(Fp[cq], Ym - Rmm, Y0 - R0m);
        const double dpp = upwind(Fq[c], R0m - Xm, R00 - X0);
        const double dpm = upwind(Fq[cp], Xm - Rmm, X0 - Rm0);
        E[a * n + c] = 0.25 * (((X0 + Xm) + (Y0 + Ym)) - ((dqp - dqm) + (dpp - dpm)));
    }
}

__global__ __launch_bounds__(kBlock) void k_mhd_update(Geo g, MhdParams p,
                                                       const double* __restrict__ in,
                                                       const double* base,
                                                       const double* __restrict__ F,
                                                       const double* __restrict__ E,
                                                       double* out, StageCoef co)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= g.n) return;
    int i, j, k;
    cell_ijk(g, c, i, j, k);
    const long long n = g.n;
    const long long cx = shifted(g, i, j, k, 0, 1);
    const long long cy = shifted(g, i, j, k, 1, 1);
    const long long cz = shifted(g, i, j, k, 2, 1);
    const double* Fx = F;
    const double* Fy = F + 7 * n;
    const double* Fz = F + 14 * n;
    double L[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        const double fx = (Fx[v * n + cx] - Fx[v * n + c]) * g.inv_dx[0];
        const double fy = (Fy[v * n + cy] - Fy[v * n + c]) * g.inv_dx[1];
        const double fz = (Fz[v * n + cz] - Fz[v * n + c]) * g.inv_dx[2];
        L[v] = -((fx + fy) + fz);
    }
    const double rho = in[c];
    L[1] += rho * p.gacc[0];
    L[2] += rho * p.gacc[1];
    L[3] += rho * p.gacc[2];
    L[4] += (in[n + c] * p.gacc[0] + in[2 * n + c] * p.gacc[1]) + in[3 * n + c] * p.gacc[2];
    const double* Ex = E;
    const double* Ey = E + n;
    const double* Ez = E + 2 * n;
    double Lb[3];
    Lb[0] = -((Ez[cy] - Ez[c]) * g.inv_dx[1] - (Ey[cz] - Ey[c]) * g.inv_dx[2]);
    Lb[1] = -((Ex[cz] - Ex[c]) * g.inv_dx[2] - (Ez[cx] - Ez[c]) * g.inv_dx[0]);
    Lb[2] = -((Ey[cx] - Ey[c]) * g.inv_dx[0] - (Ex[cy] - Ex[c]) * g.inv_dx[1]);
    double o[8];
#pragma unroll
    for (int v = 0; v < 5; ++v) o[v] = (co.g0 * in[v * n + c] + co.g1 * base[v * n + c]) + co.bdt * L[v];
#pragma unroll
    for (int v = 0; v < 3; ++v)
        o[5 + v] = (co.g0 * in[(5 + v) * n + c] + co.g1 * base[(5 + v) * n + c]) + co.bdt * Lb[v];
#pragma unroll
    for (int v = 0; v < 8; ++v) out[v * n + c] = o[v];
}

// ----------------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------------

hipError_t launch_mhd_prims(const Geo& g, const MhdParams& p, const double* U, double* W,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_mhd_prims, dim3(blocks_for(g.n)), dim3(kBlock), 0, s, g, p, U, W);
    return hipGetLastError();
}

template <int RECON, int RS>
static hipError_t flux_dir(const Geo& g, const MhdParams& p, int dir, const double* W,
                           const double* U, double* F, hipStream_t s)
{
    const long long n = g.n;
    const dim3 gr(blocks_for(n)), bl(kBlock);
    if (dir == 0)
        hipLaunchKernelGGL((k_mhd_flux<0, RECON, RS>), gr, bl, 0, s, g, p, W, U + 5 * n, F);
    else if (dir == 1)
        hipLaunchKernelGGL((k_mhd_flux<1, RECON, RS>), gr, bl, 0, s, g, p, W, U + 6 * n, F + 7 * n);
    else
        hipLaunchKernelGGL((k_mhd_flux<2, RECON, RS>), gr, bl, 0, s, g, p, W, U + 7 * n, F + 14 * n);
    return hipGetLastError();
}

hipError_t launch_mhd_flux_dir(const Geo& g, const MhdParams& p, int recon, int riemann, int dir,
                               const double* W, const double* U, double* F, hipStream_t s)
{
    if (riemann == 1) {
        if (recon == 0) return flux_dir<0, 1>(g, p, dir, W, U, F, s);
        if (recon == 1) return flux_dir<1, 1>(g, p, dir, W, U, F, s);
        return flux_dir<2, 1>(g, p, dir, W, U, F, s);
    }
    if (recon == 0) return flux_dir<0, 0>(g, p, dir, W, U, F, s);
    if (recon == 1) return flux_dir<1, 0>(g, p, dir, W, U, F, s);
    return flux_dir<2, 0>(g, p, dir, W, U, F, s);
}

hipError_t launch_mhd_edges(const Geo& g, const double* W, const double* F, double* E,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_mhd_edges, dim3(blocks_for(g.n)), dim3(kBlock), 0, s, g, W, F, E);
    return hipGetLastError();
}

hipError_t launch_mhd_update(const Geo& g, const MhdParams& p, const double* in,
                             const double* base, const double* F, const double* E,
                             double* out, StageCoef coef, hipStream_t s)
{
    hipLaunchKernelGGL(k_mhd_update, dim3(blocks_for(g.n)), dim3(kBlock), 0, s, g, p, in, base,
                       F, E, out, coef);
    return hipGetLastError();
}

}  // namespace mhd
