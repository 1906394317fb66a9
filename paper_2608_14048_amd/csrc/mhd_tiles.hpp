// mhd_tiles.hpp -- the bodies of the two stage kernels of the CT-MHD update as device
// templates on the tile shape, shared by the single-grid kernels (mhd_fused.hip) and
// the batched meshblock kernels (batch.hip).
//
// FluxTile<RECON, RS, R, TX, TY>: for each z plane of the tile's chunk the primitives
//   (floors applied, B_cc the mean of the two bounding faces) of the tile and its x/y
//   halo are staged once in LDS; the z stencil of each column lives in a per-thread
//   register window.  Every cell solves the Riemann problem on its three left faces
//   (x, y, z) -- reconstruction of the face-frame primitives (rho, v_n, v_t1, v_t2, p,
//   B_t1, B_t2), HLLE or HLLD -- and writes, per face, the mass, momentum and energy
//   fluxes in the global frame plus the two face values of the electric field
//   (E_t1 = F(B_t2), E_t2 = -F(B_t1)), and the cell-centred field E = -v x B.
//
// CtTile<CFL, IN, R, TX, TY>: per plane the Gardiner-Stone upwind edge EMFs E_z of the
//   plane and E_x, E_y of the level above are built in LDS from the face values, the
//   cell field and the mass-flux signs; the cell is updated with the flux divergence of
//   eq. (fv_update) plus sources, its faces with -curl E of eq. (ct), both in the
//   two-register form out = g0 in + g1 base + bdt L.  With CFL the time step of
//   eq. (cfl) is taken over the updated state in the same pass (the updated right-hand
//   faces needed for B_cc come from the same edge values).
//
// Precision: templated on the real type R.  R = double is the FP64 path.  R = float is
// the FP32-bulk form: density, momenta, face fields, reconstruction, Riemann solves, CT
// and the updates in FP32, while the total energy is stored in FP64 and both the
// pressure recovery p = (gamma-1)(E - kinetic - magnetic) and the energy update (from
// the FP32 fluxes) are done in FP64.
//
// Layout: every field is [nz][ny][nx], x fastest; lanes run along x so every global
// access is a contiguous row segment of TX elements.
#pragma once

#include "launch.hpp"
#include "physics.hpp"

namespace mhd {
namespace tiles {

// NaN-propagating minimum over the 64 lanes of a wavefront (valid in every lane).
__device__ __forceinline__ double wave_min64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min_nan(v, __shfl_xor(v, o, 64));
    return v;
}

// Blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous run of tiles
// so neighbouring tiles (which share halo rows) share an L2.
__device__ __forceinline__ unsigned int xcd_tile(unsigned int b, unsigned int nb)
{
    const unsigned int q = nb >> 3, rem = nb & 7u;
    const unsigned int x = b & 7u, r = b >> 3;
    return x * q + (x < rem ? x : rem) + r;
}

// Periodic index for offsets of one cell (valid for -n <= i < 2n).
__device__ __forceinline__ int wrap_once(int i, int n)
{
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Periodic index for any offset (halos of up to three cells on grids of any size).
__device__ __forceinline__ int wrap_any(int i, int n)
{
    if (i >= 0 && i < n) return i;
    const int r = i % n;
    return r < 0 ? r + n : r;
}

template <int RECON>
struct Stencil;
template <>
struct Stencil<0> {
    static constexpr int L = 1, R = 0;
};
template <>
struct Stencil<1> {
    static constexpr int L = 2, R = 1;
};
template <>
struct Stencil<2> {
    static constexpr int L = 3, R = 2;
};

template <class T>
__device__ __forceinline__ T ldT(const T* __restrict__ base, unsigned int idx)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (unsigned int)sizeof(T));
}
template <class T>
__device__ __forceinline__ void stT(T* base, unsigned int idx, T v)
{
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (unsigned int)sizeof(T)) = v;
}

// Primitives of cell (x, y, z) of the stage input (all indices already periodic).
template <class R>
struct Prim8 {
    R d, vx, vy, vz, p, bx, by, bz;
};

template <class R>
__device__ __forceinline__ Prim8<R> load_prims(const Geo& g, const MhdParams& P, const RegView<R>& U,
                                               int x, int y, int z)
{
    // explicit roundings only: the same cell gives the same primitives at every call site
#pragma clang fp contract(off)
    const unsigned int c = ((unsigned int)z * (unsigned int)g.ny + (unsigned int)y) * (unsigned int)g.nx + x;
    const unsigned int cx = x + 1 == g.nx ? c - x : c + 1;
    const unsigned int cy = y + 1 == g.ny ? c - (unsigned int)y * g.nx : c + g.nx;
    const unsigned int cz = z + 1 == g.nz ? c - (unsigned int)z * g.nx * g.ny : c + (unsigned int)g.nx * g.ny;
    Prim8<R> w;
    w.bx = R(0.5) * (ldT(U.b[0], c) + ldT(U.b[0], cx));
    w.by = R(0.5) * (ldT(U.b[1], c) + ldT(U.b[1], cy));
    w.bz = R(0.5) * (ldT(U.b[2], c) + ldT(U.b[2], cz));
    R d = ldT(U.rho, c);
    if (d < R(P.rho_floor)) d = R(P.rho_floor);
    w.d = d;
    const R id = rcp(d);
    w.vx = ldT(U.m[0], c) * id;
    w.vy = ldT(U.m[1], c) * id;
    w.vz = ldT(U.m[2], c) * id;
    // pressure from the total energy in FP64
    const double dd = d, vx = w.vx, vy = w.vy, vz = w.vz, bx = w.bx, by = w.by, bz = w.bz;
    const double ke = 0.5 * dd * ((vx * vx + vy * vy) + vz * vz);
    const double me = 0.5 * ((bx * bx + by * by) + bz * bz);
    double pr = (P.gamma - 1.0) * ((ldT(U.E, c) - ke) - me);
    if (pr < P.p_floor) pr = P.p_floor;
    w.p = R(pr);
    return w;
}

template <int RS, class R>
__device__ __forceinline__ void solve(const Prim7<R>& L, const Prim7<R>& Rt, R bn, const MhdParams& P,
                                      Flux7<R>& f)
{
    if (RS == 1)
        riemann_hlld(L, Rt, bn, R(P.gamma), R(P.gm1inv), R(P.hlld_eps), f);
    else
        riemann_hlle(L, Rt, bn, R(P.gamma), R(P.gm1inv), f);
}

// Reconstruction along z as a pipeline over the planes a column visits: each new plane
// costs one slope, one interface and one limiter (PPM), one slope (PLM) or nothing (DC).
// push(ak, a) takes the value of plane k (read back from the staged plane, so it is not
// carried in registers) and the value of plane k + AHEAD, and returns the two states on
// the face k - 1/2.
template <int RECON, class R>
struct ZPipe;

template <class R>
struct ZPipe<0, R> {
    static constexpr int AHEAD = 0, PRIME = 1;  // plane k0-1 before the march
    R prev;
    __device__ void prime(const R* a) { prev = a[0]; }
    __device__ void push(R ak, R, R& aL, R& aR)
    {
        aL = prev;
        aR = ak;
        prev = ak;
    }
};

// (PLM keeps its own copy of a(k): reading it back from the staged plane was measured
// slightly slower for this short pipeline.)
template <class R>
struct ZPipe<1, R> {
    static constexpr int AHEAD = 1, PRIME = 3;  // planes k0-2 .. k0
    R am, a0, apl;  // a(k-1), a(k), a_+(k-1)
    __device__ void prime(const R* a)
    {
        apl = fma_r(R(0.5), slope_vl(a[0], a[1], a[2]), a[1]);
        am = a[1];
        a0 = a[2];
    }
    __device__ void push(R, R a, R& aL, R& aR)
    {
        const R d = slope_vl(am, a0, a);
        aL = apl;
        aR = fma_r(R(-0.5), d, a0);
        apl = fma_r(R(0.5), d, a0);
        am = a0;
        a0 = a;
    }
};

template <class R>
struct ZPipe<2, R> {
    static constexpr int AHEAD = 2, PRIME = 5;  // planes k0-3 .. k0+1
    R a1, m0, ilo, apl;  // a(k+1), slope(k), a_{k-1/2}, a_+(k-1)
    __device__ void prime(const R* a)
    {
        const R s1 = cw_slope(a[0], a[1], a[2]);
        const R s2 = cw_slope(a[1], a[2], a[3]);
        const R s3 = cw_slope(a[2], a[3], a[4]);
        R lo = cw_interface(a[1], a[2], s1, s2);  // a_{k0-3/2}
        R hi = cw_interface(a[2], a[3], s2, s3);  // a_{k0-1/2}
        ilo = hi;
        cw_limit(a[2], lo, hi);                   // cell k0-1
        apl = hi;
        a1 = a[4];
        m0 = s3;
    }
    __device__ void push(R ak, R a, R& aL, R& aR)
    {
        const R m1 = cw_slope(ak, a1, a);         // slope of cell k+1
        R lo = ilo;
        R hi = cw_interface(ak, a1, m0, m1);      // a_{k+1/2}
        ilo = hi;
        cw_limit(ak, lo, hi);                     // cell k
        aL = apl;
        aR = lo;
        apl = hi;
        a1 = a;
        m0 = m1;
    }
};

// One tile of the flux kernel: TX x TY cells of every plane k0 <= k < k1 (the tile may
// reach past the grid edge; such cells only stage halos).  Threads: TX * TY, lanes
// along x first.
template <int RECON, int RS, class R, int TX, int TY>
struct FluxTile {
    static constexpr int SL = Stencil<RECON>::L, SR = Stencil<RECON>::R;
    static constexpr int LX = TX + SL + SR, LY = TY + SL + SR;
    // FP64 PPM: keep the compiler from hoisting the stencil loads of every variable
    // ahead of the reconstructions (it would hold them all in registers at once)
    static constexpr bool kFence = RECON == 2 && sizeof(R) == 8;
    struct Lds {
        R sw[8][LY][LX];
    };
    __device__ static void run(const Geo& g, const MhdParams& P, const RegView<R>& U, R* __restrict__ F,
                               R* __restrict__ Rc, int x0, int y0, int k0, int k1, Lds& lds)
    {
        using Pipe = ZPipe<RECON, R>;
        auto& sw = lds.sw;
        const int lane = (int)threadIdx.x % TX, row = (int)threadIdx.x / TX;
        const int i = x0 + lane, j = y0 + row;
        const bool live = i < g.nx && j < g.ny;
        const int ic = live ? i : 0, jc = live ? j : 0;
        const long long n = g.n;
        const unsigned int plane = (unsigned int)g.nx * (unsigned int)g.ny;
        R* Fo[21];
    #pragma unroll
        for (int q = 0; q < 21; ++q) Fo[q] = F + q * n;

        // z pipeline of the face-frame variables (rho, v_z, v_x, v_y, p, B_x, B_y)
        Pipe zp[7];
        {
            R pre[7][Pipe::PRIME];
    #pragma unroll
            for (int s = 0; s < Pipe::PRIME; ++s) {
                const Prim8<R> w = load_prims(g, P, U, ic, jc, wrap_any(k0 - Pipe::PRIME + Pipe::AHEAD + s, g.nz));
                pre[0][s] = w.d; pre[1][s] = w.vz; pre[2][s] = w.vx; pre[3][s] = w.vy;
                pre[4][s] = w.p; pre[5][s] = w.bx; pre[6][s] = w.by;
            }
    #pragma unroll
            for (int v = 0; v < 7; ++v) zp[v].prime(pre[v]);
        }

        for (int k = k0; k < k1; ++k) {
            // stage the primitives of plane k (tile + x/y halos, corners skipped); the
            // staging waves get issue priority so their loads go out ahead of the
            // arithmetic of the other workgroups on the CU
            __builtin_amdgcn_s_setprio(1);
            for (int q = threadIdx.x; q < LX * LY; q += TX * TY) {
                const int r = q / LX, cc = q - r * LX;
                const bool xh = cc < SL || cc >= SL + TX, yh = r < SL || r >= SL + TY;
                if (xh && yh) continue;
                const int gx = wrap_any(x0 + cc - SL, g.nx), gy = wrap_any(y0 + r - SL, g.ny);
                const Prim8<R> w = load_prims(g, P, U, gx, gy, k);
                sw[0][r][cc] = w.d; sw[1][r][cc] = w.vx; sw[2][r][cc] = w.vy; sw[3][r][cc] = w.vz;
                sw[4][r][cc] = w.p; sw[5][r][cc] = w.bx; sw[6][r][cc] = w.by; sw[7][r][cc] = w.bz;
            }
            // newest plane of the z pipeline (donor cell needs none beyond the staged one)
            Prim8<R> wz{};
            if constexpr (Pipe::AHEAD > 0) wz = load_prims(g, P, U, ic, jc, wrap_any(k + Pipe::AHEAD, g.nz));
            __syncthreads();
            __builtin_amdgcn_s_setprio(0);

            const unsigned int c = (unsigned int)k * plane + (unsigned int)jc * g.nx + ic;
            R st[6];
            Prim7<R> L, Rt;
            Flux7<R> f;
            // ---- z faces from the pipeline: (rho, vz, vx, vy, p, Bx, By)
            {
                const int r0 = row + SL, c0 = lane + SL;
                zp[0].push(sw[0][r0][c0], wz.d, L.d, Rt.d);
                zp[1].push(sw[3][r0][c0], wz.vz, L.vn, Rt.vn);
                zp[2].push(sw[1][r0][c0], wz.vx, L.vt1, Rt.vt1);
                zp[3].push(sw[2][r0][c0], wz.vy, L.vt2, Rt.vt2);
                zp[4].push(sw[4][r0][c0], wz.p, L.p, Rt.p);
                zp[5].push(sw[5][r0][c0], wz.bx, L.bt1, Rt.bt1);
                zp[6].push(sw[6][r0][c0], wz.by, L.bt2, Rt.bt2);
            }
            if (live) {
                solve<RS>(L, Rt, ldT(U.b[2], c), P, f);
                stT(Fo[14], c, f.d); stT(Fo[17], c, f.mn); stT(Fo[15], c, f.mt1); stT(Fo[16], c, f.mt2);
                stT(Fo[18], c, f.e); stT(Fo[19], c, f.bt2); stT(Fo[20], c, -f.bt1);
                if constexpr (kFence) __builtin_amdgcn_sched_barrier(0);
                // ---- x faces: (rho, vx, vy, vz, p, By, Bz)
                {
                    const int comp[7] = {0, 1, 2, 3, 4, 6, 7};
                    R* lr[7][2] = {{&L.d, &Rt.d}, {&L.vn, &Rt.vn}, {&L.vt1, &Rt.vt1}, {&L.vt2, &Rt.vt2},
                                   {&L.p, &Rt.p}, {&L.bt1, &Rt.bt1}, {&L.bt2, &Rt.bt2}};
    #pragma unroll
                    for (int v = 0; v < 7; ++v) {
    #pragma unroll
                        for (int s = -SL; s <= SR; ++s) st[3 + s] = sw[comp[v]][row + SL][lane + SL + s];
                        face_states<RECON>(st, *lr[v][0], *lr[v][1]);
                        if constexpr (kFence) __builtin_amdgcn_sched_barrier(0);
                    }
                    solve<RS>(L, Rt, ldT(U.b[0], c), P, f);
                    stT(Fo[0], c, f.d); stT(Fo[1], c, f.mn); stT(Fo[2], c, f.mt1); stT(Fo[3], c, f.mt2);
                    stT(Fo[4], c, f.e); stT(Fo[5], c, f.bt2); stT(Fo[6], c, -f.bt1);
                    if constexpr (kFence) __builtin_amdgcn_sched_barrier(0);
                }
                // ---- y faces: (rho, vy, vz, vx, p, Bz, Bx)
                {
                    const int comp[7] = {0, 2, 3, 1, 4, 7, 5};
                    R* lr[7][2] = {{&L.d, &Rt.d}, {&L.vn, &Rt.vn}, {&L.vt1, &Rt.vt1}, {&L.vt2, &Rt.vt2},
                                   {&L.p, &Rt.p}, {&L.bt1, &Rt.bt1}, {&L.bt2, &Rt.bt2}};
    #pragma unroll
                    for (int v = 0; v < 7; ++v) {
    #pragma unroll
                        for (int s = -SL; s <= SR; ++s) st[3 + s] = sw[comp[v]][row + SL + s][lane + SL];
                        face_states<RECON>(st, *lr[v][0], *lr[v][1]);
                        if constexpr (kFence) __builtin_amdgcn_sched_barrier(0);
                    }
                    solve<RS>(L, Rt, ldT(U.b[1], c), P, f);
                    stT(Fo[7], c, f.d); stT(Fo[9], c, f.mn); stT(Fo[10], c, f.mt1); stT(Fo[8], c, f.mt2);
                    stT(Fo[11], c, f.e); stT(Fo[12], c, f.bt2); stT(Fo[13], c, -f.bt1);
                }
                // ---- cell field E = -v x B
                {
                    const R vx = sw[1][row + SL][lane + SL], vy = sw[2][row + SL][lane + SL];
                    const R vz = sw[3][row + SL][lane + SL], bx = sw[5][row + SL][lane + SL];
                    const R by = sw[6][row + SL][lane + SL], bz = sw[7][row + SL][lane + SL];
                    stT(Rc, c, vz * by - vy * bz);
                    stT(Rc + n, c, vx * bz - vz * bx);
                    stT(Rc + 2 * n, c, vy * bx - vx * by);
                }
            }
            __syncthreads();
        }
    }
};

template <class R>
__device__ __forceinline__ R gs_upwind(R m, R pos, R neg)
{
    return m > R(0) ? pos : (m < R(0) ? neg : R(0.5) * (pos + neg));
}

// Gardiner-Stone edge value from the face values X (p-faces) and Y (q-faces), the cell
// field R at the four cells around the edge and the mass fluxes through the faces.
template <class R>
__device__ __forceinline__ R gs_edge(R X0, R Xm, R Y0, R Ym, R R00, R Rm0, R R0m, R Rmm, R fp0, R fpm,
                                     R fq0, R fqm)
{
    const R dqp = gs_upwind(fp0, Rm0 - Ym, R00 - Y0);
    const R dqm = gs_upwind(fpm, Ym - Rmm, Y0 - R0m);
    const R dpp = gs_upwind(fq0, R0m - Xm, R00 - X0);
    const R dpm = gs_upwind(fqm, Xm - Rmm, X0 - Rm0);
    return R(0.25) * (((X0 + Xm) + (Y0 + Ym)) - ((dqp - dqm) + (dpp - dpm)));
}

template <class R>
struct CtArgs {
    RegView<R> in;       // stage input register
    RegView<R> base;     // second register; may equal in, never out
    const R* F;          // 3 x 7 face fields
    const R* Rc;         // 3 cell E fields
    RegView<R> out;      // distinct from in and base
    double* partial;     // CFL partial minima, one per workgroup
    StageCoef co;
};

// One tile of the CT/update kernel (TX x TY cells, planes k0 <= k < k1); returns this
// thread's CFL minimum of the updated state (INFINITY unless CFL).  CFL: reduce the
// time step of the output.  IN: the stage reads its input register (g0 != 0 or a gas
// acceleration is set); otherwise only the base register is read.
template <bool CFL, bool IN, class R, int TX, int TY>
struct CtTile {
    // edges held for the tile: E_z on plane k, E_x / E_y on levels k-1/2 (slot lv^1)
    // and k+1/2 (slot lv); index ranges i in [0, TX], j in [0, TY]
    struct Lds {
        R sEz[TY + 1][TX + 1];
        R sEx[2][TY + 1][TX + 1];
        R sEy[2][TY + 1][TX + 1];
    };
    __device__ static double run(const Geo& g, const MhdParams& P, const CtArgs<R>& a, int x0, int y0,
                                 int k0, int k1, Lds& lds)
    {
        auto& sEz = lds.sEz;
        auto& sEx = lds.sEx;
        auto& sEy = lds.sEy;
        const int lane = (int)threadIdx.x % TX, row = (int)threadIdx.x / TX;
        const int i = x0 + lane, j = y0 + row;
        const bool live = i < g.nx && j < g.ny;
        const long long n = g.n;
        const unsigned int nx = g.nx, plane = (unsigned int)g.nx * (unsigned int)g.ny;
        const R* Fb[21];
    #pragma unroll
        for (int q = 0; q < 21; ++q) Fb[q] = a.F + q * n;
        const R* Rx = a.Rc;
        const R* Ry = a.Rc + n;
        const R* Rz = a.Rc + 2 * n;

        auto at = [&](int x, int y, int z) -> unsigned int {
            return (unsigned int)z * plane + (unsigned int)y * nx + (unsigned int)x;
        };
        // E_x at (x, y-1/2, z-1/2), E_y at (x-1/2, y, z-1/2), E_z at (x-1/2, y-1/2, z)
        auto edge_z = [&](int x, int y, int z) -> R {
            const int xm = wrap_once(x - 1, g.nx), ym = wrap_once(y - 1, g.ny);
            const unsigned int c = at(x, y, z), cx = at(xm, y, z), cy = at(x, ym, z), cxy = at(xm, ym, z);
            // p = x, q = y: X on x-faces (slot 6 of x), Y on y-faces (slot 5 of y)
            return gs_edge(ldT(Fb[6], c), ldT(Fb[6], cy), ldT(Fb[12], c), ldT(Fb[12], cx),
                           ldT(Rz, c), ldT(Rz, cx), ldT(Rz, cy), ldT(Rz, cxy),
                           ldT(Fb[0], c), ldT(Fb[0], cy), ldT(Fb[7], c), ldT(Fb[7], cx));
        };
        // Level edges E_x, E_y at z-level zl - 1/2 for the tile (+1 ring on the high side).
        // A thread keeps the same edge positions on every level, so the values of plane
        // zl - 1 that a level needs are the plane-zl values the level below read: they
        // stay in registers (cx*, cy*) instead of coming back from memory, for the
        // first NC edge positions of the thread.  Likewise the z fluxes of the high face
        // (fzc) and, with CFL, the updated B_z of the high face (b3c) carry over to the
        // plane above.  An FP64 kernel that also reduces the time step on tiles taller
        // than 4 rows carries nothing: at 512 threads the extra registers would cost it
        // half its occupancy, which it needs more.
        constexpr int NT = TX * TY, NE = (TX + 1) * (TY + 1), NQ = (NE + NT - 1) / NT;
        constexpr bool ZC = !(CFL && sizeof(R) == 8 && TY > 4);
        constexpr int NC = !ZC ? 0 : (sizeof(R) == 4 ? NQ : 1);
        constexpr int NA = NC > 0 ? NC : 1;
        R cx13[NA], cx7[NA], crx0[NA], crxm[NA], cy5[NA], cy0[NA], cry0[NA], cryx[NA];
    #pragma unroll
        for (int m = 0; m < NA; ++m) {
            cx13[m] = cx7[m] = crx0[m] = crxm[m] = R(0);
            cy5[m] = cy0[m] = cry0[m] = cryx[m] = R(0);
        }
        auto fill_level = [&](int slot, int zl, bool first) {
            const int zz = wrap_once(zl, g.nz), zm = wrap_once(zl - 1, g.nz);
    #pragma unroll
            for (int m = 0; m < NQ; ++m) {
                const int q = (int)threadIdx.x + m * NT;
                const int r = q / (TX + 1), cc = q - r * (TX + 1);
                const int gx = x0 + cc, gy = y0 + r;
                if (q >= NE || gx > g.nx || gy > g.ny) continue;
                const int wx = gx == g.nx ? 0 : gx, wy = gy == g.ny ? 0 : gy;
                if (cc < TX && gx < g.nx) {
                    // E_x at (x, y-1/2, z-1/2); p = y, q = z: X on y-faces (slot 6 of the
                    // y sweep), Y on z-faces (slot 5 of z)
                    const int ym = wrap_once(wy - 1, g.ny);
                    const unsigned int c = at(wx, wy, zz), cy = at(wx, ym, zz);
                    const int mc = m < NA ? m : 0;
                    R Xm = cx13[mc], R0m = crx0[mc], Rmm = crxm[mc], fpm = cx7[mc];  // plane zl - 1
                    if (first || m >= NC) {
                        const unsigned int cz = at(wx, wy, zm), cyz = at(wx, ym, zm);
                        Xm = ldT(Fb[13], cz); R0m = ldT(Rx, cz);
                        Rmm = ldT(Rx, cyz); fpm = ldT(Fb[7], cz);
                    }
                    const R X0 = ldT(Fb[13], c), R00 = ldT(Rx, c), Rm0 = ldT(Rx, cy), fp0 = ldT(Fb[7], c);
                    sEx[slot][r][cc] = gs_edge(X0, Xm, ldT(Fb[19], c), ldT(Fb[19], cy), R00, Rm0, R0m, Rmm, fp0,
                                               fpm, ldT(Fb[14], c), ldT(Fb[14], cy));
                    if (m < NC) {
                        cx13[mc] = X0; crx0[mc] = R00; crxm[mc] = Rm0; cx7[mc] = fp0;
                    }
                }
                if (r < TY && gy < g.ny) {
                    // E_y at (x-1/2, y, z-1/2); p = z, q = x: X on z-faces (slot 6 of z),
                    // Y on x-faces (slot 5 of x)
                    const int xm = wrap_once(wx - 1, g.nx);
                    const unsigned int c = at(wx, wy, zz), cx = at(xm, wy, zz);
                    const int mc = m < NA ? m : 0;
                    R Ym = cy5[mc], Rm0 = cry0[mc], Rmm = cryx[mc], fqm = cy0[mc];  // plane zl - 1
                    if (first || m >= NC) {
                        const unsigned int cz = at(wx, wy, zm), cxz = at(xm, wy, zm);
                        Ym = ldT(Fb[5], cz); Rm0 = ldT(Ry, cz);
                        Rmm = ldT(Ry, cxz); fqm = ldT(Fb[0], cz);
                    }
                    const R Y0 = ldT(Fb[5], c), R00 = ldT(Ry, c), R0m = ldT(Ry, cx), fq0 = ldT(Fb[0], c);
                    sEy[slot][r][cc] = gs_edge(ldT(Fb[20], c), ldT(Fb[20], cx), Y0, Ym, R00, Rm0, R0m, Rmm,
                                               ldT(Fb[14], c), ldT(Fb[14], cx), fq0, fqm);
                    if (m < NC) {
                        cy5[mc] = Y0; cry0[mc] = R00; cryx[mc] = R0m; cy0[mc] = fq0;
                    }
                }
            }
        };

        double vmin = INFINITY;
        int lv = 0;
        fill_level(lv ^ 1, k0, true);  // level k0 - 1/2
        // z fluxes on the low face of the current plane (the high face of the plane below)
        R fzc[5];
    #pragma unroll
        for (int v = 0; v < 5; ++v) fzc[v] = live && ZC ? ldT(Fb[14 + v], at(i, j, k0)) : R(0);
        R b3c = R(0);  // CFL: the updated B_z on the low face, from the plane below
        bool have_b3 = false;
        const double bdt = a.co.bdt, g0 = a.co.g0, g1 = a.co.g1;
        const R bdtr = R(bdt), g0r = R(g0), g1r = R(g1);
        const R idx = R(g.inv_dx[0]), idy = R(g.inv_dx[1]), idz = R(g.inv_dx[2]);

        for (int k = k0; k < k1; ++k) {
            // edges: E_z on plane k, E_x / E_y on level k + 1/2
            for (int q = threadIdx.x; q < (TX + 1) * (TY + 1); q += TX * TY) {
                const int r = q / (TX + 1), cc = q - r * (TX + 1);
                const int gx = x0 + cc, gy = y0 + r;
                if (gx > g.nx || gy > g.ny) continue;
                const int wx = gx == g.nx ? 0 : gx, wy = gy == g.ny ? 0 : gy;
                sEz[r][cc] = edge_z(wx, wy, k);
            }
            fill_level(lv, k + 1, false);
            __syncthreads();

            if (live) {
                const int ip = i + 1 == g.nx ? 0 : i + 1, jp = j + 1 == g.ny ? 0 : j + 1;
                const int kp = k + 1 == g.nz ? 0 : k + 1;
                const unsigned int c = at(i, j, k), cx = at(ip, j, k), cy = at(i, jp, k), cz = at(i, j, kp);
                // flux divergence: density and momenta in R, energy in FP64
                R L[4];
    #pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const R fzh = ldT(Fb[14 + v], cz);
                    if (!ZC) fzc[v] = ldT(Fb[14 + v], c);
                    const R fx = (ldT(Fb[v], cx) - ldT(Fb[v], c)) * idx;
                    const R fy = (ldT(Fb[7 + v], cy) - ldT(Fb[7 + v], c)) * idy;
                    const R fz = (fzh - fzc[v]) * idz;
                    L[v] = -((fx + fy) + fz);
                    fzc[v] = fzh;
                }
                double LE;
                {
                    const R fzh = ldT(Fb[18], cz);
                    if (!ZC) fzc[4] = ldT(Fb[18], c);
                    const double fx = ((double)ldT(Fb[4], cx) - (double)ldT(Fb[4], c)) * g.inv_dx[0];
                    const double fy = ((double)ldT(Fb[11], cy) - (double)ldT(Fb[11], c)) * g.inv_dx[1];
                    const double fz = ((double)fzh - (double)fzc[4]) * g.inv_dx[2];
                    LE = -((fx + fy) + fz);
                    fzc[4] = fzh;
                }
                R o[4];
                double oE;
                if (IN) {
                    const R rho_in = ldT(a.in.rho, c);
                    const R m_in[3] = {ldT(a.in.m[0], c), ldT(a.in.m[1], c), ldT(a.in.m[2], c)};
                    L[1] += rho_in * R(P.gacc[0]);
                    L[2] += rho_in * R(P.gacc[1]);
                    L[3] += rho_in * R(P.gacc[2]);
                    LE += ((double)m_in[0] * P.gacc[0] + (double)m_in[1] * P.gacc[1]) + (double)m_in[2] * P.gacc[2];
                    o[0] = (g0r * rho_in + g1r * ldT(a.base.rho, c)) + bdtr * L[0];
    #pragma unroll
                    for (int v = 0; v < 3; ++v) o[1 + v] = (g0r * m_in[v] + g1r * ldT(a.base.m[v], c)) + bdtr * L[1 + v];
                    oE = (g0 * ldT(a.in.E, c) + g1 * ldT(a.base.E, c)) + bdt * LE;
                } else {
                    o[0] = g1r * ldT(a.base.rho, c) + bdtr * L[0];
    #pragma unroll
                    for (int v = 0; v < 3; ++v) o[1 + v] = g1r * ldT(a.base.m[v], c) + bdtr * L[1 + v];
                    oE = g1 * ldT(a.base.E, c) + bdt * LE;
                }

                // faces of this cell: b1 at x_{i-1/2}, b2 at y_{j-1/2}, b3 at z_{k-1/2}
                const int ol = lv ^ 1, nl = lv;
                auto comb = [&](int comp, unsigned int cc, R lb) -> R {
                    return (IN ? g0r * ldT(a.in.b[comp], cc) + g1r * ldT(a.base.b[comp], cc)
                               : g1r * ldT(a.base.b[comp], cc)) + bdtr * lb;
                };
                auto nb1 = [&](int xl, unsigned int cc) {  // new B_x on the face at tile column xl
                    const R lb = -((sEz[row + 1][xl] - sEz[row][xl]) * idy - (sEy[nl][row][xl] - sEy[ol][row][xl]) * idz);
                    return comb(0, cc, lb);
                };
                auto nb2 = [&](int yl, unsigned int cc) {  // new B_y on the face at tile row yl
                    const R lb = -((sEx[nl][yl][lane] - sEx[ol][yl][lane]) * idz - (sEz[yl][lane + 1] - sEz[yl][lane]) * idx);
                    return comb(1, cc, lb);
                };
                auto nb3 = [&](int lvl, unsigned int cc) {  // new B_z on the z-face of level slot lvl
                    const R lb = -((sEy[lvl][row][lane + 1] - sEy[lvl][row][lane]) * idx -
                                   (sEx[lvl][row + 1][lane] - sEx[lvl][row][lane]) * idy);
                    return comb(2, cc, lb);
                };
                const R b1 = nb1(lane, c);
                const R b2 = nb2(row, c);
                const R b3 = CFL && ZC && have_b3 ? b3c : nb3(ol, c);
                if (CFL) {
                    // the updated faces on the high side give the new B_cc of this cell (FP64)
                    b3c = nb3(nl, cz);  // also the low face of the plane above
                    have_b3 = true;
                    const double bx = 0.5 * ((double)b1 + (double)nb1(lane + 1, cx));
                    const double by = 0.5 * ((double)b2 + (double)nb2(row + 1, cy));
                    const double bz = 0.5 * ((double)b3 + (double)b3c);
                    double d = o[0];
                    if (d < P.rho_floor) d = P.rho_floor;
                    const double id = rcp(d);
                    const double v[3] = {(double)o[1] * id, (double)o[2] * id, (double)o[3] * id};
                    const double ke = 0.5 * d * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
                    const double b2s = (bx * bx + by * by) + bz * bz;
                    double pr = (P.gamma - 1.0) * ((oE - ke) - 0.5 * b2s);
                    if (pr < P.p_floor) pr = P.p_floor;
                    const double bd[3] = {bx, by, bz};
    #pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const double cf = fast_speed(P.gamma, d, pr, b2s, bd[q]);
                        vmin = min_nan(vmin, div_r(g.dx[q], fabs(v[q]) + cf));
                    }
                }
                // out never aliases in or base (the host rotates three registers)
                stT(a.out.rho, c, o[0]);
    #pragma unroll
                for (int v = 0; v < 3; ++v) stT(a.out.m[v], c, o[1 + v]);
                stT(a.out.E, c, oE);
                stT(a.out.b[0], c, b1);
                stT(a.out.b[1], c, b2);
                stT(a.out.b[2], c, b3);
            }
            __syncthreads();
            lv ^= 1;
        }
        return vmin;
    }
};

}  // namespace tiles
}  // namespace mhd
