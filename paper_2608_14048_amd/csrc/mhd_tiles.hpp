// mhd_tiles.hpp -- the bodies of the two stage kernels of the CT-MHD update as device
// templates on the tile shape, shared by the single-grid kernels (mhd_fused.hip) and
// the batched meshblock kernels (batch.hip).
//
// FluxTile<RECON, RS, IN, R, TX, TY>: for each z plane of the tile's chunk the
//   primitives (floors applied, B_cc the mean of the two bounding faces) of the tile and
//   its x/y halo are staged once in LDS; the z stencil of each column lives in a
//   per-thread register window.  The Riemann problems (reconstruction of the face-frame
//   primitives (rho, v_n, v_t1, v_t2, p, B_t1, B_t2), HLLE or HLLD) are solved on every
//   face the tile's cells touch; their mass, momentum and energy fluxes meet in LDS and
//   the cell fields are updated in the same pass (flux divergence of eq. (fv_update),
//   sources, the two-register combination out = g0 in + g1 base + bdt L).  What the
//   edge EMFs need leaves the kernel: per face the mass flux and the two face values of
//   the electric field (E_t1 = F(B_t2), E_t2 = -F(B_t1)), per cell E = -v x B.
//
// CtTile<CFL, IN, R, TX, TY>: per plane the Gardiner-Stone upwind edge EMFs E_z of the
//   plane and E_x, E_y of the level above are built in LDS from the face values, the
//   cell field and the mass-flux signs; the faces are updated with -curl E of eq. (ct)
//   in the same two-register form.  With CFL the time step of eq. (cfl) is taken over
//   the updated state in the same pass (the updated right-hand faces needed for B_cc
//   come from the same edge values; the cell fields from the flux/update kernel).
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

#include <type_traits>

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

// The stored values of one cell that its primitives need: the cell fields and the two
// bounding faces of each direction.  All eleven loads are issued before any of the
// arithmetic that uses them (measured: the FP64 donor-cell flux kernel 1.55 -> 1.34 ms
// per launch at 256^3 against loads interleaved with the primitive recovery).
template <class R>
struct Raw {
    R rho, m[3], b[3], bh[3];
    double E;
};

template <class R>
__device__ __forceinline__ Raw<R> load_raw(const Geo& g, const RegView<R>& U, int x, int y, int z)
{
    const unsigned int c = ((unsigned int)z * (unsigned int)g.ny + (unsigned int)y) * (unsigned int)g.nx + x;
    const unsigned int cx = x + 1 == g.nx ? c - x : c + 1;
    const unsigned int cy = y + 1 == g.ny ? c - (unsigned int)y * g.nx : c + g.nx;
    const unsigned int cz = z + 1 == g.nz ? c - (unsigned int)z * g.nx * g.ny : c + (unsigned int)g.nx * g.ny;
    Raw<R> r;
    r.b[0] = ldT(U.b[0], c); r.bh[0] = ldT(U.b[0], cx);
    r.b[1] = ldT(U.b[1], c); r.bh[1] = ldT(U.b[1], cy);
    r.b[2] = ldT(U.b[2], c); r.bh[2] = ldT(U.b[2], cz);
    r.rho = ldT(U.rho, c);
    r.m[0] = ldT(U.m[0], c); r.m[1] = ldT(U.m[1], c); r.m[2] = ldT(U.m[2], c);
    r.E = ldT(U.E, c);
    return r;
}

template <class R>
__device__ __forceinline__ Prim8<R> prims_of(const MhdParams& P, const Raw<R>& r)
{
    // explicit roundings only: the same cell gives the same primitives at every call site
#pragma clang fp contract(off)
    Prim8<R> w;
    w.bx = R(0.5) * (r.b[0] + r.bh[0]);
    w.by = R(0.5) * (r.b[1] + r.bh[1]);
    w.bz = R(0.5) * (r.b[2] + r.bh[2]);
    R d = r.rho;
    if (d < R(P.rho_floor)) d = R(P.rho_floor);
    w.d = d;
    const R id = rcp(d);
    w.vx = r.m[0] * id;
    w.vy = r.m[1] * id;
    w.vz = r.m[2] * id;
    // pressure from the total energy in FP64
    const double dd = d, vx = w.vx, vy = w.vy, vz = w.vz, bx = w.bx, by = w.by, bz = w.bz;
    const double ke = 0.5 * dd * ((vx * vx + vy * vy) + vz * vz);
    const double me = 0.5 * ((bx * bx + by * by) + bz * bz);
    double pr = (P.gamma - 1.0) * ((r.E - ke) - me);
    if (pr < P.p_floor) pr = P.p_floor;
    w.p = R(pr);
    return w;
}

template <class R>
__device__ __forceinline__ Prim8<R> load_prims(const Geo& g, const MhdParams& P, const RegView<R>& U,
                                               int x, int y, int z)
{
    return prims_of(P, load_raw(g, U, x, y, z));
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
// push(ak, a) takes the value of plane k (loaded again rather than carried in
// registers) and the value of plane k + AHEAD, and returns the two states on the face
// k - 1/2.
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

// The PPM pipeline without the value of plane k + 1 among its state: push takes it
// beside that of plane k + 2 (loaded again rather than carried, for the FP64 kernel,
// whose third wave per SIMD needs the registers).  The same arithmetic as ZPipe<2>.
template <class R>
struct ZPipeLean {
    static constexpr int AHEAD = 2, PRIME = 5;  // planes k0-3 .. k0+1
    R m0, ilo, apl;  // slope(k), a_{k-1/2}, a_+(k-1)
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
        m0 = s3;
    }
    __device__ void push(R ak, R a1, R a, R& aL, R& aR)
    {
        const R m1 = cw_slope(ak, a1, a);         // slope of cell k+1
        R lo = ilo;
        R hi = cw_interface(ak, a1, m0, m1);      // a_{k+1/2}
        ilo = hi;
        cw_limit(ak, lo, hi);                     // cell k
        aL = apl;
        aR = lo;
        apl = hi;
        m0 = m1;
    }
};

// Stage-kernel arguments: fluxes of `in`; out = g0 in + g1 base + bdt L(in) for the
// cell fields (rho, M, E), written by FluxTile; the face fields are updated by CtTile
// from the edge EMFs that the face values written to F and Rc give.
template <class R>
struct StageArgs {
    RegView<R> in;    // stage input register
    RegView<R> base;  // second register; may equal in, never out
    RegView<R> out;   // distinct from in and base
    R* F;             // 9 face fields: x (mass flux, E_y, E_z), y (mass flux, E_z, E_x),
                      // z (mass flux, E_x, E_y), each face with the cell on its high side
    R* Rc;            // 3 cell fields E = -v x B
    StageCoef co;
};

// Field q of the 9 face fields F (direction-major).
enum FaceField { FX_MASS = 0, FX_EY, FX_EZ, FY_MASS, FY_EZ, FY_EX, FZ_MASS, FZ_EX, FZ_EY, NFACE };

// One tile of the flux/update kernel: TX x TY cells of every plane k0 <= k < k1 (the tile
// may reach past the grid edge).  Threads: TX * TY, lanes along x first.  Per plane:
//  - the primitives of the tile and its x/y halo are staged in LDS (one more column and
//    row on the high side than the cells need: the tile's high faces);
//  - every thread solves its cell's low x, y and z faces (the z stencil is a register
//    pipeline fed one plane ahead); TX + TY threads of one or two waves, a different
//    group on each plane, also solve the tile's high faces (the row above it, the
//    column right of it);
//  - the faces' mass, momentum and energy fluxes meet in LDS, and every cell gets the
//    flux divergence of eq. (fv_update) plus sources and the stage combination, in the
//    same arithmetic as a separate update pass would use;
//  - the face values of E and the mass fluxes the edge EMFs need go to F, E = -v x B of
//    the cell to Rc.
template <int RECON, int RS, bool IN, class R, int TX, int TY>
struct FluxTile {
    static constexpr int SL = Stencil<RECON>::L, SR = Stencil<RECON>::R;
    static constexpr int LX = TX + SL + SR + 1, LY = TY + SL + SR + 1;
    static constexpr int NT = TX * TY, NR = TX + TY, NW = NT / 64;
    static_assert(NT % 64 == 0 && (NW & (NW - 1)) == 0, "whole wavefronts, a power of two of them");
    static_assert(NR <= NT, "the tile's high faces need TX + TY threads");
    // FP64 PPM: keep the compiler from hoisting the stencil loads of every variable
    // ahead of the reconstructions (it would hold them all in registers at once)
    static constexpr bool kFence = RECON == 2 && sizeof(R) == 8;
    // FP64 PPM: the z pipeline reloads plane k + 1 instead of carrying it, and the x/y
    // part of a cell's flux divergence is read from LDS when the cell is completed (one
    // more barrier per plane) instead of being carried to the next pass: 24 fewer
    // registers, which lets the kernel run three waves per SIMD
    static constexpr bool kLean = RECON == 2 && sizeof(R) == 8;
    struct Lds {
        R sw[8][LY][LX];         // primitives of the plane
        R hx[5][TY][TX + 1];     // fluxes through the x faces of the plane's rows
        R hy[5][TY + 1][TX];     // fluxes through the y faces of the plane's columns
    };

    // Face states of the seven face-frame variables from a stencil line in LDS: `at(v, s)`
    // gives staged variable v at offset s from the face's high-side cell.
    template <class At>
    __device__ static void recon7(const int comp[7], At at, Prim7<R>& L, Prim7<R>& Rt)
    {
        R* lr[7][2] = {{&L.d, &Rt.d}, {&L.vn, &Rt.vn}, {&L.vt1, &Rt.vt1}, {&L.vt2, &Rt.vt2},
                       {&L.p, &Rt.p}, {&L.bt1, &Rt.bt1}, {&L.bt2, &Rt.bt2}};
        R st[6];
    #pragma unroll
        for (int v = 0; v < 7; ++v) {
    #pragma unroll
            for (int s = -SL; s <= SR; ++s) st[3 + s] = at(comp[v], s);
            face_states<RECON>(st, *lr[v][0], *lr[v][1]);
            if constexpr (kFence) __builtin_amdgcn_sched_barrier(0);
        }
    }

    __device__ static void run(const Geo& g, const MhdParams& P, const StageArgs<R>& a, int x0, int y0,
                               int k0, int k1, Lds& lds)
    {
        using Pipe = std::conditional_t<kLean, ZPipeLean<R>, ZPipe<RECON, R>>;
        auto& sw = lds.sw;
        const int lane = (int)threadIdx.x % TX, row = (int)threadIdx.x / TX;
        const int i = x0 + lane, j = y0 + row;
        const bool live = i < g.nx && j < g.ny;
        // this thread's cell, taken periodically (a lane or row just past the grid edge
        // owns the face at the edge, which is the face at 0)
        const int ic = wrap_any(i, g.nx), jc = wrap_any(j, g.ny);
        // the low faces this thread solves: those of live rows/columns and the grid's
        // high edge when the tile reaches past it
        const bool xneed = i <= g.nx && j < g.ny;
        const bool yneed = j <= g.ny && i < g.nx;
        const long long n = g.n;
        const unsigned int nx = g.nx, plane = (unsigned int)g.nx * (unsigned int)g.ny;
        R* Fo[NFACE];
    #pragma unroll
        for (int q = 0; q < NFACE; ++q) Fo[q] = a.F + q * n;
        const int wave = (int)threadIdx.x / 64, wl = (int)threadIdx.x % 64;

        // z pipeline of the face-frame variables (rho, v_z, v_x, v_y, p, B_x, B_y); plane
        // k's own values come from the staged plane (a direct load on the last pass)
        Pipe zp[7];
        {
            R pre[7][Pipe::PRIME];
    #pragma unroll
            for (int s = 0; s < Pipe::PRIME; ++s) {
                const Prim8<R> w = load_prims(g, P, a.in, ic, jc, wrap_any(k0 - Pipe::PRIME + Pipe::AHEAD + s, g.nz));
                pre[0][s] = w.d; pre[1][s] = w.vz; pre[2][s] = w.vx; pre[3][s] = w.vy;
                pre[4][s] = w.p; pre[5][s] = w.bx; pre[6][s] = w.by;
            }
    #pragma unroll
            for (int v = 0; v < 7; ++v) zp[v].prime(pre[v]);
        }
        const double bdt = a.co.bdt, g0 = a.co.g0, g1 = a.co.g1;
        const R bdtr = R(bdt), g0r = R(g0), g1r = R(g1);
        const R idx = R(g.inv_dx[0]), idy = R(g.inv_dx[1]), idz = R(g.inv_dx[2]);
        // carried from one plane to the next: the x/y part of the flux divergence of the
        // cell below (mass and momenta in R, energy in FP64) and the z flux through its
        // low face (mass, M_x, M_y, M_z, E)
        R acc[kLean ? 1 : 4], fzp[5];
        double accE = 0.0;
    #pragma unroll
        for (int v = 0; v < (kLean ? 1 : 4); ++v) acc[v] = R(0);
    #pragma unroll
        for (int v = 0; v < 5; ++v) fzp[v] = R(0);

        // pass k solves the z face k - 1/2 and completes the cell of plane k - 1, then
        // (k < k1) solves the x and y faces of plane k; the pass k = k1 only completes
        // the chunk's last cell
        for (int k = k0; k <= k1; ++k) {
            const bool full = k < k1;
            Prim8<R> wk{}, wz{}, wz1{};
            if (full) {
                // stage the primitives of plane k (tile + x/y halos, corners skipped); the
                // staging waves get issue priority so their loads go out ahead of the
                // arithmetic of the other workgroups on the CU
                __builtin_amdgcn_s_setprio(1);
                for (int t = threadIdx.x; t < LX * LY; t += NT) {
                    const int r = t / LX, cc = t - r * LX;
                    const bool xh = cc < SL || cc >= SL + TX, yh = r < SL || r >= SL + TY;
                    if (xh && yh) continue;
                    const int gx = wrap_any(x0 + cc - SL, g.nx), gy = wrap_any(y0 + r - SL, g.ny);
                    const Prim8<R> w = load_prims(g, P, a.in, gx, gy, k);
                    sw[0][r][cc] = w.d; sw[1][r][cc] = w.vx; sw[2][r][cc] = w.vy; sw[3][r][cc] = w.vz;
                    sw[4][r][cc] = w.p; sw[5][r][cc] = w.bx; sw[6][r][cc] = w.by; sw[7][r][cc] = w.bz;
                }
            } else if constexpr (RECON != 1) {
                wk = load_prims(g, P, a.in, ic, jc, wrap_any(k, g.nz));
            }
            // newest plane of the z pipeline (donor cell needs none beyond plane k)
            if constexpr (Pipe::AHEAD > 0) wz = load_prims(g, P, a.in, ic, jc, wrap_any(k + Pipe::AHEAD, g.nz));
            if constexpr (kLean) wz1 = load_prims(g, P, a.in, ic, jc, wrap_any(k + 1, g.nz));
            if (full) {
                __syncthreads();
                __builtin_amdgcn_s_setprio(0);
            }

            const unsigned int kk = (unsigned int)(k < g.nz ? k : k - g.nz);
            const unsigned int c = kk * plane + (unsigned int)jc * nx + (unsigned int)ic;
            Prim7<R> L, Rt;
            Flux7<R> f;
            // ---- z face k - 1/2 from the pipeline: (rho, vz, vx, vy, p, Bx, By)
            {
                const int r0 = row + SL, c0 = lane + SL;
                auto push = [&](Pipe& zpv, R ak, R a1, R a2, R& l, R& r) {
                    if constexpr (kLean)
                        zpv.push(ak, a1, a2, l, r);
                    else
                        zpv.push(ak, a2, l, r);
                };
                push(zp[0], full ? sw[0][r0][c0] : wk.d, wz1.d, wz.d, L.d, Rt.d);
                push(zp[1], full ? sw[3][r0][c0] : wk.vz, wz1.vz, wz.vz, L.vn, Rt.vn);
                push(zp[2], full ? sw[1][r0][c0] : wk.vx, wz1.vx, wz.vx, L.vt1, Rt.vt1);
                push(zp[3], full ? sw[2][r0][c0] : wk.vy, wz1.vy, wz.vy, L.vt2, Rt.vt2);
                push(zp[4], full ? sw[4][r0][c0] : wk.p, wz1.p, wz.p, L.p, Rt.p);
                push(zp[5], full ? sw[5][r0][c0] : wk.bx, wz1.bx, wz.bx, L.bt1, Rt.bt1);
                push(zp[6], full ? sw[6][r0][c0] : wk.by, wz1.by, wz.by, L.bt2, Rt.bt2);
            }
            if (live) {
                solve<RS>(L, Rt, ldT(a.in.b[2], c), P, f);
                const R fz[5] = {f.d, f.mt1, f.mt2, f.mn, f.e};
                // the face's E values and mass flux, stored with the cell above it (the
                // chunk's first face is stored by the chunk below, as its last)
                if (k > k0) {
    #pragma clang fp contract(off)
                    stT(Fo[FZ_MASS], c, f.d); stT(Fo[FZ_EX], c, f.bt2); stT(Fo[FZ_EY], c, -f.bt1);
                    // ---- the cell of plane k - 1: flux divergence (density and momenta
                    // in R, energy in FP64), sources of a constant gas acceleration, the
                    // stage combination
                    const unsigned int cb = (unsigned int)(k - 1) * plane + (unsigned int)jc * nx + (unsigned int)ic;
                    R Lc[4];
                    double LE;
                    if constexpr (kLean) {
                        // the x/y part from the fluxes of plane k - 1, still in LDS (the
                        // same expressions as the carried form)
    #pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const R fx = (lds.hx[v][row][lane + 1] - lds.hx[v][row][lane]) * idx;
                            const R fy = (lds.hy[v][row + 1][lane] - lds.hy[v][row][lane]) * idy;
                            const R axy = fx + fy;
                            Lc[v] = -(axy + (fz[v] - fzp[v]) * idz);
                        }
                        const double fx = ((double)lds.hx[4][row][lane + 1] - (double)lds.hx[4][row][lane]) * g.inv_dx[0];
                        const double fy = ((double)lds.hy[4][row + 1][lane] - (double)lds.hy[4][row][lane]) * g.inv_dx[1];
                        const double axyE = fx + fy;
                        LE = -(axyE + ((double)fz[4] - (double)fzp[4]) * g.inv_dx[2]);
                    } else {
    #pragma unroll
                        for (int v = 0; v < 4; ++v) Lc[v] = -(acc[v] + (fz[v] - fzp[v]) * idz);
                        LE = -(accE + ((double)fz[4] - (double)fzp[4]) * g.inv_dx[2]);
                    }
                    R o[4];
                    double oE;
                    if (IN) {
                        const R rho_in = ldT(a.in.rho, cb);
                        const R m_in[3] = {ldT(a.in.m[0], cb), ldT(a.in.m[1], cb), ldT(a.in.m[2], cb)};
                        Lc[1] += rho_in * R(P.gacc[0]);
                        Lc[2] += rho_in * R(P.gacc[1]);
                        Lc[3] += rho_in * R(P.gacc[2]);
                        LE += ((double)m_in[0] * P.gacc[0] + (double)m_in[1] * P.gacc[1]) + (double)m_in[2] * P.gacc[2];
                        o[0] = (g0r * rho_in + g1r * ldT(a.base.rho, cb)) + bdtr * Lc[0];
    #pragma unroll
                        for (int v = 0; v < 3; ++v) o[1 + v] = (g0r * m_in[v] + g1r * ldT(a.base.m[v], cb)) + bdtr * Lc[1 + v];
                        oE = (g0 * ldT(a.in.E, cb) + g1 * ldT(a.base.E, cb)) + bdt * LE;
                    } else {
                        o[0] = g1r * ldT(a.base.rho, cb) + bdtr * Lc[0];
    #pragma unroll
                        for (int v = 0; v < 3; ++v) o[1 + v] = g1r * ldT(a.base.m[v], cb) + bdtr * Lc[1 + v];
                        oE = g1 * ldT(a.base.E, cb) + bdt * LE;
                    }
                    // out never aliases in or base (the host rotates three registers)
                    stT(a.out.rho, cb, o[0]);
    #pragma unroll
                    for (int v = 0; v < 3; ++v) stT(a.out.m[v], cb, o[1 + v]);
                    stT(a.out.E, cb, oE);
                }
    #pragma unroll
                for (int v = 0; v < 5; ++v) fzp[v] = fz[v];
            }
            if (!full) break;
            // lean form: every thread has read the fluxes of plane k - 1 before any
            // thread overwrites them with those of plane k
            if constexpr (kLean) __syncthreads();
            if constexpr (kFence) __builtin_amdgcn_sched_barrier(0);
            // ---- x face (low face of the cell): (rho, vx, vy, vz, p, By, Bz)
            if (xneed) {
                const int comp[7] = {0, 1, 2, 3, 4, 6, 7};
                recon7(comp, [&](int v, int s) { return sw[v][row + SL][lane + SL + s]; }, L, Rt);
                solve<RS>(L, Rt, ldT(a.in.b[0], c), P, f);
                lds.hx[0][row][lane] = f.d; lds.hx[1][row][lane] = f.mn; lds.hx[2][row][lane] = f.mt1;
                lds.hx[3][row][lane] = f.mt2; lds.hx[4][row][lane] = f.e;
                if (live) {
                    stT(Fo[FX_MASS], c, f.d); stT(Fo[FX_EY], c, f.bt2); stT(Fo[FX_EZ], c, -f.bt1);
                }
                if constexpr (kFence) __builtin_amdgcn_sched_barrier(0);
            }
            // ---- y face: (rho, vy, vz, vx, p, Bz, Bx)
            if (yneed) {
                const int comp[7] = {0, 2, 3, 1, 4, 7, 5};
                recon7(comp, [&](int v, int s) { return sw[v][row + SL + s][lane + SL]; }, L, Rt);
                solve<RS>(L, Rt, ldT(a.in.b[1], c), P, f);
                lds.hy[0][row][lane] = f.d; lds.hy[1][row][lane] = f.mt2; lds.hy[2][row][lane] = f.mn;
                lds.hy[3][row][lane] = f.mt1; lds.hy[4][row][lane] = f.e;
                if (live) {
                    stT(Fo[FY_MASS], c, f.d); stT(Fo[FY_EZ], c, f.bt2); stT(Fo[FY_EX], c, -f.bt1);
                }
                if constexpr (kFence) __builtin_amdgcn_sched_barrier(0);
            }
            // ---- cell field E = -v x B (rounded as written, as is every expression that
            // pairs x and y terms, so that the step keeps the swap of x and y exact)
            if (live) {
    #pragma clang fp contract(off)
                const R vx = sw[1][row + SL][lane + SL], vy = sw[2][row + SL][lane + SL];
                const R vz = sw[3][row + SL][lane + SL], bx = sw[5][row + SL][lane + SL];
                const R by = sw[6][row + SL][lane + SL], bz = sw[7][row + SL][lane + SL];
                stT(a.Rc, c, vz * by - vy * bz);
                stT(a.Rc + n, c, vx * bz - vz * bx);
                stT(a.Rc + 2 * n, c, vy * bx - vx * by);
            }
            // ---- the tile's high faces (fluxes only: their E values belong to the
            // neighbouring tile's cells): ring slot q < TX is the y face above column q,
            // TX <= q < TX + TY the x face right of row q - TX.  The slots go to
            // consecutive waves starting from one that changes from plane to plane in
            // FP64 (no wave carries them every time), and both directions share one code path
            // (stencil line, variable order and flux order picked per lane), so a wave
            // solves its ring faces in one pass whatever their direction.
            {
                const int turn = sizeof(R) == 8 ? k - k0 : 0;  // (FP32 measured faster without)
                const int rs = ((wave - turn) & (NW - 1)) * 64 + wl;
                const bool ry = rs < TX;
                const int rq = ry ? rs : rs - TX;
                const bool rneed = ry ? (y0 + TY <= g.ny && x0 + rq < g.nx)
                                      : (rs < NR && x0 + TX <= g.nx && y0 + rq < g.ny);
                if (rneed) {
                    // a tile reaching the grid's high edge owns the faces at 0
                    const int rxc = ry ? x0 + rq : wrap_once(x0 + TX, g.nx);
                    const int ryc = ry ? wrap_once(y0 + TY, g.ny) : y0 + rq;
                    const unsigned int cr = (unsigned int)k * plane + (unsigned int)ryc * nx + (unsigned int)rxc;
                    constexpr int cy[7] = {0, 2, 3, 1, 4, 7, 5}, cx[7] = {0, 1, 2, 3, 4, 6, 7};
                    int comp[7];
    #pragma unroll
                    for (int v = 0; v < 7; ++v) comp[v] = ry ? cy[v] : cx[v];
                    const int base = ry ? (TY + SL) * LX + rq + SL : (rq + SL) * LX + TX + SL;
                    const int stride = ry ? LX : 1;
                    const R* swf = &sw[0][0][0];
                    recon7(comp, [&](int v, int s) { return swf[v * (LY * LX) + base + s * stride]; }, L, Rt);
                    solve<RS>(L, Rt, ldT(ry ? a.in.b[1] : a.in.b[0], cr), P, f);
                    if (ry) {
                        lds.hy[0][TY][rq] = f.d; lds.hy[1][TY][rq] = f.mt2; lds.hy[2][TY][rq] = f.mn;
                        lds.hy[3][TY][rq] = f.mt1; lds.hy[4][TY][rq] = f.e;
                    } else {
                        lds.hx[0][rq][TX] = f.d; lds.hx[1][rq][TX] = f.mn; lds.hx[2][rq][TX] = f.mt1;
                        lds.hx[3][rq][TX] = f.mt2; lds.hx[4][rq][TX] = f.e;
                    }
                }
            }
            __syncthreads();
            // ---- the x/y part of this cell's flux divergence, carried to the next pass
            if constexpr (!kLean) {
                if (live) {
    #pragma clang fp contract(off)
    #pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const R fx = (lds.hx[v][row][lane + 1] - lds.hx[v][row][lane]) * idx;
                        const R fy = (lds.hy[v][row + 1][lane] - lds.hy[v][row][lane]) * idy;
                        acc[v] = fx + fy;
                    }
                    const double fx = ((double)lds.hx[4][row][lane + 1] - (double)lds.hx[4][row][lane]) * g.inv_dx[0];
                    const double fy = ((double)lds.hy[4][row + 1][lane] - (double)lds.hy[4][row][lane]) * g.inv_dx[1];
                    accE = fx + fy;
                }
            }
            // no barrier here: the next plane's staging writes only the primitives, which
            // every thread finished reading before the barrier above, and the fluxes are
            // rewritten only after the next barrier
        }
    }
};

// Occupancy requests (waves per SIMD): four for every FP32 kernel (at most 128
// registers), two for the FP64 PLM + HLLD kernel, three for the other FP64 kernels.
// The FP64 PPM kernels reach three (168 registers) only in their reload form (see
// FluxTile::kLean): the carried form held to three spilled about 36 dwords per lane and
// ran 20 % slower (3.48 against 2.91 ms per corrector launch at 256^3), the reload form
// spills six loop-invariant dwords and runs 2.51 against 2.67 ms.
template <int RECON, int RS, class R>
struct FluxWaves {
    static constexpr int min = sizeof(R) == 4 ? 4 : (RS == 1 && RECON == 1 ? 2 : 3);
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
    const R* F;          // the 9 face fields of FaceField
    const R* Rc;         // 3 cell E fields
    RegView<R> out;      // distinct from in and base; its cell fields are already updated
    double* partial;     // CFL partial minima, one per workgroup
    StageCoef co;
};

// One tile of the CT kernel (TX x TY cells, planes k0 <= k < k1); returns this thread's
// CFL minimum of the updated state (INFINITY unless CFL).  CFL: reduce the time step of
// the output (its cell fields come from the flux/update kernel of the same stage).  IN:
// the stage reads its input register's face fields (g0 != 0); otherwise only the base
// register's.
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
        const R* Fb[NFACE];
    #pragma unroll
        for (int q = 0; q < NFACE; ++q) Fb[q] = a.F + q * n;
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
            // p = x, q = y: X on x-faces, Y on y-faces
            return gs_edge(ldT(Fb[FX_EZ], c), ldT(Fb[FX_EZ], cy), ldT(Fb[FY_EZ], c), ldT(Fb[FY_EZ], cx),
                           ldT(Rz, c), ldT(Rz, cx), ldT(Rz, cy), ldT(Rz, cxy),
                           ldT(Fb[FX_MASS], c), ldT(Fb[FX_MASS], cy), ldT(Fb[FY_MASS], c), ldT(Fb[FY_MASS], cx));
        };
        // Level edges E_x, E_y at z-level zl - 1/2 for the tile (+1 ring on the high side).
        // A thread keeps the same edge positions on every level, so the values of plane
        // zl - 1 that a level needs are the plane-zl values the level below read: they
        // stay in registers (cx*, cy*) instead of coming back from memory, for the
        // first NC edge positions of the thread.  With CFL the updated B_z of the high
        // face (b3c) carries over to the plane above.  An FP64 kernel that also reduces
        // the time step on tiles taller than 4 rows carries nothing: at 512 threads the
        // extra registers would cost it half its occupancy, which it needs more.
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
                    // E_x at (x, y-1/2, z-1/2); p = y, q = z: X on y-faces, Y on z-faces
                    const int ym = wrap_once(wy - 1, g.ny);
                    const unsigned int c = at(wx, wy, zz), cy = at(wx, ym, zz);
                    const int mc = m < NA ? m : 0;
                    R Xm = cx13[mc], R0m = crx0[mc], Rmm = crxm[mc], fpm = cx7[mc];  // plane zl - 1
                    if (first || m >= NC) {
                        const unsigned int cz = at(wx, wy, zm), cyz = at(wx, ym, zm);
                        Xm = ldT(Fb[FY_EX], cz); R0m = ldT(Rx, cz);
                        Rmm = ldT(Rx, cyz); fpm = ldT(Fb[FY_MASS], cz);
                    }
                    const R X0 = ldT(Fb[FY_EX], c), R00 = ldT(Rx, c), Rm0 = ldT(Rx, cy), fp0 = ldT(Fb[FY_MASS], c);
                    sEx[slot][r][cc] = gs_edge(X0, Xm, ldT(Fb[FZ_EX], c), ldT(Fb[FZ_EX], cy), R00, Rm0, R0m, Rmm,
                                               fp0, fpm, ldT(Fb[FZ_MASS], c), ldT(Fb[FZ_MASS], cy));
                    if (m < NC) {
                        cx13[mc] = X0; crx0[mc] = R00; crxm[mc] = Rm0; cx7[mc] = fp0;
                    }
                }
                if (r < TY && gy < g.ny) {
                    // E_y at (x-1/2, y, z-1/2); p = z, q = x: X on z-faces, Y on x-faces
                    const int xm = wrap_once(wx - 1, g.nx);
                    const unsigned int c = at(wx, wy, zz), cx = at(xm, wy, zz);
                    const int mc = m < NA ? m : 0;
                    R Ym = cy5[mc], Rm0 = cry0[mc], Rmm = cryx[mc], fqm = cy0[mc];  // plane zl - 1
                    if (first || m >= NC) {
                        const unsigned int cz = at(wx, wy, zm), cxz = at(xm, wy, zm);
                        Ym = ldT(Fb[FX_EY], cz); Rm0 = ldT(Ry, cz);
                        Rmm = ldT(Ry, cxz); fqm = ldT(Fb[FX_MASS], cz);
                    }
                    const R Y0 = ldT(Fb[FX_EY], c), R00 = ldT(Ry, c), R0m = ldT(Ry, cx), fq0 = ldT(Fb[FX_MASS], c);
                    sEy[slot][r][cc] = gs_edge(ldT(Fb[FZ_EY], c), ldT(Fb[FZ_EY], cx), Y0, Ym, R00, Rm0, R0m, Rmm,
                                               ldT(Fb[FZ_MASS], c), ldT(Fb[FZ_MASS], cx), fq0, fqm);
                    if (m < NC) {
                        cy5[mc] = Y0; cry0[mc] = R00; cryx[mc] = R0m; cy0[mc] = fq0;
                    }
                }
            }
        };

        double vmin = INFINITY;
        int lv = 0;
        fill_level(lv ^ 1, k0, true);  // level k0 - 1/2
        R b3c = R(0);  // CFL: the updated B_z on the low face, from the plane below
        bool have_b3 = false;
        const R bdtr = R(a.co.bdt), g0r = R(a.co.g0), g1r = R(a.co.g1);
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
    #pragma clang fp contract(off)
                const int ip = i + 1 == g.nx ? 0 : i + 1, jp = j + 1 == g.ny ? 0 : j + 1;
                const int kp = k + 1 == g.nz ? 0 : k + 1;
                const unsigned int c = at(i, j, k), cx = at(ip, j, k), cy = at(i, jp, k), cz = at(i, j, kp);
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
                    double d = ldT(a.out.rho, c);
                    if (d < P.rho_floor) d = P.rho_floor;
                    const double id = rcp(d);
                    const double v[3] = {(double)ldT(a.out.m[0], c) * id, (double)ldT(a.out.m[1], c) * id,
                                         (double)ldT(a.out.m[2], c) * id};
                    const double ke = 0.5 * d * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
                    const double b2s = (bx * bx + by * by) + bz * bz;
                    double pr = (P.gamma - 1.0) * ((ldT(a.out.E, c) - ke) - 0.5 * b2s);
                    if (pr < P.p_floor) pr = P.p_floor;
                    const double bd[3] = {bx, by, bz};
    #pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        const double cf = fast_speed(P.gamma, d, pr, b2s, bd[q]);
                        vmin = min_nan(vmin, div_r(g.dx[q], fabs(v[q]) + cf));
                    }
                }
                // out never aliases in or base (the host rotates three registers)
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
