// mhd_fused.hip -- one stage of the CT-MHD update in two z-marching kernels.
//
// k_flux3<RECON, RS>   (one workgroup = a 64 x 4 tile of xy columns, marching a chunk
//   of z planes).  For each plane the primitives (floors applied, B_cc the mean of the
//   two bounding faces) of the tile and its x/y halo are staged once in LDS; the z
//   stencil of each column lives in a per-thread register window.  Every cell then
//   solves the Riemann problem on its three left faces (x, y, z) -- reconstruction of
//   the face-frame primitives (rho, v_n, v_t1, v_t2, p, B_t1, B_t2), HLLE or HLLD --
//   and writes, per face, the mass, momentum and energy fluxes in the global frame
//   plus the two face values of the electric field (E_t1 = F(B_t2), E_t2 = -F(B_t1)),
//   and the cell-centred field E = -v x B.
//
// k_ct_update<CFL>     (same tiling).  Per plane: the Gardiner-Stone upwind edge EMFs
//   E_z of the plane and E_x, E_y of the level above are built in LDS from the face
//   values, the cell field and the mass-flux signs; the cell is updated with the flux
//   divergence of eq. (fv_update) plus sources, its faces with -curl E of eq. (ct),
//   both in the two-register form out = g0 in + g1 base + bdt L.  In the last stage
//   the CFL minimum of eq. (cfl) is taken over the updated state in the same pass
//   (the updated right-hand faces needed for B_cc come from the same edge values).
//
// Layout: everything is [field][nz][ny][nx] FP64, x fastest; lanes of a wavefront run
// along x so every global access is a contiguous 512-byte row segment.
#include "launch.hpp"
#include "physics.hpp"

namespace mhd {

namespace {

constexpr int TX = 64;   // lanes along x
constexpr int TY = 4;    // waves along y (flux kernel)
constexpr int TY2 = 8;   // waves along y (CT/update kernel: one halo row per 8 rows)

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

// Uniform base pointers of the 8 fields of a state register.
struct Fields8 {
    const double* f[8];
};
__device__ __forceinline__ Fields8 fields8(const double* U, long long n)
{
    Fields8 r;
#pragma unroll
    for (int q = 0; q < 8; ++q) r.f[q] = U + q * n;
    return r;
}

// Primitives of cell (x, y, z) of the stage input (all indices already periodic).
struct Prim8 {
    double d, vx, vy, vz, p, bx, by, bz;
};

__device__ __forceinline__ Prim8 load_prims(const Geo& g, const MhdParams& P, const Fields8& U,
                                            int x, int y, int z)
{
    const unsigned int c = ((unsigned int)z * (unsigned int)g.ny + (unsigned int)y) * (unsigned int)g.nx + x;
    const unsigned int o = c * 8u;
    const unsigned int ox = (x + 1 == g.nx ? c - x : c + 1) * 8u;
    const unsigned int oy = (y + 1 == g.ny ? c - (unsigned int)y * g.nx : c + g.nx) * 8u;
    const unsigned int oz = (z + 1 == g.nz ? c - (unsigned int)z * g.nx * g.ny : c + (unsigned int)g.nx * g.ny) * 8u;
    Prim8 w;
    w.bx = 0.5 * (ld_at(U.f[5], o) + ld_at(U.f[5], ox));
    w.by = 0.5 * (ld_at(U.f[6], o) + ld_at(U.f[6], oy));
    w.bz = 0.5 * (ld_at(U.f[7], o) + ld_at(U.f[7], oz));
    double d = ld_at(U.f[0], o);
    if (d < P.rho_floor) d = P.rho_floor;
    w.d = d;
    const double id = 1.0 / d;
    w.vx = ld_at(U.f[1], o) * id;
    w.vy = ld_at(U.f[2], o) * id;
    w.vz = ld_at(U.f[3], o) * id;
    const double ke = 0.5 * d * ((w.vx * w.vx + w.vy * w.vy) + w.vz * w.vz);
    const double me = 0.5 * ((w.bx * w.bx + w.by * w.by) + w.bz * w.bz);
    double pr = (P.gamma - 1.0) * ((ld_at(U.f[4], o) - ke) - me);
    if (pr < P.p_floor) pr = P.p_floor;
    w.p = pr;
    return w;
}

template <int RS>
__device__ __forceinline__ void solve(const Prim7& L, const Prim7& R, double bn, const MhdParams& P,
                                      Flux7& f)
{
    if (RS == 1)
        riemann_hlld(L, R, bn, P.gamma, P.gm1inv, P.hlld_eps, f);
    else
        riemann_hlle(L, R, bn, P.gamma, P.gm1inv, f);
}

// Reconstruction along z as a pipeline over the planes a column visits: each new plane
// costs one slope, one interface and one limiter (PPM), one slope (PLM) or nothing (DC);
// push() returns the two states on the face k - 1/2 when plane k + AHEAD arrives.
template <int RECON>
struct ZPipe;

template <>
struct ZPipe<0> {
    static constexpr int AHEAD = 0, PRIME = 1;  // planes k0-1 .. k0-1 before the march
    double prev;
    __device__ void prime(const double* a) { prev = a[0]; }
    __device__ void push(double a, double& aL, double& aR)
    {
        aL = prev;
        aR = a;
        prev = a;
    }
};

template <>
struct ZPipe<1> {
    static constexpr int AHEAD = 1, PRIME = 3;  // planes k0-2 .. k0
    double am, a0, apl;  // a(k-1), a(k), a_+(k-1)
    __device__ void prime(const double* a)
    {
        apl = a[1] + 0.5 * slope_vl(a[0], a[1], a[2]);
        am = a[1];
        a0 = a[2];
    }
    __device__ void push(double a, double& aL, double& aR)
    {
        const double d = slope_vl(am, a0, a);
        aL = apl;
        aR = a0 - 0.5 * d;
        apl = a0 + 0.5 * d;
        am = a0;
        a0 = a;
    }
};

template <>
struct ZPipe<2> {
    static constexpr int AHEAD = 2, PRIME = 5;  // planes k0-3 .. k0+1
    double a0, a1, m0, ilo, apl;  // a(k), a(k+1), slope(k), a_{k-1/2}, a_+(k-1)
    __device__ void prime(const double* a)
    {
        const double s1 = cw_slope(a[0], a[1], a[2]);
        const double s2 = cw_slope(a[1], a[2], a[3]);
        const double s3 = cw_slope(a[2], a[3], a[4]);
        double lo = cw_interface(a[1], a[2], s1, s2);  // a_{k0-3/2}
        double hi = cw_interface(a[2], a[3], s2, s3);  // a_{k0-1/2}
        ilo = hi;
        cw_limit(a[2], lo, hi);                        // cell k0-1
        apl = hi;
        a0 = a[3];
        a1 = a[4];
        m0 = s3;
    }
    __device__ void push(double a, double& aL, double& aR)
    {
        const double m1 = cw_slope(a0, a1, a);         // slope of cell k+1
        double lo = ilo;
        double hi = cw_interface(a0, a1, m0, m1);      // a_{k+1/2}
        ilo = hi;
        cw_limit(a0, lo, hi);                          // cell k
        aL = apl;
        aR = lo;
        apl = hi;
        a0 = a1;
        a1 = a;
        m0 = m1;
    }
};

}  // namespace

// ----------------------------------------------------------------------------------
// K1: face fluxes of all three directions
// ----------------------------------------------------------------------------------

template <int RECON, int RS>
__global__ __launch_bounds__(TX* TY) void k_flux3(Geo g, MhdParams P, const double* __restrict__ Ub,
                                                 double* __restrict__ F, double* __restrict__ Rc,
                                                 int kz, unsigned int ntx, unsigned int nty,
                                                 unsigned int nblk)
{
    constexpr int SL = Stencil<RECON>::L, SR = Stencil<RECON>::R;
    constexpr int LX = TX + SL + SR, LY = TY + SL + SR;
    using Pipe = ZPipe<RECON>;
    __shared__ double sw[8][LY][LX];

    const unsigned int t = xcd_tile(blockIdx.x, nblk);
    const int x0 = (int)(t % ntx) * TX;
    const int y0 = (int)((t / ntx) % nty) * TY;
    const int k0 = (int)(t / (ntx * nty)) * kz;
    const int k1 = min(k0 + kz, g.nz);
    const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
    const int i = x0 + lane, j = y0 + row;
    const bool live = i < g.nx && j < g.ny;
    const int ic = live ? i : 0, jc = live ? j : 0;
    const long long n = g.n;
    const unsigned int plane = (unsigned int)g.nx * (unsigned int)g.ny;
    const Fields8 U = fields8(Ub, n);
    double* Fo[21];
#pragma unroll
    for (int q = 0; q < 21; ++q) Fo[q] = F + q * n;

    // z pipeline of the face-frame variables (rho, v_z, v_x, v_y, p, B_x, B_y)
    Pipe zp[7];
    {
        double pre[7][Pipe::PRIME];
#pragma unroll
        for (int s = 0; s < Pipe::PRIME; ++s) {
            const Prim8 w = load_prims(g, P, U, ic, jc, wrap_any(k0 - Pipe::PRIME + Pipe::AHEAD + s, g.nz));
            pre[0][s] = w.d; pre[1][s] = w.vz; pre[2][s] = w.vx; pre[3][s] = w.vy;
            pre[4][s] = w.p; pre[5][s] = w.bx; pre[6][s] = w.by;
        }
#pragma unroll
        for (int v = 0; v < 7; ++v) zp[v].prime(pre[v]);
    }

    for (int k = k0; k < k1; ++k) {
        // stage the primitives of plane k (tile + x/y halos, corners skipped)
        for (int q = threadIdx.x; q < LX * LY; q += TX * TY) {
            const int r = q / LX, cc = q - r * LX;
            const bool xh = cc < SL || cc >= SL + TX, yh = r < SL || r >= SL + TY;
            if (xh && yh) continue;
            const int gx = wrap_any(x0 + cc - SL, g.nx), gy = wrap_any(y0 + r - SL, g.ny);
            const Prim8 w = load_prims(g, P, U, gx, gy, k);
            sw[0][r][cc] = w.d; sw[1][r][cc] = w.vx; sw[2][r][cc] = w.vy; sw[3][r][cc] = w.vz;
            sw[4][r][cc] = w.p; sw[5][r][cc] = w.bx; sw[6][r][cc] = w.by; sw[7][r][cc] = w.bz;
        }
        // newest plane of the z pipeline
        const Prim8 wz = load_prims(g, P, U, ic, jc, wrap_any(k + Pipe::AHEAD, g.nz));
        __syncthreads();

        const unsigned int o = ((unsigned int)k * plane + (unsigned int)jc * g.nx + ic) * 8u;
        double st[6];
        Prim7 L, R;
        Flux7 f;
        // ---- z faces from the pipeline: (rho, vz, vx, vy, p, Bx, By)
        zp[0].push(wz.d, L.d, R.d);
        zp[1].push(wz.vz, L.vn, R.vn);
        zp[2].push(wz.vx, L.vt1, R.vt1);
        zp[3].push(wz.vy, L.vt2, R.vt2);
        zp[4].push(wz.p, L.p, R.p);
        zp[5].push(wz.bx, L.bt1, R.bt1);
        zp[6].push(wz.by, L.bt2, R.bt2);
        if (live) {
            solve<RS>(L, R, ld_at(U.f[7], o), P, f);
            st_at(Fo[14], o, f.d); st_at(Fo[17], o, f.mn); st_at(Fo[15], o, f.mt1); st_at(Fo[16], o, f.mt2);
            st_at(Fo[18], o, f.e); st_at(Fo[19], o, f.bt2); st_at(Fo[20], o, -f.bt1);
        }
        if (live) {
            // ---- x faces: (rho, vx, vy, vz, p, By, Bz)
            {
                const int comp[7] = {0, 1, 2, 3, 4, 6, 7};
                double* lr[7][2] = {{&L.d, &R.d}, {&L.vn, &R.vn}, {&L.vt1, &R.vt1}, {&L.vt2, &R.vt2},
                                    {&L.p, &R.p}, {&L.bt1, &R.bt1}, {&L.bt2, &R.bt2}};
#pragma unroll
                for (int v = 0; v < 7; ++v) {
#pragma unroll
                    for (int s = -SL; s <= SR; ++s) st[3 + s] = sw[comp[v]][row + SL][lane + SL + s];
                    face_states<RECON>(st, *lr[v][0], *lr[v][1]);
                }
                solve<RS>(L, R, ld_at(U.f[5], o), P, f);
                st_at(Fo[0], o, f.d); st_at(Fo[1], o, f.mn); st_at(Fo[2], o, f.mt1); st_at(Fo[3], o, f.mt2);
                st_at(Fo[4], o, f.e); st_at(Fo[5], o, f.bt2); st_at(Fo[6], o, -f.bt1);
            }
            // ---- y faces: (rho, vy, vz, vx, p, Bz, Bx)
            {
                const int comp[7] = {0, 2, 3, 1, 4, 7, 5};
                double* lr[7][2] = {{&L.d, &R.d}, {&L.vn, &R.vn}, {&L.vt1, &R.vt1}, {&L.vt2, &R.vt2},
                                    {&L.p, &R.p}, {&L.bt1, &R.bt1}, {&L.bt2, &R.bt2}};
#pragma unroll
                for (int v = 0; v < 7; ++v) {
#pragma unroll
                    for (int s = -SL; s <= SR; ++s) st[3 + s] = sw[comp[v]][row + SL + s][lane + SL];
                    face_states<RECON>(st, *lr[v][0], *lr[v][1]);
                }
                solve<RS>(L, R, ld_at(U.f[6], o), P, f);
                st_at(Fo[7], o, f.d); st_at(Fo[9], o, f.mn); st_at(Fo[10], o, f.mt1); st_at(Fo[8], o, f.mt2);
                st_at(Fo[11], o, f.e); st_at(Fo[12], o, f.bt2); st_at(Fo[13], o, -f.bt1);
            }
            // ---- cell field E = -v x B
            {
                const double vx = sw[1][row + SL][lane + SL], vy = sw[2][row + SL][lane + SL];
                const double vz = sw[3][row + SL][lane + SL], bx = sw[5][row + SL][lane + SL];
                const double by = sw[6][row + SL][lane + SL], bz = sw[7][row + SL][lane + SL];
                st_at(Rc, o, vz * by - vy * bz);
                st_at(Rc + n, o, vx * bz - vz * bx);
                st_at(Rc + 2 * n, o, vy * bx - vx * by);
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------------
// K2: edge EMFs, update, CFL
// ----------------------------------------------------------------------------------

__device__ __forceinline__ double gs_upwind(double m, double pos, double neg)
{
    return m > 0.0 ? pos : (m < 0.0 ? neg : 0.5 * (pos + neg));
}

// Gardiner-Stone edge value from the face values X (p-faces) and Y (q-faces), the cell
// field R at the four cells around the edge and the mass fluxes through the faces.
__device__ __forceinline__ double gs_edge(double X0, double Xm, double Y0, double Ym, double R00,
                                          double Rm0, double R0m, double Rmm, double fp0, double fpm,
                                          double fq0, double fqm)
{
    const double dqp = gs_upwind(fp0, Rm0 - Ym, R00 - Y0);
    const double dqm = gs_upwind(fpm, Ym - Rmm, Y0 - R0m);
    const double dpp = gs_upwind(fq0, R0m - Xm, R00 - X0);
    const double dpm = gs_upwind(fqm, Xm - Rmm, X0 - Rm0);
    return 0.25 * (((X0 + Xm) + (Y0 + Ym)) - ((dqp - dqm) + (dpp - dpm)));
}

struct CtArgs {
    const double* in;    // stage input register (8 fields)
    const double* base;  // second register (8 fields); may equal in, never out
    const double* F;     // 3 x 7 face fields
    const double* Rc;    // 3 cell E fields
    double* out;         // distinct from in and base
    double* partial;     // CFL partial minima, one per workgroup
    StageCoef co;
};

// CFL: reduce the time step of the output.  IN: the stage reads its input register
// (g0 != 0 or a gas acceleration is set); otherwise only the base register is read.
template <bool CFL, bool IN>
__global__ __launch_bounds__(TX* TY2) void k_ct_update(Geo g, MhdParams P, CtArgs a, int kz,
                                                     unsigned int ntx, unsigned int nty,
                                                     unsigned int nblk)
{
    // edges held for the tile: E_z on plane k, E_x / E_y on levels k-1/2 (slot lv^1)
    // and k+1/2 (slot lv); index ranges i in [0, TX], j in [0, TY2]
    __shared__ double sEz[TY2 + 1][TX + 1];
    __shared__ double sEx[2][TY2 + 1][TX + 1];
    __shared__ double sEy[2][TY2 + 1][TX + 1];
    __shared__ double sMin[TX * TY2 / 64];

    const unsigned int bt = xcd_tile(blockIdx.x, nblk);
    const int x0 = (int)(bt % ntx) * TX;
    const int y0 = (int)((bt / ntx) % nty) * TY2;
    const int k0 = (int)(bt / (ntx * nty)) * kz;
    const int k1 = min(k0 + kz, g.nz);
    const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
    const int i = x0 + lane, j = y0 + row;
    const bool live = i < g.nx && j < g.ny;
    const long long n = g.n;
    const unsigned int nx = g.nx, plane = (unsigned int)g.nx * (unsigned int)g.ny;
    // uniform bases: face fields (dir*7 + slot), cell E, registers
    const double* Fb[21];
#pragma unroll
    for (int q = 0; q < 21; ++q) Fb[q] = a.F + q * n;
    const double* Rx = a.Rc;
    const double* Ry = a.Rc + n;
    const double* Rz = a.Rc + 2 * n;
    const Fields8 In = fields8(a.in, n);
    const Fields8 Bs = fields8(a.base, n);
    double* Out[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) Out[q] = a.out + q * n;

    auto off = [&](int x, int y, int z) -> unsigned int {
        return ((unsigned int)z * plane + (unsigned int)y * nx + (unsigned int)x) * 8u;
    };
    // E_x at (x, y-1/2, z-1/2), E_y at (x-1/2, y, z-1/2), E_z at (x-1/2, y-1/2, z)
    auto edge_x = [&](int x, int y, int z) -> double {
        const int ym = wrap_once(y - 1, g.ny), zm = wrap_once(z - 1, g.nz);
        const unsigned int c = off(x, y, z), cy = off(x, ym, z), cz = off(x, y, zm), cyz = off(x, ym, zm);
        // p = y, q = z: X on y-faces (slot 6 of the y sweep), Y on z-faces (slot 5 of z)
        return gs_edge(ld_at(Fb[13], c), ld_at(Fb[13], cz), ld_at(Fb[19], c), ld_at(Fb[19], cy),
                       ld_at(Rx, c), ld_at(Rx, cy), ld_at(Rx, cz), ld_at(Rx, cyz),
                       ld_at(Fb[7], c), ld_at(Fb[7], cz), ld_at(Fb[14], c), ld_at(Fb[14], cy));
    };
    auto edge_y = [&](int x, int y, int z) -> double {
        const int xm = wrap_once(x - 1, g.nx), zm = wrap_once(z - 1, g.nz);
        const unsigned int c = off(x, y, z), cx = off(xm, y, z), cz = off(x, y, zm), cxz = off(xm, y, zm);
        // p = z, q = x: X on z-faces (slot 6 of z), Y on x-faces (slot 5 of x)
        return gs_edge(ld_at(Fb[20], c), ld_at(Fb[20], cx), ld_at(Fb[5], c), ld_at(Fb[5], cz),
                       ld_at(Ry, c), ld_at(Ry, cz), ld_at(Ry, cx), ld_at(Ry, cxz),
                       ld_at(Fb[14], c), ld_at(Fb[14], cx), ld_at(Fb[0], c), ld_at(Fb[0], cz));
    };
    auto edge_z = [&](int x, int y, int z) -> double {
        const int xm = wrap_once(x - 1, g.nx), ym = wrap_once(y - 1, g.ny);
        const unsigned int c = off(x, y, z), cx = off(xm, y, z), cy = off(x, ym, z), cxy = off(xm, ym, z);
        // p = x, q = y: X on x-faces (slot 6 of x), Y on y-faces (slot 5 of y)
        return gs_edge(ld_at(Fb[6], c), ld_at(Fb[6], cy), ld_at(Fb[12], c), ld_at(Fb[12], cx),
                       ld_at(Rz, c), ld_at(Rz, cx), ld_at(Rz, cy), ld_at(Rz, cxy),
                       ld_at(Fb[0], c), ld_at(Fb[0], cy), ld_at(Fb[7], c), ld_at(Fb[7], cx));
    };
    // level edges E_x, E_y at z-level zl - 1/2 for the tile (+1 ring on the high side)
    auto fill_level = [&](int slot, int zl) {
        const int zz = wrap_once(zl, g.nz);
        for (int q = threadIdx.x; q < (TX + 1) * (TY2 + 1); q += TX * TY2) {
            const int r = q / (TX + 1), cc = q - r * (TX + 1);
            const int gx = x0 + cc, gy = y0 + r;
            if (gx > g.nx || gy > g.ny) continue;
            const int wx = gx == g.nx ? 0 : gx, wy = gy == g.ny ? 0 : gy;
            if (cc < TX && gx < g.nx) sEx[slot][r][cc] = edge_x(wx, wy, zz);
            if (r < TY2 && gy < g.ny) sEy[slot][r][cc] = edge_y(wx, wy, zz);
        }
    };

    double vmin = INFINITY;
    int lv = 0;
    fill_level(lv ^ 1, k0);  // level k0 - 1/2
    const double bdt = a.co.bdt, g0 = a.co.g0, g1 = a.co.g1;

    for (int k = k0; k < k1; ++k) {
        // edges: E_z on plane k, E_x / E_y on level k + 1/2
        for (int q = threadIdx.x; q < (TX + 1) * (TY2 + 1); q += TX * TY2) {
            const int r = q / (TX + 1), cc = q - r * (TX + 1);
            const int gx = x0 + cc, gy = y0 + r;
            if (gx > g.nx || gy > g.ny) continue;
            const int wx = gx == g.nx ? 0 : gx, wy = gy == g.ny ? 0 : gy;
            sEz[r][cc] = edge_z(wx, wy, k);
        }
        fill_level(lv, k + 1);
        __syncthreads();

        if (live) {
            const int ip = i + 1 == g.nx ? 0 : i + 1, jp = j + 1 == g.ny ? 0 : j + 1;
            const int kp = k + 1 == g.nz ? 0 : k + 1;
            const unsigned int c = off(i, j, k), cx = off(ip, j, k), cy = off(i, jp, k), cz = off(i, j, kp);
            double L[5];
            const int slot[5] = {0, 1, 2, 3, 4};
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const double fx = (ld_at(Fb[slot[v]], cx) - ld_at(Fb[slot[v]], c)) * g.inv_dx[0];
                const double fy = (ld_at(Fb[7 + slot[v]], cy) - ld_at(Fb[7 + slot[v]], c)) * g.inv_dx[1];
                const double fz = (ld_at(Fb[14 + slot[v]], cz) - ld_at(Fb[14 + slot[v]], c)) * g.inv_dx[2];
                L[v] = -((fx + fy) + fz);
            }
            double o[5];
            if (IN) {
                double in5[5];
#pragma unroll
                for (int v = 0; v < 5; ++v) in5[v] = ld_at(In.f[v], c);
                L[1] += in5[0] * P.gacc[0];
                L[2] += in5[0] * P.gacc[1];
                L[3] += in5[0] * P.gacc[2];
                L[4] += (in5[1] * P.gacc[0] + in5[2] * P.gacc[1]) + in5[3] * P.gacc[2];
#pragma unroll
                for (int v = 0; v < 5; ++v) o[v] = (g0 * in5[v] + g1 * ld_at(Bs.f[v], c)) + bdt * L[v];
            } else {
#pragma unroll
                for (int v = 0; v < 5; ++v) o[v] = g1 * ld_at(Bs.f[v], c) + bdt * L[v];
            }

            // faces of this cell: b1 at x_{i-1/2}, b2 at y_{j-1/2}, b3 at z_{k-1/2}
            const int ol = lv ^ 1, nl = lv;
            auto nb1 = [&](int xl, unsigned int cc) {  // new B_x on the face at tile column xl
                const double lb = -((sEz[row + 1][xl] - sEz[row][xl]) * g.inv_dx[1] -
                                    (sEy[nl][row][xl] - sEy[ol][row][xl]) * g.inv_dx[2]);
                return (IN ? g0 * ld_at(In.f[5], cc) + g1 * ld_at(Bs.f[5], cc) : g1 * ld_at(Bs.f[5], cc)) + bdt * lb;
            };
            auto nb2 = [&](int yl, unsigned int cc) {  // new B_y on the face at tile row yl
                const double lb = -((sEx[nl][yl][lane] - sEx[ol][yl][lane]) * g.inv_dx[2] -
                                    (sEz[yl][lane + 1] - sEz[yl][lane]) * g.inv_dx[0]);
                return (IN ? g0 * ld_at(In.f[6], cc) + g1 * ld_at(Bs.f[6], cc) : g1 * ld_at(Bs.f[6], cc)) + bdt * lb;
            };
            auto nb3 = [&](int lvl, unsigned int cc) {  // new B_z on the z-face of level slot lvl
                const double lb = -((sEy[lvl][row][lane + 1] - sEy[lvl][row][lane]) * g.inv_dx[0] -
                                    (sEx[lvl][row + 1][lane] - sEx[lvl][row][lane]) * g.inv_dx[1]);
                return (IN ? g0 * ld_at(In.f[7], cc) + g1 * ld_at(Bs.f[7], cc) : g1 * ld_at(Bs.f[7], cc)) + bdt * lb;
            };
            const double b1 = nb1(lane, c);
            const double b2 = nb2(row, c);
            const double b3 = nb3(ol, c);
            if (CFL) {
                // the updated faces on the high side give the new B_cc of this cell
                const double bx = 0.5 * (b1 + nb1(lane + 1, cx));
                const double by = 0.5 * (b2 + nb2(row + 1, cy));
                const double bz = 0.5 * (b3 + nb3(nl, cz));
                double d = o[0];
                if (d < P.rho_floor) d = P.rho_floor;
                const double id = 1.0 / d;
                const double v[3] = {o[1] * id, o[2] * id, o[3] * id};
                const double ke = 0.5 * d * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
                const double b2s = (bx * bx + by * by) + bz * bz;
                double pr = (P.gamma - 1.0) * ((o[4] - ke) - 0.5 * b2s);
                if (pr < P.p_floor) pr = P.p_floor;
                const double bd[3] = {bx, by, bz};
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const double cf = fast_speed(P.gamma, d, pr, b2s, bd[q]);
                    vmin = min_nan(vmin, g.dx[q] / (fabs(v[q]) + cf));
                }
            }
            // out never aliases in or base (the host rotates three registers)
#pragma unroll
            for (int v = 0; v < 5; ++v) st_at(Out[v], c, o[v]);
            st_at(Out[5], c, b1);
            st_at(Out[6], c, b2);
            st_at(Out[7], c, b3);
        }
        __syncthreads();
        lv ^= 1;
    }
    if (CFL) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) vmin = min_nan(vmin, __shfl_xor(vmin, o, 64));
        if ((threadIdx.x & 63) == 0) sMin[threadIdx.x >> 6] = vmin;
        __syncthreads();
        if (threadIdx.x == 0) {
            double r = sMin[0];
#pragma unroll
            for (int w = 1; w < TX * TY2 / 64; ++w) r = min_nan(r, sMin[w]);
            a.partial[blockIdx.x] = r;
        }
    }
}

// ----------------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------------

FusedGrid fused_grid(const Geo& g, int kz)
{
    FusedGrid fg;
    fg.kz = kz;
    fg.ntx = (unsigned int)((g.nx + TX - 1) / TX);
    fg.nty = (unsigned int)((g.ny + TY - 1) / TY);
    fg.ntz = (unsigned int)((g.nz + kz - 1) / kz);
    fg.nblk = fg.ntx * fg.nty * fg.ntz;
    fg.nty2 = (unsigned int)((g.ny + TY2 - 1) / TY2);
    fg.nblk2 = fg.ntx * fg.nty2 * fg.ntz;
    return fg;
}

template <int RECON, int RS>
static hipError_t flux3(const Geo& g, const MhdParams& p, const FusedGrid& fg, const double* U,
                        double* F, double* Rc, hipStream_t s)
{
    hipLaunchKernelGGL((k_flux3<RECON, RS>), dim3(fg.nblk), dim3(TX * TY), 0, s, g, p, U, F, Rc, fg.kz,
                       fg.ntx, fg.nty, fg.nblk);
    return hipGetLastError();
}

hipError_t launch_mhd_flux3(const Geo& g, const MhdParams& p, const FusedGrid& fg, int recon,
                            int riemann, const double* U, double* F, double* Rc, hipStream_t s)
{
    if (riemann == 1) {
        if (recon == 0) return flux3<0, 1>(g, p, fg, U, F, Rc, s);
        if (recon == 1) return flux3<1, 1>(g, p, fg, U, F, Rc, s);
        return flux3<2, 1>(g, p, fg, U, F, Rc, s);
    }
    if (recon == 0) return flux3<0, 0>(g, p, fg, U, F, Rc, s);
    if (recon == 1) return flux3<1, 0>(g, p, fg, U, F, Rc, s);
    return flux3<2, 0>(g, p, fg, U, F, Rc, s);
}

hipError_t launch_mhd_ct_update(const Geo& g, const MhdParams& p, const FusedGrid& fg,
                                const double* in, const double* base, const double* F,
                                const double* Rc, double* out, StageCoef coef, double* partial,
                                double* dt_out, double cfl_scale, hipStream_t s)
{
    CtArgs a{in, base, F, Rc, out, partial, coef};
    const bool use_in = coef.g0 != 0.0 || p.gacc[0] != 0.0 || p.gacc[1] != 0.0 || p.gacc[2] != 0.0;
    const dim3 gr(fg.nblk2), bl(TX * TY2);
    if (dt_out) {
        if (use_in)
            hipLaunchKernelGGL((k_ct_update<true, true>), gr, bl, 0, s, g, p, a, fg.kz, fg.ntx, fg.nty2, fg.nblk2);
        else
            hipLaunchKernelGGL((k_ct_update<true, false>), gr, bl, 0, s, g, p, a, fg.kz, fg.ntx, fg.nty2, fg.nblk2);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_min_final(partial, fg.nblk2, cfl_scale, dt_out, s);
    }
    if (use_in)
        hipLaunchKernelGGL((k_ct_update<false, true>), gr, bl, 0, s, g, p, a, fg.kz, fg.ntx, fg.nty2, fg.nblk2);
    else
        hipLaunchKernelGGL((k_ct_update<false, false>), gr, bl, 0, s, g, p, a, fg.kz, fg.ntx, fg.nty2, fg.nblk2);
    return hipGetLastError();
}

}  // namespace mhd
