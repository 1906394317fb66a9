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
//
// Each stage is two launches:
//   k_fluid_pass  one workgroup = one fluid on a 64 x 4 tile of xy columns marching a
//                 chunk of z planes.  The fluid's primitives of the current plane and
//                 its x/y halo are staged in LDS (double buffered: the loads of plane
//                 k+1 are issued before plane k is computed), the z stencil of each
//                 column is a register pipeline that carries the flux of the low z
//                 face.  Every cell solves the Riemann problems on both of its x and y
//                 faces (no flux array, no extra barrier) and writes the explicit part
//                 of its stage:
//                   stage 1: X = u + h L(u);  stage 2: X = cu u + c1 U1 + cf L(U1).
//                 Densities are final after this pass (drag moves only momentum).
//   k_drag        pointwise: adds the stage-1 drag rates (stage 2), solves S_h for the
//                 momenta in place and, after stage 2, reduces the CFL step of the new
//                 state (one partial per workgroup).
//
// Precision: templated on the stored real type R.  R = double is the FP64 form; with
// R = float the state, the primitives, reconstruction, Riemann solves and explicit
// updates are FP32 while the drag solve (and the CFL step) stay FP64.
#include "launch.hpp"
#include "physics.hpp"

namespace mhd {

namespace {
constexpr double kLam = 1.7071067811865475244;    // 1 + 1/sqrt(2)
constexpr double kDelta = 0.70710678118654752440;  // 1 - 1/(2 lam) = 1/sqrt(2)

constexpr int DTX = 64;  // lanes along x
constexpr int DTY = 4;   // waves along y

// Blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous run of work
// items so neighbouring tiles of one fluid share an L2.
__device__ __forceinline__ unsigned int xcd_item(unsigned int b, unsigned int nb)
{
    const unsigned int q = nb >> 3, rem = nb & 7u;
    const unsigned int x = b & 7u, r = b >> 3;
    return x * q + (x < rem ? x : rem) + r;
}

__device__ __forceinline__ int wrap_any(int i, int n)
{
    if (i >= 0 && i < n) return i;
    const int r = i % n;
    return r < 0 ? r + n : r;
}

template <class T>
__device__ __forceinline__ T ld(const T* __restrict__ base, unsigned int idx)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (unsigned int)sizeof(T));
}
template <class T>
__device__ __forceinline__ void st(T* base, unsigned int idx, T v)
{
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (unsigned int)sizeof(T)) = v;
}

// Halo (cells on each side) of the reconstruction when both faces of a cell are built.
template <int RECON>
struct Halo {
    static constexpr int H = RECON == 0 ? 1 : 2;
};

// States on the low face (lo) and high face (hi) of the middle cell of a[0..2H]:
// donor cell or van Leer-limited PLM, the same formula on every face.
template <int RECON, class R>
__device__ __forceinline__ void both_faces(const R* a, R& loL, R& loR, R& hiL, R& hiR)
{
    if constexpr (RECON == 0) {
        loL = a[0]; loR = a[1]; hiL = a[1]; hiR = a[2];
    } else {
        const R sm = slope_vl(a[0], a[1], a[2]);
        const R s0 = slope_vl(a[1], a[2], a[3]);
        const R sp = slope_vl(a[2], a[3], a[4]);
        loL = a[1] + R(0.5) * sm;
        loR = a[2] - R(0.5) * s0;
        hiL = a[2] + R(0.5) * s0;
        hiR = a[3] - R(0.5) * sp;
    }
}

// Face flux along direction D from the global-frame states; returns global-frame
// components (mass, Mx, My, Mz).
template <int D, class R>
__device__ __forceinline__ void face_flux(bool gas, R cs, const R L[4], const R Rs[4], R out[4])
{
    constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
    const Prim4<R> l{L[0], L[1 + D], L[1 + T1], L[1 + T2]};
    const Prim4<R> r{Rs[0], Rs[1 + D], Rs[1 + T1], Rs[1 + T2]};
    Flux4<R> f;
    if (gas)
        riemann_iso_hlle(l, r, cs, f);
    else
        riemann_dust(l, r, f);
    out[0] = f.d;
    out[1 + D] = f.mn;
    out[1 + T1] = f.mt1;
    out[1 + T2] = f.mt2;
}

}  // namespace

// ----------------------------------------------------------------------------------
// explicit part of a stage, one fluid per workgroup
// ----------------------------------------------------------------------------------

template <class R>
struct PassArgs {
    const R* src;   // state whose fluxes are taken (u in stage 1, U1 in stage 2)
    const R* base;  // stage 2: u (read at the own cell only); stage 1: unused
    R* out;         // stage 1: U1; stage 2: u (in place: each cell reads then writes itself)
    double h;       // stage 1: lam dt; stage 2: (1 - delta) dt
    double cu, c1;  // stage 2 weights of u and U1
};

// z reconstruction of one variable of one column as a pipeline over the planes the
// column visits: push(plane m + 1 + AHEAD) returns the two states on the face m + 1/2
// (one slope per plane for PLM).
template <int RECON, class R>
struct ZLine;
template <class R>
struct ZLine<0, R> {
    static constexpr int AHEAD = 0, PRIME = 1;
    R prev;
    __device__ void prime(const R* a) { prev = a[0]; }
    __device__ void push(R a, R& aL, R& aR)
    {
        aL = prev;
        aR = a;
        prev = a;
    }
};
template <class R>
struct ZLine<1, R> {
    static constexpr int AHEAD = 1, PRIME = 3;
    R am, a0, apl;  // a(m-1), a(m), high-side state of cell m-1
    __device__ void prime(const R* a)
    {
        apl = a[1] + R(0.5) * slope_vl(a[0], a[1], a[2]);
        am = a[1];
        a0 = a[2];
    }
    __device__ void push(R a, R& aL, R& aR)
    {
        const R d = slope_vl(am, a0, a);
        aL = apl;
        aR = a0 - R(0.5) * d;
        apl = a0 + R(0.5) * d;
        am = a0;
        a0 = a;
    }
};

template <int RECON, int STAGE, class R>
__global__ __launch_bounds__(DTX* DTY) void k_fluid_pass(Geo g, DustParams p, PassArgs<R> a, int kz,
                                                           unsigned int ntx, unsigned int nty,
                                                           unsigned int ntiles, unsigned int nblk)
{
    constexpr int H = Halo<RECON>::H, W = 2 * H + 1;
    constexpr int LX = DTX + 2 * H, LY = DTY + 2 * H;
    constexpr int NT = DTX * DTY, NI = (LX * LY + NT - 1) / NT;  // staging items per thread
    using Z = ZLine<RECON, R>;
    __shared__ R sw[2][4][LY][LX];  // primitives of plane k (and k+1 being staged)

    const unsigned int item = xcd_item(blockIdx.x, nblk);
    const int s = (int)(item / ntiles);  // fluid: 0 gas, 1.. dust
    const unsigned int t = item - (unsigned int)s * ntiles;
    const bool gas = s == 0;
    const int x0 = (int)(t % ntx) * DTX;
    const int y0 = (int)((t / ntx) % nty) * DTY;
    const int k0 = (int)(t / (ntx * nty)) * kz;
    const int k1 = min(k0 + kz, g.nz);
    const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
    const int i = x0 + lane, j = y0 + row;
    const bool live = i < g.nx && j < g.ny;
    const int ic = live ? i : 0, jc = live ? j : 0;
    const long long n = g.n;
    const unsigned int plane = (unsigned int)g.nx * (unsigned int)g.ny;
    const R* f[4];
    R* o[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        f[q] = a.src + (4LL * s + q) * n;
        o[q] = a.out + (4LL * s + q) * n;
    }
    const R* b0 = a.base + 4LL * s * n;
    const R cs = R(p.cs);
    const R rho_floor = R(p.rho_floor), dust_floor = R(p.dust_floor);
    const R gx3[3] = {R(p.gacc[0]), R(p.gacc[1]), R(p.gacc[2])};
    const R hr = R(a.h), cur_ = R(a.cu), c1r = R(a.c1);
    const R idx[3] = {R(g.inv_dx[0]), R(g.inv_dx[1]), R(g.inv_dx[2])};
    const unsigned int col = (unsigned int)jc * g.nx + ic;

    // this thread's staging items of a plane (tile + x/y halo, corners skipped)
    unsigned int soff[NI];
    int sr[NI], sc[NI];
    bool sv[NI];
#pragma unroll
    for (int m = 0; m < NI; ++m) {
        const int q = threadIdx.x + m * NT;
        sr[m] = q / LX;
        sc[m] = q - sr[m] * LX;
        const bool xh = sc[m] < H || sc[m] >= H + DTX, yh = sr[m] < H || sr[m] >= H + DTY;
        sv[m] = q < LX * LY && !(xh && yh);
        const int gx = wrap_any(x0 + sc[m] - H, g.nx), gy = wrap_any(y0 + sr[m] - H, g.ny);
        soff[m] = sv[m] ? (unsigned int)gy * g.nx + gx : 0u;
    }
    // primitives from the raw state: the gas density is floored; a dust species below
    // its floor reads as the floor at rest
    auto prim_of = [&](const R raw[4], R w[4]) {
        const bool rest = !gas && raw[0] < dust_floor;
        R d = raw[0];
        if (gas && d < rho_floor) d = rho_floor;
        const R id = rcp(d);
        w[0] = rest ? dust_floor : d;
        w[1] = rest ? R(0) : raw[1] * id;
        w[2] = rest ? R(0) : raw[2] * id;
        w[3] = rest ? R(0) : raw[3] * id;
    };
    auto load_raw = [&](unsigned int c, R raw[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) raw[q] = ld(f[q], c);
    };
    R raw[NI][4];
    auto fetch_plane = [&](int kk) {
        const unsigned int pb = (unsigned int)kk * plane;
#pragma unroll
        for (int m = 0; m < NI; ++m)
            if (sv[m]) load_raw(pb + soff[m], raw[m]);
    };
    auto store_plane = [&](int buf) {
#pragma unroll
        for (int m = 0; m < NI; ++m)
            if (sv[m]) {
                R w[4];
                prim_of(raw[m], w);
#pragma unroll
                for (int v = 0; v < 4; ++v) sw[buf][v][sr[m]][sc[m]] = w[v];
            }
    };

    // z pipeline of the own column, primed so that the first push yields face k0 - 1/2
    Z zl[4];
    {
        R pre[4][Z::PRIME];
#pragma unroll
        for (int m = 0; m < Z::PRIME; ++m) {
            R r4[4], w[4];
            load_raw((unsigned int)wrap_any(k0 - Z::PRIME + Z::AHEAD + m, g.nz) * plane + col, r4);
            prim_of(r4, w);
#pragma unroll
            for (int v = 0; v < 4; ++v) pre[v][m] = w[v];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) zl[v].prime(pre[v]);
    }
    R zraw[4];  // raw state of the next plane the z pipeline takes
    load_raw((unsigned int)wrap_any(k0 + Z::AHEAD, g.nz) * plane + col, zraw);
    R fzlo[4];  // z flux on the low face of the current cell
    {
        R w[4], L[4], Rr[4];
        prim_of(zraw, w);
#pragma unroll
        for (int v = 0; v < 4; ++v) zl[v].push(w[v], L[v], Rr[v]);
        face_flux<2>(gas, cs, L, Rr, fzlo);
    }
    load_raw((unsigned int)wrap_any(k0 + 1 + Z::AHEAD, g.nz) * plane + col, zraw);
    fetch_plane(k0);
    store_plane(k0 & 1);
    __syncthreads();

    for (int k = k0; k < k1; ++k) {
        const int cur = k & 1;
        // loads for the next plane go out first; they land while this plane computes
        const bool more = k + 1 < k1;
        if (more) fetch_plane(k + 1);
        const unsigned int c = (unsigned int)k * plane + col;
        R own[4], ub[4];
        load_raw(c, own);
        if constexpr (STAGE == 2) {
#pragma unroll
            for (int v = 0; v < 4; ++v) ub[v] = ld(b0 + v * n, c);
        }
        R zw[4];
        prim_of(zraw, zw);
        if (more) load_raw((unsigned int)wrap_any(k + 2 + Z::AHEAD, g.nz) * plane + col, zraw);

        // acc = ((fx + fy) + fz): flux differences accumulated direction by direction
        R acc[4];
        {
            R Lm[4], Rm[4], Lp[4], Rp[4], st5[W], fl[4], fh[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
#pragma unroll
                for (int m = 0; m < W; ++m) st5[m] = sw[cur][v][row + H][lane + m];
                both_faces<RECON, R>(st5, Lm[v], Rm[v], Lp[v], Rp[v]);
            }
            face_flux<0>(gas, cs, Lm, Rm, fl);
            face_flux<0>(gas, cs, Lp, Rp, fh);
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] = (fh[v] - fl[v]) * idx[0];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
#pragma unroll
                for (int m = 0; m < W; ++m) st5[m] = sw[cur][v][row + m][lane + H];
                both_faces<RECON, R>(st5, Lm[v], Rm[v], Lp[v], Rp[v]);
            }
            face_flux<1>(gas, cs, Lm, Rm, fl);
            face_flux<1>(gas, cs, Lp, Rp, fh);
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] = acc[v] + (fh[v] - fl[v]) * idx[1];
#pragma unroll
            for (int v = 0; v < 4; ++v) zl[v].push(zw[v], Lp[v], Rp[v]);
            face_flux<2>(gas, cs, Lp, Rp, fh);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                acc[v] = acc[v] + (fh[v] - fzlo[v]) * idx[2];
                fzlo[v] = fh[v];
            }
        }
        if (live) {
            // the step's input u passes the dust floor reset (a species below its floor
            // becomes the floor at rest) where it enters the combination, in both stages
            R* uin = STAGE == 1 ? own : ub;
            if (!gas && uin[0] < dust_floor) {
                uin[0] = dust_floor;
                uin[1] = uin[2] = uin[3] = R(0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                R L = -acc[v];
                // the gas acceleration acts on the raw gas density
                if (gas && v > 0) L += own[0] * gx3[v - 1];
                R X;
                if constexpr (STAGE == 1)
                    X = own[v] + hr * L;
                else
                    X = (cur_ * ub[v] + c1r * own[v]) + hr * L;
                st(o[v], c, X);
            }
        }
        if (more) store_plane(cur ^ 1);
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------------
// drag solve (and the CFL step after stage 2), pointwise
// ----------------------------------------------------------------------------------

// Constants of one drag solve S_h, computed on the host per launch (h = lam dt):
// w_k = h/(t_k + h), a_k = t_k/(t_k + h) and 1/t_k, so that no cell divides by them.
struct DragCoef {
    double w[kMaxDust], a[kMaxDust], its[kMaxDust];
    double h, cg;  // cg: weight of the stage-1 drag rates (stage 2)
};

static DragCoef drag_coef(const DustParams& p, double h, double cg)
{
    DragCoef q{};
    for (int s = 0; s < p.nd; ++s) {
        q.w[s] = h / (p.ts[s] + h);
        q.a[s] = p.ts[s] / (p.ts[s] + h);
        q.its[s] = 1.0 / p.ts[s];
    }
    q.h = h;
    q.cg = cg;
    return q;
}

// Closed-form drag solve of one momentum component, in place on mom[0..ND]:
// v_g' = (p_g + sum w_k p_k)/(rho_g + sum w_k rho_k), p_k' = a_k p_k + w_k rho_k v_g'.
template <int ND>
__device__ __forceinline__ void drag_solve(const DragCoef& q, const double* rho, double* mom)
{
    double num = mom[0], den = rho[0];
#pragma unroll
    for (int s = 1; s <= ND; ++s) {
        num += q.w[s - 1] * mom[s];
        den += q.w[s - 1] * rho[s];
    }
    const double vg = num / den;
#pragma unroll
    for (int s = 1; s <= ND; ++s) mom[s] = q.a[s - 1] * mom[s] + q.w[s - 1] * (rho[s] * vg);
    mom[0] = rho[0] * vg;
}

// Reciprocal density of fluid s for its velocity: the gas density floored; a dust
// species below its floor is at rest (0).
__device__ __forceinline__ double inv_density(const DustParams& p, int s, double d)
{
    const double f = s == 0 ? p.rho_floor : p.dust_floor;
    const double iv = 1.0 / (d < f ? f : d);
    return s > 0 && d < f ? 0.0 : iv;
}

// NaN-propagating maximum of non-negative speeds
__device__ __forceinline__ double max_nan(double a, double b)
{
    const double m = a > b ? a : b;
    return (a != a) || (b != b) ? a + b : m;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min_nan(v, __shfl_xor(v, off, 64));
    return v;
}

// X: the explicit part (densities final); U1: stage-1 state (stage 2 only).  The number
// of dust species ND is a template parameter so the per-cell vectors live in registers.
// Loads are of the stored type R; the solve is FP64.
template <int STAGE, int ND, class R>
__global__ __launch_bounds__(kBlock) void k_drag(Geo g, DustParams p, DragCoef q, R* __restrict__ X,
                                                 const R* __restrict__ U1, double* __restrict__ partial)
{
    const long long cl = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long n = g.n;
    double r = INFINITY;
    if (cl < n) {
        const unsigned int c = (unsigned int)cl;
        double rho[ND + 1], r1[ND + 1], ivn[ND + 1], ivg1 = 0.0;
#pragma unroll
        for (int s = 0; s <= ND; ++s) rho[s] = (double)ld(X + 4LL * s * n, c);
        if constexpr (STAGE == 2) {
#pragma unroll
            for (int s = 0; s <= ND; ++s) {
                r1[s] = (double)ld(U1 + 4LL * s * n, c);
                ivn[s] = inv_density(p, s, rho[s]);
            }
            ivg1 = inv_density(p, 0, r1[0]);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double mom[ND + 1];
#pragma unroll
            for (int s = 0; s <= ND; ++s) mom[s] = (double)ld(X + (4LL * s + 1 + a) * n, c);
            if constexpr (STAGE == 2) {
                // + (1 - lam - delta) dt G(U1): drag rates of the stage-1 state in their
                // momentum form (rho_k v_g - p_k)/t_k, the map the stage-1 solve inverted
                const double vg = (double)ld(U1 + (1LL + a) * n, c) * ivg1;
                double gsum = 0.0;
#pragma unroll
                for (int s = 1; s <= ND; ++s) {
                    const double pk = (double)ld(U1 + (4LL * s + 1 + a) * n, c);
                    const double fk = (r1[s] * vg - pk) * q.its[s - 1];
                    mom[s] = mom[s] + q.cg * fk;
                    gsum -= fk;
                }
                mom[0] = mom[0] + q.cg * gsum;
            }
            drag_solve<ND>(q, rho, mom);
#pragma unroll
            for (int s = 0; s <= ND; ++s) {
                st(X + (4LL * s + 1 + a) * n, c, (R)mom[s]);
                mom[s] = (double)(R)mom[s];  // the CFL step sees the stored state
            }
            if constexpr (STAGE == 2) {
                // time step of the new state, as the standalone CFL kernel takes it:
                // min_s dx/(|v_s| + c_s) = dx / max_s(|v_s| + c_s) (division is monotone)
                double sp = fabs(mom[0] * ivn[0]) + p.cs;
#pragma unroll
                for (int s = 1; s <= ND; ++s) sp = max_nan(sp, fabs(mom[s] * ivn[s]));
                r = min_nan(r, g.dx[a] / sp);
            }
        }
    }
    if constexpr (STAGE == 2) {
        __shared__ double sm[kBlock / 64];
        r = wave_min(r);
        if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = r;
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = sm[0];
#pragma unroll
            for (int w = 1; w < kBlock / 64; ++w) m = min_nan(m, sm[w]);
            partial[blockIdx.x] = m;
        }
    }
}

template <int STAGE, int ND, class R>
static void drag_launch(const Geo& g, const DustParams& p, const DragCoef& q, R* X, const R* U1,
                        double* partial, hipStream_t s)
{
    hipLaunchKernelGGL((k_drag<STAGE, ND, R>), dim3(blocks_for(g.n)), dim3(kBlock), 0, s, g, p, q, X, U1,
                       partial);
}

// Dispatch on the species count (1..kMaxDust) to the specialised kernel.
template <int STAGE, class R, int ND = 1>
static hipError_t drag_dispatch(const Geo& g, const DustParams& p, const DragCoef& q, R* X, const R* U1,
                                double* partial, hipStream_t s)
{
    if constexpr (ND > kMaxDust) {
        return hipErrorInvalidValue;
    } else {
        if (p.nd == ND) {
            drag_launch<STAGE, ND, R>(g, p, q, X, U1, partial, s);
            return hipGetLastError();
        }
        return drag_dispatch<STAGE, R, ND + 1>(g, p, q, X, U1, partial, s);
    }
}

// ----------------------------------------------------------------------------------

DustGrid dust_grid(const Geo& g, int nfluids)
{
    DustGrid d;
    d.ntx = (unsigned int)((g.nx + DTX - 1) / DTX);
    d.nty = (unsigned int)((g.ny + DTY - 1) / DTY);
    const long long tiles = (long long)d.ntx * d.nty * nfluids;
    // about 4096 workgroups, at least 8 planes each (the z window is primed per chunk)
    const long long want = (4096 + tiles - 1) / tiles;
    int kz = (int)((g.nz + want - 1) / want);
    if (kz < 8) kz = 8;
    if (kz > g.nz) kz = g.nz;
    d.kz = kz;
    d.ntz = (unsigned int)((g.nz + kz - 1) / kz);
    d.ntiles = d.ntx * d.nty * d.ntz;
    d.nblk = d.ntiles * (unsigned int)nfluids;
    return d;
}

template <int RECON, class R>
static hipError_t pass(const Geo& g, const DustParams& p, const DustGrid& d, int stage, const PassArgs<R>& a,
                       hipStream_t s)
{
    const dim3 gr(d.nblk), bl(DTX * DTY);
    if (stage == 1)
        hipLaunchKernelGGL((k_fluid_pass<RECON, 1, R>), gr, bl, 0, s, g, p, a, d.kz, d.ntx, d.nty, d.ntiles, d.nblk);
    else
        hipLaunchKernelGGL((k_fluid_pass<RECON, 2, R>), gr, bl, 0, s, g, p, a, d.kz, d.ntx, d.nty, d.ntiles, d.nblk);
    return hipGetLastError();
}

template <class R>
static hipError_t pass1(const Geo& g, const DustParams& p, const DustGrid& d, int recon, const void* u, void* U1,
                        double dt, hipStream_t s)
{
    PassArgs<R> a{(const R*)u, nullptr, (R*)U1, kLam * dt, 0.0, 0.0};
    return recon == 0 ? pass<0, R>(g, p, d, 1, a, s) : pass<1, R>(g, p, d, 1, a, s);
}

template <class R>
static hipError_t pass2(const Geo& g, const DustParams& p, const DustGrid& d, int recon, void* u, const void* U1,
                        double dt, hipStream_t s)
{
    PassArgs<R> a{(const R*)U1, (const R*)u, (R*)u, (1.0 - kDelta) * dt, 1.0 - kDelta / kLam, kDelta / kLam};
    return recon == 0 ? pass<0, R>(g, p, d, 2, a, s) : pass<1, R>(g, p, d, 2, a, s);
}

hipError_t launch_fluid_pass1(const Geo& g, const DustParams& p, const DustGrid& d, bool fp32, int recon,
                              const void* u, void* U1, double dt, hipStream_t s)
{
    return fp32 ? pass1<float>(g, p, d, recon, u, U1, dt, s) : pass1<double>(g, p, d, recon, u, U1, dt, s);
}

hipError_t launch_fluid_pass2(const Geo& g, const DustParams& p, const DustGrid& d, bool fp32, int recon,
                              void* u, const void* U1, double dt, hipStream_t s)
{
    return fp32 ? pass2<float>(g, p, d, recon, u, U1, dt, s) : pass2<double>(g, p, d, recon, u, U1, dt, s);
}

hipError_t launch_drag1(const Geo& g, const DustParams& p, bool fp32, void* U1, double dt, hipStream_t s)
{
    const DragCoef q = drag_coef(p, kLam * dt, 0.0);
    if (fp32) return drag_dispatch<1, float>(g, p, q, (float*)U1, nullptr, nullptr, s);
    return drag_dispatch<1, double>(g, p, q, (double*)U1, nullptr, nullptr, s);
}

hipError_t launch_drag2_cfl(const Geo& g, const DustParams& p, bool fp32, void* u, const void* U1, double dt,
                            double* partial, double* dt_out, double cfl_scale, hipStream_t s)
{
    const DragCoef q = drag_coef(p, kLam * dt, (1.0 - kLam - kDelta) * dt);
    hipError_t e = fp32 ? drag_dispatch<2, float>(g, p, q, (float*)u, (const float*)U1, partial, s)
                        : drag_dispatch<2, double>(g, p, q, (double*)u, (const double*)U1, partial, s);
    if (e != hipSuccess) return e;
    return launch_min_final(partial, blocks_for(g.n), cfl_scale, dt_out, s);
}

// FP32 dust register <-> canonical FP64 state (nv fields)
__global__ __launch_bounds__(kBlock) void k_dust_pack(long long m, const double* __restrict__ canon,
                                                      float* __restrict__ reg)
{
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (q < m) reg[q] = (float)canon[q];
}
__global__ __launch_bounds__(kBlock) void k_dust_unpack(long long m, const float* __restrict__ reg,
                                                        double* __restrict__ canon)
{
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (q < m) canon[q] = reg[q];
}

hipError_t launch_dust_pack(long long m, const double* canon, void* reg, hipStream_t s)
{
    hipLaunchKernelGGL(k_dust_pack, dim3(blocks_for(m)), dim3(kBlock), 0, s, m, canon, (float*)reg);
    return hipGetLastError();
}

hipError_t launch_dust_unpack(long long m, const void* reg, double* canon, hipStream_t s)
{
    hipLaunchKernelGGL(k_dust_unpack, dim3(blocks_for(m)), dim3(kBlock), 0, s, m, (const float*)reg, canon);
    return hipGetLastError();
}

}  // namespace mhd
