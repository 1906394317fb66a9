// mhd_fused.hip -- one stage of the CT-MHD update on one periodic grid in two
// z-marching kernels (bodies in mhd_tiles.hpp):
//
// k_flux3<RECON, RS, IN>  one workgroup = a TXF x TYF tile of xy columns marching a chunk
//                         of z planes; Riemann solves on every face of the tile, the
//                         cell fields of the stage output (rho, M, E), and the 9 face
//                         fields + 3 cell-E fields the edge EMFs need.
// k_ct_update<CFL, IN>    64-lane tiles of 8 rows (one halo row per 8); edge EMFs, the
//                         face-field update and, in the last stage, the CFL partials.
//                         The FP64 kernel that also reduces the time step uses 4 rows: it
//                         then keeps the previous plane's values in registers at three
//                         workgroups per CU (with 8 rows they would cost it half its
//                         occupancy).
#include "mhd_tiles.hpp"

namespace mhd {

using namespace tiles;

namespace {
constexpr int TXF = 16;  // lanes along x (flux/update kernel)
constexpr int TYF = 16;  // rows (flux/update kernel)
constexpr int TX = 64;   // lanes along x (CT kernel)
constexpr int TY = 4;    // rows (FP64 CT kernel that reduces the time step)
constexpr int TY2 = 8;   // rows (other CT kernels)
}  // namespace

template <int RECON, int RS, bool IN, class R>
__global__ __launch_bounds__(TXF* TYF) __attribute__((amdgpu_waves_per_eu(FluxWaves<RECON, RS, R>::min)))
void k_flux3(Geo g, MhdParams P, StageArgs<R> a, int kz, unsigned int ntx, unsigned int nty, unsigned int nblk)
{
    using Tile = FluxTile<RECON, RS, IN, R, TXF, TYF>;
    __shared__ typename Tile::Lds lds;
    const unsigned int t = xcd_tile(blockIdx.x, nblk);
    const int x0 = (int)(t % ntx) * TXF;
    const int y0 = (int)((t / ntx) % nty) * TYF;
    const int k0 = (int)(t / (ntx * nty)) * kz;
    Tile::run(g, P, a, x0, y0, k0, min(k0 + kz, g.nz), lds);
}

template <bool CFL, bool IN, class R, int TYC>
__global__ __launch_bounds__(TX* TYC) void k_ct_update(Geo g, MhdParams P, CtArgs<R> a, int kz,
                                                      unsigned int ntx, unsigned int nty,
                                                      unsigned int nblk)
{
    using Tile = CtTile<CFL, IN, R, TX, TYC>;
    __shared__ typename Tile::Lds lds;
    __shared__ double sMin[TX * TYC / 64];
    const unsigned int bt = xcd_tile(blockIdx.x, nblk);
    const int x0 = (int)(bt % ntx) * TX;
    const int y0 = (int)((bt / ntx) % nty) * TYC;
    const int k0 = (int)(bt / (ntx * nty)) * kz;
    double vmin = Tile::run(g, P, a, x0, y0, k0, min(k0 + kz, g.nz), lds);
    if (CFL) {
        vmin = wave_min64(vmin);
        if ((threadIdx.x & 63) == 0) sMin[threadIdx.x >> 6] = vmin;
        __syncthreads();
        if (threadIdx.x == 0) {
            double r = sMin[0];
#pragma unroll
            for (int w = 1; w < TX * TYC / 64; ++w) r = min_nan(r, sMin[w]);
            a.partial[blockIdx.x] = r;
        }
    }
}

// ----------------------------------------------------------------------------------
// FP32-bulk register <-> canonical FP64 state
// ----------------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_pack_fp32(long long n, const double* __restrict__ canon,
                                                      RegView<float> r)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    r.rho[c] = (float)canon[c];
    r.m[0][c] = (float)canon[n + c];
    r.m[1][c] = (float)canon[2 * n + c];
    r.m[2][c] = (float)canon[3 * n + c];
    r.E[c] = canon[4 * n + c];
    r.b[0][c] = (float)canon[5 * n + c];
    r.b[1][c] = (float)canon[6 * n + c];
    r.b[2][c] = (float)canon[7 * n + c];
}

__global__ __launch_bounds__(kBlock) void k_unpack_fp32(long long n, RegView<float> r,
                                                        double* __restrict__ canon)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    canon[c] = r.rho[c];
    canon[n + c] = r.m[0][c];
    canon[2 * n + c] = r.m[1][c];
    canon[3 * n + c] = r.m[2][c];
    canon[4 * n + c] = r.E[c];
    canon[5 * n + c] = r.b[0][c];
    canon[6 * n + c] = r.b[1][c];
    canon[7 * n + c] = r.b[2][c];
}

// ----------------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------------

FusedGrid fused_grid(const Geo& g, int kz)
{
    FusedGrid fg;
    fg.kz = kz;
    fg.ntx = (unsigned int)((g.nx + TXF - 1) / TXF);
    fg.nty = (unsigned int)((g.ny + TYF - 1) / TYF);
    fg.ntz = (unsigned int)((g.nz + kz - 1) / kz);
    fg.nblk = fg.ntx * fg.nty * fg.ntz;
    fg.ctx = (unsigned int)((g.nx + TX - 1) / TX);
    fg.cty4 = (unsigned int)((g.ny + TY - 1) / TY);
    fg.cty8 = (unsigned int)((g.ny + TY2 - 1) / TY2);
    return fg;
}

int flux_tile_cells() { return TXF * TYF; }

template <int RECON, int RS, bool IN, class R>
static hipError_t flux3(const Geo& g, const MhdParams& p, const FusedGrid& fg, const StageArgs<R>& a,
                        hipStream_t s)
{
    hipLaunchKernelGGL((k_flux3<RECON, RS, IN, R>), dim3(fg.nblk), dim3(TXF * TYF), 0, s, g, p, a, fg.kz,
                       fg.ntx, fg.nty, fg.nblk);
    return hipGetLastError();
}

template <int RECON, int RS, class R>
static hipError_t flux3_in(const Geo& g, const MhdParams& p, const FusedGrid& fg, const StageArgs<R>& a,
                           bool use_in, hipStream_t s)
{
    return use_in ? flux3<RECON, RS, true, R>(g, p, fg, a, s) : flux3<RECON, RS, false, R>(g, p, fg, a, s);
}

template <class R>
static hipError_t flux3_any(const Geo& g, const MhdParams& p, const FusedGrid& fg, int recon, int riemann,
                            void* in, void* base, void* out, void* F, void* Rc, StageCoef coef, hipStream_t s)
{
    const StageArgs<R> a{reg_view<R>(in, g.n), reg_view<R>(base, g.n), reg_view<R>(out, g.n), (R*)F, (R*)Rc,
                         coef};
    const bool use_in = coef.g0 != 0.0 || p.gacc[0] != 0.0 || p.gacc[1] != 0.0 || p.gacc[2] != 0.0;
    if (riemann == 1) {
        if (recon == 0) return flux3_in<0, 1, R>(g, p, fg, a, use_in, s);
        if (recon == 1) return flux3_in<1, 1, R>(g, p, fg, a, use_in, s);
        return flux3_in<2, 1, R>(g, p, fg, a, use_in, s);
    }
    if (recon == 0) return flux3_in<0, 0, R>(g, p, fg, a, use_in, s);
    if (recon == 1) return flux3_in<1, 0, R>(g, p, fg, a, use_in, s);
    return flux3_in<2, 0, R>(g, p, fg, a, use_in, s);
}

hipError_t launch_mhd_flux3(const Geo& g, const MhdParams& p, const FusedGrid& fg, bool fp32, int recon,
                            int riemann, void* in, void* base, void* out, void* F, void* Rc, StageCoef coef,
                            hipStream_t s)
{
    if (fp32) return flux3_any<float>(g, p, fg, recon, riemann, in, base, out, F, Rc, coef, s);
    return flux3_any<double>(g, p, fg, recon, riemann, in, base, out, F, Rc, coef, s);
}

template <class R>
static hipError_t ct_update(const Geo& g, const MhdParams& p, const FusedGrid& fg, void* in, void* base,
                            const void* F, const void* Rc, void* out, StageCoef coef, double* partial,
                            double* dt_out, double cfl_scale, hipStream_t s)
{
    CtArgs<R> a{reg_view<R>(in, g.n), reg_view<R>(base, g.n), (const R*)F, (const R*)Rc,
                reg_view<R>(out, g.n), partial, coef};
    const bool use_in = coef.g0 != 0.0;
    const unsigned int nb8 = fg.ctx * fg.cty8 * fg.ntz;
    if (dt_out) {
        // FP64: 4-row tiles; FP32: 8 rows
        constexpr int TYC = sizeof(R) == 8 ? TY : TY2;
        const unsigned int nty = sizeof(R) == 8 ? fg.cty4 : fg.cty8;
        const unsigned int nblk = fg.ctx * nty * fg.ntz;
        const dim3 grc(nblk), blc(TX * TYC);
        if (use_in)
            hipLaunchKernelGGL((k_ct_update<true, true, R, TYC>), grc, blc, 0, s, g, p, a, fg.kz, fg.ctx, nty, nblk);
        else
            hipLaunchKernelGGL((k_ct_update<true, false, R, TYC>), grc, blc, 0, s, g, p, a, fg.kz, fg.ctx, nty, nblk);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_min_final(partial, nblk, cfl_scale, dt_out, s);
    }
    const dim3 gr(nb8), bl(TX * TY2);
    if (use_in)
        hipLaunchKernelGGL((k_ct_update<false, true, R, TY2>), gr, bl, 0, s, g, p, a, fg.kz, fg.ctx, fg.cty8, nb8);
    else
        hipLaunchKernelGGL((k_ct_update<false, false, R, TY2>), gr, bl, 0, s, g, p, a, fg.kz, fg.ctx, fg.cty8, nb8);
    return hipGetLastError();
}

hipError_t launch_mhd_ct_update(const Geo& g, const MhdParams& p, const FusedGrid& fg, bool fp32,
                                void* in, void* base, const void* F, const void* Rc, void* out,
                                StageCoef coef, double* partial, double* dt_out, double cfl_scale,
                                hipStream_t s)
{
    if (fp32)
        return ct_update<float>(g, p, fg, in, base, F, Rc, out, coef, partial, dt_out, cfl_scale, s);
    return ct_update<double>(g, p, fg, in, base, F, Rc, out, coef, partial, dt_out, cfl_scale, s);
}

hipError_t launch_pack_fp32(const Geo& g, const double* canon, void* reg, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_fp32, dim3(blocks_for(g.n)), dim3(kBlock), 0, s, g.n, canon,
                       reg_view<float>(reg, g.n));
    return hipGetLastError();
}

hipError_t launch_unpack_fp32(const Geo& g, const void* reg, double* canon, hipStream_t s)
{
    hipLaunchKernelGGL(k_unpack_fp32, dim3(blocks_for(g.n)), dim3(kBlock), 0, s, g.n,
                       reg_view<float>(const_cast<void*>(reg), g.n), canon);
    return hipGetLastError();
}

}  // namespace mhd
