// reduce.hip -- the time step of eq. (cfl) and the conservation diagnostics.
//
// Both are two-pass reductions with a fixed assignment of cells to lanes and of
// partials to the final pass, so the result is bitwise reproducible run to run.
// Within a wavefront the 64 lanes combine by butterfly shuffles.
#include <algorithm>

#include "launch.hpp"
#include "physics.hpp"

namespace mhd {

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min_nan(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide minimum; the result is valid in thread 0.
__device__ __forceinline__ double block_min(double v)
{
    __shared__ double sm[kBlock / 64];
    v = wave_min(v);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = sm[0];
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 1; w < kBlock / 64; ++w) r = min_nan(r, sm[w]);
    }
    return r;
}

// Time step of eq. (cfl) of cell c of a grid of n cells; cx, cy, cz: the cells whose
// low faces are c's high faces.  The same arithmetic, rounded as written, as the time
// step the last stage of a step reduces (mhd_tiles.hpp), so a state gives the same bits
// whichever kernel takes its step.
__device__ __forceinline__ double cfl_cell(const Geo& g, const MhdParams& p, const double* __restrict__ U,
                                           long long n, long long c, long long cx, long long cy, long long cz)
{
#pragma clang fp contract(off)
    const double bx = 0.5 * (U[5 * n + c] + U[5 * n + cx]);
    const double by = 0.5 * (U[6 * n + c] + U[6 * n + cy]);
    const double bz = 0.5 * (U[7 * n + c] + U[7 * n + cz]);
    double d = U[c];
    if (d < p.rho_floor) d = p.rho_floor;
    const double id = rcp(d);
    const double v[3] = {U[n + c] * id, U[2 * n + c] * id, U[3 * n + c] * id};
    const double ke = 0.5 * d * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    const double b2 = (bx * bx + by * by) + bz * bz;
    double pr = (p.gamma - 1.0) * ((U[4 * n + c] - ke) - 0.5 * b2);
    if (pr < p.p_floor) pr = p.p_floor;
    const double bd[3] = {bx, by, bz};
    double r = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double cf = fast_speed(p.gamma, d, pr, b2, bd[a]);
        r = min_nan(r, div_r(g.dx[a], fabs(v[a]) + cf));
    }
    return r;
}

__global__ __launch_bounds__(kBlock) void k_cfl_mhd(Geo g, MhdParams p, const double* __restrict__ U,
                                                    double* __restrict__ partial)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    double r = INFINITY;
    if (c < g.n) {
        int i, j, k;
        cell_ijk(g, c, i, j, k);
        r = cfl_cell(g, p, U, g.n, c, shifted(g, i, j, k, 0, 1), shifted(g, i, j, k, 1, 1), shifted(g, i, j, k, 2, 1));
    }
    r = block_min(r);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// The time step over the interior cells of nb equal padded blocks (grid pg each, g
// ghost layers, interior bx x by x bz; block b's register at reg + 8 off[b] doubles):
// ghost cells are left out (the outermost layer's high neighbours are not in the block).
__global__ __launch_bounds__(kBlock) void k_cfl_blocks(Geo pg, MhdParams p, const double* __restrict__ reg,
                                                       const unsigned long long* __restrict__ off, int nb, int gh,
                                                       int bx, int by, int bz, double* __restrict__ partial)
{
    const long long per = (long long)bx * by * bz;
    double r = INFINITY;
    // a fixed grid strides over the cells, so the final pass has few partials
    for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < per * nb;
         t += (long long)gridDim.x * kBlock) {
        const int b = (int)(t / per);
        const long long q = t - (long long)b * per;
        const int i = (int)(q % bx) + gh, j = (int)((q / bx) % by) + gh, k = (int)(q / ((long long)bx * by)) + gh;
        const long long c = ((long long)k * pg.ny + j) * pg.nx + i;
        r = min_nan(r, cfl_cell(pg, p, reg + off[b] * 8ULL, pg.n, c, c + 1, c + pg.nx, c + (long long)pg.nx * pg.ny));
    }
    r = block_min(r);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ __launch_bounds__(kBlock) void k_cfl_dust(Geo g, DustParams p, const double* __restrict__ U,
                                                     double* __restrict__ partial)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    double r = INFINITY;
    if (c < g.n) {
        const long long n = g.n;
        for (int s = 0; s <= p.nd; ++s) {
            const double* u = U + 4LL * s * n;
            double d = u[c];
            double v[3];
            if (s == 0) {
                if (d < p.rho_floor) d = p.rho_floor;
                v[0] = u[n + c] / d; v[1] = u[2 * n + c] / d; v[2] = u[3 * n + c] / d;
            } else if (d < p.dust_floor) {
                v[0] = v[1] = v[2] = 0.0;
            } else {
                v[0] = u[n + c] / d; v[1] = u[2 * n + c] / d; v[2] = u[3 * n + c] / d;
            }
            const double cs = s == 0 ? p.cs : 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) r = min_nan(r, g.dx[a] / (fabs(v[a]) + cs));
        }
    }
    r = block_min(r);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ __launch_bounds__(kBlock) void k_min_final(const double* __restrict__ partial, long long m,
                                                      double scale, double* __restrict__ out)
{
    double r = INFINITY;
    for (long long q = threadIdx.x; q < m; q += kBlock) r = min_nan(r, partial[q]);
    r = block_min(r);
    if (threadIdx.x == 0) out[0] = scale * r;
}

hipError_t launch_min_final(const double* partial, long long m, double scale, double* out,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_min_final, dim3(1), dim3(kBlock), 0, s, partial, m, scale, out);
    return hipGetLastError();
}

hipError_t launch_cfl_mhd(const Geo& g, const MhdParams& p, const double* U, double* partial,
                          double* dt_out, double scale, hipStream_t s)
{
    const unsigned int nb = blocks_for(g.n);
    hipLaunchKernelGGL(k_cfl_mhd, dim3(nb), dim3(kBlock), 0, s, g, p, U, partial);
    hipLaunchKernelGGL(k_min_final, dim3(1), dim3(kBlock), 0, s, partial, (long long)nb, scale, dt_out);
    return hipGetLastError();
}

hipError_t launch_cfl_blocks(const Geo& pg, const MhdParams& p, const double* reg, const unsigned long long* off,
                             int nb, int ghost, int bx, int by, int bz, double* partial, double* dt_out,
                             double scale, hipStream_t s)
{
    const long long m = std::min<long long>(((long long)bx * by * bz * nb + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_cfl_blocks, dim3((unsigned int)m), dim3(kBlock), 0, s, pg, p, reg, off, nb, ghost, bx, by, bz,
                       partial);
    hipLaunchKernelGGL(k_min_final, dim3(1), dim3(kBlock), 0, s, partial, m, scale, dt_out);
    return hipGetLastError();
}

hipError_t launch_cfl_dust(const Geo& g, const DustParams& p, const double* U, double* partial,
                           double* dt_out, double scale, hipStream_t s)
{
    const unsigned int nb = blocks_for(g.n);
    hipLaunchKernelGGL(k_cfl_dust, dim3(nb), dim3(kBlock), 0, s, g, p, U, partial);
    hipLaunchKernelGGL(k_min_final, dim3(1), dim3(kBlock), 0, s, partial, (long long)nb, scale, dt_out);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------
// diagnostics: out[0] gas mass, [1..3] gas momentum, [4] E, [5..7] face-field
// integrals, [8] max |div B|, [9..8+nd] dust masses, [9+nd..11+nd] total momentum
// ----------------------------------------------------------------------------------

int diag_count(int ndust) { return 12 + ndust; }

__global__ __launch_bounds__(kBlock) void k_diag_partial(Geo g, int mhd, int nd,
                                                         const double* __restrict__ U,
                                                         double* __restrict__ partial)
{
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    const int nq = 12 + nd;
    const long long n = g.n;
    __shared__ double sm[kBlock / 64][12 + kMaxDust];
    const bool live = c < n;
    double vals[12 + kMaxDust];
    for (int q = 0; q < nq; ++q) vals[q] = 0.0;
    if (live) {
        if (mhd) {
            for (int q = 0; q < 8; ++q) {
                const double x = U[q * n + c];
                if (q < 5) vals[q] = x; else vals[q] = x;
            }
            int i, j, k;
            cell_ijk(g, c, i, j, k);
            const double dv = (U[5 * n + shifted(g, i, j, k, 0, 1)] - U[5 * n + c]) * g.inv_dx[0] +
                              (U[6 * n + shifted(g, i, j, k, 1, 1)] - U[6 * n + c]) * g.inv_dx[1] +
                              (U[7 * n + shifted(g, i, j, k, 2, 1)] - U[7 * n + c]) * g.inv_dx[2];
            vals[8] = fabs(dv);
            for (int a = 0; a < 3; ++a) vals[9 + a] = U[(1 + a) * n + c];
        } else {
            for (int q = 0; q < 4; ++q) vals[q] = U[q * n + c];
            for (int a = 0; a < 3; ++a) vals[9 + nd + a] = U[(1 + a) * n + c];
            for (int s = 1; s <= nd; ++s) {
                vals[9 + s - 1] = U[4LL * s * n + c];
                for (int a = 0; a < 3; ++a) vals[9 + nd + a] += U[(4LL * s + 1 + a) * n + c];
            }
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int q = 0; q < nq; ++q) {
        const double r = (q == 8) ? wave_max(vals[q]) : wave_sum(vals[q]);
        if (lane == 0) sm[w][q] = r;
    }
    __syncthreads();
    if (threadIdx.x < nq) {
        const int q = threadIdx.x;
        double r = sm[0][q];
        for (int ww = 1; ww < kBlock / 64; ++ww) r = (q == 8) ? fmax(r, sm[ww][q]) : r + sm[ww][q];
        partial[(long long)blockIdx.x * nq + q] = r;
    }
}

// One workgroup per quantity; lanes stride over the partials in a fixed order.
__global__ __launch_bounds__(kBlock) void k_diag_final(const double* __restrict__ partial, long long m,
                                                       int nq, double dV, double* __restrict__ out)
{
    const int q = blockIdx.x;
    const bool mx = (q == 8);
    double r = 0.0;
    for (long long b = threadIdx.x; b < m; b += kBlock) {
        const double x = partial[b * nq + q];
        r = mx ? fmax(r, x) : r + x;
    }
    __shared__ double sm[kBlock / 64];
    r = mx ? wave_max(r) : wave_sum(r);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = sm[0];
        for (int w = 1; w < kBlock / 64; ++w) t = mx ? fmax(t, sm[w]) : t + sm[w];
        out[q] = mx ? t : t * dV;
    }
}

hipError_t launch_diag(const Geo& g, int mhd, int ndust, const double* U, double* partial,
                       double* out, hipStream_t s)
{
    const unsigned int nb = blocks_for(g.n);
    const int nq = diag_count(ndust);
    hipLaunchKernelGGL(k_diag_partial, dim3(nb), dim3(kBlock), 0, s, g, mhd, ndust, U, partial);
    const double dV = g.dx[0] * g.dx[1] * g.dx[2];
    hipLaunchKernelGGL(k_diag_final, dim3(nq), dim3(kBlock), 0, s, partial, (long long)nb, nq, dV, out);
    return hipGetLastError();
}

}  // namespace mhd
