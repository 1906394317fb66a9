// common.hpp -- grid geometry, workspace views and launch helpers shared by the
// kernels of the library (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mhd {

constexpr int kMaxDust = 16;
constexpr int kBlock = 256;  // threads per workgroup of the cell-parallel kernels

// Uniform periodic grid; cells are numbered c = (k*ny + j)*nx + i, x fastest.
struct Geo {
    int nx, ny, nz;
    long long n;        // cells
    double dx[3];
    double inv_dx[3];
};

__device__ __forceinline__ int wrapi(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ void cell_ijk(const Geo& g, long long c, int& i, int& j, int& k)
{
    i = (int)(c % g.nx);
    long long t = c / g.nx;
    j = (int)(t % g.ny);
    k = (int)(t / g.ny);
}

__device__ __forceinline__ long long cell_at(const Geo& g, int i, int j, int k)
{
    return ((long long)k * g.ny + j) * g.nx + i;
}

// Index of the cell displaced by `off` cells along axis d (periodic).
__device__ __forceinline__ long long shifted(const Geo& g, int i, int j, int k, int d, int off)
{
    if (d == 0) return cell_at(g, wrapi(i + off, g.nx), j, k);
    if (d == 1) return cell_at(g, i, wrapi(j + off, g.ny), k);
    return cell_at(g, i, j, wrapi(k + off, g.nz));
}

// NaN-propagating minimum (a non-finite state must surface in the CFL reduction).
__device__ __forceinline__ double min_nan(double a, double b)
{
    const double m = a < b ? a : b;
    return (a != a) || (b != b) ? a + b : m;  // selects, no branch
}

// Loads and stores at a 32-bit byte offset from a uniform base pointer: the address is
// formed by the memory unit (scalar base + vector offset), not by 64-bit vector math.
// Fields must stay below 4 GiB (checked when a context is created).
__device__ __forceinline__ double ld_at(const double* __restrict__ base, unsigned int boff)
{
    return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + boff);
}
__device__ __forceinline__ void st_at(double* base, unsigned int boff, double v)
{
    *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + boff) = v;
}

// Stage combination out = g0*in + g1*base + bdt*L of eq. (two_register).
struct StageCoef {
    double g0, g1, bdt;
};

}  // namespace mhd
