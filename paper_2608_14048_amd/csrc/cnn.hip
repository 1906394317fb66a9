// cnn.hip -- the learned subgrid flux-correction closure of the coarse MHD step.
//
// An extension of this library, not part of the paper's method (the paper only
// remarks, Sec. "Discussion and Summary", that a neural surrogate could replace an
// expensive cell-local solve such as astrochemistry).  The construction around the
// network follows the method: the network sees the 8
// primitive channels of the coarse state at the start of a step and returns 15 face-
// flux corrections (rho, M_x, M_y, M_z, E through the low x, y and z face of each cell)
// and 3 edge-EMF corrections (E_x on edge (i, j-1/2, k-1/2), E_y on (i-1/2, j, k-1/2),
// E_z on (i-1/2, j-1/2, k)); they are added to the plain step in flux form (eq.
// (fv_update)) and in constrained-transport form (eq. (ct)), so the corrected step
// stays conservative and keeps div B.
//
// Network: 4 periodic 3x3x3 convolutions, widths 8 -> 32 -> 32 -> 32 -> 18, ReLU after
// the first three.  Every convolution is an implicit GEMM on the matrix cores: BF16
// operands, FP32 accumulation, v_mfma_f32_16x16x32_bf16 for the 32-channel inputs and
// v_mfma_f32_16x16x16_bf16 for the first layer's 16 (8 padded).  Activations are
// stored channel-last ([voxel][channel], channels padded to 16 or 32) so that one
// lane's K values are one or two 8-byte loads.  A wavefront owns 64 voxels (4 row
// blocks of 16 along x) x 32 output channels (2 column blocks): 8 accumulators, 27
// taps x one K step of 8 MFMAs.  The backward data pass is the same kernel on reflected,
// transposed weights with the ReLU mask of the layer below; the weight gradient is a
// GEMM over voxels per tap (MFMA with K along voxels) added atomically into FP32.
// Master weights and Adam moments are FP32; the BF16 copies are refreshed after each
// update.
//
// Conventions (shared with the FP64 reference, implemented independently there): tap
// t = (dz+1)*9 + (dy+1)*3 + (dx+1); y[v][co] = b[co] + sum_{t,ci} W[t][ci][co] x[v+off(t)][ci];
// parameters in order, per layer: W [27][cin][cout], then b [cout].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "../../include/mhd950.h"
#include "launch.hpp"

using namespace mhd;

namespace {

constexpr int kLayers = 4;
constexpr int kCin[kLayers] = {8, 32, 32, 32};
constexpr int kCout[kLayers] = {32, 32, 32, 18};
constexpr int kCinPad[kLayers] = {16, 32, 32, 32};
constexpr int kNPad = 32;        // padded output width of every layer
constexpr int kThreads = 256;    // 4 wavefronts
constexpr int kVoxPerWave = 64;

typedef unsigned short bf16_t;
typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// One 16 x 16 output block times a K chunk: 32 channels per instruction
// (v_mfma_f32_16x16x32_bf16: lane l holds A row l % 16 and B column l % 16 at K
// 8 (l / 16) + 0..7; checked on the device) where the layer input is a multiple of 32
// channels wide, else 16 (v_mfma_f32_16x16x16_bf16, K 4 (l / 16) + 0..3).  Both
// convolution forms step through K the same way, so they give the same bits.
__device__ __forceinline__ f4 mfma_k32(s4 alo, s4 ahi, s8 b, f4 c)
{
    const s8 a = {alo[0], alo[1], alo[2], alo[3], ahi[0], ahi[1], ahi[2], ahi[3]};
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

constexpr size_t layer_w(int l) { return (size_t)27 * kCin[l] * kCout[l]; }
constexpr size_t layer_params(int l) { return layer_w(l) + kCout[l]; }
size_t param_offset(int l)
{
    size_t o = 0;
    for (int q = 0; q < l; ++q) o += layer_params(q);
    return o;
}
size_t total_params() { return param_offset(kLayers); }

__device__ __forceinline__ bf16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// voxel index of (x, y, z) displaced by tap t
__device__ __forceinline__ unsigned int tap_voxel(const Geo& g, int x, int y, int z, int t)
{
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    return ((unsigned int)wrap1(z + dz, g.nz) * (unsigned int)g.ny + (unsigned int)wrap1(y + dy, g.ny)) *
               (unsigned int)g.nx + (unsigned int)wrap1(x + dx, g.nx);
}

}  // namespace

namespace mhd {

// ----------------------------------------------------------------------------------
// kernels
// ----------------------------------------------------------------------------------

// Normalised primitive channels of a canonical FP64 state -> X0 [n][16] (8 used).
__global__ __launch_bounds__(kThreads) void k_cnn_input(Geo g, double gamma, const double* __restrict__ U,
                                                        const float* __restrict__ mu, const float* __restrict__ sd,
                                                        bf16_t* __restrict__ X0)
{
    const unsigned int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= (unsigned int)g.n) return;
    const unsigned int n = (unsigned int)g.n;
    const int x = (int)(c % (unsigned int)g.nx), y = (int)((c / (unsigned int)g.nx) % (unsigned int)g.ny);
    const int z = (int)(c / ((unsigned int)g.nx * (unsigned int)g.ny));
    const unsigned int cx = tap_voxel(g, x, y, z, 14), cy = tap_voxel(g, x, y, z, 16), cz = tap_voxel(g, x, y, z, 22);
    const double rho = U[c];
    const double v[3] = {U[n + c] / rho, U[2 * n + c] / rho, U[3 * n + c] / rho};
    const double b[3] = {0.5 * (U[5 * n + c] + U[5 * n + cx]), 0.5 * (U[6 * n + c] + U[6 * n + cy]),
                         0.5 * (U[7 * n + c] + U[7 * n + cz])};
    const double ke = 0.5 * rho * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
    const double p = (gamma - 1.0) * ((U[4 * n + c] - ke) - 0.5 * ((b[0] * b[0] + b[1] * b[1]) + b[2] * b[2]));
    const double w[8] = {rho, v[0], v[1], v[2], p, b[0], b[1], b[2]};
    // the voxel's 16 channels (8 used, 8 zero padding) as two 16-byte stores
    uint32_t h[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        h[q] = (uint32_t)f2bf((float)((w[2 * q] - mu[2 * q]) / sd[2 * q])) |
               (uint32_t)f2bf((float)((w[2 * q + 1] - mu[2 * q + 1]) / sd[2 * q + 1])) << 16;
    uint4* o = reinterpret_cast<uint4*>(X0 + (size_t)c * 16);
    o[0] = uint4{h[0], h[1], h[2], h[3]};
    o[1] = uint4{0u, 0u, 0u, 0u};
}

// Y[v][nn] = sum_t sum_k X[v + off(t)][k] B[t][nn][k] (+ bias), 32 outputs.
// MODE 0: + bias, ReLU, store BF16 [n][32].  MODE 1: + bias, store FP32 planar O[nn][v]
// for nn < nstore.  MODE 2: times (M[v][nn] > 0), store BF16 [n][32].
template <int CINP, int MODE>
__global__ __launch_bounds__(kThreads) void k_conv(Geo g, const bf16_t* __restrict__ X, const bf16_t* __restrict__ B,
                                                   const float* __restrict__ bias, const bf16_t* __restrict__ M,
                                                   bf16_t* __restrict__ Y, float* __restrict__ O, int nstore)
{
    const int lane = threadIdx.x & 63;
    const unsigned int v0 = (blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6)) * kVoxPerWave;
    const unsigned int n = (unsigned int)g.n;
    if (v0 >= n) return;  // the whole wavefront (n is a multiple of 16, blocks of 16 stay in one row)
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    int bx[4], by[4], bz[4];
    bool live[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        const unsigned int vb = v0 + rb * 16;
        live[rb] = vb < n;
        const unsigned int vv = live[rb] ? vb : v0;
        bx[rb] = (int)(vv % (unsigned int)g.nx) + lr;
        by[rb] = (int)((vv / (unsigned int)g.nx) % (unsigned int)g.ny);
        bz[rb] = (int)(vv / ((unsigned int)g.nx * (unsigned int)g.ny));
    }
    f4 acc[4][2];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < 27; ++t) {
        unsigned int vs[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) vs[rb] = tap_voxel(g, bx[rb], by[rb], bz[rb], t);
        if constexpr (CINP % 32 == 0) {
            const int lk8 = (lane >> 4) * 8;
#pragma unroll
            for (int kc = 0; kc < CINP / 32; ++kc) {
                s8 bf[2];
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    bf[cb] = *reinterpret_cast<const s8*>(B + ((size_t)(t * kNPad + cb * 16 + lr) * CINP + kc * 32 + lk8));
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const bf16_t* xa = X + ((size_t)vs[rb] * CINP + kc * 32 + lk8);
                    const s4 alo = *reinterpret_cast<const s4*>(xa), ahi = *reinterpret_cast<const s4*>(xa + 4);
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = mfma_k32(alo, ahi, bf[cb], acc[rb][cb]);
                }
            }
        } else {
#pragma unroll
            for (int kc = 0; kc < CINP / 16; ++kc) {
                s4 bf[2];
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    bf[cb] = *reinterpret_cast<const s4*>(B + ((size_t)(t * kNPad + cb * 16 + lr) * CINP + kc * 16 + lk));
#pragma unroll
                for (int rb = 0; rb < 4; ++rb) {
                    const s4 af = *reinterpret_cast<const s4*>(X + ((size_t)vs[rb] * CINP + kc * 16 + lk));
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af, bf[cb], acc[rb][cb], 0, 0, 0);
                }
            }
        }
    }
    // accumulator element i of lane l: row (voxel) 4*(l/16) + i, column (channel) l % 16
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        if (!live[rb]) continue;
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const int nn = cb * 16 + lr;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const unsigned int v = v0 + rb * 16 + lk + i;
                float val = acc[rb][cb][i];
                if (MODE == 0) {
                    val = fmaxf(val + bias[nn], 0.f);
                    Y[(size_t)v * kNPad + nn] = f2bf(val);
                } else if (MODE == 1) {
                    if (nn < nstore) O[(size_t)nn * n + v] = val + bias[nn];
                } else {
                    if (!(bf2f(M[(size_t)v * kNPad + nn]) > 0.f)) val = 0.f;
                    Y[(size_t)v * kNPad + nn] = f2bf(val);
                }
            }
        }
    }
}

// The same convolution with its input staged in LDS: one workgroup computes a
// 16 x 4 x 4TZ block of voxels (wave w the 4 rows of planes z0 + TZ w ..), and the
// block's input with a one-voxel halo, 18 x 6 x (4TZ + 2) voxels of CINP channels, is
// read from memory once into LDS instead of once per tap; every tap's A fragments then
// come from LDS.  The accumulation order (taps, then K chunks) is that of k_conv, so
// the results are bitwise the same.  Needs ny a multiple of 4 and nz one of 4TZ (nx is
// one of 16).
constexpr int kTileY = 4;

// TZ: planes per wavefront (the block is 16 x 4 x 4 TZ voxels)
template <int CINP, int MODE, int TZ>
__global__ __launch_bounds__(kThreads) void k_conv_lds(Geo g, const bf16_t* __restrict__ X,
                                                       const bf16_t* __restrict__ B,
                                                       const float* __restrict__ bias,
                                                       const bf16_t* __restrict__ M, bf16_t* __restrict__ Y,
                                                       float* __restrict__ O, int nstore)
{
    constexpr int CSTR = CINP + 4;  // channels per staged voxel, padded (8-byte aligned rows)
    constexpr int kTileZ = 4 * TZ, kHalo = 18 * (kTileY + 2) * (kTileZ + 2);
    constexpr int NRB = 4 * TZ;     // 16-voxel row blocks per wavefront
    __shared__ __align__(16) bf16_t sA[kTileZ + 2][kTileY + 2][18][CSTR];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned int ntx = (unsigned int)g.nx / 16u, nty = (unsigned int)g.ny / kTileY;
    const unsigned int b = blockIdx.x;
    const int x0 = (int)(b % ntx) * 16;
    const int y0 = (int)((b / ntx) % nty) * kTileY;
    const int z0 = (int)(b / (ntx * nty)) * kTileZ;
    const unsigned int n = (unsigned int)g.n;

    // stage the input block with its halo (periodic), 16 bytes per load (two 8-byte LDS
    // writes: the padded LDS rows are 8-byte aligned only)
    constexpr int CH = CINP / 8;
    for (int q = threadIdx.x; q < kHalo * CH; q += kThreads) {
        const int vq = q / CH, part = q - vq * CH;
        const int lx = vq % 18, ly = (vq / 18) % (kTileY + 2), lz = vq / (18 * (kTileY + 2));
        const unsigned int gv = ((unsigned int)wrap1(z0 + lz - 1, g.nz) * (unsigned int)g.ny +
                                 (unsigned int)wrap1(y0 + ly - 1, g.ny)) * (unsigned int)g.nx +
                                (unsigned int)wrap1(x0 + lx - 1, g.nx);
        const uint4 v = *reinterpret_cast<const uint4*>(X + (size_t)gv * CINP + part * 8);
        *reinterpret_cast<uint2*>(&sA[lz][ly][lx][part * 8]) = uint2{v.x, v.y};
        *reinterpret_cast<uint2*>(&sA[lz][ly][lx][part * 8 + 4]) = uint2{v.z, v.w};
    }
    __syncthreads();

    const int lr = lane & 15, lk = (lane >> 4) * 4;
    // row block rb of wave w: row y0 + rb % 4 of plane z0 + TZ w + rb / 4
    f4 acc[NRB][2];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = f4{0.f, 0.f, 0.f, 0.f};
    // The weight fragments of tap t + 1 are loaded while tap t multiplies: they come from
    // L2 (a layer's weights do not fit L1), and waiting for them at every tap left the
    // matrix cores idle most of the time.
    if constexpr (CINP % 32 == 0) {
        const int lk8 = (lane >> 4) * 8;
        auto load_b = [&](int t, s8 (&bf)[CINP / 32][2]) {
#pragma unroll
            for (int kc = 0; kc < CINP / 32; ++kc)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    bf[kc][cb] = *reinterpret_cast<const s8*>(
                        B + ((size_t)(t * kNPad + cb * 16 + lr) * CINP + kc * 32 + lk8));
        };
        s8 bcur[CINP / 32][2], bnxt[CINP / 32][2];
        load_b(0, bcur);
        for (int t = 0; t < 27; ++t) {
            const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
            load_b(t < 26 ? t + 1 : t, bnxt);
#pragma unroll
            for (int kc = 0; kc < CINP / 32; ++kc) {
#pragma unroll
                for (int rb = 0; rb < NRB; ++rb) {
                    // two 8-byte reads: the padded LDS rows are 8-byte aligned only
                    const bf16_t* xa = &sA[TZ * w + rb / 4 + dz + 1][rb % 4 + dy + 1][lr + dx + 1][kc * 32 + lk8];
                    const s4 alo = *reinterpret_cast<const s4*>(xa), ahi = *reinterpret_cast<const s4*>(xa + 4);
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = mfma_k32(alo, ahi, bcur[kc][cb], acc[rb][cb]);
                }
            }
#pragma unroll
            for (int kc = 0; kc < CINP / 32; ++kc)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb) bcur[kc][cb] = bnxt[kc][cb];
        }
    } else {
        for (int t = 0; t < 27; ++t) {
            const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
#pragma unroll
            for (int kc = 0; kc < CINP / 16; ++kc) {
                s4 bf[2];
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    bf[cb] = *reinterpret_cast<const s4*>(B + ((size_t)(t * kNPad + cb * 16 + lr) * CINP + kc * 16 + lk));
#pragma unroll
                for (int rb = 0; rb < NRB; ++rb) {
                    const s4 af = *reinterpret_cast<const s4*>(
                        &sA[TZ * w + rb / 4 + dz + 1][rb % 4 + dy + 1][lr + dx + 1][kc * 16 + lk]);
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af, bf[cb], acc[rb][cb], 0, 0, 0);
                }
            }
        }
    }
    // accumulator element i of lane l: row (voxel) 4*(l/16) + i, column (channel) l % 16
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
        const unsigned int vrow = ((unsigned int)(z0 + TZ * w + rb / 4) * (unsigned int)g.ny +
                                   (unsigned int)(y0 + rb % 4)) * (unsigned int)g.nx + (unsigned int)x0;
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
            const int nn = cb * 16 + lr;
            if constexpr (MODE == 1) {
                // the four voxels of a lane are consecutive: one 16-byte store
                if (nn < nstore) {
                    const float b = bias[nn];
                    const float4 o4 = {acc[rb][cb][0] + b, acc[rb][cb][1] + b, acc[rb][cb][2] + b,
                                       acc[rb][cb][3] + b};
                    *reinterpret_cast<float4*>(O + (size_t)nn * n + vrow + lk) = o4;
                }
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const unsigned int v = vrow + lk + i;
                    float val = acc[rb][cb][i];
                    if (MODE == 0) {
                        val = fmaxf(val + bias[nn], 0.f);
                    } else {
                        if (!(bf2f(M[(size_t)v * kNPad + nn]) > 0.f)) val = 0.f;
                    }
                    Y[(size_t)v * kNPad + nn] = f2bf(val);
                }
            }
        }
    }
}

// dW[t][k][nn] += sum_v X[v + off(t)][k] D[v][nn] over a chunk of voxels per wavefront,
// added into the canonical FP32 gradient of the layer (k < cin, nn < cout only).
template <int CINP>
__global__ __launch_bounds__(kThreads) void k_wgrad(Geo g, const bf16_t* __restrict__ X, const bf16_t* __restrict__ D,
                                                    float* __restrict__ G, int cin, int cout, unsigned int vchunk)
{
    const int lane = threadIdx.x & 63;
    const unsigned int wid = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int t = (int)(wid % 27u);
    const unsigned int vbeg = (wid / 27u) * vchunk;
    const unsigned int n = (unsigned int)g.n;
    if (vbeg >= n) return;
    const unsigned int vend = vbeg + vchunk < n ? vbeg + vchunk : n;
    const int lr = lane & 15, lk = (lane >> 4) * 4;
    f4 acc[CINP / 16][2];
#pragma unroll
    for (int mb = 0; mb < CINP / 16; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = f4{0.f, 0.f, 0.f, 0.f};
    for (unsigned int vb = vbeg; vb < vend; vb += 16) {
        unsigned int vx[4];
        unsigned int vd[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const unsigned int v = vb + lk + j;  // < vend: chunks are multiples of 16 and n is too
            vd[j] = v;
            const int x = (int)(v % (unsigned int)g.nx), y = (int)((v / (unsigned int)g.nx) % (unsigned int)g.ny);
            const int z = (int)(v / ((unsigned int)g.nx * (unsigned int)g.ny));
            vx[j] = tap_voxel(g, x, y, z, t);
        }
        s4 a[CINP / 16], b[2];
#pragma unroll
        for (int mb = 0; mb < CINP / 16; ++mb)
#pragma unroll
            for (int j = 0; j < 4; ++j) a[mb][j] = (short)X[(size_t)vx[j] * CINP + mb * 16 + lr];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int j = 0; j < 4; ++j) b[nb][j] = (short)D[(size_t)vd[j] * kNPad + nb * 16 + lr];
#pragma unroll
        for (int mb = 0; mb < CINP / 16; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[mb], b[nb], acc[mb][nb], 0, 0, 0);
    }
#pragma unroll
    for (int mb = 0; mb < CINP / 16; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int k = mb * 16 + lk + i, nn = nb * 16 + lr;
                if (k < cin && nn < cout) atomicAdd(&G[((size_t)t * cin + k) * cout + nn], acc[mb][nb][i]);
            }
}

// db[nn] += sum_v D[v][nn]
__global__ __launch_bounds__(kThreads) void k_bgrad(Geo g, const bf16_t* __restrict__ D, float* __restrict__ G, int cout)
{
    __shared__ float s[kThreads];
    const int nn = threadIdx.x & 31, part = threadIdx.x >> 5;  // 8 voxel lanes per channel
    float acc = 0.f;
    const unsigned int n = (unsigned int)g.n;
    for (unsigned int v = blockIdx.x * 8 + part; v < n; v += gridDim.x * 8) acc += bf2f(D[(size_t)v * kNPad + nn]);
    s[threadIdx.x] = acc;
    __syncthreads();
    if (part == 0 && nn < cout) {
        float t = 0.f;
        for (int q = 0; q < 8; ++q) t += s[q * 32 + nn];
        atomicAdd(&G[nn], t);
    }
}

// The closure in flux and constrained-transport form: the corrected value of field q of
// cell c (q < 5: the cell field minus dt times the divergence of the face-flux
// corrections; q >= 5: the face field minus dt times the curl of the edge-EMF
// corrections).  Shared by the check and the update so that both see the same bits.
struct CorrIdx {
    unsigned int c, cp[3];  // the cell and its +x, +y, +z neighbours
};
__device__ __forceinline__ CorrIdx corr_idx(const Geo& g, unsigned int c)
{
    const int x = (int)(c % (unsigned int)g.nx), y = (int)((c / (unsigned int)g.nx) % (unsigned int)g.ny);
    const int z = (int)(c / ((unsigned int)g.nx * (unsigned int)g.ny));
    return CorrIdx{c, {tap_voxel(g, x, y, z, 14), tap_voxel(g, x, y, z, 16), tap_voxel(g, x, y, z, 22)}};
}
__device__ __forceinline__ double corrected(const Geo& g, const float* __restrict__ O, const float* __restrict__ sF,
                                            float sE, double dt, const double* __restrict__ U, const CorrIdx& k, int q)
{
    const unsigned int n = (unsigned int)g.n, c = k.c;
    if (q < 5) {
        double div = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float* o = O + (size_t)(3 * q + d) * n;
            div += (double)sF[q] * ((double)o[k.cp[d]] - (double)o[c]) * g.inv_dx[d];
        }
        return U[(size_t)q * n + c] - dt * div;
    }
    const float* Ex = O + (size_t)15 * n;
    const float* Ey = O + (size_t)16 * n;
    const float* Ez = O + (size_t)17 * n;
    auto dE = [&](const float* e, int d) { return (double)sE * ((double)e[k.cp[d]] - (double)e[c]) * g.inv_dx[d]; };
    const double curl = q == 5 ? dE(Ez, 1) - dE(Ey, 2) : (q == 6 ? dE(Ex, 2) - dE(Ez, 0) : dE(Ey, 0) - dE(Ex, 1));
    return U[(size_t)q * n + c] - dt * curl;
}

// The closure on a canonical FP64 state, in place (each thread writes only its own cell
// and faces; O is read-only).  With ok non-null nothing is written unless *ok > 0.
__global__ __launch_bounds__(kThreads) void k_closure_apply(Geo g, const float* __restrict__ O, const float* __restrict__ sF,
                                                            float sE, double dt, double* __restrict__ U,
                                                            const double* __restrict__ ok)
{
    const unsigned int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= (unsigned int)g.n) return;
    if (ok && !(ok[0] > 0.0)) return;
    const CorrIdx k = corr_idx(g, c);
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = corrected(g, O, sF, sE, dt, U, k, q);
#pragma unroll
    for (int q = 0; q < 8; ++q) U[(size_t)q * g.n + c] = v[q];
}

// Whether the closure would leave cell c valid: every corrected value finite, the density
// and the pressure (from the corrected total energy, momenta and the mean of the
// corrected bounding faces) at or above the floors.  One partial per workgroup: +inf if
// all its cells are valid, else -1.
__global__ __launch_bounds__(kThreads) void k_closure_check(Geo g, const float* __restrict__ O, const float* __restrict__ sF,
                                                            float sE, double dt, const double* __restrict__ U,
                                                            double gamma, double rho_floor, double p_floor,
                                                            double* __restrict__ partial)
{
    const unsigned int c = blockIdx.x * kThreads + threadIdx.x;
    bool good = true;
    if (c < (unsigned int)g.n) {
        const CorrIdx k = corr_idx(g, c);
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = corrected(g, O, sF, sE, dt, U, k, q);
        const double hi[3] = {corrected(g, O, sF, sE, dt, U, corr_idx(g, k.cp[0]), 5),
                              corrected(g, O, sF, sE, dt, U, corr_idx(g, k.cp[1]), 6),
                              corrected(g, O, sF, sE, dt, U, corr_idx(g, k.cp[2]), 7)};
        double bb = 0.0, mm = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double b = 0.5 * (v[5 + d] + hi[d]);
            bb += b * b;
            mm += v[1 + d] * v[1 + d];
        }
        const double p = (gamma - 1.0) * (v[4] - 0.5 * mm / v[0] - 0.5 * bb);
        for (int q = 0; q < 8; ++q) good = good && isfinite(v[q]);
        good = good && isfinite(hi[0]) && isfinite(hi[1]) && isfinite(hi[2]);
        good = good && v[0] >= rho_floor && p >= p_floor && isfinite(p);
    }
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    if (!good) atomicOr(&bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = bad ? -1.0 : INFINITY;
}

// rw[f][c] = 2 w_f (P - T) / n and the loss partial sum_f w_f (P - T)^2 / n per block.
__global__ __launch_bounds__(kThreads) void k_residual(Geo g, const double* __restrict__ P, const double* __restrict__ T,
                                                       const float* __restrict__ w8, float* __restrict__ RW,
                                                       double* __restrict__ partial)
{
    __shared__ double s[kThreads / 64];
    const unsigned int c = blockIdx.x * kThreads + threadIdx.x;
    const unsigned int n = (unsigned int)g.n;
    double l = 0.0;
    if (c < n) {
#pragma unroll
        for (int f = 0; f < 8; ++f) {
            const double r = P[(size_t)f * n + c] - T[(size_t)f * n + c];
            RW[(size_t)f * n + c] = (float)(2.0 * w8[f] * r / (double)n);
            l += w8[f] * r * r / (double)n;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

// d(loss)/d(output channel) through the adjoints of the closure, as BF16 [n][32].
__global__ __launch_bounds__(kThreads) void k_out_grad(Geo g, const float* __restrict__ RW, const float* __restrict__ sF,
                                                       float sE, double dt, bf16_t* __restrict__ D)
{
    const unsigned int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= (unsigned int)g.n) return;
    const unsigned int n = (unsigned int)g.n;
    const int x = (int)(c % (unsigned int)g.nx), y = (int)((c / (unsigned int)g.nx) % (unsigned int)g.ny);
    const int z = (int)(c / ((unsigned int)g.nx * (unsigned int)g.ny));
    // c - e_d
    const unsigned int cm[3] = {tap_voxel(g, x, y, z, 12), tap_voxel(g, x, y, z, 10), tap_voxel(g, x, y, z, 4)};
    bf16_t* o = D + (size_t)c * kNPad;
    // dF_fd[c] enters u_f[c] with +dt/dx_d and u_f[c - e_d] with -dt/dx_d
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        const float* r = RW + (size_t)f * n;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            o[3 * f + d] = f2bf((float)((double)sF[f] * dt * g.inv_dx[d] * ((double)r[c] - (double)r[cm[d]])));
    }
    const float* gx = RW + (size_t)5 * n;
    const float* gy = RW + (size_t)6 * n;
    const float* gz = RW + (size_t)7 * n;
    auto dd = [&](const float* r, int d) { return dt * g.inv_dx[d] * ((double)r[c] - (double)r[cm[d]]); };
    o[15] = f2bf((float)(sE * (dd(gy, 2) - dd(gz, 1))));
    o[16] = f2bf((float)(sE * (dd(gz, 0) - dd(gx, 2))));
    o[17] = f2bf((float)(sE * (dd(gx, 1) - dd(gy, 0))));
#pragma unroll
    for (int q = 18; q < kNPad; ++q) o[q] = 0;
}

// BF16 weight copies of layer l from the FP32 master: forward Wf[t][nn][k] = W[t][k][nn];
// backward Wb[t][nn=ci][k=co] = W[27-1-t][ci][co] (reflected tap).  Zero padded.
__global__ __launch_bounds__(kThreads) void k_pack_weights(const float* __restrict__ W, int cin, int cout, int cinp,
                                                           bf16_t* __restrict__ Wf, bf16_t* __restrict__ Wb)
{
    const unsigned int q = blockIdx.x * kThreads + threadIdx.x;
    if (q >= 27u * kNPad * (unsigned int)cinp) return;
    const int k = (int)(q % (unsigned int)cinp), nn = (int)((q / (unsigned int)cinp) % kNPad), t = (int)(q / ((unsigned int)cinp * kNPad));
    Wf[q] = (k < cin && nn < cout) ? f2bf(W[((size_t)t * cin + k) * cout + nn]) : (bf16_t)0;
    if (Wb) {
        // Wb[t][nn][k] with nn = ci (< cin), k = co (< cout); cinp == 32 == kNPad here
        const int ci = nn, co = k;
        Wb[q] = (ci < cin && co < cout) ? f2bf(W[((size_t)(26 - t) * cin + ci) * cout + co]) : (bf16_t)0;
    }
}

__global__ __launch_bounds__(kThreads) void k_adam(unsigned int np, float* __restrict__ P, const float* __restrict__ G,
                                                   float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                   float b2, float eps, float c1, float c2, float gscale)
{
    const unsigned int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= np) return;
    const float gr = G[i] * gscale;
    const float mi = b1 * m[i] + (1.f - b1) * gr;
    const float vi = b2 * v[i] + (1.f - b2) * gr * gr;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Box filter of a fine canonical state (r^3 cells, r^2 faces) onto the coarse grid.
__global__ __launch_bounds__(kThreads) void k_box_filter(Geo fine, Geo coarse, int r, const double* __restrict__ Fs,
                                                         double* __restrict__ Cs)
{
    const unsigned int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= (unsigned int)coarse.n) return;
    const unsigned int nf = (unsigned int)fine.n, nc = (unsigned int)coarse.n;
    const int X = (int)(c % (unsigned int)coarse.nx), Y = (int)((c / (unsigned int)coarse.nx) % (unsigned int)coarse.ny);
    const int Z = (int)(c / ((unsigned int)coarse.nx * (unsigned int)coarse.ny));
    auto fat = [&](int x, int y, int z) {
        return ((unsigned int)z * (unsigned int)fine.ny + (unsigned int)y) * (unsigned int)fine.nx + (unsigned int)x;
    };
    const double inv3 = 1.0 / (double)(r * r * r), inv2 = 1.0 / (double)(r * r);
    for (int f = 0; f < 5; ++f) {
        double s = 0.0;
        for (int k = 0; k < r; ++k)
            for (int j = 0; j < r; ++j)
                for (int i = 0; i < r; ++i) s += Fs[(size_t)f * nf + fat(X * r + i, Y * r + j, Z * r + k)];
        Cs[(size_t)f * nc + c] = s * inv3;
    }
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int a = 0; a < r; ++a)
        for (int b = 0; b < r; ++b) {
            sx += Fs[(size_t)5 * nf + fat(X * r, Y * r + b, Z * r + a)];
            sy += Fs[(size_t)6 * nf + fat(X * r + b, Y * r, Z * r + a)];
            sz += Fs[(size_t)7 * nf + fat(X * r + b, Y * r + a, Z * r)];
        }
    Cs[(size_t)5 * nc + c] = sx * inv2;
    Cs[(size_t)6 * nc + c] = sy * inv2;
    Cs[(size_t)7 * nc + c] = sz * inv2;
}

}  // namespace mhd

// ----------------------------------------------------------------------------------
// host runtime
// ----------------------------------------------------------------------------------

struct mhd_cnn {
    Geo g;
    double gamma;
    hipStream_t stream;
    size_t np;
    float *P, *G, *M1, *M2;  // parameters, gradients, Adam moments (FP32, canonical order)
    bf16_t* Wf[kLayers];
    bf16_t* Wb[kLayers];     // layers 1..3
    bf16_t* A[kLayers];      // layer inputs: A[0] = X0 [n][16], A[l] [n][32]
    float* O;                // output channels [18][n]
    bf16_t *D0, *D1;         // backward gradients [n][32]
    float* RW;               // weighted residual [8][n]
    double* Pred;            // corrected prediction [8][n]
    double* partial;
    float* scal;             // mu[8], sd[8], sF[5], w8[8]
    float sE;
    unsigned int nblk;
};

namespace {

size_t ca(size_t b) { return (b + 255) & ~size_t(255); }

struct CLayout {
    size_t params, wf[kLayers], wb[kLayers], a[kLayers], o, d, rw, pred, partial, scal, total;
};

CLayout clayout(const mhd_grid* g)
{
    const size_t n = (size_t)g->nx * g->ny * g->nz;
    CLayout L;
    L.params = ca(total_params() * sizeof(float));
    for (int l = 0; l < kLayers; ++l) {
        L.wf[l] = ca((size_t)27 * kNPad * kCinPad[l] * sizeof(bf16_t));
        L.wb[l] = l > 0 ? ca((size_t)27 * kNPad * kNPad * sizeof(bf16_t)) : 0;
        L.a[l] = ca(n * (l == 0 ? 16 : kNPad) * sizeof(bf16_t));
    }
    L.o = ca(n * 18 * sizeof(float));
    L.d = ca(n * kNPad * sizeof(bf16_t));
    L.rw = ca(n * 8 * sizeof(float));
    L.pred = ca(n * 8 * sizeof(double));
    L.partial = ca(((n + kThreads - 1) / kThreads + 1) * sizeof(double));  // + the closure's flag
    L.scal = ca(64 * sizeof(float));
    L.total = 4 * L.params + L.o + 2 * L.d + L.rw + L.pred + L.partial + L.scal;
    for (int l = 0; l < kLayers; ++l) L.total += L.wf[l] + L.wb[l] + L.a[l];
    return L;
}

mhd_status cvalidate(const mhd_grid* g, const mhd_physics* p)
{
    if (!g || !p) return MHD_E_INVAL;
    if (g->nx < 16 || g->ny < 1 || g->nz < 1) return MHD_E_INVAL;
    if (g->nx % 16 != 0) return MHD_E_UNSUPPORTED;  // MFMA row blocks of 16 voxels along x
    for (int a = 0; a < 3; ++a)
        if (!(g->length[a] > 0.0) || !std::isfinite(g->length[a])) return MHD_E_INVAL;
    if ((long long)g->nx * g->ny * g->nz >= (1LL << 26)) return MHD_E_UNSUPPORTED;
    if (p->eos != MHD_EOS_ADIABATIC_MHD || !(p->gamma > 1.0)) return MHD_E_UNSUPPORTED;
    return MHD_OK;
}

mhd_status cdev(hipError_t e) { return e == hipSuccess ? MHD_OK : MHD_E_DEVICE; }

unsigned int conv_blocks(const mhd_cnn* c)
{
    const unsigned int waves = (unsigned int)((c->g.n + kVoxPerWave - 1) / kVoxPerWave);
    return (waves + 3) / 4;
}

hipError_t pack_all(mhd_cnn* c)
{
    for (int l = 0; l < kLayers; ++l) {
        const unsigned int cnt = 27u * kNPad * kCinPad[l];
        hipLaunchKernelGGL(k_pack_weights, dim3((cnt + kThreads - 1) / kThreads), dim3(kThreads), 0, c->stream,
                           c->P + param_offset(l), kCin[l], kCout[l], kCinPad[l], c->Wf[l], l > 0 ? c->Wb[l] : nullptr);
    }
    return hipGetLastError();
}

// One convolution launch: the LDS-staged kernel where the grid tiles into 16 x 4 x 8 or
// 16 x 4 x 4 blocks, else the per-tap gather kernel (all give the same bits).
template <int CINP, int MODE>
void conv(const mhd_cnn* c, const bf16_t* X, const bf16_t* B, const float* bias, const bf16_t* M, bf16_t* Y,
          float* O, int nstore)
{
    if (c->g.ny % kTileY == 0 && c->g.nz % 8 == 0) {
        // 16 x 4 x 8 blocks, two planes per wavefront (78 KB of LDS: two workgroups per CU)
        const unsigned int nblk = (unsigned int)(c->g.n / (16 * kTileY * 8));
        hipLaunchKernelGGL((k_conv_lds<CINP, MODE, 2>), dim3(nblk), dim3(kThreads), 0, c->stream, c->g, X, B, bias,
                           M, Y, O, nstore);
    } else if (c->g.ny % kTileY == 0 && c->g.nz % 4 == 0) {
        const unsigned int nblk = (unsigned int)(c->g.n / (16 * kTileY * 4));
        hipLaunchKernelGGL((k_conv_lds<CINP, MODE, 1>), dim3(nblk), dim3(kThreads), 0, c->stream, c->g, X, B, bias,
                           M, Y, O, nstore);
    } else {
        hipLaunchKernelGGL((k_conv<CINP, MODE>), dim3(conv_blocks(c)), dim3(kThreads), 0, c->stream, c->g, X, B,
                           bias, M, Y, O, nstore);
    }
}

// forward pass from a canonical state; keeps every layer input for the backward pass
hipError_t forward(mhd_cnn* c, const double* U)
{
    hipLaunchKernelGGL(k_cnn_input, dim3(c->nblk), dim3(kThreads), 0, c->stream, c->g, c->gamma, U, c->scal,
                       c->scal + 8, c->A[0]);
    conv<16, 0>(c, c->A[0], c->Wf[0], c->P + param_offset(0) + layer_w(0), nullptr, c->A[1], nullptr, 0);
    conv<32, 0>(c, c->A[1], c->Wf[1], c->P + param_offset(1) + layer_w(1), nullptr, c->A[2], nullptr, 0);
    conv<32, 0>(c, c->A[2], c->Wf[2], c->P + param_offset(2) + layer_w(2), nullptr, c->A[3], nullptr, 0);
    conv<32, 1>(c, c->A[3], c->Wf[3], c->P + param_offset(3) + layer_w(3), nullptr, nullptr, c->O, 18);
    return hipGetLastError();
}

hipError_t apply(mhd_cnn* c, double dt, double* U, const double* ok = nullptr)
{
    hipLaunchKernelGGL(k_closure_apply, dim3(c->nblk), dim3(kThreads), 0, c->stream, c->g, c->O, c->scal + 16, c->sE,
                       dt, U, ok);
    return hipGetLastError();
}

// flag[0] = +inf if the closure leaves every cell of U valid, else -1 (partials in
// c->partial, the flag just after them).
hipError_t check(mhd_cnn* c, double dt, const double* U, const MhdParams& mp, double* flag)
{
    hipLaunchKernelGGL(k_closure_check, dim3(c->nblk), dim3(kThreads), 0, c->stream, c->g, c->O, c->scal + 16, c->sE,
                       dt, U, c->gamma, mp.rho_floor, mp.p_floor, c->partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_min_final(c->partial, c->nblk, 1.0, flag, c->stream);
}

}  // namespace

extern "C" {

mhd_status mhd_cnn_param_count(size_t* n)
{
    if (!n) return MHD_E_INVAL;
    *n = total_params();
    return MHD_OK;
}

mhd_status mhd_cnn_workspace_bytes(const mhd_grid* grid, const mhd_physics* phys, size_t* bytes)
{
    if (!bytes) return MHD_E_INVAL;
    const mhd_status st = cvalidate(grid, phys);
    if (st != MHD_OK) return st;
    *bytes = clayout(grid).total;
    return MHD_OK;
}

mhd_status mhd_cnn_create(const mhd_grid* grid, const mhd_physics* phys, void* workspace, size_t bytes,
                          void* hip_stream, mhd_cnn** out)
{
    if (!out) return MHD_E_INVAL;
    *out = nullptr;
    mhd_status st = cvalidate(grid, phys);
    if (st != MHD_OK) return st;
    if (!workspace || ((uintptr_t)workspace & 255u)) return MHD_E_INVAL;
    const CLayout L = clayout(grid);
    if (bytes < L.total) return MHD_E_NOMEM;
    mhd_cnn* c = new (std::nothrow) mhd_cnn();
    if (!c) return MHD_E_NOMEM;
    c->g.nx = grid->nx; c->g.ny = grid->ny; c->g.nz = grid->nz;
    c->g.n = (long long)grid->nx * grid->ny * grid->nz;
    const int ns[3] = {grid->nx, grid->ny, grid->nz};
    for (int a = 0; a < 3; ++a) {
        c->g.dx[a] = grid->length[a] / ns[a];
        c->g.inv_dx[a] = 1.0 / c->g.dx[a];
    }
    c->gamma = phys->gamma;
    c->stream = (hipStream_t)hip_stream;
    c->np = total_params();
    c->nblk = (unsigned int)((c->g.n + kThreads - 1) / kThreads);
    char* p = (char*)workspace;
    c->P = (float*)p; p += L.params;
    c->G = (float*)p; p += L.params;
    c->M1 = (float*)p; p += L.params;
    c->M2 = (float*)p; p += L.params;
    for (int l = 0; l < kLayers; ++l) {
        c->Wf[l] = (bf16_t*)p; p += L.wf[l];
        c->Wb[l] = L.wb[l] ? (bf16_t*)p : nullptr; p += L.wb[l];
        c->A[l] = (bf16_t*)p; p += L.a[l];
    }
    c->O = (float*)p; p += L.o;
    c->D0 = (bf16_t*)p; p += L.d;
    c->D1 = (bf16_t*)p; p += L.d;
    c->RW = (float*)p; p += L.rw;
    c->Pred = (double*)p; p += L.pred;
    c->partial = (double*)p; p += L.partial;
    c->scal = (float*)p;
    c->sE = 1.0f;
    // zero parameters, moments and gradients; unit normalisation
    std::vector<float> zero(c->np, 0.f);
    float sc[64];
    for (int q = 0; q < 64; ++q) sc[q] = q < 8 ? 0.f : 1.f;
    hipError_t e = hipMemcpyAsync(c->P, zero.data(), c->np * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->G, zero.data(), c->np * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->M1, zero.data(), c->np * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->M2, zero.data(), c->np * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->scal, sc, sizeof(sc), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = pack_all(c);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete c;
        return MHD_E_DEVICE;
    }
    *out = c;
    return MHD_OK;
}

mhd_status mhd_cnn_set_params(mhd_cnn* c, const float* params)
{
    if (!c || !params) return MHD_E_INVAL;
    hipError_t e = hipMemcpyAsync(c->P, params, c->np * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = pack_all(c);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return cdev(e);
}

mhd_status mhd_cnn_get_params(mhd_cnn* c, float* params)
{
    if (!c || !params) return MHD_E_INVAL;
    hipError_t e = hipMemcpyAsync(params, c->P, c->np * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return cdev(e);
}

mhd_status mhd_cnn_get_grads(mhd_cnn* c, float* grads)
{
    if (!c || !grads) return MHD_E_INVAL;
    hipError_t e = hipMemcpyAsync(grads, c->G, c->np * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return cdev(e);
}

mhd_status mhd_cnn_set_scales(mhd_cnn* c, const float* mu, const float* sd, const float* sF, float sE,
                              const float* wU, float wB)
{
    if (!c || !mu || !sd || !sF || !wU) return MHD_E_INVAL;
    float sc[64] = {0};
    for (int q = 0; q < 8; ++q) {
        if (!(sd[q] > 0.f)) return MHD_E_INVAL;
        sc[q] = mu[q];
        sc[8 + q] = sd[q];
    }
    for (int q = 0; q < 5; ++q) sc[16 + q] = sF[q];
    for (int q = 0; q < 5; ++q) sc[24 + q] = wU[q];
    for (int q = 5; q < 8; ++q) sc[24 + q] = wB;
    c->sE = sE;
    hipError_t e = hipMemcpyAsync(c->scal, sc, sizeof(sc), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return cdev(e);
}

mhd_status mhd_cnn_forward(mhd_cnn* c, const double* state)
{
    if (!c || !state) return MHD_E_INVAL;
    return cdev(forward(c, state));
}

mhd_status mhd_cnn_output(mhd_cnn* c, float* dst, int dst_is_device)
{
    if (!c || !dst) return MHD_E_INVAL;
    hipError_t e = hipMemcpyAsync(dst, c->O, (size_t)c->g.n * 18 * sizeof(float),
                                  dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && !dst_is_device) e = hipStreamSynchronize(c->stream);
    return cdev(e);
}

mhd_status mhd_closure_apply(mhd_cnn* c, double dt, double* state)
{
    if (!c || !state || !(dt > 0.0) || !std::isfinite(dt)) return MHD_E_INVAL;
    return cdev(apply(c, dt, state));
}

mhd_status mhd_cnn_zero_grad(mhd_cnn* c)
{
    if (!c) return MHD_E_INVAL;
    return cdev(hipMemsetAsync(c->G, 0, c->np * sizeof(float), c->stream));
}

mhd_status mhd_cnn_accumulate(mhd_cnn* c, const double* state_t, const double* coarse_next, const double* target,
                              double dt, double* loss)
{
    if (!c || !state_t || !coarse_next || !target || !(dt > 0.0) || !std::isfinite(dt)) return MHD_E_INVAL;
    const size_t nb = (size_t)c->g.n * 8 * sizeof(double);
    hipError_t e = forward(c, state_t);
    if (e == hipSuccess) e = hipMemcpyAsync(c->Pred, coarse_next, nb, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = apply(c, dt, c->Pred);
    if (e != hipSuccess) return MHD_E_DEVICE;
    hipLaunchKernelGGL(k_residual, dim3(c->nblk), dim3(kThreads), 0, c->stream, c->g, c->Pred, target, c->scal + 24,
                       c->RW, c->partial);
    hipLaunchKernelGGL(k_out_grad, dim3(c->nblk), dim3(kThreads), 0, c->stream, c->g, c->RW, c->scal + 16, c->sE, dt,
                       c->D0);
    // backward: layer l consumes D (its output gradient) and A[l] (its input)
    const dim3 bl(kThreads);
    const unsigned int vchunk = 1024;
    const unsigned int wwaves = 27u * (unsigned int)((c->g.n + vchunk - 1) / vchunk);
    const dim3 gw((wwaves + 3) / 4);
    const unsigned int bblk = 256;
    bf16_t* D = c->D0;
    bf16_t* Dn = c->D1;
    for (int l = kLayers - 1; l >= 0 && e == hipSuccess; --l) {
        float* Gw = c->G + param_offset(l);
        float* Gb = Gw + layer_w(l);
        if (l == 0)
            hipLaunchKernelGGL((k_wgrad<16>), gw, bl, 0, c->stream, c->g, c->A[0], D, Gw, kCin[l], kCout[l], vchunk);
        else
            hipLaunchKernelGGL((k_wgrad<32>), gw, bl, 0, c->stream, c->g, c->A[l], D, Gw, kCin[l], kCout[l], vchunk);
        hipLaunchKernelGGL(k_bgrad, dim3(bblk), bl, 0, c->stream, c->g, D, Gb, kCout[l]);
        if (l > 0) {
            // gradient of layer l's input, through the ReLU of layer l-1 (mask = A[l] > 0)
            conv<32, 2>(c, D, c->Wb[l], nullptr, c->A[l], Dn, nullptr, 0);
            bf16_t* t = D;
            D = Dn;
            Dn = t;
        }
        e = hipGetLastError();
    }
    if (e != hipSuccess) return MHD_E_DEVICE;
    if (loss) {
        std::vector<double> part(c->nblk);
        e = hipMemcpyAsync(part.data(), c->partial, c->nblk * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return MHD_E_DEVICE;
        double s = 0.0;
        for (double v : part) s += v;
        *loss = s;
    }
    return MHD_OK;
}

mhd_status mhd_cnn_adam(mhd_cnn* c, float lr, float beta1, float beta2, float eps, int step, float grad_scale)
{
    if (!c || step < 1 || !(lr > 0.f)) return MHD_E_INVAL;
    const float c1 = 1.f / (1.f - std::pow(beta1, (float)step));
    const float c2 = 1.f / (1.f - std::pow(beta2, (float)step));
    hipLaunchKernelGGL(k_adam, dim3((unsigned int)((c->np + kThreads - 1) / kThreads)), dim3(kThreads), 0, c->stream,
                       (unsigned int)c->np, c->P, c->G, c->M1, c->M2, lr, beta1, beta2, eps, c1, c2, grad_scale);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = pack_all(c);
    return cdev(e);
}

mhd_status mhd_step_closure(mhd_ctx* ctx, mhd_cnn* c, double dt, int* applied)
{
    if (!ctx || !c || !(dt > 0.0) || !std::isfinite(dt)) return MHD_E_INVAL;
    CtxView v = ctx_view(ctx);
    if (!v.state) return MHD_E_UNSUPPORTED;  // FP64 adiabatic MHD contexts
    // the same grid (cells and spacing) and the same stream: the network's kernels and
    // the context's run in one order without events between them
    if (v.geo.nx != c->g.nx || v.geo.ny != c->g.ny || v.geo.nz != c->g.nz) return MHD_E_INVAL;
    for (int a = 0; a < 3; ++a)
        if (v.geo.dx[a] != c->g.dx[a]) return MHD_E_INVAL;
    if (v.stream != c->stream) return MHD_E_INVAL;
    double* flag = c->partial + c->nblk;
    // corrections from the state at the start of the step, read where it lives
    mhd_status st = cdev(forward(c, v.state));
    // the plain step, then the closure in place on the stepped state if it leaves every
    // cell finite and above the floors (else the plain step stands), and the time step
    // of the result
    if (st == MHD_OK) st = mhd_step(ctx, dt);
    if (st != MHD_OK) return st;
    v = ctx_view(ctx);
    hipError_t e = check(c, dt, v.state, v.mp, flag);
    if (e == hipSuccess) e = apply(c, dt, v.state, flag);
    if (e == hipSuccess) e = ctx_refresh_cfl(ctx);
    if (e == hipSuccess && applied) {
        double h = 0.0;
        e = hipMemcpyAsync(&h, flag, sizeof(double), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        *applied = h > 0.0 ? 1 : 0;
    }
    return cdev(e);
}

mhd_status mhd_box_filter(const mhd_grid* fine, int r, const double* fine_state, double* coarse_state, void* hip_stream)
{
    if (!fine || !fine_state || !coarse_state || r < 1) return MHD_E_INVAL;
    if (fine->nx % r || fine->ny % r || fine->nz % r) return MHD_E_INVAL;
    Geo f, c;
    f.nx = fine->nx; f.ny = fine->ny; f.nz = fine->nz;
    f.n = (long long)f.nx * f.ny * f.nz;
    c.nx = f.nx / r; c.ny = f.ny / r; c.nz = f.nz / r;
    c.n = (long long)c.nx * c.ny * c.nz;
    if (f.n >= (1LL << 29)) return MHD_E_UNSUPPORTED;
    hipLaunchKernelGGL(k_box_filter, dim3((unsigned int)((c.n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       (hipStream_t)hip_stream, f, c, r, fine_state, coarse_state);
    return cdev(hipGetLastError());
}

void mhd_cnn_destroy(mhd_cnn* c) { delete c; }

}  // extern "C"
