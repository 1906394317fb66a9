// api.hip -- host runtime behind the C ABI of mhd950.h: validation at create time,
// workspace carve-up, stage sequencing on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/mhd950.h"
#include "launch.hpp"

using namespace mhd;

// kernel classes of the event timer
enum TimerSlot {
    T_MHD_FLUX_PRED = 0,
    T_MHD_FLUX_CORR,
    T_MHD_CT_PRED,
    T_MHD_CT_CORR,
    T_CFL,
    T_DUST_PASS1,
    T_DUST_PASS2,
    T_DUST_DRAG1,
    T_DUST_DRAG2,
    T_NSLOT
};
static const char* const kSlotNames[T_NSLOT] = {
    "mhd_flux_update_predictor", "mhd_flux_update_corrector", "mhd_ct_predictor",
    "mhd_ct_corrector", "cfl", "dust_fluid_pass_stage1", "dust_fluid_pass_stage2",
    "dust_drag_stage1", "dust_drag_cfl_stage2"};

struct EventTimer {
    int cap = 0, used = 0;
    std::vector<hipEvent_t> ev;  // 2 per launch
    std::vector<int> slot;
};

struct mhd_ctx {
    mhd_grid grid;
    mhd_physics phys;
    mhd_scheme scheme;
    Geo geo;
    MhdParams mp;
    DustParams dp;
    hipStream_t stream;
    bool is_mhd;
    int nvar;       // fields of the canonical state
    long long n;    // cells
    bool fp32;      // FP32 registers: FP32-bulk MHD form, or FP32 dust (FP64 drag solve)
    // workspace views
    void* reg[3];   // state registers (MHD rotates all three; see reg_view for the layout)
    void* F;        // MHD: the 9 face fields of the edge EMFs (the path's real type)
    void* Rc;       // cell-centred E = -v x B (MHD)
    FusedGrid fg;   // tiling of the MHD stage kernels
    DustGrid dg;    // tiling of the dust fluid passes
    double* partial;
    double* scalars;  // [0] dt of the current state, [1..] diagnostics
    int cur;        // register holding the current state
    double cfl_scale;
    EventTimer* timer;
};

// Scratch of the allocation-free entry point mhd_dt_cfl_noalloc: the partial minima of
// the CFL reduction, one per workgroup of 256 cells.  A static device array, so every
// GPU the library runs on holds its own copy until the process ends.  Host code must
// not take its name as a device address: the address of each device's copy is looked
// up once per device (hipGetSymbolAddress with that device current) and kept here.
static __device__ __align__(256) double scratch[MHD_NOALLOC_MAX_CELLS / kBlock];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (looked up on the first call on that device);
// hipErrorInvalidValue if the stream belongs to another device.
hipError_t noalloc_scratch(hipStream_t s, double** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (s) {
        hipDevice_t sd = 0;
        e = hipStreamGetDevice(s, &sd);
        if (e != hipSuccess) return e;
        if ((int)sd != dev) return hipErrorInvalidValue;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct Layout {
    size_t reg, nreg, F, Rc, partial, scalars, total;
};

Geo make_geo(const mhd_grid* grid);

// z planes per workgroup of the MHD kernels: about 3072 flux/update workgroups (four
// rounds of the 768 that the FP64 PPM kernel keeps resident, three per CU; targets of
// 1536, 2304 and 4608 measured no faster at 256^3), and at least two planes per chunk.  Each chunk primes its z pipeline once (five planes for PPM),
// which small grids afford: at 64^3 chunks of 2 planes took the step from 0.355 to
// 0.192 ms against chunks of 8, with no change at 256^3.
int choose_kz(const mhd_grid* g)
{
    const long long per_plane = (long long)flux_tile_cells();
    const long long tiles = ((long long)g->nx * g->ny + per_plane - 1) / per_plane;
    const long long want = (3072 + tiles - 1) / tiles;
    int kz = (int)((g->nz + want - 1) / want);
    if (kz < 2) kz = 2;
    if (kz > g->nz) kz = g->nz;
    return kz;
}

Geo make_geo(const mhd_grid* grid)
{
    Geo g;
    g.nx = grid->nx; g.ny = grid->ny; g.nz = grid->nz;
    g.n = (long long)grid->nx * grid->ny * grid->nz;
    const int ns[3] = {grid->nx, grid->ny, grid->nz};
    for (int a = 0; a < 3; ++a) {
        g.dx[a] = grid->length[a] / ns[a];
        g.inv_dx[a] = 1.0 / g.dx[a];
    }
    return g;
}

// Kernel parameters of a validated configuration; returns the factor C C_max of eq. (cfl).
double make_params(const mhd_physics* phys, const mhd_scheme* scheme, MhdParams* mp, DustParams* dp)
{
    *mp = MhdParams{};
    *dp = DustParams{};
    mp->gamma = phys->gamma;
    mp->gm1inv = 1.0 / (phys->gamma - 1.0);
    mp->rho_floor = phys->rho_floor;
    mp->p_floor = phys->p_floor;
    // below single-precision round-off the HLLD degeneracy test would never fire
    const bool fp32 = scheme->prec == MHD_PREC_FP32_BULK;
    mp->hlld_eps = fp32 && scheme->hlld_eps < 1e-6 ? 1e-6 : scheme->hlld_eps;
    dp->nd = phys->ndust;
    dp->cs = phys->cs_iso;
    dp->rho_floor = phys->rho_floor;
    dp->dust_floor = phys->dust_rho_floor;
    for (int a = 0; a < 3; ++a) {
        mp->gacc[a] = phys->gas_accel[a];
        dp->gacc[a] = phys->gas_accel[a];
    }
    for (int k = 0; k < phys->ndust; ++k) dp->ts[k] = phys->t_stop[k];
    const double cmax = scheme->integ == MHD_INT_IMEX2P ? 1.0 / (1.0 + 1.0 / std::sqrt(2.0)) : 1.0;
    return scheme->courant * cmax;
}

int state_fields(const mhd_physics* p)
{
    return p->eos == MHD_EOS_ADIABATIC_MHD ? 8 : 4 * (1 + p->ndust);
}

mhd_status validate(const mhd_grid* g, const mhd_physics* p, const mhd_scheme* s)
{
    if (!g || !p || !s) return MHD_E_INVAL;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return MHD_E_INVAL;
    for (int a = 0; a < 3; ++a)
        if (!(g->length[a] > 0.0) || !std::isfinite(g->length[a])) return MHD_E_INVAL;
    // every field is addressed with 32-bit byte offsets: below 4 GiB, i.e. < 2^29 cells
    if ((long long)g->nx * g->ny * g->nz >= (1LL << 29)) return MHD_E_UNSUPPORTED;
    if (!(s->courant > 0.0) || !std::isfinite(s->courant)) return MHD_E_INVAL;
    if (s->prec != MHD_PREC_FP64 && s->prec != MHD_PREC_FP32_BULK) return MHD_E_UNSUPPORTED;
    if (s->recon < MHD_RECON_DC || s->recon > MHD_RECON_PPM) return MHD_E_UNSUPPORTED;
    if (s->riemann != MHD_RS_HLLE && s->riemann != MHD_RS_HLLD) return MHD_E_UNSUPPORTED;
    if (p->eos == MHD_EOS_ADIABATIC_MHD) {
        if (p->ndust != 0) return MHD_E_UNSUPPORTED;
        if (s->integ != MHD_INT_VL2 && s->integ != MHD_INT_RK2 && s->integ != MHD_INT_EULER1)
            return MHD_E_UNSUPPORTED;
        if (!(p->gamma > 1.0)) return MHD_E_INVAL;
    } else if (p->eos == MHD_EOS_ISOTHERMAL_HYDRO) {
        if (p->ndust < 1 || p->ndust > MHD_MAX_DUST) return MHD_E_UNSUPPORTED;
        if (s->integ != MHD_INT_IMEX2P) return MHD_E_UNSUPPORTED;
        if (s->riemann != MHD_RS_HLLE) return MHD_E_UNSUPPORTED;  // no isothermal HLLD here
        if (s->recon == MHD_RECON_PPM) return MHD_E_UNSUPPORTED;
        if (!(p->cs_iso > 0.0)) return MHD_E_INVAL;
        for (int k = 0; k < p->ndust; ++k)
            if (!(p->t_stop[k] > 0.0) || !std::isfinite(p->t_stop[k])) return MHD_E_INVAL;
    } else {
        return MHD_E_UNSUPPORTED;
    }
    return MHD_OK;
}

Layout layout(const mhd_grid* g, const mhd_physics* p, const mhd_scheme* sc)
{
    const long long n = (long long)g->nx * g->ny * g->nz;
    const size_t field = (size_t)n * sizeof(double);
    const int nv = state_fields(p);
    const bool is_mhd = p->eos == MHD_EOS_ADIABATIC_MHD;
    const bool fp32 = sc->prec == MHD_PREC_FP32_BULK;
    const size_t rfield = (size_t)n * (fp32 ? sizeof(float) : sizeof(double));
    Layout L;
    L.reg = is_mhd ? align256(register_bytes(n, fp32)) : align256(rfield * nv);
    L.nreg = is_mhd ? 3 : 2;
    // for the FP32 forms the flux area also stages a canonical FP64 state (nv fields);
    // the FP64 dust path keeps no arrays besides its two registers
    if (is_mhd)
        L.F = align256(rfield * 9 > field * 8 ? rfield * 9 : field * 8);
    else
        L.F = fp32 ? align256(field * nv) : 0;
    L.Rc = is_mhd ? align256(rfield * 3) : 0;
    size_t nb = blocks_for(n);
    const size_t nf = fused_grid(make_geo(g), choose_kz(g)).nblk;
    if (nf > nb) nb = nf;
    L.partial = align256(nb * sizeof(double) * (size_t)diag_count(MHD_MAX_DUST));
    L.scalars = align256(sizeof(double) * 64);
    L.total = L.nreg * L.reg + L.F + L.Rc + L.partial + L.scalars;
    return L;
}

mhd_status dev(hipError_t e) { return e == hipSuccess ? MHD_OK : MHD_E_DEVICE; }

// Event pair around one launch (no-op unless timing is on and capacity remains).
struct Tick {
    mhd_ctx* c;
    int k;
    Tick(mhd_ctx* ctx, int slot) : c(ctx), k(-1)
    {
        EventTimer* t = c->timer;
        if (t && t->used < t->cap) {
            k = t->used++;
            t->slot[k] = slot;
            (void)hipEventRecord(t->ev[2 * k], c->stream);
        }
    }
    ~Tick()
    {
        if (k >= 0) (void)hipEventRecord(c->timer->ev[2 * k + 1], c->stream);
    }
};

// FP32 register <-> canonical FP64 state of either path.
hipError_t pack_reg(mhd_ctx* c, const double* canon, void* reg)
{
    if (c->is_mhd) return launch_pack_fp32(c->geo, canon, reg, c->stream);
    return launch_dust_pack(c->n * c->nvar, canon, reg, c->stream);
}
hipError_t unpack_reg(mhd_ctx* c, const void* reg, double* canon)
{
    if (c->is_mhd) return launch_unpack_fp32(c->geo, reg, canon, c->stream);
    return launch_dust_unpack(c->n * c->nvar, reg, canon, c->stream);
}

// The current state as canonical FP64 fields on the device: the register itself for the
// FP64 forms, else unpacked into the staging area.
const double* canonical_view(mhd_ctx* c, hipError_t* e)
{
    *e = hipSuccess;
    if (!c->fp32) return (const double*)c->reg[c->cur];
    *e = unpack_reg(c, c->reg[c->cur], (double*)c->F);
    return (const double*)c->F;
}

// Compute the CFL step of a canonical FP64 state into scalars[0].
mhd_status cfl_of(mhd_ctx* c, const double* U)
{
    Tick t(c, T_CFL);
    if (c->is_mhd) return dev(launch_cfl_mhd(c->geo, c->mp, U, c->partial, c->scalars, c->cfl_scale, c->stream));
    return dev(launch_cfl_dust(c->geo, c->dp, U, c->partial, c->scalars, c->cfl_scale, c->stream));
}

// One stage: out = g0 in + g1 base + bdt L(in): the cell fields with the fluxes of
// `in`, then the face fields from the edge EMFs (and, if last, the CFL step of out into
// scalars[0]).
mhd_status mhd_stage(mhd_ctx* c, int recon, void* in, void* base, void* out, StageCoef co,
                     bool corrector, bool last)
{
    hipError_t e;
    {
        Tick t(c, corrector ? T_MHD_FLUX_CORR : T_MHD_FLUX_PRED);
        e = launch_mhd_flux3(c->geo, c->mp, c->fg, c->fp32, recon, c->scheme.riemann, in, base, out, c->F,
                             c->Rc, co, c->stream);
    }
    if (e == hipSuccess) {
        Tick t(c, corrector ? T_MHD_CT_CORR : T_MHD_CT_PRED);
        e = launch_mhd_ct_update(c->geo, c->mp, c->fg, c->fp32, in, base, c->F, c->Rc, out, co,
                                 c->partial, last ? c->scalars : nullptr, c->cfl_scale, c->stream);
    }
    return dev(e);
}

// The registers rotate: the state S = reg[cur]; stages write only to the two others.
mhd_status step_mhd(mhd_ctx* c, double dt)
{
    const int s0 = c->cur, s1 = (c->cur + 1) % 3, s2 = (c->cur + 2) % 3;
    void* S = c->reg[s0];
    void* A = c->reg[s1];
    void* B = c->reg[s2];
    mhd_status st;
    switch (c->scheme.integ) {
    case MHD_INT_VL2:
        // predictor: donor cell, half step; corrector: configured recon, full step from U*
        st = mhd_stage(c, MHD_RECON_DC, S, S, A, StageCoef{0.0, 1.0, 0.5 * dt}, false, false);
        if (st != MHD_OK) return st;
        st = mhd_stage(c, c->scheme.recon, A, S, B, StageCoef{0.0, 1.0, dt}, true, true);
        c->cur = s2;
        break;
    case MHD_INT_RK2:
        st = mhd_stage(c, c->scheme.recon, S, S, A, StageCoef{0.0, 1.0, dt}, false, false);
        if (st != MHD_OK) return st;
        st = mhd_stage(c, c->scheme.recon, A, S, B, StageCoef{0.5, 0.5, 0.5 * dt}, true, true);
        c->cur = s2;
        break;
    default:  // EULER1
        st = mhd_stage(c, c->scheme.recon, S, S, A, StageCoef{0.0, 1.0, dt}, true, true);
        c->cur = s1;
        break;
    }
    return st;
}

// Both IMEX2P stages; stage 1 writes U1 = reg[1 - cur], stage 2 overwrites u = reg[cur]
// and leaves the CFL step of the new state in scalars[0].
mhd_status step_dust(mhd_ctx* c, double dt)
{
    void* u = c->reg[c->cur];
    void* U1 = c->reg[1 - c->cur];
    const int recon = c->scheme.recon;
    hipError_t e;
    {
        Tick t(c, T_DUST_PASS1);
        e = launch_fluid_pass1(c->geo, c->dp, c->dg, c->fp32, recon, u, U1, dt, c->stream);
    }
    if (e == hipSuccess) {
        Tick t(c, T_DUST_DRAG1);
        e = launch_drag1(c->geo, c->dp, c->fp32, U1, dt, c->stream);
    }
    if (e == hipSuccess) {
        Tick t(c, T_DUST_PASS2);
        e = launch_fluid_pass2(c->geo, c->dp, c->dg, c->fp32, recon, u, U1, dt, c->stream);
    }
    if (e == hipSuccess) {
        Tick t(c, T_DUST_DRAG2);
        e = launch_drag2_cfl(c->geo, c->dp, c->fp32, u, U1, dt, c->partial, c->scalars, c->cfl_scale,
                             c->stream);
    }
    return dev(e);
}

}  // namespace

namespace mhd {

CtxView ctx_view(mhd_ctx* c)
{
    CtxView v;
    v.geo = c->geo;
    v.mp = c->mp;
    v.stream = c->stream;
    v.state = c->is_mhd && !c->fp32 ? (double*)c->reg[c->cur] : nullptr;
    return v;
}

hipError_t ctx_refresh_cfl(mhd_ctx* c)
{
    hipError_t e;
    const double* U = canonical_view(c, &e);
    if (e != hipSuccess) return e;
    return cfl_of(c, U) == MHD_OK ? hipSuccess : hipErrorLaunchFailure;
}

}  // namespace mhd

extern "C" {

const char* mhd_strerror(mhd_status s)
{
    switch (s) {
    case MHD_OK: return "ok";
    case MHD_E_INVAL: return "invalid argument";
    case MHD_E_UNSUPPORTED: return "unsupported scheme combination";
    case MHD_E_NOMEM: return "workspace too small or host allocation failed";
    case MHD_E_DEVICE: return "HIP runtime error";
    case MHD_E_NONFINITE: return "state holds NaN or Inf";
    case MHD_E_TOOBIG: return "grid exceeds the static scratch of the allocation-free entry point";
    }
    return "unknown status";
}

mhd_status mhd_workspace_bytes(const mhd_grid* grid, const mhd_physics* phys,
                               const mhd_scheme* scheme, size_t* bytes)
{
    if (!bytes) return MHD_E_INVAL;
    mhd_status st = validate(grid, phys, scheme);
    if (st != MHD_OK) return st;
    *bytes = layout(grid, phys, scheme).total;
    return MHD_OK;
}

mhd_status mhd_create(const mhd_grid* grid, const mhd_physics* phys, const mhd_scheme* scheme,
                      void* device_workspace, size_t bytes, void* hip_stream, mhd_ctx** out)
{
    if (!out) return MHD_E_INVAL;
    *out = nullptr;
    mhd_status st = validate(grid, phys, scheme);
    if (st != MHD_OK) return st;
    if (!device_workspace || ((uintptr_t)device_workspace & 255u)) return MHD_E_INVAL;
    const Layout L = layout(grid, phys, scheme);
    if (bytes < L.total) return MHD_E_NOMEM;

    mhd_ctx* c = new (std::nothrow) mhd_ctx;
    if (!c) return MHD_E_NOMEM;
    std::memset(c, 0, sizeof(*c));
    c->grid = *grid;
    c->phys = *phys;
    c->scheme = *scheme;
    c->stream = (hipStream_t)hip_stream;
    c->is_mhd = phys->eos == MHD_EOS_ADIABATIC_MHD;
    c->nvar = state_fields(phys);
    c->n = (long long)grid->nx * grid->ny * grid->nz;

    c->geo = make_geo(grid);
    c->fg = fused_grid(c->geo, choose_kz(grid));
    c->dg = dust_grid(c->geo, 1 + (phys->eos == MHD_EOS_ADIABATIC_MHD ? 0 : phys->ndust));
    c->fp32 = scheme->prec == MHD_PREC_FP32_BULK;
    c->cfl_scale = make_params(phys, scheme, &c->mp, &c->dp);

    char* base = (char*)device_workspace;
    for (size_t r = 0; r < 3; ++r) {
        c->reg[r] = r < L.nreg ? (void*)base : nullptr;
        if (r < L.nreg) base += L.reg;
    }
    c->F = L.F ? (void*)base : nullptr; base += L.F;
    c->Rc = L.Rc ? (void*)base : nullptr; base += L.Rc;
    c->partial = (double*)base; base += L.partial;
    c->scalars = (double*)base;
    c->cur = 0;
    *out = c;
    return MHD_OK;
}

mhd_status mhd_state_len(const mhd_ctx* c, size_t* n)
{
    if (!c || !n) return MHD_E_INVAL;
    *n = (size_t)c->n * c->nvar;
    return MHD_OK;
}

mhd_status mhd_set_state(mhd_ctx* c, const double* src, int src_is_device)
{
    if (!c || !src) return MHD_E_INVAL;
    const size_t bytes = (size_t)c->n * c->nvar * sizeof(double);
    hipError_t e = hipSuccess;
    // the canonical FP64 source on the device: the register (FP64 form) or the staging
    // area (FP32 forms, or a host source that must be copied first)
    const double* canon = src;
    if (!c->fp32) {
        e = hipMemcpyAsync(c->reg[c->cur], src, bytes,
                           src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream);
        canon = (const double*)c->reg[c->cur];
    } else if (!src_is_device) {
        e = hipMemcpyAsync(c->F, src, bytes, hipMemcpyHostToDevice, c->stream);
        canon = (const double*)c->F;
    }
    if (e == hipSuccess && !src_is_device) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return MHD_E_DEVICE;
    // the time step of the state as given, then (FP32 forms) its packed register
    mhd_status st = cfl_of(c, canon);
    if (st != MHD_OK || !c->fp32) return st;
    return dev(pack_reg(c, canon, c->reg[c->cur]));
}

mhd_status mhd_get_state(mhd_ctx* c, double* dst, int dst_is_device)
{
    if (!c || !dst) return MHD_E_INVAL;
    const size_t bytes = (size_t)c->n * c->nvar * sizeof(double);
    hipError_t e;
    if (c->fp32 && dst_is_device) {
        e = unpack_reg(c, c->reg[c->cur], dst);
        return dev(e);
    }
    const double* canon = canonical_view(c, &e);
    if (e != hipSuccess) return MHD_E_DEVICE;
    e = hipMemcpyAsync(dst, canon, bytes, dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                       c->stream);
    if (e != hipSuccess) return MHD_E_DEVICE;
    if (!dst_is_device) return dev(hipStreamSynchronize(c->stream));
    return MHD_OK;
}

mhd_status mhd_step(mhd_ctx* c, double dt)
{
    if (!c) return MHD_E_INVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return MHD_E_INVAL;
    // the last stage of either path reduces the CFL step of the new state itself
    return c->is_mhd ? step_mhd(c, dt) : step_dust(c, dt);
}

mhd_status mhd_dt_cfl(mhd_ctx* c, double* dt)
{
    if (!c || !dt) return MHD_E_INVAL;
    double h = 0.0;
    hipError_t e = hipMemcpyAsync(&h, c->scalars, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return MHD_E_DEVICE;
    *dt = h;
    if (!std::isfinite(h) || !(h > 0.0)) return MHD_E_NONFINITE;
    return MHD_OK;
}

mhd_status mhd_diagnostics(mhd_ctx* c, double* out, int n)
{
    if (!c || !out) return MHD_E_INVAL;
    const int nq = diag_count(c->phys.ndust);
    if (n < nq) return MHD_E_INVAL;
    hipError_t e;
    const double* canon = canonical_view(c, &e);
    if (e == hipSuccess)
        e = launch_diag(c->geo, c->is_mhd ? 1 : 0, c->is_mhd ? 0 : c->phys.ndust, canon, c->partial,
                        c->scalars + 1, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, c->scalars + 1, sizeof(double) * nq, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return MHD_E_DEVICE;
    // keep the CFL scalar of the state (the diagnostics reuse only the partial buffer)
    return MHD_OK;
}

static void timer_free(mhd_ctx* c)
{
    if (!c->timer) return;
    for (hipEvent_t e : c->timer->ev) (void)hipEventDestroy(e);
    delete c->timer;
    c->timer = nullptr;
}

mhd_status mhd_timing_enable(mhd_ctx* c, int capacity)
{
    if (!c || capacity < 0) return MHD_E_INVAL;
    if (c->timer) {
        hipError_t e = hipStreamSynchronize(c->stream);
        timer_free(c);
        if (e != hipSuccess) return MHD_E_DEVICE;
    }
    if (capacity == 0) return MHD_OK;
    EventTimer* t = new (std::nothrow) EventTimer;
    if (!t) return MHD_E_NOMEM;
    t->cap = capacity;
    t->ev.resize(2 * (size_t)capacity);
    t->slot.resize(capacity);
    for (auto& e : t->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            delete t;
            return MHD_E_DEVICE;
        }
    c->timer = t;
    return MHD_OK;
}

mhd_status mhd_timing_read(mhd_ctx* c, double* ms, int* launches, int nslot)
{
    if (!c || !ms || !launches || nslot < 0) return MHD_E_INVAL;
    for (int q = 0; q < nslot; ++q) {
        ms[q] = 0.0;
        launches[q] = 0;
    }
    if (!c->timer) return MHD_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MHD_E_DEVICE;
    EventTimer* t = c->timer;
    for (int k = 0; k < t->used; ++k) {
        float f = 0.0f;
        if (hipEventElapsedTime(&f, t->ev[2 * k], t->ev[2 * k + 1]) != hipSuccess) return MHD_E_DEVICE;
        const int q = t->slot[k];
        if (q < nslot) {
            ms[q] += f;
            launches[q] += 1;
        }
    }
    t->used = 0;
    return MHD_OK;
}

const char* mhd_timing_name(int q) { return (q >= 0 && q < T_NSLOT) ? kSlotNames[q] : nullptr; }

mhd_status mhd_dt_cfl_noalloc(const mhd_grid* grid, const mhd_physics* phys, const mhd_scheme* scheme,
                              const double* state_device, double* dt_device, void* hip_stream)
{
    if (!state_device || !dt_device) return MHD_E_INVAL;
    mhd_status st = validate(grid, phys, scheme);
    if (st != MHD_OK) return st;
    const long long n = (long long)grid->nx * grid->ny * grid->nz;
    if (n > MHD_NOALLOC_MAX_CELLS) return MHD_E_TOOBIG;
    const hipStream_t s = (hipStream_t)hip_stream;
    double* partial = nullptr;
    const hipError_t es = noalloc_scratch(s, &partial);
    if (es == hipErrorInvalidValue) return MHD_E_INVAL;
    if (es != hipSuccess) return MHD_E_DEVICE;
    MhdParams mp;
    DustParams dp;
    const double scale = make_params(phys, scheme, &mp, &dp);
    const Geo g = make_geo(grid);
    hipError_t e = phys->eos == MHD_EOS_ADIABATIC_MHD
                       ? launch_cfl_mhd(g, mp, state_device, partial, dt_device, scale, s)
                       : launch_cfl_dust(g, dp, state_device, partial, dt_device, scale, s);
    return dev(e);
}

void mhd_destroy(mhd_ctx* c)
{
    if (!c) return;
    timer_free(c);
    delete c;
}

}  // extern "C"
