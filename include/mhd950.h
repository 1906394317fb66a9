/*
 * mhd950.h -- C ABI of the MI355X (gfx950) Godunov step for compressible ideal MHD
 * with constrained transport, and for isothermal gas coupled to N pressureless dust
 * fluids by implicit drag.
 *
 * The operation behind these calls is the per-timestep finite-volume update of the
 * paper (Aether.jl, Ho): the semi-discrete update of eq. (fv_update) with fluxes from
 * reconstructed primitives and an approximate Riemann solver (Sec. "Reconstruction and
 * Riemann Solvers"), the face-field update of eq. (ct) with upwind edge EMFs
 * (Sec. "Constrained Transport"), the two-register stages of eq. (two_register) or the
 * IMEX2P pair with closed-form drag solves (Secs. "Multifluid Dust", "Time
 * Integration"), and the time step of eq. (cfl).  The interface mirrors the paper's
 * Mesh / Simulation / set_initial_condition! / run! split (Sec. "User Interface,
 * Problem Setup, and Execution Modes"):
 * a context is created once with every choice fixed and validated, the state is set,
 * and steps are taken.
 *
 * Conventions
 *   - Every call returns an mhd_status (0 = MHD_OK); no exception crosses the ABI.
 *   - The grid is uniform, Cartesian and periodic in x, y and z.
 *   - Memory: the caller owns the device workspace and the HIP stream; the library
 *     borrows both for the lifetime of the context and allocates no device memory.
 *     The context itself is a small host object freed by mhd_destroy.
 *   - All work is enqueued on the caller's stream.  mhd_step is asynchronous;
 *     mhd_dt_cfl, mhd_diagnostics and transfers to or from host memory synchronise it.
 *   - Configuration is validated only in mhd_create (unsupported combinations are
 *     rejected there, never during a step).
 *   - Calls on one context are not thread safe; separate contexts are independent.
 *
 * Canonical state layout (FP64, what mhd_set_state/mhd_get_state exchange):
 *   cell fields, each [nz][ny][nx] with x fastest, one after the other:
 *     adiabatic MHD     : rho, M1, M2, M3, E                        (5 fields)
 *     isothermal + dust : rho, M1, M2, M3, then for each species k
 *                         rho_k, M_k1, M_k2, M_k3                    (4 + 4 N fields)
 *   then, for MHD only, the face fields b1, b2, b3, each [nz][ny][nx]; b1[k][j][i] is
 *   the area-averaged B_x on the face x_{i-1/2}, the left face of cell (i, j, k);
 *   b2 and b3 likewise on y_{j-1/2} and z_{k-1/2}.
 */
#ifndef MHD950_H
#define MHD950_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MHD_MAX_DUST 16

typedef enum {
    MHD_OK = 0,
    MHD_E_INVAL = -1,       /* bad argument: null pointer, size, dt <= 0 or not finite */
    MHD_E_UNSUPPORTED = -2, /* the scheme combination does not exist (mhd_create) */
    MHD_E_NOMEM = -3,       /* workspace smaller than mhd_workspace_bytes, or host alloc failed */
    MHD_E_DEVICE = -4,      /* a HIP runtime call failed */
    MHD_E_NONFINITE = -5,   /* the state holds NaN or Inf (found by the CFL reduction) */
    MHD_E_TOOBIG = -6       /* grid larger than the static scratch of mhd_dt_cfl_noalloc */
} mhd_status;

typedef enum { MHD_EOS_ADIABATIC_MHD = 0, MHD_EOS_ISOTHERMAL_HYDRO = 1 } mhd_eos;
typedef enum { MHD_RECON_DC = 0, MHD_RECON_PLM = 1, MHD_RECON_PPM = 2 } mhd_recon;
typedef enum { MHD_RS_HLLE = 0, MHD_RS_HLLD = 1 } mhd_riemann;
typedef enum {
    MHD_INT_VL2 = 0,   /* donor-cell half step, then a full step with the chosen recon */
    MHD_INT_RK2 = 1,   /* optimal two-stage SSP Runge-Kutta (paper's RK2) */
    MHD_INT_IMEX2P = 2,/* ARS(2,2,2) pair, implicit weight 1 + 1/sqrt(2) (dust only) */
    MHD_INT_EULER1 = 3 /* one forward-Euler stage; for tests */
} mhd_integrator;
typedef enum {
    MHD_PREC_FP64 = 0,     /* everything in FP64 */
    MHD_PREC_FP32_BULK = 1 /* adiabatic MHD: density, momenta, face fields,
                              reconstruction, Riemann solves, CT and updates in FP32; the
                              total energy stored in FP64 and the pressure recovery
                              p = (gamma-1)(E - kinetic - magnetic) and the energy update
                              done in FP64; the time step and diagnostics in FP64.
                              hlld_eps is raised to at least 1e-6.
                              Isothermal + dust: every field stored in FP32, the explicit
                              part (primitives, reconstruction, Riemann solves, flux
                              divergence, stage combination) in FP32; the implicit drag
                              solve, the time step and diagnostics in FP64. */
} mhd_precision;

/* Uniform periodic grid of nx*ny*nz cells covering a box of edges length[0..2]. */
typedef struct {
    int nx, ny, nz;
    double length[3];
} mhd_grid;

/* Closure and physical parameters (Sec. "Newtonian Magnetohydrodynamics",
 * Sec. "Multifluid Dust").  gamma: adiabatic index (MHD); cs_iso: isothermal sound
 * speed (isothermal hydro); rho_floor, p_floor: floors applied to the primitives of
 * the gas; dust_rho_floor: a step first resets every species whose density is below
 * it to the floor at rest (a species that stage 1 drives below it is read as the floor
 * at rest);
 * t_stop: constant stopping time of each of the ndust species; gas_accel: constant
 * acceleration of the gas alone, applied as an unsplit source. */
typedef struct {
    int eos;
    double gamma, cs_iso, rho_floor, p_floor;
    int ndust;
    double t_stop[MHD_MAX_DUST];
    double dust_rho_floor;
    double gas_accel[3];
} mhd_physics;

/* Scheme choices.  courant: the factor C of eq. (cfl) (the integrator's C_max is
 * applied by the library); hlld_eps: degeneracy tolerance of HLLD relative to the
 * fan's total pressure. */
typedef struct {
    int recon, riemann, integ;
    double courant;
    int prec;
    double hlld_eps;
} mhd_scheme;

typedef struct mhd_ctx mhd_ctx;

/* Bytes of device workspace a context of this configuration needs (256-byte aligned
 * base expected).  Returns MHD_E_INVAL for null pointers or non-positive sizes and
 * MHD_E_UNSUPPORTED for combinations mhd_create would reject. */
mhd_status mhd_workspace_bytes(const mhd_grid* grid, const mhd_physics* phys,
                               const mhd_scheme* scheme, size_t* bytes);

/* Create a context on the current HIP device.  device_workspace: caller-owned device
 * memory of at least mhd_workspace_bytes bytes, 256-byte aligned; hip_stream: the
 * hipStream_t all work is enqueued on (NULL = the null stream).  Supported:
 *   adiabatic MHD     with VL2, RK2 or EULER1, any recon, HLLE or HLLD, ndust = 0,
 *                     precision FP64 or FP32_BULK;
 *   isothermal + dust with IMEX2P, DC or PLM recon, HLLE gas flux, 1 <= ndust <= 16,
 *                     precision FP64 or FP32_BULK.
 * Grids of 2^29 cells or more are MHD_E_UNSUPPORTED (fields are addressed with 32-bit
 * byte offsets).  Anything else is MHD_E_UNSUPPORTED.  The state is undefined until
 * mhd_set_state. */
mhd_status mhd_create(const mhd_grid* grid, const mhd_physics* phys, const mhd_scheme* scheme,
                      void* device_workspace, size_t bytes, void* hip_stream, mhd_ctx** out);

/* Number of doubles in the canonical state of this context. */
mhd_status mhd_state_len(const mhd_ctx* ctx, size_t* n);

/* Copy a canonical FP64 state in (src on the device if src_is_device, else host
 * memory; host copies complete before return).  The state is the one the method
 * advances: cell averages of the conserved variables (Sec. "Reconstruction and Riemann
 * Solvers", eq. (fv_update)) in the i-fastest array layout of Sec. "Mesh, Coordinates,
 * and Boundary Conditions", then (MHD) the area-averaged normal field on the faces of
 * Sec. "Constrained Transport".  Also computes the CFL step of the
 * new state on the device.  The FP32-bulk form rounds every field but E to FP32 here
 * (every field for the dust path; the CFL step is that of the FP64 state as given). */
mhd_status mhd_set_state(mhd_ctx* ctx, const double* src, int src_is_device);

/* Copy the current state out in canonical layout (the complete state that continues a
 * run, as the paper's restart output writes it at working precision, Sec. "Output and
 * Restart"); a copy to host memory completes before return, a copy to device memory is
 * ordered on the stream. */
mhd_status mhd_get_state(mhd_ctx* ctx, double* dst, int dst_is_device);

/* Advance the state by exactly dt (one full step of the configured integrator; the
 * Courant-limited step of the result is computed at its end).  Asynchronous.
 * MHD_E_INVAL if dt <= 0 or not finite. */
mhd_status mhd_step(mhd_ctx* ctx, double dt);

/* The Courant-limited step C C_max min_cells min_d dx_d/(|v_d| + c_d) of the current
 * state (eq. (cfl); c_d the directional fast speed for MHD, c_s for isothermal gas,
 * 0 for dust; C_max = 1 for VL2/RK2/EULER1, 1/(1 + 1/sqrt 2) for IMEX2P).  Reads one
 * double from the device (synchronises the stream).  MHD_E_NONFINITE if the state
 * holds NaN or Inf. */
mhd_status mhd_dt_cfl(mhd_ctx* ctx, double* dt);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the Courant-limited step of
 * mhd_dt_cfl for a canonical FP64 state that the caller holds on the device, with no
 * context and no workspace.  grid, phys and scheme are validated as by mhd_create;
 * state_device: the canonical state (mhd_state_len doubles), read only; dt_device: one
 * double of device memory that receives C C_max min(...), or NaN if the state holds
 * NaN or Inf.  Asynchronous on hip_stream, which must belong to the current device;
 * no host synchronisation, no allocation, no memset (capturable in a HIP graph).  The
 * per-workgroup partial minima live in a static device array of the library, one copy
 * per GPU that holds it until the process ends: MHD_NOALLOC_MAX_CELLS cells at most
 * (4 MiB of partials), larger grids return MHD_E_TOOBIG.  Every call on one GPU shares
 * that array: calls that overlap on one GPU (other streams, other threads) race and
 * must be serialised by the caller. */
#define MHD_NOALLOC_MAX_CELLS (1LL << 27)
mhd_status mhd_dt_cfl_noalloc(const mhd_grid* grid, const mhd_physics* phys, const mhd_scheme* scheme,
                              const double* state_device, double* dt_device, void* hip_stream);

/* Volume integrals and extrema of the current state, the history diagnostics of
 * Sec. "Output and Restart" (total mass, momentum and energy, the maximum |div B| for
 * MHD), in FP64 with a fixed-order (deterministic) reduction.  out must hold n >= 12 + ndust doubles:
 *   out[0] gas mass, out[1..3] gas momentum, out[4] total energy (0 if isothermal),
 *   out[5..7] volume integral of the face fields (0 without MHD), out[8] max |div B|
 *   over cells, out[9 .. 8+ndust] dust masses, out[9+ndust .. 11+ndust] total momentum
 *   of gas and dust.  Synchronises the stream. */
mhd_status mhd_diagnostics(mhd_ctx* ctx, double* out, int n);

/* Per-kernel timing for profiling (off by default).  With capacity > 0 the library
 * records a pair of HIP events on the context's stream around each kernel launch,
 * for up to `capacity` launches between reads (later launches are not recorded);
 * capacity 0 turns timing off and releases the events.  Host-side events only: no
 * device memory is allocated. */
mhd_status mhd_timing_enable(mhd_ctx* ctx, int capacity);

/* Synchronise the stream, then write for each kernel class q < nslot the summed
 * device time in milliseconds ms[q] and the number of recorded launches launches[q]
 * since the previous read, and clear the record.  Classes are numbered as
 * mhd_timing_name lists them (nslot may be smaller than the number of classes). */
mhd_status mhd_timing_read(mhd_ctx* ctx, double* ms, int* launches, int nslot);

/* Name of kernel class q, or NULL past the last class. */
const char* mhd_timing_name(int q);

/* Release the host context (the workspace stays the caller's). */
void mhd_destroy(mhd_ctx* ctx);

/* Static description of a status code. */
const char* mhd_strerror(mhd_status status);

/* ---------------------------------------------------------------------------------
 * Batched meshblocks.  The paper advances all the meshblocks a rank owns in one launch,
 * with the block index as one more dimension of the launch (Sec. "Mesh, Coordinates,
 * and Boundary Conditions").  A batch
 * here is a set of nblocks INDEPENDENT self-periodic adiabatic-MHD boxes of any sizes
 * sharing one physics and scheme; every stage kernel is one persistent launch that
 * drains a device work queue of (block, tile, z chunk) items.  The stencil halo of
 * each block (4 cells: PPM 3 + CT 1) is its own periodic wrap, so no ghost cells are
 * stored.  Each block advances with its own time step.  A block advanced in a batch is
 * bitwise identical to the same block advanced alone through mhd_step with the same dt.
 *
 * Ownership and errors as for a single context: the caller owns the workspace (256-byte
 * aligned, mhd_batch_workspace_bytes) and the stream; the batch object is a small host
 * object freed by mhd_batch_destroy.  After an MHD_E_DEVICE from a step the batch must
 * be destroyed (its work counters may no longer match).  Dust (isothermal) batches are
 * MHD_E_UNSUPPORTED; so are grids whose padded cell total reaches 2^29.
 * --------------------------------------------------------------------------------- */
typedef struct mhd_batch mhd_batch;

/* Workspace bytes of a batch of nblocks grids (grids[b] is block b). */
mhd_status mhd_batch_workspace_bytes(int nblocks, const mhd_grid* grids, const mhd_physics* phys,
                                     const mhd_scheme* scheme, size_t* bytes);

/* Carve a batch out of the caller's workspace; uploads the block table and the default
 * work items (the widest tile that wastes no more lanes along x than the narrower). */
mhd_status mhd_batch_create(int nblocks, const mhd_grid* grids, const mhd_physics* phys,
                            const mhd_scheme* scheme, void* device_workspace, size_t bytes,
                            void* hip_stream, mhd_batch** out);

/* Doubles in the batch state: the sum over blocks of the single-context state length. */
mhd_status mhd_batch_state_len(const mhd_batch* batch, size_t* n);

/* The batch state is the blocks' canonical states concatenated in block order.  After
 * set_state, each block's CFL step is on the device (see mhd_batch_step). */
mhd_status mhd_batch_set_state(mhd_batch* batch, const double* src, int src_is_device);
mhd_status mhd_batch_get_state(mhd_batch* batch, double* dst, int dst_is_device);

/* Advance every block: block b by dt[b] (host array of nblocks positive finite values),
 * or, with dt == NULL, by the CFL step of its current state that the device already
 * holds (no host synchronisation).  Asynchronous on the stream. */
mhd_status mhd_batch_step(mhd_batch* batch, const double* dt);

/* The CFL step of every block's current state (nblocks doubles; synchronises);
 * MHD_E_NONFINITE if any block holds NaN or Inf. */
mhd_status mhd_batch_dt_cfl(mhd_batch* batch, double* dt);

/* Tile shape per block: 0 = 64-wide tiles (64x4 flux, 64x8 update), 1 = 32-wide
 * (32x8, 32x16), 2 = 16-wide (16x16, 16x32).  Results do not depend on the shapes. */
mhd_status mhd_batch_set_shapes(mhd_batch* batch, const int* shapes, int nblocks);
mhd_status mhd_batch_get_shapes(const mhd_batch* batch, int* shapes, int nblocks);

/* Autotuner: for each class of blocks with one x extent (classes in increasing nx),
 * time `reps` passes of the configured-reconstruction stage over that class alone with
 * each tile shape; then time the whole batch with those per-class picks and with each
 * uniform shape, keep the fastest assignment, and rebuild the work queue.  The current
 * state is only read.  If ms_out is not NULL it receives the per-class average ms per
 * pass, class-major (nout >= classes * 3).  Synchronises the stream. */
mhd_status mhd_batch_tune(mhd_batch* batch, int reps, float* ms_out, int nout);

/* ---------------------------------------------------------------------------------
 * One periodic domain as coupled meshblocks.  The paper divides a domain into identical
 * blocks, each padded with ghost cells that one exchange per stage fills from all its
 * face, edge and corner neighbours (Sec. "Mesh, Coordinates, and Boundary Conditions"),
 * and its single-device benchmark runs the 512 x 512 x 256 box in 128^3 blocks (Sec.
 * "Single-Device Performance").
 *
 * mhd_batch_couple turns a batch of nblocks = nbx nby nbz FP64 blocks, all of
 * (bx + 2 ghost) x (by + 2 ghost) x (bz + 2 ghost) cells, into the periodic domain of
 * (nbx bx) x (nby by) x (nbz bz) cells with side lengths length[0..2]: block
 * b = bi + nbx (bj + nby bk) holds the domain cells [bi bx, (bi+1) bx) x [bj by, ...) x
 * [bk bz, ...) as its interior, with `ghost` layers on every side.  Every block takes the
 * domain's spacing length[a] / (nb_a b_a).  From then on each stage of mhd_batch_step is
 * followed on the device by the exchange: every ghost cell of every block (all 8 fields;
 * a face field goes with the cell on its high side) is copied from the interior cell of
 * the block that owns that domain cell; and after the last stage every block is given
 * the one CFL step of the whole domain (the minimum over the interiors).  A block's
 * interior then evolves bitwise as the same cells of the domain advanced as one grid
 * with the same steps.  ghost must be at least the reconstruction's stencil plus the one
 * cell the edge EMFs reach beyond it (donor cell 2, PLM 3, PPM 4) and at most 64;
 * nblocks_xyz must multiply to the batch's block count; all blocks must have the same
 * extents, larger than 2 ghost (else MHD_E_INVAL).  FP32-bulk batches are
 * MHD_E_UNSUPPORTED.  The current state's ghost cells are refreshed and its step is put
 * on the device; a later mhd_batch_set_state does the same.  mhd_batch_step's host dt,
 * if given, must then be one value for all blocks (else MHD_E_INVAL).  Synchronises.
 * --------------------------------------------------------------------------------- */
mhd_status mhd_batch_couple(mhd_batch* batch, const int nblocks_xyz[3], int ghost, const double length[3]);

/* The domain state of a coupled batch in the single-context canonical layout of the
 * whole domain ([8][nz][ny][nx] doubles, host or device pointer as flagged).  set
 * fills every block's interior and ghost cells from it (staging a host source through
 * the workspace) and puts the domain's CFL step on the device; get gathers the
 * interiors.  MHD_E_INVAL on a batch that is not coupled.  Synchronise for host
 * buffers. */
mhd_status mhd_batch_set_domain_state(mhd_batch* batch, const double* src, int src_is_device);
mhd_status mhd_batch_get_domain_state(mhd_batch* batch, double* dst, int dst_is_device);

void mhd_batch_destroy(mhd_batch* batch);

/* ---------------------------------------------------------------------------------
 * Learned subgrid flux-correction closure of the coarse step.  This is an extension of
 * this library, not part of the paper's method: the paper only remarks that a neural
 * surrogate could stand in for an expensive cell-local solve such as astrochemistry
 * (Sec. "Discussion and Summary").  The network here sees the 8 primitive
 * channels (rho, v, p, B_cc) of the coarse state at the start of a step, normalised as
 * (w - mu) / sd, and returns 18 channels per cell: face-flux corrections of rho, M_x,
 * M_y, M_z, E through the low x, y, z faces (channel 3 f + d, scaled by sF[f]) and
 * edge-EMF corrections E_x, E_y, E_z on the cell's low edges (channels 15..17, scaled
 * by sE).  They enter the plain step in flux form (eq. (fv_update)) and in
 * constrained-transport form (eq. (ct)): U_f -= dt sum_d (dF[c+e_d] - dF[c]) / dx_d,
 * b -= dt curl(dE); mass, momentum and energy stay conservative and div B unchanged.
 * Network: 4 periodic 3x3x3 convolutions 8 -> 32 -> 32 -> 32 -> 18, ReLU after the
 * first three; BF16 operands on the matrix cores, FP32 accumulation; FP32 master
 * weights and Adam.  Parameters, in order, per layer: W [27][cin][cout] with tap
 * t = (dz+1)*9 + (dy+1)*3 + (dx+1) (y[v][co] = b[co] + sum W[t][ci][co] x[v+off(t)][ci]),
 * then b [cout].  Grids: adiabatic MHD, nx a multiple of 16, fewer than 2^26 cells
 * (else MHD_E_UNSUPPORTED).  Device pointers are canonical FP64 states (8 fields).
 * Ownership as for a context: caller's workspace and stream; calls on one network are
 * not thread safe.
 * --------------------------------------------------------------------------------- */
typedef struct mhd_cnn mhd_cnn;

mhd_status mhd_cnn_param_count(size_t* n);
mhd_status mhd_cnn_workspace_bytes(const mhd_grid* grid, const mhd_physics* phys, size_t* bytes);
/* Parameters and Adam moments start at zero (the closure is then exactly zero). */
mhd_status mhd_cnn_create(const mhd_grid* grid, const mhd_physics* phys, void* device_workspace,
                          size_t bytes, void* hip_stream, mhd_cnn** out);
/* Host FP32 arrays of mhd_cnn_param_count values (synchronising). */
mhd_status mhd_cnn_set_params(mhd_cnn* cnn, const float* params);
mhd_status mhd_cnn_get_params(mhd_cnn* cnn, float* params);
mhd_status mhd_cnn_get_grads(mhd_cnn* cnn, float* grads);
/* Input normalisation mu[8], sd[8] (> 0); output scales sF[5], sE; loss weights wU[5]
 * for rho, M_x, M_y, M_z, E and wB for each face field. */
mhd_status mhd_cnn_set_scales(mhd_cnn* cnn, const float* mu, const float* sd, const float* sF, float sE,
                              const float* wU, float wB);
/* Network output of a state into the network's output buffer; mhd_cnn_output copies it
 * out as FP32 [18][nz][ny][nx]. */
mhd_status mhd_cnn_forward(mhd_cnn* cnn, const double* state);
mhd_status mhd_cnn_output(mhd_cnn* cnn, float* dst, int dst_is_device);
/* Add the corrections of the last forward pass to a state, in place. */
mhd_status mhd_closure_apply(mhd_cnn* cnn, double dt, double* state);
/* One training sample: forward from state_t, closure applied to coarse_next (the plain
 * coarse step of state_t by dt), loss sum_f w_f (pred - target)^2 / cells against the
 * filtered fine state, gradients ADDED to the network's gradient buffer; *loss (if not
 * NULL) receives the loss (synchronising). */
mhd_status mhd_cnn_zero_grad(mhd_cnn* cnn);
mhd_status mhd_cnn_accumulate(mhd_cnn* cnn, const double* state_t, const double* coarse_next,
                              const double* target, double dt, double* loss);
/* Adam step `step` (>= 1) on grad_scale * gradients. */
mhd_status mhd_cnn_adam(mhd_cnn* cnn, float lr, float beta1, float beta2, float eps, int step,
                        float grad_scale);
/* One closure step of a context, in place: corrections from its current state (read
 * where it lives), the plain step by dt, then the corrections added to the stepped
 * state if that leaves every cell finite with density and pressure at or above the
 * floors; otherwise the plain step stands (the fallback).  The context's CFL step is
 * then refreshed.  *applied (if not NULL; reading it synchronises the stream) is 1
 * when the corrections were applied, 0 for the fallback.  The context must be FP64
 * adiabatic MHD (else MHD_E_UNSUPPORTED), on the network's grid (cells and spacing) and
 * on the network's stream (else MHD_E_INVAL). */
mhd_status mhd_step_closure(mhd_ctx* ctx, mhd_cnn* cnn, double dt, int* applied);
/* Box filter of a fine canonical state (device) onto the grid r times coarser: cell
 * fields averaged over r^3 cells, face fields over the r^2 fine faces of each coarse
 * face (so the coarse div B is the mean of the fine one).  Asynchronous. */
mhd_status mhd_box_filter(const mhd_grid* fine, int r, const double* fine_state, double* coarse_state,
                          void* hip_stream);
void mhd_cnn_destroy(mhd_cnn* cnn);

#ifdef __cplusplus
}
#endif
#endif
