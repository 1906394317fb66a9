/*
 * oracle.h -- plain FP64 CPU reference of the Godunov step (TEST INFRASTRUCTURE ONLY).
 *
 * This header and oracle.c are the checker, not the product.  Only tests/, the
 * smoke() entry and the cpu_baseline leg of bench.py may load it.  It shares no
 * source, header, table or helper with the HIP library; the two meet only through
 * the seeded input generators and the canonical state layout:
 *
 *   cell fields  [nvar][nz][ny][nx], x fastest (the i-fastest layout of the paper's
 *                Mesh section), variables
 *                  adiabatic MHD     : rho, M1, M2, M3, E
 *                  isothermal + dust : rho, M1, M2, M3, then per species rho_k, M_k1..3
 *   face fields  (MHD only) b1, b2, b3, each [nz][ny][nx]; b1[k][j][i] is the
 *                area-averaged B_x on the face x_{i-1/2} (left face of cell i).
 *
 * The grid is uniform, Cartesian and periodic in all three directions.
 */
#ifndef MHD_ORACLE_H
#define MHD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_DUST 16

enum { ORC_EOS_ADIABATIC_MHD = 0, ORC_EOS_ISOTHERMAL_HYDRO = 1 };
enum { ORC_RECON_DC = 0, ORC_RECON_PLM = 1, ORC_RECON_PPM = 2 };
enum { ORC_RS_HLLE = 0, ORC_RS_HLLD = 1 };
enum { ORC_INT_VL2 = 0, ORC_INT_RK2 = 1, ORC_INT_IMEX2P = 2, ORC_INT_EULER1 = 3 };

typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;
    int eos;
    double gamma, cs, rho_floor, p_floor, dust_rho_floor;
    int ndust;
    double tstop[ORC_MAX_DUST];
    double gacc[3];          /* constant acceleration of the gas (unsplit source) */
    int recon, riemann, integ;
    double courant;
    double hlld_eps;         /* degeneracy tolerance of HLLD, relative to P_T* */
} orc_cfg;

/* Threads the OpenMP loops of the oracle use. */
int orc_num_threads(void);

/* Threads for the OpenMP loops from now on (n > 0); the arithmetic does not depend on it. */
void orc_set_num_threads(int n);

/* Number of doubles in the canonical state of cfg. */
long orc_state_len(const orc_cfg* cfg);

/* One full step of size dt, in place on the canonical state.  Returns 0, or -1 on a
 * configuration the oracle does not implement. */
int orc_step(const orc_cfg* cfg, double* state, double dt);

/* Courant-limited step of the current state, eq. (cfl) with C_max of the integrator. */
double orc_dt_cfl(const orc_cfg* cfg, const double* state);

/* Volume integrals and extrema of the current state:
 * out[0] mass of gas, out[1..3] gas momentum, out[4] total energy (0 if isothermal),
 * out[5..7] integral of B (face fields, MHD) , out[8] max |div B| over cells,
 * out[9..9+ndust-1] dust masses, out[9+ndust .. 11+ndust] total momentum of gas+dust.
 * Returns the number of values written. */
int orc_diagnostics(const orc_cfg* cfg, const double* state, double* out);

/* ---- pieces, exposed for the pin tests ---- */

/* Face states of a periodic line a[0..n-1]: aL[f], aR[f] on the face f-1/2 between
 * cells f-1 and f. */
void orc_recon_line(int recon, int n, const double* a, double* aL, double* aR);

/* Riemann flux of the face-frame MHD problem. wl, wr = (rho, vn, vt1, vt2, p, Bt1, Bt2),
 * bn = normal field; f = (mass, mom_n, mom_t1, mom_t2, energy, flux Bt1, flux Bt2). */
void orc_riemann_mhd(const orc_cfg* cfg, const double* wl, const double* wr, double bn, double* f);

/* Isothermal HLLE (gas) and pressureless Rusanov (dust): w = (rho, vn, vt1, vt2),
 * f = (mass, mom_n, mom_t1, mom_t2). */
void orc_riemann_iso_hlle(double cs, const double* wl, const double* wr, double* f);
void orc_riemann_dust_rusanov(const double* wl, const double* wr, double* f);

/* Implicit drag solve (I - h G) p' = p for one cell and one momentum component,
 * by dense LU with partial pivoting on the (n+1)x(n+1) system.
 * rho[0] gas, rho[1..n] dust; p likewise; ts[0..n-1] stopping times. */
void orc_drag_solve(int n, const double* rho, const double* p, const double* ts, double h,
                    double* pout);

/* Right-hand side L(u) of one stage of the MHD system (recon given), for tests:
 * dudt  : 5 cell fields + 3 face fields, canonical layout (interior only);
 * emf   : 3 edge fields, E_x at (i, j-1/2, k-1/2), E_y at (i-1/2, j, k-1/2),
 *         E_z at (i-1/2, j-1/2, k), each [nz][ny][nx];
 * facee : 6 fields, the face values of the electric field that the Riemann fluxes
 *         give: (x-face E_y, x-face E_z, y-face E_z, y-face E_x, z-face E_x, z-face E_y). */
void orc_rhs_mhd_debug(const orc_cfg* cfg, int recon, const double* state, double* dudt,
                       double* emf, double* facee);

/* Cell primitives (rho, vx, vy, vz, p, Bx, By, Bz; floors applied, B_cc the mean of
 * the two bounding faces) of an MHD state, interior cells, [8][nz][ny][nx]. */
void orc_mhd_prims(const orc_cfg* cfg, const double* state, double* prims);

#ifdef __cplusplus
}
#endif
#endif
