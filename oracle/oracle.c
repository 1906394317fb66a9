/*
 * oracle.c -- plain FP64 CPU reference of the paper's Godunov step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls
 * this file; it shares no code with it.  It is written for a reader who checks it
 * against the paper by eye: every stage stores its intermediate arrays (primitives,
 * face fluxes, face and edge electric fields) on a grid padded with NG periodic ghost
 * cells, and nothing is fused or reordered beyond what the formulas state.
 *
 * Paper passages followed (Aether.jl, Ho):
 *   - conservation laws and closures ........ Sec. "Newtonian Magnetohydrodynamics",
 *                                              eqs. (mass)-(induction), (total_energy)
 *   - multifluid dust and implicit drag ..... Sec. "Multifluid Dust", eqs. (dust_mass),
 *                                              (dust_momentum); arrowhead drag solve
 *   - finite-volume update .................. Sec. "Reconstruction and Riemann Solvers",
 *                                              eq. (fv_update)
 *   - constrained transport ................. Sec. "Constrained Transport", eq. (ct)
 *   - two-register stages, IMEX2P, CFL ...... Sec. "Time Integration", eqs.
 *                                              (two_register), (cfl)
 * The formulas the paper only names (van Leer PLM, Colella-Woodward PPM, HLLE, the
 * HLLD solver of Miyoshi & Kusano, the Gardiner-Stone upwind edge EMF, the ARS(2,2,2)
 * IMEX pair) are written from the mathematics of those methods; each function says
 * which reading it takes where the paper is silent.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no contraction, so every
 * expression rounds as written).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NG 4 /* ghost width: PPM needs 3, constrained transport one more */

/* ------------------------------------------------------------------------------ */
/* padded periodic grid                                                            */
/* ------------------------------------------------------------------------------ */

typedef struct {
    int n[3];   /* interior cells per direction */
    int N[3];   /* padded extent */
    long st[3]; /* strides of the padded array */
    long ntot;
    double dx[3];
} grid_t;

static grid_t make_grid(const orc_cfg* c)
{
    grid_t g;
    g.n[0] = c->nx; g.n[1] = c->ny; g.n[2] = c->nz;
    for (int d = 0; d < 3; ++d) g.N[d] = g.n[d] + 2 * NG;
    g.st[0] = 1; g.st[1] = g.N[0]; g.st[2] = (long)g.N[0] * g.N[1];
    g.ntot = g.st[2] * g.N[2];
    g.dx[0] = c->dx; g.dx[1] = c->dy; g.dx[2] = c->dz;
    return g;
}

static inline long at(const grid_t* g, int i, int j, int k)
{
    return (long)(k + NG) * g->st[2] + (long)(j + NG) * g->st[1] + (i + NG);
}

static inline int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

static inline long cell(const grid_t* g, int i, int j, int k)
{
    return ((long)k * g->n[1] + j) * g->n[0] + i;
}

static long ncell(const grid_t* g) { return (long)g->n[0] * g->n[1] * g->n[2]; }

/* Copy one canonical field into a padded array, filling the periodic ghosts. */
static void pad_field(const grid_t* g, const double* src, double* dst)
{
#pragma omp parallel for
    for (int k = -NG; k < g->n[2] + NG; ++k)
        for (int j = -NG; j < g->n[1] + NG; ++j)
            for (int i = -NG; i < g->n[0] + NG; ++i)
                dst[at(g, i, j, k)] =
                    src[cell(g, wrap(i, g->n[0]), wrap(j, g->n[1]), wrap(k, g->n[2]))];
}

static double* zalloc(long n) { return (double*)calloc((size_t)n, sizeof(double)); }

static int nvar_cells(const orc_cfg* c)
{
    return c->eos == ORC_EOS_ADIABATIC_MHD ? 5 : 4 + 4 * c->ndust;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

long orc_state_len(const orc_cfg* c)
{
    long n = (long)c->nx * c->ny * c->nz;
    return n * (nvar_cells(c) + (c->eos == ORC_EOS_ADIABATIC_MHD ? 3 : 0));
}

/* ------------------------------------------------------------------------------ */
/* reconstruction (Sec. "Reconstruction and Riemann Solvers")                      */
/* ------------------------------------------------------------------------------ */

/* van Leer's monotonized harmonic-mean slope: 2 dm dp / (dm + dp) where the one-sided
 * differences agree in sign, zero at extrema. */
static double slope_vanleer(double am, double a0, double ap)
{
    double dm = a0 - am, dp = ap - a0;
    if (dm * dp > 0.0) return 2.0 * dm * dp / (dm + dp);
    return 0.0;
}

/* Colella & Woodward (1984) limited average slope (their eq. 1.8). */
static double ppm_dm(double am, double a0, double ap)
{
    double da = 0.5 * (ap - am);
    double dm = a0 - am, dp = ap - a0;
    if (dm * dp <= 0.0) return 0.0;
    double m = fabs(da);
    if (2.0 * fabs(dm) < m) m = 2.0 * fabs(dm);
    if (2.0 * fabs(dp) < m) m = 2.0 * fabs(dp);
    return da > 0.0 ? m : -m;
}

/* PPM interface value a_{c+1/2} from cells c-1 .. c+2 (CW84 eq. 1.6). */
static double ppm_interface(double am1, double a0, double ap1, double ap2)
{
    double d0 = ppm_dm(am1, a0, ap1);
    double d1 = ppm_dm(a0, ap1, ap2);
    return a0 + 0.5 * (ap1 - a0) - (d1 - d0) / 6.0;
}

/* Limited edge values (a_minus, a_plus) of the centre cell of s[0..4] (CW84 eq. 1.10). */
static void ppm_cell(const double* s, double* amin, double* aplu)
{
    double a0 = s[2];
    double lo = ppm_interface(s[0], s[1], s[2], s[3]); /* a_{c-1/2} */
    double hi = ppm_interface(s[1], s[2], s[3], s[4]); /* a_{c+1/2} */
    if ((hi - a0) * (a0 - lo) <= 0.0) {
        lo = a0;
        hi = a0;
    } else {
        double da = hi - lo;
        double a6 = 6.0 * (a0 - 0.5 * (lo + hi));
        if (da * a6 > da * da)
            lo = 3.0 * a0 - 2.0 * hi;
        else if (-da * da > da * a6)
            hi = 3.0 * a0 - 2.0 * lo;
    }
    *amin = lo;
    *aplu = hi;
}

/* Left/right states on the face between s[2] and s[3]; s holds six consecutive cells
 * along the sweep (the face f-1/2 sees cells f-3 .. f+2). */
static void recon_face(int recon, const double* s, double* aL, double* aR)
{
    if (recon == ORC_RECON_DC) {
        *aL = s[2];
        *aR = s[3];
    } else if (recon == ORC_RECON_PLM) {
        *aL = s[2] + 0.5 * slope_vanleer(s[1], s[2], s[3]);
        *aR = s[3] - 0.5 * slope_vanleer(s[2], s[3], s[4]);
    } else {
        double lo, hi;
        ppm_cell(s, &lo, &hi); /* cell f-1 from cells f-3 .. f+1 */
        *aL = hi;
        ppm_cell(s + 1, &lo, &hi); /* cell f from cells f-2 .. f+2 */
        *aR = lo;
    }
}

void orc_recon_line(int recon, int n, const double* a, double* aL, double* aR)
{
    double s[6];
    for (int f = 0; f < n; ++f) {
        for (int q = 0; q < 6; ++q) s[q] = a[wrap(f - 3 + q, n)];
        recon_face(recon, s, &aL[f], &aR[f]);
    }
}

/* ------------------------------------------------------------------------------ */
/* Riemann solvers in the face frame                                               */
/* ------------------------------------------------------------------------------ */

/* Conserved state, physical flux and total pressure of a face-frame MHD state
 * w = (rho, u, v, w, p, By, Bz) with normal field bn; eqs. (momentum)-(induction)
 * written along the normal, with P* = p + B.B/2 and E from eq. (total_energy). */
static void mhd_state_flux(double gam, const double* w, double bn, double* U, double* F,
                           double* pt)
{
    double rho = w[0], u = w[1], v = w[2], ww = w[3], p = w[4], by = w[5], bz = w[6];
    double b2 = bn * bn + (by * by + bz * bz);
    double v2 = u * u + (v * v + ww * ww);
    double ptot = p + 0.5 * b2;
    double E = p / (gam - 1.0) + 0.5 * rho * v2 + 0.5 * b2;
    double vb = u * bn + (v * by + ww * bz);
    U[0] = rho; U[1] = rho * u; U[2] = rho * v; U[3] = rho * ww; U[4] = E; U[5] = by; U[6] = bz;
    F[0] = rho * u;
    F[1] = rho * u * u + ptot - bn * bn;
    F[2] = rho * u * v - bn * by;
    F[3] = rho * u * ww - bn * bz;
    F[4] = (E + ptot) * u - bn * vb;
    F[5] = by * u - bn * v;
    F[6] = bz * u - bn * ww;
    *pt = ptot;
}

/* Fast magnetosonic speed along a direction whose field component is bd:
 * c_f^2 = ((a^2 + B^2/rho) + sqrt((a^2 + B^2/rho)^2 - 4 a^2 bd^2/rho)) / 2, a^2 = gamma p/rho. */
static double fast_speed(double gam, double rho, double p, double b2, double bd)
{
    double a2 = gam * p / rho;
    double s = a2 + b2 / rho;
    double disc = s * s - 4.0 * a2 * bd * bd / rho;
    if (disc < 0.0) disc = 0.0;
    return sqrt(0.5 * (s + sqrt(disc)));
}

/* Outer wave-speed bounds: min/max of the normal velocities -/+ the larger fast speed. */
static void mhd_bounds(double gam, const double* wl, const double* wr, double bn, double* sl,
                       double* sr)
{
    double b2l = bn * bn + (wl[5] * wl[5] + wl[6] * wl[6]);
    double b2r = bn * bn + (wr[5] * wr[5] + wr[6] * wr[6]);
    double cl = fast_speed(gam, wl[0], wl[4], b2l, bn);
    double cr = fast_speed(gam, wr[0], wr[4], b2r, bn);
    double cmax = cl > cr ? cl : cr;
    double umin = wl[1] < wr[1] ? wl[1] : wr[1];
    double umax = wl[1] > wr[1] ? wl[1] : wr[1];
    *sl = umin - cmax;
    *sr = umax + cmax;
}

/* HLLE: the single-state HLL average between the bounds, with b- = min(S_L,0),
 * b+ = max(S_R,0). */
static void hlle_mhd(double gam, const double* wl, const double* wr, double bn, double* f)
{
    double UL[7], FL[7], UR[7], FR[7], ptl, ptr, sl, sr;
    mhd_state_flux(gam, wl, bn, UL, FL, &ptl);
    mhd_state_flux(gam, wr, bn, UR, FR, &ptr);
    mhd_bounds(gam, wl, wr, bn, &sl, &sr);
    double bm = sl < 0.0 ? sl : 0.0;
    double bp = sr > 0.0 ? sr : 0.0;
    for (int q = 0; q < 7; ++q)
        f[q] = (bp * FL[q] - bm * FR[q] + bp * bm * (UR[q] - UL[q])) / (bp - bm);
}

/* Star state of side a of the HLLD fan (Miyoshi & Kusano 2005): density jump across the
 * fast wave, transverse velocity/field from the Rankine-Hugoniot conditions, and the
 * energy from the energy jump condition.  If the denominator D degenerates (|D| <=
 * eps*pts) the transverse quantities keep their outer values. */
typedef struct {
    double rho, v, w, by, bz, E, vb;
} star_t;

static star_t hlld_star(double eps, const double* U, const double* w, double pt, double bn,
                        double S, double SM, double pts)
{
    star_t s;
    double rho = w[0], u = w[1];
    double d = S - u;
    s.rho = rho * d / (S - SM);
    double D = rho * d * (S - SM) - bn * bn;
    if (fabs(D) <= eps * pts) {
        s.v = w[2]; s.w = w[3]; s.by = w[5]; s.bz = w[6];
    } else {
        s.v = w[2] - bn * w[5] * (SM - u) / D;
        s.w = w[3] - bn * w[6] * (SM - u) / D;
        s.by = w[5] * (rho * d * d - bn * bn) / D;
        s.bz = w[6] * (rho * d * d - bn * bn) / D;
    }
    s.vb = SM * bn + (s.v * s.by + s.w * s.bz);
    double vb = u * bn + (w[2] * w[5] + w[3] * w[6]);
    s.E = (d * U[4] - pt * u + pts * SM + bn * (vb - s.vb)) / (S - SM);
    return s;
}

static void pack_state(const star_t* s, double SM, double E, double v, double w, double by,
                       double bz, double* U)
{
    U[0] = s->rho; U[1] = s->rho * SM; U[2] = s->rho * v; U[3] = s->rho * w;
    U[4] = E; U[5] = by; U[6] = bz;
}

static void hlld_mhd(double gam, double eps, const double* wl, const double* wr, double bn,
                     double* f)
{
    double UL[7], FL[7], UR[7], FR[7], ptl, ptr, sl, sr;
    mhd_state_flux(gam, wl, bn, UL, FL, &ptl);
    mhd_state_flux(gam, wr, bn, UR, FR, &ptr);
    mhd_bounds(gam, wl, wr, bn, &sl, &sr);
    if (sl > 0.0) { memcpy(f, FL, sizeof FL); return; }
    if (sr < 0.0) { memcpy(f, FR, sizeof FR); return; }

    double dl = sl - wl[1], dr = sr - wr[1];
    double den = dr * wr[0] - dl * wl[0];
    /* entropy-wave speed and the total pressure that is constant across the fan */
    double SM = (dr * wr[0] * wr[1] - dl * wl[0] * wl[1] - ptr + ptl) / den;
    double pts = (dr * wr[0] * ptl - dl * wl[0] * ptr + wl[0] * wr[0] * dr * dl * (wr[1] - wl[1])) / den;

    star_t sL = hlld_star(eps, UL, wl, ptl, bn, sl, SM, pts);
    star_t sR = hlld_star(eps, UR, wr, ptr, bn, sr, SM, pts);
    double UsL[7], UsR[7], UssL[7], UssR[7];
    pack_state(&sL, SM, sL.E, sL.v, sL.w, sL.by, sL.bz, UsL);
    pack_state(&sR, SM, sR.E, sR.v, sR.w, sR.by, sR.bz, UsR);

    /* rotational (Alfven) waves */
    double rl = sqrt(sL.rho), rr = sqrt(sR.rho);
    double slst = SM - fabs(bn) / rl;
    double srst = SM + fabs(bn) / rr;

    if (bn * bn <= eps * pts) {
        memcpy(UssL, UsL, sizeof UsL);
        memcpy(UssR, UsR, sizeof UsR);
    } else {
        double sg = bn > 0.0 ? 1.0 : -1.0;
        double inv = 1.0 / (rl + rr);
        double vss = (rl * sL.v + rr * sR.v + (sR.by - sL.by) * sg) * inv;
        double wss = (rl * sL.w + rr * sR.w + (sR.bz - sL.bz) * sg) * inv;
        double byss = (rl * sR.by + rr * sL.by + rl * rr * (sR.v - sL.v) * sg) * inv;
        double bzss = (rl * sR.bz + rr * sL.bz + rl * rr * (sR.w - sL.w) * sg) * inv;
        double vbss = SM * bn + (vss * byss + wss * bzss);
        double EssL = sL.E - rl * (sL.vb - vbss) * sg;
        double EssR = sR.E + rr * (sR.vb - vbss) * sg;
        pack_state(&sL, SM, EssL, vss, wss, byss, bzss, UssL);
        pack_state(&sR, SM, EssR, vss, wss, byss, bzss, UssR);
    }

    double FsL[7], FsR[7];
    for (int q = 0; q < 7; ++q) {
        FsL[q] = FL[q] + sl * (UsL[q] - UL[q]);
        FsR[q] = FR[q] + sr * (UsR[q] - UR[q]);
    }
    if (slst >= 0.0) { memcpy(f, FsL, sizeof FsL); return; }
    if (SM >= 0.0) {
        for (int q = 0; q < 7; ++q) f[q] = FsL[q] + slst * (UssL[q] - UsL[q]);
        return;
    }
    if (srst >= 0.0) {
        for (int q = 0; q < 7; ++q) f[q] = FsR[q] + srst * (UssR[q] - UsR[q]);
        return;
    }
    memcpy(f, FsR, sizeof FsR);
}

void orc_riemann_mhd(const orc_cfg* c, const double* wl, const double* wr, double bn, double* f)
{
    if (c->riemann == ORC_RS_HLLD)
        hlld_mhd(c->gamma, c->hlld_eps, wl, wr, bn, f);
    else
        hlle_mhd(c->gamma, wl, wr, bn, f);
}

/* Isothermal hydro HLLE, p = cs^2 rho, bounds min/max(u) -/+ cs. */
void orc_riemann_iso_hlle(double cs, const double* wl, const double* wr, double* f)
{
    double UL[4], UR[4], FL[4], FR[4];
    const double* w[2] = {wl, wr};
    double* U[2] = {UL, UR};
    double* F[2] = {FL, FR};
    for (int s = 0; s < 2; ++s) {
        double rho = w[s][0], u = w[s][1];
        U[s][0] = rho; U[s][1] = rho * u; U[s][2] = rho * w[s][2]; U[s][3] = rho * w[s][3];
        F[s][0] = rho * u;
        F[s][1] = rho * u * u + cs * cs * rho;
        F[s][2] = rho * u * w[s][2];
        F[s][3] = rho * u * w[s][3];
    }
    double umin = wl[1] < wr[1] ? wl[1] : wr[1];
    double umax = wl[1] > wr[1] ? wl[1] : wr[1];
    double sl = umin - cs, sr = umax + cs;
    double bm = sl < 0.0 ? sl : 0.0;
    double bp = sr > 0.0 ? sr : 0.0;
    for (int q = 0; q < 4; ++q)
        f[q] = (bp * FL[q] - bm * FR[q] + bp * bm * (UR[q] - UL[q])) / (bp - bm);
}

/* Pressureless Rusanov flux (the paper's default dust flux): the central average minus
 * max(|u_L|,|u_R|)/2 times the jump; F = u U for U = (rho, rho u, rho v, rho w). */
void orc_riemann_dust_rusanov(const double* wl, const double* wr, double* f)
{
    double UL[4], UR[4];
    UL[0] = wl[0]; UL[1] = wl[0] * wl[1]; UL[2] = wl[0] * wl[2]; UL[3] = wl[0] * wl[3];
    UR[0] = wr[0]; UR[1] = wr[0] * wr[1]; UR[2] = wr[0] * wr[2]; UR[3] = wr[0] * wr[3];
    double a = fabs(wl[1]) > fabs(wr[1]) ? fabs(wl[1]) : fabs(wr[1]);
    for (int q = 0; q < 4; ++q)
        f[q] = 0.5 * (wl[1] * UL[q] + wr[1] * UR[q]) - 0.5 * a * (UR[q] - UL[q]);
}

/* ------------------------------------------------------------------------------ */
/* MHD right-hand side L(u) of one stage                                            */
/* ------------------------------------------------------------------------------ */

enum { RHO = 0, MX = 1, MY = 2, MZ = 3, EN = 4 };
enum { W_RHO = 0, W_VX = 1, W_P = 4, W_BX = 5 };

typedef struct {
    grid_t g;
    double* u[5];     /* padded conserved cell fields */
    double* b[3];     /* padded face fields */
    double* w[8];     /* padded primitives rho, vx, vy, vz, p, Bx, By, Bz (cell-centred) */
    double* F[3][5];  /* face fluxes of the cell variables, per sweep direction */
    double* FE[3][3]; /* face electric field (the two tangential components) per sweep */
    double* R[3];     /* cell-centred reference electric field -v x B */
    double* Ed[3];    /* edge electric fields */
} mhd_work;

static void mhd_work_alloc(mhd_work* W, const orc_cfg* c)
{
    W->g = make_grid(c);
    long n = W->g.ntot;
    for (int q = 0; q < 5; ++q) W->u[q] = zalloc(n);
    for (int q = 0; q < 3; ++q) W->b[q] = zalloc(n);
    for (int q = 0; q < 8; ++q) W->w[q] = zalloc(n);
    for (int d = 0; d < 3; ++d) {
        for (int q = 0; q < 5; ++q) W->F[d][q] = zalloc(n);
        for (int q = 0; q < 3; ++q) W->FE[d][q] = (q == d) ? NULL : zalloc(n);
        W->R[d] = zalloc(n);
        W->Ed[d] = zalloc(n);
    }
}

static void mhd_work_free(mhd_work* W)
{
    for (int q = 0; q < 5; ++q) free(W->u[q]);
    for (int q = 0; q < 3; ++q) free(W->b[q]);
    for (int q = 0; q < 8; ++q) free(W->w[q]);
    for (int d = 0; d < 3; ++d) {
        for (int q = 0; q < 5; ++q) free(W->F[d][q]);
        for (int q = 0; q < 3; ++q) free(W->FE[d][q]);
        free(W->R[d]);
        free(W->Ed[d]);
    }
}

/* Conserved -> primitive with the density and pressure floors (Sec. "Newtonian Magnetohydrodynamics"):
 * B_cc is the mean of the two bounding face values (Sec. "Constrained Transport"),
 * p = (gamma-1)(E - rho v^2/2 - B^2/2).  The floors act on the primitives only. */
static void mhd_prims(const orc_cfg* c, mhd_work* W)
{
    const grid_t* g = &W->g;
#pragma omp parallel for
    for (int k = -NG; k < g->n[2] + NG - 1; ++k)
        for (int j = -NG; j < g->n[1] + NG - 1; ++j)
            for (int i = -NG; i < g->n[0] + NG - 1; ++i) {
                long id = at(g, i, j, k);
                double bx = 0.5 * (W->b[0][id] + W->b[0][id + g->st[0]]);
                double by = 0.5 * (W->b[1][id] + W->b[1][id + g->st[1]]);
                double bz = 0.5 * (W->b[2][id] + W->b[2][id + g->st[2]]);
                double rho = W->u[RHO][id];
                if (rho < c->rho_floor) rho = c->rho_floor;
                double vx = W->u[MX][id] / rho, vy = W->u[MY][id] / rho, vz = W->u[MZ][id] / rho;
                double ke = 0.5 * rho * ((vx * vx + vy * vy) + vz * vz);
                double me = 0.5 * ((bx * bx + by * by) + bz * bz);
                double p = (c->gamma - 1.0) * ((W->u[EN][id] - ke) - me);
                if (p < c->p_floor) p = c->p_floor;
                W->w[0][id] = rho; W->w[1][id] = vx; W->w[2][id] = vy; W->w[3][id] = vz;
                W->w[4][id] = p; W->w[5][id] = bx; W->w[6][id] = by; W->w[7][id] = bz;
            }
}

/* Face fluxes along direction d for faces 0..n_d (left faces of cells) and transverse
 * indices -1..n_t (one extra ring for the edge fields).  Primitives are reconstructed
 * componentwise, rotated into the face frame (n, t1, t2) = (d, d+1, d+2) cyclic, solved,
 * and rotated back. */
static void mhd_fluxes(const orc_cfg* c, int recon, mhd_work* W, int d)
{
    const grid_t* g = &W->g;
    int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = -1; hi[a] = g->n[a]; }
    lo[d] = 0;
    long sd = g->st[d];
    /* primitive indices in the face frame: rho, v_n, v_t1, v_t2, p, B_t1, B_t2 */
    int comp[7] = {0, 1 + d, 1 + t1, 1 + t2, 4, 5 + t1, 5 + t2};
#pragma omp parallel for
    for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
            for (int i = lo[0]; i <= hi[0]; ++i) {
                long id = at(g, i, j, k);
                double wl[7], wr[7], s[6], f[7];
                for (int q = 0; q < 7; ++q) {
                    for (int m = 0; m < 6; ++m) s[m] = W->w[comp[q]][id + (m - 3) * sd];
                    recon_face(recon, s, &wl[q], &wr[q]);
                }
                orc_riemann_mhd(c, wl, wr, W->b[d][id], f);
                W->F[d][RHO][id] = f[0];
                W->F[d][1 + d][id] = f[1];
                W->F[d][1 + t1][id] = f[2];
                W->F[d][1 + t2][id] = f[3];
                W->F[d][EN][id] = f[4];
                /* flux of B_t1 along n is -E_t2, flux of B_t2 is +E_t1 */
                W->FE[d][t2][id] = -f[5];
                W->FE[d][t1][id] = f[6];
            }
}

/* Cell-centred electric field E = -v x B (Sec. "Constrained Transport"). */
static void mhd_ref_emf(mhd_work* W)
{
    const grid_t* g = &W->g;
#pragma omp parallel for
    for (int k = -1; k <= g->n[2]; ++k)
        for (int j = -1; j <= g->n[1]; ++j)
            for (int i = -1; i <= g->n[0]; ++i) {
                long id = at(g, i, j, k);
                double vx = W->w[1][id], vy = W->w[2][id], vz = W->w[3][id];
                double bx = W->w[5][id], by = W->w[6][id], bz = W->w[7][id];
                W->R[0][id] = vz * by - vy * bz;
                W->R[1][id] = vx * bz - vz * bx;
                W->R[2][id] = vy * bx - vx * by;
            }
}

/* Upwind choice of a gradient correction by the sign of the mass flux; a mass flux of
 * exactly zero takes the mean of the two candidates. */
static double upwind(double mflux, double if_pos, double if_neg)
{
    if (mflux > 0.0) return if_pos;
    if (mflux < 0.0) return if_neg;
    return 0.5 * (if_pos + if_neg);
}

/* Edge electric field E_a by the Gardiner & Stone (2005) upwind ("contact") averaging.
 * With (p, q) = (a+1, a+2) cyclic, the edge sits at (p-1/2, q-1/2) and the centre of
 * the cell range along a.  The four face values X (on p-faces) and Y (on q-faces) are
 * averaged, and each is extrapolated to the edge with a gradient taken between the face
 * value and the neighbouring cell-centred field R, chosen upwind of the mass flux
 * through the face the gradient lies on.  The correction enters with the sign that
 * makes the edge value equal the face value in a plane-parallel flow. */
static void mhd_edge_emf(mhd_work* W, int a)
{
    const grid_t* g = &W->g;
    int p = (a + 1) % 3, q = (a + 2) % 3;
    long sp = g->st[p], sq = g->st[q];
    int lo[3] = {0, 0, 0}, hi[3];
    for (int e = 0; e < 3; ++e) hi[e] = g->n[e];
    hi[a] = g->n[a] - 1;
    const double* X = W->FE[p][a];
    const double* Y = W->FE[q][a];
    const double* R = W->R[a];
    const double* fp = W->F[p][RHO];
    const double* fq = W->F[q][RHO];
#pragma omp parallel for
    for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
            for (int i = lo[0]; i <= hi[0]; ++i) {
                long id = at(g, i, j, k);
                double X0 = X[id], Xm = X[id - sq];
                double Y0 = Y[id], Ym = Y[id - sp];
                double R00 = R[id], Rm0 = R[id - sp], R0m = R[id - sq], Rmm = R[id - sp - sq];
                double dqp = upwind(fp[id], Rm0 - Ym, R00 - Y0);
                double dqm = upwind(fp[id - sq], Ym - Rmm, Y0 - R0m);
                double dpp = upwind(fq[id], R0m - Xm, R00 - X0);
                double dpm = upwind(fq[id - sp], Xm - Rmm, X0 - Rm0);
                W->Ed[a][id] = 0.25 * (((X0 + Xm) + (Y0 + Ym)) - ((dqp - dqm) + (dpp - dpm)));
            }
}

/* Full right-hand side: dU/dt from eq. (fv_update) plus the unsplit gas acceleration,
 * db/dt = -curl E on the faces from eq. (ct).  Inputs/outputs are canonical. */
static void mhd_rhs(const orc_cfg* c, int recon, mhd_work* W, const double* state,
                    double* dudt)
{
    const grid_t* g = &W->g;
    long nc = ncell(g);
    for (int q = 0; q < 5; ++q) pad_field(g, state + q * nc, W->u[q]);
    for (int q = 0; q < 3; ++q) pad_field(g, state + (5 + q) * nc, W->b[q]);
    mhd_prims(c, W);
    for (int d = 0; d < 3; ++d) mhd_fluxes(c, recon, W, d);
    mhd_ref_emf(W);
    for (int a = 0; a < 3; ++a) mhd_edge_emf(W, a);

    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2];
#pragma omp parallel for
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                long id = at(g, i, j, k), ci = cell(g, i, j, k);
                for (int v = 0; v < 5; ++v) {
                    double fx = (W->F[0][v][id + g->st[0]] - W->F[0][v][id]) / dx;
                    double fy = (W->F[1][v][id + g->st[1]] - W->F[1][v][id]) / dy;
                    double fz = (W->F[2][v][id + g->st[2]] - W->F[2][v][id]) / dz;
                    dudt[v * nc + ci] = -((fx + fy) + fz);
                }
                /* unsplit source of a constant gas acceleration: rho g and its work M.g */
                double rho = W->u[RHO][id];
                dudt[MX * nc + ci] += rho * c->gacc[0];
                dudt[MY * nc + ci] += rho * c->gacc[1];
                dudt[MZ * nc + ci] += rho * c->gacc[2];
                dudt[EN * nc + ci] += (W->u[MX][id] * c->gacc[0] + W->u[MY][id] * c->gacc[1]) +
                                      W->u[MZ][id] * c->gacc[2];
                /* faces: E_x at (i, j-1/2, k-1/2), E_y at (i-1/2, j, k-1/2), E_z at (i-1/2, j-1/2, k) */
                const double *Ex = W->Ed[0], *Ey = W->Ed[1], *Ez = W->Ed[2];
                double db1 = -((Ez[id + g->st[1]] - Ez[id]) / dy - (Ey[id + g->st[2]] - Ey[id]) / dz);
                double db2 = -((Ex[id + g->st[2]] - Ex[id]) / dz - (Ez[id + g->st[0]] - Ez[id]) / dx);
                double db3 = -((Ey[id + g->st[0]] - Ey[id]) / dx - (Ex[id + g->st[1]] - Ex[id]) / dy);
                dudt[5 * nc + ci] = db1;
                dudt[6 * nc + ci] = db2;
                dudt[7 * nc + ci] = db3;
            }
}

void orc_rhs_mhd_debug(const orc_cfg* c, int recon, const double* state, double* dudt,
                       double* emf, double* facee)
{
    mhd_work W;
    mhd_work_alloc(&W, c);
    mhd_rhs(c, recon, &W, state, dudt);
    const grid_t* g = &W.g;
    long nc = ncell(g);
    const double* fe[6] = {W.FE[0][1], W.FE[0][2], W.FE[1][2], W.FE[1][0], W.FE[2][0], W.FE[2][1]};
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                long id = at(g, i, j, k), ci = cell(g, i, j, k);
                for (int a = 0; a < 3; ++a) emf[a * nc + ci] = W.Ed[a][id];
                for (int q = 0; q < 6; ++q) facee[q * nc + ci] = fe[q][id];
            }
    mhd_work_free(&W);
}

/* The 8 cell primitives (rho, v, p, B_cc) of an MHD state as the stage computes them,
 * interior cells, [8][nz][ny][nx]; for tests. */
void orc_mhd_prims(const orc_cfg* c, const double* state, double* prims)
{
    mhd_work W;
    mhd_work_alloc(&W, c);
    const grid_t* g = &W.g;
    long nc = ncell(g);
    for (int q = 0; q < 5; ++q) pad_field(g, state + q * nc, W.u[q]);
    for (int q = 0; q < 3; ++q) pad_field(g, state + (5 + q) * nc, W.b[q]);
    mhd_prims(c, &W);
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                long id = at(g, i, j, k), ci = cell(g, i, j, k);
                for (int q = 0; q < 8; ++q) prims[q * nc + ci] = W.w[q][id];
            }
    mhd_work_free(&W);
}

/* ------------------------------------------------------------------------------ */
/* isothermal gas + N pressureless dust: explicit part F(u) and drag G(u)           */
/* ------------------------------------------------------------------------------ */

/* Primitives of fluid s (s = 0 gas, s >= 1 dust species s-1) from padded conserved
 * fields: density (gas floor / dust floor with zero velocity) and velocity. */
static void fluid_prims(const orc_cfg* c, int s, const double* rho_in, const double* m0,
                        const double* m1, const double* m2, double* w)
{
    double rho = *rho_in;
    if (s == 0) {
        if (rho < c->rho_floor) rho = c->rho_floor;
        w[0] = rho; w[1] = *m0 / rho; w[2] = *m1 / rho; w[3] = *m2 / rho;
    } else if (rho < c->dust_rho_floor) {
        w[0] = c->dust_rho_floor; w[1] = 0.0; w[2] = 0.0; w[3] = 0.0;
    } else {
        w[0] = rho; w[1] = *m0 / rho; w[2] = *m1 / rho; w[3] = *m2 / rho;
    }
}

/* Explicit right-hand side: minus the flux divergence of every fluid (isothermal HLLE
 * for the gas, pressureless Rusanov for each dust species) plus rho_g g on the gas. */
static void dust_explicit_rhs(const orc_cfg* c, const double* state, double* dudt)
{
    grid_t gg = make_grid(c);
    const grid_t* g = &gg;
    long nc = ncell(g);
    int nf = 1 + c->ndust, nv = 4 * nf;
    double** u = (double**)malloc(sizeof(double*) * nv);
    double** w = (double**)malloc(sizeof(double*) * nv);
    double** F = (double**)malloc(sizeof(double*) * 3 * nv);
    for (int q = 0; q < nv; ++q) {
        u[q] = zalloc(g->ntot);
        w[q] = zalloc(g->ntot);
        pad_field(g, state + q * nc, u[q]);
    }
    for (int q = 0; q < 3 * nv; ++q) F[q] = zalloc(g->ntot);

#pragma omp parallel for
    for (int k = -NG; k < g->n[2] + NG; ++k)
        for (int j = -NG; j < g->n[1] + NG; ++j)
            for (int i = -NG; i < g->n[0] + NG; ++i) {
                long id = at(g, i, j, k);
                for (int s = 0; s < nf; ++s) {
                    double ws[4];
                    fluid_prims(c, s, &u[4 * s][id], &u[4 * s + 1][id], &u[4 * s + 2][id],
                                &u[4 * s + 3][id], ws);
                    for (int q = 0; q < 4; ++q) w[4 * s + q][id] = ws[q];
                }
            }

    for (int d = 0; d < 3; ++d) {
        int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
        long sd = g->st[d];
        int comp[4] = {0, 1 + d, 1 + t1, 1 + t2};
#pragma omp parallel for
        for (int k = 0; k <= g->n[2]; ++k)
            for (int j = 0; j <= g->n[1]; ++j)
                for (int i = 0; i <= g->n[0]; ++i) {
                    long id = at(g, i, j, k);
                    for (int s = 0; s < nf; ++s) {
                        double wl[4], wr[4], st6[6], f[4];
                        for (int q = 0; q < 4; ++q) {
                            for (int m = 0; m < 6; ++m) st6[m] = w[4 * s + comp[q]][id + (m - 3) * sd];
                            recon_face(c->recon, st6, &wl[q], &wr[q]);
                        }
                        if (s == 0)
                            orc_riemann_iso_hlle(c->cs, wl, wr, f);
                        else
                            orc_riemann_dust_rusanov(wl, wr, f);
                        F[d * nv + 4 * s][id] = f[0];
                        F[d * nv + 4 * s + 1 + d][id] = f[1];
                        F[d * nv + 4 * s + 1 + t1][id] = f[2];
                        F[d * nv + 4 * s + 1 + t2][id] = f[3];
                    }
                }
    }

    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2];
#pragma omp parallel for
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                long id = at(g, i, j, k), ci = cell(g, i, j, k);
                for (int v = 0; v < nv; ++v) {
                    double fx = (F[v][id + g->st[0]] - F[v][id]) / dx;
                    double fy = (F[nv + v][id + g->st[1]] - F[nv + v][id]) / dy;
                    double fz = (F[2 * nv + v][id + g->st[2]] - F[2 * nv + v][id]) / dz;
                    dudt[v * nc + ci] = -((fx + fy) + fz);
                }
                double rho = u[0][id];
                for (int a = 0; a < 3; ++a) dudt[(1 + a) * nc + ci] += rho * c->gacc[a];
            }

    for (int q = 0; q < nv; ++q) { free(u[q]); free(w[q]); }
    for (int q = 0; q < 3 * nv; ++q) free(F[q]);
    free(u); free(w); free(F);
}

/* Drag rates G(u) on the momenta, eq. (dust_momentum) and its reaction on the gas:
 * species k: rho_k (v - v_k)/t_k = (rho_k v - p_k)/t_k, written with the species
 * momentum p_k so that it is the linear map of the momenta that the implicit solve
 * inverts; gas: minus the sum over species.  Densities are unchanged by drag. */
static void dust_drag_rate(const orc_cfg* c, const double* state, double* G)
{
    long nc = (long)c->nx * c->ny * c->nz;
    int nf = 1 + c->ndust, nv = 4 * nf;
    memset(G, 0, sizeof(double) * nv * nc);
#pragma omp parallel for
    for (long ci = 0; ci < nc; ++ci) {
        double wg[4];
        fluid_prims(c, 0, &state[ci], &state[nc + ci], &state[2 * nc + ci], &state[3 * nc + ci], wg);
        for (int s = 1; s < nf; ++s) {
            double rk = state[4 * s * nc + ci];
            for (int a = 0; a < 3; ++a) {
                double pk = state[(4 * s + 1 + a) * nc + ci];
                double fk = (rk * wg[1 + a] - pk) / c->tstop[s - 1];
                G[(4 * s + 1 + a) * nc + ci] += fk;
                G[(1 + a) * nc + ci] -= fk;
            }
        }
    }
}

/* Dense LU with partial pivoting of (I - h J) x = p, J the drag Jacobian on the momenta
 * with densities fixed.  Deliberately the plain linear-algebra route, not the closed
 * arrowhead form. */
void orc_drag_solve(int n, const double* rho, const double* p, const double* ts, double h,
                    double* pout)
{
    int m = n + 1;
    double A[ORC_MAX_DUST + 1][ORC_MAX_DUST + 1];
    double x[ORC_MAX_DUST + 1];
    for (int r = 0; r < m; ++r) {
        for (int q = 0; q < m; ++q) A[r][q] = 0.0;
        x[r] = p[r];
    }
    /* J[0][0] = -sum eps_k/t_k, J[0][k] = 1/t_k, J[k][0] = eps_k/t_k, J[k][k] = -1/t_k */
    double j00 = 0.0;
    for (int k = 1; k <= n; ++k) {
        double eps = rho[k] / rho[0];
        j00 -= eps / ts[k - 1];
        A[0][k] = -h * (1.0 / ts[k - 1]);
        A[k][0] = -h * (eps / ts[k - 1]);
        A[k][k] = 1.0 - h * (-1.0 / ts[k - 1]);
    }
    A[0][0] = 1.0 - h * j00;
    int piv[ORC_MAX_DUST + 1];
    for (int r = 0; r < m; ++r) piv[r] = r;
    for (int col = 0; col < m; ++col) {
        int best = col;
        for (int r = col + 1; r < m; ++r)
            if (fabs(A[r][col]) > fabs(A[best][col])) best = r;
        if (best != col) {
            for (int q = 0; q < m; ++q) { double t = A[col][q]; A[col][q] = A[best][q]; A[best][q] = t; }
            double t = x[col]; x[col] = x[best]; x[best] = t;
            int ti = piv[col]; piv[col] = piv[best]; piv[best] = ti;
        }
        for (int r = col + 1; r < m; ++r) {
            double l = A[r][col] / A[col][col];
            for (int q = col; q < m; ++q) A[r][q] -= l * A[col][q];
            x[r] -= l * x[col];
        }
    }
    for (int r = m - 1; r >= 0; --r) {
        double s = x[r];
        for (int q = r + 1; q < m; ++q) s -= A[r][q] * x[q];
        x[r] = s / A[r][r];
    }
    for (int r = 0; r < m; ++r) pout[r] = x[r];
}

/* S_h: solve the implicit drag stage cell by cell, component by component. */
static void dust_drag_stage(const orc_cfg* c, double* state, double h)
{
    long nc = (long)c->nx * c->ny * c->nz;
    int n = c->ndust;
#pragma omp parallel for
    for (long ci = 0; ci < nc; ++ci) {
        double rho[ORC_MAX_DUST + 1], p[ORC_MAX_DUST + 1], po[ORC_MAX_DUST + 1];
        for (int s = 0; s <= n; ++s) rho[s] = state[4 * s * nc + ci];
        for (int a = 0; a < 3; ++a) {
            for (int s = 0; s <= n; ++s) p[s] = state[(4 * s + 1 + a) * nc + ci];
            orc_drag_solve(n, rho, p, c->tstop, h, po);
            for (int s = 0; s <= n; ++s) state[(4 * s + 1 + a) * nc + ci] = po[s];
        }
    }
}

/* The dust floor of Sec. "Multifluid Dust": a species whose density is below the floor
 * is reset to the floor with zero velocity.  Reading: the reset rewrites the state a
 * step starts from (the gas density floor only limits the primitives).  Inside the
 * step a species that stage 1 drives below the floor is converted to primitives as the
 * floor at rest (fluxes, time step) but not rewritten, because the drag rate of the
 * stage-1 state is the one its implicit solve used. */
static void dust_floor_reset(const orc_cfg* c, double* state)
{
    long nc = (long)c->nx * c->ny * c->nz;
    for (int s = 1; s <= c->ndust; ++s) {
        double* rho = state + 4 * s * nc;
#pragma omp parallel for
        for (long ci = 0; ci < nc; ++ci)
            if (rho[ci] < c->dust_rho_floor) {
                rho[ci] = c->dust_rho_floor;
                for (int a = 1; a <= 3; ++a) rho[a * nc + ci] = 0.0;
            }
    }
}

/* IMEX2P: ARS(2,2,2) with the diagonal weight lambda = 1 + 1/sqrt(2) (Sec. "Time
 * Integration") and the explicit weight delta = 1 - 1/(2 lambda):
 *   U1      = u + lambda dt F(u) + lambda dt G(U1)
 *   u_new   = u + dt [delta F(u) + (1-delta) F(U1)] + dt [(1-lambda) G(U1) + lambda G(u_new)]
 * Each implicit stage is the drag solve S_h with h = lambda dt.  The state u passes the
 * dust floor reset first. */
static void imex2p_step(const orc_cfg* c, double* state, double dt)
{
    long len = orc_state_len(c);
    const double lam = 1.0 + 1.0 / sqrt(2.0);
    const double del = 1.0 - 1.0 / (2.0 * lam);
    double* Fn = zalloc(len);
    double* F1 = zalloc(len);
    double* G1 = zalloc(len);
    double* U1 = zalloc(len);
    dust_floor_reset(c, state);
    dust_explicit_rhs(c, state, Fn);
    for (long e = 0; e < len; ++e) U1[e] = state[e] + (lam * dt) * Fn[e];
    dust_drag_stage(c, U1, lam * dt);
    dust_explicit_rhs(c, U1, F1);
    dust_drag_rate(c, U1, G1);
    for (long e = 0; e < len; ++e)
        state[e] = state[e] + dt * (del * Fn[e] + (1.0 - del) * F1[e]) + (dt * (1.0 - lam)) * G1[e];
    dust_drag_stage(c, state, lam * dt);
    free(Fn); free(F1); free(G1); free(U1);
}

/* ------------------------------------------------------------------------------ */
/* two-register explicit integrators, eq. (two_register)                           */
/* ------------------------------------------------------------------------------ */

typedef struct {
    int nstage;
    double delta[2], g0[2], g1[2], beta[2];
    int recon[2];
} tableau_t;

/* VL2 (predictor-corrector): a donor-cell half step, then a full step from the
 * half-step state with the configured reconstruction.  RK2: the optimal two-stage SSP
 * scheme.  EULER1: one forward-Euler stage (tests only). */
static tableau_t make_tableau(const orc_cfg* c)
{
    tableau_t t;
    memset(&t, 0, sizeof t);
    if (c->integ == ORC_INT_VL2) {
        t.nstage = 2;
        t.delta[0] = 1; t.g0[0] = 0; t.g1[0] = 1; t.beta[0] = 0.5; t.recon[0] = ORC_RECON_DC;
        t.delta[1] = 0; t.g0[1] = 0; t.g1[1] = 1; t.beta[1] = 1.0; t.recon[1] = c->recon;
    } else if (c->integ == ORC_INT_RK2) {
        t.nstage = 2;
        t.delta[0] = 1; t.g0[0] = 0; t.g1[0] = 1; t.beta[0] = 1.0; t.recon[0] = c->recon;
        t.delta[1] = 0; t.g0[1] = 0.5; t.g1[1] = 0.5; t.beta[1] = 0.5; t.recon[1] = c->recon;
    } else {
        t.nstage = 1;
        t.delta[0] = 1; t.g0[0] = 0; t.g1[0] = 1; t.beta[0] = 1.0; t.recon[0] = c->recon;
    }
    return t;
}

static void explicit_mhd_step(const orc_cfg* c, double* state, double dt)
{
    long len = orc_state_len(c);
    tableau_t t = make_tableau(c);
    double* u2 = zalloc(len);
    double* L = zalloc(len);
    mhd_work W;
    mhd_work_alloc(&W, c);
    for (int l = 0; l < t.nstage; ++l) {
        for (long e = 0; e < len; ++e) u2[e] = u2[e] + t.delta[l] * state[e];
        mhd_rhs(c, t.recon[l], &W, state, L);
        double bdt = t.beta[l] * dt;
        for (long e = 0; e < len; ++e)
            state[e] = (t.g0[l] * state[e] + t.g1[l] * u2[e]) + bdt * L[e];
    }
    mhd_work_free(&W);
    free(u2);
    free(L);
}

int orc_step(const orc_cfg* c, double* state, double dt)
{
    if (c->eos == ORC_EOS_ADIABATIC_MHD) {
        if (c->integ == ORC_INT_IMEX2P) return -1;
        explicit_mhd_step(c, state, dt);
        return 0;
    }
    if (c->integ != ORC_INT_IMEX2P || c->ndust < 1 || c->ndust > ORC_MAX_DUST) return -1;
    imex2p_step(c, state, dt);
    return 0;
}

/* ------------------------------------------------------------------------------ */
/* time step, eq. (cfl), and diagnostics                                            */
/* ------------------------------------------------------------------------------ */

double orc_dt_cfl(const orc_cfg* c, const double* state)
{
    long nc = (long)c->nx * c->ny * c->nz;
    const double dxs[3] = {c->dx, c->dy, c->dz};
    double cmax = 1.0;
    if (c->integ == ORC_INT_IMEX2P) cmax = 1.0 / (1.0 + 1.0 / sqrt(2.0));
    double best = INFINITY;
    int bad = 0;
    for (int k = 0; k < c->nz; ++k)
        for (int j = 0; j < c->ny; ++j)
            for (int i = 0; i < c->nx; ++i) {
                long ci = ((long)k * c->ny + j) * c->nx + i;
                if (c->eos == ORC_EOS_ADIABATIC_MHD) {
                    const double* f1 = state + 5 * nc;
                    const double* f2 = state + 6 * nc;
                    const double* f3 = state + 7 * nc;
                    double bx = 0.5 * (f1[ci] + f1[((long)k * c->ny + j) * c->nx + wrap(i + 1, c->nx)]);
                    double by = 0.5 * (f2[ci] + f2[((long)k * c->ny + wrap(j + 1, c->ny)) * c->nx + i]);
                    double bz = 0.5 * (f3[ci] + f3[((long)wrap(k + 1, c->nz) * c->ny + j) * c->nx + i]);
                    double rho = state[ci];
                    if (rho < c->rho_floor) rho = c->rho_floor;
                    double v[3] = {state[nc + ci] / rho, state[2 * nc + ci] / rho, state[3 * nc + ci] / rho};
                    double ke = 0.5 * rho * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
                    double me = 0.5 * ((bx * bx + by * by) + bz * bz);
                    double p = (c->gamma - 1.0) * ((state[4 * nc + ci] - ke) - me);
                    if (p < c->p_floor) p = c->p_floor;
                    double b2 = (bx * bx + by * by) + bz * bz;
                    double bd[3] = {bx, by, bz};
                    for (int d = 0; d < 3; ++d) {
                        double cf = fast_speed(c->gamma, rho, p, b2, bd[d]);
                        double r = dxs[d] / (fabs(v[d]) + cf);
                        if (!(r == r)) bad = 1;
                        if (r < best) best = r;
                    }
                } else {
                    for (int s = 0; s <= c->ndust; ++s) {
                        double w[4];
                        const double* base = state + 4 * s * nc;
                        fluid_prims(c, s, &base[ci], &base[nc + ci], &base[2 * nc + ci], &base[3 * nc + ci], w);
                        double cs = s == 0 ? c->cs : 0.0;
                        for (int d = 0; d < 3; ++d) {
                            double r = dxs[d] / (fabs(w[1 + d]) + cs);
                            if (!(r == r)) bad = 1;
                            if (r < best) best = r;
                        }
                    }
                }
            }
    if (bad) return NAN;
    return c->courant * cmax * best;
}

int orc_diagnostics(const orc_cfg* c, const double* state, double* out)
{
    long nc = (long)c->nx * c->ny * c->nz;
    double dV = c->dx * c->dy * c->dz;
    int nout = 9 + c->ndust + 3;
    for (int q = 0; q < nout; ++q) out[q] = 0.0;
    if (c->eos == ORC_EOS_ADIABATIC_MHD) {
        for (int q = 0; q < 5; ++q) {
            double s = 0.0;
            for (long e = 0; e < nc; ++e) s += state[q * nc + e];
            out[q] = s * dV;
        }
        for (int q = 0; q < 3; ++q) {
            double s = 0.0;
            for (long e = 0; e < nc; ++e) s += state[(5 + q) * nc + e];
            out[5 + q] = s * dV;
        }
        const double* b1 = state + 5 * nc;
        const double* b2 = state + 6 * nc;
        const double* b3 = state + 7 * nc;
        double mx = 0.0;
        for (int k = 0; k < c->nz; ++k)
            for (int j = 0; j < c->ny; ++j)
                for (int i = 0; i < c->nx; ++i) {
                    long ci = ((long)k * c->ny + j) * c->nx + i;
                    double dv = (b1[((long)k * c->ny + j) * c->nx + wrap(i + 1, c->nx)] - b1[ci]) / c->dx +
                                (b2[((long)k * c->ny + wrap(j + 1, c->ny)) * c->nx + i] - b2[ci]) / c->dy +
                                (b3[((long)wrap(k + 1, c->nz) * c->ny + j) * c->nx + i] - b3[ci]) / c->dz;
                    if (fabs(dv) > mx) mx = fabs(dv);
                }
        out[8] = mx;
        for (int a = 0; a < 3; ++a) out[9 + c->ndust + a] = out[1 + a];
    } else {
        for (int q = 0; q < 4; ++q) {
            double s = 0.0;
            for (long e = 0; e < nc; ++e) s += state[q * nc + e];
            out[q] = s * dV;
        }
        for (int a = 0; a < 3; ++a) out[9 + c->ndust + a] = out[1 + a];
        for (int s = 1; s <= c->ndust; ++s) {
            double m = 0.0;
            for (long e = 0; e < nc; ++e) m += state[4 * s * nc + e];
            out[9 + s - 1] = m * dV;
            for (int a = 0; a < 3; ++a) {
                double pm = 0.0;
                for (long e = 0; e < nc; ++e) pm += state[(4 * s + 1 + a) * nc + e];
                out[9 + c->ndust + a] += pm * dV;
            }
        }
    }
    return nout;
}
