/* Drives one small step of every integrator of the CPU oracle, for a build with the
 * address and undefined-behaviour sanitizers (tests/test_oracle_sanitized.py).  The
 * states are simple closed-form fields: no external input. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.h"

static orc_cfg base_cfg(int nx, int ny, int nz)
{
    orc_cfg c;
    memset(&c, 0, sizeof c);
    c.nx = nx; c.ny = ny; c.nz = nz;
    c.dx = 1.0 / nx; c.dy = 1.0 / ny; c.dz = 1.0 / nz;
    c.gamma = 5.0 / 3.0; c.cs = 1.0;
    c.rho_floor = 1e-12; c.p_floor = 1e-10; c.dust_rho_floor = 1e-12;
    c.courant = 0.3; c.hlld_eps = 1e-12;
    return c;
}

static int run_mhd(int recon, int riemann, int integ)
{
    orc_cfg c = base_cfg(8, 6, 5);
    c.eos = ORC_EOS_ADIABATIC_MHD;
    c.recon = recon; c.riemann = riemann; c.integ = integ;
    long nc = (long)c.nx * c.ny * c.nz, len = orc_state_len(&c);
    double* s = (double*)calloc((size_t)len, sizeof(double));
    for (int k = 0; k < c.nz; ++k)
        for (int j = 0; j < c.ny; ++j)
            for (int i = 0; i < c.nx; ++i) {
                long q = ((long)k * c.ny + j) * c.nx + i;
                double x = (i + 0.5) / c.nx, y = (j + 0.5) / c.ny, z = (k + 0.5) / c.nz;
                double rho = 1.0 + 0.2 * sin(6.283185307179586 * x);
                double vx = 0.3 * sin(6.283185307179586 * y), vy = 0.2 * cos(6.283185307179586 * z);
                double vz = 0.1 * sin(6.283185307179586 * (x + y));
                double bx = 0.7, by = -0.4, bz = 0.3, p = 1.0;
                s[q] = rho; s[nc + q] = rho * vx; s[2 * nc + q] = rho * vy; s[3 * nc + q] = rho * vz;
                s[4 * nc + q] = p / (c.gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz) +
                                0.5 * (bx * bx + by * by + bz * bz);
                s[5 * nc + q] = bx; s[6 * nc + q] = by; s[7 * nc + q] = bz;
            }
    double dt = orc_dt_cfl(&c, s);
    int rc = orc_step(&c, s, dt);
    double d[16];
    orc_diagnostics(&c, s, d);
    int ok = rc == 0 && isfinite(dt) && isfinite(d[0]) && isfinite(d[4]);
    free(s);
    return ok ? 0 : 1;
}

static int run_dust(int recon)
{
    orc_cfg c = base_cfg(7, 5, 4);
    c.eos = ORC_EOS_ISOTHERMAL_HYDRO;
    c.recon = recon; c.riemann = ORC_RS_HLLE; c.integ = ORC_INT_IMEX2P;
    c.ndust = 3;
    c.tstop[0] = 1e-3; c.tstop[1] = 0.1; c.tstop[2] = 10.0;
    c.gacc[0] = 0.05;
    c.dust_rho_floor = 1e-3;
    long nc = (long)c.nx * c.ny * c.nz, len = orc_state_len(&c);
    double* s = (double*)calloc((size_t)len, sizeof(double));
    for (int f = 0; f <= c.ndust; ++f)
        for (long q = 0; q < nc; ++q) {
            double rho = f == 0 ? 1.0 : (q % 3 == 0 ? 5e-4 : 0.01);  /* some cells below the floor */
            s[4 * f * nc + q] = rho;
            s[(4 * f + 1) * nc + q] = rho * (0.01 * (double)((q * 7 + f) % 5) - 0.02);
            s[(4 * f + 2) * nc + q] = rho * 0.003 * f;
            s[(4 * f + 3) * nc + q] = -rho * 0.002;
        }
    double dt = orc_dt_cfl(&c, s);
    int rc = orc_step(&c, s, dt);
    double d[32];
    orc_diagnostics(&c, s, d);
    int ok = rc == 0 && isfinite(dt) && isfinite(d[0]);
    free(s);
    return ok ? 0 : 1;
}

int main(void)
{
    int bad = 0;
    bad += run_mhd(ORC_RECON_PPM, ORC_RS_HLLD, ORC_INT_VL2);
    bad += run_mhd(ORC_RECON_PLM, ORC_RS_HLLE, ORC_INT_RK2);
    bad += run_mhd(ORC_RECON_DC, ORC_RS_HLLD, ORC_INT_EULER1);
    bad += run_dust(ORC_RECON_PLM);
    bad += run_dust(ORC_RECON_DC);
    /* pieces exposed to the pins */
    double a[9] = {1, 2, 4, 3, 3, 5, 1, 0, 2}, aL[9], aR[9];
    orc_recon_line(ORC_RECON_PPM, 9, a, aL, aR);
    double rho[4] = {1.0, 0.01, 0.02, 0.03}, p[4] = {0.1, 0.2, -0.1, 0.0}, po[4];
    double ts[3] = {0.01, 0.1, 1.0};
    orc_drag_solve(3, rho, p, ts, 0.05, po);
    printf("sanitized oracle run: %s\n", bad ? "FAILED" : "ok");
    return bad ? 1 : 0;
}
