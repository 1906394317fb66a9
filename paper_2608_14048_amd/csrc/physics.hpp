// physics.hpp -- device functions of the Godunov step: closures, reconstruction and
// face-frame Riemann solvers (Aether.jl paper, Sec. "Newtonian Magnetohydrodynamics",
// Sec. "Multifluid Dust", Sec. "Reconstruction and Riemann Solvers").
//
// Face frame: for a sweep along direction d the frame is (n, t1, t2) = (d, d+1, d+2)
// cyclic, so it stays right handed.  A face-frame MHD state is
// (rho, v_n, v_t1, v_t2, p, B_t1, B_t2) with the normal field B_n taken from the face.
#pragma once

#include <hip/hip_runtime.h>

namespace mhd {

struct Prim7 {
    double d, vn, vt1, vt2, p, bt1, bt2;
};
struct Flux7 {
    double d, mn, mt1, mt2, e, bt1, bt2;
};
struct Prim4 {
    double d, vn, vt1, vt2;
};
struct Flux4 {
    double d, mn, mt1, mt2;
};

// ----------------------------------------------------------------------------------
// reconstruction of one scalar on the face between cells s[2] and s[3]
// ----------------------------------------------------------------------------------

// van Leer's monotonized harmonic mean of the one-sided differences.
__device__ __forceinline__ double slope_vl(double am, double a0, double ap)
{
    const double dm = a0 - am, dp = ap - a0;
    const double pr = dm * dp;
    return pr > 0.0 ? 2.0 * pr / (dm + dp) : 0.0;
}

// Colella-Woodward limited central slope of the middle cell.
__device__ __forceinline__ double cw_slope(double am, double a0, double ap)
{
    const double dm = a0 - am, dp = ap - a0;
    if (!(dm * dp > 0.0)) return 0.0;
    const double c = 0.5 * (ap - am);
    const double lim = fmin(fabs(c), fmin(2.0 * fabs(dm), 2.0 * fabs(dp)));
    return c > 0.0 ? lim : -lim;
}

// Colella-Woodward monotonisation of a parabola (centre a, edges lo, hi).
__device__ __forceinline__ void cw_limit(double a, double& lo, double& hi)
{
    if ((hi - a) * (a - lo) <= 0.0) {
        lo = a;
        hi = a;
        return;
    }
    const double da = hi - lo;
    const double a6 = 6.0 * (a - 0.5 * (lo + hi));
    const double da2 = da * da;
    if (da * a6 > da2)
        lo = 3.0 * a - 2.0 * hi;
    else if (-da2 > da * a6)
        hi = 3.0 * a - 2.0 * lo;
}

template <int RECON>
__device__ __forceinline__ void face_states(const double* s, double& aL, double& aR);

template <>
__device__ __forceinline__ void face_states<0>(const double* s, double& aL, double& aR)
{
    aL = s[2];
    aR = s[3];
}

template <>
__device__ __forceinline__ void face_states<1>(const double* s, double& aL, double& aR)
{
    aL = s[2] + 0.5 * slope_vl(s[1], s[2], s[3]);
    aR = s[3] - 0.5 * slope_vl(s[2], s[3], s[4]);
}

// Colella-Woodward interface value between cells a0 and a1 from their limited slopes
// (the fourth-order average, monotonised through the slopes).
__device__ __forceinline__ double cw_interface(double a0, double a1, double m0, double m1)
{
    constexpr double kSixth = 1.0 / 6.0;
    return a0 + 0.5 * (a1 - a0) - (m1 - m0) * kSixth;
}

// PPM: the three interface values around the two cells next to the face are shared.
template <>
__device__ __forceinline__ void face_states<2>(const double* s, double& aL, double& aR)
{
    const double m1 = cw_slope(s[0], s[1], s[2]);
    const double m2 = cw_slope(s[1], s[2], s[3]);
    const double m3 = cw_slope(s[2], s[3], s[4]);
    const double m4 = cw_slope(s[3], s[4], s[5]);
    const double i0 = cw_interface(s[1], s[2], m1, m2);  // a_{f-3/2}
    const double i1 = cw_interface(s[2], s[3], m2, m3);  // a_{f-1/2}
    const double i2 = cw_interface(s[3], s[4], m3, m4);  // a_{f+1/2}
    double lo = i0, hi = i1;
    cw_limit(s[2], lo, hi);
    aL = hi;
    lo = i1;
    hi = i2;
    cw_limit(s[3], lo, hi);
    aR = lo;
}

// ----------------------------------------------------------------------------------
// adiabatic MHD in the face frame
// ----------------------------------------------------------------------------------

// Fast magnetosonic speed along a direction with field component bd; b2 = |B|^2.
__device__ __forceinline__ double fast_speed(double gam, double d, double p, double b2, double bd)
{
    const double id = 1.0 / d;
    const double a2 = gam * p * id;
    const double s = a2 + b2 * id;
    const double disc = fmax(s * s - 4.0 * a2 * (bd * bd) * id, 0.0);
    return sqrt(0.5 * (s + sqrt(disc)));
}

// Conserved vector, physical flux and total pressure of one face-frame state.
struct Side {
    double U[7];
    double F[7];
    double pt, vb, cf;
};

__device__ __forceinline__ void side_of(const Prim7& w, double bn, double gam, double gm1inv,
                                        Side& s)
{
    const double bt2 = w.bt1 * w.bt1 + w.bt2 * w.bt2;
    const double b2 = bn * bn + bt2;
    const double v2 = w.vn * w.vn + (w.vt1 * w.vt1 + w.vt2 * w.vt2);
    const double pt = w.p + 0.5 * b2;
    const double E = w.p * gm1inv + 0.5 * w.d * v2 + 0.5 * b2;
    const double vb = w.vn * bn + (w.vt1 * w.bt1 + w.vt2 * w.bt2);
    const double mn = w.d * w.vn;
    s.U[0] = w.d;
    s.U[1] = mn;
    s.U[2] = w.d * w.vt1;
    s.U[3] = w.d * w.vt2;
    s.U[4] = E;
    s.U[5] = w.bt1;
    s.U[6] = w.bt2;
    s.F[0] = mn;
    s.F[1] = mn * w.vn + pt - bn * bn;
    s.F[2] = mn * w.vt1 - bn * w.bt1;
    s.F[3] = mn * w.vt2 - bn * w.bt2;
    s.F[4] = (E + pt) * w.vn - bn * vb;
    s.F[5] = w.bt1 * w.vn - bn * w.vt1;
    s.F[6] = w.bt2 * w.vn - bn * w.vt2;
    s.pt = pt;
    s.vb = vb;
    s.cf = fast_speed(gam, w.d, w.p, b2, bn);
}

__device__ __forceinline__ void to_flux(const double* a, Flux7& f)
{
    f.d = a[0]; f.mn = a[1]; f.mt1 = a[2]; f.mt2 = a[3]; f.e = a[4]; f.bt1 = a[5]; f.bt2 = a[6];
}

// HLLE with the outer bounds S_L = min(u) - max(c_f), S_R = max(u) + max(c_f).
__device__ __forceinline__ void riemann_hlle(const Prim7& L, const Prim7& R, double bn,
                                             double gam, double gm1inv, Flux7& f)
{
    Side a, b;
    side_of(L, bn, gam, gm1inv, a);
    side_of(R, bn, gam, gm1inv, b);
    const double cmax = fmax(a.cf, b.cf);
    const double sl = fmin(L.vn, R.vn) - cmax;
    const double sr = fmax(L.vn, R.vn) + cmax;
    const double bm = fmin(sl, 0.0), bp = fmax(sr, 0.0);
    const double inv = 1.0 / (bp - bm);
    double o[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) o[q] = (bp * a.F[q] - bm * b.F[q] + bp * bm * (b.U[q] - a.U[q])) * inv;
    to_flux(o, f);
}

// One side of the HLLD star region: density behind the fast wave, transverse velocity
// and field from the jump conditions (kept at their outer values where the
// denominator degenerates), and the energy from the energy jump condition.
struct Star {
    double d, vt1, vt2, bt1, bt2, e, vb, sqd;
};

__device__ __forceinline__ void star_of(const Prim7& w, const Side& s, double bn, double S,
                                        double SM, double pts, double eps, Star& o)
{
    const double du = S - w.vn;
    const double ds = 1.0 / (S - SM);
    o.d = w.d * du * ds;
    const double den = w.d * du * (S - SM) - bn * bn;
    if (fabs(den) <= eps * pts) {
        o.vt1 = w.vt1; o.vt2 = w.vt2; o.bt1 = w.bt1; o.bt2 = w.bt2;
    } else {
        const double r = 1.0 / den;
        const double cv = bn * (SM - w.vn) * r;
        const double cb = (w.d * du * du - bn * bn) * r;
        o.vt1 = w.vt1 - w.bt1 * cv;
        o.vt2 = w.vt2 - w.bt2 * cv;
        o.bt1 = w.bt1 * cb;
        o.bt2 = w.bt2 * cb;
    }
    o.vb = SM * bn + (o.vt1 * o.bt1 + o.vt2 * o.bt2);
    o.e = (du * s.U[4] - s.pt * w.vn + pts * SM + bn * (s.vb - o.vb)) * ds;
    o.sqd = sqrt(o.d);
}

// Miyoshi & Kusano (2005) five-wave HLLD flux.
__device__ __forceinline__ void riemann_hlld(const Prim7& L, const Prim7& R, double bn,
                                             double gam, double gm1inv, double eps, Flux7& f)
{
    Side a, b;
    side_of(L, bn, gam, gm1inv, a);
    side_of(R, bn, gam, gm1inv, b);
    const double cmax = fmax(a.cf, b.cf);
    const double sl = fmin(L.vn, R.vn) - cmax;
    const double sr = fmax(L.vn, R.vn) + cmax;
    if (sl > 0.0) { to_flux(a.F, f); return; }
    if (sr < 0.0) { to_flux(b.F, f); return; }

    const double ml = L.d * (sl - L.vn), mr = R.d * (sr - R.vn);  // mass fluxes into the fan
    const double iden = 1.0 / (mr - ml);
    const double SM = (mr * R.vn - ml * L.vn - b.pt + a.pt) * iden;
    const double pts = (mr * a.pt - ml * b.pt + ml * mr * (R.vn - L.vn)) * iden;

    Star x, y;
    star_of(L, a, bn, sl, SM, pts, eps, x);
    star_of(R, b, bn, sr, SM, pts, eps, y);
    const double slst = SM - fabs(bn) / x.sqd;
    const double srst = SM + fabs(bn) / y.sqd;

    // U* on each side
    double ul[7] = {x.d, x.d * SM, x.d * x.vt1, x.d * x.vt2, x.e, x.bt1, x.bt2};
    double ur[7] = {y.d, y.d * SM, y.d * y.vt1, y.d * y.vt2, y.e, y.bt1, y.bt2};
    double o[7];
    if (slst >= 0.0) {
#pragma unroll
        for (int q = 0; q < 7; ++q) o[q] = a.F[q] + sl * (ul[q] - a.U[q]);
        to_flux(o, f);
        return;
    }
    if (srst < 0.0) {
#pragma unroll
        for (int q = 0; q < 7; ++q) o[q] = b.F[q] + sr * (ur[q] - b.U[q]);
        to_flux(o, f);
        return;
    }
    // between the two Alfven waves
    const bool left = SM >= 0.0;
    const Star& st = left ? x : y;
    const double* us = left ? ul : ur;
    const double S = left ? sl : sr;
    const double Sst = left ? slst : srst;
    const Side& sd = left ? a : b;
    double uss[7];
    if (bn * bn <= eps * pts) {
#pragma unroll
        for (int q = 0; q < 7; ++q) uss[q] = us[q];
    } else {
        const double sg = bn > 0.0 ? 1.0 : -1.0;
        const double inv = 1.0 / (x.sqd + y.sqd);
        const double v1 = (x.sqd * x.vt1 + y.sqd * y.vt1 + (y.bt1 - x.bt1) * sg) * inv;
        const double v2 = (x.sqd * x.vt2 + y.sqd * y.vt2 + (y.bt2 - x.bt2) * sg) * inv;
        const double b1 = (x.sqd * y.bt1 + y.sqd * x.bt1 + x.sqd * y.sqd * (y.vt1 - x.vt1) * sg) * inv;
        const double b2 = (x.sqd * y.bt2 + y.sqd * x.bt2 + x.sqd * y.sqd * (y.vt2 - x.vt2) * sg) * inv;
        const double vbss = SM * bn + (v1 * b1 + v2 * b2);
        const double ess = left ? x.e - x.sqd * (x.vb - vbss) * sg : y.e + y.sqd * (y.vb - vbss) * sg;
        uss[0] = st.d; uss[1] = st.d * SM; uss[2] = st.d * v1; uss[3] = st.d * v2;
        uss[4] = ess; uss[5] = b1; uss[6] = b2;
    }
#pragma unroll
    for (int q = 0; q < 7; ++q) o[q] = sd.F[q] + S * (us[q] - sd.U[q]) + Sst * (uss[q] - us[q]);
    to_flux(o, f);
}

// ----------------------------------------------------------------------------------
// isothermal gas and pressureless dust
// ----------------------------------------------------------------------------------

__device__ __forceinline__ void riemann_iso_hlle(const Prim4& L, const Prim4& R, double cs,
                                                 Flux4& f)
{
    const double sl = fmin(L.vn, R.vn) - cs, sr = fmax(L.vn, R.vn) + cs;
    const double bm = fmin(sl, 0.0), bp = fmax(sr, 0.0);
    const double inv = 1.0 / (bp - bm);
    const double c2 = cs * cs;
    const double mL = L.d * L.vn, mR = R.d * R.vn;
    const double UL[4] = {L.d, mL, L.d * L.vt1, L.d * L.vt2};
    const double UR[4] = {R.d, mR, R.d * R.vt1, R.d * R.vt2};
    const double FL[4] = {mL, mL * L.vn + c2 * L.d, mL * L.vt1, mL * L.vt2};
    const double FR[4] = {mR, mR * R.vn + c2 * R.d, mR * R.vt1, mR * R.vt2};
    double o[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = (bp * FL[q] - bm * FR[q] + bp * bm * (UR[q] - UL[q])) * inv;
    f.d = o[0]; f.mn = o[1]; f.mt1 = o[2]; f.mt2 = o[3];
}

// Pressureless Rusanov: central average minus max(|u_L|,|u_R|)/2 times the jump.
__device__ __forceinline__ void riemann_dust(const Prim4& L, const Prim4& R, Flux4& f)
{
    const double a = fmax(fabs(L.vn), fabs(R.vn));
    const double UL[4] = {L.d, L.d * L.vn, L.d * L.vt1, L.d * L.vt2};
    const double UR[4] = {R.d, R.d * R.vn, R.d * R.vt1, R.d * R.vt2};
    double o[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = 0.5 * (L.vn * UL[q] + R.vn * UR[q]) - 0.5 * a * (UR[q] - UL[q]);
    f.d = o[0]; f.mn = o[1]; f.mt1 = o[2]; f.mt2 = o[3];
}

}  // namespace mhd
