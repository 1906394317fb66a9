// physics.hpp -- device functions of the Godunov step: closures, reconstruction and
// face-frame Riemann solvers (Aether.jl paper, Sec. "Newtonian Magnetohydrodynamics",
// Sec. "Multifluid Dust", Sec. "Reconstruction and Riemann Solvers").
//
// Face frame: for a sweep along direction d the frame is (n, t1, t2) = (d, d+1, d+2)
// cyclic, so it stays right handed.  A face-frame MHD state is
// (rho, v_n, v_t1, v_t2, p, B_t1, B_t2) with the normal field B_n taken from the face.
//
// Every function is templated on the real type R: double for the FP64 path, float for
// the FP32-bulk path (where reciprocals and square roots use the single-instruction
// hardware approximations; FP64 refines the hardware estimates to within about an ulp
// of the IEEE results).
#pragma once

#include <hip/hip_runtime.h>

namespace mhd {

template <class R>
struct Prim7 {
    R d, vn, vt1, vt2, p, bt1, bt2;
};
template <class R>
struct Flux7 {
    R d, mn, mt1, mt2, e, bt1, bt2;
};
template <class R>
struct Prim4 {
    R d, vn, vt1, vt2;
};
template <class R>
struct Flux4 {
    R d, mn, mt1, mt2;
};

// ----------------------------------------------------------------------------------
// scalar helpers per precision
// ----------------------------------------------------------------------------------

// FP64 1/x for finite, normal x != 0: the hardware estimate refined by two
// Newton-Raphson steps r <- r + r (1 - x r), each squaring the relative error.
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
    return __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// FP64 square root of a finite x >= 0: Goldschmidt's coupled iteration on the hardware
// estimate y of 1/sqrt(x) (g = x y -> sqrt(x), h = y/2 -> 1/(2 sqrt(x))), then one
// correction with the exact residual x - g^2.  x = 0 gives 0; x < 0 gives NaN.
__device__ __forceinline__ double sqrt_r(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double t = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, t, g);
    h = __builtin_fma(h, t, h);
    g = __builtin_fma(__builtin_fma(-g, g, x), h, g);
    return x == 0.0 ? 0.0 : g;
}
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double abs_r(double x) { return fabs(x); }
__device__ __forceinline__ float abs_r(float x) { return fabsf(x); }
__device__ __forceinline__ double min_r(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float min_r(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double max_r(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float max_r(float a, float b) { return fmaxf(a, b); }
// a * b + c with one rounding (written out where a formula wants it, so that the
// rounding of a helper does not depend on where the compiler inlines it)
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// a / b for finite, normal b != 0.  FP64: the hardware reciprocal refined by one
// Newton-Raphson step, then one correction of the quotient with the exact residual
// a - b q (Markstein's scheme); FP32: a times the hardware reciprocal.
__device__ __forceinline__ double div_r(double a, double b)
{
    double r = __builtin_amdgcn_rcp(b);
    r = __builtin_fma(__builtin_fma(-b, r, 1.0), r, r);
    const double q = a * r;
    return __builtin_fma(__builtin_fma(-b, q, a), r, q);
}
__device__ __forceinline__ float div_r(float a, float b) { return a * rcp(b); }

// ----------------------------------------------------------------------------------
// reconstruction of one scalar on the face between cells s[2] and s[3]
// ----------------------------------------------------------------------------------

// The reconstruction helpers keep every rounding explicit (no contraction left to the
// compiler): a z pipeline primed at the start of a chunk then reproduces bit for bit
// the values it would carry from the plane before, so results do not depend on how the
// z planes are split among workgroups.

// van Leer's monotonized harmonic mean of the one-sided differences.
template <class R>
__device__ __forceinline__ R slope_vl(R am, R a0, R ap)
{
#pragma clang fp contract(off)
    const R dm = a0 - am, dp = ap - a0;
    const R pr = dm * dp;
    return pr > R(0) ? div_r(R(2) * pr, dm + dp) : R(0);
}

// Colella-Woodward limited central slope of the middle cell.
template <class R>
__device__ __forceinline__ R cw_slope(R am, R a0, R ap)
{
#pragma clang fp contract(off)
    const R dm = a0 - am, dp = ap - a0;
    if (!(dm * dp > R(0))) return R(0);
    const R c = R(0.5) * (ap - am);
    if constexpr (sizeof(R) == 8) {
        // dm and dp share a sign here, so c = (dm + dp)/2 is nonzero and carries it; the
        // doubling is exact, so 2 min(|dm|, |dp|) = min(2|dm|, 2|dp|) bit for bit (the
        // same values in fewer FP64 instructions; FP32 compiles shorter the other way)
        const R lim = min_r(abs_r(c), R(2) * min_r(abs_r(dm), abs_r(dp)));
        return __builtin_copysign(lim, c);
    } else {
        const R lim = min_r(abs_r(c), min_r(R(2) * abs_r(dm), R(2) * abs_r(dp)));
        return c > R(0) ? lim : -lim;
    }
}

// Colella-Woodward interface value between cells a0 and a1 from their limited slopes
// (the fourth-order average, monotonised through the slopes):
// a0 + (a1 - a0)/2 - (m1 - m0)/6.
template <class R>
__device__ __forceinline__ R cw_interface(R a0, R a1, R m0, R m1)
{
#pragma clang fp contract(off)
    const R t = fma_r(R(0.5), a1 - a0, a0);
    return fma_r(m0 - m1, R(1.0 / 6.0), t);
}

// Colella-Woodward monotonisation of a parabola (centre a, edges lo, hi).
template <class R>
__device__ __forceinline__ void cw_limit(R a, R& lo, R& hi)
{
#pragma clang fp contract(off)
    if ((hi - a) * (a - lo) <= R(0)) {
        lo = a;
        hi = a;
        return;
    }
    const R da = hi - lo;
    const R a6 = R(6) * fma_r(R(-0.5), lo + hi, a);
    const R da2 = da * da;
    const R p = da * a6;
    if (p > da2)
        lo = fma_r(R(-2), hi, R(3) * a);
    else if (-da2 > p)
        hi = fma_r(R(-2), lo, R(3) * a);
}

template <int RECON, class R>
struct FaceStates;

template <class R>
struct FaceStates<0, R> {
    __device__ static void get(const R* s, R& aL, R& aR)
    {
        aL = s[2];
        aR = s[3];
    }
};

template <class R>
struct FaceStates<1, R> {
    __device__ static void get(const R* s, R& aL, R& aR)
    {
        aL = fma_r(R(0.5), slope_vl(s[1], s[2], s[3]), s[2]);
        aR = fma_r(R(-0.5), slope_vl(s[2], s[3], s[4]), s[3]);
    }
};

// PPM: the three interface values around the two cells next to the face are shared.
template <class R>
struct FaceStates<2, R> {
    __device__ static void get(const R* s, R& aL, R& aR)
    {
        const R m1 = cw_slope(s[0], s[1], s[2]);
        const R m2 = cw_slope(s[1], s[2], s[3]);
        const R m3 = cw_slope(s[2], s[3], s[4]);
        const R m4 = cw_slope(s[3], s[4], s[5]);
        const R i0 = cw_interface(s[1], s[2], m1, m2);  // a_{f-3/2}
        const R i1 = cw_interface(s[2], s[3], m2, m3);  // a_{f-1/2}
        const R i2 = cw_interface(s[3], s[4], m3, m4);  // a_{f+1/2}
        R lo = i0, hi = i1;
        cw_limit(s[2], lo, hi);
        aL = hi;
        lo = i1;
        hi = i2;
        cw_limit(s[3], lo, hi);
        aR = lo;
    }
};

// Face states of the six cells s[0..5] around the face between s[2] and s[3].
template <int RECON, class R>
__device__ __forceinline__ void face_states(const R* s, R& aL, R& aR)
{
    FaceStates<RECON, R>::get(s, aL, aR);
}

// ----------------------------------------------------------------------------------
// adiabatic MHD in the face frame
// ----------------------------------------------------------------------------------

// a1 b1 + a2 b2 over the two transverse components, rounded as written (no FMA): the
// sum of two rounded products does not depend on which transverse direction is called
// t1, so an x face and a y face that are images of each other under the swap of x and
// y (their transverse pairs come in opposite orders) give the same bits.
template <class R>
__device__ __forceinline__ R tsum(R a1, R b1, R a2, R b2)
{
#pragma clang fp contract(off)
    return a1 * b1 + a2 * b2;
}

// The Riemann solvers below round every operation as written: each product that is
// fused into an add is an explicit fma_r, nothing is left to the compiler's
// contraction.  A face then gives the same bits wherever the solver is inlined (the
// cell's own faces, the tile's high faces, the z face that opens a chunk), so results
// do not depend on how the grid is tiled or split into z chunks.

// Fast magnetosonic speed along a direction with field component bd; b2 = |B|^2.
template <class R>
__device__ __forceinline__ R fast_speed(R gam, R d, R p, R b2, R bd)
{
#pragma clang fp contract(off)
    const R id = rcp(d);
    const R a2 = gam * p * id;
    const R s = fma_r(b2, id, a2);
    const R disc = max_r(fma_r(s, s, -(R(4) * a2 * (bd * bd) * id)), R(0));
    return sqrt_r(R(0.5) * (s + sqrt_r(disc)));
}

// Conserved vector, physical flux and total pressure of one face-frame state.
template <class R>
struct Side {
    R U[7];
    R F[7];
    R pt, vb, cf;
};

// What the HLLD wave speeds and star states need of one face-frame state: total
// pressure, v.B, total energy and the fast speed (the conserved vector and the flux are
// built later for the one side the face's region needs).
template <class R>
struct Lite {
    R pt, vb, e, cf;
};

template <class R>
__device__ __forceinline__ void lite_of(const Prim7<R>& w, R bn, R gam, R gm1inv, Lite<R>& s)
{
#pragma clang fp contract(off)
    const R bt2 = tsum(w.bt1, w.bt1, w.bt2, w.bt2);
    const R b2 = fma_r(bn, bn, bt2);
    const R v2 = fma_r(w.vn, w.vn, tsum(w.vt1, w.vt1, w.vt2, w.vt2));
    s.pt = fma_r(R(0.5), b2, w.p);
    s.e = fma_r(w.p, gm1inv, fma_r(R(0.5) * w.d, v2, R(0.5) * b2));
    s.vb = fma_r(w.vn, bn, tsum(w.vt1, w.bt1, w.vt2, w.bt2));
    s.cf = fast_speed(gam, w.d, w.p, b2, bn);
}

// Conserved vector and physical flux of one state.
template <class R>
__device__ __forceinline__ void uf_of(const Prim7<R>& w, const Lite<R>& s, R bn, R U[7], R F[7])
{
#pragma clang fp contract(off)
    const R mn = w.d * w.vn;
    U[0] = w.d;
    U[1] = mn;
    U[2] = w.d * w.vt1;
    U[3] = w.d * w.vt2;
    U[4] = s.e;
    U[5] = w.bt1;
    U[6] = w.bt2;
    F[0] = mn;
    F[1] = fma_r(-bn, bn, fma_r(mn, w.vn, s.pt));
    F[2] = fma_r(mn, w.vt1, -(bn * w.bt1));
    F[3] = fma_r(mn, w.vt2, -(bn * w.bt2));
    F[4] = fma_r(s.e + s.pt, w.vn, -(bn * s.vb));
    F[5] = fma_r(w.bt1, w.vn, -(bn * w.vt1));
    F[6] = fma_r(w.bt2, w.vn, -(bn * w.vt2));
}

template <class R>
__device__ __forceinline__ void side_of(const Prim7<R>& w, R bn, R gam, R gm1inv, Side<R>& s)
{
    Lite<R> l;
    lite_of(w, bn, gam, gm1inv, l);
    uf_of(w, l, bn, s.U, s.F);
    s.pt = l.pt;
    s.vb = l.vb;
    s.cf = l.cf;
}

template <class R>
__device__ __forceinline__ void to_flux(const R* a, Flux7<R>& f)
{
    f.d = a[0]; f.mn = a[1]; f.mt1 = a[2]; f.mt2 = a[3]; f.e = a[4]; f.bt1 = a[5]; f.bt2 = a[6];
}

// HLLE with the outer bounds S_L = min(u) - max(c_f), S_R = max(u) + max(c_f).
template <class R>
__device__ __forceinline__ void riemann_hlle(const Prim7<R>& L, const Prim7<R>& Rt, R bn, R gam,
                                             R gm1inv, Flux7<R>& f)
{
#pragma clang fp contract(off)
    Side<R> a, b;
    side_of(L, bn, gam, gm1inv, a);
    side_of(Rt, bn, gam, gm1inv, b);
    const R cmax = max_r(a.cf, b.cf);
    const R sl = min_r(L.vn, Rt.vn) - cmax;
    const R sr = max_r(L.vn, Rt.vn) + cmax;
    const R bm = min_r(sl, R(0)), bp = max_r(sr, R(0));
    const R inv = rcp(bp - bm);
    const R bpm = bp * bm;
    R o[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) o[q] = fma_r(bpm, b.U[q] - a.U[q], fma_r(bp, a.F[q], -(bm * b.F[q]))) * inv;
    to_flux(o, f);
}

// One side of the HLLD star region: density behind the fast wave, transverse velocity
// and field from the jump conditions (kept at their outer values where the
// denominator degenerates), and the energy from the energy jump condition.
template <class R>
struct Star {
    R d, vt1, vt2, bt1, bt2, e, vb, sqd;
};

template <class R>
__device__ __forceinline__ void star_of(const Prim7<R>& w, const Lite<R>& s, R bn, R S, R SM, R pts,
                                        R eps, Star<R>& o)
{
#pragma clang fp contract(off)
    const R du = S - w.vn;
    const R dsm = S - SM;
    const R ds = rcp(dsm);
    const R mdu = w.d * du;
    o.d = mdu * ds;
    const R bn2 = bn * bn;
    const R den = fma_r(mdu, dsm, -bn2);
    if (abs_r(den) <= eps * pts) {
        o.vt1 = w.vt1; o.vt2 = w.vt2; o.bt1 = w.bt1; o.bt2 = w.bt2;
    } else {
        const R r = rcp(den);
        const R cv = bn * (SM - w.vn) * r;
        const R cb = fma_r(mdu, du, -bn2) * r;
        o.vt1 = fma_r(-w.bt1, cv, w.vt1);
        o.vt2 = fma_r(-w.bt2, cv, w.vt2);
        o.bt1 = w.bt1 * cb;
        o.bt2 = w.bt2 * cb;
    }
    o.vb = fma_r(SM, bn, tsum(o.vt1, o.bt1, o.vt2, o.bt2));
    o.e = fma_r(du, s.e, fma_r(-s.pt, w.vn, fma_r(pts, SM, bn * (s.vb - o.vb)))) * ds;
    o.sqd = sqrt_r(o.d);
}

// Miyoshi & Kusano (2005) five-wave HLLD flux.  Every region's flux has the form
// F(W) + S (U_a - U(W)) + S_a (U_b - U_a) for one outer state W: F(W) in the
// supersonic regions (S = S_a = 0), F(W) + S (U* - U(W)) in the outer star regions,
// and the full form between the Alfven waves, W on the side of the contact.  The
// conserved vector and flux are built once, for that W.
template <class R>
__device__ __forceinline__ void riemann_hlld(const Prim7<R>& L, const Prim7<R>& Rt, R bn, R gam,
                                             R gm1inv, R eps, Flux7<R>& f)
{
#pragma clang fp contract(off)
    Lite<R> a, b;
    lite_of(L, bn, gam, gm1inv, a);
    lite_of(Rt, bn, gam, gm1inv, b);
    const R cmax = max_r(a.cf, b.cf);
    const R sl = min_r(L.vn, Rt.vn) - cmax;
    const R sr = max_r(L.vn, Rt.vn) + cmax;

    const bool sup = sl > R(0) || sr < R(0);
    bool useL = sl > R(0);
    R S = R(0), Sa = R(0);
    R ua[7], ub[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) ua[q] = ub[q] = R(0);
    if (!sup) {
        const R ml = L.d * (sl - L.vn), mr = Rt.d * (sr - Rt.vn);  // mass fluxes into the fan
        const R iden = rcp(mr - ml);
        const R SM = (fma_r(mr, Rt.vn, -(ml * L.vn)) - b.pt + a.pt) * iden;
        const R pts = fma_r(ml * mr, Rt.vn - L.vn, fma_r(mr, a.pt, -(ml * b.pt))) * iden;

        Star<R> x, y;
        star_of(L, a, bn, sl, SM, pts, eps, x);
        star_of(Rt, b, bn, sr, SM, pts, eps, y);
        const R slst = SM - div_r(abs_r(bn), x.sqd);
        const R srst = SM + div_r(abs_r(bn), y.sqd);
        const bool outerL = slst >= R(0), outerR = !outerL && srst < R(0);
        const bool left = outerL || (!outerR && SM >= R(0));
        useL = left;
        // U* of the side of W
        const Star<R>& st = left ? x : y;
        ua[0] = st.d; ua[1] = st.d * SM; ua[2] = st.d * st.vt1; ua[3] = st.d * st.vt2;
        ua[4] = st.e; ua[5] = st.bt1; ua[6] = st.bt2;
        S = left ? sl : sr;
        if (!outerL && !outerR) {
            // between the two Alfven waves: U** of the side of W
            Sa = left ? slst : srst;
            if (bn * bn <= eps * pts) {
#pragma unroll
                for (int q = 0; q < 7; ++q) ub[q] = ua[q];
            } else {
                const R sg = bn > R(0) ? R(1) : R(-1);
                const R inv = rcp(x.sqd + y.sqd);
                const R xy = x.sqd * y.sqd;
                const R v1 = fma_r(x.sqd, x.vt1, fma_r(y.sqd, y.vt1, (y.bt1 - x.bt1) * sg)) * inv;
                const R v2 = fma_r(x.sqd, x.vt2, fma_r(y.sqd, y.vt2, (y.bt2 - x.bt2) * sg)) * inv;
                const R b1 = fma_r(x.sqd, y.bt1, fma_r(y.sqd, x.bt1, xy * (y.vt1 - x.vt1) * sg)) * inv;
                const R b2 = fma_r(x.sqd, y.bt2, fma_r(y.sqd, x.bt2, xy * (y.vt2 - x.vt2) * sg)) * inv;
                const R vbss = fma_r(SM, bn, tsum(v1, b1, v2, b2));
                const R ess = left ? fma_r(-x.sqd * sg, x.vb - vbss, x.e) : fma_r(y.sqd * sg, y.vb - vbss, y.e);
                ub[0] = st.d; ub[1] = st.d * SM; ub[2] = st.d * v1; ub[3] = st.d * v2;
                ub[4] = ess; ub[5] = b1; ub[6] = b2;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 7; ++q) ub[q] = ua[q];
        }
    }
    // the outer state W and its conserved vector and flux
    const Prim7<R>& w = useL ? L : Rt;
    const Lite<R>& sw = useL ? a : b;
    R U[7], F[7];
    uf_of(w, sw, bn, U, F);
    if (sup) {
        // supersonic: F(W) exactly
#pragma unroll
        for (int q = 0; q < 7; ++q) ua[q] = ub[q] = U[q];
    }
    R o[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) o[q] = fma_r(Sa, ub[q] - ua[q], fma_r(S, ua[q] - U[q], F[q]));
    to_flux(o, f);
}

// ----------------------------------------------------------------------------------
// isothermal gas and pressureless dust
// ----------------------------------------------------------------------------------

template <class R>
__device__ __forceinline__ void riemann_iso_hlle(const Prim4<R>& L, const Prim4<R>& Rt, R cs, Flux4<R>& f)
{
#pragma clang fp contract(off)
    const R sl = min_r(L.vn, Rt.vn) - cs, sr = max_r(L.vn, Rt.vn) + cs;
    const R bm = min_r(sl, R(0)), bp = max_r(sr, R(0));
    const R inv = rcp(bp - bm);
    const R c2 = cs * cs;
    const R mL = L.d * L.vn, mR = Rt.d * Rt.vn;
    const R UL[4] = {L.d, mL, L.d * L.vt1, L.d * L.vt2};
    const R UR[4] = {Rt.d, mR, Rt.d * Rt.vt1, Rt.d * Rt.vt2};
    const R FL[4] = {mL, fma_r(mL, L.vn, c2 * L.d), mL * L.vt1, mL * L.vt2};
    const R FR[4] = {mR, fma_r(mR, Rt.vn, c2 * Rt.d), mR * Rt.vt1, mR * Rt.vt2};
    const R bpm = bp * bm;
    R o[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = fma_r(bpm, UR[q] - UL[q], fma_r(bp, FL[q], -(bm * FR[q]))) * inv;
    f.d = o[0]; f.mn = o[1]; f.mt1 = o[2]; f.mt2 = o[3];
}

// Pressureless Rusanov: central average minus max(|u_L|,|u_R|)/2 times the jump.
template <class R>
__device__ __forceinline__ void riemann_dust(const Prim4<R>& L, const Prim4<R>& Rt, Flux4<R>& f)
{
#pragma clang fp contract(off)
    const R a = max_r(abs_r(L.vn), abs_r(Rt.vn));
    const R UL[4] = {L.d, L.d * L.vn, L.d * L.vt1, L.d * L.vt2};
    const R UR[4] = {Rt.d, Rt.d * Rt.vn, Rt.d * Rt.vt1, Rt.d * Rt.vt2};
    const R ha = R(0.5) * a;
    R o[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = fma_r(-ha, UR[q] - UL[q], R(0.5) * fma_r(L.vn, UL[q], Rt.vn * UR[q]));
    f.d = o[0]; f.mn = o[1]; f.mt1 = o[2]; f.mt2 = o[3];
}

}  // namespace mhd
