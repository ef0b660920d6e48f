// Near-field solid angle of one trimmed rational bicubic patch (host and
// device code; the host build of it is only used to test it on the CPU).
//
// The solid-angle density in parameter space g(u, v) = det[A, A_u, A_v] /
// |A|^3 (A = H - q W, weights cancel) is integrated over the visible region
// D with Green's theorem in polar form about the foot point c of q on the
// patch:
//   integral_D g = sum over boundary curves gamma of
//     integral cross(gamma - c, gamma') H(gamma) dt,
//   H(p) = integral_0^1 g(c + tau (p - c)) tau dtau,
// valid for any c in the unit square (the rays stay in the square).  The
// near-singular behaviour of g at c (width ~ dist(q, S)) sits at tau = 0 and
// is removed by tau = eps sinh(mu sigma), eps = d / L, mu = asinh(1 / eps),
// in three pieces (core, logarithmic middle, tau in [0.1, 1]).  The outer
// integrand peaks near the point of gamma closest to c and, for a strongly
// anisotropic metric J^T J at c (eigenvalues l1 < l2, e.g. next to a
// collapsed patch edge), where the ray from c runs along the weak direction
// (angular width ~ sqrt(l1 / l2)); it is split into panels graded
// geometrically from those points.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "gwn_internal.h"

#define GWN_HD __host__ __device__

namespace gwn {

constexpr int kOuterGL = 8;      // nodes per outer panel
constexpr int kRadialGL = 12;    // nodes per radial piece (two or three pieces)
constexpr int kMaxPanelsSide = 40;

struct QuadTables {
    double gxo[kOuterGL], gwo[kOuterGL];
    double gxr[kRadialGL], gwr[kRadialGL];
};


// ---------------------------------------------------------------------------
// patch evaluation
// ---------------------------------------------------------------------------
struct HomEval {
    double A[3], W, Au[3], Wu, Av[3], Wv;   // A = H - q W and partials
};

GWN_HD inline void cubic_b(double t, double *B, double *dB)
{
    const double s = 1.0 - t;
    B[0] = s * s * s; B[1] = 3.0 * s * s * t; B[2] = 3.0 * s * t * t; B[3] = t * t * t;
    dB[0] = -3.0 * s * s; dB[1] = 3.0 * s * (s - 2.0 * t); dB[2] = 3.0 * t * (2.0 * s - t); dB[3] = 3.0 * t * t;
}

GWN_HD inline void hom_eval(const double *__restrict__ h, double u, double v, double qx, double qy,
                                         double qz, HomEval &e)
{
    double bu[4], du[4], bv[4], dv[4];
    cubic_b(u, bu, du);
    cubic_b(v, bv, dv);
    double H[4] = {0, 0, 0, 0}, Hu[4] = {0, 0, 0, 0}, Hv[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double r[4] = {0, 0, 0, 0}, rv[4] = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double c = h[16 * i + 4 * j + k];
                r[k] = fma(bv[j], c, r[k]);
                rv[k] = fma(dv[j], c, rv[k]);
            }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            H[k] = fma(bu[i], r[k], H[k]);
            Hu[k] = fma(du[i], r[k], Hu[k]);
            Hv[k] = fma(bu[i], rv[k], Hv[k]);
        }
    }
    e.W = H[3]; e.Wu = Hu[3]; e.Wv = Hv[3];
    e.A[0] = fma(-qx, H[3], H[0]); e.A[1] = fma(-qy, H[3], H[1]); e.A[2] = fma(-qz, H[3], H[2]);
    e.Au[0] = fma(-qx, Hu[3], Hu[0]); e.Au[1] = fma(-qy, Hu[3], Hu[1]); e.Au[2] = fma(-qz, Hu[3], Hu[2]);
    e.Av[0] = fma(-qx, Hv[3], Hv[0]); e.Av[1] = fma(-qy, Hv[3], Hv[1]); e.Av[2] = fma(-qz, Hv[3], Hv[2]);
}

// solid angle density det[A, A_u, A_v] / |A|^3
GWN_HD inline double density(const HomEval &e)
{
    const double cx = e.Au[1] * e.Av[2] - e.Au[2] * e.Av[1];
    const double cy = e.Au[2] * e.Av[0] - e.Au[0] * e.Av[2];
    const double cz = e.Au[0] * e.Av[1] - e.Au[1] * e.Av[0];
    const double det = e.A[0] * cx + e.A[1] * cy + e.A[2] * cz;
    const double r2 = e.A[0] * e.A[0] + e.A[1] * e.A[1] + e.A[2] * e.A[2];
    if (r2 == 0.0) return 0.0;
    return det / (r2 * sqrt(r2));
}

// Euclidean offset S - q and partials from the homogeneous evaluation
GWN_HD inline void euclid(const HomEval &e, double r[3], double Su[3], double Sv[3])
{
    const double iw = 1.0 / e.W, iw2 = iw * iw;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r[k] = e.A[k] * iw;
        Su[k] = (e.Au[k] * e.W - e.A[k] * e.Wu) * iw2;
        Sv[k] = (e.Av[k] * e.W - e.A[k] * e.Wv) * iw2;
    }
}

// ---------------------------------------------------------------------------
// boundary curves in (u, v): rational quadratics (segments elevated)
// ---------------------------------------------------------------------------
struct Curve2 {
    double h[9];
};

GWN_HD inline void curve_eval(const Curve2 &c, double t, double &u, double &v, double &du, double &dv)
{
    const double s = 1.0 - t;
    const double b0 = s * s, b1 = 2.0 * s * t, b2 = t * t;
    const double d0 = -2.0 * s, d1 = 2.0 * (s - t), d2 = 2.0 * t;
    const double hu = b0 * c.h[0] + b1 * c.h[3] + b2 * c.h[6];
    const double hv = b0 * c.h[1] + b1 * c.h[4] + b2 * c.h[7];
    const double hw = b0 * c.h[2] + b1 * c.h[5] + b2 * c.h[8];
    const double gu = d0 * c.h[0] + d1 * c.h[3] + d2 * c.h[6];
    const double gv = d0 * c.h[1] + d1 * c.h[4] + d2 * c.h[7];
    const double gw = d0 * c.h[2] + d1 * c.h[5] + d2 * c.h[8];
    const double iw = 1.0 / hw;
    u = hu * iw;
    v = hv * iw;
    du = (gu - u * gw) * iw;
    dv = (gv - v * gw) * iw;
}

GWN_HD inline Curve2 square_edge(int e)
{
    // counter-clockwise: (0,0)->(1,0)->(1,1)->(0,1)->(0,0)
    const double P[5][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}, {0, 0}};
    Curve2 c;
    c.h[0] = P[e][0]; c.h[1] = P[e][1]; c.h[2] = 1.0;
    c.h[3] = 0.5 * (P[e][0] + P[e + 1][0]); c.h[4] = 0.5 * (P[e][1] + P[e + 1][1]); c.h[5] = 1.0;
    c.h[6] = P[e + 1][0]; c.h[7] = P[e + 1][1]; c.h[8] = 1.0;
    return c;
}

// H(p) = integral_0^1 g(c + tau (p - c)) tau dtau, sinh-graded at tau = 0.
template <class CtrT>
GWN_HD inline double radial(const QuadTables &Q, const double *__restrict__ h, double cu, double cv, double ru,
                            double rv, double qx, double qy, double qz, double dist, const double Su[3],
                            const double Sv[3], CtrT &ctr, bool count)
{
    const double lx = Su[0] * ru + Sv[0] * rv, ly = Su[1] * ru + Sv[1] * rv, lz = Su[2] * ru + Sv[2] * rv;
    const double L = sqrt(lx * lx + ly * ly + lz * lz);
    const double eps = L > 0.0 ? dist / L : 1.0;
    // eps >= 0.5: two uniform Gauss-Legendre pieces in tau.  Otherwise
    // pieces in sigma with tau = eps sinh(mu sigma): tau <= 4 eps,
    // 4 eps <= tau <= 0.1, tau >= 0.1 (fewer when eps is not small; no piece
    // may reach past tau = 1, where the patch is evaluated outside its
    // parameter square).  One loop, so the patch evaluation is inlined once.
    const bool uni = eps >= 0.5;
    double mu = 1.0, cuts[4] = {0.0, 0.5, 1.0, 1.0};
    int npieces = 2;
    if (!uni) {
        mu = asinh(1.0 / eps);
        const double sa = asinh(4.0) / mu, sb = asinh(0.1 / eps) / mu;
        npieces = 1;
        cuts[1] = 1.0;
        cuts[2] = 1.0;
        if (sb > sa) { cuts[1] = sa; cuts[2] = sb; npieces = 3; }
        else if (sa < 1.0) { cuts[1] = sa; npieces = 2; }
    }
    double sum = 0.0;
#pragma unroll 1
    for (int piece = 0; piece < npieces; ++piece) {
        const double a = cuts[piece], b = cuts[piece + 1];
#pragma unroll 1
        for (int i = 0; i < kRadialGL; ++i) {
            const double x = a + (b - a) * Q.gxr[i];
            double tau, wt;
            if (uni) {
                tau = x;
                wt = (b - a) * Q.gwr[i];
            } else {
                // sinh and cosh from one expm1: e - 1/e = em (1 + 1/e)
                const double em = expm1(mu * x), ie = 1.0 / (1.0 + em);
                tau = eps * 0.5 * (em + em * ie);
                wt = eps * mu * 0.5 * (1.0 + em + ie) * (b - a) * Q.gwr[i];
            }
            HomEval e;
            hom_eval(h, cu + tau * ru, cv + tau * rv, qx, qy, qz, e);
            sum += wt * tau * density(e);
        }
    }
    if (count) ctr_add(ctr, GWN_C_PIECES, npieces * kRadialGL);
    return sum;
}

// Geometric panels on [a, b] graded from `c` (in [a, b]) with first width
// h0, each integrated with the outer Gauss-Legendre rule.
template <class F>
GWN_HD inline double graded_panels(const QuadTables &Q, double a, double b, double c, double h0, F &&f)
{
    double total = 0.0;
    for (int side = 0; side < 2; ++side) {
        const double end = side == 0 ? b : a;
        double lo = c, w = h0;
        for (int k = 0; k < kMaxPanelsSide; ++k) {
            if (side == 0 ? lo >= end : lo <= end) break;
            double hi = side == 0 ? fmin(end, lo + w) : fmax(end, lo - w);
            if (k == kMaxPanelsSide - 1) hi = end;
            const double pa = fmin(lo, hi), pb = fmax(lo, hi), len = pb - pa;
            for (int i = 0; i < kOuterGL; ++i) total += len * Q.gwo[i] * f(pa + len * Q.gxo[i]);
            lo = hi;
            if (k > 0) w *= 2.0;
        }
    }
    return total;
}

struct NearFrame {
    double cu, cv;       // foot point
    double dist;         // distance from q to the surface (1e300 when on it)
    double dparam;       // grading width near c, in parameter units
    double Su[3], Sv[3]; // partials at c
    double ew_u, ew_v;   // weak metric direction
    double anis;         // sqrt(l1 / l2)
};

// Outer integral over one boundary curve, panels graded from the point
// nearest c and from the crossings of the ray from c along the weak
// direction.
template <class CtrT>
GWN_HD inline double curve_contribution(const QuadTables &Q, const double *__restrict__ h, const Curve2 &cv,
                                        const NearFrame &fr, double qx, double qy, double qz, CtrT &ctr, bool count)
{
    double centres[3], widths[3];
    int nc = 0;
    int best = 0;
    double bd = INFINITY, prev = 0.0;
    for (int k = 0; k <= 16; ++k) {
        const double t = k / 16.0;
        double u, v, du, dv;
        curve_eval(cv, t, u, v, du, dv);
        const double d2 = (u - fr.cu) * (u - fr.cu) + (v - fr.cv) * (v - fr.cv);
        if (d2 < bd) { bd = d2; best = k; }
        const double sd = (u - fr.cu) * fr.ew_v - (v - fr.cv) * fr.ew_u;
        if (fr.anis < 0.5 && k > 0 && nc < 2 && ((prev < 0.0 && sd >= 0.0) || (prev > 0.0 && sd <= 0.0))) {
            double lo = (k - 1) / 16.0, hi = t, flo = prev;
            for (int it = 0; it < 50; ++it) {
                const double m = 0.5 * (lo + hi);
                double mu, mv, mdu, mdv;
                curve_eval(cv, m, mu, mv, mdu, mdv);
                const double fm = (mu - fr.cu) * fr.ew_v - (mv - fr.cv) * fr.ew_u;
                if ((flo < 0.0) == (fm < 0.0)) { lo = m; flo = fm; } else hi = m;
            }
            const double tr = 0.5 * (lo + hi);
            double ru, rv, rdu, rdv;
            curve_eval(cv, tr, ru, rv, rdu, rdv);
            const double rr = sqrt((ru - fr.cu) * (ru - fr.cu) + (rv - fr.cv) * (rv - fr.cv));
            const double speed = sqrt(rdu * rdu + rdv * rdv);
            centres[nc] = tr;
            widths[nc++] = speed > 0.0 ? fmax(fr.anis * rr, fr.dparam) / speed : 1.0;
        }
        prev = sd;
    }
    {
        auto near2 = [&](double t) {
            double u, v, du, dv;
            curve_eval(cv, t, u, v, du, dv);
            return (u - fr.cu) * (u - fr.cu) + (v - fr.cv) * (v - fr.cv);
        };
        double a = fmax(best - 1, 0) / 16.0, b = fmin(best + 1, 16) / 16.0;
        const double gr = 0.6180339887498949;
        double x1 = b - gr * (b - a), x2 = a + gr * (b - a);
        double f1 = near2(x1), f2 = near2(x2);
        for (int it = 0; it < 40; ++it) {
            if (f1 < f2) { b = x2; x2 = x1; f2 = f1; x1 = b - gr * (b - a); f1 = near2(x1); }
            else { a = x1; x1 = x2; f1 = f2; x2 = a + gr * (b - a); f2 = near2(x2); }
        }
        double tc = 0.5 * (a + b);
        const double fc = near2(tc), f0 = near2(0.0), fe = near2(1.0);
        if (f0 <= fc && f0 <= fe) tc = 0.0;
        else if (fe <= fc) tc = 1.0;
        double u, v, du, dv;
        curve_eval(cv, tc, u, v, du, dv);
        const double delta = sqrt((u - fr.cu) * (u - fr.cu) + (v - fr.cv) * (v - fr.cv));
        const double speed = sqrt(du * du + dv * dv);
        centres[nc] = tc;
        widths[nc++] = speed > 0.0 ? fmax(delta, fr.dparam) / speed : 1.0;
    }
    for (int i = 1; i < nc; ++i)
        for (int j = i; j > 0 && centres[j] < centres[j - 1]; --j) {
            double t = centres[j]; centres[j] = centres[j - 1]; centres[j - 1] = t;
            t = widths[j]; widths[j] = widths[j - 1]; widths[j - 1] = t;
        }
    {   // merge centres that lie within each other's first panel (keep the finer)
        int m = 0;
        for (int k = 0; k < nc; ++k) {
            if (m > 0 && centres[k] - centres[m - 1] <= fmax(widths[k], widths[m - 1])) {
                if (widths[k] < widths[m - 1]) { centres[m - 1] = centres[k]; widths[m - 1] = widths[k]; }
                continue;
            }
            centres[m] = centres[k];
            widths[m] = widths[k];
            ++m;
        }
        nc = m;
    }
    auto integrand = [&](double t) {
        double pu, pv, pdu, pdv;
        curve_eval(cv, t, pu, pv, pdu, pdv);
        const double ru = pu - fr.cu, rv = pv - fr.cv;
        const double cr = ru * pdv - rv * pdu;
        if (cr == 0.0) return 0.0;
        return cr * radial(Q, h, fr.cu, fr.cv, ru, rv, qx, qy, qz, fr.dist, fr.Su, fr.Sv, ctr, count);
    };
    double total = 0.0;
    for (int k = 0; k < nc; ++k) {
        const double lo = k == 0 ? 0.0 : 0.5 * (centres[k - 1] + centres[k]);
        const double hi = k == nc - 1 ? 1.0 : 0.5 * (centres[k] + centres[k + 1]);
        // first panel at most 1/4 of the curve; 1/8 at a collapsed edge
        // (pole), where the integrand is near-singular along the whole edge
        total += graded_panels(Q, lo, hi, centres[k], fmin(widths[k], fr.anis < 0.2 ? 0.125 : 0.25), integrand);
    }
    return total;
}

// Foot point of q on the untrimmed patch: 9 x 9 samples, then projected
// Gauss-Newton steps with step halving from the best sample and from the
// best one away from it (the distance can have several local minima on
// strongly non-uniform or folded patches).
// Returns the squared distance and (u, v) the parameters; (ou, ov, od) the
// other converged minimum (possibly the same point).
GWN_HD inline double gauss_newton_foot(const double *__restrict__ h, double qx, double qy, double qz, double &bu,
                                       double &bv, double bd)
{
    double r[3], Su[3], Sv[3];
    for (int it = 0; it < 16; ++it) {
        HomEval e;
        hom_eval(h, bu, bv, qx, qy, qz, e);
        euclid(e, r, Su, Sv);
        const double a = Su[0] * Su[0] + Su[1] * Su[1] + Su[2] * Su[2];
        const double b = Su[0] * Sv[0] + Su[1] * Sv[1] + Su[2] * Sv[2];
        const double c = Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2];
        const double gu = Su[0] * r[0] + Su[1] * r[1] + Su[2] * r[2];
        const double gv = Sv[0] * r[0] + Sv[1] * r[1] + Sv[2] * r[2];
        const double det = a * c - b * b;
        double du, dv;
        if (fabs(det) > 1e-300) { du = -(c * gu - b * gv) / det; dv = -(a * gv - b * gu) / det; }
        else { du = -gu / (a + 1e-300); dv = -gv / (c + 1e-300); }
        double step = 1.0;
        bool moved = false;
        for (int ls = 0; ls < 8; ++ls) {
            const double nu = fmin(1.0, fmax(0.0, bu + step * du)), nv = fmin(1.0, fmax(0.0, bv + step * dv));
            HomEval f;
            hom_eval(h, nu, nv, qx, qy, qz, f);
            const double d2 = (f.A[0] * f.A[0] + f.A[1] * f.A[1] + f.A[2] * f.A[2]) / (f.W * f.W);
            if (d2 < bd) { bd = d2; bu = nu; bv = nv; moved = true; break; }
            step *= 0.5;
        }
        if (!moved || step * (fabs(du) + fabs(dv)) < 1e-15) break;
    }
    return bd;
}

GWN_HD inline double foot_point3d(const double *__restrict__ h, double qx, double qy, double qz, double &bu,
                                  double &bv, double &ou, double &ov, double &od)
{
    // best sample, then the best one outside its 5 x 5 neighbourhood (a
    // start in another basin when the distance has a second minimum); one
    // loop over both passes, so the patch evaluation is inlined once
    double d1 = INFINITY, d2b = INFINITY, u1 = 0.5, v1 = 0.5, u2 = 0.5, v2 = 0.5;
    int i1 = 0, j1 = 0;
#pragma unroll 1
    for (int t = 0; t < 162; ++t) {
        const bool second = t >= 81;
        const int k = second ? t - 81 : t, i = k / 9, j = k - 9 * (k / 9);
        if (second && abs(i - i1) <= 2 && abs(j - j1) <= 2) continue;
        HomEval e;
        hom_eval(h, 0.125 * i, 0.125 * j, qx, qy, qz, e);
        const double d2 = (e.A[0] * e.A[0] + e.A[1] * e.A[1] + e.A[2] * e.A[2]) / (e.W * e.W);
        if (!second && d2 < d1) { d1 = d2; u1 = 0.125 * i; v1 = 0.125 * j; i1 = i; j1 = j; }
        if (second && d2 < d2b) { d2b = d2; u2 = 0.125 * i; v2 = 0.125 * j; }
    }
#pragma unroll 1
    for (int k = 0; k < 2; ++k) {
        double u = k ? u2 : u1, v = k ? v2 : v1, d = k ? d2b : d1;
        if (d < INFINITY) d = gauss_newton_foot(h, qx, qy, qz, u, v, d);
        if (k) { u2 = u; v2 = v; d2b = d; } else { u1 = u; v1 = v; d1 = d; }
    }
    double bd = d1;
    bu = u1;
    bv = v1;
    ou = u2;
    ov = v2;
    od = d2b;
    if (d2b < d1) { bd = d2b; bu = u2; bv = v2; ou = u1; ov = v1; od = d1; }
    return bd;
}

// Polar frame at the foot point (cu, cv) with squared distance d2.
GWN_HD inline NearFrame near_frame(const double *__restrict__ h, double cu, double cv, double d2, double qx,
                                   double qy, double qz, double eps_on)
{
    NearFrame fr;
    fr.cu = cu;
    fr.cv = cv;
    double r[3];
    HomEval e;
    hom_eval(h, cu, cv, qx, qy, qz, e);
    euclid(e, r, fr.Su, fr.Sv);
    // q on the surface (within eps_on): no near-singular peak is resolved,
    // which yields the direct value (mean of the one-sided limits)
    const bool on_surface = sqrt(d2) < eps_on;
    fr.dist = on_surface ? 1e300 : sqrt(d2);
    // metric J^T J at c: eigenvalues l1 <= l2; weak direction perpendicular
    // to the major axis at angle atan2(2 gb, ga - gc) / 2 (stable also when
    // gb is pure roundoff)
    const double *Su = fr.Su, *Sv = fr.Sv;
    const double ga = Su[0] * Su[0] + Su[1] * Su[1] + Su[2] * Su[2];
    const double gb = Su[0] * Sv[0] + Su[1] * Sv[1] + Su[2] * Sv[2];
    const double gc = Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2];
    const double tr = 0.5 * (ga + gc), df = sqrt(fmax(0.25 * (ga - gc) * (ga - gc) + gb * gb, 0.0));
    const double l2 = tr + df, l1 = fmax(tr - df, 0.0);
    const double theta = 0.5 * atan2(2.0 * gb, ga - gc);
    fr.ew_u = -sin(theta);
    fr.ew_v = cos(theta);
    fr.anis = l2 > 0.0 ? sqrt(l1 / l2) : 1.0;
    fr.dparam = l2 > 0.0 ? fmax(sqrt(d2), eps_on) / sqrt(l2) : 1.0;
    return fr;
}

// Straight edge e (0..3, counter-clockwise) of [u0, u1] x [v0, v1].
GWN_HD inline Curve2 rect_edge(double u0, double u1, double v0, double v1, int e)
{
    const double P[5][2] = {{u0, v0}, {u1, v0}, {u1, v1}, {u0, v1}, {u0, v0}};
    Curve2 c;
    c.h[0] = P[e][0]; c.h[1] = P[e][1]; c.h[2] = 1.0;
    c.h[3] = 0.5 * (P[e][0] + P[e + 1][0]); c.h[4] = 0.5 * (P[e][1] + P[e + 1][1]); c.h[5] = 1.0;
    c.h[6] = P[e + 1][0]; c.h[7] = P[e + 1][1]; c.h[8] = 1.0;
    return c;
}

// Near-field solid angle of one (trimmed) patch at q.  When the distance to
// an untrimmed patch has a second local minimum (a fold, or a strongly
// non-uniform parametrisation that stretches the near-singular region) no
// farther from q than twice the two minima's separation on the surface, the
// patch is split halfway between them into two rectangles, each integrated
// about its own foot point: the rule resolves one near-singular peak per
// domain.
template <bool COUNT, class CtrT>
GWN_HD __attribute__((always_inline)) inline double near3d(const QuadTables &Q, const Prim3 *__restrict__ P,
                                                           const Trim3 *__restrict__ trims, double qx, double qy,
                                                           double qz, double eps_on, CtrT &ctr)
{
    const double *__restrict__ h = P->h;
    double bu, bv, ou, ov, od;
    const double bd = foot_point3d(h, qx, qy, qz, bu, bv, ou, ov, od);
    const int nt = P->trim_count;
    bool split = false;
    if (nt == 0 && fabs(ou - bu) + fabs(ov - bv) > 0.05 && od < INFINITY) {
        double p[3] = {0.0, 0.0, 0.0}, sep2 = 0.0;
#pragma unroll 1
        for (int k = 0; k < 2; ++k) {
            HomEval e;
            hom_eval(h, k ? ou : bu, k ? ov : bv, qx, qy, qz, e);
            for (int a = 0; a < 3; ++a) {
                const double x = e.A[a] / e.W;
                if (k) sep2 += (x - p[a]) * (x - p[a]); else p[a] = x;
            }
        }
        split = od < 4.0 * sep2;
    }
    // cut across the larger parameter gap, halfway between the minima
    const bool cut_u = fabs(ou - bu) >= fabs(ov - bv);
    const double cut = cut_u ? 0.5 * (bu + ou) : 0.5 * (bv + ov);
    double total = 0.0;
    const int nparts = split ? 2 : 1;
#pragma unroll 1
    for (int part = 0; part < nparts; ++part) {
        const double cu = part ? ou : bu, cv = part ? ov : bv, d2 = part ? od : bd;
        double u0 = 0.0, u1 = 1.0, v0 = 0.0, v1 = 1.0;
        if (split) {
            const bool low = (cut_u ? cu : cv) < cut;
            if (cut_u) { if (low) u1 = cut; else u0 = cut; }
            else { if (low) v1 = cut; else v0 = cut; }
        }
        const NearFrame fr = near_frame(h, cu, cv, d2, qx, qy, qz, eps_on);
        const int ncv = nt == 0 ? 4 : nt;
#pragma unroll 1
        for (int k = 0; k < ncv; ++k) {
            Curve2 crv;
            if (nt == 0) {
                crv = rect_edge(u0, u1, v0, v1, k);
            } else {
                const Trim3 *t = trims + P->trim_begin + k;
                for (int m = 0; m < 9; ++m) crv.h[m] = t->h[m];
            }
            total += curve_contribution(Q, h, crv, fr, qx, qy, qz, ctr, COUNT);
        }
    }
    return total;
}

}  // namespace gwn
