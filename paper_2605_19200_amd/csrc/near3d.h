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
//
// Error control to the tolerance eps_q of the direct evaluation (Sec. 3.3,
// Sec. 4.2): every outer panel and every radial piece is integrated with a
// (2n+1)-point Gauss-Kronrod rule, whose embedded n-point Gauss rule gives
// an error estimate.  The leaf's budget 4 pi eps_q (solid angle) is spent
// panel by panel over all its boundary curves: each panel may use the
// remaining budget divided by the panels still to come.  A panel whose
// estimate -- its own,
// plus the radial estimates of its nodes weighted by |cross| and the panel
// length -- exceeds its share is integrated again as 2, 4, ... 2^kOuterLevels
// equal sub-panels until the sum of their estimates meets the share; a
// radial piece likewise as 2, ... 2^kRadialLevels sub-pieces against its
// share of the node's radial tolerance.  Estimates at the rounding level of
// the sums are accepted (refinement cannot lower them).  A panel or piece
// that still misses its share at the last level raises the budget flag: the
// caller reports the query as an overflow (NaN), never as a silent value.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "gwn_internal.h"

#define GWN_HD __host__ __device__

namespace gwn {

// Gauss points of the outer (G4 / K9) and radial (G6 / K13) pairs: on the
// CAD assembly's near-field pairs the cheapest that met the tolerance
// without refinement in most leaves (about 1.3x the integrand evaluations
// of the fixed 8 x 12-point rule it replaced; pairs (5, 5) to (7, 7) took
// 1.4x to 2.4x)
constexpr int kOuterN = 4;
constexpr int kRadialN = 6;
constexpr int kGKo = 2 * kOuterN + 1;      // Kronrod nodes per outer panel
constexpr int kGKr = 2 * kRadialN + 1;     // Kronrod nodes per radial piece
constexpr int kMaxPanelsSide = 40;
constexpr int kOuterLevels = 5;    // an outer panel is refined into at most 32
constexpr int kRadialLevels = 4;   // a radial piece into at most 16

// Gauss-Kronrod nodes and weights on [0, 1] of the outer and radial pairs
// (increasing; the odd ones are the Gauss nodes, g* their Gauss weights).
struct QuadTables {
    double xo[kGKo], wo[kGKo], go[kOuterN];
    double xr[kGKr], wr[kGKr], gr[kRadialN];
};

// Error estimate of a Kronrod / Gauss pair (the truncation part): resasc =
// the Kronrod integral of |f - K / len| times the panel length.  The
// difference |K - G| measures the Gauss rule's error; for an integrand in
// the asymptotic regime the Kronrod rule's error is about resasc times
// (|K - G| / resasc)^((3n + 2) / (2n)), with an exponent of 1.6 to 1.7 for
// n = 4..7.  The estimate takes the power 1.5, as QUADPACK does, but
// without its extra factor 200 inside the power, which on these sinh-graded
// radial pieces over-estimated errors of ~1e-11 as ~1e-6.
GWN_HD inline double gk_error(double K, double G, double resasc)
{
    const double e = fabs(K - G);
    if (resasc == 0.0 || e == 0.0) return e;
    const double r = fmin(1.0, e / resasc);
    return resasc * r * sqrt(r);
}

// Rounding level of a Kronrod sum (QUADPACK's floor, 50 eps times the sum of
// |f|): an estimate below it cannot be improved by refinement.  The radial
// rule passes the sum of |f| times each node's noise factor: A = H - q W
// loses digits as |q| W / |A| near the foot point.
GWN_HD inline double gk_round(double resabs) { return 50.0 * 2.220446049250313e-16 * resabs; }

// A (query, leaf) pair stops refining after this many integrand
// evaluations (about 20 times a typical pair); running out is a budget
// overrun.
constexpr long long kMaxEvalsPerPair = 100000;

// Error budget of one leaf, spent panel by panel: a panel may use the
// remaining budget divided by the panels still to come, so the sum of the
// accepted estimates never exceeds the leaf's tolerance and what one panel
// does not use passes on to the next.
struct Budget {
    double rem;        // tolerance not yet spent
    int left;          // panels still to integrate
    long long spent;   // integrand evaluations so far
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

// H(p) = integral_0^1 g(c + tau (p - c)) tau dtau, sinh-graded at tau = 0,
// to the absolute tolerance tolH (err: its estimate; ovf set when a piece
// misses its share at the last refinement level).
template <class CtrT>
GWN_HD inline double radial(const QuadTables &Q, const double *__restrict__ h, double cu, double cv, double ru,
                            double rv, double qx, double qy, double qz, double dist, const double Su[3],
                            const double Sv[3], double tolH, double qnorm, Budget &B, double &err, double &rnd_out,
                            bool &ovf, CtrT &ctr, bool count)
{
    const double lx = Su[0] * ru + Sv[0] * rv, ly = Su[1] * ru + Sv[1] * rv, lz = Su[2] * ru + Sv[2] * rv;
    const double L = sqrt(lx * lx + ly * ly + lz * lz);
    const double eps = L > 0.0 ? dist / L : 1.0;
    // eps >= 0.5: two uniform pieces in tau.  Otherwise pieces in sigma with
    // tau = eps sinh(mu sigma): tau <= 4 eps, 4 eps <= tau <= 0.1,
    // tau >= 0.1 (fewer when eps is not small; no piece may reach past
    // tau = 1, where the patch is evaluated outside its parameter square).
    // One node loop, so the patch evaluation is inlined once.
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
    const double tol_piece = tolH / npieces;
    double sum = 0.0, esum = 0.0, rsum = 0.0;
    long long evals = 0;
#pragma unroll 1
    for (int piece = 0; piece < npieces; ++piece) {
        const double a = cuts[piece], b = cuts[piece + 1];
        double val = 0.0, e = 0.0, rnd = 0.0;
#pragma unroll 1
        for (int level = 0; level <= kRadialLevels; ++level) {
            const int nsub = 1 << level;
            const double w = (b - a) / nsub;
            rnd = 0.0;
            val = 0.0;
            e = 0.0;
#pragma unroll 1
            for (int sp = 0; sp < nsub; ++sp) {
                const double pa = a + sp * w, pw = w;
                double K = 0.0, G = 0.0, fabs_sum = 0.0, noise = 0.0;
                double fv[kGKr];
#pragma unroll 1
                for (int i = 0; i < kGKr; ++i) {
                    const double x = pa + pw * Q.xr[i];
                    double tau, jac;
                    if (uni) {
                        tau = x;
                        jac = 1.0;
                    } else {
                        // sinh and cosh from one expm1: e - 1/e = em (1 + 1/e)
                        const double em = expm1(mu * x), ie = 1.0 / (1.0 + em);
                        tau = eps * 0.5 * (em + em * ie);
                        jac = eps * mu * 0.5 * (1.0 + em + ie);
                    }
                    HomEval ev;
                    hom_eval(h, cu + tau * ru, cv + tau * rv, qx, qy, qz, ev);
                    const double f = jac * tau * density(ev);
                    const double a2 = ev.A[0] * ev.A[0] + ev.A[1] * ev.A[1] + ev.A[2] * ev.A[2];
                    fv[i] = f;
                    K += Q.wr[i] * f;
                    fabs_sum += Q.wr[i] * fabs(f);
                    noise += Q.wr[i] * fabs(f) * (1.0 + (a2 > 0.0 ? qnorm * fabs(ev.W) / sqrt(a2) : 0.0));
                }
#pragma unroll
                for (int i = 0; i < kRadialN; ++i) G += Q.gr[i] * fv[2 * i + 1];
                double asc = 0.0;
#pragma unroll
                for (int i = 0; i < kGKr; ++i) asc += Q.wr[i] * fabs(fv[i] - K);
                val += pw * K;
                e += gk_error(pw * K, pw * G, pw * asc);
                rnd += gk_round(pw * noise);
                evals += kGKr;
            }
            if (e <= fmax(tol_piece, rnd)) break;
            if (level == kRadialLevels || B.spent + evals > kMaxEvalsPerPair) {
                ovf = true;
                break;
            }
        }
        sum += val;
        esum += e;
        rsum += rnd;
    }
    if (count) ctr_add(ctr, GWN_C_PIECES, evals);
    B.spent += evals;
    err = esum;
    rnd_out = rsum;
    return sum;
}

// Geometric panels on [a, b] graded from `c` (in [a, b]) with first width
// h0: the number of panels, for sharing the tolerance.
GWN_HD inline int count_panels(double a, double b, double c, double h0)
{
    int n = 0;
    for (int side = 0; side < 2; ++side) {
        const double end = side == 0 ? b : a;
        double lo = c, w = h0;
        for (int k = 0; k < kMaxPanelsSide; ++k) {
            if (side == 0 ? lo >= end : lo <= end) break;
            double hi = side == 0 ? fmin(end, lo + w) : fmax(end, lo - w);
            if (k == kMaxPanelsSide - 1) hi = end;
            ++n;
            lo = hi;
            if (k > 0) w *= 2.0;
        }
    }
    return n;
}

// The same panels, each integrated to its share of the leaf's budget B:
// f(t, tol_f, err_f, rnd_f) returns the integrand at t, which carries its
// own error estimate err_f (computed against tol_f) and rounding level rnd_f.
// A panel whose estimate exceeds its share is integrated again as 2, 4, ...
// equal sub-panels.
template <class F>
GWN_HD inline double graded_panels(const QuadTables &Q, double a, double b, double c, double h0, Budget &B,
                                   bool &ovf, F &&f)
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
            const double share = fmax(B.rem, 0.0) / (B.left > 0 ? B.left : 1);
            double val = 0.0, e = 0.0;
#pragma unroll 1
            for (int level = 0; level <= kOuterLevels; ++level) {
                const int nsub = 1 << level;
                const double sw = len / nsub;
                double rnd = 0.0;
                e = 0.0;
                val = 0.0;
#pragma unroll 1
                for (int sp = 0; sp < nsub; ++sp) {
                    const double sa = pa + sp * sw;
                    double K = 0.0, G = 0.0, fabs_sum = 0.0, erad = 0.0, rrad = 0.0;
                    double fv[kGKo];
#pragma unroll 1
                    for (int i = 0; i < kGKo; ++i) {
                        // the radial part of the estimate stays within half
                        // the share
                        double ef = 0.0, rf = 0.0;
                        const double fx = f(sa + sw * Q.xo[i], 0.5 * share / len, ef, rf);
                        fv[i] = fx;
                        K += Q.wo[i] * fx;
                        fabs_sum += Q.wo[i] * fabs(fx);
                        erad += Q.wo[i] * ef;
                        rrad += Q.wo[i] * rf;
                    }
#pragma unroll
                    for (int i = 0; i < kOuterN; ++i) G += Q.go[i] * fv[2 * i + 1];
                    double asc = 0.0;
#pragma unroll
                    for (int i = 0; i < kGKo; ++i) asc += Q.wo[i] * fabs(fv[i] - K);
                    val += sw * K;
                    e += gk_error(sw * K, sw * G, sw * asc) + sw * erad;
                    rnd += gk_round(sw * fabs_sum) + sw * rrad;
                }
                if (e <= fmax(share, rnd)) break;
                if (level == kOuterLevels || B.spent > kMaxEvalsPerPair) {
                    ovf = true;
                    break;
                }
            }
            total += val;
            B.rem -= fmin(e, share);
            B.left -= 1;
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
                                        const NearFrame &fr, double qx, double qy, double qz, bool count_only,
                                        Budget &B, bool &ovf, CtrT &ctr, bool count)
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
    // integrand at t with its error: |cross| times the radial estimate, the
    // radial integral taken to tol_f / |cross|
    const double qnorm = sqrt(qx * qx + qy * qy + qz * qz);
    auto integrand = [&](double t, double tol_f, double &err_f, double &rnd_f) {
        double pu, pv, pdu, pdv;
        curve_eval(cv, t, pu, pv, pdu, pdv);
        const double ru = pu - fr.cu, rv = pv - fr.cv;
        const double cr = ru * pdv - rv * pdu;
        err_f = 0.0;
        rnd_f = 0.0;
        if (cr == 0.0) return 0.0;
        double eH = 0.0, rH = 0.0;
        const double H = radial(Q, h, fr.cu, fr.cv, ru, rv, qx, qy, qz, fr.dist, fr.Su, fr.Sv, tol_f / fabs(cr), qnorm,
                                B, eH, rH, ovf, ctr, count);
        err_f = fabs(cr) * eH;
        rnd_f = fabs(cr) * rH;
        return cr * H;
    };
    // first panel at most 1/4 of the curve; 1/8 at a collapsed edge (pole),
    // where the integrand is near-singular along the whole edge
    const double first = fr.anis < 0.2 ? 0.125 : 0.25;
    if (count_only) {   // the number of initial panels, for the budget
        int npanels = 0;
        for (int k = 0; k < nc; ++k) {
            const double lo = k == 0 ? 0.0 : 0.5 * (centres[k - 1] + centres[k]);
            const double hi = k == nc - 1 ? 1.0 : 0.5 * (centres[k] + centres[k + 1]);
            npanels += count_panels(lo, hi, centres[k], fmin(widths[k], first));
        }
        return (double)npanels;
    }
    double total = 0.0;
    for (int k = 0; k < nc; ++k) {
        const double lo = k == 0 ? 0.0 : 0.5 * (centres[k - 1] + centres[k]);
        const double hi = k == nc - 1 ? 1.0 : 0.5 * (centres[k] + centres[k + 1]);
        total += graded_panels(Q, lo, hi, centres[k], fmin(widths[k], first), B, ovf, integrand);
    }
    return total;
}

// Start grid of the foot-point search: kFootGrid^2 samples of the square.
constexpr int kFootGrid = 9;
constexpr double kFootStep = 1.0 / (kFootGrid - 1);

// Foot point of q on the untrimmed patch: kFootGrid^2 samples, then projected
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
    for (int t = 0; t < 2 * kFootGrid * kFootGrid; ++t) {
        const bool second = t >= kFootGrid * kFootGrid;
        const int k = second ? t - kFootGrid * kFootGrid : t, i = k / kFootGrid, j = k - kFootGrid * (k / kFootGrid);
        if (second && abs(i - i1) <= 2 && abs(j - j1) <= 2) continue;
        HomEval e;
        hom_eval(h, kFootStep * i, kFootStep * j, qx, qy, qz, e);
        const double d2 = (e.A[0] * e.A[0] + e.A[1] * e.A[1] + e.A[2] * e.A[2]) / (e.W * e.W);
        if (!second && d2 < d1) { d1 = d2; u1 = kFootStep * i; v1 = kFootStep * j; i1 = i; j1 = j; }
        if (second && d2 < d2b) { d2b = d2; u2 = kFootStep * i; v2 = kFootStep * j; }
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

// Crossings of a boundary curve with the line x_dir = c (x = u for dir 0,
// v for dir 1): the roots in (0, 1) of X(t) - c W(t), a quadratic in
// Bernstein form; false when the line passes through an end point of the
// curve or touches it tangentially (no well-defined crossing).
GWN_HD inline bool cut_roots(const Curve2 &cv, int dir, double c, double r[2], int &nr)
{
    double a[3];
    for (int j = 0; j < 3; ++j) a[j] = cv.h[3 * j + dir] - c * cv.h[3 * j + 2];
    nr = 0;
    const double scale = fabs(a[0]) + fabs(a[1]) + fabs(a[2]);
    if (fabs(a[0]) <= 1e-9 * fabs(cv.h[2]) || fabs(a[2]) <= 1e-9 * fabs(cv.h[8])) return false;
    const double A = a[0] - 2.0 * a[1] + a[2], B = 2.0 * (a[1] - a[0]), C = a[0];
    double t[2];
    int n = 0;
    if (fabs(A) <= 1e-14 * scale) {
        if (fabs(B) > 1e-14 * scale) t[n++] = -C / B;
    } else {
        const double disc = B * B - 4.0 * A * C;
        if (fabs(disc) <= 1e-12 * scale * scale) return false;
        if (disc > 0.0) {
            const double q = -0.5 * (B + copysign(sqrt(disc), B));
            t[n++] = q / A;
            if (q != 0.0) t[n++] = C / q;
        }
    }
    for (int k = 0; k < n; ++k)
        if (t[k] > 0.0 && t[k] < 1.0) {
            if (t[k] < 1e-9 || t[k] > 1.0 - 1e-9) return false;
            r[nr++] = t[k];
        }
    if (nr == 2 && r[0] > r[1]) { const double x = r[0]; r[0] = r[1]; r[1] = x; }
    if (nr == 2 && r[1] - r[0] < 1e-9) return false;
    return true;
}

// The piece of a boundary curve on [t0, t1] as a curve on [0, 1]: blossom
// values (t0, t0), (t0, t1), (t1, t1) of its control polygon.
GWN_HD inline Curve2 sub_curve(const Curve2 &c, double t0, double t1)
{
    Curve2 r;
    for (int k = 0; k < 3; ++k) {
        const double a0 = (1.0 - t0) * c.h[k] + t0 * c.h[3 + k], a1 = (1.0 - t0) * c.h[3 + k] + t0 * c.h[6 + k];
        const double b0 = (1.0 - t1) * c.h[k] + t1 * c.h[3 + k], b1 = (1.0 - t1) * c.h[3 + k] + t1 * c.h[6 + k];
        r.h[k] = (1.0 - t0) * a0 + t0 * a1;
        r.h[3 + k] = (1.0 - t1) * a0 + t1 * a1;
        r.h[6 + k] = (1.0 - t1) * b0 + t1 * b1;
    }
    return r;
}

constexpr int kMaxCross = 32;   // crossings of a trimmed leaf's loops with a cut

// Near-field solid angle of one (trimmed) patch at q.  When the distance to
// the patch has a second local minimum (a fold, a wavy surface, or a
// strongly non-uniform parametrisation that stretches the near-singular
// region) no farther from q than twice the two minima's separation on the
// surface, the parameter square is cut halfway between them and each half
// -- with the part of the visible region on its side -- is integrated about
// its own foot point: the rule resolves one near-singular peak per domain.
// tol: absolute tolerance on the leaf's solid angle (4 pi eps_q); ovf is
// set when a panel or piece misses its share of it at the last refinement
// level.
// q on the surface of the leaf (within eps_on of its untrimmed surface): the
// value is the direct one, the mean of the two one-sided limits, taken as the
// mean of the values at q +- delta n (n the unit normal at the foot point,
// delta = 1e3 eps_on), each under the same error control; where the foot
// point is trimmed away the value is continuous and the mean is the value.
template <bool COUNT, class CtrT>
GWN_HD __attribute__((always_inline)) inline double near3d(const QuadTables &Q, const Prim3 *__restrict__ P,
                                                           const Trim3 *__restrict__ trims, double qx, double qy,
                                                           double qz, double eps_on, double tol, bool &ovf,
                                                           CtrT &ctr)
{
    const double *__restrict__ h = P->h;
    double bu, bv, ou, ov, od;
    double bd = foot_point3d(h, qx, qy, qz, bu, bv, ou, ov, od);
    double mean = 0.0;
    int sides = 1;
    double nrm[3] = {0.0, 0.0, 0.0};
    if (sqrt(bd) < eps_on) {
        HomEval e;
        double r[3], Su[3], Sv[3];
        hom_eval(h, bu, bv, qx, qy, qz, e);
        euclid(e, r, Su, Sv);
        nrm[0] = Su[1] * Sv[2] - Su[2] * Sv[1];
        nrm[1] = Su[2] * Sv[0] - Su[0] * Sv[2];
        nrm[2] = Su[0] * Sv[1] - Su[1] * Sv[0];
        const double nn = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
        if (nn > 0.0) {
            sides = 2;
            for (int a = 0; a < 3; ++a) nrm[a] *= 1e3 * eps_on / nn;
        }
    }
    const double q0[3] = {qx, qy, qz};
#pragma unroll 1
    for (int side = 0; side < sides; ++side) {
        if (sides == 2) {
            qx = q0[0] + (side ? -nrm[0] : nrm[0]);
            qy = q0[1] + (side ? -nrm[1] : nrm[1]);
            qz = q0[2] + (side ? -nrm[2] : nrm[2]);
            bd = foot_point3d(h, qx, qy, qz, bu, bv, ou, ov, od);
        }
        const int nt = P->trim_count;
        bool split = false;
        if (fabs(ou - bu) + fabs(ov - bv) > 0.05 && od < INFINITY) {
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
        const int dir = cut_u ? 0 : 1;
        const double cut = cut_u ? 0.5 * (bu + ou) : 0.5 * (bv + ov);
        // A trimmed leaf cut in two: each half's boundary is the part of the trim
        // loops on its side plus the stretches of the cut line inside the visible
        // region.  Walking the loops with the region on the left, a curve that
        // crosses the line moving towards +x (dir 0) or -x (dir 1) starts such a
        // stretch, one moving the other way ends it.  A cut through a junction of
        // two curves or tangent to a loop is not taken (the leaf stays whole).
        double ycr[kMaxCross];
        int ncr = 0;
        if (split && nt > 0) {
#pragma unroll 1
            for (int k = 0; k < nt && split; ++k) {
                Curve2 cv;
                const Trim3 *t = trims + P->trim_begin + k;
                for (int m = 0; m < 9; ++m) cv.h[m] = t->h[m];
                double r[2];
                int nr = 0;
                if (!cut_roots(cv, dir, cut, r, nr) || ncr + nr > kMaxCross) { split = false; break; }
                for (int j = 0; j < nr; ++j) {
                    double u, v, du, dv;
                    curve_eval(cv, r[j], u, v, du, dv);
                    const double y = dir == 0 ? v : u, dx = dir == 0 ? du : dv;
                    const bool start = dir == 0 ? dx > 0.0 : dx < 0.0;
                    // store start crossings as y, end crossings as -(y + 2) so
                    // the sign survives the sort key below
                    ycr[ncr++] = start ? y : -(y + 2.0);
                }
            }
            if (split) {   // sort by y (insertion), then starts and ends must alternate
                auto key = [](double x) { return x >= 0.0 ? x : -x - 2.0; };
                for (int i = 1; i < ncr; ++i)
                    for (int j = i; j > 0 && key(ycr[j]) < key(ycr[j - 1]); --j) {
                        const double x = ycr[j]; ycr[j] = ycr[j - 1]; ycr[j - 1] = x;
                    }
                if (ncr % 2) split = false;
                for (int i = 0; i < ncr && split; ++i) {
                    if ((ycr[i] >= 0.0) != (i % 2 == 0)) split = false;
                    if (i > 0 && key(ycr[i]) - key(ycr[i - 1]) < 1e-12) split = false;
                }
            }
        }
        // The leaf's budget tol is spent panel by panel over all its boundary
        // curves: first the panels are counted, then integrated.
        const int nparts = split ? 2 : 1;
        NearFrame frs[2];
        double rect[2][4];
        bool lowside[2] = {true, true};
#pragma unroll 1
        for (int part = 0; part < nparts; ++part) {
            const double cu = part ? ou : bu, cv = part ? ov : bv, d2 = part ? od : bd;
            double u0 = 0.0, u1 = 1.0, v0 = 0.0, v1 = 1.0;
            if (split) {
                const bool low = (cut_u ? cu : cv) < cut;
                lowside[part] = low;
                if (cut_u) { if (low) u1 = cut; else u0 = cut; }
                else { if (low) v1 = cut; else v0 = cut; }
            }
            rect[part][0] = u0; rect[part][1] = u1; rect[part][2] = v0; rect[part][3] = v1;
            frs[part] = near_frame(h, cu, cv, d2, qx, qy, qz, eps_on);
        }
        Budget B{tol, 0, 0};
        double total = 0.0;
#pragma unroll 1
        for (int pass = 0; pass < 2; ++pass) {
            const bool count_only = pass == 0;
            auto integrate = [&](int part, const Curve2 &crv) {
                const double r = curve_contribution(Q, h, crv, frs[part], qx, qy, qz, count_only, B, ovf, ctr, COUNT);
                if (count_only) B.left += (int)r; else total += r;
            };
#pragma unroll 1
            for (int part = 0; part < nparts; ++part) {
                if (nt == 0) {
#pragma unroll 1
                    for (int k = 0; k < 4; ++k)
                        integrate(part, rect_edge(rect[part][0], rect[part][1], rect[part][2], rect[part][3], k));
                    continue;
                }
#pragma unroll 1
                for (int k = 0; k < nt; ++k) {
                    Curve2 crv;
                    const Trim3 *t = trims + P->trim_begin + k;
                    for (int m = 0; m < 9; ++m) crv.h[m] = t->h[m];
                    if (!split) {
                        integrate(part, crv);
                        continue;
                    }
                    double r[2];
                    int nr = 0;
                    cut_roots(crv, dir, cut, r, nr);
#pragma unroll 1
                    for (int j = 0; j <= nr; ++j) {
                        const double t0 = j == 0 ? 0.0 : r[j - 1], t1 = j == nr ? 1.0 : r[j];
                        double u, v, du, dv;
                        curve_eval(crv, 0.5 * (t0 + t1), u, v, du, dv);
                        if (((dir == 0 ? u : v) < cut) != lowside[part]) continue;
                        integrate(part, nr ? sub_curve(crv, t0, t1) : crv);
                    }
                }
                if (split) {
                    // stretches of the cut line inside the region, walked with this
                    // half on the left: +y for the low half of a u cut and the high
                    // half of a v cut
                    const bool up = (dir == 0) == lowside[part];
#pragma unroll 1
                    for (int i = 0; i + 1 < ncr; i += 2) {
                        const double ya = ycr[i], yb = -ycr[i + 1] - 2.0;
                        const double y0 = up ? ya : yb, y1 = up ? yb : ya;
                        integrate(part, dir == 0 ? rect_edge(cut, cut, y0, y1, 1) : rect_edge(y0, y1, cut, cut, 0));
                    }
                }
            }
        }
        mean += total;
    }
    return mean / sides;
}

}  // namespace gwn
