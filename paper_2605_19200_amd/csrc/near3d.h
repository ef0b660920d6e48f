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

// Gauss points of the outer (G4 / K9) and radial (G7 / K15) pairs.  The
// outer pair is the cheapest that met the tolerance without refinement in
// most leaves of the CAD assembly's near-field pairs.  A radial part is one
// 16-lane group's task whatever its node count, so the 15-node rule costs
// no more per part than the 13-node one and, of higher degree, needs fewer
// refined parts: near field 53.1 -> 51.8 ms on the bodies grid, 826 -> 783
// ms on the CAD assembly, and 2 instead of 5 of its queries overrun the
// refinement budget.
constexpr int kOuterN = 4;
constexpr int kRadialN = 7;
constexpr int kGKo = 2 * kOuterN + 1;      // Kronrod nodes per outer panel
constexpr int kGKr = 2 * kRadialN + 1;     // Kronrod nodes per radial piece
constexpr int kMaxPanelsSide = 40;
constexpr int kOuterLevels = 7;    // an outer panel is refined into at most 128
constexpr int kRadialLevels = 7;   // a radial piece into at most 128

// Gauss-Kronrod nodes and weights on [0, 1] of the outer and radial pairs
// (increasing; the odd ones are the Gauss nodes, g* their Gauss weights).
struct QuadTables {
    double xo[kGKo], wo[kGKo], go[kOuterN];
    double xr[kGKr], wr[kGKr], gr[kRadialN];
};

// Rounding level of a Kronrod sum (QUADPACK's floor, 50 eps times the sum of
// |f|): an estimate below it cannot be improved by refinement.  The radial
// rule passes the sum of |f| times each node's noise factor: A = H - q W
// loses digits as |q| W / |A| near the foot point.
GWN_HD inline double gk_round(double resabs) { return 50.0 * 2.220446049250313e-16 * resabs; }

// A (query, leaf) pair stops refining after this many integrand
// evaluations (a few hundred times a typical pair: only the hardest pairs,
// queries within a hair of a trim edge or a fold, come near it, one wave
// each, so a deep budget costs the launch nothing measurable); running out
// is a budget overrun.
constexpr long long kMaxEvalsPerPair = 1600000;

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
    // one row of the control net (16 values) at a time: the net is the same
    // on all lanes and is read with scalar loads row by row, so it never has
    // to be held whole.  On the device it is read through the constant
    // address space (it does not change during a launch), where a load from
    // a wave-uniform address always becomes a scalar load.
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) double *NetPtr;
    const NetPtr net = (NetPtr)(unsigned long long)h;
#else
    const double *__restrict__ net = h;
#endif
    // two rows per step: the second row's loads are in flight while the
    // first is summed (near field 61.2 -> 59.6 ms on the bodies grid, 845
    // -> 822 ms on the CAD assembly; all four rows at once exhaust the
    // scalar registers and run 25 % slower)
#pragma unroll 2
    for (int i = 0; i < 4; ++i) {
        const double bi = i == 0 ? bu[0] : i == 1 ? bu[1] : i == 2 ? bu[2] : bu[3];
        const double di = i == 0 ? du[0] : i == 1 ? du[1] : i == 2 ? du[2] : du[3];
        const auto row = net + 16 * i;
        double r[4] = {0, 0, 0, 0}, rv[4] = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double c = row[4 * j + k];
                r[k] = fma(bv[j], c, r[k]);
                rv[k] = fma(dv[j], c, rv[k]);
            }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            H[k] = fma(bi, r[k], H[k]);
            Hu[k] = fma(di, r[k], Hu[k]);
            Hv[k] = fma(bi, rv[k], Hv[k]);
        }
    }
    e.W = H[3]; e.Wu = Hu[3]; e.Wv = Hv[3];
    e.A[0] = fma(-qx, H[3], H[0]); e.A[1] = fma(-qy, H[3], H[1]); e.A[2] = fma(-qz, H[3], H[2]);
    e.Au[0] = fma(-qx, Hu[3], Hu[0]); e.Au[1] = fma(-qy, Hu[3], Hu[1]); e.Au[2] = fma(-qz, Hu[3], Hu[2]);
    e.Av[0] = fma(-qx, Hv[3], Hv[0]); e.Av[1] = fma(-qy, Hv[3], Hv[1]); e.Av[2] = fma(-qz, Hv[3], Hv[2]);
}

// 1 / sqrt(x) and 1 / x for normal x > 0: on the device the hardware
// estimates refined by two Newton steps (within an ulp or two, no IEEE
// square root or division sequence); on the host the plain operations.
GWN_HD inline double inv_sqrt(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    return y * fma(-h * y, y, 1.5);
#else
    return 1.0 / sqrt(x);
#endif
}

GWN_HD inline double inv_fast(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
#else
    return 1.0 / x;
#endif
}

// Error estimate of a Kronrod / Gauss pair (the truncation part): resasc =
// the Kronrod integral of |f - K / len| times the panel length.  The
// difference |K - G| measures the Gauss rule's error; for an integrand in
// the asymptotic regime the Kronrod rule's error is about resasc times
// (|K - G| / resasc)^((3n + 2) / (2n)), with an exponent of 1.6 to 1.7 for
// n = 4..7.  The estimate takes the power 1.5, as QUADPACK does, but
// without its extra factor 200 inside the power, which on these sinh-graded
// radial pieces over-estimated errors of ~1e-11 as ~1e-6.
// It runs once per radial part, so the quotient and the square root use
// the refined hardware estimates (inv_fast, inv_sqrt) rather than the IEEE
// sequences.
GWN_HD inline double gk_error(double K, double G, double resasc)
{
    const double e = fabs(K - G);
    if (resasc == 0.0 || e == 0.0) return e;
    const double r = fmin(1.0, e * inv_fast(resasc));
    return resasc * r * (r * inv_sqrt(r));
}

// solid angle density det[A, A_u, A_v] / |A|^3, and 1 / |A| in *rs (0 when
// A = 0, where the density is 0)
GWN_HD inline double density(const HomEval &e, double *rs)
{
    const double cx = e.Au[1] * e.Av[2] - e.Au[2] * e.Av[1];
    const double cy = e.Au[2] * e.Av[0] - e.Au[0] * e.Av[2];
    const double cz = e.Au[0] * e.Av[1] - e.Au[1] * e.Av[0];
    const double det = e.A[0] * cx + e.A[1] * cy + e.A[2] * cz;
    const double r2 = e.A[0] * e.A[0] + e.A[1] * e.A[1] + e.A[2] * e.A[2];
    *rs = 0.0;
    if (r2 == 0.0) return 0.0;
    const double ir = inv_sqrt(r2);
    *rs = ir;
    return det * (ir * ir * ir);
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

// ---------------------------------------------------------------------------
// Cross-lane operations.  The rule below runs one (query, leaf) pair per
// wave of 64 lanes: every value that steers it (foot point, panels,
// refinement levels, budget) is the same on all lanes, and the lanes share
// out the integrand evaluations.  Every call of these operations is made by
// all 64 lanes at the same point of the rule.  DevWave maps them to the
// wave's cross-lane instructions; `bcast` takes a source lane that is the
// same on all lanes.
// ---------------------------------------------------------------------------
struct DevWave {
    __device__ int lane() const { return __lane_id(); }
    __device__ double shfl(double x, int src) const { return __shfl(x, src); }
    __device__ int shfl(int x, int src) const { return __shfl(x, src); }
    __device__ double shfl_xor(double x, int m) const { return __shfl_xor(x, m); }
    __device__ int shfl_xor(int x, int m) const { return __shfl_xor(x, m); }
    __device__ double bcast(double x, int src) const
    {
        const unsigned long long b = (unsigned long long)__double_as_longlong(x);
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, src);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
        return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    }
    __device__ int bcast(int x, int src) const { return __builtin_amdgcn_readlane(x, src); }
    __device__ unsigned long long ballot(bool p) const { return __ballot(p); }
    // sum over the lane's group of 16 by DPP row moves: pairs, quads (quad
    // permutes), then the two quads of each half row (half mirror), then the
    // two half rows (mirror); every lane of the row gets the same bits
    __device__ double sum16(double x) const
    {
        x += dpp<0xB1>(x);    // quad_perm [1, 0, 3, 2]
        x += dpp<0x4E>(x);    // quad_perm [2, 3, 0, 1]
        x += dpp<0x141>(x);   // row_half_mirror
        x += dpp<0x140>(x);   // row_mirror
        return x;
    }
    // minimum of d over the wave with its index k (the smaller k on ties; an
    // exact total order, so the order of the steps does not matter): DPP
    // steps within each row of 16, then the four rows' results
    __device__ void argmin(double &d, int &k) const
    {
        argmin_step<0xB1>(d, k);
        argmin_step<0x4E>(d, k);
        argmin_step<0x141>(d, k);
        argmin_step<0x140>(d, k);
        double bd = bcast(d, 0);
        int bk = bcast(k, 0);
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            const double rd = bcast(d, 16 * r);
            const int rk = bcast(k, 16 * r);
            if (rd < bd || (rd == bd && rk < bk)) {
                bd = rd;
                bk = rk;
            }
        }
        d = bd;
        k = bk;
    }
    template <int CTRL>
    __device__ static void argmin_step(double &d, int &k)
    {
        const double od = dpp<CTRL>(d);
        const int ok = __builtin_amdgcn_update_dpp(0, k, CTRL, 0xf, 0xf, false);
        if (od < d || (od == d && ok < k)) {
            d = od;
            k = ok;
        }
    }
    template <int CTRL>
    __device__ static double dpp(double x)
    {
        const long long b = __double_as_longlong(x);
        const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
        const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    }
};

// Sum over the caller's group of 16 lanes (every lane of the group gets the
// same bits).
template <class Wv>
GWN_HD inline double sum16(const Wv &wv, double x)
{
    return wv.sum16(x);
}

// Minimum of d over the wave and its index k (the smaller k on ties; no NaN
// in d).
template <class Wv>
GWN_HD inline void argmin64(const Wv &wv, double &d, int &k)
{
    wv.argmin(d, k);
}

GWN_HD inline int imin(int a, int b) { return a < b ? a : b; }

// Position of the k-th set bit (from 0) of m, which has more than k bits.
GWN_HD inline int kth_bit(unsigned long long m, int k)
{
    int pos = 0;
    for (int w = 32; w > 0; w >>= 1) {
        const int c = __builtin_popcountll((m >> pos) & ((1ull << w) - 1));
        if (c <= k) {
            k -= c;
            pos += w;
        }
    }
    return pos;
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

struct NearFrame {
    double cu, cv;       // foot point
    double dist;         // distance from q to the surface (1e300 when on it)
    double dparam;       // grading width near c, in parameter units
    double Su[3], Sv[3]; // partials at c
    double ew_u, ew_v;   // weak metric direction
    double anis;         // sqrt(l1 / l2)
};

constexpr int kMaxCross = 32;   // crossings of a trimmed leaf's loops with a cut

// State of the rule kept in memory that the wave's lanes share (LDS on the
// device), read where it is used rather than held in every lane's
// registers through the integration: the polar frame of the part being
// integrated and the crossings of a split leaf's trim loops with the cut.
// Every lane writes the same values.
constexpr int kCurveCache = 48;   // curves whose grading centres are kept between the two passes

struct NearShared {
    NearFrame fr;
    double ycr[kMaxCross];
    // per boundary curve of the leaf (both parts of a split leaf): number of
    // grading centres, the centres and their first panel widths, found in
    // the counting pass and reused in the integration pass
    int ncen[kCurveCache];
    double cen[kCurveCache][3], wid[kCurveCache][3];
};

// Compiler barrier: values stored to the shared state before it are read
// back from memory after it, not carried in registers.
GWN_HD inline void compiler_fence()
{
#if defined(__HIP_DEVICE_COMPILE__)
    asm volatile("" ::: "memory");
#endif
}

// Sub-panels of an outer panel whose nodes are integrated together: 9 nodes
// each, three radial pieces per node, one task lane per piece.
constexpr int kSubPerChunk = 2;

// Values of the outer integrand at the Kronrod nodes of the sub-panels
// sp0 .. sp0 + nc - 1 of width sw of the panel starting at pa: lane m < 9 nc
// gets node m % 9 of sub-panel sp0 + m / 9, f = cross(gamma - c, gamma') H
// with its error estimate ef and rounding level rf, where H(p) =
// integral_0^1 g(c + tau (p - c)) tau dtau is sinh-graded at tau = 0 and
// taken to the tolerance tol_f / |cross|.
// H comes in up to three pieces (tau <= 4 eps, 4 eps <= tau <= 0.1, tau >=
// 0.1 with eps = d / |J (p - c)|; one uniform piece when eps >= 0.5; no
// piece reaches past tau = 1), each the task of lane 3 m + p: integrated
// by the 15-point Kronrod rule on 1, 2, 4, ... 2^kRadialLevels equal parts
// until its estimate meets its share.  The parts of the pending tasks are
// shared out over the wave's four groups of 16 lanes, one part (15 nodes)
// per group and round; each task adds the sums of its parts in their order.
template <class Wv, class CtrT>
GWN_HD inline void outer_values(const Wv &wv, const QuadTables &Q, const double *__restrict__ h, const Curve2 &cv,
                                const NearFrame &fr, double qx, double qy, double qz, double qnorm, double pa,
                                double sw, int sp0, int nc, double tol_f, Budget &B, bool &ovf, CtrT &ctr, bool count,
                                double &f, double &ef, double &rf, bool pair = false, double pa1 = 0.0,
                                double sw1 = 0.0, double tol_f1 = 0.0)
{
    compiler_fence();
    const int ln = wv.lane();
    const int M = kGKo * nc;
    const int m = ln / 3, p = ln - 3 * (ln / 3);
    const bool has = m < M;
    const int mj = has ? m / kGKo : 0, mi = has ? m - kGKo * (m / kGKo) : 0;
    // pair: the two chunks are two panels, (pa, sw) and (pa1, sw1)
    const bool second = pair && mj == 1;
    const double sa = second ? pa1 : pa + (sp0 + mj) * sw;
    const double csw = second ? sw1 : sw;
    double pu, pv, pdu, pdv;
    curve_eval(cv, sa + csw * Q.xo[mi], pu, pv, pdu, pdv);
    const double ru = pu - fr.cu, rv = pv - fr.cv;
    const double cr = ru * pdv - rv * pdu;
    const double lx = fr.Su[0] * ru + fr.Sv[0] * rv, ly = fr.Su[1] * ru + fr.Sv[1] * rv,
                 lz = fr.Su[2] * ru + fr.Sv[2] * rv;
    const double L = sqrt(lx * lx + ly * ly + lz * lz);
    // quotients by refined hardware reciprocals (one per lane and outer
    // node; the IEEE division sequences cost 3 % of the launch)
    const double eps = L > 0.0 ? fr.dist * inv_fast(L) : 1.0;
    const bool uni = eps >= 0.5;
    // eps >= 0.5: the integrand is smooth on [0, 1] and one piece is
    // enough (refined if its estimate says otherwise); two fixed halves cost
    // 34 % more integrand evaluations and 11 % more time on the bodies grid
    double mu = 1.0, cuts[4] = {0.0, 1.0, 1.0, 1.0};
    int np = 1;
    if (!uni) {
        const double ieps = L * inv_fast(fr.dist);
        mu = asinh(ieps);
        const double imu = inv_fast(mu);
        const double s4 = asinh(4.0) * imu, s01 = asinh(0.1 * ieps) * imu;
        np = 1;
        cuts[1] = 1.0;
        cuts[2] = 1.0;
        if (s01 > s4) { cuts[1] = s4; cuts[2] = s01; np = 3; }
        else if (s4 < 1.0) { cuts[1] = s4; np = 2; }
    }
    const double tol_piece = cr != 0.0 ? (second ? tol_f1 : tol_f) * inv_fast(fabs(cr) * np) : INFINITY;
    const double a = cuts[p], b = cuts[p + 1];
    double tval = 0.0, te = 0.0, trnd = 0.0;
    bool tovf = false;
    unsigned long long pend = wv.ballot(has && cr != 0.0 && p < np);
    long long evals = 0;
    const int g = ln >> 4, i = ln & 15;
    // this lane's node of the radial rule: abscissa, Kronrod and Gauss weights
    const double xr_i = Q.xr[i < kGKr ? i : 0];
    const double wr_i = i < kGKr ? Q.wr[i] : 0.0;
    const double gr_i = i < kGKr && (i & 1) ? Q.gr[i >> 1] : 0.0;
#pragma unroll 1
    for (int l = 0; l <= kRadialLevels && pend; ++l) {
        const int nsub = 1 << l;
        const int nra = __builtin_popcountll(pend) << l;
        if ((pend >> ln) & 1) {
            tval = 0.0;
            te = 0.0;
            trnd = 0.0;
        }
        // lane k: the lane of the k-th pending task, found once per level
        const int kpos = ln < __builtin_popcountll(pend) ? kth_bit(pend, ln) : 0;
        // this lane's rank among the pending tasks (if it holds one)
        const bool own = (pend >> ln) & 1;
        const int rank = __builtin_popcountll(pend & ((1ull << ln) - 1));
#pragma unroll 1
        for (int r0 = 0; r0 < nra; r0 += 4) {
            const int ra = r0 + g;
            const bool vra = ra < nra;
            const int task = wv.shfl(kpos, vra ? ra >> l : 0);
            const double ta = wv.shfl(a, task), tb = wv.shfl(b, task);
            const double tru = wv.shfl(ru, task), trv = wv.shfl(rv, task);
            const double teps = wv.shfl(eps, task), tmu = wv.shfl(mu, task);
            const int tuni = wv.shfl((int)uni, task);
            const double w = (tb - ta) * ldexp(1.0, -l);   // / nsub, exactly
            const double xa = ta + (ra & (nsub - 1)) * w;
            const bool node = vra && i < kGKr;
            double fx = 0.0, nz = 0.0;
            if (node) {
                const double x = xa + w * xr_i;
                double tau, jac;
                if (tuni) {
                    tau = x;
                    jac = 1.0;
                } else {
                    // sinh and cosh from one expm1: e - 1/e = em (1 + 1/e)
                    const double em = expm1(tmu * x), ie = inv_fast(1.0 + em);
                    tau = teps * 0.5 * (em + em * ie);
                    jac = teps * tmu * 0.5 * (1.0 + em + ie);
                }
                HomEval ev;
                hom_eval(h, fr.cu + tau * tru, fr.cv + tau * trv, qx, qy, qz, ev);
                double rs;
                fx = jac * tau * density(ev, &rs);
                nz = fabs(fx) * (1.0 + qnorm * fabs(ev.W) * rs);
            }
            const double wk = node ? wr_i : 0.0;
            const double wg = node ? gr_i : 0.0;
            const double K = sum16(wv, wk * fx);
            const double G = sum16(wv, wg * fx);
            const double asc = sum16(wv, wk * fabs(fx - K));
            const double noise = sum16(wv, wk * nz);
            const double pval = w * K, perr = gk_error(w * K, w * G, w * asc), prnd = gk_round(w * noise);
            if (l == 0) {
                // one part per task: the task of rank r0 + g takes group g's
                // sums, all four groups at once
                const int kk = rank - r0;
                const bool mine = own && kk >= 0 && kk < 4;
                const int src = 16 * (mine ? kk : 0);
                const double v1 = wv.shfl(pval, src), e1 = wv.shfl(perr, src), r1 = wv.shfl(prnd, src);
                if (mine) {
                    tval += v1;
                    te += e1;
                    trnd += r1;
                }
            } else {
#pragma unroll 1
                for (int gg = 0; gg < 4 && r0 + gg < nra; ++gg) {
                    const int tk = wv.bcast(task, 16 * gg);
                    const double v1 = wv.bcast(pval, 16 * gg), e1 = wv.bcast(perr, 16 * gg), r1 = wv.bcast(prnd, 16 * gg);
                    if (ln == tk) {
                        tval += v1;
                        te += e1;
                        trnd += r1;
                    }
                }
            }
        }
        evals += (long long)nra * kGKr;
        B.spent += (long long)nra * kGKr;
        bool again = false;
        if (((pend >> ln) & 1) && !(te <= fmax(tol_piece, trnd))) {
            if (l == kRadialLevels || B.spent > kMaxEvalsPerPair) tovf = true;
            else again = true;
        }
        pend = wv.ballot(again);
    }
    if (wv.ballot(tovf)) ovf = true;
    if (count && ln == 0) ctr_add(ctr, GWN_C_PIECES, evals);
    // node m (lane m) adds its pieces in order
    double H = 0.0, eH = 0.0, rH = 0.0;
#pragma unroll
    for (int pp = 0; pp < 3; ++pp) {
        const int src = imin(3 * ln + pp, 63);
        const double v1 = wv.shfl(tval, src), e1 = wv.shfl(te, src), r1 = wv.shfl(trnd, src);
        if (pp < wv.shfl(np, src)) {
            H += v1;
            eH += e1;
            rH += r1;
        }
    }
    const double crm = wv.shfl(cr, imin(3 * ln, 63));
    f = 0.0;
    ef = 0.0;
    rf = 0.0;
    if (ln < M && crm != 0.0) {
        f = crm * H;
        ef = fabs(crm) * eH;
        rf = fabs(crm) * rH;
    }
}

// The graded panels of one boundary curve on [a, b] (from `c`, first width
// h0), each integrated to its share of the leaf's budget B: a panel whose
// estimate -- its Kronrod estimate plus the radial estimates of its nodes --
// exceeds its share is integrated again as 2, 4, ... equal sub-panels.
// Panels go in pairs at the first level: one pass over the wave takes the
// nodes of a panel and of the next (18 outer nodes instead of 9, so fuller
// rounds and half the passes), the next panel's radial tolerance from the
// share it would get if this one spent all of its own, which is no larger
// than the share it gets (so its estimate is tested against its own share
// when its turn comes).  Near field 51.7 -> 49.2 ms on the bodies grid, CAD
// assembly 787 -> 733 ms per launch, the same integrand count and errors.
template <class Wv, class CtrT>
GWN_HD inline double graded_panels(const Wv &wv, const QuadTables &Q, const double *__restrict__ h, const Curve2 &cv,
                                   const NearFrame &fr, double qx, double qy, double qz, double qnorm, double a,
                                   double b, double c, double h0, Budget &B, bool &ovf, CtrT &ctr, bool count)
{
    // Kronrod sums of the nodes of chunk j of the last outer_values call,
    // scaled by the chunk width sw: value, estimate, rounding level
    auto chunk_sums = [&](double f, double ef, double rf, int j, double sw, double &val, double &e, double &rnd) {
        double K = 0.0, G = 0.0, fabs_sum = 0.0, erad = 0.0, rrad = 0.0;
        double fv[kGKo];
#pragma unroll
        for (int i = 0; i < kGKo; ++i) {
            const double fx = wv.bcast(f, kGKo * j + i);
            fv[i] = fx;
            K += Q.wo[i] * fx;
            fabs_sum += Q.wo[i] * fabs(fx);
            erad += Q.wo[i] * wv.bcast(ef, kGKo * j + i);
            rrad += Q.wo[i] * wv.bcast(rf, kGKo * j + i);
        }
#pragma unroll
        for (int i = 0; i < kOuterN; ++i) G += Q.go[i] * fv[2 * i + 1];
        double asc = 0.0;
#pragma unroll
        for (int i = 0; i < kGKo; ++i) asc += Q.wo[i] * fabs(fv[i] - K);
        val += sw * K;
        e += gk_error(sw * K, sw * G, sw * asc) + sw * erad;
        rnd += gk_round(sw * fabs_sum) + sw * rrad;
    };
    double total = 0.0;
#pragma unroll 1
    for (int side = 0; side < 2; ++side) {
        const double end = side == 0 ? b : a;
        double lo = c, w = h0;
        // first-level results of the next panel, computed with this one
        bool ahead = false;
        double ahead_val = 0.0, ahead_e = 0.0, ahead_rnd = 0.0;
#pragma unroll 1
        for (int k = 0; k < kMaxPanelsSide; ++k) {
            if (side == 0 ? lo >= end : lo <= end) break;
            double hi = side == 0 ? fmin(end, lo + w) : fmax(end, lo - w);
            if (k == kMaxPanelsSide - 1) hi = end;
            const double pa = fmin(lo, hi), pb = fmax(lo, hi), len = pb - pa;
            const double share = fmax(B.rem, 0.0) / (B.left > 0 ? B.left : 1);
            double val = 0.0, e = 0.0, rnd = 0.0;
            if (ahead) {
                // computed with the previous panel at a share no larger than
                // this one's
                val = ahead_val;
                e = ahead_e;
                rnd = ahead_rnd;
                ahead = false;
            } else {
                // the first level of this panel and of the next one share one
                // pass over the wave: the next panel's radial tolerance takes
                // the share it would get if this one spent all of its own
                const double lo1 = hi, w1 = k > 0 ? 2.0 * w : w;
                const bool pair = k + 1 < kMaxPanelsSide && !(side == 0 ? lo1 >= end : lo1 <= end);
                double pa1 = 0.0, len1 = 0.0, share1 = 0.0;
                if (pair) {
                    double hi1 = side == 0 ? fmin(end, lo1 + w1) : fmax(end, lo1 - w1);
                    if (k + 1 == kMaxPanelsSide - 1) hi1 = end;
                    pa1 = fmin(lo1, hi1);
                    len1 = fmax(lo1, hi1) - pa1;
                    share1 = fmax(B.rem - share, 0.0) / (B.left - 1 > 0 ? B.left - 1 : 1);
                }
                double f, ef, rf;
                outer_values(wv, Q, h, cv, fr, qx, qy, qz, qnorm, pa, len, 0, pair ? 2 : 1, 0.5 * share / len, B, ovf,
                             ctr, count, f, ef, rf, pair, pa1, len1, pair ? 0.5 * share1 / len1 : 0.0);
                chunk_sums(f, ef, rf, 0, len, val, e, rnd);
                if (pair) {
                    ahead_val = 0.0;
                    ahead_e = 0.0;
                    ahead_rnd = 0.0;
                    chunk_sums(f, ef, rf, 1, len1, ahead_val, ahead_e, ahead_rnd);
                    ahead = true;
                }
            }
            if (!(e <= fmax(share, rnd))) {
#pragma unroll 1
                for (int level = 1; level <= kOuterLevels; ++level) {
                    if (B.spent > kMaxEvalsPerPair) {
                        ovf = true;
                        break;
                    }
                    const int nsub = 1 << level;
                    const double sw = len / nsub;
                    rnd = 0.0;
                    e = 0.0;
                    val = 0.0;
#pragma unroll 1
                    for (int sp0 = 0; sp0 < nsub; sp0 += kSubPerChunk) {
                        const int nc = imin(kSubPerChunk, nsub - sp0);
                        double f, ef, rf;
                        // the radial part of the estimate stays within half
                        // the share
                        outer_values(wv, Q, h, cv, fr, qx, qy, qz, qnorm, pa, sw, sp0, nc, 0.5 * share / len, B, ovf,
                                     ctr, count, f, ef, rf);
#pragma unroll 1
                        for (int j = 0; j < nc; ++j) chunk_sums(f, ef, rf, j, sw, val, e, rnd);
                    }
                    if (e <= fmax(share, rnd)) break;
                    if (level == kOuterLevels) {
                        ovf = true;
                        break;
                    }
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

// Grading centres of one boundary curve, each with the width of its first
// panel: the point of the curve nearest c, and, for a strongly anisotropic
// metric at c, the crossings of the ray from c along the weak direction;
// sorted, and merged where they lie within each other's first panel.
// 17 samples of the curve locate them; 64-point multisection refines them
// (kMultisect rounds for a crossing, kMultimin for the nearest point).
constexpr int kMultisect = 8;   // width (1/16) / 65^8 ~ 2e-16
constexpr int kMultimin = 6;    // width (1/8) / 31.5^6 ~ 1e-10

template <class Wv>
GWN_HD inline int curve_centres(const Wv &wv, const Curve2 &cv, const NearFrame &fr, double centres[3],
                                double widths[3])
{
    compiler_fence();
    const int ln = wv.lane();
    int nc = 0;
    double d2 = INFINITY, sd;
    {
        const int k = ln < 16 ? ln : 16;
        double u, v, du, dv;
        curve_eval(cv, k / 16.0, u, v, du, dv);
        if (ln <= 16) d2 = (u - fr.cu) * (u - fr.cu) + (v - fr.cv) * (v - fr.cv);
        if (!(d2 < INFINITY)) d2 = INFINITY;
        sd = (u - fr.cu) * fr.ew_v - (v - fr.cv) * fr.ew_u;
    }
    int best = ln;
    {
        double bd = d2;
        argmin64(wv, bd, best);
    }
    const double prev = wv.shfl(sd, ln > 0 ? ln - 1 : 0);
    unsigned long long cm = wv.ballot(fr.anis < 0.5 && ln >= 1 && ln <= 16 &&
                                      ((prev < 0.0 && sd >= 0.0) || (prev > 0.0 && sd <= 0.0)));
#pragma unroll 1
    while (cm && nc < 2) {
        const int k = __builtin_ctzll(cm);
        cm &= cm - 1;
        double lo = (k - 1) / 16.0, hi = k / 16.0, flo = wv.bcast(sd, k - 1);
#pragma unroll 1
        for (int it = 0; it < kMultisect; ++it) {
            double mu, mv, mdu, mdv;
            curve_eval(cv, lo + (hi - lo) * (ln + 1) / 65.0, mu, mv, mdu, mdv);
            const double fm = (mu - fr.cu) * fr.ew_v - (mv - fr.cv) * fr.ew_u;
            // the first point past the sign change (64: none, the root lies
            // beyond the last point)
            const unsigned long long dm = wv.ballot((flo < 0.0) != (fm < 0.0));
            const int i = dm ? __builtin_ctzll(dm) : 64;
            const double fb = wv.bcast(fm, i > 0 ? i - 1 : 0);
            const double nlo = i > 0 ? lo + (hi - lo) * i / 65.0 : lo;
            const double nhi = i < 64 ? lo + (hi - lo) * (i + 1) / 65.0 : hi;
            if (i > 0) flo = fb;
            lo = nlo;
            hi = nhi;
        }
        const double tr = 0.5 * (lo + hi);
        double ru, rv, rdu, rdv;
        curve_eval(cv, tr, ru, rv, rdu, rdv);
        const double rr = sqrt((ru - fr.cu) * (ru - fr.cu) + (rv - fr.cv) * (rv - fr.cv));
        const double speed = sqrt(rdu * rdu + rdv * rdv);
        centres[nc] = tr;
        widths[nc++] = speed > 0.0 ? fmax(fr.anis * rr, fr.dparam) / speed : 1.0;
    }
    {
        auto near2 = [&](double t) {
            double u, v, du, dv;
            curve_eval(cv, t, u, v, du, dv);
            return (u - fr.cu) * (u - fr.cu) + (v - fr.cv) * (v - fr.cv);
        };
        double a = fmax(best - 1, 0) / 16.0, b = fmin(best + 1, 16) / 16.0;
#pragma unroll 1
        for (int it = 0; it < kMultimin; ++it) {
            double fm = near2(a + (b - a) * ln / 63.0);
            if (!(fm < INFINITY)) fm = INFINITY;
            int im = ln;
            argmin64(wv, fm, im);
            const int i0 = im > 0 ? im - 1 : 0, i1 = im < 63 ? im + 1 : 63;
            const double na = a + (b - a) * i0 / 63.0, nb = a + (b - a) * i1 / 63.0;
            a = na;
            b = nb;
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
    int m = 0;   // merge centres within each other's first panel (keep the finer)
    for (int k = 0; k < nc; ++k) {
        if (m > 0 && centres[k] - centres[m - 1] <= fmax(widths[k], widths[m - 1])) {
            if (widths[k] < widths[m - 1]) { centres[m - 1] = centres[k]; widths[m - 1] = widths[k]; }
            continue;
        }
        centres[m] = centres[k];
        widths[m] = widths[k];
        ++m;
    }
    return m;
}

// Outer integral over one boundary curve (count_only: the number of its
// initial panels, for the budget).  Curve `slot` below kCurveCache keeps
// its grading centres in the shared state from the counting pass to the
// integration pass.
template <class Wv, class CtrT>
GWN_HD inline double curve_contribution(const Wv &wv, const QuadTables &Q, const double *__restrict__ h,
                                        const Curve2 &cv, const NearFrame &fr, double qx, double qy, double qz,
                                        bool count_only, Budget &B, bool &ovf, CtrT &ctr, bool count, NearShared &sh,
                                        int slot)
{
    double centres[3], widths[3];
    int nc;
    if (!count_only && slot < kCurveCache) {
        nc = sh.ncen[slot];
        for (int k = 0; k < 3; ++k) {
            centres[k] = sh.cen[slot][k];
            widths[k] = sh.wid[slot][k];
        }
    } else {
        nc = curve_centres(wv, cv, fr, centres, widths);
        if (slot < kCurveCache) {
            sh.ncen[slot] = nc;
            for (int k = 0; k < 3; ++k) {
                sh.cen[slot][k] = centres[k];
                sh.wid[slot][k] = widths[k];
            }
        }
    }
    // first panel at most 1/4 of the curve; 1/8 at a collapsed edge (pole),
    // where the integrand is near-singular along the whole edge
    const double first = fr.anis < 0.2 ? 0.125 : 0.25;
    double total = 0.0;
    const double qnorm = sqrt(qx * qx + qy * qy + qz * qz);
#pragma unroll 1
    for (int k = 0; k < nc; ++k) {
        const double lo = k == 0 ? 0.0 : 0.5 * (centres[k - 1] + centres[k]);
        const double hi = k == nc - 1 ? 1.0 : 0.5 * (centres[k] + centres[k + 1]);
        if (count_only) total += count_panels(lo, hi, centres[k], fmin(widths[k], first));
        else total += graded_panels(wv, Q, h, cv, fr, qx, qy, qz, qnorm, lo, hi, centres[k], fmin(widths[k], first),
                                    B, ovf, ctr, count);
    }
    return total;
}

// Start grid of the foot-point search: kFootGrid^2 samples of the square,
// kFootRounds rounds of 64 lanes.  The second start is the best sample
// outside the first's neighbourhood of +-kFootExcl samples (+-1/4).
constexpr int kFootGrid = 17;
constexpr int kFootRounds = (kFootGrid * kFootGrid + 63) / 64;
constexpr int kFootExcl = (kFootGrid - 1) / 4;
constexpr double kFootStep = 1.0 / (kFootGrid - 1);

// Projected Gauss-Newton refinement of two starts at once: lanes 0-31
// refine start 0 within the rectangle rect[0] = (u0, u1, v0, v1), lanes
// 32-63 start 1 within rect[1]; the step is halved up to 7 times until the
// distance falls, the 8 step lengths tried on 8 lanes at once (the longest
// that lowers the distance is taken).  u, v, d (squared distance) are the
// starts on entry and the results on return, the same on every lane.
template <class Wv>
GWN_HD inline void gauss_newton2(const Wv &wv, const double *__restrict__ h, double qx, double qy, double qz,
                                 double u2[2], double v2[2], double d2[2], const double rect[2][4])
{
    const int ln = wv.lane();
    const int half = ln >> 5, hl = ln & 31;
    double u = u2[half], v = v2[half], d = d2[half];
    const double lu = rect[half][0], hu = rect[half][1], lv = rect[half][2], hv = rect[half][3];
    bool active = d < INFINITY;
#pragma unroll 1
    for (int it = 0; it < 16; ++it) {
        if (!wv.ballot(active)) break;
        HomEval e;
        double r[3], Su[3], Sv[3];
        hom_eval(h, u, v, qx, qy, qz, e);
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
        double nu = u, nv = v, nd = d;
        bool ok = false;
        if (active && hl < 8) {
            const double step = 1.0 / (1 << hl);
            nu = fmin(hu, fmax(lu, u + step * du));
            nv = fmin(hv, fmax(lv, v + step * dv));
            HomEval f;
            hom_eval(h, nu, nv, qx, qy, qz, f);
            nd = (f.A[0] * f.A[0] + f.A[1] * f.A[1] + f.A[2] * f.A[2]) / (f.W * f.W);
            ok = nd < d;
        }
        const unsigned hm = (unsigned)(wv.ballot(ok) >> (32 * half)) & 0xffu;
        const int s = hm ? __builtin_ctz(hm) : 0;
        const double su = wv.shfl(nu, 32 * half + s), sv = wv.shfl(nv, 32 * half + s), sdd = wv.shfl(nd, 32 * half + s);
        if (active) {
            if (hm) {
                u = su;
                v = sv;
                d = sdd;
                if ((1.0 / (1 << s)) * (fabs(du) + fabs(dv)) < 1e-15) active = false;
            } else {
                active = false;
            }
        }
    }
    for (int k = 0; k < 2; ++k) {
        u2[k] = wv.bcast(u, 32 * k);
        v2[k] = wv.bcast(v, 32 * k);
        d2[k] = wv.bcast(d, 32 * k);
    }
}

// Best of kFootGrid^2 samples of the rectangle rect = (u0, u1, v0, v1) for
// the point nearest q: its parameters and squared distance, the same on
// every lane.
template <class Wv>
GWN_HD inline void best_sample(const Wv &wv, const double *__restrict__ h, double qx, double qy, double qz,
                               const double rect[4], double &u, double &v, double &d)
{
    const int ln = wv.lane();
    constexpr int NS = kFootGrid * kFootGrid;
    double bd = INFINITY;
    int bk = ln;
#pragma unroll 1
    for (int r = 0; r < kFootRounds; ++r) {
        const int k = ln + 64 * r;
        if (k < NS) {
            const int i = k / kFootGrid, j = k - kFootGrid * (k / kFootGrid);
            HomEval e;
            hom_eval(h, rect[0] + (rect[1] - rect[0]) * (kFootStep * i), rect[2] + (rect[3] - rect[2]) * (kFootStep * j),
                     qx, qy, qz, e);
            const double d2 = (e.A[0] * e.A[0] + e.A[1] * e.A[1] + e.A[2] * e.A[2]) / (e.W * e.W);
            if (d2 < bd) { bd = d2; bk = k; }
        }
    }
    argmin64(wv, bd, bk);
    const int i = bk / kFootGrid, j = bk - kFootGrid * (bk / kFootGrid);
    u = rect[0] + (rect[1] - rect[0]) * (kFootStep * i);
    v = rect[2] + (rect[3] - rect[2]) * (kFootStep * j);
    d = bd;
}

// Foot point of q on the untrimmed patch: the best of kFootGrid^2 samples
// and the best one outside its neighbourhood (the distance can have several
// local minima on strongly non-uniform or folded patches), both refined by
// gauss_newton2 over the whole square.
// Returns the squared distance and (bu, bv) the parameters; (ou, ov, od)
// the other converged minimum (possibly the same point).
template <class Wv>
GWN_HD inline double foot_point3d(const Wv &wv, const double *__restrict__ h, double qx, double qy, double qz,
                                  double &bu, double &bv, double &ou, double &ov, double &od)
{
    const int ln = wv.lane();
    constexpr int NS = kFootGrid * kFootGrid;
    double dk[kFootRounds];
#pragma unroll
    for (int r = 0; r < kFootRounds; ++r) dk[r] = INFINITY;
#pragma unroll 1
    for (int r = 0; r < kFootRounds; ++r) {
        const int k = ln + 64 * r;
        if (k < NS) {
            const int i = k / kFootGrid, j = k - kFootGrid * (k / kFootGrid);
            HomEval e;
            hom_eval(h, kFootStep * i, kFootStep * j, qx, qy, qz, e);
            const double d2 = (e.A[0] * e.A[0] + e.A[1] * e.A[1] + e.A[2] * e.A[2]) / (e.W * e.W);
#pragma unroll
            for (int t = 0; t < kFootRounds; ++t)
                if (t == r) dk[t] = d2 < INFINITY ? d2 : INFINITY;
        }
    }
    // best sample (the first in grid order on ties)
    double d1 = INFINITY;
    int k1 = ln;
#pragma unroll
    for (int r = 0; r < kFootRounds; ++r)
        if (dk[r] < d1) { d1 = dk[r]; k1 = ln + 64 * r; }
    argmin64(wv, d1, k1);
    const int i1 = k1 / kFootGrid, j1 = k1 - kFootGrid * (k1 / kFootGrid);
    double d2b = INFINITY;
    int k2 = ln;
#pragma unroll
    for (int r = 0; r < kFootRounds; ++r) {
        const int k = ln + 64 * r, i = k / kFootGrid, j = k - kFootGrid * (k / kFootGrid);
        if ((abs(i - i1) > kFootExcl || abs(j - j1) > kFootExcl) && dk[r] < d2b) { d2b = dk[r]; k2 = k; }
    }
    argmin64(wv, d2b, k2);
    const int i2 = k2 / kFootGrid, j2 = k2 - kFootGrid * (k2 / kFootGrid);
    double u[2] = {kFootStep * i1, kFootStep * i2}, v[2] = {kFootStep * j1, kFootStep * j2}, d[2] = {d1, d2b};
    const double sq[2][4] = {{0.0, 1.0, 0.0, 1.0}, {0.0, 1.0, 0.0, 1.0}};
    gauss_newton2(wv, h, qx, qy, qz, u, v, d, sq);
    bu = u[0];
    bv = v[0];
    ou = u[1];
    ov = v[1];
    od = d[1];
    if (d[1] < d[0]) { bu = u[1]; bv = v[1]; ou = u[0]; ov = v[0]; od = d[0]; return d[1]; }
    return d[0];
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
    // to the major axis, at angle theta = atan2(2 gb, ga - gc) / 2, whose
    // sine and cosine come from the half-angle identities (the branch on the
    // sign of ga - gc keeps them accurate; stable also when gb is pure
    // roundoff)
    const double *Su = fr.Su, *Sv = fr.Sv;
    const double ga = Su[0] * Su[0] + Su[1] * Su[1] + Su[2] * Su[2];
    const double gb = Su[0] * Sv[0] + Su[1] * Sv[1] + Su[2] * Sv[2];
    const double gc = Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2];
    const double tr = 0.5 * (ga + gc), df = sqrt(fmax(0.25 * (ga - gc) * (ga - gc) + gb * gb, 0.0));
    const double l2 = tr + df, l1 = fmax(tr - df, 0.0);
    const double x2 = ga - gc, y2 = 2.0 * gb, r2 = 2.0 * df;   // r2 = |(x2, y2)|
    double ct = 1.0, st = 0.0;
    if (r2 > 0.0) {
        if (x2 >= 0.0) {
            ct = sqrt(0.5 * (1.0 + x2 / r2));
            st = y2 / (2.0 * r2 * ct);
        } else {
            st = copysign(sqrt(0.5 * (1.0 - x2 / r2)), y2);
            ct = y2 / (2.0 * r2 * st);
        }
    }
    fr.ew_u = -st;
    fr.ew_v = ct;
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
// Called by all 64 lanes of a wave with the same arguments; every lane
// returns the same value and ovf.
template <bool COUNT, class Wv, class CtrT>
GWN_HD inline double near3d(const Wv &wv, const QuadTables &Q, const Prim3 *__restrict__ P,
                            const Trim3 *__restrict__ trims, double qx, double qy, double qz, double eps_on,
                            double tol, bool &ovf, CtrT &ctr, NearShared &sh)
{
    const double *__restrict__ h = P->h;
    const int nt = P->trim_count;
    double *__restrict__ ycr = sh.ycr;
    const Trim3 *__restrict__ tr = trims + P->trim_begin;
    double bu = 0.5, bv = 0.5, ou = 0.5, ov = 0.5, od = INFINITY, bd = INFINITY;
    double mean = 0.0;
    int sides = 1;
    double nrm[3] = {0.0, 0.0, 0.0};
    const double q0[3] = {qx, qy, qz};
    // step 0 finds the foot point of q; steps 1 .. sides integrate about q
    // itself, or about q + delta n and q - delta n when q is on the surface
#pragma unroll 1
    for (int step = 0; step <= sides; ++step) {
        if (step > 0 && sides == 2) {
            qx = q0[0] + (step == 1 ? nrm[0] : -nrm[0]);
            qy = q0[1] + (step == 1 ? nrm[1] : -nrm[1]);
            qz = q0[2] + (step == 1 ? nrm[2] : -nrm[2]);
        }
        if (step == 0 || sides == 2) bd = foot_point3d(wv, h, qx, qy, qz, bu, bv, ou, ov, od);
        if (step == 0) {
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
            continue;
        }
        // Two near-singular peaks are resolved apart when the second minimum
        // is no farther from q than twice the minima's separation in space,
        // or when the minima lie far apart in parameter space compared with
        // the peaks' widths there (distance / largest singular value of the
        // Jacobian): a fold brings distant parameters close to q.
        bool split = false;
        if (fabs(ou - bu) + fabs(ov - bv) > 0.05 && od < INFINITY) {
            double p[3] = {0.0, 0.0, 0.0}, sep2 = 0.0, width = 0.0;
#pragma unroll 1
            for (int k = 0; k < 2; ++k) {
                HomEval e;
                double r[3], Su[3], Sv[3];
                hom_eval(h, k ? ou : bu, k ? ov : bv, qx, qy, qz, e);
                euclid(e, r, Su, Sv);
                for (int a = 0; a < 3; ++a) {
                    if (k) sep2 += (r[a] - p[a]) * (r[a] - p[a]); else p[a] = r[a];
                }
                const double ga = Su[0] * Su[0] + Su[1] * Su[1] + Su[2] * Su[2];
                const double gb = Su[0] * Sv[0] + Su[1] * Sv[1] + Su[2] * Sv[2];
                const double gc = Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2];
                const double l2 = 0.5 * (ga + gc) + sqrt(fmax(0.25 * (ga - gc) * (ga - gc) + gb * gb, 0.0));
                if (l2 > 0.0) width = fmax(width, sqrt(k ? od : bd) / sqrt(l2));
            }
            const double psep = sqrt((ou - bu) * (ou - bu) + (ov - bv) * (ov - bv));
            split = od < 4.0 * sep2 || psep > 8.0 * width;
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
        int ncr = 0;
        if (split && nt > 0) {
#pragma unroll 1
            for (int k = 0; k < nt && split; ++k) {
                Curve2 cv;
                for (int m = 0; m < 9; ++m) cv.h[m] = tr[k].h[m];
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
        // curves: first the panels are counted (pass 0), then integrated.
        // The boundary of a part: the square's (or its half's) four edges;
        // else the trim curves, each cut into up to three pieces when the
        // leaf is split, and the stretches of the cut line.
        const int nparts = split ? 2 : 1;
        const int ncurves = nt == 0 ? 4 : split ? 3 * nt + ncr / 2 : nt;
        // each part is integrated about its own foot point, the point of the
        // part's rectangle nearest q: the best of a sample grid of the
        // rectangle or the part's minimum, refined within the rectangle (the
        // nearest point of a part may lie on the cut, and the part's minimum
        // may be a constrained one on the square's edge)
        double pu[2] = {bu, ou}, pv[2] = {bv, ov}, pd[2] = {bd, od};
        bool lows[2] = {true, true};
        double prect[2][4] = {{0.0, 1.0, 0.0, 1.0}, {0.0, 1.0, 0.0, 1.0}};
        if (split) {
#pragma unroll 1
            for (int part = 0; part < 2; ++part) {
                lows[part] = (cut_u ? pu[part] : pv[part]) < cut;
                if (cut_u) prect[part][lows[part] ? 1 : 0] = cut;
                else prect[part][lows[part] ? 3 : 2] = cut;
                double su, sv, sd;
                best_sample(wv, h, qx, qy, qz, prect[part], su, sv, sd);
                if (sd < pd[part]) { pu[part] = su; pv[part] = sv; pd[part] = sd; }
            }
            gauss_newton2(wv, h, qx, qy, qz, pu, pv, pd, prect);
        }
        Budget B{tol, 0, 0};
        double total = 0.0;
#pragma unroll 1
        for (int pass = 0; pass < 2; ++pass) {
#pragma unroll 1
            for (int part = 0; part < nparts; ++part) {
                const double cu = pu[part], cv = pv[part], d2 = pd[part];
                const double u0 = prect[part][0], u1 = prect[part][1], v0 = prect[part][2], v1 = prect[part][3];
                const bool low = lows[part];
                sh.fr = near_frame(h, cu, cv, d2, qx, qy, qz, eps_on);
                compiler_fence();
                const NearFrame &fr = sh.fr;
                // stretches of the cut line inside the region, walked with this
                // half on the left: +y for the low half of a u cut and the high
                // half of a v cut
                const bool up = (dir == 0) == low;
#pragma unroll 1
                for (int it = 0; it < ncurves; ++it) {
                    Curve2 crv;
                    if (nt == 0) {
                        crv = rect_edge(u0, u1, v0, v1, it);
                    } else if (!split) {
                        for (int m = 0; m < 9; ++m) crv.h[m] = tr[it].h[m];
                    } else if (it < 3 * nt) {
                        const int k = it / 3, j = it - 3 * (it / 3);
                        Curve2 whole;
                        for (int m = 0; m < 9; ++m) whole.h[m] = tr[k].h[m];
                        double r[2];
                        int nr = 0;
                        cut_roots(whole, dir, cut, r, nr);
                        if (j > nr) continue;
                        const double t0 = j == 0 ? 0.0 : r[j - 1], t1 = j == nr ? 1.0 : r[j];
                        double u, v, du, dv;
                        curve_eval(whole, 0.5 * (t0 + t1), u, v, du, dv);
                        if (((dir == 0 ? u : v) < cut) != low) continue;
                        crv = nr ? sub_curve(whole, t0, t1) : whole;
                    } else {
                        const int i = 2 * (it - 3 * nt);
                        const double ya = ycr[i], yb = -ycr[i + 1] - 2.0;
                        const double y0 = up ? ya : yb, y1 = up ? yb : ya;
                        crv = dir == 0 ? rect_edge(cut, cut, y0, y1, 1) : rect_edge(y0, y1, cut, cut, 0);
                    }
                    const double r = curve_contribution(wv, Q, h, crv, fr, qx, qy, qz, pass == 0, B, ovf, ctr, COUNT,
                                                        sh, part * ncurves + it);
                    if (pass == 0) B.left += (int)r; else total += r;
                }
            }
        }
        mean += total;
    }
    return mean / sides;
}

}  // namespace gwn
