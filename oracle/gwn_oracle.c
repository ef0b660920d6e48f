/*
 * CPU oracle for the generalized winding number (GWN) of rational Bezier
 * curves (2D) and trimmed rational bicubic patches (3D).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the engine may call this file; only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * do.  It shares no code, header or table with the GPU engine.
 *
 * What it computes is the plain definition of the GWN (the paper's "direct
 * evaluation", Sec. 4.2): the sum over EVERY input primitive, with no
 * subdivision, no hierarchy and no far-field approximation, of
 *
 *   2D (Eq. gwn_sum):   w_i(q) = (1/2pi) * total signed angle swept by C_i - q
 *   3D (Eq. gwn_sum / gwn_greens):
 *                       w_i(q) = (1/4pi) * integral over the visible part of
 *                                S_i of (x - q).n / |x - q|^3 dA
 *
 * in FP64.  Quadrature is adaptive Gauss-Legendre (n = 10 nodes per panel,
 * error estimated by comparing a panel with its two halves), started from
 * panels graded geometrically toward the point of the primitive closest to q,
 * so that the near-singular peak of width ~dist(q, primitive) is always
 * resolved.
 *
 * Rational geometry is used in homogeneous form: with H(t) = sum B_i(t)
 * (w_i P_i, w_i) = (H_x, W) and A = H_x - q W, the angle of C - q equals the
 * angle of A (W > 0), so d(theta)/dt = cross(A, A') / |A|^2; in 3D
 * (S - q).(S_u x S_v) / |S - q|^3 = det[A, A_u, A_v] / |A|^3.  The weights
 * cancel in both.
 *
 * Direct value on the boundary: when q lies on a primitive, that primitive's
 * integral is taken as the (absolutely convergent) integral itself, which is
 * the mean of the two one-sided limits (0.5 at smooth points of a closed
 * boundary).  When q is within eps_on of a primitive (2D: of the curve; 3D:
 * of the patch's surface over its whole parameter square), the primitive's
 * value is computed as the mean of its values at q + delta n and q - delta n,
 * with n the unit normal at the foot point and delta = 1e3 eps_on.  At a
 * point of the visible primitive that mean is the direct value; at a
 * trimmed-away point of a patch the value is continuous across the surface,
 * so the mean is the value itself.
 *
 * Non-convergence is never silent: panels that the adaptive rule accepts at
 * a work limit with an error estimate above its tolerance are counted, and
 * their estimates, scaled by the enclosing quadrature weights, give a bound
 * on the unresolved part of each value (oracle_last_unconverged,
 * oracle_last_errbound).
 *
 * Trimmed patches (3D): the visible region D of [0,1]^2 is bounded by closed
 * loops of rational trim curves (degree 1 or 2), outer loop counter-clockwise,
 * holes clockwise; an empty trim list means D = [0,1]^2.  The surface
 * integral over D is turned into line integrals over the trim curves by
 * Green's theorem in parameter space (the formulation used for the moment
 * integrals in Sec. 3.1):  integral_D g du dv = sum over trim curves of
 * integral F(u(t), v(t)) v'(t) dt, with F(u, v) = integral_0^u g(s, v) ds.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GLN 10
#define MAX_DEPTH 48
static const double PI_ = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre nodes on [-1, 1] by Newton's method on P_n (three-term     */
/* recurrence), computed once.                                               */
/* ------------------------------------------------------------------------ */
static double gl_x[GLN], gl_w[GLN];
static int gl_ready = 0;

static void gl_init(void)
{
    if (gl_ready) return;
    const int n = GLN;
    for (int i = 0; i < n; ++i) {
        double x = cos(PI_ * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        gl_x[i] = x;
        gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    gl_ready = 1;
}

/* Panels accepted only because a work limit was reached (MAX_SPLITS,
 * MAX_DEPTH, or a panel too narrow to halve in FP64) while the error
 * estimate still exceeded both acceptance tests.  Counted per thread and
 * summed over the queries of each oracle_gwn2d / oracle_gwn3d call, so that a
 * value the quadrature did not resolve is never silent. */
static _Thread_local long long tl_unconverged = 0;
static long long g_last_unconverged = 0;
/* Error bound of those panels, carried to the final value: each one adds
 * its estimate |l + r - whole| times the factor by which the enclosing
 * quadratures scale its integral (the outer Gauss weights and |v'| of the
 * nested 3D rule, tl_mult).  The panel evaluations that only serve error
 * estimates are included, so the bound is conservative.  Reported per query
 * in units of w; the largest of a call is kept. */
static _Thread_local double tl_mult = 1.0;
static _Thread_local double tl_errbound = 0.0;
static double g_last_errbound = 0.0;

typedef double (*fn1)(double, void *);

static double gl_panel(fn1 f, void *ctx, double a, double b)
{
    double c = 0.5 * (a + b), h = 0.5 * (b - a), s = 0.0;
    const double saved = tl_mult;
    for (int i = 0; i < GLN; ++i) {
        tl_mult = saved * fabs(gl_w[i] * h);
        s += gl_w[i] * f(c + h * gl_x[i], ctx);
    }
    tl_mult = saved;
    return s * h;
}

/* Adaptive Gauss-Legendre on [a, b]: a panel is accepted when it agrees
 * with the sum over its two halves to within its share (proportional to its
 * length) of the tolerance, or to `rel` relative (the roundoff level of the
 * integrand near a near-singular peak: forming H - q W loses ~|H|/|A| digits).  Work is bounded: at most
 * MAX_SPLITS bisections and a bisection depth of MAX_DEPTH per call. */
#ifndef MAX_SPLITS
#define MAX_SPLITS 2000
#endif

static double adapt(fn1 f, void *ctx, double a, double b, double tol, double rel)
{
    if (!(b > a)) return 0.0;
    double sa[MAX_DEPTH + 2], sb[MAX_DEPTH + 2], sw[MAX_DEPTH + 2];
    int sp = 0, splits = 0;
    double total = 0.0;
    sa[0] = a; sb[0] = b; sw[0] = gl_panel(f, ctx, a, b); sp = 1;
    while (sp > 0) {
        --sp;
        double pa = sa[sp], pb = sb[sp], whole = sw[sp];
        double m = 0.5 * (pa + pb);
        double l = gl_panel(f, ctx, pa, m), r = gl_panel(f, ctx, m, pb);
        double err = fabs(l + r - whole);
        double loc = tol * (pb - pa) / (b - a);
        const int ok = err <= loc || err <= rel * fabs(l + r);
        if (ok || sp >= MAX_DEPTH || splits >= MAX_SPLITS || !(m > pa && m < pb)) {
            if (!ok) {
                ++tl_unconverged;
                tl_errbound += err * tl_mult;
            }
            total += l + r;
        } else {
            ++splits;
            sa[sp] = m; sb[sp] = pb; sw[sp] = r; ++sp;
            sa[sp] = pa; sb[sp] = m; sw[sp] = l; ++sp;
        }
    }
    return total;
}

/* Integral over [a, b] on panels graded toward the points `centres` (widths
 * h0, 2 h0, 4 h0, ... moving away from each centre), each panel adaptive. */
static int cmp_dbl(const void *x, const void *y)
{
    double a = *(const double *)x, b = *(const double *)y;
    return (a > b) - (a < b);
}

#ifndef MAX_BREAKS
#define MAX_BREAKS 1024
#endif
#define UNIFORM_2D 64   /* initial uniform panels, 2D angle integral */
#define UNIFORM_3D 2    /* initial uniform panels, each 3D level */
#ifndef REL_2D
#define REL_2D 1e-12    /* relative acceptance floor of a panel, 2D */
#endif
#ifndef REL_3D
#define REL_3D 1e-10    /* relative acceptance floor of a panel, 3D */
#endif
static double graded(fn1 f, void *ctx, double a, double b, const double *centres,
                     const double *h0, int nc, double tol, int uniform, double rel)
{
    double br[MAX_BREAKS];
    int nb = 0;
    /* a uniform partition first, so that features away from the centres
     * (e.g. fast parameter speed at a sharp turn) are seen by the error
     * estimate; then the graded breakpoints */
    for (int i = 0; i <= uniform; ++i) br[nb++] = a + (b - a) * i / uniform;
    for (int k = 0; k < nc; ++k) {
        double c = centres[k], h = h0[k];
        if (!(h > 0.0)) continue;
        if (c < a) c = a;
        if (c > b) c = b;
        if (nb < MAX_BREAKS) br[nb++] = c;
        for (double off = h; nb < MAX_BREAKS - 2; off *= 2.0) {
            int any = 0;
            if (c + off < b) { br[nb++] = c + off; any = 1; }
            if (c - off > a) { br[nb++] = c - off; any = 1; }
            if (!any) break;
        }
    }
    qsort(br, nb, sizeof(double), cmp_dbl);
    double s = 0.0;
    for (int i = 0; i + 1 < nb; ++i)
        if (br[i + 1] > br[i]) s += adapt(f, ctx, br[i], br[i + 1], tol, rel);
    return s;
}

/* Bernstein basis of degree n (<= 3) and its derivative, plain formulas
 * B_i = C(n,i) t^i (1-t)^(n-i), B_i' = n (B^{n-1}_{i-1} - B^{n-1}_i). */
static void bernstein(int n, double t, double *B, double *dB)
{
    static const double binom[4][4] = {{1, 0, 0, 0}, {1, 1, 0, 0}, {1, 2, 1, 0}, {1, 3, 3, 1}};
    double s = 1.0 - t;
    double tp[4] = {1.0, t, t * t, t * t * t}, sp[4] = {1.0, s, s * s, s * s * s};
    for (int i = 0; i <= n; ++i) {
        B[i] = binom[n][i] * tp[i] * sp[n - i];
        if (dB) {
            double d = 0.0;
            if (i > 0) d += binom[n - 1][i - 1] * tp[i - 1] * sp[n - i];
            if (i < n) d -= binom[n - 1][i] * tp[i] * sp[n - 1 - i];
            dB[i] = n * d;
        }
    }
}

/* ======================================================================== */
/* 2D                                                                        */
/* ======================================================================== */
typedef struct {
    int n;                  /* degree */
    double X[4], Y[4], W[4]; /* homogeneous control points (w x, w y, w) */
    double qx, qy;
} curve2;

static void curve_eval(const curve2 *c, double t, double *Ax, double *Ay, double *W,
                       double *dAx, double *dAy, double *dW)
{
    double B[4], dB[4];
    bernstein(c->n, t, B, dB);
    double hx = 0, hy = 0, hw = 0, gx = 0, gy = 0, gw = 0;
    for (int i = 0; i <= c->n; ++i) {
        hx += B[i] * c->X[i]; hy += B[i] * c->Y[i]; hw += B[i] * c->W[i];
        gx += dB[i] * c->X[i]; gy += dB[i] * c->Y[i]; gw += dB[i] * c->W[i];
    }
    *Ax = hx - c->qx * hw; *Ay = hy - c->qy * hw; *W = hw;
    if (dAx) { *dAx = gx - c->qx * gw; *dAy = gy - c->qy * gw; *dW = gw; }
}

/* d theta / dt of the vector C(t) - q. */
static double dtheta(double t, void *ctx)
{
    const curve2 *c = (const curve2 *)ctx;
    double ax, ay, w, bx, by, bw;
    curve_eval(c, t, &ax, &ay, &w, &bx, &by, &bw);
    double r2 = ax * ax + ay * ay;
    if (r2 == 0.0) return 0.0;
    return (ax * by - ay * bx) / r2;
}

static double orient(double ax, double ay, double bx, double by, double cx, double cy)
{
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

/* Is q strictly outside the convex hull of the n+1 Euclidean points?
 * Andrew's monotone chain, then a side test against every hull edge. */
static int outside_hull(const double *px, const double *py, int m, double qx, double qy)
{
    int idx[4];
    for (int i = 0; i < m; ++i) idx[i] = i;
    for (int i = 1; i < m; ++i)
        for (int j = i; j > 0; --j) {
            int a = idx[j - 1], b = idx[j];
            if (px[a] > px[b] || (px[a] == px[b] && py[a] > py[b])) { idx[j - 1] = b; idx[j] = a; }
        }
    int hull[10], h = 0;
    for (int i = 0; i < m; ++i) {
        while (h >= 2 && orient(px[hull[h - 2]], py[hull[h - 2]], px[hull[h - 1]], py[hull[h - 1]],
                                px[idx[i]], py[idx[i]]) <= 0) --h;
        hull[h++] = idx[i];
    }
    for (int i = m - 2, lo = h + 1; i >= 0; --i) {
        while (h >= lo && orient(px[hull[h - 2]], py[hull[h - 2]], px[hull[h - 1]], py[hull[h - 1]],
                                 px[idx[i]], py[idx[i]]) <= 0) --h;
        hull[h++] = idx[i];
    }
    --h; /* last point repeats the first */
    if (h <= 1) {
        return !(px[idx[0]] == qx && py[idx[0]] == qy);
    }
    if (h == 2) { /* segment */
        double ax = px[hull[0]], ay = py[hull[0]], bx = px[hull[1]], by = py[hull[1]];
        if (orient(ax, ay, bx, by, qx, qy) != 0.0) return 1;
        double t = (qx - ax) * (bx - ax) + (qy - ay) * (by - ay);
        double L = (bx - ax) * (bx - ax) + (by - ay) * (by - ay);
        return t < 0.0 || t > L;
    }
    for (int i = 0; i < h; ++i) {
        int a = hull[i], b = hull[(i + 1) % h];
        if (orient(px[a], py[a], px[b], py[b], qx, qy) < 0.0) return 1;
    }
    return 0;
}

static double dist2_at(const curve2 *c, double t)
{
    double ax, ay, w;
    curve_eval(c, t, &ax, &ay, &w, NULL, NULL, NULL);
    return (ax * ax + ay * ay) / (w * w);
}

/* Parameter of the point of the curve closest to q: dense sampling, then
 * golden-section refinement around the best sample. */
static double closest_t(const curve2 *c)
{
    const int S = 256;
    int best = 0;
    double bd = dist2_at(c, 0.0);
    for (int k = 1; k <= S; ++k) {
        double d = dist2_at(c, (double)k / S);
        if (d < bd) { bd = d; best = k; }
    }
    double a = (best > 0 ? best - 1 : 0) / (double)S, b = (best < S ? best + 1 : S) / (double)S;
    const double g = 0.6180339887498948482;
    double x1 = b - g * (b - a), x2 = a + g * (b - a);
    double f1 = dist2_at(c, x1), f2 = dist2_at(c, x2);
    for (int it = 0; it < 200 && b - a > 1e-16; ++it) {
        if (f1 < f2) { b = x2; x2 = x1; f2 = f1; x1 = b - g * (b - a); f1 = dist2_at(c, x1); }
        else { a = x1; x1 = x2; f1 = f2; x2 = a + g * (b - a); f2 = dist2_at(c, x2); }
    }
    double t = 0.5 * (a + b);
    double d0 = dist2_at(c, 0.0), d1 = dist2_at(c, 1.0), dt = dist2_at(c, t);
    if (d0 <= dt && d0 <= d1) return 0.0;
    if (d1 <= dt) return 1.0;
    return t;
}

static double gwn_curve(const curve2 *c, double eps_on);

/* The value ON the curve is the mean of the two one-sided limits; it is
 * approximated by the mean of the values at q +- delta n, with n the unit
 * normal at the foot point and delta = 1e3 eps_on (error O(delta)). */
static double gwn_curve_onboundary(const curve2 *c, double sx, double sy, double eps_on)
{
    double L = sqrt(sx * sx + sy * sy);
    double nx = sy / L, ny = -sx / L, delta = 1e3 * eps_on;
    curve2 a = *c, b = *c;
    a.qx += delta * nx; a.qy += delta * ny;
    b.qx -= delta * nx; b.qy -= delta * ny;
    return 0.5 * (gwn_curve(&a, eps_on) + gwn_curve(&b, eps_on));
}

static double gwn_curve(const curve2 *c, double eps_on)
{
    double px[4] = {0, 0, 0, 0}, py[4] = {0, 0, 0, 0};
    for (int i = 0; i <= c->n; ++i) { px[i] = c->X[i] / c->W[i]; py[i] = c->Y[i] / c->W[i]; }
    /* Far case: q outside the control polygon's convex hull.  The curve and
     * its reversed chord form a closed loop inside the hull, so the curve
     * subtends the same angle as its chord (Sec. 3.1, chord substitution). */
    int outside = 0;
    double xmn = px[0], xmx = px[0], ymn = py[0], ymx = py[0];
    for (int i = 1; i <= c->n; ++i) {
        xmn = fmin(xmn, px[i]); xmx = fmax(xmx, px[i]);
        ymn = fmin(ymn, py[i]); ymx = fmax(ymx, py[i]);
    }
    if (c->qx < xmn || c->qx > xmx || c->qy < ymn || c->qy > ymx) outside = 1;
    else outside = outside_hull(px, py, c->n + 1, c->qx, c->qy);
    if (outside) {
        double ax = px[0] - c->qx, ay = py[0] - c->qy, bx = px[c->n] - c->qx, by = py[c->n] - c->qy;
        return atan2(ax * by - ay * bx, ax * bx + ay * by);
    }
    /* Near case: integrate d(theta)/dt on panels graded toward the closest
     * point. */
    double ts = closest_t(c);
    double ax, ay, w, bx, by, bw;
    curve_eval(c, ts, &ax, &ay, &w, &bx, &by, &bw);
    double d = sqrt(ax * ax + ay * ay) / w;
    /* Euclidean speed |C'(t*)| = |A' W - A W'| / W^2 */
    double sx = (bx * w - ax * bw) / (w * w), sy = (by * w - ay * bw) / (w * w);
    double speed = sqrt(sx * sx + sy * sy);
    if (!(speed > 0.0)) {
        for (int k = 0; k <= 16; ++k) {
            curve_eval(c, k / 16.0, &ax, &ay, &w, &bx, &by, &bw);
            sx = (bx * w - ax * bw) / (w * w); sy = (by * w - ay * bw) / (w * w);
            speed = fmax(speed, sqrt(sx * sx + sy * sy));
        }
    }
    if (d < eps_on && speed > 0.0) return gwn_curve_onboundary(c, sx, sy, eps_on);
    double h0 = fmax(d, eps_on) / speed;
    if (!(h0 > 0.0)) h0 = 1e-16;
    double size = hypot(xmx - xmn, ymx - ymn);
    double rel = fmax(REL_2D, 64.0 * 2.220446049250313e-16 * size / fmax(d, eps_on));
    return graded(dtheta, (void *)c, 0.0, 1.0, &ts, &h0, 1, 1e-14, UNIFORM_2D, rel);
}

/*
 * oracle_gwn2d: w(q_k) = sum over all curves of w_i(q_k), for k < n_q.
 *   degree[n]      curve degrees, 1..3
 *   cp_offset[n+1] CSR offsets into cp_xy / cp_w
 *   cp_xy[2*n_cp]  Euclidean control points, cp_w[n_cp] weights (> 0)
 *   q[2*n_q]       query points, out[n_q] result
 *   eps_on         absolute on-boundary distance (grading floor)
 *   nthreads       OpenMP threads (<= 0: runtime default)
 * Returns 0, or -1 for invalid input (degree out of range, weight <= 0).
 */
int oracle_gwn2d(int64_t n, const int32_t *degree, const int64_t *cp_offset, const double *cp_xy,
                 const double *cp_w, int64_t n_q, const double *q, double *out, double eps_on,
                 int nthreads)
{
    gl_init();
    for (int64_t i = 0; i < n; ++i) {
        int d = degree[i];
        if (d < 1 || d > 3 || cp_offset[i + 1] - cp_offset[i] != d + 1) return -1;
        for (int64_t k = cp_offset[i]; k < cp_offset[i + 1]; ++k)
            if (!(cp_w[k] > 0.0)) return -1;
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    long long unconv = 0;
    double worst = 0.0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : unconv) reduction(max : worst)
    for (int64_t k = 0; k < n_q; ++k) {
        tl_unconverged = 0;
        tl_errbound = 0.0;
        tl_mult = 1.0;
        double s = 0.0;
        curve2 c;
        c.qx = q[2 * k];
        c.qy = q[2 * k + 1];
        for (int64_t i = 0; i < n; ++i) {
            c.n = degree[i];
            for (int j = 0; j <= c.n; ++j) {
                int64_t o = cp_offset[i] + j;
                c.W[j] = cp_w[o];
                c.X[j] = cp_xy[2 * o] * cp_w[o];
                c.Y[j] = cp_xy[2 * o + 1] * cp_w[o];
            }
            s += gwn_curve(&c, eps_on);
        }
        out[k] = s / (2.0 * PI_);
        unconv += tl_unconverged;
        worst = fmax(worst, tl_errbound / (2.0 * PI_));
    }
    g_last_unconverged = unconv;
    g_last_errbound = worst;
    return 0;
}

/* ======================================================================== */
/* 3D                                                                        */
/* ======================================================================== */
typedef struct {
    double H[4][4][4]; /* [i (u)][j (v)][x, y, z, w] homogeneous */
    double q[3];
} patch3;

typedef struct {
    double A[3], W, Au[3], Wu, Av[3], Wv;
} peval;

static void patch_eval(const patch3 *p, double u, double v, peval *e)
{
    double Bu[4], dBu[4], Bv[4], dBv[4];
    bernstein(3, u, Bu, dBu);
    bernstein(3, v, Bv, dBv);
    double h[4] = {0, 0, 0, 0}, hu[4] = {0, 0, 0, 0}, hv[4] = {0, 0, 0, 0};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 4; ++k) {
                h[k] += Bu[i] * Bv[j] * p->H[i][j][k];
                hu[k] += dBu[i] * Bv[j] * p->H[i][j][k];
                hv[k] += Bu[i] * dBv[j] * p->H[i][j][k];
            }
    for (int k = 0; k < 3; ++k) {
        e->A[k] = h[k] - p->q[k] * h[3];
        e->Au[k] = hu[k] - p->q[k] * hu[3];
        e->Av[k] = hv[k] - p->q[k] * hv[3];
    }
    e->W = h[3]; e->Wu = hu[3]; e->Wv = hv[3];
}

/* solid-angle density in parameter space: det[A, A_u, A_v] / |A|^3 */
static double g3(const patch3 *p, double u, double v)
{
    peval e;
    patch_eval(p, u, v, &e);
    double cx = e.Au[1] * e.Av[2] - e.Au[2] * e.Av[1];
    double cy = e.Au[2] * e.Av[0] - e.Au[0] * e.Av[2];
    double cz = e.Au[0] * e.Av[1] - e.Au[1] * e.Av[0];
    double det = e.A[0] * cx + e.A[1] * cy + e.A[2] * cz;
    double r2 = e.A[0] * e.A[0] + e.A[1] * e.A[1] + e.A[2] * e.A[2];
    if (r2 == 0.0) return 0.0;
    return det / (r2 * sqrt(r2));
}

/* Euclidean point and partial derivatives */
static void patch_point(const patch3 *p, double u, double v, double S[3], double Su[3], double Sv[3])
{
    peval e;
    patch_eval(p, u, v, &e);
    for (int k = 0; k < 3; ++k) {
        double a = e.A[k] / e.W;
        S[k] = a + p->q[k];
        if (Su) {
            Su[k] = (e.Au[k] * e.W - e.A[k] * e.Wu) / (e.W * e.W);
            Sv[k] = (e.Av[k] * e.W - e.A[k] * e.Wv) / (e.W * e.W);
        }
    }
}

static double pdist2(const patch3 *p, double u, double v)
{
    double S[3];
    patch_point(p, u, v, S, NULL, NULL);
    double dx = S[0] - p->q[0], dy = S[1] - p->q[1], dz = S[2] - p->q[2];
    return dx * dx + dy * dy + dz * dz;
}

/* Foot point of q on the untrimmed patch: 16x16 samples, then projected
 * Gauss-Newton steps (clamped to the unit square) with backtracking. */
static void foot_point(const patch3 *p, double *us, double *vs)
{
    double bu = 0, bv = 0, bd = INFINITY;
    for (int i = 0; i <= 16; ++i)
        for (int j = 0; j <= 16; ++j) {
            double d = pdist2(p, i / 16.0, j / 16.0);
            if (d < bd) { bd = d; bu = i / 16.0; bv = j / 16.0; }
        }
    for (int it = 0; it < 60; ++it) {
        double S[3], Su[3], Sv[3];
        patch_point(p, bu, bv, S, Su, Sv);
        double r[3] = {S[0] - p->q[0], S[1] - p->q[1], S[2] - p->q[2]};
        double a = Su[0] * Su[0] + Su[1] * Su[1] + Su[2] * Su[2];
        double b = Su[0] * Sv[0] + Su[1] * Sv[1] + Su[2] * Sv[2];
        double c = Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2];
        double gu = Su[0] * r[0] + Su[1] * r[1] + Su[2] * r[2];
        double gv = Sv[0] * r[0] + Sv[1] * r[1] + Sv[2] * r[2];
        double det = a * c - b * b;
        double du, dv;
        if (fabs(det) > 1e-300) { du = -(c * gu - b * gv) / det; dv = -(a * gv - b * gu) / det; }
        else { du = -gu / (a + 1e-300); dv = -gv / (c + 1e-300); }
        double step = 1.0, improved = 0;
        for (int ls = 0; ls < 30; ++ls) {
            double nu = fmin(1.0, fmax(0.0, bu + step * du)), nv = fmin(1.0, fmax(0.0, bv + step * dv));
            double d = pdist2(p, nu, nv);
            if (d < bd) { bd = d; bu = nu; bv = nv; improved = 1; break; }
            step *= 0.5;
        }
        if (!improved || step * (fabs(du) + fabs(dv)) < 1e-17) break;
    }
    *us = bu;
    *vs = bv;
}

typedef struct {
    const patch3 *p;
    int far;              /* q separated from the patch: no grading needed */
    double v;             /* inner integration at fixed v */
    int n;                /* trim curve degree */
    double U[3], V[3], Wt[3]; /* homogeneous trim control points */
    double us, vs, d, su, sv; /* foot point, its distance, |S_u|, |S_v| there */
    double eps_on;
    double rel;           /* relative acceptance floor (integrand noise level) */
    double diag;          /* control-point box diagonal */
} green_ctx;

static double inner_g(double s, void *ctx)
{
    green_ctx *g = (green_ctx *)ctx;
    return g3(g->p, s, g->v);
}

/* F(u, v) = integral_0^u g(s, v) ds, graded toward the point of [0, u]
 * nearest the foot point's u. */
static double F_inner(green_ctx *g, double u, double v)
{
    if (!(u > 0.0)) return 0.0;
    g->v = v;
    if (g->far) return adapt(inner_g, g, 0.0, u, 1e-15, g->rel);
    double c = fmin(fmax(g->us, 0.0), u);
    double S[3];
    patch_point(g->p, c, v, S, NULL, NULL);
    double dx = S[0] - g->p->q[0], dy = S[1] - g->p->q[1], dz = S[2] - g->p->q[2];
    double dist = sqrt(dx * dx + dy * dy + dz * dz);
    double h0 = fmax(dist, g->eps_on) / (g->su + 1e-300);
    return graded(inner_g, g, 0.0, u, &c, &h0, 1, 1e-15, UNIFORM_3D, g->rel);
}

static void trim_eval(const green_ctx *g, double t, double *u, double *v, double *du, double *dv)
{
    double B[3], dB[3];
    bernstein(g->n, t, B, dB);
    double hu = 0, hv = 0, hw = 0, gu = 0, gv = 0, gw = 0;
    for (int i = 0; i <= g->n; ++i) {
        hu += B[i] * g->U[i]; hv += B[i] * g->V[i]; hw += B[i] * g->Wt[i];
        gu += dB[i] * g->U[i]; gv += dB[i] * g->V[i]; gw += dB[i] * g->Wt[i];
    }
    *u = hu / hw;
    *v = hv / hw;
    if (du) {
        *du = (gu * hw - hu * gw) / (hw * hw);
        *dv = (gv * hw - hv * gw) / (hw * hw);
    }
}

static double outer_f(double t, void *ctx)
{
    green_ctx *g = (green_ctx *)ctx;
    double u, v, du, dv;
    trim_eval(g, t, &u, &v, &du, &dv);
    if (dv == 0.0) return 0.0;
    green_ctx local = *g;
    const double saved = tl_mult;
    tl_mult = saved * fabs(dv);
    const double F = F_inner(&local, u, v);
    tl_mult = saved;
    return F * dv;
}

/* Contribution of one trim curve: graded toward the parameters where the
 * curve crosses v = v* and toward its point nearest (u*, v*). */
static double trim_contribution(green_ctx *g)
{
    if (g->far) return adapt(outer_f, g, 0.0, 1.0, 1e-14, g->rel);
    double centres[8], h0[8];
    int nc = 0;
    const int S = 64;
    double prev_f = 0, prev_t = 0;
    double best_t = 0, best_d = INFINITY;
    for (int k = 0; k <= S; ++k) {
        double t = (double)k / S, u, v;
        trim_eval(g, t, &u, &v, NULL, NULL);
        double f = v - g->vs;
        double dd = (u - g->us) * (u - g->us) + (v - g->vs) * (v - g->vs);
        if (dd < best_d) { best_d = dd; best_t = t; }
        if (k > 0 && ((prev_f <= 0 && f > 0) || (prev_f >= 0 && f < 0)) && nc < 6) {
            double a = prev_t, b = t, fa = prev_f;
            for (int it = 0; it < 80; ++it) {
                double m = 0.5 * (a + b), um, vm;
                trim_eval(g, m, &um, &vm, NULL, NULL);
                double fm = vm - g->vs;
                if ((fa <= 0 && fm <= 0) || (fa >= 0 && fm >= 0)) { a = m; fa = fm; } else b = m;
            }
            centres[nc++] = 0.5 * (a + b);
        }
        prev_f = f;
        prev_t = t;
    }
    const int n_cross = nc;
    centres[nc++] = best_t;
    for (int k = 0; k < nc; ++k) {
        double u, v, du, dv, S3[3], Su[3], Sv[3];
        trim_eval(g, centres[k], &u, &v, &du, &dv);
        if (k < n_cross) {
            /* crossing of v = v*: F(u, v) has a peak of width ~ d / |S_v|
             * in v there (d = distance from q to the surface) */
            h0[k] = fmax(g->d, g->eps_on) / (g->sv * fabs(dv) + 1e-300);
            continue;
        }
        patch_point(g->p, fmin(fmax(u, 0), 1), fmin(fmax(v, 0), 1), S3, Su, Sv);
        double dx = S3[0] - g->p->q[0], dy = S3[1] - g->p->q[1], dz = S3[2] - g->p->q[2];
        double dist = sqrt(dx * dx + dy * dy + dz * dz);
        double speed = g->su * fabs(du) + g->sv * fabs(dv);
        h0[k] = fmax(dist, g->eps_on) / (speed + 1e-300);
    }
    return graded(outer_f, g, 0.0, 1.0, centres, h0, nc, 1e-14, UNIFORM_3D, g->rel);
}

static double gwn_patch(const patch3 *p, int n_trim, const int32_t *tdeg, const int64_t *tcoff,
                        const double *tuv, const double *tw, double eps_on);

/* On the surface: the mean of the two one-sided limits, approximated by the
 * mean of the values at q +- delta n (n the unit normal at the foot point,
 * delta = 1e3 eps_on). */
static double gwn_patch_onsurface(const patch3 *p, const double nrm[3], int n_trim, const int32_t *tdeg,
                                  const int64_t *tcoff, const double *tuv, const double *tw, double eps_on)
{
    patch3 a = *p, b = *p;
    double delta = 1e3 * eps_on;
    for (int k = 0; k < 3; ++k) { a.q[k] += delta * nrm[k]; b.q[k] -= delta * nrm[k]; }
    return 0.5 * (gwn_patch(&a, n_trim, tdeg, tcoff, tuv, tw, eps_on) +
                  gwn_patch(&b, n_trim, tdeg, tcoff, tuv, tw, eps_on));
}

static double gwn_patch(const patch3 *p, int n_trim, const int32_t *tdeg, const int64_t *tcoff,
                        const double *tuv, const double *tw, double eps_on)
{
    green_ctx g;
    memset(&g, 0, sizeof g);
    g.p = p;
    g.eps_on = eps_on;
    /* well separated (distance to the control-point box at least its
     * diagonal): the integrand is smooth, plain adaptive quadrature */
    {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                for (int k = 0; k < 3; ++k) {
                    double x = p->H[a][b][k] / p->H[a][b][3];
                    lo[k] = fmin(lo[k], x);
                    hi[k] = fmax(hi[k], x);
                }
        double d2 = 0, diag2 = 0;
        for (int k = 0; k < 3; ++k) {
            double e = fmax(fmax(lo[k] - p->q[k], p->q[k] - hi[k]), 0.0);
            d2 += e * e;
            diag2 += (hi[k] - lo[k]) * (hi[k] - lo[k]);
        }
        g.far = d2 >= diag2;
        g.rel = REL_3D;
        g.diag = sqrt(diag2);
    }
    if (!g.far) foot_point(p, &g.us, &g.vs);
    if (!g.far) {
        double S[3], Su[3], Sv[3];
        patch_point(p, g.us, g.vs, S, Su, Sv);
        g.su = sqrt(Su[0] * Su[0] + Su[1] * Su[1] + Su[2] * Su[2]);
        g.sv = sqrt(Sv[0] * Sv[0] + Sv[1] * Sv[1] + Sv[2] * Sv[2]);
        if (!(g.su > 0)) g.su = 1e-12;
        if (!(g.sv > 0)) g.sv = 1e-12;
        double dx = S[0] - p->q[0], dy = S[1] - p->q[1], dz = S[2] - p->q[2];
        g.d = sqrt(dx * dx + dy * dy + dz * dz);
        /* near the foot point A = H - q W carries absolute roundoff
         * ~eps |H|, i.e. relative noise ~eps diag / d */
        g.rel = fmax(REL_3D, 64.0 * 2.220446049250313e-16 * g.diag / fmax(g.d, eps_on));
        double n[3] = {Su[1] * Sv[2] - Su[2] * Sv[1], Su[2] * Sv[0] - Su[0] * Sv[2], Su[0] * Sv[1] - Su[1] * Sv[0]};
        double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (sqrt(dx * dx + dy * dy + dz * dz) < eps_on && nn > 0.0) {
            /* q on the surface S (within eps_on), taken over the whole
             * parameter square.  Where the foot point is on the visible
             * part, the value is the direct one, the mean of the two
             * one-sided limits.  Where it is on a trimmed-away part, the
             * patch's value is continuous across S there, so the same mean
             * is its value.  Either way the mean over q +- delta n is taken,
             * which also keeps the Green line integrals (whose segments
             * [0, u] x {v} may pass through the foot point) off the
             * singularity. */
            for (int k = 0; k < 3; ++k) n[k] /= nn;
            return gwn_patch_onsurface(p, n, n_trim, tdeg, tcoff, tuv, tw, eps_on);
        }
    }
    double total = 0.0;
    if (n_trim == 0) {
        /* untrimmed: only the edge u = 1 (v: 0 -> 1) has dv != 0 and F != 0 */
        g.n = 1;
        g.U[0] = 1; g.V[0] = 0; g.Wt[0] = 1;
        g.U[1] = 1; g.V[1] = 1; g.Wt[1] = 1;
        total = trim_contribution(&g);
    } else {
        for (int c = 0; c < n_trim; ++c) {
            g.n = tdeg[c];
            for (int j = 0; j <= g.n; ++j) {
                int64_t o = tcoff[c] + j;
                g.Wt[j] = tw[o];
                g.U[j] = tuv[2 * o] * tw[o];
                g.V[j] = tuv[2 * o + 1] * tw[o];
            }
            total += trim_contribution(&g);
        }
    }
    return total;
}

static int check_loops(int64_t n_trim, const int32_t *tdeg, const int64_t *tcoff, const double *tuv,
                       const double *tw)
{
    double sx = 0, sy = 0;
    int open = 0;
    for (int64_t c = 0; c < n_trim; ++c) {
        int d = tdeg[c];
        if (d < 1 || d > 2 || tcoff[c + 1] - tcoff[c] != d + 1) return -1;
        for (int64_t k = tcoff[c]; k < tcoff[c + 1]; ++k) {
            if (!(tw[k] > 0.0)) return -1;
            double u = tuv[2 * k], v = tuv[2 * k + 1];
            if (!(u >= 0.0 && u <= 1.0 && v >= 0.0 && v <= 1.0)) return -1;
        }
        double ax = tuv[2 * tcoff[c]], ay = tuv[2 * tcoff[c] + 1];
        double bx = tuv[2 * (tcoff[c + 1] - 1)], by = tuv[2 * (tcoff[c + 1] - 1) + 1];
        if (!open) { sx = ax; sy = ay; open = 1; }
        else {
            double px = tuv[2 * (tcoff[c] - 1)], py = tuv[2 * (tcoff[c] - 1) + 1];
            if (fabs(px - ax) > 1e-12 || fabs(py - ay) > 1e-12) return -2;
        }
        if (fabs(bx - sx) <= 1e-12 && fabs(by - sy) <= 1e-12) open = 0;
    }
    return open ? -2 : 0;
}

/*
 * oracle_gwn3d: w(q_k) = sum over all patches of (1/4pi) * solid angle of the
 * visible part of the patch, for k < n_q.
 *   cp_xyz[n*48]  bicubic control points, index (4*i + j)*3 + axis, i along u
 *   cp_w[n*16]    weights (> 0)
 *   trim_offset[n+1], trim_degree[], trim_cp_offset[], trim_cp_uv[], trim_cp_w[]
 *                 CSR trim curves as documented in the engine header; loops
 *                 must be closed and lie in [0,1]^2
 *   q[3*n_q], out[n_q], eps_on (absolute), nthreads
 * Returns 0, -1 for invalid control data, -2 for an open trim loop.
 */
int oracle_gwn3d(int64_t n, const double *cp_xyz, const double *cp_w, const int64_t *trim_offset,
                 const int32_t *trim_degree, const int64_t *trim_cp_offset, const double *trim_cp_uv,
                 const double *trim_cp_w, int64_t n_q, const double *q, double *out, double eps_on,
                 int nthreads)
{
    gl_init();
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < 16; ++k)
            if (!(cp_w[16 * i + k] > 0.0)) return -1;
        int64_t a = trim_offset[i], b = trim_offset[i + 1];
        if (b > a) {
            int r = check_loops(b - a, trim_degree + a, trim_cp_offset + a, trim_cp_uv, trim_cp_w);
            if (r) return r;
        }
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    long long unconv = 0;
    double worst = 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : unconv) reduction(max : worst)
    for (int64_t k = 0; k < n_q; ++k) {
        tl_unconverged = 0;
        tl_errbound = 0.0;
        tl_mult = 1.0;
        patch3 p;
        p.q[0] = q[3 * k]; p.q[1] = q[3 * k + 1]; p.q[2] = q[3 * k + 2];
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) {
                    int64_t o = 16 * i + 4 * a + b;
                    double w = cp_w[o];
                    p.H[a][b][0] = cp_xyz[3 * o] * w;
                    p.H[a][b][1] = cp_xyz[3 * o + 1] * w;
                    p.H[a][b][2] = cp_xyz[3 * o + 2] * w;
                    p.H[a][b][3] = w;
                }
            int64_t a0 = trim_offset[i], a1 = trim_offset[i + 1];
            s += gwn_patch(&p, (int)(a1 - a0), trim_degree + a0, trim_cp_offset + a0, trim_cp_uv,
                           trim_cp_w, eps_on);
        }
        out[k] = s / (4.0 * PI_);
        unconv += tl_unconverged;
        worst = fmax(worst, tl_errbound / (4.0 * PI_));
    }
    g_last_unconverged = unconv;
    g_last_errbound = worst;
    return 0;
}

/* Number of quadrature panels of the last oracle_gwn2d / oracle_gwn3d call
 * (on any thread) that were accepted unconverged at a work limit. */
long long oracle_last_unconverged(void)
{
    return g_last_unconverged;
}

/* Largest per-query error bound (units of w) of those panels in that call:
 * 0 when every panel met its tolerance. */
double oracle_last_errbound(void)
{
    return g_last_errbound;
}

/* Number of OpenMP threads a parallel region would use. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Gauss-Legendre nodes and weights on [-1,1] used by the adaptive rule. */
int oracle_gl_nodes(double *x, double *w)
{
    gl_init();
    for (int i = 0; i < GLN; ++i) { x[i] = gl_x[i]; w[i] = gl_w[i]; }
    return GLN;
}
