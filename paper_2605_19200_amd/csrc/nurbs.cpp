// Bezier extraction of 2D NURBS curves (Sec. 3.2: NURBS input is split into
// rational Bezier segments before the adaptive subdivision).
//
// For a span [a, b) = [t_k, t_k+1) of a degree-p B-spline with control points
// P_(k-p) .. P_k (homogeneous: (w x, w y, w)), the Bezier control points of
// the curve restricted to the span are the blossom values
//   B_j = f(a, ..., a, b, ..., b)   (p - j copies of a, j copies of b),
// and a blossom value f(s_1, ..., s_p) follows from de Boor's recurrence
// with s_r taking the place of the evaluation parameter at level r.  Inside
// the span every interpolation weight lies in [0, 1], so the extraction only
// forms convex combinations of the input points.
#include <cmath>
#include <string>
#include <vector>

#include "gwn_internal.h"

namespace gwn {

namespace {

struct H3 {
    double x, y, w;
};

// f(s_1..s_p) on span k of the knot vector U (degree p), control points P.
H3 blossom(const double *U, const H3 *P, int p, int64_t k, const double *s)
{
    H3 d[4];
    for (int i = 0; i <= p; ++i) d[i] = P[k - p + i];
    for (int r = 1; r <= p; ++r) {
        for (int i = p; i >= r; --i) {
            const int64_t j = k - p + i;   // control point index of d[i]
            const double a = (s[r - 1] - U[j]) / (U[j + p + 1 - r] - U[j]);
            d[i].x = (1.0 - a) * d[i - 1].x + a * d[i].x;
            d[i].y = (1.0 - a) * d[i - 1].y + a * d[i].y;
            d[i].w = (1.0 - a) * d[i - 1].w + a * d[i].w;
        }
    }
    return d[p];
}

bool check_curve(const gwn_nurbs2d &in, int64_t i, std::string &err)
{
    const int p = in.degree[i];
    if (p < 1 || p > 3) { err = "curve " + std::to_string(i) + ": degree must be 1..3"; return false; }
    const int64_t c0 = in.cp_offset[i], c1 = in.cp_offset[i + 1];
    const int64_t k0 = in.knot_offset[i], k1 = in.knot_offset[i + 1];
    const int64_t n = c1 - c0;
    if (c0 < 0 || n < p + 1) { err = "curve " + std::to_string(i) + ": needs at least degree + 1 control points"; return false; }
    if (k0 < 0 || k1 - k0 != n + p + 1) {
        err = "curve " + std::to_string(i) + ": knot count must be n_cp + degree + 1";
        return false;
    }
    for (int64_t k = c0; k < c1; ++k) {
        if (!std::isfinite(in.cp_xy[2 * k]) || !std::isfinite(in.cp_xy[2 * k + 1])) {
            err = "curve " + std::to_string(i) + ": non-finite control point";
            return false;
        }
        if (!(in.cp_w[k] > 0.0) || !std::isfinite(in.cp_w[k])) {
            err = "curve " + std::to_string(i) + ": weights must be finite and > 0";
            return false;
        }
    }
    const double *U = in.knots + k0;
    const int64_t m = k1 - k0 - 1;   // last knot index
    int run = 1;
    for (int64_t j = 0; j <= m; ++j) {
        if (!std::isfinite(U[j])) { err = "curve " + std::to_string(i) + ": non-finite knot"; return false; }
        if (j > 0) {
            if (U[j] < U[j - 1]) { err = "curve " + std::to_string(i) + ": knots must be non-decreasing"; return false; }
            run = U[j] == U[j - 1] ? run + 1 : 1;
            if (run > p + 1) {
                err = "curve " + std::to_string(i) + ": a knot is repeated more than degree + 1 times";
                return false;
            }
        }
    }
    for (int j = 1; j <= p; ++j)
        if (U[j] != U[0] || U[m - j] != U[m]) {
            err = "curve " + std::to_string(i) + ": knot vector must be clamped (first and last degree + 1 knots equal)";
            return false;
        }
    if (!(U[p] < U[m - p])) { err = "curve " + std::to_string(i) + ": empty parameter domain"; return false; }
    return true;
}

}  // namespace

bool extract_nurbs2d(const gwn_nurbs2d &in, std::vector<int32_t> &deg, std::vector<int64_t> &off,
                     std::vector<double> &xy, std::vector<double> &w, std::string &err)
{
    deg.clear();
    off.assign(1, 0);
    xy.clear();
    w.clear();
    if (in.n_curves < 0) { err = "n_curves must be >= 0"; return false; }
    if (in.n_curves == 0) return true;
    if (!in.degree || !in.cp_offset || !in.cp_xy || !in.cp_w || !in.knot_offset || !in.knots) {
        err = "NULL array in gwn_nurbs2d";
        return false;
    }
    if (in.cp_offset[0] != 0 || in.knot_offset[0] != 0) { err = "cp_offset[0] and knot_offset[0] must be 0"; return false; }
    for (int64_t i = 0; i < in.n_curves; ++i)
        if (in.cp_offset[i + 1] < in.cp_offset[i] || in.knot_offset[i + 1] < in.knot_offset[i]) {
            err = "offsets must be non-decreasing";
            return false;
        }
    std::vector<H3> P;
    for (int64_t i = 0; i < in.n_curves; ++i) {
        if (!check_curve(in, i, err)) return false;
        const int p = in.degree[i];
        const int64_t c0 = in.cp_offset[i], n = in.cp_offset[i + 1] - c0;
        const double *U = in.knots + in.knot_offset[i];
        P.resize(n);
        for (int64_t k = 0; k < n; ++k) {
            const double wk = in.cp_w[c0 + k];
            P[k] = {wk * in.cp_xy[2 * (c0 + k)], wk * in.cp_xy[2 * (c0 + k) + 1], wk};
        }
        for (int64_t k = p; k < n; ++k) {
            if (!(U[k] < U[k + 1])) continue;   // zero-length span
            const double a = U[k], b = U[k + 1];
            deg.push_back(p);
            for (int j = 0; j <= p; ++j) {
                double s[3];
                for (int r = 0; r < p; ++r) s[r] = r < p - j ? a : b;
                const H3 h = blossom(U, P.data(), p, k, s);
                xy.push_back(h.x / h.w);
                xy.push_back(h.y / h.w);
                w.push_back(h.w);
            }
            off.push_back(off.back() + p + 1);
        }
    }
    return true;
}

}  // namespace gwn
