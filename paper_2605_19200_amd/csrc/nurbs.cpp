// Bezier extraction of 2D NURBS curves and of trimmed NURBS surfaces (Sec.
// 3.2: NURBS input is split into rational Bezier pieces before the adaptive
// subdivision; Sec. 3.1: trimmed surfaces).
//
// For a span [a, b) = [t_k, t_k+1) of a degree-p B-spline with control points
// P_(k-p) .. P_k (homogeneous: (w x, w y, w)), the Bezier control points of
// the curve restricted to the span are the blossom values
//   B_j = f(a, ..., a, b, ..., b)   (p - j copies of a, j copies of b),
// and a blossom value f(s_1, ..., s_p) follows from de Boor's recurrence
// with s_r taking the place of the evaluation parameter at level r.  Inside
// the span every interpolation weight lies in [0, 1], so the extraction only
// forms convex combinations of the input points.  A tensor-product surface
// is a curve of curves: its span net is the u blossom of each column of the
// control net, then the v blossom of each resulting row.
#include <algorithm>
#include <cmath>
#include <cstring>
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

// Knot vector U of n control points at degree p: n + p + 1 finite,
// non-decreasing values, clamped, no value repeated more than p + 1 times,
// and a non-empty parameter domain [U_p, U_n].
bool check_knots(const double *U, int64_t n, int p, const std::string &tag, std::string &err)
{
    const int64_t m = n + p;   // last knot index
    int run = 1;
    for (int64_t j = 0; j <= m; ++j) {
        if (!std::isfinite(U[j])) { err = tag + ": non-finite knot"; return false; }
        if (j > 0) {
            if (U[j] < U[j - 1]) { err = tag + ": knots must be non-decreasing"; return false; }
            run = U[j] == U[j - 1] ? run + 1 : 1;
            if (run > p + 1) { err = tag + ": a knot is repeated more than degree + 1 times"; return false; }
        }
    }
    for (int j = 1; j <= p; ++j)
        if (U[j] != U[0] || U[m - j] != U[m]) {
            err = tag + ": knot vector must be clamped (first and last degree + 1 knots equal)";
            return false;
        }
    if (!(U[p] < U[m - p])) { err = tag + ": empty parameter domain"; return false; }
    return true;
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
    return check_knots(in.knots + k0, n, p, "curve " + std::to_string(i), err);
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

namespace {

struct H4 {
    double v[4];   // (w x, w y, w z, w)
};

// f(s_1..s_p) on span k of the knot vector U (degree p) of the homogeneous
// points P(0), P(1), ...
template <class Get>
H4 blossom4(const double *U, int p, int64_t k, const double *s, Get P)
{
    H4 d[4];
    for (int i = 0; i <= p; ++i) d[i] = P(k - p + i);
    for (int r = 1; r <= p; ++r)
        for (int i = p; i >= r; --i) {
            const int64_t j = k - p + i;
            const double a = (s[r - 1] - U[j]) / (U[j + p + 1 - r] - U[j]);
            for (int c = 0; c < 4; ++c) d[i].v[c] = (1.0 - a) * d[i - 1].v[c] + a * d[i].v[c];
        }
    return d[p];
}

// Bezier points B_0..B_p of span k: blossom values (a^(p-j), b^j)
template <class Get>
void span_bezier(const double *U, int p, int64_t k, Get P, H4 *B)
{
    for (int j = 0; j <= p; ++j) {
        double s[3];
        for (int r = 0; r < p; ++r) s[r] = r < p - j ? U[k] : U[k + 1];
        B[j] = blossom4(U, p, k, s, P);
    }
}

// The same Bezier polygon one degree higher (exact):
// Q_i = i / (p + 1) P_(i-1) + (1 - i / (p + 1)) P_i.
void elevate(const H4 *P, int p, H4 *Q)
{
    Q[0] = P[0];
    Q[p + 1] = P[p];
    for (int i = 1; i <= p; ++i) {
        const double a = (double)i / (p + 1);
        for (int c = 0; c < 4; ++c) Q[i].v[c] = a * P[i - 1].v[c] + (1.0 - a) * P[i].v[c];
    }
}

void to_cubic(const H4 *P, int p, H4 *Q)
{
    H4 a[4], b[4];
    for (int i = 0; i <= p; ++i) a[i] = P[i];
    for (int d = p; d < 3; ++d) {
        elevate(a, d, b);
        for (int i = 0; i <= d + 1; ++i) a[i] = b[i];
    }
    for (int i = 0; i < 4; ++i) Q[i] = a[i];
}

// first knot index of every span of positive size
std::vector<int64_t> span_starts(const double *U, int64_t n, int p)
{
    std::vector<int64_t> k;
    for (int64_t j = p; j < n; ++j)
        if (U[j] < U[j + 1]) k.push_back(j);
    return k;
}

double tc(const Trim3 &t, int j, int ax) { return t.h[3 * j + ax] / t.h[3 * j + 2]; }

// true when every loop runs along the edges of the unit square and encloses
// it counter-clockwise: the whole square is visible
bool whole_square(const std::vector<Trim3> &ts)
{
    if (ts.empty()) return false;
    for (const Trim3 &t : ts) {
        bool edge = false;
        for (int ax = 0; ax < 2 && !edge; ++ax)
            for (double e : {0.0, 1.0})
                if (tc(t, 0, ax) == e && tc(t, 1, ax) == e && tc(t, 2, ax) == e) edge = true;
        if (!edge) return false;
    }
    double area = 0.0;
    for (const Trim3 &t : ts) area += tc(t, 0, 0) * tc(t, 2, 1) - tc(t, 2, 0) * tc(t, 0, 1);
    return area > 0.0;
}

// closed loops of consecutive curves, as gwn_build3d requires
bool loops_closed(const std::vector<Trim3> &ts)
{
    bool open = false;
    double s0 = 0, s1 = 0, e0 = 0, e1 = 0;
    for (const Trim3 &t : ts) {
        const double a0 = tc(t, 0, 0), a1 = tc(t, 0, 1);
        if (!open) { s0 = a0; s1 = a1; open = true; }
        else if (std::fabs(a0 - e0) > 1e-12 || std::fabs(a1 - e1) > 1e-12) return false;
        e0 = tc(t, 2, 0);
        e1 = tc(t, 2, 1);
        if (std::fabs(e0 - s0) <= 1e-12 && std::fabs(e1 - s1) <= 1e-12) open = false;
    }
    return !open;
}

// Cut the loops of [0, 1]^2 along axis `dir` at the normalised breaks
// (ascending, inside (0, 1)) into one loop set per strip, each mapped to the
// strip's own unit square.  false: clip_trims_half failed at break `bad`.
bool strips(const std::vector<Trim3> &in, int dir, const std::vector<double> &breaks,
            std::vector<std::vector<Trim3>> &out, size_t &bad)
{
    out.assign(breaks.size() + 1, {});
    std::vector<Trim3> rest = in, high;
    double lo = 0.0;
    for (size_t b = 0; b < breaks.size(); ++b) {
        const double c = (breaks[b] - lo) / (1.0 - lo);
        if (!clip_trims_half(rest, dir, c, true, out[b]) || !clip_trims_half(rest, dir, c, false, high)) {
            bad = b;
            return false;
        }
        rest.swap(high);
        lo = breaks[b];
    }
    out.back() = rest;
    return true;
}

std::string surf(int64_t i) { return "surface " + std::to_string(i); }

bool check_surface(const gwn_nurbs3d &in, int64_t i, std::string &err)
{
    const int pu = in.degree_u[i], pv = in.degree_v[i];
    if (pu < 1 || pu > 3 || pv < 1 || pv > 3) { err = surf(i) + ": degrees must be 1..3"; return false; }
    const int64_t nu = in.n_u[i], nv = in.n_v[i];
    if (nu < pu + 1 || nv < pv + 1) { err = surf(i) + ": needs at least degree + 1 control points per direction"; return false; }
    const int64_t c0 = in.cp_offset[i], c1 = in.cp_offset[i + 1];
    if (c0 < 0 || c1 - c0 != nu * nv) { err = surf(i) + ": cp_offset range must hold n_u * n_v points"; return false; }
    if (in.knot_u_offset[i + 1] - in.knot_u_offset[i] != nu + pu + 1 ||
        in.knot_v_offset[i + 1] - in.knot_v_offset[i] != nv + pv + 1 || in.knot_u_offset[i] < 0 ||
        in.knot_v_offset[i] < 0) {
        err = surf(i) + ": knot counts must be n + degree + 1 per direction";
        return false;
    }
    for (int64_t k = c0; k < c1; ++k) {
        for (int a = 0; a < 3; ++a)
            if (!std::isfinite(in.cp_xyz[3 * k + a])) { err = surf(i) + ": non-finite control point"; return false; }
        if (!(in.cp_w[k] > 0.0) || !std::isfinite(in.cp_w[k])) { err = surf(i) + ": weights must be finite and > 0"; return false; }
    }
    return check_knots(in.knots_u + in.knot_u_offset[i], nu, pu, surf(i) + " (u knots)", err) &&
           check_knots(in.knots_v + in.knot_v_offset[i], nv, pv, surf(i) + " (v knots)", err);
}

// The surface's trim curves as Bezier segments in its normalised domain
// [0, 1]^2, homogeneous quadratics (degree 1 raised exactly).
bool surface_trims(const gwn_nurbs3d &in, int64_t i, const double dom[2][2], std::vector<Trim3> &out, std::string &err)
{
    out.clear();
    const int64_t t0 = in.trim_offset[i], t1 = in.trim_offset[i + 1];
    if (t1 == t0) return true;
    if (t0 < 0 || t1 < t0) { err = "trim_offset must be non-decreasing"; return false; }
    for (int64_t t = t0; t < t1; ++t)
        if (in.trim_degree[t] < 1 || in.trim_degree[t] > 2) {
            err = surf(i) + ": trim curves must have degree 1 or 2";
            return false;
        }
    const int64_t nt = t1 - t0, cb = in.trim_cp_offset[t0], kb = in.trim_knot_offset[t0];
    if (cb < 0 || kb < 0) { err = surf(i) + ": bad trim offsets"; return false; }
    std::vector<int64_t> co(nt + 1), ko(nt + 1);
    for (int64_t t = 0; t <= nt; ++t) {
        co[t] = in.trim_cp_offset[t0 + t] - cb;
        ko[t] = in.trim_knot_offset[t0 + t] - kb;
    }
    gwn_nurbs2d tr{nt, in.trim_degree + t0, co.data(), in.trim_cp_uv + 2 * cb, in.trim_cp_w + cb, ko.data(),
                   in.trim_knots + kb};
    std::vector<int32_t> deg;
    std::vector<int64_t> off;
    std::vector<double> xy, w;
    if (!extract_nurbs2d(tr, deg, off, xy, w, err)) { err = surf(i) + " trim " + err; return false; }
    for (size_t g = 0; g < deg.size(); ++g) {
        double P[3][3];
        for (int j = 0; j <= deg[g]; ++j) {
            const int64_t k = off[g] + j;
            double uv[2];
            for (int a = 0; a < 2; ++a) {
                const double lo = dom[a][0], hi = dom[a][1], x = xy[2 * k + a];
                if (x < lo - 1e-12 * (hi - lo) || x > hi + 1e-12 * (hi - lo)) {
                    err = surf(i) + ": trim curves must lie in the parameter domain";
                    return false;
                }
                uv[a] = std::min(1.0, std::max(0.0, (x - lo) / (hi - lo)));
                if (uv[a] < 1e-13) uv[a] = 0.0;
                if (uv[a] > 1.0 - 1e-13) uv[a] = 1.0;
            }
            P[j][0] = w[k] * uv[0];
            P[j][1] = w[k] * uv[1];
            P[j][2] = w[k];
        }
        Trim3 t;
        std::memset(&t, 0, sizeof t);
        for (int q = 0; q < 3; ++q) {
            t.h[q] = P[0][q];
            t.h[3 + q] = deg[g] == 2 ? P[1][q] : 0.5 * (P[0][q] + P[1][q]);
            t.h[6 + q] = P[deg[g]][q];
        }
        out.push_back(t);
    }
    if (!loops_closed(out)) { err = surf(i) + ": trim loops must be closed"; return false; }
    return true;
}

}  // namespace

bool extract_nurbs3d(const gwn_nurbs3d &in, NurbsPatches &out, std::string &err)
{
    out = NurbsPatches{};
    out.trim_offset.assign(1, 0);
    out.trim_cp_offset.assign(1, 0);
    if (in.n_surfaces < 0) { err = "n_surfaces must be >= 0"; return false; }
    if (in.n_surfaces == 0) return true;
    if (!in.degree_u || !in.degree_v || !in.n_u || !in.n_v || !in.cp_offset || !in.cp_xyz || !in.cp_w ||
        !in.knot_u_offset || !in.knots_u || !in.knot_v_offset || !in.knots_v || !in.trim_offset) {
        err = "NULL array in gwn_nurbs3d";
        return false;
    }
    if (in.cp_offset[0] != 0 || in.knot_u_offset[0] != 0 || in.knot_v_offset[0] != 0 || in.trim_offset[0] != 0) {
        err = "cp_offset[0], knot_u_offset[0], knot_v_offset[0] and trim_offset[0] must be 0";
        return false;
    }
    if (in.trim_offset[in.n_surfaces] > 0 &&
        (!in.trim_degree || !in.trim_cp_offset || !in.trim_cp_uv || !in.trim_cp_w || !in.trim_knot_offset ||
         !in.trim_knots)) {
        err = "NULL trim array in gwn_nurbs3d";
        return false;
    }
    for (int64_t i = 0; i < in.n_surfaces; ++i) {
        if (in.cp_offset[i + 1] < in.cp_offset[i] || in.knot_u_offset[i + 1] < in.knot_u_offset[i] ||
            in.knot_v_offset[i + 1] < in.knot_v_offset[i] || in.trim_offset[i + 1] < in.trim_offset[i]) {
            err = "offsets must be non-decreasing";
            return false;
        }
    }
    std::vector<Trim3> trims;
    std::vector<std::vector<Trim3>> cols, cells;
    std::vector<H4> C;
    for (int64_t i = 0; i < in.n_surfaces; ++i) {
        if (!check_surface(in, i, err)) return false;
        const int pu = in.degree_u[i], pv = in.degree_v[i];
        const int64_t nu = in.n_u[i], nv = in.n_v[i], c0 = in.cp_offset[i];
        const double *U = in.knots_u + in.knot_u_offset[i], *V = in.knots_v + in.knot_v_offset[i];
        const double dom[2][2] = {{U[pu], U[nu]}, {V[pv], V[nv]}};
        if (!surface_trims(in, i, dom, trims, err)) return false;
        const bool trimmed = !trims.empty();
        const std::vector<int64_t> su = span_starts(U, nu, pu), sv = span_starts(V, nv, pv);
        std::vector<double> bu, bv;
        for (size_t s = 1; s < su.size(); ++s) bu.push_back((U[su[s]] - dom[0][0]) / (dom[0][1] - dom[0][0]));
        for (size_t s = 1; s < sv.size(); ++s) bv.push_back((V[sv[s]] - dom[1][0]) / (dom[1][1] - dom[1][0]));
        size_t bad = 0;
        if (trimmed && !strips(trims, 0, bu, cols, bad)) {
            err = surf(i) + ": a trim loop meets the knot line u = " + std::to_string(U[su[bad + 1]]) +
                  " at a junction of two trim curves or tangentially";
            return false;
        }
        auto P = [&](int64_t a, int64_t b) {
            H4 h;
            const int64_t k = c0 + nv * a + b;
            const double w = in.cp_w[k];
            for (int c = 0; c < 3; ++c) h.v[c] = w * in.cp_xyz[3 * k + c];
            h.v[3] = w;
            return h;
        };
        C.resize((size_t)(pu + 1) * nv);
        for (size_t a = 0; a < su.size(); ++a) {
            if (trimmed && cols[a].empty()) continue;
            if (trimmed && !strips(cols[a], 1, bv, cells, bad)) {
                err = surf(i) + ": a trim loop meets the knot line v = " + std::to_string(V[sv[bad + 1]]) +
                      " at a junction of two trim curves or tangentially";
                return false;
            }
            // u Bezier points of every column of the net on span a
            for (int64_t b = 0; b < nv; ++b) {
                H4 B[4];
                span_bezier(U, pu, su[a], [&](int64_t k) { return P(k, b); }, B);
                for (int j = 0; j <= pu; ++j) C[(size_t)j * nv + b] = B[j];
            }
            for (size_t b = 0; b < sv.size(); ++b) {
                if (trimmed && cells[b].empty()) continue;
                H4 net[4][4], row[4], col[4], up[4];
                for (int j = 0; j <= pu; ++j) {
                    span_bezier(V, pv, sv[b], [&](int64_t k) { return C[(size_t)j * nv + k]; }, row);
                    to_cubic(row, pv, net[j]);
                }
                double xyz[48], ww[16];
                for (int k = 0; k < 4; ++k) {
                    for (int j = 0; j <= pu; ++j) col[j] = net[j][k];
                    to_cubic(col, pu, up);
                    for (int j = 0; j < 4; ++j) {
                        ww[4 * j + k] = up[j].v[3];
                        for (int c = 0; c < 3; ++c) xyz[3 * (4 * j + k) + c] = up[j].v[c] / up[j].v[3];
                    }
                }
                out.cp_xyz.insert(out.cp_xyz.end(), xyz, xyz + 48);
                out.cp_w.insert(out.cp_w.end(), ww, ww + 16);
                out.source.push_back(i);
                if (trimmed && !whole_square(cells[b]))
                    for (const Trim3 &t : cells[b]) {
                        out.trim_degree.push_back(2);
                        for (int j = 0; j < 3; ++j) {
                            out.trim_cp_uv.push_back(t.h[3 * j] / t.h[3 * j + 2]);
                            out.trim_cp_uv.push_back(t.h[3 * j + 1] / t.h[3 * j + 2]);
                            out.trim_cp_w.push_back(t.h[3 * j + 2]);
                        }
                        out.trim_cp_offset.push_back(out.trim_cp_offset.back() + 3);
                    }
                out.trim_offset.push_back((int64_t)out.trim_degree.size());
            }
        }
    }
    return true;
}

}  // namespace gwn
