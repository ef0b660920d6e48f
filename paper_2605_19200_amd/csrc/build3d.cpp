// Host preprocessing of a 3D model (Alg. 1, threaded preprocessing) for
// trimmed rational bicubic patches:
//   AdaptiveSubdivision -> ComputeUncenteredMoments -> ConstructBVH ->
//   SumUncenteredMomentsUpTree -> CenterMomentsInPlace.
//
// Moments (Sec. 3.1, Fig. quadrature_demo): the surface integrals
//   int n dA, int x (x) n dA, int x (x) x (x) n dA, int dA, int x dA
// over the visible part D of the parameter square are turned into line
// integrals over D's boundary by Green's theorem in (u, v):
//   integral_D f du dv = sum over boundary curves of
//                        integral F(u(t), v(t)) v'(t) dt,  F(u, v) = int_0^u f(s, v) ds,
// and both levels use n-point Gauss-Legendre rules, which scatters n x n
// nodes per boundary curve into D.  The nodes are query independent: each
// node keeps its position x and weighted normal N = W (S_u x S_v), which
// gives every moment as a sum over nodes and also the leaf's direct GWN for
// queries well separated from it:  Omega(q) = sum N . (x - q) / |x - q|^3.
// For an untrimmed patch the boundary is the unit square, and only the edge
// u = 1 contributes (F = 0 on u = 0, v' = 0 on the other two edges).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "gwn_internal.h"
#include "multipole3d.h"

namespace gwn {

// Gauss-Legendre rule with n nodes on [0, 1]: Newton's method on P_n from
// the Chebyshev-like initial guesses, weights 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre01(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) { p1 = z; p0 = 1.0; }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[n - 1 - i] = 0.5 * (z + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);   // (2 / (...)) / 2 for [0, 1]
    }
}

// The (2n+1)-point Gauss-Kronrod rule on [0, 1] with its embedded n-point
// Gauss rule (2 <= n <= 10), computed from the definition (Kronrod 1965):
// the n + 1 added nodes are the zeros of the Stieltjes polynomial E_{n+1},
// the monic polynomial of degree n + 1 orthogonal to every polynomial of
// degree <= n under the weight P_n on [-1, 1]; E_{n+1} has the parity of
// n + 1, and its zeros interlace the Gauss nodes.  The weights make the rule
// exact for polynomials of degree <= 2n, which with those nodes makes it
// exact to degree 3n + 1.  Nodes are returned in increasing order; the Gauss
// nodes are the odd indices and wg[i] is the Gauss weight of node 2 i + 1.
void gauss_kronrod01(int n, double *xk, double *wk, double *wg)
{
    typedef long double R;
    // power-basis coefficients of P_n by the three-term recurrence
    R pm[12] = {1}, pc[12] = {0, 1}, pn[12];
    for (int k = 2; k <= n; ++k) {
        for (int i = 0; i <= k; ++i) {
            pn[i] = -(R)(k - 1) / k * (i < k - 1 ? pm[i] : 0);
            if (i > 0) pn[i] += (R)(2 * k - 1) / k * pc[i - 1];
        }
        for (int i = 0; i < 12; ++i) { pm[i] = pc[i]; pc[i] = i <= k ? pn[i] : 0; }
    }
    const R *pol = pc;
    auto mom = [&](int m) {   // integral over [-1, 1] of P_n(x) x^m
        R s = 0;
        for (int i = 0; i <= n; ++i)
            if (pol[i] != 0 && (i + m) % 2 == 0) s += pol[i] * 2 / (R)(i + m + 1);
        return s;
    };
    // E_{n+1}(x) = x^(n+1) + sum_j a_j x^(n+1-2-2j): unknown coefficients of
    // the powers of its parity below n + 1, one condition per odd k <= n
    const int nu = (n + 1) / 2;
    R A[6][7];
    for (int r = 0; r < nu; ++r) {
        const int k = 2 * r + 1;
        for (int c = 0; c < nu; ++c) A[r][c] = mom((n + 1) % 2 + 2 * c + k);
        A[r][nu] = -mom(n + 1 + k);
    }
    for (int c = 0; c < nu; ++c) {
        int piv = c;
        for (int r = c + 1; r < nu; ++r)
            if (fabsl(A[r][c]) > fabsl(A[piv][c])) piv = r;
        for (int j = 0; j <= nu; ++j) std::swap(A[c][j], A[piv][j]);
        for (int r = 0; r < nu; ++r)
            if (r != c) {
                const R f = A[r][c] / A[c][c];
                for (int j = c; j <= nu; ++j) A[r][j] -= f * A[c][j];
            }
    }
    R a[6];
    for (int c = 0; c < nu; ++c) a[c] = A[c][nu] / A[c][c];   // coefficient of x^((n+1)%2 + 2c)
    auto E = [&](R x) {
        R s = powl(x, n + 1);
        for (int c = 0; c < nu; ++c) s += a[c] * powl(x, (n + 1) % 2 + 2 * c);
        return s;
    };
    double gx[10], gw[10];
    gauss_legendre01(n, gx, gw);
    // nonnegative nodes: Gauss ones from the n-point rule, Kronrod ones one in
    // each gap above a Gauss node (and 0 when n is even)
    std::vector<R> gpos, kpos;
    for (int i = 0; i < n; ++i) {
        const R x = 2 * (R)gx[i] - 1;
        if (x > -1e-30L) gpos.push_back(x < 1e-30L ? 0 : x);
    }
    std::sort(gpos.begin(), gpos.end());
    if (n % 2 == 0) kpos.push_back(0);
    for (size_t i = 0; i < gpos.size(); ++i) {
        R lo = gpos[i], hi = i + 1 < gpos.size() ? gpos[i + 1] : 1;
        R flo = E(lo);
        for (int it = 0; it < 200; ++it) {
            const R mid = (lo + hi) / 2, fm = E(mid);
            if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else hi = mid;
        }
        kpos.push_back((lo + hi) / 2);
    }
    std::vector<R> ys;   // distinct |x|^2, the centre first
    for (R x : gpos) ys.push_back(x * x);
    for (R x : kpos) ys.push_back(x * x);
    std::sort(ys.begin(), ys.end());
    const int m = (int)ys.size();   // n + 1
    R V[12][13];
    for (int j = 0; j < m; ++j) {
        for (int i = 0; i < m; ++i) V[j][i] = (i == 0) ? (j == 0 ? 1 : 0) : powl(ys[i], j);
        V[j][m] = 2.0L / (2 * j + 1);
    }
    for (int c = 0; c < m; ++c) {
        int piv = c;
        for (int r = c + 1; r < m; ++r)
            if (fabsl(V[r][c]) > fabsl(V[piv][c])) piv = r;
        for (int j = 0; j <= m; ++j) std::swap(V[c][j], V[piv][j]);
        for (int r = 0; r < m; ++r)
            if (r != c) {
                const R f = V[r][c] / V[c][c];
                for (int j = c; j <= m; ++j) V[r][j] -= f * V[c][j];
            }
    }
    for (int i = 0; i < m; ++i) {
        const R x = sqrtl(ys[i]), w = i == 0 ? V[0][m] / V[0][0] : V[i][m] / V[i][i] / 2;
        xk[n + i] = (double)((1 + x) / 2);
        xk[n - i] = (double)((1 - x) / 2);
        wk[n + i] = wk[n - i] = (double)(w / 2);
    }
    for (int i = 0; i < n; ++i) wg[i] = gw[i];
}

namespace {

struct Patch {
    double h[4][4][4];   // [i along u][j along v][wx, wy, wz, w]
    int64_t src;
    std::vector<Trim3> trims;   // closed loops in the patch's own (u, v); empty = whole square
};

void cubic_basis(double t, double *B, double *dB)
{
    double s = 1.0 - t;
    B[0] = s * s * s; B[1] = 3 * s * s * t; B[2] = 3 * s * t * t; B[3] = t * t * t;
    dB[0] = -3 * s * s; dB[1] = 3 * s * s - 6 * s * t; dB[2] = 6 * s * t - 3 * t * t; dB[3] = 3 * t * t;
}

// Euclidean point and partials of the rational bicubic at (u, v).
void surface(const Patch &p, double u, double v, double S[3], double Su[3], double Sv[3])
{
    double bu[4], du[4], bv[4], dv[4];
    cubic_basis(u, bu, du);
    cubic_basis(v, bv, dv);
    double H[4] = {0, 0, 0, 0}, Hu[4] = {0, 0, 0, 0}, Hv[4] = {0, 0, 0, 0};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 4; ++k) {
                H[k] += bu[i] * bv[j] * p.h[i][j][k];
                Hu[k] += du[i] * bv[j] * p.h[i][j][k];
                Hv[k] += bu[i] * dv[j] * p.h[i][j][k];
            }
    const double W = H[3];
    for (int k = 0; k < 3; ++k) {
        S[k] = H[k] / W;
        Su[k] = (Hu[k] * W - H[k] * Hu[3]) / (W * W);
        Sv[k] = (Hv[k] * W - H[k] * Hv[3]) / (W * W);
    }
}

void trim_point(const Trim3 &c, double t, double *u, double *v, double *du, double *dv)
{
    double s = 1.0 - t;
    double b[3] = {s * s, 2 * s * t, t * t}, d[3] = {-2 * s, 2 * s - 2 * t, 2 * t};
    double hu = 0, hv = 0, hw = 0, gu = 0, gv = 0, gw = 0;
    for (int i = 0; i < 3; ++i) {
        hu += b[i] * c.h[3 * i]; hv += b[i] * c.h[3 * i + 1]; hw += b[i] * c.h[3 * i + 2];
        gu += d[i] * c.h[3 * i]; gv += d[i] * c.h[3 * i + 1]; gw += d[i] * c.h[3 * i + 2];
    }
    *u = hu / hw;
    *v = hv / hw;
    *du = (gu * hw - hu * gw) / (hw * hw);
    *dv = (gv * hw - hv * gw) / (hw * hw);
}

void patch_aabb(const Patch &p, double lo[3], double hi[3])
{
    for (int k = 0; k < 3; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 3; ++k) {
                double x = p.h[i][j][k] / p.h[i][j][3];
                lo[k] = std::min(lo[k], x);
                hi[k] = std::max(hi[k], x);
            }
}

// de Casteljau split of the control net at parameter t along u (dir 0) or
// v; each half is reparametrised to [0, 1].
void split(const Patch &p, int dir, double t, Patch &L, Patch &R)
{
    L = p;
    R = p;
    const double s = 1.0 - t;
    for (int a = 0; a < 4; ++a)
        for (int k = 0; k < 4; ++k) {
            double c[4];
            for (int i = 0; i < 4; ++i) c[i] = dir == 0 ? p.h[i][a][k] : p.h[a][i][k];
            double b0 = s * c[0] + t * c[1], b1 = s * c[1] + t * c[2], b2 = s * c[2] + t * c[3];
            double c0 = s * b0 + t * b1, c1 = s * b1 + t * b2, d0 = s * c0 + t * c1;
            double l[4] = {c[0], b0, c0, d0}, r[4] = {d0, c1, b2, c[3]};
            for (int i = 0; i < 4; ++i) {
                (dir == 0 ? L.h[i][a][k] : L.h[a][i][k]) = l[i];
                (dir == 0 ? R.h[i][a][k] : R.h[a][i][k]) = r[i];
            }
        }
}

// length of the control polygon of the middle iso-curve in direction dir
double mid_iso_length(const Patch &p, int dir)
{
    double len = 0.0;
    for (int i = 0; i < 3; ++i) {
        double d2 = 0;
        for (int k = 0; k < 3; ++k) {
            // average of the two middle rows, as Euclidean points
            double a, b;
            if (dir == 0) {
                a = 0.5 * (p.h[i][1][k] / p.h[i][1][3] + p.h[i][2][k] / p.h[i][2][3]);
                b = 0.5 * (p.h[i + 1][1][k] / p.h[i + 1][1][3] + p.h[i + 1][2][k] / p.h[i + 1][2][3]);
            } else {
                a = 0.5 * (p.h[1][i][k] / p.h[1][i][3] + p.h[2][i][k] / p.h[2][i][3]);
                b = 0.5 * (p.h[1][i + 1][k] / p.h[1][i + 1][3] + p.h[2][i + 1][k] / p.h[2][i + 1][3]);
            }
            d2 += (b - a) * (b - a);
        }
        len += std::sqrt(d2);
    }
    return len;
}

}  // namespace

gwn_status build3d_host(const gwn_patches3d *c, const gwn_params *p, Model &m, std::string &err)
{
    const int64_t n = c->n_patches;
    if (n < 0) { err = "n_patches < 0"; return GWN_EINVAL; }
    if (n > 0 && (!c->cp_xyz || !c->cp_w || !c->trim_offset)) { err = "NULL patch array"; return GWN_EINVAL; }
    if (n > (int64_t)1 << 26) { err = "too many patches"; return GWN_EINVAL; }
    m.dim = 3;
    m.params = *p;
    m.n_input = n;
    m.trims.clear();
    std::vector<Patch> work;
    work.reserve((size_t)n);
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (n > 0 && c->trim_offset[0] != 0) { err = "trim_offset[0] must be 0"; return GWN_EINVAL; }
    for (int64_t i = 0; i < n; ++i) {
        Patch pt;
        pt.src = i;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                const int64_t o = 16 * i + 4 * a + b;
                const double w = c->cp_w[o];
                if (!std::isfinite(w) || !(w > 0.0)) {
                    err = "patch " + std::to_string(i) + ": weights must be finite and > 0";
                    return GWN_EINVAL;
                }
                for (int k = 0; k < 3; ++k) {
                    const double x = c->cp_xyz[3 * o + k];
                    if (!std::isfinite(x)) { err = "patch " + std::to_string(i) + ": non-finite control point"; return GWN_EINVAL; }
                    pt.h[a][b][k] = x * w;
                    lo[k] = std::min(lo[k], x);
                    hi[k] = std::max(hi[k], x);
                }
                pt.h[a][b][3] = w;
            }
        const int64_t t0 = c->trim_offset[i], t1 = c->trim_offset[i + 1];
        if (t1 < t0) { err = "trim_offset must be non-decreasing"; return GWN_EINVAL; }
        if (t1 > t0 && (!c->trim_degree || !c->trim_cp_offset || !c->trim_cp_uv || !c->trim_cp_w)) {
            err = "NULL trim array";
            return GWN_EINVAL;
        }
        double ls[2] = {0, 0}, pe[2] = {0, 0};
        bool open = false;
        for (int64_t k = t0; k < t1; ++k) {
            const int d = c->trim_degree[k];
            const int64_t a = c->trim_cp_offset[k], b = c->trim_cp_offset[k + 1];
            if (d < 1 || d > 2 || b - a != d + 1) {
                err = "patch " + std::to_string(i) + ": trim curves must have degree 1 or 2 and matching offsets";
                return GWN_EINVAL;
            }
            double P[3][3];
            for (int j = 0; j <= d; ++j) {
                const double u = c->trim_cp_uv[2 * (a + j)], v = c->trim_cp_uv[2 * (a + j) + 1], w = c->trim_cp_w[a + j];
                if (!std::isfinite(u) || !std::isfinite(v) || !std::isfinite(w) || !(w > 0.0)) {
                    err = "patch " + std::to_string(i) + ": bad trim control data";
                    return GWN_EINVAL;
                }
                if (u < 0.0 || u > 1.0 || v < 0.0 || v > 1.0) {
                    err = "patch " + std::to_string(i) + ": trim curves must lie in [0,1]^2";
                    return GWN_EINVAL;
                }
                P[j][0] = u * w; P[j][1] = v * w; P[j][2] = w;
            }
            const double su = c->trim_cp_uv[2 * a], sv = c->trim_cp_uv[2 * a + 1];
            const double eu = c->trim_cp_uv[2 * (b - 1)], ev = c->trim_cp_uv[2 * (b - 1) + 1];
            if (!open) { ls[0] = su; ls[1] = sv; open = true; }
            else if (std::fabs(su - pe[0]) > 1e-12 || std::fabs(sv - pe[1]) > 1e-12) {
                err = "patch " + std::to_string(i) + ": trim loop is not closed (curve " + std::to_string(k - t0) +
                      " does not start where the previous one ends)";
                return GWN_EINVAL;
            }
            pe[0] = eu; pe[1] = ev;
            if (std::fabs(eu - ls[0]) <= 1e-12 && std::fabs(ev - ls[1]) <= 1e-12) open = false;
            Trim3 tr;
            std::memset(&tr, 0, sizeof tr);
            if (d == 2) {
                for (int j = 0; j < 3; ++j)
                    for (int q = 0; q < 3; ++q) tr.h[3 * j + q] = P[j][q];
            } else {   // exact degree elevation of the segment
                for (int q = 0; q < 3; ++q) {
                    tr.h[q] = P[0][q];
                    tr.h[3 + q] = 0.5 * (P[0][q] + P[1][q]);
                    tr.h[6 + q] = P[1][q];
                }
            }
            pt.trims.push_back(tr);
        }
        if (open) { err = "patch " + std::to_string(i) + ": trim loop is not closed"; return GWN_EINVAL; }
        work.push_back(std::move(pt));
    }
    if (n == 0)
        for (int k = 0; k < 3; ++k) lo[k] = hi[k] = 0.0;
    double diag2 = 0;
    for (int k = 0; k < 3; ++k) {
        m.lo[k] = lo[k];
        m.hi[k] = hi[k];
        diag2 += (hi[k] - lo[k]) * (hi[k] - lo[k]);
    }
    m.diag = std::sqrt(diag2);

    // AdaptiveSubdivision (Sec. 3.2): bisect patches while their AABB
    // diagonal is not below max_diag_frac of the model diagonal, in the
    // parameter direction whose middle iso-curve has the longer control
    // polygon.  A trimmed patch's loops are clipped to each half and mapped
    // to the half's unit square (clip_trims_half); a half that holds none of
    // the visible region is dropped.  When the cut at 1/2 would pass through
    // a junction of two trim curves or touch a loop tangentially, the cut
    // moves to the nearest of 1/2 +- k/64 (k = 1..8) where it does not.
    const double limit = p->max_diag_frac * m.diag;
    std::vector<Patch> leaves;
    leaves.reserve(work.size());
    struct Item { Patch p; int depth; };
    std::vector<Item> st;
    for (int64_t i = (int64_t)work.size() - 1; i >= 0; --i) st.push_back({std::move(work[i]), 0});
    std::vector<Trim3> lo_trims, hi_trims;
    while (!st.empty()) {
        Item it = std::move(st.back());
        st.pop_back();
        double l[3], h[3];
        patch_aabb(it.p, l, h);
        const double dg = std::sqrt((h[0] - l[0]) * (h[0] - l[0]) + (h[1] - l[1]) * (h[1] - l[1]) +
                                    (h[2] - l[2]) * (h[2] - l[2]));
        bool done = true;
        if (limit > 0 && dg >= limit && it.depth < 24) {
            const int dir = mid_iso_length(it.p, 0) >= mid_iso_length(it.p, 1) ? 0 : 1;
            for (int k = 0; k <= 16; ++k) {
                const double c = 0.5 + (k == 0 ? 0.0 : ((k & 1) ? 1.0 : -1.0) * ((k + 1) / 2) / 64.0);
                if (!it.p.trims.empty() && (!clip_trims_half(it.p.trims, dir, c, true, lo_trims) ||
                                            !clip_trims_half(it.p.trims, dir, c, false, hi_trims)))
                    continue;
                Patch L, R;
                split(it.p, dir, c, L, R);
                const bool trimmed = !it.p.trims.empty();
                L.trims = trimmed ? lo_trims : std::vector<Trim3>{};
                R.trims = trimmed ? hi_trims : std::vector<Trim3>{};
                // an empty loop list of a trimmed patch's half: nothing visible
                if (!trimmed || !R.trims.empty()) st.push_back({std::move(R), it.depth + 1});
                if (!trimmed || !L.trims.empty()) st.push_back({std::move(L), it.depth + 1});
                done = false;
                break;
            }
        }
        if (done) leaves.push_back(std::move(it.p));
    }
    const int nl = (int)leaves.size();

    // ComputeUncenteredMoments via the Green-scattered Gauss-Legendre nodes
    // (n = gl_nodes per rule).  Each leaf also keeps a ladder of node sets
    // for its direct evaluation at well-separated queries (kLeafRules).
    const int g = p->gl_nodes;
    std::vector<double> gx(g), gw(g);
    gauss_legendre01(g, gx.data(), gw.data());
    std::vector<double> lx[3], lw[3];
    for (int r = 0; r < 3; ++r) {
        lx[r].resize(kLeafRules[r]);
        lw[r].resize(kLeafRules[r]);
        gauss_legendre01(kLeafRules[r], lx[r].data(), lw[r].data());
    }
    const int nm = n_moments(3);
    std::vector<double> LO(3 * (size_t)nl), HI(3 * (size_t)nl), U((size_t)nl * nm, 0.0), Wt(nl, 0.0),
        WC(3 * (size_t)nl, 0.0);
    std::vector<std::vector<QNode3>> qn(nl);
    std::vector<std::array<int, 3>> qcount(nl);
    // multipole moments of each leaf about its own centroid (far field at
    // orders above 2; see multipole3d.h)
    // (two degrees beyond the far field's, for the error-budgeted far test)
    std::vector<cplx> LN((size_t)nl * kMpoleTermsTail, cplx(0, 0));
    std::vector<double> LC(3 * (size_t)nl, 0.0);
    // leaves are independent: split them over host threads
    auto leaf_work = [&](int li) {
        const Patch &pt = leaves[li];
        patch_aabb(pt, &LO[3 * li], &HI[3 * li]);
        // boundary curves: the trims, or the edge u = 1 of the square
        std::vector<Trim3> curves;
        if (pt.trims.empty()) {
            Trim3 e;
            std::memset(&e, 0, sizeof e);
            const double P[3][3] = {{1, 0, 1}, {1, 0.5, 1}, {1, 1, 1}};
            for (int j = 0; j < 3; ++j)
                for (int q = 0; q < 3; ++q) e.h[3 * j + q] = P[j][q];
            curves.push_back(e);
        } else {
            curves = pt.trims;
        }
        double *u_out = &U[(size_t)li * nm];
        // scatter no x ni nodes per boundary curve (no along the curve, ni
        // along the horizontal segment); f(x, N, W |n|) per node
        auto scatter = [&](const double *xo, const double *wo, int no, const double *xs, const double *wsg, int nn,
                           auto &&f) {
            for (const Trim3 &cv : curves)
                for (int k = 0; k < no; ++k) {
                    double uk, vk, duk, dvk;
                    trim_point(cv, xo[k], &uk, &vk, &duk, &dvk);
                    if (dvk == 0.0 || uk == 0.0) continue;
                    for (int j = 0; j < nn; ++j) {
                        const double W = wo[k] * dvk * wsg[j] * uk;
                        double S[3], Su[3], Sv[3];
                        surface(pt, xs[j] * uk, vk, S, Su, Sv);
                        const double nrm[3] = {Su[1] * Sv[2] - Su[2] * Sv[1], Su[2] * Sv[0] - Su[0] * Sv[2],
                                               Su[0] * Sv[1] - Su[1] * Sv[0]};
                        QNode3 node;
                        for (int a = 0; a < 3; ++a) {
                            node.x[a] = S[a];
                            node.n[a] = W * nrm[a];
                        }
                        f(node, W * std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]));
                    }
                }
        };
        for (int r = 0; r < 3; ++r) {
            const size_t before = qn[li].size();
            scatter(lx[r].data(), lw[r].data(), kLeafRules[r], lx[r].data(), lw[r].data(), kLeafRules[r],
                    [&](const QNode3 &node, double) { qn[li].push_back(node); });
            qcount[li][r] = (int)(qn[li].size() - before);
        }
        scatter(gx.data(), gw.data(), g, gx.data(), gw.data(), g, [&](const QNode3 &node, double area) {
                    const double *S = node.x;
                    for (int a = 0; a < 3; ++a) u_out[a] += node.n[a];
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) u_out[3 + 3 * a + b] += S[a] * node.n[b];
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b)
                            for (int k2 = 0; k2 < 3; ++k2) u_out[12 + 9 * a + 3 * b + k2] += S[a] * S[b] * node.n[k2];
                    Wt[li] += area;
                    for (int a = 0; a < 3; ++a) WC[3 * li + a] += area * S[a];
                });
        double *cl = &LC[3 * li];
        for (int a = 0; a < 3; ++a)
            cl[a] = Wt[li] > 0.0 ? WC[3 * li + a] / Wt[li] : 0.5 * (LO[3 * li + a] + HI[3 * li + a]);
        cplx *nl_out = &LN[(size_t)li * kMpoleTermsTail];
        scatter(gx.data(), gw.data(), g, gx.data(), gw.data(), g,
                [&](const QNode3 &node, double) { mpole_add_node(node.x, node.n, cl, kMaxLTail3, nl_out); });
    };
    // A model built for a device runs the same quadrature there (quad3d.hip)
    // and keeps its node sets in device memory; a host-only model runs it on
    // up to 16 host threads.
    const bool on_device = p->device >= 0 && nl > 0;
    LeafQuad3 dq;
    if (on_device) {
        std::vector<double> nets(64 * (size_t)nl), box(6 * (size_t)nl), lnd;
        std::vector<Trim3> curves;
        std::vector<int64_t> coff(1, 0);
        for (int li = 0; li < nl; ++li) {
            const Patch &pt = leaves[li];
            std::memcpy(&nets[64 * (size_t)li], pt.h, sizeof(pt.h));
            patch_aabb(pt, &LO[3 * li], &HI[3 * li]);
            for (int a = 0; a < 3; ++a) {
                box[6 * (size_t)li + a] = LO[3 * li + a];
                box[6 * (size_t)li + 3 + a] = HI[3 * li + a];
            }
            if (pt.trims.empty()) {
                Trim3 e;
                std::memset(&e, 0, sizeof e);
                const double P[3][3] = {{1, 0, 1}, {1, 0.5, 1}, {1, 1, 1}};
                for (int j = 0; j < 3; ++j)
                    for (int q = 0; q < 3; ++q) e.h[3 * j + q] = P[j][q];
                curves.push_back(e);
            } else {
                curves.insert(curves.end(), pt.trims.begin(), pt.trims.end());
            }
            coff.push_back((int64_t)curves.size());
        }
        double rx[4][kMaxQuadRule] = {}, rw[4][kMaxQuadRule] = {};
        int rn[4];
        for (int r = 0; r < 3; ++r) {
            rn[r] = kLeafRules[r];
            std::copy(lx[r].begin(), lx[r].end(), rx[r]);
            std::copy(lw[r].begin(), lw[r].end(), rw[r]);
        }
        rn[3] = g;
        std::copy(gx.begin(), gx.end(), rx[3]);
        std::copy(gw.begin(), gw.end(), rw[3]);
        const gwn_status s = leafquad3d_moments(p->device, nets, curves, coff, box, rx, rw, rn, dq, U, Wt, WC, LC,
                                                lnd, qcount, err);
        if (s != GWN_OK) return s;
        std::memcpy(LN.data(), lnd.data(), lnd.size() * sizeof(double));
    } else {
        const int nthreads = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
        const int per = (nl + nthreads - 1) / nthreads;
        std::vector<std::thread> pool;
        for (int t = 0; t < nthreads && t * per < nl; ++t)
            pool.emplace_back([&, t] {
                for (int li = t * per; li < std::min(nl, (t + 1) * per); ++li) leaf_work(li);
            });
        for (auto &th : pool) th.join();
    }
    if (!build_tree(3, nl, LO.data(), HI.data(), U.data(), Wt.data(), WC.data(), m.lo, m.hi, m.tree, err, p->device))
        return err.rfind("device BVH", 0) == 0 ? GWN_EHIP : GWN_EINVAL;
    if (m.tree.depth > kStackDepth) {
        err = "BVH depth " + std::to_string(m.tree.depth) + " exceeds the traversal stack";
        return GWN_EOVERFLOW;
    }
    // multipole up-sweep: each node's moments are its children's (or, for a
    // leaf, its own) translated to the node's centroid.  The nodes of one
    // depth are independent, so the sweep runs depth by depth from the
    // deepest, each depth over host threads.  Stored scaled by 1/r^(l+1)
    // (r = AABB half diagonal), which keeps the FP32 mirror in range.
    {
        const size_t nn = m.tree.nodes.size();
        std::vector<cplx> NN(nn * kMpoleTermsTail, cplx(0, 0));
        std::vector<int> depth(nn, 0);
        int max_depth = 0;
        for (size_t ii = 0; ii < nn; ++ii) {   // a parent precedes its children
            const HostNode &h = m.tree.nodes[ii];
            if (!h.is_leaf) depth[ii + 1] = depth[h.right] = depth[ii] + 1;
            max_depth = std::max(max_depth, depth[ii]);
        }
        std::vector<std::vector<int>> level(max_depth + 1);
        for (size_t ii = 0; ii < nn; ++ii) level[depth[ii]].push_back((int)ii);
        auto up = [&](int ii) {
            const HostNode &h = m.tree.nodes[ii];
            cplx *dst = &NN[(size_t)ii * kMpoleTermsTail];
            if (h.is_leaf) {
                mpole_translate(&LN[(size_t)h.leaf * kMpoleTermsTail], &LC[3 * (size_t)h.leaf], h.c, kMaxLTail3,
                                dst);
            } else {
                const HostNode &a = m.tree.nodes[ii + 1], &b = m.tree.nodes[h.right];
                mpole_translate(&NN[(size_t)(ii + 1) * kMpoleTermsTail], a.c, h.c, kMaxLTail3, dst);
                mpole_translate(&NN[(size_t)h.right * kMpoleTermsTail], b.c, h.c, kMaxLTail3, dst);
            }
        };
        const int nthreads = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
        for (int d = max_depth; d >= 0; --d) {
            const std::vector<int> &lv = level[d];
            const int nt = std::min<int>(nthreads, (int)lv.size() / 64 + 1);
            if (nt == 1) {
                for (int ii : lv) up(ii);
                continue;
            }
            std::vector<std::thread> pool;
            for (int t = 0; t < nt; ++t)
                pool.emplace_back([&, t] {
                    for (size_t k = t; k < lv.size(); k += nt) up(lv[k]);
                });
            for (auto &th : pool) th.join();
        }
        // per node, the largest magnitude of each degree's term at unit
        // distance over kTailDirs directions (a Fibonacci lattice of the
        // sphere), for far_beta3d
        m.tail3.assign(nn * kMaxLTail3, 0.0);
        {
            constexpr int kTailDirs = 256;
            double dirs[kTailDirs][3];
            for (int k = 0; k < kTailDirs; ++k) {
                const double z = 1.0 - (2.0 * k + 1.0) / kTailDirs, s = std::sqrt(std::max(0.0, 1.0 - z * z));
                const double ph = 2.399963229728653 * k;   // golden angle
                dirs[k][0] = s * std::cos(ph);
                dirs[k][1] = s * std::sin(ph);
                dirs[k][2] = z;
            }
            const int nthreads = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
            std::vector<std::thread> pool;
            for (int t = 0; t < nthreads; ++t)
                pool.emplace_back([&, t] {
                    double T[kMaxLTail3];
                    for (size_t ii = t; ii < nn; ii += nthreads) {
                        double *A = &m.tail3[ii * kMaxLTail3];
                        for (int k = 0; k < kTailDirs; ++k) {
                            mpole_degree_terms(dirs[k], &NN[ii * kMpoleTermsTail], kMaxLTail3, T);
                            for (int l = 0; l < kMaxLTail3; ++l) A[l] = std::max(A[l], std::fabs(T[l]));
                        }
                    }
                });
            for (auto &th : pool) th.join();
        }
        m.mpole.assign(nn * kMpoleStride, 0.0);
        for (size_t ii = 0; ii < nn; ++ii) {
            const double r = m.tree.nodes[ii].r;
            const double ir = r > 0.0 ? 1.0 / r : 1.0;
            double *o = &m.mpole[ii * kMpoleStride];
            o[0] = ir;
            for (int l = 1; l <= kMaxL3; ++l) {
                const double sc = std::pow(ir, l + 1);
                for (int mm = 0; mm <= l; ++mm) {
                    const cplx v = NN[ii * kMpoleTermsTail + mp_index(l, mm)] * sc;
                    o[2 + 2 * mp_index(l, mm)] = v.real();
                    o[3 + 2 * mp_index(l, mm)] = v.imag();
                }
            }
        }
    }
    // leaves in BVH leaf order
    m.leaf_src.clear();
    m.leaf_h.clear();
    m.leaf_trim_begin.clear();
    m.leaf_trim_count.clear();
    m.qnodes.clear();
    m.leaf_q_begin.clear();
    m.leaf_q_count.clear();
    m.leaf_q_rules.clear();
    {   // hundreds of MB of node sets: one allocation instead of regrowth
        size_t tot = 0;
        for (const auto &v : qn) tot += v.size();
        m.qnodes.reserve(tot);
        m.leaf_h.reserve(64 * (size_t)nl);
    }
    std::vector<int64_t> qbase(on_device ? nl : 0);
    int64_t qtotal = 0;
    for (auto &nd : m.tree.nodes)
        if (nd.is_leaf) {
            const int src = nd.leaf;
            nd.leaf = (int)m.leaf_src.size();
            const Patch &pt = leaves[src];
            m.leaf_src.push_back(pt.src);
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j)
                    for (int k = 0; k < 4; ++k) m.leaf_h.push_back(pt.h[i][j][k]);
            m.leaf_trim_begin.push_back((int32_t)m.trims.size());
            m.leaf_trim_count.push_back((int32_t)pt.trims.size());
            m.trims.insert(m.trims.end(), pt.trims.begin(), pt.trims.end());
            const int64_t cnt = on_device ? (int64_t)qcount[src][0] + qcount[src][1] + qcount[src][2]
                                          : (int64_t)qn[src].size();
            m.leaf_q_begin.push_back(qtotal);
            m.leaf_q_count.push_back(cnt);
            m.leaf_q_rules.push_back(qcount[src]);
            if (on_device) qbase[src] = qtotal;
            else m.qnodes.insert(m.qnodes.end(), qn[src].begin(), qn[src].end());
            qtotal += cnt;
        }
    if (on_device) {
        const gwn_status s = leafquad3d_nodes(dq, qbase, qtotal, &m.d_qnodes, err);
        if (s != GWN_OK) return s;
        m.n_qnodes_dev = qtotal;
    }
    return GWN_OK;
}

// The order-p expansion keeps the degrees l <= p + 1; its error at distance
// rho is estimated by the first two omitted degrees, the second carrying a
// geometric bound on the rest (the degree-l term decays as rho^-(l+1), and
// successive degrees shrink at least as r / rho):
//   E(rho) = 2 [A_{p+2} rho^-(p+3) + A_{p+3} rho^-(p+4) / (1 - r / rho)],
// the factor 2 for the sampled directions' maximum.  E falls with rho, so
// the factor is found by bisection.
double far_beta3d(const double *A, double r, int order, double tol)
{
    const int l1 = order + 2, l2 = order + 3;
    if (l2 > kMaxLTail3 || !(tol > 0.0) || !(r > 0.0)) return HUGE_VAL;
    const double budget = 4.0 * kPi * tol;
    auto err = [&](double beta) {
        const double rho = beta * r;
        return 2.0 * (A[l1 - 1] * std::pow(rho, -(l1 + 1)) + A[l2 - 1] * std::pow(rho, -(l2 + 1)) / (1.0 - 1.0 / beta));
    };
    if (err(kBetaMin3) <= budget) return kBetaMin3;
    double lo = kBetaMin3, hi = 64.0;
    if (err(hi) > budget) return HUGE_VAL;
    for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (err(mid) <= budget) hi = mid; else lo = mid;
    }
    return hi;
}

void pack3d(const Model &m, std::vector<Node3> &nodes, std::vector<Prim3> &prims)
{
    const auto &T = m.tree.nodes;
    // end of each node's DFS subtree (a leaf's is the next index)
    std::vector<int32_t> end(T.size());
    for (size_t i = T.size(); i-- > 0;) end[i] = T[i].is_leaf ? (int32_t)i + 1 : end[T[i].right];
    nodes.assign(T.size(), Node3{});
    for (size_t i = 0; i < T.size(); ++i) {
        const HostNode &h = T[i];
        Node3 &n = nodes[i];
        std::memset(&n, 0, sizeof n);
        for (int a = 0; a < 3; ++a) n.c[a] = h.c[a];
        n.r2 = h.r * h.r;
        // the FP32 pass of the mixed form keeps r^2 (its factor is
        // beta_mixed); the FP64 test of an error-budgeted model compares
        // with (beta_c r)^2 at beta = 1
        double far_r2 = n.r2;
        if (m.params.far_tol > 0.0 && h.r > 0.0) {
            const double bc = far_beta3d(&m.tail3[i * kMaxLTail3], h.r, m.params.taylor_order, m.params.far_tol);
            far_r2 = std::isfinite(bc) ? (bc * h.r) * (bc * h.r) : HUGE_VAL;
        }
        if (h.is_leaf) {
            for (int a = 0; a < 3; ++a) { n.t[a] = h.lo[a]; n.t[3 + a] = h.hi[a]; }
            n.right = -1 - h.leaf;
            n.aux = m.leaf_q_begin[h.leaf];
            n.count = (int32_t)m.leaf_q_count[h.leaf];
            for (int r = 0; r < 3; ++r) n.t[6 + r] = (double)m.leaf_q_rules[h.leaf][r];
        } else {
            const double *M0 = h.M.data(), *M1 = M0 + 3, *M2 = M1 + 9;
            auto m1 = [&](int j, int k) { return M1[3 * j + k]; };
            auto m2 = [&](int i2, int j, int k) { return M2[9 * i2 + 3 * j + k]; };
            for (int a = 0; a < 3; ++a) n.t[a] = M0[a];
            n.t[3] = m1(0, 0); n.t[4] = m1(1, 1); n.t[5] = m1(2, 2);
            n.t[6] = m1(0, 1) + m1(1, 0); n.t[7] = m1(0, 2) + m1(2, 0); n.t[8] = m1(1, 2) + m1(2, 1);
            for (int k = 0; k < 3; ++k) {
                double a = 0, b = 0;
                for (int j = 0; j < 3; ++j) { a += m2(k, j, j); b += m2(j, j, k); }
                n.t[9 + k] = 2.0 * a + b;
            }
            // cubic form sum_ijk M2_ijk s_i s_j s_k: coefficient of each monomial
            // is the sum of M2 over the index triples with that multiset
            static const int mono[10][3] = {{0, 0, 0}, {1, 1, 1}, {2, 2, 2}, {0, 0, 1}, {0, 0, 2},
                                            {1, 1, 0}, {1, 1, 2}, {2, 2, 0}, {2, 2, 1}, {0, 1, 2}};
            for (int t = 0; t < 10; ++t) {
                int want[3] = {0, 0, 0};
                for (int r = 0; r < 3; ++r) want[mono[t][r]]++;
                double s = 0;
                for (int i2 = 0; i2 < 3; ++i2)
                    for (int j = 0; j < 3; ++j)
                        for (int k = 0; k < 3; ++k) {
                            int cnt[3] = {0, 0, 0};
                            cnt[i2]++; cnt[j]++; cnt[k]++;
                            if (cnt[0] == want[0] && cnt[1] == want[1] && cnt[2] == want[2]) s += m2(i2, j, k);
                        }
                n.t[12 + t] = s;
            }
            n.right = h.right;
            n.aux = 0;
            n.count = 0;
        }
        for (int a = 0; a < 3; ++a) n.fc[a] = (float)n.c[a];
        n.fr2 = (float)n.r2;
        n.r2 = far_r2;
        n.escape = end[i];
        for (int k = 0; k < 22; ++k) n.ft[k] = (float)n.t[k];
    }
    prims.assign(m.leaf_src.size(), Prim3{});
    for (size_t l = 0; l < prims.size(); ++l) {
        std::memcpy(prims[l].h, &m.leaf_h[64 * l], sizeof(double) * 64);
        prims[l].trim_begin = m.leaf_trim_begin[l];
        prims[l].trim_count = m.leaf_trim_count[l];
    }
}

}  // namespace gwn
