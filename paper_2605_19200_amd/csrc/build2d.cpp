// Host preprocessing of a 2D model (Alg. 1, threaded preprocessing):
//   AdaptiveSubdivision -> ComputeUncenteredMoments -> ConstructBVH ->
//   SumUncenteredMomentsUpTree -> CenterMomentsInPlace.
//
// Curves of degree 1..3 are degree-elevated to cubics (exact) so the kernels
// handle one shape of record; the original degree is kept for the straight
// segment fast path.
//
// Moments use the chord substitution of Sec. 3.1: far from a curve, the curve
// subtends the same angle as the segment joining its end points (the closed
// loop curve + reversed chord lies in the control polygon's convex hull, hence
// in its AABB, and the far test with beta >= 2 keeps q outside every AABB of an
// accepted cluster).  The uncentered moments of a segment a -> b with
// d = b - a and normal measure n ds = N ds, N = (d_y, -d_x) (outward for a
// counter-clockwise loop) are exact:
//   int n      = N
//   int x (x) n = (a + d/2) (x) N
//   int x (x) x (x) n = (a a^T + (a d^T + d a^T)/2 + d d^T / 3) (x) N
// and the centroid weight is the chord length with its midpoint.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "gwn_internal.h"

namespace gwn {

namespace {

// f(i) for i in [0, n) on up to 16 host threads, interleaved so that the
// large subtrees near the top of the DFS order spread over all threads.
template <class F>
void for_nodes(int n, F f)
{
    const int nt = std::max(1, std::min<int>({16, (int)std::thread::hardware_concurrency(), n / 256 + 1}));
    if (nt == 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&, t] {
            for (int i = t; i < n; i += nt) f(i);
        });
    for (auto &th : pool) th.join();
}

struct Cubic {
    double h[12];  // (wx, wy, w) x 4
    int degree;
    int64_t src;
};

void elevate_to_cubic(const double *xy, const double *w, int deg, double *h)
{
    double p[4][3];
    for (int i = 0; i <= deg; ++i) {
        p[i][0] = xy[2 * i] * w[i];
        p[i][1] = xy[2 * i + 1] * w[i];
        p[i][2] = w[i];
    }
    int n = deg;
    while (n < 3) {
        double q[4][3];
        for (int k = 0; k < 3; ++k) {
            q[0][k] = p[0][k];
            q[n + 1][k] = p[n][k];
        }
        for (int i = 1; i <= n; ++i) {
            double a = (double)i / (n + 1);
            for (int k = 0; k < 3; ++k) q[i][k] = a * p[i - 1][k] + (1.0 - a) * p[i][k];
        }
        ++n;
        std::memcpy(p, q, sizeof p);
    }
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 3; ++k) h[3 * i + k] = p[i][k];
}

void split_half(const double *h, double *L, double *R)
{
    // de Casteljau at t = 1/2 in homogeneous coordinates
    double a[4][3];
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 3; ++k) a[i][k] = h[3 * i + k];
    for (int k = 0; k < 3; ++k) {
        double b0 = 0.5 * (a[0][k] + a[1][k]), b1 = 0.5 * (a[1][k] + a[2][k]), b2 = 0.5 * (a[2][k] + a[3][k]);
        double c0 = 0.5 * (b0 + b1), c1 = 0.5 * (b1 + b2);
        double d0 = 0.5 * (c0 + c1);
        L[k] = a[0][k]; L[3 + k] = b0; L[6 + k] = c0; L[9 + k] = d0;
        R[k] = d0; R[3 + k] = c1; R[6 + k] = b2; R[9 + k] = a[3][k];
    }
}

void aabb(const double *h, double *lo, double *hi)
{
    lo[0] = lo[1] = INFINITY;
    hi[0] = hi[1] = -INFINITY;
    lo[2] = hi[2] = 0.0;
    for (int i = 0; i < 4; ++i) {
        double x = h[3 * i] / h[3 * i + 2], y = h[3 * i + 1] / h[3 * i + 2];
        lo[0] = std::min(lo[0], x); hi[0] = std::max(hi[0], x);
        lo[1] = std::min(lo[1], y); hi[1] = std::max(hi[1], y);
    }
}

}  // namespace

gwn_status build2d_host(const gwn_curves2d *c, const gwn_params *p, Model &m, std::string &err)
{
    const int64_t n = c->n_curves;
    if (n < 0) { err = "n_curves < 0"; return GWN_EINVAL; }
    if (n > 0 && (!c->degree || !c->cp_offset || !c->cp_xy || !c->cp_w)) {
        err = "NULL curve array";
        return GWN_EINVAL;
    }
    if (n > (int64_t)1 << 28) { err = "too many curves"; return GWN_EINVAL; }
    if (n > 0 && c->cp_offset[0] != 0) { err = "cp_offset[0] must be 0"; return GWN_EINVAL; }
    m.dim = 2;
    m.params = *p;
    m.n_input = n;
    double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
    std::vector<Cubic> work;
    work.reserve((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        int d = c->degree[i];
        if (d < 1 || d > 3) { err = "curve " + std::to_string(i) + ": degree must be 1..3"; return GWN_EINVAL; }
        int64_t a = c->cp_offset[i], b = c->cp_offset[i + 1];
        if (b - a != d + 1) { err = "curve " + std::to_string(i) + ": cp_offset does not match degree"; return GWN_EINVAL; }
        for (int64_t k = a; k < b; ++k) {
            double x = c->cp_xy[2 * k], y = c->cp_xy[2 * k + 1], w = c->cp_w[k];
            if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(w)) {
                err = "curve " + std::to_string(i) + ": non-finite control data";
                return GWN_EINVAL;
            }
            if (!(w > 0.0)) { err = "curve " + std::to_string(i) + ": weights must be > 0"; return GWN_EINVAL; }
            lo[0] = std::min(lo[0], x); hi[0] = std::max(hi[0], x);
            lo[1] = std::min(lo[1], y); hi[1] = std::max(hi[1], y);
        }
        Cubic cu;
        elevate_to_cubic(c->cp_xy + 2 * a, c->cp_w + a, d, cu.h);
        cu.degree = d;
        cu.src = i;
        work.push_back(cu);
    }
    if (n == 0) { lo[0] = lo[1] = 0; hi[0] = hi[1] = 0; }
    m.lo[0] = lo[0]; m.lo[1] = lo[1]; m.hi[0] = hi[0]; m.hi[1] = hi[1];
    m.lo[2] = m.hi[2] = 0;
    m.diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]));

    // AdaptiveSubdivision (Sec. 3.2): bisect while the AABB diagonal is not
    // below max_diag_frac of the model diagonal.  Depth is capped at 40.
    // The test compares the squared diagonal with the squared limit, in
    // plain IEEE operations, as the device version does (moments2d.hip): a
    // model built for a device subdivides there, to the same leaves.
    const double limit = p->max_diag_frac * m.diag, limit2 = limit > 0 ? limit * limit : 0.0;
    std::vector<Cubic> leaves;
    leaves.reserve(work.size());
    if (p->device >= 0 && !work.empty()) {
        std::vector<double> cubics(12 * work.size()), leaf_h;
        std::vector<int32_t> leaf_curve;
        for (size_t i = 0; i < work.size(); ++i) std::memcpy(&cubics[12 * i], work[i].h, sizeof work[i].h);
        const gwn_status s = subdiv2d_device(p->device, cubics, limit2, leaf_h, leaf_curve, err);
        if (s != GWN_OK) return s;
        for (size_t l = 0; l < leaf_curve.size(); ++l) {
            Cubic cu = work[leaf_curve[l]];
            std::memcpy(cu.h, &leaf_h[12 * l], sizeof cu.h);
            leaves.push_back(cu);
        }
    } else {
        struct Item { Cubic c; int depth; };
        std::vector<Item> st;
        for (int64_t i = (int64_t)work.size() - 1; i >= 0; --i) st.push_back({work[i], 0});
        while (!st.empty()) {
            Item it = st.back();
            st.pop_back();
            double l[3], h[3];
            aabb(it.c.h, l, h);
            const double dx = h[0] - l[0], dy = h[1] - l[1];
            if (limit2 > 0 && dx * dx + dy * dy >= limit2 && it.depth < 40) {
                Cubic L = it.c, R = it.c;
                split_half(it.c.h, L.h, R.h);
                st.push_back({R, it.depth + 1});
                st.push_back({L, it.depth + 1});
            } else {
                leaves.push_back(it.c);
            }
        }
    }
    const int nl = (int)leaves.size();
    if ((int64_t)nl > ((int64_t)1 << 30)) { err = "too many leaves"; return GWN_EINVAL; }

    // ComputeUncenteredMoments: exact chord moments per leaf.
    const int nm = n_moments(2);
    std::vector<double> LO(3 * (size_t)nl), HI(3 * (size_t)nl), U((size_t)nl * nm), Wt(nl), WC(3 * (size_t)nl);
    for (int i = 0; i < nl; ++i) {
        const double *h = leaves[i].h;
        aabb(h, &LO[3 * i], &HI[3 * i]);
        double ax = h[0] / h[2], ay = h[1] / h[2], bx = h[9] / h[11], by = h[10] / h[11];
        double dx = bx - ax, dy = by - ay;
        double N[2] = {dy, -dx};
        double A[2] = {ax, ay}, D[2] = {dx, dy};
        double *u = &U[(size_t)i * nm];
        u[0] = N[0];
        u[1] = N[1];
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 2; ++k) u[2 + 2 * j + k] = (A[j] + 0.5 * D[j]) * N[k];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                double s = A[a] * A[b] + 0.5 * (A[a] * D[b] + D[a] * A[b]) + D[a] * D[b] / 3.0;
                for (int k = 0; k < 2; ++k) u[6 + (2 * a + b) * 2 + k] = s * N[k];
            }
        double len = std::hypot(dx, dy);
        Wt[i] = len;
        WC[3 * i] = len * 0.5 * (ax + bx);
        WC[3 * i + 1] = len * 0.5 * (ay + by);
        WC[3 * i + 2] = 0;
    }
    if (!build_tree(2, nl, LO.data(), HI.data(), U.data(), Wt.data(), WC.data(), m.lo, m.hi, m.tree, err, p->device))
        return err.rfind("device BVH", 0) == 0 ? GWN_EHIP : GWN_EINVAL;
    if (m.tree.depth > kStackDepth) {
        err = "BVH depth " + std::to_string(m.tree.depth) + " exceeds the traversal stack";
        return GWN_EOVERFLOW;
    }
    // Complex moments about each node's own centroid, summed directly over
    // the chords of its subtree: m_k = sum (b-c)^{k+1} - (a-c)^{k+1} / (k+1),
    // written as (b - a) sum_j (b-c)^j (a-c)^{k-j} / (k+1) to avoid the
    // cancellation of short chords.  (Summing uncentered moments and shifting
    // them, as done for the Cartesian order-2 moments, loses about
    // k log10(|c| / r) digits at order k.)  A DFS subtree is the contiguous
    // node range [i, end_i).  Then the truncation data of each cluster for the
    // error-budgeted far test, in the node's scaled variables
    // a' = (a - c) / r, b' = (b - c) / r: the scaled moments
    // m_k / r^(k+1) = (b' - a') s'_k / (k + 1) up to kTailOrder2D, the scaled
    // chord length and rho = R / r.  A model built for a device computes both
    // there (moments2d.hip); a host-only model on up to 16 host threads.
    {
        const int nn = (int)m.tree.nodes.size();
        const int K = kMaxOrder2D + 1;
        std::vector<int> end(nn);
        for (int i = nn - 1; i >= 0; --i) {
            const HostNode &nd = m.tree.nodes[i];
            end[i] = nd.is_leaf ? i + 1 : end[nd.right];
        }
        if (p->device >= 0 && nn > 1) {
            std::vector<double> chord_ends;
            chord_ends.reserve(4 * (size_t)nl);
            for (const HostNode &nd : m.tree.nodes)
                if (nd.is_leaf) {
                    const double *hh = leaves[nd.leaf].h;
                    chord_ends.insert(chord_ends.end(), {hh[0] / hh[2], hh[1] / hh[2], hh[9] / hh[11], hh[10] / hh[11]});
                }
            const gwn_status s = moments2d_device(p->device, m.tree.nodes, end, chord_ends, m.cmom2, m.tail2, err);
            if (s != GWN_OK) return s;
        } else {
            m.cmom2.assign((size_t)nn * 2 * K, 0.0);
            for_nodes(nn, [&](int i) {
                const HostNode &nd = m.tree.nodes[i];
                if (nd.is_leaf) return;
                double *out = &m.cmom2[(size_t)i * 2 * K];
                for (int j = i; j < end[i]; ++j) {
                    const HostNode &lf = m.tree.nodes[j];
                    if (!lf.is_leaf) continue;
                    const double *hh = leaves[lf.leaf].h;
                    double ar = hh[0] / hh[2] - nd.c[0], ai = hh[1] / hh[2] - nd.c[1];
                    double br = hh[9] / hh[11] - nd.c[0], bi = hh[10] / hh[11] - nd.c[1];
                    double dr = br - ar, di = bi - ai;
                    // s_k = sum_{j<=k} b^j a^{k-j}: s_0 = 1, s_k = b s_{k-1} + a^k
                    double sr = 1.0, si = 0.0, pr = 1.0, pi = 0.0;  // p = a^k
                    for (int k = 0; k < K; ++k) {
                        if (k > 0) {
                            double npr = pr * ar - pi * ai, npi = pr * ai + pi * ar;
                            pr = npr; pi = npi;
                            double nsr = br * sr - bi * si + pr, nsi = br * si + bi * sr + pi;
                            sr = nsr; si = nsi;
                        }
                        out[2 * k] += (dr * sr - di * si) / (k + 1);
                        out[2 * k + 1] += (dr * si + di * sr) / (k + 1);
                    }
                }
            });
            m.tail2.assign((size_t)nn * kTailStride2D, 0.0);
            for_nodes(nn, [&](int i) {
                const HostNode &nd = m.tree.nodes[i];
                if (nd.is_leaf || !(nd.r > 0)) return;
                const double ir = 1.0 / nd.r;
                double acc[2 * (kTailOrder2D + 1)] = {};
                double len = 0.0;
                for (int j = i; j < end[i]; ++j) {
                    const HostNode &lf = m.tree.nodes[j];
                    if (!lf.is_leaf) continue;
                    const double *hh = leaves[lf.leaf].h;
                    const double ar = (hh[0] / hh[2] - nd.c[0]) * ir, ai = (hh[1] / hh[2] - nd.c[1]) * ir;
                    const double br = (hh[9] / hh[11] - nd.c[0]) * ir, bi = (hh[10] / hh[11] - nd.c[1]) * ir;
                    const double dr = br - ar, di = bi - ai;
                    len += std::hypot(dr, di);
                    double sr = 1.0, si = 0.0, pr = 1.0, pi = 0.0;
                    for (int k = 0; k <= kTailOrder2D; ++k) {
                        if (k > 0) {
                            const double npr = pr * ar - pi * ai, npi = pr * ai + pi * ar;
                            pr = npr; pi = npi;
                            const double nsr = br * sr - bi * si + pr, nsi = br * si + bi * sr + pi;
                            sr = nsr; si = nsi;
                        }
                        acc[2 * k] += (dr * sr - di * si) / (k + 1);
                        acc[2 * k + 1] += (dr * si + di * sr) / (k + 1);
                    }
                }
                double *t = &m.tail2[(size_t)i * kTailStride2D];
                for (int k = 0; k <= kTailOrder2D; ++k) t[k] = std::hypot(acc[2 * k], acc[2 * k + 1]);
                t[kTailOrder2D + 1] = len;
            });
        }
        for (int i = 0; i < nn; ++i) {
            const HostNode &nd = m.tree.nodes[i];
            if (nd.is_leaf || !(nd.r > 0)) continue;
            double R2 = 0.0;
            for (int a = 0; a < 2; ++a) {
                const double e = std::max(nd.c[a] - nd.lo[a], nd.hi[a] - nd.c[a]);
                R2 += e * e;
            }
            m.tail2[(size_t)i * kTailStride2D + kTailOrder2D + 2] = std::sqrt(R2) / nd.r;
        }
    }
    // leaves in BVH leaf order (order of appearance in the DFS layout)
    m.leaf_src.clear();
    m.leaf_h.clear();
    m.leaf_degree.clear();
    std::vector<int> leaf_pos(nl, -1);
    for (auto &nd : m.tree.nodes)
        if (nd.is_leaf) {
            int src = nd.leaf;
            nd.leaf = (int)m.leaf_src.size();
            leaf_pos[src] = nd.leaf;
            m.leaf_src.push_back(leaves[src].src);
            m.leaf_h.insert(m.leaf_h.end(), leaves[src].h, leaves[src].h + 12);
            m.leaf_degree.push_back(leaves[src].degree);
        }
    return GWN_OK;
}

// Truncation error of the order-p chord expansion of a cluster at
// x = r / ||q - c||, in turns.  With the scaled moments mt_k = m_k / r^(k+1)
// the omitted terms are sum_{k>p} mt_k v^(k+1), |v| = x (Sec. 3.1, the
// series of Eq. taylor carried on in complex form).  The terms up to
// kTailOrder2D are taken with their exact magnitudes; beyond, every chord
// point lies within R = rho r of the centroid, so |mt_k| <= (L / r) rho^k and
// the rest sums to at most (L / r) rho^(J+1) x^(J+2) / (1 - rho x).  The bound
// grows with x, so the largest admissible x is found by bisection.
double far_beta2d(const double *tail, int order, double tol)
{
    const int J = kTailOrder2D;
    const double len = tail[J + 1], rho = tail[J + 2];
    auto bound = [&](double x) -> double {
        if (rho * x >= 1.0) return HUGE_VAL;
        double s = 0.0, xp = std::pow(x, order + 2);
        for (int k = order + 1; k <= J; ++k) {
            s += tail[k] * xp;
            xp *= x;
        }
        s += len * std::pow(rho, J + 1) * xp / (1.0 - rho * x);
        return s / (2.0 * kPi);
    };
    double lo = 0.0, hi = 0.5;       // beta >= 2: the chord substitution holds outside the AABB
    if (bound(hi) <= tol) return 2.0;
    for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (bound(mid) <= tol) lo = mid;
        else hi = mid;
    }
    return lo > 0.0 ? 1.0 / lo : HUGE_VAL;
}

}  // namespace gwn
