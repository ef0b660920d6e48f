// Trim loops of a patch split in two (Alg. 1 AdaptiveSubdivision for
// trimmed patches, Sec. 3.2): the visible region D of the parameter square
// is cut by the line x_dir = c, and each half keeps D restricted to it, as
// closed loops mapped to the half's own unit square.
//
// Each trim curve is a rational quadratic in homogeneous form (w u, w v, w).
// Its crossings with the line are the roots in (0, 1) of the quadratic
// (X(t) - c W(t)) in Bernstein form; the curve is split there (exact
// homogeneous de Casteljau) and the pieces on the kept side are kept.  The
// boundary of D restricted to the half also runs along the cut line: walking
// the kept pieces of a loop with D on the left, the boundary leaves the half
// at an exit crossing and comes back at the next crossing met when walking
// along the line with the half on the left, which must be an entry; the
// straight segment between the two closes the loop.  Loops that do not meet
// the line are kept whole or dropped by the side they lie on.
//
// Cuts that touch a loop tangentially or pass through a junction of two trim
// curves have no well-defined crossings; the function then reports failure
// and the caller moves the cut.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "gwn_internal.h"

namespace gwn {

namespace {

double coord(const double *h3, int axis) { return h3[axis] / h3[2]; }

// homogeneous point of the rational quadratic at t
void point_at(const Trim3 &c, double t, double p[3])
{
    const double s = 1.0 - t, b0 = s * s, b1 = 2.0 * s * t, b2 = t * t;
    for (int k = 0; k < 3; ++k) p[k] = b0 * c.h[k] + b1 * c.h[3 + k] + b2 * c.h[6 + k];
}

// The piece of the curve on [t0, t1] as a rational quadratic on [0, 1]:
// blossom values (t0, t0), (t0, t1), (t1, t1) of the control polygon.
Trim3 sub_curve(const Trim3 &c, double t0, double t1)
{
    auto blossom = [&](double a, double b, double out[3]) {
        double l0[3], l1[3];
        for (int k = 0; k < 3; ++k) {
            l0[k] = (1.0 - a) * c.h[k] + a * c.h[3 + k];
            l1[k] = (1.0 - a) * c.h[3 + k] + a * c.h[6 + k];
            out[k] = (1.0 - b) * l0[k] + b * l1[k];
        }
    };
    Trim3 r;
    std::memset(&r, 0, sizeof r);
    blossom(t0, t0, r.h);
    blossom(t0, t1, r.h + 3);
    blossom(t1, t1, r.h + 6);
    return r;
}

Trim3 segment(double x0, double y0, double x1, double y1, int dir)
{
    // (x, y) = coordinate across / along the cut; dir 0: x = u, 1: x = v
    Trim3 r;
    std::memset(&r, 0, sizeof r);
    const double P[3][2] = {{x0, y0}, {0.5 * (x0 + x1), 0.5 * (y0 + y1)}, {x1, y1}};
    for (int j = 0; j < 3; ++j) {
        r.h[3 * j + dir] = P[j][0];
        r.h[3 * j + 1 - dir] = P[j][1];
        r.h[3 * j + 2] = 1.0;
    }
    return r;
}

// Set the Euclidean end point (k = 0 start, 2 end) of a piece, keeping its
// weight: crossing points are snapped onto the cut line exactly so that
// pieces and closing segments share their end points bit for bit.
void snap(Trim3 &c, int k, double x, double y, int dir)
{
    const double w = c.h[3 * k + 2];
    c.h[3 * k + dir] = x * w;
    c.h[3 * k + 1 - dir] = y * w;
}

// Map curves from [lo, hi] along axis ax to [0, 1]; coordinates that land
// within rounding of 0 or 1 (points on the cut line or the square's edges)
// are set to it exactly, so the loops stay inside the unit square.
void to_half(std::vector<Trim3> &cs, int ax, double lo, double hi)
{
    for (auto &t : cs)
        for (int j = 0; j < 3; ++j) {
            double &h = t.h[3 * j + ax];
            const double w = t.h[3 * j + 2];
            h = (h - lo * w) / (hi - lo);
            const double x = h / w;
            if (std::fabs(x) < 1e-13) h = 0.0;
            if (std::fabs(x - 1.0) < 1e-13) h = w;
        }
}

}  // namespace

bool clip_trims_half(const std::vector<Trim3> &in, int dir, double c, bool low, std::vector<Trim3> &out)
{
    out.clear();
    const int ax = dir, ay = 1 - dir;
    const double tol_end = 1e-9;
    // loops: consecutive curves, closed when a curve ends at the loop's start
    std::vector<std::pair<size_t, size_t>> loops;
    {
        size_t b = 0;
        for (size_t k = 0; k < in.size(); ++k) {
            const double su = coord(in[b].h, 0), sv = coord(in[b].h, 1);
            const double eu = coord(in[k].h + 6, 0), ev = coord(in[k].h + 6, 1);
            if (std::fabs(eu - su) <= 1e-12 && std::fabs(ev - sv) <= 1e-12) {
                loops.emplace_back(b, k + 1);
                b = k + 1;
            }
        }
        if (b != in.size()) return false;
    }
    // side of a point: true = kept
    auto kept = [&](double x) { return low ? x < c : x > c; };
    struct Cross {
        double y;
        int run_end;     // index of the run that ends here (exit), or -1
        int run_start;   // index of the run that starts here (entry), or -1
    };
    std::vector<Cross> cross;
    std::vector<std::vector<Trim3>> runs;           // kept chains, entry -> exit
    for (size_t L = 0; L < loops.size(); ++L) {
        // pieces of the loop in order, each tagged with its side; crossing
        // points between consecutive pieces
        struct P {
            Trim3 c;
            bool keep;
            double start_y;      // y of the crossing where it starts (NaN if none)
            double end_y;
        };
        std::vector<P> ps;
        for (size_t k = loops[L].first; k < loops[L].second; ++k) {
            const Trim3 &cv = in[k];
            double a[3];
            for (int j = 0; j < 3; ++j) a[j] = cv.h[3 * j + ax] - c * cv.h[3 * j + 2];
            const double x0 = coord(cv.h, ax), x2 = coord(cv.h + 6, ax);
            if (std::fabs(x0 - c) <= tol_end || std::fabs(x2 - c) <= tol_end) return false;
            // Bernstein -> power basis: A t^2 + B t + C
            const double A = a[0] - 2.0 * a[1] + a[2], B = 2.0 * (a[1] - a[0]), C = a[0];
            const double scale = std::fabs(a[0]) + std::fabs(a[1]) + std::fabs(a[2]);
            double roots[2];
            int nr = 0;
            if (std::fabs(A) <= 1e-14 * scale) {
                if (std::fabs(B) > 1e-14 * scale) roots[nr++] = -C / B;
            } else {
                const double disc = B * B - 4.0 * A * C;
                if (std::fabs(disc) <= 1e-12 * scale * scale) return false;   // tangency
                if (disc > 0.0) {
                    const double sq = std::sqrt(disc);
                    const double q = -0.5 * (B + std::copysign(sq, B));
                    roots[nr++] = q / A;
                    if (q != 0.0) roots[nr++] = C / q;
                }
            }
            double ts[4];
            int nt = 0;
            for (int r = 0; r < nr; ++r)
                if (roots[r] > 0.0 && roots[r] < 1.0) {
                    if (roots[r] < tol_end || roots[r] > 1.0 - tol_end) return false;
                    ts[nt++] = roots[r];
                }
            std::sort(ts, ts + nt);
            if (nt == 2 && ts[1] - ts[0] < 1e-9) return false;
            double t_prev = 0.0, y_prev = NAN;
            for (int r = 0; r <= nt; ++r) {
                const double t1 = r < nt ? ts[r] : 1.0;
                P p;
                p.c = sub_curve(cv, t_prev, t1);
                double mid[3];
                point_at(cv, 0.5 * (t_prev + t1), mid);
                p.keep = kept(mid[ax] / mid[2]);
                p.start_y = y_prev;
                if (r < nt) {
                    double pt[3];
                    point_at(cv, t1, pt);
                    p.end_y = pt[ay] / pt[2];
                    snap(p.c, 2, c, p.end_y, dir);
                } else {
                    p.end_y = NAN;
                }
                if (!std::isnan(p.start_y)) snap(p.c, 0, c, p.start_y, dir);
                ps.push_back(p);
                t_prev = t1;
                y_prev = p.end_y;
            }
        }
        // rotate so that the loop starts at a crossing (if any)
        size_t first = ps.size();
        for (size_t i = 0; i < ps.size(); ++i)
            if (!std::isnan(ps[i].start_y)) { first = i; break; }
        if (first == ps.size()) {   // no crossing: whole loop on one side
            if (ps[0].keep)
                for (auto &p : ps) out.push_back(p.c);
            continue;
        }
        std::rotate(ps.begin(), ps.begin() + first, ps.end());
        // runs of kept pieces between crossings
        for (size_t i = 0; i < ps.size();) {
            if (!ps[i].keep) { ++i; continue; }
            if (std::isnan(ps[i].start_y)) return false;
            std::vector<Trim3> run;
            const double y_in = ps[i].start_y;
            double y_out = NAN;
            while (i < ps.size() && ps[i].keep) {
                run.push_back(ps[i].c);
                y_out = ps[i].end_y;
                ++i;
                if (!std::isnan(y_out)) break;
            }
            if (std::isnan(y_out)) return false;
            const int id = (int)runs.size();
            runs.push_back(run);
            cross.push_back({y_in, -1, id});
            cross.push_back({y_out, id, -1});
        }
    }
    if (runs.empty()) {
        to_half(out, ax, low ? 0.0 : c, low ? c : 1.0);
        return true;
    }
    // walking along the cut line with the kept half on the left: +y for the
    // low half of a u cut and for the high half of a v cut, -y otherwise
    const bool up = (dir == 0) == low;
    std::sort(cross.begin(), cross.end(), [](const Cross &a, const Cross &b) { return a.y < b.y; });
    for (size_t i = 1; i < cross.size(); ++i)
        if (cross[i].y - cross[i - 1].y < 1e-12) return false;
    std::vector<int> pos_of_entry(runs.size()), pos_of_exit(runs.size());
    for (size_t i = 0; i < cross.size(); ++i) {
        if (cross[i].run_start >= 0) pos_of_entry[cross[i].run_start] = (int)i;
        if (cross[i].run_end >= 0) pos_of_exit[cross[i].run_end] = (int)i;
    }
    std::vector<char> used(runs.size(), 0);
    std::vector<Trim3> assembled;
    for (size_t r0 = 0; r0 < runs.size(); ++r0) {
        if (used[r0]) continue;
        size_t r = r0;
        for (size_t guard = 0; guard <= runs.size(); ++guard) {
            if (used[r]) return false;
            used[r] = 1;
            for (auto &t : runs[r]) assembled.push_back(t);
            const int ip = pos_of_exit[r];
            const int jp = up ? ip + 1 : ip - 1;
            if (jp < 0 || jp >= (int)cross.size() || cross[jp].run_start < 0) return false;
            assembled.push_back(segment(c, cross[ip].y, c, cross[jp].y, dir));
            r = (size_t)cross[jp].run_start;
            if (r == r0) break;
        }
        if (r != r0) return false;
    }
    out.insert(out.end(), assembled.begin(), assembled.end());
    to_half(out, ax, low ? 0.0 : c, low ? c : 1.0);
    return true;
}

}  // namespace gwn
