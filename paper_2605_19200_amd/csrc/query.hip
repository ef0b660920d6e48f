// Query phase of Alg. 1 on gfx950: space-filling-curve ordering of the
// queries, wavefront-coherent BVH traversal with the far-field Taylor
// approximation (Eq. taylor) and direct leaf evaluation (Sec. 3.3), the
// mixed-precision pass with FP64 reclassification near w = 0.5, and batched
// multi-model launches.
//
// Traversal scheme.  One lane per query; the 64 queries of a wave (adjacent
// along a Morton curve) walk the tree together with ONE stack of
// (node, lane mask) entries in LDS.  At an internal node each lane in the
// mask applies its own far test ||q - c||^2 > beta^2 r^2; lanes for which the
// cluster is far add its Taylor term, the others continue into the children
// (pushed with the mask of those lanes).  A lane therefore visits exactly the
// nodes of its own per-query depth-first (left child first) traversal, in the
// same order, so every result is bitwise independent of its wave mates.
// Node records are read at wave-uniform addresses (scalar loads).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "radix.h"
#include "gwn_internal.h"
#include "query_common.h"

namespace gwn {

// ---------------------------------------------------------------------------
// space-filling-curve keys
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t part1by1(uint64_t x)  // 24 bits -> 48
{
    x &= 0xffffffull;
    x = (x | (x << 16)) & 0x0000ffff0000ffffull;
    x = (x | (x << 8)) & 0x00ff00ff00ff00ffull;
    x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

__device__ __forceinline__ uint64_t part1by2(uint64_t x)  // 16 bits -> 48
{
    x &= 0xffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint64_t quantize(double v, double lo, double inv, double maxq)
{
    double t = (v - lo) * inv;
    t = fmin(fmax(t, 0.0), 1.0);  // NaN -> 0 or 1
    return (uint64_t)(t * maxq);
}

__device__ __forceinline__ int find_seg(const LaunchTable &T, int64_t row)
{
    int lo = 0, hi = T.n_seg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (T.qoff[mid] <= row) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_keys(LaunchTable T, int dim, const double *__restrict__ pts,
                                                 uint64_t *__restrict__ keys, int32_t *__restrict__ vals,
                                                 int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int s = find_seg(T, i);
    const DevModel &M = T.models[T.seg_model[s]];
    uint64_t code;
    if (dim == 2) {
        uint64_t x = quantize(pts[2 * i], M.lo[0], M.inv_ext[0], 16777215.0);
        uint64_t y = quantize(pts[2 * i + 1], M.lo[1], M.inv_ext[1], 16777215.0);
        code = part1by1(x) | (part1by1(y) << 1);
    } else {
        uint64_t x = quantize(pts[3 * i], M.lo[0], M.inv_ext[0], 65535.0);
        uint64_t y = quantize(pts[3 * i + 1], M.lo[1], M.inv_ext[1], 65535.0);
        uint64_t z = quantize(pts[3 * i + 2], M.lo[2], M.inv_ext[2], 65535.0);
        code = part1by2(x) | (part1by2(y) << 1) | (part1by2(z) << 2);
    }
    keys[i] = ((uint64_t)s << 48) | code;
    vals[i] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// 2D leaf: direct evaluation (Sec. 3.3)
// ---------------------------------------------------------------------------
// 1 / d for normal d > 0: hardware reciprocal refined by two Newton steps
// (within an ulp or two; no IEEE division sequence).
__device__ __forceinline__ double fast_rcp(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    return fma(r, fma(-d, r, 1.0), r);
}

__device__ __forceinline__ float fast_rcp(float d) { return __builtin_amdgcn_rcpf(d); }

// atan2(y, x) for finite (x, y) != (0, 0), absolute error ~1e-15.
// Octant reduction to t = min/max in [0, 1], then (t - 1) / (t + 1) above
// tan(pi/8), so the polynomial runs on |r| <= tan(pi/8); one division by a
// refined hardware reciprocal.  Coefficients: atan_coeffs.py.  They live in
// constant memory and arrive by scalar loads: as literals the compiler
// hoisted them out of the traversal loop into 16 vector registers and
// spilled them.
__constant__ double kAtanP[10] = {
    0.99999999999999933,  -0.33333333333221649, 0.19999999978414348,  -0.1428571266185861,
    0.11111048822077878,  -0.090895287796835464, 0.076735172520470213, -0.065058395774881372,
    0.05024193570775376,  -0.025307491891893075};

__device__ __forceinline__ double fast_atan2(double y, double x)
{
    const double ax = fabs(x), ay = fabs(y);
    const double mn = fmin(ax, ay), mx = fmax(ax, ay);
    const bool big = mn > 0.41421356237309503 * mx;
    double num = big ? mn - mx : mn;
    double den = big ? mn + mx : mx;
    if (den < 0x1p-900) { num *= 0x1p900; den *= 0x1p900; }   // keep the reciprocal normal
    const double rd = fast_rcp(den);
    double r = num * rd;
    r = fma(rd, fma(-den, r, num), r);
    const double s2 = r * r;
    double p = kAtanP[9];
#pragma unroll
    for (int k = 8; k >= 1; --k) p = fma(p, s2, kAtanP[k]);
    double a = fma(r * s2, p, r * kAtanP[0]);
    if (big) a += 0.78539816339744831;
    if (ay > ax) a = 1.5707963267948966 - a;
    if (x < 0.0) a = 3.1415926535897931 - a;
    return copysign(a, y);
}

// Signed angle at q (the origin of the translated frame) from a to b; 0 when
// q lies on the segment (the direct value of a straight piece through q).
__device__ __forceinline__ double chord_angle(double ax, double ay, double bx, double by)
{
    double cr = ax * by - ay * bx;
    double dt = ax * bx + ay * by;
    if (cr == 0.0 && dt <= 0.0) return 0.0;
    return fast_atan2(cr, dt);
}

// Sum of the chord angles seen from q (direct leaf contributions), without
// an arctangent per chord: the chord a -> b subtends arg(z), z = dot(a, b) +
// i cross(a, b), so the sum is the argument of the product of the z's plus
// 2 pi for every time the running argument passes +-pi.  Both arguments lie
// in (-pi, pi], so a pass past +pi can only happen when both are in [0, pi]
// and the product falls below the real axis, and past -pi only when both
// are negative and the product rises to or above it.  z and the product are
// rescaled by powers of two (exact), and one arctangent at the end gives
// the argument.  One complex multiply and a few sign tests per chord are
// cheaper than an FP64 arctangent.
struct AngleAcc {
    double pr, pi;      // product of the chords' (dot, cross), rescaled by powers of 2
    int turns;          // times the product's argument wrapped past +-pi
    double extra;       // terminal-piece angles
};

__device__ __forceinline__ void angle_init(AngleAcc &A) { A.pr = 1.0; A.pi = 0.0; A.turns = 0; A.extra = 0.0; }

__device__ __forceinline__ void angle_add_chord(AngleAcc &A, double cr, double dt)
{
    if (cr == 0.0 && dt <= 0.0) return;   // q on the chord or at an end point
    // z = dt + i cr has the chord's angle as argument; scale it exactly
    int ez;
    (void)frexp(fmax(fabs(dt), fabs(cr)), &ez);
    const double zr = ldexp(dt, -ez), zi = ldexp(cr, -ez);
    const double nr = A.pr * zr - A.pi * zi, ni = A.pr * zi + A.pi * zr;
    // both arguments in [0, pi] and the product below the real axis: the sum
    // passed pi; both in (-pi, 0) and the product at or above: passed -pi
    if (A.pi >= 0.0 && zi >= 0.0 && ni < 0.0) ++A.turns;
    else if (A.pi < 0.0 && zi < 0.0 && (ni > 0.0 || (ni == 0.0 && nr < 0.0))) --A.turns;
    int ep;
    (void)frexp(fmax(fabs(nr), fabs(ni)), &ep);
    A.pr = ldexp(nr, -ep);
    A.pi = ldexp(ni, -ep) + 0.0;   // no -0: its atan2 would be -pi where the count takes +pi
}

__device__ __forceinline__ double angle_total(const AngleAcc &A)
{
    return 6.283185307179586 * A.turns + fast_atan2(A.pi, A.pr) + A.extra;
}

__device__ __forceinline__ double lerp_exact(double a, double b, double t, double s)
{
    return fma(t, b, s * a);   // exact at t = 0 and t = 1
}

// Direct angle subtended by one cubic leaf at q, in radians.
// If q is outside the leaf's control-point AABB, the chord angle is exact
// (chord substitution, Sec. 3.1; AABB test instead of a hull test, Sec. 3.3).
// Otherwise the curve is bisected toward q: pieces are enumerated depth first
// as dyadic parameter intervals [k 2^-L, (k+1) 2^-L] (no stack: the next
// interval follows from (L, k)), each piece's control points are obtained by
// blossoming the leaf's control points, a piece whose AABB excludes q adds
// its chord angle, and a piece that still contains q when it is smaller than
// eps_on or after kMaxBisectLevel halvings (q on the curve) adds the mean of
// its two one-sided limits (the direct value).
// The end point of each piece is carried to the next so consecutive chords
// share their end points bit for bit.
// The box test runs in FP32 on q rounded to nearest: rounding is monotone
// and the box edges are floats rounded outward, so qf < lo_f implies q < lo
// (likewise above); a query that rounds onto an edge only takes the
// bisection path.
template <bool COUNT>
__device__ void leaf2d(const Hot2 *__restrict__ nd, const double *ends, const float *box,
                       const Prim2 *__restrict__ prims, double qx, double qy, float qxf, float qyf, double eps_on,
                       AngleAcc &A, Ctr &ctr, bool &overflow)
{
    if (COUNT) ctr.v[GWN_C_LEAVES]++;
    const bool outside = qxf < box[0] || qyf < box[1] || qxf > box[2] || qyf > box[3];
    if (outside || nd->degree == 1) {
        // chord from the end points held in the traversal record
        if (COUNT) { ctr.v[GWN_C_LEAF_FAST]++; ctr.v[GWN_C_ANGLES]++; }
        const double ax = ends[0] - qx, ay = ends[1] - qy, bx3 = ends[2] - qx, by3 = ends[3] - qy;
        angle_add_chord(A, ax * by3 - ay * bx3, ax * bx3 + ay * by3);
        return;
    }
    const int leaf = -1 - nd->right;
    const Prim2 *P = prims + leaf;
    double bx[4], by[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double w = P->h[3 * i + 2];
        bx[i] = fma(-qx, w, P->h[3 * i]);
        by[i] = fma(-qy, w, P->h[3 * i + 1]);
    }
    if (!(fabs(qx) < INFINITY && fabs(qy) < INFINITY)) { A.extra = NAN; return; }
    // On-boundary rule: a piece whose control points all lie within eps_on
    // of q (|x_i| / w_i < eps_on with w_i >= the leaf's smallest weight) is
    // terminal.
    const double wmin = fmin(fmin(P->h[2], P->h[5]), fmin(P->h[8], P->h[11]));
    const double on_tol = eps_on * wmin;
    int level = 1;
    uint64_t k = 0;
    double p0x = bx[0], p0y = by[0];
    for (int it = 0;; ++it) {
        if (it >= kMaxBisectIter) { overflow = true; A.extra = NAN; return; }
        const double inv = ldexp(1.0, -level);
        const double t0 = (double)k * inv, t1 = (double)(k + 1) * inv;
        const double s0 = 1.0 - t0, s1 = 1.0 - t1;
        // blossom levels at t0
        double ax1[3], ay1[3], ax2[2], ay2[2], cx2[2], cy2[2];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            ax1[i] = lerp_exact(bx[i], bx[i + 1], t0, s0);
            ay1[i] = lerp_exact(by[i], by[i + 1], t0, s0);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            ax2[i] = lerp_exact(ax1[i], ax1[i + 1], t0, s0);   // (t0, t0)
            ay2[i] = lerp_exact(ay1[i], ay1[i + 1], t0, s0);
            cx2[i] = lerp_exact(ax1[i], ax1[i + 1], t1, s1);   // (t0, t1)
            cy2[i] = lerp_exact(ay1[i], ay1[i + 1], t1, s1);
        }
        const double p1x = lerp_exact(ax2[0], ax2[1], t1, s1), p1y = lerp_exact(ay2[0], ay2[1], t1, s1);
        const double p2x = lerp_exact(cx2[0], cx2[1], t1, s1), p2y = lerp_exact(cy2[0], cy2[1], t1, s1);
        // end point b(t1, t1, t1)
        double ex1[3], ey1[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            ex1[i] = lerp_exact(bx[i], bx[i + 1], t1, s1);
            ey1[i] = lerp_exact(by[i], by[i + 1], t1, s1);
        }
        const double e20 = lerp_exact(ex1[0], ex1[1], t1, s1), e21 = lerp_exact(ex1[1], ex1[2], t1, s1);
        const double f20 = lerp_exact(ey1[0], ey1[1], t1, s1), f21 = lerp_exact(ey1[1], ey1[2], t1, s1);
        const double p3x = lerp_exact(e20, e21, t1, s1), p3y = lerp_exact(f20, f21, t1, s1);
        if (COUNT) ctr.v[GWN_C_PIECES]++;
        const double xmn = fmin(fmin(p0x, p1x), fmin(p2x, p3x)), xmx = fmax(fmax(p0x, p1x), fmax(p2x, p3x));
        const double ymn = fmin(fmin(p0y, p1y), fmin(p2y, p3y)), ymx = fmax(fmax(p0y, p1y), fmax(p2y, p3y));
        const bool out = xmn > 0.0 || xmx < 0.0 || ymn > 0.0 || ymx < 0.0;
        const bool on = fmax(fmax(-xmn, xmx), fmax(-ymn, ymx)) < on_tol;
        if (!out && !on && level < kMaxBisectLevel) {
            ++level;
            k <<= 1;
            continue;
        }
        if (out) {
            // outside: the chord angle is exact
            angle_add_chord(A, p0x * p3y - p0y * p3x, p0x * p3x + p0y * p3y);
        } else {
            // Terminal piece still holding q (within eps_on, or at the depth
            // limit): q is on the curve to tolerance, and the piece takes the
            // mean of its two one-sided limits, i.e. its chord angle with the
            // jump of +-pi removed when q lies between its end points.
            double a = chord_angle(p0x, p0y, p3x, p3y);
            if (fabs(a) > 0.5 * kPi) a -= copysign(kPi, a);
            A.extra += a;
        }
        if (COUNT) ctr.v[GWN_C_ANGLES]++;
        p0x = p3x;
        p0y = p3y;
        while (level > 0 && (k & 1)) { k >>= 1; --level; }
        if (level == 0) break;
        ++k;
    }
}

// Far-field contribution of an accepted 2D cluster, as an angle in radians.
// The order-p Taylor expansion of Eq. taylor about the centroid c equals
// -Im( sum_{k<=p} m_k u^{k+1} ) with u = 1/(q - c) and m_k = int (z - c)^k dz
// (complex form of the centred moments).  With the moments stored as
// m_k / r^(k+1) the series runs in v = r u, |v| < 1 / beta, whose powers
// stay in range at any model scale; each moment then enters as a
// multiplicand (two FMAs per order) instead of as the addend of a Horner
// step, which on gfx950 would cost two extra moves per moment.
template <typename T>
__device__ __forceinline__ T taylor2d(T dx, T dy, T d2, T r, const T *m, int order)
{
    const T s = r * fast_rcp(d2);   // d2 > beta^2 r^2 > 0 for an accepted cluster
    const T vr = dx * s, vi = -dy * s;
    T pr = vr, pi = vi;
    T a0 = m[0] * pi, a1 = m[1] * pr;   // two chains: Re(m) Im(v^j), Im(m) Re(v^j)
    for (int k = 1; k <= order; ++k) {
        const T nr = pr * vr - pi * vi;
        const T ni = pr * vi + pi * vr;
        pr = nr;
        pi = ni;
        a0 = fma(m[2 * k], pi, a0);
        a1 = fma(m[2 * k + 1], pr, a1);
    }
    return -(a0 + a1);   // -Im(sum m_k v^(k+1))
}

// Same term at a compile-time order: fully unrolled, so the cluster's
// moments are requested in one go instead of one load per step.  The FP32
// instance keeps Horner's rule in v (measured faster for 32-bit operands).
template <typename T, int ORDER>
__device__ __forceinline__ T taylor2d_fixed(T dx, T dy, T d2, T r, const T *__restrict__ m)
{
    const T s = r * fast_rcp(d2);
    const T vr = dx * s, vi = -dy * s;
    if constexpr (sizeof(T) == 4) {
        T tr = m[2 * ORDER], ti = m[2 * ORDER + 1];
#pragma unroll
        for (int k = ORDER - 1; k >= 0; --k) {
            const T nr = m[2 * k] + vr * tr - vi * ti;
            const T ni = m[2 * k + 1] + vr * ti + vi * tr;
            tr = nr;
            ti = ni;
        }
        return -(vr * ti + vi * tr);   // -Im(v t)
    }
    T pr = vr, pi = vi;
    T a0 = m[0] * pi, a1 = m[1] * pr;
#pragma unroll
    for (int k = 1; k <= ORDER; ++k) {
        const T nr = pr * vr - pi * vi;
        const T ni = pr * vi + pi * vr;
        pr = nr;
        pi = ni;
        a0 = fma(m[2 * k], pi, a0);
        a1 = fma(m[2 * k + 1], pr, a1);
    }
    return -(a0 + a1);
}

// Traversal with wave acceptance (FP64, or the FP32 pass of the mixed
// form): a cluster is far only when every lane of `mask` passes its test, so the wave accepts or descends as a
// whole and its lane mask never changes.  The depth-first walk then needs no
// stack: after a leaf or an accepted cluster it continues at the node's
// escape index (the first node after its subtree), after a rejected cluster
// at its left child (the next index).  Same nodes in the same order as the
// stack walk, so the same sums bit for bit.
template <bool F32, bool COUNT>
__device__ double traverse2d_wave(const DevModel &M, double qx, double qy, uint64_t mask, Ctr &ctr, bool &overflow)
{
    const Node2 *__restrict__ nodes = (const Node2 *)M.nodes;
    const Hot2 *__restrict__ hot = (const Hot2 *)M.hot;
    const Prim2 *__restrict__ prims = (const Prim2 *)M.prims;
    const bool me = (mask >> lane_id()) & 1;
    const float qxf = (float)qx, qyf = (float)qy;
    const double beta2 = M.beta2;
    const float beta2f = (float)M.beta2_mixed;
    const int order = M.order;
    const double eps_on = M.eps_on;
    const int n_nodes = M.n_nodes;
    double acc = 0.0;
    AngleAcc A;
    angle_init(A);
    int cur = 0;
    while (cur < n_nodes) {
        const Hot2 *hd = hot + cur;
        const int right = hd->right;
        const double bb[4] = {hd->a[0], hd->a[1], hd->a[2], hd->a[3]};
        const float ff[4] = {hd->f[0], hd->f[1], hd->f[2], hd->f[3]};
        if (right < 0) {
            if (me) leaf2d<COUNT>(hd, bb, ff, prims, qx, qy, qxf, qyf, eps_on, A, ctr, overflow);
            cur = cur + 1;
            continue;
        }
        if (COUNT && me) ctr.v[GWN_C_NODES]++;
        if (F32) {
            const float dx = qxf - ff[0], dy = qyf - ff[1];
            const float d2 = dx * dx + dy * dy;
            if (__ballot(me && d2 > beta2f * ff[2]) == mask) {
                if (me) {
                    acc += order >= kMaxOrder2D - 1
                               ? (double)taylor2d_fixed<float, kMaxOrder2D - 1>(dx, dy, d2, ff[3], nodes[cur].fm)
                           : order >= kMixedOrder2D
                               ? (double)taylor2d_fixed<float, kMixedOrder2D>(dx, dy, d2, ff[3], nodes[cur].fm)
                               : (double)taylor2d<float>(dx, dy, d2, ff[3], nodes[cur].fm, order);
                    if (COUNT) ctr.v[GWN_C_FAR]++;
                }
                cur = uniform_i(hd->escape);
            } else {
                cur = cur + 1;
            }
            continue;
        }
        const double dx = qx - bb[0], dy = qy - bb[1];
        const double d2 = dx * dx + dy * dy;
        if (__ballot(me && d2 > beta2 * bb[2]) == mask) {
            if (me) {
                acc += order == kMaxOrder2D ? taylor2d_fixed<double, kMaxOrder2D>(dx, dy, d2, bb[3], nodes[cur].m)
                       : order == kMixedOrder2D + 1
                           ? taylor2d_fixed<double, kMixedOrder2D + 1>(dx, dy, d2, bb[3], nodes[cur].m)
                           : taylor2d<double>(dx, dy, d2, bb[3], nodes[cur].m, order);
                if (COUNT) ctr.v[GWN_C_FAR]++;
            }
            cur = uniform_i(hd->escape);
        } else {
            cur = cur + 1;
        }
    }
    return (angle_total(A) + acc) * (1.0 / (2.0 * kPi));
}

// Traversal of one wave over a 2D model.  `mask`: lanes taking part (wave
// uniform).  F32: far-field tests and Taylor terms in FP32 (mixed form).
template <bool F32, bool COUNT>
__device__ double traverse2d(const DevModel &M, double qx, double qy, uint64_t mask, StackLDS &S, int w,
                             Ctr &ctr, bool &overflow)
{
    if (M.wave_accept) return traverse2d_wave<F32, COUNT>(M, qx, qy, mask, ctr, overflow);
    const Node2 *__restrict__ nodes = (const Node2 *)M.nodes;
    const Hot2 *__restrict__ hot = (const Hot2 *)M.hot;
    const Prim2 *__restrict__ prims = (const Prim2 *)M.prims;
    const int lane = lane_id();
    const bool me = (mask >> lane) & 1;
    const float qxf = (float)qx, qyf = (float)qy;
    const double beta2 = F32 ? M.beta2_mixed : M.beta2;
    const float beta2f = (float)M.beta2_mixed;
    // read once: inside the loop each use would be a scalar load and a wait
    // per node (the loop's LDS stores keep the compiler from hoisting them)
    const int order = M.order;
    const bool wave_accept = M.wave_accept != 0;
    const double eps_on = M.eps_on;
    double acc = 0.0;      // far-field terms, in radians
    AngleAcc A;            // direct (chord) angles
    angle_init(A);
    int cur = 0;
    uint64_t curmask = mask;
    int sp = 0;
    if (M.n_nodes == 0) return 0.0;
    while (true) {
        const Hot2 *hd = hot + cur;
        const int right = hd->right;
        // the record's fields are used on both paths below, so they are
        // requested together with `right`
        const double bb[4] = {hd->a[0], hd->a[1], hd->a[2], hd->a[3]};
        const float ff[4] = {hd->f[0], hd->f[1], hd->f[2], hd->f[3]};
        const bool active = (curmask >> lane) & 1;
        if (right < 0) {
            if (active) leaf2d<COUNT>(hd, bb, ff, prims, qx, qy, qxf, qyf, eps_on, A, ctr, overflow);
        } else {
            bool far = false;
            if (active) {
                if (COUNT) ctr.v[GWN_C_NODES]++;
                if (F32) {
                    const float dx = qxf - ff[0], dy = qyf - ff[1];
                    const float d2 = dx * dx + dy * dy;
                    far = d2 > beta2f * ff[2];
                    if (far)
                        acc += order >= kMaxOrder2D - 1
                                   ? (double)taylor2d_fixed<float, kMaxOrder2D - 1>(dx, dy, d2, ff[3], nodes[cur].fm)
                               : order >= kMixedOrder2D
                                   ? (double)taylor2d_fixed<float, kMixedOrder2D>(dx, dy, d2, ff[3], nodes[cur].fm)
                                   : (double)taylor2d<float>(dx, dy, d2, ff[3], nodes[cur].fm, order);
                } else {
                    const double dx = qx - bb[0], dy = qy - bb[1];
                    const double d2 = dx * dx + dy * dy;
                    far = d2 > beta2 * bb[2];
                    // wave acceptance: far only when every active lane is
                    if (wave_accept && __ballot(far) != curmask) far = false;
                    if (far)
                        acc += order == kMaxOrder2D
                                   ? taylor2d_fixed<double, kMaxOrder2D>(dx, dy, d2, bb[3], nodes[cur].m)
                               : order == kMixedOrder2D + 1
                                   ? taylor2d_fixed<double, kMixedOrder2D + 1>(dx, dy, d2, bb[3], nodes[cur].m)
                                   : taylor2d<double>(dx, dy, d2, bb[3], nodes[cur].m, order);
                }
                if (COUNT && far) ctr.v[GWN_C_FAR]++;
            }
            const uint64_t farmask = __ballot(active && far);
            const uint64_t nearmask = curmask & ~farmask;
            if (nearmask) {
                S.node[w][sp] = right;
                S.mask[w][sp] = nearmask;
                ++sp;
                cur = cur + 1;
                curmask = nearmask;
                continue;
            }
        }
        if (sp == 0) break;
        --sp;
        cur = uniform_i(S.node[w][sp]);
        curmask = uniform_u64(S.mask[w][sp]);
    }
    (void)me;
    return (angle_total(A) + acc) * (1.0 / (2.0 * kPi));
}

// Query body (2D): one wave per 64 consecutive sorted queries of one
// segment.  Mixed-precision segments run the FP32 far-field pass and then
// re-evaluate in FP64 the lanes with |w - 0.5| < band.
template <bool COUNT, bool MIXED>
__device__ __forceinline__ void query2d_body(const LaunchTable &T, const double *__restrict__ pts,
                                             const int32_t *__restrict__ perm, double *__restrict__ out_w,
                                             uint8_t *__restrict__ out_in, long long *counters, StackLDS &S)
{
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    // runs of 4 blocks per XCD for the FP64 kernel, 16 for the mixed one
    // (each measured fastest for its kernel)
    const int wave = xcd_block<(MIXED ? 16 : 4)>() * kWavesPerBlock + w;
    if (wave >= T.n_waves) return;
    int s = 0;
    {
        int lo = 0, hi = T.n_seg - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (T.woff[mid] <= wave) lo = mid; else hi = mid - 1;
        }
        s = uniform_i(lo);
    }
    const DevModel &M = T.models[T.seg_model[s]];
    const int64_t pos = T.qoff[s] + (int64_t)(wave - T.woff[s]) * T.qpw + lane;
    const bool valid = lane < T.qpw && pos < T.qoff[s + 1];
    const int row = valid ? perm[pos] : 0;
    const double qx = valid ? pts[2 * (int64_t)row] : 0.0;
    const double qy = valid ? pts[2 * (int64_t)row + 1] : 0.0;
    const uint64_t mask = __ballot(valid);
    Ctr ctr;
#pragma unroll
    for (int k = 0; k < GWN_NCOUNTERS; ++k) ctr.v[k] = 0;
    bool overflow = false;
    double wq;
    const bool mixed = MIXED && M.precision == GWN_MIXED;
    if (mixed) {
        // FP32 far-field pass, then the FP64 form for the lanes of this wave
        // whose value lies within the band around 0.5 (Morton neighbours, so
        // the FP64 traversal of the subset stays coherent).
        wq = traverse2d<true, COUNT>(M, qx, qy, mask, S, w, ctr, overflow);
        const bool need = valid && fabs(wq - 0.5) < M.band;
        const uint64_t rmask = __ballot(need);
        if (rmask) {
            const double r = traverse2d<false, COUNT>(M, qx, qy, rmask, S, w, ctr, overflow);
            if (need) wq = r;
            if (COUNT && need) ctr.v[GWN_C_RECLASS]++;
        }
    } else {
        wq = traverse2d<false, COUNT>(M, qx, qy, mask, S, w, ctr, overflow);
    }
    if (valid) {
        if (overflow) {
            wq = NAN;
            atomicAdd((unsigned int *)M.flag, 1u);
            if (COUNT) ctr.v[GWN_C_OVERFLOW]++;
        }
        if (out_w) out_w[row] = wq;
        if (out_in) out_in[row] = wq >= 0.5 ? 1 : 0;
    }
    flush_counters<COUNT>(ctr, counters);
}

// Launches without mixed segments use k_query2d: without the FP32 pass the
// kernel fits 93 VGPRs with no spill (five waves per SIMD); capped at 72
// VGPRs (seven waves) it spills 84 bytes per lane, around the leaf
// bisection (entered by a small share of leaf visits), and hides more of
// the dependent node loads: 5 % faster on the 1024^2
// drawing than at five waves and 3 % faster than at six.
// k_query2d_mixed carries both passes; capped at six waves per SIMD (80
// VGPRs, 72 bytes of spill) it runs 3 % faster than at five or seven and
// 7 % faster than at the 104 VGPRs (four waves) it takes uncapped.
template <bool COUNT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7))) void k_query2d(
    LaunchTable T, const double *__restrict__ pts, const int32_t *__restrict__ perm, double *__restrict__ out_w,
    uint8_t *__restrict__ out_in, long long *counters)
{
    __shared__ StackLDS S;
    query2d_body<COUNT, false>(T, pts, perm, out_w, out_in, counters, S);
}

template <bool COUNT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_query2d_mixed(LaunchTable T, const double *__restrict__ pts,
                                                          const int32_t *__restrict__ perm,
                                                          double *__restrict__ out_w, uint8_t *__restrict__ out_in,
                                                          long long *counters)
{
    __shared__ StackLDS S;
    query2d_body<COUNT, true>(T, pts, perm, out_w, out_in, counters, S);
}

// 3D kernels live in query3d.hip; near_buf holds near.total bytes
gwn_status launch_query3d(const LaunchTable &T, const double *pts, const int32_t *perm, double *out_w,
                          uint8_t *out_in, long long *counters, char *near_buf, const NearBytes &near,
                          hipStream_t stream, std::string &err);

// ---------------------------------------------------------------------------
// host launcher
// ---------------------------------------------------------------------------
static std::mutex g_prof_mu;
static bool g_prof_on = false;
struct ProfEvents {
    int kernel;
    hipEvent_t a, b;
};
static std::vector<ProfEvents> g_prof_events;
static double g_prof_ms[kProfKernels];
static int64_t g_prof_n[kProfKernels];

void prof_begin(hipStream_t s, hipEvent_t &a)
{
    a = nullptr;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    if (hipEventCreate(&a) != hipSuccess) { a = nullptr; return; }
    (void)hipEventRecord(a, s);
}

void prof_end(hipStream_t s, hipEvent_t a, int kernel)
{
    if (!a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_events.push_back({kernel, a, b});
}

gwn_status profile_control(int enable, double *total_ms, int64_t *launches)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double ms = 0.0;
    int64_t cnt = 0;
    for (int k = 0; k < kProfKernels; ++k) {
        g_prof_ms[k] = 0.0;
        g_prof_n[k] = 0;
    }
    for (auto &ev : g_prof_events) {
        float t = 0.f;
        if (hipEventSynchronize(ev.b) == hipSuccess && hipEventElapsedTime(&t, ev.a, ev.b) == hipSuccess) {
            ms += t;
            ++cnt;
            g_prof_ms[ev.kernel] += t;
            g_prof_n[ev.kernel] += 1;
        }
        (void)hipEventDestroy(ev.a);
        (void)hipEventDestroy(ev.b);
    }
    g_prof_events.clear();
    g_prof_on = enable != 0;
    if (total_ms) *total_ms = ms;
    if (launches) *launches = cnt;
    return GWN_OK;
}

gwn_status profile_kernel(int kernel, double *ms, int64_t *launches)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (kernel < 0 || kernel >= kProfKernels) return GWN_EINVAL;
    if (ms) *ms = g_prof_ms[kernel];
    if (launches) *launches = g_prof_n[kernel];
    return GWN_OK;
}
static gwn_status hip_err(hipError_t e, const char *what, std::string &err)
{
    err = std::string(what) + ": " + hipGetErrorString(e);
    return GWN_EHIP;
}

// Queries per wave of a launch of n queries: a launch of fewer than 2^18
// queries spreads them over up to 4096 waves (at least 8 queries each):
// scattered queries share few nodes, so a wave's cost grows with its number
// of queries, and more waves keep more of the 1024 SIMDs busy.  With
// per-query far tests a query's value does not depend on its wave mates, so
// results are the same at any spread; with wave acceptance they are the
// same for the same call.
static int32_t queries_per_wave(int64_t n)
{
    int32_t qpw = 64;
    while (qpw > 8 && (int64_t)(qpw / 2) * 4096 >= n) qpw /= 2;
    return qpw;
}

// Scratch of one launch chunk, in one buffer with 256-byte aligned parts:
// sort keys and row indices (double-buffered), the radix sort's temporary
// storage and, in 3D, the near-field pass's per-slot records.  Nothing in it
// needs to start at zero: every record is written before it is read.  The
// sort orders the queries for coherent waves (with per-query far tests no
// value depends on the order; with wave acceptance the order decides which
// queries decide together), so it takes the top Morton bits down to 2^8
// cells per axis (2D bits 32-47, 3D bits 24-47: a cell holds a few of a
// full grid's queries), or the top 18 bits for a launch under 2^16 queries,
// and the segment bits 48-53 only when the launch has more than one
// segment: two (2D) or three (3D) 8-bit radix passes for one segment
// instead of seven.
struct ScratchPlan {
    size_t keys = 0, vals = 0, temp = 0, temp_bytes = 0;
    NearBytes near;
    size_t total = 0;
    int sort_lo = 0;
};

static size_t al256(size_t x) { return (x + 255) / 256 * 256; }

static hipError_t plan_scratch(int dim, int64_t n, int64_t slots, hipStream_t stream, ScratchPlan &P)
{
    P.sort_lo = n < (1 << 16) ? 30 : dim == 2 ? 32 : 24;
    P.temp_bytes = radix_temp_bytes(n);
    (void)stream;
    P.keys = al256(sizeof(uint64_t) * n);
    P.vals = al256(sizeof(int32_t) * n);
    P.temp = al256(P.temp_bytes);
    P.near = dim == 3 ? near_scratch_bytes(slots) : NearBytes{};
    P.total = 2 * P.keys + 2 * P.vals + P.temp + P.near.total;
    return hipSuccess;
}

static gwn_status launch_chunk(const std::vector<Segment> &segs, size_t s0, size_t s1, int dim,
                               const double *points, double *out_gwn, uint8_t *out_inside, int64_t *counters,
                               hipStream_t stream, const ExtScratch &ext, std::string &err)
{
    LaunchTable T;
    std::memset(&T, 0, sizeof T);
    std::vector<const Model *> models;
    T.n_seg = (int32_t)(s1 - s0);
    const int64_t row0 = segs[s0].q_begin;
    int64_t n_all = 0;
    for (size_t k = s0; k < s1; ++k) n_all += segs[k].q_end - segs[k].q_begin;
    const int32_t qpw = queries_per_wave(n_all);
    T.qpw = qpw;
    int64_t q = 0;
    int32_t wv = 0;
    for (size_t k = s0; k < s1; ++k) {
        const Model *m = segs[k].model;
        int mi = -1;
        for (size_t j = 0; j < models.size(); ++j)
            if (models[j] == m) mi = (int)j;
        if (mi < 0) {
            mi = (int)models.size();
            models.push_back(m);
            T.models[mi] = m->dev;
        }
        const int j = (int)(k - s0);
        T.seg_model[j] = mi;
        T.qoff[j] = q;
        T.woff[j] = wv;
        const int64_t cnt = segs[k].q_end - segs[k].q_begin;
        q += cnt;
        wv += (int32_t)((cnt + qpw - 1) / qpw);
    }
    T.qoff[T.n_seg] = q;
    T.woff[T.n_seg] = wv;
    T.n_waves = wv;
    const int64_t n = q;
    if (n == 0) return GWN_OK;
    const double *pts = points + row0 * dim;
    double *ow = out_gwn ? out_gwn + row0 : nullptr;
    uint8_t *oi = out_inside ? out_inside + row0 : nullptr;

    ScratchPlan P;
    hipError_t e = plan_scratch(dim, n, (int64_t)T.n_waves * T.qpw, stream, P);
    if (e != hipSuccess) return hip_err(e, "radix sort sizing", err);
    char *buf = nullptr;
    if (ext.ptr) {
        if (P.total > ext.bytes) {
            err = "launch needs " + std::to_string(P.total) + " bytes of scratch, above the fixed " +
                  std::to_string(ext.bytes);
            return GWN_EINVAL;
        }
        buf = (char *)ext.ptr;
    } else {
        e = hipMallocAsync((void **)&buf, P.total, stream);
        if (e != hipSuccess) return hip_err(e, "hipMallocAsync scratch", err);
    }
    uint64_t *k_in = (uint64_t *)buf, *k_out = (uint64_t *)(buf + P.keys);
    int32_t *v_in = (int32_t *)(buf + 2 * P.keys), *v_out = (int32_t *)(buf + 2 * P.keys + P.vals);
    void *temp = buf + 2 * P.keys + 2 * P.vals;
    char *near_buf = buf + 2 * P.keys + 2 * P.vals + P.temp;

    const int grid_q = (int)((n + kBlock - 1) / kBlock);
    gwn_status st = GWN_OK;
    hipLaunchKernelGGL(k_keys, dim3(grid_q), dim3(kBlock), 0, stream, T, dim, pts, k_in, v_in, n);
    e = hipGetLastError();
    // the sorted permutation ends up in one of the two value buffers
    const int32_t *perm = v_out;
    if (e == hipSuccess) {
        uint64_t *kb[2] = {k_in, k_out};
        int32_t *vb[2] = {v_in, v_out};
        int sel = 0;
        e = radix_sort_pairs(kb, vb, n, P.sort_lo, T.n_seg > 1 ? 54 : 48, temp, stream, sel);
        perm = vb[sel];
    }
    if (e != hipSuccess) st = hip_err(e, "key/sort launch", err);
    if (!st) {
        if (dim == 2) {
            hipEvent_t ev0;
            prof_begin(stream, ev0);
            const int grid_w = (T.n_waves + kWavesPerBlock - 1) / kWavesPerBlock;
            bool any_mixed = false;
            for (int j = 0; j < T.n_seg; ++j) any_mixed |= T.models[T.seg_model[j]].precision == GWN_MIXED;
            long long *ctrs = (long long *)counters;
            if (any_mixed) {
                if (ctrs)
                    hipLaunchKernelGGL(k_query2d_mixed<true>, dim3(grid_w), dim3(kBlock), 0, stream, T, pts, perm,
                                       ow, oi, ctrs);
                else
                    hipLaunchKernelGGL(k_query2d_mixed<false>, dim3(grid_w), dim3(kBlock), 0, stream, T, pts, perm,
                                       ow, oi, ctrs);
            } else {
                if (ctrs)
                    hipLaunchKernelGGL(k_query2d<true>, dim3(grid_w), dim3(kBlock), 0, stream, T, pts, perm, ow, oi,
                                       ctrs);
                else
                    hipLaunchKernelGGL(k_query2d<false>, dim3(grid_w), dim3(kBlock), 0, stream, T, pts, perm, ow,
                                       oi, ctrs);
            }
            e = hipGetLastError();
            if (e != hipSuccess) st = hip_err(e, "query launch", err);
            prof_end(stream, ev0, GWN_K_QUERY2D);
        } else {
            st = launch_query3d(T, pts, perm, ow, oi, (long long *)counters, near_buf, P.near, stream, err);
        }
    }
    if (!ext.ptr) {
        hipError_t e2 = hipFreeAsync(buf, stream);
        if (!st && e2 != hipSuccess) st = hip_err(e2, "hipFreeAsync scratch", err);
    }
    return st;
}

gwn_status launch_queries(const std::vector<Segment> &segs, int dim, const double *points, double *out_gwn,
                          uint8_t *out_inside, int64_t *counters, void *stream, std::string &err,
                          const ExtScratch &ext)
{
    hipStream_t s = (hipStream_t)stream;
    size_t a = 0;
    while (a < segs.size()) {
        // chunk: <= kMaxSeg segments, <= kMaxModels distinct models, contiguous rows
        std::vector<const Model *> seen;
        size_t b = a;
        while (b < segs.size() && b - a < (size_t)kMaxSeg) {
            const Model *m = segs[b].model;
            bool known = std::find(seen.begin(), seen.end(), m) != seen.end();
            if (!known && seen.size() == (size_t)kMaxModels) break;
            if (!known) seen.push_back(m);
            if (b > a && segs[b].q_begin != segs[b - 1].q_end) break;
            ++b;
        }
        gwn_status st = launch_chunk(segs, a, b, dim, points, out_gwn, out_inside, counters, s, ext, err);
        if (st) return st;
        a = b;
    }
    return GWN_OK;
}

gwn_status query_scratch_bytes(int dim, int64_t n, int32_t n_seg, int64_t &bytes, std::string &err)
{
    bytes = 0;
    if (n <= 0) return GWN_OK;
    // the launch is cut into chunks of at most kMaxSeg segments, one after
    // another on the stream: the largest chunk's scratch bounds the call's.
    // Each segment after the first adds at most one partly filled wave.
    const int32_t segs_per_chunk = std::min<int32_t>(std::max<int32_t>(n_seg, 1), kMaxSeg);
    const int32_t qpw = queries_per_wave(n);
    const int64_t waves = (n + qpw - 1) / qpw + (segs_per_chunk - 1);
    ScratchPlan P;
    hipError_t e = plan_scratch(dim, n, waves * qpw, nullptr, P);
    if (e != hipSuccess) return hip_err(e, "radix sort sizing", err);
    bytes = (int64_t)P.total;
    return GWN_OK;
}

// Fixed scratch of the entry point that allocates nothing: one array per
// GPU, held from the library's first such call on that GPU to the end of the
// process.  Host code never uses the array's name as an address (on the host
// it only names the symbol): the device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

gwn_status noalloc_scratch(ExtScratch &out, std::string &err)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_err(e, "hipGetDevice", err);
    if (dev < 0 || dev >= kMaxDevices) {
        err = "device ordinal " + std::to_string(dev) + " beyond the fixed-scratch table";
        return GWN_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_err(e, "hipGetSymbolAddress(scratch)", err);
        if (!p) {
            err = "hipGetSymbolAddress(scratch) returned NULL";
            return GWN_EHIP;
        }
        addr[dev] = p;
    }
    out.ptr = addr[dev];
    out.bytes = kNoAllocScratchBytes;
    return GWN_OK;
}

}  // namespace gwn
