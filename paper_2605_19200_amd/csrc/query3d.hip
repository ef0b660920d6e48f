// 3D query phase of Alg. 1 on gfx950 (trimmed rational bicubic patches).
//
// Traversal: the same wavefront-coherent scheme as 2D (one LDS stack of
// (node, lane mask) per wave, per-lane far tests, left-first order per lane).
//
// Far clusters: order 0..2 expansion of Eq. taylor with the derivative
// tensors of G3 = -1 / (4 pi |x - q|) written out (s = c - q, rho = |s|):
//   T0 = s.M0 / rho^3
//   T1 = tr M1 / rho^3 - 3 s^T M1 s / rho^5
//   T2 = ( -3 (2 a + b).s / rho^5 + 15 M2:sss / rho^7 ) / 2
// with a_i = sum_j M2_ijj, b_k = sum_i M2_iik; w += (T0 + T1 + T2) / 4 pi.
//
// Leaves (Sec. 3.3, always evaluated directly):
//  * q farther than near_ratio x diagonal from the leaf's AABB: the leaf's
//    precomputed Green-scattered Gauss-Legendre nodes (x_k, N_k):
//    Omega = sum N_k . (x_k - q) / |x_k - q|^3.
//  * otherwise the near-field rule: the solid angle density in parameter
//    space g(u, v) = det[A, A_u, A_v] / |A|^3 (A = H - q W, weights cancel)
//    is integrated over the visible region D with Green's theorem in polar
//    form about the foot point c of q on the patch:
//      integral_D g = sum over boundary curves gamma of
//        integral cross(gamma - c, gamma') H(gamma) dt,
//      H(p) = integral_0^1 g(c + tau (p - c)) tau dtau,
//    valid for any c in the unit square (the rays stay in the square).  The
//    near-singular behaviour of g at c (width ~ dist(q, S)) sits at tau = 0
//    and is removed by the substitution tau = eps sinh(mu sigma),
//    eps = d / L, mu = asinh(1 / eps); the outer integral is split into
//    panels graded geometrically from the point of gamma nearest c.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "near3d.h"
#include "query_common.h"

namespace gwn {

void gauss_kronrod01(int n, double *xk, double *wk, double *wg);   // build3d.cpp

__constant__ QuadTables c_quad;

__device__ __forceinline__ void ctr_add(Ctr &c, int k, long long v) { c.v[k] += v; }

// Runs of 16 blocks per XCD (see xcd_block); both 3D passes must map
// blocks to waves the same way, since the near-field pass reads the
// traversal's per-slot scratch.
constexpr int kXcdRun3 = 16;

struct NearScratch {
    double *part;      // [n_waves * qpw] solid angle of the far field and node-set leaves
    int32_t *cnt;      // [n_waves * qpw] near leaves met by the traversal
    int32_t *list;     // [n_waves * qpw * kNearSlots] their node indices
    uint8_t *need;     // [n_waves * qpw] mixed form: query re-evaluated in FP64
};

// Direct solid angle of one leaf at q by its precomputed node set, chosen by
// distance / half-diagonal ratio (finest near, coarsest far).  A leaf within
// near_ratio of its diagonal is recorded for the near-field pass instead.
// The model fields the traversal reads at every node, copied to registers
// once: read through the model inside the loop, each would be a scalar load
// and a wait per node (the loop's LDS stores keep the compiler from hoisting
// them).
struct TravParams {
    const void *mpole, *fmpole, *qnodes;
    double beta2, near_ratio2;
    float beta2_mixed;
    int order, wave_accept, leaf_far;
};

__device__ __forceinline__ TravParams trav_params(const DevModel &M)
{
    return TravParams{M.mpole, M.fmpole, M.qnodes, M.beta2, M.near_ratio2, (float)M.beta2_mixed,
                      M.order, M.wave_accept, M.leaf_far};
}

template <bool COUNT>
__device__ double leaf3d(const TravParams &M, const Node3 *__restrict__ nd, int cur, double qx, double qy, double qz,
                         bool active, int &ncnt, int32_t *__restrict__ mylist, Ctr &ctr)
{
    const double dx = fmax(fmax(nd->t[0] - qx, qx - nd->t[3]), 0.0);
    const double dy = fmax(fmax(nd->t[1] - qy, qy - nd->t[4]), 0.0);
    const double dz = fmax(fmax(nd->t[2] - qz, qz - nd->t[5]), 0.0);
    const double ex = nd->t[3] - nd->t[0], ey = nd->t[4] - nd->t[1], ez = nd->t[5] - nd->t[2];
    const double d2 = dx * dx + dy * dy + dz * dz, diag2 = ex * ex + ey * ey + ez * ez;
    const bool near = d2 < M.near_ratio2 * diag2;
    double om = 0.0;
    if (COUNT && active) ctr.v[GWN_C_LEAVES]++;
    if (active && near) {
        if (ncnt < kNearSlots) mylist[ncnt] = cur;
        ++ncnt;
    }
    if (active && !near) {
        const double r2 = 4.0 * d2 / diag2;
        const int c0 = (int)nd->t[6], c1 = (int)nd->t[7], c2 = (int)nd->t[8];
        int off = 0, cnt = c0;
        if (r2 >= kLeafRuleRatio[2] * kLeafRuleRatio[2]) { off = c0 + c1; cnt = c2; }
        else if (r2 >= kLeafRuleRatio[1] * kLeafRuleRatio[1]) { off = c0; cnt = c1; }
        const QNode3 *__restrict__ qn = (const QNode3 *)M.qnodes + nd->aux + off;
        // four nodes' scalar loads in flight before the first is used (the
        // sum keeps its order): traversal 149 -> 113 ms on the CAD
        // assembly, 36.0 -> 34.5 ms on the bodies grid (eight: no better)
#pragma unroll 4
        for (int k = 0; k < cnt; ++k) {
            const double rx = qn[k].x[0] - qx, ry = qn[k].x[1] - qy, rz = qn[k].x[2] - qz;
            const double rr = rx * rx + ry * ry + rz * rz;
            const double inv = inv_sqrt(rr);
            om += (qn[k].n[0] * rx + qn[k].n[1] * ry + qn[k].n[2] * rz) * (inv * inv * inv);
        }
        if (COUNT) { ctr.v[GWN_C_LEAF_FAST]++; ctr.v[GWN_C_ANGLES] += cnt; }
    }
    return om;
}

// Far field of an accepted cluster (Eq. taylor to order p = L - 1), as a
// solid angle: sum over 1 <= l <= L of I_l^0 N_l^0 + 2 sum_{m>0} Re(I_l^m
// N_l^m), with the irregular solid harmonics I_l^m(q - c) generated per m by
//   I_m^m = I_{m-1}^{m-1} (2m - 1)(x + i y) / rho^2,  I_0^0 = 1 / rho,
//   I_l^m = ((2l - 1) z I_{l-1}^m - (l + m - 1)(l - m - 1) I_{l-2}^m) / rho^2
// and contracted on the fly (a handful of registers at any order).  The
// moments are stored scaled by r^-(l+1), so the harmonics are taken at
// (q - c) / r.  mp[0] = 1 / r, mp[2 + 2k], mp[3 + 2k] = (re, im) of moment
// k = l (l + 1) / 2 - 1 + m.
template <typename T>
__device__ __forceinline__ T multipole3d(T sx, T sy, T sz, const T *__restrict__ mp, int L)
{
    const T ir = mp[0];
    const T x = sx * ir, y = sy * ir, z = sz * ir;
    T inv2, mmr;
    if constexpr (sizeof(T) == 8) {
        mmr = inv_sqrt(x * x + y * y + z * z);   // 1 / rho
        inv2 = mmr * mmr;
    } else {
        inv2 = T(1) / (x * x + y * y + z * z);
        mmr = sqrt(inv2);
    }
    T mmi = T(0);
    T omega = T(0);
    for (int m = 0; m <= L; ++m) {
        if (m > 0) {
            const T f = T(2 * m - 1) * inv2;
            const T nr = (mmr * x - mmi * y) * f;
            const T ni = (mmr * y + mmi * x) * f;
            mmr = nr;
            mmi = ni;
        }
        const T wgt = m == 0 ? T(1) : T(2);
        T pr = T(0), pi = T(0), cr = mmr, ci = mmi;
        for (int l = m; l <= L; ++l) {
            if (l > m) {
                const T a = T(2 * l - 1) * z * inv2;
                const T b = T((l + m - 1) * (l - m - 1)) * inv2;
                const T nr = a * cr - b * pr;
                const T ni = a * ci - b * pi;
                pr = cr;
                pi = ci;
                cr = nr;
                ci = ni;
            }
            if (l >= 1) {
                const int k = l * (l + 1) / 2 - 1 + m;
                omega += wgt * (cr * mp[2 + 2 * k] - ci * mp[3 + 2 * k]);
            }
        }
    }
    return omega;
}

// Traversal of one wave over a 3D model; returns the lane's solid angle of
// the far field and the node-set leaves, and records its near leaves.
// Same sum at a compile-time degree: fully unrolled, so the cluster's moments
// are requested in a few wide loads instead of one load per term.
template <typename T, int L>
__device__ __forceinline__ T multipole3d_fixed(T sx, T sy, T sz, const T *__restrict__ mp)
{
    const T ir = mp[0];
    const T x = sx * ir, y = sy * ir, z = sz * ir;
    T inv2, mmr;
    if constexpr (sizeof(T) == 8) {
        mmr = inv_sqrt(x * x + y * y + z * z);   // 1 / rho
        inv2 = mmr * mmr;
    } else {
        inv2 = T(1) / (x * x + y * y + z * z);
        mmr = sqrt(inv2);
    }
    T mmi = T(0);
    T omega = T(0);
#pragma unroll
    for (int m = 0; m <= L; ++m) {
        if (m > 0) {
            const T f = T(2 * m - 1) * inv2;
            const T nr = (mmr * x - mmi * y) * f;
            const T ni = (mmr * y + mmi * x) * f;
            mmr = nr;
            mmi = ni;
        }
        const T wgt = m == 0 ? T(1) : T(2);
        T pr = T(0), pi = T(0), cr = mmr, ci = mmi;
#pragma unroll
        for (int l = m; l <= L; ++l) {
            if (l > m) {
                const T a = T(2 * l - 1) * z * inv2;
                const T b = T((l + m - 1) * (l - m - 1)) * inv2;
                const T nr = a * cr - b * pr;
                const T ni = a * ci - b * pi;
                pr = cr;
                pi = ci;
                cr = nr;
                ci = ni;
            }
            if (l >= 1) {
                const int k = l * (l + 1) / 2 - 1 + m;
                omega += wgt * (cr * mp[2 + 2 * k] - ci * mp[3 + 2 * k]);
            }
        }
    }
    return omega;
}

// Far test of node `cur` for one lane, adding its far-field term when the
// test passes; true when it does.  With wave acceptance the test passes only
// when it passes for every lane of `curmask` (the lanes at this node).
template <bool F32>
__device__ __forceinline__ bool far_term3d(const TravParams &M, const Node3 *__restrict__ nd, int cur, double qx,
                                           double qy, double qz, double &acc_far, uint64_t curmask)
{
    if (F32) {
        const float sx = nd->fc[0] - (float)qx, sy = nd->fc[1] - (float)qy, sz = nd->fc[2] - (float)qz;
        const float r2 = sx * sx + sy * sy + sz * sz;
        bool far = r2 > M.beta2_mixed * nd->fr2;
        if (M.wave_accept && __ballot(far) != curmask) far = false;
        if (far) {
            const float *mp = (const float *)M.fmpole + (size_t)cur * kMpoleStride;
            acc_far += M.order + 1 == kMaxL3 ? (double)multipole3d_fixed<float, kMaxL3>(-sx, -sy, -sz, mp)
                                             : (double)multipole3d<float>(-sx, -sy, -sz, mp, M.order + 1);
        }
        return far;
    }
    const double sx = nd->c[0] - qx, sy = nd->c[1] - qy, sz = nd->c[2] - qz;
    const double r2 = sx * sx + sy * sy + sz * sz;
    bool far = r2 > M.beta2 * nd->r2;
    // wave acceptance: far only when every active lane is
    if (M.wave_accept && __ballot(far) != curmask) far = false;
    if (far) {
        const double *mp = (const double *)M.mpole + (size_t)cur * kMpoleStride;
        acc_far += M.order + 1 == kMaxL3 ? multipole3d_fixed<double, kMaxL3>(-sx, -sy, -sz, mp)
                                         : multipole3d<double>(-sx, -sy, -sz, mp, M.order + 1);
    }
    return far;
}

// Traversal with wave acceptance (FP64, or the FP32 pass of the mixed
// form): every test is decided for the whole wave, so its lane mask never
// changes and the depth-first walk needs no stack (after a leaf or an
// accepted cluster: the node's escape index; after a rejected cluster: the
// next index).  The same nodes in the same order as
// the stack walk, the same sums bit for bit.
template <bool F32, bool COUNT>
__device__ double traverse3d_wave(const DevModel &Mdl, double qx, double qy, double qz, uint64_t mask, int &ncnt,
                                  int32_t *__restrict__ mylist, Ctr &ctr)
{
    const Node3 *__restrict__ nodes = (const Node3 *)Mdl.nodes;
    const TravParams M = trav_params(Mdl);
    const bool me = (mask >> lane_id()) & 1;
    const int n_nodes = Mdl.n_nodes;
    double acc_far = 0.0, acc_leaf = 0.0;
    int cur = 0;
    while (cur < n_nodes) {
        const Node3 *nd = nodes + cur;
        const int right = nd->right;
        bool far = false;
        if (right < 0) {
            if (me && M.leaf_far) {
                far = far_term3d<F32>(M, nd, cur, qx, qy, qz, acc_far, mask);
                if (COUNT && far) { ctr.v[GWN_C_FAR]++; ctr.v[GWN_C_LEAVES]++; }
            }
            acc_leaf += leaf3d<COUNT>(M, nd, cur, qx, qy, qz, me && !far, ncnt, mylist, ctr);
            cur = cur + 1;
            continue;
        }
        if (me) {
            if (COUNT) ctr.v[GWN_C_NODES]++;
            far = far_term3d<F32>(M, nd, cur, qx, qy, qz, acc_far, mask);
            if (COUNT && far) ctr.v[GWN_C_FAR]++;
        }
        cur = __ballot(me && far) ? uniform_i(nd->escape) : cur + 1;
    }
    return acc_far + acc_leaf;
}

// Traversal of one wave (Alg. 1 query loop) over a 3D model.  With
// leaf_far, a reached leaf that passes the far test itself takes its own
// far-field expansion, like a cluster; the rest of the reached leaves are
// evaluated directly (node sets, or recorded for the near-field pass).
template <bool F32, bool COUNT>
__device__ double traverse3d(const DevModel &Mdl, double qx, double qy, double qz, uint64_t mask, StackLDS &S,
                             int w, int &ncnt, int32_t *__restrict__ mylist, Ctr &ctr)
{
    if (Mdl.wave_accept) return traverse3d_wave<F32, COUNT>(Mdl, qx, qy, qz, mask, ncnt, mylist, ctr);
    const Node3 *__restrict__ nodes = (const Node3 *)Mdl.nodes;
    const TravParams M = trav_params(Mdl);
    const int lane = lane_id();
    double acc_far = 0.0, acc_leaf = 0.0;
    int cur = 0;
    uint64_t curmask = mask;
    int sp = 0;
    if (Mdl.n_nodes == 0) return 0.0;
    while (true) {
        const Node3 *nd = nodes + cur;
        const int right = nd->right;
        const bool active = (curmask >> lane) & 1;
        if (right < 0) {
            bool far = false;
            if (active && M.leaf_far) {
                far = far_term3d<F32>(M, nd, cur, qx, qy, qz, acc_far, curmask);
                if (COUNT && far) { ctr.v[GWN_C_FAR]++; ctr.v[GWN_C_LEAVES]++; }
            }
            acc_leaf += leaf3d<COUNT>(M, nd, cur, qx, qy, qz, active && !far, ncnt, mylist, ctr);
        } else {
            bool far = false;
            if (active) {
                if (COUNT) ctr.v[GWN_C_NODES]++;
                far = far_term3d<F32>(M, nd, cur, qx, qy, qz, acc_far, curmask);
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
    return acc_far + acc_leaf;
}

__device__ __forceinline__ int wave_segment(const LaunchTable &T, int wave)
{
    int lo = 0, hi = T.n_seg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (T.woff[mid] <= wave) lo = mid; else hi = mid - 1;
    }
    return uniform_i(lo);
}

// Pass 1 (3D): traversal of one wave of 64 sorted queries of one segment:
// far field and node-set leaves, near leaves recorded.  RECLASS: only the
// lanes flagged by the mixed form's first near pass, in FP64.
template <bool COUNT, bool RECLASS>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_trav3d(LaunchTable T, const double *__restrict__ pts,
                                                   const int32_t *__restrict__ perm, NearScratch NS,
                                                   long long *counters)
{
    __shared__ StackLDS S;
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    const int wave = xcd_block<kXcdRun3>() * kWavesPerBlock + w;
    if (wave >= T.n_waves) return;
    const int s = wave_segment(T, wave);
    const DevModel &M = T.models[T.seg_model[s]];
    const int64_t pos = T.qoff[s] + (int64_t)(wave - T.woff[s]) * T.qpw + lane;
    // per-query records are indexed by the query's position in the wave
    // grid (qpw per wave), read and written by valid lanes only
    const bool valid = lane < T.qpw && pos < T.qoff[s + 1];
    const int64_t slot = (int64_t)wave * T.qpw + (valid ? lane : 0);
    const bool act = valid && (!RECLASS || NS.need[slot]);
    const uint64_t mask = __ballot(act);
    if (!mask) return;
    const int row = act ? perm[pos] : 0;
    const double qx = act ? pts[3 * (int64_t)row] : 0.0;
    const double qy = act ? pts[3 * (int64_t)row + 1] : 0.0;
    const double qz = act ? pts[3 * (int64_t)row + 2] : 0.0;
    Ctr ctr;
#pragma unroll
    for (int k = 0; k < GWN_NCOUNTERS; ++k) ctr.v[k] = 0;
    int ncnt = 0;
    int32_t *mylist = NS.list + slot * kNearSlots;
    double part;
    if (!RECLASS && M.precision == GWN_MIXED)
        part = traverse3d<true, COUNT>(M, qx, qy, qz, mask, S, w, ncnt, mylist, ctr);
    else
        part = traverse3d<false, COUNT>(M, qx, qy, qz, mask, S, w, ncnt, mylist, ctr);
    if (act) {
        NS.part[slot] = part;
        NS.cnt[slot] = ncnt;
    }
    if (COUNT && RECLASS && act) ctr.v[GWN_C_RECLASS]++;
    flush_counters<COUNT>(ctr, counters);
}

// Pass 2 (3D): the near-field leaves of one query, in a workgroup of one
// wave.  The wave takes the query's (query, leaf) pairs one at a time in the
// traversal's order, and all 64 lanes evaluate each pair together (the
// rule's integrand evaluations are shared out over the lanes, its control
// is the same on all of them); the query adds its pairs' values one by one
// in that order, so its result does not depend on its batch mates.  Then
// classification and scatter.  Mixed form, first pass: a query with
// |w - 0.5| < band is flagged for the FP64 re-evaluation instead of
// written.
// One query per wave keeps the work of a wave small and even: a query has
// at most kNearSlots pairs, while the 64 queries of a traversal wave near a
// surface can hold hundreds of trimmed pairs (one such wave set the launch
// time on the CAD assembly).  Runs of kXcdRunNear consecutive queries stay
// on one XCD (neighbouring queries share leaves).  Two waves per SIMD (256
// registers each, some spilled) ran the bodies grid 13 % faster than one
// wave with no spill; four (128 registers) were slower again.
constexpr int kXcdRunNear = 256;

template <bool COUNT, bool RECLASS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_near3d(
    LaunchTable T, const int32_t *__restrict__ perm, NearScratch NS, const double *__restrict__ pts,
    double *__restrict__ out_w, uint8_t *__restrict__ out_in, long long *counters)
{
    const int lane = lane_id();
    const int64_t slot = uniform_i(xcd_block<kXcdRunNear>());   // query position in the wave grid
    const int wave = (int)(slot / T.qpw), j = (int)(slot - (int64_t)wave * T.qpw);
    if (wave >= T.n_waves) return;
    const int s = wave_segment(T, wave);
    const DevModel &M = T.models[T.seg_model[s]];
    const int64_t pos = T.qoff[s] + (int64_t)(wave - T.woff[s]) * T.qpw + j;
    if (pos >= T.qoff[s + 1]) return;
    if (RECLASS && !NS.need[slot]) return;
    const int row = perm[pos];
    const double qx = pts[3 * (int64_t)row], qy = pts[3 * (int64_t)row + 1], qz = pts[3 * (int64_t)row + 2];
    const int full = NS.cnt[slot];
    const int c = min(full, kNearSlots);
    Ctr ctr;
#pragma unroll
    for (int k = 0; k < GWN_NCOUNTERS; ++k) ctr.v[k] = 0;
    const DevWave wv;
    const Prim3 *__restrict__ prims = (const Prim3 *)M.prims;
    const Trim3 *__restrict__ trims = (const Trim3 *)M.trims;
    const Node3 *__restrict__ nodes = (const Node3 *)M.nodes;
    const double tol = 4.0 * kPi * M.eps_q;
    __shared__ NearShared sh;
    const int32_t *__restrict__ list = NS.list + slot * kNearSlots;
    double near_sum = 0.0;
    for (int k = 0; k < c; ++k) {
        const int leaf = uniform_i(-1 - nodes[list[k]].right);
        bool budget = false;   // a panel or piece missed its share of 4 pi eps_q
        double v = near3d<COUNT>(wv, c_quad, prims + leaf, trims, qx, qy, qz, M.eps_on, tol, budget, ctr, sh);
        if (budget) v = NAN;
        near_sum += v;
    }
    if (lane == 0) {
        double wq = (NS.part[slot] + near_sum) * (1.0 / (4.0 * kPi));
        // more near leaves than slots, or a leaf whose near-field rule could
        // not meet eps_q within its refinement budget (its value is NaN)
        const bool overflow = full > kNearSlots || !(wq == wq);
        if (overflow) {
            wq = NAN;
            atomicAdd((unsigned int *)M.flag, 1u);
            if (COUNT) ctr.v[GWN_C_OVERFLOW]++;
        }
        const bool band = !RECLASS && M.precision == GWN_MIXED && !overflow && fabs(wq - 0.5) < M.band;
        if (!RECLASS) NS.need[slot] = band ? 1 : 0;
        if (!band) {
            if (out_w) out_w[row] = wq;
            if (out_in) out_in[row] = wq >= 0.5 ? 1 : 0;
        }
    }
    flush_counters<COUNT>(ctr, counters);
}

static std::mutex g_tab_mu;
static bool g_tab_ready[64] = {false};

static hipError_t ensure_tables()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_tab_mu);
    if (dev >= 0 && dev < 64 && g_tab_ready[dev]) return hipSuccess;
    QuadTables t;
    gauss_kronrod01(kOuterN, t.xo, t.wo, t.go);
    gauss_kronrod01(kRadialN, t.xr, t.wr, t.gr);
    e = hipMemcpyToSymbol(HIP_SYMBOL(c_quad), &t, sizeof t);
    if (e == hipSuccess && dev >= 0 && dev < 64) g_tab_ready[dev] = true;
    return e;
}

gwn_status launch_query3d(const LaunchTable &T, const double *pts, const int32_t *perm, double *out_w,
                          uint8_t *out_in, long long *counters, char *near_buf, const NearBytes &near,
                          hipStream_t stream, std::string &err)
{
    hipError_t e = ensure_tables();
    if (e != hipSuccess) {
        err = std::string("quadrature tables: ") + hipGetErrorString(e);
        return GWN_EHIP;
    }
    const int grid = (T.n_waves + kWavesPerBlock - 1) / kWavesPerBlock;
    if (grid == 0) return GWN_OK;
    // per-slot records of the two passes, carved from the launch's scratch
    NearScratch NS;
    NS.part = (double *)near_buf;
    NS.cnt = (int32_t *)(near_buf + near.part);
    NS.list = (int32_t *)(near_buf + near.part + near.cnt);
    NS.need = (uint8_t *)(near_buf + near.part + near.cnt + near.list);
    bool any_mixed = false;
    for (int j = 0; j < T.n_seg; ++j) any_mixed |= T.models[T.seg_model[j]].precision == GWN_MIXED;
    const dim3 g(grid), b(kBlock);
    const dim3 gn((unsigned)((int64_t)T.n_waves * T.qpw)), bn(64);   // k_near3d: one wave per query slot
    if (counters) {
        hipLaunchKernelGGL((k_trav3d<true, false>), g, b, 0, stream, T, pts, perm, NS, counters);
        hipLaunchKernelGGL((k_near3d<true, false>), gn, bn, 0, stream, T, perm, NS, pts, out_w, out_in, counters);
        if (any_mixed) {
            hipLaunchKernelGGL((k_trav3d<true, true>), g, b, 0, stream, T, pts, perm, NS, counters);
            hipLaunchKernelGGL((k_near3d<true, true>), gn, bn, 0, stream, T, perm, NS, pts, out_w, out_in, counters);
        }
    } else {
        // each launch timed on its own while kernel timing is on
        hipEvent_t ev;
        prof_begin(stream, ev);
        hipLaunchKernelGGL((k_trav3d<false, false>), g, b, 0, stream, T, pts, perm, NS, counters);
        prof_end(stream, ev, GWN_K_TRAV3D);
        prof_begin(stream, ev);
        hipLaunchKernelGGL((k_near3d<false, false>), gn, bn, 0, stream, T, perm, NS, pts, out_w, out_in, counters);
        prof_end(stream, ev, GWN_K_NEAR3D);
        if (any_mixed) {
            prof_begin(stream, ev);
            hipLaunchKernelGGL((k_trav3d<false, true>), g, b, 0, stream, T, pts, perm, NS, counters);
            prof_end(stream, ev, GWN_K_TRAV3D);
            prof_begin(stream, ev);
            hipLaunchKernelGGL((k_near3d<false, true>), gn, bn, 0, stream, T, perm, NS, pts, out_w, out_in,
                               counters);
            prof_end(stream, ev, GWN_K_NEAR3D);
        }
    }
    e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("3D query launch: ") + hipGetErrorString(e);
        return GWN_EHIP;
    }
    return GWN_OK;
}

}  // namespace gwn
