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

void gauss_legendre01(int n, double *x, double *w);   // build3d.cpp

__constant__ QuadTables c_quad;

__device__ __forceinline__ void ctr_add(Ctr &c, int k, long long v) { c.v[k] += v; }

// Direct solid angle of one leaf at q (radians of solid angle).
template <bool COUNT>
__device__ double leaf3d(const DevModel &M, const Node3 *__restrict__ nd, double qx, double qy, double qz,
                         bool active, Ctr &ctr)
{
    const int leaf = -1 - nd->right;
    const double dx = fmax(fmax(nd->t[0] - qx, qx - nd->t[3]), 0.0);
    const double dy = fmax(fmax(nd->t[1] - qy, qy - nd->t[4]), 0.0);
    const double dz = fmax(fmax(nd->t[2] - qz, qz - nd->t[5]), 0.0);
    const double ex = nd->t[3] - nd->t[0], ey = nd->t[4] - nd->t[1], ez = nd->t[5] - nd->t[2];
    const double d2 = dx * dx + dy * dy + dz * dz, diag2 = ex * ex + ey * ey + ez * ez;
    const bool near = d2 < M.near_ratio2 * diag2;
    double om = 0.0;
    if (COUNT && active) ctr.v[GWN_C_LEAVES]++;
    if (active && !near) {
        // rule by distance / half-diagonal ratio (finest near, coarsest far)
        const double r2 = 4.0 * d2 / diag2;
        const int c0 = (int)nd->t[6], c1 = (int)nd->t[7], c2 = (int)nd->t[8];
        int off = 0, cnt = c0;
        if (r2 >= kLeafRuleRatio[2] * kLeafRuleRatio[2]) { off = c0 + c1; cnt = c2; }
        else if (r2 >= kLeafRuleRatio[1] * kLeafRuleRatio[1]) { off = c0; cnt = c1; }
        const QNode3 *__restrict__ qn = (const QNode3 *)M.qnodes + nd->aux + off;
        for (int k = 0; k < cnt; ++k) {
            const double rx = qn[k].x[0] - qx, ry = qn[k].x[1] - qy, rz = qn[k].x[2] - qz;
            const double r2 = rx * rx + ry * ry + rz * rz;
            const double inv = 1.0 / sqrt(r2);
            om += (qn[k].n[0] * rx + qn[k].n[1] * ry + qn[k].n[2] * rz) * (inv * inv * inv);
        }
        if (COUNT) { ctr.v[GWN_C_LEAF_FAST]++; ctr.v[GWN_C_ANGLES] += cnt; }
    }
    if (active && near) {
        om = near3d<COUNT>(c_quad, (const Prim3 *)M.prims + leaf, (const Trim3 *)M.trims, qx, qy, qz, M.eps_on, ctr);
    }
    return om;
}

template <typename T>
__device__ __forceinline__ T taylor3d(T sx, T sy, T sz, T r2, const T *t, int order)
{
    const T inv2 = T(1) / r2;
    const T inv1 = sqrt(inv2);
    const T inv3 = inv1 * inv2;
    T w = (sx * t[0] + sy * t[1] + sz * t[2]) * inv3;
    if (order >= 1) {
        const T tr = t[3] + t[4] + t[5];
        const T sms = t[3] * sx * sx + t[4] * sy * sy + t[5] * sz * sz + t[6] * sx * sy + t[7] * sx * sz +
                      t[8] * sy * sz;
        w += tr * inv3 - T(3) * sms * inv3 * inv2;
    }
    if (order >= 2) {
        const T es = t[9] * sx + t[10] * sy + t[11] * sz;
        const T cub = t[12] * sx * sx * sx + t[13] * sy * sy * sy + t[14] * sz * sz * sz + t[15] * sx * sx * sy +
                      t[16] * sx * sx * sz + t[17] * sy * sy * sx + t[18] * sy * sy * sz + t[19] * sz * sz * sx +
                      t[20] * sz * sz * sy + t[21] * sx * sy * sz;
        const T inv5 = inv3 * inv2;
        w += T(0.5) * (T(-3) * es * inv5 + T(15) * cub * inv5 * inv2);
    }
    return w;   // solid angle (times 4 pi of w)
}

template <bool F32, bool COUNT>
__device__ double traverse3d(const DevModel &M, double qx, double qy, double qz, uint64_t mask, StackLDS &S, int w,
                             Ctr &ctr)
{
    const Node3 *__restrict__ nodes = (const Node3 *)M.nodes;
    const int lane = lane_id();
    const float qxf = (float)qx, qyf = (float)qy, qzf = (float)qz;
    const double beta2 = F32 ? M.beta2_mixed : M.beta2;
    const float beta2f = (float)M.beta2_mixed;
    double acc_far = 0.0, acc_leaf = 0.0;
    int cur = 0;
    uint64_t curmask = mask;
    int sp = 0;
    if (M.n_nodes == 0) return 0.0;
    while (true) {
        const Node3 *nd = nodes + cur;
        const int right = nd->right;
        const bool active = (curmask >> lane) & 1;
        if (right < 0) {
            acc_leaf += leaf3d<COUNT>(M, nd, qx, qy, qz, active, ctr);
        } else {
            bool far = false;
            if (active) {
                if (COUNT) ctr.v[GWN_C_NODES]++;
                if (F32) {
                    const float sx = nd->fc[0] - qxf, sy = nd->fc[1] - qyf, sz = nd->fc[2] - qzf;
                    const float r2 = sx * sx + sy * sy + sz * sz;
                    far = r2 > beta2f * nd->fr2;
                    if (far) acc_far += (double)taylor3d<float>(sx, sy, sz, r2, nd->ft, M.order);
                } else {
                    const double sx = nd->c[0] - qx, sy = nd->c[1] - qy, sz = nd->c[2] - qz;
                    const double r2 = sx * sx + sy * sy + sz * sz;
                    far = r2 > beta2 * nd->r2;
                    if (far) acc_far += taylor3d<double>(sx, sy, sz, r2, nd->t, M.order);
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
    return (acc_far + acc_leaf) * (1.0 / (4.0 * kPi));
}

template <bool COUNT>
__global__ __launch_bounds__(kBlock) void k_query3d(LaunchTable T, const double *__restrict__ pts,
                                                    const int32_t *__restrict__ perm, double *__restrict__ out_w,
                                                    uint8_t *__restrict__ out_in, long long *counters)
{
    __shared__ StackLDS S;
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    const int wave = blockIdx.x * kWavesPerBlock + w;
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
    const int64_t pos = T.qoff[s] + (int64_t)(wave - T.woff[s]) * 64 + lane;
    const bool valid = pos < T.qoff[s + 1];
    const int row = valid ? perm[pos] : 0;
    const double qx = valid ? pts[3 * (int64_t)row] : 0.0;
    const double qy = valid ? pts[3 * (int64_t)row + 1] : 0.0;
    const double qz = valid ? pts[3 * (int64_t)row + 2] : 0.0;
    const uint64_t mask = __ballot(valid);
    Ctr ctr;
#pragma unroll
    for (int k = 0; k < GWN_NCOUNTERS; ++k) ctr.v[k] = 0;
    double wq;
    if (M.precision == GWN_MIXED) {
        wq = traverse3d<true, COUNT>(M, qx, qy, qz, mask, S, w, ctr);
        const bool need = valid && fabs(wq - 0.5) < M.band;
        const uint64_t rmask = __ballot(need);
        if (rmask) {
            const double r = traverse3d<false, COUNT>(M, qx, qy, qz, rmask, S, w, ctr);
            if (need) wq = r;
            if (COUNT && need) ctr.v[GWN_C_RECLASS]++;
        }
    } else {
        wq = traverse3d<false, COUNT>(M, qx, qy, qz, mask, S, w, ctr);
    }
    if (valid) {
        if (out_w) out_w[row] = wq;
        if (out_in) out_in[row] = wq >= 0.5 ? 1 : 0;
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
    gauss_legendre01(kOuterGL, t.gx8, t.gw8);
    gauss_legendre01(kRadialGL, t.gx12, t.gw12);
    e = hipMemcpyToSymbol(HIP_SYMBOL(c_quad), &t, sizeof t);
    if (e == hipSuccess && dev >= 0 && dev < 64) g_tab_ready[dev] = true;
    return e;
}

gwn_status launch_query3d(const LaunchTable &T, const double *pts, const int32_t *perm, double *out_w,
                          uint8_t *out_in, long long *counters, hipStream_t stream, std::string &err)
{
    hipError_t e = ensure_tables();
    if (e != hipSuccess) {
        err = std::string("quadrature tables: ") + hipGetErrorString(e);
        return GWN_EHIP;
    }
    const int grid = (T.n_waves + kWavesPerBlock - 1) / kWavesPerBlock;
    if (grid == 0) return GWN_OK;
    if (counters)
        hipLaunchKernelGGL(k_query3d<true>, dim3(grid), dim3(kBlock), 0, stream, T, pts, perm, out_w, out_in,
                           counters);
    else
        hipLaunchKernelGGL(k_query3d<false>, dim3(grid), dim3(kBlock), 0, stream, T, pts, perm, out_w, out_in,
                           nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("3D query launch: ") + hipGetErrorString(e);
        return GWN_EHIP;
    }
    return GWN_OK;
}

}  // namespace gwn
