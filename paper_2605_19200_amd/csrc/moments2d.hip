// Device preprocessing of a 2D model: the adaptive subdivision of the input
// curves (Sec. 3.2) and the per-cluster chord moments.
//
// Subdivision: one thread per input curve walks its halving tree depth
// first, left half first, with the same arithmetic as the host build (exact
// midpoints, box by division, the squared diagonal against the squared
// limit, no FMA contraction), so the leaves are the host's bit for bit; a
// counting pass sizes each curve's leaves, a second pass writes them.
//
// Chord moments: the per-cluster chord moments of a 2D model
// (ComputeUncenteredMoments of Alg. 1, taken directly about each cluster's
// centroid): the centred complex moments m_k = integral (z - c)^k dz over the
// chords of the cluster's leaves (Sec. 3.1, the series of Eq. taylor in
// complex form), and the magnitudes of the scaled moments m_k / r^(k+1) up
// to kTailOrder2D with the total scaled chord length, which the
// error-budgeted far test bounds its truncation with.
//
// One wave per cluster.  A DFS subtree's leaves are contiguous in leaf
// order, so a cluster is a range [lb, le) of the chord array; the lanes take
// its chords in turn and the wave sums their partial moments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "gwn_internal.h"

namespace gwn {

namespace {

struct MomIn {
    double cx, cy;   // centroid
    double scale;    // 1 (centred moments) or 1 / r (scaled magnitudes)
    int32_t lb, le;  // chord range; empty for leaves and for skipped clusters
};

constexpr int kMomWaves = 4;

// K orders of sum over chords of (b - a) s_k / (k + 1), s_k = sum_{j<=k}
// b^j a^(k-j), in the variables (z - c) * scale.  MAG: write |m_k| for
// k < K and the summed chord length; else the (re, im) pairs.
template <int K, bool MAG>
__global__ __launch_bounds__(64 * kMomWaves) void k_moments2d(const MomIn *__restrict__ in,
                                                            const double *__restrict__ ends, int n_nodes,
                                                            double *__restrict__ out, int stride)
{
    const int lane = threadIdx.x & 63;
    const int node = blockIdx.x * kMomWaves + (threadIdx.x >> 6);
    if (node >= n_nodes) return;
    const MomIn t = in[node];
    if (t.le <= t.lb) return;
    double acc[2 * K];
#pragma unroll
    for (int k = 0; k < 2 * K; ++k) acc[k] = 0.0;
    double len = 0.0;
    for (int j = t.lb + lane; j < t.le; j += 64) {
        const double ar = (ends[4 * j] - t.cx) * t.scale, ai = (ends[4 * j + 1] - t.cy) * t.scale;
        const double br = (ends[4 * j + 2] - t.cx) * t.scale, bi = (ends[4 * j + 3] - t.cy) * t.scale;
        const double dr = br - ar, di = bi - ai;
        if (MAG) len += sqrt(dr * dr + di * di);
        double sr = 1.0, si = 0.0, pr = 1.0, pi = 0.0;   // s_k and a^k
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k > 0) {
                const double npr = pr * ar - pi * ai, npi = pr * ai + pi * ar;
                pr = npr;
                pi = npi;
                const double nsr = br * sr - bi * si + pr, nsi = br * si + bi * sr + pi;
                sr = nsr;
                si = nsi;
            }
            acc[2 * k] += (dr * sr - di * si) / (k + 1);
            acc[2 * k + 1] += (dr * si + di * sr) / (k + 1);
        }
    }
#pragma unroll
    for (int k = 0; k < 2 * K; ++k)
        for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off);
    if (MAG)
        for (int off = 32; off > 0; off >>= 1) len += __shfl_xor(len, off);
    if (lane != 0) return;
    double *o = out + (size_t)node * stride;
    if (MAG) {
#pragma unroll
        for (int k = 0; k < K; ++k) o[k] = sqrt(acc[2 * k] * acc[2 * k] + acc[2 * k + 1] * acc[2 * k + 1]);
        o[K] = len;
    } else {
#pragma unroll
        for (int k = 0; k < 2 * K; ++k) o[k] = acc[k];
    }
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

gwn_status moments2d_device(int device, const std::vector<HostNode> &nodes, const std::vector<int> &end,
                            const std::vector<double> &chord_ends, std::vector<double> &cmom2,
                            std::vector<double> &tail2, std::string &err)
{
    const int nn = (int)nodes.size();
    const int nl = (int)(chord_ends.size() / 4);
    // leaves before each DFS position: a subtree [i, end_i) holds the chords
    // [before[i], before[end_i])
    std::vector<int> before(nn + 1, 0);
    for (int i = 0; i < nn; ++i) before[i + 1] = before[i] + (nodes[i].is_leaf ? 1 : 0);
    if (before[nn] != nl) { err = "moments: leaf count mismatch"; return GWN_EINVAL; }
    std::vector<MomIn> cin(nn), tin(nn);
    for (int i = 0; i < nn; ++i) {
        const HostNode &nd = nodes[i];
        const int lb = before[i], le = before[end[i]];
        const bool internal = !nd.is_leaf;
        cin[i] = MomIn{nd.c[0], nd.c[1], 1.0, lb, internal ? le : lb};
        const bool scaled = internal && nd.r > 0;
        tin[i] = MomIn{nd.c[0], nd.c[1], scaled ? 1.0 / nd.r : 1.0, lb, scaled ? le : lb};
    }
    constexpr int KC = kMaxOrder2D + 1, KT = kTailOrder2D + 1;
    const size_t cbytes = (size_t)nn * 2 * KC * sizeof(double), tbytes = (size_t)nn * kTailStride2D * sizeof(double);
    DevBuf d_ends, d_cin, d_tin, d_cout, d_tout;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMalloc(&d_ends.p, std::max<size_t>(chord_ends.size() * sizeof(double), 8));
    if (e == hipSuccess) e = hipMalloc(&d_cin.p, nn * sizeof(MomIn));
    if (e == hipSuccess) e = hipMalloc(&d_tin.p, nn * sizeof(MomIn));
    if (e == hipSuccess) e = hipMalloc(&d_cout.p, cbytes);
    if (e == hipSuccess) e = hipMalloc(&d_tout.p, tbytes);
    if (e == hipSuccess && !chord_ends.empty())
        e = hipMemcpy(d_ends.p, chord_ends.data(), chord_ends.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_cin.p, cin.data(), nn * sizeof(MomIn), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_tin.p, tin.data(), nn * sizeof(MomIn), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(d_cout.p, 0, cbytes);
    if (e == hipSuccess) e = hipMemset(d_tout.p, 0, tbytes);
    if (e == hipSuccess) {
        const dim3 grid((nn + kMomWaves - 1) / kMomWaves), block(64 * kMomWaves);
        hipLaunchKernelGGL((k_moments2d<KC, false>), grid, block, 0, 0, (const MomIn *)d_cin.p,
                           (const double *)d_ends.p, nn, (double *)d_cout.p, 2 * KC);
        hipLaunchKernelGGL((k_moments2d<KT, true>), grid, block, 0, 0, (const MomIn *)d_tin.p,
                           (const double *)d_ends.p, nn, (double *)d_tout.p, kTailStride2D);
        e = hipGetLastError();
    }
    cmom2.assign((size_t)nn * 2 * KC, 0.0);
    tail2.assign((size_t)nn * kTailStride2D, 0.0);
    if (e == hipSuccess) e = hipMemcpy(cmom2.data(), d_cout.p, cbytes, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(tail2.data(), d_tout.p, tbytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        err = std::string("device moments: ") + hipGetErrorString(e);
        return GWN_EHIP;
    }
    return GWN_OK;
}

namespace {

constexpr int kMaxSplitDepth = 40;

// Leaves of curve i: counted (out_h == nullptr) into counts[i], or written
// from offs[i] on (at most counts[i] of them: the counting pass bounds the
// writes).
__global__ __launch_bounds__(256) void k_subdiv2d(int64_t n, const double *__restrict__ cubics, double limit2,
                                                int64_t *__restrict__ counts, const int64_t *__restrict__ offs,
                                                double *__restrict__ out_h, int32_t *__restrict__ out_curve)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double stk[kMaxSplitDepth + 1][12];
    int dep[kMaxSplitDepth + 1];
    for (int k = 0; k < 12; ++k) stk[0][k] = cubics[12 * i + k];
    dep[0] = 0;
    int sp = 1;
    int64_t pos = out_h ? offs[i] : 0, cnt = 0;
    const int64_t end = out_h ? pos + counts[i] : 0;
    while (sp > 0) {
        --sp;
        double c[12];
        for (int k = 0; k < 12; ++k) c[k] = stk[sp][k];
        const int depth = dep[sp];
        double lo0 = INFINITY, lo1 = INFINITY, hi0 = -INFINITY, hi1 = -INFINITY;
        for (int j = 0; j < 4; ++j) {
            const double x = c[3 * j] / c[3 * j + 2], y = c[3 * j + 1] / c[3 * j + 2];
            lo0 = fmin(lo0, x); hi0 = fmax(hi0, x);
            lo1 = fmin(lo1, y); hi1 = fmax(hi1, y);
        }
        const double dx = hi0 - lo0, dy = hi1 - lo1;
        if (limit2 > 0.0 && dx * dx + dy * dy >= limit2 && depth < kMaxSplitDepth) {
            // halves at t = 1/2: right pushed first, so the left is taken next
            double L[12], R[12];
            for (int k = 0; k < 3; ++k) {
                const double b0 = 0.5 * (c[k] + c[3 + k]), b1 = 0.5 * (c[3 + k] + c[6 + k]),
                             b2 = 0.5 * (c[6 + k] + c[9 + k]);
                const double c0 = 0.5 * (b0 + b1), c1 = 0.5 * (b1 + b2);
                const double d0 = 0.5 * (c0 + c1);
                L[k] = c[k]; L[3 + k] = b0; L[6 + k] = c0; L[9 + k] = d0;
                R[k] = d0; R[3 + k] = c1; R[6 + k] = b2; R[9 + k] = c[9 + k];
            }
            for (int k = 0; k < 12; ++k) stk[sp][k] = R[k];
            dep[sp] = depth + 1;
            for (int k = 0; k < 12; ++k) stk[sp + 1][k] = L[k];
            dep[sp + 1] = depth + 1;
            sp += 2;
        } else {
            if (out_h && pos < end) {
                for (int k = 0; k < 12; ++k) out_h[12 * pos + k] = c[k];
                out_curve[pos] = (int32_t)i;
                ++pos;
            }
            ++cnt;
        }
    }
    if (!out_h) counts[i] = cnt;
}

}  // namespace

gwn_status subdiv2d_device(int device, const std::vector<double> &cubics, double limit2,
                           std::vector<double> &leaf_h, std::vector<int32_t> &leaf_curve, std::string &err)
{
    const int64_t n = (int64_t)(cubics.size() / 12);
    leaf_h.clear();
    leaf_curve.clear();
    if (n == 0) return GWN_OK;
    DevBuf d_c, d_cnt, d_off, d_h, d_i;
    std::vector<int64_t> cnt(n), off(n);
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMalloc(&d_c.p, cubics.size() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&d_cnt.p, n * sizeof(int64_t));
    if (e == hipSuccess) e = hipMemcpy(d_c.p, cubics.data(), cubics.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_subdiv2d, grid, block, 0, 0, n, (const double *)d_c.p, limit2, (int64_t *)d_cnt.p,
                           (const int64_t *)nullptr, (double *)nullptr, (int32_t *)nullptr);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(cnt.data(), d_cnt.p, n * sizeof(int64_t), hipMemcpyDeviceToHost);
    int64_t total = 0;
    if (e == hipSuccess)
        for (int64_t i = 0; i < n; ++i) {
            off[i] = total;
            total += cnt[i];
        }
    if (e == hipSuccess && total > ((int64_t)1 << 30)) {
        err = "too many leaves";
        return GWN_EINVAL;
    }
    if (e == hipSuccess) e = hipMalloc(&d_off.p, n * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc(&d_h.p, (size_t)total * 12 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&d_i.p, (size_t)total * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemcpy(d_off.p, off.data(), n * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_subdiv2d, grid, block, 0, 0, n, (const double *)d_c.p, limit2, (int64_t *)d_cnt.p,
                           (const int64_t *)d_off.p, (double *)d_h.p, (int32_t *)d_i.p);
        e = hipGetLastError();
    }
    leaf_h.resize((size_t)total * 12);
    leaf_curve.resize((size_t)total);
    if (e == hipSuccess) e = hipMemcpy(leaf_h.data(), d_h.p, leaf_h.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(leaf_curve.data(), d_i.p, leaf_curve.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        err = std::string("device subdivision: ") + hipGetErrorString(e);
        return GWN_EHIP;
    }
    return GWN_OK;
}

}  // namespace gwn
