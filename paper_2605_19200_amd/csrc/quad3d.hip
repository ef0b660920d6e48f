// Device leaf quadrature of a 3D model (Alg. 1 ComputeUncenteredMoments for
// trimmed rational patches, Sec. 3.1): the Green-scattered Gauss-Legendre
// nodes of every leaf, their moments, and the node sets of the leaf's direct
// rules, computed where the model lives instead of on host threads.
//
// The visible region of a leaf's parameter square is bounded by its trim
// loops (or, untrimmed, by the square, whose only contributing edge is
// u = 1).  Green's theorem turns the surface integral of f over that region
// into a line integral over the boundary of the integral of f along the
// horizontal segment from u = 0 to the boundary point: an outer rule of n_o
// nodes along each boundary curve, an inner rule of n_i nodes along each
// segment, weight w_o dv/dt w_i u per node, the surface point at (t u, v)
// and its normal S_u x S_v.  The same scattering gives the moment rule (the
// model's gl_nodes per direction) and the three node-set rules of the
// leaf's direct evaluation (12, 8 and 6 per direction).  Outer nodes where
// u = 0 or dv/dt = 0 carry no weight and are left out, as on the host.
//
// One wave per leaf.  Moments: each lane sums the nodes it takes, the wave
// then adds the lanes' sums (the order differs from the host's, so values
// agree to rounding); the multipole moments about the leaf's centroid are
// added term by term across the wave per group of 64 nodes.  Node sets: in
// the order of the host build (rule, curve, outer node, inner node), each
// group of outer nodes compacted through a ballot, written at the leaf's
// place in the tree's leaf order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "gwn_internal.h"

namespace gwn {

namespace {

struct QuadTab {
    double x[4][kMaxQuadRule], w[4][kMaxQuadRule];   // rules 0-2: node sets; 3: moments
    int32_t n[4];
};

__device__ __forceinline__ void cubic_basis_d(double t, double *B, double *dB)
{
    const double s = 1.0 - t;
    B[0] = s * s * s; B[1] = 3 * s * s * t; B[2] = 3 * s * t * t; B[3] = t * t * t;
    dB[0] = -3 * s * s; dB[1] = 3 * s * s - 6 * s * t; dB[2] = 6 * s * t - 3 * t * t; dB[3] = 3 * t * t;
}

// Euclidean point S and normal S_u x S_v of the rational bicubic h (the
// homogeneous net [i along u][j along v][wx, wy, wz, w], in LDS) at (u, v).
__device__ __forceinline__ void surface_d(const double *h, double u, double v, double S[3], double N[3])
{
    double bu[4], du[4], bv[4], dv[4];
    cubic_basis_d(u, bu, du);
    cubic_basis_d(v, bv, dv);
    double H[4] = {0, 0, 0, 0}, Hu[4] = {0, 0, 0, 0}, Hv[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double c = h[16 * i + 4 * j + k];
                H[k] += bu[i] * bv[j] * c;
                Hu[k] += du[i] * bv[j] * c;
                Hv[k] += bu[i] * dv[j] * c;
            }
    const double W = H[3];
    double Su[3], Sv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        S[k] = H[k] / W;
        Su[k] = (Hu[k] * W - H[k] * Hu[3]) / (W * W);
        Sv[k] = (Hv[k] * W - H[k] * Hv[3]) / (W * W);
    }
    N[0] = Su[1] * Sv[2] - Su[2] * Sv[1];
    N[1] = Su[2] * Sv[0] - Su[0] * Sv[2];
    N[2] = Su[0] * Sv[1] - Su[1] * Sv[0];
}

// point (u, v) and derivative (du, dv) of the rational quadratic trim curve
// (homogeneous control points (w u, w v, w) x 3) at t.  Whether an outer
// node carries weight (u != 0 and dv != 0) decides the node-set sizes, which
// two kernels must agree on bit for bit: no contraction into FMAs here, so
// every instance rounds alike (and as the host does).
__device__ __forceinline__ void trim_point_d(const Trim3 &c, double t, double &u, double &v, double &du, double &dv)
{
#pragma clang fp contract(off)
    const double s = 1.0 - t;
    const double b[3] = {s * s, 2 * s * t, t * t}, d[3] = {-2 * s, 2 * s - 2 * t, 2 * t};
    double hu = 0, hv = 0, hw = 0, gu = 0, gv = 0, gw = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        hu += b[i] * c.h[3 * i]; hv += b[i] * c.h[3 * i + 1]; hw += b[i] * c.h[3 * i + 2];
        gu += d[i] * c.h[3 * i]; gv += d[i] * c.h[3 * i + 1]; gw += d[i] * c.h[3 * i + 2];
    }
    u = hu / hw;
    v = hv / hw;
    du = (gu * hw - hu * gw) / (hw * hw);
    dv = (gv * hw - hv * gw) / (hw * hw);
}

__device__ __forceinline__ double wave_sum(double v)
{
    // butterfly: every lane ends with the same sum (x + y == y + x)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int kMomU = 39;   // n_moments(3)

// One wave per leaf: uncentred moments U, area Wt, area-weighted centroid
// sums WC, centroid LC, multipole moments LN about LC, node-set sizes.
__global__ __launch_bounds__(64) void k_leaf_moments3d(int nl, const double *__restrict__ nets,
                                                       const Trim3 *__restrict__ curves,
                                                       const int64_t *__restrict__ coff,
                                                       const double *__restrict__ box, const QuadTab *__restrict__ tab,
                                                       double *__restrict__ U, double *__restrict__ Wt,
                                                       double *__restrict__ WC, double *__restrict__ LC,
                                                       double *__restrict__ LN, int32_t *__restrict__ counts)
{
    const int li = blockIdx.x;
    if (li >= nl) return;
    const int lane = threadIdx.x;
    __shared__ double h[64];
    h[lane] = nets[64 * (int64_t)li + lane];
    __syncthreads();
    const int64_t c0 = coff[li];
    const int nc = (int)(coff[li + 1] - c0);
    const int g = tab->n[3];
    const double *gx = tab->x[3], *gw = tab->w[3];
    const int items = nc * g * g;

    // uncentred moments, area and centroid sums
    double u[kMomU + 4];
#pragma unroll
    for (int k = 0; k < kMomU + 4; ++k) u[k] = 0.0;
    for (int it = lane; it < items; it += 64) {
        const int c = it / (g * g), k = (it / g) % g, j = it % g;
        double uk, vk, duk, dvk;
        trim_point_d(curves[c0 + c], gx[k], uk, vk, duk, dvk);
        if (dvk == 0.0 || uk == 0.0) continue;
        const double W = gw[k] * dvk * gw[j] * uk;
        double S[3], N[3];
        surface_d(h, gx[j] * uk, vk, S, N);
        const double n[3] = {W * N[0], W * N[1], W * N[2]};
        const double area = W * sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] += n[a];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) u[3 + 3 * a + b] += S[a] * n[b];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int k2 = 0; k2 < 3; ++k2) u[12 + 9 * a + 3 * b + k2] += S[a] * S[b] * n[k2];
        u[kMomU] += area;
#pragma unroll
        for (int a = 0; a < 3; ++a) u[kMomU + 1 + a] += area * S[a];
    }
#pragma unroll
    for (int k = 0; k < kMomU + 4; ++k) u[k] = wave_sum(u[k]);
    const double wt = u[kMomU];
    double cl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        cl[a] = wt > 0.0 ? u[kMomU + 1 + a] / wt : 0.5 * (box[6 * (int64_t)li + a] + box[6 * (int64_t)li + 3 + a]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < kMomU; ++k) U[kMomU * (int64_t)li + k] = u[k];
        Wt[li] = wt;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            WC[3 * (int64_t)li + a] = u[kMomU + 1 + a];
            LC[3 * (int64_t)li + a] = cl[a];
        }
    }

    // multipole moments N_l^m = - sum n . conj(grad R_l^m(x - c)), 1 <= l <=
    // kMaxLTail3, with R and its gradient by the recurrences of the host
    // (multipole3d.h); lane t keeps term t's sum
    double nre = 0.0, nim = 0.0;
    const int rounds = (items + 63) / 64;
    for (int rd = 0; rd < rounds; ++rd) {
        const int it = rd * 64 + lane;
        double W = 0.0, S[3] = {cl[0], cl[1], cl[2]}, N[3] = {0.0, 0.0, 0.0};
        if (it < items) {
            const int c = it / (g * g), k = (it / g) % g, j = it % g;
            double uk, vk, duk, dvk;
            trim_point_d(curves[c0 + c], gx[k], uk, vk, duk, dvk);
            if (!(dvk == 0.0 || uk == 0.0)) {
                W = gw[k] * dvk * gw[j] * uk;
                surface_d(h, gx[j] * uk, vk, S, N);
            }
        }
        const double nw[3] = {W * N[0], W * N[1], W * N[2]};
        const double d[3] = {S[0] - cl[0], S[1] - cl[1], S[2] - cl[2]};
        const double rho2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        double mr = 1.0, mi = 0.0;                      // R_m^m
        double gr[3] = {0, 0, 0}, gi[3] = {0, 0, 0};    // grad R_m^m
#pragma unroll
        for (int m = 0; m <= kMaxLTail3; ++m) {
            if (m > 0) {
                const double f = 1.0 / (2 * m);
                // (R + grad) * (x + i y) / (2m), with d(x + i y) = (1, i, 0)
                double ngr[3], ngi[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    ngr[a] = (gr[a] * d[0] - gi[a] * d[1]) * f;
                    ngi[a] = (gr[a] * d[1] + gi[a] * d[0]) * f;
                }
                ngr[0] += mr * f;
                ngi[0] += mi * f;
                ngr[1] -= mi * f;
                ngi[1] += mr * f;
                const double nr = (mr * d[0] - mi * d[1]) * f, ni = (mr * d[1] + mi * d[0]) * f;
                mr = nr;
                mi = ni;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    gr[a] = ngr[a];
                    gi[a] = ngi[a];
                }
            }
            // column m: (l - 1, l - 2) values and gradients
            double r1r = mr, r1i = mi, r2r = 0.0, r2i = 0.0;
            double g1r[3] = {gr[0], gr[1], gr[2]}, g1i[3] = {gi[0], gi[1], gi[2]};
            double g2r[3] = {0, 0, 0}, g2i[3] = {0, 0, 0};
#pragma unroll
            for (int l = m; l <= kMaxLTail3; ++l) {
                if (l > m) {
                    const double den = 1.0 / ((double)(l - m) * (l + m));
                    const double c1 = (2.0 * l - 1.0) * d[2];
                    const double rr = (c1 * r1r - rho2 * r2r) * den, ri = (c1 * r1i - rho2 * r2i) * den;
                    double hr[3], hi[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const double dz = a == 2 ? 1.0 : 0.0;
                        hr[a] = ((2.0 * l - 1.0) * (dz * r1r + d[2] * g1r[a]) - (2.0 * d[a] * r2r + rho2 * g2r[a])) * den;
                        hi[a] = ((2.0 * l - 1.0) * (dz * r1i + d[2] * g1i[a]) - (2.0 * d[a] * r2i + rho2 * g2i[a])) * den;
                    }
                    r2r = r1r; r2i = r1i;
                    r1r = rr; r1i = ri;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        g2r[a] = g1r[a]; g2i[a] = g1i[a];
                        g1r[a] = hr[a]; g1i[a] = hi[a];
                    }
                }
                if (l >= 1) {
                    // - n . conj(grad R): real part -sum n gr, imaginary +sum n gi
                    const double sre = wave_sum(-(nw[0] * g1r[0] + nw[1] * g1r[1] + nw[2] * g1r[2]));
                    const double sim = wave_sum(nw[0] * g1i[0] + nw[1] * g1i[1] + nw[2] * g1i[2]);
                    if (lane == l * (l + 1) / 2 - 1 + m) {
                        nre += sre;
                        nim += sim;
                    }
                }
            }
        }
    }
    if (lane < kMpoleTermsTail) {
        LN[2 * ((int64_t)li * kMpoleTermsTail + lane)] = nre;
        LN[2 * ((int64_t)li * kMpoleTermsTail + lane) + 1] = nim;
    }

    // node-set sizes: outer nodes that carry weight, times the inner rule
    for (int r = 0; r < 3; ++r) {
        const int no = tab->n[r];
        int valid = 0;
        for (int p = lane; p < nc * no; p += 64) {
            double uk, vk, duk, dvk;
            trim_point_d(curves[c0 + p / no], tab->x[r][p % no], uk, vk, duk, dvk);
            valid += (dvk == 0.0 || uk == 0.0) ? 0 : 1;
        }
        const double tot = wave_sum((double)valid);
        if (lane == 0) counts[3 * (int64_t)li + r] = (int32_t)tot * no;
    }
}

// One wave per leaf: the node sets of the three rules, at qbase[li] in the
// model's node-set array, in the host's order.
__global__ __launch_bounds__(64) void k_leaf_nodes3d(int nl, const double *__restrict__ nets,
                                                     const Trim3 *__restrict__ curves,
                                                     const int64_t *__restrict__ coff,
                                                     const QuadTab *__restrict__ tab,
                                                     const int64_t *__restrict__ qbase,
                                                     const int32_t *__restrict__ counts, QNode3 *__restrict__ out)
{
    const int li = blockIdx.x;
    if (li >= nl) return;
    const int lane = threadIdx.x;
    __shared__ double h[64];
    __shared__ double pk[64][4];   // compacted outer nodes: u, v, weight factor w_o dv/dt u, and unused
    h[lane] = nets[64 * (int64_t)li + lane];
    __syncthreads();
    const int64_t c0 = coff[li];
    const int nc = (int)(coff[li + 1] - c0);
    int64_t pos = qbase[li];
    // the sizes counted by k_leaf_moments3d bound every write
    const int64_t end = pos + (int64_t)counts[3 * (int64_t)li] + counts[3 * (int64_t)li + 1] + counts[3 * (int64_t)li + 2];
    for (int r = 0; r < 3; ++r) {
        const int no = tab->n[r];
        const double *xr = tab->x[r], *wr = tab->w[r];
        for (int p0 = 0; p0 < nc * no; p0 += 64) {
            const int p = p0 + lane;
            double uk = 0.0, vk = 0.0, duk = 0.0, dvk = 0.0;
            bool ok = false;
            if (p < nc * no) {
                trim_point_d(curves[c0 + p / no], xr[p % no], uk, vk, duk, dvk);
                ok = !(dvk == 0.0 || uk == 0.0);
            }
            const uint64_t bal = __ballot(ok);
            const int slot = __popcll(bal & ((1ull << lane) - 1ull));
            __syncthreads();
            if (ok) {
                pk[slot][0] = uk;
                pk[slot][1] = vk;
                pk[slot][2] = wr[p % no] * dvk * uk;
            }
            __syncthreads();
            const int nv = __popcll(bal);
            for (int it = lane; it < nv * no; it += 64) {
                const int s = it / no, j = it % no;
                const double W = pk[s][2] * wr[j];
                double S[3], N[3];
                surface_d(h, xr[j] * pk[s][0], pk[s][1], S, N);
                QNode3 q;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    q.x[a] = S[a];
                    q.n[a] = W * N[a];
                }
                if (pos + it < end) out[pos + it] = q;
            }
            pos += (int64_t)nv * no;
        }
    }
}

}  // namespace

LeafQuad3::~LeafQuad3()
{
    if (device < 0) return;
    (void)hipSetDevice(device);
    for (void *p : {nets, curves, coff, tab, counts})
        if (p) (void)hipFree(p);
}

gwn_status leafquad3d_moments(int device, const std::vector<double> &nets, const std::vector<Trim3> &curves,
                              const std::vector<int64_t> &coff, const std::vector<double> &box,
                              const double (*rule_x)[kMaxQuadRule], const double (*rule_w)[kMaxQuadRule],
                              const int *rule_n, LeafQuad3 &st, std::vector<double> &U, std::vector<double> &Wt,
                              std::vector<double> &WC, std::vector<double> &LC, std::vector<double> &LN,
                              std::vector<std::array<int, 3>> &counts, std::string &err)
{
    const int64_t nl = (int64_t)coff.size() - 1;
    st.device = device;
    st.nl = nl;
    if (nl <= 0) return GWN_OK;
    QuadTab tab;
    for (int r = 0; r < 4; ++r) {
        if (rule_n[r] < 1 || rule_n[r] > kMaxQuadRule) { err = "leaf quadrature: bad rule size"; return GWN_EINVAL; }
        tab.n[r] = rule_n[r];
        for (int i = 0; i < kMaxQuadRule; ++i) {
            tab.x[r][i] = i < rule_n[r] ? rule_x[r][i] : 0.0;
            tab.w[r][i] = i < rule_n[r] ? rule_w[r][i] : 0.0;
        }
    }
    struct Buf {
        void *p = nullptr;
        ~Buf() { if (p) (void)hipFree(p); }
    } dbox, dU, dWt, dWC, dLC, dLN;
    const size_t nb = (size_t)nl;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMalloc(&st.nets, nets.size() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&st.curves, std::max<size_t>(curves.size(), 1) * sizeof(Trim3));
    if (e == hipSuccess) e = hipMalloc(&st.coff, coff.size() * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc(&st.tab, sizeof(QuadTab));
    if (e == hipSuccess) e = hipMalloc(&dbox.p, box.size() * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&dU.p, nb * kMomU * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&dWt.p, nb * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&dWC.p, nb * 3 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&dLC.p, nb * 3 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&dLN.p, nb * 2 * kMpoleTermsTail * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&st.counts, nb * 3 * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemcpy(st.nets, nets.data(), nets.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess && !curves.empty())
        e = hipMemcpy(st.curves, curves.data(), curves.size() * sizeof(Trim3), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(st.coff, coff.data(), coff.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(st.tab, &tab, sizeof(QuadTab), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dbox.p, box.data(), box.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_leaf_moments3d, dim3((unsigned)nl), dim3(64), 0, 0, (int)nl, (const double *)st.nets,
                           (const Trim3 *)st.curves, (const int64_t *)st.coff, (const double *)dbox.p,
                           (const QuadTab *)st.tab, (double *)dU.p, (double *)dWt.p, (double *)dWC.p,
                           (double *)dLC.p, (double *)dLN.p, (int32_t *)st.counts);
        e = hipGetLastError();
    }
    std::vector<int32_t> cnt(nb * 3);
    U.resize(nb * kMomU);
    Wt.resize(nb);
    WC.resize(nb * 3);
    LC.resize(nb * 3);
    LN.resize(nb * 2 * kMpoleTermsTail);
    if (e == hipSuccess) e = hipMemcpy(U.data(), dU.p, U.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(Wt.data(), dWt.p, Wt.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(WC.data(), dWC.p, WC.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(LC.data(), dLC.p, LC.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(LN.data(), dLN.p, LN.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(cnt.data(), st.counts, cnt.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        err = std::string("device leaf quadrature: ") + hipGetErrorString(e);
        return GWN_EHIP;
    }
    counts.resize(nb);
    for (size_t l = 0; l < nb; ++l)
        for (int r = 0; r < 3; ++r) counts[l][r] = cnt[3 * l + r];
    return GWN_OK;
}

gwn_status leafquad3d_nodes(LeafQuad3 &st, const std::vector<int64_t> &qbase, int64_t total, void **out,
                            std::string &err)
{
    *out = nullptr;
    if (st.nl <= 0 || total <= 0) return GWN_OK;
    void *dq = nullptr, *dbase = nullptr;
    hipError_t e = hipSetDevice(st.device);
    if (e == hipSuccess) e = hipMalloc(&dbase, qbase.size() * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc(&dq, (size_t)total * sizeof(QNode3));
    if (e == hipSuccess) e = hipMemcpy(dbase, qbase.data(), qbase.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_leaf_nodes3d, dim3((unsigned)st.nl), dim3(64), 0, 0, (int)st.nl,
                           (const double *)st.nets, (const Trim3 *)st.curves, (const int64_t *)st.coff,
                           (const QuadTab *)st.tab, (const int64_t *)dbase, (const int32_t *)st.counts,
                           (QNode3 *)dq);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (dbase) (void)hipFree(dbase);
    if (e != hipSuccess) {
        if (dq) (void)hipFree(dq);
        err = std::string("device node sets: ") + hipGetErrorString(e);
        return GWN_EHIP;
    }
    *out = dq;
    return GWN_OK;
}

}  // namespace gwn
