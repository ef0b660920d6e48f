// Device construction of the radix tree of a model's leaves (Alg. 1
// ConstructBVH; Karras, HPG 2012): Morton codes of the leaf AABB centres,
// quantised in the model box exactly as the host build does, a stable radix
// sort of (code, leaf), then the two children of every internal node, each
// node independently.  The depth-first layout and the moment up-sweep stay
// on the host (tree.cpp), which receives the sorted leaf order and the child
// links and produces the same tree as a host-only build.
#include <hip/hip_runtime.h>
#include "radix.h"

#include <algorithm>
#include <string>
#include <vector>

#include "gwn_internal.h"

namespace gwn {

namespace {

constexpr int kLbvhBlock = 256;

__device__ uint64_t spread2_d(uint64_t x)
{
    x &= 0xffffffffull;
    x = (x | (x << 16)) & 0x0000ffff0000ffffull;
    x = (x | (x << 8)) & 0x00ff00ff00ff00ffull;
    x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

__device__ uint64_t spread3_d(uint64_t x)
{
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

struct Box {
    double lo[3], hi[3];
};

// Morton code of each leaf's AABB centre: t = (v - lo) / ext clamped to
// [0, 1], floor(t (2^bits - 1)); IEEE division, as on the host.
__global__ __launch_bounds__(kLbvhBlock) void k_leaf_codes(int dim, int n, const double *__restrict__ lo,
                                                           const double *__restrict__ hi, Box model,
                                                           uint64_t *__restrict__ keys, int32_t *__restrict__ idx)
{
    const int i = blockIdx.x * kLbvhBlock + threadIdx.x;
    if (i >= n) return;
    const int bits = dim == 2 ? 32 : 21;
    const double maxq = (double)((1ull << bits) - 1);
    uint64_t k = 0;
    for (int a = 0; a < dim; ++a) {
        const double cc = 0.5 * (lo[3 * i + a] + hi[3 * i + a]);
        const double ext = model.hi[a] - model.lo[a];
        double t = ext > 0 ? (cc - model.lo[a]) / ext : 0.5;
        t = fmin(fmax(t, 0.0), 1.0);
        const uint64_t q = (uint64_t)floor(t * maxq);
        k |= (dim == 2 ? spread2_d(q) : spread3_d(q)) << a;
    }
    keys[i] = k;
    idx[i] = i;
}

// Length of the common prefix of sorted positions i and j (-1 outside),
// equal codes disambiguated by position.
__device__ __forceinline__ int delta(const uint64_t *__restrict__ code, int n, int i, int j)
{
    if (j < 0 || j >= n) return -1;
    const uint64_t a = code[i], b = code[j];
    if (a == b) return i == j ? 128 : 64 + __clz((int)((unsigned)(i ^ j)));
    return __clzll((long long)(a ^ b));
}

// Children of internal node i: the range it covers grows from i in the
// direction of the longer common prefix; its split is the last position
// sharing more than the range's common prefix with i.  Encoding: >= 0
// internal node, < 0 leaf (-1 - sorted position).
__global__ __launch_bounds__(kLbvhBlock) void k_karras(const uint64_t *__restrict__ code, int n,
                                                       int32_t *__restrict__ cl, int32_t *__restrict__ cr)
{
    const int i = blockIdx.x * kLbvhBlock + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (delta(code, n, i, i + 1) - delta(code, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = delta(code, n, i, i - d);
    int lmax = 2;
    while (delta(code, n, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (delta(code, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = delta(code, n, i, j);
    int s = 0;
    for (int div = 2;; div *= 2) {
        const int t = (l + div - 1) / div;
        if (delta(code, n, i, i + (s + t) * d) > dnode) s += t;
        if (t <= 1) break;
    }
    const int gamma = i + s * d + min(d, 0);
    const int a = min(i, j), b = max(i, j);
    cl[i] = (a == gamma) ? -1 - gamma : gamma;
    cr[i] = (b == gamma + 1) ? -1 - (gamma + 1) : gamma + 1;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

bool lbvh_device(int device, int dim, int n, const double *lo, const double *hi, const double *model_lo,
                 const double *model_hi, std::vector<int> &order, std::vector<int> &cl, std::vector<int> &cr,
                 std::string &err)
{
    Box mb{};
    for (int a = 0; a < 3; ++a) { mb.lo[a] = model_lo[a]; mb.hi[a] = model_hi[a]; }
    const size_t nb = (size_t)n;
    DevBuf d_lo, d_hi, d_k0, d_k1, d_i0, d_i1, d_cl, d_cr, d_tmp;
    size_t tmp_bytes = 0;
    hipError_t e = hipSetDevice(device);
    tmp_bytes = radix_temp_bytes(n);
    if (e == hipSuccess) e = hipMalloc(&d_lo.p, 3 * nb * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&d_hi.p, 3 * nb * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&d_k0.p, nb * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc(&d_k1.p, nb * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc(&d_i0.p, nb * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&d_i1.p, nb * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&d_cl.p, std::max<size_t>(nb - 1, 1) * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&d_cr.p, std::max<size_t>(nb - 1, 1) * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&d_tmp.p, std::max<size_t>(tmp_bytes, 8));
    if (e == hipSuccess) e = hipMemcpy(d_lo.p, lo, 3 * nb * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_hi.p, hi, 3 * nb * sizeof(double), hipMemcpyHostToDevice);
    const dim3 grid((unsigned)((nb + kLbvhBlock - 1) / kLbvhBlock)), block(kLbvhBlock);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_leaf_codes, grid, block, 0, 0, dim, n, (const double *)d_lo.p, (const double *)d_hi.p,
                           mb, (uint64_t *)d_k0.p, (int32_t *)d_i0.p);
        e = hipGetLastError();
    }
    // LSD radix sort: stable, so equal codes keep leaf order, as the host's
    // stable sort does; the sorted pairs end up in buffer `sel`
    uint64_t *kb[2] = {(uint64_t *)d_k0.p, (uint64_t *)d_k1.p};
    int32_t *ib[2] = {(int32_t *)d_i0.p, (int32_t *)d_i1.p};
    int sel = 0;
    if (e == hipSuccess) e = radix_sort_pairs(kb, ib, n, 0, 64, d_tmp.p, 0, sel);
    if (e == hipSuccess && n > 1) {
        hipLaunchKernelGGL(k_karras, grid, block, 0, 0, (const uint64_t *)kb[sel], n, (int32_t *)d_cl.p,
                           (int32_t *)d_cr.p);
        e = hipGetLastError();
    }
    order.assign(nb, 0);
    cl.assign(nb > 1 ? nb - 1 : 0, 0);
    cr.assign(nb > 1 ? nb - 1 : 0, 0);
    if (e == hipSuccess) e = hipMemcpy(order.data(), ib[sel], nb * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && n > 1) e = hipMemcpy(cl.data(), d_cl.p, (nb - 1) * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && n > 1) e = hipMemcpy(cr.data(), d_cr.p, (nb - 1) * sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        err = std::string("device BVH: ") + hipGetErrorString(e);
        return false;
    }
    return true;
}

}  // namespace gwn
