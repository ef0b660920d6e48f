// Host construction of the BVH over leaves and of its per-node moment data
// (Alg. 1: ConstructBVH, SumUncenteredMomentsUpTree, CenterMomentsInPlace).
//
// The hierarchy is the binary radix tree of Karras (HPG 2012) over Morton
// codes of the leaf AABB centres, quantised in the model bounding box (2D:
// 32 bits per axis, 3D: 21 bits per axis).  Equal codes are disambiguated by
// leaf index, as in that paper.  The tree is then laid out depth first
// (left child = parent + 1), which is the order the traversal kernels use.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "gwn_internal.h"

namespace gwn {

static uint64_t spread2(uint64_t x)  // 32 bits -> even bit positions of 64
{
    x &= 0xffffffffull;
    x = (x | (x << 16)) & 0x0000ffff0000ffffull;
    x = (x | (x << 8)) & 0x00ff00ff00ff00ffull;
    x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

static uint64_t spread3(uint64_t x)  // 21 bits -> every third bit of 63
{
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

static uint64_t quant(double v, double lo, double hi, int bits)
{
    double ext = hi - lo;
    double t = ext > 0 ? (v - lo) / ext : 0.5;
    t = std::min(std::max(t, 0.0), 1.0);
    double maxq = std::ldexp(1.0, bits) - 1.0;
    return (uint64_t)std::floor(t * maxq);
}

namespace {
struct Karras {
    const std::vector<uint64_t> &code;
    int n;
    int delta(int i, int j) const
    {
        if (j < 0 || j >= n) return -1;
        uint64_t a = code[i], b = code[j];
        if (a == b) return i == j ? 128 : 64 + __builtin_clz((unsigned)(i ^ j));
        return __builtin_clzll(a ^ b);
    }
};
}  // namespace

bool build_tree(int dim, int n, const double *lo, const double *hi, const double *leafU,
                const double *leafW, const double *leafWC, const double *model_lo,
                const double *model_hi, HostTree &tree, std::string &err, int device)
{
    tree.dim = dim;
    tree.nodes.clear();
    tree.depth = 0;
    const int nm = n_moments(dim);
    if (n <= 0) return true;

    std::vector<int> order(n);
    std::vector<int> cl(std::max(n - 1, 0)), cr(std::max(n - 1, 0));
    if (device >= 0 && n > 1) {
        // same codes, order and links, computed on the device (lbvh.hip)
        if (!lbvh_device(device, dim, n, lo, hi, model_lo, model_hi, order, cl, cr, err)) return false;
    } else {
        // Morton codes of leaf AABB centres, sorted (stable on leaf index).
        std::vector<uint64_t> key(n);
        for (int i = 0; i < n; ++i) {
            uint64_t k = 0;
            for (int a = 0; a < dim; ++a) {
                double cc = 0.5 * (lo[3 * i + a] + hi[3 * i + a]);
                uint64_t qv = quant(cc, model_lo[a], model_hi[a], dim == 2 ? 32 : 21);
                k |= (dim == 2 ? spread2(qv) : spread3(qv)) << a;
            }
            key[i] = k;
        }
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
        std::vector<uint64_t> code(n);
        for (int i = 0; i < n; ++i) code[i] = key[order[i]];

        // Karras: internal node i covers a key range and splits it at gamma.
        // Children encoding: >= 0 internal index, < 0 leaf (-1 - sorted position).
        Karras K{code, n};
        for (int i = 0; i < n - 1; ++i) {
            int d = (K.delta(i, i + 1) - K.delta(i, i - 1)) >= 0 ? 1 : -1;
            int dmin = K.delta(i, i - d);
            int lmax = 2;
            while (K.delta(i, i + lmax * d) > dmin) lmax *= 2;
            int l = 0;
            for (int t = lmax / 2; t >= 1; t /= 2)
                if (K.delta(i, i + (l + t) * d) > dmin) l += t;
            int j = i + l * d;
            int dnode = K.delta(i, j);
            int s = 0;
            for (int div = 2;; div *= 2) {
                int t = (l + div - 1) / div;
                if (K.delta(i, i + (s + t) * d) > dnode) s += t;
                if (t <= 1) break;
            }
            int gamma = i + s * d + std::min(d, 0);
            int a = std::min(i, j), b = std::max(i, j);
            cl[i] = (a == gamma) ? -1 - gamma : gamma;
            cr[i] = (b == gamma + 1) ? -1 - (gamma + 1) : gamma + 1;
        }
    }

    // Depth-first pre-order layout.
    tree.nodes.reserve(2 * n - 1);
    struct Item { int code; int parent; int side; int depth; };
    std::vector<Item> st;
    st.push_back({n == 1 ? -1 : 0, -1, 0, 1});
    while (!st.empty()) {
        Item it = st.back();
        st.pop_back();
        int idx = (int)tree.nodes.size();
        tree.nodes.emplace_back();
        HostNode &nd = tree.nodes.back();
        nd.U.assign(nm, 0.0);
        nd.M.assign(nm, 0.0);
        tree.depth = std::max(tree.depth, it.depth);
        if (it.parent >= 0) {
            if (it.side == 0) tree.nodes[it.parent].left = idx;
            else tree.nodes[it.parent].right = idx;
        }
        if (it.code < 0) {
            nd.is_leaf = 1;
            nd.leaf = order[-1 - it.code];
        } else {
            // push right first so the left subtree is laid out next
            st.push_back({cr[it.code], idx, 1, it.depth + 1});
            st.push_back({cl[it.code], idx, 0, it.depth + 1});
        }
    }
    if ((int)tree.nodes.size() != 2 * n - 1) {
        err = "internal error: BVH node count mismatch";
        return false;
    }

    // Bottom-up: leaves take their data, internal nodes sum their children
    // (reverse pre-order visits children before parents).
    for (int k = (int)tree.nodes.size() - 1; k >= 0; --k) {
        HostNode &nd = tree.nodes[k];
        if (nd.is_leaf) {
            int l = nd.leaf;
            for (int a = 0; a < 3; ++a) { nd.lo[a] = lo[3 * l + a]; nd.hi[a] = hi[3 * l + a]; }
            for (int t = 0; t < nm; ++t) nd.U[t] = leafU[(size_t)l * nm + t];
            nd.wsum = leafW[l];
            for (int a = 0; a < 3; ++a) nd.wc[a] = leafWC[3 * l + a];
        } else {
            const HostNode &L = tree.nodes[nd.left], &R = tree.nodes[nd.right];
            for (int a = 0; a < 3; ++a) {
                nd.lo[a] = std::min(L.lo[a], R.lo[a]);
                nd.hi[a] = std::max(L.hi[a], R.hi[a]);
                nd.wc[a] = L.wc[a] + R.wc[a];
            }
            for (int t = 0; t < nm; ++t) nd.U[t] = L.U[t] + R.U[t];
            nd.wsum = L.wsum + R.wsum;
        }
        // centroid: weighted mean of the constituents; AABB centre if the
        // weight vanishes.  Radius: AABB half diagonal.
        double r2 = 0;
        for (int a = 0; a < dim; ++a) {
            double mid = 0.5 * (nd.lo[a] + nd.hi[a]);
            double cval = nd.wsum > 0 ? nd.wc[a] / nd.wsum : mid;
            if (!(cval >= nd.lo[a] && cval <= nd.hi[a])) cval = mid;
            nd.c[a] = cval;
            double h = 0.5 * (nd.hi[a] - nd.lo[a]);
            r2 += h * h;
        }
        nd.r = std::sqrt(r2);
        // Centre in place (Eq. moment_transform and its order-2 analogue):
        //   M1_jk  = U1_jk - c_j U0_k
        //   M2_ijk = U2_ijk - c_i U1_jk - c_j U1_ik + c_i c_j U0_k
        const int d = dim;
        const double *U0 = nd.U.data(), *U1 = U0 + d, *U2 = U1 + d * d;
        double *M0 = nd.M.data(), *M1 = M0 + d, *M2 = M1 + d * d;
        for (int k2 = 0; k2 < d; ++k2) M0[k2] = U0[k2];
        for (int j = 0; j < d; ++j)
            for (int k2 = 0; k2 < d; ++k2) M1[j * d + k2] = U1[j * d + k2] - nd.c[j] * U0[k2];
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                for (int k2 = 0; k2 < d; ++k2)
                    M2[(i * d + j) * d + k2] = U2[(i * d + j) * d + k2] - nd.c[i] * U1[j * d + k2] -
                                               nd.c[j] * U1[i * d + k2] + nd.c[i] * nd.c[j] * U0[k2];
    }
    return true;
}

}  // namespace gwn
