// C ABI of the engine (declared in include/gwn.h): validation, parameter
// handling, packing of the host tree into device records and upload.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "gwn_internal.h"
#include "multipole3d.h"

using namespace gwn;

static thread_local std::string g_err;

static gwn_status fail(gwn_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

static gwn_status hip_fail(hipError_t e, const char *what)
{
    return fail(GWN_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct gwn_model {
    Model m;
    // device node sets of a build that never reached the upload
    ~gwn_model() { if (m.d_qnodes) (void)hipFree(m.d_qnodes); }
};

extern "C" void gwn_default_params(gwn_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->beta = 2.0;
    p->beta_mixed = 4.0;
    p->taylor_order = 2;
    p->precision = GWN_FP64;
    p->reclass_band = 1e-2;
    p->max_diag_frac = 0.10;
    p->eps_on = 1e-12;
    p->gl_nodes = 10;
    p->device = 0;
    p->near_ratio = 0.25;
    p->eps_q = 1e-6;
    p->leaf_far = 1;
    p->wave_accept = 0;
    p->far_tol = 0.0;
}

static gwn_status check_query_params(int dim, const gwn_params *p)
{
    if (!(p->beta > 0) || !std::isfinite(p->beta)) return fail(GWN_EINVAL, "beta must be finite and > 0");
    if (!(p->beta_mixed > 0) || !std::isfinite(p->beta_mixed))
        return fail(GWN_EINVAL, "beta_mixed must be finite and > 0");
    if (dim == 2 && (p->beta < 2.0 || p->beta_mixed < 2.0))
        return fail(GWN_EINVAL, "2D requires beta >= 2 (chord substitution needs q outside every accepted AABB)");
    if (p->taylor_order < 0 || p->taylor_order > (dim == 2 ? kMaxOrder2D : kMaxOrder3D))
        return fail(GWN_EINVAL, dim == 2 ? "taylor_order must be 0..16 in 2D" : "taylor_order must be 0..6 in 3D");
    if (p->precision != GWN_FP64 && p->precision != GWN_MIXED) return fail(GWN_EINVAL, "bad precision");
    if (!(p->reclass_band >= 0) || !std::isfinite(p->reclass_band)) return fail(GWN_EINVAL, "bad reclass_band");
    if (!(p->near_ratio >= 0) || !std::isfinite(p->near_ratio)) return fail(GWN_EINVAL, "bad near_ratio");
    if (!(p->eps_q > 0)) return fail(GWN_EINVAL, "eps_q must be > 0");
    if (p->leaf_far != 0 && p->leaf_far != 1) return fail(GWN_EINVAL, "leaf_far must be 0 or 1");
    if (p->wave_accept != 0 && p->wave_accept != 1) return fail(GWN_EINVAL, "wave_accept must be 0 or 1");
    if (!(p->far_tol >= 0) || !std::isfinite(p->far_tol)) return fail(GWN_EINVAL, "far_tol must be finite and >= 0");
    return GWN_OK;
}

static gwn_status check_build_params(int dim, const gwn_params *p)
{
    gwn_status s = check_query_params(dim, p);
    if (s) return s;
    if (!(p->max_diag_frac >= 0) || !std::isfinite(p->max_diag_frac)) return fail(GWN_EINVAL, "bad max_diag_frac");
    if (!(p->eps_on >= 0) || !std::isfinite(p->eps_on)) return fail(GWN_EINVAL, "bad eps_on");
    if (p->gl_nodes < 1 || p->gl_nodes > 32) return fail(GWN_EINVAL, "gl_nodes must be 1..32");
    return GWN_OK;
}

namespace gwn {

void refresh_dev_params(Model &m)
{
    const gwn_params &p = m.params;
    m.dev.dim = m.dim;
    m.dev.order = p.taylor_order;
    m.dev.precision = p.precision;
    // error-budgeted far test: the cluster radii carry their own factor
    m.dev.beta2 = p.far_tol > 0.0 ? 1.0 : p.beta * p.beta;
    m.dev.beta2_mixed = p.beta_mixed * p.beta_mixed;
    m.dev.band = p.reclass_band;
    for (int a = 0; a < 3; ++a) {
        m.dev.lo[a] = m.lo[a];
        double ext = m.hi[a] - m.lo[a];
        m.dev.inv_ext[a] = ext > 0 ? 1.0 / ext : 0.0;
    }
    m.dev.eps_on = p.eps_on * m.diag;
    m.dev.near_ratio2 = p.near_ratio * p.near_ratio;
    m.dev.leaf_far = p.leaf_far;
    m.dev.wave_accept = p.wave_accept;
    m.dev.eps_q = p.eps_q;
    m.dev.gl_n = p.gl_nodes;
}

static void pack2d(const Model &m, std::vector<Node2> &nodes, std::vector<Hot2> &hot, std::vector<Prim2> &prims)
{
    const auto &T = m.tree.nodes;
    nodes.assign(T.size(), Node2{});
    hot.assign(T.size(), Hot2{});
    // end of each node's DFS subtree: a leaf's is the next index, an
    // internal node's its right child's
    std::vector<int32_t> end(T.size());
    for (size_t i = T.size(); i-- > 0;) end[i] = T[i].is_leaf ? (int32_t)i + 1 : end[T[i].right];
    for (size_t i = 0; i < T.size(); ++i) {
        const HostNode &h = T[i];
        Node2 &n = nodes[i];
        std::memset(&n, 0, sizeof n);
        n.c[0] = h.c[0];
        n.c[1] = h.c[1];
        n.r2 = h.r * h.r;
        if (h.is_leaf) {
            n.m[0] = h.lo[0]; n.m[1] = h.lo[1]; n.m[2] = h.hi[0]; n.m[3] = h.hi[1];
            n.right = -1 - h.leaf;
            n.degree = m.leaf_degree[h.leaf];
        } else {
            // centred complex moments m_k = integral (z - c)^k dz (build2d),
            // stored as m_k / r^(k+1); r = 0 only for a cluster of points,
            // whose moments are all zero
            const double *cm = &m.cmom2[i * 2 * (kMaxOrder2D + 1)];
            for (int k = 0; k <= kMaxOrder2D; ++k) {
                double re = cm[2 * k], im = cm[2 * k + 1];
                for (int j = 0; j <= k && h.r > 0.0; ++j) { re /= h.r; im /= h.r; }
                n.m[2 * k] = h.r > 0.0 ? re : 0.0;
                n.m[2 * k + 1] = h.r > 0.0 ? im : 0.0;
            }
            n.right = h.right;
            n.degree = 0;
        }
        n.fc[0] = (float)n.c[0];
        n.fc[1] = (float)n.c[1];
        n.fr2 = (float)n.r2;
        for (int k = 0; k < 2 * kMaxOrder2D; ++k) n.fm[k] = (float)n.m[k];
        Hot2 &t = hot[i];
        std::memset(&t, 0, sizeof t);
        if (h.is_leaf) {
            const double *lh = &m.leaf_h[12 * (size_t)h.leaf];
            t.a[0] = lh[0] / lh[2]; t.a[1] = lh[1] / lh[2];
            t.a[2] = lh[9] / lh[11]; t.a[3] = lh[10] / lh[11];
            for (int k = 0; k < 2; ++k) {
                float lo = (float)h.lo[k], hi = (float)h.hi[k];
                if ((double)lo > h.lo[k]) lo = std::nextafter(lo, -INFINITY);
                if ((double)hi < h.hi[k]) hi = std::nextafter(hi, INFINITY);
                t.f[k] = lo;
                t.f[2 + k] = hi;
            }
        } else {
            t.a[0] = n.c[0]; t.a[1] = n.c[1]; t.a[2] = n.r2; t.a[3] = h.r;
            if (m.params.far_tol > 0.0 && h.r > 0.0) {
                // (beta_c r)^2, compared with ||q - c||^2 at beta2 = 1
                const double bc = far_beta2d(&m.tail2[i * kTailStride2D], m.params.taylor_order, m.params.far_tol);
                t.a[2] = std::isfinite(bc) ? (bc * h.r) * (bc * h.r) : HUGE_VAL;
            }
            t.f[0] = n.fc[0]; t.f[1] = n.fc[1]; t.f[2] = n.fr2; t.f[3] = (float)h.r;
        }
        t.right = n.right;
        t.degree = n.degree;
        t.escape = end[i];
    }
    prims.assign(m.leaf_src.size(), Prim2{});
    for (size_t l = 0; l < prims.size(); ++l)
        std::memcpy(prims[l].h, &m.leaf_h[12 * l], sizeof(double) * 12);
}

void pack3d(const Model &m, std::vector<Node3> &nodes, std::vector<Prim3> &prims);  // build3d.cpp

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Query launches take their scratch (sort keys, permutation, near-field
// pairs) from the device's default stream-ordered pool.  With the pool's
// default release threshold of zero, every synchronisation hands the freed
// scratch back to the driver and the next launch maps it again; keeping up
// to kPoolKeepBytes cached removes that from each call.  Set once per device.
constexpr uint64_t kPoolKeepBytes = 1ull << 30;

static void keep_pool_scratch(int device)
{
    static std::mutex mu;
    static std::vector<int> done;
    std::lock_guard<std::mutex> lock(mu);
    if (std::find(done.begin(), done.end(), device) != done.end()) return;
    done.push_back(device);
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, device) != hipSuccess || !pool) return;
    uint64_t keep = kPoolKeepBytes;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
}

gwn_status upload_model(Model &m, std::string &err)
{
    hipError_t e = hipSetDevice(m.device);
    if (e != hipSuccess) { err = std::string("hipSetDevice: ") + hipGetErrorString(e); return GWN_EHIP; }
    keep_pool_scratch(m.device);
    // Arena: nodes | prims | trims | qnodes | mpole | fmpole | hot, each
    // 256-byte aligned (trims to fmpole are 3D only, hot 2D only).
    std::vector<Node2> n2; std::vector<Prim2> p2; std::vector<Hot2> h2;
    std::vector<Node3> n3; std::vector<Prim3> p3;
    std::vector<float> fmp;
    const void *src[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    size_t bytes[7] = {0, 0, 0, 0, 0, 0, 0};
    if (m.dim == 2) {
        pack2d(m, n2, h2, p2);
        src[0] = n2.data(); bytes[0] = n2.size() * sizeof(Node2);
        src[1] = p2.data(); bytes[1] = p2.size() * sizeof(Prim2);
        src[6] = h2.data(); bytes[6] = h2.size() * sizeof(Hot2);
    } else {
        pack3d(m, n3, p3);
        src[0] = n3.data(); bytes[0] = n3.size() * sizeof(Node3);
        src[1] = p3.data(); bytes[1] = p3.size() * sizeof(Prim3);
        src[2] = m.trims.data(); bytes[2] = m.trims.size() * sizeof(Trim3);
        // node sets: host vector, or (device build) already in device memory
        src[3] = m.d_qnodes ? nullptr : m.qnodes.data();
        bytes[3] = (m.d_qnodes ? (size_t)m.n_qnodes_dev : m.qnodes.size()) * sizeof(QNode3);
        fmp.assign(m.mpole.begin(), m.mpole.end());
        src[4] = m.mpole.data(); bytes[4] = m.mpole.size() * sizeof(double);
        src[5] = fmp.data(); bytes[5] = fmp.size() * sizeof(float);
    }
    size_t off[8];
    off[0] = 0;
    for (int k = 0; k < 7; ++k) off[k + 1] = align_up(off[k] + bytes[k], 256);
    size_t total = std::max<size_t>(off[7], 256);
    void *arena = nullptr;
    auto drop_dev_qnodes = [&] {
        if (m.d_qnodes) (void)hipFree(m.d_qnodes);
        m.d_qnodes = nullptr;
    };
    e = hipMalloc(&arena, total);
    if (e != hipSuccess) {
        drop_dev_qnodes();
        err = std::string("hipMalloc arena: ") + hipGetErrorString(e);
        return GWN_ENOMEM;
    }
    for (int k = 0; k < 7; ++k)
        if (bytes[k]) {
            e = src[k] ? hipMemcpy((char *)arena + off[k], src[k], bytes[k], hipMemcpyHostToDevice)
                       : hipMemcpy((char *)arena + off[k], m.d_qnodes, bytes[k], hipMemcpyDeviceToDevice);
            if (e != hipSuccess) {
                (void)hipFree(arena);
                drop_dev_qnodes();
                err = std::string("hipMemcpy arena: ") + hipGetErrorString(e);
                return GWN_EHIP;
            }
        }
    drop_dev_qnodes();
    int32_t *flag = nullptr;
    e = hipMalloc((void **)&flag, 256);
    if (e == hipSuccess) e = hipMemset(flag, 0, 256);
    int32_t *hflag = nullptr;
    if (e == hipSuccess) e = hipHostMalloc((void **)&hflag, 256, hipHostMallocDefault);
    hipEvent_t ev = nullptr;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipFree(arena);
        if (flag) (void)hipFree(flag);
        if (hflag) (void)hipHostFree(hflag);
        err = std::string("device flag setup: ") + hipGetErrorString(e);
        return GWN_EHIP;
    }
    *hflag = 0;
    m.d_arena = arena;
    m.arena_bytes = (int64_t)total;
    m.d_flag = flag;
    m.h_flag = hflag;
    m.flag_event = ev;
    m.dev.nodes = (char *)arena + off[0];
    m.dev.prims = (char *)arena + off[1];
    m.dev.trims = (char *)arena + off[2];
    m.dev.qnodes = (char *)arena + off[3];
    m.dev.mpole = (char *)arena + off[4];
    m.dev.fmpole = (char *)arena + off[5];
    m.dev.hot = (char *)arena + off[6];
    m.dev.flag = flag;
    m.dev.n_nodes = (int32_t)m.tree.nodes.size();
    refresh_dev_params(m);
    return GWN_OK;
}

void release_device(Model &m)
{
    if (m.device < 0) return;
    (void)hipSetDevice(m.device);
    if (m.flag_event) (void)hipEventSynchronize((hipEvent_t)m.flag_event);
    (void)hipDeviceSynchronize();
    if (m.d_arena) (void)hipFree(m.d_arena);
    if (m.d_flag) (void)hipFree(m.d_flag);
    if (m.h_flag) (void)hipHostFree(m.h_flag);
    if (m.flag_event) (void)hipEventDestroy((hipEvent_t)m.flag_event);
    m.d_arena = nullptr;
    m.d_flag = nullptr;
    m.h_flag = nullptr;
    m.flag_event = nullptr;
}

}  // namespace gwn

template <class F>
static gwn_status build_common(int dim, const gwn_params *params, gwn_handle *out, F &&host_build)
{
    if (!out) return fail(GWN_EINVAL, "out handle pointer is NULL");
    *out = nullptr;
    gwn_params p;
    if (params) p = *params;
    else gwn_default_params(&p);
    gwn_status s = check_build_params(dim, &p);
    if (s) return s;
    gwn_model *h = new (std::nothrow) gwn_model();
    if (!h) return fail(GWN_ENOMEM, "host allocation failed");
    std::string err;
    try {
        s = host_build(p, h->m, err);
    } catch (const std::bad_alloc &) {
        s = GWN_ENOMEM;
        err = "host allocation failed during build";
    } catch (const std::exception &ex) {
        s = GWN_EINVAL;
        err = ex.what();
    }
    if (s) {
        delete h;
        return fail(s, err);
    }
    h->m.device = p.device;
    if (p.device >= 0) {
        int ndev = 0;
        hipError_t e = hipGetDeviceCount(&ndev);
        if (e != hipSuccess || p.device >= ndev) {
            delete h;
            return fail(GWN_EHIP, std::string("no HIP device ") + std::to_string(p.device) +
                                      (e != hipSuccess ? std::string(": ") + hipGetErrorString(e) : std::string()));
        }
        s = upload_model(h->m, err);
        if (s) {
            h->m.device = -1;
            delete h;
            return fail(s, err);
        }
    } else {
        refresh_dev_params(h->m);
    }
    *out = h;
    return GWN_OK;
}

extern "C" gwn_status gwn_build2d(const gwn_curves2d *curves, const gwn_params *params, gwn_handle *out)
{
    if (!curves) return fail(GWN_EINVAL, "curves is NULL");
    return build_common(2, params, out, [&](const gwn_params &p, Model &m, std::string &err) {
        return build2d_host(curves, &p, m, err);
    });
}

extern "C" gwn_status gwn_nurbs2d_extract(const gwn_nurbs2d *in, int64_t *n_segments, int64_t *n_points,
                                          int32_t *degree, int64_t *cp_offset, double *cp_xy, double *cp_w)
{
    if (!in || !n_segments || !n_points) return fail(GWN_EINVAL, "NULL input or count pointer");
    std::vector<int32_t> deg;
    std::vector<int64_t> off;
    std::vector<double> xy, w;
    std::string err;
    try {
        if (!extract_nurbs2d(*in, deg, off, xy, w, err)) return fail(GWN_EINVAL, err);
    } catch (const std::bad_alloc &) {
        return fail(GWN_ENOMEM, "host allocation failed during NURBS extraction");
    }
    const int64_t ns = (int64_t)deg.size(), np = (int64_t)w.size();
    if (!degree) {
        *n_segments = ns;
        *n_points = np;
        return GWN_OK;
    }
    if (!cp_offset || !cp_xy || !cp_w) return fail(GWN_EINVAL, "NULL output array");
    if (*n_segments < ns || *n_points < np)
        return fail(GWN_EINVAL, "output capacity too small: need " + std::to_string(ns) + " segments and " +
                                    std::to_string(np) + " points");
    std::copy(deg.begin(), deg.end(), degree);
    std::copy(off.begin(), off.end(), cp_offset);
    std::copy(xy.begin(), xy.end(), cp_xy);
    std::copy(w.begin(), w.end(), cp_w);
    *n_segments = ns;
    *n_points = np;
    return GWN_OK;
}

extern "C" gwn_status gwn_nurbs3d_extract(const gwn_nurbs3d *in, int64_t *n_patches, int64_t *n_trims,
                                          int64_t *n_trim_cp, double *cp_xyz, double *cp_w, int64_t *trim_offset,
                                          int32_t *trim_degree, int64_t *trim_cp_offset, double *trim_cp_uv,
                                          double *trim_cp_w)
{
    if (!in || !n_patches || !n_trims || !n_trim_cp) return fail(GWN_EINVAL, "NULL input or count pointer");
    NurbsPatches x;
    std::string err;
    try {
        if (!extract_nurbs3d(*in, x, err)) return fail(GWN_EINVAL, err);
    } catch (const std::bad_alloc &) {
        return fail(GWN_ENOMEM, "host allocation failed during NURBS extraction");
    }
    const int64_t np = (int64_t)x.cp_w.size() / 16, nt = (int64_t)x.trim_degree.size(),
                  nc = (int64_t)x.trim_cp_w.size();
    if (!cp_xyz) {
        *n_patches = np;
        *n_trims = nt;
        *n_trim_cp = nc;
        return GWN_OK;
    }
    if (!cp_w || !trim_offset || (nt > 0 && (!trim_degree || !trim_cp_offset || !trim_cp_uv || !trim_cp_w)))
        return fail(GWN_EINVAL, "NULL output array");
    if (*n_patches < np || *n_trims < nt || *n_trim_cp < nc)
        return fail(GWN_EINVAL, "output capacity too small: need " + std::to_string(np) + " patches, " +
                                    std::to_string(nt) + " trim curves and " + std::to_string(nc) + " trim points");
    std::copy(x.cp_xyz.begin(), x.cp_xyz.end(), cp_xyz);
    std::copy(x.cp_w.begin(), x.cp_w.end(), cp_w);
    std::copy(x.trim_offset.begin(), x.trim_offset.end(), trim_offset);
    if (nt > 0) {
        std::copy(x.trim_degree.begin(), x.trim_degree.end(), trim_degree);
        std::copy(x.trim_cp_offset.begin(), x.trim_cp_offset.end(), trim_cp_offset);
        std::copy(x.trim_cp_uv.begin(), x.trim_cp_uv.end(), trim_cp_uv);
        std::copy(x.trim_cp_w.begin(), x.trim_cp_w.end(), trim_cp_w);
    } else if (trim_cp_offset) {
        trim_cp_offset[0] = 0;
    }
    *n_patches = np;
    *n_trims = nt;
    *n_trim_cp = nc;
    return GWN_OK;
}

extern "C" gwn_status gwn_build3d(const gwn_patches3d *patches, const gwn_params *params, gwn_handle *out)
{
    if (!patches) return fail(GWN_EINVAL, "patches is NULL");
    return build_common(3, params, out, [&](const gwn_params &p, Model &m, std::string &err) {
        return build3d_host(patches, &p, m, err);
    });
}

extern "C" gwn_status gwn_set_params(gwn_handle h, const gwn_params *params)
{
    if (!h || !params) return fail(GWN_EINVAL, "NULL handle or params");
    gwn_params p = h->m.params;
    p.beta = params->beta;
    p.beta_mixed = params->beta_mixed;
    p.taylor_order = params->taylor_order;
    p.precision = params->precision;
    p.reclass_band = params->reclass_band;
    p.near_ratio = params->near_ratio;
    p.leaf_far = params->leaf_far;
    p.eps_q = params->eps_q;
    p.far_tol = params->far_tol;
    p.wave_accept = params->wave_accept;
    gwn_status s = check_query_params(h->m.dim, &p);
    if (s) return s;
    const gwn_params old = h->m.params;
    h->m.params = p;
    const bool radii = p.far_tol != old.far_tol || (p.far_tol > 0.0 && p.taylor_order != old.taylor_order);
    if (radii && h->m.d_arena) {
        // the far radii live in the node records: rewrite them once no
        // launch can still read them
        std::vector<Node2> n2; std::vector<Hot2> h2; std::vector<Prim2> p2;
        std::vector<Node3> n3; std::vector<Prim3> p3;
        const void *src;
        void *dst;
        size_t bytes;
        if (h->m.dim == 2) {
            pack2d(h->m, n2, h2, p2);
            src = h2.data(); dst = (void *)h->m.dev.hot; bytes = h2.size() * sizeof(Hot2);
        } else {
            pack3d(h->m, n3, p3);
            src = n3.data(); dst = (void *)h->m.dev.nodes; bytes = n3.size() * sizeof(Node3);
        }
        hipError_t e = hipSetDevice(h->m.device);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e == hipSuccess) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            h->m.params = old;
            return fail(GWN_EHIP, std::string("far radii update: ") + hipGetErrorString(e));
        }
    }
    refresh_dev_params(h->m);
    return GWN_OK;
}

extern "C" gwn_status gwn_get_params(gwn_handle h, gwn_params *out)
{
    if (!h || !out) return fail(GWN_EINVAL, "NULL handle or output");
    *out = h->m.params;
    return GWN_OK;
}

static gwn_status check_flag(Model &m)
{
    // The device keeps a monotonic count of the queries that hit a limit;
    // each launch copies it back.  Once the latest copy has landed, a count
    // above the one already reported is reported once.  The count is never
    // reset, so a copy that lands later can only carry a larger value and
    // no overflow is lost or reported twice.
    if (!m.flag_event || !m.h_flag) return GWN_OK;
    if (hipEventQuery((hipEvent_t)m.flag_event) != hipSuccess) return GWN_OK;
    const uint32_t now = (uint32_t)*m.h_flag;
    if (now != m.flag_seen) {
        const uint32_t fresh = now - m.flag_seen;
        m.flag_seen = now;
        return fail(GWN_EOVERFLOW, std::to_string(fresh) + " query(ies) of an earlier call hit a traversal or "
                                   "near-field limit (their outputs are NaN)");
    }
    return GWN_OK;
}

static gwn_status after_launch(Model &m, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(m.h_flag, m.d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord((hipEvent_t)m.flag_event, s);
    if (e != hipSuccess) return hip_fail(e, "flag readback");
    return GWN_OK;
}

static gwn_status query_common(gwn_handle h, const double *points, int64_t n, double *out_gwn,
                               uint8_t *out_inside, void *stream, bool fixed_scratch)
{
    if (!h) return fail(GWN_EINVAL, "NULL handle");
    if (n < 0) return fail(GWN_EINVAL, "n < 0");
    if (h->m.device < 0) return fail(GWN_EINVAL, "host-only handle cannot be queried");
    if (n > 0 && (!points || !out_gwn)) return fail(GWN_EINVAL, "NULL points or output");
    if (n > ((int64_t)1 << 31) - 1024) return fail(GWN_EINVAL, "n too large for one call");
    gwn_status s = check_flag(h->m);
    if (s) return s;
    if (n == 0) return GWN_OK;
    hipError_t e = hipSetDevice(h->m.device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    std::string err;
    ExtScratch ext;
    if (fixed_scratch) {
        s = noalloc_scratch(ext, err);
        if (s) return fail(s, err);
        int64_t need = 0;
        s = query_scratch_bytes(h->m.dim, n, 1, need, err);
        if (s) return fail(s, err);
        if ((size_t)need > ext.bytes)
            return fail(GWN_EINVAL, std::to_string(n) + " queries need " + std::to_string(need) +
                                        " bytes of scratch, above the fixed " + std::to_string(ext.bytes) +
                                        " (GWN_NOALLOC_SCRATCH_BYTES); split the call");
    }
    std::vector<Segment> segs{{&h->m, 0, n}};
    s = launch_queries(segs, h->m.dim, points, out_gwn, out_inside, nullptr, stream, err, ext);
    if (s) return fail(s, err);
    return after_launch(h->m, stream);
}

extern "C" gwn_status gwn_query(gwn_handle h, const double *points, int64_t n, double *out_gwn,
                                uint8_t *out_inside, void *stream)
{
    return query_common(h, points, n, out_gwn, out_inside, stream, false);
}

extern "C" gwn_status gwn_query_noalloc(gwn_handle h, const double *points, int64_t n, double *out_gwn,
                                        uint8_t *out_inside, void *stream)
{
    return query_common(h, points, n, out_gwn, out_inside, stream, true);
}

extern "C" gwn_status gwn_query_scratch_bytes(gwn_handle h, int64_t n, int32_t n_seg, int64_t *bytes)
{
    if (!h || !bytes) return fail(GWN_EINVAL, "NULL handle or output");
    if (n < 0 || n_seg < 0) return fail(GWN_EINVAL, "n and n_seg must be >= 0");
    std::string err;
    gwn_status s = query_scratch_bytes(h->m.dim, n, n_seg, *bytes, err);
    return s ? fail(s, err) : GWN_OK;
}

extern "C" gwn_status gwn_query_counters(gwn_handle h, const double *points, int64_t n, int64_t *counters,
                                         void *stream)
{
    if (!h || !counters) return fail(GWN_EINVAL, "NULL handle or counters");
    if (n < 0) return fail(GWN_EINVAL, "n < 0");
    if (h->m.device < 0) return fail(GWN_EINVAL, "host-only handle cannot be queried");
    if (n > 0 && !points) return fail(GWN_EINVAL, "NULL points");
    hipError_t e = hipSetDevice(h->m.device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = hipMemsetAsync(counters, 0, sizeof(int64_t) * GWN_NCOUNTERS, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "counter reset");
    if (n == 0) return GWN_OK;
    std::vector<Segment> segs{{&h->m, 0, n}};
    std::string err;
    gwn_status s = launch_queries(segs, h->m.dim, points, nullptr, nullptr, counters, stream, err);
    if (s) return fail(s, err);
    return GWN_OK;
}

extern "C" gwn_status gwn_query_batch(int32_t n_seg, const gwn_handle *seg_model, const int64_t *seg_offset,
                                      const double *points, double *out_gwn, uint8_t *out_inside, void *stream)
{
    if (n_seg < 0) return fail(GWN_EINVAL, "n_seg < 0");
    if (n_seg == 0) return GWN_OK;
    if (!seg_model || !seg_offset) return fail(GWN_EINVAL, "NULL segment arrays");
    if (seg_offset[0] != 0) return fail(GWN_EINVAL, "seg_offset[0] must be 0");
    int dim = 0, device = -1;
    std::vector<Segment> segs;
    segs.reserve(n_seg);
    for (int32_t s = 0; s < n_seg; ++s) {
        gwn_handle h = seg_model[s];
        if (!h) return fail(GWN_EINVAL, "NULL model in segment " + std::to_string(s));
        if (h->m.device < 0) return fail(GWN_EINVAL, "host-only handle in segment " + std::to_string(s));
        if (seg_offset[s + 1] < seg_offset[s]) return fail(GWN_EINVAL, "seg_offset must be non-decreasing");
        if (dim == 0) { dim = h->m.dim; device = h->m.device; }
        if (h->m.dim != dim) return fail(GWN_EINVAL, "2D and 3D models cannot share one batch");
        if (h->m.device != device) return fail(GWN_EINVAL, "all models of a batch must live on one device");
        gwn_status st = check_flag(h->m);
        if (st) return st;
        segs.push_back({&h->m, seg_offset[s], seg_offset[s + 1]});
    }
    int64_t n = seg_offset[n_seg];
    if (n > ((int64_t)1 << 31) - 1024) return fail(GWN_EINVAL, "batch too large for one call");
    if (n == 0) return GWN_OK;
    if (!points || !out_gwn) return fail(GWN_EINVAL, "NULL points or output");
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    std::string err;
    gwn_status s = launch_queries(segs, dim, points, out_gwn, out_inside, nullptr, stream, err);
    if (s) return fail(s, err);
    for (int32_t k = 0; k < n_seg; ++k) {
        bool seen = false;
        for (int32_t j = 0; j < k; ++j) seen |= seg_model[j] == seg_model[k];
        if (!seen) {
            s = after_launch(seg_model[k]->m, stream);
            if (s) return s;
        }
    }
    return GWN_OK;
}

extern "C" gwn_status gwn_model_bytes(gwn_handle h, int64_t *resident, int64_t *per_query)
{
    if (!h) return fail(GWN_EINVAL, "NULL handle");
    if (resident) *resident = h->m.arena_bytes + 256;
    // keys x2, permutation x2, sort temp; 3D adds the near-field pass:
    // partial sum, count, 64 leaf slots, reclassify flag.  Per query at 64
    // queries per wave; launches under 2^18 queries take more per query
    // (gwn_query_scratch_bytes gives the exact figure of a launch).
    if (per_query) *per_query = 8 + 8 + 4 + 4 + 16 + (h->m.dim == 3 ? 8 + 4 + 4 * 64 + 1 : 0);
    return GWN_OK;
}

extern "C" gwn_status gwn_inspect(gwn_handle h, int32_t what, double *out, int64_t capacity, int64_t *count)
{
    if (!h) return fail(GWN_EINVAL, "NULL handle");
    const Model &m = h->m;
    const int d = m.dim, nm = n_moments(d);
    std::vector<double> buf;
    int64_t items = 0, width = 0;
    switch (what) {
    case GWN_I_SUMMARY:
        buf = {(double)d, (double)m.n_input, (double)m.leaf_src.size(), (double)m.tree.nodes.size(),
               (double)m.tree.depth, m.diag, m.lo[0], m.hi[0]};
        items = 1; width = 8;
        break;
    case GWN_I_LEAVES: {
        width = (d == 2) ? 13 : 65;
        items = (int64_t)m.leaf_src.size();
        buf.resize(items * width);
        for (int64_t l = 0; l < items; ++l) {
            buf[l * width] = (double)m.leaf_src[l];
            std::memcpy(&buf[l * width + 1], &m.leaf_h[l * (width - 1)], sizeof(double) * (width - 1));
        }
        break;
    }
    case GWN_I_NODES: {
        width = 13;
        items = (int64_t)m.tree.nodes.size();
        buf.resize(items * width);
        for (int64_t i = 0; i < items; ++i) {
            const HostNode &n = m.tree.nodes[i];
            double *b = &buf[i * width];
            b[0] = n.is_leaf; b[1] = n.is_leaf ? n.leaf : n.left; b[2] = n.right;
            for (int a = 0; a < 3; ++a) { b[3 + a] = n.c[a]; b[7 + a] = n.lo[a]; b[10 + a] = n.hi[a]; }
            b[6] = n.r;
        }
        break;
    }
    case GWN_I_COMPLEX: {
        if (d != 2) return fail(GWN_EINVAL, "complex moments exist for 2D models only");
        width = 2 * (kMaxOrder2D + 1);
        items = (int64_t)m.tree.nodes.size();
        buf.assign(m.cmom2.begin(), m.cmom2.end());
        break;
    }
    case GWN_I_FARBETA: {
        width = 1;
        items = (int64_t)m.tree.nodes.size();
        buf.assign(items, 0.0);
        for (int64_t i = 0; i < items; ++i) {
            const HostNode &n = m.tree.nodes[i];
            // 2D leaves are never far-tested; 3D leaves are with leaf_far
            if (n.is_leaf && d == 2) continue;
            if (!(m.params.far_tol > 0.0 && n.r > 0.0)) buf[i] = m.params.beta;
            else if (d == 2) buf[i] = far_beta2d(&m.tail2[i * kTailStride2D], m.params.taylor_order, m.params.far_tol);
            else buf[i] = far_beta3d(&m.tail3[i * kMaxLTail3], n.r, m.params.taylor_order, m.params.far_tol);
        }
        break;
    }
    case GWN_I_LEAF_TRIMS: {
        if (d != 3) return fail(GWN_EINVAL, "trim curves exist for 3D models only");
        width = 10;
        items = (int64_t)m.trims.size();
        buf.resize(items * width);
        int64_t k = 0;
        for (size_t l = 0; l < m.leaf_trim_begin.size(); ++l)
            for (int32_t j = 0; j < m.leaf_trim_count[l]; ++j, ++k) {
                buf[k * width] = (double)l;
                std::memcpy(&buf[k * width + 1], m.trims[m.leaf_trim_begin[l] + j].h, sizeof(double) * 9);
            }
        break;
    }
    case GWN_I_MULTIPOLE: {
        if (d != 3) return fail(GWN_EINVAL, "multipole moments exist for 3D models only");
        width = kMpoleStride;
        items = (int64_t)m.tree.nodes.size();
        buf.assign(m.mpole.begin(), m.mpole.end());
        break;
    }
    case GWN_I_MOMENTS:
    case GWN_I_UNCENTERED: {
        width = nm;
        items = (int64_t)m.tree.nodes.size();
        buf.resize(items * width);
        for (int64_t i = 0; i < items; ++i) {
            const auto &v = (what == GWN_I_MOMENTS) ? m.tree.nodes[i].M : m.tree.nodes[i].U;
            std::memcpy(&buf[i * width], v.data(), sizeof(double) * nm);
        }
        break;
    }
    default:
        return fail(GWN_EINVAL, "unknown inspection kind");
    }
    if (count) *count = items;
    if (out && capacity > 0) {
        int64_t nitems = std::min(capacity, items);
        std::memcpy(out, buf.data(), sizeof(double) * nitems * width);
    }
    return GWN_OK;
}

extern "C" gwn_status gwn_free(gwn_handle h)
{
    if (!h) return GWN_OK;
    release_device(h->m);
    delete h;
    return GWN_OK;
}

namespace gwn {
gwn_status profile_control(int enable, double *total_ms, int64_t *launches);
}

extern "C" gwn_status gwn_profile(int32_t enable, double *total_ms, int64_t *launches)
{
    return profile_control(enable, total_ms, launches);
}

extern "C" gwn_status gwn_profile_kernel(int32_t kernel, double *ms, int64_t *launches)
{
    if (profile_kernel(kernel, ms, launches)) return fail(GWN_EINVAL, "kernel must be GWN_K_QUERY2D, GWN_K_TRAV3D or GWN_K_NEAR3D");
    return GWN_OK;
}

extern "C" const char *gwn_last_error(void) { return g_err.c_str(); }
