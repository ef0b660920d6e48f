// The engine's host-side builders under AddressSanitizer and UBSan (test
// infrastructure, compiled and run by tests/test_sanitize_host.py with g++
// and no GPU).  Reads a case file of 2D curves, 2D NURBS, 3D patches, query
// points (skipped here) and 3D NURBS surfaces
// (arrays in a fixed order, each an int64 element count followed by the raw
// little-endian values), then builds host-only models from them at several
// subdivision thresholds, and prints one summary line per build.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gwn_internal.h"

namespace gwn {
// The device hooks are not part of this build; host-only handles never call
// them.
gwn_status moments2d_device(int, const std::vector<HostNode> &, const std::vector<int> &,
                            const std::vector<double> &, std::vector<double> &, std::vector<double> &,
                            std::string &err)
{
    err = "no device in the host build";
    return GWN_EUNSUPPORTED;
}
bool lbvh_device(int, int, int, const double *, const double *, const double *, const double *, std::vector<int> &,
                 std::vector<int> &, std::vector<int> &, std::string &err)
{
    err = "no device in the host build";
    return false;
}
gwn_status subdiv2d_device(int, const std::vector<double> &, double, std::vector<double> &, std::vector<int32_t> &,
                           std::string &err)
{
    err = "no device in the host build";
    return GWN_EUNSUPPORTED;
}
LeafQuad3::~LeafQuad3() {}
gwn_status leafquad3d_moments(int, const std::vector<double> &, const std::vector<Trim3> &,
                              const std::vector<int64_t> &, const std::vector<double> &,
                              const double (*)[kMaxQuadRule], const double (*)[kMaxQuadRule], const int *,
                              LeafQuad3 &, std::vector<double> &, std::vector<double> &, std::vector<double> &,
                              std::vector<double> &, std::vector<double> &, std::vector<std::array<int, 3>> &,
                              std::string &err)
{
    err = "no device in the host build";
    return GWN_EUNSUPPORTED;
}
gwn_status leafquad3d_nodes(LeafQuad3 &, const std::vector<int64_t> &, int64_t, void **, std::string &err)
{
    err = "no device in the host build";
    return GWN_EUNSUPPORTED;
}
}  // namespace gwn

using namespace gwn;

namespace {

struct Reader {
    FILE *f;
    template <class T>
    std::vector<T> next()
    {
        int64_t n = 0;
        if (std::fread(&n, sizeof n, 1, f) != 1 || n < 0) throw std::string("truncated case file");
        std::vector<T> v((size_t)n);
        if (n && std::fread(v.data(), sizeof(T), (size_t)n, f) != (size_t)n) throw std::string("truncated case file");
        return v;
    }
};

gwn_params params(double frac, double far_tol)
{
    gwn_params p;
    std::memset(&p, 0, sizeof p);
    p.beta = 2.0;
    p.beta_mixed = 4.0;
    p.taylor_order = far_tol > 0 ? 12 : 2;
    p.precision = GWN_FP64;
    p.reclass_band = 1e-2;
    p.max_diag_frac = frac;
    p.eps_on = 1e-12;
    p.gl_nodes = 10;
    p.device = -1;
    p.near_ratio = 0.25;
    p.eps_q = 1e-8;
    p.leaf_far = 1;
    p.far_tol = far_tol;
    return p;
}

}  // namespace

int main(int argc, char **argv)
{
    if (argc != 2) {
        std::fprintf(stderr, "usage: %s case-file\n", argv[0]);
        return 2;
    }
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) {
        std::perror(argv[1]);
        return 2;
    }
    try {
        Reader r{f};
        // 2D curves
        auto deg = r.next<int32_t>();
        auto off = r.next<int64_t>();
        auto xy = r.next<double>();
        auto w = r.next<double>();
        // 2D NURBS
        auto ndeg = r.next<int32_t>();
        auto noff = r.next<int64_t>();
        auto nxy = r.next<double>();
        auto nw = r.next<double>();
        auto nkoff = r.next<int64_t>();
        auto nk = r.next<double>();
        // 3D patches
        auto cp = r.next<double>();
        auto cw = r.next<double>();
        auto toff = r.next<int64_t>();
        auto tdeg = r.next<int32_t>();
        auto tcoff = r.next<int64_t>();
        auto tuv = r.next<double>();
        auto tw = r.next<double>();
        (void)r.next<double>();   // 2D and 3D query points: the oracle driver's
        (void)r.next<double>();
        // 3D NURBS surfaces
        auto sdu = r.next<int32_t>();
        auto sdv = r.next<int32_t>();
        auto snu = r.next<int32_t>();
        auto snv = r.next<int32_t>();
        auto scoff = r.next<int64_t>();
        auto sxyz = r.next<double>();
        auto sw = r.next<double>();
        auto skuo = r.next<int64_t>();
        auto sku = r.next<double>();
        auto skvo = r.next<int64_t>();
        auto skv = r.next<double>();
        auto stoff = r.next<int64_t>();
        auto stdeg = r.next<int32_t>();
        auto stcoff = r.next<int64_t>();
        auto stuv = r.next<double>();
        auto stw = r.next<double>();
        auto stkoff = r.next<int64_t>();
        auto stk = r.next<double>();
        std::fclose(f);

        gwn_curves2d c2{(int64_t)deg.size(), deg.data(), off.data(), xy.data(), w.data()};
        for (double frac : {0.1, 0.0125}) {
            for (double tol : {0.0, 1e-8}) {
                Model m;
                m.dim = 2;
                std::string err;
                const gwn_params p = params(frac, tol);
                m.params = p;
                const gwn_status s = build2d_host(&c2, &p, m, err);
                std::printf("2d frac %g far_tol %g: status %d leaves %zu nodes %zu %s\n", frac, tol, s,
                            m.leaf_src.size(), m.tree.nodes.size(), err.c_str());
                if (s) return 1;
            }
        }

        gwn_nurbs2d nb{(int64_t)ndeg.size(), ndeg.data(), noff.data(), nxy.data(), nw.data(), nkoff.data(),
                       nk.data()};
        std::vector<int32_t> edeg;
        std::vector<int64_t> eoff;
        std::vector<double> exy, ew;
        std::string nerr;
        if (!extract_nurbs2d(nb, edeg, eoff, exy, ew, nerr)) {
            std::printf("nurbs: %s\n", nerr.c_str());
            return 1;
        }
        std::printf("nurbs: %zu segments\n", edeg.size());

        gwn_nurbs3d n3{(int64_t)sdu.size(), sdu.data(), sdv.data(), snu.data(), snv.data(), scoff.data(),
                       sxyz.data(), sw.data(), skuo.data(), sku.data(), skvo.data(), skv.data(), stoff.data(),
                       stdeg.data(), stcoff.data(), stuv.data(), stw.data(), stkoff.data(), stk.data()};
        NurbsPatches np3;
        if (!extract_nurbs3d(n3, np3, nerr)) {
            std::printf("nurbs3d: %s\n", nerr.c_str());
            return 1;
        }
        std::printf("nurbs3d: %zu patches %zu trim curves\n", np3.cp_w.size() / 16, np3.trim_degree.size());

        const int64_t np = (int64_t)cw.size() / 16;
        gwn_patches3d c3{np, cp.data(), cw.data(), toff.data(), tdeg.data(), tcoff.data(), tuv.data(), tw.data()};
        for (double frac : {0.1, 0.0125}) {
            Model m;
            m.dim = 3;
            std::string err;
            const gwn_params p = params(frac, 0.0);
            m.params = p;
            const gwn_status s = build3d_host(&c3, &p, m, err);
            std::printf("3d frac %g: status %d leaves %zu trims %zu %s\n", frac, s, m.leaf_src.size(),
                        m.trims.size(), err.c_str());
            if (s) return 1;
        }
    } catch (const std::string &e) {
        std::fprintf(stderr, "%s\n", e.c_str());
        return 2;
    }
    return 0;
}
