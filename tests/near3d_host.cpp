// Host build of the engine's 3D near-field rule (csrc/near3d.h), for CPU
// tests against the oracle.  Test infrastructure: compiled by
// tests/test_near3d_host.py, linked against the engine's library for the
// Gauss-Kronrod tables.
#include "../paper_2605_19200_amd/csrc/near3d.h"

#include <vector>

namespace gwn {
void gauss_kronrod01(int n, double *xk, double *wk, double *wg);
struct HostCtr {
    long long v[GWN_NCOUNTERS];
};
inline void ctr_add(HostCtr &c, int k, long long v) { c.v[k] += v; }
}  // namespace gwn

using namespace gwn;

// Solid angle / 4 pi of one leaf (homogeneous bicubic net h64, trim curves
// trims9 as 9 homogeneous values each) at q; *evals: integrand evaluations,
// *budget: 1 when the rule could not meet eps_q.
extern "C" double near_leaf(const double *h64, const double *trims9, int ntrim, double qx, double qy, double qz,
                            double eps_on, double eps_q, long long *evals, int *budget)
{
    static QuadTables Q = [] {
        QuadTables t;
        gauss_kronrod01(kOuterN, t.xo, t.wo, t.go);
        gauss_kronrod01(kRadialN, t.xr, t.wr, t.gr);
        return t;
    }();
    Prim3 P;
    for (int i = 0; i < 64; ++i) P.h[i] = h64[i];
    P.trim_begin = 0;
    P.trim_count = ntrim;
    std::vector<Trim3> tr(ntrim > 0 ? ntrim : 1);
    for (int k = 0; k < ntrim; ++k)
        for (int j = 0; j < 9; ++j) tr[k].h[j] = trims9[9 * k + j];
    HostCtr c{};
    bool ovf = false;
    const double v = near3d<true>(Q, &P, tr.data(), qx, qy, qz, eps_on, 4.0 * kPi * eps_q, ovf, c);
    *evals = c.v[GWN_C_PIECES];
    *budget = ovf ? 1 : 0;
    return v / (4.0 * kPi);
}

// The (2n+1)-point Kronrod extension of the n-point Gauss rule on [0, 1]
// that the engine builds at start-up: nodes xk, weights wk, Gauss weights wg
// (the Gauss nodes are xk[1], xk[3], ...).
extern "C" void gk_table(int n, double *xk, double *wk, double *wg) { gauss_kronrod01(n, xk, wk, wg); }
