// Host build of the engine's 3D near-field rule (csrc/near3d.h), for CPU
// tests against the oracle.  Test infrastructure: compiled by
// tests/test_near3d_host.py, linked against the engine's library for the
// Gauss-Kronrod tables.
//
// The rule runs one (query, leaf) pair on the 64 lanes of a wave, with
// cross-lane operations.  Here each lane is a fiber (ucontext) of one host
// thread: a cross-lane operation stores the lane's value, switches to the
// next lane, and reads the values once all 64 lanes have stored theirs (two
// buffers, alternating, so a lane that runs ahead cannot overwrite values
// that others have still to read).  The harness checks that every lane
// made the same number of cross-lane calls and returned the same bits,
// which is what the rule's uniform control requires on the GPU.
#include <ucontext.h>

#include <cstring>
#include <vector>

#include "../paper_2605_19200_amd/csrc/near3d.h"

namespace gwn {
void gauss_kronrod01(int n, double *xk, double *wk, double *wg);
struct HostCtr {
    long long v[GWN_NCOUNTERS];
};
inline void ctr_add(HostCtr &c, int k, long long v) { c.v[k] += v; }
}  // namespace gwn

using namespace gwn;

namespace {

constexpr int kLanes = 64;
constexpr size_t kStack = 512 * 1024;

struct Sched {
    ucontext_t main, ctx[kLanes];
    std::vector<char> stack[kLanes];
    unsigned long long buf[2][kLanes];
    int parity[kLanes];
    long long calls[kLanes];
    bool done[kLanes];
    bool broken;
};

struct FiberWave {
    Sched *s;
    int ln;
    int lane() const { return ln; }
    unsigned long long xchg(unsigned long long v, int src) const
    {
        const int p = s->parity[ln];
        s->buf[p][ln] = v;
        s->parity[ln] ^= 1;
        s->calls[ln]++;
        const int nx = (ln + 1) % kLanes;
        if (s->done[nx]) {   // lanes out of step: give up
            s->broken = true;
            setcontext(&s->main);
        }
        swapcontext(&s->ctx[ln], &s->ctx[nx]);
        return s->buf[p][src & (kLanes - 1)];
    }
    static unsigned long long bits(double x)
    {
        unsigned long long b;
        std::memcpy(&b, &x, 8);
        return b;
    }
    static double real(unsigned long long b)
    {
        double x;
        std::memcpy(&x, &b, 8);
        return x;
    }
    double shfl(double x, int src) const { return real(xchg(bits(x), src)); }
    int shfl(int x, int src) const { return (int)(unsigned)xchg((unsigned)x, src); }
    double shfl_xor(double x, int m) const { return shfl(x, ln ^ m); }
    int shfl_xor(int x, int m) const { return shfl(x, ln ^ m); }
    double bcast(double x, int src) const { return shfl(x, src); }
    int bcast(int x, int src) const { return shfl(x, src); }
    // the device's order: pairs, quads, half-row mirror, row mirror
    double sum16(double x) const
    {
        x += shfl(x, ln ^ 1);
        x += shfl(x, ln ^ 2);
        x += shfl(x, (ln & ~7) | (7 - (ln & 7)));
        x += shfl(x, (ln & ~15) | (15 - (ln & 15)));
        return x;
    }
    void argmin(double &d, int &k) const
    {
        for (int m = 32; m > 0; m >>= 1) {
            const double od = shfl(d, ln ^ m);
            const int ok = shfl(k, ln ^ m);
            if (od < d || (od == d && ok < k)) {
                d = od;
                k = ok;
            }
        }
    }
    unsigned long long ballot(bool p) const
    {
        const int par = s->parity[ln];
        xchg(p ? 1 : 0, 0);
        unsigned long long m = 0;
        for (int i = 0; i < kLanes; ++i)
            if (s->buf[par][i]) m |= 1ull << i;
        return m;
    }
};

struct Job {
    Sched *s;
    const QuadTables *Q;
    Prim3 P;
    std::vector<Trim3> tr;
    double q[3], eps_on, tol;
    double v[kLanes];
    bool ovf[kLanes];
    long long evals[kLanes];
};

Job *g_job = nullptr;

void lane_main(int lane)
{
    Job *J = g_job;
    FiberWave wv{J->s, lane};
    HostCtr c{};
    bool ovf = false;
    NearShared sh;   // the lane's own copy (the lanes run one after another)
    J->v[lane] =
        near3d<true>(wv, *J->Q, &J->P, J->tr.data(), J->q[0], J->q[1], J->q[2], J->eps_on, J->tol, ovf, c, sh);
    J->ovf[lane] = ovf;
    J->evals[lane] = c.v[GWN_C_PIECES];
    J->s->done[lane] = true;
    // hand over to the next lane, which is waiting in its last cross-lane
    // call; the last lane returns to the caller
    setcontext(lane == kLanes - 1 ? &J->s->main : &J->s->ctx[lane + 1]);
}

}  // namespace

// Solid angle / 4 pi of one leaf (homogeneous bicubic net h64, trim curves
// trims9 as 9 homogeneous values each) at q; *evals: integrand evaluations,
// *budget: 1 when the rule could not meet eps_q.  Returns NaN with *budget
// = -1 when the lanes did not stay in step or disagreed.
extern "C" double near_leaf(const double *h64, const double *trims9, int ntrim, double qx, double qy, double qz,
                            double eps_on, double eps_q, long long *evals, int *budget)
{
    static QuadTables Q = [] {
        QuadTables t;
        gauss_kronrod01(kOuterN, t.xo, t.wo, t.go);
        gauss_kronrod01(kRadialN, t.xr, t.wr, t.gr);
        return t;
    }();
    static Sched S;
    Job J;
    J.s = &S;
    J.Q = &Q;
    for (int i = 0; i < 64; ++i) J.P.h[i] = h64[i];
    J.P.trim_begin = 0;
    J.P.trim_count = ntrim;
    J.tr.resize(ntrim > 0 ? ntrim : 1);
    for (int k = 0; k < ntrim; ++k)
        for (int j = 0; j < 9; ++j) J.tr[k].h[j] = trims9[9 * k + j];
    J.q[0] = qx;
    J.q[1] = qy;
    J.q[2] = qz;
    J.eps_on = eps_on;
    J.tol = 4.0 * kPi * eps_q;
    g_job = &J;
    S.broken = false;
    for (int l = 0; l < kLanes; ++l) {
        S.parity[l] = 0;
        S.calls[l] = 0;
        S.done[l] = false;
        S.stack[l].resize(kStack);
        getcontext(&S.ctx[l]);
        S.ctx[l].uc_stack.ss_sp = S.stack[l].data();
        S.ctx[l].uc_stack.ss_size = kStack;
        S.ctx[l].uc_link = nullptr;
        makecontext(&S.ctx[l], (void (*)())lane_main, 1, l);
    }
    swapcontext(&S.main, &S.ctx[0]);
    bool same = !S.broken;
    for (int l = 1; l < kLanes && same; ++l)
        same = S.calls[l] == S.calls[0] && J.ovf[l] == J.ovf[0] && std::memcmp(&J.v[l], &J.v[0], 8) == 0;
    if (!same) {
        *evals = 0;
        *budget = -1;
        return NAN;
    }
    *evals = J.evals[0];   // counted by lane 0
    *budget = J.ovf[0] ? 1 : 0;
    return J.v[0] / (4.0 * kPi);
}

// The (2n+1)-point Kronrod extension of the n-point Gauss rule on [0, 1]
// that the engine builds at start-up: nodes xk, weights wk, Gauss weights wg
// (the Gauss nodes are xk[1], xk[3], ...).
extern "C" void gk_table(int n, double *xk, double *wk, double *wg) { gauss_kronrod01(n, xk, wk, wg); }
