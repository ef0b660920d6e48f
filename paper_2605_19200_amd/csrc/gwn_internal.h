// Internal definitions of the GWN engine: host model, device record layouts
// and the launch interface between the host build and the HIP kernels.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gwn.h"

namespace gwn {

constexpr int kStackDepth = 96;       // per-wave traversal stack (LDS entries)
constexpr int kBlock = 256;           // threads per block (4 wave64)
constexpr int kMaxBisectLevel = 48;   // 2D near-field bisection depth
constexpr double kPi = 3.14159265358979323846264338327950288;

// ---------------------------------------------------------------------------
// Device records.  Nodes are stored in depth-first pre-order: the left child
// of internal node i is i + 1, `right` holds the right child; a leaf stores
// -1 - leaf_index there.
// ---------------------------------------------------------------------------

// 2D node, three 128-byte lines.  Internal: centroid, squared AABB half
// diagonal r^2 and the complex form of the centred moments, stored scaled
// as m_k / r^(k+1) with m_k = integral (z - c)^k dz over the cluster's
// chords (re, im pairs, k = 0..16), so the far field is a series in
// r / (q - c), whose modulus is below 1 / beta for an accepted cluster.
// Leaf: m[0..3] holds the leaf's control-point AABB (lo.x, lo.y, hi.x,
// hi.y).  The float fields mirror c, r2 and the scaled m_0..m_15 for the
// FP32 pass.
constexpr int kMaxOrder2D = 16;
// The FP32 pass has a second unrolled instance at order 11 (FP32 rounding
// dominates beyond), used by the mixed form at FP64 order 12..14; the FP64
// pass has one at order 12 beside kMaxOrder2D.
constexpr int kMixedOrder2D = 11;
// Error-budgeted far test (2D): per internal node, the magnitudes of the
// scaled moments |m_k| / r^(k+1) for k = 0..kTailOrder2D, then L / r (L the
// total chord length) and rho = R / r (R the largest distance from the
// centroid to the node's AABB); see far_beta2d.
constexpr int kTailOrder2D = 32;
constexpr int kTailStride2D = kTailOrder2D + 3;
constexpr int kMaxOrder3D = 6;   // harmonic degree <= 7, see multipole3d.h
constexpr int kMaxL3 = kMaxOrder3D + 1;   // highest solid-harmonic degree
constexpr int kMpoleTerms = 35;           // (l, m) with 1 <= l <= 7, 0 <= m <= l
constexpr int kMpoleStride = 72;          // per node: 1/r, 0, then 35 (re, im) pairs
// The host also carries two more degrees, for the error-budgeted far test
// (far_beta3d): per node, the largest magnitude of each degree's term.
constexpr int kMaxLTail3 = kMaxL3 + 2;
constexpr int kMpoleTermsTail = kMaxLTail3 * (kMaxLTail3 + 3) / 2;   // (l, m) with 1 <= l <= 9
struct alignas(128) Node2 {
    double c[2];
    double r2;
    double m[2 * (kMaxOrder2D + 1)];
    int32_t right;
    int32_t degree;
    float fc[2];
    float fr2;
    float fm[2 * kMaxOrder2D];
    float pad[1];
};
static_assert(sizeof(Node2) == 512, "Node2 must be four 128-byte lines");

// 2D traversal record, 64 bytes, one array of them beside the Node2 array
// (same DFS index).  It holds everything a node test or a leaf's fast path
// reads, so the traversal's working set stays small enough for each XCD's
// L2.  Internal node: a = (c.x, c.y, r^2, r), f = the same in FP32 for the
// mixed form's pass.  Leaf: a = the curve's end points (x0, y0, x3, y3),
// f = its control-point AABB (lo.x, lo.y, hi.x, hi.y) rounded outward to
// FP32, so the chord angle of a query outside the box needs no other load.
// `right` and `degree` as in Node2.  The moments stay in Node2 and are read
// for accepted clusters only.
struct alignas(64) Hot2 {
    double a[4];
    int32_t right;
    int32_t degree;
    float f[4];
    int32_t escape;   // first node after this node's subtree in DFS order
    float pad;
};
static_assert(sizeof(Hot2) == 64, "Hot2 must be 64 bytes");

// 2D leaf primitive: homogeneous cubic control points (w x, w y, w) x 4.
struct Prim2 {
    double h[12];
};

// 3D node, three 128-byte lines.  Internal: centroid, squared AABB half diagonal and the
// contracted centred moments used by the order-2 expansion:
//   t[0..2]   M0_k
//   t[3..8]   symmetric part of M1: M1_00, M1_11, M1_22, M1_01+M1_10,
//             M1_02+M1_20, M1_12+M1_21
//   t[9..11]  e_k = 2 a_k + b_k with a_i = sum_j M2_ijj, b_k = sum_i M2_iik
//   t[12..21] coefficients of the cubic form sum_ijk M2_ijk s_i s_j s_k on
//             the monomials s0^3, s1^3, s2^3, s0^2 s1, s0^2 s2, s1^2 s0,
//             s1^2 s2, s2^2 s0, s2^2 s1, s0 s1 s2
// Leaf: t[0..5] = AABB lo[3], hi[3]; `aux` = first index of the leaf's
// precomputed quadrature nodes, `count` = their number, t[6..8] = the node
// counts of the three rules of kLeafRules stored one after the other,
// `right` = -1 - leaf.
struct alignas(128) Node3 {
    double c[3];
    double r2;
    double t[22];
    int32_t right;
    int32_t count;
    int64_t aux;
    float fc[3];
    float fr2;
    float ft[22];
    int32_t escape;   // first node after this node's subtree in DFS order
    float pad[5];
};
static_assert(sizeof(Node3) == 384, "Node3 layout");

// 3D leaf: homogeneous bicubic control net, 16 x (wx, wy, wz, w), u-major,
// plus the trim-curve range and the untrimmed flag.
struct Prim3 {
    double h[64];
    int32_t trim_begin;   // index into the model's trim-curve array
    int32_t trim_count;   // 0 = untrimmed (whole square)
    int32_t pad[2];
};

// Trim curve in (u, v), homogeneous, degree 1 or 2 stored as 3 points
// (degree 1 is elevated to 2).
struct Trim3 {
    double h[9];          // (w u, w v, w) x 3
    double pad;
};

// Gauss-Legendre orders of a 3D leaf's direct rules for well-separated
// queries, finest first, with the distance/half-diagonal ratios from which
// each is used (checked against the oracle: the 8- and 6-point rules hold the
// bound at these ratios on rational trimmed patches, where the weights limit
// the convergence of lower orders).
constexpr int kLeafRules[3] = {12, 8, 6};
constexpr double kLeafRuleRatio[3] = {0.0, 2.5, 6.0};

// Precomputed far-rule quadrature node of a 3D leaf: position and weighted
// normal (Green-scattered Gauss-Legendre node, Sec. 3.1).
struct QNode3 {
    double x[3];
    double n[3];
};

// ---------------------------------------------------------------------------
// Kernel-side model descriptor (passed by value / stored in device arrays).
// ---------------------------------------------------------------------------
struct DevModel {
    const void *nodes;      // Node2* or Node3*
    const void *hot;        // Hot2* (2D)
    const void *prims;      // Prim2* or Prim3*
    const void *trims;      // Trim3* (3D)
    const void *qnodes;     // QNode3* (3D)
    const void *mpole;      // 3D: per node 72 doubles, 1/r then scaled multipole moments
    const void *fmpole;     // 3D: FP32 mirror of mpole
    int32_t *flag;          // overflow count (device): queries that hit a limit, never reset
    int32_t dim;
    int32_t n_nodes;
    int32_t order;
    int32_t precision;
    double beta2;           // beta^2 (FP64 form / reclassification)
    double beta2_mixed;     // beta_mixed^2 (FP32 pass)
    double band;            // reclassification band
    double lo[3];           // bbox for space-filling-curve keys
    double inv_ext[3];
    double eps_on;          // absolute on-boundary distance
    double near_ratio2;     // 3D: (near_ratio)^2 factor on squared AABB diagonal
    double eps_q;           // 3D near-field tolerance
    int32_t gl_n;           // 3D GL nodes
    int32_t leaf_far;       // 3D: far leaves by their own expansion (gwn_params)
    int32_t wave_accept;    // FP64 far tests decided for the whole wave (gwn_params)
};

// ---------------------------------------------------------------------------
// Host-side tree (shared by 2D and 3D builds).
// ---------------------------------------------------------------------------
struct HostNode {
    int is_leaf = 0;
    int left = -1, right = -1;   // DFS indices of children (internal)
    int leaf = -1;               // leaf index (leaf)
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    double c[3] = {0, 0, 0};
    double r = 0;
    double wsum = 0;             // centroid weight (chord length / area)
    double wc[3] = {0, 0, 0};    // weighted centroid sum
    std::vector<double> U;       // uncentered moments: M0[d], M1[d*d], M2[d^3]
    std::vector<double> M;       // centred moments, same layout
};

struct HostTree {
    int dim = 2;
    std::vector<HostNode> nodes;  // DFS pre-order, root = 0
    int depth = 0;
};

// Build the Karras BVH over `n` leaves (AABBs lo/hi stride 3), sum the leaves'
// uncentered moments up the tree and centre them in place (Alg. 1
// ConstructBVH, SumUncenteredMomentsUpTree, CenterMomentsInPlace).
// leafU: n * nm uncentered moments, leafW: n centroid weights, leafWC: n * 3
// weighted centroid sums.  Returns false with `err` set on failure.
// device >= 0: the Morton codes, their sort and the child links run on that
// device (lbvh_device); the tree is the same.
bool build_tree(int dim, int n, const double *lo, const double *hi, const double *leafU,
                const double *leafW, const double *leafWC, const double *model_lo,
                const double *model_hi, HostTree &tree, std::string &err, int device = -1);
// Sorted leaf order and Karras child links (>= 0 internal, < 0 leaf at
// sorted position -1 - x) of n >= 2 leaves, computed on `device`.
bool lbvh_device(int device, int dim, int n, const double *lo, const double *hi, const double *model_lo,
                 const double *model_hi, std::vector<int> &order, std::vector<int> &cl, std::vector<int> &cr,
                 std::string &err);

inline int n_moments(int dim) { return dim + dim * dim + dim * dim * dim; }

// ---------------------------------------------------------------------------
// Host model (behind gwn_handle).
// ---------------------------------------------------------------------------
struct Model {
    int dim = 2;
    gwn_params params{};
    int64_t n_input = 0;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    double diag = 0;
    HostTree tree;
    // leaves in BVH leaf order
    std::vector<int64_t> leaf_src;
    std::vector<double> leaf_h;       // 12 (2D) or 64 (3D) doubles per leaf
    std::vector<int32_t> leaf_degree; // 2D original degree
    std::vector<double> cmom2;        // 2D: per node 2*(kMaxOrder2D+1) centred complex moments
    std::vector<double> tail2;        // 2D: per node kTailStride2D doubles (far_beta2d)
    // 3D only
    std::vector<Trim3> trims;
    std::vector<int32_t> leaf_trim_begin, leaf_trim_count;
    std::vector<QNode3> qnodes;       // 3D node sets of a host build
    void *d_qnodes = nullptr;          // 3D node sets of a device build (device memory until upload)
    int64_t n_qnodes_dev = 0;
    std::vector<int64_t> leaf_q_begin, leaf_q_count;
    std::vector<std::array<int, 3>> leaf_q_rules;
    std::vector<double> mpole;        // 3D: per node kMpoleStride doubles (multipole3d.h)
    std::vector<double> tail3;        // 3D: per node kMaxLTail3 doubles (far_beta3d)
    // device
    int device = -1;
    void *d_arena = nullptr;
    int64_t arena_bytes = 0;
    int32_t *d_flag = nullptr;     // device overflow count (monotonic)
    int32_t *h_flag = nullptr;     // pinned copy of it, taken after each launch
    uint32_t flag_seen = 0;        // count already reported as GWN_EOVERFLOW
    void *flag_event = nullptr;    // hipEvent_t
    DevModel dev{};
};

// builders (host)
// Far-field factor of one 2D cluster under an error budget: the smallest
// beta >= 2 for which the truncation error of its order-`order` expansion
// is at most `tol` (in turns) wherever ||q - c|| > beta r.  +inf when no
// beta meets the budget.
double far_beta2d(const double *tail, int order, double tol);
// Far-field factor of one 3D cluster under an error budget (build3d.cpp):
// the smallest beta in [kBetaMin3, 64] for which the estimated truncation
// error of its order-`order` expansion is at most 4 pi tol (solid angle)
// wherever ||q - c|| > beta r; +inf when none is.  A[l - 1], l = 1 ..
// kMaxLTail3: the largest magnitude of the cluster's degree-l term at unit
// distance.
constexpr double kBetaMin3 = 1.5;
double far_beta3d(const double *A, double r, int order, double tol);
// Chord moments of every 2D cluster on `device` (moments2d.hip): cmom2 and
// tail2 as the host build lays them out, except tail2's rho entries, which
// the caller fills.  chord_ends holds (ax, ay, bx, by) per leaf in DFS order;
// end[i] is the end of node i's DFS subtree.
// AdaptiveSubdivision of a 2D model on `device` (moments2d.hip): curve i is
// the homogeneous cubic cubics[12 i .. 12 i + 11]; a piece is halved (de
// Casteljau at t = 1/2) while the squared diagonal of its control-point box
// is >= limit2 and its depth < 40.  Returns the leaves in the host build's
// order (curve by curve, left to right in t): leaf_h (12 doubles each) and
// the index of the curve each came from.
gwn_status subdiv2d_device(int device, const std::vector<double> &cubics, double limit2,
                           std::vector<double> &leaf_h, std::vector<int32_t> &leaf_curve, std::string &err);
gwn_status moments2d_device(int device, const std::vector<HostNode> &nodes, const std::vector<int> &end,
                            const std::vector<double> &chord_ends, std::vector<double> &cmom2,
                            std::vector<double> &tail2, std::string &err);
gwn_status build2d_host(const gwn_curves2d *c, const gwn_params *p, Model &m, std::string &err);
gwn_status build3d_host(const gwn_patches3d *c, const gwn_params *p, Model &m, std::string &err);
// Bezier extraction of 2D NURBS curves (nurbs.cpp); false with err set on
// invalid input
bool extract_nurbs2d(const gwn_nurbs2d &in, std::vector<int32_t> &deg, std::vector<int64_t> &off,
                     std::vector<double> &xy, std::vector<double> &w, std::string &err);
// Bezier extraction of trimmed NURBS surfaces (nurbs.cpp), in the layout of
// gwn_patches3d plus each patch's source surface; false with err set on
// invalid input
struct NurbsPatches {
    std::vector<double> cp_xyz, cp_w;
    std::vector<int64_t> trim_offset, trim_cp_offset, source;
    std::vector<int32_t> trim_degree;
    std::vector<double> trim_cp_uv, trim_cp_w;
};
bool extract_nurbs3d(const gwn_nurbs3d &in, NurbsPatches &out, std::string &err);
// Device leaf quadrature of a 3D model (quad3d.hip).  leafquad3d_moments
// uploads the leaves (nets: 64 doubles per leaf, the homogeneous bicubic net
// [i][j][wx, wy, wz, w]; curves: each leaf's boundary curves, its trims or
// the edge u = 1 of an untrimmed square, leaf l's at [coff[l], coff[l+1]);
// box: lo[3], hi[3] per leaf) and returns, per leaf in that order, the
// uncentred moments U (n_moments(3) each), area Wt, area-weighted centroid
// sums WC, centroid LC, multipole moments LN about LC (kMpoleTermsTail
// (re, im) pairs each) and the sizes of the three node-set rules.  Rule r of
// rule_x / rule_w has rule_n[r] nodes: 0-2 the node-set rules, 3 the moment
// rule.  leafquad3d_nodes then writes the node sets of leaf l at qbase[l]
// of a new device array of `total` QNode3 (returned in *out, owned by the
// caller).  The uploaded leaves stay in `st` between the two calls.
constexpr int kMaxQuadRule = 32;
struct LeafQuad3 {
    int device = -1;
    int64_t nl = 0;
    void *nets = nullptr, *curves = nullptr, *coff = nullptr, *tab = nullptr, *counts = nullptr;
    ~LeafQuad3();
};
gwn_status leafquad3d_moments(int device, const std::vector<double> &nets, const std::vector<Trim3> &curves,
                              const std::vector<int64_t> &coff, const std::vector<double> &box,
                              const double (*rule_x)[kMaxQuadRule], const double (*rule_w)[kMaxQuadRule],
                              const int *rule_n, LeafQuad3 &st, std::vector<double> &U, std::vector<double> &Wt,
                              std::vector<double> &WC, std::vector<double> &LC, std::vector<double> &LN,
                              std::vector<std::array<int, 3>> &counts, std::string &err);
gwn_status leafquad3d_nodes(LeafQuad3 &st, const std::vector<int64_t> &qbase, int64_t total, void **out,
                            std::string &err);
// Clip the closed trim loops `in` of a patch's visible region to the half
// x_dir <= c (low) or >= c of the unit square and map them to the half's
// own unit square (trimclip.cpp).  false: the cut passes through a junction
// of two trim curves or touches a loop tangentially (move the cut).  An
// empty `out` means the half holds none of the visible region.
bool clip_trims_half(const std::vector<Trim3> &in, int dir, double c, bool low, std::vector<Trim3> &out);
// upload to device and fill m.dev
gwn_status upload_model(Model &m, std::string &err);
void refresh_dev_params(Model &m);
void release_device(Model &m);

// query launchers (query.hip)
struct Segment {
    const Model *model;
    int64_t q_begin, q_end;   // rows of the points/output arrays
};
// Scratch handed to a launch instead of stream-ordered allocation (the entry
// point that allocates nothing); ptr == nullptr: allocate from the pool.
struct ExtScratch {
    void *ptr = nullptr;
    size_t bytes = 0;
};
constexpr size_t kNoAllocScratchBytes = (size_t)96 << 20;   // per GPU
constexpr int kMaxDevices = 64;
gwn_status launch_queries(const std::vector<Segment> &segs, int dim, const double *points,
                          double *out_gwn, uint8_t *out_inside, int64_t *counters, void *stream,
                          std::string &err, const ExtScratch &ext = ExtScratch{});
// Scratch bytes of one query call over n rows in n_seg segments (an upper
// bound; exact for one segment).
gwn_status query_scratch_bytes(int dim, int64_t n, int32_t n_seg, int64_t &bytes, std::string &err);
// This device's fixed scratch array (address looked up once per device).
gwn_status noalloc_scratch(ExtScratch &out, std::string &err);
// Kernel timing (query.hip): per-kernel sums of the last collected set of
// recorded launches (gwn_profile, gwn_profile_kernel).
constexpr int kProfKernels = 3;   // GWN_K_QUERY2D, GWN_K_TRAV3D, GWN_K_NEAR3D
gwn_status profile_control(int enable, double *total_ms, int64_t *launches);
gwn_status profile_kernel(int kernel, double *ms, int64_t *launches);

}  // namespace gwn
