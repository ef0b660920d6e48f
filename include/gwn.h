/*
 * gwn.h -- C ABI of the MI355X (gfx950) engine for spatially accelerated
 * generalized winding numbers (GWN) on curved boundaries.
 *
 * The problem (Alg. 1 of the paper, "AgglomeratedGWN"): given a collection of
 * NURBS objects {Gamma} -- rational Bezier curves in 2D, trimmed rational
 * bicubic patches in 3D -- and query points {q}, return the GWN w_q at each q
 * (Eq. gwn_sum: the sum over all primitives of the (solid) angle each one
 * subtends at q, normalised so that a closed counter-clockwise / outward
 * oriented boundary gives 1 inside) and the containment decision
 * inside = (w_q >= 0.5), i.e. round(w_q) >= 1 (Sec. 4.3).
 *
 * gwn_build2d / gwn_build3d run the preprocessing phase of Alg. 1 on the host
 * (adaptive subdivision to the 10% bounding-box rule of Sec. 3.2, uncentered
 * moments of Sec. 3.1, Karras BVH, moment up-sweep and centering) and upload
 * the result to one GPU.  gwn_query runs the query phase of Alg. 1 on the
 * GPU: BVH traversal, the far-field test ||q - centroid|| > beta * radius,
 * the Taylor approximation of Eq. taylor (order 0..16 in 2D, 0..6 in 3D)
 * for far clusters, and
 * direct evaluation (Sec. 3.3) of every leaf reached.
 *
 * Conventions common to every entry point:
 *  - Every function returns a gwn_status; GWN_OK is 0.  On any other status
 *    gwn_last_error() returns a message (thread-local, valid until the next
 *    call on the same thread).  No C++ exception crosses this boundary.
 *  - Host arrays passed to gwn_build* are read during the call only and are
 *    never retained: the caller keeps ownership.
 *  - Query points and outputs are DEVICE pointers owned by the caller.  Query
 *    calls only enqueue work on `stream` (a hipStream_t, NULL = the null
 *    stream) and return without synchronising; results are ready when the
 *    stream reaches that point.  Scratch memory is taken from HIP's
 *    stream-ordered allocator and released on the same stream.
 *  - A handle is immutable while queries may be in flight, and may be queried
 *    from several streams at once.  gwn_set_params and gwn_free must not race
 *    with queries that use the handle.
 */
#ifndef GWN_H
#define GWN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gwn_model *gwn_handle;
typedef int32_t gwn_status;

enum {
    GWN_OK = 0,
    GWN_EINVAL = 1,        /* invalid argument or malformed geometry            */
    GWN_ENOMEM = 2,        /* host or device allocation failed                  */
    GWN_EHIP = 3,          /* a HIP runtime call failed (message has the code)  */
    GWN_EUNSUPPORTED = 4,  /* valid request the engine does not implement       */
    GWN_EOVERFLOW = 5      /* a traversal or subdivision stack limit was hit    */
};

enum { GWN_FP64 = 0, GWN_MIXED = 1 };

/* 2D input: rational Bezier curves of degree 1..3 (Sec. 3, P0 of Alg. 1).
 * Curve i has control points cp_xy[2*k], cp_xy[2*k+1] and weights cp_w[k]
 * for k in [cp_offset[i], cp_offset[i+1]), which must hold degree[i]+1
 * points.  Weights must be finite and > 0, coordinates finite. */
typedef struct {
    int64_t n_curves;
    const int32_t *degree;     /* [n_curves]                  */
    const int64_t *cp_offset;  /* [n_curves + 1], cp_offset[0] == 0 */
    const double *cp_xy;       /* [2 * n_cp] Euclidean points */
    const double *cp_w;        /* [n_cp] weights              */
} gwn_curves2d;

/* 2D NURBS input, converted to gwn_curves2d by gwn_nurbs2d_extract.  Curve i
 * has degree p = degree[i] (1..3), control points cp_xy / weights cp_w at
 * k in [cp_offset[i], cp_offset[i+1]) (n_i >= p + 1 of them; weights finite
 * and > 0) and the knot vector knots[knot_offset[i] .. knot_offset[i+1]-1]
 * of n_i + p + 1 finite, non-decreasing values, clamped (its first p + 1 and
 * last p + 1 values equal) and with no interior value repeated more than
 * p + 1 times. */
typedef struct {
    int64_t n_curves;
    const int32_t *degree;       /* [n_curves]                  */
    const int64_t *cp_offset;    /* [n_curves + 1], cp_offset[0] == 0 */
    const double *cp_xy;         /* [2 * n_cp] Euclidean points */
    const double *cp_w;          /* [n_cp] weights              */
    const int64_t *knot_offset;  /* [n_curves + 1], knot_offset[0] == 0 */
    const double *knots;         /* [n_knots]                   */
} gwn_nurbs2d;

/* 3D input: rational bicubic Bezier patches with optional trimming (Sec. 3.1,
 * Fig. quadrature_demo).  Patch i has control points
 * cp_xyz[48*i + 3*(4*a + b) + axis] (a indexes u, b indexes v) and weights
 * cp_w[16*i + 4*a + b] (> 0).  Its trim curves are trim_offset[i] ..
 * trim_offset[i+1]-1 (an empty range means the whole square [0,1]^2 is
 * visible).  Trim curve c is a rational Bezier in (u, v) of degree
 * trim_degree[c] (1 or 2) with control points trim_cp_uv[2*k..2*k+1] and
 * weights trim_cp_w[k] for k in [trim_cp_offset[c], trim_cp_offset[c+1]).
 * A patch's trim curves form closed loops of consecutive curves inside
 * [0,1]^2: the outer boundary counter-clockwise (the square must be given
 * explicitly when other loops are present), holes clockwise.  The surface
 * normal S_u x S_v must point out of the body. */
typedef struct {
    int64_t n_patches;
    const double *cp_xyz;          /* [48 * n_patches] */
    const double *cp_w;            /* [16 * n_patches] */
    const int64_t *trim_offset;    /* [n_patches + 1]  */
    const int32_t *trim_degree;    /* [n_trim]         */
    const int64_t *trim_cp_offset; /* [n_trim + 1]     */
    const double *trim_cp_uv;      /* [2 * n_trim_cp]  */
    const double *trim_cp_w;       /* [n_trim_cp]      */
} gwn_patches3d;

/* 3D NURBS input, converted to gwn_patches3d by gwn_nurbs3d_extract (Sec. 3.1:
 * trimmed NURBS surfaces, Bezier extraction as in Sec. 3.2).  Surface i has
 * degrees degree_u[i], degree_v[i] (1..3 each) and an n_u[i] x n_v[i] net:
 * control point (a, b) (a indexes u) is cp_xyz[3*k..3*k+2] with weight
 * cp_w[k] (finite, > 0), k = cp_offset[i] + n_v[i]*a + b; cp_offset[i+1] -
 * cp_offset[i] must equal n_u[i] * n_v[i].  Its knot vectors are
 * knots_u[knot_u_offset[i] ..] (n_u[i] + degree_u[i] + 1 values) and
 * knots_v[knot_v_offset[i] ..], each clamped, non-decreasing, finite, no
 * interior value repeated more than degree + 1 times (as for
 * gwn_nurbs2d); the parameter domain is [U_p, U_n] x [V_q, V_n].  Its trim
 * curves are trim_offset[i] .. trim_offset[i+1]-1 (none: the whole domain is
 * visible): 2D NURBS curves in (u, v) of degree 1 or 2, laid out as in
 * gwn_nurbs2d (trim_cp_offset / trim_cp_uv / trim_cp_w, trim_knot_offset /
 * trim_knots), lying in the domain and forming closed loops there with the
 * orientation rules of gwn_patches3d (outer boundary counter-clockwise and
 * given explicitly, holes clockwise). */
typedef struct {
    int64_t n_surfaces;
    const int32_t *degree_u, *degree_v;   /* [n_surfaces] */
    const int32_t *n_u, *n_v;             /* [n_surfaces] */
    const int64_t *cp_offset;             /* [n_surfaces + 1], cp_offset[0] == 0 */
    const double *cp_xyz;                 /* [3 * n_cp] */
    const double *cp_w;                   /* [n_cp] */
    const int64_t *knot_u_offset;         /* [n_surfaces + 1], [0] == 0 */
    const double *knots_u;
    const int64_t *knot_v_offset;         /* [n_surfaces + 1], [0] == 0 */
    const double *knots_v;
    const int64_t *trim_offset;           /* [n_surfaces + 1], [0] == 0 */
    const int32_t *trim_degree;           /* [n_trim] */
    const int64_t *trim_cp_offset;        /* [n_trim + 1], [0] == 0 */
    const double *trim_cp_uv;             /* [2 * n_trim_cp] */
    const double *trim_cp_w;              /* [n_trim_cp] */
    const int64_t *trim_knot_offset;      /* [n_trim + 1], [0] == 0 */
    const double *trim_knots;
} gwn_nurbs3d;

/* Parameters.  Build-time fields fix the tree; query-time fields (marked Q)
 * may be changed later with gwn_set_params. */
typedef struct {
    double beta;           /* Q: far-field factor of the FP64 form: a cluster is
                              far when ||q - c|| > beta * r, r = AABB half
                              diagonal (Alg. 1; default 2, Sec. 3).  2D needs
                              beta >= 2 (chord substitution, Sec. 3.1).       */
    double beta_mixed;     /* Q: far-field factor of the FP32 pass of the mixed
                              form (default 4)                               */
    int32_t taylor_order;  /* Q: expansion order of Eq. taylor; default 2
                              (Sec. 4.2).  2D: 0..16, 3D: 0..6 -- orders above
                              2 carry the same expansion further (2D: exact
                              chord moments in complex form; 3D: solid
                              harmonics, see GWN_I_MULTIPOLE)                */
    int32_t precision;     /* Q: GWN_FP64 or GWN_MIXED                         */
    double reclass_band;   /* Q: mixed form: queries with |w - 0.5| < band are
                              re-evaluated in FP64 (default 1e-2)            */
    double max_diag_frac;  /* subdivision threshold: split a primitive while its
                              AABB diagonal >= frac * model diagonal
                              (default 0.10, Sec. 3.2)                        */
    double eps_on;         /* on-boundary distance relative to the model
                              diagonal (default 1e-12)                        */
    int32_t gl_nodes;      /* 3D: Gauss-Legendre nodes per rule for leaf and
                              moment quadrature (default 10, Sec. 3.1)        */
    int32_t device;        /* HIP device ordinal; -1 builds a host-only handle
                              that can be inspected but not queried           */
    double near_ratio;     /* Q, 3D: a leaf is evaluated with the near-field
                              rule (Green's theorem about the foot point, graded
                              panels) when dist(q, AABB) < near_ratio * AABB
                              diagonal (default 0.25); farther leaves use their
                              precomputed Gauss-Legendre node sets            */
    double eps_q;          /* Q, 3D: tolerance of a leaf's direct evaluation by
                              the near-field rule, in units of w (Sec. 3.3;
                              default 1e-6, the paper's value for the
                              accelerated method, Sec. 4.2).  Each panel and
                              radial piece carries a Gauss-Kronrod error
                              estimate; a leaf is refined until the estimates
                              meet eps_q, and a leaf that cannot meet it
                              within its refinement budget makes its query NaN
                              and is reported as GWN_EOVERFLOW              */
    int32_t leaf_far;      /* Q, 3D: 1 = a leaf reached by the traversal that
                              passes the far test ||q - c|| > beta * r itself is
                              evaluated by its own far-field expansion, like a
                              cluster (the same error criterion; its direct
                              rule costs hundreds to thousands of quadrature
                              nodes); 0 = every reached leaf is evaluated
                              directly, as in Alg. 1.  Default 1; 2D leaves
                              are always direct (the chord angle is exact)   */
    int32_t wave_accept;   /* Q: 0 (default): each query takes a cluster as
                              far by its own test, as in Alg. 1, so a query's
                              value does not depend on the other queries of
                              the call.  1: a cluster is taken as far only
                              when every query of the wave (the 64
                              neighbouring queries of the call's
                              space-filling-curve order that share one
                              traversal) passes its test, otherwise all of
                              them descend: the far-field terms then run on
                              full waves instead of a few lanes, and each
                              query's accepted clusters are the same or
                              smaller ones (same error bound per cluster).
                              A query's value then depends on the queries
                              that share its wave: a call repeats bit for
                              bit, but the same point in another call (a
                              subset, a split, another order of points
                              that share a sort key, or another call size,
                              which sets the queries per wave) may differ
                              within the error budget.  Applies to every
                              far test: the FP64 form and both passes of
                              the mixed form.                              */
    double far_tol;        /* Q: error budget of the FP64 far test, per
                              accepted cluster.  0 (default): a cluster is
                              far when ||q - c|| > beta * r.  > 0: each
                              cluster gets its own factor beta_c, so that
                              the truncation error of its order-taylor_order
                              expansion is <= far_tol wherever ||q - c|| >
                              beta_c * r (the paper's future work on a
                              geometry-aware beta, Sec. 5).  2D (units of w,
                              turns): the smallest beta_c >= 2 for which a
                              bound from the moments up to order 32 and the
                              extent beyond holds.  3D (units of w too, the
                              solid angle over 4 pi): the smallest beta_c in
                              [1.5, 64] for which an estimate from the two
                              first omitted harmonic degrees, sampled over
                              256 directions, holds (an estimate, not a
                              bound); with leaf_far the same applies to
                              leaves.  The truncation error of a query is
                              then about far_tol times the number of
                              clusters accepted for it; `beta` is not used
                              by the FP64 tests, the FP32 pass of the mixed
                              form keeps beta_mixed.  Changing far_tol, or
                              taylor_order while far_tol > 0, through
                              gwn_set_params rewrites the cluster radii on
                              the device after a device-wide
                              synchronisation.                              */
} gwn_params;

/* Fill *p with the defaults listed above. */
void gwn_default_params(gwn_params *p);

/* Build a 2D model (Alg. 1 preprocessing).  `curves` and `params` are read
 * during the call only.  On success *out owns host and device memory until
 * gwn_free.  Errors: GWN_EINVAL (NULL pointers, bad degree/offsets/weights,
 * non-finite data, beta < 2), GWN_ENOMEM, GWN_EHIP, GWN_EOVERFLOW (tree deeper
 * than the traversal stack). */
gwn_status gwn_build2d(const gwn_curves2d *curves, const gwn_params *params, gwn_handle *out);

/* Bezier extraction of 2D NURBS curves (Sec. 3.2: NURBS input is split into
 * its rational Bezier segments ahead of the adaptive subdivision).  Each knot
 * span [t_k, t_k+1) of positive length gives one segment of the curve's
 * degree, whose control points are the blossom values of the span at
 * (t_k^(p-j), t_k+1^j), j = 0..p, in homogeneous coordinates; zero-length
 * spans give none.  Segments keep the curve order and the parameter
 * direction, so the output describes the same point set with the same
 * orientation and can be passed to gwn_build2d as it is.
 * Two calls: with degree == NULL only *n_segments and *n_points are written
 * (the output sizes).  Then, with *n_segments and *n_points holding the
 * capacities of degree[], cp_offset[] (capacity + 1 entries), cp_xy[]
 * (2 * capacity) and cp_w[], the arrays are filled and the two counts
 * receive the sizes written.  All arrays are host memory owned by the
 * caller.  Errors: GWN_EINVAL (NULL pointers, bad degree, offsets, knot
 * count or order, unclamped knots, non-finite data, weight <= 0, capacity
 * too small). */
gwn_status gwn_nurbs2d_extract(const gwn_nurbs2d *in, int64_t *n_segments, int64_t *n_points,
                               int32_t *degree, int64_t *cp_offset, double *cp_xy, double *cp_w);

/* Bezier extraction of trimmed NURBS surfaces into the gwn_patches3d layout.
 * Every knot span (u, v) of positive size becomes one rational bicubic
 * patch (the span's Bezier net by blossoming, raised to degree 3 in each
 * direction by exact degree elevation), spans in surface order, u-major.
 * A trimmed surface's loops are clipped to each span and mapped to the
 * span's unit square, as degree-2 trim curves; a span that holds none of
 * the visible region is dropped, and a span that is wholly visible gets no
 * trim curves.  Two calls, as gwn_nurbs2d_extract: with cp_xyz == NULL only
 * *n_patches, *n_trims and *n_trim_cp are written; then, with those holding
 * the capacities of cp_xyz[48 * n], cp_w[16 * n], trim_offset[n + 1],
 * trim_degree[n_trims], trim_cp_offset[n_trims + 1], trim_cp_uv[2 * n_trim_cp]
 * and trim_cp_w[n_trim_cp], the arrays are filled and the counts receive the
 * sizes written.  Host memory owned by the caller.  Errors: GWN_EINVAL (NULL
 * pointers, bad degrees, counts, offsets or knot vectors, non-finite data,
 * weights <= 0, trim curves outside the domain or not closed, a trim loop
 * that passes through a junction of two trim curves on an interior knot
 * line or touches one tangentially -- the message names the surface and
 * the knot --, capacity too small). */
gwn_status gwn_nurbs3d_extract(const gwn_nurbs3d *in, int64_t *n_patches, int64_t *n_trims, int64_t *n_trim_cp,
                               double *cp_xyz, double *cp_w, int64_t *trim_offset, int32_t *trim_degree,
                               int64_t *trim_cp_offset, double *trim_cp_uv, double *trim_cp_w);

/* Build a 3D model (Alg. 1 preprocessing, moments by Gauss-Legendre quadrature
 * over the trimmed domain via Green's theorem, Sec. 3.1).  Errors as for
 * gwn_build2d, plus GWN_EINVAL for trim curves outside [0,1]^2, open trim
 * loops or a bad trim degree. */
gwn_status gwn_build3d(const gwn_patches3d *patches, const gwn_params *params, gwn_handle *out);

/* Replace the query-time (Q) fields of a handle's parameters.  Build-time
 * fields of `params` are ignored.  GWN_EINVAL for out-of-range values. */
gwn_status gwn_set_params(gwn_handle h, const gwn_params *params);

/* Read back a handle's parameters. */
gwn_status gwn_get_params(gwn_handle h, gwn_params *out);

/* Query phase of Alg. 1.  points: device double[n * dim] interleaved
 * (x, y[, z]); out_gwn: device double[n]; out_inside: device uint8[n]
 * (1 when w >= 0.5) or NULL.  n may be 0.  Asynchronous on `stream`.
 * Errors: GWN_EINVAL (NULL handle, n < 0, NULL buffers with n > 0, host-only
 * handle), GWN_EHIP, GWN_EOVERFLOW (a query of an earlier call on the handle
 * hit a traversal, near-field or bisection limit; its output is NaN.  Each
 * such call is reported once, by the first call on the handle that starts
 * after the earlier call's work has completed on its stream).
 * Scratch comes from the device's default stream-ordered pool (hipMallocAsync
 * on `stream`, freed on it at the end of the call); building a model for a
 * device raises that pool's release threshold to 1 GiB, process-wide, so the
 * scratch stays mapped between calls. */
gwn_status gwn_query(gwn_handle h, const double *points, int64_t n, double *out_gwn,
                     uint8_t *out_inside, void *stream);

/* gwn_query for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and results (bitwise) as gwn_query, but the launch's
 * scratch (sort keys and permutation, sort temporaries, 3D near-field
 * records) is a fixed array of GWN_NOALLOC_SCRATCH_BYTES in device memory,
 * one per GPU, reserved by the library from its first such call on that GPU
 * until the process ends.  The call makes no hipMalloc / hipFree and no
 * other allocation.  All calls on one GPU share that array and it keeps the
 * last call's contents (nothing in it needs clearing: every record is
 * written before it is read); calls that overlap on one GPU -- e.g. on two
 * streams -- race on it and must be serialised by the caller.  A call whose
 * scratch (gwn_query_scratch_bytes(h, n, 1, ...)) exceeds the array fails
 * with GWN_EINVAL before any launch: about 3.5M queries fit in 2D, about
 * 320k in 3D. */
#define GWN_NOALLOC_SCRATCH_BYTES ((int64_t)96 << 20)
gwn_status gwn_query_noalloc(gwn_handle h, const double *points, int64_t n, double *out_gwn,
                             uint8_t *out_inside, void *stream);

/* Device scratch bytes one gwn_query / gwn_query_batch call takes at once for
 * n query rows in n_seg segments (exact for n_seg = 1, an upper bound
 * otherwise), for admission by memory budget.  Host-only; needs a HIP
 * runtime (the sort's temporary size is asked from it). */
gwn_status gwn_query_scratch_bytes(gwn_handle h, int64_t n, int32_t n_seg, int64_t *bytes);

/* Batched query over several models in shared launches (the served form).
 * Segment s covers query rows [seg_offset[s], seg_offset[s+1]) of `points`,
 * `out_gwn` and `out_inside` and is evaluated against model seg_model[s].
 * seg_model and seg_offset are HOST arrays (n_seg and n_seg + 1 entries,
 * seg_offset[0] == 0, non-decreasing); points/outputs are device arrays whose
 * row width follows each segment's model dimension: 2D and 3D segments may
 * not share one call (GWN_EINVAL).  Every row's result is bitwise identical
 * to what gwn_query returns for that row alone. */
gwn_status gwn_query_batch(int32_t n_seg, const gwn_handle *seg_model, const int64_t *seg_offset,
                           const double *points, double *out_gwn, uint8_t *out_inside,
                           void *stream);

/* Work counters of one query pass (same traversal, instrumented), summed over
 * all n queries into the device array counters[GWN_NCOUNTERS] (int64,
 * overwritten).  Used to compute algorithmic work.  Order of entries: */
enum {
    GWN_C_NODES = 0,       /* internal nodes tested                        */
    GWN_C_FAR = 1,         /* clusters evaluated by the Taylor expansion   */
    GWN_C_LEAVES = 2,      /* leaves evaluated directly                    */
    GWN_C_LEAF_FAST = 3,   /* 2D: leaves resolved by one chord angle;
                              3D: leaves evaluated by the precomputed rule */
    GWN_C_PIECES = 4,      /* 2D: bisection pieces examined near q;
                              3D: near-field integrand evaluations         */
    GWN_C_ANGLES = 5,      /* 2D: atan2 evaluations; 3D: far-rule nodes    */
    GWN_C_RECLASS = 6,     /* mixed form: queries re-evaluated in FP64     */
    GWN_C_OVERFLOW = 7,    /* queries that hit a stack limit               */
    GWN_NCOUNTERS = 8
};
gwn_status gwn_query_counters(gwn_handle h, const double *points, int64_t n, int64_t *counters,
                              void *stream);

/* Memory accounting: bytes resident on the device for this model, and device
 * scratch bytes per query of a gwn_query / gwn_query_batch launch, without
 * the sort's temporary storage and alignment padding (gwn_query_scratch_bytes
 * gives the exact bytes of a launch). */
gwn_status gwn_model_bytes(gwn_handle h, int64_t *resident, int64_t *per_query_scratch);

/* Host-side inspection of a built model (also for host-only handles).  Copies
 * up to `capacity` items of kind `what` into `out` and stores the total item
 * count in *count.  Kinds and item layouts (all double unless noted):
 *   GWN_I_SUMMARY   1 item of 8 doubles: dim, n_input, n_leaves, n_nodes,
 *                   tree depth, model diagonal, bbox_lo[0], bbox_hi[0]
 *   GWN_I_LEAVES    per leaf (in BVH leaf order): input primitive index, then
 *                   the leaf's homogeneous control points (2D: 4 x (wx,wy,w);
 *                   3D: 16 x (wx,wy,wz,w)) -- 13 or 65 doubles
 *   GWN_I_NODES     per node (DFS order): is_leaf, left, right, centroid[3],
 *                   r (AABB half diagonal), aabb_lo[3], aabb_hi[3]  -- 13 doubles
 *   GWN_I_MOMENTS   per node: centred Cartesian moments (Eq. taylor) about the
 *                   centroid, M0[d], M1[d*d] (M1[j*d+k] = int (x-c)_j n_k),
 *                   M2[d*d*d] (M2[(i*d+j)*d+k] = int (x-c)_i (x-c)_j n_k);
 *                   14 doubles in 2D, 39 in 3D
 *   GWN_I_UNCENTERED per node: the uncentered moments (same layout)
 *   GWN_I_COMPLEX   2D only, per node: the centred complex moments
 *                   m_k = integral over the cluster's chords of (z - c)^k dz,
 *                   k = 0..16, as (re, im) pairs -- 34 doubles (zero for leaves)
 *   GWN_I_MULTIPOLE 3D only, per node: 1/r (r = AABB half diagonal), 0, then
 *                   for l = 1..7, m = 0..l the moments
 *                   N_l^m = -integral n . conj(grad R_l^m(x - c)) dA scaled
 *                   by r^-(l+1), as (re, im) pairs -- 72 doubles.  R_l^m are
 *                   the regular solid harmonics r^l P_l^m(cos t) e^{i m p} /
 *                   (l + m)! (no Condon-Shortley phase); the solid angle of
 *                   the cluster at q is sum_l [I_l^0 N_l^0 + 2 sum_m>0
 *                   Re(I_l^m N_l^m)] with I_l^m(q - c) = (l - m)!
 *                   P_l^m(cos t) e^{i m p} / |q - c|^(l+1).  The order-p far
 *                   field (Eq. taylor) is the truncation l <= p + 1.
 *   GWN_I_LEAF_TRIMS 3D only, per trim curve of every leaf, leaf by leaf (BVH
 *                   leaf order): leaf index, then the curve's homogeneous
 *                   control points (w u, w v, w) x 3 in the leaf's own
 *                   parameter square -- 10 doubles.  A leaf cut from a
 *                   trimmed patch holds its clipped loops (closed, in loop
 *                   order); an untrimmed leaf has none.
 *   GWN_I_FARBETA   per node: the far-field factor the FP64 test uses
 *                   under the handle's current parameters -- beta, or with
 *                   far_tol > 0 the cluster's own beta_c (+inf when no
 *                   factor meets the budget); 0 for 2D leaves (never far
 *                   tested).  1 double.
 */
enum { GWN_I_SUMMARY = 0, GWN_I_LEAVES = 1, GWN_I_NODES = 2, GWN_I_MOMENTS = 3, GWN_I_UNCENTERED = 4,
       GWN_I_COMPLEX = 5, GWN_I_MULTIPOLE = 6, GWN_I_FARBETA = 7, GWN_I_LEAF_TRIMS = 8 };
gwn_status gwn_inspect(gwn_handle h, int32_t what, double *out, int64_t capacity, int64_t *count);

/* Kernel timing.  gwn_profile(1, NULL, NULL) starts recording a pair of HIP
 * events around every launch of the query kernels (on the stream the kernel
 * runs on): the 2D query kernel, and the 3D traversal and near-field
 * kernels, each timed on its own.  gwn_profile(0, &ms, &launches) waits for
 * the recorded events, returns the summed time in milliseconds and the
 * number of timed launches, and stops recording.  gwn_profile_kernel then
 * returns the same sums for one kernel of that set (GWN_K_*; GWN_EINVAL for
 * another value).  Process-wide; not for concurrent use. */
enum { GWN_K_QUERY2D = 0, GWN_K_TRAV3D = 1, GWN_K_NEAR3D = 2 };
gwn_status gwn_profile(int32_t enable, double *total_ms, int64_t *launches);
gwn_status gwn_profile_kernel(int32_t kernel, double *ms, int64_t *launches);

/* Release a handle (host and device memory).  NULL is accepted. */
gwn_status gwn_free(gwn_handle h);

/* Message for the last non-OK status on this thread. */
const char *gwn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GWN_H */
