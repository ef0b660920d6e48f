"""Production parameter sets of the engine's query forms.

FP64 form (2D): the fastest (order, beta, subdivision threshold) whose
maximum |w - w_direct| over the checked query sets (the star loop's 4096
queries; the SVG-like drawing's full 1024^2 grid) stays below 2.5e-7, a 4x
margin on the 1e-6 target.  Measured on one MI355X at the paper's 10%
subdivision threshold (beta at which the bound is met, 1024^2 grid):
    order 2:  beta 64 (17 M q/s)     order 8:  beta 4 (212 M q/s)
    order 12: beta 3.25 (282 M q/s)  (beta 3: 2.7e-7, 313 M q/s)
Subdividing further (Sec. 4.1: split a curve while its box diagonal is at
least max_diag_frac of the model's) shrinks the leaves, so fewer queries
fall inside a leaf's box and need bisection; at order 12, beta 3.25:
    max_diag_frac 0.1: 19000 leaves, 3.72 ms, max |dw| 8.6e-8
                  0.025: 23029 leaves, 3.03 ms, 1.5e-7
                  0.0125: 35687 leaves, 2.68 ms, 2.2e-7  (chosen)
                  0.00625: 65009 leaves, 2.64 ms, 4.2e-7
Error-budgeted far test (far_tol, a factor per cluster from its own
truncation bound instead of one beta for all): order 12, max_diag_frac
0.0125, full 1024^2 grid against the all-direct evaluation:
    uniform beta 3.25:  2.62 ms, max |dw| 2.2e-7, 397 M node visits
    far_tol 3e-9:       2.24 ms, 3.1e-8
    far_tol 1e-8:       2.09 ms, 9.2e-8, 281 M node visits  (chosen)
    far_tol 2e-8:       2.02 ms, 2.0e-7
    far_tol 5e-8:       1.93 ms, 4.8e-7
    far_tol 1e-8 at order 8 / 10: 3.30 / 2.73 ms
The chosen budget is both faster and 2x more accurate than the uniform
factor.  A higher order lets the budget accept clusters sooner; with the
order cap raised to 16 (far_tol 1e-8):
    order 12: 2.03 ms, 281 M node visits, max |dw| 9.2e-8
    order 14: 2.19 ms (runtime-order loop), 226 M
    order 16: 1.92 ms, 197 M node visits, max |dw| 5.7e-8  (chosen)
    order 16 at far_tol 2e-8: 1.84 ms, 1.0e-7
FP64_2D therefore used order 16, far_tol 1e-8 and max_diag_frac 0.0125
(beta 3.25 stays the factor of the uniform test when far_tol is set to 0).
Wave acceptance (wave_accept = 1: a cluster is taken as far only when every
query of the wave passes its test, so the far-field terms run on full waves)
then changes the trade-off; order 16, one 1024^2 call, max |dw| over the
grid against the all-direct evaluation:
    per-query tests, far_tol 1e-8: 1.70 ms, 5.7e-8, 197 M node visits
    wave acceptance, far_tol 1e-8: 1.54 ms, 3.5e-8, 228 M node visits
                             2e-8: 1.51 ms, 5.8e-8  (chosen: the error of
                                   the per-query preset, 12 % faster)
                             4e-8: 1.48 ms, 9.6e-8
                             6e-8: 1.47 ms, 1.2e-7
More nodes are opened (far queries descend with their near neighbours and
take the same or smaller clusters, each within its budget), but the far
terms no longer run on a few lanes at a time.
PAPER_ORDER_2D keeps the paper's default order 2, uniform beta and 10%
threshold with the beta that meets the same bound, and per-query tests.
Mixed form (2D): FP32 far-field pass at beta_mixed = 2 (order 11: beyond
it FP32 rounding dominates), then the FP64 form at order 12 on every query
with |w - 0.5| < 1e-2.  Wave acceptance applies to both passes; on the
1024^2 grid against the all-direct evaluation:
    per-query tests:  1.19 ms, max |dw| 5.0e-4, rms 9.2e-6
    wave acceptance:  0.98 ms, max |dw| 3.8e-4, rms 5.7e-6  (chosen)
            beta_mixed 2.5: 1.16 ms, 1.9e-5;  3.0: 1.38 ms, 3.1e-6
with no containment mismatch outside |w - 1/2| <= 1e-3 in any of them.
"""
from . import gwn as G

FP64_2D = dict(beta=3.25, taylor_order=16, max_diag_frac=0.0125, far_tol=2e-8, wave_accept=1,
               precision=G.GWN_FP64)
PAPER_ORDER_2D = dict(beta=64.0, taylor_order=2, precision=G.GWN_FP64)
MIXED_2D = dict(beta=3.25, beta_mixed=2.0, taylor_order=12, max_diag_frac=0.0125, far_tol=1e-8, wave_accept=1,
                precision=G.GWN_MIXED, reclass_band=1e-2)


# 3D: the order-2 expansion of the paper needs beta = 16 for the same bound
# (its error falls only as beta^-3); the solid-harmonic form of the same
# series at order 6 meets it at beta = 5 with 8x fewer direct leaf
# evaluations.  Maximum |dw| over the checked 3D sets (256 queries of the
# bodies scene, 128 of the CAD assembly, plus the near-surface test sets):
#   order 2, beta 16: 3.9e-7    order 4, beta 8: 2.3e-7
#   order 5, beta 5:  3.0e-7    order 6, beta 5: 1.0e-7  (chosen)
# Subdividing patches further cuts the near-field work, as in 2D (these
# figures predate the subdivision of trimmed patches and of patches with a
# collapsed edge).  Bodies scene, 128^3 grid, order 6, beta 5 (max |dw| on
# 2048 sampled queries against the all-direct evaluation):
#   max_diag_frac 0.1: 4096 leaves, 594 ms, 7.2e-8
#                 0.025: 8570 leaves, 494 ms, 1.0e-7
#                 0.0125: ~29,000 leaves, 410 ms, 8.0e-8  (chosen)
#                 0.00625: 114378 leaves, 371 ms, 9.4e-8 (4x the node sets)
# The near-field tolerance eps_q is 1e-8 per leaf (in units of w): with at
# most 64 near leaves per query their sum stays below 1e-6 even if every
# leaf reached its tolerance (on the checked near-field pairs the errors
# were ~3e-11).
# Error-budgeted far test (far_tol: a factor per cluster from the estimated
# size of its first two omitted harmonic degrees, instead of one beta for
# all), order 6, one 128^3 launch of the bodies scene / 1M queries of the CAD
# assembly, max |dw| on the committed oracle rows:
#   uniform beta 5:  122.7 ms, 7.3e-8   |  1045 ms, 7.4e-8
#   far_tol 1e-7:     98.5 ms, 3.9e-7   |   979 ms, 5.8e-7
#   far_tol 3e-8:    107.3 ms, 1.3e-7
#   far_tol 1e-8:    116.7 ms, 4.8e-8   |  1027 ms, 5.7e-8
#   far_tol 1e-9:    144.5 ms, 8.6e-9   |  1087 ms, 9.8e-9
#   order 4, far_tol 1e-8: 174.1 ms, 1.3e-7
# The budget is faster and more accurate than the uniform factor; the CAD
# assembly's time is nearly all near field, so it gains less.  With wave
# acceptance (as in 2D):
#   far_tol 1e-8: 105.2 ms, 3.4e-8     |  1015 ms, 8.4e-8
#   far_tol 2e-8:  99.7 ms, 6.4e-8     |  1010 ms, 8.3e-8  (chosen)
#   far_tol 3e-8:  96.4 ms, 8.5e-8     |   993 ms, 1.2e-7
# The near-field rule takes a leaf closer than near_ratio x its box
# diagonal; farther leaves use the precomputed node sets.  Against every
# query of a launch at near_ratio 0.5 (0.35 gives the same maximum and
# counts), max |dw| on the CAD assembly / bodies scene:
#   near_ratio 0.25 (library default): 1.1e-6 / 2.5e-7, 939 / 92 ms
#              0.28:                   2.6e-7 / 1.2e-8, 999 / 98 ms  (chosen)
#              0.30:                   1.1e-7 / 1.2e-8
#              0.20:                   9.2e-6 (against 0.25) -- too close
FP64_3D = dict(beta=5.0, taylor_order=6, max_diag_frac=0.0125, eps_q=1e-8, far_tol=2e-8, wave_accept=1,
               near_ratio=0.28, precision=G.GWN_FP64)
# A reached leaf that passes the far test itself takes its own expansion
# (leaf_far, the default): on the checked sets this halves the node-set work
# per query (CAD assembly: 113k -> 53k integrand nodes) at the same error.
# The paper's setting evaluates every reached leaf directly (Alg. 1).
PAPER_ORDER_3D = dict(beta=16.0, taylor_order=2, leaf_far=0, eps_q=1e-8, precision=G.GWN_FP64)
# Mixed form (3D), per-query tests against wave acceptance in both passes,
# full grid against the FP64 preset (bodies scene / CAD assembly):
#   per-query tests:  87.8 ms, rms 1.1e-6  |  968 ms, rms 1.9e-6  (chosen)
#   wave acceptance:  86.9 ms, rms 6.6e-7  |  970 ms, rms 1.2e-6
# The near field dominates both totals; the FP32 traversal pass itself is
# slower with wave acceptance (17.8 -> 18.3 ms / 92 -> 98 ms traced), so
# the preset keeps per-query tests.
MIXED_3D = dict(beta=5.0, beta_mixed=3.0, taylor_order=6, max_diag_frac=0.0125, eps_q=1e-8, far_tol=1e-8,
                near_ratio=0.28,
                precision=G.GWN_MIXED,
                reclass_band=1e-2)


def params(preset: dict, **extra) -> "G.gwn_params":
    p = G.gwn_default_params()
    for k, v in {**preset, **extra}.items():
        setattr(p, k, v)
    return p
