/*
 * A plain C client of the engine's C ABI (include/gwn.h): the unit circle,
 * given once as four rational quadratic arcs and once as a clamped quadratic
 * NURBS curve (Bezier extraction through gwn_nurbs2d_extract), queried on the
 * GPU at points inside and outside it.  The winding number is 1 inside and 0
 * outside; the program checks both models against that and exits with 0 when
 * every value is within the FP64 form's 1e-6 and every containment flag is
 * right.
 *
 * Build (the package's build step does this):
 *   gcc -std=c99 -D__HIP_PLATFORM_AMD__ -I include -I /opt/rocm/include circle.c
 *       -L <package> -lgwn -L /opt/rocm/lib -lamdhip64 -lm -o circle
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "gwn.h"

#define NQ 64

static int fail_msg(const char *what)
{
    fprintf(stderr, "circle: %s: %s\n", what, gwn_last_error());
    return 1;
}

/* query model h at the NQ points of q (host), compare with the exact values */
static int check(gwn_handle h, const double *q, const double *expect, const char *name)
{
    double *d_q = NULL, *d_w = NULL;
    uint8_t *d_in = NULL;
    double w[NQ];
    uint8_t in[NQ];
    if (hipMalloc((void **)&d_q, sizeof(double) * 2 * NQ) != hipSuccess ||
        hipMalloc((void **)&d_w, sizeof(double) * NQ) != hipSuccess ||
        hipMalloc((void **)&d_in, NQ) != hipSuccess) {
        fprintf(stderr, "circle: hipMalloc failed\n");
        return 1;
    }
    int bad = 0;
    if (hipMemcpy(d_q, q, sizeof(double) * 2 * NQ, hipMemcpyHostToDevice) != hipSuccess) bad = 1;
    if (!bad && gwn_query(h, d_q, NQ, d_w, d_in, NULL) != GWN_OK) bad = fail_msg("gwn_query");
    if (!bad && (hipMemcpy(w, d_w, sizeof w, hipMemcpyDeviceToHost) != hipSuccess ||
                 hipMemcpy(in, d_in, sizeof in, hipMemcpyDeviceToHost) != hipSuccess))
        bad = 1;
    double err = 0.0;
    int flags = 0;
    for (int i = 0; i < NQ && !bad; ++i) {
        err = fmax(err, fabs(w[i] - expect[i]));
        flags += in[i] != (expect[i] >= 0.5);
    }
    hipFree(d_q);
    hipFree(d_w);
    hipFree(d_in);
    if (bad) return 1;
    printf("%s: max |w - exact| = %.3e, wrong containment flags = %d\n", name, err, flags);
    return !(err <= 1e-6 && flags == 0);
}

int main(void)
{
    const double s = sqrt(0.5);
    /* four quarter arcs, counter-clockwise */
    const double xy[4][3][2] = {{{1, 0}, {1, 1}, {0, 1}},
                                {{0, 1}, {-1, 1}, {-1, 0}},
                                {{-1, 0}, {-1, -1}, {0, -1}},
                                {{0, -1}, {1, -1}, {1, 0}}};
    double cp_xy[24], cp_w[12];
    int32_t degree[4];
    int64_t cp_offset[5];
    for (int c = 0; c < 4; ++c) {
        degree[c] = 2;
        cp_offset[c] = 3 * c;
        for (int k = 0; k < 3; ++k) {
            cp_xy[2 * (3 * c + k)] = xy[c][k][0];
            cp_xy[2 * (3 * c + k) + 1] = xy[c][k][1];
            cp_w[3 * c + k] = k == 1 ? s : 1.0;
        }
    }
    cp_offset[4] = 12;
    gwn_curves2d arcs = {4, degree, cp_offset, cp_xy, cp_w};

    /* the same circle as one clamped quadratic NURBS curve of 9 points */
    const double nxy[18] = {1, 0, 1, 1, 0, 1, -1, 1, -1, 0, -1, -1, 0, -1, 1, -1, 1, 0};
    const double nw[9] = {1, s, 1, s, 1, s, 1, s, 1};
    const double knots[12] = {0, 0, 0, 0.25, 0.25, 0.5, 0.5, 0.75, 0.75, 1, 1, 1};
    const int32_t ndeg = 2;
    const int64_t ncp[2] = {0, 9}, nkn[2] = {0, 12};
    gwn_nurbs2d nurbs = {1, &ndeg, ncp, nxy, nw, nkn, knots};
    int64_t nseg = 0, npt = 0;
    if (gwn_nurbs2d_extract(&nurbs, &nseg, &npt, NULL, NULL, NULL, NULL) != GWN_OK) return fail_msg("extract");
    int32_t *sdeg = malloc(sizeof(int32_t) * nseg);
    int64_t *soff = malloc(sizeof(int64_t) * (nseg + 1));
    double *sxy = malloc(sizeof(double) * 2 * npt), *sw = malloc(sizeof(double) * npt);
    if (gwn_nurbs2d_extract(&nurbs, &nseg, &npt, sdeg, soff, sxy, sw) != GWN_OK) return fail_msg("extract");
    gwn_curves2d segments = {nseg, sdeg, soff, sxy, sw};

    /* queries on two rings, inside (r = 0.5) and outside (r = 1.5) */
    double q[2 * NQ], expect[NQ];
    for (int i = 0; i < NQ; ++i) {
        const double r = i % 2 ? 1.5 : 0.5, t = 8.0 * atan(1.0) * i / NQ;
        q[2 * i] = r * cos(t);
        q[2 * i + 1] = r * sin(t);
        expect[i] = r < 1.0 ? 1.0 : 0.0;
    }

    gwn_params p;
    gwn_default_params(&p);
    p.beta = 3.25;
    p.taylor_order = 12;
    gwn_handle h1 = NULL, h2 = NULL;
    if (gwn_build2d(&arcs, &p, &h1) != GWN_OK) return fail_msg("gwn_build2d (arcs)");
    if (gwn_build2d(&segments, &p, &h2) != GWN_OK) return fail_msg("gwn_build2d (NURBS)");
    int rc = check(h1, q, expect, "rational arcs");
    rc |= check(h2, q, expect, "NURBS circle");
    gwn_free(h1);
    gwn_free(h2);
    free(sdeg);
    free(soff);
    free(sxy);
    free(sw);
    printf(rc ? "circle: FAILED\n" : "circle: ok\n");
    return rc;
}
