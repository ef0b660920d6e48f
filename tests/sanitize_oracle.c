/* The oracle under AddressSanitizer and UBSan (test infrastructure, compiled
 * and run by tests/test_sanitize_host.py with gcc, single-threaded).  Reads
 * the same case file as sanitize_host.cpp followed by two query arrays (2D,
 * 3D), evaluates the oracle at them and prints one value per line. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_gwn2d(int64_t n, const int32_t *degree, const int64_t *cp_offset, const double *cp_xy,
                 const double *cp_w, int64_t n_q, const double *q, double *out, double eps_on, int nthreads);
int oracle_gwn3d(int64_t n, const double *cp_xyz, const double *cp_w, const int64_t *trim_offset,
                 const int32_t *trim_degree, const int64_t *trim_cp_offset, const double *trim_cp_uv,
                 const double *trim_cp_w, int64_t n_q, const double *q, double *out, double eps_on,
                 int nthreads);
long long oracle_last_unconverged(void);

static void *next(FILE *f, size_t elem, int64_t *count)
{
    int64_t n = 0;
    if (fread(&n, sizeof n, 1, f) != 1 || n < 0) {
        fprintf(stderr, "truncated case file\n");
        exit(2);
    }
    void *p = malloc(n ? (size_t)n * elem : 1);
    if (n && fread(p, elem, (size_t)n, f) != (size_t)n) {
        fprintf(stderr, "truncated case file\n");
        exit(2);
    }
    if (count) *count = n;
    return p;
}

int main(int argc, char **argv)
{
    if (argc != 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n2, n3w, nq2, nq3, tmp;
    int32_t *deg = next(f, 4, &n2);
    int64_t *off = next(f, 8, NULL);
    double *xy = next(f, 8, NULL), *w = next(f, 8, NULL);
    for (int k = 0; k < 6; ++k) free(next(f, k == 0 ? 4 : 8, &tmp)); /* NURBS arrays: not the oracle's input */
    double *cp = next(f, 8, NULL), *cw = next(f, 8, &n3w);
    int64_t *toff = next(f, 8, NULL);
    int32_t *tdeg = next(f, 4, NULL);
    int64_t *tcoff = next(f, 8, NULL);
    double *tuv = next(f, 8, NULL), *tw = next(f, 8, NULL);
    double *q2 = next(f, 8, &nq2), *q3 = next(f, 8, &nq3);
    fclose(f);
    double *o2 = malloc(sizeof(double) * (size_t)(nq2 / 2 + 1)), *o3 = malloc(sizeof(double) * (size_t)(nq3 / 3 + 1));
    int r = oracle_gwn2d(n2, deg, off, xy, w, nq2 / 2, q2, o2, 1e-12, 1);
    if (r) return 3;
    printf("unconverged2d %lld\n", oracle_last_unconverged());
    r = oracle_gwn3d(n3w / 16, cp, cw, toff, tdeg, tcoff, tuv, tw, nq3 / 3, q3, o3, 1e-12, 1);
    if (r) return 3;
    printf("unconverged3d %lld\n", oracle_last_unconverged());
    for (int64_t i = 0; i < nq2 / 2; ++i) printf("%.17g\n", o2[i]);
    for (int64_t i = 0; i < nq3 / 3; ++i) printf("%.17g\n", o3[i]);
    free(deg); free(off); free(xy); free(w); free(cp); free(cw); free(toff); free(tdeg); free(tcoff);
    free(tuv); free(tw); free(q2); free(q3); free(o2); free(o3);
    return 0;
}
