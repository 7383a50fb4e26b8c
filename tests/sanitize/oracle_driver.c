/* Runs the oracle's entry points on small fields under AddressSanitizer and UBSan
 * (built without OpenMP): a linear field with a closed form, a null region, a NaN,
 * seeds outside the box, maps with one-sided and mixed-face stencils, a 3-D map with
 * rotated S0 and the sampled-point entry points. Exits nonzero on a wrong value. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fq_oracle.h"

static int fails = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            fails++;                                                              \
        }                                                                         \
    } while (0)

typedef struct {
    orc_field f;
    double *buf;
} holder;

/* B = M r + c on an n^3 grid of [0,1]^3 */
static holder linear(int n, const double M[3][3], const double c[3])
{
    holder h;
    memset(&h, 0, sizeof h);
    size_t nn = (size_t)n * n * n;
    h.buf = (double *)calloc(6 * nn, sizeof(double));
    for (int a = 0; a < 3; a++) {
        h.f.n[a] = n;
        h.f.spacing[a] = 1.0 / (n - 1);
        h.f.b[a] = h.buf + a * nn;
        h.f.j[a] = h.buf + (3 + a) * nn;
    }
    for (int k = 0; k < n; k++)
        for (int j = 0; j < n; j++)
            for (int i = 0; i < n; i++) {
                double r[3] = {i / (n - 1.0), j / (n - 1.0), k / (n - 1.0)};
                size_t q = ((size_t)k * n + j) * n + i;
                for (int a = 0; a < 3; a++)
                    ((double *)h.f.b[a])[q] = M[a][0] * r[0] + M[a][1] * r[1] + M[a][2] * r[2] + c[a];
            }
    orc_curl(&h.f, (double *)h.f.j[0], (double *)h.f.j[1], (double *)h.f.j[2]);
    return h;
}

int main(void)
{
    orc_opts o;
    orc_default_opts(&o);
    /* sheared field: Q = 2 + s^2 */
    const double s = 0.5;
    const double Ms[3][3] = {{0, s, 0}, {0, 0, 0}, {0, 0, 0}};
    const double cs[3] = {-s * 0.5, 0, 1};
    holder h = linear(9, Ms, cs);
    int nu = 7, nv = 6;
    double org[3] = {0.3, 0.3, 0.0}, u[3] = {1, 0, 0}, v[3] = {0, 1, 0};
    size_t np = (size_t)nu * nv;
    double *q = malloc(np * sizeof *q), *tw = malloc(np * sizeof *tw), *len = malloc(np * sizeof *len);
    uint16_t *st = malloc(np * sizeof *st);
    CHECK(orc_q2d(&h.f, org, u, v, nu, nv, 0.01, 0.01, &o, q, tw, len, st, NULL) == 0);
    CHECK(fabs(q[nu + 1] - (2 + s * s)) < 1e-8);
    /* a map larger than the box: seeds outside, one-sided and mixed stencils */
    double org2[3] = {0.7, 0.2, 0.0};
    CHECK(orc_q2d(&h.f, org2, u, v, nu, nv, 0.1, 0.1, &o, q, tw, len, st, NULL) == 0);
    int outside = 0;
    for (size_t p = 0; p < np; p++) outside += (st[p] & ORC_OUTSIDE) != 0;
    CHECK(outside > 0);
    /* sampled points, including the last one, and one out of range */
    int64_t pts[3] = {0, (int64_t)np - 1, 5};
    CHECK(orc_q2d_points(&h.f, org, u, v, nu, nv, 0.01, 0.01, pts, 3, &o, q, tw, len, st, NULL) == 0);
    int64_t badpt[1] = {(int64_t)np};
    CHECK(orc_q2d_points(&h.f, org, u, v, nu, nv, 0.01, 0.01, badpt, 1, &o, q, tw, len, st, NULL) != 0);
    /* 3-D map with rotated S0: B = (1, 0.3, s (y - 0.4)) */
    const double Mr[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, s, 0}};
    const double cr[3] = {1.0, 0.3, -s * 0.4};
    holder hr = linear(9, Mr, cr);
    double vo[3] = {0.4, 0.35, 0.45}, vs[3] = {0.01, 0.01, 0.05};
    int64_t nvox[3] = {4, 11, 3};
    size_t nvx = 4 * 11 * 3;
    double *q3 = malloc(nvx * sizeof *q3), *t3 = malloc(nvx * sizeof *t3), *l3 = malloc(nvx * sizeof *l3);
    uint16_t *s3 = malloc(nvx * sizeof *s3);
    CHECK(orc_q3d(&hr.f, vo, vs, nvox, &o, q3, t3, l3, s3, NULL) == 0);
    int rot = 0;
    for (size_t p = 0; p < nvx; p++) rot += (s3[p] & ORC_ROTATED) != 0;
    CHECK(rot > 0);
    int64_t p3[2] = {0, (int64_t)nvx - 1};
    CHECK(orc_q3d_points(&hr.f, vo, vs, nvox, p3, 2, &o, q3, t3, l3, s3, NULL) == 0);
    /* failure paths: NaN, null region, step budget */
    double seeds[6] = {0.5, 0.5, 0.1, 1.5, 0.5, 0.5};
    double eb[6], ef[6], bnb[2], bnf[2], bn0[2], lt[2], ll[2];
    int8_t fb[2], ff[2];
    uint16_t ls[2];
    int64_t ns[2];
    orc_lines L = {eb, ef, fb, ff, bnb, bnf, bn0, lt, ll, ls, ns};
    ((double *)h.f.b[2])[4 * 81 + 4 * 9 + 4] = NAN;
    CHECK(orc_trace(&h.f, seeds, 2, NULL, &o, &L) == 0);
    CHECK((ls[0] & ORC_NONFINITE) && (ls[1] & ORC_OUTSIDE));
    for (int a = 0; a < 3; a++)
        for (size_t k = 5 * 81; k < 9 * 81; k++) ((double *)h.f.b[a])[k] = 0.0;
    ((double *)h.f.b[2])[4 * 81 + 4 * 9 + 4] = 1.0;
    CHECK(orc_trace(&h.f, seeds, 1, NULL, &o, &L) == 0);
    CHECK(ls[0] & ORC_NULLB);
    o.max_steps = 1;
    CHECK(orc_trace(&hr.f, seeds, 1, NULL, &o, &L) == 0);
    CHECK(ls[0] & ORC_MAXSTEPS);
    free(q), free(tw), free(len), free(st), free(q3), free(t3), free(l3), free(s3);
    free(h.buf), free(hr.buf);
    printf("oracle: %d failures\n", fails);
    return fails ? 1 : 0;
}
