/* Driver for the address/undefined-behaviour sanitizer build of the CPU
 * oracle (oracle/oracle.c): calls every oracle function on small seeded
 * inputs, including the edge cases the library must also handle (one body,
 * an empty block, out-of-range rows, nb_cap 0 with no list, overflowing
 * lists, rows with no neighbours), and checks that every output is finite
 * and every list entry is a valid body index.  Exit status 0 = clean. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void or_predict(int64_t n, double t, const double *x, const double *v, const double *a,
                const double *jk, const double *t0, double *xp, double *vp);
void or_regular(int64_t n, const double *xp, const double *vp, const double *m, int32_t n_i,
                const int32_t *i_block, const double *rs2, int32_t nb_cap, double *acc,
                double *jerk, int32_t *nb_count, int32_t *nb_list, int32_t *overflow,
                int32_t *bad);
void or_irregular(int64_t n, const double *xp, const double *vp, const double *m, int32_t n_i,
                  const int32_t *i_block, int32_t nb_cap, const int32_t *nb_count,
                  const int32_t *nb_list, double *acc, double *jerk);
double or_potential(int64_t n, const double *x, const double *m, double *phi);
void or_potential_rows(int64_t n, const double *x, const double *m, int64_t n_r,
                       const int32_t *rows, double *phi);
void or_adjoint(int64_t n, const double *xp, const double *vp, const double *m,
                const double *xm, int32_t n_i, const int32_t *i_block, const double *rs2,
                const double *w_a, const double *w_j, double *gx, double *gv, double *gm);
double or_local_loss(int64_t n, const double *xp, const double *vp, const double *m,
                     const double *xm, int32_t n_i, const int32_t *i_block, const double *rs2,
                     const double *w_a, const double *w_j, int64_t body);
void or_hermite_correct(int64_t n, const double *h, const double *x0, const double *v0,
                        const double *a0, const double *j0, const double *a1,
                        const double *j1, double *x1, double *v1, double *a2, double *a3);

static uint64_t g_state = 0x243F6A8885A308D3ull;
static double urand(void)
{
    g_state ^= g_state >> 12;
    g_state ^= g_state << 25;
    g_state ^= g_state >> 27;
    return (double)((g_state * 2685821657736338717ull) >> 11) * 0x1p-53;
}

static int g_fail = 0;
static void check_finite(const char *what, const double *p, int64_t k)
{
    for (int64_t q = 0; q < k; ++q)
        if (!isfinite(p[q])) {
            fprintf(stderr, "%s[%lld] not finite\n", what, (long long)q);
            g_fail = 1;
            return;
        }
}

static double *dalloc(int64_t k)
{
    double *p = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
    for (int64_t q = 0; q < k; ++q) p[q] = 2.0 * urand() - 1.0;
    return p;
}

static void run(int64_t n, int32_t n_i, int32_t cap)
{
    double *x = dalloc(3 * n), *v = dalloc(3 * n), *a = dalloc(3 * n), *jk = dalloc(3 * n);
    double *t0 = dalloc(n), *m = dalloc(n), *xp = dalloc(3 * n), *vp = dalloc(3 * n);
    for (int64_t j = 0; j < n; ++j) {
        t0[j] = 0.0;
        m[j] = 0.5 + urand();
    }
    or_predict(n, 0x1p-8, x, v, a, jk, t0, xp, vp);
    check_finite("xp", xp, 3 * n);
    check_finite("vp", vp, 3 * n);

    int32_t *ib = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_i > 0 ? n_i : 1));
    double *rs2 = dalloc(n_i);
    for (int32_t b = 0; b < n_i; ++b) {
        ib[b] = (int32_t)(urand() * (double)n);
        rs2[b] = b % 5 == 0 ? 0.0 : 0.5 * urand();   /* some rows without neighbours */
    }
    double *acc = dalloc(3 * n_i), *jerk = dalloc(3 * n_i);
    int32_t *cnt = (int32_t *)calloc((size_t)(n_i > 0 ? n_i : 1), sizeof(int32_t));
    int32_t *lst = cap > 0 ? (int32_t *)calloc((size_t)n_i * (size_t)cap + 1, sizeof(int32_t))
                           : NULL;
    int32_t ovf = -1, bad = -1;
    or_regular(n, xp, vp, m, n_i, ib, rs2, cap, acc, jerk, cnt, lst, &ovf, &bad);
    check_finite("acc", acc, 3 * n_i);
    check_finite("jerk", jerk, 3 * n_i);
    for (int32_t b = 0; b < n_i; ++b) {
        const int32_t k = cnt[b] < cap ? cnt[b] : cap;
        for (int32_t q = 0; q < k; ++q)
            if (lst[(int64_t)b * cap + q] < 0 || lst[(int64_t)b * cap + q] >= n) g_fail = 1;
    }
    if (ovf < 0 || bad != 0) g_fail = 1;
    or_irregular(n, xp, vp, m, n_i, ib, cap, cnt, lst, acc, jerk);
    check_finite("irr acc", acc, 3 * n_i);

    /* a row outside [0, n) is zeroed and flagged */
    if (n_i > 1) {
        ib[1] = (int32_t)n;
        or_regular(n, xp, vp, m, n_i, ib, rs2, cap, acc, jerk, cnt, lst, &ovf, &bad);
        if (bad != 1 || cnt[1] != 0 || acc[1] != 0.0) g_fail = 1;
        ib[1] = 0;
    }

    double *phi = dalloc(n);
    const double e = or_potential(n, xp, m, phi);
    if (!isfinite(e)) g_fail = 1;
    or_potential_rows(n, xp, m, n_i, ib, phi);

    double *wa = dalloc(3 * n_i), *wj = dalloc(3 * n_i);
    double *gx = dalloc(3 * n), *gv = dalloc(3 * n), *gm = dalloc(n);
    or_adjoint(n, xp, vp, m, xp, n_i, ib, rs2, wa, wj, gx, gv, gm);
    check_finite("gx", gx, 3 * n);
    check_finite("gv", gv, 3 * n);
    check_finite("gm", gm, n);
    if (n > 0 && !isfinite(or_local_loss(n, xp, vp, m, xp, n_i, ib, rs2, wa, wj, n - 1)))
        g_fail = 1;

    double *h = dalloc(n);
    for (int64_t j = 0; j < n; ++j) h[j] = 0x1p-6;
    double *x1 = dalloc(3 * n), *v1 = dalloc(3 * n), *a2 = dalloc(3 * n), *a3 = dalloc(3 * n);
    or_hermite_correct(n, h, x, v, a, jk, a, jk, x1, v1, a2, a3);
    check_finite("x1", x1, 3 * n);

    free(x); free(v); free(a); free(jk); free(t0); free(m); free(xp); free(vp);
    free(ib); free(rs2); free(acc); free(jerk); free(cnt); free(lst); free(phi);
    free(wa); free(wj); free(gx); free(gv); free(gm);
    free(h); free(x1); free(v1); free(a2); free(a3);
}

int main(void)
{
    run(1, 1, 4);        /* a single body: no pairs at all */
    run(2, 2, 1);
    run(37, 0, 8);       /* empty block */
    run(37, 23, 0);      /* no list storage */
    run(37, 23, 2);      /* lists overflow */
    run(257, 64, 40);
    if (g_fail) fprintf(stderr, "oracle sanitizer driver: FAILED\n");
    else printf("oracle sanitizer driver: ok\n");
    return g_fail;
}
