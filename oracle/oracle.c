/*
 * oracle.c -- plain, slow FP64 reference for the Ahmad-Cohen regular-force step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the HIP library: it is written from the paper's
 * definitions and textbook Hermite formulas.
 *
 * What is computed (Wang et al. 2015, NBODY6++GPU):
 *   - the Hermite predictor of all bodies to the block time (section 3.3.3;
 *     Table 1 "Pred."; force and first derivative kept from the last step,
 *     section 2);
 *   - the regular force: for each active body i, the sum of the Newtonian pair
 *     accelerations from every body OUTSIDE i's neighbour radius, plus its first
 *     time derivative (jerk), with the neighbour list (bodies inside the radius)
 *     collected in the same pass (section 2 on the Ahmad-Cohen split; section
 *     3.2.1; Table 1 "Reg.");
 *   - the irregular force over the neighbour list (section 2), the potential
 *     energy (section 3.2.1, section 3.3.2), and the hand-derived adjoint of the
 *     regular force (no counterpart in the paper).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - G = 1, no softening.  The self pair j == i is excluded by index.
 *   - "outside the neighbour radius": j is a neighbour iff r2f < rs2f strictly,
 *     with the canonical FP32 test
 *         fx = (float)(x_j - x_i) (FP64 difference, then round), same for y, z;
 *         r2f = fmaf(fz, fz, fmaf(fy, fy, fx * fx));  rs2f = (float) rs2.
 *   - neighbour lists are in ascending j; a list longer than nb_cap keeps its
 *     first nb_cap entries, nb_count holds the true count, *overflow is set.
 *   - sums run over ascending j with Neumaier-compensated FP64 accumulation.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared (no
 * -ffast-math: every operation is IEEE round-to-nearest and nothing is fused
 * except where fma()/fmaf() is written out).
 *
 * Layout: positions, velocities and their derivatives are FP64 planes [3][n]
 * (component k of body j at index k*n + j); per-row outputs are [3][n_i].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Neumaier compensated sum                                                   */
/* ------------------------------------------------------------------------- */
typedef struct { double s, c; } csum;

static inline void cs_add(csum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static inline double cs_get(const csum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------- */
/* Hermite predictor (section 3.3.3, all-particle prediction for the regular  */
/* force): 3rd-order Taylor series in x, 2nd-order in v, Horner form in dt.   */
/*   xp = x + v dt + a dt^2/2 + j dt^3/6,   vp = v + a dt + j dt^2/2           */
/* The 1/6 factor is the FP64 number nearest to 1/6, applied by multiply.     */
/* ------------------------------------------------------------------------- */
static const double ONE_SIXTH = 0x1.5555555555555p-3;

void or_predict(int64_t n, double t, const double *x, const double *v,
                const double *a, const double *jk, const double *t0,
                double *xp, double *vp)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double dt = t - t0[i];
        for (int k = 0; k < 3; ++k) {
            int64_t q = (int64_t)k * n + i;
            double c3 = jk[q] * ONE_SIXTH;
            double c2 = a[q] * 0.5;
            xp[q] = fma(dt, fma(dt, fma(dt, c3, c2), v[q]), x[q]);
            vp[q] = fma(dt, fma(dt, jk[q] * 0.5, a[q]), v[q]);
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Canonical neighbour test (inside the neighbour radius, section 2).         */
/* ------------------------------------------------------------------------- */
static inline int inside(double dx, double dy, double dz, float rs2f)
{
    float fx = (float)dx, fy = (float)dy, fz = (float)dz;
    float r2f = fmaf(fz, fz, fmaf(fy, fy, fx * fx));
    return r2f < rs2f;
}

/* Newtonian pair acceleration m r / |r|^3 and its time derivative
 * m [ u / |r|^3 - 3 (r.u) r / |r|^5 ]  (G = 1), r = x_j - x_i, u = v_j - v_i.
 * Plain textbook form: r3 = r2 * sqrt(r2), divisions written out.           */
static inline void pair_terms(double m, const double r[3], const double u[3],
                              double ta[3], double tj[3])
{
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double r3 = r2 * sqrt(r2);
    double s = r[0] * u[0] + r[1] * u[1] + r[2] * u[2];
    for (int k = 0; k < 3; ++k) {
        ta[k] = m * r[k] / r3;
        tj[k] = m * (u[k] / r3 - 3.0 * s * r[k] / (r3 * r2));
    }
}

/* ------------------------------------------------------------------------- */
/* Regular force + jerk + neighbour lists for an active block.               */
/* Row b is body i = i_block[b] with squared neighbour radius rs2[b].         */
/* Out-of-range i gives a zero row with nb_count = 0 and *bad = 1.            */
/* ------------------------------------------------------------------------- */
void or_regular(int64_t n, const double *xp, const double *vp, const double *m,
                int32_t n_i, const int32_t *i_block, const double *rs2, int32_t nb_cap,
                double *acc, double *jerk, int32_t *nb_count, int32_t *nb_list,
                int32_t *overflow, int32_t *bad)
{
    int32_t ovf = 0, badf = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(| : ovf, badf)
    for (int32_t b = 0; b < n_i; ++b) {
        int64_t i = i_block[b];
        if (i < 0 || i >= n) {
            for (int k = 0; k < 3; ++k)
                acc[(int64_t)k * n_i + b] = jerk[(int64_t)k * n_i + b] = 0.0;
            nb_count[b] = 0;
            badf = 1;
            continue;
        }
        float rs2f = (float)rs2[b];
        csum A[3] = {{0, 0}, {0, 0}, {0, 0}}, J[3] = {{0, 0}, {0, 0}, {0, 0}};
        int32_t cnt = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            double r[3], u[3];
            for (int k = 0; k < 3; ++k) {
                r[k] = xp[(int64_t)k * n + j] - xp[(int64_t)k * n + i];
                u[k] = vp[(int64_t)k * n + j] - vp[(int64_t)k * n + i];
            }
            if (inside(r[0], r[1], r[2], rs2f)) {
                if (cnt < nb_cap)
                    nb_list[(int64_t)b * nb_cap + cnt] = (int32_t)j;
                ++cnt;
                continue;
            }
            double ta[3], tj[3];
            pair_terms(m[j], r, u, ta, tj);
            for (int k = 0; k < 3; ++k) {
                cs_add(&A[k], ta[k]);
                cs_add(&J[k], tj[k]);
            }
        }
        for (int k = 0; k < 3; ++k) {
            acc[(int64_t)k * n_i + b] = cs_get(&A[k]);
            jerk[(int64_t)k * n_i + b] = cs_get(&J[k]);
        }
        nb_count[b] = cnt;
        if (cnt > nb_cap)
            ovf = 1;
    }
    *overflow = ovf;
    if (bad)
        *bad = badf;
}

/* ------------------------------------------------------------------------- */
/* Irregular force + jerk: the same pair terms over an explicit neighbour     */
/* list (section 2: the irregular force accumulates only neighbour forces).   */
/* Rows whose list overflowed (count > cap) are computed from the first cap.  */
/* ------------------------------------------------------------------------- */
void or_irregular(int64_t n, const double *xp, const double *vp, const double *m,
                  int32_t n_i, const int32_t *i_block, int32_t nb_cap,
                  const int32_t *nb_count, const int32_t *nb_list,
                  double *acc, double *jerk)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t b = 0; b < n_i; ++b) {
        int64_t i = i_block[b];
        csum A[3] = {{0, 0}, {0, 0}, {0, 0}}, J[3] = {{0, 0}, {0, 0}, {0, 0}};
        int32_t cnt = nb_count[b] < nb_cap ? nb_count[b] : nb_cap;
        for (int32_t q = 0; q < cnt; ++q) {
            int64_t j = nb_list[(int64_t)b * nb_cap + q];
            double r[3], u[3], ta[3], tj[3];
            for (int k = 0; k < 3; ++k) {
                r[k] = xp[(int64_t)k * n + j] - xp[(int64_t)k * n + i];
                u[k] = vp[(int64_t)k * n + j] - vp[(int64_t)k * n + i];
            }
            pair_terms(m[j], r, u, ta, tj);
            for (int k = 0; k < 3; ++k) {
                cs_add(&A[k], ta[k]);
                cs_add(&J[k], tj[k]);
            }
        }
        for (int k = 0; k < 3; ++k) {
            acc[(int64_t)k * n_i + b] = cs_get(&A[k]);
            jerk[(int64_t)k * n_i + b] = cs_get(&J[k]);
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Potential: phi_i = -sum_{j != i} m_j / |x_j - x_i| for every body, and the */
/* total potential energy U = 1/2 sum_i m_i phi_i (section 3.2.1; used for    */
/* the energy check and the scaling to N-body units, section 3.3.2).          */
/* ------------------------------------------------------------------------- */
double or_potential(int64_t n, const double *x, const double *m, double *phi)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        csum p = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            double dx = x[j] - x[i], dy = x[n + j] - x[n + i], dz = x[2 * n + j] - x[2 * n + i];
            cs_add(&p, -m[j] / sqrt(dx * dx + dy * dy + dz * dz));
        }
        phi[i] = cs_get(&p);
    }
    csum u = {0, 0};
    for (int64_t i = 0; i < n; ++i)
        cs_add(&u, 0.5 * m[i] * phi[i]);
    return cs_get(&u);
}

/* Potential at selected bodies only: phi_r = -sum_{j != rows[r]} m_j / |x_j -
 * x_i|, i = rows[r], the same sum as or_potential for one body. */
void or_potential_rows(int64_t n, const double *x, const double *m, int64_t n_r,
                       const int32_t *rows, double *phi)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < n_r; ++r) {
        const int64_t i = rows[r];
        csum p = {0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i)
                continue;
            double dx = x[j] - x[i], dy = x[n + j] - x[n + i], dz = x[2 * n + j] - x[2 * n + i];
            cs_add(&p, -m[j] / sqrt(dx * dx + dy * dy + dz * dz));
        }
        phi[r] = cs_get(&p);
    }
}

/* ------------------------------------------------------------------------- */
/* Adjoint of the regular force (no counterpart in the paper).                */
/*   L = sum_b  w_a[:,b] . acc_b  +  w_j[:,b] . jerk_b                          */
/* Membership is frozen at its forward value (the canonical test above).      */
/* For a regular pair (b, j), with A = w_a[:,b], B = w_j[:,b], r, u as above, */
/* R3 = |r|^-3, R5 = |r|^-5, R7 = |r|^-7, s = r.u, the pair loss is            */
/*   l = m_j [ (A.r) R3 + (B.u) R3 - 3 s (B.r) R5 ]                            */
/* with                                                                      */
/*   dl/dm_j = (A.r) R3 + (B.u) R3 - 3 s (B.r) R5                              */
/*   dl/dr   = m_j [ A R3 - 3 (A.r) r R5 - 3 (B.u) r R5 - 3 (B.r) u R5          */
/*                   - 3 s B R5 + 15 s (B.r) r R7 ]                           */
/*   dl/du   = m_j [ B R3 - 3 (B.r) r R5 ]                                     */
/* and r = x_j - x_i, u = v_j - v_i give +dl/dr to body j, -dl/dr to body i.  */
/* Written as two plain loops so that every output element is the sum of its */
/* own terms in a fixed order: per row (the "-" terms onto i) and per body    */
/* (the "+" terms onto j, over all rows b).                                  */
/* ------------------------------------------------------------------------- */
static inline void pair_grad(double mj, const double A[3], const double B[3],
                             const double r[3], const double u[3],
                             double gr[3], double gu[3], double *gm)
{
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double rr = sqrt(r2);
    double R3 = 1.0 / (r2 * rr);
    double R5 = R3 / r2;
    double R7 = R5 / r2;
    double s = r[0] * u[0] + r[1] * u[1] + r[2] * u[2];
    double Ar = A[0] * r[0] + A[1] * r[1] + A[2] * r[2];
    double Br = B[0] * r[0] + B[1] * r[1] + B[2] * r[2];
    double Bu = B[0] * u[0] + B[1] * u[1] + B[2] * u[2];
    *gm = Ar * R3 + Bu * R3 - 3.0 * s * Br * R5;
    for (int k = 0; k < 3; ++k) {
        gr[k] = mj * (A[k] * R3 - 3.0 * Ar * r[k] * R5 - 3.0 * Bu * r[k] * R5
                      - 3.0 * Br * u[k] * R5 - 3.0 * s * B[k] * R5
                      + 15.0 * s * Br * r[k] * R7);
        gu[k] = mj * (B[k] * R3 - 3.0 * Br * r[k] * R5);
    }
}

static inline int member_regular(int64_t n, const double *x, int64_t i, int64_t j, float rs2f)
{
    if (j == i)
        return 0;
    return !inside(x[j] - x[i], x[n + j] - x[n + i], x[2 * n + j] - x[2 * n + i], rs2f);
}

/* xm: positions used for the (frozen) membership test; normally == xp.       */
void or_adjoint(int64_t n, const double *xp, const double *vp, const double *m,
                const double *xm, int32_t n_i, const int32_t *i_block, const double *rs2,
                const double *w_a, const double *w_j, double *gx, double *gv, double *gm)
{
    /* per-row part: -dl/dr and -dl/du summed over j, to a row buffer */
    double *row = (double *)malloc(sizeof(double) * 6 * (size_t)(n_i > 0 ? n_i : 1));
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t b = 0; b < n_i; ++b) {
        int64_t i = i_block[b];
        float rs2f = (float)rs2[b];
        double A[3], B[3];
        for (int k = 0; k < 3; ++k) {
            A[k] = w_a[(int64_t)k * n_i + b];
            B[k] = w_j[(int64_t)k * n_i + b];
        }
        csum R[3] = {{0, 0}, {0, 0}, {0, 0}}, U[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t j = 0; j < n; ++j) {
            if (!member_regular(n, xm, i, j, rs2f))
                continue;
            double r[3], u[3], gr[3], gu[3], g;
            for (int k = 0; k < 3; ++k) {
                r[k] = xp[(int64_t)k * n + j] - xp[(int64_t)k * n + i];
                u[k] = vp[(int64_t)k * n + j] - vp[(int64_t)k * n + i];
            }
            pair_grad(m[j], A, B, r, u, gr, gu, &g);
            for (int k = 0; k < 3; ++k) {
                cs_add(&R[k], gr[k]);
                cs_add(&U[k], gu[k]);
            }
        }
        for (int k = 0; k < 3; ++k) {
            row[6 * (size_t)b + k] = cs_get(&R[k]);
            row[6 * (size_t)b + 3 + k] = cs_get(&U[k]);
        }
    }
    /* per-body part: +dl/dr, +dl/du, dl/dm over all rows where j is regular */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < n; ++j) {
        csum R[3] = {{0, 0}, {0, 0}, {0, 0}}, U[3] = {{0, 0}, {0, 0}, {0, 0}}, M = {0, 0};
        for (int32_t b = 0; b < n_i; ++b) {
            int64_t i = i_block[b];
            if (!member_regular(n, xm, i, j, (float)rs2[b]))
                continue;
            double A[3], B[3], r[3], u[3], gr[3], gu[3], g;
            for (int k = 0; k < 3; ++k) {
                A[k] = w_a[(int64_t)k * n_i + b];
                B[k] = w_j[(int64_t)k * n_i + b];
                r[k] = xp[(int64_t)k * n + j] - xp[(int64_t)k * n + i];
                u[k] = vp[(int64_t)k * n + j] - vp[(int64_t)k * n + i];
            }
            pair_grad(m[j], A, B, r, u, gr, gu, &g);
            for (int k = 0; k < 3; ++k) {
                cs_add(&R[k], gr[k]);
                cs_add(&U[k], gu[k]);
            }
            cs_add(&M, g);
        }
        for (int k = 0; k < 3; ++k) {
            gx[(int64_t)k * n + j] = cs_get(&R[k]);
            gv[(int64_t)k * n + j] = cs_get(&U[k]);
        }
        gm[j] = cs_get(&M);
    }
    /* subtract the per-row parts, in row order */
    for (int32_t b = 0; b < n_i; ++b) {
        int64_t i = i_block[b];
        for (int k = 0; k < 3; ++k) {
            gx[(int64_t)k * n + i] -= row[6 * (size_t)b + k];
            gv[(int64_t)k * n + i] -= row[6 * (size_t)b + 3 + k];
        }
    }
    free(row);
}

/* Local loss of body k: the sum of the pair losses l(b, j) (see above) over  */
/* every regular pair that involves body k, either as the row body i_b or as  */
/* the source j.  Its derivative with respect to body k's own coordinates is  */
/* the full dL/d(x_k, v_k, m_k), but its value is small, so central finite    */
/* differences of it are not swamped by the rounding of the whole of L.       */
/* Membership is frozen: tested on xm, while the pair terms use xp.           */
double or_local_loss(int64_t n, const double *xp, const double *vp, const double *m,
                     const double *xm, int32_t n_i, const int32_t *i_block, const double *rs2,
                     const double *w_a, const double *w_j, int64_t body)
{
    csum L = {0, 0};
    for (int32_t b = 0; b < n_i; ++b) {
        int64_t i = i_block[b];
        float rs2f = (float)rs2[b];
        double A[3], B[3];
        for (int kk = 0; kk < 3; ++kk) {
            A[kk] = w_a[(int64_t)kk * n_i + b];
            B[kk] = w_j[(int64_t)kk * n_i + b];
        }
        /* only pairs that involve body: all j when it is the row body, else j = body */
        int64_t j_lo = i == body ? 0 : body, j_hi = i == body ? n : body + 1;
        for (int64_t j = j_lo; j < j_hi; ++j) {
            if (!member_regular(n, xm, i, j, rs2f))
                continue;
            double r[3], u[3];
            for (int kk = 0; kk < 3; ++kk) {
                r[kk] = xp[(int64_t)kk * n + j] - xp[(int64_t)kk * n + i];
                u[kk] = vp[(int64_t)kk * n + j] - vp[(int64_t)kk * n + i];
            }
            double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            double R3 = 1.0 / (r2 * sqrt(r2));
            double R5 = R3 / r2;
            double s = r[0] * u[0] + r[1] * u[1] + r[2] * u[2];
            double Ar = A[0] * r[0] + A[1] * r[1] + A[2] * r[2];
            double Br = B[0] * r[0] + B[1] * r[1] + B[2] * r[2];
            double Bu = B[0] * u[0] + B[1] * u[1] + B[2] * u[2];
            cs_add(&L, m[j] * (Ar * R3 + Bu * R3 - 3.0 * s * Br * R5));
        }
    }
    return cs_get(&L);
}

/* ------------------------------------------------------------------------- */
/* Fourth-order Hermite corrector (the integrator of section 2, after Makino  */
/* 1991): with the force a0 and its derivative j0 at the start of a step of   */
/* length h and the new a1, j1 at its end (evaluated at the predicted state), */
/*   v1 = v0 + h/2 (a0 + a1) + h^2/12 (j0 - j1)                                */
/*   x1 = x0 + h/2 (v0 + v1) + h^2/12 (a0 - a1)                                */
/* and the second and third force derivatives at the end of the step from the */
/* cubic Hermite interpolant of a over the step:                              */
/*   a2(t0) = (-6 (a0 - a1) - h (4 j0 + 2 j1)) / h^2                           */
/*   a3     = (12 (a0 - a1) + 6 h (j0 + j1)) / h^3                             */
/*   a2(t1) = a2(t0) + h a3                                                    */
/* All [3][n] planes, per-body step h[n].                                      */
/* ------------------------------------------------------------------------- */
void or_hermite_correct(int64_t n, const double *h, const double *x0, const double *v0,
                        const double *a0, const double *j0, const double *a1,
                        const double *j1, double *x1, double *v1, double *a2, double *a3)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double dt = h[i];
        for (int k = 0; k < 3; ++k) {
            int64_t q = (int64_t)k * n + i;
            double vn = v0[q] + dt / 2 * (a0[q] + a1[q]) + dt * dt / 12 * (j0[q] - j1[q]);
            double xn = x0[q] + dt / 2 * (v0[q] + vn) + dt * dt / 12 * (a0[q] - a1[q]);
            double s0 = (-6 * (a0[q] - a1[q]) - dt * (4 * j0[q] + 2 * j1[q])) / (dt * dt);
            double c = (12 * (a0[q] - a1[q]) + 6 * dt * (j0[q] + j1[q])) / (dt * dt * dt);
            v1[q] = vn;
            x1[q] = xn;
            a2[q] = s0 + dt * c;
            a3[q] = c;
        }
    }
}

int or_version(void) { return 1; }
