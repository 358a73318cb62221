/*
 * D3 dispersion oracle: plain, slow FP64 reference of the dispersion term of
 * NEP-D3 (the correction the paper adds to its MOF model, Sec. II.C "NEP for
 * MOFs": D3 with Becke-Johnson damping, 12 A dispersion cutoff, 6 A
 * coordination-number cutoff).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; it shares no code, header or table with the HIP library.
 *
 * The paper names the correction without its formulas; this file follows
 * the published D3 form (Grimme et al. 2010 for the coordination number and
 * the C6 interpolation, Grimme, Ehrlich and Goerigk 2011 for the damping),
 * in eV and Angstrom:
 *   CN_i  = sum_{j != i, r_ij < rc_cn} 1 / (1 + exp(-k1 (k2 (R_i + R_j) / r_ij - 1)))
 *   C6_ij = sum_ab C6ref_ij(a,b) L_ab / sum_ab L_ab,
 *           L_ab = exp(-k3 [(CN_i - CNref_i(a))^2 + (CN_j - CNref_j(b))^2])
 *   C8_ij = 3 C6_ij q_i q_j
 *   f_ij  = a1 sqrt(C8_ij / C6_ij) + a2
 *   E     = -1/2 sum_i sum_{j != i, r_ij < rc} [s6 C6_ij / (r^6 + f^6) + s8 C8_ij / (r^8 + f^8)]
 * with hard cutoffs (strict r^2 < rc^2, the same minimum image as the NEP
 * oracle).  The reference tables (R_i, q_i, CNref, C6ref) and the damping
 * constants come from the parameter file; the tests use seeded synthetic
 * tables, so agreement with the published element tables is not claimed.
 *
 * Forces: F_i = -dE/dr_i with both the explicit distance dependence and the
 * dependence through CN_i and CN_j.  Virial: W_ab = -sum over ordered pairs
 * (i, j) of r_ij^a (dE/dr_ij)^b, E written through ordered pair vectors.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define D3_MAXS 4
#define D3_MAXREF 5

void or_mic(const double *ri, const double *rj, const double *box, double *d, double *r2);

typedef struct or_d3 {
    int S;
    double rc, rcn;             /* dispersion and coordination cutoffs, A */
    double s6, s8, a1, a2;      /* damping: a2 in A */
    double k1, k2, k3;
    double rcov[D3_MAXS], q[D3_MAXS];
    int nref[D3_MAXS];
    double cnref[D3_MAXS][D3_MAXREF];
    double c6ref[D3_MAXS][D3_MAXS][D3_MAXREF][D3_MAXREF];   /* eV A^6 */
} or_d3;

static int rd(FILE *f, double *v) { return fscanf(f, "%lf", v) == 1 ? 0 : 1; }

static int expect(FILE *f, const char *w)
{
    char buf[64];
    return (fscanf(f, "%63s", buf) == 1 && strcmp(buf, w) == 0) ? 0 : 1;
}

int or_d3_load(const char *path, or_d3 **out)
{
    FILE *f = fopen(path, "r");
    if (!f) return 1;
    or_d3 *d = (or_d3 *)calloc(1, sizeof *d);
    int err = 0, ver = 0;
    err |= expect(f, "nep_d3_params") || fscanf(f, "%d", &ver) != 1 || ver != 1;
    err |= expect(f, "species") || fscanf(f, "%d", &d->S) != 1 || d->S < 1 || d->S > D3_MAXS;
    err |= expect(f, "cutoff") || rd(f, &d->rc) || rd(f, &d->rcn);
    err |= expect(f, "damping") || rd(f, &d->s6) || rd(f, &d->s8) || rd(f, &d->a1) || rd(f, &d->a2);
    err |= expect(f, "constants") || rd(f, &d->k1) || rd(f, &d->k2) || rd(f, &d->k3);
    if (!err) {
        err |= expect(f, "rcov");
        for (int s = 0; s < d->S && !err; ++s) err |= rd(f, &d->rcov[s]);
        err |= expect(f, "q");
        for (int s = 0; s < d->S && !err; ++s) err |= rd(f, &d->q[s]);
        err |= expect(f, "nref");
        for (int s = 0; s < d->S && !err; ++s)
            err |= fscanf(f, "%d", &d->nref[s]) != 1 || d->nref[s] < 1 || d->nref[s] > D3_MAXREF;
        err |= expect(f, "cnref");
        for (int s = 0; s < d->S && !err; ++s)
            for (int a = 0; a < d->nref[s] && !err; ++a) err |= rd(f, &d->cnref[s][a]);
        err |= expect(f, "c6ref");
        for (int si = 0; si < d->S && !err; ++si)
            for (int sj = 0; sj < d->S && !err; ++sj)
                for (int a = 0; a < d->nref[si] && !err; ++a)
                    for (int b = 0; b < d->nref[sj] && !err; ++b) err |= rd(f, &d->c6ref[si][sj][a][b]);
    }
    fclose(f);
    if (err) { free(d); return 2; }
    *out = d;
    return 0;
}

void or_d3_free(or_d3 *d) { free(d); }

/* One coordination-number term and its derivative with respect to r. */
void or_d3_cn_term(const or_d3 *d, int ti, int tj, double r, double *c, double *dc)
{
    const double R = d->rcov[ti] + d->rcov[tj];
    const double g = exp(-d->k1 * (d->k2 * R / r - 1.0));
    *c = 1.0 / (1.0 + g);
    /* dg/dr = g k1 k2 R / r^2;  dc/dr = -(dg/dr) / (1 + g)^2 */
    *dc = -g * d->k1 * d->k2 * R / (r * r) / ((1.0 + g) * (1.0 + g));
}

/* C6 of a species pair at coordination numbers (cni, cnj), with its
 * derivatives: the weighted mean of the reference values.  The mean does
 * not change when every weight is multiplied by one factor, so the weights
 * are taken relative to the largest, exp(-k3 (D_ab - D_min)) with
 * D_ab = (cni - CNref_a)^2 + (cnj - CNref_b)^2: far from every reference
 * the plain weights would all underflow (0/0), while the mean tends to the
 * nearest reference's C6.  The factor depends on the coordination numbers
 * but drops out of the derivative of the mean as well, so the weights'
 * derivatives are taken at a fixed factor. */
void or_d3_c6(const or_d3 *d, int ti, int tj, double cni, double cnj, double *c6, double *dc6i, double *dc6j)
{
    double Z = 0.0, W = 0.0, dZi = 0.0, dWi = 0.0, dZj = 0.0, dWj = 0.0;
    double Dmin = INFINITY;
    for (int a = 0; a < d->nref[ti]; ++a)
        for (int b = 0; b < d->nref[tj]; ++b) {
            const double xi = cni - d->cnref[ti][a], xj = cnj - d->cnref[tj][b];
            const double D = xi * xi + xj * xj;
            if (D < Dmin) Dmin = D;
        }
    for (int a = 0; a < d->nref[ti]; ++a)
        for (int b = 0; b < d->nref[tj]; ++b) {
            const double xi = cni - d->cnref[ti][a], xj = cnj - d->cnref[tj][b];
            const double L = exp(-d->k3 * ((xi * xi + xj * xj) - Dmin));
            const double c = d->c6ref[ti][tj][a][b];
            Z += c * L;
            W += L;
            /* dL/dcn_i = -2 k3 x_i L */
            dZi += c * (-2.0 * d->k3 * xi * L);
            dWi += -2.0 * d->k3 * xi * L;
            dZj += c * (-2.0 * d->k3 * xj * L);
            dWj += -2.0 * d->k3 * xj * L;
        }
    *c6 = Z / W;
    *dc6i = (dZi * W - Z * dWi) / (W * W);
    *dc6j = (dZj * W - Z * dWj) / (W * W);
}

/* Pair energy e(r) = s6 C6 / (r^6 + f^6) + s8 C8 / (r^8 + f^8) at fixed C6,
 * its r derivative and its C6 derivative. */
static void pair_e(const or_d3 *d, int ti, int tj, double c6, double r, double *e, double *dedr, double *dedc6)
{
    const double qq = 3.0 * d->q[ti] * d->q[tj];      /* C8 / C6 */
    const double c8 = qq * c6;
    const double f = d->a1 * sqrt(qq) + d->a2;
    const double f2 = f * f, f6 = f2 * f2 * f2, f8 = f6 * f2;
    const double r2 = r * r, r6 = r2 * r2 * r2, r8 = r6 * r2;
    const double d6 = r6 + f6, d8 = r8 + f8;
    *e = d->s6 * c6 / d6 + d->s8 * c8 / d8;
    *dedr = -d->s6 * c6 * 6.0 * r6 / r / (d6 * d6) - d->s8 * c8 * 8.0 * r8 / r / (d8 * d8);
    *dedc6 = d->s6 / d6 + d->s8 * qq / d8;
}

/* Coordination numbers of one configuration. */
void or_d3_cn(const or_d3 *d, const double *pos, const int *types, int N, const double *box, double *CN)
{
    const double rcn2 = d->rcn * d->rcn;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i) {
        double s = 0.0;
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            double v[3], r2;
            or_mic(pos + 3 * i, pos + 3 * j, box, v, &r2);
            if (r2 < rcn2) {
                double c, dc;
                or_d3_cn_term(d, types[i], types[j], sqrt(r2), &c, &dc);
                s += c;
            }
        }
        CN[i] = s;
    }
}

/* Energy, forces and virial of one configuration (see the header).  CN [N]
 * receives the coordination numbers and U [N] the site energies
 * U_i = -1/2 sum_j e_ij (either may be NULL). */
int or_d3_config(const or_d3 *d, const double *pos, const int *types, int N, const double *box, double *E,
                 double *F, double *W, double *CN, double *U)
{
    double *cn = (double *)malloc(sizeof(double) * (N ? N : 1));
    double *dEdcn = (double *)calloc(N ? N : 1, sizeof(double));
    if (!cn || !dEdcn) { free(cn); free(dEdcn); return 1; }
    or_d3_cn(d, pos, types, N, box, cn);
    const double rc2 = d->rc * d->rc, rcn2 = d->rcn * d->rcn;
    double Etot = 0.0, Wt[9] = {0};
    for (int i = 0; i < N; ++i) F[3 * i] = F[3 * i + 1] = F[3 * i + 2] = 0.0;
    /* explicit distance dependence: E = -1/2 sum over ordered pairs of e_ij */
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : Etot) reduction(+ : Wt[:9])
    for (int i = 0; i < N; ++i) {
        double Ui = 0.0;
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            double v[3], r2;
            or_mic(pos + 3 * i, pos + 3 * j, box, v, &r2);
            if (!(r2 < rc2)) continue;
            const double r = sqrt(r2);
            double c6, dc6i, dc6j, e, dedr, dedc6;
            or_d3_c6(d, types[i], types[j], cn[i], cn[j], &c6, &dc6i, &dc6j);
            pair_e(d, types[i], types[j], c6, r, &e, &dedr, &dedc6);
            Ui += -0.5 * e;
            /* dE/dCN_i = -sum_j de_ij/dC6 dC6_ij/dCN_i (each unordered pair twice, with 1/2) */
            dEdcn[i] += -dedc6 * dc6i;
            /* F_i = -dE/dr_i = -sum_j e'_ij u_ij, u_ij = (r_j - r_i) / r */
            for (int a = 0; a < 3; ++a) F[3 * i + a] += -dedr * v[a] / r;
            /* W += -r_ij (x) dE/dr_ij with dE/dr_ij = -1/2 e' u_ij */
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Wt[3 * a + b] += 0.5 * dedr * v[a] * v[b] / r;
        }
        if (U) U[i] = Ui;
        Etot += Ui;
    }
    /* dependence through the coordination numbers: CN_i = sum_j c(r_ij) */
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : Wt[:9])
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            double v[3], r2;
            or_mic(pos + 3 * i, pos + 3 * j, box, v, &r2);
            if (!(r2 < rcn2)) continue;
            const double r = sqrt(r2);
            double c, dc;
            or_d3_cn_term(d, types[i], types[j], r, &c, &dc);
            /* r_ij enters CN_i and CN_j: F_i += (dE/dCN_i + dE/dCN_j) c'(r) u_ij */
            for (int a = 0; a < 3; ++a) F[3 * i + a] += (dEdcn[i] + dEdcn[j]) * dc * v[a] / r;
            /* ordered pair (i, j) through CN_i: dE/dr_ij = dE/dCN_i c' u_ij */
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Wt[3 * a + b] += -dEdcn[i] * dc * v[a] * v[b] / r;
        }
    }
    *E = Etot;
    for (int k = 0; k < 9; ++k) W[k] = Wt[k];
    if (CN) memcpy(CN, cn, sizeof(double) * N);
    free(cn);
    free(dEdcn);
    return 0;
}

/* All beads of a ring polymer: pos [P][N][3] -> E [P], F [P][N][3], W [P][9]. */
int or_d3_beads(const or_d3 *d, const double *pos, const int *types, int P, int N, const double *box, double *E,
                double *F, double *W)
{
    int err = 0;
    for (int b = 0; b < P; ++b)
        err |= or_d3_config(d, pos + (size_t)b * N * 3, types, N, box, E + b, F + (size_t)b * N * 3, W + 9 * b,
                            NULL, NULL);
    return err;
}
