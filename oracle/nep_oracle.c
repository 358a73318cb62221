/*
 * NEP oracle: plain, slow FP64 reference for the NEP energy, forces and
 * virial (paper Sec. II.C; force and virial definitions of Sec. II.A).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or table with the HIP
 * library.
 *
 * The paper names the NEP descriptor but defers its explicit form to the NEP
 * papers.  This file follows the published NEP form:
 *   f_c(r)  = (1 + cos(pi r / rc)) / 2                       (r < rc)
 *   x       = 2 (r/rc - 1)^2 - 1,  T_k Chebyshev polynomials
 *   f_k(r)  = (T_k(x) + 1) / 2 * f_c(r),              k = 0..K
 *   g_n(r)  = sum_k c^{ti tj}_{nk} f_k(r)
 *   radial   q_n    = sum_{j in R(i)} g_n(r_ij)
 *   angular  q_nl   = (2l+1)/(4 pi) sum_{j,k in A(i)} g_n(r_ij) g_n(r_ik) P_l(cos theta_ijk)
 *                     for l = 1..l_max (the j = k terms included)
 *   4-body   q4_n   = kappa tr(M_n^3),  M_n = sum_j g_n(r_ij) (u u^T - I/3),
 *                     kappa = -(9/2) sqrt(2/35) (5/(4 pi))^{3/2}
 *   site energy U_i = sum_mu w1_mu tanh(sum_nu W0_{mu nu} s_nu q_nu - b0_mu) - b1
 * Descriptor order: radial n; angular (l-1)(n_A+1)+n; then four-body n.
 * The angular term is evaluated as the Legendre double sum above (not through
 * spherical-harmonic sums) and its gradient is the analytic derivative of
 * that double sum.
 *
 * Forces: F_i = -dU/dr_i = sum_j (dU_i/dr_ij - dU_j/dr_ji), r_ij = r_j - r_i
 * under the minimum image.  Virial: W_ab = -sum_i sum_j r_ij^a (dU_i/dr_ij)^b;
 * the per-atom split gives each of i and j half of -r_ij (x) dU_i/dr_ij.
 *
 * Built with -ffp-contract=off so that the minimum-image distance test is the
 * literal IEEE expression below.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

typedef struct or_model {
    int S, nR, nA, kR, kA, L, four, H, D;
    double rcR, rcA;
    double *cR, *cA, *qs, *W0, *b0, *w1;
    double b1;
} or_model;

/* ------------------------------------------------------------------ */
/* model file                                                          */
/* ------------------------------------------------------------------ */

typedef struct { char **tok; int n, pos; char *buf; } toks_t;

static int tok_read(const char *path, toks_t *t)
{
    FILE *f = fopen(path, "rb");
    if (!f) return 1;
    fseek(f, 0, SEEK_END);
    long len = ftell(f);
    fseek(f, 0, SEEK_SET);
    t->buf = (char *)malloc((size_t)len + 1);
    if (fread(t->buf, 1, (size_t)len, f) != (size_t)len) { fclose(f); return 1; }
    fclose(f);
    t->buf[len] = 0;
    int cap = 1024;
    t->tok = (char **)malloc(sizeof(char *) * cap);
    t->n = 0; t->pos = 0;
    char *p = t->buf;
    int line_start = 1;
    while (*p) {
        if (*p == '\n') { line_start = 1; *p++ = 0; continue; }
        if (*p == ' ' || *p == '\t' || *p == '\r') { *p++ = 0; continue; }
        if (line_start && *p == '#') { while (*p && *p != '\n') *p++ = 0; continue; }
        line_start = 0;
        if (t->n == cap) { cap *= 2; t->tok = (char **)realloc(t->tok, sizeof(char *) * cap); }
        t->tok[t->n++] = p;
        while (*p && *p != ' ' && *p != '\t' && *p != '\n' && *p != '\r') p++;
    }
    return 0;
}

static const char *tok_next(toks_t *t) { return t->pos < t->n ? t->tok[t->pos++] : NULL; }
static int tok_expect(toks_t *t, const char *w) { const char *s = tok_next(t); return !s || strcmp(s, w) != 0; }
static int tok_int(toks_t *t, int *v) { const char *s = tok_next(t); if (!s) return 1; *v = atoi(s); return 0; }
static int tok_dbl(toks_t *t, double *v) { const char *s = tok_next(t); if (!s) return 1; *v = strtod(s, NULL); return 0; }
static int tok_arr(toks_t *t, double *a, int n) { for (int i = 0; i < n; ++i) if (tok_dbl(t, a + i)) return 1; return 0; }

void or_model_free(or_model *m)
{
    if (!m) return;
    free(m->cR); free(m->cA); free(m->qs); free(m->W0); free(m->b0); free(m->w1);
    free(m);
}

int or_model_load(const char *path, or_model **out)
{
    toks_t t; memset(&t, 0, sizeof t);
    if (tok_read(path, &t)) return 1;
    or_model *m = (or_model *)calloc(1, sizeof *m);
    int ver, err = 0;
    err |= tok_expect(&t, "nep_pimd_model") || tok_int(&t, &ver) || ver != 1;
    err |= tok_expect(&t, "species") || tok_int(&t, &m->S);
    err |= tok_expect(&t, "cutoff") || tok_dbl(&t, &m->rcR) || tok_dbl(&t, &m->rcA);
    err |= tok_expect(&t, "n_max") || tok_int(&t, &m->nR) || tok_int(&t, &m->nA);
    err |= tok_expect(&t, "basis") || tok_int(&t, &m->kR) || tok_int(&t, &m->kA);
    err |= tok_expect(&t, "l_max") || tok_int(&t, &m->L);
    err |= tok_expect(&t, "four_body") || tok_int(&t, &m->four);
    err |= tok_expect(&t, "hidden") || tok_int(&t, &m->H);
    if (!err && (m->S < 1 || m->nR < 0 || m->nA < 0 || m->kR < 1 || m->kA < 1 ||
                 m->L < 1 || m->L > 8 || m->H < 1)) err = 1;
    if (!err) {
        m->D = (m->nR + 1) + m->L * (m->nA + 1) + (m->four ? m->nA + 1 : 0);
        int nc_r = m->S * m->S * (m->nR + 1) * (m->kR + 1);
        int nc_a = m->S * m->S * (m->nA + 1) * (m->kA + 1);
        m->cR = (double *)malloc(sizeof(double) * nc_r);
        m->cA = (double *)malloc(sizeof(double) * nc_a);
        m->qs = (double *)malloc(sizeof(double) * m->D);
        m->W0 = (double *)malloc(sizeof(double) * m->S * m->H * m->D);
        m->b0 = (double *)malloc(sizeof(double) * m->S * m->H);
        m->w1 = (double *)malloc(sizeof(double) * m->S * m->H);
        err |= tok_expect(&t, "c_radial") || tok_arr(&t, m->cR, nc_r);
        err |= tok_expect(&t, "c_angular") || tok_arr(&t, m->cA, nc_a);
        err |= tok_expect(&t, "q_scale") || tok_arr(&t, m->qs, m->D);
        err |= tok_expect(&t, "ann");
        for (int s = 0; s < m->S && !err; ++s) {
            err |= tok_arr(&t, m->W0 + (size_t)s * m->H * m->D, m->H * m->D);
            err |= tok_arr(&t, m->b0 + (size_t)s * m->H, m->H);
            err |= tok_arr(&t, m->w1 + (size_t)s * m->H, m->H);
        }
        err |= tok_expect(&t, "b1") || tok_dbl(&t, &m->b1);
    }
    free(t.tok); free(t.buf);
    if (err) { or_model_free(m); return 2; }
    *out = m;
    return 0;
}

/* dims: S nR nA kR kA L four H D ; rc: rcR rcA */
void or_model_dims(const or_model *m, int *dims, double *rc)
{
    dims[0] = m->S; dims[1] = m->nR; dims[2] = m->nA; dims[3] = m->kR; dims[4] = m->kA;
    dims[5] = m->L; dims[6] = m->four; dims[7] = m->H; dims[8] = m->D;
    rc[0] = m->rcR; rc[1] = m->rcA;
}

/* ------------------------------------------------------------------ */
/* BF16 weights                                                        */
/* ------------------------------------------------------------------ */

/* The BF16 number nearest to the FP32 number nearest to x (BF16: 8
 * significant bits and the FP32 exponent range; ties to the even
 * significand).  From the definition: with f = m 2^e, 1/2 <= |m| < 1, the
 * BF16 numbers of that binade are k 2^(e-8), 128 <= k <= 256. */
double or_bf16_round(double x)
{
    const float f = (float)x;
    if (f == 0.0f || !isfinite(f)) return (double)f;
    int e;
    const double m = frexp((double)f, &e);
    const double k = nearbyint(ldexp(m, 8));   /* default rounding: to nearest, ties to even */
    return ldexp(k, e - 8);
}

void or_bf16_round_array(const double *x, double *y, int n)
{
    for (int i = 0; i < n; ++i) y[i] = or_bf16_round(x[i]);
}

/* Replace the first-layer weights W0 of every species by their BF16 values
 * (the network of the matrix-core inference path). */
void or_model_round_w0_bf16(or_model *m)
{
    const size_t n = (size_t)m->S * m->H * m->D;
    for (size_t i = 0; i < n; ++i) m->W0[i] = or_bf16_round(m->W0[i]);
}

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */

/* Periodic cells are given by their three edge vectors as the rows of
 * box[9] (row-major H: r = s H with fractional coordinates s).  A cell is
 * orthorhombic when every off-diagonal entry is zero. */
static int cell_is_orthorhombic(const double *box)
{
    return box[1] == 0.0 && box[2] == 0.0 && box[3] == 0.0 && box[5] == 0.0 && box[6] == 0.0 && box[7] == 0.0;
}

/* G = H^-1 from the cofactors: row vectors map to fractional coordinates
 * as s = x G. */
static void cell_inverse(const double *H, double *G)
{
    const double c00 = H[4] * H[8] - H[5] * H[7], c01 = H[5] * H[6] - H[3] * H[8], c02 = H[3] * H[7] - H[4] * H[6];
    const double det = H[0] * c00 + H[1] * c01 + H[2] * c02;
    G[0] = c00 / det;
    G[3] = c01 / det;
    G[6] = c02 / det;
    G[1] = (H[2] * H[7] - H[1] * H[8]) / det;
    G[4] = (H[0] * H[8] - H[2] * H[6]) / det;
    G[7] = (H[1] * H[6] - H[0] * H[7]) / det;
    G[2] = (H[1] * H[5] - H[2] * H[4]) / det;
    G[5] = (H[2] * H[3] - H[0] * H[5]) / det;
    G[8] = (H[0] * H[4] - H[1] * H[3]) / det;
}

/* Minimum-image difference d = r_j - r_i and its squared length.
 * Orthorhombic cells: per axis x - L rint(x / L).  Other cells: the
 * fractional difference s = x G is reduced by rint per axis and mapped back,
 * d = (s - rint(s)) H; this is the nearest image whenever it is shorter than
 * half the smallest distance between opposite faces of the cell. */
static void mic(const double *ri, const double *rj, const double *box, double *d, double *r2)
{
    if (cell_is_orthorhombic(box)) {
        for (int a = 0; a < 3; ++a) {
            double x = rj[a] - ri[a];
            double L = box[4 * a];
            double k = rint(x / L);
            double s = L * k;
            d[a] = x - s;
        }
    } else {
        double G[9], x[3], f[3];
        cell_inverse(box, G);
        for (int a = 0; a < 3; ++a) x[a] = rj[a] - ri[a];
        for (int c = 0; c < 3; ++c) {
            double s = (x[0] * G[c] + x[1] * G[3 + c]) + x[2] * G[6 + c];
            f[c] = s - rint(s);
        }
        for (int a = 0; a < 3; ++a) d[a] = (f[0] * box[a] + f[1] * box[3 + a]) + f[2] * box[6 + a];
    }
    double xx = d[0] * d[0];
    double yy = d[1] * d[1];
    double zz = d[2] * d[2];
    *r2 = (xx + yy) + zz;
}

/* mic() for the other oracle source. */
void or_mic(const double *ri, const double *rj, const double *box, double *d, double *r2) { mic(ri, rj, box, d, r2); }

/* Volume of the cell (the determinant of H). */
double or_cell_volume(const double *box)
{
    const double c00 = box[4] * box[8] - box[5] * box[7], c01 = box[5] * box[6] - box[3] * box[8],
                 c02 = box[3] * box[7] - box[4] * box[6];
    return box[0] * c00 + box[1] * c01 + box[2] * c02;
}

/* Brute-force neighbour list of one configuration: every j != i with
 * |mic(r_j - r_i)|^2 < rc^2, in ascending j.  cnt[i] is the full count even
 * when it exceeds cap (entries beyond cap are not stored).  Returns the
 * largest count. */
int or_neighbors(const double *pos, int N, const double *box, double rc, int cap, int *cnt, int *idx)
{
    double rc2 = rc * rc;
    int mx = 0;
#pragma omp parallel for schedule(static) reduction(max : mx)
    for (int i = 0; i < N; ++i) {
        int c = 0;
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            double d[3], r2;
            mic(pos + 3 * i, pos + 3 * j, box, d, &r2);
            if (r2 < rc2) {
                if (c < cap) idx[(size_t)i * cap + c] = j;
                ++c;
            }
        }
        cnt[i] = c;
        if (c > mx) mx = c;
    }
    return mx;
}

/* The same brute-force search for M selected atoms only (sampled checks of
 * large systems): row r holds the neighbours of atom atoms[r], ascending. */
int or_neighbors_of(const double *pos, int N, const double *box, double rc, int M, const int *atoms, int cap,
                    int *cnt, int *idx)
{
    double rc2 = rc * rc;
    int mx = 0;
#pragma omp parallel for schedule(static) reduction(max : mx)
    for (int r = 0; r < M; ++r) {
        const int i = atoms[r];
        int c = 0;
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            double d[3], r2;
            mic(pos + 3 * i, pos + 3 * j, box, d, &r2);
            if (r2 < rc2) {
                if (c < cap) idx[(size_t)r * cap + c] = j;
                ++c;
            }
        }
        cnt[r] = c;
        if (c > mx) mx = c;
    }
    return mx;
}

/* ------------------------------------------------------------------ */
/* basis functions                                                     */
/* ------------------------------------------------------------------ */

/* f_k and df_k/dr for k = 0..K at distance r (< rc). */
static void cheb(double r, double rc, int K, double *f, double *fp)
{
    double fc = 0.5 * (1.0 + cos(OR_PI * r / rc));
    double fcp = -0.5 * OR_PI / rc * sin(OR_PI * r / rc);
    double y = r / rc - 1.0;
    double x = 2.0 * y * y - 1.0;
    double dx = 4.0 * y / rc;
    double T[64], dT[64];
    T[0] = 1.0; dT[0] = 0.0;
    if (K >= 1) { T[1] = x; dT[1] = 1.0; }
    for (int k = 2; k <= K; ++k) {
        T[k] = 2.0 * x * T[k - 1] - T[k - 2];
        dT[k] = 2.0 * T[k - 1] + 2.0 * x * dT[k - 1] - dT[k - 2];
    }
    for (int k = 0; k <= K; ++k) {
        f[k] = 0.5 * (T[k] + 1.0) * fc;
        fp[k] = 0.5 * dT[k] * dx * fc + 0.5 * (T[k] + 1.0) * fcp;
    }
}

/* g_n and dg_n/dr, n = 0..nmax, for species pair (ti, tj). */
static void radial_g(const double *c, int S, int nmax, int K, int ti, int tj, double r, double rc,
                     double *g, double *gp)
{
    double f[64], fp[64];
    cheb(r, rc, K, f, fp);
    const double *cc = c + ((size_t)(ti * S + tj)) * (nmax + 1) * (K + 1);
    for (int n = 0; n <= nmax; ++n) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k <= K; ++k) {
            a += cc[n * (K + 1) + k] * f[k];
            b += cc[n * (K + 1) + k] * fp[k];
        }
        g[n] = a; gp[n] = b;
    }
}

/* Legendre P_l(x) and P_l'(x), l = 0..L. */
static void legendre(double x, int L, double *P, double *dP)
{
    P[0] = 1.0; dP[0] = 0.0;
    if (L >= 1) { P[1] = x; dP[1] = 1.0; }
    for (int l = 1; l < L; ++l) {
        P[l + 1] = ((2.0 * l + 1.0) * x * P[l] - l * P[l - 1]) / (l + 1.0);
        dP[l + 1] = dP[l - 1] + (2.0 * l + 1.0) * P[l];
    }
}

/* kappa = -(9/2) sqrt(2/35) (5/(4 pi))^{3/2}: makes kappa tr(M^3) the (2 2 2) Wigner-3j
 * contraction of the l = 2 spherical-harmonic sums. */
static double kappa4(void) { return -4.5 * sqrt(2.0 / 35.0) * pow(5.0 / (4.0 * OR_PI), 1.5); }

/* ------------------------------------------------------------------ */
/* one atom: descriptors, site energy, dU_i/dr_ij                      */
/* ------------------------------------------------------------------ */

typedef struct {
    int nR_cnt, nA_cnt;
    const int *jR, *jA;
} atom_lists;

/* Computes U_i, the raw descriptors q (unscaled, length D) and the
 * derivative vectors dR[j] = dU_i/dr_ij (radial part, for j in R(i)) and
 * dA[j] (angular + four-body part, for j in A(i)). */
static void atom_eval(const or_model *m, int i, const double *pos, const int *types, const double *box,
                      const atom_lists *nl, double *U, double *q, double *dR, double *dA)
{
    const int ti = types[i];
    const int nR1 = m->nR + 1, nA1 = m->nA + 1, L = m->L, D = m->D;
    for (int v = 0; v < D; ++v) q[v] = 0.0;

    /* radial */
    double g[64], gp[64];
    for (int a = 0; a < nl->nR_cnt; ++a) {
        int j = nl->jR[a];
        double d[3], r2;
        mic(pos + 3 * i, pos + 3 * j, box, d, &r2);
        double r = sqrt(r2);
        radial_g(m->cR, m->S, m->nR, m->kR, ti, types[j], r, m->rcR, g, gp);
        for (int n = 0; n < nR1; ++n) q[n] += g[n];
    }

    /* angular: per-neighbour geometry */
    int nA = nl->nA_cnt;
    double *u = (double *)malloc(sizeof(double) * 3 * (nA + 1));
    double *rr = (double *)malloc(sizeof(double) * (nA + 1));
    double *ga = (double *)malloc(sizeof(double) * nA1 * (nA + 1));
    double *gap = (double *)malloc(sizeof(double) * nA1 * (nA + 1));
    for (int a = 0; a < nA; ++a) {
        int j = nl->jA[a];
        double d[3], r2;
        mic(pos + 3 * i, pos + 3 * j, box, d, &r2);
        double r = sqrt(r2);
        rr[a] = r;
        for (int c = 0; c < 3; ++c) u[3 * a + c] = d[c] / r;
        radial_g(m->cA, m->S, m->nA, m->kA, ti, types[j], r, m->rcA, ga + nA1 * a, gap + nA1 * a);
    }
    double Pl[16], dPl[16];
    for (int a = 0; a < nA; ++a) {
        for (int b = 0; b < nA; ++b) {
            double c = u[3 * a] * u[3 * b] + u[3 * a + 1] * u[3 * b + 1] + u[3 * a + 2] * u[3 * b + 2];
            legendre(c, L, Pl, dPl);
            for (int l = 1; l <= L; ++l) {
                double pref = (2.0 * l + 1.0) / (4.0 * OR_PI) * Pl[l];
                for (int n = 0; n < nA1; ++n)
                    q[nR1 + (l - 1) * nA1 + n] += pref * ga[nA1 * a + n] * ga[nA1 * b + n];
            }
        }
    }
    /* four-body */
    double M[16][9];
    if (m->four) {
        for (int n = 0; n < nA1; ++n) {
            for (int e = 0; e < 9; ++e) M[n][e] = 0.0;
            for (int a = 0; a < nA; ++a)
                for (int p = 0; p < 3; ++p)
                    for (int s = 0; s < 3; ++s)
                        M[n][3 * p + s] += ga[nA1 * a + n] * (u[3 * a + p] * u[3 * a + s] - (p == s ? 1.0 / 3.0 : 0.0));
            double M2[9], tr3 = 0.0;
            for (int p = 0; p < 3; ++p)
                for (int s = 0; s < 3; ++s) {
                    double acc = 0.0;
                    for (int k = 0; k < 3; ++k) acc += M[n][3 * p + k] * M[n][3 * k + s];
                    M2[3 * p + s] = acc;
                }
            for (int p = 0; p < 3; ++p)
                for (int k = 0; k < 3; ++k) tr3 += M2[3 * p + k] * M[n][3 * k + p];
            q[nR1 + L * nA1 + n] = kappa4() * tr3;
        }
    }

    /* network */
    const double *W0 = m->W0 + (size_t)ti * m->H * D;
    const double *b0 = m->b0 + (size_t)ti * m->H;
    const double *w1 = m->w1 + (size_t)ti * m->H;
    double Ui = -m->b1;
    double *G = (double *)calloc((size_t)D, sizeof(double));
    for (int mu = 0; mu < m->H; ++mu) {
        double z = -b0[mu];
        for (int v = 0; v < D; ++v) z += W0[mu * D + v] * (m->qs[v] * q[v]);
        double h = tanh(z);
        Ui += w1[mu] * h;
        double gz = w1[mu] * (1.0 - h * h);
        for (int v = 0; v < D; ++v) G[v] += gz * W0[mu * D + v];
    }
    for (int v = 0; v < D; ++v) G[v] *= m->qs[v];   /* dU_i/dq_v (unscaled q) */
    *U = Ui;

    /* radial derivatives */
    for (int a = 0; a < nl->nR_cnt; ++a) {
        int j = nl->jR[a];
        double d[3], r2;
        mic(pos + 3 * i, pos + 3 * j, box, d, &r2);
        double r = sqrt(r2);
        radial_g(m->cR, m->S, m->nR, m->kR, ti, types[j], r, m->rcR, g, gp);
        double s = 0.0;
        for (int n = 0; n < nR1; ++n) s += G[n] * gp[n];
        for (int c = 0; c < 3; ++c) dR[3 * a + c] = s * d[c] / r;
    }

    /* angular derivatives: d/dr_ij of the Legendre double sum */
    for (int a = 0; a < nA; ++a) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < nA; ++b) {
            double c = u[3 * a] * u[3 * b] + u[3 * a + 1] * u[3 * b + 1] + u[3 * a + 2] * u[3 * b + 2];
            legendre(c, L, Pl, dPl);
            double s_u = 0.0, s_t = 0.0;   /* coefficients of u_a and of (u_b - c u_a)/r_a */
            for (int l = 1; l <= L; ++l) {
                double pref = 2.0 * (2.0 * l + 1.0) / (4.0 * OR_PI);
                for (int n = 0; n < nA1; ++n) {
                    double Gnl = G[nR1 + (l - 1) * nA1 + n];
                    s_u += Gnl * pref * gap[nA1 * a + n] * ga[nA1 * b + n] * Pl[l];
                    s_t += Gnl * pref * ga[nA1 * a + n] * ga[nA1 * b + n] * dPl[l];
                }
            }
            for (int k = 0; k < 3; ++k)
                acc[k] += s_u * u[3 * a + k] + s_t * (u[3 * b + k] - c * u[3 * a + k]) / rr[a];
        }
        if (m->four) {
            for (int n = 0; n < nA1; ++n) {
                double M2[9], trM2 = 0.0;
                for (int p = 0; p < 3; ++p)
                    for (int s = 0; s < 3; ++s) {
                        double t = 0.0;
                        for (int k = 0; k < 3; ++k) t += M[n][3 * p + k] * M[n][3 * k + s];
                        M2[3 * p + s] = t;
                    }
                trM2 = M2[0] + M2[4] + M2[8];
                double M2u[3], uM2u = 0.0;
                for (int p = 0; p < 3; ++p) {
                    M2u[p] = M2[3 * p] * u[3 * a] + M2[3 * p + 1] * u[3 * a + 1] + M2[3 * p + 2] * u[3 * a + 2];
                    uM2u += u[3 * a + p] * M2u[p];
                }
                double G4 = G[nR1 + L * nA1 + n] * 3.0 * kappa4();
                double gv = ga[nA1 * a + n], gpv = gap[nA1 * a + n];
                for (int k = 0; k < 3; ++k)
                    acc[k] += G4 * (gpv * (uM2u - trM2 / 3.0) * u[3 * a + k] +
                                    2.0 * gv / rr[a] * (M2u[k] - uM2u * u[3 * a + k]));
            }
        }
        for (int k = 0; k < 3; ++k) dA[3 * a + k] = acc[k];
    }
    free(u); free(rr); free(ga); free(gap); free(G);
}

/* ------------------------------------------------------------------ */
/* one configuration                                                   */
/* ------------------------------------------------------------------ */

/* NEP energy, forces and virial of one configuration (one bead).
 * pos [N,3]; box [9] cell edge vectors as rows.  Outputs: E (total), F [N,3],
 * W [9] (row-major W_ab), optional U [N], Wat [N,9], q [N,D].
 * cap: neighbour-list capacity per atom.  Returns 0, or 3 if cap is too
 * small (the call is then incomplete). */
int or_nep_config(const or_model *m, const double *pos, const int *types, int N, const double *box,
                  int cap, double *E, double *F, double *W, double *U, double *Wat, double *qout)
{
    int *cR = (int *)malloc(sizeof(int) * N), *cA = (int *)malloc(sizeof(int) * N);
    int *iR = (int *)malloc(sizeof(int) * (size_t)N * cap), *iA = (int *)malloc(sizeof(int) * (size_t)N * cap);
    int mR = or_neighbors(pos, N, box, m->rcR, cap, cR, iR);
    int mA = or_neighbors(pos, N, box, m->rcA, cap, cA, iA);
    if (mR > cap || mA > cap) { free(cR); free(cA); free(iR); free(iA); return 3; }
    double *Ui = (double *)malloc(sizeof(double) * N);
    double *dR = (double *)malloc(sizeof(double) * (size_t)N * cap * 3);
    double *dA = (double *)malloc(sizeof(double) * (size_t)N * cap * 3);
    double *qq = (double *)malloc(sizeof(double) * (size_t)N * m->D);
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < N; ++i) {
        atom_lists nl = {cR[i], cA[i], iR + (size_t)i * cap, iA + (size_t)i * cap};
        atom_eval(m, i, pos, types, box, &nl, Ui + i, qq + (size_t)i * m->D,
                  dR + (size_t)i * cap * 3, dA + (size_t)i * cap * 3);
    }
    /* scatter: F_i += d_ij, F_j -= d_ij; each of W_i, W_j gets -1/2 r_ij (x) d_ij */
    double Et = 0.0;
    for (int i = 0; i < N; ++i) Et += Ui[i];
    for (int k = 0; k < 3 * N; ++k) F[k] = 0.0;
    double *Wl = (double *)calloc((size_t)N * 9, sizeof(double));
    for (int i = 0; i < N; ++i) {
        for (int pass = 0; pass < 2; ++pass) {
            int cnt = pass ? cA[i] : cR[i];
            const int *js = (pass ? iA : iR) + (size_t)i * cap;
            const double *dd = (pass ? dA : dR) + (size_t)i * cap * 3;
            for (int a = 0; a < cnt; ++a) {
                int j = js[a];
                double d[3], r2;
                mic(pos + 3 * i, pos + 3 * j, box, d, &r2);
                for (int c = 0; c < 3; ++c) {
                    F[3 * i + c] += dd[3 * a + c];
                    F[3 * j + c] -= dd[3 * a + c];
                }
                for (int p = 0; p < 3; ++p)
                    for (int s = 0; s < 3; ++s) {
                        double w = -0.5 * d[p] * dd[3 * a + s];
                        Wl[9 * i + 3 * p + s] += w;
                        Wl[9 * j + 3 * p + s] += w;
                    }
            }
        }
    }
    for (int e = 0; e < 9; ++e) W[e] = 0.0;
    for (int i = 0; i < N; ++i)
        for (int e = 0; e < 9; ++e) W[e] += Wl[9 * i + e];
    *E = Et;
    if (U) memcpy(U, Ui, sizeof(double) * N);
    if (Wat) memcpy(Wat, Wl, sizeof(double) * N * 9);
    if (qout) memcpy(qout, qq, sizeof(double) * (size_t)N * m->D);
    free(cR); free(cA); free(iR); free(iA); free(Ui); free(dR); free(dA); free(qq); free(Wl);
    return 0;
}

/* All P beads: pos [P,N,3] -> E [P], F [P,N,3], W [P,9], optional U [P,N], Wat [P,N,9]. */
int or_nep_beads(const or_model *m, const double *pos, const int *types, int P, int N, const double *box,
                 int cap, double *E, double *F, double *W, double *U, double *Wat)
{
    for (int b = 0; b < P; ++b) {
        int rc = or_nep_config(m, pos + (size_t)b * N * 3, types, N, box, cap, E + b,
                               F + (size_t)b * N * 3, W + 9 * b, U ? U + (size_t)b * N : NULL,
                               Wat ? Wat + (size_t)b * N * 9 : NULL, NULL);
        if (rc) return rc;
    }
    return 0;
}

/* Threads of the oracle's parallel loops (timing on one core). */
void or_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Partial radial distribution functions (the paper's water analysis,  */
/* Sec. III): pair histogram per species pair over every bead.         */
/*                                                                      */
/* counts[(a*S + b)*nbins + k] += number of ordered pairs (i of species a, */
/* j != i of species b) in one bead with k = floor(r * nbins / rmax) <     */
/* nbins, r = sqrt(|mic(r_j - r_i)|^2) in FP64 (minimum image as in mic()).*/
/* Pairs of one bead only (the same imaginary-time slice); all P beads    */
/* are summed.  pos [P][N][3], types [N] in 0..S-1, box [9] (rows: edges). */
/* ------------------------------------------------------------------ */
void or_rdf_counts(int P, int N, const double *pos, const int *types, int S, const double *box, double rmax,
                   int nbins, uint64_t *counts)
{
    const double inv = nbins / rmax;
    for (int b = 0; b < P; ++b) {
        const double *x = pos + (size_t)b * N * 3;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                if (j == i) continue;
                double d[3], r2;
                mic(x + 3 * i, x + 3 * j, box, d, &r2);
                const double t = sqrt(r2) * inv;
                if (t < nbins) counts[((size_t)types[i] * S + types[j]) * nbins + (int)t] += 1;
            }
    }
}

/* Centroid of a bead array: out[i][a] = (sum_j x[j][i][a]) / P, beads summed
 * in order j = 0..P-1 (plain mean: unwrapped ring polymers). */
void or_centroid(int P, int N, const double *x, double *out)
{
    for (size_t e = 0; e < (size_t)N * 3; ++e) {
        double s = 0.0;
        for (int j = 0; j < P; ++j) s += x[(size_t)j * N * 3 + e];
        out[e] = s / P;
    }
}
