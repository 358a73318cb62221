/*
 * Ring-polymer oracle: plain FP64 reference for the normal-mode transform,
 * the Cayley free ring-polymer step, the half-kick and the Langevin
 * (PILE / TRPMD / RPMD) thermostat of paper Sec. II.A, Eqs. (1)-(12).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code with the HIP library.
 *
 * Readings of the paper taken here:
 *  - Bead index j runs 1..P exactly as printed in the definition of C_jk
 *    (array index b = j - 1).  For odd P there is no (-1)^j row: cosine rows
 *    for 1 <= k < P/2, sine rows for k > P/2.
 *  - The back transform uses q_j = sum_k C_jk q~_k (the transpose), as the
 *    thermostat's Eq. (12) prints it; C is orthogonal.
 *  - Eqs. (5)-(6) update p~ and q~ simultaneously (both right-hand sides use
 *    the old values).  At omega_0 = 0 the limit is q~ += dt p~/m.
 *  - beta_P = 1 / (P kB T), consistent with omega_P = P kB T / hbar.
 *  - The thermostat acts before and after the free-polymer part: one step is
 *    O B A (force) B O, each O with c1 = exp(-gamma_k dt/2).
 *  - Random normals: Philox-4x32-10 (Salmon et al., SC'11) keyed by the seed,
 *    counter (atom, component*ceil(P/4) + k/4, step low, 2*step high + stage);
 *    normal k&3 of the block; uniforms u = (x + 1) 2^-32, Box-Muller pairs
 *    (u0,u1) -> normals 0,1 and (u2,u3) -> normals 2,3 (cos first).
 * Units: A, fs, amu, eV, K; velocities in A/fs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846
static const double OR_KB = 8.617333262e-5;       /* eV/K */
static const double OR_HBAR = 0.6582119569;       /* eV fs */

/* 1 amu A^2 / fs^2 expressed in eV */
static double amu_a2_fs2_ev(void) { return 1.66053906660e-27 * 1e10 / 1.602176634e-19; }

/* ------------------------------------------------------------------ */
/* Philox-4xW-10 counter-based generator (Salmon et al., SC'11).       */
/* One round: (hi0,lo0) = M0*x0, (hi1,lo1) = M1*x2;                     */
/*   x <- (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0); key += (W0, W1)     */
/* between rounds.  Written once as a macro so that the 64-bit member,  */
/* which numpy ships, can pin the round structure used by the 32-bit   */
/* member.                                                             */
/* ------------------------------------------------------------------ */

static inline void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

static inline void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    __uint128_t p = (__uint128_t)a * (__uint128_t)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

#define PHILOX_DEFINE(NAME, T, MULHILO, M0, M1, W0, W1)                          \
    void NAME(const T key_in[2], const T ctr_in[4], T out[4])                     \
    {                                                                             \
        T k0 = key_in[0], k1 = key_in[1];                                         \
        T x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];         \
        for (int r = 0; r < 10; ++r) {                                            \
            if (r > 0) { k0 += (T)(W0); k1 += (T)(W1); }                          \
            T hi0, lo0, hi1, lo1;                                                 \
            MULHILO((T)(M0), x0, &hi0, &lo0);                                     \
            MULHILO((T)(M1), x2, &hi1, &lo1);                                     \
            T y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;         \
            x0 = y0; x1 = y1; x2 = y2; x3 = y3;                                   \
        }                                                                         \
        out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;                       \
    }

PHILOX_DEFINE(or_philox4x32, uint32_t, mulhilo32, 0xD2511F53u, 0xCD9E8D57u, 0x9E3779B9u, 0xBB67AE85u)
PHILOX_DEFINE(or_philox4x64, uint64_t, mulhilo64, 0xD2E7470EE14C6C93ull, 0xCA5A826395121157ull,
              0x9E3779B97F4A7C15ull, 0xBB67AE8584CAA73Bull)

/* Standard normal of mode k, Cartesian component a of atom i at (step, stage),
 * for a ring polymer of P beads. */
static double normal_at(uint64_t seed, int64_t step, int stage, int i, int a, int k, int P)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint64_t st = (uint64_t)step;
    uint32_t nb = (uint32_t)((P + 3) / 4);
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)a * nb + (uint32_t)(k >> 2), (uint32_t)st,
                       (uint32_t)((st >> 32) * 2u + (uint32_t)stage)};
    uint32_t x[4];
    or_philox4x32(key, ctr, x);
    int m = k & 3;
    int pair = m >> 1;
    double u0 = ((double)x[2 * pair] + 1.0) * (1.0 / 4294967296.0);
    double u1 = ((double)x[2 * pair + 1] + 1.0) * (1.0 / 4294967296.0);
    double rad = sqrt(-2.0 * log(u0));
    double ang = 2.0 * OR_PI * u1;
    return (m & 1) ? rad * sin(ang) : rad * cos(ang);
}

/* out[a*P + k] = normal of (component a, mode k), a = 0..2, k = 0..P-1. */
void or_normals(uint64_t seed, int64_t step, int stage, int i, int P, double *out)
{
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < P; ++k) out[a * P + k] = normal_at(seed, step, stage, i, a, k, P);
}

/* ------------------------------------------------------------------ */
/* normal modes                                                        */
/* ------------------------------------------------------------------ */

/* C[b*P + k] = C_jk with j = b + 1. */
void or_nm_matrix(int P, double *C)
{
    for (int b = 0; b < P; ++b) {
        int j = b + 1;
        for (int k = 0; k < P; ++k) {
            double v;
            if (k == 0) v = 1.0 / sqrt((double)P);
            else if (2 * k == P) v = ((j & 1) ? -1.0 : 1.0) / sqrt((double)P);
            else if (2 * k < P) v = sqrt(2.0 / P) * cos(2.0 * OR_PI * j * k / P);
            else v = sqrt(2.0 / P) * sin(2.0 * OR_PI * j * k / P);
            C[b * P + k] = v;
        }
    }
}

/* omega_k = 2 omega_P sin(k pi / P), omega_P = P kB T / hbar (1/fs). */
void or_nm_freqs(int P, double T, double *w)
{
    double wP = P * OR_KB * T / OR_HBAR;
    for (int k = 0; k < P; ++k) w[k] = 2.0 * wP * sin(k * OR_PI / P);
}

/* x [P, M] (bead-major, M = 3N) -> y = modes (dir=+1: y_k = sum_j C_jk x_j)
 * or beads (dir=-1: y_j = sum_k C_jk x_k). */
void or_nm_transform(int P, int M, int dir, const double *x, double *y)
{
    double *C = (double *)malloc(sizeof(double) * P * P);
    or_nm_matrix(P, C);
    for (int c = 0; c < M; ++c)
        for (int o = 0; o < P; ++o) {
            double s = 0.0;
            for (int i = 0; i < P; ++i)
                s += (dir > 0 ? C[i * P + o] : C[o * P + i]) * x[(size_t)i * M + c];
            y[(size_t)o * M + c] = s;
        }
    free(C);
}

/* ------------------------------------------------------------------ */
/* integrator stages                                                   */
/* ------------------------------------------------------------------ */

enum { OR_PIMD = 0, OR_TRPMD = 1, OR_RPMD = 2 };
enum { OR_PRE = 0, OR_POST = 1, OR_FUSED = 2 };

typedef struct {
    int P, N, mode;
    double dt, T, tau;
    uint64_t seed;
    const double *mass;
    double *C, *w, *c1, *c2;
} rp_t;

static void thermo_O(const rp_t *s, double *v, int i, int a, int64_t step, int stage)
{
    int P = s->P, N = s->N;
    double *vt = (double *)malloc(sizeof(double) * P);
    for (int k = 0; k < P; ++k) {
        double acc = 0.0;
        for (int b = 0; b < P; ++b) acc += v[((size_t)b * N + i) * 3 + a] * s->C[b * P + k];
        vt[k] = acc;
    }
    /* sqrt(m / beta_P) in momentum = sqrt(P kB T / m) in velocity */
    double sig = sqrt(P * OR_KB * s->T / (s->mass[i] * amu_a2_fs2_ev()));
    for (int k = 0; k < P; ++k) {
        int on = (s->mode == OR_PIMD) || (s->mode == OR_TRPMD && k > 0);
        if (!on) continue;
        double xi = normal_at(s->seed, step, stage, i, a, k, P);
        vt[k] = s->c1[k] * vt[k] + sig * s->c2[k] * xi;
    }
    for (int b = 0; b < P; ++b) {
        double acc = 0.0;
        for (int k = 0; k < P; ++k) acc += s->C[b * P + k] * vt[k];
        v[((size_t)b * N + i) * 3 + a] = acc;
    }
    free(vt);
}

static void kick_B(const rp_t *s, double *v, const double *F, int i, int a)
{
    double f = 0.5 * s->dt / (s->mass[i] * amu_a2_fs2_ev());
    for (int b = 0; b < s->P; ++b) {
        size_t e = ((size_t)b * s->N + i) * 3 + a;
        v[e] = v[e] + F[e] * f;
    }
}

static void free_A(const rp_t *s, double *q, double *v, int i, int a)
{
    int P = s->P, N = s->N;
    double *qt = (double *)malloc(sizeof(double) * P), *vt = (double *)malloc(sizeof(double) * P);
    for (int k = 0; k < P; ++k) {
        double sq = 0.0, sv = 0.0;
        for (int b = 0; b < P; ++b) {
            size_t e = ((size_t)b * N + i) * 3 + a;
            sq += q[e] * s->C[b * P + k];
            sv += v[e] * s->C[b * P + k];
        }
        qt[k] = sq; vt[k] = sv;
    }
    for (int k = 0; k < P; ++k) {
        /* Eqs. (5)-(6) in velocity form, simultaneous update */
        double h = 0.5 * s->w[k] * s->dt;
        double den = 1.0 + h * h;
        double cq = (1.0 - h * h) / den;
        double qv = s->dt / den;                       /* sin-like / (m w) in velocity form */
        double vq = s->w[k] * s->w[k] * s->dt / den;   /* m w * sin-like in velocity form */
        double qn = cq * qt[k] + qv * vt[k];
        double vn = cq * vt[k] - vq * qt[k];
        qt[k] = qn; vt[k] = vn;
    }
    for (int b = 0; b < P; ++b) {
        double sq = 0.0, sv = 0.0;
        for (int k = 0; k < P; ++k) {
            sq += s->C[b * P + k] * qt[k];
            sv += s->C[b * P + k] * vt[k];
        }
        size_t e = ((size_t)b * N + i) * 3 + a;
        q[e] = sq; v[e] = sv;
    }
    free(qt); free(vt);
}

/* One integrator stage on pos/vel [P,N,3] with forces F [P,N,3] (eV/A).
 * stage PRE = O B A (noise stage 0 of `step`), POST = B O (noise stage 1 of
 * `step`), FUSED = POST(step) then PRE(step + 1). */
int or_trpmd_stage(int P, int N, int mode, double dt, double T, double tau, uint64_t seed,
                   const double *mass, double *pos, double *vel, const double *F, int64_t step, int stage)
{
    if (P < 1 || N < 0 || mode < 0 || mode > 2 || stage < 0 || stage > 2) return 1;
    rp_t s = {P, N, mode, dt, T, tau, seed, mass, NULL, NULL, NULL, NULL};
    s.C = (double *)malloc(sizeof(double) * P * P);
    s.w = (double *)malloc(sizeof(double) * P);
    s.c1 = (double *)malloc(sizeof(double) * P);
    s.c2 = (double *)malloc(sizeof(double) * P);
    or_nm_matrix(P, s.C);
    or_nm_freqs(P, T, s.w);
    for (int k = 0; k < P; ++k) {
        double g = (k == 0) ? 1.0 / tau : s.w[k];
        s.c1[k] = exp(-0.5 * dt * g);
        s.c2[k] = sqrt(1.0 - s.c1[k] * s.c1[k]);
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (int a = 0; a < 3; ++a) {
            if (stage == OR_POST || stage == OR_FUSED) {
                kick_B(&s, vel, F, i, a);
                thermo_O(&s, vel, i, a, step, 1);
            }
            if (stage == OR_PRE || stage == OR_FUSED) {
                int64_t st = (stage == OR_FUSED) ? step + 1 : step;
                thermo_O(&s, vel, i, a, st, 0);
                kick_B(&s, vel, F, i, a);
                free_A(&s, pos, vel, i, a);
            }
        }
    free(s.C); free(s.w); free(s.c1); free(s.c2);
    return 0;
}

/* Free ring-polymer Cayley map coefficients for tests: per mode
 * [cq, qv, vq] so that q' = cq q + qv v, v' = cq v - vq q. */
void or_cayley_coeffs(int P, double T, double dt, double *out)
{
    double *w = (double *)malloc(sizeof(double) * P);
    or_nm_freqs(P, T, w);
    for (int k = 0; k < P; ++k) {
        double h = 0.5 * w[k] * dt, den = 1.0 + h * h;
        out[3 * k] = (1.0 - h * h) / den;
        out[3 * k + 1] = dt / den;
        out[3 * k + 2] = w[k] * w[k] * dt / den;
    }
    free(w);
}

/* ------------------------------------------------------------------ */
/* Observables of the ring polymer (Sec. II.A: kinetic energy by the    */
/* centroid virial estimator, the virial tensor and the pressure        */
/* tensor) and the Berendsen-like pressure control of the workflow      */
/* (Sec. II.D).                                                          */
/*                                                                      */
/* Readings:                                                            */
/*  - The centroid of atom i follows the periodic boundaries: each bead  */
/*    is first brought to the image nearest bead 1 of the same atom,     */
/*    r~_j = r_1 + mic(r_j - r_1), and r_c = (1/P) sum_j r~_j; bead       */
/*    displacements from it are r~_j - r_c.  For unwrapped ring polymers  */
/*    (all beads of an atom in one image) this is the plain mean.        */
/*  - T in K and N kB T is the physical temperature's term; the pressure */
/*    tensor is (N kB T 1 + W) / V with W the centroid virial tensor      */
/*    (outer product with the displacement first, the force second) plus */
/*    the bead average of the potential's virial.                        */
/*  - Pressure control: mu_a = 1 - beta dt / (3 tau_p) (p0_a - p_a), with */
/*    p_a = P_aa (anisotropic) or tr(P) / 3 for every axis (isotropic);   */
/*    every bead coordinate and box edge is multiplied by mu_a.  Pressure */
/*    in GPa, beta (compressibility) in 1/GPa, dt and tau_p in fs.        */
/* ------------------------------------------------------------------ */

/* 1 eV / A^3 in GPa */
static double ev_a3_gpa(void) { return 1.602176634e-19 / 1e-30 / 1e9; }

/* minimum image and cell volume of the NEP oracle (box [9]: edge vectors as rows) */
void or_mic(const double *ri, const double *rj, const double *box, double *d, double *r2);
double or_cell_volume(const double *box);

/* out[0]  potential energy, mean of E_bead over the beads (eV)
 * out[1]  kinetic energy K = 3/2 N kB T - 1/2 sum_i (1/P) sum_j dr_j . F_j (eV)
 * out[2..10]  W_ab = -sum_i (1/P) sum_j dr_j,a F_j,b + (1/P) sum_j W_bead[j][ab] (eV)
 * out[11..19] pressure tensor (N kB T delta_ab + W_ab) / V (GPa)
 * out[20] scalar pressure tr / 3 (GPa)
 * pos [P][N][3], F [P][N][3] (eV/A), W_bead [P][9], E_bead [P], box [9] (A,
 * edge vectors as rows; V its determinant). */
void or_observables(int P, int N, const double *pos, const double *F, const double *W_bead, const double *E_bead,
                    const double *box, double T, double *out)
{
    double Wcv[9] = {0};
    for (int i = 0; i < N; ++i) {
        const double *r1 = pos + (size_t)i * 3;
        double rc[3] = {0, 0, 0};
        for (int j = 0; j < P; ++j) {
            double d[3], r2;
            or_mic(r1, pos + ((size_t)j * N + i) * 3, box, d, &r2);
            for (int a = 0; a < 3; ++a) rc[a] += r1[a] + d[a];
        }
        for (int a = 0; a < 3; ++a) rc[a] /= P;
        for (int j = 0; j < P; ++j) {
            double d[3], r2, dr[3];
            or_mic(r1, pos + ((size_t)j * N + i) * 3, box, d, &r2);
            for (int a = 0; a < 3; ++a) dr[a] = r1[a] + d[a] - rc[a];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Wcv[a * 3 + b] += dr[a] * F[((size_t)j * N + i) * 3 + b];
        }
    }
    double Wpot[9] = {0}, Epot = 0.0;
    for (int j = 0; j < P; ++j) {
        Epot += E_bead[j];
        for (int e = 0; e < 9; ++e) Wpot[e] += W_bead[j * 9 + e];
    }
    const double NkT = N * OR_KB * T, V = or_cell_volume(box);
    out[0] = Epot / P;
    out[1] = 1.5 * NkT - 0.5 * (Wcv[0] + Wcv[4] + Wcv[8]) / P;
    for (int e = 0; e < 9; ++e) {
        out[2 + e] = -Wcv[e] / P + Wpot[e] / P;
        out[11 + e] = ((e % 4 == 0 ? NkT : 0.0) + out[2 + e]) / V * ev_a3_gpa();
    }
    out[20] = (out[11] + out[15] + out[19]) / 3.0;
}

/* Berendsen-like scaling: mu[3] from the pressure tensor ptens[9] (GPa), then
 * every Cartesian coordinate a of pos [P][N][3] and of the cell's edge
 * vectors box [9] (rows) multiplied by mu[a], in place. */
void or_berendsen(int P, int N, double *pos, double *box, const double *ptens, const double *p0, double beta,
                  double tau_p, double dt, int aniso, double *mu)
{
    const double p_iso = (ptens[0] + ptens[4] + ptens[8]) / 3.0;
    for (int a = 0; a < 3; ++a) {
        const double p = aniso ? ptens[a * 4] : p_iso;
        mu[a] = 1.0 - beta * dt / (3.0 * tau_p) * (p0[a] - p);
    }
    for (size_t e = 0; e < (size_t)P * N; ++e)
        for (int a = 0; a < 3; ++a) pos[e * 3 + a] *= mu[a];
    for (int r = 0; r < 3; ++r)
        for (int a = 0; a < 3; ++a) box[3 * r + a] *= mu[a];
}
