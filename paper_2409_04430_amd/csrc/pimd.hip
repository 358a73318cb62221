// Ring-polymer integrator on gfx950 (Sec. II.A of arXiv:2409.04430):
// normal-mode transform (Eqs. (3)-(4), (7)-(8)), Cayley free ring-polymer
// step (Eqs. (5)-(6)), half kick (Eq. (9)) and the Langevin thermostat on
// normal-mode momenta (Eqs. (10)-(12)).
//
// P lanes per (atom, Cartesian component), one per normal mode, with the
// element's bead and mode vectors staged in LDS.  Because C is orthogonal, the
// kicks and the thermostat of a stage are applied in mode space: a stage
// maps each mode as v~ <- alpha_k v~ + beta_k hk F~ + gamma_k, with
//   PRE   (O then B):        alpha = c1, beta = 1,          gamma = sig c2 xi0
//   POST  (B then O):        alpha = c1, beta = c1,         gamma = sig c2 xi1
//   FUSED (B, O, O, B):      alpha = c1^2, beta = c1^2 + 1, gamma = sig c2 (c1 xi1 + xi0)
// (c1 = 1, c2 = 0 on modes that are not thermostatted), followed for PRE
// and FUSED by the Cayley map.  The bead data move once: read q, v, F and
// write q, v.
#include <cmath>

#include "internal.hpp"

namespace nep {

constexpr double kKB = 8.617333262e-5;     // eV/K
constexpr double kHbar = 0.6582119569;     // eV fs
// 1 amu A^2/fs^2 in eV
inline double amu_a2_fs2_ev() { return 1.66053906660e-27 * 1e10 / 1.602176634e-19; }
// 1 eV/A^3 in GPa
inline double ev_a3_gpa() { return 1.602176634e-19 / 1e-30 / 1e9; }

// Offsets into the per-context constant block.
struct PimdLayout {
    int P;
    int C, c1, sc2, cq, qv, vq, total;
    __host__ __device__ explicit PimdLayout(int p) : P(p)
    {
        C = 0;
        c1 = P * P;
        sc2 = c1 + P;
        cq = sc2 + P;
        qv = cq + P;
        vq = qv + P;
        total = vq + P;
    }
};

// ---------------------------------------------------- Philox-4x32-10 ---
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC'11: ten rounds of two 32x32->64 multiplies with Weyl key schedule.
__device__ __forceinline__ void philox4x32_10(uint32_t k0, uint32_t k1, uint32_t c[4])
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// Philox block kb of component a of atom i for (step, stage).
__device__ __forceinline__ void noise_block(uint64_t seed, uint64_t step, int stage, int i, int a, int nb, int kb,
                                            uint32_t (&c)[4])
{
    c[0] = (uint32_t)i;
    c[1] = (uint32_t)(a * nb + kb);
    c[2] = (uint32_t)step;
    c[3] = (uint32_t)((step >> 32) * 2u + (uint64_t)stage);
    philox4x32_10((uint32_t)seed, (uint32_t)(seed >> 32), c);
}

// Box-Muller pair from two Philox words (uniforms (x + 1) 2^-32).
__device__ __forceinline__ void box_muller(uint32_t x0, uint32_t x1, double &zc, double &zs)
{
    const double s = 1.0 / 4294967296.0;
    const double u0 = ((double)x0 + 1.0) * s;
    const double u1 = ((double)x1 + 1.0) * s;
    const double rad = sqrt(-2.0 * log(u0));
    double sn, cs;
    sincospi(2.0 * u1, &sn, &cs);   // the angle 2 pi u1, without a range reduction by pi
    zc = rad * cs;
    zs = rad * sn;
}

// Standard normal e4 (0..3) of block kb of component a of atom i: the
// block's Philox output gives two Box-Muller pairs, normals 0, 1 from the
// first pair (cosine, sine) and 2, 3 from the second.  Each lane evaluates
// only its own pair (kept out of line: one copy of the FP64 Box-Muller code).
__device__ __noinline__ double normal1(uint64_t seed, uint64_t step, int stage, int i, int a, int nb, int kb, int e4)
{
    uint32_t c[4];
    noise_block(seed, step, stage, i, a, nb, kb, c);
    const bool second = e4 >= 2;
    double zc, zs;
    box_muller(second ? c[2] : c[0], second ? c[3] : c[1], zc, zs);
    return (e4 & 1) ? zs : zc;
}

// All four normals of block kb (the values normal1 returns for e4 = 0..3).
__device__ __forceinline__ void normal4(uint64_t seed, uint64_t step, int stage, int i, int a, int nb, int kb,
                                     double (&z)[4])
{
    uint32_t c[4];
    noise_block(seed, step, stage, i, a, nb, kb, c);
    box_muller(c[0], c[1], z[0], z[1]);
    box_muller(c[2], c[3], z[2], z[3]);
}

struct StepArgs {
    double *pos, *vel;
    const float *F;
    const double *mass;
    int N, P;
    double dt, kTP, conv;
    uint64_t seed;
    int64_t step;
    const int64_t *step_dev;   // if set, the step number is read from device memory
    int64_t *step_out;         // if set (device counter mode), step + 1 is written there by a closing stage
    int stage, noise;
    PendingReduce red;         // energy/virial sums completed by this launch (red.nout = 0: none)
    int int_blocks = 0;        // workgroups of the integrator proper; later ones carry the sums
};

// The pending sums on their own launch (integrator forms without the fold).
__global__ __launch_bounds__(64) void k_reduce_pending(PendingReduce r)
{
    reduce_output(r, blockIdx.x, threadIdx.x);
}

// One workgroup holds floor(512 / P) (atom, component) elements; lane
// (element, k) works on normal mode k of its element (and bead k for the
// back transform), so every P x P transform becomes P-long dot products
// spread over P lanes.  Bead data, mode data and C are staged in LDS; global
// loads and stores run over consecutive elements of one bead.
constexpr int kStepBlock = 512;
__global__ __launch_bounds__(kStepBlock) void k_trpmd(StepArgs a, const double *__restrict__ cst)
{
    extern __shared__ double sh[];
    const int P = a.P;
    const int EPB = kStepBlock / P;
    const PimdLayout Lo(P);
    double *Cs = sh;                 // [P][P]: C[b][k]
    double *vb = Cs + P * P;         // [EPB][P]
    double *qb = vb + EPB * P;
    double *fb = qb + EPB * P;
    const int M = 3 * a.N;
    const int e0 = blockIdx.x * EPB;
    const int t = threadIdx.x;
    const bool pre = a.stage != PIMD_STAGE_POST, post = a.stage != PIMD_STAGE_PRE;
    const int64_t step = a.step_dev ? *a.step_dev : a.step;
    // the next step's counter (a different word: every workgroup reads step_dev)
    if (a.step_out && post && blockIdx.x == 0 && threadIdx.x == 0) *a.step_out = step + 1;

    for (int x = t; x < P * P; x += blockDim.x) Cs[x] = cst[Lo.C + x];
    for (int x = t; x < EPB * P; x += blockDim.x) {
        const int b = x / EPB, el = x - b * EPB, e = e0 + el;
        double v = 0.0, q = 0.0, f = 0.0;
        if (e < M) {
            v = a.vel[(size_t)b * M + e];
            f = (double)a.F[(size_t)b * M + e];
            if (pre) q = a.pos[(size_t)b * M + e];
        }
        vb[el * P + b] = v;
        qb[el * P + b] = q;
        fb[el * P + b] = f;
    }
    __syncthreads();

    const int el = t / P, k = t - el * P;
    const bool act = el < EPB && e0 + el < M;
    double qn = 0.0, vn = 0.0;
    if (act) {
        const int e = e0 + el;
        const int i = e / 3, comp = e - 3 * i;
        const double m = a.mass[i];
        const double hk = 0.5 * a.dt / (m * a.conv);
        const double sig = sqrt(a.kTP / (m * a.conv));
        double vt = 0.0, ft = 0.0, qt = 0.0;
        for (int b = 0; b < P; ++b) {
            const double c = Cs[b * P + k];
            vt += c * vb[el * P + b];
            ft += c * fb[el * P + b];
            if (pre) qt += c * qb[el * P + b];
        }
        const double c1 = cst[Lo.c1 + k];
        double alpha = c1, beta = 1.0, gamma = 0.0;
        if (a.stage == PIMD_STAGE_POST) beta = c1;
        if (a.stage == PIMD_STAGE_FUSED) {
            alpha = c1 * c1;
            beta = c1 * c1 + 1.0;
        }
        if (a.noise) {
            const int NB = (P + 3) / 4, kb = k >> 2, e4 = k & 3;
            const double gs = sig * cst[Lo.sc2 + k];
            if (a.stage == PIMD_STAGE_FUSED) {
                const double z1 = normal1(a.seed, (uint64_t)step, 1, i, comp, NB, kb, e4);
                const double z0 = normal1(a.seed, (uint64_t)(step + 1), 0, i, comp, NB, kb, e4);
                gamma = gs * (c1 * z1 + z0);
            } else {
                gamma = gs * normal1(a.seed, (uint64_t)step, post ? 1 : 0, i, comp, NB, kb, e4);
            }
        }
        vt = alpha * vt + gamma + beta * (hk * ft);
        if (pre) {
            const double cq = cst[Lo.cq + k], qv = cst[Lo.qv + k], vq = cst[Lo.vq + k];
            qn = cq * qt + qv * vt;
            vn = cq * vt - vq * qt;
        } else {
            vn = vt;
        }
    }
    __syncthreads();
    if (act) {
        vb[el * P + k] = vn;
        qb[el * P + k] = qn;
    }
    __syncthreads();
    double sv = 0.0, sq = 0.0;
    if (act) {   // back transform: lane (element, bead k)
        for (int kk = 0; kk < P; ++kk) {
            const double c = Cs[k * P + kk];
            sv += c * vb[el * P + kk];
            if (pre) sq += c * qb[el * P + kk];
        }
    }
    __syncthreads();
    if (act) {
        vb[el * P + k] = sv;
        qb[el * P + k] = sq;
    }
    __syncthreads();
    for (int x = t; x < EPB * P; x += blockDim.x) {
        const int b = x / EPB, elx = x - b * EPB, e = e0 + elx;
        if (e < M) {
            a.vel[(size_t)b * M + e] = vb[elx * P + b];
            if (pre) a.pos[(size_t)b * M + e] = qb[elx * P + b];
        }
    }
}

// The same stage with the mode transforms on the matrix cores, for P a
// multiple of 16: both transforms are products with the P x P matrix C over
// a block of elements, (C^T X) and (C X~), done as 16 x 16 x 4 FP64 tiles.
// A pair of wavefronts takes 16 elements and one 16-mode tile, each summing
// over half of the beads (forward) and half of the modes (back): the bead
// values come straight from the bead-major arrays as B fragments (16
// consecutive elements of one bead per lane group); the second wavefront's
// partial tiles meet the first's in LDS, in a fixed order; the per-mode
// update runs on the result tile (lane j + 16 g holds modes g, g + 4, g + 8,
// g + 12 of the tile for element j); the new mode vectors of all mode tiles
// meet in LDS, and each pair back-transforms one 16-bead tile.  The tile's
// thermostat normals (16 elements x 16 modes, 16 x 4 Philox blocks per
// draw) are drawn once each, the two draws of the fused stage by the two
// wavefronts of the pair: lane j + 16 g draws block 4 mt + g of element j
// and leaves its four normals in LDS for the lanes that hold those modes.
// FP64 fragment layout: A(i, k) in lane i + 16 k, B(k, j) in lane j + 16 k,
// result (i, j) in lane j + 16 (i % 4), slot i / 4.
typedef double f64x4 __attribute__((ext_vector_type(4)));
// Workgroup: ET element tiles x MT mode tiles x 2 halves, one wavefront each (8 or 6).
template <int P> constexpr int step_mf_et() { return P == 48 ? 1 : 64 / P; }
constexpr int kStepHalves = 2;

template <int P>
__global__ __launch_bounds__(64 * 8) void k_trpmd_mf(StepArgs a, const double *__restrict__ cst)
{
    static_assert(P % 16 == 0 && P <= 64, "matrix-core stage needs P = 16, 32, 48 or 64");
    constexpr int MT = P / 16, KS = P / 4, ET = step_mf_et<P>(), NT = ET * MT, KH = KS / kStepHalves;
    __shared__ double xt[ET][2][P][16];        // new mode vectors v~, q~ of each element tile
    __shared__ double zn[NT][2][16][16];       // thermostat normals [tile][draw][mode in tile][element]
    __shared__ f64x4 part[NT][3][64];          // the second half's partial tiles (forward v, f, q; back v, q)
    if ((int)blockIdx.x >= a.int_blocks) {
        // workgroups past the integrator's: one wavefront per output of the
        // pending energy/virial sums (independent of the stage's data)
        const int o = ((int)blockIdx.x - a.int_blocks) * ((int)blockDim.x >> 6) + ((int)threadIdx.x >> 6);
        if (o < a.red.nout) reduce_output(a.red, o, threadIdx.x & 63);
        return;
    }
    const PimdLayout Lo(P);
    const int M = 3 * a.N;
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lg = l >> 4;
    const int tile = wv % NT, half = wv / NT;
    const int et = tile / MT, mt = tile - et * MT;   // this pair's element tile and 16-mode (16-bead) tile
    const int e0 = (blockIdx.x * ET + et) * 16;
    const int e = e0 + lr;
    const bool ok = e < M;
    const bool pre = a.stage != PIMD_STAGE_POST, post = a.stage != PIMD_STAGE_PRE;
    const int64_t step = a.step_dev ? *a.step_dev : a.step;
    // the next step's counter (a different word: every workgroup reads step_dev)
    if (a.step_out && post && blockIdx.x == 0 && threadIdx.x == 0) *a.step_out = step + 1;
    const double *C = cst + Lo.C;   // C[b * P + k]
    const int ks0 = half * KH;      // this wavefront's beads (forward) and modes (back): 4 ks + lg

    // bead values of the element tile, all loads in flight at once (lanes
    // past the last element read element 0 and drop it) and issued before
    // the noise draws, which do not depend on them
    double xv[KH], xq[KH], cf[KH], cb[KH];
    float xf[KH];
#pragma unroll
    for (int h = 0; h < KH; ++h) {
        const int ks = ks0 + h;
        const size_t at = (size_t)(4 * ks + lg) * M + (ok ? e : 0);
        xv[h] = a.vel[at];
        xf[h] = a.F[at];
        xq[h] = pre ? a.pos[at] : 0.0;
        cf[h] = C[(size_t)(4 * ks + lg) * P + 16 * mt + lr];   // C^T(mode 16 mt + lr, bead 4 ks + lg)
        cb[h] = C[(size_t)(16 * mt + lr) * P + 4 * ks + lg];   // C(bead 16 mt + lr, mode 4 ks + lg)
    }
    const int i = e / 3, comp = e - 3 * i;
    const int NB = (P + 3) / 4;
    const bool fused = a.stage == PIMD_STAGE_FUSED;
    if (a.noise && (fused || half == 0)) {
        // draw 0 (first half): (step, closing half, or the stage's own half);
        // the fused stage's draw 1 (second half): (step + 1, opening half)
        const int d = half;
        double z4[4];
        normal4(a.seed, (uint64_t)step + (uint64_t)d, fused ? 1 - d : (post ? 1 : 0), i, comp, NB, 4 * mt + lg, z4);
#pragma unroll
        for (int q = 0; q < 4; ++q) zn[tile][d][4 * lg + q][lr] = z4[q];
    }

    // forward, modes 16 mt .. 16 mt + 15, this half's beads: v~ = C^T v, f~ = C^T F, q~ = C^T q
    f64x4 vt = {0.0, 0.0, 0.0, 0.0}, ft = {0.0, 0.0, 0.0, 0.0}, qt = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int h = 0; h < KH; ++h) {
        vt = __builtin_amdgcn_mfma_f64_16x16x4f64(cf[h], ok ? xv[h] : 0.0, vt, 0, 0, 0);
        ft = __builtin_amdgcn_mfma_f64_16x16x4f64(cf[h], ok ? (double)xf[h] : 0.0, ft, 0, 0, 0);
        if (pre) qt = __builtin_amdgcn_mfma_f64_16x16x4f64(cf[h], ok ? xq[h] : 0.0, qt, 0, 0, 0);
    }
    if (half == 1) {
        part[tile][0][l] = vt;
        part[tile][1][l] = ft;
        part[tile][2][l] = qt;
    }
    __syncthreads();   // the normals and the second half's partial tiles are in LDS

    if (half == 0) {
        vt += part[tile][0][l];
        ft += part[tile][1][l];
        if (pre) qt += part[tile][2][l];
        const double mi = a.mass[ok ? i : 0];
        const double m = ok ? mi : 1.0;
        const double hk = 0.5 * a.dt / (m * a.conv);
        const double sig = sqrt(a.kTP / (m * a.conv));
        // per (mode, element): thermostat, kicks and the Cayley map, for
        // this lane's four modes k = 16 mt + lg + 4 s4
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int k = 16 * mt + lg + 4 * s4;
            const double c1 = cst[Lo.c1 + k];
            double alpha = c1, beta = 1.0, gamma = 0.0;
            if (a.stage == PIMD_STAGE_POST) beta = c1;
            if (fused) {
                alpha = c1 * c1;
                beta = c1 * c1 + 1.0;
            }
            if (a.noise && ok) {
                // normal k & 3 of block k >> 2: mode k - 16 mt = lg + 4 s4 of the tile
                const double gs = sig * cst[Lo.sc2 + k];
                const double z1 = zn[tile][0][lg + 4 * s4][lr];
                gamma = fused ? gs * (c1 * z1 + zn[tile][1][lg + 4 * s4][lr]) : gs * z1;
            }
            const double v1 = alpha * vt[s4] + gamma + beta * (hk * ft[s4]);
            double vn = v1, qn = 0.0;
            if (pre) {
                const double cq = cst[Lo.cq + k], qv = cst[Lo.qv + k], vq = cst[Lo.vq + k];
                qn = cq * qt[s4] + qv * v1;
                vn = cq * v1 - vq * qt[s4];
            }
            xt[et][0][k][lr] = vn;
            xt[et][1][k][lr] = qn;
        }
    }
    __syncthreads();   // every mode tile of the element tile is in LDS; part is free

    // back transform, beads 16 mt .. 16 mt + 15, this half's modes: v = C v~, q = C q~
    f64x4 vb = {0.0, 0.0, 0.0, 0.0}, qb = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int h = 0; h < KH; ++h) {
        const int k = 4 * (ks0 + h) + lg;
        vb = __builtin_amdgcn_mfma_f64_16x16x4f64(cb[h], xt[et][0][k][lr], vb, 0, 0, 0);
        if (pre) qb = __builtin_amdgcn_mfma_f64_16x16x4f64(cb[h], xt[et][1][k][lr], qb, 0, 0, 0);
    }
    if (half == 1) {
        part[tile][0][l] = vb;
        part[tile][1][l] = qb;
    }
    __syncthreads();   // the second half's partial tiles are in LDS
    if (half == 0 && ok) {
        vb += part[tile][0][l];
        if (pre) qb += part[tile][1][l];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const size_t at = (size_t)(16 * mt + lg + 4 * s4) * M + e;
            a.vel[at] = vb[s4];
            if (pre) a.pos[at] = qb[s4];
        }
    }
}


// ------------------------------------------------------- observables ---
//
// Centroid virial estimator of the kinetic energy, the virial tensor and the
// pressure tensor (Sec. II.A).  One lane per (atom, bead), the P beads of an
// atom in G = 2^ceil(log2 P) adjacent lanes.  A bead's displacement from the
// centroid is taken through the periodic boundaries: each bead is brought to
// the image nearest the atom's first bead, r~_j = r_1 + mic(r_j - r_1), and
// dr_j = r~_j - mean_k r~_k.  Each workgroup reduces its lanes' dr (x) F to
// nine FP64 partial sums in a fixed order; a second launch of one workgroup
// reduces the partials in a fixed order and forms the outputs (bitwise
// reproducible).  A last-workgroup ticket in one launch was slower: the
// device-scope fence each workgroup then needs costs more than a launch.

constexpr int kObsBlock = 256;

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

struct ObsCell {
    double L[3];          // orthorhombic edges
    double H[9], G[9];    // general cell: edge vectors as rows and H^-1
    int tri;
};

struct ObsFinal {
    const double *part;        // [nblk][9] partial sums
    int nblk;
    const double *Wb, *Eb;
    int P, N;
    double NkT, inv_vol_gpa;   // N kB T (eV); 1 / V in GPa per eV
    double *out;
};

__global__ __launch_bounds__(kObsBlock) void k_obs_partial(const double *__restrict__ pos, const float *__restrict__ F,
                                                           int N, int P, int lg, ObsCell cell,
                                                           double *__restrict__ part)
{
    const int G = 1 << lg;
    const int t = blockIdx.x * kObsBlock + threadIdx.x;
    const int i = t >> lg, b = t & (G - 1);
    const bool valid = i < N && b < P;
    double rel[3] = {0.0, 0.0, 0.0}, f[3] = {0.0, 0.0, 0.0};
    if (valid) {
        const double *r = pos + ((size_t)b * N + i) * 3;
        const double *r1 = pos + (size_t)i * 3;
        const float *fb = F + ((size_t)b * N + i) * 3;
        const double d[3] = {r[0] - r1[0], r[1] - r1[1], r[2] - r1[2]};
        if (cell.tri) {
            double fr[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double sc = d[0] * cell.G[c] + d[1] * cell.G[3 + c] + d[2] * cell.G[6 + c];
                fr[c] = sc - rint(sc);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) rel[a] = fr[0] * cell.H[a] + fr[1] * cell.H[3 + a] + fr[2] * cell.H[6 + a];
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) rel[a] = d[a] - cell.L[a] * rint(d[a] / cell.L[a]);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) f[a] = (double)fb[a];
    }
    // mean over the atom's beads (lanes b >= P hold zeros)
    double dr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double sa = rel[a];
        for (int o = 1; o < G; o <<= 1) sa += __shfl_xor(sa, o);
        dr[a] = valid ? rel[a] - sa / P : 0.0;
    }
    __shared__ double red[kObsBlock / 64][9];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = wave_sum(dr[a] * f[c]);
            if (lane == 0) red[w][a * 3 + c] = v;
        }
    __syncthreads();
    if (threadIdx.x < 9) {
        double acc = 0.0;
        for (int k = 0; k < kObsBlock / 64; ++k) acc += red[k][threadIdx.x];
        part[(size_t)blockIdx.x * 9 + threadIdx.x] = acc;
    }

}

__global__ __launch_bounds__(kObsBlock) void k_obs_final(ObsFinal a)
{
    // nine running sums per thread over the partials, then one LDS tree
    __shared__ double tree[9][kObsBlock];
    __shared__ double wcv[9];
    {
        double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int k = threadIdx.x; k < a.nblk; k += kObsBlock)
#pragma unroll
            for (int e = 0; e < 9; ++e) acc[e] += a.part[(size_t)k * 9 + e];
#pragma unroll
        for (int e = 0; e < 9; ++e) tree[e][threadIdx.x] = acc[e];
    }
    __syncthreads();
    for (int h = kObsBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h)
#pragma unroll
            for (int e = 0; e < 9; ++e) tree[e][threadIdx.x] += tree[e][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 9) wcv[threadIdx.x] = tree[threadIdx.x][0];
    __syncthreads();
    if (threadIdx.x == 0) {
        double Ep = 0.0, Wp[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int j = 0; j < a.P; ++j) {
            Ep += a.Eb[j];
            for (int e = 0; e < 9; ++e) Wp[e] += a.Wb[j * 9 + e];
        }
        a.out[PIMD_OBS_EPOT] = Ep / a.P;
        a.out[PIMD_OBS_KINETIC] = 1.5 * a.NkT - 0.5 * (wcv[0] + wcv[4] + wcv[8]) / a.P;
        for (int e = 0; e < 9; ++e) {
            const double W = (Wp[e] - wcv[e]) / a.P;
            a.out[PIMD_OBS_VIRIAL + e] = W;
            a.out[PIMD_OBS_PRESSURE + e] = ((e % 4 == 0 ? a.NkT : 0.0) + W) * a.inv_vol_gpa;
        }
        a.out[PIMD_OBS_PSCALAR] =
            (a.out[PIMD_OBS_PRESSURE] + a.out[PIMD_OBS_PRESSURE + 4] + a.out[PIMD_OBS_PRESSURE + 8]) / 3.0;
    }
}

// Berendsen-like pressure control (Sec. II.D): per axis
// mu_a = 1 - c (p0_a - p_a), c = beta dt / (3 tau_p), p_a the diagonal
// pressure (anisotropic) or tr(P) / 3 (isotropic); every bead coordinate is
// multiplied by mu of its axis.  The factors are also written to mu[3].
__global__ __launch_bounds__(256) void k_berendsen(double *__restrict__ pos, int64_t M, const double *__restrict__ obs,
                                                   double p0x, double p0y, double p0z, double c, int aniso,
                                                   double *__restrict__ mu_out)
{
    const double *pt = obs + PIMD_OBS_PRESSURE;
    const double piso = (pt[0] + pt[4] + pt[8]) / 3.0;
    const double mu[3] = {1.0 - c * (p0x - (aniso ? pt[0] : piso)), 1.0 - c * (p0y - (aniso ? pt[4] : piso)),
                          1.0 - c * (p0z - (aniso ? pt[8] : piso))};
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < M) pos[e] *= mu[e % 3];
    if (e < 3) mu_out[e] = mu[e];
}

template <int P>
__global__ __launch_bounds__(256) void k_modes(const double *__restrict__ in, double *__restrict__ out, int M,
                                               int dir, const double *__restrict__ cst)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= M) return;
    double x[P];
#pragma unroll
    for (int b = 0; b < P; ++b) x[b] = in[(size_t)b * M + e];
#pragma unroll 1
    for (int o = 0; o < P; ++o) {
        double s = 0.0;
        if (dir > 0) {
#pragma unroll
            for (int k = 0; k < P; ++k) s += cst[k * P + o] * x[k];
        } else {
#pragma unroll
            for (int k = 0; k < P; ++k) s += cst[o * P + k] * x[k];
        }
        out[(size_t)o * M + e] = s;
    }
}

static void launch_step(StepArgs a, const double *cst, hipStream_t s)
{
    ProfScope ps_(K_TRPMD, s);
#define NEP_STEP_MF(PP)                                                                                     \
    case PP: {                                                                                              \
        constexpr int waves = step_mf_et<PP>() * (PP / 16) * kStepHalves;                                  \
        a.int_blocks = div_up(3 * a.N, 16 * step_mf_et<PP>());                                             \
        const int extra = div_up(a.red.nout, waves);                                                       \
        hipLaunchKernelGGL(k_trpmd_mf<PP>, dim3(a.int_blocks + extra), dim3(64 * waves), 0, s, a, cst);    \
        return;                                                                                             \
    }
    switch (a.P) {   // matrix-core transforms where P is a multiple of 16
        NEP_STEP_MF(16) NEP_STEP_MF(32) NEP_STEP_MF(48) NEP_STEP_MF(64)
    default: break;
    }
#undef NEP_STEP_MF
    if (a.red.nout > 0) hipLaunchKernelGGL(k_reduce_pending, dim3(a.red.nout), dim3(64), 0, s, a.red);
    const int EPB = kStepBlock / a.P;
    const size_t lds = sizeof(double) * ((size_t)a.P * a.P + 3 * (size_t)EPB * a.P);
    hipLaunchKernelGGL(k_trpmd, dim3(div_up(3 * a.N, EPB)), dim3(kStepBlock), lds, s, a, cst);
}

template <int P>
static void launch_modes(const double *in, double *out, int M, int dir, const double *cst, hipStream_t s)
{
    {
        ProfScope ps_(K_MODES, s);
        hipLaunchKernelGGL(k_modes<P>, dim3(div_up(M, 256)), dim3(256), 0, s, in, out, M, dir, cst);
    }
}

#define NEP_P_CASES(X)                                                                                  \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18)   \
    X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32) X(33) X(34)      \
    X(35) X(36) X(37) X(38) X(39) X(40) X(41) X(42) X(43) X(44) X(45) X(46) X(47) X(48) X(49) X(50)      \
    X(51) X(52) X(53) X(54) X(55) X(56) X(57) X(58) X(59) X(60) X(61) X(62) X(63) X(64)

}  // namespace nep

using namespace nep;

extern "C" int32_t pimd_create(int32_t P, int32_t N, const pimd_params *prm, const double *mass, pimd_ctx **out)
{
    if (!prm || !out) return fail(NEP_ERR_INVALID_ARG, "pimd_create: null argument");
    *out = nullptr;
    if (P < 1 || P > kMaxBeads) return fail(NEP_ERR_UNSUPPORTED, "pimd_create: P=%d outside 1..%d", P, kMaxBeads);
    if (N < 0 || (N > 0 && !mass)) return fail(NEP_ERR_INVALID_ARG, "pimd_create: bad N or mass");
    if (!(prm->dt_fs > 0.0) || !(prm->T_K >= 0.0) || prm->mode < 0 || prm->mode > 2 ||
        (prm->mode == PIMD_MODE_PILE && !(prm->tau_T_fs > 0.0)))
        return fail(NEP_ERR_INVALID_ARG, "pimd_create: bad dt/T/tau/mode");
    pimd_ctx *c = new (std::nothrow) pimd_ctx;
    if (!c) return fail(NEP_ERR_NOMEM, "host allocation failed");
    c->P = P;
    c->N = N;
    c->prm = *prm;
    // host tables
    PimdLayout Lo(P);
    std::vector<double> h(Lo.total, 0.0);
    const double sq = std::sqrt((double)P), sq2 = std::sqrt(2.0 / P);
    for (int b = 0; b < P; ++b) {
        const int j = b + 1;
        for (int k = 0; k < P; ++k) {
            double v;
            if (k == 0) v = 1.0 / sq;
            else if (2 * k == P) v = ((j % 2) ? -1.0 : 1.0) / sq;
            else if (2 * k < P) v = sq2 * std::cos(2.0 * M_PI * j * k / P);
            else v = sq2 * std::sin(2.0 * M_PI * j * k / P);
            h[Lo.C + b * P + k] = v;
        }
    }
    const double wP = P * kKB * prm->T_K / kHbar;
    for (int k = 0; k < P; ++k) {
        const double wk = 2.0 * wP * std::sin(k * M_PI / P);
        const bool th = prm->mode == PIMD_MODE_PILE || (prm->mode == PIMD_MODE_TRPMD && k > 0);
        const double gamma = (k == 0) ? (prm->mode == PIMD_MODE_PILE ? 1.0 / prm->tau_T_fs : 0.0) : wk;
        const double c1 = th ? std::exp(-0.5 * prm->dt_fs * gamma) : 1.0;
        const double c2 = th ? std::sqrt(1.0 - c1 * c1) : 0.0;
        h[Lo.c1 + k] = c1;
        h[Lo.sc2 + k] = c2;
        const double hh = 0.5 * wk * prm->dt_fs, den = 1.0 + hh * hh;
        h[Lo.cq + k] = (1.0 - hh * hh) / den;
        h[Lo.qv + k] = prm->dt_fs / den;
        h[Lo.vq + k] = wk * wk * prm->dt_fs / den;
    }
    c->hC.assign(h.begin(), h.begin() + P * P);
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipMalloc(&c->consts, sizeof(double) * Lo.total);
    if (e == hipSuccess) e = hipMalloc(&c->mass, sizeof(double) * (N > 0 ? N : 1));
    {
        int G = 1;
        while (G < P) G <<= 1;
        c->obs_blocks = (int)(((int64_t)N * G + kObsBlock - 1) / kObsBlock);
        if (e == hipSuccess) e = hipMalloc(&c->obs_part, sizeof(double) * 9 * (c->obs_blocks > 0 ? c->obs_blocks : 1));
    }
    if (e == hipSuccess) e = hipMemcpy(c->consts, h.data(), sizeof(double) * Lo.total, hipMemcpyHostToDevice);
    if (e == hipSuccess && N > 0) e = hipMemcpy(c->mass, mass, sizeof(double) * N, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        pimd_destroy(c);
        return fail(e == hipErrorOutOfMemory ? NEP_ERR_NOMEM : NEP_ERR_HIP, "pimd_create: %s", hipGetErrorString(e));
    }
    *out = c;
    return NEP_OK;
}

extern "C" void pimd_destroy(pimd_ctx *c)
{
    if (!c) return;
    if (c->consts) (void)hipFree(c->consts);
    if (c->mass) (void)hipFree(c->mass);
    if (c->obs_part) (void)hipFree(c->obs_part);
    delete c;
}

extern "C" int32_t rp_normal_modes(const pimd_ctx *c, int32_t dir, const double *in, double *out, hipStream_t s)
{
    if (!c) return fail(NEP_ERR_INVALID_ARG, "rp_normal_modes: null context");
    if (dir != 1 && dir != -1) return fail(NEP_ERR_INVALID_ARG, "rp_normal_modes: dir must be +1 or -1");
    if (c->N == 0) return NEP_OK;
    if (!in || !out || in == out) return fail(NEP_ERR_INVALID_ARG, "rp_normal_modes: bad arrays");
    const int M = 3 * c->N;
    switch (c->P) {
#define X(p) case p: launch_modes<p>(in, out, M, dir, c->consts, s); break;
        NEP_P_CASES(X)
#undef X
    default: return fail(NEP_ERR_UNSUPPORTED, "rp_normal_modes: P=%d", c->P);
    }
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}

static int32_t step_common(const pimd_ctx *c, double *pos, double *vel, const float *F, int64_t step,
                           const int64_t *step_dev, int64_t *step_out, int32_t stage, hipStream_t s,
                           nep_ws *ws = nullptr)
{
    if (!c) return fail(NEP_ERR_INVALID_ARG, "trpmd_step: null context");
    if (stage < PIMD_STAGE_PRE || stage > PIMD_STAGE_FUSED) return fail(NEP_ERR_INVALID_ARG, "trpmd_step: bad stage");
    if (step < 0) return fail(NEP_ERR_INVALID_ARG, "trpmd_step: negative step");
    if (c->N == 0) return NEP_OK;
    if (!pos || !vel || !F) return fail(NEP_ERR_INVALID_ARG, "trpmd_step: null array");
    StepArgs a;
    a.pos = pos; a.vel = vel; a.F = F; a.mass = c->mass; a.N = c->N; a.P = c->P;
    a.dt = c->prm.dt_fs;
    a.kTP = c->P * kKB * c->prm.T_K;
    a.conv = amu_a2_fs2_ev();
    a.seed = c->prm.seed;
    a.step = step;
    a.step_dev = step_dev;
    a.step_out = step_out;
    a.stage = stage;
    a.noise = c->prm.mode != PIMD_MODE_RPMD && !(c->prm.mode == PIMD_MODE_TRPMD && c->P == 1);
    if (c->P < 1 || c->P > kMaxBeads) return fail(NEP_ERR_UNSUPPORTED, "trpmd_step: P=%d", c->P);
    if (ws) {   // the sums are taken once, by this launch
        a.red = ws->pending;
        ws->pending = PendingReduce{};
    }
    launch_step(a, c->consts, s);
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}

extern "C" int32_t trpmd_step(const pimd_ctx *c, double *pos, double *vel, const float *F, int64_t step, int32_t stage,
                              hipStream_t s)
{
    return step_common(c, pos, vel, F, step, nullptr, nullptr, stage, s);
}

extern "C" int32_t trpmd_step_dev(const pimd_ctx *c, double *pos, double *vel, const float *F, const int64_t *step_in,
                                  int64_t *step_out, int32_t stage, hipStream_t s)
{
    if (!step_in) return fail(NEP_ERR_INVALID_ARG, "trpmd_step_dev: null step counter");
    if (stage != PIMD_STAGE_PRE && (!step_out || step_out == step_in))
        return fail(NEP_ERR_INVALID_ARG, "trpmd_step_dev: a closing stage needs an output counter other than the input");
    return step_common(c, pos, vel, F, 0, step_in, stage == PIMD_STAGE_PRE ? nullptr : step_out, stage, s);
}

extern "C" int32_t trpmd_step_nep(const pimd_ctx *c, double *pos, double *vel, const float *F, int64_t step,
                                  const int64_t *step_in, int64_t *step_out, int32_t stage, nep_ws *ws, hipStream_t s)
{
    if (!c || !ws) return fail(NEP_ERR_INVALID_ARG, "trpmd_step_nep: null context or workspace");
    if (ws->pending.nout > 0 && (ws->P != c->P || ws->N != c->N))
        return fail(NEP_ERR_INVALID_ARG, "trpmd_step_nep: workspace P=%d N=%d, integrator P=%d N=%d", ws->P, ws->N,
                    c->P, c->N);
    if (!step_in) return step_common(c, pos, vel, F, step, nullptr, nullptr, stage, s, ws);
    if (stage != PIMD_STAGE_PRE && (!step_out || step_out == step_in))
        return fail(NEP_ERR_INVALID_ARG, "trpmd_step_nep: a closing stage needs an output counter other than the input");
    return step_common(c, pos, vel, F, 0, step_in, stage == PIMD_STAGE_PRE ? nullptr : step_out, stage, s, ws);
}

extern "C" int32_t pimd_observables(const pimd_ctx *c, const double *pos, const float *F, const double *W_bead,
                                    const double *E_bead, const double box[9], double *out, hipStream_t s)
{
    if (!c || !box) return fail(NEP_ERR_INVALID_ARG, "pimd_observables: null argument");
    if ((c->N > 0 && (!pos || !F)) || !W_bead || !E_bead || !out)
        return fail(NEP_ERR_INVALID_ARG, "pimd_observables: null array");
    CellInfo ci;
    if (!cell_info(box, ci)) return fail(NEP_ERR_INVALID_ARG, "pimd_observables: singular, left-handed or non-finite cell");
    ObsCell cell{};
    cell.tri = ci.tri;
    for (int k = 0; k < 9; ++k) {
        cell.H[k] = ci.H[k];
        cell.G[k] = ci.G[k];
    }
    for (int a = 0; a < 3; ++a) cell.L[a] = ci.H[4 * a];
    int lg = 0;
    while ((1 << lg) < c->P) ++lg;
    const int nblk = c->obs_blocks;
    ProfScope ps_(K_OBS, s);
    if (nblk > 0)
        hipLaunchKernelGGL(k_obs_partial, dim3(nblk), dim3(kObsBlock), 0, s, pos, F, c->N, c->P, lg, cell,
                           c->obs_part);
    ObsFinal a;
    a.part = c->obs_part;
    a.nblk = nblk;
    a.Wb = W_bead;
    a.Eb = E_bead;
    a.P = c->P;
    a.N = c->N;
    a.NkT = c->N * kKB * c->prm.T_K;
    a.inv_vol_gpa = ev_a3_gpa() / ci.vol;
    a.out = out;
    hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(kObsBlock), 0, s, a);
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}

extern "C" int32_t pimd_berendsen(const pimd_ctx *c, double *pos, const double *obs, const pimd_barostat *prm,
                                  double *mu, hipStream_t s)
{
    if (!c || !prm) return fail(NEP_ERR_INVALID_ARG, "pimd_berendsen: null argument");
    if (!obs || !mu || (c->N > 0 && !pos)) return fail(NEP_ERR_INVALID_ARG, "pimd_berendsen: null array");
    if (!(prm->beta_per_GPa >= 0.0) || !(prm->tau_p_fs > 0.0) || !std::isfinite(prm->p0_GPa[0]) ||
        !std::isfinite(prm->p0_GPa[1]) || !std::isfinite(prm->p0_GPa[2]) || !std::isfinite(prm->beta_per_GPa) ||
        !std::isfinite(prm->tau_p_fs))
        return fail(NEP_ERR_INVALID_ARG, "pimd_berendsen: bad target pressure, compressibility or tau_p");
    const double cc = prm->beta_per_GPa * c->prm.dt_fs / (3.0 * prm->tau_p_fs);
    const int64_t M = (int64_t)3 * c->P * c->N;
    const int64_t nblk = M > 3 ? (M + 255) / 256 : 1;
    ProfScope ps_(K_BARO, s);
    hipLaunchKernelGGL(k_berendsen, dim3((unsigned)nblk), dim3(256), 0, s, pos, M, obs, prm->p0_GPa[0],
                       prm->p0_GPa[1], prm->p0_GPa[2], cc, prm->anisotropic ? 1 : 0, mu);
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}
