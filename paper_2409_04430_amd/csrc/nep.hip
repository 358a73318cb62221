// NEP energy, forces and virial on gfx950 (site-energy model of Sec. II.C,
// bead forces and virial of Sec. II.A of arXiv:2409.04430).
//
// Four kernels per call, one lane per (bead, atom), neighbours taken from
// the per-bead compact lists built over the shared centroid candidate rows:
//   k_descriptor  radial sums, angular sums A_nlm = sum_j g_n(r_ij) Y_lm(u_ij)
//                 over real orthonormal spherical harmonics, q_nl = sum_m A_nlm^2
//                 (equal to the Legendre double sum by the addition theorem),
//                 the optional (2,2,2) four-body invariant, the tanh network,
//                 and the adjoints: B_nlm = dU_i/dA_nlm and the radial
//                 a_k(t) = sum_n dU_i/dq_n c^{ti t}_nk;
//   k_force_ang   angular pair terms d_ij = dU_i/dr_ij from the atom's own
//                 adjoints, kept per (bead, atom, candidate slot);
//   k_force_rad   radial pair terms (a^i_k(tj) + a^j_k(ti)) f'_k(r) u, the
//                 reverse angular terms d_ji gathered through the reverse
//                 slots, so that F_i = sum_j (dU_i/dr_ij - dU_j/dr_ji) needs no
//                 atomics; per-atom virial -1/2 sum_j r_ij (x) (d_ij - d_ji);
//   k_reduce      per-bead energy and virial from per-block partial sums in
//                 a fixed order (bitwise reproducible).
// The descriptor and angular-force passes run species-uniform groups of
// lanes, which makes every model-coefficient address wave-uniform (scalar
// loads, SGPR operands).  Neighbour loops keep several gathers in flight.
#include "internal.hpp"

namespace nep {

constexpr float kPi = 3.14159265358979f;

struct NepArgs {
    const float4 *p4;   // packed positions [P][N]: offsets in a fine grid cell, cell index bits in w
    const int32_t *types;
    int N, S, H;
    int M[3];            // fine grid cells per axis
    float h[3];          // fine grid spacing L / M
    float rcRinv, rcAinv;
    float kappa4;
    // per-bead lists, slot-major: list[(b * cap + s) * N + i]
    const int32_t *listR, *endR, *listA, *endA, *slotA;
    const uint64_t *maskA;   // [P][WC][N] angular hits per candidate word | hits before the word << 32
    int capR, capA, capC, WC;
    float4 *pairbuf;   // [P][capA][N] dU_j/dr_ji at the receiving atom's list position (w unused)
    // workspace
    float *B;
    float *arad;
    float *Fang;
    int KRP;
    double *partE, *partWa, *partWr;
    uint32_t *flags;
    // outputs
    float *F;
    float *Eatom;
    float *Watom;
    // parameter offsets
    int oR, oA, oq, oW0, ob0, ow1, ob1, osh;
};

// Start and end of species block t in the list of (bead b, atom i).
__device__ __forceinline__ void block_range(const int32_t *end, int b, int t, int N, int i, int &s0, int &s1)
{
    const size_t base = (size_t)b * kMaxSpecies * N + i;
    s0 = t ? end[base + (size_t)(t - 1) * N] : 0;
    s1 = end[base + (size_t)t * N];
}

// Pair vector r_j - r_i from packed positions (see FineGrid).
__device__ __forceinline__ void pair_vec(const float4 &pj, const float4 &pi, const NepArgs &a, float &dx, float &dy,
                                         float &dz)
{
    packed_pair(pj, pi, a.M, a.h, dx, dy, dz);
}

// sin(pi z) and cos(pi z) for z in [0, 1]: with w = z - 1/2, cos(pi z) =
// -sin(pi w) and sin(pi z) = cos(pi w), and |pi w| <= pi/2, where the Taylor
// series through x^13 (sin) and x^14 (cos) is accurate to ~2e-7 in FP32.
__device__ __forceinline__ void sincospi01(float z, float &s, float &c)
{
    const float x = kPi * (z - 0.5f);
    const float x2 = x * x;
    float ps = (float)(-1.0 / 6227020800.0);
    ps = ps * x2 + (float)(1.0 / 39916800.0);
    ps = ps * x2 + (float)(-1.0 / 362880.0);
    ps = ps * x2 + (float)(1.0 / 5040.0);
    ps = ps * x2 + (float)(-1.0 / 120.0);
    ps = ps * x2 + (float)(1.0 / 6.0);
    float sw = x - x * x2 * ps;
    float pc = (float)(-1.0 / 87178291200.0);
    pc = pc * x2 + (float)(1.0 / 479001600.0);
    pc = pc * x2 + (float)(-1.0 / 3628800.0);
    pc = pc * x2 + (float)(1.0 / 40320.0);
    pc = pc * x2 + (float)(-1.0 / 720.0);
    pc = pc * x2 + (float)(1.0 / 24.0);
    pc = pc * x2 + (float)(-1.0 / 2.0);
    float cw = 1.0f + x2 * pc;
    c = -sw;
    s = cw;
}

// f_k(r) = (T_k(x) + 1)/2 f_c(r), x = 2 (r/rc - 1)^2 - 1, f_c = (1 + cos(pi r/rc))/2.
template <int K1>
__device__ __forceinline__ void cheb_f(float r, float rcinv, float *f)
{
    float sn, cs;
    const float z = r * rcinv;
    sincospi01(z, sn, cs);
    const float fc = 0.5f + 0.5f * cs;
    const float y = z - 1.0f;
    const float x = 2.0f * y * y - 1.0f;
    float t0 = 1.0f, t1 = x;
    f[0] = fc;
    if (K1 > 1) f[1] = 0.5f * (x + 1.0f) * fc;
#pragma unroll
    for (int k = 2; k < K1; ++k) {
        const float t2 = 2.0f * x * t1 - t0;
        f[k] = 0.5f * (t2 + 1.0f) * fc;
        t0 = t1;
        t1 = t2;
    }
}

// f_k and df_k/dr.
template <int K1>
__device__ __forceinline__ void cheb_fd(float r, float rcinv, float *f, float *fp)
{
    float sn, cs;
    const float z = r * rcinv;
    sincospi01(z, sn, cs);
    const float fc = 0.5f + 0.5f * cs;
    const float fcp = -0.5f * kPi * rcinv * sn;
    const float y = z - 1.0f;
    const float x = 2.0f * y * y - 1.0f;
    const float dx = 4.0f * y * rcinv;
    float t0 = 1.0f, t1 = x, d0 = 0.0f, d1 = 1.0f;
    f[0] = fc;
    fp[0] = fcp;
    if (K1 > 1) {
        f[1] = 0.5f * (x + 1.0f) * fc;
        fp[1] = 0.5f * dx * fc + 0.5f * (x + 1.0f) * fcp;
    }
#pragma unroll
    for (int k = 2; k < K1; ++k) {
        const float t2 = 2.0f * x * t1 - t0;
        const float d2 = 2.0f * t1 + 2.0f * x * d1 - d0;
        f[k] = 0.5f * (t2 + 1.0f) * fc;
        fp[k] = 0.5f * d2 * dx * fc + 0.5f * (t2 + 1.0f) * fcp;
        t0 = t1; t1 = t2;
        d0 = d1; d1 = d2;
    }
}

// Real spherical harmonics l = 1..4 (m = -l..l) at unit vector (x, y, z);
// c holds the normalisations.
__device__ __forceinline__ void sh_eval(float x, float y, float z, const float *__restrict__ c, float *Y)
{
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    Y[0] = c[0] * y;
    Y[1] = c[1] * z;
    Y[2] = c[2] * x;
    Y[3] = c[3] * x * y;
    Y[4] = c[4] * y * z;
    Y[5] = c[5] * (3.0f * z2 - 1.0f);
    Y[6] = c[6] * x * z;
    Y[7] = c[7] * (x2 - y2);
    Y[8] = c[8] * y * (3.0f * x2 - y2);
    Y[9] = c[9] * x * y * z;
    Y[10] = c[10] * y * (5.0f * z2 - 1.0f);
    Y[11] = c[11] * z * (5.0f * z2 - 3.0f);
    Y[12] = c[12] * x * (5.0f * z2 - 1.0f);
    Y[13] = c[13] * z * (x2 - y2);
    Y[14] = c[14] * x * (x2 - 3.0f * y2);
    Y[15] = c[15] * x * y * (x2 - y2);
    Y[16] = c[16] * y * z * (3.0f * x2 - y2);
    Y[17] = c[17] * x * y * (7.0f * z2 - 1.0f);
    Y[18] = c[18] * y * z * (7.0f * z2 - 3.0f);
    Y[19] = c[19] * (35.0f * z2 * z2 - 30.0f * z2 + 3.0f);
    Y[20] = c[20] * x * z * (7.0f * z2 - 3.0f);
    Y[21] = c[21] * (x2 - y2) * (7.0f * z2 - 1.0f);
    Y[22] = c[22] * x * z * (x2 - 3.0f * y2);
    Y[23] = c[23] * (x2 * (x2 - 3.0f * y2) - y2 * (3.0f * x2 - y2));
}

// sY = sum_m bp_m Y_m(u);  g = sum_m b_m grad p_m(u), where Y_m = c_m p_m and
// the polynomial p_m is differentiated as a function on R^3 (the tangential
// projection is applied by the caller).
__device__ __forceinline__ void sh_contract(float x, float y, float z, const float *__restrict__ c, const float *b,
                                            const float *bp, float &sY, float &gx, float &gy, float &gz)
{
    float Y[kNumSH];
    sh_eval(x, y, z, c, Y);
    float s = 0.0f;
#pragma unroll
    for (int m = 0; m < kNumSH; ++m) s += bp[m] * Y[m];
    sY = s;
    float w[kNumSH];
#pragma unroll
    for (int m = 0; m < kNumSH; ++m) w[m] = b[m] * c[m];
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    const float xy = x * y, yz = y * z, xz = x * z;
    float X = 0.0f, Yv = 0.0f, Z = 0.0f;
    // l = 1
    Yv += w[0];
    Z += w[1];
    X += w[2];
    // l = 2
    X += w[3] * y;  Yv += w[3] * x;
    Yv += w[4] * z; Z += w[4] * y;
    Z += w[5] * 6.0f * z;
    X += w[6] * z;  Z += w[6] * x;
    X += w[7] * 2.0f * x; Yv -= w[7] * 2.0f * y;
    // l = 3
    X += w[8] * 6.0f * xy;  Yv += w[8] * 3.0f * (x2 - y2);
    X += w[9] * yz; Yv += w[9] * xz; Z += w[9] * xy;
    Yv += w[10] * (5.0f * z2 - 1.0f); Z += w[10] * 10.0f * yz;
    Z += w[11] * (15.0f * z2 - 3.0f);
    X += w[12] * (5.0f * z2 - 1.0f); Z += w[12] * 10.0f * xz;
    X += w[13] * 2.0f * xz; Yv -= w[13] * 2.0f * yz; Z += w[13] * (x2 - y2);
    X += w[14] * 3.0f * (x2 - y2); Yv -= w[14] * 6.0f * xy;
    // l = 4
    X += w[15] * (3.0f * x2 * y - y2 * y); Yv += w[15] * (x2 * x - 3.0f * x * y2);
    X += w[16] * 6.0f * xy * z; Yv += w[16] * 3.0f * z * (x2 - y2); Z += w[16] * (3.0f * x2 * y - y2 * y);
    X += w[17] * y * (7.0f * z2 - 1.0f); Yv += w[17] * x * (7.0f * z2 - 1.0f); Z += w[17] * 14.0f * xy * z;
    Yv += w[18] * z * (7.0f * z2 - 3.0f); Z += w[18] * y * (21.0f * z2 - 3.0f);
    Z += w[19] * z * (140.0f * z2 - 60.0f);
    X += w[20] * z * (7.0f * z2 - 3.0f); Z += w[20] * x * (21.0f * z2 - 3.0f);
    X += w[21] * 2.0f * x * (7.0f * z2 - 1.0f); Yv -= w[21] * 2.0f * y * (7.0f * z2 - 1.0f);
    Z += w[21] * 14.0f * z * (x2 - y2);
    X += w[22] * 3.0f * z * (x2 - y2); Yv -= w[22] * 6.0f * xy * z; Z += w[22] * x * (x2 - 3.0f * y2);
    X += w[23] * (4.0f * x2 * x - 12.0f * x * y2); Yv += w[23] * (4.0f * y2 * y - 12.0f * x2 * y);
    gx = X;
    gy = Yv;
    gz = Z;
}

// l of spherical-harmonic slot m (0..23).
__host__ __device__ constexpr int sh_l(int m) { return m < 3 ? 1 : (m < 8 ? 2 : (m < 15 ? 3 : 4)); }

template <int NR1, int NA1, bool FOUR>
struct Dims {
    static constexpr int D = NR1 + kLmax * NA1 + (FOUR ? NA1 : 0);
};

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Block-wide sum (256 threads = 4 waves) in a fixed order; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = (lds[0] + lds[1]) + (lds[2] + lds[3]);
    __syncthreads();
    return r;
}

// Four-body helper: M_n = sum_j g_n (u u^T - I/3) rebuilt from the l = 2 sums
// (slots 3..7 hold m = -2..2): returns mxy, myz, mzz, mxz, d = mxx - myy.
__device__ __forceinline__ void m_from_l2(const float *A2, const float *shc, float *M)
{
    M[0] = A2[0] / shc[3];
    M[1] = A2[1] / shc[4];
    M[2] = A2[2] / (3.0f * shc[5]);
    M[3] = A2[3] / shc[6];
    M[4] = A2[4] / shc[7];
}

constexpr int kBatch = 4;   // neighbours whose index and position are loaded together

// Hide a uniform pointer from loop-invariant code motion, so that the model
// coefficients it addresses are re-read through the scalar cache inside a
// neighbour loop instead of being hoisted into (scarce) vector registers.
__device__ __forceinline__ const float *launder(const float *p)
{
    asm volatile("" : "+s"(p));
    return p;
}

// ----------------------------------------------------------- pass 1 ---

template <int NR1, int NA1, int KR1, int KA1, bool FOUR>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
void k_descriptor(NepArgs a, const float *__restrict__ prm)
{
    constexpr int D = Dims<NR1, NA1, FOUR>::D;
    int b, tile;
    bead_tile(b, tile);
    const int i = tile * blockDim.x + threadIdx.x;
    const int N = a.N, S = a.S;
    const bool valid = i < N;
    const int ii = valid ? i : N - 1;
    const int ti = a.types[ii];
    const bool tok = ti >= 0 && ti < S;
    const float4 *pb = a.p4 + (size_t)b * N;
    const float4 pi = pb[ii];
    const float *shc = prm + a.osh;
    float U = 0.0f;

    uint64_t todo = __ballot(valid && tok);
    while (todo) {
        const int lead = __builtin_ctzll(todo);
        const int tc = __builtin_amdgcn_readlane(ti, lead);
        const bool mine = valid && tok && ti == tc;
        todo &= ~__ballot(mine);
        if (!mine) continue;

        float q[D];
#pragma unroll
        for (int v = 0; v < D; ++v) q[v] = 0.0f;

        // radial: per neighbour species, sum the basis, then contract with c
        const int32_t *lR = a.listR + (size_t)b * a.capR * N + i;
        const int32_t *lA = a.listA + (size_t)b * a.capA * N + i;
        for (int t = 0; t < S; ++t) {
            int s0, s1;
            block_range(a.endR, b, t, N, i, s0, s1);
            float sk[KR1];
#pragma unroll
            for (int k = 0; k < KR1; ++k) sk[k] = 0.0f;
            for (int sb = s0; sb < s1; sb += kBatch) {
                float4 pj[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int j = (sb + u < s1) ? lR[(size_t)(sb + u) * N] : i;
                    pj[u] = pb[j];
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    if (sb + u < s1) {
                        float dx, dy, dz;
                        pair_vec(pj[u], pi, a, dx, dy, dz);
                        const float r = __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz);
                        float f[KR1];
                        cheb_f<KR1>(r, a.rcRinv, f);
#pragma unroll
                        for (int q2 = 0; q2 < KR1; ++q2) sk[q2] += f[q2];
                    }
                }
            }
            const float *c = prm + a.oR + (tc * S + t) * NR1 * KR1;
#pragma unroll
            for (int n = 0; n < NR1; ++n) {
                float acc = q[n];
#pragma unroll
                for (int q2 = 0; q2 < KR1; ++q2) acc += c[n * KR1 + q2] * sk[q2];
                q[n] = acc;
            }
        }

        // angular: A_nlm = sum_j g_n(r_ij) Y_lm(u_ij)
        float A[NA1][kNumSH];
#pragma unroll
        for (int n = 0; n < NA1; ++n)
#pragma unroll
            for (int m = 0; m < kNumSH; ++m) A[n][m] = 0.0f;
        for (int t = 0; t < S; ++t) {
            int s0, s1;
            block_range(a.endA, b, t, N, i, s0, s1);
            const float *c = prm + a.oA + (tc * S + t) * NA1 * KA1;
            float4 pn = pb[s0 < s1 ? lA[(size_t)s0 * N] : i];
            for (int sn = s0; sn < s1; ++sn) {
                const float4 pc = pn;
                if (sn + 1 < s1) pn = pb[lA[(size_t)(sn + 1) * N]];
                float dx, dy, dz;
                pair_vec(pc, pi, a, dx, dy, dz);
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float rinv = __builtin_amdgcn_rsqf(r2);
                const float r = r2 * rinv;
                float f[KA1];
                cheb_f<KA1>(r, a.rcAinv, f);
                float Y[kNumSH];
                sh_eval(dx * rinv, dy * rinv, dz * rinv, shc, Y);
#pragma unroll
                for (int n = 0; n < NA1; ++n) {
                    float g = 0.0f;
#pragma unroll
                    for (int q2 = 0; q2 < KA1; ++q2) g += c[n * KA1 + q2] * f[q2];
#pragma unroll
                    for (int m = 0; m < kNumSH; ++m) A[n][m] += g * Y[m];
                }
            }
        }
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
#pragma unroll
            for (int l = 1; l <= kLmax; ++l) {
                float s2 = 0.0f;
#pragma unroll
                for (int m = 0; m < kNumSH; ++m)
                    if (sh_l(m) == l) s2 += A[n][m] * A[n][m];
                q[NR1 + (l - 1) * NA1 + n] = s2;
            }
            if (FOUR) {
                float M[5];
                m_from_l2(&A[n][3], shc, M);
                const float mxy = M[0], myz = M[1], mzz = M[2], mxz = M[3], dd = M[4];
                const float mxx = 0.5f * (dd - mzz), myy = 0.5f * (-dd - mzz);
                const float tr3 = mxx * mxx * mxx + myy * myy * myy + mzz * mzz * mzz +
                                  3.0f * mxx * (mxy * mxy + mxz * mxz) + 3.0f * myy * (mxy * mxy + myz * myz) +
                                  3.0f * mzz * (mxz * mxz + myz * myz) + 6.0f * mxy * myz * mxz;
                q[NR1 + kLmax * NA1 + n] = a.kappa4 * tr3;
            }
        }
        // park A in this atom's adjoint row (overwritten with B below)
        float *Bo = a.B + ((size_t)b * N + i) * (NA1 * kNumSH);
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            float4 *o4 = reinterpret_cast<float4 *>(Bo + n * kNumSH);
#pragma unroll
            for (int q4 = 0; q4 < kNumSH / 4; ++q4)
                o4[q4] = make_float4(A[n][4 * q4], A[n][4 * q4 + 1], A[n][4 * q4 + 2], A[n][4 * q4 + 3]);
        }

        // network: U = sum_mu w1 tanh(sum_nu W0 s_nu q_nu - b0) - b1;  G_nu = dU/dq_nu
        const float *qs = prm + a.oq;
        float qh[D], G[D];
#pragma unroll
        for (int v = 0; v < D; ++v) {
            qh[v] = qs[v] * q[v];
            G[v] = 0.0f;
        }
        const float *W0 = prm + a.oW0 + tc * a.H * D;
        const float *b0 = prm + a.ob0 + tc * a.H;
        const float *w1 = prm + a.ow1 + tc * a.H;
        float u = -prm[a.ob1];
        for (int mu = 0; mu < a.H; ++mu) {
            float z = -b0[mu];
#pragma unroll
            for (int v = 0; v < D; ++v) z += W0[mu * D + v] * qh[v];
            const float h = tanhf(z);
            u += w1[mu] * h;
            const float gz = w1[mu] * (1.0f - h * h);
#pragma unroll
            for (int v = 0; v < D; ++v) G[v] += gz * W0[mu * D + v];
        }
#pragma unroll
        for (int v = 0; v < D; ++v) G[v] *= qs[v];
        U = u;

        // adjoints: B_nlm = dU/dA_nlm (A read back from the parked row)
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            float An[kNumSH];
            float4 *o4 = reinterpret_cast<float4 *>(Bo + n * kNumSH);
#pragma unroll
            for (int q4 = 0; q4 < kNumSH / 4; ++q4) {
                const float4 v4 = o4[q4];
                An[4 * q4] = v4.x; An[4 * q4 + 1] = v4.y; An[4 * q4 + 2] = v4.z; An[4 * q4 + 3] = v4.w;
            }
            float Bn[kNumSH];
#pragma unroll
            for (int m = 0; m < kNumSH; ++m) Bn[m] = 2.0f * G[NR1 + (sh_l(m) - 1) * NA1 + n] * An[m];
            if (FOUR) {
                float M[5];
                m_from_l2(&An[3], shc, M);
                const float mxy = M[0], myz = M[1], mzz = M[2], mxz = M[3], dd = M[4];
                const float mxx = 0.5f * (dd - mzz), myy = 0.5f * (-dd - mzz);
                // entries of M^2
                const float sxx = mxx * mxx + mxy * mxy + mxz * mxz;
                const float syy = mxy * mxy + myy * myy + myz * myz;
                const float szz = mxz * mxz + myz * myz + mzz * mzz;
                const float sxy = mxx * mxy + mxy * myy + mxz * myz;
                const float syz = mxy * mxz + myy * myz + myz * mzz;
                const float sxz = mxx * mxz + mxy * myz + mxz * mzz;
                const float g4 = G[NR1 + kLmax * NA1 + n] * a.kappa4;
                Bn[3] += g4 * 6.0f * sxy / shc[3];
                Bn[4] += g4 * 6.0f * syz / shc[4];
                Bn[5] += g4 * 3.0f * (szz - 0.5f * sxx - 0.5f * syy) / (3.0f * shc[5]);
                Bn[6] += g4 * 6.0f * sxz / shc[6];
                Bn[7] += g4 * 1.5f * (sxx - syy) / shc[7];
            }
#pragma unroll
            for (int q4 = 0; q4 < kNumSH / 4; ++q4)
                o4[q4] = make_float4(Bn[4 * q4], Bn[4 * q4 + 1], Bn[4 * q4 + 2], Bn[4 * q4 + 3]);
        }
        // radial adjoints a_k(t) = sum_n G_n c^{tc t}_nk
        float *ao = a.arad + ((size_t)b * N + i) * S * a.KRP;
        for (int t = 0; t < S; ++t) {
            const float *c = prm + a.oR + (tc * S + t) * NR1 * KR1;
#pragma unroll
            for (int k = 0; k < KR1; ++k) {
                float acc = 0.0f;
#pragma unroll
                for (int n = 0; n < NR1; ++n) acc += G[n] * c[n * KR1 + k];
                ao[t * a.KRP + k] = acc;
            }
        }
    }

    if (valid && a.Eatom) a.Eatom[(size_t)b * N + i] = U;
    if (valid && !tok) atomicOr(a.flags, (uint32_t)NEP_FLAG_BAD_TYPE);
    __shared__ double lds[4];
    const double e = block_sum(valid ? (double)U : 0.0, lds);
    if (threadIdx.x == 0) a.partE[(size_t)b * gridDim.x + tile] = e;
}

// ------------------------------------------------ pass 2: angular, own ---

// One lane per (bead, atom i): the angular pair terms d_ij = dU_i/dr_ij of
// the atom's own site energy, contracted with its own adjoints only:
//   d_ij = sum_n sum_lm B^i_nlm d/dr_ij [ g^{ij}_n(r) Y_lm(u) ],
// stored at (bead, i, candidate slot of j) for the reverse gather of the
// radial pass, and summed into the angular force part F_i += d_ij and the
// virial -r_ij (x) d_ij (the total needs no reverse terms).  BREG keeps B^i
// in registers (small n_max); otherwise it is re-read from its L1-resident
// row.  Control flow stays wave-uniform: lanes outside the current centre
// species, or past their last neighbour, compute on a dummy pair and
// contribute nothing.
template <int NA1, int KA1, bool BREG>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
void k_force_ang(NepArgs a, const float *__restrict__ prm)
{
    int b, tile;
    bead_tile(b, tile);
    const int i = tile * blockDim.x + threadIdx.x;
    const int N = a.N, S = a.S;
    const bool valid = i < N;
    const int ii = valid ? i : N - 1;
    const int ti = a.types[ii];
    const bool tok = ti >= 0 && ti < S;
    const float4 *pb = a.p4 + (size_t)b * N;
    const float4 pi = pb[ii];
    const float *shc = prm + a.osh;
    const int32_t *lA = a.listA + (size_t)b * a.capA * N + ii;
    const int32_t *sA = a.slotA + (size_t)b * a.capA * N + ii;
    const uint64_t *mkb = a.maskA + (size_t)b * a.WC * N;
    float4 *pbuf = a.pairbuf + (size_t)b * a.capA * N;
    float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f;
    float Wv[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) Wv[e] = 0.0f;

    uint64_t todo = __ballot(valid && tok);
    while (todo) {
        const int lead = __builtin_ctzll(todo);
        const int tc = __builtin_amdgcn_readlane(ti, lead);
        const bool mine = valid && tok && ti == tc;
        todo &= ~__ballot(mine);

        const float4 *bi4 = reinterpret_cast<const float4 *>(a.B + ((size_t)b * N + ii) * (NA1 * kNumSH));
        float Bi[BREG ? NA1 : 1][kNumSH];
        if (BREG) {
#pragma unroll
            for (int n = 0; n < (BREG ? NA1 : 1); ++n)
#pragma unroll
                for (int q4 = 0; q4 < kNumSH / 4; ++q4) {
                    const float4 v4 = bi4[n * (kNumSH / 4) + q4];
                    Bi[n][4 * q4] = v4.x; Bi[n][4 * q4 + 1] = v4.y;
                    Bi[n][4 * q4 + 2] = v4.z; Bi[n][4 * q4 + 3] = v4.w;
                }
        }
        for (int t = 0; t < S; ++t) {
            int s0 = 0, s1 = 0;
            if (mine) block_range(a.endA, b, t, N, ii, s0, s1);
            const int cnt = s1 - s0;
            int cmax = cnt;
            for (int o = 32; o > 0; o >>= 1) cmax = max(cmax, __shfl_xor(cmax, o));
            cmax = __builtin_amdgcn_readfirstlane(cmax);
            const float *cij = prm + a.oA + (tc * S + t) * NA1 * KA1;
            int jn = cnt > 0 ? lA[(size_t)s0 * N] : ii;
            int rn = cnt > 0 ? (int)((uint32_t)sA[(size_t)s0 * N] >> 16) : 0xffff;
            for (int sc = 0; sc < cmax; ++sc) {
                const float *cij_l = launder(cij), *shc_l = launder(shc);
                const bool act = sc < cnt;
                const int j = jn, rc = rn;
                if (sc + 1 < cnt) {
                    jn = lA[(size_t)(s0 + sc + 1) * N];
                    rn = (int)((uint32_t)sA[(size_t)(s0 + sc + 1) * N] >> 16);
                }
                // list position of i in j's angular list: angular hits of j before its slot rc
                int dst = -1;
                if (act && rc != 0xffff) {
                    const uint64_t m = mkb[(size_t)(rc >> 5) * N + j];
                    dst = (int)(m >> 32) + __popc((uint32_t)m & ((1u << (rc & 31)) - 1u));
                    if (dst >= a.capA) dst = -1;
                }
                float dx, dy, dz;
                pair_vec(pb[j], pi, a, dx, dy, dz);
                if (!act) {
                    dx = 1.0f;
                    dy = 0.0f;
                    dz = 0.0f;
                }
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float rinv = __builtin_amdgcn_rsqf(r2);
                const float r = r2 * rinv;
                const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
                float gij[NA1], gpij[NA1];
                {
                    float f[KA1], fp[KA1];
                    cheb_fd<KA1>(r, a.rcAinv, f, fp);
#pragma unroll
                    for (int n = 0; n < NA1; ++n) {
                        float g0 = 0.0f, g1 = 0.0f;
#pragma unroll
                        for (int q2 = 0; q2 < KA1; ++q2) {
                            g0 = fmaf(cij_l[n * KA1 + q2], f[q2], g0);
                            g1 = fmaf(cij_l[n * KA1 + q2], fp[q2], g1);
                        }
                        gij[n] = g0;
                        gpij[n] = g1;
                    }
                }
                float beta[kNumSH], betap[kNumSH];
#pragma unroll
                for (int m = 0; m < kNumSH; ++m) {
                    beta[m] = 0.0f;
                    betap[m] = 0.0f;
                }
#pragma unroll
                for (int n = 0; n < NA1; ++n) {
#pragma unroll
                    for (int q4 = 0; q4 < kNumSH / 4; ++q4) {
                        float bx[4];
                        if (!BREG) {
                            const float4 x4 = bi4[n * (kNumSH / 4) + q4];
                            bx[0] = x4.x; bx[1] = x4.y; bx[2] = x4.z; bx[3] = x4.w;
                        }
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int m = 4 * q4 + e;
                            const float bi = BREG ? Bi[BREG ? n : 0][m] : bx[e];
                            beta[m] = fmaf(bi, gij[n], beta[m]);
                            betap[m] = fmaf(bi, gpij[n], betap[m]);
                        }
                    }
                }
                float sY, gx, gy, gz;
                sh_contract(ux, uy, uz, shc_l, beta, betap, sY, gx, gy, gz);
                const float ug = ux * gx + uy * gy + uz * gz;
                const float px = sY * ux + (gx - ux * ug) * rinv;
                const float py = sY * uy + (gy - uy * ug) * rinv;
                const float pz = sY * uz + (gz - uz * ug) * rinv;
                if (act) {
                    if (dst >= 0) pbuf[(size_t)dst * N + j] = make_float4(px, py, pz, 0.0f);
                    Fx += px; Fy += py; Fz += pz;
                    Wv[0] = fmaf(-dx, px, Wv[0]); Wv[1] = fmaf(-dx, py, Wv[1]); Wv[2] = fmaf(-dx, pz, Wv[2]);
                    Wv[3] = fmaf(-dy, px, Wv[3]); Wv[4] = fmaf(-dy, py, Wv[4]); Wv[5] = fmaf(-dy, pz, Wv[5]);
                    Wv[6] = fmaf(-dz, px, Wv[6]); Wv[7] = fmaf(-dz, py, Wv[7]); Wv[8] = fmaf(-dz, pz, Wv[8]);
                }
            }
        }
    }

    if (valid) {
        float *Fo = a.Fang + ((size_t)b * N + i) * 3;
        Fo[0] = Fx;
        Fo[1] = Fy;
        Fo[2] = Fz;
        if (a.Watom) {
            // own half of the per-atom split; the reverse half is added by the radial pass
            float *wo = a.Watom + ((size_t)b * N + i) * 9;
#pragma unroll
            for (int e = 0; e < 9; ++e) wo[e] = 0.5f * Wv[e];
        }
    }
    __shared__ double lds[4];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const double w = block_sum(valid ? (double)Wv[e] : 0.0, lds);
        if (threadIdx.x == 0) a.partWa[((size_t)b * gridDim.x + tile) * 9 + e] = w;
    }
}

// ----------------------------------------- pass 3: radial + combination ---

// One lane per (bead, atom i): radial pair terms (a^i_k(tj) + a^j_k(ti)) f'_k(r) u
// (both site energies at once, the adjoints a_k are gathered), then the
// reverse angular terms -dU_j/dr_ji gathered from the pair buffer through the
// reverse slot of each angular neighbour, then the angular own part of pass 2.
// Force and per-atom virial sums are kept in FP64.
template <int KR1>
__global__ __launch_bounds__(kBlock) void k_force_rad(NepArgs a)
{
    int b, tile;
    bead_tile(b, tile);
    const int i = tile * blockDim.x + threadIdx.x;
    const int N = a.N, S = a.S;
    const bool valid = i < N;
    const int ii = valid ? i : N - 1;
    const int ti = a.types[ii];
    const bool tok = ti >= 0 && ti < S;
    const float4 *pb = a.p4 + (size_t)b * N;
    const float4 pi = pb[ii];
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    double Wv[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) Wv[e] = 0.0;
    float Wa[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) Wa[e] = 0.0f;
    if (valid && tok) {
        const float *ai_base = a.arad + ((size_t)b * N + i) * S * a.KRP;
        const int32_t *lR = a.listR + (size_t)b * a.capR * N + i;
        for (int t = 0; t < S; ++t) {
            int s0, s1;
            block_range(a.endR, b, t, N, i, s0, s1);
            float ai[KR1];
#pragma unroll
            for (int q2 = 0; q2 < KR1; ++q2) ai[q2] = ai_base[t * a.KRP + q2];
            for (int sb = s0; sb < s1; sb += kBatch) {
                float4 pj[kBatch];
                float aj[kBatch][KR1];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int j = (sb + u < s1) ? lR[(size_t)(sb + u) * N] : i;
                    pj[u] = pb[j];
                    const float *ajp = a.arad + ((size_t)b * N + j) * S * a.KRP + ti * a.KRP;
#pragma unroll
                    for (int q2 = 0; q2 < KR1; ++q2) aj[u][q2] = ajp[q2];
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    if (sb + u < s1) {
                        float dx, dy, dz;
                        pair_vec(pj[u], pi, a, dx, dy, dz);
                        const float r2 = dx * dx + dy * dy + dz * dz;
                        const float rinv = __builtin_amdgcn_rsqf(r2);
                        const float r = r2 * rinv;
                        float f[KR1], fp[KR1];
                        cheb_fd<KR1>(r, a.rcRinv, f, fp);
                        float sc = 0.0f;
#pragma unroll
                        for (int q2 = 0; q2 < KR1; ++q2) sc += (ai[q2] + aj[u][q2]) * fp[q2];
                        const float w = sc * rinv;
                        const float qx = w * dx, qy = w * dy, qz = w * dz;
                        Fx += qx; Fy += qy; Fz += qz;
                        Wv[0] -= 0.5 * dx * qx; Wv[1] -= 0.5 * dx * qy; Wv[2] -= 0.5 * dx * qz;
                        Wv[3] -= 0.5 * dy * qx; Wv[4] -= 0.5 * dy * qy; Wv[5] -= 0.5 * dy * qz;
                        Wv[6] -= 0.5 * dz * qx; Wv[7] -= 0.5 * dz * qy; Wv[8] -= 0.5 * dz * qz;
                    }
                }
            }
        }

        // reverse angular terms: F_i -= dU_j/dr_ji for every angular neighbour j,
        // deposited at this atom's own list positions by the angular pass
        const int32_t *lA = a.listA + (size_t)b * a.capA * N + i;
        const float4 *pbuf = a.pairbuf + (size_t)b * a.capA * N + i;
        const int nA = a.endA[((size_t)b * kMaxSpecies + (S - 1)) * N + i];
        float gx = 0.0f, gy = 0.0f, gz = 0.0f;
        for (int sb = 0; sb < nA; sb += kBatch) {
            float4 d[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u)
                d[u] = sb + u < nA ? pbuf[(size_t)(sb + u) * N] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                gx -= d[u].x; gy -= d[u].y; gz -= d[u].z;
            }
            if (a.Watom) {
                // reverse half of the per-atom split: +1/2 r_ij (x) dU_j/dr_ji
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    if (sb + u < nA) {
                        float dx, dy, dz;
                        pair_vec(pb[lA[(size_t)(sb + u) * N]], pi, a, dx, dy, dz);
                        const float hx = 0.5f * dx, hy = 0.5f * dy, hz = 0.5f * dz;
                        Wa[0] = fmaf(hx, d[u].x, Wa[0]); Wa[1] = fmaf(hx, d[u].y, Wa[1]); Wa[2] = fmaf(hx, d[u].z, Wa[2]);
                        Wa[3] = fmaf(hy, d[u].x, Wa[3]); Wa[4] = fmaf(hy, d[u].y, Wa[4]); Wa[5] = fmaf(hy, d[u].z, Wa[5]);
                        Wa[6] = fmaf(hz, d[u].x, Wa[6]); Wa[7] = fmaf(hz, d[u].y, Wa[7]); Wa[8] = fmaf(hz, d[u].z, Wa[8]);
                    }
                }
            }
        }
        Fx += (double)gx;
        Fy += (double)gy;
        Fz += (double)gz;
    }
    if (valid) {
        const float *fa = a.Fang + ((size_t)b * N + i) * 3;
        const double gx = Fx + (double)fa[0], gy = Fy + (double)fa[1], gz = Fz + (double)fa[2];
        float *Fo = a.F + ((size_t)b * N + i) * 3;
        Fo[0] = (float)gx;
        Fo[1] = (float)gy;
        Fo[2] = (float)gz;
        if (a.Watom) {
            float *wo = a.Watom + ((size_t)b * N + i) * 9;
#pragma unroll
            for (int e = 0; e < 9; ++e) wo[e] = (float)(Wv[e] + (double)Wa[e] + (double)wo[e]);
        }
        if (!(isfinite(gx) && isfinite(gy) && isfinite(gz))) atomicOr(a.flags, (uint32_t)NEP_FLAG_NONFINITE);
    }
    __shared__ double lds[4];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const double w = block_sum(valid ? Wv[e] : 0.0, lds);
        if (threadIdx.x == 0) a.partWr[((size_t)b * gridDim.x + tile) * 9 + e] = w;
    }
}

// Per-bead totals from the per-block partial sums, in block order.
__global__ void k_reduce(const double *__restrict__ partE, const double *__restrict__ partWa,
                         const double *__restrict__ partWr, int nblk, double *__restrict__ E, double *__restrict__ W)
{
    const int b = blockIdx.x, t = threadIdx.x;
    if (t == 0) {
        double s = 0.0;
        for (int k = 0; k < nblk; ++k) s += partE[(size_t)b * nblk + k];
        E[b] = s;
    } else if (t <= 9) {
        double s = 0.0;
        for (int k = 0; k < nblk; ++k) {
            const size_t o = ((size_t)b * nblk + k) * 9 + (t - 1);
            s += partWa[o] + partWr[o];
        }
        W[(size_t)b * 9 + (t - 1)] = s;
    }
}

template <int NR1, int NA1, bool FOUR>
static void launch(const NepArgs &a, const float *prm, int P, hipStream_t s)
{
    const dim3 g(div_up(a.N, kBlock), P);
    {
        ProfScope ps_(K_DESCRIPTOR, s);
        hipLaunchKernelGGL((k_descriptor<NR1, NA1, 9, 9, FOUR>), g, dim3(kBlock), 0, s, a, prm);
    }
    {
        ProfScope ps_(K_FORCE_ANG, s);
        hipLaunchKernelGGL((k_force_ang<NA1, 9, (NA1 <= 5)>), g, dim3(kBlock), 0, s, a, prm);
    }
    {
        ProfScope ps_(K_FORCE, s);
        hipLaunchKernelGGL((k_force_rad<9>), g, dim3(kBlock), 0, s, a);
    }
}

}  // namespace nep

using namespace nep;

extern "C" int32_t nep_compute(const nep_model *m, nep_nlist *nl, nep_ws *ws, const double *pos,
                               const double box[9], const int32_t *types, int32_t P, int32_t N, double *E, float *F,
                               double *W, float *E_atom, float *W_atom, hipStream_t s)
{
    if (!m || !nl || !ws || !box) return fail(NEP_ERR_INVALID_ARG, "nep_compute: null argument");
    if (nl->P != P || nl->N != N || ws->P != P || ws->N != N || nl->S != m->hp.n_species || ws->S != m->hp.n_species ||
        ws->NA1 != m->hp.n_max_angular + 1)
        return fail(NEP_ERR_INVALID_ARG, "nep_compute: P=%d N=%d do not match the list/workspace handles", P, N);
    if (P == 0) return NEP_OK;
    if (!E || !W) return fail(NEP_ERR_INVALID_ARG, "nep_compute: null E or W");
    if (N == 0) {
        fill_u32(reinterpret_cast<uint32_t *>(E), 0u, (size_t)P * 2, s);
        fill_u32(reinterpret_cast<uint32_t *>(W), 0u, (size_t)P * 18, s);
        NEP_HIP(hipGetLastError());
        return NEP_OK;
    }
    if (!pos || !types || !F) return fail(NEP_ERR_INVALID_ARG, "nep_compute: null array");
    NepArgs a{};
    double L[3];
    if (!box_lengths(box, L)) return fail(NEP_ERR_UNSUPPORTED, "nep_compute: only orthorhombic cells");
    for (int d = 0; d < 3; ++d)
        if (!(L[d] > 0.0) || !std::isfinite(L[d]))
            return fail(NEP_ERR_INVALID_ARG, "nep_compute: bad box edge %g", L[d]);
    const FineGrid fg = fine_grid(L, std::max(m->hp.rc_radial, m->hp.rc_angular));
    if (!fg.exact)
        return fail(NEP_ERR_BOX_TOO_SMALL, "nep_compute: box edges %g %g %g leave no margin over twice the cutoff",
                    L[0], L[1], L[2]);
    for (int d = 0; d < 3; ++d) {
        a.M[d] = fg.M[d];
        a.h[d] = fg.h[d];
    }
    const nep_hparams &h = m->hp;
    a.p4 = reinterpret_cast<const float4 *>(ws->pos4); a.types = types; a.N = N; a.S = h.n_species; a.H = h.hidden;
    a.rcRinv = (float)(1.0 / h.rc_radial); a.rcAinv = (float)(1.0 / h.rc_angular);
    a.kappa4 = (float)(-4.5 * std::sqrt(2.0 / 35.0) * std::pow(5.0 / (4.0 * M_PI), 1.5));
    a.listR = nl->listR; a.endR = nl->endR; a.listA = nl->listA; a.endA = nl->endA; a.slotA = nl->slotA;
    a.maskA = nl->maskA;
    a.capR = nl->capR; a.capA = nl->capA; a.capC = nl->capC; a.WC = nl->WC;
    a.pairbuf = reinterpret_cast<float4 *>(nl->pairbuf);
    a.B = ws->B; a.arad = ws->arad; a.Fang = ws->Fang; a.KRP = ws->KRP;
    a.partE = ws->partE; a.partWa = ws->partW; a.partWr = ws->partW + (size_t)P * ws->nblk * 9;
    a.flags = ws->flags;
    a.F = F; a.Eatom = E_atom; a.Watom = W_atom;
    a.oR = m->off.cR; a.oA = m->off.cA; a.oq = m->off.qs; a.oW0 = m->off.W0; a.ob0 = m->off.b0;
    a.ow1 = m->off.w1; a.ob1 = m->off.b1; a.osh = m->off.sh;
    const int key = h.n_max_radial * 100 + h.n_max_angular * 10 + h.four_body;
    if (key != 440 && key != 441 && key != 640 && key != 860 && key != 881)
        return fail(NEP_ERR_UNSUPPORTED, "nep_compute: unsupported model shape");
    pack_positions(pos, (size_t)P * N, fg, reinterpret_cast<float4 *>(ws->pos4), s);
    switch (key) {
    case 440: launch<5, 5, false>(a, m->dev, P, s); break;
    case 441: launch<5, 5, true>(a, m->dev, P, s); break;
    case 640: launch<7, 5, false>(a, m->dev, P, s); break;
    case 860: launch<9, 7, false>(a, m->dev, P, s); break;
    case 881: launch<9, 9, true>(a, m->dev, P, s); break;
    default: return fail(NEP_ERR_UNSUPPORTED, "nep_compute: unsupported model shape");
    }
    {
        ProfScope ps_(K_REDUCE, s);
        hipLaunchKernelGGL(k_reduce, dim3(P), dim3(64), 0, s, ws->partE, a.partWa, a.partWr, ws->nblk, E, W);
    }
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}
