// NEP energy, forces and virial on gfx950 (site-energy model of Sec. II.C,
// bead forces and virial of Sec. II.A of arXiv:2409.04430).
//
// Four kernels per call, one lane per (bead, atom):
//   k_descriptor  radial sums, angular sums A_nlm = sum_j g_n(r_ij) Y_lm(u_ij)
//                 over real orthonormal spherical harmonics, q_nl = sum_m A_nlm^2
//                 (equal to the Legendre double sum by the addition theorem),
//                 the optional (2,2,2) four-body invariant, the tanh network,
//                 and the adjoints: B_nlm = dU_i/dA_nlm and the radial
//                 a_k(t) = sum_n dU_i/dq_n c^{ti t}_nk;
//   k_force_ang   angular pair terms in gather form, one contraction with
//                 B^i_nlm g^{ij}_n + (-1)^l B^j_nlm g^{ji}_n per neighbour, so
//                 F_i = sum_j (dU_i/dr_ij - dU_j/dr_ji) needs no atomics;
//   k_force_rad   radial pair terms (a^i_k(tj) + a^j_k(ti)) f'_k(r) u, added to
//                 the angular part; per-atom virial -1/2 sum_j r_ij (x) phi_ij;
//   k_reduce      per-bead energy and virial from per-block partial sums in
//                 a fixed order (bitwise reproducible).
// The descriptor and angular-force passes run species-uniform groups of
// lanes, which makes every model-coefficient address wave-uniform (scalar
// loads, SGPR operands).  Neighbour loops prefetch the next index and
// position so that gathers overlap arithmetic.
#include "internal.hpp"

namespace nep {

constexpr float kPi = 3.14159265358979f;

struct NepArgs {
    const double *pos;
    const int32_t *types;
    int N, S, H;
    double L[3], invL[3];
    float rcRinv, rcAinv;
    float kappa4;
    // lists
    const int32_t *cntR, *idxR, *cntA, *idxA;
    int capR, capA;
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

// Pair vector r_j - r_i under the minimum image, formed in FP64, returned in FP32.
__device__ __forceinline__ void pair_vec(double xj, double yj, double zj, double xi, double yi, double zi,
                                         const NepArgs &a, float &dx, float &dy, float &dz)
{
    double x = xj - xi, y = yj - yi, z = zj - zi;
    x -= a.L[0] * rint(x * a.invL[0]);
    y -= a.L[1] * rint(y * a.invL[1]);
    z -= a.L[2] * rint(z * a.invL[2]);
    dx = (float)x;
    dy = (float)y;
    dz = (float)z;
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
    const double *pb = a.pos + (size_t)b * N * 3;
    const double xi = pb[3 * ii], yi = pb[3 * ii + 1], zi = pb[3 * ii + 2];
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
        for (int t = 0; t < S; ++t) {
            const size_t blk = ((size_t)b * S + t);
            const int cnt = min(a.cntR[blk * N + i], a.capR);
            const int32_t *ix = a.idxR + blk * a.capR * N + i;
            float sk[KR1];
#pragma unroll
            for (int k = 0; k < KR1; ++k) sk[k] = 0.0f;
            for (int s0 = 0; s0 < cnt; s0 += kBatch) {
                int jj[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) jj[u] = (s0 + u < cnt) ? ix[(size_t)(s0 + u) * N] : i;
                double px[kBatch], py[kBatch], pz[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    px[u] = pb[3 * jj[u]];
                    py[u] = pb[3 * jj[u] + 1];
                    pz[u] = pb[3 * jj[u] + 2];
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    if (s0 + u < cnt) {
                        float dx, dy, dz;
                        pair_vec(px[u], py[u], pz[u], xi, yi, zi, a, dx, dy, dz);
                        const float r = __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz);
                        float f[KR1];
                        cheb_f<KR1>(r, a.rcRinv, f);
#pragma unroll
                        for (int k = 0; k < KR1; ++k) sk[k] += f[k];
                    }
                }
            }
            const float *c = prm + a.oR + (tc * S + t) * NR1 * KR1;
#pragma unroll
            for (int n = 0; n < NR1; ++n) {
                float acc = q[n];
#pragma unroll
                for (int k = 0; k < KR1; ++k) acc += c[n * KR1 + k] * sk[k];
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
            const size_t blk = ((size_t)b * S + t);
            const int cnt = min(a.cntA[blk * N + i], a.capA);
            const int32_t *ix = a.idxA + blk * a.capA * N + i;
            const float *c = prm + a.oA + (tc * S + t) * NA1 * KA1;
            int jn = cnt > 0 ? ix[0] : i;
            double nx = pb[3 * jn], ny = pb[3 * jn + 1], nz = pb[3 * jn + 2];
            for (int s = 0; s < cnt; ++s) {
                const double cx = nx, cy = ny, cz = nz;
                if (s + 1 < cnt) {
                    jn = ix[(size_t)(s + 1) * N];
                    nx = pb[3 * jn];
                    ny = pb[3 * jn + 1];
                    nz = pb[3 * jn + 2];
                }
                float dx, dy, dz;
                pair_vec(cx, cy, cz, xi, yi, zi, a, dx, dy, dz);
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
                    for (int k = 0; k < KA1; ++k) g += c[n * KA1 + k] * f[k];
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

// ------------------------------------------------------ pass 2: angular ---

// SYM: one species, so c^{ij} = c^{ji} and the pair term uses
// B~ = B^i + (-1)^l B^j once.  BREG: the own adjoints stay in registers
// (small n_max); otherwise they are re-read row by row (L1-resident).
// Per-atom sums of the 26-odd angular pair terms are kept in FP32; the radial
// pass adds them to its FP64 sums.
template <int NA1, int KA1, bool SYM, bool BREG>
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
    const double *pb = a.pos + (size_t)b * N * 3;
    const double xi = pb[3 * ii], yi = pb[3 * ii + 1], zi = pb[3 * ii + 2];
    const float *shc = prm + a.osh;
    float Fx = 0.0f, Fy = 0.0f, Fz = 0.0f;
    float Wv[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) Wv[e] = 0.0f;

    // Control flow stays wave-uniform: lanes outside the current centre
    // species (or past their neighbour count) compute on a dummy pair and
    // contribute nothing.
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
            const size_t blk = ((size_t)b * S + t);
            const int cnt = mine ? min(a.cntA[blk * N + i], a.capA) : 0;
            int cmax = cnt;
            for (int o = 32; o > 0; o >>= 1) cmax = max(cmax, __shfl_xor(cmax, o));
            cmax = __builtin_amdgcn_readfirstlane(cmax);
            const int32_t *ix = a.idxA + blk * a.capA * N + ii;
            const float *cij = prm + a.oA + (tc * S + t) * NA1 * KA1;
            const float *cji = prm + a.oA + (t * S + tc) * NA1 * KA1;
            int jn = cnt > 0 ? ix[0] : ii;
            for (int s = 0; s < cmax; ++s) {
                const float *cij_l = launder(cij), *cji_l = launder(cji), *shc_l = launder(shc);
                const bool act = s < cnt;
                const int j = jn;
                if (s + 1 < cnt) jn = ix[(size_t)(s + 1) * N];
                const float4 *bj4 = reinterpret_cast<const float4 *>(a.B + ((size_t)b * N + j) * (NA1 * kNumSH));
                float dx, dy, dz;
                pair_vec(pb[3 * j], pb[3 * j + 1], pb[3 * j + 2], xi, yi, zi, a, dx, dy, dz);
                if (!act) {
                    dx = 1.0f;
                    dy = 0.0f;
                    dz = 0.0f;
                }
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float rinv = __builtin_amdgcn_rsqf(r2);
                const float r = r2 * rinv;
                const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
                float gij[NA1], gpij[NA1], gji[SYM ? 1 : NA1], gpji[SYM ? 1 : NA1];
                {
                    float f[KA1], fp[KA1];
                    cheb_fd<KA1>(r, a.rcAinv, f, fp);
#pragma unroll
                    for (int n = 0; n < NA1; ++n) {
                        float g0 = 0.0f, g1 = 0.0f;
#pragma unroll
                        for (int k = 0; k < KA1; ++k) {
                            g0 = fmaf(cij_l[n * KA1 + k], f[k], g0);
                            g1 = fmaf(cij_l[n * KA1 + k], fp[k], g1);
                        }
                        gij[n] = g0;
                        gpij[n] = g1;
                        if (!SYM) {
                            float h0 = 0.0f, h1 = 0.0f;
#pragma unroll
                            for (int k = 0; k < KA1; ++k) {
                                h0 = fmaf(cji_l[n * KA1 + k], f[k], h0);
                                h1 = fmaf(cji_l[n * KA1 + k], fp[k], h1);
                            }
                            gji[SYM ? 0 : n] = h0;
                            gpji[SYM ? 0 : n] = h1;
                        }
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
                        const float4 y4 = bj4[n * (kNumSH / 4) + q4];
                        const float bj[4] = {y4.x, y4.y, y4.z, y4.w};
                        float bx[4];
                        if (!BREG) {
                            const float4 x4 = bi4[n * (kNumSH / 4) + q4];
                            bx[0] = x4.x; bx[1] = x4.y; bx[2] = x4.z; bx[3] = x4.w;
                        }
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int m = 4 * q4 + e;
                            const float bi = BREG ? Bi[BREG ? n : 0][m] : bx[e];
                            const float sj = (sh_l(m) & 1) ? -bj[e] : bj[e];
                            if (SYM) {
                                const float bt = bi + sj;
                                beta[m] = fmaf(bt, gij[n], beta[m]);
                                betap[m] = fmaf(bt, gpij[n], betap[m]);
                            } else {
                                beta[m] = fmaf(sj, gji[SYM ? 0 : n], fmaf(bi, gij[n], beta[m]));
                                betap[m] = fmaf(sj, gpji[SYM ? 0 : n], fmaf(bi, gpij[n], betap[m]));
                            }
                        }
                    }
                    // keep the loads of row n + 1 behind this row's arithmetic (register pressure)
                    __builtin_amdgcn_sched_barrier(0);
                }
                float sY, gx, gy, gz;
                sh_contract(ux, uy, uz, shc_l, beta, betap, sY, gx, gy, gz);
                const float ug = ux * gx + uy * gy + uz * gz;
                const float sel = act ? 1.0f : 0.0f;
                const float px = sel * (sY * ux + (gx - ux * ug) * rinv);
                const float py = sel * (sY * uy + (gy - uy * ug) * rinv);
                const float pz = sel * (sY * uz + (gz - uz * ug) * rinv);
                Fx += px; Fy += py; Fz += pz;
                const float hx = -0.5f * dx, hy = -0.5f * dy, hz = -0.5f * dz;
                Wv[0] = fmaf(hx, px, Wv[0]); Wv[1] = fmaf(hx, py, Wv[1]); Wv[2] = fmaf(hx, pz, Wv[2]);
                Wv[3] = fmaf(hy, px, Wv[3]); Wv[4] = fmaf(hy, py, Wv[4]); Wv[5] = fmaf(hy, pz, Wv[5]);
                Wv[6] = fmaf(hz, px, Wv[6]); Wv[7] = fmaf(hz, py, Wv[7]); Wv[8] = fmaf(hz, pz, Wv[8]);
            }
        }
    }

    if (valid) {
        float *Fo = a.Fang + ((size_t)b * N + i) * 3;
        Fo[0] = Fx;
        Fo[1] = Fy;
        Fo[2] = Fz;
        if (a.Watom) {
            float *wo = a.Watom + ((size_t)b * N + i) * 9;
#pragma unroll
            for (int e = 0; e < 9; ++e) wo[e] = Wv[e];
        }
    }
    __shared__ double lds[4];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const double w = block_sum(valid ? (double)Wv[e] : 0.0, lds);
        if (threadIdx.x == 0) a.partWa[((size_t)b * gridDim.x + tile) * 9 + e] = w;
    }
}

// ------------------------------------------------------- pass 2: radial ---

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
    const double *pb = a.pos + (size_t)b * N * 3;
    const double xi = pb[3 * ii], yi = pb[3 * ii + 1], zi = pb[3 * ii + 2];
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    double Wv[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) Wv[e] = 0.0;
    if (valid && tok) {
        const float *ai_base = a.arad + ((size_t)b * N + i) * S * a.KRP;
        for (int t = 0; t < S; ++t) {
            const size_t blk = ((size_t)b * S + t);
            const int cnt = min(a.cntR[blk * N + i], a.capR);
            const int32_t *ix = a.idxR + blk * a.capR * N + i;
            float ai[KR1];
#pragma unroll
            for (int k = 0; k < KR1; ++k) ai[k] = ai_base[t * a.KRP + k];
            for (int s0 = 0; s0 < cnt; s0 += kBatch) {
                int jj[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) jj[u] = (s0 + u < cnt) ? ix[(size_t)(s0 + u) * N] : i;
                double px[kBatch], py[kBatch], pz[kBatch];
                float aj[kBatch][KR1];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    px[u] = pb[3 * jj[u]];
                    py[u] = pb[3 * jj[u] + 1];
                    pz[u] = pb[3 * jj[u] + 2];
                    const float *ajp = a.arad + ((size_t)b * N + jj[u]) * S * a.KRP + ti * a.KRP;
#pragma unroll
                    for (int k = 0; k < KR1; ++k) aj[u][k] = ajp[k];
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    if (s0 + u < cnt) {
                        float dx, dy, dz;
                        pair_vec(px[u], py[u], pz[u], xi, yi, zi, a, dx, dy, dz);
                        const float r2 = dx * dx + dy * dy + dz * dz;
                        const float rinv = __builtin_amdgcn_rsqf(r2);
                        const float r = r2 * rinv;
                        float f[KR1], fp[KR1];
                        cheb_fd<KR1>(r, a.rcRinv, f, fp);
                        float sc = 0.0f;
#pragma unroll
                        for (int k = 0; k < KR1; ++k) sc += (ai[k] + aj[u][k]) * fp[k];
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
            for (int e = 0; e < 9; ++e) wo[e] = (float)(Wv[e] + (double)wo[e]);
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
static void launch(const NepArgs &a, const float *prm, int P, bool sym, hipStream_t s)
{
    const dim3 g(div_up(a.N, kBlock), P);
    {
        ProfScope ps_(K_DESCRIPTOR, s);
        hipLaunchKernelGGL((k_descriptor<NR1, NA1, 9, 9, FOUR>), g, dim3(kBlock), 0, s, a, prm);
    }
    {
        ProfScope ps_(K_FORCE_ANG, s);
        if (sym)
            hipLaunchKernelGGL((k_force_ang<NA1, 9, true, (NA1 <= 5)>), g, dim3(kBlock), 0, s, a, prm);
        else
            hipLaunchKernelGGL((k_force_ang<NA1, 9, false, (NA1 <= 5)>), g, dim3(kBlock), 0, s, a, prm);
    }
    {
        ProfScope ps_(K_FORCE, s);
        hipLaunchKernelGGL((k_force_rad<9>), g, dim3(kBlock), 0, s, a);
    }
}

}  // namespace nep

using namespace nep;

extern "C" int32_t nep_compute(const nep_model *m, const nep_nlist *nl, nep_ws *ws, const double *pos,
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
    if (!box_lengths(box, a.L)) return fail(NEP_ERR_UNSUPPORTED, "nep_compute: only orthorhombic cells");
    for (int d = 0; d < 3; ++d) {
        if (!(a.L[d] > 0.0)) return fail(NEP_ERR_INVALID_ARG, "nep_compute: bad box edge %g", a.L[d]);
        a.invL[d] = 1.0 / a.L[d];
    }
    const nep_hparams &h = m->hp;
    a.pos = pos; a.types = types; a.N = N; a.S = h.n_species; a.H = h.hidden;
    a.rcRinv = (float)(1.0 / h.rc_radial); a.rcAinv = (float)(1.0 / h.rc_angular);
    a.kappa4 = (float)(-4.5 * std::sqrt(2.0 / 35.0) * std::pow(5.0 / (4.0 * M_PI), 1.5));
    a.cntR = nl->cntR; a.idxR = nl->idxR; a.cntA = nl->cntA; a.idxA = nl->idxA;
    a.capR = nl->capR; a.capA = nl->capA;
    a.B = ws->B; a.arad = ws->arad; a.Fang = ws->Fang; a.KRP = ws->KRP;
    a.partE = ws->partE; a.partWa = ws->partW; a.partWr = ws->partW + (size_t)P * ws->nblk * 9;
    a.flags = ws->flags;
    a.F = F; a.Eatom = E_atom; a.Watom = W_atom;
    a.oR = m->off.cR; a.oA = m->off.cA; a.oq = m->off.qs; a.oW0 = m->off.W0; a.ob0 = m->off.b0;
    a.ow1 = m->off.w1; a.ob1 = m->off.b1; a.osh = m->off.sh;
    const bool sym = h.n_species == 1;
    const int key = h.n_max_radial * 100 + h.n_max_angular * 10 + h.four_body;
    switch (key) {
    case 440: launch<5, 5, false>(a, m->dev, P, sym, s); break;
    case 441: launch<5, 5, true>(a, m->dev, P, sym, s); break;
    case 640: launch<7, 5, false>(a, m->dev, P, sym, s); break;
    case 860: launch<9, 7, false>(a, m->dev, P, sym, s); break;
    case 881: launch<9, 9, true>(a, m->dev, P, sym, s); break;
    default: return fail(NEP_ERR_UNSUPPORTED, "nep_compute: unsupported model shape");
    }
    {
        ProfScope ps_(K_REDUCE, s);
        hipLaunchKernelGGL(k_reduce, dim3(P), dim3(64), 0, s, ws->partE, a.partWa, a.partWr, ws->nblk, E, W);
    }
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}
