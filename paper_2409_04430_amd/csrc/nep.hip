// NEP energy, forces and virial on gfx950 (site-energy model of Sec. II.C,
// bead forces and virial of Sec. II.A of arXiv:2409.04430).
//
// Three kernels per call, one lane per (bead, atom):
//   k_descriptor  radial sums, angular sums A_nlm = sum_j g_n(r_ij) Y_lm(u_ij)
//                 over real orthonormal spherical harmonics, q_nl = sum_m A_nlm^2
//                 (equal to the Legendre double sum by the addition theorem),
//                 the optional (2,2,2) four-body invariant, the tanh network,
//                 and the adjoints: B_nlm = dU_i/dA_nlm and the radial
//                 a_k(t) = sum_n dU_i/dq_n c^{ti t}_nk;
//   k_force       gather form F_i = sum_j (dU_i/dr_ij - dU_j/dr_ji) using the
//                 neighbour's adjoints, so no atomics: the angular pair term
//                 is one contraction with B^i_nlm g^{ij}_n + (-1)^l B^j_nlm g^{ji}_n;
//                 per-atom virial -1/2 sum_j r_ij (x) (dU_i/dr_ij - dU_j/dr_ji);
//   k_reduce      per-bead energy and virial from per-block partial sums in
//                 a fixed order (bitwise reproducible).
// Waves run species-uniform: the lanes of a wave are processed in groups
// that share the centre species, which makes every model-coefficient address
// wave-uniform (scalar loads, SGPR operands).
#include "internal.hpp"

namespace nep {

constexpr float kPi = 3.14159265358979f;

struct NepArgs {
    const double *pos;
    const int32_t *types;
    int N, S, H;
    double L[3], invL[3];
    float rcR, rcA, rcRinv, rcAinv;
    float kappa4;
    // lists
    const int32_t *cntR, *idxR, *cntA, *idxA;
    int capR, capA;
    // workspace
    float *B;
    float *arad;
    int KRP;
    double *partE, *partW;
    uint32_t *flags;
    // outputs
    float *F;
    float *Eatom;
    float *Watom;
    // parameter offsets
    int oR, oA, oq, oW0, ob0, ow1, ob1, osh;
};

// Pair vector r_j - r_i under the minimum image, formed in FP64, returned in FP32.
__device__ __forceinline__ void pair_vec(const double *__restrict__ pb, double xi, double yi, double zi, int j,
                                         const NepArgs &a, float &dx, float &dy, float &dz)
{
    double x = pb[3 * j] - xi, y = pb[3 * j + 1] - yi, z = pb[3 * j + 2] - zi;
    x -= a.L[0] * rint(x * a.invL[0]);
    y -= a.L[1] * rint(y * a.invL[1]);
    z -= a.L[2] * rint(z * a.invL[2]);
    dx = (float)x;
    dy = (float)y;
    dz = (float)z;
}

// f_k(r) = (T_k(x) + 1)/2 f_c(r), x = 2 (r/rc - 1)^2 - 1.
template <int K1>
__device__ __forceinline__ void cheb_f(float r, float rcinv, float *f)
{
    const float fc = 0.5f + 0.5f * cosf(kPi * r * rcinv);
    const float y = r * rcinv - 1.0f;
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
    sincosf(kPi * r * rcinv, &sn, &cs);
    const float fc = 0.5f + 0.5f * cs;
    const float fcp = -0.5f * kPi * rcinv * sn;
    const float y = r * rcinv - 1.0f;
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

// ----------------------------------------------------------- pass 1 ---

template <int NR1, int NA1, int KR1, int KA1, bool FOUR>
__global__ __launch_bounds__(kBlock) void k_descriptor(NepArgs a, const float *__restrict__ prm)
{
    constexpr int D = Dims<NR1, NA1, FOUR>::D;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    const int N = a.N, S = a.S;
    const bool valid = i < N;
    const int ii = valid ? i : N - 1;
    int ti = a.types[ii];
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
            for (int s = 0; s < cnt; ++s) {
                const int j = ix[(size_t)s * N];
                float dx, dy, dz;
                pair_vec(pb, xi, yi, zi, j, a, dx, dy, dz);
                const float r = sqrtf(dx * dx + dy * dy + dz * dz);
                float f[KR1];
                cheb_f<KR1>(r, a.rcRinv, f);
#pragma unroll
                for (int k = 0; k < KR1; ++k) sk[k] += f[k];
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
            for (int s = 0; s < cnt; ++s) {
                const int j = ix[(size_t)s * N];
                float dx, dy, dz;
                pair_vec(pb, xi, yi, zi, j, a, dx, dy, dz);
                const float r = sqrtf(dx * dx + dy * dy + dz * dz);
                const float rinv = 1.0f / r;
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
        }
        // four-body: M_n = sum_j g_n (u u^T - I/3) rebuilt from the l = 2 sums
        float Mc[FOUR ? NA1 : 1][5];   // mxy, myz, mzz, mxz, d = mxx - myy
        if (FOUR) {
#pragma unroll
            for (int n = 0; n < (FOUR ? NA1 : 1); ++n) {
                const float mxy = A[n][3] / shc[3], myz = A[n][4] / shc[4];
                const float mzz = A[n][5] / (3.0f * shc[5]), mxz = A[n][6] / shc[6], dd = A[n][7] / shc[7];
                const float mxx = 0.5f * (dd - mzz), myy = 0.5f * (-dd - mzz);
                Mc[n][0] = mxy; Mc[n][1] = myz; Mc[n][2] = mzz; Mc[n][3] = mxz; Mc[n][4] = dd;
                const float tr3 = mxx * mxx * mxx + myy * myy * myy + mzz * mzz * mzz +
                                  3.0f * mxx * (mxy * mxy + mxz * mxz) + 3.0f * myy * (mxy * mxy + myz * myz) +
                                  3.0f * mzz * (mxz * mxz + myz * myz) + 6.0f * mxy * myz * mxz;
                q[NR1 + kLmax * NA1 + n] = a.kappa4 * tr3;
            }
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

        // adjoints: B_nlm = dU/dA_nlm
        float *Bo = a.B + ((size_t)b * N + i) * (NA1 * kNumSH);
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            float Bn[kNumSH];
#pragma unroll
            for (int m = 0; m < kNumSH; ++m) Bn[m] = 2.0f * G[NR1 + (sh_l(m) - 1) * NA1 + n] * A[n][m];
            if (FOUR) {
                const float mxy = Mc[n][0], myz = Mc[n][1], mzz = Mc[n][2], mxz = Mc[n][3], dd = Mc[n][4];
                const float mxx = 0.5f * (dd - mzz), myy = 0.5f * (-dd - mzz);
                // M^2 entries
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
            float4 *o4 = reinterpret_cast<float4 *>(Bo + n * kNumSH);
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
    if (threadIdx.x == 0) a.partE[(size_t)b * gridDim.x + blockIdx.x] = e;
}

// ----------------------------------------------------------- pass 2 ---

template <int NR1, int NA1, int KR1, int KA1, bool FOUR>
__global__ __launch_bounds__(kBlock) void k_force(NepArgs a, const float *__restrict__ prm)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    const int N = a.N, S = a.S;
    const bool valid = i < N;
    const int ii = valid ? i : N - 1;
    const int ti = a.types[ii];
    const bool tok = ti >= 0 && ti < S;
    const double *pb = a.pos + (size_t)b * N * 3;
    const double xi = pb[3 * ii], yi = pb[3 * ii + 1], zi = pb[3 * ii + 2];
    const float *shc = prm + a.osh;
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    double Wv[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) Wv[e] = 0.0;

    uint64_t todo = __ballot(valid && tok);
    while (todo) {
        const int lead = __builtin_ctzll(todo);
        const int tc = __builtin_amdgcn_readlane(ti, lead);
        const bool mine = valid && tok && ti == tc;
        todo &= ~__ballot(mine);
        if (!mine) continue;

        // radial: phi = sum_k (a^i_k(tj) + a^j_k(ti)) f'_k(r) u
        const float *ai_base = a.arad + ((size_t)b * N + i) * S * a.KRP;
        for (int t = 0; t < S; ++t) {
            const size_t blk = ((size_t)b * S + t);
            const int cnt = min(a.cntR[blk * N + i], a.capR);
            const int32_t *ix = a.idxR + blk * a.capR * N + i;
            float ai[KR1];
#pragma unroll
            for (int k = 0; k < KR1; ++k) ai[k] = ai_base[t * a.KRP + k];
            for (int s = 0; s < cnt; ++s) {
                const int j = ix[(size_t)s * N];
                float dx, dy, dz;
                pair_vec(pb, xi, yi, zi, j, a, dx, dy, dz);
                const float r = sqrtf(dx * dx + dy * dy + dz * dz);
                float f[KR1], fp[KR1];
                cheb_fd<KR1>(r, a.rcRinv, f, fp);
                const float *aj = a.arad + ((size_t)b * N + j) * S * a.KRP + tc * a.KRP;
                float sc = 0.0f;
#pragma unroll
                for (int k = 0; k < KR1; ++k) sc += (ai[k] + aj[k]) * fp[k];
                const float w = sc / r;
                const float px = w * dx, py = w * dy, pz = w * dz;
                Fx += px; Fy += py; Fz += pz;
                Wv[0] -= 0.5 * dx * px; Wv[1] -= 0.5 * dx * py; Wv[2] -= 0.5 * dx * pz;
                Wv[3] -= 0.5 * dy * px; Wv[4] -= 0.5 * dy * py; Wv[5] -= 0.5 * dy * pz;
                Wv[6] -= 0.5 * dz * px; Wv[7] -= 0.5 * dz * py; Wv[8] -= 0.5 * dz * pz;
            }
        }

        // angular
        const float *Bi = a.B + ((size_t)b * N + i) * (NA1 * kNumSH);
        for (int t = 0; t < S; ++t) {
            const size_t blk = ((size_t)b * S + t);
            const int cnt = min(a.cntA[blk * N + i], a.capA);
            const int32_t *ix = a.idxA + blk * a.capA * N + i;
            const float *cij = prm + a.oA + (tc * S + t) * NA1 * KA1;
            const float *cji = prm + a.oA + (t * S + tc) * NA1 * KA1;
            for (int s = 0; s < cnt; ++s) {
                const int j = ix[(size_t)s * N];
                float dx, dy, dz;
                pair_vec(pb, xi, yi, zi, j, a, dx, dy, dz);
                const float r = sqrtf(dx * dx + dy * dy + dz * dz);
                const float rinv = 1.0f / r;
                const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
                float f[KA1], fp[KA1];
                cheb_fd<KA1>(r, a.rcAinv, f, fp);
                const float *Bj = a.B + ((size_t)b * N + j) * (NA1 * kNumSH);
                float beta[kNumSH], betap[kNumSH];
#pragma unroll
                for (int m = 0; m < kNumSH; ++m) {
                    beta[m] = 0.0f;
                    betap[m] = 0.0f;
                }
#pragma unroll
                for (int n = 0; n < NA1; ++n) {
                    float gij = 0.0f, gpij = 0.0f, gji = 0.0f, gpji = 0.0f;
#pragma unroll
                    for (int k = 0; k < KA1; ++k) {
                        gij += cij[n * KA1 + k] * f[k];
                        gpij += cij[n * KA1 + k] * fp[k];
                        gji += cji[n * KA1 + k] * f[k];
                        gpji += cji[n * KA1 + k] * fp[k];
                    }
                    const float4 *bi4 = reinterpret_cast<const float4 *>(Bi + n * kNumSH);
                    const float4 *bj4 = reinterpret_cast<const float4 *>(Bj + n * kNumSH);
#pragma unroll
                    for (int q4 = 0; q4 < kNumSH / 4; ++q4) {
                        const float4 x = bi4[q4], y = bj4[q4];
                        const float bi[4] = {x.x, x.y, x.z, x.w};
                        const float bj[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int m = 4 * q4 + e;
                            const float sj = (sh_l(m) & 1) ? -bj[e] : bj[e];
                            beta[m] += bi[e] * gij + sj * gji;
                            betap[m] += bi[e] * gpij + sj * gpji;
                        }
                    }
                }
                float sY, gx, gy, gz;
                sh_contract(ux, uy, uz, shc, beta, betap, sY, gx, gy, gz);
                const float ug = ux * gx + uy * gy + uz * gz;
                const float px = sY * ux + (gx - ux * ug) * rinv;
                const float py = sY * uy + (gy - uy * ug) * rinv;
                const float pz = sY * uz + (gz - uz * ug) * rinv;
                Fx += px; Fy += py; Fz += pz;
                Wv[0] -= 0.5 * dx * px; Wv[1] -= 0.5 * dx * py; Wv[2] -= 0.5 * dx * pz;
                Wv[3] -= 0.5 * dy * px; Wv[4] -= 0.5 * dy * py; Wv[5] -= 0.5 * dy * pz;
                Wv[6] -= 0.5 * dz * px; Wv[7] -= 0.5 * dz * py; Wv[8] -= 0.5 * dz * pz;
            }
        }
    }

    if (valid) {
        float *Fo = a.F + ((size_t)b * N + i) * 3;
        Fo[0] = (float)Fx;
        Fo[1] = (float)Fy;
        Fo[2] = (float)Fz;
        if (a.Watom) {
            float *wo = a.Watom + ((size_t)b * N + i) * 9;
#pragma unroll
            for (int e = 0; e < 9; ++e) wo[e] = (float)Wv[e];
        }
        if (!(isfinite(Fx) && isfinite(Fy) && isfinite(Fz))) atomicOr(a.flags, (uint32_t)NEP_FLAG_NONFINITE);
    }
    __shared__ double lds[4];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const double w = block_sum(valid ? Wv[e] : 0.0, lds);
        if (threadIdx.x == 0) a.partW[((size_t)b * gridDim.x + blockIdx.x) * 9 + e] = w;
    }
}

// Per-bead totals from the per-block partial sums, in block order.
__global__ void k_reduce(const double *__restrict__ partE, const double *__restrict__ partW, int nblk,
                         double *__restrict__ E, double *__restrict__ W)
{
    const int b = blockIdx.x, t = threadIdx.x;
    if (t == 0) {
        double s = 0.0;
        for (int k = 0; k < nblk; ++k) s += partE[(size_t)b * nblk + k];
        E[b] = s;
    } else if (t <= 9) {
        double s = 0.0;
        for (int k = 0; k < nblk; ++k) s += partW[((size_t)b * nblk + k) * 9 + (t - 1)];
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
        ProfScope ps_(K_FORCE, s);
        hipLaunchKernelGGL((k_force<NR1, NA1, 9, 9, FOUR>), g, dim3(kBlock), 0, s, a, prm);
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
    a.rcR = (float)h.rc_radial; a.rcA = (float)h.rc_angular;
    a.rcRinv = (float)(1.0 / h.rc_radial); a.rcAinv = (float)(1.0 / h.rc_angular);
    a.kappa4 = (float)(-4.5 * std::sqrt(2.0 / 35.0) * std::pow(5.0 / (4.0 * M_PI), 1.5));
    a.cntR = nl->cntR; a.idxR = nl->idxR; a.cntA = nl->cntA; a.idxA = nl->idxA;
    a.capR = nl->capR; a.capA = nl->capA;
    a.B = ws->B; a.arad = ws->arad; a.KRP = ws->KRP;
    a.partE = ws->partE; a.partW = ws->partW; a.flags = ws->flags;
    a.F = F; a.Eatom = E_atom; a.Watom = W_atom;
    a.oR = m->off.cR; a.oA = m->off.cA; a.oq = m->off.qs; a.oW0 = m->off.W0; a.ob0 = m->off.b0;
    a.ow1 = m->off.w1; a.ob1 = m->off.b1; a.osh = m->off.sh;
    const int key = h.n_max_radial * 100 + h.n_max_angular * 10 + h.four_body;
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
        hipLaunchKernelGGL(k_reduce, dim3(P), dim3(64), 0, s, ws->partE, ws->partW, ws->nblk, E, W);
    }
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}
