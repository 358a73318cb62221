// NEP energy, forces and virial on gfx950 (site-energy model of Sec. II.C,
// bead forces and virial of Sec. II.A of arXiv:2409.04430).
//
// Four kernels per call, one lane per (bead, atom), neighbours taken from
// the per-bead compact lists built over the shared centroid candidate rows:
//   k_descriptor  radial sums, angular sums A_nlm = sum_j g_n(r_ij) Y_lm(u_ij)
//                 over real orthonormal spherical harmonics, q_nl = sum_m A_nlm^2
//                 (equal to the Legendre double sum by the addition theorem),
//                 the optional (2,2,2) four-body invariant, the tanh network,
//                 and the adjoints: B_nlm = dU_i/dA_nlm (stored times the
//                 harmonic's normalisation c_m) and the radial
//                 a_k(t) = sum_n dU_i/dq_n c^{ti t}_nk (with their sum over k > 0);
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
#include "nep_kernels.hpp"

namespace nep {

// ------------------------------------------ matrix-core network ---

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Orders this wavefront's LDS writes before its later LDS reads (LDS
// operations of one wavefront complete in issue order).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Eight FP32 values as three BF16 vectors whose sum is exact: truncation
// keeps the top 8 significant bits, the remainder's top 8 bits follow, and
// the last remainder has at most 8 significant bits left.
__device__ __forceinline__ void split3(const float (&x)[8], bf16x8 &hi, bf16x8 &mid, bf16x8 &lo)
{
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const uint32_t u0 = __float_as_uint(x[e]) & 0xffff0000u;
        const float r1 = x[e] - __uint_as_float(u0);
        const uint32_t u1 = __float_as_uint(r1) & 0xffff0000u;
        const float r2 = r1 - __uint_as_float(u1);
        hi[e] = __builtin_bit_cast(__bf16, (uint16_t)(u0 >> 16));
        mid[e] = __builtin_bit_cast(__bf16, (uint16_t)(u1 >> 16));
        lo[e] = __builtin_bit_cast(__bf16, (uint16_t)(__float_as_uint(r2) >> 16));
    }
}

// C += A B over the BF16 terms of both operands: A (weights) with WT terms,
// B (activations) with three.  WT = 1: the three products; WT = 3: the six
// products of term indices i + j <= 2 (a dropped product is below 2^-22 of
// the full one).
template <int WT>
__device__ __forceinline__ f32x4 mfma_terms(const bf16x8 (&a)[WT], const bf16x8 (&b)[3], f32x4 c)
{
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], b[2], c, 0, 0, 0);
    if constexpr (WT == 3) {
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], b[1], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], b[0], c, 0, 0, 0);
    }
    return c;
}

// tanh and its slope, both to a few units in the last place over the whole
// range.  With a = |z| and r = 2 / (exp(2 a) + 1) in (0, 1]:
// |tanh z| = 1 - r and 1 - tanh^2 z = r (2 - r), free of cancellation for
// a >= 1/2 (r <= 0.54) and, for the slope, everywhere (exp saturates to inf
// for large a, so r = 0).  Below a = 1/2, tanh z = z f(z^2) with f the
// Maclaurin series of tanh(z) / z, whose coefficients are
// 2^2k (2^2k - 1) B_2k / (2k)! (B the Bernoulli numbers); through z^15 the
// series is exact to 1e-8 relative there.
__device__ __forceinline__ void tanh_and_slope(float z, float &h, float &dh)
{
    const float a = fabsf(z);
    const float r = 2.0f * __builtin_amdgcn_rcpf(__expf(2.0f * a) + 1.0f);
    dh = r * (2.0f - r);
    const float t = z * z;
    float f = -929569.0f / 638512875.0f;
    f = fmaf(f, t, 21844.0f / 6081075.0f);
    f = fmaf(f, t, -1382.0f / 155925.0f);
    f = fmaf(f, t, 62.0f / 2835.0f);
    f = fmaf(f, t, -17.0f / 315.0f);
    f = fmaf(f, t, 2.0f / 15.0f);
    f = fmaf(f, t, -1.0f / 3.0f);
    f = fmaf(f, t, 1.0f);
    h = a < 0.5f ? z * f : copysignf(1.0f - r, z);
}

// The network of the wavefront's 64 (atom, bead) rows on the matrix cores,
// as transposed products: Z^T = W0 Qh^T (A operand = weights, rows = hidden
// units; B operand = the scaled descriptors, columns = rows of the batch),
// h = tanh(Z - b0), U = w1 . h - b1, and G^T = W0^T (w1 (1 - h^2))^T.  The
// hidden units of a forward result tile sit in the lanes exactly where the
// adjoint product takes them as its B operand (its K order is permuted to
// match, in the weight fragments), so the hidden layer never leaves
// registers.  Qh is staged once in this wavefront's LDS tile X (64 rows of
// XS floats); each row's G and U are written back over it.  Zero rows for
// lanes outside the current species (mine = false).  Returns U of the
// lane's row and G (without the descriptor scale) in G[0..D).
template <int D, int WT>
__device__ float mlp_mf(const float (&qh)[D], bool mine, const uint16_t *__restrict__ frag, const float *b0,
                        const float *w1, float b1, int H, float *X, float (&G)[D])
{
    constexpr int DP = D <= 32 ? 32 : 64, KC = DP / 32, DT = DP / 16, XS = DP + 4;
    // batch tiles (16 rows each) per pass: every weight fragment is loaded
    // once per pass, and a pass keeps its tiles' operands and accumulators
    // in registers
    constexpr int JB = DP == 32 ? 4 : 2;
    const int HC = (H + 31) >> 5, HT = 2 * HC;
    const int l = threadIdx.x & 63, c = l & 15, g = l >> 4;
#pragma unroll
    for (int v4 = 0; v4 < DP / 4; ++v4) {
        float w[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int v = 4 * v4 + e;
            w[e] = (mine && v < D) ? qh[v < D ? v : 0] : 0.0f;
        }
        *reinterpret_cast<float4 *>(X + l * XS + 4 * v4) = make_float4(w[0], w[1], w[2], w[3]);
    }
    wave_lds_sync();
    const bf16x8 *fw = reinterpret_cast<const bf16x8 *>(frag) + l;   // one 8-entry fragment per lane and block
    const int fwd = HT * KC, tstride = fwd + DT * HC;                 // blocks per term
    for (int j0 = 0; j0 < 4; j0 += JB) {
        // B operands of the forward product: column c of tile j = batch row 16 j + c
        bf16x8 xb[JB][KC][3];
#pragma unroll
        for (int jj = 0; jj < JB; ++jj) {
            const float *xr = X + (16 * (j0 + jj) + c) * XS + 8 * g;
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                const float4 a0 = *reinterpret_cast<const float4 *>(xr + 32 * kc);
                const float4 a1 = *reinterpret_cast<const float4 *>(xr + 32 * kc + 4);
                const float x8[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
                split3(x8, xb[jj][kc][0], xb[jj][kc][1], xb[jj][kc][2]);
            }
        }
        f32x4 gacc[JB][DT];
        float uacc[JB];
#pragma unroll
        for (int jj = 0; jj < JB; ++jj) {
            uacc[jj] = 0.0f;
#pragma unroll
            for (int dt = 0; dt < DT; ++dt) gacc[jj][dt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        }
        for (int hc = 0; hc < HC; ++hc) {
            // this lane's eight hidden units of the chunk: 32 hc + 16 h2 + 4 g + e
            float bq[8], wq[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int mu = 32 * hc + 16 * (q >> 2) + 4 * g + (q & 3);
                bq[q] = mu < H ? b0[mu] : 0.0f;
                wq[q] = mu < H ? w1[mu] : 0.0f;
            }
            float gz[JB][8];
#pragma unroll
            for (int h2 = 0; h2 < 2; ++h2) {
                const int ht = 2 * hc + h2;
                bf16x8 wa[KC][WT];
#pragma unroll
                for (int kc = 0; kc < KC; ++kc)
#pragma unroll
                    for (int t = 0; t < WT; ++t) wa[kc][t] = fw[(t * tstride + ht * KC + kc) * 64];
#pragma unroll
                for (int jj = 0; jj < JB; ++jj) {
                    f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                    for (int kc = 0; kc < KC; ++kc) z = mfma_terms<WT>(wa[kc], xb[jj][kc], z);
                    // z[e]: hidden unit 16 ht + 4 g + e of batch row 16 (j0 + jj) + c
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        float hh, dh;
                        tanh_and_slope(z[e] - bq[4 * h2 + e], hh, dh);
                        uacc[jj] = fmaf(wq[4 * h2 + e], hh, uacc[jj]);
                        gz[jj][4 * h2 + e] = wq[4 * h2 + e] * dh;
                    }
                }
            }
            // adjoint: B operand gz^T in K order (4 g + e, 16 + 4 g + e) as in the fragments
            bf16x8 wt[DT][WT];
#pragma unroll
            for (int dt = 0; dt < DT; ++dt)
#pragma unroll
                for (int t = 0; t < WT; ++t) wt[dt][t] = fw[(t * tstride + fwd + dt * HC + hc) * 64];
#pragma unroll
            for (int jj = 0; jj < JB; ++jj) {
                bf16x8 gb[3];
                split3(gz[jj], gb[0], gb[1], gb[2]);
#pragma unroll
                for (int dt = 0; dt < DT; ++dt) gacc[jj][dt] = mfma_terms<WT>(wt[dt], gb, gacc[jj][dt]);
            }
        }
#pragma unroll
        for (int jj = 0; jj < JB; ++jj) {
            // U of column c: the four lane groups hold different hidden units
            float u = uacc[jj];
            u += __shfl_xor(u, 16, 64);
            u += __shfl_xor(u, 32, 64);
            // G^T (descriptor 16 dt + 4 g + e, column c) back over the row, which
            // this wavefront has finished reading (its LDS operations run in order)
            float *xo = X + (16 * (j0 + jj) + c) * XS;
#pragma unroll
            for (int dt = 0; dt < DT; ++dt)
                *reinterpret_cast<float4 *>(xo + 16 * dt + 4 * g) =
                    make_float4(gacc[jj][dt][0], gacc[jj][dt][1], gacc[jj][dt][2], gacc[jj][dt][3]);
            if (g == 0) xo[DP] = u;
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int v = 0; v < D; ++v) G[v] = X[l * XS + v];
    const float u = X[l * XS + DP] - b1;
    wave_lds_sync();   // X is rewritten by the next species of this wavefront
    return u;
}

// LDS floats per wavefront of the matrix-core network.
template <int D>
constexpr int mf_lds_floats() { return 64 * ((D <= 32 ? 32 : 64) + 4); }

// Network arithmetic of k_descriptor: FP32 vector units with the weights
// read from global memory or staged in LDS; BF16 matrix cores with BF16
// weights (the student); or BF16 matrix cores with the FP32 weights as
// three exact BF16 terms (FP32 accuracy).  (FP32 operands on the matrix
// cores, 16 x 16 x 4 FP32 tiles, measured slower than the LDS-staged vector
// form: two wavefronts per SIMD cannot hide their dependent chains.)
constexpr int kNetGlobal = 0, kNetLds = 1, kNetBf16 = 2, kNetMf32 = 3;
constexpr int kNetRowRegs = 40;   // longest descriptor whose weight rows the LDS network holds in registers

// ----------------------------------------------------------- pass 1 ---

template <int NR1, int NA1, int KR1, int KA1, bool FOUR, int NET, bool TRI>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
void k_descriptor(NepArgs a, const float *__restrict__ prm)
{
    constexpr bool MF = NET == kNetBf16 || NET == kNetMf32;   // whole-wavefront network on the matrix cores
    constexpr bool NL = NET == kNetLds;
    // dynamic LDS: matrix-core network, one 64 x (32 or 64, + 4) tile per
    // wavefront; LDS weights, W0 [S][H][DP] (rows padded to DP = 4 ceil(D / 4)),
    // b0 [S][H], w1 [S][H]
    extern __shared__ float dyn[];
    constexpr int D = Dims<NR1, NA1, FOUR>::D;
    const LaneMap lm = lane_map(a);
    const int i = lm.i, b = lm.b, P = a.P, S = a.S;
    const bool valid = lm.valid;
    const int ti = a.types[i];
    const bool tok = ti >= 0 && ti < S;
    const float4 *p4 = a.p4;
    const float4 pi = p4[(size_t)i * P + b];
    const float *shc = prm + a.osh;
    float U = 0.0f;

    constexpr int DP = (D + 3) & ~3;
    if constexpr (NL) {
        const int nw = S * a.H * DP, nb = S * a.H;
        for (int x = threadIdx.x; x < nw; x += blockDim.x) {
            const int row = x / DP, v = x - row * DP;
            dyn[x] = v < D ? prm[a.oW0 + row * D + v] : 0.0f;
        }
        for (int x = threadIdx.x; x < nb; x += blockDim.x) {
            dyn[nw + x] = prm[a.ob0 + x];
            dyn[nw + nb + x] = prm[a.ow1 + x];
        }
        __syncthreads();
    }

    uint64_t todo = __ballot(valid && tok);
    while (todo) {
        const int lead = __builtin_ctzll(todo);
        const int tc = __builtin_amdgcn_readlane(ti, lead);
        const bool mine = valid && tok && ti == tc;
        todo &= ~__ballot(mine);
        if constexpr (!MF) {
            if (!mine) continue;
        }

        float q[D];
#pragma unroll
        for (int v = 0; v < D; ++v) q[v] = 0.0f;
        // the wavefront's adjoint rows, interleaved (adj_rows): each float4
        // store or load of the wavefront covers 1 KiB contiguously
        const __amdgpu_buffer_rsrc_t Bo = adj_rows(a.B, NA1 * (kNumSH / 4));
        // A stays in registers through the network for small angular sets;
        // otherwise it is parked in the lane's adjoint row, where the
        // angular force kernel reads it
        constexpr bool PARK = adj_parked(MF, NA1);
        float Ar[PARK ? 1 : NA1][kNumSH];
        if (MF ? mine : true) {

        // radial: per neighbour species, sum the basis, then contract with c
        const int32_t *uR = a.uniR + (size_t)i * a.capR;
        const uint64_t *mR = a.umR + (size_t)i * a.capR;
        for (int t = 0; t < S; ++t) {
            int s0, s1;
            block_range(a.uendR, i, t, s0, s1);
            float sk[KR1];
#pragma unroll
            for (int k = 0; k < KR1; ++k) sk[k] = 0.0f;
            for (int sb = s0; sb < s1; sb += kBatchR) {
                int jj[kBatchR];
                bool in[kBatchR];
                float4 pj[kBatchR];
                // every load unconditional (slots past the block end reread
                // its last entry, masked off) so that the batch's loads are
                // in flight together
#pragma unroll
                for (int u = 0; u < kBatchR; ++u) {
                    const int su = min(sb + u, s1 - 1);
                    jj[u] = uR[su];
                    const uint64_t mu = mR[su];
                    in[u] = (sb + u < s1) & (((mu >> b) & 1u) != 0);
                }
#pragma unroll
                for (int u = 0; u < kBatchR; ++u) pj[u] = p4[(size_t)jj[u] * P + b];
#pragma unroll
                for (int u = 0; u < kBatchR; ++u) keep(pj[u]);
#pragma unroll
                for (int u = 0; u < kBatchR; ++u) {
                    if (in[u]) {
                        float dx, dy, dz;
                        pair_vec<TRI>(pj[u], pi, lm, dx, dy, dz);
                        const float r2 = dx * dx + dy * dy + dz * dz;
                        {
                            // sk[0] collects f_c, sk[k > 0] collects f_c T_k
                            const float r = __builtin_amdgcn_sqrtf(r2);
                            float fc, T[KR1];
                            cheb_t<KR1>(r, a.rcRinv, fc, T);
                            sk[0] += fc;
#pragma unroll
                            for (int q2 = 1; q2 < KR1; ++q2) sk[q2] = fmaf(fc, T[q2], sk[q2]);
                        }
                    }
                }
            }
            // sum_j f_k = (sum f_c T_k + sum f_c) / 2 for k > 0, sum f_c for k = 0
#pragma unroll
            for (int q2 = 1; q2 < KR1; ++q2) sk[q2] = 0.5f * (sk[q2] + sk[0]);
            const float *c = prm + a.oR + (tc * S + t) * NR1 * KR1;
#pragma unroll
            for (int n = 0; n < NR1; ++n) {
                float acc = q[n];
#pragma unroll
                for (int q2 = 0; q2 < KR1; ++q2) acc += c[n * KR1 + q2] * sk[q2];
                q[n] = acc;
            }
        }

        // angular: A_nlm = sum_j g_n(r_ij) Y_lm(u_ij), NG radial functions n
        // per pass over the neighbours (all of them when A stays in
        // registers; in three passes when more than five are parked, so that
        // the accumulators of one pass fit the registers), each pass's q
        // entries formed and its A parked before the next
        constexpr int NG = NA1 > 5 ? (NA1 + 2) / 3 : NA1;
        const int32_t *uA = a.uniA + (size_t)i * a.capA;
        const uint64_t *mA = a.umA + (size_t)i * a.capA;
        const int32_t *rowA = a.candA + (size_t)i * a.capA;
#pragma unroll
        for (int n0 = 0; n0 < NA1; n0 += NG) {
        float A[NG][kNumSH];
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int m = 0; m < kNumSH; ++m) A[g][m] = 0.0f;
        for (int t = 0; t < S; ++t) {
            int s0, s1;
            block_range(a.uendA, i, t, s0, s1);
            const float *c = prm + __builtin_amdgcn_readfirstlane(a.oA + (tc * S + t) * NA1 * KA1);   // uniform
            // g_n = f_c / 2 (cs_n + sum_{k>0} c_nk T_k), cs_n = c_n0 + sum_k c_nk
            float cs[NG];
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int n = n0 + g < NA1 ? n0 + g : NA1 - 1;
                float acc = c[n * KA1];
#pragma unroll
                for (int q2 = 0; q2 < KA1; ++q2) acc += c[n * KA1 + q2];
                cs[g] = acc;
            }
            // batches of kBatch entries: slots, then partners, then their
            // positions, each level's loads in flight together (slots past
            // the block end reread its last entry, masked off)
            for (int sb = s0; sb < s1; sb += kBatch) {
                // coefficients through scalar loads, which do not wait on the gathers
                const cf32p cl = launder(c);
                int kq[kBatch];
                bool in[kBatch];
                float4 pj[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int su = min(sb + u, s1 - 1);
                    kq[u] = uA[su];
                    const uint64_t mu = mA[su];
                    in[u] = (sb + u < s1) & (((mu >> b) & 1u) != 0);
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) kq[u] = rowA[kq[u]] >> 2;
#pragma unroll
                for (int u = 0; u < kBatch; ++u) pj[u] = p4[(size_t)kq[u] * P + b];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) keep(pj[u]);
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    if (!in[u]) continue;
                    float dx, dy, dz;
                    pair_vec<TRI>(pj[u], pi, lm, dx, dy, dz);
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    const float rinv = __builtin_amdgcn_rsqf(r2);
                    const float r = r2 * rinv;
                    float fc, T[KA1];
                    cheb_t<KA1>(r, a.rcAinv, fc, T);
                    const float hf = 0.5f * fc;
                    // bare polynomials: the normalisations c_m are applied to the sums below
                    float Y[kNumSH];
                    sh_eval(dx * rinv, dy * rinv, dz * rinv, UnitNorm{}, Y);
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        const int n = n0 + g;
                        if (n >= NA1) break;
                        float gn = cs[g];
#pragma unroll
                        for (int q2 = 1; q2 < KA1; ++q2) gn = fmaf(cl[n * KA1 + q2], T[q2], gn);
                        gn *= hf;
#pragma unroll
                        for (int m = 0; m < kNumSH; ++m) A[g][m] += gn * Y[m];
                    }
                }
            }
        }
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const int n = n0 + g;
            if (n >= NA1) break;
#pragma unroll
            for (int m = 0; m < kNumSH; ++m) A[g][m] *= shc[m];   // A_nlm = c_m sum_j g_n p_m
#pragma unroll
            for (int l = 1; l <= kLmax; ++l) {
                float s2 = 0.0f;
#pragma unroll
                for (int m = 0; m < kNumSH; ++m)
                    if (sh_l(m) == l) s2 += A[g][m] * A[g][m];
                q[NR1 + (l - 1) * NA1 + n] = s2;
            }
            if (FOUR) {
                float M[5];
                m_from_l2(&A[g][3], shc, M);
                const float mxy = M[0], myz = M[1], mzz = M[2], mxz = M[3], dd = M[4];
                const float mxx = 0.5f * (dd - mzz), myy = 0.5f * (-dd - mzz);
                const float tr3 = mxx * mxx * mxx + myy * myy * myy + mzz * mzz * mzz +
                                  3.0f * mxx * (mxy * mxy + mxz * mxz) + 3.0f * myy * (mxy * mxy + myz * myz) +
                                  3.0f * mzz * (mxz * mxz + myz * myz) + 6.0f * mxy * myz * mxz;
                q[NR1 + kLmax * NA1 + n] = a.kappa4 * tr3;
            }
            if constexpr (PARK) {
                // park A in this lane's adjoint row (the angular force kernel forms B from it)
#pragma unroll
                for (int q4 = 0; q4 < kNumSH / 4; ++q4)
                    adj_store(Bo, n * (kNumSH / 4) + q4,
                              make_float4(A[g][4 * q4], A[g][4 * q4 + 1], A[g][4 * q4 + 2], A[g][4 * q4 + 3]));
            } else {
#pragma unroll
                for (int m = 0; m < kNumSH; ++m) Ar[PARK ? 0 : n][m] = A[g][m];
            }
        }
        }   // angular passes
        }   // descriptors of the lanes of species tc

        // network: U = sum_mu w1 tanh(sum_nu W0 s_nu q_nu - b0) - b1;  G_nu = dU/dq_nu
        const float *qs = prm + a.oq;
        float qh[D], G[D];
#pragma unroll
        for (int v = 0; v < D; ++v) {
            qh[v] = qs[v] * q[v];
            G[v] = 0.0f;
        }
        if constexpr (MF) {
            constexpr int WT = NET == kNetMf32 ? 3 : 1;
            const float *b0 = prm + a.ob0 + tc * a.H;
            const float *w1 = prm + a.ow1 + tc * a.H;
            float *X = dyn + (threadIdx.x >> 6) * mf_lds_floats<D>();
            const MlpFrag fl = mlp_frag_layout(D, a.H, WT);
            const float u = mlp_mf<D, WT>(qh, mine, a.w0b + (size_t)tc * fl.species_stride, b0, w1, prm[a.ob1],
                                          a.H, X, G);
            if (mine) U = u;
        } else if constexpr (NL) {
            const int nw = S * a.H * DP, nb = S * a.H;
            const float *W0 = dyn + tc * a.H * DP;
            const float *b0 = dyn + nw + tc * a.H;
            const float *w1 = dyn + nw + nb + tc * a.H;
            float u = -prm[a.ob1];
            if constexpr (D <= kNetRowRegs) {
                for (int mu = 0; mu < a.H; ++mu) {
                    // the weight row in registers, read from LDS once for both products
                    const float4 *w4 = reinterpret_cast<const float4 *>(W0 + mu * DP);
                    float wr[DP];
#pragma unroll
                    for (int v4 = 0; v4 < DP / 4; ++v4) {
                        const float4 t4 = w4[v4];
                        wr[4 * v4] = t4.x; wr[4 * v4 + 1] = t4.y; wr[4 * v4 + 2] = t4.z; wr[4 * v4 + 3] = t4.w;
                    }
                    float z = -b0[mu];
#pragma unroll
                    for (int v = 0; v < D; ++v) z += wr[v] * qh[v];
                    float h, dh;
                    tanh_and_slope(z, h, dh);
                    u += w1[mu] * h;
                    const float gz = w1[mu] * dh;
#pragma unroll
                    for (int v = 0; v < D; ++v) G[v] += gz * wr[v];
                }
            } else {
                // long rows: read from LDS in 4-wide chunks for each product
                // (broadcast reads), so the row takes no registers; one hidden
                // unit per iteration (unrolling interleaves rows and spills)
#pragma unroll 1
                for (int mu = 0; mu < a.H; ++mu) {
                    const float4 *w4 = reinterpret_cast<const float4 *>(W0 + mu * DP);
                    float z = -b0[mu];
#pragma unroll
                    for (int v4 = 0; v4 < DP / 4; ++v4) {
                        const float4 t4 = w4[v4];
                        const float wq[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (4 * v4 + e < D) z += wq[e] * qh[4 * v4 + e < D ? 4 * v4 + e : 0];
                    }
                    float h, dh;
                    tanh_and_slope(z, h, dh);
                    u += w1[mu] * h;
                    const float gz = w1[mu] * dh;
#pragma unroll
                    for (int v4 = 0; v4 < DP / 4; ++v4) {
                        const float4 t4 = w4[v4];
                        const float wq[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (4 * v4 + e < D) G[4 * v4 + e < D ? 4 * v4 + e : 0] += gz * wq[e];
                    }
                }
            }
            U = u;
        } else {
            const float *W0 = prm + a.oW0 + tc * a.H * D;
            const float *b0 = prm + a.ob0 + tc * a.H;
            const float *w1 = prm + a.ow1 + tc * a.H;
            float u = -prm[a.ob1];
            for (int mu = 0; mu < a.H; ++mu) {
                float z = -b0[mu];
#pragma unroll
                for (int v = 0; v < D; ++v) z += W0[mu * D + v] * qh[v];
                float h, dh;
                tanh_and_slope(z, h, dh);
                u += w1[mu] * h;
                const float gz = w1[mu] * dh;
#pragma unroll
                for (int v = 0; v < D; ++v) G[v] += gz * W0[mu * D + v];
            }
            U = u;
        }
#pragma unroll
        for (int v = 0; v < D; ++v) G[v] *= qs[v];
        if (MF ? !mine : false) continue;

        // adjoints: B_nlm = dU/dA_nlm, formed here from the sums in
        // registers, or, with the sums parked in the adjoint rows, by the
        // angular force kernel from them and the descriptor adjoints stored
        // here (no read-back of the parked sums)
        if constexpr (PARK) {
            const __amdgpu_buffer_rsrc_t go = adj_rows(a.Gad, gad_q(NA1, FOUR));
#pragma unroll
            for (int n = 0; n < NA1; ++n)
                adj_store(go, n, make_float4(G[NR1 + n], G[NR1 + NA1 + n], G[NR1 + 2 * NA1 + n], G[NR1 + 3 * NA1 + n]));
            if constexpr (FOUR) {
#pragma unroll
                for (int c4 = 0; c4 < (NA1 + 3) / 4; ++c4) {
                    float g4[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int n = 4 * c4 + e;
                        g4[e] = n < NA1 ? G[NR1 + kLmax * NA1 + (n < NA1 ? n : 0)] * a.kappa4 : 0.0f;
                    }
                    adj_store(go, NA1 + c4, make_float4(g4[0], g4[1], g4[2], g4[3]));
                }
            }
        } else {
#pragma unroll
            for (int n = 0; n < NA1; ++n) {
                const float Gl[kLmax] = {G[NR1 + n], G[NR1 + NA1 + n], G[NR1 + 2 * NA1 + n], G[NR1 + 3 * NA1 + n]};
                const float g4 = FOUR ? G[NR1 + kLmax * NA1 + n] * a.kappa4 : 0.0f;
                float Bn[kNumSH];
                form_adjoint<FOUR>(Ar[PARK ? 0 : n], Gl, g4, shc, Bn);
#pragma unroll
                for (int q4 = 0; q4 < kNumSH / 4; ++q4)
                    adj_store(Bo, n * (kNumSH / 4) + q4,
                              make_float4(Bn[4 * q4], Bn[4 * q4 + 1], Bn[4 * q4 + 2], Bn[4 * q4 + 3]));
            }
        }
        // radial adjoints a_k(t) = sum_n G_n c^{tc t}_nk, [atom][species][bead][12],
        // and in slot KR1 their sum over k >= 1 (the pair terms need it)
        static_assert(KR1 < kRadPad, "radial basis exceeds the padded adjoint row");
        for (int t = 0; t < S; ++t) {
            const float *c = prm + a.oR + (tc * S + t) * NR1 * KR1;
            float acc[kRadPad];
#pragma unroll
            for (int k = 0; k < kRadPad; ++k) {
                acc[k] = 0.0f;
                if (k < KR1) {
#pragma unroll
                    for (int n = 0; n < NR1; ++n) acc[k] += G[n] * c[n * KR1 + k];
                }
            }
#pragma unroll
            for (int k = 1; k < KR1; ++k) acc[KR1] += acc[k];
            float4 *ao = reinterpret_cast<float4 *>(a.arad + (((size_t)i * S + t) * P + b) * kRadPad);
#pragma unroll
            for (int q4 = 0; q4 < kRadPad / 4; ++q4)
                ao[q4] = make_float4(acc[4 * q4], acc[4 * q4 + 1], acc[4 * q4 + 2], acc[4 * q4 + 3]);
        }
    }

    if (valid && a.Eatom) a.Eatom[(size_t)b * a.N + i] = U;
    if (valid && !tok) atomicOr(a.flags, (uint32_t)NEP_FLAG_BAD_TYPE);
    __shared__ double lds[kBlock];
    // partials bead-major, [P][workgroups]: the reduction reads them contiguously
    bead_block_sum(valid ? (double)U : 0.0, lds, P, a.lg, a.partE + blockIdx.x, gridDim.x);
}

// ------------------------------------------------ pass 2: angular, own ---

// One lane per (atom i, bead): the angular pair terms d_ij = dU_i/dr_ij of
// the atom's own site energy, contracted with its own adjoints only:
//   d_ij = sum_n sum_lm B^i_nlm d/dr_ij [ g^{ij}_n(r) Y_lm(u) ],
// deposited where the partner j reads it back (its angular slot of i, same
// bead), and summed into the angular force part F_i += d_ij and the virial
// -r_ij (x) d_ij (the total needs no reverse terms).  B^i stays in
// registers for the whole neighbour walk; with more than five radial
// functions that takes the register file of one wavefront per SIMD
// (VGPRs and AGPRs): re-reading the row per neighbour instead streamed it
// from memory, the rows of a CU's wavefronts being larger than its caches.
// Control flow stays wave-uniform: lanes outside the current centre species,
// past their atom's last candidate or outside the cutoff compute on a dummy
// pair and contribute nothing; a candidate outside for every lane is
// skipped.
constexpr int kBatchAng = 4;   // angular entries whose loads are issued together
// Wavefronts per SIMD of k_force_ang.
template <int NA1> constexpr int kAngWaves() { return NA1 > 5 ? 1 : 2; }
constexpr int kBatchRev = 8;   // reverse angular terms read together by the radial force kernel

template <int NA1, int KA1, bool FOUR, bool PARKED, bool TRI>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kAngWaves<NA1>())))
void k_force_ang(NepArgs a, const float *__restrict__ prm)
{
    const LaneMap lm = lane_map(a);
    const int i = lm.i, b = lm.b, P = a.P, S = a.S;
    const bool valid = lm.valid;
    const int ii = i;
    const int ti = a.types[i];
    const bool tok = ti >= 0 && ti < S;
    const float4 *p4 = a.p4;
    const float4 pi = p4[(size_t)i * P + b];
    const float *shc = prm + a.osh;
    const int32_t *uA = a.uniA + (size_t)i * a.capA;
    const uint64_t *mA = a.umA + (size_t)i * a.capA;
    const int32_t *rowA = a.candA + (size_t)i * a.capA;
    const int32_t *rvA = a.revA + (size_t)i * a.capA;
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

        // B^i from the adjoint rows, or formed from the parked sums A^i and
        // the descriptor adjoints (see the descriptor kernel): their loads
        // are issued after the first neighbour batch's, so that the wait for
        // them overlaps that batch's gathers
        float Bi[NA1][kNumSH];
        bool formed = false;   // wave-uniform
        auto get_adjoints = [&]() {
            const __amdgpu_buffer_rsrc_t bi4 = adj_rows(a.B, NA1 * (kNumSH / 4));
#pragma unroll
            for (int n = 0; n < NA1; ++n)
#pragma unroll
                for (int q4 = 0; q4 < kNumSH / 4; ++q4) {
                    const float4 v4 = adj_load(bi4, n * (kNumSH / 4) + q4);
                    Bi[n][4 * q4] = v4.x; Bi[n][4 * q4 + 1] = v4.y;
                    Bi[n][4 * q4 + 2] = v4.z; Bi[n][4 * q4 + 3] = v4.w;
                }
            if constexpr (PARKED) {
                const __amdgpu_buffer_rsrc_t gi = adj_rows(a.Gad, gad_q(NA1, FOUR));
                const float *shc = prm + a.osh;
#pragma unroll
                for (int n = 0; n < NA1; ++n) {
                    const float4 gl = adj_load(gi, n);
                    const float Gl[kLmax] = {gl.x, gl.y, gl.z, gl.w};
                    float g4 = 0.0f;
                    if constexpr (FOUR) {
                        const float4 q = adj_load(gi, NA1 + n / 4);
                        g4 = (n & 3) == 0 ? q.x : (n & 3) == 1 ? q.y : (n & 3) == 2 ? q.z : q.w;
                    }
                    form_adjoint<FOUR>(Bi[n], Gl, g4, shc, Bi[n]);
                }
            }
            formed = true;
        };
        for (int t = 0; t < S; ++t) {
            int s0 = 0, s1 = 0;
            if (mine) block_range(a.uendA, i, t, s0, s1);
            const int cnt = s1 - s0;
            int cmax = cnt;
            for (int o = 32; o > 0; o >>= 1) cmax = max(cmax, __shfl_xor(cmax, o));
            cmax = __builtin_amdgcn_readfirstlane(cmax);
            const float *cij = prm + a.oA + (tc * S + t) * NA1 * KA1;
            for (int sb = 0; sb < cmax; sb += kBatchAng) {
                // the batch's slots, partners, positions and reverse slots,
                // each level's loads in flight together: every index is
                // clamped into the row (a lane with an empty block reads its
                // row's first entry) and its value selected after the load
                int kq[kBatchAng], jq[kBatchAng], rq[kBatchAng];
                bool aq[kBatchAng];
                float4 pq[kBatchAng];
#pragma unroll
                for (int u = 0; u < kBatchAng; ++u) {
                    const int su = min(s0 + max(min(sb + u, cnt - 1), 0), a.capA - 1);
                    const int k0 = uA[su];
                    const uint64_t mu = mA[su];
                    kq[u] = cnt > 0 ? k0 : 0;
                    aq[u] = (sb + u < cnt) & (((mu >> b) & 1u) != 0);
                }
#pragma unroll
                for (int u = 0; u < kBatchAng; ++u) {
                    const int r0 = rowA[kq[u]];
                    rq[u] = rvA[kq[u]];
                    jq[u] = cnt > 0 ? (r0 >> 2) : i;
                }
#pragma unroll
                for (int u = 0; u < kBatchAng; ++u) pq[u] = p4[(size_t)jq[u] * P + b];
                if (!formed) get_adjoints();
#pragma unroll
                for (int u = 0; u < kBatchAng; ++u) keep(pq[u]);
#pragma unroll
                for (int u = 0; u < kBatchAng; ++u) {
                const cf32p cij_l = launder(cij);
                const int j = jq[u];
                const bool act = aq[u];
                if (__ballot(act) == 0) continue;
                float dx, dy, dz;
                pair_vec<TRI>(pq[u], pi, lm, dx, dy, dz);
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
                    // g = f_c Pn / 2, g' = (dx/dr f_c Qn + f_c' Pn) / 2 with
                    // Pn = sum_k c_nk (T_k + 1), Qn = sum_k c_nk T_k'
                    float fc, fcp, dxdr, T[KA1], Tp[KA1];
                    cheb_td<KA1>(r, a.rcAinv, fc, fcp, dxdr, T, Tp);
                    const float hf = 0.5f * fc, hfp = 0.5f * fcp, hd = hf * dxdr;
#pragma unroll
                    for (int n = 0; n < NA1; ++n) {
                        float pn = 2.0f * cij_l[n * KA1], qn = 0.0f;
#pragma unroll
                        for (int q2 = 1; q2 < KA1; ++q2) {
                            pn = fmaf(cij_l[n * KA1 + q2], T[q2] + 1.0f, pn);
                            qn = fmaf(cij_l[n * KA1 + q2], Tp[q2], qn);
                        }
                        gij[n] = hf * pn;
                        gpij[n] = fmaf(hd, qn, hfp * pn);
                    }
                }
                float sY, gx, gy, gz;
                // B^i is stored as B_nlm c_m: bare polynomials here
                adjoint_contract<NA1>(ux, uy, uz, UnitNorm{}, Bi, gij, gpij, sY, gx, gy, gz);
                const float ug = ux * gx + uy * gy + uz * gz;
                const float px = sY * ux + (gx - ux * ug) * rinv;
                const float py = sY * uy + (gy - uy * ug) * rinv;
                const float pz = sY * uz + (gz - uz * ug) * rinv;
                if (act) {
                    const int rk = rq[u];
                    if (rk >= 0) a.pairbuf[((size_t)j * a.capA + rk) * P + b] = make_float4(px, py, pz, 0.0f);
                    Fx += px; Fy += py; Fz += pz;
                    Wv[0] = fmaf(-dx, px, Wv[0]); Wv[1] = fmaf(-dx, py, Wv[1]); Wv[2] = fmaf(-dx, pz, Wv[2]);
                    Wv[3] = fmaf(-dy, px, Wv[3]); Wv[4] = fmaf(-dy, py, Wv[4]); Wv[5] = fmaf(-dy, pz, Wv[5]);
                    Wv[6] = fmaf(-dz, px, Wv[6]); Wv[7] = fmaf(-dz, py, Wv[7]); Wv[8] = fmaf(-dz, pz, Wv[8]);
                }
                }
            }
        }
    }

    if (valid) {
        float *Fo = a.Fang + ((size_t)i * P + b) * 3;
        Fo[0] = Fx;
        Fo[1] = Fy;
        Fo[2] = Fz;
        if (a.Watom) {
            // own half of the per-atom split; the reverse half is added by the radial pass
            float *wo = a.Watom + ((size_t)b * a.N + i) * 9;
#pragma unroll
            for (int e = 0; e < 9; ++e) wo[e] = 0.5f * Wv[e];
        }
    }
    __shared__ double lds[kBlock];
    for (int e = 0; e < 9; ++e)
        bead_block_sum(valid ? (double)Wv[e] : 0.0, lds, P, a.lg, a.partWa + (size_t)e * gridDim.x + blockIdx.x,
                       9 * gridDim.x);
}

// ----------------------------------------- pass 3: radial + combination ---

// One lane per (atom i, bead): radial pair terms (a^i_k(tj) + a^j_k(ti))
// f'_k(r) u (both site energies at once, the partner's adjoints gathered
// bead-minor), then the reverse angular terms -dU_j/dr_ji that the angular
// pass deposited at this atom's slots, then the angular own part.  Force and
// per-atom virial sums are kept in FP64.
template <int KR1, bool TRI>
__global__ __launch_bounds__(kBlock) void k_force_rad(NepArgs a)
{
    const LaneMap lm = lane_map(a);
    const int i = lm.i, b = lm.b, P = a.P, S = a.S;
    const bool valid = lm.valid;
    const int ti = a.types[i];
    const bool tok = ti >= 0 && ti < S;
    const float4 *p4 = a.p4;
    const float4 pi = p4[(size_t)i * P + b];
    double Fx = 0.0, Fy = 0.0, Fz = 0.0;
    float Wf[9];   // radial pair virial of this (atom, bead), FP32 (a sum of like-signed terms)
#pragma unroll
    for (int e = 0; e < 9; ++e) Wf[e] = 0.0f;
    float Wa[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) Wa[e] = 0.0f;
    if (valid && tok) {
        auto load_a = [&](int atom, int sp, float *out) {
            const float4 *p = reinterpret_cast<const float4 *>(a.arad + (((size_t)atom * S + sp) * P + b) * kRadPad);
#pragma unroll
            for (int q4 = 0; q4 < kRadPad / 4; ++q4) {
                const float4 v = p[q4];
                if (4 * q4 <= KR1) out[4 * q4] = v.x;
                if (4 * q4 + 1 <= KR1) out[4 * q4 + 1] = v.y;
                if (4 * q4 + 2 <= KR1) out[4 * q4 + 2] = v.z;
                if (4 * q4 + 3 <= KR1) out[4 * q4 + 3] = v.w;
            }
        };
        const int32_t *uR = a.uniR + (size_t)i * a.capR;
        const uint64_t *mR = a.umR + (size_t)i * a.capR;
        for (int t = 0; t < S; ++t) {
            int s0, s1;
            block_range(a.uendR, i, t, s0, s1);
            float ai[KR1 + 1];   // a_k and, last, their sum over k >= 1
            load_a(i, t, ai);
            for (int sb = s0; sb < s1; sb += kBatch) {
                int jj[kBatch];
                bool in[kBatch];
                float4 pj[kBatch];
                float aj[kBatch][KR1 + 1];
                // unconditional loads, as in the descriptor's radial batches
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int su = min(sb + u, s1 - 1);
                    jj[u] = uR[su];
                    const uint64_t mu = mR[su];
                    in[u] = (sb + u < s1) & (((mu >> b) & 1u) != 0);
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    pj[u] = p4[(size_t)jj[u] * P + b];
                    load_a(jj[u], ti, aj[u]);
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) keep(pj[u]);
                float bx = 0.0f, by = 0.0f, bz = 0.0f;   // the batch's force, FP32, into the FP64 sum once
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    if (in[u]) {
                        float dx, dy, dz;
                        pair_vec<TRI>(pj[u], pi, lm, dx, dy, dz);
                        const float r2 = dx * dx + dy * dy + dz * dz;
                        const float rinv = __builtin_amdgcn_rsqf(r2);
                        const float r = r2 * rinv;
                        // sum_k A_k f_k' = (dx/dr f_c sum A_k T_k' + f_c' sum A_k (T_k + 1)) / 2,
                        // sum_{k>0} A_k (T_k + 1) = sum_{k>0} A_k T_k + (the stored sums of a_k)
                        float fc, fcp, dxdr, T[KR1], Tp[KR1];
                        cheb_td<KR1>(r, a.rcRinv, fc, fcp, dxdr, T, Tp);
                        float s1 = 2.0f * (ai[0] + aj[u][0]) + (ai[KR1] + aj[u][KR1]), s2 = 0.0f;
#pragma unroll
                        for (int q2 = 1; q2 < KR1; ++q2) {
                            const float A = ai[q2] + aj[u][q2];
                            s1 = fmaf(A, T[q2], s1);
                            s2 = fmaf(A, Tp[q2], s2);
                        }
                        const float sc = 0.5f * fmaf(dxdr * fc, s2, fcp * s1);
                        const float w = sc * rinv;
                        const float qx = w * dx, qy = w * dy, qz = w * dz;
                        bx += qx; by += qy; bz += qz;
                        const float hx = -0.5f * dx, hy = -0.5f * dy, hz = -0.5f * dz;
                        // a central pair term: r (x) q is symmetric, six entries
                        Wf[0] = fmaf(hx, qx, Wf[0]); Wf[1] = fmaf(hx, qy, Wf[1]); Wf[2] = fmaf(hx, qz, Wf[2]);
                        Wf[4] = fmaf(hy, qy, Wf[4]); Wf[5] = fmaf(hy, qz, Wf[5]); Wf[8] = fmaf(hz, qz, Wf[8]);
                    }
                }
                Fx += (double)bx; Fy += (double)by; Fz += (double)bz;
            }
        }

        Wf[3] = Wf[1];
        Wf[6] = Wf[2];
        Wf[7] = Wf[5];

        // reverse angular terms: F_i -= dU_j/dr_ji for every angular neighbour j
        const int32_t *uA = a.uniA + (size_t)i * a.capA;
        const uint64_t *mA = a.umA + (size_t)i * a.capA;
        const int32_t *rowA = a.candA + (size_t)i * a.capA;
        const float4 *pbuf = a.pairbuf + (size_t)i * a.capA * P + b;
        const int nA = a.uendA[(size_t)i * kMaxSpecies + S - 1];
        float gx = 0.0f, gy = 0.0f, gz = 0.0f;
        for (int sb = 0; sb < nA; sb += kBatchRev) {
            int kk[kBatchRev];
            bool in[kBatchRev];
            float4 d[kBatchRev];
            // unconditional loads (slots past the list end reread its last
            // entry; values outside the bead mask are dropped)
#pragma unroll
            for (int u = 0; u < kBatchRev; ++u) {
                const int su = min(sb + u, nA - 1);
                kk[u] = uA[su];
                const uint64_t mu = mA[su];
                in[u] = (sb + u < nA) & (((mu >> b) & 1u) != 0);
            }
#pragma unroll
            for (int u = 0; u < kBatchRev; ++u) d[u] = pbuf[(size_t)kk[u] * P];
#pragma unroll
            for (int u = 0; u < kBatchRev; ++u) {
                keep(d[u]);
                if (!in[u]) d[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
#pragma unroll
            for (int u = 0; u < kBatchRev; ++u) {
                gx -= d[u].x; gy -= d[u].y; gz -= d[u].z;
            }
            if (a.Watom) {
#pragma unroll
                for (int u = 0; u < kBatchRev; ++u) {
                    if (!in[u]) continue;
                    float dx, dy, dz;
                    pair_vec<TRI>(p4[(size_t)(rowA[kk[u]] >> 2) * P + b], pi, lm, dx, dy, dz);
                    const float4 dd = d[u];
                    // reverse half of the per-atom split: +1/2 r_ij (x) dU_j/dr_ji
                    const float hx = 0.5f * dx, hy = 0.5f * dy, hz = 0.5f * dz;
                    Wa[0] = fmaf(hx, dd.x, Wa[0]); Wa[1] = fmaf(hx, dd.y, Wa[1]); Wa[2] = fmaf(hx, dd.z, Wa[2]);
                    Wa[3] = fmaf(hy, dd.x, Wa[3]); Wa[4] = fmaf(hy, dd.y, Wa[4]); Wa[5] = fmaf(hy, dd.z, Wa[5]);
                    Wa[6] = fmaf(hz, dd.x, Wa[6]); Wa[7] = fmaf(hz, dd.y, Wa[7]); Wa[8] = fmaf(hz, dd.z, Wa[8]);
                }
            }
        }
        Fx += (double)gx;
        Fy += (double)gy;
        Fz += (double)gz;
    }
    if (valid) {
        const float *fa = a.Fang + ((size_t)i * P + b) * 3;
        const double gx = Fx + (double)fa[0], gy = Fy + (double)fa[1], gz = Fz + (double)fa[2];
        float *Fo = a.F + ((size_t)b * a.N + i) * 3;
        Fo[0] = (float)gx;
        Fo[1] = (float)gy;
        Fo[2] = (float)gz;
        if (a.Watom) {
            float *wo = a.Watom + ((size_t)b * a.N + i) * 9;
#pragma unroll
            for (int e = 0; e < 9; ++e) wo[e] = (float)((double)Wf[e] + (double)Wa[e] + (double)wo[e]);
        }
        if (!(isfinite(gx) && isfinite(gy) && isfinite(gz))) atomicOr(a.flags, (uint32_t)NEP_FLAG_NONFINITE);
    }
    __shared__ double lds[kBlock];
    for (int e = 0; e < 9; ++e)
        bead_block_sum(valid ? (double)Wf[e] : 0.0, lds, P, a.lg, a.partWr + (size_t)e * gridDim.x + blockIdx.x,
                       9 * gridDim.x);
}

// Per-(system, bead) energy and virial from the per-workgroup partial sums
// of the system's tiles, stored [P][nblk] (energy) and [P][9][nblk] (virial
// parts): one wavefront per (system, bead, component), in the fixed order of
// reduce_output.
__global__ __launch_bounds__(64) void k_reduce(PendingReduce r)
{
    reduce_output(r, blockIdx.x, threadIdx.x);
}

constexpr size_t kNetLdsMax = 60 * 1024;   // bytes of LDS for the staged network weights

// mlp: NEP_MLP_FP32 (vector units), NEP_MLP_BF16_MFMA or NEP_MLP_FP32_MFMA (matrix cores).
template <int NR1, int NA1, bool FOUR, bool TRI>
static void launch_t(const NepArgs &a, const float *prm, int nblk, int wpb, int mlp, bool lds_net, hipStream_t s)
{
    const dim3 g(nblk);
    const dim3 blk(64 * wpb);
    {
        ProfScope ps_(K_DESCRIPTOR, s);
        constexpr int D = Dims<NR1, NA1, FOUR>::D, DP = (D + 3) & ~3;
        const size_t net = sizeof(float) * (size_t)a.S * a.H * (DP + 2);
        const size_t mf = sizeof(float) * (size_t)mf_lds_floats<D>() * wpb;
        if (mlp == NEP_MLP_BF16_MFMA)   // BF16 weights (the student)
            hipLaunchKernelGGL((k_descriptor<NR1, NA1, 9, 9, FOUR, kNetBf16, TRI>), g, blk, mf, s, a, prm);
        else if (mlp == NEP_MLP_FP32_MFMA)   // FP32 weights as three BF16 terms
            hipLaunchKernelGGL((k_descriptor<NR1, NA1, 9, 9, FOUR, kNetMf32, TRI>), g, blk, mf, s, a, prm);
        else if (lds_net && net <= kNetLdsMax)   // network weights staged in LDS
            hipLaunchKernelGGL((k_descriptor<NR1, NA1, 9, 9, FOUR, kNetLds, TRI>), g, blk, net, s, a, prm);
        else
            hipLaunchKernelGGL((k_descriptor<NR1, NA1, 9, 9, FOUR, kNetGlobal, TRI>), g, blk, 0, s, a, prm);
    }
    {
        ProfScope ps_(K_FORCE_ANG, s);
        if (adj_parked(mlp == NEP_MLP_BF16_MFMA || mlp == NEP_MLP_FP32_MFMA, NA1))
            hipLaunchKernelGGL((k_force_ang<NA1, 9, FOUR, true, TRI>), g, blk, 0, s, a, prm);
        else
            hipLaunchKernelGGL((k_force_ang<NA1, 9, FOUR, false, TRI>), g, blk, 0, s, a, prm);
    }
    {
        ProfScope ps_(K_FORCE, s);
        hipLaunchKernelGGL((k_force_rad<9, TRI>), g, blk, 0, s, a);
    }
}

// General (triclinic) cells get the kernels with the general pair vector;
// orthorhombic-only lists the ones without it.
template <int NR1, int NA1, bool FOUR>
static void launch(const NepArgs &a, const float *prm, int nblk, int wpb, bool tri, int mlp, bool lds_net,
                   hipStream_t s)
{
    if (tri) launch_t<NR1, NA1, FOUR, true>(a, prm, nblk, wpb, mlp, lds_net, s);
    else launch_t<NR1, NA1, FOUR, false>(a, prm, nblk, wpb, mlp, lds_net, s);
}

}  // namespace nep

using namespace nep;

extern "C" int32_t nep_compute_batched(const nep_model *m, nep_nlist *nl, nep_ws *ws, const double *pos,
                                       const double *boxes, const int32_t *types, int32_t P, int32_t N, double *E,
                                       float *F, double *W, float *E_atom, float *W_atom, hipStream_t s)
{
    if (!m || !nl || !ws || !boxes) return fail(NEP_ERR_INVALID_ARG, "nep_compute: null argument");
    if (m->cutoffs_only) return fail(NEP_ERR_INVALID_ARG, "nep_compute: a list cutoff descriptor has no network");
    if (nl->P != P || nl->N != N || ws->P != P || ws->N != N || nl->S != m->hp.n_species || ws->S != m->hp.n_species ||
        ws->NA1 != m->hp.n_max_angular + 1 || nl->off != ws->off)
        return fail(NEP_ERR_INVALID_ARG, "nep_compute: P=%d N=%d do not match the list/workspace handles", P, N);
    // a deferral applies to this call only; a new call drops sums left pending
    const bool defer = ws->defer_next != 0;
    ws->defer_next = 0;
    ws->pending = PendingReduce{};
    if (P == 0) return NEP_OK;
    if (!E || !W) return fail(NEP_ERR_INVALID_ARG, "nep_compute: null E or W");
    const int nsys = nl->nsys;
    if (N == 0) {
        fill_u32(reinterpret_cast<uint32_t *>(E), 0u, (size_t)nsys * P * 2, s);
        fill_u32(reinterpret_cast<uint32_t *>(W), 0u, (size_t)nsys * P * 18, s);
        NEP_HIP(hipGetLastError());
        return NEP_OK;
    }
    if (!pos || !types || !F) return fail(NEP_ERR_INVALID_ARG, "nep_compute: null array");
    if (!nl->built) return fail(NEP_ERR_INVALID_ARG, "nep_compute: the neighbour lists were never built");
    if (nl->rc_built[0] != m->hp.rc_radial || nl->rc_built[1] != m->hp.rc_angular)
        return fail(NEP_ERR_INVALID_ARG, "nep_compute: the lists were built for cutoffs %g/%g, the model has %g/%g",
                    nl->rc_built[0], nl->rc_built[1], m->hp.rc_radial, m->hp.rc_angular);
    for (int sy = 0; sy < nsys; ++sy)
        for (int k = 0; k < 9; ++k)
            if (boxes[9 * sy + k] != nl->boxL[9 * sy + k])
                return fail(NEP_ERR_INVALID_ARG, "nep_compute: box of system %d differs from the last neighbor_build",
                            sy);
    const nep_hparams &h = m->hp;
    NepArgs a{};
    // packed positions of the last neighbor_build (the same positions, see the header)
    a.p4 = reinterpret_cast<const float4 *>(nl->pos4); a.pos = pos; a.types = types; a.N = N; a.S = h.n_species;
    a.H = h.hidden; a.P = P; a.lg = lanes_log2(P);
    a.geom = nl->geom; a.tile_atom0 = ws->tile_atom0; a.tile_atom1 = ws->tile_atom1; a.tile_sys = ws->tile_sys;
    a.rcRinv = (float)(1.0 / h.rc_radial); a.rcAinv = (float)(1.0 / h.rc_angular);
    a.kappa4 = (float)(-4.5 * std::sqrt(2.0 / 35.0) * std::pow(5.0 / (4.0 * M_PI), 1.5));
    a.candA = nl->candA; a.revA = nl->revA; a.uniR = nl->uniR; a.uendR = nl->uendR; a.uniA = nl->uniA;
    a.umR = nl->umR; a.umA = nl->umA;
    a.uendA = nl->uendA; a.capR = nl->capR; a.capA = nl->capA;
    a.pairbuf = reinterpret_cast<float4 *>(nl->pairbuf);
    a.B = ws->B; a.Gad = ws->Gad; a.arad = ws->arad; a.Fang = ws->Fang;
    a.partE = ws->partE; a.partWa = ws->partW; a.partWr = ws->partW + (size_t)P * ws->nblk * 9;
    a.flags = ws->flags;
    a.F = F; a.Eatom = E_atom; a.Watom = W_atom;
    a.oR = m->off.cR; a.oA = m->off.cA; a.oq = m->off.qs; a.oW0 = m->off.W0; a.ob0 = m->off.b0;
    a.ow1 = m->off.w1; a.ob1 = m->off.b1; a.osh = m->off.sh;
    a.w0b = m->w0b;
    const int mlp = m->mlp;
    const int key = h.n_max_radial * 100 + h.n_max_angular * 10 + h.four_body;
    const bool tri = nl->any_tri != 0;
    switch (key) {
    case 440: launch<5, 5, false>(a, m->dev, ws->nblk, ws->wpb, tri, mlp, !ws->net_global, s); break;
    case 441: launch<5, 5, true>(a, m->dev, ws->nblk, ws->wpb, tri, mlp, !ws->net_global, s); break;
    case 640: launch<7, 5, false>(a, m->dev, ws->nblk, ws->wpb, tri, mlp, !ws->net_global, s); break;
    case 860: launch<9, 7, false>(a, m->dev, ws->nblk, ws->wpb, tri, mlp, !ws->net_global, s); break;
    case 881: launch<9, 9, true>(a, m->dev, ws->nblk, ws->wpb, tri, mlp, !ws->net_global, s); break;
    default: return fail(NEP_ERR_UNSUPPORTED, "nep_compute: unsupported model shape");
    }
    PendingReduce r;
    r.partE = ws->partE; r.partWa = a.partWa; r.partWr = a.partWr; r.sys_tile0 = ws->sys_tile0;
    r.P = P; r.nblk = ws->nblk; r.nout = nsys * P * 10; r.E = E; r.W = W;
    if (defer) {   // completed by the next integrator launch (trpmd_step_nep)
        ws->pending = r;
    } else {
        ProfScope ps_(K_REDUCE, s);
        hipLaunchKernelGGL(k_reduce, dim3(r.nout), dim3(64), 0, s, r);
    }
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}

extern "C" int32_t nep_compute(const nep_model *m, nep_nlist *nl, nep_ws *ws, const double *pos,
                               const double box[9], const int32_t *types, int32_t P, int32_t N, double *E, float *F,
                               double *W, float *E_atom, float *W_atom, hipStream_t s)
{
    if (nl && nl->nsys != 1) return fail(NEP_ERR_INVALID_ARG, "nep_compute: the list holds a batch of systems");
    return nep_compute_batched(m, nl, ws, pos, box, types, P, N, E, F, W, E_atom, W_atom, s);
}

extern "C" int32_t nep_ws_defer_reduce(nep_ws *ws)
{
    if (!ws) return fail(NEP_ERR_INVALID_ARG, "nep_ws_defer_reduce: null workspace");
    ws->defer_next = 1;
    return NEP_OK;
}

extern "C" int32_t nep_autotune(const nep_model *m, nep_nlist *nl, nep_ws *ws, const double *pos, const double *boxes,
                                const int32_t *types, int32_t P, int32_t N, double *E, float *F, double *W,
                                int32_t reps, float *ms_out, int32_t *best_out, hipStream_t s)
{
    if (!m || !nl || !ws) return fail(NEP_ERR_INVALID_ARG, "nep_autotune: null argument");
    if (reps < 1 || reps > 100) return fail(NEP_ERR_INVALID_ARG, "nep_autotune: reps must be in 1..100");
    const int choices[3] = {1, 2, 4};
    // the staging knob exists for the vector-unit network whose weights fit LDS
    const nep_hparams &h = m->hp;
    const size_t net = sizeof(float) * (size_t)h.n_species * h.hidden * (((h.dim + 3) & ~3) + 2);
    const int nst = (m->mlp == NEP_MLP_FP32 && net <= kNetLdsMax) ? 2 : 1;
    float best_ms = 0.0f;
    int best = 4, best_st = NEP_WEIGHTS_LDS;
    if (ms_out)
        for (int k = 0; k < 6; ++k) ms_out[k] = -1.0f;
    hipEvent_t e0, e1;
    NEP_HIP(hipEventCreate(&e0));
    NEP_HIP(hipEventCreate(&e1));
    int32_t rc = NEP_OK;
    bool first = true;
    for (int c = 0; c < 3 && rc == NEP_OK; ++c)
        for (int st = 0; st < nst && rc == NEP_OK; ++st) {
            rc = nep_ws_set_tile(ws, choices[c]);
            if (rc == NEP_OK) rc = nep_ws_set_weight_staging(ws, st);
            if (rc != NEP_OK) break;
            rc = nep_compute_batched(m, nl, ws, pos, boxes, types, P, N, E, F, W, nullptr, nullptr, s);   // warm-up
            if (rc != NEP_OK) break;
            if (hipEventRecord(e0, s) != hipSuccess) rc = fail(NEP_ERR_HIP, "nep_autotune: event record failed");
            for (int r = 0; r < reps && rc == NEP_OK; ++r)
                rc = nep_compute_batched(m, nl, ws, pos, boxes, types, P, N, E, F, W, nullptr, nullptr, s);
            if (rc != NEP_OK) break;
            float ms = 0.0f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = fail(NEP_ERR_HIP, "nep_autotune: event timing failed");
                break;
            }
            ms /= (float)reps;
            if (ms_out) ms_out[2 * c + st] = ms;
            if (first || ms < best_ms) {
                best_ms = ms;
                best = choices[c];
                best_st = st;
                first = false;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != NEP_OK) return rc;
    if (best_out) {
        best_out[0] = best;
        best_out[1] = best_st;
    }
    rc = nep_ws_set_weight_staging(ws, best_st);
    return rc != NEP_OK ? rc : nep_ws_set_tile(ws, best);
}
