// Training of a NEP model on GPU: gradient of an energy / force / virial
// loss with respect to the network parameters (W0, b0, w1, b1) and the radial
// and angular descriptor coefficients c^R, c^A, and an Adam update (Kingma
// and Ba, ICLR 2015).
// The NEP site-energy model is that of Sec. II.C of arXiv:2409.04430; the
// paper fits its models by SNES, this library by gradients.
//
// For the P configurations of each system of one call (the beads of a
// neighbour handle, each with reference E, F, W; a batch of systems is a
// batch of independent snapshots) the loss is, summed over the systems,
//   L = sum_b [ lE (dE_b / N)^2 + lF sum_i |dF_bi|^2 / (3 N) + lW sum_ab (dW_b,ab / N)^2 ]
// with N the system's atom count.
// Force and virial terms are derivatives of E, so their parameter gradient
// is a mixed derivative.  With g_ij = dU_i/dr_ij and a per-pair field
//   d_ij = -(2 lF / 3N) (dF_j - dF_i) - (2 lW / N^2) dW_b^T r_ij
// one has dL_{F,W}/dtheta = d/dtheta sum_ij g_ij . d_ij  (d held fixed), and
// sum_ij g_ij . d_ij = sum_i G_i . qdot_i, G = dU/dq, qdot the derivative of
// the descriptor along d (a forward-mode pass).  The kernels therefore
// compute per (atom, bead): q, qdot, the network values and their forward
// derivatives, and write one row of factors; a reduction kernel forms the
// outer products that make up the gradient.
#include "internal.hpp"
#include "nep_kernels.hpp"

namespace nep {

struct TrainArgs {
    const float4 *dF;   // [N][P] scaled force residuals -2 lF/(3N) (F - F_ref), bead-minor
    const float *cW;    // [nsys][P][9] -2 lW/N^2 (W - W_ref)
    const float *eE;    // [nsys][P] 2 lE/N^2 (E - E_ref)
    float *rows;        // [N*P][RW] factor rows, row i * P + b
    int RW;
    float *xb;          // [N*P][2][NA1][24] scratch: X and B of the angular-coefficient pass
};

// Row layout (floats): type | u[H] | v[H] | gw1[H] | sq[D] | sqd[D] | gR[NR1] | GR[NR1] | sk[S][KR1] |
// skd[S][KR1] | eE | gA[S][NA1][KA1].
struct RowLayout {
    int u, v, gw1, sq, sqd, gR, GR, sk, skd, eE, gA, RW;
    __host__ __device__ RowLayout(int H, int D, int NR1, int S, int KR1, int NA1, int KA1)
    {
        u = 1; v = u + H; gw1 = v + H; sq = gw1 + H; sqd = sq + D; gR = sqd + D; GR = gR + NR1; sk = GR + NR1;
        skd = sk + S * KR1; eE = skd + S * KR1; gA = eE + 1; RW = gA + S * NA1 * KA1;
    }
};

// Residuals: scaled force residuals per (atom, bead) and per-(system, bead)
// energy and virial factors; loss parts accumulated into loss[1..3]
// (diagnostic).  atom_sys [N] and sys_off [nsys+1] give each atom's system
// and the systems' atom counts.
__global__ void k_residual(const float *__restrict__ F, const float *__restrict__ Fref, const double *__restrict__ E,
                           const double *__restrict__ Eref, const double *__restrict__ W,
                           const double *__restrict__ Wref, int P, int N, int nsys,
                           const int32_t *__restrict__ atom_sys, const int32_t *__restrict__ sys_off, double lE,
                           double lF, double lW, float4 *__restrict__ dF, float *__restrict__ cW,
                           float *__restrict__ eE, double *__restrict__ loss)
{
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double lf = 0.0;
    if (e < (size_t)P * N) {
        const int b = (int)(e / (size_t)N), i = (int)(e - (size_t)b * N);
        const int sy = atom_sys[i];
        const double Ns = (double)(sys_off[sy + 1] - sys_off[sy]);
        const double dx = (double)F[3 * e] - Fref[3 * e], dy = (double)F[3 * e + 1] - Fref[3 * e + 1],
                     dz = (double)F[3 * e + 2] - Fref[3 * e + 2];
        lf = lF * (dx * dx + dy * dy + dz * dz) / (3.0 * Ns);
        const double cf = -2.0 * lF / (3.0 * Ns);
        dF[(size_t)i * P + b] = make_float4((float)(cf * dx), (float)(cf * dy), (float)(cf * dz), 0.0f);
    }
    // one pair of atomics per workgroup (same-address atomics serialise)
    __shared__ double red[4];
    for (int o = 32; o > 0; o >>= 1) lf += __shfl_xor(lf, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lf;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) lf += red[w];
        if (lf != 0.0) {
            atomicAdd(&loss[2], lf);
            atomicAdd(&loss[0], lf);
        }
    }
    if (blockIdx.x == 0)
        for (int x = threadIdx.x; x < nsys * P; x += blockDim.x) {
            const int sy = x / P;
            const double Ns = (double)(sys_off[sy + 1] - sys_off[sy]);
            if (!(Ns > 0.0)) {
                eE[x] = 0.0f;
                for (int k = 0; k < 9; ++k) cW[9 * x + k] = 0.0f;
                continue;
            }
            const double de = E[x] - Eref[x];
            eE[x] = (float)(2.0 * lE * de / (Ns * Ns));
            atomicAdd(&loss[1], lE * (de / Ns) * (de / Ns));
            atomicAdd(&loss[0], lE * (de / Ns) * (de / Ns));
            double lw = 0.0;
            for (int k = 0; k < 9; ++k) {
                const double dw = W[9 * x + k] - Wref[9 * x + k];
                cW[9 * x + k] = (float)(-2.0 * lW * dw / (Ns * Ns));
                lw += lW * (dw / Ns) * (dw / Ns);
            }
            atomicAdd(&loss[3], lw);
            atomicAdd(&loss[0], lw);
        }
}

// Descriptor, its derivative along the pair field d, and the network with
// its forward derivative; writes the factor row of (atom, bead).
//
// Angular coefficients: with T_klm = sum_j f_k(r_ij) Y_lm(u_ij) (per
// neighbour species), A_nlm = sum_k c_nk T_klm and q_nl = sum_m A_nlm^2, the
// row's share of dL/dc_nk is sum_lm [X_nlm T_klm + B_nlm Tdot_klm] with
// B = 2 G_nl A_nlm (the energy adjoint), X = eE B + Bdot and Bdot = 2 (Gdot_nl
// A_nlm + G_nl Adot_nlm).  B and X are parked in the row's scratch, then a
// second pass over the angular neighbours (one n at a time) accumulates
// f_k (X.Y + B.Ydot) + fdot_k (u.d) (B.Y) into the row.
constexpr int kJvpGroup = 2;   // angular radial functions accumulated per neighbour pass
template <int NR1, int NA1, int KR1, int KA1>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
void k_train_jvp(NepArgs a, TrainArgs ta, const float *__restrict__ prm)
{
    constexpr int D = Dims<NR1, NA1, false>::D;
    const LaneMap lm = lane_map(a);
    const int i = lm.i, b = lm.b, P = a.P, S = a.S, H = a.H;
    const bool valid = lm.valid;
    const int ti = a.types[i];
    const bool tok = ti >= 0 && ti < S;
    const float4 *p4 = a.p4;
    const float4 pi = p4[(size_t)i * P + b];
    const float4 di = ta.dF[(size_t)i * P + b];
    const int sb = a.tile_sys[blockIdx.x] * P + b;   // (system, bead) of the lane
    float cw[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) cw[e] = ta.cW[9 * sb + e];
    const float *shc = prm + a.osh;
    const RowLayout R(H, D, NR1, S, KR1, NA1, KA1);
    float *row = ta.rows + ((size_t)i * P + b) * ta.RW;
    float *xb = ta.xb + ((size_t)i * P + b) * (2 * NA1 * kNumSH);

    uint64_t todo = __ballot(valid && tok);
    while (todo) {
        const int lead = __builtin_ctzll(todo);
        const int tc = __builtin_amdgcn_readlane(ti, lead);
        const bool mine = valid && tok && ti == tc;
        todo &= ~__ballot(mine);
        if (!mine) continue;

        // pair field along r_ij: d = (dF_j - dF_i) + cW^T r_ij
        auto field = [&](const float4 &dj, float dx, float dy, float dz, float &ex, float &ey, float &ez) {
            ex = dj.x - di.x + cw[0] * dx + cw[3] * dy + cw[6] * dz;
            ey = dj.y - di.y + cw[1] * dx + cw[4] * dy + cw[7] * dz;
            ez = dj.z - di.z + cw[2] * dx + cw[5] * dy + cw[8] * dz;
        };

        // descriptors q and their derivatives along d go to the row, scaled,
        // as soon as each is final (row[R.sq + v], row[R.sqd + v])
        const float *qs = prm + a.oq;
        float qr[NR1], qrd[NR1];
#pragma unroll
        for (int n = 0; n < NR1; ++n) {
            qr[n] = 0.0f;
            qrd[n] = 0.0f;
        }
        // radial: per neighbour species, the basis sums and their derivatives
        // along d (written to the row at once), contracted with c
        const int32_t *uR = a.uniR + (size_t)i * a.capR;
        const uint64_t *mR = a.umR + (size_t)i * a.capR;
        for (int t = 0; t < S; ++t) {
            int s0, s1;
            block_range(a.uendR, i, t, s0, s1);
            float sk[KR1], skd[KR1];
#pragma unroll
            for (int k = 0; k < KR1; ++k) {
                sk[k] = 0.0f;
                skd[k] = 0.0f;
            }
            for (int s = s0; s < s1; ++s) {
                if (!((mR[s] >> b) & 1u)) continue;
                const int j = uR[s];
                float dx, dy, dz;
                pair_vec<true>(p4[(size_t)j * P + b], pi, lm, dx, dy, dz);
                const float r2 = dx * dx + dy * dy + dz * dz;
                const float rinv = __builtin_amdgcn_rsqf(r2);
                const float r = r2 * rinv;
                float ex, ey, ez;
                field(ta.dF[(size_t)j * P + b], dx, dy, dz, ex, ey, ez);
                const float rdot = (dx * ex + dy * ey + dz * ez) * rinv;
                float f[KR1], fp[KR1];
                cheb_fd<KR1>(r, a.rcRinv, f, fp);
#pragma unroll
                for (int k = 0; k < KR1; ++k) {
                    sk[k] += f[k];
                    skd[k] = fmaf(fp[k], rdot, skd[k]);
                }
            }
            const float *c = prm + a.oR + (tc * S + t) * NR1 * KR1;
#pragma unroll
            for (int n = 0; n < NR1; ++n) {
                float acc = qr[n], accd = qrd[n];
#pragma unroll
                for (int k = 0; k < KR1; ++k) {
                    acc = fmaf(c[n * KR1 + k], sk[k], acc);
                    accd = fmaf(c[n * KR1 + k], skd[k], accd);
                }
                qr[n] = acc;
                qrd[n] = accd;
            }
#pragma unroll
            for (int k = 0; k < KR1; ++k) {
                row[R.sk + t * KR1 + k] = sk[k];
                row[R.skd + t * KR1 + k] = skd[k];
            }
        }
#pragma unroll
        for (int n = 0; n < NR1; ++n) {
            row[R.sq + n] = qs[n] * qr[n];
            row[R.sqd + n] = qs[n] * qrd[n];
        }
        // angular: A_nlm and its derivative along d, kJvpGroup radial
        // functions n per pass over the neighbours (their accumulators in
        // registers), each group's q, qdot entries formed and its A, Adot
        // parked (replaced by X and B once the network adjoints are known)
        const int32_t *uA = a.uniA + (size_t)i * a.capA;
        const uint64_t *mA = a.umA + (size_t)i * a.capA;
        const int32_t *rowA = a.candA + (size_t)i * a.capA;
#pragma unroll
        for (int n0 = 0; n0 < NA1; n0 += kJvpGroup) {
            float A[kJvpGroup][kNumSH], Ad[kJvpGroup][kNumSH];
#pragma unroll
            for (int g = 0; g < kJvpGroup; ++g)
#pragma unroll
                for (int m = 0; m < kNumSH; ++m) {
                    A[g][m] = 0.0f;
                    Ad[g][m] = 0.0f;
                }
            for (int t = 0; t < S; ++t) {
                int s0, s1;
                block_range(a.uendA, i, t, s0, s1);
                const float *c = prm + a.oA + (tc * S + t) * NA1 * KA1;
                for (int s = s0; s < s1; ++s) {
                    if (!((mA[s] >> b) & 1u)) continue;
                    const int j = rowA[uA[s]] >> 2;
                    float dx, dy, dz;
                    pair_vec<true>(p4[(size_t)j * P + b], pi, lm, dx, dy, dz);
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    const float rinv = __builtin_amdgcn_rsqf(r2);
                    const float r = r2 * rinv;
                    const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
                    float ex, ey, ez;
                    field(ta.dF[(size_t)j * P + b], dx, dy, dz, ex, ey, ez);
                    const float rdot = ux * ex + uy * ey + uz * ez;
                    // du/de = (d - u (u . d)) / r
                    const float vx = (ex - ux * rdot) * rinv, vy = (ey - uy * rdot) * rinv,
                                vz = (ez - uz * rdot) * rinv;
                    float f[KA1], fp[KA1];
                    cheb_fd<KA1>(r, a.rcAinv, f, fp);
                    float Y[kNumSH], Dm[kNumSH];
                    sh_eval(ux, uy, uz, shc, Y);
                    sh_dir(ux, uy, uz, vx, vy, vz, shc, Dm);
#pragma unroll
                    for (int g = 0; g < kJvpGroup; ++g) {
                        const int n = n0 + g;
                        if (n >= NA1) break;
                        float gn = 0.0f, gp = 0.0f;
#pragma unroll
                        for (int k = 0; k < KA1; ++k) {
                            gn = fmaf(c[n * KA1 + k], f[k], gn);
                            gp = fmaf(c[n * KA1 + k], fp[k], gp);
                        }
                        const float gpr = gp * rdot;
#pragma unroll
                        for (int m = 0; m < kNumSH; ++m) {
                            A[g][m] = fmaf(gn, Y[m], A[g][m]);
                            Ad[g][m] = fmaf(gpr, Y[m], fmaf(gn, Dm[m], Ad[g][m]));
                        }
                    }
                }
            }
#pragma unroll
            for (int g = 0; g < kJvpGroup; ++g) {
                const int n = n0 + g;
                if (n >= NA1) break;
#pragma unroll
                for (int l = 1; l <= kLmax; ++l) {
                    float s2 = 0.0f, s2d = 0.0f;
#pragma unroll
                    for (int m = 0; m < kNumSH; ++m)
                        if (sh_l(m) == l) {
                            s2 = fmaf(A[g][m], A[g][m], s2);
                            s2d = fmaf(2.0f * A[g][m], Ad[g][m], s2d);
                        }
                    const int vv = NR1 + (l - 1) * NA1 + n;
                    row[R.sq + vv] = qs[vv] * s2;
                    row[R.sqd + vv] = qs[vv] * s2d;
                }
#pragma unroll
                for (int m = 0; m < kNumSH; ++m) {
                    xb[n * kNumSH + m] = A[g][m];
                    xb[(NA1 + n) * kNumSH + m] = Ad[g][m];
                }
            }
        }

        // network and its forward derivative (the scaled descriptors read
        // back from the row, written by this lane)
        float qh[D], qhd[D], G[D], Gd[D];
#pragma unroll
        for (int v = 0; v < D; ++v) {
            qh[v] = row[R.sq + v];
            qhd[v] = row[R.sqd + v];
            G[v] = 0.0f;
            Gd[v] = 0.0f;
        }
        const float *W0 = prm + a.oW0 + tc * H * D;
        const float *b0 = prm + a.ob0 + tc * H;
        const float *w1 = prm + a.ow1 + tc * H;
        const float eEb = ta.eE[sb];
        for (int mu = 0; mu < H; ++mu) {
            float z = -b0[mu], zd = 0.0f;
#pragma unroll
            for (int v = 0; v < D; ++v) {
                z = fmaf(W0[mu * D + v], qh[v], z);
                zd = fmaf(W0[mu * D + v], qhd[v], zd);
            }
            const float h = tanhf(z);
            const float dh = 1.0f - h * h;
            const float u = w1[mu] * dh;                   // dU/dz
            const float ud = -2.0f * w1[mu] * h * dh * zd;  // its derivative along d
#pragma unroll
            for (int v = 0; v < D; ++v) {
                G[v] = fmaf(u, W0[mu * D + v], G[v]);
                Gd[v] = fmaf(ud, W0[mu * D + v], Gd[v]);
            }
            row[R.u + mu] = u;
            row[R.v + mu] = eEb * u + ud;
            row[R.gw1 + mu] = eEb * h + dh * zd;
        }
#pragma unroll
        for (int n = 0; n < NR1; ++n) {
            const float g = qs[n] * G[n], gd = qs[n] * Gd[n];
            row[R.gR + n] = eEb * g + gd;
            row[R.GR + n] = g;
        }
        row[R.eE] = eEb;
        row[0] = __int_as_float(tc);

        // angular coefficients: park X and B, then one neighbour pass per n
#pragma unroll
        for (int n = 0; n < NA1; ++n)
#pragma unroll
            for (int m = 0; m < kNumSH; ++m) {
                const int vv = NR1 + (sh_l(m) - 1) * NA1 + n;
                const float g = qs[vv] * G[vv], gd = qs[vv] * Gd[vv];
                const float An = xb[n * kNumSH + m], Adn = xb[(NA1 + n) * kNumSH + m];
                const float Bv = 2.0f * g * An;
                xb[n * kNumSH + m] = eEb * Bv + 2.0f * (gd * An + g * Adn);
                xb[(NA1 + n) * kNumSH + m] = Bv;
            }
        for (int t = 0; t < S; ++t) {
            int s0, s1;
            block_range(a.uendA, i, t, s0, s1);
            for (int n = 0; n < NA1; ++n) {
                float Xn[kNumSH], Bn[kNumSH];
#pragma unroll
                for (int m = 0; m < kNumSH; ++m) {
                    Xn[m] = xb[n * kNumSH + m];
                    Bn[m] = xb[(NA1 + n) * kNumSH + m];
                }
                float acc[KA1];
#pragma unroll
                for (int k = 0; k < KA1; ++k) acc[k] = 0.0f;
                for (int s = s0; s < s1; ++s) {
                    if (!((mA[s] >> b) & 1u)) continue;
                    const int j = rowA[uA[s]] >> 2;
                    float dx, dy, dz;
                    pair_vec<true>(p4[(size_t)j * P + b], pi, lm, dx, dy, dz);
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    const float rinv = __builtin_amdgcn_rsqf(r2);
                    const float r = r2 * rinv;
                    const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
                    float ex, ey, ez;
                    field(ta.dF[(size_t)j * P + b], dx, dy, dz, ex, ey, ez);
                    const float rdot = ux * ex + uy * ey + uz * ez;
                    const float vx = (ex - ux * rdot) * rinv, vy = (ey - uy * rdot) * rinv,
                                vz = (ez - uz * rdot) * rinv;
                    float f[KA1], fp[KA1];
                    cheb_fd<KA1>(r, a.rcAinv, f, fp);
                    float Y[kNumSH], Dm[kNumSH];
                    sh_eval(ux, uy, uz, shc, Y);
                    sh_dir(ux, uy, uz, vx, vy, vz, shc, Dm);
                    float al = 0.0f, be = 0.0f;
#pragma unroll
                    for (int m = 0; m < kNumSH; ++m) {
                        al = fmaf(Xn[m], Y[m], fmaf(Bn[m], Dm[m], al));
                        be = fmaf(Bn[m], Y[m], be);
                    }
                    be *= rdot;
#pragma unroll
                    for (int k = 0; k < KA1; ++k) acc[k] = fmaf(al, f[k], fmaf(be, fp[k], acc[k]));
                }
#pragma unroll
                for (int k = 0; k < KA1; ++k) row[R.gA + (t * NA1 + n) * KA1 + k] = acc[k];
            }
        }
    }
}

// Parameter-gradient partial sums over a chunk of rows.  Output o of a
// species s (o < per-species count) maps to one parameter:
//   W0[s][mu][nu] += u_mu sqd_nu + v_mu sq_nu,  b0[s][mu] -= v_mu,
//   w1[s][mu] += gw1_mu,  cR[s][t][n][k] += gR_n sk_tk + GR_n skd_tk,
// and the last output of the call is b1 -= sum eE.
constexpr int kRowChunk = 16;
__global__ __launch_bounds__(256) void k_grad_partial(const float *__restrict__ rows, size_t nrow, int RW, int S,
                                                      int H, int D, int NR1, int KR1, int NA1, int KA1,
                                                      int rows_per_block, float *__restrict__ part)
{
    extern __shared__ float sh[];   // [kRowChunk][RW]
    const RowLayout R(H, D, NR1, S, KR1, NA1, KA1);
    const int per = H * D + 2 * H + S * NR1 * KR1 + S * NA1 * KA1;
    const int nout = S * per + 1;
    const size_t r0 = (size_t)blockIdx.x * rows_per_block;
    const size_t r1 = r0 + rows_per_block < nrow ? r0 + rows_per_block : nrow;
    // one output per thread and pass; the block's rows are streamed through LDS once per pass
    for (int o0 = 0; o0 < nout; o0 += blockDim.x) {
        const int o = o0 + threadIdx.x;
        int kind = -1, sp = 0, i1 = 0, i2 = 0, t = 0;
        if (o == nout - 1) {
            kind = 4;
        } else if (o < nout) {
            sp = o / per;
            const int q = o - sp * per;
            if (q < H * D) {
                kind = 0; i1 = q / D; i2 = q - i1 * D;
            } else if (q < H * D + H) {
                kind = 1; i1 = q - H * D;
            } else if (q < H * D + 2 * H) {
                kind = 2; i1 = q - H * D - H;
            } else if (q < H * D + 2 * H + S * NR1 * KR1) {
                const int c = q - H * D - 2 * H;   // [t][n][k]
                kind = 3; t = c / (NR1 * KR1);
                const int nk = c - t * NR1 * KR1;
                i1 = nk / KR1; i2 = nk - i1 * KR1;
            } else {
                kind = 5; i1 = q - H * D - 2 * H - S * NR1 * KR1;   // [t][n][k] of the angular coefficients
            }
        }
        float acc = 0.0f;
        for (size_t c0 = r0; c0 < r1; c0 += kRowChunk) {
            const int nr = (int)((r1 - c0) < (size_t)kRowChunk ? (r1 - c0) : (size_t)kRowChunk);
            __syncthreads();
            for (int x = threadIdx.x; x < nr * RW; x += blockDim.x) sh[x] = rows[c0 * RW + x];
            __syncthreads();
            for (int r = 0; r < nr; ++r) {
                const float *rw = sh + r * RW;
                const int ty = __float_as_int(rw[0]);
                if (kind == 4) {
                    if (ty >= 0) acc -= rw[R.eE];
                } else if (kind >= 0 && ty == sp) {
                    if (kind == 0) acc = fmaf(rw[R.u + i1], rw[R.sqd + i2], fmaf(rw[R.v + i1], rw[R.sq + i2], acc));
                    else if (kind == 1) acc -= rw[R.v + i1];
                    else if (kind == 2) acc += rw[R.gw1 + i1];
                    else if (kind == 5) acc += rw[R.gA + i1];
                    else acc = fmaf(rw[R.gR + i1], rw[R.sk + t * KR1 + i2], fmaf(rw[R.GR + i1], rw[R.skd + t * KR1 + i2], acc));
                }
            }
        }
        if (o < nout) part[(size_t)blockIdx.x * nout + o] = acc;
    }
}

// Sums the partials and scatters them to the parameter layout.  A
// workgroup takes 64 consecutive outputs (one per lane, coalesced reads);
// its kGradWaves wavefronts take every kGradWaves-th block in order, and
// the wavefronts' sums are added in wavefront order (fixed order).
constexpr int kGradWaves = 16;
__global__ __launch_bounds__(64 * kGradWaves) void k_grad_final(const float *__restrict__ part, int nblk, int S, int H,
                                                                int D, int NR1, int KR1, int NA1, int KA1,
                                                                ParamLayout off, float *__restrict__ grad)
{
    const int per = H * D + 2 * H + S * NR1 * KR1 + S * NA1 * KA1;
    const int nout = S * per + 1;
    const int w = threadIdx.x >> 6;
    const int o = blockIdx.x * 64 + (threadIdx.x & 63);
    __shared__ double red[kGradWaves][64];
    double acc = 0.0;
    if (o < nout)
        for (int k = w; k < nblk; k += kGradWaves) acc += part[(size_t)k * nout + o];
    red[w][threadIdx.x & 63] = acc;
    __syncthreads();
    if (w != 0 || o >= nout) return;
    double s = 0.0;
    for (int v = 0; v < kGradWaves; ++v) s += red[v][threadIdx.x];
    int idx;
    if (o == nout - 1) {
        idx = off.b1;
    } else {
        const int sp = o / per, q = o - sp * per;
        if (q < H * D) idx = off.W0 + sp * H * D + q;
        else if (q < H * D + H) idx = off.b0 + sp * H + (q - H * D);
        else if (q < H * D + 2 * H) idx = off.w1 + sp * H + (q - H * D - H);
        else if (q < H * D + 2 * H + S * NR1 * KR1) idx = off.cR + sp * S * NR1 * KR1 + (q - H * D - 2 * H);
        else idx = off.cA + sp * S * NA1 * KA1 + (q - H * D - 2 * H - S * NR1 * KR1);
    }
    grad[idx] += (float)s;
}

// Adam with bias correction over the trainable parameter ranges.
__global__ void k_adam(float *__restrict__ th, const float *__restrict__ g, float *__restrict__ m1,
                       float *__restrict__ m2, int n, const int32_t *__restrict__ trainable, float lr, float b1,
                       float b2, float eps, float c1, float c2)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || !trainable[k]) return;
    const float gk = g[k];
    const float a = b1 * m1[k] + (1.0f - b1) * gk;
    const float v = b2 * m2[k] + (1.0f - b2) * gk * gk;
    m1[k] = a;
    m2[k] = v;
    th[k] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

template <int NR1, int NA1>
static void launch_jvp(const NepArgs &a, const TrainArgs &t, const float *prm, int nblk, int wpb, hipStream_t s)
{
    hipLaunchKernelGGL((k_train_jvp<NR1, NA1, 9, 9>), dim3(nblk), dim3(64 * wpb), 0, s, a, t, prm);
}

}  // namespace nep

using namespace nep;

struct nep_train_ws {
    int P = 0, N = 0, nsys = 1;
    std::vector<int> off;                // host [nsys+1]
    int32_t *atom_sys = nullptr;         // [N] system of each atom
    int32_t *sys_off = nullptr;          // [nsys+1]
    double *E = nullptr, *W = nullptr;   // [nsys][P], [nsys][P][9]
    float *F = nullptr;                  // [P][N][3]
    float4 *dF = nullptr;                // [N][P]
    float *cW = nullptr, *eE = nullptr;  // [nsys][P][9], [nsys][P]
    float *rows = nullptr;               // [N*P][RW]
    float *xb = nullptr;                 // [N*P][2][NA1][24]
    float *part = nullptr;               // [nblk][nout]
    int RW = 0, nout = 0, nblk = 0, rows_per_block = 0;
    int32_t *trainable = nullptr;        // [params] 0/1
    int ntrain_mask = -1;
};

extern "C" int32_t nep_train_ws_create_batched(const nep_model *m, int32_t P, int32_t nsys, const int32_t *off,
                                               nep_train_ws **out)
{
    if (!m || !out) return fail(NEP_ERR_INVALID_ARG, "nep_train_ws_create: null argument");
    if (m->cutoffs_only) return fail(NEP_ERR_INVALID_ARG, "nep_train_ws_create: a list cutoff descriptor has no network");
    if (m->embedded)
        return fail(NEP_ERR_UNSUPPORTED, "nep_train_ws_create: a model embedded in a larger kernel shape is not trainable");
    const int32_t rc0 = check_offsets(nsys, off, "nep_train_ws_create");
    if (rc0 != NEP_OK) return rc0;
    const int32_t N = off[nsys];
    if (P < 1 || P > kMaxBeads || N < 1) return fail(NEP_ERR_INVALID_ARG, "nep_train_ws_create: bad sizes");
    const nep_hparams &h = m->hp;
    if (h.four_body) return fail(NEP_ERR_UNSUPPORTED, "nep_train_ws_create: four-body models are not trainable");
    const int key = h.n_max_radial * 100 + h.n_max_angular * 10;
    if (key != 440 && key != 640 && key != 860)
        return fail(NEP_ERR_UNSUPPORTED, "nep_train_ws_create: unsupported model shape");
    const int S = h.n_species, H = h.hidden, D = h.dim, NR1 = h.n_max_radial + 1, KR1 = h.basis_radial + 1;
    const int NA1 = h.n_max_angular + 1, KA1 = h.basis_angular + 1;
    const RowLayout R(H, D, NR1, S, KR1, NA1, KA1);
    const int nout = S * (H * D + 2 * H + S * NR1 * KR1 + S * NA1 * KA1) + 1;
    if ((nout + 255) / 256 > 64) return fail(NEP_ERR_UNSUPPORTED, "nep_train_ws_create: model too large to train");
    *out = nullptr;
    nep_train_ws *w = new (std::nothrow) nep_train_ws;
    if (!w) return fail(NEP_ERR_NOMEM, "host allocation failed");
    w->P = P; w->N = N; w->RW = R.RW; w->nout = nout;
    w->nsys = nsys;
    w->off.assign(off, off + nsys + 1);
    std::vector<int32_t> asys((size_t)N);
    for (int sy = 0; sy < nsys; ++sy)
        for (int i = off[sy]; i < off[sy + 1]; ++i) asys[i] = sy;
    const size_t PN = (size_t)P * N;
    // enough workgroups to fill the chip for a single snapshot, at most 512 rows each
    w->rows_per_block = (int)std::min<size_t>(512, std::max<size_t>(kRowChunk, (PN + 1023) / 1024));
    w->nblk = (int)((PN + w->rows_per_block - 1) / w->rows_per_block);
    hipError_t e = hipSuccess;
    auto al = [&](void **p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes ? bytes : 4);
    };
    al((void **)&w->atom_sys, sizeof(int32_t) * N);
    al((void **)&w->sys_off, sizeof(int32_t) * (nsys + 1));
    if (e == hipSuccess) e = hipMemcpy(w->atom_sys, asys.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(w->sys_off, off, sizeof(int32_t) * (nsys + 1), hipMemcpyHostToDevice);
    al((void **)&w->E, sizeof(double) * nsys * P);
    al((void **)&w->W, sizeof(double) * 9 * nsys * P);
    al((void **)&w->F, sizeof(float) * 3 * PN);
    al((void **)&w->dF, sizeof(float4) * PN);
    al((void **)&w->cW, sizeof(float) * 9 * nsys * P);
    al((void **)&w->eE, sizeof(float) * nsys * P);
    al((void **)&w->rows, sizeof(float) * PN * R.RW);
    al((void **)&w->xb, sizeof(float) * PN * 2 * NA1 * kNumSH);
    al((void **)&w->part, sizeof(float) * (size_t)w->nblk * nout);
    al((void **)&w->trainable, sizeof(int32_t) * m->off.total);
    if (e != hipSuccess) {
        nep_train_ws_destroy(w);
        return fail(e == hipErrorOutOfMemory ? NEP_ERR_NOMEM : NEP_ERR_HIP, "training workspace: %s",
                    hipGetErrorString(e));
    }
    *out = w;
    return NEP_OK;
}

extern "C" void nep_train_ws_destroy(nep_train_ws *w)
{
    if (!w) return;
    for (void *p : {(void *)w->atom_sys, (void *)w->sys_off, (void *)w->E, (void *)w->W, (void *)w->F, (void *)w->dF, (void *)w->cW, (void *)w->eE,
                    (void *)w->rows, (void *)w->xb, (void *)w->part, (void *)w->trainable})
        if (p) (void)hipFree(p);
    delete w;
}

extern "C" int32_t nep_train_ws_create(const nep_model *m, int32_t P, int32_t N, nep_train_ws **out)
{
    if (N < 1) return fail(NEP_ERR_INVALID_ARG, "nep_train_ws_create: bad sizes");
    const int32_t off[2] = {0, N};
    return nep_train_ws_create_batched(m, P, 1, off, out);
}

extern "C" int32_t nep_param_grad_batched(const nep_model *m, nep_nlist *nl, nep_ws *ws, nep_train_ws *tw,
                                          const double *pos, const double *boxes, const int32_t *types, int32_t P,
                                          int32_t N, const double *E_ref, const float *F_ref, const double *W_ref,
                                          const double lambda[3], float *grad, double *loss, hipStream_t s)
{
    if (!m || !nl || !ws || !tw || !lambda || !grad || !loss || !E_ref || !F_ref || !W_ref)
        return fail(NEP_ERR_INVALID_ARG, "nep_param_grad: null argument");
    if (m->cutoffs_only) return fail(NEP_ERR_INVALID_ARG, "nep_param_grad: a list cutoff descriptor has no network");
    if (tw->P != P || tw->N != N || nl->nsys != tw->nsys || ws->nsys != tw->nsys || nl->off != tw->off ||
        ws->off != tw->off)
        return fail(NEP_ERR_INVALID_ARG, "nep_param_grad: sizes or systems do not match the training workspace");
    if (m->mlp == NEP_MLP_BF16_MFMA)
        return fail(NEP_ERR_INVALID_ARG, "nep_param_grad: training needs the FP32 weights (nep_model_set_mlp)");
    int32_t rc = nep_compute_batched(m, nl, ws, pos, boxes, types, P, N, tw->E, tw->F, tw->W, nullptr, nullptr, s);
    if (rc != NEP_OK) return rc;
    const size_t PN = (size_t)P * N;
    hipLaunchKernelGGL(k_residual, dim3((unsigned)((PN + 255) / 256)), dim3(256), 0, s, tw->F, F_ref, tw->E, E_ref,
                       tw->W, W_ref, P, N, tw->nsys, tw->atom_sys, tw->sys_off, lambda[0], lambda[1], lambda[2],
                       tw->dF, tw->cW, tw->eE, loss);
    const nep_hparams &h = m->hp;
    NepArgs a{};
    a.p4 = reinterpret_cast<const float4 *>(nl->pos4); a.pos = pos; a.types = types; a.N = N; a.S = h.n_species;
    a.H = h.hidden; a.P = P; a.lg = lanes_log2(P);
    a.geom = nl->geom; a.tile_atom0 = ws->tile_atom0; a.tile_atom1 = ws->tile_atom1; a.tile_sys = ws->tile_sys;
    a.rcRinv = (float)(1.0 / h.rc_radial); a.rcAinv = (float)(1.0 / h.rc_angular);
    a.candA = nl->candA; a.revA = nl->revA; a.uniR = nl->uniR; a.uendR = nl->uendR; a.uniA = nl->uniA;
    a.umR = nl->umR; a.umA = nl->umA; a.uendA = nl->uendA; a.capR = nl->capR; a.capA = nl->capA;
    a.oR = m->off.cR; a.oA = m->off.cA; a.oq = m->off.qs; a.oW0 = m->off.W0; a.ob0 = m->off.b0;
    a.ow1 = m->off.w1; a.ob1 = m->off.b1; a.osh = m->off.sh;
    TrainArgs t{tw->dF, tw->cW, tw->eE, tw->rows, tw->RW, tw->xb};
    // rows of idle lanes stay unused: mark every row unused first
    fill_u32(reinterpret_cast<uint32_t *>(tw->rows), 0xffffffffu, PN * tw->RW, s);
    const int key = h.n_max_radial * 100 + h.n_max_angular * 10;
    switch (key) {
    case 440: launch_jvp<5, 5>(a, t, m->dev, ws->nblk, ws->wpb, s); break;
    case 640: launch_jvp<7, 5>(a, t, m->dev, ws->nblk, ws->wpb, s); break;
    case 860: launch_jvp<9, 7>(a, t, m->dev, ws->nblk, ws->wpb, s); break;
    default: return fail(NEP_ERR_UNSUPPORTED, "nep_param_grad: unsupported model shape");
    }
    const int S = h.n_species, H = h.hidden, D = h.dim, NR1 = h.n_max_radial + 1, KR1 = h.basis_radial + 1;
    const int NA1 = h.n_max_angular + 1, KA1 = h.basis_angular + 1;
    hipLaunchKernelGGL(k_grad_partial, dim3(tw->nblk), dim3(256), sizeof(float) * kRowChunk * tw->RW, s, tw->rows,
                       PN, tw->RW, S, H, D, NR1, KR1, NA1, KA1, tw->rows_per_block, tw->part);
    hipLaunchKernelGGL(k_grad_final, dim3((tw->nout + 63) / 64), dim3(64 * kGradWaves), 0, s, tw->part, tw->nblk, S,
                       H, D, NR1, KR1, NA1, KA1, m->off, grad);
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}

extern "C" int32_t nep_param_grad(const nep_model *m, nep_nlist *nl, nep_ws *ws, nep_train_ws *tw, const double *pos,
                                  const double box[9], const int32_t *types, int32_t P, int32_t N,
                                  const double *E_ref, const float *F_ref, const double *W_ref,
                                  const double lambda[3], float *grad, double *loss, hipStream_t s)
{
    if ((nl && nl->nsys != 1) || (tw && tw->nsys != 1))
        return fail(NEP_ERR_INVALID_ARG, "nep_param_grad: the list or workspace holds a batch of systems");
    return nep_param_grad_batched(m, nl, ws, tw, pos, box, types, P, N, E_ref, F_ref, W_ref, lambda, grad, loss, s);
}

extern "C" int32_t nep_model_params(nep_model *m, float **params, int32_t *count, nep_param_offsets *off)
{
    if (!m || !params || !count) return fail(NEP_ERR_INVALID_ARG, "nep_model_params: null argument");
    if (m->cutoffs_only) return fail(NEP_ERR_INVALID_ARG, "nep_model_params: a list cutoff descriptor has no network");
    if (m->embedded)
        return fail(NEP_ERR_UNSUPPORTED, "nep_model_params: the parameters of a model embedded in a larger kernel "
                                         "shape are not exposed");
    *params = m->dev;
    *count = m->off.total;
    if (off) {
        off->c_radial = m->off.cR; off->c_angular = m->off.cA; off->q_scale = m->off.qs; off->W0 = m->off.W0;
        off->b0 = m->off.b0; off->w1 = m->off.w1; off->b1 = m->off.b1; off->sh = m->off.sh;
    }
    return NEP_OK;
}

extern "C" int32_t nep_adam_step(nep_model *m, nep_train_ws *tw, const float *grad, float *m1, float *m2,
                                 int64_t step, float lr, float beta1, float beta2, float eps, int32_t mask,
                                 hipStream_t s)
{
    if (!m || !tw || !grad || !m1 || !m2) return fail(NEP_ERR_INVALID_ARG, "nep_adam_step: null argument");
    if (step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
        !(eps > 0.0f) || mask < 1 || mask > 7)
        return fail(NEP_ERR_INVALID_ARG, "nep_adam_step: bad hyperparameters");
    const int n = m->off.total;
    if (tw->ntrain_mask != mask) {
        const nep_hparams &h = m->hp;
        std::vector<int32_t> tr(n, 0);
        if (mask & 1)
            for (int k = m->off.W0; k < m->off.b1 + 1; ++k) tr[k] = 1;   // W0, b0, w1, b1
        if (mask & 2) {
            const int nR = h.n_species * h.n_species * (h.n_max_radial + 1) * (h.basis_radial + 1);
            for (int k = m->off.cR; k < m->off.cR + nR; ++k) tr[k] = 1;
        }
        if (mask & 4) {
            const int nA = h.n_species * h.n_species * (h.n_max_angular + 1) * (h.basis_angular + 1);
            for (int k = m->off.cA; k < m->off.cA + nA; ++k) tr[k] = 1;
        }
        NEP_HIP(hipStreamSynchronize(s));
        NEP_HIP(hipMemcpy(tw->trainable, tr.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
        tw->ntrain_mask = mask;
    }
    const double c1 = 1.0 - std::pow((double)beta1, (double)step), c2 = 1.0 - std::pow((double)beta2, (double)step);
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, m->dev, grad, m1, m2, n, tw->trainable, lr,
                       beta1, beta2, eps, (float)c1, (float)c2);
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}

// ------------------------------------------------------- force judge ---

// Root-mean-square difference of two force arrays over every component,
// sqrt(sum (Fa - Fb)^2 / n): fixed-grid partial sums in FP64, then one
// block adds the partials in a fixed order (bitwise reproducible).
constexpr int kRmseBlocks = 1024;

__global__ __launch_bounds__(256) void k_rmse_partial(const float *__restrict__ Fa, const float *__restrict__ Fb,
                                                      int64_t n, double *__restrict__ part)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)Fa[e] - (double)Fb[e];
        acc += d * d;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_rmse_final(const double *__restrict__ part, int nblk, int64_t n,
                                                    double *__restrict__ out)
{
    __shared__ double red[256];
    double acc = 0.0;
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) acc += part[k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = n > 0 ? sqrt(red[0] / (double)n) : 0.0;
}

extern "C" int32_t nep_force_rmse(const float *Fa, const float *Fb, int64_t n, double *work, hipStream_t s)
{
    if (!work) return fail(NEP_ERR_INVALID_ARG, "nep_force_rmse: null work array");
    if (n < 0) return fail(NEP_ERR_INVALID_ARG, "nep_force_rmse: negative length");
    if (n > 0 && (!Fa || !Fb)) return fail(NEP_ERR_INVALID_ARG, "nep_force_rmse: null force array");
    const int nblk = (int)std::min<int64_t>(kRmseBlocks, std::max<int64_t>(1, (n + 255) / 256));
    if (n > 0)
        hipLaunchKernelGGL(k_rmse_partial, dim3(nblk), dim3(256), 0, s, Fa, Fb, n, work + 1);
    hipLaunchKernelGGL(k_rmse_final, dim3(1), dim3(256), 0, s, work + 1, n > 0 ? nblk : 0, n, work);
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}
