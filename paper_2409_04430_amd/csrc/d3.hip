// D3 dispersion with Becke-Johnson damping, the dispersion term of NEP-D3
// (the paper's MOF model, Sec. II.C: 12 A dispersion cutoff, 6 A
// coordination-number cutoff), for every bead of a ring polymer on gfx950.
//
// Published D3 form (Grimme et al. 2010: coordination numbers and the C6
// interpolation; Grimme, Ehrlich and Goerigk 2011: the damping), eV and A:
//   CN_i  = sum_{j, r < rc_cn} 1 / (1 + exp(-k1 (k2 (R_i + R_j) / r - 1)))
//   C6_ij = sum_ab C6ref(a, b) L_i,a L_j,b / (sum_a L_i,a sum_b L_j,b),
//           L_i,a = exp(-k3 (CN_i - CNref_i,a)^2)
//   C8_ij = 3 C6_ij q_i q_j,  f_ij = a1 sqrt(3 q_i q_j) + a2
//   E     = -1/2 sum_i sum_{j, r < rc} [s6 C6 / (r^6 + f^6) + s8 C8 / (r^8 + f^8)]
// The weights of one atom share the factor exp(-k3 m_i), m_i the smallest
// squared distance to a reference, which cancels in C6 and its derivative;
// dividing it out keeps the largest weight at 1 (far from every reference
// the plain weights underflow).  FP64 throughout: pair vectors from a
// bead-minor FP64 copy of the positions with the minimum image of the list
// test, FP64 weights and sums (the many pair terms of a near-perfect
// crystal nearly cancel, which FP32 terms would not resolve).
//
// Lists: a neighbour handle built with the cutoff descriptor of the D3
// parameters (dispersion cutoff as its radial cutoff, coordination cutoff as
// its angular one), so the per-bead pair sets are the exact FP64 decisions
// of the union lists' bead masks.  Passes, one lane per (atom, bead), the
// beads of an atom in adjacent lanes, gathers only (no atomics):
//   k_d3_cn       CN_i over the coordination list, and the atom's reference
//                 weights divided by their sum, w_i,a = L_i,a / sum_a L_i,a,
//                 which its partners gather in the next pass;
//   k_d3_pair     site energy, direct forces and virial over the dispersion
//                 list, and dE/dCN_i = -sum_j (de_ij/dC6) dC6_ij/dCN_i.
//                 C6_ij = sum_b V_i,b w_j,b with V_i,b = sum_a w_i,a
//                 C6ref(a, b) formed once per (lane, partner species), and
//                 dC6_ij/dCN_i = sum_b V'_i,b w_j,b with V' built from
//                 dw_i,a/dCN_i: two 5-term dot products per pair;
//   k_d3_cnforce  forces (dE/dCN_i + dE/dCN_j) c'(r) u_ij and virial
//                 -dE/dCN_i c'(r) r_ij (x) u_ij through the coordination
//                 numbers, the total force written (or added);
//   k_d3_reduce   per-bead energy and virial from per-workgroup partial sums
//                 in a fixed order.
#include <cmath>
#include <fstream>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"
#include "nep_kernels.hpp"

namespace nep {

constexpr int kD3Ref = 5;
// table: rcov [4], q [4], cnref [4][5], c6ref [4][4][5][5], f^6 [4][4], f^8 [4][4], 3 q_i q_j [4][4],
// reference counts [4]
constexpr int kTRcov = 0, kTQ = 4, kTCn = 8, kTC6 = kTCn + kMaxSpecies * kD3Ref,
              kTF6 = kTC6 + kMaxSpecies * kMaxSpecies * kD3Ref * kD3Ref, kTF8 = kTF6 + 16, kTQQ = kTF8 + 16,
              kTNref = kTQQ + 16, kTab = kTNref + kMaxSpecies;
constexpr int kD3Batch = 4;       // list entries whose loads are issued together (coordination passes)
constexpr int kD3PairBatch = 2;   // the same in the dispersion pass (FP64 registers)
constexpr double kD3PadCn = 1.0e4;   // reference slots past a species' count: weight exp(-k3 1e8) = 0

struct D3Args {
    const double *posT;   // [N][P][3] FP64 positions, bead-minor
    const int32_t *types;
    int N, P, lg, S;
    int lgc;                     // dispersion pass: 2^lgc lanes per atom, one bead chunk each
    const SysGeom *geom;
    const int32_t *candA, *uniR, *uendR, *uniA, *uendA;
    const uint64_t *umR, *umA;
    int capR, capA;
    const double *tab;
    double s6, s8, k1, k2, k3;
    double *cn, *dedcn, *fdir;   // [N][P], [N][P], [N][P][3]
    double *wts;                 // [5][N][P]: normalised reference weights w_0..4, one plane per reference
    double *partE, *partW0, *partW1;   // [P][nblk], [P][9][nblk] twice
    float *F;
    int accumulate;
};

// (atom, bead) of this lane in the coordination passes: 2^lg lanes per
// atom, 256 >> lg atoms per workgroup, in launch order (a permutation that
// gives each XCD one contiguous run of atoms measured slower in these
// passes).
__device__ __forceinline__ bool d3_lane(const D3Args &a, int &i, int &b)
{
    const int G = 1 << a.lg;
    i = blockIdx.x * (256 >> a.lg) + ((int)threadIdx.x >> a.lg);
    b = threadIdx.x & (G - 1);
    const bool ok = i < a.N && b < a.P;
    i = i < a.N ? i : a.N - 1;
    b = b < a.P ? b : a.P - 1;
    return ok;
}

__device__ __forceinline__ void load_tab(const D3Args &a, double *t)
{
    for (int x = threadIdx.x; x < kTab; x += blockDim.x) t[x] = a.tab[x];
    __syncthreads();
}

// Bead-minor FP64 copy of the positions: the beads of a neighbour are one
// contiguous run for the lanes that gather them.
__global__ void k_d3_beads_minor(const double *__restrict__ pos, double *__restrict__ posT, int P, int N)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (i, b) with b fastest
    if (e >= (int64_t)N * P) return;
    const int i = (int)(e / P), b = (int)(e - (int64_t)i * P);
    const double *src = pos + ((size_t)b * N + i) * 3;
    double *dst = posT + (size_t)e * 3;
    dst[0] = src[0];
    dst[1] = src[1];
    dst[2] = src[2];
}

// Minimum-image vector r_j - r_i in FP64 (every listed pair is closer than
// half the smallest face distance, so the rint reduction gives the nearest
// image, as in the list test).
// TRI = false: launches on orthorhombic cells only, no general-cell code.
template <bool TRI>
__device__ __forceinline__ void d3_pair_vec(const double *rj, double xi, double yi, double zi, const SysGeom &g,
                                            double &dx, double &dy, double &dz)
{
    double d[3] = {rj[0] - xi, rj[1] - yi, rj[2] - zi};
    if (!TRI || !g.tri) {
#pragma unroll
        for (int c = 0; c < 3; ++c) d[c] -= g.L[c] * rint(d[c] * g.invL[c]);
    } else {
        double f[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double sc = d[0] * g.G[c] + d[1] * g.G[3 + c] + d[2] * g.G[6 + c];
            f[c] = sc - rint(sc);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) d[c] = f[0] * g.H[c] + f[1] * g.H[3 + c] + f[2] * g.H[6 + c];
    }
    dx = d[0];
    dy = d[1];
    dz = d[2];
}

// Reference weights of one atom at coordination number cn, divided by
// exp(-k3 m), m the smallest squared distance to a reference (the factor
// cancels in C6 and in its derivative), with their derivatives at a fixed
// factor; returns the sums.
__device__ __forceinline__ void ref_weights(const double *t, int ty, double cn, double k3, double (&L)[kD3Ref],
                                            double (&dL)[kD3Ref], double &sL, double &sdL)
{
    double x[kD3Ref], m = 1.0e300;
#pragma unroll
    for (int r = 0; r < kD3Ref; ++r) {
        x[r] = cn - t[kTCn + ty * kD3Ref + r];
        m = fmin(m, x[r] * x[r]);
    }
    sL = 0.0;
    sdL = 0.0;
#pragma unroll
    for (int r = 0; r < kD3Ref; ++r) {
        L[r] = exp(-k3 * (x[r] * x[r] - m));
        dL[r] = -2.0 * k3 * x[r] * L[r];
        sL += L[r];
        sdL += dL[r];
    }
}

// Lanes of the dispersion pass: 2^lgc <= 16 lanes per atom take one chunk
// of 2^lgc beads, grid (atom blocks, bead chunks), so that the partner data
// a workgroup gathers (positions and weights of its chunk of beads) is a
// quarter of a 64-bead atom's and the run of atoms an XCD works through at
// once keeps its partners in that XCD's L2.  Workgroups go to the 8 XCDs
// round-robin; when their number is a multiple of 8 the linear workgroup id
// (bead chunk slowest) is permuted so that each XCD works through one
// contiguous run of it, i.e. a run of neighbouring atoms (whose partners
// are nearby atom indices) for one bead chunk.  Returns the atom block in
// blk and the chunk's first bead in b0.
__device__ __forceinline__ bool d3_chunk_lane(const D3Args &a, int &i, int &b, int &blk, int &b0)
{
    const int Gc = 1 << a.lgc, nb = gridDim.x, total = nb * gridDim.y;
    int lin = blockIdx.y * nb + blockIdx.x;
    if ((total & 7) == 0) lin = (lin & 7) * (total >> 3) + (lin >> 3);
    const int chunk = lin / nb;
    blk = lin - chunk * nb;
    b0 = chunk * Gc;
    i = blk * (256 >> a.lgc) + ((int)threadIdx.x >> a.lgc);
    b = b0 + ((int)threadIdx.x & (Gc - 1));
    const bool ok = i < a.N && b < a.P;
    i = i < a.N ? i : a.N - 1;
    b = b < a.P ? b : a.P - 1;
    return ok;
}

// Per-bead sums over a workgroup of the chunked pass: lane t < 2^lgc adds
// lanes t, t + 2^lgc, ... in order and writes bead b0 + t at out[bead * stride].
__device__ __forceinline__ void chunk_block_sum(double v, double *lds, int lgc, int b0, int P, double *out,
                                                int stride)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    const int t = threadIdx.x, Gc = 1 << lgc;
    if (t < Gc && b0 + t < P) {
        double s = 0.0;
        for (int x = t; x < (int)blockDim.x; x += Gc) s += lds[x];
        out[(size_t)(b0 + t) * stride] = s;
    }
    __syncthreads();
}

// ------------------------------------------------ coordination numbers ---

template <bool TRI>
__global__ __launch_bounds__(256) void k_d3_cn(D3Args a)
{
    __shared__ double t[kTab];
    load_tab(a, t);
    int i, b;
    const bool ok = d3_lane(a, i, b);
    if (!ok) return;
    const SysGeom &g = a.geom[0];
    const int P = a.P, ti = a.types[i] & 3;
    const double *ri = a.posT + ((size_t)i * P + b) * 3;
    const int32_t *uA = a.uniA + (size_t)i * a.capA;
    const uint64_t *mA = a.umA + (size_t)i * a.capA;
    const int32_t *row = a.candA + (size_t)i * a.capA;
    const int n = a.uendA[(size_t)i * kMaxSpecies + a.S - 1];
    const double xi = ri[0], yi = ri[1], zi = ri[2];
    const double Ri = t[kTRcov + ti], kk = a.k1 * a.k2;
    double cn = 0.0;
    // entries four at a time: every load of a batch issued before its arithmetic
    for (int e0 = 0; e0 < n; e0 += kD3Batch) {
        uint64_t mm[kD3Batch];
        int w[kD3Batch];
#pragma unroll
        for (int k = 0; k < kD3Batch; ++k) {
            const int e = min(e0 + k, n - 1);
            const uint64_t m = mA[e];
            mm[k] = e0 + k < n ? m : 0ull;
            w[k] = uA[e];
        }
#pragma unroll
        for (int k = 0; k < kD3Batch; ++k) w[k] = row[w[k]];
        double pj[kD3Batch][3];
#pragma unroll
        for (int k = 0; k < kD3Batch; ++k) {
            const double *q = a.posT + ((size_t)(w[k] >> 2) * P + b) * 3;
            pj[k][0] = q[0];
            pj[k][1] = q[1];
            pj[k][2] = q[2];
        }
#pragma unroll
        for (int k = 0; k < kD3Batch; ++k) {
            double dx, dy, dz;
            d3_pair_vec<TRI>(pj[k], xi, yi, zi, g, dx, dy, dz);
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double c = 1.0 / (1.0 + exp(a.k1 - kk * (Ri + t[kTRcov + (w[k] & 3)]) / r));
            cn += ((mm[k] >> b) & 1u) ? c : 0.0;
        }
    }
    a.cn[(size_t)i * P + b] = cn;
    // this atom's normalised reference weights, gathered by every partner in the pair pass
    double L[kD3Ref], dL[kD3Ref], sL, sdL;
    ref_weights(t, ti, cn, a.k3, L, dL, sL, sdL);
    const double is = 1.0 / sL;
    const size_t PN = (size_t)a.N * P;
#pragma unroll
    for (int r = 0; r < kD3Ref; ++r) a.wts[r * PN + (size_t)i * P + b] = L[r] * is;
}

// ------------------------------------------- dispersion pairs, dE/dCN ---

template <bool TRI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_d3_pair(D3Args a)
{
    __shared__ double t[kTab];
    __shared__ double lds[256];
    load_tab(a, t);
    int i, b, blk, bc0;
    const bool ok = d3_chunk_lane(a, i, b, blk, bc0);
    const SysGeom &g = a.geom[0];
    const int P = a.P, S = a.S, ti = a.types[i] & 3;
    const double *ri = a.posT + ((size_t)i * P + b) * 3;
    const double xi = ri[0], yi = ri[1], zi = ri[2];
    // this lane's normalised weights w_a and their derivatives
    // dw_a/dCN = (dL_a - w_a sum dL) / sum L, parked in LDS (column per
    // lane) until each partner species block forms its V and V'
    __shared__ double wsh[2 * kD3Ref][256];
    {
        double L[kD3Ref], dL[kD3Ref], sL, sdL;
        ref_weights(t, ti, a.cn[(size_t)i * P + b], a.k3, L, dL, sL, sdL);
        const double is = 1.0 / sL;
#pragma unroll
        for (int r = 0; r < kD3Ref; ++r) {
            const double w = L[r] * is;
            wsh[r][threadIdx.x] = w;
            wsh[kD3Ref + r][threadIdx.x] = (dL[r] - w * sdL) * is;
        }
    }
    double U = 0.0, dE = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    double Wv[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // xx yy zz xy xz yz (symmetric), halved at the end
    const int32_t *uR = a.uniR + (size_t)i * a.capR;
    const uint64_t *mR = a.umR + (size_t)i * a.capR;
    const size_t PN = (size_t)a.N * P;
    for (int tj = 0; tj < S && ok; ++tj) {
        int s0, s1;
        block_range(a.uendR, i, tj, s0, s1);
        if (s1 <= s0) continue;
        // V_b = sum_a w_i,a C6ref(a, b) and its CN_i derivative for this partner species
        const double *c6 = t + kTC6 + (ti * kMaxSpecies + tj) * kD3Ref * kD3Ref;
        double V[kD3Ref], dV[kD3Ref];
#pragma unroll
        for (int rb = 0; rb < kD3Ref; ++rb) {
            double v = 0.0, dv = 0.0;
#pragma unroll
            for (int ra = 0; ra < kD3Ref; ++ra) {
                v = fma(wsh[ra][threadIdx.x], c6[ra * kD3Ref + rb], v);
                dv = fma(wsh[kD3Ref + ra][threadIdx.x], c6[ra * kD3Ref + rb], dv);
            }
            V[rb] = v;
            dV[rb] = dv;
        }
        const int nr = (int)t[kTNref + tj];   // the partner's weight planes past its reference count are 0
        const double f6 = t[kTF6 + ti * 4 + tj], f8 = t[kTF8 + ti * 4 + tj];
        const double s6 = a.s6, s8q = a.s8 * t[kTQQ + ti * 4 + tj];
        for (int e0 = s0; e0 < s1; e0 += kD3PairBatch) {
            uint64_t mm[kD3PairBatch];
            int jj[kD3PairBatch];
#pragma unroll
            for (int k = 0; k < kD3PairBatch; ++k) {
                const int e = min(e0 + k, s1 - 1);
                const uint64_t m = mR[e];
                mm[k] = e0 + k < s1 ? m : 0ull;
                jj[k] = uR[e];
            }
            double pj[kD3PairBatch][3], wj[kD3PairBatch][kD3Ref];
#pragma unroll
            for (int k = 0; k < kD3PairBatch; ++k) {
                const size_t o = (size_t)jj[k] * P + b;
                const double *q = a.posT + o * 3;
                pj[k][0] = q[0];
                pj[k][1] = q[1];
                pj[k][2] = q[2];
#pragma unroll
                for (int r = 0; r < kD3Ref; ++r) wj[k][r] = r < nr ? a.wts[r * PN + o] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < kD3PairBatch; ++k) {
                double dx, dy, dz;
                d3_pair_vec<TRI>(pj[k], xi, yi, zi, g, dx, dy, dz);
                const double r2 = dx * dx + dy * dy + dz * dz;
                double C6 = 0.0, dC6 = 0.0;
#pragma unroll
                for (int r = 0; r < kD3Ref; ++r) {
                    C6 = fma(V[r], wj[k][r], C6);
                    dC6 = fma(dV[r], wj[k][r], dC6);
                }
                const double r6 = r2 * r2 * r2, r8 = r6 * r2;
                const double a6 = r6 + f6, a8 = r8 + f8;
                // one division for 1/a6, 1/a8 and 1/r2
                const double inv = 1.0 / (a6 * a8 * r2);
                const double a8r = a8 * r2, a6r = a6 * r2;
                const double d6inv = a8r * inv, d8inv = a6r * inv, ir2 = a6 * a8 * inv;
                const double e6 = s6 * C6 * d6inv, e8 = s8q * C6 * d8inv;
                // de/dr / r = -(6 e6 r^6 / (r^6 + f^6) + 8 e8 r^8 / (r^8 + f^8)) / r^2
                const double on = ((mm[k] >> b) & 1u) ? 1.0 : 0.0;
                const double dedr_r = -on * (6.0 * e6 * r6 * d6inv + 8.0 * e8 * r8 * d8inv) * ir2;
                const double dedc6 = on * (s6 * d6inv + s8q * d8inv);
                U += on * (e6 + e8);
                dE -= dedc6 * dC6;
                // F_i = -sum_j e' u_ij;  W += 1/2 e' r_ij (x) u_ij
                fx -= dedr_r * dx;
                fy -= dedr_r * dy;
                fz -= dedr_r * dz;
                Wv[0] += dedr_r * dx * dx; Wv[1] += dedr_r * dy * dy; Wv[2] += dedr_r * dz * dz;
                Wv[3] += dedr_r * dx * dy; Wv[4] += dedr_r * dx * dz; Wv[5] += dedr_r * dy * dz;
            }
        }
    }
    U *= -0.5;
#pragma unroll
    for (int c = 0; c < 6; ++c) Wv[c] *= 0.5;
    if (ok) {
        a.dedcn[(size_t)i * P + b] = dE;
        double *fo = a.fdir + ((size_t)i * P + b) * 3;
        fo[0] = fx;
        fo[1] = fy;
        fo[2] = fz;
    }
    const int nblk = gridDim.x;   // atom blocks of this pass
    chunk_block_sum(ok ? U : 0.0, lds, a.lgc, bc0, P, a.partE + blk, nblk);
    const int comp[9] = {0, 3, 4, 3, 1, 5, 4, 5, 2};
    for (int c = 0; c < 9; ++c)
        chunk_block_sum(ok ? Wv[comp[c]] : 0.0, lds, a.lgc, bc0, P, a.partW0 + (size_t)c * nblk + blk, 9 * nblk);
}

// ------------------------------------ forces through the coordination ---

template <bool TRI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_d3_cnforce(D3Args a)
{
    __shared__ double t[kTab];
    __shared__ double lds[256];
    load_tab(a, t);
    int i, b;
    const bool ok = d3_lane(a, i, b);
    const SysGeom &g = a.geom[0];
    const int P = a.P, ti = a.types[i] & 3;
    const double *ri = a.posT + ((size_t)i * P + b) * 3;
    const double xi = ri[0], yi = ri[1], zi = ri[2];
    const double dEi = a.dedcn[(size_t)i * P + b];
    const int32_t *uA = a.uniA + (size_t)i * a.capA;
    const uint64_t *mA = a.umA + (size_t)i * a.capA;
    const int32_t *row = a.candA + (size_t)i * a.capA;
    const int n = ok ? a.uendA[(size_t)i * kMaxSpecies + a.S - 1] : 0;
    const double Ri = t[kTRcov + ti], kk = a.k1 * a.k2;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    double Wv[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int e0 = 0; e0 < n; e0 += kD3Batch) {
        uint64_t mm[kD3Batch];
        int w[kD3Batch];
#pragma unroll
        for (int k = 0; k < kD3Batch; ++k) {
            const int e = min(e0 + k, n - 1);
            const uint64_t m = mA[e];
            mm[k] = e0 + k < n ? m : 0ull;
            w[k] = uA[e];
        }
#pragma unroll
        for (int k = 0; k < kD3Batch; ++k) w[k] = row[w[k]];
        double pj[kD3Batch][3], dEj[kD3Batch];
#pragma unroll
        for (int k = 0; k < kD3Batch; ++k) {
            const size_t o = (size_t)(w[k] >> 2) * P + b;
            const double *q = a.posT + o * 3;
            pj[k][0] = q[0];
            pj[k][1] = q[1];
            pj[k][2] = q[2];
            dEj[k] = a.dedcn[o];
        }
#pragma unroll
        for (int k = 0; k < kD3Batch; ++k) {
            double dx, dy, dz;
            d3_pair_vec<TRI>(pj[k], xi, yi, zi, g, dx, dy, dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double r = sqrt(r2);
            const double R = Ri + t[kTRcov + (w[k] & 3)];
            const double ex = exp(a.k1 - kk * R / r);
            const double den = 1.0 + ex;
            // c'(r) / r = -ex k1 k2 R / (r^3 (1 + ex)^2)
            const double on = ((mm[k] >> b) & 1u) ? 1.0 : 0.0;
            const double dc_r = -on * ex * kk * R / (r2 * r * den * den);
            const double sum = (dEi + dEj[k]) * dc_r;
            fx += sum * dx;
            fy += sum * dy;
            fz += sum * dz;
            const double hw = -dEi * dc_r;
            Wv[0] += hw * dx * dx; Wv[1] += hw * dy * dy; Wv[2] += hw * dz * dz;
            Wv[3] += hw * dx * dy; Wv[4] += hw * dx * dz; Wv[5] += hw * dy * dz;
        }
    }
    if (ok) {
        const double *fd = a.fdir + ((size_t)i * P + b) * 3;
        float *fo = a.F + ((size_t)b * a.N + i) * 3;
        const double gx = fx + fd[0], gy = fy + fd[1], gz = fz + fd[2];
        if (a.accumulate) {
            fo[0] = (float)((double)fo[0] + gx);
            fo[1] = (float)((double)fo[1] + gy);
            fo[2] = (float)((double)fo[2] + gz);
        } else {
            fo[0] = (float)gx;
            fo[1] = (float)gy;
            fo[2] = (float)gz;
        }
    }
    const int nblk = gridDim.x;
    const int comp[9] = {0, 3, 4, 3, 1, 5, 4, 5, 2};
    for (int c = 0; c < 9; ++c)
        bead_block_sum(ok ? Wv[comp[c]] : 0.0, lds, P, a.lg, a.partW1 + (size_t)c * nblk + blockIdx.x, 9 * nblk);
}

// One workgroup per (bead, component c): c = 0 energy, 1..9 virial; partial
// sums added in a fixed order.
__global__ __launch_bounds__(256) void k_d3_reduce(const double *__restrict__ partE, const double *__restrict__ partW0,
                                                   const double *__restrict__ partW1, int nblk0, int nblk, int accumulate,
                                                   double *__restrict__ E, double *__restrict__ W)
{
    __shared__ double red[256];
    const int b = blockIdx.x, c = blockIdx.y, t = threadIdx.x;
    double acc = 0.0;
    if (c == 0) {
        for (int k = t; k < nblk0; k += blockDim.x) acc += partE[(size_t)b * nblk0 + k];
    } else {
        // the dispersion pass's partials (nblk0 atom blocks), then the coordination pass's (nblk)
        const size_t o0 = ((size_t)b * 9 + (c - 1)) * nblk0, o = ((size_t)b * 9 + (c - 1)) * nblk;
        for (int k = t; k < nblk0; k += blockDim.x) acc += partW0[o0 + k];
        for (int k = t; k < nblk; k += blockDim.x) acc += partW1[o + k];
    }
    red[t] = acc;
    __syncthreads();
    for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) {
        double *out = c == 0 ? E + b : W + (size_t)b * 9 + (c - 1);
        *out = accumulate ? *out + red[0] : red[0];
    }
}

}  // namespace nep

using namespace nep;

struct nep_d3 {
    nep_model lists;            // cutoff descriptor of the neighbour lists (no weights)
    int S = 0;
    double rc = 0.0, rcn = 0.0;
    double s6 = 0, s8 = 0, a1 = 0, a2 = 0, k1 = 0, k2 = 0, k3 = 0;
    std::vector<double> host;   // the kTab table
    double *dev = nullptr;
    int device = 0;
};

struct nep_d3_ws {
    int P = 0, N = 0, nblk = 0, lg = 0;
    int lgc = 0, nblkc = 0, nchunk = 1;           // the dispersion pass's lanes per atom, atom blocks, bead chunks
    int device = 0;
    double *posT = nullptr;                      // [N][P][3] bead-minor positions
    double *wts = nullptr;                       // [5][N][P] normalised reference weights of each (atom, bead)
    double *cn = nullptr, *dedcn = nullptr, *fdir = nullptr;
    double *partE = nullptr, *partW = nullptr;   // [P][nblk], 2 x [P][9][nblk]
};

extern "C" int32_t nep_d3_load(const char *path, nep_d3 **out)
{
    if (!path || !out) return fail(NEP_ERR_INVALID_ARG, "nep_d3_load: null argument");
    *out = nullptr;
    std::ifstream f(path);
    if (!f) return fail(NEP_ERR_PARAMS_FILE, "nep_d3_load: cannot open %s", path);
    auto word = [&](const char *w) {
        std::string s;
        return (f >> s) && s == w;
    };
    int ver = 0, S = 0;
    double rc = 0, rcn = 0, s6, s8, a1, a2, k1, k2, k3;
    if (!word("nep_d3_params") || !(f >> ver) || ver != 1 || !word("species") || !(f >> S) || !word("cutoff") ||
        !(f >> rc >> rcn) || !word("damping") || !(f >> s6 >> s8 >> a1 >> a2) || !word("constants") ||
        !(f >> k1 >> k2 >> k3))
        return fail(NEP_ERR_PARAMS_FILE, "nep_d3_load: %s: malformed header", path);
    if (S < 1 || S > kMaxSpecies) return fail(NEP_ERR_UNSUPPORTED, "nep_d3_load: %d species (1..4)", S);
    if (!(rc > 0.0) || !(rcn > 0.0) || rcn > rc || !(k3 > 0.0) || !(a1 >= 0.0) || !(a2 >= 0.0) || !(k1 > 0.0) ||
        !(k2 > 0.0))
        return fail(NEP_ERR_PARAMS_FILE, "nep_d3_load: %s: bad cutoffs or constants", path);
    double rcov[kMaxSpecies] = {0}, q[kMaxSpecies] = {0};
    int nref[kMaxSpecies] = {0};
    bool okr = word("rcov");
    for (int s = 0; s < S && okr; ++s) okr = okr && (f >> rcov[s]) && rcov[s] > 0.0;
    okr = okr && word("q");
    for (int s = 0; s < S && okr; ++s) okr = okr && (f >> q[s]) && q[s] > 0.0;
    okr = okr && word("nref");
    for (int s = 0; s < S && okr; ++s) okr = okr && (f >> nref[s]) && nref[s] >= 1 && nref[s] <= kD3Ref;
    if (!okr) return fail(NEP_ERR_PARAMS_FILE, "nep_d3_load: %s: bad species tables", path);
    nep_d3 *d = new (std::nothrow) nep_d3;
    if (!d) return fail(NEP_ERR_NOMEM, "host allocation failed");
    d->host.assign(kTab, 0.0);
    double *t = d->host.data();
    bool ok = word("cnref");
    for (int s = 0; s < S; ++s)
        for (int r = 0; r < kD3Ref; ++r) {
            double v = kD3PadCn;
            if (r < nref[s]) ok = ok && (f >> v);
            t[kTCn + s * kD3Ref + r] = v;
        }
    ok = ok && word("c6ref");
    for (int si = 0; si < S; ++si)
        for (int sj = 0; sj < S; ++sj)
            for (int ra = 0; ra < nref[si]; ++ra)
                for (int rb = 0; rb < nref[sj]; ++rb) {
                    double v = 0.0;
                    ok = ok && (f >> v) && v >= 0.0;
                    t[kTC6 + ((si * kMaxSpecies + sj) * kD3Ref + ra) * kD3Ref + rb] = v;
                }
    if (!ok) {
        delete d;
        return fail(NEP_ERR_PARAMS_FILE, "nep_d3_load: %s: bad reference tables", path);
    }
    for (int s = 0; s < S; ++s) {
        t[kTRcov + s] = rcov[s];
        t[kTQ + s] = q[s];
        t[kTNref + s] = nref[s];
    }
    for (int si = 0; si < S; ++si)
        for (int sj = 0; sj < S; ++sj) {
            const double qq = 3.0 * q[si] * q[sj];
            const double fd = a1 * std::sqrt(qq) + a2;
            const double f2 = fd * fd;
            t[kTF6 + si * 4 + sj] = f2 * f2 * f2;
            t[kTF8 + si * 4 + sj] = f2 * f2 * f2 * f2;
            t[kTQQ + si * 4 + sj] = qq;
        }
    d->S = S;
    d->rc = rc;
    d->rcn = rcn;
    d->s6 = s6; d->s8 = s8; d->a1 = a1; d->a2 = a2;
    d->k1 = k1; d->k2 = k2; d->k3 = k3;
    d->lists.hp = nep_hparams{};
    d->lists.cutoffs_only = true;
    d->lists.hp.n_species = S;
    d->lists.hp.rc_radial = rc;
    d->lists.hp.rc_angular = rcn;
    hipError_t e = hipGetDevice(&d->device);
    if (e == hipSuccess) e = hipMalloc((void **)&d->dev, sizeof(double) * kTab);
    if (e == hipSuccess) e = hipMemcpy(d->dev, t, sizeof(double) * kTab, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (d->dev) (void)hipFree(d->dev);
        delete d;
        return fail(e == hipErrorOutOfMemory ? NEP_ERR_NOMEM : NEP_ERR_HIP, "nep_d3_load: %s", hipGetErrorString(e));
    }
    *out = d;
    return NEP_OK;
}

extern "C" void nep_d3_destroy(nep_d3 *d)
{
    if (!d) return;
    if (d->dev) (void)hipFree(d->dev);
    delete d;
}

extern "C" int32_t nep_d3_list_model(const nep_d3 *d, const nep_model **out)
{
    if (!d || !out) return fail(NEP_ERR_INVALID_ARG, "nep_d3_list_model: null argument");
    *out = &d->lists;
    return NEP_OK;
}

extern "C" int32_t nep_d3_ws_create(const nep_d3 *d, int32_t P, int32_t N, nep_d3_ws **out)
{
    if (!d || !out) return fail(NEP_ERR_INVALID_ARG, "nep_d3_ws_create: null argument");
    if (P < 0 || P > kMaxBeads || N < 0) return fail(NEP_ERR_INVALID_ARG, "nep_d3_ws_create: bad sizes P=%d N=%d", P, N);
    *out = nullptr;
    nep_d3_ws *w = new (std::nothrow) nep_d3_ws;
    if (!w) return fail(NEP_ERR_NOMEM, "host allocation failed");
    w->P = P;
    w->N = N;
    w->lg = lanes_log2(P > 0 ? P : 1);
    w->nblk = div_up(N > 0 ? N : 1, 256 >> w->lg);
    w->lgc = w->lg < 4 ? w->lg : 4;
    w->nblkc = div_up(N > 0 ? N : 1, 256 >> w->lgc);
    w->nchunk = div_up(P > 0 ? P : 1, 1 << w->lgc);
    const size_t PN = (size_t)(P > 0 ? P : 1) * (N > 0 ? N : 1), Pp = P > 0 ? P : 1;
    hipError_t e = hipGetDevice(&w->device);
    if (e == hipSuccess) e = hipMalloc((void **)&w->posT, sizeof(double) * 3 * PN);
    if (e == hipSuccess) e = hipMalloc((void **)&w->wts, sizeof(double) * kD3Ref * PN);
    if (e == hipSuccess) e = hipMalloc((void **)&w->cn, sizeof(double) * PN);
    if (e == hipSuccess) e = hipMalloc((void **)&w->dedcn, sizeof(double) * PN);
    if (e == hipSuccess) e = hipMalloc((void **)&w->fdir, sizeof(double) * 3 * PN);
    if (e == hipSuccess) e = hipMalloc((void **)&w->partE, sizeof(double) * Pp * w->nblkc);
    if (e == hipSuccess) e = hipMalloc((void **)&w->partW, sizeof(double) * 9 * Pp * (w->nblkc + w->nblk));
    if (e != hipSuccess) {
        for (void *p : {(void *)w->posT, (void *)w->wts, (void *)w->cn, (void *)w->dedcn, (void *)w->fdir,
                        (void *)w->partE, (void *)w->partW})
            if (p) (void)hipFree(p);
        delete w;
        return fail(e == hipErrorOutOfMemory ? NEP_ERR_NOMEM : NEP_ERR_HIP, "nep_d3_ws_create: %s",
                    hipGetErrorString(e));
    }
    *out = w;
    return NEP_OK;
}

extern "C" void nep_d3_ws_destroy(nep_d3_ws *w)
{
    if (!w) return;
    for (void *p : {(void *)w->posT, (void *)w->wts, (void *)w->cn, (void *)w->dedcn, (void *)w->fdir,
                    (void *)w->partE, (void *)w->partW})
        if (p) (void)hipFree(p);
    delete w;
}

extern "C" int32_t nep_d3_compute(const nep_d3 *d, nep_nlist *nl, nep_d3_ws *w, const double *pos, const double box[9],
                                  const int32_t *types, int32_t P, int32_t N, double *E, float *F, double *W,
                                  int32_t accumulate, hipStream_t s)
{
    if (!d || !nl || !w || !box) return fail(NEP_ERR_INVALID_ARG, "nep_d3_compute: null argument");
    if (nl->P != P || nl->N != N || w->P != P || w->N != N || nl->S != d->S)
        return fail(NEP_ERR_INVALID_ARG, "nep_d3_compute: P=%d N=%d do not match the list/workspace handles", P, N);
    if (nl->nsys != 1) return fail(NEP_ERR_UNSUPPORTED, "nep_d3_compute: one system per list");
    if (P == 0) return NEP_OK;
    if (!E || !W) return fail(NEP_ERR_INVALID_ARG, "nep_d3_compute: null E or W");
    if (N == 0) {
        if (!accumulate) {
            fill_u32(reinterpret_cast<uint32_t *>(E), 0u, (size_t)P * 2, s);
            fill_u32(reinterpret_cast<uint32_t *>(W), 0u, (size_t)P * 18, s);
        }
        NEP_HIP(hipGetLastError());
        return NEP_OK;
    }
    if (!pos || !types || !F) return fail(NEP_ERR_INVALID_ARG, "nep_d3_compute: null array");
    if (!nl->built) return fail(NEP_ERR_INVALID_ARG, "nep_d3_compute: the neighbour lists were never built");
    if (nl->rc_built[0] != d->rc || nl->rc_built[1] != d->rcn)
        return fail(NEP_ERR_INVALID_ARG, "nep_d3_compute: the lists were built for cutoffs %g/%g, D3 needs %g/%g "
                                         "(build them with the model of nep_d3_list_model)",
                    nl->rc_built[0], nl->rc_built[1], d->rc, d->rcn);
    for (int k = 0; k < 9; ++k)
        if (box[k] != nl->boxL[k]) return fail(NEP_ERR_INVALID_ARG, "nep_d3_compute: box differs from the last build");
    D3Args a{};
    a.posT = w->posT;
    a.types = types;
    a.N = N; a.P = P; a.lg = w->lg; a.lgc = w->lgc; a.S = d->S;
    a.geom = nl->geom;
    a.candA = nl->candA; a.uniR = nl->uniR; a.uendR = nl->uendR; a.uniA = nl->uniA; a.uendA = nl->uendA;
    a.umR = nl->umR; a.umA = nl->umA; a.capR = nl->capR; a.capA = nl->capA;
    a.tab = d->dev;
    a.s6 = d->s6; a.s8 = d->s8; a.k1 = d->k1; a.k2 = d->k2; a.k3 = d->k3;
    a.cn = w->cn; a.dedcn = w->dedcn; a.fdir = w->fdir; a.wts = w->wts;
    a.partE = w->partE; a.partW0 = w->partW; a.partW1 = w->partW + (size_t)9 * P * w->nblkc;
    a.F = F;
    a.accumulate = accumulate ? 1 : 0;
    const dim3 grid(w->nblk), block(256);
    const bool tri = nl->any_tri != 0;
    {
        ProfScope ps_(K_D3_CN, s);
        const int64_t PN = (int64_t)P * N;
        hipLaunchKernelGGL(k_d3_beads_minor, dim3((unsigned)((PN + 255) / 256)), dim3(256), 0, s, pos, w->posT, P, N);
        if (tri) hipLaunchKernelGGL(k_d3_cn<true>, grid, block, 0, s, a);
        else hipLaunchKernelGGL(k_d3_cn<false>, grid, block, 0, s, a);
    }
    {
        ProfScope ps_(K_D3_PAIR, s);
        const dim3 gc(w->nblkc, w->nchunk);
        if (tri) hipLaunchKernelGGL(k_d3_pair<true>, gc, block, 0, s, a);
        else hipLaunchKernelGGL(k_d3_pair<false>, gc, block, 0, s, a);
    }
    {
        ProfScope ps_(K_D3_CNFORCE, s);
        if (tri) hipLaunchKernelGGL(k_d3_cnforce<true>, grid, block, 0, s, a);
        else hipLaunchKernelGGL(k_d3_cnforce<false>, grid, block, 0, s, a);
    }
    {
        ProfScope ps_(K_D3_REDUCE, s);
        hipLaunchKernelGGL(k_d3_reduce, dim3(P, 10), dim3(256), 0, s, w->partE, w->partW,
                           w->partW + (size_t)9 * P * w->nblkc, w->nblkc, w->nblk, a.accumulate, E, W);
    }
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}
