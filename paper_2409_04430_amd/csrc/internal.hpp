// Library-internal declarations shared by the HIP translation units of
// libneppimd.so.  Nothing here is part of the C ABI (see include/neppimd.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <string>
#include <vector>

#include "neppimd.h"

namespace nep {

constexpr int kMaxSpecies = 4;
constexpr int kLmax = 4;
constexpr int kNumSH = 24;          // real spherical harmonics l = 1..4
constexpr int kMaxBeads = 64;
// 32-bit words per system in the neighbour list's device grid record (after 16 global words)
constexpr int kDevSysWords = 10;

int fail(int code, const char *fmt, ...);   // records the thread-local message, returns code

#define NEP_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::nep::fail(NEP_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

// Offsets (in floats) of the packed device parameter block of a model.
struct ParamLayout {
    int cR, cA, qs, W0, b0, w1, b1, sh;   // sh: 24 spherical-harmonic normalisations
    int total;
};

}  // namespace nep

struct nep_model {
    nep_hparams hp;            // the kernel shape: the model's own, or the compiled shape it is embedded in
    nep_hparams own;           // the shape of the model file (equal to hp unless embedded)
    bool embedded = false;     // parameters zero-padded into the larger kernel shape hp
    nep::ParamLayout off;
    std::vector<float> host;   // packed parameters (FP32)
    float *dev = nullptr;      // device copy
    int device = 0;
    int mlp = 0;               // NEP_MLP_FP32, NEP_MLP_BF16_MFMA or NEP_MLP_FP32_MFMA (AUTO resolved)
    uint16_t *w0b = nullptr;   // W0 as matrix-core operand fragments (nep::MlpFrag layout), BF16 terms
    size_t w0b_len = 0;        // elements allocated at w0b
    bool cutoffs_only = false; // a cutoff descriptor for neighbour lists (no weights; owned by another handle)
};

namespace nep {
// Fragment layout of the matrix-core network's first-layer weights, per
// species and BF16 term: forward blocks (ht, kc) for ht < HT = 2 HC and
// kc < KC = DP / 32, then adjoint blocks (dt, hc) for dt < DT = DP / 16 and
// hc < HC = ceil(H / 32); 512 entries (64 lanes x 8) per block.  DP = 32
// for D <= 32, else 64.
struct MlpFrag {
    int DP, KC, DT, HC, HT, wt;
    int fwd_blocks, adj_blocks;
    int term_stride, species_stride;   // entries
};
__host__ __device__ inline MlpFrag mlp_frag_layout(int D, int H, int wt)
{
    MlpFrag f;
    f.DP = D <= 32 ? 32 : 64;
    f.KC = f.DP / 32;
    f.DT = f.DP / 16;
    f.HC = (H + 31) / 32;
    f.HT = 2 * f.HC;
    f.wt = wt;
    f.fwd_blocks = f.HT * f.KC;
    f.adj_blocks = f.DT * f.HC;
    f.term_stride = (f.fwd_blocks + f.adj_blocks) * 512;
    f.species_stride = wt * f.term_stride;
    return f;
}
}  // namespace nep

namespace nep {
// Geometry of one system of a batch (device copy in the list handle).
struct SysGeom {
    double L[3], invL[3];     // orthorhombic box edges (triclinic: the diagonal of H, unused)
    double hd[3], Minv[3];    // fine grid spacing and M / L (packing, orthorhombic)
    float h[3];               // fine grid spacing (FP32, pair vectors, orthorhombic)
    int M[3];                 // fine grid cells per axis (along the cell's edge vectors)
    int nc_cap[3];            // cell-list allocation bound per axis
    int cell_base;            // first global cell of the system
    int atom0, atom1;         // atom range [atom0, atom1)
    int tri;                  // 1: general (triclinic) cell, fractional-coordinate geometry
    double H[9], G[9];        // edge vectors as rows (r = s H) and G = H^-1 (s = r G)
    double w[3];              // distance between opposite faces, per axis
    double GM[9];             // G with column d scaled by M[d] (fine-grid coordinates)
    double hvd[9];            // fine-grid step vectors H_d / M_d (rows, FP64, packing)
    float hv[9];              // the same in FP32 (pair vectors)
};

// Geometry of one periodic cell given by its edge vectors as rows of box[9]:
// inverse, face distances, volume, whether it is orthorhombic.  False for a
// singular, left-handed or non-finite cell.
struct CellInfo {
    double H[9], G[9], w[3], len[3], vol;
    int tri;
};
bool cell_info(const double box[9], CellInfo &c);
}  // namespace nep

// Validates a batch partition: offsets [nsys+1], non-decreasing from 0
// (NEP_OK, or the error code after fail()).
int32_t check_offsets(int32_t nsys, const int32_t *off, const char *who);

struct nep_nlist {
    int P = 0, N = 0, S = 0;
    int capR = 0, capA = 0;       // candidate row capacities per atom (radial, angular radius)
    int device = 0;
    // Batch of independent systems: atoms [off[s], off[s+1]) form system s.
    int nsys = 1;
    std::vector<int> off;         // host [nsys+1]
    std::vector<double> boxL;     // host [nsys][9] cells of the last build (0: none yet)
    float margin = 0.0f;          // FP32 pre-test margin of the last build's geometry
    int any_tri = 0;              // some system of the last build has a general (triclinic) cell
    nep::SysGeom *geom = nullptr; // [nsys]
    int32_t *atom_sys = nullptr;  // [N]
    int32_t *cell_sys = nullptr;  // [ncell_alloc]
    // Candidate rows are reused across calls while the skin covers the motion.
    double skin = 0.0;            // extra candidate radius, A (0: rebuild every call)
    int built = 0;                // candidate rows valid for box_built
    double box_built[3] = {0.0, 0.0, 0.0};
    // Shared by all beads: ring-polymer centroids and candidate rows.
    double *cen = nullptr;        // [N][3] centroids of this call
    float *spr = nullptr;         // [N] largest bead distance from the centroid (rounded up) of this call
    float *cmax = nullptr;        // [ceil(kCenLanes N / kBlock)][2] per-workgroup maxima of the centroid kernel
    double *cen_ref = nullptr;    // [N][3] centroids at the last rebuild
    int32_t *candR = nullptr;     // [N][capR] entries (j << 2) | species(j), sorted by (species, j)
    int32_t *candRs = nullptr;    // [N][capR] the same rows unsorted, as the candidate search leaves them
    int32_t *candAs = nullptr;    // [N][capA] the angular rows unsorted
    int32_t *lenR = nullptr;      // [N] candidates found (may exceed capR: overflow)
    int32_t *offR = nullptr;      // [N][5] species block starts, [S] = row length
    int32_t *candA = nullptr;     // [N][capA] the same for the angular radius
    int32_t *lenA = nullptr;      // [N]
    int32_t *offA = nullptr;      // [N][5]
    int32_t *revA = nullptr;      // [N][capA] slot of i in the angular row of candA[i][k] (-1 if absent)
    // Per call: slots of the candidates inside the cutoff for at least one
    // bead (row order), with per-species block ends.
    int32_t *uniR = nullptr;      // [N][capR] atom indices j
    uint64_t *umR = nullptr;      // [N][capR] bit b: inside the radial cutoff in bead b
    int32_t *uendR = nullptr;     // [N][4]
    int32_t *uniA = nullptr;      // [N][capA] angular slots k
    uint64_t *umA = nullptr;      // [N][capA] bit b: inside the angular cutoff in bead b
    int32_t *uendA = nullptr;     // [N][4]
    // Angular pair terms dU_j/dr_ji at the receiving atom i's angular slot of j: [N][capA][P] xyz + pad.
    float *pairbuf = nullptr;
    float *pos4 = nullptr;        // [N][P][4] packed positions of the last build (bead-minor)
    double *posT = nullptr;       // [N][P][3] bead-minor FP64 positions (pair histograms; allocated on first use)
    // Centroid cell list (grown on demand): cell_cnt [ncell], cell_start [ncell+1], cell_atoms [N].
    int ncell_alloc = 0, ncell_total = 0;
    int32_t *cell_cnt = nullptr, *cell_start = nullptr, *cell_atoms = nullptr;
    double rc_built[2] = {0.0, 0.0};   // cutoffs (radial, angular) of the last neighbor_build
    uint32_t *grid = nullptr;     // device-chosen grid record: 16 global words + kDevSysWords per system
    uint32_t *status = nullptr;   // [0] flags, [1] max radial union, [2] max angular union,
                                  // [3] max radial candidates, [4] spread (float bits), [5] rebuilds,
                                  // [6] max angular candidates
};

// Per-(system, bead) energy and virial sums over the force kernels'
// per-workgroup partials: launched by nep_compute itself, or left pending by
// a deferred call and carried out inside the next integrator launch.
struct PendingReduce {
    const double *partE = nullptr, *partWa = nullptr, *partWr = nullptr;
    const int32_t *sys_tile0 = nullptr;
    int P = 0, nblk = 0;
    int nout = 0;              // outputs: systems x P x 10 (energy, 9 virial entries); 0 = nothing pending
    double *E = nullptr, *W = nullptr;
};

struct nep_ws {
    int P = 0, N = 0, S = 0, nblk = 0;
    int device = 0;
    int NA1 = 0;
    int nsys = 1;
    std::vector<int> off;      // host [nsys+1]
    // Tiles: each workgroup of the NEP kernels takes up to 4 * 64 / G atoms
    // (all their beads) of one system.
    int wpb = 4;                    // wavefronts per workgroup (tile shape), set by nep_ws_set_tile / nep_autotune
    int net_global = 0;             // 1: FP32 network weights read from global memory even where they fit LDS
    int nblk_cap = 0;               // tile capacity (the count for one wavefront per workgroup)
    int32_t *tile_atom0 = nullptr, *tile_atom1 = nullptr, *tile_sys = nullptr;   // [nblk_cap]
    int32_t *sys_tile0 = nullptr;   // [nsys + 1]
    float *B = nullptr;        // angular adjoints dU_i/dA_nlm times c_m (the harmonic's normalisation), one
                               // row of NA1*24 per lane of a launch, wavefront-interleaved (adj_rows)
    size_t B_waves = 0;        // wavefronts whose rows B holds
    float *Gad = nullptr;      // descriptor adjoints dU/dq_nl (and the four-body ones) per lane, for parked
                               // angular sums (the angular force forms B from both), wavefront-interleaved
    float *arad = nullptr;     // [N][S][P][12] radial adjoints sum_n dU_i/dq_n c_nk (9 used)
    double *partE = nullptr;   // [P][nblk] per-workgroup partial energies (bead-major)
    double *partW = nullptr;   // angular pass [P][9][nblk], then radial pass [P][9][nblk] (room for nblk_cap)
    float *Fang = nullptr;     // [N][P][3] angular part of the forces
    uint32_t *flags = nullptr; // [1]
    int defer_next = 0;        // the next nep_compute leaves its E/W sums pending (nep_ws_defer_reduce)
    PendingReduce pending;     // sums of a deferred call, until an integrator launch completes them
};

struct pimd_ctx {
    int P = 0, N = 0;
    pimd_params prm;
    int device = 0;
    double *mass = nullptr;    // [N]
    double *consts = nullptr;  // C [P][P] then per mode c1, c2, cq, qv, vq
    std::vector<double> hC;    // host copy of C
    double *obs_part = nullptr;  // [obs_blocks][9] partial sums of the observables
    int obs_blocks = 0;
};

namespace nep {

// Number of threads per block used by the per-atom kernels.
constexpr int kBlock = 256;
// Lanes per atom of the centroid kernel (a power of two dividing 64).
constexpr int kCenLanes = 16;

inline int div_up(int a, int b) { return (a + b - 1) / b; }

// (bead, tile) of this workgroup for a grid (tiles, beads).  Workgroups are
// handed to the 8 XCDs round-robin in linear order; when the grid size is a
// multiple of 8 the linear id is permuted so that each XCD receives one
// contiguous run of (bead, tile) pairs, i.e. works through a few beads at a
// time and their gathers stay in its own L2.
__device__ __forceinline__ void bead_tile(int &bead, int &tile)
{
    const int nt = gridDim.x;
    const int total = nt * gridDim.y;
    int lin = blockIdx.y * nt + blockIdx.x;
    if ((total & 7) == 0) lin = (lin & 7) * (total >> 3) + (lin >> 3);
    bead = lin / nt;
    tile = lin - bead * nt;
}

// Output o of a pending reduction, o = (system * P + bead) * 10 + c (c = 0
// energy, 1..9 virial), on one wavefront (lane t): lane t adds the system's
// workgroup partials t, t + 64, ... in order (four loads in flight), then a
// fixed butterfly over the lanes, so the result is bitwise reproducible
// whichever launch carries it.
__device__ __forceinline__ void reduce_output(const PendingReduce &r, int o, int t)
{
    const int sb = o / 10, c = o - sb * 10, sy = sb / r.P, b = sb - sy * r.P;
    const int k0 = r.sys_tile0[sy], k1 = r.sys_tile0[sy + 1];
    const double *pa = c == 0 ? r.partE + (size_t)b * r.nblk : r.partWa + ((size_t)b * 9 + (c - 1)) * r.nblk;
    const double *pr = c == 0 ? nullptr : r.partWr + ((size_t)b * 9 + (c - 1)) * r.nblk;
    double acc = 0.0;
    int k = k0 + t;
    for (; k + 192 < k1; k += 256) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = pa[k + 64 * u] + (pr ? pr[k + 64 * u] : 0.0);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += v[u];
    }
    for (; k < k1; k += 64) acc += pa[k] + (pr ? pr[k] : 0.0);
    for (int s = 32; s > 0; s >>= 1) acc += __shfl_xor(acc, s);
    if (t == 0) {
        if (c == 0) r.E[sb] = acc;
        else r.W[(size_t)sb * 9 + (c - 1)] = acc;
    }
}

// Orthorhombic edge lengths from a row-vector cell; false if not orthorhombic.
bool box_lengths(const double box[9], double L[3]);

// Packed positions: per axis a fine grid of M cells of width h = L / M; a
// bead position is stored as FP32 offsets inside its cell plus the three
// cell indices (10 bits each) in the w word.  h <= 1 A and h <= (L/2 - rc)/2,
// so every pair closer than rc takes its minimum image from the integer cell
// difference (exact = 1); the pair vector is then accurate to about 1e-6 A.
struct FineGrid {
    int M[3];
    float h[3];
    double Minv[3], hd[3];
    int exact;
};
FineGrid fine_grid(const double L[3], double rc);
// The same for a general cell: M_d cells along edge vector d with
// w_d / M_d <= (w_d / 2 - rc) / 2 and |H_d| / M_d <= 1 A (w_d the face
// distance); for an orthorhombic cell it equals fine_grid(L, rc).
FineGrid fine_grid_cell(const CellInfo &c, double rc);


// One packed position: per axis the fine cell c = floor(x / h) mod M
// (10 bits per axis in w; unwrapped coordinates allowed) and the FP32
// offset x - floor(x / h) h inside it; a non-finite coordinate gives a NaN
// offset.
__device__ __forceinline__ float4 pack_one_tri(const double *x3, const SysGeom &g)
{
    // fine-grid coordinates u_d = (x G)_d M_d, cell floor(u_d) mod M_d, and the
    // Cartesian offset from the cell corner sum_d floor(u_d) H_d / M_d
    double fl[3];
    bool fin = isfinite(x3[0]) && isfinite(x3[1]) && isfinite(x3[2]);
    int bits = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double u = x3[0] * g.GM[d] + x3[1] * g.GM[3 + d] + x3[2] * g.GM[6 + d];
        double f = floor(u);
        if (!isfinite(f)) f = 0.0;
        fl[d] = f;
        int ci = (int)(f - (double)g.M[d] * floor(f / (double)g.M[d]));
        ci = ci < 0 ? 0 : (ci >= g.M[d] ? g.M[d] - 1 : ci);
        bits |= ci << (10 * d);
    }
    float o[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        o[a] = (float)(x3[a] - (fl[0] * g.hvd[a] + fl[1] * g.hvd[3 + a] + fl[2] * g.hvd[6 + a]));
    if (!fin) o[0] = __int_as_float(0x7fc00000);
    return make_float4(o[0], o[1], o[2], __int_as_float(bits));
}

__device__ __forceinline__ float4 pack_one(const double *x3, const SysGeom &g)
{
    if (g.tri) return pack_one_tri(x3, g);
    float o[3];
    int bits = 0;
    bool fin = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double x = x3[d];
        fin = fin && isfinite(x);
        double fl = floor(x * g.Minv[d]);
        if (!isfinite(fl)) fl = 0.0;
        o[d] = (float)(x - fl * g.hd[d]);
        int ci = (int)(fl - (double)g.M[d] * floor(fl / (double)g.M[d]));
        ci = ci < 0 ? 0 : (ci >= g.M[d] ? g.M[d] - 1 : ci);
        bits |= ci << (10 * d);
    }
    if (!fin) o[0] = __int_as_float(0x7fc00000);
    return make_float4(o[0], o[1], o[2], __int_as_float(bits));
}

__device__ __forceinline__ int wrap_cell(int d, int M)
{
    const int hM = M >> 1;
    return d > hM ? d - M : (d < -hM ? d + M : d);
}

// Minimum-image cell difference d - M rint(d / M) in FP32 (d, M small
// integers, so exact).  It equals wrap_cell except, for even M, at
// |d| = M / 2, where either image lies farther than L/2 - h > rc.
__device__ __forceinline__ float wrap_cell_f(int d, float Mf, float Minv)
{
    const float f = (float)d;
    return fmaf(-Mf, rintf(f * Minv), f);
}

// r_j - r_i from packed positions.
__device__ __forceinline__ void packed_pair(const float4 &pj, const float4 &pi, const int M[3], const float h[3],
                                            float &dx, float &dy, float &dz)
{
    const int wj = __float_as_int(pj.w), wi = __float_as_int(pi.w);
    const float cx = wrap_cell_f((wj & 1023) - (wi & 1023), (float)M[0], 1.0f / (float)M[0]);
    const float cy = wrap_cell_f(((wj >> 10) & 1023) - ((wi >> 10) & 1023), (float)M[1], 1.0f / (float)M[1]);
    const float cz = wrap_cell_f(((wj >> 20) & 1023) - ((wi >> 20) & 1023), (float)M[2], 1.0f / (float)M[2]);
    dx = fmaf(h[0], cx, pj.x - pi.x);
    dy = fmaf(h[1], cy, pj.y - pi.y);
    dz = fmaf(h[2], cz, pj.z - pi.z);
}

// r_j - r_i from packed positions in a general cell: the offset difference
// plus sum_d wrap(c_j,d - c_i,d) H_d / M_d.
__device__ __forceinline__ void packed_pair_tri(const float4 &pj, const float4 &pi, const int M[3], const float hv[9],
                                                float &dx, float &dy, float &dz)
{
    const int wj = __float_as_int(pj.w), wi = __float_as_int(pi.w);
    const float c0 = wrap_cell_f((wj & 1023) - (wi & 1023), (float)M[0], 1.0f / (float)M[0]);
    const float c1 = wrap_cell_f(((wj >> 10) & 1023) - ((wi >> 10) & 1023), (float)M[1], 1.0f / (float)M[1]);
    const float c2 = wrap_cell_f(((wj >> 20) & 1023) - ((wi >> 20) & 1023), (float)M[2], 1.0f / (float)M[2]);
    dx = fmaf(hv[6], c2, fmaf(hv[3], c1, fmaf(hv[0], c0, pj.x - pi.x)));
    dy = fmaf(hv[7], c2, fmaf(hv[4], c1, fmaf(hv[1], c0, pj.y - pi.y)));
    dz = fmaf(hv[8], c2, fmaf(hv[5], c1, fmaf(hv[2], c0, pj.z - pi.z)));
}

// Exact FP64 minimum-image squared distance in a general cell, the literal
// expression (no contraction; every step antisymmetric in i and j)
//   s_c = (d_x G_xc + d_y G_yc) + d_z G_zc;  f_c = s_c - rint(s_c);
//   e_a = (f_0 H_0a + f_1 H_1a) + f_2 H_2a;  (e_x^2 + e_y^2) + e_z^2
__device__ __forceinline__ double mic_r2_exact_tri(const double *ri, const double *rj, const double H[9],
                                                   const double G[9])
{
#pragma clang fp contract(off)
    const double d[3] = {rj[0] - ri[0], rj[1] - ri[1], rj[2] - ri[2]};
    double f[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double sc = (d[0] * G[c] + d[1] * G[3 + c]) + d[2] * G[6 + c];
        f[c] = sc - rint(sc);
    }
    double e2[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double e = (f[0] * H[a] + f[1] * H[3 + a]) + f[2] * H[6 + a];
        e2[a] = e * e;
    }
    return (e2[0] + e2[1]) + e2[2];
}

// Nearest-image vector in place (FP64; cell-list and centroid distances).
// tri: the cell is a general one (g.tri; a compile-time false removes the
// general branch from orthorhombic-only kernels).  In a general cell the
// fractional reduction f - rint(f) gives a vector e; every other image is
// e + v with v a non-zero lattice vector, |v| >= w_min (the smallest face
// distance), so e is the nearest image when |e| < w_min / 2.  Otherwise the
// 26 neighbouring images are compared as well, which finds the nearest one
// whenever it is shorter than w_min (its fractional coordinates then differ
// from those of e by at most 1 per axis).  Callers need distances below
// w_min only (candidate radii; the list build flags larger ones).
__device__ __forceinline__ void mic_vec(double d[3], const SysGeom &g, bool tri)
{
    if (!tri) {
#pragma unroll
        for (int a = 0; a < 3; ++a) d[a] -= g.L[a] * rint(d[a] * g.invL[a]);
        return;
    }
    double f[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double sc = d[0] * g.G[c] + d[1] * g.G[3 + c] + d[2] * g.G[6 + c];
        f[c] = sc - rint(sc);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) d[a] = f[0] * g.H[a] + f[1] * g.H[3 + a] + f[2] * g.H[6 + a];
    const double wmin = fmin(g.w[0], fmin(g.w[1], g.w[2]));
    double best = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(best >= 0.25 * wmin * wmin)) return;   // nearest already (or non-finite)
    double e0 = d[0], e1 = d[1], e2 = d[2];
    for (int n0 = -1; n0 <= 1; ++n0)
        for (int n1 = -1; n1 <= 1; ++n1)
            for (int n2 = -1; n2 <= 1; ++n2) {
                const double x = d[0] + n0 * g.H[0] + n1 * g.H[3] + n2 * g.H[6];
                const double y = d[1] + n0 * g.H[1] + n1 * g.H[4] + n2 * g.H[7];
                const double z = d[2] + n0 * g.H[2] + n1 * g.H[5] + n2 * g.H[8];
                const double r2 = x * x + y * y + z * z;
                if (r2 < best) {
                    best = r2;
                    e0 = x; e1 = y; e2 = z;
                }
            }
    d[0] = e0; d[1] = e1; d[2] = e2;
}

// Fractional coordinate d of a point (cell lists).
__device__ __forceinline__ double frac_coord(const double x[3], const SysGeom &g, int d)
{
    return g.tri ? x[0] * g.G[d] + x[1] * g.G[3 + d] + x[2] * g.G[6 + d] : x[d] * g.invL[d];
}

// Exact FP64 minimum-image squared distance, the literal expression
//   d = r_j - r_i;  d -= L rint(d / L);  (dx*dx + dy*dy) + dz*dz
// without contraction.  The division is replaced by a multiply with 1/L
// whenever that provably gives the same integer (d/L farther than 1e-9 from
// a half-integer and |d/L| < 2^20).  Every step is exactly antisymmetric in
// i and j, so the test is symmetric.
__device__ __forceinline__ double mic_r2_exact(const double *ri, const double *rj, const double L[3],
                                               const double invL[3])
{
#pragma clang fp contract(off)
    double e2[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double d = rj[a] - ri[a];
        const double t = d * invL[a];
        double k = rint(t);
        const double off = t - k;
        if (!(fabs(off) < 0.499999999) || !(fabs(t) < 1048576.0)) k = rint(d / L[a]);
        const double sft = L[a] * k;
        const double e = d - sft;
        e2[a] = e * e;
    }
    return (e2[0] + e2[1]) + e2[2];
}

// Cutoff decision for a pair of one bead.  It is taken on the packed FP32
// squared distance when that lies farther than `margin` from rc^2 (far above
// the packed error bound, so the answer equals the FP64 one) and by the FP64
// test otherwise.  pos points to the bead's [N][3] FP64 positions.
struct CutTest {
    float rc2f, margin;
    double rc2;
};
__device__ __forceinline__ bool pair_within(float r2f, const CutTest &c, const double *__restrict__ pos, int i, int j,
                                            const SysGeom &g, bool tri)
{
    if (fabsf(r2f - c.rc2f) > c.margin) return r2f < c.rc2f;
    const double ri[3] = {pos[3 * (size_t)i], pos[3 * (size_t)i + 1], pos[3 * (size_t)i + 2]};
    const double rj[3] = {pos[3 * (size_t)j], pos[3 * (size_t)j + 1], pos[3 * (size_t)j + 2]};
    return (tri ? mic_r2_exact_tri(ri, rj, g.H, g.G) : mic_r2_exact(ri, rj, g.L, g.invL)) < c.rc2;
}

// r_j - r_i from packed positions of the system's fine grid (tri as for mic_vec).
__device__ __forceinline__ void packed_pair_g(const float4 &pj, const float4 &pi, const SysGeom &g, bool tri,
                                              float &dx, float &dy, float &dz)
{
    if (tri) packed_pair_tri(pj, pi, g.M, g.hv, dx, dy, dz);
    else packed_pair(pj, pi, g.M, g.h, dx, dy, dz);
}

// Lanes per atom: the beads of one atom occupy G = 2^lg consecutive lanes of
// a wavefront (G >= P, lanes with bead >= P idle), 64 / G atoms per wave.
inline int lanes_log2(int P)
{
    int lg = 0;
    while ((1 << lg) < P) ++lg;
    return lg;
}

// Checks the boxes [nsys][9] of a batch against the model's cutoffs and
// refreshes the per-system geometry of the list handle (synchronous upload
// when a box changed).  margin: decision margin of the FP32 pre-test, about
// 30x the packed error bound.
int32_t update_geometry(const nep_model *m, nep_nlist *nl, const double *boxes, bool &changed, float &margin,
                        bool &tri_changed);

// Kernel timing (hipEvents around launches on the caller's stream), off by default.
enum KernelId {
    K_FILL = 0, K_CENTROID, K_CANDIDATES, K_NLIST, K_MATERIALIZE,
    K_DESCRIPTOR, K_FORCE_ANG, K_FORCE, K_REDUCE, K_TRPMD, K_MODES, K_OBS, K_BARO, K_RDF, K_D3_CN, K_D3_PAIR,
    K_D3_CNFORCE, K_D3_REDUCE, K_NUM
};
struct ProfScope {
    int id;
    hipStream_t s;
    hipEvent_t e0 = nullptr;
    ProfScope(int kid, hipStream_t stream);
    ~ProfScope();
};

// Zero-fill on a stream by a kernel (capturable into graphs).
void fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
void fill_i32(int32_t *p, int32_t v, size_t n, hipStream_t s);

}  // namespace nep
