// Arguments, lane mapping and reductions shared by the NEP force kernels
// and the training kernels: one workgroup per tile (an atom range of one
// system), the P beads of an atom in adjacent lanes.
#pragma once

#include "internal.hpp"
#include "nep_math.hpp"

namespace nep {

constexpr int kRadPad = 12;   // padded length of a radial adjoint row (float4 access)

struct NepArgs {
    const float4 *p4;    // [N][P] packed positions (bead-minor)
    const double *pos;   // [P][N][3] FP64 positions (exact test near the cutoff)
    const int32_t *types;
    int N, S, H, P, lg;  // lg: log2 of the lanes per atom
    const SysGeom *geom; // per system: fine grid of the packed positions
    const int32_t *tile_atom0, *tile_atom1, *tile_sys;   // per workgroup: atom range and system
    float rcRinv, rcAinv;
    float kappa4;
    // candidate rows and union lists of the neighbour handle
    const int32_t *candA, *revA, *uniR, *uendR, *uniA, *uendA;
    const uint64_t *umR, *umA;   // bead masks of the union entries
    int capR, capA;
    float4 *pairbuf;     // [N][capA][P] dU_j/dr_ji at the receiving atom's angular slot of j
    // workspace
    float *B;            // adjoint rows B_nlm c_m, or the parked sums A_nlm, per lane (adj_rows)
    float *Gad;          // with parked sums: dU/dq_nl per lane, l = 1..4 per float4, then kappa dU/dq4_n (adj_rows)
    float *arad;         // [N][S][P][kRadPad] radial adjoints a_k (k < 9) and, in slot 9, their sum over k >= 1
    float *Fang;         // [N][P][3]
    double *partE, *partWa, *partWr;   // [P][blocks], [P][9][blocks]
    uint32_t *flags;
    // outputs
    float *F;
    float *Eatom;
    float *Watom;
    // parameter offsets
    int oR, oA, oq, oW0, ob0, ow1, ob1, osh;
    const uint16_t *w0b; // BF16 first-layer weights of the matrix-core network ([S][2][32][32])
};

// Lane -> (atom, bead): the beads of one atom occupy 2^lg adjacent lanes;
// a workgroup takes one tile (an atom range of one system).  M and h are
// the fine grid of the tile's system (wave-uniform).
struct LaneMap {
    int i, b;        // atom and bead (clamped into range for idle lanes)
    bool valid;      // a real (atom, bead)
    int M[3];
    float h[3];
    int tri;         // general cell: pair vectors through the step vectors hv
    float hv[9];
};
__device__ __forceinline__ LaneMap lane_map(const NepArgs &a)
{
    const int lane = threadIdx.x & 63;
    const int a0 = a.tile_atom0[blockIdx.x], a1 = a.tile_atom1[blockIdx.x];
    const int ia = a0 + (threadIdx.x >> 6) * (64 >> a.lg) + (lane >> a.lg);
    const int b = lane & ((1 << a.lg) - 1);
    LaneMap m;
    m.valid = ia < a1 && b < a.P;
    m.i = ia < a1 ? ia : a1 - 1;
    m.b = b < a.P ? b : a.P - 1;
    const SysGeom &g = a.geom[a.tile_sys[blockIdx.x]];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        m.M[d] = g.M[d];
        m.h[d] = g.h[d];
    }
    m.tri = g.tri;
#pragma unroll
    for (int k = 0; k < 9; ++k) m.hv[k] = g.hv[k];
    return m;
}

// Start and end of species block t in a union list.
__device__ __forceinline__ void block_range(const int32_t *uend, int i, int t, int &s0, int &s1)
{
    s0 = t ? uend[(size_t)i * kMaxSpecies + t - 1] : 0;
    s1 = uend[(size_t)i * kMaxSpecies + t];
}

// Pair vector r_j - r_i from packed positions (see FineGrid).
// TRI: the launch covers general (triclinic) cells, each lane's system
// choosing its form (a uniform branch); orthorhombic-only launches take
// TRI = false and carry no general-cell code.
template <bool TRI>
__device__ __forceinline__ void pair_vec(const float4 &pj, const float4 &pi, const LaneMap &lm, float &dx, float &dy,
                                         float &dz)
{
    if (TRI && lm.tri) packed_pair_tri(pj, pi, lm.M, lm.hv, dx, dy, dz);
    else packed_pair(pj, pi, lm.M, lm.h, dx, dy, dz);
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Per-bead sums over the atoms of a block in a fixed order: thread b < P
// adds the values of the lanes of bead b and writes out[b * stride].
__device__ __forceinline__ void bead_block_sum(double v, double *lds, int P, int lg, double *out, int stride)
{
    lds[threadIdx.x] = v;
    __syncthreads();
    if ((int)threadIdx.x < P) {
        double s = 0.0;
        for (int x = threadIdx.x; x < (int)blockDim.x; x += 1 << lg) s += lds[x];
        out[(size_t)threadIdx.x * stride] = s;
    }
    __syncthreads();
}

// Adjoint rows B_i (and the angular sums parked in them) are stored
// wavefront-interleaved: float4 q of the row of lane L of the launch's
// wavefront w (w = workgroup index * wavefronts per workgroup + wavefront in
// the workgroup) sits at float4 index (w * NA1 * 6 + q) * 64 + L, so that
// one store or load of the wavefront's q-th float4 covers 1 KiB
// contiguously (a row per lane would put every lane of it on another cache
// line).  The kernels that write and read the rows share one launch shape,
// the workspace's tile table; the array holds a row for every lane of a
// launch, idle lanes included (never written; zero from creation).  The
// accesses go through a buffer resource over the wavefront's rows: the
// lane's byte offset in a vector register, the float4 index as a scalar
// offset, so that no per-float4 64-bit address is kept in registers (the
// rows of one lane span more than the immediate offset of a global access).
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
constexpr int kBufWord3 = 0x00020000;   // buffer resource word 3 of gfx9-family chips: 32-bit data format

// nq: float4 entries per lane.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t adj_rows(float *B, int nq)
{
    const uint32_t w = __builtin_amdgcn_readfirstlane((uint32_t)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
    const int bytes = nq * 64 * 16;
    return __builtin_amdgcn_make_buffer_rsrc(B + (size_t)w * (bytes / 4), (short)0, bytes, kBufWord3);
}

// Whether the descriptor kernel parks the angular sums A in the adjoint
// rows (the matrix-core network needs their registers, and wide angular
// sets do not fit beside the network): then it stores A there and the
// descriptor adjoints dU/dq_nl in Gad, and the angular force forms B from
// both; otherwise the descriptor stores B itself.
constexpr bool adj_parked(bool matrix_core_net, int NA1) { return matrix_core_net || NA1 > 5; }

// float4 entries per lane of Gad: one per radial function (l = 1..4), then
// the four-body adjoints four to an entry.
constexpr int gad_q(int NA1, bool four) { return NA1 + (four ? (NA1 + 3) / 4 : 0); }

__device__ __forceinline__ void adj_store(__amdgpu_buffer_rsrc_t r, int q, float4 v)
{
    const u32x4_t u = {__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z), __float_as_uint(v.w)};
    __builtin_amdgcn_raw_buffer_store_b128(u, r, (int)(threadIdx.x & 63) * 16, q * 1024, 0);
}

__device__ __forceinline__ float4 adj_load(__amdgpu_buffer_rsrc_t r, int q)
{
    const u32x4_t u = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(threadIdx.x & 63) * 16, q * 1024, 0);
    return make_float4(__uint_as_float(u.x), __uint_as_float(u.y), __uint_as_float(u.z), __uint_as_float(u.w));
}

constexpr int kBatch = 4;    // neighbours whose index and position are loaded together
constexpr int kBatchR = 8;   // the same for the descriptor's radial loop

// Hide a uniform pointer from loop-invariant code motion, so that the model
// coefficients it addresses are re-read through the scalar cache inside a
// neighbour loop instead of being hoisted into (scarce) vector registers.
// Pins a gathered value at this point: without it the compiler sinks a
// load that only a masked branch uses into that branch, where it waits for
// the loads issued before it, so a batch's gathers run one after another.
__device__ __forceinline__ void keep(float4 &v)
{
    asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w));
}

// Model coefficients (read-only during a launch) through the constant
// address space: loads at a wave-uniform address become scalar loads, which
// do not wait on the vector gathers in flight.
typedef const float __attribute__((address_space(4))) *cf32p;

// A uniform coefficient pointer re-materialised in SGPRs at its point of use
// (keeps the compiler from hoisting every coefficient out of a loop into
// VGPRs), returned in the constant address space.
__device__ __forceinline__ cf32p launder(const float *p)
{
    asm volatile("" : "+s"(p));
    return (cf32p)p;
}

}  // namespace nep
