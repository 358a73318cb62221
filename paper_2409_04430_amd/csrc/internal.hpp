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
    nep_hparams hp;
    nep::ParamLayout off;
    std::vector<float> host;   // packed parameters (FP32)
    float *dev = nullptr;      // device copy
    int device = 0;
};

struct nep_nlist {
    int P = 0, N = 0, S = 0;
    int capC = 0;                 // candidate row capacity per atom
    int capR = 0, capA = 0;       // per-bead neighbour capacities per atom (radial, angular)
    int device = 0;
    // Candidate rows are reused across calls while the skin covers the motion.
    double skin = 0.0;            // extra candidate radius, A (0: rebuild every call)
    int built = 0;                // candidate rows valid for box_built
    double box_built[3] = {0.0, 0.0, 0.0};
    // Shared by all beads: ring-polymer centroids and candidate rows.
    double *cen = nullptr;        // [N][3] centroids of this call
    double *cen_ref = nullptr;    // [N][3] centroids at the last rebuild
    int32_t *cand = nullptr;      // [N][capC], entries (j << 2) | species(j), sorted by (species, j)
    int32_t *rowlen = nullptr;    // [N] candidates found (may exceed capC: overflow)
    int32_t *offC = nullptr;      // [N][5], species block starts, [S] = row length
    int32_t *revC = nullptr;      // [N][capC], slot of i in the row of cand[i][k] (-1 if absent)
    // Per bead: compact lists, slot-major ([bead][slot][atom]).
    int32_t *listR = nullptr;     // [P][capR][N] neighbour index j
    int32_t *endR = nullptr;      // [P][4][N] species block ends
    int32_t *listA = nullptr;     // [P][capA][N]
    int32_t *endA = nullptr;      // [P][4][N]
    int32_t *slotA = nullptr;     // [P][capA][N] candidate slot k | reverse slot << 16 (0xffff: none)
    int WC = 0;                   // words of one candidate-row bitmask: ceil(capC / 32)
    uint64_t *maskA = nullptr;    // [P][WC][N] angular hits of word w (low 32 bits) | hits before w << 32
    // Angular pair terms dU_j/dr_ji stored at the receiving atom i's list
    // position s of j: [P][capA][N] xyz + pad.
    float *pairbuf = nullptr;
    float *pos4 = nullptr;        // [P][N][4] packed positions of the last build
    // Centroid cell list (grown on demand): cell_cnt [ncell], cell_start [ncell+1], cell_atoms [N].
    int ncell_alloc = 0;
    int32_t *cell_cnt = nullptr, *cell_start = nullptr, *cell_atoms = nullptr;
    uint32_t *grid = nullptr;     // device-chosen grid record
    uint32_t *status = nullptr;   // [0] flags, [1] max radial neighbours, [2] max angular neighbours,
                                  // [3] max candidates, [4] spread (float bits), [5] rebuilds
};

struct nep_ws {
    int P = 0, N = 0, S = 0, nblk = 0;
    int device = 0;
    int NA1 = 0, KRP = 0;
    float *B = nullptr;        // [P*N][NA1*24] angular adjoints dU_i/dA_nlm
    float *arad = nullptr;     // [P*N][S][KRP] radial adjoints sum_n dU_i/dq_n c_nk
    double *partE = nullptr;   // [P][nblk]
    double *partW = nullptr;   // [2][P][nblk][9] (angular pass, radial pass)
    float *Fang = nullptr;     // [P*N][3] angular part of the forces
    float *pos4 = nullptr;     // [P*N][4] packed positions: offsets in a fine grid cell + cell index bits
    uint32_t *flags = nullptr; // [1]
};

struct pimd_ctx {
    int P = 0, N = 0;
    pimd_params prm;
    int device = 0;
    double *mass = nullptr;    // [N]
    double *consts = nullptr;  // C [P][P] then per mode c1, c2, cq, qv, vq
    std::vector<double> hC;    // host copy of C
};

namespace nep {

// Number of threads per block used by the per-atom kernels.
constexpr int kBlock = 256;

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
void pack_positions(const double *pos, size_t n, const FineGrid &g, float4 *out, hipStream_t s);

__device__ __forceinline__ int wrap_cell(int d, int M)
{
    const int hM = M >> 1;
    return d > hM ? d - M : (d < -hM ? d + M : d);
}

// r_j - r_i from packed positions.
__device__ __forceinline__ void packed_pair(const float4 &pj, const float4 &pi, const int M[3], const float h[3],
                                            float &dx, float &dy, float &dz)
{
    const int wj = __float_as_int(pj.w), wi = __float_as_int(pi.w);
    const int cx = wrap_cell((wj & 1023) - (wi & 1023), M[0]);
    const int cy = wrap_cell(((wj >> 10) & 1023) - ((wi >> 10) & 1023), M[1]);
    const int cz = wrap_cell(((wj >> 20) & 1023) - ((wi >> 20) & 1023), M[2]);
    dx = fmaf(h[0], (float)cx, pj.x - pi.x);
    dy = fmaf(h[1], (float)cy, pj.y - pi.y);
    dz = fmaf(h[2], (float)cz, pj.z - pi.z);
}

// Kernel timing (hipEvents around launches on the caller's stream), off by default.
enum KernelId {
    K_FILL = 0, K_PACK, K_CENTROID, K_GRID, K_CELL_COUNT, K_CELL_SCAN, K_CELL_FILL, K_CELL_SORT, K_CANDIDATES,
    K_SORT_ROWS, K_REVERSE, K_NLIST,
    K_DESCRIPTOR, K_FORCE_ANG, K_FORCE, K_REDUCE, K_TRPMD, K_MODES, K_NUM
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
