// Per-bead neighbour sets through ring-polymer centroids (orthorhombic box).
//
// Pairs are accepted by the literal FP64 minimum-image test
//   d = r_j - r_i;  d -= L * rint(d / L)  (per axis);  (dx*dx + dy*dy) + dz*dz < rc*rc
// without contraction, so the sets equal those of a brute-force search over
// all pairs of a bead.  The division is replaced by a multiply with 1/L
// whenever that provably gives the same integer (t = d/L farther than 1e-9
// from a half-integer and |t| < 2^20); otherwise the division runs.  The
// test is symmetric in i and j (every step of it is exactly antisymmetric),
// so j is a neighbour of i exactly when i is one of j.
//
// Candidates: the P beads of an atom stay within D of their centroid, so a
// bead pair closer than rc has centroids closer than rc + 2D.  One cell-list
// search over the N centroids gives each atom two candidate rows (radius
// rc_radial + 2D and rc_angular + 2D, plus the skin when rows are reused),
// sorted by (species, index), and for the angular row the slot at which the
// atom sits in each candidate's own row.  Every call then keeps, per atom,
// the slots whose candidate is inside the cutoff for at least one bead (the
// union lists the force kernels walk, one atom's beads in adjacent lanes).
// D, the cell grid and the radii are computed on the device in the same
// call, so the launch sequence needs no host round trip.
//
// Kernels per call: pack positions -> centroids, D and drift -> rebuild
// decision and grid; on a rebuild: count atoms per cell -> scan -> scatter
// -> order each cell -> candidate rows (a workgroup per cell, stencil
// centroids staged in LDS) -> sort rows -> reverse slots; always: union
// lists.
#include "internal.hpp"

namespace nep {

// Device grid record: 16 global words, then 4 words per system.
// Global words 2-3 and 5-11 describe the candidate rows of the last rebuild
// and persist across calls; 0-1 are per-call maxima; 4 is the rebuild
// decision of this call.
struct DevGlobal {
    float d_build;          // D at the last rebuild
    uint32_t rows_overflow; // a candidate row of the last rebuild was truncated
    int rebuild;            // 1: rebuild the candidate rows in this call
    double R2;              // radial candidate radius squared of the last rebuild
    double RA2;             // angular candidate radius squared
};
static_assert(sizeof(DevGlobal) <= 16 * sizeof(uint32_t), "grid record exceeds its 16 global words");
struct DevSys {
    int nc[3];              // cells per axis of this system (last rebuild)
    int ncell;
    double Lb[3];           // box edges at the last rebuild
};
static_assert(sizeof(DevSys) == kDevSysWords * sizeof(uint32_t), "per-system grid record size");
__device__ __forceinline__ DevGlobal *dev_global(uint32_t *grid) { return reinterpret_cast<DevGlobal *>(grid); }
__device__ __forceinline__ const DevGlobal *dev_global(const uint32_t *grid)
{
    return reinterpret_cast<const DevGlobal *>(grid);
}
__device__ __forceinline__ DevSys *dev_sys(uint32_t *grid, int s) { return reinterpret_cast<DevSys *>(grid + 16) + s; }
__device__ __forceinline__ const DevSys *dev_sys(const uint32_t *grid, int s)
{
    return reinterpret_cast<const DevSys *>(grid + 16) + s;
}

__device__ __forceinline__ int cell_axis(double s, int nc)
{
    s = s - floor(s);
    if (!(s >= 0.0) || !(s < 1.0)) s = 0.0;   // NaN / Inf, or s rounded up to 1
    int c = (int)(s * nc);
    return c >= nc ? nc - 1 : c;
}

__device__ __forceinline__ int wave_max_i(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ float wave_max_f(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}

// Sticky maximum of a status word: thousands of wavefronts updating one
// address serialise in the L2, so the atomic is issued only when v exceeds
// the stored value.  The words only grow between the host's clears, and a
// kernel never sees a value older than the last clear, so a stale read can
// only cost an extra atomic, never lose a maximum.
__device__ __forceinline__ void raise_max(uint32_t *word, uint32_t v)
{
    if (v > __atomic_load_n(word, __ATOMIC_RELAXED)) atomicMax(word, v);
}

// Centroid of each atom's ring polymer, its largest bead distance D_i and
// its displacement |dc_i| from the centroid of the last rebuild (both
// rounded up); each workgroup's maxima of D_i and of D_i + |dc_i| go to the
// skin test through cmax.
__device__ void grid_decision(const SysGeom *__restrict__ geom, int nsys, double rcR, double rcA, double skin,
                              int force, uint32_t *__restrict__ grid, uint32_t *__restrict__ status,
                              const float *__restrict__ cmax, int nblk);

// kCenLanes lanes per atom (adjacent), each summing every kCenLanes-th bead
// (kept in registers for the spread) and packing those beads' positions on
// the fine grid (the packed positions [N][P] of the list); the atom's sums
// and the bead spread meet by shuffles, and the atom's first lane writes
// its centroid and spread.  Each workgroup writes its two maxima to
// cmax[2 blockIdx.x ..] (one store each: same-address atomics from every
// workgroup serialise in the L2), reduced by the decision.
constexpr int kCenBeads = kMaxBeads / kCenLanes;   // beads per lane at most
__global__ __launch_bounds__(kBlock) void k_centroid(const double *__restrict__ pos, const int32_t *__restrict__ types,
                                                     const int32_t *__restrict__ atom_sys,
                                                     int P, int N, int S, double *__restrict__ cen,
                                                     float *__restrict__ spr, const double *__restrict__ cen_ref,
                                                     const SysGeom *__restrict__ geom, const uint32_t *__restrict__ grid,
                                                     uint32_t *__restrict__ status, float4 *__restrict__ pos4,
                                                     float *__restrict__ cmax)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = t / kCenLanes, q = t % kCenLanes;
    const bool has = i < N;
    const int ic = has ? i : N - 1;
    // per-atom records first: their loads do not wait on the positions
    const int sy = atom_sys[ic];
    const int ty = types[ic];
    const double cr0 = cen_ref[3 * ic], cr1 = cen_ref[3 * ic + 1], cr2 = cen_ref[3 * ic + 2];
    const SysGeom &g = geom[sy];
    const size_t st = (size_t)N * 3;
    double x[kCenBeads][3];
#pragma unroll
    for (int u = 0; u < kCenBeads; ++u) {
        const int b = q + u * kCenLanes;
        const double *p = pos + (size_t)(b < P ? b : 0) * st + 3 * (size_t)ic;
        x[u][0] = p[0];
        x[u][1] = p[1];
        x[u][2] = p[2];
    }
    uint32_t f = 0;
    float spread = 0.0f, reach = 0.0f;
    double c[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < kCenBeads; ++u) {
        const int b = q + u * kCenLanes;
        if (has && b < P) {
            c[0] += x[u][0];
            c[1] += x[u][1];
            c[2] += x[u][2];
            pos4[(size_t)i * P + b] = pack_one(x[u], g);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        for (int o = 1; o < kCenLanes; o <<= 1) c[a] += __shfl_xor(c[a], o);
    }
    const double inv = 1.0 / P;
    c[0] *= inv; c[1] *= inv; c[2] *= inv;
    double m2 = 0.0;
#pragma unroll
    for (int u = 0; u < kCenBeads; ++u) {
        const int b = q + u * kCenLanes;
        if (has && b < P) {
            const double dx = x[u][0] - c[0], dy = x[u][1] - c[1], dz = x[u][2] - c[2];
            m2 = fmax(m2, dx * dx + dy * dy + dz * dz);
        }
    }
    for (int o = 1; o < kCenLanes; o <<= 1) m2 = fmax(m2, __shfl_xor(m2, o));
    if (has && q == 0) {
        cen[3 * i] = c[0];
        cen[3 * i + 1] = c[1];
        cen[3 * i + 2] = c[2];
        const bool finite = isfinite(c[0]) && isfinite(c[1]) && isfinite(c[2]) && isfinite(m2);
        spr[i] = finite ? (float)sqrt(m2) * 1.000001f + 1e-7f : 3.0e38f;
        if (!finite) {
            f |= NEP_FLAG_NONFINITE;
        } else {
            const double di = sqrt(m2);
            spread = (float)di * 1.000001f + 1e-7f;   // rounded up
            // displacement from the build centroid carried along with the box:
            // c - lambda c_build, lambda = L / L_build per axis (1 for an unchanged box)
            const DevSys *ds = dev_sys(grid, sy);
            double lam[3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                lam[a] = (!g.tri && ds->Lb[a] > 0.0) ? g.L[a] / ds->Lb[a] : 1.0;   // a changed general cell rebuilds
            const double dx = c[0] - lam[0] * cr0, dy = c[1] - lam[1] * cr1, dz = c[2] - lam[2] * cr2;
            const double d2 = dx * dx + dy * dy + dz * dz;
            reach = isfinite(d2) ? (float)(di + sqrt(d2)) * 1.000001f + 1e-7f : 3.0e38f;
        }
        if (ty < 0 || ty >= S) f |= NEP_FLAG_BAD_TYPE;
    }
    __shared__ float red[2][kBlock / 64];
    spread = wave_max_f(spread);
    reach = wave_max_f(reach);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wv] = spread;
        red[1][wv] = reach;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
            spread = fmaxf(spread, red[0][w]);
            reach = fmaxf(reach, red[1][w]);
        }
        *reinterpret_cast<float2 *>(cmax + 2 * (size_t)blockIdx.x) = make_float2(spread, reach);
    }
    if (f) atomicOr(&status[0], f);
}


// Rebuild decision and, on a rebuild, the grid and candidate radius from the
// measured spread.  Rows built with radius rc + 2 D0 + skin on edges L0 hold
// every j whose periodic centroid distance was below that radius.  With the
// box now L = lambda L0 (per axis) and e = c_j - c_i + n L a minimum-image
// centroid vector, e0 = c0_j - c0_i + n L0 satisfies
//   lambda (x) e0 = e - (dc_j - dc_i),  dc = c - lambda (x) c0,
// so |e0| <= (|e| + |dc_i| + |dc_j|) / lambda_min, whatever the image n.
// A bead pair inside the cutoff has |e| < rc + D_i + D_j (D_i: largest bead
// distance from atom i's centroid), so |e0| < (rc + 2 max_k (D_k + |dc_k|))
// / lambda_min and the rows stay complete while
// (rc + 2 max_k (D_k + |dc_k|)) / lambda_min - rc - 2 D0 <= skin for both
// cutoffs (for an unchanged box: 2 max_k (D_k + |dc_k|) - 2 D0 <= skin);
// otherwise they are rebuilt.  Pairing each atom's spread with its own
// displacement keeps the rows longer than the separate maxima would.  Run
// by k_decide, one workgroup launched after k_centroid (a last-workgroup
// ticket inside k_centroid cost more: every workgroup then needs a
// device-scope fence).
__device__ void grid_decision(const SysGeom *__restrict__ geom, int nsys, double rcR, double rcA, double skin,
                              int force, uint32_t *__restrict__ grid, uint32_t *__restrict__ status,
                              const float *__restrict__ cmax, int nblk)
{
    DevGlobal *dg = dev_global(grid);
    // maxima over the centroid kernel's workgroups
    __shared__ float dred[2][32];
    float spread = 0.0f, reach1 = 0.0f;
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
        const float2 v = *reinterpret_cast<const float2 *>(cmax + 2 * (size_t)k);
        spread = fmaxf(spread, v.x);
        reach1 = fmaxf(reach1, v.y);
    }
    spread = wave_max_f(spread);
    reach1 = wave_max_f(reach1);
    if ((threadIdx.x & 63) == 0) {
        dred[0][threadIdx.x >> 6] = spread;
        dred[1][threadIdx.x >> 6] = reach1;
    }
    __syncthreads();
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        spread = fmaxf(spread, dred[0][w]);
        reach1 = fmaxf(reach1, dred[1][w]);
    }
    double lam_min = 1.0;
    for (int s = 0; s < nsys; ++s) {
        const DevSys *ds = dev_sys(grid, s);
        for (int a = 0; a < 3; ++a)
            if (!geom[s].tri && ds->Lb[a] > 0.0) lam_min = fmin(lam_min, geom[s].L[a] / ds->Lb[a]);
    }
    const double reach = 2.0 * (double)reach1, d0 = 2.0 * (double)dg->d_build;
    const double needR = (rcR + reach) / lam_min - rcR - d0, needA = (rcA + reach) / lam_min - rcA - d0;
    const int rebuild = force || !(needR <= skin && needA <= skin);
    const double rc = rcR > rcA ? rcR : rcA;
    const double R = rc + 2.0 * (double)spread + skin + 1e-9 * (1.0 + rc);
    const double RA = rcA + 2.0 * (double)spread + skin + 1e-9 * (1.0 + rcA);
    const double R_rows = rebuild ? R : sqrt(dg->R2);   // radius of the rows this call uses
    // every thread has read the records (lambda_min, the last build) before any is rewritten
    __syncthreads();
    if (rebuild) {
        for (int s = threadIdx.x; s < nsys; s += blockDim.x) {
            int ncell = 1;
            DevSys *ds = dev_sys(grid, s);
            for (int a = 0; a < 3; ++a) {
                int nc = (int)floor(geom[s].w[a] / (R * (1.0 + 1e-9)));
                nc = nc < 1 ? 1 : (nc > geom[s].nc_cap[a] ? geom[s].nc_cap[a] : nc);
                ds->nc[a] = nc;
                ds->Lb[a] = geom[s].L[a];
                ncell *= nc;
            }
            ds->ncell = ncell;
        }
    }
    __syncthreads();   // every thread has read the record of the last rebuild
    if (threadIdx.x == 0) {
        dg->rebuild = rebuild;
        // general cells: centroid distances are nearest-image distances only
        // below the smallest face distance (mic_vec), and every candidate
        // pair must lie there (rows of radius R_rows)
        for (int s = 0; s < nsys; ++s) {
            if (!geom[s].tri) continue;
            const double wmin = fmin(geom[s].w[0], fmin(geom[s].w[1], geom[s].w[2]));
            if (!(R_rows < wmin)) atomicOr(&status[0], (uint32_t)NEP_FLAG_CELL_TOO_SMALL);
        }
        atomicMax(&status[4], __float_as_uint(spread));
        if (!rebuild) {
            // reused rows that were truncated keep the overflow flag raised
            if (dg->rows_overflow) atomicOr(&status[0], (uint32_t)NEP_FLAG_NEIGHBOR_OVERFLOW);
        } else {
            dg->rows_overflow = 0;
            dg->R2 = R * R;
            dg->RA2 = RA * RA;
            dg->d_build = spread;
            atomicAdd(&status[5], 1u);
        }
    }
    __syncthreads();   // the decision is visible to the whole workgroup
}

// Global cell of atom i's centroid (system s).
__device__ __forceinline__ int atom_cell(const double *__restrict__ cen, int i, const SysGeom &g, const DevSys &ds)
{
    const double c[3] = {cen[3 * i], cen[3 * i + 1], cen[3 * i + 2]};
    const int cx = cell_axis(frac_coord(c, g, 0), ds.nc[0]);
    const int cy = cell_axis(frac_coord(c, g, 1), ds.nc[1]);
    const int cz = cell_axis(frac_coord(c, g, 2), ds.nc[2]);
    return g.cell_base + (cz * ds.nc[1] + cy) * ds.nc[0] + cx;
}

// Cell populations, then (last workgroup) their exclusive prefix sums, the
// counts reset for use as fill counters.
constexpr int kDecideBlock = 1024;   // threads of the decision / cell-list workgroup

__device__ void cell_scan_block(int ncell, int32_t *__restrict__ cnt, int32_t *__restrict__ st)
{
    __shared__ int32_t part[kDecideBlock];
    const int t = threadIdx.x, nt = blockDim.x;
    const int per = (ncell + nt - 1) / nt;
    const int c0 = min(t * per, ncell), c1 = min(c0 + per, ncell);
    int s = 0;
    for (int c = c0; c < c1; ++c) s += __atomic_load_n(&cnt[c], __ATOMIC_RELAXED);
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
        const int v = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;
    for (int c = c0; c < c1; ++c) {
        st[c] = run;
        run += __atomic_load_n(&cnt[c], __ATOMIC_RELAXED);
        cnt[c] = 0;   // reused as fill counter
    }
    if (t == nt - 1) st[ncell] = part[nt - 1];
}

constexpr int kCellLds = 8192;   // cells whose counts the decision kernel keeps in LDS

// The rebuild decision after every workgroup's maxima, and on a rebuild
// the centroid cell list: cell populations, their exclusive prefix sums and
// the atoms sorted into cells (one workgroup; the steps are separated by
// workgroup barriers, so most steps, which keep their rows, cost one launch
// instead of three).  Up to kCellLds cells the counts and the fill slots are
// LDS atomics; larger grids use global ones.
__global__ __launch_bounds__(kDecideBlock) void k_decide(const SysGeom *__restrict__ geom, int nsys, double rcR,
                                                   double rcA, double skin, int force, uint32_t *__restrict__ grid,
                                                   uint32_t *__restrict__ status, const double *__restrict__ cen,
                                                   int N, const int32_t *__restrict__ atom_sys, int ncell,
                                                   int32_t *__restrict__ cell_cnt, int32_t *__restrict__ cell_start,
                                                   int32_t *__restrict__ cell_atoms,
                                                   const float *__restrict__ cmax, int nblk)
{
    grid_decision(geom, nsys, rcR, rcA, skin, force, grid, status, cmax, nblk);
    // values written by other threads of the workgroup are read through L2
    if (!__atomic_load_n(&dev_global(grid)->rebuild, __ATOMIC_RELAXED)) return;   // whole workgroup
    if (ncell <= kCellLds) {
        // counts in LDS; after the scan each counter holds its cell's start and
        // an LDS atomic on it hands out the atom's slot
        __shared__ int32_t lc[kCellLds];
        __shared__ int32_t part[kDecideBlock];
        for (int c = threadIdx.x; c < ncell; c += blockDim.x) lc[c] = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            const int s = atom_sys[i];
            atomicAdd(&lc[atom_cell(cen, i, geom[s], *dev_sys(grid, s))], 1);
        }
        __syncthreads();
        const int t = threadIdx.x, nt = blockDim.x;
        const int per = (ncell + nt - 1) / nt;
        const int c0 = min(t * per, ncell), c1 = min(c0 + per, ncell);
        int sum = 0;
        for (int c = c0; c < c1; ++c) sum += lc[c];
        part[t] = sum;
        __syncthreads();
        for (int off = 1; off < nt; off <<= 1) {
            const int v = (t >= off) ? part[t - off] : 0;
            __syncthreads();
            part[t] += v;
            __syncthreads();
        }
        int run = part[t] - sum;
        for (int c = c0; c < c1; ++c) {
            const int n = lc[c];
            cell_start[c] = run;
            lc[c] = run;
            run += n;
        }
        if (t == nt - 1) cell_start[ncell] = part[nt - 1];
        __syncthreads();
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            const int s = atom_sys[i];
            cell_atoms[atomicAdd(&lc[atom_cell(cen, i, geom[s], *dev_sys(grid, s))], 1)] = i;
        }
        return;
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int s = atom_sys[i];
        atomicAdd(&cell_cnt[atom_cell(cen, i, geom[s], *dev_sys(grid, s))], 1);
    }
    __syncthreads();
    cell_scan_block(ncell, cell_cnt, cell_start);   // leaves the counts at zero for the fill
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const int s = atom_sys[i];
        const int c = atom_cell(cen, i, geom[s], *dev_sys(grid, s));
        const int slot = atomicAdd(&cell_cnt[c], 1);
        cell_atoms[__atomic_load_n(&cell_start[c], __ATOMIC_RELAXED) + slot] = i;
    }
}




// One candidate row sorted by (species, index) into dst, with its species
// block starts, by one wavefront.  Rows of up to kSortLds entries: the keys
// go to lds, padded to a power of two with keys above every entry, and a
// bitonic network sorts them there (log2(n) (log2(n) + 1) / 2 exchange
// stages, n / 128 exchanges per lane each); longer rows: rank sort straight
// from src (each element's position is the number of smaller keys).  src
// is not modified, so other wavefronts may read it meanwhile.
constexpr int kSortLds = 1024;
__device__ __forceinline__ uint32_t cand_key(int32_t w)
{
    return ((uint32_t)(w & 3) << 29) | (uint32_t)(w >> 2);   // species above index; entries are distinct
}
__device__ __forceinline__ int32_t cand_entry(uint32_t key)
{
    return (int32_t)(((key & 0x1fffffffu) << 2) | (key >> 29));
}

__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ void sort_row_into(int32_t *__restrict__ dst, int n, const int32_t *__restrict__ src,
                              int32_t *__restrict__ lds, int S, int32_t *__restrict__ off)
{
    const int lane = threadIdx.x & 63;
    int cntS[kMaxSpecies] = {0, 0, 0, 0};
    if (n <= kSortLds) {
        uint32_t *key = reinterpret_cast<uint32_t *>(lds);
        int np = 64;
        while (np < n) np <<= 1;
        for (int e = lane; e < np; e += 64) {
            const int32_t w = e < n ? src[e] : 0;
            key[e] = e < n ? cand_key(w) : 0xffffffffu;
            if (e < n) {
#pragma unroll
                for (int t = 0; t < kMaxSpecies; ++t) cntS[t] += (w & 3) == t;
            }
        }
        wave_lds_fence();
        for (int size = 2; size <= np; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int t = lane; t < (np >> 1); t += 64) {
                    const int lo = 2 * stride * (t / stride) + (t % stride), hi = lo + stride;
                    const uint32_t a = key[lo], b = key[hi];
                    const bool up = (lo & size) == 0;   // ascending block
                    if ((a > b) == up) {
                        key[lo] = b;
                        key[hi] = a;
                    }
                }
                wave_lds_fence();
            }
        }
        for (int e = lane; e < n; e += 64) dst[e] = cand_entry(key[e]);
    } else {
        for (int e = lane; e < n; e += 64) {
            const int32_t w = src[e];
            const uint32_t kw = cand_key(w);
            int r = 0;
            for (int f = 0; f < n; ++f) r += cand_key(src[f]) < kw;
            dst[r] = w;
#pragma unroll
            for (int t = 0; t < kMaxSpecies; ++t) cntS[t] += (w & 3) == t;
        }
    }
#pragma unroll
    for (int t = 0; t < kMaxSpecies; ++t)
        for (int o = 32; o > 0; o >>= 1) cntS[t] += __shfl_xor(cntS[t], o);
    if (lane == 0) {
        int run = 0;
        for (int t = 0; t < S; ++t) {
            off[t] = run;
            run += cntS[t];
        }
        off[S] = run;
    }
    // the sorted row, its block starts and the buffer are read next by
    // every lane of this wavefront
    wave_lds_fence();
}

// Candidate rows.  gridDim.y workgroups per cell, each taking every
// gridDim.y-th group of the cell's atoms (small or skewed cells have few
// cells with large stencils); the centroids of the cell's stencil cells
// (3 x 3 x 3, fewer along an axis with fewer than 3 cells) are staged in
// LDS when they fit, and each wavefront takes one atom at a time, its lanes
// testing 64 stencil atoms at once and appending the accepted ones by
// ballot + prefix popcount (stencil order, into the unsorted staging rows,
// which k_union sorts).  A stencil too large for LDS is read from global
// memory instead.
constexpr int kStage = 2048;
constexpr int kCandSplitMax = 16;   // workgroups per cell at most
__global__ __launch_bounds__(256) void k_candidates(const double *__restrict__ cen, const int32_t *__restrict__ types,
                                                    int N, int S, const SysGeom *__restrict__ geom,
                                                    const int32_t *__restrict__ cell_sys, uint32_t *__restrict__ grid,
                                                    const int32_t *__restrict__ cell_start,
                                                    const int32_t *__restrict__ cell_atoms,
                                                    int32_t *__restrict__ cell_cnt, int capR, int capA,
                                                    int32_t *__restrict__ candR, int32_t *__restrict__ lenR,
                                                    int32_t *__restrict__ candA, int32_t *__restrict__ lenA,
                                                    double *__restrict__ cen_ref, uint32_t *__restrict__ status)
{
    __shared__ double sx[kStage], sy[kStage], sz[kStage];
    __shared__ int32_t sw[kStage];
    __shared__ int32_t rs[28], rp[28];
    __shared__ int nrange;
    DevGlobal *dg = dev_global(grid);
    const int sy_ = cell_sys[blockIdx.x];
    const SysGeom &g = geom[sy_];
    const DevSys ds = *dev_sys(grid, sy_);
    const int c = blockIdx.x - g.cell_base;   // cell within its system
    if (!dg->rebuild || c >= ds.ncell) return;   // whole workgroup
    if (threadIdx.x == 0 && blockIdx.y == 0) cell_cnt[blockIdx.x] = 0;   // counts start from zero at the next rebuild
    const int nc0 = ds.nc[0], nc1 = ds.nc[1], nc2 = ds.nc[2];
    const double R2 = dg->R2, RA2 = dg->RA2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) {
        const int cx = c % nc0, cy = (c / nc0) % nc1, cz = c / (nc0 * nc1);
        const int oz_n = nc2 >= 3 ? 3 : nc2, oy_n = nc1 >= 3 ? 3 : nc1, ox_n = nc0 >= 3 ? 3 : nc0;
        int nr = 0, tot = 0;
        for (int oz = 0; oz < oz_n; ++oz) {
            int z = nc2 >= 3 ? cz + oz - 1 : oz;
            z = z < 0 ? z + nc2 : (z >= nc2 ? z - nc2 : z);
            for (int oy = 0; oy < oy_n; ++oy) {
                int y = nc1 >= 3 ? cy + oy - 1 : oy;
                y = y < 0 ? y + nc1 : (y >= nc1 ? y - nc1 : y);
                for (int ox = 0; ox < ox_n; ++ox) {
                    int x = nc0 >= 3 ? cx + ox - 1 : ox;
                    x = x < 0 ? x + nc0 : (x >= nc0 ? x - nc0 : x);
                    const int cc = g.cell_base + (z * nc1 + y) * nc0 + x;
                    rs[nr] = cell_start[cc];
                    rp[nr] = tot;
                    tot += cell_start[cc + 1] - cell_start[cc];
                    ++nr;
                }
            }
        }
        rp[nr] = tot;
        nrange = nr;
    }
    __syncthreads();
    const int nr = nrange, total = rp[nr];
    const bool staged = total <= kStage;
    // flat stencil position q -> index into cell_atoms (the last range starting at or before q)
    auto at = [&](int q) {
        int lo = 0, hi = nr - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rp[mid] <= q) lo = mid;
            else hi = mid - 1;
        }
        return rs[lo] + (q - rp[lo]);
    };
    if (staged) {
        for (int q = threadIdx.x; q < total; q += blockDim.x) {
            const int j = cell_atoms[at(q)];
            const int tj = types[j];
            sx[q] = cen[3 * j];
            sy[q] = cen[3 * j + 1];
            sz[q] = cen[3 * j + 2];
            sw[q] = (tj >= 0 && tj < S) ? ((j << 2) | tj) : -1;
        }
    }
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int a0 = cell_start[blockIdx.x], a1 = cell_start[blockIdx.x + 1];
    const int waves = blockDim.x >> 6;
    for (int a = a0 + blockIdx.y * waves + wv; a < a1; a += gridDim.y * waves) {
        const int i = cell_atoms[a];
        const double ci[3] = {cen[3 * i], cen[3 * i + 1], cen[3 * i + 2]};
        int32_t *rowR = candR + (size_t)i * capR;
        int32_t *rowA = candA + (size_t)i * capA;
        int cR = 0, cA = 0;
        for (int q0 = 0; q0 < total; q0 += 64) {
            const int q = q0 + lane;
            bool okR = false, okA = false;
            int w = -1;
            if (q < total) {
                double p[3];
                if (staged) {
                    p[0] = sx[q]; p[1] = sy[q]; p[2] = sz[q];
                    w = sw[q];
                } else {
                    const int j = cell_atoms[at(q)];
                    const int tj = types[j];
                    p[0] = cen[3 * j]; p[1] = cen[3 * j + 1]; p[2] = cen[3 * j + 2];
                    w = (tj >= 0 && tj < S) ? ((j << 2) | tj) : -1;
                }
                if (w >= 0 && (w >> 2) != i) {
                    double d[3] = {p[0] - ci[0], p[1] - ci[1], p[2] - ci[2]};
                    mic_vec(d, g, g.tri);
                    const double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                    okR = r2 < R2;
                    okA = r2 < RA2;
                }
            }
            const uint64_t mR = __ballot(okR), mA = __ballot(okA);
            const int pR = cR + __popcll(mR & below), pA = cA + __popcll(mA & below);
            if (okR && pR < capR) rowR[pR] = w;
            if (okA && pA < capA) rowA[pA] = w;
            cR += __popcll(mR);
            cA += __popcll(mA);
        }
        if (lane == 0) {
            lenR[i] = cR;
            lenA[i] = cA;
            cen_ref[3 * i] = ci[0];
            cen_ref[3 * i + 1] = ci[1];
            cen_ref[3 * i + 2] = ci[2];
            raise_max(&status[3], (uint32_t)cR);
            raise_max(&status[6], (uint32_t)cA);
            if (cR > capR || cA > capA) {
                atomicOr(&status[0], (uint32_t)NEP_FLAG_NEIGHBOR_OVERFLOW);
                atomicOr(&dg->rows_overflow, 1u);
            }
        }
    }
}



// Union lists.  One wavefront per atom and list (grid.y picks the radial or
// angular list).  A candidate is kept when the pair is inside the cutoff for
// at least one bead; the radial list stores the atom index j, the angular
// list the candidate slot k, both with the bead mask of the exact per-bead
// decisions, in candidate order.
//
// Each batch of 64 candidates (one per lane) is first classified from the
// centroids: with d the minimum-image centroid distance and s = s_i + s_j
// the two atoms' largest bead distances from their centroids, every bead
// pair lies within [d - s, d + s] (the minimum image is the shortest image),
// so d + s < rc - eps keeps all beads and d - s > rc + eps none (d is the
// nearest-image distance, also in general cells: mic_vec).  Only the
// remaining shell candidates are tested bead by bead (the exact test of the
// per-bead lists), their G lanes per candidate holding the beads; each mask
// is written back to its candidate's lane, and the kept candidates are
// appended with one ballot-ranked store per lane.
constexpr double kShellEps = 1e-3;   // A; far above the rounding of d and s
constexpr int kUnionRounds = 4;      // shell rounds whose partner loads are in flight together

template <bool TRI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TRI ? 4 : 5))) void k_union(const double *__restrict__ pos, const float4 *__restrict__ pos4,
                                               const double *__restrict__ cen, const float *__restrict__ spr, int P,
                                               int N, int S, int lg, const int32_t *__restrict__ atom_sys,
                                               const SysGeom *__restrict__ geom, CutTest cR, CutTest cA,
                                               int32_t *__restrict__ candR, int32_t *__restrict__ offR,
                                               int32_t *__restrict__ candA, int32_t *__restrict__ offA,
                                               const int32_t *__restrict__ candRs, const int32_t *__restrict__ candAs,
                                               const int32_t *__restrict__ lenR, const int32_t *__restrict__ lenA,
                                               int capR, int capA, int32_t *__restrict__ uniR,
                                               uint64_t *__restrict__ umR, int32_t *__restrict__ uendR,
                                               int32_t *__restrict__ uniA, uint64_t *__restrict__ umA,
                                               int32_t *__restrict__ uendA, uint32_t *__restrict__ status,
                                               const uint32_t *__restrict__ grid, const int32_t *__restrict__ types,
                                               int32_t *__restrict__ revA)
{
    const int lane = threadIdx.x & 63, G = 1 << lg, CPW = 64 >> lg;
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int kind = blockIdx.y;   // 0: radial list, 1: angular list
    if (i >= N) return;            // whole wavefront
    if (dev_global(grid)->rebuild) {
        // rows rebuilt in this call: this wavefront's row, left unsorted in
        // the staging array by the candidate search, sorted into the list
        __shared__ int32_t sbuf[4][kSortLds];   // one buffer per wavefront of the 256-lane workgroup
        const int cap = kind ? capA : capR;
        const int n = min((kind ? lenA : lenR)[i], cap);
        int32_t *srow = (kind ? candA : candR) + (size_t)i * cap;
        sort_row_into(srow, n, (kind ? candAs : candRs) + (size_t)i * cap, sbuf[threadIdx.x >> 6], S,
                      (kind ? offA : offR) + (size_t)i * (kMaxSpecies + 1));
        if (kind == 1) {
            // reverse slot of every angular candidate: for candidate j of i
            // (slot k) the slot of i in j's sorted row, i.e. the number of
            // smaller keys in j's row, counted in its unsorted staging copy
            // (no other row need be sorted yet); -1 if i is missing (only
            // when j's row overflowed).  The whole wavefront scans each
            // partner's row (contiguous loads), one candidate after another;
            // lane k % 64 keeps slot k's result for one store per 64 slots.
            const int ti = types[i] & 3;
            const int32_t wi = (int32_t)(((uint32_t)i << 2) | (uint32_t)ti);
            const uint32_t ki = cand_key(wi);
            for (int k0 = 0; k0 < n; k0 += 64) {
                const int kn = min(64, n - k0);
                const int jl = lane < kn ? (srow[k0 + lane] >> 2) : i;   // the partners of these 64 slots
                int res = -1;
                for (int kk = 0; kk < kn; ++kk) {
                    const int j = __builtin_amdgcn_readlane(jl, kk);
                    const int nj = min(lenA[j], capA);
                    const int32_t *rj = candAs + (size_t)j * capA;
                    int r = 0;
                    bool found = false;
                    for (int f = lane; f < nj; f += 64) {
                        const int32_t w = rj[f];
                        r += cand_key(w) < ki;
                        found |= w == wi;
                    }
                    for (int o = 32; o > 0; o >>= 1) r += __shfl_xor(r, o);
                    const bool any = __ballot(found) != 0;
                    if (lane == kk) res = any ? r : -1;
                }
                if (lane < kn) revA[(size_t)i * capA + k0 + lane] = res;
            }
        }
    }
    const int cg = lane >> lg, b = lane & (G - 1);
    const bool bead_ok = b < P;
    const int bb = bead_ok ? b : P - 1;
    const float4 pi = pos4[(size_t)i * P + bb];
    const double *pb = pos + (size_t)bb * N * 3;
    const SysGeom &g = geom[atom_sys[i]];
    const bool tri = TRI && g.tri;   // orthorhombic-only launches carry no general-cell code
    const uint64_t gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
    const uint64_t full = (P == 64) ? ~0ull : ((1ull << P) - 1ull);
    const double ci0 = cen[3 * (size_t)i], ci1 = cen[3 * (size_t)i + 1], ci2 = cen[3 * (size_t)i + 2];
    const double si = (double)spr[i];

    const int cap = kind ? capA : capR;
    const int32_t *row = (kind ? candA : candR) + (size_t)i * cap;
    const int32_t *o = (kind ? offA : offR) + (size_t)i * (kMaxSpecies + 1);
    int32_t *uni = (kind ? uniA : uniR) + (size_t)i * cap;
    uint64_t *um = (kind ? umA : umR) + (size_t)i * cap;
    int32_t *uend = (kind ? uendA : uendR) + (size_t)i * kMaxSpecies;
    const CutTest c = kind ? cA : cR;
    const double rc = sqrt(c.rc2);
    // batches of 64 row entries run across the species blocks (the row is
    // sorted by species, so the kept entries stay in blocks); each species'
    // kept count gives the block ends
    int cnt = 0;   // wave-uniform
    int cntS[kMaxSpecies] = {0, 0, 0, 0};
    const int kend = min(o[S], cap);
    {
        for (int kb = 0; kb < kend; kb += 64) {
            const int k = kb + lane;
            const bool kin = k < kend;
            const int32_t wrow = kin ? row[k] : 0;
            const int j = kin ? wrow >> 2 : i;
            double dv[3] = {cen[3 * (size_t)j] - ci0, cen[3 * (size_t)j + 1] - ci1, cen[3 * (size_t)j + 2] - ci2};
            mic_vec(dv, g, tri);
            // d + s < rc - eps and d - s > rc + eps, on squares
            const double d2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
            const double sp = si + (double)spr[j];
            const double lo = rc - kShellEps - sp, hi = rc + kShellEps + sp;
            const bool all_in = kin && lo > 0.0 && d2 < lo * lo;
            const bool shell = kin && !all_in && !(d2 > hi * hi);
            int mlo = 0, mhi = 0;
            uint64_t rem = __ballot(shell);
            while (rem) {
                // kUnionRounds rounds of the next CPW shell candidates (one
                // per group of G lanes), their partners' positions loaded
                // together; rounds past the last candidate load lane 0's
                // partner and test nothing
                uint64_t take[kUnionRounds];
                int nq[kUnionRounds], jq[kUnionRounds];
#pragma unroll
                for (int u = 0; u < kUnionRounds; ++u) {
                    take[u] = rem;
                    int my = 0, n = 0;
                    for (int q = 0; q < CPW && rem; ++q) {
                        const int sq = __builtin_ctzll(rem);
                        rem &= rem - 1;
                        if (q == cg) my = sq;
                        n = q + 1;
                    }
                    nq[u] = n;
                    jq[u] = __shfl(j, my, 64);
                }
                float4 pj[kUnionRounds];
#pragma unroll
                for (int u = 0; u < kUnionRounds; ++u) pj[u] = pos4[(size_t)jq[u] * P + bb];
#pragma unroll
                for (int u = 0; u < kUnionRounds; ++u) {
                    float ex, ey, ez;
                    packed_pair_g(pj[u], pi, g, tri, ex, ey, ez);
                    const float r2f = ex * ex + ey * ey + ez * ez;
                    const bool in = cg < nq[u] && bead_ok && pair_within(r2f, c, pb, i, jq[u], g, tri);
                    const uint64_t m = __ballot(in);
                    uint64_t tk = take[u];
                    for (int q = 0; q < nq[u]; ++q) {
                        const int sq = __builtin_ctzll(tk);
                        tk &= tk - 1;
                        const uint64_t gm = (m >> (q * G)) & gmask;
                        if (lane == sq) {
                            mlo = (int)(uint32_t)gm;
                            mhi = (int)(uint32_t)(gm >> 32);
                        }
                    }
                }
            }
            const uint64_t mask = all_in ? full : (shell ? (((uint64_t)(uint32_t)mhi << 32) | (uint32_t)mlo) : 0ull);
            const bool keep = mask != 0ull;
            const uint64_t bal = __ballot(keep);
            const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
            if (keep) {
                // radial lists keep the atom index, angular ones the candidate slot
                uni[cnt + rank] = kind ? k : j;
                um[cnt + rank] = mask;
            }
            cnt += __popcll(bal);
            for (int t = 0; t < S; ++t) cntS[t] += __popcll(__ballot(keep && (wrow & 3) == t));
        }
    }
    if (lane == 0) {
        int run = 0;
        for (int t = 0; t < S; ++t) {
            run += cntS[t];
            uend[t] = run;
        }
        raise_max(&status[1 + kind], (uint32_t)cnt);
    }
}

// Per-bead lists written out for tests and analysis: one lane per (bead,
// atom), the same decision as the force path over the candidate rows.
__global__ __launch_bounds__(256) void k_materialize(const double *__restrict__ pos, const float4 *__restrict__ pos4,
                                                     int P, int N, int S, const int32_t *__restrict__ atom_sys,
                                                     const SysGeom *__restrict__ geom, CutTest cR,
                                                     CutTest cA, const int32_t *__restrict__ candR,
                                                     const int32_t *__restrict__ offR,
                                                     const int32_t *__restrict__ candA,
                                                     const int32_t *__restrict__ offA, int capR, int capA,
                                                     int outR, int outA, int32_t *__restrict__ nbrR,
                                                     int32_t *__restrict__ cntR, int32_t *__restrict__ nbrA,
                                                     int32_t *__restrict__ cntA)
{
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)P * N) return;
    const int b = (int)(e / (size_t)N), i = (int)(e - (size_t)b * N);
    const float4 pi = pos4[(size_t)i * P + b];
    const double *pb = pos + (size_t)b * N * 3;
    const SysGeom &g = geom[atom_sys[i]];
    for (int kind = 0; kind < 2; ++kind) {
        const int cap = kind ? capA : capR, out = kind ? outA : outR;
        const int32_t *row = (kind ? candA : candR) + (size_t)i * cap;
        const int n = min((kind ? offA : offR)[(size_t)i * (kMaxSpecies + 1) + S], cap);
        int32_t *nb = (kind ? nbrA : nbrR) + (size_t)b * out * N + i;
        const CutTest c = kind ? cA : cR;
        int cnt = 0;
        for (int k = 0; k < n; ++k) {
            const int j = row[k] >> 2;
            float dx, dy, dz;
            packed_pair_g(pos4[(size_t)j * P + b], pi, g, g.tri, dx, dy, dz);
            if (pair_within(dx * dx + dy * dy + dz * dz, c, pb, i, j, g, g.tri)) {
                if (cnt < out) nb[(size_t)cnt * N] = j;
                ++cnt;
            }
        }
        (kind ? cntA : cntR)[(size_t)b * N + i] = cnt;
    }
}

// Checks the boxes of a batch and refreshes the per-system geometry (fine
// grids, cell bounds, cell ranges).  The device copy is rewritten, with a
// synchronous copy, only when a box changed; `changed` reports that.
int32_t update_geometry(const nep_model *m, nep_nlist *nl, const double *boxes, bool &changed, float &margin,
                        bool &tri_changed)
{
    const double rc = std::max(m->hp.rc_radial, m->hp.rc_angular);
    std::vector<SysGeom> G(nl->nsys);
    int cell_total = 0;
    double hmax = 0.0;
    changed = false;
    tri_changed = false;
    for (int s = 0; s < nl->nsys; ++s) {
        SysGeom &g = G[s];
        const double *box = boxes + 9 * s;
        CellInfo ci;
        if (!cell_info(box, ci))
            return fail(NEP_ERR_INVALID_ARG, "system %d: singular, left-handed or non-finite cell", s);
        for (int a = 0; a < 3; ++a)
            if (ci.w[a] < 2.0 * rc)
                return fail(NEP_ERR_BOX_TOO_SMALL,
                            "system %d: the cell's faces %d lie %g apart, less than twice the cutoff %g", s, a,
                            ci.w[a], rc);
        const FineGrid fg = fine_grid_cell(ci, rc);
        if (!fg.exact)
            return fail(NEP_ERR_BOX_TOO_SMALL, "system %d: face distances %g %g %g leave no margin over twice the "
                                               "cutoff", s, ci.w[0], ci.w[1], ci.w[2]);
        g.tri = ci.tri;
        bool diff = false;
        for (int k = 0; k < 9; ++k) {
            g.H[k] = ci.H[k];
            g.G[k] = ci.G[k];
            if (nl->boxL[9 * s + k] != box[k]) diff = true;
        }
        int ncap = 1;
        for (int a = 0; a < 3; ++a) {
            g.L[a] = ci.tri ? 1.0 : ci.H[4 * a];
            g.invL[a] = 1.0 / g.L[a];
            g.w[a] = ci.w[a];
            g.hd[a] = fg.hd[a];
            g.Minv[a] = fg.Minv[a];
            g.h[a] = fg.h[a];
            g.M[a] = fg.M[a];
            const int nc = (int)std::floor(ci.w[a] / (rc * (1.0 + 1e-9)));
            g.nc_cap[a] = nc < 1 ? 1 : (nc > 64 ? 64 : nc);
            ncap *= g.nc_cap[a];
            hmax = std::max(hmax, fg.hd[a]);
        }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                g.GM[3 * r + c] = ci.G[3 * r + c] * g.M[c];
                g.hvd[3 * r + c] = ci.H[3 * r + c] / g.M[r];
                g.hv[3 * r + c] = (float)g.hvd[3 * r + c];
            }
        if (ci.tri) hmax = std::max(hmax, fg.hd[0] + fg.hd[1] + fg.hd[2]);   // offsets span the skewed fine cell
        if (diff) {
            changed = true;
            // the scaled skin test covers per-axis scaling of orthorhombic cells only
            bool was_tri = false;
            for (int k : {1, 2, 3, 5, 6, 7}) was_tri = was_tri || nl->boxL[9 * s + k] != 0.0;
            if (ci.tri || was_tri) tri_changed = true;
        }
        g.cell_base = cell_total;
        cell_total += ncap;
        g.atom0 = nl->off[s];
        g.atom1 = nl->off[s + 1];
    }
    margin = (float)(1e-3 * std::max(1.0, hmax * hmax) * std::max(1.0, rc * rc / 36.0));
    nl->margin = margin;
    nl->any_tri = 0;
    for (int s = 0; s < nl->nsys; ++s) nl->any_tri |= G[s].tri;
    if (!changed) return NEP_OK;
    if (cell_total > nl->ncell_alloc) {
        for (int32_t **p : {&nl->cell_cnt, &nl->cell_start, &nl->cell_sys}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
        nl->ncell_alloc = 0;
        NEP_HIP(hipMalloc(&nl->cell_cnt, sizeof(int32_t) * (size_t)cell_total));
        NEP_HIP(hipMemset(nl->cell_cnt, 0, sizeof(int32_t) * (size_t)cell_total));   // kept zero between rebuilds
        NEP_HIP(hipMalloc(&nl->cell_start, sizeof(int32_t) * (size_t)(cell_total + 1)));
        NEP_HIP(hipMalloc(&nl->cell_sys, sizeof(int32_t) * (size_t)cell_total));
        nl->ncell_alloc = cell_total;
    }
    std::vector<int32_t> cs(cell_total);
    for (int s = 0; s < nl->nsys; ++s) {
        const int n = G[s].nc_cap[0] * G[s].nc_cap[1] * G[s].nc_cap[2];
        for (int c = 0; c < n; ++c) cs[G[s].cell_base + c] = s;
    }
    NEP_HIP(hipDeviceSynchronize());
    NEP_HIP(hipMemcpy(nl->cell_sys, cs.data(), sizeof(int32_t) * cs.size(), hipMemcpyHostToDevice));
    NEP_HIP(hipMemcpy(nl->geom, G.data(), sizeof(SysGeom) * G.size(), hipMemcpyHostToDevice));
    nl->ncell_total = cell_total;
    for (int s = 0; s < nl->nsys; ++s)
        for (int k = 0; k < 9; ++k) nl->boxL[9 * s + k] = boxes[9 * s + k];
    return NEP_OK;
}

}  // namespace nep

using namespace nep;

extern "C" int32_t neighbor_build_batched(const nep_model *m, nep_nlist *nl, const double *pos, const double *boxes,
                                          const int32_t *types, int32_t P, int32_t N, hipStream_t s)
{
    if (!m || !nl || !boxes) return fail(NEP_ERR_INVALID_ARG, "neighbor_build: null argument");
    if (P != nl->P || N != nl->N || nl->S != m->hp.n_species)
        return fail(NEP_ERR_INVALID_ARG, "neighbor_build: P=%d N=%d do not match the list (P=%d N=%d)", P, N,
                    nl->P, nl->N);
    if (P == 0 || N == 0) return NEP_OK;
    if (!pos || !types) return fail(NEP_ERR_INVALID_ARG, "neighbor_build: null array");
    bool changed = false, tri_changed = false;
    float margin = 0.0f;
    const int32_t rc_ = update_geometry(m, nl, boxes, changed, margin, tri_changed);
    if (rc_ != NEP_OK) return rc_;
    // a per-axis scaling of an orthorhombic cell is covered by the device-side skin test
    const bool force = !nl->built || tri_changed;
    const dim3 gw(div_up(N, kBlock / 64));
    // enough workgroups for the candidate search even when the cells are few
    const dim3 gc(nl->ncell_total, std::min(kCandSplitMax, std::max(1, div_up(1024, nl->ncell_total))));
    {
        ProfScope ps_(K_CENTROID, s);
        const int nblk = div_up(N * kCenLanes, kBlock);
        hipLaunchKernelGGL(k_centroid, dim3(nblk), dim3(kBlock), 0, s, pos, types, nl->atom_sys, P, N, nl->S,
                           nl->cen, nl->spr, nl->cen_ref, nl->geom, nl->grid, nl->status,
                           reinterpret_cast<float4 *>(nl->pos4), nl->cmax);
        hipLaunchKernelGGL(k_decide, dim3(1), dim3(kDecideBlock), 0, s, nl->geom, nl->nsys, m->hp.rc_radial,
                           m->hp.rc_angular, nl->skin, force ? 1 : 0, nl->grid, nl->status, nl->cen, N, nl->atom_sys,
                           nl->ncell_total, nl->cell_cnt, nl->cell_start, nl->cell_atoms, nl->cmax, nblk);
    }
    {
        ProfScope ps_(K_CANDIDATES, s);
        hipLaunchKernelGGL(k_candidates, gc, dim3(kBlock), 0, s, nl->cen, types, N, nl->S, nl->geom, nl->cell_sys,
                           nl->grid, nl->cell_start, nl->cell_atoms, nl->cell_cnt, nl->capR, nl->capA, nl->candRs,
                           nl->lenR,
                           nl->candAs, nl->lenA, nl->cen_ref, nl->status);
    }
    {
        ProfScope ps_(K_NLIST, s);
        const int lg = lanes_log2(P);
        const double rR2 = m->hp.rc_radial * m->hp.rc_radial, rA2 = m->hp.rc_angular * m->hp.rc_angular;
        const CutTest cR{(float)rR2, margin, rR2};
        const CutTest cA{(float)rA2, margin, rA2};
        auto kern = nl->any_tri ? k_union<true> : k_union<false>;
        hipLaunchKernelGGL(kern, dim3(div_up(N, kBlock / 64), 2), dim3(kBlock), 0, s, pos,
                           reinterpret_cast<const float4 *>(nl->pos4), nl->cen, nl->spr, P, N, nl->S, lg, nl->atom_sys, nl->geom, cR,
                           cA, nl->candR, nl->offR, nl->candA, nl->offA, nl->candRs, nl->candAs, nl->lenR, nl->lenA,
                           nl->capR, nl->capA, nl->uniR, nl->umR,
                           nl->uendR, nl->uniA, nl->umA, nl->uendA, nl->status, nl->grid, types, nl->revA);
    }
    NEP_HIP(hipGetLastError());
    nl->built = 1;
    nl->rc_built[0] = m->hp.rc_radial;
    nl->rc_built[1] = m->hp.rc_angular;
    return NEP_OK;
}

extern "C" int32_t neighbor_build(const nep_model *m, nep_nlist *nl, const double *pos, const double box[9],
                                  const int32_t *types, int32_t P, int32_t N, hipStream_t s)
{
    if (nl && nl->nsys != 1) return fail(NEP_ERR_INVALID_ARG, "neighbor_build: the list holds a batch of systems");
    return neighbor_build_batched(m, nl, pos, box, types, P, N, s);
}

extern "C" int32_t nep_nlist_materialize(const nep_model *m, const nep_nlist *nl, const double *pos,
                                         const double *boxes, int32_t P, int32_t N, int32_t outR, int32_t outA,
                                         int32_t *nbrR, int32_t *cntR, int32_t *nbrA, int32_t *cntA, hipStream_t s)
{
    if (!m || !nl || !boxes) return fail(NEP_ERR_INVALID_ARG, "nep_nlist_materialize: null argument");
    if (P != nl->P || N != nl->N || outR < 1 || outA < 1)
        return fail(NEP_ERR_INVALID_ARG, "nep_nlist_materialize: bad sizes");
    if (P == 0 || N == 0) return NEP_OK;
    if (!pos || !nbrR || !cntR || !nbrA || !cntA) return fail(NEP_ERR_INVALID_ARG, "nep_nlist_materialize: null array");
    if (!nl->built) return fail(NEP_ERR_INVALID_ARG, "nep_nlist_materialize: no neighbor_build yet");
    for (int sy = 0; sy < nl->nsys; ++sy)
        for (int k = 0; k < 9; ++k)
            if (boxes[9 * sy + k] != nl->boxL[9 * sy + k])
                return fail(NEP_ERR_INVALID_ARG, "nep_nlist_materialize: box of system %d differs from the last build",
                            sy);
    const float margin = nl->margin;
    const double rR2 = m->hp.rc_radial * m->hp.rc_radial, rA2 = m->hp.rc_angular * m->hp.rc_angular;
    const CutTest cR{(float)rR2, margin, rR2};
    const CutTest cA{(float)rA2, margin, rA2};
    const size_t n = (size_t)P * N;
    {
        ProfScope ps_(K_MATERIALIZE, s);
        hipLaunchKernelGGL(k_materialize, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, pos,
                           reinterpret_cast<const float4 *>(nl->pos4), P, N, nl->S, nl->atom_sys, nl->geom, cR, cA,
                           nl->candR, nl->offR, nl->candA, nl->offA, nl->capR, nl->capA, outR, outA, nbrR, cntR, nbrA,
                           cntA);
    }
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}

extern "C" int32_t nep_nlist_set_skin(nep_nlist *nl, double skin)
{
    if (!nl) return fail(NEP_ERR_INVALID_ARG, "nep_nlist_set_skin: null argument");
    if (!(skin >= 0.0) || !(skin <= 10.0)) return fail(NEP_ERR_INVALID_ARG, "nep_nlist_set_skin: bad skin %g", skin);
    nl->skin = skin;
    nl->built = 0;
    return NEP_OK;
}

extern "C" int32_t nep_nlist_invalidate(nep_nlist *nl)
{
    if (!nl) return fail(NEP_ERR_INVALID_ARG, "nep_nlist_invalidate: null argument");
    nl->built = 0;
    return NEP_OK;
}
