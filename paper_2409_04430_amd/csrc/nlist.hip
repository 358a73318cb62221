// Per-bead neighbour lists by a cell list (minimum image, orthorhombic box).
//
// Pairs are accepted by the literal FP64 minimum-image test
//   d = r_j - r_i;  d -= L * rint(d / L)  (per axis);  (dx*dx + dy*dy) + dz*dz < rc*rc
// evaluated without contraction, so the sets equal those of a brute-force
// search over all pairs.  The cell list only limits the candidates: cells
// are at least rc wide (plus a relative margin that absorbs rounding in the
// cell assignment), and with fewer than three cells along an axis the
// stencil visits each distinct cell once.
//
// Kernels per call: zero counts -> count atoms per cell -> per-bead scan ->
// scatter atoms into cells -> sort each cell (deterministic order) ->
// per-atom search writing species-blocked, slot-major lists.
#include "internal.hpp"

namespace nep {

struct Grid {
    double L[3];
    int nc[3];
    int ncell;
};

__device__ __forceinline__ int cell_axis(double x, double L, int nc, bool &bad)
{
    double s = x / L;
    s = s - floor(s);
    if (!(s >= 0.0) || !(s < 1.0)) {   // NaN / Inf positions, or s rounded up to 1
        bad = bad || !(s == s) || !(x - x == 0.0);
        s = 0.0;
    }
    int c = (int)(s * nc);
    return c >= nc ? nc - 1 : c;
}

__device__ __forceinline__ int cell_of(const double *p, const Grid &g, bool &bad)
{
    int cx = cell_axis(p[0], g.L[0], g.nc[0], bad);
    int cy = cell_axis(p[1], g.L[1], g.nc[1], bad);
    int cz = cell_axis(p[2], g.L[2], g.nc[2], bad);
    return (cz * g.nc[1] + cy) * g.nc[0] + cx;
}

// Minimum-image squared distance, IEEE FP64 without contraction.
__device__ __forceinline__ double mic_r2(const double *ri, const double *rj, const Grid &g)
{
#pragma clang fp contract(off)
    double dx = rj[0] - ri[0];
    double dy = rj[1] - ri[1];
    double dz = rj[2] - ri[2];
    double kx = rint(dx / g.L[0]);
    double ky = rint(dy / g.L[1]);
    double kz = rint(dz / g.L[2]);
    double sx = g.L[0] * kx;
    double sy = g.L[1] * ky;
    double sz = g.L[2] * kz;
    dx = dx - sx;
    dy = dy - sy;
    dz = dz - sz;
    double xx = dx * dx;
    double yy = dy * dy;
    double zz = dz * dz;
    return (xx + yy) + zz;
}

__device__ __forceinline__ int wave_max(int v)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__global__ void k_cell_count(const double *__restrict__ pos, const int32_t *__restrict__ types, int N, int S,
                             Grid g, int32_t *__restrict__ cell_cnt, uint32_t *__restrict__ status)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    bool bad = false;
    bool badt = false;
    if (i < N) {
        const double *p = pos + ((size_t)b * N + i) * 3;
        int c = cell_of(p, g, bad);
        atomicAdd(&cell_cnt[(size_t)b * g.ncell + c], 1);
        if (b == 0) {
            int t = types[i];
            badt = (t < 0 || t >= S);
        }
    }
    uint32_t f = (bad ? (uint32_t)NEP_FLAG_NONFINITE : 0u) | (badt ? (uint32_t)NEP_FLAG_BAD_TYPE : 0u);
    if (__any(f != 0) && f) atomicOr(&status[0], f);
}

__global__ __launch_bounds__(1024) void k_cell_scan(int32_t *__restrict__ cell_cnt, int32_t *__restrict__ cell_start,
                                                    int ncell)
{
    __shared__ int32_t part[1024];
    const int b = blockIdx.x, t = threadIdx.x;
    int32_t *cnt = cell_cnt + (size_t)b * ncell;
    int32_t *st = cell_start + (size_t)b * (ncell + 1);
    const int per = (ncell + 1023) / 1024;
    const int c0 = min(t * per, ncell), c1 = min(c0 + per, ncell);
    int s = 0;
    for (int c = c0; c < c1; ++c) s += cnt[c];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;
    for (int c = c0; c < c1; ++c) {
        st[c] = run;
        run += cnt[c];
        cnt[c] = 0;            // reused as fill counter
    }
    if (t == 1023) st[ncell] = part[1023];
}

__global__ void k_cell_fill(const double *__restrict__ pos, int N, Grid g, int32_t *__restrict__ cell_cnt,
                            const int32_t *__restrict__ cell_start, int32_t *__restrict__ cell_atoms)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= N) return;
    bool bad = false;
    int c = cell_of(pos + ((size_t)b * N + i) * 3, g, bad);
    int slot = atomicAdd(&cell_cnt[(size_t)b * g.ncell + c], 1);
    cell_atoms[(size_t)b * N + cell_start[(size_t)b * (g.ncell + 1) + c] + slot] = i;
}

// Sort the atoms of each cell ascending, so traversal order does not depend
// on the order in which atomics were served.
__global__ void k_cell_sort(int N, int ncell, const int32_t *__restrict__ cell_start, int32_t *__restrict__ cell_atoms)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (c >= ncell) return;
    const int32_t *st = cell_start + (size_t)b * (ncell + 1);
    int32_t *a = cell_atoms + (size_t)b * N;
    const int s0 = st[c], s1 = st[c + 1];
    for (int p = s0 + 1; p < s1; ++p) {
        int v = a[p];
        int q = p - 1;
        while (q >= s0 && a[q] > v) {
            a[q + 1] = a[q];
            --q;
        }
        a[q + 1] = v;
    }
}

__global__ __launch_bounds__(256) void k_nlist(const double *__restrict__ pos, const int32_t *__restrict__ types,
                                               int N, int S, Grid g, const int32_t *__restrict__ cell_start,
                                               const int32_t *__restrict__ cell_atoms, double rcR2, double rcA2,
                                               int capR, int capA, int32_t *__restrict__ cntR,
                                               int32_t *__restrict__ idxR, int32_t *__restrict__ cntA,
                                               int32_t *__restrict__ idxA, uint32_t *__restrict__ status)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    const bool valid = i < N;
    int nR[kMaxSpecies] = {0, 0, 0, 0};
    int nA[kMaxSpecies] = {0, 0, 0, 0};
    if (valid) {
        const double *pb = pos + (size_t)b * N * 3;
        const double ri[3] = {pb[3 * i], pb[3 * i + 1], pb[3 * i + 2]};
        bool bad = false;
        const int cx = cell_axis(ri[0], g.L[0], g.nc[0], bad);
        const int cy = cell_axis(ri[1], g.L[1], g.nc[1], bad);
        const int cz = cell_axis(ri[2], g.L[2], g.nc[2], bad);
        const int32_t *st = cell_start + (size_t)b * (g.ncell + 1);
        const int32_t *ca = cell_atoms + (size_t)b * N;
        const int offz = g.nc[2] >= 3 ? 3 : g.nc[2];
        const int offy = g.nc[1] >= 3 ? 3 : g.nc[1];
        const int offx = g.nc[0] >= 3 ? 3 : g.nc[0];
        for (int oz = 0; oz < offz; ++oz) {
            int z = cz + (g.nc[2] >= 3 ? oz - 1 : oz);
            z = z < 0 ? z + g.nc[2] : (z >= g.nc[2] ? z - g.nc[2] : z);
            for (int oy = 0; oy < offy; ++oy) {
                int y = cy + (g.nc[1] >= 3 ? oy - 1 : oy);
                y = y < 0 ? y + g.nc[1] : (y >= g.nc[1] ? y - g.nc[1] : y);
                for (int ox = 0; ox < offx; ++ox) {
                    int x = cx + (g.nc[0] >= 3 ? ox - 1 : ox);
                    x = x < 0 ? x + g.nc[0] : (x >= g.nc[0] ? x - g.nc[0] : x);
                    const int c = (z * g.nc[1] + y) * g.nc[0] + x;
                    const int s1 = st[c + 1];
                    for (int p = st[c]; p < s1; ++p) {
                        const int j = ca[p];
                        if (j == i) continue;
                        const double r2 = mic_r2(ri, pb + 3 * j, g);
                        if (r2 < rcR2) {
                            const int t = types[j];
                            if (t >= 0 && t < S) {
                                int k = 0;
#pragma unroll
                                for (int s = 0; s < kMaxSpecies; ++s)
                                    if (s == t) k = nR[s]++;
                                if (k < capR) idxR[(((size_t)b * S + t) * capR + k) * N + i] = j;
                                if (r2 < rcA2) {
                                    int ka = 0;
#pragma unroll
                                    for (int s = 0; s < kMaxSpecies; ++s)
                                        if (s == t) ka = nA[s]++;
                                    if (ka < capA) idxA[(((size_t)b * S + t) * capA + ka) * N + i] = j;
                                }
                            }
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < kMaxSpecies; ++s) {
            if (s < S) {
                cntR[((size_t)b * S + s) * N + i] = nR[s];
                cntA[((size_t)b * S + s) * N + i] = nA[s];
            }
        }
    }
    int mR = 0, mA = 0;
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) {
        mR = max(mR, nR[s]);
        mA = max(mA, nA[s]);
    }
    const int wR = wave_max(mR), wA = wave_max(mA);
    if ((threadIdx.x & 63) == 0) {
        if (wR > 0) atomicMax(&status[1], (uint32_t)wR);
        if (wA > 0) atomicMax(&status[2], (uint32_t)wA);
        if (wR > capR || wA > capA) atomicOr(&status[0], (uint32_t)NEP_FLAG_NEIGHBOR_OVERFLOW);
    }
}

}  // namespace nep

using namespace nep;

extern "C" int32_t neighbor_build(const nep_model *m, nep_nlist *nl, const double *pos, const double box[9],
                                  const int32_t *types, int32_t P, int32_t N, hipStream_t s)
{
    if (!m || !nl || !box) return fail(NEP_ERR_INVALID_ARG, "neighbor_build: null argument");
    if (P != nl->P || N != nl->N || nl->S != m->hp.n_species)
        return fail(NEP_ERR_INVALID_ARG, "neighbor_build: P=%d N=%d do not match the list (P=%d N=%d)", P, N,
                    nl->P, nl->N);
    if (P == 0 || N == 0) return NEP_OK;
    if (!pos || !types) return fail(NEP_ERR_INVALID_ARG, "neighbor_build: null array");
    Grid g;
    if (!box_lengths(box, g.L)) return fail(NEP_ERR_UNSUPPORTED, "neighbor_build: only orthorhombic cells");
    const double rc = m->hp.rc_radial > m->hp.rc_angular ? m->hp.rc_radial : m->hp.rc_angular;
    for (int a = 0; a < 3; ++a) {
        if (!(g.L[a] > 0.0) || !std::isfinite(g.L[a]))
            return fail(NEP_ERR_INVALID_ARG, "neighbor_build: bad box edge %g", g.L[a]);
        if (g.L[a] < 2.0 * rc)
            return fail(NEP_ERR_BOX_TOO_SMALL, "box edge %g is shorter than twice the cutoff %g", g.L[a], rc);
        int nc = (int)std::floor(g.L[a] / (rc * (1.0 + 1e-9)));
        g.nc[a] = nc < 1 ? 1 : (nc > 64 ? 64 : nc);
    }
    g.ncell = g.nc[0] * g.nc[1] * g.nc[2];
    if (g.ncell > nl->ncell_alloc) {
        if (nl->cell_cnt) (void)hipFree(nl->cell_cnt);
        if (nl->cell_start) (void)hipFree(nl->cell_start);
        nl->cell_cnt = nullptr;
        nl->cell_start = nullptr;
        nl->ncell_alloc = 0;
        NEP_HIP(hipMalloc(&nl->cell_cnt, sizeof(int32_t) * (size_t)P * g.ncell));
        NEP_HIP(hipMalloc(&nl->cell_start, sizeof(int32_t) * (size_t)P * (g.ncell + 1)));
        nl->ncell_alloc = g.ncell;
    }
    const double rcR2 = m->hp.rc_radial * m->hp.rc_radial;
    const double rcA2 = m->hp.rc_angular * m->hp.rc_angular;
    fill_i32(nl->cell_cnt, 0, (size_t)P * g.ncell, s);
    const dim3 ga(div_up(N, kBlock), P);
    {
        ProfScope ps_(K_CELL_COUNT, s);
        hipLaunchKernelGGL(k_cell_count, ga, dim3(kBlock), 0, s, pos, types, N, nl->S, g, nl->cell_cnt, nl->status);
    }
    {
        ProfScope ps_(K_CELL_SCAN, s);
        hipLaunchKernelGGL(k_cell_scan, dim3(P), dim3(1024), 0, s, nl->cell_cnt, nl->cell_start, g.ncell);
    }
    {
        ProfScope ps_(K_CELL_FILL, s);
        hipLaunchKernelGGL(k_cell_fill, ga, dim3(kBlock), 0, s, pos, N, g, nl->cell_cnt, nl->cell_start,
                           nl->cell_atoms);
    }
    {
        ProfScope ps_(K_CELL_SORT, s);
        hipLaunchKernelGGL(k_cell_sort, dim3(div_up(g.ncell, kBlock), P), dim3(kBlock), 0, s, N, g.ncell,
                           nl->cell_start, nl->cell_atoms);
    }
    {
        ProfScope ps_(K_NLIST, s);
        hipLaunchKernelGGL(k_nlist, ga, dim3(kBlock), 0, s, pos, types, N, nl->S, g, nl->cell_start, nl->cell_atoms,
                           rcR2, rcA2, nl->capR, nl->capA, nl->cntR, nl->idxR, nl->cntA, nl->idxA, nl->status);
    }
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}
