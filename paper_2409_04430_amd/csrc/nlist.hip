// Per-bead neighbour lists through ring-polymer centroids (orthorhombic box).
//
// Pairs are accepted by the literal FP64 minimum-image test
//   d = r_j - r_i;  d -= L * rint(d / L)  (per axis);  (dx*dx + dy*dy) + dz*dz < rc*rc
// without contraction, so the sets equal those of a brute-force search over
// all pairs of a bead.  The division is replaced by a multiply with 1/L
// whenever that provably gives the same integer (t = d/L farther than 1e-9
// from a half-integer and |t| < 2^20); otherwise the division runs.
//
// Candidates: the P beads of an atom stay within D of their centroid, so a
// bead pair closer than rc has centroids closer than rc + 2D.  One cell-list
// search over the N centroids (instead of P searches over N beads) gives a
// candidate list shared by every bead; each bead then filters it with the
// exact test.  D, the cell grid and the search radius are computed on the
// device in the same call (no host round trip), so the launch sequence can
// be captured in a graph.
//
// Kernels per call: centroids and D -> grid -> count atoms per cell ->
// scan -> scatter -> order each cell (rank sort, deterministic) ->
// centroid candidates -> per-bead exact filter into species-blocked,
// slot-major lists.
#include "internal.hpp"

namespace nep {

struct HostGrid {
    double L[3], invL[3];
    int nc_cap[3];     // allocation bound: floor(L / rc) per axis, at most 64
    double rc;         // largest cutoff
};

// Device grid record (written by k_grid): nc[3], ncell, spread (float bits), pad, R^2 (double).
struct DevGrid {
    int nc[3];
    int ncell;
    uint32_t spread_bits;
    uint32_t pad;
    double R2;
};

__device__ __forceinline__ int cell_axis(double x, double L, double invL, int nc)
{
    double s = x * invL;
    s = s - floor(s);
    if (!(s >= 0.0) || !(s < 1.0)) s = 0.0;   // NaN / Inf, or s rounded up to 1
    int c = (int)(s * nc);
    return c >= nc ? nc - 1 : c;
}

// Exact minimum-image squared distance (see the file comment).
__device__ __forceinline__ double mic_r2_exact(const double *ri, const double *rj, const HostGrid &g)
{
#pragma clang fp contract(off)
    double e2[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double d = rj[a] - ri[a];
        const double t = d * g.invL[a];
        double k = rint(t);
        const double off = t - k;
        if (!(fabs(off) < 0.499999999) || !(fabs(t) < 1048576.0)) k = rint(d / g.L[a]);
        const double sft = g.L[a] * k;
        const double e = d - sft;
        e2[a] = e * e;
    }
    return (e2[0] + e2[1]) + e2[2];
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

// Centroid of each atom's ring polymer and its largest bead distance.
__global__ void k_centroid(const double *__restrict__ pos, const int32_t *__restrict__ types, int P, int N, int S,
                           double *__restrict__ cen, uint32_t *__restrict__ grid, uint32_t *__restrict__ status)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t f = 0;
    float spread = 0.0f;
    if (i < N) {
        const size_t st = (size_t)N * 3;
        double c[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < P; ++b) {
            const double *p = pos + b * st + 3 * (size_t)i;
            c[0] += p[0];
            c[1] += p[1];
            c[2] += p[2];
        }
        const double inv = 1.0 / P;
        c[0] *= inv; c[1] *= inv; c[2] *= inv;
        double m2 = 0.0;
        for (int b = 0; b < P; ++b) {
            const double *p = pos + b * st + 3 * (size_t)i;
            const double dx = p[0] - c[0], dy = p[1] - c[1], dz = p[2] - c[2];
            m2 = fmax(m2, dx * dx + dy * dy + dz * dz);
        }
        cen[3 * i] = c[0];
        cen[3 * i + 1] = c[1];
        cen[3 * i + 2] = c[2];
        const bool finite = isfinite(c[0]) && isfinite(c[1]) && isfinite(c[2]) && isfinite(m2);
        if (!finite) f |= NEP_FLAG_NONFINITE;
        else spread = (float)sqrt(m2) * 1.000001f + 1e-7f;   // rounded up
        const int t = types[i];
        if (t < 0 || t >= S) f |= NEP_FLAG_BAD_TYPE;
    }
    spread = wave_max_f(spread);
    if ((threadIdx.x & 63) == 0 && spread > 0.0f) atomicMax(&grid[4], __float_as_uint(spread));
    if (f) atomicOr(&status[0], f);
}

// Grid and search radius from the measured spread.
__global__ void k_grid(HostGrid g, uint32_t *__restrict__ grid, uint32_t *__restrict__ status)
{
    DevGrid *dg = reinterpret_cast<DevGrid *>(grid);
    const float spread = __uint_as_float(dg->spread_bits);
    const double R = g.rc + 2.0 * (double)spread + 1e-9 * (1.0 + g.rc);
    int ncell = 1;
    for (int a = 0; a < 3; ++a) {
        int nc = (int)floor(g.L[a] / (R * (1.0 + 1e-9)));
        nc = nc < 1 ? 1 : (nc > g.nc_cap[a] ? g.nc_cap[a] : nc);
        dg->nc[a] = nc;
        ncell *= nc;
    }
    dg->ncell = ncell;
    dg->R2 = R * R;
    atomicMax(&status[4], dg->spread_bits);
}

__global__ void k_cell_count(const double *__restrict__ cen, int N, HostGrid g, const uint32_t *__restrict__ grid,
                             int32_t *__restrict__ cell_cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const DevGrid *dg = reinterpret_cast<const DevGrid *>(grid);
    const int cx = cell_axis(cen[3 * i], g.L[0], g.invL[0], dg->nc[0]);
    const int cy = cell_axis(cen[3 * i + 1], g.L[1], g.invL[1], dg->nc[1]);
    const int cz = cell_axis(cen[3 * i + 2], g.L[2], g.invL[2], dg->nc[2]);
    atomicAdd(&cell_cnt[(cz * dg->nc[1] + cy) * dg->nc[0] + cx], 1);
}

__global__ __launch_bounds__(1024) void k_cell_scan(const uint32_t *__restrict__ grid, int32_t *__restrict__ cnt,
                                                    int32_t *__restrict__ st)
{
    __shared__ int32_t part[1024];
    const int ncell = reinterpret_cast<const DevGrid *>(grid)->ncell;
    const int t = threadIdx.x;
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
        cnt[c] = 0;   // reused as fill counter
    }
    if (t == 1023) st[ncell] = part[1023];
}

__global__ void k_cell_fill(const double *__restrict__ cen, int N, HostGrid g, const uint32_t *__restrict__ grid,
                            int32_t *__restrict__ cell_cnt, const int32_t *__restrict__ cell_start,
                            int32_t *__restrict__ cell_atoms)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const DevGrid *dg = reinterpret_cast<const DevGrid *>(grid);
    const int cx = cell_axis(cen[3 * i], g.L[0], g.invL[0], dg->nc[0]);
    const int cy = cell_axis(cen[3 * i + 1], g.L[1], g.invL[1], dg->nc[1]);
    const int cz = cell_axis(cen[3 * i + 2], g.L[2], g.invL[2], dg->nc[2]);
    const int c = (cz * dg->nc[1] + cy) * dg->nc[0] + cx;
    const int slot = atomicAdd(&cell_cnt[c], 1);
    cell_atoms[cell_start[c] + slot] = i;
}

// Ascending order inside each cell by rank sort: lane e places element e at
// the number of smaller elements (entries are distinct atom indices).
constexpr int kRankMax = 1024;
__global__ __launch_bounds__(64) void k_cell_rank(const uint32_t *__restrict__ grid,
                                                  const int32_t *__restrict__ cell_start,
                                                  int32_t *__restrict__ cell_atoms)
{
    __shared__ int32_t v[kRankMax];
    __shared__ int32_t out[kRankMax];
    const int c = blockIdx.x;
    if (c >= reinterpret_cast<const DevGrid *>(grid)->ncell) return;
    const int s0 = cell_start[c], n = cell_start[c + 1] - s0;
    int32_t *a = cell_atoms + s0;
    if (n <= kRankMax) {
        for (int e = threadIdx.x; e < n; e += 64) v[e] = a[e];
        __syncthreads();
        for (int e = threadIdx.x; e < n; e += 64) {
            const int x = v[e];
            int r = 0;
            for (int k = 0; k < n; ++k) r += v[k] < x;
            out[r] = x;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < n; e += 64) a[e] = out[e];
    } else if (threadIdx.x == 0) {   // very crowded cell: serial insertion
        for (int p = 1; p < n; ++p) {
            const int x = a[p];
            int q = p - 1;
            while (q >= 0 && a[q] > x) {
                a[q + 1] = a[q];
                --q;
            }
            a[q + 1] = x;
        }
    }
}

// Candidates of atom i: centroids within R of its centroid (conservative
// test).  One wavefront per atom: the lanes take the members of each stencil
// cell together and append the accepted ones in order with a ballot and a
// prefix popcount, so the order is fixed (stencil order, ascending index in
// a cell).
__global__ __launch_bounds__(256) void k_candidates(const double *__restrict__ cen, const int32_t *__restrict__ types,
                                                    int N, int S, HostGrid g, const uint32_t *__restrict__ grid,
                                                    const int32_t *__restrict__ cell_start,
                                                    const int32_t *__restrict__ cell_atoms, int capC,
                                                    int32_t *__restrict__ cand, int32_t *__restrict__ candN,
                                                    uint32_t *__restrict__ status)
{
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (i >= N) return;   // whole wavefront
    const DevGrid *dg = reinterpret_cast<const DevGrid *>(grid);
    const int nc0 = dg->nc[0], nc1 = dg->nc[1], nc2 = dg->nc[2];
    const double R2 = dg->R2;
    const double ci[3] = {cen[3 * i], cen[3 * i + 1], cen[3 * i + 2]};
    const int cx = cell_axis(ci[0], g.L[0], g.invL[0], nc0);
    const int cy = cell_axis(ci[1], g.L[1], g.invL[1], nc1);
    const int cz = cell_axis(ci[2], g.L[2], g.invL[2], nc2);
    const int oz_n = nc2 >= 3 ? 3 : nc2, oy_n = nc1 >= 3 ? 3 : nc1, ox_n = nc0 >= 3 ? 3 : nc0;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int n = 0;
    for (int oz = 0; oz < oz_n; ++oz) {
        int z = cz + (nc2 >= 3 ? oz - 1 : oz);
        z = z < 0 ? z + nc2 : (z >= nc2 ? z - nc2 : z);
        for (int oy = 0; oy < oy_n; ++oy) {
            int y = cy + (nc1 >= 3 ? oy - 1 : oy);
            y = y < 0 ? y + nc1 : (y >= nc1 ? y - nc1 : y);
            for (int ox = 0; ox < ox_n; ++ox) {
                int x = cx + (nc0 >= 3 ? ox - 1 : ox);
                x = x < 0 ? x + nc0 : (x >= nc0 ? x - nc0 : x);
                const int c = (z * nc1 + y) * nc0 + x;
                const int p0 = cell_start[c], p1 = cell_start[c + 1];
                for (int base = p0; base < p1; base += 64) {
                    const int p = base + lane;
                    bool ok = false;
                    int w = 0;
                    if (p < p1) {
                        const int j = cell_atoms[p];
                        if (j != i) {
                            double r2 = 0.0;
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                double d = cen[3 * j + a] - ci[a];
                                d -= g.L[a] * rint(d * g.invL[a]);
                                r2 += d * d;
                            }
                            const int t = types[j];
                            ok = r2 < R2 && t >= 0 && t < S;
                            w = (j << 2) | t;
                        }
                    }
                    const uint64_t mball = __ballot(ok);
                    const int slot = n + __popcll(mball & below);
                    if (ok && slot < capC) cand[(size_t)slot * N + i] = w;
                    n += __popcll(mball);
                }
            }
        }
    }
    if (lane == 0) {
        candN[i] = n;
        atomicMax(&status[3], (uint32_t)n);
        if (n > capC) atomicOr(&status[0], (uint32_t)NEP_FLAG_NEIGHBOR_OVERFLOW);
    }
}

// Per-bead exact filter of the shared candidates.  Candidates are taken in
// batches so that several index and position loads are in flight at once.
constexpr int kFilterBatch = 8;
__global__ __launch_bounds__(256) void k_filter(const double *__restrict__ pos, int N, int S, HostGrid g,
                                                const int32_t *__restrict__ cand, const int32_t *__restrict__ candN,
                                                int capC, double rcR2, double rcA2, int capR, int capA,
                                                int32_t *__restrict__ cntR, int32_t *__restrict__ idxR,
                                                int32_t *__restrict__ cntA, int32_t *__restrict__ idxA,
                                                uint32_t *__restrict__ status)
{
    int b, tile;
    bead_tile(b, tile);
    const int i = tile * blockDim.x + threadIdx.x;
    int nR[kMaxSpecies] = {0, 0, 0, 0};
    int nA[kMaxSpecies] = {0, 0, 0, 0};
    if (i < N) {
        const double *pb = pos + (size_t)b * N * 3;
        const double ri[3] = {pb[3 * i], pb[3 * i + 1], pb[3 * i + 2]};
        const int nc = min(candN[i], capC);
        int32_t *oR = idxR + (size_t)b * S * capR * N + i;
        int32_t *oA = idxA + (size_t)b * S * capA * N + i;
        for (int k0 = 0; k0 < nc; k0 += kFilterBatch) {
            int w[kFilterBatch];
            double pj[kFilterBatch][3];
#pragma unroll
            for (int u = 0; u < kFilterBatch; ++u) w[u] = (k0 + u < nc) ? cand[(size_t)(k0 + u) * N + i] : -1;
#pragma unroll
            for (int u = 0; u < kFilterBatch; ++u) {
                const int j = w[u] >= 0 ? (w[u] >> 2) : i;
                pj[u][0] = pb[3 * j];
                pj[u][1] = pb[3 * j + 1];
                pj[u][2] = pb[3 * j + 2];
            }
#pragma unroll
            for (int u = 0; u < kFilterBatch; ++u) {
                if (w[u] < 0) continue;
                const int j = w[u] >> 2, t = w[u] & 3;
                const double r2 = mic_r2_exact(ri, pj[u], g);
                if (r2 < rcR2) {
                    int kr = 0;
#pragma unroll
                    for (int s = 0; s < kMaxSpecies; ++s)
                        if (s == t) kr = nR[s]++;
                    if (kr < capR) oR[((size_t)t * capR + kr) * N] = j;
                    if (r2 < rcA2) {
                        int ka = 0;
#pragma unroll
                        for (int s = 0; s < kMaxSpecies; ++s)
                            if (s == t) ka = nA[s]++;
                        if (ka < capA) oA[((size_t)t * capA + ka) * N] = j;
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
    const int wR = wave_max_i(mR), wA = wave_max_i(mA);
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
    HostGrid g;
    if (!box_lengths(box, g.L)) return fail(NEP_ERR_UNSUPPORTED, "neighbor_build: only orthorhombic cells");
    g.rc = m->hp.rc_radial > m->hp.rc_angular ? m->hp.rc_radial : m->hp.rc_angular;
    int ncell_cap = 1;
    for (int a = 0; a < 3; ++a) {
        if (!(g.L[a] > 0.0) || !std::isfinite(g.L[a]))
            return fail(NEP_ERR_INVALID_ARG, "neighbor_build: bad box edge %g", g.L[a]);
        if (g.L[a] < 2.0 * g.rc)
            return fail(NEP_ERR_BOX_TOO_SMALL, "box edge %g is shorter than twice the cutoff %g", g.L[a], g.rc);
        g.invL[a] = 1.0 / g.L[a];
        int nc = (int)std::floor(g.L[a] / (g.rc * (1.0 + 1e-9)));
        g.nc_cap[a] = nc < 1 ? 1 : (nc > 64 ? 64 : nc);
        ncell_cap *= g.nc_cap[a];
    }
    if (ncell_cap > nl->ncell_alloc) {
        if (nl->cell_cnt) (void)hipFree(nl->cell_cnt);
        if (nl->cell_start) (void)hipFree(nl->cell_start);
        nl->cell_cnt = nullptr;
        nl->cell_start = nullptr;
        nl->ncell_alloc = 0;
        NEP_HIP(hipMalloc(&nl->cell_cnt, sizeof(int32_t) * (size_t)ncell_cap));
        NEP_HIP(hipMalloc(&nl->cell_start, sizeof(int32_t) * (size_t)(ncell_cap + 1)));
        nl->ncell_alloc = ncell_cap;
    }
    const double rcR2 = m->hp.rc_radial * m->hp.rc_radial;
    const double rcA2 = m->hp.rc_angular * m->hp.rc_angular;
    fill_u32(nl->grid, 0u, 8, s);
    fill_i32(nl->cell_cnt, 0, (size_t)ncell_cap, s);
    const dim3 g1(div_up(N, kBlock));
    {
        ProfScope ps_(K_CENTROID, s);
        hipLaunchKernelGGL(k_centroid, g1, dim3(kBlock), 0, s, pos, types, P, N, nl->S, nl->cen, nl->grid, nl->status);
    }
    {
        ProfScope ps_(K_GRID, s);
        hipLaunchKernelGGL(k_grid, dim3(1), dim3(1), 0, s, g, nl->grid, nl->status);
    }
    {
        ProfScope ps_(K_CELL_COUNT, s);
        hipLaunchKernelGGL(k_cell_count, g1, dim3(kBlock), 0, s, nl->cen, N, g, nl->grid, nl->cell_cnt);
    }
    {
        ProfScope ps_(K_CELL_SCAN, s);
        hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(1024), 0, s, nl->grid, nl->cell_cnt, nl->cell_start);
    }
    {
        ProfScope ps_(K_CELL_FILL, s);
        hipLaunchKernelGGL(k_cell_fill, g1, dim3(kBlock), 0, s, nl->cen, N, g, nl->grid, nl->cell_cnt,
                           nl->cell_start, nl->cell_atoms);
    }
    {
        ProfScope ps_(K_CELL_SORT, s);
        hipLaunchKernelGGL(k_cell_rank, dim3(ncell_cap), dim3(64), 0, s, nl->grid, nl->cell_start, nl->cell_atoms);
    }
    {
        ProfScope ps_(K_CANDIDATES, s);
        hipLaunchKernelGGL(k_candidates, dim3(div_up(N, kBlock / 64)), dim3(kBlock), 0, s, nl->cen, types, N, nl->S,
                           g, nl->grid,
                           nl->cell_start, nl->cell_atoms, nl->capC, nl->cand, nl->candN, nl->status);
    }
    {
        ProfScope ps_(K_NLIST, s);
        hipLaunchKernelGGL(k_filter, dim3(div_up(N, kBlock), P), dim3(kBlock), 0, s, pos, N, nl->S, g, nl->cand,
                           nl->candN, nl->capC, rcR2, rcA2, nl->capR, nl->capA, nl->cntR, nl->idxR, nl->cntA,
                           nl->idxA, nl->status);
    }
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}
