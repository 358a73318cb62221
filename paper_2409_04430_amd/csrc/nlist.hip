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
// search over the N centroids (radius rc_radial + 2D, the larger cutoff)
// gives each atom one candidate row, sorted by (species, index), and for
// every candidate the slot at which the atom sits in the candidate's own
// row.  Each bead then filters the row exactly into compact radial and
// angular lists (slot-major, so that lanes read them coalesced), with
// per-species block ends; each angular entry also carries the candidate
// slot and the reverse slot used to address the angular pair terms.
// D, the cell grid and the radius are computed on the device in the same
// call, so the launch sequence needs no host round trip.
//
// Kernels per call: centroids and D -> grid -> count atoms per cell -> scan
// -> scatter -> order each cell -> candidate rows (a workgroup per cell,
// stencil centroids staged in LDS) -> sort rows -> reverse slots ->
// per-bead exact lists.
#include "internal.hpp"

namespace nep {

struct HostGrid {
    double L[3], invL[3];
    int nc_cap[3];     // allocation bound: floor(L / rc) per axis, at most 64
    double rcR, rcA;
};

// Device grid record.  Words 0-3 and 7-9 describe the candidate rows of the
// last rebuild and persist across calls; 4-5 are per-call maxima; 6 is the
// rebuild decision of this call.
struct DevGrid {
    int nc[3];
    int ncell;
    uint32_t spread_bits;   // D of this call (float bits, atomicMax)
    uint32_t disp_bits;     // largest centroid displacement since the rebuild (float bits)
    int rebuild;            // 1: rebuild the candidate rows in this call
    float d_build;          // D at the last rebuild
    double R2;              // candidate radius squared of the last rebuild
    uint32_t rows_overflow; // a candidate row of the last rebuild was truncated
};
static_assert(sizeof(DevGrid) <= 16 * sizeof(uint32_t), "grid record exceeds its 16-word buffer");

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

// Centroid of each atom's ring polymer, its largest bead distance and its
// displacement from the centroid of the last rebuild (both rounded up).
__global__ void k_centroid(const double *__restrict__ pos, const int32_t *__restrict__ types, int P, int N, int S,
                           double *__restrict__ cen, const double *__restrict__ cen_ref, uint32_t *__restrict__ grid,
                           uint32_t *__restrict__ status)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t f = 0;
    float spread = 0.0f, disp = 0.0f;
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
        if (!finite) {
            f |= NEP_FLAG_NONFINITE;
        } else {
            spread = (float)sqrt(m2) * 1.000001f + 1e-7f;   // rounded up
            const double dx = c[0] - cen_ref[3 * i], dy = c[1] - cen_ref[3 * i + 1], dz = c[2] - cen_ref[3 * i + 2];
            const double d2 = dx * dx + dy * dy + dz * dz;
            disp = isfinite(d2) ? (float)sqrt(d2) * 1.000001f + 1e-7f : 3.0e38f;
        }
        const int t = types[i];
        if (t < 0 || t >= S) f |= NEP_FLAG_BAD_TYPE;
    }
    spread = wave_max_f(spread);
    disp = wave_max_f(disp);
    if ((threadIdx.x & 63) == 0 && spread > 0.0f) atomicMax(&grid[4], __float_as_uint(spread));
    if ((threadIdx.x & 63) == 0 && disp > 0.0f) atomicMax(&grid[5], __float_as_uint(disp));
    if (f) atomicOr(&status[0], f);
}

// Rebuild decision and, on a rebuild, the grid and candidate radius from the
// measured spread.  Candidate rows built with radius rc + 2 D0 + skin stay
// complete while 2 (D - D0) + 2 max|c - c0| <= skin (triangle inequality on
// the periodic centroid distance); otherwise they are rebuilt.
__global__ void k_grid(HostGrid g, double skin, int force, uint32_t *__restrict__ grid, uint32_t *__restrict__ status)
{
    DevGrid *dg = reinterpret_cast<DevGrid *>(grid);
    const float spread = __uint_as_float(dg->spread_bits);
    const float disp = __uint_as_float(dg->disp_bits);
    const double need = 2.0 * ((double)spread - (double)dg->d_build) + 2.0 * (double)disp;
    const int rebuild = force || !(need <= skin);
    dg->rebuild = rebuild;
    atomicMax(&status[4], dg->spread_bits);
    if (!rebuild) {
        // reused rows that were truncated keep the overflow flag raised
        if (dg->rows_overflow) atomicOr(&status[0], (uint32_t)NEP_FLAG_NEIGHBOR_OVERFLOW);
        return;
    }
    dg->rows_overflow = 0;
    const double rc = g.rcR > g.rcA ? g.rcR : g.rcA;
    const double R = rc + 2.0 * (double)spread + skin + 1e-9 * (1.0 + rc);
    int ncell = 1;
    for (int a = 0; a < 3; ++a) {
        int nc = (int)floor(g.L[a] / (R * (1.0 + 1e-9)));
        nc = nc < 1 ? 1 : (nc > g.nc_cap[a] ? g.nc_cap[a] : nc);
        dg->nc[a] = nc;
        ncell *= nc;
    }
    dg->ncell = ncell;
    dg->R2 = R * R;
    dg->d_build = spread;
    atomicAdd(&status[5], 1u);
}

__global__ void k_cell_count(const double *__restrict__ cen, int N, HostGrid g, const uint32_t *__restrict__ grid,
                             int32_t *__restrict__ cell_cnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const DevGrid *dg = reinterpret_cast<const DevGrid *>(grid);
    if (i >= N || !dg->rebuild) return;
    const int cx = cell_axis(cen[3 * i], g.L[0], g.invL[0], dg->nc[0]);
    const int cy = cell_axis(cen[3 * i + 1], g.L[1], g.invL[1], dg->nc[1]);
    const int cz = cell_axis(cen[3 * i + 2], g.L[2], g.invL[2], dg->nc[2]);
    atomicAdd(&cell_cnt[(cz * dg->nc[1] + cy) * dg->nc[0] + cx], 1);
}

__global__ __launch_bounds__(1024) void k_cell_scan(const uint32_t *__restrict__ grid, int32_t *__restrict__ cnt,
                                                    int32_t *__restrict__ st)
{
    __shared__ int32_t part[1024];
    if (!reinterpret_cast<const DevGrid *>(grid)->rebuild) return;   // whole workgroup
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
    const DevGrid *dg = reinterpret_cast<const DevGrid *>(grid);
    if (i >= N || !dg->rebuild) return;
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
    if (!reinterpret_cast<const DevGrid *>(grid)->rebuild || c >= reinterpret_cast<const DevGrid *>(grid)->ncell)
        return;
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

// Candidate rows.  One workgroup per cell; the centroids of its stencil
// cells (3 x 3 x 3, fewer along an axis with fewer than 3 cells) are staged
// in LDS when they fit, and each wavefront takes one atom of the cell at a
// time, its lanes testing 64 stencil atoms at once and appending the
// accepted ones by ballot + prefix popcount (stencil order; sorted later).
// A stencil too large for LDS is read from global memory instead.
constexpr int kStage = 2048;
__global__ __launch_bounds__(256) void k_candidates(const double *__restrict__ cen, const int32_t *__restrict__ types,
                                                    int N, int S, HostGrid g, uint32_t *__restrict__ grid,
                                                    const int32_t *__restrict__ cell_start,
                                                    const int32_t *__restrict__ cell_atoms, int capC,
                                                    int32_t *__restrict__ cand, int32_t *__restrict__ rowlen,
                                                    double *__restrict__ cen_ref, uint32_t *__restrict__ status)
{
    __shared__ double sx[kStage], sy[kStage], sz[kStage];
    __shared__ int32_t sw[kStage];
    __shared__ int32_t rs[28], rp[28];
    __shared__ int nrange;
    DevGrid *dg = reinterpret_cast<DevGrid *>(grid);
    const int c = blockIdx.x;
    if (!dg->rebuild || c >= dg->ncell) return;   // whole workgroup
    const int nc0 = dg->nc[0], nc1 = dg->nc[1], nc2 = dg->nc[2];
    const double R2 = dg->R2;
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
                    const int cc = (z * nc1 + y) * nc0 + x;
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
    // flat stencil position q -> index into cell_atoms
    auto at = [&](int q) {
        int r = 0;
        while (r + 1 < nr && rp[r + 1] <= q) ++r;
        return rs[r] + (q - rp[r]);
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
    const int a0 = cell_start[c], a1 = cell_start[c + 1];
    for (int a = a0 + wv; a < a1; a += blockDim.x >> 6) {
        const int i = cell_atoms[a];
        const double ci[3] = {cen[3 * i], cen[3 * i + 1], cen[3 * i + 2]};
        int32_t *row = cand + (size_t)i * capC;
        int cnt = 0;
        for (int q0 = 0; q0 < total; q0 += 64) {
            const int q = q0 + lane;
            bool ok = false;
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
                    double r2 = 0.0;
#pragma unroll
                    for (int e = 0; e < 3; ++e) {
                        double d = p[e] - ci[e];
                        d -= g.L[e] * rint(d * g.invL[e]);
                        r2 += d * d;
                    }
                    ok = r2 < R2;
                }
            }
            const uint64_t m = __ballot(ok);
            const int pos = cnt + __popcll(m & below);
            if (ok && pos < capC) row[pos] = w;
            cnt += __popcll(m);
        }
        if (lane == 0) {
            rowlen[i] = cnt;
            cen_ref[3 * i] = ci[0];
            cen_ref[3 * i + 1] = ci[1];
            cen_ref[3 * i + 2] = ci[2];
            atomicMax(&status[3], (uint32_t)cnt);
            if (cnt > capC) {
                atomicOr(&status[0], (uint32_t)NEP_FLAG_NEIGHBOR_OVERFLOW);
                atomicOr(&dg->rows_overflow, 1u);
            }
        }
    }
}

// Sort each candidate row by (species, index) and record the species block
// starts.  One wavefront per atom: rank sort (each element's position is the
// number of smaller keys), in LDS for rows up to kSortLds, otherwise through
// the atom's reverse-slot row as scratch (it is rewritten afterwards).
constexpr int kSortLds = 512;
__global__ __launch_bounds__(256) void k_sort_rows(const uint32_t *__restrict__ grid, int N, int S, int capC,
                                                   int32_t *__restrict__ cand, const int32_t *__restrict__ rowlen,
                                                   int32_t *__restrict__ off, int32_t *__restrict__ scratch)
{
    if (!reinterpret_cast<const DevGrid *>(grid)->rebuild) return;   // whole workgroup
    __shared__ int32_t buf[kBlock / 64][kSortLds];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * (kBlock / 64) + wv;
    if (i >= N) return;   // whole wavefront
    const int n = min(rowlen[i], capC);
    int32_t *row = cand + (size_t)i * capC;
    const bool lds = n <= kSortLds;
    int32_t *src = lds ? buf[wv] : scratch + (size_t)i * capC;
    for (int e = lane; e < n; e += 64) src[e] = row[e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // key: species above index; entries are distinct
    auto key = [](int32_t w) { return ((uint32_t)(w & 3) << 29) | (uint32_t)(w >> 2); };
    int cntS[kMaxSpecies] = {0, 0, 0, 0};
    for (int e = lane; e < n; e += 64) {
        const int32_t w = src[e];
        const uint32_t kw = key(w);
        int r = 0;
        for (int f = 0; f < n; ++f) r += key(src[f]) < kw;
        row[r] = w;
#pragma unroll
        for (int t = 0; t < kMaxSpecies; ++t) cntS[t] += (w & 3) == t;
    }
#pragma unroll
    for (int t = 0; t < kMaxSpecies; ++t)
        for (int o = 32; o > 0; o >>= 1) cntS[t] += __shfl_xor(cntS[t], o);
    if (lane == 0) {
        int run = 0;
        for (int t = 0; t < S; ++t) {
            off[(size_t)i * (kMaxSpecies + 1) + t] = run;
            run += cntS[t];
        }
        off[(size_t)i * (kMaxSpecies + 1) + S] = run;
    }
}

// Reverse slots: for candidate j of i (slot k), the slot of i in j's row,
// by binary search in the species block of i (ordered by index); -1 if i
// is missing (only when j's row overflowed).  One wavefront per atom.
__global__ __launch_bounds__(256) void k_reverse(const uint32_t *__restrict__ grid, int N, int capC,
                                                 const int32_t *__restrict__ types, const int32_t *__restrict__ cand,
                                                 const int32_t *__restrict__ off, int32_t *__restrict__ rev)
{
    if (!reinterpret_cast<const DevGrid *>(grid)->rebuild) return;   // whole workgroup
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (i >= N) return;
    const int ti = types[i] & 3;
    const int S1 = kMaxSpecies + 1;
    int n = 0;
    for (int t = 0; t < kMaxSpecies; ++t) n = max(n, off[(size_t)i * S1 + t + 1]);
    n = min(n, capC);
    for (int k = lane; k < n; k += 64) {
        const int j = cand[(size_t)i * capC + k] >> 2;
        const int32_t *rj = cand + (size_t)j * capC;
        int lo = min(off[(size_t)j * S1 + ti], capC), hi = min(off[(size_t)j * S1 + ti + 1], capC);
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((rj[mid] >> 2) < i) lo = mid + 1;
            else hi = mid;
        }
        rev[(size_t)i * capC + k] = (lo < min(off[(size_t)j * S1 + ti + 1], capC) && (rj[lo] >> 2) == i) ? lo : -1;
    }
}

// Per-bead exact lists.  One lane per (bead, atom); candidates are taken in
// batches so that several position loads are in flight at once.  The test
// runs first on the packed FP32 positions; only a pair whose FP32 squared
// distance lies within `margin` of a cutoff squared (far above the packed
// error bound) is decided by the FP64 test, so every decision equals the
// FP64 one.
constexpr int kFilterBatch = 8;
__global__ __launch_bounds__(256) void k_filter(const double *__restrict__ pos, const float4 *__restrict__ pos4,
                                                FineGrid fg, float margin, int N, int S, HostGrid g,
                                                const int32_t *__restrict__ cand, const int32_t *__restrict__ off,
                                                const int32_t *__restrict__ rev, int capC, int capR, int capA,
                                                double rcR2, double rcA2, int32_t *__restrict__ listR,
                                                int32_t *__restrict__ endR, int32_t *__restrict__ listA,
                                                int32_t *__restrict__ endA, int32_t *__restrict__ slotA,
                                                uint64_t *__restrict__ maskA, uint32_t *__restrict__ status)
{
    int b, tile;
    bead_tile(b, tile);
    const int i = tile * blockDim.x + threadIdx.x;
    int sR = 0, sA = 0;
    if (i < N) {
        const double *pb = pos + (size_t)b * N * 3;
        const float4 *p4 = pos4 + (size_t)b * N;
        const float4 pi = p4[i];
        const float rR2f = (float)rcR2, rA2f = (float)rcA2;
        const int32_t *row = cand + (size_t)i * capC;
        const int32_t *rrow = rev + (size_t)i * capC;
        const int32_t *oi = off + (size_t)i * (kMaxSpecies + 1);
        int32_t *lR = listR + (size_t)b * capR * N + i;
        int32_t *lA = listA + (size_t)b * capA * N + i;
        int32_t *sl = slotA + (size_t)b * capA * N + i;
        uint64_t *mk = maskA + (size_t)b * ((capC + 31) >> 5) * N + i;
        uint32_t word = 0;   // angular hits of the current 32-slot word
        int wcur = 0;        // index of that word
        int before = 0;      // angular hits in the words before it
        for (int t = 0; t < S; ++t) {
            const int k0 = min(oi[t], capC), k1 = min(oi[t + 1], capC);
            for (int kb = k0; kb < k1; kb += kFilterBatch) {
                int w[kFilterBatch];
                float4 pj[kFilterBatch];
#pragma unroll
                for (int u = 0; u < kFilterBatch; ++u) {
                    const int k = kb + u;
                    w[u] = row[k < k1 ? k : k0];
                    pj[u] = p4[w[u] >> 2];
                }
#pragma unroll
                for (int u = 0; u < kFilterBatch; ++u) {
                    const int k = kb + u;
                    if (k < k1) {
                        float dx, dy, dz;
                        packed_pair(pj[u], pi, fg.M, fg.h, dx, dy, dz);
                        const float r2f = dx * dx + dy * dy + dz * dz;
                        bool inR = r2f < rR2f, inA = r2f < rA2f;
                        if (fabsf(r2f - rR2f) <= margin || fabsf(r2f - rA2f) <= margin) {
                            const int j = w[u] >> 2;
                            const double ri[3] = {pb[3 * i], pb[3 * i + 1], pb[3 * i + 2]};
                            const double rj[3] = {pb[3 * j], pb[3 * j + 1], pb[3 * j + 2]};
                            const double r2 = mic_r2_exact(ri, rj, g);
                            inR = r2 < rcR2;
                            inA = r2 < rcA2;
                        }
                        while ((k >> 5) > wcur) {   // close the finished words
                            mk[(size_t)wcur * N] = (uint64_t)word | ((uint64_t)before << 32);
                            before += __popc(word);
                            word = 0;
                            ++wcur;
                        }
                        if (inR) {
                            if (sR < capR) lR[(size_t)sR * N] = w[u] >> 2;
                            ++sR;
                            if (inA) {
                                word |= 1u << (k & 31);
                                if (sA < capA) {
                                    lA[(size_t)sA * N] = w[u] >> 2;
                                    sl[(size_t)sA * N] = k | (int32_t)((uint32_t)(rrow[k] & 0xffff) << 16);
                                }
                                ++sA;
                            }
                        }
                    }
                }
            }
            endR[((size_t)b * kMaxSpecies + t) * N + i] = min(sR, capR);
            endA[((size_t)b * kMaxSpecies + t) * N + i] = min(sA, capA);
        }
        if (min(off[(size_t)i * (kMaxSpecies + 1) + S], capC) > 0)
            mk[(size_t)wcur * N] = (uint64_t)word | ((uint64_t)before << 32);
    }
    const int wR = wave_max_i(sR), wA = wave_max_i(sA);
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
    g.rcR = m->hp.rc_radial;
    g.rcA = m->hp.rc_angular;
    const double rc = g.rcR > g.rcA ? g.rcR : g.rcA;
    int ncell_cap = 1;
    for (int a = 0; a < 3; ++a) {
        if (!(g.L[a] > 0.0) || !std::isfinite(g.L[a]))
            return fail(NEP_ERR_INVALID_ARG, "neighbor_build: bad box edge %g", g.L[a]);
        if (g.L[a] < 2.0 * rc)
            return fail(NEP_ERR_BOX_TOO_SMALL, "box edge %g is shorter than twice the cutoff %g", g.L[a], rc);
        g.invL[a] = 1.0 / g.L[a];
        int nc = (int)std::floor(g.L[a] / (rc * (1.0 + 1e-9)));
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
    const FineGrid fg = fine_grid(g.L, rc);
    if (!fg.exact)
        return fail(NEP_ERR_BOX_TOO_SMALL, "box edges %g %g %g leave no margin over twice the cutoff %g", g.L[0],
                    g.L[1], g.L[2], rc);
    // decision margin for the FP32 prefilter: ~50x the packed error bound
    const double hmax = std::max(std::max(fg.hd[0], fg.hd[1]), fg.hd[2]);
    const float margin = (float)(1e-3 * std::max(1.0, hmax * hmax) * std::max(1.0, rc * rc / 36.0));
    // a changed box invalidates the candidate rows
    bool force = !nl->built;
    for (int a = 0; a < 3; ++a) force = force || g.L[a] != nl->box_built[a];
    fill_u32(nl->grid + 4, 0u, 2, s);
    pack_positions(pos, (size_t)P * N, fg, reinterpret_cast<float4 *>(nl->pos4), s);
    fill_i32(nl->cell_cnt, 0, (size_t)ncell_cap, s);
    const dim3 g1(div_up(N, kBlock));
    const dim3 gw(div_up(N, kBlock / 64));
    {
        ProfScope ps_(K_CENTROID, s);
        hipLaunchKernelGGL(k_centroid, g1, dim3(kBlock), 0, s, pos, types, P, N, nl->S, nl->cen, nl->cen_ref, nl->grid,
                           nl->status);
    }
    {
        ProfScope ps_(K_GRID, s);
        hipLaunchKernelGGL(k_grid, dim3(1), dim3(1), 0, s, g, nl->skin, force ? 1 : 0, nl->grid, nl->status);
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
        hipLaunchKernelGGL(k_candidates, dim3(ncell_cap), dim3(kBlock), 0, s, nl->cen, types, N, nl->S, g, nl->grid,
                           nl->cell_start, nl->cell_atoms, nl->capC, nl->cand, nl->rowlen, nl->cen_ref, nl->status);
    }
    {
        ProfScope ps_(K_SORT_ROWS, s);
        hipLaunchKernelGGL(k_sort_rows, gw, dim3(kBlock), 0, s, nl->grid, N, nl->S, nl->capC, nl->cand, nl->rowlen,
                           nl->offC, nl->revC);
    }
    {
        ProfScope ps_(K_REVERSE, s);
        hipLaunchKernelGGL(k_reverse, gw, dim3(kBlock), 0, s, nl->grid, N, nl->capC, types, nl->cand, nl->offC,
                           nl->revC);
    }
    {
        ProfScope ps_(K_NLIST, s);
        hipLaunchKernelGGL(k_filter, dim3(div_up(N, kBlock), P), dim3(kBlock), 0, s, pos,
                           reinterpret_cast<const float4 *>(nl->pos4), fg, margin, N, nl->S, g, nl->cand,
                           nl->offC, nl->revC, nl->capC, nl->capR, nl->capA, rcR2, rcA2, nl->listR, nl->endR,
                           nl->listA, nl->endA, nl->slotA, nl->maskA, nl->status);
    }
    NEP_HIP(hipGetLastError());
    nl->built = 1;
    for (int a = 0; a < 3; ++a) nl->box_built[a] = g.L[a];
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
