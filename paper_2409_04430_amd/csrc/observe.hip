// Observables read off the neighbour lists: per species pair, the histogram
// of same-bead pair distances over every bead, from which the partial radial
// distribution functions of the water analysis (Sec. III) follow.
//
// Compiled without floating-point contraction: the distance of a pair is
// formed as x - L rint(x / L) per axis, then (dx^2 + dy^2) + dz^2 and sqrt,
// and its bin as floor(r * nbins / rmax), each step rounded separately.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "internal.hpp"

namespace nep {

// Scratch of nep_rdf_accumulate_noalloc: the bead-minor position copy in a
// file-scope device array instead of a list-owned allocation.  Each device
// holds its own copy from the first use until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns for the
// device (kept per device in g_rdf_scratch), never through the array's name.
constexpr size_t kRdfScratchBytes = (size_t)24 << 20;   // 24 MiB: P N <= 1,048,576 (bead, atom) rows
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kRdfScratchBytes / sizeof(double)];
static double *g_rdf_scratch[kMaxDevices];
static std::mutex g_rdf_scratch_mu;

// Device address of `scratch` on device dev (looked up once per device, with
// dev current); NEP_ERR_HIP if the lookup fails.
static int32_t rdf_scratch(int dev, double **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(NEP_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_rdf_scratch_mu);
    if (!g_rdf_scratch[dev]) {
        int cur = 0;
        NEP_HIP(hipGetDevice(&cur));
        if (cur != dev) NEP_HIP(hipSetDevice(dev));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) NEP_HIP(hipSetDevice(cur));
        if (e != hipSuccess || !p)
            return fail(NEP_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_rdf_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_rdf_scratch[dev];
    return NEP_OK;
}

constexpr int kRdfBlock = 256;
constexpr int kRdfMaxWords = 16384;   // S * S * nbins bins of 32-bit counts in LDS (64 KB)
constexpr int kRdfMaxGroups = 512;
constexpr int kRdfBatch = 8;

// Bead-minor copy of the positions, [N][P][3]: the beads of a neighbour are
// then one contiguous run for the lanes that gather them.
__global__ void k_beads_minor(const double *__restrict__ pos, double *__restrict__ posT, int P, int N)
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

// One lane per (atom, bead) in a grid-stride loop, the beads of an atom in
// G = 2^lg adjacent lanes.  Each lane walks its atom's radial union list in
// batches whose loads are in flight together, keeps the entries whose bead
// mask holds its bead, and counts the pair's bin in the workgroup's LDS
// histogram; the workgroup then adds its non-zero bins to the global 64-bit
// histogram.  Orthorhombic cells: the image shift is rint(x (1/L)); every
// listed pair is closer than the cutoff, far from the half-integer points
// where it could differ from rint(x / L), so the distance is the same double
// as with the division.  General cells: the fractional difference reduced by
// rint and mapped back, in the same order of operations as the list test.
struct RdfCell {
    double L[3], iL[3];     // orthorhombic: edges and their inverses
    double H[9], G[9];      // general: edge vectors as rows and H^-1
    int tri;
};

__global__ __launch_bounds__(kRdfBlock) void k_rdf(const double *__restrict__ posT, const int32_t *__restrict__ types,
                                                   int P, int N, int S, int lg, RdfCell cell,
                                                   double inv, int nbins, const int32_t *__restrict__ uni,
                                                   const uint64_t *__restrict__ um, const int32_t *__restrict__ uend,
                                                   int cap, unsigned long long *__restrict__ hist)
{
    extern __shared__ uint32_t h[];
    const int nw = S * S * nbins;
    for (int x = threadIdx.x; x < nw; x += blockDim.x) h[x] = 0u;
    __syncthreads();
    const int G = 1 << lg;
    const int64_t lanes = (int64_t)N << lg;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < lanes; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t >> lg), b = (int)(t & (G - 1));
        if (b >= P) continue;
        const int ti = types[i];
        if (ti < 0 || ti >= S) continue;
        const double *xi = posT + ((size_t)i * P + b) * 3;
        const double xi0 = xi[0], xi1 = xi[1], xi2 = xi[2];
        for (int tt = 0; tt < S; ++tt) {
            const int s0 = tt ? uend[(size_t)i * kMaxSpecies + tt - 1] : 0;
            const int s1 = uend[(size_t)i * kMaxSpecies + tt];
            const int base = (ti * S + tt) * nbins;
            for (int sb = s0; sb < s1; sb += kRdfBatch) {
                int jj[kRdfBatch];
                bool in[kRdfBatch];
#pragma unroll
                for (int u = 0; u < kRdfBatch; ++u) {
                    const bool ok = sb + u < s1;
                    const size_t at = (size_t)i * cap + (ok ? sb + u : s0);
                    jj[u] = ok ? uni[at] : i;
                    in[u] = ok && ((um[at] >> b) & 1u);
                }
                double xj[kRdfBatch][3];
#pragma unroll
                for (int u = 0; u < kRdfBatch; ++u) {
                    const double *pj = posT + ((size_t)jj[u] * P + b) * 3;
                    xj[u][0] = pj[0];
                    xj[u][1] = pj[1];
                    xj[u][2] = pj[2];
                }
#pragma unroll
                for (int u = 0; u < kRdfBatch; ++u) {
                    if (!in[u]) continue;
                    const double xv[3] = {xj[u][0] - xi0, xj[u][1] - xi1, xj[u][2] - xi2};
                    double d[3];
                    if (cell.tri) {
                        // fractional difference reduced by rint, mapped back
                        double f[3];
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const double sc = (xv[0] * cell.G[c] + xv[1] * cell.G[3 + c]) + xv[2] * cell.G[6 + c];
                            f[c] = sc - rint(sc);
                        }
#pragma unroll
                        for (int a = 0; a < 3; ++a)
                            d[a] = (f[0] * cell.H[a] + f[1] * cell.H[3 + a]) + f[2] * cell.H[6 + a];
                    } else {
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            const double k = rint(xv[a] * cell.iL[a]);
                            const double sh = cell.L[a] * k;
                            d[a] = xv[a] - sh;
                        }
                    }
                    const double xx = d[0] * d[0], yy = d[1] * d[1], zz = d[2] * d[2];
                    const double r2 = (xx + yy) + zz;
                    const double q = sqrt(r2) * inv;
                    if (q < nbins) atomicAdd(&h[base + (int)q], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < nw; x += blockDim.x)
        if (h[x]) atomicAdd(&hist[x], (unsigned long long)h[x]);
}

__global__ void k_centroid_beads(const double *__restrict__ x, double *__restrict__ out, int64_t M, int P)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= M) return;
    double s = 0.0;
    for (int j = 0; j < P; ++j) s += x[(size_t)j * M + e];
    out[e] = s / P;
}

}  // namespace nep

using namespace nep;

// Argument checks and the launches of the pair histogram, with the
// bead-minor copy of the positions at posT (null: the list's own copy,
// allocated on the first call).
static int32_t rdf_accumulate(const nep_model *m, nep_nlist *nl, const double *pos, const double box[9],
                              const int32_t *types, int32_t P, int32_t N, double rmax, int32_t nbins, uint64_t *hist,
                              double *posT, hipStream_t s)
{
    const int S = nl->S;
    if (nbins < 1 || (int64_t)S * S * nbins > kRdfMaxWords)
        return fail(NEP_ERR_INVALID_ARG, "nep_rdf_accumulate: %d bins x %d species pairs exceed %d", nbins, S * S,
                    kRdfMaxWords);
    const double rcR = m->hp.rc_radial;
    if (!(rmax > 0.0) || !(rmax <= rcR * (1.0 - 1e-9)))
        return fail(NEP_ERR_INVALID_ARG, "nep_rdf_accumulate: rmax %g must lie in (0, rc_radial (1 - 1e-9)], "
                                         "rc_radial = %g", rmax, rcR);
    for (int k = 0; k < 9; ++k)
        if (box[k] != nl->boxL[k])
            return fail(NEP_ERR_INVALID_ARG, "nep_rdf_accumulate: box differs from the last neighbor_build");
    CellInfo ci;
    if (!cell_info(box, ci)) return fail(NEP_ERR_INVALID_ARG, "nep_rdf_accumulate: bad cell");
    if (!nl->built) return fail(NEP_ERR_INVALID_ARG, "nep_rdf_accumulate: lists not built");
    if (!hist) return fail(NEP_ERR_INVALID_ARG, "nep_rdf_accumulate: null histogram");
    if (P == 0 || N == 0) return NEP_OK;
    if (!pos || !types) return fail(NEP_ERR_INVALID_ARG, "nep_rdf_accumulate: null array");
    int lg = 0;
    while ((1 << lg) < P) ++lg;
    const int64_t lanes = (int64_t)N << lg;
    const int groups = (int)std::min<int64_t>((lanes + kRdfBlock - 1) / kRdfBlock, kRdfMaxGroups);
    const size_t lds = sizeof(uint32_t) * (size_t)S * S * nbins;
    const bool own = !posT;   // the library's own copy; timed when kernel timing is on
    if (own) {
        if (!nl->posT) NEP_HIP(hipMalloc(&nl->posT, sizeof(double) * 3 * (size_t)N * P));   // first call only
        posT = nl->posT;
    }
    // the allocation-free form creates no timing events either
    ProfScope ps_(own ? K_RDF : K_NUM, s);
    const int64_t PN = (int64_t)P * N;
    hipLaunchKernelGGL(k_beads_minor, dim3((unsigned)((PN + 255) / 256)), dim3(256), 0, s, pos, posT, P, N);
    RdfCell cell{};
    cell.tri = ci.tri;
    for (int k = 0; k < 9; ++k) {
        cell.H[k] = ci.H[k];
        cell.G[k] = ci.G[k];
    }
    for (int a = 0; a < 3; ++a) {
        cell.L[a] = ci.H[4 * a];
        cell.iL[a] = 1.0 / ci.H[4 * a];
    }
    hipLaunchKernelGGL(k_rdf, dim3(groups), dim3(kRdfBlock), lds, s, posT, types, P, N, S, lg, cell, nbins / rmax,
                       nbins, nl->uniR, nl->umR, nl->uendR, nl->capR, reinterpret_cast<unsigned long long *>(hist));
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}

extern "C" int32_t nep_rdf_accumulate(const nep_model *m, nep_nlist *nl, const double *pos, const double box[9],
                                      const int32_t *types, int32_t P, int32_t N, double rmax, int32_t nbins,
                                      uint64_t *hist, hipStream_t s)
{
    if (!m || !nl || !box) return fail(NEP_ERR_INVALID_ARG, "nep_rdf_accumulate: null argument");
    if (P != nl->P || N != nl->N) return fail(NEP_ERR_INVALID_ARG, "nep_rdf_accumulate: P/N do not match the list");
    if (nl->nsys != 1) return fail(NEP_ERR_UNSUPPORTED, "nep_rdf_accumulate: one system per list");
    return rdf_accumulate(m, nl, pos, box, types, P, N, rmax, nbins, hist, nullptr, s);
}

extern "C" int32_t nep_rdf_accumulate_noalloc(const nep_model *m, nep_nlist *nl, const double *pos,
                                              const double box[9], const int32_t *types, int32_t P, int32_t N,
                                              double rmax, int32_t nbins, uint64_t *hist, hipStream_t s)
{
    if (!m || !nl || !box) return fail(NEP_ERR_INVALID_ARG, "nep_rdf_accumulate_noalloc: null argument");
    if (P != nl->P || N != nl->N)
        return fail(NEP_ERR_INVALID_ARG, "nep_rdf_accumulate_noalloc: P/N do not match the list");
    if (nl->nsys != 1) return fail(NEP_ERR_UNSUPPORTED, "nep_rdf_accumulate_noalloc: one system per list");
    const size_t need = sizeof(double) * 3 * (size_t)P * (size_t)N;
    if (need > kRdfScratchBytes)
        return fail(NEP_ERR_INVALID_ARG, "nep_rdf_accumulate_noalloc: P N = %lld (bead, atom) rows need %zu bytes "
                                         "of scratch, more than its %zu (at most %zu rows)",
                    (long long)P * N, need, kRdfScratchBytes, kRdfScratchBytes / (3 * sizeof(double)));
    double *posT = nullptr;
    const int32_t rc = rdf_scratch(nl->device, &posT);
    if (rc != NEP_OK) return rc;
    return rdf_accumulate(m, nl, pos, box, types, P, N, rmax, nbins, hist, posT, s);
}

extern "C" int32_t pimd_centroid(const pimd_ctx *c, const double *x, double *out, hipStream_t s)
{
    if (!c) return fail(NEP_ERR_INVALID_ARG, "pimd_centroid: null context");
    if (c->N == 0) return NEP_OK;
    if (!x || !out || x == out) return fail(NEP_ERR_INVALID_ARG, "pimd_centroid: bad arrays");
    const int64_t M = (int64_t)3 * c->N;
    hipLaunchKernelGGL(k_centroid_beads, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, x, out, M, c->P);
    NEP_HIP(hipGetLastError());
    return NEP_OK;
}
