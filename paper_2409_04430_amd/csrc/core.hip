// Host side of libneppimd.so: error state, model file, handle lifetimes.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>

#include "internal.hpp"

namespace nep {

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

bool box_lengths(const double box[9], double L[3])
{
    if (box[1] != 0.0 || box[2] != 0.0 || box[3] != 0.0 || box[5] != 0.0 || box[6] != 0.0 || box[7] != 0.0)
        return false;
    L[0] = box[0];
    L[1] = box[4];
    L[2] = box[8];
    return true;
}

bool cell_info(const double box[9], CellInfo &c)
{
#pragma clang fp contract(off)
    for (int k = 0; k < 9; ++k) {
        if (!std::isfinite(box[k])) return false;
        c.H[k] = box[k];
    }
    const double *H = c.H;
    c.tri = !(H[1] == 0.0 && H[2] == 0.0 && H[3] == 0.0 && H[5] == 0.0 && H[6] == 0.0 && H[7] == 0.0);
    // inverse from the cofactors (s = r G for row vectors)
    const double c00 = H[4] * H[8] - H[5] * H[7], c01 = H[5] * H[6] - H[3] * H[8], c02 = H[3] * H[7] - H[4] * H[6];
    const double det = H[0] * c00 + H[1] * c01 + H[2] * c02;
    if (!(det > 0.0) || !std::isfinite(det)) return false;
    c.vol = det;
    double *G = c.G;
    G[0] = c00 / det;
    G[3] = c01 / det;
    G[6] = c02 / det;
    G[1] = (H[2] * H[7] - H[1] * H[8]) / det;
    G[4] = (H[0] * H[8] - H[2] * H[6]) / det;
    G[7] = (H[1] * H[6] - H[0] * H[7]) / det;
    G[2] = (H[1] * H[5] - H[2] * H[4]) / det;
    G[5] = (H[2] * H[3] - H[0] * H[5]) / det;
    G[8] = (H[0] * H[4] - H[1] * H[3]) / det;
    for (int d = 0; d < 3; ++d) {
        const double *u = H + 3 * ((d + 1) % 3), *v = H + 3 * ((d + 2) % 3);
        const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
        c.w[d] = det / std::sqrt(cx * cx + cy * cy + cz * cz);
        c.len[d] = std::sqrt(H[3 * d] * H[3 * d] + H[3 * d + 1] * H[3 * d + 1] + H[3 * d + 2] * H[3 * d + 2]);
    }
    return true;
}

FineGrid fine_grid_cell(const CellInfo &c, double rc)
{
    if (!c.tri) {
        const double L[3] = {c.H[0], c.H[4], c.H[8]};
        return fine_grid(L, rc);
    }
    FineGrid g{};
    g.exact = 1;
    for (int d = 0; d < 3; ++d) {
        const double room = 0.5 * (0.5 * c.w[d] - rc);
        int M = 1023;
        if (room > 0.0) {
            const double need = std::ceil(std::max(c.w[d] / room, c.len[d] / 1.0));
            if (need <= 1023.0) M = std::max(1, (int)need);
            else g.exact = 0;
        } else {
            g.exact = 0;
        }
        g.M[d] = M;
        g.hd[d] = c.len[d] / M;
        g.h[d] = (float)g.hd[d];
        g.Minv[d] = M / c.len[d];
    }
    return g;
}

FineGrid fine_grid(const double L[3], double rc)
{
    FineGrid g{};
    g.exact = 1;
    for (int d = 0; d < 3; ++d) {
        const double room = 0.5 * (0.5 * L[d] - rc);
        const double hmax = std::min(1.0, room);
        int M = 1023;
        if (hmax > L[d] / 1023.0) M = (int)std::ceil(L[d] / hmax);
        else g.exact = 0;
        M = std::max(1, std::min(M, 1023));
        g.M[d] = M;
        g.h[d] = (float)(L[d] / M);
        g.Minv[d] = M / L[d];
        g.hd[d] = L[d] / M;
    }
    return g;
}


// ---------------------------------------------------------- profiling ---

static const char *kKernelNames[K_NUM] = {"fill",   "centroid", "candidates", "nlist",       "materialize",
                                          "descriptor", "force_ang", "force", "reduce",   "trpmd",
                                          "modes", "observables", "barostat", "rdf", "d3_cn", "d3_pair",
                                          "d3_cnforce", "d3_reduce"};
static std::atomic<int> g_prof_on{0};
static std::atomic<int> g_prof_only{-1};   // -1: every kind
static std::mutex g_prof_mu;
struct ProfRecord {
    int id;
    hipEvent_t e0, e1;
};
static std::vector<ProfRecord> g_prof_pending;
static std::vector<hipEvent_t> g_prof_pool;

static hipEvent_t prof_event()
{
    // caller holds g_prof_mu
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(int kid, hipStream_t stream) : id(kid), s(stream)
{
    if (kid < 0 || kid >= K_NUM) return;   // untimed launches
    if (!g_prof_on.load(std::memory_order_relaxed)) return;
    const int only = g_prof_only.load(std::memory_order_relaxed);
    if (only >= 0 && only != kid) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    e0 = prof_event();
    if (e0 && hipEventRecord(e0, s) != hipSuccess) {
        g_prof_pool.push_back(e0);
        e0 = nullptr;
    }
}

ProfScope::~ProfScope()
{
    if (!e0) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEvent_t e1 = prof_event();
    if (e1 && hipEventRecord(e1, s) == hipSuccess) {
        g_prof_pending.push_back({id, e0, e1});
    } else {
        g_prof_pool.push_back(e0);
        if (e1) g_prof_pool.push_back(e1);
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

void fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s)
{
    if (n == 0) return;
    unsigned g = (unsigned)((n + 255) / 256);
    ProfScope ps(K_FILL, s);
    hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, s, p, v, n);
}

void fill_i32(int32_t *p, int32_t v, size_t n, hipStream_t s)
{
    fill_u32(reinterpret_cast<uint32_t *>(p), (uint32_t)v, n, s);
}

// ---------------------------------------------------------------- model ---

static bool read_tokens(const char *path, std::vector<std::string> &tok)
{
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    while (std::getline(f, line)) {
        size_t p = line.find_first_not_of(" \t\r");
        if (p == std::string::npos || line[p] == '#') continue;
        std::istringstream ss(line);
        std::string w;
        while (ss >> w) tok.push_back(w);
    }
    return true;
}

struct TokReader {
    const std::vector<std::string> &t;
    size_t i = 0;
    bool ok = true;
    explicit TokReader(const std::vector<std::string> &tt) : t(tt) {}
    const std::string *next()
    {
        if (i >= t.size()) { ok = false; return nullptr; }
        return &t[i++];
    }
    void expect(const char *w)
    {
        const std::string *s = next();
        if (!s || *s != w) ok = false;
    }
    int geti()
    {
        const std::string *s = next();
        if (!s) return 0;
        char *e = nullptr;
        long v = strtol(s->c_str(), &e, 10);
        if (*e) ok = false;
        return (int)v;
    }
    double getd()
    {
        const std::string *s = next();
        if (!s) return 0.0;
        char *e = nullptr;
        double v = strtod(s->c_str(), &e);
        if (*e) ok = false;
        return v;
    }
};

// Kernel shapes compiled into the library, (n_max_radial, n_max_angular,
// four_body) with basis sizes 8 and l_max = 4, in order of descriptor length.
// A model of another shape runs on the first that contains it: its
// Chebyshev coefficients and network columns sit in the kernel shape's
// layout with zeros everywhere else, so every extra basis function, radial
// function, angular order or four-body entry contributes an exact zero (a
// zero coefficient times a finite basis value; a zero descriptor scale and
// a zero weight column for the extra descriptors, whose adjoints are then
// zero too).
static const int kKernelShapes[][3] = {{4, 4, 0}, {6, 4, 0}, {4, 4, 1}, {8, 6, 0}, {8, 8, 1}};

static int kernel_shape(const nep_hparams &h)
{
    for (int k = 0; k < (int)(sizeof kKernelShapes / sizeof kKernelShapes[0]); ++k) {
        const int *s = kKernelShapes[k];
        if (h.n_max_radial <= s[0] && h.n_max_angular <= s[1] && h.four_body <= s[2]) return k;
    }
    return -1;
}

static bool shape_supported(const nep_hparams &h)
{
    if (h.l_max < 1 || h.l_max > kLmax) return false;
    if (h.basis_radial < 1 || h.basis_radial > 8 || h.basis_angular < 1 || h.basis_angular > 8) return false;
    if (h.n_max_radial < 0 || h.n_max_angular < 0) return false;
    if (h.four_body != 0 && h.four_body != 1) return false;
    if (h.four_body && h.l_max < 2) return false;   // the four-body invariant couples l = 2 sums
    if (h.n_species < 1 || h.n_species > kMaxSpecies) return false;
    if (h.hidden < 1 || h.hidden > 512) return false;
    if (!(h.rc_angular > 0.0) || !(h.rc_radial >= h.rc_angular)) return false;
    return kernel_shape(h) >= 0;
}

static int descriptor_dim(const nep_hparams &h)
{
    return (h.n_max_radial + 1) + h.l_max * (h.n_max_angular + 1) + (h.four_body ? h.n_max_angular + 1 : 0);
}

// Offsets of the packed parameter blocks of a shape (the spherical-harmonic
// normalisations last).
static ParamLayout param_layout(const nep_hparams &h)
{
    const int S = h.n_species, H = h.hidden, D = descriptor_dim(h);
    ParamLayout o;
    int p = 0;
    o.cR = p; p += S * S * (h.n_max_radial + 1) * (h.basis_radial + 1);
    o.cA = p; p += S * S * (h.n_max_angular + 1) * (h.basis_angular + 1);
    o.qs = p; p += D;
    o.W0 = p; p += S * H * D;
    o.b0 = p; p += S * H;
    o.w1 = p; p += S * H;
    o.b1 = p; p += 1;
    o.sh = p; p += kNumSH;
    o.total = p;
    return o;
}

// Copy the parameters va of shape a (layout oa) into the zero-filled vb of
// the containing shape b (layout ob).  Descriptor order in both: radial n,
// then angular (l - 1)(n_max_angular + 1) + n, then four-body n.
static void embed_params(const nep_hparams &a, const ParamLayout &oa, const std::vector<float> &va,
                         const nep_hparams &b, const ParamLayout &ob, std::vector<float> &vb)
{
    const int S = a.n_species, H = a.hidden, Da = descriptor_dim(a), Db = descriptor_dim(b);
    const int aR = a.n_max_radial + 1, aA = a.n_max_angular + 1, bR = b.n_max_radial + 1, bA = b.n_max_angular + 1;
    vb.assign((size_t)ob.total, 0.0f);
    auto coef = [&](int offa, int offb, int na, int nb, int ka, int kb) {
        for (int tt = 0; tt < S * S; ++tt)
            for (int n = 0; n < na; ++n)
                for (int k = 0; k < ka; ++k) vb[offb + (tt * nb + n) * kb + k] = va[offa + (tt * na + n) * ka + k];
    };
    coef(oa.cR, ob.cR, aR, bR, a.basis_radial + 1, b.basis_radial + 1);
    coef(oa.cA, ob.cA, aA, bA, a.basis_angular + 1, b.basis_angular + 1);
    std::vector<int> col((size_t)Da);
    for (int n = 0; n < aR; ++n) col[n] = n;
    for (int l = 1; l <= a.l_max; ++l)
        for (int n = 0; n < aA; ++n) col[aR + (l - 1) * aA + n] = bR + (l - 1) * bA + n;
    if (a.four_body)
        for (int n = 0; n < aA; ++n) col[aR + a.l_max * aA + n] = bR + b.l_max * bA + n;
    for (int v = 0; v < Da; ++v) vb[ob.qs + col[v]] = va[oa.qs + v];
    for (int sm = 0; sm < S * H; ++sm)
        for (int v = 0; v < Da; ++v) vb[ob.W0 + sm * Db + col[v]] = va[oa.W0 + sm * Da + v];
    for (int x = 0; x < S * H; ++x) {
        vb[ob.b0 + x] = va[oa.b0 + x];
        vb[ob.w1 + x] = va[oa.w1 + x];
    }
    vb[ob.b1] = va[oa.b1];
}

// Orthonormal real spherical harmonics l = 1..4 as constant x polynomial;
// these are the constants, in m = -l..l order.
static void sh_norms(double *c)
{
    const double pi = M_PI;
    double v[kNumSH] = {
        std::sqrt(3 / (4 * pi)), std::sqrt(3 / (4 * pi)), std::sqrt(3 / (4 * pi)),
        0.5 * std::sqrt(15 / pi), 0.5 * std::sqrt(15 / pi), 0.25 * std::sqrt(5 / pi), 0.5 * std::sqrt(15 / pi),
        0.25 * std::sqrt(15 / pi),
        0.25 * std::sqrt(35 / (2 * pi)), 0.5 * std::sqrt(105 / pi), 0.25 * std::sqrt(21 / (2 * pi)),
        0.25 * std::sqrt(7 / pi), 0.25 * std::sqrt(21 / (2 * pi)), 0.25 * std::sqrt(105 / pi),
        0.25 * std::sqrt(35 / (2 * pi)),
        0.75 * std::sqrt(35 / pi), 0.75 * std::sqrt(35 / (2 * pi)), 0.75 * std::sqrt(5 / pi),
        0.75 * std::sqrt(5 / (2 * pi)), 3.0 / 16.0 * std::sqrt(1 / pi), 0.75 * std::sqrt(5 / (2 * pi)),
        0.375 * std::sqrt(5 / pi), 0.75 * std::sqrt(35 / (2 * pi)), 3.0 / 16.0 * std::sqrt(35 / pi)};
    for (int i = 0; i < kNumSH; ++i) c[i] = v[i];
}

}  // namespace nep

using namespace nep;

extern "C" const char *nep_last_error(void) { return g_err.c_str(); }

extern "C" int32_t nep_profile_enable(int32_t on)
{
    g_prof_on.store(on ? 1 : 0);
    return NEP_OK;
}

extern "C" int32_t nep_profile_select(int32_t id)
{
    if (id < -1 || id >= K_NUM) return fail(NEP_ERR_INVALID_ARG, "nep_profile_select: unknown kernel kind %d", id);
    g_prof_only.store(id);
    return NEP_OK;
}

extern "C" int32_t nep_profile_num_kernels(void) { return K_NUM; }

extern "C" const char *nep_profile_kernel_name(int32_t id)
{
    return (id >= 0 && id < K_NUM) ? kKernelNames[id] : "";
}

extern "C" int32_t nep_profile_read(double *total_ms, int64_t *launches, int32_t reset)
{
    if (!total_ms || !launches) return fail(NEP_ERR_INVALID_ARG, "nep_profile_read: null argument");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    static double acc_ms[K_NUM] = {0};
    static int64_t acc_n[K_NUM] = {0};
    for (auto &r : g_prof_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.e1) != hipSuccess || hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess)
            return fail(NEP_ERR_HIP, "nep_profile_read: event query failed");
        acc_ms[r.id] += ms;
        acc_n[r.id] += 1;
        g_prof_pool.push_back(r.e0);
        g_prof_pool.push_back(r.e1);
    }
    g_prof_pending.clear();
    for (int k = 0; k < K_NUM; ++k) {
        total_ms[k] = acc_ms[k];
        launches[k] = acc_n[k];
        if (reset) {
            acc_ms[k] = 0.0;
            acc_n[k] = 0;
        }
    }
    return NEP_OK;
}

extern "C" int32_t nep_load_params(const char *path, nep_model **out)
{
    if (!path || !out) return fail(NEP_ERR_INVALID_ARG, "nep_load_params: null argument");
    *out = nullptr;
    std::vector<std::string> tok;
    if (!read_tokens(path, tok)) return fail(NEP_ERR_PARAMS_FILE, "cannot open model file '%s'", path);
    TokReader r(tok);
    nep_hparams h{};
    r.expect("nep_pimd_model");
    if (r.geti() != 1) r.ok = false;
    r.expect("species"); h.n_species = r.geti();
    r.expect("cutoff"); h.rc_radial = r.getd(); h.rc_angular = r.getd();
    r.expect("n_max"); h.n_max_radial = r.geti(); h.n_max_angular = r.geti();
    r.expect("basis"); h.basis_radial = r.geti(); h.basis_angular = r.geti();
    r.expect("l_max"); h.l_max = r.geti();
    r.expect("four_body"); h.four_body = r.geti();
    r.expect("hidden"); h.hidden = r.geti();
    if (!r.ok) return fail(NEP_ERR_PARAMS_FILE, "malformed header in model file '%s'", path);
    if (!shape_supported(h))
        return fail(NEP_ERR_UNSUPPORTED,
                    "unsupported model shape (species %d, n_max %d/%d, basis %d/%d, l_max %d, four_body %d, "
                    "hidden %d, rc %g/%g)", h.n_species, h.n_max_radial, h.n_max_angular, h.basis_radial,
                    h.basis_angular, h.l_max, h.four_body, h.hidden, h.rc_radial, h.rc_angular);
    const int S = h.n_species, NR1 = h.n_max_radial + 1, NA1 = h.n_max_angular + 1;
    const int KR1 = h.basis_radial + 1, KA1 = h.basis_angular + 1, H = h.hidden;
    h.dim = descriptor_dim(h);
    const int D = h.dim;
    // the kernel shape that runs this model (its own when compiled)
    const int *ks = kKernelShapes[kernel_shape(h)];
    nep_hparams hk = h;
    hk.n_max_radial = ks[0];
    hk.n_max_angular = ks[1];
    hk.four_body = ks[2];
    hk.basis_radial = hk.basis_angular = 8;
    hk.l_max = kLmax;
    hk.dim = descriptor_dim(hk);
    const bool embedded = hk.n_max_radial != h.n_max_radial || hk.n_max_angular != h.n_max_angular ||
                          hk.four_body != h.four_body || hk.basis_radial != h.basis_radial ||
                          hk.basis_angular != h.basis_angular || hk.l_max != h.l_max;

    nep_model *m = new (std::nothrow) nep_model;
    if (!m) return fail(NEP_ERR_NOMEM, "host allocation failed");
    m->hp = hk;
    m->own = h;
    m->embedded = embedded;
    const ParamLayout oo = param_layout(h);
    std::vector<float> vo((size_t)oo.total, 0.0f);
    auto rd = [&](int off, int n) {
        for (int i = 0; i < n; ++i) vo[off + i] = (float)r.getd();
    };
    r.expect("c_radial"); rd(oo.cR, S * S * NR1 * KR1);
    r.expect("c_angular"); rd(oo.cA, S * S * NA1 * KA1);
    r.expect("q_scale"); rd(oo.qs, D);
    r.expect("ann");
    for (int s = 0; s < S; ++s) {
        rd(oo.W0 + s * H * D, H * D);
        rd(oo.b0 + s * H, H);
        rd(oo.w1 + s * H, H);
    }
    r.expect("b1"); rd(oo.b1, 1);
    if (!r.ok) {
        delete m;
        return fail(NEP_ERR_PARAMS_FILE, "malformed or truncated parameter blocks in '%s'", path);
    }
    m->off = param_layout(hk);
    const ParamLayout &o = m->off;
    if (embedded)
        embed_params(h, oo, vo, hk, o, m->host);
    else
        m->host.swap(vo);
    double shc[kNumSH];
    sh_norms(shc);
    for (int i = 0; i < kNumSH; ++i) m->host[o.sh + i] = (float)shc[i];

    hipError_t e = hipGetDevice(&m->device);
    if (e == hipSuccess) e = hipMalloc(&m->dev, sizeof(float) * (size_t)o.total);
    if (e == hipSuccess)
        e = hipMemcpy(m->dev, m->host.data(), sizeof(float) * (size_t)o.total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (m->dev) (void)hipFree(m->dev);
        delete m;
        return fail(e == hipErrorOutOfMemory ? NEP_ERR_NOMEM : NEP_ERR_HIP, "model upload failed: %s",
                    hipGetErrorString(e));
    }
    *out = m;
    return NEP_OK;
}

extern "C" int32_t nep_model_info(const nep_model *m, nep_hparams *out)
{
    if (!m || !out) return fail(NEP_ERR_INVALID_ARG, "nep_model_info: null argument");
    *out = m->embedded ? m->own : m->hp;
    return NEP_OK;
}

extern "C" void nep_model_destroy(nep_model *m)
{
    if (!m || m->cutoffs_only) return;   // a descriptor owned by its D3 handle
    if (m->dev) (void)hipFree(m->dev);
    if (m->w0b) (void)hipFree(m->w0b);
    delete m;
}

// First-layer weights as matrix-core operand fragments (16 x 16 x 32 BF16
// tiles; see mlp_frag_layout).  NEP_MLP_BF16_MFMA: one term per weight, the
// FP32 weight rounded to the nearest BF16 value (ties to even).
// NEP_MLP_FP32_MFMA: three terms whose sum is the FP32 weight exactly (the
// top 8 significant bits by truncation, then the top 8 of the remainder,
// then the rest, at most 8 bits).  Entry (species, term, block, lane, e):
//   forward block (ht, kc): W0[16 ht + lane % 16][32 kc + 8 (lane / 16) + e]
//   adjoint block (dt, hc): W0[mu][16 dt + lane % 16] with
//       mu = 32 hc + 4 (lane / 16) + e (e < 4), 32 hc + 16 + 4 (lane / 16) + e - 4 (e >= 4)
// zero outside the model's H x D weights.
__device__ __forceinline__ uint16_t bf16_term(float x, int term, int wt)
{
    if (wt == 1) {
        const uint32_t u = __float_as_uint(x);
        return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    }
    float r = x;
    uint32_t part = 0;
    for (int k = 0; k <= term; ++k) {
        part = __float_as_uint(r) & 0xffff0000u;
        r -= __uint_as_float(part);
    }
    return (uint16_t)(part >> 16);
}

__global__ void k_w0_frag(const float *__restrict__ W0, int S, int H, int D, int wt, MlpFrag fl,
                          uint16_t *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int per_term = fl.fwd_blocks + fl.adj_blocks;
    const int64_t total = (int64_t)S * wt * per_term * 512;
    if (t >= total) return;
    const int e = (int)(t & 7), lane = (int)((t >> 3) & 63);
    int64_t rest = t >> 9;
    const int blk = (int)(rest % per_term);
    rest /= per_term;
    const int term = (int)(rest % wt), s = (int)(rest / wt);
    int mu, v;
    if (blk < fl.fwd_blocks) {
        const int ht = blk / fl.KC, kc = blk - ht * fl.KC;
        mu = 16 * ht + (lane & 15);
        v = 32 * kc + 8 * (lane >> 4) + e;
    } else {
        const int b2 = blk - fl.fwd_blocks, dt = b2 / fl.HC, hc = b2 - dt * fl.HC;
        const int g = lane >> 4;
        mu = 32 * hc + (e < 4 ? 4 * g + e : 16 + 4 * g + e - 4);
        v = 16 * dt + (lane & 15);
    }
    const float w = (mu < H && v < D) ? W0[(size_t)s * H * D + (size_t)mu * D + v] : 0.0f;
    out[t] = bf16_term(w, term, wt);
}

extern "C" int32_t nep_model_set_mlp(nep_model *m, int32_t mode, hipStream_t s)
{
    if (!m) return fail(NEP_ERR_INVALID_ARG, "nep_model_set_mlp: null model");
    if (m->cutoffs_only) return fail(NEP_ERR_INVALID_ARG, "nep_model_set_mlp: a list cutoff descriptor has no network");
    const nep_hparams &h = m->hp;
    if (mode == NEP_MLP_FP32_AUTO) {
        // k_descriptor keeps the angular sums of up to five radial functions
        // in registers through a vector-unit network; the matrix-core network
        // needs those registers and parks the sums in memory, which pays only
        // where they are parked either way
        const bool fits = h.dim <= 64 && h.hidden <= 128;
        mode = (fits && h.n_max_angular + 1 > 5) ? NEP_MLP_FP32_MFMA : NEP_MLP_FP32;
    }
    if (mode == NEP_MLP_FP32) {
        m->mlp = mode;
        return NEP_OK;
    }
    if (mode != NEP_MLP_BF16_MFMA && mode != NEP_MLP_FP32_MFMA)
        return fail(NEP_ERR_INVALID_ARG, "nep_model_set_mlp: unknown mode %d", mode);
    if (h.dim > 64 || h.hidden > 128)
        return fail(NEP_ERR_UNSUPPORTED, "nep_model_set_mlp: the matrix-core network needs D <= 64 and H <= 128 "
                                         "(model has D = %d, H = %d)", h.dim, h.hidden);
    const int wt = mode == NEP_MLP_FP32_MFMA ? 3 : 1;
    const MlpFrag fl = mlp_frag_layout(h.dim, h.hidden, wt);
    const size_t n = (size_t)h.n_species * fl.species_stride;
    if (m->w0b && m->w0b_len < n) {
        (void)hipFree(m->w0b);
        m->w0b = nullptr;
        m->w0b_len = 0;
    }
    if (!m->w0b) {
        NEP_HIP(hipMalloc(&m->w0b, sizeof(uint16_t) * n));
        m->w0b_len = n;
    }
    hipLaunchKernelGGL(k_w0_frag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, m->dev + m->off.W0,
                       h.n_species, h.hidden, h.dim, wt, fl, m->w0b);
    NEP_HIP(hipGetLastError());
    m->mlp = mode;
    return NEP_OK;
}

extern "C" int32_t nep_model_mlp(const nep_model *m, int32_t *mode)
{
    if (!m || !mode) return fail(NEP_ERR_INVALID_ARG, "nep_model_mlp: null argument");
    if (m->cutoffs_only) return fail(NEP_ERR_INVALID_ARG, "nep_model_mlp: a list cutoff descriptor has no network");
    *mode = m->mlp;
    return NEP_OK;
}

// ----------------------------------------------------------- neighbour ---

template <class T>
static hipError_t dalloc(T **p, size_t n)
{
    return hipMalloc((void **)p, sizeof(T) * (n ? n : 1));
}

// Validates a batch partition: offsets [nsys+1], non-decreasing from 0.
int32_t check_offsets(int32_t nsys, const int32_t *off, const char *who)
{
    if (nsys < 1 || nsys > 4096 || !off) return fail(NEP_ERR_INVALID_ARG, "%s: bad system count %d", who, nsys);
    if (off[0] != 0) return fail(NEP_ERR_INVALID_ARG, "%s: offsets must start at 0", who);
    for (int s = 0; s < nsys; ++s)
        if (off[s + 1] < off[s]) return fail(NEP_ERR_INVALID_ARG, "%s: offsets must not decrease", who);
    if (off[nsys] > (1 << 28)) return fail(NEP_ERR_INVALID_ARG, "%s: too many atoms", who);
    return NEP_OK;
}

extern "C" int32_t nep_nlist_create_batched(const nep_model *m, int32_t P, int32_t nsys, const int32_t *off,
                                            int32_t capR, int32_t capA, nep_nlist **out)
{
    if (!m || !out) return fail(NEP_ERR_INVALID_ARG, "nep_nlist_create: null argument");
    const int32_t rc0 = check_offsets(nsys, off, "nep_nlist_create");
    if (rc0 != NEP_OK) return rc0;
    const int32_t N = off[nsys];
    if (P < 0 || P > kMaxBeads || capR < 1 || capA < 1 || capR > 8192 || capA > 8192)
        return fail(NEP_ERR_INVALID_ARG, "nep_nlist_create: bad sizes P=%d N=%d caps=%d/%d", P, N, capR, capA);
    *out = nullptr;
    nep_nlist *nl = new (std::nothrow) nep_nlist;
    if (!nl) return fail(NEP_ERR_NOMEM, "host allocation failed");
    nl->P = P; nl->N = N; nl->S = m->hp.n_species;
    nl->capR = capR; nl->capA = capA;
    nl->nsys = nsys;
    nl->off.assign(off, off + nsys + 1);
    nl->boxL.assign(9 * (size_t)nsys, 0.0);
    std::vector<int32_t> asys((size_t)N);
    for (int s = 0; s < nsys; ++s)
        for (int i = off[s]; i < off[s + 1]; ++i) asys[i] = s;
    const size_t Nn = (size_t)N, PN = (size_t)P * N;
    hipError_t e = hipGetDevice(&nl->device);
    if (e == hipSuccess) e = dalloc(&nl->geom, (size_t)nsys);
    if (e == hipSuccess) e = dalloc(&nl->atom_sys, Nn);
    if (e == hipSuccess && Nn) e = hipMemcpy(nl->atom_sys, asys.data(), sizeof(int32_t) * Nn, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = dalloc(&nl->cen, Nn * 3);
    if (e == hipSuccess) e = dalloc(&nl->spr, Nn);
    if (e == hipSuccess) e = dalloc(&nl->cmax, 2 * ((kCenLanes * Nn + kBlock - 1) / kBlock));
    if (e == hipSuccess) e = dalloc(&nl->cen_ref, Nn * 3);
    if (e == hipSuccess) e = dalloc(&nl->candR, Nn * capR);
    if (e == hipSuccess) e = dalloc(&nl->candRs, Nn * capR);
    if (e == hipSuccess) e = dalloc(&nl->candAs, Nn * capA);
    if (e == hipSuccess) e = dalloc(&nl->lenR, Nn);
    if (e == hipSuccess) e = dalloc(&nl->offR, Nn * (kMaxSpecies + 1));
    if (e == hipSuccess) e = dalloc(&nl->candA, Nn * capA);
    if (e == hipSuccess) e = dalloc(&nl->lenA, Nn);
    if (e == hipSuccess) e = dalloc(&nl->offA, Nn * (kMaxSpecies + 1));
    if (e == hipSuccess) e = dalloc(&nl->revA, Nn * capA);
    if (e == hipSuccess) e = dalloc(&nl->uniR, Nn * capR);
    if (e == hipSuccess) e = dalloc(&nl->umR, Nn * capR);
    if (e == hipSuccess) e = dalloc(&nl->umA, Nn * capA);
    if (e == hipSuccess) e = dalloc(&nl->uendR, Nn * kMaxSpecies);
    if (e == hipSuccess) e = dalloc(&nl->uniA, Nn * capA);
    if (e == hipSuccess) e = dalloc(&nl->uendA, Nn * kMaxSpecies);
    if (e == hipSuccess) e = dalloc(&nl->pairbuf, 4 * PN * capA);
    if (e == hipSuccess) e = dalloc(&nl->pos4, 4 * PN);
    if (e == hipSuccess) e = dalloc(&nl->cell_atoms, Nn);
    if (e == hipSuccess) e = dalloc(&nl->grid, 16 + kDevSysWords * (size_t)nsys);
    if (e == hipSuccess) e = dalloc(&nl->status, 8);
    if (e == hipSuccess) e = hipMemset(nl->status, 0, 8 * sizeof(uint32_t));
    // pair terms start at zero: a slot that a step with truncated rows leaves
    // unwritten then holds a finite stale value, never uninitialised bits
    if (e == hipSuccess && PN) e = hipMemset(nl->pairbuf, 0, sizeof(float) * 4 * PN * capA);
    if (e == hipSuccess) e = hipMemset(nl->grid, 0, (16 + kDevSysWords * (size_t)nsys) * sizeof(uint32_t));
    if (e == hipSuccess && Nn) e = hipMemset(nl->offR, 0, sizeof(int32_t) * Nn * (kMaxSpecies + 1));
    if (e == hipSuccess && Nn) e = hipMemset(nl->offA, 0, sizeof(int32_t) * Nn * (kMaxSpecies + 1));
    if (e == hipSuccess && Nn) e = hipMemset(nl->uendR, 0, sizeof(int32_t) * Nn * kMaxSpecies);
    if (e == hipSuccess && Nn) e = hipMemset(nl->uendA, 0, sizeof(int32_t) * Nn * kMaxSpecies);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        nep_nlist_destroy(nl);
        return fail(e == hipErrorOutOfMemory ? NEP_ERR_NOMEM : NEP_ERR_HIP, "nlist allocation failed: %s",
                    hipGetErrorString(e));
    }
    *out = nl;
    return NEP_OK;
}

extern "C" int32_t nep_nlist_create(const nep_model *m, int32_t P, int32_t N, int32_t capR, int32_t capA,
                                    nep_nlist **out)
{
    if (N < 0) return fail(NEP_ERR_INVALID_ARG, "nep_nlist_create: bad sizes P=%d N=%d", P, N);
    const int32_t off[2] = {0, N};
    return nep_nlist_create_batched(m, P, 1, off, capR, capA, out);
}

extern "C" void nep_nlist_destroy(nep_nlist *nl)
{
    if (!nl) return;
    for (void *p : {(void *)nl->geom, (void *)nl->atom_sys, (void *)nl->cell_sys, (void *)nl->cen, (void *)nl->spr, (void *)nl->cmax, (void *)nl->cen_ref, (void *)nl->candR, (void *)nl->candRs, (void *)nl->candAs, (void *)nl->lenR, (void *)nl->offR,
                    (void *)nl->candA, (void *)nl->lenA, (void *)nl->offA, (void *)nl->revA, (void *)nl->uniR,
                    (void *)nl->umR, (void *)nl->umA, (void *)nl->uendR, (void *)nl->uniA, (void *)nl->uendA, (void *)nl->pairbuf, (void *)nl->pos4, (void *)nl->posT,
                    (void *)nl->cell_cnt, (void *)nl->cell_start, (void *)nl->cell_atoms, (void *)nl->grid,
                    (void *)nl->status})
        if (p) (void)hipFree(p);
    delete nl;
}

extern "C" int32_t nep_nlist_view(const nep_nlist *nl, nep_nlist_layout *out)
{
    if (!nl || !out) return fail(NEP_ERR_INVALID_ARG, "nep_nlist_view: null argument");
    out->P = nl->P; out->N = nl->N; out->n_species = nl->S;
    out->cap_radial = nl->capR; out->cap_angular = nl->capA;
    out->cand_radial = nl->candR; out->cand_radial_off = nl->offR;
    out->cand_angular = nl->candA; out->cand_angular_off = nl->offA; out->cand_angular_rev = nl->revA;
    out->union_radial = nl->uniR; out->union_radial_end = nl->uendR;
    out->union_angular = nl->uniA; out->union_angular_end = nl->uendA;
    out->union_radial_mask = nl->umR; out->union_angular_mask = nl->umA;
    return NEP_OK;
}

extern "C" int32_t nep_nlist_poll(nep_nlist *nl, nep_nlist_status *out, int32_t clear, hipStream_t s)
{
    if (!nl || !out) return fail(NEP_ERR_INVALID_ARG, "nep_nlist_poll: null argument");
    uint32_t h[8];
    NEP_HIP(hipStreamSynchronize(s));
    NEP_HIP(hipMemcpy(h, nl->status, sizeof h, hipMemcpyDeviceToHost));
    out->flags = h[0];
    out->max_union_radial = (int32_t)h[1];
    out->max_union_angular = (int32_t)h[2];
    out->max_cand_radial = (int32_t)h[3];
    out->max_cand_angular = (int32_t)h[6];
    float spread;
    std::memcpy(&spread, &h[4], sizeof spread);
    out->bead_spread = spread;
    out->rebuilds = (int32_t)h[5];
    if (clear) {
        fill_u32(nl->status, 0u, 8, s);
        NEP_HIP(hipGetLastError());
        NEP_HIP(hipStreamSynchronize(s));
    }
    if (h[0] & NEP_FLAG_NEIGHBOR_OVERFLOW)
        return fail(NEP_ERR_NEIGHBOR_OVERFLOW, "candidate overflow (longest rows %u/%u, capacities %d/%d)", h[3],
                    h[6], nl->capR, nl->capA);
    return NEP_OK;
}

// ----------------------------------------------------------- workspace ---

// Tile table for `wpb` wavefronts per workgroup: each tile is up to
// wpb * 64 / G atoms of one system (G lanes per atom).  Synchronous upload.
static int32_t set_tiles(nep_ws *w, int wpb)
{
    const int apb = wpb * (64 >> lanes_log2(w->P > 0 ? w->P : 1));
    std::vector<int32_t> t0, t1, ts, st(w->nsys + 1, 0);
    for (int s = 0; s < w->nsys; ++s) {
        st[s] = (int32_t)t0.size();
        for (int a = w->off[s]; a < w->off[s + 1]; a += apb) {
            t0.push_back(a);
            t1.push_back(std::min(a + apb, w->off[s + 1]));
            ts.push_back(s);
        }
    }
    st[w->nsys] = (int32_t)t0.size();
    if ((int)t0.size() > std::max(w->nblk_cap, 1)) return fail(NEP_ERR_INVALID_ARG, "tile table overflow");
    if (w->B && t0.size() * (size_t)wpb > w->B_waves) return fail(NEP_ERR_INVALID_ARG, "adjoint rows overflow");
    NEP_HIP(hipDeviceSynchronize());
    if (!t0.empty()) {
        NEP_HIP(hipMemcpy(w->tile_atom0, t0.data(), sizeof(int32_t) * t0.size(), hipMemcpyHostToDevice));
        NEP_HIP(hipMemcpy(w->tile_atom1, t1.data(), sizeof(int32_t) * t1.size(), hipMemcpyHostToDevice));
        NEP_HIP(hipMemcpy(w->tile_sys, ts.data(), sizeof(int32_t) * ts.size(), hipMemcpyHostToDevice));
    }
    NEP_HIP(hipMemcpy(w->sys_tile0, st.data(), sizeof(int32_t) * st.size(), hipMemcpyHostToDevice));
    w->nblk = (int)t0.size();
    w->wpb = wpb;
    return NEP_OK;
}

extern "C" int32_t nep_ws_set_tile(nep_ws *w, int32_t waves_per_group)
{
    if (!w) return fail(NEP_ERR_INVALID_ARG, "nep_ws_set_tile: null argument");
    if (waves_per_group != 1 && waves_per_group != 2 && waves_per_group != 4)
        return fail(NEP_ERR_INVALID_ARG, "nep_ws_set_tile: waves per workgroup must be 1, 2 or 4");
    return set_tiles(w, waves_per_group);
}

extern "C" int32_t nep_ws_get_tile(const nep_ws *w, int32_t *waves_per_group)
{
    if (!w || !waves_per_group) return fail(NEP_ERR_INVALID_ARG, "nep_ws_get_tile: null argument");
    *waves_per_group = w->wpb;
    return NEP_OK;
}

extern "C" int32_t nep_ws_set_weight_staging(nep_ws *w, int32_t staging)
{
    if (!w) return fail(NEP_ERR_INVALID_ARG, "nep_ws_set_weight_staging: null argument");
    if (staging != NEP_WEIGHTS_LDS && staging != NEP_WEIGHTS_GLOBAL)
        return fail(NEP_ERR_INVALID_ARG, "nep_ws_set_weight_staging: unknown staging %d", staging);
    w->net_global = staging == NEP_WEIGHTS_GLOBAL;
    return NEP_OK;
}

extern "C" int32_t nep_ws_get_weight_staging(const nep_ws *w, int32_t *staging)
{
    if (!w || !staging) return fail(NEP_ERR_INVALID_ARG, "nep_ws_get_weight_staging: null argument");
    *staging = w->net_global ? NEP_WEIGHTS_GLOBAL : NEP_WEIGHTS_LDS;
    return NEP_OK;
}

extern "C" int32_t nep_ws_create_batched(const nep_model *m, int32_t P, int32_t nsys, const int32_t *off,
                                         nep_ws **out)
{
    if (!m || !out) return fail(NEP_ERR_INVALID_ARG, "nep_ws_create: null argument");
    if (m->cutoffs_only) return fail(NEP_ERR_INVALID_ARG, "nep_ws_create: a list cutoff descriptor has no network");
    const int32_t rc0 = check_offsets(nsys, off, "nep_ws_create");
    if (rc0 != NEP_OK) return rc0;
    const int32_t N = off[nsys];
    if (P < 0 || P > kMaxBeads) return fail(NEP_ERR_INVALID_ARG, "nep_ws_create: bad sizes P=%d N=%d", P, N);
    *out = nullptr;
    nep_ws *w = new (std::nothrow) nep_ws;
    if (!w) return fail(NEP_ERR_NOMEM, "host allocation failed");
    w->P = P; w->N = N; w->S = m->hp.n_species;
    w->NA1 = m->hp.n_max_angular + 1;
    w->nsys = nsys;
    w->off.assign(off, off + nsys + 1);
    const int apw = 64 >> lanes_log2(P > 0 ? P : 1);
    int cap = 0;
    for (int s = 0; s < nsys; ++s) cap += div_up(off[s + 1] - off[s], apw);
    w->nblk_cap = cap;
    const size_t nb = (size_t)std::max(cap, 1);
    const size_t PN = (size_t)P * N;
    hipError_t e = hipGetDevice(&w->device);
    if (e == hipSuccess) e = dalloc(&w->tile_atom0, nb);
    if (e == hipSuccess) e = dalloc(&w->tile_atom1, nb);
    if (e == hipSuccess) e = dalloc(&w->tile_sys, nb);
    if (e == hipSuccess) e = dalloc(&w->sys_tile0, (size_t)nsys + 1);
    if (e == hipSuccess && set_tiles(w, 4) != NEP_OK) e = hipErrorUnknown;
    // adjoint rows, one per lane of a launch (wavefront-interleaved): with
    // wpb wavefronts per workgroup a system takes at most wpb - 1 more
    // wavefronts than its count at one per workgroup
    w->B_waves = (size_t)cap + (size_t)3 * nsys;
    if (e == hipSuccess) e = dalloc(&w->B, w->B_waves * 64 * w->NA1 * kNumSH);
    if (e == hipSuccess) e = hipMemset(w->B, 0, sizeof(float) * w->B_waves * 64 * w->NA1 * kNumSH);
    // descriptor adjoints beside parked angular sums, the same lanes (room for the four-body entries)
    const size_t gq = (size_t)w->NA1 + (w->NA1 + 3) / 4;
    if (e == hipSuccess) e = dalloc(&w->Gad, w->B_waves * 64 * gq * 4);
    if (e == hipSuccess) e = hipMemset(w->Gad, 0, sizeof(float) * w->B_waves * 64 * gq * 4);
    if (e == hipSuccess) e = dalloc(&w->arad, PN * w->S * 12);
    if (e == hipSuccess) e = dalloc(&w->partE, (size_t)std::max(P, 1) * nb);
    if (e == hipSuccess) e = dalloc(&w->partW, (size_t)2 * std::max(P, 1) * nb * 9);
    if (e == hipSuccess) e = dalloc(&w->Fang, PN * 3);
    if (e == hipSuccess) e = dalloc(&w->flags, 4);
    if (e == hipSuccess) e = hipMemset(w->flags, 0, 4 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        nep_ws_destroy(w);
        return fail(e == hipErrorOutOfMemory ? NEP_ERR_NOMEM : NEP_ERR_HIP, "workspace allocation failed: %s",
                    hipGetErrorString(e));
    }
    *out = w;
    return NEP_OK;
}

extern "C" int32_t nep_ws_create(const nep_model *m, int32_t P, int32_t N, nep_ws **out)
{
    if (N < 0) return fail(NEP_ERR_INVALID_ARG, "nep_ws_create: bad sizes P=%d N=%d", P, N);
    const int32_t off[2] = {0, N};
    return nep_ws_create_batched(m, P, 1, off, out);
}

extern "C" void nep_ws_destroy(nep_ws *w)
{
    if (!w) return;
    for (void *p : {(void *)w->B, (void *)w->Gad, (void *)w->arad, (void *)w->partE, (void *)w->partW, (void *)w->Fang,
                    (void *)w->flags, (void *)w->tile_atom0, (void *)w->tile_atom1, (void *)w->tile_sys,
                    (void *)w->sys_tile0})
        if (p) (void)hipFree(p);
    delete w;
}

extern "C" int32_t nep_poll_flags(nep_ws *w, uint32_t *flags, int32_t clear, hipStream_t s)
{
    if (!w || !flags) return fail(NEP_ERR_INVALID_ARG, "nep_poll_flags: null argument");
    uint32_t h[4];
    NEP_HIP(hipStreamSynchronize(s));
    NEP_HIP(hipMemcpy(h, w->flags, sizeof h, hipMemcpyDeviceToHost));
    *flags = h[0];
    if (clear) {
        fill_u32(w->flags, 0u, 4, s);
        NEP_HIP(hipGetLastError());
        NEP_HIP(hipStreamSynchronize(s));
    }
    if (h[0] & NEP_FLAG_NONFINITE) return fail(NEP_ERR_NONFINITE, "non-finite force or position");
    return NEP_OK;
}
