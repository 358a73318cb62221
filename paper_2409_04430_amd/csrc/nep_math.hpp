// Device math shared by the NEP force kernels and the training kernels:
// the Chebyshev radial basis with its smooth cutoff, the real spherical
// harmonics l = 1..4 and their gradients, the adjoint contraction and the
// four-body helper (site-energy descriptors of Sec. II.C of arXiv:2409.04430).
#pragma once

#include "internal.hpp"

namespace nep {

constexpr float kPi = 3.14159265358979f;

// sin(pi z) and cos(pi z) for z in [0, 1]: with w = z - 1/2, cos(pi z) =
// -sin(pi w) and sin(pi z) = cos(pi w), and |pi w| <= pi/2, where the Taylor
// series through x^13 (sin) and x^14 (cos) is accurate to ~2e-7 in FP32.
__device__ __forceinline__ void sincospi01(float z, float &s, float &c)
{
    const float x = kPi * (z - 0.5f);
    const float x2 = x * x;
    float ps = (float)(-1.0 / 6227020800.0);
    ps = ps * x2 + (float)(1.0 / 39916800.0);
    ps = ps * x2 + (float)(-1.0 / 362880.0);
    ps = ps * x2 + (float)(1.0 / 5040.0);
    ps = ps * x2 + (float)(-1.0 / 120.0);
    ps = ps * x2 + (float)(1.0 / 6.0);
    float sw = x - x * x2 * ps;
    float pc = (float)(-1.0 / 87178291200.0);
    pc = pc * x2 + (float)(1.0 / 479001600.0);
    pc = pc * x2 + (float)(-1.0 / 3628800.0);
    pc = pc * x2 + (float)(1.0 / 40320.0);
    pc = pc * x2 + (float)(-1.0 / 720.0);
    pc = pc * x2 + (float)(1.0 / 24.0);
    pc = pc * x2 + (float)(-1.0 / 2.0);
    float cw = 1.0f + x2 * pc;
    c = -sw;
    s = cw;
}

// f_k(r) = (T_k(x) + 1)/2 f_c(r), x = 2 (r/rc - 1)^2 - 1, f_c = (1 + cos(pi r/rc))/2.
template <int K1>
__device__ __forceinline__ void cheb_f(float r, float rcinv, float *f)
{
    float sn, cs;
    const float z = r * rcinv;
    sincospi01(z, sn, cs);
    const float fc = 0.5f + 0.5f * cs;
    const float y = z - 1.0f;
    const float x = 2.0f * y * y - 1.0f;
    float t0 = 1.0f, t1 = x;
    f[0] = fc;
    if (K1 > 1) f[1] = 0.5f * (x + 1.0f) * fc;
#pragma unroll
    for (int k = 2; k < K1; ++k) {
        const float t2 = 2.0f * x * t1 - t0;
        f[k] = 0.5f * (t2 + 1.0f) * fc;
        t0 = t1;
        t1 = t2;
    }
}

// The cutoff function and the Chebyshev polynomials alone:
// f_c(r) and T_k(x), x = 2 (r/rc - 1)^2 - 1, so that f_k = (T_k + 1)/2 f_c.
// Sums of f_k then follow from sums of f_c T_k and of f_c.
template <int K1>
__device__ __forceinline__ void cheb_t(float r, float rcinv, float &fc, float *T)
{
    float sn, cs;
    const float z = r * rcinv;
    sincospi01(z, sn, cs);
    fc = 0.5f + 0.5f * cs;
    const float y = z - 1.0f;
    const float x = 2.0f * y * y - 1.0f;
    const float x2 = x + x;
    T[0] = 1.0f;
    if (K1 > 1) T[1] = x;
#pragma unroll
    for (int k = 2; k < K1; ++k) T[k] = fmaf(x2, T[k - 1], -T[k - 2]);
}

// f_c, df_c/dr, dx/dr, T_k(x) and T_k'(x) (T_{k+1}' = 2 T_k + 2x T_k' - T_{k-1}'),
// so that df_k/dr = (T_k' dx/dr f_c + (T_k + 1) df_c/dr) / 2.
template <int K1>
__device__ __forceinline__ void cheb_td(float r, float rcinv, float &fc, float &fcp, float &dxdr, float *T, float *Tp)
{
    float sn, cs;
    const float z = r * rcinv;
    sincospi01(z, sn, cs);
    fc = 0.5f + 0.5f * cs;
    fcp = -0.5f * kPi * rcinv * sn;
    const float y = z - 1.0f;
    const float x = 2.0f * y * y - 1.0f;
    dxdr = 4.0f * y * rcinv;
    const float x2 = x + x;
    T[0] = 1.0f;
    Tp[0] = 0.0f;
    if (K1 > 1) {
        T[1] = x;
        Tp[1] = 1.0f;
    }
#pragma unroll
    for (int k = 2; k < K1; ++k) {
        T[k] = fmaf(x2, T[k - 1], -T[k - 2]);
        Tp[k] = fmaf(x2, Tp[k - 1], fmaf(2.0f, T[k - 1], -Tp[k - 2]));
    }
}

// f_k and df_k/dr.
template <int K1>
__device__ __forceinline__ void cheb_fd(float r, float rcinv, float *f, float *fp)
{
    float sn, cs;
    const float z = r * rcinv;
    sincospi01(z, sn, cs);
    const float fc = 0.5f + 0.5f * cs;
    const float fcp = -0.5f * kPi * rcinv * sn;
    const float y = z - 1.0f;
    const float x = 2.0f * y * y - 1.0f;
    const float dx = 4.0f * y * rcinv;
    float t0 = 1.0f, t1 = x, d0 = 0.0f, d1 = 1.0f;
    f[0] = fc;
    fp[0] = fcp;
    if (K1 > 1) {
        f[1] = 0.5f * (x + 1.0f) * fc;
        fp[1] = 0.5f * dx * fc + 0.5f * (x + 1.0f) * fcp;
    }
#pragma unroll
    for (int k = 2; k < K1; ++k) {
        const float t2 = 2.0f * x * t1 - t0;
        const float d2 = 2.0f * t1 + 2.0f * x * d1 - d0;
        f[k] = 0.5f * (t2 + 1.0f) * fc;
        fp[k] = 0.5f * d2 * dx * fc + 0.5f * (t2 + 1.0f) * fcp;
        t0 = t1; t1 = t2;
        d0 = d1; d1 = d2;
    }
}

// Normalisations of 1 for sh_eval / adjoint_contract: the bare polynomials
// p_m of Y_m = c_m p_m (the multiplications fold away), for sums that apply
// c_m once after the neighbour loop.
struct UnitNorm {
    __device__ constexpr float operator[](int) const { return 1.0f; }
};

// Real spherical harmonics l = 1..4 (m = -l..l) at unit vector (x, y, z);
// c holds the normalisations (a generic or constant-space pointer, or
// UnitNorm for the bare polynomials).
template <typename CP>
__device__ __forceinline__ void sh_eval(float x, float y, float z, CP c, float *Y)
{
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    Y[0] = c[0] * y;
    Y[1] = c[1] * z;
    Y[2] = c[2] * x;
    Y[3] = c[3] * x * y;
    Y[4] = c[4] * y * z;
    Y[5] = c[5] * (3.0f * z2 - 1.0f);
    Y[6] = c[6] * x * z;
    Y[7] = c[7] * (x2 - y2);
    Y[8] = c[8] * y * (3.0f * x2 - y2);
    Y[9] = c[9] * x * y * z;
    Y[10] = c[10] * y * (5.0f * z2 - 1.0f);
    Y[11] = c[11] * z * (5.0f * z2 - 3.0f);
    Y[12] = c[12] * x * (5.0f * z2 - 1.0f);
    Y[13] = c[13] * z * (x2 - y2);
    Y[14] = c[14] * x * (x2 - 3.0f * y2);
    Y[15] = c[15] * x * y * (x2 - y2);
    Y[16] = c[16] * y * z * (3.0f * x2 - y2);
    Y[17] = c[17] * x * y * (7.0f * z2 - 1.0f);
    Y[18] = c[18] * y * z * (7.0f * z2 - 3.0f);
    Y[19] = c[19] * (35.0f * z2 * z2 - 30.0f * z2 + 3.0f);
    Y[20] = c[20] * x * z * (7.0f * z2 - 3.0f);
    Y[21] = c[21] * (x2 - y2) * (7.0f * z2 - 1.0f);
    Y[22] = c[22] * x * z * (x2 - 3.0f * y2);
    Y[23] = c[23] * (x2 * (x2 - 3.0f * y2) - y2 * (3.0f * x2 - y2));
}

// Contraction of the own adjoints with the harmonics of one pair, one m at a
// time so that no per-m array stays live:
//   sY = sum_m (sum_n B_nm g'_n) Y_m(u),  grad = sum_m (sum_n B_nm g_n) c_m grad p_m(u)
// (p_m the polynomial of Y_m = c_m p_m, differentiated on R^3).
template <int NA1, typename CP>
__device__ __forceinline__ void adjoint_contract(float x, float y, float z, CP c,
                                                 const float (*B)[kNumSH], const float *g, const float *gp, float &sY,
                                                 float &gx, float &gy, float &gz)
{
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    const float xy = x * y, yz = y * z, xz = x * z;
    sY = 0.0f;
    gx = 0.0f;
    gy = 0.0f;
    gz = 0.0f;
    {  // m = 0
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][0], g[n], bm);
            bpm = fmaf(B[n][0], gp[n], bpm);
        }
        sY = fmaf(bpm, c[0] * (y), sY);
        const float w = bm * c[0];
        gy += w;
    }
    {  // m = 1
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][1], g[n], bm);
            bpm = fmaf(B[n][1], gp[n], bpm);
        }
        sY = fmaf(bpm, c[1] * (z), sY);
        const float w = bm * c[1];
        gz += w;
    }
    {  // m = 2
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][2], g[n], bm);
            bpm = fmaf(B[n][2], gp[n], bpm);
        }
        sY = fmaf(bpm, c[2] * (x), sY);
        const float w = bm * c[2];
        gx += w;
    }
    {  // m = 3
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][3], g[n], bm);
            bpm = fmaf(B[n][3], gp[n], bpm);
        }
        sY = fmaf(bpm, c[3] * (x * y), sY);
        const float w = bm * c[3];
        gx += w * (y);
        gy += w * (x);
    }
    {  // m = 4
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][4], g[n], bm);
            bpm = fmaf(B[n][4], gp[n], bpm);
        }
        sY = fmaf(bpm, c[4] * (y * z), sY);
        const float w = bm * c[4];
        gy += w * (z);
        gz += w * (y);
    }
    {  // m = 5
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][5], g[n], bm);
            bpm = fmaf(B[n][5], gp[n], bpm);
        }
        sY = fmaf(bpm, c[5] * ((3.0f * z2 - 1.0f)), sY);
        const float w = bm * c[5];
        gz += w * (6.0f * z);
    }
    {  // m = 6
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][6], g[n], bm);
            bpm = fmaf(B[n][6], gp[n], bpm);
        }
        sY = fmaf(bpm, c[6] * (x * z), sY);
        const float w = bm * c[6];
        gx += w * (z);
        gz += w * (x);
    }
    {  // m = 7
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][7], g[n], bm);
            bpm = fmaf(B[n][7], gp[n], bpm);
        }
        sY = fmaf(bpm, c[7] * ((x2 - y2)), sY);
        const float w = bm * c[7];
        gx += w * (2.0f * x);
        gy -= w * (2.0f * y);
    }
    {  // m = 8
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][8], g[n], bm);
            bpm = fmaf(B[n][8], gp[n], bpm);
        }
        sY = fmaf(bpm, c[8] * (y * (3.0f * x2 - y2)), sY);
        const float w = bm * c[8];
        gx += w * (6.0f * xy);
        gy += w * (3.0f * (x2 - y2));
    }
    {  // m = 9
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][9], g[n], bm);
            bpm = fmaf(B[n][9], gp[n], bpm);
        }
        sY = fmaf(bpm, c[9] * (x * y * z), sY);
        const float w = bm * c[9];
        gx += w * (yz);
        gy += w * (xz);
        gz += w * (xy);
    }
    {  // m = 10
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][10], g[n], bm);
            bpm = fmaf(B[n][10], gp[n], bpm);
        }
        sY = fmaf(bpm, c[10] * (y * (5.0f * z2 - 1.0f)), sY);
        const float w = bm * c[10];
        gy += w * ((5.0f * z2 - 1.0f));
        gz += w * (10.0f * yz);
    }
    {  // m = 11
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][11], g[n], bm);
            bpm = fmaf(B[n][11], gp[n], bpm);
        }
        sY = fmaf(bpm, c[11] * (z * (5.0f * z2 - 3.0f)), sY);
        const float w = bm * c[11];
        gz += w * ((15.0f * z2 - 3.0f));
    }
    {  // m = 12
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][12], g[n], bm);
            bpm = fmaf(B[n][12], gp[n], bpm);
        }
        sY = fmaf(bpm, c[12] * (x * (5.0f * z2 - 1.0f)), sY);
        const float w = bm * c[12];
        gx += w * ((5.0f * z2 - 1.0f));
        gz += w * (10.0f * xz);
    }
    {  // m = 13
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][13], g[n], bm);
            bpm = fmaf(B[n][13], gp[n], bpm);
        }
        sY = fmaf(bpm, c[13] * (z * (x2 - y2)), sY);
        const float w = bm * c[13];
        gx += w * (2.0f * xz);
        gy -= w * (2.0f * yz);
        gz += w * ((x2 - y2));
    }
    {  // m = 14
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][14], g[n], bm);
            bpm = fmaf(B[n][14], gp[n], bpm);
        }
        sY = fmaf(bpm, c[14] * (x * (x2 - 3.0f * y2)), sY);
        const float w = bm * c[14];
        gx += w * (3.0f * (x2 - y2));
        gy -= w * (6.0f * xy);
    }
    {  // m = 15
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][15], g[n], bm);
            bpm = fmaf(B[n][15], gp[n], bpm);
        }
        sY = fmaf(bpm, c[15] * (x * y * (x2 - y2)), sY);
        const float w = bm * c[15];
        gx += w * ((3.0f * x2 * y - y2 * y));
        gy += w * ((x2 * x - 3.0f * x * y2));
    }
    {  // m = 16
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][16], g[n], bm);
            bpm = fmaf(B[n][16], gp[n], bpm);
        }
        sY = fmaf(bpm, c[16] * (y * z * (3.0f * x2 - y2)), sY);
        const float w = bm * c[16];
        gx += w * (6.0f * xy * z);
        gy += w * (3.0f * z * (x2 - y2));
        gz += w * ((3.0f * x2 * y - y2 * y));
    }
    {  // m = 17
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][17], g[n], bm);
            bpm = fmaf(B[n][17], gp[n], bpm);
        }
        sY = fmaf(bpm, c[17] * (x * y * (7.0f * z2 - 1.0f)), sY);
        const float w = bm * c[17];
        gx += w * (y * (7.0f * z2 - 1.0f));
        gy += w * (x * (7.0f * z2 - 1.0f));
        gz += w * (14.0f * xy * z);
    }
    {  // m = 18
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][18], g[n], bm);
            bpm = fmaf(B[n][18], gp[n], bpm);
        }
        sY = fmaf(bpm, c[18] * (y * z * (7.0f * z2 - 3.0f)), sY);
        const float w = bm * c[18];
        gy += w * (z * (7.0f * z2 - 3.0f));
        gz += w * (y * (21.0f * z2 - 3.0f));
    }
    {  // m = 19
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][19], g[n], bm);
            bpm = fmaf(B[n][19], gp[n], bpm);
        }
        sY = fmaf(bpm, c[19] * ((35.0f * z2 * z2 - 30.0f * z2 + 3.0f)), sY);
        const float w = bm * c[19];
        gz += w * (z * (140.0f * z2 - 60.0f));
    }
    {  // m = 20
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][20], g[n], bm);
            bpm = fmaf(B[n][20], gp[n], bpm);
        }
        sY = fmaf(bpm, c[20] * (x * z * (7.0f * z2 - 3.0f)), sY);
        const float w = bm * c[20];
        gx += w * (z * (7.0f * z2 - 3.0f));
        gz += w * (x * (21.0f * z2 - 3.0f));
    }
    {  // m = 21
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][21], g[n], bm);
            bpm = fmaf(B[n][21], gp[n], bpm);
        }
        sY = fmaf(bpm, c[21] * ((x2 - y2) * (7.0f * z2 - 1.0f)), sY);
        const float w = bm * c[21];
        gx += w * (2.0f * x * (7.0f * z2 - 1.0f));
        gy -= w * (2.0f * y * (7.0f * z2 - 1.0f));
        gz += w * (14.0f * z * (x2 - y2));
    }
    {  // m = 22
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][22], g[n], bm);
            bpm = fmaf(B[n][22], gp[n], bpm);
        }
        sY = fmaf(bpm, c[22] * (x * z * (x2 - 3.0f * y2)), sY);
        const float w = bm * c[22];
        gx += w * (3.0f * z * (x2 - y2));
        gy -= w * (6.0f * xy * z);
        gz += w * (x * (x2 - 3.0f * y2));
    }
    {  // m = 23
        float bm = 0.0f, bpm = 0.0f;
#pragma unroll
        for (int n = 0; n < NA1; ++n) {
            bm = fmaf(B[n][23], g[n], bm);
            bpm = fmaf(B[n][23], gp[n], bpm);
        }
        sY = fmaf(bpm, c[23] * ((x2 * (x2 - 3.0f * y2) - y2 * (3.0f * x2 - y2))), sY);
        const float w = bm * c[23];
        gx += w * ((4.0f * x2 * x - 12.0f * x * y2));
        gy += w * ((4.0f * y2 * y - 12.0f * x2 * y));
    }
}

// l of spherical-harmonic slot m (0..23).
__host__ __device__ constexpr int sh_l(int m) { return m < 3 ? 1 : (m < 8 ? 2 : (m < 15 ? 3 : 4)); }

template <int NR1, int NA1, bool FOUR>
struct Dims {
    static constexpr int D = NR1 + kLmax * NA1 + (FOUR ? NA1 : 0);
};

// Four-body helper: M_n = sum_j g_n (u u^T - I/3) rebuilt from the l = 2 sums
// (slots 3..7 hold m = -2..2): returns mxy, myz, mzz, mxz, d = mxx - myy.
__device__ __forceinline__ void m_from_l2(const float *A2, const float *shc, float *M)
{
    M[0] = A2[0] / shc[3];
    M[1] = A2[1] / shc[4];
    M[2] = A2[2] / (3.0f * shc[5]);
    M[3] = A2[3] / shc[6];
    M[4] = A2[4] / shc[7];
}

// Adjoint of one radial function n's angular sums, stored as B_nlm c_m:
// B_nlm = dU/dA_nlm = 2 (dU/dq_nl) A_nlm, plus for the four-body invariant
// q4_n = kappa tr(M_n^3) the derivative through M_n's l = 2 entries,
// 3 kappa (dU/dq4_n) d tr(M^3)/dM = 3 g4 M^2 mapped back onto m = -2..2.
// Gl[l - 1] = dU/dq_nl, g4 = kappa dU/dq4_n.  An and Bn may be the same
// array (M is formed before any entry is written).
template <bool FOUR>
__device__ __forceinline__ void form_adjoint(const float *An, const float (&Gl)[kLmax], float g4,
                                             const float *__restrict__ shc, float *Bn)
{
    float M[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (FOUR) m_from_l2(&An[3], shc, M);
#pragma unroll
    for (int m = 0; m < kNumSH; ++m) Bn[m] = 2.0f * Gl[sh_l(m) - 1] * An[m];
    if (FOUR) {
        const float mxy = M[0], myz = M[1], mzz = M[2], mxz = M[3], dd = M[4];
        const float mxx = 0.5f * (dd - mzz), myy = 0.5f * (-dd - mzz);
        // entries of M^2
        const float sxx = mxx * mxx + mxy * mxy + mxz * mxz;
        const float syy = mxy * mxy + myy * myy + myz * myz;
        const float szz = mxz * mxz + myz * myz + mzz * mzz;
        const float sxy = mxx * mxy + mxy * myy + mxz * myz;
        const float syz = mxy * mxz + myy * myz + myz * mzz;
        const float sxz = mxx * mxz + mxy * myz + mxz * mzz;
        Bn[3] += g4 * 6.0f * sxy / shc[3];
        Bn[4] += g4 * 6.0f * syz / shc[4];
        Bn[5] += g4 * 3.0f * (szz - 0.5f * sxx - 0.5f * syy) / (3.0f * shc[5]);
        Bn[6] += g4 * 6.0f * sxz / shc[6];
        Bn[7] += g4 * 1.5f * (sxx - syy) / shc[7];
    }
    // stored as B_nlm c_m, the factor the pair terms need with the bare polynomials
#pragma unroll
    for (int m = 0; m < kNumSH; ++m) Bn[m] *= shc[m];
}

// Directional derivatives D_m = c_m grad p_m(u) . v of the 24 harmonics
// (Y_m = c_m p_m) along v, p_m differentiated on R^3.
__device__ __forceinline__ void sh_dir(float x, float y, float z, float vx, float vy, float vz,
                                       const float *__restrict__ c, float *D)
{
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    const float xy = x * y, yz = y * z, xz = x * z;
    D[0] = c[0] * (vy);
    D[1] = c[1] * (vz);
    D[2] = c[2] * (vx);
    D[3] = c[3] * (vx * (y) + vy * (x));
    D[4] = c[4] * (vy * (z) + vz * (y));
    D[5] = c[5] * (vz * (6.0f * z));
    D[6] = c[6] * (vx * (z) + vz * (x));
    D[7] = c[7] * (vx * (2.0f * x) - vy * (2.0f * y));
    D[8] = c[8] * (vx * (6.0f * xy) + vy * (3.0f * (x2 - y2)));
    D[9] = c[9] * (vx * (yz) + vy * (xz) + vz * (xy));
    D[10] = c[10] * (vy * ((5.0f * z2 - 1.0f)) + vz * (10.0f * yz));
    D[11] = c[11] * (vz * ((15.0f * z2 - 3.0f)));
    D[12] = c[12] * (vx * ((5.0f * z2 - 1.0f)) + vz * (10.0f * xz));
    D[13] = c[13] * (vx * (2.0f * xz) - vy * (2.0f * yz) + vz * ((x2 - y2)));
    D[14] = c[14] * (vx * (3.0f * (x2 - y2)) - vy * (6.0f * xy));
    D[15] = c[15] * (vx * ((3.0f * x2 * y - y2 * y)) + vy * ((x2 * x - 3.0f * x * y2)));
    D[16] = c[16] * (vx * (6.0f * xy * z) + vy * (3.0f * z * (x2 - y2)) + vz * ((3.0f * x2 * y - y2 * y)));
    D[17] = c[17] * (vx * (y * (7.0f * z2 - 1.0f)) + vy * (x * (7.0f * z2 - 1.0f)) + vz * (14.0f * xy * z));
    D[18] = c[18] * (vy * (z * (7.0f * z2 - 3.0f)) + vz * (y * (21.0f * z2 - 3.0f)));
    D[19] = c[19] * (vz * (z * (140.0f * z2 - 60.0f)));
    D[20] = c[20] * (vx * (z * (7.0f * z2 - 3.0f)) + vz * (x * (21.0f * z2 - 3.0f)));
    D[21] = c[21] * (vx * (2.0f * x * (7.0f * z2 - 1.0f)) - vy * (2.0f * y * (7.0f * z2 - 1.0f)) + vz * (14.0f * z * (x2 - y2)));
    D[22] = c[22] * (vx * (3.0f * z * (x2 - y2)) - vy * (6.0f * xy * z) + vz * (x * (x2 - 3.0f * y2)));
    D[23] = c[23] * (vx * ((4.0f * x2 * x - 12.0f * x * y2)) + vy * ((4.0f * y2 * y - 12.0f * x2 * y)));
}

}  // namespace nep
