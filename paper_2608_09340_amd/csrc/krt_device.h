// krt_device.h -- device helpers shared by the transport and escape kernels:
// Philox4x32-10, the uniform map, hardware transcendental wrappers, the tally
// bin rule and the LDS table lookups (Voigt profile, atom-velocity sampler).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "krt_internal.h"
#include "krt_kernels.h"

namespace krt {

// ------------------------------------------------------------------ Philox ---
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two 32x32
// multiplies with key schedule increments (W0, W1) between rounds.
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// uniform on (0,1): an odd multiple of 2^-24, exact in binary32
__device__ __forceinline__ float u01(uint32_t w) {
    return (float)(w >> 9) * 0x1p-23f + 0x1p-24f;
}

// ------------------------------------------------------------- fast math ---
constexpr float kPiF = 3.14159265358979f;
constexpr uint32_t kMaxCrossings = 1u << 30;  // per packet: a packet that never interacts is retired as stuck
constexpr float kInvSqrtPiF = 0.564189583547756f;
constexpr float kInvSqrt2F = 0.707106781186547524f;
constexpr float kLn2F = 0.693147180559945f;
__device__ __forceinline__ float f_log(float x) { return __builtin_amdgcn_logf(x) * kLn2F; }
__device__ __forceinline__ float f_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896f); }
__device__ __forceinline__ float f_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float f_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float f_rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// sin / cos of 2 pi r (the hardware takes revolutions)
__device__ __forceinline__ float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }
__device__ __forceinline__ float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }

// ------------------------------------------------------------------- bins ---
// Index rule shared by every tally: edges[k] (k = 0..nb) are the binary32 values
// of lo + (hi - lo) * k / nb computed in FP64 on the host; the bin is 1 + the
// largest k with edges[k] <= x, 0 below edges[0], nb + 1 at or above edges[nb],
// -1 for NaN.  The first guess from (x - lo) / width is corrected against the
// edges themselves, so the result is exact whatever the rounding of the guess.
__device__ __forceinline__ int bin_index(float x, const float *edges, int nb, float inv_w) {
    if (!(x == x)) return -1;
    const float e0 = edges[0];
    if (x < e0) return 0;
    if (x >= edges[nb]) return nb + 1;
    int k = (int)((x - e0) * inv_w);
    k = max(0, min(nb - 1, k));
    while (k > 0 && edges[k] > x) --k;
    while (k < nb - 1 && edges[k + 1] <= x) ++k;
    return k + 1;
}

// ----------------------------------------------------------- LDS lookups ---
__device__ __forceinline__ float voigt_lds(const float *T, float xa) {
    if (xa < 8.0f) {
        float t = xa * 64.0f;
        int i = max(0, min((int)t, kVoigtCoreN - 1));
        float f = t - (float)i;
        float4 c = *reinterpret_cast<const float4 *>(T + kOffVoigtCore + 4 * i);
        return fmaf(f, fmaf(f, fmaf(f, c.w, c.z), c.y), c.x);
    }
    float w = 8.0f * f_rcp(xa);
    float t = w * (float)kVoigtWingN;
    int j = max(0, min((int)t, kVoigtWingN - 1));
    float f = t - (float)j;
    float4 c = *reinterpret_cast<const float4 *>(T + kOffVoigtWing + 4 * j);
    float G = fmaf(f, fmaf(f, fmaf(f, c.w, c.z), c.y), c.x);
    return G * w * w * (1.0f / 64.0f);
}

// Analytic approximation of H(a, u) that blends the Doppler core exp(-u^2) and
// the damping wing a / (sqrt(pi) (u^2 + a^2)) with the switch
// w = (1 + tanh(2|u| - 2 u0)) / 2 centred at the crossing point u0 of the two
// asymptotes (Sec. 2.2.1, the third profile mode).  Accurate in the core and
// the wing, rough between them: offered to show why the opacity profile must
// be the one the redistribution sampler assumes, not for production runs.
__device__ __forceinline__ float voigt_analytic(float a, float u0, float ua) {
    const float core = f_exp(-ua * ua);
    const float wing = a * kInvSqrtPiF * f_rcp(fmaf(ua, ua, a * a));
    const float w = 0.5f * (1.0f + tanhf(2.0f * (ua - u0)));
    return fmaf(w, wing - core, core);
}

// Atom parallel velocity for gas-frame frequency x (Sec. 2.1.1): piece by r1
// against the cumulative piece probabilities, quantile by r2, bilinear in
// (row of |x|, quantile node).
__device__ __forceinline__ float upar_lds(const float *T, float x, float a, float thd,
                                          float r1, float r2) {
    float xa = fabsf(x);
    float c1 = 0.0f, c2 = 0.0f, c3 = 1.0f;
    if (xa < 8.0f) {
        float pm = xa * (float)(kMassN / 8);
        int im = max(0, min((int)pm, kMassN - 1));
        float fm = pm - (float)im;
        float4 m0 = *reinterpret_cast<const float4 *>(T + kOffMass + 4 * im);
        float4 m1 = *reinterpret_cast<const float4 *>(T + kOffMass + 4 * im + 4);
        c1 = fmaf(fm, m1.x - m0.x, m0.x);
        c2 = fmaf(fm, m1.y - m0.y, m0.y);
        c3 = fmaf(fm, m1.z - m0.z, m0.z);
    }
    float p;
    if (xa < 8.0f) p = xa * 6.0f;
    else p = fminf(48.0f + f_log(xa * 0.125f) * kRowInvLog, 63.0f);
    int j = max(0, min((int)p, kRows - 2));
    float fr = p - (float)j;
    int kind = (r1 < c1) ? 0 : ((r1 < c2) ? 1 : ((r1 < c3) ? 2 : 3));
    int nq = (kind == 0) ? kQS : kQL1;  // kQL1 == kQL2 == kQR
    int off = (kind == 0) ? kOffSpike : ((kind == 1) ? kOffL1 : ((kind == 2) ? kOffL2 : kOffRight));
    // wing pieces: nodes at q = 4 xi^3 (xi < 1/2), 1 - 4 (1 - xi)^3 (xi >= 1/2)
    float xi = r2;
    if (kind != 0) {
        float t = (r2 < 0.5f) ? r2 : 1.0f - r2;
        float cb = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(0.25f * t) * (1.0f / 3.0f));
        xi = (r2 < 0.5f) ? cb : 1.0f - cb;
    }
    float qp = xi * (float)(nq - 1);
    int k = max(0, min((int)qp, nq - 2));
    float fq = qp - (float)k;
    const float *r0 = T + off + j * nq + k;
    float v0 = fmaf(fq, r0[1] - r0[0], r0[0]);
    float v1 = fmaf(fq, r0[nq + 1] - r0[nq], r0[nq]);
    float v = fmaf(fr, v1 - v0, v0);
    float u;
    if (kind == 0) {
        float th = v * thd * (1.0f / (2.0f * kPiF));
        u = xa + a * sin_rev(th) * f_rcp(cos_rev(th));
    } else if (kind == 2) {
        u = v;
    } else {
        float s = (float)kDelta * f_exp(v);
        u = (kind == 1) ? xa - s : xa + s;
    }
    return (x < 0.0f) ? -u : u;  // p(u | -x) = p(-u | x)
}

// Dipole phase (3/8)(1 + g^2): g = 2 sinh(asinh(4u - 2)/3).
__device__ __forceinline__ float dipole_g(float u) {
    float q = 4.0f * u - 2.0f;
    float aq = fabsf(q);
    float t = f_log(aq + f_sqrt(fmaf(aq, aq, 1.0f))) * (1.0f / 3.0f);
    float e = f_exp(t);
    float g = e - f_rcp(e);
    return copysignf(g, q);
}

}  // namespace krt
