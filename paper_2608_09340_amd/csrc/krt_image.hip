// krt_image.hip -- deterministic ray-tracing imaging pass (Sec. 2.2.2): the
// formal solution of eq. imaging-formal along lines of sight toward a camera
// on a grid axis, in every Doppler channel, over the scattering emissivity
// that the Monte Carlo pass tallied toward that camera.
//
// Per cell and channel k, from the far side of the grid to the camera:
//   I <- I exp(-dtau_k) + j_k dl (1 - exp(-dtau_k)) / dtau_k + S_emis,k (1 - exp(-dtau_k)),
//   dtau_k = (k0 H(a, x_k - n_cam.v) + kappa_abs) dl   (eq. imaging-alphas; kappa_abs
//   an optional grey absorption, zero when absent),
// with x_k the lab-frame centre of channel k.
//
// Layout.  One lane per (pixel, channel); a wave holds 64 consecutive
// (pixel, channel) pairs, so its lanes read a cell's fields at one address
// per pixel of the wave (one or two at 32 channels or more) and the emissivity of consecutive channels from
// consecutive addresses: the pass streams the emissivity array once.  The
// Voigt table sits in LDS.  The recurrence is affine in I, so a ray can be
// cut into segments: the wave of segment s folds its cells into a map
// I -> A_s I + B_s, and the maps are composed in order, far side first,
// through LDS.  Short rays on small grids take several segments so that the
// launch still fills the chip; long ones take one.  A wave issues the loads
// of a chunk of cells together and then folds them in order (the march is a
// dependent chain, its memory is not); memory latency is hidden by the other
// waves on the SIMD (eight without a source function), whose number a second
// register buffer for the next chunk would halve.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "krt_internal.h"
#include "krt_kernels.h"
#include "krt_device.h"
#include "krt_image.h"

namespace krt {

constexpr int kImgVoigtFloats = kOffVoigtWing + 4 * kVoigtWingN;  // core and wing of H(a, x)
constexpr int kImgChunk = 8;            // cells whose loads are in flight together
constexpr int kImgWaves = 8;            // waves per block
constexpr int kImgMaxSeg = kImgWaves;   // segments of one ray (waves of one block)
constexpr int kImgMinSegCells = 4;      // shortest segment worth a wave
constexpr int64_t kImgTargetWaves = 16384;  // twice the chip's resident waves at 8 per SIMD

// fields of a chunk of cells along the ray (the arrays a kernel instance does
// not read are never written and cost nothing)
struct ImgChunk {
    float k0[kImgChunk], v[kImgChunk], ab[kImgChunk], j[kImgChunk], s[kImgChunk];
};

// loads of cells t .. t + m - 1 of the segment (m <= kImgChunk, compile-time
// in the full-chunk path); cell t sits at offset o (fields) and o * nch (channels)
template <bool kVel, bool kAbs, bool kSrc, int M>
__device__ __forceinline__ void img_load(const ImageParams &Q, int64_t o, int64_t step, int64_t cstep,
                                         const float *pe, const float *ps, ImgChunk &b) {
#pragma unroll
    for (int u = 0; u < M; ++u) {
        const int64_t oc = o + u * step;
        b.k0[u] = Q.k0[oc];
        if constexpr (kVel) b.v[u] = Q.vel_axis[oc];
        if constexpr (kAbs) b.ab[u] = Q.kabs[oc];
        b.j[u] = pe[u * cstep];
        if constexpr (kSrc) b.s[u] = ps[u * cstep];
    }
}

// H(a, |x|) from the core / wing table in LDS, without a branch: the lanes
// of a wave span channels on both sides of |x| = 8, so the two pieces share
// one address computation and one LDS read
__device__ __forceinline__ float img_voigt(const float *T, float xa) {
    const bool core = xa < 8.0f;
    const float w = 8.0f * f_rcp(xa);
    const float t = core ? xa * 64.0f : w * (float)kVoigtWingN;
    const int i = max(0, min((int)t, core ? kVoigtCoreN - 1 : kVoigtWingN - 1));
    const float f = t - (float)i;
    const float4 c = *reinterpret_cast<const float4 *>(T + (core ? kOffVoigtCore : kOffVoigtWing) + 4 * i);
    const float G = fmaf(f, fmaf(f, fmaf(f, c.w, c.z), c.y), c.x);
    return core ? G : G * w * w * (1.0f / 64.0f);
}

template <bool kVel, bool kAbs, bool kSrc, int M>
__device__ __forceinline__ void img_fold(const ImageParams &Q, const float *TV, float xk,
                                         const ImgChunk &b, float &A, float &B) {
#pragma unroll
    for (int u = 0; u < M; ++u) {
        const float xg = kVel ? xk - Q.sgnf * b.v[u] : xk;
        const float H = (b.k0[u] > 0.0f) ? img_voigt(TV, fabsf(xg)) : 0.0f;
        const float dtau = (kAbs ? fmaf(b.k0[u], H, b.ab[u]) : b.k0[u] * H) * Q.dl;
        const float att = f_exp(-dtau);
        // (1 - e^{-dtau}) / dtau, with its series below 1e-3
        const float frac = (dtau < 1e-3f) ? 1.0f - dtau * (0.5f - dtau * (1.0f / 6.0f)) : (1.0f - att) * f_rcp(dtau);
        B = fmaf(B, att, b.j[u] * Q.dl * frac);
        if constexpr (kSrc) B = fmaf(b.s[u], dtau * frac, B);
        A *= att;
    }
}

template <bool kVel, bool kAbs, bool kSrc>
__device__ __forceinline__ void image_body(const ImageParams &Q, int nseg, int seglen) {
    __shared__ float4 tv4[kImgVoigtFloats / 4];
    __shared__ float2 part[kImgWaves][64];  // (A_s, B_s) of every wave's segment
    float *TV = reinterpret_cast<float *>(tv4);
    const float4 *src = reinterpret_cast<const float4 *>(Q.tab);
    for (int i = threadIdx.x; i < kImgVoigtFloats / 4; i += blockDim.x) tv4[i] = src[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int seg = wave % nseg;                // segment of the ray, far side = 0
    const int grp = wave / nseg;                // group of 64 (pixel, channel) pairs
    const int64_t tid = ((int64_t)blockIdx.x * (kImgWaves / nseg) + grp) * 64 + lane;
    const bool live = tid < Q.npix * (int64_t)Q.nch;
    float A = 1.0f, B = 0.0f;
    if (live) {
        const int64_t pix = tid / Q.nch;
        const int c = (int)(tid - pix * Q.nch);
        // pixel -> first cell of its column and the stride along the ray
        const int p0 = (int)(pix % Q.n0), p1 = (int)(pix / Q.n0);
        int64_t cell0;
        if (Q.d == 0) cell0 = ((int64_t)p1 * Q.n[1] + p0) * Q.n[0];           // (k, j)
        else if (Q.d == 1) cell0 = (int64_t)p1 * Q.n[1] * Q.n[0] + p0;         // (k, i)
        else cell0 = (int64_t)p1 * Q.n[0] + p0;                                // (j, i)
        const int nl = Q.n[Q.d];
        const int t0 = seg * seglen, t1 = min(nl, t0 + seglen);
        // step t (far side first) is cell s = t toward +axis cameras, nl - 1 - t otherwise
        const int64_t step = Q.sgn > 0 ? Q.stride : -Q.stride;
        const int64_t cstep = step * Q.nch;
        int64_t o = cell0 + (int64_t)(Q.sgn > 0 ? t0 : nl - 1 - t0) * Q.stride;
        const float *pe = Q.emis + o * Q.nch + c;
        const float *ps = kSrc ? Q.srcf + o * Q.nch + c : nullptr;
        const float xk = Q.ch_lo + ((float)c + 0.5f) * Q.ch_w;
        const int nfull = max(0, t1 - t0) / kImgChunk;
        ImgChunk cur{};
        for (int i = 0; i < nfull; ++i) {
            img_load<kVel, kAbs, kSrc, kImgChunk>(Q, o, step, cstep, pe, ps, cur);
            img_fold<kVel, kAbs, kSrc, kImgChunk>(Q, TV, xk, cur, A, B);
            o += kImgChunk * step;
            pe += kImgChunk * cstep;
            if constexpr (kSrc) ps += kImgChunk * cstep;
        }
        for (int t = t0 + nfull * kImgChunk; t < t1; ++t) {  // ragged end of the segment
            img_load<kVel, kAbs, kSrc, 1>(Q, o, step, cstep, pe, ps, cur);
            img_fold<kVel, kAbs, kSrc, 1>(Q, TV, xk, cur, A, B);
            o += step;
            pe += cstep;
            if constexpr (kSrc) ps += cstep;
        }
    }
    if (nseg == 1) {
        if (live) Q.out[tid] = B;
        return;
    }
    part[wave][lane] = make_float2(A, B);
    __syncthreads();
    if (seg == 0 && live) {
        float I = 0.0f;
        for (int s = 0; s < nseg; ++s) {
            const float2 p = part[wave + s][lane];
            I = fmaf(p.x, I, p.y);
        }
        Q.out[tid] = I;
    }
}

// Without a source function the fold fits the register budget of eight
// waves per SIMD (64 VGPRs), the occupancy that hides the memory latency;
// with one it would spill, so that kernel keeps the compiler's budget.
template <bool kVel, bool kAbs>
__global__ void __launch_bounds__(64 * kImgWaves) __attribute__((amdgpu_waves_per_eu(8, 8)))
image_kernel(ImageParams Q, int nseg, int seglen) {
    image_body<kVel, kAbs, false>(Q, nseg, seglen);
}

template <bool kVel, bool kAbs>
__global__ void __launch_bounds__(64 * kImgWaves) image_src_kernel(ImageParams Q, int nseg, int seglen) {
    image_body<kVel, kAbs, true>(Q, nseg, seglen);
}

template <bool kVel, bool kAbs, bool kSrc>
static void launch_image_t(const ImageParams &Q, int nseg, int seglen, int64_t blocks, hipStream_t s,
                           hipEvent_t start, hipEvent_t stop) {
    if constexpr (kSrc)
        hipExtLaunchKernelGGL((image_src_kernel<kVel, kAbs>), dim3((unsigned)blocks), dim3(64 * kImgWaves), 0, s,
                              start, stop, 0, Q, nseg, seglen);
    else
        hipExtLaunchKernelGGL((image_kernel<kVel, kAbs>), dim3((unsigned)blocks), dim3(64 * kImgWaves), 0, s,
                              start, stop, 0, Q, nseg, seglen);
}

// segments per ray: doubled while the launch has fewer waves than the chip
// keeps busy and the segments stay at least kImgMinSegCells cells long
static int image_segments(int64_t npix, int nch, int nl) {
    const int64_t groups = (npix * nch + 63) / 64;
    int nseg = 1;
    while (nseg < kImgMaxSeg && groups * nseg < kImgTargetWaves &&
           (nl + 2 * nseg - 1) / (2 * nseg) >= kImgMinSegCells)
        nseg *= 2;
    return nseg;
}

hipError_t launch_image_timed(const ImageParams &Q, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
    const int64_t n = Q.npix * (int64_t)Q.nch;
    if (n <= 0) {  // nothing to launch: an empty interval
        if (start) { hipError_t e = hipEventRecord(start, s); if (e != hipSuccess) return e; }
        if (stop) { hipError_t e = hipEventRecord(stop, s); if (e != hipSuccess) return e; }
        return hipSuccess;
    }
    const int nl = Q.n[Q.d];
    const int nseg = image_segments(Q.npix, Q.nch, nl);
    const int seglen = (nl + nseg - 1) / nseg;
    const int64_t groups = (n + 63) / 64;
    const int64_t per_block = kImgWaves / nseg;
    const int64_t blocks = (groups + per_block - 1) / per_block;
    const int key = (Q.vel_axis ? 4 : 0) | (Q.kabs ? 2 : 0) | (Q.srcf ? 1 : 0);
    switch (key) {
        case 0: launch_image_t<false, false, false>(Q, nseg, seglen, blocks, s, start, stop); break;
        case 1: launch_image_t<false, false, true>(Q, nseg, seglen, blocks, s, start, stop); break;
        case 2: launch_image_t<false, true, false>(Q, nseg, seglen, blocks, s, start, stop); break;
        case 3: launch_image_t<false, true, true>(Q, nseg, seglen, blocks, s, start, stop); break;
        case 4: launch_image_t<true, false, false>(Q, nseg, seglen, blocks, s, start, stop); break;
        case 5: launch_image_t<true, false, true>(Q, nseg, seglen, blocks, s, start, stop); break;
        case 6: launch_image_t<true, true, false>(Q, nseg, seglen, blocks, s, start, stop); break;
        default: launch_image_t<true, true, true>(Q, nseg, seglen, blocks, s, start, stop); break;
    }
    return hipGetLastError();
}

hipError_t launch_image(const ImageParams &Q, hipStream_t s) { return launch_image_timed(Q, s, nullptr, nullptr); }

}  // namespace krt
