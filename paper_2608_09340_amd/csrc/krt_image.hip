// krt_image.hip -- deterministic ray-tracing imaging pass (Sec. 2.2.2): the
// formal solution of eq. imaging-formal along lines of sight toward a camera
// on a grid axis, in every Doppler channel, over the scattering emissivity
// that the Monte Carlo pass tallied toward that camera.
//
// Per cell and channel k, from the far side of the grid to the camera:
//   I <- I exp(-dtau_k) + j_k dl (1 - exp(-dtau_k)) / dtau_k + S_emis,k (1 - exp(-dtau_k)),
//   dtau_k = (k0 H(a, x_k - n_cam.v) + kappa_abs) dl   (eq. imaging-alphas; kappa_abs
//   an optional grey absorption, zero when absent),
// with x_k the lab-frame centre of channel k.  One lane per (pixel, channel):
// the lanes of a pixel read its cells' fields at one address (broadcast) and
// the emissivity of consecutive channels from consecutive addresses, so the
// pass streams the emissivity array once; the Voigt table sits in LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "krt_internal.h"
#include "krt_kernels.h"
#include "krt_device.h"

namespace krt {

constexpr int kImgVoigtFloats = kOffVoigtWing + 4 * kVoigtWingN;  // core and wing of H(a, x)
constexpr int kImgChunk = 8;                                        // cells loaded ahead

__global__ void __launch_bounds__(256) image_kernel(ImageParams Q) {
    __shared__ float4 tv4[kImgVoigtFloats / 4];
    float *TV = reinterpret_cast<float *>(tv4);
    const float4 *src = reinterpret_cast<const float4 *>(Q.tab);
    for (int i = threadIdx.x; i < kImgVoigtFloats / 4; i += blockDim.x) tv4[i] = src[i];
    __syncthreads();
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= Q.npix * (int64_t)Q.nch) return;
    const int64_t pix = tid / Q.nch;
    const int c = (int)(tid - pix * Q.nch);
    // pixel -> first cell of its column and the stride along the ray
    const int p0 = (int)(pix % Q.n0), p1 = (int)(pix / Q.n0);
    int64_t cell0;
    if (Q.d == 0) cell0 = ((int64_t)p1 * Q.n[1] + p0) * Q.n[0];           // (k, j)
    else if (Q.d == 1) cell0 = (int64_t)p1 * Q.n[1] * Q.n[0] + p0;         // (k, i)
    else cell0 = (int64_t)p1 * Q.n[0] + p0;                                // (j, i)
    const int nl = Q.n[Q.d];
    const float xk = Q.ch_lo + ((float)c + 0.5f) * Q.ch_w;
    const float *vd = Q.vel_axis;  // velocity component along the camera axis, or null
    float I = 0.0f;
    // the loads of kImgChunk cells are issued together, then the cells are
    // folded in order: the march is a dependent chain, its memory is not
    for (int t0 = 0; t0 < nl; t0 += kImgChunk) {
        float k0v[kImgChunk], vv[kImgChunk], jv[kImgChunk], sv[kImgChunk], av[kImgChunk];
#pragma unroll
        for (int u = 0; u < kImgChunk; ++u) {
            const int t = t0 + u;
            k0v[u] = 0.0f; vv[u] = 0.0f; jv[u] = 0.0f; sv[u] = 0.0f; av[u] = 0.0f;
            if (t < nl) {
                const int s = (Q.sgn > 0) ? t : nl - 1 - t;  // far side first
                const int64_t cell = cell0 + (int64_t)s * Q.stride;
                k0v[u] = Q.k0[cell];
                if (vd) vv[u] = vd[cell];
                if (Q.kabs) av[u] = Q.kabs[cell];
                jv[u] = Q.emis[cell * Q.nch + c];
                if (Q.srcf) sv[u] = Q.srcf[cell * Q.nch + c];
            }
        }
#pragma unroll
        for (int u = 0; u < kImgChunk; ++u) {
            if (t0 + u >= nl) break;
            const float xg = xk - Q.sgnf * vv[u];
            const float H = (k0v[u] > 0.0f) ? voigt_lds(TV, fabsf(xg)) : 0.0f;
            const float dtau = fmaf(k0v[u], H, av[u]) * Q.dl;
            const float att = f_exp(-dtau);
            // (1 - e^{-dtau}) / dtau, with its series below 1e-3
            const float frac = (dtau < 1e-3f) ? 1.0f - dtau * (0.5f - dtau * (1.0f / 6.0f)) : (1.0f - att) * f_rcp(dtau);
            I = fmaf(I, att, jv[u] * Q.dl * frac);
            I = fmaf(sv[u], dtau * frac, I);
        }
    }
    Q.out[tid] = I;
}

hipError_t launch_image(const ImageParams &Q, hipStream_t s) {
    const int64_t n = Q.npix * (int64_t)Q.nch;
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(image_kernel, dim3((unsigned)blocks), dim3(256), 0, s, Q);
    return hipGetLastError();
}

}  // namespace krt
