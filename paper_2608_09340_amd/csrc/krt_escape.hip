// krt_escape.hip -- learned whole-cell escape: training data from single-cell
// walks run with the plain transport arithmetic, BF16-MFMA training (forward
// and backward per 16-sample block, weight gradients as a split-K product over
// the stored activations, Adam) and batched inference for tests.
//
// Whole-cell walk (training data): a homogeneous static cube [-1, 1]^3 (units
// of its half-width) of line-centre opacity tau_c per unit length; a photon of
// gas-frame frequency x_in >= 0 arriving along n_in scatters at a start point
// q in the reduced frame (0 <= q0 <= q1 <= q2 < 1), then takes the transport's
// flights and resonant scatterings (isotropic phase) until it leaves.  The
// record is the condition and the exit (face, offsets, cosine, alpha, x_out),
// the number of scatterings N_s and the mean x^2 over them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "krt_internal.h"
#include "krt_kernels.h"
#include "krt_mlp.h"
#include "krt_device.h"

namespace krt {

// ------------------------------------------------------------- recording ---
// Persistent pool: each lane takes record indices from one wave-aggregated
// atomic on `counter` (zeroed by the caller) and walks one event per loop
// iteration, so records of very different lengths share waves without idling.
__global__ void __launch_bounds__(256) cell_record_kernel(RecordParams R) {
    extern __shared__ float4 lds4[];
    float *T = reinterpret_cast<float *>(lds4);
    const float4 *src = reinterpret_cast<const float4 *>(R.tab);
    for (int i = threadIdx.x; i < kTabFloats / 4; i += blockDim.x) lds4[i] = src[i];
    __syncthreads();
    const int lane = __lane_id();
    const uint64_t lanemask_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const float la = __log10f(R.a);
    bool have = false, done = false;
    uint64_t idx = 0, pid = 0;
    float lt = 0.f, tauc = 0.f, xin = 0.f, q0 = 0.f, q1 = 0.f, q2 = 0.f;
    float m0 = 0.f, m1 = 0.f, m2 = 1.f;
    float px = 0.f, py = 0.f, pz = 0.f, nx = 0.f, ny = 0.f, nz = 1.f, x = 0.f, sx2 = 0.f;
    uint32_t ev = 0, ns = 0;
    for (;;) {
        const bool need = !have && !done;
        const uint64_t need_mask = __ballot(need);
        if (need_mask) {
            const int leader = __ffsll((long long)need_mask) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(R.counter, (unsigned long long)__popcll(need_mask));
            base = __shfl(base, leader, 64);
            if (need) {
                idx = base + (uint64_t)__popcll(need_mask & lanemask_lt);
                if (idx >= R.n) {
                    done = true;
                } else {
                    pid = R.offset + idx;
                    const uint32_t plo = (uint32_t)pid, phi = (uint32_t)(pid >> 32);
                    const uint4 c = philox(make_uint4(0u, plo, phi, 3u), R.k0, R.k1);
                    const uint4 d = philox(make_uint4(0u, plo, phi, 4u), R.k0, R.k1);
                    const uint4 e = philox(make_uint4(0u, plo, phi, 5u), R.k0, R.k1);
                    lt = R.lt_lo + (R.lt_hi - R.lt_lo) * u01(c.x);
                    tauc = f_exp(lt * 2.302585093f);
                    if (R.fixed) {
                        xin = R.x_in;
                        q0 = R.q[0]; q1 = R.q[1]; q2 = R.q[2];
                    } else {
                        // |x_in| from 1/2 N(0, 1/2) + 1/2 U[-3, 3]
                        if (u01(c.y) < 0.5f) xin = fabsf(f_sqrt(-f_log(u01(c.z))) * cos_rev(u01(c.w)));
                        else xin = kRecXMax * u01(c.z);
                        // depth to the nearest face log-uniform in [depth_lo, tau_c]
                        const float ld = fminf(R.ld_lo, lt) + (lt - fminf(R.ld_lo, lt)) * u01(e.x);
                        q2 = fminf(fmaxf(1.0f - f_exp((ld - lt) * 2.302585093f), 0.0f), 0.99999f);
                        float a0 = q2 * u01(e.y), a1 = q2 * u01(e.z);
                        q0 = fminf(a0, a1);
                        q1 = fmaxf(a0, a1);
                    }
                    if (R.fixed && !R.iso_dir) {
                        m0 = R.n_in[0]; m1 = R.n_in[1]; m2 = R.n_in[2];
                    } else {
                        const float mu0 = 2.0f * u01(d.x) - 1.0f, st0 = f_sqrt(fmaxf(0.0f, 1.0f - mu0 * mu0));
                        const float ph0 = u01(d.y);
                        m0 = st0 * cos_rev(ph0); m1 = st0 * sin_rev(ph0); m2 = mu0;
                    }
                    px = q0; py = q1; pz = q2;
                    nx = m0; ny = m1; nz = m2;
                    x = xin;
                    sx2 = 0.0f;
                    ns = 0;
                    ev = 1;
                    have = true;
                }
            }
        }
        if (__ballot(have) == 0ull) break;
        if (!have) continue;
        const uint32_t plo = (uint32_t)pid, phi = (uint32_t)(pid >> 32);
        const uint4 A = philox(make_uint4(ev, plo, phi, 0u), R.k0, R.k1);
        bool exited = false;
        int ax = 0;
        if (ev > 1) {
            // flight from the last interaction point
            const float tau = -f_log(u01(A.x));
            const float kap = tauc * voigt_lds(T, fabsf(x));
            const float tx = (nx > 0.f) ? (1.f - px) * f_rcp(nx) : ((nx < 0.f) ? (-1.f - px) * f_rcp(nx) : INFINITY);
            const float ty = (ny > 0.f) ? (1.f - py) * f_rcp(ny) : ((ny < 0.f) ? (-1.f - py) * f_rcp(ny) : INFINITY);
            const float tz = (nz > 0.f) ? (1.f - pz) * f_rcp(nz) : ((nz < 0.f) ? (-1.f - pz) * f_rcp(nz) : INFINITY);
            float dm = tx;
            if (ty < dm) { dm = ty; ax = 1; }
            if (tz < dm) { dm = tz; ax = 2; }
            dm = fmaxf(dm, 0.0f);
            if (kap * dm < tau) {
                px += dm * nx; py += dm * ny; pz += dm * nz;
                exited = true;
            } else {
                const float l = tau * f_rcp(kap);
                px = fminf(fmaxf(px + l * nx, -1.f), 1.f);
                py = fminf(fmaxf(py + l * ny, -1.f), 1.f);
                pz = fminf(fmaxf(pz + l * nz, -1.f), 1.f);
            }
        }
        if (!exited) {
            // resonant scattering (isotropic phase), event ev's words
            const uint4 B = philox(make_uint4(ev, plo, phi, 1u), R.k0, R.k1);
            const float upar = upar_lds(T, x, R.a, R.thd, u01(A.z), u01(A.w));
            const float rr = f_sqrt(-f_log(u01(B.x)));
            const float th = u01(B.y);
            const float up1 = rr * cos_rev(th), up2 = rr * sin_rev(th);
            const float g = 2.0f * u01(B.z) - 1.0f;
            const float psi = u01(B.w);
            const float sg = f_sqrt(fmaxf(0.0f, 1.0f - g * g));
            const float sgn = copysignf(1.0f, nz);
            const float A_ = -f_rcp(sgn + nz);
            const float B_ = nx * ny * A_;
            const float e1x = 1.0f + sgn * nx * nx * A_, e1y = sgn * B_, e1z = -sgn * nx;
            const float e2x = B_, e2y = sgn + ny * ny * A_, e2z = -ny;
            const float cp = cos_rev(psi), sp = sin_rev(psi);
            const float ox = g * nx + sg * (cp * e1x + sp * e2x);
            const float oy = g * ny + sg * (cp * e1y + sp * e2y);
            const float oz = g * nz + sg * (cp * e1z + sp * e2z);
            const float rn = f_rsq(ox * ox + oy * oy + oz * oz);
            sx2 += x * x;
            x = x + upar * (g - 1.0f) + sg * (up1 * cp + up2 * sp);
            nx = ox * rn; ny = oy * rn; nz = oz * rn;
            ns += 1;
            ev += 1;
        }
        const bool capped = !exited && ns > R.max_scat;
        if (exited || capped) {
            float *o = R.out + (int64_t)kRec * idx;
            o[kRecLT] = lt;
            o[kRecLA] = la;
            o[kRecX] = xin;
            o[kRecQ0] = q0; o[kRecQ0 + 1] = q1; o[kRecQ0 + 2] = q2;
            o[kRecLD] = lt + __log10f(fmaxf(1.0f - q2, 1e-30f));
            o[kRecN0] = m0; o[kRecN0 + 1] = m1; o[kRecN0 + 2] = m2;
            if (exited) {
                const float qq[3] = {q0, q1, q2}, P[3] = {px, py, pz}, N[3] = {nx, ny, nz};
                float side = 0.f, dpl = 1.f, ds = 0.f, dt = 0.f, n1 = 0.f, n2 = 0.f, nn = 0.f;
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    if (k == ax) {
                        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
                        side = N[k] > 0.f ? 1.f : -1.f;
                        dpl = 1.f - side * qq[k];
                        ds = fminf(fmaxf(P[k1], -1.f), 1.f) - qq[k1];
                        dt = fminf(fmaxf(P[k2], -1.f), 1.f) - qq[k2];
                        n1 = N[k1]; n2 = N[k2]; nn = N[k];
                    }
                o[kRecFace] = (float)(2 * ax + (side > 0.f ? 1 : 0));
                o[kRecYS] = ds / dpl;
                o[kRecYT] = dt / dpl;
                o[kRecMu] = fabsf(nn);
                o[kRecAlpha] = atan2f(fabsf(ds * n2 - dt * n1), ds * n1 + dt * n2);
                o[kRecXOut] = x;
                o[kRecLogN] = logf((float)ns);
                o[kRecLogX2] = logf(fmaxf(sx2 / (float)ns, 1e-6f));
                o[kRecValid] = 1.0f;
            } else {
                for (int k = kRecFace; k <= kRecValid; ++k) o[k] = 0.0f;
            }
            o[kRec - 1] = 0.0f;
            have = false;
        }
    }
}

// ---------------------------------------------------------- parameters ---
// He-uniform initialisation from Philox (counter = (param index, 0, 0, 7))
__global__ void mlp_init_kernel(float *p, uint32_t k0, uint32_t k1) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParams) return;
    uint4 r = philox(make_uint4((uint32_t)i, 0u, 0u, 7u), k0, k1);
    float u = 2.0f * u01(r.x) - 1.0f;
    float fan_in = 0.0f;
    bool bias = false;
    if (i < kPB1) fan_in = kMlpIn;
    else if (i < kPW2) bias = true;
    else if (i < kPB2) fan_in = kMlpHid;
    else if (i < kPW3) bias = true;
    else if (i < kPB3) fan_in = kMlpHid;
    else if (i < kPW4) bias = true;
    else if (i < kPB4) fan_in = kMlpHid;
    else bias = true;
    p[i] = bias ? 0.0f : u * sqrtf(6.0f / fan_in);
}

// Pack the FP32 master parameters into BF16 A-operand tiles (with the chunk
// permutation kperm of the reduction index) + FP32 biases + normalisation.
// One thread per (tile, lane).
__global__ void mlp_pack_kernel(const float *p, const float *norm, unsigned char *blob) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid < kTilesAll * 64) {
        const int t = gid / 64, lane = gid % 64;
        const int i = lane % 16, g = lane / 16;
        uint16_t *dst = reinterpret_cast<uint16_t *>(blob + t * kTileBytes + lane * 16);
        for (int j = 0; j < 8; ++j) {
            const int kp = 8 * g + j;  // reduction slot
            float w = 0.0f;
            if (t < kTileFwdL2) {  // L1 fwd: W1^T, inputs in natural order, level residual slots tied
                const int mo = t - kTileFwdL1;
                if (kp < kMlpIn) w = p[kPW1 + kp * kMlpHid + 16 * mo + i];
                else if (kp < kMlpOperandIn) w = p[kPW1 + (kMlpLevelIn + kp - kMlpResIn) * kMlpHid + 16 * mo + i];
            } else if (t < kTileFwdL4) {  // L2/L3 fwd: tile mo*4+c, A[i][k'] = W[kperm(c,k')][16mo+i]
                const int base = (t < kTileFwdL3) ? kPW2 : kPW3;
                const int tt = t - ((t < kTileFwdL3) ? kTileFwdL2 : kTileFwdL3);
                const int mo = tt / 4, c = tt % 4;
                w = p[base + kperm(c, kp) * kMlpHid + 16 * mo + i];
            } else if (t < kTilesFwd) {  // L4 fwd: tile 4 ot + c, A[i][k'] = W4[kperm(c,k')][16 ot + i]
                const int ot = (t - kTileFwdL4) / 4, c = (t - kTileFwdL4) % 4;
                w = p[kPW4 + kperm(c, kp) * kMlpOut + 16 * ot + i];
            } else if (t < kTileBwdL3) {  // L4 bwd: tile mi, A[i][k'] = W4[16mi+i][kperm(0,k')]
                const int mi = t - kTileBwdL4;
                w = p[kPW4 + (16 * mi + i) * kMlpOut + kperm(0, kp)];
            } else {  // L3/L2 bwd: tile mi*4+c, A[i][k'] = W[16mi+i][kperm(c,k')]
                const int base = (t < kTileBwdL2) ? kPW3 : kPW2;
                const int tt = t - ((t < kTileBwdL2) ? kTileBwdL3 : kTileBwdL2);
                const int mi = tt / 4, c = tt % 4;
                w = p[base + (16 * mi + i) * kMlpHid + kperm(c, kp)];
            }
            dst[j] = f2bf(w);
        }
    }
    // biases and normalisation (b1 b2 b3 b4 norm)
    float *fb = reinterpret_cast<float *>(blob + kTilesAll * kTileBytes);
    if (gid < kBiasFloats) {
        float b;
        if (gid < kMlpHid) b = p[kPB1 + gid];
        else if (gid < 2 * kMlpHid) b = p[kPB2 + gid - kMlpHid];
        else if (gid < 3 * kMlpHid) b = p[kPB3 + gid - 2 * kMlpHid];
        else b = p[kPB4 + gid - 3 * kMlpHid];
        fb[gid] = b;
    }
    if (gid < kNNorm) fb[kBiasFloats + gid] = norm[gid];
}

// Copy of the forward part (tiles + biases + norm) into one contiguous image,
// the layout staged into LDS by the transport kernel.
__global__ void mlp_fwd_image_kernel(const unsigned char *blob, unsigned char *img) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int tiles_b = kTilesFwd * kTileBytes;
    const int tail_b = (kBiasFloats + kNNorm) * 4;
    if (i < tiles_b) img[i] = blob[i];
    else if (i < tiles_b + tail_b) img[i] = blob[kTilesAll * kTileBytes + (i - tiles_b)];
}

// Regression target of output k on record r, in the output's own variable
// (|x_out| only for the record's exit face, asinh of the offsets, the cosine
// squared); false where the output has none (faces, side, unused outputs,
// another face's |x_out|).
__device__ __forceinline__ bool target_value(const float *r, int k, float &y) {
    if (k >= kOutXAbs && k < kOutXAbs + 6) {
        if ((int)r[kRecFace] != k - kOutXAbs) return false;
        y = fabsf(r[kRecXOut]);
        return true;
    }
    switch (k) {
        case kOutLogN: y = r[kRecLogN]; return true;
        case kOutLogX2: y = r[kRecLogX2]; return true;
        case kOutYS: y = asinhf(r[kRecYS]); return true;
        case kOutYT: y = asinhf(r[kRecYT]); return true;
        case kOutMu2: y = r[kRecMu] * r[kRecMu]; return true;
        case kOutAlpha: y = r[kRecAlpha]; return true;
        default: return false;
    }
}

__device__ __forceinline__ bool conditional_output(int k) { return k >= kOutYS && k <= kOutAlpha; }
__device__ __forceinline__ bool used_output(int k) { return k <= kOutAlpha || (k >= kOutXAbs && k < kOutXAbs + 6); }

// ----------------------------------------------------- forward + backward ---
// Activation store of a training step, bf16 [row][cap] (samples contiguous):
// H0 32 rows (inputs, row 24 = 1 for the bias), H1..H3 144 rows (leaky ReLU
// activations, row 128 = 1), dZ1..dZ3 128 rows, dZ4 32 rows.  The constant
// rows are written once when the store is allocated.
constexpr int kActRowsH0 = 32, kActRowsH = 144;
constexpr int kActH0 = 0, kActH1 = kActH0 + kActRowsH0, kActH2 = kActH1 + kActRowsH, kActH3 = kActH2 + kActRowsH,
              kActZ1 = kActH3 + kActRowsH, kActZ2 = kActZ1 + kMlpHid, kActZ3 = kActZ2 + kMlpHid,
              kActZ4 = kActZ3 + kMlpHid, kActRows = kActZ4 + kMlpOut;   // 880
static_assert(kActRows == kActRowsAll, "activation store layout");

// One wave per 16-sample block.  Row si uses record idx[si] and uq[5 si ..] =
// (u_a, u_b, u_c, u_d, 1 for a conditional row); a conditional row takes the
// record's exit face and exit frequency as inputs.  Losses (each averaged over
// the batch): softmax cross-entropy for the exit face, logistic for the side
// of x_out, pinball for the quantiles at their own levels (|x_out| of face F
// only on records leaving through F), log-deviance for ln N_s.  Marginal rows
// train outputs 0-8 and 16-21, conditional rows 9-12.  Samples past the batch
// (up to the next multiple of 32) get zero gradients.
__global__ void __launch_bounds__(256) mlp_fwdbwd_kernel(const unsigned char *blob, const float *rec,
                                                         const int32_t *idx, const float *uq, int batch,
                                                         uint16_t *act, int64_t cap, float *loss) {
    const int lane = __lane_id(), w = threadIdx.x / 64;
    const int block = blockIdx.x * (blockDim.x / 64) + w;
    const int nblocks = 2 * ((batch + 31) / 32);
    if (block >= nblocks) return;  // wave-uniform
    const int s = lane % 16, g = lane / 16;
    const int si = block * 16 + s;
    const int ri = (si < batch) ? idx[si] : idx[0];
    const float *r = rec + (int64_t)kRec * ri;
    const bool live = si < batch && r[kRecValid] > 0.5f;
    const float *bias = reinterpret_cast<const float *>(blob + kTilesAll * kTileBytes);
    const float *norm = bias + kBiasFloats;
    const float *ul = uq + 5 * (int64_t)(si < batch ? si : 0);
    const float ua = ul[0], ub = ul[1], uc = ul[2], ud = ul[3];
    const bool cond = ul[4] > 0.5f;
    float in[kMlpIn];
    mlp_inputs(r, ua, ub, uc, ud, cond, r[kRecXOut], (int)r[kRecFace], in);
    if (!live)
        for (int k = 0; k < kMlpIn; ++k) in[k] = 0.0f;
    // the hidden activations go to the activation store as the forward pass
    // makes them; the backward pass keeps only the sign of each
    // pre-activation (bit 4 tile + component of zpos[layer]), all that the
    // derivative of the leaky ReLU needs
    const int64_t col = (int64_t)block * 16 + s;
    auto store4 = [&](int row0, float a0, float a1, float a2, float a3) {  // rows row0 + 4g + j
        uint16_t *p = act + (int64_t)(row0 + 4 * g) * cap + col;
        p[0] = f2bf(a0); p[cap] = f2bf(a1); p[2 * cap] = f2bf(a2); p[3 * cap] = f2bf(a3);
    };
    uint32_t zpos[3] = {0u, 0u, 0u};
    auto epi = [&](int layer, int mo, const v4f32 &z) __attribute__((always_inline)) {
        store4((layer == 0 ? kActH1 : (layer == 1 ? kActH2 : kActH3)) + 16 * mo, leaky(z.x), leaky(z.y), leaky(z.z),
               leaky(z.w));
        const uint32_t b = (z.x > 0.0f ? 1u : 0u) | (z.y > 0.0f ? 2u : 0u) | (z.z > 0.0f ? 4u : 0u) |
                           (z.w > 0.0f ? 8u : 0u);
        zpos[layer] |= b << (4 * mo);
    };
    v4f32 o, ob;
    mlp_forward_block(blob, bias, xin_operand(in, lane), lane, epi, o, ob);
    const float ov[8] = {o.x, o.y, o.z, o.w, ob.x, ob.y, ob.z, ob.w};
    // the six face logits of this lane's sample (lanes s and s + 16)
    float fl[6];
    fl[0] = __shfl(o.x, s, 64); fl[1] = __shfl(o.y, s, 64); fl[2] = __shfl(o.z, s, 64); fl[3] = __shfl(o.w, s, 64);
    fl[4] = __shfl(o.x, s + 16, 64); fl[5] = __shfl(o.y, s + 16, 64);
    float mx = fl[0];
#pragma unroll
    for (int f = 1; f < 6; ++f) mx = fmaxf(mx, fl[f]);
    float se = 0.0f, sm[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) { sm[f] = __expf(fl[f] - mx); se += sm[f]; }
    const float ise = 1.0f / se;
    const int face = (int)r[kRecFace];
    float flf = 0.0f;
#pragma unroll
    for (int f = 0; f < 6; ++f) if (f == face) flf = fl[f];
    const float invB = 1.0f / (float)batch;
    const float xo = r[kRecXOut];
    float dO[8], lsum = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = (j < 4) ? 4 * g + j : 16 + 4 * g + (j - 4);
        const float oj = ov[j];
        dO[j] = 0.0f;
        if (!live || !used_output(k) || conditional_output(k) != cond) continue;
        if (k < 6) {
            float smk = 0.0f;
#pragma unroll
            for (int f = 0; f < 6; ++f) if (f == k) smk = sm[f];
            dO[j] = (smk * ise - (k == face ? 1.0f : 0.0f)) * invB;
            if (k == 0) lsum += mx + __logf(se) - flf;
            continue;
        }
        if (k == kOutSide) {
            const float b = (xo >= 0.0f) ? 1.0f : 0.0f;
            dO[j] = (sigmoid_f(oj) - b) * invB;
            lsum += fmaxf(oj, 0.0f) + __logf(1.0f + __expf(-fabsf(oj))) - b * oj;
            continue;
        }
        float raw;
        if (!target_value(r, k, raw)) continue;
        const float y = (raw - norm[k]) / norm[kMlpOut + k];
        if (k == kOutLogN) {
            // weighted, scaled log-deviance w f(d) / s, d = s (y - o), f(d) = e^d - 1 - d,
            // continued linearly beyond d = kDevClamp
            const float sc = norm[kMlpOut + k];
            const float d = sc * (y - oj);
            const float dc = fminf(d, kDevClamp);
            const float ed = __expf(dc);
            dO[j] = kDevWeight * (1.0f - ed) * invB;
            lsum += kDevWeight * (ed - 1.0f - dc + (__expf(kDevClamp) - 1.0f) * fmaxf(d - kDevClamp, 0.0f)) / sc;
            continue;
        }
        // quantile level of this output on its kind of row
        float u;
        if (k >= kOutXAbs || k == kOutYS) u = ua;
        else if (k == kOutLogX2 || k == kOutYT) u = ub;
        else if (k == kOutMu2) u = uc;
        else u = ud;
        const float ind = (y < oj) ? 1.0f : 0.0f;
        dO[j] = (ind - u) * invB;
        lsum += (y - oj) * (u - ind);
    }
    for (int off = 32; off >= 1; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if (lane == 0 && loss) atomicAdd(loss, lsum * invB);

    // ---- backward through the layers (dZ4 = dO)
    // the leaky ReLU's derivative at pre-activation component j of tile mi
    auto dl = [&](int layer, int mi, int j) { return ((zpos[layer] >> (4 * mi + j)) & 1u) ? 1.0f : kLeak; };
    // inputs (rows 0..23; lane group g holds inputs 8g..8g+7)
    if (g < 3) {
        uint16_t *p = act + (int64_t)(kActH0 + 8 * g) * cap + col;
#pragma unroll
        for (int j = 0; j < 8; ++j) p[j * cap] = f2bf(g == 0 ? in[j] : (g == 1 ? in[8 + j] : in[16 + j]));
    }
    store4(kActZ4, dO[0], dO[1], dO[2], dO[3]);
    store4(kActZ4 + 16, dO[4], dO[5], dO[6], dO[7]);
    // B operand of the output layer's backward: slots 8g + j hold outputs
    // 4g + j and 16 + 4g + j, the permutation of the hidden layers' chunks
    const v8i16 dOb = cat8(pack4(dO[0], dO[1], dO[2], dO[3]), pack4(dO[4], dO[5], dO[6], dO[7]));
    v4f32 dz[8];
#pragma unroll
    for (int mi = 0; mi < 8; ++mi) {
        v4f32 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma32(tileA(blob, kTileBwdL4 + mi, lane), dOb, acc);
        dz[mi] = (v4f32){acc.x * dl(2, mi, 0), acc.y * dl(2, mi, 1), acc.z * dl(2, mi, 2), acc.w * dl(2, mi, 3)};
        store4(kActZ3 + 16 * mi, dz[mi].x, dz[mi].y, dz[mi].z, dz[mi].w);
    }
    // layer 3 -> dZ2, layer 2 -> dZ1 (unrolled so the activations stay in registers)
#pragma unroll
    for (int layer = 3; layer >= 2; --layer) {
        const int tb = (layer == 3) ? kTileBwdL3 : kTileBwdL2;
        v4i16 dzb[8];
#pragma unroll
        for (int mo = 0; mo < 8; ++mo) dzb[mo] = pack4(dz[mo].x, dz[mo].y, dz[mo].z, dz[mo].w);
#pragma unroll
        for (int mi = 0; mi < 8; ++mi) {
            v4f32 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < 4; ++c) acc = mfma32(tileA(blob, tb + mi * 4 + c, lane), cat8(dzb[2 * c], dzb[2 * c + 1]), acc);
            const int zl = (layer == 3) ? 1 : 0;
            dz[mi] = (v4f32){acc.x * dl(zl, mi, 0), acc.y * dl(zl, mi, 1), acc.z * dl(zl, mi, 2), acc.w * dl(zl, mi, 3)};
            store4((layer == 3 ? kActZ2 : kActZ1) + 16 * mi, dz[mi].x, dz[mi].y, dz[mi].z, dz[mi].w);
        }
    }
}

// Weight gradients as products over the stored activations: dW_l[in][out] =
// sum_s H_{l-1}[in][s] dZ_l[out][s], the bias from the constant row.  One wave
// per (layer, 16-row tile, pair of 16-column tiles, sample split): the H
// operand of a chunk feeds both tiles' products.  Results go to
// part[split][param] (every parameter is written by exactly one wave per
// split, so the sum over splits in fixed order is deterministic).
constexpr int kGradJobsL1 = 2 * 4, kGradJobsL2 = 9 * 4, kGradJobsL3 = 9 * 4, kGradJobsL4 = 9 * 1;
constexpr int kGradJobs = kGradJobsL1 + kGradJobsL2 + kGradJobsL3 + kGradJobsL4;   // 89

__global__ void __launch_bounds__(256) mlp_wgrad_kernel(const uint16_t *act, int64_t cap, int kcols, float *part) {
    const int lane = __lane_id(), w = threadIdx.x / 64;
    const int job = blockIdx.x * (blockDim.x / 64) + w;
    if (job >= kGradJobs * kGradSplits) return;
    const int split = job / kGradJobs;
    int jj = job % kGradJobs;
    int hrow, zrow, it, jp, nin, ldw, pw, pb;
    if (jj < kGradJobsL1) {
        it = jj / 4; jp = jj % 4; hrow = kActH0; zrow = kActZ1; nin = kMlpIn; ldw = kMlpHid; pw = kPW1; pb = kPB1;
    } else if ((jj -= kGradJobsL1) < kGradJobsL2) {
        it = jj / 4; jp = jj % 4; hrow = kActH1; zrow = kActZ2; nin = kMlpHid; ldw = kMlpHid; pw = kPW2; pb = kPB2;
    } else if ((jj -= kGradJobsL2) < kGradJobsL3) {
        it = jj / 4; jp = jj % 4; hrow = kActH2; zrow = kActZ3; nin = kMlpHid; ldw = kMlpHid; pw = kPW3; pb = kPB3;
    } else {
        jj -= kGradJobsL3;
        it = jj; jp = 0; hrow = kActH3; zrow = kActZ4; nin = kMlpHid; ldw = kMlpOut; pw = kPW4; pb = kPB4;
    }
    const int s = lane % 16, g = lane / 16;
    // this split's columns: chunks of 32 samples
    const int nchunk = kcols / 32;
    const int c0 = (int)((int64_t)nchunk * split / kGradSplits), c1 = (int)((int64_t)nchunk * (split + 1) / kGradSplits);
    const uint16_t *ha = act + (int64_t)(hrow + 16 * it + s) * cap + 8 * g;
    const uint16_t *zb0 = act + (int64_t)(zrow + 32 * jp + s) * cap + 8 * g;
    const uint16_t *zb1 = zb0 + 16 * cap;
    v4f32 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    for (int c = c0; c < c1; ++c) {
        const v8i16 a = *reinterpret_cast<const v8i16 *>(ha + 32 * c);
        const v8i16 b0 = *reinterpret_cast<const v8i16 *>(zb0 + 32 * c);
        const v8i16 b1 = *reinterpret_cast<const v8i16 *>(zb1 + 32 * c);
        acc0 = mfma32(a, b0, acc0);
        acc1 = mfma32(a, b1, acc1);
    }
    float *dst = part + (int64_t)split * kNParams;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const v4f32 acc = t ? acc1 : acc0;
        const float v[4] = {acc.x, acc.y, acc.z, acc.w};
        const int out = 16 * (2 * jp + t) + s;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int in = 16 * it + 4 * g + r;
            if (in < nin) dst[pw + in * ldw + out] = v[r];
            else if (in == nin) dst[pb + out] = v[r];  // the constant row: bias gradient
        }
    }
}

// The ones rows of the activation store (bias rows of H0..H3).
__global__ void mlp_act_init_kernel(uint16_t *act, int64_t cap) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap) return;
    const uint16_t one = 0x3F80;  // 1.0 in bf16
    for (int r = kMlpIn; r < kActRowsH0; ++r) act[(int64_t)(kActH0 + r) * cap + i] = (r == kMlpIn) ? one : 0;
    for (int l = 0; l < 3; ++l)
        for (int r = kMlpHid; r < kActRowsH; ++r)
            act[(int64_t)(kActH1 + l * kActRowsH + r) * cap + i] = (r == kMlpHid) ? one : 0;
}

// sum of the split partial gradients (fixed order)
__global__ void mlp_gsum_kernel(const float *part, float *grad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParams) return;
    float gsum = 0.0f;
    for (int sp = 0; sp < kGradSplits; ++sp) gsum += part[(int64_t)sp * kNParams + i];
    grad[i] = gsum;
}

// Adam (FP32 master, bias-corrected) on the summed split gradients.
__global__ void mlp_adam_kernel(float *p, float *m, float *v, const float *part, float lr, float b1, float b2,
                                float eps, float c1, float c2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParams) return;
    float gi = 0.0f;
    for (int sp = 0; sp < kGradSplits; ++sp) gi += part[(int64_t)sp * kNParams + i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Training quantile levels are uniform, clamped to the encoded range [1e-4, 1 - 1e-4]
// (the pinball loss uses the clamped level too).
__device__ __forceinline__ float train_level(uint32_t w) {
    return fminf(fmaxf(u01(w), kLevelMin), 1.0f - kLevelMin);
}

// Random batch: indices uniform over the records, four quantile levels and the
// row kind (conditional with probability 1/3).
__global__ void mlp_batch_kernel(int64_t n, uint32_t k0, uint32_t k1, uint32_t step, int batch, int32_t *idx,
                                 float *uq) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= batch) return;
    const uint4 r = philox(make_uint4(step, (uint32_t)i, 0u, 9u), k0, k1);
    const uint4 e = philox(make_uint4(step, (uint32_t)i, 1u, 9u), k0, k1);
    idx[i] = (int32_t)__umulhi(r.x, (uint32_t)n);
    float *q = uq + 5 * (int64_t)i;
    q[0] = train_level(r.y);
    q[1] = train_level(r.z);
    q[2] = train_level(r.w);
    q[3] = train_level(e.y);
    q[4] = (u01(e.x) < (1.0f / 3.0f)) ? 1.0f : 0.0f;
}

// Normalisation of the targets: mean and standard deviation over the valid
// records of each output's own target (|x_out| of face F over the records
// leaving through F; the face and side logits and the unused outputs keep
// mean 0, scale 1), FP64 accumulation, one block of 256 threads per output; three more
// blocks record the ranges of log10 a and log10 tau_c and the smallest log10
// depth of the valid records (where the network may then be used).
__global__ void mlp_norm_kernel(const float *rec, int64_t n, float *norm) {
    __shared__ double s0[256], s1[256], s2[256];
    const int k = blockIdx.x;
    double a = 0.0, b = 0.0, c = 0.0;
    if (k >= kMlpOut) {
        // ranges over the valid records: log10 a (block kMlpOut), log10 tau_c
        // (kMlpOut + 1), and the lower end of log10 depth (kMlpOut + 2)
        const int col = (k == kMlpOut) ? kRecLA : ((k == kMlpOut + 1) ? kRecLT : kRecLD);
        float lo = 1e30f, hi = -1e30f;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            const float *r = rec + (int64_t)kRec * i;
            if (r[kRecValid] < 0.5f) continue;
            lo = fminf(lo, r[col]);
            hi = fmaxf(hi, r[col]);
        }
        s1[threadIdx.x] = lo;
        s2[threadIdx.x] = hi;
        __syncthreads();
        for (int st = 128; st >= 1; st >>= 1) {
            if ((int)threadIdx.x < st) {
                s1[threadIdx.x] = fmin(s1[threadIdx.x], s1[threadIdx.x + st]);
                s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + st]);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const int o = kNormARange + 2 * (k - kMlpOut);
            norm[o] = (float)s1[0];
            if (k < kMlpOut + 2) norm[o + 1] = (float)s2[0];
            else norm[o + 1] = 0.0f;  // padding after the depth minimum
        }
        return;
    }
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const float *r = rec + (int64_t)kRec * i;
        float yf;
        if (r[kRecValid] < 0.5f || !target_value(r, k, yf)) continue;
        const double y = yf;
        a += y;
        b += y * y;
        c += 1.0;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    s0[threadIdx.x] = c;
    __syncthreads();
    for (int st = 128; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) {
            s1[threadIdx.x] += s1[threadIdx.x + st];
            s2[threadIdx.x] += s2[threadIdx.x + st];
            s0[threadIdx.x] += s0[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (s0[0] < 1.0) {
            norm[k] = 0.0f;
            norm[kMlpOut + k] = 1.0f;
        } else {
            const double mean = s1[0] / s0[0];
            const double var = s2[0] / s0[0] - mean * mean;
            norm[k] = (float)mean;
            norm[kMlpOut + k] = (float)sqrt(var > 1e-12 ? var : 1e-12);
        }
    }
}

// Forward for a list of raw rows in[n][kFwdRaw] = (log10 tau_c, log10 a, |x_in|,
// q0, q1, q2, log10 depth, m0, m1, m2, u_a, u_b, u_c, u_d, flag, x_out, face):
// out[n][32] normalised outputs back in their own variables (face and side
// logits as logits; ln E[N_s] with its calibration term; asinh of the offsets
// and mu^2 as learned).
__global__ void __launch_bounds__(256) mlp_forward_kernel(const unsigned char *blob, const float *inp,
                                                          int64_t n, float *out) {
    const int lane = __lane_id(), w = threadIdx.x / 64;
    const int64_t block = (int64_t)blockIdx.x * (blockDim.x / 64) + w;
    const int s = lane % 16, g = lane / 16;
    const int64_t si = block * 16 + s;
    if (block * 16 >= n) return;
    const bool live = si < n;
    const float *bias = reinterpret_cast<const float *>(blob + kTilesAll * kTileBytes);
    const float *norm = bias + kBiasFloats;
    const float *r = inp + (int64_t)kFwdRaw * (live ? si : 0);
    float in[kMlpIn];
    mlp_inputs(r, r[10], r[11], r[12], r[13], r[14] > 0.5f, r[15], (int)r[16], in);
    v4f32 o, ob;
    mlp_forward_block(blob, bias, xin_operand(in, lane), lane, NoEpi{}, o, ob);
    if (!live) return;
    const float v[8] = {o.x, o.y, o.z, o.w, ob.x, ob.y, ob.z, ob.w};
    for (int j = 0; j < 8; ++j) {
        const int k = (j < 4) ? 4 * g + j : 16 + 4 * g + (j - 4);
        out[kMlpOut * si + k] = v[j] * norm[kMlpOut + k] + norm[k] +
                                ((k == kOutLogN) ? norm[kNormCal + cal_bin(r[0], r[6], r[2])] : 0.0f);
    }
}

// Calibration sums over valid records with |x_in| <= kEscXMax (the range where
// the network is asked): per bin of (log10 tau_c, log10 depth, |x_in|), the
// number of records, sum N_s and sum exp(network ln E[N_s]) (without
// calibration), FP64.  One wave per 16-record block; block partial sums in LDS,
// then global atomics.
__global__ void __launch_bounds__(256) mlp_calib_kernel(const unsigned char *blob, const float *rec, int64_t n,
                                                        double *sums) {
    __shared__ double ls[3 * kNCal];
    for (int i = threadIdx.x; i < 3 * kNCal; i += blockDim.x) ls[i] = 0.0;
    __syncthreads();
    const int lane = __lane_id(), w = threadIdx.x / 64;
    const int64_t block = (int64_t)blockIdx.x * (blockDim.x / 64) + w;
    const int s = lane % 16, g = lane / 16;
    const int64_t si = block * 16 + s;
    if (block * 16 < n) {  // wave-uniform
        const float *r = rec + (int64_t)kRec * (si < n ? si : 0);
        const bool live = si < n && r[kRecValid] > 0.5f;
        const float *bias = reinterpret_cast<const float *>(blob + kTilesAll * kTileBytes);
        const float *norm = bias + kBiasFloats;
        // marginal row with quantile levels as the transport draws them: uniform,
        // from Philox(record index)
        const uint4 q = philox(make_uint4((uint32_t)si, (uint32_t)(si >> 32), 0u, 9u), 0x6C1Bu, 0x5EEDu);
        float in[kMlpIn];
        mlp_inputs(r, u01(q.x), u01(q.y), u01(q.z), u01(q.w), false, 0.0f, 0, in);
        v4f32 o, ob;
        mlp_forward_block(blob, bias, xin_operand(in, lane), lane, NoEpi{}, o, ob);
        static_assert(kOutLogN == 7, "ln E[N_s] sits in lane group 1, component 3");
        if (live && g == 1 && r[kRecX] <= kEscXMax) {
            const int b = cal_bin(r[kRecLT], r[kRecLD], r[kRecX]);
            const double pred = exp((double)(o.w * norm[kMlpOut + kOutLogN] + norm[kOutLogN]));
            atomicAdd(&ls[b], 1.0);
            atomicAdd(&ls[kNCal + b], exp((double)r[kRecLogN]));
            atomicAdd(&ls[2 * kNCal + b], pred);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * kNCal; i += blockDim.x)
        if (ls[i] != 0.0) atomicAdd(&sums[i], ls[i]);
}

// cal[b] = ln(sum N_s / sum predicted) for bins with at least 100 records, else 0
__global__ void mlp_calib_finish_kernel(const double *sums, float *norm) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= kNCal) return;
    const double cnt = sums[b], sn = sums[kNCal + b], sp = sums[2 * kNCal + b];
    norm[kNormCal + b] = (cnt >= 100.0 && sn > 0.0 && sp > 0.0) ? (float)log(sn / sp) : 0.0f;
}

// --------------------------------------------------------------- launch ---
hipError_t launch_cell_record(const RecordParams &R, int grid, hipStream_t s) {
    size_t lds = sizeof(float) * kTabFloats;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(cell_record_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(cell_record_kernel, dim3(grid), dim3(256), lds, s, R);
    return hipGetLastError();
}

hipError_t launch_mlp_init(float *p, uint32_t k0, uint32_t k1, hipStream_t s) {
    hipLaunchKernelGGL(mlp_init_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, s, p, k0, k1);
    return hipGetLastError();
}

hipError_t launch_mlp_pack(const float *p, const float *norm, unsigned char *blob, unsigned char *img,
                           hipStream_t s) {
    int n = kTilesAll * 64;
    hipLaunchKernelGGL(mlp_pack_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, norm, blob);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !img) return e;
    int nb = kMlpFwdBytes;
    hipLaunchKernelGGL(mlp_fwd_image_kernel, dim3((nb + 255) / 256), dim3(256), 0, s, blob, img);
    return hipGetLastError();
}

hipError_t launch_mlp_act_init(uint16_t *act, int64_t cap, hipStream_t s) {
    hipLaunchKernelGGL(mlp_act_init_kernel, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, act, cap);
    return hipGetLastError();
}

// Gradient of the mean loss over a batch into the split partials `part`.
hipError_t launch_mlp_grad(const unsigned char *blob, const float *rec, const int32_t *idx, const float *uq,
                           int batch, uint16_t *act, int64_t cap, float *part, float *loss, hipStream_t s) {
    const int kcols = 32 * ((batch + 31) / 32);
    const int nblocks = kcols / 16;
    hipLaunchKernelGGL(mlp_fwdbwd_kernel, dim3((nblocks + 3) / 4), dim3(256), 0, s, blob, rec, idx, uq, batch, act,
                       cap, loss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int jobs = kGradJobs * kGradSplits;
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3((jobs + 3) / 4), dim3(256), 0, s, act, cap, kcols, part);
    return hipGetLastError();
}

hipError_t launch_mlp_gsum(const float *part, float *grad, hipStream_t s) {
    hipLaunchKernelGGL(mlp_gsum_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, s, part, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *p, float *m, float *v, const float *part, float lr, int step, hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f;
    float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, s, p, m, v, part, lr, b1, b2,
                       1e-8f, c1, c2);
    return hipGetLastError();
}

hipError_t launch_mlp_batch(int64_t n, uint32_t k0, uint32_t k1, uint32_t step, int batch, int32_t *idx,
                            float *uq, hipStream_t s) {
    hipLaunchKernelGGL(mlp_batch_kernel, dim3((batch + 255) / 256), dim3(256), 0, s, n, k0, k1, step, batch,
                       idx, uq);
    return hipGetLastError();
}

hipError_t launch_mlp_calib(const unsigned char *blob, const float *rec, int64_t n, double *sums, float *norm,
                            hipStream_t s) {
    int64_t blocks = (n + 63) / 64;  // 4 waves of 16 records per block
    hipLaunchKernelGGL(mlp_calib_kernel, dim3((unsigned)blocks), dim3(256), 0, s, blob, rec, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp_calib_finish_kernel, dim3((kNCal + 255) / 256), dim3(256), 0, s, sums, norm);
    return hipGetLastError();
}

hipError_t launch_mlp_norm(const float *rec, int64_t n, float *norm, hipStream_t s) {
    hipLaunchKernelGGL(mlp_norm_kernel, dim3(kMlpOut + 3), dim3(256), 0, s, rec, n, norm);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const unsigned char *blob, const float *inp, int64_t n, float *out, hipStream_t s) {
    int64_t nblocks = (n + 15) / 16;
    int grid = (int)((nblocks + 3) / 4);
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(grid), dim3(256), 0, s, blob, inp, n, out);
    return hipGetLastError();
}

}  // namespace krt
