// krt_mlp.h -- the learned escape proposal: layout constants and the BF16-MFMA
// forward pass shared by the transport kernel (inference) and the training
// kernels.  Not part of the C ABI.
//
// Network: 8 inputs -> 128 -> 128 -> 128 (SiLU) -> 10 outputs.
// Inputs  : ((log10 tau_R - 3.5)/1.5, log10 a + 3, x_in / 4, L(u_a), L(u_b),
//           w, r_in, flag), L(u) = logit(u) / 4 the encoding of a quantile
//           level: extreme levels get distinct inputs, so the far wing of the
//           exit frequency (the rare long flights by which photons leave a thick
//           medium) is not flattened.  A *marginal* evaluation (flag 0,
//           w = L(u_c), r_in 0) gives the exit frequency, exit point and count at three
//           independent quantile levels; a *conditional* one (flag 1,
//           w = x_out / 4, r_in = sqrt2 r - 1) gives the exit direction given
//           the sampled exit frequency and the exit point's distance r from the
//           face centre, since photons leaving near an edge travel more
//           obliquely and away from the centre, and wing photons leave closer
//           to the normal.
// Outputs (normalised): marginal: 0 quantile at u_a of x_out given x_out >= 0;
//           1, 2 quantiles at u_b, u_c of the exit point (s, t) on the exit
//           face; 4 ln E[N_s] (scatterings inside the cube); 5 quantile at u_a
//           of ln <x^2> over those scatterings; 6 logit P(x_out >= 0); 7
//           quantile at u_a of -x_out given x_out < 0.  Conditional: 3 quantile
//           at u_a of the cosine mu of the exit direction to the face normal; 8
//           quantile at u_b of the angle alpha between the direction's
//           tangential part and the exit point's offset (s, t).  9 unused (the
//           parameter count stays even).  The exit frequency is bimodal, so it
//           is drawn as a two-component mixture (side, then a one-sided
//           quantile): a single smooth quantile function of the signed x_out
//           would fill the empty line core between the peaks.
//
// The layers are evaluated transposed, H^T_{l+1} = SiLU(W_l^T H^T_l + b_l),
// with v_mfma_f32_16x16x16_bf16 on 16-sample blocks: the accumulator layout of
// one layer (lane l holds features 4(l/16)+j of sample l%16) is exactly the B
// operand layout of the next, so activations never leave registers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace krt {

constexpr int kMlpIn = 8, kMlpHid = 128, kMlpOut = 10;
// output indices
constexpr int kOutXPos = 0, kOutS = 1, kOutT = 2, kOutMu = 3, kOutLogN = 4, kOutLogX2 = 5, kOutLogit = 6,
              kOutXNeg = 7, kOutAlpha = 8, kOutSpare = 9;
// escape record layout (floats per record) and its columns
constexpr int kRec = 11;
constexpr int kRecXOut = 3, kRecS = 4, kRecT = 5, kRecMu = 6, kRecLogN = 7, kRecLogX2 = 8, kRecValid = 9,
              kRecAlpha = 10;
// ln E[N_s]: weighted log-deviance loss with its exponent clamped
constexpr float kDevClamp = 4.0f;
constexpr float kDevWeight = 0.25f;
// FP32 master parameter block (offsets in floats)
constexpr int kPW1 = 0;                                  // W1[8][128]   (in, out)
constexpr int kPB1 = kPW1 + kMlpIn * kMlpHid;            // b1[128]
constexpr int kPW2 = kPB1 + kMlpHid;                     // W2[128][128]
constexpr int kPB2 = kPW2 + kMlpHid * kMlpHid;
constexpr int kPW3 = kPB2 + kMlpHid;
constexpr int kPB3 = kPW3 + kMlpHid * kMlpHid;
constexpr int kPW4 = kPB3 + kMlpHid;                     // W4[128][10]
constexpr int kPB4 = kPW4 + kMlpHid * kMlpOut;           // b4[10]
constexpr int kNParams = kPB4 + kMlpOut;                 // 35466
// target normalisation: y_norm = (y - mean) / scale, stored after the params
// (output 6, the side logit, and the unused output 9 have mean 0 and scale 1),
// followed by the
// calibration of ln E[N_s]: an additive term per bin of (log10 tau_R, |x_in|)
constexpr int kNCalT = 32, kNCalX = 8, kNCal = kNCalT * kNCalX;
constexpr float kCalLo = 1.0f, kCalInvW = 8.0f;  // bins of 0.125 in log10 tau_R from 1 to 5
// then the range of log10 a of the training records (min, max; a network is
// used only at damping values inside it) and two floats of padding
constexpr int kNormARange = 2 * kMlpOut + kNCal;
constexpr int kNNorm = 2 * kMlpOut + kNCal + 4;

// The network is asked only for |x_in| <= kEscXMax (gas frame).  Beyond it the
// mean count is a steep mixture of photons that leave at once and photons
// redistributed into the core; a wing photon takes plain scatterings until it
// is back in the core, which costs little (about 0.5% of the scatterings in a
// thick cell have |x| > 2).  Records draw x_in over [-kRecXMax, kRecXMax].
constexpr float kEscXMax = 2.0f;
constexpr float kRecXMax = 3.0f;

// |x_in| bins of 0.25 over [0, kEscXMax) (the last one also takes larger |x_in|)
__device__ __forceinline__ int cal_bin(float lt, float xin) {
    const int bt = min(max((int)((lt - kCalLo) * kCalInvW), 0), kNCalT - 1);
    const int bx = min((int)(fabsf(xin) * (kNCalX / kEscXMax)), kNCalX - 1);
    return bt * kNCalX + bx;
}

// Packed BF16 A-operand tiles (16x16, 512 B each: 64 lanes x 4 bf16).
// Forward (W^T, rows = out-features): L1 8 tiles (K padded 8 -> 16), L2 64, L3 64, L4 8 (rows padded 10 -> 16).
constexpr int kTilesL1 = 8, kTilesL2 = 64, kTilesL3 = 64, kTilesL4 = 8;
constexpr int kTileFwdL1 = 0, kTileFwdL2 = kTilesL1, kTileFwdL3 = kTileFwdL2 + kTilesL2,
              kTileFwdL4 = kTileFwdL3 + kTilesL3, kTilesFwd = kTileFwdL4 + kTilesL4;   // 144
// Backward (W, rows = in-features): L4 8 tiles (K = 16 padded outputs), L3 64, L2 64.
constexpr int kTileBwdL4 = kTilesFwd, kTileBwdL3 = kTileBwdL4 + 8, kTileBwdL2 = kTileBwdL3 + 64,
              kTilesAll = kTileBwdL2 + 64;                                              // 280
constexpr int kTileBytes = 512;
// biases as FP32 after the tiles: b1 128, b2 128, b3 128, b4 16 (padded)
constexpr int kBiasFloats = 3 * kMlpHid + 16;
constexpr int kMlpFwdBytes = kTilesFwd * kTileBytes + kBiasFloats * 4 + kNNorm * 4;  // LDS image for inference
constexpr int kMlpBlobBytes = kTilesAll * kTileBytes + kBiasFloats * 4 + kNNorm * 4;
static_assert(kMlpIn <= 8 && kMlpOut <= 16, "inputs fill two lane groups, outputs one 16-row tile");
static_assert(kMlpFwdBytes % 16 == 0, "the inference image is staged into LDS in 16-byte words");

// Network input of a quantile level u: logit(u) / 4 with u clamped to the
// trained levels [1e-4, 1 - 1e-4]: beyond them the network would extrapolate
// the quantile function (far too far into the wing), so the outermost 2e-4 of
// the draws take the 1e-4 and 1 - 1e-4 quantiles
constexpr float kLevelMin = 1e-4f;
__device__ __forceinline__ float level_in(float u) {
    u = fminf(fmaxf(u, kLevelMin), 1.0f - kLevelMin);
    return 0.25f * (__logf(u) - __logf(1.0f - u));
}

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

// logistic(z) from the hardware exp2 and reciprocal (about 1 ulp each; the
// activations are stored as bfloat16, 8 significant bits)
__device__ __forceinline__ float sigmoid_f(float z) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.44269504088896f * z));
}
__device__ __forceinline__ float silu(float z) { return z * sigmoid_f(z); }

__device__ __forceinline__ v4i16 pack4(float a, float b, float c, float d) {
    v4i16 r;
    r.x = (short)f2bf(a); r.y = (short)f2bf(b); r.z = (short)f2bf(c); r.w = (short)f2bf(d);
    return r;
}

__device__ __forceinline__ v4f32 mfma16(v4i16 a, v4i16 b, v4f32 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// A operand of tile t for this lane from a byte blob (LDS or global)
__device__ __forceinline__ v4i16 tileA(const unsigned char *blob, int t, int lane) {
    return *reinterpret_cast<const v4i16 *>(blob + t * kTileBytes + lane * 8);
}

// Forward pass of one 16-sample block.  xin: this lane's B operand for layer 1
// (lanes 0..15 hold inputs 0..3 of sample l%16, lanes 16..31 inputs 4..7,
// other lanes zeros).  Returns
// the output tile (lane l: outputs 4(l/16)+j of sample l%16).  If z1..z3 are
// given, the pre-activations are stored (8 tiles each) for the backward pass.
__device__ __forceinline__ v4f32 mlp_forward_block(const unsigned char *tiles, const float *bias,
                                                   v4i16 xin, int lane, v4f32 *z1, v4f32 *z2,
                                                   v4f32 *z3) {
    const int g = lane >> 4;
    v4i16 h[8];
    // layer 1
#pragma unroll
    for (int mo = 0; mo < 8; ++mo) {
        const float *b = bias + 16 * mo + 4 * g;
        v4f32 acc = {b[0], b[1], b[2], b[3]};
        acc = mfma16(tileA(tiles, kTileFwdL1 + mo, lane), xin, acc);
        if (z1) z1[mo] = acc;
        h[mo] = pack4(silu(acc.x), silu(acc.y), silu(acc.z), silu(acc.w));
    }
    // layers 2, 3
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const int t0 = layer == 0 ? kTileFwdL2 : kTileFwdL3;
        const float *bl = bias + kMlpHid * (layer + 1);
        v4f32 acc[8];
#pragma unroll
        for (int mo = 0; mo < 8; ++mo) {
            const float *b = bl + 16 * mo + 4 * g;
            acc[mo] = (v4f32){b[0], b[1], b[2], b[3]};
#pragma unroll
            for (int ki = 0; ki < 8; ++ki) acc[mo] = mfma16(tileA(tiles, t0 + mo * 8 + ki, lane), h[ki], acc[mo]);
        }
        v4f32 *zs = layer == 0 ? z2 : z3;
#pragma unroll
        for (int mo = 0; mo < 8; ++mo) {
            if (zs) zs[mo] = acc[mo];
            h[mo] = pack4(silu(acc[mo].x), silu(acc[mo].y), silu(acc[mo].z), silu(acc[mo].w));
        }
    }
    // layer 4 (outputs padded to 16)
    const float *b4 = bias + 3 * kMlpHid + 4 * g;
    v4f32 out = {b4[0], b4[1], b4[2], b4[3]};
#pragma unroll
    for (int ki = 0; ki < 8; ++ki) out = mfma16(tileA(tiles, kTileFwdL4 + ki, lane), h[ki], out);
    return out;
}

}  // namespace krt
