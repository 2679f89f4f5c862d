// krt_mlp.h -- the learned whole-cell escape: layout constants and the
// BF16-MFMA forward pass shared by the transport kernel (inference) and the
// training kernels.  Not part of the C ABI.
//
// The network describes how a photon that scatters inside a homogeneous static
// cubic cell leaves it.  Conditions are taken in the cell's reduced frame: the
// start point's absolute offsets from the cell centre (in half-widths) sorted
// ascending, q0 <= q1 <= q2 (axis 2 points to the nearest face), the incoming
// direction reflected and permuted alike, and |x_in| (the medium is symmetric
// under x -> -x, so the exit frequency takes x_in's sign).
//
// Network: 24 inputs -> 128 -> 128 -> 128 (leaky ReLU) -> 32 outputs.
// Inputs: 0 (log10 tau_c - 3)/1.2 (tau_c the line-centre depth centre to face),
//   1 log10 a + 3, 2 |x_in| - 1, 3-5 2 q - 1, 6 (log10 depth - 2)/1.2 (depth
//   tau_c (1 - q2) to the nearest face), 7-9 incoming direction, 10-13 quantile
//   levels L(u_a..u_d), L(u) = logit(u)/4, 14 flag (0 marginal, 1 conditional),
//   15 conditional: x_out/4, 16-21 conditional: one-hot exit face, 22-23 zero.
// Outputs (normalised): marginal: 0-5 exit-face logits (face F = 2 axis +
//   (outward normal along +axis)); 6 logit P(x_out >= 0); 7 ln E[N_s];
//   8 quantile at u_b of ln <x^2> over the skipped scatterings; 16 + F
//   quantile at u_a of |x_out| given exit face F (the magnitude depends
//   strongly on the face, its sign hardly).  Conditional (given the exit face
//   and x_out): 9, 10 quantiles at u_a, u_b of asinh of the exit offsets ys, yt
//   from the start point's projection onto the exit face (along the two axes
//   following the exit axis cyclically) over the start point's distance to
//   that face's plane; 11 quantile at u_c of mu^2, mu the exit cosine; 12
//   quantile at u_d of the angle alpha between the exit direction's
//   tangential part and that offset.  13-15 and 22-31 unused.  asinh and the
//   square are monotone, so the quantiles map back through their inverses;
//   they remove the offsets' heavy tails and the steep quantile function of
//   mu near 0.
//
// Layers run transposed, H^T_{l+1} = leaky(W_l^T H^T_l + b_l), on 16-sample
// blocks with v_mfma_f32_16x16x32_bf16.  The accumulator of a 16-feature tile
// leaves lane l with features 4(l/16)+r of sample l%16; the B operand of the
// next layer wants 8 features per lane.  The reduction index of each 32-wide
// chunk c is therefore permuted: B slot 8g+j holds feature
// 32c + 4g + j (j < 4) or 32c + 16 + 4g + (j - 4) (j >= 4), i.e. the
// accumulators of tiles 2c and 2c+1 side by side, and the weight tiles are
// packed with the same permutation (kperm), so activations never leave
// registers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace krt {

constexpr int kMlpIn = 24, kMlpInPad = 32, kMlpHid = 128, kMlpOut = 32;
// Layer 1 sees 28 operand slots: the 24 inputs rounded to bfloat16, then in
// slots 24-27 the rounding residuals of the four quantile levels (inputs
// 10-13), whose weights are tied to those levels' rows of W1.  A level then
// enters with about 16 significant bits instead of 8: with the level alone in
// bfloat16, the samples of a quantile output would take a few hundred
// discrete values per condition (a comb in the sampled distributions).
constexpr int kMlpLevelIn = 10, kMlpResIn = 24, kMlpOperandIn = 28;
// output indices
constexpr int kOutFace = 0, kOutSide = 6, kOutLogN = 7, kOutLogX2 = 8, kOutYS = 9, kOutYT = 10, kOutMu2 = 11,
              kOutAlpha = 12, kOutXAbs = 16;
// whole-cell escape record (floats per record) and its columns
constexpr int kRec = 20;
constexpr int kRecLT = 0, kRecLA = 1, kRecX = 2, kRecQ0 = 3, kRecLD = 6, kRecN0 = 7, kRecFace = 10, kRecYS = 11,
              kRecYT = 12, kRecMu = 13, kRecAlpha = 14, kRecXOut = 15, kRecLogN = 16, kRecLogX2 = 17,
              kRecValid = 18;
// ln E[N_s]: weighted log-deviance loss with its exponent clamped
constexpr float kDevClamp = 4.0f;
constexpr float kDevWeight = 0.25f;
// FP32 master parameter block (offsets in floats)
constexpr int kPW1 = 0;                                  // W1[24][128]   (in, out)
constexpr int kPB1 = kPW1 + kMlpIn * kMlpHid;            // b1[128]
constexpr int kPW2 = kPB1 + kMlpHid;                     // W2[128][128]
constexpr int kPB2 = kPW2 + kMlpHid * kMlpHid;
constexpr int kPW3 = kPB2 + kMlpHid;
constexpr int kPB3 = kPW3 + kMlpHid * kMlpHid;
constexpr int kPW4 = kPB3 + kMlpHid;                     // W4[128][32]
constexpr int kPB4 = kPW4 + kMlpHid * kMlpOut;           // b4[32]
constexpr int kNParams = kPB4 + kMlpOut;                 // 40352
// Normalisation block after the parameters: target mean[32], scale[32] (face
// logits, side logit and the unused outputs: 0 and 1), then the calibration of
// ln E[N_s] (an additive term per bin of log10 tau_c, log10 depth and |x_in|),
// then the ranges of the training records, where the network may be used:
// log10 a (min, max), log10 tau_c (min, max), the smallest log10 depth, and
// three floats of padding (the LDS image stays a whole number of 16-byte words).
constexpr int kNCalT = 8, kNCalD = 8, kNCalX = 4, kNCal = kNCalT * kNCalD * kNCalX;  // 256
constexpr int kNormCal = 2 * kMlpOut;
constexpr int kNormARange = kNormCal + kNCal;
constexpr int kNormTauRange = kNormARange + 2;
constexpr int kNormDepthMin = kNormARange + 4;
constexpr int kNNorm = kNormARange + 8;                  // 328

// The network is asked only for gas-frame |x_in| <= kEscXMax: beyond it the
// count is a steep mixture of photons that leave at once and photons sent back
// into the core; wing photons take plain scatterings until they are back in
// the core.  Records draw |x_in| up to kRecXMax.
constexpr float kEscXMax = 2.0f;
constexpr float kRecXMax = 3.0f;

// calibration bin: log10 tau_c in 8 bins of 0.5 over [1, 5), log10 depth in 8
// bins of 0.5 over [0, 4), |x_in| in 4 bins of 0.5 over [0, 2) (ends clamped)
__device__ __forceinline__ int cal_bin(float lt, float ld, float xa) {
    const int bt = min(max((int)((lt - 1.0f) * 2.0f), 0), kNCalT - 1);
    const int bd = min(max((int)(ld * 2.0f), 0), kNCalD - 1);
    const int bx = min(max((int)(xa * 2.0f), 0), kNCalX - 1);
    return (bt * kNCalD + bd) * kNCalX + bx;
}

// Packed BF16 A-operand tiles, 16 rows x 32 reduction entries (1 KiB: 64 lanes
// x 8 bf16; lane l holds row l%16, entries 8(l/16)..8(l/16)+7).
// Forward (W^T, rows = out-features): L1 8 tiles (inputs 24 padded to 32),
// L2 32 (8 row tiles x 4 chunks), L3 32, L4 8 (2 row tiles of 16 outputs x 4
// chunks, tile 4 ot + c).
constexpr int kTileFwdL1 = 0, kTileFwdL2 = 8, kTileFwdL3 = kTileFwdL2 + 32, kTileFwdL4 = kTileFwdL3 + 32,
              kTilesFwd = kTileFwdL4 + 8;                                                 // 80
// Backward (W, rows = in-features): L4 8 tiles (the 32 outputs are one chunk), L3 32, L2 32.
constexpr int kTileBwdL4 = kTilesFwd, kTileBwdL3 = kTileBwdL4 + 8, kTileBwdL2 = kTileBwdL3 + 32,
              kTilesAll = kTileBwdL2 + 32;                                               // 152
constexpr int kTileBytes = 1024;
// biases as FP32 after the tiles: b1 128, b2 128, b3 128, b4 32
constexpr int kBiasFloats = 3 * kMlpHid + kMlpOut;
constexpr int kMlpFwdBytes = kTilesFwd * kTileBytes + kBiasFloats * 4 + kNNorm * 4;  // LDS image for inference
constexpr int kMlpBlobBytes = kTilesAll * kTileBytes + kBiasFloats * 4 + kNNorm * 4;
static_assert(kMlpIn <= kMlpInPad && kMlpOut == 32, "inputs fill one 32-wide chunk, outputs two tiles");
// training: activation-store rows and the sample splits of the weight-gradient product
constexpr int kActRowsAll = 32 + 3 * 144 + 3 * kMlpHid + kMlpOut;   // 880
constexpr int kGradSplits = 8;
// raw input row of krt_escape_forward: (log10 tau_c, log10 a, |x_in|, q0, q1,
// q2, log10 depth, m0, m1, m2, u_a, u_b, u_c, u_d, flag, x_out, face)
constexpr int kFwdRaw = 17;
static_assert(kMlpFwdBytes % 16 == 0, "the inference image is staged into LDS in 16-byte words");

// Feature held by B-operand slot k' = 8g + j of 32-wide chunk c (see above).
__host__ __device__ constexpr int kperm(int c, int kp) {
    return 32 * c + ((kp & 7) < 4 ? 4 * (kp >> 3) + (kp & 7) : 16 + 4 * (kp >> 3) + (kp & 7) - 4);
}

// Network input of a quantile level u: logit(u) / 4 with u clamped to the
// trained levels [1e-4, 1 - 1e-4]: beyond them the network would extrapolate
// the quantile function, so the outermost 2e-4 of the draws take the 1e-4 and
// 1 - 1e-4 quantiles
constexpr float kLevelMin = 1e-4f;
__device__ __forceinline__ float level_in(float u) {
    u = fminf(fmaxf(u, kLevelMin), 1.0f - kLevelMin);
    return 0.25f * (__logf(u) - __logf(1.0f - u));
}

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef short v8i16 __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf16 __attribute__((ext_vector_type(8)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

typedef __bf16 v2bf16 __attribute__((ext_vector_type(2)));
typedef float v2f32 __attribute__((ext_vector_type(2)));

// float -> bfloat16, round to nearest even: one v_cvt_pk_bf16_f32 per pair
__device__ __forceinline__ uint32_t pack2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f32){a, b}, v2bf16));
}
__device__ __forceinline__ uint16_t f2bf(float f) { return (uint16_t)(pack2(f, 0.0f) & 0xFFFFu); }

// logistic(z) from the hardware exp2 and reciprocal (about 1 ulp each)
__device__ __forceinline__ float sigmoid_f(float z) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.44269504088896f * z));
}
// Hidden activation: leaky ReLU, max(z, z / 16) (derivative 1 or 1/16).  Two
// full-rate instructions per value: the network runs inside the transport
// kernel, where a transcendental activation (SiLU: an exp and a reciprocal,
// quarter rate each) cost more issue cycles than the matrix products.  The max
// is the median of (z, z / 16, +inf): fmaxf would first quiet a possible
// signalling NaN in the MFMA result with one more instruction per value.
constexpr float kLeak = 0.0625f;
__device__ __forceinline__ float leaky(float z) { return __builtin_amdgcn_fmed3f(z, kLeak * z, 3.40282347e38f); }

__device__ __forceinline__ v4i16 pack4(float a, float b, float c, float d) {
    const uint32_t lo = pack2(a, b), hi = pack2(c, d);
    return (v4i16){(short)(lo & 0xFFFFu), (short)(lo >> 16), (short)(hi & 0xFFFFu), (short)(hi >> 16)};
}

__device__ __forceinline__ v8i16 cat8(v4i16 a, v4i16 b) { return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7); }

__device__ __forceinline__ v4f32 mfma32(v8i16 a, v8i16 b, v4f32 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf16, a), __builtin_bit_cast(v8bf16, b), c,
                                                   0, 0, 0);
}

// A operand of tile t for this lane from a byte blob (LDS or global)
__device__ __forceinline__ v8i16 tileA(const unsigned char *blob, int t, int lane) {
    return *reinterpret_cast<const v8i16 *>(blob + t * kTileBytes + lane * 16);
}

// Forward pass of one 16-sample block.  xin: this lane's B operand for layer 1
// (lane l holds inputs 8(l/16)..8(l/16)+7 of sample l%16).  Returns the two
// output tiles: lane l holds outputs 4(l/16)+r (oa) and 16+4(l/16)+r (ob) of
// sample l%16.  epi(layer, tile, z) sees each hidden layer's pre-activations
// (layer 0..2, row tile 0..7) before the activation: the training pass stores
// what its backward pass needs; inference passes NoEpi.
//
// The 80 products run in one fixed order (fwd_tile): layer 1's 8 row tiles,
// layers 2 and 3 chunk-major (the 8 row tiles of reduction chunk c, then
// c + 1, so consecutive products never wait on each other's result), the
// output layer chunk-major over its 2 row tiles.  Weight tiles stream through
// a window of 8 registers: product i reads slot i % 8 and the same slot is
// refilled at once with tile i + 8, so every LDS read is issued 8 products
// (about 130 cycles of matrix work) before its use and only 8 tiles are live.
// A scheduling barrier after each step keeps that order; left free, the
// compiler sinks each read to just before its product and waits on it (on the
// turbulent cloud the pinned order makes the fused transport kernel 7% faster
// for 20 bytes of spill per lane).
// A layer's epilogue applies the activation, packs the bf16 activations and loads the
// next layer's biases into the freed accumulators.
__host__ __device__ constexpr int fwd_tile(int i) {
    return i < 8    ? kTileFwdL1 + i
           : i < 40 ? kTileFwdL2 + ((i - 8) % 8) * 4 + (i - 8) / 8
           : i < 72 ? kTileFwdL3 + ((i - 40) % 8) * 4 + (i - 40) / 8
                    : kTileFwdL4 + ((i - 72) % 2) * 4 + (i - 72) / 2;
}
constexpr int kFwdSteps = 80;
static_assert(kTilesFwd == kFwdSteps, "one product per forward tile");

__device__ __forceinline__ v4f32 ld4(const float *p) { return *reinterpret_cast<const v4f32 *>(p); }

struct NoEpi {
    __device__ __forceinline__ void operator()(int, int, const v4f32 &) const {}
};

template <class Epi>
__device__ __forceinline__ void mlp_forward_block(const unsigned char *tiles, const float *bias, v8i16 xin,
                                                  int lane, Epi epi, v4f32 &oa, v4f32 &ob) {
    const int g = lane >> 4;
    v8i16 w[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = tileA(tiles, fwd_tile(i), lane);
    v4f32 acc[8];
#pragma unroll
    for (int mo = 0; mo < 8; ++mo) acc[mo] = ld4(bias + 16 * mo + 4 * g);
    v4i16 h[8];
    // product i (a compile-time index once unrolled) into accumulator c
#define KRT_FWD_STEP(i, bop, c)                                                         \
    do {                                                                                \
        (c) = mfma32(w[(i) % 8], (bop), (c));                                           \
        if ((i) + 8 < kFwdSteps) w[(i) % 8] = tileA(tiles, fwd_tile((i) + 8), lane);    \
        __builtin_amdgcn_sched_barrier(0);                                              \
    } while (0)
    // layer 1: one chunk (the inputs)
#pragma unroll
    for (int mo = 0; mo < 8; ++mo) KRT_FWD_STEP(mo, xin, acc[mo]);
#pragma unroll
    for (int mo = 0; mo < 8; ++mo) {
        epi(0, mo, acc[mo]);
        h[mo] = pack4(leaky(acc[mo].x), leaky(acc[mo].y), leaky(acc[mo].z), leaky(acc[mo].w));
        acc[mo] = ld4(bias + kMlpHid + 16 * mo + 4 * g);
    }
    // layers 2 and 3
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const int base = 8 + 32 * layer;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const v8i16 bop = cat8(h[2 * c], h[2 * c + 1]);
#pragma unroll
            for (int mo = 0; mo < 8; ++mo) KRT_FWD_STEP(base + 8 * c + mo, bop, acc[mo]);
        }
#pragma unroll
        for (int mo = 0; mo < 8; ++mo) {
            epi(1 + layer, mo, acc[mo]);
            h[mo] = pack4(leaky(acc[mo].x), leaky(acc[mo].y), leaky(acc[mo].z), leaky(acc[mo].w));
            if (layer == 0) acc[mo] = ld4(bias + 2 * kMlpHid + 16 * mo + 4 * g);
        }
    }
    // output layer: two row tiles, biases b4
    v4f32 o[2] = {ld4(bias + 3 * kMlpHid + 4 * g), ld4(bias + 3 * kMlpHid + 16 + 4 * g)};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const v8i16 bop = cat8(h[2 * c], h[2 * c + 1]);
#pragma unroll
        for (int ot = 0; ot < 2; ++ot) KRT_FWD_STEP(72 + 2 * c + ot, bop, o[ot]);
    }
#undef KRT_FWD_STEP
    oa = o[0];
    ob = o[1];
}

// ------------------------------------------------------------- inputs ---
// Raw condition (lt, la, |x|, q0, q1, q2, ld, m0, m1, m2) + levels + row kind
// (+ exit face and x_out of a conditional row) -> normalised inputs.
__device__ __forceinline__ void mlp_inputs(const float *c, float ua, float ub, float uc, float ud, bool cond,
                                           float xout, int face, float in[kMlpIn]) {
    in[0] = (c[0] - 3.0f) * (1.0f / 1.2f);
    in[1] = c[1] + 3.0f;
    in[2] = c[2] - 1.0f;
    in[3] = 2.0f * c[3] - 1.0f;
    in[4] = 2.0f * c[4] - 1.0f;
    in[5] = 2.0f * c[5] - 1.0f;
    in[6] = (c[6] - 2.0f) * (1.0f / 1.2f);
    in[7] = c[7];
    in[8] = c[8];
    in[9] = c[9];
    in[10] = level_in(ua);
    in[11] = level_in(ub);
    in[12] = level_in(uc);
    in[13] = level_in(ud);
    in[14] = cond ? 1.0f : 0.0f;
    in[15] = cond ? 0.25f * xout : 0.0f;
#pragma unroll
    for (int f = 0; f < 6; ++f) in[16 + f] = (cond && face == f) ? 1.0f : 0.0f;
    in[22] = 0.0f;
    in[23] = 0.0f;
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// operand slot k of layer 1 (k < kMlpOperandIn): the inputs, then the level residuals
__device__ __forceinline__ float operand_in(const float in[kMlpIn], int k) {
    if (k < kMlpIn) return in[k];
    const float l = in[kMlpLevelIn + k - kMlpResIn];
    return l - bf2f(f2bf(l));
}

// this lane's layer-1 B operand: slots 8(l/16)..8(l/16)+7 (slots 28-31 zero)
__device__ __forceinline__ v8i16 xin_operand(const float in[kMlpIn], int lane) {
    const int g = lane >> 4;
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float a0 = operand_in(in, j), a1 = operand_in(in, 8 + j), a2 = operand_in(in, 16 + j);
        const float a3 = (j < 4) ? operand_in(in, 24 + j) : 0.0f;
        v[j] = (g == 0) ? a0 : ((g == 1) ? a1 : ((g == 2) ? a2 : a3));
    }
    return cat8(pack4(v[0], v[1], v[2], v[3]), pack4(v[4], v[5], v[6], v[7]));
}

// the 28 operand slots as 14 dwords of bf16 pairs (dwords 4g..4g+3 are the
// layer-1 B operand of lane group g; group 3 has two)
constexpr int kMlpPackDw = kMlpOperandIn / 2;
__device__ __forceinline__ void pack_inputs(const float in[kMlpIn], uint32_t pk[kMlpPackDw]) {
#pragma unroll
    for (int d = 0; d < kMlpPackDw; ++d)
        pk[d] = pack2(operand_in(in, 2 * d), operand_in(in, 2 * d + 1));
}

// ------------------------------------------------------ the reduced frame ---
// Reduction of a start state in a cubic cell: p in [-1, 1]^3 (offsets from the
// cell centre in half-widths), n the incoming direction.  sg[k] = sign of p_k
// (+1 at 0); perm[r] = the cell axis of reduced axis r (ascending |p|; ties
// keep axis order); q[r] = |p_perm[r]|; m[r] = sg[perm[r]] n_perm[r].
struct CellFrame {
    int perm[3];
    float sg[3];
    float q[3];
};

__device__ __forceinline__ void cell_reduce(float px, float py, float pz, CellFrame &F) {
    F.sg[0] = px < 0.0f ? -1.0f : 1.0f;
    F.sg[1] = py < 0.0f ? -1.0f : 1.0f;
    F.sg[2] = pz < 0.0f ? -1.0f : 1.0f;
    const float a0 = fabsf(px), a1 = fabsf(py), a2 = fabsf(pz);
    // stable sort of three values by compare-and-swap on (value, axis)
    float v0 = a0, v1 = a1, v2 = a2;
    int i0 = 0, i1 = 1, i2 = 2;
    if (v1 < v0) { float t = v0; v0 = v1; v1 = t; int s = i0; i0 = i1; i1 = s; }
    if (v2 < v1) { float t = v1; v1 = v2; v2 = t; int s = i1; i1 = i2; i2 = s; }
    if (v1 < v0) { float t = v0; v0 = v1; v1 = t; int s = i0; i0 = i1; i1 = s; }
    F.perm[0] = i0; F.perm[1] = i1; F.perm[2] = i2;
    F.q[0] = v0; F.q[1] = v1; F.q[2] = v2;
}

// component r of a cell-frame vector v in the reduced frame, and back
__device__ __forceinline__ float pick3(float x, float y, float z, int k) { return k == 0 ? x : (k == 1 ? y : z); }

}  // namespace krt
