// krt_transport.hip -- gfx950 kernels of the Monte Carlo line-transfer pass.
//
// One photon packet per lane in a persistent wavefront pool (Sec. 2.3.2 runs
// packets from a global work queue; here each wave refills its retired lanes
// from one wave-aggregated atomic, so lanes stay busy while packets of very
// different lengths finish).  Per loop iteration a lane does one flight
// segment (to its next interaction or to the next cell face) and, on an
// interaction, one resonant scattering.  Fields are SoA binary32 read once per
// cell entry; the per-line Voigt and atom-velocity tables live in LDS.
// Tallies are int64 fixed point: per-lane register caches for the current
// cell, flushed with one atomic per (cell, channel) when the packet leaves.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "krt_internal.h"
#include "krt_kernels.h"
#include "krt_device.h"
#include "krt_mlp.h"

namespace krt {

// --------------------------------------------------------- tally helpers ---
// Integer tally atomics return nothing, so a wave never waits on them; sums
// past 2^62 are detected after the launch (saturation_check_kernel).
__device__ __forceinline__ void tally_add_i64(int64_t *p, int64_t v) {
    atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}

// Four direct-mapped (channel -> fixed-point sum) slots, slot = channel & 3; a
// slot is written back only when another channel takes it or the packet leaves
// the cell.
struct EmisCache {
    int ch[4];
    int64_t acc[4];
};

__device__ __forceinline__ void emis_reset(EmisCache &E) {
#pragma unroll
    for (int s = 0; s < 4; ++s) { E.ch[s] = -1; E.acc[s] = 0; }
}

__device__ __forceinline__ void emis_flush(EmisCache &E, int64_t *base) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (E.ch[s] >= 0) tally_add_i64(base + E.ch[s], E.acc[s]);
        E.ch[s] = -1;
        E.acc[s] = 0;
    }
}

__device__ __forceinline__ void emis_add(EmisCache &E, int ch, int64_t v, int64_t *base) {
    const int slot = ch & 3;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (s == slot) {
            if (E.ch[s] != ch) {
                if (E.ch[s] >= 0) tally_add_i64(base + E.ch[s], E.acc[s]);
                E.ch[s] = ch;
                E.acc[s] = 0;
            }
            E.acc[s] += v;
        }
    }
}

// wave-wide sum of a 64-bit value, then one atomic from the first active lane
__device__ __forceinline__ void wave_add_counter(int64_t *dst, int64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (__lane_id() == 0 && v != 0) atomicAdd(reinterpret_cast<unsigned long long *>(dst), (unsigned long long)v);
}

// ------------------------------------------------------ learned escape ---
// Lane index of the k-th set bit (k counted from 0) of m; k < popcount(m).
__device__ __forceinline__ int nth_set_lane(uint64_t m, int k) {
    int pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const uint64_t low = (w == 64) ? m : (m & ((1ull << w) - 1ull));
        const int c = __popcll(low);
        if (k >= c) { k -= c; m >>= w; pos += w; }
        else m = low;
    }
    return pos;
}

// Batched evaluation of the escape network for the lanes of the wave set in
// `ask` (wave-uniform control flow: every lane executes the MFMA).  The asking
// lanes are packed in rank order into blocks of 16 samples, so a call costs
// ceil(popcount(ask) / 16) block evaluations.  pk[] holds this lane's inputs
// as bf16 pairs; an asking lane receives the normalised outputs k set in the
// wave-uniform `want` (a subset of kMlpFetch) in out[k] (the others keep their
// values).
constexpr uint32_t kMlpFetch = 0x003F1FFFu;  // outputs 0-12 and 16-21: all the transport reads
__device__ __forceinline__ void mlp_eval_wave(const unsigned char *img, const float *bias, const uint32_t pk[kMlpPackDw],
                                              int lane, uint64_t ask, uint32_t want, float out[kMlpOut]) {
    const int nask = __popcll(ask);
    const int nblk = (nask + 15) >> 4;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int rank = __popcll(ask & lt);
    const bool mine = (ask >> lane) & 1ull;
    const int g = lane >> 4;
#pragma unroll 1
    for (int b = 0; b < nblk; ++b) {
        // block position p = lane & 15 holds the asker of rank 16 b + p (if any);
        // lane group g takes that asker's input dwords 4g .. 4g + 3
        const int r = 16 * b + (lane & 15);
        const int src = (r < nask) ? nth_set_lane(ask, r) : lane;
        uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int d = 0; d < kMlpPackDw; ++d) {
            const uint32_t v = (uint32_t)__shfl((int)pk[d], src, 64);
            if ((d >> 2) == g) w[d & 3] = v;
        }
        const bool use = r < nask;
        const v4i16 lo = {(short)(use ? w[0] & 0xFFFFu : 0u), (short)(use ? w[0] >> 16 : 0u),
                          (short)(use ? w[1] & 0xFFFFu : 0u), (short)(use ? w[1] >> 16 : 0u)};
        const v4i16 hi = {(short)(use ? w[2] & 0xFFFFu : 0u), (short)(use ? w[2] >> 16 : 0u),
                          (short)(use ? w[3] & 0xFFFFu : 0u), (short)(use ? w[3] >> 16 : 0u)};
        v4f32 oa, ob;
        mlp_forward_block(img, bias, cat8(lo, hi), lane, NoEpi{}, oa, ob);
        // output k of block position p sits in lane 16 ((k % 16) / 4) + p,
        // component k % 4, of tile k / 16
        const bool take = mine && (rank >> 4) == b;
#pragma unroll
        for (int k = 0; k < kMlpOut; ++k) {
            if (!((kMlpFetch >> k) & 1u) || !((want >> k) & 1u)) continue;  // wave-uniform
            const v4f32 o = (k < 16) ? oa : ob;
            const float comp = (k % 4 == 0) ? o.x : (k % 4 == 1) ? o.y : (k % 4 == 2) ? o.z : o.w;
            const float v = __shfl(comp, 16 * ((k % 16) / 4) + (rank & 15), 64);
            if (take) out[k] = v;
        }
    }
}

// ------------------------------------------------------ network call ---
// The pieces of one learned whole-cell escape, shared by the transport kernel
// (calls batched inside it) and escape_call_kernel (parked calls), so both
// apply a call with the same arithmetic.

// Whether a scattering at the cell-frame position (fx, fy, fz) in [0, 1]^3 of a
// cell of line-centre opacity k0c, at gas-frame frequency xc, qualifies for a
// call: a cubic cell with tau_c = k0c half_dx in range, the point at least
// esc_depth_min below its nearest face, |xc| <= esc_x_max.  Returns the reduced
// frame and log10 tau_c, log10 depth.
__device__ __forceinline__ void call_frame(const RunParams &P, float k0c, float fx, float fy, float fz,
                                           CellFrame &CF, float &tc, float &dep) {
    tc = k0c * P.esc_half_dx;  // line-centre depth, centre to face
    cell_reduce(2.0f * fx - 1.0f, 2.0f * fy - 1.0f, 2.0f * fz - 1.0f, CF);
    dep = tc * (1.0f - CF.q[2]);
}
__device__ __forceinline__ bool call_eligible(const RunParams &P, float k0c, float fx, float fy, float fz, float xc,
                                              CellFrame &CF, float &ltc, float &ldep) {
    if (!P.esc_cubic) return false;
    float tc, dep;
    call_frame(P, k0c, fx, fy, fz, CF, tc, dep);
    if (tc >= P.esc_tc_min && tc <= P.esc_tc_max && dep >= P.esc_depth_min && fabsf(xc) <= P.esc_x_max) {
        ltc = __log10f(tc);
        ldep = __log10f(dep);
        return true;
    }
    return false;
}

// call_eligible's test without the frame: the transport kernel tests every
// scattering and reduces the frame only inside a call batch (same decisions:
// the largest |offset| is the last of the sorted three)
__device__ __forceinline__ bool call_ok(const RunParams &P, float k0c, float fx, float fy, float fz, float xc) {
    if (!P.esc_cubic) return false;
    const float tc = k0c * P.esc_half_dx;
    const float qm = fmaxf(fabsf(2.0f * fx - 1.0f), fmaxf(fabsf(2.0f * fy - 1.0f), fabsf(2.0f * fz - 1.0f)));
    const float dep = tc * (1.0f - qm);
    return tc >= P.esc_tc_min && tc <= P.esc_tc_max && dep >= P.esc_depth_min && fabsf(xc) <= P.esc_x_max;
}

// The two evaluations of a call for the lanes in `ask` (wave-uniform): the
// marginal one (exit face from the softmax at level u01(C.z), side of x_out
// from the learned P(x_out >= 0) at u01(C.w), |x_out| from the exit face's
// quantile at u_a = u01(C.x)), then the one conditional on the sampled face and
// x_out (offsets, cosine, alpha at the levels of D).  cnd: the raw condition
// (log10 tau_c, log10 a, |x_in|, q0, q1, q2, log10 depth, incoming direction in
// the reduced frame).  xo carries x_in's sign convention (reduced frame).
__device__ __forceinline__ void call_network(const unsigned char *mimg, const float *mbias, const float *mnorm,
                                             int lane, uint64_t ask, const float cnd[10], uint4 C, uint4 D,
                                             int &face, float &xo, float mo[kMlpOut]) {
    float in[kMlpIn];
    uint32_t pk[kMlpPackDw];
#pragma unroll
    for (int k = 0; k < kMlpOut; ++k) mo[k] = 0.0f;
    face = 5;
    xo = 0.0f;
#pragma unroll 1
    for (int e = 0; e < 2; ++e) {
        if (e == 0) mlp_inputs(cnd, u01(C.x), u01(C.y), u01(D.z), u01(D.w), false, 0.0f, 0, in);
        else mlp_inputs(cnd, u01(D.x), u01(D.y), u01(D.z), u01(D.w), true, xo, face, in);
        pack_inputs(in, pk);
        mlp_eval_wave(mimg, mbias, pk, lane, ask, e == 0 ? 0x003F01FFu : 0x00001E00u, mo);
        if (e == 0) {
            float mx = mo[0];
#pragma unroll
            for (int f = 1; f < 6; ++f) mx = fmaxf(mx, mo[f]);
            float ef[6], se = 0.0f;
#pragma unroll
            for (int f = 0; f < 6; ++f) { ef[f] = __expf(mo[f] - mx); se += ef[f]; }
            const float uf = u01(C.z) * se;
            float c2 = 0.0f;
            bool found = false;
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                c2 += ef[f];
                if (!found && uf < c2) { face = f; found = true; }
            }
            const bool pos = u01(C.w) < sigmoid_f(mo[kOutSide]);
            float ma = mo[kOutXAbs], mm = mnorm[kOutXAbs], ms = mnorm[kMlpOut + kOutXAbs];
#pragma unroll
            for (int f = 1; f < 6; ++f)
                if (face == f) {
                    ma = mo[kOutXAbs + f];
                    mm = mnorm[kOutXAbs + f];
                    ms = mnorm[kMlpOut + kOutXAbs + f];
                }
            const float mag = fmaxf(fmaf(ma, ms, mm), 0.0f);
            xo = pos ? mag : -mag;
        }
    }
}

// erf by the rational approximation of Abramowitz & Stegun (Handbook of
// Mathematical Functions, 7.1.26; absolute error at most 1.5e-7): one
// reciprocal and one exp instead of the library's longer evaluation.  It
// integrates the skipped scatterings' Gaussian over the channels, whose
// weights carry about 1e-7 of their own rounding.
__device__ __forceinline__ float erf_fast(float x) {
    const float ax = fabsf(x);
    const float t = f_rcp(fmaf(0.3275911f, ax, 1.0f));
    const float p = fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f),
                         0.254829592f);
    return copysignf(1.0f - t * p * f_exp(-ax * ax), x);
}

// The sampled exit applied to the packet: the exit point on the face (cell
// frame, fx, fy, fz in [0, 1]), the exit direction, the lab frequency
// x = sign(xc) xo + n.v, and the expected number of skipped scatterings
// E[N_s] (calibrated), whose emissivity -- thermalised core, camera frequency
// ~ N(n_cam.v, (<x^2> + 1)/3), integrated exactly over the whole channels that
// meet the central +-3 sd and renormalised to their share of it (the tails
// beyond hold 0.27%) -- goes to dep(channel, fixed-point weight); mass outside
// the channel grid is added to n_drop.  alpha takes its sign from the lowest
// bit of C.z.
template <class Dep>
__device__ __forceinline__ void call_apply(const RunParams &P, const float *mnorm, const float *cedges,
                                           const CellFrame &CF, const float mo[kMlpOut], int face, float xo,
                                           uint32_t cz, float ltc, float ldep, float xc, float vxc, float vyc,
                                           float vzc, float &fx, float &fy, float &fz, float &nx, float &ny,
                                           float &nz, float &x, int64_t &n_skip, int64_t &n_drop, Dep dep) {
    const float lns = mo[kOutLogN] * mnorm[kMlpOut + kOutLogN] + mnorm[kOutLogN] +
                      mnorm[kNormCal + cal_bin(ltc, ldep, fabsf(xc))];
    const float lx2 = mo[kOutLogX2] * mnorm[kMlpOut + kOutLogX2] + mnorm[kOutLogX2];
    // offsets learned as asinh, the cosine as mu^2
    auto sinh_f = [](float v) { const float ev = f_exp(v); return 0.5f * (ev - f_rcp(ev)); };
    const float ys = sinh_f(mo[kOutYS] * mnorm[kMlpOut + kOutYS] + mnorm[kOutYS]);
    const float yt = sinh_f(mo[kOutYT] * mnorm[kMlpOut + kOutYT] + mnorm[kOutYT]);
    const float mu = f_sqrt(fminf(fmaxf(mo[kOutMu2] * mnorm[kMlpOut + kOutMu2] + mnorm[kOutMu2], 1e-6f), 1.0f));
    const float al = fminf(fmaxf(mo[kOutAlpha] * mnorm[kMlpOut + kOutAlpha] + mnorm[kOutAlpha], 0.0f), 3.14159265f);
    // exit point and direction in the reduced frame: face axis k, outward side
    const int k = face >> 1;
    const float side = (face & 1) ? 1.0f : -1.0f;
    const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
    const float qk = pick3(CF.q[0], CF.q[1], CF.q[2], k);
    const float qa = pick3(CF.q[0], CF.q[1], CF.q[2], k1);
    const float qb = pick3(CF.q[0], CF.q[1], CF.q[2], k2);
    const float dpl = 1.0f - side * qk;
    const float es = fminf(fmaxf(qa + dpl * ys, -1.0f), 1.0f);
    const float et = fminf(fmaxf(qb + dpl * yt, -1.0f), 1.0f);
    // tangential direction at angle +-alpha from the offset (es - qa, et - qb)
    const float ds = es - qa, dt = et - qb;
    const float rr = f_sqrt(ds * ds + dt * dt);
    const float ir = (rr > 0.0f) ? f_rcp(rr) : 0.0f;
    const float c0 = (rr > 0.0f) ? ds * ir : 1.0f, s0 = dt * ir;
    const float arev = al * 0.159154943f * ((cz & 1u) ? -1.0f : 1.0f);
    const float ca = cos_rev(arev), sa = sin_rev(arev);
    const float sm = f_sqrt(fmaxf(0.0f, 1.0f - mu * mu));
    const float d1 = sm * (c0 * ca - s0 * sa), d2 = sm * (s0 * ca + c0 * sa);
    // back to the cell frame: reduced axis r is cell axis perm[r] with sign sg
    float pc[3] = {0.0f, 0.0f, 0.0f}, nc[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float R_ = (r == k) ? side : ((r == k1) ? es : et);
        const float V_ = (r == k) ? side * mu : ((r == k1) ? d1 : d2);
        const int axc = CF.perm[r];
        const float sgc = pick3(CF.sg[0], CF.sg[1], CF.sg[2], axc);
#pragma unroll
        for (int a3 = 0; a3 < 3; ++a3)
            if (a3 == axc) { pc[a3] = sgc * R_; nc[a3] = sgc * V_; }
    }
    fx = fminf(fmaxf(0.5f * (pc[0] + 1.0f), 0.0f), 1.0f);
    fy = fminf(fmaxf(0.5f * (pc[1] + 1.0f), 0.0f), 1.0f);
    fz = fminf(fmaxf(0.5f * (pc[2] + 1.0f), 0.0f), 1.0f);
    nx = nc[0]; ny = nc[1]; nz = nc[2];
    const float Ns = fmaxf(f_exp(lns), 1.0f);  // E[N_s | condition]
    if (P.emis_raw) {
        const float sd = f_sqrt((f_exp(lx2) + 1.0f) * (1.0f / 3.0f));
        const float vc = P.n_cam[0] * vxc + P.n_cam[1] * vyc + P.n_cam[2] * vzc;
        const float isd = kInvSqrt2F * f_rcp(sd);
        auto cdf = [&](float e) { return 0.5f * (1.0f + erf_fast((e - vc) * isd)); };
        const float wlo = vc - 3.0f * sd, whi = vc + 3.0f * sd;
        const int kb0u = bin_index(wlo, cedges, P.emis_nch, P.ch_inv_w);
        const int kb1u = bin_index(whi, cedges, P.emis_nch, P.ch_inv_w);
        const int kb0 = max(kb0u, 1), kb1 = min(kb1u, P.emis_nch);
        float cdf_lo = cdf(cedges[kb0 - 1]);
        // the Gaussian's mass over the channels met (the window's own ends where
        // it leaves the grid): the deposits are scaled by its inverse
        const float c_first = (kb0u >= 1) ? cdf_lo : cdf(wlo);
        const float c_last = cdf((kb1u >= 0 && kb1u <= P.emis_nch) ? cedges[kb1] : whi);
        const float inv_cov = f_rcp(fmaxf(c_last - c_first, 0.5f));
        const float W = Ns * P.frac_scale * inv_cov;
        float inside = 0.0f;
        for (int kb = kb0; kb <= kb1; ++kb) {
            const float cdf_hi = 0.5f * (1.0f + erf_fast((cedges[kb] - vc) * isd));
            const float fr = cdf_hi - cdf_lo;
            cdf_lo = cdf_hi;
            inside += fr;
            const int64_t wq = (int64_t)__float2ll_rn(W * fr);
            if (wq != 0) dep(kb - 1, wq);
        }
        n_drop += (int64_t)__float2ll_rn(Ns * fmaxf(0.0f, 1.0f - inside * inv_cov));
    }
    const float sx = (xc < 0.0f) ? -1.0f : 1.0f;
    x = sx * xo + nx * vxc + ny * vyc + nz * vzc;
    n_skip += (int64_t)__float2ll_rn(Ns);
}

// raw condition of a call: (log10 tau_c, log10 a, |x_in|, q0, q1, q2, log10
// depth, incoming direction in the reduced frame)
__device__ __forceinline__ void call_condition(const RunParams &P, const CellFrame &CF, float ltc, float ldep,
                                               float xc, float nx, float ny, float nz, float cnd[10]) {
    cnd[0] = ltc;
    cnd[1] = P.esc_log10a;
    cnd[2] = fabsf(xc);
    cnd[3] = CF.q[0]; cnd[4] = CF.q[1]; cnd[5] = CF.q[2];
    cnd[6] = ldep;
#pragma unroll
    for (int r = 0; r < 3; ++r)
        cnd[7 + r] = pick3(CF.sg[0], CF.sg[1], CF.sg[2], CF.perm[r]) * pick3(nx, ny, nz, CF.perm[r]);
}

// ------------------------------------------------ continuous temperature ---
// A cell of Doppler width r b_ref: frequency scale sc = 1 / r (and back, isc),
// its damping ac = a / r, the Voigt blocks around ac with the weight of the
// upper one (linear in ln a), and the nearest sampler node (block offset, its
// damping and sampler threshold).
struct ContCell {
    float sc, isc, ac, tv, sa, sthd;
    int voff, toff;
};
__device__ __forceinline__ ContCell cont_cell(const RunParams &P, float a, float r) {
    ContCell c;
    c.isc = r;
    c.sc = 1.0f / r;
    c.ac = a * c.sc;
    const float s = logf(c.ac) - P.cv_lna0;
    const float uv = fminf(fmaxf(s * P.cv_inv_step, 0.0f), (float)(P.cv_n - 1));
    const int kv = min((int)uv, max(P.cv_n - 2, 0));
    c.tv = uv - (float)kv;
    c.voff = kv * kVoigtFloats;
    const int ks = min((int)(fmaxf(s * P.cs_inv_step, 0.0f) + 0.5f), P.cs_n - 1);
    c.toff = ks * kTabFloats;
    const float2 sp = P.cs_par[ks];
    c.sa = sp.x;
    c.sthd = sp.y;
    return c;
}
// H(ac, |x|) between the two Voigt blocks
__device__ __forceinline__ float cont_voigt(const RunParams &P, int voff, float tv, float xa) {
    const float h0 = voigt_lds(P.cv_tab + voff, xa);
    return fmaf(tv, voigt_lds(P.cv_tab + voff + kVoigtFloats, xa) - h0, h0);
}

// --------------------------------------------------------------- kernel ---
// Draws of the second random block of an event: the two u_perp components
// (Box-Muller, N(0, 1/2) each), the cosine g of the scattering angle
// (isotropic or dipole) with sqrt(1 - g^2), and cos, sin of the azimuth psi.
struct SDraws {
    float up1, up2, g, sg, cp, sp;
};

// A prepared scattering: outgoing direction and gas-frame frequency, the
// emissivity channel (1-based, out of range = dropped) and its contribution.
struct ScatPrep {
    float ox, oy, oz, xo;
    int kb;
    int64_t wq;
};

__device__ __forceinline__ void scatter_draws(uint4 B, bool dipole, SDraws &d) {
    const float rr = f_sqrt(-f_log(u01(B.x)));
    const float th = u01(B.y);
    d.up1 = rr * cos_rev(th);
    d.up2 = rr * sin_rev(th);
    d.g = dipole ? dipole_g(u01(B.z)) : 2.0f * u01(B.z) - 1.0f;
    d.sg = f_sqrt(fmaxf(0.0f, 1.0f - d.g * d.g));
    const float psi = u01(B.w);
    d.cp = cos_rev(psi);
    d.sp = sin_rev(psi);
}

// kProf: 0 tables in LDS (production); 1 the same tables read from global
// memory (the workgroup still stages them, so occupancy is unchanged and only
// the memory space of the lookups differs); 2 analytic opacity profile in the
// flights, tables for the redistribution; 3 per-cell temperature classes: in a
// cell of Doppler width b the gas-frame frequency is (x - n.v) b_ref / b, the
// damping a b_ref / b, and the class's own tables (global memory) serve the
// opacity and the redistribution; frequencies return to reference units on
// leaving the cell's frame.
template <int kMode, int kMaxThreads, int kProf = 0>
__global__ void __launch_bounds__(kMaxThreads) mc_transport_kernel(RunParams P) {
    constexpr bool kEsc = kMode == kModeFused, kPark = kMode == kModePark;
    constexpr bool kTemp = kProf == 3 || kProf == 4;  // per-cell temperature: classes or continuum
    extern __shared__ float4 lds4[];
    const float *T = (kProf == 1) ? P.tab : reinterpret_cast<const float *>(lds4);
    // bin edges after the tables: spectrum then channels; the network variant
    // reads the spectrum edges (once per escaped packet) from global memory, so
    // that its LDS holds the tables, the channel edges and the network image
    constexpr int kLdsSpec = kEsc ? 0 : (kMaxSpecBins + 1);
    constexpr int kLdsMlp = kTabFloats + kChanEdgeFloats;  // floats before the network image
    float *ledges = reinterpret_cast<float *>(lds4) + kTabFloats;
    const float *sedges = kEsc ? P.spec_edges : ledges;  // spectrum edges
    float *cedges = ledges + kLdsSpec;                    // channel edges
    {
        const float4 *src = reinterpret_cast<const float4 *>(P.tab);
        for (int i = threadIdx.x; i < kTabFloats / 4; i += blockDim.x) lds4[i] = src[i];
        if (!kEsc)
            for (int i = threadIdx.x; i <= P.spec_nb; i += blockDim.x) ledges[i] = P.spec_edges[i];
        for (int i = threadIdx.x; i <= P.emis_nch; i += blockDim.x) cedges[i] = P.ch_edges[i];
        if (kEsc) {
            const float4 *ms = reinterpret_cast<const float4 *>(P.mlp_img);
            float4 *md = lds4 + kLdsMlp / 4;
            for (int i = threadIdx.x; i < kMlpFwdBytes / 16; i += blockDim.x) md[i] = ms[i];
        }
    }
    __syncthreads();
    const unsigned char *mimg = reinterpret_cast<const unsigned char *>(lds4 + kLdsMlp / 4);
    const float *mbias = reinterpret_cast<const float *>(mimg + kTilesFwd * kTileBytes);
    const float *mnorm = mbias + kBiasFloats;

    const int lane = __lane_id();
    const uint64_t lanemask_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const float a = P.a, thd = P.thd;

    // lane state
    float sc = 1.0f, isc = 1.0f, ac = a, thdc = thd;  // cell temperature (kProf 3, 4)
    float sac = a, tv = 0.0f;  // continuum (kProf 4): the sampler node's damping, upper Voigt weight
    int toff = 0, voff = 0;
    bool have = false, done = false;
    uint64_t pid = 0;
    int ci = 0, cj = 0, ck = 0, cell = 0;
    float fx = 0.f, fy = 0.f, fz = 0.f;
    float nx = 0.f, ny = 0.f, nz = 1.f;
    float x = 0.f, tau = 0.f;
    uint32_t ev = 0, wa1 = 0, wa2 = 0, wa3 = 0;
    float k0c = 0.f, vxc = 0.f, vyc = 0.f, vzc = 0.f, epsc = 0.f, kabsc = 0.f;
    uint32_t nscat_pkt = 0, ncross_pkt = 0;
    uint32_t seg = 0;  // plain scatterings of the packet in this launch (park mode)
    bool pend = false;   // fused mode: a qualifying scattering waits for its wave's next call batch
    uint32_t pwait = 0;  // ... for this many loop iterations so far
    int outcome = 0;  // 1 escaped, 2 destroyed, 3 stuck
    int64_t jacc = 0;
    EmisCache E;
    emis_reset(E);
    // per-lane counters
    int64_t c_emit = 0, c_esc = 0, c_des = 0, c_scat = 0, c_cross = 0, c_stuck = 0, c_drop = 0;
    int64_t c_mlp = 0, c_skip = 0;
    uint32_t *status = P.status;
    const float jscale = P.jbar_scale * kInvSqrtPiF;

    // entering a cell with temperature classes or a continuum of widths: its
    // frequency scale, damping, sampler threshold and table set
    auto enter_cell = [&]() {
        if constexpr (kProf == 3) {
            const int k = P.tclass[cell];
            const float4 cp = P.cls_par[k];
            sc = cp.x; ac = cp.y; thdc = cp.z; isc = cp.w;
            sac = ac;
            toff = k * kTabFloats;
        }
        if constexpr (kProf == 4) {
            const ContCell cc = cont_cell(P, a, P.bratio[cell]);
            sc = cc.sc; isc = cc.isc; ac = cc.ac; tv = cc.tv;
            sac = cc.sa; thdc = cc.sthd;
            voff = cc.voff; toff = cc.toff;
        }
    };

    // one flight segment of a live lane: to the next interaction (scat = true,
    // or destruction) or across one cell face (escape / periodic wrap / next cell)
    auto flight = [&](float ue, bool &scat, float &xc) {
        xc = x - (nx * vxc + ny * vyc + nz * vzc);
        if constexpr (kTemp) xc *= sc;
        float H = 0.0f;
        if (k0c > 0.0f) {
            if constexpr (kProf == 2) H = voigt_analytic(a, P.voigt_u0, fabsf(xc));
            else if constexpr (kProf == 4) H = cont_voigt(P, voff, tv, fabsf(xc));
            else H = voigt_lds((kProf == 3) ? P.cls_tab + toff : T, fabsf(xc));
        }
        // line opacity plus the cell's grey absorption (exactly k0 H without one)
        float kap = fmaf(k0c, H, kabsc);
        float tx = (nx > 0.0f) ? (1.0f - fx) * P.dx[0] * f_rcp(nx) : ((nx < 0.0f) ? fx * P.dx[0] * f_rcp(-nx) : INFINITY);
        float ty = (ny > 0.0f) ? (1.0f - fy) * P.dx[1] * f_rcp(ny) : ((ny < 0.0f) ? fy * P.dx[1] * f_rcp(-ny) : INFINITY);
        float tz = (nz > 0.0f) ? (1.0f - fz) * P.dx[2] * f_rcp(nz) : ((nz < 0.0f) ? fz * P.dx[2] * f_rcp(-nz) : INFINITY);
        int ax = 0;
        float dmin = tx;
        if (ty < dmin) { dmin = ty; ax = 1; }
        if (tz < dmin) { dmin = tz; ax = 2; }
        dmin = fmaxf(dmin, 0.0f);

        if (kap > 0.0f && kap * dmin >= tau) {
            // interaction inside the cell
            float l = tau * f_rcp(kap);
            fx = fminf(fmaxf(fmaf(l * nx, P.inv_dx[0], fx), 0.0f), 1.0f);
            fy = fminf(fmaxf(fmaf(l * ny, P.inv_dx[1], fy), 0.0f), 1.0f);
            fz = fminf(fmaxf(fmaf(l * nz, P.inv_dx[2], fz), 0.0f), 1.0f);
            if (P.jbar_raw) jacc += (int64_t)__float2ll_rn(l * H * jscale);
            // an absorption with probability p_d = kabs / kap, else a line scattering
            // destroyed with probability eps: one uniform decides both
            const float pd = (kabsc > 0.0f) ? kabsc * f_rcp(kap) : 0.0f;
            if ((P.eps != nullptr || P.kabs != nullptr) && (ue < fmaf(1.0f - pd, epsc, pd))) {
                c_des += 1;
                outcome = 2;
                have = false;
            } else {
                scat = true;
            }
        } else {
            // cross the face of axis ax
            tau -= kap * dmin;
            if (P.jbar_raw) jacc += (int64_t)__float2ll_rn(dmin * H * jscale);
            float adv = dmin;
            if (ax != 0) fx = fminf(fmaxf(fmaf(adv * nx, P.inv_dx[0], fx), 0.0f), 1.0f);
            if (ax != 1) fy = fminf(fmaxf(fmaf(adv * ny, P.inv_dx[1], fy), 0.0f), 1.0f);
            if (ax != 2) fz = fminf(fmaxf(fmaf(adv * nz, P.inv_dx[2], fz), 0.0f), 1.0f);
            c_cross += 1;
            ncross_pkt += 1;
            // leaving the cell: flush its register tallies
            if (P.jbar_raw && jacc != 0) { tally_add_i64(P.jbar_raw + cell, jacc); jacc = 0; }
            if (P.emis_raw) emis_flush(E, P.emis_raw + (int64_t)cell * P.emis_nch);
            bool escaped = false;
            if (ax == 0) {
                int st = (nx > 0.0f) ? 1 : -1;
                ci += st; fx = (st > 0) ? 0.0f : 1.0f;
                if (ci < 0 || ci >= P.n[0]) { if (P.bc[0]) ci = (ci < 0) ? P.n[0] - 1 : 0; else escaped = true; }
            } else if (ax == 1) {
                int st = (ny > 0.0f) ? 1 : -1;
                cj += st; fy = (st > 0) ? 0.0f : 1.0f;
                if (cj < 0 || cj >= P.n[1]) { if (P.bc[1]) cj = (cj < 0) ? P.n[1] - 1 : 0; else escaped = true; }
            } else {
                int st = (nz > 0.0f) ? 1 : -1;
                ck += st; fz = (st > 0) ? 0.0f : 1.0f;
                if (ck < 0 || ck >= P.n[2]) { if (P.bc[2]) ck = (ck < 0) ? P.n[2] - 1 : 0; else escaped = true; }
            }
            if (escaped) {
                c_esc += 1;
                int b = bin_index(x, sedges, P.spec_nb, P.spec_inv_w);
                if (b < 0) atomicOr(status, (uint32_t)KRT_ST_NAN_BIT);
                else atomicAdd(reinterpret_cast<unsigned long long *>(P.spec_raw + b), 1ull);
                outcome = 1;
                have = false;
            } else if (ncross_pkt > kMaxCrossings) {
                c_stuck += 1;
                atomicOr(status, (uint32_t)KRT_ST_STUCK_BIT);
                outcome = 3;
                have = false;
            } else {
                cell = (ck * P.n[1] + cj) * P.n[0] + ci;
                k0c = P.k0[cell];
                if (P.vx) { vxc = P.vx[cell]; vyc = P.vy[cell]; vzc = P.vz[cell]; }
                epsc = P.eps ? P.eps[cell] : 0.0f;
                kabsc = P.kabs ? P.kabs[cell] : 0.0f;
                enter_cell();
            }
        }
    };

    // A resonant scattering of a live lane at gas-frame frequency xc with the
    // event's draws (sampler uniforms r1, r2; u_perp components; g, sin, cos psi)
    // depends only on xc, the direction and the draws, not on where the flight
    // ends: it is prepared before the flight resolves (so the sampler's LDS
    // lookups overlap the flight's) and committed if the flight ends in a
    // scattering.
    auto prepare = [&](float xc, float r1, float r2, const SDraws &b, ScatPrep &q) {
        const float up1 = b.up1, up2 = b.up2, g = b.g, sg = b.sg, cp = b.cp, sp = b.sp;
        float upar = kTemp ? upar_lds(((kProf == 4) ? P.cs_tab : P.cls_tab) + toff, xc, sac, thdc, r1, r2)
                           : upar_lds(T, xc, a, thd, r1, r2);
        // orthonormal basis about n (Duff et al. 2017)
        float sgn = copysignf(1.0f, nz);
        float A_ = -f_rcp(sgn + nz);
        float B_ = nx * ny * A_;
        float e1x = 1.0f + sgn * nx * nx * A_, e1y = sgn * B_, e1z = -sgn * nx;
        float e2x = B_, e2y = sgn + ny * ny * A_, e2z = -ny;
        float ox = g * nx + sg * (cp * e1x + sp * e2x);
        float oy = g * ny + sg * (cp * e1y + sp * e2y);
        float oz = g * nz + sg * (cp * e1z + sp * e2z);
        float rn = f_rsq(ox * ox + oy * oy + oz * oz);
        q.ox = ox * rn; q.oy = oy * rn; q.oz = oz * rn;
        // eq. riia-scatter
        q.xo = xc + upar * (g - 1.0f) + sg * (up1 * cp + up2 * sp);
        if constexpr (kTemp) q.xo *= isc;  // back to reference units
        q.kb = -1;
        q.wq = 0;
        if (P.emis_raw) {
            float gc = nx * P.n_cam[0] + ny * P.n_cam[1] + nz * P.n_cam[2];
            float upc = up1 * (e1x * P.n_cam[0] + e1y * P.n_cam[1] + e1z * P.n_cam[2]) +
                        up2 * (e2x * P.n_cam[0] + e2y * P.n_cam[1] + e2z * P.n_cam[2]);
            float xcam = xc + upar * (gc - 1.0f) + upc;
            if constexpr (kTemp) xcam *= isc;
            xcam += P.n_cam[0] * vxc + P.n_cam[1] * vyc + P.n_cam[2] * vzc;
            q.kb = bin_index(xcam, cedges, P.emis_nch, P.ch_inv_w);
            float wph = (P.phase == KRT_PHASE_DIPOLE_I) ? 0.75f * (1.0f + gc * gc) : 1.0f;
            // contributions below 2^32 (F <= 30) convert through 32 bits
            const float wf = wph * P.frac_scale;
            q.wq = P.emis_w32 ? (int64_t)__float2uint_rn(wf) : (int64_t)__float2ll_rn(wf);
        }
    };
    auto commit = [&](const ScatPrep &q) {
        if (P.emis_raw) {
            if (q.kb >= 1 && q.kb <= P.emis_nch)
                emis_add(E, q.kb - 1, q.wq, P.emis_raw + (int64_t)cell * P.emis_nch);
            else
                c_drop += 1;
        }
        nx = q.ox; ny = q.oy; nz = q.oz;
        x = q.xo + nx * vxc + ny * vyc + nz * vzc;
        nscat_pkt += 1;
        c_scat += 1;
    };

    // a retired packet: flush the tallies of its last cell, log it
    auto retire = [&]() {
        if (P.jbar_raw && jacc != 0) { tally_add_i64(P.jbar_raw + cell, jacc); jacc = 0; }
        if (P.emis_raw) emis_flush(E, P.emis_raw + (int64_t)cell * P.emis_nch);
        if (P.plog) {
            float *L = P.plog + 8 * (pid - P.packet_offset);
            L[0] = x; L[1] = (float)nscat_pkt; L[2] = (float)outcome;
            L[3] = nx; L[4] = ny; L[5] = nz;
            L[6] = (float)cell; L[7] = (float)ev;
        }
        outcome = 0;
    };

    // park mode: lanes with a qualifying scattering (kind 1), or past their
    // round's budget of plain scatterings (kind 0, after committing one), leave
    // as records (their cell's register tallies flushed first); one
    // wave-aggregated atomic takes the slots.  A parked lane is free for new
    // work, with no outcome.  The budget bounds a round by its slowest packet.
    auto park = [&](bool want, bool &scat, float xc, uint32_t kind) {
        const uint64_t pm = __ballot(want);
        if (pm == 0ull) return;
        const int leader = __ffsll((long long)pm) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(P.park_count, (unsigned long long)__popcll(pm));
        base = __shfl(base, leader, 64);
        if (want) {
            if (P.jbar_raw && jacc != 0) { tally_add_i64(P.jbar_raw + cell, jacc); jacc = 0; }
            if (P.emis_raw) emis_flush(E, P.emis_raw + (int64_t)cell * P.emis_nch);
            const uint64_t slot = base + (uint64_t)__popcll(pm & lanemask_lt);
            if (slot < P.park_cap) {
                uint4 *r = P.park_out + kParkQuads * slot;
                r[0] = make_uint4((uint32_t)pid, (uint32_t)(pid >> 32), ev, (uint32_t)cell);
                r[1] = make_uint4(__float_as_uint(fx), __float_as_uint(fy), __float_as_uint(fz), __float_as_uint(x));
                r[2] = make_uint4(__float_as_uint(nx), __float_as_uint(ny), __float_as_uint(nz), nscat_pkt);
                r[3] = make_uint4(ncross_pkt, __float_as_uint(xc), kind, 0u);
            } else {
                atomicOr(status, (uint32_t)KRT_ST_STUCK_BIT);  // the host sizes the list; never expected
                c_stuck += 1;
            }
            have = false;
            scat = false;
        }
    };

    bool tail = false;
    for (;;) {
        // ---- refill retired lanes from the global queue -------------------
        bool need = !have && !done;
        uint64_t need_mask = __ballot(need);
        if (need_mask) {
            int cnt = __popcll(need_mask);
            int leader = __ffsll((long long)need_mask) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(P.work_counter, (unsigned long long)cnt);
            base = __shfl(base, leader, 64);
            if (need) {
                uint64_t idx = base + (uint64_t)__popcll(need_mask & lanemask_lt);
                if (idx < P.n_res) {
                    // ---- a packet back from a network call: its next event ----
                    const uint4 *r = P.res_in + kParkQuads * idx;
                    const uint4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
                    pid = (uint64_t)r0.x | ((uint64_t)r0.y << 32);
                    ev = r0.z;
                    cell = (int)r0.w;
                    ci = cell % P.n[0];
                    cj = (cell / P.n[0]) % P.n[1];
                    ck = cell / (P.n[0] * P.n[1]);
                    fx = __uint_as_float(r1.x); fy = __uint_as_float(r1.y); fz = __uint_as_float(r1.z);
                    x = __uint_as_float(r1.w);
                    nx = __uint_as_float(r2.x); ny = __uint_as_float(r2.y); nz = __uint_as_float(r2.z);
                    nscat_pkt = r2.w;
                    ncross_pkt = r3.x;
                    k0c = P.k0[cell];
                    if (P.vx) { vxc = P.vx[cell]; vyc = P.vy[cell]; vzc = P.vz[cell]; }
                    else { vxc = vyc = vzc = 0.0f; }
                    epsc = P.eps ? P.eps[cell] : 0.0f;
                    kabsc = P.kabs ? P.kabs[cell] : 0.0f;
                    enter_cell();
                    jacc = 0;
                    seg = 0;
                    ev += 1;
                    if ((uint64_t)ev > P.max_events) {
                        c_stuck += 1;
                        atomicOr(status, (uint32_t)KRT_ST_STUCK_BIT);
                        outcome = 3;
                        have = false;
                    } else {
                        const uint4 A = philox(make_uint4(ev, r0.x, r0.y, 0u), P.key0, P.key1);
                        tau = -f_log(u01(A.x));
                        wa1 = A.y; wa2 = A.z; wa3 = A.w;
                        have = true;
                    }
                } else if (idx - P.n_res >= P.n_packets) {
                    done = true;
                } else {
                    // ---- emission (event 0) ----------------------------------
                    pid = P.packet_offset + P.new_lo + (idx - P.n_res);
                    const uint32_t plo = (uint32_t)pid, phi = (uint32_t)(pid >> 32);
                    uint4 e0 = philox(make_uint4(0u, plo, phi, 0u), P.key0, P.key1);
                    if (P.source == KRT_SRC_BEAM_I) {
                        nx = P.src_dir[0]; ny = P.src_dir[1]; nz = P.src_dir[2];
                    } else {
                        float mu = 2.0f * u01(e0.x) - 1.0f;
                        float st = f_sqrt(fmaxf(0.0f, 1.0f - mu * mu));
                        float ph = u01(e0.y);
                        nx = st * cos_rev(ph); ny = st * sin_rev(ph); nz = mu;
                    }
                    if (P.source == KRT_SRC_VOLUME_I) {
                        uint4 e1 = philox(make_uint4(0u, plo, phi, 1u), P.key0, P.key1);
                        int col = (int)__umulhi(e0.z, (uint32_t)P.ncell);
                        cell = (u01(e0.w) < P.alias_prob[col]) ? col : P.alias_idx[col];
                        ci = cell % P.n[0];
                        cj = (cell / P.n[0]) % P.n[1];
                        ck = cell / (P.n[0] * P.n[1]);
                        fx = u01(e1.x); fy = u01(e1.y); fz = u01(e1.z);
                    } else {
                        int c3[3]; float f3[3];
                        float nd[3] = {nx, ny, nz};
                        double u2[2] = {0.0, 0.0};
                        if (P.source == KRT_SRC_PLANE_I) {
                            uint4 e1 = philox(make_uint4(0u, plo, phi, 1u), P.key0, P.key1);
                            u2[0] = (double)u01(e1.x); u2[1] = (double)u01(e1.y);
                        }
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            double X = P.src_pos[d];
                            if (P.source == KRT_SRC_PLANE_I && d < 2) X = P.lo[d] + u2[d] * (P.hi[d] - P.lo[d]);
                            double f = (X - P.lo[d]) / P.dxd[d];
                            double fl = floor(f);
                            int c = (int)fl;
                            float fr = (float)(f - fl);
                            if (fl == f && nd[d] < 0.0f) { c -= 1; fr = 1.0f; }
                            if (c < 0) { c = 0; fr = 0.0f; }
                            if (c >= P.n[d]) { c = P.n[d] - 1; fr = 1.0f; }
                            c3[d] = c; f3[d] = fr;
                        }
                        ci = c3[0]; cj = c3[1]; ck = c3[2];
                        fx = f3[0]; fy = f3[1]; fz = f3[2];
                        cell = (ck * P.n[1] + cj) * P.n[0] + ci;
                    }
                    k0c = P.k0[cell];
                    if (P.vx) { vxc = P.vx[cell]; vyc = P.vy[cell]; vzc = P.vz[cell]; }
                    else { vxc = vyc = vzc = 0.0f; }
                    epsc = P.eps ? P.eps[cell] : 0.0f;
                kabsc = P.kabs ? P.kabs[cell] : 0.0f;
                    enter_cell();
                    float xg = P.src_x0;
                    if (P.src_profile != KRT_PROF_DELTA_I) {
                        uint4 e2 = philox(make_uint4(0u, plo, phi, 2u), P.key0, P.key1);
                        float rr = f_sqrt(-f_log(u01(e2.x)));
                        float th = u01(e2.y);
                        xg = rr * cos_rev(th);
                        if (P.src_profile == KRT_PROF_VOIGT_I) {
                            float c = u01(e2.z) - 0.5f;  // Cauchy(a): a tan(pi c)
                            xg += (kTemp ? ac : a) * sin_rev(0.5f * c) * f_rcp(cos_rev(0.5f * c));
                        }
                        if constexpr (kTemp) xg *= isc;  // the emitting cell's units -> reference
                    }
                    x = xg + nx * vxc + ny * vyc + nz * vzc;
                    ev = 1;
                    uint4 A = philox(make_uint4(1u, plo, phi, 0u), P.key0, P.key1);
                    tau = -f_log(u01(A.x));
                    wa1 = A.y; wa2 = A.z; wa3 = A.w;
                    nscat_pkt = 0;
                    ncross_pkt = 0;
                    seg = 0;
                    jacc = 0;
                    have = true;
                    c_emit += 1;
                }
            }
        }
        const uint64_t live_mask = __ballot(have);
        if (live_mask == 0ull) break;
        // pool exhausted and few live lanes: continue in tail mode
        if (!kEsc && P.tail_lanes > 0 && __ballot(done) != 0ull && __popcll(live_mask) <= P.tail_lanes) {
            tail = true;
            break;
        }

        // ---- one flight segment (divergent) --------------------------------
        bool scat = false;
        float xc = 0.0f;
        ScatPrep q;
        if (kEsc && pend) xc = x - (nx * vxc + ny * vyc + nz * vzc);  // held at its scattering
        if (have && !pend) {
            const float xg = (x - (nx * vxc + ny * vyc + nz * vzc)) * (kTemp ? sc : 1.0f);
            SDraws b;
            scatter_draws(philox(make_uint4(ev, (uint32_t)pid, (uint32_t)(pid >> 32), 1u), P.key0, P.key1),
                          P.phase == KRT_PHASE_DIPOLE_I, b);
            prepare(xg, u01(wa2), u01(wa3), b, q);
            flight(u01(wa1), scat, xc);
        }

        // ---- learned whole-cell escape ---------------------------------------
        // At a scattering inside a thick cubic cell, at least esc_depth_min below
        // its nearest face and in the line core, one network sample replaces the
        // walk until the photon leaves the cell: exit face, point, direction and
        // frequency, and the expected number of scatterings skipped.  Fused mode
        // evaluates the network here, batched over the asking lanes of the wave
        // (wave-uniform); park mode writes the packet to the park list and frees
        // the lane, and escape_call_kernel applies the call.
        bool mlp = false;
        if (kEsc || kPark) {
            CellFrame CF{};
            float ltc = 0.0f, ldep = 0.0f;
            if (kPark && scat) mlp = call_eligible(P, k0c, fx, fy, fz, xc, CF, ltc, ldep);
            if (kEsc && (scat || pend)) mlp = call_ok(P, k0c, fx, fy, fz, xc);
            if (kPark) {
                bool cont = false;
                if (!mlp && scat) {
                    commit(q);
                    cont = ++seg >= P.park_budget;
                }
                park(mlp || cont, scat, xc, mlp ? 1u : 0u);
            } else {
                // once the packet pool is exhausted (some lane of this wave is done) the
                // wave lives only as long as its slowest packet: fewer asking lanes suffice.
                // With waiting on (esc_wait > 0) a qualifying lane that finds too few
                // others holds its scattering (pend) instead of walking it, for at most
                // esc_wait iterations; the batch also goes when every live lane asks.
                // While the pool lasts and nothing forces the batch, it takes whole
                // 16-sample blocks only: the askers past them, in lane order, stay held.
                uint64_t wm = __ballot(mlp);
                const bool tailw = __ballot(done) != 0ull;
                const int need_lanes = tailw ? P.esc_tail_lanes : P.esc_min_lanes;
                const bool forced = wm == __ballot(have) || __ballot(pend && pwait >= P.esc_wait) != 0ull;
                const bool go = wm != 0ull && (__popcll(wm) >= need_lanes || forced);  // wave-uniform
                bool held = !go;
                if (go && !tailw && !forced && P.esc_wait > 0 && mlp && __popcll(wm) >= 16)
                    held = __popcll(wm & lanemask_lt) >= (__popcll(wm) & ~15);
                if (held) {
                    if (mlp && P.esc_wait > 0) {
                        pwait = pend ? pwait + 1 : 1;
                        pend = true;
                    }
                    mlp = false;
                }
                wm = __ballot(mlp);  // the lanes this batch serves
                // this event's plain scatterings first, so their prepared state is
                // not live across the network evaluation
                if (scat && !mlp && !pend) commit(q);
                if (go) {
                    {
                        float tc, dep;
                        call_frame(P, k0c, fx, fy, fz, CF, tc, dep);
                        ltc = __log10f(tc);
                        ldep = __log10f(dep);
                    }
                    const uint32_t plo = (uint32_t)pid, phi = (uint32_t)(pid >> 32);
                    const uint4 C = philox(make_uint4(ev, plo, phi, 2u), P.key0, P.key1);
                    const uint4 D = philox(make_uint4(ev, plo, phi, 3u), P.key0, P.key1);
                    float cnd[10];
                    call_condition(P, CF, ltc, ldep, xc, nx, ny, nz, cnd);
                    int face;
                    float xo, mo[kMlpOut];
                    call_network(mimg, mbias, mnorm, lane, wm, cnd, C, D, face, xo, mo);
                    if (mlp) {
                        int64_t *ebase = P.emis_raw ? P.emis_raw + (int64_t)cell * P.emis_nch : nullptr;
                        // the deposit spans consecutive channels, each once: direct atomics
                        call_apply(P, mnorm, cedges, CF, mo, face, xo, C.z, ltc, ldep, xc, vxc, vyc, vzc, fx, fy,
                                   fz, nx, ny, nz, x, c_skip, c_drop,
                                   [&](int ch, int64_t w) __attribute__((always_inline)) { tally_add_i64(ebase + ch, w); });
                        c_mlp += 1;
                    }
                }
                // an event is consumed by a walked scattering or a call; a held one waits
                const bool served = go && mlp;
                if (served) pend = false;
                scat = (scat && !pend) || served;
            }
        }

        // ---- resonant scattering (event ev), divergent -----------------------
        if (scat) {
            const uint32_t plo = (uint32_t)pid, phi = (uint32_t)(pid >> 32);
            if (!kEsc && !kPark) commit(q);  // the network modes committed above
            // next event
            ev += 1;
            if ((uint64_t)ev > P.max_events) {
                c_stuck += 1;
                atomicOr(status, (uint32_t)KRT_ST_STUCK_BIT);
                outcome = 3;
                have = false;
            } else {
                uint4 A = philox(make_uint4(ev, plo, phi, 0u), P.key0, P.key1);
                tau = -f_log(u01(A.x));
                wa1 = A.y; wa2 = A.z; wa3 = A.w;
            }
        }
        if (!have && outcome != 0) retire();
    }
    // ---- tail mode ------------------------------------------------------------
    // The packet pool is exhausted and at most tail_lanes lanes are live, so the
    // wave lasts as long as its slowest packet.  The idle lanes precompute the
    // random draws of the live packets' coming events: with k live lanes, lane j
    // holds the draws of event ev0 + j / k of the live lane of rank j % k, and a
    // live lane fetches its event's draws by a cross-lane read.  The draws are
    // the same words mapped by the same functions as in the loop above, so the
    // tallies do not depend on where a packet switches mode.
    if (!kEsc && tail) {
        const bool dipole = P.phase == KRT_PHASE_DIPOLE_I;
        uint64_t bank_live = 0ull;
        uint32_t ev0 = 0;
        bool fresh = false;  // set after a scattering: tau of the new event comes from the draws
        float pt = 0.f, pue = 0.f, pr1 = 0.f, pr2 = 0.f;
        SDraws pb;
        pb.up1 = pb.up2 = pb.g = pb.sg = pb.cp = pb.sp = 0.f;
        for (;;) {
            const uint64_t live = __ballot(have);
            if (live == 0ull) break;
            const int k = __popcll(live);
            const int rank = __popcll(live & lanemask_lt);
            const int nslot = (63 - rank) / k + 1;
            const bool out_of_draws = have && (int)(ev - ev0) >= nslot;
            if (live != bank_live || __ballot(out_of_draws) != 0ull) {
                if (have) ev0 = ev;
                const int r = lane % k, sl = lane / k;
                const int owner = nth_set_lane(live, r);
                const uint32_t olo = __shfl((uint32_t)pid, owner, 64);
                const uint32_t ohi = __shfl((uint32_t)(pid >> 32), owner, 64);
                const uint32_t e = __shfl(ev0, owner, 64) + (uint32_t)sl;
                const uint4 A = philox(make_uint4(e, olo, ohi, 0u), P.key0, P.key1);
                pt = -f_log(u01(A.x));
                pue = u01(A.y);
                pr1 = u01(A.z);
                pr2 = u01(A.w);
                scatter_draws(philox(make_uint4(e, olo, ohi, 1u), P.key0, P.key1), dipole, pb);
                bank_live = live;
            }
            const int src = have ? (int)(ev - ev0) * k + rank : lane;
            const float dt = __shfl(pt, src, 64), due = __shfl(pue, src, 64);
            const float dr1 = __shfl(pr1, src, 64), dr2 = __shfl(pr2, src, 64);
            SDraws db;
            db.up1 = __shfl(pb.up1, src, 64); db.up2 = __shfl(pb.up2, src, 64);
            db.g = __shfl(pb.g, src, 64); db.sg = __shfl(pb.sg, src, 64);
            db.cp = __shfl(pb.cp, src, 64); db.sp = __shfl(pb.sp, src, 64);
            if (have && fresh) { tau = dt; fresh = false; }
            bool scat = false;
            float xc = 0.0f;
            ScatPrep q;
            if (have) {
                prepare((x - (nx * vxc + ny * vyc + nz * vzc)) * (kTemp ? sc : 1.0f), dr1, dr2, db, q);
                flight(due, scat, xc);
            }
            bool called = false;
            if (kPark) {
                CellFrame CF{};
                float ltc = 0.0f, ldep = 0.0f;
                called = scat && call_eligible(P, k0c, fx, fy, fz, xc, CF, ltc, ldep);
                bool cont = false;
                if (scat && !called) {
                    commit(q);
                    cont = ++seg >= P.park_budget;
                }
                park(called || cont, scat, xc, called ? 1u : 0u);
            }
            if (scat) {
                if (!kPark) commit(q);
                ev += 1;
                if ((uint64_t)ev > P.max_events) {
                    c_stuck += 1;
                    atomicOr(status, (uint32_t)KRT_ST_STUCK_BIT);
                    outcome = 3;
                    have = false;
                } else {
                    fresh = true;
                }
            }
            if (!have && outcome != 0) retire();
        }
    }

    wave_add_counter(P.counters + KRT_C_EMITTED, c_emit);
    wave_add_counter(P.counters + KRT_C_ESCAPED, c_esc);
    wave_add_counter(P.counters + KRT_C_DESTROYED, c_des);
    wave_add_counter(P.counters + KRT_C_SCATTER, c_scat);
    wave_add_counter(P.counters + KRT_C_CROSS, c_cross);
    wave_add_counter(P.counters + KRT_C_STUCK, c_stuck);
    wave_add_counter(P.counters + KRT_C_EMIS_DROP, c_drop);
    if (kEsc) {
        wave_add_counter(P.counters + KRT_C_MLP_I, c_mlp);
        wave_add_counter(P.counters + KRT_C_SKIPPED_I, c_skip);
    }
}

// -------------------------------------------------------------- finalise ---
__global__ void finalize_kernel(const int64_t *raw, float *out, int64_t n, double scale) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) out[i] = (float)((double)raw[i] * scale);
}

// Sets the saturation bit if any integer tally left [0, 2^62].
__global__ void saturation_check_kernel(const int64_t *p, int64_t n, uint32_t *status) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (; i < n; i += stride) bad |= (p[i] < 0) || (p[i] > (int64_t(1) << 62));
    if (__ballot(bad) != 0ull && __lane_id() == 0) atomicOr(status, (uint32_t)KRT_ST_SATURATE_BIT);
}

__global__ void zero_i64_kernel(int64_t *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0;
}

// ----------------------------------------------------------- diagnostics ---
__global__ void debug_philox_kernel(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint4 c = make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]);
    uint4 r = philox(c, key[2 * i], key[2 * i + 1]);
    out[4 * i] = r.x; out[4 * i + 1] = r.y; out[4 * i + 2] = r.z; out[4 * i + 3] = r.w;
}

__global__ void debug_bins_kernel(const float *x, int64_t n, int nb, const float *edges, float inv_w,
                                  int32_t *out) {
    __shared__ float e[kMaxSpecBins + 1];
    for (int i = threadIdx.x; i <= nb; i += blockDim.x) e[i] = edges[i];
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = bin_index(x[i], e, nb, inv_w);
}

// H(a / r, |x|) for the widths r[i] as the continuum transport evaluates it
__global__ void debug_voigt_cont_kernel(RunParams P, float a, const float *r, const float *x, int64_t n, float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const ContCell cc = cont_cell(P, a, r[i]);
    out[i] = cont_voigt(P, cc.voff, cc.tv, fabsf(x[i]));
}

__global__ void debug_voigt_kernel(const float *tab, const float *x, int64_t n, float *out) {
    extern __shared__ float4 lds4[];
    float *T = reinterpret_cast<float *>(lds4);
    const float4 *src = reinterpret_cast<const float4 *>(tab);
    for (int i = threadIdx.x; i < kTabFloats / 4; i += blockDim.x) lds4[i] = src[i];
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = voigt_lds(T, fabsf(x[i]));
}

__global__ void debug_voigt_analytic_kernel(float a, float u0, const float *x, int64_t n, float *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = voigt_analytic(a, u0, fabsf(x[i]));
}

__global__ void debug_upar_kernel(const float *tab, float a, float thd, float x, uint32_t k0, uint32_t k1,
                                  uint64_t packet, uint32_t ev0, int64_t n, float *out) {
    extern __shared__ float4 lds4[];
    float *T = reinterpret_cast<float *>(lds4);
    const float4 *src = reinterpret_cast<const float4 *>(tab);
    for (int i = threadIdx.x; i < kTabFloats / 4; i += blockDim.x) lds4[i] = src[i];
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint4 A = philox(make_uint4(ev0 + (uint32_t)i, (uint32_t)packet, (uint32_t)(packet >> 32), 0u), k0, k1);
    out[i] = upar_lds(T, x, a, thd, u01(A.z), u01(A.w));
}

// ---------------------------------------------------------------- launch ---
hipError_t launch_transport(const RunParams &P, int mode, int grid, int block, hipStream_t s) {
    const bool fused = mode == kModeFused;
    // plain and park: tables and both edge sets; fused: tables, channel edges, image
    static_assert(sizeof(float) * (kTabFloats + kChanEdgeFloats) + kMlpFwdBytes <= 160 * 1024,
                  "the network variant's LDS fits one CU (160 KiB)");
    const size_t lds = fused ? sizeof(float) * (kTabFloats + kChanEdgeFloats) + (size_t)kMlpFwdBytes
                             : sizeof(float) * (kTabFloats + kEdgeFloats);
    // the fused variant is compiled for the block size: up to 512 lanes 256
    // VGPRs (no spills, 2 waves per SIMD; the default), up to 768 lanes 168
    // VGPRs (spills, 3 waves), above that 128 (4 waves, heavy spills).
    // Profile modes 1 and 2 exist for the plain walk only; park mode has the
    // plain walk's register budget (1024 lanes).
    const int variant = fused ? (block <= 512 ? 2 : (block <= 768 ? 5 : 1))
                              : (mode == kModePark ? 7
                                                   : (P.bratio ? 8 : (P.tclass ? 6 : (P.profile_mode == 1 ? 3
                                                                      : (P.profile_mode == 2 ? 4 : 0)))));
    static bool attr_set[9] = {false, false, false, false, false, false, false, false, false};
    const void *fns[9] = {reinterpret_cast<const void *>(mc_transport_kernel<kModePlain, 1024>),
                          reinterpret_cast<const void *>(mc_transport_kernel<kModeFused, 1024>),
                          reinterpret_cast<const void *>(mc_transport_kernel<kModeFused, 512>),
                          reinterpret_cast<const void *>(mc_transport_kernel<kModePlain, 1024, 1>),
                          reinterpret_cast<const void *>(mc_transport_kernel<kModePlain, 1024, 2>),
                          reinterpret_cast<const void *>(mc_transport_kernel<kModeFused, 768>),
                          reinterpret_cast<const void *>(mc_transport_kernel<kModePlain, 1024, 3>),
                          reinterpret_cast<const void *>(mc_transport_kernel<kModePark, 1024>),
                          reinterpret_cast<const void *>(mc_transport_kernel<kModePlain, 1024, 4>)};
    if (!attr_set[variant]) {
        hipError_t e = hipFuncSetAttribute(fns[variant], hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set[variant] = true;
    }
    switch (variant) {
        case 0: hipLaunchKernelGGL((mc_transport_kernel<kModePlain, 1024>), dim3(grid), dim3(block), lds, s, P); break;
        case 1: hipLaunchKernelGGL((mc_transport_kernel<kModeFused, 1024>), dim3(grid), dim3(block), lds, s, P); break;
        case 2: hipLaunchKernelGGL((mc_transport_kernel<kModeFused, 512>), dim3(grid), dim3(block), lds, s, P); break;
        case 3: hipLaunchKernelGGL((mc_transport_kernel<kModePlain, 1024, 1>), dim3(grid), dim3(block), lds, s, P); break;
        case 5: hipLaunchKernelGGL((mc_transport_kernel<kModeFused, 768>), dim3(grid), dim3(block), lds, s, P); break;
        case 6: hipLaunchKernelGGL((mc_transport_kernel<kModePlain, 1024, 3>), dim3(grid), dim3(block), lds, s, P); break;
        case 7: hipLaunchKernelGGL((mc_transport_kernel<kModePark, 1024>), dim3(grid), dim3(block), lds, s, P); break;
        case 8: hipLaunchKernelGGL((mc_transport_kernel<kModePlain, 1024, 4>), dim3(grid), dim3(block), lds, s, P); break;
        default: hipLaunchKernelGGL((mc_transport_kernel<kModePlain, 1024, 2>), dim3(grid), dim3(block), lds, s, P); break;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ call kernel ---
// The network calls of parked packets, in place.  Every lane takes one record
// (wave-strided over the list), so each evaluation runs on full 16-sample
// blocks and no transport state is live around it.  The condition, the two
// evaluations and the applied exit are the transport's own (call_eligible,
// call_condition, call_network, call_apply); the skipped scatterings'
// emissivity goes straight to the int64 tallies.
constexpr int kCallThreads = 512;
__global__ void __launch_bounds__(kCallThreads) escape_call_kernel(RunParams P, uint4 *rec, uint64_t n) {
    extern __shared__ float4 lds4[];
    float *cedges = reinterpret_cast<float *>(lds4);
    {
        for (int i = threadIdx.x; i <= P.emis_nch; i += blockDim.x) cedges[i] = P.ch_edges[i];
        const float4 *ms = reinterpret_cast<const float4 *>(P.mlp_img);
        float4 *md = lds4 + kChanEdgeFloats / 4;
        for (int i = threadIdx.x; i < kMlpFwdBytes / 16; i += blockDim.x) md[i] = ms[i];
    }
    __syncthreads();
    const unsigned char *mimg = reinterpret_cast<const unsigned char *>(lds4 + kChanEdgeFloats / 4);
    const float *mbias = reinterpret_cast<const float *>(mimg + kTilesFwd * kTileBytes);
    const float *mnorm = mbias + kBiasFloats;
    const int lane = __lane_id();
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    int64_t c_mlp = 0, c_skip = 0, c_drop = 0;
    for (uint64_t base = ((uint64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) * 64; base < n;
         base += waves * 64) {  // wave-uniform
        const uint64_t i = base + (uint64_t)lane;
        const bool live = i < n;
        uint4 r0 = make_uint4(0u, 0u, 0u, 0u), r1 = r0, r2 = r0, r3 = r0;
        if (live) {
            const uint4 *r = rec + kParkQuads * i;
            r0 = r[0]; r1 = r[1]; r2 = r[2]; r3 = r[3];
        }
        const int cell = (int)r0.w;
        float fx = __uint_as_float(r1.x), fy = __uint_as_float(r1.y), fz = __uint_as_float(r1.z);
        float x = __uint_as_float(r1.w);
        float nx = __uint_as_float(r2.x), ny = __uint_as_float(r2.y), nz = __uint_as_float(r2.z);
        float k0c = 0.0f, vxc = 0.0f, vyc = 0.0f, vzc = 0.0f;
        if (live) {
            k0c = P.k0[cell];
            if (P.vx) { vxc = P.vx[cell]; vyc = P.vy[cell]; vzc = P.vz[cell]; }
        }
        // every record qualified when it was parked (the gas-frame frequency the
        // transport tested is in the record): only the frame and depths are rebuilt
        const float xc = __uint_as_float(r3.y);
        CellFrame CF{};
        float tc = 1.0f, dep = 1.0f;
        if (live) call_frame(P, k0c, fx, fy, fz, CF, tc, dep);
        const float ltc = __log10f(tc), ldep = __log10f(dep);
        const bool ask = live && r3.z == 1u;  // kind 0: parked to continue, no call
        const uint64_t am = __ballot(ask);
        if (am == 0ull) continue;
        const uint4 C = philox(make_uint4(r0.z, r0.x, r0.y, 2u), P.key0, P.key1);
        const uint4 D = philox(make_uint4(r0.z, r0.x, r0.y, 3u), P.key0, P.key1);
        float cnd[10];
        call_condition(P, CF, ltc, ldep, xc, nx, ny, nz, cnd);
        int face;
        float xo, mo[kMlpOut];
        call_network(mimg, mbias, mnorm, lane, am, cnd, C, D, face, xo, mo);
        if (ask) {
            int64_t *ebase = P.emis_raw ? P.emis_raw + (int64_t)cell * P.emis_nch : nullptr;
            call_apply(P, mnorm, cedges, CF, mo, face, xo, C.z, ltc, ldep, xc, vxc, vyc, vzc, fx, fy, fz, nx, ny, nz,
                       x, c_skip, c_drop, [&](int ch, int64_t w) __attribute__((always_inline)) { tally_add_i64(ebase + ch, w); });
            c_mlp += 1;
            uint4 *r = rec + kParkQuads * i;
            r[1] = make_uint4(__float_as_uint(fx), __float_as_uint(fy), __float_as_uint(fz), __float_as_uint(x));
            r[2] = make_uint4(__float_as_uint(nx), __float_as_uint(ny), __float_as_uint(nz), r2.w);
        }
    }
    wave_add_counter(P.counters + KRT_C_MLP_I, c_mlp);
    wave_add_counter(P.counters + KRT_C_SKIPPED_I, c_skip);
    wave_add_counter(P.counters + KRT_C_EMIS_DROP, c_drop);
}

hipError_t launch_escape_call(const RunParams &P, uint4 *rec, uint64_t n, int grid, hipStream_t s) {
    static_assert(sizeof(float) * kChanEdgeFloats + kMlpFwdBytes <= 160 * 1024, "the call kernel's LDS fits one CU");
    const size_t lds = sizeof(float) * kChanEdgeFloats + (size_t)kMlpFwdBytes;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(escape_call_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(escape_call_kernel, dim3(grid), dim3(kCallThreads), lds, s, P, rec, n);
    return hipGetLastError();
}

hipError_t launch_finalize(const int64_t *raw, float *out, int64_t n, double scale, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int grid = (int)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(finalize_kernel, dim3(grid), dim3(256), 0, s, raw, out, n, scale);
    return hipGetLastError();
}

hipError_t launch_saturation_check(const int64_t *p, int64_t n, uint32_t *status, hipStream_t s) {
    if (n <= 0 || !p) return hipSuccess;
    int grid = (int)std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(saturation_check_kernel, dim3(grid), dim3(256), 0, s, p, n, status);
    return hipGetLastError();
}

hipError_t launch_debug_voigt_analytic(float a, float u0, const float *x, int64_t n, float *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(debug_voigt_analytic_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, u0, x, n,
                       out);
    return hipGetLastError();
}

hipError_t launch_zero_i64(int64_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int grid = (int)std::min<int64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(zero_i64_kernel, dim3(grid), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_debug_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n, hipStream_t s) {
    int grid = (int)((n + 255) / 256);
    hipLaunchKernelGGL(debug_philox_kernel, dim3(grid), dim3(256), 0, s, ctr, key, out, n);
    return hipGetLastError();
}

hipError_t launch_debug_bins(const float *x, int64_t n, int nb, const float *edges, float inv_w, int32_t *out,
                             hipStream_t s) {
    int grid = (int)((n + 255) / 256);
    hipLaunchKernelGGL(debug_bins_kernel, dim3(grid), dim3(256), 0, s, x, n, nb, edges, inv_w, out);
    return hipGetLastError();
}

hipError_t launch_debug_voigt_cont(const RunParams &P, float a, const float *r, const float *x, int64_t n, float *out,
                                   hipStream_t s) {
    hipLaunchKernelGGL(debug_voigt_cont_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, P, a, r, x, n, out);
    return hipGetLastError();
}

hipError_t launch_debug_voigt(const float *tab, const float *x, int64_t n, float *out, hipStream_t s) {
    size_t lds = sizeof(float) * kTabFloats;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(debug_voigt_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    int grid = (int)((n + 255) / 256);
    hipLaunchKernelGGL(debug_voigt_kernel, dim3(grid), dim3(256), lds, s, tab, x, n, out);
    return hipGetLastError();
}

hipError_t launch_debug_upar(const float *tab, float a, float thd, float x, uint32_t k0, uint32_t k1,
                             uint64_t packet, uint32_t ev0, int64_t n, float *out, hipStream_t s) {
    size_t lds = sizeof(float) * kTabFloats;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(debug_upar_kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    int grid = (int)((n + 255) / 256);
    hipLaunchKernelGGL(debug_upar_kernel, dim3(grid), dim3(256), lds, s, tab, a, thd, x, k0, k1, packet, ev0, n, out);
    return hipGetLastError();
}

}  // namespace krt
