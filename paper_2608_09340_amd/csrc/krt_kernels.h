// krt_kernels.h -- kernel parameter block and launch wrappers (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <cmath>
#include <algorithm>

namespace krt {

// counter slots / status bits, as in include/krt.h
enum {
    KRT_C_EMITTED_I = 0, KRT_C_ESCAPED_I, KRT_C_DESTROYED_I, KRT_C_SCATTER_I, KRT_C_CROSS_I,
    KRT_C_STUCK_I, KRT_C_MLP_I, KRT_C_STATUS_I, KRT_C_EMIS_DROP_I, KRT_C_SKIPPED_I,
};
#define KRT_C_EMITTED KRT_C_EMITTED_I
#define KRT_C_ESCAPED KRT_C_ESCAPED_I
#define KRT_C_DESTROYED KRT_C_DESTROYED_I
#define KRT_C_SCATTER KRT_C_SCATTER_I
#define KRT_C_CROSS KRT_C_CROSS_I
#define KRT_C_STUCK KRT_C_STUCK_I
#define KRT_C_EMIS_DROP KRT_C_EMIS_DROP_I
#define KRT_C_MLP KRT_C_MLP_I
enum { KRT_ST_NAN_BIT = 1, KRT_ST_STUCK_BIT = 2, KRT_ST_SATURATE_BIT = 4 };
enum { KRT_SRC_POINT_I = 0, KRT_SRC_PLANE_I = 1, KRT_SRC_VOLUME_I = 2, KRT_SRC_BEAM_I = 3 };
enum { KRT_PROF_DELTA_I = 0, KRT_PROF_VOIGT_I = 1, KRT_PROF_GAUSS_I = 2 };
enum { KRT_PHASE_ISO_I = 0, KRT_PHASE_DIPOLE_I = 1 };

// bin-edge tables staged in LDS after the line tables
constexpr int kMaxSpecBins = 1024, kMaxChannels = 256;
constexpr int kEdgeFloats = (kMaxSpecBins + 1) + (kMaxChannels + 1) + 2;  // padded to a multiple of 4
constexpr int kChanEdgeFloats = (kMaxChannels + 1) + 3;                 // channel edges alone, padded

// 1 / ln((300/8)^(1/15)): logarithmic row spacing of the sampler above |x| = 8
constexpr float kRowInvLog = 4.1386840f;

// imaging pass (krt_image.hip)
struct ImageParams {
    const float *tab;       // table set of the line (Voigt core and wing used)
    const float *k0;        // [ncell] line-centre opacity of the line
    const float *vel_axis;  // [ncell] velocity component along the camera axis, or null
    const float *emis;      // [ncell][nch]
    const float *srcf;      // [ncell][nch] or null
    const float *kabs;      // [ncell] grey absorption coefficient, or null
    float *out;             // [npix][nch]
    int64_t npix, stride;
    int n[3];
    int d, sgn, n0, nch;
    float sgnf, dl, ch_lo, ch_w;
};
hipError_t launch_image(const ImageParams &Q, hipStream_t s);

struct RunParams {
    // grid
    int n[3];
    int ncell;
    double lo[3], hi[3], dxd[3];
    float dx[3], inv_dx[3];
    int bc[3];
    const float *k0, *vx, *vy, *vz, *eps;
    const float *kabs;  // [ncell] grey absorption coefficient, or null
    const float *alias_prob;
    const int *alias_idx;
    // line
    const float *tab;
    float a, thd;
    int phase;
    // source
    int source, src_profile;
    float src_x0;
    double src_pos[3];
    float src_dir[3];
    // tallies (edges: binary32 bin edges computed on the host, staged in LDS)
    int spec_nb;
    float spec_inv_w;
    const float *spec_edges;  // [spec_nb + 1]
    int emis_nch;
    float ch_inv_w;
    const float *ch_edges;    // [emis_nch + 1]
    float n_cam[3];
    float frac_scale;  // 2^F, emissivity
    float jbar_scale;  // 2^Fj, mean intensity
    int64_t *spec_raw, *emis_raw, *jbar_raw, *counters;
    uint32_t *status;
    float *plog;
    // work: packets resumed after a network call (res_in[0, n_res)) come first,
    // then n_packets new ones with ids packet_offset + new_lo + [0, n_packets)
    uint64_t n_packets, packet_offset, max_events;
    uint32_t key0, key1;
    unsigned long long *work_counter;
    const uint4 *res_in;
    uint64_t n_res, new_lo;
    // parking (kernel mode kModePark): a packet whose scattering qualifies for a
    // network call leaves its lane as a record in park_out (slot from park_count,
    // at most park_cap); escape_call_kernel then applies the call to the record
    uint4 *park_out;
    unsigned long long *park_count;
    uint64_t park_cap;
    uint32_t park_budget;  // plain scatterings of a packet per round before it is parked to continue
    // learned whole-cell escape (mlp_img == nullptr: plain random walk only).
    // Calls happen only in cubic cells (esc_cubic) whose line-centre depth from
    // centre to face tau_c = k0 half_dx lies in [esc_tc_min, esc_tc_max], at
    // scattering points at least esc_depth_min (line-centre) below the nearest
    // face, for gas-frame |x| <= esc_x_max.
    const unsigned char *mlp_img;
    int esc_cubic;
    float esc_half_dx, esc_tc_min, esc_tc_max, esc_depth_min, esc_x_max, esc_log10a;
    int esc_min_lanes;
    int esc_tail_lanes;
    uint32_t esc_wait;  // fused: iterations a qualifying lane may hold its scattering for a batch (0 = never)
    int tail_lanes;
    int emis_w32;  // emissivity contributions fit 32 bits (fraction bits <= 30)
    // opacity profile of the flights: 0 LDS tables, 1 the same tables read from
    // global memory, 2 analytic blend (voigt_analytic, crossing point voigt_u0)
    int profile_mode;
    float voigt_u0;
    // per-cell temperature classes (null: every cell at the reference width):
    // class per cell, per class (b_ref / b, damping, sampler threshold,
    // b / b_ref), and the class table sets [class][kTabFloats] in global memory
    const uint8_t *tclass;
    const float4 *cls_par;
    const float *cls_tab;
    // continuous per-cell temperature (null: none): b / b_ref per cell; Voigt
    // blocks [cv_n + 1][kVoigtFloats] at damping exp(cv_lna0 + k / cv_inv_step)
    // (the last block repeats the one before it, so the upper neighbour of
    // any node exists), sampler blocks [cs_n][kTabFloats] at
    // exp(cv_lna0 + k / cs_inv_step) with (a, sampler threshold) per node
    const float *bratio;
    const float *cv_tab;
    const float *cs_tab;
    const float2 *cs_par;
    float cv_lna0, cv_inv_step, cs_inv_step;
    int cv_n, cs_n;
};

// transport kernel modes: plain walk, network calls batched inside the
// transport kernel, qualifying scatterings parked for escape_call_kernel
constexpr int kModePlain = 0, kModeFused = 1, kModePark = 2;
// A parked packet: 4 x uint4 (64 B).  w0 = (id lo, id hi, event of the call or
// of the last scattering, cell); w1 = (fx, fy, fz, x lab) as float bits;
// w2 = (nx, ny, nz, scatterings of the packet); w3 = (cell crossings of the
// packet, the gas-frame frequency the call was qualified at, 1 for a call or 0
// for a packet parked after its round's budget of plain scatterings, 0).  After the call
// the record holds the exit point (still in the cell, on the exit face), the
// exit direction and the lab exit frequency; the transport resumes it with the
// next event.
constexpr int kParkQuads = 4;
hipError_t launch_transport(const RunParams &P, int mode, int grid, int block, hipStream_t s);
// the network call of each of n parked records, in place (learned escape)
hipError_t launch_escape_call(const RunParams &P, uint4 *rec, uint64_t n, int grid, hipStream_t s);
hipError_t launch_finalize(const int64_t *raw, float *out, int64_t n, double scale, hipStream_t s);
hipError_t launch_zero_i64(int64_t *p, int64_t n, hipStream_t s);
hipError_t launch_saturation_check(const int64_t *p, int64_t n, uint32_t *status, hipStream_t s);
hipError_t launch_debug_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n,
                               hipStream_t s);
hipError_t launch_debug_bins(const float *x, int64_t n, int nb, const float *edges, float inv_w, int32_t *out,
                             hipStream_t s);
hipError_t launch_debug_voigt(const float *tab, const float *x, int64_t n, float *out, hipStream_t s);
hipError_t launch_debug_voigt_cont(const RunParams &P, float a, const float *r, const float *x, int64_t n, float *out,
                                   hipStream_t s);
hipError_t launch_debug_voigt_analytic(float a, float u0, const float *x, int64_t n, float *out, hipStream_t s);
hipError_t launch_debug_upar(const float *tab, float a, float thd, float x, uint32_t k0, uint32_t k1,
                             uint64_t packet, uint32_t ev0, int64_t n, float *out, hipStream_t s);
// whole-cell escape records (krt_escape.hip)
struct RecordParams {
    const float *tab;
    float a, thd;
    uint32_t k0, k1;
    uint64_t offset, n;
    float lt_lo, lt_hi, ld_lo;    // log10 tau_c range, lower end of log10 depth
    uint32_t max_scat;            // records past this many scatterings are invalid
    int fixed, iso_dir;           // fixed start (x_in, q, n_in) / isotropic n_in with it
    float x_in, q[3], n_in[3];
    unsigned long long *counter;  // record pool, zeroed before the launch
    float *out;                   // [n][kRec]
};
hipError_t launch_cell_record(const RecordParams &R, int grid, hipStream_t s);
hipError_t launch_mlp_init(float *p, uint32_t k0, uint32_t k1, hipStream_t s);
hipError_t launch_mlp_pack(const float *p, const float *norm, unsigned char *blob, unsigned char *img,
                           hipStream_t s);
hipError_t launch_mlp_act_init(uint16_t *act, int64_t cap, hipStream_t s);
hipError_t launch_mlp_grad(const unsigned char *blob, const float *rec, const int32_t *idx, const float *uq,
                           int batch, uint16_t *act, int64_t cap, float *part, float *loss, hipStream_t s);
hipError_t launch_mlp_gsum(const float *part, float *grad, hipStream_t s);
hipError_t launch_mlp_adam(float *p, float *m, float *v, const float *part, float lr, int step, hipStream_t s);
hipError_t launch_mlp_batch(int64_t n, uint32_t k0, uint32_t k1, uint32_t step, int batch, int32_t *idx,
                            float *uq, hipStream_t s);
hipError_t launch_mlp_norm(const float *rec, int64_t n, float *norm, hipStream_t s);
hipError_t launch_mlp_calib(const unsigned char *blob, const float *rec, int64_t n, double *sums, float *norm,
                            hipStream_t s);
hipError_t launch_mlp_forward(const unsigned char *blob, const float *inp, int64_t n, float *out, hipStream_t s);
hipError_t launch_levels(int nl, int64_t ncell, const double *consts, const double *ncoll,
                         const double *ntot, const float *jbar, double *pops, float *k0_out,
                         float *eps_out, float *emis_out, hipStream_t s);

}  // namespace krt
