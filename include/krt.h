/*
 * krt.h -- C ABI of libkrt, the MI355X (gfx950) Monte Carlo line-transfer pass.
 *
 * The pass follows "Kratos-linerad: GPU-accelerated Monte Carlo radiative
 * transfer of lines with efficient imaging" (L. Wang): photon packets random-walk
 * through a uniform Cartesian grid of line-centre opacity, bulk velocity and
 * destruction probability; every interaction is a resonant scattering with
 * partial frequency redistribution (Sec. 2.1.1-2.1.2, eq. riia-scatter); the
 * packets tally the escaped spectrum, the camera-directed velocity-resolved
 * scattering emissivity (Sec. 2.2.1, eq. scat-line) and the profile-weighted
 * mean intensity that drives the level populations (Sec. 2.1.3).
 *
 * Conventions for every call:
 *   - Return 0 (KRT_OK) or a negative status; krt_last_error() gives a message.
 *   - Pointers named *_dev are DEVICE pointers on the context's device, owned
 *     by the caller, never freed by the library.  Host pointers are read during
 *     the call only.
 *   - Work is enqueued on the HIP stream given to krt_create, in call order.
 *     krt_mc_run and krt_levels_update synchronise that stream before they
 *     return (they read back a status word), so outputs are ready on return.
 *   - A context is not thread-safe; several contexts may coexist.
 *   - Arrays over cells use cell = (k * ny + j) * nx + i (x fastest).
 *   - Units: frequency x in Doppler widths (eq. xdef), velocities in units of
 *     the thermal speed b, lengths in the grid's own unit.
 */
#ifndef KRT_H_
#define KRT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum krt_status {
    KRT_OK = 0,
    KRT_EINVAL = -1,   /* bad argument, detected on the host before any launch */
    KRT_EHIP = -2,     /* a HIP runtime call failed */
    KRT_EDEVICE = -3,  /* the kernels flagged an anomaly (see KRT_ST_* in counters) */
    KRT_ESTATE = -4,   /* call out of order (e.g. run before grid/tables) */
};

/* boundary conditions per axis */
enum { KRT_BC_VACUUM = 0, KRT_BC_PERIODIC = 1 };
/* phase function of the re-emission about the incoming direction */
enum { KRT_PHASE_ISO = 0, KRT_PHASE_DIPOLE = 1 };
/* packet sources */
enum { KRT_SRC_POINT = 0, KRT_SRC_PLANE_Z = 1, KRT_SRC_VOLUME = 2, KRT_SRC_BEAM = 3 };
/* gas-frame emission profile */
enum { KRT_PROF_DELTA = 0, KRT_PROF_VOIGT = 1, KRT_PROF_GAUSS = 2 };

/* counters[] layout (int64) */
enum {
    KRT_C_EMITTED = 0, KRT_C_ESCAPED, KRT_C_DESTROYED, KRT_C_SCATTER, KRT_C_CROSS,
    KRT_C_STUCK, KRT_C_MLP, KRT_C_STATUS, KRT_C_EMIS_DROP, KRT_C_SKIPPED_SCAT,
    KRT_NCOUNTERS = 16
};
/* bits of counters[KRT_C_STATUS] */
enum { KRT_ST_NAN = 1, KRT_ST_STUCK = 2, KRT_ST_SATURATE = 4 };

typedef struct krt_ctx krt_ctx;

/* Create a context on HIP device `hip_device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the handle. */
int krt_create(krt_ctx **out, int hip_device, void *hip_stream);
void krt_destroy(krt_ctx *ctx);
const char *krt_last_error(const krt_ctx *ctx);
/* Number of compute units of the context's device (launch sizing). */
int krt_device_cus(const krt_ctx *ctx);
/* Duration in ms of the transport of the last krt_mc_run, from HIP events
 * recorded on the context's stream around its launch (plain and fused
 * schedules) or around all its rounds, host round trips included (park). */
double krt_last_transport_ms(const krt_ctx *ctx);
/* Learned escape in park mode: the summed time of the call-kernel launches of
 * the last krt_mc_run (ms, HIP events; 0 otherwise) and its number of rounds
 * (transport launches; 1 for the other schedules). */
double krt_last_network_ms(const krt_ctx *ctx);
int64_t krt_last_rounds(const krt_ctx *ctx);

/* ---------------------------------------------------------------- grid --- */
/* Uniform Cartesian grid with cell-wise constant fields (Sec. 2.2.1: the
 * emissivity is recorded per cell of a mesh; eq. sigma0: k0 = n_l sigma_0).
 * All field pointers are DEVICE pointers borrowed until the next upload or
 * krt_destroy; the library copies nothing except the volume-emission weights,
 * from which it builds an alias table (Walker/Vose) on the device.
 * Errors: KRT_EINVAL for n <= 0, hi <= lo, bad bc, n_lines outside 1..8,
 * k0 == NULL, ncell >= 2^31, or (with tclass_dev) n_tclass outside 1..8, a
 * ratio outside [0.05, 20] or a class index >= n_tclass (the indices are
 * copied to the host once and checked at upload), or (with bratio_dev) a
 * ratio outside [0.05, 20] or tclass_dev set as well. */
typedef struct {
    int32_t n[3];
    double lo[3], hi[3];
    int32_t bc[3];             /* KRT_BC_* per axis */
    int32_t n_lines;           /* number of line slices in k0/eps/emis */
    const float *k0_dev;       /* [n_lines][ncell] line-centre opacity per unit length */
    const float *vel_dev;      /* [3][ncell] bulk velocity / b (SoA), or NULL = static */
    const float *eps_dev;      /* [n_lines][ncell] destruction probability, or NULL = 0 */
    const float *emis_dev;     /* [n_lines][ncell] volume emission weights, or NULL */
    const float *kabs_dev;     /* [ncell] grey absorption coefficient (dust; units of k0), or NULL:
                                  it adds to every line's flight opacity, and an interaction is an
                                  absorption (packet destroyed) with probability
                                  kabs / (k0 H(a, x) + kabs), else a line scattering (Sec. 3.2) */
    /* Per-cell temperature as classes (frequencies are in units of the local
     * Doppler width, Sec. 2.1): tclass_dev [ncell] class of each cell, or NULL
     * (every cell at the reference width b_ref, the default).  Class k has
     * Doppler width b_k = tclass_bratio[k] b_ref (0.05..20): in its cells the
     * gas-frame frequency is (x - n.v) b_ref / b_k, the damping a b_ref / b_k
     * and each class gets its own exact table set; velocities, spectra and
     * channels stay in reference units, k0 is the cell's own line-centre
     * opacity.  Plain walk with profile_mode 0 only. */
    const uint8_t *tclass_dev;
    int32_t n_tclass;          /* 1..8 when tclass_dev is set */
    double tclass_bratio[8];
    /* Per-cell temperature as a continuum (Sec. 2.2.1: the two-dimensional Voigt
     * table over 64 logarithmically spaced damping values): bratio_dev [ncell]
     * b_cell / b_ref per cell (finite, 0.05..20), or NULL; not together with
     * tclass_dev.  Frequencies, damping and units as for the classes, each cell
     * with its own width; the opacity H(a_cell, x) is interpolated linearly in
     * ln a between 64 Voigt tables at log-spaced damping values spanning the
     * grid's range, and u_par is drawn from the sampler tables at the nearest
     * of 16 log-spaced damping values.  Plain walk with profile_mode 0 only;
     * the values are copied to the host once at upload, for their range. */
    const float *bratio_dev;
} krt_grid_desc;
int krt_grid_upload(krt_ctx *ctx, const krt_grid_desc *desc);

/* --------------------------------------------------------------- tables --- */
/* Per line: FP64 host construction of (i) the Voigt profile H(a, x) and its
 * derivative for cubic Hermite lookup (Sec. 2.1, ph_mode 2's one-dimensional
 * table at the run's damping parameter), (ii) the atom-velocity sampler for
 * p(u | x) ~ exp(-u^2)/(a^2 + (x-u)^2) (Sec. 2.1.1, the USampler), stored as
 * quantile tables of three pieces of the density, then uploaded as binary32
 * and staged into LDS by the transport kernel.  Errors: KRT_EINVAL for
 * a <= 0 or a > 1, phase not in KRT_PHASE_*, n_lines outside 1..8. */
typedef struct {
    double a;                  /* Voigt damping parameter A_ul / (4 pi nu_D) */
    int32_t phase;             /* KRT_PHASE_ISO | KRT_PHASE_DIPOLE */
    int32_t reserved;
} krt_line_desc;
int krt_tables_build(krt_ctx *ctx, const krt_line_desc *lines, int n_lines);

/* ------------------------------------------------------------------ run --- */
typedef struct {
    int32_t line;              /* which line slice / table set to use */
    int32_t source;            /* KRT_SRC_* */
    double src_pos[3];         /* point / beam position; plane: z = src_pos[2] */
    double src_dir[3];         /* beam direction (unit) */
    int32_t src_profile;       /* KRT_PROF_* */
    double src_x0;             /* line offset for KRT_PROF_DELTA */
    int32_t spec_nbins;        /* escaped spectrum bins over [spec_lo, spec_hi), 1..1024 */
    double spec_lo, spec_hi;
    int32_t emis_nch;          /* emissivity channels over [ch_lo, ch_hi), 0 (off)..256 */
    double ch_lo, ch_hi;
    double n_cam[3];           /* camera direction (unit) */
    int32_t jbar;              /* 1 = tally mean intensity per cell */
    int32_t accumulate;        /* 1 = add into the raw tallies, 0 = zero them first */
    uint64_t packet_offset;    /* first packet id (resume / sharding) */
    uint64_t max_events;       /* per packet; 0 = unlimited (2^32 - 2) */
    int32_t escape_mode;       /* 0 = plain random walk; 1 = learned escape in thick cells (needs
                                  krt_escape_init/train or put_weights; a in [1e-4, 1e-2]; no jbar;
                                  isotropic phase and no destruction or absorption field, else
                                  KRT_EINVAL: the network is trained on isotropic re-emission without
                                  either) */
    int32_t wg_size;           /* launch geometry: threads per workgroup (0 = 1024 plain, 512
                                  learned; the learned kernel is built for 256 VGPRs at <= 512
                                  lanes, 168 at <= 768, 128 above) */
    int32_t wg_per_cu;         /* workgroups per CU (0 = 1) */
    int32_t emis_frac_bits;    /* fixed-point fraction bits F of the emissivity tally (0 = 20) */
    int32_t jbar_frac_bits;    /* fraction bits of the mean-intensity tally (0 = 36) */
    uint64_t norm_packets;     /* packets for the FP32 normalisation (0 = n_packets) */
    double luminosity;         /* photons/s carried by all N packets; scales the FP32 outputs (0 = 1) */
    double esc_tau_min;        /* learned escape only at scattering points at least this line-centre
                                  depth below the nearest face of their cell (0 = 3) */
    double esc_cell_tau_min;   /* ... and only in cells of line-centre depth k0 dx at least this
                                  (0 = 100); both are raised to the smallest values the network's
                                  training records covered */
    int32_t esc_min_lanes;     /* network call when at least this many lanes of a wave ask (0 = 16);
                                  see esc_wait for the lanes that find fewer */
    int32_t esc_tail_lanes;    /* as esc_min_lanes once the packet pool is exhausted (0 = 1):
                                  the wave then lives only as long as its slowest packet */
    int32_t tail_lanes;        /* plain transport: once the pool is exhausted, a wave with at most
                                  this many live lanes lets its idle lanes precompute the live
                                  packets' random draws (0 = 32, negative = never); the tallies
                                  are the same either way */
    int32_t profile_mode;      /* opacity profile of the flights (Sec. 2.2.1, the paper's profile
                                  modes; plain walk only): 0 tables in LDS (production); 1 the
                                  same tables read from global memory (identical tallies, an A/B
                                  of the table placement); 2 analytic blend of the Doppler core
                                  exp(-u^2) and the damping wing a / (sqrt(pi)(u^2 + a^2)) by
                                  w = (1 + tanh(2|u| - 2 u0)) / 2, u0 where the two cross, with
                                  the exact redistribution: a demonstration of why the profile
                                  must match the sampler, not for production */
    int32_t esc_park;          /* learned-escape schedule.  0 (default): fused -- the network runs
                                  inside the transport kernel, batched over the asking lanes of a
                                  wave (esc_min_lanes).  1: park -- a packet whose scattering
                                  qualifies for a network call leaves the transport kernel as a
                                  64-byte record, a separate kernel evaluates the calls of all
                                  parked packets over full 16-sample blocks, and the packets resume
                                  in the next round; every qualifying scattering takes the network,
                                  so the tallies equal the fused schedule's at esc_min_lanes =
                                  esc_tail_lanes = 1 bit for bit and do not depend on launch
                                  geometry.  On the turbulent cloud park is 2-3x slower than fused
                                  (each round waits on host round trips and short segments).
                                  krt_mc_run_noalloc always runs fused */
    uint32_t esc_park_cap;     /* park: packets in flight at most (0 = 2^22; two lists of 64 B per
                                  packet, [1024, 2^28]) */
    uint32_t esc_park_tail;    /* park: once every packet is admitted and at most this many are in
                                  flight, one fused launch finishes them (0 = 65536) */
    uint32_t esc_park_budget;  /* park: a packet that takes this many plain scatterings in one round
                                  is parked after the last of them and resumes in the next round
                                  (0 = 256), so no round waits on one long walk */
    int32_t esc_wait;          /* fused: a lane whose scattering qualifies while fewer than
                                  esc_min_lanes lanes of its wave ask holds the scattering and
                                  waits for a batch, for at most this many loop iterations (0 = 32;
                                  a batch also goes when every live lane of the wave asks; while
                                  the packet pool lasts a batch of 16 or more takes whole
                                  16-sample blocks and the askers past them stay held).  Every
                                  qualifying scattering then takes the network with its own
                                  event's draws, so the tallies do not depend on launch geometry
                                  or batching and equal esc_min_lanes = 1's bit for bit.
                                  Negative: no waiting -- the lane walks that scattering and asks
                                  again at its next one, so which scatterings take the network
                                  depends on the packets sharing a wave (tallies statistically,
                                  not bitwise, reproducible) */
} krt_run_opts;

/* Caller-allocated DEVICE buffers.  Raw tallies are int64 fixed point, so their
 * sums are exact and independent of thread order and launch geometry:
 *   spec_raw [spec_nbins + 2]   packet counts; [0] below spec_lo, [nb+1] at/above spec_hi
 *   emis_raw [ncell][emis_nch]  sum of round(phase(g_cam) * 2^F) over scatterings
 *   jbar_raw [ncell]            sum of round(dl * H(a, x_gas) / sqrt(pi) * 2^Fj) over segments
 * Each contribution is rounded to the nearest integer before it is added, so
 * the sums are exact integers whatever the order.  A sum that passes 2^62 sets
 * KRT_ST_SATURATE (F = 20 allows 2.9e12 unit contributions per bin).
 *   counters [KRT_NCOUNTERS]
 *   packet_log [n_packets][8]   FP32 (x_lab, n_scat, outcome, n_x, n_y, n_z, cell, events)
 * Finalised FP32 outputs (FP64 scaling), each optional:
 *   spec  = L spec_raw / (N dx_bin)                   per unit x
 *   emis  = L emis_raw 2^-F / (4 pi N V_cell dx_ch)   per volume, steradian, unit x
 *   jbar  = L jbar_raw 2^-Fj / (4 pi N V_cell)
 * where N is norm_packets (or n_packets) and L the luminosity (or 1). */
typedef struct {
    int64_t *spec_raw_dev;
    int64_t *emis_raw_dev;
    int64_t *jbar_raw_dev;
    int64_t *counters_dev;
    float *packet_log_dev;
    float *spec_dev;
    float *emis_dev;
    float *jbar_dev;
} krt_tallies;

/* Run packets [packet_offset, packet_offset + n_packets) with Philox4x32-10
 * key `seed`.  The tallies are a pure function of (grid, tables, options,
 * seed, packet range).  Errors: KRT_EINVAL (n_packets == 0, missing required
 * buffer, bad bins, n_cam not unit, line out of range), KRT_ESTATE (no grid or
 * tables), KRT_EDEVICE (status bits set: NaN, stuck packets, saturation). */
int krt_mc_run(krt_ctx *ctx, uint64_t n_packets, uint64_t seed, const krt_run_opts *opts,
               krt_tallies *tallies);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * pass as krt_mc_run, identical tallies, calling no hipMalloc, hipFree or
 * allocating library routine.  Its scratch -- the packet-pool counter and the
 * staged bin edges -- lives in one 8 KiB array per GPU inside the library
 * (held until the process ends), the edges are staged through a pinned block
 * allocated by krt_create; inputs and outputs are the caller's, as for
 * krt_mc_run.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other contexts or streams) race and must not run
 * concurrently.  Limits: at most 1024 spectrum bins and 256 channels (the
 * scratch's capacity; larger requests return KRT_EINVAL); temperature classes
 * are refused (KRT_EINVAL: their tables are built on first use by krt_mc_run). */
int krt_mc_run_noalloc(krt_ctx *ctx, uint64_t n_packets, uint64_t seed, const krt_run_opts *opts,
                       krt_tallies *tallies);

/* -------------------------------------------------------------- imaging --- */
/* Deterministic ray-tracing imaging pass (Sec. 2.2.2, eq. imaging-formal,
 * eq. imaging-alphas): along lines of sight parallel to a
 * grid axis toward the camera, for every channel k and from the far side of
 * the grid to the camera, cell by cell
 *   I <- I exp(-dtau_k) + (j_k / alpha_k + S_emis,k) (1 - exp(-dtau_k)),
 *   alpha_k = k0 H(a, x_k - n_cam.v) + kappa_abs, dtau_k = alpha_k dl,
 * x_k the lab-frame centre of channel k over [ch_lo, ch_hi), k0 and v the
 * uploaded grid fields of `line`, kappa_abs an optional grey (channel-
 * independent) absorption coefficient per cell, e.g. dust, in the units of k0
 * (the Monte Carlo pass samples scattering only and the absorption enters
 * here: the paper's two-step scheme), H from that line's tables, dl the cell width
 * along the axis.  The scattering term is evaluated as j_k dl (1 - e^-dtau)/dtau,
 * finite as dtau -> 0.  j is the emissivity krt_mc_run finalised toward the
 * same camera (n_cam = the axis).  Pixels are the cells of the plane normal to
 * the axis, the lower remaining axis fastest: axis x -> pixel k*ny + j,
 * y -> k*nx + i, z -> j*nx + i.  Device arrays, caller-owned:
 *   emis_dev [ncell][nch], src_dev [ncell][nch] or NULL, kabs_dev [ncell] or
 *   NULL (no absorption), image_dev [npix][nch].
 * Errors: KRT_EINVAL (axis, nch outside 1..256, empty range, NULL arrays,
 * npix * nch above 2^31), KRT_ESTATE (no grid, no tables or opacity slice for
 * the line). */
typedef struct {
    int32_t line;
    int32_t axis;              /* camera direction: 0 +x, 1 +y, 2 +z, 3 -x, 4 -y, 5 -z */
    int32_t nch;
    double ch_lo, ch_hi;
    const float *emis_dev;
    const float *src_dev;
    float *image_dev;
    const float *kabs_dev;     /* absorption coefficient per cell (units of k0), or NULL */
} krt_image_desc;
int krt_image(krt_ctx *ctx, const krt_image_desc *desc);
/* Duration in ms of the last krt_image kernel, from HIP events that its dispatch records at the
 * kernel's start and end (host launch latency excluded). */
float krt_last_image_ms(const krt_ctx *ctx);

/* --------------------------------------------------------------- levels --- */
/* Statistical equilibrium per cell (Sec. 2.1.3; eq. boltzmann for two levels,
 * eq. eps for the destruction probability), FP64 on the device.  Levels
 * 0..nl-1 with radiative lines l -> l+1 (l = 0..nl-2) feeding the transport.
 * Rate matrix: A[u][l] decays, absorption Gamma_l per lower-level molecule with
 * Gamma_l = 4 pi sqrt(pi) sigma0_l jbar_l (the track-length estimate of the
 * absorption rate), stimulated emission (g_l/g_u) Gamma_l, collisions
 * Cd[u][l] * ncoll downward and (g_u/g_l) exp(-(E_u - E_l)) Cd ncoll upward
 * (detailed balance; E in units of kT); the last equation is replaced by
 * sum_i n_i = ntot.  Outputs k0_l = n_l sigma0_l,
 * eps_l = C_u,tot / (A[u][l] + C_u,tot) with C_u,tot the total collisional
 * rate out of level u = l+1, the emission n_u A_ul per unit volume and the
 * line power (cell volume x sum of n_u A_ul): the source of the Lambda
 * iteration, frozen at the collisional-equilibrium populations (Sec. 2.1.3).  Host arrays: E[nl], g[nl], A[nl*nl], Cd[nl*nl],
 * sigma0[nl-1].  The device arrays hold `ncell` cells each; the call is
 * independent of the uploaded grid (it may precede krt_grid_upload, and the
 * caller sizes every device array for `ncell`).  Errors: KRT_EINVAL (nl
 * outside 2..8, ncell outside 1..2^31-1, NULL arrays, non-finite constants,
 * lum_out without a finite cell_volume > 0). */
typedef struct {
    int32_t n_levels;
    int64_t ncell;                           /* cells in every device array */
    const double *E, *g, *A, *Cd, *sigma0;   /* host */
    const double *ncoll_dev, *ntot_dev;      /* device [ncell] */
    double *pops_dev;                        /* device [ncell][nl], written */
    float *k0_out_dev, *eps_out_dev;         /* device [nl-1][ncell], written (may be NULL) */
    float *emis_out_dev;                     /* device [nl-1][ncell], written (may be NULL): n_u A_ul,
                                                the line's spontaneous emission per unit volume */
    double cell_volume;                      /* volume of one cell (needed with lum_out) */
    double *lum_out;                         /* host [nl-1], written (may be NULL): cell_volume times
                                                the sum over cells of n_u A_ul, FP64 in a fixed
                                                order (the line's total power) */
} krt_levels_desc;
int krt_levels_update(krt_ctx *ctx, const krt_levels_desc *desc,
                      const float *jbar_dev /* [nl-1][ncell], NULL = no radiation */);

/* ------------------------------------------------------- learned escape --- */
/* A small network (24 -> 3 x 128 leaky ReLU -> 32, BF16 weights and activations,
 * FP32 accumulation on MFMA) replaces the random walk of a photon inside one
 * homogeneous cubic cell: at a scattering in a cell whose line-centre depth
 * k0 dx is at least esc_cell_tau_min, at least esc_tau_min (line-centre) below
 * the cell's nearest face and with gas-frame |x| <= 2, one sample gives where
 * the photon leaves the cell (exit face, point on it, direction, frequency)
 * and the expected number of scatterings it skipped, whose emissivity is
 * deposited in the cell.  The paper itself propagates every photon through the
 * full optical depth (Sec. 2.3.2, Sec. 4.1); this proposal is the accelerated
 * alternative it points to for extreme depths, and the plain random walk
 * remains the fallback (thin cells, shallow points, wing photons, a outside
 * [1e-4, 1e-2], non-cubic cells, and anything outside the training records'
 * ranges).
 *
 * Conditions are taken in the cell's reduced frame (its 48 symmetries and
 * x -> -x): the start point's offsets from the cell centre in half-widths,
 * absolute values sorted ascending (q0 <= q1 <= q2, axis 2 toward the nearest
 * face), the incoming direction reflected and permuted alike, |x_in| (the exit
 * frequency takes x_in's sign), tau_c = k0 dx / 2 (line-centre depth centre to
 * face) and depth = tau_c (1 - q2).  Exit face F = 2 axis + (outward normal
 * along +axis) in that frame; exit offsets ys, yt = (exit point - the start
 * point's projection onto the face) along the two axes following the face
 * axis cyclically, over the start point's distance to the face's plane; exit
 * cosine mu to the outward normal; alpha in [0, pi] the angle between the
 * exit direction's tangential part and that offset (its sign is drawn
 * uniformly).  Inputs (normalised): (log10 tau_c - 3)/1.2, log10 a + 3,
 * |x_in| - 1, 2 q - 1 (3), (log10 depth - 2)/1.2, incoming direction (3), four
 * quantile levels as logit(u)/4, a flag (0 marginal, 1 conditional), and for
 * conditional rows x_out/4 and the one-hot exit face.  The network has 32
 * outputs; a call takes two evaluations: marginal (outputs 0-5 exit-face
 * logits, 6 logit P(x_out >= 0), 7 ln E[N_s], 8 quantile of ln <x^2> at u_b,
 * 16 + F quantile of |x_out| at u_a given exit face F), then conditional on
 * the sampled face and x_out (9, 10 quantiles of asinh ys, asinh yt at u_a,
 * u_b; 11 of mu^2 at u_c; 12 of alpha at u_d); 13-15 and 22-31 are unused.
 * Losses: softmax cross-entropy (face), logistic (side), pinball (quantiles;
 * output 16 + F only on walks leaving through F), log-deviance e^d - 1 - d,
 * d = ln N_s - output, for output 7; a third of the training rows are
 * conditional.
 *
 * Parameters: kNParams = 40352 FP32 master values, then 328 constants: target
 * mean[32] and scale[32], 256 additive calibration terms of ln E[N_s] (per bin
 * of log10 tau_c in 8 bins of 0.5 over [1, 5), log10 depth in 8 bins of 0.5
 * over [0, 4) and |x_in| in 4 bins of 0.5 over [0, 2), ends clamped; index =
 * (tau bin * 8 + depth bin) * 4 + x bin), then the training records' ranges:
 * log10 a (min, max), log10 tau_c (min, max), the smallest log10 depth, three
 * floats of padding.  krt_mc_run refuses escape_mode 1 for a line whose log10 a
 * lies outside the a range by more than 0.01 (KRT_EINVAL), and makes no call
 * outside the tau_c range or above the smallest depth.
 *
 * krt_escape_init: He-uniform parameters from Philox(seed), Adam state zeroed.
 * krt_escape_record: 1 <= n <= 2^31 whole-cell walks for line `line` (ids
 *   [offset, offset + n), Philox key seed), conditions from *cond:
 *   log10 tau_c uniform in [log10_tau_lo, log10_tau_hi] (within [0, 6]); then
 *   either (fixed = 0) |x_in| from 1/2 |N(0, 1/2)| + 1/2 U[0, 3], log10 depth
 *   uniform in [log10_depth_lo, log10 tau_c], q0, q1 uniform in [0, q2] and an
 *   isotropic incoming direction, or (fixed = 1) the given x_in >= 0 and
 *   0 <= q0 <= q1 <= q2 < 1, with n_in (unit) or isotropic directions
 *   (iso_dir = 1).  samples_dev [n][20] FP32: (log10 tau_c, log10 a, |x_in|,
 *   q0, q1, q2, log10 depth, n_in (3), F, ys, yt, mu, alpha, x_out, ln N_s,
 *   ln <x^2>, valid, 0); a walk past 2e7 scatterings is stored invalid.
 * krt_escape_fit_norm: target mean / scale and the training ranges from the
 *   valid records; clears the calibration.
 * krt_escape_calibrate: n < 2^30 records; per calibration bin with at least
 *   100 valid records with |x_in| <= 2, the term ln(sum N_s / sum exp(network
 *   ln E[N_s])) over the records (marginal rows, quantile levels drawn per
 *   record), so that the predicted mean count is unbiased bin by bin; other
 *   bins get 0.
 * krt_escape_grad: gradient of the mean loss over the batch given by
 *   idx_dev [batch] (record indices, 1 <= batch <= 2^20) and u_dev [batch][5]
 *   = (u_a, u_b, u_c, u_d, 1 for a conditional row else 0); grad_out_dev
 *   [40352], loss_out_dev [1] (may be NULL).
 * krt_escape_train: `steps` Adam steps (lr, betas 0.9/0.999) on random batches
 *   (Philox(seed)) of 1 <= batch <= 2^20 out of n < 2^31 records;
 *   loss_hist_dev [steps] or NULL.
 * krt_escape_get_weights / put_weights: [40352 + 328] FP32 device buffers.
 * krt_escape_forward: in_dev [n][17] raw (log10 tau_c, log10 a, |x_in|, q0,
 *   q1, q2, log10 depth, n_in (3), u_a, u_b, u_c, u_d, flag, x_out, F) ->
 *   out_dev [n][32] de-normalised (logits as logits, output 7 with its
 *   calibration term, outputs 9-11 as asinh ys, asinh yt, mu^2); n < 2^30.
 * Errors: KRT_EINVAL (sizes, ranges), KRT_ESTATE (no init / no tables). */
typedef struct {
    double log10_tau_lo, log10_tau_hi;  /* log10 tau_c range */
    double log10_depth_lo;              /* lower end of log10 depth (fixed = 0), in [-2, 6] */
    int32_t fixed;                      /* 1: every walk starts from x_in, q, n_in below */
    int32_t iso_dir;                    /* with fixed: isotropic incoming directions */
    double x_in, q[3], n_in[3];
} krt_escape_cond;
int krt_escape_init(krt_ctx *ctx, uint64_t seed);
int krt_escape_record(krt_ctx *ctx, int32_t line, uint64_t n, uint64_t seed, uint64_t offset,
                      const krt_escape_cond *cond, float *samples_dev);
int krt_escape_fit_norm(krt_ctx *ctx, const float *samples_dev, uint64_t n);
int krt_escape_calibrate(krt_ctx *ctx, const float *samples_dev, uint64_t n);
int krt_escape_grad(krt_ctx *ctx, const float *samples_dev, const int32_t *idx_dev, const float *u_dev,
                    int32_t batch, float *grad_out_dev, float *loss_out_dev);
int krt_escape_train(krt_ctx *ctx, const float *samples_dev, uint64_t n, int32_t steps, int32_t batch,
                     double lr, uint64_t seed, float *loss_hist_dev);
int krt_escape_get_weights(krt_ctx *ctx, float *dev, uint64_t nfloats);
int krt_escape_put_weights(krt_ctx *ctx, const float *dev, uint64_t nfloats);
int krt_escape_forward(krt_ctx *ctx, const float *in_dev, int64_t n, float *out_dev);

/* ----------------------------------------------------------- diagnostics --- */
/* Device-side evaluations of the individual steps, for parity tests.
 * krt_debug_philox: out[i] = Philox4x32-10(ctr[i], key[i]); ctr [n][4],
 *   key [n][2], out [n][4], uint32, device.
 * krt_debug_bins: out[i] = bin of x[i] over nb bins in [lo, hi) (0 below,
 *   nb+1 at/above, -1 NaN), the index rule of every tally.
 * krt_debug_voigt: out[i] = H(a_line, x[i]) from the staged tables.
 * krt_debug_upar: out[i] = u_par drawn for gas-frame frequency x from event
 *   ev0 + i of packet `packet` (the words the transport uses).
 * Every diagnostic takes 1 <= n <= 2^31 elements, else KRT_EINVAL. */
int krt_debug_philox(krt_ctx *ctx, const uint32_t *ctr_dev, const uint32_t *key_dev,
                     uint32_t *out_dev, int64_t n);
int krt_debug_bins(krt_ctx *ctx, const float *x_dev, int64_t n, int32_t nb, double lo,
                   double hi, int32_t *out_dev);
/* krt_debug_voigt_analytic: out[i] = the analytic profile of profile_mode 2 at
 * x[i] for damping a (u0 from a as krt_mc_run computes it); device arrays. */
int krt_debug_voigt_analytic(krt_ctx *ctx, double a, const float *x, int64_t n, float *out);
int krt_debug_voigt(krt_ctx *ctx, int32_t line, const float *x_dev, int64_t n, float *out_dev);
/* krt_debug_voigt_cont: out[i] = H(a_line b_ref / b, x[i]) at the width ratio
 * r[i] = b / b_ref (within the uploaded grid's range) as the transport of a
 * grid with per-cell widths (bratio_dev) evaluates it: the two neighbouring
 * Voigt tables of the 64 log-spaced damping nodes, interpolated linearly in
 * ln a (Sec. 2.2.1's two-dimensional table).  Device arrays of n floats;
 * KRT_ESTATE without such a grid or tables for the line. */
int krt_debug_voigt_cont(krt_ctx *ctx, int32_t line, const float *r_dev, const float *x_dev, int64_t n,
                         float *out_dev);
int krt_debug_upar(krt_ctx *ctx, int32_t line, float x, uint64_t seed, uint64_t packet,
                   uint32_t ev0, int64_t n, float *out_dev);

#ifdef __cplusplus
}
#endif
#endif /* KRT_H_ */
