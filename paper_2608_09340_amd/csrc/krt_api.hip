// krt_api.hip -- the C ABI of libkrt (include/krt.h): argument validation,
// device-side state, launches, and the per-cell statistical-equilibrium kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <string>
#include <thread>
#include <system_error>
#include <vector>

#include "krt.h"
#include "krt_internal.h"
#include "krt_image.h"
#include "krt_kernels.h"
#include "krt_mlp.h"

using namespace krt;

struct krt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int cus = 256;
    std::string err;
    // grid
    bool have_grid = false;
    krt_grid_desc grid{};
    int64_t ncell = 0;
    std::vector<float *> alias_prob;
    std::vector<int *> alias_idx;
    // tables
    std::vector<float *> tab;
    // temperature classes: table sets [class][kTabFloats] and per-class
    // parameters for the line they were built for (cache key: line, ratios, a)
    float *cls_tab = nullptr;
    float4 *cls_par = nullptr;
    int cls_line = -1;
    double cls_key[9] = {0};
    // continuous per-cell temperature: the grid's range of b / b_ref, the Voigt
    // blocks [kContVoigtN + 1][kVoigtFloats], sampler blocks [kContSampN][kTabFloats]
    // and their (damping, threshold), built for one line (cache key: a, range)
    float br_lo = 1.0f, br_hi = 1.0f;
    float *cv_tab = nullptr, *cs_tab = nullptr;
    float2 *cs_par = nullptr;
    int cont_n_v = 0, cont_n_s = 0;
    double cont_lna0 = 0.0, cont_inv_v = 0.0, cont_inv_s = 0.0;
    double cont_key[3] = {-1.0, 0.0, 0.0};
    std::vector<krt_line_desc> lines;
    // scratch
    unsigned long long *work_counter = nullptr;
    double *level_consts = nullptr;
    double *level_power = nullptr;   // per-line partial and total powers of krt_levels_update
    int64_t *host_pinned = nullptr;
    float *host_edges = nullptr;          // pinned staging of the bin edges for krt_mc_run_noalloc
    unsigned char *scratch_dev = nullptr; // this device's address of the no-allocation scratch array
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // bracket the last run's transport launches
    hipEvent_t evn0 = nullptr, evn1 = nullptr; // bracket one launch of the call kernel
    float last_ms = 0.0f, last_net_ms = 0.0f;
    int64_t last_rounds = 0;
    // learned escape in park mode: two lists of parked packets and their counter
    uint4 *park_buf[2] = {nullptr, nullptr};
    uint64_t park_alloc = 0;                   // records per list
    unsigned long long *park_counter = nullptr;
    // learned escape: FP32 master parameters, Adam moments, gradient, packed BF16 image
    float *edges = nullptr;                    // [kEdgeFloats]: spectrum then channel edges
    bool mlp_ready = false;
    float esc_la_lo = 1.0f, esc_la_hi = -1.0f;  // log10 a range the network was fitted on (empty: none)
    float esc_lt_lo = 1.0f, esc_lt_hi = -1.0f;  // log10 tau_c range of its training records
    float esc_ld_min = 0.0f;                    // smallest log10 depth of its training records
    float *mlp_p = nullptr, *mlp_m = nullptr, *mlp_v = nullptr, *mlp_g = nullptr, *mlp_norm = nullptr;
    float *mlp_loss = nullptr, *mlp_u = nullptr;
    float *mlp_part = nullptr;                 // [kGradSplits][kNParams] split gradients
    uint16_t *mlp_act = nullptr;               // [kActRowsAll][mlp_act_cap] bf16 activation store
    int64_t mlp_act_cap = 0;
    int32_t *mlp_idx = nullptr;
    int mlp_batch_cap = 0;
    int mlp_step = 0;
    unsigned char *mlp_blob = nullptr, *mlp_img = nullptr;
    double *mlp_calsum = nullptr;
    float last_image_ms = 0.0f;
};

namespace {

int fail(krt_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(ctx, expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), KRT_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

void free_grid(krt_ctx *c) {
    for (auto p : c->alias_prob) if (p) (void)hipFree(p);
    for (auto p : c->alias_idx) if (p) (void)hipFree(p);
    c->alias_prob.clear();
    c->alias_idx.clear();
    c->have_grid = false;
}

void free_tables(krt_ctx *c) {
    for (auto p : c->tab) if (p) (void)hipFree(p);
    c->tab.clear();
    c->lines.clear();
    c->cls_line = -1;  // class tables follow the line tables
    c->cont_key[0] = -1.0;  // and so do the continuum's
}

// Table sets of the grid's temperature classes for line l (damping
// a_l b_ref / b_k per class), rebuilt only when the line or the ratios change.
static int ensure_class_tables(krt_ctx *c, int l) {
    const krt_grid_desc &g = c->grid;
    double key[9];
    key[0] = c->lines[l].a;
    for (int k = 0; k < 8; ++k) key[k + 1] = k < g.n_tclass ? g.tclass_bratio[k] : 0.0;
    if (c->cls_line == l && std::equal(key, key + 9, c->cls_key)) return KRT_OK;
    if (!c->cls_tab) HIPCHK(c, hipMalloc(&c->cls_tab, sizeof(float) * 8 * (size_t)kTabFloats));
    if (!c->cls_par) HIPCHK(c, hipMalloc(&c->cls_par, sizeof(float4) * 8));
    std::vector<float> tab;
    float4 par[8];
    for (int k = 0; k < g.n_tclass; ++k) {
        const double s = 1.0 / g.tclass_bratio[k], ak = c->lines[l].a * s;
        build_line_tables(ak, tab);
        HIPCHK(c, hipMemcpy(c->cls_tab + (size_t)k * kTabFloats, tab.data(), sizeof(float) * kTabFloats,
                            hipMemcpyHostToDevice));
        par[k] = make_float4((float)s, (float)ak, (float)std::atan(kDelta / ak), (float)g.tclass_bratio[k]);
    }
    HIPCHK(c, hipMemcpy(c->cls_par, par, sizeof(float4) * g.n_tclass, hipMemcpyHostToDevice));
    c->cls_line = l;
    std::copy(key, key + 9, c->cls_key);
    return KRT_OK;
}

// Table blocks of a continuum of cell temperatures for line l: kContVoigtN
// Voigt blocks and kContSampN sampler blocks at damping values log-spaced over
// [a_l / br_hi, a_l / br_lo] (one node of each when the grid has one width),
// built on the host threads in parallel (the FP64 Voigt quadrature takes
// seconds per damping value), then copied to the device.
constexpr int kContVoigtN = 64, kContSampN = 16;
static int ensure_cont_tables(krt_ctx *c, int l) {
    const double a_l = c->lines[l].a;
    const double key[3] = {a_l, (double)c->br_lo, (double)c->br_hi};
    if (std::equal(key, key + 3, c->cont_key)) return KRT_OK;
    const double lna0 = std::log(a_l / c->br_hi), span = std::log((double)c->br_hi / (double)c->br_lo);
    const bool one = !(span > 1e-9);
    const int nv = one ? 1 : kContVoigtN, ns = one ? 1 : kContSampN;
    std::vector<float> hv((size_t)(nv + 1) * kVoigtFloats), hs((size_t)ns * kTabFloats, 0.0f);
    std::vector<float2> hp(ns);
    auto node_a = [&](int k, int n) { return n == 1 ? a_l / c->br_hi : std::exp(lna0 + span * k / (n - 1)); };
    std::atomic<int> next{0};
    auto work = [&]() {
        std::vector<float> tmp(kTabFloats);
        for (int j = next++; j < nv + ns; j = next++) {
            if (j < nv) {
                build_voigt_block(node_a(j, nv), tmp.data());
                std::copy(tmp.begin(), tmp.begin() + kVoigtFloats, hv.begin() + (size_t)j * kVoigtFloats);
            } else {
                const int k = j - nv;
                build_sampler_block(node_a(k, ns), hs.data() + (size_t)k * kTabFloats);
            }
        }
    };
    const int nt = std::max(1, std::min<int>((int)std::thread::hardware_concurrency(), nv + ns));
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) {
        try {
            pool.emplace_back(work);
        } catch (const std::system_error &) {
            break;  // no more threads: the ones started (and this one) take the rest
        }
    }
    work();
    for (auto &t : pool) t.join();
    std::copy(hv.begin() + (size_t)(nv - 1) * kVoigtFloats, hv.begin() + (size_t)nv * kVoigtFloats,
              hv.begin() + (size_t)nv * kVoigtFloats);  // the upper neighbour of the last node
    for (int k = 0; k < ns; ++k) {
        const double ak = node_a(k, ns);
        hp[k] = make_float2((float)ak, (float)std::atan(kDelta / ak));
    }
    if (!c->cv_tab) HIPCHK(c, hipMalloc(&c->cv_tab, sizeof(float) * (size_t)(kContVoigtN + 1) * kVoigtFloats));
    if (!c->cs_tab) HIPCHK(c, hipMalloc(&c->cs_tab, sizeof(float) * (size_t)kContSampN * kTabFloats));
    if (!c->cs_par) HIPCHK(c, hipMalloc(&c->cs_par, sizeof(float2) * kContSampN));
    HIPCHK(c, hipMemcpy(c->cv_tab, hv.data(), sizeof(float) * hv.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->cs_tab, hs.data(), sizeof(float) * hs.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->cs_par, hp.data(), sizeof(float2) * ns, hipMemcpyHostToDevice));
    c->cont_n_v = nv;
    c->cont_n_s = ns;
    c->cont_lna0 = lna0;
    c->cont_inv_v = one ? 0.0 : (nv - 1) / span;
    c->cont_inv_s = one ? 0.0 : (ns - 1) / span;
    std::copy(key, key + 3, c->cont_key);
    return KRT_OK;
}

static void set_cont_params(const krt_ctx *c, RunParams &P) {
    P.bratio = c->grid.bratio_dev;
    P.cv_tab = c->cv_tab;
    P.cs_tab = c->cs_tab;
    P.cs_par = c->cs_par;
    P.cv_lna0 = (float)c->cont_lna0;
    P.cv_inv_step = (float)c->cont_inv_v;
    P.cs_inv_step = (float)c->cont_inv_s;
    P.cv_n = c->cont_n_v;
    P.cs_n = c->cont_n_s;
}

// Walker/Vose alias table over non-negative weights (FP64 build).
void build_alias(const std::vector<float> &w, std::vector<float> &prob, std::vector<int> &alias) {
    const int64_t n = (int64_t)w.size();
    prob.assign(n, 0.0f);
    alias.assign(n, 0);
    double tot = 0.0;
    for (float v : w) tot += (double)v;
    std::vector<double> q(n);
    std::vector<int64_t> small, large;
    for (int64_t i = 0; i < n; ++i) {
        q[i] = (double)w[i] * (double)n / tot;
        (q[i] < 1.0 ? small : large).push_back(i);
    }
    while (!small.empty() && !large.empty()) {
        int64_t s = small.back(); small.pop_back();
        int64_t l = large.back();
        prob[s] = (float)q[s];
        alias[s] = (int)l;
        q[l] -= 1.0 - q[s];
        if (q[l] < 1.0) { large.pop_back(); small.push_back(l); }
    }
    for (int64_t i : large) { prob[i] = 1.0f; alias[i] = (int)i; }
    for (int64_t i : small) { prob[i] = 1.0f; alias[i] = (int)i; }
}

bool valid_bins(int nb, double lo, double hi) {
    return nb > 0 && nb < (1 << 24) && std::isfinite(lo) && std::isfinite(hi) && hi > lo;
}

// binary32 bin edges lo + (hi - lo) k / nb, k = 0..nb, evaluated in FP64
void fill_edges(float *e, int nb, double lo, double hi) {
    for (int k = 0; k <= nb; ++k) e[k] = (float)(lo + (hi - lo) * (double)k / (double)nb);
}

}  // namespace

// ------------------------------------------------------------------ ctx ---
// Scratch of krt_mc_run_noalloc, one copy per GPU in the library's code object:
// the packet-pool counter (first 256 bytes), then the binary32 bin edges of the
// spectrum and the channels staged for the transport kernel.  Host code never
// passes the array's name to a kernel: each context resolves this device's
// address with hipGetSymbolAddress at creation (scratch_dev).
constexpr size_t kNoAllocScratchBytes = 8192;
constexpr size_t kNoAllocEdgeOffset = 256;
static_assert(kNoAllocEdgeOffset + sizeof(float) * kEdgeFloats <= kNoAllocScratchBytes, "edges fit the scratch");
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

extern "C" int krt_create(krt_ctx **out, int hip_device, void *hip_stream) {
    if (!out) return KRT_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return KRT_EINVAL;
    krt_ctx *c = new krt_ctx();
    c->device = hip_device;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(hip_device) != hipSuccess) { delete c; return KRT_EHIP; }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && cus > 0)
        c->cus = cus;
    if (hipMalloc(&c->work_counter, sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&c->level_consts, sizeof(double) * 256) != hipSuccess ||
        hipHostMalloc(&c->host_pinned, sizeof(int64_t) * 64, hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipEventCreate(&c->evn0) != hipSuccess || hipEventCreate(&c->evn1) != hipSuccess ||
        hipMalloc(&c->park_counter, sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc(&c->edges, sizeof(float) * kEdgeFloats) != hipSuccess ||
        hipHostMalloc(&c->host_edges, sizeof(float) * kEdgeFloats, hipHostMallocDefault) != hipSuccess) {
        krt_destroy(c);
        return KRT_EHIP;
    }
    // this device's copy of the no-allocation scratch (the device is current)
    if (hipGetSymbolAddress(reinterpret_cast<void **>(&c->scratch_dev), HIP_SYMBOL(scratch)) != hipSuccess ||
        c->scratch_dev == nullptr) {
        krt_destroy(c);
        return KRT_EHIP;
    }
    *out = c;
    return KRT_OK;
}

extern "C" void krt_destroy(krt_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream); else (void)hipDeviceSynchronize();
    free_grid(c);
    free_tables(c);
    if (c->cls_tab) (void)hipFree(c->cls_tab);
    if (c->cls_par) (void)hipFree(c->cls_par);
    if (c->cv_tab) (void)hipFree(c->cv_tab);
    if (c->cs_tab) (void)hipFree(c->cs_tab);
    if (c->cs_par) (void)hipFree(c->cs_par);
    if (c->work_counter) (void)hipFree(c->work_counter);
    if (c->level_consts) (void)hipFree(c->level_consts);
    if (c->level_power) (void)hipFree(c->level_power);
    if (c->host_pinned) (void)hipHostFree(c->host_pinned);
    if (c->host_edges) (void)hipHostFree(c->host_edges);
    for (void *p : {(void *)c->mlp_p, (void *)c->mlp_m, (void *)c->mlp_v, (void *)c->mlp_g, (void *)c->mlp_norm,
                    (void *)c->mlp_loss, (void *)c->mlp_u, (void *)c->mlp_idx, (void *)c->mlp_blob,
                    (void *)c->mlp_img, (void *)c->mlp_calsum, (void *)c->mlp_part, (void *)c->mlp_act})
        if (p) (void)hipFree(p);
    if (c->edges) (void)hipFree(c->edges);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->evn0) (void)hipEventDestroy(c->evn0);
    if (c->evn1) (void)hipEventDestroy(c->evn1);
    if (c->park_counter) (void)hipFree(c->park_counter);
    for (int k = 0; k < 2; ++k)
        if (c->park_buf[k]) (void)hipFree(c->park_buf[k]);
    delete c;
}

extern "C" const char *krt_last_error(const krt_ctx *c) { return c ? c->err.c_str() : "null context"; }

extern "C" int krt_device_cus(const krt_ctx *c) { return c ? c->cus : 0; }

extern "C" double krt_last_transport_ms(const krt_ctx *c) { return c ? (double)c->last_ms : -1.0; }
extern "C" double krt_last_network_ms(const krt_ctx *c) { return c ? (double)c->last_net_ms : -1.0; }
extern "C" int64_t krt_last_rounds(const krt_ctx *c) { return c ? c->last_rounds : -1; }

// ----------------------------------------------------------------- grid ---
extern "C" int krt_grid_upload(krt_ctx *c, const krt_grid_desc *d) {
    if (!c) return KRT_EINVAL;
    if (!d) return fail(c, KRT_EINVAL, "grid desc is NULL");
    int64_t ncell = 1;
    for (int k = 0; k < 3; ++k) {
        if (d->n[k] <= 0) return fail(c, KRT_EINVAL, "n[%d] = %d must be > 0", k, d->n[k]);
        if (!(d->hi[k] > d->lo[k]) || !std::isfinite(d->lo[k]) || !std::isfinite(d->hi[k]))
            return fail(c, KRT_EINVAL, "axis %d: need finite hi > lo", k);
        if (d->bc[k] != KRT_BC_VACUUM && d->bc[k] != KRT_BC_PERIODIC)
            return fail(c, KRT_EINVAL, "bc[%d] = %d invalid", k, d->bc[k]);
        ncell *= d->n[k];
    }
    if (ncell >= (1LL << 31)) return fail(c, KRT_EINVAL, "too many cells (%lld)", (long long)ncell);
    if (d->n_lines < 1 || d->n_lines > 8) return fail(c, KRT_EINVAL, "n_lines = %d outside 1..8", d->n_lines);
    if (!d->k0_dev) return fail(c, KRT_EINVAL, "k0 is NULL");
    if (d->tclass_dev) {
        if (d->n_tclass < 1 || d->n_tclass > 8) return fail(c, KRT_EINVAL, "n_tclass = %d outside 1..8", d->n_tclass);
        for (int k = 0; k < d->n_tclass; ++k)
            if (!(d->tclass_bratio[k] >= 0.05 && d->tclass_bratio[k] <= 20.0))
                return fail(c, KRT_EINVAL, "tclass_bratio[%d] = %g outside [0.05, 20]", k, d->tclass_bratio[k]);
    }
    if (d->bratio_dev && d->tclass_dev) return fail(c, KRT_EINVAL, "bratio and temperature classes are exclusive");
    HIPCHK(c, hipSetDevice(c->device));
    float br_lo = 1.0f, br_hi = 1.0f;
    if (d->bratio_dev) {
        // the range of widths sets the damping nodes of the tables
        std::vector<float> br((size_t)ncell);
        HIPCHK(c, hipMemcpy(br.data(), d->bratio_dev, sizeof(float) * (size_t)ncell, hipMemcpyDeviceToHost));
        br_lo = br_hi = br[0];
        for (float v : br) {
            if (!(v >= 0.05f && v <= 20.0f)) return fail(c, KRT_EINVAL, "bratio %g outside [0.05, 20]", (double)v);
            br_lo = std::min(br_lo, v);
            br_hi = std::max(br_hi, v);
        }
    }
    if (d->tclass_dev) {
        // every class index must name a class: the transport indexes the class
        // parameters and table sets with it
        std::vector<uint8_t> cls((size_t)ncell);
        HIPCHK(c, hipMemcpy(cls.data(), d->tclass_dev, (size_t)ncell, hipMemcpyDeviceToHost));
        const uint8_t mx = *std::max_element(cls.begin(), cls.end());
        if (mx >= d->n_tclass) return fail(c, KRT_EINVAL, "class index %d >= n_tclass %d", (int)mx, d->n_tclass);
    }
    free_grid(c);
    c->grid = *d;
    c->cls_line = -1;
    c->br_lo = br_lo;
    c->br_hi = br_hi;
    c->ncell = ncell;
    c->alias_prob.assign(d->n_lines, nullptr);
    c->alias_idx.assign(d->n_lines, nullptr);
    if (d->emis_dev) {
        std::vector<float> w(ncell), prob;
        std::vector<int> alias;
        for (int l = 0; l < d->n_lines; ++l) {
            HIPCHK(c, hipMemcpyAsync(w.data(), d->emis_dev + (int64_t)l * ncell, sizeof(float) * ncell,
                                     hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            double tot = 0.0;
            for (float v : w) {
                if (!(v >= 0.0f) || !std::isfinite(v)) return fail(c, KRT_EINVAL, "emission weights must be finite and >= 0");
                tot += v;
            }
            if (!(tot > 0.0)) continue;  // no volume source for this line
            build_alias(w, prob, alias);
            HIPCHK(c, hipMalloc(&c->alias_prob[l], sizeof(float) * ncell));
            HIPCHK(c, hipMalloc(&c->alias_idx[l], sizeof(int) * ncell));
            HIPCHK(c, hipMemcpyAsync(c->alias_prob[l], prob.data(), sizeof(float) * ncell, hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->alias_idx[l], alias.data(), sizeof(int) * ncell, hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
    }
    c->have_grid = true;
    return KRT_OK;
}

// --------------------------------------------------------------- tables ---
extern "C" int krt_tables_build(krt_ctx *c, const krt_line_desc *lines, int n_lines) {
    if (!c) return KRT_EINVAL;
    if (!lines || n_lines < 1 || n_lines > 8) return fail(c, KRT_EINVAL, "n_lines = %d outside 1..8", n_lines);
    for (int l = 0; l < n_lines; ++l) {
        if (!(lines[l].a > 0.0 && lines[l].a <= 1.0)) return fail(c, KRT_EINVAL, "line %d: a = %g outside (0, 1]", l, lines[l].a);
        if (lines[l].phase != KRT_PHASE_ISO && lines[l].phase != KRT_PHASE_DIPOLE)
            return fail(c, KRT_EINVAL, "line %d: phase %d invalid", l, lines[l].phase);
    }
    HIPCHK(c, hipSetDevice(c->device));
    free_tables(c);
    std::vector<float> tab;
    for (int l = 0; l < n_lines; ++l) {
        build_line_tables(lines[l].a, tab);
        float *d = nullptr;
        HIPCHK(c, hipMalloc(&d, sizeof(float) * kTabFloats));
        c->tab.push_back(d);
        HIPCHK(c, hipMemcpyAsync(d, tab.data(), sizeof(float) * kTabFloats, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->lines.push_back(lines[l]);
    }
    return KRT_OK;
}

// ------------------------------------------------------------------ run ---
// Crossing point u0 > 1 of the Doppler core exp(-u^2) and the damping wing
// a / (sqrt(pi) (u^2 + a^2)) (the centre of the analytic profile's switch), by
// bisection in FP64: core - wing is positive at u = 1 and negative at u = 10
// for damping 0 < a < 1 (the range of lines this library tabulates).
static double voigt_crossing(double a) {
    auto f = [a](double u) { return std::exp(-u * u) - a / (std::sqrt(M_PI) * (u * u + a * a)); };
    double lo = 1.0, hi = 10.0;
    for (int k = 0; k < 200; ++k) {
        const double m = 0.5 * (lo + hi);
        (f(m) > 0.0 ? lo : hi) = m;
    }
    return 0.5 * (lo + hi);
}

// Learned escape in park mode, in rounds: a transport launch walks the
// packets resumed from the last round's calls and newly admitted ones until
// each one retires or parks at a qualifying scattering; the call kernel then
// applies the parked calls in place, and those packets resume in the next
// round.  At most cap packets are in flight (new ones are admitted as others
// retire).  Once every packet is admitted and fewer than `tail` are in flight,
// one fused launch (network inside the transport kernel, a call whenever a
// scattering qualifies, as here) finishes them, so the last rounds, each a
// launch pair and a host round trip for few packets, are not run one by one.
static int run_parked(krt_ctx *c, const RunParams &P0, uint64_t n_packets, uint64_t cap, uint64_t tail, int grid,
                      int block_fused) {
    if (c->park_alloc < cap) {
        for (int k = 0; k < 2; ++k) {
            if (c->park_buf[k]) (void)hipFree(c->park_buf[k]);
            c->park_buf[k] = nullptr;
        }
        c->park_alloc = 0;
        for (int k = 0; k < 2; ++k)
            HIPCHK(c, hipMalloc(&c->park_buf[k], sizeof(uint4) * kParkQuads * cap));
        c->park_alloc = cap;
    }
    HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    uint64_t n_res = 0, new_done = 0;
    int cur = 0;
    int64_t rounds = 0;
    bool net_pending = false;
    for (;;) {
        const uint64_t admit = std::min(n_packets - new_done, cap - n_res);
        if (n_res + admit == 0) break;
        RunParams Q = P0;
        Q.res_in = c->park_buf[cur];
        Q.n_res = n_res;
        Q.new_lo = new_done;
        Q.n_packets = admit;
        HIPCHK(c, launch_zero_i64(reinterpret_cast<int64_t *>(Q.work_counter), 1, c->stream));
        ++rounds;
        if (new_done + admit == n_packets && n_res + admit <= tail) {
            Q.esc_min_lanes = 1;
            Q.esc_tail_lanes = 1;
            Q.esc_wait = 0;
            HIPCHK(c, launch_transport(Q, kModeFused, grid, block_fused, c->stream));
            break;
        }
        Q.park_out = c->park_buf[1 - cur];
        Q.park_count = c->park_counter;
        Q.park_cap = cap;
        HIPCHK(c, launch_zero_i64(reinterpret_cast<int64_t *>(c->park_counter), 1, c->stream));
        HIPCHK(c, launch_transport(Q, kModePark, grid, 1024, c->stream));
        new_done += admit;
        HIPCHK(c, hipMemcpyAsync(c->host_pinned, c->park_counter, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (net_pending) {
            float ms = 0.0f;
            HIPCHK(c, hipEventElapsedTime(&ms, c->evn0, c->evn1));
            c->last_net_ms += ms;
            net_pending = false;
        }
        const uint64_t np = (uint64_t)c->host_pinned[0];
        if (np > cap) return fail(c, KRT_EDEVICE, "park list overflow (%llu > %llu)", (unsigned long long)np,
                                  (unsigned long long)cap);
        if (np > 0) {
            const uint64_t waves = (np + 63) / 64;
            const int cgrid = (int)std::min<uint64_t>((waves + 7) / 8, (uint64_t)c->cus * 16);
            HIPCHK(c, hipEventRecord(c->evn0, c->stream));
            HIPCHK(c, launch_escape_call(Q, c->park_buf[1 - cur], np, cgrid, c->stream));
            HIPCHK(c, hipEventRecord(c->evn1, c->stream));
            net_pending = true;
        }
        cur = 1 - cur;
        n_res = np;
    }
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (net_pending) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->evn0, c->evn1));
        c->last_net_ms += ms;
    }
    c->last_rounds = rounds;
    return KRT_OK;
}

// krt_mc_run and krt_mc_run_noalloc: with noalloc the packet-pool counter and
// the bin edges live in the per-device scratch array and the edges are staged
// through a pinned block allocated at context creation, so the call allocates
// nothing (temperature classes, whose tables are built on first use, are
// refused).
static int mc_run_impl(krt_ctx *c, uint64_t n_packets, uint64_t seed, const krt_run_opts *o, krt_tallies *t,
                       bool noalloc) {
    if (!c) return KRT_EINVAL;
    if (!o || !t) return fail(c, KRT_EINVAL, "opts / tallies NULL");
    if (!c->have_grid) return fail(c, KRT_ESTATE, "no grid uploaded");
    if (c->tab.empty()) return fail(c, KRT_ESTATE, "no tables built");
    if (n_packets == 0) return fail(c, KRT_EINVAL, "n_packets must be > 0");
    if (o->line < 0 || o->line >= (int)c->tab.size() || o->line >= c->grid.n_lines)
        return fail(c, KRT_EINVAL, "line %d out of range", o->line);
    if (!t->spec_raw_dev || !t->counters_dev) return fail(c, KRT_EINVAL, "spec_raw and counters are required");
    if (!valid_bins(o->spec_nbins, o->spec_lo, o->spec_hi) || o->spec_nbins > kMaxSpecBins)
        return fail(c, KRT_EINVAL, "bad spectrum bins (1..%d bins, finite hi > lo)", kMaxSpecBins);
    if (o->source < KRT_SRC_POINT || o->source > KRT_SRC_BEAM) return fail(c, KRT_EINVAL, "bad source %d", o->source);
    if (o->src_profile < KRT_PROF_DELTA || o->src_profile > KRT_PROF_GAUSS) return fail(c, KRT_EINVAL, "bad profile");
    if (o->source == KRT_SRC_VOLUME && !c->alias_prob[o->line])
        return fail(c, KRT_EINVAL, "volume source needs emission weights for line %d", o->line);
    if (o->source == KRT_SRC_BEAM) {
        double nn = o->src_dir[0] * o->src_dir[0] + o->src_dir[1] * o->src_dir[1] + o->src_dir[2] * o->src_dir[2];
        if (!(std::fabs(nn - 1.0) < 1e-6)) return fail(c, KRT_EINVAL, "src_dir must be a unit vector");
    }
    if (o->emis_nch < 0) return fail(c, KRT_EINVAL, "emis_nch < 0");
    if (o->emis_nch > 0) {
        if (!t->emis_raw_dev) return fail(c, KRT_EINVAL, "emis_nch > 0 needs emis_raw");
        if (!valid_bins(o->emis_nch, o->ch_lo, o->ch_hi) || o->emis_nch > kMaxChannels)
            return fail(c, KRT_EINVAL, "bad channels (1..%d, finite hi > lo)", kMaxChannels);
        double nn = o->n_cam[0] * o->n_cam[0] + o->n_cam[1] * o->n_cam[1] + o->n_cam[2] * o->n_cam[2];
        if (!(std::fabs(nn - 1.0) < 1e-6)) return fail(c, KRT_EINVAL, "n_cam must be a unit vector");
    }
    if (o->jbar && !t->jbar_raw_dev) return fail(c, KRT_EINVAL, "jbar needs jbar_raw");
    int fb = o->emis_frac_bits ? o->emis_frac_bits : 20;
    if (fb < 8 || fb > 40) return fail(c, KRT_EINVAL, "emis_frac_bits %d outside 8..40", fb);
    int fj = o->jbar_frac_bits ? o->jbar_frac_bits : 36;
    if (fj < 8 || fj > 48) return fail(c, KRT_EINVAL, "jbar_frac_bits %d outside 8..48", fj);
    const double lum = (o->luminosity != 0.0) ? o->luminosity : 1.0;
    if (!(lum > 0.0) || !std::isfinite(lum)) return fail(c, KRT_EINVAL, "luminosity must be finite and > 0");
    const bool esc = o->escape_mode == 1;
    if (o->escape_mode < 0 || o->escape_mode > 1) return fail(c, KRT_EINVAL, "escape_mode %d invalid", o->escape_mode);
    if (esc) {
        if (!c->mlp_ready) return fail(c, KRT_ESTATE, "escape_mode 1 needs trained escape weights");
        if (o->jbar) return fail(c, KRT_EINVAL, "escape_mode 1 does not tally the mean intensity");
        // the network is trained on isotropic re-emission without destruction
        // or absorption: the scatterings it skips would apply neither the
        // dipole phase nor the survival probability of the skipped walk
        if (c->lines[o->line].phase != KRT_PHASE_ISO)
            return fail(c, KRT_EINVAL, "escape_mode 1 needs isotropic phase (line %d is dipole)", o->line);
        if (c->grid.eps_dev)
            return fail(c, KRT_EINVAL, "escape_mode 1 needs a grid without destruction (eps_dev is set)");
        if (c->grid.kabs_dev)
            return fail(c, KRT_EINVAL, "escape_mode 1 needs a grid without absorption (kabs_dev is set)");
        double al = c->lines[o->line].a;
        if (al < 1e-4 * (1 - 1e-9) || al > 1e-2 * (1 + 1e-9))
            return fail(c, KRT_EINVAL, "learned escape covers a in [1e-4, 1e-2] (line a = %g)", al);
        // the network is used only at damping values it was fitted on (0.01 dex of slack)
        const double la = std::log10(al);
        if (la < c->esc_la_lo - 0.01 || la > c->esc_la_hi + 0.01)
            return fail(c, KRT_EINVAL, "escape network fitted on log10 a in [%g, %g], line has %g", c->esc_la_lo,
                        c->esc_la_hi, la);
    }
    // default: one workgroup per CU holding the LDS tables, 16 waves (plain) or 8
    // waves (learned: compiled for 512-lane blocks, up to 256 VGPRs, no spills,
    // 2 waves per SIMD; on the turbulent cloud 25% faster than 768 lanes with
    // 168 VGPRs and spills)
    int block = o->wg_size ? o->wg_size : (esc ? 512 : 1024);
    int per_cu = o->wg_per_cu ? o->wg_per_cu : 1;
    // learned escape schedule: fused (default) or park; the no-allocation
    // entry point has no lists to park in
    const bool park = esc && o->esc_park && !noalloc;
    const uint64_t park_cap = o->esc_park_cap ? o->esc_park_cap : (1ull << 22);
    const uint64_t park_tail = o->esc_park_tail ? o->esc_park_tail : 65536;
    const uint32_t park_budget = o->esc_park_budget ? o->esc_park_budget : 256;
    if (park && (park_cap < 1024 || park_cap > (1ull << 28)))
        return fail(c, KRT_EINVAL, "esc_park_cap %llu outside [1024, 2^28]", (unsigned long long)park_cap);
    if (block < 64 || block > 1024 || block % 64) return fail(c, KRT_EINVAL, "wg_size %d invalid", block);
    if (per_cu < 1 || per_cu > 64) return fail(c, KRT_EINVAL, "wg_per_cu %d invalid", per_cu);
    if (o->max_events > 0xFFFFFFFEull) return fail(c, KRT_EINVAL, "max_events too large");
    if (o->profile_mode < 0 || o->profile_mode > 2) return fail(c, KRT_EINVAL, "profile_mode %d", o->profile_mode);
    if (o->profile_mode != 0 && esc) return fail(c, KRT_EINVAL, "profile_mode %d is for the plain walk", o->profile_mode);
    if (c->have_grid && c->grid.tclass_dev && (esc || o->profile_mode != 0))
        return fail(c, KRT_EINVAL, "temperature classes need the plain walk with profile_mode 0");
    if (c->have_grid && c->grid.bratio_dev && (esc || o->profile_mode != 0))
        return fail(c, KRT_EINVAL, "per-cell widths (bratio) need the plain walk with profile_mode 0");

    HIPCHK(c, hipSetDevice(c->device));
    const krt_grid_desc &g = c->grid;
    const int64_t nc = c->ncell;
    const int l = o->line;
    const int nsb = o->spec_nbins + 2;
    if (!o->accumulate) {
        HIPCHK(c, launch_zero_i64(t->spec_raw_dev, nsb, c->stream));
        HIPCHK(c, launch_zero_i64(t->counters_dev, KRT_NCOUNTERS, c->stream));
        if (o->emis_nch > 0) HIPCHK(c, launch_zero_i64(t->emis_raw_dev, nc * o->emis_nch, c->stream));
        if (o->jbar) HIPCHK(c, launch_zero_i64(t->jbar_raw_dev, nc, c->stream));
    }
    if (noalloc && (c->grid.tclass_dev || c->grid.bratio_dev))
        return fail(c, KRT_EINVAL, "krt_mc_run_noalloc: per-cell temperatures build their tables on first use; "
                                   "use krt_mc_run");
    unsigned long long *counter = noalloc ? reinterpret_cast<unsigned long long *>(c->scratch_dev) : c->work_counter;
    float *edges = noalloc ? reinterpret_cast<float *>(c->scratch_dev + kNoAllocEdgeOffset) : c->edges;
    HIPCHK(c, launch_zero_i64(reinterpret_cast<int64_t *>(counter), 1, c->stream));

    RunParams P;
    std::memset(&P, 0, sizeof(P));
    for (int k = 0; k < 3; ++k) {
        P.n[k] = g.n[k];
        P.lo[k] = g.lo[k];
        P.hi[k] = g.hi[k];
        P.dxd[k] = (g.hi[k] - g.lo[k]) / g.n[k];
        P.dx[k] = (float)P.dxd[k];
        P.inv_dx[k] = (float)(1.0 / P.dxd[k]);
        P.bc[k] = g.bc[k];
        P.src_pos[k] = o->src_pos[k];
        P.src_dir[k] = (float)o->src_dir[k];
        P.n_cam[k] = (float)o->n_cam[k];
    }
    P.ncell = (int)nc;
    P.k0 = g.k0_dev + (int64_t)l * nc;
    if (g.vel_dev) { P.vx = g.vel_dev; P.vy = g.vel_dev + nc; P.vz = g.vel_dev + 2 * nc; }
    P.eps = g.eps_dev ? g.eps_dev + (int64_t)l * nc : nullptr;
    P.kabs = g.kabs_dev;
    P.alias_prob = c->alias_prob[l];
    P.alias_idx = c->alias_idx[l];
    P.tab = c->tab[l];
    P.a = (float)c->lines[l].a;
    P.thd = (float)std::atan(kDelta / c->lines[l].a);
    P.phase = c->lines[l].phase;
    P.source = o->source;
    P.src_profile = o->src_profile;
    P.src_x0 = (float)o->src_x0;
    if (noalloc) {
        // the pinned block is reused only after this call's stream synchronisation
        float *e = c->host_edges;
        for (int k = 0; k < kEdgeFloats; ++k) e[k] = 0.0f;
        fill_edges(e, o->spec_nbins, o->spec_lo, o->spec_hi);
        if (o->emis_nch > 0) fill_edges(e + kMaxSpecBins + 1, o->emis_nch, o->ch_lo, o->ch_hi);
        HIPCHK(c, hipMemcpyAsync(edges, e, sizeof(float) * kEdgeFloats, hipMemcpyHostToDevice, c->stream));
    } else {
        std::vector<float> e(kEdgeFloats, 0.0f);
        fill_edges(e.data(), o->spec_nbins, o->spec_lo, o->spec_hi);
        if (o->emis_nch > 0) fill_edges(e.data() + kMaxSpecBins + 1, o->emis_nch, o->ch_lo, o->ch_hi);
        HIPCHK(c, hipMemcpyAsync(edges, e.data(), sizeof(float) * kEdgeFloats, hipMemcpyHostToDevice, c->stream));
    }
    P.spec_nb = o->spec_nbins;
    P.spec_inv_w = (float)(o->spec_nbins / (o->spec_hi - o->spec_lo));
    P.spec_edges = edges;
    P.emis_nch = o->emis_nch;
    P.ch_inv_w = o->emis_nch > 0 ? (float)(o->emis_nch / (o->ch_hi - o->ch_lo)) : 0.0f;
    P.ch_edges = edges + kMaxSpecBins + 1;
    P.frac_scale = std::ldexp(1.0f, fb);
    P.emis_w32 = fb <= 30 ? 1 : 0;
    P.jbar_scale = std::ldexp(1.0f, fj);
    P.spec_raw = t->spec_raw_dev;
    P.emis_raw = o->emis_nch > 0 ? t->emis_raw_dev : nullptr;
    P.jbar_raw = o->jbar ? t->jbar_raw_dev : nullptr;
    P.counters = t->counters_dev;
    P.status = reinterpret_cast<uint32_t *>(t->counters_dev + KRT_C_STATUS);
    P.plog = t->packet_log_dev;
    P.n_packets = n_packets;
    P.packet_offset = o->packet_offset;
    P.max_events = o->max_events ? o->max_events : 0xFFFFFFFEull;
    P.key0 = (uint32_t)seed;
    P.key1 = (uint32_t)(seed >> 32);
    P.work_counter = counter;
    P.mlp_img = esc ? c->mlp_img : nullptr;
    // whole-cell calls: cubic cells only, inside the records' ranges of the cell
    // depth tau_c and of the depth of the scattering point below the nearest face
    P.esc_cubic = (std::fabs(P.dxd[1] - P.dxd[0]) <= 1e-6 * P.dxd[0] &&
                   std::fabs(P.dxd[2] - P.dxd[0]) <= 1e-6 * P.dxd[0]) ? 1 : 0;
    P.esc_half_dx = (float)(0.5 * P.dxd[0]);
    P.esc_tc_min = (float)std::max(0.5 * (o->esc_cell_tau_min > 0.0 ? o->esc_cell_tau_min : 100.0),
                                   std::pow(10.0, (double)c->esc_lt_lo));
    P.esc_tc_max = (float)std::pow(10.0, (double)c->esc_lt_hi);
    P.esc_depth_min = (float)std::max(o->esc_tau_min > 0.0 ? o->esc_tau_min : 3.0,
                                      std::pow(10.0, (double)c->esc_ld_min));
    P.esc_x_max = kEscXMax;
    P.esc_log10a = (float)std::log10(c->lines[l].a);
    P.esc_min_lanes = o->esc_min_lanes > 0 ? o->esc_min_lanes : 16;
    P.esc_tail_lanes = o->esc_tail_lanes > 0 ? o->esc_tail_lanes : 1;
    P.esc_wait = o->esc_wait > 0 ? (uint32_t)o->esc_wait : (o->esc_wait == 0 ? 32u : 0u);
    P.tail_lanes = o->tail_lanes == 0 ? 32 : (o->tail_lanes < 0 ? 0 : std::min(o->tail_lanes, 64));
    P.profile_mode = o->profile_mode;
    P.tclass = nullptr;
    P.cls_par = nullptr;
    P.cls_tab = nullptr;
    if (c->grid.tclass_dev) {
        int rc = ensure_class_tables(c, l);
        if (rc) return rc;
        P.tclass = c->grid.tclass_dev;
        P.cls_par = c->cls_par;
        P.cls_tab = c->cls_tab;
    }
    P.bratio = nullptr;
    if (c->grid.bratio_dev) {
        int rc = ensure_cont_tables(c, l);
        if (rc) return rc;
        set_cont_params(c, P);
    }
    P.voigt_u0 = (float)voigt_crossing(c->lines[l].a);
    P.n_res = 0;
    P.new_lo = 0;
    P.park_budget = park_budget;
    int grid = c->cus * per_cu;
    c->last_net_ms = 0.0f;
    c->last_rounds = 1;
    if (!park) {
        HIPCHK(c, hipEventRecord(c->ev0, c->stream));
        HIPCHK(c, launch_transport(P, esc ? kModeFused : kModePlain, grid, block, c->stream));
        HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    } else {
        int rc = run_parked(c, P, n_packets, park_cap, park_tail, grid, block);
        if (rc) return rc;
    }
    // integer tallies that left [0, 2^62] (the transport's atomics return nothing)
    HIPCHK(c, launch_saturation_check(t->spec_raw_dev, nsb, P.status, c->stream));
    if (o->emis_nch > 0) HIPCHK(c, launch_saturation_check(t->emis_raw_dev, nc * o->emis_nch, P.status, c->stream));
    if (o->jbar) HIPCHK(c, launch_saturation_check(t->jbar_raw_dev, nc, P.status, c->stream));

    // finalise (FP64 scaling -> FP32)
    const double N = (double)(o->norm_packets ? o->norm_packets : n_packets);
    const double vcell = P.dxd[0] * P.dxd[1] * P.dxd[2];
    const double inv_f = std::ldexp(1.0, -fb), inv_fj = std::ldexp(1.0, -fj);
    const double four_pi = 4.0 * 3.14159265358979323846;
    if (t->spec_dev)
        HIPCHK(c, launch_finalize(t->spec_raw_dev, t->spec_dev, nsb, lum / (N * (o->spec_hi - o->spec_lo) / o->spec_nbins), c->stream));
    if (t->emis_dev && o->emis_nch > 0)
        HIPCHK(c, launch_finalize(t->emis_raw_dev, t->emis_dev, nc * o->emis_nch,
                                  lum * inv_f / (four_pi * N * vcell * ((o->ch_hi - o->ch_lo) / o->emis_nch)), c->stream));
    if (t->jbar_dev && o->jbar)
        HIPCHK(c, launch_finalize(t->jbar_raw_dev, t->jbar_dev, nc, lum * inv_fj / (four_pi * N * vcell), c->stream));

    HIPCHK(c, hipMemcpyAsync(c->host_pinned, t->counters_dev, sizeof(int64_t) * KRT_NCOUNTERS,
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipEventElapsedTime(&c->last_ms, c->ev0, c->ev1));
    int64_t st = c->host_pinned[KRT_C_STATUS];
    if (st != 0) return fail(c, KRT_EDEVICE, "device status 0x%llx (nan=1 stuck=2 saturate=4)", (long long)st);
    return KRT_OK;
}

extern "C" int krt_mc_run(krt_ctx *c, uint64_t n_packets, uint64_t seed, const krt_run_opts *o,
                          krt_tallies *t) {
    return mc_run_impl(c, n_packets, seed, o, t, false);
}

extern "C" int krt_mc_run_noalloc(krt_ctx *c, uint64_t n_packets, uint64_t seed, const krt_run_opts *o,
                                  krt_tallies *t) {
    if (o && (o->spec_nbins > kMaxSpecBins || o->emis_nch > kMaxChannels))
        return fail(c, KRT_EINVAL, "krt_mc_run_noalloc: the %zu-byte scratch holds at most %d spectrum bins and %d "
                                   "channels", kNoAllocScratchBytes, kMaxSpecBins, kMaxChannels);
    return mc_run_impl(c, n_packets, seed, o, t, true);
}

// -------------------------------------------------------------- imaging ---
extern "C" int krt_image(krt_ctx *c, const krt_image_desc *d) {
    if (!c) return KRT_EINVAL;
    if (!d) return fail(c, KRT_EINVAL, "image desc NULL");
    if (!c->have_grid) return fail(c, KRT_ESTATE, "no grid uploaded");
    if (d->line < 0 || d->line >= (int)c->tab.size() || d->line >= c->grid.n_lines)
        return fail(c, KRT_ESTATE, "line %d has no tables or no opacity slice", d->line);
    if (d->axis < 0 || d->axis > 5) return fail(c, KRT_EINVAL, "axis %d outside 0..5", d->axis);
    if (d->nch < 1 || d->nch > 256) return fail(c, KRT_EINVAL, "nch %d outside 1..256", d->nch);
    if (!(d->ch_hi > d->ch_lo)) return fail(c, KRT_EINVAL, "empty channel range");
    if (!d->emis_dev || !d->image_dev) return fail(c, KRT_EINVAL, "image desc has NULL arrays");
    const krt_grid_desc &g = c->grid;
    ImageParams Q{};
    Q.d = d->axis % 3;
    Q.sgn = d->axis < 3 ? 1 : -1;
    Q.sgnf = (float)Q.sgn;
    for (int k = 0; k < 3; ++k) Q.n[k] = g.n[k];
    Q.dl = (float)((g.hi[Q.d] - g.lo[Q.d]) / g.n[Q.d]);
    if (Q.d == 0) { Q.n0 = g.n[1]; Q.npix = (int64_t)g.n[1] * g.n[2]; Q.stride = 1; }
    else if (Q.d == 1) { Q.n0 = g.n[0]; Q.npix = (int64_t)g.n[0] * g.n[2]; Q.stride = g.n[0]; }
    else { Q.n0 = g.n[0]; Q.npix = (int64_t)g.n[0] * g.n[1]; Q.stride = (int64_t)g.n[0] * g.n[1]; }
    Q.nch = d->nch;
    // one launch covers every (pixel, channel) pair with a work-item (a few
    // more when rays are cut into segments, which happens only for small images)
    if (Q.npix * (int64_t)Q.nch > (int64_t(1) << 31))
        return fail(c, KRT_EINVAL, "image of %lld pixels x %d channels exceeds 2^31 (pixel, channel) pairs",
                    (long long)Q.npix, Q.nch);
    Q.ch_lo = (float)d->ch_lo;
    Q.ch_w = (float)((d->ch_hi - d->ch_lo) / d->nch);
    Q.tab = c->tab[d->line];
    Q.k0 = g.k0_dev + (int64_t)d->line * c->ncell;
    Q.vel_axis = g.vel_dev ? g.vel_dev + (int64_t)Q.d * c->ncell : nullptr;
    Q.emis = d->emis_dev;
    Q.srcf = d->src_dev;
    Q.kabs = d->kabs_dev;
    Q.out = d->image_dev;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_image_timed(Q, c->stream, c->ev0, c->ev1));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipEventElapsedTime(&c->last_image_ms, c->ev0, c->ev1));
    return KRT_OK;
}

extern "C" float krt_last_image_ms(const krt_ctx *c) { return c ? c->last_image_ms : -1.0f; }

// --------------------------------------------------------------- levels ---
// Per-cell rate matrix, FP64 Gaussian elimination with partial pivoting.
// consts: E[nl] g[nl] A[nl*nl] Cd[nl*nl] sigma0[nl-1]
// The level count is a template argument: every index into the matrices is
// then a compile-time constant after unrolling (the pivot row is swapped by
// selects over the candidate rows), so they live in registers; a run-time
// count would index them dynamically and put them in scratch memory.
template <int NL>
__global__ void __launch_bounds__(256) levels_kernel(int64_t ncell, const double *K, const double *ncoll,
                                                     const double *ntot, const float *jbar, double *pops,
                                                     float *k0_out, float *eps_out, float *emis_out) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const double *E = K, *g = K + NL, *A = K + 2 * NL, *Cd = K + 2 * NL + NL * NL, *s0 = K + 2 * NL + 2 * NL * NL;
    double R[NL][NL], M[NL][NL], b[NL];
    const double nc = ncoll[c];
#pragma unroll
    for (int i = 0; i < NL; ++i)
#pragma unroll
        for (int j = 0; j < NL; ++j) R[i][j] = 0.0;
#pragma unroll
    for (int u = 1; u < NL; ++u)
#pragma unroll
        for (int l = 0; l < u; ++l) {
            double cd = Cd[u * NL + l] * nc;
            double cu = cd * (g[u] / g[l]) * exp(-(E[u] - E[l]));
            R[u][l] += A[u * NL + l] + cd;
            R[l][u] += cu;
        }
    const double kGam = 4.0 * 3.14159265358979323846 * 1.77245385090551602730;
    if (jbar) {
#pragma unroll
        for (int l = 0; l + 1 < NL; ++l) {
            double G = kGam * s0[l] * (double)jbar[(int64_t)l * ncell + c];
            R[l][l + 1] += G;
            R[l + 1][l] += (g[l] / g[l + 1]) * G;
        }
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        double out = 0.0;
#pragma unroll
        for (int j = 0; j < NL; ++j) {
            M[i][j] = (j != i) ? R[j][i] : 0.0;
            if (j != i) out += R[i][j];
        }
        M[i][i] = -out;
        b[i] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < NL; ++j) M[NL - 1][j] = 1.0;
    b[NL - 1] = ntot[c];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        int p = k;
        double mx = fabs(M[k][k]);
#pragma unroll
        for (int i = k + 1; i < NL; ++i) if (fabs(M[i][k]) > mx) { mx = fabs(M[i][k]); p = i; }
#pragma unroll
        for (int i = k + 1; i < NL; ++i) {
            const bool sw = (i == p);
#pragma unroll
            for (int j = 0; j < NL; ++j) {
                const double t = M[k][j];
                M[k][j] = sw ? M[i][j] : t;
                M[i][j] = sw ? t : M[i][j];
            }
            const double t = b[k];
            b[k] = sw ? b[i] : t;
            b[i] = sw ? t : b[i];
        }
#pragma unroll
        for (int i = k + 1; i < NL; ++i) {
            double f = M[i][k] / M[k][k];
#pragma unroll
            for (int j = k; j < NL; ++j) M[i][j] -= f * M[k][j];
            b[i] -= f * b[k];
        }
    }
#pragma unroll
    for (int i = NL - 1; i >= 0; --i) {
        double s = b[i];
#pragma unroll
        for (int j = i + 1; j < NL; ++j) s -= M[i][j] * b[j];
        b[i] = s / M[i][i];
    }
#pragma unroll
    for (int i = 0; i < NL; ++i) pops[c * NL + i] = b[i];
#pragma unroll
    for (int l = 0; l + 1 < NL; ++l) {
        int u = l + 1;
        if (k0_out) k0_out[(int64_t)l * ncell + c] = (float)(b[l] * s0[l]);
        // spontaneous emission of the line per unit volume, n_u A_ul (the
        // Lambda iteration's source)
        if (emis_out) emis_out[(int64_t)l * ncell + c] = (float)(b[u] * A[u * NL + l]);
        if (eps_out) {
            double ctot = 0.0;
#pragma unroll
            for (int j = 0; j < NL; ++j) if (j != u) {
                double cd = (j < u) ? Cd[u * NL + j] * nc : Cd[j * NL + u] * nc * (g[j] / g[u]) * exp(-(E[j] - E[u]));
                ctot += cd;
            }
            eps_out[(int64_t)l * ncell + c] = (float)(ctot / (A[u * NL + l] + ctot));
        }
    }
}

template <int NL>
static void launch_levels_t(int64_t ncell, const double *consts, const double *ncoll, const double *ntot,
                            const float *jbar, double *pops, float *k0_out, float *eps_out, float *emis_out,
                            hipStream_t s) {
    int grid = (int)((ncell + 255) / 256);
    hipLaunchKernelGGL(levels_kernel<NL>, dim3(grid), dim3(256), 0, s, ncell, consts, ncoll, ntot, jbar, pops,
                       k0_out, eps_out, emis_out);
}

hipError_t krt::launch_levels(int nl, int64_t ncell, const double *consts, const double *ncoll,
                              const double *ntot, const float *jbar, double *pops, float *k0_out,
                              float *eps_out, float *emis_out, hipStream_t s) {
    switch (nl) {
        case 2: launch_levels_t<2>(ncell, consts, ncoll, ntot, jbar, pops, k0_out, eps_out, emis_out, s); break;
        case 3: launch_levels_t<3>(ncell, consts, ncoll, ntot, jbar, pops, k0_out, eps_out, emis_out, s); break;
        case 4: launch_levels_t<4>(ncell, consts, ncoll, ntot, jbar, pops, k0_out, eps_out, emis_out, s); break;
        case 5: launch_levels_t<5>(ncell, consts, ncoll, ntot, jbar, pops, k0_out, eps_out, emis_out, s); break;
        case 6: launch_levels_t<6>(ncell, consts, ncoll, ntot, jbar, pops, k0_out, eps_out, emis_out, s); break;
        case 7: launch_levels_t<7>(ncell, consts, ncoll, ntot, jbar, pops, k0_out, eps_out, emis_out, s); break;
        case 8: launch_levels_t<8>(ncell, consts, ncoll, ntot, jbar, pops, k0_out, eps_out, emis_out, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Line powers: sum over cells of n_u A_ul for each line, FP64, deterministic
// (per-block partial sums over fixed cell ranges, then a fixed-order sum).
constexpr int kPowBlocks = 256;
__global__ void __launch_bounds__(256) line_power_partial_kernel(int nl, int64_t ncell, const double *K,
                                                                 const double *pops, double *partial) {
    __shared__ double red[256];
    const int line = blockIdx.y;
    const int u = line + 1;
    const double A_ul = K[2 * nl + u * nl + line];
    const int64_t c0 = ncell * blockIdx.x / kPowBlocks, c1 = ncell * (blockIdx.x + 1) / kPowBlocks;
    double acc = 0.0;
    for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) acc += pops[c * nl + u] * A_ul;
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st >= 1; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[line * kPowBlocks + blockIdx.x] = red[0];
}

__global__ void line_power_final_kernel(int nlines, const double *partial, double *out) {
    const int line = threadIdx.x;
    if (line >= nlines) return;
    double s = 0.0;
    for (int b = 0; b < kPowBlocks; ++b) s += partial[line * kPowBlocks + b];
    out[line] = s;
}

extern "C" int krt_levels_update(krt_ctx *c, const krt_levels_desc *d, const float *jbar_dev) {
    if (!c) return KRT_EINVAL;
    if (!d) return fail(c, KRT_EINVAL, "levels desc NULL");
    const int nl = d->n_levels;
    if (nl < 2 || nl > 8) return fail(c, KRT_EINVAL, "n_levels %d outside 2..8", nl);
    if (d->ncell < 1 || d->ncell >= (int64_t(1) << 31)) return fail(c, KRT_EINVAL, "levels ncell %lld", (long long)d->ncell);
    if (!d->E || !d->g || !d->A || !d->Cd || !d->sigma0 || !d->ncoll_dev || !d->ntot_dev || !d->pops_dev)
        return fail(c, KRT_EINVAL, "levels desc has NULL arrays");
    std::vector<double> K;
    K.insert(K.end(), d->E, d->E + nl);
    K.insert(K.end(), d->g, d->g + nl);
    K.insert(K.end(), d->A, d->A + nl * nl);
    K.insert(K.end(), d->Cd, d->Cd + nl * nl);
    K.insert(K.end(), d->sigma0, d->sigma0 + (nl - 1));
    for (double v : K) if (!std::isfinite(v)) return fail(c, KRT_EINVAL, "non-finite level constant");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(c->level_consts, K.data(), sizeof(double) * K.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_levels(nl, d->ncell, c->level_consts, d->ncoll_dev, d->ntot_dev, jbar_dev, d->pops_dev,
                            d->k0_out_dev, d->eps_out_dev, d->emis_out_dev, c->stream));
    if (d->lum_out) {
        if (!(d->cell_volume > 0.0) || !std::isfinite(d->cell_volume))
            return fail(c, KRT_EINVAL, "lum_out needs a finite cell_volume > 0");
        if (!c->level_power) HIPCHK(c, hipMalloc(&c->level_power, sizeof(double) * 8 * (kPowBlocks + 1)));
        double *partial = c->level_power, *sums = c->level_power + 8 * kPowBlocks;
        hipLaunchKernelGGL(line_power_partial_kernel, dim3(kPowBlocks, nl - 1), dim3(256), 0, c->stream, nl,
                           (int64_t)d->ncell, (const double *)c->level_consts, (const double *)d->pops_dev, partial);
        HIPCHK(c, hipGetLastError());
        hipLaunchKernelGGL(line_power_final_kernel, dim3(1), dim3(64), 0, c->stream, nl - 1, (const double *)partial,
                           sums);
        HIPCHK(c, hipGetLastError());
        double host[8];
        HIPCHK(c, hipMemcpyAsync(host, sums, sizeof(double) * (nl - 1), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int l = 0; l + 1 < nl; ++l) d->lum_out[l] = host[l] * d->cell_volume;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KRT_OK;
}

// ----------------------------------------------------------- diagnostics ---
// The diagnostics launch one work-item per element: at most 2^31 of them
// keeps a launch within the 2^32 work-items of a grid dimension.
constexpr int64_t kMaxDebugElems = int64_t(1) << 31;

extern "C" int krt_debug_philox(krt_ctx *c, const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n) {
    if (!c) return KRT_EINVAL;
    if (!ctr || !key || !out || n <= 0 || n > kMaxDebugElems) return fail(c, KRT_EINVAL, "bad philox args");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_debug_philox(ctr, key, out, n, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KRT_OK;
}

extern "C" int krt_debug_bins(krt_ctx *c, const float *x, int64_t n, int32_t nb, double lo, double hi, int32_t *out) {
    if (!c) return KRT_EINVAL;
    if (!x || !out || n <= 0 || n > kMaxDebugElems || !valid_bins(nb, lo, hi) || nb > kMaxSpecBins)
        return fail(c, KRT_EINVAL, "bad bins args");
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<float> e(nb + 1);
    fill_edges(e.data(), nb, lo, hi);
    HIPCHK(c, hipMemcpyAsync(c->edges, e.data(), sizeof(float) * (nb + 1), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_debug_bins(x, n, nb, c->edges, (float)(nb / (hi - lo)), out, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KRT_OK;
}

extern "C" int krt_debug_voigt_analytic(krt_ctx *c, double a, const float *x, int64_t n, float *out) {
    if (!c) return KRT_EINVAL;
    if (!x || !out || n <= 0 || n > kMaxDebugElems || !(a > 0.0 && a < 1.0)) return fail(c, KRT_EINVAL, "bad voigt args");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_debug_voigt_analytic((float)a, (float)voigt_crossing(a), x, n, out, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KRT_OK;
}

extern "C" int krt_debug_voigt(krt_ctx *c, int32_t line, const float *x, int64_t n, float *out) {
    if (!c) return KRT_EINVAL;
    if (line < 0 || line >= (int)c->tab.size()) return fail(c, KRT_ESTATE, "line %d has no tables", line);
    if (!x || !out || n <= 0 || n > kMaxDebugElems) return fail(c, KRT_EINVAL, "bad voigt args");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_debug_voigt(c->tab[line], x, n, out, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KRT_OK;
}

extern "C" int krt_debug_voigt_cont(krt_ctx *c, int32_t line, const float *r, const float *x, int64_t n, float *out) {
    if (!c) return KRT_EINVAL;
    if (line < 0 || line >= (int)c->tab.size()) return fail(c, KRT_ESTATE, "line %d has no tables", line);
    if (!c->have_grid || !c->grid.bratio_dev) return fail(c, KRT_ESTATE, "the grid has no per-cell widths (bratio)");
    if (!r || !x || !out || n <= 0 || n > kMaxDebugElems) return fail(c, KRT_EINVAL, "bad voigt_cont args");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = ensure_cont_tables(c, line);
    if (rc) return rc;
    RunParams P;
    std::memset(&P, 0, sizeof(P));
    set_cont_params(c, P);
    HIPCHK(c, launch_debug_voigt_cont(P, (float)c->lines[line].a, r, x, n, out, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KRT_OK;
}

extern "C" int krt_debug_upar(krt_ctx *c, int32_t line, float x, uint64_t seed, uint64_t packet, uint32_t ev0,
                              int64_t n, float *out) {
    if (!c) return KRT_EINVAL;
    if (line < 0 || line >= (int)c->tab.size()) return fail(c, KRT_ESTATE, "line %d has no tables", line);
    if (!out || n <= 0 || n > kMaxDebugElems || !std::isfinite(x)) return fail(c, KRT_EINVAL, "bad upar args");
    HIPCHK(c, hipSetDevice(c->device));
    float a = (float)c->lines[line].a, thd = (float)std::atan(kDelta / c->lines[line].a);
    HIPCHK(c, launch_debug_upar(c->tab[line], a, thd, x, (uint32_t)seed, (uint32_t)(seed >> 32), packet, ev0, n,
                                out, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KRT_OK;
}

// ------------------------------------------------------- learned escape ---
namespace {
int mlp_alloc(krt_ctx *c) {
    if (c->mlp_p) return KRT_OK;
    HIPCHK(c, hipMalloc(&c->mlp_p, sizeof(float) * kNParams));
    HIPCHK(c, hipMalloc(&c->mlp_m, sizeof(float) * kNParams));
    HIPCHK(c, hipMalloc(&c->mlp_calsum, sizeof(double) * 3 * kNCal));
    HIPCHK(c, hipMalloc(&c->mlp_v, sizeof(float) * kNParams));
    HIPCHK(c, hipMalloc(&c->mlp_g, sizeof(float) * kNParams));
    HIPCHK(c, hipMalloc(&c->mlp_part, sizeof(float) * kNParams * kGradSplits));
    HIPCHK(c, hipMalloc(&c->mlp_norm, sizeof(float) * kNNorm));
    HIPCHK(c, hipMalloc(&c->mlp_loss, sizeof(float) * 2));
    HIPCHK(c, hipMalloc(&c->mlp_blob, kMlpBlobBytes));
    HIPCHK(c, hipMalloc(&c->mlp_img, kMlpFwdBytes));
    return KRT_OK;
}

int mlp_zero_state(krt_ctx *c) {
    HIPCHK(c, launch_zero_i64(reinterpret_cast<int64_t *>(c->mlp_m), kNParams / 2, c->stream));
    HIPCHK(c, launch_zero_i64(reinterpret_cast<int64_t *>(c->mlp_v), kNParams / 2, c->stream));
    c->mlp_step = 0;
    return KRT_OK;
}

// batch buffers: indices, levels [batch][5] and the activation store with
// room for the batch rounded up to 32 samples
int mlp_ensure_batch(krt_ctx *c, int batch) {
    if (batch <= c->mlp_batch_cap) return KRT_OK;
    for (void *p : {(void *)c->mlp_idx, (void *)c->mlp_u, (void *)c->mlp_act})
        if (p) (void)hipFree(p);
    c->mlp_idx = nullptr;
    c->mlp_u = nullptr;
    c->mlp_act = nullptr;
    c->mlp_batch_cap = 0;
    const int64_t cap = 32 * (((int64_t)batch + 31) / 32);
    HIPCHK(c, hipMalloc(&c->mlp_idx, sizeof(int32_t) * batch));
    HIPCHK(c, hipMalloc(&c->mlp_u, sizeof(float) * 5 * (size_t)batch));
    HIPCHK(c, hipMalloc(&c->mlp_act, sizeof(uint16_t) * (size_t)kActRowsAll * cap));
    HIPCHK(c, launch_mlp_act_init(c->mlp_act, cap, c->stream));
    c->mlp_act_cap = cap;
    c->mlp_batch_cap = batch;
    return KRT_OK;
}
}  // namespace

static_assert(kNParams % 2 == 0, "parameter count is even (zeroed as int64 pairs)");

// Host copy of the log10 a range stored in the normalisation block (after a
// fit or a weight upload); synchronises the library stream.
static int read_a_range(krt_ctx *c) {
    float r[5];
    HIPCHK(c, hipMemcpyAsync(r, c->mlp_norm + kNormARange, sizeof(r), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->esc_la_lo = r[0];
    c->esc_la_hi = r[1];
    c->esc_lt_lo = r[2];
    c->esc_lt_hi = r[3];
    c->esc_ld_min = r[4];
    return KRT_OK;
}

extern "C" int krt_escape_init(krt_ctx *c, uint64_t seed) {
    if (!c) return KRT_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    int rc = mlp_alloc(c);
    if (rc) return rc;
    HIPCHK(c, launch_mlp_init(c->mlp_p, (uint32_t)seed, (uint32_t)(seed >> 32), c->stream));
    rc = mlp_zero_state(c);
    if (rc) return rc;
    float norm[kNNorm];
    for (int k = 0; k < kNNorm; ++k) norm[k] = 0.0f;
    for (int k = 0; k < kMlpOut; ++k) norm[kMlpOut + k] = 1.0f;
    norm[kNormARange] = 1.0f;  // empty ranges until krt_escape_fit_norm
    norm[kNormARange + 1] = -1.0f;
    norm[kNormTauRange] = 1.0f;
    norm[kNormTauRange + 1] = -1.0f;
    c->esc_la_lo = 1.0f;
    c->esc_la_hi = -1.0f;
    c->esc_lt_lo = 1.0f;
    c->esc_lt_hi = -1.0f;
    c->esc_ld_min = 0.0f;
    HIPCHK(c, hipMemcpyAsync(c->mlp_norm, norm, sizeof(norm), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_mlp_pack(c->mlp_p, c->mlp_norm, c->mlp_blob, c->mlp_img, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->mlp_ready = true;
    return KRT_OK;
}

extern "C" int krt_escape_record(krt_ctx *c, int32_t line, uint64_t n, uint64_t seed, uint64_t offset,
                                 const krt_escape_cond *cond, float *samples_dev) {
    if (!c) return KRT_EINVAL;
    if (line < 0 || line >= (int)c->tab.size()) return fail(c, KRT_ESTATE, "line %d has no tables", line);
    if (!samples_dev || !cond || n == 0 || n > (1ull << 31)) return fail(c, KRT_EINVAL, "bad record args");
    if (!(cond->log10_tau_hi >= cond->log10_tau_lo) || cond->log10_tau_lo < 0.0 || cond->log10_tau_hi > 6.0)
        return fail(c, KRT_EINVAL, "log10 tau_c range must lie in [0, 6]");
    if (!(cond->log10_depth_lo >= -2.0 && cond->log10_depth_lo <= 6.0))
        return fail(c, KRT_EINVAL, "log10_depth_lo outside [-2, 6]");
    if (cond->fixed) {
        const double *q = cond->q;
        if (!(q[0] >= 0.0 && q[0] <= q[1] && q[1] <= q[2] && q[2] < 1.0))
            return fail(c, KRT_EINVAL, "fixed start needs 0 <= q0 <= q1 <= q2 < 1");
        if (!(cond->x_in >= 0.0 && cond->x_in <= 50.0)) return fail(c, KRT_EINVAL, "fixed x_in outside [0, 50]");
        const double nn = cond->n_in[0] * cond->n_in[0] + cond->n_in[1] * cond->n_in[1] + cond->n_in[2] * cond->n_in[2];
        if (!cond->iso_dir && !(std::fabs(nn - 1.0) < 1e-6)) return fail(c, KRT_EINVAL, "n_in must be a unit vector");
    }
    HIPCHK(c, hipSetDevice(c->device));
    RecordParams R{};
    R.tab = c->tab[line];
    R.a = (float)c->lines[line].a;
    R.thd = (float)std::atan(kDelta / c->lines[line].a);
    R.k0 = (uint32_t)seed;
    R.k1 = (uint32_t)(seed >> 32);
    R.offset = offset;
    R.n = n;
    R.lt_lo = (float)cond->log10_tau_lo;
    R.lt_hi = (float)cond->log10_tau_hi;
    R.ld_lo = (float)cond->log10_depth_lo;
    R.max_scat = 20000000u;
    R.fixed = cond->fixed ? 1 : 0;
    R.iso_dir = cond->iso_dir ? 1 : 0;
    R.x_in = (float)cond->x_in;
    for (int k = 0; k < 3; ++k) { R.q[k] = (float)cond->q[k]; R.n_in[k] = (float)cond->n_in[k]; }
    R.counter = c->work_counter;
    R.out = samples_dev;
    HIPCHK(c, launch_zero_i64(reinterpret_cast<int64_t *>(c->work_counter), 1, c->stream));
    HIPCHK(c, launch_cell_record(R, 4 * c->cus, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KRT_OK;
}

extern "C" int krt_escape_fit_norm(krt_ctx *c, const float *samples_dev, uint64_t n) {
    if (!c) return KRT_EINVAL;
    if (!c->mlp_ready) return fail(c, KRT_ESTATE, "call krt_escape_init first");
    if (!samples_dev || n == 0) return fail(c, KRT_EINVAL, "bad norm args");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_mlp_norm(samples_dev, (int64_t)n, c->mlp_norm, c->stream));
    // a new normalisation invalidates the calibration of ln E[N_s]
    static_assert(kNormCal % 2 == 0 && kNCal % 2 == 0, "calibration block is int64-aligned");
    HIPCHK(c, launch_zero_i64(reinterpret_cast<int64_t *>(c->mlp_norm + kNormCal), kNCal / 2, c->stream));
    HIPCHK(c, launch_mlp_pack(c->mlp_p, c->mlp_norm, c->mlp_blob, c->mlp_img, c->stream));
    return read_a_range(c);
}

extern "C" int krt_escape_calibrate(krt_ctx *c, const float *samples_dev, uint64_t n) {
    if (!c) return KRT_EINVAL;
    if (!c->mlp_ready) return fail(c, KRT_ESTATE, "call krt_escape_init first");
    if (!samples_dev || n == 0 || n >= (1ull << 30))  // four work-items per record
        return fail(c, KRT_EINVAL, "bad calibration args");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_zero_i64(reinterpret_cast<int64_t *>(c->mlp_calsum), 3 * kNCal, c->stream));
    HIPCHK(c, launch_mlp_calib(c->mlp_blob, samples_dev, (int64_t)n, c->mlp_calsum, c->mlp_norm, c->stream));
    HIPCHK(c, launch_mlp_pack(c->mlp_p, c->mlp_norm, c->mlp_blob, c->mlp_img, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KRT_OK;
}

extern "C" int krt_escape_grad(krt_ctx *c, const float *samples_dev, const int32_t *idx_dev, const float *u_dev,
                               int32_t batch, float *grad_out_dev, float *loss_out_dev) {
    if (!c) return KRT_EINVAL;
    if (!c->mlp_ready) return fail(c, KRT_ESTATE, "call krt_escape_init first");
    if (!samples_dev || !idx_dev || !u_dev || !grad_out_dev || batch <= 0 || batch > (1 << 20))
        return fail(c, KRT_EINVAL, "bad grad args");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = mlp_ensure_batch(c, batch);
    if (rc) return rc;
    HIPCHK(c, launch_zero_i64(reinterpret_cast<int64_t *>(c->mlp_loss), 1, c->stream));
    HIPCHK(c, launch_mlp_grad(c->mlp_blob, samples_dev, idx_dev, u_dev, batch, c->mlp_act, c->mlp_act_cap,
                              c->mlp_part, c->mlp_loss, c->stream));
    HIPCHK(c, launch_mlp_gsum(c->mlp_part, grad_out_dev, c->stream));
    if (loss_out_dev) HIPCHK(c, hipMemcpyAsync(loss_out_dev, c->mlp_loss, sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KRT_OK;
}

extern "C" int krt_escape_train(krt_ctx *c, const float *samples_dev, uint64_t n, int32_t steps, int32_t batch,
                                double lr, uint64_t seed, float *loss_hist_dev) {
    if (!c) return KRT_EINVAL;
    if (!c->mlp_ready) return fail(c, KRT_ESTATE, "call krt_escape_init first");
    if (!samples_dev || n == 0 || n >= (1ull << 31) || steps <= 0 || batch <= 0 || batch > (1 << 20) ||
        !(lr > 0.0))
        return fail(c, KRT_EINVAL, "bad train args");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = mlp_ensure_batch(c, batch);
    if (rc) return rc;
    // each step's loss is summed straight into its slot of the history
    if (loss_hist_dev) HIPCHK(c, hipMemsetAsync(loss_hist_dev, 0, sizeof(float) * (size_t)steps, c->stream));
    for (int s = 0; s < steps; ++s) {
        c->mlp_step += 1;
        HIPCHK(c, launch_mlp_batch((int64_t)n, (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)c->mlp_step, batch,
                                   c->mlp_idx, c->mlp_u, c->stream));
        HIPCHK(c, launch_mlp_grad(c->mlp_blob, samples_dev, c->mlp_idx, c->mlp_u, batch, c->mlp_act, c->mlp_act_cap,
                                  c->mlp_part, loss_hist_dev ? loss_hist_dev + s : nullptr, c->stream));
        HIPCHK(c, launch_mlp_adam(c->mlp_p, c->mlp_m, c->mlp_v, c->mlp_part, (float)lr, c->mlp_step, c->stream));
        HIPCHK(c, launch_mlp_pack(c->mlp_p, c->mlp_norm, c->mlp_blob, (s == steps - 1) ? c->mlp_img : nullptr,
                                  c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KRT_OK;
}

extern "C" int krt_escape_get_weights(krt_ctx *c, float *dev, uint64_t nfloats) {
    if (!c) return KRT_EINVAL;
    if (!c->mlp_ready) return fail(c, KRT_ESTATE, "call krt_escape_init first");
    if (!dev || nfloats != (uint64_t)(kNParams + kNNorm)) return fail(c, KRT_EINVAL, "need %d floats", kNParams + kNNorm);
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(dev, c->mlp_p, sizeof(float) * kNParams, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(dev + kNParams, c->mlp_norm, sizeof(float) * kNNorm, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KRT_OK;
}

extern "C" int krt_escape_put_weights(krt_ctx *c, const float *dev, uint64_t nfloats) {
    if (!c) return KRT_EINVAL;
    if (!dev || nfloats != (uint64_t)(kNParams + kNNorm)) return fail(c, KRT_EINVAL, "need %d floats", kNParams + kNNorm);
    HIPCHK(c, hipSetDevice(c->device));
    int rc = mlp_alloc(c);
    if (rc) return rc;
    if (!c->mlp_ready) { rc = mlp_zero_state(c); if (rc) return rc; }
    HIPCHK(c, hipMemcpyAsync(c->mlp_p, dev, sizeof(float) * kNParams, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->mlp_norm, dev + kNParams, sizeof(float) * kNNorm, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, launch_mlp_pack(c->mlp_p, c->mlp_norm, c->mlp_blob, c->mlp_img, c->stream));
    c->mlp_ready = true;
    return read_a_range(c);
}

extern "C" int krt_escape_forward(krt_ctx *c, const float *in_dev, int64_t n, float *out_dev) {
    if (!c) return KRT_EINVAL;
    if (!c->mlp_ready) return fail(c, KRT_ESTATE, "call krt_escape_init first");
    if (!in_dev || !out_dev || n <= 0 || n >= (int64_t(1) << 30))  // four work-items per row
        return fail(c, KRT_EINVAL, "bad forward args");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_mlp_forward(c->mlp_blob, in_dev, n, out_dev, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return KRT_OK;
}
