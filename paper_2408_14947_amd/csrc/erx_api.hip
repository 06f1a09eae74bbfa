// C-ABI runtime of the ERX library: handles, validation, device memory, the
// per-pass launch sequence and the state / diagnostics accessors.  All
// arithmetic of the detector runs in the kernels of erx_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/erx.h"
#include "erx_internal.h"
#include "erx_runtime.h"

using namespace erx;

namespace {

#define fail erx::set_error
#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(ERX_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

size_t elem_size(int dtype) { return dtype == ERX_F32 ? 4 : 2; }

}  // namespace

struct erx_ctx {
    erx_config cfg;
    int wb = 0;  // bands the detector works in: srp_dims when the projection is on, else bands
    int NT = 0, NTL = 0, bpad = 0;
    long long E = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;
    long long t = 0;  // lines absorbed
    // device memory
    // the three below hold FP64 values, or FP32 ones with cfg.state_fp32 (ss bytes each)
    void* state = nullptr;     // [E + bpad] background after line t (packed), then (IMC) the reference mean
    void* stats = nullptr;     // [C][E] per-line statistics, then segment-local scan
    void* carry = nullptr;     // [nseg][E] background entering each scan segment
    size_t ss = sizeof(double);
    float* Mt = nullptr;       // [C][NTL][256] inverse-factor tiles
    float* mu32 = nullptr;     // [C][bpad] background mean per line
    float* mscale = nullptr;   // [C] max |L^{-1}| per line (split-FP16 score)
    int* gredo = nullptr;      // [C][GRAM_MACROS_MAX] split-FP16 Gram blocks left to FP32
    unsigned long long* ctr = nullptr;  // fp64 re-factors, not-PD lines, max cond (float bits)
    int* flags = nullptr;      // [cap] per line of the last push
    float* cond = nullptr;     // [cap]
    float* scores = nullptr;   // [cap][p]
    float* scores_n = nullptr; // [cap][p]
    unsigned char* labels = nullptr;  // [cap][p]
    void* staging = nullptr;   // [C][p][b] host-input staging
    float* srpW = nullptr;     // [b][d] projection weights (srp_dims > 0)
    float* zbuf = nullptr;     // [C][p][d] projected lines of one pass
    // the projection is taken relative to a reference pixel, z - W^T x_ref = W^T (x - x_ref):
    // the scores do not change (a common shift of all pixels) and the FP32 projection keeps
    // the residuals' digits; the reference is the first pixel the detector sees
    float* srp_xref = nullptr; // [b] FP32 reference pixel (device)
    std::vector<float> srpW_h; // [b][d] host copy of W
    bool srp_ref_set = false;
    long long cap = 0;
    int last_n = 0;
    long long last_t0 = 0;
    bool have_scores = false;
    // kernel timing
    bool profile = false;
    Profiler prof;
};

namespace {

void free_all(erx_ctx* h)
{
    void* ptrs[] = {h->state, h->stats, h->carry, h->Mt, h->mu32, h->mscale, h->gredo, h->ctr, h->flags, h->cond,
                    h->scores, h->scores_n, h->labels, h->staging, h->srpW, h->zbuf, h->srp_xref};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    h->prof.release();
    if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
}

template <class T> hipError_t dmalloc(T** p, size_t bytes)
{
    return hipMalloc((void**)p, bytes ? bytes : 16);
}

int ensure_capacity(erx_ctx* h, long long n)
{
    if (n <= h->cap) return ERX_OK;
    HIPCHK(hipStreamSynchronize(h->stream));
    void* old[] = {h->flags, h->cond, h->scores, h->scores_n, h->labels};
    for (void* p : old)
        if (p) (void)hipFree(p);
    h->flags = nullptr;
    h->cond = nullptr;
    h->scores = h->scores_n = nullptr;
    h->labels = nullptr;
    h->cap = 0;
    const size_t p = (size_t)h->cfg.pixels;
    if (dmalloc(&h->flags, n * sizeof(int)) != hipSuccess || dmalloc(&h->cond, n * sizeof(float)) != hipSuccess ||
        dmalloc(&h->scores, n * p * sizeof(float)) != hipSuccess ||
        (h->cfg.normalise && dmalloc(&h->scores_n, n * p * sizeof(float)) != hipSuccess) ||
        (h->cfg.normalise && dmalloc(&h->labels, n * p) != hipSuccess)) {
        (void)hipGetLastError();
        return fail(ERX_ENOMEM, "cannot allocate result buffers for %lld lines", n);
    }
    h->cap = n;
    return ERX_OK;
}

bool is_device_ptr(const void* ptr)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// offset of element (r, c) of the packed upper triangle (r <= c in tile terms)
long long packed_offset(int r, int c, int NT)
{
    const int I = r >> 4, J = c >> 4, rr = r & 15, cc = c & 15;
    const long long u = (long long)I * NT - (long long)I * (I - 1) / 2 + (J - I);
    return u * 256 + (16 * (rr >> 2) + cc) * 4 + (rr & 3);
}

// W^T x_ref in FP64 (zeros without a projection): the state holds the background
// of z - W^T x_ref
hipError_t srp_zref(erx_ctx* h, std::vector<double>& zref)
{
    zref.assign(h->wb, 0.0);
    if (!h->srpW) return hipSuccess;
    const int b = h->cfg.bands, d = h->wb;
    std::vector<float> xr(b);
    hipError_t e = hipMemcpyAsync(xr.data(), h->srp_xref, b * sizeof(float), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return e;
    for (int i = 0; i < b; ++i)
        for (int j = 0; j < d; ++j) zref[j] += (double)h->srpW_h[(size_t)i * d + j] * (double)xr[i];
    return hipSuccess;
}

}  // namespace

extern "C" {

const char* erx_last_error(void) { return erx::get_error(); }

void erx_config_default(erx_config* cfg, int bands, int pixels, float momentum)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof *cfg);
    cfg->bands = bands;
    cfg->pixels = pixels;
    cfg->momentum = momentum;
    cfg->ridge = 1e-5f;
    cfg->warmup = 0;
    cfg->dtype = ERX_F32;
    cfg->precision = ERX_GRAM_SPLIT16;
    cfg->fp64_cond_threshold = 0.0;
    cfg->normalise = 0;
    cfg->block_lines = 2048;
    cfg->scan_lines = 64;
    cfg->cond_estimate = -1;
    cfg->score_arith = ERX_SCORE_SPLIT16;
}

erx_ctx* erx_create_ex(const erx_config* cfg)
{
    if (!cfg) {
        fail(ERX_EINVAL, "erx_create_ex: cfg is NULL");
        return nullptr;
    }
    const erx_config& c = *cfg;
    if (c.bands < 1 || c.bands > ERX_MAX_BANDS) {
        fail(ERX_EINVAL, "bands must be in [1, %d], got %d", ERX_MAX_BANDS, c.bands);
        return nullptr;
    }
    if (c.pixels < 2) {
        fail(ERX_EINVAL, "pixels must be >= 2 (the line covariance divides by p-1), got %d", c.pixels);
        return nullptr;
    }
    if (!(c.momentum > 0.0f && c.momentum <= 1.0f)) {
        fail(ERX_EINVAL, "momentum must be in (0, 1], got %g", (double)c.momentum);
        return nullptr;
    }
    if (!(c.ridge >= 0.0f) || !std::isfinite(c.ridge)) {
        fail(ERX_EINVAL, "ridge must be finite and >= 0, got %g", (double)c.ridge);
        return nullptr;
    }
    if (c.dtype != ERX_F32 && c.dtype != ERX_F16 && c.dtype != ERX_U16) {
        fail(ERX_EINVAL, "unknown dtype %d", c.dtype);
        return nullptr;
    }
    if (c.precision < ERX_GRAM_FP32 || c.precision > ERX_GRAM_SPLIT16) {
        fail(ERX_EINVAL, "unknown precision %d", c.precision);
        return nullptr;
    }
    if (!(c.fp64_cond_threshold >= 0.0)) {
        fail(ERX_EINVAL, "fp64_cond_threshold must be >= 0");
        return nullptr;
    }
    if (c.cond_estimate < -1 || c.cond_estimate > 1) {
        fail(ERX_EINVAL, "cond_estimate must be -1, 0 or 1");
        return nullptr;
    }
    if (c.score_arith != ERX_SCORE_SPLIT16 && c.score_arith != ERX_SCORE_FP32) {
        fail(ERX_EINVAL, "unknown score_arith %d", c.score_arith);
        return nullptr;
    }
    if (c.background != ERX_BG_EMA && c.background != ERX_BG_IMC) {
        fail(ERX_EINVAL, "background must be ERX_BG_EMA or ERX_BG_IMC, got %d", c.background);
        return nullptr;
    }
    if (c.gram_macro != 0 && c.gram_macro != 64 && c.gram_macro != 128) {
        fail(ERX_EINVAL, "gram_macro must be 0, 64 or 128, got %d", c.gram_macro);
        return nullptr;
    }
    if (c.score_tiles < 0 || c.score_tiles > 2) {
        fail(ERX_EINVAL, "score_tiles must be 0, 1 or 2, got %d", c.score_tiles);
        return nullptr;
    }
    if (c.state_fp32 != 0 && c.state_fp32 != 1) {
        fail(ERX_EINVAL, "state_fp32 must be 0 or 1, got %d", c.state_fp32);
        return nullptr;
    }
    if (c.state_fp32 && c.background == ERX_BG_IMC) {
        fail(ERX_EINVAL, "state_fp32 = 1 needs background ERX_BG_EMA (the IMC moments are kept in FP64)");
        return nullptr;
    }
    if (c.srp_dims < 0 || c.srp_dims > ERX_SRP_MAX_DIMS) {
        fail(ERX_EINVAL, "srp_dims must be 0 (off) or in [1, %d], got %d", ERX_SRP_MAX_DIMS, c.srp_dims);
        return nullptr;
    }
    if (c.block_lines < 1 || c.scan_lines < 1 || c.warmup < 0 || (c.normalise != 0 && c.normalise != 1)) {
        fail(ERX_EINVAL, "block_lines and scan_lines must be >= 1, warmup >= 0, normalise 0/1");
        return nullptr;
    }
    erx_ctx* h = new (std::nothrow) erx_ctx();
    if (!h) {
        fail(ERX_ENOMEM, "out of host memory");
        return nullptr;
    }
    h->cfg = c;
    h->wb = c.srp_dims > 0 ? c.srp_dims : c.bands;
    h->NT = (h->wb + 15) / 16;
    h->NTL = h->NT * (h->NT + 1) / 2;
    h->bpad = 16 * h->NT;
    h->E = stat_entries(h->NT);
    h->ss = c.state_fp32 ? sizeof(float) : sizeof(double);
    const size_t C = (size_t)c.block_lines;
    const size_t nseg = (C + c.scan_lines - 1) / c.scan_lines;
    bool ok = hipGetDevice(&h->device) == hipSuccess && hipStreamCreate(&h->own_stream) == hipSuccess;
    h->stream = h->own_stream;
    // the state, then (IMC) the stream's reference mean
    ok = ok && dmalloc(&h->state, (h->E + h->bpad) * h->ss) == hipSuccess &&
         dmalloc(&h->stats, C * h->E * h->ss) == hipSuccess &&
         dmalloc(&h->carry, nseg * h->E * h->ss) == hipSuccess &&
         dmalloc(&h->Mt, C * h->NTL * 256 * sizeof(float)) == hipSuccess &&
         dmalloc(&h->mu32, C * h->bpad * sizeof(float)) == hipSuccess &&
         dmalloc(&h->mscale, C * sizeof(float)) == hipSuccess &&
         dmalloc(&h->gredo, C * GRAM_MACROS_MAX * sizeof(int)) == hipSuccess &&
         dmalloc(&h->ctr, 4 * sizeof(unsigned long long)) == hipSuccess;
    if (ok && c.srp_dims > 0) {
        std::vector<float>& W = h->srpW_h;
        W.resize((size_t)c.bands * c.srp_dims);
        ok = erx_srp_matrix(c.bands, c.srp_dims, c.srp_seed, W.data()) == ERX_OK &&
             dmalloc(&h->srpW, W.size() * sizeof(float)) == hipSuccess &&
             dmalloc(&h->srp_xref, (size_t)c.bands * sizeof(float)) == hipSuccess &&
             hipMemset(h->srp_xref, 0, (size_t)c.bands * sizeof(float)) == hipSuccess &&
             hipMemcpy(h->srpW, W.data(), W.size() * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
             dmalloc(&h->zbuf, C * (size_t)c.pixels * c.srp_dims * sizeof(float)) == hipSuccess;
    }
    ok = ok && hipMemset(h->state, 0, (h->E + h->bpad) * h->ss) == hipSuccess &&
         hipMemset(h->ctr, 0, 4 * sizeof(unsigned long long)) == hipSuccess;
    if (!ok) {
        const hipError_t e = hipGetLastError();
        free_all(h);
        delete h;
        fail(ERX_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
        return nullptr;
    }
    return h;
}

erx_ctx* erx_create(int bands, int pixels, float momentum)
{
    erx_config c;
    erx_config_default(&c, bands, pixels, momentum);
    return erx_create_ex(&c);
}

int erx_set_stream(erx_ctx* h, void* s)
{
    if (!h) return fail(ERX_EINVAL, "NULL handle");
    HIPCHK(hipStreamSynchronize(h->stream));
    h->stream = (hipStream_t)s;
    return ERX_OK;
}

int erx_push_lines_ex(erx_ctx* h, const void* lines, int n)
{
    if (!h) return fail(ERX_EINVAL, "NULL handle");
    if (!lines || n < 1) return fail(ERX_EINVAL, "need a non-NULL line buffer and n >= 1 (got n=%d)", n);
    const erx_config& c = h->cfg;
    int rc = ensure_capacity(h, n);
    if (rc) return rc;
    const bool dev = is_device_ptr(lines);
    const size_t esz = elem_size(c.dtype);
    if (dev && ((uintptr_t)lines % esz) != 0)
        return fail(ERX_EINVAL, "device line buffer must be aligned to its element size (%zu bytes)", esz);
    const size_t line_bytes = (size_t)c.pixels * c.bands * esz;
    const int C = c.block_lines, seg = c.scan_lines;
    if (!dev && !h->staging) {
        if (hipMalloc(&h->staging, (size_t)C * line_bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ERX_ENOMEM, "cannot allocate the input staging buffer");
        }
    }
    const double thr = c.fp64_cond_threshold;
    const bool decides = thr > 0.0 && !std::isinf(thr);  // the estimate picks the FP64 lines
    const int want_cond = c.cond_estimate == 1 || (c.cond_estimate == -1 && decides) ? 1 : 0;
    const bool fp64_pass = !std::isinf(thr);
    h->last_t0 = h->t;
    for (int c0 = 0; c0 < n; c0 += C) {
        const int nc = (n - c0) < C ? (n - c0) : C;
        const void* src;
        if (dev) {
            src = (const char*)lines + (size_t)c0 * line_bytes;
        } else {
            HIPCHK(hipMemcpyAsync(h->staging, (const char*)lines + (size_t)c0 * line_bytes, nc * line_bytes,
                                  hipMemcpyHostToDevice, h->stream));
            src = h->staging;
        }
        // the sparse random projection (Sec. III-B) turns the pass into one over Z = X W in FP32
        int pdt = c.dtype;
        if (h->srpW) {
            if (!h->srp_ref_set) {  // the first pixel the detector sees becomes the reference
                HIPCHK(launch_srp_ref(c.dtype, src, c.bands, h->srp_xref, h->stream));
                h->srp_ref_set = true;
            }
            HIPCHK(launch_srp_project(c.dtype, src, (long long)nc * c.pixels, c.bands, h->srpW, h->srp_xref, h->wb,
                                      h->zbuf, h->stream));
            src = h->zbuf;
            pdt = ERX_F32;
        }
        Pass P{};
        P.sd = nullptr;
        P.one.x = src;
        P.one.out = h->scores + (size_t)c0 * c.pixels;
        P.one.outn = c.normalise ? h->scores_n + (size_t)c0 * c.pixels : nullptr;
        P.one.state = h->state;
        P.one.t0 = h->t;
        P.one.alpha = c.momentum;
        P.one.bg = c.background;
        P.one.eps = c.ridge;
        P.one.p = c.pixels;
        P.one.b = h->wb;
        P.one.n = nc;
        P.one.line0 = 0;
        P.one.seg0 = 0;
        P.nstreams = 1;
        P.nlines = nc;
        P.nseg = (nc + seg - 1) / seg;
        P.seg = seg;
        P.pmax = c.pixels;
        // 4-band vector loads need b % 4 == 0 and a 4-element aligned buffer
        P.vec4 = (h->wb % 4) == 0 && ((uintptr_t)src % (4 * elem_size(pdt))) == 0;
        P.mscale = h->mscale;
        P.gredo = h->gredo;
        P.sf32 = c.state_fp32;
        P.spt = c.score_tiles;
        P.gmacro = c.gram_macro;
        HIPCHK(run_pass(h->stream, P, h->NT, pdt, c.precision, c.score_arith, h->stats, h->carry, h->Mt, h->mu32, h->flags + c0,
                        h->cond + c0, thr, want_cond, fp64_pass, c.normalise != 0, h->ctr,
                        h->profile ? &h->prof : nullptr));
        h->t += nc;
        if (!dev) HIPCHK(hipStreamSynchronize(h->stream));  // the staging buffer is reused
    }
    h->last_n = n;
    h->have_scores = true;
    return ERX_OK;
}

int erx_push_lines(erx_ctx* h, const float* lines, int n)
{
    if (h && h->cfg.dtype != ERX_F32) return fail(ERX_EINVAL, "erx_push_lines needs a F32 handle");
    return erx_push_lines_ex(h, lines, n);
}

static int check_notpd(erx_ctx* h)
{
    std::vector<int> f(h->last_n);
    HIPCHK(hipMemcpyAsync(f.data(), h->flags, f.size() * sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int v : f)
        if (v & FLAG_NOTPD) return fail(ERX_ENOTPD, "at least one line had a covariance that is not positive definite");
    return ERX_OK;
}

int erx_scores(erx_ctx* h, float* out)
{
    if (!h || !out) return fail(ERX_EINVAL, "NULL argument");
    if (!h->have_scores) return fail(ERX_ESTATE, "no lines pushed yet");
    const size_t bytes = (size_t)h->last_n * h->cfg.pixels * sizeof(float);
    HIPCHK(hipMemcpyAsync(out, h->scores, bytes, hipMemcpyDefault, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return check_notpd(h);
}

int erx_scores_device(erx_ctx* h, float* dev_out)
{
    if (!h || !dev_out) return fail(ERX_EINVAL, "NULL argument");
    if (!h->have_scores) return fail(ERX_ESTATE, "no lines pushed yet");
    const size_t bytes = (size_t)h->last_n * h->cfg.pixels * sizeof(float);
    HIPCHK(hipMemcpyAsync(dev_out, h->scores, bytes, hipMemcpyDeviceToDevice, h->stream));
    return ERX_OK;
}

int erx_scores_normalised(erx_ctx* h, float* out)
{
    if (!h || !out) return fail(ERX_EINVAL, "NULL argument");
    if (!h->cfg.normalise) return fail(ERX_EINVAL, "handle created without normalise = 1");
    if (!h->have_scores) return fail(ERX_ESTATE, "no lines pushed yet");
    const size_t bytes = (size_t)h->last_n * h->cfg.pixels * sizeof(float);
    HIPCHK(hipMemcpyAsync(out, h->scores_n, bytes, hipMemcpyDefault, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return check_notpd(h);
}

int erx_labels(erx_ctx* h, float tau, unsigned char* out)
{
    if (!h || !out) return fail(ERX_EINVAL, "NULL argument");
    if (!h->cfg.normalise) return fail(ERX_EINVAL, "handle created without normalise = 1");
    if (!h->have_scores) return fail(ERX_ESTATE, "no lines pushed yet");
    HIPCHK(launch_labels(h->scores_n, h->last_n, h->cfg.pixels, tau, h->last_t0, h->cfg.warmup, h->labels,
                         h->stream));
    HIPCHK(hipMemcpyAsync(out, h->labels, (size_t)h->last_n * h->cfg.pixels, hipMemcpyDefault, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return ERX_OK;
}

// the device state as FP64 values on the host, whatever its storage type
static hipError_t read_state(erx_ctx* h, std::vector<double>& s)
{
    const size_t n = (size_t)(h->E + h->bpad);
    s.resize(n);
    if (h->ss == sizeof(double)) {
        const hipError_t e = hipMemcpyAsync(s.data(), h->state, n * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        return e == hipSuccess ? hipStreamSynchronize(h->stream) : e;
    }
    std::vector<float> f(n);
    hipError_t e = hipMemcpyAsync(f.data(), h->state, n * sizeof(float), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    for (size_t i = 0; i < n; ++i) s[i] = f[i];
    return e;
}

static hipError_t write_state(erx_ctx* h, const std::vector<double>& s)
{
    hipError_t e;
    if (h->ss == sizeof(double)) {
        e = hipMemcpyAsync(h->state, s.data(), s.size() * sizeof(double), hipMemcpyHostToDevice, h->stream);
        return e == hipSuccess ? hipStreamSynchronize(h->stream) : e;
    }
    std::vector<float> f(s.begin(), s.end());  // rounded to nearest
    e = hipMemcpyAsync(h->state, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, h->stream);
    return e == hipSuccess ? hipStreamSynchronize(h->stream) : e;  // f must outlive the copy
}

int erx_get_state(erx_ctx* h, long long* t, double* mu, double* K)
{
    if (!h) return fail(ERX_EINVAL, "NULL handle");
    std::vector<double> s;
    HIPCHK(read_state(h, s));
    const int b = h->wb, NT = h->NT;
    if (t) *t = h->t;
    std::vector<double> zref;
    HIPCHK(srp_zref(h, zref));
    const double* m = &s[(size_t)h->NTL * 256];
    const double* cref = &s[h->E];
    const bool imc = h->cfg.background == ERX_BG_IMC && h->t > 0;
    // IMC: the state holds second moments about the reference mean; K = N/(N-1) (C - (mu-c)(mu-c)^T)
    const double N = (double)h->t * h->cfg.pixels, f = imc ? N / (N - 1.0) : 1.0;
    if (mu)
        for (int j = 0; j < b; ++j) mu[j] = m[j] + zref[j];
    if (K)
        for (int r = 0; r < b; ++r)
            for (int c = 0; c < b; ++c) {
                double v = (r <= c) ? s[packed_offset(r, c, NT)] : s[packed_offset(c, r, NT)];
                if (imc) v = f * (v - (m[r] - cref[r]) * (m[c] - cref[c]));
                K[(size_t)r * b + c] = v;
            }
    return ERX_OK;
}

int erx_set_state(erx_ctx* h, long long t, const double* mu, const double* K)
{
    if (!h) return fail(ERX_EINVAL, "NULL handle");
    if (t < 0) return fail(ERX_EINVAL, "t must be >= 0");
    if (t > 0 && (!mu || !K)) return fail(ERX_EINVAL, "mu and K are required when t > 0");
    std::vector<double> s(h->E + h->bpad, 0.0);
    const int b = h->wb, NT = h->NT;
    if (h->srpW && !h->srp_ref_set) h->srp_ref_set = true;  // the state fixes the reference: x_ref = 0
    std::vector<double> zref;
    HIPCHK(srp_zref(h, zref));
    // IMC: second moments about the reference c = mu, C = (N-1)/N K
    const bool imc = h->cfg.background == ERX_BG_IMC && t > 0;
    const double N = (double)t * h->cfg.pixels, f = imc ? (N - 1.0) / N : 1.0;
    if (t > 0) {
        for (int j = 0; j < b; ++j) {
            s[(size_t)h->NTL * 256 + j] = mu[j] - zref[j];
            if (imc) s[h->E + j] = mu[j] - zref[j];
        }
        for (int r = 0; r < b; ++r)
            for (int c = r; c < b; ++c) {
                s[packed_offset(r, c, NT)] = f * K[(size_t)r * b + c];
                // diagonal tiles are stored whole (both triangles), as the kernels write them
                if ((r >> 4) == (c >> 4)) s[packed_offset(c, r, NT)] = f * K[(size_t)c * b + r];
            }
    }
    HIPCHK(write_state(h, s));
    h->t = t;
    h->have_scores = false;
    return ERX_OK;
}

int erx_stats(erx_ctx* h, erx_stats_t* out)
{
    if (!h || !out) return fail(ERX_EINVAL, "NULL argument");
    unsigned long long c[4];
    HIPCHK(hipMemcpyAsync(c, h->ctr, sizeof c, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    out->lines = h->t;
    out->fp64_refactors = (long long)c[0];
    out->notpd = (long long)c[1];
    float mc;
    const unsigned int bits = (unsigned int)(c[2] & 0xffffffffull);
    std::memcpy(&mc, &bits, sizeof mc);
    out->max_cond = mc;
    return ERX_OK;
}

int erx_line_info(erx_ctx* h, float* cond, int* flags)
{
    if (!h) return fail(ERX_EINVAL, "NULL handle");
    if (!h->have_scores) return fail(ERX_ESTATE, "no lines pushed yet");
    if (cond)
        HIPCHK(hipMemcpyAsync(cond, h->cond, (size_t)h->last_n * sizeof(float), hipMemcpyDefault, h->stream));
    if (flags)
        HIPCHK(hipMemcpyAsync(flags, h->flags, (size_t)h->last_n * sizeof(int), hipMemcpyDefault, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return ERX_OK;
}

int erx_profile_enable(erx_ctx* h, int on)
{
    if (!h) return fail(ERX_EINVAL, "NULL handle");
    h->profile = on != 0;
    return ERX_OK;
}

int erx_profile_read(erx_ctx* h, erx_kernel_time* out, int max)
{
    if (!h || (max > 0 && !out) || max < 0) return fail(ERX_EINVAL, "bad arguments");
    HIPCHK(hipStreamSynchronize(h->stream));
    return h->prof.read(out, max);
}

int erx_synchronize(erx_ctx* h)
{
    if (!h) return fail(ERX_EINVAL, "NULL handle");
    HIPCHK(hipStreamSynchronize(h->stream));
    return ERX_OK;
}

void erx_destroy(erx_ctx* h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    free_all(h);
    delete h;
}

}  // extern "C"
