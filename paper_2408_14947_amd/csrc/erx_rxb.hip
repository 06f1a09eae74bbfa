// RX Baseline of the paper's comparison (Sec. IV-B): a rolling buffer of the
// last W lines; the mean and the covariance (divisor n, the RX definition of
// Sec. II-A) of all pixels in the buffer score the buffer's centre line.  The
// window ending at stream line t (0-based) scores line t - (W-1)/2, once W
// lines have arrived.
//
// Built from the kernels of the detector: per-line mean and Gram, the
// per-line second moments about the stream's first mean X_j (k_imc_moments),
// their running mean A_t over lines (the chunked scan with weights 1/(t+1)),
// so that P_t = (t+1) A_t is the prefix sum of X_j (and of the line means).
// The window sums are prefix differences P_t - P_{t-W}; P of the W lines
// before a pass comes from a ring kept in device memory.  The window's
// statistics are then factored and the centre lines scored by the ordinary
// factorisation and score kernels (the factorisation reads them as they are:
// momentum 1 leaves no carry).  The last (W-1)/2 lines of every pass are kept
// for the next pass, whose windows centre on them.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/erx.h"
#include "erx_device.h"
#include "erx_runtime.h"

namespace erx {
namespace {

// running mean A of pass line j (stream-local, one stream) at entry e: the
// segment-local scan plus the decayed carry, as the factorisation reads it
__device__ __forceinline__ double run_mean(const Pass& P, const double* stats, const double* carry, long long E,
                                           int j, long long e)
{
    const StreamDesc& d = P.one;
    const int sg = j / P.seg, l0 = sg * P.seg;
    double D = 1.0;
    for (int l = l0; l <= j; ++l) D *= 1.0 - avg_weight(d, d.t0 + l);
    return stats[(size_t)j * E + e] + D * carry[(size_t)sg * E + e];
}

// prefix sum P of stream line tm (>= 0): from this pass or from the ring
__device__ __forceinline__ double prefix(const Pass& P, const double* stats, const double* carry,
                                         const double* ring, long long E, int W, long long tm, long long e)
{
    const long long t0 = P.one.t0;
    if (tm >= t0) return (double)(tm + 1) * run_mean(P, stats, carry, E, (int)(tm - t0), e);
    return ring[(size_t)(tm % W) * E + e];
}

// window statistics of pass line l (l >= lstart): mean and population covariance
// of the pixels of stream lines t-W+1..t, into fin[l - lstart]
__global__ __launch_bounds__(256) void k_rxb_window(const Pass P, const double* __restrict__ stats,
                                                    const double* __restrict__ carry,
                                                    const double* __restrict__ ring, double* __restrict__ fin,
                                                    long long E, int NT, int W, int lstart)
{
    const int l = lstart + blockIdx.y;
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= E) return;
    const StreamDesc& d = P.one;
    const long long t = d.t0 + l, tm = t - W;
    const long long ntU = (long long)NT * (NT + 1) / 2, m0 = ntU * 256;
    auto wsum = [&](long long q) __attribute__((always_inline)) {  // (1/W) sum over the window's lines
        const double a = prefix(P, stats, carry, ring, E, W, t, q);
        const double z = tm < 0 ? 0.0 : prefix(P, stats, carry, ring, E, W, tm, q);
        return (a - z) / (double)W;
    };
    double* out = fin + (size_t)(l - lstart) * E;
    if (e >= m0) {  // mean entries: the window mean
        out[e] = wsum(e);
        return;
    }
    int u = (int)(e >> 8), I = 0;
    while (u >= NT - I) {
        u -= NT - I;
        ++I;
    }
    const int J = I + u, pos = (int)(e & 255), q = pos >> 2;
    const int r = 16 * I + 4 * (q >> 4) + (pos & 3), c = 16 * J + (q & 15);
    if (r >= d.b || c >= d.b) {
        out[e] = 0.0;
        return;
    }
    const double* cref = (const double*)d.state + E;  // the moments are taken about this mean
    const double mr = wsum(m0 + r) - cref[r], mc = wsum(m0 + c) - cref[c];
    out[e] = wsum(e) - mr * mc;
}

// prefix sums of the pass's last min(W, n) lines into the ring
__global__ __launch_bounds__(256) void k_rxb_ring(const Pass P, const double* __restrict__ stats,
                                                  const double* __restrict__ carry, double* __restrict__ ring,
                                                  long long E, int W, int lfirst)
{
    const int l = lfirst + blockIdx.y;
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= E) return;
    const long long t = P.one.t0 + l;
    ring[(size_t)(t % W) * E + e] = (double)(t + 1) * run_mean(P, stats, carry, E, l, e);
}

}  // namespace
}  // namespace erx

using namespace erx;

struct erx_rxb {
    erx_config cfg;
    int W = 0, half = 0;
    int NT = 0, NTL = 0, bpad = 0;
    long long E = 0;
    hipStream_t stream = nullptr;
    long long t = 0;
    size_t line_bytes = 0;
    double* state = nullptr;  // [E + bpad] equal-weight scan state, then the reference mean
    double* stats = nullptr;  // [C][E]
    double* carry = nullptr;  // [nseg][E]
    double* ring = nullptr;   // [W][E] prefix sums of the last W lines
    double* fin = nullptr;    // [C][E] window statistics
    float* Mt = nullptr;
    float* mu32 = nullptr;
    float* mscale = nullptr;
    int* gredo = nullptr;
    int* flags = nullptr;
    float* cond = nullptr;
    unsigned long long* ctr = nullptr;
    char* in[2] = {nullptr, nullptr};  // [half + C] lines: the previous pass's last half lines, then this pass's
    int cur = 0;
    float* scores = nullptr;  // [cap][p]
    long long cap = 0;
    int last_m = 0;
    long long last_first = -1;
};

namespace {

#define RCHK(call)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return set_error(ERX_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

void rxb_free(erx_rxb* r)
{
    void* p[] = {r->state, r->stats, r->carry, r->ring, r->fin, r->Mt, r->mu32, r->mscale, r->gredo, r->flags, r->cond,
                 r->ctr, r->in[0], r->in[1], r->scores};
    for (void* q : p)
        if (q) (void)hipFree(q);
    if (r->stream) (void)hipStreamDestroy(r->stream);
}

bool dev_ptr(const void* ptr)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

}  // namespace

extern "C" {

erx_rxb* erx_rxb_create(const erx_config* cfg, int window)
{
    if (!cfg) {
        set_error(ERX_EINVAL, "erx_rxb_create: cfg is NULL");
        return nullptr;
    }
    const erx_config& c = *cfg;
    if (window < 1 || window % 2 == 0) {
        set_error(ERX_EINVAL, "window must be odd and >= 1 (it has a centre line), got %d", window);
        return nullptr;
    }
    if (c.bands < 1 || c.bands > ERX_MAX_BANDS || c.pixels < 2 || !(c.ridge >= 0.0f) || !std::isfinite(c.ridge) ||
        (c.dtype != ERX_F32 && c.dtype != ERX_F16 && c.dtype != ERX_U16) ||
        c.precision < ERX_GRAM_FP32 || c.precision > ERX_GRAM_SPLIT16 ||
        !(c.fp64_cond_threshold >= 0.0) || c.block_lines < 1 || c.scan_lines < 1 ||
        (c.score_arith != ERX_SCORE_SPLIT16 && c.score_arith != ERX_SCORE_FP32) || c.srp_dims != 0 ||
        c.normalise != 0 || c.cond_estimate < -1 || c.cond_estimate > 1 || c.state_fp32 != 0 || c.score_tiles < 0 ||
        c.score_tiles > 2 || (c.gram_macro != 0 && c.gram_macro != 64 && c.gram_macro != 128)) {
        set_error(ERX_EINVAL, "erx_rxb_create: invalid configuration (bands in [1, %d], pixels >= 2, ridge >= 0, "
                              "no projection, no normalisation, FP64 state)", ERX_MAX_BANDS);
        return nullptr;
    }
    erx_rxb* r = new (std::nothrow) erx_rxb();
    if (!r) {
        set_error(ERX_ENOMEM, "out of host memory");
        return nullptr;
    }
    r->cfg = c;
    r->W = window;
    r->half = (window - 1) / 2;
    r->NT = (c.bands + 15) / 16;
    r->NTL = r->NT * (r->NT + 1) / 2;
    r->bpad = 16 * r->NT;
    r->E = stat_entries(r->NT);
    r->line_bytes = (size_t)c.pixels * c.bands * (c.dtype == ERX_F32 ? 4 : 2);
    const size_t C = (size_t)c.block_lines, nseg = (C + c.scan_lines - 1) / c.scan_lines;
    bool ok = hipStreamCreate(&r->stream) == hipSuccess;
    ok = ok && hipMalloc(&r->state, (r->E + r->bpad) * sizeof(double)) == hipSuccess &&
         hipMemset(r->state, 0, (r->E + r->bpad) * sizeof(double)) == hipSuccess &&
         hipMalloc(&r->stats, C * r->E * sizeof(double)) == hipSuccess &&
         hipMalloc(&r->carry, nseg * r->E * sizeof(double)) == hipSuccess &&
         hipMalloc(&r->ring, (size_t)window * r->E * sizeof(double)) == hipSuccess &&
         hipMalloc(&r->fin, C * r->E * sizeof(double)) == hipSuccess &&
         hipMalloc(&r->Mt, C * r->NTL * 256 * sizeof(float)) == hipSuccess &&
         hipMalloc(&r->mu32, C * r->bpad * sizeof(float)) == hipSuccess &&
         hipMalloc(&r->mscale, C * sizeof(float)) == hipSuccess &&
         hipMalloc(&r->gredo, C * GRAM_MACROS_MAX * sizeof(int)) == hipSuccess &&
         hipMalloc(&r->flags, C * sizeof(int)) == hipSuccess && hipMalloc(&r->cond, C * sizeof(float)) == hipSuccess &&
         hipMalloc(&r->ctr, 4 * sizeof(unsigned long long)) == hipSuccess &&
         hipMemset(r->ctr, 0, 4 * sizeof(unsigned long long)) == hipSuccess &&
         hipMalloc(&r->in[0], (r->half + C) * r->line_bytes + 16) == hipSuccess &&
         hipMalloc(&r->in[1], (r->half + C) * r->line_bytes + 16) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        rxb_free(r);
        delete r;
        set_error(ERX_ENOMEM, "device allocation failed");
        return nullptr;
    }
    return r;
}

int erx_rxb_push(erx_rxb* r, const void* lines, int n)
{
    if (!r || !lines || n < 1) return set_error(ERX_EINVAL, "erx_rxb_push: NULL handle or buffer, or n < 1");
    const erx_config& c = r->cfg;
    const size_t esz = c.dtype == ERX_F32 ? 4 : 2;
    if (!dev_ptr(lines) || (uintptr_t)lines % esz) return set_error(ERX_EINVAL, "lines must be aligned device memory");
    // lines scored by this push: centres of the windows ending at t >= W-1
    const long long t_end = r->t + n;
    const long long m = std::max(0LL, t_end - (r->W - 1)) - std::max(0LL, r->t - (r->W - 1));
    if (m > r->cap) {
        if (r->scores) (void)hipFree(r->scores);
        r->scores = nullptr;
        r->cap = 0;
        if (hipMalloc(&r->scores, (size_t)m * c.pixels * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(ERX_ENOMEM, "cannot allocate scores for %lld lines", m);
        }
        r->cap = m;
    }
    r->last_m = (int)m;
    r->last_first = m > 0 ? std::max(r->t, (long long)(r->W - 1)) - r->half : -1;
    const int C = c.block_lines, seg = c.scan_lines;
    const double thr = c.fp64_cond_threshold;
    const bool decides = thr > 0.0 && !std::isinf(thr);
    const int want_cond = c.cond_estimate == 1 || (c.cond_estimate == -1 && decides) ? 1 : 0;
    const bool fp64_pass = !std::isinf(thr);
    long long written = 0;
    for (int c0 = 0; c0 < n; c0 += C) {
        const int nc = (n - c0) < C ? (n - c0) : C;
        char* cur = r->in[r->cur];
        char* nxt = r->in[r->cur ^ 1];
        RCHK(hipMemcpyAsync(cur + (size_t)r->half * r->line_bytes, (const char*)lines + (size_t)c0 * r->line_bytes,
                            (size_t)nc * r->line_bytes, hipMemcpyDeviceToDevice, r->stream));
        // statistics and their equal-weight running means
        Pass P{};
        P.one.x = cur + (size_t)r->half * r->line_bytes;
        P.one.out = nullptr;
        P.one.state = r->state;
        P.one.t0 = r->t;
        P.one.alpha = 1.0;
        P.one.eps = c.ridge;
        P.one.p = c.pixels;
        P.one.b = c.bands;
        P.one.n = nc;
        P.one.bg = BG_IMC;
        P.nstreams = 1;
        P.nlines = nc;
        P.nseg = (nc + seg - 1) / seg;
        P.seg = seg;
        P.pmax = c.pixels;
        P.vec4 = (c.bands % 4) == 0 && ((uintptr_t)P.one.x % (4 * esz)) == 0;
        P.gredo = r->gredo;
        RCHK(launch_gram(c.dtype, c.precision, P, r->NT, r->stats, r->stream));
        RCHK(launch_imc_moments(P, r->NT, r->stats, r->stream));
        RCHK(launch_scan_local(P, r->NT, r->stats, r->stream));
        RCHK(launch_scan_carry(P, r->NT, r->stats, r->carry, r->stream));
        // windows that end in this pass and are complete
        const int lstart = (int)std::max(0LL, (long long)(r->W - 1) - r->t);
        const dim3 blk(256);
        if (lstart < nc) {
            hipLaunchKernelGGL(k_rxb_window, dim3((unsigned)((r->E + 255) / 256), (unsigned)(nc - lstart)), blk, 0,
                               r->stream, P, r->stats, r->carry, r->ring, r->fin, r->E, r->NT, r->W, lstart);
            RCHK(hipGetLastError());
        }
        const int lring = std::max(0, nc - r->W);
        hipLaunchKernelGGL(k_rxb_ring, dim3((unsigned)((r->E + 255) / 256), (unsigned)(nc - lring)), blk, 0, r->stream,
                           P, r->stats, r->carry, r->ring, r->E, r->W, lring);
        RCHK(hipGetLastError());
        if (lstart < nc) {
            // factor the window statistics as they are (momentum 1: no carry) and score the centre lines
            const int nw = nc - lstart;
            Pass Q{};
            Q.one.x = cur + (size_t)lstart * r->line_bytes;  // stream line t0 + lstart - half
            Q.one.out = r->scores + (size_t)written * c.pixels;
            Q.one.state = r->state;
            Q.one.t0 = 1;
            Q.one.alpha = 1.0;
            Q.one.eps = c.ridge;
            Q.one.p = c.pixels;
            Q.one.b = c.bands;
            Q.one.n = nw;
            Q.one.bg = BG_EMA;
            Q.nstreams = 1;
            Q.nlines = nw;
            Q.nseg = (nw + seg - 1) / seg;
            Q.seg = seg;
            Q.pmax = c.pixels;
            Q.vec4 = (c.bands % 4) == 0 && ((uintptr_t)Q.one.x % (4 * esz)) == 0;
            Q.mscale = r->mscale;
            Q.spt = c.score_tiles;
            Q.gmacro = c.gram_macro;
            hipError_t e;
            if (thr > 0.0) {
                e = launch_chol(0, fp64_pass ? 0 : 1, Q, r->NT, r->fin, r->fin, r->Mt, r->mu32, r->flags, r->cond,
                                thr, want_cond, r->ctr, r->stream);
                if (e == hipSuccess && fp64_pass)
                    e = launch_chol(1, 0, Q, r->NT, r->fin, r->fin, r->Mt, r->mu32, r->flags, r->cond, thr, want_cond,
                                    r->ctr, r->stream);
            } else {
                e = launch_chol(1, 1, Q, r->NT, r->fin, r->fin, r->Mt, r->mu32, r->flags, r->cond, thr, want_cond,
                                r->ctr, r->stream);
            }
            if (e == hipSuccess) {
                if (c.score_arith == ERX_SCORE_SPLIT16) {
                    e = launch_score16(c.dtype, Q, r->NT, r->Mt, r->mu32, r->flags, r->stream);
                    if (e == hipSuccess) e = launch_score(c.dtype, Q, r->NT, r->Mt, r->mu32, r->stream, r->flags);
                } else {
                    e = launch_score(c.dtype, Q, r->NT, r->Mt, r->mu32, r->stream);
                }
            }
            if (e != hipSuccess) return set_error(ERX_EDEVICE, "launch failed: %s", hipGetErrorString(e));
            written += nw;
        }
        // the last half lines of this pass open the next one
        if (r->half > 0)
            RCHK(hipMemcpyAsync(nxt, cur + (size_t)nc * r->line_bytes, (size_t)r->half * r->line_bytes,
                                hipMemcpyDeviceToDevice, r->stream));
        r->cur ^= 1;
        r->t += nc;
    }
    return ERX_OK;
}

int erx_rxb_scores(erx_rxb* r, float* out, long long* first_line, int* nlines)
{
    if (!r) return set_error(ERX_EINVAL, "NULL handle");
    if (first_line) *first_line = r->last_first;
    if (nlines) *nlines = r->last_m;
    if (out && r->last_m > 0)
        RCHK(hipMemcpyAsync(out, r->scores, (size_t)r->last_m * r->cfg.pixels * sizeof(float), hipMemcpyDefault,
                            r->stream));
    RCHK(hipStreamSynchronize(r->stream));
    return ERX_OK;
}

void erx_rxb_destroy(erx_rxb* r)
{
    if (!r) return;
    (void)hipStreamSynchronize(r->stream);
    rxb_free(r);
    delete r;
}

}  // extern "C"
