// Allocation-free push: the single-stream hot path of erx_push_lines_ex with
// every intermediate buffer (per-line statistics, segment carries, inverse
// factors, means, flags) carved out of one file-scope device array instead of
// memory the library allocates.  The caller owns the input lines, the scores
// and the moving-average state; nothing here calls hipMalloc or hipFree.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "../../include/erx.h"
#include "erx_internal.h"
#include "erx_runtime.h"

using namespace erx;

namespace {

static_assert(ERX_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must be a multiple of 256");

// One copy per GPU, alive until the process ends.  In host code this name is
// a host-side stand-in, never a device address: kernels get the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[ERX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on `dev` (looked up once per device, with that
// device current), or null with the HIP error in *err.
unsigned char* scratch_of(int dev, hipError_t* err)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_scratch[dev]) return g_scratch[dev];
    void* ptr = nullptr;
    *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (*err != hipSuccess || !ptr) return nullptr;
    g_scratch[dev] = (unsigned char*)ptr;
    return g_scratch[dev];
}

size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }

// Byte offsets of the buffers of one pass of C lines inside the scratch.
struct Layout {
    size_t stats, carry, Mt, mu32, mscale, gredo, flags, cond, ctr, end;
};

Layout layout(int C, int seg, long long E, int NTL, int bpad)
{
    const size_t nseg = (size_t)(C + seg - 1) / seg;
    Layout L;
    L.stats = 0;
    L.carry = up256(L.stats + (size_t)C * E * sizeof(double));
    L.Mt = up256(L.carry + nseg * E * sizeof(double));
    L.mu32 = up256(L.Mt + (size_t)C * NTL * 256 * sizeof(float));
    L.mscale = up256(L.mu32 + (size_t)C * bpad * sizeof(float));
    L.gredo = up256(L.mscale + (size_t)C * sizeof(float));
    L.flags = up256(L.gredo + (size_t)C * GRAM_MACROS_MAX * sizeof(int));
    L.cond = up256(L.flags + (size_t)C * sizeof(int));
    L.ctr = up256(L.cond + (size_t)C * sizeof(float));
    L.end = up256(L.ctr + 4 * sizeof(unsigned long long));
    return L;
}

// The stream's state is cleared by a kernel rather than hipMemsetAsync, so a
// caller may capture the call in a HIP graph.
__global__ void k_zero(double* __restrict__ v, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = 0.0;
}

bool device_ptr(const void* ptr)
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

int erx_push_lines_noalloc(const erx_config* cfg, double* state, long long t0, const void* lines, int n,
                           float* out, void* hip_stream)
{
    // ---- argument checks (host only, before any device call)
    if (!cfg || !state || !lines || !out) return set_error(ERX_EINVAL, "erx_push_lines_noalloc: NULL argument");
    const erx_config& c = *cfg;
    if (c.bands < 1 || c.bands > ERX_MAX_BANDS)
        return set_error(ERX_EINVAL, "bands must be in [1, %d] (the scratch is sized for that maximum), got %d",
                         ERX_MAX_BANDS, c.bands);
    if (c.pixels < 2) return set_error(ERX_EINVAL, "pixels must be >= 2, got %d", c.pixels);
    if (!(c.momentum > 0.0f && c.momentum <= 1.0f))
        return set_error(ERX_EINVAL, "momentum must be in (0, 1], got %g", (double)c.momentum);
    if (!(c.ridge >= 0.0f) || !std::isfinite(c.ridge)) return set_error(ERX_EINVAL, "ridge must be finite and >= 0");
    if (c.dtype != ERX_F32 && c.dtype != ERX_F16 && c.dtype != ERX_U16)
        return set_error(ERX_EINVAL, "unknown dtype %d", c.dtype);
    if (c.precision < ERX_GRAM_FP32 || c.precision > ERX_GRAM_SPLIT16)
        return set_error(ERX_EINVAL, "unknown precision %d", c.precision);
    if (!(c.fp64_cond_threshold >= 0.0)) return set_error(ERX_EINVAL, "fp64_cond_threshold must be >= 0");
    if (c.cond_estimate < -1 || c.cond_estimate > 1) return set_error(ERX_EINVAL, "cond_estimate must be -1, 0 or 1");
    if (c.score_arith != ERX_SCORE_SPLIT16 && c.score_arith != ERX_SCORE_FP32)
        return set_error(ERX_EINVAL, "unknown score_arith %d", c.score_arith);
    if (c.normalise != 0) return set_error(ERX_EINVAL, "erx_push_lines_noalloc does not normalise (normalise must be 0)");
    if (c.srp_dims != 0) return set_error(ERX_EINVAL, "erx_push_lines_noalloc keeps every band (srp_dims must be 0)");
    if (c.background != ERX_BG_EMA) return set_error(ERX_EINVAL, "erx_push_lines_noalloc runs the moving averages (background must be ERX_BG_EMA)");
    if (c.state_fp32 != 0) return set_error(ERX_EINVAL, "erx_push_lines_noalloc keeps an FP64 state (state_fp32 must be 0)");
    if (c.score_tiles < 0 || c.score_tiles > 2) return set_error(ERX_EINVAL, "score_tiles must be 0, 1 or 2");
    if (c.gram_macro != 0 && c.gram_macro != 64 && c.gram_macro != 128)
        return set_error(ERX_EINVAL, "gram_macro must be 0, 64 or 128");
    if (c.block_lines < 1 || c.scan_lines < 1) return set_error(ERX_EINVAL, "block_lines and scan_lines must be >= 1");
    if (n < 1) return set_error(ERX_EINVAL, "n must be >= 1, got %d", n);
    if (t0 < 0) return set_error(ERX_EINVAL, "t0 must be >= 0");
    const size_t esz = c.dtype == ERX_F32 ? 4 : 2;

    const int NT = (c.bands + 15) / 16, NTL = NT * (NT + 1) / 2, bpad = 16 * NT;
    const long long E = stat_entries(NT);
    const int seg = c.scan_lines;
    // lines per pass: the configured block, cut to what the scratch holds
    int C = c.block_lines;
    if (layout(1, seg, E, NTL, bpad).end > ERX_NOALLOC_SCRATCH_BYTES)
        return set_error(ERX_EINVAL, "one line of %d bands with scan_lines %d needs %zu bytes, more than the %u-byte "
                                     "scratch", c.bands, seg, layout(1, seg, E, NTL, bpad).end,
                         (unsigned)ERX_NOALLOC_SCRATCH_BYTES);
    if (layout(C, seg, E, NTL, bpad).end > ERX_NOALLOC_SCRATCH_BYTES) {
        int lo = 1, hi = C;  // largest C that fits
        while (lo < hi) {
            const int mid = lo + (hi - lo + 1) / 2;
            if (layout(mid, seg, E, NTL, bpad).end <= ERX_NOALLOC_SCRATCH_BYTES) lo = mid;
            else hi = mid - 1;
        }
        C = lo;
    }

    // ---- device checks
    if (!device_ptr(lines) || !device_ptr(state) || !device_ptr(out))
        return set_error(ERX_EINVAL, "lines, state and out must be device memory");
    if ((uintptr_t)lines % esz != 0)
        return set_error(ERX_EINVAL, "line buffer must be aligned to its element size (%zu bytes)", esz);
    if ((uintptr_t)state % sizeof(double) != 0 || (uintptr_t)out % sizeof(float) != 0)
        return set_error(ERX_EINVAL, "state must be 8-byte and out 4-byte aligned");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(ERX_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return set_error(ERX_EDEVICE, "device %d out of range", dev);
    e = hipSuccess;
    unsigned char* base = scratch_of(dev, &e);
    if (!base) return set_error(ERX_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));

    const Layout L = layout(C, seg, E, NTL, bpad);
    double* stats = (double*)(base + L.stats);
    double* carry = (double*)(base + L.carry);
    float* Mt = (float*)(base + L.Mt);
    float* mu32 = (float*)(base + L.mu32);
    float* mscale = (float*)(base + L.mscale);
    int* gredo = (int*)(base + L.gredo);
    int* flags = (int*)(base + L.flags);
    float* cond = (float*)(base + L.cond);
    unsigned long long* ctr = (unsigned long long*)(base + L.ctr);  // counters, not reported here

    hipStream_t s = (hipStream_t)hip_stream;
    if (t0 == 0) {  // a fresh stream: the first line initialises the background
        hipLaunchKernelGGL(k_zero, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, s, state, E);
        if ((e = hipGetLastError()) != hipSuccess) return set_error(ERX_EDEVICE, "k_zero: %s", hipGetErrorString(e));
    }
    const double thr = c.fp64_cond_threshold;
    const bool decides = thr > 0.0 && !std::isinf(thr);
    const int want_cond = c.cond_estimate == 1 || (c.cond_estimate == -1 && decides) ? 1 : 0;
    const bool fp64_pass = !std::isinf(thr);
    const size_t line_bytes = (size_t)c.pixels * c.bands * esz;
    long long t = t0;
    for (int c0 = 0; c0 < n; c0 += C) {
        const int nc = (n - c0) < C ? (n - c0) : C;
        const void* src = (const char*)lines + (size_t)c0 * line_bytes;
        Pass P{};
        P.sd = nullptr;
        P.one.x = src;
        P.one.out = out + (size_t)c0 * c.pixels;
        P.one.outn = nullptr;
        P.one.state = state;
        P.one.t0 = t;
        P.one.alpha = c.momentum;
        P.one.eps = c.ridge;
        P.one.p = c.pixels;
        P.one.b = c.bands;
        P.one.n = nc;
        P.one.line0 = 0;
        P.one.seg0 = 0;
        P.nstreams = 1;
        P.nlines = nc;
        P.nseg = (nc + seg - 1) / seg;
        P.seg = seg;
        P.pmax = c.pixels;
        P.vec4 = (c.bands % 4) == 0 && ((uintptr_t)src % (4 * esz)) == 0;
        P.mscale = mscale;
        P.spt = c.score_tiles;
        P.gmacro = c.gram_macro;
        P.gredo = gredo;
        e = run_pass(s, P, NT, c.dtype, c.precision, c.score_arith, stats, carry, Mt, mu32, flags, cond, thr, want_cond, fp64_pass,
                     false, ctr, nullptr);
        if (e != hipSuccess) return set_error(ERX_EDEVICE, "launch failed: %s", hipGetErrorString(e));
        t += nc;
    }
    return ERX_OK;
}

}  // extern "C"
