// Autotuner of the library's launch settings (a project addition, not part of
// the method): for one workload shape every candidate setting is run on
// synthetic lines of that shape through the public entry points, timed with
// HIP events on a stream of the tuner's own, and the fastest is kept.  Results
// are cached in a small JSON file so that a shape is timed once.
//
// Candidates change only how the work is cut into launches and tiles (lines per
// device pass, lines per scan segment, the small-band path variant, the score
// kernel's 16-pixel tiles per wave), never what is computed, so a tuned handle
// gives the scores of an untuned one up to the rounding of the FP64
// moving-average state (the score tile shape changes nothing at all: each
// pixel's products are the same).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/erx.h"
#include "erx_internal.h"
#include "erx_runtime.h"

namespace {

#define fail erx::set_error

// Synthetic lines: values 0.25 + 0.5 u with u uniform on [0, 1) from the
// SplitMix64 output function of (seed, element index), stored in the
// workload's dtype.  Independent bands give a well-conditioned background, so
// the timings are those of lines that need no FP64 re-factor.
__global__ __launch_bounds__(256) void k_tune_fill(void* X, long long n, int dtype, unsigned long long seed)
{
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(i + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const float v = 0.25f + 0.5f * ((float)(z >> 40) * (1.0f / 16777216.0f));
        if (dtype == ERX_F32) ((float*)X)[i] = v;
        else if (dtype == ERX_F16) ((__half*)X)[i] = __float2half(v);
        else ((unsigned short*)X)[i] = (unsigned short)(v * 65536.0f);
    }
}

struct Key {
    int bands, pixels, dtype, precision, normalise, nstreams;
    double thr;
    int score_arith, state_fp32;  // entries written before these were keyed read as 0 (the defaults then)
};

Key key_of(const erx_config& c, int nstreams)
{
    return Key{c.bands, c.pixels, c.dtype, c.precision, c.normalise, nstreams, c.fp64_cond_threshold,
               c.score_arith, c.state_fp32};
}

bool same(const Key& a, const Key& b)
{
    return a.bands == b.bands && a.pixels == b.pixels && a.dtype == b.dtype && a.precision == b.precision &&
           a.normalise == b.normalise && a.nstreams == b.nstreams && a.thr == b.thr &&
           a.score_arith == b.score_arith && a.state_fp32 == b.state_fp32;
}

struct Entry {
    Key k;
    erx_tune_result r;
};

// value of "name": <number> inside one JSON object's text
bool field(const std::string& obj, const char* name, double* v)
{
    const std::string pat = std::string("\"") + name + "\"";
    size_t i = obj.find(pat);
    if (i == std::string::npos) return false;
    i = obj.find(':', i + pat.size());
    if (i == std::string::npos) return false;
    const char* s = obj.c_str() + i + 1;
    char* end = nullptr;
    errno = 0;
    const double x = std::strtod(s, &end);
    if (end == s || errno == ERANGE) return false;
    *v = x;
    return true;
}

// Cache file: {"erx_tune": 1, "entries": [{...}, ...]} with one flat object of
// numbers per entry.  A missing file is an empty cache; *bad is set when the
// file exists but is not in that form.
std::vector<Entry> load_cache(const char* path, bool* bad)
{
    std::vector<Entry> out;
    *bad = false;
    FILE* f = std::fopen(path, "rb");
    if (!f) return out;
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
    std::fclose(f);
    size_t i = txt.find("\"entries\"");
    if (txt.find("\"erx_tune\"") == std::string::npos || i == std::string::npos) {
        *bad = true;
        return out;
    }
    i = txt.find('[', i);
    if (i == std::string::npos) {
        *bad = true;
        return out;
    }
    for (;;) {
        const size_t a = txt.find_first_of("{]", i + 1);
        if (a == std::string::npos) {
            *bad = true;
            return out;
        }
        if (txt[a] == ']') break;
        const size_t b = txt.find('}', a);
        if (b == std::string::npos) {
            *bad = true;
            return out;
        }
        const std::string obj = txt.substr(a, b - a + 1);
        double v[11];
        const char* names[11] = {"bands",       "pixels",     "dtype",      "precision",  "normalise", "nstreams",
                                 "fp64_cond_threshold", "block_lines", "scan_lines", "small_path", "us_per_line"};
        for (int q = 0; q < 11; ++q)
            if (!field(obj, names[q], &v[q])) {
                *bad = true;
                return out;
            }
        Entry e{};
        double sa = 0.0, s32 = 0.0;
        (void)field(obj, "score_arith", &sa);
        (void)field(obj, "state_fp32", &s32);
        e.k = Key{(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], (int)v[5], v[6], (int)sa, (int)s32};
        e.r.block_lines = (int)v[7];
        e.r.scan_lines = (int)v[8];
        e.r.small_path = (int)v[9];
        e.r.us_per_line = v[10];
        double st = 0.0, gm = 0.0;  // entries written before these were tuned: the defaults
        e.r.score_tiles = field(obj, "score_tiles", &st) ? (int)st : 0;
        e.r.gram_macro = field(obj, "gram_macro", &gm) ? (int)gm : 0;
        e.r.candidates = 0;
        out.push_back(e);
        i = b;
    }
    return out;
}

bool save_cache(const char* path, const std::vector<Entry>& es)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    std::fprintf(f, "{\"erx_tune\": 1, \"entries\": [\n");
    for (size_t i = 0; i < es.size(); ++i) {
        const Entry& e = es[i];
        std::fprintf(f,
                     "  {\"bands\": %d, \"pixels\": %d, \"dtype\": %d, \"precision\": %d, \"normalise\": %d, "
                     "\"nstreams\": %d, \"fp64_cond_threshold\": %.17g, \"score_arith\": %d, \"state_fp32\": %d, "
                     "\"block_lines\": %d, \"scan_lines\": %d, "
                     "\"small_path\": %d, \"score_tiles\": %d, \"gram_macro\": %d, \"us_per_line\": %.6g}%s\n",
                     e.k.bands, e.k.pixels, e.k.dtype, e.k.precision, e.k.normalise, e.k.nstreams, e.k.thr,
                     e.k.score_arith, e.k.state_fp32,
                     e.r.block_lines, e.r.scan_lines, e.r.small_path, e.r.score_tiles, e.r.gram_macro, e.r.us_per_line,
                     i + 1 < es.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

int check_args(const erx_config* cfg, int nstreams, erx_tune_result* out)
{
    if (!cfg || !out) return fail(ERX_EINVAL, "erx_autotune: NULL argument");
    if (nstreams < 1) return fail(ERX_EINVAL, "nstreams must be >= 1, got %d", nstreams);
    if (cfg->bands < 1 || cfg->bands > ERX_MAX_BANDS || cfg->pixels < 2 || cfg->dtype < ERX_F32 ||
        cfg->dtype > ERX_U16 || cfg->precision < ERX_GRAM_FP32 || cfg->precision > ERX_GRAM_SPLIT16)
        return fail(ERX_EINVAL, "invalid configuration (bands %d, pixels %d, dtype %d, precision %d)", cfg->bands,
                    cfg->pixels, cfg->dtype, cfg->precision);
    return ERX_OK;
}

struct Bench {
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void* X = nullptr;
    ~Bench()
    {
        if (X) (void)hipFree(X);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st) (void)hipStreamDestroy(st);
    }
};

// milliseconds of one push of n lines by a single detector with the given
// setting (after a warm-up push), or a negative value with the error set
double time_single(const erx_config& base, int B, int S, int pt, int gm, Bench& bn, int n)
{
    erx_config c = base;
    c.block_lines = B;
    c.scan_lines = S;
    c.score_tiles = pt;
    c.gram_macro = gm;
    erx_ctx* h = erx_create_ex(&c);
    if (!h) return -1.0;
    double ms = -1.0;
    float t = 0.f;
    if (erx_set_stream(h, bn.st) == ERX_OK && erx_push_lines_ex(h, bn.X, std::min(n, B)) == ERX_OK &&
        hipEventRecord(bn.e0, bn.st) == hipSuccess && erx_push_lines_ex(h, bn.X, n) == ERX_OK &&
        hipEventRecord(bn.e1, bn.st) == hipSuccess && hipEventSynchronize(bn.e1) == hipSuccess &&
        hipEventElapsedTime(&t, bn.e0, bn.e1) == hipSuccess)
        ms = t;
    erx_destroy(h);
    return ms;
}

// milliseconds of one push of T lines to each of ns identical streams of a batch
double time_batch(const erx_config& base, int ns, int B, int mode, int pt, int gm, Bench& bn, int T)
{
    erx_config c = base;
    c.block_lines = B;
    c.score_tiles = pt;
    c.gram_macro = gm;
    std::vector<int> bands(ns, base.bands), pixels(ns, base.pixels), nl(ns, T);
    std::vector<float> mom(ns, base.momentum);
    erx_batch* bt = erx_batch_create(ns, bands.data(), pixels.data(), mom.data(), &c);
    if (!bt) return -1.0;
    const size_t line_bytes = (size_t)base.pixels * base.bands * (base.dtype == ERX_F32 ? 4 : 2);
    std::vector<const void*> ptr(ns);
    for (int s = 0; s < ns; ++s) ptr[s] = (const char*)bn.X + (size_t)s * T * line_bytes;
    double ms = -1.0;
    float t = 0.f;
    if (erx_batch_small_path(bt, mode) == ERX_OK && erx_batch_set_stream(bt, bn.st) == ERX_OK &&
        erx_batch_push(bt, ptr.data(), nl.data()) == ERX_OK && hipEventRecord(bn.e0, bn.st) == hipSuccess &&
        erx_batch_push(bt, ptr.data(), nl.data()) == ERX_OK && hipEventRecord(bn.e1, bn.st) == hipSuccess &&
        hipEventSynchronize(bn.e1) == hipSuccess && hipEventElapsedTime(&t, bn.e0, bn.e1) == hipSuccess)
        ms = t;
    erx_batch_destroy(bt);
    return ms;
}

}  // namespace

int erx_tune_lookup(const erx_config* cfg, int nstreams, const char* cache_path, erx_tune_result* out)
{
    const int rc = check_args(cfg, nstreams, out);
    if (rc != ERX_OK) return rc;
    if (!cache_path) return fail(ERX_EINVAL, "erx_tune_lookup: NULL cache path");
    bool bad = false;
    const std::vector<Entry> es = load_cache(cache_path, &bad);
    if (bad) return fail(ERX_EINVAL, "%s is not a tuning cache", cache_path);
    const Key k = key_of(*cfg, nstreams);
    for (const Entry& e : es)
        if (same(e.k, k)) {
            *out = e.r;
            return ERX_OK;
        }
    return fail(ERX_ESTATE, "no entry for this shape in %s", cache_path);
}

int erx_autotune(const erx_config* cfg, int nstreams, const char* cache_path, erx_tune_result* out)
{
    int rc = check_args(cfg, nstreams, out);
    if (rc != ERX_OK) return rc;
    std::vector<Entry> es;
    if (cache_path) {
        bool bad = false;
        es = load_cache(cache_path, &bad);
        if (bad) return fail(ERX_EINVAL, "%s is not a tuning cache", cache_path);
        const Key k = key_of(*cfg, nstreams);
        for (const Entry& e : es)
            if (same(e.k, k)) {
                *out = e.r;
                return ERX_OK;
            }
    }
    // validate the rest of the configuration the way a handle would
    {
        erx_config c = *cfg;
        c.block_lines = 64;
        c.scan_lines = 64;
        erx_ctx* h = erx_create_ex(&c);
        if (!h) return ERX_EINVAL;
        erx_destroy(h);
    }
    const size_t line_bytes = (size_t)cfg->pixels * cfg->bands * (cfg->dtype == ERX_F32 ? 4 : 2);
    const size_t cap = (size_t)4 << 30;  // synthetic input at most 4 GiB
    Bench bn;
    int n = 0, T = 0;
    if (nstreams == 1) n = (int)std::max<size_t>(64, std::min<size_t>(8192, cap / line_bytes));
    else T = (int)std::max<size_t>(16, std::min<size_t>(256, cap / (line_bytes * nstreams)));
    const size_t elems = (size_t)cfg->pixels * cfg->bands * (nstreams == 1 ? (size_t)n : (size_t)T * nstreams);
    if (hipStreamCreateWithFlags(&bn.st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&bn.e0) != hipSuccess ||
        hipEventCreate(&bn.e1) != hipSuccess)
        return fail(ERX_EDEVICE, "erx_autotune: cannot create a stream or events");
    if (hipMalloc(&bn.X, elems * (cfg->dtype == ERX_F32 ? 4 : 2)) != hipSuccess)
        return fail(ERX_ENOMEM, "erx_autotune: cannot allocate %zu synthetic elements", elems);
    hipLaunchKernelGGL(k_tune_fill, dim3(4096), dim3(256), 0, bn.st, bn.X, (long long)elems, cfg->dtype,
                       0x5EEDull + (unsigned long long)cfg->bands * 1000003ull + (unsigned long long)cfg->pixels);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(bn.st) != hipSuccess)
        return fail(ERX_EDEVICE, "erx_autotune: filling the synthetic lines failed");

    erx_tune_result best{};
    best.us_per_line = -1.0;
    int timed = 0;
    // the score tile shapes matter only to the split-FP16 score kernel
    std::vector<int> pts = {2};
    if (cfg->score_arith == ERX_SCORE_SPLIT16) pts = {1, 2};
    // and the Gram's blocking only to the split-FP16 Gram, with more than one 64-band macro tile
    std::vector<int> gms = {0};
    if (cfg->precision == ERX_GRAM_SPLIT16 && cfg->bands > 64) gms = {64, 128};
    if (nstreams == 1) {
        for (int B : {512, 1024, 2048, 4096, 8192}) {
            if (B > n && B != 512) continue;
            for (int S : {32, 64, 128})
                for (int pt : pts)
                    for (int gm : gms) {
                        const double ms = time_single(*cfg, B, S, pt, gm, bn, n);
                        if (ms < 0.0) return ERX_EDEVICE;
                        ++timed;
                        const double us = ms * 1e3 / n;
                        if (best.us_per_line < 0.0 || us < best.us_per_line)
                            best = erx_tune_result{B, S, -1, 0, us, pt, gm};
                    }
        }
    } else {
        std::vector<int> modes = {0};
        if (cfg->bands <= 16) modes = {0, 1, 2};
        for (int B : {1024, 4096, 16384})
            for (int mode : modes)
                for (int pt : pts)
                    for (int gm : gms) {
                        // the fused path cuts no passes and scores in its own kernel
                        if (mode != 0 && (B != 1024 || pt != pts.back() || gm != gms.back())) continue;
                        const double ms = time_batch(*cfg, nstreams, B, mode, pt, gm, bn, T);
                        if (ms < 0.0) return ERX_EDEVICE;
                        ++timed;
                        const double us = ms * 1e3 / ((double)T * nstreams);
                        if (best.us_per_line < 0.0 || us < best.us_per_line)
                            best = erx_tune_result{B, 64, mode, 0, us, pt, gm};
                    }
    }
    best.candidates = timed;
    *out = best;
    if (cache_path) {
        Entry e{key_of(*cfg, nstreams), best};
        e.r.candidates = 0;
        es.push_back(e);
        if (!save_cache(cache_path, es)) return fail(ERX_EINVAL, "cannot write %s", cache_path);
    }
    return ERX_OK;
}
