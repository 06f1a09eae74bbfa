// Launch sequence of one device pass, kernel timing, error reporting.
#include "erx_runtime.h"

#include <cstdarg>
#include <cstdio>

namespace erx {

namespace {
thread_local std::string g_err = "no error";
const char* kKernelNames[K_COUNT] = {"gram", "scan_local", "scan_carry", "chol_fp32", "chol_fp64", "score",
                                     "score_fp32_redo", "normalise"};
}  // namespace

int set_error(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

const char* get_error() { return g_err.c_str(); }

hipEvent_t Profiler::take()
{
    if (pool.empty()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
}

int Profiler::read(erx_kernel_time* out, int max)
{
    double ms[K_COUNT] = {0};
    long long cnt[K_COUNT] = {0};
    for (auto& r : recs) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) t = 0.f;
        ms[r.kernel] += t;
        cnt[r.kernel] += 1;
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    recs.clear();
    int k = 0;
    for (int i = 0; i < K_COUNT && k < max; ++i) {
        if (!cnt[i]) continue;
        std::snprintf(out[k].name, sizeof out[k].name, "%s", kKernelNames[i]);
        out[k].launches = cnt[i];
        out[k].total_ms = ms[i];
        ++k;
    }
    return k;
}

void Profiler::release()
{
    for (auto& r : recs) {
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    recs.clear();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
}

hipError_t run_pass(hipStream_t s, const Pass& P, int NT, int dtype, int prec, int sarith, void* stats,
                    void* carry, float* Mt,
                    float* mu32, int* flags, float* cond, double thr, int want_cond, bool fp64_pass,
                    bool normalise, unsigned long long* ctr, Profiler* prof)
{
    auto T = [&](int k, auto&& f) -> hipError_t { return prof ? prof->timed(s, k, f) : f(); };
    hipError_t e;
    if ((e = T(K_GRAM, [&] { return launch_gram(dtype, prec, P, NT, stats, s); })) != hipSuccess) return e;
    if (P.nstreams == 1 && !P.sd && P.one.bg == BG_IMC)
        if ((e = launch_imc_moments(P, NT, (double*)stats, s)) != hipSuccess) return e;
    if ((e = T(K_SCAN_LOCAL, [&] { return launch_scan_local(P, NT, stats, s); })) != hipSuccess) return e;
    if ((e = T(K_SCAN_CARRY, [&] { return launch_scan_carry(P, NT, stats, carry, s); })) != hipSuccess) return e;
    if (thr > 0.0) {
        e = T(K_CHOL32, [&] {
            return launch_chol(0, fp64_pass ? 0 : 1, P, NT, stats, carry, Mt, mu32, flags, cond, thr, want_cond,
                               ctr, s);
        });
        if (e != hipSuccess) return e;
        if (fp64_pass) {
            e = T(K_CHOL64, [&] {
                return launch_chol(1, 0, P, NT, stats, carry, Mt, mu32, flags, cond, thr, want_cond, ctr, s);
            });
            if (e != hipSuccess) return e;
        }
    } else {
        e = T(K_CHOL64, [&] {
            return launch_chol(1, 1, P, NT, stats, carry, Mt, mu32, flags, cond, thr, want_cond, ctr, s);
        });
        if (e != hipSuccess) return e;
    }
    if (sarith == ERX_SCORE_SPLIT16 && P.mscale) {
        if ((e = T(K_SCORE, [&] { return launch_score16(dtype, P, NT, Mt, mu32, flags, s); })) != hipSuccess)
            return e;
        // lines the split kernel flagged (each workgroup of the others returns at once)
        if ((e = T(K_SCORE_REDO, [&] { return launch_score(dtype, P, NT, Mt, mu32, s, flags); })) != hipSuccess)
            return e;
    } else {
        if ((e = T(K_SCORE, [&] { return launch_score(dtype, P, NT, Mt, mu32, s); })) != hipSuccess) return e;
    }
    if (normalise)
        if ((e = T(K_NORMALISE, [&] { return launch_normalise(P, s); })) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace erx
