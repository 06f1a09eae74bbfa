// Host-side pieces shared by the single-stream and the batched C-ABI
// front ends: kernel timing and the launch sequence of one device pass.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/erx.h"
#include "erx_internal.h"

namespace erx {

enum { K_GRAM, K_SCAN_LOCAL, K_SCAN_CARRY, K_CHOL32, K_CHOL64, K_SCORE, K_SCORE_REDO, K_NORMALISE, K_COUNT };

// Brackets launches with HIP events on the launch stream and sums their
// durations per kernel kind.
struct Profiler {
    struct Rec {
        int kernel;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Rec> recs;

    hipEvent_t take();
    template <class F> hipError_t timed(hipStream_t s, int kernel, F&& launch)
    {
        hipEvent_t a = take(), b = take();
        if (!a || !b) return hipErrorOutOfMemory;
        hipError_t e = hipEventRecord(a, s);
        if (e == hipSuccess) e = launch();
        if (e == hipSuccess) e = hipEventRecord(b, s);
        recs.push_back({kernel, a, b});
        return e;
    }
    int read(erx_kernel_time* out, int max);  // the stream must be idle
    void release();
};

// Launch the whole hot path for one pass: per-line mean and Gram, segment
// scan, carries, factorisation (FP32 with FP64 re-factor when thr > 0,
// FP64 for every line when thr == 0), scores (split FP16 with an FP32 pass
// over the lines it flags, or FP32; the split kernel needs P.mscale),
// optional normalisation.
hipError_t run_pass(hipStream_t s, const Pass& P, int NT, int dtype, int prec, int sarith, void* stats,
                    void* carry, float* Mt,
                    float* mu32, int* flags, float* cond, double thr, int want_cond, bool fp64_pass,
                    bool normalise, unsigned long long* ctr, Profiler* prof);

// thread-local error message of the C ABI
int set_error(int code, const char* fmt, ...);
const char* get_error();

}  // namespace erx
