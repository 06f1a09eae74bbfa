// Detection metrics of Sec. IV-C on the device: ROC AUC over all thresholds,
// and the threshold-curve areas behind AUC_TD and AUC_BS (Eqs. (26)-(29)).
//
// AUC.  The ROC curve visits every distinct score as a threshold; between
// consecutive thresholds it is straight, so its trapezoid area equals the
// fraction of (anomaly, background) pairs in which the anomaly scores higher,
// ties counting one half.  That count is exact in integers: the finite
// scores of the smaller class are compacted and sorted (bitonic network: a
// 2048-element LDS sort per workgroup, then the cross-chunk stages in global
// memory), and every pixel of the other class counts the sorted pixels below
// and equal to its score by two binary searches.  The sum of 2 * below + equal
// (64-bit atomics) over the pixels, divided by 2 P N, is the AUC.
//
// Threshold areas.  With the scores min-max normalised over the evaluated
// pixels, TPR(tau) = P(v >= tau | anomaly) for tau in [0, 1], and its area is
// the mean normalised anomaly score (the area under a survival function is
// the mean); likewise FPR for the background.  So one pass gathers the class
// counts, the class sums of the scores (FP64) and the minimum and maximum.
// All equal scores normalise to 0.  Non-finite scores are left out and counted.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/erx.h"
#include "erx_internal.h"
#include "erx_runtime.h"

namespace erx {
namespace {

struct MetAcc {
    unsigned long long cnt[3];  // anomalies, background, excluded
    double sum[2];              // score sums: anomalies, background
    unsigned int lo, hi;        // order-preserving bits of the smallest / largest finite score
    unsigned int pad_[2];
    unsigned long long pairs2;  // sum of 2 * below + equal
    unsigned long long ngath;   // compaction counter
};

// float -> unsigned with the same order (negative values reversed)
__device__ __forceinline__ unsigned int ord_bits(float f)
{
    const unsigned int u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float ord_float(unsigned int o)
{
    const unsigned int u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    float f;
    __builtin_memcpy(&f, &u, sizeof f);
    return f;
}

template <class T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ __launch_bounds__(256) void k_met_count(const float* __restrict__ s, const unsigned char* __restrict__ y,
                                                   long long n, MetAcc* acc)
{
    unsigned long long c0 = 0, c1 = 0, c2 = 0;
    double s0 = 0.0, s1 = 0.0;
    unsigned int lo = 0xffffffffu, hi = 0u;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const float v = s[i];
        if (!isfinite(v)) {
            ++c2;
            continue;
        }
        const unsigned int o = ord_bits(v);
        lo = min(lo, o);
        hi = max(hi, o);
        if (y[i]) {
            ++c0;
            s0 += (double)v;
        } else {
            ++c1;
            s1 += (double)v;
        }
    }
    c0 = wave_sum(c0);
    c1 = wave_sum(c1);
    c2 = wave_sum(c2);
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = min(lo, (unsigned int)__shfl_xor((int)lo, o));
        hi = max(hi, (unsigned int)__shfl_xor((int)hi, o));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&acc->cnt[0], c0);
        atomicAdd(&acc->cnt[1], c1);
        atomicAdd(&acc->cnt[2], c2);
        atomicAdd(&acc->sum[0], s0);
        atomicAdd(&acc->sum[1], s1);
        atomicMin(&acc->lo, lo);
        atomicMax(&acc->hi, hi);
    }
}

// finite scores of class cls appended to out (order irrelevant: sorted next)
__global__ __launch_bounds__(256) void k_met_gather(const float* __restrict__ s, const unsigned char* __restrict__ y,
                                                    long long n, int cls, float* __restrict__ out, MetAcc* acc)
{
    for (long long i0 = (long long)blockIdx.x * 256; i0 < n; i0 += (long long)gridDim.x * 256) {
        const long long i = i0 + threadIdx.x;
        bool take = false;
        float v = 0.f;
        if (i < n) {
            v = s[i];
            take = isfinite(v) && ((y[i] != 0) == (cls == 0));
        }
        // one atomic per wave
        const unsigned long long mask = __ballot(take);
        const int lane = threadIdx.x & 63;
        unsigned long long base = 0;
        const int leader = mask ? __ffsll((long long)mask) - 1 : 0;
        if (mask && lane == leader) base = atomicAdd(&acc->ngath, (unsigned long long)__popcll(mask));
        base = __shfl(base, leader);
        if (take) out[base + __popcll(mask & ((1ull << lane) - 1ull))] = v;
    }
}

__global__ __launch_bounds__(256) void k_met_fill(float* __restrict__ a, long long from, long long to)
{
    const long long i = from + (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < to) a[i] = __builtin_inff();
}

__device__ __forceinline__ void cmp_swap(float* a, long long i, long long l, bool up)
{
    const float x = a[i], z = a[l];
    if ((x > z) == up) {
        a[i] = z;
        a[l] = x;
    }
}

// every bitonic stage of sizes k <= 2048 on each 2048-element chunk (LDS);
// directions follow the global index, as in the full network
__global__ __launch_bounds__(1024) void k_bitonic_chunk(float* __restrict__ a, long long kmax_first)
{
    __shared__ float t[2048];
    const long long base = (long long)blockIdx.x * 2048;
    const int tid = threadIdx.x;
    t[tid] = a[base + tid];
    t[tid + 1024] = a[base + tid + 1024];
    __syncthreads();
    for (long long k = 2; k <= kmax_first; k <<= 1) {
        for (int j = (int)(k >> 1); j > 0; j >>= 1) {
            const int i = (tid / j) * 2 * j + (tid % j);
            const bool up = ((base + i) & k) == 0;
            const float x = t[i], z = t[i + j];
            if ((x > z) == up) {
                t[i] = z;
                t[i + j] = x;
            }
            __syncthreads();
        }
    }
    a[base + tid] = t[tid];
    a[base + tid + 1024] = t[tid + 1024];
}

// stages j <= 1024 of size k (k > 2048) on each 2048-element chunk
__global__ __launch_bounds__(1024) void k_bitonic_tail(float* __restrict__ a, long long k)
{
    __shared__ float t[2048];
    const long long base = (long long)blockIdx.x * 2048;
    const int tid = threadIdx.x;
    t[tid] = a[base + tid];
    t[tid + 1024] = a[base + tid + 1024];
    __syncthreads();
    const bool up = (base & k) == 0;  // the whole chunk lies in one k-block
    for (int j = 1024; j > 0; j >>= 1) {
        const int i = (tid / j) * 2 * j + (tid % j);
        const float x = t[i], z = t[i + j];
        if ((x > z) == up) {
            t[i] = z;
            t[i + j] = x;
        }
        __syncthreads();
    }
    a[base + tid] = t[tid];
    a[base + tid + 1024] = t[tid + 1024];
}

// one stage j >= 2048 of size k in global memory: thread t handles pair (i, i + j)
__global__ __launch_bounds__(256) void k_bitonic_global(float* __restrict__ a, long long half, long long j, long long k)
{
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= half) return;
    const long long i = (t / j) * 2 * j + (t % j);
    cmp_swap(a, i, i + j, (i & k) == 0);
}

__device__ __forceinline__ long long lower_bound(const float* a, long long m, float v)
{
    long long lo = 0, hi = m;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ long long upper_bound(const float* a, long long m, float v)
{
    long long lo = 0, hi = m;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (a[mid] <= v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// pixels of the class that was not sorted count the sorted ones below / equal
__global__ __launch_bounds__(256) void k_met_pairs(const float* __restrict__ s, const unsigned char* __restrict__ y,
                                                   long long n, int sorted_cls, const float* __restrict__ srt,
                                                   long long m, MetAcc* acc)
{
    unsigned long long c = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const float v = s[i];
        if (!isfinite(v) || ((y[i] != 0) == (sorted_cls == 0))) continue;
        const long long lo = lower_bound(srt, m, v), hi = upper_bound(srt, m, v);
        // sorted anomalies: pairs with the anomaly above this background pixel;
        // sorted background: pairs with this anomaly above the sorted pixel
        c += sorted_cls == 0 ? 2ull * (unsigned long long)(m - hi) + (unsigned long long)(hi - lo)
                             : 2ull * (unsigned long long)lo + (unsigned long long)(hi - lo);
    }
    c = wave_sum(c);
    if ((threadIdx.x & 63) == 0) atomicAdd(&acc->pairs2, c);
}

__global__ void k_met_init(MetAcc* acc)
{
    acc->cnt[0] = acc->cnt[1] = acc->cnt[2] = 0;
    acc->sum[0] = acc->sum[1] = 0.0;
    acc->lo = 0xffffffffu;
    acc->hi = 0u;
    acc->pairs2 = 0;
    acc->ngath = 0;
}

}  // namespace
}  // namespace erx

using namespace erx;

#define MCHK(call)                                                                                \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            rc = set_error(ERX_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));                  \
            goto done;                                                                            \
        }                                                                                         \
    } while (0)

extern "C" int erx_detection_metrics(const float* scores, const unsigned char* truth, long long n, void* hip_stream,
                                     erx_detection_metrics_t* out)
{
    if (!scores || !truth || !out || n < 2) return set_error(ERX_EINVAL, "erx_detection_metrics: bad arguments");
    hipPointerAttribute_t pa, pb;
    if (hipPointerGetAttributes(&pa, scores) != hipSuccess || hipPointerGetAttributes(&pb, truth) != hipSuccess ||
        (pa.type != hipMemoryTypeDevice && pa.type != hipMemoryTypeManaged) ||
        (pb.type != hipMemoryTypeDevice && pb.type != hipMemoryTypeManaged)) {
        (void)hipGetLastError();
        return set_error(ERX_EINVAL, "scores and truth must be device memory");
    }
    hipStream_t st = (hipStream_t)hip_stream;
    int rc = ERX_OK;
    MetAcc* acc = nullptr;
    float* buf = nullptr;
    MetAcc h{};
    long long m = 0, m2 = 2048;
    int cls = 0;
    const unsigned grid = (unsigned)std::min<long long>((n + 255) / 256, 4096);
    MCHK(hipMalloc(&acc, sizeof(MetAcc)));
    hipLaunchKernelGGL(k_met_init, dim3(1), dim3(1), 0, st, acc);
    hipLaunchKernelGGL(k_met_count, dim3(grid), dim3(256), 0, st, scores, truth, n, acc);
    MCHK(hipGetLastError());
    MCHK(hipMemcpyAsync(&h, acc, sizeof h, hipMemcpyDeviceToHost, st));
    MCHK(hipStreamSynchronize(st));
    if (h.cnt[0] == 0 || h.cnt[1] == 0) {
        rc = set_error(ERX_EINVAL, "need at least one anomaly and one background pixel with finite scores "
                                   "(got %llu and %llu)", h.cnt[0], h.cnt[1]);
        goto done;
    }
    // sort the smaller class
    cls = h.cnt[0] <= h.cnt[1] ? 0 : 1;
    m = (long long)h.cnt[cls];
    while (m2 < m) m2 <<= 1;
    MCHK(hipMalloc(&buf, (size_t)m2 * sizeof(float)));
    hipLaunchKernelGGL(k_met_gather, dim3(grid), dim3(256), 0, st, scores, truth, n, cls, buf, acc);
    if (m2 > m)
        hipLaunchKernelGGL(k_met_fill, dim3((unsigned)((m2 - m + 255) / 256)), dim3(256), 0, st, buf, m, m2);
    hipLaunchKernelGGL(k_bitonic_chunk, dim3((unsigned)(m2 / 2048)), dim3(1024), 0, st, buf, (long long)2048);
    for (long long k = 4096; k <= m2; k <<= 1) {
        for (long long j = k >> 1; j >= 2048; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_global, dim3((unsigned)((m2 / 2 + 255) / 256)), dim3(256), 0, st, buf,
                               m2 / 2, j, k);
        hipLaunchKernelGGL(k_bitonic_tail, dim3((unsigned)(m2 / 2048)), dim3(1024), 0, st, buf, k);
    }
    hipLaunchKernelGGL(k_met_pairs, dim3(grid), dim3(256), 0, st, scores, truth, n, cls, buf, m, acc);
    MCHK(hipGetLastError());
    MCHK(hipMemcpyAsync(&h, acc, sizeof h, hipMemcpyDeviceToHost, st));
    MCHK(hipStreamSynchronize(st));
    {
        const double P = (double)h.cnt[0], N = (double)h.cnt[1];
        const double lo = ord_float(h.lo), hi = ord_float(h.hi);
        const double span = hi - lo;
        out->auc = (double)h.pairs2 / (2.0 * P * N);
        out->auc_tpr_tau = span > 0.0 ? (h.sum[0] / P - lo) / span : 0.0;
        out->auc_fpr_tau = span > 0.0 ? (h.sum[1] / N - lo) / span : 0.0;
        out->auc_td = (out->auc + out->auc_tpr_tau) / 2.0;
        out->auc_bs = (out->auc - out->auc_fpr_tau + 1.0) / 2.0;
        out->positives = (long long)h.cnt[0];
        out->negatives = (long long)h.cnt[1];
        out->excluded = (long long)h.cnt[2];
    }
done:
    if (buf) (void)hipFree(buf);
    if (acc) (void)hipFree(acc);
    return rc;
}
