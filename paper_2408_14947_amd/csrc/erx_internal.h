// Internal declarations shared by the kernels and the C-ABI runtime.
#pragma once
#include <hip/hip_runtime.h>

namespace erx {

enum { DT_F32 = 0, DT_F16 = 1, DT_U16 = 2 };
enum { FLAG_NEED_FP64 = 1, FLAG_FP64_DONE = 2, FLAG_NOTPD = 4 };

constexpr int MAX_NT = 19;   // 16-band tiles: up to 304 bands
constexpr int SCORE_PT = 2;  // 16-pixel tiles per wave in the score kernel

// Entries of the packed per-line statistics: the upper triangle of the band
// covariance as NT(NT+1)/2 tiles of 256 doubles (accumulator layout) followed
// by the 16*NT mean entries.
inline long long stat_entries(int NT) { return (long long)NT * (NT + 1) / 2 * 256 + 16LL * NT; }

hipError_t launch_gram(int dtype, const void* X, int n, int p, int b, int NT, double* stats, long long E,
                       hipStream_t s);
hipError_t launch_scan_local(double* stats, long long E, int n, int seg, long long t0, double alpha,
                             hipStream_t s);
hipError_t launch_scan_carry(const double* stats, double* carry, double* state, long long E, int n, int seg,
                             long long t0, double alpha, hipStream_t s);
hipError_t launch_chol(int fp64, int force, int NT, const double* stats, const double* carry, long long E,
                       int n, int seg, long long t0, double alpha, double eps, int b, float* Mt, float* mu32,
                       int* flags, float* cond, double thr, int want_cond, unsigned long long* ctr,
                       hipStream_t s);
hipError_t launch_score(int dtype, int NT, const void* X, const float* Mt, const float* mu32, int n, int p,
                        int b, float* out, hipStream_t s);
hipError_t launch_normalise(const float* d, float* dn, int n, int p, hipStream_t s);
hipError_t launch_labels(const float* dn, int n, int p, float tau, long long t0, int warmup,
                         unsigned char* out, hipStream_t s);

}  // namespace erx
