// Internal declarations shared by the kernels and the C-ABI runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "../../include/erx.h"

namespace erx {

enum { DT_F32 = 0, DT_F16 = 1, DT_U16 = 2 };
enum { BG_EMA = 0, BG_IMC = 1 };
enum { FLAG_NEED_FP64 = 1, FLAG_FP64_DONE = 2, FLAG_NOTPD = 4, FLAG_SCORE32 = 8 };

constexpr int MAX_NT = 19;   // 16-band tiles: up to 304 bands
constexpr int SCORE_PT = 2;  // 16-pixel tiles per wave in the score kernel

// Entries of the packed per-line statistics: the upper triangle of the band
// covariance as NT(NT+1)/2 tiles of 256 values (accumulator layout) followed
// by the 16*NT mean entries.  The values are FP64, or FP32 in a pass with
// Pass::sf32 set (statistics, scan carries and the stream's state alike).
inline long long stat_entries(int NT) { return (long long)NT * (NT + 1) / 2 * 256 + 16LL * NT; }

// One stream's share of a device pass.  A pass processes lines of one or more
// streams with the same number of 16-band tiles; its lines are numbered
// 0..nlines-1 stream after stream (per-line scratch is indexed by that
// number) and each stream's lines are cut into scan segments of `seg` lines,
// numbered the same way.
struct StreamDesc {
    const void* x;    // first line of the stream in this pass (device memory)
    float* out;       // scores of that line ([n][p])
    float* outn;      // line-normalised scores, or null
    void* state;      // moving-average carry of the stream (stat_entries entries of the
                      // pass's storage type: double, or float when Pass::sf32 is set)
    long long t0;     // lines the stream had absorbed before this pass
    double alpha;     // momentum
    double eps;       // ridge
    int p, b;         // pixels, bands
    int n;            // lines of the stream in this pass
    int line0;        // index of its first line in the pass
    int seg0;         // index of its first scan segment in the pass
    int bg;           // BG_EMA, or BG_IMC (equal weights: statistics hold second moments about
                      // the reference mean kept after the state, see k_imc_moments)
};

struct Pass {
    const StreamDesc* sd;  // device table of nstreams entries, or null for one stream
    StreamDesc one;        // the stream when sd is null
    int nstreams;
    int nlines;            // lines in the pass
    int nseg;              // scan segments in the pass
    int seg;               // lines per scan segment
    int pmax;              // largest pixel count (sizes the score grid)
    int vec4;              // every stream of the pass has a band count divisible by 4
    float* mscale;         // per pass line: max |L^{-1}| (written by the factorisation when
                           // non-null, read by the split-FP16 score kernel)
    int* gredo;            // per pass line and Gram macro tile (GRAM_MACROS_MAX): 1 when the
                           // split-FP16 Gram left it to the FP32 pass; null: no split Gram
    int sf32;              // 1: statistics, carries and states are stored in FP32 (the
                           // averaging itself still runs in FP64); 0: FP64 storage
    int spt;               // 16-pixel tiles per wave of the split-FP16 score kernel: 1, 2, or 0
                           // for 1 from 13 band tiles on and SCORE_PT below
    int gmacro;            // bands per macro tile of the split-FP16 Gram: 64 (k_gram4), 128
                           // (k_gram8), or 0 for 128 from 5 band tiles on and 64 below
};
constexpr int GRAM_MACROS_MAX = 15;  // upper 64x64 macro tiles of a 304-band Gram

// stats / carry: FP64 or (P.sf32) FP32 arrays of stat_entries(NT) values per line / segment
hipError_t launch_gram(int dtype, int prec, const Pass& P, int NT, void* stats, hipStream_t s);
// split-FP16 Gram on 128-band macro tiles; nm = upper 64-band macro tiles (the Pass::gredo stride)
hipError_t launch_gram8(int dtype, const Pass& P, int NT, int nm, void* stats, long long E, hipStream_t s);
hipError_t launch_scan_local(const Pass& P, int NT, void* stats, hipStream_t s);
// IMC: per-line statistics (K_hat, mu_hat) -> second moments about the stream's reference mean
// (FP64 storage only)
hipError_t launch_imc_moments(const Pass& P, int NT, double* stats, hipStream_t s);
hipError_t launch_scan_carry(const Pass& P, int NT, const void* stats, void* carry, hipStream_t s);
// fp64 = 1: FP64 factorisation of every line (force = 1) or of the lines the
// FP32 pass flagged (force = 0).  fp64 = 0: FP32 factorisation; force = 1
// there means no FP64 pass follows, so a failed pivot marks the line not PD.
hipError_t launch_chol(int fp64, int force, const Pass& P, int NT, const void* stats, const void* carry,
                       float* Mt, float* mu32, int* flags, float* cond, double thr, int want_cond,
                       unsigned long long* ctr, hipStream_t s);
// FP32 scores of every line, or (only != null) of the lines flagged FLAG_SCORE32 in only[]
hipError_t launch_score(int dtype, const Pass& P, int NT, const float* Mt, const float* mu32, hipStream_t s,
                        const int* only = nullptr);
// the same scores on FP16 matrix cores with split operands (needs P.mscale); lines it
// cannot represent are flagged FLAG_SCORE32 in flags[] for the FP32 kernel
hipError_t launch_score16(int dtype, const Pass& P, int NT, const float* Mt, const float* mu32, int* flags,
                          hipStream_t s);
hipError_t launch_normalise(const Pass& P, hipStream_t s);
// surrogate projection z - zref = W (x - xref) for npx FP32 pixels of b bands (W: FP16 [16][b])
hipError_t launch_sproj(const float* X, long long npx, int b, const __half* W16, const float* xref, float* Z,
                        hipStream_t s);
// exact (FP64) statistics of one-tile FP32 streams, in the k_gram layout
hipError_t launch_gram1x(const Pass& P, double* stats, hipStream_t s);
// fused path for streams with at most 16 bands: one workgroup per stream, its
// n lines in order, state read from and written back to StreamDesc::state.
// lds_line_bytes > 0 (the largest line of the pass, every line starting on a
// 16-byte boundary) selects the variant that holds the line in LDS when it fits;
// 0 selects the variant that streams every tile from global memory.
hipError_t launch_small(int dtype, const Pass& P, int normalise, unsigned long long* ctr, int lds_line_bytes,
                        hipStream_t s);
// sparse random projection Z = (X - 1 xref^T) W of npix pixels of b bands (W device FP32 [b][d],
// xref FP32 [b], Z FP32 [npix][d]); launch_srp_ref stores the first pixel of X as xref
hipError_t launch_srp_project(int dtype, const void* X, long long npix, int b, const float* W, const float* xref,
                              int d, float* Z, hipStream_t s);
hipError_t launch_srp_ref(int dtype, const void* X, int b, float* xref, hipStream_t s);
hipError_t launch_labels(const float* dn, int n, int p, float tau, long long t0, int warmup,
                         unsigned char* out, hipStream_t s);

}  // namespace erx
