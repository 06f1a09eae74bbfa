// Learned band-projection surrogate of ERX: kernels and C-ABI front end.
//
// A stated change to the method, the learned analogue of the sparse random
// projection of Sec. III-B.  For a stream of b-band lines:
//     z     = W x + c                     (16 outputs; W held in FP16 for the
//                                          projection, FP32 master copy)
//     u     = L_z^{-1} (z - mu_z)          ERX (Sec. III-C/D) on the z stream
//     o     = w2 . relu(A1 u + a1) + c2    (16 -> 64 -> 1)
//     score = ||u|| exp(o)
// Training minimises mean (log score - log target)^2 over the pixels of a
// batch of consecutive lines of a stream (scored from its first line), the
// targets being plain-ERX scores; mu_z and L_z are held fixed in the gradient.
// Adam with FP32 master weights; FP16 copies of the weights (W, A1, w2) are
// refreshed at every step and used by every forward pass (biases stay FP32).
// The loss and the gradient are summed in a fixed order (per-workgroup
// partials, then one ordered reduction), so a step is deterministic.
//
// Inference runs as one kernel per call, a workgroup per line: projection,
// the line's mean and covariance, the moving average through a decoupled
// look-back over the preceding lines of the launch, the 16x16 factorisation
// and the network, reading each line once.
//
// The surrogate detector scores a stream with the surrogate and checks it:
// every R-th line is scored twice more, by plain ERX and by the surrogate, both
// on backgrounds that see only the check lines (momentum 1 - (1 - alpha)^R),
// so that the comparison measures the projection and the network and not the
// difference between a check-line background and the full one; when the median
// over the line's pixels of |log surrogate - log plain| exceeds theta on two
// consecutive checks, the stream switches to plain ERX, re-initialised from
// the next line.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/erx.h"
#include "erx_device.h"
#include "erx_internal.h"
#include "erx_runtime.h"

using namespace erx;

#define fail erx::set_error
#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return fail(ERX_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

namespace {

constexpr int SK = ERX_SURR_K;       // projection width
constexpr int SH = ERX_SURR_HIDDEN;  // hidden units
constexpr int SEG = 64;              // scan segment of the projected stream
constexpr double SURR_RIDGE = 1e-5;  // ridge of the projected stream
constexpr float LOSS_WCAP = 100.f;   // largest weight of a pixel in the training loss

struct Off {
    int W, c, A1, a1, w2, c2, n;
};
__host__ __device__ inline Off offsets(int b)
{
    Off o;
    o.W = 0;
    o.c = SK * b;
    o.A1 = o.c + SK;
    o.a1 = o.A1 + SH * SK;
    o.w2 = o.a1 + SH;
    o.c2 = o.w2 + SH;
    o.n = o.c2 + 1;
    return o;
}

// ---------------------------------------------------------------- kernels
// Per pixel: u = M (z - mu), the network, the score; with TRAIN also the loss
// term, d loss / d log score (G), the hidden pre-activations, u and
// d loss / dz, for the reduction kernel.  One workgroup per (line, 256
// pixels); M (from the transposed accumulator-layout tile of the ERX pass), mu
// and the network in LDS.
template <bool TRAIN>
__global__ __launch_bounds__(256) void k_surr_pix(const float* __restrict__ Z, int p, int ngrp,
                                                  const float* __restrict__ Mt, const float* __restrict__ mu32,
                                                  const float* __restrict__ P, const __half* __restrict__ P16,
                                                  int offA1, int offa1, int offw2,
                                                  int offc2, float* __restrict__ out, const float* __restrict__ target,
                                                  float* __restrict__ U, float* __restrict__ Pre,
                                                  float* __restrict__ G, float* __restrict__ dZ,
                                                  float* __restrict__ lossp, float inv_n, float inv_b)
{
    __shared__ float Ms[SK * SK];  // M[r][q]
    __shared__ float A1s[SH * SK];
    __shared__ float a1s[SH], w2s[SH], mus[SK];
    __shared__ float red[4];
    const int line = blockIdx.x / ngrp, grp = blockIdx.x - line * ngrp;
    const int tid = threadIdx.x;
    {
        const int r = tid >> 4, q = tid & 15;  // Mt holds M^T: element (r, q) of M at lane 16(q/4)+r, reg q%4
        Ms[r * SK + q] = Mt[(size_t)line * 256 + (16 * (q >> 2) + r) * 4 + (q & 3)];
    }
    for (int i = tid; i < SH * SK; i += 256) A1s[i] = __half2float(P16[offA1 + i]);
    if (tid < SH) {
        a1s[tid] = P[offa1 + tid];
        w2s[tid] = __half2float(P16[offw2 + tid]);
    }
    if (tid < SK) mus[tid] = mu32[(size_t)line * SK + tid];
    const float c2 = P[offc2];
    __syncthreads();
    const int px = grp * 256 + tid;
    const bool ok = px < p;
    const size_t idx = (size_t)line * p + (ok ? px : 0);
    float r[SK], u[SK];
    const float* zr = Z + idx * SK;
#pragma unroll
    for (int q = 0; q < SK; ++q) r[q] = zr[q] - mus[q];
    float nu2 = 0.f;
#pragma unroll
    for (int i = 0; i < SK; ++i) {
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < SK; ++q) s += Ms[i * SK + q] * r[q];
        u[i] = s;
        nu2 += s * s;
    }
    float o = c2;
    float pre[TRAIN ? SH : 1];
#pragma unroll
    for (int j = 0; j < SH; ++j) {
        float s = a1s[j];
#pragma unroll
        for (int i = 0; i < SK; ++i) s += A1s[j * SK + i] * u[i];
        if (TRAIN) pre[j] = s;
        o += w2s[j] * fmaxf(s, 0.f);
    }
    if (!TRAIN) {
        if (ok) out[idx] = sqrtf(nu2) * expf(o);
        return;
    }
    // weight of the pixel: its plain-ERX distance squared over the band count (about 1
    // for background, whose squared distance averages b), clamped to [1, LOSS_WCAP]
    const float t = ok ? target[idx] : 1.f;
    const float wt = fminf(LOSS_WCAP, fmaxf(1.f, t * t * inv_b));
    const float e = ok ? 0.5f * logf(nu2) + o - logf(t) : 0.f;
    const float g = 2.f * wt * e * inv_n;
    float dU[SK];
#pragma unroll
    for (int i = 0; i < SK; ++i) dU[i] = g * u[i] / nu2;
#pragma unroll
    for (int j = 0; j < SH; ++j) {
        const float dp = pre[j] > 0.f ? g * w2s[j] : 0.f;
#pragma unroll
        for (int i = 0; i < SK; ++i) dU[i] += dp * A1s[j * SK + i];
    }
    if (ok) {
        G[idx] = g;
        float* ur = U + idx * SK;
        float* dz = dZ + idx * SK;
#pragma unroll
        for (int i = 0; i < SK; ++i) ur[i] = u[i];
#pragma unroll
        for (int q = 0; q < SK; ++q) {  // dz = M^T du
            float s = 0.f;
#pragma unroll
            for (int i = 0; i < SK; ++i) s += dU[i] * Ms[i * SK + q];
            dz[q] = s;
        }
        float* pr = Pre + idx * SH;
#pragma unroll
        for (int j = 0; j < SH; ++j) pr[j] = pre[j];
    }
    // loss: wave sums, then one partial per workgroup (summed in order by k_sum_ordered)
    float e2 = wt * e * e * inv_n;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) e2 += __shfl_xor(e2, m);
    if ((tid & 63) == 0) red[tid >> 6] = e2;
    __syncthreads();
    if (tid == 0) lossp[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out[e] = sum over k of part[k * stride + e], k in order (one thread per entry)
__global__ __launch_bounds__(256) void k_sum_ordered(const float* __restrict__ part, int nk, long long stride,
                                                     int n, float* __restrict__ out)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    float s = 0.f;
    for (int k = 0; k < nk; ++k) s += part[(size_t)k * stride + e];
    out[e] = s;
}

// Gradient sums over a chunk of pixels, one thread per parameter entry (the
// parameter layout: W [16][b], c [16], A1 [64][16], a1 [64], w2 [64], c2);
// chunk k writes its sums to gpart[k][.] for the ordered reduction.
__global__ __launch_bounds__(256) void k_surr_reduce(const float* __restrict__ X, int b, long long npx, int chunk,
                                                     const float* __restrict__ U, const float* __restrict__ Pre,
                                                     const float* __restrict__ G, const float* __restrict__ dZ,
                                                     const __half* __restrict__ P16, float* __restrict__ gpart)
{
    const Off off = offsets(b);
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= off.n) return;
    const long long p0 = (long long)blockIdx.y * chunk;
    const long long p1 = std::min<long long>(npx, p0 + chunk);
    float s = 0.f;
    if (e < off.c) {  // dW[o][k] = sum dz_o x_k
        const int o = e / b, k = e - o * b;
        for (long long px = p0; px < p1; ++px) s += dZ[px * SK + o] * X[px * b + k];
    } else if (e < off.A1) {  // dc = sum dz
        const int o = e - off.c;
        for (long long px = p0; px < p1; ++px) s += dZ[px * SK + o];
    } else if (e < off.a1) {  // dA1[j][i] = sum [pre_j > 0] g w2_j u_i
        const int j = (e - off.A1) / SK, i = (e - off.A1) % SK;
        const float w2j = __half2float(P16[off.w2 + j]);
        for (long long px = p0; px < p1; ++px)
            s += Pre[px * SH + j] > 0.f ? G[px] * w2j * U[px * SK + i] : 0.f;
    } else if (e < off.w2) {  // da1[j] = sum [pre_j > 0] g w2_j
        const int j = e - off.a1;
        const float w2j = __half2float(P16[off.w2 + j]);
        for (long long px = p0; px < p1; ++px) s += Pre[px * SH + j] > 0.f ? G[px] * w2j : 0.f;
    } else if (e < off.c2) {  // dw2[j] = sum g relu(pre_j)
        const int j = e - off.w2;
        for (long long px = p0; px < p1; ++px) s += G[px] * fmaxf(Pre[px * SH + j], 0.f);
    } else {  // dc2 = sum g
        for (long long px = p0; px < p1; ++px) s += G[px];
    }
    gpart[(size_t)blockIdx.y * off.n + e] = s;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ P, const float* __restrict__ grad,
                                              float* __restrict__ m, float* __restrict__ v, __half* __restrict__ P16,
                                              int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float g = grad[e];
    const float mm = b1 * m[e] + (1.f - b1) * g;
    const float vv = b2 * v[e] + (1.f - b2) * g * g;
    m[e] = mm;
    v[e] = vv;
    const float w = P[e] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    P[e] = w;
    P16[e] = __float2half(w);
}

__global__ __launch_bounds__(256) void k_to_half(const float* __restrict__ P, __half* __restrict__ P16, int n)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e < n) P16[e] = __float2half(P[e]);
}


// ---------------------------------------------------------------- fused inference
// One workgroup per line of the launch, in the order of a ticket taken at its
// start (so a workgroup only ever waits for workgroups that are already
// running, which never wait for it):
//  1. z - zref = W (x - xref) for the line's pixels (FP32 matrix cores, FP16 W),
//     kept in LDS (band-major, padded rows);
//  2. the line's mean and covariance (divisor p - 1) of z with FP64 products;
//  3. the moving average (Eqs. (20)-(21)) as a decoupled look-back (the
//     single-pass scan of Merrill and Garland, 2016): the workgroup publishes
//     its aggregate (a_l S_l, decay 1 - a_l), combines the aggregates of the
//     preceding lines until it meets one whose inclusive value is published
//     (or the state the previous launch left), and publishes its own inclusive
//     value C_l = (1 - a_l) C_{l-1} + a_l S_l.  Flags carry the launch's epoch,
//     so nothing is cleared between launches;
//  4. L L^T = K_l + eps I in FP64 by one wave, M = L^{-1};
//  5. per pixel u = M (z - mu_l), the network and the score.
// A wait that does not end within a bounded number of polls marks the launch
// failed (err) and the line is scored NaN; every wave always reaches the end.
constexpr int FP_MAX = 1024;         // pixels of a line the fused kernel holds in LDS
constexpr int ZS = FP_MAX + 4;       // LDS row of one projected band (padding against bank conflicts)
constexpr int FW = 8;                // waves per workgroup
constexpr int SE = SK * SK + SK;     // moving-average state: K row-major [16][16], then mu [16]
constexpr int SPIN_LIMIT = 1 << 22;  // polls of a look-back flag before the launch is declared failed

template <bool VEC>
__global__ __launch_bounds__(FW * 64) void k_surr_fused(const float* __restrict__ X, int p, int b, int NTx,
                                                       const __half* __restrict__ P16,
                                                       const float* __restrict__ P32, Off off,
                                                       const float* __restrict__ xref, double alpha, long long t0,
                                                       double eps, const double* __restrict__ fs_in,
                                                       double* __restrict__ fs_out,
                                                       double* __restrict__ lval, double* __restrict__ ldec,
                                                       unsigned* __restrict__ lflag,
                                                       unsigned long long* __restrict__ ticket,
                                                       unsigned long long tbase, unsigned epoch,
                                                       float* __restrict__ out, int* __restrict__ err)
{
    __shared__ f4 Wt[MAX_NT * 64];       // W tiles in operand form (as k_sproj)
    __shared__ float xr_s[16 * MAX_NT];
    __shared__ float zs[SK * ZS];        // zs[q * ZS + px]
    __shared__ double red_s[FW][256];
    __shared__ double msum_s[32][16];
    __shared__ double S_s[SE];           // the line's statistics
    __shared__ double C_s[SE];           // the moving average after the line
    __shared__ double L_s[SK * 17];
    __shared__ float M_s[SK * SK], mu_s[SK];
    __shared__ float A1s[SH * SK], a1s[SH], w2s[SH];
    __shared__ int line_s, status_s, kind_s, bad_s;
    __shared__ double coef_s[65];

    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
    constexpr int NTH = FW * 64;
    if (tid == 0) {
        line_s = (int)(atomicAdd(ticket, 1ull) - tbase);
        bad_s = 0;
    }
    for (int i = tid; i < NTx * 64; i += NTH) {
        const int K = i >> 6, l = i & 63, gg = l >> 4, cc = l & 15;
        f4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int band = 16 * K + 4 * gg + q;
            v[q] = band < b ? __half2float(P16[off.W + cc * b + band]) : 0.f;
        }
        Wt[i] = v;
    }
    for (int i = tid; i < 16 * NTx; i += NTH) xr_s[i] = i < b ? xref[i] : 0.f;
    for (int i = tid; i < SH * SK; i += NTH) A1s[i] = __half2float(P16[off.A1 + i]);
    if (tid < SH) {
        a1s[tid] = P32[off.a1 + tid];
        w2s[tid] = __half2float(P16[off.w2 + tid]);
    }
    __syncthreads();
    const int L = line_s;
    const float* Xl = X + (size_t)L * p * b;

    // 1. projection of the line into LDS
    const int ntile = (p + 15) >> 4;
    // every band load of a tile is issued before its products, so that each wave keeps
    // up to MAX_NT loads in flight (one workgroup per CU: the loads in flight set the
    // bandwidth)
    for (int tt = w; tt < ntile; tt += FW) {
        const int px = 16 * tt + c;
        const bool okp = px < p;
        f4 v[MAX_NT];
#pragma unroll
        for (int K = 0; K < MAX_NT; ++K) {
            if (K < NTx) {
                const int band0 = 16 * K + 4 * g;
                const bool okl = okp && band0 < b;
                v[K] = ldq<DT_F32, VEC>(Xl, okl ? (size_t)px * b + band0 : 0, okl ? b - band0 : 0);
            }
        }
        f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int K = 0; K < MAX_NT; ++K) {
            if (K < NTx) {
                const int band0 = 16 * K + 4 * g;
                const bool okl = okp && band0 < b;
                f4 r;
#pragma unroll
                for (int q = 0; q < 4; ++q) r[q] = (okl && band0 + q < b) ? v[K][q] - xr_s[band0 + q] : 0.f;
                acc = mma_xty(acc, Wt[K * 64 + lane], r);
            }
        }
        if (okp) {
#pragma unroll
            for (int q = 0; q < 4; ++q) zs[(4 * g + q) * ZS + px] = acc[q];
        }
    }
    __syncthreads();

    // 2. mean, then the centred covariance from FP64 differences and FP64 products
    {
        const int j = tid >> 5, k0 = tid & 31;
        double sm = 0.0;
        for (int px = k0; px < p; px += 32) sm += (double)zs[j * ZS + px];
        msum_s[k0][j] = sm;
    }
    __syncthreads();
    if (tid < SK) {
        double sm = 0.0;
        for (int k = 0; k < 32; ++k) sm += msum_s[k][tid];
        S_s[SK * SK + tid] = sm / (double)p;
    }
    __syncthreads();
    {
        const double mc = S_s[SK * SK + c];
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
        for (int tt = w; tt < ntile; tt += FW) {
            d4 xv;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int px = 16 * tt + 4 * g + i;
                xv[i] = px < p ? (double)zs[c * ZS + px] - mc : 0.0;
            }
            acc = mma_xty(acc, xv, xv);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) red_s[w][(4 * i + g) * 16 + c] = acc[i];  // FP64 layout: row 4i+g
    }
    __syncthreads();
    if (tid < SK * SK) {
        double sm = 0.0;
#pragma unroll
        for (int v = 0; v < FW; ++v) sm += red_s[v][tid];
        S_s[tid] = sm / (double)(p - 1);
    }
    __syncthreads();

    // 3. moving average by decoupled look-back
    const double a = (t0 + L == 0) ? 1.0 : alpha, dL = 1.0 - a;
    const unsigned fA = 2u * epoch + 1u, fP = 2u * epoch + 2u;
    // publication: the barrier completes every wave's stores to the (per-XCD) L2, then one
    // agent-scope release by the flag's writer makes them visible device-wide
    if (tid < SE) lval[((size_t)L * 2) * SE + tid] = a * S_s[tid];
    if (tid == 0) ldec[L] = dL;
    __syncthreads();
    if (tid == 0) __hip_atomic_store(&lflag[L], fA, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    double accv = 0.0;  // this thread's entry of the exclusive prefix C_{L-1}
    if (dL != 0.0) {
        // Windows of 64 preceding lines, newest first: wave 0 polls their flags at once
        // (lane k the line j0 - k) until each holds at least an aggregate, and finds the
        // newest line whose inclusive value is published (or the start of the launch);
        // then every thread folds the aggregates before it into its entry.
        double accd = 1.0;  // product of the decays of the lines folded so far
        int j0 = L - 1;
        for (;;) {
            if (w == 0) {
                const int j = j0 - lane;
                int st = 3;  // before the launch: the state the previous launch left
                if (j >= 0) {
                    unsigned f = 0;
                    for (int it = 0; it < SPIN_LIMIT; ++it) {
                        f = __hip_atomic_load(&lflag[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (f >= fA) break;
                        __builtin_amdgcn_s_sleep(1);
                    }
                    st = f == fP ? 2 : (f == fA ? 1 : 0);
                }
                // one acquire for the flags just read: the values they publish (and, through
                // the CU's caches, the whole workgroup's later loads) are current
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const unsigned long long stop = __ballot(st >= 2), lost = __ballot(st == 0);
                const int d = stop ? __builtin_ctzll(stop) : 64;  // aggregates to fold first
                const bool lostw = (lost & (d == 64 ? ~0ull : ((1ull << d) - 1))) != 0;
                // coefficient of lane k's term: accd times the decays of the newer lines of
                // the window (an exclusive prefix product over the lanes)
                double dk = (lane < d && st == 1) ? ldec[j] : 1.0;
                double incl = dk;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    const double o = __shfl_up(incl, off);
                    if (lane >= off) incl *= o;
                }
                double excl = __shfl_up(incl, 1);
                if (lane == 0) excl = 1.0;
                coef_s[lane] = accd * excl;
                if (lane == 63) coef_s[64] = accd * incl;
                if (lane == 0) status_s = lostw ? 0 : 1 + 4 * d;  // 0: failed, else 1 + 4 d
                if (lane == (d < 64 ? d : 0)) kind_s = d < 64 ? st : 1;  // what ends the window
            }
            __syncthreads();
            const int code = status_s, kind = kind_s;
            if (code == 0) {  // no progress: give up on this line
                if (tid == 0) {
                    bad_s = 1;
                    atomicOr(err, 1);
                }
                break;
            }
            const int d = (code - 1) >> 2;
            if (tid < SE) {
                double sacc = 0.0;
#pragma unroll 8
                for (int k = 0; k < d; ++k) {
                    const double cf = coef_s[k];
                    const double v = lval[((size_t)(j0 - k) * 2) * SE + tid];
                    sacc += cf != 0.0 ? cf * v : 0.0;  // a zero coefficient: lines before the stream's first
                }
                if (d < 64) {
                    const double cf = coef_s[d];
                    if (cf != 0.0) {
                        if (kind == 2) sacc += cf * lval[((size_t)(j0 - d) * 2 + 1) * SE + tid];
                        else sacc += cf * fs_in[tid];
                    }
                }
                accv += sacc;
            }
            accd = coef_s[64];
            const bool done = d < 64 || accd == 0.0;
            __syncthreads();  // the window's shared values are rewritten by the next one
            if (done) break;
            j0 -= 64;
        }
    }
    __syncthreads();
    const bool bad = bad_s != 0;
    if (tid < SE) {
        double v = a * S_s[tid];
        if (dL != 0.0) v += dL * accv;
        if (bad) v = __builtin_nan("");
        C_s[tid] = v;
        lval[((size_t)L * 2 + 1) * SE + tid] = v;
    }
    __syncthreads();
    if (tid == 0) __hip_atomic_store(&lflag[L], fP, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    // the next launch of the stream starts from here (a second slot: lines of this launch
    // may still read the state this launch started from)
    if (L == (int)gridDim.x - 1 && tid < SE) fs_out[tid] = C_s[tid];

    // 4. L L^T = K + eps I: lanes 0..15 of wave 0, lane i owning row i (kept in its own
    //    row of L_s; values of other rows arrive by shuffles), then M = L^{-1} by columns
    if (tid < SK) {
        const int i = tid;
        double* row = L_s + i * 17;
#pragma unroll 1
        for (int k = 0; k < SK; ++k) row[k] = C_s[i * SK + k] + (i == k ? eps : 0.0);
        bool ok = true;
#pragma unroll 1
        for (int k = 0; k < SK; ++k) {
            const double dkk = __shfl(row[k], k, SK);
            ok = ok && dkk > 0.0;
            const double d = sqrt(fmax(dkk, 0.0));
            const double lik = i > k ? row[k] / d : (i == k ? d : 0.0);
            row[k] = lik;
#pragma unroll 1
            for (int jj = k + 1; jj < SK; ++jj) {
                const double ljk = __shfl(lik, jj, SK);
                if (i > k && jj <= i) row[jj] -= lik * ljk;
            }
        }
        if (!ok) bad_s = 1;  // not positive definite
    }
    __syncthreads();
    if (tid < SK) {  // column tid of L^{-1}
        const int j = tid;
        double m[SK];
#pragma unroll
        for (int ii = 0; ii < SK; ++ii) {
            double v = ii == j ? 1.0 : 0.0;
            if (ii > j) {
#pragma unroll
                for (int k = 0; k < ii; ++k)
                    if (k >= j) v -= L_s[ii * 17 + k] * m[k];
            }
            m[ii] = ii < j ? 0.0 : v / L_s[ii * 17 + ii];
        }
#pragma unroll
        for (int ii = 0; ii < SK; ++ii) M_s[ii * SK + j] = (float)m[ii];
        mu_s[tid] = (float)C_s[SK * SK + tid];
    }
    __syncthreads();

    // 5. scores: u = M (z - mu), o = w2 . relu(A1 u + a1) + c2, score = ||u|| exp(o)
    const bool badl = bad_s != 0;
    const float c2 = P32[off.c2];
    for (int px = tid; px < p; px += NTH) {
        float rr[SK];
#pragma unroll
        for (int q = 0; q < SK; ++q) rr[q] = zs[q * ZS + px] - mu_s[q];
        float u[SK], nu2 = 0.f;
#pragma unroll
        for (int ii = 0; ii < SK; ++ii) {
            float sm = 0.f;
#pragma unroll
            for (int q = 0; q <= ii; ++q) sm = fmaf(M_s[ii * SK + q], rr[q], sm);
            u[ii] = sm;
            nu2 = fmaf(sm, sm, nu2);
        }
        float o = c2;
#pragma unroll 8
        for (int jj = 0; jj < SH; ++jj) {
            float sm = a1s[jj];
#pragma unroll
            for (int ii = 0; ii < SK; ++ii) sm = fmaf(A1s[jj * SK + ii], u[ii], sm);
            o = fmaf(w2s[jj], fmaxf(sm, 0.f), o);
        }
        out[(size_t)L * p + px] = badl ? __builtin_nanf("") : sqrtf(nu2) * expf(o);
    }
}

// ERX workspace of a projected (16-band) stream
struct Erx16 {
    long long cap = 0;  // lines
    int capp = 0;       // pixels
    float* Z = nullptr;
    double* stats = nullptr;
    double* carry = nullptr;
    float* Mt = nullptr;
    float* mu32 = nullptr;
    int* flags = nullptr;
    float* cond = nullptr;
    double* state = nullptr;
    float* xref = nullptr;  // the stream's first pixel
    unsigned long long* ctr = nullptr;
    // fused inference: two state slots, the look-back values, decays and flags of
    // the lines of a launch, the ticket counter and the failure flag
    double* fstate = nullptr;  // [2][SE]
    double* lval = nullptr;    // [cap][2][SE]
    double* ldec = nullptr;    // [cap]
    unsigned* lflag = nullptr; // [cap]
    unsigned long long* ticket = nullptr;
    int* err = nullptr;
    unsigned epoch = 0;             // launches so far (the next launch uses epoch + 1)
    unsigned long long tickets = 0; // tickets taken so far
    void release()
    {
        void* d[] = {Z, stats, carry, Mt, mu32, flags, cond, state, xref, ctr, fstate, lval, ldec, lflag, ticket, err};
        for (void* q : d)
            if (q) (void)hipFree(q);
        *this = Erx16();
    }
    hipError_t ensure(long long n, int p)
    {
        if (!state) {
            if (hipMalloc(&state, stat_entries(1) * sizeof(double)) != hipSuccess ||
                hipMalloc(&xref, ERX_MAX_BANDS * sizeof(float)) != hipSuccess ||
                hipMalloc(&ctr, 4 * sizeof(unsigned long long)) != hipSuccess ||
                hipMalloc(&fstate, 2 * SE * sizeof(double)) != hipSuccess ||
                hipMalloc(&ticket, sizeof(unsigned long long)) != hipSuccess ||
                hipMalloc(&err, sizeof(int)) != hipSuccess ||
                hipMemset(state, 0, stat_entries(1) * sizeof(double)) != hipSuccess ||
                hipMemset(fstate, 0, 2 * SE * sizeof(double)) != hipSuccess ||
                hipMemset(ticket, 0, sizeof(unsigned long long)) != hipSuccess ||
                hipMemset(err, 0, sizeof(int)) != hipSuccess ||
                hipMemset(ctr, 0, 4 * sizeof(unsigned long long)) != hipSuccess)
                return hipErrorOutOfMemory;
        }
        if (n <= cap && p <= capp) return hipSuccess;
        const long long N = std::max(n, cap);
        const int Pp = std::max(p, capp);
        void* d[] = {Z, stats, carry, Mt, mu32, flags, cond, lval, ldec, lflag};
        for (void* q : d)
            if (q) (void)hipFree(q);
        Z = nullptr;
        stats = carry = lval = ldec = nullptr;
        Mt = mu32 = cond = nullptr;
        flags = nullptr;
        lflag = nullptr;
        const long long E = stat_entries(1);
        const long long nseg = (N + SEG - 1) / SEG + 2;
        if (hipMalloc(&Z, (size_t)N * Pp * SK * sizeof(float)) != hipSuccess ||
            hipMalloc(&stats, (size_t)N * E * sizeof(double)) != hipSuccess ||
            hipMalloc(&carry, (size_t)nseg * E * sizeof(double)) != hipSuccess ||
            hipMalloc(&Mt, (size_t)N * 256 * sizeof(float)) != hipSuccess ||
            hipMalloc(&mu32, (size_t)N * SK * sizeof(float)) != hipSuccess ||
            hipMalloc(&flags, (size_t)N * sizeof(int)) != hipSuccess ||
            hipMalloc(&cond, (size_t)N * sizeof(float)) != hipSuccess ||
            hipMalloc(&lval, (size_t)N * 2 * SE * sizeof(double)) != hipSuccess ||
            hipMalloc(&ldec, (size_t)N * sizeof(double)) != hipSuccess ||
            hipMalloc(&lflag, (size_t)N * sizeof(unsigned)) != hipSuccess ||
            hipMemset(lflag, 0, (size_t)N * sizeof(unsigned)) != hipSuccess)
            return hipErrorOutOfMemory;
        cap = N;
        capp = Pp;
        return hipSuccess;
    }
    // statistics and inverse factors of the n projected lines in Z (state carried)
    hipError_t pass(hipStream_t s, int n, int p, double alpha, long long t0, float* dummy_out)
    {
        Pass P{};
        P.sd = nullptr;
        P.one.x = Z;
        P.one.out = dummy_out;
        P.one.outn = nullptr;
        P.one.state = state;
        P.one.t0 = t0;
        P.one.alpha = alpha;
        P.one.eps = SURR_RIDGE;
        P.one.p = p;
        P.one.b = SK;
        P.one.n = n;
        P.nstreams = 1;
        P.nlines = n;
        P.nseg = (n + SEG - 1) / SEG;
        P.seg = SEG;
        P.pmax = p;
        P.vec4 = 1;
        hipError_t e;
        if ((e = launch_gram1x(P, stats, s)) != hipSuccess) return e;
        if ((e = launch_scan_local(P, 1, stats, s)) != hipSuccess) return e;
        if ((e = launch_scan_carry(P, 1, stats, carry, s)) != hipSuccess) return e;
        return launch_chol(1, 1, P, 1, stats, carry, Mt, mu32, flags, cond, 0.0, 0, ctr, s);
    }
    // the fused kernel over n lines of b bands (p <= FP_MAX): scores into out
    hipError_t fused(hipStream_t s, const float* X, int n, int p, int b, const __half* P16, const float* P32,
                     const Off& off, double alpha, long long t0, float* out)
    {
        const unsigned ep = epoch + 1;
        const double* fin = fstate + (size_t)(ep & 1) * SE;
        double* fout = fstate + (size_t)((ep + 1) & 1) * SE;
        const int NTx = (b + 15) / 16;
        const dim3 grid((unsigned)n), block(FW * 64);
        if (b % 4 == 0 && (uintptr_t)X % 16 == 0)
            hipLaunchKernelGGL(k_surr_fused<true>, grid, block, 0, s, X, p, b, NTx, P16, P32, off, xref, alpha, t0,
                               SURR_RIDGE, fin, fout, lval, ldec, lflag, ticket, tickets, ep, out, err);
        else
            hipLaunchKernelGGL(k_surr_fused<false>, grid, block, 0, s, X, p, b, NTx, P16, P32, off, xref, alpha, t0,
                               SURR_RIDGE, fin, fout, lval, ldec, lflag, ticket, tickets, ep, out, err);
        const hipError_t e = hipGetLastError();
        if (e == hipSuccess) {
            epoch = ep;
            tickets += (unsigned long long)n;
        }
        return e;
    }
    // the failure flag of the fused launches so far (waits for the stream)
    hipError_t failed(hipStream_t s, bool* out)
    {
        int v = 0;
        hipError_t e = hipMemcpyAsync(&v, err, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        *out = v != 0;
        return e;
    }
};

bool is_device(const void* ptr)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

}  // namespace

struct erx_surr {
    int b = 0;
    Off off{};
    float* P = nullptr;
    float* grad = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    __half* P16 = nullptr;  // FP16 copy of every parameter (the kernels read W, A1 and w2 from it)
    float* loss = nullptr;
    long long step = 0;
    hipStream_t stream = nullptr;
    Erx16 erx;
    // training workspace
    long long capN = 0;
    float* U = nullptr;
    float* Pre = nullptr;
    float* G = nullptr;
    float* dZ = nullptr;
    float* dummy = nullptr;
    float* lossp = nullptr;  // per-workgroup loss partials
    float* gpart = nullptr;  // per-chunk gradient partials
    long long capParts = 0;
};

struct erx_sdet {
    erx_surr* net = nullptr;
    int p = 0;
    float alpha = 0.f, theta = 0.f;
    int R = 0;
    long long t = 0;
    bool active = true;
    int drift_run = 0;
    long long checks = 0, drifts = 0, switched_at = -1;
    double drift_sum = 0.0;
    float drift_last = 0.f, drift_max = 0.f;
    erx_ctx* monitor = nullptr;  // plain ERX on the check lines
    erx_ctx* plain = nullptr;    // plain ERX after a switch (made up front: switching allocates nothing)
    hipStream_t stream = nullptr;
    Erx16 erx;                   // the surrogate's projected stream
    Erx16 mon16;                 // the surrogate on the check lines
    float* mscore = nullptr;
    float alpha_r = 0.f;
    float* scores = nullptr;
    long long cap = 0;
    int last_n = 0;
    float* dummy = nullptr;
    std::vector<float> hs, hp;
};

namespace {

// projection of n lines into erx.Z; at the first line of a stream (t0 == 0)
// the stream's reference pixel xref is set to its first pixel
hipError_t project(erx_surr* net, hipStream_t s, Erx16& erx, const float* X, long long npx, long long t0)
{
    if (t0 == 0) {
        const hipError_t e = hipMemcpyAsync(erx.xref, X, net->b * sizeof(float), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return launch_sproj(X, npx, net->b, net->P16, erx.xref, erx.Z, s);
}

// Surrogate scores of n lines continuing the stream held by erx (t0 lines before).
// Lines of at most FP_MAX pixels take the fused kernel; longer ones the staged
// path (projection, the ERX pass on z, the per-pixel network).  A stream keeps
// one pixel count, so it stays on one path.
hipError_t net_forward(erx_surr* net, hipStream_t s, Erx16& erx, const float* X, int n, int p, double alpha,
                       long long t0, float* out, float* dummy)
{
    if (p <= FP_MAX) {
        if (t0 == 0) {
            const hipError_t e = hipMemcpyAsync(erx.xref, X, net->b * sizeof(float), hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return e;
        }
        return erx.fused(s, X, n, p, net->b, net->P16, net->P, net->off, alpha, t0, out);
    }
    const long long npx = (long long)n * p;
    hipError_t e = project(net, s, erx, X, npx, t0);
    if (e != hipSuccess) return e;
    if ((e = erx.pass(s, n, p, alpha, t0, dummy)) != hipSuccess) return e;
    const int ngrp = (p + 255) / 256;
    hipLaunchKernelGGL((k_surr_pix<false>), dim3((unsigned)((long long)n * ngrp)), dim3(256), 0, s, erx.Z, p, ngrp,
                       erx.Mt, erx.mu32, net->P, net->P16, net->off.A1, net->off.a1, net->off.w2, net->off.c2, out,
                       nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0.f, 0.f);
    return hipGetLastError();
}

}  // namespace

extern "C" {

erx_surr* erx_surrogate_create(int bands, unsigned long long seed)
{
    if (bands < 1 || bands > ERX_MAX_BANDS) {
        fail(ERX_EINVAL, "erx_surrogate_create: bands must be in [1, %d]", ERX_MAX_BANDS);
        return nullptr;
    }
    erx_surr* net = new (std::nothrow) erx_surr();
    if (!net) {
        fail(ERX_ENOMEM, "out of host memory");
        return nullptr;
    }
    net->b = bands;
    net->off = offsets(bands);
    const int n = net->off.n;
    // initialisation: W ~ N(0, 1/b), A1 ~ N(0, 1/16), w2 ~ N(0, 0.01^2), biases 0
    std::vector<float> h(n, 0.f);
    unsigned long long st = seed * 0x9E3779B97F4A7C15ull + 1;
    auto unif = [&]() {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        return ((st >> 11) + 0.5) / 9007199254740992.0;
    };
    auto normal = [&]() { return std::sqrt(-2.0 * std::log(unif())) * std::cos(6.283185307179586 * unif()); };
    for (int i = 0; i < SK * bands; ++i) h[net->off.W + i] = (float)(normal() / std::sqrt((double)bands));
    for (int i = 0; i < SH * SK; ++i) h[net->off.A1 + i] = (float)(normal() / std::sqrt((double)SK));
    for (int i = 0; i < SH; ++i) h[net->off.w2 + i] = (float)(0.01 * normal());
    bool ok = hipStreamCreateWithFlags(&net->stream, hipStreamNonBlocking) == hipSuccess &&
              hipMalloc(&net->P, n * sizeof(float)) == hipSuccess &&
              hipMalloc(&net->grad, n * sizeof(float)) == hipSuccess &&
              hipMalloc(&net->m, n * sizeof(float)) == hipSuccess && hipMalloc(&net->v, n * sizeof(float)) == hipSuccess &&
              hipMalloc(&net->P16, n * sizeof(__half)) == hipSuccess &&
              hipMalloc(&net->loss, sizeof(float)) == hipSuccess &&
              hipMemcpy(net->P, h.data(), n * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
              hipMemset(net->grad, 0, n * sizeof(float)) == hipSuccess &&
              hipMemset(net->m, 0, n * sizeof(float)) == hipSuccess &&
              hipMemset(net->v, 0, n * sizeof(float)) == hipSuccess;
    if (ok) {
        hipLaunchKernelGGL(k_to_half, dim3((n + 255) / 256), dim3(256), 0, net->stream, net->P, net->P16, n);
        ok = hipStreamSynchronize(net->stream) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        erx_surrogate_destroy(net);
        fail(ERX_ENOMEM, "erx_surrogate_create: device allocation failed");
        return nullptr;
    }
    return net;
}

void erx_surrogate_destroy(erx_surr* net)
{
    if (!net) return;
    if (net->stream) (void)hipStreamSynchronize(net->stream);
    void* d[] = {net->P,  net->grad, net->m,  net->v,     net->P16,   net->loss, net->U,
                 net->Pre, net->G,    net->dZ, net->dummy, net->lossp, net->gpart};
    for (void* q : d)
        if (q) (void)hipFree(q);
    net->erx.release();
    if (net->stream) (void)hipStreamDestroy(net->stream);
    delete net;
}

int erx_surrogate_num_params(const erx_surr* net)
{
    if (!net) return fail(ERX_EINVAL, "NULL surrogate");
    return net->off.n;
}

int erx_surrogate_set_params(erx_surr* net, const float* params)
{
    if (!net || !params) return fail(ERX_EINVAL, "NULL argument");
    HIPCHK(hipMemcpyAsync(net->P, params, net->off.n * sizeof(float), hipMemcpyHostToDevice, net->stream));
    HIPCHK(hipMemsetAsync(net->m, 0, net->off.n * sizeof(float), net->stream));
    HIPCHK(hipMemsetAsync(net->v, 0, net->off.n * sizeof(float), net->stream));
    hipLaunchKernelGGL(k_to_half, dim3((net->off.n + 255) / 256), dim3(256), 0, net->stream, net->P, net->P16,
                       net->off.n);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(net->stream));
    net->step = 0;
    return ERX_OK;
}

int erx_surrogate_get_params(const erx_surr* net, float* params)
{
    if (!net || !params) return fail(ERX_EINVAL, "NULL argument");
    HIPCHK(hipMemcpyAsync(params, net->P, net->off.n * sizeof(float), hipMemcpyDeviceToHost, net->stream));
    HIPCHK(hipStreamSynchronize(net->stream));
    return ERX_OK;
}

int erx_surrogate_scores(erx_surr* net, const float* lines, int n, int pixels, float momentum, float* out)
{
    if (!net || !lines || !out || n < 1 || pixels < 2 || !(momentum > 0.f && momentum <= 1.f))
        return fail(ERX_EINVAL, "erx_surrogate_scores: invalid arguments");
    if (!is_device(lines) || !is_device(out)) return fail(ERX_EINVAL, "lines and out must be device memory");
    if (((uintptr_t)lines % 4) || ((uintptr_t)out % 4)) return fail(ERX_EINVAL, "buffers must be 4-byte aligned");
    HIPCHK(net->erx.ensure(n, pixels));
    if (!net->dummy) HIPCHK(hipMalloc(&net->dummy, (size_t)net->erx.cap * net->erx.capp * sizeof(float)));
    HIPCHK(hipMemsetAsync(net->erx.state, 0, stat_entries(1) * sizeof(double), net->stream));
    HIPCHK(net_forward(net, net->stream, net->erx, lines, n, pixels, momentum, 0, out, net->dummy));
    bool bad = false;
    HIPCHK(net->erx.failed(net->stream, &bad));
    if (bad) return fail(ERX_EDEVICE, "erx_surrogate_scores: a look-back wait did not complete");
    return ERX_OK;
}

int erx_surrogate_train_step(erx_surr* net, const float* lines, const float* targets, int n, int pixels,
                             float momentum, float lr, float* loss)
{
    if (!net || !lines || !targets || n < 1 || pixels < 2 || !(momentum > 0.f && momentum <= 1.f) || !(lr >= 0.f))
        return fail(ERX_EINVAL, "erx_surrogate_train_step: invalid arguments");
    if (!is_device(lines) || !is_device(targets)) return fail(ERX_EINVAL, "lines and targets must be device memory");
    if (((uintptr_t)lines % 4) || ((uintptr_t)targets % 4)) return fail(ERX_EINVAL, "buffers must be 4-byte aligned");
    hipStream_t s = net->stream;
    HIPCHK(net->erx.ensure(n, pixels));
    const long long N = (long long)n * pixels;
    if (N > net->capN || !net->dummy) {
        void* d[] = {net->U, net->Pre, net->G, net->dZ, net->dummy};
        for (void* q : d)
            if (q) (void)hipFree(q);
        const long long C = std::max<long long>(N, (long long)net->erx.cap * net->erx.capp);
        if (hipMalloc(&net->U, C * SK * sizeof(float)) != hipSuccess ||
            hipMalloc(&net->Pre, C * SH * sizeof(float)) != hipSuccess ||
            hipMalloc(&net->G, C * sizeof(float)) != hipSuccess ||
            hipMalloc(&net->dZ, C * SK * sizeof(float)) != hipSuccess ||
            hipMalloc(&net->dummy, C * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            net->U = net->Pre = net->G = net->dZ = net->dummy = nullptr;
            net->capN = 0;
            return fail(ERX_ENOMEM, "erx_surrogate_train_step: cannot allocate the workspace");
        }
        net->capN = C;
    }
    // forward pass of the projection and the ERX statistics of the z stream
    HIPCHK(hipMemsetAsync(net->erx.state, 0, stat_entries(1) * sizeof(double), s));
    HIPCHK(project(net, s, net->erx, lines, N, 0));
    HIPCHK(net->erx.pass(s, n, pixels, momentum, 0, net->dummy));
    // per-pixel forward and backward, then the gradient sums, each in a fixed order
    const int ngrp = (pixels + 255) / 256;
    const long long nblk = (long long)n * ngrp;
    const int chunk = 256;
    const long long nch = (N + chunk - 1) / chunk;
    const long long parts = std::max<long long>(nblk, nch * net->off.n);
    if (parts > net->capParts) {
        if (net->lossp) (void)hipFree(net->lossp);
        if (net->gpart) (void)hipFree(net->gpart);
        net->lossp = net->gpart = nullptr;
        net->capParts = 0;
        if (hipMalloc(&net->lossp, parts * sizeof(float)) != hipSuccess ||
            hipMalloc(&net->gpart, parts * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ERX_ENOMEM, "erx_surrogate_train_step: cannot allocate the reduction buffers");
        }
        net->capParts = parts;
    }
    hipLaunchKernelGGL((k_surr_pix<true>), dim3((unsigned)nblk), dim3(256), 0, s, net->erx.Z, pixels, ngrp,
                       net->erx.Mt, net->erx.mu32, net->P, net->P16, net->off.A1, net->off.a1, net->off.w2,
                       net->off.c2, nullptr, targets, net->U, net->Pre, net->G, net->dZ, net->lossp,
                       (float)(1.0 / (double)N), (float)(1.0 / (double)net->b));
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_sum_ordered, dim3(1), dim3(256), 0, s, net->lossp, (int)nblk, 1LL, 1, net->loss);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_surr_reduce, dim3((unsigned)((net->off.n + 255) / 256), (unsigned)nch), dim3(256), 0, s,
                       lines, net->b, N, chunk, net->U, net->Pre, net->G, net->dZ, net->P16, net->gpart);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_sum_ordered, dim3((unsigned)((net->off.n + 255) / 256)), dim3(256), 0, s, net->gpart,
                       (int)nch, (long long)net->off.n, net->off.n, net->grad);
    HIPCHK(hipGetLastError());
    if (lr > 0.f) {
        ++net->step;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - std::pow(b1, (float)net->step), c2 = 1.f - std::pow(b2, (float)net->step);
        hipLaunchKernelGGL(k_adam, dim3((net->off.n + 255) / 256), dim3(256), 0, s, net->P, net->grad, net->m, net->v,
                           net->P16, net->off.n, lr, b1, b2, 1e-8f, c1, c2);
        HIPCHK(hipGetLastError());
    }
    float l = 0.f;
    HIPCHK(hipMemcpyAsync(&l, net->loss, sizeof(float), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (loss) *loss = l;
    return ERX_OK;
}

int erx_surrogate_grads(const erx_surr* net, float* grads)
{
    if (!net || !grads) return fail(ERX_EINVAL, "NULL argument");
    HIPCHK(hipMemcpyAsync(grads, net->grad, net->off.n * sizeof(float), hipMemcpyDeviceToHost, net->stream));
    HIPCHK(hipStreamSynchronize(net->stream));
    return ERX_OK;
}

// ------------------------------------------------------------ surrogate detector
erx_sdet* erx_surrogate_detector_create(erx_surr* net, int pixels, float momentum, float drift_threshold,
                                        int check_every)
{
    if (!net || pixels < 2 || !(momentum > 0.f && momentum <= 1.f) || !(drift_threshold > 0.f) || check_every < 1) {
        fail(ERX_EINVAL, "erx_surrogate_detector_create: invalid arguments");
        return nullptr;
    }
    erx_sdet* sd = new (std::nothrow) erx_sdet();
    if (!sd) {
        fail(ERX_ENOMEM, "out of host memory");
        return nullptr;
    }
    sd->net = net;
    sd->p = pixels;
    sd->alpha = momentum;
    sd->theta = drift_threshold;
    sd->R = check_every;
    sd->alpha_r = (float)(1.0 - std::pow(1.0 - (double)momentum, (double)check_every));
    erx_config c;
    erx_config_default(&c, net->b, pixels, sd->alpha_r);
    c.block_lines = 1;
    c.scan_lines = 1;
    sd->monitor = erx_create_ex(&c);
    erx_config cp;
    erx_config_default(&cp, net->b, pixels, momentum);
    cp.block_lines = 256;  // lines per pass of the fallback detector
    sd->plain = erx_create_ex(&cp);
    bool ok = sd->monitor && sd->plain && hipStreamCreateWithFlags(&sd->stream, hipStreamNonBlocking) == hipSuccess &&
              erx_set_stream(sd->monitor, sd->stream) == ERX_OK && erx_set_stream(sd->plain, sd->stream) == ERX_OK &&
              hipMalloc(&sd->dummy, (size_t)pixels * 256 * sizeof(float)) == hipSuccess &&
              hipMalloc(&sd->mscore, (size_t)pixels * sizeof(float)) == hipSuccess &&
              sd->erx.ensure(256, pixels) == hipSuccess && sd->mon16.ensure(1, pixels) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        erx_surrogate_detector_destroy(sd);
        fail(ERX_ENOMEM, "erx_surrogate_detector_create: allocation failed");
        return nullptr;
    }
    return sd;
}

void erx_surrogate_detector_destroy(erx_sdet* sd)
{
    if (!sd) return;
    if (sd->stream) (void)hipStreamSynchronize(sd->stream);
    if (sd->monitor) erx_destroy(sd->monitor);
    if (sd->plain) erx_destroy(sd->plain);
    if (sd->scores) (void)hipFree(sd->scores);
    if (sd->dummy) (void)hipFree(sd->dummy);
    if (sd->mscore) (void)hipFree(sd->mscore);
    sd->erx.release();
    sd->mon16.release();
    if (sd->stream) (void)hipStreamDestroy(sd->stream);
    delete sd;
}

int erx_surrogate_detector_push(erx_sdet* sd, const float* lines, int n)
{
    if (!sd || !lines || n < 1) return fail(ERX_EINVAL, "erx_surrogate_detector_push: invalid arguments");
    if (!is_device(lines) || ((uintptr_t)lines % 4)) return fail(ERX_EINVAL, "lines must be aligned device memory");
    const int p = sd->p, b = sd->net->b;
    if (n > sd->cap) {
        if (sd->scores) (void)hipFree(sd->scores);
        sd->scores = nullptr;
        if (hipMalloc(&sd->scores, (size_t)n * p * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            sd->cap = 0;
            return fail(ERX_ENOMEM, "cannot allocate the score buffer");
        }
        sd->cap = n;
    }
    hipStream_t s = sd->stream;
    const size_t lsz = (size_t)p * b;
    int done = 0;
    while (done < n) {
        if (!sd->active) {  // plain ERX from here on
            const int k = n - done;
            if (erx_push_lines_ex(sd->plain, lines + (size_t)done * lsz, k) != ERX_OK) return ERX_EDEVICE;
            const int rc = erx_scores_device(sd->plain, sd->scores + (size_t)done * p);
            if (rc != ERX_OK && rc != ERX_ENOTPD) return rc;
            done = n;
            break;
        }
        // surrogate block up to (and including) the next check line
        const long long t0 = sd->t + done;
        const long long next_check = ((t0 / sd->R) + 1) * sd->R - 1;  // global index of the next check line
        const int k = (int)std::min<long long>({(long long)(n - done), next_check - t0 + 1, 256});
        const float* X = lines + (size_t)done * lsz;
        HIPCHK(net_forward(sd->net, s, sd->erx, X, k, p, sd->alpha, t0, sd->scores + (size_t)done * p, sd->dummy));
        done += k;
        const long long last = t0 + k - 1;
        if (last == next_check) {  // the check line: plain ERX on the monitor state
            const float* xc = lines + (size_t)(done - 1) * lsz;
            if (erx_push_lines_ex(sd->monitor, xc, 1) != ERX_OK) return ERX_EDEVICE;
            HIPCHK(net_forward(sd->net, s, sd->mon16, xc, 1, p, sd->alpha_r, sd->checks, sd->mscore, sd->dummy));
            sd->hs.resize(p);
            sd->hp.resize(p);
            HIPCHK(hipMemcpyAsync(sd->hs.data(), sd->mscore, p * sizeof(float), hipMemcpyDeviceToHost, s));
            bool bad1 = false, bad2 = false;
            HIPCHK(sd->erx.failed(s, &bad1));
            HIPCHK(sd->mon16.failed(s, &bad2));
            if (bad1 || bad2) return fail(ERX_EDEVICE, "surrogate detector: a look-back wait did not complete");
            const int rc = erx_scores(sd->monitor, sd->hp.data());
            if (rc != ERX_OK && rc != ERX_ENOTPD) return rc;
            std::vector<float> dev(p);
            for (int i = 0; i < p; ++i) dev[i] = std::fabs(std::log(sd->hs[i]) - std::log(sd->hp[i]));
            std::nth_element(dev.begin(), dev.begin() + p / 2, dev.end());
            float med = dev[p / 2];
            if (!(p & 1)) {
                const float lo = *std::max_element(dev.begin(), dev.begin() + p / 2);
                med = 0.5f * (med + lo);
            }
            ++sd->checks;
            sd->drift_last = med;
            sd->drift_sum += med;
            sd->drift_max = std::isnan(med) || med > sd->drift_max ? med : sd->drift_max;
            const bool drift = !(med <= sd->theta);  // NaN counts as drift
            sd->drifts += drift ? 1 : 0;
            sd->drift_run = drift ? sd->drift_run + 1 : 0;
            if (sd->drift_run >= 2) {  // the fallback detector starts from the next line
                sd->active = false;
                sd->switched_at = last + 1;
            }
        }
    }
    sd->t += n;
    sd->last_n = n;
    return ERX_OK;
}

int erx_surrogate_detector_scores(erx_sdet* sd, float* out)
{
    if (!sd || !out) return fail(ERX_EINVAL, "NULL argument");
    if (sd->last_n == 0) return fail(ERX_ESTATE, "no lines pushed yet");
    bool bad = false;
    HIPCHK(sd->erx.failed(sd->stream, &bad));
    if (bad) return fail(ERX_EDEVICE, "surrogate detector: a look-back wait did not complete");
    HIPCHK(hipMemcpyAsync(out, sd->scores, (size_t)sd->last_n * sd->p * sizeof(float), hipMemcpyDefault,
                          sd->stream));
    HIPCHK(hipStreamSynchronize(sd->stream));
    return ERX_OK;
}

int erx_surrogate_detector_drift_stats(const erx_sdet* sd, float* last, float* mean, float* max)
{
    if (!sd) return fail(ERX_EINVAL, "NULL detector");
    if (sd->checks == 0) return fail(ERX_ESTATE, "no check line scored yet");
    if (last) *last = sd->drift_last;
    if (mean) *mean = (float)(sd->drift_sum / (double)sd->checks);
    if (max) *max = sd->drift_max;
    return ERX_OK;
}

int erx_surrogate_detector_status(const erx_sdet* sd, int* active, long long* checks, long long* drifts,
                                  long long* switched_at)
{
    if (!sd) return fail(ERX_EINVAL, "NULL detector");
    if (active) *active = sd->active ? 1 : 0;
    if (checks) *checks = sd->checks;
    if (drifts) *drifts = sd->drifts;
    if (switched_at) *switched_at = sd->switched_at;
    return ERX_OK;
}

}  // extern "C"
