// HIP kernels of the ERX hot path for gfx950 (CDNA4).
//
// One pass over a block of n consecutive lines of one stream runs:
//   k_gram        per-line mean and centred Gram on FP32 matrix cores
//                 (paper Sec. III-C, Eqs. (18)-(19))
//   k_scan_local  segment-local exponential moving average (Eqs. (20)-(21))
//   k_scan_carry  carries between segments (and into the next pass)
//   k_chol        ridge + Cholesky + triangular inverse + condition estimate
//                 (Sec. III-D), FP32 with an FP64 re-factor of flagged lines
//   k_score       residual, whitening product L^{-1}(x - mu), row norm
//                 (Sec. III-D, Eqs. (22)-(23)) on FP32 matrix cores
//   k_normalise   line-wise standardisation (Sec. III-E, Eq. (24))
//
// Matrix tiles are 16x16 and are kept in the accumulator layout of the
// 16x16x4 MFMA instructions: lane l = 16*g + c holds four rows of column c
// (FP32: register i <-> row 4g+i; FP64: register i <-> row 4i+g).  With that
// layout four MFMAs whose A and B operands are register i of two such tiles
// X and Y compute X^T Y (in the same layout), so tiles produced by one
// product feed the next without any data movement.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <type_traits>

#include "erx_internal.h"

namespace erx {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

template <class T> struct VT;
template <> struct VT<float> { typedef f4 v; };
template <> struct VT<double> { typedef d4 v; };

// Row held by lane (g, c), register i, of a 16x16 accumulator tile.  The
// 16x16x4 FP32 MFMA places row 4g+i there, the FP64 one row 4i+g.  Products
// X^T Y are layout-agnostic (the contraction runs over every row once), so
// only code that names rows explicitly uses this.
template <class T> __device__ __forceinline__ int rowof(int g, int i)
{
    return std::is_same<T, double>::value ? 4 * i + g : 4 * g + i;
}

__device__ __forceinline__ f4 mfma(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4 mfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// acc += X^T Y for two accumulator-layout tiles held as register quadruples
template <class V>
__device__ __forceinline__ V mma_xty(V acc, const V x, const V y)
{
    acc = mfma(x[0], y[0], acc);
    acc = mfma(x[1], y[1], acc);
    acc = mfma(x[2], y[2], acc);
    acc = mfma(x[3], y[3], acc);
    return acc;
}

// ---------------------------------------------------------------- input loads
template <int DT> __device__ __forceinline__ float ld1(const void* X, size_t i);
template <> __device__ __forceinline__ float ld1<DT_F32>(const void* X, size_t i)
{
    return ((const float*)X)[i];
}
template <> __device__ __forceinline__ float ld1<DT_F16>(const void* X, size_t i)
{
    return __half2float(((const __half*)X)[i]);
}
template <> __device__ __forceinline__ float ld1<DT_U16>(const void* X, size_t i)
{
    return (float)((const uint16_t*)X)[i] * (1.0f / 65536.0f);  // exact
}

// four consecutive bands [band0, band0+4) of one pixel row; bands >= b read 0
template <int DT>
__device__ __forceinline__ f4 ld4(const void* X, size_t row, int band0, int b)
{
    f4 v;
    if (band0 + 4 <= b && (b & 3) == 0) {
        const size_t i = row + band0;
        if (DT == DT_F32) {
            v = *(const f4*)((const float*)X + i);
        } else if (DT == DT_F16) {
            const uint2 u = *(const uint2*)((const __half*)X + i);
            const __half2 h0 = *(const __half2*)&u.x, h1 = *(const __half2*)&u.y;
            const float2 a = __half22float2(h0), c = __half22float2(h1);
            v = f4{a.x, a.y, c.x, c.y};
        } else {
            const uint2 u = *(const uint2*)((const uint16_t*)X + i);
            const float s = 1.0f / 65536.0f;
            v = f4{(float)(u.x & 0xffffu) * s, (float)(u.x >> 16) * s,
                   (float)(u.y & 0xffffu) * s, (float)(u.y >> 16) * s};
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (band0 + q < b) ? ld1<DT>(X, row + band0 + q) : 0.0f;
    }
    return v;
}

template <int DT> __device__ __forceinline__ const void* advance(const void* x, size_t elems)
{
    return (const char*)x + elems * (DT == DT_F32 ? 4 : 2);
}

// the stream owning pass line `line` (streams are stored in line order)
__device__ __forceinline__ StreamDesc stream_of_line(const Pass& P, int line)
{
    if (!P.sd) return P.one;
    int lo = 0, hi = P.nstreams - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P.sd[mid].line0 <= line) lo = mid;
        else hi = mid - 1;
    }
    return P.sd[lo];
}

// the stream owning pass scan segment `g`
__device__ __forceinline__ StreamDesc stream_of_seg(const Pass& P, int g)
{
    if (!P.sd) return P.one;
    int lo = 0, hi = P.nstreams - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (P.sd[mid].seg0 <= g) lo = mid;
        else hi = mid - 1;
    }
    return P.sd[lo];
}

__device__ __forceinline__ long long tile_u(int I, int J, int NT)  // upper tile I <= J
{
    return (long long)I * NT - (long long)I * (I - 1) / 2 + (J - I);
}

// ============================================================================
// Gram: per line, mean and centred covariance (Sec. III-C, Eqs. (18)-(19)).
//
// A workgroup of 4 waves computes one 64x64 block ("macro tile", 4x4 tiles of
// 16 bands) of the upper triangle of the band x band Gram matrix of one line;
// wave w owns tile row 4*MI+w.  Pixels are the contraction index.
//
// Data are shifted by s = the FP32 mean of the first min(64, p) pixels of each
// band (the same value in every workgroup).  Chunks of GCH pixels of the 64
// row bands and the 64 column bands are loaded with 16-byte loads (one chunk
// ahead, in registers), shifted, and stored transposed in LDS (band-major,
// pixels contiguous), so that one 16-byte LDS read gives a lane the operands
// of four consecutive MFMA k-steps.  Products are accumulated on FP32 MFMA
// over 64-pixel chunks and the chunk partials are summed in FP64; the exact
// identity
//     sum (x-mu)(x-mu)^T = sum (x-s)(x-s)^T - p (mu-s)(mu-s)^T
// turns the shifted sums into the centred covariance.
//
// Grid: 8 * ceil(n/8) * nmacro workgroups; block ids are spread so that all
// macro tiles of one line run on the same XCD (consecutive block ids are
// dispatched round-robin over the 8 XCDs) and share its L2.
// ============================================================================
constexpr int GCH = 32;           // pixels per LDS chunk
constexpr int GTS = GCH + 4;      // LDS stride of one band row (floats), 16-byte aligned
constexpr int GSR = 16 * GCH / 256;  // float4 per thread per panel and chunk
constexpr int GSG = 256 / GCH;       // band-group stride between a thread's float4

// four consecutive bands of one pixel row; bands >= b read 0.  With
// vec_ok (b % 4 == 0, band0 % 4 == 0) the four bands are all valid or all
// invalid, so one predicated 16-byte (8-byte) load serves.
template <int DT>
__device__ __forceinline__ f4 ld4_any(const void* X, size_t row, int band0, int b, bool vec_ok)
{
    f4 v = f4{0.f, 0.f, 0.f, 0.f};
    if (vec_ok) {
        if (band0 >= b) return v;
        const size_t i = row + band0;
        if (DT == DT_F32) {
            v = *(const f4*)((const float*)X + i);
        } else if (DT == DT_F16) {
            const uint2 u = *(const uint2*)((const __half*)X + i);
            const float2 a = __half22float2(*(const __half2*)&u.x), c = __half22float2(*(const __half2*)&u.y);
            v = f4{a.x, a.y, c.x, c.y};
        } else {
            const uint2 u = *(const uint2*)((const uint16_t*)X + i);
            const float s = 1.0f / 65536.0f;
            v = f4{(float)(u.x & 0xffffu) * s, (float)(u.x >> 16) * s, (float)(u.y & 0xffffu) * s,
                   (float)(u.y >> 16) * s};
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = (band0 + q < b) ? ld1<DT>(X, row + band0 + q) : 0.0f;
    }
    return v;
}

// MFMA products of one LDS chunk for NQ column tiles (unconditional, so the
// accumulators stay in place): lane group g supplies pixels u+4g..u+4g+3 for
// the four k-steps of each 16-pixel group.
template <int NQ>
__device__ __forceinline__ void gram_chunk(const float* Rt, const float* Cp, int w, int c, int g, int kend,
                                           f4* acc)
{
    for (int u = 0; u < kend; u += 16) {
        const f4 av = *(const f4*)&Rt[(16 * w + c) * GTS + u + 4 * g];
        f4 bv[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) bv[q] = *(const f4*)&Cp[(16 * q + c) * GTS + u + 4 * g];
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] = mfma(av[st], bv[q][st], acc[q]);
    }
}

template <int DT>
__global__ __launch_bounds__(256) void k_gram(const Pass P, int NT, int nmacro, double* __restrict__ stats,
                                              long long E)
{
    const int bid = blockIdx.x;
    const int xcd = bid & 7;
    const int kk = bid >> 3;
    const int ll = kk / nmacro;
    int m = kk - ll * nmacro;
    const int line = ll * 8 + xcd;
    if (line >= P.nlines) return;  // uniform for the workgroup
    const StreamDesc d = stream_of_line(P, line);
    const int p = d.p, b = d.b;
    const void* X = advance<DT>(d.x, (size_t)(line - d.line0) * p * b);
    const int MT = (NT + 3) >> 2;
    int MI = 0;
    while (m >= MT - MI) {
        m -= MT - MI;
        ++MI;
    }
    const int MJ = MI + m;
    const bool dg = (MI == MJ);
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63, g = lane >> 4, c = lane & 15;
    const int I = 4 * MI + w;  // this wave's tile row
    const bool rowok = I < NT;
    const int rb0 = 64 * MI, cb0 = 64 * MJ;  // first band of the row / column panels

    __shared__ __attribute__((aligned(16))) float Rt[64 * GTS];  // [band][pixel]
    __shared__ __attribute__((aligned(16))) float Ct[64 * GTS];
    __shared__ float shift_s[128];
    __shared__ double bsum_s[128];

    const size_t lbase = 0;
    const bool vec_ok = (b & 3) == 0;
    // staging map: a panel chunk is GCH pixels x 16 groups of 4 bands; thread
    // tid handles pixel tid % GCH of band groups tid / GCH + GSG * r, so that
    // consecutive lanes write consecutive LDS words
    const int spx = tid % GCH, sg0 = tid / GCH;
    f4 pr[GSR], pc[GSR];
    auto fetch = [&](int k0) __attribute__((always_inline)) {
        const int px = k0 + spx;
        const bool okp = px < p;
        const size_t row = lbase + (size_t)(okp ? px : 0) * b;
#pragma unroll
        for (int r = 0; r < GSR; ++r) {
            const int b4 = 4 * (sg0 + GSG * r);
            pr[r] = okp ? ld4_any<DT>(X, row, rb0 + b4, b, vec_ok) : f4{0.f, 0.f, 0.f, 0.f};
            if (!dg) pc[r] = okp ? ld4_any<DT>(X, row, cb0 + b4, b, vec_ok) : f4{0.f, 0.f, 0.f, 0.f};
        }
    };

    // shift from the first min(64, p) pixels, summed in pixel order
    const int p0 = p < 64 ? p : 64;
    if (tid < 128) {
        const int col = tid & 63;
        const int band = (tid < 64 ? rb0 : cb0) + col;
        float sum = 0.f;
        if (band < b)
            for (int k = 0; k < p0; ++k) sum += ld1<DT>(X, lbase + (size_t)k * b + band);
        shift_s[tid] = (band < b) ? sum / (float)p0 : 0.f;
    }
    fetch(0);
    __syncthreads();
    auto stage = [&](int k0) __attribute__((always_inline)) {
        const bool okp = k0 + spx < p;
#pragma unroll
        for (int r = 0; r < GSR; ++r)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int band = 4 * (sg0 + GSG * r) + j;
                Rt[band * GTS + spx] = okp ? pr[r][j] - shift_s[band] : 0.f;
                if (!dg) Ct[band * GTS + spx] = okp ? pc[r][j] - shift_s[64 + band] : 0.f;
            }
    };
    // band sums of the shifted values: thread tid sums band (tid & 63) of panel
    // (tid >> 6) & 1 over half (tid >> 7) of each chunk, straight from LDS
    const int sband = tid & 63, spanel = (tid >> 6) & 1, shalf = tid >> 7;
    const float* sumsrc = (spanel && !dg) ? Ct : Rt;
    double bpart = 0.0;
    const float* Cp = dg ? Rt : Ct;

    // column tiles of this macro (the lower tiles of a diagonal macro are
    // computed with the others and simply not stored)
    const int nq = __builtin_amdgcn_readfirstlane((NT - 4 * MJ) < 4 ? (NT - 4 * MJ) : 4);
    int tbits = 0;  // column tiles this wave stores (wave-uniform)
#pragma unroll
    for (int q = 0; q < 4; ++q) tbits |= (rowok && (4 * MJ + q) < NT && (!dg || q >= w)) ? (1 << q) : 0;
    tbits = __builtin_amdgcn_readfirstlane(tbits);

    double S[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) S[q][i] = 0.0;
    f4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < p; k0 += GCH) {
        stage(k0);
        __syncthreads();
        if (k0 + GCH < p) fetch(k0 + GCH);  // prefetch the next chunk into registers
        {
            const float* rowp = sumsrc + sband * GTS + (GCH / 2) * shalf;
            float ps = 0.f;
#pragma unroll
            for (int q = 0; q < GCH / 8; ++q) {
                const f4 v = *(const f4*)(rowp + 4 * q);
                ps += (v[0] + v[1]) + (v[2] + v[3]);
            }
            bpart += (double)ps;
        }
        if (rowok) {
            const int kend = (p - k0) < GCH ? (p - k0) : GCH;
            switch (nq) {
            case 1: gram_chunk<1>(Rt, Cp, w, c, g, kend, acc); break;
            case 2: gram_chunk<2>(Rt, Cp, w, c, g, kend, acc); break;
            case 3: gram_chunk<3>(Rt, Cp, w, c, g, kend, acc); break;
            default: gram_chunk<4>(Rt, Cp, w, c, g, kend, acc); break;
            }
        }
        // FP64 sums of the FP32 partials every 64 pixels and at the end
        if (((k0 + GCH) & 63) == 0 || k0 + GCH >= p) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int i = 0; i < 4; ++i) S[q][i] += (double)acc[q][i];
                acc[q] = f4{0.f, 0.f, 0.f, 0.f};
            }
        }
        __syncthreads();  // LDS is rewritten by the next chunk
    }

    // band sums: add the two halves
    if (shalf == 1) bsum_s[spanel * 64 + sband] = bpart;
    __syncthreads();
    if (shalf == 0) bsum_s[spanel * 64 + sband] += bpart;
    __syncthreads();
    if (!rowok) return;

    const double inv_p = 1.0 / (double)p, inv_p1 = 1.0 / (double)(p - 1);
    double* ls = stats + (size_t)line * E;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (!(tbits & (1 << q))) continue;
        const double scol = bsum_s[(dg ? 0 : 64) + 16 * q + c];
        double o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double srho = bsum_s[16 * w + 4 * g + i];  // sum of row band 16I+4g+i
            o[i] = (S[q][i] - srho * scol * inv_p) * inv_p1;
        }
        double* dst = ls + tile_u(I, 4 * MJ + q, NT) * 256 + lane * 4;
        *(double2*)dst = double2{o[0], o[1]};
        *(double2*)(dst + 2) = double2{o[2], o[3]};
    }
    if (dg && g == 0) {
        const long long ntU = (long long)NT * (NT + 1) / 2;
        const int band = 16 * I + c;
        ls[ntU * 256 + band] = (band < b) ? (double)shift_s[16 * w + c] + bsum_s[16 * w + c] * inv_p : 0.0;
    }
}

// ============================================================================
// Exponential moving average as a chunked linear-recurrence scan
// (Sec. III-C, Eqs. (20)-(21)).  With a_l = 1 for the stream's first line and
// a_l = alpha afterwards, C_l = (1-a_l) C_{l-1} + a_l S_l for every entry of
// the packed statistics.  Pass 1 runs the recurrence inside each segment from
// a zero carry; pass 2 walks the segments to produce the carry entering each
// segment; the Cholesky kernel adds D_l * carry, D_l = prod_{segment start..l}
// (1-a_j), to obtain the full background of line l.
// ============================================================================
__global__ __launch_bounds__(256) void k_scan_local(const Pass P, double* __restrict__ stats, long long E)
{
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= E) return;
    const int gsg = blockIdx.y;  // pass segment
    const StreamDesc d = stream_of_seg(P, gsg);
    const int l0 = (gsg - d.seg0) * P.seg;  // stream-local first line
    const int l1 = (l0 + P.seg) < d.n ? (l0 + P.seg) : d.n;
    const double alpha = d.alpha;
    const long long t0 = d.t0;
    double* ptr = stats + (size_t)d.line0 * E + e;
    double acc = 0.0;
    int l = l0;
    for (; l + 8 <= l1; l += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = ptr[(size_t)(l + q) * E];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double a = (t0 + l + q == 0) ? 1.0 : alpha;
            acc = (1.0 - a) * acc + a * v[q];
            v[q] = acc;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) ptr[(size_t)(l + q) * E] = v[q];
    }
    for (; l < l1; ++l) {
        const double a = (t0 + l == 0) ? 1.0 : alpha;
        acc = (1.0 - a) * acc + a * ptr[(size_t)l * E];
        ptr[(size_t)l * E] = acc;
    }
}

__device__ __forceinline__ double seg_decay(long long t0, int l0, int l1, double alpha)
{
    double P = 1.0;
    for (int l = l0; l < l1; ++l) P *= (t0 + l == 0) ? 0.0 : (1.0 - alpha);
    return P;
}

__global__ __launch_bounds__(256) void k_scan_carry(const Pass P, const double* __restrict__ stats,
                                                    double* __restrict__ carry, long long E)
{
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= E) return;
    const StreamDesc d = P.sd ? P.sd[blockIdx.y] : P.one;
    double cv = d.state[e];
    const int nseg = (d.n + P.seg - 1) / P.seg;
    for (int gs = 0; gs < nseg; ++gs) {
        carry[(size_t)(d.seg0 + gs) * E + e] = cv;
        const int l0 = gs * P.seg;
        const int l1 = (l0 + P.seg) < d.n ? (l0 + P.seg) : d.n;
        cv = seg_decay(d.t0, l0, l1, d.alpha) * cv + stats[(size_t)(d.line0 + l1 - 1) * E + e];
    }
    d.state[e] = cv;
}

// ============================================================================
// Cholesky of A_t = K_t + eps I, inverse factor M = L^{-1}, 1-norm condition
// estimate (Sec. III-D).
//
// One workgroup per line.  The lower triangle of A is held in registers as
// 16x16 tiles spread round-robin over the waves (tile s = I(I+1)/2 + J of
// wave s % NW).  A tile slot holds A_IJ^T until its column is factored, then
// L_IJ^T (panel), then the accumulator T_IJ of the inverse, finally M_IJ.
// Right-looking blocked algorithm, for each block column K:
//   1. the 16x16 diagonal block is factored and inverted by one wave with
//      lane broadcasts;
//   2. panel L_IK^T = L_KK^{-1} A_IK^T and inverse row M_KJ = L_KK^{-1} T_KJ;
//   3. trailing update A_IJ^T -= L_JK L_IK^T and T_IJ -= L_IK M_KJ,
// all on MFMA (FP32, or FP64 for the re-factor pass).  The condition number
// estimate is ||A||_1 times Hager's estimate of ||A^{-1}||_1 (the LAPACK
// xLACN2 iteration), applying A^{-1} = M^T M with the register tiles.
//
// The FP32 pass flags lines whose estimate exceeds the threshold (or whose
// factorisation met a non-positive pivot); the FP64 instantiation then
// re-factors only those lines.  Output: M^T tiles (FP32, accumulator layout,
// the operand form the score kernel needs), mu_t (FP32), flags, estimate.
// ============================================================================
__device__ __forceinline__ float bcast(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double bcast(double v, int l)
{
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1/sqrt(x): the hardware estimate, refined by Newton steps (two for FP64,
// giving close to full double precision; one for FP32).
__device__ __forceinline__ float rsqrt_nr(float x)
{
    float y = __builtin_amdgcn_rsqf(x);
    return y * (1.5f - 0.5f * x * y * y);
}
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = y * (1.5 - 0.5 * x * y * y);
    y = y * (1.5 - 0.5 * x * y * y);
    return y;
}

// Cholesky and inverse of one 16x16 diagonal block by a single wave.
// diag_s holds the block (row-major, stride 17) on entry; xt_s receives
// X = L^{-1} (row-major, stride 17).  Rows of L live in lanes 0..15 and are
// shared with lane broadcasts; the reciprocal pivots are wave-uniform and are
// reused by the inverse, whose columns are computed by lanes 0..15 from the
// broadcast rows of L.  Returns 1 if a pivot was not positive.
template <class T>
__device__ __forceinline__ int factor_diag16(T* diag_s, T* xt_s, int lane)
{
    const int r = lane & 15;
    int bad = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    T a[16], invd[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) a[q] = (q <= r) ? diag_s[r * 17 + q] : (T)0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const T akk = bcast(a[k], k);
        if (!(akk > (T)0) && !(akk != akk)) bad = 1;  // a NaN pivot propagates, it is not "not PD"
        const T inv = rsqrt_nr(akk);
        invd[k] = inv;
        const T lrk = (r > k) ? a[k] * inv : ((r == k) ? akk * inv : (T)0);
        a[k] = lrk;
#pragma unroll
        for (int q = k + 1; q < 16; ++q) {
            const T lqk = bcast(lrk, q);
            if (r >= q) a[q] -= lrk * lqk;
        }
    }
    // X = L^{-1}: lane c (= r) computes column c by forward substitution
    T x[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        T s0 = (q == r) ? (T)1 : (T)0, s1 = (T)0;
#pragma unroll
        for (int k = 0; k < q; ++k) {
            const T lqk = bcast(a[k], q);
            if (k & 1) s1 -= lqk * x[k];
            else s0 -= lqk * x[k];
        }
        x[q] = (s0 + s1) * invd[q];
    }
    if (lane < 16)
#pragma unroll
        for (int q = 0; q < 16; ++q) xt_s[q * 17 + lane] = x[q];  // xt[row][col] = X[row][col]
    return bad;
}

template <int NT> struct CholLds {
    float part[NT * (NT + 1) / 2 * 32];  // per-tile partial sums (norms, mat-vecs)
    float vec[4][16 * NT];                // x, y, z, scratch vectors
    float red[64];
};

template <class T, int NT, int NW>
__global__ __launch_bounds__(NW * 64) void k_chol(const Pass P, const double* __restrict__ stats,
                                                  const double* __restrict__ carry, long long E,
                                                  float* __restrict__ Mt, float* __restrict__ mu32,
                                                  int* __restrict__ flags, float* __restrict__ cond,
                                                  double threshold, int want_cond, int force,
                                                  unsigned long long* __restrict__ counters)
{
    typedef typename VT<T>::v V;
    constexpr int NTL = NT * (NT + 1) / 2;
    constexpr int SLOTS = (NTL + NW - 1) / NW;
    constexpr bool FB = std::is_same<T, double>::value;
    constexpr int BP = 16 * NT;
    const int line = blockIdx.x;
    if (line >= P.nlines) return;
    const StreamDesc sdl = stream_of_line(P, line);
    const int b = sdl.b, seg = P.seg;
    const double eps = sdl.eps, alpha = sdl.alpha;
    const long long t0 = sdl.t0;
    // the FP64 instantiation factors every line (force) or the lines the FP32 pass flagged
    if (FB && !force && !(flags[line] & FLAG_NEED_FP64)) return;  // uniform for the workgroup

    __shared__ __attribute__((aligned(32))) T diag_s[16 * 17];
    __shared__ __attribute__((aligned(32))) T xt_s[16 * 17];
    __shared__ __attribute__((aligned(32))) T panel_s[NT * 256];
    __shared__ __attribute__((aligned(32))) T mrow_s[NT * 256];
    __shared__ __attribute__((aligned(16))) CholLds<NT> aux;
    __shared__ int fail_s;

    const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63,
              g = lane >> 4, c = lane & 15;
    const int lloc = line - sdl.line0;  // stream-local line index
    const int gseg = sdl.seg0 + lloc / seg, l0 = (lloc / seg) * seg;
    double D = 1.0;
    for (int l = l0; l <= lloc; ++l) D *= (t0 + l == 0) ? 0.0 : (1.0 - alpha);
    if (tid == 0) fail_s = 0;

    // ---- load A_IJ^T = (K_loc + D carry)_{JI} (+ eps on the diagonal)
    V A[SLOTS];
    int tI[SLOTS], tJ[SLOTS];
    const double* st = stats + (size_t)line * E;
    const double* cr = carry + (size_t)gseg * E;
#pragma unroll
    for (int j = 0; j < SLOTS; ++j) {
        const int s = j * NW + w;
        int I = -1, J = -1;
        if (s < NTL) {  // scalar decode of the lower-triangle tile index
            I = 0;
            while ((I + 1) * (I + 2) / 2 <= s) ++I;
            J = s - I * (I + 1) / 2;
        }
        tI[j] = I;
        tJ[j] = J;
        if (I >= 0) {
            const long long u = tile_u(J, I, NT) * 256;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = rowof<T>(g, i);  // stored in the FP32 accumulator layout
                const long long o = u + (16 * (row >> 2) + c) * 4 + (row & 3);
                double v = st[o] + D * cr[o];
                const int rb = 16 * J + row, cb = 16 * I + c;
                if (rb == cb) v += eps;
                if (rb >= b || cb >= b) v = (rb == cb) ? 1.0 : 0.0;
                A[j][i] = (T)v;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) A[j][i] = (T)0;
        }
        __builtin_amdgcn_sched_barrier(0);  // bound the number of loads in flight (registers)
    }
    if (!FB || force) {
        const long long ntU = NTL;
        for (int q = tid; q < BP; q += NW * 64) {
            const double v = st[ntU * 256 + q] + D * cr[ntU * 256 + q];
            mu32[(size_t)line * BP + q] = (q < b) ? (float)v : 0.0f;
        }
    }

    // ---- ||A||_1 (row sums of |A| over the real bands), deterministic
    float anorm = 0.f;
    if (want_cond) {
#pragma unroll
        for (int j = 0; j < SLOTS; ++j) {
            if (tI[j] < 0) continue;
            const int s = tI[j] * (tI[j] + 1) / 2 + tJ[j];
            // slot element (row, c) is A[16J+row][16I+c]
            float ra = 0.f;  // row 16I+c of A_IJ: sum over i, then over g
#pragma unroll
            for (int i = 0; i < 4; ++i) ra += fabsf((float)A[j][i]);
            ra += __shfl_xor(ra, 16);
            ra += __shfl_xor(ra, 32);
            float rb[4];  // rows 16J+row of A_JI (mirror), sum over c
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = (tI[j] != tJ[j]) ? fabsf((float)A[j][i]) : 0.f;
                v += __shfl_xor(v, 8);
                v += __shfl_xor(v, 4);
                v += __shfl_xor(v, 2);
                v += __shfl_xor(v, 1);
                rb[i] = v;
            }
            if (g == 0) aux.part[s * 32 + c] = ra;
            if (c == 0)
#pragma unroll
                for (int i = 0; i < 4; ++i) aux.part[s * 32 + 16 + rowof<T>(g, i)] = rb[i];
        }
        __syncthreads();
        float mx = 0.f;
        for (int q = tid; q < BP; q += NW * 64) {
            const int R = q >> 4, r = q & 15;
            float sum = 0.f;
            for (int J = 0; J <= R; ++J) sum += aux.part[(R * (R + 1) / 2 + J) * 32 + r];
            for (int I = R + 1; I < NT; ++I) sum += aux.part[(I * (I + 1) / 2 + R) * 32 + 16 + r];
            if (q < b) mx = fmaxf(mx, sum);
        }
        for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
        if (lane == 0) aux.red[w] = mx;
        __syncthreads();
        mx = 0.f;
        for (int q = 0; q < NW; ++q) mx = fmaxf(mx, aux.red[q]);
        anorm = mx;
        __syncthreads();
    }

    // ---- blocked factorisation and inversion, with a one-step lookahead: the
    //      wave that owns diagonal tile K+1 updates and factors it while the
    //      other waves apply the rest of step K's trailing update
    {
        bool own = false;
#pragma unroll
        for (int j = 0; j < SLOTS; ++j)
            if (tI[j] == 0 && tJ[j] == 0) {
#pragma unroll
                for (int i = 0; i < 4; ++i) diag_s[c * 17 + rowof<T>(g, i)] = A[j][i];
                own = true;
            }
        if (own && factor_diag16(diag_s, xt_s, lane) && lane == 0) fail_s = 1;
    }
    __syncthreads();
    for (int K = 0; K < NT; ++K) {
        // 2. panel L_IK^T = X A_IK^T and inverse row M_KJ = X T_KJ, X = L_KK^{-1}
        V xinvT;  // X^T in accumulator layout: element (row, c) = X[c][row]
#pragma unroll
        for (int i = 0; i < 4; ++i) xinvT[i] = xt_s[c * 17 + rowof<T>(g, i)];
#pragma unroll
        for (int j = 0; j < SLOTS; ++j) {
            if (tJ[j] == K && tI[j] > K) {
                V z = {};
                A[j] = mma_xty(z, xinvT, A[j]);
                *(V*)&panel_s[tI[j] * 256 + lane * 4] = A[j];
            } else if (tI[j] == K && tJ[j] < K) {
                V z = {};
                A[j] = mma_xty(z, xinvT, A[j]);
                *(V*)&mrow_s[tJ[j] * 256 + lane * 4] = A[j];
            } else if (tI[j] == K && tJ[j] == K) {
#pragma unroll
                for (int i = 0; i < 4; ++i) A[j][i] = xt_s[rowof<T>(g, i) * 17 + c];  // M_KK = X
                *(V*)&mrow_s[K * 256 + lane * 4] = A[j];
            }
        }
        __syncthreads();
        // 3a. lookahead: diagonal tile K+1 is updated and factored first
        {
            bool own = false;
#pragma unroll
            for (int j = 0; j < SLOTS; ++j) {
                if (tI[j] == K + 1 && tJ[j] == K + 1) {
                    V xp = *(const V*)&panel_s[(K + 1) * 256 + lane * 4];
                    const V yp = xp;
                    xp = -xp;
                    A[j] = mma_xty(A[j], xp, yp);
#pragma unroll
                    for (int i = 0; i < 4; ++i) diag_s[c * 17 + rowof<T>(g, i)] = A[j][i];
                    own = true;
                }
            }
            if (own && factor_diag16(diag_s, xt_s, lane) && lane == 0) fail_s = 1;
        }
        // 3b. the rest of the trailing update and the inverse accumulators
#pragma unroll
        for (int j = 0; j < SLOTS; ++j) {
            const int I = tI[j], J = tJ[j];
            if (I <= K || (I == K + 1 && J == K + 1)) continue;
            if (J > K) {
                V xp = *(const V*)&panel_s[J * 256 + lane * 4];
                const V yp = *(const V*)&panel_s[I * 256 + lane * 4];
                xp = -xp;
                A[j] = mma_xty(A[j], xp, yp);  // A_IJ^T -= L_JK L_IK^T
            } else {
                V xp = *(const V*)&panel_s[I * 256 + lane * 4];
                const V yp = *(const V*)&mrow_s[J * 256 + lane * 4];
                xp = -xp;
                if (J == K) {
                    V z = {};
                    A[j] = mma_xty(z, xp, yp);  // T_IK = -L_IK M_KK
                } else {
                    A[j] = mma_xty(A[j], xp, yp);  // T_IJ -= L_IK M_KJ
                }
            }
        }
        __syncthreads();
    }
    const int fail = fail_s;

    // ---- M^T tiles for the score kernel, in the FP32 accumulator layout
    //      (element (r,q) of M_JK goes to lane 16(q/4)+r, register q%4)
    {
        float* dstl = Mt + (size_t)line * NTL * 256;
        const bool nanout = FB && fail;
#pragma unroll
        for (int j = 0; j < SLOTS; ++j) {
            if (tI[j] < 0) continue;
            const int s = tI[j] * (tI[j] + 1) / 2 + tJ[j];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int off = 64 * (c >> 2) + 4 * rowof<T>(g, i) + (c & 3);
                dstl[(size_t)s * 256 + off] = nanout ? __builtin_nanf("") : (float)A[j][i];
            }
        }
    }

    // ---- Hager / Higham estimate of ||A^{-1}||_1 with A^{-1} = M^T M
    float est = 0.f;
    if (want_cond && !fail) {
        float* xv = aux.vec[0];
        float* yv = aux.vec[1];
        float* zv = aux.vec[2];
        float* sg = aux.vec[3];
        const int NTH = NW * 64;
        // y <- M x, then z <- M^T y : z = A^{-1} x (x in xv, result in zv)
        auto apply = [&]() __attribute__((always_inline)) {
#pragma unroll
            for (int j = 0; j < SLOTS; ++j) {
                if (tI[j] < 0) continue;
                const int s = tI[j] * (tI[j] + 1) / 2 + tJ[j];
                const float xc = xv[16 * tJ[j] + c];
                float v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    v[i] = (float)A[j][i] * xc;
                    v[i] += __shfl_xor(v[i], 8);
                    v[i] += __shfl_xor(v[i], 4);
                    v[i] += __shfl_xor(v[i], 2);
                    v[i] += __shfl_xor(v[i], 1);
                }
                if (c == 0)
#pragma unroll
                    for (int i = 0; i < 4; ++i) aux.part[s * 32 + rowof<T>(g, i)] = v[i];
            }
            __syncthreads();
            for (int q = tid; q < BP; q += NTH) {
                const int R = q >> 4, r = q & 15;
                float sum = 0.f;
                for (int J = 0; J <= R; ++J) sum += aux.part[(R * (R + 1) / 2 + J) * 32 + r];
                yv[q] = sum;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < SLOTS; ++j) {
                if (tI[j] < 0) continue;
                const int s = tI[j] * (tI[j] + 1) / 2 + tJ[j];
                float v = 0.f;
#pragma unroll
                for (int i = 0; i < 4; ++i) v += (float)A[j][i] * yv[16 * tI[j] + rowof<T>(g, i)];
                v += __shfl_xor(v, 16);
                v += __shfl_xor(v, 32);
                if (g == 0) aux.part[s * 32 + 16 + c] = v;
            }
            __syncthreads();
            for (int q = tid; q < BP; q += NTH) {
                const int Jc = q >> 4, cc = q & 15;
                float sum = 0.f;
                for (int I = Jc; I < NT; ++I) sum += aux.part[(I * (I + 1) / 2 + Jc) * 32 + 16 + cc];
                zv[q] = (q < b) ? sum : 0.f;
            }
            __syncthreads();
        };
        // block reductions over the b real entries of zv
        auto norm1 = [&]() __attribute__((always_inline)) -> float {
            float s = 0.f;
            for (int q = tid; q < b; q += NTH) s += fabsf(zv[q]);
            for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
            if (lane == 0) aux.red[w] = s;
            __syncthreads();
            float t = 0.f;
            for (int q = 0; q < NW; ++q) t += aux.red[q];
            __syncthreads();
            return t;
        };
        auto argmax_abs = [&]() __attribute__((always_inline)) -> int {  // first index of the largest |zv|
            float best = -1.f;
            int bi = 0;
            for (int q = tid; q < b; q += NTH) {
                const float v = fabsf(zv[q]);
                if (v > best) { best = v; bi = q; }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const float ob = __shfl_xor(best, o);
                const int oi = __shfl_xor(bi, o);
                if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
            }
            if (lane == 0) {
                aux.red[w] = best;
                aux.red[32 + w] = __int_as_float(bi);
            }
            __syncthreads();
            float bb = -1.f;
            int ii = 0;
            for (int q = 0; q < NW; ++q) {
                const float v = aux.red[q];
                const int iq = __float_as_int(aux.red[32 + q]);
                if (v > bb || (v == bb && iq < ii)) { bb = v; ii = iq; }
            }
            __syncthreads();
            return ii;
        };
        // x = 1/b
        for (int q = tid; q < BP; q += NTH) xv[q] = (q < b) ? 1.0f / (float)b : 0.f;
        __syncthreads();
        apply();
        est = norm1();
        if (b > 1) {
            // sign vector of y (ties to +1), then z = A^{-1} sign
            for (int q = tid; q < BP; q += NTH) {
                const float sv = (zv[q] >= 0.f) ? 1.f : -1.f;
                sg[q] = sv;
                xv[q] = (q < b) ? sv : 0.f;
            }
            __syncthreads();
            apply();
            int jx = argmax_abs();
            for (int it = 2; it <= 5; ++it) {
                for (int q = tid; q < BP; q += NTH) xv[q] = (q == jx) ? 1.f : 0.f;
                __syncthreads();
                apply();
                const float estold = est;
                const float e2 = norm1();
                est = fmaxf(est, e2);
                // repeated sign vector?
                int diff = 0;
                for (int q = tid; q < b; q += NTH) diff |= (((zv[q] >= 0.f) ? 1.f : -1.f) != sg[q]);
                diff = __syncthreads_or(diff);
                if (!diff || e2 <= estold) break;
                for (int q = tid; q < BP; q += NTH) {
                    const float sv = (zv[q] >= 0.f) ? 1.f : -1.f;
                    sg[q] = sv;
                    xv[q] = (q < b) ? sv : 0.f;
                }
                __syncthreads();
                apply();
                const float zlast = fabsf(zv[jx]);
                const int jn = argmax_abs();
                if (zlast == fabsf(zv[jn])) break;
                jx = jn;
            }
            // alternating-sign safeguard
            for (int q = tid; q < BP; q += NTH)
                xv[q] = (q < b) ? ((q & 1) ? -1.f : 1.f) * (1.f + (float)q / (float)(b - 1)) : 0.f;
            __syncthreads();
            apply();
            const float tmp = 2.f * norm1() / (3.f * (float)b);
            est = fmaxf(est, tmp);
        }
        est *= anorm;
    }

    if (tid == 0) {
        const bool fin = want_cond && !fail && isfinite(est);
        int f;
        if (!FB) {
            f = 0;
            if (fail || threshold <= 0.0 || (want_cond && (double)est > threshold)) f |= FLAG_NEED_FP64;
            cond[line] = fail ? __builtin_inff() : (want_cond ? est : 0.f);
            if (!(f & FLAG_NEED_FP64) && fin) atomicMax((unsigned int*)&counters[2], __float_as_uint(est));
        } else {
            f = (force ? 0 : flags[line]) | FLAG_FP64_DONE | (fail ? FLAG_NOTPD : 0);
            cond[line] = fail ? __builtin_inff() : est;
            if (fin) atomicMax((unsigned int*)&counters[2], __float_as_uint(est));
            atomicAdd(&counters[0], 1ull);
            if (fail) atomicAdd(&counters[1], 1ull);
        }
        flags[line] = f;
    }
}

// ============================================================================
// Score (Sec. III-D, Eqs. (22)-(23)): for each pixel, r = x - mu_t, m = M r
// with M = L_t^{-1} lower triangular, delta = ||m||.  Y_J = sum_{K<=J} M_JK R_K
// for 16-pixel column tiles R_K (bands 16K..16K+15) on FP32 MFMA: the M^T
// tiles are read in operand form and R_K is four consecutive bands of one
// pixel per lane, which is exactly the accumulator-layout operand of X^T Y.
// Each wave scores PT tiles of 16 pixels; a workgroup is 4 waves.
// ============================================================================
template <int NT, int DT>
__global__ __launch_bounds__(256) void k_score(const Pass P, const float* __restrict__ Mt,
                                               const float* __restrict__ mu32, int ngrp)
{
    constexpr int NTL = NT * (NT + 1) / 2;
    constexpr int PT = SCORE_PT;
    const int line = blockIdx.x / ngrp, grp = blockIdx.x - line * ngrp;
    if (line >= P.nlines) return;
    const StreamDesc d = stream_of_line(P, line);
    const int p = d.p, b = d.b;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const int pix0 = (grp * 4 + w) * PT * 16;
    if (pix0 >= p) return;  // wave-uniform; the kernel has no barrier
    const void* X = advance<DT>(d.x, (size_t)(line - d.line0) * p * b);
    float* out = d.out + (size_t)(line - d.line0) * p;
    const float* mu = mu32 + (size_t)line * 16 * NT;
    const float* Ml = Mt + (size_t)line * NTL * 256 + lane * 4;
    const size_t lrow = 0;

    f4 acc[NT][PT];
#pragma unroll
    for (int J = 0; J < NT; ++J)
#pragma unroll
        for (int t = 0; t < PT; ++t) acc[J][t] = f4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
    for (int K = 0; K < NT; ++K) {
        const int band0 = 16 * K + 4 * g;
        const f4 m4 = *(const f4*)(mu + band0);
        f4 y[PT];
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            const int pix = pix0 + 16 * t + c;
            if (pix < p) {
                y[t] = ld4<DT>(X, (lrow + pix) * (size_t)b, band0, b) - m4;
                // padded bands read 0 and have mu 0
            } else {
                y[t] = f4{0.f, 0.f, 0.f, 0.f};
            }
        }
#pragma unroll
        for (int J = K; J < NT; ++J) {
            const f4 xm = *(const f4*)(Ml + (J * (J + 1) / 2 + K) * 256);
#pragma unroll
            for (int t = 0; t < PT; ++t) acc[J][t] = mma_xty(acc[J][t], xm, y[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < PT; ++t) {
        float ss = 0.f;
#pragma unroll
        for (int J = 0; J < NT; ++J)
#pragma unroll
            for (int i = 0; i < 4; ++i) ss += acc[J][t][i] * acc[J][t][i];
        ss += __shfl_xor(ss, 16);
        ss += __shfl_xor(ss, 32);
        const int pix = pix0 + 16 * t + c;
        if (g == 0 && pix < p) out[lrow + pix] = sqrtf(ss);
    }
}

// ============================================================================
// Line normalisation (Sec. III-E, Eq. (24)): population mean and deviation of
// the p scores of each line in FP64, (delta - mean) / std, 0 when std is 0.
// ============================================================================
__global__ __launch_bounds__(256) void k_normalise(const Pass P)
{
    const int line = blockIdx.x;
    if (line >= P.nlines) return;
    const StreamDesc d = stream_of_line(P, line);
    const int p = d.p;
    __shared__ double red[256];
    const float* x = d.out + (size_t)(line - d.line0) * p;
    float* dn = d.outn + (size_t)(line - d.line0) * p;
    double s = 0.0;
    for (int i = threadIdx.x; i < p; i += 256) s += (double)x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double mean = red[0] / (double)p;
    __syncthreads();
    double v = 0.0;
    for (int i = threadIdx.x; i < p; i += 256) {
        const double q = (double)x[i] - mean;
        v += q * q;
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double sd = sqrt(red[0] / (double)p);
    for (int i = threadIdx.x; i < p; i += 256)
        dn[i] = (sd > 0.0) ? (float)(((double)x[i] - mean) / sd) : (sd == 0.0 ? 0.0f : (float)sd);
}

// ============================================================================
// Labels (Sec. III-E, Eq. (25)): y = [delta_N >= tau]; lines inside the
// warm-up buffer give 0.
// ============================================================================
__global__ __launch_bounds__(256) void k_labels(const float* __restrict__ dn, int n, int p, float tau,
                                                long long t0, int warmup, unsigned char* __restrict__ out)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)n * p) return;
    const long long line = t0 + i / p;
    out[i] = (line >= warmup && dn[i] >= tau) ? 1 : 0;
}

// ============================================================================
// host-side launchers
// ============================================================================
static int gram_macros(int NT)
{
    const int MT = (NT + 3) / 4;
    return MT * (MT + 1) / 2;
}

hipError_t launch_gram(int dtype, const Pass& P, int NT, double* stats, hipStream_t s)
{
    const int nm = gram_macros(NT);
    const long long E = stat_entries(NT);
    const long long nblk = (long long)((P.nlines + 7) / 8) * 8 * nm;
    dim3 grid((unsigned)nblk), block(256);
    switch (dtype) {
    case DT_F32: hipLaunchKernelGGL(k_gram<DT_F32>, grid, block, 0, s, P, NT, nm, stats, E); break;
    case DT_F16: hipLaunchKernelGGL(k_gram<DT_F16>, grid, block, 0, s, P, NT, nm, stats, E); break;
    default: hipLaunchKernelGGL(k_gram<DT_U16>, grid, block, 0, s, P, NT, nm, stats, E); break;
    }
    return hipGetLastError();
}

hipError_t launch_scan_local(const Pass& P, int NT, double* stats, hipStream_t s)
{
    const long long E = stat_entries(NT);
    dim3 g1((unsigned)((E + 255) / 256), (unsigned)P.nseg);
    hipLaunchKernelGGL(k_scan_local, g1, dim3(256), 0, s, P, stats, E);
    return hipGetLastError();
}

hipError_t launch_scan_carry(const Pass& P, int NT, const double* stats, double* carry, hipStream_t s)
{
    const long long E = stat_entries(NT);
    dim3 g2((unsigned)((E + 255) / 256), (unsigned)P.nstreams);
    hipLaunchKernelGGL(k_scan_carry, g2, dim3(256), 0, s, P, stats, carry, E);
    return hipGetLastError();
}

template <class T, int NT> constexpr int chol_waves()
{
    return NT <= 6 ? 4 : 8;
}

template <class T, int NT>
static void chol_one(const Pass& P, const double* stats, const double* carry, float* Mt, float* mu32,
                     int* flags, float* cond, double thr, int want, int force, unsigned long long* ctr,
                     hipStream_t s)
{
    constexpr int NW = chol_waves<T, NT>();
    const long long E = stat_entries(NT);
    hipLaunchKernelGGL((k_chol<T, NT, NW>), dim3(P.nlines), dim3(NW * 64), 0, s, P, stats, carry, E, Mt, mu32,
                       flags, cond, thr, want, force, ctr);
}

template <class T, int... NTs>
static void chol_dispatch(std::integer_sequence<int, NTs...>, int NT, const Pass& P, const double* stats,
                          const double* carry, float* Mt, float* mu32, int* flags, float* cond, double thr,
                          int want, int force, unsigned long long* ctr, hipStream_t s)
{
    ((NT == NTs + 1 ? chol_one<T, NTs + 1>(P, stats, carry, Mt, mu32, flags, cond, thr, want, force, ctr, s)
                    : void()),
     ...);
}

hipError_t launch_chol(int fp64, int force, const Pass& P, int NT, const double* stats, const double* carry,
                       float* Mt, float* mu32, int* flags, float* cond, double thr, int want_cond,
                       unsigned long long* ctr, hipStream_t s)
{
    if (NT < 1 || NT > MAX_NT) return hipErrorInvalidValue;
    auto seq = std::make_integer_sequence<int, MAX_NT>();
    if (fp64)
        chol_dispatch<double>(seq, NT, P, stats, carry, Mt, mu32, flags, cond, thr, want_cond, force, ctr, s);
    else
        chol_dispatch<float>(seq, NT, P, stats, carry, Mt, mu32, flags, cond, thr, want_cond, 0, ctr, s);
    return hipGetLastError();
}

template <int NT, int DT>
static void score_one(const Pass& P, const float* Mt, const float* mu32, hipStream_t s)
{
    const int per = 4 * SCORE_PT * 16;
    const int ngrp = (P.pmax + per - 1) / per;
    hipLaunchKernelGGL((k_score<NT, DT>), dim3((unsigned)((long long)P.nlines * ngrp)), dim3(256), 0, s, P, Mt,
                       mu32, ngrp);
}

template <int DT, int... NTs>
static void score_dispatch(std::integer_sequence<int, NTs...>, int NT, const Pass& P, const float* Mt,
                           const float* mu32, hipStream_t s)
{
    ((NT == NTs + 1 ? score_one<NTs + 1, DT>(P, Mt, mu32, s) : void()), ...);
}

hipError_t launch_score(int dtype, const Pass& P, int NT, const float* Mt, const float* mu32, hipStream_t s)
{
    if (NT < 1 || NT > MAX_NT) return hipErrorInvalidValue;
    auto seq = std::make_integer_sequence<int, MAX_NT>();
    switch (dtype) {
    case DT_F32: score_dispatch<DT_F32>(seq, NT, P, Mt, mu32, s); break;
    case DT_F16: score_dispatch<DT_F16>(seq, NT, P, Mt, mu32, s); break;
    default: score_dispatch<DT_U16>(seq, NT, P, Mt, mu32, s); break;
    }
    return hipGetLastError();
}

hipError_t launch_labels(const float* dn, int n, int p, float tau, long long t0, int warmup,
                         unsigned char* out, hipStream_t s)
{
    const long long N = (long long)n * p;
    hipLaunchKernelGGL(k_labels, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, dn, n, p, tau, t0,
                       warmup, out);
    return hipGetLastError();
}

hipError_t launch_normalise(const Pass& P, hipStream_t s)
{
    hipLaunchKernelGGL(k_normalise, dim3(P.nlines), dim3(256), 0, s, P);
    return hipGetLastError();
}

}  // namespace erx
