// Score on FP16 matrix cores with split operands (Sec. III-D, Eqs. (22)-(23)):
// delta = ||M (x - mu)|| with M = L^{-1}, the same product as k_score, in an
// arithmetic of FP32-class accuracy that runs on the 16-bit matrix cores.
//
// The M^T tiles of a line are scaled by one power of two sM so that max |M sM|
// lies in [2^13, 2^14) (the factorisation kernel leaves max |M| per line in
// Pass::mscale), and the residuals of each pixel by a power of two sR that
// puts the pixel's largest residual over its first 16 bands in [2^7, 2^8)
// (set at the first non-zero column); both are split into two FP16 halves,
// v s = h + l with h = fp16(v s) and l = fp16(v s - h), so h carries 11
// significant bits and l the next 11.  A tile product becomes
// M R = (Mh Rh + Mh Rl + Ml Rh) / (sM sR) up to the dropped Ml Rl term (below
// 2^-22 of the product): three 16x16x16 FP16 MFMAs with FP32 accumulation,
// whose products are exact in FP32, accumulated straight into the row's FP32
// accumulator.  Residuals far below the first column's lose only what lies
// below 2^-25 / sR, about 2^-33 of that column's largest residual.  A pixel
// with a later residual 2^15 / sR or larger (128 times its first column's
// largest; infinite inputs included) would overflow FP16: its line is flagged
// FLAG_SCORE32 and scored again by the FP32 kernel.  The score is
// sqrt(sum of squares) / (sM sR), exact powers of two again.
//
// Structure as in k_score: a workgroup of 4 waves scores 4 * PT tiles of 16
// pixels of one line; column K of M^T (tiles (J, K), J >= K) is staged once
// per workgroup in double-buffered LDS, already scaled and split, while the
// next column's loads are in flight.
#include "erx_device.h"

namespace erx {

typedef _Float16 hv4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ f4 mfma_h16(hv4 a, hv4 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}

// Power-of-two scale s with m s in [2^T, 2^(T+1)), and 1/s; s = 1 when m is 0,
// infinite or NaN.  Both are built from the exponent field, so they are exact.
template <int T> __device__ __forceinline__ void pow2_scale(float m, float& s, float& inv)
{
    int E = ((__float_as_int(m) >> 23) & 0xff) - 127;
    const bool ok = m > 0.f && E < 128;
    E = E < T - 126 ? T - 126 : E;
    E = E > T + 126 ? T + 126 : E;
    s = ok ? __int_as_float((127 + T - E) << 23) : 1.f;
    inv = ok ? __int_as_float((127 - T + E) << 23) : 1.f;
}

struct HL {
    hv4 hi, lo;
};

__device__ __forceinline__ HL split16(const f4 v, float s)
{
    f4 w;
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = v[q] * s;
    HL r;
    r.hi = __builtin_convertvector(w, hv4);
    const f4 back = __builtin_convertvector(r.hi, f4);
    f4 d;
#pragma unroll
    for (int q = 0; q < 4; ++q) d[q] = w[q] - back[q];
    r.lo = __builtin_convertvector(d, hv4);
    return r;
}

}  // namespace

// PT: 16-pixel tiles per wave (the tile shape the autotuner chooses: one tile keeps
// fewer accumulators per lane and more workgroups per line, two reuse each staged M tile
// for twice the pixels).  Waves per SIMD: as many as the registers allow without spills
// (one tile: 124 VGPRs at 14 band tiles; two: 184 at 13-14)
template <int NT, int DT, bool VEC, int PT>
__global__ __launch_bounds__(256, PT == 1 ? (NT <= 14 ? 4 : 3) : (NT <= 12 ? 3 : 2)) void k_score16(const Pass P,
                                                                                   const float* __restrict__ Mt,
                                                                    const float* __restrict__ mu32,
                                                                    int* __restrict__ flags, int ngrp)
{
    constexpr int NTL = NT * (NT + 1) / 2;
    constexpr int MR = (NT * 64 + 255) / 256;  // rounds of 256 threads to stage the longest column
    // all pixel groups of a line on one XCD (block ids are dealt to the 8 XCDs
    // round robin), so the line's M tiles are fetched into one L2
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int lx = j / ngrp, grp = j - lx * ngrp;
    const int line = lx * 8 + xcd;
    if (line >= P.nlines) return;  // uniform for the workgroup
    const StreamDesc d = stream_of_line(P, line);
    const int p = d.p, b = d.b;
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
    const int pix0 = (grp * 4 + w) * PT * 16;  // waves past the last pixel still stage tiles
    const void* X = advance<DT>(d.x, (size_t)(line - d.line0) * p * b);
    GLB float* out = glb(d.out + (size_t)(line - d.line0) * p);
    const float* mu = mu32 + (size_t)line * 16 * NT;
    const f4* Ml = (const f4*)(Mt + (size_t)line * NTL * 256);

    float sM, invM;
    pow2_scale<13>(glb(P.mscale)[line], sM, invM);
    __shared__ HL Ms[2][MR * 256];
    f4 st[MR];
    // column K has (NT - K) tiles of 64 quads: only the rounds of 256 quads that reach
    // into it run (the condition is uniform, and fixed for each K of the unrolled loop)
    auto gload = [&](int K) __attribute__((always_inline)) {
        const int n = (NT - K) * 64;
        const f4* src = Ml + (size_t)tile_lc(K, K, NT) * 64;
#pragma unroll
        for (int i = 0; i < MR; ++i)
            if (256 * i < n) st[i] = src[min(tid + 256 * i, n - 1)];
    };
    auto lstore = [&](int buf, int K) __attribute__((always_inline)) {
        const int n = (NT - K) * 64;
#pragma unroll
        for (int i = 0; i < MR; ++i)
            if (256 * i < n) Ms[buf][tid + 256 * i] = split16(st[i], sM);
    };
    f4 y[2][PT];
    auto yload = [&](int K, f4* yy) __attribute__((always_inline)) {
        const int band0 = 16 * K + 4 * g;
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            const int pix = pix0 + 16 * t + c;
            const bool okl = pix < p && band0 < b;
            yy[t] = ldq<DT, VEC>(X, okl ? (size_t)pix * b + band0 : 0, okl ? b - band0 : 0);
        }
    };
    f4 mv[2];
    auto mload = [&](int K, f4& m) __attribute__((always_inline)) { m = *(const GLB f4*)glb(mu + 16 * K + 4 * g); };

    f4 acc[NT][PT];
#pragma unroll
    for (int J = 0; J < NT; ++J)
#pragma unroll
        for (int t = 0; t < PT; ++t) acc[J][t] = f4{0.f, 0.f, 0.f, 0.f};

    // per-pixel residual scale (1 / scale), and whether it has been set
    float sR[PT], iR[PT];
    bool have[PT] = {};
    bool ovf = false;
    gload(0);
    yload(0, y[0]);
    mload(0, mv[0]);
    lstore(0, 0);
    __syncthreads();
#pragma unroll
    for (int K = 0; K < NT; ++K) {
        if (K + 1 < NT) {
            gload(K + 1);
            yload(K + 1, y[(K + 1) & 1]);
            mload(K + 1, mv[(K + 1) & 1]);
        }
        __builtin_amdgcn_sched_barrier(0);
        // residuals of this column's bands (missing pixels and bands are zero),
        // scaled per pixel and split
        const int band0 = 16 * K + 4 * g;
        const f4 m4 = mv[K & 1];
        HL rr[PT];
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            const bool okp = pix0 + 16 * t + c < p;
            f4 r;
#pragma unroll
            for (int q = 0; q < 4; ++q) r[q] = (okp && band0 + q < b) ? y[K & 1][t][q] - m4[q] : 0.f;
            float m = absmax4(r);  // the pixel's 16 bands sit in lanes c, c+16, c+32, c+48
            m = fmaxf(m, __shfl_xor(m, 16));
            m = fmaxf(m, __shfl_xor(m, 32));
            if (K == 0 || !have[t]) {  // per-lane selects, no branch
                float s2, i2;
                pow2_scale<7>(m, s2, i2);
                const bool set = K == 0 || m > 0.f;
                sR[t] = set ? s2 : sR[t];
                iR[t] = set ? i2 : iR[t];
                have[t] = have[t] || m > 0.f;
            }
            ovf = ovf || m * sR[t] >= 32768.f;
            rr[t] = split16(r, sR[t]);
        }
        const HL* Mc = Ms[K & 1];
        // the tile of row J+1 is read before the products of row J
        HL xm = Mc[lane];
#pragma unroll
        for (int J = K; J < NT; ++J) {
            HL xn;
            if (J + 1 < NT) xn = Mc[(J + 1 - K) * 64 + lane];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < PT; ++t) {
                acc[J][t] = mfma_h16(xm.hi, rr[t].hi, acc[J][t]);
                acc[J][t] = mfma_h16(xm.hi, rr[t].lo, acc[J][t]);
                acc[J][t] = mfma_h16(xm.lo, rr[t].hi, acc[J][t]);
            }
            __builtin_amdgcn_sched_barrier(0);
            xm = xn;
        }
        __builtin_amdgcn_sched_barrier(0);
        if (K + 1 < NT) lstore((K + 1) & 1, K + 1);
        __syncthreads();
    }
    if (__ballot(ovf) && tid % 64 == 0) atomicOr(flags + line, FLAG_SCORE32);
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
        if (g == 0 && pix < p) out[pix] = sqrtf(ss) * iR[t] * invM;
    }
}

template <int NT, int DT, int PT>
static void score16_pt(const Pass& P, const float* Mt, const float* mu32, int* flags, hipStream_t s)
{
    const int per = 4 * PT * 16;
    const int ngrp = (P.pmax + per - 1) / per;
    const dim3 grid((unsigned)((long long)(P.nlines + 7) / 8 * 8 * ngrp));
    if (P.vec4) hipLaunchKernelGGL((k_score16<NT, DT, true, PT>), grid, dim3(256), 0, s, P, Mt, mu32, flags, ngrp);
    else hipLaunchKernelGGL((k_score16<NT, DT, false, PT>), grid, dim3(256), 0, s, P, Mt, mu32, flags, ngrp);
}

template <int NT, int DT>
static void score16_one(const Pass& P, const float* Mt, const float* mu32, int* flags, hipStream_t s)
{
    // default: one tile per wave from 13 band tiles on, where two would spill registers
    if (P.spt == 1 || (P.spt == 0 && NT >= 13)) score16_pt<NT, DT, 1>(P, Mt, mu32, flags, s);
    else score16_pt<NT, DT, SCORE_PT>(P, Mt, mu32, flags, s);
}

template <int DT, int... NTs>
static void score16_dispatch(std::integer_sequence<int, NTs...>, int NT, const Pass& P, const float* Mt,
                             const float* mu32, int* flags, hipStream_t s)
{
    ((NT == NTs + 1 ? score16_one<NTs + 1, DT>(P, Mt, mu32, flags, s) : void()), ...);
}

hipError_t launch_score16(int dtype, const Pass& P, int NT, const float* Mt, const float* mu32, int* flags,
                          hipStream_t s)
{
    if (NT < 1 || NT > MAX_NT) return hipErrorInvalidValue;
    auto seq = std::make_integer_sequence<int, MAX_NT>();
    switch (dtype) {
    case DT_F32: score16_dispatch<DT_F32>(seq, NT, P, Mt, mu32, flags, s); break;
    case DT_F16: score16_dispatch<DT_F16>(seq, NT, P, Mt, mu32, flags, s); break;
    default: score16_dispatch<DT_U16>(seq, NT, P, Mt, mu32, flags, s); break;
    }
    return hipGetLastError();
}

}  // namespace erx
