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
#include "erx_device.h"

namespace erx {

typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

template <int PREC> struct LP;
template <> struct LP<ERX_GRAM_BF16> {
    typedef bf4 v4;
    typedef bf8 v8;
    static __device__ __forceinline__ f4 mma(v8 a, v8 b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct LP<ERX_GRAM_FP16> {
    typedef h4 v4;
    typedef h8 v8;
    static __device__ __forceinline__ f4 mma(v8 a, v8 b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// ============================================================================
// Gram: per line, mean and centred covariance (Sec. III-C, Eqs. (18)-(19)).
//
// A workgroup of 4 waves computes one 64x64 block ("macro tile", 4x4 tiles of
// 16 bands) of the upper triangle of the band x band Gram matrix of one line;
// wave w owns tile row 4*MI+w.  Pixels are the contraction index.  Grid:
// 8 * ceil(n/8) * nmacro workgroups; block ids are spread so that all macro
// tiles of one line run on the same XCD (consecutive block ids are dispatched
// round-robin over the 8 XCDs) and share its L2.
//
// Data are shifted by s = the FP32 mean of the first min(64, p) pixels of
// each band (the same value in every workgroup), and the exact identity
//     sum (x-mu)(x-mu)^T = sum (x-s)(x-s)^T - p (mu-s)(mu-s)^T
// turns the shifted sums into the centred covariance.
//
// Operand precision (PREC):
//   FP32         16x16x4 FP32 MFMA, FP32 partials over 64 pixels, FP64 sums.
//   BF16 / FP16  a stated change to the method's arithmetic: x - s is rounded
//                to 16 bits and multiplied on the 16x16x32 instructions with
//                FP32 accumulation over 256 pixels, FP64 sums.  The score
//                error grows from FP32 rounding to the 16-bit input rounding
//                (2^-9 relative for BF16, 2^-12 for FP16), amplified by the
//                conditioning of the covariance.  The band sums that give the
//                mean are taken from the FP32 values, so the mean keeps FP32
//                accuracy.  FP16 operands need |x - s| < 65504.
//
// Staging.  A chunk is 64 pixels.  Thread (bg, pq) = (tid % 16, tid / 16)
// loads pixels 4pq..4pq+3 of the bands 4bg..4bg+3 of each panel, so the 16
// consecutive lanes with equal pq read one contiguous 256-byte segment of a
// pixel row.  All loads are unconditional (addresses of missing pixels and
// bands are clamped into the line and their values zeroed afterwards): a load
// under a divergent branch makes the compiler wait for every load already in
// flight, which would serialise the one-chunk-ahead prefetch.  The thread
// holds a 4 x 4 block (pixels x bands); transposed in registers, each band
// row of 4 pixels is one 16-byte (FP32) or 8-byte (16-bit) LDS store.
//
// LDS holds band rows of 64 pixels.  FP32 rows are 16 quads of 4 pixels; the
// quad index is XOR-swizzled with sw(r) = (r mod 16) xor (r div 16), so that
// both the 16 lanes of a store (16 band groups) and the 16 lanes of an MFMA
// operand read (16 consecutive band rows) hit 16 different 16-byte bank
// groups.  16-bit rows are 8 octets of 8 pixels, swizzled with (r div 2) mod 8.
// A lane (g, c) of an operand reads consecutive pixels of band c; A and B use
// the same pixel order, so each step contracts over all of its pixels
// whatever order the instruction pairs them in.
//
// Band sums for the mean are FP32 per thread over 4 pixels per chunk, FP64
// across chunks and threads.
// ============================================================================
__device__ __forceinline__ int g4_sw(int r) { return (r & 15) ^ (r >> 4); }
__device__ __forceinline__ int g4_sw8(int r) { return (r >> 1) & 7; }

template <int PREC> struct G4;
template <> struct G4<ERX_GRAM_FP32> {
    static constexpr int WORDS = 64 * 64;  // 32-bit words per panel
    static constexpr int FLUSH = 64;       // pixels per FP32 partial
    static __device__ __forceinline__ void put(uint32_t* T, int r, int pq, const f4 v, float)
    {
        *(f4*)&T[r * 64 + 4 * (pq ^ g4_sw(r))] = v;
    }
    template <int NQ>
    static __device__ __forceinline__ void chunk(const uint32_t* Rt, const uint32_t* Cp, int w, int c, int g,
                                                 int kend, int qoff, f4* acc)
    {
        const int ra = 16 * w + c;
        // operands of 16 pixels (four per lane)
        auto rd = [&](int u, f4& av, f4 (&bv)[NQ]) __attribute__((always_inline)) {
            const int qd = (u >> 2) + g;
            av = *(const f4*)&Rt[ra * 64 + 4 * (qd ^ g4_sw(ra))];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int rb = 16 * (q + qoff) + c;
                bv[q] = *(const f4*)&Cp[rb * 64 + 4 * (qd ^ g4_sw(rb))];
            }
        };
        auto mul = [&](const f4& av, const f4 (&bv)[NQ]) __attribute__((always_inline)) {
#pragma unroll
            for (int st = 0; st < 4; ++st)
#pragma unroll
                for (int q = 0; q < NQ; ++q) acc[q] = mfma(av[st], bv[q][st], acc[q]);
        };
        if (kend == 64) {
            // full chunk: the reads of step k+1 are issued before the products of
            // step k (scheduling barriers keep the compiler from sinking them
            // back next to their use), so LDS latency overlaps the MFMAs
            f4 av[4], bv[4][NQ];
            rd(0, av[0], bv[0]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k < 3) rd(16 * (k + 1), av[k + 1], bv[k + 1]);
                __builtin_amdgcn_sched_barrier(0);
                mul(av[k], bv[k]);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            for (int u = 0; u < kend; u += 16) {
                f4 av, bv[NQ];
                rd(u, av, bv);
                mul(av, bv);
            }
        }
    }
    // Wave 3 of a full diagonal macro tile: tile (3, 3) into acc[0] and tile
    // (0, 3) into acc[1] (the panel is shared, so row tile 3 is also the column
    // operand of both)
    static __device__ __forceinline__ void chunk_pair(const uint32_t* Rt, int c, int g, int kend, f4* acc)
    {
        const int r3 = 48 + c, r0 = c;
        auto rd = [&](int u, f4& a3, f4& a0) __attribute__((always_inline)) {
            const int qd = (u >> 2) + g;
            a3 = *(const f4*)&Rt[r3 * 64 + 4 * (qd ^ g4_sw(r3))];
            a0 = *(const f4*)&Rt[r0 * 64 + 4 * (qd ^ g4_sw(r0))];
        };
        auto mul = [&](const f4& a3, const f4& a0) __attribute__((always_inline)) {
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                acc[0] = mfma(a3[st], a3[st], acc[0]);
                acc[1] = mfma(a0[st], a3[st], acc[1]);
            }
        };
        if (kend == 64) {
            f4 a3[4], a0[4];
            rd(0, a3[0], a0[0]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k < 3) rd(16 * (k + 1), a3[k + 1], a0[k + 1]);
                __builtin_amdgcn_sched_barrier(0);
                mul(a3[k], a0[k]);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
            for (int u = 0; u < kend; u += 16) {
                f4 a3, a0;
                rd(u, a3, a0);
                mul(a3, a0);
            }
        }
    }
};
template <int PREC> struct G4H {
    typedef typename LP<PREC>::v4 v4;
    typedef typename LP<PREC>::v8 v8;
    static constexpr int WORDS = 64 * 32;
    static constexpr int FLUSH = 256;
    static __device__ __forceinline__ void put(uint32_t* T, int r, int pq, const f4 v, float)
    {
        uint16_t* H = (uint16_t*)T;
        *(v4*)&H[r * 64 + 8 * ((pq >> 1) ^ g4_sw8(r)) + 4 * (pq & 1)] = __builtin_convertvector(v, v4);
    }
    template <int NQ>
    static __device__ __forceinline__ void chunk(const uint32_t* Rt, const uint32_t* Cp, int w, int c, int g,
                                                 int kend, int qoff, f4* acc)
    {
        const uint16_t* RH = (const uint16_t*)Rt;
        const uint16_t* CH = (const uint16_t*)Cp;
        const int ra = 16 * w + c;
        // operands of 32 pixels (eight per lane)
        auto rd = [&](int u, v8& av, v8 (&bv)[NQ]) __attribute__((always_inline)) {
            const int oc = (u >> 3) + g;
            av = *(const v8*)&RH[ra * 64 + 8 * (oc ^ g4_sw8(ra))];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int rb = 16 * (q + qoff) + c;
                bv[q] = *(const v8*)&CH[rb * 64 + 8 * (oc ^ g4_sw8(rb))];
            }
        };
        auto mul = [&](const v8& av, const v8 (&bv)[NQ]) __attribute__((always_inline)) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] = LP<PREC>::mma(av, bv[q], acc[q]);
        };
        if (kend == 64) {
            // both 32-pixel steps' reads first, so the second overlaps the
            // first step's products (as in the FP32 chunk)
            v8 av[2], bv[2][NQ];
            rd(0, av[0], bv[0]);
            rd(32, av[1], bv[1]);
            __builtin_amdgcn_sched_barrier(0);
            mul(av[0], bv[0]);
            mul(av[1], bv[1]);
        } else {
            for (int u = 0; u < kend; u += 32) {
                v8 av, bv[NQ];
                rd(u, av, bv);
                mul(av, bv);
            }
        }
    }
};
template <> struct G4<ERX_GRAM_BF16> : G4H<ERX_GRAM_BF16> {};
template <> struct G4<ERX_GRAM_FP16> : G4H<ERX_GRAM_FP16> {};

// Split FP16: x - s, scaled by the band's power of two c (|.| < 2^15), is held as
// two FP16 halves h = fp16(v c), l = fp16(v c - h) in two planes laid out as the
// 16-bit rows above; a 32-pixel step of a tile is h_a h_b + h_a l_b + l_a h_b on
// the 16x16x32 FP16 instruction (products exact in FP32, the dropped l_a l_b
// below 2^-22 of the product), FP32 partials over 64 pixels.
template <> struct G4<ERX_GRAM_SPLIT16> {
    static constexpr int WORDS = 64 * 64;  // hi plane, then lo plane
    static constexpr int LO = 64 * 64;     // offset of the lo plane in halves
    static constexpr int FLUSH = 64;
    static __device__ __forceinline__ void put(uint32_t* T, int r, int pq, const f4 v, float sc)
    {
        uint16_t* H = (uint16_t*)T;
        f4 w4;
#pragma unroll
        for (int q = 0; q < 4; ++q) w4[q] = v[q] * sc;
        const h4 hi = __builtin_convertvector(w4, h4);
        const f4 back = __builtin_convertvector(hi, f4);
        f4 d4;
#pragma unroll
        for (int q = 0; q < 4; ++q) d4[q] = w4[q] - back[q];
        const int off = r * 64 + 8 * ((pq >> 1) ^ g4_sw8(r)) + 4 * (pq & 1);
        *(h4*)&H[off] = hi;
        *(h4*)&H[LO + off] = __builtin_convertvector(d4, h4);
    }
    static __device__ __forceinline__ f4 mma(h8 a, h8 b, f4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
    template <int NQ>
    static __device__ __forceinline__ void chunk(const uint32_t* Rt, const uint32_t* Cp, int w, int c, int g,
                                                 int kend, int qoff, f4* acc)
    {
        const uint16_t* RH = (const uint16_t*)Rt;
        const uint16_t* CH = (const uint16_t*)Cp;
        const int ra = 16 * w + c;
        auto rd = [&](int u, h8& ah, h8& al, h8 (&bh)[NQ], h8 (&bl)[NQ]) __attribute__((always_inline)) {
            const int oc = (u >> 3) + g;
            const int oa = ra * 64 + 8 * (oc ^ g4_sw8(ra));
            ah = *(const h8*)&RH[oa];
            al = *(const h8*)&RH[LO + oa];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int rb = 16 * (q + qoff) + c;
                const int ob = rb * 64 + 8 * (oc ^ g4_sw8(rb));
                bh[q] = *(const h8*)&CH[ob];
                bl[q] = *(const h8*)&CH[LO + ob];
            }
        };
        auto mul = [&](const h8& ah, const h8& al, const h8 (&bh)[NQ], const h8 (&bl)[NQ]) __attribute__((always_inline)) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                acc[q] = mma(ah, bh[q], acc[q]);
                acc[q] = mma(ah, bl[q], acc[q]);
                acc[q] = mma(al, bh[q], acc[q]);
            }
        };
        // one 32-pixel step's operands at a time (both steps' hi and lo would take 80 registers)
        for (int u = 0; u < kend; u += 32) {
            h8 ah, al, bh[NQ], bl[NQ];
            rd(u, ah, al, bh, bl);
            mul(ah, al, bh, bl);
        }
    }
};

// The part of a macro tile's work that depends on whether it is diagonal (one
// panel, rows = columns) is compiled separately for both cases, so that no
// load sits under a branch.
template <int DT, int PREC, bool VEC, bool DG>
__device__ __forceinline__ void gram4_macro(const void* X, int p, int b, int NT, int MI, int MJ, int line,
                                            void* __restrict__ stats, int sf32, long long E, uint32_t* Rt,
                                            uint32_t* Ct, float* shift_s, double* red_s, double* bsum_s,
                                            float* scl_s, int* redo_s, int* redo_out)
{
    constexpr bool SPLIT = PREC == ERX_GRAM_SPLIT16;
    typedef G4<PREC> G;
    constexpr bool dg = DG;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63, g = lane >> 4, c = lane & 15;
    const int I = 4 * MI + w;
    const bool rowok = I < NT;
    const int rb0 = 64 * MI, cb0 = 64 * MJ;

    const int bg = tid & 15, pq = tid >> 4;
    // bands of this thread that exist (missing bands are zero in the products)
    const int rband = rb0 + 4 * bg, cband = cb0 + 4 * bg;
    bool rok[4], cok[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        rok[j] = rband + j < b;
        cok[j] = cband + j < b;
    }
    // two register sets of fetched chunks: chunk j is staged from set j & 1
    f4 pr2[2][4], pc2[2][4];
    f4(&pr)[4] = pr2[0];
    f4(&pc)[4] = pc2[0];
    // unconditional: past the last pixel the addresses are clamped into the
    // line and the values are masked by stage()
    auto fetch = [&](int k0, f4(&fr)[4], f4(&fc)[4]) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int px = k0 + 4 * pq + r;
            const bool okp = px < p;
            const size_t row = (size_t)(okp ? px : 0) * b;
            const bool okr = okp && rok[0], okc = okp && cok[0];
            fr[r] = ldq<DT, VEC>(X, okr ? row + rband : 0, okr ? b - rband : 0);
            if (!dg) fc[r] = ldq<DT, VEC>(X, okc ? row + cband : 0, okc ? b - cband : 0);
        }
    };
    fetch(0, pr2[0], pc2[0]);
    {
        // shift from the first chunk: per-thread sums of 4 pixels, then the 4
        // pixel quads of a wave (lanes bg + 16k), then the 4 waves via LDS
        const int nv0 = p - 4 * pq;
        float a[4], e[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] = e[j] = 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                a[j] += (r < nv0 && rok[j]) ? pr[r][j] : 0.f;
                if (!dg) e[j] += (r < nv0 && cok[j]) ? pc[r][j] : 0.f;
            }
            if (dg) e[j] = a[j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] += __shfl_xor(a[j], 16);
            a[j] += __shfl_xor(a[j], 32);
            e[j] += __shfl_xor(e[j], 16);
            e[j] += __shfl_xor(e[j], 32);
        }
        float* part = (float*)Rt;  // [4 waves][128 bands], before the first stage
        if (lane < 16)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                part[w * 128 + 4 * bg + j] = a[j];
                part[w * 128 + 64 + 4 * bg + j] = e[j];
            }
        __syncthreads();
        if (tid < 128) {
            const float inv0 = 1.0f / (float)(p < 64 ? p : 64);
            shift_s[tid] = ((part[tid] + part[128 + tid]) + (part[256 + tid] + part[384 + tid])) * inv0;
        }
        __syncthreads();
    }
    float shr[4], shc[4], sr[4], sc[4];
    double dsr[4], dsc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        shr[j] = shift_s[4 * bg + j];
        shc[j] = shift_s[64 + 4 * bg + j];
        sr[j] = sc[j] = 0.f;
        dsr[j] = dsc[j] = 0.0;
    }
    // split FP16: per-band scales from the largest |x - s| of the first chunk
    // (scl_s: 128 scales, then 128 inverses); a band that is constant over the
    // first chunk, or a later value beyond the scale's headroom, sends this macro
    // tile to the FP32 pass (redo)
    float cr_[4] = {1.f, 1.f, 1.f, 1.f}, cc_[4] = {1.f, 1.f, 1.f, 1.f};
    bool ovf = false;
    if constexpr (SPLIT) {
        const int nv0 = p - 4 * pq;
        float a[4], e[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] = e[j] = 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                a[j] = fmaxf(a[j], (r < nv0 && rok[j]) ? fabsf(pr[r][j] - shr[j]) : 0.f);
                if (!dg) e[j] = fmaxf(e[j], (r < nv0 && cok[j]) ? fabsf(pc[r][j] - shc[j]) : 0.f);
            }
            if (dg) e[j] = a[j];
            a[j] = fmaxf(a[j], __shfl_xor(a[j], 16));
            a[j] = fmaxf(a[j], __shfl_xor(a[j], 32));
            e[j] = fmaxf(e[j], __shfl_xor(e[j], 16));
            e[j] = fmaxf(e[j], __shfl_xor(e[j], 32));
        }
        float* part = (float*)Rt;  // [4 waves][128 bands], before the first stage
        if (lane < 16)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                part[w * 128 + 4 * bg + j] = a[j];
                part[w * 128 + 64 + 4 * bg + j] = e[j];
            }
        if (tid == 0) *redo_s = 0;
        __syncthreads();
        if (tid < 128) {
            const float m = fmaxf(fmaxf(part[tid], part[128 + tid]), fmaxf(part[256 + tid], part[384 + tid]));
            const int band = (tid < 64 ? rb0 : cb0) + (tid & 63);
            float cs, ci;
            split_scale(m, cs, ci);
            scl_s[tid] = cs;
            scl_s[128 + tid] = ci;
            if (band < b && !(m > 0.f)) *redo_s = 1;  // constant over the first chunk (or NaN)
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            cr_[j] = scl_s[4 * bg + j];
            cc_[j] = scl_s[64 + 4 * bg + j];
        }
    }
    auto stage = [&](int k0, int buf, const f4(&fr)[4], const f4(&fc)[4]) __attribute__((always_inline)) {
        uint32_t* Rb = Rt + buf * G::WORDS;
        uint32_t* Cb = Ct + buf * G::WORDS;
        const int nv = p - k0 - 4 * pq;  // valid pixels among this thread's four
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            f4 v;
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = (r < nv && rok[j]) ? fr[r][j] - shr[j] : 0.f;
            sr[j] += (v[0] + v[1]) + (v[2] + v[3]);
            if constexpr (SPLIT)
                ovf = ovf || absmax4(v) * cr_[j] >= 32768.f;
            G::put(Rb, 4 * bg + j, pq, v, cr_[j]);
            if (!dg) {
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = (r < nv && cok[j]) ? fc[r][j] - shc[j] : 0.f;
                sc[j] += (v[0] + v[1]) + (v[2] + v[3]);
                if constexpr (SPLIT)
                    ovf = ovf || absmax4(v) * cc_[j] >= 32768.f;
                G::put(Cb, 4 * bg + j, pq, v, cc_[j]);
            }
        }
    };

    // Column tiles of this wave: 4MJ + qoff + q for q < nq.  In a diagonal
    // macro tile wave w needs only the tiles on and right of the diagonal
    // (qoff = w): the tiles below it are neither computed nor stored.
    // In a full diagonal macro tile (FP32) tile (0, 3) moves from wave 0 to
    // wave 3, so that the waves carry 3, 3, 2 and 2 tiles instead of 4, 3, 2, 1.
    const int qoff = dg ? w : 0;
    const int ncol = (NT - 4 * MJ) < 4 ? (NT - 4 * MJ) : 4;
    const bool split = dg && PREC == ERX_GRAM_FP32 && ncol == 4;
    const bool pairw = split && w == 3;  // wave 3: tiles (3, 3) and (0, 3)
    const int nq = __builtin_amdgcn_readfirstlane(pairw ? 2 : (split && w == 0) ? 3
                                                                   : (ncol - qoff > 0 ? ncol - qoff : 1));
    int tbits = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) tbits |= (rowok && q < nq) ? (1 << q) : 0;
    tbits = __builtin_amdgcn_readfirstlane(tbits);

    double S[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) S[q][i] = 0.0;
    f4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};

    // Double-buffered LDS, two register sets: the products of chunk j read LDS
    // buffer j & 1 while chunk j+1 is staged (from register set (j+1) & 1)
    // into the other buffer and the loads of chunk j+3 are issued into the set
    // just staged, so a chunk's loads have two chunks of products to land; one
    // barrier per chunk.  Staging and fetching run unconditionally (past the
    // last pixel they stage zeros and load clamped addresses), so no load sits
    // under a branch.  The loop is unrolled by two so that the register sets
    // are named statically.
    auto step = [&](int k0, int it, f4(&sr_)[4], f4(&sc_)[4]) __attribute__((always_inline)) {
        const uint32_t* Rb = Rt + (it & 1) * G::WORDS;
        const uint32_t* Cb = dg ? Rb : (const uint32_t*)(Ct + (it & 1) * G::WORDS);
        if (rowok) {
            const int kend = (p - k0) < 64 ? (p - k0) : 64;
            bool paired = false;
            if constexpr (PREC == ERX_GRAM_FP32 && DG) {
                if (pairw) {
                    G::chunk_pair(Rb, c, g, kend, acc);
                    paired = true;
                }
            }
            if (!paired) {
                switch (nq) {
                case 1: G::template chunk<1>(Rb, Cb, w, c, g, kend, qoff, acc); break;
                case 2: G::template chunk<2>(Rb, Cb, w, c, g, kend, qoff, acc); break;
                case 3: G::template chunk<3>(Rb, Cb, w, c, g, kend, qoff, acc); break;
                default: G::template chunk<4>(Rb, Cb, w, c, g, kend, qoff, acc); break;
                }
            }
        }
        if (((k0 + 64) % G::FLUSH) == 0 || k0 + 64 >= p) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if constexpr (SPLIT) {
                    // undo the band scales of row 16w+4g+i and column 16(qoff+q)+c
                    const double icq = (double)scl_s[128 + 64 + 16 * ((qoff + q) & 3) + c];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        S[q][i] += (double)acc[q][i] * ((double)scl_s[128 + 16 * w + 4 * g + i] * icq);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) S[q][i] += (double)acc[q][i];
                }
                acc[q] = f4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {  // band sums of the chunks staged so far
                dsr[j] += (double)sr[j];
                dsc[j] += (double)sc[j];
                sr[j] = sc[j] = 0.f;
            }
        }
        stage(k0 + 64, (it + 1) & 1, sr_, sc_);  // chunk j+1 from its set ...
        fetch(k0 + 192, sr_, sc_);               // ... which then receives chunk j+3
        __syncthreads();
    };
    stage(0, 0, pr2[0], pc2[0]);
    fetch(64, pr2[1], pc2[1]);
    fetch(128, pr2[0], pc2[0]);
    __syncthreads();
    for (int k0 = 0, it = 0; k0 < p; k0 += 128, it += 2) {
        step(k0, it, pr2[1], pc2[1]);
        if (k0 + 64 >= p) break;
        step(k0 + 64, it + 1, pr2[0], pc2[0]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        dsr[j] += (double)sr[j];
        dsc[j] += (double)sc[j];
    }

    // band sums: the 4 pixel quads of a wave, then the 4 waves
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        dsr[j] += __shfl_xor(dsr[j], 16);
        dsr[j] += __shfl_xor(dsr[j], 32);
        dsc[j] += __shfl_xor(dsc[j], 16);
        dsc[j] += __shfl_xor(dsc[j], 32);
    }
    if (lane < 16)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            red_s[w * 128 + 4 * bg + j] = dsr[j];
            red_s[w * 128 + 64 + 4 * bg + j] = dsc[j];
        }
    __syncthreads();
    if (tid < 128) {
        const int t = (dg && tid >= 64) ? tid - 64 : tid;
        bsum_s[tid] = (red_s[t] + red_s[128 + t]) + (red_s[256 + t] + red_s[384 + t]);
    }
    __syncthreads();
    if constexpr (SPLIT) {
        if (ovf) *redo_s = 1;  // benign race: every writer stores 1
        __syncthreads();
        if (tid == 0) *redo_out = *redo_s;
        if (*redo_s) return;  // uniform: the FP32 pass writes this macro tile
    }
    if (!rowok) return;

    const double inv_p = 1.0 / (double)p, inv_p1 = 1.0 / (double)(p - 1);
    double* ls = (double*)stats + (size_t)line * E;
    float* ls32 = (float*)stats + (size_t)line * E;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (!(tbits & (1 << q))) continue;
        const int rt = (pairw && q == 1) ? 0 : w;  // row and column tile within the macro tile
        const int ct = pairw ? 3 : qoff + q;
        const double scol = bsum_s[64 + 16 * ct + c];
        double o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double srho = bsum_s[16 * rt + 4 * g + i];
            o[i] = (S[q][i] - srho * scol * inv_p) * inv_p1;
        }
        const long long off = tile_u(4 * MI + rt, 4 * MJ + ct, NT) * 256 + lane * 4;
        if (sf32) {
            *(float4*)(ls32 + off) = float4{(float)o[0], (float)o[1], (float)o[2], (float)o[3]};
        } else {
            *(double2*)(ls + off) = double2{o[0], o[1]};
            *(double2*)(ls + off + 2) = double2{o[2], o[3]};
        }
    }
    if (dg && g == 0) {
        const long long ntU = (long long)NT * (NT + 1) / 2;
        const int band = 16 * I + c;
        const double m = (band < b) ? (double)shift_s[16 * w + c] + bsum_s[16 * w + c] * inv_p : 0.0;
        if (sf32) ls32[ntU * 256 + band] = (float)m;
        else ls[ntU * 256 + band] = m;
    }
}


template <int DT, int PREC, bool VEC>
__global__ __launch_bounds__(256) void k_gram4(const Pass P, int NT, int nmacro, void* __restrict__ stats,
                                               long long E, const int* __restrict__ only)
{
    typedef G4<PREC> G;
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
    // the FP32 pass after a split-FP16 one recomputes only the macro tiles that one flagged
    if (only && !glb(only)[(size_t)line * nmacro + (kk - ll * nmacro)]) return;
    __shared__ __attribute__((aligned(16))) uint32_t Rt[2 * G::WORDS];  // two chunk buffers per panel
    __shared__ __attribute__((aligned(16))) uint32_t Ct[2 * G::WORDS];
    __shared__ float shift_s[128];
    __shared__ double red_s[4 * 128];
    __shared__ double bsum_s[128];
    __shared__ float scl_s[PREC == ERX_GRAM_SPLIT16 ? 256 : 1];
    __shared__ int redo_s;
    int* redo_out = P.gredo ? P.gredo + (size_t)line * nmacro + (kk - ll * nmacro) : nullptr;
    if (MI == MJ)
        gram4_macro<DT, PREC, VEC, true>(X, p, b, NT, MI, MJ, line, stats, P.sf32, E, Rt, Ct, shift_s, red_s,
                                         bsum_s, scl_s, &redo_s, redo_out);
    else
        gram4_macro<DT, PREC, VEC, false>(X, p, b, NT, MI, MJ, line, stats, P.sf32, E, Rt, Ct, shift_s, red_s,
                                          bsum_s, scl_s, &redo_s, redo_out);
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
template <class TS>
__global__ __launch_bounds__(256) void k_scan_local(const Pass P, TS* __restrict__ stats, long long E)
{
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= E) return;
    const int gsg = blockIdx.y;  // pass segment
    const StreamDesc d = stream_of_seg(P, gsg);
    const int l0 = (gsg - d.seg0) * P.seg;  // stream-local first line
    const int l1 = (l0 + P.seg) < d.n ? (l0 + P.seg) : d.n;
    const long long t0 = d.t0;
    TS* ptr = stats + (size_t)d.line0 * E + e;
    double acc = 0.0;  // the recurrence runs in FP64 whatever the storage type
    int l = l0;
    for (; l + 8 <= l1; l += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (double)ptr[(size_t)(l + q) * E];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double a = avg_weight(d, t0 + l + q);
            acc = (1.0 - a) * acc + a * v[q];
            v[q] = acc;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) ptr[(size_t)(l + q) * E] = (TS)v[q];
    }
    for (; l < l1; ++l) {
        const double a = avg_weight(d, t0 + l);
        acc = (1.0 - a) * acc + a * (double)ptr[(size_t)l * E];
        ptr[(size_t)l * E] = (TS)acc;
    }
}

// IMC (equally weighted background): the statistics of line j become its second
// moments about the stream's reference mean c, X_j = ((p-1)/p) K_hat_j +
// (mu_hat_j - c)(mu_hat_j - c)^T = (1/p) sum over its pixels of (x-c)(x-c)^T, so that
// their running mean over lines is (1/N) sum over all pooled pixels.  c is the
// first line's mean, stored after the state when the stream starts.  The mean
// entries are left as they are (their running mean is the pooled mean).
__global__ __launch_bounds__(256) void k_imc_moments(const Pass P, double* __restrict__ stats, long long E, int NT)
{
    const int line = blockIdx.y;
    const StreamDesc d = stream_of_line(P, line);
    const long long ntU = (long long)NT * (NT + 1) / 2;
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    const double* mu0 = stats + (size_t)d.line0 * E + ntU * 256;  // the pass's first line of the stream
    const bool fresh = d.t0 == 0;
    double* state = (double*)d.state;
    const double* c = fresh ? mu0 : state + E;
    double* ls = stats + (size_t)line * E;
    if (fresh && line == d.line0 && e < 16 * NT) state[E + e] = mu0[e];
    if (e >= ntU * 256) return;
    int u = (int)(e >> 8), I = 0;
    while (u >= NT - I) {
        u -= NT - I;
        ++I;
    }
    const int J = I + u, pos = (int)(e & 255), q = pos >> 2;
    const int r = 16 * I + 4 * (q >> 4) + (pos & 3), cc = 16 * J + (q & 15);
    const double* mh = ls + ntU * 256;
    const double pf = (double)(d.p - 1) / (double)d.p;
    ls[e] = (r < d.b && cc < d.b) ? pf * ls[e] + (mh[r] - c[r]) * (mh[cc] - c[cc]) : 0.0;
}

__device__ __forceinline__ double seg_decay(const StreamDesc& d, long long t0, int l0, int l1)
{
    double P = 1.0;
    for (int l = l0; l < l1; ++l) P *= 1.0 - avg_weight(d, t0 + l);
    return P;
}

template <class TS>
__global__ __launch_bounds__(256) void k_scan_carry(const Pass P, const TS* __restrict__ stats,
                                                    TS* __restrict__ carry, long long E)
{
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= E) return;
    const StreamDesc d = P.sd ? load_desc(P.sd + blockIdx.y) : P.one;
    GLB TS* state = glb((TS*)d.state);
    double cv = (double)state[e];
    const int nseg = (d.n + P.seg - 1) / P.seg;
    // decay over a whole segment that does not hold the stream's first line
    // (the same product as seg_decay); other segments take seg_decay
    const double full = seg_decay(d, 1, 0, P.seg);  // used for EMA streams only
    // the segment end values are read eight at a time ahead of the serial chain
    constexpr int U = 8;
    for (int g0 = 0; g0 < nseg; g0 += U) {
        double ev[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int gs = g0 + u < nseg ? g0 + u : nseg - 1;
            const int l1 = (gs * P.seg + P.seg) < d.n ? (gs * P.seg + P.seg) : d.n;
            ev[u] = (double)stats[(size_t)(d.line0 + l1 - 1) * E + e];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int gs = g0 + u;
            if (gs < nseg) {
                carry[(size_t)(d.seg0 + gs) * E + e] = (TS)cv;
                const int l0 = gs * P.seg;
                const int l1 = (l0 + P.seg) < d.n ? (l0 + P.seg) : d.n;
                const bool whole = l1 - l0 == P.seg && d.t0 + l0 > 0 && d.bg == BG_EMA;
                cv = (whole ? full : seg_decay(d, d.t0, l0, l1)) * cv + ev[u];
            }
        }
    }
    state[e] = (TS)cv;
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
template <int NT> struct CholLds {
    float part[NT * (NT + 1) / 2 * 32];  // per-tile partial sums (norms, mat-vecs)
    float vec[4][16 * NT];                // x, y, z, scratch vectors
    float red[64];
};

template <class T, int NT, int NW>
__global__ __launch_bounds__(NW * 64) void k_chol(const Pass P, const void* __restrict__ stats,
                                                  const void* __restrict__ carry, long long E,
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
    const double eps = sdl.eps;
    const long long t0 = sdl.t0;
    // the FP64 instantiation factors every line (force) or the lines the FP32 pass flagged
    if (FB && !force && !(flags[line] & FLAG_NEED_FP64)) return;  // uniform for the workgroup

    __shared__ __attribute__((aligned(32))) T diag_s[16 * 17];
    __shared__ __attribute__((aligned(32))) T xt_s[16 * 17];
    __shared__ __attribute__((aligned(32))) T panel_s[NT * 256];
    __shared__ __attribute__((aligned(32))) T mrow_s[NT * 256];
    __shared__ __attribute__((aligned(16))) CholLds<NT> aux;
    __shared__ int fail_s;
    __shared__ unsigned mmax_s;

    const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63,
              g = lane >> 4, c = lane & 15;
    const int lloc = line - sdl.line0;  // stream-local line index
    const int gseg = sdl.seg0 + lloc / seg, l0 = (lloc / seg) * seg;
    double D = 1.0;
    for (int l = l0; l <= lloc; ++l) D *= 1.0 - avg_weight(sdl, t0 + l);
    if (tid == 0) {
        fail_s = 0;
        mmax_s = 0u;
    }

    // ---- load A_IJ^T = (K_loc + D carry)_{JI} (+ eps on the diagonal)
    V A[SLOTS];
    int tI[SLOTS], tJ[SLOTS];
    // IMC: the averaged statistics are second moments about the reference mean c
    // (kept after the stream's state); the sample covariance of the N = t p pooled
    // pixels is N / (N - 1) (C - (mu - c)(mu - c)^T)
    const bool imc = sdl.bg == BG_IMC;
    const double* cref = (const double*)sdl.state + E;  // IMC passes store FP64
    const double nfac = imc ? (double)((t0 + lloc + 1) * sdl.p) / (double)((t0 + lloc + 1) * sdl.p - 1) : 1.0;
    // the same loads for FP64 and FP32 storage (st, cr: this line's statistics and
    // its segment's carry); the sums are formed in FP64 either way
    auto load = [&](const auto* __restrict__ st, const auto* __restrict__ cr) __attribute__((always_inline)) {
        auto mean_at = [&](int q) __attribute__((always_inline)) {
            return (double)st[(long long)NTL * 256 + q] + D * (double)cr[(long long)NTL * 256 + q];
        };
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
                    double v = (double)st[o] + D * (double)cr[o];
                    const int rb = 16 * J + row, cb = 16 * I + c;
                    if (imc && rb < b && cb < b)
                        v = nfac * (v - (mean_at(rb) - glb(cref)[rb]) * (mean_at(cb) - glb(cref)[cb]));
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
            for (int q = tid; q < BP; q += NW * 64) {
                const double v = mean_at(q);
                mu32[(size_t)line * BP + q] = (q < b) ? (float)v : 0.0f;
            }
        }
    };
    if (P.sf32) load((const float*)stats + (size_t)line * E, (const float*)carry + (size_t)gseg * E);
    else load((const double*)stats + (size_t)line * E, (const double*)carry + (size_t)gseg * E);

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
        float mloc = 0.f;  // max |M| of this thread's entries (NaN entries are skipped by fmaxf)
#pragma unroll
        for (int j = 0; j < SLOTS; ++j) {
            if (tI[j] < 0) continue;
            const int s = tile_lc(tI[j], tJ[j], NT);  // column-major, as the score kernel reads them
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int off = 64 * (c >> 2) + 4 * rowof<T>(g, i) + (c & 3);
                const float v = (float)A[j][i];
                dstl[(size_t)s * 256 + off] = nanout ? __builtin_nanf("") : v;
                mloc = fmaxf(mloc, fabsf(v));
            }
        }
        // max |M| of the line for the split-FP16 score (wave, then workgroup)
        if (P.mscale) {  // uniform
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) mloc = fmaxf(mloc, __shfl_xor(mloc, o));
            if (lane == 0) atomicMax(&mmax_s, __float_as_uint(mloc));
            __syncthreads();
            if (tid == 0) glb(P.mscale)[line] = __uint_as_float(mmax_s);
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
            // force on the FP32 instantiation: no FP64 pass follows, so a failed pivot is final
            if (fail && force) {
                f |= FLAG_NOTPD;
                atomicAdd(&counters[1], 1ull);
            }
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
// tiles are held in operand form and R_K is four consecutive bands of one
// pixel per lane, which is exactly the accumulator-layout operand of X^T Y.
//
// A workgroup of 4 waves scores 4 * PT tiles of 16 pixels of one line.  The
// M^T tiles are stored column by column (all tiles (J, K), J >= K, of column
// K contiguous); the workgroup stages column K in LDS (double-buffered, the
// next column's global loads in flight during the products of this one), so
// each tile is read from L2 once per workgroup rather than once per wave.  The
// pixel data of the next column is prefetched into registers the same way.
// ============================================================================
template <int NT, int DT, bool VEC>
// three workgroups per CU (three waves per SIMD) up to 14 tiles: at 14 a few
// registers spill and the extra wave still wins (1.92 -> 1.86 ms at 224 bands);
// above 14 tiles the spills grow, so two
__global__ __launch_bounds__(256, NT <= 14 ? 3 : 2) void k_score(const Pass P, const float* __restrict__ Mt,
                                               const float* __restrict__ mu32, const int* __restrict__ only,
                                               int ngrp)
{
    constexpr int NTL = NT * (NT + 1) / 2;
    constexpr int PT = SCORE_PT;
    constexpr int MR = (NT * 64 + 255) / 256;  // float4 per thread to stage the longest column
    // Workgroups are dispatched to the 8 XCDs round robin (bid mod 8), each with
    // its own L2: all pixel groups of a line go to one XCD, one after another in
    // its dispatch order, so the line's M tiles are fetched into one L2 once.
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int lx = j / ngrp, grp = j - lx * ngrp;
    const int line = lx * 8 + xcd;
    if (line >= P.nlines) return;  // uniform for the workgroup
    // the re-scoring pass of lines the split-FP16 kernel could not represent
    if (only && !(glb(only)[line] & FLAG_SCORE32)) return;
    const StreamDesc d = stream_of_line(P, line);
    const int p = d.p, b = d.b;
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
    // waves past the last pixel still stage tiles and meet the barriers
    const int pix0 = (grp * 4 + w) * PT * 16;
    const void* X = advance<DT>(d.x, (size_t)(line - d.line0) * p * b);
    GLB float* out = glb(d.out + (size_t)(line - d.line0) * p);
    const float* mu = mu32 + (size_t)line * 16 * NT;
    const f4* Ml = (const f4*)(Mt + (size_t)line * NTL * 256);

    // staging buffers padded to whole rounds of 256 threads, so that the
    // stores need no condition (a conditional store, or a select on a load
    // address, becomes a branch with a wait for every load in flight)
    __shared__ f4 Ms[2][MR * 256];
    f4 st[MR];
    auto gload = [&](int K) __attribute__((always_inline)) {
        const int n = (NT - K) * 64;
        const f4* src = Ml + (size_t)tile_lc(K, K, NT) * 64;
#pragma unroll
        for (int i = 0; i < MR; ++i) st[i] = src[min(tid + 256 * i, n - 1)];
    };
    auto lstore = [&](int K, int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < MR; ++i) Ms[buf][tid + 256 * i] = st[i];
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

    f4 acc[NT][PT];
#pragma unroll
    for (int J = 0; J < NT; ++J)
#pragma unroll
        for (int t = 0; t < PT; ++t) acc[J][t] = f4{0.f, 0.f, 0.f, 0.f};

    // mu of a column's bands, loaded with the column's pixels (a load consumed
    // right away would make the wait cover every prefetch in flight)
    f4 mv[2];
    auto mload = [&](int K, f4& m) __attribute__((always_inline)) { m = *(const GLB f4*)glb(mu + 16 * K + 4 * g); };
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
        // keep the next column's loads here, ahead of this column's products
        // (left to itself the compiler sinks them next to their use)
        __builtin_amdgcn_sched_barrier(0);
        // residual of this column's bands: missing pixels and bands are zero
        // (padded bands also have mu 0)
        const int band0 = 16 * K + 4 * g;
        const f4 m4 = mv[K & 1];
        f4 r[PT];
#pragma unroll
        for (int t = 0; t < PT; ++t) {
            const bool okp = pix0 + 16 * t + c < p;
#pragma unroll
            for (int q = 0; q < 4; ++q) r[t][q] = (okp && band0 + q < b) ? y[K & 1][t][q] - m4[q] : 0.f;
        }
        const f4* Mc = Ms[K & 1];
        // the tile of row J+1 is read before the products of row J
        f4 xm = Mc[lane];
#pragma unroll
        for (int J = K; J < NT; ++J) {
            f4 xn;
            if (J + 1 < NT) xn = Mc[(J + 1 - K) * 64 + lane];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < PT; ++t) acc[J][t] = mma_xty(acc[J][t], xm, r[t]);
            __builtin_amdgcn_sched_barrier(0);
            xm = xn;
        }
        __builtin_amdgcn_sched_barrier(0);
        if (K + 1 < NT) lstore(K + 1, (K + 1) & 1);
        __syncthreads();
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
        if (g == 0 && pix < p) out[pix] = sqrtf(ss);
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
    const GLB float* x = glb(d.out + (size_t)(line - d.line0) * p);
    GLB float* dn = glb(d.outn + (size_t)(line - d.line0) * p);
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

template <int PREC, bool VEC>
static void launch_gram4(int dtype, dim3 grid, dim3 block, hipStream_t s, const Pass& P, int NT, int nm,
                         void* stats, long long E, const int* only)
{
    switch (dtype) {
    case DT_F32: hipLaunchKernelGGL((k_gram4<DT_F32, PREC, VEC>), grid, block, 0, s, P, NT, nm, stats, E, only); break;
    case DT_F16: hipLaunchKernelGGL((k_gram4<DT_F16, PREC, VEC>), grid, block, 0, s, P, NT, nm, stats, E, only); break;
    default: hipLaunchKernelGGL((k_gram4<DT_U16, PREC, VEC>), grid, block, 0, s, P, NT, nm, stats, E, only); break;
    }
}

template <int PREC>
static void launch_gram4(int dtype, dim3 grid, dim3 block, hipStream_t s, const Pass& P, int NT, int nm,
                         void* stats, long long E, const int* only = nullptr)
{
    if (P.vec4) launch_gram4<PREC, true>(dtype, grid, block, s, P, NT, nm, stats, E, only);
    else launch_gram4<PREC, false>(dtype, grid, block, s, P, NT, nm, stats, E, only);
}

hipError_t launch_gram(int dtype, int prec, const Pass& P, int NT, void* stats, hipStream_t s)
{
    const int nm = gram_macros(NT);
    const long long E = stat_entries(NT);
    const long long nblk = (long long)((P.nlines + 7) / 8) * 8 * nm;
    dim3 grid((unsigned)nblk), block(256);
    if (prec == ERX_GRAM_BF16) launch_gram4<ERX_GRAM_BF16>(dtype, grid, block, s, P, NT, nm, stats, E);
    else if (prec == ERX_GRAM_FP16) launch_gram4<ERX_GRAM_FP16>(dtype, grid, block, s, P, NT, nm, stats, E);
    else if (prec == ERX_GRAM_SPLIT16 && P.gredo) {
        // split FP16, then FP32 for the macro tiles it flagged (the others return at once)
        if (P.gmacro == 128 || (P.gmacro == 0 && NT >= 5)) launch_gram8(dtype, P, NT, nm, stats, E, s);
        else launch_gram4<ERX_GRAM_SPLIT16>(dtype, grid, block, s, P, NT, nm, stats, E);
        launch_gram4<ERX_GRAM_FP32>(dtype, grid, block, s, P, NT, nm, stats, E, P.gredo);
    } else launch_gram4<ERX_GRAM_FP32>(dtype, grid, block, s, P, NT, nm, stats, E);
    return hipGetLastError();
}

hipError_t launch_scan_local(const Pass& P, int NT, void* stats, hipStream_t s)
{
    const long long E = stat_entries(NT);
    dim3 g1((unsigned)((E + 255) / 256), (unsigned)P.nseg);
    if (P.sf32) hipLaunchKernelGGL(k_scan_local<float>, g1, dim3(256), 0, s, P, (float*)stats, E);
    else hipLaunchKernelGGL(k_scan_local<double>, g1, dim3(256), 0, s, P, (double*)stats, E);
    return hipGetLastError();
}

hipError_t launch_imc_moments(const Pass& P, int NT, double* stats, hipStream_t s)
{
    if (P.sf32) return hipErrorInvalidValue;
    const long long E = stat_entries(NT);
    dim3 g((unsigned)(((long long)NT * (NT + 1) / 2 * 256 + 255) / 256), (unsigned)P.nlines);
    hipLaunchKernelGGL(k_imc_moments, g, dim3(256), 0, s, P, stats, E, NT);
    return hipGetLastError();
}

hipError_t launch_scan_carry(const Pass& P, int NT, const void* stats, void* carry, hipStream_t s)
{
    const long long E = stat_entries(NT);
    dim3 g2((unsigned)((E + 255) / 256), (unsigned)P.nstreams);
    if (P.sf32)
        hipLaunchKernelGGL(k_scan_carry<float>, g2, dim3(256), 0, s, P, (const float*)stats, (float*)carry, E);
    else
        hipLaunchKernelGGL(k_scan_carry<double>, g2, dim3(256), 0, s, P, (const double*)stats, (double*)carry, E);
    return hipGetLastError();
}

template <class T, int NT> constexpr int chol_waves()
{
    return NT <= 6 ? 4 : (NT <= 10 ? 8 : 16);
}

template <class T, int NT>
static void chol_one(const Pass& P, const void* stats, const void* carry, float* Mt, float* mu32,
                     int* flags, float* cond, double thr, int want, int force, unsigned long long* ctr,
                     hipStream_t s)
{
    constexpr int NW = chol_waves<T, NT>();
    const long long E = stat_entries(NT);
    hipLaunchKernelGGL((k_chol<T, NT, NW>), dim3(P.nlines), dim3(NW * 64), 0, s, P, stats, carry, E, Mt, mu32,
                       flags, cond, thr, want, force, ctr);
}

template <class T, int... NTs>
static void chol_dispatch(std::integer_sequence<int, NTs...>, int NT, const Pass& P, const void* stats,
                          const void* carry, float* Mt, float* mu32, int* flags, float* cond, double thr,
                          int want, int force, unsigned long long* ctr, hipStream_t s)
{
    ((NT == NTs + 1 ? chol_one<T, NTs + 1>(P, stats, carry, Mt, mu32, flags, cond, thr, want, force, ctr, s)
                    : void()),
     ...);
}

hipError_t launch_chol(int fp64, int force, const Pass& P, int NT, const void* stats, const void* carry,
                       float* Mt, float* mu32, int* flags, float* cond, double thr, int want_cond,
                       unsigned long long* ctr, hipStream_t s)
{
    if (NT < 1 || NT > MAX_NT) return hipErrorInvalidValue;
    auto seq = std::make_integer_sequence<int, MAX_NT>();
    if (fp64)
        chol_dispatch<double>(seq, NT, P, stats, carry, Mt, mu32, flags, cond, thr, want_cond, force, ctr, s);
    else
        chol_dispatch<float>(seq, NT, P, stats, carry, Mt, mu32, flags, cond, thr, want_cond, force, ctr, s);
    return hipGetLastError();
}

template <int NT, int DT>
static void score_one(const Pass& P, const float* Mt, const float* mu32, const int* only, hipStream_t s)
{
    const int per = 4 * SCORE_PT * 16;
    const int ngrp = (P.pmax + per - 1) / per;
    const dim3 grid((unsigned)((long long)(P.nlines + 7) / 8 * 8 * ngrp));
    if (P.vec4) hipLaunchKernelGGL((k_score<NT, DT, true>), grid, dim3(256), 0, s, P, Mt, mu32, only, ngrp);
    else hipLaunchKernelGGL((k_score<NT, DT, false>), grid, dim3(256), 0, s, P, Mt, mu32, only, ngrp);
}

template <int DT, int... NTs>
static void score_dispatch(std::integer_sequence<int, NTs...>, int NT, const Pass& P, const float* Mt,
                           const float* mu32, const int* only, hipStream_t s)
{
    ((NT == NTs + 1 ? score_one<NTs + 1, DT>(P, Mt, mu32, only, s) : void()), ...);
}

hipError_t launch_score(int dtype, const Pass& P, int NT, const float* Mt, const float* mu32, hipStream_t s,
                        const int* only)
{
    if (NT < 1 || NT > MAX_NT) return hipErrorInvalidValue;
    auto seq = std::make_integer_sequence<int, MAX_NT>();
    switch (dtype) {
    case DT_F32: score_dispatch<DT_F32>(seq, NT, P, Mt, mu32, only, s); break;
    case DT_F16: score_dispatch<DT_F16>(seq, NT, P, Mt, mu32, only, s); break;
    default: score_dispatch<DT_U16>(seq, NT, P, Mt, mu32, only, s); break;
    }
    return hipGetLastError();
}

// ============================================================================
// Exact statistics of one-tile FP32 streams (b <= 16) for the pass pipeline:
// per line the mean and centred covariance (Eqs. (18)-(19)) with FP64
// differences and FP64 MFMA products, written in the layout of k_gram4.  One
// workgroup per line; each wave takes tiles w, w+4, ... with its own shift
// (the first pixel of its first tile) and the wave sums are combined exactly.
// Used for the projected stream of the learned surrogate, whose covariance can
// be far less well conditioned than the data's.
// ============================================================================
__global__ __launch_bounds__(256) void k_gram1x(const Pass P, double* __restrict__ stats, long long E)
{
    const int line = blockIdx.x;
    if (line >= P.nlines) return;  // uniform for the workgroup
    const StreamDesc d = stream_of_line(P, line);
    const int p = d.p, b = d.b;
    const float* X = (const float*)d.x + (size_t)(line - d.line0) * p * b;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
    __shared__ double red_s[4][256 + 16];
    __shared__ double wsh_s[4][16];
    __shared__ int wn_s[4];
    const int ntile = (p + 15) >> 4;
    const int ntw = ntile > w ? (ntile - w + 3) >> 2 : 0;
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    double bsd = 0.0, sh = 0.0;
    for (int tt = w; tt < ntile; tt += 4) {
        float xf[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int px = 16 * tt + 4 * g + i;
            const bool ok = px < p && c < b;
            const float v = glb(X)[ok ? (size_t)px * b + c : 0];
            xf[i] = ok ? v : 0.f;
        }
        if (tt == w) sh = (double)__shfl(xf[0], c);
        d4 xv;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int px = 16 * tt + 4 * g + i;
            xv[i] = (px < p && c < b) ? (double)xf[i] - sh : 0.0;
        }
        bsd += (xv[0] + xv[1]) + (xv[2] + xv[3]);
        acc = mma_xty(acc, xv, xv);
    }
    bsd += __shfl_xor(bsd, 16);
    bsd += __shfl_xor(bsd, 32);
#pragma unroll
    for (int i = 0; i < 4; ++i) red_s[w][(4 * i + g) * 16 + c] = acc[i];  // FP64 layout: row 4i+g
    if (g == 0) {
        red_s[w][256 + c] = bsd;
        wsh_s[w][c] = ntw ? sh : 0.0;
    }
    if (lane == 0) wn_s[w] = ntw ? 16 * ntw - (((ntile - 1 - w) & 3) == 0 ? 16 * ntile - p : 0) : 0;
    __syncthreads();
    if (w != 0) return;
    const double inv_p = 1.0 / (double)p, inv_p1 = 1.0 / (double)(p - 1);
    double mw_c[4], m_c = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int nw = wn_s[v];
        mw_c[v] = nw ? wsh_s[v][c] + red_s[v][256 + c] / nw : 0.0;
        m_c += nw * mw_c[v];
    }
    m_c *= inv_p;
    double* ls = stats + (size_t)line * E;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = 4 * g + i;
        double cs = 0.0, m_r = 0.0, mw_r[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int nw = wn_s[v];
            mw_r[v] = nw ? wsh_s[v][row] + red_s[v][256 + row] / nw : 0.0;
            m_r += nw * mw_r[v];
        }
        m_r *= inv_p;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int nw = wn_s[v];
            if (nw == 0) continue;
            cs += red_s[v][row * 16 + c] - red_s[v][256 + row] * red_s[v][256 + c] / nw +
                  nw * (mw_r[v] - m_r) * (mw_c[v] - m_c);
        }
        ls[lane * 4 + i] = cs * inv_p1;  // state layout: lane (g, c), register i = row 4g+i
    }
    if (g == 0) ls[256 + c] = (c < b) ? m_c : 0.0;
}

// ============================================================================
// Projection of the learned surrogate: z - zref = W (x - xref) on FP32 matrix
// cores, with xref the stream's first pixel and zref = W xref + c.  ERX is
// exactly invariant to a constant shift of its input, and subtracting xref
// before the product keeps the accumulated values (and their FP32 rounding) at
// the scale of the data's spread, which is what the statistics of the z stream
// resolve.  A wave projects 16-pixel tiles: lane (g, c) supplies bands
// 16K+4g..16K+4g+3 of pixel c and holds the W tile of those bands in operand
// form, so four 16x16x4 MFMAs per 16 bands accumulate the 16 outputs of the 16
// pixels (outputs 4g..4g+3 of pixel c in lane (g, c)).  W is FP16.
// ============================================================================
template <bool VEC>
__global__ __launch_bounds__(256) void k_sproj(const float* __restrict__ X, long long npx, int b, int NTx,
                                               const __half* __restrict__ W16, const float* __restrict__ xref,
                                               float* __restrict__ Z)
{
    extern __shared__ f4 Wt[];  // [NTx][64] W tiles in operand form, then xref [16 NTx]
    float* xr_s = (float*)(Wt + NTx * 64);
    for (int i = threadIdx.x; i < NTx * 64; i += 256) {
        const int K = i >> 6, l = i & 63, g = l >> 4, c = l & 15;
        f4 v;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int band = 16 * K + 4 * g + q;
            v[q] = band < b ? __half2float(W16[c * b + band]) : 0.f;
        }
        Wt[i] = v;
    }
    for (int i = threadIdx.x; i < 16 * NTx; i += 256) xr_s[i] = i < b ? xref[i] : 0.f;
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
    const long long px = ((long long)blockIdx.x * 4 + w) * 16 + c;
    const bool okp = px < npx;
    f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int K = 0; K < NTx; ++K) {
        const int band0 = 16 * K + 4 * g;
        const bool okl = okp && band0 < b;
        const f4 v = ldq<DT_F32, VEC>(X, okl ? (size_t)px * b + band0 : 0, okl ? b - band0 : 0);
        f4 r;
#pragma unroll
        for (int q = 0; q < 4; ++q) r[q] = (okl && band0 + q < b) ? v[q] - xr_s[band0 + q] : 0.f;
        acc = mma_xty(acc, Wt[K * 64 + lane], r);
    }
    if (okp) *(f4*)(Z + px * 16 + 4 * g) = acc;
}

hipError_t launch_sproj(const float* X, long long npx, int b, const __half* W16, const float* xref, float* Z,
                        hipStream_t s)
{
    const int NTx = (b + 15) / 16;
    const size_t lds = (size_t)NTx * 64 * sizeof(f4) + 16 * NTx * sizeof(float);
    const dim3 grid((unsigned)((npx + 63) / 64));
    if (b % 4 == 0 && (uintptr_t)X % 16 == 0)
        hipLaunchKernelGGL(k_sproj<true>, grid, dim3(256), lds, s, X, npx, b, NTx, W16, xref, Z);
    else
        hipLaunchKernelGGL(k_sproj<false>, grid, dim3(256), lds, s, X, npx, b, NTx, W16, xref, Z);
    return hipGetLastError();
}

hipError_t launch_gram1x(const Pass& P, double* stats, hipStream_t s)
{
    hipLaunchKernelGGL(k_gram1x, dim3((unsigned)P.nlines), dim3(256), 0, s, P, stats, stat_entries(1));
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
