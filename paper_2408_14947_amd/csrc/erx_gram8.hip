// Split-FP16 line Gram on 128-band macro tiles (Sec. III-C, Eqs. (18)-(19)).
//
// The arithmetic is that of the split-FP16 branch of k_gram4, operation for
// operation: each band is shifted by the FP32 mean s of its first min(64, p)
// pixels and scaled by the power of two c set by the largest |x - s| of those
// pixels; v c splits into FP16 halves h + l; a 32-pixel step of a 16x16 tile is
// h_a h_b + h_a l_b + l_a h_b on the 16x16x32 FP16 MFMA; FP32 partials over 64
// pixels go into FP64 after the scales are undone; band sums are FP64; and
// sum (x-mu)(x-mu)^T = sum (x-s)(x-s)^T - p (mu-s)(mu-s)^T gives the centred
// Gram.  Both kernels therefore write the same statistics bit for bit.
//
// What differs is the blocking.  A workgroup of 16 waves computes one 128x128
// block (8x8 tiles of 16 bands) of the upper triangle of one line, so an
// element is shifted, range-checked and split once per macro tile that needs
// its band: at 224 bands twice (as a row and as a column), where 64-band macro
// tiles do it four times; that conversion, not the matrix cores, bounded the
// split Gram on 64-band macro tiles.  Here the per-chunk barrier makes the
// staging and the products of all 16 waves take turns.  Wave w owns tile row w mod 8 and tile columns 4 (w div 8) + 0..3
// of the macro tile (on a diagonal macro tile only those on or right of the
// diagonal).
//
// Staging: per 64-pixel chunk, waves 0-7 load the row panel and waves 8-15 the
// column panel (a diagonal macro tile has one panel, staged by waves 0-7).
// Within a panel, wave v covers band half v mod 2 (64 bands) and pixel quads
// pq = 4 (v div 2) + k, k = lane div 16; lane (k, j) loads pixels
// 4pq..4pq+3 of bands 4j..4j+3 of its half, so 16 lanes read one contiguous
// 256-byte segment of a pixel row, and transposes the 4x4 block in registers
// into 8-byte band-row stores.  LDS holds, per panel, an FP16 hi plane and an
// FP16 lo plane of 128 band rows x 64 pixels, octets XOR-swizzled by
// (row div 2) mod 8, double-buffered (128 KiB).  Loads run one chunk ahead in
// registers, one barrier per chunk.
//
// A macro tile that meets a band constant over its first chunk, or a later
// value beyond the scale's headroom, is left to the FP32 Gram: the 64-band
// macro tiles it covers are flagged in Pass::gredo (each pass writes every
// flag, 0 or 1, since the 128-band macro tiles partition the 64-band ones).
#include "erx_device.h"

namespace erx {

namespace {

typedef _Float16 g8h4 __attribute__((ext_vector_type(4)));
typedef _Float16 g8h8 __attribute__((ext_vector_type(8)));

constexpr int G8_B = 128;            // bands per panel
constexpr int G8_PLANE = G8_B * 64;  // halves per plane: 128 band rows x 64 pixels

__device__ __forceinline__ int g8_sw(int r) { return (r >> 1) & 7; }

// the FP16 halves of the scaled values w4 of pixels 4pq..4pq+3 of band row r
__device__ __forceinline__ void g8_put(uint16_t* H, int r, int pq, const f4 w4)
{
    const g8h4 hi = __builtin_convertvector(w4, g8h4);
    const f4 back = __builtin_convertvector(hi, f4);
    f4 d4;
#pragma unroll
    for (int q = 0; q < 4; ++q) d4[q] = w4[q] - back[q];
    const int off = r * 64 + 8 * ((pq >> 1) ^ g8_sw(r)) + 4 * (pq & 1);
    *(g8h4*)&H[off] = hi;
    *(g8h4*)&H[G8_PLANE + off] = __builtin_convertvector(d4, g8h4);
}

__device__ __forceinline__ f4 g8_mma(g8h8 a, g8h8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// One 64-pixel chunk of tiles (rt, ct0 + q), q < NQ: A rows from panel RA, B
// rows from panel RB; pixel octet (u / 8) + g of band row 16t + c per lane.
template <int NQ>
__device__ __forceinline__ void g8_chunk(const uint16_t* RA, const uint16_t* RB, int rt, int ct0, int c, int g,
                                         int kend, f4* acc)
{
    const int ra = 16 * rt + c;
    for (int u = 0; u < kend; u += 32) {
        const int oc = (u >> 3) + g;
        const int oa = ra * 64 + 8 * (oc ^ g8_sw(ra));
        const g8h8 ah = *(const g8h8*)&RA[oa];
        const g8h8 al = *(const g8h8*)&RA[G8_PLANE + oa];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int rb = 16 * (ct0 + q) + c;
            const int ob = rb * 64 + 8 * (oc ^ g8_sw(rb));
            const g8h8 bh = *(const g8h8*)&RB[ob];
            const g8h8 bl = *(const g8h8*)&RB[G8_PLANE + ob];
            acc[q] = g8_mma(ah, bh, acc[q]);
            acc[q] = g8_mma(ah, bl, acc[q]);
            acc[q] = g8_mma(al, bh, acc[q]);
        }
    }
}

template <int DT, bool VEC, bool DG>
__device__ __forceinline__ void gram8_macro(const void* X, int p, int b, int NT, int nm, int MI, int MJ, int line,
                                            const Pass& P, void* __restrict__ stats, long long E,
                                            uint16_t (*pl)[2][2 * G8_PLANE], float* shift_s, float* scl_s,
                                            double* bsum_s, int* redo_s)
{
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63, g = lane >> 4, c = lane & 15;

    // staging role: panel pn (0 rows, 1 columns), band half bh, pixel quad pq
    const int pn = w >> 3, v = w & 7, bh = v & 1, pq = 4 * (v >> 1) + g;
    const bool stager = !(DG && pn == 1);  // wave-uniform
    const int pr = 64 * bh + 4 * c;        // first band of this lane within its panel
    const int gb0 = G8_B * (pn ? MJ : MI) + pr;
    bool bok[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bok[j] = gb0 + j < b;

    f4 fs[4];
    auto fetch = [&](int k0, f4(&fr)[4]) __attribute__((always_inline)) {
        if (!stager) return;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int px = k0 + 4 * pq + r;
            const bool ok = px < p && bok[0];
            fr[r] = ldq<DT, VEC>(X, ok ? (size_t)px * b + gb0 : 0, ok ? b - gb0 : 0);
        }
    };
    fetch(0, fs);

    // shift s and split scale c of every band from the first chunk: per-lane
    // sums (maxima) over 4 pixels, then the 4 pixel quads of a wave, then the 4
    // waves of a band half through LDS (the order k_gram4 uses)
    float* part = (float*)pl[1][0];  // [panel][4][128] sums, then maxima; free before the first stage
    const int nv0 = p - 4 * pq;
    if (stager) {
        float a[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] = 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) a[j] += (r < nv0 && bok[j]) ? fs[r][j] : 0.f;
            a[j] += __shfl_xor(a[j], 16);
            a[j] += __shfl_xor(a[j], 32);
        }
        if (g == 0)
#pragma unroll
            for (int j = 0; j < 4; ++j) part[(pn * 4 + (v >> 1)) * 128 + pr + j] = a[j];
    }
    if (tid == 0) *redo_s = 0;
    __syncthreads();
    if (tid < 256) {
        const int pp = DG ? 0 : tid >> 7, bi = tid & 127;
        const float* q = part + pp * 512 + bi;
        const float inv0 = 1.0f / (float)(p < 64 ? p : 64);
        shift_s[tid] = ((q[0] + q[128]) + (q[256] + q[384])) * inv0;
    }
    __syncthreads();
    float sr[4];
    double dsr[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        sr[j] = 0.f;
        dsr[j] = 0.0;
    }
    if (stager) {
        const f4 sh = *(const f4*)&shift_s[pn * 128 + pr];
        float a[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] = 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) a[j] = fmaxf(a[j], (r < nv0 && bok[j]) ? fabsf(fs[r][j] - sh[j]) : 0.f);
            a[j] = fmaxf(a[j], __shfl_xor(a[j], 16));
            a[j] = fmaxf(a[j], __shfl_xor(a[j], 32));
        }
        if (g == 0)
#pragma unroll
            for (int j = 0; j < 4; ++j) part[1024 + (pn * 4 + (v >> 1)) * 128 + pr + j] = a[j];
    }
    __syncthreads();
    if (tid < 256) {
        const int pp = DG ? 0 : tid >> 7, bi = tid & 127;
        const float* q = part + 1024 + pp * 512 + bi;
        const float m = fmaxf(fmaxf(q[0], q[128]), fmaxf(q[256], q[384]));
        const int band = G8_B * (pp ? MJ : MI) + bi;
        float cv, ci;
        split_scale(m, cv, ci);
        scl_s[tid] = cv;
        scl_s[256 + tid] = ci;
        scl_s[512 + tid] = -(shift_s[tid] * cv);  // exact: c is a power of two
        if (band < b && !(m > 0.f)) *redo_s = 1;  // constant over the first chunk (or NaN)
    }
    __syncthreads();

    // (x - s) c is formed as one FMA, x c + (-s c): c is a power of two, so this is
    // the rounded x - s scaled exactly, the value k_gram4 forms in two steps.  The
    // band sums are kept in that scale (exactly c times the unscaled sums) and
    // unscaled when they are added into FP64.
    bool ovf = false;
    auto stage = [&](int k0, int buf, const f4(&fr)[4]) __attribute__((always_inline)) {
        if (!stager) return;
        uint16_t* H = pl[buf][pn];
        const int nv = p - k0 - 4 * pq;  // valid pixels among this lane's four
        // scales and shifts are read back from LDS, which keeps registers for the tiles
        const f4 cs = *(const f4*)&scl_s[pn * 128 + pr];
        const f4 ns = *(const f4*)&scl_s[512 + pn * 128 + pr];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            f4 x;
#pragma unroll
            for (int r = 0; r < 4; ++r) x[r] = (r < nv && bok[j]) ? fmaf(fr[r][j], cs[j], ns[j]) : 0.f;
            sr[j] += (x[0] + x[1]) + (x[2] + x[3]);
            ovf = ovf || absmax4(x) >= 32768.f;
            g8_put(H, pr + j, pq, x);
        }
    };

    // tiles of this wave: row rt, columns ct0 .. ct0 + nq - 1 of the macro tile
    const int rt = w & 7, hc = w >> 3;
    const int ncol = (NT - 8 * MJ) < 8 ? (NT - 8 * MJ) : 8;
    const bool rowok = 8 * MI + rt < NT;
    int ct0 = 4 * hc;
    if (DG && ct0 < rt) ct0 = rt;
    const int cth = (4 * hc + 3) < (ncol - 1) ? (4 * hc + 3) : (ncol - 1);
    const int nq = __builtin_amdgcn_readfirstlane(rowok && cth >= ct0 ? cth - ct0 + 1 : 0);

    double S[4][4];
    f4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        acc[q] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < 4; ++i) S[q][i] = 0.0;
    }

    // chunk j is multiplied from LDS buffer j & 1 while chunk j+1 is staged
    // from the registers into the other buffer, which then receive the loads
    // of chunk j+2; one barrier per chunk
    stage(0, 0, fs);
    fetch(64, fs);
    __syncthreads();
    for (int k0 = 0, it = 0;; k0 += 64, ++it) {
        const uint16_t* RA = pl[it & 1][0];
        const uint16_t* RB = pl[it & 1][DG ? 0 : 1];
        const int kend = (p - k0) < 64 ? (p - k0) : 64;
        switch (nq) {
        case 0: break;
        case 1: g8_chunk<1>(RA, RB, rt, ct0, c, g, kend, acc); break;
        case 2: g8_chunk<2>(RA, RB, rt, ct0, c, g, kend, acc); break;
        case 3: g8_chunk<3>(RA, RB, rt, ct0, c, g, kend, acc); break;
        default: g8_chunk<4>(RA, RB, rt, ct0, c, g, kend, acc); break;
        }
        // undo the band scales of row 16rt+4g+i and column 16(ct0+q)+c
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q < nq) {
                const double icq = (double)scl_s[256 + 128 + 16 * (ct0 + q) + c];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    S[q][i] += (double)acc[q][i] * ((double)scl_s[256 + 16 * rt + 4 * g + i] * icq);
            }
            acc[q] = f4{0.f, 0.f, 0.f, 0.f};
        }
        if (stager) {  // band sums of the chunks staged so far, unscaled
            const f4 ci = *(const f4*)&scl_s[256 + pn * 128 + pr];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                dsr[j] += (double)sr[j] * (double)ci[j];
                sr[j] = 0.f;
            }
        }
        if (k0 + 64 >= p) break;
        stage(k0 + 64, (it + 1) & 1, fs);
        fetch(k0 + 128, fs);
        __syncthreads();
    }
    __syncthreads();  // every wave has read its last operands before LDS is reused

    // band sums: the 4 pixel quads of a wave, then the 4 waves of a band half
    double* red = (double*)pl[0][0];  // [panel][4][128]
    if (stager) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            dsr[j] += __shfl_xor(dsr[j], 16);
            dsr[j] += __shfl_xor(dsr[j], 32);
        }
        if (g == 0)
#pragma unroll
            for (int j = 0; j < 4; ++j) red[(pn * 4 + (v >> 1)) * 128 + pr + j] = dsr[j];
    }
    if (ovf) *redo_s = 1;  // benign race: every writer stores 1
    __syncthreads();
    if (tid < 256) {
        const int pp = DG ? 0 : tid >> 7, bi = tid & 127;
        const double* q = red + pp * 512 + bi;
        bsum_s[tid] = (q[0] + q[128]) + (q[256] + q[384]);
    }
    __syncthreads();
    const int redo = *redo_s;
    if (tid == 0 && P.gredo) {
        // the 64-band macro tiles (a, e), a <= e, that this one covers
        const int MT4 = (NT + 3) >> 2;
        for (int a = 2 * MI; a < 2 * MI + 2 && a < MT4; ++a)
            for (int e = 2 * MJ; e < 2 * MJ + 2 && e < MT4; ++e)
                if (a <= e) P.gredo[(size_t)line * nm + a * MT4 - a * (a - 1) / 2 + (e - a)] = redo;
    }
    if (redo) return;  // uniform: the FP32 pass writes these tiles

    const double inv_p = 1.0 / (double)p, inv_p1 = 1.0 / (double)(p - 1);
    double* ls = (double*)stats + (size_t)line * E;
    float* ls32 = (float*)stats + (size_t)line * E;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= nq) continue;
        const int ct = ct0 + q;
        const double scol = bsum_s[128 + 16 * ct + c];
        double o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double srho = bsum_s[16 * rt + 4 * g + i];
            o[i] = (S[q][i] - srho * scol * inv_p) * inv_p1;
        }
        const long long off = tile_u(8 * MI + rt, 8 * MJ + ct, NT) * 256 + lane * 4;
        if (P.sf32) {
            *(float4*)(ls32 + off) = float4{(float)o[0], (float)o[1], (float)o[2], (float)o[3]};
        } else {
            *(double2*)(ls + off) = double2{o[0], o[1]};
            *(double2*)(ls + off + 2) = double2{o[2], o[3]};
        }
    }
    if (DG && w < 8 && g == 0 && rowok) {
        const long long ntU = (long long)NT * (NT + 1) / 2;
        const int band = G8_B * MI + 16 * w + c;
        const double m = (band < b) ? (double)shift_s[16 * w + c] + bsum_s[16 * w + c] * inv_p : 0.0;
        if (P.sf32) ls32[ntU * 256 + band] = (float)m;
        else ls[ntU * 256 + band] = m;
    }
}

// Grid: 8 * ceil(n/8) * nm8 workgroups of 1024 threads; all macro tiles of a
// line run on one XCD (block id mod 8), as in k_gram4.
template <int DT, bool VEC>
__global__ __launch_bounds__(1024) void k_gram8(const Pass P, int NT, int nm8, int nm, void* __restrict__ stats,
                                                long long E)
{
    const int bid = blockIdx.x;
    const int xcd = bid & 7;
    const int kk = bid >> 3;
    const int ll = kk / nm8;
    int m = kk - ll * nm8;
    const int line = ll * 8 + xcd;
    if (line >= P.nlines) return;  // uniform for the workgroup
    const StreamDesc d = stream_of_line(P, line);
    const int p = d.p, b = d.b;
    const void* X = advance<DT>(d.x, (size_t)(line - d.line0) * p * b);
    const int MT = (NT + 7) >> 3;
    int MI = 0;
    while (m >= MT - MI) {
        m -= MT - MI;
        ++MI;
    }
    const int MJ = MI + m;
    __shared__ __attribute__((aligned(16))) uint16_t pl[2][2][2 * G8_PLANE];  // [buffer][panel][hi, lo]
    __shared__ float shift_s[256];  // row panel bands, then column panel bands
    __shared__ float scl_s[768];    // scales (rows, columns), their inverses, then -shift * scale
    __shared__ double bsum_s[256];
    __shared__ int redo_s;
    if (MI == MJ)
        gram8_macro<DT, VEC, true>(X, p, b, NT, nm, MI, MJ, line, P, stats, E, pl, shift_s, scl_s, bsum_s, &redo_s);
    else
        gram8_macro<DT, VEC, false>(X, p, b, NT, nm, MI, MJ, line, P, stats, E, pl, shift_s, scl_s, bsum_s, &redo_s);
}

template <bool VEC>
void gram8_launch(int dtype, dim3 grid, hipStream_t s, const Pass& P, int NT, int nm8, int nm, void* stats,
                  long long E)
{
    const dim3 block(1024);
    switch (dtype) {
    case DT_F32: hipLaunchKernelGGL((k_gram8<DT_F32, VEC>), grid, block, 0, s, P, NT, nm8, nm, stats, E); break;
    case DT_F16: hipLaunchKernelGGL((k_gram8<DT_F16, VEC>), grid, block, 0, s, P, NT, nm8, nm, stats, E); break;
    default: hipLaunchKernelGGL((k_gram8<DT_U16, VEC>), grid, block, 0, s, P, NT, nm8, nm, stats, E); break;
    }
}

}  // namespace

hipError_t launch_gram8(int dtype, const Pass& P, int NT, int nm, void* stats, long long E, hipStream_t s)
{
    const int MT = (NT + 7) >> 3, nm8 = MT * (MT + 1) / 2;
    const dim3 grid((unsigned)((long long)((P.nlines + 7) / 8) * 8 * nm8));
    if (P.vec4) gram8_launch<true>(dtype, grid, s, P, NT, nm8, nm, stats, E);
    else gram8_launch<false>(dtype, grid, s, P, NT, nm8, nm, stats, E);
    return hipGetLastError();
}

}  // namespace erx
