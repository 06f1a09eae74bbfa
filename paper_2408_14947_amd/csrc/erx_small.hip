// Fused path for streams of at most 16 bands (one 16-band tile): the whole
// method of Sec. III-C to III-E in one kernel per pass, the moving-average
// recurrence of each stream kept on chip across its lines.
#include "erx_device.h"

namespace erx {

// ============================================================================
// Small band counts (b <= 16, one 16-band tile): the whole method fused, with
// the moving-average recurrence kept on chip (Sec. III-C to III-E).
//
// One workgroup (4 waves) per stream walks that stream's lines in order:
//   Gram    wave w takes 16-pixel tiles w, w+4, ...; a tile (lane (g, c):
//           pixels 4g..4g+3 of band c) gives X^T X in four FP64 MFMAs.  Each
//           wave shifts its values by the first pixel of its first tile, in
//           FP64, so the products and sums are exact for every storage type
//           (an FP32 Gram would lose up to kappa * 2^-24 on the ill-conditioned
//           backgrounds of lines with fewer pixels than bands; here the cost is
//           small); the four waves' shifted sums are combined exactly.
//   EMA     wave 0 holds K_t and mu_t in FP64 registers (the state layout).
//   Factor  wave 0: K_t + eps I (padded bands: identity), Cholesky and
//           inverse of the 16 x 16 block in FP64.
//   Score   Y = L^{-1} R for 16-pixel tiles (four FP32 MFMAs), delta = ||y||.
//   Norm    optional per-line standardisation of the scores.
// The line is read from global memory twice (statistics, then scores); the
// second read comes from L2.  Every line is factored in FP64 (counted as an
// FP64 factorisation); lines whose block is not positive definite score NaN.
// ============================================================================
// Loads are issued in batches of SB tiles per wave (one: more batches in
// flight per wave would cost a wave per SIMD), the next batch in flight
// while the current one is multiplied, and the first batch of the next phase
// (the scores of this line, the Gram of the next line) is issued before the
// barrier that precedes it.  All loads are unconditional (clamped addresses,
// values masked where used).
constexpr int SB = 1;

// Raw storage values, converted to FP32 only where they are used (a
// conversion right after a load would make the compiler wait for it).
template <int DT> struct Raw1 {
    typedef unsigned short T;
    static __device__ __forceinline__ T ld(const void* X, size_t i) { return glb((const unsigned short*)X)[i]; }
    static __device__ __forceinline__ float cvt(T v)
    {
        return DT == DT_F16 ? __half2float(__ushort_as_half(v)) : (float)v * (1.0f / 65536.0f);
    }
};
template <> struct Raw1<DT_F32> {
    typedef float T;
    static __device__ __forceinline__ T ld(const void* X, size_t i) { return glb((const float*)X)[i]; }
    static __device__ __forceinline__ float cvt(T v) { return v; }
};
// four consecutive elements [i, i+4): one vector load with VEC, else element
// loads of the first `left` ones (offset clamped to 0 for the rest)
template <int DT, bool VEC> struct Raw4 {
    typename Raw1<DT>::T e[4];
    __device__ __forceinline__ void ld(const void* X, size_t i, int left)
    {
#pragma unroll
        for (int q = 0; q < 4; ++q) e[q] = Raw1<DT>::ld(X, q < left ? i + q : 0);
    }
    __device__ __forceinline__ f4 cvt() const
    {
        return f4{Raw1<DT>::cvt(e[0]), Raw1<DT>::cvt(e[1]), Raw1<DT>::cvt(e[2]), Raw1<DT>::cvt(e[3])};
    }
};
template <> struct Raw4<DT_F32, true> {
    f4 v;
    __device__ __forceinline__ void ld(const void* X, size_t i, int) { v = *(const GLB f4*)glb((const float*)X + i); }
    __device__ __forceinline__ f4 cvt() const { return v; }
};
template <int DT> struct Raw4H {
    u2v v;
    __device__ __forceinline__ void ld(const void* X, size_t i, int)
    {
        v = *(const GLB u2v*)glb((const unsigned short*)X + i);
    }
    __device__ __forceinline__ f4 cvt() const
    {
        return f4{Raw1<DT>::cvt((unsigned short)(v.x & 0xffffu)), Raw1<DT>::cvt((unsigned short)(v.x >> 16)),
                  Raw1<DT>::cvt((unsigned short)(v.y & 0xffffu)), Raw1<DT>::cvt((unsigned short)(v.y >> 16))};
    }
};
template <> struct Raw4<DT_F16, true> : Raw4H<DT_F16> {};
template <> struct Raw4<DT_U16, true> : Raw4H<DT_U16> {};

template <int DT, bool VEC>
__global__ __launch_bounds__(256) void k_small(const Pass P, int normalise, unsigned long long* __restrict__ ctr)
{
    const int sidx = blockIdx.x;
    if (sidx >= P.nstreams) return;  // uniform for the workgroup
    const StreamDesc d = P.sd ? load_desc(P.sd + sidx) : P.one;
    const int p = d.p, b = d.b;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
    __shared__ double red_s[4][256 + 16];
    __shared__ double xt_s[16 * 17];
    __shared__ double nrm_s[4][2];
    __shared__ double wsh_s[4][16];
    __shared__ float mu_s[16];
    __shared__ int wn_s[4];
    __shared__ int bad_s;

    GLB double* state = glb((double*)d.state);  // the fused path keeps an FP64 state
    double Kst[4] = {0.0, 0.0, 0.0, 0.0}, mst = 0.0;  // wave 0: K (state layout) and mu of band c
    if (w == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) Kst[i] = state[lane * 4 + i];
        mst = state[256 + c];
    }
    const int ntile = (p + 15) >> 4;
    const int ntw = ntile > w ? (ntile - w + 3) >> 2 : 0;  // tiles of this wave: w, w+4, ...
    const int nbat = (ntw + SB - 1) / SB;
    const double inv_p = 1.0 / (double)p, inv_p1 = 1.0 / (double)(p - 1);
    const size_t line_elems = (size_t)p * b;
    const int band0 = 4 * g;

    // Gram operands: lane (g, c) holds pixels 4g..4g+3 of band c of a tile
    typedef typename Raw1<DT>::T RT;
    auto gload = [&](const void* X, int j, RT (&buf)[SB][4]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int tt = w + 4 * (SB * j + u);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int px = 16 * tt + 4 * g + i;
                const bool ok = px < p && c < b;
                buf[u][i] = Raw1<DT>::ld(X, ok ? (size_t)px * b + c : 0);
            }
        }
    };
    // score operands: lane (g, c) holds bands 4g..4g+3 of pixel c of a tile
    auto sload = [&](const void* X, int j, Raw4<DT, VEC> (&buf)[SB]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int tt = w + 4 * (SB * j + u);
            const int px = 16 * tt + c;
            const bool okl = px < p && band0 < b;
            buf[u].ld(X, okl ? (size_t)px * b + band0 : 0, okl ? b - band0 : 0);
        }
    };

    RT ga[SB][4], gb[SB][4];
    Raw4<DT, VEC> sa[SB], sb[SB];
    if (d.n > 0) gload(d.x, 0, ga);
    long long t = d.t0;
    for (int l = 0; l < d.n; ++l, ++t) {
        const void* X = advance<DT>(d.x, (size_t)l * line_elems);
        GLB float* out = glb(d.out + (size_t)l * p);

        // ---- Gram of this wave's tiles, shifted by the first pixel of the wave's
        //      first tile (a value of this line, so the sums stay well scaled).
        //      Differences in FP64 and FP64 products: exact for the storage types.
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
        double bsd = 0.0;
        const double sh = (double)__shfl(Raw1<DT>::cvt(ga[0][0]), c);  // pixel 16w, band c (lane c holds it)
        for (int j = 0; j < nbat; ++j) {
            gload(X, j + 1, gb);  // next batch (clamped past the end)
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int tt = w + 4 * (SB * j + u);
                d4 xv;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int px = 16 * tt + 4 * g + i;
                    xv[i] = (px < p && c < b) ? (double)Raw1<DT>::cvt(ga[u][i]) - sh : 0.0;
                }
                bsd += (xv[0] + xv[1]) + (xv[2] + xv[3]);
                acc = mma_xty(acc, xv, xv);
            }
#pragma unroll
            for (int u = 0; u < SB; ++u)
#pragma unroll
                for (int i = 0; i < 4; ++i) ga[u][i] = gb[u][i];
        }
        bsd += __shfl_xor(bsd, 16);
        bsd += __shfl_xor(bsd, 32);
        // FP64 accumulator layout: register i of lane (g, c) is row 4i+g, column c
#pragma unroll
        for (int i = 0; i < 4; ++i) red_s[w][(4 * i + g) * 16 + c] = acc[i];
        if (g == 0) {
            red_s[w][256 + c] = bsd;
            wsh_s[w][c] = ntw ? sh : 0.0;
        }
        // pixels of this wave: 16 per tile, less the shortfall of the last tile if it is this wave's
        if (lane == 0) wn_s[w] = ntw ? 16 * ntw - (((ntile - 1 - w) & 3) == 0 ? 16 * ntile - p : 0) : 0;
        sload(X, 0, sa);  // first score batch, in flight during the factorisation
        __syncthreads();

        // ---- line statistics, moving averages and factorisation (wave 0).
        //      The per-wave sums (shift s_w, n_w pixels, B_w = sum(x - s_w),
        //      S_w = sum (x - s_w)(x - s_w)^T) combine exactly:
        //      m_w = s_w + B_w / n_w, m = sum n_w m_w / p,
        //      C = sum_w [S_w - B_w B_w^T / n_w + n_w (m_w - m)(m_w - m)^T].
        if (w == 0) {
            const double a = (t == 0) ? 1.0 : d.alpha;
            double mw_c[4], m_c = 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int nw = wn_s[v];
                mw_c[v] = nw ? wsh_s[v][c] + red_s[v][256 + c] / nw : 0.0;
                m_c += nw * mw_c[v];
            }
            m_c *= inv_p;
            double aa[4];
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
                const double kh = cs * inv_p1;
                Kst[i] = (1.0 - a) * Kst[i] + a * kh;
                double av = Kst[i];
                if (row >= b || c >= b) av = (row == c) ? 1.0 : 0.0;
                else if (row == c) av += d.eps;
                aa[i] = av;
            }
            const double muh = (c < b) ? m_c : 0.0;
            mst = (1.0 - a) * mst + a * muh;
            if (lane < 16) mu_s[lane] = (float)mst;
            double xx[4];
            const int bad = factor16(aa, xx, lane, b);
#pragma unroll
            for (int i = 0; i < 4; ++i) xt_s[(4 * g + i) * 17 + c] = xx[i];  // X[4g+i][c]
            if (lane == 0) {
                bad_s = bad;
                atomicAdd(&ctr[0], 1ull);
                if (bad) atomicAdd(&ctr[1], 1ull);
            }
        }
        __syncthreads();

        // ---- scores
        const bool bad = bad_s != 0;
        f4 xt, m4;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            xt[i] = (float)xt_s[c * 17 + 4 * g + i];  // X^T[4g+i][c]
            m4[i] = mu_s[4 * g + i];
        }
        double s1 = 0.0, s2 = 0.0;
        const void* Xn = advance<DT>(d.x, (size_t)(l + 1 < d.n ? l + 1 : l) * line_elems);
        for (int j = 0; j < nbat; ++j) {
            if (j + 1 < nbat) sload(X, j + 1, sb);
            else gload(Xn, 0, ga);  // the next line's first Gram batch
#pragma unroll
            for (int u = 0; u < SB; ++u) {
                const int tt = w + 4 * (SB * j + u);
                const int px = 16 * tt + c;
                const bool okp = px < p;
                f4 r;
                const f4 xr = sa[u].cvt();
#pragma unroll
                for (int q = 0; q < 4; ++q) r[q] = (okp && band0 + q < b) ? xr[q] - m4[q] : 0.f;
                const f4 y = mma_xty(f4{0.f, 0.f, 0.f, 0.f}, xt, r);  // L^{-1} r of pixel c, rows 4g..4g+3
                float ss = (y[0] * y[0] + y[1] * y[1]) + (y[2] * y[2] + y[3] * y[3]);
                ss += __shfl_xor(ss, 16);
                ss += __shfl_xor(ss, 32);
                const float dl = bad ? __builtin_nanf("") : sqrtf(ss);
                if (g == 0 && okp) {
                    out[px] = dl;
                    s1 += (double)dl;
                    s2 += (double)dl * (double)dl;
                }
            }
#pragma unroll
            for (int u = 0; u < SB; ++u) sa[u] = sb[u];
        }
        if (nbat == 0) gload(Xn, 0, ga);
        if (normalise && d.outn) {
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                s1 += __shfl_xor(s1, o);
                s2 += __shfl_xor(s2, o);
            }
            if (lane == 0) {
                nrm_s[w][0] = s1;
                nrm_s[w][1] = s2;
            }
            __syncthreads();
            const double m1 = (nrm_s[0][0] + nrm_s[1][0] + nrm_s[2][0] + nrm_s[3][0]) * inv_p;
            const double m2 = (nrm_s[0][1] + nrm_s[1][1] + nrm_s[2][1] + nrm_s[3][1]) * inv_p;
            const double var = m2 - m1 * m1;
            const double sd = var > 0.0 ? sqrt(var) : 0.0;
            GLB float* outn = glb(d.outn + (size_t)l * p);
            for (int px = tid; px < p; px += 256)
                outn[px] = sd > 0.0 ? (float)(((double)out[px] - m1) / sd) : 0.f;
        }
        __syncthreads();
    }
    if (w == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) state[lane * 4 + i] = Kst[i];
        if (lane < 16) state[256 + lane] = mst;
    }
}


// ============================================================================
// The same fused method with the line held in LDS, for passes whose lines fit
// the buffer and start on 16-byte boundaries.  Each thread keeps NR 16-byte
// words of the NEXT line in registers: their loads are issued as soon as the
// current line has been copied to LDS and complete while it is processed, so
// a line costs one memory round trip that overlaps the previous line's work
// instead of one per tile.  The Gram and the scores both read the line from
// LDS in the layout their MFMA operands need (a tile transposes between the
// two), so the line is read from global memory once.
//
// The Gram shift is the line's first pixel, common to the four waves, so their
// FP64 sums S = sum (x - s)(x - s)^T and B = sum (x - s) add directly and the
// centred covariance is S - B B^T / p (FP64 differences and products, as in
// the path above).
// ============================================================================
template <int DT, int NR>
__global__ __launch_bounds__(256, 3) void k_small_l(const Pass P, int normalise, unsigned long long* __restrict__ ctr)
{
    extern __shared__ u4v lbuf[];  // the current line, raw storage values
    const int sidx = blockIdx.x;
    if (sidx >= P.nstreams) return;  // uniform for the workgroup
    const StreamDesc d = P.sd ? load_desc(P.sd + sidx) : P.one;
    const int p = d.p, b = d.b;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
    __shared__ double red_s[4][256 + 16];
    __shared__ double xt_s[16 * 17];
    __shared__ double nrm_s[4][2];
    __shared__ float mu_s[16];
    __shared__ int bad_s;

    typedef typename Raw1<DT>::T RT;
    const RT* lx = (const RT*)lbuf;
    const size_t line_elems = (size_t)p * b;
    const int nq = (int)(line_elems * sizeof(RT) / 16);  // 16-byte words of a line (exact)
    u4v pf[NR];
    // unconditional loads of the line's words (clamped to the last one), kept raw
    auto lload = [&](const void* X, int tl) __attribute__((always_inline)) {
        const GLB u4v* q = (const GLB u4v*)X;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int i = tl + 256 * r;
            pf[r] = q[i < nq ? i : nq - 1];
        }
    };
    auto lstore = [&](int tl) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int i = tl + 256 * r;
            if (i < nq) lbuf[i] = pf[r];
        }
    };

    GLB double* state = glb((double*)d.state);  // the fused path keeps an FP64 state
    double Kst[4] = {0.0, 0.0, 0.0, 0.0}, mst = 0.0;  // wave 0: K (state layout) and mu of band c
    if (w == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) Kst[i] = state[lane * 4 + i];
        mst = state[256 + c];
    }
    const int ntile = (p + 15) >> 4;
    const double inv_p = 1.0 / (double)p, inv_p1 = 1.0 / (double)(p - 1);

    if (d.n > 0) lload(d.x, tid);
    long long t = d.t0;
    for (int l = 0; l < d.n; ++l, ++t) {
        // Lane-dependent indices are re-derived each line from a thread index the
        // compiler cannot see through: hoisted out of the loop, the many masks and
        // addresses computed from them would stay live across it and spill.
        int tl = tid;
        __asm__ volatile("" : "+v"(tl));
        const int lane = tl & 63, g = lane >> 4, c = lane & 15;
        GLB float* out = glb(d.out + (size_t)l * p);
        __syncthreads();  // the previous line's reads of the buffer are done
        lstore(tl);
        if (l + 1 < d.n) lload(advance<DT>(d.x, (size_t)(l + 1) * line_elems), tl);
        __syncthreads();

        // ---- Gram of tiles w, w+4, ... shifted by pixel 0 (lane (g, c): pixels
        //      4g..4g+3 of band c), two tiles per step: the next two tiles' LDS
        //      reads are in flight during this step's products, whose two MFMA
        //      chains (one accumulator per tile) are interleaved.  Tiles past the
        //      end read element 0 and are masked to zero.
        // LDS addresses are clamped into the line (pixel p-1, band b-1) rather than
        // selected: a select on the address becomes a branch around each read and a
        // wait after it.  Values outside the line are masked where they are used.
        // Narrow streams (b <= 8) pack G = 16 / bp pixel groups into the 16 band
        // rows of a tile (bp = 4 or 8, group j in rows j*bp..j*bp+bp-1): the
        // diagonal bp x bp blocks of the product are the Gram sums of the groups'
        // pixels and add up to the line's, with G times fewer products.
        const int lg = b <= 4 ? 2 : (b <= 8 ? 3 : 4);
        const int bp = 1 << lg, G = 16 >> lg, SP = 16 * G;  // SP pixels per tile
        const int band = c & (bp - 1), grp = c >> lg;
        const int nst = (p + SP - 1) / SP;
        const int cb = band < b ? band : b - 1;
        const double sh = (band < b) ? (double)Raw1<DT>::cvt(lx[cb]) : 0.0;
        auto graw = [&](int tt, RT (&v)[4]) __attribute__((always_inline)) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int px = SP * tt + 16 * grp + 4 * g + i;
                v[i] = lx[(px < p ? px : p - 1) * b + cb];
            }
        };
        auto gval = [&](int tt, const RT (&v)[4]) __attribute__((always_inline)) {
            d4 xv;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int px = SP * tt + 16 * grp + 4 * g + i;
                xv[i] = (px < p && band < b) ? (double)Raw1<DT>::cvt(v[i]) - sh : 0.0;
            }
            return xv;
        };
        d4 acc0 = d4{0.0, 0.0, 0.0, 0.0}, acc1 = d4{0.0, 0.0, 0.0, 0.0};
        double bsd = 0.0;
        RT ra[4], rb[4];
        graw(w, ra);
        graw(w + 4, rb);
        for (int tt = w; tt < nst; tt += 8) {
            const d4 x0 = gval(tt, ra), x1 = gval(tt + 4, rb);
            graw(tt + 8, ra);
            graw(tt + 12, rb);
            bsd += ((x0[0] + x0[1]) + (x0[2] + x0[3])) + ((x1[0] + x1[1]) + (x1[2] + x1[3]));
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                acc0 = mfma(x0[k], x0[k], acc0);
                acc1 = mfma(x1[k], x1[k], acc1);
            }
        }
        bsd += __shfl_xor(bsd, 16);
        bsd += __shfl_xor(bsd, 32);
        // FP64 accumulator layout: register i of lane (g, c) is row 4i+g, column c
#pragma unroll
        for (int i = 0; i < 4; ++i) red_s[w][(4 * i + g) * 16 + c] = acc0[i] + acc1[i];
        if (g == 0) red_s[w][256 + c] = bsd;
        __syncthreads();

        // ---- line statistics, moving averages and factorisation (wave 0)
        if (w == 0) {
            const double a = (t == 0) ? 1.0 : d.alpha;
            // sums over the four waves and the G pixel groups (band r of group j
            // is row j*bp + r of the waves' products)
            auto bsum = [&](int r) __attribute__((always_inline)) {
                double v = 0.0;
                for (int j = 0; j < G; ++j)
                    v += (red_s[0][256 + j * bp + r] + red_s[1][256 + j * bp + r]) +
                         (red_s[2][256 + j * bp + r] + red_s[3][256 + j * bp + r]);
                return v;
            };
            const double bc = c < bp ? bsum(c) : 0.0;
            double aa[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 4 * g + i;
                double s = 0.0, br = 0.0;
                if (row < bp && c < bp) {
                    br = bsum(row);
                    for (int j = 0; j < G; ++j) {
                        const int e = (j * bp + row) * 16 + j * bp + c;
                        s += (red_s[0][e] + red_s[1][e]) + (red_s[2][e] + red_s[3][e]);
                    }
                }
                const double kh = (s - br * bc * inv_p) * inv_p1;
                Kst[i] = (1.0 - a) * Kst[i] + a * kh;
                double av = Kst[i];
                if (row >= b || c >= b) av = (row == c) ? 1.0 : 0.0;
                else if (row == c) av += d.eps;
                aa[i] = av;
            }
            const double muh = (c < b) ? sh + bc * inv_p : 0.0;
            mst = (1.0 - a) * mst + a * muh;
            if (lane < 16) mu_s[lane] = (float)mst;
            double xx[4];
            const int bad = factor16(aa, xx, lane, b);
            // X[4g+i][c], zero in the padded rows and columns: the scores then
            // need no band mask (padded residual entries are finite, see below)
#pragma unroll
            for (int i = 0; i < 4; ++i) xt_s[(4 * g + i) * 17 + c] = (4 * g + i < b && c < b) ? xx[i] : 0.0;
            if (lane == 0) {
                bad_s = bad;
                atomicAdd(&ctr[0], 1ull);
                if (bad) atomicAdd(&ctr[1], 1ull);
            }
        }
        __syncthreads();

        // ---- scores (lane (g, c): bands g, 4+g, 8+g, 12+g of pixel c of a tile,
        //      so that product k contracts bands 4k..4k+3 and the products past
        //      the stream's band count are skipped)
        const bool bad = bad_s != 0;
        const int nkb = (b + 3) >> 2;  // 4-band groups holding real bands
        f4 xt, m4;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            xt[i] = (float)xt_s[c * 17 + 4 * i + g];  // X[c][4i+g]
            m4[i] = mu_s[4 * i + g];
        }
        double s1 = 0.0, s2 = 0.0;
        // two tiles per step as in the Gram: next reads in flight, chains interleaved
        auto sraw = [&](int tt, RT (&v)[4]) __attribute__((always_inline)) {
            const int px = 16 * tt + c;
            const int row = (px < p ? px : p - 1) * b;
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = lx[row + (4 * q + g < b ? 4 * q + g : b - 1)];
        };
        // Reads outside the line were clamped to an element of it, so every
        // residual entry is finite: padded bands meet zero columns of X and
        // pixels past p are not stored, so no mask is needed.
        auto sval = [&](int tt, const RT (&v)[4]) __attribute__((always_inline)) {
            f4 r;
#pragma unroll
            for (int q = 0; q < 4; ++q) r[q] = Raw1<DT>::cvt(v[q]) - m4[q];
            return r;
        };
        auto emit = [&](int tt, const f4 y) __attribute__((always_inline)) {
            float ss = (y[0] * y[0] + y[1] * y[1]) + (y[2] * y[2] + y[3] * y[3]);
            ss += __shfl_xor(ss, 16);
            ss += __shfl_xor(ss, 32);
            const float dl = bad ? __builtin_nanf("") : __builtin_amdgcn_sqrtf(ss);
            const int px = 16 * tt + c;
            if (g == 0 && px < p) {
                out[px] = dl;
                if (normalise) {
                    s1 += (double)dl;
                    s2 += (double)dl * (double)dl;
                }
            }
        };
        RT qa[4], qb[4];
        sraw(w, qa);
        sraw(w + 4, qb);
        for (int tt = w; tt < ntile; tt += 8) {
            const f4 r0 = sval(tt, qa), r1 = sval(tt + 4, qb);
            sraw(tt + 8, qa);
            sraw(tt + 12, qb);
            f4 y0 = f4{0.f, 0.f, 0.f, 0.f}, y1 = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < 4; ++k) {  // L^{-1} r of pixel c, rows 4g..4g+3
                if (k < nkb) {
                    y0 = mfma(xt[k], r0[k], y0);
                    y1 = mfma(xt[k], r1[k], y1);
                }
            }
            emit(tt, y0);
            emit(tt + 4, y1);
        }
        if (normalise && d.outn) {
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                s1 += __shfl_xor(s1, o);
                s2 += __shfl_xor(s2, o);
            }
            if (lane == 0) {
                nrm_s[w][0] = s1;
                nrm_s[w][1] = s2;
            }
            __syncthreads();
            const double m1 = (nrm_s[0][0] + nrm_s[1][0] + nrm_s[2][0] + nrm_s[3][0]) * inv_p;
            const double m2 = (nrm_s[0][1] + nrm_s[1][1] + nrm_s[2][1] + nrm_s[3][1]) * inv_p;
            const double var = m2 - m1 * m1;
            const double sd = var > 0.0 ? sqrt(var) : 0.0;
            GLB float* outn = glb(d.outn + (size_t)l * p);
            for (int px = tl; px < p; px += 256)
                outn[px] = sd > 0.0 ? (float)(((double)out[px] - m1) / sd) : 0.f;
        }
    }
    if (w == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) state[lane * 4 + i] = Kst[i];
        if (lane < 16) state[256 + lane] = mst;
    }
}

// largest line (bytes) the LDS-resident variant takes: 10 words per thread
constexpr int SMALL_LDS_MAX = 10 * 256 * 16;

template <int DT, int NR>
static void small_l(const Pass& P, int normalise, unsigned long long* ctr, hipStream_t s)
{
    hipLaunchKernelGGL((k_small_l<DT, NR>), dim3((unsigned)P.nstreams), dim3(256), (size_t)NR * 256 * 16, s, P,
                       normalise, ctr);
}

template <int DT>
static void small_l(int line_bytes, const Pass& P, int normalise, unsigned long long* ctr, hipStream_t s)
{
    if (line_bytes <= 2 * 4096) small_l<DT, 2>(P, normalise, ctr, s);
    else if (line_bytes <= 4 * 4096) small_l<DT, 4>(P, normalise, ctr, s);
    else small_l<DT, 10>(P, normalise, ctr, s);
}

hipError_t launch_small(int dtype, const Pass& P, int normalise, unsigned long long* ctr, int lds_line_bytes,
                        hipStream_t s)
{
    if (lds_line_bytes > 0 && lds_line_bytes <= SMALL_LDS_MAX) {
        switch (dtype) {
        case DT_F32: small_l<DT_F32>(lds_line_bytes, P, normalise, ctr, s); break;
        case DT_F16: small_l<DT_F16>(lds_line_bytes, P, normalise, ctr, s); break;
        default: small_l<DT_U16>(lds_line_bytes, P, normalise, ctr, s); break;
        }
        return hipGetLastError();
    }
    const dim3 grid((unsigned)P.nstreams), block(256);
#define ERX_SMALL(DTV)                                                                                      \
    if (P.vec4) hipLaunchKernelGGL((k_small<DTV, true>), grid, block, 0, s, P, normalise, ctr);            \
    else hipLaunchKernelGGL((k_small<DTV, false>), grid, block, 0, s, P, normalise, ctr);
    switch (dtype) {
    case DT_F32: ERX_SMALL(DT_F32) break;
    case DT_F16: ERX_SMALL(DT_F16) break;
    default: ERX_SMALL(DT_U16) break;
    }
#undef ERX_SMALL
    return hipGetLastError();
}

}  // namespace erx
