// Device helpers shared by the ERX kernels: matrix-core tile products in the
// accumulator layout, global-memory access, pass descriptors and the
// single-wave factorisation of a 16x16 block.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <type_traits>
#include <utility>

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

__device__ __forceinline__ float absmax4(const f4 v)
{
    return fmaxf(fmaxf(fabsf(v[0]), fabsf(v[1])), fmaxf(fabsf(v[2]), fabsf(v[3])));
}

// Split-FP16 Gram operands: the power of two c with m c in [2^7, 2^8), so that
// values up to 128 m stay below 2^15 after scaling (1 when m is 0 or not
// finite), and 1 / c
__device__ __forceinline__ void split_scale(float m, float& c, float& inv)
{
    int E = ((__float_as_int(m) >> 23) & 0xff) - 127;
    const bool ok = m > 0.f && E < 128;
    E = E < -119 ? -119 : (E > 120 ? 120 : E);
    c = ok ? __int_as_float((127 + 7 - E) << 23) : 1.f;
    inv = ok ? __int_as_float((127 - 7 + E) << 23) : 1.f;
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
// Pointers that reach a kernel inside the pass descriptors are generic; the
// memory behind them is always device global memory, and accessing it through
// global-address-space pointers gives global (not flat) instructions, whose
// completion is tracked separately from LDS traffic.
#define GLB __attribute__((address_space(1)))
template <class T> __device__ __forceinline__ GLB T* glb(T* p) { return (GLB T*)p; }
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

// copy of a pass descriptor from global memory (class types cannot be copied
// out of a global-address-space lvalue directly)
__device__ __forceinline__ StreamDesc load_desc(const StreamDesc* p)
{
    static_assert(sizeof(StreamDesc) % 16 == 0, "descriptor size");
    u4v w[sizeof(StreamDesc) / 16];
    const GLB u4v* q = (const GLB u4v*)glb(p);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(StreamDesc) / 16); ++i) w[i] = q[i];
    StreamDesc d;
    __builtin_memcpy(&d, w, sizeof d);
    return d;
}

template <int DT> __device__ __forceinline__ float ld1(const void* X, size_t i);
template <> __device__ __forceinline__ float ld1<DT_F32>(const void* X, size_t i)
{
    return glb((const float*)X)[i];
}
template <> __device__ __forceinline__ float ld1<DT_F16>(const void* X, size_t i)
{
    return __half2float(__ushort_as_half(glb((const unsigned short*)X)[i]));
}
template <> __device__ __forceinline__ float ld1<DT_U16>(const void* X, size_t i)
{
    return (float)glb((const uint16_t*)X)[i] * (1.0f / 65536.0f);  // exact
}

// Four consecutive elements [i, i+4) of a line as FP32, with no branches.  With
// VEC (b % 4 == 0 and i % 4 == 0) one 8- or 16-byte load; otherwise element
// loads, where the caller passes ok[q] = false for elements that do not exist:
// their offset is clamped to 0 (in bounds) and the caller ignores the value.
// A load under a divergent branch, or a use right after it, makes the compiler
// wait for every load in flight, so callers mask the values where they use
// them, not here.
template <int DT, bool VEC>
__device__ __forceinline__ f4 ldq(const void* X, size_t i, int b_left)
{
    f4 v;
    if (VEC) {
        if (DT == DT_F32) {
            v = *(const GLB f4*)glb((const float*)X + i);
        } else if (DT == DT_F16) {
            const u2v uv = *(const GLB u2v*)glb((const __half*)X + i);
            const uint2 u = make_uint2(uv.x, uv.y);
            const float2 a = __half22float2(*(const __half2*)&u.x), c = __half22float2(*(const __half2*)&u.y);
            v = f4{a.x, a.y, c.x, c.y};
        } else {
            const u2v u = *(const GLB u2v*)glb((const uint16_t*)X + i);
            const float sc = 1.0f / 65536.0f;
            v = f4{(float)(u.x & 0xffffu) * sc, (float)(u.x >> 16) * sc, (float)(u.y & 0xffffu) * sc,
                   (float)(u.y >> 16) * sc};
        }
    } else {
        // b_left: elements of the row from i on (<= 0 when i itself is clamped)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = ld1<DT>(X, q < b_left ? i + q : 0);
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
    const GLB StreamDesc* sd = glb(P.sd);
    int lo = 0, hi = P.nstreams - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sd[mid].line0 <= line) lo = mid;
        else hi = mid - 1;
    }
    return load_desc(P.sd + lo);
}

// the stream owning pass scan segment `g`
__device__ __forceinline__ StreamDesc stream_of_seg(const Pass& P, int g)
{
    if (!P.sd) return P.one;
    const GLB StreamDesc* sd = glb(P.sd);
    int lo = 0, hi = P.nstreams - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sd[mid].seg0 <= g) lo = mid;
        else hi = mid - 1;
    }
    return load_desc(P.sd + lo);
}

// Weight of stream line tg (0-based, over the stream's life) in the moving average
// C_tg = (1 - a) C_{tg-1} + a S_tg: the momentum (Sec. III-C; the first line
// initialises, a = 1), or 1 / (tg + 1) for the equally weighted IMC background
// (the running mean of the per-line values).
__device__ __forceinline__ double avg_weight(const StreamDesc& d, long long tg)
{
    if (d.bg == BG_IMC) return 1.0 / (double)(tg + 1);
    return tg == 0 ? 1.0 : d.alpha;
}

__device__ __forceinline__ long long tile_u(int I, int J, int NT)  // upper tile I <= J
{
    return (long long)I * NT - (long long)I * (I - 1) / 2 + (J - I);
}

__device__ __forceinline__ int tile_lc(int J, int K, int NT)  // lower tile J >= K, column-major
{
    return K * NT - K * (K - 1) / 2 + (J - K);
}

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
// diag_s holds the block (row-major, stride 17) on entry and L on return; xt_s
// receives X = L^{-1} (row-major, stride 17).  Rows of L live in lanes 0..15 and are
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
    // L to LDS (rows in lanes 0..15; diag_s is no longer needed), read back
    // by every lane with broadcast loads: broadcasting the rows again from
    // registers would keep all 120 column values live in scalar registers
    if (lane < 16)
#pragma unroll
        for (int q = 0; q < 16; ++q) diag_s[r * 17 + q] = a[q];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // X = L^{-1}: lane c (= r) computes column c by forward substitution
    T x[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        T s0 = (q == r) ? (T)1 : (T)0, s1 = (T)0;
#pragma unroll
        for (int k = 0; k < q; ++k) {
            const T lqk = diag_s[q * 17 + k];
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

// Cholesky factor L of a 16x16 FP64 block A and its inverse X = L^{-1}, by one
// wave holding both in the state layout (lane (g, c), register i: row 4g+i,
// column c): four values per lane, so the factorisation costs the kernel few
// registers.  Right-looking: at step k the pivot comes from lane (k/4, k), the
// rows of column k from lane (g, k) of each lane's own row group (a DPP row
// broadcast), and entry
// (c, k) from lane (k/4, c) through the symmetry of the trailing block (both
// triangles are updated).  Row k of X is eliminated in the same step: it needs
// only column k of L and the rows of X above it, which are final by then.
// On entry a holds A (both triangles); on return a holds L (zero above the
// diagonal) and x holds X.  When rows and columns nb..15 of A are those of the
// identity (padded bands) the steps from nb on change nothing and are skipped.
// Returns 1 if a pivot was not positive (a NaN pivot propagates and is not
// counted).
// value of lane K of each row of 16 lanes (DPP row_newbcast), for an FP64 value
template <int K> __device__ __forceinline__ double row_bcast(double v)
{
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffll), 0x150 + K, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), 0x150 + K, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// BF: branch-free row updates (fewer instructions; more registers live, which
// spills in callers that already hold many tiles in registers)
template <int K, bool BF>
__device__ __forceinline__ void factor16_step(double (&a)[4], double (&x)[4], int g, int c, int& bad)
{
    constexpr int kg = K >> 2, ki = K & 3;
    double ar[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) ar[i] = row_bcast<K>(a[i]);  // A[4g+i][K]: lane K of the lane's row
    const double ac = __shfl(a[ki], 16 * kg + c);           // A[K][c] = A[c][K]
    const double akk = bcast(a[ki], 16 * kg + K);
    if (!(akk > 0.0) && !(akk != akk)) bad = 1;
    const double inv = rsqrt_nr(akk);
    double lr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = 4 * g + i;
        lr[i] = r > K ? ar[i] * inv : (r == K ? akk * inv : 0.0);  // L[r][K]
    }
    const double lc = c > K ? ac * inv : 0.0;                      // L[c][K] below the pivot
    if (BF) {
        x[ki] = (g == kg) ? x[ki] * inv : x[ki];                   // row K of X is final
        const double xk = __shfl(x[ki], 16 * kg + c);              // X[K][c]
        // lr is zero above row K and lc zero up to column K, so the rank-one
        // update changes only the trailing block and row K of the columns right
        // of K; those entries are above the diagonal and are overwritten with
        // the column of L at their own step.
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 4 * g + i;
            a[i] = (c == K) ? lr[i] : a[i] - lr[i] * lc;
            x[i] -= (r > K ? lr[i] : 0.0) * xk;
        }
    } else {
        if (g == kg) x[ki] *= inv;
        const double xk = __shfl(x[ki], 16 * kg + c);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 4 * g + i;
            if (c == K) a[i] = lr[i];
            else if (r > K && c > K) a[i] -= lr[i] * lc;
            if (r > K) x[i] -= lr[i] * xk;
        }
    }
}

template <bool BF, int... Ks>
__device__ __forceinline__ void factor16_steps(std::integer_sequence<int, Ks...>, double (&a)[4], double (&x)[4],
                                               int g, int c, int nb, int& bad)
{
    // rows and columns from nb on are the identity and stay so
    ((Ks < nb ? factor16_step<Ks, BF>(a, x, g, c, bad) : void()), ...);
}

template <bool BF = true>
__device__ __forceinline__ int factor16(double (&a)[4], double (&x)[4], int lane, int nb = 16)
{
    const int g = lane >> 4, c = lane & 15;
    int bad = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = (4 * g + i == c) ? 1.0 : 0.0;
    factor16_steps<BF>(std::make_integer_sequence<int, 16>(), a, x, g, c, nb, bad);
    return bad;
}


// The FP64 instantiation with the contract of factor_diag16 above (the block's
// lower triangle in diag_s, L back in diag_s with zeros above the diagonal,
// X = L^{-1} in xt_s), computed by the register-lean factor16 on the block
// mirrored from its lower triangle.  The lane index is re-derived from a value
// the compiler cannot see through, so that the lane masks of the sixteen
// steps are not hoisted out of a caller's loop (where they would stay live).
template <>
__device__ __forceinline__ int factor_diag16<double>(double* diag_s, double* xt_s, int lane)
{
    int ln = lane;
    __asm__ volatile("" : "+v"(ln));
    const int g = ln >> 4, c = ln & 15;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double a[4], x[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = 4 * g + i;
        a[i] = r >= c ? diag_s[r * 17 + c] : diag_s[c * 17 + r];
    }
    const int bad = factor16<false>(a, x, ln);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        diag_s[(4 * g + i) * 17 + c] = a[i];
        xt_s[(4 * g + i) * 17 + c] = x[i];
    }
    return bad;
}

}  // namespace erx
