// Sparse random projection front end of ERX (Sec. III-B): the weight matrix
// W in R^{b x d} drawn at creation, and the projection Z_t = X_t W of every
// pushed line, after which the detector runs on Z_t in d dimensions.
//
// Weights: w_ij = sqrt(s/d) * (+1 with probability 1/(2s), 0 with 1 - 1/s,
// -1 with 1/(2s)), s = sqrt(b).  The draws come from SplitMix64 used as a
// counter-based generator: weight (i, j) takes output number k = i d + j + 1
// of the generator started from the seed, as the uniform (u >> 11) 2^-53.
//
// Projection, relative to a reference pixel x_ref (the first one the detector
// sees): z - W^T x_ref = W^T (x - x_ref).  Shifting every pixel alike leaves
// the moving covariance and every score unchanged, and the FP32 result then
// carries the pixel's deviation from the background rather than its full
// value, so its rounding stays small against the residuals that are scored.
// A workgroup of 256 threads takes 32 pixels; their rows
// (32 b contiguous values) are copied into LDS with coalesced loads, and eight
// threads per pixel each take every eighth band (W read through the caches)
// and reduce their d partial sums over the eight.  The kernel reads each line
// once; it is bound by that read.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/erx.h"
#include "erx_device.h"
#include "erx_runtime.h"

namespace erx {
namespace {

uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr int SRP_PIX = 32;  // pixels per workgroup; 8 threads per pixel

template <int DT, int DMAX>
__global__ __launch_bounds__(256) void k_srp_project(const void* __restrict__ X, long long npix, int b,
                                                     const float* __restrict__ W, const float* __restrict__ xref,
                                                     int d, float* __restrict__ Z)
{
    extern __shared__ float xs[];  // [SRP_PIX][b]
    const long long p0 = (long long)blockIdx.x * SRP_PIX;
    const int np = (int)((npix - p0) < SRP_PIX ? (npix - p0) : SRP_PIX);
    const int tid = threadIdx.x;
    const long long e0 = p0 * b;
    const int ne = np * b;
    for (int i = tid; i < ne; i += 256) xs[i] = ld1<DT>(X, (size_t)(e0 + i)) - glb(xref)[i % b];
    __syncthreads();
    const int px = tid >> 3, q = tid & 7;
    float z[DMAX];
#pragma unroll
    for (int j = 0; j < DMAX; ++j) z[j] = 0.f;
    if (px < np) {
        const float* xr = xs + px * b;
        for (int i = q; i < b; i += 8) {
            const float v = xr[i];
            const GLB float* wr = glb(W) + (size_t)i * d;  // W (at most 39 KB) stays in the caches
#pragma unroll
            for (int j = 0; j < DMAX; ++j)
                if (j < d) z[j] = fmaf(v, wr[j], z[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < DMAX; ++j) {
        z[j] += __shfl_xor(z[j], 1);
        z[j] += __shfl_xor(z[j], 2);
        z[j] += __shfl_xor(z[j], 4);
    }
    if (px < np && q == 0) {
        float* zo = Z + (p0 + px) * d;
#pragma unroll
        for (int j = 0; j < DMAX; ++j)
            if (j < d) zo[j] = z[j];
    }
}

template <int DMAX>
void srp_launch(int dtype, dim3 grid, size_t lds, hipStream_t s, const void* X, long long npix, int b, const float* W,
                const float* xr, int d, float* Z)
{
    switch (dtype) {
    case DT_F32:
        hipLaunchKernelGGL((k_srp_project<DT_F32, DMAX>), grid, dim3(256), lds, s, X, npix, b, W, xr, d, Z);
        break;
    case DT_F16:
        hipLaunchKernelGGL((k_srp_project<DT_F16, DMAX>), grid, dim3(256), lds, s, X, npix, b, W, xr, d, Z);
        break;
    default: hipLaunchKernelGGL((k_srp_project<DT_U16, DMAX>), grid, dim3(256), lds, s, X, npix, b, W, xr, d, Z); break;
    }
}

template <int DT> __global__ void k_srp_ref(const void* __restrict__ X, int b, float* __restrict__ xref)
{
    for (int i = threadIdx.x; i < b; i += blockDim.x) xref[i] = ld1<DT>(X, (size_t)i);
}

}  // namespace

hipError_t launch_srp_ref(int dtype, const void* X, int b, float* xref, hipStream_t s)
{
    switch (dtype) {
    case DT_F32: hipLaunchKernelGGL(k_srp_ref<DT_F32>, dim3(1), dim3(256), 0, s, X, b, xref); break;
    case DT_F16: hipLaunchKernelGGL(k_srp_ref<DT_F16>, dim3(1), dim3(256), 0, s, X, b, xref); break;
    default: hipLaunchKernelGGL(k_srp_ref<DT_U16>, dim3(1), dim3(256), 0, s, X, b, xref); break;
    }
    return hipGetLastError();
}

hipError_t launch_srp_project(int dtype, const void* X, long long npix, int b, const float* W, const float* xref,
                              int d, float* Z, hipStream_t s)
{
    if (npix <= 0) return hipSuccess;
    if (d < 1 || d > ERX_SRP_MAX_DIMS) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((npix + SRP_PIX - 1) / SRP_PIX));
    const size_t lds = (size_t)SRP_PIX * b * sizeof(float);
    if (d <= 8) srp_launch<8>(dtype, grid, lds, s, X, npix, b, W, xref, d, Z);
    else if (d <= 16) srp_launch<16>(dtype, grid, lds, s, X, npix, b, W, xref, d, Z);
    else srp_launch<32>(dtype, grid, lds, s, X, npix, b, W, xref, d, Z);
    return hipGetLastError();
}

}  // namespace erx

using namespace erx;

extern "C" int erx_srp_matrix(int bands, int dims, unsigned long long seed, float* W)
{
    if (bands < 1 || bands > ERX_MAX_BANDS || dims < 1 || dims > ERX_SRP_MAX_DIMS || !W)
        return set_error(ERX_EINVAL, "erx_srp_matrix: bands in [1, %d], dims in [1, %d] and W are required",
                         ERX_MAX_BANDS, ERX_SRP_MAX_DIMS);
    const double s = std::sqrt((double)bands);
    const float scale = (float)std::sqrt(s / (double)dims);
    const double p_half = 1.0 / (2.0 * s);
    for (int i = 0; i < bands; ++i)
        for (int j = 0; j < dims; ++j) {
            const double u = (double)(splitmix64_at(seed, (uint64_t)i * dims + j + 1) >> 11) * 0x1.0p-53;
            W[(size_t)i * dims + j] = u < p_half ? scale : (u < 2.0 * p_half ? -scale : 0.0f);
        }
    return ERX_OK;
}
