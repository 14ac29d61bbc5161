// Auxiliary bandwidth-bound kernels: status reset, precision conversion,
// copies, transposes and deterministic Frobenius-norm reductions.
#include <hip/hip_runtime.h>

#include <climits>

#include "spin_kernels.hpp"

namespace spin {
namespace {

constexpr int kNormBlocks = 1024;

__global__ void k_status_reset(int *status, int spec) {
    const int i = threadIdx.x;
    if (i < kStatusWords) status[i] = (i == kStatusSpecWord && !spec) ? 0 : INT_MAX;
}

__global__ void k_status_copy(const int *status, int *info) {
    if (threadIdx.x == 0) info[0] = status[0] == INT_MAX ? 0 : status[0];
}

// 2-D grid-stride conversion of an (m x n) column-major view.
template <typename S, typename D>
__global__ void __launch_bounds__(256)
    k_convert(const S *__restrict__ src, int64_t lds, D *__restrict__ dst, int64_t ldd, int64_t m,
              int64_t n) {
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m;
             i += (int64_t)gridDim.x * 256)
            dst[i + j * ldd] = (D)src[i + j * lds];
}

// dst (n x m, ldd) = src (m x n, lds)^T.  A workgroup moves one 64 x 64 tile
// through LDS: it reads down the source columns and writes down the
// destination columns, so both sides coalesce.  The row pitch of 65 doubles
// spreads the transposed LDS reads over the banks.
constexpr int kTT = 64;
__global__ void __launch_bounds__(256)
    k_transpose(const double *__restrict__ src, int64_t lds, double *__restrict__ dst, int64_t ldd,
                int64_t m, int64_t n) {
    __shared__ double tile[kTT][kTT + 1];
    const int64_t i0 = (int64_t)blockIdx.x * kTT, j0 = (int64_t)blockIdx.y * kTT;
    const int tx = threadIdx.x & (kTT - 1), ty = threadIdx.x / kTT;
    for (int jj = ty; jj < kTT; jj += 256 / kTT) {
        const int64_t i = i0 + tx, j = j0 + jj;
        if (i < m && j < n) tile[jj][tx] = src[i + j * lds];
    }
    __syncthreads();
    for (int ii = ty; ii < kTT; ii += 256 / kTT) {
        const int64_t r = j0 + tx, c = i0 + ii;  // dst row = src column
        if (r < n && c < m) dst[r + c * ldd] = tile[tx][ii];
    }
}

// Lower triangle of an order-n view mirrored onto the upper one, in place:
// d[i][j] = d[j][i] for j > i.  Workgroup t takes lower tile (r, c), r >= c
// (row by row over the T (T + 1) / 2 of them), reads it whole into LDS and
// writes its transpose into upper tile (c, r); a diagonal tile writes only its
// own strict upper part.  Each tile is read by one workgroup, and no tile
// that is written is read by another, so the update needs no ordering.
__global__ void __launch_bounds__(256) k_mirror_lower(double *__restrict__ d, int64_t ld, int64_t n) {
    __shared__ double tile[kTT][kTT + 1];
    const int t = blockIdx.x;
    int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while (r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    const int c = t - r * (r + 1) / 2;
    const int64_t i0 = (int64_t)r * kTT, j0 = (int64_t)c * kTT;  // source rows i0.., columns j0..
    const int tx = threadIdx.x & (kTT - 1), ty = threadIdx.x / kTT;
    for (int jj = ty; jj < kTT; jj += 256 / kTT) {
        const int64_t i = i0 + tx, j = j0 + jj;
        if (i < n && j < n) tile[jj][tx] = d[i + j * ld];
    }
    __syncthreads();
    for (int ii = ty; ii < kTT; ii += 256 / kTT) {
        const int64_t row = j0 + tx, col = i0 + ii;  // destination (row, col) = source (col, row)
        if (row < n && col < n && col > row) d[row + col * ld] = tile[tx][ii];
    }
}

// 2-D grid-stride zero fill of an (m x n) column-major view.
__global__ void __launch_bounds__(256) k_fill_zero(double *__restrict__ d, int64_t ld, int64_t m, int64_t n) {
    for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256)
            d[i + j * ld] = 0.0;
}

// Per-block partial sums of squares over whole columns (fixed assignment of
// columns to blocks and fixed in-block order: the result does not depend on
// scheduling).
__global__ void __launch_bounds__(256)
    k_frob_partial(const double *__restrict__ src, int64_t ld, int64_t m, int64_t n,
                   double *__restrict__ partials) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t j = blockIdx.x; j < n; j += gridDim.x)
        for (int64_t i = threadIdx.x; i < m; i += 256) {
            const double v = src[i + j * ld];
            s = fma(v, v, s);
        }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_frob_final(const double *__restrict__ partials, int np,
                                                      double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) s += partials[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Refinement monitor: flags divergence when |R_j|_F did not decrease.
__global__ void k_ns_check(const double *norms, int j, int *status) {
    if (threadIdx.x == 0 && j > 0 && !(norms[j] < norms[j - 1])) status[0] = kStatusNsDiverged;
}

// Acceptance of a refined inverse: flags divergence unless
// rho = |R|_F / (|A|_F |X|_F) <= tol (a NaN anywhere fails the test).
__global__ void k_ns_final(const double *r2, const double *a2, const double *x2, double tol,
                           int *status) {
    if (threadIdx.x == 0) {
        const double rho = sqrt(*r2) / (sqrt(*a2) * sqrt(*x2));
        if (!(rho <= tol)) status[0] = kStatusNsDiverged;
    }
}

template <typename S, typename D>
hipError_t convert(const S *src, int64_t lds, D *dst, int64_t ldd, int64_t m, int64_t n,
                   hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    const int64_t bx = (m + 255) / 256;
    dim3 grid((unsigned)(bx < 64 ? bx : 64), (unsigned)(n < 4096 ? n : 4096));
    hipLaunchKernelGGL((k_convert<S, D>), grid, dim3(256), 0, s, src, lds, dst, ldd, m, n);
    return hipGetLastError();
}

}  // namespace

hipError_t status_reset(int *status, bool spec, hipStream_t s) {
    hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, s, status, spec ? 1 : 0);
    return hipGetLastError();
}

hipError_t status_copy(const int *status, int *info, hipStream_t s) {
    hipLaunchKernelGGL(k_status_copy, dim3(1), dim3(64), 0, s, status, info);
    return hipGetLastError();
}

hipError_t cast_f64_to_f32(const double *src, int64_t lds, float *dst, int64_t ldd, int64_t m,
                           int64_t n, hipStream_t s) {
    return convert<double, float>(src, lds, dst, ldd, m, n, s);
}

hipError_t cast_f32_to_f64(const float *src, int64_t lds, double *dst, int64_t ldd, int64_t m,
                           int64_t n, hipStream_t s) {
    return convert<float, double>(src, lds, dst, ldd, m, n, s);
}

hipError_t copy_f64(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t m,
                    int64_t n, hipStream_t s) {
    return convert<double, double>(src, lds, dst, ldd, m, n, s);
}

hipError_t fill_zero_f64(double *d, int64_t ld, int64_t m, int64_t n, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    const int64_t bx = (m + 255) / 256;
    dim3 grid((unsigned)(bx < 64 ? bx : 64), (unsigned)(n < 4096 ? n : 4096));
    hipLaunchKernelGGL(k_fill_zero, grid, dim3(256), 0, s, d, ld, m, n);
    return hipGetLastError();
}

hipError_t mirror_lower_f64(double *d, int64_t ld, int64_t n, hipStream_t s) {
    if (n <= 1) return hipSuccess;
    const int64_t T = (n + kTT - 1) / kTT, blocks = T * (T + 1) / 2;
    if (blocks > INT_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mirror_lower, dim3((unsigned)blocks), dim3(256), 0, s, d, ld, n);
    return hipGetLastError();
}

hipError_t transpose_f64(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t m,
                         int64_t n, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    const int64_t gx = (m + kTT - 1) / kTT, gy = (n + kTT - 1) / kTT;
    if (gx > INT_MAX || gy > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, src, lds, dst,
                       ldd, m, n);
    return hipGetLastError();
}

hipError_t ns_check(const double *norms, int j, int *status, hipStream_t s) {
    hipLaunchKernelGGL(k_ns_check, dim3(1), dim3(64), 0, s, norms, j, status);
    return hipGetLastError();
}

hipError_t ns_final(const double *r2, const double *a2, const double *x2, double tol, int *status,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_ns_final, dim3(1), dim3(64), 0, s, r2, a2, x2, tol, status);
    return hipGetLastError();
}

int frob_partials_count(int64_t m, int64_t n) {
    (void)m;
    return (int)(n < kNormBlocks ? (n > 0 ? n : 1) : kNormBlocks);
}

hipError_t frob2(const double *src, int64_t ld, int64_t m, int64_t n, double *partials,
                 double *out, hipStream_t s) {
    const int np = frob_partials_count(m, n);
    hipLaunchKernelGGL(k_frob_partial, dim3(np), dim3(256), 0, s, src, ld, m, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_frob_final, dim3(1), dim3(256), 0, s, partials, np, out);
    return hipGetLastError();
}

}  // namespace spin
