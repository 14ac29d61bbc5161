// Leaf of the block-LU inversion, the method the paper compares SPIN with
// (Sec. 5, after Liu et al.): A = L U without pivoting, then L^-1 and U^-1.
// The block recursion around it (spin_api.cpp) uses the product kernels.
#include <hip/hip_runtime.h>

#include <cfloat>

#include "spin_kernels.hpp"

namespace spin {
namespace {

constexpr int kLuLd = kLuLeafMax + 1;  // LDS column pitch

// One workgroup inverts the factors of an order-L block (L <= kLuLeafMax)
// held in LDS:
//   1. Doolittle LU without pivoting: multipliers below the diagonal, U on
//      and above it; a zero or non-finite pivot is reported at its column;
//   2. U^-1 and L^-1 in place, one column of each per step: column j of U^-1
//      is -U^-1[0:j, 0:j] U[0:j, j] / u_jj, with j ascending, and column j of
//      L^-1 is -L^-1[j+1:, j+1:] L[j+1:, j], with j descending.  Each uses only
//      blocks inverted in earlier steps, the two live in disjoint triangles,
//      and a step reads its columns before a barrier and writes them after;
//   3. L^-1 (unit lower) and U^-1 (upper) stored as full blocks with zeros in
//      the other triangle.
__global__ void __launch_bounds__(256)
    k_lu_leaf_inv(const double *__restrict__ A, int64_t lda, double *__restrict__ Li, int64_t ldl,
                  double *__restrict__ Ui, int64_t ldu, int L, int col0, int *status) {
    __shared__ double F[kLuLeafMax * kLuLd];
    const int t = threadIdx.x;
    for (int idx = t; idx < L * L; idx += 256) {
        const int i = idx % L, j = idx / L;
        F[i + j * kLuLd] = A[i + (int64_t)j * lda];
    }
    __syncthreads();
    int bad = 0;
    for (int k = 0; k < L; ++k) {
        const double piv = F[k + k * kLuLd];
        if (bad == 0 && !(piv != 0.0 && fabs(piv) <= DBL_MAX)) bad = k + 1;
        for (int i = k + 1 + t; i < L; i += 256) F[i + k * kLuLd] = F[i + k * kLuLd] / piv;
        __syncthreads();
        const int r = L - k - 1;
        for (int idx = t; idx < r * r; idx += 256) {
            const int i = k + 1 + idx % r, j = k + 1 + idx / r;
            F[i + j * kLuLd] = F[i + j * kLuLd] - F[i + k * kLuLd] * F[k + j * kLuLd];
        }
        __syncthreads();
    }
    // threads 0..127 work on U (rows i < ju), threads 128..255 on L (rows i > jl)
    const int half = t >> 7, i = t & 127;
    for (int s = 0; s < L; ++s) {
        const int ju = s, jl = L - 1 - s;
        double v = 0.0;
        if (half == 0 && i < ju) {
            for (int k = i; k < ju; ++k) v += F[i + k * kLuLd] * F[k + ju * kLuLd];
        } else if (half == 1 && i > jl && i < L) {
            v = F[i + jl * kLuLd];
            for (int k = jl + 1; k < i; ++k) v += F[i + k * kLuLd] * F[k + jl * kLuLd];
        }
        const double ujj = F[ju + ju * kLuLd];
        __syncthreads();
        if (half == 0 && i < ju) F[i + ju * kLuLd] = -v / ujj;
        if (half == 0 && i == ju) F[ju + ju * kLuLd] = 1.0 / ujj;
        if (half == 1 && i > jl && i < L) F[i + jl * kLuLd] = -v;
        __syncthreads();
    }
    for (int idx = t; idx < L * L; idx += 256) {
        const int r = idx % L, c = idx / L;
        const double f = F[r + c * kLuLd];
        Li[r + (int64_t)c * ldl] = r > c ? f : (r == c ? 1.0 : 0.0);
        Ui[r + (int64_t)c * ldu] = r <= c ? f : 0.0;
    }
    if (t == 0 && bad) atomicMin(status, col0 + bad);
}

}  // namespace

hipError_t lu_leaf_launch(const double *A, int64_t lda, double *Li, int64_t ldl, double *Ui,
                          int64_t ldu, int64_t L, int64_t col0, int *status, hipStream_t s) {
    if (L < 1 || L > kLuLeafMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lu_leaf_inv, dim3(1), dim3(256), 0, s, A, lda, Li, ldl, Ui, ldu, (int)L,
                       (int)col0, status);
    return hipGetLastError();
}

}  // namespace spin
