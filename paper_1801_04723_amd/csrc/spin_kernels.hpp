// Internal interface between the host scheduler (spin_api.cpp) and the HIP
// kernels (gemm.hip, leaf.hip, aux.hip).  Not installed; the public ABI is
// include/spin.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace spin {

inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// Element types.  kBF16 and kBF16X3 are product flavours on FP32 storage:
// the operands are rounded to BF16 (X3: split into two BF16 terms) on their
// way into the matrix cores, and accumulation and results stay FP32.
enum DType : int32_t { kF64 = 0, kF32 = 1, kBF16 = 2, kBF16X3 = 3 };

// Storage type of a product flavour.
inline DType storage_type(DType d) { return d == kF64 ? kF64 : kF32; }

// Largest leaf order the leaf kernels accept.
constexpr int kLeafMaxOrder = 2048;

// One block product  D = alpha * A * B + beta * C0 (+ I),  column-major views.
// lower != 0 with m == n: only the tiles on or below the diagonal are
// computed and only the elements on or below the diagonal are stored (a
// symmetric result whose strict upper part a mirror fills).
// DT != nullptr: every stored element (i, j) is also stored at DT[j + i lddt]
// (the result transposed, n x m); for a lower problem only the elements below
// the diagonal are, so DT == D, lddt == ldd is the mirror.  DT must not
// overlap A, B or C0 (except where DT == D == C0 in the mirror form).
// 112 bytes: a group of kMaxBatch products stays within the 4 KiB of kernel
// arguments.
struct GemmProb {
    const void *A;
    const void *B;
    const void *C0;
    void *D;
    int64_t lda, ldb, ldc, ldd;
    int32_t m, n, k;
    int32_t add_identity;
    double alpha, beta;
    int32_t lower;
    int32_t lddt;
    void *DT;
};
static_assert(sizeof(GemmProb) == 112, "GemmProb layout");

// One gemm_launch() call takes up to kMaxBatch independent products; products
// that share a kernel configuration run in one grid (every workgroup finds
// its problem from the tile prefix sums).
constexpr int kMaxBatch = 32;

// Per-launch bookkeeping returned to the scheduler for tracing.
struct LaunchInfo {
    const char *name;  // kernel family + tile shape (static string)
    double flops;
    double bytes;
};

// GEMM family (gemm.hip).  dt selects operand/result type and MFMA flavour.
// The kernel configuration of each product depends only on that product, so
// grouping products from different requests does not change any result bit.
hipError_t gemm_launch(const GemmProb *probs, int count, DType dt, hipStream_t s,
                       LaunchInfo *info);

// Leaf inversion, Gauss-Jordan with partial pivoting in FP64 (leaf.hip).
//   in  : order-L block, element type `in_dt`, leading dimension ldi
//   out : order-L block, element type `out_dt`, leading dimension ldo
//   status : device int, atomically lowered to col0 + k + 1 on a failing pivot
//   scratch: FP64 scratch for the blocked tier (leaf_scratch_bytes(L) bytes);
//            it starts with the exchange areas of the two-workgroup panels
//   exch_filled: those areas already hold their fill pattern, because the
//            last leaf_launch on this scratch, earlier on the same stream, was
//            for an order with leaf_fills_exchange() true and no other leaf or
//            kernel has written the scratch since; otherwise (always safe)
//            a leaf that needs them fills them first
size_t leaf_scratch_bytes(int64_t L);
hipError_t leaf_launch(const void *in, DType in_dt, int64_t ldi, void *out, DType out_dt,
                       int64_t ldo, int64_t L, int64_t col0, int *status, void *scratch,
                       bool exch_filled, hipStream_t s,
                       void (*trace_cb)(void *, const LaunchInfo &, int), void *trace_ctx);
// True when leaf_launch() for order L leaves the exchange areas filled at its
// end.  Leaves of other orders leave them as they found them.
bool leaf_fills_exchange(int64_t L);

// Whole leaves of order <= 128 from independent requests, one workgroup each,
// in one launch (per leaf size class); each leaf's result is identical to the
// one leaf_launch() produces for it.
struct LeafItem {
    const void *in;
    int64_t ldi;
    void *out;
    int64_t ldo;
    int64_t L, col0;
    int *status;
};
constexpr int kMaxLeafBatch = 32;
struct LeafBatch {
    LeafItem item[kMaxLeafBatch];
    int32_t count;
};
hipError_t leaf_batch_launch(const LeafItem *items, int count, DType dt, hipStream_t s,
                             LaunchInfo *info);

// Auxiliary kernels (aux.hip).
// Status words of an inversion: word 0 the pivot status and word 1 the
// refinement status start at INT_MAX ("no event") and are lowered
// atomically; word kStatusSpecWord is the leaves' speculation switch
// (nonzero: try the speculative elimination first).
constexpr int kStatusWords = 3;
constexpr int kStatusSpecWord = 2;
hipError_t status_reset(int *status, bool spec, hipStream_t s);
// *info = the pivot status word (0 when it holds "no event"), by a kernel.
hipError_t status_copy(const int *status, int *info, hipStream_t s);
// Value written to the refinement status word on divergence (SPIN_NS_DIVERGED).
constexpr int kStatusNsDiverged = -100;
hipError_t ns_check(const double *norms, int j, int *status, hipStream_t s);
// Residual bound a refined inverse must meet: rho = |A X - I|_F / (|A|_F
// |X|_F) <= kNsTol after the refinement steps, else the refinement status
// word gets SPIN_NS_DIVERGED.
constexpr double kNsTol = 1e-12;
// Moduli of the refinement's INT8-emulated products (SPIN_REFINE_INT8): 14
// give about 110 bits of modulus, operands of 47 bits at order 16384.
constexpr int kRefineModuli = 14;
// Longest inner dimension of an INT8-emulated product: the matrix cores sum
// k products of symmetric residues (|r| <= 128) in int32, exact while
// k 128^2 < 2^31.
constexpr int64_t kOzakiMaxK = 131071;
hipError_t ns_final(const double *r2, const double *a2, const double *x2, double tol, int *status,
                    hipStream_t s);
hipError_t cast_f64_to_f32(const double *src, int64_t lds, float *dst, int64_t ldd, int64_t m,
                           int64_t n, hipStream_t s);
hipError_t cast_f32_to_f64(const float *src, int64_t lds, double *dst, int64_t ldd, int64_t m,
                           int64_t n, hipStream_t s);
hipError_t copy_f64(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t m,
                    int64_t n, hipStream_t s);
// dst (n x m, ldd) = src (m x n, lds)^T; the views must not overlap.
hipError_t transpose_f64(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t m,
                         int64_t n, hipStream_t s);
// In place on an order-n view: d[i][j] = d[j][i] for j > i.
hipError_t mirror_lower_f64(double *d, int64_t ld, int64_t n, hipStream_t s);
// d (m x n, ld) = 0, by a kernel (so that it can be captured in a graph).
hipError_t fill_zero_f64(double *d, int64_t ld, int64_t m, int64_t n, hipStream_t s);

// Leaf of the block-LU inversion (lu.hip): for an order-L block (L <=
// kLuLeafMax) A = L U without pivoting; Li = L^-1 and Ui = U^-1 written as
// full blocks.  A zero or non-finite pivot lowers *status to col0 + k + 1.
constexpr int kLuLeafMax = 128;
hipError_t lu_leaf_launch(const double *A, int64_t lda, double *Li, int64_t ldl, double *Ui,
                          int64_t ldu, int64_t L, int64_t col0, int *status, hipStream_t s);
// FP64-accurate product on INT8 matrix cores (ozaki.hip): D = epilogue(A B)
// with A (m x k, lda), B (k x n, ldb) column-major FP64; epilogue 0: D = A B,
// 1: D = I - A B (m == n), 2: D = C0 + A B.  `moduli` residue products
// (2 .. kOzakiMaxModuli); the operands are rounded to integers of at most
// beta_a / beta_b bits per row / column, which must satisfy
// 2 k 2^(beta_a + beta_b) < the product of the moduli (ozaki_beta gives the
// largest equal pair).  ws: ozaki_workspace_bytes(m, n, k, moduli) bytes.
constexpr int kOzakiMaxModuli = 15;
struct OzakiProb {
    const double *A;
    int64_t lda;
    const double *B;
    int64_t ldb;
    const double *C0;
    int64_t ldc;
    double *D;
    int64_t ldd;
    int64_t m, n, k;
    int epilogue;
    int moduli;
    int beta_a, beta_b;
};
double ozaki_log2_modulus(int count);
int ozaki_beta(int count, int64_t k);
size_t ozaki_workspace_bytes(int64_t m, int64_t n, int64_t k, int count);
hipError_t ozaki_product(const OzakiProb &p, void *ws, hipStream_t s);

// Sum of squares of an (m x n) FP64 view, deterministic two-pass reduction:
// partials (>= frob_partials_count(m, n) doubles) then one block writes *out.
int frob_partials_count(int64_t m, int64_t n);
hipError_t frob2(const double *src, int64_t ld, int64_t m, int64_t n, double *partials,
                 double *out, hipStream_t s);

}  // namespace spin
