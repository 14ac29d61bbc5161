// Recursion planner shared by the single-call executor (spin_api.cpp) and
// the batching server (spin_server.cpp).  Not installed.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

#include "spin.h"
#include "spin_kernels.hpp"

namespace spin {

enum Buf { BUF_A = 0, BUF_X = 1, BUF_WS = 2 };

// A view: buffer id, element offset and leading dimension.
struct Ref {
    int buf;
    int64_t off;
    int64_t ld;
};

// One block product of the schedule: D = alpha A B + beta C (+ I).  With
// lower set (m == n) only the tiles on or below the diagonal are computed.
struct PGemm {
    Ref a, b, c, d;
    int64_t m, n, k;
    double alpha, beta;
    int add_identity;
    int lower;
};

// One step: a group of independent products (kind 0), a leaf (kind 1), a
// transpose (kind 2: out (tn x tm) := in (tm x tn)^T), a mirror (kind 3:
// the lower triangle of the order-tm block `out` copied onto its upper one),
// an LU leaf (kind 4: out := L^-1 and out2 := U^-1 of the order-L block in)
// or a zero fill (kind 5: the tm x tn block out).
struct POp {
    int kind;
    int count;
    int level;
    PGemm g[2];
    Ref in, out, out2;
    int64_t L, col0;
    int64_t tm, tn;
};

struct Plan {
    int64_t n = 0, lda = 0, ldx = 0, leaf = 0;
    std::vector<POp> ops;
    int64_t ws_elems = 0;
    int64_t max_leaf = 0;
    double flops = 0;
};

// Layout of one inversion's workspace (bytes):
//   [0, 256)          status words (int): 0 = pivot status, 1 = refinement status
//   [256, 4096)       small doubles: 0..7 refinement norms, 8..15 misc norms
//   [4096, +8 KiB)    Frobenius-norm partials
//   then              recursion workspace, leaf scratch, mixed-mode buffers
constexpr size_t kHdr = 4096 + 8192 + 4096;
constexpr int kNormSlots = 8;

// Precision modes of the C ABI.
inline bool is_mixed_mode(int mode) {
    return mode == SPIN_MIXED_FP32 || mode == SPIN_MIXED_BF16 || mode == SPIN_MIXED_BF16X3;
}
inline bool is_mode(int mode) { return mode == SPIN_FP64 || is_mixed_mode(mode); }
// Product flavour of the block products of a mode (operands stay FP32 in
// every mixed mode; leaves, residual and refinement stay FP64).
inline DType mixed_product_type(int mode) {
    return mode == SPIN_MIXED_BF16 ? kBF16 : mode == SPIN_MIXED_BF16X3 ? kBF16X3 : kF32;
}

struct Layout {
    size_t rec_off, rec_bytes;
    size_t leaf_off, leaf_bytes;
    size_t a32_off, x32_off, r_off, xalt_off;
    size_t total;
};
Layout layout_for(int64_t n, int64_t leaf, int mode, int64_t ws_elems, int64_t max_leaf);

// The kernel-level product of a scheduled one, for buffers A, X and the
// workspace at base[0..2] with element size es.
GemmProb make_prob(char *const base[3], size_t es, const PGemm &g);

// Whether the step after product step ops[i] can be done by that product's
// epilogue with the same result bit for bit: 3 for the mirror of a lower-half
// product's result, 2 for the transpose of a product's result into a block
// that none of its operands occupies (single-product steps), else 0.
int fold_kind(const Plan &P, size_t i);
// Whether every mirror and transpose of P is taken over by the product before
// it (required for plans on FP32 storage).
bool plan_folds_all(const Plan &P);
// Applies fold_kind to the kernel-level product pr[0] of a plan with element
// size es (8: FP64, 4: FP32 storage): sets pr[0].DT / lddt and returns true
// when ops[i + 1] is taken over.
bool fold_next_step(const Plan &P, size_t i, char *const base[3], size_t es, GemmProb pr[2]);

// Whether leaves try the speculative elimination first (environment
// variable SPIN_NO_SPEC unset or 0).
bool leaf_spec_enabled();

// Bytes of workspace the FP64 schedule of an order-n inversion needs, and
// that inversion on a caller-provided workspace: launched eagerly on s (no
// graph, no trace, no allocation); its numerical status (0 or the 1-based
// failing pivot column) is copied to the device int *info when info is set.
size_t invert_workspace_bytes(int64_t n, int64_t leaf);
int invert_on_workspace(const double *A, int64_t n, int64_t lda, double *Ainv, int64_t ldx,
                        int64_t leaf, char *ws, size_t ws_bytes, int *info, hipStream_t s);

// Order of the leading block when an order-m block is split.
int64_t split_order(int64_t m);
// Depth-first S-form schedule of Alg. 1 for an order-n matrix.
Plan make_plan(int64_t n, int64_t lda, int64_t ldx, int64_t leaf);
// The same for a symmetric matrix: four products and one transpose per node.
Plan make_plan_spd(int64_t n, int64_t lda, int64_t ldx, int64_t leaf);
// Inversion through a block LU factorisation (the comparison method).
Plan make_plan_lu(int64_t n, int64_t lda, int64_t ldx, int64_t leaf);

}  // namespace spin
