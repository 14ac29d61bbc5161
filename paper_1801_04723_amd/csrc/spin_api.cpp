// Host side of the library: recursion planner, executor, per-stream
// workspace, graph cache, tracing and the exported C ABI (include/spin.h).
//
// The planner turns Strassen's inversion scheme (Alg. 1, Sec. 3.1; recursive
// form Alg. 2, Sec. 3.3) into a flat depth-first list of steps.  The paper's
// primitives map as follows:
//   breakMat / xy / arrange (Algs. 3, 4, 6) -> pointer offsets into
//       column-major storage (no data movement);
//   multiply + subtract + scalarMul (Alg. 2, Alg. 5) -> block products with a
//       fused epilogue, S-form: the Schur complement S = A22 - A21 A11^-1 A12
//       (= -V) is formed directly and inverted into C22, so C22 = S^-1 = -VI,
//       C12 = -III C22 = III VI and C21 = -C22 II = VI II;
//   locInverse (Alg. 2, leaf case) -> the leaf Gauss-Jordan kernels.
// Every internal node issues four launches: {II, III} grouped, S, {C12, C21}
// grouped, and C11 = C11 - III C21 in place.  The schedule for symmetric
// matrices (spin_invert_spd) lists II, S with its mirror, C21, the transpose
// C12 = C21^T, and C11 = C11 - C12 II with its mirror; the executor folds the
// mirrors and the transpose into the product epilogues, so it too launches
// four kernels per node.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "spin.h"
#include "spin_kernels.hpp"
#include "spin_plan.hpp"

namespace spin {

// ------------------------------------------------------------------ plan ----
// Order of the leading block when an order-m block is split: exact halving
// for m = leaf * 2^k, otherwise the half rounded up to a multiple of 64 so
// that block products stay aligned with the 64-wide tiles.
int64_t split_order(int64_t m) { return m >= 128 ? 64 * ((m + 127) / 128) : (m + 1) / 2; }

namespace {
Ref sub(const Ref &r, int64_t i, int64_t j) { return Ref{r.buf, r.off + i + j * r.ld, r.ld}; }

void push_products(Plan &P, int level, const PGemm &g0, const PGemm *g1) {
    POp op{};
    op.kind = 0;
    op.level = level;
    op.g[0] = g0;
    op.count = 1;
    if (g1) {
        op.g[1] = *g1;
        op.count = 2;
    }
    // a lower-triangle product counts the m (m + 1) / 2 outputs it has to form
    for (int q = 0; q < op.count; ++q)
        P.flops += op.g[q].lower ? (double)op.g[q].m * (op.g[q].m + 1) * op.g[q].k
                                 : 2.0 * op.g[q].m * op.g[q].n * op.g[q].k;
    P.ops.push_back(op);
}

void plan_node(Plan &P, Ref in, Ref out, int64_t m, int64_t wsoff, int level, int64_t col0) {
    if (m <= P.leaf) {
        POp op{};
        op.kind = 1;
        op.count = 1;
        op.level = level;
        op.in = in;
        op.out = out;
        op.L = m;
        op.col0 = col0;
        P.ops.push_back(op);
        P.max_leaf = std::max(P.max_leaf, m);
        P.flops += 2.0 * m * m * m;
        return;
    }
    const int64_t n1 = split_order(m), n2 = m - n1;
    const Ref A11 = sub(in, 0, 0), A21 = sub(in, n1, 0), A12 = sub(in, 0, n1),
              A22 = sub(in, n1, n1);
    const Ref C11 = sub(out, 0, 0), C21 = sub(out, n1, 0), C12 = sub(out, 0, n1),
              C22 = sub(out, n1, n1);
    // I = A11^-1, stored in the C11 view
    plan_node(P, A11, C11, n1, wsoff, level + 1, col0);
    // II (n2 x n1), III (n1 x n2) and S (n2 x n2) live until C11 is final
    const Ref II{BUF_WS, wsoff, n2};
    const Ref III{BUF_WS, wsoff + n2 * n1, n1};
    const Ref S{BUF_WS, wsoff + 2 * n1 * n2, n2};
    const int64_t next = wsoff + 2 * n1 * n2 + n2 * n2;
    P.ws_elems = std::max(P.ws_elems, next);
    const Ref none{BUF_WS, 0, 1};
    // II = A21 I, III = I A12                                   (one launch)
    const PGemm g_ii{A21, C11, none, II, n2, n1, n1, 1.0, 0.0, 0};
    const PGemm g_iii{C11, A12, none, III, n1, n2, n1, 1.0, 0.0, 0};
    push_products(P, level, g_ii, &g_iii);
    // S = A22 - A21 III  (= -V)
    push_products(P, level, PGemm{A21, III, A22, S, n2, n2, n1, -1.0, 1.0, 0}, nullptr);
    // C22 = S^-1  (= -VI)
    plan_node(P, S, C22, n2, next, level + 1, col0 + n1);
    // C12 = -III C22 (= III VI), C21 = -C22 II (= VI II)       (one launch)
    const PGemm g_c12{III, C22, none, C12, n1, n2, n2, -1.0, 0.0, 0};
    const PGemm g_c21{C22, II, none, C21, n2, n1, n2, -1.0, 0.0, 0};
    push_products(P, level, g_c12, &g_c21);
    // C11 = I - III C21, in place on the C11 view
    push_products(P, level, PGemm{III, C21, C11, C11, n1, n1, n2, -1.0, 1.0, 0}, nullptr);
}

// Alg. 1 for a symmetric A (the positive-definite matrices of Sec. 2.1),
// S-form.  Every block the recursion inverts is then symmetric, so III =
// I A12 = II^T and
//   S   = A22 - A21 III = A22 - II A12,
//   C12 = -III C22      = C21^T,
//   C11 = I - III C21   = I - C12 II.
// S and C11 are symmetric too: only their lower triangles are computed
// (tiles on or below the diagonal) and then mirrored onto the upper ones, so
// every block a node passes on is exactly symmetric outside the leaves.
// Passing on the rounding asymmetry instead breaks III = II^T at the next
// level and the residual grows like kappa u.  A node: II, S (lower half),
// mirror S, recursion, C21, transpose C12 = C21^T, C11 (lower half), mirror
// C11; about 6 h^3 flops against 12 h^3.  II (n2 x n1) and S live in the
// workspace.
void push_mirror(Plan &P, int level, const Ref &blk, int64_t m) {
    POp op{};
    op.kind = 3;
    op.count = 1;
    op.level = level;
    op.out = blk;
    op.tm = m;
    P.ops.push_back(op);
}

void plan_node_spd(Plan &P, Ref in, Ref out, int64_t m, int64_t wsoff, int level, int64_t col0) {
    if (m <= P.leaf) {
        plan_node(P, in, out, m, wsoff, level, col0);
        return;
    }
    const int64_t n1 = split_order(m), n2 = m - n1;
    const Ref A21 = sub(in, n1, 0), A12 = sub(in, 0, n1), A22 = sub(in, n1, n1);
    const Ref C11 = sub(out, 0, 0), C21 = sub(out, n1, 0), C12 = sub(out, 0, n1),
              C22 = sub(out, n1, n1);
    // I = A11^-1, stored in the C11 view
    plan_node_spd(P, sub(in, 0, 0), C11, n1, wsoff, level + 1, col0);
    const Ref II{BUF_WS, wsoff, n2};
    const Ref S{BUF_WS, wsoff + n2 * n1, n2};
    const int64_t next = wsoff + n2 * n1 + n2 * n2;
    P.ws_elems = std::max(P.ws_elems, next);
    const Ref none{BUF_WS, 0, 1};
    // II = A21 I
    push_products(P, level, PGemm{A21, C11, none, II, n2, n1, n1, 1.0, 0.0, 0}, nullptr);
    // S = A22 - II A12  (= A22 - A21 III = -V), lower half, then mirrored
    push_products(P, level, PGemm{II, A12, A22, S, n2, n2, n1, -1.0, 1.0, 0, 1}, nullptr);
    push_mirror(P, level, S, n2);
    // C22 = S^-1  (= -VI)
    plan_node_spd(P, S, C22, n2, next, level + 1, col0 + n1);
    // C21 = -C22 II  (= VI II)
    push_products(P, level, PGemm{C22, II, none, C21, n2, n1, n2, -1.0, 0.0, 0}, nullptr);
    // C12 = C21^T  (= III VI)
    POp t{};
    t.kind = 2;
    t.count = 1;
    t.level = level;
    t.in = C21;
    t.out = C12;
    t.tm = n2;
    t.tn = n1;
    P.ops.push_back(t);
    // C11 = I - C12 II  (= I - III C21), in place on the C11 view, lower half,
    // then mirrored
    push_products(P, level, PGemm{C12, II, C11, C11, n1, n1, n2, -1.0, 1.0, 0, 1}, nullptr);
    push_mirror(P, level, C11, n1);
}

// Inversion through a block LU factorisation without pivoting (the method the
// paper compares SPIN with, Sec. 5): the recursion produces Li = L^-1 and
// Ui = U^-1 into two full order-n workspace blocks that start zeroed,
//   (Li11, Ui11) = rec(A11);  {U12 = Li11 A12, L21 = A21 Ui11};
//   S = A22 - L21 U12;  {T1 = L21 Li11, T2 = Ui11 U12};  (Li22, Ui22) = rec(S);
//   {Li21 = -Li22 T1, Ui12 = -T2 Ui22},
// and X = Ui Li closes the schedule.  Leaves factor and invert in one kernel.
void plan_node_lu(Plan &P, Ref in, Ref li, Ref ui, int64_t m, int64_t wsoff, int level,
                  int64_t col0) {
    if (m <= P.leaf) {
        POp op{};
        op.kind = 4;
        op.count = 1;
        op.level = level;
        op.in = in;
        op.out = li;
        op.out2 = ui;
        op.L = m;
        op.col0 = col0;
        P.ops.push_back(op);
        P.flops += 4.0 / 3.0 * m * m * m;  // LU and two triangular inverses
        return;
    }
    const int64_t n1 = split_order(m), n2 = m - n1;
    const Ref A12 = sub(in, 0, n1), A21 = sub(in, n1, 0), A22 = sub(in, n1, n1);
    const Ref Li11 = sub(li, 0, 0), Li21 = sub(li, n1, 0), Li22 = sub(li, n1, n1);
    const Ref Ui11 = sub(ui, 0, 0), Ui12 = sub(ui, 0, n1), Ui22 = sub(ui, n1, n1);
    plan_node_lu(P, sub(in, 0, 0), Li11, Ui11, n1, wsoff, level + 1, col0);
    const Ref U12{BUF_WS, wsoff, n1};
    const Ref L21{BUF_WS, wsoff + n1 * n2, n2};
    const Ref S{BUF_WS, wsoff + 2 * n1 * n2, n2};
    const Ref T1{BUF_WS, wsoff + 2 * n1 * n2 + n2 * n2, n2};
    const Ref T2{BUF_WS, wsoff + 3 * n1 * n2 + n2 * n2, n1};
    const int64_t next = wsoff + 4 * n1 * n2 + n2 * n2;
    P.ws_elems = std::max(P.ws_elems, next);
    const Ref none{BUF_WS, 0, 1};
    const PGemm g_u12{Li11, A12, none, U12, n1, n2, n1, 1.0, 0.0, 0};
    const PGemm g_l21{A21, Ui11, none, L21, n2, n1, n1, 1.0, 0.0, 0};
    push_products(P, level, g_u12, &g_l21);
    push_products(P, level, PGemm{L21, U12, A22, S, n2, n2, n1, -1.0, 1.0, 0}, nullptr);
    const PGemm g_t1{L21, Li11, none, T1, n2, n1, n1, 1.0, 0.0, 0};
    const PGemm g_t2{Ui11, U12, none, T2, n1, n2, n1, 1.0, 0.0, 0};
    push_products(P, level, g_t1, &g_t2);
    plan_node_lu(P, S, Li22, Ui22, n2, next, level + 1, col0 + n1);
    const PGemm g_li21{Li22, T1, none, Li21, n2, n1, n2, -1.0, 0.0, 0};
    const PGemm g_ui12{T2, Ui22, none, Ui12, n1, n2, n2, -1.0, 0.0, 0};
    push_products(P, level, g_li21, &g_ui12);
}

}  // namespace

Plan make_plan_lu(int64_t n, int64_t lda, int64_t ldx, int64_t leaf) {
    Plan P;
    P.n = n;
    P.lda = lda;
    P.ldx = ldx;
    P.leaf = leaf;
    const Ref LI{BUF_WS, 0, n}, UI{BUF_WS, n * n, n};
    P.ws_elems = 2 * n * n;
    for (const Ref &r : {LI, UI}) {
        POp z{};
        z.kind = 5;
        z.count = 1;
        z.out = r;
        z.tm = n;
        z.tn = n;
        P.ops.push_back(z);
    }
    plan_node_lu(P, Ref{BUF_A, 0, lda}, LI, UI, n, 2 * n * n, 0, 0);
    const Ref none{BUF_WS, 0, 1};
    push_products(P, 0, PGemm{UI, LI, none, Ref{BUF_X, 0, ldx}, n, n, n, 1.0, 0.0, 0}, nullptr);
    return P;
}

Plan make_plan_spd(int64_t n, int64_t lda, int64_t ldx, int64_t leaf) {
    Plan P;
    P.n = n;
    P.lda = lda;
    P.ldx = ldx;
    P.leaf = leaf;
    plan_node_spd(P, Ref{BUF_A, 0, lda}, Ref{BUF_X, 0, ldx}, n, 0, 0, 0);
    return P;
}

Plan make_plan(int64_t n, int64_t lda, int64_t ldx, int64_t leaf) {
    Plan P;
    P.n = n;
    P.lda = lda;
    P.ldx = ldx;
    P.leaf = leaf;
    plan_node(P, Ref{BUF_A, 0, lda}, Ref{BUF_X, 0, ldx}, n, 0, 0, 0);
    return P;
}


// ------------------------------------------------------------ workspace ----
// Layout of a stream's workspace (bytes):
//   [0, 256)          status words (int): 0 = pivot status, 1 = refinement status
//   [256, 4096)       small doubles: 0..7 refinement norms, 8..15 misc norms
//   [4096, +8 KiB)    Frobenius-norm partials
//   then              recursion workspace, leaf scratch, mixed-mode buffers



Layout layout_for(int64_t n, int64_t leaf, int mode, int64_t ws_elems, int64_t max_leaf) {
    Layout L{};
    const size_t es = (mode == SPIN_FP64) ? 8 : 4;
    size_t off = kHdr;
    L.rec_off = off;
    L.rec_bytes = al256((size_t)ws_elems * es);
    off += L.rec_bytes;
    L.leaf_off = off;
    L.leaf_bytes = al256(leaf_scratch_bytes(max_leaf));
    off += L.leaf_bytes;
    if (mode != SPIN_FP64) {
        const size_t nn = (size_t)n * (size_t)n;
        L.a32_off = off;
        off += al256(nn * 4);
        L.x32_off = off;
        off += al256(nn * 4);
        L.r_off = off;
        off += al256(nn * 8);
        L.xalt_off = off;
        off += al256(nn * 8);
    }
    (void)leaf;
    L.total = off;
    return L;
}


GemmProb make_prob(char *const base[3], size_t es, const PGemm &g) {
    const bool use_c = g.beta != 0.0;
    auto at = [&](const Ref &r) -> void * { return base[r.buf] + (size_t)r.off * es; };
    return GemmProb{at(g.a),          at(g.b),       use_c ? at(g.c) : nullptr,
                    at(g.d),          g.a.ld,        g.b.ld,
                    use_c ? g.c.ld : 1, g.d.ld,      (int32_t)g.m,
                    (int32_t)g.n,     (int32_t)g.k,  g.add_identity,
                    g.alpha,          g.beta,        g.lower};
}

namespace {
// A rows x cols view; two views overlap only if they share a buffer and their
// element ranges meet and, for equal leading dimensions with neither view
// wrapping past a column end, both their row and their column ranges meet.
bool views_disjoint(const Ref &x, int64_t xr, int64_t xc, const Ref &y, int64_t yr, int64_t yc) {
    if (x.buf != y.buf || xr <= 0 || xc <= 0 || yr <= 0 || yc <= 0) return true;
    const int64_t xe = x.off + (xc - 1) * x.ld + xr, ye = y.off + (yc - 1) * y.ld + yr;
    if (xe <= y.off || ye <= x.off) return true;
    if (x.ld == y.ld && x.ld > 0) {
        const int64_t ld = x.ld;
        const int64_t x0 = x.off % ld, x1 = x.off / ld, y0 = y.off % ld, y1 = y.off / ld;
        if (x0 + xr > ld || y0 + yr > ld) return false;
        return x0 + xr <= y0 || y0 + yr <= x0 || x1 + xc <= y1 || y1 + yc <= x1;
    }
    return false;
}

bool same_ref(const Ref &x, const Ref &y) { return x.buf == y.buf && x.off == y.off && x.ld == y.ld; }
}  // namespace

int fold_kind(const Plan &P, size_t i) {
    if (i + 1 >= P.ops.size()) return 0;
    const POp &op = P.ops[i], &nx = P.ops[i + 1];
    if (op.kind != 0 || op.count != 1) return 0;
    const PGemm &g = op.g[0];
    if (g.m <= 0 || g.n <= 0) return 0;
    const bool use_c = g.beta != 0.0;
    if (nx.kind == 3) {
        // mirror of this lower-half product's result; the in-place form
        // C0 == D is safe because upper elements are neither read nor formed
        if (!g.lower || g.m != g.n || !same_ref(nx.out, g.d) || nx.tm != g.m) return 0;
        if (g.d.ld > INT32_MAX) return 0;
        if (!views_disjoint(g.a, g.m, g.k, g.d, g.m, g.n) || !views_disjoint(g.b, g.k, g.n, g.d, g.m, g.n))
            return 0;
        if (use_c && !same_ref(g.c, g.d) && !views_disjoint(g.c, g.m, g.n, g.d, g.m, g.n)) return 0;
        return 3;
    }
    if (nx.kind == 2) {
        // transpose of this product's full result into a block of its own
        if (g.lower || !same_ref(nx.in, g.d) || nx.tm != g.m || nx.tn != g.n) return 0;
        if (nx.out.ld > INT32_MAX) return 0;
        const Ref &t = nx.out;
        if (!views_disjoint(t, g.n, g.m, g.a, g.m, g.k) || !views_disjoint(t, g.n, g.m, g.b, g.k, g.n) ||
            !views_disjoint(t, g.n, g.m, g.d, g.m, g.n))
            return 0;
        if (use_c && !views_disjoint(t, g.n, g.m, g.c, g.m, g.n)) return 0;
        return 2;
    }
    return 0;
}

bool plan_folds_all(const Plan &P) {
    for (size_t i = 0; i < P.ops.size(); ++i)
        if ((P.ops[i].kind == 2 || P.ops[i].kind == 3) && (i == 0 || fold_kind(P, i - 1) == 0))
            return false;
    return true;
}

bool fold_next_step(const Plan &P, size_t i, char *const base[3], size_t es, GemmProb pr[2]) {
    if (es != 8 && es != 4) return false;
    const int f = fold_kind(P, i);
    if (f == 3) {
        pr[0].DT = pr[0].D;
        pr[0].lddt = (int32_t)P.ops[i].g[0].d.ld;
        return true;
    }
    if (f == 2) {
        const Ref &t = P.ops[i + 1].out;
        pr[0].DT = base[t.buf] + (size_t)t.off * es;
        pr[0].lddt = (int32_t)t.ld;
        return true;
    }
    return false;
}

namespace {

// ------------------------------------------------------------- tracing ----
struct TraceRec {
    std::string name;
    double flops, bytes;
    int level;
    hipEvent_t start, stop;
};

std::mutex g_mu;
bool g_trace_on = false;
std::vector<TraceRec> g_trace;

struct TraceCtx {
    hipStream_t s;
    int level;
    hipEvent_t pending;
};

void trace_cb(void *vctx, const LaunchInfo &li, int phase) {
    TraceCtx *ctx = static_cast<TraceCtx *>(vctx);
    if (phase == 0) {
        hipEventCreate(&ctx->pending);
        hipEventRecord(ctx->pending, ctx->s);
    } else {
        hipEvent_t stop;
        hipEventCreate(&stop);
        hipEventRecord(stop, ctx->s);
        g_trace.push_back(TraceRec{li.name ? li.name : "?", li.flops, li.bytes, ctx->level,
                                   ctx->pending, stop});
        ctx->pending = nullptr;
    }
}

struct Workspace {
    char *base = nullptr;
    size_t bytes = 0;
};

std::map<hipStream_t, Workspace> g_ws;
std::map<std::tuple<int, int64_t, int64_t, int64_t, int64_t, const void *, void *, void *, int>,
         hipGraphExec_t>
    g_graphs;
hipStream_t g_capture = nullptr;
// Largest number of cached graphs (one per mode, shape, buffer set and stream
// workspace) before the cache is emptied.
constexpr size_t kMaxGraphs = 64;
// Added to a graph key's entry-point id when leaves skip the speculative
// elimination.
constexpr int kNoSpecKey = 1 << 12;

void drop_graphs_for(void *base) {
    for (auto it = g_graphs.begin(); it != g_graphs.end();) {
        if (std::get<7>(it->first) == base) {
            hipGraphExecDestroy(it->second);
            it = g_graphs.erase(it);
        } else {
            ++it;
        }
    }
}

// Returns the stream's workspace with at least `bytes` (caller holds g_mu).
int ws_acquire(hipStream_t s, size_t bytes, Workspace **out) {
    Workspace &w = g_ws[s];
    if (w.bytes < bytes) {
        void *p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess || !p) {
            (void)hipGetLastError();
            return SPIN_E_NOMEM;
        }
        if (w.base) {
            // the status words of the last call on the stream move along, so
            // that spin_info still reports it after a later call grew the
            // workspace without writing them (spin_residual)
            hipError_t e = hipMemcpyAsync(p, w.base, 256, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                hipFree(p);
                return SPIN_E_HIP;
            }
            drop_graphs_for(w.base);
            hipFree(w.base);
        } else {
            // a fresh workspace reports "no event" until an inversion runs
            if (status_reset(static_cast<int *>(p), true, s) != hipSuccess) {
                (void)hipGetLastError();
                hipFree(p);
                return SPIN_E_HIP;
            }
        }
        w.base = static_cast<char *>(p);
        w.bytes = bytes;
    }
    *out = &w;
    return SPIN_OK;
}

// ------------------------------------------------------------- executor ----
struct Exec {
    hipStream_t s;
    char *base[3];
    size_t es;
    DType dt;  // storage type of the plan's operands and leaves
    int *status;
    void *leaf_scratch;
    DType gdt = kF64;  // product flavour of the plan's products
    bool no_trace = false;  // never trace (the allocation-free entry point)
};

inline void *at(const Exec &E, const Ref &r) {
    return E.base[r.buf] + (size_t)r.off * E.es;
}

hipError_t run_plan(const Plan &P, const Exec &E) {
    bool exch_filled = false;  // the leaf scratch's exchange areas (leaf_launch)
    for (size_t i = 0; i < P.ops.size(); ++i) {
        const POp &op = P.ops[i];
        TraceCtx ctx{E.s, op.level, nullptr};
        const bool tr = g_trace_on && !E.no_trace;
        if (op.kind == 0) {
            GemmProb pr[2];
            for (int q = 0; q < op.count; ++q) pr[q] = make_prob(E.base, E.es, op.g[q]);
            if (fold_next_step(P, i, E.base, E.es, pr)) ++i;  // mirror / transpose in the epilogue
            LaunchInfo li{};
            if (tr) trace_cb(&ctx, li, 0);
            hipError_t e = gemm_launch(pr, op.count, E.gdt, E.s, &li);
            if (tr) trace_cb(&ctx, li, 1);
            if (e != hipSuccess) return e;
        } else if (op.kind == 2) {
            if (E.dt != kF64) return hipErrorInvalidValue;
            LaunchInfo li{"transpose", 0.0, 16.0 * (double)op.tm * (double)op.tn};
            if (tr) trace_cb(&ctx, li, 0);
            hipError_t e = transpose_f64(static_cast<const double *>(at(E, op.in)), op.in.ld,
                                         static_cast<double *>(at(E, op.out)), op.out.ld, op.tm,
                                         op.tn, E.s);
            if (tr) trace_cb(&ctx, li, 1);
            if (e != hipSuccess) return e;
        } else if (op.kind == 4) {
            if (E.dt != kF64) return hipErrorInvalidValue;
            const double Ld = (double)op.L;
            LaunchInfo li{"lu_leaf", 4.0 / 3.0 * Ld * Ld * Ld, 24.0 * Ld * Ld};
            if (tr) trace_cb(&ctx, li, 0);
            hipError_t e = lu_leaf_launch(static_cast<const double *>(at(E, op.in)), op.in.ld,
                                          static_cast<double *>(at(E, op.out)), op.out.ld,
                                          static_cast<double *>(at(E, op.out2)), op.out2.ld, op.L,
                                          op.col0, E.status, E.s);
            if (tr) trace_cb(&ctx, li, 1);
            if (e != hipSuccess) return e;
        } else if (op.kind == 5) {
            if (E.dt != kF64) return hipErrorInvalidValue;
            LaunchInfo li{"fill", 0.0, 8.0 * (double)op.tm * (double)op.tn};
            if (tr) trace_cb(&ctx, li, 0);
            hipError_t e = fill_zero_f64(static_cast<double *>(at(E, op.out)), op.out.ld, op.tm,
                                         op.tn, E.s);
            if (tr) trace_cb(&ctx, li, 1);
            if (e != hipSuccess) return e;
        } else if (op.kind == 3) {
            if (E.dt != kF64) return hipErrorInvalidValue;
            LaunchInfo li{"mirror", 0.0, 8.0 * (double)op.tm * (double)op.tm};
            if (tr) trace_cb(&ctx, li, 0);
            hipError_t e = mirror_lower_f64(static_cast<double *>(at(E, op.out)), op.out.ld, op.tm, E.s);
            if (tr) trace_cb(&ctx, li, 1);
            if (e != hipSuccess) return e;
        } else {
            hipError_t e = leaf_launch(at(E, op.in), E.dt, op.in.ld, at(E, op.out), E.dt,
                                       op.out.ld, op.L, op.col0, E.status, E.leaf_scratch,
                                       exch_filled, E.s, tr ? trace_cb : nullptr, &ctx);
            if (e != hipSuccess) return e;
            exch_filled = exch_filled || leaf_fills_exchange(op.L);
        }
    }
    return hipSuccess;
}

// ------------------------------------------------------------- helpers ----
int validate(const void *A, int64_t n, int64_t lda, const void *X, int64_t ldx, int64_t leaf) {
    if (!A || !X) return SPIN_E_NULL;
    if (n < 1 || n > SPIN_MAX_N) return SPIN_E_N;
    if (lda < n || ldx < n) return SPIN_E_LD;
    if (leaf < 1 || leaf > SPIN_MAX_LEAF) return SPIN_E_LEAF;
    const char *a0 = static_cast<const char *>(A);
    const char *a1 = a0 + ((size_t)(n - 1) * lda + n) * sizeof(double);
    const char *x0 = static_cast<const char *>(X);
    const char *x1 = x0 + ((size_t)(n - 1) * ldx + n) * sizeof(double);
    if (a0 < x1 && x0 < a1) return SPIN_E_ALIAS;
    return SPIN_OK;
}

}  // namespace

// Whether leaves try the speculative elimination first (SPIN_NO_SPEC=1 turns
// it off; the results are the same either way).
bool leaf_spec_enabled() {
    const char *e = std::getenv("SPIN_NO_SPEC");
    return !(e && e[0] && e[0] != '0');
}

namespace {

bool graphs_enabled() {
    const char *e = std::getenv("SPIN_NO_GRAPH");
    return !(e && e[0] && e[0] != '0') && !g_trace_on;
}

int hip_fail(hipError_t e) {
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? SPIN_E_NOMEM : SPIN_E_HIP;
}

// Enqueue `body(stream)` either directly or through a cached graph.
template <typename F>
int run_maybe_graph(const std::tuple<int, int64_t, int64_t, int64_t, int64_t, const void *, void *,
                                     void *, int> &key,
                    hipStream_t s, F body) {
    if (!graphs_enabled()) {
        hipError_t e = body(s);
        return e == hipSuccess ? SPIN_OK : hip_fail(e);
    }
    auto it = g_graphs.find(key);
    if (it == g_graphs.end() && g_graphs.size() >= kMaxGraphs) {
        // bounded cache: callers that cycle through many buffers must not grow
        // it without limit.  Wait for every launch, then drop all graphs; they
        // are captured again on their next use.
        if (hipDeviceSynchronize() != hipSuccess) return hip_fail(hipErrorUnknown);
        for (auto &kv : g_graphs) hipGraphExecDestroy(kv.second);
        g_graphs.clear();
    }
    if (it == g_graphs.end()) {
        if (!g_capture && hipStreamCreateWithFlags(&g_capture, hipStreamNonBlocking) != hipSuccess)
            return hip_fail(hipErrorUnknown);
        if (hipStreamBeginCapture(g_capture, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return hip_fail(hipErrorUnknown);
        hipError_t e = body(g_capture);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(g_capture, &graph);
        if (e != hipSuccess || e2 != hipSuccess || !graph) {
            if (graph) hipGraphDestroy(graph);
            return hip_fail(e != hipSuccess ? e : e2);
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e);
        it = g_graphs.emplace(key, exec).first;
    }
    hipError_t e = hipGraphLaunch(it->second, s);
    return e == hipSuccess ? SPIN_OK : hip_fail(e);
}

int *status_ptr(Workspace *w) { return reinterpret_cast<int *>(w->base); }
double *norm_ptr(Workspace *w) { return reinterpret_cast<double *>(w->base + 256); }
double *partials_ptr(Workspace *w) { return reinterpret_cast<double *>(w->base + 4096); }

}  // namespace
}  // namespace spin

namespace spin {

size_t invert_workspace_bytes(int64_t n, int64_t leaf) {
    const Plan P = make_plan(n, n, n, leaf);
    return layout_for(n, leaf, SPIN_FP64, P.ws_elems, P.max_leaf).total;
}

int invert_on_workspace(const double *A, int64_t n, int64_t lda, double *Ainv, int64_t ldx,
                        int64_t leaf, char *ws, size_t ws_bytes, int *info, hipStream_t s) {
    int rc = validate(A, n, lda, Ainv, ldx, leaf);
    if (rc) return rc;
    const Plan P = make_plan(n, lda, ldx, leaf);
    const Layout L = layout_for(n, leaf, SPIN_FP64, P.ws_elems, P.max_leaf);
    if (L.total > ws_bytes) return SPIN_E_SCRATCH;
    Exec E{s, {(char *)A, (char *)Ainv, ws + L.rec_off}, 8, kF64, reinterpret_cast<int *>(ws),
           ws + L.leaf_off};
    E.no_trace = true;
    hipError_t e = status_reset(E.status, leaf_spec_enabled(), s);
    if (e == hipSuccess) e = run_plan(P, E);
    if (e == hipSuccess && info) e = status_copy(E.status, info, s);
    return e == hipSuccess ? SPIN_OK : hip_fail(e);
}

}  // namespace spin

using namespace spin;

extern "C" {

int spin_invert(const double *A, int64_t n, int64_t lda, double *Ainv, int64_t ldx, int64_t leaf,
                spin_stream_t stream) {
    int rc = validate(A, n, lda, Ainv, ldx, leaf);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(g_mu);
    Plan P = make_plan(n, lda, ldx, leaf);
    Layout L = layout_for(n, leaf, SPIN_FP64, P.ws_elems, P.max_leaf);
    Workspace *w = nullptr;
    rc = ws_acquire(s, L.total, &w);
    if (rc) return rc;
    Exec E{s, {(char *)A, (char *)Ainv, w->base + L.rec_off}, 8, kF64, status_ptr(w),
           w->base + L.leaf_off};
    const bool spec = leaf_spec_enabled();
    auto body = [&](hipStream_t qs) -> hipError_t {
        Exec Eq = E;
        Eq.s = qs;
        hipError_t e = status_reset(Eq.status, spec, qs);
        if (e != hipSuccess) return e;
        return run_plan(P, Eq);
    };
    return run_maybe_graph(std::make_tuple(spec ? 0 : kNoSpecKey, n, lda, ldx, leaf, (const void *)A, (void *)Ainv,
                                           (void *)w->base, 0),
                           s, body);
}

int spin_invert_spd(const double *A, int64_t n, int64_t lda, double *Ainv, int64_t ldx,
                    int64_t leaf, spin_stream_t stream) {
    int rc = validate(A, n, lda, Ainv, ldx, leaf);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(g_mu);
    Plan P = make_plan_spd(n, lda, ldx, leaf);
    Layout L = layout_for(n, leaf, SPIN_FP64, P.ws_elems, P.max_leaf);
    Workspace *w = nullptr;
    rc = ws_acquire(s, L.total, &w);
    if (rc) return rc;
    Exec E{s, {(char *)A, (char *)Ainv, w->base + L.rec_off}, 8, kF64, status_ptr(w),
           w->base + L.leaf_off};
    const bool spec = leaf_spec_enabled();
    auto body = [&](hipStream_t qs) -> hipError_t {
        Exec Eq = E;
        Eq.s = qs;
        hipError_t e = status_reset(Eq.status, spec, qs);
        if (e != hipSuccess) return e;
        return run_plan(P, Eq);
    };
    return run_maybe_graph(std::make_tuple(spec ? 2 : 2 + kNoSpecKey, n, lda, ldx, leaf, (const void *)A, (void *)Ainv,
                                           (void *)w->base, 0),
                           s, body);
}

int spin_invert_lu(const double *A, int64_t n, int64_t lda, double *Ainv, int64_t ldx,
                   int64_t leaf, spin_stream_t stream) {
    int rc = validate(A, n, lda, Ainv, ldx, leaf);
    if (rc) return rc;
    if (leaf > kLuLeafMax) return SPIN_E_LEAF;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(g_mu);
    Plan P = make_plan_lu(n, lda, ldx, leaf);
    Layout L = layout_for(n, leaf, SPIN_FP64, P.ws_elems, 0);
    Workspace *w = nullptr;
    rc = ws_acquire(s, L.total, &w);
    if (rc) return rc;
    Exec E{s, {(char *)A, (char *)Ainv, w->base + L.rec_off}, 8, kF64, status_ptr(w),
           w->base + L.leaf_off};
    const bool spec = leaf_spec_enabled();
    auto body = [&](hipStream_t qs) -> hipError_t {
        Exec Eq = E;
        Eq.s = qs;
        hipError_t e = status_reset(Eq.status, spec, qs);
        if (e != hipSuccess) return e;
        return run_plan(P, Eq);
    };
    return run_maybe_graph(std::make_tuple(spec ? 3 : 3 + kNoSpecKey, n, lda, ldx, leaf, (const void *)A, (void *)Ainv,
                                           (void *)w->base, 0),
                           s, body);
}

int spin_invert_mixed(const double *A, int64_t n, int64_t lda, double *Ainv, int64_t ldx,
                      int64_t leaf, int mode, int ns_steps, spin_report *rep,
                      spin_stream_t stream) {
    int rc = validate(A, n, lda, Ainv, ldx, leaf);
    if (rc) return rc;
    // SPIN_SYMMETRIC: the symmetric schedule with the mode's product flavour;
    // SPIN_REFINE_INT8: the refinement's products emulated on INT8 cores
    const bool sym = (mode & SPIN_SYMMETRIC) != 0;
    const bool emu = (mode & SPIN_REFINE_INT8) != 0;
    const int pmode = mode & ~(SPIN_SYMMETRIC | SPIN_REFINE_INT8);
    if (!is_mixed_mode(pmode) || ns_steps < 0 || ns_steps > kNormSlots) return SPIN_E_MODE;
    if (emu && n > kOzakiMaxK) return SPIN_E_N;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(g_mu);
    Plan P = sym ? make_plan_spd(n, n, n, leaf) : make_plan(n, n, n, leaf);
    // FP32 storage has no mirror or transpose kernel of its own
    if (!plan_folds_all(P)) return SPIN_E_MODE;
    Layout L = layout_for(n, leaf, pmode, P.ws_elems, P.max_leaf);
    const size_t oz_off = L.total;
    const int oz_beta = std::min(53, ozaki_beta(kRefineModuli, n));
    const size_t oz_bytes = emu ? ozaki_workspace_bytes(n, n, n, kRefineModuli) : 0;
    Workspace *w = nullptr;
    rc = ws_acquire(s, oz_off + oz_bytes, &w);
    if (rc) return rc;
    char *base = w->base;
    // residual / update product of the refinement: FP64 matrix cores, or
    // the INT8 emulation (epilogue 1: I - P, 2: C0 + P)
    auto refine_product = [&](const double *pa, int64_t la, const double *pb, int64_t lb, int epi,
                              const double *c0, int64_t lc, double *d, int64_t ld, hipStream_t qs,
                              LaunchInfo *li) -> hipError_t {
        if (emu) {
            OzakiProb op{pa, la, pb, lb, c0, lc, d, ld, n, n, n, epi, kRefineModuli, oz_beta, oz_beta};
            if (li) *li = LaunchInfo{"gemm_int8_emulated", 2.0 * n * (double)n * n, 24.0 * n * (double)n};
            return ozaki_product(op, base + oz_off, qs);
        }
        GemmProb pr{pa, pb, epi == 2 ? c0 : nullptr, d, la, lb, epi == 2 ? lc : 1, ld,
                    (int32_t)n, (int32_t)n, (int32_t)n, epi == 1 ? 1 : 0, epi == 1 ? -1.0 : 1.0,
                    epi == 2 ? 1.0 : 0.0};
        return gemm_launch(&pr, 1, kF64, qs, li);
    };
    float *A32 = reinterpret_cast<float *>(base + L.a32_off);
    float *X32 = reinterpret_cast<float *>(base + L.x32_off);
    double *R = reinterpret_cast<double *>(base + L.r_off);
    double *Xalt = reinterpret_cast<double *>(base + L.xalt_off);
    int *status = status_ptr(w);
    double *norms = norm_ptr(w);
    double *parts = partials_ptr(w);
    // Buffers alternate between refinement steps so that the last step writes Ainv.
    double *buf0 = (ns_steps % 2 == 0) ? Ainv : Xalt;
    const int64_t ld0 = (ns_steps % 2 == 0) ? ldx : n;
    double *buf1 = (ns_steps % 2 == 0) ? Xalt : Ainv;
    const int64_t ld1 = (ns_steps % 2 == 0) ? n : ldx;

    const bool spec = leaf_spec_enabled();
    auto body = [&](hipStream_t qs) -> hipError_t {
        hipError_t e = status_reset(status, spec, qs);
        if (e != hipSuccess) return e;
        e = cast_f64_to_f32(A, lda, A32, n, n, n, qs);
        if (e != hipSuccess) return e;
        Exec E{qs, {(char *)A32, (char *)X32, base + L.rec_off}, 4, kF32, status,
               base + L.leaf_off, mixed_product_type(pmode)};
        e = run_plan(P, E);
        if (e != hipSuccess) return e;
        e = cast_f32_to_f64(X32, n, buf0, ld0, n, n, qs);
        if (e != hipSuccess) return e;
        for (int j = 0; j < ns_steps; ++j) {
            double *xc = (j % 2 == 0) ? buf0 : buf1;
            const int64_t ldc = (j % 2 == 0) ? ld0 : ld1;
            double *xn = (j % 2 == 0) ? buf1 : buf0;
            const int64_t ldn = (j % 2 == 0) ? ld1 : ld0;
            TraceCtx ctx{qs, -1, nullptr};
            // R = I - A X
            LaunchInfo li{};
            if (g_trace_on) trace_cb(&ctx, li, 0);
            e = refine_product(A, lda, xc, ldc, 1, nullptr, 1, R, n, qs, &li);
            if (g_trace_on) trace_cb(&ctx, li, 1);
            if (e != hipSuccess) return e;
            e = frob2(R, n, n, n, parts, norms + j, qs);
            if (e != hipSuccess) return e;
            e = ns_check(norms, j, status + 1, qs);
            if (e != hipSuccess) return e;
            // X' = X + X R
            if (g_trace_on) trace_cb(&ctx, li, 0);
            e = refine_product(xc, ldc, R, n, 2, xc, ldc, xn, ldn, qs, &li);
            if (g_trace_on) trace_cb(&ctx, li, 1);
            if (e != hipSuccess) return e;
        }
        if (ns_steps > 0) {
            // acceptance of the refined inverse (now in Ainv): rho <= kNsTol
            double *misc = norms + kNormSlots;  // 0: |A|^2, 2: |R_final|^2, 3: |X|^2
            TraceCtx ctx{qs, -1, nullptr};
            LaunchInfo li{};
            if (g_trace_on) trace_cb(&ctx, li, 0);
            e = refine_product(A, lda, Ainv, ldx, 1, nullptr, 1, R, n, qs, &li);
            if (g_trace_on) trace_cb(&ctx, li, 1);
            if (e == hipSuccess) e = frob2(R, n, n, n, parts, misc + 2, qs);
            if (e == hipSuccess) e = frob2(A, lda, n, n, parts, misc + 0, qs);
            if (e == hipSuccess) e = frob2(Ainv, ldx, n, n, parts, misc + 3, qs);
            if (e == hipSuccess) e = ns_final(misc + 2, misc + 0, misc + 3, kNsTol, status + 1, qs);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    rc = run_maybe_graph(std::make_tuple(1 + 16 * mode + (spec ? 0 : kNoSpecKey), n, lda, ldx, leaf, (const void *)A,
                                         (void *)Ainv, (void *)base, ns_steps),
                         s, body);
    if (rc || !rep) return rc;

    // Report: residual of the unrefined and of the final inverse.  With
    // refinement the final residual and the norms of A and X come from the
    // acceptance test above; X0 is no longer stored, so it is recomputed
    // from X32.  Without refinement X0 is the result.
    std::memset(rep, 0, sizeof(*rep));
    rep->steps = ns_steps;
    double *misc = norms + kNormSlots;  // 0: |A|^2, 1: |X0|^2, 2: |R_final|^2, 3: |X|^2
    hipError_t e = hipSuccess;
    if (ns_steps > 0) {
        e = cast_f32_to_f64(X32, n, R, n, n, n, s);
        if (e == hipSuccess) e = frob2(R, n, n, n, parts, misc + 1, s);
    } else {
        GemmProb pr{A, Ainv, nullptr, R, lda, ldx, 1, n, (int32_t)n, (int32_t)n, (int32_t)n,
                    1, -1.0, 0.0};
        e = gemm_launch(&pr, 1, kF64, s, nullptr);
        if (e == hipSuccess) e = frob2(R, n, n, n, parts, norms + 0, s);
        if (e == hipSuccess) e = frob2(R, n, n, n, parts, misc + 2, s);
        if (e == hipSuccess) e = frob2(A, lda, n, n, parts, misc + 0, s);
        if (e == hipSuccess) e = frob2(Ainv, ldx, n, n, parts, misc + 1, s);
        if (e == hipSuccess) e = frob2(Ainv, ldx, n, n, parts, misc + 3, s);
    }
    // copies ordered on the caller's stream (not the null stream), then wait for it
    double h_norms[kNormSlots + 4];
    int h_status[2];
    if (e == hipSuccess) e = hipMemcpyAsync(h_norms, norms, sizeof(h_norms), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h_status, status, sizeof(h_status), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    const double na = std::sqrt(h_norms[kNormSlots + 0]);
    const double nx0 = std::sqrt(h_norms[kNormSlots + 1]);
    const double nr = std::sqrt(h_norms[kNormSlots + 2]);
    const double nx = std::sqrt(h_norms[kNormSlots + 3]);
    rep->r0_fro = std::sqrt(h_norms[0]);
    for (int j = 0; j < ns_steps; ++j) rep->r_fro[j] = std::sqrt(h_norms[j]);
    rep->rho_before = rep->r0_fro / (na * nx0);
    rep->rho_after = nr / (na * nx);
    rep->status = (h_status[0] != INT32_MAX) ? h_status[0]
                  : (h_status[1] != INT32_MAX) ? h_status[1]
                                               : 0;
    return SPIN_OK;
}

int spin_gemm(int dtype, int64_t m, int64_t n, int64_t k, double alpha, const void *A,
              int64_t lda, const void *B, int64_t ldb, double beta, const void *C0, int64_t ldc,
              void *D, int64_t ldd, int add_identity, spin_stream_t stream) {
    if (!is_mode(dtype)) return SPIN_E_MODE;
    if (m < 0 || n < 0 || k < 0 || m > INT32_MAX || n > INT32_MAX || k > INT32_MAX)
        return SPIN_E_N;
    if (!D || (k > 0 && (!A || !B)) || (beta != 0.0 && !C0)) return SPIN_E_NULL;
    if (ldd < std::max<int64_t>(m, 1) || (k > 0 && (lda < std::max<int64_t>(m, 1) ||
                                                    ldb < std::max<int64_t>(k, 1))) ||
        (beta != 0.0 && ldc < std::max<int64_t>(m, 1)))
        return SPIN_E_LD;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    GemmProb pr{A, B, beta != 0.0 ? C0 : nullptr, D, lda, ldb, beta != 0.0 ? ldc : 1, ldd,
                (int32_t)m, (int32_t)n, (int32_t)k, add_identity ? 1 : 0, alpha, beta};
    std::lock_guard<std::mutex> lk(g_mu);
    TraceCtx ctx{s, -1, nullptr};
    LaunchInfo li{};
    if (g_trace_on) trace_cb(&ctx, li, 0);
    hipError_t e = gemm_launch(&pr, 1, dtype == SPIN_FP64 ? kF64 : mixed_product_type(dtype), s, &li);
    if (g_trace_on) trace_cb(&ctx, li, 1);
    return e == hipSuccess ? SPIN_OK : hip_fail(e);
}

int spin_gemm_int8(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda, const double *B,
                   int64_t ldb, int epilogue, const double *C0, int64_t ldc, double *D, int64_t ldd,
                   int moduli, int beta_a, int beta_b, spin_stream_t stream) {
    if (epilogue < 0 || epilogue > 2 || moduli < 2 || moduli > kOzakiMaxModuli) return SPIN_E_MODE;
    if (m < 0 || n < 0 || k < 0 || m > INT32_MAX / 2 || n > INT32_MAX / 2 || k > kOzakiMaxK)
        return SPIN_E_N;
    if (epilogue == 1 && m != n) return SPIN_E_N;
    if (!D || (k > 0 && (!A || !B)) || (epilogue == 2 && !C0)) return SPIN_E_NULL;
    if (ldd < std::max<int64_t>(m, 1) || (k > 0 && (lda < std::max<int64_t>(m, 1) ||
                                                    ldb < std::max<int64_t>(k, 1))) ||
        (epilogue == 2 && ldc < std::max<int64_t>(m, 1)))
        return SPIN_E_LD;
    if (beta_a <= 0 || beta_b <= 0) beta_a = beta_b = std::min(53, ozaki_beta(moduli, k));
    if (beta_a < 1 || beta_b < 1 || beta_a > 53 || beta_b > 53 ||
        1.0 + std::log2((double)std::max<int64_t>(k, 1)) + beta_a + beta_b >= ozaki_log2_modulus(moduli))
        return SPIN_E_MODE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace *w = nullptr;
    int rc = ws_acquire(s, kHdr + ozaki_workspace_bytes(m, n, k, moduli), &w);
    if (rc) return rc;
    OzakiProb p{A, lda, B, ldb, C0, ldc, D, ldd, m, n, k, epilogue, moduli, beta_a, beta_b};
    TraceCtx ctx{s, -1, nullptr};
    LaunchInfo li{"gemm_int8_emulated", 2.0 * (double)m * (double)n * (double)k,
                  8.0 * (double)(m * k + k * n + m * n)};
    if (g_trace_on) trace_cb(&ctx, li, 0);
    hipError_t e = ozaki_product(p, w->base + kHdr, s);
    if (g_trace_on) trace_cb(&ctx, li, 1);
    return e == hipSuccess ? SPIN_OK : hip_fail(e);
}

int spin_info(spin_stream_t stream) {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int h[2] = {INT32_MAX, INT32_MAX};
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_ws.find(s);
        if (it == g_ws.end() || !it->second.base) return SPIN_OK;
        if (hipMemcpyAsync(h, it->second.base, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return hip_fail(hipErrorUnknown);
    }
    if (h[0] != INT32_MAX) return h[0];
    if (h[1] != INT32_MAX) return h[1];
    return SPIN_OK;
}

int spin_residual(const double *A, int64_t n, int64_t lda, const double *X, int64_t ldx,
                  double *rho, spin_stream_t stream) {
    if (!A || !X || !rho) return SPIN_E_NULL;
    if (n < 1 || n > SPIN_MAX_N) return SPIN_E_N;
    if (lda < n || ldx < n) return SPIN_E_LD;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(g_mu);
    Workspace *w = nullptr;
    int rc = ws_acquire(s, kHdr + al256((size_t)n * n * 8), &w);
    if (rc) return rc;
    double *R = reinterpret_cast<double *>(w->base + kHdr);
    double *norms = norm_ptr(w) + kNormSlots + 4;  // 3 slots after the mixed-mode ones
    double *parts = partials_ptr(w);
    GemmProb pr{A, X, nullptr, R, lda, ldx, 1, n, (int32_t)n, (int32_t)n, (int32_t)n, 1, -1.0, 0.0};
    hipError_t e = gemm_launch(&pr, 1, kF64, s, nullptr);
    if (e == hipSuccess) e = frob2(R, n, n, n, parts, norms + 0, s);
    if (e == hipSuccess) e = frob2(A, lda, n, n, parts, norms + 1, s);
    if (e == hipSuccess) e = frob2(X, ldx, n, n, parts, norms + 2, s);
    double h[3];
    if (e == hipSuccess) e = hipMemcpyAsync(h, norms, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    *rho = std::sqrt(h[0]) / (std::sqrt(h[1]) * std::sqrt(h[2]));
    return SPIN_OK;
}

size_t spin_workspace_bytes(int64_t n, int64_t leaf, int mode) {
    if (n < 1 || n > SPIN_MAX_N || leaf < 1 || leaf > SPIN_MAX_LEAF) return 0;
    const bool sym = (mode & SPIN_SYMMETRIC) != 0;
    const int pmode = mode & ~SPIN_SYMMETRIC;
    if (!is_mode(pmode)) return 0;
    Plan P = sym ? make_plan_spd(n, n, n, leaf) : make_plan(n, n, n, leaf);
    return layout_for(n, leaf, pmode, P.ws_elems, P.max_leaf).total;
}

const char *spin_strerror(int code) {
    switch (code) {
    case SPIN_OK: return "success";
    case SPIN_E_NULL: return "null pointer argument";
    case SPIN_E_N: return "matrix order out of range";
    case SPIN_E_LD: return "leading dimension smaller than the matrix order";
    case SPIN_E_LEAF: return "leaf order out of range";
    case SPIN_E_ALIAS: return "input and output overlap";
    case SPIN_E_MODE: return "unknown precision mode or refinement step count";
    case SPIN_E_COUNT: return "batch count out of range";
    case SPIN_E_SCRATCH: return "order too large for the fixed scratch of spin_invert_noalloc";
    case SPIN_E_NOMEM: return "device memory allocation failed";
    case SPIN_E_HIP: return "HIP runtime or kernel launch error";
    case SPIN_NS_DIVERGED: return "Newton refinement diverged or missed the residual bound";
    default: return code > 0 ? "zero or non-finite pivot in a leaf block" : "unknown status";
    }
}

void spin_release(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    hipDeviceSynchronize();
    for (auto &kv : g_graphs) hipGraphExecDestroy(kv.second);
    g_graphs.clear();
    for (auto &kv : g_ws)
        if (kv.second.base) hipFree(kv.second.base);
    g_ws.clear();
}

}  // extern "C"

namespace {
int64_t describe_plan(const Plan &P, spin_plan_op *ops, int64_t cap, double *flops) {
    if (flops) *flops = P.flops;
    const int64_t cnt = (int64_t)P.ops.size();
    for (int64_t i = 0; i < cnt && i < cap; ++i) {
        const POp &op = P.ops[(size_t)i];
        spin_plan_op o;
        std::memset(&o, 0, sizeof(o));
        o.kind = op.kind;
        o.count = op.count;
        o.level = op.level;
        if (op.kind == 0) {
            for (int q = 0; q < op.count; ++q) {
                const PGemm &g = op.g[q];
                o.m[q] = g.m;
                o.n[q] = g.n;
                o.k[q] = g.k;
                o.a_buf[q] = g.a.buf;
                o.b_buf[q] = g.b.buf;
                o.c_buf[q] = g.beta != 0.0 ? g.c.buf : -1;
                o.d_buf[q] = g.d.buf;
                o.a_off[q] = g.a.off;
                o.b_off[q] = g.b.off;
                o.c_off[q] = g.c.off;
                o.d_off[q] = g.d.off;
                o.a_ld[q] = g.a.ld;
                o.b_ld[q] = g.b.ld;
                o.c_ld[q] = g.c.ld;
                o.d_ld[q] = g.d.ld;
                o.alpha[q] = g.alpha;
                o.beta[q] = g.beta;
                if (g.lower) o.flags |= 1 << q;
            }
            if (fold_kind(P, (size_t)i)) o.flags |= 4;
        } else if (op.kind == 4) {
            o.a_buf[0] = op.in.buf;
            o.a_off[0] = op.in.off;
            o.a_ld[0] = op.in.ld;
            o.d_buf[0] = op.out.buf;
            o.d_off[0] = op.out.off;
            o.d_ld[0] = op.out.ld;
            o.c_buf[0] = op.out2.buf;
            o.c_off[0] = op.out2.off;
            o.c_ld[0] = op.out2.ld;
            o.leaf_order = op.L;
            o.col0 = op.col0;
        } else if (op.kind == 5) {
            o.m[0] = op.tm;
            o.n[0] = op.tn;
            o.d_buf[0] = op.out.buf;
            o.d_off[0] = op.out.off;
            o.d_ld[0] = op.out.ld;
        } else if (op.kind == 3) {
            o.m[0] = op.tm;
            o.n[0] = op.tm;
            o.d_buf[0] = op.out.buf;
            o.d_off[0] = op.out.off;
            o.d_ld[0] = op.out.ld;
        } else if (op.kind == 2) {
            o.m[0] = op.tm;
            o.n[0] = op.tn;
            o.a_buf[0] = op.in.buf;
            o.a_off[0] = op.in.off;
            o.a_ld[0] = op.in.ld;
            o.d_buf[0] = op.out.buf;
            o.d_off[0] = op.out.off;
            o.d_ld[0] = op.out.ld;
        } else {
            o.a_buf[0] = op.in.buf;
            o.a_off[0] = op.in.off;
            o.a_ld[0] = op.in.ld;
            o.d_buf[0] = op.out.buf;
            o.d_off[0] = op.out.off;
            o.d_ld[0] = op.out.ld;
            o.leaf_order = op.L;
            o.col0 = op.col0;
        }
        ops[i] = o;
    }
    return cnt;
}

}  // namespace

extern "C" {

int64_t spin_plan_describe(int64_t n, int64_t lda, int64_t ldx, int64_t leaf, spin_plan_op *ops,
                           int64_t cap, double *flops) {
    if (n < 1 || n > SPIN_MAX_N) return SPIN_E_N;
    if (lda < n || ldx < n) return SPIN_E_LD;
    if (leaf < 1 || leaf > SPIN_MAX_LEAF) return SPIN_E_LEAF;
    if (cap > 0 && !ops) return SPIN_E_NULL;
    return describe_plan(make_plan(n, lda, ldx, leaf), ops, cap, flops);
}

int64_t spin_plan_describe_lu(int64_t n, int64_t lda, int64_t ldx, int64_t leaf,
                              spin_plan_op *ops, int64_t cap, double *flops) {
    if (n < 1 || n > SPIN_MAX_N) return SPIN_E_N;
    if (lda < n || ldx < n) return SPIN_E_LD;
    if (leaf < 1 || leaf > kLuLeafMax) return SPIN_E_LEAF;
    if (cap > 0 && !ops) return SPIN_E_NULL;
    return describe_plan(make_plan_lu(n, lda, ldx, leaf), ops, cap, flops);
}

int64_t spin_plan_ws_elems_lu(int64_t n, int64_t leaf) {
    if (n < 1 || n > SPIN_MAX_N || leaf < 1 || leaf > kLuLeafMax) return SPIN_E_N;
    return make_plan_lu(n, n, n, leaf).ws_elems;
}

int64_t spin_plan_describe_spd(int64_t n, int64_t lda, int64_t ldx, int64_t leaf,
                               spin_plan_op *ops, int64_t cap, double *flops) {
    if (n < 1 || n > SPIN_MAX_N) return SPIN_E_N;
    if (lda < n || ldx < n) return SPIN_E_LD;
    if (leaf < 1 || leaf > SPIN_MAX_LEAF) return SPIN_E_LEAF;
    if (cap > 0 && !ops) return SPIN_E_NULL;
    return describe_plan(make_plan_spd(n, lda, ldx, leaf), ops, cap, flops);
}

int64_t spin_plan_ws_elems(int64_t n, int64_t leaf) {
    if (n < 1 || n > SPIN_MAX_N || leaf < 1 || leaf > SPIN_MAX_LEAF) return SPIN_E_N;
    return make_plan(n, n, n, leaf).ws_elems;
}

int spin_trace_enable(int on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_trace_on = on != 0;
    return SPIN_OK;
}

int64_t spin_trace_collect(spin_trace_rec *recs, int64_t cap) {
    std::lock_guard<std::mutex> lk(g_mu);
    const int64_t cnt = (int64_t)g_trace.size();
    for (int64_t i = 0; i < cnt; ++i) {
        TraceRec &t = g_trace[(size_t)i];
        float ms = 0.f;
        hipEventSynchronize(t.stop);
        hipEventElapsedTime(&ms, t.start, t.stop);
        if (recs && i < cap) {
            spin_trace_rec &r = recs[i];
            std::memset(&r, 0, sizeof(r));
            std::snprintf(r.kernel, sizeof(r.kernel), "%s", t.name.c_str());
            r.ms = ms;
            r.flops = t.flops;
            r.bytes = t.bytes;
            r.level = t.level;
        }
        hipEventDestroy(t.start);
        hipEventDestroy(t.stop);
    }
    g_trace.clear();
    return cnt;
}

}  // extern "C"
