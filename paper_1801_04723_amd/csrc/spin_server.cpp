// Batched inversion and continuous-batching server.
//
// Every admitted request owns a private workspace carved from one device
// pool and a list of steps: exactly the kernel launches the single-call path
// makes for it (status reset, precision conversions, the recursion schedule
// of Alg. 1 in S-form, Newton refinement).  A tick takes the next step of
// every active request: block products from all requests go into grouped
// matrix-core launches (one grid per kernel configuration), whole leaves into
// one batched leaf launch, and the small auxiliary kernels (status resets,
// conversions, norms, and any transpose or mirror of the symmetric schedule
// that no product epilogue takes over) run as they come.
// Steps of one request stay in order (one product/leaf step per request per
// tick, all launched on one stream), and every kernel computes each
// product/leaf exactly as it does alone, so a request's result is bit for bit
// the same alone and in the mix.
//
// Admission is FIFO by workspace footprint: a queued request starts when a
// slot is free and its workspace fits in the pool; a request that does not fit
// blocks the ones behind it (no starvation of large requests).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "spin.h"
#include "spin_kernels.hpp"
#include "spin_plan.hpp"

namespace spin {
namespace {

// ---------------------------------------------------------------- pool ----
// First-fit allocator over [0, size) in 256-byte units, coalescing on free.
class PoolAllocator {
  public:
    explicit PoolAllocator(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off) {
        bytes = al256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = al256(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

  private:
    size_t size_;
    size_t used_ = 0;
    std::map<size_t, size_t> free_;
};

// --------------------------------------------------------------- steps ----
enum StepKind { STEP_GEMM = 0, STEP_LEAF = 1, STEP_AUX = 2 };
enum AuxOp { AUX_RESET, AUX_CAST_IN, AUX_WIDEN, AUX_FROB, AUX_NSCHECK, AUX_TRANSPOSE, AUX_MIRROR, AUX_NSFINAL };

// A mode with SPIN_SYMMETRIC runs the symmetric schedule of spin_invert_spd
// with the mode's product flavour.
constexpr int kModeSym = SPIN_FP64 | SPIN_SYMMETRIC;
bool server_mode(int mode) {
    return is_mode(mode) || ((mode & SPIN_SYMMETRIC) && is_mode(mode & ~SPIN_SYMMETRIC));
}
int product_mode(int mode) { return mode & ~SPIN_SYMMETRIC; }

struct Step {
    int kind;
    DType dt;
    int nprob;
    GemmProb prob[2];
    LeafItem leaf;
    void *leaf_scratch;
    int aux;
    const void *src;
    int64_t lds;
    void *dst;
    int64_t ldd;
    int64_t m, n;
    double *norms;
    double *partials;
    int j;
    int *status;
};

struct Request {
    int64_t tag;
    int mode;
    int64_t n, lda, ldx;
    const double *A;
    double *X;
    size_t ws_off = 0, ws_bytes = 0;
    char *ws = nullptr;
    std::vector<Step> steps;
    size_t next = 0;
    bool exch_filled = false;  // the leaf scratch's exchange areas (leaf_launch)
    hipEvent_t done = nullptr;
};

Step aux_step(int op) {
    Step s;
    std::memset(&s, 0, sizeof(s));
    s.kind = STEP_AUX;
    s.aux = op;
    return s;
}

// gdt: product flavour of the plan's products; leaves use its storage type.
// Transposes and mirrors that no product epilogue takes over become auxiliary
// steps (FP64 kernels); in an FP32-storage plan that is an error (false).
bool add_plan_steps(const Plan &P, char *const base[3], size_t es, DType gdt, int *status,
                    void *leaf_scratch, std::vector<Step> &out) {
    for (size_t i = 0; i < P.ops.size(); ++i) {
        const POp &op = P.ops[i];
        Step st;
        std::memset(&st, 0, sizeof(st));
        st.dt = op.kind == 0 ? gdt : storage_type(gdt);
        if (op.kind == 0) {
            st.kind = STEP_GEMM;
            st.nprob = op.count;
            for (int q = 0; q < op.count; ++q) st.prob[q] = make_prob(base, es, op.g[q]);
            // as in the single-call executor: a following mirror or transpose
            // is done by this product's epilogue
            if (fold_next_step(P, i, base, es, st.prob)) ++i;
        } else if (op.kind == 2 || op.kind == 3) {
            if (es != 8) return false;
            st.kind = STEP_AUX;
            st.aux = op.kind == 2 ? AUX_TRANSPOSE : AUX_MIRROR;
            if (op.kind == 2) {
                st.src = base[op.in.buf] + (size_t)op.in.off * es;
                st.lds = op.in.ld;
            }
            st.dst = base[op.out.buf] + (size_t)op.out.off * es;
            st.ldd = op.out.ld;
            st.m = op.tm;
            st.n = op.tn;
        } else {
            st.kind = STEP_LEAF;
            st.leaf = LeafItem{base[op.in.buf] + (size_t)op.in.off * es, op.in.ld,
                               base[op.out.buf] + (size_t)op.out.off * es, op.out.ld, op.L,
                               op.col0, status};
            st.leaf_scratch = leaf_scratch;
        }
        out.push_back(st);
    }
    return true;
}

// The steps of one request: the same launches spin_invert / spin_invert_spd /
// spin_invert_mixed make, in the same order, with the request's own workspace.
bool build_steps(Request &r, int64_t leaf, int ns_steps) {
    const int64_t n = r.n;
    char *w = r.ws;
    int *status = reinterpret_cast<int *>(w);
    double *norms = reinterpret_cast<double *>(w + 256);
    double *parts = reinterpret_cast<double *>(w + 4096);
    Step rs = aux_step(AUX_RESET);
    rs.status = status;
    r.steps.push_back(rs);
    if (r.mode == SPIN_FP64 || r.mode == kModeSym) {
        Plan P = r.mode == kModeSym ? make_plan_spd(n, r.lda, r.ldx, leaf)
                                    : make_plan(n, r.lda, r.ldx, leaf);
        Layout L = layout_for(n, leaf, SPIN_FP64, P.ws_elems, P.max_leaf);
        char *const base[3] = {(char *)r.A, (char *)r.X, w + L.rec_off};
        return add_plan_steps(P, base, 8, kF64, status, w + L.leaf_off, r.steps);
    }
    const int pm = product_mode(r.mode);
    Plan P = (r.mode & SPIN_SYMMETRIC) ? make_plan_spd(n, n, n, leaf) : make_plan(n, n, n, leaf);
    Layout L = layout_for(n, leaf, pm, P.ws_elems, P.max_leaf);
    float *A32 = reinterpret_cast<float *>(w + L.a32_off);
    float *X32 = reinterpret_cast<float *>(w + L.x32_off);
    double *R = reinterpret_cast<double *>(w + L.r_off);
    double *Xalt = reinterpret_cast<double *>(w + L.xalt_off);
    double *buf0 = (ns_steps % 2 == 0) ? r.X : Xalt;
    const int64_t ld0 = (ns_steps % 2 == 0) ? r.ldx : n;
    double *buf1 = (ns_steps % 2 == 0) ? Xalt : r.X;
    const int64_t ld1 = (ns_steps % 2 == 0) ? n : r.ldx;
    Step c = aux_step(AUX_CAST_IN);
    c.src = r.A, c.lds = r.lda, c.dst = A32, c.ldd = n, c.m = n, c.n = n;
    r.steps.push_back(c);
    char *const base[3] = {(char *)A32, (char *)X32, w + L.rec_off};
    if (!add_plan_steps(P, base, 4, mixed_product_type(pm), status, w + L.leaf_off, r.steps))
        return false;
    Step wd = aux_step(AUX_WIDEN);
    wd.src = X32, wd.lds = n, wd.dst = buf0, wd.ldd = ld0, wd.m = n, wd.n = n;
    r.steps.push_back(wd);
    for (int j = 0; j < ns_steps; ++j) {
        double *xc = (j % 2 == 0) ? buf0 : buf1;
        const int64_t ldc = (j % 2 == 0) ? ld0 : ld1;
        double *xn = (j % 2 == 0) ? buf1 : buf0;
        const int64_t ldn = (j % 2 == 0) ? ld1 : ld0;
        Step g;
        std::memset(&g, 0, sizeof(g));
        g.kind = STEP_GEMM;
        g.dt = kF64;
        g.nprob = 1;
        g.prob[0] = GemmProb{r.A, xc, nullptr, R, r.lda, ldc, 1, n, (int32_t)n, (int32_t)n,
                             (int32_t)n, 1, -1.0, 0.0};
        r.steps.push_back(g);
        Step fr = aux_step(AUX_FROB);
        fr.src = R, fr.lds = n, fr.m = n, fr.n = n, fr.norms = norms + j, fr.partials = parts;
        r.steps.push_back(fr);
        Step ck = aux_step(AUX_NSCHECK);
        ck.norms = norms, ck.j = j, ck.status = status + 1;
        r.steps.push_back(ck);
        Step u;
        std::memset(&u, 0, sizeof(u));
        u.kind = STEP_GEMM;
        u.dt = kF64;
        u.nprob = 1;
        u.prob[0] = GemmProb{xc, R, xc, xn, ldc, n, ldc, ldn, (int32_t)n, (int32_t)n, (int32_t)n,
                             0, 1.0, 1.0};
        r.steps.push_back(u);
    }
    if (ns_steps > 0) {
        // acceptance of the refined inverse (now in X), as in spin_invert_mixed
        double *misc = norms + kNormSlots;
        Step g;
        std::memset(&g, 0, sizeof(g));
        g.kind = STEP_GEMM;
        g.dt = kF64;
        g.nprob = 1;
        g.prob[0] = GemmProb{r.A, r.X, nullptr, R, r.lda, r.ldx, 1, n, (int32_t)n, (int32_t)n,
                             (int32_t)n, 1, -1.0, 0.0};
        r.steps.push_back(g);
        const double *src[3] = {R, r.A, r.X};
        const int64_t ld[3] = {n, r.lda, r.ldx};
        const int slot[3] = {2, 0, 3};
        for (int q = 0; q < 3; ++q) {
            Step fr = aux_step(AUX_FROB);
            fr.src = src[q], fr.lds = ld[q], fr.m = n, fr.n = n, fr.norms = misc + slot[q];
            fr.partials = parts;
            r.steps.push_back(fr);
        }
        Step fin = aux_step(AUX_NSFINAL);
        fin.norms = misc, fin.status = status + 1;
        r.steps.push_back(fin);
    }
    return true;
}

hipError_t run_aux(const Step &s, hipStream_t st) {
    switch (s.aux) {
    case AUX_RESET: return status_reset(s.status, leaf_spec_enabled(), st);
    case AUX_CAST_IN:
        return cast_f64_to_f32(static_cast<const double *>(s.src), s.lds, static_cast<float *>(s.dst),
                               s.ldd, s.m, s.n, st);
    case AUX_WIDEN:
        return cast_f32_to_f64(static_cast<const float *>(s.src), s.lds, static_cast<double *>(s.dst),
                               s.ldd, s.m, s.n, st);
    case AUX_FROB:
        return frob2(static_cast<const double *>(s.src), s.lds, s.m, s.n, s.partials, s.norms, st);
    case AUX_NSCHECK: return ns_check(s.norms, s.j, s.status, st);
    case AUX_NSFINAL: return ns_final(s.norms + 2, s.norms + 0, s.norms + 3, kNsTol, s.status, st);
    case AUX_TRANSPOSE:
        return transpose_f64(static_cast<const double *>(s.src), s.lds, static_cast<double *>(s.dst),
                             s.ldd, s.m, s.n, st);
    case AUX_MIRROR: return mirror_lower_f64(static_cast<double *>(s.dst), s.ldd, s.m, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace
}  // namespace spin

using namespace spin;

struct spin_server {
    size_t pool_bytes;
    int max_active;
    int64_t leaf;
    int ns_steps;
    char *pool = nullptr;
    PoolAllocator alloc;
    std::deque<Request *> queue;
    std::vector<Request *> active;  // admission order
    std::vector<std::pair<int64_t, int>> completed;
    // private non-blocking stream for reading finished requests' status
    // words: a copy there waits for nothing but itself
    hipStream_t poll_stream = nullptr;
    spin_server(size_t b, int m, int64_t l, int s)
        : pool_bytes(b), max_active(m), leaf(l), ns_steps(s), alloc(b) {}
};

namespace {

// A symmetric request on FP32 storage needs every mirror and transpose folded.
bool schedule_ok(int64_t n, int64_t leaf, int mode) {
    if (!(mode & SPIN_SYMMETRIC) || product_mode(mode) == SPIN_FP64) return true;
    return plan_folds_all(make_plan_spd(n, n, n, leaf));
}

size_t request_bytes(int64_t n, int64_t leaf, int mode) {
    Plan P = (mode & SPIN_SYMMETRIC) ? make_plan_spd(n, n, n, leaf) : make_plan(n, n, n, leaf);
    return layout_for(n, leaf, product_mode(mode), P.ws_elems, P.max_leaf).total;
}

int hipfail(hipError_t e) {
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? SPIN_E_NOMEM : SPIN_E_HIP;
}

int admit(spin_server *s) {
    int admitted = 0;
    while (!s->queue.empty() && (int)s->active.size() < s->max_active) {
        Request *r = s->queue.front();
        size_t off = 0;
        if (!s->alloc.alloc(r->ws_bytes, &off)) break;  // FIFO: wait for space
        r->ws_off = off;
        r->ws = s->pool ? s->pool + off : nullptr;
        s->queue.pop_front();
        s->active.push_back(r);
        ++admitted;
    }
    return admitted;
}

}  // namespace

extern "C" {

spin_server *spin_server_create(size_t pool_bytes, int max_active, int64_t leaf, int ns_steps) {
    if (pool_bytes == 0 || max_active < 1 || leaf < 1 || leaf > SPIN_MAX_LEAF || ns_steps < 0 ||
        ns_steps > kNormSlots)
        return nullptr;
    return new (std::nothrow) spin_server(pool_bytes, max_active, leaf, ns_steps);
}

void spin_server_destroy(spin_server *s) {
    if (!s) return;
    if (s->pool) {
        hipDeviceSynchronize();
        hipFree(s->pool);
    }
    if (s->poll_stream) hipStreamDestroy(s->poll_stream);
    for (Request *r : s->active) {
        if (r->done) hipEventDestroy(r->done);
        delete r;
    }
    for (Request *r : s->queue) delete r;
    delete s;
}

int spin_server_submit(spin_server *s, const double *A, int64_t n, int64_t lda, double *Ainv,
                       int64_t ldx, int mode, int64_t tag) {
    if (!s || !A || !Ainv) return SPIN_E_NULL;
    if (n < 1 || n > SPIN_MAX_N) return SPIN_E_N;
    if (lda < n || ldx < n) return SPIN_E_LD;
    if (!server_mode(mode) || !schedule_ok(n, s->leaf, mode)) return SPIN_E_MODE;
    const char *a0 = reinterpret_cast<const char *>(A), *x0 = reinterpret_cast<const char *>(Ainv);
    const char *a1 = a0 + ((size_t)(n - 1) * lda + n) * 8, *x1 = x0 + ((size_t)(n - 1) * ldx + n) * 8;
    if (a0 < x1 && x0 < a1) return SPIN_E_ALIAS;
    const size_t bytes = request_bytes(n, s->leaf, mode);
    if (bytes > s->pool_bytes) return SPIN_E_NOMEM;  // could never be admitted
    Request *r = new (std::nothrow) Request();
    if (!r) return SPIN_E_NOMEM;
    r->tag = tag;
    r->mode = mode;
    r->n = n;
    r->lda = lda;
    r->ldx = ldx;
    r->A = A;
    r->X = Ainv;
    r->ws_bytes = bytes;
    s->queue.push_back(r);
    return SPIN_OK;
}

int spin_server_admit(spin_server *s) {
    if (!s) return SPIN_E_NULL;
    return admit(s);
}

int spin_server_tick(spin_server *s, spin_stream_t stream) {
    if (!s) return SPIN_E_NULL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (!s->pool) {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, s->pool_bytes);
        if (e != hipSuccess || !p) return hipfail(e);
        s->pool = static_cast<char *>(p);
        for (Request *r : s->active) r->ws = s->pool + r->ws_off;
    }
    admit(s);
    std::vector<GemmProb> g[4];  // by product flavour (DType)
    std::vector<LeafItem> lf[2];  // by storage type
    std::vector<Request *> finished;
    hipError_t e = hipSuccess;
    for (Request *r : s->active) {
        if (r->done) continue;  // all steps launched, waiting for completion
        // submit checked that the request's schedule builds
        if (r->steps.empty() && !build_steps(*r, s->leaf, s->ns_steps)) {
            e = hipErrorInvalidValue;
            break;
        }
        // leading auxiliary steps run now; then one product/leaf step joins the groups
        while (r->next < r->steps.size() && e == hipSuccess) {
            const Step &stp = r->steps[r->next];
            if (stp.kind == STEP_AUX) {
                e = run_aux(stp, st);
                ++r->next;
                continue;
            }
            if (stp.kind == STEP_GEMM) {
                for (int q = 0; q < stp.nprob; ++q) g[(int)stp.dt].push_back(stp.prob[q]);
            } else if (stp.leaf.L <= 128) {
                lf[stp.dt == kF64 ? 0 : 1].push_back(stp.leaf);
            } else {
                e = leaf_launch(stp.leaf.in, stp.dt, stp.leaf.ldi, stp.leaf.out, stp.dt,
                                stp.leaf.ldo, stp.leaf.L, stp.leaf.col0, stp.leaf.status,
                                stp.leaf_scratch, r->exch_filled, st, nullptr, nullptr);
                if (e == hipSuccess && leaf_fills_exchange(stp.leaf.L)) r->exch_filled = true;
            }
            ++r->next;
            break;
        }
        if (r->next >= r->steps.size()) finished.push_back(r);
    }
    for (int d = 0; d < 4 && e == hipSuccess; ++d) {
        for (size_t i = 0; i < g[d].size() && e == hipSuccess; i += kMaxBatch) {
            const int cnt = (int)std::min<size_t>(kMaxBatch, g[d].size() - i);
            e = gemm_launch(g[d].data() + i, cnt, (DType)d, st, nullptr);
        }
        if (d >= 2) continue;
        for (size_t i = 0; i < lf[d].size() && e == hipSuccess; i += kMaxLeafBatch) {
            const int cnt = (int)std::min<size_t>(kMaxLeafBatch, lf[d].size() - i);
            e = leaf_batch_launch(lf[d].data() + i, cnt, d == 0 ? kF64 : kF32, st, nullptr);
        }
    }
    for (Request *r : finished) {
        if (e != hipSuccess) break;
        e = hipEventCreateWithFlags(&r->done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(r->done, st);
    }
    if (e != hipSuccess) return hipfail(e);
    return (int)s->active.size();
}

int64_t spin_server_poll(spin_server *s, int64_t *tags, int *info, int64_t cap) {
    if (!s) return SPIN_E_NULL;
    for (auto it = s->active.begin(); it != s->active.end();) {
        Request *r = *it;
        if (r->done && hipEventQuery(r->done) == hipSuccess) {
            if (!s->poll_stream &&
                hipStreamCreateWithFlags(&s->poll_stream, hipStreamNonBlocking) != hipSuccess) {
                s->poll_stream = nullptr;
                return hipfail(hipErrorUnknown);
            }
            int h[2] = {INT_MAX, INT_MAX};
            hipError_t e = hipMemcpyAsync(h, r->ws, sizeof(h), hipMemcpyDeviceToHost, s->poll_stream);
            if (e == hipSuccess) e = hipStreamSynchronize(s->poll_stream);
            const int code = (e != hipSuccess)  ? SPIN_E_HIP
                             : (h[0] != INT_MAX) ? h[0]
                             : (h[1] != INT_MAX) ? h[1]
                                                 : 0;
            s->completed.emplace_back(r->tag, code);
            hipEventDestroy(r->done);
            s->alloc.release(r->ws_off, r->ws_bytes);
            delete r;
            it = s->active.erase(it);
        } else {
            ++it;
        }
    }
    const int64_t cnt = std::min<int64_t>(cap, (int64_t)s->completed.size());
    for (int64_t i = 0; i < cnt; ++i) {
        if (tags) tags[i] = s->completed[(size_t)i].first;
        if (info) info[i] = s->completed[(size_t)i].second;
    }
    s->completed.erase(s->completed.begin(), s->completed.begin() + cnt);
    return cnt;
}

int spin_server_stats(spin_server *s, int64_t *queued, int64_t *active, size_t *pool_used) {
    if (!s) return SPIN_E_NULL;
    if (queued) *queued = (int64_t)s->queue.size();
    if (active) *active = (int64_t)s->active.size();
    if (pool_used) *pool_used = s->alloc.used();
    return SPIN_OK;
}

size_t spin_server_request_bytes(int64_t n, int64_t leaf, int mode) {
    if (n < 1 || n > SPIN_MAX_N || leaf < 1 || leaf > SPIN_MAX_LEAF) return 0;
    if (!server_mode(mode) || !schedule_ok(n, leaf, mode)) return 0;
    return al256(request_bytes(n, leaf, mode));
}

int spin_invert_batch(int64_t count, const double *const *A, const int64_t *n, const int64_t *lda,
                      double *const *Ainv, const int64_t *ldx, const int *mode, int64_t leaf,
                      int ns_steps, int *info, spin_stream_t stream) {
    if (count < 0 || count > SPIN_MAX_BATCH) return SPIN_E_COUNT;
    if (count == 0) return SPIN_OK;
    if (!A || !n || !lda || !Ainv || !ldx || !mode) return SPIN_E_NULL;
    if (leaf < 1 || leaf > SPIN_MAX_LEAF) return SPIN_E_LEAF;
    if (ns_steps < 0 || ns_steps > kNormSlots) return SPIN_E_MODE;
    size_t total = 0;
    for (int64_t i = 0; i < count; ++i) {
        if (n[i] < 1 || n[i] > SPIN_MAX_N) return SPIN_E_N;
        if (!server_mode(mode[i]) || !schedule_ok(n[i], leaf, mode[i])) return SPIN_E_MODE;
        total += al256(request_bytes(n[i], leaf, mode[i]));
    }
    spin_server *s = spin_server_create(total, (int)count, leaf, ns_steps);
    if (!s) return SPIN_E_NOMEM;
    int rc = SPIN_OK;
    for (int64_t i = 0; i < count && rc == SPIN_OK; ++i)
        rc = spin_server_submit(s, A[i], n[i], lda[i], Ainv[i], ldx[i], mode[i], i);
    while (rc == SPIN_OK) {
        const int act = spin_server_tick(s, stream);
        if (act < 0) {
            rc = act;
            break;
        }
        bool pending = !s->queue.empty();
        for (Request *r : s->active) pending |= (r->done == nullptr);
        if (!pending) break;
    }
    if (rc == SPIN_OK) {
        if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
            rc = SPIN_E_HIP;
    }
    if (rc == SPIN_OK) {
        std::vector<int64_t> tags((size_t)count);
        std::vector<int> codes((size_t)count);
        int64_t got = 0;
        while (got < count) {
            const int64_t c = spin_server_poll(s, tags.data() + got, codes.data() + got, count - got);
            if (c <= 0) break;
            got += c;
        }
        if (info)
            for (int64_t i = 0; i < got; ++i) info[tags[(size_t)i]] = codes[(size_t)i];
    }
    spin_server_destroy(s);
    return rc;
}

}  // extern "C"
