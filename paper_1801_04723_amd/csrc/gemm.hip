// Block products of the recursion on gfx950 matrix cores.
//
//   D = alpha * A * B + beta * C0 (+ I on the diagonal)        column-major views
//
// This is the paper's `multiply` (Sec. 3.3) with the `subtract` steps of
// Alg. 2 (V = IV - A22, C11 = I - VII) and the sign of `scalarMul` folded into
// the epilogue: the scheduler forms S = A22 - A21*III (alpha = -1, beta = 1),
// C12 = -III*C22 and C21 = -C22*II (alpha = -1), C11 = C11 - III*C21 in place
// (alpha = -1, beta = 1, C0 == D), and the Newton residual R = I - A*X
// (alpha = -1, add_identity).
//
// Kernel shape: 256 threads = 4 wave64s; a BM x BN output tile per workgroup,
// split 2 x 2 into WM x WN wave tiles of 16 x 16 MFMA blocks.  K advances in
// BK slabs staged global -> registers -> LDS with two LDS buffers, so the
// global loads of slab k+1 are in flight while the matrix cores consume
// slab k, with one barrier per slab.
//
// Matrix-core operands are issued transposed (B^T tile as the first operand,
// A^T tile as the second), so each accumulator holds a 16 x 16 block of D^T:
// lane l owns output row m = l % 16, which makes the epilogue's stores
// contiguous down each column of the column-major result.
//   v_mfma_f64_16x16x4f64 : lane l, element v  ->  D^T row 4*v + l/16
//   v_mfma_f32_16x16x4f32 : lane l, element v  ->  D^T row 4*(l/16) + v
#include <hip/hip_runtime.h>

#include "spin_kernels.hpp"

namespace spin {
namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T>
struct Mma;

template <>
struct Mma<double> {
    using acc_t = d4_t;
    __device__ static inline acc_t mma(double bt, double at, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(bt, at, c, 0, 0, 0);
    }
    __device__ static inline int ncol(int lane, int v) { return 4 * v + (lane >> 4); }
};

template <>
struct Mma<float> {
    using acc_t = f4_t;
    __device__ static inline acc_t mma(float bt, float at, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(bt, at, c, 0, 0, 0);
    }
    __device__ static inline int ncol(int lane, int v) { return 4 * (lane >> 4) + v; }
};

struct GroupArgs {
    GemmProb p[kMaxGroup];
    int32_t count;
    int32_t tile_start[kMaxGroup + 1];
    int32_t tiles_m[kMaxGroup];
};

template <int BM, int BN, int BK, int WM, int WN, typename T>
__global__ void __launch_bounds__(256) gemm_kernel(GroupArgs g) {
    constexpr int NT = 256;
    constexpr int WAVES_M = BM / WM;
    static_assert(WAVES_M * (BN / WN) == 4, "four waves per workgroup");
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int A_LD = BM + 1;  // LDS pitch of an A slab row (one k)
    constexpr int B_LD = BN + 1;  // LDS pitch of a B slab row (one k); +1 spreads banks
    constexpr int A_PT = BM * BK / NT;
    constexpr int B_PT = BN * BK / NT;
    static_assert(A_PT * NT == BM * BK && B_PT * NT == BN * BK, "tile/thread mismatch");
    using acc_t = typename Mma<T>::acc_t;

    __shared__ T As[2][BK * A_LD];
    __shared__ T Bs[2][BK * B_LD];

    // ---- which problem of the group and which tile --------------------------
    const int bid = blockIdx.x;
    int pi = 0;
#pragma unroll
    for (int q = 1; q < kMaxGroup; ++q)
        if (q < g.count && bid >= g.tile_start[q]) pi = q;
    GemmProb P = g.p[0];
    int tstart = g.tile_start[0], tiles_m = g.tiles_m[0];
#pragma unroll
    for (int q = 1; q < kMaxGroup; ++q)
        if (pi == q) {
            P = g.p[q];
            tstart = g.tile_start[q];
            tiles_m = g.tiles_m[q];
        }
    const int t = bid - tstart;
    const int tm = t % tiles_m, tn = t / tiles_m;

    const int M = P.m, N = P.n, K = P.k;
    const int m0 = tm * BM, n0 = tn * BN;
    const T *__restrict__ A = static_cast<const T *>(P.A);
    const T *__restrict__ B = static_cast<const T *>(P.B);
    const int64_t lda = P.lda, ldb = P.ldb;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % WAVES_M) * WM, wn0 = (wave / WAVES_M) * WN;

    T ra[A_PT], rb[B_PT];
    auto gload = [&](int k0) {
        const bool full = (m0 + BM <= M) && (n0 + BN <= N) && (k0 + BK <= K);
        if (full) {
#pragma unroll
            for (int i = 0; i < A_PT; ++i) {
                const int e = tid + NT * i, r = e % BM, c = e / BM;
                ra[i] = A[(m0 + r) + (int64_t)(k0 + c) * lda];
            }
#pragma unroll
            for (int i = 0; i < B_PT; ++i) {
                const int e = tid + NT * i, r = e % BK, c = e / BK;
                rb[i] = B[(k0 + r) + (int64_t)(n0 + c) * ldb];
            }
        } else {
#pragma unroll
            for (int i = 0; i < A_PT; ++i) {
                const int e = tid + NT * i, r = e % BM, c = e / BM;
                const bool ok = (m0 + r < M) && (k0 + c < K);
                ra[i] = ok ? A[(m0 + r) + (int64_t)(k0 + c) * lda] : T(0);
            }
#pragma unroll
            for (int i = 0; i < B_PT; ++i) {
                const int e = tid + NT * i, r = e % BK, c = e / BK;
                const bool ok = (k0 + r < K) && (n0 + c < N);
                rb[i] = ok ? B[(k0 + r) + (int64_t)(n0 + c) * ldb] : T(0);
            }
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < A_PT; ++i) {
            const int e = tid + NT * i, r = e % BM, c = e / BM;
            As[buf][c * A_LD + r] = ra[i];
        }
#pragma unroll
        for (int i = 0; i < B_PT; ++i) {
            const int e = tid + NT * i, r = e % BK, c = e / BK;
            Bs[buf][r * B_LD + c] = rb[i];
        }
    };

    acc_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    const int KT = (K + BK - 1) / BK;
    if (KT > 0) {
        gload(0);
        sstore(0);
    }
    __syncthreads();
    const int krow = lane >> 4, kcol = lane & 15;
    for (int kt = 0; kt < KT; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < KT) gload((kt + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            T a[TM], b[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = As[cur][(kk * 4 + krow) * A_LD + wm0 + i * 16 + kcol];
#pragma unroll
            for (int j = 0; j < TN; ++j) b[j] = Bs[cur][(kk * 4 + krow) * B_LD + wn0 + j * 16 + kcol];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = Mma<T>::mma(b[j], a[i], acc[i][j]);
        }
        if (kt + 1 < KT) sstore(cur ^ 1);
        __syncthreads();
    }

    // ---- epilogue: D = alpha * acc + beta * C0 (+ I) ------------------------
    const T *__restrict__ C0 = static_cast<const T *>(P.C0);
    T *D = static_cast<T *>(P.D);
    const double alpha = P.alpha, beta = P.beta;
    const bool use_c = (beta != 0.0) && (C0 != nullptr);
    const bool add_i = P.add_identity != 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int gm = m0 + wm0 + i * 16 + kcol;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gn = n0 + wn0 + j * 16 + Mma<T>::ncol(lane, v);
                if (gm < M && gn < N) {
                    double val = alpha * (double)acc[i][j][v];
                    if (use_c) val += beta * (double)C0[gm + (int64_t)gn * P.ldc];
                    if (add_i && gm == gn) val += 1.0;
                    D[gm + (int64_t)gn * P.ldd] = (T)val;
                }
            }
        }
    }
}

// Fast path.  Requires 16-byte aligned operands, leading dimensions that are
// multiples of the vector width, M a multiple of the vector width and K a
// multiple of BK -- true for every block product of the recursion when the
// order is a multiple of 64.  The main loop then has no control flow: the
// edge rows/columns of a tile are clamped once and masked, each thread keeps
// one pointer per 16-byte global load and advances it by one slab per step.
//
// The K slab is split into four contiguous chunks of KQ = BK/4 values, one per
// lane group q = lane/16, and MFMA step kk consumes k = q*KQ + kk in group q
// (any assignment of k to the four MFMA k-slots is valid as long as A and B
// agree).  B is staged k-contiguous (Bs[n][k]) so that a lane fetches its KQ
// B values with 16-byte LDS reads; A is staged m-contiguous (As[k][m]).
template <int BM, int BN, int BK, int WM, int WN, typename T>
__global__ void __launch_bounds__(256, 2) gemm_fast(GroupArgs g) {
    constexpr int NT = 256;
    constexpr int VW = 16 / sizeof(T);
    typedef T vec_t __attribute__((ext_vector_type(VW)));
    constexpr int WAVES_M = BM / WM;
    static_assert(WAVES_M * (BN / WN) == 4, "four waves per workgroup");
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int KQ = BK / 4;
    static_assert(KQ % VW == 0, "lane chunk must be whole vectors");
    constexpr int A_LD = BM + VW;  // As[k][m]
    constexpr int B_LD = BK + VW;  // Bs[n][k]
    constexpr int AV = BM * BK / VW / NT;
    constexpr int BV = BN * BK / VW / NT;
    static_assert(AV * VW * NT == BM * BK && BV * VW * NT == BN * BK, "tile/thread mismatch");
    using acc_t = typename Mma<T>::acc_t;

    __shared__ __attribute__((aligned(16))) T As[2][BK * A_LD];
    __shared__ __attribute__((aligned(16))) T Bs[2][BN * B_LD];

    const int bid = blockIdx.x;
    int pi = 0;
#pragma unroll
    for (int q = 1; q < kMaxGroup; ++q)
        if (q < g.count && bid >= g.tile_start[q]) pi = q;
    GemmProb P = g.p[0];
    int tstart = g.tile_start[0], tiles_m = g.tiles_m[0];
#pragma unroll
    for (int q = 1; q < kMaxGroup; ++q)
        if (pi == q) {
            P = g.p[q];
            tstart = g.tile_start[q];
            tiles_m = g.tiles_m[q];
        }
    const int t = bid - tstart;
    const int tm = t % tiles_m, tn = t / tiles_m;
    const int M = P.m, N = P.n, K = P.k;
    const int m0 = tm * BM, n0 = tn * BN;
    const int64_t lda = P.lda, ldb = P.ldb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % WAVES_M) * WM, wn0 = (wave / WAVES_M) * WN;

    const T *pa[AV];
    bool am[AV];
    int sa[AV];
#pragma unroll
    for (int i = 0; i < AV; ++i) {
        const int v = tid + NT * i, r = (v % (BM / VW)) * VW, c = v / (BM / VW);
        am[i] = m0 + r < M;
        const int row = am[i] ? m0 + r : M - VW;
        pa[i] = static_cast<const T *>(P.A) + row + (int64_t)c * lda;
        sa[i] = c * A_LD + r;
    }
    const T *pb[BV];
    bool bm[BV];
    int sb[BV];
#pragma unroll
    for (int i = 0; i < BV; ++i) {
        const int v = tid + NT * i, k = (v % (BK / VW)) * VW, n = v / (BK / VW);
        bm[i] = n0 + n < N;
        const int col = bm[i] ? n0 + n : N - 1;
        pb[i] = static_cast<const T *>(P.B) + k + (int64_t)col * ldb;
        sb[i] = n * B_LD + k;
    }
    const int64_t astep = (int64_t)BK * lda;

    vec_t ra[AV], rb[BV];
    auto gload = [&]() {
#pragma unroll
        for (int i = 0; i < AV; ++i) {
            const vec_t x = *reinterpret_cast<const vec_t *>(pa[i]);
            ra[i] = am[i] ? x : vec_t(0);
            pa[i] += astep;
        }
#pragma unroll
        for (int i = 0; i < BV; ++i) {
            const vec_t x = *reinterpret_cast<const vec_t *>(pb[i]);
            rb[i] = bm[i] ? x : vec_t(0);
            pb[i] += BK;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < AV; ++i) *reinterpret_cast<vec_t *>(&As[buf][sa[i]]) = ra[i];
#pragma unroll
        for (int i = 0; i < BV; ++i) *reinterpret_cast<vec_t *>(&Bs[buf][sb[i]]) = rb[i];
    };

    acc_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    const int q = lane >> 4, c16 = lane & 15;
    auto compute = [&](int buf) {
        const T *as = &As[buf][(q * KQ) * A_LD + wm0 + c16];
        const T *bs = &Bs[buf][(wn0 + c16) * B_LD + q * KQ];
        vec_t bv[TN][KQ / VW];
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int h = 0; h < KQ / VW; ++h)
                bv[j][h] = *reinterpret_cast<const vec_t *>(bs + j * 16 * B_LD + h * VW);
#pragma unroll
        for (int kk = 0; kk < KQ; ++kk) {
            T a[TM];
#pragma unroll
            for (int i = 0; i < TM; ++i) a[i] = as[kk * A_LD + i * 16];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = Mma<T>::mma(bv[j][kk / VW][kk % VW], a[i], acc[i][j]);
        }
    };

    const int KT = K / BK;
    if (KT > 0) {
        gload();
        sstore(0);
        __syncthreads();
        for (int kt = 0; kt + 1 < KT; ++kt) {
            gload();
            compute(kt & 1);
            sstore((kt & 1) ^ 1);
            __syncthreads();
        }
        compute((KT - 1) & 1);
    }

    const T *__restrict__ C0 = static_cast<const T *>(P.C0);
    T *D = static_cast<T *>(P.D);
    const double alpha = P.alpha, beta = P.beta;
    const bool use_c = (beta != 0.0) && (C0 != nullptr);
    const bool add_i = P.add_identity != 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int gm = m0 + wm0 + i * 16 + c16;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gn = n0 + wn0 + j * 16 + Mma<T>::ncol(lane, v);
                if (gm < M && gn < N) {
                    double val = alpha * (double)acc[i][j][v];
                    if (use_c) val += beta * (double)C0[gm + (int64_t)gn * P.ldc];
                    if (add_i && gm == gn) val += 1.0;
                    D[gm + (int64_t)gn * P.ldd] = (T)val;
                }
            }
        }
    }
}

template <int BM, int BN, int BK, int WM, int WN, typename T>
hipError_t launch_cfg(const GemmProb *probs, int count, hipStream_t s) {
    GroupArgs g{};
    g.count = count;
    int total = 0;
    for (int q = 0; q < kMaxGroup; ++q) {
        if (q < count) {
            g.p[q] = probs[q];
            const int tm = (probs[q].m + BM - 1) / BM, tn = (probs[q].n + BN - 1) / BN;
            g.tile_start[q] = total;
            g.tiles_m[q] = tm > 0 ? tm : 1;
            total += tm * tn;
        } else {
            g.p[q] = probs[0];
            g.tile_start[q] = 1 << 30;
            g.tiles_m[q] = 1;
        }
    }
    g.tile_start[kMaxGroup] = total;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL((gemm_kernel<BM, BN, BK, WM, WN, T>), dim3(total), dim3(256), 0, s, g);
    return hipGetLastError();
}

int64_t tiles_for(const GemmProb *probs, int count, int bm, int bn) {
    int64_t t = 0;
    for (int q = 0; q < count; ++q)
        t += (int64_t)((probs[q].m + bm - 1) / bm) * ((probs[q].n + bn - 1) / bn);
    return t;
}


constexpr int kFastBK128 = 16;

// Conditions of the fast path for every product of a launch.
bool fast_ok(const GemmProb *probs, int count, int vw, int bk) {
    for (int q = 0; q < count; ++q) {
        const GemmProb &p = probs[q];
        if (p.k <= 0 || p.k % bk != 0 || p.m % vw != 0) return false;
        if (p.lda % vw != 0 || p.ldb % vw != 0) return false;
        if ((reinterpret_cast<uintptr_t>(p.A) | reinterpret_cast<uintptr_t>(p.B)) & 15) return false;
    }
    return true;
}

template <int BM, int BN, int BK, int WM, int WN, typename T>
hipError_t launch_fast(const GemmProb *probs, int count, hipStream_t s) {
    GroupArgs g{};
    g.count = count;
    int total = 0;
    for (int q = 0; q < kMaxGroup; ++q) {
        if (q < count) {
            g.p[q] = probs[q];
            const int tm = (probs[q].m + BM - 1) / BM, tn = (probs[q].n + BN - 1) / BN;
            g.tile_start[q] = total;
            g.tiles_m[q] = tm > 0 ? tm : 1;
            total += tm * tn;
        } else {
            g.p[q] = probs[0];
            g.tile_start[q] = 1 << 30;
            g.tiles_m[q] = 1;
        }
    }
    g.tile_start[kMaxGroup] = total;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL((gemm_fast<BM, BN, BK, WM, WN, T>), dim3(total), dim3(256), 0, s, g);
    return hipGetLastError();
}

}  // namespace

hipError_t gemm_launch(const GemmProb *probs, int count, DType dt, hipStream_t s, LaunchInfo *info) {
    if (count < 1 || count > kMaxGroup) return hipErrorInvalidValue;
    // Products with an empty reduction still need their epilogue; drop only
    // products with an empty output.
    GemmProb live[kMaxGroup];
    int n_live = 0;
    double flops = 0, bytes = 0;
    const double es = (dt == kF64) ? 8.0 : 4.0;
    for (int q = 0; q < count; ++q) {
        if (probs[q].m <= 0 || probs[q].n <= 0) continue;
        live[n_live++] = probs[q];
        const double m = probs[q].m, n = probs[q].n, k = probs[q].k;
        flops += 2.0 * m * n * k;
        bytes += es * (m * k + k * n + m * n + ((probs[q].beta != 0.0) ? m * n : 0.0));
    }
    // Largest tile that still gives every compute unit work; small problems
    // fall back to smaller tiles so that more workgroups run concurrently.
    const int64_t t128 = tiles_for(live, n_live, 128, 128);
    const int64_t t64 = tiles_for(live, n_live, 64, 64);
    const int tile = (t128 >= 256) ? 128 : (t64 >= 256) ? 64 : 32;
    const int bk = (tile == 128) ? kFastBK128 : 32;
    const bool fast = n_live > 0 && fast_ok(live, n_live, dt == kF64 ? 2 : 4, bk);
    const char *name = "gemm_empty";
    hipError_t e = hipSuccess;
    if (n_live > 0) {
        if (dt == kF64) {
            if (tile == 128) {
                name = fast ? "gemm_f64_128x128" : "gemm_f64_128x128_edge";
                e = fast ? launch_fast<128, 128, kFastBK128, 64, 64, double>(live, n_live, s)
                         : launch_cfg<128, 128, 16, 64, 64, double>(live, n_live, s);
            } else if (tile == 64) {
                name = fast ? "gemm_f64_64x64" : "gemm_f64_64x64_edge";
                e = fast ? launch_fast<64, 64, 32, 32, 32, double>(live, n_live, s)
                         : launch_cfg<64, 64, 16, 32, 32, double>(live, n_live, s);
            } else {
                name = fast ? "gemm_f64_32x32" : "gemm_f64_32x32_edge";
                e = fast ? launch_fast<32, 32, 32, 16, 16, double>(live, n_live, s)
                         : launch_cfg<32, 32, 32, 16, 16, double>(live, n_live, s);
            }
        } else {
            if (tile == 128) {
                name = fast ? "gemm_f32_128x128" : "gemm_f32_128x128_edge";
                e = fast ? launch_fast<128, 128, 32, 64, 64, float>(live, n_live, s)
                         : launch_cfg<128, 128, 16, 64, 64, float>(live, n_live, s);
            } else if (tile == 64) {
                name = fast ? "gemm_f32_64x64" : "gemm_f32_64x64_edge";
                e = fast ? launch_fast<64, 64, 32, 32, 32, float>(live, n_live, s)
                         : launch_cfg<64, 64, 16, 32, 32, float>(live, n_live, s);
            } else {
                name = fast ? "gemm_f32_32x32" : "gemm_f32_32x32_edge";
                e = fast ? launch_fast<32, 32, 32, 16, 16, float>(live, n_live, s)
                         : launch_cfg<32, 32, 32, 16, 16, float>(live, n_live, s);
            }
        }
    }
    if (info) {
        info->name = name;
        info->flops = flops;
        info->bytes = bytes;
    }
    return e;
}

}  // namespace spin
