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

// Up to N independent products in one grid: workgroup b belongs to the
// problem whose tile range [tile_start[q], tile_start[q+1]) contains b.
template <int N>
struct GroupArgs {
    GemmProb p[N];
    int32_t count;
    int32_t tile_start[N + 1];
    int32_t tiles_m[N];
};
static_assert(sizeof(GroupArgs<kMaxBatch>) <= 4096, "kernel arguments above 4 KiB");

// Problem of workgroup `bid` (uniform scan over the prefix sums).
template <int N>
__device__ inline int group_member(const GroupArgs<N> &g, int bid) {
    int pi = 0;
#pragma unroll
    for (int q = 1; q < N; ++q)
        if (q < g.count && bid >= g.tile_start[q]) pi = q;
    return pi;
}

// Tile (tm, tn) of the t-th workgroup of a problem with tiles_m x tiles_n
// tiles whose range starts at workgroup tstart. Workgroups are dealt to the
// eight XCDs round-robin (workgroup b runs on XCD b mod 8), and each XCD has
// its own L2: when the range and both tile counts are multiples of 8, XCD x
// gets the contiguous stretch [x T/8, (x+1) T/8) of an order made of 8 x 8
// tile blocks, so the A rows and B columns it reads stay in its own L2.
// Otherwise tiles go in plain column-major order. A lower-triangle problem
// (square tile grid) has only the T (T + 1) / 2 tiles on or below the
// diagonal, row by row: row r holds (r, 0) ... (r, r).  Every tile is
// computed exactly once, with the same arithmetic, whatever the order.
__device__ inline void tile_coords(int t, int tstart, int tiles_m, int tiles_n, bool lower, int &tm,
                                   int &tn) {
    if (lower) {
        int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while (r * (r + 1) / 2 > t) --r;
        while ((r + 1) * (r + 2) / 2 <= t) ++r;
        tm = r;
        tn = t - r * (r + 1) / 2;
        return;
    }
    if ((tstart & 7) == 0 && (tiles_m & 7) == 0 && (tiles_n & 7) == 0) {
        const int u = (t & 7) * ((tiles_m * tiles_n) >> 3) + (t >> 3);
        const int blk = u >> 6, in = u & 63;
        const int bms = tiles_m >> 3;
        tm = (blk % bms) * 8 + (in & 7);
        tn = (blk / bms) * 8 + (in >> 3);
    } else {
        tm = t % tiles_m;
        tn = t / tiles_m;
    }
}

template <int BM, int BN, int BK, int WM, int WN, typename T, int NG>
__global__ void __launch_bounds__(256) gemm_kernel(GroupArgs<NG> g) {
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

    const int bid = blockIdx.x;
    const int pi = group_member(g, bid);
    const GemmProb P = g.p[pi];
    const int tstart = g.tile_start[pi], tiles_m = g.tiles_m[pi];
    int tm, tn;
    tile_coords(bid - tstart, tstart, tiles_m, (P.n + BN - 1) / BN, P.lower != 0, tm, tn);

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
    T *DT = static_cast<T *>(P.DT);
    const double alpha = P.alpha, beta = P.beta;
    const bool use_c = (beta != 0.0) && (C0 != nullptr);
    const bool add_i = P.add_identity != 0;
    const bool low = P.lower != 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int gm = m0 + wm0 + i * 16 + kcol;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gn = n0 + wn0 + j * 16 + Mma<T>::ncol(lane, v);
                if (gm < M && gn < N && !(low && gm < gn)) {
                    double val = alpha * (double)acc[i][j][v];
                    if (use_c) val += beta * (double)C0[gm + (int64_t)gn * P.ldc];
                    if (add_i && gm == gn) val += 1.0;
                    D[gm + (int64_t)gn * P.ldd] = (T)val;
                    if (DT != nullptr && !(low && gm == gn)) DT[gn + (int64_t)gm * P.lddt] = (T)val;
                }
            }
        }
    }
}

// Fast path.  Requires 16-byte aligned operands, leading dimensions that are
// multiples of the vector width, M a multiple of the vector width and K a
// multiple of BK -- true for every block product of the recursion when the
// order is a multiple of 64.  The main loop then has no control flow: the
// edge rows/columns of a tile are clamped once (what they load only reaches
// outputs the epilogue discards), each thread keeps one pointer per 16-byte
// global load and advances it by one slab per step.
//
// The K slab is split into four contiguous chunks of KQ = BK/4 values, one per
// lane group q = lane/16, and MFMA step kk consumes k = q*KQ + kk in group q
// (any assignment of k to the four MFMA k-slots is valid as long as A and B
// agree).  B is staged k-contiguous (Bs[n][k]) so that a lane fetches its KQ
// B values with 16-byte LDS reads; A is staged m-contiguous (As[k][m]).
// NW waves per workgroup, two workgroups per CU: eight for the 128 x 128
// tile (64 x 32 each) and the 64 x 64 tile (32 x 16 each), four for the
// 32 x 32 tile.  Eight waves put four on each SIMD (two when a product
// leaves one workgroup per CU), so more of the slab loads and barriers hide
// behind other waves' matrix instructions.
template <int BM, int BN, int BK, int WM, int WN, typename T, int NG, int NW>
__global__ void __launch_bounds__(64 * NW, NW / 2) gemm_fast(GroupArgs<NG> g) {
    constexpr int NT = 64 * NW;
    constexpr int VW = 16 / sizeof(T);
    typedef T vec_t __attribute__((ext_vector_type(VW)));
    constexpr int WAVES_M = BM / WM;
    static_assert(WAVES_M * (BN / WN) == NW, "NW waves per workgroup");
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
    const int pi = group_member(g, bid);
    const GemmProb P = g.p[pi];
    const int tstart = g.tile_start[pi], tiles_m = g.tiles_m[pi];
    int tm, tn;
    tile_coords(bid - tstart, tstart, tiles_m, (P.n + BN - 1) / BN, P.lower != 0, tm, tn);
    const int M = P.m, N = P.n, K = P.k;
    const int m0 = tm * BM, n0 = tn * BN;
    const int64_t lda = P.lda, ldb = P.ldb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % WAVES_M) * WM, wn0 = (wave / WAVES_M) * WN;

    const T *pa[AV];
    int sa[AV];
#pragma unroll
    for (int i = 0; i < AV; ++i) {
        const int v = tid + NT * i, r = (v % (BM / VW)) * VW, c = v / (BM / VW);
        const int row = m0 + r < M ? m0 + r : M - VW;
        pa[i] = static_cast<const T *>(P.A) + row + (int64_t)c * lda;
        sa[i] = c * A_LD + r;
    }
    const T *pb[BV];
    int sb[BV];
#pragma unroll
    for (int i = 0; i < BV; ++i) {
        const int v = tid + NT * i, k = (v % (BK / VW)) * VW, n = v / (BK / VW);
        const int col = n0 + n < N ? n0 + n : N - 1;
        pb[i] = static_cast<const T *>(P.B) + k + (int64_t)col * ldb;
        sb[i] = n * B_LD + k;
    }
    const int64_t astep = (int64_t)BK * lda;

    vec_t ra[AV], rb[BV];
    // Rows of A beyond M and columns of B beyond N are loaded from clamped
    // (valid) addresses and not zeroed: they only reach accumulator rows and
    // columns that the epilogue discards, so the loaded values are consumed
    // by the LDS stores alone and the compute phase never waits on them.
    auto gload = [&]() {
#pragma unroll
        for (int i = 0; i < AV; ++i) {
            ra[i] = *reinterpret_cast<const vec_t *>(pa[i]);
            pa[i] += astep;
        }
#pragma unroll
        for (int i = 0; i < BV; ++i) {
            rb[i] = *reinterpret_cast<const vec_t *>(pb[i]);
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
    // B fragments are fetched one 16-byte vector (VW consecutive k) per
    // column block at a time, which bounds their registers to TN vectors.
    auto compute = [&](int buf) {
        const T *as = &As[buf][(q * KQ) * A_LD + wm0 + c16];
        const T *bs = &Bs[buf][(wn0 + c16) * B_LD + q * KQ];
#pragma unroll
        for (int kc = 0; kc < KQ / VW; ++kc) {
            vec_t bv[TN];
#pragma unroll
            for (int j = 0; j < TN; ++j)
                bv[j] = *reinterpret_cast<const vec_t *>(bs + j * 16 * B_LD + kc * VW);
#pragma unroll
            for (int t = 0; t < VW; ++t) {
                const int kk = kc * VW + t;
                T a[TM];
#pragma unroll
                for (int i = 0; i < TM; ++i) a[i] = as[kk * A_LD + i * 16];
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) acc[i][j] = Mma<T>::mma(bv[j][t], a[i], acc[i][j]);
            }
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
    T *DT = static_cast<T *>(P.DT);
    const double alpha = P.alpha, beta = P.beta;
    const bool use_c = (beta != 0.0) && (C0 != nullptr);
    const bool add_i = P.add_identity != 0;
    const bool low = P.lower != 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int gm = m0 + wm0 + i * 16 + c16;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gn = n0 + wn0 + j * 16 + Mma<T>::ncol(lane, v);
                if (gm < M && gn < N && !(low && gm < gn)) {
                    double val = alpha * (double)acc[i][j][v];
                    if (use_c) val += beta * (double)C0[gm + (int64_t)gn * P.ldc];
                    if (add_i && gm == gn) val += 1.0;
                    D[gm + (int64_t)gn * P.ldd] = (T)val;
                    if (DT != nullptr && !(low && gm == gn)) DT[gn + (int64_t)gm * P.lddt] = (T)val;
                }
            }
        }
    }
}

// ------------------------------------------------------------ BF16 path ---
// Products of FP32 matrices on the BF16 matrix cores with FP32 accumulation.
// v_mfma_f32_16x16x32_bf16: lane l supplies row l % 16 of an operand at
// k = 8*(l/16) .. 8*(l/16) + 7 and receives rows 4*(l/16) + v of the result
// (operands transposed as above, so the result block is D^T).  Operands are
// rounded to BF16 (round to nearest even) while they are staged into LDS,
// k-contiguous per m (A) or n (B) row so that each lane fetches its eight k
// with one 16-byte read; the 80-byte row pitch spreads the 16 rows a
// quarter-wave reads over all 64 banks, and the four 16-byte k chunks of a
// row are stored in the order chunk ^ ((row >> 4) & 3), which spreads the
// stores of lanes 64 or 80 bytes x 4 rows apart over the banks while every
// 16-row read block keeps one order.  X3 splits every operand into
// hi = bf16(x) and lo = bf16(x - hi) (x - hi is exact in FP32) and
// accumulates hi*hi + lo*hi + hi*lo, about 16 significant bits per operand
// (the lo*lo term, of relative size 2^-16, is dropped).
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

template <int KN>
struct BfVec {
    typedef __bf16 type __attribute__((ext_vector_type(KN)));
};

template <int BM, int BN, int WM, int WN, bool X3, bool VEC, int NG, int NW = 4>
__global__ void __launch_bounds__(64 * NW, NW / 2) gemm_bf16(GroupArgs<NG> g) {
    constexpr int BK = 32;
    constexpr int NT = 64 * NW;
    constexpr int WAVES_M = BM / WM;
    static_assert(WAVES_M * (BN / WN) == NW, "NW waves per workgroup");
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int LDK = BK + 8;           // LDS pitch (elements) of one m or n row
    constexpr int KPA = BM * BK / NT / 4;  // k per thread in the A slab (4 rows each)
    constexpr int TPC = NT / BN;           // threads per column of the B slab
    constexpr int KPB = BK / TPC;          // k per thread in the B slab
    constexpr int NP = X3 ? 2 : 1;         // hi (and lo) planes
    static_assert(KPA >= 1 && KPB % 4 == 0, "slab/thread mismatch");
    typedef typename BfVec<KPA>::type va_t;
    static_assert(BK == 32, "four 16-byte k chunks per row");
    auto swz = [](int row) { return (row >> 4) & 3; };

    __shared__ __attribute__((aligned(16))) __bf16 As[2][NP][BM * LDK];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][NP][BN * LDK];

    const int bid = blockIdx.x;
    const int pi = group_member(g, bid);
    const GemmProb P = g.p[pi];
    const int tstart = g.tile_start[pi], tiles_m = g.tiles_m[pi];
    int tm, tn;
    tile_coords(bid - tstart, tstart, tiles_m, (P.n + BN - 1) / BN, P.lower != 0, tm, tn);
    const int M = P.m, N = P.n, K = P.k;
    const int m0 = tm * BM, n0 = tn * BN;
    const float *__restrict__ A = static_cast<const float *>(P.A);
    const float *__restrict__ B = static_cast<const float *>(P.B);
    const int64_t lda = P.lda, ldb = P.ldb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % WAVES_M) * WM, wn0 = (wave / WAVES_M) * WN;

    // A slab: rows 4*mq .. 4*mq+3, k = kq*KPA .. kq*KPA + KPA-1
    const int mq = tid % (BM / 4), kq = tid / (BM / 4);
    const int am = m0 + 4 * mq;
    // B slab: column bn, k = bk .. bk + KPB-1
    const int bn = tid / TPC, bk = (tid % TPC) * KPB;
    const int bcol = n0 + bn;

    float ra[KPA][4], rb[KPB];
    auto gload = [&](int k0) {
#pragma unroll
        for (int j = 0; j < KPA; ++j) {
            const int k = k0 + kq * KPA + j;
            if (VEC) {
                const bool ok = am < M && k < K;
                const float4 x = *reinterpret_cast<const float4 *>(ok ? A + am + (int64_t)k * lda : A);
                ra[j][0] = ok ? x.x : 0.f;
                ra[j][1] = ok ? x.y : 0.f;
                ra[j][2] = ok ? x.z : 0.f;
                ra[j][3] = ok ? x.w : 0.f;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const bool ok = am + i < M && k < K;
                    const float x = *(ok ? A + am + i + (int64_t)k * lda : A);
                    ra[j][i] = ok ? x : 0.f;
                }
            }
        }
#pragma unroll
        for (int h = 0; h < KPB / 4; ++h) {
            const int k = k0 + bk + 4 * h;
            if (VEC) {
                const bool ok = bcol < N && k < K;
                const float4 x = *reinterpret_cast<const float4 *>(ok ? B + k + (int64_t)bcol * ldb : B);
                rb[4 * h + 0] = ok ? x.x : 0.f;
                rb[4 * h + 1] = ok ? x.y : 0.f;
                rb[4 * h + 2] = ok ? x.z : 0.f;
                rb[4 * h + 3] = ok ? x.w : 0.f;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const bool ok = bcol < N && k + i < K;
                    const float x = *(ok ? B + k + i + (int64_t)bcol * ldb : B);
                    rb[4 * h + i] = ok ? x : 0.f;
                }
            }
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            va_t hi, lo;
#pragma unroll
            for (int j = 0; j < KPA; ++j) {
                const __bf16 h = (__bf16)ra[j][i];
                hi[j] = h;
                if (X3) lo[j] = (__bf16)(ra[j][i] - (float)h);
            }
            const int row = 4 * mq + i, k = kq * KPA;
            const int off = row * LDK + (((k >> 3) ^ swz(row)) << 3) + (k & 7);
            *reinterpret_cast<va_t *>(&As[buf][0][off]) = hi;
            if (X3) *reinterpret_cast<va_t *>(&As[buf][NP - 1][off]) = lo;
        }
        typedef __bf16 bc_t __attribute__((ext_vector_type(KPB < 8 ? KPB : 8)));
        constexpr int CW = KPB < 8 ? KPB : 8;  // elements per store
#pragma unroll
        for (int h0 = 0; h0 < KPB; h0 += CW) {
            bc_t hi, lo;
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                const __bf16 h = (__bf16)rb[h0 + j];
                hi[j] = h;
                if (X3) lo[j] = (__bf16)(rb[h0 + j] - (float)h);
            }
            const int k = bk + h0;
            const int off = bn * LDK + (((k >> 3) ^ swz(bn)) << 3) + (k & 7);
            *reinterpret_cast<bc_t *>(&Bs[buf][0][off]) = hi;
            if (X3) *reinterpret_cast<bc_t *>(&Bs[buf][NP - 1][off]) = lo;
        }
    };

    f4_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f4_t{0, 0, 0, 0};

    const int g4 = lane >> 4, c16 = lane & 15;
    auto compute = [&](int buf) {
        bf8_t a[NP][TM], b[NP][TN];
#pragma unroll
        for (int pl = 0; pl < NP; ++pl) {
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int row = wm0 + 16 * i + c16;
                a[pl][i] = *reinterpret_cast<const bf8_t *>(&As[buf][pl][row * LDK + ((g4 ^ swz(row)) << 3)]);
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int row = wn0 + 16 * j + c16;
                b[pl][j] = *reinterpret_cast<const bf8_t *>(&Bs[buf][pl][row * LDK + ((g4 ^ swz(row)) << 3)]);
            }
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[0][j], a[0][i], acc[i][j], 0, 0, 0);
                if (X3) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[0][j], a[NP - 1][i], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[NP - 1][j], a[0][i], acc[i][j], 0, 0, 0);
                }
            }
    };

    const int KT = (K + BK - 1) / BK;
    if (KT > 0) {
        gload(0);
        sstore(0);
        __syncthreads();
        for (int kt = 0; kt + 1 < KT; ++kt) {
            gload((kt + 1) * BK);
            compute(kt & 1);
            sstore((kt & 1) ^ 1);
            __syncthreads();
        }
        compute((KT - 1) & 1);
    }

    const float *__restrict__ C0 = static_cast<const float *>(P.C0);
    float *D = static_cast<float *>(P.D);
    float *DT = static_cast<float *>(P.DT);
    const double alpha = P.alpha, beta = P.beta;
    const bool use_c = (beta != 0.0) && (C0 != nullptr);
    const bool add_i = P.add_identity != 0;
    const bool low = P.lower != 0;
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int gm = m0 + wm0 + i * 16 + c16;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gn = n0 + wn0 + j * 16 + 4 * g4 + v;
                if (gm < M && gn < N && !(low && gm < gn)) {
                    double val = alpha * (double)acc[i][j][v];
                    if (use_c) val += beta * (double)C0[gm + (int64_t)gn * P.ldc];
                    if (add_i && gm == gn) val += 1.0;
                    D[gm + (int64_t)gn * P.ldd] = (float)val;
                    if (DT != nullptr && !(low && gm == gn)) DT[gn + (int64_t)gm * P.lddt] = (float)val;
                }
            }
        }
    }
}

// Large products on the BF16 matrix cores: eight waves share a 256 x 256
// tile (128 x 64 per wave), for products of at least 256 such tiles with
// 16-byte aligned rows of whole float4 vectors.  A 32-deep slab carries twice
// the flops per byte of FP32 operands loaded that the 128 x 128 tile does,
// and each wave issues 32 matrix instructions between two barriers instead
// of 16, which covers more of the next slab's load latency.  Staging
// (rounding, swizzled k chunks) and epilogue are gemm_bf16's (plain BF16
// only: bf16x3 keeps the 128 x 128 tile, whose hi and lo planes fit two
// workgroups per CU).
template <int BM, int BN, int WM, int WN, int NG>
__global__ void __launch_bounds__(512, 1) gemm_bf16_big(GroupArgs<NG> g) {
    constexpr int BK = 32;
    constexpr int NT = 512;
    constexpr int WAVES_M = BM / WM;
    static_assert(WAVES_M * (BN / WN) == 8, "eight waves per workgroup");
    constexpr int TM = WM / 16, TN = WN / 16;
    constexpr int LDK = BK + 8;            // LDS pitch (elements) of one m or n row
    constexpr int KPA = BM * BK / NT / 4;  // k per thread in the A slab (4 rows each)
    constexpr int TPC = NT / BN;           // threads per column of the B slab
    constexpr int KPB = BK / TPC;          // k per thread in the B slab
    static_assert(KPA >= 1 && KPB % 8 == 0, "slab/thread mismatch");
    typedef typename BfVec<KPA>::type va_t;
    auto swz = [](int row) { return (row >> 4) & 3; };

    __shared__ __attribute__((aligned(16))) __bf16 As[2][BM * LDK];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][BN * LDK];

    const int bid = blockIdx.x;
    const int pi = group_member(g, bid);
    const GemmProb P = g.p[pi];
    const int tstart = g.tile_start[pi], tiles_m = g.tiles_m[pi];
    int tm, tn;
    tile_coords(bid - tstart, tstart, tiles_m, (P.n + BN - 1) / BN, false, tm, tn);
    const int M = P.m, N = P.n, K = P.k;
    const int m0 = tm * BM, n0 = tn * BN;
    const float *__restrict__ A = static_cast<const float *>(P.A);
    const float *__restrict__ B = static_cast<const float *>(P.B);
    const int64_t lda = P.lda, ldb = P.ldb;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave % WAVES_M) * WM, wn0 = (wave / WAVES_M) * WN;

    // A slab: rows 4*mq .. 4*mq+3, k = kq*KPA .. kq*KPA + KPA-1
    const int mq = tid % (BM / 4), kq = tid / (BM / 4);
    const int am = m0 + 4 * mq;
    // B slab: column bn, k = bk .. bk + KPB-1
    const int bn = tid / TPC, bk = (tid % TPC) * KPB;
    const int bcol = n0 + bn;

    float ra[KPA][4], rb[KPB];
    auto gload = [&](int k0) {
#pragma unroll
        for (int j = 0; j < KPA; ++j) {
            const int k = k0 + kq * KPA + j;
            const bool ok = am < M && k < K;
            const float4 x = *reinterpret_cast<const float4 *>(ok ? A + am + (int64_t)k * lda : A);
            ra[j][0] = ok ? x.x : 0.f;
            ra[j][1] = ok ? x.y : 0.f;
            ra[j][2] = ok ? x.z : 0.f;
            ra[j][3] = ok ? x.w : 0.f;
        }
#pragma unroll
        for (int h = 0; h < KPB / 4; ++h) {
            const int k = k0 + bk + 4 * h;
            const bool ok = bcol < N && k < K;
            const float4 x = *reinterpret_cast<const float4 *>(ok ? B + k + (int64_t)bcol * ldb : B);
            rb[4 * h + 0] = ok ? x.x : 0.f;
            rb[4 * h + 1] = ok ? x.y : 0.f;
            rb[4 * h + 2] = ok ? x.z : 0.f;
            rb[4 * h + 3] = ok ? x.w : 0.f;
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            va_t hi;
#pragma unroll
            for (int j = 0; j < KPA; ++j) hi[j] = (__bf16)ra[j][i];
            const int row = 4 * mq + i, k = kq * KPA;
            *reinterpret_cast<va_t *>(&As[buf][row * LDK + (((k >> 3) ^ swz(row)) << 3) + (k & 7)]) = hi;
        }
#pragma unroll
        for (int h0 = 0; h0 < KPB; h0 += 8) {
            bf8_t hi;
#pragma unroll
            for (int j = 0; j < 8; ++j) hi[j] = (__bf16)rb[h0 + j];
            const int k = bk + h0;
            *reinterpret_cast<bf8_t *>(&Bs[buf][bn * LDK + (((k >> 3) ^ swz(bn)) << 3) + (k & 7)]) = hi;
        }
    };

    f4_t acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f4_t{0, 0, 0, 0};

    const int g4 = lane >> 4, c16 = lane & 15;
    auto compute = [&](int buf) {
        bf8_t b[TN];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int row = wn0 + 16 * j + c16;
            b[j] = *reinterpret_cast<const bf8_t *>(&Bs[buf][row * LDK + ((g4 ^ swz(row)) << 3)]);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int row = wm0 + 16 * i + c16;
            const bf8_t a = *reinterpret_cast<const bf8_t *>(&As[buf][row * LDK + ((g4 ^ swz(row)) << 3)]);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a, acc[i][j], 0, 0, 0);
        }
    };

    const int KT = (K + BK - 1) / BK;
    if (KT > 0) {
        gload(0);
        sstore(0);
        __syncthreads();
        for (int kt = 0; kt + 1 < KT; ++kt) {
            gload((kt + 1) * BK);
            compute(kt & 1);
            sstore((kt & 1) ^ 1);
            __syncthreads();
        }
        compute((KT - 1) & 1);
    }

    const float *__restrict__ C0 = static_cast<const float *>(P.C0);
    float *D = static_cast<float *>(P.D);
    float *DT = static_cast<float *>(P.DT);
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
                const int gn = n0 + wn0 + j * 16 + 4 * g4 + v;
                if (gm < M && gn < N) {
                    double val = alpha * (double)acc[i][j][v];
                    if (use_c) val += beta * (double)C0[gm + (int64_t)gn * P.ldc];
                    if (add_i && gm == gn) val += 1.0;
                    D[gm + (int64_t)gn * P.ldd] = (float)val;
                    if (DT != nullptr) DT[gn + (int64_t)gm * P.lddt] = (float)val;
                }
            }
        }
    }
}

// Tile prefix sums of up to N products for a BM x BN tiling; returns the
// number of workgroups.
template <int BM, int BN, int N>
int make_group(const GemmProb *probs, int count, GroupArgs<N> &g) {
    g = GroupArgs<N>{};
    g.count = count;
    int total = 0;
    for (int q = 0; q < N; ++q) {
        if (q < count) {
            g.p[q] = probs[q];
            const int tm = (probs[q].m + BM - 1) / BM, tn = (probs[q].n + BN - 1) / BN;
            // lower-triangle mode needs a square problem on a square tile grid
            const bool low = probs[q].lower && probs[q].m == probs[q].n && BM == BN;
            g.p[q].lower = low ? 1 : 0;
            g.tile_start[q] = total;
            g.tiles_m[q] = tm > 0 ? tm : 1;
            total += low ? tm * (tm + 1) / 2 : tm * tn;
        } else {
            g.p[q] = probs[0];
            g.tile_start[q] = 1 << 30;
            g.tiles_m[q] = 1;
        }
    }
    g.tile_start[N] = total;
    return total;
}

// One launch of up to N products that share a kernel configuration.
template <bool FAST, int BM, int BN, int BK, int WM, int WN, typename T, int N, int NW = 4>
hipError_t launch_group(const GemmProb *probs, int count, hipStream_t s) {
    GroupArgs<N> g;
    const int total = make_group<BM, BN, N>(probs, count, g);
    if (total == 0) return hipSuccess;
    if constexpr (FAST)
        hipLaunchKernelGGL((gemm_fast<BM, BN, BK, WM, WN, T, N, NW>), dim3(total), dim3(64 * NW), 0, s, g);
    else
        hipLaunchKernelGGL((gemm_kernel<BM, BN, BK, WM, WN, T, N>), dim3(total), dim3(256), 0, s, g);
    return hipGetLastError();
}

template <int BM, int BN, int WM, int WN, bool X3, bool VEC, int N, int NW = 4>
hipError_t launch_bf16_group(const GemmProb *probs, int count, hipStream_t s) {
    GroupArgs<N> g;
    const int total = make_group<BM, BN, N>(probs, count, g);
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL((gemm_bf16<BM, BN, WM, WN, X3, VEC, N, NW>), dim3(total), dim3(64 * NW), 0, s, g);
    return hipGetLastError();
}

template <int BM, int BN, int WM, int WN, int N>
hipError_t launch_bf16_big_group(const GemmProb *probs, int count, hipStream_t s) {
    GroupArgs<N> g;
    const int total = make_group<BM, BN, N>(probs, count, g);
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL((gemm_bf16_big<BM, BN, WM, WN, N>), dim3(total), dim3(512), 0, s, g);
    return hipGetLastError();
}

// K slab of the fast 128x128 kernel (FP64: 16 keeps two workgroups per CU;
// FP32: 32).  Every other fast configuration uses 32.
constexpr int kFastBK128 = 16;
constexpr int fast_bk(int tile, int es) { return (tile == 128 && es == 8) ? kFastBK128 : 32; }

// Kernel configuration of one product, a function of that product alone (its
// shape, leading dimensions and alignment), so that a product is computed
// bit for bit the same whether it is launched alone or grouped with others.
struct Cfg {
    int tile;   // 128, 64 or 32; 256 for the eight-wave BF16 tiles
    bool fast;  // branch-free vector path
    bool operator==(const Cfg &o) const { return tile == o.tile && fast == o.fast; }
};

Cfg choose_cfg(const GemmProb &p, DType dt) {
    const int es = dt == kF64 ? 8 : 4;
    const int vw = 16 / es;
    // a lower-triangle problem runs only the T (T + 1) / 2 tiles on or below
    // the diagonal, so that is the count that has to fill the GPU
    const bool low = p.lower && p.m == p.n;
    auto count = [&](int64_t t) {
        const int64_t tm = (p.m + t - 1) / t, tn = (p.n + t - 1) / t;
        return low ? tm * (tm + 1) / 2 : tm * tn;
    };
    const int64_t t128 = count(128);
    const int64_t t64 = count(64);
    Cfg c;
    c.tile = (t128 >= 192) ? 128 : (t64 >= 128) ? 64 : 32;
    const bool aligned =
        ((reinterpret_cast<uintptr_t>(p.A) | reinterpret_cast<uintptr_t>(p.B)) & 15) == 0;
    if (dt == kBF16 || dt == kBF16X3) {
        // float4 loads along m (A) and along k (B)
        c.fast = p.m % 4 == 0 && p.k % 4 == 0 && p.lda % 4 == 0 && p.ldb % 4 == 0 && aligned;
        // plain BF16: eight-wave 256 x 256 tiles once they alone fill the
        // GPU; not for the lower-triangle mode
        const int64_t big = ((p.m + 255) / 256) * ((p.n + 255) / 256);
        if (dt == kBF16 && c.fast && !p.lower && big >= 256) c.tile = 256;
        return c;
    }
    const int bk = fast_bk(c.tile, es);
    c.fast = p.k > 0 && p.k % bk == 0 && p.m % vw == 0 && p.lda % vw == 0 && p.ldb % vw == 0 &&
             aligned;
    return c;
}

template <typename T, int N>
hipError_t launch_cfg(Cfg c, const GemmProb *probs, int count, hipStream_t s) {
    constexpr int ES = sizeof(T);
    if (c.tile == 128)
        return c.fast ? launch_group<true, 128, 128, fast_bk(128, ES), 64, 32, T, N, 8>(probs, count, s)
                      : launch_group<false, 128, 128, 16, 64, 64, T, N>(probs, count, s);
    if (c.tile == 64)
        return c.fast ? launch_group<true, 64, 64, fast_bk(64, ES), 32, 16, T, N, 8>(probs, count, s)
                      : launch_group<false, 64, 64, 16, 32, 32, T, N>(probs, count, s);
    return c.fast ? launch_group<true, 32, 32, fast_bk(32, ES), 16, 16, T, N>(probs, count, s)
                  : launch_group<false, 32, 32, 32, 16, 16, T, N>(probs, count, s);
}

template <bool X3, int N>
hipError_t launch_cfg_bf16(Cfg c, const GemmProb *probs, int count, hipStream_t s) {
    if constexpr (!X3)
        if (c.tile == 256) return launch_bf16_big_group<256, 256, 128, 64, N>(probs, count, s);
    if (c.tile == 128)
        return c.fast ? launch_bf16_group<128, 128, 64, 32, X3, true, N, 8>(probs, count, s)
                      : launch_bf16_group<128, 128, 64, 64, X3, false, N>(probs, count, s);
    if (c.tile == 64)
        return c.fast ? launch_bf16_group<64, 64, 32, 32, X3, true, N>(probs, count, s)
                      : launch_bf16_group<64, 64, 32, 32, X3, false, N>(probs, count, s);
    return c.fast ? launch_bf16_group<32, 32, 16, 16, X3, true, N>(probs, count, s)
                  : launch_bf16_group<32, 32, 16, 16, X3, false, N>(probs, count, s);
}

const char *cfg_name(Cfg c, DType dt) {
    static const char *names[4][3][2] = {
        {{"gemm_f64_128x128_edge", "gemm_f64_128x128"}, {"gemm_f64_64x64_edge", "gemm_f64_64x64"},
         {"gemm_f64_32x32_edge", "gemm_f64_32x32"}},
        {{"gemm_f32_128x128_edge", "gemm_f32_128x128"}, {"gemm_f32_64x64_edge", "gemm_f32_64x64"},
         {"gemm_f32_32x32_edge", "gemm_f32_32x32"}},
        {{"gemm_bf16_128x128_edge", "gemm_bf16_128x128"},
         {"gemm_bf16_64x64_edge", "gemm_bf16_64x64"},
         {"gemm_bf16_32x32_edge", "gemm_bf16_32x32"}},
        {{"gemm_bf16x3_128x128_edge", "gemm_bf16x3_128x128"},
         {"gemm_bf16x3_64x64_edge", "gemm_bf16x3_64x64"},
         {"gemm_bf16x3_32x32_edge", "gemm_bf16x3_32x32"}}};
    if (c.tile == 256) return "gemm_bf16_256x256";
    const int ti = c.tile == 128 ? 0 : c.tile == 64 ? 1 : 2;
    return names[(int)dt][ti][c.fast ? 1 : 0];
}

}  // namespace

hipError_t gemm_launch(const GemmProb *probs, int count, DType dt, hipStream_t s, LaunchInfo *info) {
    if (count < 1 || count > kMaxBatch) return hipErrorInvalidValue;
    if (dt != kF64 && dt != kF32 && dt != kBF16 && dt != kBF16X3) return hipErrorInvalidValue;
    const int esz = (dt == kF64) ? 8 : 4;
    const double es = esz;
    // Products with an empty reduction still need their epilogue; drop only
    // products with an empty output.  Group the rest by configuration.
    GemmProb part[kMaxBatch];
    Cfg cfgs[kMaxBatch];
    bool done[kMaxBatch];
    int n_live = 0;
    double flops = 0, bytes = 0;
    // the mirror form (DT == D) relies on the lower-triangle mode, which every
    // tile shape honours for a square problem
    for (int q = 0; q < count; ++q)
        if (probs[q].DT != nullptr && probs[q].DT == probs[q].D &&
            !(probs[q].lower && probs[q].m == probs[q].n))
            return hipErrorInvalidValue;
    for (int q = 0; q < count; ++q) {
        if (probs[q].m <= 0 || probs[q].n <= 0) continue;
        part[n_live] = probs[q];
        cfgs[n_live] = choose_cfg(probs[q], dt);
        done[n_live] = false;
        ++n_live;
        const double m = probs[q].m, n = probs[q].n, k = probs[q].k;
        // a lower-triangle product computes about m (m + tile) / 2 outputs
        flops += (probs[q].lower && probs[q].m == probs[q].n) ? k * m * (m + cfgs[n_live - 1].tile)
                                                               : 2.0 * m * n * k;
        bytes += es * (m * k + k * n + m * n + ((probs[q].beta != 0.0) ? m * n : 0.0));
        if (probs[q].DT != nullptr) bytes += es * m * n * (probs[q].lower ? 0.5 : 1.0);
    }
    const char *name = "gemm_empty";
    hipError_t e = hipSuccess;
    for (int q = 0; q < n_live && e == hipSuccess; ++q) {
        if (done[q]) continue;
        GemmProb grp[kMaxBatch];
        int ng = 0;
        for (int r = q; r < n_live; ++r)
            if (!done[r] && cfgs[r] == cfgs[q]) {
                grp[ng++] = part[r];
                done[r] = true;
            }
        name = cfg_name(cfgs[q], dt);
        if (dt == kF64)
            e = (ng <= 2) ? launch_cfg<double, 2>(cfgs[q], grp, ng, s)
                          : launch_cfg<double, kMaxBatch>(cfgs[q], grp, ng, s);
        else if (dt == kF32)
            e = (ng <= 2) ? launch_cfg<float, 2>(cfgs[q], grp, ng, s)
                          : launch_cfg<float, kMaxBatch>(cfgs[q], grp, ng, s);
        else if (dt == kBF16)
            e = (ng <= 2) ? launch_cfg_bf16<false, 2>(cfgs[q], grp, ng, s)
                          : launch_cfg_bf16<false, kMaxBatch>(cfgs[q], grp, ng, s);
        else
            e = (ng <= 2) ? launch_cfg_bf16<true, 2>(cfgs[q], grp, ng, s)
                          : launch_cfg_bf16<true, kMaxBatch>(cfgs[q], grp, ng, s);
    }
    if (info) {
        info->name = name;
        info->flops = flops;
        info->bytes = bytes;
    }
    return e;
}

}  // namespace spin
