// FP64-accurate block products on INT8 matrix cores, for the Newton
// refinement's residual R = I - A X and update X + X R (Newton iteration as
// the stabiliser of Strassen inversion, Sec. 2.1).
//
// The emulation is the integer modular scheme of Ozaki, Uchino and Imamura
// (Ozaki scheme II, 2025) on the error-free splitting of Ozaki, Ogita, Oishi
// and Rump (2012):
//   1. split: row i of the left operand is scaled by 2^s_i and rounded to the
//      nearest integer (ties to even), column j of the right operand by 2^t_j,
//      with s_i = beta - E_i for a row maximum f 2^E_i, f in [1/2, 1), so that
//      no integer exceeds 2^beta; for each modulus m_l (pairwise coprime, at
//      most 256) the symmetric residue of every integer is stored as an int8,
//      K-contiguous per row (left) or per column (right), zero padded;
//   2. product: for each modulus, the INT8 matrix-core product of the residue
//      matrices is exact in int32 (|sum| <= k 128^2 < 2^31); it is reduced
//      into [0, m_l) and stored as one byte per element;
//   3. reconstruction: P = sum_l r_l w_l mod M (M the product of the moduli,
//      w_l its Chinese-remainder weights) in 128-bit integers is the exact
//      integer product A' B' once 2 k 2^(beta_a + beta_b) < M; P is taken
//      symmetric, rounded once to FP64 (nearest, ties to even), scaled by
//      2^-(s_i + t_j), and the epilogue (I - D, or C0 + D) rounds once more.
// A row of the left operand or a column of the right one that holds a
// non-finite value gives NaN in its row or column of the result.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <cmath>
#include <cstdint>

#include "spin_kernels.hpp"

namespace spin {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned __int128 u128;

// Pairwise coprime moduli, largest first; the first n are used.
constexpr int kModuli[kOzakiMaxModuli] = {256, 255, 253, 251, 247, 241, 239, 233,
                                          229, 227, 223, 217, 211, 199, 197};

struct ModArgs {
    int count;
    int m[kOzakiMaxModuli];
    double inv[kOzakiMaxModuli];          // 1 / m_l
    unsigned long long w_lo[kOzakiMaxModuli], w_hi[kOzakiMaxModuli];  // CRT weights
    unsigned long long M_lo, M_hi;        // product of the moduli
    double invM;                          // 1 / M (approximate)
    int every;                            // terms summed between reductions mod M
};

constexpr unsigned long long kNonFinite = 0x7ff0000000000000ull;  // |x| bits at or above: Inf / NaN
constexpr int kBadShift = INT_MIN;                                 // shift of a non-finite row

// ------------------------------------------------------------ row maxima ---
// rmax[i] = max over the row's |a| as IEEE bits (ordered like the values for
// non-negative doubles; Inf and NaN compare above every finite value).
__global__ void __launch_bounds__(256) k_rowmax(const double *__restrict__ a, int64_t lda, int m,
                                                 int k, int kchunk, unsigned long long *rmax) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const int k0 = blockIdx.y * kchunk, k1 = min(k, k0 + kchunk);
    unsigned long long mx = 0;
    for (int q = k0; q < k1; ++q) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(a[i + (int64_t)q * lda]) &
                                     0x7fffffffffffffffull;
        mx = b > mx ? b : mx;
    }
    if (mx) atomicMax(rmax + i, mx);
}

// cmax[j] for a column-major (k x n) view: one workgroup per column.
__global__ void __launch_bounds__(256) k_colmax(const double *__restrict__ b, int64_t ldb, int k,
                                                 unsigned long long *cmax) {
    __shared__ unsigned long long red[256];
    const int j = blockIdx.x;
    unsigned long long mx = 0;
    for (int q = threadIdx.x; q < k; q += 256) {
        const unsigned long long v = (unsigned long long)__double_as_longlong(b[q + (int64_t)j * ldb]) &
                                     0x7fffffffffffffffull;
        mx = v > mx ? v : mx;
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) cmax[j] = red[0];
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

// shift[i] = beta - E for max = f 2^E, f in [1/2, 1); 0 for a zero maximum;
// kBadShift for a non-finite one.
__global__ void k_shifts(const unsigned long long *mx, int n, int beta, int *shift) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const unsigned long long b = mx[i];
    if (b >= kNonFinite) {
        shift[i] = kBadShift;
    } else if (b == 0) {
        shift[i] = 0;
    } else {
        int e;
        (void)frexp(__longlong_as_double((long long)b), &e);
        shift[i] = beta - e;
    }
}

// Symmetric residue of the integer-valued double v modulo m.
__device__ inline int sym_residue(double v, int m, double inv) {
    double q = floor(v * inv);
    double r = v - q * (double)m;  // exact: |q m| <= |v| + m < 2^53
    if (r < 0.0) r += (double)m;
    if (r >= (double)m) r -= (double)m;
    int ri = (int)r;
    if (ri >= (m + 1) / 2) ri -= m;
    return ri;
}

// The scaled, rounded integer of x under shift s (0 for a non-finite row).
__device__ inline double split_value(double x, int s) {
    return s == kBadShift ? 0.0 : rint(ldexp(x, s));
}

// Left operand: residue planes with rows K-contiguous, plane[l][i * kp + q].
// A workgroup moves a 64 (rows) x 64 (k) block through LDS so that both the
// column-major reads and the row-contiguous writes coalesce.
__global__ void __launch_bounds__(256) k_split_rows(const double *__restrict__ a, int64_t lda, int m,
                                                     int k, const int *__restrict__ shift, int8_t *planes,
                                                     int64_t mp, int kp, ModArgs md) {
    __shared__ double tile[64][65];
    __shared__ __attribute__((aligned(16))) int8_t res[64][64 + 16];
    const int i0 = blockIdx.x * 64, q0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int qq = ty; qq < 64; qq += 4) {
        const int i = i0 + tx, q = q0 + qq;
        double v = 0.0;
        if (i < m && q < k) v = split_value(a[i + (int64_t)q * lda], shift[i]);
        tile[tx][qq] = v;
    }
    __syncthreads();
    const int row = threadIdx.x >> 2, c16 = (threadIdx.x & 3) * 16;  // 16 bytes per thread
    for (int l = 0; l < md.count; ++l) {
        for (int e = threadIdx.x; e < 64 * 64; e += 256) {
            const int r = e >> 6, c = e & 63;
            res[r][c] = (int8_t)sym_residue(tile[r][c], md.m[l], md.inv[l]);
        }
        __syncthreads();
        int8_t *dst = planes + (int64_t)l * mp * kp + (int64_t)(i0 + row) * kp + q0 + c16;
        *reinterpret_cast<v4i *>(dst) = *reinterpret_cast<const v4i *>(&res[row][c16]);
        __syncthreads();
    }
}

// Right operand: residue planes with columns K-contiguous, plane[l][j * kp + q]
// (the column-major order of the operand itself).  Thread: 16 k of one column.
__global__ void __launch_bounds__(256) k_split_cols(const double *__restrict__ b, int64_t ldb, int k,
                                                     int n, const int *__restrict__ shift, int8_t *planes,
                                                     int64_t np_, int kp, ModArgs md) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int chunks = kp / 16;
    if (e >= (int64_t)np_ * chunks) return;
    const int j = (int)(e / chunks), q0 = (int)(e % chunks) * 16;
    double v[16];
    const int s = j < n ? shift[j] : 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int q = q0 + u;
        v[u] = (j < n && q < k) ? split_value(b[q + (int64_t)j * ldb], s) : 0.0;
    }
    for (int l = 0; l < md.count; ++l) {
        union {
            int8_t b8[16];
            v4i w;
        } pk;
#pragma unroll
        for (int u = 0; u < 16; ++u) pk.b8[u] = (int8_t)sym_residue(v[u], md.m[l], md.inv[l]);
        *reinterpret_cast<v4i *>(planes + (int64_t)l * np_ * kp + (int64_t)j * kp + q0) = pk.w;
    }
}

// ------------------------------------------------------------ INT8 GEMM ---
// For modulus l = blockIdx.z: C_l = A_l B_l over the residue planes, a 128 x
// 128 tile per workgroup (four waves of 64 x 64, 4 x 4 blocks of
// v_mfma_i32_16x16x64_i8), K in 64-byte slabs staged through LDS (two
// buffers, one barrier per slab).  Output bytes (the sums reduced into
// [0, m_l)) go to cplanes[l][i + j * mp], four consecutive rows per lane.
constexpr int kTB = 128, kSK = 64, kPitch = 80;  // 80-byte LDS rows: conflict-free fragment reads

__global__ void __launch_bounds__(256, 2) k_gemm_i8(const int8_t *__restrict__ ap, const int8_t *__restrict__ bp,
                                                     uint8_t *__restrict__ cp, int m, int n, int64_t mp,
                                                     int64_t np_, int kp, ModArgs md) {
    __shared__ __attribute__((aligned(16))) int8_t As[2][kTB * kPitch];
    __shared__ __attribute__((aligned(16))) int8_t Bs[2][kTB * kPitch];
    const int l = blockIdx.z;
    const int i0 = blockIdx.x * kTB, j0 = blockIdx.y * kTB;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = (w & 1) * 64, wn = (w >> 1) * 64;
    const int8_t *A = ap + (int64_t)l * mp * kp + (int64_t)i0 * kp;
    const int8_t *B = bp + (int64_t)l * np_ * kp + (int64_t)j0 * kp;
    // slab loads: chunk c (of 512) = row c / 4, 16-byte piece c % 4
    const int r0 = t >> 2, r1 = (t + 256) >> 2, pc = (t & 3) * 16;
    v4i ra0, ra1, rb0, rb1;
    auto load = [&](int q0) {
        ra0 = *reinterpret_cast<const v4i *>(A + (int64_t)r0 * kp + q0 + pc);
        ra1 = *reinterpret_cast<const v4i *>(A + (int64_t)r1 * kp + q0 + pc);
        rb0 = *reinterpret_cast<const v4i *>(B + (int64_t)r0 * kp + q0 + pc);
        rb1 = *reinterpret_cast<const v4i *>(B + (int64_t)r1 * kp + q0 + pc);
    };
    auto store = [&](int buf) {
        *reinterpret_cast<v4i *>(&As[buf][r0 * kPitch + pc]) = ra0;
        *reinterpret_cast<v4i *>(&As[buf][r1 * kPitch + pc]) = ra1;
        *reinterpret_cast<v4i *>(&Bs[buf][r0 * kPitch + pc]) = rb0;
        *reinterpret_cast<v4i *>(&Bs[buf][r1 * kPitch + pc]) = rb1;
    };
    v4i acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4i{0, 0, 0, 0};
    const int nk = kp / kSK;
    load(0);
    store(0);
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 16;
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load((kt + 1) * kSK);
        v4i fa[4], fb[4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
            fa[a] = *reinterpret_cast<const v4i *>(&As[buf][(wm + 16 * a + fr) * kPitch + fk]);
#pragma unroll
        for (int b = 0; b < 4; ++b)
            fb[b] = *reinterpret_cast<const v4i *>(&Bs[buf][(wn + 16 * b + fr) * kPitch + fk]);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
        if (kt + 1 < nk) store(buf ^ 1);
        __syncthreads();
    }
    // lane holds rows 4 (lane / 16) + v, v = 0..3, of column lane % 16 of each block
    const int mod = md.m[l];
    uint8_t *C = cp + (int64_t)l * mp * np_;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + wm + 16 * a + 4 * (lane >> 4);
            const int j = j0 + wn + 16 * b + (lane & 15);
            if (j >= n || i >= m) continue;
            unsigned int packed = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int r = acc[a][b][v] % mod;
                if (r < 0) r += mod;
                packed |= (unsigned int)r << (8 * v);
            }
            *reinterpret_cast<unsigned int *>(C + i + (int64_t)j * mp) = packed;
        }
}

// The same product with 256 x 256 tiles: eight waves, each 128 x 64 (8 x 4
// blocks), twice the integer operations per byte of residues moved, for the
// large products of the refinement.  Residue planes padded to 256 rows.
constexpr int kTB2 = 256;

__global__ void __launch_bounds__(512, 1) k_gemm_i8_256(const int8_t *__restrict__ ap,
                                                         const int8_t *__restrict__ bp,
                                                         uint8_t *__restrict__ cp, int m, int n,
                                                         int64_t mp, int64_t np_, int kp, ModArgs md) {
    __shared__ __attribute__((aligned(16))) int8_t As[2][kTB2 * kPitch];
    __shared__ __attribute__((aligned(16))) int8_t Bs[2][kTB2 * kPitch];
    const int l = blockIdx.z;
    const int i0 = blockIdx.x * kTB2, j0 = blockIdx.y * kTB2;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = (w & 1) * 128, wn = (w >> 1) * 64;
    const int8_t *A = ap + (int64_t)l * mp * kp + (int64_t)i0 * kp;
    const int8_t *B = bp + (int64_t)l * np_ * kp + (int64_t)j0 * kp;
    // slab loads: 1024 pieces of 16 bytes per operand, two per thread
    const int r0 = t >> 2, r1 = (t + 512) >> 2, pc = (t & 3) * 16;
    v4i ra0, ra1, rb0, rb1;
    auto load = [&](int q0) {
        ra0 = *reinterpret_cast<const v4i *>(A + (int64_t)r0 * kp + q0 + pc);
        ra1 = *reinterpret_cast<const v4i *>(A + (int64_t)r1 * kp + q0 + pc);
        rb0 = *reinterpret_cast<const v4i *>(B + (int64_t)r0 * kp + q0 + pc);
        rb1 = *reinterpret_cast<const v4i *>(B + (int64_t)r1 * kp + q0 + pc);
    };
    auto store = [&](int buf) {
        *reinterpret_cast<v4i *>(&As[buf][r0 * kPitch + pc]) = ra0;
        *reinterpret_cast<v4i *>(&As[buf][r1 * kPitch + pc]) = ra1;
        *reinterpret_cast<v4i *>(&Bs[buf][r0 * kPitch + pc]) = rb0;
        *reinterpret_cast<v4i *>(&Bs[buf][r1 * kPitch + pc]) = rb1;
    };
    v4i acc[8][4];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4i{0, 0, 0, 0};
    const int nk = kp / kSK;
    load(0);
    store(0);
    __syncthreads();
    const int fr = lane & 15, fk = (lane >> 4) * 16;
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load((kt + 1) * kSK);
        v4i fb[4];
#pragma unroll
        for (int b = 0; b < 4; ++b)
            fb[b] = *reinterpret_cast<const v4i *>(&Bs[buf][(wn + 16 * b + fr) * kPitch + fk]);
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const v4i fa = *reinterpret_cast<const v4i *>(&As[buf][(wm + 16 * a + fr) * kPitch + fk]);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa, fb[b], acc[a][b], 0, 0, 0);
        }
        if (kt + 1 < nk) store(buf ^ 1);
        __syncthreads();
    }
    const int mod = md.m[l];
    uint8_t *C = cp + (int64_t)l * mp * np_;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + wm + 16 * a + 4 * (lane >> 4);
            const int j = j0 + wn + 16 * b + (lane & 15);
            if (j >= n || i >= m) continue;
            unsigned int packed = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int r = acc[a][b][v] % mod;
                if (r < 0) r += mod;
                packed |= (unsigned int)r << (8 * v);
            }
            *reinterpret_cast<unsigned int *>(C + i + (int64_t)j * mp) = packed;
        }
}

// ------------------------------------------------------- reconstruction ---
__device__ inline u128 mk128(unsigned long long lo, unsigned long long hi) {
    return ((u128)hi << 64) | lo;
}

__device__ inline double u128_to_double(u128 v) {
    return ldexp((double)(unsigned long long)(v >> 64), 64) + (double)(unsigned long long)v;
}

// Correct rounding (nearest, ties to even) of a < 2^127 to FP64.
__device__ inline double round_u128(u128 a) {
    const unsigned long long hi = (unsigned long long)(a >> 64), lo = (unsigned long long)a;
    if (hi == 0 && (lo >> 53) == 0) return (double)lo;
    const int msb = hi ? 127 - __builtin_clzll(hi) : 63 - __builtin_clzll(lo);
    const int sh = msb - 52;  // bits dropped, >= 1
    u128 mant = a >> sh;
    const u128 rem = a & (((u128)1 << sh) - 1), half = (u128)1 << (sh - 1);
    if (rem > half || (rem == half && (mant & 1))) mant += 1;
    return ldexp((double)(unsigned long long)mant, sh);
}

// D = epilogue(P 2^-(s_i + t_j)) with P rebuilt from its residues.
// epi 0: D = P; 1: D = I - P (m == n); 2: D = C0 + P.
__global__ void __launch_bounds__(256) k_crt(const uint8_t *__restrict__ cp, int64_t mp, int64_t np_, int m,
                                              int n, const int *__restrict__ sa, const int *__restrict__ tb,
                                              int epi, const double *__restrict__ c0, int64_t ldc,
                                              double *__restrict__ d, int64_t ldd, ModArgs md) {
    const u128 M = mk128(md.M_lo, md.M_hi), halfM = M >> 1;
    const int64_t total = (int64_t)m * n;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int i = (int)(e % m), j = (int)(e / m);
        // sum of r_l w_l, reduced mod M after every `every` terms (the host
        // picks `every` so that the partial sum stays below 2^127)
        u128 S = 0;
        for (int l = 0; l < md.count; ++l) {
            const unsigned int r = cp[(int64_t)l * mp * np_ + i + (int64_t)j * mp];
            S += (u128)r * mk128(md.w_lo[l], md.w_hi[l]);
            if ((l + 1) % md.every == 0 || l + 1 == md.count) {
                unsigned long long q = (unsigned long long)(u128_to_double(S) * md.invM);
                if (q) S -= (u128)q * M;        // the estimate may be one too high or low
                if ((S >> 127) != 0) S += M;    // wrapped below zero
                if (S >= M) S -= M;
            }
        }
        const bool neg = S > halfM;
        const u128 mag = neg ? M - S : S;
        double v = round_u128(mag);
        v = neg ? -v : v;
        const int s = sa[i], tt = tb[j];
        if (s == kBadShift || tt == kBadShift)
            v = __longlong_as_double(0x7ff8000000000000ll);
        else
            v = ldexp(v, -(s + tt));
        double out;
        if (epi == 1)
            out = (i == j ? 1.0 : 0.0) - v;
        else if (epi == 2)
            out = c0[i + (int64_t)j * ldc] + v;
        else
            out = v;
        d[i + (int64_t)j * ldd] = out;
    }
}

}  // namespace

// ------------------------------------------------------------------ host ---
namespace {
u128 h_mul_mod(u128 a, u128 b, u128 M) {  // (a * b) mod M for b < 2^9
    return (a * b) % M;
}

int h_inv_mod(long long a, long long m) {  // a^-1 mod m (a, m coprime)
    long long t = 0, nt = 1, r = m, nr = ((a % m) + m) % m;
    while (nr) {
        const long long q = r / nr;
        long long tmp = t - q * nt;
        t = nt;
        nt = tmp;
        tmp = r - q * nr;
        r = nr;
        nr = tmp;
    }
    return (int)((t % m + m) % m);
}

ModArgs make_moduli(int count) {
    ModArgs md{};
    md.count = count;
    u128 M = 1;
    for (int l = 0; l < count; ++l) M *= (u128)kModuli[l];
    for (int l = 0; l < count; ++l) {
        md.m[l] = kModuli[l];
        md.inv[l] = 1.0 / (double)kModuli[l];
        const u128 Ml = M / (u128)kModuli[l];
        const int ml_mod = (int)(Ml % (u128)kModuli[l]);
        const u128 wl = h_mul_mod(Ml, (u128)h_inv_mod(ml_mod, kModuli[l]), M);
        md.w_lo[l] = (unsigned long long)wl;
        md.w_hi[l] = (unsigned long long)(wl >> 64);
    }
    md.M_lo = (unsigned long long)M;
    md.M_hi = (unsigned long long)(M >> 64);
    md.invM = 1.0 / ((double)md.M_hi * 18446744073709551616.0 + (double)md.M_lo);
    // a partial sum below M plus `every` terms below 256 M each must stay
    // below 2^127 (the top bit marks a wrap in the reduction)
    const u128 lim = ((u128)1 << 127) / M;  // floor(2^127 / M)
    md.every = (int)std::max<u128>(1, std::min<u128>((lim - 1) / 256, (u128)count));
    return md;
}

int64_t rup(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Tile of the INT8 product: 256 x 256 when both sides hold at least four
// such tiles, else 128 x 128.
int64_t tile_for(int64_t m, int64_t n) { return (m >= 4 * kTB2 && n >= 4 * kTB2) ? kTB2 : kTB; }
}  // namespace

double ozaki_log2_modulus(int count) {
    double s = 0.0;
    for (int l = 0; l < count; ++l) s += std::log2((double)kModuli[l]);
    return s;
}

int ozaki_beta(int count, int64_t k) {
    const double lm = ozaki_log2_modulus(count);
    return (int)std::floor((lm - 1.0 - std::log2((double)(k > 0 ? k : 1))) / 2.0 - 1e-9);
}

size_t ozaki_workspace_bytes(int64_t m, int64_t n, int64_t k, int count) {
    const int64_t tile = tile_for(m, n);
    const int64_t mp = rup(m, tile), np_ = rup(n, tile), kp = rup(k > 0 ? k : 1, kSK);
    size_t b = 0;
    b += al256((size_t)count * mp * kp);   // left residues
    b += al256((size_t)count * np_ * kp);  // right residues
    b += al256((size_t)count * mp * np_);  // product residues
    b += al256(8 * (size_t)(mp + np_));    // maxima
    b += al256(4 * (size_t)(mp + np_));    // shifts
    return b;
}

hipError_t ozaki_product(const OzakiProb &p, void *ws, hipStream_t s) {
    if (p.moduli < 2 || p.moduli > kOzakiMaxModuli || p.k > kOzakiMaxK) return hipErrorInvalidValue;
    if (p.m <= 0 || p.n <= 0) return hipSuccess;
    const int64_t m = p.m, n = p.n, k = p.k;
    const int64_t tile = tile_for(m, n);
    const int64_t mp = rup(m, tile), np_ = rup(n, tile), kp = rup(k > 0 ? k : 1, kSK);
    if (mp > INT_MAX / 2 || np_ > INT_MAX / 2 || kp > INT_MAX / 2) return hipErrorInvalidValue;
    const ModArgs md = make_moduli(p.moduli);
    char *w = static_cast<char *>(ws);
    int8_t *apl = reinterpret_cast<int8_t *>(w);
    w += al256((size_t)p.moduli * mp * kp);
    int8_t *bpl = reinterpret_cast<int8_t *>(w);
    w += al256((size_t)p.moduli * np_ * kp);
    uint8_t *cpl = reinterpret_cast<uint8_t *>(w);
    w += al256((size_t)p.moduli * mp * np_);
    unsigned long long *amax = reinterpret_cast<unsigned long long *>(w);
    unsigned long long *bmax = amax + mp;
    w += al256(8 * (size_t)(mp + np_));
    int *sa = reinterpret_cast<int *>(w);
    int *tb = sa + mp;

    const int nz = (int)(mp + np_);
    hipLaunchKernelGGL(k_zero_u64, dim3((nz + 255) / 256), dim3(256), 0, s, amax, nz);
    if (k > 0) {
        const int kchunk = 64;
        const int gy = (int)std::min<int64_t>((k + kchunk - 1) / kchunk, 65535);
        hipLaunchKernelGGL(k_rowmax, dim3((unsigned)((m + 255) / 256), (unsigned)gy), dim3(256), 0, s,
                           p.A, p.lda, (int)m, (int)k, (int)((k + gy - 1) / gy), amax);
        hipLaunchKernelGGL(k_colmax, dim3((unsigned)n), dim3(256), 0, s, p.B, p.ldb, (int)k, bmax);
    }
    hipLaunchKernelGGL(k_shifts, dim3((unsigned)((mp + 255) / 256)), dim3(256), 0, s, amax, (int)mp,
                       p.beta_a, sa);
    hipLaunchKernelGGL(k_shifts, dim3((unsigned)((np_ + 255) / 256)), dim3(256), 0, s, bmax, (int)np_,
                       p.beta_b, tb);
    hipLaunchKernelGGL(k_split_rows, dim3((unsigned)(mp / 64), (unsigned)(kp / 64)), dim3(256), 0, s,
                       p.A, p.lda, (int)m, (int)k, sa, apl, mp, (int)kp, md);
    const int64_t cchunks = np_ * (kp / 16);
    hipLaunchKernelGGL(k_split_cols, dim3((unsigned)((cchunks + 255) / 256)), dim3(256), 0, s, p.B,
                       p.ldb, (int)k, (int)n, tb, bpl, np_, (int)kp, md);
    if (tile == kTB2)
        hipLaunchKernelGGL(k_gemm_i8_256, dim3((unsigned)(mp / kTB2), (unsigned)(np_ / kTB2), (unsigned)p.moduli),
                           dim3(512), 0, s, apl, bpl, cpl, (int)m, (int)n, mp, np_, (int)kp, md);
    else
        hipLaunchKernelGGL(k_gemm_i8, dim3((unsigned)(mp / kTB), (unsigned)(np_ / kTB), (unsigned)p.moduli),
                           dim3(256), 0, s, apl, bpl, cpl, (int)m, (int)n, mp, np_, (int)kp, md);
    const int64_t total = m * n;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_crt, dim3((unsigned)blocks), dim3(256), 0, s, cpl, mp, np_, (int)m, (int)n, sa,
                       tb, p.epilogue, p.C0, p.ldc, p.D, p.ldd, md);
    return hipGetLastError();
}

}  // namespace spin
