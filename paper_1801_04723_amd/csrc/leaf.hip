// Leaf inversion: Gauss-Jordan elimination with partial pivoting in FP64.
//
// The paper leaves the method of the leaf inversion open and runs it on a
// single node (Alg. 1, Alg. 2 `locInverse`, Sec. 3.3); here it is Gauss-Jordan with
// partial pivoting, always in FP64 (also when the surrounding products run in
// FP32).
//
// Every tier uses implicit pivoting: rows are never moved.  Step k picks the
// unused row p with the largest |z[p][k]| (ties to the smallest row index),
// scales row p by 1/pivot and eliminates column k from every other row.  The
// storage is in place: after step k the slot of column k holds column p of
// the accumulated row transformation (it replaces the unit column that an
// augmented [A | I] would carry).  With r[k] = pivot row of step k and
// rinv[r[k]] = k, the inverse is  X[rinv[i]][r[c]] = Z[i][c].
//
// Tier 1 (L <= 128): one workgroup holds the whole block in registers,
//   cyclically distributed (thread (tr, tc) of a TR x 16 grid owns rows
//   tr + TR*a and columns tc + 16b).  A step costs two barriers: the owners of
//   column k publish it to LDS, every wave finds the pivot redundantly (DPP
//   max, then ballots for the smallest row index), the owners of the pivot
//   row publish the scaled row, and every thread applies the rank-1 update.
// Tier 2 (L > 128): blocked Gauss-Jordan over column panels of width NB on a
//   working copy Z.  One workgroup eliminates a panel (all L rows x NB
//   columns in registers) and emits the panel's transformation U' = U - E
//   (E = unit entries at the pivot rows) and the pivot rows Q of the other
//   columns; those columns are then updated by one grouped matrix-core
//   product  Z[:, out] += U' * Q.  A final pass writes the permuted result.
//   Up to order 512 the panel's search kernel is the same 2-D kernel, its
//   speculative elimination a column-block kernel, and an FP64 leaf is not
//   copied first: the first panel and its product read the leaf's input in
//   place.  Above 512 a rotating-slot panel kernel works on narrower panels
//   and the input is copied into Z.
//
// Speculation: every kernel up to order 512 first tries the diagonal pivots,
// checks each choice exactly and falls back to its search when a check fails
// (gj2d_any); the result is the search's bit for bit either way.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <cstdlib>

#include "spin_kernels.hpp"

namespace spin {
namespace {

__device__ inline bool better(double ov, int oi, double v, int i) {
    return ov > v || (ov == v && oi < i);
}

// ---------------------------------------------------------- wave helpers ---
// DPP control words (GFX9 encoding).
constexpr int kDppQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;

// Every control used here reads a lane of the same row, so all lanes are
// written and the move needs no initial value.
template <int CTRL>
__device__ inline double dpp_f64(double x) {
    const int lo =
        __builtin_amdgcn_mov_dpp((int)(__double_as_longlong(x) & 0xffffffff), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(__double_as_longlong(x) >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double readlane_f64(double x, int lane) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Maximum over the 64 lanes of a wave (every lane receives it).  Keys are
// finite (no NaN), so max is exact and order independent.
__device__ inline double wave_max(double x) {
    x = fmax(x, dpp_f64<kDppQuadXor1>(x));
    x = fmax(x, dpp_f64<kDppQuadXor2>(x));
    x = fmax(x, dpp_f64<kDppHalfMirror>(x));
    x = fmax(x, dpp_f64<kDppMirror>(x));
    const double a = fmax(readlane_f64(x, 0), readlane_f64(x, 16));
    const double b = fmax(readlane_f64(x, 32), readlane_f64(x, 48));
    return fmax(a, b);
}

// ------------------------------------------------------------ 2-D kernel ---
// One workgroup of 16*TR threads eliminates a block of L <= TR*RR rows and
// nb <= 16*RC columns held in registers: thread (tr, tc) owns rows tr + TR*r
// and columns tc + 16*q.  A step:
//   1. the owners of column c publish it to LDS (its register slot restarts
//      as the implicit unit column);
//   2. every wave finds the pivot redundantly: key |v| of each unused row
//      (-0.5 for non-finite values, -1 for used rows), a DPP max over the
//      wave, and the smallest row index holding the maximum via ballots;
//   3. the owners of the pivot row publish it scaled by 1/pivot;
//   4. every thread applies the rank-1 update to its registers.
// WHOLE = true : the block is a whole leaf (columns = rows), read from `in`
//                and written to `out` with the pivot permutation applied.
// WHOLE = false: the block is one column panel of a blocked elimination
//                whose working copy is Z (the first panel of an FP64 leaf
//                reads the leaf's input instead); the kernel writes the panel
//                to Z, its transformation U' = U - E, the used-row flags and
//                the gathered pivot rows Q of the other columns.
struct LeafArgs {
    const void *in;
    int64_t ldi;
    void *out;
    int64_t ldo;
    int L, col0;
    int *status;
    // panel mode
    double *Z;
    int64_t ldz;
    int k0, nb;
    int *used, *rsel;
    double *Up, *Q;
    // Speculation switch of the inversion (nullable): nonzero lets the kernel
    // try the speculative elimination first; a failed attempt sets it to 0 so
    // that the later leaves of the same inversion go straight to the search.
    int *spec;
    // Two-workgroup panels: this panel's exchange area (multipliers and
    // inverse pivots of its 64 steps), its verdict and decision words, and
    // the number of polls after which a wait for the other workgroup gives
    // up (and the panel falls back to the search).
    double *xg;
    int *xc;
    int duo_spin;
};

template <int TR, int RR, int RC, bool WHOLE, typename TI, typename TO>
__device__ __attribute__((always_inline)) inline void gj2d_run(const LeafArgs &a) {
    constexpr int NT = 16 * TR;
    constexpr int LMAX = TR * RR;
    constexpr int NBMAX = 16 * RC;
    constexpr int CPL = LMAX / 64;
    static_assert(CPL * 64 == LMAX, "rows must cover whole waves");
    __shared__ double colbuf[2][LMAX];
    // Panels: the multipliers, i.e. column c with 0 at the pivot row (the
    // pivot row is scaled in place instead), so the update needs no select.
    __shared__ double fbuf[2][LMAX];
    __shared__ double rowbuf[2][NBMAX];
    __shared__ int pivstep[LMAX];  // step at which a row was the pivot, or -1
    __shared__ int prow_s[NBMAX];  // pivot row of each step
    // Thread t holds rows tr + TR r of columns tc + 16 q.  Whole leaves put
    // the 16 threads of a row group in one wave (t = 16 tr + tc), so one wave
    // publishes the pivot row.  Panels put TR consecutive rows of one column
    // in consecutive lanes (t = TR tc + tr): their loads of the panel and
    // stores of Z and Up then cover whole column segments, which outweighs
    // spreading the pivot-row publication over all waves.
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int tr = WHOLE ? t >> 4 : t % TR, tc = WHOLE ? t & 15 : t / TR;
    const int L = a.L;
    const int k0 = WHOLE ? 0 : a.k0;
    const int nb = WHOLE ? a.L : a.nb;

    for (int i = t; i < LMAX; i += NT) pivstep[i] = -1;
    // Panel mode reads the panel and the pivot rows from `in` when it is set
    // (the first panel of an FP64 leaf, straight from the leaf's input) and
    // from Z otherwise; it always writes Z.
    const double *src = WHOLE ? nullptr : (a.in ? static_cast<const double *>(a.in) : a.Z);
    const int64_t lds = WHOLE ? 0 : (a.in ? a.ldi : a.ldz);
    double z[RR][RC];
#pragma unroll
    for (int r = 0; r < RR; ++r)
#pragma unroll
        for (int q = 0; q < RC; ++q) {
            const int row = tr + TR * r, col = tc + 16 * q;
            double v = 0.0;
            if (row < L && col < nb) {
                if (WHOLE)
                    v = (double)static_cast<const TI *>(a.in)[row + (int64_t)col * a.ldi];
                else
                    v = src[row + (int64_t)(k0 + col) * lds];
            }
            z[r][q] = v;
        }
    // Bit j: row lane + 64 j is used (or beyond L).  A per-lane integer keeps
    // the flags in a vector register; as bool arrays they become wave-wide
    // lane masks whose per-step merges cost scalar instructions, and the
    // scalar unit is shared by the CU's SIMDs.
    int usdm = 0;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const int row = lane + 64 * j;
        if (row >= L || (!WHOLE && k0 > 0 && a.used[row] != 0)) usdm |= 1 << j;
    }
    int bad = 0;
    // Panels gather the pivot rows of the columns outside the panel during
    // the steps: thread t < L - nb owns outside column gj, loads its entry in
    // row p at step c and stores it to Q one step later, when the load has
    // long completed.  The panel kernel never writes those columns, so the
    // values are the ones a gather after the last step would read.
    static_assert(WHOLE || LMAX <= NT, "one gathering thread per outside column");
    const bool gth = !WHOLE && nb < L && t < L - nb;
    const int gj = t < k0 ? t : t + nb;
    const double *gsrc = WHOLE ? nullptr : src + (int64_t)gj * lds;
    double *gdst = WHOLE ? nullptr : a.Q + (int64_t)gj * nb;
    double gv = 0.0;
    // All initial loads complete here (vmcnt(0), the other counters left at
    // their maximum).  Otherwise the first uses of z inside the loop carry a
    // wait for every outstanding load, which would include the gathered one.
    if constexpr (!WHOLE) __builtin_amdgcn_s_waitcnt(0xF70);
    __syncthreads();

#pragma unroll
    for (int cb = 0; cb < RC; ++cb) {
        for (int cc = 0; cc < 16; ++cc) {
            const int c = cb * 16 + cc;
            if (c >= nb) break;
            const int buf = c & 1;
            if (tc == cc) {
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    colbuf[buf][tr + TR * r] = z[r][cb];
                    if (!WHOLE) fbuf[buf][tr + TR * r] = z[r][cb];
                    z[r][cb] = 0.0;
                }
            }
            __syncthreads();
            double key[CPL];
            // Panels keep the non-finite flag as a bool, test it in thread 0's
            // wave only and take p mod TR unsigned; whole leaves measured
            // 1.8 % slower with those forms, so they keep the int forms.
            int nf = 0;
#pragma unroll
            for (int j = 0; j < CPL; ++j) {
                const double av = fabs(colbuf[buf][lane + 64 * j]);
                const bool fin = av <= DBL_MAX;
                const bool u = (usdm >> j) & 1;
                if (WHOLE)
                    nf |= (!u && !fin);
                else
                    nf = nf || (!u && !fin);
                key[j] = u ? -1.0 : (fin ? av : -0.5);
            }
            double lm = key[0];
#pragma unroll
            for (int j = 1; j < CPL; ++j) lm = fmax(lm, key[j]);
            const double best = wave_max(lm);
            int p = 0;
#pragma unroll
            for (int j = CPL - 1; j >= 0; --j) {
                const unsigned long long m = __ballot(key[j] == best);
                if (m) p = 64 * j + __builtin_ctzll(m);
            }
            p = __builtin_amdgcn_readfirstlane(p);
            if (WHOLE) {
                if ((__any(nf) || !(best > 0.0)) && bad == 0) bad = c + 1;
            } else if (wave == 0 && bad == 0 && (__any(nf) || !(best > 0.0))) {
                bad = c + 1;  // only thread 0 reports the failing step
            }
            usdm |= (p & 63) == lane ? 1 << (p >> 6) : 0;
            const double pinv = 1.0 / colbuf[buf][p];
            if (tr == (WHOLE ? p % TR : (int)((unsigned)p % TR))) {
                const int rp = WHOLE ? p / TR : (int)((unsigned)p / TR);
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    if (r == rp) {
                        if (WHOLE) {
#pragma unroll
                            for (int q = 0; q < RC; ++q) {
                                rowbuf[buf][tc + 16 * q] = z[r][q] * pinv;
                                z[r][q] = 0.0;
                            }
                            if (tc == cc) rowbuf[buf][c] = pinv;
                        } else {
                            // scaled in place; its multiplier becomes 0
#pragma unroll
                            for (int q = 0; q < RC; ++q) {
                                z[r][q] = z[r][q] * pinv;
                                rowbuf[buf][tc + 16 * q] = z[r][q];
                            }
                            if (tc == cc) {
                                rowbuf[buf][c] = pinv;
                                z[r][cb] = pinv;
                                fbuf[buf][p] = 0.0;
                            }
                        }
                    }
                }
            }
            if (t == 0) {
                pivstep[p] = c;
                prow_s[c] = p;
            }
            __syncthreads();
            if (gth) {
                if (c > 0) gdst[c - 1] = gv;
                gv = gsrc[p];
            }
            double f[RR], rv[RC];
#pragma unroll
            for (int r = 0; r < RR; ++r)
                f[r] = WHOLE ? ((tr + TR * r == p) ? -1.0 : colbuf[buf][tr + TR * r]) : fbuf[buf][tr + TR * r];
#pragma unroll
            for (int q = 0; q < RC; ++q) rv[q] = rowbuf[buf][tc + 16 * q];
#pragma unroll
            for (int r = 0; r < RR; ++r)
#pragma unroll
                for (int q = 0; q < RC; ++q) z[r][q] = fma(-f[r], rv[q], z[r][q]);
        }
    }
    __syncthreads();
    if (WHOLE) {
        // X[rinv[i]][r[c]] = Z[i][c]  with r[c] = prow_s[c], rinv[i] = pivstep[i]
        TO *out = static_cast<TO *>(a.out);
#pragma unroll
        for (int r = 0; r < RR; ++r)
#pragma unroll
            for (int q = 0; q < RC; ++q) {
                const int row = tr + TR * r, col = tc + 16 * q;
                if (row < L && col < L) {
                    const int ri = pivstep[row], rc = prow_s[col];
                    if ((unsigned)ri < (unsigned)L && (unsigned)rc < (unsigned)L)
                        out[ri + (int64_t)rc * a.ldo] = (TO)z[r][q];
                }
            }
    } else {
#pragma unroll
        for (int r = 0; r < RR; ++r)
#pragma unroll
            for (int q = 0; q < RC; ++q) {
                const int row = tr + TR * r, col = tc + 16 * q;
                if (row < L && col < nb) {
                    a.Z[row + (int64_t)(k0 + col) * a.ldz] = z[r][q];
                    a.Up[row + (int64_t)col * L] = z[r][q] - ((pivstep[row] == col) ? 1.0 : 0.0);
                }
            }
        for (int c = t; c < nb; c += NT) a.rsel[k0 + c] = prow_s[c];
        for (int row = t; row < L; row += NT) {
            if (k0 == 0)
                a.used[row] = pivstep[row] >= 0 ? 1 : 0;
            else if (pivstep[row] >= 0)
                a.used[row] = 1;
        }
        if (gth) gdst[nb - 1] = gv;
    }
    if (t == 0 && bad) atomicMin(a.status, a.col0 + k0 + bad);
}

// ------------------------------------------ speculative whole-leaf kernel ---
// The elimination of gj2d_run for blocks whose partial-pivoting choice at
// step k is row k itself, as it is at every step for strictly diagonally
// dominant blocks (their Schur complements stay dominant) and, in practice,
// for well-conditioned positive-definite ones.  Each step takes that row as
// its pivot and checks the choice exactly: the step stands when the pivot is
// finite and nonzero and no unused row holds a larger magnitude or a
// non-finite value.  As long as every earlier step stood, the unused rows are
// exactly the rows below the pivot, so a tie goes to the pivot row, which is
// what the search's smallest-index rule picks.
//
// With the pivot row known in advance the search leaves the dependent chain,
// and so does one barrier: once step c is applied, the owners of column c+1
// publish its multipliers and the owners of row c+1 (one wave, which also
// holds the pivot) the scaled pivot row, and after one barrier every thread
// applies step c+1.  Every element goes through the same operations as in
// gj2d_run (the same division, products and fused multiply-adds), so when
// every check passes the outputs are gj2d_run's bit for bit.  They are written
// only then.  Returns whether every check passed (the same in every thread);
// on false nothing has been written.  Whole leaves only (panels have their
// own kernels below).
template <int TR, int RR, int RC, typename TI, typename TO>
__device__ __attribute__((always_inline)) inline bool gj2d_spec(const LeafArgs &a) {
    constexpr int LMAX = TR * RR;
    constexpr int NBMAX = 16 * RC;
    static_assert(TR == 16 || TR == 32, "row groups of 16 or 32 threads");
    // Shared arrays are indexed by register slot, not by row: entry tr + TR r
    // belongs to slot r of the threads with that tr (the same map in every
    // thread), so that every access is a per-thread base plus a constant.
    __shared__ double fbs[2][LMAX];   // multipliers of a step, -1 at its pivot row
    __shared__ double rws[2][NBMAX];  // its scaled pivot row
    __shared__ double pvs[2];         // |pivot|
    const int t = threadIdx.x, wave = t >> 6;
    const int tr = t >> 4, tc = t & 15;
    const int L = a.L;

    double z[RR][RC];
#pragma unroll
    for (int r = 0; r < RR; ++r)
#pragma unroll
        for (int q = 0; q < RC; ++q) {
            const int row = tr + TR * r, col = tc + 16 * q;
            z[r][q] = (row < L && col < L) ? (double)static_cast<const TI *>(a.in)[row + (int64_t)col * a.ldi]
                                           : 0.0;
        }
    bool viol = false;
    double *const fbt = &fbs[0][tr];
    double *const rwt = &rws[0][tc];

    // One step c = 16 cb + cc, LDS buffer B = c & 1: publication (its column
    // and pivot row are final once step c - 1 is applied), one barrier, the
    // check and the update.  cb and B are constants after unrolling.
    auto step = [&](const int cb, const int cc, const int B) {
        const int PR = (16 * cb) / TR;       // register slot of the pivot row
        const int pt = (16 * cb) % TR + cc;  // its owners' tr
        // the 16 owners of row c are lanes 16 pt .. 16 pt + 15 of one wave
        if (wave == (16 * pt) >> 6) {
            const double piv = readlane_f64(z[PR][cb], (16 * pt + cc) & 63);
            if (tr == pt) {
                const double pinv = 1.0 / piv;
#pragma unroll
                for (int q = 0; q < RC; ++q) {
                    rwt[B * NBMAX + 16 * q] = (q == cb && tc == cc) ? pinv : z[PR][q] * pinv;
                    z[PR][q] = 0.0;  // the update adds the scaled row (multiplier -1)
                }
                if (tc == cc) pvs[B] = fabs(piv);
            }
        }
        if (tc == cc) {
#pragma unroll
            for (int r = 0; r < RR; ++r) {
                fbt[B * LMAX + TR * r] = (r == PR && tr == pt) ? -1.0 : z[r][cb];
                z[r][cb] = 0.0;
            }
        }
        __syncthreads();
        double f[RR], rv[RC];
#pragma unroll
        for (int r = 0; r < RR; ++r) f[r] = fbt[B * LMAX + TR * r];
#pragma unroll
        for (int q = 0; q < RC; ++q) rv[q] = rwt[B * NBMAX + 16 * q];
        // check of step c: the pivot, then the unused rows of this thread
        const double apiv = pvs[B];
        bool v = !(apiv > 0.0) || !(apiv <= DBL_MAX);
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            if (r < PR) continue;  // rows before the pivot: used
            const bool used = (r == PR) && (tr <= pt);
            v = v || (!used && !(fabs(f[r]) <= apiv));
        }
        viol = viol || v;
#pragma unroll
        for (int r = 0; r < RR; ++r)
#pragma unroll
            for (int q = 0; q < RC; ++q) z[r][q] = fma(-f[r], rv[q], z[r][q]);
    };

#pragma unroll
    for (int cb = 0; cb < RC; ++cb) {
        for (int cc = 0; cc < 16; cc += 2) {
            if (16 * cb + cc >= L) break;
            step(cb, cc, 0);
            if (16 * cb + cc + 1 >= L) break;
            step(cb, cc + 1, 1);
        }
    }
    if (__syncthreads_or(viol)) return false;

    TO *out = static_cast<TO *>(a.out);
#pragma unroll
    for (int r = 0; r < RR; ++r)
#pragma unroll
        for (int q = 0; q < RC; ++q) {
            const int row = tr + TR * r, col = tc + 16 * q;
            if (row < L && col < L) out[row + (int64_t)col * a.ldo] = (TO)z[r][q];
        }
    return true;
}

// -------------------------------------- speculative column-block panel ---
// The speculative elimination of a panel (nb <= 64 columns from k0, a
// multiple of 64, L <= 64 RR rows) with one barrier per column block instead
// of one per step.  Each of the NW waves holds CW = 64 / NW panel columns in
// full: lane l, slot i of wave w holds row l + 64 ((i + rot) mod RR),
// rot = k0 / 64, of columns CW w .. CW w + CW - 1, so the pivot row k0 + c of
// step c sits in slot 0 of lane c and the multipliers of step c are one
// column of a single wave.  Wave s runs the steps of its own columns alone,
// taking the pivot row from lane c with readlane, and publishes each step's
// multipliers, pivot and inverse pivot; after one barrier every other wave
// applies those steps to its own columns, the pivot row again read from its
// lane c, and wave s + NW/2 checks them against every unused row.  Wave s + 1
// has then applied every earlier step to its columns and runs its own; it is
// the critical path and runs at raised issue priority meanwhile.
// Each element goes through the operations of gj2d_run in the same order
// (the pivot row scaled by the inverse pivot, the multipliers taken before
// the step, the pivot column restarting from 0, one fused multiply-add per
// step), so when every pivot check passes the outputs are gj2d_run's bit for
// bit.  Returns whether every check passed; on false nothing is written.
// Used for panels of 257 .. 512 rows; smaller ones take wpanel_pipe below.
template <int RR, int NW>
__device__ __attribute__((always_inline)) inline bool wpanel_spec(const LeafArgs &a) {
    constexpr int NT = 64 * NW, CW = 64 / NW;  // threads, columns per wave
    static_assert(CW * NW == 64, "the waves cover 64 columns");
    __shared__ double fpub[2][RR][CW][64];  // multipliers of a column block's steps
    __shared__ double ppub[2][2][CW];       // their inverse pivots and pivots
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int L = a.L, k0 = a.k0, nb = a.nb;
    const double *src = a.in ? static_cast<const double *>(a.in) : a.Z;
    const int64_t lds = a.in ? a.ldi : a.ldz;
    const int rot = k0 >> 6;
    bool viol = (k0 & 63) != 0 || L > 64 * RR || nb > 64 || nb < 1;
    if (viol) return false;  // the same in every thread
    int rowr[RR];
    int rel[RR];  // row - k0 for rows inside the leaf from k0 on, else -1
#pragma unroll
    for (int i = 0; i < RR; ++i) {
        rowr[i] = lane + 64 * ((i + rot) % RR);
        rel[i] = (i + rot < RR && rowr[i] < L) ? lane + 64 * i : -1;
    }
    double z[RR][CW];
#pragma unroll
    for (int i = 0; i < RR; ++i)
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            const int col = CW * w + j;
            z[i][j] = (rowr[i] < L && col < nb) ? src[rowr[i] + (int64_t)(k0 + col) * lds] : 0.0;
        }
    // the rows before the panel must be the used ones and no other
    if (w == 0 && k0 > 0) {
#pragma unroll
        for (int i = 0; i < RR; ++i)
            if (rowr[i] < L && ((a.used[rowr[i]] != 0) != (rowr[i] < k0))) viol = true;
    }

    // Step c = 8w + j on the wave's own columns (j a constant after
    // unrolling); no branch, so that consecutive steps overlap.
    auto own_step = [&](const int j, const int B) {
        const int c = CW * w + j;
        const double piv = readlane_f64(z[0][j], c);
        const double pinv = 1.0 / piv;
        const bool pl = lane == c;
        double rv[CW], f[RR];
#pragma unroll
        for (int jj = 0; jj < CW; ++jj) rv[jj] = (jj == j) ? pinv : readlane_f64(z[0][jj], c) * pinv;
#pragma unroll
        for (int i = 0; i < RR; ++i) {
            f[i] = (i == 0 && pl) ? 0.0 : z[i][j];
            fpub[B][i][j][lane] = f[i];
        }
        if (lane == 0) {
            ppub[B][0][j] = pinv;
            ppub[B][1][j] = piv;
        }
        // the pivot row (multiplier 0) restarts from the scaled row, the
        // pivot column from 0
#pragma unroll
        for (int i = 0; i < RR; ++i)
#pragma unroll
            for (int jj = 0; jj < CW; ++jj) {
                double base = (jj == j) ? 0.0 : z[i][jj];
                if (i == 0) base = pl ? rv[jj] : base;
                z[i][jj] = fma(-f[i], rv[jj], base);
            }
    };
    // Step c = 8s + j of another wave's block, applied to this wave's columns,
    // with the step's multipliers f and inverse pivot pinv already loaded.
    auto replay_step = [&](const int s, const int j, const double (&f)[RR], const double pinv) {
        const int c = CW * s + j;
        const bool pl = lane == c;
        double rv[CW];
#pragma unroll
        for (int jj = 0; jj < CW; ++jj) rv[jj] = readlane_f64(z[0][jj], c) * pinv;
#pragma unroll
        for (int i = 0; i < RR; ++i)
#pragma unroll
            for (int jj = 0; jj < CW; ++jj) z[i][jj] = fma(-f[i], rv[jj], z[i][jj]);
        if (pl) {
#pragma unroll
            for (int jj = 0; jj < CW; ++jj) z[0][jj] = fma(-0.0, rv[jj], rv[jj]);
        }
    };
    // A block's replay reads each step's multipliers one step ahead, so the
    // LDS latency overlaps the previous step's update.
    auto replay_block = [&](const int s, const int B) {
        double fc[RR], pc = ppub[B][0][0];
#pragma unroll
        for (int i = 0; i < RR; ++i) fc[i] = fpub[B][i][0][lane];
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            if (CW * s + j >= nb) break;
            double fn[RR], pn = 0.0;
            if (j + 1 < CW) {
                pn = ppub[B][0][j + 1];
#pragma unroll
                for (int i = 0; i < RR; ++i) fn[i] = fpub[B][i][j + 1][lane];
            }
            replay_step(s, j, fc, pc);
            if (j + 1 < CW) {
                pc = pn;
#pragma unroll
                for (int i = 0; i < RR; ++i) fc[i] = fn[i];
            }
        }
    };
    // The checks of block s: each pivot finite and nonzero, and no unused row
    // (rel > c; the pivot row's published multiplier is 0) larger in
    // magnitude or not finite.
    auto check_block = [&](const int s, const int B) {
        bool v = false;
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            const int c = CW * s + j;
            if (c >= nb) break;
            const double apiv = fabs(ppub[B][1][j]);
            v = v || !(apiv > 0.0) || !(apiv <= DBL_MAX);
#pragma unroll
            for (int i = 0; i < RR; ++i) v = v || (rel[i] > c && !(fabs(fpub[B][i][j][lane]) <= apiv));
        }
        viol = viol || v;
    };

    const int nblk = (nb + CW - 1) / CW;
    for (int s = 0; s < nblk; ++s) {
        const int B = s & 1;
        if (w == s) {
#pragma unroll
            for (int j = 0; j < CW; ++j)
                if (CW * s + j < nb) own_step(j, B);
            __builtin_amdgcn_s_setprio(0);
        }
        __syncthreads();
        if (w == s + 1) __builtin_amdgcn_s_setprio(2);
        if (w != s && CW * w < nb) replay_block(s, B);
        if (w == (s + NW / 2) % NW) check_block(s, B);
    }
    if (__syncthreads_or(viol)) return false;

#pragma unroll
    for (int i = 0; i < RR; ++i)
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            const int row = rowr[i], col = CW * w + j;
            if (row < L && col < nb) {
                a.Z[row + (int64_t)(k0 + col) * a.ldz] = z[i][j];
                a.Up[row + (int64_t)col * L] = z[i][j] - ((row == k0 + col) ? 1.0 : 0.0);
            }
        }
    for (int c = t; c < nb; c += NT) a.rsel[k0 + c] = k0 + c;
    for (int row = t; row < L; row += NT) {
        const bool piv = row >= k0 && row < k0 + nb;
        if (k0 == 0)
            a.used[row] = piv ? 1 : 0;
        else if (piv)
            a.used[row] = 1;
    }
    // pivot rows of the columns outside the panel: rows k0 .. k0 + nb - 1
    const int nout = L - nb;
    for (int e = t; e < nb * nout; e += NT) {
        const int c = e % nb, j = e / nb;
        const int gj = j < k0 ? j : j + nb;
        a.Q[c + (int64_t)gj * nb] = src[(k0 + c) + (int64_t)gj * lds];
    }
    return true;
}

// The same elimination for panels of up to 256 rows with a flag per step
// instead of a barrier per column block (k0 a multiple of 32 here, and the
// pivot row k0 + c in slot 0 of lane k0 mod 64 + c).  LDS holds the multipliers of all
// 64 steps (128 KB), so nothing is overwritten: the owner of step c
// publishes its multipliers, pivot and inverse pivot and then raises the
// step's flag, and every other wave applies step c as soon as it sees the
// flag.  Waves run the steps in order, and a step only waits for steps of
// lower-numbered waves, so every wait ends.  Issue priority goes by distance
// to ownership (the owner of the running block, then the next two owners),
// and the checks of block b are done by a wave that replays it anyway
// (b + 4, else 0; for b = 0 and a panel of at most eight columns, wave 1,
// which then only follows the steps).
template <int RR>
__device__ __attribute__((always_inline)) inline bool wpanel_pipe(const LeafArgs &a) {
    constexpr int NW = 8, NT = 64 * NW, CW = 64 / NW;  // waves, threads, columns per wave
    static_assert(RR <= 4, "the multipliers of 64 steps fill 128 KB of LDS at 256 rows");
    __shared__ double fst[64][RR][64];  // multipliers of each step, by slot and lane
    __shared__ double pst[2][64];       // inverse pivot and pivot of each step
    __shared__ int rdy[64];             // step published
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int L = a.L, k0 = a.k0, nb = a.nb;
    const double *src = a.in ? static_cast<const double *>(a.in) : a.Z;
    const int64_t lds = a.in ? a.ldi : a.ldz;
    // slot 0 of lane o + c holds row k0 + c, o = k0 mod 64 (0, or 32 for
    // 32-column panels)
    const int rot = k0 >> 6, o = k0 & 63;
    bool viol = o + nb > 64 || L > 64 * RR || nb < 1;
    if (viol) return false;  // the same in every thread
    if (t < 64) rdy[t] = 0;
    int rowr[RR];
    int rel[RR];  // row - k0 for rows inside the leaf (negative before k0), else -1
#pragma unroll
    for (int i = 0; i < RR; ++i) {
        rowr[i] = lane + 64 * ((i + rot) % RR);
        rel[i] = (i + rot < RR && rowr[i] < L) ? lane + 64 * i - o : -1;
    }
    double z[RR][CW];
#pragma unroll
    for (int i = 0; i < RR; ++i)
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            const int col = CW * w + j;
            z[i][j] = (rowr[i] < L && col < nb) ? src[rowr[i] + (int64_t)(k0 + col) * lds] : 0.0;
        }
    const int nout = L - nb;
    // pivot rows of the columns outside the panel (rows k0 .. k0 + nb - 1,
    // gathered into Q once every check has passed), loaded now so that the
    // loads complete during the elimination
    constexpr int QPT = 4096 * (RR - 1) / NT;  // nb (L - nb) <= 64 (64 RR - 64)
    double qv[QPT > 0 ? QPT : 1];
#pragma unroll
    for (int r = 0; r < QPT; ++r) {
        const int e = t + NT * r, c = e % nb, j = e / nb;
        const int gj = j < k0 ? j : j + nb;
        qv[r] = e < nb * nout ? src[(k0 + c) + (int64_t)gj * lds] : 0.0;
    }
    if (w == 0 && k0 > 0) {
#pragma unroll
        for (int i = 0; i < RR; ++i)
            if (rowr[i] < L && ((a.used[rowr[i]] != 0) != (rowr[i] < k0))) viol = true;
    }
    __syncthreads();  // the flags are cleared

    // The pivot row of a step first takes the scaled row; its multiplier is
    // 0, so the step's fused multiply-add turns it into fma(-0, rv, rv), the
    // value gj2d_run gives it.
    auto own_step = [&](const int j) {
        const int c = CW * w + j, pc = o + c;  // step, pivot lane
        const double piv = readlane_f64(z[0][j], pc);
        const double pinv = 1.0 / piv;
        const bool pl = lane == pc;
        double rv[CW], f[RR];
#pragma unroll
        for (int jj = 0; jj < CW; ++jj) rv[jj] = (jj == j) ? pinv : readlane_f64(z[0][jj], pc) * pinv;
#pragma unroll
        for (int i = 0; i < RR; ++i) {
            f[i] = (i == 0 && pl) ? 0.0 : z[i][j];
            fst[c][i][lane] = f[i];
        }
        if (lane == 0) {
            pst[0][c] = pinv;
            pst[1][c] = piv;
        }
#pragma unroll
        for (int i = 0; i < RR; ++i) z[i][j] = 0.0;  // the pivot column restarts from 0
        if (pl) {
#pragma unroll
            for (int jj = 0; jj < CW; ++jj) z[0][jj] = rv[jj];
        }
#pragma unroll
        for (int i = 0; i < RR; ++i)
#pragma unroll
            for (int jj = 0; jj < CW; ++jj) z[i][jj] = fma(-f[i], rv[jj], z[i][jj]);
        // the flag last: its release orders it after the stores above
        if (lane == 0) __hip_atomic_store(&rdy[c], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    auto wait_step = [&](const int c) {
        while (__hip_atomic_load(&rdy[c], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == 0)
            __builtin_amdgcn_s_sleep(1);
    };
    // The checks of step c: the pivot finite and nonzero, and no unused row
    // (rel > c; the pivot row's published multiplier is 0) larger in
    // magnitude or not finite.
    auto check = [&](const int c, const double (&f)[RR]) {
        const double apiv = fabs(pst[1][c]);
        bool v = !(apiv > 0.0) | !(apiv <= DBL_MAX);
#pragma unroll
        for (int i = 0; i < RR; ++i) v |= (rel[i] > c) & !(fabs(f[i]) <= apiv);
        viol |= v;
    };
    auto replay_step = [&](const int c, const bool chk) {
        const double pinv = pst[0][c];
        const bool pl = lane == o + c;
        double rv[CW], f[RR];
#pragma unroll
        for (int i = 0; i < RR; ++i) f[i] = fst[c][i][lane];
#pragma unroll
        for (int jj = 0; jj < CW; ++jj) rv[jj] = readlane_f64(z[0][jj], o + c) * pinv;
        if (pl) {
#pragma unroll
            for (int jj = 0; jj < CW; ++jj) z[0][jj] = rv[jj];
        }
#pragma unroll
        for (int i = 0; i < RR; ++i)
#pragma unroll
            for (int jj = 0; jj < CW; ++jj) z[i][jj] = fma(-f[i], rv[jj], z[i][jj]);
        if (chk) check(c, f);
    };
    auto check_step = [&](const int c) {
        double f[RR];
#pragma unroll
        for (int i = 0; i < RR; ++i) f[i] = fst[c][i][lane];
        check(c, f);
    };

    const bool cols = CW * w < nb;
    const int nblk = (nb + CW - 1) / CW;
    for (int b = 0; b < nblk; ++b) {
        // issue priority by distance to ownership: the owner first, then the
        // waves whose blocks come next
        if (w == b)
            __builtin_amdgcn_s_setprio(3);
        else if (w == b + 1)
            __builtin_amdgcn_s_setprio(2);
        else if (w == b + 2)
            __builtin_amdgcn_s_setprio(1);
        // the checking wave of block b (see above)
        int cw = (b + NW / 2) % NW;
        if (CW * cw >= nb) cw = b == 0 ? 1 : 0;
        const bool chk = w == cw;
        if (w == b) {
#pragma unroll
            for (int j = 0; j < CW; ++j)
                if (CW * b + j < nb) own_step(j);
            __builtin_amdgcn_s_setprio(0);
        } else if (cols) {
            for (int c = CW * b; c < CW * b + CW && c < nb; ++c) {
                wait_step(c);
                replay_step(c, chk);
            }
        } else if (chk) {
            for (int c = CW * b; c < CW * b + CW && c < nb; ++c) {
                wait_step(c);
                check_step(c);
            }
        }
    }
    // Outputs the search rewrites in full if a check failed, and that it does
    // not read, are stored before the vote: U' always, the panel's columns of
    // Z when the panel is read from the leaf's input.
    const bool zout = a.in != nullptr;
#pragma unroll
    for (int i = 0; i < RR; ++i)
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            const int row = rowr[i], col = CW * w + j;
            if (row < L && col < nb) {
                a.Up[row + (int64_t)col * L] = z[i][j] - ((row == k0 + col) ? 1.0 : 0.0);
                if (zout) a.Z[row + (int64_t)(k0 + col) * a.ldz] = z[i][j];
            }
        }
    if (__syncthreads_or(viol)) return false;

    if (!zout) {
#pragma unroll
        for (int i = 0; i < RR; ++i)
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                const int row = rowr[i], col = CW * w + j;
                if (row < L && col < nb) a.Z[row + (int64_t)(k0 + col) * a.ldz] = z[i][j];
            }
    }
    for (int c = t; c < nb; c += NT) a.rsel[k0 + c] = k0 + c;
    for (int row = t; row < L; row += NT) {
        const bool piv = row >= k0 && row < k0 + nb;
        if (k0 == 0)
            a.used[row] = piv ? 1 : 0;
        else if (piv)
            a.used[row] = 1;
    }
#pragma unroll
    for (int r = 0; r < QPT; ++r) {
        const int e = t + NT * r, c = e % nb, j = e / nb;
        const int gj = j < k0 ? j : j + nb;
        if (e < nb * nout) a.Q[c + (int64_t)gj * nb] = qv[r];
    }
    return true;
}

// ------------------------------------------------- two-workgroup panel ---
// The pipelined elimination of a full 64-column panel of at most 256 rows on
// two workgroups (two CUs), each holding 32 of its columns (eight waves of
// four), so that each CU replays half of the steps' updates.  Workgroup h
// owns steps 32h .. 32h + 31 and runs them as wpanel_pipe does (LDS flags);
// the wave that owned the previous column block, which is then caught up and
// far from its next turn, stores each step's multipliers and inverse pivot
// to the panel's exchange area in device memory, and the other workgroup
// replays the step from there.
//
// The exchange area holds a signalling-NaN pattern before the panel (filled
// by leaf_duo_reset, or by the previous leaf's leaf_unpermute), so a value
// read back is either that pattern (not yet stored: read again) or the
// stored value: every 8-byte access is single-copy atomic, and no flag or
// ordering between stores is needed.  The loads and stores are device-
// coherent (agent scope), and the values of the step after next are loaded
// before the current step's update.
//
// Every wait is bounded.  Workgroup 0 posts a verdict on its own steps when
// they are done.  Workgroup 1 posts its verdict (all its checks passed, or
// not) and waits for workgroup 0's decision; workgroup 0 waits for that
// verdict, decides (commit only if both workgroups' checks passed and
// nothing timed out), and posts the decision.  Workgroup 0 is dispatched
// before workgroup 1, so a running workgroup 1 always gets a decision.
// Outputs that are not the search's input are stored before the decision
// where they cannot differ from the search's (workgroup 0's own, which it
// orders before the search; workgroup 1's once both verdicts passed); the
// rest on commit.  On abort workgroup 0 runs the search (leaf_duo).  A value
// equal to the pattern in the input only makes a wait run out, which aborts
// to the search.
constexpr unsigned long long kDuoPoison = 0x7FF4DEADBEEF0001ull;  // a signalling NaN
constexpr int kDuoSpin = 1 << 15;        // default polls of a data wait (about 64 clocks each and more)
constexpr int kDuoDecideSpin = 1 << 24;  // polls of workgroup 1's wait for the decision

__device__ inline double ld_agent(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_agent(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int ld_agent_i(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_agent_i(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline bool is_poison(double v) {
    return (unsigned long long)__double_as_longlong(v) == kDuoPoison;
}

// Doubles of one panel's exchange area at RR slots per lane: the 64 steps'
// multipliers [step][slot][lane], then the inverse pivots.
template <int RR>
constexpr int duo_panel_doubles() { return 64 * RR * 64 + 64; }
// Ints of one panel's decision area: verdict of workgroup 1, decision,
// verdict of workgroup 0 on its own steps.
constexpr int kDuoPanelInts = 3;

template <int RR>
__device__ __attribute__((always_inline)) inline bool wpanel_duo(const LeafArgs &a) {
    constexpr int NW = 8, NT = 512, CW = 4, HALF = 32;  // waves, threads, columns per wave, per workgroup
    static_assert(RR <= 4 && CW * NW == HALF, "two workgroups of 32 columns, at most 256 rows");
    __shared__ double fst[HALF][RR][64];  // this workgroup's steps' multipliers
    __shared__ double pst[2][HALF];       // their inverse pivots and pivots
    __shared__ int rdy[HALF];
    const int h = blockIdx.x;  // 0 or 1: columns and steps 32h .. 32h + 31
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int L = a.L, k0 = a.k0, nb = a.nb;
    const double *src = a.in ? static_cast<const double *>(a.in) : a.Z;
    const int64_t lds = a.in ? a.ldi : a.ldz;
    const int rot = k0 >> 6;
    if ((k0 & 63) != 0 || nb != 64 || L > 64 * RR || L <= 64 || !a.xg || !a.xc)
        return false;  // the same in both workgroups
    double *gf = a.xg;                // [64][RR][64]
    double *gp = a.xg + 64 * RR * 64;  // [64]
    int *verdict1 = a.xc, *decision = a.xc + 1, *verdict0 = a.xc + 2;
    if (t < HALF) rdy[t] = 0;
    int rowr[RR];
    int rel[RR];  // row - k0 for rows inside the leaf from k0 on, else -1
#pragma unroll
    for (int i = 0; i < RR; ++i) {
        rowr[i] = lane + 64 * ((i + rot) % RR);
        rel[i] = (i + rot < RR && rowr[i] < L) ? lane + 64 * i : -1;
    }
    double z[RR][CW];
#pragma unroll
    for (int i = 0; i < RR; ++i)
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            const int col = HALF * h + CW * w + j;
            z[i][j] = rowr[i] < L ? src[rowr[i] + (int64_t)(k0 + col) * lds] : 0.0;
        }
    // this workgroup's half of the pivot rows of the outside columns (Q)
    const int nout = L - nb, qtot = nb * nout, qhalf = (qtot + 1) / 2;
    constexpr int QPT = (4096 * (RR - 1) / 2 + NT - 1) / NT;
    double qv[QPT];
#pragma unroll
    for (int r = 0; r < QPT; ++r) {
        const int e = h * qhalf + t + NT * r, c = e % nb, j = e / nb;
        const int gj = j < k0 ? j : j + nb;
        qv[r] = (t + NT * r < qhalf && e < qtot) ? src[(k0 + c) + (int64_t)gj * lds] : 0.0;
    }
    // output stores: Q (this workgroup's half), U' with or without Z, Z
    auto store_q = [&]() {
#pragma unroll
        for (int r = 0; r < QPT; ++r) {
            const int e = h * qhalf + t + NT * r, c = e % nb, j = e / nb;
            const int gj = j < k0 ? j : j + nb;
            if (t + NT * r < qhalf && e < qtot) a.Q[c + (int64_t)gj * nb] = qv[r];
        }
    };
    auto store_up = [&](const bool with_z) {
#pragma unroll
        for (int i = 0; i < RR; ++i)
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                const int row = rowr[i], col = HALF * h + CW * w + j;
                if (row < L) {
                    a.Up[row + (int64_t)col * L] = z[i][j] - ((row == k0 + col) ? 1.0 : 0.0);
                    if (with_z) a.Z[row + (int64_t)(k0 + col) * a.ldz] = z[i][j];
                }
            }
    };
    auto store_z = [&]() {
#pragma unroll
        for (int i = 0; i < RR; ++i)
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                const int row = rowr[i], col = HALF * h + CW * w + j;
                if (row < L) a.Z[row + (int64_t)(k0 + col) * a.ldz] = z[i][j];
            }
    };
    // Z may be written before the decision only when the panel is read from
    // the leaf's input; otherwise Z holds the search's input.
    const bool z_early = a.in != nullptr;
    bool viol = false;
    if (h == 0 && w == 0 && k0 > 0) {
#pragma unroll
        for (int i = 0; i < RR; ++i)
            if (rowr[i] < L && ((a.used[rowr[i]] != 0) != (rowr[i] < k0))) viol = true;
    }
    __syncthreads();  // the flags are cleared

    auto own_step = [&](const int j) {
        const int c = HALF * h + CW * w + j, lc = c - HALF * h;
        const double piv = readlane_f64(z[0][j], c);
        const double pinv = 1.0 / piv;
        const bool pl = lane == c;
        double rv[CW], f[RR];
#pragma unroll
        for (int jj = 0; jj < CW; ++jj) rv[jj] = (jj == j) ? pinv : readlane_f64(z[0][jj], c) * pinv;
#pragma unroll
        for (int i = 0; i < RR; ++i) {
            f[i] = (i == 0 && pl) ? 0.0 : z[i][j];
            fst[lc][i][lane] = f[i];
        }
        if (lane == 0) {
            pst[0][lc] = pinv;
            pst[1][lc] = piv;
        }
#pragma unroll
        for (int i = 0; i < RR; ++i) z[i][j] = 0.0;  // the pivot column restarts from 0
        if (pl) {
#pragma unroll
            for (int jj = 0; jj < CW; ++jj) z[0][jj] = rv[jj];
        }
#pragma unroll
        for (int i = 0; i < RR; ++i)
#pragma unroll
            for (int jj = 0; jj < CW; ++jj) z[i][jj] = fma(-f[i], rv[jj], z[i][jj]);
        if (lane == 0) __hip_atomic_store(&rdy[lc], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    // the update of step c with its multipliers and inverse pivot
    auto apply = [&](const int c, const double (&f)[RR], const double pinv) {
        const bool pl = lane == c;
        double rv[CW];
#pragma unroll
        for (int jj = 0; jj < CW; ++jj) rv[jj] = readlane_f64(z[0][jj], c) * pinv;
        if (pl) {
#pragma unroll
            for (int jj = 0; jj < CW; ++jj) z[0][jj] = rv[jj];
        }
#pragma unroll
        for (int i = 0; i < RR; ++i)
#pragma unroll
            for (int jj = 0; jj < CW; ++jj) z[i][jj] = fma(-f[i], rv[jj], z[i][jj]);
    };
    // a local step of another wave, checked by the checking wave and passed
    // to the other workgroup by the forwarding wave
    auto local_step = [&](const int c, const bool chk, const bool fwd) {
        const int lc = c - HALF * h;
        while (__hip_atomic_load(&rdy[lc], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == 0)
            __builtin_amdgcn_s_sleep(1);
        const double pinv = pst[0][lc];
        double f[RR];
#pragma unroll
        for (int i = 0; i < RR; ++i) f[i] = fst[lc][i][lane];
        if (fwd) {
#pragma unroll
            for (int i = 0; i < RR; ++i) st_agent(&gf[((int64_t)c * RR + i) * 64 + lane], f[i]);
            if (lane == 0) st_agent(&gp[c], pinv);
        }
        apply(c, f, pinv);
        if (chk) {
            const double piv = pst[1][lc];
            const double apiv = fabs(piv);
            bool v = !(apiv > 0.0) | !(apiv <= DBL_MAX);
#pragma unroll
            for (int i = 0; i < RR; ++i) v |= (rel[i] > c) & !(fabs(f[i]) <= apiv);
            viol |= v;
        }
    };
    // The other workgroup's 32 steps c0 .. c0 + 31, each read back from the
    // exchange area once every lane sees stored values.  The values of the
    // next DEPTH steps are in flight while a step is applied: a device-
    // coherent load takes about as long as two steps' work, and a load issued
    // further ahead is more often issued before the value is stored and must
    // be repeated.  False if a wait ran out.
    constexpr int DEPTH = 2;
    auto remote_steps = [&](const int c0) -> bool {
        double rf[DEPTH][RR], rp[DEPTH];
        auto load = [&](const int c, double (&ff)[RR], double &pp) {
#pragma unroll
            for (int i = 0; i < RR; ++i) ff[i] = ld_agent(&gf[((int64_t)c * RR + i) * 64 + lane]);
            pp = ld_agent(&gp[c]);
        };
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) load(c0 + d, rf[d], rp[d]);
#pragma unroll
        for (int k = 0; k < HALF; ++k) {
            const int c = c0 + k, d = k % DEPTH;
            auto missing = [&](const double (&ff)[RR], const double pp) {
                bool bad = is_poison(pp);
#pragma unroll
                for (int i = 0; i < RR; ++i) bad |= is_poison(ff[i]);
                return __any(bad) != 0;
            };
            // The first look is outside any loop, so the loads of the later
            // steps stay in flight; a step not yet stored is read again into
            // other registers until it is.
            if (missing(rf[d], rp[d])) {
                double tf[RR], tp;
                int spins = 0;
                do {
                    if (++spins > a.duo_spin) return false;
                    __builtin_amdgcn_s_sleep(2);
                    load(c, tf, tp);
                } while (missing(tf, tp));
#pragma unroll
                for (int i = 0; i < RR; ++i) rf[d][i] = tf[i];
                rp[d] = tp;
            }
            double f[RR];
#pragma unroll
            for (int i = 0; i < RR; ++i) f[i] = rf[d][i];
            const double pinv = rp[d];
            if (k + DEPTH < HALF) load(c + DEPTH, rf[d], rp[d]);
            apply(c, f, pinv);
        }
        return true;
    };

    bool ok = true;
    // steps 0 .. 31 (workgroup 0's), then 32 .. 63 (workgroup 1's)
    for (int half = 0; half < 2; ++half) {
        if (half != h) {
            if (ok) ok = remote_steps(HALF * half);
            continue;
        }
        for (int b = 0; b < NW; ++b) {
            // issue priority by distance to ownership
            if (w == b)
                __builtin_amdgcn_s_setprio(3);
            else if (w == b + 1)
                __builtin_amdgcn_s_setprio(2);
            else if (w == b + 2)
                __builtin_amdgcn_s_setprio(1);
            // the previous owner, just caught up, forwards the block's steps
            const bool chk = w == (b + NW / 2) % NW;
            const bool fwd = w == (b + NW - 1) % NW;
            if (w == b) {
#pragma unroll
                for (int j = 0; j < CW; ++j) own_step(j);
                __builtin_amdgcn_s_setprio(0);
            } else {
                for (int c = HALF * h + CW * b; c < HALF * h + CW * b + CW; ++c) local_step(c, chk, fwd);
            }
        }
        if (h == 0) {
            // workgroup 0's steps are all checked: post the verdict on them,
            // and store this workgroup's half of Q (the search rewrites it)
            const bool bad0 = __syncthreads_or(viol);
            if (t == 0) st_agent_i(verdict0, bad0 ? 1 : 0);
            store_q();
        }
    }
    __builtin_amdgcn_s_setprio(0);
    if (h == 0) store_up(z_early);
    const bool bad = __syncthreads_or(viol || !ok);
    // Workgroup 1 stores U' and Q (and Z when the input is separate) before
    // the decision when every step of the panel passed its check: they then
    // equal what the search would write, bit for bit, so it does not matter
    // whether they land before or after the search's own stores.
    __shared__ int early_s;

    // verdict and decision
    __shared__ int commit_s;
    if (h == 1) {
        if (t == 0) {
            st_agent_i(verdict1, bad ? 1 : 0);
            int v = -1;
            for (int spins = 0; !bad && spins < a.duo_spin; ++spins) {
                v = ld_agent_i(verdict0);
                if (v >= 0) break;
                __builtin_amdgcn_s_sleep(8);
            }
            early_s = !bad && v == 0;
        }
        __syncthreads();
        if (early_s) {
            store_q();
            store_up(z_early);
        }
    }
    if (t == 0) {
        if (h == 1) {
            int d = -1;
            for (int spins = 0; spins < kDuoDecideSpin; ++spins) {
                d = ld_agent_i(decision);
                if (d >= 0) break;
                __builtin_amdgcn_s_sleep(8);
            }
            commit_s = d == 1;
        } else {
            int v = -1;
            for (int spins = 0; !bad && spins < a.duo_spin; ++spins) {
                v = ld_agent_i(verdict1);
                if (v >= 0) break;
                __builtin_amdgcn_s_sleep(8);
            }
            const bool c = !bad && v == 0;
            st_agent_i(decision, c ? 1 : 0);
            commit_s = c;
        }
    }
    __syncthreads();
    if (!commit_s) return false;

    if (h == 1 && !early_s) {
        store_q();
        store_up(true);
    } else if (!z_early) {
        store_z();
    }
    if (h == 0) {
        for (int c = t; c < nb; c += NT) a.rsel[k0 + c] = k0 + c;
        for (int row = t; row < L; row += NT) {
            const bool piv = row >= k0 && row < k0 + nb;
            if (k0 == 0)
                a.used[row] = piv ? 1 : 0;
            else if (piv)
                a.used[row] = 1;
        }
    }
    return true;
}

// A full panel of a leaf of order 129 .. 256 on two workgroups; on abort
// (or with speculation off) workgroup 0 runs the search kernel.
__global__ void __launch_bounds__(512) leaf_duo(LeafArgs a) {
    if (a.spec && *a.spec != 0) {
        if (wpanel_duo<4>(a)) return;
        if (blockIdx.x != 0) return;
        if (threadIdx.x == 0) *a.spec = 0;
        // the stores made before the decision are complete before the search
        // rewrites the same outputs
        __threadfence();
        __syncthreads();
    } else if (blockIdx.x != 0) {
        return;
    }
    gj2d_run<32, 8, 4, false, double, double>(a);
}

// Fills the exchange areas of a leaf's two-workgroup panels: every value
// with the pattern, every verdict and decision word with -1.
__global__ void __launch_bounds__(256) leaf_duo_reset(double *xg, int64_t nd, int *xc, int ni) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < nd) xg[e] = __longlong_as_double((long long)kDuoPoison);
    if (e < ni) xc[e] = -1;
}

template <int TR, int RR, int RC, bool WHOLE, typename TI, typename TO>
__device__ __attribute__((always_inline)) inline void gj2d_any(const LeafArgs &a) {
    if (a.spec && *a.spec != 0) {
        bool ok;
        if constexpr (WHOLE) {
            ok = gj2d_spec<TR, RR, RC, TI, TO>(a);
        } else {
            static_assert(TR * RR % 64 == 0, "whole waves hold the panel's rows");
            if constexpr (TR == 32 && TR * RR <= 256)
                ok = wpanel_pipe<TR * RR / 64>(a);
            else
                ok = wpanel_spec<TR * RR / 64, TR / 4>(a);
        }
        if (ok) return;
        if (threadIdx.x == 0) *a.spec = 0;
    }
    gj2d_run<TR, RR, RC, WHOLE, TI, TO>(a);
}

template <int TR, int RR, int RC, bool WHOLE, typename TI, typename TO>
__global__ void __launch_bounds__(16 * TR) leaf_gj2d(LeafArgs a) {
    gj2d_any<TR, RR, RC, WHOLE, TI, TO>(a);
}

// Many independent whole leaves in one grid (one workgroup each); the same
// device code as a single leaf, so every leaf's result is identical to the
// one it gets when launched alone.
template <int TR, int RR, int RC, typename TI, typename TO>
__global__ void __launch_bounds__(16 * TR) leaf_gj2d_batch(LeafBatch b) {
    const LeafItem &it = b.item[blockIdx.x];
    LeafArgs a{};
    a.in = it.in;
    a.ldi = it.ldi;
    a.out = it.out;
    a.ldo = it.ldo;
    a.L = (int)it.L;
    a.col0 = (int)it.col0;
    a.status = it.status;
    a.spec = it.status + kStatusSpecWord;
    gj2d_any<TR, RR, RC, true, TI, TO>(a);
}

// ---------------------------------------------------------------- tier 2 ---
struct PanelArgs {
    double *Z;
    int64_t ldz;
    int L, k0, nb, col0;
    int *used;   // L flags: row already chosen as a pivot
    int *rsel;   // L entries: pivot row of global step k
    double *Up;  // L x NB, ld L: panel transformation minus the pivot units
    int *status;
};

// The panel lives in registers with a rotating slot map: at step c, slot s of
// every thread holds panel column (s + c) mod NB, so the active column is
// always slot 0 and no register is indexed by a run-time value.
template <int NB, int RPT, int NT>
__global__ void __launch_bounds__(NT) leaf_panel(PanelArgs a) {
    constexpr int NW = NT / 64;
    __shared__ double red_v[2][NW];
    __shared__ int red_i[2][NW];
    __shared__ int red_f[2][NW];
    __shared__ double rowbuf[2][NB];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int L = a.L, k0 = a.k0, nb = a.nb;

    double z[RPT][NB];
    bool usd[RPT];
    int pst[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int row = t + NT * q;
        usd[q] = row >= L || (k0 > 0 && a.used[row] != 0);
        pst[q] = -1;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            z[q][c] = (row < L && c < nb) ? a.Z[row + (int64_t)(k0 + c) * a.ldz] : 0.0;
    }
    int bad = 0;

    for (int c = 0; c < nb; ++c) {
        const int buf = c & 1;
        double best = -1.0;
        int bi = INT_MAX, nf = 0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            if (!usd[q]) {
                // non-finite candidates keep key -0.5 so that an unused row
                // is always chosen (see tier 1)
                double av = fabs(z[q][0]);
                if (!(av <= DBL_MAX)) {
                    nf = 1;
                    av = -0.5;
                }
                if (av > best) {
                    best = av;
                    bi = t + NT * q;
                }
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off);
            const int oi = __shfl_xor(bi, off);
            if (better(ob, oi, best, bi)) {
                best = ob;
                bi = oi;
            }
        }
        const int wnf = __any(nf);
        if (lane == 0) {
            red_v[buf][w] = best;
            red_i[buf][w] = bi;
            red_f[buf][w] = wnf;
        }
        __syncthreads();
        best = red_v[buf][0];
        bi = red_i[buf][0];
        nf = red_f[buf][0];
#pragma unroll
        for (int ww = 1; ww < NW; ++ww) {
            const double ob = red_v[buf][ww];
            const int oi = red_i[buf][ww];
            nf |= red_f[buf][ww];
            if (better(ob, oi, best, bi)) {
                best = ob;
                bi = oi;
            }
        }
        const int p = bi;
        if ((nf || !(best > 0.0)) && bad == 0) bad = c + 1;
        if (t == p % NT) {
            const int pq = p / NT;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                if (q == pq) {
                    const double pinv = 1.0 / z[q][0];
#pragma unroll
                    for (int sl = 0; sl < NB; ++sl) {
                        rowbuf[buf][sl] = z[q][sl] * pinv;
                        z[q][sl] = 0.0;
                    }
                    rowbuf[buf][0] = pinv;
                    usd[q] = true;
                    pst[q] = c;
                }
            }
        }
        if (t == 0) a.rsel[k0 + c] = p;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const double f = (pst[q] == c) ? -1.0 : z[q][0];
            z[q][0] = 0.0;
#pragma unroll
            for (int sl = 0; sl < NB; ++sl) z[q][sl] = fma(-f, rowbuf[buf][sl], z[q][sl]);
            // rotate: slot s takes panel column (s + c + 1) mod NB
            const double z0 = z[q][0];
#pragma unroll
            for (int sl = 0; sl + 1 < NB; ++sl) z[q][sl] = z[q][sl + 1];
            z[q][NB - 1] = z0;
        }
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int row = t + NT * q;
        if (row < L) {
#pragma unroll
            for (int sl = 0; sl < NB; ++sl) {
                const int c = (sl + nb) & (NB - 1);
                if (c < nb) {
                    a.Z[row + (int64_t)(k0 + c) * a.ldz] = z[q][sl];
                    a.Up[row + (int64_t)c * L] = z[q][sl] - ((pst[q] == c) ? 1.0 : 0.0);
                }
            }
            if (k0 == 0)
                a.used[row] = pst[q] >= 0 ? 1 : 0;
            else if (pst[q] >= 0)
                a.used[row] = 1;
        }
    }
    if (t == 0 && bad) atomicMin(a.status, a.col0 + k0 + bad);
}

// Q (nb x L, ld nb): Q[c][j] = Z[rsel[k0 + c]][j] for columns outside the panel.
__global__ void __launch_bounds__(256)
    leaf_gather_q(const double *__restrict__ Z, int64_t ldz, int L, int k0, int nb,
                  const int *__restrict__ rsel, double *__restrict__ Q) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)L * nb) return;
    const int c = (int)(e % nb), j = (int)(e / nb);
    if (j >= k0 && j < k0 + nb) return;
    Q[c + (int64_t)j * nb] = Z[rsel[k0 + c] + (int64_t)j * ldz];
}

template <typename TI>
__global__ void __launch_bounds__(256)
    leaf_copy_in(const TI *__restrict__ in, int64_t ldi, double *__restrict__ Z, int L) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)L * L) return;
    const int i = (int)(e % L), j = (int)(e / L);
    Z[i + (int64_t)j * L] = (double)in[i + (int64_t)j * ldi];
}

// out[rinv[i]][rsel[c]] = Z[i][c].  When xg is given, also fills the leaf's
// exchange areas for the two-workgroup panels of the next leaf (nd doubles
// with the pattern, ni decision words with -1); the leaf's panels have all
// completed when this kernel runs.
template <typename TO>
__global__ void __launch_bounds__(256)
    leaf_unpermute(const double *__restrict__ Z, int L, const int *__restrict__ rsel,
                   TO *__restrict__ out, int64_t ldo, double *__restrict__ xg, int nd,
                   int *__restrict__ xc, int ni) {
    if (xg) {
        for (int e = blockIdx.x * 256 + threadIdx.x; e < nd; e += gridDim.x * 256)
            xg[e] = __longlong_as_double((long long)kDuoPoison);
        if (blockIdx.x == 0 && (int)threadIdx.x < ni) xc[threadIdx.x] = -1;
    }
    __shared__ int rinv[kLeafMaxOrder];
    for (int k = threadIdx.x; k < L; k += 256) rinv[k] = -1;
    __syncthreads();
    for (int k = threadIdx.x; k < L; k += 256) {
        const int r = rsel[k];
        if ((unsigned)r < (unsigned)L) rinv[r] = k;
    }
    __syncthreads();
    // one column per workgroup at a time
    for (int c = blockIdx.x; c < L; c += gridDim.x) {
        const int rc = rsel[c];
        if ((unsigned)rc >= (unsigned)L) continue;
        const double *zc = Z + (int64_t)c * L;
        TO *oc = out + (int64_t)rc * ldo;
        for (int i = threadIdx.x; i < L; i += 256) {
            const int ri = rinv[i];
            if ((unsigned)ri < (unsigned)L) oc[ri] = (TO)zc[i];
        }
    }
}

// ---------------------------------------------------------------- launch ---
template <int TR, int RR, int RC, bool WHOLE, typename TI, typename TO>
hipError_t gj2d_launch(const LeafArgs &la, hipStream_t s) {
    hipLaunchKernelGGL((leaf_gj2d<TR, RR, RC, WHOLE, TI, TO>), dim3(1), dim3(16 * TR), 0, s, la);
    return hipGetLastError();
}

// Threads per row group of the 2-D kernel for whole leaves of order <= 128
// and for panels of leaves of order <= 256 and <= 512 (measured best on
// MI355X: 32, i.e. 512 threads, in all three; a 512-row panel takes 147 us
// with 512 threads against 169 us with 1024, a 256-row panel 93 us against
// 110 us with 256 or 1024).
constexpr int kLeaf128TR = 32;
constexpr int kPanel256TR = 32;
constexpr int kPanel512TR = 32;

template <typename TI, typename TO>
hipError_t whole_dispatch(const LeafArgs &la, hipStream_t s, const char **name) {
    if (la.L <= 64) {
        *name = "leaf_gj_regs_64";
        return gj2d_launch<16, 4, 4, true, TI, TO>(la, s);
    }
    *name = "leaf_gj_regs_128";
    return gj2d_launch<kLeaf128TR, 128 / kLeaf128TR, 8, true, TI, TO>(la, s);
}

int panel_width(int64_t L) {
    if (L <= 512) return 64;
    if (L <= 1024) return 32;
    return 16;
}

hipError_t panel_launch(const PanelArgs &pa, hipStream_t s) {
    const int L = pa.L;
    if (L <= 256)
        hipLaunchKernelGGL((leaf_panel<64, 1, 256>), dim3(1), dim3(256), 0, s, pa);
    else if (L <= 512)
        hipLaunchKernelGGL((leaf_panel<64, 1, 512>), dim3(1), dim3(512), 0, s, pa);
    else if (L <= 1024)
        hipLaunchKernelGGL((leaf_panel<32, 1, 1024>), dim3(1), dim3(1024), 0, s, pa);
    else
        hipLaunchKernelGGL((leaf_panel<16, 2, 1024>), dim3(1), dim3(1024), 0, s, pa);
    return hipGetLastError();
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Leaves of order 129 .. 256 run their full panels on two workgroups
// (leaf_duo), with an exchange area per panel.  The areas sit at the start
// of every blocked leaf's scratch, so that leaves of every order find them at
// the same place and no other leaf writes them.
constexpr int kDuoPanels = 4;
constexpr int kDuoDoubles = kDuoPanels * duo_panel_doubles<4>();
constexpr int kDuoInts = kDuoPanels * kDuoPanelInts;
static_assert(kDuoInts <= 256, "the decision words are filled by one workgroup");
bool duo_leaf(int64_t L) { return L > 128 && L <= 256; }
// Polls after which a two-workgroup panel gives up waiting for the other
// workgroup: kDuoSpin, or SPIN_DUO_SPIN (a positive count; small values make
// the panels fall back to the search, for tests of that path).
int duo_spin_limit() {
    const char *e = std::getenv("SPIN_DUO_SPIN");
    const long v = e ? std::strtol(e, nullptr, 10) : 0;
    return (v > 0 && v <= kDuoSpin) ? (int)v : kDuoSpin;
}
size_t duo_bytes() { return align256(sizeof(double) * kDuoDoubles) + align256(sizeof(int) * kDuoInts); }

}  // namespace

size_t leaf_scratch_bytes(int64_t L) {
    if (L <= 128) return 0;
    const int64_t nb = panel_width(L);
    return duo_bytes() + align256(sizeof(double) * L * L) + align256(sizeof(double) * L * nb) +
           align256(sizeof(double) * L * nb) + align256(sizeof(int) * L) + align256(sizeof(int) * L);
}

bool leaf_fills_exchange(int64_t L) { return duo_leaf(L); }

hipError_t leaf_launch(const void *in, DType in_dt, int64_t ldi, void *out, DType out_dt,
                       int64_t ldo, int64_t L64, int64_t col0, int *status, void *scratch,
                       bool exch_filled, hipStream_t s,
                       void (*trace_cb)(void *, const LaunchInfo &, int), void *trace_ctx) {
    if (L64 < 1 || L64 > kLeafMaxOrder) return hipErrorInvalidValue;
    const int L = (int)L64;
    const double Ld = (double)L;
    auto cb = [&](const LaunchInfo &li, int phase) {
        if (trace_cb) trace_cb(trace_ctx, li, phase);
    };
    if (L <= 128) {
        LaunchInfo li{"leaf_gj_regs", 2.0 * Ld * Ld * Ld, 16.0 * Ld * Ld};
        cb(li, 0);
        LeafArgs la{};
        la.in = in;
        la.ldi = ldi;
        la.out = out;
        la.ldo = ldo;
        la.L = L;
        la.col0 = (int)col0;
        la.status = status;
        la.spec = status + kStatusSpecWord;
        hipError_t e;
        const char *name = "leaf_gj_regs";
        if (in_dt == kF64 && out_dt == kF64)
            e = whole_dispatch<double, double>(la, s, &name);
        else if (in_dt == kF32 && out_dt == kF32)
            e = whole_dispatch<float, float>(la, s, &name);
        else
            return hipErrorInvalidValue;
        li.name = name;
        cb(li, 1);
        return e;
    }
    if (!scratch) return hipErrorInvalidValue;
    const int nb = panel_width(L);
    char *p = static_cast<char *>(scratch);
    double *const xg = reinterpret_cast<double *>(p);
    p += align256(sizeof(double) * kDuoDoubles);
    int *const xc = reinterpret_cast<int *>(p);
    p += align256(sizeof(int) * kDuoInts);
    double *Z = reinterpret_cast<double *>(p);
    p += align256(sizeof(double) * L * L);
    double *Up = reinterpret_cast<double *>(p);
    p += align256(sizeof(double) * L * nb);
    double *Q = reinterpret_cast<double *>(p);
    p += align256(sizeof(double) * L * nb);
    int *rsel = reinterpret_cast<int *>(p);
    p += align256(sizeof(int) * L);
    int *used = reinterpret_cast<int *>(p);
    p += align256(sizeof(int) * L);
    const bool duo = duo_leaf(L);
    if (duo && !exch_filled) {
        LaunchInfo li{"leaf_duo_reset", 0.0, 8.0 * kDuoDoubles};
        cb(li, 0);
        hipLaunchKernelGGL(leaf_duo_reset, dim3((unsigned)((kDuoDoubles + 255) / 256)), dim3(256), 0, s,
                           xg, (int64_t)kDuoDoubles, xc, kDuoInts);
        hipError_t e = hipGetLastError();
        cb(li, 1);
        if (e != hipSuccess) return e;
    }

    const int nblk = (int)(((int64_t)L * L + 255) / 256);
    // Up to order 512 an FP64 input is read in place by the first panel and
    // its update (which writes Z); otherwise it is copied into Z first.
    const bool direct = L <= 512 && in_dt == kF64;
    if (!direct) {
        LaunchInfo li{"leaf_copy_in", 0.0, (in_dt == kF64 ? 16.0 : 12.0) * Ld * Ld};
        cb(li, 0);
        if (in_dt == kF64)
            hipLaunchKernelGGL((leaf_copy_in<double>), dim3(nblk), dim3(256), 0, s,
                               static_cast<const double *>(in), ldi, Z, L);
        else
            hipLaunchKernelGGL((leaf_copy_in<float>), dim3(nblk), dim3(256), 0, s,
                               static_cast<const float *>(in), ldi, Z, L);
        hipError_t e = hipGetLastError();
        cb(li, 1);
        if (e != hipSuccess) return e;
    }
    for (int k0 = 0; k0 < L; k0 += nb) {
        const int w = (L - k0 < nb) ? (L - k0) : nb;
        PanelArgs pa{Z, (int64_t)L, L, k0, w, (int)col0, used, rsel, Up, status};
        const bool fused = L <= 512;  // the 2-D panel kernel also gathers Q
        {
            LaunchInfo li{"leaf_gj_panel", 2.0 * Ld * w * w, 16.0 * Ld * w};
            cb(li, 0);
            hipError_t e;
            if (fused) {
                LeafArgs la{};
                la.L = L;
                la.col0 = (int)col0;
                la.status = status;
                la.spec = status + kStatusSpecWord;
                la.Z = Z;
                la.ldz = L;
                la.k0 = k0;
                la.nb = w;
                if (direct && k0 == 0) {
                    la.in = in;
                    la.ldi = ldi;
                }
                la.used = used;
                la.rsel = rsel;
                la.Up = Up;
                la.Q = Q;
                if (duo && w == 64 && k0 % 64 == 0 && k0 / 64 < kDuoPanels) {
                    la.xg = xg + (int64_t)(k0 / 64) * duo_panel_doubles<4>();
                    la.xc = xc + (k0 / 64) * kDuoPanelInts;
                    la.duo_spin = duo_spin_limit();
                    hipLaunchKernelGGL(leaf_duo, dim3(2), dim3(512), 0, s, la);
                    e = hipGetLastError();
                } else if (L <= 256)
                    e = gj2d_launch<kPanel256TR, 256 / kPanel256TR, 4, false, double, double>(la, s);
                else
                    e = gj2d_launch<kPanel512TR, 512 / kPanel512TR, 4, false, double, double>(la, s);
            } else {
                e = panel_launch(pa, s);
            }
            cb(li, 1);
            if (e != hipSuccess) return e;
        }
        if (w == L) break;
        if (!fused) {
            LaunchInfo li{"leaf_gather_q", 0.0, 16.0 * Ld * w};
            cb(li, 0);
            const int gb = (int)(((int64_t)L * w + 255) / 256);
            hipLaunchKernelGGL(leaf_gather_q, dim3(gb), dim3(256), 0, s, Z, (int64_t)L, L, k0, w,
                               rsel, Q);
            hipError_t e = hipGetLastError();
            cb(li, 1);
            if (e != hipSuccess) return e;
        }
        GemmProb pr[2];
        int np = 0;
        if (k0 > 0)
            pr[np++] = GemmProb{Up, Q, Z, Z, (int64_t)L, (int64_t)w, (int64_t)L, (int64_t)L,
                                L, k0, w, 0, 1.0, 1.0};
        if (k0 + w < L) {
            // the columns right of the first panel still live in the input
            const bool from_in = direct && k0 == 0;
            const double *c0 = from_in ? static_cast<const double *>(in) + (int64_t)(k0 + w) * ldi
                                       : Z + (int64_t)(k0 + w) * L;
            pr[np++] = GemmProb{Up, Q + (int64_t)(k0 + w) * w, c0, Z + (int64_t)(k0 + w) * L,
                                (int64_t)L, (int64_t)w, from_in ? ldi : (int64_t)L, (int64_t)L,
                                L, L - k0 - w, w, 0, 1.0, 1.0};
        }
        LaunchInfo gi{};
        cb(gi, 0);
        hipError_t e = gemm_launch(pr, np, kF64, s, &gi);
        cb(gi, 1);
        if (e != hipSuccess) return e;
    }
    {
        LaunchInfo li{"leaf_unpermute", 0.0,
                      (out_dt == kF64 ? 16.0 : 12.0) * Ld * Ld + (duo ? 8.0 * kDuoDoubles : 0.0)};
        cb(li, 0);
        const int gb = L < 1024 ? L : 1024;
        // a two-workgroup leaf leaves its exchange areas filled for the next
        double *fxg = duo ? xg : nullptr;
        if (out_dt == kF64)
            hipLaunchKernelGGL((leaf_unpermute<double>), dim3(gb), dim3(256), 0, s, Z, L, rsel,
                               static_cast<double *>(out), ldo, fxg, kDuoDoubles, xc, kDuoInts);
        else
            hipLaunchKernelGGL((leaf_unpermute<float>), dim3(gb), dim3(256), 0, s, Z, L, rsel,
                               static_cast<float *>(out), ldo, fxg, kDuoDoubles, xc, kDuoInts);
        hipError_t e = hipGetLastError();
        cb(li, 1);
        return e;
    }
}


hipError_t leaf_batch_launch(const LeafItem *items, int count, DType dt, hipStream_t s,
                             LaunchInfo *info) {
    if (count < 0 || count > kMaxLeafBatch) return hipErrorInvalidValue;
    double flops = 0, bytes = 0;
    LeafBatch small{}, big{};
    for (int i = 0; i < count; ++i) {
        if (items[i].L < 1 || items[i].L > 128) return hipErrorInvalidValue;
        const double L = (double)items[i].L;
        flops += 2.0 * L * L * L;
        bytes += 16.0 * L * L;
        if (items[i].L <= 64)
            small.item[small.count++] = items[i];
        else
            big.item[big.count++] = items[i];
    }
    hipError_t e = hipSuccess;
    if (small.count) {
        if (dt == kF64)
            hipLaunchKernelGGL((leaf_gj2d_batch<16, 4, 4, double, double>), dim3(small.count),
                               dim3(256), 0, s, small);
        else
            hipLaunchKernelGGL((leaf_gj2d_batch<16, 4, 4, float, float>), dim3(small.count),
                               dim3(256), 0, s, small);
        e = hipGetLastError();
    }
    if (e == hipSuccess && big.count) {
        if (dt == kF64)
            hipLaunchKernelGGL((leaf_gj2d_batch<kLeaf128TR, 128 / kLeaf128TR, 8, double, double>),
                               dim3(big.count), dim3(16 * kLeaf128TR), 0, s, big);
        else
            hipLaunchKernelGGL((leaf_gj2d_batch<kLeaf128TR, 128 / kLeaf128TR, 8, float, float>),
                               dim3(big.count), dim3(16 * kLeaf128TR), 0, s, big);
        e = hipGetLastError();
    }
    if (info) {
        info->name = "leaf_gj_regs_batch";
        info->flops = flops;
        info->bytes = bytes;
    }
    return e;
}

}  // namespace spin
