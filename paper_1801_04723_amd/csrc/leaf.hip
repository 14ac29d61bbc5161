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
//   Up to order 512 the panel kernel is the same 2-D kernel, and an FP64
//   leaf is not copied first: the first panel and its product read the
//   leaf's input in place.  Above 512 a rotating-slot panel kernel works on
//   narrower panels and the input is copied into Z.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>

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

// ------------------------------------------------ speculative 2-D kernel ---
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
// publish its multipliers and the owners of row c+1 the pivot row (whole
// leaves: scaled, since the pivot row's wave also holds the pivot; panels:
// raw, with the inverse pivot published by the pivot's owner), and after one
// barrier every thread applies step c+1.  Every element goes through the
// same operations as in gj2d_run (the same division, products and fused
// multiply-adds), so when every check passes the outputs are gj2d_run's bit
// for bit.  They are written only then.  Returns whether every check passed
// (the same in every thread); on false nothing has been written.
template <int TR, int RR, int RC, bool WHOLE, typename TI, typename TO>
__device__ __attribute__((always_inline)) inline bool gj2d_spec(const LeafArgs &a) {
    constexpr int NT = 16 * TR;
    constexpr int LMAX = TR * RR;
    constexpr int NBMAX = 16 * RC;
    static_assert(TR == 16 || TR == 32, "row groups of 16 or 32 threads");
    // Shared arrays are indexed by register slot, not by row: entry tr + TR r
    // belongs to slot r of the threads with that tr (the same map in every
    // thread), so that every access is a per-thread base plus a constant.
    __shared__ double fbs[2][LMAX];   // multipliers of a step, -1 / 0 at its pivot row
    __shared__ double rws[2][NBMAX];  // its pivot row (see above)
    __shared__ double pvs[2][2];      // |pivot| (whole leaves) and 1 / pivot (panels)
    const int t = threadIdx.x, wave = t >> 6;
    const int tr = WHOLE ? t >> 4 : t % TR, tc = WHOLE ? t & 15 : t / TR;
    const int L = a.L;
    const int k0 = WHOLE ? 0 : a.k0;
    const int nb = WHOLE ? a.L : a.nb;
    const double *src = WHOLE ? nullptr : (a.in ? static_cast<const double *>(a.in) : a.Z);
    const int64_t lds = WHOLE ? 0 : (a.in ? a.ldi : a.ldz);
    // Register slot r holds row tr + TR ((r + rot) mod RR), rot = k0 / TR: the
    // row map turns with the panel's first column (a multiple of TR), so that
    // the pivot row of step c (row k0 + c) sits in slot c / TR of thread
    // c mod TR, a constant of the unrolled column block cb = c / 16.  Slots
    // r >= RR - rot hold the rows before the panel, all of them used.
    const int rot = k0 / TR;
    int rowr[RR];
#pragma unroll
    for (int r = 0; r < RR; ++r) rowr[r] = tr + TR * ((r + rot) % RR);

    double z[RR][RC];
    bool viol = !WHOLE && (k0 % TR) != 0;
#pragma unroll
    for (int r = 0; r < RR; ++r) {
        const int row = rowr[r];
        // the rows before the panel must be the used ones and no other
        if (!WHOLE && k0 > 0 && row < L && ((a.used[row] != 0) != (row < k0))) viol = true;
#pragma unroll
        for (int q = 0; q < RC; ++q) {
            const int col = tc + 16 * q;
            double v = 0.0;
            if (row < L && col < nb) {
                if (WHOLE)
                    v = (double)static_cast<const TI *>(a.in)[row + (int64_t)col * a.ldi];
                else
                    v = src[row + (int64_t)(k0 + col) * lds];
            }
            z[r][q] = v;
        }
    }
    double *const fbt = &fbs[0][tr];
    double *const rwt = &rws[0][tc];

    // One step c = 16 cb + cc, LDS buffer B = c & 1: publication (its column
    // and pivot row are final once step c - 1 is applied), one barrier, the
    // update.  cb and B are constants after unrolling.
    auto step = [&](const int cb, const int cc, const int B) {
        const int c = 16 * cb + cc, p = k0 + c;
        const int PR = (16 * cb) / TR;          // register slot of the pivot row
        const int pt = (16 * cb) % TR + cc;     // its owners' tr
        if (WHOLE) {
            // the 16 owners of row p are lanes 16 pt .. 16 pt + 15 of one wave
            if (wave == (16 * pt) >> 6) {
                const double piv = readlane_f64(z[PR][cb], (16 * pt + cc) & 63);
                if (tr == pt) {
                    const double pinv = 1.0 / piv;
#pragma unroll
                    for (int q = 0; q < RC; ++q) {
                        rwt[B * NBMAX + 16 * q] = (q == cb && tc == cc) ? pinv : z[PR][q] * pinv;
                        z[PR][q] = 0.0;  // the update adds the scaled row (multiplier -1)
                    }
                    if (tc == cc) pvs[B][0] = fabs(piv);
                }
            }
            if (tc == cc) {
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    fbt[B * LMAX + TR * r] = (r == PR && tr == pt) ? -1.0 : z[r][cb];
                    z[r][cb] = 0.0;
                }
            }
        } else {
            if (tr == pt) {
#pragma unroll
                for (int q = 0; q < RC; ++q)
                    rwt[B * NBMAX + 16 * q] = (q == cb && tc == cc) ? 1.0 : z[PR][q];
                if (tc == cc) pvs[B][1] = 1.0 / z[PR][cb];
            }
            // the owners of column c (half of wave cc / 2 when TR = 32) also
            // check the step: the pivot, read from its lane, against every
            // unused row they hold
            if (wave == (TR * cc) >> 6) {
                const double piv = readlane_f64(z[PR][cb], (TR * cc + pt) & 63);
                const double apiv = fabs(piv);
                bool v = !(apiv > 0.0) || !(apiv <= DBL_MAX);
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    if (r < PR) continue;  // rows before the pivot: used
                    const bool used = (r == PR) ? (tr <= pt) : (r + rot >= RR);
                    v = v || (!used && !(fabs(z[r][cb]) <= apiv));
                }
                if (tc == cc) viol = viol || v;
            }
            if (tc == cc) {
#pragma unroll
                for (int r = 0; r < RR; ++r) {
                    fbt[B * LMAX + TR * r] = (r == PR && tr == pt) ? 0.0 : z[r][cb];
                    z[r][cb] = 0.0;
                }
            }
        }
        __syncthreads();
        double f[RR], rv[RC];
#pragma unroll
        for (int r = 0; r < RR; ++r) f[r] = fbt[B * LMAX + TR * r];
#pragma unroll
        for (int q = 0; q < RC; ++q) rv[q] = rwt[B * NBMAX + 16 * q];
        if (WHOLE) {
            // check of step c: the pivot, then the unused rows of this thread
            const double apiv = pvs[B][0];
            bool v = !(apiv > 0.0) || !(apiv <= DBL_MAX);
#pragma unroll
            for (int r = 0; r < RR; ++r) {
                if (r < PR) continue;  // rows before the pivot: used
                const bool used = (r == PR) && (tr <= pt);
                v = v || (!used && !(fabs(f[r]) <= apiv));
            }
            viol = viol || v;
        } else {
            const double pinv = pvs[B][1];
#pragma unroll
            for (int q = 0; q < RC; ++q) rv[q] = rv[q] * pinv;
            if (tr == pt) {
#pragma unroll
                for (int q = 0; q < RC; ++q) z[PR][q] = rv[q];
            }
        }
#pragma unroll
        for (int r = 0; r < RR; ++r)
#pragma unroll
            for (int q = 0; q < RC; ++q) z[r][q] = fma(-f[r], rv[q], z[r][q]);
    };

#pragma unroll
    for (int cb = 0; cb < RC; ++cb) {
        for (int cc = 0; cc < 16; cc += 2) {
            if (16 * cb + cc >= nb) break;
            step(cb, cc, 0);
            if (16 * cb + cc + 1 >= nb) break;
            step(cb, cc + 1, 1);
        }
    }
    if (__syncthreads_or(viol)) return false;

    if (WHOLE) {
        TO *out = static_cast<TO *>(a.out);
#pragma unroll
        for (int r = 0; r < RR; ++r)
#pragma unroll
            for (int q = 0; q < RC; ++q) {
                const int row = rowr[r], col = tc + 16 * q;
                if (row < L && col < L) out[row + (int64_t)col * a.ldo] = (TO)z[r][q];
            }
    } else {
#pragma unroll
        for (int r = 0; r < RR; ++r)
#pragma unroll
            for (int q = 0; q < RC; ++q) {
                const int row = rowr[r], col = tc + 16 * q;
                if (row < L && col < nb) {
                    a.Z[row + (int64_t)(k0 + col) * a.ldz] = z[r][q];
                    a.Up[row + (int64_t)col * L] = z[r][q] - ((row == k0 + col) ? 1.0 : 0.0);
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
    }
    return true;
}

template <int TR, int RR, int RC, bool WHOLE, typename TI, typename TO>
__device__ __attribute__((always_inline)) inline void gj2d_any(const LeafArgs &a) {
    if (a.spec && *a.spec != 0) {
        if (gj2d_spec<TR, RR, RC, WHOLE, TI, TO>(a)) return;
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

template <typename TO>
__global__ void __launch_bounds__(256)
    leaf_unpermute(const double *__restrict__ Z, int L, const int *__restrict__ rsel,
                   TO *__restrict__ out, int64_t ldo) {
    __shared__ int rinv[kLeafMaxOrder];
    for (int k = threadIdx.x; k < L; k += 256) rinv[k] = -1;
    __syncthreads();
    for (int k = threadIdx.x; k < L; k += 256) {
        const int r = rsel[k];
        if ((unsigned)r < (unsigned)L) rinv[r] = k;
    }
    __syncthreads();
    const int64_t total = (int64_t)L * L;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * 256) {
        const int i = (int)(e % L), c = (int)(e / L);
        const int ri = rinv[i], rc = rsel[c];
        if ((unsigned)ri < (unsigned)L && (unsigned)rc < (unsigned)L)
            out[ri + (int64_t)rc * ldo] = (TO)Z[e];
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

}  // namespace

size_t leaf_scratch_bytes(int64_t L) {
    if (L <= 128) return 0;
    const int64_t nb = panel_width(L);
    return align256(sizeof(double) * L * L) + align256(sizeof(double) * L * nb) +
           align256(sizeof(double) * L * nb) + align256(sizeof(int) * L) +
           align256(sizeof(int) * L);
}

hipError_t leaf_launch(const void *in, DType in_dt, int64_t ldi, void *out, DType out_dt,
                       int64_t ldo, int64_t L64, int64_t col0, int *status, void *scratch,
                       hipStream_t s, void (*trace_cb)(void *, const LaunchInfo &, int),
                       void *trace_ctx) {
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
    double *Z = reinterpret_cast<double *>(p);
    p += align256(sizeof(double) * L * L);
    double *Up = reinterpret_cast<double *>(p);
    p += align256(sizeof(double) * L * nb);
    double *Q = reinterpret_cast<double *>(p);
    p += align256(sizeof(double) * L * nb);
    int *rsel = reinterpret_cast<int *>(p);
    p += align256(sizeof(int) * L);
    int *used = reinterpret_cast<int *>(p);

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
                if (L <= 256)
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
        LaunchInfo li{"leaf_unpermute", 0.0, (out_dt == kF64 ? 16.0 : 12.0) * Ld * Ld};
        cb(li, 0);
        const int gb = nblk < 1024 ? nblk : 1024;
        if (out_dt == kF64)
            hipLaunchKernelGGL((leaf_unpermute<double>), dim3(gb), dim3(256), 0, s, Z, L, rsel,
                               static_cast<double *>(out), ldo);
        else
            hipLaunchKernelGGL((leaf_unpermute<float>), dim3(gb), dim3(256), 0, s, Z, L, rsel,
                               static_cast<float *>(out), ldo);
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
