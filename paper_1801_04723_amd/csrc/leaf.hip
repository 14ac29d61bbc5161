// Leaf inversion: Gauss-Jordan elimination with partial pivoting in FP64.
//
// The paper inverts each leaf block "in any approach" on a single node
// (Alg. 1, Alg. 2 `locInverse`, Sec. 3.3); here it is Gauss-Jordan with
// partial pivoting, always in FP64 (also when the surrounding products run in
// FP32).
//
// Both tiers use implicit pivoting: rows are never moved.  Step k picks the
// unused row p with the largest |z[p][k]| (ties to the smallest row index),
// scales row p by 1/pivot and eliminates column k from every other row.  The
// storage is in place: after step k the slot of column k holds column p of
// the accumulated row transformation (it replaces the unit column that an
// augmented [A | I] would carry).  With r[k] = pivot row of step k and
// rinv[r[k]] = k, the inverse is  X[rinv[i]][r[c]] = Z[i][c].
//
// Tier 1 (L <= 128): one workgroup of 256 threads holds the whole block in
//   registers, cyclically distributed (thread (tr, tc) owns rows tr + 16a and
//   columns tc + 16b).  A step costs two barriers: the owners of column k
//   publish it to LDS, every wave finds the pivot redundantly with a wave
//   reduction, the owners of the pivot row publish the scaled row, and every
//   thread applies the rank-1 update to its registers.
// Tier 2 (L > 128): blocked Gauss-Jordan over column panels of width NB.  One
//   workgroup eliminates a panel (all L rows x NB columns in registers) and
//   emits the panel's transformation U' = U - E (E = unit entries at the
//   pivot rows); the columns outside the panel are then updated by one
//   grouped matrix-core product  Z[:, out] += U' * Z[pivot rows, out].
//   A final pass writes the permuted result.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>

#include "spin_kernels.hpp"

namespace spin {
namespace {

__device__ inline bool better(double ov, int oi, double v, int i) {
    return ov > v || (ov == v && oi < i);
}

// ---------------------------------------------------------------- tier 1 ---
template <int R, typename TI, typename TO>
__global__ void __launch_bounds__(256)
    leaf_small(const TI *__restrict__ in, int64_t ldi, TO *__restrict__ out, int64_t ldo, int L,
               int col0, int *status) {
    __shared__ double colbuf[2][128];
    __shared__ double rowbuf[2][128];
    __shared__ int rsel[128];
    __shared__ int rinv[128];
    const int t = threadIdx.x, tr = t >> 4, tc = t & 15, lane = t & 63;

    double z[R][R];
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) {
            const int i = tr + 16 * a, j = tc + 16 * b;
            z[a][b] = (i < L && j < L) ? (double)in[i + (int64_t)j * ldi] : 0.0;
        }
    // Rows lane and lane + 64 are this lane's pivot candidates in the
    // (redundant, per wave) argmax; padding rows never qualify.
    bool u0 = lane >= L, u1 = (lane + 64) >= L;
    int bad = 0;

#pragma unroll
    for (int kb = 0; kb < R; ++kb) {
        for (int kk = 0; kk < 16; ++kk) {
            const int k = kb * 16 + kk;
            if (k >= L) break;
            const int buf = k & 1;
            // column k to LDS; its slot restarts from the (implicit) unit column
            if (tc == kk) {
#pragma unroll
                for (int a = 0; a < R; ++a) {
                    colbuf[buf][tr + 16 * a] = z[a][kb];
                    z[a][kb] = 0.0;
                }
            }
            __syncthreads();
            const double v0 = colbuf[buf][lane];
            const double v1 = colbuf[buf][lane + 64];
            const double f0 = fabs(v0), f1 = fabs(v1);
            const int nf = (!u0 && !(f0 <= DBL_MAX)) || (!u1 && !(f1 <= DBL_MAX));
            // key: |v| for usable candidates, -0.5 for non-finite ones (so an
            // unused row is always chosen and the pivot order stays a
            // permutation even when the step fails), -1 for used rows
            double best = u0 ? -1.0 : (f0 <= DBL_MAX ? f0 : -0.5);
            int bi = lane;
            const double c1 = u1 ? -1.0 : (f1 <= DBL_MAX ? f1 : -0.5);
            if (c1 > best) {
                best = c1;
                bi = lane + 64;
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
            const int p = __builtin_amdgcn_readfirstlane(bi);
            const bool fail = __any(nf) || !(best > 0.0);
            if (fail && bad == 0) bad = k + 1;
            if (lane == p) u0 = true;
            if (lane + 64 == p) u1 = true;
            // the owners of row p publish it scaled by 1/pivot
            if (tr == (p & 15)) {
                const int ap = p >> 4;
#pragma unroll
                for (int a = 0; a < R; ++a) {
                    if (a == ap) {
                        const double pinv = 1.0 / colbuf[buf][p];
#pragma unroll
                        for (int b = 0; b < R; ++b) {
                            rowbuf[buf][tc + 16 * b] = z[a][b] * pinv;
                            z[a][b] = 0.0;
                        }
                        if (tc == kk) rowbuf[buf][k] = pinv;
                    }
                }
            }
            __syncthreads();
            double f[R], rv[R];
#pragma unroll
            for (int a = 0; a < R; ++a) f[a] = (tr + 16 * a == p) ? -1.0 : colbuf[buf][tr + 16 * a];
#pragma unroll
            for (int b = 0; b < R; ++b) rv[b] = rowbuf[buf][tc + 16 * b];
#pragma unroll
            for (int a = 0; a < R; ++a)
#pragma unroll
                for (int b = 0; b < R; ++b) z[a][b] = fma(-f[a], rv[b], z[a][b]);
            if (t == 0) {
                rsel[k] = p;
                rinv[p] = k;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) {
            const int i = tr + 16 * a, c = tc + 16 * b;
            if (i < L && c < L) {
                const int ri = rinv[i], rc = rsel[c];
                if ((unsigned)ri < (unsigned)L && (unsigned)rc < (unsigned)L)
                    out[ri + (int64_t)rc * ldo] = (TO)z[a][b];
            }
        }
    if (t == 0 && bad) atomicMin(status, col0 + bad);
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
template <int R, typename TI, typename TO>
hipError_t small_launch(const void *in, int64_t ldi, void *out, int64_t ldo, int L, int col0,
                        int *status, hipStream_t s) {
    hipLaunchKernelGGL((leaf_small<R, TI, TO>), dim3(1), dim3(256), 0, s,
                       static_cast<const TI *>(in), ldi, static_cast<TO *>(out), ldo, L, col0,
                       status);
    return hipGetLastError();
}

template <typename TI, typename TO>
hipError_t small_dispatch(const void *in, int64_t ldi, void *out, int64_t ldo, int L, int col0,
                          int *status, hipStream_t s, const char **name) {
    if (L <= 16) {
        *name = "leaf_gj_regs_16";
        return small_launch<1, TI, TO>(in, ldi, out, ldo, L, col0, status, s);
    }
    if (L <= 32) {
        *name = "leaf_gj_regs_32";
        return small_launch<2, TI, TO>(in, ldi, out, ldo, L, col0, status, s);
    }
    if (L <= 64) {
        *name = "leaf_gj_regs_64";
        return small_launch<4, TI, TO>(in, ldi, out, ldo, L, col0, status, s);
    }
    *name = "leaf_gj_regs_128";
    return small_launch<8, TI, TO>(in, ldi, out, ldo, L, col0, status, s);
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
        hipError_t e;
        const char *name = "leaf_gj_regs";
        if (in_dt == kF64 && out_dt == kF64)
            e = small_dispatch<double, double>(in, ldi, out, ldo, L, (int)col0, status, s, &name);
        else if (in_dt == kF32 && out_dt == kF32)
            e = small_dispatch<float, float>(in, ldi, out, ldo, L, (int)col0, status, s, &name);
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
    {
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
        {
            LaunchInfo li{"leaf_gj_panel", 2.0 * Ld * w * w, 16.0 * Ld * w};
            cb(li, 0);
            hipError_t e = panel_launch(pa, s);
            cb(li, 1);
            if (e != hipSuccess) return e;
        }
        if (w == L) break;
        {
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
        if (k0 + w < L)
            pr[np++] = GemmProb{Up, Q + (int64_t)(k0 + w) * w, Z + (int64_t)(k0 + w) * L,
                                Z + (int64_t)(k0 + w) * L, (int64_t)L, (int64_t)w, (int64_t)L,
                                (int64_t)L, L, L - k0 - w, w, 0, 1.0, 1.0};
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

}  // namespace spin
