// gfx950 kernels of the blocked sparse LU (right-looking, Algorithm 1).
//
// Storage (see analyze.hpp): per level i a dense diagonal block D_i
// (column-major b x b) and two panels over the coupled index sets,
// P_i[a, t] = L(rows_i[a], r0 + K_i[t]) and Qt_i[a, t] = U(r0 + K_i[t], rows_i[a]),
// both m x kappa column-major.  Entries of those dense arrays that lie outside
// the symbolic pattern start at 0.0 and stay exactly 0.0: every product that
// could reach them has a structurally zero factor.
#include "kernels.hpp"

#include <hip/hip_runtime.h>

#include <cmath>

namespace slu {

typedef double double4_t __attribute__((ext_vector_type(4)));

// Value of a lane's double in every lane (the lane index must be the same in
// all lanes of the wave): two v_readlane into scalar registers.
__device__ __forceinline__ double bcast_lane(double v, int k) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)x, k);
    const int hi = __builtin_amdgcn_readlane((int)(x >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 1 / x in FP64: hardware estimate refined by two Newton steps (relative
// error within a few ulps; used where a pivot's reciprocal scales a column).
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// In-place no-pivot LU of the w x w (w <= 16) leading block of the LDS array
// A (element (i, j) at A[j * lda + i]) by wave 0: lane i holds row i, the
// pivot row is broadcast with readlane.  Records a zero / non-finite pivot.
__device__ __forceinline__ void lu16_wave0(double *A, int lda, int w, int lane, int col0,
                                           unsigned long long *__restrict__ info) {
    double v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = (j < w && lane < w) ? A[j * lda + lane] : 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k < w) {
            double u[16];
#pragma unroll
            for (int j = k; j < 16; ++j) u[j] = bcast_lane(v[j], k);
            const double piv = u[k];
            if (lane == 0 && !(piv != 0.0 && isfinite(piv))) atomicMin(info, (unsigned long long)(col0 + k));
            const double rp = recip(piv);
            if (lane > k) {
                const double l = v[k] * rp;
                v[k] = l;
#pragma unroll
                for (int j = k + 1; j < 16; ++j) v[j] -= l * u[j];
            }
        }
    }
    if (lane < w) {
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (j < w) A[j * lda + lane] = v[j];
    }
}

// Inverses of the factors of a w x w LU held in LDS (as left by lu16_wave0).
// Lane j < 16 of the calling wave forms column j of U^{-1} (upper == true)
// or of L^{-1} (unit lower); the two are meant to run in different waves.
// Ui / Li are 16 x 16 with row stride 17, element (r, c) at [r * 17 + c];
// rows / columns beyond w are the identity.  Each triangle row is read from
// LDS as one batch before its products.
__device__ __forceinline__ void tri_inverse16(const double *A, int lda, int w, int lane, bool upper,
                                              double *Out) {
    if (lane >= 16) return;
    const int j = lane;
    double x[16];
    if (upper) {
        double rd[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) rd[i] = i < w ? recip(A[i * lda + i]) : 1.0;
#pragma unroll
        for (int i = 15; i >= 0; --i) {
            double row[16];
#pragma unroll
            for (int t = i + 1; t < 16; ++t) row[t] = (i < w && t < w) ? A[t * lda + i] : 0.0;
            double sacc = (i == j) ? 1.0 : 0.0;
#pragma unroll
            for (int t = 15; t > i; --t) sacc -= row[t] * x[t];
            x[i] = (i <= j) ? sacc * rd[i] : 0.0;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            double row[16];
#pragma unroll
            for (int t = 0; t < i; ++t) row[t] = (i < w && t < w) ? A[t * lda + i] : 0.0;
            double sacc = (i == j) ? 1.0 : 0.0;
#pragma unroll
            for (int t = 0; t < i; ++t) sacc -= row[t] * x[t];
            x[i] = (i >= j) ? sacc : 0.0;
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) Out[i * 17 + j] = x[i];
}
// ------------------------------------------------------------------ helpers
__global__ void k_zero(double *__restrict__ p, int64_t count) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0.0;
}

hipError_t launch_zero(double *p, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

// Alg. 1 "construct blocks": place every value of A at its precomputed slot.
__global__ void k_scatter(const double *__restrict__ vals, const int64_t *__restrict__ slot,
                          double *__restrict__ slab, int64_t nnz) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz; q += stride)
        slab[slot[q]] = vals[q];
}

hipError_t launch_scatter(const DevPlan &d, const double *values, hipStream_t s) {
    if (d.nnz_a <= 0) return hipSuccess;
    int64_t blocks = (d.nnz_a + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)blocks), dim3(256), 0, s, values, d.slot, d.slab, d.nnz_a);
    return hipGetLastError();
}

__global__ void k_info_reset(unsigned long long *info) {
    if (threadIdx.x == 0) info[0] = ~0ull;
}

hipError_t launch_info_reset(const DevPlan &d, hipStream_t s) {
    hipLaunchKernelGGL(k_info_reset, dim3(1), dim3(64), 0, s, d.info);
    return hipGetLastError();
}

// --------------------------------------------------------------------- GETRF
// Alg. 1 line "B_ii -> L_ii U_ii" for diagonal blocks above 128 rows: no-pivot
// LU of the dense diagonal block by one workgroup, right-looking over column
// chunks [c0, c0 + w) (w <= 16).  Only the block rows R that S couples to a
// chunk are touched by it:
//   1. wave 0 factors the w x w diagonal of the chunk in registers and forms
//      the inverses of its two triangles;
//   2. the coupled rows (L = A U_cc^{-1}) and coupled columns
//      (U = L_cc^{-1} A) are 16 x 16 x 16 FP64 MFMA products;
//   3. the four waves update the R x R trailing entries with FP64 MFMA.
// Pivot divisions are FP64 divisions; a zero or non-finite pivot records its
// permuted column in info[0].
// One column chunk of the chunked GETRF.  W = 16 is the full-width chunk
// (every width guard folds away); W = 0 takes the width at run time (the
// last chunk of a block).  Loads guarded per lane read a clamped, valid
// address and select zero, so they are issued without branches.
template <int W>
__device__ __forceinline__ void getrf_chunk_step(double *__restrict__ D, int b, int r0, const ChunkDev &C,
                                                 const int *Rs, double *Ui, double *Li, double *work,
                                                 unsigned long long *__restrict__ info, int wave, int lane,
                                                 int tid) {
    const int li = lane & 15, lk = lane >> 4;
    const int c0 = C.c0, w = W ? W : C.w, nr = C.nr;
    const int T = w + nr;
    const int wu = w + 1;
    double *Pn = work;                     // Pn[j*T + t]: chunk column j, panel row t (t < w: chunk rows)
    double *Uc = work + (size_t)T * w;     // Uc[s*wu + j]: U(c0 + j, Rs[s])
    const int nrt = (nr + 15) >> 4;
    const int ntl = nrt;
    const int ntiles = ntl * ntl;
    // Trailing tiles are transposed 16 x 16 tiles of the coupled rows x
    // coupled columns: output element (coupled column 16tj + lk + 4r,
    // coupled row 16ti + li), so the 16 lanes of a group read and write
    // consecutive rows of a column.  A wave takes up to eight tiles per round.
    double4_t acc[8];
    bool vr[8];
    size_t rowo[8];
    auto load_tiles = [&](int q0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + 4 * u;
            const int qc = q < ntiles ? q : ntiles - 1;
            const int ti = qc / ntl, tj = qc - ti * ntl;
            const int ra = 16 * ti + li;
            vr[u] = q < ntiles && ra < nr;
            rowo[u] = (size_t)Rs[ra < nr ? ra : nr - 1];
            // entries outside the coupled set read a clamped valid address;
            // an MFMA output element depends only on its own accumulator
            // input and those elements are never stored, so no select is
            // needed (it would make each load wait at once)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int sc = 16 * tj + lk + 4 * r;
                acc[u][r] = D[rowo[u] + (size_t)Rs[sc < nr ? sc : nr - 1] * b];
            }
        }
    };
    // one item per panel row (its w values) or per coupled column (its w
    // values, contiguous in D): the loads of an item are issued together
    for (int it = tid; it < T + nr; it += 256) {
        double v[16];
        if (it < T) {
            const int row = it < w ? c0 + it : Rs[it - w];
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = j < w ? D[row + (size_t)(c0 + j) * b] : 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (j < w) Pn[j * T + it] = v[j];
        } else {
            const int sI = it - T;
            const double *__restrict__ col = D + c0 + (size_t)Rs[sI] * b;
#pragma unroll
            for (int j = 0; j < 16; ++j) v[j] = j < w ? col[j] : 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (j < w) Uc[sI * wu + j] = v[j];
        }
    }
    // The coupled rows x coupled columns entries are not touched by steps
    // 1 and 2, so the first round of trailing tiles is loaded now and its
    // latency overlaps the diagonal LU, the inverses and the solves.  (A
    // barrier waits for LDS traffic only; these loads stay in flight.)
    if (nr > 0) load_tiles(wave);
    __syncthreads();
    if (wave == 0) lu16_wave0(Pn, T, w, lane, r0 + c0, info);
    __syncthreads();
    if (wave == 0) {
        if (lane < w) {
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (j < w) D[c0 + lane + (size_t)(c0 + j) * b] = Pn[j * T + lane];
        }
    } else if (wave == 1) {
        tri_inverse16(Pn, T, w, lane, true, Ui);
    } else if (wave == 2) {
        tri_inverse16(Pn, T, w, lane, false, Li);
    }
    __syncthreads();
    // coupled rows and columns: 16 x 16 output tiles, four waves
    for (int q = wave; q < 2 * nrt; q += 4) {
        double4_t sacc = {0, 0, 0, 0};
        if (q < nrt) {
            // L rows, transposed: X^T = U^{-T} A_rows^T, output element
            // (chunk column lk + 4r, coupled row 16q + li)
            const int ar = 16 * q + li;
            const bool va = ar < nr;
            const int arc = va ? ar : nr - 1;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * kk + lk;
                const double a = Ui[k * 17 + li];                            // (U^{-T})[li][k]
                const double bl = Pn[(k < w ? k : 0) * T + w + arc];
                const double bv = (k < w && va) ? bl : 0.0;
                sacc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, sacc, 0, 0, 0);
            }
            if (va) {
                const size_t row = (size_t)Rs[ar];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int j = lk + 4 * r;
                    if (j < w) {
                        Pn[j * T + w + ar] = sacc[r];
                        D[row + (size_t)(c0 + j) * b] = sacc[r];
                    }
                }
            }
        } else {
            // U columns, transposed: Y^T = A_cols^T L^{-T}, output element
            // (coupled column 16q' + lk + 4r, chunk row li)
            const int qq = q - nrt;
            const int sc = 16 * qq + li;
            const bool vs = sc < nr;
            const int scc = vs ? sc : nr - 1;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * kk + lk;
                const double al = Uc[scc * wu + (k < w ? k : 0)];
                const double a = (k < w && vs) ? al : 0.0;                   // (A_cols^T)[li][k]
                const double bv = Li[li * 17 + k];                            // (L^{-T})[k][li]
                sacc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, sacc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s2 = 16 * qq + lk + 4 * r;
                if (s2 < nr && li < w) {
                    Uc[s2 * wu + li] = sacc[r];
                    D[c0 + li + (size_t)Rs[s2] * b] = sacc[r];
                }
            }
        }
    }
    __syncthreads();
    // trailing update of the coupled rows x coupled columns: the rank-w
    // product on MFMA applied to each wave's loaded tiles, stored back
    for (int q0 = wave; q0 < ntiles; q0 += 32) {
        if (q0 != wave) load_tiles(q0);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + 4 * u;
            if (q < ntiles) {
                const int ti = q / ntl, tj = q - ti * ntl;
                const int sc = 16 * tj + li;
                const int ar = 16 * ti + li;
                const int scc = sc < nr ? sc : nr - 1, arc = ar < nr ? ar : nr - 1;
                const bool va = ar < nr, vcc = sc < nr;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 4 * kk + lk;
                    if (4 * kk < w) {
                        const int kc = k < w ? k : 0;
                        const double al = Uc[scc * wu + kc], bl = Pn[kc * T + w + arc];
                        const double a = (k < w && vcc) ? -al : 0.0;   // (U^T)[sc][k]
                        const double bv = (k < w && va) ? bl : 0.0;    // (L^T)[k][ar]
                        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[u], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int sc2 = 16 * tj + lk + 4 * r;
                    if (vr[u] && sc2 < nr) D[rowo[u] + (size_t)Rs[sc2] * b] = acc[u][r];
                }
            }
        }
    }
    __syncthreads();
}

__device__ __attribute__((always_inline)) void getrf_chunked(double *__restrict__ slab, const LevelDev &L,
                                                              const ChunkDev *__restrict__ chunks,
                                                              const int32_t *__restrict__ crows, double *lds,
                                                              unsigned long long *__restrict__ info) {
    double *__restrict__ D = slab + L.offD;
    const int b = L.b;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int maxnr = L.pad;                    // largest coupled-row count of a chunk
    int *Rbuf0 = (int *)lds;                    // coupled rows of the current / next chunk
    int *Rbuf1 = Rbuf0 + maxnr;
    double *Ui = lds + ((2 * maxnr + 1) >> 1);  // 16 x 17 inverse of U_cc
    double *Li = Ui + 16 * 17;                  // 16 x 17 inverse of L_cc
    double *work = Li + 16 * 17;
    {
        const ChunkDev C = chunks[L.chunk_begin];
        for (int q = tid; q < C.nr; q += 256) Rbuf0[q] = crows[C.roff + q];
    }
    __syncthreads();
    for (int ch = L.chunk_begin; ch < L.chunk_end; ++ch) {
        const ChunkDev C = chunks[ch];
        const int *Rs = ((ch - L.chunk_begin) & 1) ? Rbuf1 : Rbuf0;
        int *Rn = ((ch - L.chunk_begin) & 1) ? Rbuf0 : Rbuf1;
        // the next chunk's coupled rows go to the other buffer; the step's
        // first barrier orders them before their use
        if (ch + 1 < L.chunk_end) {
            const ChunkDev Cn = chunks[ch + 1];
            for (int q = tid; q < Cn.nr; q += 256) Rn[q] = crows[Cn.roff + q];
        }
        if (C.w == 16)
            getrf_chunk_step<16>(D, b, L.r0, C, Rs, Ui, Li, work, info, wave, lane, tid);
        else
            getrf_chunk_step<0>(D, b, L.r0, C, Rs, Ui, Li, work, info, wave, lane, tid);
    }
}

// ------------------------------------------------- dense GETRF (b <= 128)
// Diagonal blocks of at most 128 rows: the whole block in LDS, blocked
// right-looking LU with 16-column panels.  One wave factors the panel in
// registers (each lane owns up to two rows; pivot row values are broadcast
// with lane shuffles), all threads solve the panel's U rows, and the four
// waves apply the trailing update as 16 x 16 FP64 MFMA tiles.
__device__ void getrf_dense(double *__restrict__ slab, const LevelDev &L, double *ds,
                            unsigned long long *__restrict__ info) {
    double *__restrict__ D = slab + L.offD;
    const int b = L.b;
    const int ldd = b | 1;                 // odd stride: conflict-free column-strided LDS access
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int bb = b * b;
    for (int e0 = tid; e0 < bb; e0 += 256 * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + 256 * u;
            v[u] = e < bb ? D[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + 256 * u;
            if (e < bb) {
                const int c = e / b;
                ds[c * ldd + (e - c * b)] = v[u];
            }
        }
    }
    __syncthreads();
    for (int c0 = 0; c0 < b; c0 += 16) {
        const int cw = min(16, b - c0);
        if (wave == 0) {
            const int r0 = c0 + lane, r1 = c0 + 64 + lane;
            const bool v0ok = r0 < b, v1ok = r1 < b;
            double v0[16], v1[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                v0[j] = (j < cw && v0ok) ? ds[(c0 + j) * ldd + r0] : 0.0;
                v1[j] = (j < cw && v1ok) ? ds[(c0 + j) * ldd + r1] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (k < cw) {
                    // pivot row c0 + k (held by lane k): all shuffles issued first
                    double u[16];
#pragma unroll
                    for (int j = k; j < 16; ++j) u[j] = __shfl(v0[j], k, 64);
                    const double piv = u[k];
                    if (lane == 0 && !(piv != 0.0 && isfinite(piv)))
                        atomicMin(info, (unsigned long long)(L.r0 + c0 + k));
                    const double l1 = v1[k] / piv;
                    v1[k] = l1;
#pragma unroll
                    for (int j = k + 1; j < 16; ++j) v1[j] -= l1 * u[j];
                    if (lane > k) {
                        const double l0 = v0[k] / piv;
                        v0[k] = l0;
#pragma unroll
                        for (int j = k + 1; j < 16; ++j) v0[j] -= l0 * u[j];
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (j < cw && v0ok) ds[(c0 + j) * ldd + r0] = v0[j];
                if (j < cw && v1ok) ds[(c0 + j) * ldd + r1] = v1[j];
            }
        }
        __syncthreads();
        for (int col = c0 + cw + tid; col < b; col += 256) {
            double u[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) u[j] = j < cw ? ds[col * ldd + c0 + j] : 0.0;
#pragma unroll
            for (int j = 1; j < 16; ++j) {
                double v = u[j];
#pragma unroll
                for (int jp = 0; jp < j; ++jp) v -= ds[(c0 + jp) * ldd + c0 + j] * u[jp];
                u[j] = v;
            }
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (j < cw) ds[col * ldd + c0 + j] = u[j];
        }
        __syncthreads();
        const int t0 = c0 + cw;
        const int nrem = b - t0;
        const int ntl = (nrem + 15) >> 4;
        for (int t = wave; t < ntl * ntl; t += 4) {
            const int ti = t / ntl, tj = t - ti * ntl;
            const int row0 = t0 + 16 * ti, col0 = t0 + 16 * tj;
            const int ccol = col0 + li;
            double4_t acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + lk + 4 * r;
                acc[r] = (row < b && ccol < b) ? ds[ccol * ldd + row] : 0.0;
            }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * kk + lk;
                const double a = (k < cw && row0 + li < b) ? -ds[(c0 + k) * ldd + row0 + li] : 0.0;
                const double bv = (k < cw && ccol < b) ? ds[ccol * ldd + c0 + k] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + lk + 4 * r;
                if (row < b && ccol < b) ds[ccol * ldd + row] = acc[r];
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < bb; e += 256) {
        const int c = e / b;
        D[e] = ds[c * ldd + (e - c * b)];
    }
}

// GETRF of every level of a wave: one workgroup per diagonal block, the
// LDS-resident path for blocks up to 128 rows, the chunked path above.
__global__ __launch_bounds__(256) void k_getrf_wave(double *__restrict__ slab, const LevelDev *__restrict__ levels,
                                                    const int32_t *__restrict__ lvl,
                                                    const ChunkDev *__restrict__ chunks,
                                                    const int32_t *__restrict__ crows,
                                                    unsigned long long *__restrict__ info) {
    extern __shared__ double lds[];
    const LevelDev L = levels[lvl[blockIdx.x]];
    if (L.b <= 128)
        getrf_dense(slab, L, lds, info);
    else
        getrf_chunked(slab, L, chunks, crows, lds, info);
}

hipError_t launch_getrf_wave(const DevPlan &d, const int32_t *lvl, int nlev, int lds_bytes, hipStream_t s) {
    hipLaunchKernelGGL(k_getrf_wave, dim3((unsigned)nlev), dim3(256), (size_t)lds_bytes, s, d.slab, d.levels, lvl,
                       d.chunks, d.chunk_rows, d.info);
    return hipGetLastError();
}

// ------------------------------------------- compact coupled triangles
// One workgroup per tile row tr of the compact triangles (see LevelDev):
// copies rows [16 tr, 16 tr + 16) of Tu = U_ii[K, K] and Tl = L_ii[K, K]^T
// from the factored diagonal block, then inverts the two diagonal tiles
// (back substitution per column, FP64 divisions by the pivots).
__global__ __launch_bounds__(256) void k_tri_gather(const double *__restrict__ slab, double *__restrict__ tri,
                                                    const LevelDev *__restrict__ levels,
                                                    const int32_t *__restrict__ lvl,
                                                    const int32_t *__restrict__ Kidx) {
    __shared__ double du[16][17], dl[16][17];
    const LevelDev L = levels[lvl[blockIdx.y]];
    const int kp = L.kp, kap = L.kappa, b = L.b, nt = kp >> 4;
    const int tr = blockIdx.x;
    if (tr >= nt) return;
    const double *__restrict__ D = slab + L.offD;
    const int32_t *__restrict__ K = Kidx + L.Koff;
    double *__restrict__ Tu = tri + L.offT;
    double *__restrict__ Tl = Tu + (size_t)kp * kp;
    double *__restrict__ Iu = Tl + (size_t)kp * kp;
    double *__restrict__ Il = Iu + (size_t)nt * 256;
    const int width = kp - 16 * tr;
    // thread (column cc, row rr): column index K[t2] from global once, then
    // the 16 rows' values of U and L^T issued together
    for (int cc = threadIdx.x; cc < width; cc += 256) {
        const int t2 = 16 * tr + cc;
        const bool c_in = t2 < kap;
        const size_t k2 = c_in ? (size_t)K[t2] : 0;
        double u[16], lt[16];
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            const int t1 = 16 * tr + rr;
            const bool in = c_in && t1 < kap;
            const size_t k1 = in ? (size_t)K[t1] : 0;
            u[rr] = (in && t1 <= t2) ? D[k1 + k2 * b] : 0.0;
            lt[rr] = (in && t1 < t2) ? D[k2 + k1 * b] : 0.0;
        }
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            const int t1 = 16 * tr + rr;
            const bool in = c_in && t1 < kap;
            double uu = u[rr], ll = lt[rr];
            if (t1 == t2) {
                ll = 1.0;
                if (!in) uu = 1.0;
            }
            Tu[(size_t)t1 * kp + t2] = uu;
            Tl[(size_t)t1 * kp + t2] = ll;
            if (cc < 16) {
                du[rr][cc] = uu;
                dl[rr][cc] = ll;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        const int j = threadIdx.x & 15;
        const bool upper = threadIdx.x < 16;
        double x[16];
#pragma unroll
        for (int r = 15; r >= 0; --r) {
            double v = (r == j) ? 1.0 : 0.0;
#pragma unroll
            for (int q = r + 1; q < 16; ++q) v -= (upper ? du[r][q] : dl[r][q]) * x[q];
            x[r] = upper ? v / du[r][r] : v;
        }
        double *out = (upper ? Iu : Il) + (size_t)tr * 256;
#pragma unroll
        for (int r = 0; r < 16; ++r) out[r * 16 + j] = x[r];
    }
}

hipError_t launch_tri_gather_wave(const DevPlan &d, const int32_t *lvl, int nlev, int max_nt, hipStream_t s) {
    if (max_nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tri_gather, dim3((unsigned)max_nt, (unsigned)nlev), dim3(256), 0, s, d.slab, d.tri,
                       d.levels, lvl, d.K_idx);
    return hipGetLastError();
}

// ------------------------------------------------------ panel solves (v2)
// Alg. 1 "B_ij <- L_ii^{-1} B_ij" and "B_ji <- B_ji U_ii^{-1}" for all panel
// rows of level i: X <- X T^{-1} with X = P_i, T = Tu (blockIdx.y == 0) or
// X = Qt_i, T = Tl (blockIdx.y == 1).  A workgroup holds RT = 32 (or 16)
// panel rows; right-looking over 16-column chunks c: X_c <- X_c T_cc^{-1}
// (inverted diagonal tile), then X_c' -= X_c T_cc' for the structurally
// nonzero tiles c' > c.  Every product is a 16 x 16 x 16 FP64 MFMA block.
// The rows live in LDS when RT x kp doubles fit, else in the panel itself.
template <int RT, bool IN_LDS>
__global__ __launch_bounds__(256) void k_panel_solve(double *__restrict__ slab, const double *__restrict__ tri,
                                                     const LevelDev *__restrict__ levels,
                                                     const int32_t *__restrict__ lvl,
                                                     const int32_t *__restrict__ trow_ptr,
                                                     const int32_t *__restrict__ trow_idx) {
    extern __shared__ double xs_lds[];
    const LevelDev L = levels[lvl[blockIdx.z]];
    const int kp = L.kp, kap = L.kappa, m = L.m, nt = kp >> 4;
    if (kp == 0 || (int)blockIdx.x * RT >= m) return;
    const int panel = blockIdx.y;
    double *__restrict__ X = slab + (panel == 0 ? L.offP : L.offQ);
    const double *__restrict__ T = tri + L.offT + (size_t)panel * kp * kp;
    const double *__restrict__ Tinv = tri + L.offT + 2 * (size_t)kp * kp + (size_t)panel * nt * 256;
    const int32_t *__restrict__ tptr = trow_ptr + L.trow;
    const int a0 = blockIdx.x * RT;
    const int nrow = min(RT, m - a0);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    constexpr int LD = RT + 1;
    constexpr int NH = RT / 16;
    // element (t, r) of the row block: column t of K space, row r
    auto ld_x = [&](int t, int r) -> double {
        if (IN_LDS) return xs_lds[t * LD + r];
        return (r < nrow && t < kap) ? X[a0 + r + (size_t)t * m] : 0.0;
    };
    auto st_x = [&](int t, int r, double v) {
        if (IN_LDS)
            xs_lds[t * LD + r] = v;
        else if (r < nrow && t < kap)
            X[a0 + r + (size_t)t * m] = v;
    };
    if (IN_LDS) {
        // column t of the row block is RT contiguous doubles of X
        for (int t0 = tid / RT; t0 < kp; t0 += 8 * (256 / RT)) {
            const int r = tid % RT;
            // unconditional loads from clamped addresses, issued together;
            // the padding is zeroed when the values are stored to LDS
            const int rc = r < nrow ? r : nrow - 1;
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = t0 + u * (256 / RT);
                v[u] = X[a0 + rc + (size_t)(t < kap ? t : kap - 1) * m];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = t0 + u * (256 / RT);
                if (t < kp) xs_lds[t * LD + r] = (r < nrow && t < kap) ? v[u] : 0.0;
            }
        }
        __syncthreads();
    }
    for (int c = 0; c < nt; ++c) {
        double4_t acc = {0, 0, 0, 0};
        if (wave < NH) {
            const int h = wave;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * kk + lk;
                const double a = ld_x(16 * c + k, 16 * h + li);
                const double bv = Tinv[(size_t)c * 256 + k * 16 + li];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
            }
        }
        __syncthreads();
        if (wave < NH) {
#pragma unroll
            for (int r = 0; r < 4; ++r) st_x(16 * c + li, 16 * wave + lk + 4 * r, acc[r]);
        }
        __syncthreads();
        const int q0 = tptr[c], q1 = tptr[c + 1];
        for (int q = wave; q < (q1 - q0) * NH; q += 4) {
            const int cc = trow_idx[q0 + q / NH];
            const int h = q % NH;
            double4_t u;
#pragma unroll
            for (int r = 0; r < 4; ++r) u[r] = ld_x(16 * cc + li, 16 * h + lk + 4 * r);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * kk + lk;
                const double a = -ld_x(16 * c + k, 16 * h + li);
                const double bv = T[(size_t)(16 * c + k) * kp + 16 * cc + li];
                u = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, u, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) st_x(16 * cc + li, 16 * h + lk + 4 * r, u[r]);
        }
        __syncthreads();
    }
    if (IN_LDS) {
        for (int e = tid; e < RT * kap; e += 256) {
            const int t = e / RT, r = e - t * RT;
            if (r < nrow) X[a0 + r + (size_t)t * m] = xs_lds[t * LD + r];
        }
    }
}

hipError_t launch_panel_solve_wave(const DevPlan &d, const int32_t *lvl, int nlev, int max_m, int max_kp,
                                   hipStream_t s) {
    if (max_m <= 0 || max_kp <= 0) return hipSuccess;
    const size_t lds32 = (size_t)33 * max_kp * sizeof(double), lds16 = (size_t)17 * max_kp * sizeof(double);
    if (lds32 <= 150 * 1024) {
        dim3 grid((unsigned)((max_m + 31) / 32), 2, (unsigned)nlev);
        hipLaunchKernelGGL((k_panel_solve<32, true>), grid, dim3(256), lds32, s, d.slab, d.tri, d.levels, lvl,
                           d.trow_ptr, d.trow_idx);
    } else if (lds16 <= 150 * 1024) {
        dim3 grid((unsigned)((max_m + 15) / 16), 2, (unsigned)nlev);
        hipLaunchKernelGGL((k_panel_solve<16, true>), grid, dim3(256), lds16, s, d.slab, d.tri, d.levels, lvl,
                           d.trow_ptr, d.trow_idx);
    } else {
        dim3 grid((unsigned)((max_m + 15) / 16), 2, (unsigned)nlev);
        hipLaunchKernelGGL((k_panel_solve<16, false>), grid, dim3(256), 0, s, d.slab, d.tri, d.levels, lvl,
                           d.trow_ptr, d.trow_idx);
    }
    return hipGetLastError();
}

// --------------------------------------------------------------------- SSSSM
// Alg. 1 "B_kj <- B_kj - B_ki B_ij" for every target (k, j) of level i in one
// launch: the product C = P_i Qt_i^T (m x m, inner dimension kappa) on FP64
// MFMA (v_mfma_f64_16x16x4f64), tiled 64 x 64 over the whole m x m range
// regardless of segment boundaries.  One workgroup per tile, four waves of
// 32 x 32 (2 x 2 MFMA blocks each); both operands are staged through LDS 16
// inner indices at a time, double-buffered, the next slice's global loads in
// flight during the current slice's MFMAs.  Element (a, b) of C belongs to
// the target of segment pair (seg(a), seg(b)) and is subtracted at
//     stgt[seg(a) * nseg + seg(b)] + RO[seg(b)][a] + CO[seg(a)][b]
// unless an offset is -1 (S has no entry there).  Targets are distinct
// within a level, so the stores never collide.
//
// MFMA f64 16x16x4 operand layout (lane l): A[i][k] with i = l % 16,
// k = l / 16; B[k][j] with j = l % 16, k = l / 16; result element r of lane l
// is D[l / 16 + 4 * r][l % 16] (checked on gfx950 with a lane-layout probe).
constexpr int kSsKC = 16;               // inner indices per LDS slice
constexpr int kSsLd = kSsssmTile + 4;   // LDS row stride (doubles)

__global__ __launch_bounds__(256) void k_ssssm(double *__restrict__ slab, const LevelDev *__restrict__ levels,
                                               int level, const int32_t *__restrict__ rseg,
                                               const int64_t *__restrict__ stgt,
                                               const int32_t *__restrict__ maps) {
    __shared__ double As[2][kSsKC][kSsLd], Bs[2][kSsKC][kSsLd];
    const LevelDev L = levels[level];
    const int m = L.m, kp = (L.kappa + 15) & ~15, nseg = L.seg_end - L.seg_begin;
    const int nt = (m + kSsssmTile - 1) / kSsssmTile;
    const int ti = blockIdx.x / nt, tj = blockIdx.x - ti * nt;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int wr = wave >> 1, wc = wave & 1;

    // epilogue addressing, loaded first so that its latency overlaps the
    // products: this lane's 8 rows a and 2 columns b of the tile
    const int32_t *__restrict__ RS = rseg + L.Roff;
    const int32_t *__restrict__ RO = maps + L.moff;
    const int32_t *__restrict__ CO = RO + (size_t)nseg * m;
    const int64_t *__restrict__ TG = stgt + L.task_begin;
    int rowa[2][4], colb[2], sa[2][4], sb[2];
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        colb[bj] = tj * kSsssmTile + wc * 32 + bj * 16 + li;
        sb[bj] = RS[min(colb[bj], m - 1)];
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            rowa[bi][r] = ti * kSsssmTile + wr * 32 + bi * 16 + lk + 4 * r;
            sa[bi][r] = RS[min(rowa[bi][r], m - 1)];
        }
    int ro[2][2][4], co[2][2][4];
    int64_t tg[2][2][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                ro[bi][bj][r] = RO[(size_t)sb[bj] * m + min(rowa[bi][r], m - 1)];
                co[bi][bj][r] = CO[(size_t)sa[bi][r] * m + min(colb[bj], m - 1)];
                tg[bi][bj][r] = TG[sa[bi][r] * nseg + sb[bj]];
            }

    // operand staging: thread (row lr, inner kq) moves P / Qt entries
    // (row, k0 + kq + 4u), u < 4; rows past m read row m - 1 (never stored)
    const int lr = tid & 63, kq = tid >> 6;
    const double *__restrict__ pp = slab + L.offP + min(ti * kSsssmTile + lr, m - 1) + (size_t)kq * m;
    const double *__restrict__ qp = slab + L.offQ + min(tj * kSsssmTile + lr, m - 1) + (size_t)kq * m;
    double ra[4], rb[4];
    auto gload = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ra[u] = pp[(size_t)(k0 + 4 * u) * m];
            rb[u] = qp[(size_t)(k0 + 4 * u) * m];
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            As[buf][kq + 4 * u][lr] = ra[u];
            Bs[buf][kq + 4 * u][lr] = rb[u];
        }
    };
    double4_t c00 = {0, 0, 0, 0}, c01 = c00, c10 = c00, c11 = c00;
    const int nch = kp / kSsKC;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (c + 1 < nch) gload((c + 1) * kSsKC);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = 4 * kk + lk;
            const double a0 = As[buf][k][wr * 32 + li], a1 = As[buf][k][wr * 32 + 16 + li];
            const double b0 = Bs[buf][k][wc * 32 + li], b1 = Bs[buf][k][wc * 32 + 16 + li];
            c00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, c00, 0, 0, 0);
            c01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, c01, 0, 0, 0);
            c10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, c10, 0, 0, 0);
            c11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, c11, 0, 0, 0);
        }
        if (c + 1 < nch) lstore(buf ^ 1);
        __syncthreads();
    }

    // subtract from the targets: all loads first, then the stores
    const double4_t acc[2][2] = {{c00, c01}, {c10, c11}};
    int64_t off[2][2][4];
    double tv[2][2][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const bool ok = rowa[bi][r] < m && colb[bj] < m && ro[bi][bj][r] >= 0 && co[bi][bj][r] >= 0;
                off[bi][bj][r] = ok ? tg[bi][bj][r] + ro[bi][bj][r] + co[bi][bj][r] : -1;
                tv[bi][bj][r] = slab[ok ? off[bi][bj][r] : 0];
            }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (off[bi][bj][r] >= 0) slab[off[bi][bj][r]] = tv[bi][bj][r] - acc[bi][bj][r];
}

hipError_t launch_ssssm(const DevPlan &d, int level, int m, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    const int nt = (m + kSsssmTile - 1) / kSsssmTile;
    hipLaunchKernelGGL(k_ssssm, dim3((unsigned)(nt * nt)), dim3(256), 0, s, d.slab, d.levels, level, d.rseg,
                       d.stgt, d.maps);
    return hipGetLastError();
}

// --------------------------------------------------------------------- solve
// W (n x nc, ld n) holds the permuted right-hand sides.  Non-transposed:
// forward with L (unit lower, D_i strict lower part and P_i), backward with U
// (D_i upper part and Qt_i).  Transposed: forward with U^T (D_i^T upper part,
// Qt_i), backward with L^T (D_i^T strict lower part, P_i).
__global__ void k_gather_perm(const double *__restrict__ B, int64_t ld, double *__restrict__ W,
                              const int32_t *__restrict__ perm, int64_t n, int nc) {
    const int64_t total = n * nc;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t c = e / n, k = e - c * n;
        W[e] = B[perm[k] + c * ld];
    }
}

__global__ void k_scatter_perm(const double *__restrict__ W, double *__restrict__ X, int64_t ld,
                               const int32_t *__restrict__ perm, int64_t n, int nc) {
    const int64_t total = n * nc;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t c = e / n, k = e - c * n;
        X[perm[k] + c * ld] = W[e];
    }
}

hipError_t launch_gather_perm(const DevPlan &d, const double *B, int64_t ld, int nc, hipStream_t s) {
    int64_t blocks = (d.n * nc + 255) / 256;
    if (blocks < 1) return hipSuccess;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_gather_perm, dim3((unsigned)blocks), dim3(256), 0, s, B, ld, d.scratch, d.perm, d.n, nc);
    return hipGetLastError();
}

hipError_t launch_scatter_perm(const DevPlan &d, double *X, int64_t ld, int nc, hipStream_t s) {
    int64_t blocks = (d.n * nc + 255) / 256;
    if (blocks < 1) return hipSuccess;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_scatter_perm, dim3((unsigned)blocks), dim3(256), 0, s, d.scratch, X, ld, d.perm, d.n, nc);
    return hipGetLastError();
}

// Lower-triangular sweep inside D_i.  trans == 0: unit lower L (D[r + k*b],
// r > k).  trans == 1: U^T, lower with diagonal (U^T[r][k] = D[k + r*b]).
__global__ __launch_bounds__(1024) void k_fwd_diag(const double *__restrict__ slab, const LevelDev *__restrict__ levels,
                                                   int level, double *__restrict__ W, int64_t n, int nc, int trans) {
    extern __shared__ double cv[];  // cv[c*b + r]
    const LevelDev L = levels[level];
    const int b = L.b;
    const double *__restrict__ D = slab + L.offD;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < b * nc; e += nt) {
        const int c = e / b, r = e - c * b;
        cv[e] = W[L.r0 + r + (size_t)c * n];
    }
    __syncthreads();
    for (int k = 0; k < b; ++k) {
        if (trans) {
            if (tid < nc) cv[tid * b + k] = cv[tid * b + k] / D[k + (size_t)k * b];
            __syncthreads();
        }
        const int rows = b - k - 1;
        for (int e = tid; e < rows * nc; e += nt) {
            const int c = e / rows, r = k + 1 + (e - c * rows);
            const double lv = trans ? D[k + (size_t)r * b] : D[r + (size_t)k * b];
            cv[c * b + r] -= lv * cv[c * b + k];
        }
        __syncthreads();
    }
    for (int e = tid; e < b * nc; e += nt) {
        const int c = e / b, r = e - c * b;
        W[L.r0 + r + (size_t)c * n] = cv[e];
    }
}

// Upper-triangular sweep inside D_i.  trans == 0: U (D[r + k*b], r <= k).
// trans == 1: L^T, unit upper (L^T[r][k] = D[k + r*b], r < k).
__global__ __launch_bounds__(1024) void k_bwd_diag(const double *__restrict__ slab, const LevelDev *__restrict__ levels,
                                                   int level, double *__restrict__ W, int64_t n, int nc, int trans) {
    extern __shared__ double cv[];
    const LevelDev L = levels[level];
    const int b = L.b;
    const double *__restrict__ D = slab + L.offD;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int e = tid; e < b * nc; e += nt) {
        const int c = e / b, r = e - c * b;
        cv[e] = W[L.r0 + r + (size_t)c * n];
    }
    __syncthreads();
    for (int k = b - 1; k >= 0; --k) {
        if (!trans) {
            if (tid < nc) cv[tid * b + k] = cv[tid * b + k] / D[k + (size_t)k * b];
            __syncthreads();
        }
        const int rows = k;
        for (int e = tid; e < rows * nc; e += nt) {
            const int c = e / rows, r = e - c * rows;
            const double uv = trans ? D[k + (size_t)r * b] : D[r + (size_t)k * b];
            cv[c * b + r] -= uv * cv[c * b + k];
        }
        __syncthreads();
    }
    for (int e = tid; e < b * nc; e += nt) {
        const int c = e / b, r = e - c * b;
        W[L.r0 + r + (size_t)c * n] = cv[e];
    }
}

// W[rows_i[a]] -= X[a, :] . W[r0 + K_i]   (X = P_i, or Qt_i when transposed)
__global__ void k_fwd_update(const double *__restrict__ slab, const LevelDev *__restrict__ levels, int level,
                             const int32_t *__restrict__ Kidx, const int32_t *__restrict__ Ridx,
                             double *__restrict__ W, int64_t n, int nc, int trans) {
    const LevelDev L = levels[level];
    const int m = L.m, kap = L.kappa;
    const double *__restrict__ X = slab + (trans ? L.offQ : L.offP);
    const int32_t *__restrict__ K = Kidx + L.Koff;
    const int32_t *__restrict__ R = Ridx + L.Roff;
    const int64_t total = (int64_t)m * nc;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / m), a = (int)(e - (int64_t)c * m);
        const double *__restrict__ Wc = W + (size_t)c * n;
        double acc = 0.0;
        for (int t = 0; t < kap; ++t) acc += X[a + (size_t)t * m] * Wc[L.r0 + K[t]];
        W[R[a] + (size_t)c * n] -= acc;
    }
}

// W[r0 + K_i[t]] -= sum_a X[a, t] W[rows_i[a]]   (X = Qt_i, or P_i when transposed)
__global__ __launch_bounds__(64) void k_bwd_update(const double *__restrict__ slab, const LevelDev *__restrict__ levels,
                                                   int level, const int32_t *__restrict__ Kidx,
                                                   const int32_t *__restrict__ Ridx, double *__restrict__ W,
                                                   int64_t n, int trans) {
    const LevelDev L = levels[level];
    const int m = L.m;
    const int t = blockIdx.x, c = blockIdx.y;
    const double *__restrict__ X = slab + (trans ? L.offP : L.offQ) + (size_t)t * m;
    const int32_t *__restrict__ R = Ridx + L.Roff;
    const double *__restrict__ Wc = W + (size_t)c * n;
    double acc = 0.0;
    for (int a = threadIdx.x; a < m; a += 64) acc += X[a] * Wc[R[a]];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (threadIdx.x == 0) W[L.r0 + Kidx[L.Koff + t] + (size_t)c * n] -= acc;
}

hipError_t launch_fwd_diag(const DevPlan &d, int level, int b, int nc, int trans, hipStream_t s) {
    hipLaunchKernelGGL(k_fwd_diag, dim3(1), dim3(1024), (size_t)b * nc * sizeof(double), s, d.slab, d.levels,
                       level, d.scratch, d.n, nc, trans);
    return hipGetLastError();
}

hipError_t launch_bwd_diag(const DevPlan &d, int level, int b, int nc, int trans, hipStream_t s) {
    hipLaunchKernelGGL(k_bwd_diag, dim3(1), dim3(1024), (size_t)b * nc * sizeof(double), s, d.slab, d.levels,
                       level, d.scratch, d.n, nc, trans);
    return hipGetLastError();
}

hipError_t launch_fwd_update(const DevPlan &d, int level, int m, int nc, int trans, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    int64_t blocks = ((int64_t)m * nc + 255) / 256;
    hipLaunchKernelGGL(k_fwd_update, dim3((unsigned)blocks), dim3(256), 0, s, d.slab, d.levels, level, d.K_idx,
                       d.R_idx, d.scratch, d.n, nc, trans);
    return hipGetLastError();
}

hipError_t launch_bwd_update(const DevPlan &d, int level, int kappa, int nc, int trans, hipStream_t s) {
    if (kappa <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bwd_update, dim3((unsigned)kappa, (unsigned)nc), dim3(64), 0, s, d.slab, d.levels, level,
                       d.K_idx, d.R_idx, d.scratch, d.n, trans);
    return hipGetLastError();
}

// ------------------------------------------------------------ backward error
// norms (as bit patterns of non-negative doubles, so integer max == fp max):
// [c] = ||b_c - op(A) x_c||_inf, [16 + c] = ||x_c||_inf, [32 + c] = ||b_c||_inf,
// [48] = ||op(A)||_inf.  op(A) = A uses the CSR rows; op(A) = A^T the CSC columns.
__device__ inline void atomic_max_nonneg(unsigned long long *p, double v) {
    atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

__global__ void k_residual_norms(const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                 const int64_t *__restrict__ vidx, const double *__restrict__ vals,
                                 const double *__restrict__ B, const double *__restrict__ X, int64_t ld,
                                 int64_t n, int nc, unsigned long long *__restrict__ norms) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double asum = 0.0;
        for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) asum += fabs(vals[vidx ? vidx[q] : q]);
        atomic_max_nonneg(norms + 48, asum);
        for (int c = 0; c < nc; ++c) {
            const double *__restrict__ xc = X + (size_t)c * ld;
            double r = B[i + (size_t)c * ld];
            for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) r -= vals[vidx ? vidx[q] : q] * xc[idx[q]];
            atomic_max_nonneg(norms + c, fabs(r));
            atomic_max_nonneg(norms + 16 + c, fabs(xc[i]));
            atomic_max_nonneg(norms + 32 + c, fabs(B[i + (size_t)c * ld]));
        }
    }
}

__global__ void k_norms_reset(unsigned long long *norms) {
    if (threadIdx.x < 64) norms[threadIdx.x] = 0ull;
}

hipError_t launch_residual_norms(const DevPlan &d, const double *values, const double *B, const double *X,
                                 int64_t ld, int nc, int trans, hipStream_t s) {
    hipLaunchKernelGGL(k_norms_reset, dim3(1), dim3(64), 0, s, d.norms);
    if (d.n <= 0) return hipGetLastError();
    int64_t blocks = (d.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (!trans)
        hipLaunchKernelGGL(k_residual_norms, dim3((unsigned)blocks), dim3(256), 0, s, d.a_rowptr, d.a_colidx,
                           (const int64_t *)nullptr, values, B, X, ld, d.n, nc, d.norms);
    else
        hipLaunchKernelGGL(k_residual_norms, dim3((unsigned)blocks), dim3(256), 0, s, d.at_colptr, d.at_rowidx,
                           d.at_vidx, values, B, X, ld, d.n, nc, d.norms);
    return hipGetLastError();
}

hipError_t setup_kernel_attributes() {
    hipError_t e;
    e = hipFuncSetAttribute((const void *)k_fwd_diag, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_bwd_diag, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_getrf_wave, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_panel_solve<32, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_panel_solve<16, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    return e;
}

}  // namespace slu
