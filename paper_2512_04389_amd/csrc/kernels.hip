// gfx950 kernels of the blocked sparse LU (right-looking, Algorithm 1).
//
// Storage (see analyze.hpp): per level i a dense diagonal block D_i
// (column-major b x b) and two panels over the coupled index sets,
// P_i[a, t] = L(rows_i[a], r0 + K_i[t]) and Qt_i[a, t] = U(r0 + K_i[t], rows_i[a]),
// both m x kappa column-major.  Entries of those dense arrays that lie outside
// the symbolic pattern start at 0.0 and stay exactly 0.0: every product that
// could reach them has a structurally zero factor.
#include "kernels.hpp"

#include <type_traits>

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

namespace slu {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// Value of a lane's double in every lane (the lane index must be the same in
// all lanes of the wave): two v_readlane into scalar registers.
__device__ __forceinline__ double bcast_lane(double v, int k) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)x, k);
    const int hi = __builtin_amdgcn_readlane((int)(x >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Value of lane J of each 16-lane row in every lane of that row (DPP
// row_newbcast, two 32-bit moves).
template <int J>
__device__ __forceinline__ double bcast16(double v) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)x, 0x150 + J, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), 0x150 + J, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Value of v in lane src of the wave, per lane (LDS crossbar permute, no LDS
// memory; every lane of the wave must be active).
__device__ __forceinline__ double perm_lane(double v, int src) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)x);
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(x >> 32));
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

// In-place no-pivot LU of a w x w (w <= 16) block held by one wave in a 2D
// layout: lane i + 16 g holds a[s] = A(i, 4 g + s) (zeros outside w x w).
// Pivot k: its value by readlane, the pivot row to every lane of each
// 16-lane row by DPP row broadcast, the multipliers of column k from its
// column group to the other groups by a lane permute; each lane then
// updates its four entries.  Lane k of group 0 ends with 1 / U(k, k) in
// myrd; bad is the first zero / non-finite pivot (16 if none), uniform.
template <int K>
__device__ __forceinline__ void lu16_step(double (&a)[4], int i, int g, int w, int &bad, double &myrd) {
    if (K < w) {
        constexpr int g0 = K >> 2, s0 = K & 3;
        const double piv = bcast_lane(a[s0], K + 16 * g0);
        if (!(piv != 0.0 && isfinite(piv))) bad = min(bad, K);
        const double rp = recip(piv);
        myrd = (i == K && g == 0) ? rp : myrd;
        const double lg = a[s0] * rp;
        if (g == g0 && i > K) a[s0] = lg;
        const double l = perm_lane(lg, i + 16 * g0);
        double u[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) u[s] = bcast16<K>(a[s]);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bool upd = i > K && 4 * g + s > K;
            const double nv = a[s] - l * u[s];
            a[s] = upd ? nv : a[s];
        }
    }
    if constexpr (K + 1 < 16) lu16_step<K + 1>(a, i, g, w, bad, myrd);
}

__device__ __forceinline__ void lu16_2d(double (&a)[4], int w, int lane, int &bad, double &myrd) {
    bad = 16;
    myrd = 0.0;
    lu16_step<0>(a, lane & 15, lane >> 4, w, bad, myrd);
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
//   1. wave 0 factors the w x w diagonal of the chunk in registers;
//   2. the coupled rows (L = A U_cc^{-1}) and coupled columns
//      (U = L_cc^{-1} A) are solved by substitution, one per lane;
//   3. the four waves update the R x R trailing entries with FP64 MFMA;
//   4. the solved panel of steps 1-2 (kept in LDS) is written to D at the
//      start of step 3.
// Pivots are inverted by a reciprocal refined with two Newton steps; a zero
// or non-finite pivot records its permuted column in info[0].
// One column chunk of the chunked GETRF.  W = 16 is the full-width chunk
// (every width guard folds away), W = 8 the width that large dense blocks
// take under the LDS budget; W = 0 takes the width at run time (the last
// chunk of a block, narrower budgets).  Loads guarded per lane read a clamped, valid
// address and select zero, so they are issued without branches.
template <int W, bool TRAIL = true>
__device__ __forceinline__ void getrf_chunk_step(double *__restrict__ D, int b, int r0, const ChunkDev &C,
                                                 const int *Rs, const double *Rd, double *work,
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
    // The coupled-row indices of a round are read from LDS first, all
    // together, and only then are the 32 loads issued: interleaved, every
    // load would wait for its own LDS read.
    auto load_tiles = [&](int q0) {
        int cix[8][4];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + 4 * u;
            const int qc = q < ntiles ? q : ntiles - 1;
            const int ti = qc / ntl, tj = qc - ti * ntl;
            const int ra = 16 * ti + li;
            vr[u] = q < ntiles && ra < nr;
            rowo[u] = (size_t)Rs[ra < nr ? ra : nr - 1];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int sc = 16 * tj + lk + 4 * r;
                cix[u][r] = Rs[sc < nr ? sc : nr - 1];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        // entries outside the coupled set read a clamped valid address; an
        // MFMA output element depends only on its own accumulator input and
        // those elements are never stored, so no select is needed (it would
        // make each load wait at once)
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[u][r] = D[rowo[u] + (size_t)cix[u][r] * b];
    };
    // 0/1. Wave 0 loads the chunk's w x w diagonal straight from D and
    // factors it in registers while waves 1-3 stage the coupled part of the
    // panel in LDS: the nr coupled rows of the chunk's columns (items
    // [0, nr)) and the nr coupled columns of its rows (items [nr, 2 nr),
    // contiguous in D), two items per pass so both items' loads are in
    // flight together.  Entries past w are read at a clamped valid address
    // and never stored.  Every wave also issues its first round of trailing
    // tile loads (entries not touched before the trailing update), whose
    // latency overlaps the LU and the solves; a barrier waits for LDS
    // traffic only.
    if (wave == 0) {
        // 2D layout: lane gi + 16 gg holds D(c0 + gi, c0 + 4 gg + s)
        const int gi = lane & 15, gg = lane >> 4;
        const int gic = gi < w ? gi : w - 1;
        double a[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int j = 4 * gg + s;
            a[s] = D[c0 + gic + (size_t)(c0 + (j < w ? j : w - 1)) * b];
        }
        // the diagonal's loads go out first, then the tile loads; the LU
        // waits for the former only.  (The LU is written out in both arms so
        // the wait counts stay exact: after a join the compiler would wait
        // as if the tile loads had been issued on the path without them.)
        int bad;
        double myrd;
        auto lu = [&]() {
#pragma unroll
            for (int s = 0; s < 4; ++s) a[s] = (4 * gg + s < w && gi < w) ? a[s] : 0.0;
            lu16_2d(a, w, lane, bad, myrd);
        };
        if (TRAIL && nr > 0) {
            __builtin_amdgcn_sched_barrier(0);
            load_tiles(0);
            __builtin_amdgcn_sched_barrier(0);
            lu();
        } else {
            lu();
        }
        if (gi < w) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int j = 4 * gg + s;
                if (j < w) {
                    Pn[j * T + gi] = a[s];
                    D[c0 + gi + (size_t)(c0 + j) * b] = a[s];
                }
            }
            if (gg == 0) const_cast<double *>(Rd)[gi] = myrd;
        }
        if (bad < 16 && lane == 0) atomicMin(info, (unsigned long long)(r0 + c0 + bad));
    } else {
        auto load_item = [&](int it, double (&v)[16]) {
            if (it < nr) {
                const size_t row = (size_t)Rs[it];
#pragma unroll
                for (int j = 0; j < 16; ++j) v[j] = D[row + (size_t)(c0 + (j < w ? j : w - 1)) * b];
            } else {
                const double *__restrict__ col = D + c0 + (size_t)Rs[it - nr] * b;
#pragma unroll
                for (int j = 0; j < 16; ++j) v[j] = col[j < w ? j : w - 1];
            }
        };
        auto store_item = [&](int it, const double (&v)[16]) {
            if (it < nr) {
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if (j < w) Pn[j * T + w + it] = v[j];
            } else {
                const int sI = it - nr;
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if (j < w) Uc[sI * wu + j] = v[j];
            }
        };
        for (int it = tid - 64; it < 2 * nr; it += 384) {
            const int it2 = it + 192;
            double v[16], v2[16];
            load_item(it, v);
            if (it2 < 2 * nr) load_item(it2, v2);
            store_item(it, v);
            if (it2 < 2 * nr) store_item(it2, v2);
        }
        if (TRAIL && nr > 0) load_tiles(wave);
    }
    __syncthreads();
    // 2. coupled rows (x U_cc = a) and coupled columns (L_cc y = a): one
    // per lane, forward substitution over the chunk's w columns with the
    // factor entries broadcast from LDS.  Rows take items [0, nr64),
    // columns [nr64, nr64 + nr), so no wave mixes the two kinds.  The
    // results stay in LDS; they go to D in step 4.
    const int nr64 = (nr + 63) & ~63;
    for (int it = tid; it < nr64 + nr; it += 256) {
        double x[16];
        if (it < nr64) {
            if (it < nr) {
#pragma unroll
                for (int j = 0; j < 16; ++j) x[j] = j < w ? Pn[j * T + w + it] : 0.0;
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    if (j < w) {
                        const double xj = x[j] * Rd[j];
                        x[j] = xj;
#pragma unroll
                        for (int j2 = j + 1; j2 < 16; ++j2)
                            if (j2 < w) x[j2] -= xj * Pn[j2 * T + j];          // U(j, j2)
                    }
                }
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if (j < w) Pn[j * T + w + it] = x[j];
            }
        } else {
            const int sI = it - nr64;
#pragma unroll
            for (int j = 0; j < 16; ++j) x[j] = j < w ? Uc[sI * wu + j] : 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (j < w) {
#pragma unroll
                    for (int j2 = j + 1; j2 < 16; ++j2)
                        if (j2 < w) x[j2] -= Pn[j * T + j2] * x[j];            // L(j2, j)
                }
            }
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (j < w) Uc[sI * wu + j] = x[j];
        }
    }
    __syncthreads();
    // 4. the solved panel goes from LDS to D, once the first round of
    // trailing tiles (loaded in steps 0/1, long since arrived) has been
    // waited for: no later step of the block reads these entries, and
    // stores issued any earlier would sit ahead of that wait in the in-order
    // memory counter.  Consecutive threads write consecutive coupled rows of
    // a column, and 16-entry runs of a coupled column.
    if (TRAIL) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    for (int e = tid; e < nr * w; e += 256) {
        const int j = e / nr, it = e - j * nr;
        D[(size_t)Rs[it] + (size_t)(c0 + j) * b] = Pn[j * T + w + it];
    }
    for (int e = tid; e < nr * w; e += 256) {
        const int sI = e / w, j = e - sI * w;
        D[c0 + j + (size_t)Rs[sI] * b] = Uc[sI * wu + j];
    }
    // trailing update of the coupled rows x coupled columns: the rank-w
    // product on MFMA applied to each wave's loaded tiles, stored back.  The
    // first round (tiles loaded in steps 0/1) is peeled off the loop of later
    // rounds, which load their own tiles, so its MFMAs need no wait beyond
    // the one above.
    auto tile_round = [&](int q0) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + 4 * u;
            if (q < ntiles) {
                const int ti = q / ntl, tj = q - ti * ntl;
                const int sc = 16 * tj + li;
                const int ar = 16 * ti + li;
                const int scc = sc < nr ? sc : nr - 1, arc = ar < nr ? ar : nr - 1;
                const bool va = ar < nr, vcc = sc < nr;
                // every LDS read of the tile (operands, store columns) is
                // issued before its MFMAs, so they wait once
                double al[4], bl[4];
                int cs[4];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 4 * kk + lk;
                    const int kc = k < w ? k : 0;
                    al[kk] = Uc[scc * wu + kc];
                    bl[kk] = Pn[kc * T + w + arc];
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int sc2 = 16 * tj + lk + 4 * r;
                    cs[r] = Rs[sc2 < nr ? sc2 : nr - 1];
                }
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = 4 * kk + lk;
                    if (4 * kk < w) {
                        const double a = (k < w && vcc) ? -al[kk] : 0.0;   // (U^T)[sc][k]
                        const double bv = (k < w && va) ? bl[kk] : 0.0;    // (L^T)[k][ar]
                        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[u], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int sc2 = 16 * tj + lk + 4 * r;
                    if (vr[u] && sc2 < nr) D[rowo[u] + (size_t)cs[r] * b] = acc[u][r];
                }
            }
        }
    };
    if (TRAIL) {
        tile_round(wave);
        for (int q0 = wave + 32; q0 < ntiles; q0 += 32) {
            load_tiles(q0);
            tile_round(q0);
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
    double *Rd = lds + ((2 * maxnr + 1) >> 1);  // 1 / U(j, j) of the current chunk
    double *work = Rd + 16;
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
            getrf_chunk_step<16>(D, b, L.r0, C, Rs, Rd, work, info, wave, lane, tid);
        else if (C.w == 8)
            getrf_chunk_step<8>(D, b, L.r0, C, Rs, Rd, work, info, wave, lane, tid);
        else
            getrf_chunk_step<0>(D, b, L.r0, C, Rs, Rd, work, info, wave, lane, tid);
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
    // copy-in: up to 32 loads per thread in flight (clamped addresses), then
    // the LDS stores; blocks of at most 128 rows take two such rounds
    for (int e0 = tid; e0 < bb; e0 += 256 * 32) {
        double v[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) v[u] = D[min(e0 + 256 * u, bb - 1)];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
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
                    for (int j = k; j < 16; ++j) u[j] = bcast_lane(v0[j], k);
                    const double piv = u[k];
                    if (lane == 0 && !(piv != 0.0 && isfinite(piv)))
                        atomicMin(info, (unsigned long long)(L.r0 + c0 + k));
                    const double rp = recip(piv);        // one reciprocal per pivot
                    const double l1 = v1[k] * rp;
                    v1[k] = l1;
#pragma unroll
                    for (int j = k + 1; j < 16; ++j) v1[j] -= l1 * u[j];
                    if (lane > k) {
                        const double l0 = v0[k] * rp;
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

// Split GETRF for waves whose chunked blocks are dense enough that one
// workgroup's trailing updates dominate: step k of every level of the wave
// runs in two launches.  k_getrf_step: one workgroup per level factors the
// diagonal of chunk k, solves its coupled rows and columns and writes them to
// D (a level with b <= 128 is factored whole at k = 0; a level without a
// chunk k does nothing).  k_getrf_trail: one wave per 16 x 16 trailing tile
// of chunk k, numbered per level, applies the rank-w update with FP64 MFMA,
// reading the solved panel from D.  Arithmetic per entry as in the one-launch
// chunked GETRF.
__global__ __launch_bounds__(256) void k_getrf_step(double *__restrict__ slab, const LevelDev *__restrict__ levels,
                                                    const int32_t *__restrict__ lvl, int k,
                                                    const ChunkDev *__restrict__ chunks,
                                                    const int32_t *__restrict__ crows,
                                                    unsigned long long *__restrict__ info) {
    extern __shared__ double lds[];
    const LevelDev L = levels[lvl[blockIdx.x]];
    if (L.b <= 128) {
        if (k == 0) getrf_dense(slab, L, lds, info);
        return;
    }
    const int ch = L.chunk_begin + k;
    if (ch >= L.chunk_end) return;
    double *__restrict__ D = slab + L.offD;
    const int b = L.b;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int maxnr = L.pad;
    int *Rs = (int *)lds;
    double *Rd = lds + ((2 * maxnr + 1) >> 1);
    double *work = Rd + 16;
    const ChunkDev C = chunks[ch];
    for (int q = tid; q < C.nr; q += 256) Rs[q] = crows[C.roff + q];
    __syncthreads();
    if (C.w == 16)
        getrf_chunk_step<16, false>(D, b, L.r0, C, Rs, Rd, work, info, wave, lane, tid);
    else if (C.w == 8)
        getrf_chunk_step<8, false>(D, b, L.r0, C, Rs, Rd, work, info, wave, lane, tid);
    else
        getrf_chunk_step<0, false>(D, b, L.r0, C, Rs, Rd, work, info, wave, lane, tid);
}

__global__ __launch_bounds__(64) void k_getrf_trail(double *__restrict__ slab, const LevelDev *__restrict__ levels,
                                                    const int32_t *__restrict__ lvl, int k,
                                                    const ChunkDev *__restrict__ chunks,
                                                    const int32_t *__restrict__ crows) {
    const LevelDev L = levels[lvl[blockIdx.y]];
    if (L.b <= 128) return;
    const int ch = L.chunk_begin + k;
    if (ch >= L.chunk_end) return;
    const ChunkDev C = chunks[ch];
    const int nr = C.nr, w = C.w, c0 = C.c0, b = L.b;
    const int ntl = (nr + 15) >> 4;
    const int q = blockIdx.x;
    if (q >= ntl * ntl) return;
    double *__restrict__ D = slab + L.offD;
    const int32_t *__restrict__ Rs = crows + C.roff;
    const int lane = threadIdx.x, li = lane & 15, lk = lane >> 4;
    const int ti = q / ntl, tj = q - ti * ntl;
    // output element (coupled column 16 tj + lk + 4 r, coupled row 16 ti + li)
    const int ar = 16 * ti + li, sc = 16 * tj + li;
    const bool va = ar < nr, vcc = sc < nr;
    const size_t rowo = (size_t)Rs[va ? ar : nr - 1];
    const size_t colo = (size_t)Rs[vcc ? sc : nr - 1] * b;
    int cs[4];
    double4_t acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int sc2 = 16 * tj + lk + 4 * r;
        cs[r] = Rs[sc2 < nr ? sc2 : nr - 1];
        acc[r] = D[rowo + (size_t)cs[r] * b];
    }
    double al[4], bl[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int kx = 4 * kk + lk;
        const int kc = kx < w ? kx : 0;
        al[kk] = D[c0 + kc + colo];                      // U(c0 + k, Rs[sc])
        bl[kk] = D[rowo + (size_t)(c0 + kc) * b];        // L(Rs[ar], c0 + k)
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int kx = 4 * kk + lk;
        if (4 * kk < w) {
            const double a = (kx < w && vcc) ? -al[kk] : 0.0;
            const double bv = (kx < w && va) ? bl[kk] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int sc2 = 16 * tj + lk + 4 * r;
        if (va && sc2 < nr) D[rowo + (size_t)cs[r] * b] = acc[r];
    }
}

hipError_t launch_getrf_step(const DevPlan &d, const int32_t *lvl, int nlev, int k, int lds_bytes, hipStream_t s) {
    hipLaunchKernelGGL(k_getrf_step, dim3((unsigned)nlev), dim3(256), (size_t)lds_bytes, s, d.slab, d.levels, lvl, k,
                       d.chunks, d.chunk_rows, d.info);
    return hipGetLastError();
}

hipError_t launch_getrf_trail(const DevPlan &d, const int32_t *lvl, int nlev, int k, int max_tiles, hipStream_t s) {
    if (max_tiles <= 0 || nlev <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_getrf_trail, dim3((unsigned)max_tiles, (unsigned)nlev), dim3(64), 0, s, d.slab, d.levels,
                       lvl, k, d.chunks, d.chunk_rows);
    return hipGetLastError();
}

// ------------------------------------------------------------ tiled GETRF
// Pivot K of the no-pivot LU of a 16 x 16 tile in the 2D layout of lu16_2d
// (lane i + 16 g holds a[s] = A(i, 4 g + s)), which also builds the inverses
// of both factors: e (same layout, starts as I) takes the row operations of
// the elimination and ends as L^{-1}; f (starts as I) takes the column
// operations that clear U's rows right of the diagonal, col_j -= U(K, j) /
// U(K, K) col_K, which turn I into the inverse of U's unit-diagonal form;
// column K of f is final after pivot K and is divided by U(K, K) there, so f
// ends as U^{-1}.  bad: the first zero or non-finite pivot (16 if none).
template <int K>
__device__ __forceinline__ void lu16inv_step(double (&a)[4], double (&e)[4], double (&f)[4], int i, int g,
                                             int &bad) {
    constexpr int g0 = K >> 2, s0 = K & 3;
    const double piv = bcast_lane(a[s0], K + 16 * g0);
    if (!(piv != 0.0 && isfinite(piv))) bad = min(bad, K);
    const double rp = recip(piv);
    const double lg = a[s0] * rp;
    if (g == g0 && i > K) a[s0] = lg;
    const double l = perm_lane(lg, i + 16 * g0);       // L(i, K) for i > K
    const double fk = perm_lane(f[s0], i + 16 * g0);   // f(i, K)
    double u[4], ek[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        u[s] = bcast16<K>(a[s]);                       // U(K, 4 g + s)
        ek[s] = bcast16<K>(e[s]);                      // row K of L^{-1} (final)
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int j = 4 * g + s;
        const double na = a[s] - l * u[s];
        a[s] = (i > K && j > K) ? na : a[s];
        const double ne = e[s] - l * ek[s];
        e[s] = i > K ? ne : e[s];
        const double nf = f[s] - (u[s] * rp) * fk;
        f[s] = j > K ? nf : f[s];
    }
    if (g == g0) f[s0] *= rp;
    if constexpr (K + 1 < 16) lu16inv_step<K + 1>(a, e, f, i, g, bad);
}

// Right-looking LU of dense diagonal blocks in 16 x 16 tiles, one launch per
// tile step s for every level of a wave (grid.y), one wave per tile.  Launch
// s >= 1 takes the panel p = s - 1 and updates every trailing tile (I, J),
// I, J >= s:
//     Lt = A(I, p) U_pp^{-1},   Ut = L_pp^{-1} A(p, J),   A(I, J) -= Lt Ut
// (three 16 x 16 x 16 FP64 MFMA products); the inverted diagonal tiles come
// from the previous launch.  Tiles (I, s) write Lt as the final L(I, p),
// tiles (s, J) write Ut as U(p, J); the updated tiles of tile column and row
// s are the next panel and go to a panel copy (two copies, by step parity),
// so no launch reads a tile of D that it writes.  Tile (s, s) then factors
// itself (lu16inv_step) and writes its L and U into D and their inverses for
// the next launch.  Launch 0 factors tile (0, 0) and copies panel 0.  The
// panel products are the substitutions of Algorithm 1's GESSM / TSTRF steps
// inside the diagonal block, applied as products with the inverted triangles.
// Entries outside S stay exactly zero: every term reaching one has a
// structurally zero factor, and so do the inverses' entries they meet.
__global__ __launch_bounds__(64) void k_getrf_tile(double *__restrict__ slab, const LevelDev *__restrict__ levels,
                                                   const int32_t *__restrict__ lvl, int s,
                                                   double *__restrict__ work,
                                                   unsigned long long *__restrict__ info) {
    __shared__ double tl[16 * 17];
    const LevelDev L = levels[lvl[blockIdx.y]];
    const int b = L.b;
    const int nt = (b + 15) >> 4;
    if (s >= nt) return;
    const int q = blockIdx.x;
    int I, J;
    if (s == 0) {
        if (q >= 2 * nt - 1) return;
        I = q < nt ? q : 0;
        J = q < nt ? 0 : q - nt + 1;
    } else {
        const int m = nt - s;
        if (q >= m * m) return;
        I = s + q / m;
        J = s + q - (q / m) * m;
    }
    double *__restrict__ D = slab + L.offD;
    double *__restrict__ W = work + (L.offW >= 0 ? L.offW : 0);
    const int lane = threadIdx.x, li = lane & 15, g = lane >> 4;
    const int rI = 16 * I, cJ = 16 * J;
    const bool rowok = rI + li < b, colok = cJ + li < b;
    // tile (I, J) in the MFMA result layout: lane li + 16 g holds C(g + 4 r, li)
    double4_t acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = rI + g + 4 * r;
        acc[r] = (colok && row < b) ? D[(size_t)(cJ + li) * b + row] : 0.0;
    }
    if (s >= 1) {
        const int p = s - 1;
        const double *__restrict__ Pc = W + (size_t)(p & 1) * 32 * b;   // tile column p, b x 16
        const double *__restrict__ Pr = Pc + (size_t)16 * b;           // tile row p, 16 x b (column-major, ld 16)
        const double *__restrict__ iL = W + 64 * (size_t)b + (p & 1) * 512;   // row-major
        const double *__restrict__ iU = iL + 256;
        double xa[4], ya[4], xb[4], yb[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = 4 * kk + g;
            xa[kk] = iU[k * 16 + li];                              // (iU^T)(li, k)
            ya[kk] = rowok ? Pc[(size_t)k * b + rI + li] : 0.0;     // (A(I, p)^T)(k, li)
            xb[kk] = iL[li * 16 + k];                              // iL(li, k)
            yb[kk] = colok ? Pr[(size_t)(cJ + li) * 16 + k] : 0.0;  // A(p, J)(k, li)
        }
        // lt(r) = Lt^T(g + 4 r, li) = Lt(li, g + 4 r);  ut(r) = Ut(g + 4 r, li)
        double4_t lt = {0.0, 0.0, 0.0, 0.0}, ut = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            lt = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[kk], ya[kk], lt, 0, 0, 0);
            ut = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[kk], yb[kk], ut, 0, 0, 0);
        }
        // A(I, J) -= Lt Ut: Lt(li, 4 kk + g) and Ut(4 kk + g, li) are the
        // operands of step kk exactly as the two products left them
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-lt[kk], ut[kk], acc, 0, 0, 0);
        if (J == s && rowok) {
#pragma unroll
            for (int r = 0; r < 4; ++r) D[(size_t)(16 * p + g + 4 * r) * b + rI + li] = lt[r];
        }
        if (I == s && colok) {
#pragma unroll
            for (int r = 0; r < 4; ++r) D[(size_t)(cJ + li) * b + 16 * p + g + 4 * r] = ut[r];
        }
    }
    if (I != s || J != s) {
        if (J == s) {   // next panel, tile column: its copy only (launch s + 1 writes L there)
            double *__restrict__ Pc = W + (size_t)(s & 1) * 32 * b;
            if (colok) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = rI + g + 4 * r;
                    if (row < b) Pc[(size_t)li * b + row] = acc[r];
                }
            }
        } else if (I == s) {   // next panel, tile row
            double *__restrict__ Pr = W + (size_t)(s & 1) * 32 * b + (size_t)16 * b;
            if (colok) {
#pragma unroll
                for (int r = 0; r < 4; ++r) Pr[(size_t)(cJ + li) * 16 + g + 4 * r] = acc[r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rI + g + 4 * r;
                if (colok && row < b) D[(size_t)(cJ + li) * b + row] = acc[r];
            }
        }
        return;
    }
    // tile (s, s): factor it.  Rows / columns past b are an identity, so the
    // padding never yields a bad pivot.
    const int w = min(16, b - rI);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = g + 4 * r;
        double v = acc[r];
        if (row >= w || li >= w) v = row == li ? 1.0 : 0.0;
        tl[row * 17 + li] = v;
    }
    __syncthreads();
    double a[4], e[4], f[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        a[t] = tl[li * 17 + 4 * g + t];
        e[t] = li == 4 * g + t ? 1.0 : 0.0;
        f[t] = e[t];
    }
    int bad = 16;
    lu16inv_step<0>(a, e, f, li, g, bad);
    if (bad < w && lane == 0) atomicMin(info, (unsigned long long)(L.r0 + rI + bad));
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int col = 4 * g + t;
        if (li < w && col < w) D[(size_t)(rI + col) * b + rI + li] = a[t];
    }
    if (s + 1 < nt) {
        double *__restrict__ iL = W + 64 * (size_t)b + (s & 1) * 512;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            iL[li * 16 + 4 * g + t] = e[t];
            iL[256 + li * 16 + 4 * g + t] = f[t];
        }
    }
}

hipError_t launch_getrf_tile(const DevPlan &d, const int32_t *lvl, int nlev, int s, int max_nt, hipStream_t st) {
    if (nlev <= 0 || s >= max_nt) return hipSuccess;
    const int m = max_nt - s;
    const unsigned gx = s == 0 ? (unsigned)(2 * max_nt - 1) : (unsigned)(m * m);
    hipLaunchKernelGGL(k_getrf_tile, dim3(gx, (unsigned)nlev), dim3(64), 0, st, d.slab, d.levels, lvl, s, d.tgetrf,
                       d.info);
    return hipGetLastError();
}

// 16 x 16 product of two LDS operands (row-major, leading dimensions la and
// lb) by one wave, in the MFMA result layout (lane li + 16 g holds
// C(g + 4 r, li)), and its store (times sign) to a row-major LDS image.
__device__ __forceinline__ double4_t mm16_lds(const double *A, int la, const double *B, int lb, int li, int g) {
    double a[4], bb[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        a[kk] = A[li * la + 4 * kk + g];
        bb[kk] = B[(4 * kk + g) * lb + li];
    }
    double4_t c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], bb[kk], c, 0, 0, 0);
    return c;
}

__device__ __forceinline__ void st16_lds(double *C, int lc, const double4_t &c, int li, int g, double sign) {
#pragma unroll
    for (int r = 0; r < 4; ++r) C[(g + 4 * r) * lc + li] = sign * c[r];
}

// Pivot K of the no-pivot LU of a 16 x 16 block held by one wave in the
// strided layout, lane i + 16 g holding a[s] = A(i, g + 4 s): the layout in
// which an MFMA result C lands as C^T, so a product can feed the LU without
// going through LDS.  The elimination's row operations are applied to e as
// well (e starts as I and ends as L^{-1}).  With SCALE, every row of e is
// finally divided by its pivot (the lane keeps its row's pivot reciprocal in
// rrow), which gives D^{-1} L^{-1} for pivots D: run on A^T = U^T L^T, whose
// unit lower factor is U^T D^{-1}, that is (U^{-1})^T.  Only the columns
// that can change at step K are touched: a's columns right of K and e's
// columns up to K (row K of e is zero right of K).  bad: the first zero or
// non-finite pivot (16 if none).
template <int K, bool SCALE>
__device__ __forceinline__ void lu16s_step(double (&a)[4], double (&e)[4], int i, int g, int &bad,
                                           double &rrow) {
    constexpr int g0 = K & 3, s0 = K >> 2;
    const double piv = bcast_lane(a[s0], K + 16 * g0);
    if (!(piv != 0.0 && isfinite(piv))) bad = min(bad, K);
    const double rp = recip(piv);
    if constexpr (SCALE) rrow = i == K ? rp : rrow;
    const double lg = i > K ? a[s0] * rp : 0.0;          // L(i, K) in column group g0
    if (g == g0 && i > K) a[s0] = lg;
    const double l = perm_lane(lg, i + 16 * g0);        // zero on rows <= K
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (4 * s + 3 > K) {                             // columns g + 4 s > K exist
            double u = bcast16<K>(a[s]);                 // U(K, g + 4 s)
            if (s == s0) u = g > g0 ? u : 0.0;
            a[s] = a[s] - l * u;
        }
        if (4 * s <= K) {                                // columns g + 4 s <= K exist
            const double ek = bcast16<K>(e[s]);
            e[s] = e[s] - l * ek;
        }
    }
    if constexpr (K + 1 < 16) lu16s_step<K + 1, SCALE>(a, e, i, g, bad, rrow);
}

// LU of the 16 x 16 block a (strided layout) with e = L^{-1}, or, with SCALE,
// e = (U^{-1})^T of the block's transpose; returns the first bad pivot.
template <bool SCALE>
__device__ __forceinline__ int lu16s(double (&a)[4], double (&e)[4], int li, int g) {
#pragma unroll
    for (int t = 0; t < 4; ++t) e[t] = li == g + 4 * t ? 1.0 : 0.0;
    int bad = 16;
    double rrow = 1.0;
    lu16s_step<0, SCALE>(a, e, li, g, bad, rrow);
    if constexpr (SCALE) {
#pragma unroll
        for (int t = 0; t < 4; ++t) e[t] *= rrow;
    }
    return bad;
}

// The tiled GETRF of k_getrf_tile with 32 x 32 tiles and one workgroup of
// four waves per tile, wave (qi, qj) owning the 16 x 16 quadrant (qi, qj):
// launch s updates every trailing tile with the 32-column panel p = s - 1,
//     Lt = A(I, p) U_pp^{-1},   Ut = L_pp^{-1} A(p, J),   A(I, J) -= Lt Ut,
// each wave forming its quadrants of Lt and Ut (K = 32) and taking the other
// halves it needs from its neighbours through LDS.  Tile (s, s) is then
// factored as 2 x 2 blocks of 16 with the inverses of its factors:
//   waves 0, 1: LU of block 00 with L00^{-1} (wave 0), and the same
//               elimination of its transpose giving U00^{-T} (wave 1);
//               U01 = L00^{-1} A01, L10 = A10 U00^{-1};
//   waves 2, 3: A11 - L10 U01, formed by each in the layout its LU needs,
//               LU with L11^{-1} (wave 2) and U11^{-T} (wave 3); meanwhile
//               waves 0, 1 form U00^{-1} U01 and L10 L00^{-1};
//   waves 2, 3: U^{-1}_01 = -U00^{-1} U01 U11^{-1}, L^{-1}_10 = -L11^{-1} L10 L00^{-1}.
// Every result goes to global memory from the registers that hold it.  With
// ONE the wave has a single level, whose fields the kernel needs are its
// first arguments (b1, r01, offD1, offW1: preloaded into scalar registers at
// launch, no load before the first address is known).
// Panel copies and inverses live in the level's work region: two copies of
// 64 b doubles by step parity (tile column b x 32 row-major, tile row 32 x b
// column-major), then the 32 x 32 inverses of L (row-major) and U
// (column-major) of every diagonal tile (kept for the solves): every operand
// of the panel products is then contiguous in the inner index.
constexpr int kT32Ld = 33;

template <bool ONE>
__global__ __launch_bounds__(256) void k_getrf_tile32(int s, int b1, int r01, int64_t offD1, int64_t offW1,
                                                      double *__restrict__ slab, double *__restrict__ work,
                                                      unsigned long long *__restrict__ info,
                                                      const LevelDev *__restrict__ levels,
                                                      const int32_t *__restrict__ lvl) {
    __builtin_amdgcn_s_setprio(3);   // issue ahead of co-resident deferred Schur-update waves
    __shared__ double xch[2][4][4][64];   // [lt / ut][wave][r][lane]
    __shared__ double T[32 * kT32Ld];
    __shared__ double IL0[16 * 17], IU0[16 * 17], S1[16 * 17], S2[16 * 17];
    int b, r0;
    int64_t offD, offW;
    if constexpr (ONE) {
        b = b1;
        r0 = r01;
        offD = offD1;
        offW = offW1;
    } else {
        const LevelDev &L = levels[lvl[blockIdx.y]];
        b = L.b;
        r0 = L.r0;
        offD = L.offD;
        offW = L.offW;
    }
    const int nt = (b + 31) >> 5;
    if (s >= nt) return;
    const int q = blockIdx.x;
    int I, J;
    if (s == 0) {
        if (q >= 2 * nt - 1) return;
        I = q < nt ? q : 0;
        J = q < nt ? 0 : q - nt + 1;
    } else {
        const int m = nt - s;
        if (q >= m * m) return;
        I = s + q / m;
        J = s + q - (q / m) * m;
    }
    double *__restrict__ D = slab + offD;
    double *__restrict__ W = work + (offW >= 0 ? offW : 0);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
    const int qi = wave >> 1, qj = wave & 1;
    const int rI = 32 * I, cJ = 32 * J;
    const int row0 = rI + 16 * qi, col0 = cJ + 16 * qj;
    const bool colok = col0 + li < b;
    const size_t colc = (size_t)min(col0 + li, b - 1);
    // every load below is issued unconditionally from a clamped address, so
    // that they all go out together: rows and columns past b hold copies of
    // in-range values, are never stored and never reach an in-range entry
    // (the diagonal tile replaces them by the identity)
    double4_t acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = D[colc * b + min(row0 + g + 4 * r, b - 1)];
    if (s >= 1) {
        const int p = s - 1;
        const double *__restrict__ Pc = W + (size_t)(p & 1) * 64 * b;   // tile column p, b x 32 (ld 32)
        const double *__restrict__ Pr = Pc + (size_t)32 * b;           // tile row p, 32 x b (ld 32)
        const double *__restrict__ iLg = W + 128 * (size_t)b + (size_t)p * 2048;   // row-major
        const double *__restrict__ iUg = iLg + 1024;                               // column-major
        const int rowq = row0 + li;
        const bool rowok = rowq < b;
        const int rowc = min(rowq, b - 1);
        // product step kk takes the inner index k = 8 g + kk in lane group g
        // (the same for both operands), eight consecutive doubles per lane
        double4_t lt = {0.0, 0.0, 0.0, 0.0}, ut = {0.0, 0.0, 0.0, 0.0};
        double xa[8], ya[8], xb[8], yb[8];
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            const int k = 8 * g + kk;
            xa[kk] = iUg[(16 * qj + li) * 32 + k];                         // iU(k, 16 qj + li)
            ya[kk] = Pc[(size_t)rowc * 32 + k];                            // A(I, p)(16 qi + li, k)
            xb[kk] = iLg[(16 * qi + li) * 32 + k];                         // iL(16 qi + li, k)
            yb[kk] = Pr[colc * 32 + k];                                    // A(p, J)(k, 16 qj + li)
        }
        // lt(r) = Lt(16 qi + li, 16 qj + g + 4 r); ut(r) = Ut(16 qi + g + 4 r, 16 qj + li)
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            lt = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[kk], ya[kk], lt, 0, 0, 0);
            ut = __builtin_amdgcn_mfma_f64_16x16x4f64(xb[kk], yb[kk], ut, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            xch[0][wave][r][lane] = lt[r];
            xch[1][wave][r][lane] = ut[r];
        }
        __syncthreads();
        // quadrant (qi, qj) -= Lt(qi, h) Ut(h, qj), h = 0, 1 (waves 2 qi + h
        // and 2 h + qj hold them, in operand layout)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int wl = 2 * qi + h, wu = 2 * h + qj;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-xch[0][wl][kk][lane], xch[1][wu][kk][lane], acc, 0, 0,
                                                           0);
        }
        if (J == s && rowok) {
#pragma unroll
            for (int r = 0; r < 4; ++r) D[(size_t)(32 * p + 16 * qj + g + 4 * r) * b + rowq] = lt[r];
        }
        if (I == s && colok) {
#pragma unroll
            for (int r = 0; r < 4; ++r) D[(size_t)(col0 + li) * b + 32 * p + 16 * qi + g + 4 * r] = ut[r];
        }
    }
    if (I != s || J != s) {
        if (J == s) {   // next panel, tile column: its copy only
            double *__restrict__ Pc = W + (size_t)(s & 1) * 64 * b;
            if (colok) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = row0 + g + 4 * r;
                    if (row < b) Pc[(size_t)row * 32 + 16 * qj + li] = acc[r];
                }
            }
        } else if (I == s) {   // next panel, tile row
            double *__restrict__ Pr = W + (size_t)(s & 1) * 64 * b + (size_t)32 * b;
            if (colok) {
#pragma unroll
                for (int r = 0; r < 4; ++r) Pr[(size_t)(col0 + li) * 32 + 16 * qi + g + 4 * r] = acc[r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = row0 + g + 4 * r;
                if (colok && row < b) D[(size_t)(col0 + li) * b + row] = acc[r];
            }
        }
        return;
    }
    // tile (s, s): rows / columns past b are an identity
    const int w = min(32, b - rI);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * qi + g + 4 * r, col = 16 * qj + li;
        double v = acc[r];
        if (row >= w || col >= w) v = row == col ? 1.0 : 0.0;
        T[row * kT32Ld + col] = v;
    }
    __syncthreads();
    const bool keep = offW >= 0;
    double *__restrict__ iLw = W + 128 * (size_t)b + (size_t)s * 2048;   // row-major 32 x 32
    double *__restrict__ iUw = iLw + 1024;                               // column-major 32 x 32
    double *__restrict__ Dt = D + (size_t)rI * b + rI;                   // the tile, column-major, ld b
    double a[4], e[4];
    if (wave == 0) {
        // block 00: LU and L00^{-1}; U01 = L00^{-1} A01
#pragma unroll
        for (int t = 0; t < 4; ++t) a[t] = T[li * kT32Ld + g + 4 * t];
        const int bad = lu16s<false>(a, e, li, g);
        if (lane == 0 && bad < min(16, w)) atomicMin(info, (unsigned long long)(r0 + rI + bad));
        double4_t c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            c = __builtin_amdgcn_mfma_f64_16x16x4f64(e[kk], T[(g + 4 * kk) * kT32Ld + 16 + li], c, 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int col = g + 4 * t;
            IL0[li * 17 + col] = e[t];
            if (li < w && col < w) Dt[(size_t)col * b + li] = a[t];
            if (keep) {
                iLw[li * 32 + col] = e[t];
                iLw[(g + 4 * t) * 32 + 16 + li] = 0.0;                      // L^{-1}_01
            }
        }
        st16_lds(T + 16, kT32Ld, c, li, g, 1.0);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (g + 4 * r < w && 16 + li < w) Dt[(size_t)(16 + li) * b + g + 4 * r] = c[r];
    } else if (wave == 1) {
        // block 00 transposed: U00^{-T}; L10 = A10 U00^{-1}
#pragma unroll
        for (int t = 0; t < 4; ++t) a[t] = T[(g + 4 * t) * kT32Ld + li];
        (void)lu16s<true>(a, e, li, g);                                     // e(li, g + 4 t) = U00^{-1}(g + 4 t, li)
        double4_t c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
            c = __builtin_amdgcn_mfma_f64_16x16x4f64(T[(16 + li) * kT32Ld + g + 4 * kk], e[kk], c, 0, 0, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            IU0[(g + 4 * t) * 17 + li] = e[t];
            if (keep) {
                iUw[li * 32 + g + 4 * t] = e[t];
                iUw[li * 32 + 16 + g + 4 * t] = 0.0;                        // U^{-1}_10
            }
        }
        st16_lds(T + 16 * kT32Ld, kT32Ld, c, li, g, 1.0);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (16 + g + 4 * r < w && li < w) Dt[(size_t)li * b + 16 + g + 4 * r] = c[r];
    }
    __syncthreads();
    if (wave >= 2) {
        // A11 - L10 U01: wave 2 forms its transpose (the strided layout of
        // the block), wave 3 the block itself (the strided layout of its
        // transpose)
        const bool tr = wave == 2;
        double4_t c;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            c[r] = tr ? T[(16 + li) * kT32Ld + 16 + g + 4 * r] : T[(16 + g + 4 * r) * kT32Ld + 16 + li];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const double u01 = T[(g + 4 * kk) * kT32Ld + 16 + li];         // U01(g + 4 kk, li)
            const double l10 = T[(16 + li) * kT32Ld + g + 4 * kk];         // L10(li, g + 4 kk)
            c = __builtin_amdgcn_mfma_f64_16x16x4f64(tr ? -u01 : -l10, tr ? l10 : u01, c, 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) a[t] = c[t];
        if (tr) {
            const int bad = lu16s<false>(a, e, li, g);
            if (lane == 0 && bad < w - 16) atomicMin(info, (unsigned long long)(r0 + rI + 16 + bad));
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int col = 16 + g + 4 * t;
                if (16 + li < w && col < w) Dt[(size_t)col * b + 16 + li] = a[t];
                if (keep) iLw[(16 + li) * 32 + col] = e[t];
            }
        } else {
            (void)lu16s<true>(a, e, li, g);
            if (keep) {
#pragma unroll
                for (int t = 0; t < 4; ++t) iUw[(16 + li) * 32 + 16 + g + 4 * t] = e[t];
            }
        }
    } else if (wave == 0) {   // U00^{-1} U01
        const double4_t c = mm16_lds(IU0, 17, T + 16, kT32Ld, li, g);
        st16_lds(S1, 17, c, li, g, 1.0);
    } else {                  // L10 L00^{-1}
        const double4_t c = mm16_lds(T + 16 * kT32Ld, kT32Ld, IL0, 17, li, g);
        st16_lds(S2, 17, c, li, g, 1.0);
    }
    __syncthreads();
    if (wave >= 2 && keep) {
        double4_t c = {0.0, 0.0, 0.0, 0.0};
        if (wave == 2) {      // L^{-1}_10 = -L11^{-1} (L10 L00^{-1})
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                c = __builtin_amdgcn_mfma_f64_16x16x4f64(e[kk], S2[(g + 4 * kk) * 17 + li], c, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) iLw[(16 + g + 4 * r) * 32 + li] = -c[r];
        } else {              // U^{-1}_01 = -(U00^{-1} U01) U11^{-1}
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                c = __builtin_amdgcn_mfma_f64_16x16x4f64(S1[li * 17 + g + 4 * kk], e[kk], c, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) iUw[(16 + li) * 32 + g + 4 * r] = -c[r];
        }
    }
}

hipError_t launch_getrf_tile32(const DevPlan &d, const int32_t *lvl, int nlev, int s, int max_nt,
                               const LevelDev *one, hipStream_t st) {
    if (nlev <= 0 || s >= max_nt) return hipSuccess;
    const int m = max_nt - s;
    const unsigned gx = s == 0 ? (unsigned)(2 * max_nt - 1) : (unsigned)(m * m);
    if (nlev == 1 && one)
        hipLaunchKernelGGL(k_getrf_tile32<true>, dim3(gx, 1), dim3(256), 0, st, s, one->b, one->r0, one->offD,
                           one->offW, d.slab, d.tgetrf, d.info, d.levels, lvl);
    else
        hipLaunchKernelGGL(k_getrf_tile32<false>, dim3(gx, (unsigned)nlev), dim3(256), 0, st, s, 0, 0, (int64_t)0,
                           (int64_t)0, d.slab, d.tgetrf, d.info, d.levels, lvl);
    return hipGetLastError();
}

// ------------------------------------------- compact coupled triangles
// One workgroup per 16 x 16 tile that the panel solves read, numbered over
// the wave's levels (soff: first workgroup of each level): per level the nt
// diagonal tiles, then the structurally nonzero tiles of its tile rows
// (trow).  A thread copies one element of Tu = U_ii[K, K] and one of
// Tl = L_ii[K, K]^T from the factored diagonal block; a diagonal tile's
// workgroup then inverts its two triangles (back substitution per column,
// FP64 divisions by the pivots).  Tiles outside these lists are never
// written and never read.
__global__ __launch_bounds__(256) void k_tri_gather(const double *__restrict__ slab, double *__restrict__ tri,
                                                    const LevelDev *__restrict__ levels,
                                                    const int32_t *__restrict__ lvl,
                                                    const int32_t *__restrict__ soff, int nlev,
                                                    const int32_t *__restrict__ Kidx,
                                                    const int32_t *__restrict__ trow_ptr,
                                                    const int32_t *__restrict__ trow_idx) {
    __builtin_amdgcn_s_setprio(3);   // issue ahead of co-resident deferred Schur-update waves
    __shared__ double du[16][17], dl[16][17];
    // the level of this workgroup: the last one whose first slot is <= it
    const int bid = blockIdx.x;
    int lo = 0, hi = nlev - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (soff[mid] <= bid) lo = mid; else hi = mid - 1;
    }
    const LevelDev L = levels[lvl[lo]];
    const int kp = L.kp, kap = L.kappa, b = L.b, nt = kp >> 4;
    const int32_t *__restrict__ tptr = trow_ptr + L.trow;
    const int slot = bid - soff[lo];
    if (nt == 0) return;
    const int tb = tptr[0];
    if (slot >= nt + (tptr[nt] - tb)) return;
    int tr, tc;
    if (slot < nt) {
        tr = tc = slot;
    } else {
        // tile row of off-diagonal tile e: the last row r with tptr[r] - tb <= e
        const int e = slot - nt;
        tc = trow_idx[tb + e];
        int rlo = 0, rhi = nt - 1;
        while (rlo < rhi) {
            const int mid = (rlo + rhi + 1) >> 1;
            if (tptr[mid] - tb <= e) rlo = mid; else rhi = mid - 1;
        }
        tr = rlo;
    }
    const double *__restrict__ D = slab + L.offD;
    const int32_t *__restrict__ K = Kidx + L.Koff;
    double *__restrict__ Tu = tri + L.offT;
    double *__restrict__ Tl = Tu + (size_t)kp * kp;
    double *__restrict__ Iu = Tl + (size_t)kp * kp;
    double *__restrict__ Il = Iu + (size_t)nt * 256;
    const int rr = threadIdx.x >> 4, cc = threadIdx.x & 15;
    const int t1 = 16 * tr + rr, t2 = 16 * tc + cc;
    const bool in = t1 < kap && t2 < kap;
    const size_t k1 = in ? (size_t)K[t1] : 0, k2 = in ? (size_t)K[t2] : 0;
    double uu = (in && t1 <= t2) ? D[k1 + k2 * b] : 0.0;
    double ll = (in && t1 < t2) ? D[k2 + k1 * b] : 0.0;
    if (t1 == t2) {
        ll = 1.0;
        if (!in) uu = 1.0;
    }
    Tu[(size_t)t1 * kp + t2] = uu;
    Tl[(size_t)t1 * kp + t2] = ll;
    if (slot >= nt) return;
    du[rr][cc] = uu;
    dl[rr][cc] = ll;
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

hipError_t launch_tri_gather_wave(const DevPlan &d, const int32_t *lvl, const int32_t *soff, int nlev, int slots,
                                  hipStream_t s) {
    if (slots <= 0 || nlev <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tri_gather, dim3((unsigned)slots), dim3(256), 0, s, d.slab, d.tri, d.levels, lvl, soff, nlev,
                       d.K_idx, d.trow_ptr, d.trow_idx);
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
                                                     const int32_t *__restrict__ trow_idx, int skip_blocked) {
    __builtin_amdgcn_s_setprio(3);   // issue ahead of co-resident deferred Schur-update waves
    extern __shared__ double xs_lds[];
    const LevelDev L = levels[lvl[blockIdx.z]];
    const int kp = L.kp, kap = L.kappa, m = L.m, nt = kp >> 4;
    if (kp == 0 || (int)blockIdx.x * RT >= m || (skip_blocked && L.offB >= 0)) return;
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

// Variant for waves of few levels (same results): the level's tile lists
// are staged in LDS after the rows, the triangle operands of a step (the
// inverted diagonal tile and the wave's first kPanelPf update tiles) are
// loaded one step ahead, so their latency overlaps the previous step, and
// the update tiles are taken two at a time.
constexpr int kPanelPf = 6;   // even: the tiles are taken two at a time

size_t panel_tables_bytes(int max_kp) {
    const size_t ntm = (size_t)(max_kp >> 4);
    return (ntm + 1 + ntm * (ntm + 1) / 2) * sizeof(int32_t);
}

template <int RT, bool IN_LDS>
__global__ __launch_bounds__(256) void k_panel_solve_pf(double *__restrict__ slab, const double *__restrict__ tri,
                                                     const LevelDev *__restrict__ levels,
                                                     const int32_t *__restrict__ lvl,
                                                     const int32_t *__restrict__ trow_ptr,
                                                     const int32_t *__restrict__ trow_idx, int skip_blocked) {
    __builtin_amdgcn_s_setprio(3);   // issue ahead of co-resident deferred Schur-update waves
    extern __shared__ double xs_lds[];
    const LevelDev L = levels[lvl[blockIdx.z]];
    const int kp = L.kp, kap = L.kappa, m = L.m, nt = kp >> 4;
    if (kp == 0 || (int)blockIdx.x * RT >= m || (skip_blocked && L.offB >= 0)) return;
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
    }
    // tile lists: SP(0..nt) row pointers (rebased), SX() tile columns,
    // staged in LDS after the rows (read from global memory when the rows
    // themselves do not fit in LDS)
    int *sp = (int *)(xs_lds + (IN_LDS ? (size_t)kp * LD : 0));
    const int tb = tptr[0];
    const int ntile = tptr[nt] - tb;
    int *sx = sp + nt + 1;
    if (IN_LDS) {
        for (int e = tid; e <= nt; e += 256) sp[e] = tptr[e] - tb;
        for (int e = tid; e < ntile; e += 256) sx[e] = trow_idx[tb + e];
    }
    __syncthreads();
    auto SP = [&](int e) -> int { return IN_LDS ? sp[e] : tptr[e] - tb; };
    auto SX = [&](int e) -> int { return IN_LDS ? sx[e] : trow_idx[tb + e]; };
    // operands of step c: the diagonal inverse and the wave's update tiles
    // q = wave + 4 i (i < kPanelPf); every load is issued, from a clamped
    // valid address, so the wait counts stay exact
    double tbn[4], ubn[kPanelPf][4];
    auto fetch = [&](int c) {
        const int cq = c < nt ? c : nt - 1;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) tbn[kk] = Tinv[(size_t)cq * 256 + (4 * kk + lk) * 16 + li];
        const int q0 = SP(cq), ntq = (SP(cq + 1) - q0) * NH;
#pragma unroll
        for (int i = 0; i < kPanelPf; ++i) {
            const int q = wave + 4 * i;
            const int cc = ntq > 0 ? SX(q0 + (q < ntq ? q : ntq - 1) / NH) : cq;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) ubn[i][kk] = T[(size_t)(16 * cq + 4 * kk + lk) * kp + 16 * cc + li];
        }
    };
    fetch(0);
    for (int c = 0; c < nt; ++c) {
        double tbc[4], ubc[kPanelPf][4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) tbc[kk] = tbn[kk];
#pragma unroll
        for (int i = 0; i < kPanelPf; ++i)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) ubc[i][kk] = ubn[i][kk];
        fetch(c + 1);
        // diagonal tile of the wave's own 16 rows (read and written by this
        // wave only, so no barrier between the product and its store)
        if (wave < NH) {
            double4_t acc = {0, 0, 0, 0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int k = 4 * kk + lk;
                const double a = ld_x(16 * c + k, 16 * wave + li);
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, tbc[kk], acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) st_x(16 * c + li, 16 * wave + lk + 4 * r, acc[r]);
        }
        __syncthreads();
        const int q0 = SP(c), ntq = (SP(c + 1) - q0) * NH;
        // two update tiles of the wave at a time (distinct columns cc), so
        // their MFMA chains interleave; without a second tile the first is
        // computed twice and stored once
        auto update2 = [&](int qa, const double (&bva)[4], int qb, const double (&bvb)[4], bool hasb) {
            const int qs[2] = {qa, hasb ? qb : qa};
            int cc[2], hh[2];
            double4_t u[2];
            double a[2][4];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                cc[t] = SX(q0 + qs[t] / NH);
                hh[t] = qs[t] % NH;
#pragma unroll
                for (int r = 0; r < 4; ++r) u[t][r] = ld_x(16 * cc[t] + li, 16 * hh[t] + lk + 4 * r);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) a[t][kk] = -ld_x(16 * c + 4 * kk + lk, 16 * hh[t] + li);
            }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                u[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0][kk], bva[kk], u[0], 0, 0, 0);
                u[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1][kk], bvb[kk], u[1], 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) st_x(16 * cc[0] + li, 16 * hh[0] + lk + 4 * r, u[0][r]);
            if (hasb) {
#pragma unroll
                for (int r = 0; r < 4; ++r) st_x(16 * cc[1] + li, 16 * hh[1] + lk + 4 * r, u[1][r]);
            }
        };
#pragma unroll
        for (int i = 0; i < kPanelPf; i += 2) {
            const int q = wave + 4 * i;
            if (q < ntq) update2(q, ubc[i], q + 4, ubc[i + 1], q + 4 < ntq);
        }
        for (int q = wave + 4 * kPanelPf; q < ntq; q += 8) {
            const bool hasb = q + 4 < ntq;
            const int cca = SX(q0 + q / NH), ccb = SX(q0 + (hasb ? q + 4 : q) / NH);
            double bva[4], bvb[4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                bva[kk] = T[(size_t)(16 * c + 4 * kk + lk) * kp + 16 * cca + li];
                bvb[kk] = T[(size_t)(16 * c + 4 * kk + lk) * kp + 16 * ccb + li];
            }
            update2(q, bva, q + 4, bvb, hasb);
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

// ------------------------------------------------- blocked panel solves
// For levels with wide coupled triangles (kp >= kPanelBlkKp) the panel solves
// X <- X T^{-1} (X = P_i with T = Tu, X = Qt_i with T = Tl, both upper) run
// in column blocks of kPanelBlk = 128 across the whole GPU:
//   k_tri_binv: the inverse of every 128 x 128 diagonal block of T, one wave
//     per 16-column tile j of a block: X_jj is the inverted 16 x 16 tile,
//     X_ij = -T_ii^{-1} sum_{k = i+1..j} T_ik X_kj for i = j-1 .. 0;
//   k_panel_blk, one launch per block step J: every workgroup takes 32 panel
//     rows and one column block C > J and subtracts X(:, J) T(J, C) (the
//     right-looking update with the solved block J); the workgroups of block
//     C = J + 1 then multiply their rows by T_CC^{-1}, which solves block
//     J + 1.  Launch J = -1 solves block 0.  No launch writes a block that
//     another of its workgroups reads.
// Every product is an FP64 MFMA 16 x 16 x 4 chain; the same X T^{-1} as the
// tile-by-tile solve, with the substitutions grouped into block inverses.
__global__ __launch_bounds__(64, 4) void k_tri_binv(const double *__restrict__ tri, double *__restrict__ binv,
                                                 const LevelDev *__restrict__ levels,
                                                 const int32_t *__restrict__ lvl) {
    __builtin_amdgcn_s_setprio(3);   // issue ahead of co-resident deferred Schur-update waves
    const LevelDev L = levels[lvl[blockIdx.y]];
    if (L.offB < 0) return;
    const int kp = L.kp, nt = kp >> 4, nbk = (kp + kPanelBlk - 1) / kPanelBlk;
    const int jb = blockIdx.x >> 3, j = blockIdx.x & 7;
    if (jb >= nbk) return;
    const int t0 = jb * 8, nbt = min(8, nt - t0);
    if (j >= nbt) return;
    const int panel = blockIdx.z;
    const double *__restrict__ T = tri + L.offT + (size_t)panel * kp * kp;
    const double *__restrict__ Iv = tri + L.offT + 2 * (size_t)kp * kp + (size_t)panel * nt * 256;
    double *__restrict__ out = binv + L.offB + ((size_t)panel * nbk + jb) * kPanelBlk * kPanelBlk;
    const int lane = threadIdx.x, li = lane & 15, g = lane >> 4;
    // X[k] = tile (k, j) of the block inverse in the MFMA result layout,
    // which is also the B-operand layout of a product with it
    double4_t X[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) X[k] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (k == j) {
#pragma unroll
            for (int r = 0; r < 4; ++r) X[k][r] = Iv[(size_t)(t0 + k) * 256 + (g + 4 * r) * 16 + li];
        }
#pragma unroll
    for (int i = 7; i >= 0; --i) {
        if (i >= j) continue;
        double4_t S = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (k <= i || k > j) continue;
            double a[4];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                a[kk] = T[(size_t)(16 * (t0 + i) + li) * kp + 16 * (t0 + k) + 4 * kk + g];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) S = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], X[k][kk], S, 0, 0, 0);
        }
        double a[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) a[kk] = -Iv[(size_t)(t0 + i) * 256 + li * 16 + 4 * kk + g];
        double4_t Y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) Y = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk], S[kk], Y, 0, 0, 0);
        X[i] = Y;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (k >= nbt) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            out[(size_t)(16 * k + g + 4 * r) * kPanelBlk + 16 * j + li] = k <= j ? X[k][r] : 0.0;
    }
}

__global__ __launch_bounds__(256, 4) void k_panel_blk(double *__restrict__ slab, const double *__restrict__ tri,
                                                   const double *__restrict__ binv,
                                                   const LevelDev *__restrict__ levels,
                                                   const int32_t *__restrict__ lvl, int J, int rtiles_max) {
    __builtin_amdgcn_s_setprio(3);   // issue ahead of co-resident deferred Schur-update waves
    __shared__ double xs[32 * (kPanelBlk + 1)];
    const LevelDev L = levels[lvl[blockIdx.y]];
    if (L.offB < 0) return;
    const int kp = L.kp, m = L.m, nbk = (kp + kPanelBlk - 1) / kPanelBlk;
    const int rt = blockIdx.x % rtiles_max, cb = blockIdx.x / rtiles_max;
    const int C = J + 1 + cb;
    if (32 * rt >= m || C >= nbk) return;
    const int panel = blockIdx.z;
    double *__restrict__ X = slab + (panel == 0 ? L.offP : L.offQ);
    const double *__restrict__ T = tri + L.offT + (size_t)panel * kp * kp;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
    const int r0 = 32 * rt, c0 = kPanelBlk * C, wb = min(kPanelBlk, kp - c0);
    // the wave's output: rows r0 + 16 h + (g + 4 r), columns cw + 16 t + li
    const int cw = c0 + 32 * wave;
    const bool wact = 32 * wave < wb;
    double4_t acc[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int col = cw + 16 * t + li;
            const bool cok = wact && col < c0 + wb;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + 16 * h + g + 4 * r;
                acc[h][t][r] = (cok && row < m) ? X[(size_t)col * m + row] : 0.0;
            }
        }
    if (J >= 0 && wact) {
        // K = 128 in eight batches of four 4-deep steps; the loads of the
        // next batch are in flight while the current one's MFMAs run (short
        // batches keep the registers low enough for three waves per SIMD,
        // whose interleaving hides more latency than a deeper prefetch)
        const int k0 = kPanelBlk * J;
        const bool rok0 = r0 + li < m, rok1 = r0 + 16 + li < m;
        const bool cok0 = cw + li < c0 + wb, cok1 = cw + 16 + li < c0 + wb;
        constexpr int KB = 4, NB = kPanelBlk / 4 / KB;
        double ca[2][KB][2], cbv[2][KB][2];
        auto fetch = [&](int nb, double (&a)[KB][2], double (&bv)[KB][2]) {
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                const int k = k0 + 4 * (nb * KB + u) + g;
                a[u][0] = rok0 ? X[(size_t)k * m + r0 + li] : 0.0;
                a[u][1] = rok1 ? X[(size_t)k * m + r0 + 16 + li] : 0.0;
                bv[u][0] = cok0 ? T[(size_t)k * kp + cw + li] : 0.0;
                bv[u][1] = cok1 ? T[(size_t)k * kp + cw + 16 + li] : 0.0;
            }
        };
        fetch(0, ca[0], cbv[0]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            if (nb + 1 < NB) fetch(nb + 1, ca[(nb + 1) & 1], cbv[(nb + 1) & 1]);
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                const double a0 = ca[nb & 1][u][0], a1 = ca[nb & 1][u][1];
                const double b0 = cbv[nb & 1][u][0], b1 = cbv[nb & 1][u][1];
                acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a1, b1, acc[1][1], 0, 0, 0);
            }
        }
    }
    if (cb == 0) {
        // block C = J + 1 is now final up to its own triangle: times T_CC^{-1}
        constexpr int LD = kPanelBlk + 1;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) xs[(16 * h + g + 4 * r) * LD + 32 * wave + 16 * t + li] = acc[h][t][r];
        __syncthreads();
        const double *__restrict__ Bi = binv + L.offB + ((size_t)panel * nbk + C) * kPanelBlk * kPanelBlk;
        double4_t out[2][2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int t = 0; t < 2; ++t) out[h][t] = double4_t{0.0, 0.0, 0.0, 0.0};
        if (wact) {
            // wb / 4 steps (a multiple of 4) in batches of four, the inverse's
            // loads of the next batch in flight during the current MFMAs
            const int nk = wb >> 2;
            const bool bo0 = 32 * wave + li < wb, bo1 = 32 * wave + 16 + li < wb;
            double bq[2][4][2];
            auto fetchb = [&](int kb, double (&bv)[4][2]) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int k = 4 * (4 * kb + u) + g;
                    bv[u][0] = bo0 ? Bi[(size_t)k * kPanelBlk + 32 * wave + li] : 0.0;
                    bv[u][1] = bo1 ? Bi[(size_t)k * kPanelBlk + 32 * wave + 16 + li] : 0.0;
                }
            };
            const int nkb = nk >> 2;
            fetchb(0, bq[0]);
            for (int kb = 0; kb < nkb; ++kb) {
                if (kb + 1 < nkb) fetchb(kb + 1, bq[(kb + 1) & 1]);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int k = 4 * (4 * kb + u) + g;
                    const double a0 = xs[li * LD + k], a1 = xs[(16 + li) * LD + k];
                    const double b0 = bq[kb & 1][u][0], b1 = bq[kb & 1][u][1];
                    out[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, out[0][0], 0, 0, 0);
                    out[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, out[0][1], 0, 0, 0);
                    out[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, out[1][0], 0, 0, 0);
                    out[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, out[1][1], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int t = 0; t < 2; ++t) acc[h][t] = out[h][t];
    }
    if (!wact) return;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int col = cw + 16 * t + li;
            if (col >= c0 + wb) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + 16 * h + g + 4 * r;
                if (row < m) X[(size_t)col * m + row] = acc[h][t][r];
            }
        }
}

hipError_t launch_panel_blk_wave(const DevPlan &d, const int32_t *lvl, int nlev, int max_m, int max_kp,
                                 hipStream_t s) {
    if (nlev <= 0 || max_m <= 0 || max_kp < kPanelBlkKp) return hipSuccess;
    const int nbk = (max_kp + kPanelBlk - 1) / kPanelBlk;
    hipLaunchKernelGGL(k_tri_binv, dim3((unsigned)(8 * nbk), (unsigned)nlev, 2), dim3(64), 0, s, d.tri, d.binv,
                       d.levels, lvl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int rt = (max_m + 31) / 32;
    for (int J = -1; J + 1 < nbk; ++J) {
        const int ncb = J < 0 ? 1 : nbk - (J + 1);
        hipLaunchKernelGGL(k_panel_blk, dim3((unsigned)(rt * ncb), (unsigned)nlev, 2), dim3(256), 0, s, d.slab,
                           d.tri, d.binv, d.levels, lvl, J, rt);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Waves of at most kPanelPfLevels levels take the prefetching variant; waves
// of many small levels (batches) the plain one, whose workgroups are
// lighter (measured: 26 us against 60 us per launch on such waves).
constexpr int kPanelPfLevels = 8;

hipError_t launch_panel_solve_wave(const DevPlan &d, const int32_t *lvl, int nlev, int max_m, int max_kp,
                                   int skip_blocked, hipStream_t s) {
    if (max_m <= 0 || max_kp <= 0) return hipSuccess;
    if (nlev <= kPanelPfLevels) {
        const size_t tab = panel_tables_bytes(max_kp);
        const size_t lds32 = (size_t)33 * max_kp * sizeof(double) + tab;
        const size_t lds16 = (size_t)17 * max_kp * sizeof(double) + tab;
        if (lds32 <= 150 * 1024) {
            dim3 grid((unsigned)((max_m + 31) / 32), 2, (unsigned)nlev);
            hipLaunchKernelGGL((k_panel_solve_pf<32, true>), grid, dim3(256), lds32, s, d.slab, d.tri, d.levels, lvl,
                               d.trow_ptr, d.trow_idx, skip_blocked);
            return hipGetLastError();
        }
        if (lds16 <= 150 * 1024) {
            dim3 grid((unsigned)((max_m + 15) / 16), 2, (unsigned)nlev);
            hipLaunchKernelGGL((k_panel_solve_pf<16, true>), grid, dim3(256), lds16, s, d.slab, d.tri, d.levels, lvl,
                               d.trow_ptr, d.trow_idx, skip_blocked);
            return hipGetLastError();
        }
    }
    const size_t lds32 = (size_t)33 * max_kp * sizeof(double), lds16 = (size_t)17 * max_kp * sizeof(double);
    if (lds32 <= 150 * 1024) {
        dim3 grid((unsigned)((max_m + 31) / 32), 2, (unsigned)nlev);
        hipLaunchKernelGGL((k_panel_solve<32, true>), grid, dim3(256), lds32, s, d.slab, d.tri, d.levels, lvl,
                           d.trow_ptr, d.trow_idx, skip_blocked);
    } else if (lds16 <= 150 * 1024) {
        dim3 grid((unsigned)((max_m + 15) / 16), 2, (unsigned)nlev);
        hipLaunchKernelGGL((k_panel_solve<16, true>), grid, dim3(256), lds16, s, d.slab, d.tri, d.levels, lvl,
                           d.trow_ptr, d.trow_idx, skip_blocked);
    } else {
        dim3 grid((unsigned)((max_m + 15) / 16), 2, (unsigned)nlev);
        hipLaunchKernelGGL((k_panel_solve<16, false>), grid, dim3(256), 0, s, d.slab, d.tri, d.levels, lvl,
                           d.trow_ptr, d.trow_idx, skip_blocked);
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

//
// F32: the product is formed in FP32 (operands rounded to FP32 when staged,
// v_mfma_f32_16x16x4f32 with FP32 accumulation, whose result element r of
// lane l is D[4 * (l / 16) + r][l % 16], probed on gfx950); the target is
// updated in FP64.  This is the FP32 factorization mode: the Schur updates,
// which hold nearly all of the flops, run at the FP32 MFMA rate.
//
// One launch covers a round: levels of a wave with disjoint targets; the
// workgroup finds its level by binary search over the levels' first tiles.
// TT = 64: 256 threads, four waves of 32 x 32; TT = 32: one wave of 32 x 32
// (rounds of small levels, for more workgroups).  Workgroups are dealt to
// the eight XCDs in turn, so the tile number is remapped to give each XCD a
// contiguous run of row-major tiles: its share of P_i stays in its L2.
// mode selects the tiles of each level: all (0); those in its first sscrit
// tile rows or columns, which hold every target of the next wave's blocks
// (1: tile rows 0 .. sscrit - 1 whole, then the first sscrit columns of the
// later rows); the others (2: the square of later rows and columns); of
// mode 1, the square of the first sscrit rows and columns, which holds the
// next wave's diagonal blocks (3), and the two bands beside it, which hold
// its panels (4: rows 0 .. sscrit - 1 times the later columns, then the later
// rows times the first sscrit columns).  The
// 64 x 64 tiles are compiled for four resident workgroups per CU (110
// registers, no spills; LDS allows four): 13 % faster than the three that
// the unconstrained allocation (144 registers) left room for.  A grid
// smaller than the round's tile count walks the tiles (tile, tile + grid,
// ...; the grid a multiple of 8 keeps every tile on its XCD): the deferred
// updates that run beside the next wave's work take few workgroups, so they
// leave room on every CU for the launches of the factor's own stream.
template <bool F32, int TT>
__device__ __forceinline__ void ssssm_tile(int64_t bid, int64_t total, double *__restrict__ slab,
                                           const LevelDev *__restrict__ levels, const int32_t *__restrict__ rlev,
                                           const int64_t *__restrict__ rtile, int nlev,
                                           const int32_t *__restrict__ rseg, const int64_t *__restrict__ stgt,
                                           const int32_t *__restrict__ maps, int mode) {
    typedef typename std::conditional<F32, float, double>::type elem;
    typedef typename std::conditional<F32, float4_t, double4_t>::type acc4;
    constexpr int NT = TT == 64 ? 256 : 64;
    constexpr int LD = TT + 4;             // LDS row stride
    __shared__ elem As[2][kSsKC][LD], Bs[2][kSsKC][LD];
    {
        const int64_t q = total >> 3, r = total & 7;
        const int64_t x = bid & 7, i = bid >> 3;
        bid = x * q + (x < r ? x : r) + i;
    }
    int lo = 0, hi = nlev - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rtile[5 * mid + mode] <= bid) lo = mid; else hi = mid - 1;
    }
    const LevelDev L = levels[rlev[lo]];
    const int tile = (int)(bid - rtile[5 * lo + mode]);
    const int m = L.m, kp = (L.kappa + 15) & ~15, nseg = L.seg_end - L.seg_begin;
    const int nt = (m + TT - 1) / TT;
    int ti, tj;
    if (mode == 0) {
        ti = tile / nt;
        tj = tile - ti * nt;
    } else if (mode == 1) {
        const int nc = L.sscrit;
        if (tile < nc * nt) {
            ti = tile / nt;
            tj = tile - ti * nt;
        } else {
            const int q = tile - nc * nt;
            ti = nc + q / nc;
            tj = q - (q / nc) * nc;
        }
    } else if (mode == 2) {
        const int nc = L.sscrit, nr = nt - nc;
        ti = nc + tile / nr;
        tj = nc + tile - (tile / nr) * nr;
    } else if (mode == 3) {
        const int nc = L.sscrit;
        ti = tile / nc;
        tj = tile - ti * nc;
    } else {
        const int nc = L.sscrit, nr = nt - nc;
        if (tile < nc * nr) {
            ti = tile / nr;
            tj = nc + tile - ti * nr;
        } else {
            const int q = tile - nc * nr;
            ti = nc + q / nc;
            tj = q - (q / nc) * nc;
        }
    }
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int wr = TT == 64 ? wave >> 1 : 0, wc = TT == 64 ? wave & 1 : 0;

    // one-wave tiles (TT = 32): the epilogue addressing is loaded first so
    // that its latency overlaps the products (these kernels are held to
    // their resident count by LDS, not registers).  This lane's 8 rows a
    // and 2 columns b of the tile:
    const int32_t *__restrict__ RS = rseg + L.Roff;
    const int32_t *__restrict__ RO = maps + L.moff;
    const int32_t *__restrict__ CO = RO + (size_t)nseg * m;
    const int64_t *__restrict__ TG = stgt + L.task_begin;
    int rowa[2][4], colb[2], sa[2][4], sb[2];
    int ro[2][2][4], co[2][2][4];
    int64_t tg[2][2][4];
    if constexpr (TT == 32) {
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            colb[bj] = tj * TT + wc * 32 + bj * 16 + li;
            sb[bj] = RS[min(colb[bj], m - 1)];
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                rowa[bi][r] = ti * TT + wr * 32 + bi * 16 + (F32 ? 4 * lk + r : lk + 4 * r);
                sa[bi][r] = RS[min(rowa[bi][r], m - 1)];
            }
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
    }

    // operand staging: thread (row lr, inner kq) moves P / Qt entries
    // (row, k0 + kq + KS u), u < KU; rows past m read row m - 1 (never stored)
    constexpr int KS = NT / TT, KU = kSsKC / KS;
    const int lr = tid % TT, kq = tid / TT;
    const double *__restrict__ pp = slab + L.offP + min(ti * TT + lr, m - 1) + (size_t)kq * m;
    const double *__restrict__ qp = slab + L.offQ + min(tj * TT + lr, m - 1) + (size_t)kq * m;
    double ra[KU], rb[KU];
    auto gload = [&](int k0) {
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            ra[u] = pp[(size_t)(k0 + KS * u) * m];
            rb[u] = qp[(size_t)(k0 + KS * u) * m];
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            As[buf][kq + KS * u][lr] = (elem)ra[u];
            Bs[buf][kq + KS * u][lr] = (elem)rb[u];
        }
    };
    acc4 c00 = {0, 0, 0, 0}, c01 = c00, c10 = c00, c11 = c00;
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
            const elem a0 = As[buf][k][wr * 32 + li], a1 = As[buf][k][wr * 32 + 16 + li];
            const elem b0 = Bs[buf][k][wc * 32 + li], b1 = Bs[buf][k][wc * 32 + 16 + li];
            if constexpr (F32) {
                c00 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, c00, 0, 0, 0);
                c01 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, c01, 0, 0, 0);
                c10 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, c10, 0, 0, 0);
                c11 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, c11, 0, 0, 0);
            } else {
                c00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, c00, 0, 0, 0);
                c01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, c01, 0, 0, 0);
                c10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, c10, 0, 0, 0);
                c11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, c11, 0, 0, 0);
            }
        }
        if (c + 1 < nch) lstore(buf ^ 1);
        __syncthreads();
    }

    const acc4 acc[2][2] = {{c00, c01}, {c10, c11}};
    if constexpr (TT == 32) {
        // subtract from the targets: all loads first, then the stores
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
                    if (off[bi][bj][r] >= 0) slab[off[bi][bj][r]] = tv[bi][bj][r] - (double)acc[bi][bj][r];
    } else {
        // subtract from the targets, one 16-row half (bi) at a time so that
        // few registers are live: the half's offsets (segment of every row and
        // column, then the offset tables) and target values are loaded first,
        // then its stores.  This lane's rows a and columns b of the tile:
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            colb[bj] = tj * TT + wc * 32 + bj * 16 + li;
            sb[bj] = RS[min(colb[bj], m - 1)];
        }
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
            int rh[4], sh[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                rh[r] = ti * TT + wr * 32 + bi * 16 + (F32 ? 4 * lk + r : lk + 4 * r);
                sh[r] = RS[min(rh[r], m - 1)];
            }
            int64_t off[2][4];
            double tv[2][4];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int roh = RO[(size_t)sb[bj] * m + min(rh[r], m - 1)];
                    const int coh = CO[(size_t)sh[r] * m + min(colb[bj], m - 1)];
                    const int64_t tgh = TG[sh[r] * nseg + sb[bj]];
                    const bool ok = rh[r] < m && colb[bj] < m && roh >= 0 && coh >= 0;
                    off[bj][r] = ok ? tgh + roh + coh : -1;
                    tv[bj][r] = slab[ok ? off[bj][r] : 0];
                }
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (off[bj][r] >= 0) slab[off[bj][r]] = tv[bj][r] - (double)acc[bi][bj][r];
        }
    }
}

template <bool F32, int TT>
__global__ __launch_bounds__(TT == 64 ? 256 : 64, TT == 64 ? 4 : 1) void k_ssssm(double *__restrict__ slab, const LevelDev *__restrict__ levels,
                                               const int32_t *__restrict__ rlev, const int64_t *__restrict__ rtile,
                                               int nlev, const int32_t *__restrict__ rseg,
                                               const int64_t *__restrict__ stgt,
                                               const int32_t *__restrict__ maps, int mode, int64_t total) {
    for (int64_t bid = blockIdx.x; bid < total; bid += gridDim.x) {
        ssssm_tile<F32, TT>(bid, total, slab, levels, rlev, rtile, nlev, rseg, stgt, maps, mode);
        __syncthreads();   // the next tile restages the LDS operands
    }
}

hipError_t launch_ssssm_round(const DevPlan &d, const RoundInfo &r, bool f32, int mode, int max_groups,
                              hipStream_t s) {
    const int64_t counts[5] = {r.tiles, r.tiles_c, r.tiles_r, r.tiles_d, r.tiles_pq};
    const int64_t tiles = counts[mode];
    if (tiles <= 0) return hipSuccess;
    const int nlev = r.end - r.begin;
    const int32_t *rl = d.round_levels + r.begin;
    const int64_t *rt = d.round_tiles + 5 * (size_t)r.begin;
    const dim3 g((unsigned)(max_groups > 0 && tiles > max_groups ? max_groups : tiles));
    if (r.tile == 64) {
        if (f32)
            hipLaunchKernelGGL((k_ssssm<true, 64>), g, dim3(256), 0, s, d.slab, d.levels, rl, rt, nlev, d.rseg,
                               d.stgt, d.maps, mode, tiles);
        else
            hipLaunchKernelGGL((k_ssssm<false, 64>), g, dim3(256), 0, s, d.slab, d.levels, rl, rt, nlev, d.rseg,
                               d.stgt, d.maps, mode, tiles);
    } else {
        if (f32)
            hipLaunchKernelGGL((k_ssssm<true, 32>), g, dim3(64), 0, s, d.slab, d.levels, rl, rt, nlev, d.rseg,
                               d.stgt, d.maps, mode, tiles);
        else
            hipLaunchKernelGGL((k_ssssm<false, 32>), g, dim3(64), 0, s, d.slab, d.levels, rl, rt, nlev, d.rseg,
                               d.stgt, d.maps, mode, tiles);
    }
    return hipGetLastError();
}

// ----------------------------------------------- fixed solve scratch
// Device scratch of the allocation-free solve (slu_solve_noalloc): the
// permuted right-hand-side block of one call, n x nc doubles.  Every device
// the library runs on holds its own copy until the process ends; calls on one
// device share it.
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

hipError_t static_scratch(double **ptr) {
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        // the host-side name stands for the array, not its device address:
        // ask the runtime for this device's copy, once per device
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = (double *)p;
    }
    *ptr = addr[dev];
    return hipSuccess;
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

// ------------------------------------------------- triangular solves in D_i

// Forward substitution with a w x w lower triangle F held by the 16 lanes of
// a row: lane i has x_i and its row f[j] = F(i, j); diagonal scaled by dinv
// unless the triangle has a unit diagonal.
template <int J>
__device__ __forceinline__ void tri_fwd16(double &xi, const double (&f)[16], double dinv, int i, int w,
                                          bool unit) {
    if (J < w) {
        xi = (!unit && i == J) ? xi * dinv : xi;
        const double xj = bcast16<J>(xi);
        xi = (i > J) ? xi - f[J] * xj : xi;
    }
    if constexpr (J + 1 < 16) tri_fwd16<J + 1>(xi, f, dinv, i, w, unit);
}

// Backward substitution with a w x w upper triangle G: lane i has x_i and
// g[j] = G(i, j).
template <int J>
__device__ __forceinline__ void tri_bwd16(double &xi, const double (&g)[16], double dinv, int i, int w,
                                          bool unit) {
    if (J < w) {
        xi = (!unit && i == J) ? xi * dinv : xi;
        const double xj = bcast16<J>(xi);
        xi = (i < J) ? xi - g[J] * xj : xi;
    }
    if constexpr (J > 0) tri_bwd16<J - 1>(xi, g, dinv, i, w, unit);
}

// Solves with the diagonal blocks of all levels of a wave, one workgroup per
// level, on nc right-hand sides of the permuted work block W (x of the block
// in LDS throughout).  FWD: x_i <- F^{-1} x_i with F = L_ii (trans == 0,
// unit) or U_ii^T (trans == 1); otherwise x_i <- G^{-1} x_i with G = U_ii
// (trans == 0) or L_ii^T (trans == 1, unit).  The block is walked in column
// chunks (ascending forward, descending backward):
//   forward:  x_c <- F_cc^{-1} x_c, then x_R -= F(R, c) x_c
//   backward: x_c -= G(c, R) x_R,   then x_c <- G_cc^{-1} x_c
// with R the coupled rows of the chunk.  Chunk panels are staged in LDS a
// batch of chunks at a time by all threads: item t of a chunk (panel row t,
// block row row_t) holds the 16 entries (row_t, c0 + j) of D_i ("column
// panel": forward L, backward L^T) or (c0 + j, row_t) ("row panel": forward
// U^T, backward U), which covers both the chunk's triangles and its coupled
// part.  Each wave then owns four right-hand sides and walks the batch's
// chunks on its own (no barriers): triangles by 16 lanes per right-hand side
// with DPP broadcasts, coupled updates by the wave's 64 lanes.
constexpr int kPnLd = 17;

template <bool FWD>
__global__ __launch_bounds__(256) void k_solve_diag(const double *__restrict__ slab,
                                                    const LevelDev *__restrict__ levels,
                                                    const int32_t *__restrict__ lvl,
                                                    const ChunkDev *__restrict__ schunks,
                                                    const int32_t *__restrict__ sitems,
                                                    const int32_t *__restrict__ sbatch, double *__restrict__ W,
                                                    int64_t n, int nc, int trans) {
    extern __shared__ double lds[];
    const LevelDev L = levels[lvl[blockIdx.x]];
    const int b = L.b;
    const double *__restrict__ D = slab + L.offD;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const bool colpanel = FWD ? trans == 0 : trans != 0;
    const bool unit = FWD ? trans == 0 : trans != 0;
    double *xs = lds;                                        // xs[c * b + r]
    double *Pn = lds + (((size_t)b * nc + 1) & ~(size_t)1);  // kSolveItems x kPnLd
    int *rowb = (int *)(Pn + kSolveItems * kPnLd);           // block row of every item
    int *icw = rowb + kSolveItems;                           // c0 << 5 | w of every item
    int *desc = icw + kSolveItems;                           // (c0, w, nr, item) per chunk
    const int32_t *__restrict__ brec = sbatch + 2 * (size_t)L.sb_begin;   // batch records of the level
    const int nb = L.sb_end - L.sb_begin - 1;
    for (int e0 = tid; e0 < b * nc; e0 += 256 * 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = min(e0 + 256 * u, b * nc - 1);
            const int c = e / b, r = e - c * b;
            v[u] = W[L.r0 + r + (size_t)c * n];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (e0 + 256 * u < b * nc) xs[e0 + 256 * u] = v[u];
    }
    // this wave's right-hand sides: cw0 + g for g < ncw
    const int cw0 = 4 * wave;
    const int ncw = max(0, min(4, nc - cw0));
    const int g = lane >> 4, i16 = lane & 15;
    for (int bq = 0; bq < nb; ++bq) {
        __syncthreads();
        const int bi = FWD ? bq : nb - 1 - bq;
        const int kb = brec[2 * bi], ke = brec[2 * bi + 2];
        const int i0 = brec[2 * bi + 1], i1 = brec[2 * bi + 3];
        // stage the batch: chunk descriptors and item records first, then
        // the 16 entries of every item with all of a thread's loads in flight
        for (int q = tid; q < ke - kb; q += 256) {
            const ChunkDev C = schunks[kb + q];
            desc[4 * q] = C.c0;
            desc[4 * q + 1] = C.w;
            desc[4 * q + 2] = C.nr;
            desc[4 * q + 3] = C.pad;
        }
        const int nit = i1 - i0;
        for (int q = tid; q < nit; q += 256) {
            const int2 rec = reinterpret_cast<const int2 *>(sitems)[L.sitem + i0 + q];
            rowb[q] = rec.x;
            icw[q] = rec.y;
        }
        __syncthreads();
        {
            // column panels: entry (item, j) is e = j * 512 + item, so that
            // consecutive lanes take consecutive items of one column; row
            // panels: e = item * 16 + j, the 16 entries of an item contiguous
            constexpr int PER = kSolveItems * 16 / 256;
            static_assert(kSolveItems == 512, "column-panel staging assumes 512 items");
            double v[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int e = tid + 256 * u;
                const int it = min(colpanel ? (e & 511) : (e >> 4), nit - 1);
                const int j = colpanel ? (e >> 9) : (e & 15);
                const int row = rowb[it], cw = icw[it];
                // entries j >= w are never read: clamp to a valid address
                const int col = (cw >> 5) + min(j, (cw & 31) - 1);
                v[u] = colpanel ? D[row + (size_t)col * b] : D[col + (size_t)row * b];
            }
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int e = tid + 256 * u;
                const int it = colpanel ? (e & 511) : (e >> 4);
                const int j = colpanel ? (e >> 9) : (e & 15);
                if (it < nit) Pn[it * kPnLd + j] = v[u];
            }
        }
        __syncthreads();
        if (ncw == 0) continue;
        for (int kq = 0; kq < ke - kb; ++kq) {
            const int kk = FWD ? kq : ke - kb - 1 - kq;
            const int c0 = desc[4 * kk], wf = desc[4 * kk + 1], nr = desc[4 * kk + 2];
            const int w = wf & (kSolveCont - 1);
            const bool first = (wf & kSolveCont) == 0;    // continuation parts skip the triangle
            const int ib = desc[4 * kk + 3] - i0;
            const double *__restrict__ base = Pn + (size_t)ib * kPnLd;
            const int *__restrict__ rows = rowb + ib;         // rows[t], t >= w: coupled rows
            if (!FWD) {
                // x_c -= G(c, R) x_R: lpi lanes per (row i, right-hand side)
                const int lpi = ncw == 1 ? 4 : (ncw == 2 ? 2 : 1);
                const int item = lane / lpi, sub = lane - item * lpi;
                const int cc = item >> 4, i = item & 15;
                double acc = 0.0;
                if (cc < ncw && i < w) {
                    const double *xc = xs + (size_t)(cw0 + cc) * b;
                    for (int sI = sub; sI < nr; sI += lpi) acc += base[(w + sI) * kPnLd + i] * xc[rows[w + sI]];
                }
                if (lpi >= 2) acc += __shfl_xor(acc, 1, 64);
                if (lpi >= 4) acc += __shfl_xor(acc, 2, 64);
                if (cc < ncw && i < w && sub == 0) xs[(size_t)(cw0 + cc) * b + c0 + i] -= acc;
            }
            if (first && g < ncw) {
                // the chunk's triangle: 16 lanes per right-hand side
                const int i = i16;
                const int ic = i < w ? i : w - 1;
                double *xc = xs + (size_t)(cw0 + g) * b;
                double xi = xc[c0 + ic];
                double f[16];
                if (FWD) {
#pragma unroll
                    for (int j = 0; j < 16; ++j) f[j] = base[ic * kPnLd + j];               // F(i, j)
                } else {
#pragma unroll
                    for (int j = 0; j < 16; ++j) f[j] = base[min(j, w - 1) * kPnLd + ic];   // G(i, j)
                }
                const double dinv = unit ? 1.0 : 1.0 / base[ic * kPnLd + ic];
                if (FWD)
                    tri_fwd16<0>(xi, f, dinv, i, w, unit);
                else
                    tri_bwd16<15>(xi, f, dinv, i, w, unit);
                if (i < w) xc[c0 + i] = xi;
            }
            if (FWD) {
                // x_R -= F(R, c) x_c for the wave's right-hand sides
                for (int q = lane; q < nr * ncw; q += 64) {
                    const int cc = q / nr, sI = q - cc * nr;
                    double *xc = xs + (size_t)(cw0 + cc) * b;
                    const double *__restrict__ prow = base + (size_t)(w + sI) * kPnLd;
                    double acc = 0.0;
#pragma unroll
                    for (int j = 0; j < 16; ++j)
                        if (j < w) acc += prow[j] * xc[c0 + j];
                    xc[rows[w + sI]] -= acc;
                }
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < b * nc; e += 256) {
        const int c = e / b, r = e - c * b;
        W[L.r0 + r + (size_t)c * n] = xs[e];
    }
}

size_t solve_diag_lds_bytes(int max_b, int nc) {
    return ((((size_t)max_b * nc + 1) & ~(size_t)1) + (size_t)kSolveItems * kPnLd) * sizeof(double) +
           (size_t)(2 * kSolveItems + 4 * kSolveBatchChunks) * sizeof(int);
}

hipError_t launch_solve_diag_wave(const DevPlan &d, const int32_t *lvl, int nlev, int max_b, bool fwd, int nc,
                                  int trans, hipStream_t s) {
    const size_t lds = solve_diag_lds_bytes(max_b, nc);
    if (fwd)
        hipLaunchKernelGGL(k_solve_diag<true>, dim3((unsigned)nlev), dim3(256), lds, s, d.slab, d.levels, lvl,
                           d.schunks, d.sitems, d.sbatch, d.scratch, d.n, nc, trans);
    else
        hipLaunchKernelGGL(k_solve_diag<false>, dim3((unsigned)nlev), dim3(256), lds, s, d.slab, d.levels, lvl,
                           d.schunks, d.sitems, d.sbatch, d.scratch, d.n, nc, trans);
    return hipGetLastError();
}

// ------------------------------------------------ tiled diagonal solves
// Diagonal-block solves of a wave whose blocks were factored by the 32 x 32
// tiled GETRF, with the inverted diagonal tiles it kept: for the forward
// sweep (L, or U^T when transposed) tile t gives x_t = M_t b_t and every
// later row tile r takes b_r -= A_rt x_t; the backward sweep (U, or L^T)
// runs the same from the last tile up.  The tiles are taken two at a time,
// in sweep order: pair p = (t0, t1) gives x_t0 = M_t0 b_t0,
// x_t1 = M_t1 (b_t1 - A_t1t0 x_t0), and every later row tile r takes
// b_r -= A_rt0 x_t0 + A_rt1 x_t1.  One launch per pair step u, one wave per
// (level, row tile r beyond pair u): each wave forms both x of pair u itself
// from b_t0 and b_t1 (read-only in step u) and updates its own rows.  The
// wave q = 0 of step u > 0 stores x of pair u - 1 (nobody reads those rows in
// step u); the last pair, which has no row tile beyond it, is stored by a
// wave of its own step.  M_t is iL_t, iU_t^T, iU_t or iL_t^T; A_rt is the
// block's tile (r, t), transposed for the transposed solve.  The right-hand
// sides of a 32-row tile are the 16 columns of 16 x 16 x 4 FP64 MFMA
// products (nc <= 16); a product's result layout is also the layout of the
// operand the next product takes, so x_t0 feeds A_t1t0 x_t0 directly.
template <bool ONE>
__global__ __launch_bounds__(64) void k_solve_tile(int b1, int r01, int64_t offD1, int64_t offW1,
                                                   const double *__restrict__ slab, const double *__restrict__ work,
                                                   double *__restrict__ Wx, int64_t n, int u, int fwd, int trans,
                                                   int nc, const LevelDev *__restrict__ levels,
                                                   const int32_t *__restrict__ lvl) {
    int b, r0;
    int64_t offD, offW;
    if constexpr (ONE) {
        b = b1, r0 = r01, offD = offD1, offW = offW1;
    } else {
        const LevelDev &L = levels[lvl[blockIdx.y]];
        b = L.b, r0 = L.r0, offD = L.offD, offW = L.offW;
    }
    const int nt = (b + 31) >> 5;
    if (2 * u >= nt) return;   // this block's last pair came before step u
    const int q = blockIdx.x;
    // Tiles are counted in sweep order (tile j is j forward, nt - 1 - j
    // backward).  Workgroup q: pair u - 1 to store (q = 0, when u > 0), then
    // the row tiles beyond pair u, walking away from it; at the last pair the
    // first of those stores pair u instead.
    const int q0 = u > 0 ? 1 : 0;
    const int nrow = nt - 2 * u - 2;
    int pair, jr;   // pair solved; row tile updated in sweep order (-1: store the pair)
    if (u > 0 && q == 0) {
        pair = u - 1, jr = -1;
    } else {
        const int j = q - q0;
        if (j >= (nrow > 0 ? nrow : 1)) return;
        pair = u, jr = nrow > 0 ? 2 * u + 2 + j : -1;
    }
    const int j0 = 2 * pair;
    const bool has1 = j0 + 1 < nt;   // false only for a single last tile
    const int t0 = fwd ? j0 : nt - 1 - j0;
    // a missing second tile is read as t0 again (in range) and never stored
    const int t1 = has1 ? (fwd ? j0 + 1 : nt - 2 - j0) : t0;
    const int r = jr >= 0 ? (fwd ? jr : nt - 1 - jr) : t0;   // row tile, or t0 again when storing
    const double *__restrict__ D = slab + offD;
    const double *__restrict__ Inv = work + offW + 128 * (size_t)b;
    const int lane = threadIdx.x, li = lane & 15, g = lane >> 4;
    const bool rhs_ok = li < nc;
    double *__restrict__ Xc = Wx + (size_t)(rhs_ok ? li : 0) * n + r0;   // this lane's right-hand side
    // Loads are unconditional from clamped addresses, so that they all go out
    // together.  Rows past b read an in-range value: the inverted tiles are
    // the identity there and zero beside it, so such a value only reaches
    // rows past b of x, which are never stored and meet only zeroed entries
    // of A below (entries past b are multiplied by 0).
    const bool use_l = (fwd != 0) == (trans == 0);   // M and A from L (else from U)
    // M_s (32 x 32 inverses of tile s, iL row-major, iU column-major):
    // element (i, k) of the operator applied, i.e. iL / iU, transposed for
    // the transposed solve
    const bool mtr = use_l ? trans != 0 : trans == 0;
    // rows of tile s in result layout: half h, lane (li, g), element e ->
    // row 16 h + g + 4 e, right-hand side li (also the B-operand layout of a
    // product over tile s: step kk, lane (li, g) -> row 16 hk + 4 kk + g)
    auto load_b = [&](int s, double4_t(&v)[2]) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < 4; ++e) v[h][e] = Xc[min(32 * s + 16 * h + g + 4 * e, b - 1)];
    };
    auto load_m = [&](int s, double(&m)[2][2][4]) {
        const double *Mb = Inv + (size_t)s * 2048 + (use_l ? 0 : 1024);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int hk = 0; hk < 2; ++hk)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int i = 16 * h + li, k = 16 * hk + 4 * kk + g;
                    m[h][hk][kk] = mtr ? Mb[k * 32 + i] : Mb[i * 32 + k];
                }
    };
    // -A_rt (i, k) = -D(32 r + i, 32 t + k), or -D(32 t + k, 32 r + i) for
    // the transposed solve; zero past b, and everywhere when on == 0
    auto load_a = [&](int rr, int tt, double on, double(&a)[2][2][4]) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ri = 32 * rr + 16 * h + li;
#pragma unroll
            for (int hk = 0; hk < 2; ++hk)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int ck = 32 * tt + 16 * hk + 4 * kk + g;
                    const size_t ric = (size_t)min(ri, b - 1), ckc = (size_t)min(ck, b - 1);
                    a[h][hk][kk] = (trans ? D[ric * b + ckc] : D[ckc * b + ric]) * ((ri < b && ck < b) ? -on : 0.0);
                }
        }
    };
    // x = m bin
    auto apply_m = [&](const double(&m)[2][2][4], const double4_t(&bin)[2], double4_t(&x)[2]) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            x[h] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int hk = 0; hk < 2; ++hk)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    x[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(m[h][hk][kk], bin[hk][kk], x[h], 0, 0, 0);
        }
    };
    // acc += a x
    auto apply_a = [&](const double(&a)[2][2][4], const double4_t(&x)[2], double4_t(&acc)[2]) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int hk = 0; hk < 2; ++hk)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[h][hk][kk], x[hk][kk], acc[h], 0, 0, 0);
    };
    auto store = [&](int s, const double4_t(&v)[2]) {
        if (rhs_ok) {
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = 32 * s + 16 * h + g + 4 * e;
                    if (row < b) Xc[row] = v[h][e];
                }
        }
    };
    double4_t bt0[2], bt1[2], br[2];
    double m0[2][2][4], m1[2][2][4], a10[2][2][4], ar0[2][2][4], ar1[2][2][4];
    load_b(t0, bt0);
    load_b(t1, bt1);
    load_m(t0, m0);
    load_m(t1, m1);
    load_a(t1, t0, has1 ? 1.0 : 0.0, a10);
    load_b(r, br);
    load_a(r, t0, 1.0, ar0);
    load_a(r, t1, 1.0, ar1);
    // keep every load ahead of the products: one memory round trip in all
    __builtin_amdgcn_sched_barrier(0);
    double4_t x0[2], x1[2];
    apply_m(m0, bt0, x0);
    apply_a(a10, x0, bt1);
    apply_m(m1, bt1, x1);
    // formed by the storing wave too (on its own rows, and not stored), so
    // that no load is left for a branch
    apply_a(ar0, x0, br);
    apply_a(ar1, x1, br);
    if (jr >= 0) {
        store(r, br);
    } else {
        store(t0, x0);
        if (has1) store(t1, x1);
    }
}

hipError_t launch_solve_tile_wave(const DevPlan &d, const int32_t *lvl, int nlev, int max_b, bool fwd, int nc,
                                  int trans, const LevelDev *one, hipStream_t s) {
    if (nlev <= 0 || nlev > 65535) return hipErrorInvalidValue;
    const int nt = (max_b + 31) / 32;
    for (int u = 0; 2 * u < nt; ++u) {
        // waves of step u: pair u - 1 stored, then the row tiles beyond pair
        // u (or, at the last pair, the wave that stores it)
        const int rows = nt - 2 * u - 2;
        const unsigned gx = (unsigned)((u > 0 ? 1 : 0) + (rows > 1 ? rows : 1));
        if (nlev == 1 && one)
            hipLaunchKernelGGL(k_solve_tile<true>, dim3(gx, 1), dim3(64), 0, s, one->b, one->r0, one->offD, one->offW,
                               d.slab, d.tgetrf, d.scratch, d.n, u, fwd ? 1 : 0, trans, nc, d.levels, lvl);
        else
            hipLaunchKernelGGL(k_solve_tile<false>, dim3(gx, (unsigned)nlev), dim3(64), 0, s, 0, 0, (int64_t)0,
                               (int64_t)0, d.slab, d.tgetrf, d.scratch, d.n, u, fwd ? 1 : 0, trans, nc, d.levels,
                               lvl);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// W[rows_i[a]] -= X[a, :] . W[r0 + K_i]   (X = P_i, or Qt_i when transposed)
// for the levels of one Schur-update round, whose target rows are disjoint:
// blockIdx.x picks the level, blockIdx.y (striding by gridDim.y) its 32-row
// tiles.  The right-hand sides are the 16 columns of FP64 MFMA 16 x 16 x 4
// products (columns past nc are zero); the four waves split the inner index
// in interleaved 4-deep steps, with its W values staged in LDS 256 at a time
// (column-major, padded against bank conflicts); the four partial sums are
// added in LDS in a fixed order.  Loads go out in batches from clamped
// addresses (values past the slice masked by a product), sized to the
// slice, so that it costs a few memory round trips instead of one per step
// and right-hand side.
constexpr int kUpdSlice = 256;

__global__ __launch_bounds__(256) void k_fwd_update(const double *__restrict__ slab,
                                                    const LevelDev *__restrict__ levels,
                                                    const int32_t *__restrict__ lvl,
                                                    const int32_t *__restrict__ Kidx,
                                                    const int32_t *__restrict__ Ridx, double *__restrict__ W,
                                                    int64_t n, int nc, int trans) {
    constexpr int XL = kUpdSlice + 1;
    __shared__ double xk[16 * XL];               // [c][t]
    __shared__ double part[4][2][4][64];         // [wave][h][r][lane]
    const LevelDev L = levels[lvl[blockIdx.x]];
    const int m = L.m, kap = L.kappa;
    const double *__restrict__ X = slab + (trans ? L.offQ : L.offP);
    const int32_t *__restrict__ K = Kidx + L.Koff;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
    for (int e = tid; e < 16 * XL; e += 256) xk[e] = 0.0;   // columns past nc stay zero
    for (int tile = blockIdx.y; tile * 32 < m; tile += gridDim.y) {
        const int row0 = tile * 32;
        const size_t ra0 = (size_t)min(row0 + li, m - 1), ra1 = (size_t)min(row0 + 16 + li, m - 1);
        double4_t acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
        for (int t0 = 0; t0 < kap; t0 += kUpdSlice) {
            const int nt = min(kUpdSlice, kap - t0);
            // thread tid stages inner index tid of the slice for every
            // right-hand side (kUpdSlice == the workgroup size)
            double xv[16];
            if (tid < nt) {
                const size_t kt = (size_t)L.r0 + K[t0 + tid];
#pragma unroll
                for (int c = 0; c < 16; ++c) xv[c] = W[kt + (size_t)min(c, nc - 1) * n];
            }
            __syncthreads();
            if (tid < nt) {
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    if (c < nc) xk[c * XL + tid] = xv[c];
            }
            __syncthreads();
            // step j: inner index t = 16 j + 4 wave + g in lane group g;
            // the operands of NS steps load before their products: eight
            // at a time, then four for the rest
            const int nst = (nt + 15) >> 4;
            auto steps = [&](auto ns, int j0) {
                constexpr int NS = decltype(ns)::value;
                double a0[NS], a1[NS], bv[NS];
#pragma unroll
                for (int jj = 0; jj < NS; ++jj) {
                    const int t = 16 * (j0 + jj) + 4 * wave + g;
                    const int tcl = min(t, nt - 1);
                    const size_t tc = (size_t)(t0 + tcl);
                    const double msk = t < nt ? 1.0 : 0.0;
                    a0[jj] = X[tc * m + ra0] * msk;
                    a1[jj] = X[tc * m + ra1] * msk;
                    bv[jj] = xk[li * XL + tcl] * msk;
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int jj = 0; jj < NS; ++jj) {
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[jj], bv[jj], acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[jj], bv[jj], acc1, 0, 0, 0);
                }
            };
            int j0 = 0;
            for (; j0 + 8 <= nst; j0 += 8) steps(std::integral_constant<int, 8>{}, j0);
            for (; j0 < nst; j0 += 4) steps(std::integral_constant<int, 4>{}, j0);
        }
        // acc_h[r] of lane (li, g): row 16 h + g + 4 r of the tile, column li
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            part[wave][0][r][lane] = acc0[r];
            part[wave][1][r][lane] = acc1[r];
        }
        __syncthreads();
        for (int e = tid; e < 32 * nc; e += 256) {
            const int c = e >> 5, row = e & 31;
            const int h = row >> 4, rr = row & 15, pl = c + 16 * (rr & 3), pr = rr >> 2;
            if (row0 + row < m) {
                const double v = (part[0][h][pr][pl] + part[1][h][pr][pl]) + (part[2][h][pr][pl] + part[3][h][pr][pl]);
                W[Ridx[L.Roff + row0 + row] + (size_t)c * n] -= v;
            }
        }
    }
}

// W[r0 + K_i[t]] -= sum_a X[a, t] W[rows_i[a]]   (X = Qt_i, or P_i when transposed)
// for the levels of one wave (each writes only its own block's rows):
// blockIdx.x picks the level, blockIdx.y (striding by gridDim.y) the column
// t, blockIdx.z the right-hand side; one wave reduces over a, eight rows per
// lane at a time and two for the rest (their indices, then the gathered
// values, load together: two memory round trips per 512 rows) into four
// partial sums added in a fixed order.
__global__ __launch_bounds__(64) void k_bwd_update(const double *__restrict__ slab, const LevelDev *__restrict__ levels,
                                                   const int32_t *__restrict__ lvl,
                                                   const int32_t *__restrict__ Kidx,
                                                   const int32_t *__restrict__ Ridx, double *__restrict__ W,
                                                   int64_t n, int trans) {
    const LevelDev L = levels[lvl[blockIdx.x]];
    const int m = L.m;
    if (m == 0) return;
    const int c = blockIdx.z;
    const int32_t *__restrict__ R = Ridx + L.Roff;
    const double *__restrict__ Wc = W + (size_t)c * n;
    for (int t = blockIdx.y; t < L.kappa; t += gridDim.y) {
        const double *__restrict__ X = slab + (trans ? L.offP : L.offQ) + (size_t)t * m;
        double part[4] = {0.0, 0.0, 0.0, 0.0};
        // NS rows per lane at a time: eight, then two for the rest
        auto rows = [&](auto ns, int a0) {
            constexpr int NS = decltype(ns)::value;
            int32_t ri[NS];
            double xv[NS];
#pragma unroll
            for (int jj = 0; jj < NS; ++jj) {
                const int a = a0 + 64 * jj + (int)threadIdx.x;
                const int ac = min(a, m - 1);
                ri[jj] = R[ac];
                xv[jj] = X[ac] * (a < m ? 1.0 : 0.0);
            }
#pragma unroll
            for (int jj = 0; jj < NS; ++jj) part[jj & 3] += xv[jj] * Wc[ri[jj]];
        };
        int a0 = 0;
        for (; a0 + 512 <= m; a0 += 512) rows(std::integral_constant<int, 8>{}, a0);
        for (; a0 < m; a0 += 128) rows(std::integral_constant<int, 2>{}, a0);
        double acc = (part[0] + part[1]) + (part[2] + part[3]);
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if (threadIdx.x == 0) W[L.r0 + Kidx[L.Koff + t] + (size_t)c * n] -= acc;
    }
}

hipError_t launch_fwd_update(const DevPlan &d, const int32_t *lvl, int nlev, int max_m, int nc, int trans,
                             hipStream_t s) {
    if (nlev <= 0 || max_m <= 0) return hipSuccess;
    const int64_t tiles = ((int64_t)max_m + 31) / 32;
    hipLaunchKernelGGL(k_fwd_update, dim3((unsigned)nlev, (unsigned)std::min<int64_t>(tiles, 65535)), dim3(256), 0,
                       s, d.slab, d.levels, lvl, d.K_idx, d.R_idx, d.scratch, d.n, nc, trans);
    return hipGetLastError();
}

hipError_t launch_bwd_update(const DevPlan &d, const int32_t *lvl, int nlev, int max_kappa, int nc, int trans,
                             hipStream_t s) {
    if (nlev <= 0 || max_kappa <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bwd_update, dim3((unsigned)nlev, (unsigned)std::min(max_kappa, 4096), (unsigned)nc),
                       dim3(64), 0, s, d.slab, d.levels, lvl, d.K_idx, d.R_idx, d.scratch, d.n, trans);
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

// grad[q] = -sum_c G[i, c] X[j, c] for CSR entry q = (i, j): one thread per row.
__global__ void k_value_gradient(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                                 const double *__restrict__ G, const double *__restrict__ X, int64_t ld,
                                 int64_t n, int64_t nrhs, double *__restrict__ grad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
            const int64_t j = colidx[q];
            double acc = 0.0;
            for (int64_t c = 0; c < nrhs; ++c) acc += G[i + c * ld] * X[j + c * ld];
            grad[q] = -acc;
        }
    }
}

hipError_t launch_value_gradient(const DevPlan &d, const double *G, const double *X, int64_t nrhs, int64_t ld,
                                 double *grad, hipStream_t s) {
    if (d.n <= 0) return hipSuccess;
    int64_t blocks = (d.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_value_gradient, dim3((unsigned)blocks), dim3(256), 0, s, d.a_rowptr, d.a_colidx, G, X,
                       ld, d.n, nrhs, grad);
    return hipGetLastError();
}

// R = B - A X for nc columns (A in CSR, original order): one thread per row.
__global__ void k_residual(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                           const double *__restrict__ vals, const double *__restrict__ B, int64_t ldb,
                           const double *__restrict__ X, int64_t ldx, double *__restrict__ R, int64_t ldr,
                           int64_t n, int nc) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        for (int c = 0; c < nc; ++c) {
            const double *__restrict__ xc = X + (size_t)c * ldx;
            double r = B[i + (size_t)c * ldb];
            for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) r -= vals[q] * xc[colidx[q]];
            R[i + (size_t)c * ldr] = r;
        }
    }
}

__global__ void k_axpy(double *__restrict__ X, int64_t ldx, const double *__restrict__ Dv, int64_t ldd, int64_t n,
                       int nc) {
    const int64_t total = n * nc;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t c = e / n, i = e - c * n;
        X[i + c * ldx] += Dv[i + c * ldd];
    }
}

hipError_t launch_residual(const DevPlan &d, const double *values, const double *B, int64_t ldb, const double *X,
                           int64_t ldx, double *R, int64_t ldr, int nc, hipStream_t s) {
    if (d.n <= 0) return hipSuccess;
    int64_t blocks = (d.n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_residual, dim3((unsigned)blocks), dim3(256), 0, s, d.a_rowptr, d.a_colidx, values, B, ldb,
                       X, ldx, R, ldr, d.n, nc);
    return hipGetLastError();
}

hipError_t launch_axpy(const DevPlan &d, double *X, int64_t ldx, const double *Dv, int64_t ldd, int nc,
                       hipStream_t s) {
    int64_t blocks = (d.n * nc + 255) / 256;
    if (blocks < 1) return hipSuccess;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_axpy, dim3((unsigned)blocks), dim3(256), 0, s, X, ldx, Dv, ldd, d.n, nc);
    return hipGetLastError();
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
    e = hipFuncSetAttribute((const void *)k_solve_diag<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_solve_diag<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_getrf_wave, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)k_getrf_step, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_panel_solve<32, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_panel_solve_pf<32, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_panel_solve_pf<16, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_panel_solve<16, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    return e;
}

}  // namespace slu
