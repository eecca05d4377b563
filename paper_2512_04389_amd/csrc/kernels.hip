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
// Alg. 1 line "B_ii -> L_ii U_ii": no-pivot LU of the dense diagonal block,
// one workgroup.  The block is processed in column chunks [c0, c0 + w):
// the chunk's panel (its own rows plus the coupled rows R below it) is
// factored in LDS, the chunk's U rows over R are forward-substituted, and the
// trailing entries R x R are updated.  Entries outside the rows/columns R are
// structurally untouched by the chunk.  Blocks of at most 128 rows are a
// single chunk that lives entirely in LDS.
__global__ __launch_bounds__(1024) void k_getrf(double *__restrict__ slab, const LevelDev *__restrict__ levels,
                                                int level, const ChunkDev *__restrict__ chunks,
                                                const int32_t *__restrict__ crows,
                                                unsigned long long *__restrict__ info) {
    extern __shared__ double lds[];
    const LevelDev L = levels[level];
    double *__restrict__ D = slab + L.offD;
    const int b = L.b;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int ch = L.chunk_begin; ch < L.chunk_end; ++ch) {
        const ChunkDev C = chunks[ch];
        const int c0 = C.c0, w = C.w, nr = C.nr;
        const int32_t *__restrict__ R = crows + C.roff;
        const int T = w + nr;
        double *Pn = lds;                      // Pn[j*T + t]: panel column j, panel row t
        double *Ur = lds + (size_t)T * w;      // Ur[s*w + j]: U(c0 + j, R[s])
        for (int e = tid; e < T * w; e += nt) {
            const int j = e / T, t = e - j * T;
            const int row = t < w ? c0 + t : R[t - w];
            Pn[e] = D[row + (size_t)(c0 + j) * b];
        }
        __syncthreads();
        for (int k = 0; k < w; ++k) {
            const double piv = Pn[k * T + k];
            if (tid == 0 && !(piv != 0.0 && isfinite(piv)))
                atomicMin(info, (unsigned long long)(L.r0 + c0 + k));
            for (int t = k + 1 + tid; t < T; t += nt) Pn[k * T + t] = Pn[k * T + t] / piv;
            __syncthreads();
            const int rows = T - k - 1, cols = w - k - 1;
            for (int e = tid; e < rows * cols; e += nt) {
                const int jj = e / rows, tt = e - jj * rows;
                const int j = k + 1 + jj, t = k + 1 + tt;
                Pn[j * T + t] -= Pn[k * T + t] * Pn[j * T + k];
            }
            __syncthreads();
        }
        for (int e = tid; e < T * w; e += nt) {
            const int j = e / T, t = e - j * T;
            const int row = t < w ? c0 + t : R[t - w];
            D[row + (size_t)(c0 + j) * b] = Pn[e];
        }
        if (nr > 0) {
            for (int sI = tid; sI < nr; sI += nt) {
                double u[16];
                const size_t colo = (size_t)R[sI] * b;
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if (j < w) u[j] = D[c0 + j + colo];
#pragma unroll
                for (int j = 1; j < 16; ++j) {
                    if (j < w) {
                        double v = u[j];
#pragma unroll
                        for (int jp = 0; jp < j; ++jp) v -= Pn[jp * T + j] * u[jp];
                        u[j] = v;
                    }
                }
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    if (j < w) {
                        Ur[sI * w + j] = u[j];
                        D[c0 + j + colo] = u[j];
                    }
            }
            __syncthreads();
            for (int e = tid; e < nr * nr; e += nt) {
                const int sI = e / nr, t = e - sI * nr;
                double acc = 0.0;
                for (int j = 0; j < w; ++j) acc += Pn[j * T + w + t] * Ur[sI * w + j];
                D[R[t] + (size_t)R[sI] * b] -= acc;
            }
        }
        __syncthreads();
    }
}

hipError_t launch_getrf(const DevPlan &d, int level, int lds_bytes, hipStream_t s) {
    hipLaunchKernelGGL(k_getrf, dim3(1), dim3(1024), (size_t)lds_bytes, s, d.slab, d.levels, level, d.chunks,
                       d.chunk_rows, d.info);
    return hipGetLastError();
}

// ------------------------------------------------------------ GESSM / TSTRF
// Alg. 1 "B_ij <- L_ii^{-1} B_ij" and "B_ji <- B_ji U_ii^{-1}" on the whole
// U and L panels of level i.  On the coupled index set K_i both become a
// right-side triangular solve X <- X T^{-1} of an m x kappa panel:
//   L panel  (blockIdx.y == 0): X = P_i,  T = U_ii[K, K]          (pivot division)
//   U panel  (blockIdx.y == 1): X = Qt_i, T = L_ii[K, K]^T        (unit diagonal)
// One workgroup owns rt (16, 8, 4, 2 or 1) panel rows held in LDS, so that
// kappa * rt doubles fit; the columns are processed in chunks of 16: a
// product with the finished columns, then a 16-column triangular solve.
__global__ __launch_bounds__(256) void k_trsm_panels(double *__restrict__ slab, const LevelDev *__restrict__ levels,
                                                     int level, const int32_t *__restrict__ Kidx, int rt) {
    extern __shared__ double xs[];  // xs[t*rt + r]
    const LevelDev L = levels[level];
    const int kap = L.kappa, m = L.m, b = L.b;
    const bool lpanel = blockIdx.y == 0;
    double *__restrict__ X = slab + (lpanel ? L.offP : L.offQ);
    const double *__restrict__ D = slab + L.offD;
    const int32_t *__restrict__ K = Kidx + L.Koff;
    const int a0 = blockIdx.x * rt;
    const int nrow = min(rt, m - a0);
    const int tid = threadIdx.x;
    for (int e = tid; e < rt * kap; e += 256) {
        const int t = e / rt, r = e - t * rt;
        xs[e] = r < nrow ? X[a0 + r + (size_t)t * m] : 0.0;
    }
    __syncthreads();
    const int r = tid % rt, jj = tid / rt;
    for (int c0 = 0; c0 < kap; c0 += 16) {
        const int cw = min(16, kap - c0);
        if (jj < cw) {
            const int col = c0 + jj;
            const size_t Kc = (size_t)K[col];
            double acc = 0.0;
            if (lpanel) {
                const double *__restrict__ Dc = D + Kc * b;     // U(K[t], K[col]) = D[K[t] + K[col]*b]
                for (int t = 0; t < c0; ++t) acc += xs[t * rt + r] * Dc[K[t]];
            } else {
                const double *__restrict__ Dr = D + Kc;         // L(K[col], K[t]) = D[K[col] + K[t]*b]
                for (int t = 0; t < c0; ++t) acc += xs[t * rt + r] * Dr[(size_t)K[t] * b];
            }
            xs[col * rt + r] -= acc;
        }
        __syncthreads();
        if (jj == 0) {
            for (int j = 0; j < cw; ++j) {
                const int col = c0 + j;
                const size_t Kc = (size_t)K[col];
                double v = xs[col * rt + r];
                for (int jp = 0; jp < j; ++jp) {
                    const size_t Kp = (size_t)K[c0 + jp];
                    const double tv = lpanel ? D[Kp + Kc * b] : D[Kc + Kp * b];
                    v -= xs[(c0 + jp) * rt + r] * tv;
                }
                if (lpanel) v = v / D[Kc + Kc * b];
                xs[col * rt + r] = v;
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < rt * kap; e += 256) {
        const int t = e / rt, rr = e - t * rt;
        if (rr < nrow) X[a0 + rr + (size_t)t * m] = xs[e];
    }
}

int trsm_rows_per_group(int kappa) {
    int rt = 16;
    while (rt > 1 && (int64_t)kappa * rt * 8 > 150 * 1024) rt /= 2;
    return rt;
}

hipError_t launch_trsm_panels(const DevPlan &d, int level, int m, int kappa, hipStream_t s) {
    if (m <= 0 || kappa <= 0) return hipSuccess;
    const int rt = trsm_rows_per_group(kappa);
    dim3 grid((unsigned)((m + rt - 1) / rt), 2);
    hipLaunchKernelGGL(k_trsm_panels, grid, dim3(256), (size_t)kappa * rt * sizeof(double), s, d.slab, d.levels,
                       level, d.K_idx, rt);
    return hipGetLastError();
}

// ------------------------------------------------- dense GETRF (b <= 128)
// Diagonal blocks of at most 128 rows: the whole block in LDS, blocked
// right-looking LU with 16-column panels.  One wave factors the panel in
// registers (each lane owns up to two rows; pivot row values are broadcast
// with lane shuffles), all threads solve the panel's U rows, and the four
// waves apply the trailing update as 16 x 16 FP64 MFMA tiles.
__global__ __launch_bounds__(256) void k_getrf_dense(double *__restrict__ slab, const LevelDev *__restrict__ levels,
                                                     int level, unsigned long long *__restrict__ info) {
    extern __shared__ double ds[];
    const LevelDev L = levels[level];
    double *__restrict__ D = slab + L.offD;
    const int b = L.b;
    const int ldd = b | 1;                 // odd stride: conflict-free column-strided LDS access
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    for (int c = 0; c < b; ++c)
        for (int r = tid; r < b; r += 256) ds[c * ldd + r] = D[r + (size_t)c * b];
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
                    const double piv = __shfl(v0[k], k, 64);
                    if (lane == 0 && !(piv != 0.0 && isfinite(piv)))
                        atomicMin(info, (unsigned long long)(L.r0 + c0 + k));
                    if (lane > k) v0[k] = v0[k] / piv;
                    v1[k] = v1[k] / piv;
                    const double l0 = v0[k], l1 = v1[k];
#pragma unroll
                    for (int j = k + 1; j < 16; ++j) {
                        const double u = __shfl(v0[j], k, 64);
                        if (lane > k) v0[j] -= l0 * u;
                        v1[j] -= l1 * u;
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
    for (int c = 0; c < b; ++c)
        for (int r = tid; r < b; r += 256) D[r + (size_t)c * b] = ds[c * ldd + r];
}

hipError_t launch_getrf_dense(const DevPlan &d, int level, int b, hipStream_t s) {
    const size_t lds = (size_t)b * (b | 1) * sizeof(double);
    hipLaunchKernelGGL(k_getrf_dense, dim3(1), dim3(256), lds, s, d.slab, d.levels, level, d.info);
    return hipGetLastError();
}

// ------------------------------------------- compact coupled triangles
// One workgroup per tile row tr of the compact triangles (see LevelDev):
// copies rows [16 tr, 16 tr + 16) of Tu = U_ii[K, K] and Tl = L_ii[K, K]^T
// from the factored diagonal block, then inverts the two diagonal tiles
// (back substitution per column, FP64 divisions by the pivots).
__global__ __launch_bounds__(256) void k_tri_gather(const double *__restrict__ slab, double *__restrict__ tri,
                                                    const LevelDev *__restrict__ levels, int level,
                                                    const int32_t *__restrict__ Kidx) {
    __shared__ double du[16][17], dl[16][17];
    const LevelDev L = levels[level];
    const int kp = L.kp, kap = L.kappa, b = L.b, nt = kp >> 4;
    const int tr = blockIdx.x;
    const double *__restrict__ D = slab + L.offD;
    const int32_t *__restrict__ K = Kidx + L.Koff;
    double *__restrict__ Tu = tri + L.offT;
    double *__restrict__ Tl = Tu + (size_t)kp * kp;
    double *__restrict__ Iu = Tl + (size_t)kp * kp;
    double *__restrict__ Il = Iu + (size_t)nt * 256;
    const int width = kp - 16 * tr;
    for (int e = threadIdx.x; e < 16 * width; e += 256) {
        const int rr = e / width, cc = e - rr * width;
        const int t1 = 16 * tr + rr, t2 = 16 * tr + cc;
        double u, lt;
        if (t1 < kap && t2 < kap) {
            const size_t k1 = (size_t)K[t1], k2 = (size_t)K[t2];
            u = t1 <= t2 ? D[k1 + k2 * b] : 0.0;
            lt = t1 < t2 ? D[k2 + k1 * b] : (t1 == t2 ? 1.0 : 0.0);
        } else {
            u = t1 == t2 ? 1.0 : 0.0;
            lt = u;
        }
        Tu[(size_t)t1 * kp + t2] = u;
        Tl[(size_t)t1 * kp + t2] = lt;
        if (cc < 16) {
            du[rr][cc] = u;
            dl[rr][cc] = lt;
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

hipError_t launch_tri_gather(const DevPlan &d, int level, int kp, hipStream_t s) {
    if (kp <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tri_gather, dim3((unsigned)(kp / 16)), dim3(256), 0, s, d.slab, d.tri, d.levels, level,
                       d.K_idx);
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
                                                     const LevelDev *__restrict__ levels, int level,
                                                     const int32_t *__restrict__ trow_ptr,
                                                     const int32_t *__restrict__ trow_idx) {
    extern __shared__ double xs_lds[];
    const LevelDev L = levels[level];
    const int kp = L.kp, kap = L.kappa, m = L.m, nt = kp >> 4;
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
        for (int e = tid; e < RT * kp; e += 256) {
            const int t = e / RT, r = e - t * RT;
            xs_lds[t * LD + r] = (r < nrow && t < kap) ? X[a0 + r + (size_t)t * m] : 0.0;
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

hipError_t launch_panel_solve(const DevPlan &d, int level, int m, int kp, hipStream_t s) {
    if (m <= 0 || kp <= 0) return hipSuccess;
    const size_t lds32 = (size_t)33 * kp * sizeof(double), lds16 = (size_t)17 * kp * sizeof(double);
    if (lds32 <= 150 * 1024) {
        dim3 grid((unsigned)((m + 31) / 32), 2);
        hipLaunchKernelGGL((k_panel_solve<32, true>), grid, dim3(256), lds32, s, d.slab, d.tri, d.levels, level,
                           d.trow_ptr, d.trow_idx);
    } else if (lds16 <= 150 * 1024) {
        dim3 grid((unsigned)((m + 15) / 16), 2);
        hipLaunchKernelGGL((k_panel_solve<16, true>), grid, dim3(256), lds16, s, d.slab, d.tri, d.levels, level,
                           d.trow_ptr, d.trow_idx);
    } else {
        dim3 grid((unsigned)((m + 15) / 16), 2);
        hipLaunchKernelGGL((k_panel_solve<16, false>), grid, dim3(256), 0, s, d.slab, d.tri, d.levels, level,
                           d.trow_ptr, d.trow_idx);
    }
    return hipGetLastError();
}

// --------------------------------------------------------------------- SSSSM
// Alg. 1 "B_kj <- B_kj - B_ki B_ij" for every target (k, j) of level i: the
// product P_i[a-segment] * Qt_i[b-segment]^T over the coupled index set,
// on FP64 MFMA (v_mfma_f64_16x16x4f64).  One wave computes a 32 x 32 output
// tile as 2 x 2 MFMA blocks and subtracts it from the target through the
// task's row / column maps.  Targets are distinct within a level, so the
// stores never collide.
//
// MFMA f64 16x16x4 operand layout (lane l): A[i][k] with i = l % 16,
// k = l / 16; B[k][j] with j = l % 16, k = l / 16; result element r of lane l
// is D[l / 16 + 4 * r][l % 16] (checked on gfx950 with a lane-layout probe).
__global__ __launch_bounds__(64) void k_ssssm(double *__restrict__ slab, const LevelDev *__restrict__ levels,
                                              int level, const TaskDev *__restrict__ tasks,
                                              const int32_t *__restrict__ maps,
                                              const TileDev *__restrict__ tiles) {
    const LevelDev L = levels[level];
    const TileDev tl = tiles[L.tile_begin + blockIdx.x];
    const TaskDev T = tasks[tl.task];
    const int ti = tl.tij >> 16, tj = tl.tij & 0xffff;
    const double *__restrict__ P = slab + L.offP;
    const double *__restrict__ Q = slab + L.offQ;
    const int m = L.m, kap = L.kappa;
    const int lane = threadIdx.x;
    const int lr = lane & 15, lk = lane >> 4;
    const int ar0 = ti * 32 + lr, ar1 = ar0 + 16;
    const int bc0 = tj * 32 + lr, bc1 = bc0 + 16;
    const bool va0 = ar0 < T.alen, va1 = ar1 < T.alen, vb0 = bc0 < T.blen, vb1 = bc1 < T.blen;
    const double *__restrict__ pa0 = P + T.a0 + ar0;
    const double *__restrict__ pa1 = P + T.a0 + ar1;
    const double *__restrict__ qb0 = Q + T.b0 + bc0;
    const double *__restrict__ qb1 = Q + T.b0 + bc1;
    double4_t c00 = {0, 0, 0, 0}, c01 = c00, c10 = c00, c11 = c00;
    for (int k0 = 0; k0 < kap; k0 += 4) {
        const int k = k0 + lk;
        const bool vk = k < kap;
        const size_t ko = (size_t)k * m;
        const double a0 = (va0 && vk) ? pa0[ko] : 0.0;
        const double a1 = (va1 && vk) ? pa1[ko] : 0.0;
        const double b0 = (vb0 && vk) ? qb0[ko] : 0.0;
        const double b1 = (vb1 && vk) ? qb1[ko] : 0.0;
        c00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, c00, 0, 0, 0);
        c01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, c01, 0, 0, 0);
        c10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, c10, 0, 0, 0);
        c11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, c11, 0, 0, 0);
    }
    const int32_t *__restrict__ rmap = maps + T.rmap;
    const int32_t *__restrict__ cmap = maps + T.cmap;
    double *__restrict__ tgt = slab + T.tgt;
    const double4_t acc[2][2] = {{c00, c01}, {c10, c11}};
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            const int bcol = tj * 32 + bj * 16 + lr;
            if (bcol >= T.blen) continue;
            const int cp = cmap[bcol];
            if (cp < 0) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int a = ti * 32 + bi * 16 + lk + 4 * r;
                if (a >= T.alen) continue;
                const int rp = rmap[a];
                if (rp < 0) continue;
                tgt[(int64_t)rp * T.rs + (int64_t)cp * T.cs] -= acc[bi][bj][r];
            }
        }
    }
}

hipError_t launch_ssssm(const DevPlan &d, int level, int64_t ntiles, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ssssm, dim3((unsigned)ntiles), dim3(64), 0, s, d.slab, d.levels, level, d.tasks, d.maps,
                       d.tiles);
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
    e = hipFuncSetAttribute((const void *)k_getrf, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_trsm_panels, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_fwd_diag, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_bwd_diag, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_getrf_dense, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_panel_solve<32, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_panel_solve<16, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    return e;
}

}  // namespace slu
