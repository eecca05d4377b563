// Launch helpers for the gfx950 kernels of the blocked sparse LU.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "analyze.hpp"

namespace slu {

// Device view of the uploaded structure (all pointers inside the workspace).
struct DevPlan {
    double *slab;
    double *tri;                // compact coupled triangles (see LevelDev)
    double *tgetrf;             // tiled GETRF panel copies and inverted tiles (LevelDev.offW)
    double *binv;               // blocked panel solve: inverted diagonal blocks (LevelDev.offB)
    const int32_t *trow_ptr;
    const int32_t *trow_idx;
    const LevelDev *levels;
    const int32_t *K_idx;
    const int32_t *R_idx;
    const ChunkDev *chunks;
    const int32_t *chunk_rows;
    const ChunkDev *schunks;    // triangular-solve chunks
    const int32_t *sitems;
    const int32_t *sbatch;
    const int32_t *rseg;        // segment of every row of R_idx
    const int64_t *stgt;        // SSSSM target base per segment pair
    const int32_t *maps;        // SSSSM row / column offset tables
    const int64_t *slot;
    const int64_t *a_rowptr;
    const int32_t *a_colidx;
    const int64_t *at_colptr;   // CSC of A: column pointers
    const int32_t *at_rowidx;   // CSC of A: row of every entry
    const int64_t *at_vidx;     // CSC of A: index of the entry in CSR order
    const int32_t *perm;
    const int32_t *wave_levels; // levels of every wave, consecutive
    const int32_t *round_levels;
    const int64_t *round_tiles;
    const int32_t *tslot_off;   // first triangle-gather workgroup of every level in its wave
    unsigned long long *info;   // [0] smallest failed pivot column (or ~0)
    double *scratch;            // n * kSolveCols doubles
    double *ir;                 // 2 * n * kSolveCols doubles: refinement residual and correction
    unsigned long long *norms;  // 4 * kSolveCols (non-negative doubles as bits)
    int64_t n, nnz_a, slab_doubles;
};

constexpr int kSolveCols = 16;
// Fixed device scratch of slu_solve_noalloc (doubles; 32 MiB), and the
// device ordinals it is kept for.
constexpr size_t kStaticScratchDoubles = (size_t)4 << 20;
constexpr int kMaxDevices = 64;
// Address of the current device's fixed scratch (looked up once per device).
hipError_t static_scratch(double **ptr);

hipError_t setup_kernel_attributes();
hipError_t launch_residual(const DevPlan &d, const double *values, const double *B, int64_t ldb, const double *X,
                           int64_t ldx, double *R, int64_t ldr, int nc, hipStream_t s);
hipError_t launch_axpy(const DevPlan &d, double *X, int64_t ldx, const double *Dv, int64_t ldd, int nc,
                       hipStream_t s);
hipError_t launch_value_gradient(const DevPlan &d, const double *G, const double *X, int64_t nrhs, int64_t ld,
                                 double *grad, hipStream_t s);

hipError_t launch_zero(double *p, int64_t count, hipStream_t s);
hipError_t launch_scatter(const DevPlan &d, const double *values, hipStream_t s);
hipError_t launch_info_reset(const DevPlan &d, hipStream_t s);
hipError_t launch_getrf_wave(const DevPlan &d, const int32_t *lvl, int nlev, int lds_bytes, hipStream_t s);
// Split GETRF of a wave, step k: the chunk-k panel of every level, then the
// chunk-k trailing tiles (max_tiles: the most over the wave's levels).
hipError_t launch_getrf_step(const DevPlan &d, const int32_t *lvl, int nlev, int k, int lds_bytes, hipStream_t s);
hipError_t launch_getrf_trail(const DevPlan &d, const int32_t *lvl, int nlev, int k, int max_tiles, hipStream_t s);
// Tiled GETRF of a wave, tile step s (0 <= s < max_nt, the largest number of
// 16-row tiles of the wave's diagonal blocks).
hipError_t launch_getrf_tile(const DevPlan &d, const int32_t *lvl, int nlev, int s, int max_nt, hipStream_t st);
// The same with 32 x 32 tiles (max_nt in 32-row tiles); one: the host copy
// of the level's record when the wave has a single level (else null).
hipError_t launch_getrf_tile32(const DevPlan &d, const int32_t *lvl, int nlev, int s, int max_nt,
                               const LevelDev *one, hipStream_t st);
// soff: first workgroup of each of the wave's levels; slots: their total.
hipError_t launch_tri_gather_wave(const DevPlan &d, const int32_t *lvl, const int32_t *soff, int nlev, int slots,
                                  hipStream_t s);
// skip_blocked: leave out the levels that take the blocked panel solve.
hipError_t launch_panel_solve_wave(const DevPlan &d, const int32_t *lvl, int nlev, int max_m, int max_kp,
                                   int skip_blocked, hipStream_t s);
// Blocked panel solve of the wave's levels with kp >= kPanelBlkKp: the
// inverted diagonal blocks, then one launch per column block.
hipError_t launch_panel_blk_wave(const DevPlan &d, const int32_t *lvl, int nlev, int max_m, int max_kp,
                                 hipStream_t s);
// mode: 0 all tiles of the round's levels, 1 those that update the next
// wave, 2 the rest, 3 / 4 the next wave's diagonal square / panel bands (see
// k_ssssm); max_groups > 0 (a multiple of 8) caps the workgroups, which then
// walk the tiles.
hipError_t launch_ssssm_round(const DevPlan &d, const RoundInfo &r, bool f32, int mode, int max_groups,
                              hipStream_t s);

// Solve pieces on the permuted work block W (n x nc, leading dimension n).
hipError_t launch_gather_perm(const DevPlan &d, const double *B, int64_t ld, int nc, hipStream_t s);
hipError_t launch_scatter_perm(const DevPlan &d, double *X, int64_t ld, int nc, hipStream_t s);
// LDS bytes of a diagonal-solve launch over blocks of at most max_b rows.
size_t solve_diag_lds_bytes(int max_b, int nc);
hipError_t launch_solve_diag_wave(const DevPlan &d, const int32_t *lvl, int nlev, int max_b, bool fwd, int nc,
                                  int trans, hipStream_t s);
// Tiled diagonal solves of a wave factored by the 32 x 32 tiled GETRF (its
// inverted diagonal tiles kept): one launch per tile step, max_b + 31 / 32 + 1.
hipError_t launch_solve_tile_wave(const DevPlan &d, const int32_t *lvl, int nlev, int max_b, bool fwd, int nc,
                                  int trans, const LevelDev *one, hipStream_t s);
// Forward updates of the nlev levels in lvl (levels whose target rows are
// disjoint: one Schur-update round); max_m is their largest m.
hipError_t launch_fwd_update(const DevPlan &d, const int32_t *lvl, int nlev, int max_m, int nc, int trans,
                             hipStream_t s);
// Backward updates of the nlev levels in lvl (one wave: each writes only its
// own block's rows); max_kappa is their largest kappa.
hipError_t launch_bwd_update(const DevPlan &d, const int32_t *lvl, int nlev, int max_kappa, int nc, int trans,
                             hipStream_t s);

// Backward-error pieces: norms[0..nc) = ||r||, [16..) = ||x||, [32..) = ||b||, [48] = ||op(A)||.
hipError_t launch_residual_norms(const DevPlan &d, const double *values, const double *B,
                                 const double *X, int64_t ld, int nc, int trans, hipStream_t s);

}  // namespace slu
