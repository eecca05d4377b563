// Host-side analysis for the blocked sparse LU: ordering, symbolic fill,
// diagonal block pointer (Algorithm 2), irregular blocking (Algorithm 3) and
// the storage plan / task lists the device kernels walk.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "slu.h"

namespace slu {

// Storage plan of one block column ("level" i of Algorithm 1).
//
// Rows and columns of block i are [r0, r0 + b).  The diagonal block D_i is
// dense b x b, column-major.  K_i lists the local columns of block i that
// have an entry of S below the block; rows_i lists (sorted, global) the rows
// below the block that have an entry of S in block column i.  Because S is
// symmetric, the U blocks to the right of D_i couple the same index sets.
//   P_i  (m x kappa, column-major, ld = m):  P_i[a, t]  = L(rows_i[a], r0 + K_i[t])
//   Qt_i (m x kappa, column-major, ld = m):  Qt_i[a, t] = U(r0 + K_i[t], rows_i[a])
// Both are followed by zero columns up to kappa rounded to 16.
// rows_i is cut into segments, one per target block row k > i.
//
// The panel solves use compact copies of the coupled triangles in the "tri"
// region at offT (kp = kappa rounded up to 16, nt = kp / 16):
//   Tu  (kp x kp, row-major) = U_ii[K_i, K_i]      upper, identity padding
//   Tl  (kp x kp, row-major) = L_ii[K_i, K_i]^T    unit upper
//   then nt inverted 16 x 16 diagonal tiles of Tu, then nt of Tl.
// trow_ptr[trow + c] .. trow_ptr[trow + c + 1] list the tile columns c' > c
// with a structurally nonzero tile (c, c') of Tu (and so of Tl).
struct LevelDev {
    int64_t offD, offP, offQ;   // slab offsets in doubles
    int64_t offT;               // tri region offset in doubles
    int64_t offW;               // tiled GETRF work region offset in doubles (-1: none)
    int64_t offB;               // blocked panel solve: inverted diagonal blocks (-1: none)
    int64_t Koff, Roff;         // offsets into K_idx / R_idx
    int64_t task_begin, task_end;   // segment pairs (SSSSM targets) in stgt, sa-major
    int64_t moff;                   // SSSSM offset tables in maps
    int32_t r0, b, kappa, m;
    int32_t chunk_begin, chunk_end;
    int32_t seg_begin, seg_end;
    int32_t lds_getrf;          // dynamic LDS bytes for GETRF
    int32_t kp;                 // kappa rounded up to a multiple of 16
    int32_t trow;               // offset into trow_ptr
    int32_t pad;                // chunked GETRF: largest coupled-row count of a chunk
    int32_t sch_begin, sch_end; // triangular-solve chunks in schunks
    int32_t sb_begin, sb_end;   // solve batch records (sbatch pairs), end = sentinel
    int64_t sitem;              // first solve item of the level in sitems
    // Schur-update tile rows (at its round's tile edge) that cover every
    // coupled row of the next wave's blocks: the tiles in those rows or
    // columns update the next wave; the others only later waves
    int32_t sscrit, pad2;
};

// One column chunk of the right-looking GETRF of D_i: local columns
// [c0, c0 + w) and the local rows >= c0 + w of the block coupled to them.
struct ChunkDev {
    int32_t c0, w, nr, pad;
    int64_t roff;               // offset into chunk_rows
};

// Levels that run together: equal height in the block dependency tree
// (parent of block i = the first block below it coupled to it).  Launch
// parameters are the maxima over the wave's levels.
// Levels of one wave whose SSSSM targets are disjoint, launched together.
struct RoundInfo {
    int32_t begin, end;         // range in round_levels
    int64_t tiles;              // SSSSM workgroups of the round
    int64_t tiles_c, tiles_r;   // of which update the next wave / only later waves
    int64_t tiles_d, tiles_pq;  // the next-wave tiles: the square of its first rows
                                // (its diagonal blocks) / the two bands beside it
    int32_t tile, pad;          // tile edge (64, or 32 when every level is small)
};

struct WaveInfo {
    int32_t begin, end;         // range in wave_levels
    int32_t lds_getrf;          // dynamic LDS bytes of the GETRF launch
    int32_t max_nt;             // largest kp / 16
    int32_t tslots;             // triangle tiles read by the wave's panel solves (all levels)
    int32_t max_m;              // largest panel row count
    int32_t max_kp;             // largest kp
    int32_t any_dense, any_chunked;
    int32_t max_b;              // largest diagonal block
    int32_t min_b;              // smallest diagonal block
    int32_t min_dense_pct = 100; // least share (%) of a block's lower triangle in S, blocks of 33+ rows
    int32_t round_begin, round_end;
};

struct Segment {
    int32_t blk, start, len;
};

struct Analysis {
    int64_t n = 0, nnz_a = 0;
    slu_options opt{};
    std::vector<int64_t> a_rowptr;
    std::vector<int32_t> a_colidx;
    std::vector<int32_t> perm, iperm;
    std::vector<int64_t> s_colptr;   // lower CSC of S, diagonal first
    std::vector<int32_t> s_rowidx;
    std::vector<int64_t> blockptr;   // Algorithm 2, n + 1
    std::vector<int64_t> bptr;       // block boundaries, p + 1
    int64_t p = 0;
    std::vector<int32_t> bid;        // block of every (permuted) row

    std::vector<LevelDev> levels;
    std::vector<int32_t> K_idx;      // local columns, concatenated per level
    std::vector<int32_t> R_idx;      // global rows, concatenated per level
    std::vector<Segment> segs;
    std::vector<ChunkDev> chunks;
    std::vector<int32_t> chunk_rows; // local rows
    // Triangular solves inside D_i walk column chunks of at most 16 columns
    // (the GETRF chunks of a chunked block; 16-column chunks coupled to all
    // later rows of a dense block).  ChunkDev.pad holds the chunk's first item
    // within its level; rows come from chunk_rows.  Item t of a chunk is its
    // panel row t (t < w: chunk row c0 + t, else coupled row t - w), stored
    // as (block-local row, c0 << 5 | w) in sitems.
    std::vector<ChunkDev> schunks;
    std::vector<int32_t> sitems;
    int32_t max_solve_items = 0;     // largest w + nr of a solve chunk
    // Solve chunks are staged through LDS in batches of consecutive chunks
    // holding at most kSolveItems items and kSolveBatchChunks chunks; per
    // level, sbatch holds (first chunk, first item) pairs of its batches and
    // a closing (sch_end, item count) pair.
    std::vector<int32_t> sbatch;
    std::vector<int32_t> R_seg;      // segment (local index) of every row of R_idx
    std::vector<int64_t> stgt;       // SSSSM target base offset per segment pair
    std::vector<int32_t> maps;       // SSSSM row / column offset tables
    std::vector<WaveInfo> waves;
    std::vector<int32_t> wave_levels;
    std::vector<RoundInfo> rounds;
    std::vector<int32_t> round_levels;   // levels of every round, consecutive
    // first SSSSM workgroup of each level within its round, five per level:
    // counting all its tiles, the tiles that update the next wave, the rest,
    // the next wave's square and its two bands (see k_ssssm)
    std::vector<int64_t> round_tiles;
    std::vector<int32_t> tslot_off;      // per wave_levels entry: first triangle-gather workgroup of the level in its wave
    std::vector<int32_t> trow_ptr;   // nonzero tile lists of the coupled triangles
    std::vector<int32_t> trow_idx;
    int64_t tri_doubles = 0;
    int64_t tgetrf_doubles = 0;      // tiled GETRF work region (panel copies, tile inverses)
    int64_t binv_doubles = 0;        // blocked panel solve: inverted diagonal blocks
    std::vector<int64_t> slot;       // A entry (CSR order) -> slab position
    std::vector<int32_t> posK;       // global column -> position in K of its block, or -1

    int64_t slab_doubles = 0;
    int64_t nonempty_blocks = 0;
    double flops = 0.0;
    double flops_getrf = 0.0, flops_panel = 0.0, flops_ssssm = 0.0;
    double stored_flops = 0.0;
    int32_t max_block = 0;
    int32_t max_gemm_k = 0;
};

// Tile edge of the SSSSM output tiles (one workgroup each), and the level
// size below which a round uses 32 x 32 tiles.
constexpr int kSsssmTile = 64;
constexpr int kSsssmSmallM = 1200;
// LDS staging of the triangular solves: items (panel rows) and chunks per batch.
constexpr int kSolveItems = 512;
constexpr int kSolveBatchChunks = 64;
constexpr int kSolveCont = 1 << 8;   // solve chunk continuing the previous one's coupled rows
// Blocked panel solve: levels whose coupled triangles have at least
// kPanelBlkKp columns solve their panels in column blocks of kPanelBlk with
// the blocks' inverted diagonal triangles (chip-wide products).
constexpr int kPanelBlk = 128;
constexpr int kPanelBlkKp = 256;
// Largest diagonal block factored in one LDS-resident chunk.
constexpr int kLdsDenseMax = 128;
// LDS budget of the chunked GETRF (bytes).
constexpr int kGetrfLdsBudget = 150 * 1024;
// Tiled GETRF: per level with b > 16 rows, two panel copies (a tile column
// and a tile row of the diagonal block, 64 b doubles for 32-wide tiles) and
// the inverted L and U of every 32 x 32 diagonal tile (2048 doubles per
// tile, kept for the tiled solves); the 16-wide tiles use the first
// 64 b + 1024 doubles.
inline int64_t tgetrf_level_doubles(int32_t b) {
    return b > 16 ? 128 * (int64_t)b + 2048 * (int64_t)((b + 31) / 32) : 0;
}

// Returns SLU_OK or an SLU_ERR_* code; fills *out.
// segments (optional): ascending row offsets 0 = s_0 < s_1 < ... < s_k = n of
// independent systems stacked block-diagonally; the blocking is then
// computed on every system's own range (blocks never cross a boundary).
int analyze(int64_t n, const int64_t *rowptr, const int32_t *colidx, const slu_options &opt,
            Analysis *out, const std::vector<int64_t> *segments = nullptr);

// Geometric nested dissection of an nx x ny x nz grid (new -> old).
void nd_grid_order(int32_t nx, int32_t ny, int32_t nz, std::vector<int32_t> *perm);

// Graph nested dissection of the pattern of A + A^T (new -> old): dense
// vertices last, connected components apart, level-structure cuts with
// minimum vertex covers as separators (nd_graph.cpp).
void nd_graph_order(int64_t n, const int64_t *rowptr, const int32_t *colidx, std::vector<int32_t> *perm);

// Host threads of the analysis' parallel parts (0: hardware count, at most 16).
void set_host_threads(int threads);

// Algorithm 3 with the exact-integer readings of the sampling.
void irregular_blocking(const std::vector<int64_t> &blockptr, int sample_points, int step,
                        int max_num, int advance, std::vector<int64_t> *ptr);

}  // namespace slu
