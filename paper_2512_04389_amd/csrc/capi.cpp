// C ABI of the blocked sparse LU (declared in include/slu.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "analyze.hpp"
#include "kernels.hpp"
#include "slu.h"

struct slu_handle {
    slu::Analysis an;
    size_t ws_bytes = 0;
    void *ws = nullptr;
    slu::DevPlan dev{};
    // byte offsets of the workspace regions
    size_t o_slab, o_tri, o_tgetrf, o_binv, o_trow_ptr, o_trow_idx, o_levels, o_K, o_R, o_chunks, o_crows, o_schunks, o_sitems, o_sbatch, o_rseg, o_stgt, o_maps, o_slot, o_arow, o_acol,
        o_atcol, o_atrow, o_atv, o_perm, o_wlev, o_rlev, o_rtile, o_tsoff, o_info, o_scratch, o_ir, o_norms, o_vals;
    std::vector<int64_t> at_colptr;
    std::vector<int32_t> at_rowidx;
    std::vector<int64_t> at_vidx;
    bool profiling = false;
    std::vector<hipEvent_t> ev;          // event pool for per-kernel timing
    std::vector<int> ev_kind;            // kernel class of each recorded pair
    std::vector<int64_t> ev_count;       // launches inside each recorded pair
    double kern_ms[SLU_NUM_KERNELS] = {0, 0, 0, 0};
    int64_t kern_n[SLU_NUM_KERNELS] = {0, 0, 0, 0};
    bool bound = false;
    bool factored = false;
    int64_t zero_pivot_col = -1;
    int solve_cols = slu::kSolveCols;
    int precision = SLU_PRECISION_FP64;
    // graph mode: the factor's launch sequence captured once, replayed
    bool use_graph = false;
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_stream = nullptr;
    int graph_precision = -1;
    // waves whose chunked diagonal blocks reach this trailing work (sum over
    // a block's chunks of nr^2) take the split GETRF
    double getrf_split_work = 2e5;
    // waves whose largest diagonal block has at least this many rows take
    // the tiled GETRF (0: none)
    int getrf_tiled_rows = 1;
    int getrf_tile = 32;        // tile edge of the tiled GETRF (16 or 32)
    bool panel_blocked = true;  // blocked panel solve for wide coupled triangles
    // diagonal solves of waves whose largest block has at least this many
    // rows use the tiled solve when their blocks were factored by the 32 x 32
    // tiled GETRF (0: never); wave_tinv: per wave, the last factor kept the
    // inverted diagonal tiles
    int solve_tiled_rows = 64;
    int solve_tiled_sparse_rows = 64;   // ... and, for blocks under half dense, at least this many
    std::vector<char> wave_tinv;
    // Schur updates of a wave (of one round) that reach only later waves run
    // on a second stream (default priority) while the next wave factors its
    // diagonal blocks and panels; the updates of the next wave's blocks stay
    // on the factor's stream.  Events: this wave's updates of the next wave
    // are done / the second stream's updates so far are done.
    bool lookahead = false;
    int la_groups = 512;        // workgroups of a deferred update launch (0: one per tile)
    hipStream_t la_stream = nullptr;
    hipEvent_t ev_panel = nullptr, ev_rest = nullptr, ev_pq = nullptr;
};

namespace {

// Code of the last failed HIP call on this thread (slu_last_hip_error).
thread_local int t_last_hip = 0;

bool hip_failed(hipError_t e) {
    if (e == hipSuccess) return false;
    t_last_hip = (int)e;
    return true;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

void plan_workspace(slu_handle *h) {
    const slu::Analysis &an = h->an;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    h->o_slab = take((size_t)an.slab_doubles * 8);
    h->o_tri = take((size_t)an.tri_doubles * 8);
    h->o_tgetrf = take((size_t)an.tgetrf_doubles * 8);
    h->o_binv = take((size_t)an.binv_doubles * 8);
    h->o_trow_ptr = take(an.trow_ptr.size() * 4);
    h->o_trow_idx = take(an.trow_idx.size() * 4);
    h->o_levels = take(an.levels.size() * sizeof(slu::LevelDev));
    h->o_K = take(an.K_idx.size() * 4);
    h->o_R = take(an.R_idx.size() * 4);
    h->o_chunks = take(an.chunks.size() * sizeof(slu::ChunkDev));
    h->o_crows = take(an.chunk_rows.size() * 4);
    h->o_schunks = take(an.schunks.size() * sizeof(slu::ChunkDev));
    h->o_sitems = take(an.sitems.size() * 4);
    h->o_sbatch = take(an.sbatch.size() * 4);
    h->o_rseg = take(an.R_seg.size() * 4);
    h->o_stgt = take(an.stgt.size() * 8);
    h->o_maps = take(an.maps.size() * 4);
    h->o_slot = take(an.slot.size() * 8);
    h->o_arow = take(an.a_rowptr.size() * 8);
    h->o_acol = take(an.a_colidx.size() * 4);
    h->o_atcol = take(h->at_colptr.size() * 8);
    h->o_atrow = take(h->at_rowidx.size() * 4);
    h->o_atv = take(h->at_vidx.size() * 8);
    h->o_perm = take(an.perm.size() * 4);
    h->o_wlev = take(an.wave_levels.size() * 4);
    h->o_rlev = take(an.round_levels.size() * 4);
    h->o_rtile = take(an.round_tiles.size() * 8);
    h->o_tsoff = take(an.tslot_off.size() * 4);
    h->o_info = take(64);
    h->o_scratch = take((size_t)an.n * slu::kSolveCols * 8);
    h->o_ir = take((size_t)2 * an.n * slu::kSolveCols * 8);
    h->o_norms = take(64 * 8);
    h->o_vals = take((size_t)an.nnz_a * 8);    // staged values of a graph replay
    h->ws_bytes = o;
}

void build_transpose(slu_handle *h) {
    const slu::Analysis &an = h->an;
    const int64_t n = an.n, nnz = an.nnz_a;
    h->at_colptr.assign(n + 1, 0);
    for (int64_t q = 0; q < nnz; ++q) h->at_colptr[an.a_colidx[q] + 1] += 1;
    for (int64_t j = 0; j < n; ++j) h->at_colptr[j + 1] += h->at_colptr[j];
    h->at_rowidx.assign(nnz, 0);
    h->at_vidx.assign(nnz, 0);
    std::vector<int64_t> fill(h->at_colptr.begin(), h->at_colptr.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t q = an.a_rowptr[i]; q < an.a_rowptr[i + 1]; ++q) {
            const int64_t at = fill[an.a_colidx[q]]++;
            h->at_rowidx[at] = (int32_t)i;
            h->at_vidx[at] = q;
        }
}

template <class T>
hipError_t upload(void *base, size_t off, const std::vector<T> &v, hipStream_t s) {
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync((char *)base + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

// The diagonal solves of wave wi take the tiled solve: its blocks were
// factored by the 32 x 32 tiled GETRF (the inverted diagonal tiles are kept),
// every block has a tiled work region, the wave's largest block reaches the
// threshold and its blocks are dense (at least half of every block's lower
// triangle in S) or all reach the sparse-block threshold (the one-workgroup
// solve walks only the coupled rows of a sparse block, and wins only on small
// ones).
bool tiled_solve(const slu_handle *h, size_t wi) {
    const slu::WaveInfo &w = h->an.waves[wi];
    // dense blocks, or blocks large enough (min_sparse_rows) that the
    // one-workgroup walk of their column chunks, a chain of b / 16 steps,
    // takes longer than the b / 64 (rounded up) chip-wide tile-pair steps
    // whatever their density
    const bool worth = w.min_dense_pct >= 50 || w.min_b >= h->solve_tiled_sparse_rows;
    return h->solve_tiled_rows > 0 && wi < h->wave_tinv.size() && h->wave_tinv[wi] && w.min_b > 16 &&
           w.max_b >= h->solve_tiled_rows && worth && w.end - w.begin <= 65535;
}

int solve_check(const slu_handle *h, const double *B, const double *X, int64_t nrhs, int64_t ld) {
    if (!h || (!B && nrhs > 0) || (!X && nrhs > 0) || nrhs < 0) return SLU_ERR_ARG;
    if (!h->bound) return SLU_ERR_STATE;
    if (!h->factored) return SLU_ERR_NOT_FACTORED;
    if (ld < h->an.n || ld < 1) return SLU_ERR_ARG;
    return SLU_OK;
}

// The solve sweeps on the permuted work block d.scratch (n x cols doubles),
// cols right-hand sides at a time.
int solve_sweeps(slu_handle *h, const slu::DevPlan &d, int cols, const double *B, double *X, int64_t nrhs,
                 int64_t ld, int trans, hipStream_t s) {
    const slu::Analysis &an = h->an;
    for (int64_t c0 = 0; c0 < nrhs; c0 += cols) {
        const int nc = (int)std::min<int64_t>(cols, nrhs - c0);
        hipError_t e = slu::launch_gather_perm(d, B + c0 * ld, ld, nc, s);
        if (hip_failed(e)) return SLU_ERR_HIP;
        // forward sweep wave by wave: the diagonal solves of a wave's levels
        // together, then their updates of later rows one Schur-update round
        // at a time (a round's levels have disjoint target rows, and every
        // row takes its updates in round order, so the sums are
        // deterministic); the backward sweep mirrors it, with the updates of
        // a whole wave together (each level writes only its own block)
        for (size_t wi = 0; wi < an.waves.size(); ++wi) {
            const slu::WaveInfo &w = an.waves[wi];
            const int nlev = w.end - w.begin;
            if (tiled_solve(h, wi)) {
                const slu::LevelDev *one = nlev == 1 ? &an.levels[an.wave_levels[w.begin]] : nullptr;
                if (hip_failed(
                        slu::launch_solve_tile_wave(d, d.wave_levels + w.begin, nlev, w.max_b, true, nc, trans, one, s)))
                    return SLU_ERR_HIP;
            } else if (hip_failed(slu::launch_solve_diag_wave(d, d.wave_levels + w.begin, nlev, w.max_b, true, nc, trans,
                                                              s))) {
                return SLU_ERR_HIP;
            }
            for (int r = w.round_begin; r < w.round_end; ++r) {
                const slu::RoundInfo &ri = an.rounds[r];
                int max_m = 0;
                for (int q = ri.begin; q < ri.end; ++q) max_m = std::max(max_m, an.levels[an.round_levels[q]].m);
                if (hip_failed(slu::launch_fwd_update(d, d.round_levels + ri.begin, ri.end - ri.begin, max_m, nc,
                                                      trans, s)))
                    return SLU_ERR_HIP;
            }
        }
        for (size_t wi = an.waves.size(); wi-- > 0;) {
            const slu::WaveInfo &w = an.waves[wi];
            const int nlev = w.end - w.begin;
            int max_kappa = 0;
            for (int q = w.begin; q < w.end; ++q) {
                const slu::LevelDev &L = an.levels[an.wave_levels[q]];
                if (L.m > 0) max_kappa = std::max(max_kappa, L.kappa);
            }
            if (hip_failed(slu::launch_bwd_update(d, d.wave_levels + w.begin, nlev, max_kappa, nc, trans, s)))
                return SLU_ERR_HIP;
            if (tiled_solve(h, wi)) {
                if (hip_failed(
                        slu::launch_solve_tile_wave(d, d.wave_levels + w.begin, nlev, w.max_b, false, nc, trans,
                                                    nlev == 1 ? &an.levels[an.wave_levels[w.begin]] : nullptr, s)))
                    return SLU_ERR_HIP;
            } else if (hip_failed(slu::launch_solve_diag_wave(d, d.wave_levels + w.begin, nlev, w.max_b, false, nc,
                                                              trans, s))) {
                return SLU_ERR_HIP;
            }
        }
        e = slu::launch_scatter_perm(d, X + c0 * ld, ld, nc, s);
        if (hip_failed(e)) return SLU_ERR_HIP;
    }
    return SLU_OK;
}

int solve_impl(slu_handle *h, const double *B, double *X, int64_t nrhs, int64_t ld, int trans, hipStream_t s) {
    const int rc = solve_check(h, B, X, nrhs, ld);
    if (rc != SLU_OK) return rc;
    return solve_sweeps(h, h->dev, h->solve_cols, B, X, nrhs, ld, trans, s);
}

}  // namespace

extern "C" {

void slu_default_options(slu_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->sample_points = 1000;
    opt->step = 2;
    opt->max_num = 3;
    opt->advance = 1;
    opt->blocking = SLU_BLOCK_IRREGULAR;
    opt->regular_block = 0;
    opt->ordering = SLU_ORDER_NATURAL;
    opt->user_perm = nullptr;
}

}  // extern "C"

namespace {

int analyze_into(int64_t n, const int64_t *rowptr, const int32_t *colidx, const slu_options &o,
                 const std::vector<int64_t> *segments, slu_handle **out) {
    slu_handle *h = new (std::nothrow) slu_handle();
    if (!h) return SLU_ERR_NOMEM;
    int rc;
    try {
        rc = slu::analyze(n, rowptr, colidx, o, &h->an, segments);
        if (rc == SLU_OK) {
            build_transpose(h);
            // the diagonal sweeps of the solve hold b x nc doubles in LDS
            // next to the staged chunk panels
            const int mb = std::max<int32_t>(h->an.max_block, 1);
            h->solve_cols = 0;
            for (int nc = slu::kSolveCols; nc >= 1; --nc)
                if (slu::solve_diag_lds_bytes(mb, nc) <= 160 * 1024) {
                    h->solve_cols = nc;
                    break;
                }
            if (h->solve_cols < 1) rc = SLU_ERR_LIMIT;
            plan_workspace(h);
        }
    } catch (const std::bad_alloc &) {
        rc = SLU_ERR_NOMEM;
    }
    if (rc != SLU_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return SLU_OK;
}

}  // namespace

extern "C" {

int slu_analyze(int64_t n, const int64_t *rowptr, const int32_t *colidx, const slu_options *opt,
                slu_handle **out) {
    if (!out) return SLU_ERR_ARG;
    *out = nullptr;
    slu_options o;
    if (opt)
        o = *opt;
    else
        slu_default_options(&o);
    return analyze_into(n, rowptr, colidx, o, nullptr, out);
}

int slu_analyze_batch(int64_t nsys, const int64_t *n, const int64_t *const *rowptr, const int32_t *const *colidx,
                      const int32_t *grid_dims, const slu_options *opt, slu_handle **out) {
    if (!out) return SLU_ERR_ARG;
    *out = nullptr;
    if (nsys < 1 || !n || !rowptr || !colidx) return SLU_ERR_ARG;
    slu_options o;
    if (opt)
        o = *opt;
    else
        slu_default_options(&o);
    if (o.ordering != SLU_ORDER_NATURAL && o.ordering != SLU_ORDER_GRID_ND && o.ordering != SLU_ORDER_GRAPH_ND)
        return SLU_ERR_ARG;
    if (o.ordering == SLU_ORDER_GRID_ND && !grid_dims) return SLU_ERR_ARG;
    try {
        std::vector<int64_t> seg(1, 0), rp(1, 0);
        std::vector<int32_t> ci, perm, p1;
        for (int64_t q = 0; q < nsys; ++q) {
            const int64_t ns = n[q], off = seg.back();
            if (ns < 1 || !rowptr[q] || !colidx[q] || off + ns >= ((int64_t)1 << 31) - 1) return SLU_ERR_ARG;
            const int64_t *r = rowptr[q];
            if (r[0] != 0) return SLU_ERR_ROWPTR;
            for (int64_t i = 0; i < ns; ++i) {
                if (r[i + 1] < r[i]) return SLU_ERR_ROWPTR;
                for (int64_t e = r[i]; e < r[i + 1]; ++e) {
                    const int32_t c = colidx[q][e];
                    if (c < 0 || c >= ns) return SLU_ERR_COLIDX;
                    ci.push_back((int32_t)(c + off));
                }
                rp.push_back((int64_t)ci.size());
            }
            if (o.ordering == SLU_ORDER_GRID_ND) {
                const int32_t *g = grid_dims + 3 * q;
                if (g[0] < 1 || g[1] < 1 || g[2] < 1 || (int64_t)g[0] * g[1] * g[2] != ns) return SLU_ERR_ARG;
                slu::nd_grid_order(g[0], g[1], g[2], &p1);
            } else if (o.ordering == SLU_ORDER_GRAPH_ND) {
                slu::nd_graph_order(ns, rowptr[q], colidx[q], &p1);
            } else {
                p1.resize(ns);
                for (int64_t i = 0; i < ns; ++i) p1[i] = (int32_t)i;
            }
            for (int32_t v : p1) perm.push_back((int32_t)(v + off));
            seg.push_back(off + ns);
        }
        o.ordering = SLU_ORDER_USER;
        o.user_perm = perm.data();
        return analyze_into(seg.back(), rp.data(), ci.data(), o, &seg, out);
    } catch (const std::bad_alloc &) {
        return SLU_ERR_NOMEM;
    }
}

int slu_workspace_size(const slu_handle *h, size_t *bytes) {
    if (!h || !bytes) return SLU_ERR_ARG;
    *bytes = h->ws_bytes;
    return SLU_OK;
}

int slu_bind_workspace(slu_handle *h, void *device_ptr, size_t bytes, void *stream) {
    if (!h || !device_ptr) return SLU_ERR_ARG;
    if (bytes < h->ws_bytes || ((uintptr_t)device_ptr & 255) != 0) return SLU_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (hip_failed(slu::setup_kernel_attributes())) return SLU_ERR_HIP;
    char *base = (char *)device_ptr;
    const slu::Analysis &an = h->an;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = upload(base, h->o_levels, an.levels, s);
    if (e == hipSuccess) e = upload(base, h->o_trow_ptr, an.trow_ptr, s);
    if (e == hipSuccess) e = upload(base, h->o_trow_idx, an.trow_idx, s);
    if (e == hipSuccess) e = upload(base, h->o_K, an.K_idx, s);
    if (e == hipSuccess) e = upload(base, h->o_R, an.R_idx, s);
    if (e == hipSuccess) e = upload(base, h->o_chunks, an.chunks, s);
    if (e == hipSuccess) e = upload(base, h->o_crows, an.chunk_rows, s);
    if (e == hipSuccess) e = upload(base, h->o_schunks, an.schunks, s);
    if (e == hipSuccess) e = upload(base, h->o_sitems, an.sitems, s);
    if (e == hipSuccess) e = upload(base, h->o_sbatch, an.sbatch, s);
    if (e == hipSuccess) e = upload(base, h->o_rseg, an.R_seg, s);
    if (e == hipSuccess) e = upload(base, h->o_stgt, an.stgt, s);
    if (e == hipSuccess) e = upload(base, h->o_maps, an.maps, s);
    if (e == hipSuccess) e = upload(base, h->o_slot, an.slot, s);
    if (e == hipSuccess) e = upload(base, h->o_arow, an.a_rowptr, s);
    if (e == hipSuccess) e = upload(base, h->o_acol, an.a_colidx, s);
    if (e == hipSuccess) e = upload(base, h->o_atcol, h->at_colptr, s);
    if (e == hipSuccess) e = upload(base, h->o_atrow, h->at_rowidx, s);
    if (e == hipSuccess) e = upload(base, h->o_atv, h->at_vidx, s);
    if (e == hipSuccess) e = upload(base, h->o_perm, an.perm, s);
    if (e == hipSuccess) e = upload(base, h->o_wlev, an.wave_levels, s);
    if (e == hipSuccess) e = upload(base, h->o_rlev, an.round_levels, s);
    if (e == hipSuccess) e = upload(base, h->o_rtile, an.round_tiles, s);
    if (e == hipSuccess) e = upload(base, h->o_tsoff, an.tslot_off, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (hip_failed(e)) return SLU_ERR_HIP;
    slu::DevPlan &d = h->dev;
    d.slab = (double *)(base + h->o_slab);
    d.tri = (double *)(base + h->o_tri);
    d.tgetrf = an.tgetrf_doubles > 0 ? (double *)(base + h->o_tgetrf) : nullptr;
    d.binv = an.binv_doubles > 0 ? (double *)(base + h->o_binv) : nullptr;
    d.trow_ptr = (const int32_t *)(base + h->o_trow_ptr);
    d.trow_idx = (const int32_t *)(base + h->o_trow_idx);
    d.levels = (const slu::LevelDev *)(base + h->o_levels);
    d.K_idx = (const int32_t *)(base + h->o_K);
    d.R_idx = (const int32_t *)(base + h->o_R);
    d.chunks = (const slu::ChunkDev *)(base + h->o_chunks);
    d.chunk_rows = (const int32_t *)(base + h->o_crows);
    d.schunks = (const slu::ChunkDev *)(base + h->o_schunks);
    d.sitems = (const int32_t *)(base + h->o_sitems);
    d.sbatch = (const int32_t *)(base + h->o_sbatch);
    d.rseg = (const int32_t *)(base + h->o_rseg);
    d.stgt = (const int64_t *)(base + h->o_stgt);
    d.maps = (const int32_t *)(base + h->o_maps);
    d.slot = (const int64_t *)(base + h->o_slot);
    d.a_rowptr = (const int64_t *)(base + h->o_arow);
    d.a_colidx = (const int32_t *)(base + h->o_acol);
    d.at_colptr = (const int64_t *)(base + h->o_atcol);
    d.at_rowidx = (const int32_t *)(base + h->o_atrow);
    d.at_vidx = (const int64_t *)(base + h->o_atv);
    d.perm = (const int32_t *)(base + h->o_perm);
    d.wave_levels = (const int32_t *)(base + h->o_wlev);
    d.round_levels = (const int32_t *)(base + h->o_rlev);
    d.round_tiles = (const int64_t *)(base + h->o_rtile);
    d.tslot_off = (const int32_t *)(base + h->o_tsoff);
    d.info = (unsigned long long *)(base + h->o_info);
    d.scratch = (double *)(base + h->o_scratch);
    d.ir = (double *)(base + h->o_ir);
    d.norms = (unsigned long long *)(base + h->o_norms);
    d.n = an.n;
    d.nnz_a = an.nnz_a;
    d.slab_doubles = an.slab_doubles;
    if (h->gexec) {   // the captured graph holds the old workspace's addresses
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
    }
    h->ws = device_ptr;
    h->bound = true;
    h->factored = false;
    return SLU_OK;
}

namespace {
// Per-kernel timing when profiling is on: an event pair around each run of
// consecutive launches of one kernel class (a wave's GETRF steps, its panel
// solves, its Schur-update rounds), with the number of launches inside, so
// the events add little to the launch sequence they time.
struct KernelTimer {
    slu_handle *h;
    hipStream_t s;
    size_t used = 0;
    hipError_t begin(int kind) {
        if (!h->profiling) return hipSuccess;
        if (used + 2 > h->ev.size()) {
            for (int k = 0; k < 64; ++k) {
                hipEvent_t e;
                hipError_t err = hipEventCreate(&e);
                if (hip_failed(err)) return err;
                h->ev.push_back(e);
            }
        }
        if (h->ev_kind.size() < h->ev.size() / 2) {
            h->ev_kind.resize(h->ev.size() / 2);
            h->ev_count.resize(h->ev.size() / 2);
        }
        h->ev_kind[used / 2] = kind;
        h->ev_count[used / 2] = 0;
        return hipEventRecord(h->ev[used], s);
    }
    void launched(int count = 1) {
        if (h->profiling) h->ev_count[used / 2] += count;
    }
    hipError_t end() {
        if (!h->profiling) return hipSuccess;
        hipError_t e = hipEventRecord(h->ev[used + 1], s);
        used += 2;
        return e;
    }
    hipError_t collect() {
        for (int k = 0; k < SLU_NUM_KERNELS; ++k) {
            h->kern_ms[k] = 0.0;
            h->kern_n[k] = 0;
        }
        if (!h->profiling) return hipSuccess;
        for (size_t q = 0; q < used; q += 2) {
            float ms = 0.f;
            hipError_t e = hipEventElapsedTime(&ms, h->ev[q], h->ev[q + 1]);
            if (hip_failed(e)) return e;
            h->kern_ms[h->ev_kind[q / 2]] += ms;
            h->kern_n[h->ev_kind[q / 2]] += h->ev_count[q / 2];
        }
        return hipSuccess;
    }
};
}  // namespace

// Enqueues the whole factorization on s (no host synchronization).
static int enqueue_factor(slu_handle *h, const double *values, hipStream_t s, KernelTimer &kt) {
    const slu::Analysis &an = h->an;
    const slu::DevPlan &d = h->dev;
#define SLU_BEGIN(kind)                                                    \
    do {                                                                   \
        if (hip_failed(kt.begin(kind))) return SLU_ERR_HIP;              \
    } while (0)
#define SLU_LAUNCH(call)                                                   \
    do {                                                                   \
        if (hip_failed((call))) return SLU_ERR_HIP;                      \
        kt.launched();                                                     \
    } while (0)
#define SLU_END()                                                          \
    do {                                                                   \
        if (hip_failed(kt.end())) return SLU_ERR_HIP;                    \
    } while (0)
    if (hip_failed(slu::launch_info_reset(d, s))) return SLU_ERR_HIP;
    SLU_BEGIN(SLU_KERNEL_SCATTER);
    SLU_LAUNCH(slu::launch_zero(d.slab, an.slab_doubles, s));
    SLU_LAUNCH(slu::launch_scatter(d, values, s));
    SLU_END();
    h->wave_tinv.assign(an.waves.size(), 0);
    // lookahead (not under per-kernel timing, which times the classes apart)
    const bool la = h->lookahead && !h->profiling;
    if (la) {
        if (!h->la_stream && hip_failed(hipStreamCreateWithFlags(&h->la_stream, hipStreamNonBlocking)))
            return SLU_ERR_HIP;
        if (!h->ev_panel && hip_failed(hipEventCreateWithFlags(&h->ev_panel, hipEventDisableTiming)))
            return SLU_ERR_HIP;
        if (!h->ev_rest && hip_failed(hipEventCreateWithFlags(&h->ev_rest, hipEventDisableTiming)))
            return SLU_ERR_HIP;
        if (!h->ev_pq && hip_failed(hipEventCreateWithFlags(&h->ev_pq, hipEventDisableTiming)))
            return SLU_ERR_HIP;
    }
    // wave whose deferred updates the factor's stream has not waited for yet
    // (-1: none); they reach waves two or more later, so wave wi waits for
    // them before its first launch at the latest
    int64_t rest_wave = -1;
    // wave whose updates of the next wave's panels run on the second stream
    // and have not been waited for (the next wave's panel solve waits)
    int64_t pq_wave = -1;
    for (size_t wi = 0; wi < an.waves.size(); ++wi) {
        const slu::WaveInfo &w = an.waves[wi];
        const int nlev = w.end - w.begin;
        const int32_t *lv = d.wave_levels + w.begin;
        if (rest_wave >= 0 && rest_wave + 2 <= (int64_t)wi) {
            if (hip_failed(hipStreamWaitEvent(s, h->ev_rest, 0))) return SLU_ERR_HIP;
            rest_wave = -1;
            pq_wave = -1;
        }
        SLU_BEGIN(SLU_KERNEL_GETRF);
        // the tiled GETRF when selected, and for waves whose chunked GETRF
        // would not fit the LDS
        const bool chunk_fits = w.lds_getrf <= 160 * 1024;
        if ((h->getrf_tiled_rows > 0 && w.max_b >= h->getrf_tiled_rows) || !chunk_fits) {
            if (nlev > 65535) return SLU_ERR_LIMIT;
            if (h->getrf_tile == 32) {
                const int max_nt = (w.max_b + 31) / 32;
                const slu::LevelDev *one = nlev == 1 ? &an.levels[an.wave_levels[w.begin]] : nullptr;
                for (int k = 0; k < max_nt; ++k) SLU_LAUNCH(slu::launch_getrf_tile32(d, lv, nlev, k, max_nt, one, s));
                h->wave_tinv[wi] = 1;
            } else {
                const int max_nt = (w.max_b + 15) / 16;
                for (int k = 0; k < max_nt; ++k) SLU_LAUNCH(slu::launch_getrf_tile(d, lv, nlev, k, max_nt, s));
            }
            goto getrf_done;
        }
        {
        // split GETRF when one of the wave's chunked blocks has enough
        // trailing work to be worth spreading over the chip
        bool split = false;
        int nsteps = 1;
        if (nlev <= 65535) {
            for (int q = w.begin; q < w.end; ++q) {
                const slu::LevelDev &L = an.levels[an.wave_levels[q]];
                if (L.b <= slu::kLdsDenseMax) continue;
                double work = 0.0;
                for (int c = L.chunk_begin; c < L.chunk_end; ++c)
                    work += (double)an.chunks[c].nr * an.chunks[c].nr;
                if (work >= h->getrf_split_work) split = true;
                nsteps = std::max(nsteps, L.chunk_end - L.chunk_begin);
            }
        }
        if (!split) {
            SLU_LAUNCH(slu::launch_getrf_wave(d, lv, nlev, w.lds_getrf, s));
        } else {
            for (int k = 0; k < nsteps; ++k) {
                SLU_LAUNCH(slu::launch_getrf_step(d, lv, nlev, k, w.lds_getrf, s));
                int max_tiles = 0;
                for (int q = w.begin; q < w.end; ++q) {
                    const slu::LevelDev &L = an.levels[an.wave_levels[q]];
                    if (L.b <= slu::kLdsDenseMax || L.chunk_begin + k >= L.chunk_end) continue;
                    const int ntl = (an.chunks[L.chunk_begin + k].nr + 15) / 16;
                    max_tiles = std::max(max_tiles, ntl * ntl);
                }
                if (max_tiles > 0) SLU_LAUNCH(slu::launch_getrf_trail(d, lv, nlev, k, max_tiles, s));
            }
        }
        }
    getrf_done:
        SLU_END();
        if (w.max_m > 0 && w.max_kp > 0) {
            SLU_BEGIN(SLU_KERNEL_PANEL);
            if (pq_wave >= 0) {
                if (hip_failed(hipStreamWaitEvent(s, h->ev_pq, 0))) return SLU_ERR_HIP;
                pq_wave = -1;
            }
            SLU_LAUNCH(slu::launch_tri_gather_wave(d, lv, d.tslot_off + w.begin, nlev, w.tslots, s));
            const bool blk = h->panel_blocked && w.max_kp >= slu::kPanelBlkKp;
            // the tile-wise solve, unless every level of the wave takes the
            // blocked one
            bool tilewise = !blk;
            for (int q = w.begin; q < w.end && !tilewise; ++q) {
                const slu::LevelDev &L = an.levels[an.wave_levels[q]];
                if (L.m > 0 && L.kp > 0 && L.offB < 0) tilewise = true;
            }
            if (tilewise) SLU_LAUNCH(slu::launch_panel_solve_wave(d, lv, nlev, w.max_m, w.max_kp, blk ? 1 : 0, s));
            if (blk) {
                if (hip_failed(slu::launch_panel_blk_wave(d, lv, nlev, w.max_m, w.max_kp, s))) return SLU_ERR_HIP;
                kt.launched(1 + (w.max_kp + slu::kPanelBlk - 1) / slu::kPanelBlk);
            }
            SLU_END();
        }
        if (w.round_end > w.round_begin) {
            SLU_BEGIN(SLU_KERNEL_SSSSM);
            const bool f32 = h->precision == SLU_PRECISION_FP32;
            if (!la) {
                for (int r = w.round_begin; r < w.round_end; ++r)
                    SLU_LAUNCH(slu::launch_ssssm_round(d, an.rounds[r], f32, 0, 0, s));
            } else {
                // only a wave with one round is split: the rounds of a wave
                // share targets, so a later round's updates must not run
                // beside an earlier round's deferred ones
                const bool split = w.round_end - w.round_begin == 1;
                // the updates on this stream come after the previous wave's
                // deferred updates (they may share targets)
                if (rest_wave >= 0) {
                    if (hip_failed(hipStreamWaitEvent(s, h->ev_rest, 0))) return SLU_ERR_HIP;
                    rest_wave = -1;
                    pq_wave = -1;
                }
                if (!split) {
                    for (int r = w.round_begin; r < w.round_end; ++r)
                        SLU_LAUNCH(slu::launch_ssssm_round(d, an.rounds[r], f32, 0, 0, s));
                } else {
                    const slu::RoundInfo &ri = an.rounds[w.round_begin];
                    // the next wave's diagonal blocks here; its panels and the
                    // later waves' targets on the second stream, beside the
                    // next wave's GETRF (panels first, at full width; the
                    // rest in a capped grid)
                    SLU_LAUNCH(slu::launch_ssssm_round(d, ri, f32, 3, 0, s));
                    if (ri.tiles_pq > 0 || ri.tiles_r > 0) {
                        hipStream_t b = h->la_stream;
                        if (hip_failed(hipEventRecord(h->ev_panel, s))) return SLU_ERR_HIP;
                        if (hip_failed(hipStreamWaitEvent(b, h->ev_panel, 0))) return SLU_ERR_HIP;
                        SLU_LAUNCH(slu::launch_ssssm_round(d, ri, f32, 4, 0, b));
                        if (hip_failed(hipEventRecord(h->ev_pq, b))) return SLU_ERR_HIP;
                        SLU_LAUNCH(slu::launch_ssssm_round(d, ri, f32, 2, h->la_groups, b));
                        if (hip_failed(hipEventRecord(h->ev_rest, b))) return SLU_ERR_HIP;
                        rest_wave = (int64_t)wi;
                        pq_wave = (int64_t)wi;
                    }
                }
            }
            SLU_END();
        }
    }
    if (rest_wave >= 0 && hip_failed(hipStreamWaitEvent(s, h->ev_rest, 0))) return SLU_ERR_HIP;
#undef SLU_BEGIN
#undef SLU_LAUNCH
#undef SLU_END
    return SLU_OK;
}

int slu_factor(slu_handle *h, const double *values, void *stream) {
    if (!h || (!values && h->an.nnz_a > 0)) return SLU_ERR_ARG;
    if (!h->bound) return SLU_ERR_STATE;
    hipStream_t s = (hipStream_t)stream;
    const slu::DevPlan &d = h->dev;
    h->factored = false;
    h->zero_pivot_col = -1;
    KernelTimer kt{h, s};
    if (h->use_graph && !h->profiling) {
        // the graph reads the values from the workspace copy
        double *staged = (double *)((char *)h->ws + h->o_vals);
        if (h->an.nnz_a > 0 &&
            hip_failed(hipMemcpyAsync(staged, values, (size_t)h->an.nnz_a * 8, hipMemcpyDeviceToDevice, s)))
            return SLU_ERR_HIP;
        if (!h->gexec || h->graph_precision != h->precision) {
            if (h->gexec) {
                (void)hipGraphExecDestroy(h->gexec);
                h->gexec = nullptr;
            }
            if (!h->cap_stream && hip_failed(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking)))
                return SLU_ERR_HIP;
            hipGraph_t g = nullptr;
            if (hip_failed(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal)))
                return SLU_ERR_HIP;
            KernelTimer none{h, h->cap_stream};
            const int rc = enqueue_factor(h, staged, h->cap_stream, none);
            const hipError_t ec = hipStreamEndCapture(h->cap_stream, &g);
            if (rc != SLU_OK || hip_failed(ec)) {
                if (g) (void)hipGraphDestroy(g);
                return rc != SLU_OK ? rc : SLU_ERR_HIP;
            }
            const hipError_t ei = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (hip_failed(ei)) {
                h->gexec = nullptr;
                return SLU_ERR_HIP;
            }
            h->graph_precision = h->precision;
        }
        if (hip_failed(hipGraphLaunch(h->gexec, s))) return SLU_ERR_HIP;
    } else {
        const int rc = enqueue_factor(h, values, s, kt);
        if (rc != SLU_OK) return rc;
    }
    unsigned long long flag = 0;
    if (hip_failed(hipMemcpyAsync(&flag, d.info, sizeof(flag), hipMemcpyDeviceToHost, s))) return SLU_ERR_HIP;
    if (hip_failed(hipStreamSynchronize(s))) return SLU_ERR_HIP;
    if (hip_failed(kt.collect())) return SLU_ERR_HIP;
    if (flag != ~0ull) {
        h->zero_pivot_col = (int64_t)flag;
        return SLU_ZERO_PIVOT;
    }
    h->factored = true;
    return SLU_OK;
}

int slu_solve(slu_handle *h, const double *B, double *X, int64_t nrhs, int64_t ld, void *stream) {
    return solve_impl(h, B, X, nrhs, ld, 0, (hipStream_t)stream);
}

int slu_solve_transpose(slu_handle *h, const double *B, double *X, int64_t nrhs, int64_t ld, void *stream) {
    return solve_impl(h, B, X, nrhs, ld, 1, (hipStream_t)stream);
}

int slu_solve_noalloc(slu_handle *h, const double *B, double *X, int64_t nrhs, int64_t ld, int transpose,
                      void *stream) {
    if (!h || (transpose != 0 && transpose != 1)) return SLU_ERR_ARG;
    // the work block must fit the fixed scratch: at least one column of n
    if (h->an.n > (int64_t)slu::kStaticScratchDoubles) return SLU_ERR_LIMIT;
    const int rc = solve_check(h, B, X, nrhs, ld);
    if (rc != SLU_OK) return rc;
    if (nrhs == 0) return SLU_OK;
    double *fixed = nullptr;
    if (hip_failed(slu::static_scratch(&fixed))) return SLU_ERR_HIP;
    slu::DevPlan d = h->dev;
    d.scratch = fixed;
    const int64_t fit = (int64_t)slu::kStaticScratchDoubles / std::max<int64_t>(h->an.n, 1);
    const int cols = (int)std::min<int64_t>(h->solve_cols, fit);
    return solve_sweeps(h, d, cols, B, X, nrhs, ld, transpose, (hipStream_t)stream);
}

int slu_value_gradient(slu_handle *h, const double *G, const double *X, int64_t nrhs, int64_t ld,
                       double *grad_values, void *stream) {
    if (!h || nrhs < 0 || (h->an.nnz_a > 0 && !grad_values) || (nrhs > 0 && (!G || !X))) return SLU_ERR_ARG;
    if (!h->bound) return SLU_ERR_STATE;
    if (ld < h->an.n || ld < 1) return SLU_ERR_ARG;
    if (hip_failed(slu::launch_value_gradient(h->dev, G, X, nrhs, ld, grad_values, (hipStream_t)stream)))
        return SLU_ERR_HIP;
    return SLU_OK;
}

int slu_set_graph(slu_handle *h, int enable) {
    if (!h) return SLU_ERR_ARG;
    h->use_graph = enable != 0;
    if (!h->use_graph && h->gexec) {
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
    }
    return SLU_OK;
}

int slu_set_getrf_split(slu_handle *h, double min_work) {
    if (!h || !(min_work >= 0.0)) return SLU_ERR_ARG;
    h->getrf_split_work = min_work;
    if (h->gexec) {   // a captured graph holds the other launch sequence
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
    }
    return SLU_OK;
}

int slu_set_getrf_tiled(slu_handle *h, int min_rows) {
    if (!h || min_rows < 0) return SLU_ERR_ARG;
    h->getrf_tiled_rows = min_rows;
    if (h->gexec) {   // a captured graph holds the other launch sequence
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
    }
    return SLU_OK;
}

int slu_set_getrf_tile(slu_handle *h, int tile) {
    if (!h || (tile != 16 && tile != 32)) return SLU_ERR_ARG;
    h->getrf_tile = tile;
    if (h->gexec) {   // a captured graph holds the other launch sequence
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
    }
    return SLU_OK;
}

int slu_set_lookahead(slu_handle *h, int enable, int max_groups) {
    if (!h || (enable != 0 && enable != 1) || max_groups < 0 || max_groups % 8 != 0) return SLU_ERR_ARG;
    h->lookahead = enable != 0;
    h->la_groups = max_groups;
    if (h->gexec) {   // a captured graph holds the other launch sequence
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
    }
    return SLU_OK;
}

int slu_set_panel_blocked(slu_handle *h, int enable) {
    if (!h || (enable != 0 && enable != 1)) return SLU_ERR_ARG;
    h->panel_blocked = enable != 0;
    if (h->gexec) {   // a captured graph holds the other launch sequence
        (void)hipGraphExecDestroy(h->gexec);
        h->gexec = nullptr;
    }
    return SLU_OK;
}

int slu_autotune(slu_handle *h, const double *values, int reps, slu_tune_entry *table, int capacity, int *count,
                 void *stream) {
    if (!h || (!values && h->an.nnz_a > 0) || reps < 1 || capacity < 0 || (capacity > 0 && !table)) return SLU_ERR_ARG;
    if (!h->bound) return SLU_ERR_STATE;
    hipStream_t s = (hipStream_t)stream;
    // the launch-shape settings tried: GETRF path x panel path x graph
    // replay x lookahead
    struct Cfg {
        int tiled_rows, tile, panel, graph, lookahead;
    };
    const Cfg cfgs[] = {{1, 32, 1, 0, 0}, {1, 32, 1, 0, 1}, {1, 32, 0, 0, 0}, {1, 16, 1, 0, 0}, {0, 32, 1, 0, 0},
                        {1, 32, 1, 1, 0}, {1, 32, 1, 1, 1}, {1, 16, 1, 1, 0}, {0, 32, 1, 1, 0}};
    const int ncfg = (int)(sizeof(cfgs) / sizeof(cfgs[0]));
    const bool prof = h->profiling;
    h->profiling = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = SLU_OK;
    if (hip_failed(hipEventCreate(&e0)) || hip_failed(hipEventCreate(&e1))) rc = SLU_ERR_HIP;
    int best = -1;
    double best_ms = 0.0;
    int n = 0;
    std::vector<float> t((size_t)reps);
    for (int c = 0; c < ncfg && rc == SLU_OK; ++c) {
        h->getrf_tiled_rows = cfgs[c].tiled_rows;
        h->getrf_tile = cfgs[c].tile;
        h->panel_blocked = cfgs[c].panel != 0;
        h->lookahead = cfgs[c].lookahead != 0;
        if (h->gexec) {
            (void)hipGraphExecDestroy(h->gexec);
            h->gexec = nullptr;
        }
        h->use_graph = cfgs[c].graph != 0;
        rc = slu_factor(h, values, stream);   // warm-up (and graph capture)
        for (int r = 0; r < reps && rc == SLU_OK; ++r) {
            if (hip_failed(hipEventRecord(e0, s))) rc = SLU_ERR_HIP;
            if (rc == SLU_OK) rc = slu_factor(h, values, stream);
            if (rc == SLU_OK && hip_failed(hipEventRecord(e1, s))) rc = SLU_ERR_HIP;
            if (rc == SLU_OK && hip_failed(hipEventSynchronize(e1))) rc = SLU_ERR_HIP;
            if (rc == SLU_OK && hip_failed(hipEventElapsedTime(&t[r], e0, e1))) rc = SLU_ERR_HIP;
        }
        if (rc != SLU_OK) break;
        std::sort(t.begin(), t.end());
        const double ms = t[(size_t)reps / 2];
        if (n < capacity) {
            table[n].getrf_tiled_rows = cfgs[c].tiled_rows;
            table[n].getrf_tile = cfgs[c].tile;
            table[n].panel_blocked = cfgs[c].panel;
            table[n].graph = cfgs[c].graph;
            table[n].lookahead = cfgs[c].lookahead;
            table[n].ms = ms;
        }
        ++n;
        if (best < 0 || ms < best_ms) {
            best = c;
            best_ms = ms;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (count) *count = n;
    if (best >= 0) {
        h->getrf_tiled_rows = cfgs[best].tiled_rows;
        h->getrf_tile = cfgs[best].tile;
        h->panel_blocked = cfgs[best].panel != 0;
        h->lookahead = cfgs[best].lookahead != 0;
        if (h->gexec) {
            (void)hipGraphExecDestroy(h->gexec);
            h->gexec = nullptr;
        }
        h->use_graph = cfgs[best].graph != 0;
        if (rc == SLU_OK) rc = slu_factor(h, values, stream);   // the handle ends factored with the choice
    }
    h->profiling = prof;
    return rc;
}

int slu_set_solve_tiled(slu_handle *h, int min_rows, int min_sparse_rows) {
    if (!h || min_rows < 0 || min_sparse_rows < 0) return SLU_ERR_ARG;
    h->solve_tiled_rows = min_rows;
    h->solve_tiled_sparse_rows = min_sparse_rows == 0 ? INT32_MAX : min_sparse_rows;
    return SLU_OK;
}

int slu_set_precision(slu_handle *h, int precision) {
    if (!h || (precision != SLU_PRECISION_FP64 && precision != SLU_PRECISION_FP32)) return SLU_ERR_ARG;
    h->precision = precision;
    return SLU_OK;
}

int slu_solve_refined(slu_handle *h, const double *values, const double *B, double *X, int64_t nrhs, int64_t ld,
                      double tol, int maxit, int *iters, double *eta, void *stream) {
    if (!h || nrhs < 0 || maxit < 0 || (nrhs > 0 && (!values || !B || !X || B == X))) return SLU_ERR_ARG;
    if (!h->bound) return SLU_ERR_STATE;
    if (!h->factored) return SLU_ERR_NOT_FACTORED;
    if (ld < h->an.n || ld < 1) return SLU_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    const slu::DevPlan &d = h->dev;
    const int64_t n = h->an.n;
    double *R = d.ir, *Dv = d.ir + (size_t)n * slu::kSolveCols;
    int used = 0;
    bool converged = true;
    for (int64_t c0 = 0; c0 < nrhs; c0 += slu::kSolveCols) {
        const int nc = (int)std::min<int64_t>(slu::kSolveCols, nrhs - c0);
        const double *Bc = B + c0 * ld;
        double *Xc = X + c0 * ld;
        int rc = solve_impl(h, Bc, Xc, nc, ld, 0, s);
        if (rc != SLU_OK) return rc;
        double prev[slu::kSolveCols], cur[slu::kSolveCols];
        for (int c = 0; c < nc; ++c) prev[c] = 1.0 / 0.0;
        int it = 0;
        for (;;) {
            rc = slu_backward_error(h, values, Bc, Xc, nc, ld, 0, cur, stream);
            if (rc != SLU_OK) return rc;
            bool done = true, progress = false;
            for (int c = 0; c < nc; ++c) {
                if (!(cur[c] <= tol)) done = false;
                if (cur[c] <= 0.5 * prev[c]) progress = true;
            }
            if (done || it >= maxit || !progress) {
                if (!done) converged = false;
                break;
            }
            if (hip_failed(slu::launch_residual(d, values, Bc, ld, Xc, ld, R, n, nc, s))) return SLU_ERR_HIP;
            rc = solve_impl(h, R, Dv, nc, n, 0, s);
            if (rc != SLU_OK) return rc;
            if (hip_failed(slu::launch_axpy(d, Xc, ld, Dv, n, nc, s))) return SLU_ERR_HIP;
            for (int c = 0; c < nc; ++c) prev[c] = cur[c];
            ++it;
        }
        used = std::max(used, it);
        if (eta)
            for (int c = 0; c < nc; ++c) eta[c0 + c] = cur[c];
    }
    if (iters) *iters = used;
    return converged ? SLU_OK : SLU_NOT_CONVERGED;
}

int slu_backward_error(slu_handle *h, const double *values, const double *B, const double *X, int64_t nrhs,
                       int64_t ld, int transpose, double *eta, void *stream) {
    if (!h || !eta || nrhs < 0 || (nrhs > 0 && (!B || !X || !values))) return SLU_ERR_ARG;
    if (!h->bound) return SLU_ERR_STATE;
    if (ld < h->an.n || ld < 1) return SLU_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    for (int64_t c0 = 0; c0 < nrhs; c0 += slu::kSolveCols) {
        const int nc = (int)std::min<int64_t>(slu::kSolveCols, nrhs - c0);
        if (hip_failed(slu::launch_residual_norms(h->dev, values, B + c0 * ld, X + c0 * ld, ld, nc, transpose ? 1 : 0, s)))
            return SLU_ERR_HIP;
        unsigned long long nb[64];
        if (hip_failed(hipMemcpyAsync(nb, h->dev.norms, sizeof(nb), hipMemcpyDeviceToHost, s))) return SLU_ERR_HIP;
        if (hip_failed(hipStreamSynchronize(s))) return SLU_ERR_HIP;
        double v[64];
        std::memcpy(v, nb, sizeof(v));
        for (int c = 0; c < nc; ++c) {
            const double den = v[48] * v[16 + c] + v[32 + c];
            eta[c0 + c] = den > 0.0 ? v[c] / den : (v[c] > 0.0 ? 1.0 / 0.0 : 0.0);
        }
    }
    return SLU_OK;
}

int slu_get_info(const slu_handle *h, slu_info *info) {
    if (!h || !info) return SLU_ERR_ARG;
    const slu::Analysis &an = h->an;
    std::memset(info, 0, sizeof(*info));
    info->n = an.n;
    info->nnz_a = an.nnz_a;
    info->nnz_s = 2 * (an.s_colptr.empty() ? 0 : an.s_colptr[an.n]) - an.n;
    info->nblocks = an.p;
    info->nonempty_blocks = an.nonempty_blocks;
    info->ssssm_tasks = (int64_t)an.stgt.size();
    info->flops = an.flops;
    info->flops_getrf = an.flops_getrf;
    info->flops_panel = an.flops_panel;
    info->flops_ssssm = an.flops_ssssm;
    info->stored_flops = an.stored_flops;
    info->slab_bytes = an.slab_doubles * 8;
    info->workspace_bytes = (int64_t)h->ws_bytes;
    info->zero_pivot_col = h->zero_pivot_col;
    info->factored = h->factored ? 1 : 0;
    info->max_block = an.max_block;
    info->precision = h->precision;
    info->waves = (int32_t)an.waves.size();
    info->rounds = (int32_t)an.rounds.size();
    return SLU_OK;
}

int slu_get_perm(const slu_handle *h, int32_t *perm) {
    if (!h || (!perm && h->an.n > 0)) return SLU_ERR_ARG;
    std::copy(h->an.perm.begin(), h->an.perm.end(), perm);
    return SLU_OK;
}

int slu_get_blockptr(const slu_handle *h, int64_t *blockptr) {
    if (!h || !blockptr) return SLU_ERR_ARG;
    std::copy(h->an.blockptr.begin(), h->an.blockptr.end(), blockptr);
    return SLU_OK;
}

int slu_get_blocking(const slu_handle *h, int64_t *ptr) {
    if (!h || !ptr) return SLU_ERR_ARG;
    std::copy(h->an.bptr.begin(), h->an.bptr.end(), ptr);
    return SLU_OK;
}

int slu_get_pattern(const slu_handle *h, int64_t *colptr, int32_t *rowidx) {
    if (!h || !colptr || (!rowidx && !h->an.s_rowidx.empty())) return SLU_ERR_ARG;
    std::copy(h->an.s_colptr.begin(), h->an.s_colptr.end(), colptr);
    std::copy(h->an.s_rowidx.begin(), h->an.s_rowidx.end(), rowidx);
    return SLU_OK;
}

int slu_get_factors(const slu_handle *h, double *lval, double *uval, void *stream) {
    if (!h || !lval || !uval) return SLU_ERR_ARG;
    if (!h->bound) return SLU_ERR_STATE;
    if (!h->factored) return SLU_ERR_NOT_FACTORED;
    const slu::Analysis &an = h->an;
    std::vector<double> slab;
    try {
        slab.resize((size_t)an.slab_doubles);
    } catch (const std::bad_alloc &) {
        return SLU_ERR_NOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    if (!slab.empty() &&
        hip_failed(hipMemcpyAsync(slab.data(), h->dev.slab, slab.size() * 8, hipMemcpyDeviceToHost, s)))
        return SLU_ERR_HIP;
    if (hip_failed(hipStreamSynchronize(s))) return SLU_ERR_HIP;
    for (int64_t c = 0; c < an.n; ++c) {
        const int32_t J = an.bid[c];
        const slu::LevelDev &LJ = an.levels[J];
        for (int64_t q = an.s_colptr[c]; q < an.s_colptr[c + 1]; ++q) {
            const int32_t r = an.s_rowidx[q];
            const int32_t I = an.bid[r];
            if (I == J) {
                const int64_t lr = r - LJ.r0, lc = c - LJ.r0;
                lval[q] = slab[LJ.offD + lr + lc * LJ.b];
                uval[q] = slab[LJ.offD + lc + lr * LJ.b];
            } else {
                const int32_t *rows = an.R_idx.data() + LJ.Roff;
                const int64_t rp = std::lower_bound(rows, rows + LJ.m, r) - rows;
                const int64_t kp = an.posK[c];
                lval[q] = slab[LJ.offP + rp + kp * LJ.m];
                uval[q] = slab[LJ.offQ + rp + kp * LJ.m];
            }
        }
    }
    return SLU_OK;
}

const char *slu_error_string(int code) {
    switch (code) {
        case SLU_OK: return "success";
        case SLU_ZERO_PIVOT: return "zero or non-finite pivot";
        case SLU_NOT_CONVERGED: return "iterative refinement stopped above its tolerance";
        case SLU_ERR_ARG: return "invalid argument";
        case SLU_ERR_ROWPTR: return "rowptr does not start at 0 or is not monotone";
        case SLU_ERR_COLIDX: return "column index out of range";
        case SLU_ERR_UNSORTED: return "column indices of a row unsorted or duplicated";
        case SLU_ERR_PERM: return "user ordering is not a permutation";
        case SLU_ERR_STATE: return "call out of order (bind a workspace first)";
        case SLU_ERR_WORKSPACE: return "workspace too small or not 256-byte aligned";
        case SLU_ERR_HIP: return "HIP runtime error";
        case SLU_ERR_NOMEM: return "host allocation failed";
        case SLU_ERR_NOT_FACTORED: return "no successful factorization";
        case SLU_ERR_LIMIT: return "problem exceeds the library's size limits";
        default: return "unknown error code";
    }
}

int slu_set_host_threads(int threads) {
    if (threads < 0) return SLU_ERR_ARG;
    slu::set_host_threads(threads);
    return SLU_OK;
}

int slu_last_hip_error(void) { return t_last_hip; }

const char *slu_hip_error_string(int hip_code) { return hipGetErrorString((hipError_t)hip_code); }

int slu_set_profiling(slu_handle *h, int enable) {
    if (!h) return SLU_ERR_ARG;
    h->profiling = enable != 0;
    return SLU_OK;
}

int slu_get_kernel_times(const slu_handle *h, double *ms, int64_t *launches) {
    if (!h || !ms || !launches) return SLU_ERR_ARG;
    for (int k = 0; k < SLU_NUM_KERNELS; ++k) {
        ms[k] = h->kern_ms[k];
        launches[k] = h->kern_n[k];
    }
    return SLU_OK;
}

void slu_free(slu_handle *h) {
    if (!h) return;
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->la_stream) (void)hipStreamDestroy(h->la_stream);
    if (h->ev_panel) (void)hipEventDestroy(h->ev_panel);
    if (h->ev_rest) (void)hipEventDestroy(h->ev_rest);
    if (h->ev_pq) (void)hipEventDestroy(h->ev_pq);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    delete h;
}

}  // extern "C"
