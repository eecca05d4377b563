// Host-side analysis: validation, ordering, symbolic fill, Algorithm 2,
// Algorithm 3 and the block storage plan used by the device kernels.
#include "analyze.hpp"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <new>
#include <numeric>
#include <thread>

namespace slu {

// ---------------------------------------------------------------- ordering
// The paper requires a fill-reducing reordering (Section 1, Section 2.1,
// Fig. 2) without naming one.  Geometric nested dissection of a grid with a
// fixed rule: cut the longest axis (lowest axis on ties) at lo + (hi-lo)/2;
// order the first part, the second part, then the separator plane; boxes of
// volume <= 8 or with every extent <= 2 are listed in grid-index order.
namespace {
struct Box {
    int32_t lo[3], hi[3];
};

void box_points(const Box &bx, int32_t nx, int32_t ny, std::vector<int32_t> *out) {
    for (int32_t z = bx.lo[2]; z < bx.hi[2]; ++z)
        for (int32_t y = bx.lo[1]; y < bx.hi[1]; ++y)
            for (int32_t x = bx.lo[0]; x < bx.hi[0]; ++x)
                out->push_back(x + nx * (y + ny * z));
}

void nd_rec(const Box &bx, int32_t nx, int32_t ny, std::vector<int32_t> *out) {
    int64_t ext[3];
    for (int d = 0; d < 3; ++d) ext[d] = (int64_t)bx.hi[d] - bx.lo[d];
    if (ext[0] <= 0 || ext[1] <= 0 || ext[2] <= 0) return;
    int64_t vol = ext[0] * ext[1] * ext[2];
    int64_t mx = std::max(ext[0], std::max(ext[1], ext[2]));
    if (vol <= 8 || mx <= 2) {
        box_points(bx, nx, ny, out);
        return;
    }
    int d = 0;
    for (int e = 1; e < 3; ++e)
        if (ext[e] > ext[d]) d = e;
    int32_t m = bx.lo[d] + (bx.hi[d] - bx.lo[d]) / 2;
    Box a = bx, c = bx, s = bx;
    a.hi[d] = m;
    c.lo[d] = m + 1;
    s.lo[d] = m;
    s.hi[d] = m + 1;
    nd_rec(a, nx, ny, out);
    nd_rec(c, nx, ny, out);
    box_points(s, nx, ny, out);
}
}  // namespace

void nd_grid_order(int32_t nx, int32_t ny, int32_t nz, std::vector<int32_t> *perm) {
    perm->clear();
    perm->reserve((size_t)nx * ny * nz);
    Box root{{0, 0, 0}, {nx, ny, nz}};
    nd_rec(root, nx, ny, perm);
}

// ------------------------------------------------------------ Algorithm 3
// Structure-aware blocking (Section 4.3).  The feature curve blockptr is read
// at Sp + 1 rows, Sp = min(sample_points, N), sample s at floor(s N / Sp).
// Windows of `step` sample intervals are tested in order, the start moving by
// `advance` samples.  A window's end becomes a block boundary when the window
// holds at least step/Sp of all entries of S (a dense stretch: fine blocks),
// or when max_num windows have passed since the last boundary (a sparse
// stretch: blocks of a bounded number of windows).  The threshold test is
// exact in integers, increment * Sp >= step * blockptr[N]; N closes the
// last block.
void irregular_blocking(const std::vector<int64_t> &blockptr, int sample_points, int step,
                        int max_num, int advance, std::vector<int64_t> *ptr) {
    ptr->clear();
    const int64_t N = (int64_t)blockptr.size() - 1;
    ptr->push_back(0);
    if (N <= 0) return;
    const int64_t sp = std::min<int64_t>(sample_points, N);
    auto row = [&](int64_t s) { return (int64_t)(((__int128)s * N) / sp); };
    const __int128 need = (__int128)step * blockptr[N];
    int64_t passed = 0;   // windows since the last boundary
    for (int64_t s = 0; s + step <= sp; s += advance) {
        const int64_t end = row(s + step);
        const bool dense = (__int128)(blockptr[end] - blockptr[row(s)]) * sp >= need;
        if (dense || passed >= max_num) {
            ptr->push_back(end);
            passed = 0;
        } else {
            ++passed;
        }
    }
    if (ptr->back() != N) ptr->push_back(N);
}

// ---------------------------------------------------------------- analysis
namespace {

int validate(int64_t n, const int64_t *rowptr, const int32_t *colidx) {
    if (n < 0) return SLU_ERR_ARG;
    if (n >= ((int64_t)1 << 31) - 1) return SLU_ERR_LIMIT;
    if (!rowptr) return SLU_ERR_ARG;
    if (rowptr[0] != 0) return SLU_ERR_ROWPTR;
    for (int64_t i = 0; i < n; ++i)
        if (rowptr[i + 1] < rowptr[i]) return SLU_ERR_ROWPTR;
    if (rowptr[n] > 0 && !colidx) return SLU_ERR_ARG;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
            const int32_t c = colidx[q];
            if (c < 0 || c >= n) return SLU_ERR_COLIDX;
            if (q > rowptr[i] && c <= colidx[q - 1]) return SLU_ERR_UNSORTED;
        }
    }
    return SLU_OK;
}

// Pattern of B = P0[perm][:, perm] with P0 = A + A^T + I, as sorted CSR.
void permuted_symmetric(const Analysis &an, std::vector<int64_t> *bp, std::vector<int32_t> *bi) {
    const int64_t n = an.n;
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t r = an.iperm[i];
        cnt[r + 1] += 1;  // diagonal
        for (int64_t q = an.a_rowptr[i]; q < an.a_rowptr[i + 1]; ++q) {
            const int64_t c = an.iperm[an.a_colidx[q]];
            if (c == r) continue;
            cnt[r + 1] += 1;
            cnt[c + 1] += 1;
        }
    }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> tmp(cnt[n]);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t r = an.iperm[i];
        tmp[fill[r]++] = (int32_t)r;
        for (int64_t q = an.a_rowptr[i]; q < an.a_rowptr[i + 1]; ++q) {
            const int64_t c = an.iperm[an.a_colidx[q]];
            if (c == r) continue;
            tmp[fill[r]++] = (int32_t)c;
            tmp[fill[c]++] = (int32_t)r;
        }
    }
    bp->assign(n + 1, 0);
    bi->clear();
    bi->reserve(tmp.size());
    for (int64_t r = 0; r < n; ++r) {
        auto b = tmp.begin() + cnt[r], e = tmp.begin() + cnt[r + 1];
        std::sort(b, e);
        auto u = std::unique(b, e);
        bi->insert(bi->end(), b, u);
        (*bp)[r + 1] = (int64_t)bi->size();
    }
}

// Lower CSC of the fill of symmetric pattern B: Struct(L_k) = Adj_{>k}(k)
// union (Struct(L_c) minus {k}) over the elimination-tree children c of k.
void symbolic_fill(int64_t n, const std::vector<int64_t> &bp, const std::vector<int32_t> &bi,
                   std::vector<int64_t> *colptr, std::vector<int32_t> *rowidx) {
    colptr->assign(n + 1, 0);
    rowidx->clear();
    rowidx->reserve(bi.size());
    std::vector<int32_t> mark(n, -1), head(n, -1), next(n, -1), list;
    for (int64_t k = 0; k < n; ++k) {
        list.clear();
        mark[k] = (int32_t)k;
        for (int64_t q = bp[k]; q < bp[k + 1]; ++q) {
            const int32_t r = bi[q];
            if (r > k && mark[r] != k) {
                mark[r] = (int32_t)k;
                list.push_back(r);
            }
        }
        for (int32_t c = head[k]; c >= 0; c = next[c]) {
            // skip the diagonal and the first sub-diagonal row (== k)
            for (int64_t q = (*colptr)[c] + 2; q < (*colptr)[c + 1]; ++q) {
                const int32_t r = (*rowidx)[q];
                if (mark[r] != k) {
                    mark[r] = (int32_t)k;
                    list.push_back(r);
                }
            }
        }
        std::sort(list.begin(), list.end());
        rowidx->push_back((int32_t)k);
        rowidx->insert(rowidx->end(), list.begin(), list.end());
        (*colptr)[k + 1] = (int64_t)rowidx->size();
        if (!list.empty()) {
            const int32_t par = list[0];
            next[k] = head[par];
            head[par] = (int32_t)k;
        }
    }
}

inline int64_t align32(int64_t x) { return (x + 31) & ~(int64_t)31; }

// Host threads for the parallel parts of the analysis (0: the hardware's
// count, at most 16).
std::atomic<int> g_host_threads{0};

int host_threads() {
    int t = g_host_threads.load();
    if (t <= 0) {
        const unsigned hw = std::thread::hardware_concurrency();
        t = hw == 0 ? 1 : (int)std::min(hw, 16u);
    }
    return t;
}

// f(i) for i in [0, count), chunks of `chunk` indices handed out in order to
// the host threads; f must touch only data that no other index touches.  An
// allocation failure in any thread is rethrown (std::bad_alloc) in the
// caller's thread once every thread has stopped.
template <class F>
void parallel_for(int64_t count, int64_t chunk, F &&f) {
    const int nt = (int)std::min<int64_t>(host_threads(), (count + chunk - 1) / chunk);
    if (nt <= 1) {
        for (int64_t i = 0; i < count; ++i) f(i);
        return;
    }
    std::atomic<int64_t> next{0};
    std::atomic<int> failed{0};
    auto work = [&]() {
        try {
            for (;;) {
                const int64_t b = next.fetch_add(chunk);
                if (b >= count || failed.load()) break;
                const int64_t e = std::min(count, b + chunk);
                for (int64_t i = b; i < e; ++i) f(i);
            }
        } catch (const std::bad_alloc &) {
            failed.store(1);
        }
    };
    std::vector<std::thread> pool;
    pool.reserve(nt - 1);
    for (int t = 1; t < nt; ++t) pool.emplace_back(work);
    work();
    for (std::thread &th : pool) th.join();
    if (failed.load()) throw std::bad_alloc();
}

// Positions of the increasing values v[0..nv) in the sorted array b[0..len)
// (-1 where absent): a binary search for the first, then a forward walk
// (the values of one segment are close together in b).
void sorted_pos(const int32_t *b, int32_t len, const int32_t *v, int32_t nv, int32_t *out) {
    if (nv <= 0) return;
    int32_t p = (int32_t)(std::lower_bound(b, b + len, v[0]) - b);
    for (int32_t a = 0; a < nv; ++a) {
        while (p < len && b[p] < v[a]) ++p;
        out[a] = (p < len && b[p] == v[a]) ? p : -1;
    }
}

int32_t lower_pos(const int32_t *b, int32_t len, int32_t v) {
    const int32_t *it = std::lower_bound(b, b + len, v);
    if (it == b + len || *it != v) return -1;
    return (int32_t)(it - b);
}

}  // namespace

void set_host_threads(int threads) { g_host_threads.store(threads < 0 ? 0 : threads); }

int analyze(int64_t n, const int64_t *rowptr, const int32_t *colidx, const slu_options &opt,
            Analysis *out, const std::vector<int64_t> *segments) {
    int rc = validate(n, rowptr, colidx);
    if (rc != SLU_OK) return rc;
    if (opt.sample_points < 1 || opt.step < 1 || opt.max_num < 0 || opt.advance < 1)
        return SLU_ERR_ARG;
    if (opt.blocking != SLU_BLOCK_IRREGULAR && opt.blocking != SLU_BLOCK_REGULAR) return SLU_ERR_ARG;
    if (opt.schedule != SLU_SCHEDULE_WAVES && opt.schedule != SLU_SCHEDULE_LEVELS) return SLU_ERR_ARG;
    if (opt.blocking == SLU_BLOCK_REGULAR && opt.regular_block < 1) return SLU_ERR_ARG;

    Analysis &an = *out;
    an = Analysis();
    an.n = n;
    an.opt = opt;
    an.opt.user_perm = nullptr;
    an.nnz_a = rowptr[n];
    an.a_rowptr.assign(rowptr, rowptr + n + 1);
    an.a_colidx.assign(colidx, colidx + an.nnz_a);

    // ordering
    if (opt.ordering == SLU_ORDER_NATURAL) {
        an.perm.resize(n);
        std::iota(an.perm.begin(), an.perm.end(), 0);
    } else if (opt.ordering == SLU_ORDER_GRID_ND) {
        const int64_t nx = opt.grid_dims[0], ny = opt.grid_dims[1], nz = opt.grid_dims[2];
        if (nx < 1 || ny < 1 || nz < 1 || nx * ny * nz != n) return SLU_ERR_ARG;
        nd_grid_order((int32_t)nx, (int32_t)ny, (int32_t)nz, &an.perm);
    } else if (opt.ordering == SLU_ORDER_GRAPH_ND) {
        nd_graph_order(n, rowptr, colidx, &an.perm);
    } else if (opt.ordering == SLU_ORDER_USER) {
        if (!opt.user_perm && n > 0) return SLU_ERR_ARG;
        an.perm.assign(opt.user_perm, opt.user_perm + n);
    } else {
        return SLU_ERR_ARG;
    }
    an.iperm.assign(n, -1);
    for (int64_t k = 0; k < n; ++k) {
        const int32_t v = an.perm[k];
        if (v < 0 || v >= n || an.iperm[v] != -1) return SLU_ERR_PERM;
        an.iperm[v] = (int32_t)k;
    }

    // symbolic fill of the permuted symmetrised pattern; stacked independent
    // systems (no entry couples two of them) are filled on host threads, one
    // system per task, and concatenated
    {
        std::vector<int64_t> bp;
        std::vector<int32_t> bi;
        permuted_symmetric(an, &bp, &bi);
        bool split = segments && segments->size() > 2;
        if (split) {
            const std::vector<int64_t> &sg = *segments;
            for (size_t q = 0; q + 1 < sg.size() && split; ++q)
                for (int64_t k = sg[q]; k < sg[q + 1] && split; ++k)
                    for (int64_t e = bp[k]; e < bp[k + 1]; ++e)
                        if (bi[e] < sg[q] || bi[e] >= sg[q + 1]) {
                            split = false;
                            break;
                        }
        }
        if (!split) {
            symbolic_fill(n, bp, bi, &an.s_colptr, &an.s_rowidx);
        } else {
            const std::vector<int64_t> &sg = *segments;
            const int64_t ns = (int64_t)sg.size() - 1;
            std::vector<std::vector<int64_t>> cps(ns);
            std::vector<std::vector<int32_t>> ris(ns);
            parallel_for(ns, 1, [&](int64_t q) {
                const int64_t s0 = sg[q], s1 = sg[q + 1], nq = s1 - s0;
                std::vector<int64_t> lp(nq + 1);
                std::vector<int32_t> li((size_t)(bp[s1] - bp[s0]));
                for (int64_t k = 0; k <= nq; ++k) lp[k] = bp[s0 + k] - bp[s0];
                for (int64_t e = bp[s0]; e < bp[s1]; ++e) li[e - bp[s0]] = (int32_t)(bi[e] - s0);
                symbolic_fill(nq, lp, li, &cps[q], &ris[q]);
            });
            an.s_colptr.assign(n + 1, 0);
            int64_t tot = 0;
            for (int64_t q = 0; q < ns; ++q) tot += (int64_t)ris[q].size();
            an.s_rowidx.resize((size_t)tot);
            int64_t base = 0;
            for (int64_t q = 0; q < ns; ++q) {
                const int64_t s0 = sg[q], nq = sg[q + 1] - s0;
                for (int64_t k = 0; k < nq; ++k) an.s_colptr[s0 + k + 1] = base + cps[q][k + 1];
                for (size_t e = 0; e < ris[q].size(); ++e) an.s_rowidx[(size_t)base + e] = (int32_t)(ris[q][e] + s0);
                base += (int64_t)ris[q].size();
                std::vector<int64_t>().swap(cps[q]);
                std::vector<int32_t>().swap(ris[q]);
            }
        }
    }
    const int64_t nnzL = an.s_colptr[n];

    // Algorithm 2: blockptr[i+1] = blockptr[i] + 2*num[i] + 1 where num[r]
    // counts the entries of S below the diagonal in row r.
    {
        std::vector<int64_t> num(n, 0);
        for (int64_t k = 0; k < n; ++k)
            for (int64_t q = an.s_colptr[k] + 1; q < an.s_colptr[k + 1]; ++q) num[an.s_rowidx[q]] += 1;
        an.blockptr.assign(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) an.blockptr[i + 1] = an.blockptr[i] + 2 * num[i] + 1;
    }

    // blocking (per system when the matrix stacks independent systems)
    {
        std::vector<int64_t> seg = {0, n};
        if (segments) {
            seg = *segments;
            if (seg.size() < 2 || seg.front() != 0 || seg.back() != n) return SLU_ERR_ARG;
            for (size_t q = 1; q < seg.size(); ++q)
                if (seg[q] <= seg[q - 1]) return SLU_ERR_ARG;
        }
        an.bptr.assign(1, 0);
        std::vector<int64_t> part, ptr;
        for (size_t q = 0; q + 1 < seg.size(); ++q) {
            const int64_t s0 = seg[q], s1 = seg[q + 1];
            if (opt.blocking == SLU_BLOCK_IRREGULAR) {
                // the system's own block pointer: S has no entry coupling systems
                part.assign(an.blockptr.begin() + s0, an.blockptr.begin() + s1 + 1);
                for (int64_t &x : part) x -= an.blockptr[s0];
                irregular_blocking(part, opt.sample_points, opt.step, opt.max_num, opt.advance, &ptr);
            } else {
                ptr.clear();
                for (int64_t r = 0; r < s1 - s0; r += opt.regular_block) ptr.push_back(r);
                ptr.push_back(s1 - s0);
            }
            for (size_t t = 1; t < ptr.size(); ++t) an.bptr.push_back(s0 + ptr[t]);
        }
    }
    const int64_t p = (int64_t)an.bptr.size() - 1;
    an.p = p;
    an.bid.assign(n, 0);
    for (int64_t i = 0; i < p; ++i) {
        for (int64_t r = an.bptr[i]; r < an.bptr[i + 1]; ++r) an.bid[r] = (int32_t)i;
        an.max_block = std::max<int32_t>(an.max_block, (int32_t)(an.bptr[i + 1] - an.bptr[i]));
    }

    // flop count on S (identical for every blocking), split by the block
    // kernel that performs each operation: for pivot k of block I with
    // n_in sub-diagonal rows inside I and n_out below it, the divisions and
    // the updates inside I belong to GETRF, the mixed updates and the
    // divisions below I to GESSM / TSTRF, the updates below I to SSSSM.
    for (int64_t k = 0; k < n; ++k) {
        const int64_t rend = an.bptr[an.bid[k] + 1];
        int64_t nin = 0, nout = 0;
        for (int64_t q = an.s_colptr[k] + 1; q < an.s_colptr[k + 1]; ++q) {
            if (an.s_rowidx[q] < rend) ++nin; else ++nout;
        }
        const double a = (double)nin, o = (double)nout, l = a + o;
        an.flops += l + 2.0 * l * l;
        an.flops_getrf += a + 2.0 * a * a;
        an.flops_panel += o + 4.0 * a * o;
        an.flops_ssssm += 2.0 * o * o;
    }

    // per level: K_i, rows_i, segments, slab offsets
    an.levels.assign(p, LevelDev());
    an.posK.assign(n, -1);
    std::vector<int32_t> mark(n, -1);
    int64_t off = 0;
    {
        std::vector<int32_t> rows;
        for (int64_t i = 0; i < p; ++i) {
            LevelDev &L = an.levels[i];
            const int64_t r0 = an.bptr[i], r1 = an.bptr[i + 1];
            L.r0 = (int32_t)r0;
            L.b = (int32_t)(r1 - r0);
            L.Koff = (int64_t)an.K_idx.size();
            L.Roff = (int64_t)an.R_idx.size();
            rows.clear();
            int32_t kap = 0;
            for (int64_t c = r0; c < r1; ++c) {
                const int64_t q0 = an.s_colptr[c], q1 = an.s_colptr[c + 1];
                if (an.s_rowidx[q1 - 1] >= r1) {
                    an.posK[c] = kap++;
                    an.K_idx.push_back((int32_t)(c - r0));
                }
                for (int64_t q = q1 - 1; q > q0 && an.s_rowidx[q] >= r1; --q) {
                    const int32_t r = an.s_rowidx[q];
                    if (mark[r] != i) {
                        mark[r] = (int32_t)i;
                        rows.push_back(r);
                    }
                }
            }
            std::sort(rows.begin(), rows.end());
            an.R_idx.insert(an.R_idx.end(), rows.begin(), rows.end());
            L.kappa = kap;
            L.m = (int32_t)rows.size();
            L.seg_begin = (int32_t)an.segs.size();
            for (size_t a = 0; a < rows.size();) {
                const int32_t k = an.bid[rows[a]];
                size_t e = a;
                while (e < rows.size() && an.bid[rows[e]] == k) ++e;
                an.segs.push_back(Segment{k, (int32_t)a, (int32_t)(e - a)});
                a = e;
            }
            L.seg_end = (int32_t)an.segs.size();
            L.offD = off;
            off += align32((int64_t)L.b * L.b);
            // P_i and Qt_i keep kappa rounded up to 16 columns; the padding
            // columns stay zero, so GEMM operand loads need no masking
            const int64_t kpad = (int64_t)(L.kappa + 15) / 16 * 16;
            L.offP = off;
            off += align32((int64_t)L.m * kpad);
            L.offQ = off;
            off += align32((int64_t)L.m * kpad);
            for (size_t a = 0, sgi = 0; a < rows.size(); ++a) {
                while (an.segs[L.seg_begin + sgi].start + an.segs[L.seg_begin + sgi].len <= (int32_t)a) ++sgi;
                an.R_seg.push_back((int32_t)sgi);
            }
            an.max_gemm_k = std::max(an.max_gemm_k, kap);
        }
    }
    an.slab_doubles = off;

    // non-empty blocks of S (both triangles): diagonal blocks + 2 * segments
    an.nonempty_blocks = p + 2 * (int64_t)an.segs.size();

    // GETRF chunks.  Blocks up to kLdsDenseMax are one LDS-resident chunk;
    // larger ones are factored right-looking in chunks of w columns, each
    // with the block rows below the chunk that S couples to it.
    std::vector<int32_t> cmark(n, 0);
    int32_t chunk_stamp = 0;
    for (int64_t i = 0; i < p; ++i) {
        LevelDev &L = an.levels[i];
        const int32_t b = L.b, r0 = L.r0;
        L.chunk_begin = (int32_t)an.chunks.size();
        if (b <= kLdsDenseMax) {
            an.chunks.push_back(ChunkDev{0, b, 0, 0, (int64_t)an.chunk_rows.size()});
            L.lds_getrf = (int32_t)((int64_t)b * b * 8);
            an.stored_flops += 2.0 / 3.0 * (double)b * b * b;
        } else {
            // widest chunk (16, 8, ...) whose panel and U part fit in LDS
            std::vector<ChunkDev> best;
            std::vector<int32_t> best_rows;
            int64_t maxl = 0, best_mnr = 0;
            double sflops = 0.0;
            for (int32_t w = 16; w >= 1; w /= 2) {
                std::vector<ChunkDev> ch;
                std::vector<int32_t> rows_all, rl;
                int64_t ml = 0, mnr = 0;
                double fl = 0.0;
                for (int32_t c0 = 0; c0 < b; c0 += w) {
                    const int32_t ww = std::min(w, b - c0);
                    const int32_t c1 = c0 + ww;
                    const int32_t stamp = ++chunk_stamp;
                    rl.clear();
                    for (int32_t c = c0; c < c1; ++c) {
                        const int64_t gc = r0 + c;
                        for (int64_t q = an.s_colptr[gc] + 1; q < an.s_colptr[gc + 1]; ++q) {
                            const int32_t r = an.s_rowidx[q];
                            if (r >= r0 + b) break;
                            if (r >= r0 + c1 && cmark[r] != stamp) {
                                cmark[r] = stamp;
                                rl.push_back(r - r0);
                            }
                        }
                    }
                    std::sort(rl.begin(), rl.end());
                    ch.push_back(ChunkDev{c0, ww, (int32_t)rl.size(), 0, (int64_t)rows_all.size()});
                    rows_all.insert(rows_all.end(), rl.begin(), rl.end());
                    const int64_t nr = (int64_t)rl.size();
                    ml = std::max<int64_t>(ml, ((int64_t)(ww + nr) * ww + (int64_t)(ww + 1) * nr) * 8);
                    mnr = std::max<int64_t>(mnr, nr);
                    fl += 2.0 * (double)nr * nr * ww + (double)(ww + 2 * nr) * ww * ww;
                }
                best.swap(ch);
                best_rows.swap(rows_all);
                // two coupled-row buffers (ints) precede the chunk's panel
                ml += ((2 * mnr + 1) / 2) * 8 + 16 * 8;   // + the pivot reciprocals
                maxl = ml;
                best_mnr = mnr;
                sflops = fl;
                if (ml <= kGetrfLdsBudget || w == 1) break;
            }
            const int64_t base = (int64_t)an.chunk_rows.size();
            for (ChunkDev &c : best) {
                c.roff += base;
                an.chunks.push_back(c);
            }
            an.chunk_rows.insert(an.chunk_rows.end(), best_rows.begin(), best_rows.end());
            an.stored_flops += sflops;
            L.lds_getrf = (int32_t)maxl;
            L.pad = (int32_t)best_mnr;
        }
        L.chunk_end = (int32_t)an.chunks.size();
    }

    // triangular-solve chunks and items
    for (int64_t i = 0; i < p; ++i) {
        LevelDev &L = an.levels[i];
        const int32_t b = L.b;
        L.sch_begin = (int32_t)an.schunks.size();
        L.sitem = (int64_t)an.sitems.size() / 2;
        int32_t item = 0;
        // a chunk with more than kSolveItems items is cut into parts of its
        // coupled rows; every part repeats the chunk's w rows as its first
        // items, and parts after the first are marked (w | kSolveCont) so
        // that only the first solves the chunk's triangle
        auto add_chunk = [&](int32_t c0, int32_t w, int32_t nr, int64_t roff) {
            int32_t done = 0;
            do {
                const int32_t part = std::min(nr - done, kSolveItems - w);
                const int32_t flag = done > 0 ? kSolveCont : 0;
                an.schunks.push_back(ChunkDev{c0, w | flag, part, item, roff + done});
                for (int32_t t = 0; t < w + part; ++t) {
                    an.sitems.push_back(t < w ? c0 + t : an.chunk_rows[roff + done + t - w]);
                    an.sitems.push_back((c0 << 5) | w);
                }
                item += w + part;
                an.max_solve_items = std::max(an.max_solve_items, w + part);
                done += part;
            } while (done < nr);
        };
        if (b <= kLdsDenseMax) {
            for (int32_t c0 = 0; c0 < b; c0 += 16) {
                const int32_t w = std::min(16, b - c0);
                const int64_t roff = (int64_t)an.chunk_rows.size();
                for (int32_t r = c0 + w; r < b; ++r) an.chunk_rows.push_back(r);
                add_chunk(c0, w, b - c0 - w, roff);
            }
        } else {
            for (int32_t c = L.chunk_begin; c < L.chunk_end; ++c) {
                const ChunkDev C = an.chunks[c];
                add_chunk(C.c0, C.w, C.nr, C.roff);
            }
        }
        L.sch_end = (int32_t)an.schunks.size();
        if (b >= (1 << 26) || an.max_solve_items > kSolveItems) return SLU_ERR_LIMIT;
        // batches of consecutive chunks
        L.sb_begin = (int32_t)an.sbatch.size() / 2;
        int32_t items = 0, nch = 0;
        for (int32_t c = L.sch_begin; c < L.sch_end; ++c) {
            const ChunkDev &C = an.schunks[c];
            const int32_t t = (C.w & ~kSolveCont) + C.nr;
            if (c == L.sch_begin || items + t > kSolveItems || nch == kSolveBatchChunks) {
                an.sbatch.push_back(c);
                an.sbatch.push_back(C.pad);
                items = 0;
                nch = 0;
            }
            items += t;
            ++nch;
        }
        an.sbatch.push_back(L.sch_end);
        an.sbatch.push_back(item);
        L.sb_end = (int32_t)an.sbatch.size() / 2;
    }

    // compact coupled triangles for the panel solves: sizes and the
    // structurally nonzero 16 x 16 tiles of U_ii[K_i, K_i]
    {
        int64_t toff = 0;
        std::vector<int64_t> keys;
        for (int64_t i = 0; i < p; ++i) {
            LevelDev &L = an.levels[i];
            const int32_t kp = (L.kappa + 15) / 16 * 16;
            const int32_t nt = kp / 16;
            L.kp = kp;
            L.offT = toff;
            toff += align32(2 * (int64_t)kp * kp + 2 * (int64_t)nt * 256);
            L.trow = (int32_t)an.trow_ptr.size();
            keys.clear();
            const int64_t r0 = L.r0, r1 = (int64_t)L.r0 + L.b;
            for (int64_t c = r0; c < r1; ++c) {
                const int32_t tc = an.posK[c];
                if (tc < 0) continue;
                for (int64_t q = an.s_colptr[c] + 1; q < an.s_colptr[c + 1]; ++q) {
                    const int32_t r = an.s_rowidx[q];
                    if (r >= r1) break;
                    const int32_t tr = an.posK[r];
                    if (tr < 0) continue;
                    // U(c, r) with c < r: tile (tc / 16, tr / 16) of the upper triangle
                    if (tr / 16 != tc / 16) keys.push_back((int64_t)(tc / 16) * nt + tr / 16);
                }
            }
            if (kp >= kPanelBlkKp && L.m > 0) {
                // blocked panel solve: it reads every upper tile of the
                // coupled triangles, so the gather writes all of them
                keys.clear();
                for (int32_t row = 0; row < nt; ++row)
                    for (int32_t col = row + 1; col < nt; ++col) keys.push_back((int64_t)row * nt + col);
            }
            std::sort(keys.begin(), keys.end());
            keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
            size_t q = 0;
            for (int32_t row = 0; row < nt; ++row) {
                an.trow_ptr.push_back((int32_t)an.trow_idx.size());
                while (q < keys.size() && keys[q] / nt == row) an.trow_idx.push_back((int32_t)(keys[q++] % nt));
            }
            an.trow_ptr.push_back((int32_t)an.trow_idx.size());
        }
        an.tri_doubles = toff;
    }

    // inverses of the kPanelBlk-column diagonal blocks of the coupled
    // triangles, for the levels that take the blocked panel solve
    {
        int64_t boff = 0;
        for (int64_t i = 0; i < p; ++i) {
            LevelDev &L = an.levels[i];
            if (L.kp >= kPanelBlkKp && L.m > 0) {
                const int64_t nbk = (L.kp + kPanelBlk - 1) / kPanelBlk;
                L.offB = boff;
                boff += 2 * nbk * kPanelBlk * kPanelBlk;
            } else {
                L.offB = -1;
            }
        }
        an.binv_doubles = boff;
    }

    // tiled GETRF work region (levels of more than one 16-row tile)
    {
        int64_t woff = 0;
        for (int64_t i = 0; i < p; ++i) {
            LevelDev &L = an.levels[i];
            const int64_t need = tgetrf_level_doubles(L.b);
            L.offW = need > 0 ? woff : -1;
            woff += align32(need);
        }
        an.tgetrf_doubles = woff;
    }

    // SSSSM: every pair (sa, sb) of segments of level i is a target
    // block (k, j) (sa-major order in stgt).  Product element (a, b), with a
    // in segment sa and b in segment sb, lands at
    //     stgt[task_begin + sa * nseg + sb] + RO[sb][a] + CO[sa][b]
    // where RO[sb] (m entries at maps[moff + sb * m]) and CO[sa] (m entries
    // at maps[moff + (nseg + sa) * m]) are the row / column offsets inside
    // the target, -1 where S has no entry there.
    // The tables are sized in level order first; then the levels fill their
    // disjoint parts on host threads (dynamic chunks of levels).
    {
        int64_t moff = 0, toff = 0;
        for (int64_t i = 0; i < p; ++i) {
            LevelDev &L = an.levels[i];
            const int32_t nseg = L.seg_end - L.seg_begin;
            L.task_begin = toff;
            L.moff = moff;
            if (L.kappa > 0) {
                an.stored_flops += 2.0 * 2.0 * (double)L.m * L.kappa * L.kappa / 2.0;
                an.stored_flops += 2.0 * (double)L.m * L.m * L.kappa;
                moff += 2 * (int64_t)nseg * L.m;
                toff += (int64_t)nseg * nseg;
            }
            L.task_end = toff;
        }
        if (toff >= ((int64_t)1 << 31) || moff >= ((int64_t)1 << 40)) return SLU_ERR_LIMIT;
        an.maps.assign((size_t)moff, -1);
        an.stgt.assign((size_t)toff, 0);
        std::atomic<int> too_big{0};
        parallel_for(p, 16, [&](int64_t i) {
            const LevelDev &L = an.levels[i];
            if (L.kappa <= 0) return;
            const int32_t *rows_i = an.R_idx.data() + L.Roff;
            const int32_t nseg = L.seg_end - L.seg_begin;
            int32_t *RO = an.maps.data() + L.moff;
            int32_t *CO = RO + (size_t)nseg * L.m;
            for (int32_t sa = 0; sa < nseg; ++sa) {
                const Segment A = an.segs[L.seg_begin + sa];
                const int32_t k = A.blk;
                const LevelDev &Lk = an.levels[k];
                for (int32_t sb = 0; sb < nseg; ++sb) {
                    const Segment B = an.segs[L.seg_begin + sb];
                    const int32_t j = B.blk;
                    const LevelDev &Lj = an.levels[j];
                    int32_t *ro = RO + (size_t)sb * L.m + A.start;   // rows of segment sa
                    int32_t *co = CO + (size_t)sa * L.m + B.start;   // columns of segment sb
                    int64_t tgt;
                    if (k == j) {
                        // diagonal block D_k, column-major
                        tgt = Lk.offD;
                        for (int32_t a = 0; a < A.len; ++a) ro[a] = rows_i[A.start + a] - Lk.r0;
                        for (int32_t c = 0; c < B.len; ++c)
                            co[c] = (rows_i[B.start + c] - Lk.r0) * Lk.b;
                    } else if (k > j) {
                        // L block (k, j) inside P_j: row = position in rows_j, column = position in K_j
                        tgt = Lj.offP;
                        const int32_t *rows_j = an.R_idx.data() + Lj.Roff;
                        sorted_pos(rows_j, Lj.m, rows_i + A.start, A.len, ro);
                        for (int32_t c = 0; c < B.len; ++c) {
                            const int64_t t = an.posK[rows_i[B.start + c]];
                            if (t >= 0 && t * Lj.m >= ((int64_t)1 << 31)) {
                                too_big.store(1);
                                return;
                            }
                            co[c] = t < 0 ? -1 : (int32_t)(t * Lj.m);
                        }
                    } else {
                        // U block (k, j) inside Qt_k: Qt_k[position in rows_k, position in K_k]
                        tgt = Lk.offQ;
                        const int32_t *rows_k = an.R_idx.data() + Lk.Roff;
                        for (int32_t a = 0; a < A.len; ++a) {
                            const int64_t t = an.posK[rows_i[A.start + a]];
                            if (t >= 0 && t * Lk.m >= ((int64_t)1 << 31)) {
                                too_big.store(1);
                                return;
                            }
                            ro[a] = t < 0 ? -1 : (int32_t)(t * Lk.m);
                        }
                        sorted_pos(rows_k, Lk.m, rows_i + B.start, B.len, co);
                    }
                    an.stgt[(size_t)L.task_begin + (size_t)sa * nseg + sb] = tgt;
                }
            }
        });
        if (too_big.load()) return SLU_ERR_LIMIT;
    }

    // schedule: waves of levels with equal height in the dependency tree of
    // the blocks.  Level i waits for every level j < i whose panels couple to
    // block i (B_ij or B_ji nonempty, so SSSSM of j updates row / column i);
    // height(i) = 1 + the largest height among those levels, so levels of one
    // wave never update each other's rows or columns.
    {
        std::vector<int32_t> height(p, 0);
        for (int64_t j = 0; j < p; ++j) {
            const LevelDev &L = an.levels[j];
            for (int32_t sgi = L.seg_begin; sgi < L.seg_end; ++sgi) {
                const int32_t i = an.segs[sgi].blk;
                height[i] = std::max(height[i], height[j] + 1);
            }
        }
        int32_t H = 0;
        for (int64_t i = 0; i < p; ++i) H = std::max(H, height[i] + 1);
        std::vector<std::vector<int32_t>> byh;
        if (opt.schedule == SLU_SCHEDULE_LEVELS) {
            for (int64_t i = 0; i < p; ++i) byh.push_back({(int32_t)i});
        } else {
            byh.assign(H, {});
            for (int64_t i = 0; i < p; ++i) byh[height[i]].push_back((int32_t)i);
        }
        for (const auto &lv : byh) {
            if (lv.empty()) continue;
            WaveInfo w{};
            w.begin = (int32_t)an.wave_levels.size();
            for (int32_t i : lv) {
                const LevelDev &L = an.levels[i];
                an.wave_levels.push_back(i);
                const int32_t lds = L.b <= kLdsDenseMax ? (int32_t)((int64_t)L.b * (L.b | 1) * 8) : L.lds_getrf;
                w.lds_getrf = std::max(w.lds_getrf, lds);
                w.max_nt = std::max(w.max_nt, L.kp / 16);
                an.tslot_off.push_back(w.tslots);
                w.tslots += L.kp / 16 + an.trow_ptr[L.trow + L.kp / 16] - an.trow_ptr[L.trow];
                w.max_kp = std::max(w.max_kp, L.kp);
                w.max_m = std::max(w.max_m, L.m);
                w.max_b = std::max(w.max_b, L.b);
                w.min_b = w.min_b == 0 ? L.b : std::min(w.min_b, L.b);
                if (L.b > 32) {
                    // share of the block's lower triangle that S fills
                    int64_t in = 0;
                    const int64_t r0 = L.r0, r1 = (int64_t)L.r0 + L.b;
                    for (int64_t c = r0; c < r1; ++c) {
                        const int32_t *lo = an.s_rowidx.data() + an.s_colptr[c];
                        const int32_t *hi = an.s_rowidx.data() + an.s_colptr[c + 1];
                        in += std::lower_bound(lo, hi, (int32_t)r1) - lo;
                    }
                    const int32_t pct = (int32_t)(100 * in / ((int64_t)L.b * (L.b + 1) / 2));
                    w.min_dense_pct = std::min(w.min_dense_pct, pct);
                }
                if (L.b <= kLdsDenseMax) w.any_dense = 1; else w.any_chunked = 1;
            }
            w.end = (int32_t)an.wave_levels.size();
            an.waves.push_back(w);
        }
        // coupled rows of every level up to its last row in a block of the
        // next wave (R is sorted, segments go by block)
        std::vector<int32_t> wave_of(p, 0), crit_rows(p, 0);
        for (size_t wi = 0; wi < an.waves.size(); ++wi)
            for (int32_t q = an.waves[wi].begin; q < an.waves[wi].end; ++q) wave_of[an.wave_levels[q]] = (int32_t)wi;
        for (int64_t i = 0; i < p; ++i) {
            const LevelDev &L = an.levels[i];
            for (int32_t sgi = L.seg_begin; sgi < L.seg_end; ++sgi)
                if (wave_of[an.segs[sgi].blk] == wave_of[i] + 1) crit_rows[i] = an.segs[sgi].start + an.segs[sgi].len;
        }
        // SSSSM rounds: levels of a wave whose sets of target blocks are
        // disjoint (first fit, in level order); a level whose blocks meet an
        // earlier level's goes to a later round, so every target receives its
        // updates in a fixed order
        std::vector<uint64_t> used(p, 0);
        for (WaveInfo &w : an.waves) {
            w.round_begin = (int32_t)an.rounds.size();
            std::vector<std::vector<int32_t>> rl;
            for (int32_t q = w.begin; q < w.end; ++q) {
                const int32_t i = an.wave_levels[q];
                const LevelDev &L = an.levels[i];
                if (L.kappa == 0 || L.m == 0) continue;
                uint64_t busy = 0;
                for (int32_t sgi = L.seg_begin; sgi < L.seg_end; ++sgi) busy |= used[an.segs[sgi].blk];
                // first free round among the first 64 (tracked by the block
                // masks); past those every level opens a round of its own
                int32_t r = 0;
                while (r < 64 && (busy >> r & 1)) ++r;
                if (r >= (int32_t)rl.size()) {
                    r = (int32_t)rl.size();
                    rl.push_back({});
                }
                rl[r].push_back(i);
                if (r < 64)
                    for (int32_t sgi = L.seg_begin; sgi < L.seg_end; ++sgi) used[an.segs[sgi].blk] |= 1ull << r;
            }
            for (int32_t q = w.begin; q < w.end; ++q) {
                const LevelDev &L = an.levels[an.wave_levels[q]];
                for (int32_t sgi = L.seg_begin; sgi < L.seg_end; ++sgi) used[an.segs[sgi].blk] = 0;
            }
            for (const auto &r : rl) {
                RoundInfo ri{};
                ri.begin = (int32_t)an.round_levels.size();
                int32_t mmax = 0;
                for (int32_t i : r) mmax = std::max(mmax, an.levels[i].m);
                ri.tile = mmax < kSsssmSmallM ? 32 : kSsssmTile;
                int64_t t = 0, tc = 0, tr = 0, td = 0, tq = 0;
                for (int32_t i : r) {
                    LevelDev &L = an.levels[i];
                    const int64_t nt = ((int64_t)L.m + ri.tile - 1) / ri.tile;
                    const int64_t nc = std::min<int64_t>(nt, ((int64_t)crit_rows[i] + ri.tile - 1) / ri.tile);
                    L.sscrit = (int32_t)nc;
                    an.round_levels.push_back(i);
                    for (int64_t v : {t, tc, tr, td, tq}) an.round_tiles.push_back(v);
                    t += nt * nt;
                    tr += (nt - nc) * (nt - nc);
                    tc += nt * nt - (nt - nc) * (nt - nc);
                    td += nc * nc;
                    tq += 2 * nc * (nt - nc);
                }
                ri.end = (int32_t)an.round_levels.size();
                ri.tiles = t;
                ri.tiles_c = tc;
                ri.tiles_r = tr;
                ri.tiles_d = td;
                ri.tiles_pq = tq;
                if (t >= ((int64_t)1 << 31)) return SLU_ERR_LIMIT;
                an.rounds.push_back(ri);
            }
            w.round_end = (int32_t)an.rounds.size();
        }
    }

    // slot of every entry of A in the slab
    an.slot.assign(an.nnz_a, -1);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t r = an.iperm[i];
        const int32_t I = an.bid[r];
        const LevelDev &LI = an.levels[I];
        for (int64_t q = an.a_rowptr[i]; q < an.a_rowptr[i + 1]; ++q) {
            const int32_t c = an.iperm[an.a_colidx[q]];
            const int32_t J = an.bid[c];
            const LevelDev &LJ = an.levels[J];
            int64_t s;
            if (I == J) {
                s = LI.offD + (int64_t)(r - LI.r0) + (int64_t)(c - LI.r0) * LI.b;
            } else if (I > J) {
                const int32_t rp = lower_pos(an.R_idx.data() + LJ.Roff, LJ.m, r);
                s = LJ.offP + rp + (int64_t)an.posK[c] * LJ.m;
            } else {
                const int32_t cp = lower_pos(an.R_idx.data() + LI.Roff, LI.m, c);
                s = LI.offQ + cp + (int64_t)an.posK[r] * LI.m;
            }
            if (s < 0 || s >= an.slab_doubles) return SLU_ERR_LIMIT;  // cannot happen for a closed S
            an.slot[q] = s;
        }
    }
    // every product element must address inside the slab
    for (int64_t i = 0; i < p; ++i) {
        const LevelDev &L = an.levels[i];
        const int32_t nseg = L.seg_end - L.seg_begin;
        if (L.task_end - L.task_begin != (L.kappa > 0 ? (int64_t)nseg * nseg : 0)) return SLU_ERR_LIMIT;
        if (L.kappa == 0) continue;
        const int32_t *RO = an.maps.data() + L.moff;
        const int32_t *CO = RO + (size_t)nseg * L.m;
        for (int32_t sa = 0; sa < nseg; ++sa) {
            const Segment A = an.segs[L.seg_begin + sa];
            for (int32_t sb = 0; sb < nseg; ++sb) {
                const Segment B = an.segs[L.seg_begin + sb];
                int64_t rmax = 0, cmax = 0;
                for (int32_t a = 0; a < A.len; ++a) rmax = std::max<int64_t>(rmax, RO[(size_t)sb * L.m + A.start + a]);
                for (int32_t c = 0; c < B.len; ++c) cmax = std::max<int64_t>(cmax, CO[(size_t)sa * L.m + B.start + c]);
                if (an.stgt[L.task_begin + (int64_t)sa * nseg + sb] + rmax + cmax >= an.slab_doubles)
                    return SLU_ERR_LIMIT;
            }
        }
    }
    (void)nnzL;
    return SLU_OK;
}

}  // namespace slu
