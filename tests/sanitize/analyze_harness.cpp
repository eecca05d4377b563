// Host analysis under the address / undefined-behaviour / thread sanitizers:
// slu::analyze on grids, random unsymmetric patterns, a bordered
// block-diagonal matrix and stacked independent systems, in every ordering,
// with one and several host threads; the plans must not depend on the
// thread count.  Prints "ok" on success, exits non-zero on a mismatch.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "analyze.hpp"

namespace {

struct Csr {
    int64_t n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
};

Csr from_lists(int64_t n, std::vector<std::vector<int32_t>> &rows) {
    Csr a;
    a.n = n;
    a.rp.assign(1, 0);
    for (int64_t i = 0; i < n; ++i) {
        std::vector<int32_t> &r = rows[i];
        r.push_back((int32_t)i);
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        a.ci.insert(a.ci.end(), r.begin(), r.end());
        a.rp.push_back((int64_t)a.ci.size());
    }
    return a;
}

Csr grid(int nx, int ny, int nz) {
    const int64_t n = (int64_t)nx * ny * nz;
    std::vector<std::vector<int32_t>> rows(n);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int32_t i = x + nx * (y + ny * z);
                if (x > 0) rows[i].push_back(i - 1);
                if (x + 1 < nx) rows[i].push_back(i + 1);
                if (y > 0) rows[i].push_back(i - nx);
                if (y + 1 < ny) rows[i].push_back(i + nx);
                if (z > 0) rows[i].push_back(i - nx * ny);
                if (z + 1 < nz) rows[i].push_back(i + nx * ny);
            }
    return from_lists(n, rows);
}

Csr random_unsym(int64_t n, int per_row, unsigned seed) {
    std::mt19937 rng(seed);
    std::vector<std::vector<int32_t>> rows(n);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < per_row; ++k) rows[i].push_back((int32_t)(rng() % n));
    return from_lists(n, rows);
}

Csr bbd(int nblocks, int bsize, int border, int border_nnz, unsigned seed) {
    std::mt19937 rng(seed);
    const int64_t inner = (int64_t)nblocks * bsize, n = inner + border;
    std::vector<std::vector<int32_t>> rows(n);
    for (int b = 0; b < nblocks; ++b)
        for (int i = 0; i < bsize; ++i)
            for (int k = 0; k < 4; ++k) rows[b * bsize + i].push_back((int32_t)(b * bsize + rng() % bsize));
    for (int e = 0; e < border_nnz; ++e) {
        rows[inner + rng() % border].push_back((int32_t)(rng() % n));
        rows[rng() % n].push_back((int32_t)(inner + rng() % border));
    }
    return from_lists(n, rows);
}

bool same_plan(const slu::Analysis &a, const slu::Analysis &b) {
    return a.perm == b.perm && a.s_colptr == b.s_colptr && a.s_rowidx == b.s_rowidx && a.bptr == b.bptr &&
           a.maps == b.maps && a.stgt == b.stgt && a.chunk_rows == b.chunk_rows && a.slot == b.slot &&
           a.wave_levels == b.wave_levels && a.round_levels == b.round_levels && a.sitems == b.sitems &&
           a.slab_doubles == b.slab_doubles && a.tgetrf_doubles == b.tgetrf_doubles &&
           a.round_tiles == b.round_tiles;
}

// The Schur-update split of every round: critical and other tiles add up to
// all tiles (three prefix counts per level), and no tile outside a level's
// first sscrit tile rows and columns holds a coupled row of a block in the
// next wave.
bool split_ok(const slu::Analysis &an) {
    std::vector<int32_t> wave_of(an.levels.size(), 0);
    for (size_t wi = 0; wi < an.waves.size(); ++wi)
        for (int32_t q = an.waves[wi].begin; q < an.waves[wi].end; ++q) wave_of[an.wave_levels[q]] = (int32_t)wi;
    if (an.round_tiles.size() != 5 * an.round_levels.size()) return false;
    for (const slu::RoundInfo &r : an.rounds) {
        if (r.tiles_c + r.tiles_r != r.tiles || r.tiles_d + r.tiles_pq != r.tiles_c) return false;
        int64_t t = 0, tc = 0, tr = 0, td = 0, tq = 0;
        for (int32_t q = r.begin; q < r.end; ++q) {
            if (an.round_tiles[5 * q] != t || an.round_tiles[5 * q + 1] != tc || an.round_tiles[5 * q + 2] != tr ||
                an.round_tiles[5 * q + 3] != td || an.round_tiles[5 * q + 4] != tq)
                return false;
            const int32_t i = an.round_levels[q];
            const slu::LevelDev &L = an.levels[i];
            const int64_t nt = ((int64_t)L.m + r.tile - 1) / r.tile, nc = L.sscrit;
            if (nc < 0 || nc > nt) return false;
            t += nt * nt;
            tc += nt * nt - (nt - nc) * (nt - nc);
            tr += (nt - nc) * (nt - nc);
            td += nc * nc;
            tq += 2 * nc * (nt - nc);
            for (int32_t sgi = L.seg_begin; sgi < L.seg_end; ++sgi) {
                const slu::Segment &g = an.segs[sgi];
                if (wave_of[g.blk] == wave_of[i] + 1 && (int64_t)(g.start + g.len) > nc * r.tile) return false;
            }
        }
        if (t != r.tiles || tc != r.tiles_c || tr != r.tiles_r || td != r.tiles_d || tq != r.tiles_pq) return false;
    }
    return true;
}

int run(const char *name, const Csr &a, slu_options o, const std::vector<int64_t> *seg = nullptr) {
    slu::Analysis one, many;
    slu::set_host_threads(1);
    int rc1 = slu::analyze(a.n, a.rp.data(), a.ci.data(), o, &one, seg);
    slu::set_host_threads(8);
    int rc8 = slu::analyze(a.n, a.rp.data(), a.ci.data(), o, &many, seg);
    if (rc1 != SLU_OK || rc8 != SLU_OK || !same_plan(one, many)) {
        std::fprintf(stderr, "%s: rc %d / %d or plans differ\n", name, rc1, rc8);
        return 1;
    }
    if (!split_ok(one)) {
        std::fprintf(stderr, "%s: Schur-update split reaches the next wave\n", name);
        return 1;
    }
    std::printf("%s: n %lld levels %lld nnz(S) %lld\n", name, (long long)a.n, (long long)one.p,
                (long long)(2 * (one.s_colptr.back() - a.n) + a.n));
    return 0;
}

}  // namespace

int main() {
    int bad = 0;
    slu_options o;
    slu_default_options(&o);
    Csr g2 = grid(30, 30, 1), g3 = grid(10, 10, 10), ru = random_unsym(400, 2, 7), bb = bbd(4, 120, 30, 1500, 3);
    bad += run("grid2d natural", g2, o);
    slu_options og = o;
    og.ordering = SLU_ORDER_GRID_ND;
    og.grid_dims[0] = 30, og.grid_dims[1] = 30, og.grid_dims[2] = 1;
    bad += run("grid2d grid-nd", g2, og);
    og.grid_dims[0] = 10, og.grid_dims[1] = 10, og.grid_dims[2] = 10;
    bad += run("grid3d grid-nd", g3, og);
    og.blocking = SLU_BLOCK_REGULAR;
    og.regular_block = 150;
    bad += run("grid3d grid-nd regular 150", g3, og);
    slu_options on = o;
    on.ordering = SLU_ORDER_GRAPH_ND;
    bad += run("grid3d graph-nd", g3, on);
    bad += run("random graph-nd", ru, on);
    bad += run("bbd graph-nd", bb, on);
    bad += run("bbd natural", bb, o);
    slu_options ou = o;
    std::vector<int32_t> perm(ru.n);
    for (int64_t i = 0; i < ru.n; ++i) perm[i] = (int32_t)((i * 7919) % ru.n);
    ou.ordering = SLU_ORDER_USER;
    ou.user_perm = perm.data();
    bad += run("random user order", ru, ou);
    // stacked independent systems (the batch path): two grids and a bbd
    Csr s1 = grid(16, 16, 1), s2 = grid(7, 7, 7), s3 = bbd(3, 60, 15, 400, 5);
    Csr st;
    st.rp.assign(1, 0);
    std::vector<int64_t> seg(1, 0);
    for (const Csr *c : {&s1, &s2, &s3}) {
        const int64_t off = st.n;
        for (int64_t i = 0; i < c->n; ++i) {
            for (int64_t e = c->rp[i]; e < c->rp[i + 1]; ++e) st.ci.push_back((int32_t)(c->ci[e] + off));
            st.rp.push_back((int64_t)st.ci.size());
        }
        st.n += c->n;
        seg.push_back(st.n);
    }
    bad += run("stacked systems natural", st, o, &seg);
    // malformed input is rejected, not read out of bounds
    {
        Csr m = g2;
        m.ci[5] = (int32_t)m.n;
        slu::Analysis an;
        if (slu::analyze(m.n, m.rp.data(), m.ci.data(), o, &an) != SLU_ERR_COLIDX) bad += 1;
    }
    if (bad) return 1;
    std::printf("ok\n");
    return 0;
}
