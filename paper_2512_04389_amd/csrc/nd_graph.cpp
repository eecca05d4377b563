// Graph nested dissection for patterns without grid geometry.
//
// The paper relies on a fill-reducing reordering that gathers the factor's
// nonzeros bottom-right in a bordered-block-diagonal shape (Section 1,
// Section 2.1, Fig. 2) without naming the algorithm.  This one is
// deterministic (every choice breaks ties by vertex index) and works on the
// graph of A + A^T without its diagonal:
//
//   1. Dense vertices, whose degree exceeds kDenseFactor times the mean
//      degree (and kDenseMin), are numbered last, by increasing degree then
//      index: the border of a bordered-block-diagonal matrix ends up there, as
//      the hub of Fig. 2's arrowhead does.
//   2. The remaining vertices split into connected components; each is
//      numbered on its own, in order of its smallest vertex, so independent
//      systems become independent subtrees of the elimination tree.
//   3. A connected set is bisected with a vertex separator: a level structure
//      (breadth-first levels) from a pseudo-peripheral vertex; for a few cuts
//      between consecutive levels near the middle, the bipartite graph of the
//      cut edges gets a minimum vertex cover (maximum matching and Konig's
//      construction); the smallest cover whose sides stay balanced (each at
//      most 3/4 of the set and larger than the cover) is the separator.  The
//      two sides come first (each dissected again), the separator last.
//   4. Sets of at most kLeaf vertices, and sets without a balanced cut
//      (expander-like parts, where no order avoids fill), keep their index
//      order.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "analyze.hpp"

namespace slu {
namespace {

constexpr int64_t kLeaf = 64;
constexpr double kDenseFactor = 4.0;
constexpr int64_t kDenseMin = 32;
constexpr int kCutCandidates = 6;

struct Graph {
    std::vector<int64_t> ptr;
    std::vector<int32_t> adj;
};

// Adjacency of A + A^T without the diagonal (sorted, no duplicates).
void symmetric_graph(int64_t n, const int64_t *rowptr, const int32_t *colidx, Graph *g) {
    std::vector<int64_t> deg(n + 1, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int32_t j = colidx[e];
            if (j == i) continue;
            ++deg[i + 1];
            ++deg[(int64_t)j + 1];
        }
    for (int64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
    std::vector<int32_t> tmp(deg[n]);
    std::vector<int64_t> fill(deg.begin(), deg.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            const int32_t j = colidx[e];
            if (j == i) continue;
            tmp[fill[i]++] = j;
            tmp[fill[j]++] = (int32_t)i;
        }
    g->ptr.assign(n + 1, 0);
    g->adj.clear();
    g->adj.reserve(tmp.size());
    for (int64_t i = 0; i < n; ++i) {
        std::sort(tmp.begin() + deg[i], tmp.begin() + deg[i + 1]);
        int32_t last = -1;
        for (int64_t e = deg[i]; e < deg[i + 1]; ++e)
            if (tmp[e] != last) {
                last = tmp[e];
                g->adj.push_back(last);
            }
        g->ptr[i + 1] = (int64_t)g->adj.size();
    }
}

// Work state shared by the dissection of all parts.  owner[v] names the set
// v currently belongs to (a fresh id per set), so the breadth-first searches
// stay inside their set without clearing arrays.
struct Dissector {
    const Graph &g;
    std::vector<int32_t> owner;
    std::vector<int32_t> level;    // breadth-first level inside the current set
    std::vector<int32_t> mate;     // matching partner, -1 if unmatched
    std::vector<int32_t> dist;     // Hopcroft-Karp layer of an X vertex
    std::vector<int32_t> queue;
    int32_t next_id = 1;

    explicit Dissector(const Graph &gr, int64_t n)
        : g(gr), owner(n, 0), level(n, -1), mate(n, -1), dist(n, 0), queue(n) {}

    // Breadth-first levels of the set `id` from src; returns the number of
    // levels and leaves the visit order in queue[0..count).
    int32_t bfs(int32_t src, int32_t id, int64_t *count) {
        int64_t head = 0, tail = 0;
        queue[tail++] = src;
        level[src] = 0;
        int32_t depth = 0;
        while (head < tail) {
            const int32_t v = queue[head++];
            depth = level[v];
            for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
                const int32_t u = g.adj[e];
                if (owner[u] == id && level[u] < 0) {
                    level[u] = level[v] + 1;
                    queue[tail++] = u;
                }
            }
        }
        *count = tail;
        return depth + 1;
    }

    void clear_levels(int64_t count) {
        for (int64_t q = 0; q < count; ++q) level[queue[q]] = -1;
    }

    int32_t degree_in(int32_t v, int32_t id) const {
        int32_t d = 0;
        for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) d += owner[g.adj[e]] == id;
        return d;
    }

    // A pseudo-peripheral vertex of the connected set `id` (George-Liu):
    // restart from a vertex of the last level with the smallest degree while
    // the number of levels grows.
    int32_t peripheral(const std::vector<int32_t> &set, int32_t id) {
        int32_t r = set[0];
        int32_t best = degree_in(r, id);
        for (int32_t v : set) {
            const int32_t d = degree_in(v, id);
            if (d < best || (d == best && v < r)) {
                r = v;
                best = d;
            }
        }
        int64_t cnt = 0;
        int32_t depth = bfs(r, id, &cnt);
        for (int it = 0; it < 8; ++it) {
            int32_t cand = -1, cd = 0;
            for (int64_t q = 0; q < cnt; ++q) {
                const int32_t v = queue[q];
                if (level[v] != depth - 1) continue;
                const int32_t d = degree_in(v, id);
                if (cand < 0 || d < cd || (d == cd && v < cand)) {
                    cand = v;
                    cd = d;
                }
            }
            clear_levels(cnt);
            int64_t c2 = 0;
            const int32_t d2 = bfs(cand, id, &c2);
            if (d2 <= depth) {
                clear_levels(c2);
                bfs(r, id, &cnt);
                return r;
            }
            r = cand;
            depth = d2;
            cnt = c2;
        }
        return r;   // levels of r are in place
    }

    // Minimum vertex cover of the bipartite graph of the edges between X
    // (vertices of level a) and Y (level a + 1) of the set `id`: a maximum
    // matching (Hopcroft-Karp: shortest augmenting paths in phases, from a
    // greedy start), then Konig's construction (vertices of X not reachable
    // from an unmatched X vertex by alternating paths, plus the vertices of
    // Y that are).  X, Y hold the endpoints of cut edges.
    void cover(const std::vector<int32_t> &X, const std::vector<int32_t> &Y, int32_t id, int32_t a,
               std::vector<int32_t> *out) {
        for (int32_t v : X) mate[v] = -1;
        for (int32_t v : Y) mate[v] = -1;
        auto is_y = [&](int32_t u) { return owner[u] == id && level[u] == a + 1; };
        for (int32_t x : X)
            for (int64_t e = g.ptr[x]; e < g.ptr[x + 1]; ++e) {
                const int32_t y = g.adj[e];
                if (is_y(y) && mate[y] < 0) {
                    mate[x] = y;
                    mate[y] = x;
                    break;
                }
            }
        constexpr int32_t kInf = 0x7fffffff;
        std::vector<int32_t> q, stk;
        std::vector<int64_t> pos;
        for (;;) {
            // layers of X by alternating distance from the free X vertices
            q.clear();
            for (int32_t x : X) {
                if (mate[x] < 0) {
                    dist[x] = 0;
                    q.push_back(x);
                } else {
                    dist[x] = kInf;
                }
            }
            bool reach_free = false;
            for (size_t h = 0; h < q.size(); ++h) {
                const int32_t x = q[h];
                for (int64_t e = g.ptr[x]; e < g.ptr[x + 1]; ++e) {
                    const int32_t y = g.adj[e];
                    if (!is_y(y)) continue;
                    const int32_t x2 = mate[y];
                    if (x2 < 0) {
                        reach_free = true;
                    } else if (dist[x2] == kInf) {
                        dist[x2] = dist[x] + 1;
                        q.push_back(x2);
                    }
                }
            }
            if (!reach_free) break;
            // vertex-disjoint shortest augmenting paths, depth first along
            // the layers (explicit stack; pos: next edge of each x on it)
            for (int32_t x0 : X) {
                if (mate[x0] >= 0 || dist[x0] != 0) continue;
                stk.assign(1, x0);
                pos.assign(1, g.ptr[x0]);
                while (!stk.empty()) {
                    const int32_t x = stk.back();
                    int64_t &e = pos.back();
                    int32_t go = -1, freey = -1;
                    for (; e < g.ptr[x + 1]; ++e) {
                        const int32_t y = g.adj[e];
                        if (!is_y(y)) continue;
                        const int32_t x2 = mate[y];
                        if (x2 < 0) {
                            freey = y;
                            break;
                        }
                        if (dist[x2] == dist[x] + 1) {
                            go = x2;
                            ++e;
                            break;
                        }
                    }
                    if (freey >= 0) {
                        // flip the path: stk[k] takes the y through which
                        // stk[k + 1] was reached, the last x takes freey
                        int32_t y = freey;
                        for (size_t k = stk.size(); k-- > 0;) {
                            const int32_t xk = stk[k];
                            const int32_t prev = mate[xk];
                            mate[xk] = y;
                            mate[y] = xk;
                            y = prev;
                        }
                        break;
                    }
                    if (go >= 0) {
                        stk.push_back(go);
                        pos.push_back(g.ptr[go]);
                    } else {
                        dist[x] = kInf;   // dead end for this phase
                        stk.pop_back();
                        pos.pop_back();
                    }
                }
            }
        }
        // Konig: Z = vertices reachable from unmatched X by alternating paths
        ++stamp;
        q.clear();
        for (int32_t x : X)
            if (mate[x] < 0) {
                visit_mark(x);
                q.push_back(x);
            }
        for (size_t h = 0; h < q.size(); ++h) {
            const int32_t x = q[h];
            for (int64_t e = g.ptr[x]; e < g.ptr[x + 1]; ++e) {
                const int32_t y = g.adj[e];
                if (!is_y(y) || visited(y)) continue;
                visit_mark(y);
                const int32_t x2 = mate[y];
                if (x2 >= 0 && !visited(x2)) {
                    visit_mark(x2);
                    q.push_back(x2);
                }
            }
        }
        out->clear();
        for (int32_t x : X)
            if (!visited(x)) out->push_back(x);
        for (int32_t y : Y)
            if (visited(y)) out->push_back(y);
        for (int32_t v : X) mate[v] = -1;
        for (int32_t v : Y) mate[v] = -1;
    }

    std::vector<int32_t> seen;
    int32_t stamp = 0;
    void visit_mark(int32_t v) { seen[v] = stamp; }
    bool visited(int32_t v) const { return seen[v] == stamp; }
};

struct Task {
    std::vector<int32_t> set;   // vertices, ascending
    int64_t lo;                 // first position
};

}  // namespace

void nd_graph_order(int64_t n, const int64_t *rowptr, const int32_t *colidx, std::vector<int32_t> *perm) {
    perm->assign(n, -1);
    if (n <= 0) return;
    Graph g;
    symmetric_graph(n, rowptr, colidx, &g);
    Dissector ds(g, n);
    ds.seen.assign(n, 0);

    // 1. dense vertices last
    const double mean = (double)g.adj.size() / (double)n;
    const int64_t thresh = std::max<int64_t>(kDenseMin, (int64_t)(kDenseFactor * mean));
    std::vector<int32_t> dense, rest;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t d = g.ptr[v + 1] - g.ptr[v];
        (d > thresh ? dense : rest).push_back((int32_t)v);
    }
    std::sort(dense.begin(), dense.end(), [&](int32_t a, int32_t b) {
        const int64_t da = g.ptr[a + 1] - g.ptr[a], db = g.ptr[b + 1] - g.ptr[b];
        return da != db ? da < db : a < b;
    });
    const int64_t nrest = (int64_t)rest.size();
    for (size_t k = 0; k < dense.size(); ++k) (*perm)[nrest + (int64_t)k] = dense[k];
    for (int32_t v : dense) ds.owner[v] = -1;   // outside every set

    std::vector<Task> work;
    {
        const int32_t id = ds.next_id++;
        for (int32_t v : rest) ds.owner[v] = id;
        work.push_back(Task{std::move(rest), 0});
    }
    std::vector<int32_t> comp, X, Y, sep, best_sep;
    while (!work.empty()) {
        Task t = std::move(work.back());
        work.pop_back();
        const int64_t m = (int64_t)t.set.size();
        if (m == 0) continue;
        const int32_t id = ds.owner[t.set[0]];
        if (m <= kLeaf) {
            for (int64_t k = 0; k < m; ++k) (*perm)[t.lo + k] = t.set[k];
            continue;
        }
        // 2. connected components, in order of their smallest vertex
        int64_t cnt = 0;
        ds.bfs(t.set[0], id, &cnt);
        if (cnt < m) {
            std::vector<Task> parts;
            int64_t pos = t.lo;
            for (int32_t v : t.set) {
                if (ds.owner[v] != id) continue;       // already taken by an earlier component
                int64_t c = 0;
                if (ds.level[v] < 0) ds.bfs(v, id, &c);
                else {
                    c = cnt;   // the first component's visit order is still in queue
                }
                comp.assign(ds.queue.begin(), ds.queue.begin() + c);
                ds.clear_levels(c);
                std::sort(comp.begin(), comp.end());
                const int32_t cid = ds.next_id++;
                for (int32_t u : comp) ds.owner[u] = cid;
                parts.push_back(Task{comp, pos});
                pos += (int64_t)comp.size();
            }
            for (size_t k = parts.size(); k-- > 0;) work.push_back(std::move(parts[k]));
            continue;
        }
        ds.clear_levels(cnt);
        // 3. level structure from a pseudo-peripheral vertex
        const int32_t r = ds.peripheral(t.set, id);
        (void)r;
        int32_t depth = 0;
        for (int32_t v : t.set) depth = std::max(depth, ds.level[v] + 1);
        std::vector<int64_t> lsize(depth, 0);
        for (int32_t v : t.set) ++lsize[ds.level[v]];
        if (depth < 2) {   // a clique-like set: no cut between levels
            for (int64_t k = 0; k < m; ++k) (*perm)[t.lo + k] = t.set[k];
            for (int32_t v : t.set) ds.level[v] = -1;
            continue;
        }
        // cuts between levels a and a + 1, nearest the middle first
        std::vector<int64_t> below(depth, 0);   // vertices in levels <= a
        int64_t acc = 0;
        for (int32_t a = 0; a < depth; ++a) {
            acc += lsize[a];
            below[a] = acc;
        }
        std::vector<int32_t> cand;
        for (int32_t a = 0; a + 1 < depth; ++a) cand.push_back(a);
        std::sort(cand.begin(), cand.end(), [&](int32_t x, int32_t y) {
            const int64_t dx = std::llabs(2 * below[x] - m), dy = std::llabs(2 * below[y] - m);
            return dx != dy ? dx < dy : x < y;
        });
        if ((int)cand.size() > kCutCandidates) cand.resize(kCutCandidates);
        int32_t best_a = -1;
        int64_t best_size = 0;
        for (int32_t a : cand) {
            X.clear();
            Y.clear();
            ++ds.stamp;
            for (int32_t v : t.set) {
                if (ds.level[v] != a) continue;
                bool cut = false;
                for (int64_t e = g.ptr[v]; e < g.ptr[v + 1]; ++e) {
                    const int32_t u = g.adj[e];
                    if (ds.owner[u] == id && ds.level[u] == a + 1) {
                        cut = true;
                        if (!ds.visited(u)) {
                            ds.visit_mark(u);
                            Y.push_back(u);
                        }
                    }
                }
                if (cut) X.push_back(v);
            }
            std::sort(Y.begin(), Y.end());
            ds.cover(X, Y, id, a, &sep);
            // sides after removing the separator
            int64_t sa = below[a], sb = m - below[a];
            for (int32_t v : sep) (ds.level[v] <= a ? sa : sb) -= 1;
            // balanced cuts only: both sides at most 3/4 of the set, and a
            // separator smaller than either side
            const int64_t big = std::max(sa, sb), small = std::min(sa, sb);
            if (big * 4 > 3 * m || (int64_t)sep.size() >= small) continue;
            if (best_a < 0 || (int64_t)sep.size() < best_size) {
                best_a = a;
                best_size = (int64_t)sep.size();
                best_sep = sep;
            }
        }
        if (best_a < 0) {   // no balanced cut (an expander-like set): keep index order
            for (int32_t v : t.set) ds.level[v] = -1;
            for (int64_t k = 0; k < m; ++k) (*perm)[t.lo + k] = t.set[k];
            continue;
        }
        // 4. sides first (each dissected again), separator last
        std::sort(best_sep.begin(), best_sep.end());
        const int32_t sid = ds.next_id++;
        for (int32_t v : best_sep) ds.owner[v] = sid;
        std::vector<int32_t> A, B;
        for (int32_t v : t.set) {
            if (ds.owner[v] == sid) continue;
            (ds.level[v] <= best_a ? A : B).push_back(v);
        }
        for (int32_t v : t.set) ds.level[v] = -1;
        const int64_t ls = (int64_t)best_sep.size();
        for (int64_t k = 0; k < ls; ++k) (*perm)[t.lo + m - ls + k] = best_sep[k];
        const int32_t aid = ds.next_id++, bid = ds.next_id++;
        for (int32_t v : A) ds.owner[v] = aid;
        for (int32_t v : B) ds.owner[v] = bid;
        const int64_t la = (int64_t)A.size();
        work.push_back(Task{std::move(B), t.lo + la});
        work.push_back(Task{std::move(A), t.lo});
    }
}

}  // namespace slu
