// Host symbolic analysis: pattern union, own approximate-minimum-degree
// ordering, elimination tree, postorder, column counts, supernodes (with
// relaxed amalgamation), assembly map, extend-add maps, level schedules and
// the permuted operators. See analysis.hpp.
#include "analysis.hpp"

#include <algorithm>
#include <map>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>

namespace hkkt {

std::string validate_pattern(i64 n, i64 m, const i64* Hp, const i32* Hi, const i64* Jp, const i32* Ji) {
    if (n < 1) return "n_x must be >= 1";
    if (m < 0) return "m must be >= 0";
    if (!Hp || (Hp[n] > 0 && !Hi)) return "tril(H) arrays missing";
    if (Hp[0] != 0) return "H_rowptr[0] != 0";
    for (i64 i = 0; i < n; i++) {
        if (Hp[i + 1] < Hp[i]) return "H_rowptr not monotone at row " + std::to_string(i);
        for (i64 p = Hp[i]; p < Hp[i + 1]; p++) {
            i64 c = Hi[p];
            if (c < 0 || c > i) return "tril(H) column out of range (must be 0 <= col <= row) at row " + std::to_string(i);
            if (p > Hp[i] && Hi[p - 1] >= c) return "tril(H) columns unsorted or duplicated at row " + std::to_string(i);
        }
    }
    if (m > 0) {
        if (!Jp || (Jp[m] > 0 && !Ji)) return "J arrays missing";
        if (Jp[0] != 0) return "J_rowptr[0] != 0";
        for (i64 i = 0; i < m; i++) {
            if (Jp[i + 1] < Jp[i]) return "J_rowptr not monotone at row " + std::to_string(i);
            for (i64 p = Jp[i]; p < Jp[i + 1]; p++) {
                i64 c = Ji[p];
                if (c < 0 || c >= n) return "J column out of range at row " + std::to_string(i);
                if (p > Jp[i] && Ji[p - 1] >= c) return "J columns unsorted or duplicated at row " + std::to_string(i);
            }
        }
    }
    if (n > INT32_MAX / 2 || m > INT32_MAX / 2) return "dimension too large";
    return "";
}

// ---------------------------------------------------------------------------
// symmetric graph of H_gamma without the diagonal
// ---------------------------------------------------------------------------
static void build_graph(i64 n, i64 m, const i64* Hp, const i32* Hi, const i64* Jp, const i32* Ji,
                        std::vector<i64>& ptr, std::vector<i32>& adj) {
    std::vector<i64> cnt(n + 1, 0);
    for (i64 i = 0; i < n; i++)
        for (i64 p = Hp[i]; p < Hp[i + 1]; p++)
            if (Hi[p] != i) { cnt[i + 1]++; cnt[Hi[p] + 1]++; }
    for (i64 r = 0; r < m; r++) {
        i64 k = Jp[r + 1] - Jp[r];
        for (i64 p = Jp[r]; p < Jp[r + 1]; p++) cnt[Ji[p] + 1] += k - 1;
    }
    for (i64 i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    std::vector<i32> tmp(cnt[n]);
    std::vector<i64> pos(cnt.begin(), cnt.end() - 1);
    for (i64 i = 0; i < n; i++)
        for (i64 p = Hp[i]; p < Hp[i + 1]; p++)
            if (Hi[p] != i) { tmp[pos[i]++] = Hi[p]; tmp[pos[Hi[p]]++] = (i32)i; }
    for (i64 r = 0; r < m; r++)
        for (i64 a = Jp[r]; a < Jp[r + 1]; a++)
            for (i64 b = Jp[r]; b < Jp[r + 1]; b++)
                if (a != b) tmp[pos[Ji[a]]++] = Ji[b];
    ptr.assign(n + 1, 0);
    adj.clear();
    adj.reserve(tmp.size());
    for (i64 i = 0; i < n; i++) {
        auto b = tmp.begin() + cnt[i], e = tmp.begin() + cnt[i + 1];
        std::sort(b, e);
        auto u = std::unique(b, e);
        adj.insert(adj.end(), b, u);
        ptr[i + 1] = (i64)adj.size();
    }
}

// ---------------------------------------------------------------------------
// nested dissection by level structures (George 1973), own implementation:
// a part of the graph is split by the middle level of a breadth-first level
// structure rooted at a pseudo-peripheral vertex; the separator (that
// level, less the vertices with no neighbour on the far side, which join the
// near side) is ordered after both halves, recursively. Parts that are not
// connected are ordered component by component; parts of at most `leaf`
// vertices are ordered by AMD on their induced subgraph. A more balanced
// elimination tree than minimum degree gives: fewer supernode levels (fewer
// level-synchronous steps in the triangular solves) at some more fill.
// ---------------------------------------------------------------------------
std::vector<i32> nd_order(i64 n, const std::vector<i64>& ptr, const std::vector<i32>& adj, int leaf) {
    std::vector<i32> order;
    order.reserve(n);
    std::vector<i32> part(n, 0), lev(n, -1), loc(n, -1);
    int next_part = 1;
    // BFS within part id p from root; returns the vertices in visiting
    // order, levels in lev[]
    auto bfs = [&](i32 root, int p, std::vector<i32>& q, int& height) {
        q.clear();
        q.push_back(root);
        lev[root] = 0;
        height = 0;
        for (size_t h = 0; h < q.size(); h++) {
            const i32 u = q[h];
            height = std::max(height, lev[u]);
            for (i64 e = ptr[u]; e < ptr[u + 1]; e++) {
                const i32 v = adj[e];
                if (part[v] == p && lev[v] < 0) {
                    lev[v] = lev[u] + 1;
                    q.push_back(v);
                }
            }
        }
    };
    auto clear_lev = [&](const std::vector<i32>& q) {
        for (i32 v : q) lev[v] = -1;
    };
    auto order_leaf = [&](const std::vector<i32>& vs) {
        for (size_t k = 0; k < vs.size(); k++) loc[vs[k]] = (i32)k;
        std::vector<i64> lp(vs.size() + 1, 0);
        std::vector<i32> la;
        for (size_t k = 0; k < vs.size(); k++) {
            const i32 u = vs[k];
            for (i64 e = ptr[u]; e < ptr[u + 1]; e++)
                if (loc[adj[e]] >= 0 && part[adj[e]] == part[u]) la.push_back(loc[adj[e]]);
            lp[k + 1] = (i64)la.size();
        }
        const std::vector<i32> o = amd_order((i64)vs.size(), lp, la);
        for (i32 k : o) order.push_back(vs[k]);
        for (i32 v : vs) loc[v] = -1;
    };
    // work list of parts (vertex lists, all carrying one part id); a part's
    // separator is pushed as a "done" entry below its halves so that it is
    // emitted after them
    struct Item {
        std::vector<i32> vs;
        bool emit;
    };
    std::vector<Item> stack;
    {
        std::vector<i32> all(n);
        for (i64 i = 0; i < n; i++) all[i] = (i32)i;
        stack.push_back({std::move(all), false});
    }
    std::vector<i32> q, q2;
    while (!stack.empty()) {
        Item it = std::move(stack.back());
        stack.pop_back();
        if (it.emit) {
            for (i32 v : it.vs) order.push_back(v);
            continue;
        }
        std::vector<i32>& vs = it.vs;
        if (vs.empty()) continue;
        const int p = next_part++;
        for (i32 v : vs) part[v] = p;
        if ((i64)vs.size() <= leaf) {
            order_leaf(vs);
            continue;
        }
        // pseudo-peripheral root: repeat BFS from a vertex of the last level
        int height = 0, h2 = 0;
        bfs(vs[0], p, q, height);
        if (q.size() < vs.size()) {   // not connected: this component, then the rest
            std::vector<i32> comp(q), rest;
            for (i32 v : q) lev[v] = -2;   // mark
            for (i32 v : vs)
                if (lev[v] != -2) rest.push_back(v);
            for (i32 v : comp) lev[v] = -1;
            stack.push_back({std::move(rest), false});
            stack.push_back({std::move(comp), false});
            continue;
        }
        for (int rep = 0; rep < 4; rep++) {
            // last level's vertex of smallest degree
            i32 best = q.back();
            for (size_t k = q.size(); k-- > 0 && lev[q[k]] == height;)
                if (ptr[q[k] + 1] - ptr[q[k]] < ptr[best + 1] - ptr[best]) best = q[k];
            clear_lev(q);
            bfs(best, p, q2, h2);
            if (h2 <= height) {   // no longer growing: keep this structure
                std::swap(q, q2);
                height = h2;
                break;
            }
            std::swap(q, q2);
            height = h2;
        }
        if (height < 2) {   // too shallow to split: order as a leaf
            clear_lev(q);
            order_leaf(vs);
            continue;
        }
        // separator level: the smallest level whose near side holds between
        // a third and two thirds of the part (else the level at the half)
        std::vector<i64> cnt(height + 2, 0);
        for (i32 v : q) cnt[lev[v]]++;
        int mid = -1;
        {
            const i64 tot = (i64)vs.size();
            i64 below = 0;
            int half = 1;
            for (int l = 0; l <= height; l++) {
                if (2 * (below + cnt[l]) >= tot && half == 1 && l >= 1) half = std::min(l, height - 1);
                if (l >= 1 && l <= height - 1 && 3 * below >= tot && 3 * below <= 2 * tot &&
                    (mid < 0 || cnt[l] < cnt[mid]))
                    mid = l;
                below += cnt[l];
            }
            if (mid < 0) mid = std::max(1, std::min(half, height - 1));
        }
        std::vector<i32> A, B, Sep;
        for (i32 v : q) {
            if (lev[v] < mid) A.push_back(v);
            else if (lev[v] > mid) B.push_back(v);
            else {
                bool far = false;
                for (i64 e = ptr[v]; e < ptr[v + 1] && !far; e++)
                    far = part[adj[e]] == p && lev[adj[e]] == mid + 1;
                (far ? Sep : A).push_back(v);
            }
        }
        clear_lev(q);
        stack.push_back({std::move(Sep), true});
        stack.push_back({std::move(B), false});
        stack.push_back({std::move(A), false});
    }
    return order;
}

// ---------------------------------------------------------------------------
// approximate minimum degree (Amestoy, Davis & Duff 1996), own implementation
// on a quotient graph with per-node vectors: element absorption, approximate
// external degrees, mass elimination, supervariable detection by hashing and
// aggressive absorption. Very dense nodes are ordered last.
// ---------------------------------------------------------------------------
std::vector<i32> amd_order(i64 n, const std::vector<i64>& ptr, const std::vector<i32>& adj) {
    enum : int8_t { VAR = 0, ELEM = 1, DEAD = 2, DENSE = 3 };
    std::vector<int8_t> st(n, VAR);
    std::vector<std::vector<i32>> A(n), E(n), Le(n), members(n);
    std::vector<i64> nv(n, 1), deg(n, 0), esize(n, 0);
    std::vector<i32> order;
    order.reserve(n);

    const i64 dense_thr = std::max<i64>(16, (i64)(10.0 * std::sqrt((double)n)));
    std::vector<i32> dense;
    for (i64 i = 0; i < n; i++)
        if (ptr[i + 1] - ptr[i] > dense_thr && n > 64) { st[i] = DENSE; dense.push_back((i32)i); }
    for (i64 i = 0; i < n; i++) {
        if (st[i] != VAR) continue;
        for (i64 p = ptr[i]; p < ptr[i + 1]; p++)
            if (st[adj[p]] == VAR && adj[p] != i) A[i].push_back(adj[p]);
        deg[i] = (i64)A[i].size();
    }
    i64 nlive = n - (i64)dense.size();

    // degree buckets
    std::vector<i32> head(n + 1, -1), nxt(n, -1), prv(n, -1);
    auto ins = [&](i32 i) {
        i64 d = deg[i];
        nxt[i] = head[d]; prv[i] = -1;
        if (head[d] >= 0) prv[head[d]] = i;
        head[d] = i;
    };
    auto rem = [&](i32 i) {
        if (prv[i] >= 0) nxt[prv[i]] = nxt[i]; else head[deg[i]] = nxt[i];
        if (nxt[i] >= 0) prv[nxt[i]] = prv[i];
        nxt[i] = prv[i] = -1;
    };
    for (i64 i = 0; i < n; i++) if (st[i] == VAR) ins((i32)i);

    std::vector<i64> mark(n, 0), wcnt(n, 0), wstamp(n, 0);
    i64 mtag = 0, wtag = 0;
    i64 nel = 0, mindeg = 0;
    std::vector<i32> Lp;
    std::vector<std::pair<uint64_t, i32>> hb;

    while (nel < nlive) {
        while (mindeg <= n && head[mindeg] < 0) mindeg++;
        if (mindeg > n) break;  // cannot happen
        i32 p = head[mindeg];
        rem(p);
        // ---- new element p: Lp = (A_p U  union of Le over adjacent elements) \ p
        ++mtag;
        mark[p] = mtag;
        Lp.clear();
        for (i32 e : E[p]) {
            if (st[e] != ELEM) continue;
            for (i32 i : Le[e])
                if (st[i] == VAR && mark[i] != mtag) { mark[i] = mtag; Lp.push_back(i); }
            st[e] = DEAD;                          // element absorption
            std::vector<i32>().swap(Le[e]);
        }
        for (i32 i : A[p])
            if (st[i] == VAR && mark[i] != mtag) { mark[i] = mtag; Lp.push_back(i); }
        order.push_back(p);
        for (i32 q : members[p]) order.push_back(q);
        nel += nv[p];
        st[p] = ELEM;
        std::vector<i32>().swap(A[p]);
        std::vector<i32>().swap(E[p]);
        std::vector<i32>().swap(members[p]);
        for (i32 i : Lp) rem(i);
        i64 degme = 0;
        for (i32 i : Lp) degme += nv[i];
        // ---- |Le \ Lp| for every element adjacent to Lp
        ++wtag;
        for (i32 i : Lp)
            for (i32 e : E[i]) {
                if (st[e] != ELEM) continue;
                if (wstamp[e] != wtag) { wstamp[e] = wtag; wcnt[e] = esize[e]; }
                wcnt[e] -= nv[i];
            }
        i64 nleft = nlive - nel;
        // ---- approximate degree update
        for (i32 i : Lp) {
            i64 ext = 0;
            size_t k = 0;
            for (i32 e : E[i]) {
                if (st[e] != ELEM) continue;
                if (wcnt[e] <= 0) {                // Le subset of Lp: aggressive absorption
                    st[e] = DEAD;
                    std::vector<i32>().swap(Le[e]);
                    continue;
                }
                ext += wcnt[e];
                E[i][k++] = e;
            }
            E[i].resize(k);
            E[i].push_back(p);
            i64 a = 0;
            k = 0;
            for (i32 j : A[i])
                if (st[j] == VAR && mark[j] != mtag) { A[i][k++] = j; a += nv[j]; }
            A[i].resize(k);
            i64 d = std::min(deg[i] + degme - nv[i], a + (degme - nv[i]) + ext);
            d = std::min(d, nleft - nv[i]);
            deg[i] = std::max<i64>(d, 0);
        }
        // ---- mass elimination: variables adjacent only to p
        size_t k = 0;
        for (i32 i : Lp) {
            if (A[i].empty() && E[i].size() == 1) {
                order.push_back(i);
                for (i32 q : members[i]) order.push_back(q);
                nel += nv[i];
                st[i] = DEAD;
                std::vector<i32>().swap(E[i]);
                std::vector<i32>().swap(members[i]);
            } else {
                Lp[k++] = i;
            }
        }
        Lp.resize(k);
        nleft = nlive - nel;
        // ---- supervariable detection among Lp
        hb.clear();
        for (i32 i : Lp) {
            uint64_t h = 0;
            for (i32 j : A[i]) h += (uint64_t)j * 0x9E3779B97F4A7C15ull + 1;
            for (i32 e : E[i]) h += (uint64_t)e * 0xC2B2AE3D27D4EB4Full + 7;
            h ^= (uint64_t)A[i].size() << 40 ^ (uint64_t)E[i].size() << 20;
            hb.emplace_back(h, i);
        }
        std::sort(hb.begin(), hb.end());
        for (size_t a = 0; a < hb.size();) {
            size_t b = a;
            while (b < hb.size() && hb[b].first == hb[a].first) b++;
            for (size_t x = a; x < b; x++) {
                i32 i = hb[x].second;
                if (st[i] != VAR) continue;
                bool marked = false;
                for (size_t y = x + 1; y < b; y++) {
                    i32 j = hb[y].second;
                    if (st[j] != VAR || A[j].size() != A[i].size() || E[j].size() != E[i].size()) continue;
                    if (!marked) {
                        ++mtag;
                        for (i32 t : A[i]) mark[t] = mtag;
                        for (i32 t : E[i]) mark[t] = mtag;
                        marked = true;
                    }
                    bool same = true;
                    for (i32 t : A[j]) if (mark[t] != mtag) { same = false; break; }
                    if (same) for (i32 t : E[j]) if (mark[t] != mtag) { same = false; break; }
                    if (!same) continue;
                    // merge j into i
                    nv[i] += nv[j];
                    deg[i] -= nv[j];
                    members[i].push_back(j);
                    members[i].insert(members[i].end(), members[j].begin(), members[j].end());
                    std::vector<i32>().swap(members[j]);
                    st[j] = DEAD;
                    std::vector<i32>().swap(A[j]);
                    std::vector<i32>().swap(E[j]);
                }
            }
            a = b;
        }
        // ---- finish element p, reinsert its variables
        k = 0;
        i64 es = 0;
        for (i32 i : Lp)
            if (st[i] == VAR) { Lp[k++] = i; es += nv[i]; }
        Lp.resize(k);
        Le[p] = Lp;
        esize[p] = es;
        for (i32 i : Lp) {
            deg[i] = std::max<i64>(0, std::min(deg[i], nleft - nv[i]));
            ins(i);
            if (deg[i] < mindeg) mindeg = deg[i];
        }
    }
    for (i32 d : dense) order.push_back(d);
    return order;
}

// ---------------------------------------------------------------------------
// full analysis
// ---------------------------------------------------------------------------
std::string analyze(Symbolic& S, i64 n, i64 m, const i64* Hp, const i32* Hi, const i64* Jp,
                    const i32* Ji, const i32* perm_in, const AnalyzeOptions& opt, int G, const i64* x_off,
                    const i64* y_off) {
    std::string err = validate_pattern(n, m, Hp, Hi, Jp, Ji);
    if (!err.empty()) return err;
    static const i64 zero_ptr[1] = {0};
    if (m == 0) Jp = zero_ptr;
    S = Symbolic();
    S.n = n; S.m = m;
    S.nnzH = Hp[n];
    S.nnzJ = Jp[m];
    // ---- members (uneven group) and their block structure
    if (G < 1) return "group size must be >= 1";
    S.G = G;
    if (G == 1 || !x_off || !y_off) {
        if (G > 1) return "group offsets missing";
        S.x_off = {0, n};
        S.y_off = {0, m};
    } else {
        S.x_off.assign(x_off, x_off + G + 1);
        S.y_off.assign(y_off, y_off + G + 1);
        if (S.x_off[0] != 0 || S.x_off[G] != n || S.y_off[0] != 0 || S.y_off[G] != m) return "group offsets do not cover the system";
        for (int k = 0; k < G; k++)
            if (S.x_off[k + 1] <= S.x_off[k] || S.y_off[k + 1] < S.y_off[k]) return "group offsets not increasing (every member needs n_x >= 1)";
    }
    std::vector<i32> xmem(n);
    for (int k = 0; k < G; k++)
        for (i64 i = S.x_off[k]; i < S.x_off[k + 1]; i++) xmem[i] = k;
    S.y_mem.resize(m);
    for (int k = 0; k < G; k++)
        for (i64 r = S.y_off[k]; r < S.y_off[k + 1]; r++) S.y_mem[r] = k;
    if (G > 1) {
        for (i64 i = 0; i < n; i++)
            for (i64 p = Hp[i]; p < Hp[i + 1]; p++)
                if (xmem[Hi[p]] != xmem[i]) return "tril(H) entry couples two group members at row " + std::to_string(i);
        for (i64 r = 0; r < m; r++)
            for (i64 p = Jp[r]; p < Jp[r + 1]; p++)
                if (xmem[Ji[p]] != S.y_mem[r]) return "J row " + std::to_string(r) + " has a column outside its member";
    }

    std::vector<i64> gptr;
    std::vector<i32> gadj;
    build_graph(n, m, Hp, Hi, Jp, Ji, gptr, gadj);

    // ---- ordering
    std::vector<i32> perm0;
    if (perm_in) {
        perm0.assign(perm_in, perm_in + n);
        std::vector<char> seen(n, 0);
        for (i64 k = 0; k < n; k++) {
            if (perm0[k] < 0 || perm0[k] >= n || seen[perm0[k]]) return "perm is not a permutation";
            seen[perm0[k]] = 1;
        }
    } else if (opt.ordering == 1) {
        perm0.resize(n);
        std::iota(perm0.begin(), perm0.end(), 0);
    } else if (opt.ordering == 2) {
        perm0 = nd_order(n, gptr, gadj, 256);
        if ((i64)perm0.size() != n) return "internal: nested dissection incomplete";
    } else {
        perm0 = amd_order(n, gptr, gadj);
        if ((i64)perm0.size() != n) return "internal: ordering incomplete";
    }
    if (G > 1) {
        // the members are decoupled: keep each member's pivots in its own
        // range, in the order the ordering chose (same fill per member)
        std::vector<i32> part;
        part.reserve(n);
        for (int k = 0; k < G; k++)
            for (i32 v : perm0)
                if (xmem[v] == k) part.push_back(v);
        perm0.swap(part);
    }
    std::vector<i32> ip0(n);
    for (i64 k = 0; k < n; k++) ip0[perm0[k]] = (i32)k;

    // ---- elimination tree of P A P^T (Liu, with path compression)
    std::vector<i32> parent(n, -1), anc(n, -1);
    for (i64 i = 0; i < n; i++) {
        i32 u = perm0[i];
        for (i64 q = gptr[u]; q < gptr[u + 1]; q++) {
            i32 k = ip0[gadj[q]];
            if (k >= i) continue;
            i32 r = k;
            while (anc[r] != -1 && anc[r] != i) { i32 t = anc[r]; anc[r] = (i32)i; r = t; }
            if (anc[r] == -1) { anc[r] = (i32)i; parent[r] = (i32)i; }
        }
    }
    // ---- postorder (children visited in increasing order)
    std::vector<i32> chead(n, -1), cnext(n, -1);
    for (i64 j = n - 1; j >= 0; j--)
        if (parent[j] >= 0) { cnext[j] = chead[parent[j]]; chead[parent[j]] = (i32)j; }
    std::vector<i32> post;
    post.reserve(n);
    {
        std::vector<i32> stack;
        for (i64 r = 0; r < n; r++) {
            if (parent[r] != -1) continue;
            stack.push_back((i32)r);
            while (!stack.empty()) {
                i32 v = stack.back();
                if (chead[v] >= 0) {
                    i32 c = chead[v];
                    chead[v] = cnext[c];
                    stack.push_back(c);
                } else {
                    stack.pop_back();
                    post.push_back(v);
                }
            }
        }
    }
    std::vector<i32>& perm = S.perm;
    perm.resize(n);
    std::vector<i32> newpos(n);
    for (i64 k = 0; k < n; k++) { perm[k] = perm0[post[k]]; newpos[post[k]] = (i32)k; }
    std::vector<i32> par(n);
    for (i64 k = 0; k < n; k++) { i32 o = parent[post[k]]; par[k] = o < 0 ? -1 : newpos[o]; }
    S.iperm.resize(n);
    for (i64 k = 0; k < n; k++) S.iperm[perm[k]] = (i32)k;
    const std::vector<i32>& ip = S.iperm;

    // ---- column counts by row subtrees
    std::vector<i64> cc(n, 0);   // off-diagonal count per column
    {
        std::vector<i32> mk(n, -1);
        for (i64 i = 0; i < n; i++) {
            mk[i] = (i32)i;
            i32 u = perm[i];
            for (i64 q = gptr[u]; q < gptr[u + 1]; q++) {
                i32 t = ip[gadj[q]];
                if (t >= i) continue;
                while (mk[t] != i) { mk[t] = (i32)i; cc[t]++; t = par[t]; }
            }
        }
    }
    {
        S.nnzL = 0; S.flops_proxy = 0;
        for (i64 j = 0; j < n; j++) { S.nnzL += cc[j] + 1; S.flops_proxy += (double)cc[j] * (double)cc[j]; }
        std::vector<i64> depth(n, 0);
        i64 h = 0;
        for (i64 j = n - 1; j >= 0; j--) { depth[j] = par[j] < 0 ? 1 : depth[par[j]] + 1; h = std::max(h, depth[j]); }
        S.etree_height = h;
    }
    std::vector<i32> nchild(n, 0);
    for (i64 j = 0; j < n; j++) if (par[j] >= 0) nchild[par[j]]++;

    // ---- fundamental supernodes
    std::vector<i32> fs_first;
    for (i64 j = 0; j < n; j++) {
        bool join = j > 0 && par[j - 1] == j && nchild[j] == 1 && cc[j - 1] == cc[j] + 1;
        if (!join) fs_first.push_back((i32)j);
    }
    i32 nf = (i32)fs_first.size();
    fs_first.push_back((i32)n);
    std::vector<i32> c2f(n);
    for (i32 s = 0; s < nf; s++) for (i32 j = fs_first[s]; j < fs_first[s + 1]; j++) c2f[j] = s;

    // ---- relaxed amalgamation: a supernode absorbs the child that ends right
    // before its first column while the added explicit zeros stay small.
    std::vector<i32> sfirst(nf), swidth(nf), srep(nf);
    std::vector<i64> snr(nf), strue(nf);
    std::vector<i32> sparent(nf, -1);
    for (i32 s = 0; s < nf; s++) {
        sfirst[s] = fs_first[s];
        swidth[s] = fs_first[s + 1] - fs_first[s];
        i32 last = fs_first[s + 1] - 1;
        snr[s] = swidth[s] + cc[last];
        i64 t = 0;
        for (i32 j = fs_first[s]; j <= last; j++) t += cc[j] + 1;
        strue[s] = t;
        srep[s] = s;
        sparent[s] = par[last] < 0 ? -1 : c2f[par[last]];
    }
    auto find = [&](i32 x) { while (srep[x] != x) { srep[x] = srep[srep[x]]; x = srep[x]; } return x; };
    std::vector<char> alive(nf, 1);
    if (opt.relax > 0) {
        for (i32 s = 0; s < nf; s++) {
            for (;;) {
                if (sfirst[s] == 0) break;
                i32 c = find(c2f[sfirst[s] - 1]);
                if (c == s || !alive[c] || sparent[c] < 0 || find(sparent[c]) != s) break;
                i64 w = (i64)swidth[c] + swidth[s];
                i64 nr = (i64)swidth[c] + snr[s];
                if (nr < snr[c]) break;  // cannot happen: child rows are covered
                i64 dense = w * (w + 1) / 2 + (nr - w) * w;
                i64 tru = strue[c] + strue[s];
                double z = (double)(dense - tru) / (double)dense;
                bool ok;
                if (w <= 4) ok = true;
                else if (w <= 16) ok = z < 0.5;
                else if (w <= 48) ok = z < 0.1;
                else ok = z < 0.05;
                if (opt.relax > 1) ok = ok || (w <= 32 && z < 0.6);
                if (!ok) break;
                sfirst[s] = sfirst[c];
                swidth[s] = (i32)w;
                snr[s] = nr;
                strue[s] = tru;
                alive[c] = 0;
                srep[c] = s;
            }
        }
    }
    // ---- final supernodes in column order
    std::vector<i32> order_s;
    for (i32 s = 0; s < nf; s++) if (alive[s]) order_s.push_back(s);
    std::sort(order_s.begin(), order_s.end(), [&](i32 a, i32 b) { return sfirst[a] < sfirst[b]; });
    i32 ns = (i32)order_s.size();
    S.ns = ns;
    S.sn_first.resize(ns + 1);
    for (i32 t = 0; t < ns; t++) S.sn_first[t] = sfirst[order_s[t]];
    S.sn_first[ns] = (i32)n;
    S.col2sn.resize(n);
    for (i32 t = 0; t < ns; t++) for (i32 j = S.sn_first[t]; j < S.sn_first[t + 1]; j++) S.col2sn[j] = t;

    // ---- supernode row structures: own columns, original entries below the
    // block, and the children's rows below their blocks
    S.sn_parent.assign(ns, -1);
    S.sn_rowptr.assign(ns + 1, 0);
    S.sn_rows.clear();
    {
        std::vector<i32> mk(n, -1);
        std::vector<std::vector<i32>> kids(ns);
        std::vector<i32> rows;
        for (i32 s = 0; s < ns; s++) {
            i32 f = S.sn_first[s], l = S.sn_first[s + 1];
            rows.clear();
            for (i32 j = f; j < l; j++) { rows.push_back(j); mk[j] = s; }
            for (i32 j = f; j < l; j++) {
                i32 u = perm[j];
                for (i64 q = gptr[u]; q < gptr[u + 1]; q++) {
                    i32 i = ip[gadj[q]];
                    if (i >= l && mk[i] != s) { mk[i] = s; rows.push_back(i); }
                }
            }
            for (i32 c : kids[s]) {
                for (i64 q = S.sn_rowptr[c] + (S.sn_first[c + 1] - S.sn_first[c]); q < S.sn_rowptr[c + 1]; q++) {
                    i32 i = S.sn_rows[q];
                    if (i >= l && mk[i] != s) { mk[i] = s; rows.push_back(i); }
                }
            }
            std::sort(rows.begin() + (l - f), rows.end());
            S.sn_rows.insert(S.sn_rows.end(), rows.begin(), rows.end());
            S.sn_rowptr[s + 1] = (i64)S.sn_rows.size();
            if ((i64)rows.size() > l - f) {
                i32 p = S.col2sn[rows[l - f]];
                S.sn_parent[s] = p;
                kids[p].push_back(s);
            }
        }
        S.child_ptr.assign(ns + 1, 0);
        S.child_list.clear();
        for (i32 s = 0; s < ns; s++) {
            S.child_list.insert(S.child_list.end(), kids[s].begin(), kids[s].end());
            S.child_ptr[s + 1] = (i32)S.child_list.size();
        }
    }
    // ---- offsets, relative maps
    S.sn_lptr.assign(ns + 1, 0);
    S.sn_cbptr.assign(ns + 1, 0);
    S.sn_uvptr.assign(ns + 1, 0);
    S.max_w = 0; S.max_nr = 0;
    for (i32 s = 0; s < ns; s++) {
        i64 w = S.sn_first[s + 1] - S.sn_first[s];
        i64 nr = S.sn_rowptr[s + 1] - S.sn_rowptr[s];
        S.sn_lptr[s + 1] = S.sn_lptr[s] + nr * w;
        S.sn_cbptr[s + 1] = S.sn_cbptr[s] + (nr - w) * (nr - w);
        S.sn_uvptr[s + 1] = S.sn_uvptr[s] + (nr - w);
        S.max_w = std::max<i32>(S.max_w, (i32)w);
        S.max_nr = std::max<i32>(S.max_nr, (i32)nr);
    }
    S.Lsize = S.sn_lptr[ns];
    S.CBsize = S.sn_cbptr[ns];
    S.UVsize = S.sn_uvptr[ns];
    S.relmap.assign(S.UVsize, -1);
    for (i32 s = 0; s < ns; s++) {
        i32 p = S.sn_parent[s];
        if (p < 0) continue;
        i64 w = S.sn_first[s + 1] - S.sn_first[s];
        const i32* pr = S.sn_rows.data() + S.sn_rowptr[p];
        i64 pn = S.sn_rowptr[p + 1] - S.sn_rowptr[p];
        for (i64 k = 0; k < S.sn_rowptr[s + 1] - S.sn_rowptr[s] - w; k++) {
            i32 row = S.sn_rows[S.sn_rowptr[s] + w + k];
            const i32* hit = std::lower_bound(pr, pr + pn, row);
            if (hit == pr + pn || *hit != row) return "internal: child row not in parent structure";
            S.relmap[S.sn_uvptr[s] + k] = (i32)(hit - pr);
        }
    }
    // ---- gather lists: for every row slot of a supernode, the update-vector
    // entries of its children that map onto that row (children in order)
    {
        if (S.UVsize >= (i64)INT32_MAX) return "update-vector workspace exceeds 2^31 entries";
        const i64 nrows = (i64)S.sn_rows.size();
        std::vector<i64> cnt(nrows + 1, 0);
        for (i32 s = 0; s < ns; s++) {
            const i32 p = S.sn_parent[s];
            if (p < 0) continue;
            for (i64 k = 0; k < S.sn_uvptr[s + 1] - S.sn_uvptr[s]; k++)
                cnt[S.sn_rowptr[p] + S.relmap[S.sn_uvptr[s] + k] + 1]++;
        }
        for (i64 r = 0; r < nrows; r++) cnt[r + 1] += cnt[r];
        S.ga_row.assign(2 * nrows, 0);
        for (i64 r = 0; r < nrows; r++) { S.ga_row[2 * r] = (i32)cnt[r]; S.ga_row[2 * r + 1] = (i32)(cnt[r + 1] - cnt[r]); }
        S.ga_idx.assign(cnt[nrows], 0);
        std::vector<i64> pos(cnt.begin(), cnt.end() - 1);
        for (i32 p = 0; p < ns; p++)
            for (i32 q = S.child_ptr[p]; q < S.child_ptr[p + 1]; q++) {
                const i32 c = S.child_list[q];
                for (i64 k = 0; k < S.sn_uvptr[c + 1] - S.sn_uvptr[c]; k++) {
                    const i64 slot = S.sn_rowptr[p] + S.relmap[S.sn_uvptr[c] + k];
                    S.ga_idx[pos[slot]++] = (i32)(S.sn_uvptr[c] + k);
                }
            }
    }
    // ---- levels
    {
        std::vector<i32> lev(ns, 0);
        i32 maxl = 0;
        for (i32 s = 0; s < ns; s++) {
            i32 l = 0;
            for (i32 q = S.child_ptr[s]; q < S.child_ptr[s + 1]; q++) l = std::max(l, lev[S.child_list[q]] + 1);
            lev[s] = l;
            maxl = std::max(maxl, l);
        }
        S.nlevels = ns ? maxl + 1 : 0;
        S.level_ptr.assign(S.nlevels + 1, 0);
        for (i32 s = 0; s < ns; s++) S.level_ptr[lev[s] + 1]++;
        for (i32 l = 0; l < S.nlevels; l++) S.level_ptr[l + 1] += S.level_ptr[l];
        S.level_sn.resize(ns);
        std::vector<i32> pos(S.level_ptr.begin(), S.level_ptr.end() - 1);
        for (i32 s = 0; s < ns; s++) S.level_sn[pos[lev[s]]++] = s;
        // panels stored level by level (the supernodes of a level in one
        // contiguous range, in level_sn order): a level's solve or factor
        // reads one range, and the top levels' panels can be staged as a block
        i64 off = 0;
        for (i32 q = 0; q < ns; q++) {
            const i32 s = S.level_sn[q];
            S.sn_lptr[s] = off;
            off += (i64)(S.sn_first[s + 1] - S.sn_first[s]) * (S.sn_rowptr[s + 1] - S.sn_rowptr[s]);
        }
        S.sn_lptr[ns] = off;

        // ---- contribution blocks by lifetime: the block of supernode s is
        // written while its level is factored and read while its parent's
        // level is; its range is free again from the level after the
        // parent's. Best-fit reuse of freed ranges, blocks rounded to whole
        // 256-byte lines of FP32.
        std::map<i64, i64> by_off;                 // free range offset -> size
        std::multimap<i64, i64> by_size;           // free range size -> offset
        auto drop = [&](i64 off, i64 sz) {
            auto r = by_size.equal_range(sz);
            for (auto it = r.first; it != r.second; ++it)
                if (it->second == off) { by_size.erase(it); break; }
            by_off.erase(off);
        };
        auto release = [&](i64 off, i64 sz) {
            auto nx = by_off.lower_bound(off);
            if (nx != by_off.end() && off + sz == nx->first) {
                const i64 o = nx->first, z = nx->second;
                drop(o, z);
                sz += z;
            }
            auto pv = by_off.lower_bound(off);
            if (pv != by_off.begin()) {
                --pv;
                if (pv->first + pv->second == off) {
                    const i64 o = pv->first, z = pv->second;
                    drop(o, z);
                    off = o;
                    sz += z;
                }
            }
            by_off[off] = sz;
            by_size.emplace(sz, off);
        };
        std::vector<std::vector<std::pair<i64, i64>>> frees(S.nlevels + 1);
        i64 top = 0;
        for (i32 l = 0; l < S.nlevels; l++) {
            for (const auto& f : frees[l]) release(f.first, f.second);
            for (i32 q = S.level_ptr[l]; q < S.level_ptr[l + 1]; q++) {
                const i32 s = S.level_sn[q];
                const i64 nc = (S.sn_rowptr[s + 1] - S.sn_rowptr[s]) - (S.sn_first[s + 1] - S.sn_first[s]);
                if (nc == 0) { S.sn_cbptr[s] = 0; continue; }
                if (S.sn_parent[s] < 0) return "internal: root supernode with rows below its columns";
                const i64 sz = (nc * nc + 63) / 64 * 64;
                i64 off;
                auto it = by_size.lower_bound(sz);
                if (it != by_size.end()) {
                    const i64 fo = it->second, fz = it->first;
                    drop(fo, fz);
                    off = fo;
                    if (fz > sz) { by_off[fo + sz] = fz - sz; by_size.emplace(fz - sz, fo + sz); }
                } else {
                    off = top;
                    top += sz;
                }
                S.sn_cbptr[s] = off;
                frees[lev[S.sn_parent[s]] + 1].push_back({off, sz});
            }
        }
        S.CBsize = top;
        S.sn_cbptr[ns] = top;
    }

    // ---- assembly map: every entry of tril(P H_gamma P^T) with its sources,
    // in a fixed order (H entry, then D_x + delta, then J pairs by J row)
    {
        struct Src { i64 key; i32 kind; i32 a; i32 b; i64 seq; };
        std::vector<Src> src;
        i64 npairs = 0;
        for (i64 r = 0; r < m; r++) { i64 k = Jp[r + 1] - Jp[r]; npairs += k * (k + 1) / 2; }
        src.reserve(Hp[n] + n + npairs);
        i64 seq = 0;
        auto key = [&](i64 i, i64 j) { i64 a = ip[i], b = ip[j]; if (a < b) std::swap(a, b); return b * n + a; };
        for (i64 i = 0; i < n; i++)
            for (i64 p = Hp[i]; p < Hp[i + 1]; p++) src.push_back({key(i, Hi[p]), 0, (i32)p, 0, seq++});
        for (i64 j = 0; j < n; j++) src.push_back({key(j, j), 1, (i32)j, 0, seq++});
        for (i64 r = 0; r < m; r++)
            for (i64 a = Jp[r]; a < Jp[r + 1]; a++)
                for (i64 b = Jp[r]; b <= a; b++) src.push_back({key(Ji[a], Ji[b]), 2, (i32)a, (i32)b, seq++});
        std::sort(src.begin(), src.end(), [](const Src& x, const Src& y) { return x.key != y.key ? x.key < y.key : x.seq < y.seq; });
        S.a_dst.clear(); S.a_h.clear(); S.a_d.clear(); S.a_pa.clear(); S.a_pb.clear();
        S.a_pptr.assign(1, 0);
        for (size_t q = 0; q < src.size();) {
            size_t e = q;
            i64 k = src[q].key;
            i64 j = k / n, i = k % n;   // column j, row i >= j (permuted)
            i32 s = S.col2sn[j];
            const i32* rb = S.sn_rows.data() + S.sn_rowptr[s];
            i64 nr = S.sn_rowptr[s + 1] - S.sn_rowptr[s];
            const i32* hit = std::lower_bound(rb, rb + nr, (i32)i);
            if (hit == rb + nr || *hit != i) return "internal: entry outside supernode structure";
            S.a_dst.push_back(S.sn_lptr[s] + (j - S.sn_first[s]) * nr + (hit - rb));
            i32 h = -1, d = -1;
            while (e < src.size() && src[e].key == k) {
                if (src[e].kind == 0) h = src[e].a;
                else if (src[e].kind == 1) d = src[e].a;
                else { S.a_pa.push_back(src[e].a); S.a_pb.push_back(src[e].b); }
                e++;
            }
            S.a_h.push_back(h);
            S.a_d.push_back(d);
            S.a_pptr.push_back((i64)S.a_pa.size());
            q = e;
        }
        S.nnzA = (i64)S.a_dst.size();
    }
    // ---- operators in the permuted order
    S.J_rowptr.assign(Jp, Jp + m + 1);
    S.J_colp.resize(S.nnzJ);
    for (i64 p = 0; p < S.nnzJ; p++) S.J_colp[p] = ip[Ji[p]];
    {
        S.JT_rowptr.assign(n + 1, 0);
        for (i64 p = 0; p < S.nnzJ; p++) S.JT_rowptr[S.J_colp[p] + 1]++;
        for (i64 i = 0; i < n; i++) S.JT_rowptr[i + 1] += S.JT_rowptr[i];
        S.JT_col.resize(S.nnzJ);
        S.JT_src.resize(S.nnzJ);
        std::vector<i64> pos(S.JT_rowptr.begin(), S.JT_rowptr.end() - 1);
        for (i64 r = 0; r < m; r++)
            for (i64 p = Jp[r]; p < Jp[r + 1]; p++) {
                i64 c = S.J_colp[p];
                S.JT_col[pos[c]] = (i32)r;
                S.JT_src[pos[c]] = (i32)p;
                pos[c]++;
            }
    }
    {
        S.HF_rowptr.assign(n + 1, 0);
        for (i64 i = 0; i < n; i++)
            for (i64 p = Hp[i]; p < Hp[i + 1]; p++) {
                S.HF_rowptr[ip[i] + 1]++;
                if (Hi[p] != i) S.HF_rowptr[ip[Hi[p]] + 1]++;
            }
        for (i64 i = 0; i < n; i++) S.HF_rowptr[i + 1] += S.HF_rowptr[i];
        i64 nz = S.HF_rowptr[n];
        S.HF_col.resize(nz);
        S.HF_src.resize(nz);
        std::vector<i64> pos(S.HF_rowptr.begin(), S.HF_rowptr.end() - 1);
        for (i64 i = 0; i < n; i++)
            for (i64 p = Hp[i]; p < Hp[i + 1]; p++) {
                i64 a = ip[i], b = ip[Hi[p]];
                S.HF_col[pos[a]] = (i32)b; S.HF_src[pos[a]] = (i32)p; pos[a]++;
                if (a != b) { S.HF_col[pos[b]] = (i32)a; S.HF_src[pos[b]] = (i32)p; pos[b]++; }
            }
    }
    // ---- member maps and member-aligned reduction blocks
    S.xp_mem.resize(n);
    for (i64 k = 0; k < n; k++) {
        S.xp_mem[k] = xmem[perm[k]];
        if (S.xp_mem[k] != xmem[k]) return "internal: elimination order mixes group members";
    }
    S.a_mem.resize(S.nnzA);
    S.sn_mem.resize(ns);
    for (i32 s2 = 0; s2 < ns; s2++) S.sn_mem[s2] = S.xp_mem[S.sn_first[s2]];
    {
        // supernode whose panel holds the entry (panels ordered by offset)
        std::vector<std::pair<i64, i32>> po(ns);
        for (i32 s2 = 0; s2 < ns; s2++) po[s2] = {S.sn_lptr[s2], s2};
        std::sort(po.begin(), po.end());
        for (i64 e = 0; e < S.nnzA; e++) {
            const size_t k = (size_t)(std::upper_bound(po.begin(), po.end(), std::make_pair(S.a_dst[e], INT32_MAX)) -
                                      po.begin()) - 1;
            S.a_mem[e] = S.sn_mem[po[k].second];
        }
    }
    S.mblk.clear();
    S.mblk_off.assign(G + 1, 0);
    for (int k = 0; k < G; k++) {
        S.mblk_off[k] = (i32)(S.mblk.size() / 3);
        for (i64 r = S.y_off[k]; r < S.y_off[k + 1]; r += kRedBlock) {
            S.mblk.push_back((i32)r);
            S.mblk.push_back((i32)std::min<i64>(r + kRedBlock, S.y_off[k + 1]));
            S.mblk.push_back(k);
        }
    }
    S.mblk_off[G] = (i32)(S.mblk.size() / 3);
    S.rblk.clear();
    S.rblk_off.assign(G + 1, 0);
    for (int k = 0; k < G; k++) {
        S.rblk_off[k] = (i32)(S.rblk.size() / 3);
        for (i64 i = S.x_off[k]; i < S.x_off[k + 1]; i += kRedBlock) {
            S.rblk.push_back((i32)i);
            S.rblk.push_back((i32)std::min<i64>(i + kRedBlock, S.x_off[k + 1]));
            S.rblk.push_back(k);
        }
        for (i64 r = S.y_off[k]; r < S.y_off[k + 1]; r += kRedBlock) {
            S.rblk.push_back((i32)(n + r));
            S.rblk.push_back((i32)(n + std::min<i64>(r + kRedBlock, S.y_off[k + 1])));
            S.rblk.push_back(k);
        }
    }
    S.rblk_off[G] = (i32)(S.rblk.size() / 3);
    return "";
}

}  // namespace hkkt
