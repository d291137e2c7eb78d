// Joint blocks of commuting crossing gates (Sec. III-A, Sec. V).  Diagonal
// gates commute, so inside a run of consecutive diagonal gates the crossing
// ones may be reordered freely.  A set of crossing two-qubit diagonal gates
// that share one qubit (a cascade, Sec. V) has Schmidt rank at most 2:
// conditioned on the shared qubit's basis state, every gate reduces to a
// one-qubit phase on its other qubit.  Covering the crossing gates of a run
// with the fewest such stars is a minimum vertex cover of the bipartite graph
// (side-b qubits, side-a qubits; one edge per crossing gate), which by
// Koenig's theorem is read off a maximum matching.
#include <algorithm>
#include <map>
#include <set>
#include <vector>

#include "internal.h"

namespace hsf {

namespace {

struct Bipartite {
    std::vector<int> left, right;                 // qubit ids, ascending
    std::vector<std::vector<int>> adj;            // left index -> right indices, ascending
};

// Maximum matching by augmenting paths (Kuhn), deterministic order.
bool augment(const Bipartite& g, int l, std::vector<int>& match_r, std::vector<char>& seen) {
    for (int r : g.adj[l]) {
        if (seen[r]) continue;
        seen[r] = 1;
        if (match_r[r] < 0 || augment(g, match_r[r], match_r, seen)) {
            match_r[r] = l;
            return true;
        }
    }
    return false;
}

// Minimum vertex cover: (left not reachable) + (right reachable), reachable
// = along alternating paths from unmatched left vertices.
void min_cover(const Bipartite& g, std::vector<char>& cover_l, std::vector<char>& cover_r) {
    const int nl = (int)g.left.size(), nr = (int)g.right.size();
    std::vector<int> match_r(nr, -1), match_l(nl, -1);
    for (int l = 0; l < nl; ++l) {
        std::vector<char> seen(nr, 0);
        augment(g, l, match_r, seen);
    }
    for (int r = 0; r < nr; ++r)
        if (match_r[r] >= 0) match_l[match_r[r]] = r;
    std::vector<char> zl(nl, 0), zr(nr, 0);
    std::vector<int> stack;
    for (int l = 0; l < nl; ++l)
        if (match_l[l] < 0) {
            zl[l] = 1;
            stack.push_back(l);
        }
    while (!stack.empty()) {
        const int l = stack.back();
        stack.pop_back();
        for (int r : g.adj[l]) {
            if (zr[r]) continue;
            zr[r] = 1;
            const int l2 = match_r[r];
            if (l2 >= 0 && !zl[l2]) {
                zl[l2] = 1;
                stack.push_back(l2);
            }
        }
    }
    cover_l.assign(nl, 0);
    cover_r.assign(nr, 0);
    for (int l = 0; l < nl; ++l) cover_l[l] = !zl[l];
    for (int r = 0; r < nr; ++r) cover_r[r] = zr[r];
}

}  // namespace

hsf_status find_blocks(const hsf_circuit* c, int32_t cut, int64_t* order, int64_t* ids, int64_t* offs,
                       int32_t* n_blocks) {
    if (!c || !order || !ids || !offs || !n_blocks) return fail(HSF_E_ARG, "null argument");
    if (c->n_qubits < 2 || c->n_qubits > 62) return fail(HSF_E_ARG, "n_qubits must be in 2..62");
    if (c->n_gates < 0 || (c->n_gates > 0 && !c->gates)) return fail(HSF_E_ARG, "bad gate array");
    const int n = c->n_qubits;
    if (cut < 0 || cut > n - 2) return fail(HSF_E_CUT, "cut must lie in 0..n-2");
    const int64_t G = c->n_gates;
    std::vector<Gate> gs(G);
    for (int64_t i = 0; i < G; ++i) {
        hsf_status s = load_gate(c->gates[i], n, i, gs[i]);
        if (s != HSF_OK) return s;
    }
    auto crossing = [&](const Gate& g) {
        int lo = 0;
        for (int j = 0; j < g.nq; ++j) lo += g.q[j] <= cut;
        return lo > 0 && lo < g.nq;
    };
    int64_t pos = 0, nid = 0;
    int32_t nb = 0;
    offs[0] = 0;
    auto close_block = [&]() { offs[++nb] = nid; };
    for (int64_t i = 0; i < G;) {
        if (!gs[i].diag) {
            // a non-diagonal gate stays in place; crossing, it is cut alone
            order[pos] = i;
            if (crossing(gs[i])) {
                ids[nid++] = pos;
                close_block();
            }
            ++pos;
            ++i;
            continue;
        }
        int64_t j = i;
        while (j < G && gs[j].diag) ++j;
        // run [i, j) of mutually commuting gates: non-crossing gates first,
        // in circuit order, then each star's gates in turn
        std::vector<int64_t> edges, loose;
        for (int64_t t = i; t < j; ++t) {
            const Gate& g = gs[t];
            if (!crossing(g)) {
                order[pos++] = t;
            } else if (g.nq == 2) {
                edges.push_back(t);
            } else {
                loose.push_back(t);
            }
        }
        Bipartite bg;
        std::map<int, int> li, ri;
        std::set<int> ls, rs;
        for (int64_t t : edges) {
            const Gate& g = gs[t];
            const int lo = std::min(g.q[0], g.q[1]), hi = std::max(g.q[0], g.q[1]);
            ls.insert(lo);
            rs.insert(hi);
        }
        for (int q : ls) {
            li[q] = (int)bg.left.size();
            bg.left.push_back(q);
        }
        for (int q : rs) {
            ri[q] = (int)bg.right.size();
            bg.right.push_back(q);
        }
        bg.adj.assign(bg.left.size(), {});
        for (int64_t t : edges) {
            const Gate& g = gs[t];
            const int lo = std::min(g.q[0], g.q[1]), hi = std::max(g.q[0], g.q[1]);
            bg.adj[li[lo]].push_back(ri[hi]);
        }
        for (auto& a : bg.adj) {
            std::sort(a.begin(), a.end());
            a.erase(std::unique(a.begin(), a.end()), a.end());
        }
        std::vector<char> cl, cr;
        min_cover(bg, cl, cr);
        // star of each gate: its side-b qubit if that is in the cover, else its side-a qubit
        std::map<std::pair<int, int>, std::vector<int64_t>> stars;   // (side, center) -> gates
        for (int64_t t : edges) {
            const Gate& g = gs[t];
            const int lo = std::min(g.q[0], g.q[1]), hi = std::max(g.q[0], g.q[1]);
            if (cl[li[lo]]) stars[{0, lo}].push_back(t);
            else stars[{1, hi}].push_back(t);
        }
        for (const auto& st : stars) {
            for (int64_t t : st.second) {
                order[pos] = t;
                ids[nid++] = pos++;
            }
            close_block();
        }
        for (int64_t t : loose) {
            order[pos] = t;
            ids[nid++] = pos++;
            close_block();
        }
        i = j;
    }
    *n_blocks = nb;
    return HSF_OK;
}

}  // namespace hsf
