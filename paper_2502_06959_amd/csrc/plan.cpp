// Host planner: partition, block hulls, block operators, operator-Schmidt
// decomposition, path table, side programs and their LDS pass schedule.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <queue>
#include <set>
#include <utility>

#include "internal.h"

namespace hsf {

namespace {

bool matrix_is_diag(const std::vector<cd>& m, int d) {
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            if (i != j && m[(size_t)i * d + j] != cd(0)) return false;
    return true;
}

// U <- G U, where G acts on local bits lb[0..k) (lb[0] most significant) of
// an nl-qubit register and U is a row-major 2^nl x 2^nl matrix.
void left_multiply(std::vector<cd>& U, int nl, const int* lb, int k, const std::vector<cd>& g) {
    const int d = 1 << nl, dk = 1 << k;
    int mask = 0;
    for (int i = 0; i < k; ++i) mask |= 1 << lb[i];
    std::vector<cd> v(dk);
    std::vector<int> idx(dk);
    for (int base = 0; base < d; ++base) {
        if (base & mask) continue;
        for (int j = 0; j < dk; ++j) {
            int x = base;
            for (int i = 0; i < k; ++i)
                if ((j >> (k - 1 - i)) & 1) x |= 1 << lb[i];
            idx[j] = x;
        }
        for (int c = 0; c < d; ++c) {
            for (int j = 0; j < dk; ++j) v[j] = U[(size_t)idx[j] * d + c];
            for (int r = 0; r < dk; ++r) {
                cd acc = 0;
                for (int j = 0; j < dk; ++j) acc += g[(size_t)r * dk + j] * v[j];
                U[(size_t)idx[r] * d + c] = acc;
            }
        }
    }
}

// Gates reachable from the seed set along shared-qubit succession, forward
// (later gates) or backward (earlier gates).
std::vector<char> closure(const std::vector<Gate>& gs, int n, const std::vector<char>& seed, bool fwd) {
    std::vector<char> in = seed;
    std::vector<char> last(n, 0);
    const int64_t G = (int64_t)gs.size();
    for (int64_t t = 0; t < G; ++t) {
        const int64_t i = fwd ? t : G - 1 - t;
        bool r = in[i];
        for (int j = 0; j < gs[i].nq && !r; ++j) r = last[gs[i].q[j]];
        in[i] = r;
        for (int j = 0; j < gs[i].nq; ++j) last[gs[i].q[j]] = r;
    }
    return in;
}

}  // namespace

namespace {

// Counts singular values above the plan's tolerance; fails inside the
// ambiguity window around it.
hsf_status count_rank(const Plan& p, const std::vector<double>& sigma, int& rank) {
    const double s0 = sigma.empty() ? 0.0 : sigma[0];
    if (!(s0 > 0)) return fail(HSF_E_RANK_AMBIGUOUS, "operator is zero");
    int r = 0;
    for (double sv : sigma) {
        const double rel = sv / s0;
        if (rel > p.rank_tol * 1e-3 && rel <= p.rank_tol * 1e3)
            return fail(HSF_E_RANK_AMBIGUOUS, "singular value ratio " + std::to_string(rel) + " near the rank tolerance");
        if (rel > p.rank_tol) ++r;
    }
    rank = r;
    return HSF_OK;
}

// Diagonal entry of gate g (matrix m) at the basis state given by bit(q).
template <typename BitOf>
cd diag_entry(const Gate& g, const std::vector<cd>& m, BitOf bit) {
    int idx = 0;
    for (int j = 0; j < g.nq; ++j) idx |= bit(g.q[j]) << (g.nq - 1 - j);
    const int d = 1 << g.nq;
    return m[(size_t)idx * d + idx];
}

// Product form (computational basis of the narrow side s, Sec. IV's
// cascade example): possible when every hull gate is diagonal and touches at
// most one qubit of the wide side.  Then U = sum_m c(m) |m><m| (x) prod_j
// diag(phi_j(m, 0), phi_j(m, 1)).  Taken only when its rank 2^|s| is the
// operator's Schmidt rank (the singular values of u(m, x_wide)).
hsf_status try_product(const Plan& p, const Block& blk, int64_t gate_id, double param, Factors& f,
                       bool& taken) {
    taken = false;
    const int ka = (int)blk.sa.size(), kb = (int)blk.sb.size();
    if (ka == 0 || kb == 0) return HSF_OK;
    for (int64_t gi : blk.hull)
        if (!p.gates[gi].diag) return HSF_OK;
    std::vector<cd> alt;
    auto mat = [&](int64_t gi) -> const std::vector<cd>& {
        if (gi != gate_id) return p.gates[gi].m;
        gate_matrix(p.gates[gi].kind, p.gates[gi].nq, param, nullptr, alt);
        return alt;
    };
    for (int narrow_a = 0; narrow_a < 2; ++narrow_a) {
        // try the smaller side first (side b on a tie)
        const bool a_narrow = (ka < kb) ? narrow_a == 0 : narrow_a == 1;
        const std::vector<int>& sq = a_narrow ? blk.sa : blk.sb;
        const std::vector<int>& wq = a_narrow ? blk.sb : blk.sa;
        const int ks = (int)sq.size(), kw = (int)wq.size();
        if (ks > 4 || kw > kMaxProductSide) continue;
        std::vector<int> wpos(64, -1), spos(64, -1);
        for (int j = 0; j < kw; ++j) wpos[wq[j]] = j;
        for (int i = 0; i < ks; ++i) spos[sq[i]] = i;
        // gates: the wide qubit each one touches (-1: none)
        std::vector<int> wide_of;
        bool ok = true;
        for (int64_t gi : blk.hull) {
            const Gate& g = p.gates[gi];
            int w = -1, nw = 0;
            for (int j = 0; j < g.nq; ++j)
                if (wpos[g.q[j]] >= 0) {
                    w = wpos[g.q[j]];
                    ++nw;
                }
            if (nw > 1) ok = false;
            wide_of.push_back(w);
        }
        if (!ok) continue;
        const int R = 1 << ks;
        // c(m) and phi_j(m, z)
        std::vector<cd> c(R, cd(1.0)), phi((size_t)R * kw * 2, cd(1.0));
        for (int m = 0; m < R; ++m)
            for (size_t h = 0; h < blk.hull.size(); ++h) {
                const int64_t gi = blk.hull[h];
                const Gate& g = p.gates[gi];
                const std::vector<cd>& gm = mat(gi);
                const int w = wide_of[h];
                if (w < 0) {
                    c[m] *= diag_entry(g, gm, [&](int q) { return (m >> spos[q]) & 1; });
                    continue;
                }
                for (int z = 0; z < 2; ++z)
                    phi[((size_t)m * kw + w) * 2 + z] *=
                        diag_entry(g, gm, [&](int q) { return spos[q] >= 0 ? (m >> spos[q]) & 1 : z; });
            }
        // Schmidt coefficients: singular values of u(m, x_w) (rows m)
        const int64_t W = int64_t(1) << kw;
        std::vector<cd> u((size_t)R * W);
        for (int m = 0; m < R; ++m)
            for (int64_t x = 0; x < W; ++x) {
                cd v = c[m];
                for (int j = 0; j < kw; ++j) v *= phi[((size_t)m * kw + j) * 2 + ((x >> j) & 1)];
                u[(size_t)m * W + x] = v;
            }
        std::vector<cd> Wl, Vh;
        std::vector<double> sigma;
        jacobi_svd(R, (int)W, u, Wl, sigma, Vh);
        int rank = 0;
        hsf_status st = count_rank(p, sigma, rank);
        if (st != HSF_OK) return st;
        if (rank != R) continue;
        f.sigma = sigma;
        f.rank = R;
        f.product = true;
        std::vector<FactorPiece> ns(ks), ws(kw);
        for (int i = 0; i < ks; ++i) {
            ns[i].q = {sq[i]};
            ns[i].m.assign((size_t)R * 4, cd(0));
            for (int m = 0; m < R; ++m) {
                const int bit = (m >> i) & 1;
                ns[i].m[(size_t)m * 4 + bit * 3] = i == 0 ? c[m] : cd(1.0);
            }
        }
        for (int j = 0; j < kw; ++j) {
            ws[j].q = {wq[j]};
            ws[j].m.assign((size_t)R * 4, cd(0));
            for (int m = 0; m < R; ++m) {
                ws[j].m[(size_t)m * 4] = phi[((size_t)m * kw + j) * 2];
                ws[j].m[(size_t)m * 4 + 3] = phi[((size_t)m * kw + j) * 2 + 1];
            }
        }
        f.pa = a_narrow ? ns : ws;
        f.pb = a_narrow ? ws : ns;
        taken = true;
        return HSF_OK;
    }
    return HSF_OK;
}

}  // namespace

// The block operator with gate `gate_id` at `param` (gate_id < 0: unchanged),
// reshaped for the operator-Schmidt decomposition (Sec. IV-A): rows (i_b,
// j_b), columns (i_a, j_a).
static void reshaped_block(const Plan& p, const Block& blk, int64_t gate_id, double param, std::vector<cd>& At) {
    const int ka = (int)blk.sa.size(), kb = (int)blk.sb.size(), nl = ka + kb;
    const int da = 1 << ka, db = 1 << kb, d = 1 << nl;
    int local[64];
    for (int i = 0; i < kb; ++i) local[blk.sb[i]] = i;
    for (int i = 0; i < ka; ++i) local[blk.sa[i]] = kb + i;
    std::vector<cd> U((size_t)d * d, cd(0));
    for (int i = 0; i < d; ++i) U[(size_t)i * d + i] = 1.0;
    std::vector<cd> alt;
    for (int64_t gi : blk.hull) {
        const Gate& g = p.gates[gi];
        int lb[4];
        for (int j = 0; j < g.nq; ++j) lb[j] = local[g.q[j]];
        const std::vector<cd>* m = &g.m;
        if (gi == gate_id) {
            gate_matrix(g.kind, g.nq, param, nullptr, alt);
            m = &alt;
        }
        left_multiply(U, nl, lb, g.nq, *m);
    }
    const int rows = db * db, cols = da * da;
    At.assign((size_t)rows * cols, cd(0));
    for (int ia = 0; ia < da; ++ia)
        for (int ib = 0; ib < db; ++ib)
            for (int ja = 0; ja < da; ++ja)
                for (int jb = 0; jb < db; ++jb)
                    At[(size_t)(ib * db + jb) * cols + (ia * da + ja)] = U[(size_t)(ia * db + ib) * d + (ja * db + jb)];
}

// Factor pieces from a decomposition At = sum_m Y_m X_m^T with the singular
// values folded in (Y_m = sqrt(s_m) W[:, m], X_m = sqrt(s_m) Vh[m, :]).
static void pieces_from_svd(const Block& blk, int r, const std::vector<double>& sig, const std::vector<cd>& W,
                            int w_ld, const std::vector<cd>& Vh, int vh_ld, Factors& f) {
    const int ka = (int)blk.sa.size(), kb = (int)blk.sb.size();
    const int da = 1 << ka, db = 1 << kb;
    std::vector<cd> xa((size_t)r * da * da, cd(0)), yb((size_t)r * db * db, cd(0));
    for (int m = 0; m < r; ++m) {
        const double rt = std::sqrt(sig[m]);
        for (int e = 0; e < da * da; ++e) xa[(size_t)m * da * da + e] = rt * Vh[(size_t)m * vh_ld + e];
        for (int e = 0; e < db * db; ++e) yb[(size_t)m * db * db + e] = rt * W[(size_t)m * w_ld + e];
    }
    // a side with no qubit in the block carries a scalar: fold it into the other side
    if (ka == 0)
        for (int m = 0; m < r; ++m)
            for (int e = 0; e < db * db; ++e) yb[(size_t)m * db * db + e] *= xa[m];
    if (kb == 0)
        for (int m = 0; m < r; ++m)
            for (int e = 0; e < da * da; ++e) xa[(size_t)m * da * da + e] *= yb[m];
    if (ka > 0) f.pa.push_back(FactorPiece{blk.sa, std::move(xa)});
    if (kb > 0) f.pb.push_back(FactorPiece{blk.sb, std::move(yb)});
}

hsf_status factor_block(const Plan& p, const Block& blk, int64_t gate_id, double param, Factors& f) {
    const int ka = (int)blk.sa.size(), kb = (int)blk.sb.size();
    f = Factors();
    bool taken = false;
    hsf_status ps = try_product(p, blk, gate_id, param, f, taken);
    if (ps != HSF_OK || taken) return ps;
    if (ka > p.max_side || kb > p.max_side)
        return fail(HSF_E_BLOCK_TOO_LARGE, "support " + std::to_string(ka) + "|" + std::to_string(kb) +
                                               " exceeds the per-side limit of SVD-factored blocks");
    std::vector<cd> At;
    reshaped_block(p, blk, gate_id, param, At);
    const int rows = 1 << (2 * kb), cols = 1 << (2 * ka);
    std::vector<cd> W, Vh;
    jacobi_svd(rows, cols, At, W, f.sigma, Vh);
    int r = 0;
    hsf_status st = count_rank(p, f.sigma, r);
    if (st != HSF_OK) return st;
    f.rank = r;
    pieces_from_svd(blk, r, f.sigma, W, rows, Vh, cols, f);
    return HSF_OK;
}

hsf_status factor_block_rank(const Plan& p, const Block& blk, int64_t gate_id, double param, int rank, Factors& f) {
    const int ka = (int)blk.sa.size(), kb = (int)blk.sb.size();
    const int rows = 1 << (2 * kb), cols = 1 << (2 * ka);
    if (ka > p.max_side || kb > p.max_side || rank <= 0 || rank >= std::min(rows, cols))
        return factor_block(p, blk, gate_id, param, f);
    f = Factors();
    bool taken = false;
    hsf_status ps = try_product(p, blk, gate_id, param, f, taken);
    if (ps != HSF_OK || taken) return ps;
    std::vector<cd> At;
    reshaped_block(p, blk, gate_id, param, At);
    double nrm = 0;
    for (const cd& v : At) nrm += std::norm(v);
    nrm = std::sqrt(nrm);
    // range of At from `rank` fixed probe vectors (a fixed integer hash gives
    // entries in [-1, 1]; any probes in general position serve), columns of
    // Q orthonormalised twice by modified Gram-Schmidt
    const int r = rank;
    std::vector<cd> Q((size_t)r * rows, cd(0));            // column m at Q[m * rows]
    for (int m = 0; m < r; ++m)
        for (int c = 0; c < cols; ++c) {
            uint32_t h = (uint32_t)(m * 7919 + c) * 2654435761u;
            h ^= h >> 15;
            h *= 2246822519u;
            h ^= h >> 13;
            const cd w((double)(h & 0xffff) / 32768.0 - 1.0, (double)(h >> 16) / 32768.0 - 1.0);
            for (int i = 0; i < rows; ++i) Q[(size_t)m * rows + i] += At[(size_t)i * cols + c] * w;
        }
    for (int m = 0; m < r; ++m) {
        cd* qm = &Q[(size_t)m * rows];
        for (int pass = 0; pass < 2; ++pass)
            for (int k = 0; k < m; ++k) {
                const cd* qk = &Q[(size_t)k * rows];
                cd dot = 0;
                for (int i = 0; i < rows; ++i) dot += std::conj(qk[i]) * qm[i];
                for (int i = 0; i < rows; ++i) qm[i] -= dot * qk[i];
            }
        double n2 = 0;
        for (int i = 0; i < rows; ++i) n2 += std::norm(qm[i]);
        // a lower rank than the plan's: the full decomposition finds it
        if (std::sqrt(n2) <= 1e-10 * nrm) return factor_block(p, blk, gate_id, param, f);
        const double inv = 1.0 / std::sqrt(n2);
        for (int i = 0; i < rows; ++i) qm[i] *= inv;
    }
    // B = Q^H At (r x cols), then At = Q B checked element by element
    std::vector<cd> B((size_t)r * cols, cd(0));
    for (int m = 0; m < r; ++m)
        for (int i = 0; i < rows; ++i) {
            const cd qc = std::conj(Q[(size_t)m * rows + i]);
            for (int c = 0; c < cols; ++c) B[(size_t)m * cols + c] += qc * At[(size_t)i * cols + c];
        }
    double res = 0;
    for (int i = 0; i < rows; ++i)
        for (int c = 0; c < cols; ++c) {
            cd v = At[(size_t)i * cols + c];
            for (int m = 0; m < r; ++m) v -= Q[(size_t)m * rows + i] * B[(size_t)m * cols + c];
            res += std::norm(v);
        }
    if (std::sqrt(res) > 1e-11 * nrm) return factor_block(p, blk, gate_id, param, f);
    // B = Wb diag(s) Vbh (r x r, r x cols): At = (Q Wb) diag(s) Vbh
    std::vector<cd> Wb, Vbh;
    jacobi_svd(r, cols, B, Wb, f.sigma, Vbh);
    int rr = 0;
    hsf_status st = count_rank(p, f.sigma, rr);
    if (st != HSF_OK) return st;
    f.rank = rr;
    std::vector<cd> W((size_t)r * rows, cd(0));             // column m of Q Wb at W[m * rows]
    for (int m = 0; m < r; ++m)
        for (int k = 0; k < r; ++k) {
            const cd w = Wb[(size_t)m * r + k];
            for (int i = 0; i < rows; ++i) W[(size_t)m * rows + i] += Q[(size_t)k * rows + i] * w;
        }
    pieces_from_svd(blk, rr, f.sigma, W, rows, Vbh, cols, f);
    return HSF_OK;
}

void expand_factors(const Block& b, const Factors& f, std::vector<cd>& xa, std::vector<cd>& yb) {
    for (int s = 0; s < 2; ++s) {
        const std::vector<int>& sup = s == 0 ? b.sa : b.sb;
        const std::vector<FactorPiece>& pcs = s == 0 ? f.pa : f.pb;
        std::vector<cd>& out = s == 0 ? xa : yb;
        out.clear();
        const int k = (int)sup.size();
        if (k == 0 || k > kMaxExpandSide) continue;
        if (!f.product) {
            out = pcs[0].m;
            continue;
        }
        // product of 1-qubit pieces; piece i acts on sup[i], bit i of the index
        const int64_t d = int64_t(1) << k;
        out.assign((size_t)f.rank * d * d, cd(0));
        for (int m = 0; m < f.rank; ++m)
            for (int64_t r = 0; r < d; ++r)
                for (int64_t c = 0; c < d; ++c) {
                    cd v(1.0);
                    for (int i = 0; i < k && v != cd(0); ++i)
                        v *= pcs[i].m[(size_t)m * 4 + ((r >> i) & 1) * 2 + ((c >> i) & 1)];
                    out[((size_t)m * d + r) * d + c] = v;
                }
    }
}

hsf_status load_gate(const hsf_gate& in, int n, int64_t i, Gate& g) {
    g.kind = in.kind;
    g.nq = in.nq;
    g.param = in.param;
    g.param_id = in.param_id;
    if (in.nq < 1 || in.nq > 3) return fail(HSF_E_ARG, "gate " + std::to_string(i) + ": nq must be 1..3");
    for (int j = 0; j < in.nq; ++j) {
        if (in.q[j] < 0 || in.q[j] >= n) return fail(HSF_E_ARG, "gate " + std::to_string(i) + ": qubit out of range");
        for (int l = 0; l < j; ++l)
            if (in.q[l] == in.q[j]) return fail(HSF_E_ARG, "gate " + std::to_string(i) + ": repeated qubit");
        g.q[j] = in.q[j];
    }
    const int want = (in.kind >= HSF_GATE_H && in.kind <= HSF_GATE_PHASE) ? 1
                     : (in.kind >= HSF_GATE_CX && in.kind <= HSF_GATE_ISWAP) ? 2 : 0;
    if (in.kind != HSF_GATE_U && want != in.nq)
        return fail(HSF_E_ARG, "gate " + std::to_string(i) + ": kind does not match nq");
    if (in.kind == HSF_GATE_U && !in.matrix) return fail(HSF_E_ARG, "gate " + std::to_string(i) + ": U needs a matrix");
    if (!gate_matrix(in.kind, in.nq, in.param, in.matrix, g.m))
        return fail(HSF_E_ARG, "gate " + std::to_string(i) + ": unknown kind");
    g.diag = matrix_is_diag(g.m, 1 << in.nq);
    return HSF_OK;
}

hsf_status build_plan(const hsf_circuit* c, int32_t cut, const int64_t* ids, const int64_t* offs,
                      int32_t n_blocks, const hsf_plan_options* opts, Plan** out) {
    if (!c || !out) return fail(HSF_E_ARG, "null circuit or output pointer");
    if (c->n_qubits < 2 || c->n_qubits > 62) return fail(HSF_E_ARG, "n_qubits must be in 2..62");
    if (c->n_gates < 0 || (c->n_gates > 0 && !c->gates)) return fail(HSF_E_ARG, "bad gate array");
    if (n_blocks < 0 || (n_blocks > 0 && (!ids || !offs))) return fail(HSF_E_ARG, "bad block arrays");
    const int n = c->n_qubits;
    if (cut < 0 || cut > n - 2) return fail(HSF_E_CUT, "cut must lie in 0..n-2");

    Plan* p = new Plan();
    std::unique_ptr<Plan> guard(p);
    p->n = n;
    p->cut = cut;
    p->nb = cut + 1;
    p->na = n - cut - 1;
    if (opts) {
        if (opts->rank_tol > 0) p->rank_tol = opts->rank_tol;
        if (opts->max_side_qubits > 0) p->max_side = std::min(opts->max_side_qubits, kMaxSideQubits);
        if (opts->dtype != HSF_C64 && opts->dtype != HSF_C128) return fail(HSF_E_ARG, "dtype must be HSF_C64 or HSF_C128");
        p->dtype = opts->dtype;
        p->tile_req = opts->tile_qubits;
        p->fuse = opts->fuse;
        if (opts->tree < 0 || opts->tree > 2) return fail(HSF_E_ARG, "tree must be 0, 1 or 2");
        p->tree_mode = opts->tree;
            if (opts->defer_b_suffix != 0 && opts->defer_b_suffix != 1) return fail(HSF_E_ARG, "defer_b_suffix must be 0 or 1");
        p->defer_b = opts->defer_b_suffix;
    }
    if (p->tile_req < 0 || p->tile_req > max_tile_bits(p->dtype))
        return fail(HSF_E_ARG, "tile_qubits out of range");

    // ---- ingest gates
    const int64_t G = c->n_gates;
    p->gates.resize(G);
    for (int64_t i = 0; i < G; ++i) {
        Gate& g = p->gates[i];
        hsf_status gs = load_gate(c->gates[i], n, i, g);
        if (gs != HSF_OK) return gs;
        if (g.param_id >= 0) p->n_params = std::max<int64_t>(p->n_params, g.param_id + 1);
    }

    // ---- sides: 0 = a (all qubits > cut), 1 = b (all <= cut), 2 = crossing
    std::vector<int> side(G);
    for (int64_t i = 0; i < G; ++i) {
        int lo = 0;
        for (int j = 0; j < p->gates[i].nq; ++j) lo += p->gates[i].q[j] <= cut;
        side[i] = lo == 0 ? 0 : (lo == p->gates[i].nq ? 1 : 2);
    }

    // ---- block hulls
    std::vector<int> owner(G, -1);
    std::vector<std::vector<int64_t>> hulls(n_blocks);
    for (int b = 0; b < n_blocks; ++b) {
        const int64_t b0 = offs[b], b1 = offs[b + 1];
        if (b1 <= b0) return fail(HSF_E_ARG, "block " + std::to_string(b) + " is empty");
        std::vector<char> seed(G, 0);
        for (int64_t t = b0; t < b1; ++t) {
            if (ids[t] < 0 || ids[t] >= G) return fail(HSF_E_ARG, "block " + std::to_string(b) + ": gate id out of range");
            seed[ids[t]] = 1;
        }
        std::vector<char> dn = closure(p->gates, n, seed, true);
        std::vector<char> up = closure(p->gates, n, seed, false);
        for (int64_t i = 0; i < G; ++i)
            if (dn[i] && up[i]) {
                if (owner[i] >= 0) return fail(HSF_E_BLOCK_OVERLAP, "blocks " + std::to_string(owner[i]) + " and " + std::to_string(b) + " share gate " + std::to_string(i));
                owner[i] = b;
                hulls[b].push_back(i);
            }
    }
    for (int64_t i = 0; i < G; ++i)
        if (side[i] == 2 && owner[i] < 0) return fail(HSF_E_BLOCK_UNCOVERED, "crossing gate " + std::to_string(i) + " is in no block");

    // ---- contracted DAG, Kahn's algorithm (smallest original gate id first)
    const int64_t NN = G + n_blocks;
    auto node_of = [&](int64_t i) -> int64_t { return owner[i] >= 0 ? G + owner[i] : i; };
    std::vector<int64_t> key(NN, -1);
    for (int64_t i = 0; i < G; ++i) {
        const int64_t nd = node_of(i);
        if (key[nd] < 0) key[nd] = i;
    }
    std::vector<std::vector<int64_t>> succ(NN);
    std::vector<int64_t> indeg(NN, 0);
    {
        std::set<std::pair<int64_t, int64_t>> seen;
        std::vector<int64_t> last(n, -1);
        for (int64_t i = 0; i < G; ++i) {
            const int64_t nd = node_of(i);
            for (int j = 0; j < p->gates[i].nq; ++j) {
                const int q = p->gates[i].q[j];
                if (last[q] >= 0 && last[q] != nd && seen.insert({last[q], nd}).second) {
                    succ[last[q]].push_back(nd);
                    indeg[nd]++;
                }
                last[q] = nd;
            }
        }
    }
    std::priority_queue<std::pair<int64_t, int64_t>, std::vector<std::pair<int64_t, int64_t>>, std::greater<>> ready;
    int64_t live = 0;
    for (int64_t nd = 0; nd < NN; ++nd)
        if (key[nd] >= 0) {
            ++live;
            if (indeg[nd] == 0) ready.push({key[nd], nd});
        }
    std::vector<int64_t> order;
    while (!ready.empty()) {
        const int64_t nd = ready.top().second;
        ready.pop();
        order.push_back(nd);
        for (int64_t s : succ[nd])
            if (--indeg[s] == 0) ready.push({key[s], s});
    }
    if ((int64_t)order.size() != live) return fail(HSF_E_BLOCK_CYCLE, "blocks form a cycle in the contracted circuit");

    // ---- blocks in plan order: operator, Schmidt decomposition, rank
    std::vector<int> plan_index(n_blocks, -1);
    for (int64_t nd : order) {
        if (nd < G) continue;
        const int b = (int)(nd - G);
        plan_index[b] = (int)p->blocks.size();
        Block blk;
        blk.caller_index = b;
        blk.hull = hulls[b];
        std::set<int> qs;
        for (int64_t gi : blk.hull)
            for (int j = 0; j < p->gates[gi].nq; ++j) qs.insert(p->gates[gi].q[j]);
        for (int q : qs) (q > cut ? blk.sa : blk.sb).push_back(q);
        for (int64_t gi : blk.hull)
            if (p->gates[gi].param_id >= 0) blk.params.push_back({gi, p->gates[gi].param_id});
        Factors fb;
        hsf_status fs = factor_block(*p, blk, -1, 0.0, fb);
        if (fs != HSF_OK) return fail(fs, "block " + std::to_string(b) + ": " + hsf::g_last_error_copy());
        blk.sigma = fb.sigma;
        blk.rank = fb.rank;
        blk.product = fb.product;
        expand_factors(blk, fb, blk.xa, blk.yb);
        blk.pa = std::move(fb.pa);
        blk.pb = std::move(fb.pb);
        p->blocks.push_back(std::move(blk));
    }

    // ---- path table
    p->P = 1;
    for (const Block& b : p->blocks) {
        if (p->P > (int64_t(1) << 62) / b.rank) return fail(HSF_E_PATHS_OVERFLOW, "more than 2^62 paths");
        p->P *= b.rank;
    }
    {
        int64_t R = 1;
        for (int k = (int)p->blocks.size() - 1; k >= 0; --k) {
            p->blocks[k].stride = R;
            R *= p->blocks[k].rank;
        }
    }

    // ---- side programs (topological order projected to each side)
    for (int s = 0; s < 2; ++s) {
        p->side[s].nq = s == 0 ? p->na : p->nb;
        p->side[s].ops.clear();
    }
    for (int64_t nd : order) {
        if (nd < G) {
            const Gate& g = p->gates[nd];
            const int s = side[nd];
            const int off = s == 0 ? p->nb : 0;
            SideOp op;
            op.kind = g.diag ? SideOp::DIAG : SideOp::DENSE;
            op.k = g.nq;
            for (int j = 0; j < g.nq; ++j) op.q[j] = g.q[j] - off;
            const int dd = 1 << g.nq;
            if (g.diag) {
                op.m.resize(dd);
                for (int i = 0; i < dd; ++i) op.m[i] = g.m[(size_t)i * dd + i];
            } else {
                op.m = g.m;
            }
            if (g.param_id >= 0 && gate_generator(g.kind, g.nq, op.dgen)) op.param_id = g.param_id;
            p->side[s].ops.push_back(std::move(op));
        } else {
            const int k = plan_index[nd - G];
            const Block& b = p->blocks[k];
            for (int s = 0; s < 2; ++s) {
                const std::vector<FactorPiece>& pcs = s == 0 ? b.pa : b.pb;
                const int off = s == 0 ? p->nb : 0;
                for (size_t pi = 0; pi < pcs.size(); ++pi) {
                    const FactorPiece& pc = pcs[pi];
                    SideOp op;
                    op.kind = SideOp::SLOT;
                    op.k = (int)pc.q.size();
                    // factor index: ascending qubit = ascending significance => q[0] is the top qubit
                    for (int j = 0; j < op.k; ++j) op.q[j] = pc.q[op.k - 1 - j] - off;
                    op.m = pc.m;
                    op.block = k;
                    op.piece = (int)pi;
                    op.product = b.product;
                    op.rank = b.rank;
                    op.stride = b.stride;
                    p->side[s].ops.push_back(std::move(op));
                }
            }
        }
    }
    // side b's ops after its last factor slot, deferred to the output rows:
    // the same gates act on every path's side-b state, and the path sum is
    // linear in that state
    std::vector<SideOp> b_post;
    if (p->defer_b) {
        std::vector<SideOp>& v = p->side[1].ops;
        int last = -1;
        for (int i = 0; i < (int)v.size(); ++i)
            if (v[i].kind == SideOp::SLOT) last = i;
        if (last >= 0 && last + 1 < (int)v.size()) {
            b_post.assign(v.begin() + last + 1, v.end());
            v.resize((size_t)last + 1);
        }
    }
    for (int s = 0; s < 2; ++s) {
        p->side[s].ops_logical = (int64_t)p->side[s].ops.size();
        p->side[s].raw = p->side[s].ops;
        fuse_side(*p, s);
        order_prefix(p->side[s]);
        const int nq = std::max(p->side[s].nq, 1);
        const int tmax = p->tile_req > 0 ? p->tile_req : max_tile_bits(p->dtype);
        // candidate tile sizes, largest first (a requested size is the only one)
        const int top = std::min(tmax, nq);
        const int bottom = p->tile_req > 0 ? top : std::max(std::min(nq, 8), top - 5);
        const std::vector<int> flat_cuts = {0, p->side[s].n_prefix, (int)p->side[s].ops.size()};
        for (int L = top; L >= bottom; --L)
            p->side[s].sched.push_back(schedule_side(*p, s, L, p->side[s].ops, flat_cuts, {}, false));
        // replay segments of the raw program for gradients, on one tile size
        // that suits many rows (12 qubits, or the whole side)
        if (p->n_params > 0) {
            const std::vector<SideOp>& raw = p->side[s].raw;
            const int n = (int)raw.size();
            for (int lo = 0; lo < n;) {
                if (raw[lo].kind == SideOp::SLOT) {
                    ++lo;
                    continue;
                }
                int hi = lo;
                while (hi < n && raw[hi].kind != SideOp::SLOT) ++hi;
                p->side[s].seg.push_back(schedule_side(*p, s, std::min(12, tmax), raw, {lo, lo, hi}, {}, false));
                p->side[s].seg_lo.push_back(lo);
                p->side[s].seg_hi.push_back(hi);
                lo = hi;
            }
        }
        if (s == 1 && !b_post.empty()) {
            p->side[1].post_ops = (int64_t)b_post.size();
            fuse_list(*p, b_post, nq);
            const int n_post = (int)b_post.size();
            Schedule sc = schedule_side(*p, 1, std::min(std::min(12, tmax), nq), b_post, {0, 0, n_post}, {}, false);
            // the rows hold the summed state: no pass starts from |0...0>
            for (Pass& q : sc.passes) q.init_zero = 0;
            p->side[1].post.push_back(std::move(sc));
        }
        if (!p->blocks.empty()) {
            std::vector<int> cuts, levels;
            const std::vector<SideOp> lops = level_order(*p, s, cuts, levels);
            // every block has a slot on both sides, so the last level holds
            // all digits; a side without per-path ops keeps the flat form only
            if (levels.size() >= 2 && levels.back() == (int)p->blocks.size())
                for (int L = top; L >= bottom; --L)
                    p->side[s].tree.push_back(schedule_side(*p, s, L, lops, cuts, levels, true));
        }
    }
    *out = guard.release();
    return HSF_OK;
}

// ---------------------------------------------------------------- fusion --

namespace {

std::vector<cd> mat_mul(const std::vector<cd>& a, const std::vector<cd>& b, int d) {
    std::vector<cd> c((size_t)d * d, cd(0));
    for (int i = 0; i < d; ++i)
        for (int k = 0; k < d; ++k)
            for (int j = 0; j < d; ++j) c[(size_t)i * d + j] += a[(size_t)i * d + k] * b[(size_t)k * d + j];
    return c;
}

std::vector<cd> as_dense1(const SideOp& o) {
    if (o.kind == SideOp::DENSE) return o.m;
    return {o.m[0], 0, 0, o.m[1]};
}

// Merge runs of one-qubit ops on the same qubit (exact in real arithmetic),
// fold one-qubit ops that directly follow a one-qubit factor piece on its
// qubit into the piece (its `post`: the path's digit still picks the piece,
// the folded gates are the same for every digit), then fold diagonal ops
// into the diagonal op placed before them when their union stays within
// kMaxOpQubits qubits and nothing in between touches them.
void fuse_ops(std::vector<SideOp>& ops, int nq) {
    std::vector<SideOp> out;
    std::vector<int> pend(nq, -1);  // index in `out` of a one-qubit op still open on q
    std::vector<int> spend(nq, -1); // index in `out` of a one-qubit factor piece still open on q
    for (SideOp& o : ops) {
        if (o.kind != SideOp::SLOT && o.k == 1 && spend[o.q[0]] >= 0) {
            SideOp& t = out[spend[o.q[0]]];
            const std::vector<cd> prev = t.post.empty() ? std::vector<cd>{1, 0, 0, 1} : t.post;
            t.post = mat_mul(as_dense1(o), prev, 2);
            t.logical += o.logical;
            continue;
        }
        if (o.kind != SideOp::SLOT && o.k == 1 && pend[o.q[0]] >= 0) {
            SideOp& t = out[pend[o.q[0]]];
            if (t.kind == SideOp::DIAG && o.kind == SideOp::DIAG) {
                t.m[0] *= o.m[0];
                t.m[1] *= o.m[1];
            } else {
                t.m = mat_mul(as_dense1(o), as_dense1(t), 2);
                t.kind = SideOp::DENSE;
            }
            t.logical += o.logical;
            continue;
        }
        for (int j = 0; j < o.k; ++j) pend[o.q[j]] = spend[o.q[j]] = -1;
        out.push_back(std::move(o));
        if (out.back().kind != SideOp::SLOT && out.back().k == 1) pend[out.back().q[0]] = (int)out.size() - 1;
        if (out.back().kind == SideOp::SLOT && out.back().k == 1) spend[out.back().q[0]] = (int)out.size() - 1;
    }
    // diagonal folding
    std::vector<SideOp> res;
    std::vector<int> last_touch(nq, -1);   // index in res of the last op touching q
    for (SideOp& o : out) {
        if (o.kind == SideOp::DIAG) {
            // candidate: the latest diag op in res that no later op blocks
            int cand = -1;
            for (int j = 0; j < o.k; ++j) cand = std::max(cand, last_touch[o.q[j]]);
            // the op at cand must be diagonal; walk back over diag ops not touching o
            int tgt = -1;
            if (cand >= 0 && res[cand].kind == SideOp::DIAG) tgt = cand;
            if (cand < 0 && !res.empty()) {
                // nothing touches o's qubits yet: fold into the last diag op if any
                for (int i = (int)res.size() - 1; i >= 0; --i)
                    if (res[i].kind == SideOp::DIAG) { tgt = i; break; }
            }
            if (tgt >= 0) {
                SideOp& t = res[tgt];
                // every op after tgt must not touch o's qubits (then o can move up to tgt)
                bool ok = true;
                for (int j = 0; j < o.k && ok; ++j)
                    if (last_touch[o.q[j]] > tgt) ok = false;
                // union of qubits
                int uq[8], nu = 0;
                for (int j = 0; j < t.k; ++j) uq[nu++] = t.q[j];
                for (int j = 0; j < o.k; ++j) {
                    bool have = false;
                    for (int l = 0; l < nu; ++l) have |= uq[l] == o.q[j];
                    if (!have) uq[nu++] = o.q[j];
                }
                if (ok && nu <= kMaxOpQubits) {
                    std::vector<cd> m(1u << nu);
                    for (int e = 0; e < (1 << nu); ++e) {
                        int et = 0, eo = 0;
                        for (int j = 0; j < t.k; ++j) {
                            int pos = 0;
                            while (uq[pos] != t.q[j]) ++pos;
                            et |= ((e >> (nu - 1 - pos)) & 1) << (t.k - 1 - j);
                        }
                        for (int j = 0; j < o.k; ++j) {
                            int pos = 0;
                            while (uq[pos] != o.q[j]) ++pos;
                            eo |= ((e >> (nu - 1 - pos)) & 1) << (o.k - 1 - j);
                        }
                        m[e] = t.m[et] * o.m[eo];
                    }
                    t.k = nu;
                    for (int j = 0; j < nu; ++j) t.q[j] = uq[j];
                    t.m = std::move(m);
                    t.logical += o.logical;
                    for (int j = 0; j < nu; ++j) last_touch[uq[j]] = std::max(last_touch[uq[j]], tgt);
                    continue;
                }
            }
        }
        res.push_back(std::move(o));
        for (int j = 0; j < res.back().k; ++j) last_touch[res.back().q[j]] = (int)res.size() - 1;
    }
    ops.swap(res);
}

}  // namespace

// ------------------------------------------------------- pass scheduling --

void fuse_list(const Plan& p, std::vector<SideOp>& ops, int nq) {
    if (p.fuse) fuse_ops(ops, std::max(nq, 1));
}

void fuse_side(Plan& p, int s) {
    if (p.fuse) fuse_ops(p.side[s].ops, std::max(p.side[s].nq, 1));
}

// An op that is diagonal.  A factor slot counts only in the product form,
// which is diagonal for every angle of its block: the backward pass
// re-factors blocks at shifted angles and reuses this plan's op order.
std::vector<cd> slot_matrix(const SideOp& o, int r) {
    const size_t d2 = (size_t)1 << (2 * o.k);
    std::vector<cd> m(o.m.begin() + (size_t)r * d2, o.m.begin() + (size_t)(r + 1) * d2);
    if (o.post.empty()) return m;
    return mat_mul(o.post, m, 2);
}

bool op_is_diagonal(const SideOp& o) {
    if (o.kind == SideOp::DIAG) return true;
    if (o.kind == SideOp::SLOT) return o.product && (o.post.empty() || (o.post[1] == cd(0) && o.post[2] == cd(0)));
    const int d = 1 << o.k;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
            if (i != j && o.m[(size_t)i * d + j] != cd(0.0)) return false;
    return true;
}

// Ops that act the same way on all paths can run once, on one shared state,
// before every path's factor slots: an op joins that prefix when it is not a
// factor slot and commutes with every op left behind it -- they act on
// disjoint qubits, or both are diagonal.  Prefix and rest each keep their
// order.  In a brickwork this is every gate outside the forward light cone of
// the first block; for the cascades of Sec. V the cost layer outside the
// blocks.
namespace {

// Within each run of diagonal ops in v[lo, hi), the one-qubit factor pieces
// go last, ordered by qubit, so that the pieces on one qubit meet in a
// register group and are multiplied before being applied.
void order_pieces(std::vector<SideOp>& v, size_t lo, size_t hi) {
    for (size_t i = lo; i < hi;) {
        size_t j = i;
        while (j < hi && op_is_diagonal(v[j])) ++j;
        if (j > i + 1) {
            auto piece = [](const SideOp& o) { return o.kind == SideOp::SLOT && o.k == 1; };
            auto mid = std::stable_partition(v.begin() + (std::ptrdiff_t)i, v.begin() + (std::ptrdiff_t)j,
                                             [&](const SideOp& o) { return !piece(o); });
            std::stable_sort(mid, v.begin() + (std::ptrdiff_t)j,
                             [](const SideOp& x, const SideOp& y) { return x.q[0] < y.q[0]; });
        }
        i = j > i ? j : i + 1;
    }
}

}  // namespace

void order_prefix(SideProgram& sp) {
    const int nq = std::max(sp.nq, 1);
    std::vector<char> dense_left(nq, 0), diag_left(nq, 0);   // qubits of the ops left behind
    std::vector<SideOp> pre, rest;
    for (SideOp& o : sp.ops) {
        const bool od = op_is_diagonal(o);
        bool hoist = o.kind != SideOp::SLOT;
        for (int j = 0; j < o.k && hoist; ++j)
            if (dense_left[o.q[j]] || (!od && diag_left[o.q[j]])) hoist = false;
        if (hoist) {
            pre.push_back(std::move(o));
        } else {
            for (int j = 0; j < o.k; ++j) (od ? diag_left : dense_left)[o.q[j]] = 1;
            rest.push_back(std::move(o));
        }
    }
    order_pieces(rest, 0, rest.size());
    sp.n_prefix = (int)pre.size();
    sp.ops = std::move(pre);
    sp.ops.insert(sp.ops.end(), std::make_move_iterator(rest.begin()), std::make_move_iterator(rest.end()));
}


// Path-tree order.  A path's half-state after an op depends on the path
// only through the digits of the factor slots applied so far (Sec. II-B:
// every other op acts the same way on all paths), so the paths that agree
// on m_0 .. m_{d-1} share one state up to the first op that needs a later
// digit.  The level of an op is the number of leading digits its result
// depends on: a slot of block k needs k + 1, and an op must follow every
// earlier op it does not commute with (disjoint qubits, or both diagonal,
// commute), so it takes the largest level among those.  Sorting the ops
// stably by level keeps every such pair in order; level 0 is the shared
// prefix.
std::vector<SideOp> level_order(const Plan& p, int side, std::vector<int>& cuts, std::vector<int>& levels) {
    const SideProgram& sp = p.side[side];
    const int nq = std::max(sp.nq, 1);
    const int n = (int)sp.ops.size();
    std::vector<int> dense_lev(nq, 0), diag_lev(nq, 0), lev(n, 0);
    for (int i = 0; i < n; ++i) {
        const SideOp& o = sp.ops[i];
        const bool od = op_is_diagonal(o);
        int l = o.kind == SideOp::SLOT ? o.block + 1 : 0;
        for (int j = 0; j < o.k; ++j) {
            l = std::max(l, dense_lev[o.q[j]]);
            if (!od) l = std::max(l, diag_lev[o.q[j]]);
        }
        lev[i] = l;
        for (int j = 0; j < o.k; ++j) {
            int& t = (od ? diag_lev : dense_lev)[o.q[j]];
            t = std::max(t, l);
        }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return lev[a] < lev[b]; });
    std::vector<SideOp> out;
    out.reserve(n);
    cuts.assign(1, 0);
    levels.assign(1, 0);
    // range 0 is level 0 (possibly empty); then one range per level present
    for (int i = 0; i < n; ++i) {
        const int l = lev[idx[i]];
        if (l != levels.back()) {
            cuts.push_back(i);
            levels.push_back(l);
        }
        out.push_back(sp.ops[idx[i]]);
    }
    cuts.push_back(n);
    // A thin level costs a pass of its own (every state read and written)
    // for few ops: it joins the next level when repeating its ops on the
    // next level's states costs less than that pass -- about 1.5 units per op
    // and state against 8 for a state's load, store and launch share (the
    // sweep estimate's units).  Level 0, the shared prefix, stays.
    auto states = [&](int lv) {
        double st = 1;
        for (int k = 0; k < lv && k < (int)p.blocks.size(); ++k) st *= (double)p.blocks[k].rank;
        return st;
    };
    for (size_t r = 1; r + 2 < cuts.size();) {
        const double ops = (double)(cuts[r + 1] - cuts[r]);
        const double ratio = states(levels[r + 1]) / states(levels[r]);
        if (ops * 1.5 * (ratio - 1.0) < 8.0) {
            cuts.erase(cuts.begin() + (std::ptrdiff_t)(r + 1));   // range r absorbs range r + 1
            levels.erase(levels.begin() + (std::ptrdiff_t)r);    // and takes its (higher) level
        } else {
            ++r;
        }
    }
    for (size_t r = 1; r + 1 < cuts.size(); ++r) order_pieces(out, (size_t)cuts[r], (size_t)cuts[r + 1]);
    return out;
}

namespace {


// Turns the ops of one pass into device ops: runs of one-qubit gates (on at
// most four tile bits) and diagonal gates (on any qubits) become one
// register-resident group; wider dense ops and factor slots stand alone.
// group_slots: one-qubit factor pieces join register groups (as SUB_SLOT1);
// otherwise they stay separate ops.
void emit_pass(const std::vector<SideOp>& sops, Schedule& sc, const Pass& ps, const std::vector<int>& ids,
               bool group_slots) {
    const int L = ps.n_local;
    const int KG = group_bits(L);
    auto tbit = [&](int q) -> int {
        for (int l = 0; l < L; ++l)
            if (ps.local_q[l] == q) return l;
        return -1 - q;
    };
    auto pos_in = [](const std::vector<int>& v, int x) -> int {
        for (size_t i = 0; i < v.size(); ++i)
            if (v[i] == x) return (int)i;
        return -1;
    };
    std::vector<int> grp, gbits;
    auto close = [&]() {
        if (grp.empty()) return;
        std::vector<int> bits = gbits;
        for (int id : grp) {
            const SideOp& o = sops[id];
            if (o.kind != SideOp::DIAG) continue;
            for (int j = 0; j < o.k && (int)bits.size() < KG; ++j) {
                const int b = tbit(o.q[j]);
                if (b >= 0 && pos_in(bits, b) < 0) bits.push_back(b);
            }
        }
        for (int b = 0; b < L && (int)bits.size() < KG; ++b)
            if (pos_in(bits, b) < 0) bits.push_back(b);
        DevOp d{};
        d.type = DOP_GROUP;
        d.block = -1;
        d.k = KG;
        for (int g = 0; g < KG; ++g) d.bit[g] = bits[g];
        d.mat = (int32_t)sc.subs.size();
        d.rank = (int32_t)grp.size();
        for (int id : grp) {
            const SideOp& o = sops[id];
            SubOp so{};
            if (o.kind == SideOp::SLOT) {
                so.type = SUB_SLOT1;
                so.g = pos_in(bits, tbit(o.q[0]));
                so.qb[0] = op_is_diagonal(o) ? 1 : 0;   // bit 0: diagonal; bits 1, 2: chains (below)
                // a diagonal piece off the register bits (g < 0) scales every
                // amplitude by the entry its qubit's bit selects (tile bit
                // qb[1] >= 0, or non-local qubit -1 - qb[1])
                so.qb[1] = tbit(o.q[0]);
                so.mat = (int32_t)sc.pool.size();
                for (int r = 0; r < o.rank; ++r) {
                    const std::vector<cd> f = slot_matrix(o, r);
                    sc.pool.insert(sc.pool.end(), f.begin(), f.end());
                }
                so.post = o.post;
                so.rank = o.rank;
                so.stride = o.stride;
                so.block = o.block;
                so.piece = o.piece;
            } else if (o.kind == SideOp::DENSE) {
                so.type = SUB_D1;
                so.g = pos_in(bits, tbit(o.q[0]));
                for (int i = 0; i < 4; ++i) {
                    so.m[2 * i] = o.m[i].real();
                    so.m[2 * i + 1] = o.m[i].imag();
                }
            } else {
                int regpos[4], cpos[4], nc = 0;
                for (int j = 0; j < o.k; ++j) {
                    const int b = tbit(o.q[j]);
                    const int pp = b >= 0 ? pos_in(bits, b) : -1;
                    regpos[j] = pp;
                    cpos[j] = -1;
                    if (pp < 0) {
                        so.qb[nc] = b;
                        cpos[j] = nc++;
                    }
                }
                so.nc = nc;
                const int D = 1 << KG;
                std::vector<cd> T((size_t)(1 << nc) * D);
                bool sign = true;
                for (int c = 0; c < (1 << nc); ++c)
                    for (int jj = 0; jj < D; ++jj) {
                        int idx = 0;
                        for (int j = 0; j < o.k; ++j) {
                            const int bit = regpos[j] >= 0 ? (jj >> regpos[j]) & 1 : (c >> cpos[j]) & 1;
                            idx |= bit << (o.k - 1 - j);
                        }
                        const cd v = o.m[idx];
                        T[(size_t)c * D + jj] = v;
                        if (!(v == cd(1.0) || v == cd(-1.0))) sign = false;
                    }
                if (sign) {
                    so.type = SUB_SIGN;
                    for (int c = 0; c < (1 << nc); ++c) {
                        uint32_t m16 = 0;
                        for (int jj = 0; jj < D; ++jj)
                            if (T[(size_t)c * D + jj] == cd(-1.0)) m16 |= 1u << jj;
                        so.mask[c >> 1] |= m16 << (16 * (c & 1));
                    }
                } else {
                    so.type = SUB_PHASE;
                    so.mat = (int32_t)sc.pool.size();
                    sc.pool.insert(sc.pool.end(), T.begin(), T.end());
                }
            }
            sc.subs.push_back(so);
        }
        // a diagonal piece followed by another on the same register bit only
        // multiplies into the chain; the last of the chain (diagonal, or a
        // piece with folded gates) applies it
        for (int j = d.mat; j + 1 < d.mat + d.rank; ++j) {
            SubOp& x = sc.subs[j];
            const SubOp& y = sc.subs[j + 1];
            SubOp& y2 = sc.subs[j + 1];
            if (x.type == SUB_SLOT1 && y.type == SUB_SLOT1 && (x.qb[0] & 1) && x.g >= 0 && x.g == y.g) {
                x.qb[0] |= 2;    // bit 1: chained into the next
                y2.qb[0] |= 4;   // bit 2: ends (or continues) a chain
            }
        }
        sc.devops.push_back(d);
        grp.clear();
        gbits.clear();
    };
    for (int id : ids) {
        const SideOp& o = sops[id];
        // one-qubit gates and one-qubit factor pieces join register groups;
        // a diagonal piece on a bit the group does not hold joins as is
        // (like a diagonal gate, it needs no register bit)
        if (o.kind == SideOp::SLOT && group_slots && o.k == 1 && op_is_diagonal(o) &&
            pos_in(gbits, tbit(o.q[0])) < 0 && (int)gbits.size() >= KG) {
            grp.push_back(id);
            if (grp.size() >= 24) close();
        } else if ((o.kind == SideOp::DENSE || (o.kind == SideOp::SLOT && group_slots)) && o.k == 1) {
            const int b = tbit(o.q[0]);
            if (pos_in(gbits, b) < 0 && (int)gbits.size() >= KG) close();
            if (pos_in(gbits, b) < 0) gbits.push_back(b);
            grp.push_back(id);
            if (grp.size() >= 24) close();
        } else if (o.kind == SideOp::DIAG) {
            grp.push_back(id);
            if (grp.size() >= 24) close();
        } else {
            close();
            DevOp d{};
            d.type = o.kind == SideOp::SLOT ? DOP_SLOT : DOP_DENSEK;
            d.k = o.k;
            for (int j = 0; j < o.k; ++j) d.bit[j] = tbit(o.q[j]);
            d.mat = (int32_t)sc.pool.size();
            d.rank = o.rank;
            d.stride = o.stride;
            d.block = o.block;
            d.piece = o.piece;
            if (o.kind == SideOp::SLOT) {
                for (int r = 0; r < o.rank; ++r) {
                    const std::vector<cd> f = slot_matrix(o, r);
                    sc.pool.insert(sc.pool.end(), f.begin(), f.end());
                }
            } else {
                sc.pool.insert(sc.pool.end(), o.m.begin(), o.m.end());
            }
            sc.devops.push_back(d);
        }
    }
    close();
}

}  // namespace

Schedule schedule_side(const Plan& p, int s, int L, const std::vector<SideOp>& ops, const std::vector<int>& cuts,
                       const std::vector<int>& levels, bool tree) {
    const SideProgram& sp = p.side[s];
    Schedule sc;
    const int nq = sp.nq;
    // a multi-pass tile needs room for the widest op beside the coalesced low qubits
    L = std::max(std::min(nq, 8), std::min(L, nq));
    L = std::max(L, 1);
    sc.tile_bits = L;
    const int nops = (int)ops.size();
    // fold one-qubit factor pieces into register groups only when blocks
    // bring several of them to this side (cascades, Sec. V): then the group
    // saves LDS passes; a lone piece per block is cheaper as its own op
    std::set<int> piece_blocks;
    int pieces = 0;
    for (const SideOp& o : ops)
        if (o.kind == SideOp::SLOT && o.k == 1) {
            ++pieces;
            piece_blocks.insert(o.block);
        }
    const bool group_slots = pieces > (int)piece_blocks.size();
    const int low = L >= nq ? L : std::max(0, std::min(5, L - kMaxOpQubits));
    // ops [lo, hi) into passes; the first starts from |0...0> when lo == 0
    // and otherwise reads the state the previous passes left
    auto schedule_range = [&](int lo, int hi, bool prefix) {
        std::vector<char> done(nops, 1);
        for (int i = lo; i < hi; ++i) done[i] = 0;
        int remaining = hi - lo;
        bool first = true;
        while (first || remaining > 0) {
            Pass ps;
            ps.init_zero = (first && lo == 0) ? 1 : 0;
            ps.prefix = prefix ? 1 : 0;
            std::vector<char> local(std::max(nq, 1), 0);
            int nloc = 0;
            if (L >= nq) {
                for (int q = 0; q < nq; ++q) local[q] = 1;
                nloc = nq;
            } else {
                for (int q = 0; q < low; ++q) local[q] = 1, ++nloc;
                // the qubits of the earliest pending non-diagonal ops
                for (int i = 0; i < nops && nloc < L; ++i) {
                    if (done[i]) continue;
                    const SideOp& o = ops[i];
                    if (o.kind != SideOp::DIAG) {
                        int need = 0;
                        for (int j = 0; j < o.k; ++j) need += !local[o.q[j]];
                        if (nloc + need <= L)
                            for (int j = 0; j < o.k; ++j)
                                if (!local[o.q[j]]) local[o.q[j]] = 1, ++nloc;
                    }
                }
                for (int q = nq - 1; q >= 0 && nloc < L; --q)
                    if (!local[q]) local[q] = 1, ++nloc;
            }
            int t = 0, u = 0;
            for (int q = 0; q < nq; ++q) {
                if (local[q]) ps.local_q[t++] = q;
                else ps.nonlocal_q[u++] = q;
            }
            ps.n_local = std::max(t, 1);
            ps.n_nonlocal = u;
            std::vector<int> ids;
            std::vector<char> blocked(std::max(nq, 1), 0);
            for (int i = 0; i < nops; ++i) {
                if (done[i]) continue;
                const SideOp& o = ops[i];
                bool blk = false, fits = true;
                for (int j = 0; j < o.k; ++j) {
                    blk |= (bool)blocked[o.q[j]];
                    fits &= (bool)local[o.q[j]];
                }
                if (!blk && (fits || o.kind == SideOp::DIAG)) {
                    done[i] = 1;
                    --remaining;
                    ids.push_back(i);
                } else {
                    for (int j = 0; j < o.k; ++j) blocked[o.q[j]] = 1;
                }
            }
            ps.op_begin = (int32_t)sc.devops.size();
            emit_pass(ops, sc, ps, ids, group_slots);
            ps.op_end = (int32_t)sc.devops.size();
            // a pass that is one register group runs without the LDS tile; the
            // group's filler bits (positions no sub-op reads) move to the
            // highest free tile bits, so the lanes of a wave, which vary the
            // low bits, read and write runs of contiguous amplitudes
            if (ps.op_end == ps.op_begin + 1 && sc.devops[(size_t)ps.op_begin].type == DOP_GROUP) {
                DevOp& d = sc.devops[(size_t)ps.op_begin];
                std::vector<char> used_pos((size_t)d.k, 0), taken((size_t)ps.n_local, 0);
                for (int j = d.mat; j < d.mat + d.rank; ++j) {
                    const SubOp& so = sc.subs[(size_t)j];
                    if (so.type == SUB_SLOT1 && so.g < 0) {
                        // a diagonal piece off the register bits: its tile bit
                        // must stay outside the group
                        if (so.qb[1] >= 0) taken[(size_t)so.qb[1]] = 1;
                    } else if (so.type == SUB_D1 || so.type == SUB_SLOT1) {
                        used_pos[(size_t)so.g] = 1;
                    } else {
                        // a diagonal op's table depends on every register position; its
                        // controls outside the group must stay outside it
                        for (int g = 0; g < d.k; ++g) used_pos[(size_t)g] = 1;
                        for (int i = 0; i < so.nc; ++i)
                            if (so.qb[i] >= 0) taken[(size_t)so.qb[i]] = 1;
                    }
                }
                for (int g = 0; g < d.k; ++g)
                    if (used_pos[(size_t)g]) taken[(size_t)d.bit[g]] = 1;
                int nb[kMaxTileBits];
                for (int g = 0; g < d.k; ++g) nb[g] = d.bit[g];
                int hi = ps.n_local - 1;
                bool ok = true;
                for (int g = 0; g < d.k && ok; ++g) {
                    if (used_pos[(size_t)g]) continue;
                    while (hi >= 0 && taken[(size_t)hi]) --hi;
                    if (hi < 0) ok = false;
                    else {
                        nb[g] = hi;
                        taken[(size_t)hi] = 1;
                    }
                }
                for (int g = 0; g < d.k && ok; ++g)
                    for (int h = g + 1; h < d.k; ++h) ok = ok && nb[g] != nb[h];
                // a group on the three lowest tile bits would read eight
                // scattered amplitudes per lane: keep the LDS tile there
                for (int g = 0; g < d.k && ok; ++g) ok = nb[g] >= 3;
                if (ok) {
                    for (int g = 0; g < d.k; ++g) d.bit[g] = nb[g];
                    ps.direct = 1;
                }
            }
            // barriers: only between ops that are not both wave-private (a wave
            // holds 64 lanes x 2^k amplitudes of a group, tile bits 0 .. 5+k)
            auto wave_private = [&](const DevOp& d) {
                if (d.type != DOP_GROUP) return false;
                for (int g = 0; g < d.k; ++g)
                    if (d.bit[g] >= 6 + d.k) return false;
                return true;
            };
            for (int32_t i = ps.op_begin; i < ps.op_end; ++i) {
                const bool last = i + 1 == ps.op_end;
                sc.devops[i].barrier =
                    (last || !wave_private(sc.devops[i]) || !wave_private(sc.devops[i + 1])) ? 1 : 0;
                const DevOp& d = sc.devops[i];
                if (d.type == DOP_GROUP)
                    for (int j = d.mat; j < d.mat + d.rank; ++j) ps.has_slot1 |= sc.subs[j].type == SUB_SLOT1;
            }
            sc.passes.push_back(ps);
            first = false;
            if (sc.passes.size() > (size_t)4 * nops + 8) break;  // every pass applies an op; never reached
        }
    };
    // the shared prefix, then the per-path ranges (each at least one pass:
    // the first also copies the prefix state into each path's row)
    if (cuts[1] > cuts[0]) schedule_range(cuts[0], cuts[1], true);
    sc.n_prefix_passes = (int)sc.passes.size();
    for (size_t r = 1; r + 1 < cuts.size(); ++r) {
        const int pb = (int)sc.passes.size();
        schedule_range(cuts[r], cuts[r + 1], false);
        if (tree) {
            TreeLevel tl;
            tl.pass_begin = pb;
            tl.pass_end = (int)sc.passes.size();
            // paths per state: the digits of blocks levels[r] .. K-1 still open
            tl.S = 1;
            for (size_t k = (size_t)levels[r]; k < p.blocks.size(); ++k) tl.S *= p.blocks[k].rank;
            tl.ops = cuts[r + 1] - cuts[r];
            sc.levels.push_back(tl);
        }
    }
    return sc;
}

int pick_schedule(const Plan& p, int64_t n_paths) {
    // smallest tile that still gives every compute unit a workgroup; more
    // passes cost extra trips through HBM, so stop at the first that does
    const int64_t target = 256;
    const size_t n = std::max(p.side[0].sched.size(), p.side[1].sched.size());
    for (size_t i = 0; i < n; ++i) {
        int64_t wgs = 0;
        for (int s = 0; s < 2; ++s) {
            const auto& v = p.side[s].sched;
            const Schedule& sc = v[std::min(i, v.size() - 1)];
            wgs += n_paths << std::max(0, p.side[s].nq - sc.tile_bits);
        }
        if (wgs >= target) return (int)i;
    }
    return (int)n - 1;
}

namespace {

// Estimated time (ns) of a chunk of sweeps.  A pass costs each workgroup
// about 2^L x (its work) x 0.13 ns on an L-qubit tile: every register group
// is one round trip of the tile through LDS and every sub-op one sweep of
// the VALU over it, a dense k-qubit op about 2^k of those, the tile's load
// and store about six.  The workgroups of both sides share 256 compute
// units: a round of launches takes the larger of its total work spread over
// them (scaled by the tile size's throughput factor) and one workgroup's
// own time, plus about 10 us (the shortest sweep launch measured).  The
// constants are fitted to MI355X timings of the c2p, C2, C3, C4 and QAOA
// sweeps at forced tile sizes 9 .. 14; the estimate ranks the candidates of
// one workload, its absolute scale is loose.
struct PassRun {
    const Schedule* sc;
    int k;
    int64_t rows;
};

double pass_ns(const Schedule& sc, int k) {
    const Pass& ps = sc.passes[(size_t)k];
    double work = 6.0;
    for (int32_t i = ps.op_begin; i < ps.op_end; ++i) {
        const DevOp& d = sc.devops[(size_t)i];
        work += d.type == DOP_GROUP ? 1.0 + (double)d.rank : 1.0 + (double)(1 << d.k);
    }
    return std::ldexp(work * 0.13, ps.n_local);
}

// One workgroup's own time on the pass: the work above, and at least about
// 400 ns per device op however small the tile (LDS and record latency and
// the barrier between groups do not shrink with it).
double pass_latency_ns(const Schedule& sc, int k) {
    const Pass& ps = sc.passes[(size_t)k];
    return pass_ns(sc, k) + 400.0 * (double)(ps.op_end - ps.op_begin);
}

// Throughput factor of a tile size when the chip is full: larger tiles hold
// fewer waves per SIMD to hide each group's LDS latency.  Measured on
// MI355X (path-tree sweeps of C4 and the q31-1 / q33-3 QAOA shapes at forced
// tile sizes), complex64 tiles of 9 .. 14 qubits relative to 9; a complex128
// tile of L qubits takes the LDS of a complex64 tile of L + 1.
double tile_factor(int L, size_t esz) {
    static const double f[] = {1.0, 1.04, 1.09, 1.15, 1.4, 2.2};   // L = 9 .. 14
    const int i = std::min(5, std::max(0, L + (esz > 8 ? 1 : 0) - 9));
    return f[i];
}

std::vector<PassRun> side_runs(const Schedule& sc, bool tree, int64_t n) {
    std::vector<PassRun> v;
    if (!tree) {
        for (size_t k = (size_t)sc.n_prefix_passes; k < sc.passes.size(); ++k) v.push_back({&sc, (int)k, n});
        return v;
    }
    for (const TreeLevel& tl : sc.levels)
        for (int k = tl.pass_begin; k < tl.pass_end; ++k) v.push_back({&sc, k, (n - 1) / tl.S + 1});
    return v;
}

double sweep_ns(const Plan& p, bool tree, size_t i, int64_t n) {
    const size_t esz = p.dtype == HSF_C128 ? 16 : 8;
    std::vector<PassRun> runs[2];
    for (int s = 0; s < 2; ++s) {
        const std::vector<Schedule>& v = tree ? p.side[s].tree : p.side[s].sched;
        runs[s] = side_runs(v[std::min(i, v.size() - 1)], tree, n);
    }
    double t = 0;
    for (size_t j = 0; j < std::max(runs[0].size(), runs[1].size()); ++j) {
        double spread = 0, one = 0;
        for (int s = 0; s < 2; ++s) {
            if (j >= runs[s].size()) continue;
            const PassRun& r = runs[s][j];
            const double c = pass_ns(*r.sc, r.k);
            const Pass& ps = r.sc->passes[(size_t)r.k];
            spread += (double)(r.rows << ps.n_nonlocal) * c * tile_factor(ps.n_local, esz) / 256.0;
            one = std::max(one, pass_latency_ns(*r.sc, r.k));
        }
        t += 10000.0 + std::max(spread, one);
    }
    return t;
}

}  // namespace

SweepChoice choose_sweep(const Plan& p, int64_t n_paths, bool allow_tree) {
    SweepChoice best;
    best.tree = false;
    best.sched = pick_schedule(p, n_paths);
    if (n_paths <= 0) return best;
    const bool have_tree = allow_tree && !p.side[0].tree.empty() && !p.side[1].tree.empty() && p.tree_mode != 1;
    const bool have_flat = !(have_tree && p.tree_mode == 2);
    const size_t nc = std::max(p.side[0].sched.size(), p.side[1].sched.size());
    double t_best = -1;
    for (int tree = 0; tree < 2; ++tree) {
        if ((tree && !have_tree) || (!tree && !have_flat)) continue;
        for (size_t i = 0; i < nc; ++i) {
            const double t = sweep_ns(p, tree != 0, i, n_paths);
            if (t_best < 0 || t < t_best) {
                t_best = t;
                best.tree = tree != 0;
                best.sched = (int)i;
            }
        }
    }
    return best;
}

}  // namespace hsf
