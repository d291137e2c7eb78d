"""Plain FP64 hybrid Schroedinger-Feynman simulation with joint cutting
(oracle; test-only).

The steps follow the paper in its order:

1. Partition (Sec. IV-A): cut between qubit l and l+1; side b = qubits 0..l,
   side a = qubits l+1..n-1.  A gate with qubits on both sides crosses.
2. Blocks (Sec. III-A): the caller groups gates; every crossing gate must be
   covered.  A block is closed to its hull: every gate g with a <= g <= b for
   some a, b in the block, where <= is "comes no later and is connected
   through shared qubits".  (Reading: the paper only cuts blocks whose gates
   are adjacent after reordering commuting RZZs, Sec. V; the hull is the
   smallest set that can be multiplied into one operator.)
3. Block operator (Sec. IV-C): product of the hull's gates in circuit order,
   on the block's qubits, side-a bits above side-b bits, ascending qubit =
   ascending significance inside each side (index order of Sec. II-A).
4. Operator-Schmidt decomposition (Sec. IV-A, the SVD equation and the
   definitions of X_m and Y_m): reshape to rows (i^b, j^b) and columns
   (i^a, j^a), SVD, X_m from V*, Y_m from U, so A = sum_m s_m X_m (x) Y_m
   (the Schmidt form of Sec. II-B).
5. Rank: s_m > 1e-10 s_0 (reading; the paper gives no threshold); s_m/s_0 in
   (1e-13, 1e-7] is rejected as ambiguous.  sqrt(s_m) is folded into both
   factors (reading; the product is unchanged).
6. Order: blocks contracted to single nodes; Kahn's algorithm, smallest
   original gate id first (reading; the paper does not fix it).
7. Paths (Sec. III): n_p = prod_k r_k, path p has digits
   m_k = floor(p / R_k) mod r_k with R_k = prod_{k' > k} r_k' (reading: block 0
   is the most significant digit).
8. Per path, the side-a and side-b subcircuits with their factors are
   simulated separately (Sec. II-B), and the state is the sum over paths of
   the Kronecker products of the two half-states (Sec. II-B).
"""
import math

import numpy as np

from . import gates as G
from . import sv

RANK_TOL = 1e-10
AMBIG_LO = 1e-13
AMBIG_HI = 1e-7
MAX_SIDE_QUBITS = 4


class PlanError(ValueError):
    def __init__(self, code, msg):
        super().__init__(f"{code}: {msg}")
        self.code = code


def sides(circuit):
    """Per gate: 'A' (all qubits above the cut), 'B' (all at or below), 'X'."""
    cut = circuit["cut"]
    out = []
    for g in circuit["gates"]:
        lo = [q <= cut for q in g["q"]]
        out.append("B" if all(lo) else ("A" if not any(lo) else "X"))
    return out


def _closure(circuit, seed, forward):
    """Gates reachable from `seed` along shared-qubit succession."""
    gs = circuit["gates"]
    inset = np.zeros(len(gs), dtype=bool)
    inset[list(seed)] = True
    marked = {}  # qubit -> whether the latest visited gate on it is reached
    order = range(len(gs)) if forward else range(len(gs) - 1, -1, -1)
    for i in order:
        reach = inset[i] or any(marked.get(q, False) for q in gs[i]["q"])
        inset[i] = reach
        for q in gs[i]["q"]:
            marked[q] = reach
    return inset


def hull(circuit, block):
    down = _closure(circuit, block, True)
    up = _closure(circuit, block, False)
    return [int(i) for i in np.nonzero(down & up)[0]]


def block_operator(circuit, hull_ids, sa, sb):
    """Product of the hull's gates on the local register (sa bits above sb)."""
    local = {q: i for i, q in enumerate(sb)}
    local.update({q: len(sb) + i for i, q in enumerate(sa)})
    nl = len(sa) + len(sb)
    u = np.eye(1 << nl, dtype=np.complex128)
    for gid in hull_ids:
        g = circuit["gates"][gid]
        u = sv.embed(nl, [local[q] for q in g["q"]], G.matrix(g)) @ u
    return u


def schmidt(u, na, nb):
    """Operator-Schmidt decomposition of a (2^(na+nb))^2 operator whose
    index is (i^a, i^b) with i^a more significant.  Returns (s, X, Y) with
    u = sum_m s[m] kron(X[m], Y[m]), s descending."""
    da, db = 1 << na, 1 << nb
    t = u.reshape(da, db, da, db)            # [i_a, i_b, j_a, j_b]
    at = t.transpose(1, 3, 0, 2).reshape(db * db, da * da)  # rows (i_b,j_b), cols (i_a,j_a)
    w, s, vh = np.linalg.svd(at, full_matrices=False)
    X = np.stack([vh[m].reshape(da, da) for m in range(len(s))])
    Y = np.stack([w[:, m].reshape(db, db) for m in range(len(s))])
    return s, X, Y


def rank_of(s, tol=RANK_TOL):
    if len(s) == 0 or s[0] == 0.0:
        raise PlanError("RANK_AMBIGUOUS", "zero block operator")
    rel = s / s[0]
    amb = (rel > AMBIG_LO) & (rel <= AMBIG_HI)
    if np.any(amb):
        raise PlanError("RANK_AMBIGUOUS", f"singular value ratio {rel[amb][0]:.3e}")
    return int(np.sum(rel > tol))


def plan(circuit, blocks=None, tol=RANK_TOL, max_side=MAX_SIDE_QUBITS):
    n, cut = circuit["n"], circuit["cut"]
    if not (0 <= cut < n - 1):
        raise PlanError("CUT", f"cut {cut} outside 0..{n - 2}")
    gs = circuit["gates"]
    blocks = circuit["blocks"] if blocks is None else blocks
    side = sides(circuit)
    nb = cut + 1
    na = n - nb

    owner = -np.ones(len(gs), dtype=np.int64)
    hulls = []
    for bi, blk in enumerate(blocks):
        if len(blk) == 0:
            raise PlanError("ARG", "empty block")
        h = hull(circuit, blk)
        if np.any(owner[h] >= 0):
            raise PlanError("BLOCK_OVERLAP", f"block {bi} overlaps another block")
        owner[h] = bi
        hulls.append(h)
    for i, s_ in enumerate(side):
        if s_ == "X" and owner[i] < 0:
            raise PlanError("BLOCK_UNCOVERED", f"crossing gate {i} is in no block")

    # contracted DAG: node id = ("g", gid) or ("b", block index)
    def node(i):
        return ("b", int(owner[i])) if owner[i] >= 0 else ("g", i)

    key = {}
    for i in range(len(gs)):
        nd = node(i)
        key.setdefault(nd, i)
    succ = {nd: set() for nd in key}
    indeg = {nd: 0 for nd in key}
    last = {}
    for i, g in enumerate(gs):
        nd = node(i)
        for q in g["q"]:
            if q in last and last[q] != nd and nd not in succ[last[q]]:
                succ[last[q]].add(nd)
                indeg[nd] += 1
            last[q] = nd
    import heapq
    ready = [(key[nd], nd) for nd in key if indeg[nd] == 0]
    heapq.heapify(ready)
    order = []
    while ready:
        _, nd = heapq.heappop(ready)
        order.append(nd)
        for s2 in succ[nd]:
            indeg[s2] -= 1
            if indeg[s2] == 0:
                heapq.heappush(ready, (key[s2], s2))
    if len(order) != len(key):
        raise PlanError("BLOCK_CYCLE", "blocks form a cycle in the contracted circuit")

    # number blocks in topological order
    blk_order = [nd[1] for nd in order if nd[0] == "b"]
    info = []
    for bi in blk_order:
        h = hulls[bi]
        qs = sorted({q for gid in h for q in gs[gid]["q"]})
        sa = [q for q in qs if q > cut]
        sb = [q for q in qs if q <= cut]
        if len(sa) > max_side or len(sb) > max_side:
            raise PlanError("BLOCK_TOO_LARGE", f"block support {len(sa)}|{len(sb)}")
        u = block_operator(circuit, h, sa, sb)
        s, X, Y = schmidt(u, len(sa), len(sb))
        r = rank_of(s, tol)
        root = np.sqrt(s[:r])
        info.append({"hull": h, "sa": sa, "sb": sb, "rank": r, "sigma": s,
                     "Xh": X[:r] * root[:, None, None], "Yh": Y[:r] * root[:, None, None],
                     "U": u, "caller_index": bi})
    ranks = [b["rank"] for b in info]
    P = 1
    for r in ranks:
        P *= r
        if P > 2 ** 62:
            raise PlanError("PATHS_OVERFLOW", "more than 2^62 paths")
    strides = [1] * len(ranks)
    for k in range(len(ranks) - 2, -1, -1):
        strides[k] = strides[k + 1] * ranks[k + 1]
    kpos = {bi: k for k, bi in enumerate(blk_order)}

    prog_a, prog_b = [], []
    for nd in order:
        if nd[0] == "g":
            g = gs[nd[1]]
            if side[nd[1]] == "A":
                prog_a.append(("gate", nd[1]))
            else:
                prog_b.append(("gate", nd[1]))
        else:
            k = kpos[nd[1]]
            prog_a.append(("slot", k))
            prog_b.append(("slot", k))
    return {"n": n, "cut": cut, "na": na, "nb": nb, "blocks": info, "ranks": ranks,
            "strides": strides, "P": P, "order": order, "prog": {"A": prog_a, "B": prog_b}}


def digits(pl, p):
    return [(p // R) % r for R, r in zip(pl["strides"], pl["ranks"])]


def path_table(pl):
    """Integer path table: ranks, hull ids, block supports (bit-exact part)."""
    return {"K": len(pl["ranks"]), "ranks": list(pl["ranks"]),
            "hulls": [list(b["hull"]) for b in pl["blocks"]],
            "sa": [list(b["sa"]) for b in pl["blocks"]],
            "sb": [list(b["sb"]) for b in pl["blocks"]], "P": pl["P"]}


def side_ops(circuit, pl, side, factors=None):
    """Op list of one side's subcircuit on its local register: gates as
    (qubits, [matrix]); factor slots as (qubits, [factor_0, ..., factor_r-1]).
    `factors[k]` replaces the plan's factors of block k (used to compare
    half-states with another implementation's Schmidt factors)."""
    off = 0 if side == "B" else pl["nb"]
    ops, slot_of = [], []
    for kind, idx in pl["prog"][side]:
        if kind == "gate":
            g = circuit["gates"][idx]
            ops.append(([q - off for q in g["q"]], [G.matrix(g)]))
            slot_of.append(-1)
        else:
            b = pl["blocks"][idx]
            sup = b["sa"] if side == "A" else b["sb"]
            fac = (factors[idx] if factors is not None else (b["Xh"] if side == "A" else b["Yh"]))
            if len(sup) == 0:
                # 1x1 factor: a scalar.  Kept as a scalar on side b only, the
                # other side takes the product (identity op skipped).
                continue
            ops.append(([q - off for q in reversed(sup)], list(fac)))
            slot_of.append(idx)
    return ops, slot_of


def _scalar_fold(pl, side, factors=None):
    """Blocks with no qubit on one side: the 1x1 factor becomes a per-path
    scalar.  Returns per-block scalar arrays for `side` (ones if none)."""
    out = []
    for k, b in enumerate(pl["blocks"]):
        sup = b["sa"] if side == "A" else b["sb"]
        if len(sup) == 0:
            fac = factors[k] if factors is not None else (b["Xh"] if side == "A" else b["Yh"])
            out.append(np.array([f.reshape(-1)[0] for f in fac]))
        else:
            out.append(np.ones(b["rank"], dtype=np.complex128))
    return out


def half_states(circuit, pl, side, paths=None, factors=None):
    """psi_{side,p} for the given paths (default all), shape [len, 2^n_side]."""
    paths = np.arange(pl["P"], dtype=np.int64) if paths is None else np.asarray(paths, dtype=np.int64)
    ops, slot_of = side_ops(circuit, pl, side, factors)
    n_loc = pl["na"] if side == "A" else pl["nb"]
    dig = np.array([digits(pl, int(p)) for p in paths], dtype=np.int64).reshape(len(paths), -1)
    sel = np.zeros((len(paths), len(ops)), dtype=np.int64)
    for j, k in enumerate(slot_of):
        if k >= 0:
            sel[:, j] = dig[:, k]
    psi = sv.run_many(n_loc, ops, sel)
    scal = _scalar_fold(pl, side, factors)
    for k in range(len(pl["blocks"])):
        psi *= scal[k][dig[:, k]][:, None]
    return psi


def amplitudes(circuit, pl=None, psi_a=None, psi_b=None):
    """Full state: psi[x] = sum_p psi_a[p, x >> n_b] psi_b[p, x & (2^n_b - 1)]."""
    pl = plan(circuit) if pl is None else pl
    psi_a = half_states(circuit, pl, "A") if psi_a is None else psi_a
    psi_b = half_states(circuit, pl, "B") if psi_b is None else psi_b
    return (psi_a.T @ psi_b).reshape(-1)


def amplitudes_rows(psi_a, psi_b, rows):
    """Rows x_a of the output matrix C[x_a, x_b] = psi[x_a 2^n_b + x_b]."""
    return psi_a[:, rows].T @ psi_b


def amplitudes_at(psi_a, psi_b, xs, nb):
    xs = np.asarray(xs, dtype=np.uint64)
    ia = (xs >> np.uint64(nb)).astype(np.int64)
    ib = (xs & np.uint64((1 << nb) - 1)).astype(np.int64)
    return np.einsum("pk,pk->k", psi_a[:, ia], psi_b[:, ib])


def gram_norm2(psi_a, psi_b):
    """||psi||^2 = sum_{p,q} <a_p|a_q> <b_p|b_q> without forming psi."""
    ga = psi_a.conj() @ psi_a.T
    gb = psi_b.conj() @ psi_b.T
    return float(np.real(np.sum(ga * gb)))


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.complex128).ravel()
    ref = np.asarray(ref, dtype=np.complex128).ravel()
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
