"""Seeded synthetic circuit generators.

This module only *describes* circuits: gate kinds, qubit lists, rotation
angles and (for generic gates) unitaries drawn at random.  It holds none of
the simulation arithmetic of hybrid Schroedinger-Feynman simulation: named
gates are passed on by kind and angle, and every consumer builds their
matrices from the definitions on its own.  Both the FP64 oracle and the GPU
library read circuits produced here, and nothing else is shared by them.

Conventions (Sec. II-A of the paper):

* An amplitude index is ``i = sum_q i_q 2**q`` (qubit 0 least significant).
* For a gate on qubits ``q = (q[0], ..., q[k-1])`` the gate matrix is written
  in the basis where ``q[0]`` is the most significant bit of the gate's local
  index; e.g. ``CX(q=(c, t))`` has the control as the left Kronecker factor,
  as the CNOT of Example 2.
* ``cut`` is the last qubit of the lower partition ``b``: ``b = 0..cut`` and
  ``a = cut+1..n-1`` (Sec. IV-A; Table II's "cut pos.").
* ``blocks`` lists, per jointly cut block, the gate ids the caller groups.

A gate is a dict ``{"kind", "q", "param", "param_id", "matrix"}``; a circuit
is a dict ``{"name", "n", "gates", "cut", "blocks", "meta"}``.
"""
from __future__ import annotations

import json
import math

import numpy as np

GATE_KINDS = {
    # kind: number of qubits (None = given by the matrix)
    "H": 1, "X": 1, "Y": 1, "Z": 1, "S": 1, "SDG": 1, "T": 1, "TDG": 1,
    "RX": 1, "RY": 1, "RZ": 1, "PHASE": 1,
    "CX": 2, "CZ": 2, "CP": 2, "RZZ": 2, "SWAP": 2, "ISWAP": 2,
    "U": None,
}
PARAM_KINDS = {"RX", "RY", "RZ", "PHASE", "CP", "RZZ"}


def gate(kind, q, param=None, param_id=-1, matrix=None):
    q = tuple(int(x) for x in q)
    if kind not in GATE_KINDS:
        raise ValueError(f"unknown gate kind {kind}")
    if kind == "U":
        m = np.asarray(matrix, dtype=np.complex128)
        if m.shape != (2 ** len(q), 2 ** len(q)):
            raise ValueError("U matrix shape does not match its qubits")
        matrix = m
    elif GATE_KINDS[kind] != len(q):
        raise ValueError(f"{kind} acts on {GATE_KINDS[kind]} qubits")
    if len(set(q)) != len(q):
        raise ValueError("repeated qubit in gate")
    if kind in PARAM_KINDS and param is None:
        raise ValueError(f"{kind} needs an angle")
    return {"kind": kind, "q": q, "param": None if param is None else float(param),
            "param_id": int(param_id), "matrix": matrix}


def circuit(name, n, gates, cut, blocks, **meta):
    return {"name": name, "n": int(n), "gates": list(gates), "cut": int(cut),
            "blocks": [list(map(int, b)) for b in blocks], "meta": dict(meta)}


# ---------------------------------------------------------------- sampling --

def haar_unitary(rng, d=2):
    """Haar-random d x d unitary: QR of a complex Ginibre matrix with the
    phases of R's diagonal moved into Q (Mezzadri, 'How to generate random
    matrices from the classical compact groups', Notices AMS 54, 2007)."""
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d_ = np.diagonal(r)
    return q * (d_ / np.abs(d_))[None, :]


def random_diag_phase(rng):
    a, b = rng.uniform(0.0, 2 * math.pi, size=2)
    return np.diag([np.exp(1j * a), np.exp(1j * b)])


def crossing(g, cut):
    q = g["q"]
    return any(x <= cut for x in q) and any(x > cut for x in q)


# ---------------------------------------------------------- small circuits --

def bell():
    """Example 1: H on qubit 1 (left Kronecker factor), then CNOT(1 -> 0)."""
    gs = [gate("H", (1,)), gate("CX", (1, 0))]
    return circuit("bell", 2, gs, cut=0, blocks=[[1]])


def ghz(n, cut=None):
    """H on the top qubit, then a CNOT chain downwards; one crossing CNOT."""
    cut = (n // 2 - 1) if cut is None else cut
    gs = [gate("H", (n - 1,))]
    for q in range(n - 1, 0, -1):
        gs.append(gate("CX", (q, q - 1)))
    blocks = [[i] for i, g in enumerate(gs) if crossing(g, cut)]
    return circuit(f"ghz{n}", n, gs, cut, blocks)


def qft_basis(n, x, cut=None):
    """|x> prepared with X gates, then the textbook QFT without the final
    swaps (output in bit-reversed order).  For each target qubit j, from the
    top down: H(j), then CP(pi/2**(j-k)) with every lower qubit k, k from j-1
    down to 0.  The crossing CPs of one upper-side target are one block
    (a cascade of diagonal gates, Sec. IV-D)."""
    cut = (n // 2 - 1) if cut is None else cut
    gs = [gate("X", (q,)) for q in range(n) if (x >> q) & 1]
    blocks = []
    for j in range(n - 1, -1, -1):
        gs.append(gate("H", (j,)))
        blk = []
        for k in range(j - 1, -1, -1):
            gs.append(gate("CP", (k, j), param=math.pi / 2 ** (j - k)))
            if crossing(gs[-1], cut):
                blk.append(len(gs) - 1)
        if blk:
            blocks.append(blk)
    return circuit(f"qft{n}_x{x}", n, gs, cut, blocks, x=x)


def cnot_cascade(n_targets=3):
    """Example 4: one control on the upper side, n_targets targets below."""
    n = n_targets + 1
    c = n - 1
    gs = [gate("H", (c,))] + [gate("CX", (c, t)) for t in range(n_targets - 1, -1, -1)]
    return circuit(f"cnot_cascade{n_targets}", n, gs, cut=n - 2,
                   blocks=[list(range(1, len(gs)))])


def random_circuit(seed, n, n_gates, cut=None, two_q_kinds=("CZ", "CX", "RZZ", "CP", "SWAP"),
                   p2=0.5, group=2):
    """Random circuit: Haar 1q gates and random 2q gates on random pairs.
    Consecutive crossing gates are grouped into blocks of up to `group`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cut = (n // 2 - 1) if cut is None else cut
    gs = []
    pid = 0
    for _ in range(n_gates):
        if rng.random() < p2:
            a, b = rng.choice(n, size=2, replace=False)
            kind = two_q_kinds[rng.integers(len(two_q_kinds))]
            if kind in PARAM_KINDS:
                gs.append(gate(kind, (a, b), param=rng.uniform(0, 2 * math.pi), param_id=pid))
                pid += 1
            else:
                gs.append(gate(kind, (a, b)))
        else:
            q = int(rng.integers(n))
            gs.append(gate("U", (q,), matrix=haar_unitary(rng)))
    cross = [i for i, g in enumerate(gs) if crossing(g, cut)]
    blocks = [cross[i:i + group] for i in range(0, len(cross), group)]
    return circuit(f"rand_s{seed}_n{n}", n, gs, cut, blocks, seed=seed)


# ------------------------------------------------------- brickwork helper --

def _brickwork(rng, n, depth, parity_fn, two_q, one_q="haar", diag_qubit_layers=None):
    """Layers of 1q gates on every qubit (ascending), then 2q gates on the
    pairs (q, q+1) that parity_fn(t) selects, in the order it returns them.
    Returns the gate list and, per layer, the gate id of each 2q pair."""
    gs = []
    layer_pairs = []
    diag_qubit_layers = diag_qubit_layers or set()
    for t in range(depth):
        for q in range(n):
            if (q, t) in diag_qubit_layers:
                gs.append(gate("U", (q,), matrix=random_diag_phase(rng)))
            else:
                gs.append(gate("U", (q,), matrix=haar_unitary(rng)))
        ids = {}
        for q in parity_fn(t):
            if q + 1 >= n:
                continue
            gs.append(two_q(rng, q))
            ids[q] = len(gs) - 1
        layer_pairs.append(ids)
    return gs, layer_pairs


def _cz(rng, q):
    return gate("CZ", (q, q + 1))


def _alt(n):
    return lambda t: list(range(t % 2, n - 1, 2))


def _full(n):
    return lambda t: list(range(0, n - 1, 2)) + list(range(1, n - 1, 2))


# ------------------------------------------------------------ workloads ----

def c1(seed=1):
    """n=12 on a line, cut 6|6 (b = 0..5), 8 layers of Haar 1q gates then CZ
    on alternating nearest-neighbour pairs.  The crossing CZ(5,6) occurs in
    the odd layers only; each is its own block (4 blocks, rank 2, P=16).
    Simulated in complex128."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n, cut = 12, 5
    gs, lp = _brickwork(rng, n, 8, _alt(n), _cz)
    blocks = [[lp[t][cut]] for t in range(8) if cut in lp[t]]
    return circuit("c1_n12_cut6_d8", n, gs, cut, blocks, dtype="c128", seed=seed)


def c1b(seed=1):
    """As c1, but every layer has CZ on both pair parities (even pairs, then
    odd pairs), and the crossing CZs of layers {0,1},{2,3},{4,5},{6,7} form
    4 joint blocks (2|2 hulls, rank 4, P=256).  complex128."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n, cut = 12, 5
    gs, lp = _brickwork(rng, n, 8, _full(n), _cz)
    blocks = [[lp[t][cut], lp[t + 1][cut]] for t in range(0, 8, 2)]
    return circuit("c1b_n12_cut6_d8_full", n, gs, cut, blocks, dtype="c128", seed=seed)


def _c2_blocks(lp, cut, depth):
    odd = [t for t in range(depth) if cut in lp[t]]
    return [[lp[odd[i]][cut], lp[odd[i + 1]][cut]] for i in range(0, len(odd) - 1, 2)]


def c2(seed=2):
    """n=28, cut 14|14 (b = 0..13), depth 20 of Haar 1q gates and
    alternating-brick CZ.  The 10 crossing CZ(13,14) (odd layers) form 5
    blocks {1,3},{5,7},...,{17,19}.  With Haar gates inside each block's hull
    the block rank is 4 (P=1024).  complex64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n, cut, depth = 28, 13, 20
    gs, lp = _brickwork(rng, n, depth, _alt(n), _cz)
    return circuit("c2_n28_cut14_d20", n, gs, cut, _c2_blocks(lp, cut, depth),
                   dtype="c64", seed=seed)


def c2p(seed=2):
    """C2 with the 1q gates on qubit 13 that fall inside each block's hull
    (layers L+1 and L+2 of block {L, L+2}) drawn as diagonal phases
    diag(e^{ia}, e^{ib}).  Every block then has rank 2 and P=32, the
    path-sum shape 2^14 x 32 . 32 x 2^14.  complex64."""
    n, cut, depth = 28, 13, 20
    odd = [t for t in range(depth) if t % 2 == cut % 2]
    diag = set()
    for i in range(0, len(odd) - 1, 2):
        L = odd[i]
        diag.add((cut, L + 1))
        diag.add((cut, L + 2))
    rng = np.random.Generator(np.random.PCG64(seed))
    gs, lp = _brickwork(rng, n, depth, _alt(n), _cz, diag_qubit_layers=diag)
    return circuit("c2p_n28_cut14_d20_p32", n, gs, cut, _c2_blocks(lp, cut, depth),
                   dtype="c64", seed=seed)


def c3(seed=3, n=30, layers=12, cut=None):
    """Variational circuit: layer t has RY(theta) on every qubit if t is even
    and RZ(theta) if t is odd, then RZZ(phi) on the even pairs, then on the
    odd pairs (angles uniform in [0, 2pi)).  The crossing RZZ(14,15) of
    layers {0,1,2}, {3,4,5}, ... are jointly cut (3|3 hulls, rank 4, P=256).
    Parameter ids follow gate order: 12*30 + 12*29 = 708 for n=30."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cut = (n // 2 - 1) if cut is None else cut
    gs = []
    pid = 0
    cross = []
    for t in range(layers):
        kind = "RY" if t % 2 == 0 else "RZ"
        for q in range(n):
            gs.append(gate(kind, (q,), param=rng.uniform(0, 2 * math.pi), param_id=pid))
            pid += 1
        for q in list(range(0, n - 1, 2)) + list(range(1, n - 1, 2)):
            gs.append(gate("RZZ", (q, q + 1), param=rng.uniform(0, 2 * math.pi), param_id=pid))
            pid += 1
            if q == cut:
                cross.append(len(gs) - 1)
    blocks = [cross[i:i + 3] for i in range(0, len(cross), 3)]
    return circuit(f"c3_n{n}_cut{cut + 1}_l{layers}", n, gs, cut, blocks, dtype="c64",
                   seed=seed, n_params=pid)


def c3_bitstrings(n=30, count=1024, seed=33):
    """`count` distinct uniform bitstrings in [0, 2^n); bit q is qubit q."""
    rng = np.random.Generator(np.random.PCG64(seed))
    seen = []
    s = set()
    while len(seen) < count:
        x = int(rng.integers(0, 2 ** n, dtype=np.int64))
        if x not in s:
            s.add(x)
            seen.append(x)
    return np.array(seen, dtype=np.uint64)


def c4(seed=4, n=34, depth=24, cut=None):
    """n=34, cut 17|17 (b = 0..16), depth 24 of Haar 1q gates and
    alternating-brick CZ.  The 12 crossing CZ(16,17) (even layers) form 6
    blocks {0,2},{4,6},...,{20,22} (2|2 hulls, rank 4, P=4096)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cut = (n // 2 - 1) if cut is None else cut
    gs, lp = _brickwork(rng, n, depth, _alt(n), _cz)
    ts = [t for t in range(depth) if cut in lp[t]]
    blocks = [[lp[ts[i]][cut], lp[ts[i + 1]][cut]] for i in range(0, len(ts) - 1, 2)]
    return circuit(f"c4_n{n}_cut{cut + 1}_d{depth}", n, gs, cut, blocks, dtype="c64", seed=seed)


def c5(master_seed=5, count=64, n_range=(20, 30), depth_range=(8, 24), max_cross=10, min_cross=4):
    """Batch of `count` independent circuits.  Per circuit (own spawned seed):
    n ~ U{20..30}; lower-side size n_b ~ U{n//2-2 .. n//2+2}; depth ~ U{8..24};
    Haar 1q layers and alternating-brick 2q gates, each CZ or RZZ(phi) with
    probability 1/2; crossing gates grouped in time order into consecutive
    blocks of g ~ U{1,2,3}.  A draw is repeated (same child stream) until the
    number of crossing gates lies in [min_cross, max_cross]; for Haar
    brickwork every crossing gate adds a factor 2 to the path count, which
    keeps P in 16..1024."""
    out = []
    children = np.random.SeedSequence(master_seed).spawn(count)
    for ci, ss in enumerate(children):
        rng = np.random.Generator(np.random.PCG64(ss))
        redraws = 0
        while True:
            n = int(rng.integers(n_range[0], n_range[1] + 1))
            nb = int(rng.integers(n // 2 - 2, n // 2 + 3))
            cut = nb - 1
            depth = int(rng.integers(depth_range[0], depth_range[1] + 1))
            n_cross = sum(1 for t in range(depth) if t % 2 == cut % 2)
            if min_cross <= n_cross <= max_cross:
                break
            redraws += 1
        pid = [0]

        def two_q(rng_, q, _pid=pid):
            if rng_.random() < 0.5:
                return gate("CZ", (q, q + 1))
            g = gate("RZZ", (q, q + 1), param=rng_.uniform(0, 2 * math.pi), param_id=_pid[0])
            _pid[0] += 1
            return g

        gs, lp = _brickwork(rng, n, depth, _alt(n), two_q)
        cross = [lp[t][cut] for t in range(depth) if cut in lp[t]]
        blocks = []
        i = 0
        while i < len(cross):
            g = int(rng.integers(1, 4))
            blocks.append(cross[i:i + g])
            i += g
        out.append(circuit(f"c5_{ci}_n{n}_cut{cut + 1}_d{depth}", n, gs, cut, blocks,
                           dtype="c64", redraws=redraws))
    return out


def qaoa_sbm(seed, sizes=(15, 15), p_intra=0.8, p_inter=0.1, gamma=None, beta=None):
    """Single-layer QAOA MaxCut circuit (Sec. V): H on every qubit, one RZZ
    per edge of a stochastic-block-model graph (two communities of the given
    sizes, edge probabilities p_intra inside and p_inter across), then RX on
    every qubit.  Community 0 sits on the lower qubits; the cut lies between
    the communities.  Edges are emitted community-0 edges first, then the
    crossing edges sorted by their upper endpoint, then community-1 edges, so
    that crossing RZZs with the same upper qubit are consecutive (RZZs
    commute, Sec. V).  Blocks: the crossing RZZs sharing an upper qubit."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n0, n1 = sizes
    n = n0 + n1
    cut = n0 - 1
    gamma = rng.uniform(0, math.pi) if gamma is None else gamma
    beta = rng.uniform(0, math.pi) if beta is None else beta
    edges_in0, edges_x, edges_in1 = [], [], []
    for a in range(n):
        for b in range(a + 1, n):
            same = (a < n0) == (b < n0)
            if rng.random() < (p_intra if same else p_inter):
                if same and a < n0:
                    edges_in0.append((a, b))
                elif same:
                    edges_in1.append((a, b))
                else:
                    edges_x.append((a, b))
    edges_x.sort(key=lambda e: (e[1], e[0]))
    gs = [gate("H", (q,)) for q in range(n)]
    for (a, b) in edges_in0:
        gs.append(gate("RZZ", (a, b), param=2 * gamma, param_id=0))
    blocks = []
    cur_top, cur = None, []
    for (a, b) in edges_x:
        gs.append(gate("RZZ", (a, b), param=2 * gamma, param_id=0))
        if b != cur_top and cur:
            blocks.append(cur)
            cur = []
        cur_top = b
        cur.append(len(gs) - 1)
    if cur:
        blocks.append(cur)
    for (a, b) in edges_in1:
        gs.append(gate("RZZ", (a, b), param=2 * gamma, param_id=0))
    for q in range(n):
        gs.append(gate("RX", (q,), param=2 * beta, param_id=1))
    return circuit(f"qaoa_sbm_s{seed}_{n0}_{n1}", n, gs, cut, blocks, dtype="c64",
                   n_edges=len(edges_in0) + len(edges_x) + len(edges_in1),
                   n_cross=len(edges_x))


WORKLOADS = {"c1": c1, "c1b": c1b, "c2": c2, "c2p": c2p, "c3": c3, "c4": c4}


# ---------------------------------------------------------- serialisation --

def to_json(c):
    def enc(g):
        d = {"kind": g["kind"], "q": list(g["q"]), "param": g["param"], "param_id": g["param_id"]}
        if g["matrix"] is not None:
            m = np.asarray(g["matrix"])
            d["matrix"] = [[[float(v.real), float(v.imag)] for v in row] for row in m]
        return d
    return json.dumps({**{k: c[k] for k in ("name", "n", "cut", "blocks", "meta")},
                       "gates": [enc(g) for g in c["gates"]]})


def from_json(s):
    d = json.loads(s)
    gs = []
    for g in d["gates"]:
        m = None
        if "matrix" in g:
            m = np.array([[complex(re, im) for re, im in row] for row in g["matrix"]])
        gs.append(gate(g["kind"], g["q"], g["param"], g["param_id"], m))
    return circuit(d["name"], d["n"], gs, d["cut"], d["blocks"], **d["meta"])
