"""Pins of the FP64 oracle to facts the paper and the mathematics fix.

Each test compares the oracle with something other than itself: values
printed in the paper (fixtures under tests/golden/), closed forms, library
routines (scipy expm, numpy FFT), brute-force constructions and invariants.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import circuitgen as cg
from oracle import gates as G
from oracle import hsf, sv

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _m(rows):
    return np.array([[complex(*v) if isinstance(v, list) else v for v in r] for r in rows],
                    dtype=np.complex128)


# ------------------------------------------------------------ gate matrices

@pytest.mark.parametrize("kind", ["H", "X", "Y", "Z", "S", "SDG", "T", "TDG", "CX", "CZ", "SWAP", "ISWAP"])
def test_fixed_gates_unitary(kind):
    nq = cg.GATE_KINDS[kind]
    m = G.matrix(cg.gate(kind, tuple(range(nq))))
    assert np.allclose(m @ m.conj().T, np.eye(m.shape[0]), atol=1e-15)


@pytest.mark.parametrize("kind,pauli", [("RX", "X"), ("RY", "Y"), ("RZ", "Z"), ("RZZ", "ZZ")])
@pytest.mark.parametrize("theta", [0.0, 0.3, 1.234, math.pi, 5.9])
def test_rotations_match_expm(kind, pauli, theta):
    p = {"X": G.X, "Y": G.Y, "Z": G.Z, "ZZ": np.kron(G.Z, G.Z)}[pauli]
    q = (0,) if len(pauli) == 1 else (0, 1)
    m = G.matrix(cg.gate(kind, q, param=theta))
    assert np.allclose(m, scipy.linalg.expm(-0.5j * theta * p), atol=1e-14)


def test_cnot_is_printed_decomposition():
    gold = _gold("cnot_schmidt.json")
    total = sum(np.kron(np.array(t["left"], dtype=complex), np.array(t["right"], dtype=complex))
                for t in gold["terms"])
    assert np.array_equal(G.matrix(cg.gate("CX", (1, 0))), total)


# --------------------------------------------------------- Schroedinger core

def test_bell_state():
    gold = _gold("bell.json")
    want = _m(gold["amplitudes_times_sqrt2"])[:, 0] / math.sqrt(2)
    psi = sv.run(cg.bell())
    assert np.allclose(psi, want, atol=1e-15)


@pytest.mark.parametrize("n", [3, 6, 9])
def test_ghz_closed_form(n):
    psi = sv.run(cg.ghz(n))
    want = np.zeros(1 << n, dtype=complex)
    want[0] = want[-1] = 1 / math.sqrt(2)
    assert np.allclose(psi, want, atol=1e-14)


def _bitrev(y, n):
    return int(format(y, f"0{n}b")[::-1], 2)


@pytest.mark.parametrize("n,x", [(3, 5), (5, 0), (6, 37), (8, 201)])
def test_qft_of_basis_state(n, x):
    """QFT|x> = sqrt(N) ifft(e_x) (numpy), read out in bit-reversed order
    because the final swaps are omitted."""
    N = 1 << n
    e = np.zeros(N, dtype=complex)
    e[x] = 1
    f = np.fft.ifft(e) * math.sqrt(N)
    psi = sv.run(cg.qft_basis(n, x))
    got = np.array([psi[_bitrev(y, n)] for y in range(N)])
    assert np.allclose(got, f, atol=1e-13)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_core_vs_dense_unitary(seed):
    c = cg.random_circuit(seed, n=7, n_gates=60, two_q_kinds=("CZ", "CX", "RZZ", "CP", "SWAP", "ISWAP"))
    u = sv.dense_unitary(c)
    assert np.allclose(u @ u.conj().T, np.eye(u.shape[0]), atol=1e-12)
    assert np.allclose(sv.run(c), u[:, 0], atol=1e-13)


def test_core_three_qubit_matrix_any_order():
    rng = np.random.default_rng(3)
    m = cg.haar_unitary(rng, 8)
    c = cg.circuit("u3", 5, [cg.gate("H", (q,)) for q in range(5)] + [cg.gate("U", (4, 0, 2), matrix=m)], 1, [])
    assert np.allclose(sv.run(c), sv.dense_unitary(c)[:, 0], atol=1e-13)


# ----------------------------------------------------------- Schmidt step

def _sch(u, na, nb):
    s, X, Y = hsf.schmidt(u, na, nb)
    r = hsf.rank_of(s)
    return s, X, Y, r


@pytest.mark.parametrize("kind", ["CX", "CZ"])
def test_cnot_cz_schmidt(kind):
    s, X, Y, r = _sch(G.matrix(cg.gate(kind, (1, 0))), 1, 1)
    assert r == _gold("cnot_schmidt.json")["rank"]
    assert np.allclose(s[:2], [math.sqrt(2), math.sqrt(2)], atol=1e-14)


@pytest.mark.parametrize("phi", [0.3, 1.234, 2.5, 4.0])
def test_rzz_schmidt_closed_form(phi):
    s, *_ = _sch(G.matrix(cg.gate("RZZ", (1, 0), param=phi)), 1, 1)
    want = sorted([2 * abs(math.cos(phi / 2)), 2 * abs(math.sin(phi / 2))], reverse=True)
    assert np.allclose(s[:2], want, atol=1e-14)
    assert np.all(s[2:] < 1e-14)


def test_swap_rank_four():
    s, *_ , r = _sch(G.matrix(cg.gate("SWAP", (1, 0))), 1, 1)
    assert r == _gold("fig3_saturation.json")["swap_rank"]
    assert np.allclose(s, [1, 1, 1, 1], atol=1e-14)


def test_cnot_cascade_rank_two():
    gold = _gold("cnot_cascade.json")
    c = cg.cnot_cascade(gold["targets"])
    pl = hsf.plan(c)
    assert pl["ranks"] == [gold["rank_joint"]]
    singles = [[i] for i in c["blocks"][0]]
    assert hsf.plan(c, blocks=singles)["P"] == gold["paths_standard"]
    # joint and separate cutting give the same state
    psi_j = hsf.amplitudes(c, pl)
    psi_s = hsf.amplitudes(c, hsf.plan(c, blocks=singles))
    assert np.allclose(psi_j, psi_s, atol=1e-14)
    assert np.allclose(psi_j, sv.run(c), atol=1e-14)


@pytest.mark.parametrize("na,nb,seed", [(1, 1, 0), (1, 2, 1), (2, 2, 2), (3, 1, 3), (2, 3, 4)])
def test_schmidt_reconstruction_and_invariants(na, nb, seed):
    rng = np.random.default_rng(seed)
    u = cg.haar_unitary(rng, 1 << (na + nb))
    s, X, Y = hsf.schmidt(u, na, nb)
    recon = sum(s[m] * np.kron(X[m], Y[m]) for m in range(len(s)))
    assert np.max(np.abs(recon - u)) < 1e-12
    assert abs(np.sum(s ** 2) - 2 ** (na + nb)) < 1e-10       # sum s^2 = ||U||_F^2
    assert hsf.rank_of(s) <= min(4 ** na, 4 ** nb)           # Sec. IV-B bound
    assert np.all(np.diff(s) <= 1e-12)


def test_rank_saturates_for_deep_two_two_block():
    """Sec. III-A Example 3: a deep block across a 2|2 split saturates at 16
    paths, while separate cutting keeps multiplying ranks."""
    gold = _gold("fig3_saturation.json")
    rng = np.random.default_rng(7)
    gs = []
    for layer in range(8):
        for q in range(4):
            gs.append(cg.gate("U", (q,), matrix=cg.haar_unitary(rng)))
        gs.append(cg.gate("CZ", (1, 2)))
        gs.append(cg.gate("SWAP", (0, 3)) if layer == 3 else cg.gate("CX", (3, 0)))
    c = cg.circuit("deep", 4, gs, 1, [])
    cross = [i for i, g in enumerate(gs) if cg.crossing(g, 1)]
    joint = hsf.plan(c, blocks=[cross])
    assert joint["P"] == gold["saturation"]
    sep = hsf.plan(c, blocks=[[i] for i in cross])
    assert sep["P"] == 2 ** (len(cross) - 1) * 4
    assert joint["P"] <= sep["P"]
    assert np.allclose(hsf.amplitudes(c, joint), sv.run(c), atol=1e-12)


@pytest.mark.parametrize("seed", [21, 22, 23, 24])
def test_joint_rank_submultiplicative(seed):
    c = cg.random_circuit(seed, n=6, n_gates=40, group=3)
    pj = hsf.plan(c)
    for b in pj["blocks"]:
        cross = [i for i in b["hull"] if cg.crossing(c["gates"][i], c["cut"])]
        single = 1
        for i in cross:
            u = G.matrix(c["gates"][i])
            single *= hsf.rank_of(hsf.schmidt(u, 1, 1)[0]) if len(u) == 4 else 1
        assert b["rank"] <= single


def test_rank_ambiguous_rejected():
    u = np.kron(G.P0, G.I2) + np.kron(G.P1, G.X) * 1e-9
    with pytest.raises(hsf.PlanError) as e:
        hsf.rank_of(hsf.schmidt(u, 1, 1)[0])
    assert e.value.code == "RANK_AMBIGUOUS"


# ------------------------------------------------------------- HSF itself

@pytest.mark.parametrize("seed,n,group,mult,p2", [(31, 6, 1, 6, 0.5), (32, 8, 2, 4, 0.3), (33, 10, 2, 4, 0.3),
                                                   (34, 12, 3, 4, 0.3), (35, 14, 2, 4, 0.3)])
def test_hsf_equals_schroedinger(seed, n, group, mult, p2):
    c = cg.random_circuit(seed, n=n, n_gates=mult * n, group=group, p2=p2,
                          two_q_kinds=("CZ", "CX", "RZZ", "CP", "ISWAP"))
    pl = hsf.plan(c)
    assert 2 <= pl["P"] <= 1024
    ref = sv.run(c)
    got = hsf.amplitudes(c, pl)
    assert hsf.rel_l2(got, ref) < 1e-12
    assert abs(np.linalg.norm(got) - 1) < 1e-12


@pytest.mark.parametrize("maker", [cg.c1, cg.c1b])
def test_hsf_equals_schroedinger_c1(maker):
    c = maker()
    got = hsf.amplitudes(c)
    assert hsf.rel_l2(got, sv.run(c)) < 1e-12


def test_singleton_and_joint_blocks_agree():
    c = cg.c1b()
    cross = [i for i, g in enumerate(c["gates"]) if cg.crossing(g, c["cut"])]
    ps = hsf.plan(c, blocks=[[i] for i in cross])
    pj = hsf.plan(c)
    assert ps["P"] == 2 ** len(cross) and pj["P"] == 256
    assert hsf.rel_l2(hsf.amplitudes(c, ps), hsf.amplitudes(c, pj)) < 1e-12


def test_no_crossing_gates_is_a_kronecker_product():
    rng = np.random.default_rng(5)
    gs = [cg.gate("U", (q,), matrix=cg.haar_unitary(rng)) for q in range(6)]
    gs += [cg.gate("CZ", (0, 1)), cg.gate("CX", (2, 1)), cg.gate("CZ", (4, 5)), cg.gate("RZZ", (3, 4), param=0.7)]
    c = cg.circuit("split", 6, gs, 2, [])
    pl = hsf.plan(c)
    assert pl["P"] == 1 and pl["ranks"] == []
    a = hsf.half_states(c, pl, "A")[0]
    b = hsf.half_states(c, pl, "B")[0]
    assert np.allclose(np.kron(a, b), sv.run(c), atol=1e-14)


@pytest.mark.parametrize("n", [4, 6, 8])
def test_qft_cascades_give_two_to_the_upper_side(n):
    c = cg.qft_basis(n, 3)
    pl = hsf.plan(c)
    assert pl["P"] == 2 ** pl["na"]
    assert all(r == 2 for r in pl["ranks"])
    assert hsf.rel_l2(hsf.amplitudes(c, pl), sv.run(c)) < 1e-12


def test_ghz_two_paths():
    c = cg.ghz(8)
    pl = hsf.plan(c)
    assert pl["P"] == 2
    assert np.allclose(hsf.amplitudes(c, pl), sv.run(c), atol=1e-14)


def test_gram_norm_matches_direct():
    c = cg.c1b()
    pl = hsf.plan(c)
    a = hsf.half_states(c, pl, "A")
    b = hsf.half_states(c, pl, "B")
    assert abs(hsf.gram_norm2(a, b) - 1) < 1e-12
    assert abs(hsf.gram_norm2(a, b) - np.linalg.norm(hsf.amplitudes(c, pl, a, b)) ** 2) < 1e-12


def test_chunked_path_sum_is_additive():
    c = cg.c1b()
    pl = hsf.plan(c)
    a = hsf.half_states(c, pl, "A")
    b = hsf.half_states(c, pl, "B")
    full = a.T @ b
    half = pl["P"] // 2
    parts = a[:half].T @ b[:half] + a[half:].T @ b[half:]
    assert np.allclose(parts, full, atol=1e-15)


def test_amplitudes_at_and_rows():
    c = cg.c1()
    pl = hsf.plan(c)
    a = hsf.half_states(c, pl, "A")
    b = hsf.half_states(c, pl, "B")
    psi = sv.run(c)
    xs = np.array([0, 1, 77, 4095, 2048, 123], dtype=np.uint64)
    assert np.allclose(hsf.amplitudes_at(a, b, xs, pl["nb"]), psi[xs.astype(np.int64)], atol=1e-14)
    rows = [0, 5, 63]
    r = hsf.amplitudes_rows(a, b, rows)
    assert np.allclose(r, psi.reshape(64, 64)[rows], atol=1e-14)


# --------------------------------------------------------------- path table

def test_path_digits_bijection():
    c = cg.c1b()
    pl = hsf.plan(c)
    seen = [tuple(hsf.digits(pl, p)) for p in range(pl["P"])]
    assert seen == list(itertools.product(*[range(r) for r in pl["ranks"]]))


def test_paths_equal_product_of_ranks():
    for maker in (cg.c1, cg.c1b, cg.c2p, cg.c3):
        pl = hsf.plan(maker())
        assert pl["P"] == int(np.prod(pl["ranks"]))


def test_table2_path_identity():
    """Table I/II: joint paths 2^(blocks+sep), standard 2^(sep cuts)."""
    gold = _gold("table2_paths.json")
    for row in gold["rows"]:
        d = dict(zip(gold["columns"], row))
        assert d["paths_joint_log2"] == d["blocks"] + d["sep"]
        assert d["paths_standard_log2"] == d["sep_cuts"]


@pytest.mark.parametrize("seed", [1, 2])
def test_qaoa_cascades_rank_two(seed):
    """Sec. IV-D / Sec. V: RZZ cascades sharing a qubit have rank 2, so the
    joint path count is 2^(number of blocks) as in Table I/II."""
    c = cg.qaoa_sbm(seed, sizes=(5, 5), p_intra=0.6, p_inter=0.4)
    pl = hsf.plan(c)
    assert all(r == 2 for r in pl["ranks"])
    assert pl["P"] == 2 ** len(c["blocks"])
    singles = [[i] for b in c["blocks"] for i in b]
    assert hsf.plan(c, blocks=singles)["P"] == 2 ** c["meta"]["n_cross"]
    assert hsf.rel_l2(hsf.amplitudes(c, pl), sv.run(c)) < 1e-12


# ------------------------------------------------------------ planner errors

def test_plan_errors():
    c = cg.c1()
    with pytest.raises(hsf.PlanError) as e:
        hsf.plan(c, blocks=c["blocks"][:-1])
    assert e.value.code == "BLOCK_UNCOVERED"
    with pytest.raises(hsf.PlanError) as e:
        hsf.plan(c, blocks=c["blocks"] + [c["blocks"][0]])
    assert e.value.code == "BLOCK_OVERLAP"
    with pytest.raises(hsf.PlanError) as e:
        hsf.plan(cg.circuit("x", 4, c["gates"][:0], 3, []))
    assert e.value.code == "CUT"
    big = cg.c1b()
    cross = [i for b in big["blocks"] for i in b]
    with pytest.raises(hsf.PlanError) as e:
        hsf.plan(big, blocks=[cross])
    assert e.value.code == "BLOCK_TOO_LARGE"


def test_plan_cycle_detected():
    """Two convex blocks that each need the other first: B1 = {CZ(1,2), CZ(1,3)},
    B2 = {CZ(0,3), CZ(2,0)}; CZ(0,3) precedes CZ(1,3) and CZ(1,2) precedes CZ(2,0)."""
    gs = [cg.gate("CZ", (1, 2)), cg.gate("CZ", (0, 3)), cg.gate("CZ", (1, 3)), cg.gate("CZ", (2, 0))]
    c = cg.circuit("cyc", 4, gs, 1, [])
    assert hsf.hull(c, [0, 2]) == [0, 2] and hsf.hull(c, [1, 3]) == [1, 3]
    with pytest.raises(hsf.PlanError) as e:
        hsf.plan(c, blocks=[[0, 2], [1, 3]])
    assert e.value.code == "BLOCK_CYCLE"
