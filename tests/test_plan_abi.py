"""Host-side tests of libhsf through its C ABI (no GPU needed): the library
loads and exports every declared symbol, the planner's integer path table
equals the oracle's independent planner bit for bit, its Schmidt factors
reproduce the oracle's block operators, and every error status is reachable.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import circuitgen as cg
from oracle import hsf as ohsf
from paper_2502_06959_amd import HsfError, Plan
from paper_2502_06959_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_header_symbol():
    hdr = open(os.path.join(ROOT, "include", "hsf.h")).read()
    names = set(re.findall(r"\b(hsf_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) >= 15
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing
    assert set(L.SIGNATURES) == names
    assert L.lib().hsf_version().decode().startswith("libhsf")


def _workloads():
    out = [cg.bell(), cg.ghz(9), cg.qft_basis(8, 77), cg.cnot_cascade(3), cg.c1(), cg.c1b(), cg.c2(), cg.c2p(),
           cg.c3(), cg.c4(), cg.qaoa_sbm(3, sizes=(6, 7), p_intra=0.5, p_inter=0.3)]
    for s in range(40, 46):
        out.append(cg.random_circuit(s, n=9, n_gates=40, group=2, p2=0.4))
    out += cg.c5(count=6)
    return out


@pytest.mark.parametrize("c", _workloads(), ids=lambda c: c["name"])
def test_path_table_bit_exact(c):
    o = ohsf.plan(c)
    p = Plan(c)
    assert (p.n, p.cut, p.na, p.nb, p.K, p.P) == (o["n"], o["cut"], o["na"], o["nb"], len(o["ranks"]), o["P"])
    for k in range(p.K):
        bi = p.block_info(k)
        ob = o["blocks"][k]
        assert bi["rank"] == ob["rank"]
        assert bi["stride"] == o["strides"][k]
        assert bi["hull"] == ob["hull"]
        assert bi["sa"] == ob["sa"] and bi["sb"] == ob["sb"]
        assert bi["caller_index"] == ob["caller_index"]
    rng = np.random.default_rng(0)
    ps = range(p.P) if p.P <= 4096 else rng.integers(0, p.P, 512)
    for q in ps:
        assert p.digits(int(q)) == ohsf.digits(o, int(q))


@pytest.mark.parametrize("maker", [cg.c1, cg.c1b, cg.c2p, cg.c3, cg.c4, cg.cnot_cascade],
                         ids=lambda f: f.__name__)
def test_factors_reproduce_block_operator(maker):
    c = maker()
    o = ohsf.plan(c)
    p = Plan(c)
    for k in range(p.K):
        sig, xa, yb = p.block_factors(k)
        ob = o["blocks"][k]
        assert np.allclose(sig, ob["sigma"], atol=1e-12)
        recon = sum(np.kron(xa[m], yb[m]) for m in range(len(xa)))
        assert np.max(np.abs(recon - ob["U"])) < 1e-12


def test_singleton_blocks_standard_cutting():
    c = cg.c1b()
    cross = [i for i, g in enumerate(c["gates"]) if cg.crossing(g, c["cut"])]
    p = Plan(c, blocks=[[i] for i in cross])
    assert p.P == 2 ** len(cross)


def _code(fn):
    with pytest.raises(HsfError) as e:
        fn()
    return e.value.code


def test_error_statuses():
    c = cg.c1()
    assert _code(lambda: Plan(c, blocks=c["blocks"][:-1])) == "HSF_E_BLOCK_UNCOVERED"
    assert _code(lambda: Plan(c, blocks=c["blocks"] + [c["blocks"][0]])) == "HSF_E_BLOCK_OVERLAP"
    assert _code(lambda: Plan(c, cut=11)) == "HSF_E_CUT"
    assert _code(lambda: Plan(c, cut=-1)) == "HSF_E_CUT"
    big = cg.c1b()
    assert _code(lambda: Plan(big, blocks=[[i for b in big["blocks"] for i in b]])) == "HSF_E_BLOCK_TOO_LARGE"
    gs = [cg.gate("CZ", (1, 2)), cg.gate("CZ", (0, 3)), cg.gate("CZ", (1, 3)), cg.gate("CZ", (2, 0))]
    cyc = cg.circuit("cyc", 4, gs, 1, [[0, 2], [1, 3]])
    assert _code(lambda: Plan(cyc)) == "HSF_E_BLOCK_CYCLE"
    near = np.eye(4, dtype=complex)
    near[3, 3] = 1 + 1e-9          # diag(1,1,1,1+1e-9): Schmidt ratio ~ 2.5e-10
    amb = cg.circuit("amb", 2, [cg.gate("U", (1, 0), matrix=near)], 0, [[0]])
    assert _code(lambda: Plan(amb)) == "HSF_E_RANK_AMBIGUOUS"
    # 32 blocks of rank 4 -> 2^64 paths
    rng = np.random.default_rng(1)
    many = []
    for _ in range(33):
        many.append(cg.gate("U", (1, 0), matrix=cg.haar_unitary(rng, 4)))
    ov = cg.circuit("ov", 2, many, 0, [[i] for i in range(33)])
    assert _code(lambda: Plan(ov)) == "HSF_E_PATHS_OVERFLOW"
    bad = cg.circuit("bad", 3, [cg.gate("CZ", (0, 1))], 0, [[5]])
    assert _code(lambda: Plan(bad)) == "HSF_E_ARG"


def test_ambiguous_matches_oracle_rule():
    near = np.eye(4, dtype=complex)
    near[3, 3] = 1 + 1e-9
    amb = cg.circuit("amb", 2, [cg.gate("U", (1, 0), matrix=near)], 0, [[0]])
    with pytest.raises(ohsf.PlanError) as e:
        ohsf.plan(amb)
    assert e.value.code == "RANK_AMBIGUOUS"


def test_null_and_range_arguments():
    lib = L.lib()
    assert lib.hsf_run_paths(None, 0, 1, None, 0, None, 0, None, 0, None) == 1
    assert lib.hsf_num_paths(None) == -1
    p = Plan(cg.c1())
    assert lib.hsf_run_paths(ctypes.c_void_p(p.handle), 0, p.P + 1, None, 0, None, 0, None, 0, None) == 1
    assert "path range" in lib.hsf_last_error().decode()
    d = (ctypes.c_int32 * 8)()
    assert lib.hsf_path_digits(ctypes.c_void_p(p.handle), p.P, d) == 1
    assert lib.hsf_workspace_size(ctypes.c_void_p(p.handle), 1, 16, 1) > 0
    # empty calls need no buffers and return before any device work
    h, ma, mb = ctypes.c_void_p(p.handle), 1 << p.na, 1 << p.nb
    assert lib.hsf_run_paths(h, 3, 3, None, 0, None, 0, None, 0, None) == 0
    assert lib.hsf_amplitudes_full(h, None, ma, None, mb, 0, 3, 3, None, mb, 3, 0, None, 0, None) == 0
    assert lib.hsf_amplitudes_bitstrings(h, None, ma, None, mb, 0, None, 0, None, 0, None) == 0
    # paths without operands, or rows without an output: errors
    assert lib.hsf_amplitudes_full(h, None, ma, None, mb, 4, 0, 1, None, mb, 3, 0, None, 0, None) == 1
    assert "null" in lib.hsf_last_error().decode()
    assert lib.hsf_amplitudes_bitstrings(h, None, ma, None, mb, 4, None, 2, None, 0, None) == 1


def test_multi_pass_schedule_shapes():
    c = cg.c2p()
    for tq in (8, 10, 12, 14):
        p = Plan(c, tile_qubits=tq)
        for s in (0, 1):
            st = p.side_stats(s)
            assert st["tile_qubits"] == tq
            assert (st["passes"] == 1) == (tq >= 14)


def test_path_tree_levels_by_hand():
    """Levels of the path tree (hsf_side_levels): an op's level is the number
    of leading digits its result depends on -- a slot of block k needs
    k + 1, and an op follows every earlier op it does not commute with
    (disjoint qubits, or both diagonal).  Derived by hand for this circuit
    (no fusion): the two crossing CZ(1, 2) are blocks 0 and 1 (product form,
    rank 2, diagonal slots on qubit 2 of side a and qubit 1 of side b)."""
    g = cg.gate
    gates = [g("H", (0,)), g("H", (1,)), g("H", (2,)), g("H", (3,)),   # level 0
             g("CZ", (1, 2)),                 # block 0: slots at level 1
             g("RX", (2,), 0.4, 0),           # a: dense after slot 0 on qubit 2 -> 1
             g("H", (3,)),                    # a: disjoint from both slots -> 0
             g("CZ", (1, 2)),                 # block 1: slots at level 2
             g("RX", (0,), 0.5, 1),           # b: disjoint -> 0
             g("RX", (1,), 0.6, 2),           # b: dense after slot 1 on qubit 1 -> 2
             g("RZ", (2,), 0.7, 3)]           # a: diagonal; the level-2 slot on 2 is diagonal
    #                                           and commutes, RX(2) at level 1 does not -> 1
    c = cg.circuit("levels", 4, gates, 1, [[4], [7]])
    p = Plan(c, fuse=False, tree="on")
    assert p.P == 4
    # levels -- side a: H2 H3 H3 | slot0 RX2 RZ2 | slot1 ; side b: H0 H1 RX0 |
    # slot0 | slot1 RX1.  Then a thin level joins the next when repeating its
    # ops on the next level's states costs less than its own pass (1.5 per op
    # and extra state against 8 per state): side a's level 1 (3 ops, 2 -> 4
    # states: 4.5 < 8) and side b's (1 op: 1.5 < 8) both join level 2
    assert p.side_levels(0) == [(3, 1), (4, 4)]
    assert p.side_levels(1) == [(3, 1), (3, 4)]
    assert p.side_stats(0)["ops_shared"] == 3 and p.side_stats(1)["ops_shared"] == 3
    # thick levels keep their boundaries (C3 at n=12, side a: 13, 10 and 2
    # ops on 4, 16 and 32 states)
    q = Plan(cg.c3(seed=3, n=12, layers=8), tree="on")
    assert [n for _, n in q.side_levels(0)] == [1, 4, 16, 32]


def test_path_tree_options_and_invariants():
    from paper_2502_06959_amd.hsf import hsf_workspace_size
    c = cg.c3(seed=3, n=12, layers=8)
    on, off, auto = Plan(c, tree="on"), Plan(c, tree="off"), Plan(c)
    assert on.uses_tree(on.P) and not off.uses_tree(off.P)
    assert hsf_workspace_size(on.handle, 0, on.P, 0) > 0 and hsf_workspace_size(off.handle, 0, off.P, 0) == 0
    assert hsf_workspace_size(auto.handle, 0, auto.P, 0) == (hsf_workspace_size(on.handle, 0, on.P, 0)
                                                             if auto.uses_tree(auto.P) else 0)
    for s in (0, 1):
        lv, st = on.side_levels(s), on.side_stats(s)
        assert lv == off.side_levels(s)                 # levels are a property of the plan
        assert sum(o for o, _ in lv) == st["ops_fused"] and lv[0] == (st["ops_shared"], 1)
        states = [n for _, n in lv]
        assert states[-1] == on.P and all(a < b for a, b in zip(states, states[1:]))
        assert all(on.P % n == 0 for n in states)
    # no blocks: one level, everything shared; the tree is never taken
    g = Plan(cg.circuit("noblocks", 4, [cg.gate("H", (0,)), cg.gate("H", (3,))], 1, []), tree="on")
    assert g.side_levels(0) == [(1, 1)] and not g.uses_tree(1)
    # the sweep form: a candidate tile size of the plan (12-qubit sides: 12
    # down to 8); a forced form and tile size are kept
    w = cg.c3(seed=3, n=24, layers=4)
    for mode in ("on", "off", "auto"):
        plan = Plan(w, tree=mode)
        tree, tiles = plan.sweep_form(plan.P)
        assert tree == plan.uses_tree(plan.P) and tree == (mode != "off" and (mode == "on" or tree))
        assert all(8 <= t <= 12 for t in tiles)
    one = Plan(w, tile_qubits=9, tree="on")
    assert one.sweep_form(one.P) == (True, (9, 9))
    assert on.sweep_form(on.P)[1] == (6, 6)                 # 6-qubit sides: one tile
    with pytest.raises(HsfError):
        on.sweep_form(0)
    # an out-of-range option is the caller's error
    from paper_2502_06959_amd import hsf as H
    H._TREE["bad"] = 3
    try:
        with pytest.raises(HsfError) as e:
            Plan(c, tree="bad")
        assert e.value.code == "HSF_E_ARG"
    finally:
        del H._TREE["bad"]


def test_shared_prefix_hoists_commuting_ops():
    """Ops that commute with every factor slot before them (disjoint qubits,
    or both diagonal) join the prefix every path shares; ops that do not
    stay per path (Sec. II-B: paths differ only in the factor slots)."""
    g = cg.gate
    # cut 1: side b = qubits 0, 1; side a = qubits 2, 3.  The block is the
    # crossing CZ(1, 2); its factors (product form) are diagonal.
    gates = [g("CZ", (1, 2)),          # block: factor slots on qubit 2 (a) and 1 (b)
             g("H", (3,)),             # a: disjoint from the slot -> shared
             g("RZZ", (2, 3), 0.3),    # a: diagonal, the slot is diagonal -> shared
             g("H", (2,)),             # a: dense on the slot's qubit -> per path
             g("H", (3,)),             # a: disjoint from everything left behind -> shared
             g("H", (0,)),             # b: disjoint from the slot on 1 -> shared
             g("H", (1,))]             # b: right after the slot on its qubit -> folded into its pieces
    p = Plan(cg.circuit("prefix", 4, gates, 1, [[0]]))
    a, b = p.side_stats(0), p.side_stats(1)
    # side a: slot, H(3), RZZ, H(2), H(3) (the RZZ keeps the two H(3) apart);
    # shared: H(3), RZZ, H(3)
    assert a["ops_shared"] == 3 and a["ops_fused"] == 5
    # side b: the slot (with H(1) folded in, per path) and H(0) (shared)
    assert b["ops_shared"] == 1 and b["ops_fused"] == 2
    # a dense op on the qubit of a dense factor slot stays per path
    gates2 = [g("CX", (1, 2)), g("H", (2,)), g("H", (3,))]
    p2 = Plan(cg.circuit("prefix2", 4, gates2, 1, [[0]]))
    assert p2.side_stats(0)["ops_shared"] == 1     # H(3) only
    # every side's shared ops are a part of its fused ops
    p3 = Plan(cg.ghz(6))
    for s in (0, 1):
        st = p3.side_stats(s)
        assert 0 <= st["ops_shared"] <= st["ops_fused"]
        assert st["passes"] >= 1


def test_run_paths_rows_argument_checks():
    """hsf_run_paths_rows rejects a null psiA, row ranges outside [0, 2^n_a)
    or wider than 2^20, a short ldA and bad path ranges before any device
    work; an empty path range returns at once."""
    lib = L.lib()
    p = Plan(cg.c1())
    h, ma, mb = ctypes.c_void_p(p.handle), 1 << p.na, 1 << p.nb
    dummy = ctypes.c_void_p(0x1000)      # never dereferenced: every call below fails its checks first
    assert lib.hsf_run_paths_rows(None, 0, 1, 0, 1, dummy, ma, None, 0, None, 0, None) == 1
    assert lib.hsf_run_paths_rows(h, 0, 1, 0, 1, None, ma, None, 0, None, 0, None) == 1
    assert "null" in lib.hsf_last_error().decode()
    assert lib.hsf_run_paths_rows(h, 0, 1, 2, 1, dummy, ma, None, 0, None, 0, None) == 1
    assert lib.hsf_run_paths_rows(h, 0, 1, 0, ma + 1, dummy, ma, None, 0, None, 0, None) == 1
    assert "row range" in lib.hsf_last_error().decode()
    assert lib.hsf_run_paths_rows(h, 0, 1, 0, 1, dummy, ma - 1, None, 0, None, 0, None) == 1
    assert lib.hsf_run_paths_rows(h, 0, 1, 0, 1, dummy, ma, dummy, mb - 1, None, 0, None) == 1
    assert lib.hsf_run_paths_rows(h, 0, p.P + 1, 0, 1, dummy, ma, None, 0, None, 0, None) == 1
    assert "path range" in lib.hsf_last_error().decode()
    assert lib.hsf_run_paths_rows(h, 2, 2, 0, 1, dummy, ma, None, 0, None, 0, None) == 0


def test_batch_tune_cache_lookup_on_the_host():
    """hsf_batch_tune_cached: no recorded policy for a fresh batch shape (-1,
    host only, no device work), argument checks through the C ABI."""
    from paper_2502_06959_amd.hsf import Batch
    plans = [Plan(c, dtype="c64") for c in cg.c5(count=2)]
    b = Batch(plans)
    try:
        assert b.tuned_policy("bf16x3") == -1
        assert b.tuned_policy("f32") == -1
        pol = ctypes.c_int32(7)
        assert L.lib().hsf_batch_tune_cached(ctypes.c_void_p(b.handle), L.SUM_MODE["f64"], ctypes.byref(pol)) != 0
        assert L.lib().hsf_batch_tune_cached(None, L.SUM_MODE["bf16x3"], ctypes.byref(pol)) != 0
        assert L.lib().hsf_batch_tune_cached(ctypes.c_void_p(b.handle), L.SUM_MODE["bf16x3"], None) != 0
        assert pol.value == 7
    finally:
        b.close()


def test_deferred_b_suffix_planning_and_argument_checks():
    """defer_b_suffix: side b's gates after its last factor slot leave its
    program (QAOA: the mixer's RX on every side-b qubit); option and
    hsf_apply_b_suffix argument checks on the host."""
    from paper_2502_06959_amd import joint_blocked
    c = joint_blocked(cg.qaoa_sbm(3, sizes=(6, 7), p_intra=0.5, p_inter=0.3))
    base, plan = Plan(c), Plan(c, defer_b_suffix=True)
    nb = plan.nb
    assert base.side_stats(1)["ops_logical"] - plan.side_stats(1)["ops_logical"] == nb
    assert base.side_stats(0) == plan.side_stats(0) and base.P == plan.P
    from paper_2502_06959_amd.hsf import _circuit_struct
    lib = L.lib()
    cs, keep = _circuit_struct(c)
    ids = np.array([int(i) for b in c["blocks"] for i in b], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum([len(b) for b in c["blocks"]])]).astype(np.int64)
    opts = L.HsfPlanOptions(rank_tol=1e-10, max_side_qubits=4, dtype=0, tile_qubits=0, fuse=1, tree=0,
                            defer_b_suffix=2)
    h = ctypes.c_void_p()
    st = lib.hsf_plan(ctypes.byref(cs), int(c["cut"]), ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                      offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(c["blocks"]), ctypes.byref(opts),
                      ctypes.byref(h))
    assert st != 0 and not h.value
    del keep
    dummy = ctypes.c_void_p(16)
    assert lib.hsf_apply_b_suffix(None, dummy, 1 << nb, 1, None) != 0
    assert lib.hsf_apply_b_suffix(ctypes.c_void_p(plan.handle), None, 1 << nb, 1, None) != 0
    assert lib.hsf_apply_b_suffix(ctypes.c_void_p(plan.handle), dummy, 1 << nb, -1, None) != 0
    assert lib.hsf_apply_b_suffix(ctypes.c_void_p(plan.handle), dummy, (1 << nb) - 1, 1, None) != 0
    # no rows, or no deferred gates: nothing to do, no device call
    assert lib.hsf_apply_b_suffix(ctypes.c_void_p(plan.handle), dummy, 1 << nb, 0, None) == 0
    assert lib.hsf_apply_b_suffix(ctypes.c_void_p(base.handle), dummy, 1 << nb, 4, None) == 0
