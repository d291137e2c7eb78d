"""GPU parity of the paper's own workload (Sec. V): single-layer QAOA MaxCut
circuits on stochastic-block-model graphs, cut between the two communities,
with the crossing RZZs regrouped into joint cascade blocks by
hsf_find_blocks (product-form factors).

  - small instances: the joint-cut HSF state against the FP64 Schroedinger
    oracle (complex64 rel-L2 <= 1e-5, complex128 <= 1e-12), and against
    standard cutting (every crossing gate its own block) of the same circuit;
  - the half-states against the oracle's, fed the library's factors;
  - Table II's q30-1 shape at full size: the first 10^6 amplitudes (Sec. V
    computes that many) against FP64 oracle samples, and the norm of all
    2^30 amplitudes."""
import os

import numpy as np
import pytest
import torch

import circuitgen as cg
from oracle import hsf as ohsf
from oracle import sv
from paper_2502_06959_amd import Plan, hsf_norm2, joint_blocked

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.empty_cache()


def _state(plan, mode=None):
    A, B = plan.run_paths()
    return plan.amplitudes_full(A, B, mode=mode).cpu().numpy().reshape(-1)


SMALL = [(31, (6, 6), 0.8, 0.3), (32, (7, 8), 0.8, 0.25), (33, (9, 8), 0.7, 0.2), (34, (8, 10), 0.8, 0.17)]


@pytest.mark.parametrize("seed,sizes,pin,pout", SMALL)
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_joint_cut_qaoa_against_schroedinger(seed, sizes, pin, pout, dtype):
    c = cg.qaoa_sbm(seed, sizes, pin, pout)
    r = joint_blocked(c)
    plan = Plan(r, dtype=dtype)
    assert plan.P == 2 ** len(r["blocks"])
    ref = sv.run(c)
    got = _state(plan)
    assert ohsf.rel_l2(got, ref) < (1e-12 if dtype == "c128" else 1e-5)
    if dtype == "c64":
        for mode in ("bf16x3", "f64"):
            assert ohsf.rel_l2(_state(plan, mode), ref) < 1e-5, mode


@pytest.mark.parametrize("seed,sizes,pin,pout", SMALL[:2])
def test_joint_equals_standard_cutting(seed, sizes, pin, pout):
    c = cg.qaoa_sbm(seed, sizes, pin, pout)
    r = joint_blocked(c)
    std = dict(c)
    std["blocks"] = [[i] for i, g in enumerate(c["gates"])
                     if 0 < sum(q <= c["cut"] for q in g["q"]) < len(g["q"])]
    pj, ps = Plan(r, dtype="c128"), Plan(std, dtype="c128")
    assert ps.P == 2 ** c["meta"]["n_cross"] > pj.P
    assert ohsf.rel_l2(_state(pj), _state(ps)) < 1e-12


def test_half_states_with_shared_product_factors():
    c = cg.qaoa_sbm(35, (7, 7), 0.8, 0.3)
    r = joint_blocked(c)
    plan = Plan(r, dtype="c64")
    opl = ohsf.plan(r, max_side=8)
    fa, fb = [], []
    for k in range(plan.K):
        _, xa, yb = plan.block_factors(k)
        fa.append(xa)
        fb.append(yb)
    A, B = plan.run_paths()
    for side, got, fac in (("A", A, fa), ("B", B, fb)):
        ref = ohsf.half_states(r, opl, side, factors=fac)
        g = got.cpu().numpy()
        for p in range(plan.P):
            assert ohsf.rel_l2(g[p], ref[p]) < 1e-5, (side, p)


def test_q30_first_million_amplitudes_and_norm():
    g = np.load(os.path.join(GOLDEN, "qaoa_q30.npz"))
    c = cg.qaoa_sbm(100, (15, 15), 0.8, 0.1)
    r = joint_blocked(c)
    plan = Plan(r)
    assert plan.P == 2 ** len(r["blocks"]) and plan.nb == 15
    A, B = plan.run_paths()
    rows = (10 ** 6 + (1 << plan.nb) - 1) >> plan.nb          # 31 rows = the first 1,015,808 amplitudes
    first = plan.amplitudes_full(A, B, rows=(0, rows), mode="bf16x3").reshape(-1)
    xs = torch.from_numpy(np.asarray(g["x"], dtype=np.uint64).astype(np.int64)).cuda()
    assert ohsf.rel_l2(first[xs].cpu().numpy(), g["psi"]) < 1e-5
    exact = plan.amplitudes_bitstrings(A, B, xs).cpu().numpy()
    assert ohsf.rel_l2(exact, g["psi"]) < 1e-5
    tile = torch.empty((1 << 12, 1 << plan.nb), dtype=torch.complex64, device="cuda")
    total = 0.0
    for r0 in range(0, 1 << plan.na, 1 << 12):
        plan.amplitudes_full(A, B, rows=(r0, r0 + (1 << 12)), mode="bf16x3", out=tile)
        total += float(hsf_norm2(tile.reshape(-1)).cpu().numpy()[0])
    assert abs(total - 1.0) < 1e-5


@pytest.mark.parametrize("tree", ["on", "off"])
@pytest.mark.parametrize("kind", ["qaoa", "brick"])
def test_run_paths_rows_equals_full_rows(tree, kind):
    """hsf_run_paths_rows (side a's passes, from the last back, only on the
    tiles the wanted rows depend on): those rows bit for bit hsf_run_paths',
    side b in full, on
    product-form QAOA blocks and dense brickwork blocks, path tree and flat,
    with two path chunks; row ranges inside one tile, across tiles, at the
    end and the whole side."""
    # 8-qubit tiles on sides of 12-13 qubits: 16-32 tiles per row
    if kind == "qaoa":
        plan = Plan(joint_blocked(cg.qaoa_sbm(41, (13, 12), 0.8, 0.15)), tree=tree, tile_qubits=8)
    else:
        plan = Plan(cg.c3(seed=6, n=24, layers=6), tree=tree, tile_qubits=8)
    assert plan.side_stats(0)["tile_qubits"] == 8 and plan.na >= 12
    ref_A, ref_B = plan.run_paths()
    M = 1 << plan.na
    for r0, r1 in ((0, 16), (0, 1), (37, 60), (M - 40, M - 8), (M // 2 - 5, M // 2 + 7), (1, 3), (0, M)):
        A, B = plan.alloc_halves(plan.P)
        A.fill_(float("nan"))
        h = plan.P // 2
        plan.run_paths(0, h, A[:h], B[:h], rows=(r0, r1))
        plan.run_paths(h, plan.P, A[h:], B[h:], rows=(r0, r1))
        assert torch.equal(A[:, r0:r1], ref_A[:, r0:r1]), (r0, r1)
        assert torch.equal(B, ref_B), (r0, r1)


def test_q30_first_million_amplitudes_rows_only():
    """The first 10^6 amplitudes of q30-1 from side a's first 31 rows only
    (hsf_run_paths_rows) and the row-panel path sum, against the oracle."""
    g = np.load(os.path.join(GOLDEN, "qaoa_q30.npz"))
    plan = Plan(joint_blocked(cg.qaoa_sbm(100, (15, 15), 0.8, 0.1)))
    rows = (10 ** 6 + (1 << plan.nb) - 1) >> plan.nb
    A, B = plan.run_paths(rows=(0, rows))
    first = plan.amplitudes_full(A, B, rows=(0, rows), mode="bf16x3").reshape(-1)
    xs = torch.from_numpy(np.asarray(g["x"], dtype=np.uint64).astype(np.int64)).cuda()
    assert ohsf.rel_l2(first[xs].cpu().numpy(), g["psi"]) < 1e-5
