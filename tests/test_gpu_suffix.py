"""Deferred side-b suffix (hsf_plan_options.defer_b_suffix,
hsf_apply_b_suffix): side b's gates after its last factor slot leave the
half-states and act once on each output row after the sum over paths (the
path sum is linear in side b's state, Sec. II-B).

  - full states against the FP64 Schroedinger oracle (QAOA cascades, dense
    brickwork blocks; c64 and c128; FP32 and split-BF16 x3 path sums);
  - a row range summed over path chunks with accumulate, then the suffix:
    equal to the same rows of the plan without deferral;
  - the first 10^6 amplitudes of Table II's q30-1 shape against the stored
    oracle samples;
  - the entry points that cannot take such a plan reject it."""
import ctypes
import os

import numpy as np
import pytest
import torch

import circuitgen as cg
from oracle import hsf as ohsf
from oracle import sv
from paper_2502_06959_amd import HsfError, Plan, joint_blocked
from paper_2502_06959_amd import _lib as L

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.empty_cache()


# QAOA cascades (the mixer on side b is the suffix), SVD-factored dense
# brickwork blocks (C1b: Haar gates after the last block) and random
# circuits with dense two-qubit blocks
CASES = [
    ("qaoa", lambda: joint_blocked(cg.qaoa_sbm(31, (6, 6), 0.8, 0.3))),
    ("qaoa", lambda: joint_blocked(cg.qaoa_sbm(33, (9, 8), 0.7, 0.2))),
    ("dense", lambda: cg.c1b()),
    ("dense", lambda: cg.random_circuit(40, n=9, n_gates=40, group=2, p2=0.4)),
    ("dense", lambda: cg.random_circuit(43, n=9, n_gates=40, group=2, p2=0.4)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_deferred_suffix_full_state(case, dtype):
    kind, make = CASES[case]
    c = make()
    plan = Plan(c, dtype=dtype, defer_b_suffix=True)
    base = Plan(c, dtype=dtype)
    # some of side b's gates are deferred
    assert plan.side_stats(1)["ops_logical"] < base.side_stats(1)["ops_logical"]
    ref = sv.run(c)
    A, B = plan.run_paths()
    modes = ["c128"] if dtype == "c128" else ["f32", "bf16x3"]
    for mode in modes:
        out = plan.amplitudes_full(A, B, mode=mode)
        plan.apply_b_suffix(out)
        tol = 1e-12 if dtype == "c128" else 1e-5
        assert ohsf.rel_l2(out.cpu().numpy().reshape(-1), ref) < tol, mode


@pytest.mark.parametrize("tree", ["on", "off"])
def test_deferred_suffix_rows_over_path_chunks(tree):
    c = joint_blocked(cg.qaoa_sbm(41, (13, 12), 0.8, 0.15))
    plan = Plan(c, tree=tree, defer_b_suffix=True)
    base = Plan(c, tree=tree)
    r0, r1 = 3, 40
    A0, B0 = base.run_paths()
    want = base.amplitudes_full(A0, B0, rows=(r0, r1))
    out = torch.empty_like(want)
    chunk = max(1, plan.P // 3)
    A, B = plan.alloc_halves(chunk)
    for p0 in range(0, plan.P, chunk):
        n = min(chunk, plan.P - p0)
        plan.run_paths(p0, p0 + n, A[:n], B[:n], rows=(r0, r1))
        plan.amplitudes_full(A[:n], B[:n], n_paths=n, rows=(r0, r1), out=out, accumulate=p0 > 0)
    plan.apply_b_suffix(out)
    assert ohsf.rel_l2(out.cpu().numpy(), want.cpu().numpy()) < 2e-6
    # a strided output: rows of a wider buffer
    wide = torch.zeros((r1 - r0, (1 << plan.nb) + 64), dtype=torch.complex64, device="cuda")
    view = wide[:, : 1 << plan.nb]
    Af, Bf = plan.run_paths()
    plan.amplitudes_full(Af, Bf, rows=(r0, r1), out=view)
    plan.apply_b_suffix(view)
    assert ohsf.rel_l2(view.cpu().numpy(), want.cpu().numpy()) < 2e-6
    assert bool((wide[:, 1 << plan.nb:] == 0).all())


def test_deferred_suffix_q30_first_million_amplitudes():
    g = np.load(os.path.join(GOLDEN, "qaoa_q30.npz"))
    plan = Plan(joint_blocked(cg.qaoa_sbm(100, (15, 15), 0.8, 0.1)), defer_b_suffix=True)
    rows = (10 ** 6 + (1 << plan.nb) - 1) >> plan.nb
    A, B = plan.run_paths(rows=(0, rows))
    first = plan.amplitudes_full(A, B, rows=(0, rows), mode="bf16x3")
    plan.apply_b_suffix(first)
    xs = torch.from_numpy(np.asarray(g["x"], dtype=np.uint64).astype(np.int64)).cuda()
    assert ohsf.rel_l2(first.reshape(-1)[xs].cpu().numpy(), g["psi"]) < 1e-5


def test_deferred_suffix_rejections_and_no_op():
    from paper_2502_06959_amd.hsf import Batch
    c = joint_blocked(cg.qaoa_sbm(31, (6, 6), 0.8, 0.3))
    plan = Plan(c, defer_b_suffix=True)
    A, B = plan.run_paths()
    xs = torch.arange(8, dtype=torch.int64, device="cuda")
    with pytest.raises(HsfError) as e:
        plan.amplitudes_bitstrings(A, B, xs)
    assert e.value.code == "HSF_E_UNSUPPORTED"
    with pytest.raises(HsfError) as e:
        plan.loss(xs)
    assert e.value.code == "HSF_E_UNSUPPORTED"
    with pytest.raises(HsfError) as e:
        Batch([plan])
    assert e.value.code == "HSF_E_UNSUPPORTED"
    out = plan.amplitudes_full(A, B)
    with pytest.raises(ValueError):
        plan.apply_b_suffix(out.to(torch.complex128))
    # a plan without deferral: the call leaves the rows alone
    base = Plan(c)
    before = out.clone()
    base.apply_b_suffix(out)
    torch.cuda.synchronize()
    assert torch.equal(out, before)
    lib = L.lib()
    assert lib.hsf_apply_b_suffix(ctypes.c_void_p(plan.handle), None, 1 << plan.nb, 1, None) != 0
    assert lib.hsf_apply_b_suffix(ctypes.c_void_p(plan.handle), ctypes.c_void_p(out.data_ptr()), 3, 1, None) != 0
