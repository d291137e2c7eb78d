"""Full-size GPU parity: the C2 (literal, P=1024), C3, C4 (P=4096) and C5
(64 circuits) workloads at their real sizes, through the same launches the benchmark
times, against values the FP64 oracle wrote (tests/golden/make_golden.py,
which calls only oracle/).

Amplitudes: rel-L2 <= 1e-5 over the sampled basis states (complex64 bar).
C4 computes every one of its 2^34 amplitudes in row tiles, so the norm of
the whole output (a property that holds at any size: the state is unit norm)
covers the rows that no golden sample hits.  C3 gradients: max |g - g_ref|
<= 1e-4 max |g_ref| on all 708 angles (the oracle's adjoint) and on the 16
shift-rule samples."""
import os

import numpy as np
import pytest
import torch

import circuitgen as cg
from oracle import hsf as ohsf
from paper_2502_06959_amd import Batch, Plan, hsf_norm2

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
C64_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.empty_cache()


def _golden(name):
    z = np.load(os.path.join(GOLDEN, name))
    return {k: z[k] for k in z.files}


def _x(xs):
    return torch.from_numpy(np.asarray(xs, dtype=np.uint64).astype(np.int64)).cuda()


def test_c2_literal_bitstrings_and_full_output():
    g = _golden("c2_literal.npz")
    plan = Plan(cg.c2(), dtype="c64")
    assert plan.P == 1024
    A, B = plan.run_paths()
    amp = plan.amplitudes_bitstrings(A, B, _x(g["x"])).cpu().numpy()
    assert ohsf.rel_l2(amp, g["psi"]) < C64_TOL
    for mode in ("f32", "bf16x3"):
        out = plan.amplitudes_full(A, B, mode=mode)
        nrm = hsf_norm2(out.reshape(-1)).cpu().numpy()[0]
        got = out.reshape(-1)[_x(g["x"])].cpu().numpy()
        del out
        assert ohsf.rel_l2(got, g["psi"]) < C64_TOL, mode
        assert abs(nrm - 1.0) < 1e-5, mode


def test_c3_amplitudes_loss_and_gradients():
    g = _golden("c3.npz")
    c = cg.c3()
    plan = Plan(c, dtype="c64")
    assert plan.P == 256 and plan.n_params == 708
    x = _x(g["x"])
    A, B = plan.run_paths()
    amp = plan.amplitudes_bitstrings(A, B, x).cpu().numpy()
    del A, B
    assert ohsf.rel_l2(amp, g["psi"]) < C64_TOL
    L = plan.loss(x)
    assert abs(L - float(g["loss"])) < 1e-5 * float(g["loss"])
    grad = plan.backward(x).cpu().numpy()
    ref = g["grad"]
    got = grad[g["grad_ids"]]
    assert np.max(np.abs(got - ref)) <= 1e-4 * np.max(np.abs(ref)), (got, ref)
    # all 708 angles against the oracle's adjoint gradient
    full = _golden("c3_grad.npz")["grad"]
    err = np.abs(grad - full)
    assert np.max(err) <= 1e-4 * np.max(np.abs(full)), (int(np.argmax(err)), float(np.max(err)))


def test_c4_all_row_tiles_sampled_and_norm():
    """Every output row tile in split-BF16 x3 (the chosen form), samples
    checked, the norm summed over all tiles; then FP32 and FP64 on a 64-row
    block of every tile against the same samples."""
    g = _golden("c4.npz")
    plan = Plan(cg.c4(), dtype="c64")
    assert plan.P == 4096 and plan.na == 17 and plan.nb == 17
    A, B = plan.run_paths()
    xs = np.asarray(g["x"], dtype=np.uint64)
    ref = g["psi"]
    amp = plan.amplitudes_bitstrings(A, B, _x(xs)).cpu().numpy()
    assert ohsf.rel_l2(amp, ref) < C64_TOL
    rows = 1 << 13
    tile = torch.empty((rows, 1 << plan.nb), dtype=torch.complex64, device="cuda")
    row_of = (xs >> np.uint64(plan.nb)).astype(np.int64)
    col_of = (xs & np.uint64((1 << plan.nb) - 1)).astype(np.int64)
    got = np.zeros(len(xs), dtype=np.complex128)
    total = 0.0
    for r0 in range(0, 1 << plan.na, rows):
        plan.amplitudes_full(A, B, rows=(r0, r0 + rows), mode="bf16x3", out=tile)
        total += float(hsf_norm2(tile.reshape(-1)).cpu().numpy()[0])
        sel = np.nonzero((row_of >= r0) & (row_of < r0 + rows))[0]
        if len(sel):
            idx = torch.from_numpy((row_of[sel] - r0) * (1 << plan.nb) + col_of[sel]).cuda()
            got[sel] = tile.reshape(-1)[idx].cpu().numpy()
    assert ohsf.rel_l2(got, ref) < C64_TOL
    assert abs(total - 1.0) < 1e-5
    del tile
    # FP32 and FP64 path sums on every row tile: in each tile the 64-row
    # block holding the most samples (the same LDS-staged kernels the full
    # tiles run, on a ragged 64-row product)
    for mode in ("f32", "f64"):
        got = []
        refs = []
        for r0 in range(0, 1 << plan.na, rows):
            in_tile = (row_of >= r0) & (row_of < r0 + rows)
            blocks = np.bincount((row_of[in_tile] - r0) // 64, minlength=rows // 64)
            b0 = r0 + int(np.argmax(blocks)) * 64
            sel = np.nonzero((row_of >= b0) & (row_of < b0 + 64))[0]
            assert len(sel) >= 2, (mode, r0)
            out = plan.amplitudes_full(A, B, rows=(b0, b0 + 64), mode=mode)
            idx = torch.from_numpy((row_of[sel] - b0) * (1 << plan.nb) + col_of[sel]).cuda()
            got.append(out.reshape(-1)[idx].cpu().numpy())
            refs.append(ref[sel])
            del out
        # the FP64 path sum still sums complex64 half-states, so the sweeps'
        # FP32 rounding (about 1e-6 here) remains in every mode
        assert ohsf.rel_l2(np.concatenate(got), np.concatenate(refs)) < C64_TOL, mode


def _c5_row_weights(i, nb):
    # the projection weights tests/golden/make_golden.py drew for circuit i
    rng = np.random.default_rng(6000 + i)
    return rng.standard_normal((8, 1 << nb)) + 1j * rng.standard_normal((8, 1 << nb))


def test_c5_whole_batch_tuned_and_replayed():
    """All 64 circuits in one tuned batch replayed from a HIP graph (73.7 GiB
    of output): 64 oracle samples and the norm of every circuit's state, and
    four whole output rows of every circuit (row 0, the last row, two seeded)
    through their norms and 8 random projections against the oracle's."""
    g = _golden("c5.npz")
    gr = _golden("c5_rows.npz")
    plans = [Plan(c) for c in cg.c5()]
    b = Batch(plans)
    outs = b.alloc_outputs()
    b.tune(outs, mode="bf16x3")
    for o in outs:
        o.zero_()
    b.run(outs, mode="bf16x3", graph=True)
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        sel = g["circuit"] == i
        got = o.reshape(-1)[_x(g["x"][sel])].cpu().numpy()
        assert ohsf.rel_l2(got, g["psi"][sel]) < C64_TOL, i
        nrm = float(hsf_norm2(o.reshape(-1)).cpu().numpy()[0])
        assert abs(nrm - 1.0) < 1e-5, i
        rows = gr["rows"][i]
        whole = o[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.complex128)
        n2 = np.sum(np.abs(whole) ** 2, axis=1)
        assert np.max(np.abs(n2 - gr["norm2"][i]) / gr["norm2"][i]) < 1e-5, i
        proj = whole @ _c5_row_weights(i, plans[i].nb).T
        assert ohsf.rel_l2(proj, gr["proj"][i]) < C64_TOL, i
    del outs
