"""GPU parity of the path sum (Sec. II-B reconstruction, C = PsiA^T PsiB) in
every arithmetic mode, on random half-states with ragged shapes, against the
exact product in FP64 on the host (numpy).  Tolerances: FP32 and split-BF16
x3 rel-L2 <= 1e-5 (the c64 amplitude bar), FP64 <= 1e-12."""
import numpy as np
import pytest
import torch

import circuitgen as cg
from oracle import hsf as ohsf
from paper_2502_06959_amd import Plan, hsf_norm2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _shape_plan(na, nb, dtype="c64"):
    # a gate-free circuit: only its dimensions matter to the path sum
    return Plan(cg.circuit("dims", na + nb, [], nb - 1, []), dtype=dtype)


def _rand(rng, k, d, dtype):
    x = (rng.standard_normal((k, d)) + 1j * rng.standard_normal((k, d))) / np.sqrt(2 * d * max(k, 1) ** 0.5)
    return x.astype(dtype)


# K >= 64 takes the LDS-staged kernels: several tiles, ragged path chunks
# (K mod 16, K mod 32 != 0) and tiles cut by M or N < 128
CASES = [(1, 1, 1), (5, 3, 2), (6, 6, 3), (7, 8, 17), (9, 7, 33), (8, 8, 64), (10, 6, 100), (6, 10, 257),
         (12, 12, 32), (3, 11, 7), (7, 7, 128), (9, 8, 300), (5, 10, 1000), (10, 4, 161), (8, 9, 4096)]


@pytest.mark.parametrize("na,nb,K", CASES)
@pytest.mark.parametrize("mode", ["f32", "bf16x3", "f64"])
def test_path_sum_modes(na, nb, K, mode):
    rng = np.random.default_rng(na * 1000 + nb * 10 + K)
    A = _rand(rng, K, 1 << na, np.complex64)
    B = _rand(rng, K, 1 << nb, np.complex64)
    ref = A.astype(np.complex128).T @ B.astype(np.complex128)
    plan = _shape_plan(na, nb)
    out = plan.amplitudes_full(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), n_paths=K, mode=mode)
    torch.cuda.synchronize()
    tol = 1e-12 if mode == "f64" else 1e-5
    assert ohsf.rel_l2(out.cpu().numpy(), ref) < tol


@pytest.mark.parametrize("mode", ["f32", "bf16x3", "f64"])
def test_path_sum_row_range_ld_and_accumulate(mode):
    rng = np.random.default_rng(3)
    na, nb, K = 9, 8, 40
    A = _rand(rng, K, 1 << na, np.complex64)
    B = _rand(rng, K, 1 << nb, np.complex64)
    ref = A.astype(np.complex128).T @ B.astype(np.complex128)
    plan = _shape_plan(na, nb)
    # padded leading dimensions
    Ad = torch.zeros((K, (1 << na) + 24), dtype=torch.complex64, device="cuda")
    Bd = torch.zeros((K, (1 << nb) + 8), dtype=torch.complex64, device="cuda")
    Ad[:, :1 << na] = torch.from_numpy(A).cuda()
    Bd[:, :1 << nb] = torch.from_numpy(B).cuda()
    odt = torch.complex128 if mode == "f64" else torch.complex64
    out = torch.zeros((300, (1 << nb) + 16), dtype=odt, device="cuda")
    h = K // 2
    plan.amplitudes_full(Ad[:h], Bd[:h], n_paths=h, rows=(100, 400), mode=mode, out=out)
    plan.amplitudes_full(Ad[h:], Bd[h:], n_paths=K - h, rows=(100, 400), mode=mode, out=out, accumulate=True)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert ohsf.rel_l2(got[:, :1 << nb], ref[100:400]) < (1e-12 if mode == "f64" else 1e-5)
    assert np.all(got[:, 1 << nb:] == 0)          # padding columns untouched


@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
def test_many_paths_row_ranges(mode):
    """LDS-staged path sums on row ranges that cut tiles (M = 322, even, and
    M = 333, odd: FP32 then falls back to the streaming kernel), with
    accumulation over two path chunks."""
    rng = np.random.default_rng(11)
    na, nb, K = 10, 9, 400
    A = _rand(rng, K, 1 << na, np.complex64)
    B = _rand(rng, K, 1 << nb, np.complex64)
    ref = A.astype(np.complex128).T @ B.astype(np.complex128)
    plan = _shape_plan(na, nb)
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    for r0, r1 in ((64, 386), (101, 434)):
        out = plan.amplitudes_full(Ad[:250], Bd[:250], n_paths=250, rows=(r0, r1), mode=mode)
        plan.amplitudes_full(Ad[250:], Bd[250:], n_paths=K - 250, rows=(r0, r1), mode=mode, out=out,
                             accumulate=True)
        assert ohsf.rel_l2(out.cpu().numpy(), ref[r0:r1]) < 1e-5, (r0, r1)


def test_lds_and_streaming_fp32_sums_agree_bitwise():
    """The LDS-staged FP32 kernel runs the streaming kernel's MFMA sequence:
    rows 0..M-1 (even M, staged) equal rows 0..M-2 (odd M, streamed) bit for bit."""
    rng = np.random.default_rng(12)
    na, nb, K = 9, 8, 333
    A = torch.from_numpy(_rand(rng, K, 1 << na, np.complex64)).cuda()
    B = torch.from_numpy(_rand(rng, K, 1 << nb, np.complex64)).cuda()
    plan = _shape_plan(na, nb)
    staged = plan.amplitudes_full(A, B, mode="f32")
    streamed = plan.amplitudes_full(A, B, mode="f32", rows=(0, (1 << na) - 1))
    assert torch.equal(staged[:-1], streamed)


@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
@pytest.mark.parametrize("K", [40, 200])
def test_odd_leading_dimension_output(mode, K):
    """An output whose leading dimension is odd cannot take the 16-byte paired
    stores; the per-lane stores must give the same values (streaming and
    LDS-staged kernels)."""
    rng = np.random.default_rng(13)
    na, nb = 9, 8
    A = _rand(rng, K, 1 << na, np.complex64)
    B = _rand(rng, K, 1 << nb, np.complex64)
    ref = A.astype(np.complex128).T @ B.astype(np.complex128)
    plan = _shape_plan(na, nb)
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    odd = torch.zeros((1 << na, (1 << nb) + 1), dtype=torch.complex64, device="cuda")
    plan.amplitudes_full(Ad, Bd, mode=mode, out=odd)
    even = plan.amplitudes_full(Ad, Bd, mode=mode)
    got = odd.cpu().numpy()
    assert ohsf.rel_l2(got[:, :1 << nb], ref) < 1e-5
    assert np.all(got[:, 1 << nb:] == 0)
    assert np.array_equal(got[:, :1 << nb], even.cpu().numpy())


def test_bf16x3_on_c2p_matches_fp64_mode():
    """The chosen form on the benchmarked workload: split-BF16 x3 against the
    FP64 path sum of the same half-states, over all 2^28 amplitudes."""
    c = cg.c2p()
    plan = Plan(c)
    A, B = plan.run_paths()
    rows = (0, 1 << 12)
    o16 = plan.amplitudes_full(A, B, mode="bf16x3", rows=rows)
    o64 = plan.amplitudes_full(A, B, mode="f64", rows=rows)
    s = hsf_norm2(o16.reshape(-1), o64.reshape(-1)).cpu().numpy()
    ref = hsf_norm2(o64.reshape(-1)).cpu().numpy()
    assert np.sqrt(s[1] / ref[0]) < 1e-5
    full = plan.amplitudes_full(A, B, mode="bf16x3")
    nrm = hsf_norm2(full.reshape(-1)).cpu().numpy()[0]
    assert abs(nrm - 1) < 1e-5


@pytest.mark.parametrize("na,nb,K", [(9, 8, 40), (10, 9, 400), (8, 10, 17), (11, 7, 4096)])
def test_presplit_row_tiles_equal_per_call_split(na, nb, K):
    """hsf_split_operands once, then HSF_SUM_BF16X3_SPLIT on row tiles (some
    cut by the tile size, the last one ragged): bit for bit the per-call
    split-BF16 x3 sums of the same rows (the planes and the MFMA sequence are
    the same), and within the c64 bar of the exact product.  Streaming
    (K < 64) and LDS-staged (K >= 64) layouts."""
    rng = np.random.default_rng(na * 100 + nb + K)
    A = _rand(rng, K, 1 << na, np.complex64)
    B = _rand(rng, K, 1 << nb, np.complex64)
    ref = A.astype(np.complex128).T @ B.astype(np.complex128)
    plan = _shape_plan(na, nb)
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ws = plan.split_operands(Ad, Bd)
    M = 1 << na
    cuts = sorted({0, 64, 200, M // 2 + 3, M})
    full = torch.zeros((M, 1 << nb), dtype=torch.complex64, device="cuda")
    for r0, r1 in zip(cuts[:-1], cuts[1:]):
        plan.amplitudes_full(Ad, Bd, rows=(r0, r1), mode="bf16x3_split", out=full[r0:r1], ws=ws)
        one = plan.amplitudes_full(Ad, Bd, rows=(r0, r1), mode="bf16x3")
        assert torch.equal(full[r0:r1], one), (r0, r1)
    assert ohsf.rel_l2(full.cpu().numpy(), ref) < 1e-5


def test_presplit_needs_the_split_workspace_and_path_count():
    """HSF_SUM_BF16X3_SPLIT with another workspace or path count than the
    plan's last split is rejected before any launch."""
    from paper_2502_06959_amd import HsfError
    rng = np.random.default_rng(5)
    na, nb, K = 8, 8, 70
    plan = _shape_plan(na, nb)
    Ad = torch.from_numpy(_rand(rng, K, 1 << na, np.complex64)).cuda()
    Bd = torch.from_numpy(_rand(rng, K, 1 << nb, np.complex64)).cuda()
    ws = plan.split_operands(Ad, Bd)
    other = torch.empty_like(ws)
    out = torch.zeros((1 << na, 1 << nb), dtype=torch.complex64, device="cuda")
    with pytest.raises(HsfError) as e:
        plan.amplitudes_full(Ad, Bd, mode="bf16x3_split", out=out, ws=other)
    assert e.value.code == "HSF_E_ARG"
    with pytest.raises(HsfError) as e:
        plan.amplitudes_full(Ad[:K - 1], Bd[:K - 1], n_paths=K - 1, mode="bf16x3_split", out=out, ws=ws)
    assert e.value.code == "HSF_E_ARG"
    assert torch.count_nonzero(out).item() == 0


@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
@pytest.mark.parametrize("rows,K,nb", [((0, 1), 1, 5), ((3, 10), 17, 7), ((0, 16), 33, 9), ((100, 131), 100, 8),
                                       ((64, 96), 1000, 11), ((5, 37), 2, 4), ((0, 32), 4099, 10)])
def test_row_panels(mode, rows, K, nb):
    """Row ranges of at most 32 rows take the FP32 row-panel kernel in both
    modes (prefetch ring deeper than K for small K, ragged K and N, a
    column count below one workgroup's 128), with accumulation over two path
    chunks and an odd output leading dimension."""
    na = 9
    rng = np.random.default_rng(rows[0] * 7 + K + nb)
    A = _rand(rng, K, 1 << na, np.complex64)
    B = _rand(rng, K, 1 << nb, np.complex64)
    ref = A.astype(np.complex128).T @ B.astype(np.complex128)
    plan = _shape_plan(na, nb)
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    r0, r1 = rows
    out = torch.full((r1 - r0, (1 << nb) + 1), 7.0, dtype=torch.complex64, device="cuda")
    h = K // 2
    if h:
        plan.amplitudes_full(Ad[:h], Bd[:h], n_paths=h, rows=rows, mode=mode, out=out)
        plan.amplitudes_full(Ad[h:], Bd[h:], n_paths=K - h, rows=rows, mode=mode, out=out, accumulate=True)
    else:
        plan.amplitudes_full(Ad, Bd, n_paths=K, rows=rows, mode=mode, out=out)
    got = out.cpu().numpy()
    assert ohsf.rel_l2(got[:, :1 << nb], ref[r0:r1]) < 1e-5
    assert np.all(got[:, 1 << nb:] == 7.0)
