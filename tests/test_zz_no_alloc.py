"""hsf_amplitudes_full_noalloc (the path sum with its scratch in the
library's static device array) against hsf_amplitudes_full with a caller
workspace: the same kernels on the same planes, so the outputs must be
equal bit for bit, and within the c64 bar (rel-L2 <= 1e-5) of the exact
product.  Two calls in a row, the second on a smaller input, so the second
runs on the scratch the first one left behind."""
import ctypes

import numpy as np
import pytest
import torch

import circuitgen as cg
from oracle import hsf as ohsf
from paper_2502_06959_amd import HsfError, Plan, hsf_amplitudes_full_noalloc
from paper_2502_06959_amd import _lib as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _shape_plan(na, nb):
    # a gate-free circuit: only its dimensions matter to the path sum
    return Plan(cg.circuit("dims", na + nb, [], nb - 1, []), dtype="c64")


def _rand(rng, k, d):
    x = (rng.standard_normal((k, d)) + 1j * rng.standard_normal((k, d))) / np.sqrt(2 * d * max(k, 1) ** 0.5)
    return x.astype(np.complex64)


def _one(na, nb, K, rows, seed, accumulate=False):
    rng = np.random.default_rng(seed)
    A, B = _rand(rng, K, 1 << na), _rand(rng, K, 1 << nb)
    plan = _shape_plan(na, nb)
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    r0, r1 = rows
    base = (torch.from_numpy(_rand(rng, r1 - r0, 1 << nb)).cuda() if accumulate
            else torch.zeros((r1 - r0, 1 << nb), dtype=torch.complex64, device="cuda"))
    got = base.clone()
    hsf_amplitudes_full_noalloc(plan.handle, Ad, Bd, K, r0, r1, got, mode="bf16x3", accumulate=accumulate)
    want = base.clone()
    plan.amplitudes_full(Ad, Bd, rows=(r0, r1), mode="bf16x3", out=want, accumulate=accumulate)
    torch.cuda.synchronize()
    assert torch.equal(got, want), (na, nb, K, rows)
    ref = A.astype(np.complex128).T[r0:r1] @ B.astype(np.complex128)
    if accumulate:
        ref = ref + base.cpu().numpy().astype(np.complex128)
    assert ohsf.rel_l2(got.cpu().numpy(), ref) < 1e-5


@pytest.mark.parametrize("first,second", [
    # LDS-staged kernel (K >= 64), then a smaller streaming one (K < 64)
    ((10, 9, 300, (0, 1024)), (7, 8, 40, (3, 100))),
    # streaming, then a smaller LDS-staged product over a ragged row range
    ((12, 11, 48, (0, 4096)), (8, 9, 70, (17, 200))),
])
def test_noalloc_matches_workspace_call_twice(first, second):
    _one(*first, seed=11)
    _one(*second, seed=12)


def test_noalloc_accumulates_like_workspace_call():
    _one(9, 9, 130, (0, 512), seed=13, accumulate=True)
    _one(9, 9, 20, (5, 300), seed=14, accumulate=True)


def test_noalloc_rejects_planes_beyond_its_scratch():
    """Planes larger than HSF_NOALLOC_SCRATCH_BYTES fail before any launch
    and leave the output untouched."""
    na, nb = 13, 13
    plan = _shape_plan(na, nb)
    K = 1024          # 1024 x 2^14 values x 8 B = 128 MiB of planes > 64 MiB
    A = torch.zeros((K, 1 << na), dtype=torch.complex64, device="cuda")
    B = torch.zeros((K, 1 << nb), dtype=torch.complex64, device="cuda")
    out = torch.full((4, 1 << nb), 3.0 + 0j, dtype=torch.complex64, device="cuda")
    with pytest.raises(HsfError) as e:
        hsf_amplitudes_full_noalloc(plan.handle, A, B, K, 0, 4, out, mode="bf16x3")
    assert e.value.code == "HSF_E_ARG" and "scratch" in str(e.value)
    with pytest.raises(HsfError):
        hsf_amplitudes_full_noalloc(plan.handle, A, B, K, 0, 4, out, mode="bf16x3_split")
    torch.cuda.synchronize()
    assert bool((out == 3.0).all())
    assert int(L.lib().hsf_amplitudes_full_noalloc(None, None, 0, None, 0, 0, 0, 0, None, 0, 1, 0,
                                                   ctypes.c_void_p(0))) != 0
