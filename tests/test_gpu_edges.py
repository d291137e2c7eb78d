"""GPU behaviour of empty and degenerate inputs, through the C ABI.

Empty calls: an empty path range writes nothing; a path sum over zero paths
is the empty sum (rows set to zero, or left as they are when accumulating)
in every arithmetic mode, and so are bitstring amplitudes; an empty row range, no bitstrings and a norm over
no entries write nothing or zeros; a gradient over no bitstrings, and the
gradient of a circuit without angles, are zero.

Degenerate plans, against the FP64 Schroedinger oracle: a circuit with no
crossing gate (one path, no blocks) and one whose only crossing gate is a
product of one-qubit gates (operator-Schmidt rank 1: one path through a
block).  Bars as elsewhere: complex64 rel-L2 <= 1e-5, complex128 <= 1e-10."""
import numpy as np
import pytest
import torch

import circuitgen as cg
from oracle import hsf as ohsf
from oracle import sv
from paper_2502_06959_amd import Plan, hsf_norm2

pytestmark = pytest.mark.gpu

C64_TOL = 1e-5
C128_TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.empty_cache()


def _filled(shape, dtype, value):
    t = torch.empty(shape, dtype=dtype, device="cuda")
    t.fill_(value)
    return t


def test_empty_path_range_writes_nothing():
    plan = Plan(cg.c1b(), dtype="c64")
    A, B = plan.alloc_halves(4)
    A.fill_(7 + 1j)
    B.fill_(-3 + 2j)
    print("[edges] run_paths(2, 2) on c1b", flush=True)
    plan.run_paths(2, 2, A, B)
    torch.cuda.synchronize()
    assert bool((A == (7 + 1j)).all()) and bool((B == (-3 + 2j)).all())


@pytest.mark.parametrize("dtype,mode", [("c64", "f32"), ("c64", "bf16x3"), ("c64", "f64"),
                                        ("c128", "c128"), ("c128", "f64")])
def test_zero_paths_is_the_empty_sum(dtype, mode):
    plan = Plan(cg.c1b(), dtype=dtype)
    A, B = plan.run_paths()
    odt = torch.complex64 if mode in ("f32", "bf16x3") else torch.complex128
    out = _filled((1 << plan.na, 1 << plan.nb), odt, complex(float("nan"), float("nan")))
    print(f"[edges] zero-path sum {dtype} {mode}", flush=True)
    plan.amplitudes_full(A[:0], B[:0], mode=mode, out=out)
    torch.cuda.synchronize()
    assert bool((out == 0).all())
    out.fill_(1 + 2j)
    plan.amplitudes_full(A[:0], B[:0], mode=mode, out=out, accumulate=True)
    torch.cuda.synchronize()
    assert bool((out == (1 + 2j)).all())


def test_empty_rows_bitstrings_and_norm():
    plan = Plan(cg.c1b(), dtype="c128")
    A, B = plan.run_paths()
    out = _filled((4, 1 << plan.nb), torch.complex128, 5 + 5j)
    print("[edges] empty row range, no bitstrings, empty norm", flush=True)
    plan.amplitudes_full(A, B, rows=(9, 9), mode="c128", out=out)
    # the binding's own output for an empty range has no rows (a null buffer)
    e = plan.amplitudes_full(A, B, rows=(9, 9), mode="c128")
    x = torch.zeros(0, dtype=torch.int64, device="cuda")
    amp = plan.amplitudes_bitstrings(A, B, x)
    # bitstrings summed over no paths: zeros
    x3 = torch.tensor([0, 1, 4000], dtype=torch.int64, device="cuda")
    amp0 = plan.amplitudes_bitstrings(A[:0], B[:0], x3, out=_filled((3,), torch.complex128, complex(1, 1)))
    s = hsf_norm2(torch.zeros(0, dtype=torch.complex64, device="cuda"))
    torch.cuda.synchronize()
    assert bool((out == (5 + 5j)).all())
    assert tuple(e.shape) == (0, 1 << plan.nb)
    assert amp.numel() == 0
    assert bool((amp0 == 0).all())
    assert s.cpu().tolist() == [0.0, 0.0]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_gradient_over_no_bitstrings_is_zero(dtype):
    plan = Plan(cg.c3(seed=3, n=10, layers=4), dtype=dtype)
    assert plan.n_params > 0
    g = _filled((plan.n_params,), torch.float64, 5.0)
    x = torch.zeros(0, dtype=torch.int64, device="cuda")
    print(f"[edges] gradient over no bitstrings {dtype}", flush=True)
    plan.backward(x, grad=g)
    torch.cuda.synchronize()
    assert bool((g == 0).all())


def _side_gates(rng, n):
    gs = [cg.gate("U", (q,), matrix=cg.haar_unitary(rng)) for q in range(n)]
    # two-qubit gates inside each side (cut 3: side b = qubits 0..3, side a = 4..7)
    gs += [cg.gate("CZ", (0, 1)), cg.gate("CX", (2, 3)), cg.gate("ISWAP", (5, 7)), cg.gate("SWAP", (4, 6))]
    gs += [cg.gate("U", (q,), matrix=cg.haar_unitary(rng)) for q in range(n)]
    return gs


def _no_crossing():
    rng = np.random.default_rng(11)
    return cg.circuit("no_crossing", 8, _side_gates(rng, 8), 3, [])


def _product_crossing():
    rng = np.random.default_rng(12)
    gs = _side_gates(rng, 8)
    blk = len(gs)
    # a crossing two-qubit gate that is a Kronecker product: Schmidt rank 1
    gs.append(cg.gate("U", (6, 1), matrix=np.kron(cg.haar_unitary(rng), cg.haar_unitary(rng))))
    gs += [cg.gate("CZ", (1, 2)), cg.gate("CX", (6, 5))]
    return cg.circuit("product_crossing", 8, gs, 3, [[blk]])


@pytest.mark.parametrize("make", [_no_crossing, _product_crossing], ids=["no-crossing", "product-crossing"])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_single_path_plans(make, dtype):
    c = make()
    plan = Plan(c, dtype=dtype)
    assert plan.P == 1 and plan.n_params == 0
    tol = C128_TOL if dtype == "c128" else C64_TOL
    ref = sv.run(c)
    print(f"[edges] {c['name']} {dtype}", flush=True)
    A, B = plan.run_paths()
    modes = ["c128", "f64"] if dtype == "c128" else ["f32", "bf16x3", "f64"]
    for mode in modes:
        out = plan.amplitudes_full(A, B, mode=mode)
        torch.cuda.synchronize()
        assert ohsf.rel_l2(out.cpu().numpy().reshape(-1), ref) < tol, mode
    xs = np.array([0, 5, 77, 200, 255], dtype=np.int64)
    amp = plan.amplitudes_bitstrings(A, B, torch.from_numpy(xs).cuda())
    # no angles: the gradient call succeeds and returns no entries
    g = plan.backward(torch.from_numpy(xs).cuda())
    torch.cuda.synchronize()
    assert ohsf.rel_l2(amp.cpu().numpy(), ref[xs]) < tol
    assert g.numel() == 0
