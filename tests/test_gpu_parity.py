"""GPU parity: libhsf's HIP path, called through the C ABI, against the FP64
oracle on the same seeded circuits.

Tolerances: complex128 paths rel-L2 <= 1e-10; complex64 paths rel-L2 <= 1e-5
(the accuracy bar for c64 amplitudes).  Integer tables are compared exactly.
Half-states are compared only with an oracle fed the library's own Schmidt
factors, since the factors are unique only up to a gauge.
"""
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
    torch.cuda.init()


def _rel(x, ref):
    return ohsf.rel_l2(np.asarray(x), np.asarray(ref))


def _full_state(plan, mode=None):
    A, B = plan.run_paths()
    out = plan.amplitudes_full(A, B, mode=mode)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(-1), A, B


def _lib_factors(plan, side):
    facs = []
    for k in range(plan.K):
        _, xa, yb = plan.block_factors(k)
        facs.append(xa if side == "A" else yb)
    return facs


@pytest.mark.parametrize("maker", [cg.c1, cg.c1b], ids=lambda f: f.__name__)
def test_c1_complex128_full_state(maker):
    c = maker()
    plan = Plan(c, dtype="c128")
    psi, _, _ = _full_state(plan, mode="c128")
    ref = sv.run(c)
    assert _rel(psi, ref) < C128_TOL


@pytest.mark.parametrize("maker", [cg.c1, cg.c1b], ids=lambda f: f.__name__)
def test_c1_complex64_full_state(maker):
    c = maker()
    plan = Plan(c, dtype="c64")
    psi, _, _ = _full_state(plan, mode="f32")
    assert _rel(psi, sv.run(c)) < C64_TOL
    psi64, _, _ = _full_state(plan, mode="f64")
    assert _rel(psi64, sv.run(c)) < C64_TOL


@pytest.mark.parametrize("maker,dtype", [(cg.c1b, "c128"), (cg.c1, "c64")], ids=["c1b-c128", "c1-c64"])
def test_half_states_with_shared_factors(maker, dtype):
    c = maker()
    plan = Plan(c, dtype=dtype)
    A, B = plan.run_paths()
    torch.cuda.synchronize()
    o = ohsf.plan(c)
    tol = C128_TOL if dtype == "c128" else C64_TOL
    for side, got in (("A", A), ("B", B)):
        ref = ohsf.half_states(c, o, side, factors=_lib_factors(plan, side))
        g = got.cpu().numpy()
        for p in range(plan.P):
            assert _rel(g[p], ref[p]) < tol, (side, p)


RANDOM_CASES = [
    # seed, n, cut, dtype, tile_qubits (8 forces several LDS passes on sides wider than 8 qubits)
    (100, 9, 3, "c128", 0), (100, 10, 6, "c64", 0), (100, 11, 4, "c64", 0), (100, 12, 5, "c128", 0),
    (100, 14, 3, "c64", 8), (100, 16, 5, "c64", 8), (100, 16, 9, "c128", 8), (100, 7, 0, "c64", 0),
    (103, 8, 6, "c64", 0), (100, 18, 8, "c64", 8), (100, 20, 9, "c128", 8),
]


@pytest.mark.parametrize("seed,n,cut,dtype,tq", RANDOM_CASES)
def test_random_circuits_against_schroedinger(seed, n, cut, dtype, tq):
    c = cg.random_circuit(seed, n=n, n_gates=4 * n, cut=cut, group=2, p2=0.3,
                          two_q_kinds=("CZ", "CX", "RZZ", "CP", "ISWAP", "SWAP"))
    plan = Plan(c, dtype=dtype, tile_qubits=tq)
    assert plan.P == ohsf.plan(c)["P"] and plan.P <= 1024
    psi, _, _ = _full_state(plan, mode="c128" if dtype == "c128" else "f32")
    tol = C128_TOL if dtype == "c128" else C64_TOL
    assert _rel(psi, sv.run(c)) < tol


def test_multi_pass_equals_single_pass():
    c = cg.random_circuit(100, n=20, n_gates=80, cut=9, group=2, p2=0.3,
                          two_q_kinds=("CZ", "CX", "RZZ", "CP", "ISWAP", "SWAP"))
    outs = []
    for tq in (0, 8, 9):
        plan = Plan(c, dtype="c128", tile_qubits=tq)
        st = plan.side_stats(0)
        # the shared prefix and the per-path rest are separate pass ranges;
        # a tile narrower than the side needs more than one pass per range
        ranges = 1 + (st["shared_passes"] > 0)
        assert (st["passes"] + st["shared_passes"] > ranges) == (tq > 0)
        A, B = plan.run_paths()
        outs.append((A.cpu().numpy(), B.cpu().numpy()))
    for A, B in outs[1:]:
        assert np.max(np.abs(A - outs[0][0])) < 1e-12
        assert np.max(np.abs(B - outs[0][1])) < 1e-12


def test_poisoned_outputs_are_overwritten():
    c = cg.c1()
    plan = Plan(c, dtype="c64")
    A, B = plan.alloc_halves(plan.P)
    A.fill_(float("nan"))
    B.fill_(float("nan"))
    plan.run_paths(0, plan.P, A, B)
    out = torch.full((1 << plan.na, 1 << plan.nb), float("nan"), dtype=torch.complex64, device="cuda")
    plan.amplitudes_full(A, B, out=out)
    torch.cuda.synchronize()
    assert torch.isfinite(torch.view_as_real(A)).all() and torch.isfinite(torch.view_as_real(B)).all()
    assert torch.isfinite(torch.view_as_real(out)).all()


def test_runs_are_bitwise_deterministic():
    c = cg.c1b()
    plan = Plan(c, dtype="c64")
    r1 = _full_state(plan)[0]
    r2 = _full_state(plan)[0]
    assert np.array_equal(r1, r2)


def test_path_chunks_accumulate():
    c = cg.c1b()
    plan = Plan(c, dtype="c64")
    A, B = plan.run_paths()
    one = plan.amplitudes_full(A, B)
    h = plan.P // 2
    acc = plan.amplitudes_full(A[:h], B[:h])
    plan.amplitudes_full(A[h:], B[h:], out=acc, accumulate=True)
    # chunk-wise half-states: paths [h, P) computed on their own equal the slice
    A2, B2 = plan.alloc_halves(plan.P - h)
    plan.run_paths(h, plan.P, A2, B2)
    torch.cuda.synchronize()
    assert torch.equal(A2, A[h:]) and torch.equal(B2, B[h:])
    assert _rel(acc.cpu().numpy(), one.cpu().numpy()) < 1e-6


def test_row_ranges_and_bitstrings():
    c = cg.c1b()
    plan = Plan(c, dtype="c128")
    A, B = plan.run_paths()
    ref = sv.run(c).reshape(1 << plan.na, 1 << plan.nb)
    part = plan.amplitudes_full(A, B, rows=(5, 37), mode="c128")
    torch.cuda.synchronize()
    assert _rel(part.cpu().numpy(), ref[5:37]) < C128_TOL
    xs = np.array([0, 1, 4095, 77, 2048, 1234, 3000], dtype=np.uint64)
    x = torch.from_numpy(xs.astype(np.int64)).to("cuda")
    amp = plan.amplitudes_bitstrings(A, B, x)
    torch.cuda.synchronize()
    assert _rel(amp.cpu().numpy(), ref.reshape(-1)[xs.astype(np.int64)]) < C128_TOL


def test_norm_and_difference():
    c = cg.c1b()
    plan = Plan(c, dtype="c64")
    psi, A, B = _full_state(plan)
    out = plan.amplitudes_full(A, B)
    ref = torch.from_numpy(sv.run(c)).to("cuda")
    s = hsf_norm2(out.reshape(-1), ref).cpu().numpy()
    assert abs(s[0] - 1) < 1e-5
    assert np.sqrt(s[1]) < C64_TOL


@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
def test_c2p_full_size_sampled_rows_and_norm(mode):
    """The C2' workload (n=28, cut 14|14, P=32): all 2^28 amplitudes through
    the FP32 and the split-BF16 x3 path sums (the form the benchmark times
    with --workload c2p); whole rows sampled against the oracle, the norm of
    the whole output checked on the device."""
    c = cg.c2p()
    plan = Plan(c, dtype="c64")
    assert plan.P == 32
    A, B = plan.run_paths()
    out = plan.amplitudes_full(A, B, mode=mode)
    nrm = hsf_norm2(out.reshape(-1)).cpu().numpy()[0]
    o = ohsf.plan(c)
    oa = ohsf.half_states(c, o, "A")
    ob = ohsf.half_states(c, o, "B")
    rows = np.random.default_rng(28).choice(1 << plan.na, 48, replace=False)
    rows = np.concatenate([[0, (1 << plan.na) - 1], rows])
    got = out[torch.from_numpy(rows).to("cuda")].cpu().numpy()
    ref = ohsf.amplitudes_rows(oa, ob, rows)
    assert _rel(got, ref) < C64_TOL
    assert abs(nrm - 1.0) < 1e-5
    del out
    torch.cuda.empty_cache()
