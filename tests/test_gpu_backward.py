"""GPU gradients of the probability mass L = sum_j |psi(x_j)|^2 (hsf_backward)
against the FP64 oracle's parameter-shift gradients (which are pinned to
finite differences and to the full-state adjoint in test_oracle_grad.py).
Bar: max |g - g_ref| <= 1e-4 max |g_ref| (complex64), 1e-9 (complex128)."""
import numpy as np
import pytest
import torch

import circuitgen as cg
from oracle import grad as OG
from paper_2502_06959_amd import Plan, ProbabilityMass

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check(c, xs, dtype, chunk=None, tol=None):
    ref = OG.loss_grad_shift(c, xs, use_hsf=True)
    plan = Plan(c, dtype=dtype)
    x = torch.from_numpy(np.asarray(xs, dtype=np.int64)).cuda()
    g = plan.backward(x, chunk).cpu().numpy()
    r = np.array([ref.get(t, 0.0) for t in range(plan.n_params)])
    tol = tol or (1e-9 if dtype == "c128" else 1e-4)
    err = np.max(np.abs(g - r)) / np.max(np.abs(r))
    assert err < tol, err
    lo = OG.loss(c, xs)
    assert abs(plan.loss(x) - lo) < (1e-12 if dtype == "c128" else 1e-6) * max(1.0, lo)
    return g


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_variational_small(dtype):
    # the C3 recipe at n=10: RY/RZ layers, RZZ brick, blocks of 3 crossing RZZs (3|3 hulls)
    c = cg.c3(seed=3, n=10, layers=6)
    xs = cg.c3_bitstrings(n=10, count=64, seed=9)
    _check(c, xs, dtype)


def test_variational_chunks_and_determinism():
    c = cg.c3(seed=4, n=10, layers=6)
    xs = cg.c3_bitstrings(n=10, count=48, seed=10)
    plan = Plan(c)
    x = torch.from_numpy(np.asarray(xs, dtype=np.int64)).cuda()
    g1 = plan.backward(x, chunk=plan.P).cpu().numpy()
    g2 = plan.backward(x, chunk=plan.P).cpu().numpy()
    g3 = plan.backward(x, chunk=5).cpu().numpy()
    assert np.array_equal(g1, g2)
    assert np.max(np.abs(g1 - g3)) <= 1e-5 * np.max(np.abs(g1))


def test_qaoa_shared_parameters():
    c = cg.qaoa_sbm(4, sizes=(5, 5), p_intra=0.6, p_inter=0.3)
    xs = np.arange(0, 1 << 10, 7, dtype=np.uint64)
    _check(c, xs, "c128")


def test_random_rotations_outside_blocks_only():
    rng = np.random.default_rng(12)
    gs, pid = [], 0
    for layer in range(4):
        for q in range(8):
            gs.append(cg.gate(["RX", "RY", "RZ"][rng.integers(3)], (q,), param=rng.uniform(0, 6), param_id=pid))
            pid += 1
        for q in range(0, 7, 2) if layer % 2 == 0 else range(1, 7, 2):
            gs.append(cg.gate("CZ", (q, q + 1)))
    c = cg.circuit("rot", 8, gs, 3, [[i] for i, g in enumerate(gs) if cg.crossing(g, 3)])
    xs = np.arange(0, 256, 3, dtype=np.uint64)
    _check(c, xs, "c64")


def test_autograd_function():
    c = cg.c3(seed=5, n=8, layers=4)
    xs = cg.c3_bitstrings(n=8, count=32, seed=11)
    x = torch.from_numpy(np.asarray(xs, dtype=np.int64)).cuda()
    theta = torch.tensor([g["param"] for g in c["gates"] if g["param_id"] >= 0], dtype=torch.float64,
                         requires_grad=True)
    L = ProbabilityMass.apply(theta, c, x, "c128")
    L.backward()
    ref = OG.loss_grad_shift(c, xs)
    r = np.array([ref[t] for t in range(len(theta))])
    assert np.max(np.abs(theta.grad.numpy() - r)) < 1e-9 * np.max(np.abs(r))
    assert abs(L.item() - OG.loss(c, xs)) < 1e-12
