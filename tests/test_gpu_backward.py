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


@pytest.mark.parametrize("chunk", [None, 5])
def test_shifted_runs_in_batches_of_any_size(chunk):
    """The shifted forward runs go as copies of one run, as many per batch as
    the workspace holds: the least workspace (one copy per batch), one of
    three copies and the preferred one give the same gradient bit for bit."""
    c = cg.c3(seed=5, n=10, layers=6)
    xs = cg.c3_bitstrings(n=10, count=40, seed=11)
    plan = Plan(c)
    x = torch.from_numpy(np.asarray(xs, dtype=np.int64)).cuda()
    n_min = plan.workspace_backward(x.numel(), chunk, minimal=True)
    n_pref = plan.workspace_backward(x.numel(), chunk)
    assert n_pref > n_min
    g = plan.backward(x, chunk).cpu().numpy()
    for nbytes in (n_min, (2 * n_min + n_pref) // 3):
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        assert np.array_equal(plan.backward(x, chunk, ws=ws).cpu().numpy(), g), nbytes
    from paper_2502_06959_amd import HsfError
    with pytest.raises(HsfError):
        plan.backward(x, chunk, ws=torch.empty(n_min - 256, dtype=torch.uint8, device="cuda"))


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


def _runs_circuit(kinds_1q, kinds_2q, seed):
    # long runs of one- and two-qubit rotations on few qubits, a three-qubit
    # unitary in the middle of them, angles at every position of a run
    rng = np.random.default_rng(seed)
    gs, pid = [], 0
    for layer in range(5):
        for q in (0, 1, 2, 5, 6, 7):
            gs.append(cg.gate(kinds_1q[rng.integers(len(kinds_1q))], (q,), param=rng.uniform(0, 6), param_id=pid))
            pid += 1
        for a, b in ((0, 1), (1, 2), (5, 6), (6, 7)):
            gs.append(cg.gate(kinds_2q[rng.integers(len(kinds_2q))], (a, b), param=rng.uniform(0, 6), param_id=pid))
            pid += 1
        if layer == 2:
            gs.append(cg.gate("U", (0, 1, 2), matrix=cg.haar_unitary(rng, 8)))
            gs.append(cg.gate("U", (7, 6, 5), matrix=cg.haar_unitary(rng, 8)))
        gs.append(cg.gate("CZ", (3, 4)))
        gs.append(cg.gate("RY", (3,), param=rng.uniform(0, 6), param_id=pid))
        pid += 1
        gs.append(cg.gate("RY", (4,), param=rng.uniform(0, 6), param_id=pid))
        pid += 1
    return cg.circuit("runs", 8, gs, 3, [[i] for i, g in enumerate(gs) if cg.crossing(g, 3)])


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_adjoint_runs_and_wide_gates(dtype):
    # the adjoint pass undoes runs of gates on up to three qubits in
    # registers and wider gates one by one
    c = _runs_circuit(("RX", "RY", "RZ"), ("RZZ",), 21)
    _check(c, np.arange(1, 256, 5, dtype=np.uint64), dtype)


def test_phase_angles_against_finite_differences():
    # PHASE and CP angles (generator i|1><1|) in runs, against the oracle's
    # central differences (h = 1e-4: truncation far below the bar)
    c = _runs_circuit(("PHASE", "RY"), ("CP", "RZZ"), 22)
    xs = np.arange(1, 256, 5, dtype=np.uint64)
    ref = OG.loss_grad_fd(c, xs, h=1e-4, use_hsf=True)
    plan = Plan(c, dtype="c128")
    x = torch.from_numpy(np.asarray(xs, dtype=np.int64)).cuda()
    g = plan.backward(x).cpu().numpy()
    r = np.array([ref.get(t, 0.0) for t in range(plan.n_params)])
    assert np.max(np.abs(g - r)) / np.max(np.abs(r)) < 1e-6


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


def test_autograd_function_on_device_angles():
    """Angles held on the GPU: the loss and the gradient come back on the
    GPU, and a non-scalar cotangent path (a weighted sum) works."""
    c = cg.c3(seed=6, n=8, layers=4)
    xs = cg.c3_bitstrings(n=8, count=32, seed=12)
    x = torch.from_numpy(np.asarray(xs, dtype=np.int64)).cuda()
    theta = torch.tensor([g["param"] for g in c["gates"] if g["param_id"] >= 0], dtype=torch.float64,
                         device="cuda", requires_grad=True)
    L = ProbabilityMass.apply(theta, c, x, "c128")
    assert L.device.type == "cuda"
    (3.0 * L).backward()
    assert theta.grad.device.type == "cuda"
    ref = OG.loss_grad_shift(c, xs)
    r = 3.0 * np.array([ref[t] for t in range(len(theta))])
    assert np.max(np.abs(theta.grad.cpu().numpy() - r)) < 1e-9 * np.max(np.abs(r))


def _amps_oracle(c, xs):
    from oracle import sv
    return sv.run(c)[np.asarray(xs, dtype=np.int64)]


def _fd_linear(c, xs, gco, h=1e-5):
    """Central differences (FP64 Schroedinger oracle) of the real functional
    L_g(t) = sum_j Re(conj(g_j) psi_j(t)), every occurrence of a parameter id
    shifted together: its gradient is sum_j Re(conj(g_j) dpsi_j/dt)."""
    occ = OG.occurrences(c)
    out = np.zeros(max(occ) + 1)
    for t, ids in occ.items():
        lp = np.sum(np.real(np.conj(gco) * _amps_oracle(OG._with_param(c, ids, h), xs)))
        lm = np.sum(np.real(np.conj(gco) * _amps_oracle(OG._with_param(c, ids, -h), xs)))
        out[t] = (lp - lm) / (2 * h)
    return out


def test_loss_entry_point_matches_oracle():
    """hsf_loss: psi(x_j) and L = sum_j |psi(x_j)|^2 summed inside the
    library over path chunks, against the Schroedinger oracle; any chunking
    gives the same amplitudes to rounding; no bitstrings give L = 0."""
    c = cg.c3(seed=7, n=10, layers=6)
    xs = cg.c3_bitstrings(n=10, count=64, seed=13)
    plan = Plan(c, dtype="c128")
    x = torch.from_numpy(np.asarray(xs, dtype=np.int64)).cuda()
    ref = _amps_oracle(c, xs)
    amps = torch.empty(len(xs), dtype=torch.complex128, device="cuda")
    L = plan.loss_device(x, chunk=plan.P, amps=amps).item()
    assert np.max(np.abs(amps.cpu().numpy() - ref)) < 1e-12
    assert abs(L - np.sum(np.abs(ref) ** 2)) < 1e-12
    amps5 = torch.empty_like(amps)
    L5 = plan.loss_device(x, chunk=5, amps=amps5).item()
    assert np.max(np.abs(amps5.cpu().numpy() - ref)) < 1e-12 and abs(L5 - L) < 1e-13
    empty = torch.empty(0, dtype=torch.int64, device="cuda")
    assert plan.loss_device(empty).item() == 0.0
    p64 = Plan(c)
    assert abs(p64.loss(x) - L) < 1e-6 * L


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_caller_cotangent_gradient(dtype):
    """hsf_backward with caller cotangents g_j: sum_j Re(conj(g_j) dpsi_j/dt)
    for every angle (inside the 3|3 block hulls as well) against central
    differences of the oracle's amplitudes; g = 2 psi gives the probability
    mass gradient."""
    c = cg.c3(seed=8, n=10, layers=6)
    xs = cg.c3_bitstrings(n=10, count=40, seed=14)
    rng = np.random.default_rng(15)
    gco = rng.standard_normal(len(xs)) + 1j * rng.standard_normal(len(xs))
    plan = Plan(c, dtype=dtype)
    x = torch.from_numpy(np.asarray(xs, dtype=np.int64)).cuda()
    g = plan.backward(x, dl_dpsi=torch.from_numpy(gco).cuda()).cpu().numpy()
    ref = _fd_linear(c, xs, gco)
    tol = 1e-6 if dtype == "c128" else 1e-4
    assert np.max(np.abs(g - ref)) < tol * np.max(np.abs(ref))
    amps = torch.empty(len(xs), dtype=torch.complex128, device="cuda")
    plan.loss_device(x, amps=amps)
    g2 = plan.backward(x, dl_dpsi=2 * amps).cpu().numpy()
    g0 = plan.backward(x).cpu().numpy()
    assert np.max(np.abs(g2 - g0)) <= 1e-12 * np.max(np.abs(g0))


def test_amplitudes_autograd_nonlinear_loss():
    """Amplitudes (torch.autograd.Function over hsf_loss / hsf_backward with
    cotangents): L = sum_j |psi_j|^4 + Re(psi_0 psi_1), gradient against
    central differences of the same L on the oracle's amplitudes."""
    from paper_2502_06959_amd import Amplitudes
    c = cg.c3(seed=9, n=8, layers=4)
    xs = cg.c3_bitstrings(n=8, count=24, seed=16)
    x = torch.from_numpy(np.asarray(xs, dtype=np.int64)).cuda()
    theta = torch.tensor([g["param"] for g in c["gates"] if g["param_id"] >= 0], dtype=torch.float64,
                         device="cuda", requires_grad=True)
    psi = Amplitudes.apply(theta, c, x, "c128")
    L = (psi.abs() ** 4).sum() + (psi[0] * psi[1]).real
    L.backward()

    def Lo(cc):
        a = _amps_oracle(cc, xs)
        return np.sum(np.abs(a) ** 4) + np.real(a[0] * a[1])

    assert abs(L.item() - Lo(c)) < 1e-12
    h = 1e-5
    ref = np.array([(Lo(OG._with_param(c, ids, h)) - Lo(OG._with_param(c, ids, -h))) / (2 * h)
                    for t, ids in sorted(OG.occurrences(c).items())])
    got = theta.grad.cpu().numpy()
    assert theta.grad.device.type == "cuda"
    assert np.max(np.abs(got - ref)) < 1e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_medium_c3_every_angle_multipass_tree(dtype):
    """A C3-recipe circuit at n=26 (13-qubit sides): forced path-tree sweeps on
    8-qubit tiles (several passes per level) and 13-qubit adjoint rows (two
    adjoint tiles per row in complex64, four in complex128), against the
    oracle's full-state adjoint gradient for every angle
    (tests/golden/c3_medium_grad.npz)."""
    import os
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_medium_grad.npz"))
    c = cg.c3(seed=7, n=26, layers=6)
    plan = Plan(c, dtype=dtype, tree="on", tile_qubits=8)
    assert plan.na == 13 and plan.side_stats(0)["tile_qubits"] == 8 and plan.uses_tree(plan.P)
    x = torch.from_numpy(np.asarray(g["x"], dtype=np.int64)).cuda()
    got = plan.backward(x).cpu().numpy()
    ref = g["grad"]
    tol = 1e-9 if dtype == "c128" else 1e-4
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    assert err < tol, err
    assert abs(plan.loss(x) - float(g["loss"])) < (1e-12 if dtype == "c128" else 1e-6) * float(g["loss"])
