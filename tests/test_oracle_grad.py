"""Pins of the oracle's gradient routes to the definition of the derivative:
the parameter-shift rule equals central finite differences, the full-state
adjoint equals both, and the HSF loss equals the Schroedinger loss."""
import numpy as np
import pytest

import circuitgen as cg
from oracle import grad as OG


def _small_c3(n=8, layers=6, seed=3):
    return cg.c3(seed=seed, n=n, layers=layers)


def _xs(n, count, seed):
    return cg.c3_bitstrings(n=n, count=count, seed=seed)


@pytest.mark.parametrize("n,layers", [(6, 3), (8, 6)])
def test_shift_rule_equals_finite_differences(n, layers):
    c = _small_c3(n, layers)
    xs = _xs(n, 16, 5)
    ids = sorted(OG.occurrences(c))[::3]
    gs = OG.loss_grad_shift(c, xs, ids, use_hsf=False)
    gf = OG.loss_grad_fd(c, xs, ids, h=1e-5, use_hsf=False)
    ref = max(abs(v) for v in gs.values())
    assert max(abs(gs[t] - gf[t]) for t in ids) < 1e-6 * max(ref, 1e-3)


def test_adjoint_equals_shift_rule():
    c = _small_c3(8, 6)
    xs = _xs(8, 20, 6)
    ga = OG.loss_grad_adjoint(c, xs)
    gs = OG.loss_grad_shift(c, xs, use_hsf=False)
    assert set(ga) == set(gs)
    assert max(abs(ga[t] - gs[t]) for t in gs) < 1e-12


def test_hsf_loss_equals_schroedinger_loss():
    c = _small_c3(10, 6)
    xs = _xs(10, 40, 7)
    assert abs(OG.loss(c, xs, True) - OG.loss(c, xs, False)) < 1e-14


def test_shared_parameter_sums_occurrences():
    c = cg.qaoa_sbm(2, sizes=(3, 3), p_intra=0.7, p_inter=0.4)
    xs = np.arange(64, dtype=np.uint64)[::3]
    gs = OG.loss_grad_shift(c, xs, use_hsf=False)
    gf = OG.loss_grad_fd(c, xs, h=1e-5, use_hsf=False)
    for t in gs:
        assert abs(gs[t] - gf[t]) < 1e-7


def test_braket_is_matrix_element_of_embedded_gate():
    """sv.braket(l, r, q, M) = l^H (M on q, as a dense 2^n x 2^n matrix built
    entry by entry) r, for random states and a random non-unitary 2-qubit M
    on non-adjacent qubits in both orders."""
    import numpy as np
    from oracle import sv
    rng = np.random.default_rng(17)
    n = 6
    l = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    r = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    m = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    for q in ([1, 4], [4, 1], [0, 5]):
        want = np.vdot(l, sv.embed(n, q, m) @ r)
        got = sv.braket(l, r, n, q, m)
        assert abs(got - want) < 1e-12 * abs(want)
    m1 = rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2))
    want = np.vdot(l, sv.embed(n, [3], m1) @ r)
    assert abs(sv.braket(l, r, n, [3], m1) - want) < 1e-12 * abs(want)


def test_c3_stored_gradients_agree_across_routes():
    """The stored full-size C3 gradient (all 708 angles, the oracle's
    two-state adjoint) against two other routes the oracle took for the same
    loss: the parameter-shift rule on 16 sampled angles (golden c3.npz) and
    central finite differences on 24 more (step h, truncation error O(h^2))."""
    import os
    gold = os.path.join(os.path.dirname(__file__), "golden")
    z = np.load(os.path.join(gold, "c3_grad.npz"))
    c = np.load(os.path.join(gold, "c3.npz"))
    g = z["grad"]
    assert g.shape == (708,) and np.all(np.isfinite(g))
    scale = np.max(np.abs(g))
    assert scale > 0
    assert np.max(np.abs(g[c["grad_ids"]] - c["grad"])) < 1e-10 * scale
    assert np.max(np.abs(g[z["fd_ids"]] - z["fd"])) < 1e-6 * scale
