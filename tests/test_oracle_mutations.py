"""Planted mistakes in the oracle (on the CPU) must be caught by its pins.

Each case patches one plausible error into the oracle -- a transposed
operand, a dropped factor, a wrong bit order, a wrong index -- and checks
that the comparison with the Schroedinger core (itself pinned to closed forms
and brute force) or the printed Schmidt values fails.
"""
import itertools
import math

import numpy as np
import pytest

import circuitgen as cg
from oracle import gates as G
from oracle import hsf, sv


def _hsf_matches(c):
    try:
        return hsf.rel_l2(hsf.amplitudes(c), sv.run(c)) < 1e-10
    except hsf.PlanError:
        return False


CASES = [cg.c1b(), cg.qft_basis(6, 11), cg.random_circuit(33, n=10, n_gates=40, group=2, p2=0.3,
                                                            two_q_kinds=("CZ", "CX", "RZZ", "CP", "ISWAP"))]


def test_unmodified_oracle_passes():
    assert all(_hsf_matches(c) for c in CASES)


def _caught(monkeypatch, name, fake):
    monkeypatch.setattr(hsf, name, fake)
    return not all(_hsf_matches(c) for c in CASES)


def test_swapped_schmidt_factors_caught(monkeypatch):
    real = hsf.schmidt

    def bad(u, na, nb):
        s, X, Y = real(u, na, nb)
        return s, np.conj(X), Y          # V* vs V confused
    assert _caught(monkeypatch, "schmidt", bad)


def test_transposed_factor_caught(monkeypatch):
    real = hsf.schmidt

    def bad(u, na, nb):
        s, X, Y = real(u, na, nb)
        return s, X, np.transpose(Y, (0, 2, 1))   # (i_b, j_b) read as (j_b, i_b)
    assert _caught(monkeypatch, "schmidt", bad)


def test_dropped_singular_value_caught(monkeypatch):
    real = hsf.schmidt

    def bad(u, na, nb):
        s, X, Y = real(u, na, nb)
        return np.ones_like(s) * (s > 1e-10 * s[0]), X, Y   # sigma dropped
    assert _caught(monkeypatch, "schmidt", bad)


def test_wrong_block_bit_order_caught(monkeypatch):
    real = hsf.block_operator

    def bad(circuit, hull_ids, sa, sb):
        return real(circuit, hull_ids, sb, sa)         # side b placed above side a
    assert _caught(monkeypatch, "block_operator", bad)


def test_reversed_slot_qubits_caught(monkeypatch):
    real = hsf.side_ops

    def bad(circuit, pl, side, factors=None):
        ops, slot_of = real(circuit, pl, side, factors)
        ops = [(list(reversed(q)) if k >= 0 else q, m) for (q, m), k in zip(ops, slot_of)]
        return ops, slot_of
    assert _caught(monkeypatch, "side_ops", bad)


def test_missing_hull_gate_caught(monkeypatch):
    real = hsf.hull

    def bad(circuit, block):
        h = real(circuit, block)
        inner = [i for i in h if i not in block]
        return [i for i in h if i != (inner[0] if inner else -1)]
    assert _caught(monkeypatch, "hull", bad)


def test_wrong_path_digit_order_caught(monkeypatch):
    """Digits decoded with block 0 least significant break lexicographic order."""
    pl = hsf.plan(cg.c1b())
    bad = lambda p: [(p // R) % r for R, r in zip(reversed(pl["strides"]), pl["ranks"])]
    lex = list(itertools.product(*[range(r) for r in pl["ranks"]]))
    assert [tuple(bad(p)) for p in range(pl["P"])] != lex


def test_wrong_rzz_sign_caught():
    """RZZ with exp(+i phi ZZ/2) instead of exp(-i phi ZZ/2)."""
    phi = 1.234
    good = G.matrix(cg.gate("RZZ", (0, 1), param=phi))
    bad = np.conj(good)
    s_good = hsf.schmidt(good, 1, 1)[0]
    want = sorted([2 * abs(math.cos(phi / 2)), 2 * abs(math.sin(phi / 2))], reverse=True)
    assert np.allclose(s_good[:2], want)
    import scipy.linalg
    ref = scipy.linalg.expm(-0.5j * phi * np.kron(G.Z, G.Z))
    assert np.allclose(good, ref) and not np.allclose(bad, ref)


def test_wrong_core_bit_significance_caught():
    """Gate matrix with q[1] as the most significant bit fails the Bell pin."""
    psi = np.zeros(4, dtype=complex)
    psi[0] = 1
    sv.apply(psi, 2, [1], G.H)
    sv.apply(psi, 2, [0, 1], G.matrix(cg.gate("CX", (1, 0))))   # operands swapped
    assert not np.allclose(psi, np.array([1, 0, 0, 1]) / math.sqrt(2))
