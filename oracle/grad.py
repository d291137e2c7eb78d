"""Gradients of the probability mass L = sum_j |<x_j|psi>|^2 with respect to
rotation angles (oracle; test-only).

Three independent FP64 routes:
* `loss_grad_shift`: the parameter-shift rule.  Every parametrised gate here
  is exp(-i t P / 2) with P^2 = 1 (RX, RY, RZ, RZZ), so
  dL/dt = [L(t + pi/2) - L(t - pi/2)] / 2 exactly; a parameter id shared by
  several gates sums the rule over its occurrences.  Each L comes from the
  plain HSF of `oracle.hsf` (or from the Schroedinger core for small n).
* `loss_grad_fd`: central finite differences of the same L.
* `loss_grad_adjoint`: the adjoint method on the full state (small n):
  dL/dt = 2 Re <lambda| dU/dt |state before the gate>, propagated backwards.
"""
import copy
import math

import numpy as np

from . import gates as G
from . import hsf as H
from . import sv

SHIFT_KINDS = {"RX", "RY", "RZ", "RZZ"}


def loss(circuit, xs, use_hsf=True):
    """L = sum_j |psi(x_j)|^2."""
    xs = np.asarray(xs, dtype=np.uint64)
    if use_hsf:
        pl = H.plan(circuit)
        a = H.half_states(circuit, pl, "A")
        b = H.half_states(circuit, pl, "B")
        amp = H.amplitudes_at(a, b, xs, pl["nb"])
    else:
        amp = sv.run(circuit)[xs.astype(np.int64)]
    return float(np.sum(np.abs(amp) ** 2))


def _with_param(circuit, gate_ids, delta):
    c = copy.copy(circuit)
    gs = list(circuit["gates"])
    for gid in gate_ids:
        g = dict(gs[gid])
        g["param"] = g["param"] + delta
        gs[gid] = g
    c["gates"] = gs
    return c


def occurrences(circuit):
    occ = {}
    for i, g in enumerate(circuit["gates"]):
        if g["param_id"] >= 0:
            occ.setdefault(g["param_id"], []).append(i)
    return occ


def loss_grad_shift(circuit, xs, param_ids=None, use_hsf=True):
    occ = occurrences(circuit)
    param_ids = sorted(occ) if param_ids is None else list(param_ids)
    out = {}
    for t in param_ids:
        tot = 0.0
        for gid in occ.get(t, []):
            if circuit["gates"][gid]["kind"] not in SHIFT_KINDS:
                raise ValueError("shift rule needs a Pauli rotation")
            lp = loss(_with_param(circuit, [gid], math.pi / 2), xs, use_hsf)
            lm = loss(_with_param(circuit, [gid], -math.pi / 2), xs, use_hsf)
            tot += 0.5 * (lp - lm)
        out[t] = tot
    return out


def loss_grad_fd(circuit, xs, param_ids=None, h=1e-4, use_hsf=True):
    occ = occurrences(circuit)
    param_ids = sorted(occ) if param_ids is None else list(param_ids)
    out = {}
    for t in param_ids:
        ids = occ.get(t, [])
        lp = loss(_with_param(circuit, ids, h), xs, use_hsf)
        lm = loss(_with_param(circuit, ids, -h), xs, use_hsf)
        out[t] = (lp - lm) / (2 * h)
    return out


def loss_grad_adjoint(circuit, xs, log=None):
    """Full-state adjoint: forward to the end, then walk back with the bra
    lambda = sum_j conj(psi_j) <x_j| and the state, un-applying each
    (unitary) gate in place.  Two state vectors in memory (2 x 16 GiB at
    n = 30); each rotation's term is one read-only inner product."""
    n = circuit["n"]
    xs = np.asarray(xs, dtype=np.uint64).astype(np.int64)
    state = sv.run(circuit)
    lam = np.zeros_like(state)
    lam[xs] = state[xs]              # ket form of the bra: <lam| = sum_j conj(psi_j) <x_j|
    grad = {}
    gates = circuit["gates"]
    for i in range(len(gates) - 1, -1, -1):
        g = gates[i]
        if g["param_id"] >= 0 and g["kind"] in SHIFT_KINDS:
            # dU/dt = -i/2 P U  =>  contribution 2 Re <lam| (-i/2) P |state after gate>
            val = 2.0 * float(np.real(-0.5j * sv.braket(lam, state, n, g["q"], G.generator(g))))
            grad[g["param_id"]] = grad.get(g["param_id"], 0.0) + val
        mh = np.ascontiguousarray(G.matrix(g).conj().T)
        sv.apply(state, n, g["q"], mh)
        sv.apply(lam, n, g["q"], mh)
        if log is not None and i % 50 == 0:
            log(f"adjoint: gate {i} of {len(gates)}")
    return grad
