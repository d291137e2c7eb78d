"""Writes the expected values used by the full-size GPU parity tests.

Calls only the FP64 oracle (`oracle/`) and the seeded circuit generators:

    python tests/golden/make_golden.py [c2 c3 c4]

c2_literal.npz  C2 (P=1024): psi at 4096 seeded basis states
c3.npz          C3: psi at its 1024 bitstrings, L, and dL/dt for 16 seeded
                parameter ids (parameter-shift rule on the oracle HSF)
c3_grad.npz     C3: dL/dt for all 708 parameter ids by the full-state FP64
                adjoint (two 2^30 states; about two hours on 8 cores), and
                central differences (h = 1e-4) of the oracle HSF loss for 24
                seeded ids
c3_medium_grad.npz  a C3-recipe circuit at n=26 (seed 7, 6 layers; 13-qubit
                sides): L over 256 seeded bitstrings and dL/dt for all its
                parameter ids by the full-state FP64 adjoint
c4.npz          C4 (P=4096): psi at 4096 seeded basis states
c5.npz          C5 (64 circuits): psi at 64 seeded basis states of each circuit
c5_rows.npz     C5: four whole output rows of each circuit (row 0, the last
                row, two seeded), kept as the FP64 norm of each row and 8
                seeded random complex projections sum_c w_c psi[r, c]
                (rows from numpy PCG64 seed 5000 + circuit, weights from
                seed 6000 + circuit)
qaoa_q30.npz    single-layer QAOA MaxCut on a seeded SBM graph with Table II's
                q30-1 shape (15|15 qubits, p_intra 0.8, p_inter 0.1): psi at
                4096 seeded basis states among the first 10^6 (the oracle HSF
                over the generator's own cascades, not the library's blocks)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import circuitgen as cg  # noqa: E402
from oracle import grad as OG  # noqa: E402
from oracle import hsf as H  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def sampled_psi(c, count, seed):
    t = time.time()
    pl = H.plan(c)
    a = H.half_states(c, pl, "A")
    b = H.half_states(c, pl, "B")
    rng = np.random.default_rng(seed)
    xs = np.unique(rng.integers(0, 1 << c["n"], size=count, dtype=np.uint64))
    amp = H.amplitudes_at(a, b, xs, pl["nb"])
    print(c["name"], "P", pl["P"], "sampled", len(xs), f"{time.time() - t:.1f}s", flush=True)
    return xs, amp


def c5_row_weights(i, nb):
    """The 8 x 2^nb complex projection weights of circuit i's rows (numpy
    PCG64, seed 6000 + i; the GPU test draws the same ones)."""
    rng = np.random.default_rng(6000 + i)
    return rng.standard_normal((8, 1 << nb)) + 1j * rng.standard_normal((8, 1 << nb))


def main(which):
    if "c2" in which:
        xs, amp = sampled_psi(cg.c2(), 4096, 22)
        np.savez(os.path.join(OUT, "c2_literal.npz"), x=xs, psi=amp)
    if "c3" in which:
        c = cg.c3()
        xs = cg.c3_bitstrings()
        t = time.time()
        pl = H.plan(c)
        a = H.half_states(c, pl, "A")
        b = H.half_states(c, pl, "B")
        amp = H.amplitudes_at(a, b, xs, pl["nb"])
        L = float(np.sum(np.abs(amp) ** 2))
        print("c3 psi", f"{time.time() - t:.1f}s", flush=True)
        inhull = sorted({c["gates"][g]["param_id"] for blk in pl["blocks"] for g in blk["hull"]
                         if c["gates"][g]["param_id"] >= 0})
        rng = np.random.default_rng(333)
        outside = [t_ for t_ in range(c["meta"]["n_params"]) if t_ not in set(inhull)]
        ids = sorted(set(rng.choice(outside, 12, replace=False).tolist()) | set(rng.choice(inhull, 4, replace=False).tolist()))
        g = OG.loss_grad_shift(c, xs, ids, use_hsf=True)
        print("c3 grads", f"{time.time() - t:.1f}s", flush=True)
        np.savez(os.path.join(OUT, "c3.npz"), x=xs, psi=amp, loss=L, grad_ids=np.array(ids),
                 grad=np.array([g[i] for i in ids]))
    if "c3grad" in which:
        c = cg.c3()
        xs = cg.c3_bitstrings()
        t = time.time()
        log = lambda m: print(f"{m} ({time.time() - t:.0f}s)", flush=True)  # noqa: E731
        rng = np.random.default_rng(3333)
        fd_ids = sorted(rng.choice(c["meta"]["n_params"], 24, replace=False).tolist())
        fd = OG.loss_grad_fd(c, xs, fd_ids, h=1e-4, use_hsf=True)
        log("c3 central differences")
        adj = OG.loss_grad_adjoint(c, xs, log=log)
        log("c3 adjoint")
        ids = np.arange(c["meta"]["n_params"])
        np.savez(os.path.join(OUT, "c3_grad.npz"), grad=np.array([adj[i] for i in ids]),
                 fd_ids=np.array(fd_ids), fd=np.array([fd[i] for i in fd_ids]), fd_h=1e-4)
    if "c3med" in which:
        # a medium C3-recipe circuit (n=26: 13-qubit sides, more than one
        # adjoint tile per row in complex64 and complex128), every angle
        c = cg.c3(seed=7, n=26, layers=6)
        xs = cg.c3_bitstrings(n=26, count=256, seed=8)
        t = time.time()
        log = lambda m: print(f"{m} ({time.time() - t:.0f}s)", flush=True)  # noqa: E731
        adj = OG.loss_grad_adjoint(c, xs, log=log)
        log("c3med adjoint")
        ids = np.arange(c["meta"]["n_params"])
        np.savez(os.path.join(OUT, "c3_medium_grad.npz"), x=xs, grad=np.array([adj[i] for i in ids]),
                 loss=OG.loss(c, xs, False))
    if "c4" in which:
        xs, amp = sampled_psi(cg.c4(), 4096, 44)
        np.savez(os.path.join(OUT, "c4.npz"), x=xs, psi=amp)
    if "c5" in which:
        xs_all, psi_all, owner = [], [], []
        for i, c in enumerate(cg.c5()):
            xs, amp = sampled_psi(c, 64, 500 + i)
            xs_all.append(xs)
            psi_all.append(amp)
            owner.append(np.full(len(xs), i, dtype=np.int32))
        np.savez(os.path.join(OUT, "c5.npz"), x=np.concatenate(xs_all), psi=np.concatenate(psi_all),
                 circuit=np.concatenate(owner))
    if "c5rows" in which:
        rows_all, norm_all, proj_all = [], [], []
        for i, c in enumerate(cg.c5()):
            t = time.time()
            pl = H.plan(c)
            a = H.half_states(c, pl, "A")
            b = H.half_states(c, pl, "B")
            na, nb = c["n"] - pl["nb"], pl["nb"]
            rng = np.random.default_rng(5000 + i)
            rows = np.array([0, (1 << na) - 1] + list(rng.choice(np.arange(1, (1 << na) - 1), 2, replace=False)),
                            dtype=np.int64)
            w = c5_row_weights(i, nb)
            psi = H.amplitudes_rows(a, b, rows)            # 4 x 2^nb
            rows_all.append(rows)
            norm_all.append(np.sum(np.abs(psi) ** 2, axis=1))
            proj_all.append(psi @ w.T)                     # 4 x 8
            print(c["name"], "P", pl["P"], "rows", f"{time.time() - t:.1f}s", flush=True)
        np.savez(os.path.join(OUT, "c5_rows.npz"), rows=np.array(rows_all), norm2=np.array(norm_all),
                 proj=np.array(proj_all))
    if "qaoa" in which:
        c = cg.qaoa_sbm(100, (15, 15), 0.8, 0.1)
        t = time.time()
        pl = H.plan(c)
        a = H.half_states(c, pl, "A")
        b = H.half_states(c, pl, "B")
        rng = np.random.default_rng(300)
        xs = np.unique(rng.integers(0, 10 ** 6, size=4096, dtype=np.uint64))
        amp = H.amplitudes_at(a, b, xs, pl["nb"])
        print(c["name"], "P", pl["P"], "sampled", len(xs), f"{time.time() - t:.1f}s", flush=True)
        np.savez(os.path.join(OUT, "qaoa_q30.npz"), x=xs, psi=amp)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c2", "c3", "c4", "c5", "qaoa"])
