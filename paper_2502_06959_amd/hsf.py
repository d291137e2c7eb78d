"""Python binding of libhsf with the C names.  Device buffers are torch
tensors (complex64 / complex128 / uint64 / float64 on a HIP device); work is
enqueued on torch's current stream of the tensors' device."""
import ctypes

import numpy as np
import torch

from . import _lib as L

_DT = {"c64": L.HSF_C64, "c128": L.HSF_C128}
_TORCH_DT = {L.HSF_C64: torch.complex64, L.HSF_C128: torch.complex128}


def _stream(t=None):
    dev = t.device if t is not None else torch.device("cuda", torch.cuda.current_device())
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _gate_struct(g):
    s = L.HsfGate()
    s.kind = L.GATE_KIND[g["kind"]]
    s.nq = len(g["q"])
    for i, q in enumerate(g["q"]):
        s.q[i] = int(q)
    s.param = float(g["param"]) if g.get("param") is not None else 0.0
    s.param_id = int(g.get("param_id", -1))
    m = None
    if g.get("matrix") is not None:
        m = np.ascontiguousarray(np.asarray(g["matrix"], dtype=np.complex128))
        s.matrix = m.ctypes.data
    return s, m


def _circuit_struct(circuit):
    gates = circuit["gates"]
    arr = (L.HsfGate * max(1, len(gates)))()
    keep = [arr]
    for i, g in enumerate(gates):
        s, m = _gate_struct(g)
        arr[i] = s
        keep.append(m)
    c = L.HsfCircuit(n_qubits=int(circuit["n"]), reserved=0, n_gates=len(gates),
                     gates=ctypes.cast(arr, ctypes.POINTER(L.HsfGate)))
    return c, keep


def hsf_find_blocks(circuit, cut=None):
    """(order, blocks): a gate order with the same unitary and joint blocks of
    the commuting crossing gates, as positions in that order."""
    cut = circuit["cut"] if cut is None else cut
    c, keep = _circuit_struct(circuit)
    G = len(circuit["gates"])
    order = np.zeros(max(1, G), dtype=np.int64)
    ids = np.zeros(max(1, G), dtype=np.int64)
    offs = np.zeros(G + 1, dtype=np.int64)
    nb = ctypes.c_int32()
    p64 = ctypes.POINTER(ctypes.c_int64)
    L.check(L.lib().hsf_find_blocks(ctypes.byref(c), int(cut), order.ctypes.data_as(p64), ids.ctypes.data_as(p64),
                                    offs.ctypes.data_as(p64), ctypes.byref(nb)))
    del keep
    blocks = [[int(v) for v in ids[offs[k]:offs[k + 1]]] for k in range(nb.value)]
    return [int(v) for v in order[:G]], blocks


def joint_blocked(circuit, cut=None):
    """The circuit with its gates in hsf_find_blocks' order and those blocks."""
    order, blocks = hsf_find_blocks(circuit, cut)
    out = dict(circuit)
    out["gates"] = [circuit["gates"][i] for i in order]
    out["blocks"] = blocks
    if cut is not None:
        out["cut"] = cut
    return out


_TREE = {"auto": 0, "off": 1, "on": 2}


def hsf_plan(circuit, cut=None, blocks=None, dtype="c64", rank_tol=1e-10, max_side_qubits=4, tile_qubits=0,
             fuse=True, tree="auto", defer_b_suffix=False):
    """Plan for `circuit` (a dict with n, gates[, cut, blocks]); returns the
    opaque handle (int).  tree: path-tree sweeps "auto" (by the planner's
    cost estimate), "off" or "on".  defer_b_suffix: side b's gates after its
    last factor slot are applied to output rows by Plan.apply_b_suffix
    instead of to every path.  Raises HsfError with the library's status."""
    lib = L.lib()
    cut = circuit["cut"] if cut is None else cut
    blocks = circuit.get("blocks", []) if blocks is None else blocks
    c, keep = _circuit_struct(circuit)
    ids = np.array([int(i) for b in blocks for i in b] or [0], dtype=np.int64)
    offs = np.zeros(len(blocks) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(b) for b in blocks]) if blocks else []
    opts = L.HsfPlanOptions(rank_tol=rank_tol, max_side_qubits=max_side_qubits, dtype=_DT[dtype],
                            tile_qubits=tile_qubits, fuse=1 if fuse else 0, tree=_TREE[tree],
                            defer_b_suffix=1 if defer_b_suffix else 0)
    h = ctypes.c_void_p()
    L.check(lib.hsf_plan(ctypes.byref(c), int(cut), ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(blocks), ctypes.byref(opts),
                         ctypes.byref(h)))
    del keep
    return h.value


def hsf_workspace_size(plan, op, n_paths, mode=0):
    return int(L.lib().hsf_workspace_size(ctypes.c_void_p(plan), op, n_paths, mode))


def hsf_run_paths(plan, p_begin, p_end, psiA, psiB, ws=None):
    """Half-states of paths [p_begin, p_end) into rows of psiA / psiB.  ws:
    device workspace for the path-tree levels (allocated here when None)."""
    ref = psiA if psiA is not None else psiB
    if ws is None and p_end > p_begin:
        nbytes = hsf_workspace_size(plan, 0, p_end - p_begin, 0)
        if nbytes > 0:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=ref.device)
    L.check(L.lib().hsf_run_paths(ctypes.c_void_p(plan), p_begin, p_end, _ptr(psiA),
                                  psiA.stride(0) if psiA is not None else 0, _ptr(psiB),
                                  psiB.stride(0) if psiB is not None else 0, _ptr(ws),
                                  ws.numel() * ws.element_size() if ws is not None else 0, _stream(ref)))


def hsf_run_paths_rows(plan, p_begin, p_end, row_begin, row_end, psiA, psiB, ws=None):
    """hsf_run_paths keeping only side a's amplitudes [row_begin, row_end)
    of each psiA row (the rest is left unspecified)."""
    if ws is None and p_end > p_begin:
        nbytes = hsf_workspace_size(plan, 0, p_end - p_begin, 0)
        if nbytes > 0:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=psiA.device)
    L.check(L.lib().hsf_run_paths_rows(ctypes.c_void_p(plan), p_begin, p_end, row_begin, row_end, _ptr(psiA),
                                       psiA.stride(0), _ptr(psiB), psiB.stride(0) if psiB is not None else 0,
                                       _ptr(ws), ws.numel() * ws.element_size() if ws is not None else 0,
                                       _stream(psiA)))


def hsf_amplitudes_full(plan, psiA, psiB, n_paths, row_begin, row_end, out, mode="f32", accumulate=False,
                        ws=None):
    L.check(L.lib().hsf_amplitudes_full(ctypes.c_void_p(plan), _ptr(psiA), psiA.stride(0), _ptr(psiB),
                                        psiB.stride(0), n_paths, row_begin, row_end, _ptr(out), out.stride(0),
                                        L.SUM_MODE[mode], 1 if accumulate else 0, _ptr(ws),
                                        ws.numel() * ws.element_size() if ws is not None else 0,
                                        _stream(psiA)))


def hsf_amplitudes_full_noalloc(plan, psiA, psiB, n_paths, row_begin, row_end, out, mode="bf16x3",
                                accumulate=False):
    """hsf_amplitudes_full with its scratch in the library's static device
    array (no workspace, no allocation)."""
    L.check(L.lib().hsf_amplitudes_full_noalloc(ctypes.c_void_p(plan), _ptr(psiA), psiA.stride(0), _ptr(psiB),
                                                psiB.stride(0), n_paths, row_begin, row_end, _ptr(out),
                                                out.stride(0), L.SUM_MODE[mode], 1 if accumulate else 0,
                                                _stream(psiA)))


def hsf_split_operands(plan, psiA, psiB, n_paths, ws):
    """Split-BF16 planes of both operands (all rows) into ws, for later
    HSF_SUM_BF16X3_SPLIT path sums ("bf16x3_split") over row ranges."""
    L.check(L.lib().hsf_split_operands(ctypes.c_void_p(plan), _ptr(psiA), psiA.stride(0), _ptr(psiB),
                                       psiB.stride(0), n_paths, _ptr(ws), ws.numel() * ws.element_size(),
                                       _stream(psiA)))


def hsf_amplitudes_bitstrings(plan, psiA, psiB, n_paths, x, out, accumulate=False):
    L.check(L.lib().hsf_amplitudes_bitstrings(ctypes.c_void_p(plan), _ptr(psiA), psiA.stride(0), _ptr(psiB),
                                              psiB.stride(0), n_paths, _ptr(x), x.numel(), _ptr(out),
                                              1 if accumulate else 0, _stream(psiA)))


def hsf_norm2(a, b=None):
    """(sum |a|^2, sum |a - b|^2) accumulated in FP64 on the device."""
    dev = a.device
    out = torch.empty(2, dtype=torch.float64, device=dev)
    ws = torch.empty(8192, dtype=torch.float64, device=dev)
    adt = L.HSF_C128 if a.dtype == torch.complex128 else L.HSF_C64
    bdt = (L.HSF_C128 if b.dtype == torch.complex128 else L.HSF_C64) if b is not None else 0
    if b is not None and b.numel() != a.numel():
        raise ValueError("a and b differ in size")
    L.check(L.lib().hsf_norm2(_ptr(a), adt, _ptr(b), bdt, a.numel(), _ptr(out), _ptr(ws), 8192 * 8, _stream(a)))
    return out


def hsf_backward(plan, x, grad, chunk, ws, dl_dpsi=None):
    """grad <- dL/dt for every parameter id; dl_dpsi: None (probability mass)
    or complex128 cotangents of psi(x_j) on the device."""
    if dl_dpsi is not None:
        assert dl_dpsi.dtype == torch.complex128 and dl_dpsi.is_contiguous() and dl_dpsi.numel() == x.numel()
    L.check(L.lib().hsf_backward(ctypes.c_void_p(plan), _ptr(x), x.numel(), _ptr(dl_dpsi), _ptr(grad), grad.numel(),
                                 chunk, _ptr(ws), ws.numel() * ws.element_size(), _stream(grad)))


def hsf_loss(plan, x, loss, chunk, ws, amps=None):
    """loss (one float64 device entry) <- sum_j |psi(x_j)|^2; amps (optional
    complex128, x.numel() entries) <- psi(x_j)."""
    L.check(L.lib().hsf_loss(ctypes.c_void_p(plan), _ptr(x), x.numel(), _ptr(loss), _ptr(amps), chunk, _ptr(ws),
                             ws.numel() * ws.element_size(), _stream(loss)))


class Plan:
    """A planned circuit.  `circuit` is a dict with keys n, gates, cut and
    blocks (the format of circuitgen); dtype "c64" or "c128"."""

    def __init__(self, circuit, cut=None, blocks=None, dtype=None, **opts):
        dtype = dtype or circuit.get("meta", {}).get("dtype", "c64")
        self.dtype = dtype
        self.n_params = 1 + max([g.get("param_id", -1) for g in circuit["gates"]] + [-1])
        self.handle = hsf_plan(circuit, cut, blocks, dtype=dtype, **opts)
        n, c, na, nb, k = (ctypes.c_int32() for _ in range(5))
        p = ctypes.c_int64()
        L.check(L.lib().hsf_plan_dims(ctypes.c_void_p(self.handle), *(ctypes.byref(v) for v in (n, c, na, nb, k)),
                                      ctypes.byref(p)))
        self.n, self.cut, self.na, self.nb, self.K, self.P = n.value, c.value, na.value, nb.value, k.value, p.value
        self.torch_dtype = _TORCH_DT[_DT[dtype]]

    def close(self):
        if getattr(self, "handle", None):
            L.lib().hsf_plan_destroy(ctypes.c_void_p(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply_b_suffix(self, out, rows=None):
        """Side b's deferred gates on the first `rows` rows of `out` (rows x
        2^n_b, the plan's dtype, on the device), in place
        (hsf_apply_b_suffix); a no-op for a plan without a deferred suffix."""
        rows = out.shape[0] if rows is None else rows
        if out.dtype != self.torch_dtype:
            raise ValueError(f"rows must be {self.torch_dtype} like the plan's half-states")
        L.check(L.lib().hsf_apply_b_suffix(ctypes.c_void_p(self.handle), _ptr(out), out.stride(0), rows,
                                           _stream(out)))
        return out

    # ---------------------------------------------------------- tables ----
    def block_info(self, k):
        r, na_, nb_, ci = (ctypes.c_int32() for _ in range(4))
        st, hl = ctypes.c_int64(), ctypes.c_int64()
        sa, sb = (ctypes.c_int32 * L.HSF_MAX_BLOCK_SIDE)(), (ctypes.c_int32 * L.HSF_MAX_BLOCK_SIDE)()
        L.check(L.lib().hsf_block_info(ctypes.c_void_p(self.handle), k, ctypes.byref(r), ctypes.byref(st),
                                       ctypes.byref(na_), sa, ctypes.byref(nb_), sb, ctypes.byref(hl),
                                       ctypes.byref(ci)))
        hull = np.zeros(max(1, hl.value), dtype=np.int64)
        L.check(L.lib().hsf_block_hull(ctypes.c_void_p(self.handle), k,
                                       hull.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return {"rank": r.value, "stride": st.value, "sa": list(sa[:na_.value]), "sb": list(sb[:nb_.value]),
                "hull": [int(v) for v in hull[:hl.value]], "caller_index": ci.value}

    def block_factors(self, k):
        """(sigma, xa, yb): singular values and the dense side factors of
        block k (a side wider than 8 qubits gives None)."""
        info = self.block_info(k)
        ka, kb, r = len(info["sa"]), len(info["sb"]), info["rank"]
        sig = np.zeros(4 ** min(ka, kb, 8), dtype=np.float64)
        xa = np.zeros((r, 2 ** ka, 2 ** ka), dtype=np.complex128) if ka <= 8 else None
        yb = np.zeros((r, 2 ** kb, 2 ** kb), dtype=np.complex128) if kb <= 8 else None
        L.check(L.lib().hsf_block_factors(ctypes.c_void_p(self.handle), k, sig.ctypes.data,
                                          xa.ctypes.data if xa is not None else None,
                                          yb.ctypes.data if yb is not None else None))
        return sig, xa, yb

    def digits(self, p):
        d = (ctypes.c_int32 * max(1, self.K))()
        L.check(L.lib().hsf_path_digits(ctypes.c_void_p(self.handle), int(p), d))
        return list(d[:self.K])

    def side_stats(self, side):
        a, b, e = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        c, d, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        L.check(L.lib().hsf_side_stats(ctypes.c_void_p(self.handle), side, ctypes.byref(a), ctypes.byref(b),
                                       ctypes.byref(c), ctypes.byref(d), ctypes.byref(e), ctypes.byref(f)))
        return {"ops_logical": a.value, "ops_fused": b.value, "passes": c.value, "tile_qubits": d.value,
                "ops_shared": e.value, "shared_passes": f.value}

    def side_levels(self, side):
        """Path-tree levels of a side: [(fused ops, states for all P paths)],
        level 0 being the shared prefix."""
        n = ctypes.c_int32()
        L.check(L.lib().hsf_side_levels(ctypes.c_void_p(self.handle), side, 0, ctypes.byref(n), None, None))
        ops = (ctypes.c_int64 * n.value)()
        st = (ctypes.c_int64 * n.value)()
        L.check(L.lib().hsf_side_levels(ctypes.c_void_p(self.handle), side, n.value, ctypes.byref(n), ops, st))
        return [(int(ops[i]), int(st[i])) for i in range(n.value)]

    def sweep_form(self, n_paths):
        """(tree, (tile qubits a, b)) of a sweep over n_paths paths."""
        t = ctypes.c_int32()
        q = (ctypes.c_int32 * 2)()
        L.check(L.lib().hsf_sweep_form(ctypes.c_void_p(self.handle), int(n_paths), ctypes.byref(t), q))
        return t.value == 1, (q[0], q[1])

    def uses_tree(self, n_paths):
        """Whether a sweep over n_paths paths runs level by level."""
        return self.sweep_form(n_paths)[0]

    # ------------------------------------------------------------ device ----
    def alloc_halves(self, n_paths, device="cuda"):
        A = torch.empty((n_paths, 1 << self.na), dtype=self.torch_dtype, device=device)
        B = torch.empty((n_paths, 1 << self.nb), dtype=self.torch_dtype, device=device)
        return A, B

    def run_paths(self, p_begin=0, p_end=None, psiA=None, psiB=None, ws=None, rows=None):
        """Half-states of paths [p_begin, p_end).  rows = (r0, r1): only side
        a's amplitudes r0 .. r1 - 1 are wanted (hsf_run_paths_rows)."""
        p_end = self.P if p_end is None else p_end
        if psiA is None and psiB is None:
            psiA, psiB = self.alloc_halves(p_end - p_begin)
        if rows is None:
            hsf_run_paths(self.handle, p_begin, p_end, psiA, psiB, ws)
        else:
            hsf_run_paths_rows(self.handle, p_begin, p_end, rows[0], rows[1], psiA, psiB, ws)
        return psiA, psiB

    def amplitudes_full(self, psiA, psiB, n_paths=None, rows=None, mode=None, out=None, accumulate=False,
                        ws=None):
        """Rows [r0, r1) of the path sum.  mode "bf16x3_split" reads the
        planes of the last split_operands call from ws (psiA and psiB then
        only give the device and the path count)."""
        n_paths = psiA.shape[0] if n_paths is None else n_paths
        r0, r1 = (0, 1 << self.na) if rows is None else rows
        mode = mode or ("c128" if self.dtype == "c128" else "f32")
        odt = torch.complex64 if mode in ("f32", "bf16x3", "bf16x3_split") else torch.complex128
        if out is None:
            out = torch.empty((r1 - r0, 1 << self.nb), dtype=odt, device=psiA.device)
        if mode == "bf16x3" and ws is None:
            nbytes = hsf_workspace_size(self.handle, 1, n_paths, L.SUM_MODE[mode])
            ws = torch.empty(nbytes, dtype=torch.uint8, device=psiA.device)
        if mode == "bf16x3_split" and ws is None:
            raise ValueError("mode bf16x3_split needs the workspace of split_operands")
        hsf_amplitudes_full(self.handle, psiA, psiB, n_paths, r0, r1, out, mode, accumulate, ws)
        return out

    def split_operands(self, psiA, psiB, n_paths=None, ws=None):
        """BF16 hi/lo planes of the first n_paths rows of both operands, for
        amplitudes_full(..., mode="bf16x3_split", ws=ws).  Returns ws."""
        n_paths = psiA.shape[0] if n_paths is None else n_paths
        if ws is None:
            nbytes = hsf_workspace_size(self.handle, 1, n_paths, L.SUM_MODE["bf16x3"])
            ws = torch.empty(nbytes, dtype=torch.uint8, device=psiA.device)
        hsf_split_operands(self.handle, psiA, psiB, n_paths, ws)
        return ws

    def amplitudes_bitstrings(self, psiA, psiB, x, n_paths=None, out=None, accumulate=False):
        n_paths = psiA.shape[0] if n_paths is None else n_paths
        if out is None:
            out = torch.zeros(x.numel(), dtype=torch.complex128, device=psiA.device)
        hsf_amplitudes_bitstrings(self.handle, psiA, psiB, n_paths, x, out, accumulate)
        return out

    def backward(self, x, chunk=None, grad=None, dl_dpsi=None, ws=None):
        """dL/dt for every parameter id (float64 tensor of n_params entries).
        x: device tensor of basis-state indices.  dl_dpsi: None for L =
        sum_j |psi(x_j)|^2, else complex128 cotangents dL/dRe psi(x_j) +
        i dL/dIm psi(x_j).  ws: a uint8 device workspace of at least
        workspace_backward(..., minimal=True) bytes (default: the preferred
        size)."""
        chunk = min(self.P, 256) if chunk is None else chunk
        if ws is None:
            ws = torch.empty(self.workspace_backward(x.numel(), chunk), dtype=torch.uint8, device=x.device)
        if grad is None:
            grad = torch.zeros(max(self.n_params, 1), dtype=torch.float64, device=x.device)
        hsf_backward(self.handle, x, grad, chunk, ws, dl_dpsi)
        return grad[:self.n_params]

    def workspace_backward(self, n_x, chunk=None, minimal=False):
        """Bytes of hsf_backward's workspace for n_x bitstrings: the preferred
        size, or the least it accepts (the shifted forward runs then go one
        copy per batch)."""
        chunk = min(self.P, 256) if chunk is None else chunk
        return hsf_workspace_size(self.handle, 4 if minimal else 2, chunk, n_x)

    def loss_device(self, x, chunk=None, amps=None):
        """L = sum_j |psi(x_j)|^2 as a one-entry float64 device tensor, from
        hsf_loss (every path chunk and the reduction inside the library);
        amps, if given, receives psi(x_j)."""
        chunk = min(self.P, 256) if chunk is None else chunk
        ws = torch.empty(hsf_workspace_size(self.handle, 3, chunk, x.numel()), dtype=torch.uint8, device=x.device)
        loss = torch.empty(1, dtype=torch.float64, device=x.device)
        hsf_loss(self.handle, x, loss, chunk, ws, amps)
        return loss

    def loss(self, x, chunk=None):
        """L = sum_j |psi(x_j)|^2 (forward only), as a float."""
        return float(self.loss_device(x, chunk).item())


def _with_params(circuit, theta):
    gs = []
    for g in circuit["gates"]:
        if g.get("param_id", -1) >= 0:
            g = dict(g)
            g["param"] = float(theta[g["param_id"]])
        gs.append(g)
    c = dict(circuit)
    c["gates"] = gs
    return c


class ProbabilityMass(torch.autograd.Function):
    """L(theta) = sum_j |<x_j| U(theta) |0>|^2 through joint-cut HSF.

    forward plans the circuit at the given angles and sums the bitstring
    amplitudes over all paths; backward calls hsf_backward."""

    @staticmethod
    def forward(ctx, theta, circuit, x, dtype="c64", chunk=None):
        th = theta.detach().double().cpu().numpy()
        plan = Plan(_with_params(circuit, th), dtype=dtype)
        ctx.plan, ctx.x, ctx.chunk = plan, x, chunk
        ctx.theta_device, ctx.theta_dtype = theta.device, theta.dtype
        return plan.loss_device(x, chunk)[0].to(theta.device)

    @staticmethod
    def backward(ctx, gout):
        # gradients come back on theta's device and in its dtype
        g = ctx.plan.backward(ctx.x, ctx.chunk)
        g = (gout.to(g.device, torch.float64) * g).to(device=ctx.theta_device, dtype=ctx.theta_dtype)
        return g, None, None, None, None


class Amplitudes(torch.autograd.Function):
    """psi(x_j; theta) = <x_j| U(theta) |0> through joint-cut HSF, as a
    complex128 tensor: forward from hsf_loss's amplitudes, backward passes
    the incoming cotangents to hsf_backward, so any real loss built on the
    amplitudes differentiates through the library."""

    @staticmethod
    def forward(ctx, theta, circuit, x, dtype="c64", chunk=None):
        th = theta.detach().double().cpu().numpy()
        plan = Plan(_with_params(circuit, th), dtype=dtype)
        ctx.plan, ctx.x, ctx.chunk = plan, x, chunk
        ctx.theta_device, ctx.theta_dtype = theta.device, theta.dtype
        amps = torch.empty(x.numel(), dtype=torch.complex128, device=x.device)
        plan.loss_device(x, chunk, amps)
        return amps

    @staticmethod
    def backward(ctx, gout):
        g = ctx.plan.backward(ctx.x, ctx.chunk, dl_dpsi=gout.to(ctx.x.device, torch.complex128).contiguous())
        return g.to(device=ctx.theta_device, dtype=ctx.theta_dtype), None, None, None, None


class Batch:
    """Many planned circuits run together (hsf_batch_*): batched LDS passes,
    one persistent path-sum launch, optionally replayed from a HIP graph."""

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle for p in self.plans])
        h = ctypes.c_void_p()
        L.check(L.lib().hsf_batch_create(arr, len(self.plans), ctypes.byref(h)))
        self.handle = h.value
        self._ws = {}

    def close(self):
        if getattr(self, "handle", None):
            L.lib().hsf_batch_destroy(ctypes.c_void_p(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, mode, device="cuda"):
        m = L.SUM_MODE[mode]
        if m not in self._ws:
            n = int(L.lib().hsf_batch_workspace_size(ctypes.c_void_p(self.handle), m))
            self._ws[m] = torch.empty(n, dtype=torch.uint8, device=device)
        return self._ws[m]

    def alloc_outputs(self, device="cuda"):
        return [torch.empty((1 << p.na, 1 << p.nb), dtype=torch.complex64, device=device) for p in self.plans]

    def _outs(self, outs):
        return (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])

    def run(self, outs, mode="bf16x3", graph=True):
        ws = self.workspace(mode, outs[0].device)
        L.check(L.lib().hsf_batch_run(ctypes.c_void_p(self.handle), self._outs(outs), L.SUM_MODE[mode],
                                      1 if graph else 0, _ptr(ws), ws.numel(), _stream(outs[0])))
        return outs

    def tune(self, outs, mode="bf16x3", cached=False):
        """Times the sweep policies and keeps the fastest (hsf_batch_tune);
        with cached=True a policy recorded for a batch of the same shapes in
        this process is applied instead when there is one."""
        if cached:
            pol = self.tuned_policy(mode)
            if pol >= 0:
                return pol
        ws = self.workspace(mode, outs[0].device)
        pol = ctypes.c_int32()
        L.check(L.lib().hsf_batch_tune(ctypes.c_void_p(self.handle), self._outs(outs), L.SUM_MODE[mode], _ptr(ws),
                                       ws.numel(), _stream(outs[0]), ctypes.byref(pol)))
        return pol.value

    def tuned_policy(self, mode="bf16x3"):
        """The policy recorded for this batch's shapes (applied to it), or -1
        (hsf_batch_tune_cached; host only)."""
        pol = ctypes.c_int32()
        L.check(L.lib().hsf_batch_tune_cached(ctypes.c_void_p(self.handle), L.SUM_MODE[mode], ctypes.byref(pol)))
        return pol.value
