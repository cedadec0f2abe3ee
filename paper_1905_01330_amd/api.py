"""Python entry points with the names of the C ABI (include/tn.h).

Each function checks nothing beyond what ctypes needs, allocates outputs and
workspaces with torch on the current device, and calls libtn.so on torch's
current stream.  All arithmetic runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L


def _dev(t):
    if not t.is_cuda:
        raise ValueError("tensors must live on the GPU (there is no CPU path)")
    return t


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def contract_between(a, b, axes_a, axes_b, out=None, prec="fp32", conj_a=False, conj_b=False):
    """Contract axes_a[i] of a with axes_b[i] of b (section III.B, flattened edges).

    Output axes: free axes of a (ascending) then free axes of b.  `out` may be
    any strided view of that shape (a permuted view fuses reorder_edges).
    Complex (complex64) operands take the complex path, with optional
    conjugation of either operand.
    """
    _dev(a), _dev(b)
    if a.is_complex() or b.is_complex():
        return _contract_c64(a, b, axes_a, axes_b, out, prec, conj_a, conj_b)
    if conj_a or conj_b:
        raise ValueError("conjugation applies to complex operands")
    axes_a = [int(x) % max(a.dim(), 1) for x in axes_a]
    axes_b = [int(x) % max(b.dim(), 1) for x in axes_b]
    if out is None:
        shape = [a.shape[i] for i in range(a.dim()) if i not in axes_a] + \
                [b.shape[j] for j in range(b.dim()) if j not in axes_b]
        out = torch.empty(shape, dtype=torch.float32, device=a.device)
    da, db, do = L.tensor_desc(a), L.tensor_desc(b), L.tensor_desc(out)
    # few outputs may be long sums, which split over workgroups with a small scratch
    ws = _workspace(L.REDUCE_WORKSPACE_BYTES, a.device) if out.numel() < 1024 else None
    L.check(L.lib().tn_contract_between(C.byref(da), C.byref(db), len(axes_a), L.int_array(axes_a),
                                        L.int_array(axes_b), C.byref(do),
                                        C.c_void_p(ws.data_ptr()) if ws is not None else None,
                                        ws.numel() if ws is not None else 0, L.prec_code(prec), L.stream_ptr()))
    return out


def _contract_c64(a, b, axes_a, axes_b, out, prec, conj_a, conj_b):
    if a.dtype != torch.complex64 or b.dtype != torch.complex64:
        raise TypeError("complex contractions take complex64 operands")
    axes_a = [int(x) % max(a.dim(), 1) for x in axes_a]
    axes_b = [int(x) % max(b.dim(), 1) for x in axes_b]
    if out is None:
        shape = [a.shape[i] for i in range(a.dim()) if i not in axes_a] + \
                [b.shape[j] for j in range(b.dim()) if j not in axes_b]
        out = torch.empty(shape, dtype=torch.complex64, device=a.device)
    da, db, do = L.tensor_desc(a), L.tensor_desc(b), L.tensor_desc(out)
    nbytes = C.c_size_t(0)
    L.check(L.lib().tn_contract_between_c64_workspace(C.byref(db), C.byref(nbytes)))
    ws = _workspace(nbytes.value, a.device)
    L.check(L.lib().tn_contract_between_c64(C.byref(da), C.byref(db), len(axes_a), L.int_array(axes_a),
                                            L.int_array(axes_b), int(bool(conj_a)), int(bool(conj_b)), C.byref(do),
                                            C.c_void_p(ws.data_ptr()), nbytes.value, L.prec_code(prec),
                                            L.stream_ptr()))
    return out


def mps_inner_complex(psi, phi, prec="fp32"):
    """<psi|phi> for complex64 chains as a device float64 tensor [Re m, Im m, s]
    with value m * exp(s) (psi's sites are conjugated)."""
    n = len(psi)
    dp, dq = L.tensor_array(psi), L.tensor_array(phi)
    nbytes = C.c_size_t(0)
    L.check(L.lib().tn_mps_inner_c64_workspace(n, dp, dq, C.byref(nbytes)))
    dev = psi[0].device
    ws = _workspace(nbytes.value, dev)
    out4 = torch.empty(4, dtype=torch.float64, device=dev)
    L.check(L.lib().tn_mps_inner_c64(n, dp, dq, C.c_void_p(out4.data_ptr()), C.c_void_p(ws.data_ptr()),
                                     nbytes.value, L.prec_code(prec), L.stream_ptr()))
    return out4[:3]


def tensordot(a, b, axes_a, axes_b, prec="fp32"):
    return contract_between(a, b, axes_a, axes_b, prec=prec)


def trace_edge(a, axis1, axis2, out=None):
    """Trace over two axes of one node (section III.A, trace edges)."""
    _dev(a)
    a1, a2 = int(axis1) % a.dim(), int(axis2) % a.dim()
    if out is None:
        shape = [a.shape[i] for i in range(a.dim()) if i not in (a1, a2)]
        out = torch.empty(shape, dtype=torch.float32, device=a.device)
    da, do = L.tensor_desc(a), L.tensor_desc(out)
    L.check(L.lib().tn_trace_edge(C.byref(da), a1, a2, C.byref(do), L.stream_ptr()))
    return out


def outer_product(a, b, out=None):
    """(A (x) B)[i..., j...] = A[i...] B[j...] (section III.B)."""
    _dev(a), _dev(b)
    if out is None:
        out = torch.empty(list(a.shape) + list(b.shape), dtype=torch.float32, device=a.device)
    da, db, do = L.tensor_desc(a), L.tensor_desc(b), L.tensor_desc(out)
    L.check(L.lib().tn_outer_product(C.byref(da), C.byref(db), C.byref(do), L.stream_ptr()))
    return out


def network_order(tensors, labels, method="greedy"):
    """A contraction order for contract_network and its pairwise flop count.

    method "greedy" (cheapest connected pair first) or "optimal" (exact
    minimum over contraction trees, up to 12 nodes per connected part).
    Reads only the shapes."""
    flat, offs = [], [0]
    for l in labels:
        flat.extend(int(x) for x in l)
        offs.append(len(flat))
    nodes = L.tensor_array(tensors)
    n_conn = sum(1 for x in flat if x >= 0) // 2 + 1
    order = (C.c_int32 * max(n_conn, 1))()
    n_order = C.c_int32(0)
    flops = C.c_double(0.0)
    code = {"greedy": 0, "optimal": 1}[method]
    L.check(L.lib().tn_network_order(len(tensors), nodes, L.int_array(flat), L.int_array(offs), code, order,
                                     C.byref(n_order), C.byref(flops)))
    return [int(order[i]) for i in range(n_order.value)], float(flops.value)


def contract_network(tensors, labels, order=None, out=None, prec="fp32"):
    """ncon (Appendix B): labels >= 0 connect, labels < 0 are outputs -1, -2, ...

    order: a list of connected labels, None (ascending labels), or "greedy" /
    "optimal" (network_order)."""
    for t in tensors:
        _dev(t)
    if isinstance(order, str):
        order = network_order(tensors, labels, order)[0]
    flat, offs = [], [0]
    for l in labels:
        flat.extend(int(x) for x in l)
        offs.append(len(flat))
    nodes = L.tensor_array(tensors)
    lab = L.int_array(flat)
    off = L.int_array(offs)
    order = list(order) if order is not None else []
    ordp = L.int_array(order)
    nbytes = C.c_size_t(0)
    L.check(L.lib().tn_contract_network_workspace(len(tensors), nodes, lab, off, len(order), ordp, C.byref(nbytes)))
    if out is None:
        dims = {}
        for t, l in zip(tensors, labels):
            for ax, x in enumerate(l):
                dims[int(x)] = t.shape[ax]
        n_out = sum(1 for x in flat if x < 0)
        out = torch.empty([dims[-(q + 1)] for q in range(n_out)], dtype=torch.float32, device=tensors[0].device)
    ws = _workspace(nbytes.value, tensors[0].device)
    do = L.tensor_desc(out)
    L.check(L.lib().tn_contract_network(len(tensors), nodes, lab, off, len(order), ordp, C.byref(do),
                                        C.c_void_p(ws.data_ptr()), nbytes.value, L.prec_code(prec), L.stream_ptr()))
    return out


def mps_inner(psi, phi, prec="fp32"):
    """<psi|phi> as a device float64 tensor [m, s] with value m * exp(s)."""
    n = len(psi)
    dp, dq = L.tensor_array(psi), L.tensor_array(phi)
    nbytes = C.c_size_t(0)
    L.check(L.lib().tn_mps_inner_workspace(n, dp, dq, C.byref(nbytes)))
    dev = psi[0].device
    ws = _workspace(nbytes.value, dev)
    out2 = torch.empty(2, dtype=torch.float64, device=dev)
    L.check(L.lib().tn_mps_inner(n, dp, dq, C.c_void_p(out2.data_ptr()), C.c_void_p(ws.data_ptr()), nbytes.value,
                                 L.prec_code(prec), L.stream_ptr()))
    return out2


class BatchedInner:
    """Prepared uneven batch: descriptors are built and the work tables
    uploaded once; run() only launches kernels, so it can be repeated and
    recorded in a Graph."""

    def __init__(self, chains, prec="fp32"):
        self.psi = [t for p, _ in chains for t in p]
        self.phi = [t for _, q in chains for t in q]
        offs = [0]
        for p, _ in chains:
            offs.append(offs[-1] + len(p))
        self.n = len(chains)
        self.offs = L.int_array(offs)
        self.dp, self.dq = L.tensor_array(self.psi), L.tensor_array(self.phi)
        nbytes = C.c_size_t(0)
        L.check(L.lib().tn_mps_inner_batched_workspace(self.n, self.offs, self.dp, self.dq, C.byref(nbytes)))
        dev = self.psi[0].device
        self.nbytes = nbytes.value
        self.ws = _workspace(self.nbytes, dev)
        self.out2 = torch.empty((self.n, 2), dtype=torch.float64, device=dev)
        self.prec = L.prec_code(prec)
        L.check(L.lib().tn_mps_inner_batched_upload(self.n, self.offs, self.dp, self.dq, C.c_void_p(self.ws.data_ptr()),
                                                    self.nbytes, L.stream_ptr()))

    def run(self):
        L.check(L.lib().tn_mps_inner_batched_launch(self.n, self.offs, self.dp, self.dq,
                                                    C.c_void_p(self.out2.data_ptr()), C.c_void_p(self.ws.data_ptr()),
                                                    self.nbytes, self.prec, L.stream_ptr()))
        return self.out2


class Graph:
    """A sequence of library calls recorded once as a HIP graph and replayed.

    fn runs once eagerly on a side stream (so workspaces and tile choices
    exist), then once under stream capture.  Calls that only launch kernels
    can be recorded: contract_between, trace_edge, outer_product,
    contract_network, mps_inner, BatchedInner.run, EnvSweep.run and the
    classifier's forward and backward (the tile tuner never times
    candidates while a stream is capturing).  Tensors that fn allocates come
    from the graph's memory pool and are rewritten by every replay.
    """

    def __init__(self, fn):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fn()
        torch.cuda.current_stream().wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.result = fn()

    def replay(self):
        self.graph.replay()
        return self.result


def mps_inner_batched(chains, prec="fp32"):
    """Inner products of many (psi, phi) chains of uneven length and bond dimension."""
    return BatchedInner(chains, prec).run()


class EnvSweep:
    """Prepared MPS-MPO-MPS environment sweep (workspace and outputs allocated once)."""

    def __init__(self, psi, mpo, left=True, right=True, store=True, prec="fp32"):
        self.n = len(psi)
        self.psi, self.mpo = psi, mpo
        self.dp = L.tensor_array(psi)
        self.dw = L.tensor_array(mpo)
        nbytes = C.c_size_t(0)
        L.check(L.lib().tn_mps_env_sweep_workspace(self.n, self.dp, self.dw, C.byref(nbytes)))
        dev = psi[0].device
        self.nbytes = nbytes.value
        self.ws = _workspace(self.nbytes, dev)
        dims = [1] + [int(a.shape[2]) for a in psi]
        ws_ = [1] + [int(w.shape[1]) for w in mpo]
        self.which = (1 if left else 0) | (2 if right else 0)
        self.L = [torch.empty((dims[k], ws_[k], dims[k]), device=dev) for k in range(self.n + 1)] if (store and left) else None
        self.R = [torch.empty((dims[k], ws_[k], dims[k]), device=dev) for k in range(self.n + 1)] if (store and right) else None
        self.dL = L.tensor_array(self.L) if self.L else None
        self.dR = L.tensor_array(self.R) if self.R else None
        self.energy = torch.zeros(2, dtype=torch.float64, device=dev)
        self.prec = L.prec_code(prec)

    def run(self):
        L.check(L.lib().tn_mps_env_sweep(self.n, self.dp, self.dw, self.dL, self.dR, C.c_void_p(self.energy.data_ptr()),
                                         self.which, C.c_void_p(self.ws.data_ptr()), self.nbytes, self.prec,
                                         L.stream_ptr()))
        return self


def mps_env_sweep(psi, mpo, left=True, right=True, store=True, prec="fp32"):
    """Left/right environments of <psi|H|psi>; returns (Ls, Rs, energy[L_N, R_0])."""
    s = EnvSweep(psi, mpo, left, right, store, prec).run()
    return s.L, s.R, s.energy


def mps_left_canonicalize(sites):
    """In-place FP64 left-canonical gauge (Householder QR); returns the log-norm (device)."""
    n = len(sites)
    ds = L.tensor_array(sites)
    nbytes = C.c_size_t(0)
    L.check(L.lib().tn_mps_left_canonicalize_workspace(n, ds, C.byref(nbytes)))
    dev = sites[0].device
    ws = _workspace(nbytes.value, dev)
    lognorm = torch.empty(1, dtype=torch.float64, device=dev)
    L.check(L.lib().tn_mps_left_canonicalize(n, ds, C.c_void_p(lognorm.data_ptr()), C.c_void_p(ws.data_ptr()),
                                             nbytes.value, L.stream_ptr()))
    return lognorm


def _split(t, left_axes, right_axes, max_singular_values, max_truncation_err, full):
    _dev(t)
    left_axes = [int(x) % t.dim() for x in left_axes]
    right_axes = [int(x) % t.dim() for x in right_axes]
    if sorted(left_axes + right_axes) != list(range(t.dim())):
        raise ValueError("left_axes + right_axes must list every axis of the node once")
    view = t.permute(*(left_axes + right_axes))
    n_left = len(left_axes)
    da = L.tensor_desc(view)
    nbytes = C.c_size_t(0)
    L.check(L.lib().tn_split_node_workspace(C.byref(da), n_left, C.byref(nbytes)))
    ws = _workspace(nbytes.value, t.device)
    k, sweeps = C.c_int32(0), C.c_int32(0)
    L.check(L.lib().tn_split_node_decompose(C.byref(da), n_left,
                                            -1 if max_singular_values is None else int(max_singular_values),
                                            -1.0 if max_truncation_err is None else float(max_truncation_err),
                                            C.byref(k), C.byref(sweeps), C.c_void_p(ws.data_ptr()), nbytes.value,
                                            L.stream_ptr()))
    k = k.value
    ldims = [view.shape[i] for i in range(n_left)]
    rdims = [view.shape[i] for i in range(n_left, view.dim())]
    kmax = min(int(torch.tensor(ldims).prod()), int(torch.tensor(rdims).prod()))
    left = torch.empty(ldims + [k], dtype=t.dtype, device=t.device)
    right = torch.empty([k] + rdims, dtype=t.dtype, device=t.device)
    trun = torch.empty(kmax - k, dtype=t.dtype, device=t.device)
    dl, dr = L.tensor_desc(left), L.tensor_desc(right)
    dt = L.tensor_desc(trun) if kmax > k else None
    tp = C.byref(dt) if dt is not None else None
    if full:
        s = torch.empty((k, k), dtype=t.dtype, device=t.device)
        ds = L.tensor_desc(s)
        L.check(L.lib().tn_split_node_full_svd(C.byref(da), n_left, k, C.byref(dl), C.byref(ds), C.byref(dr), tp,
                                               C.c_void_p(ws.data_ptr()), nbytes.value, L.stream_ptr()))
        return left, s, right, trun
    L.check(L.lib().tn_split_node(C.byref(da), n_left, k, C.byref(dl), C.byref(dr), tp, C.c_void_p(ws.data_ptr()),
                                  nbytes.value, L.stream_ptr()))
    return left, right, trun


def split_node(t, left_axes, right_axes, max_singular_values=None, max_truncation_err=None):
    """Section III.B "Node Splitting": (U sqrt(S), sqrt(S) V^T, trun_err) of the
    node read as a matrix of its left and right axes, truncated as in
    Appendix A.  The decomposition synchronises the current stream."""
    return _split(t, left_axes, right_axes, max_singular_values, max_truncation_err, False)


def split_node_full_svd(t, left_axes, right_axes, max_singular_values=None, max_truncation_err=None):
    """(U, S as a diagonal [k, k] node, V^T, trun_err); see split_node."""
    return _split(t, left_axes, right_axes, max_singular_values, max_truncation_err, True)


# ---------------------------------------------------------------------------
# two-site DMRG


def _dmrg_descs(L_, R_, W1, W2, theta):
    return [L.tensor_desc(x) for x in (L_, R_, W1, W2, theta)]


def dmrg_apply_heff(L_, R_, W1, W2, theta, out=None, prec="fp32", krylov=2):
    """H_eff theta for the two-site tensor theta[a, s1, s2, b]."""
    if out is None:
        out = torch.empty_like(theta)
    dl, dr, d1, d2, dt = _dmrg_descs(L_, R_, W1, W2, theta)
    nbytes = C.c_size_t(0)
    L.check(L.lib().tn_dmrg_workspace(C.byref(dl), C.byref(dr), C.byref(d1), C.byref(d2), C.byref(dt), krylov,
                                      C.byref(nbytes)))
    ws = _workspace(nbytes.value, theta.device)
    do = L.tensor_desc(out)
    L.check(L.lib().tn_dmrg_apply_heff(C.byref(dl), C.byref(dr), C.byref(d1), C.byref(d2), C.byref(dt), C.byref(do),
                                       C.c_void_p(ws.data_ptr()), nbytes.value, L.prec_code(prec), L.stream_ptr()))
    return out


def dmrg_eigensolve(L_, R_, W1, W2, theta, krylov=24, restarts=3, prec="fp32"):
    """Lowest eigenpair of H_eff by Lanczos; theta (contiguous) is the start and
    becomes the eigenvector.  Returns a device float64 tensor [energy, residual]."""
    dl, dr, d1, d2, dt = _dmrg_descs(L_, R_, W1, W2, theta)
    nbytes = C.c_size_t(0)
    L.check(L.lib().tn_dmrg_workspace(C.byref(dl), C.byref(dr), C.byref(d1), C.byref(d2), C.byref(dt), krylov,
                                      C.byref(nbytes)))
    ws = _workspace(nbytes.value, theta.device)
    out2 = torch.empty(2, dtype=torch.float64, device=theta.device)
    L.check(L.lib().tn_dmrg_eigensolve(C.byref(dl), C.byref(dr), C.byref(d1), C.byref(d2), C.byref(dt), krylov,
                                       restarts, C.c_void_p(out2.data_ptr()), C.c_void_p(ws.data_ptr()), nbytes.value,
                                       L.prec_code(prec), L.stream_ptr()))
    return out2


def dmrg_two_site_update(L_, R_, W1, W2, theta, chi_max=None, direction="right", krylov=24, restarts=3,
                         prec="fp32", max_truncation_err=None):
    """One two-site DMRG update: the lowest eigenvector of H_eff (theta is the
    starting vector and is overwritten), split with truncation.  direction
    "right": (U, S V^T); "left": (U S, V^T).  Returns (energy/residual device
    tensor, a_left, a_right, trun_err)."""
    out2 = dmrg_eigensolve(L_, R_, W1, W2, theta, krylov, restarts, prec)
    u, s, vt, trun = split_node_full_svd(theta, [0, 1], [2, 3], chi_max, max_truncation_err)
    if direction == "right":
        return out2, u, contract_between(s, vt, [1], [0], prec="fp32"), trun
    return out2, contract_between(u, s, [2], [0], prec="fp32"), vt, trun


_ENV_LEFT = ([[1, 2, 3], [3, 4, -3], [2, -2, 5, 4], [1, 5, -1]], [3, 2, 4, 1, 5])
_ENV_RIGHT = ([[1, 2, 3], [-3, 4, 3], [-2, 2, 5, 4], [-1, 5, 1]], [3, 2, 4, 1, 5])


def _theta_of(a, b, prec):
    return contract_between(a, b, [2], [0], prec=prec).contiguous()


def dmrg(mpo, psi, chi_max, sweeps=2, krylov=24, restarts=2, prec="fp32"):
    """Two-site DMRG for the ground state of an MPO (lists of device FP32
    tensors).  psi must be left-canonical (tn_mps_left_canonicalize gives
    one); it is updated in place, sweeping right to left, then left to right.
    Environments are updated with tn_contract_network steps.  Returns the
    energy after every update (a host list) and psi."""
    n = len(psi)
    ls, _, _ = mps_env_sweep(psi, mpo, left=True, right=False, store=True, prec=prec)
    rs = [None] * (n + 1)
    rs[n] = torch.ones((1, 1, 1), device=psi[0].device)
    energies = []
    for _ in range(sweeps):
        for k in range(n - 2, -1, -1):
            th = _theta_of(psi[k], psi[k + 1], prec)
            out2, a, b, _ = dmrg_two_site_update(ls[k], rs[k + 2], mpo[k], mpo[k + 1], th, chi_max, "left",
                                                 krylov, restarts, prec)
            psi[k], psi[k + 1] = a, b
            rs[k + 1] = contract_network([rs[k + 2], b, mpo[k + 1], b], _ENV_RIGHT[0], order=_ENV_RIGHT[1],
                                         prec=prec)
            energies.append(float(out2[0].cpu()))
        for k in range(0, n - 1):
            th = _theta_of(psi[k], psi[k + 1], prec)
            out2, a, b, _ = dmrg_two_site_update(ls[k], rs[k + 2], mpo[k], mpo[k + 1], th, chi_max, "right",
                                                 krylov, restarts, prec)
            psi[k], psi[k + 1] = a, b
            ls[k + 1] = contract_network([ls[k], a, mpo[k], a], _ENV_LEFT[0], order=_ENV_LEFT[1], prec=prec)
            energies.append(float(out2[0].cpu()))
    return energies, psi


def tune(cache_path=None, level: int = 1):
    """Tile autotuner level (0 heuristic, 1 quick, 2 full) and, optionally, a
    text file that persists the tile choices across processes."""
    path = None if cache_path is None else str(cache_path).encode()
    L.check(L.lib().tn_tune(path, int(level)))


def tune_set_level(level: int):
    L.check(L.lib().tn_tune_set_level(int(level)))


def tune_force_config(cfg: int):
    L.check(L.lib().tn_tune_force_config(int(cfg)))


def tune_force_grouped_config(cfg: int):
    """Pin the tile of the uneven batched inner product's site steps (-1: per-step choice)."""
    L.check(L.lib().tn_tune_force_grouped_config(int(cfg)))


def tune_last_choice() -> int:
    return int(L.lib().tn_tune_last_choice())


def tune_num_configs() -> int:
    return int(L.lib().tn_tune_num_configs())


def measure_split_mfma_rate(out, n_steps: int = 64, zero_operands: bool = False):
    """Launch the split-BF16 term-product rate measurement on the current
    stream (tn_measure_split_mfma_rate); out: CUDA float32 tensor of 131072
    elements."""
    if out.dtype != torch.float32 or not out.is_cuda or out.numel() < 131072:
        raise ValueError("out must be a CUDA float32 tensor of at least 131072 elements")
    L.check(L.lib().tn_measure_split_mfma_rate(int(n_steps), int(bool(zero_operands)), out.data_ptr(), L.stream_ptr()))


# ---------------------------------------------------------------------------
# MPS classifier (section IV.A)


class MPSClassifier:
    """Prepared classifier evaluation: workspace and checkpoints allocated once.

    sites: list of contiguous float32 device tensors [D_k, 2, D_{k+1}] with the
    label site [chi, 2, n_labels, chi]; pixels [B, N] in [0, 1].
    """

    def __init__(self, n_sites, label_site, n_labels, chi, batch, ckpt_every=28, prec="fp32", device="cuda:0"):
        self.n, self.c, self.L, self.chi, self.B, self.E = n_sites, label_site, n_labels, chi, batch, ckpt_every
        self.prec = L.prec_code(prec)
        nb = C.c_size_t(0)
        L.check(L.lib().tn_mps_classifier_workspace(n_sites, label_site, n_labels, batch, chi, ckpt_every, C.byref(nb)))
        self.nbytes = nb.value
        self.ws = _workspace(self.nbytes, device)
        nf = C.c_int64(0)
        L.check(L.lib().tn_mps_classifier_ckpt_shape(n_sites, label_site, batch, chi, ckpt_every, C.byref(nf)))
        self.ckpt = torch.empty(max(nf.value, 1), dtype=torch.float32, device=device)

    def forward(self, sites, pixels, logits=None):
        if logits is None:
            logits = torch.empty((self.B, self.L), dtype=torch.float32, device=pixels.device)
        ds, dp, dl = L.tensor_array(sites), L.tensor_desc(pixels), L.tensor_desc(logits)
        L.check(L.lib().tn_mps_classifier_forward(self.n, self.c, self.L, ds, C.byref(dp), C.byref(dl),
                                                  C.c_void_p(self.ckpt.data_ptr()), self.E,
                                                  C.c_void_p(self.ws.data_ptr()), self.nbytes, self.prec,
                                                  L.stream_ptr()))
        return logits

    def backward(self, sites, pixels, dlogits, dsites=None):
        if dsites is None:
            dsites = [torch.empty_like(s) for s in sites]
        ds, dp, dg, dd = L.tensor_array(sites), L.tensor_desc(pixels), L.tensor_desc(dlogits), L.tensor_array(dsites)
        L.check(L.lib().tn_mps_classifier_backward(self.n, self.c, self.L, ds, C.byref(dp),
                                                   C.c_void_p(self.ckpt.data_ptr()), self.E, C.byref(dg), dd,
                                                   C.c_void_p(self.ws.data_ptr()), self.nbytes, self.prec,
                                                   L.stream_ptr()))
        return dsites


def softmax_xent(logits, labels):
    """Batch-mean softmax cross-entropy and its gradient with respect to the logits."""
    B = logits.shape[0]
    loss = torch.empty(1, dtype=torch.float64, device=logits.device)
    dlogits = torch.empty_like(logits)
    ws = _workspace(8 * B, logits.device)
    dl, dd = L.tensor_desc(logits), L.tensor_desc(dlogits)
    L.check(L.lib().tn_softmax_xent(C.byref(dl), C.c_void_p(labels.data_ptr()), B, C.c_void_p(loss.data_ptr()),
                                    C.byref(dd), C.c_void_p(ws.data_ptr()), 8 * B, L.stream_ptr()))
    return loss, dlogits


class ClassifierFunction(torch.autograd.Function):
    """logits = f(sites; pixels) with the library's adjoint as the backward.

    Use as ClassifierFunction.apply(model, pixels, *sites) where model is an
    MPSClassifier sized for the batch; the forward keeps the checkpoints the
    backward recomputes from.
    """

    @staticmethod
    def forward(ctx, model, pixels, *sites):
        sites = [s.contiguous() for s in sites]
        logits = model.forward(sites, pixels)
        ctx.model = model
        ctx.save_for_backward(pixels, *sites)
        return logits

    @staticmethod
    def backward(ctx, dlogits):
        pixels, *sites = ctx.saved_tensors
        dsites = ctx.model.backward(sites, pixels, dlogits.contiguous())
        return (None, None, *dsites)
