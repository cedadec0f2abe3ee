"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects invalid calls before anything is launched (so these run
without a GPU: the data pointers below are never dereferenced)."""
import ctypes as C
import os
import re

import pytest

from paper_1905_01330_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 1 << 40   # a plausible device address; validation never touches it


def header_functions():
    txt = open(os.path.join(ROOT, "include", "tn.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tn_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    lib = L.lib()
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), f"{n} declared in tn.h but not exported"
    for n in L._PROTOS:
        assert n in names, f"binding names {n} which tn.h does not declare"


def test_version_and_status_strings():
    lib = L.lib()
    assert b"gfx950" in lib.tn_version()
    assert lib.tn_status_string(0) == b"ok"
    assert lib.tn_status_string(-2) == b"shape mismatch"
    assert lib.tn_status_string(-5) == b"output aliases an input"


def desc(shape, base, strides=None, dtype=L.F32):
    d = L.TnTensor()
    d.data = base
    d.dtype = dtype
    d.rank = len(shape)
    if strides is None:
        strides, st = [], 1
        for s in reversed(shape):
            strides.insert(0, st)
            st *= s
    for i, (s, t) in enumerate(zip(shape, strides)):
        d.shape[i] = s
        d.stride[i] = t
    return d


def contract(a, b, axes_a, axes_b, out, prec=0):
    return L.lib().tn_contract_between(C.byref(a), C.byref(b), len(axes_a), L.int_array(axes_a),
                                       L.int_array(axes_b), C.byref(out), None, 0, prec, None)


A0, B0, O0 = FAKE, FAKE + (1 << 30), FAKE + (2 << 30)


def test_contract_rejects_mismatched_dims():
    r = contract(desc([3, 4], A0), desc([5, 6], B0), [1], [0], desc([3, 6], O0))
    assert r == -2
    assert b"differ" in L.lib().tn_last_error()


def test_contract_rejects_bad_axes():
    assert contract(desc([3, 4], A0), desc([4, 6], B0), [2], [0], desc([3, 6], O0)) == -1
    assert contract(desc([4, 4], A0), desc([4, 4], B0), [0, 0], [0, 1], desc([], O0)) == -1


def test_contract_rejects_wrong_output_shape():
    assert contract(desc([3, 4], A0), desc([4, 6], B0), [1], [0], desc([6, 3], O0)) == -2
    assert contract(desc([3, 4], A0), desc([4, 6], B0), [1], [0], desc([3, 6, 1], O0)) == -2


def test_contract_rejects_aliasing_and_overlapping_output():
    assert contract(desc([3, 4], A0), desc([4, 6], B0), [1], [0], desc([3, 6], A0 + 8)) == -5
    assert contract(desc([3, 4], A0), desc([4, 6], B0), [1], [0], desc([3, 6], O0, [1, 1])) == -1


def test_contract_rejects_unknown_precision_and_dtype():
    assert contract(desc([3, 4], A0), desc([4, 6], B0), [1], [0], desc([3, 6], O0), prec=7) == -3
    assert contract(desc([3, 4], A0, dtype=L.F64), desc([4, 6], B0), [1], [0], desc([3, 6], O0)) == -3


def test_contract_rejects_null_and_bad_shapes():
    lib = L.lib()
    b = desc([4, 6], B0)
    o = desc([3, 6], O0)
    assert lib.tn_contract_between(None, C.byref(b), 0, None, None, C.byref(o), None, 0, 0, None) == -1
    # a byte count without a buffer
    assert lib.tn_contract_between(C.byref(desc([3, 4], A0)), C.byref(desc([4, 6], B0)), 1, L.int_array([1]),
                                   L.int_array([0]), C.byref(o), None, 64, 0, None) == -1
    assert contract(desc([3, 0], A0), desc([4, 6], B0), [], [], desc([3, 0, 4, 6], O0)) == -1
    assert contract(desc([3, 4], 0), desc([4, 6], B0), [1], [0], desc([3, 6], O0)) == -1


def test_trace_validation():
    lib = L.lib()
    a = desc([3, 4, 3], A0)
    out = desc([4], O0)
    assert lib.tn_trace_edge(C.byref(a), 0, 1, C.byref(out), None) == -2
    assert lib.tn_trace_edge(C.byref(a), 0, 0, C.byref(out), None) == -1
    bad = desc([5], O0)
    assert lib.tn_trace_edge(C.byref(a), 0, 2, C.byref(bad), None) == -2


def test_outer_validation():
    lib = L.lib()
    a, b = desc([2, 3], A0), desc([4, 5, 6], B0)
    assert lib.tn_outer_product(C.byref(a), C.byref(b), C.byref(desc([2, 3, 4, 5], O0)), None) == -2
    assert lib.tn_outer_product(C.byref(a), C.byref(b), C.byref(desc([2, 3, 4, 5, 6], A0)), None) == -5


def _network(tensors, labels, order=None):
    flat, offs = [], [0]
    for l in labels:
        flat += l
        offs.append(len(flat))
    nodes = (L.TnTensor * len(tensors))(*tensors)
    order = order or []
    nb = C.c_size_t(0)
    r = L.lib().tn_contract_network_workspace(len(tensors), nodes, L.int_array(flat), L.int_array(offs), len(order),
                                              L.int_array(order), C.byref(nb))
    return r, nb.value


def test_network_workspace_and_validation():
    # chain a(2,3) - b(3,4) - c(4,5): one intermediate of 2x4 floats (one
    # 256-byte slot), then the scratch of the split rank-0/1 sums, then the
    # k-slice partials: 64 results of the largest step (2x5 floats; 3x5
    # when b and c are contracted first)
    ts = [desc([2, 3], A0), desc([3, 4], B0), desc([4, 5], O0)]
    r, nb = _network(ts, [[-1, 0], [0, 1], [1, -2]])
    assert r == 0 and nb == 256 + L.REDUCE_WORKSPACE_BYTES + 64 * 10 * 4
    r, nb = _network(ts, [[-1, 0], [0, 1], [1, -2]], order=[1, 0])
    assert r == 0 and nb == 256 + L.REDUCE_WORKSPACE_BYTES + 64 * 15 * 4
    assert _network(ts, [[-1, 0], [0, 1], [2, -2]])[0] == -1         # label 2 appears once
    assert _network(ts, [[-1, 0], [0, -1], [1, -2]])[0] == -1        # open label repeated
    assert _network(ts, [[-1, 0], [1, 0], [1, -2]])[0] == -2         # dims 3 vs 4 on label 0 ... and 1
    assert _network(ts, [[-1, 0], [0, 1], [1, -3]])[0] == -1         # outputs must be -1..-n
    assert _network(ts, [[-1, 0], [0, 1], [1, -2]], order=[0])[0] == -1  # incomplete order


def test_mps_workspace_queries():
    lib = L.lib()
    dims = [1, 2, 4, 2, 1]
    psi = (L.TnTensor * 4)(*[desc([dims[k], 2, dims[k + 1]], A0 + k * 4096) for k in range(4)])
    nb = C.c_size_t(0)
    assert lib.tn_mps_inner_workspace(4, psi, psi, C.byref(nb)) == 0 and nb.value > 0
    mpo_shapes = [[1, 3, 2, 2], [3, 3, 2, 2], [3, 3, 2, 2], [3, 1, 2, 2]]
    mpo = (L.TnTensor * 4)(*[desc(s, B0 + k * 4096) for k, s in enumerate(mpo_shapes)])
    assert lib.tn_mps_env_sweep_workspace(4, psi, mpo, C.byref(nb)) == 0 and nb.value > 0
    bad = (L.TnTensor * 4)(*[desc([dims[k], 2, dims[k + 1] + (k == 1)], A0 + k * 4096) for k in range(4)])
    assert lib.tn_mps_inner_workspace(4, bad, psi, C.byref(nb)) == -2
    bad_mpo = (L.TnTensor * 4)(*[desc(s, B0 + k * 4096) for k, s in enumerate([[1, 3, 2, 2], [3, 2, 2, 2], [3, 3, 2, 2], [3, 1, 2, 2]])])
    assert lib.tn_mps_env_sweep_workspace(4, psi, bad_mpo, C.byref(nb)) == -2
    f64 = (L.TnTensor * 4)(*[desc([dims[k], 2, dims[k + 1]], A0 + k * 4096, dtype=L.F64) for k in range(4)])
    assert lib.tn_mps_left_canonicalize_workspace(4, f64, C.byref(nb)) == 0 and nb.value > 0
    assert lib.tn_mps_left_canonicalize_workspace(4, psi, C.byref(nb)) == -3    # needs FP64
    offs = L.int_array([0, 4, 8])
    both = (L.TnTensor * 8)(*(list(psi) + list(psi)))
    assert lib.tn_mps_inner_batched_workspace(2, offs, both, both, C.byref(nb)) == 0 and nb.value > 0


def test_workspace_too_small_is_reported_before_launch():
    lib = L.lib()
    dims = [1, 2, 4, 2, 1]
    psi = (L.TnTensor * 4)(*[desc([dims[k], 2, dims[k + 1]], A0 + k * 4096) for k in range(4)])
    r = lib.tn_mps_inner(4, psi, psi, C.c_void_p(O0), C.c_void_p(B0), 16, 0, None)
    assert r == -4


def test_tuner_controls():
    lib = L.lib()
    n = lib.tn_tune_num_configs()
    assert n >= 4
    assert lib.tn_tune_force_config(n) == -1
    assert lib.tn_tune_force_config(-1) == 0
    assert lib.tn_tune_force_grouped_config(5) == -1
    assert lib.tn_tune_force_grouped_config(-2) == -1
    assert lib.tn_tune_force_grouped_config(-1) == 0
    assert lib.tn_tune_set_level(5) == -1
    assert lib.tn_tune_set_level(0) == 0


def test_mfma_rate_measurement_validation():
    """The rate measurement rejects a NULL output and an odd or non-positive
    step count before it launches anything."""
    import ctypes as C
    lib = L.lib()
    buf = C.c_void_p(0x1000)   # never dereferenced: every call below fails validation first
    assert lib.tn_measure_split_mfma_rate(64, 0, None, None) == -1
    assert lib.tn_measure_split_mfma_rate(63, 0, buf, None) == -1
    assert lib.tn_measure_split_mfma_rate(0, 1, buf, None) == -1
    assert lib.tn_measure_split_mfma_rate(-2, 0, buf, None) == -1


def test_binding_refuses_cpu_tensors():
    import torch
    import paper_1905_01330_amd as tn

    with pytest.raises(ValueError):
        tn.contract_between(torch.ones(2), torch.ones(2), [0], [0])


def test_reduce_workspace_constant_matches_header():
    import os
    import re

    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "tn.h")).read()
    m = re.search(r"#define\s+TN_REDUCE_WORKSPACE_BYTES\s+(\d+)", hdr)
    assert m and int(m.group(1)) == L.REDUCE_WORKSPACE_BYTES


def test_tune_levels_and_cache_file(tmp_path):
    lib = L.lib()
    assert lib.tn_tune(None, 3) == -1
    assert lib.tn_tune(None, -1) == -1
    assert lib.tn_tune(str(tmp_path / "no" / "such" / "dir" / "c.txt").encode(), 1) == -6
    path = tmp_path / "tiles.txt"
    # a cache with valid entries (a whole GEMM, a tile in two k-slices), an
    # out-of-range tile, an out-of-range slice count and a malformed line
    path.write_text("384 320 256 1 1 2 1 2 111 -> 3\n256 768 512 1 1 1 0 2 1111 -> 114\n"
                    "1 2 3 4 5 6 7 8 9 -> 999\n1 2 3 4 5 6 7 8 9 -> 714\nnot a line\n")
    assert lib.tn_tune(str(path).encode(), 2) == 0
    assert path.read_text().startswith("384 320 256")   # loading never rewrites the file
    assert lib.tn_tune(None, 0) == 0
    assert lib.tn_tune_set_level(2) == -1
    assert lib.tn_tune_set_level(0) == 0


def test_noalloc_network_rejects_networks_beyond_its_scratch():
    """a[8192, 8192] . b[8192, 8192] . c[8192] contracted a-b first: the
    8192 x 8192 intermediate (256 MiB) exceeds the 128 MiB static scratch."""
    lib = L.lib()
    n = 8192
    nodes = (L.TnTensor * 3)()
    nodes[0], nodes[1], nodes[2] = desc([n, n], A0), desc([n, n], B0), desc([n], O0)
    labels = L.int_array([-1, 1, 1, 2, 2])
    offs = L.int_array([0, 2, 4, 5])
    order = L.int_array([1, 2])
    out = desc([n], FAKE + (3 << 30))
    nbytes = C.c_size_t(0)
    assert lib.tn_contract_network_workspace(3, nodes, labels, offs, 2, order, C.byref(nbytes)) == 0
    assert nbytes.value > (128 << 20)
    r = lib.tn_contract_network_noalloc(3, nodes, labels, offs, 2, order, C.byref(out), 0, None)
    assert r == -3
    assert b"static scratch" in lib.tn_last_error()


def test_split_node_validation_before_launch():
    lib = L.lib()
    a = desc([6, 4, 5], A0, dtype=L.F64)
    nbytes = C.c_size_t(0)
    assert lib.tn_split_node_workspace(C.byref(a), 0, C.byref(nbytes)) == -1      # no left legs
    assert lib.tn_split_node_workspace(C.byref(a), 3, C.byref(nbytes)) == -1      # no right legs
    assert lib.tn_split_node_workspace(C.byref(a), 1, C.byref(nbytes)) == 0 and nbytes.value > 0
    k = C.c_int32(0)
    ws = B0
    assert lib.tn_split_node_decompose(C.byref(a), 1, -1, -1.0, C.byref(k), None, ws, 0, None) == -4
    assert lib.tn_split_node_decompose(C.byref(a), 1, -1, float("nan"), C.byref(k), None, ws, nbytes.value, None) == -1
    # writers: k in 1..min(6, 20) and the new bond's extent
    left, right = desc([6, 3], O0, dtype=L.F64), desc([3, 4, 5], O0 + (1 << 20), dtype=L.F64)
    assert lib.tn_split_node(C.byref(a), 1, 7, C.byref(left), C.byref(right), None, ws, nbytes.value, None) == -1
    assert lib.tn_split_node(C.byref(a), 1, 2, C.byref(left), C.byref(right), None, ws, nbytes.value, None) == -2
    tr = desc([2], O0 + (2 << 20), dtype=L.F64)    # 6 - 3 = 3 dropped values expected
    assert lib.tn_split_node(C.byref(a), 1, 3, C.byref(left), C.byref(right), C.byref(tr), ws, nbytes.value, None) == -2
    bad_dtype = desc([6, 3], O0, dtype=L.F32)
    assert lib.tn_split_node(C.byref(a), 1, 3, C.byref(bad_dtype), C.byref(right), None, ws, nbytes.value, None) == -3
    overlap = desc([3, 4, 5], O0 + 8, dtype=L.F64)
    assert lib.tn_split_node(C.byref(a), 1, 3, C.byref(left), C.byref(overlap), None, ws, nbytes.value, None) == -5
    s_bad = desc([3, 2], O0 + (3 << 20), dtype=L.F64)
    assert lib.tn_split_node_full_svd(C.byref(a), 1, 3, C.byref(left), C.byref(s_bad), C.byref(right), None, ws,
                                      nbytes.value, None) == -2


def test_dmrg_validation_and_workspace_on_host():
    """The effective-Hamiltonian network is planned on the host: the
    workspace query succeeds for consistent shapes and rejects others."""
    lib = L.lib()
    Lt, Rt = desc([8, 3, 8], A0), desc([6, 3, 6], A0 + (1 << 20))
    w1, w2 = desc([3, 3, 2, 2], A0 + (2 << 20)), desc([3, 3, 2, 2], A0 + (3 << 20))
    th = desc([8, 2, 2, 6], B0)
    nbytes = C.c_size_t(0)
    assert lib.tn_dmrg_workspace(C.byref(Lt), C.byref(Rt), C.byref(w1), C.byref(w2), C.byref(th), 24,
                                 C.byref(nbytes)) == 0
    assert nbytes.value > 33 * 8 * 2 * 2 * 6 * 4
    assert lib.tn_dmrg_workspace(C.byref(Lt), C.byref(Rt), C.byref(w1), C.byref(w2), C.byref(th), 40,
                                 C.byref(nbytes)) == -1
    bad = desc([8, 2, 2, 7], B0)
    assert lib.tn_dmrg_workspace(C.byref(Lt), C.byref(Rt), C.byref(w1), C.byref(w2), C.byref(bad), 24,
                                 C.byref(nbytes)) == -2


def test_complex_validation_before_launch():
    lib = L.lib()
    a = desc([4, 5], A0, dtype=L.C64)
    b = desc([5, 6], B0, dtype=L.C64)
    out = desc([4, 6], O0, dtype=L.C64)
    nbytes = C.c_size_t(0)
    assert lib.tn_contract_between_c64_workspace(C.byref(b), C.byref(nbytes)) == 0 and nbytes.value >= 16 * 30
    call = lambda x, y, o, pa, pb: lib.tn_contract_between_c64(C.byref(x), C.byref(y), len(pa), L.int_array(pa),
                                                              L.int_array(pb), 1, 0, C.byref(o), FAKE + (5 << 30),
                                                              nbytes.value, 0, None)
    assert call(a, b, desc([4, 6], O0), [1], [0]) == -3                 # real out
    assert call(a, desc([6, 6], B0, dtype=L.C64), out, [1], [0]) == -2  # 5 vs 6
    assert call(a, b, out, [2], [0]) == -1
    assert lib.tn_contract_between_c64(C.byref(a), C.byref(b), 1, L.int_array([1]), L.int_array([0]), 0, 0,
                                       C.byref(out), FAKE + (5 << 30), 16, 0, None) == -4
    big = desc([2] * 7, B0, dtype=L.C64)                                 # b of rank 7: above 6
    assert lib.tn_contract_between_c64_workspace(C.byref(big), C.byref(nbytes)) == -3
