"""CPU-side checks of the C-ABI library: it loads without a GPU, exports every
symbol include/psp.h declares, rejects bad input with the documented status,
and its symbolic analysis equals the oracle's bit for bit."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def psp():
    from paper_2311_11833_amd import psp as m
    m.lib()
    return m


def test_exports_every_declared_symbol(psp):
    hdr = open(os.path.join(ROOT, "include", "psp.h")).read()
    declared = set(re.findall(r"PSP_API\s+[\w\s\*]+?\b(psp_\w+)\s*\(", hdr))
    assert declared == set(psp.EXPORTED)
    for name in declared:
        assert hasattr(psp.lib(), name), name


def test_weights_and_errors(psp, O):
    for eps in ([1e-2, 5e-3, 2.5e-3], [1e-3 * 0.5 ** k for k in range(5)], [2e-3, -2e-3, 4e-3, -4e-3]):
        assert np.array_equal(psp.weights(eps), O.weights(eps))
    for bad in ([1e-3, 1e-3], [0.0], [float("nan")]):
        with pytest.raises(psp.PSPError) as e:
            psp.weights(bad)
        assert e.value.status == psp.PSP_E_EPS


@pytest.mark.parametrize("bad", ["unsorted", "range", "ptr"])
def test_plan_rejects_malformed_csr(psp, bad):
    ip = np.array([0, 2, 3, 5], np.int32)
    ix = np.array([0, 2, 1, 0, 2], np.int32)
    if bad == "unsorted":
        ix = np.array([2, 0, 1, 0, 2], np.int32)
    elif bad == "range":
        ix = np.array([0, 3, 1, 0, 2], np.int32)
    else:
        ip = np.array([0, 3, 2, 5], np.int32)
    with pytest.raises(psp.PSPError) as e:
        psp.Plan(ip, ix)
    assert e.value.status == psp.PSP_E_INVALID


def _same(a, s):
    return (np.array_equal(a.perm, s.perm) and np.array_equal(a.iperm, s.iperm) and np.array_equal(a.parent, s.parent)
            and np.array_equal(a.l_ptr, s.lp) and np.array_equal(a.l_idx, s.li)
            and all(np.array_equal(a.levels[t][0], s.levels[t][0]) and np.array_equal(a.levels[t][1], s.levels[t][1])
                    for t in range(3)))


@pytest.mark.parametrize("N", [14, 30, 118, 300, 500, 1354])
@pytest.mark.parametrize("order", ["md", "natural"])
def test_symbolic_bit_exact_with_oracle(psp, O, W, N, order):
    ip, ix, _, _ = W.scenario_batch(N, 1)
    n = len(ip) - 1
    if order == "natural" and n > 1100:
        pytest.skip("natural-order fill of the largest pattern is covered at n=1001")
    a = psp.Plan(ip, ix, order=order).export()
    s = O.symbolic(n, ip, ix, natural=(order == "natural"))
    assert _same(a, s)


def test_symbolic_bit_exact_random_patterns(psp, O):
    import scipy.sparse as sp
    rng = np.random.default_rng(21)
    for t in range(12):
        n = int(rng.integers(5, 300))
        M = sp.random(n, n, density=float(rng.uniform(0.005, 0.1)), random_state=np.random.RandomState(t), format="csr")
        M = (M + sp.eye(n)).tocsr()
        if t % 3 == 0:
            M = M.tolil()
            for r in rng.choice(n, min(3, n), replace=False):
                M[r, :] = 1.0
            M = M.tocsr()
        M.sort_indices()
        ip, ix = M.indptr.astype(np.int32), M.indices.astype(np.int32)
        assert _same(psp.Plan(ip, ix).export(), O.symbolic(n, ip, ix)), t


@pytest.mark.slow
def test_symbolic_bit_exact_large(psp, O, W):
    """The 20,001-unknown pattern (10,000-bus network)."""
    net = W.make_network(10000)
    vm, va, p = W.make_state(10000, W.seed_state(10000, 0))
    J = W.jacobian(net, vm, va, p)
    a = psp.Plan(J.indptr, J.indices).export()
    s = O.symbolic(J.n, J.indptr, J.indices)
    assert _same(a, s)


def test_residual_argument_errors_before_any_device_call(psp):
    """psp_residual validates on the host: NULL required pointers -> PSP_E_INVALID, and
    n > 16384 without the R output -> PSP_E_UNSUPPORTED (no device memory is touched)."""
    import ctypes as C
    L = psp.lib()
    ip = np.array([0, 1, 2], np.int32)
    ix = np.array([0, 1], np.int32)
    plan = psp.Plan(ip, ix)
    assert L.psp_residual(plan.handle, 1, None, 1, None, None, None, None, None, None) == psp.PSP_E_INVALID
    assert L.psp_residual(None, 1, None, 1, None, None, None, None, None, None) == psp.PSP_E_INVALID
    n = 16385
    big = psp.Plan(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32))
    dummy = C.c_void_p(16)    # never dereferenced: the size check comes first
    st = L.psp_residual(big.handle, 1, dummy, 1, dummy, dummy, None, dummy, None, None)
    assert st == psp.PSP_E_UNSUPPORTED and b"needs the R output" in L.psp_last_error()


def test_group_rejects_bad_items_on_the_host(psp):
    """psp_group_create returns PSP_E_INVALID for an empty list, a NULL plan, batch < 1 or a
    bad nrhs, and PSP_E_EPS for bad nodes -- before any device call."""
    import ctypes as C
    L = psp.lib()
    ip = np.array([0, 1, 2], np.int32)
    ix = np.array([0, 1], np.int32)
    plan = psp.Plan(ip, ix)
    arr = (psp.GroupShape * 2)()
    arr[0] = psp.GroupShape(plan.handle.value, 3, 0)
    arr[1] = psp.GroupShape(None, 3, 0)
    eps = np.array([1e-3, 5e-4])
    ep = eps.ctypes.data_as(C.c_void_p)
    h = C.c_void_p()
    assert L.psp_group_create(2, C.byref(arr), 2, ep, 1, C.byref(h)) == psp.PSP_E_INVALID
    arr[1] = psp.GroupShape(plan.handle.value, 0, 0)
    assert L.psp_group_create(2, C.byref(arr), 2, ep, 1, C.byref(h)) == psp.PSP_E_INVALID
    assert L.psp_group_create(0, None, 2, ep, 1, C.byref(h)) == psp.PSP_E_INVALID
    arr[1] = psp.GroupShape(plan.handle.value, 3, 0)
    assert L.psp_group_create(2, C.byref(arr), 2, ep, 0, C.byref(h)) == psp.PSP_E_INVALID
    same = np.array([1e-3, 1e-3])
    assert L.psp_group_create(2, C.byref(arr), 2, same.ctypes.data_as(C.c_void_p), 1, C.byref(h)) == psp.PSP_E_EPS
    assert h.value is None
    assert L.psp_group_workspace_bytes(None) == 0
    dummy = C.c_void_p(256)
    assert L.psp_group_run(None, dummy, dummy, 1 << 20, None) == psp.PSP_E_INVALID
    assert L.psp_group_capture(None, dummy, dummy, 1 << 20, None, C.byref(h)) == psp.PSP_E_INVALID
    assert L.psp_graph_launch(None, None) == psp.PSP_E_INVALID


def test_plan_upload_checks_and_image_size_on_the_host(psp, W):
    """The plan's device image is sized on the host; psp_plan_upload rejects NULL, misaligned
    or short buffers before any device call, and numeric calls need an uploaded plan."""
    import ctypes as C
    L = psp.lib()
    ip, ix, _, _ = W.scenario_batch(300, 1)
    plan = psp.Plan(ip, ix)
    nb = plan.device_bytes()
    inf = plan.info()
    assert nb > 0 and nb % 256 == 0 and inf.device_bytes == nb
    assert L.psp_plan_device_bytes(None) == 0
    assert L.psp_plan_upload(plan.handle, None, nb, None) == psp.PSP_E_INVALID
    assert L.psp_plan_upload(plan.handle, C.c_void_p(256 + 8), nb, None) == psp.PSP_E_INVALID
    st = L.psp_plan_upload(plan.handle, C.c_void_p(256), nb - 256, None)
    assert st == psp.PSP_E_NOMEM and b"too small" in L.psp_last_error()


@pytest.mark.parametrize("N", [14, 30, 118, 300, 500])
def test_step_schedule_lds_budget(psp, W, N):
    """The step kernel's dynamic LDS plus its static LDS (at most 512 bytes reserved) fits the
    CU's 160 KiB, and twice that when two workgroups are counted per CU."""
    ip, ix, _, _ = W.scenario_batch(N, 1)
    inf = psp.Plan(ip, ix).info()
    assert inf.steps > 0
    assert inf.steps_per_cu in (1, 2)
    assert inf.steps_lds_bytes + 512 <= 160 * 1024
    if inf.steps_per_cu == 2:
        assert 2 * (inf.steps_lds_bytes + 512) <= 160 * 1024


def test_power_flow_create_rejects_mismatched_networks_on_the_host(psp, W):
    """psp_pf_create checks the network against the plan's pattern before any device call."""
    import ctypes as C
    L = psp.lib()
    c = W.pf_case(14)
    plan = psp.Plan(c.indptr, c.indices)

    def create(plan_h, nbus, yp, yc, g, b, pv):
        h = C.c_void_p()
        arrs = [np.ascontiguousarray(a) for a in (yp, yc, g, b, pv)]
        dummy = C.c_void_p(256)   # never dereferenced: every check comes before the copy
        st = L.psp_pf_create(plan_h, nbus, *[a.ctypes.data_as(C.c_void_p) for a in arrs], dummy, 1 << 30, None,
                             C.byref(h))
        return st, L.psp_last_error()

    good = (c.y_indptr, c.y_indices, c.g, c.b, c.pv)
    assert create(None, 14, *good)[0] == psp.PSP_E_INVALID
    st, msg = create(plan.handle, 13, *good)
    assert st == psp.PSP_E_INVALID and b"2*nbus + 1" in msg
    g = c.g.copy()
    g[3] = np.nan
    st, msg = create(plan.handle, 14, c.y_indptr, c.y_indices, g, c.b, c.pv)
    assert st == psp.PSP_E_INVALID and b"non-finite" in msg
    # a network with one branch fewer than the plan's pattern
    c2 = W.pf_case(14)
    net = c2.net
    keep = np.arange(len(net.fbus)) != len(net.fbus) - 1
    net2 = W.Network(14, net.fbus[keep], net.tbus[keep], net.r[keep], net.x[keep])
    yr, yc, yv = W._ybus_entries(net2)
    o = np.lexsort((yc, yr))
    yp = np.concatenate([[0], np.cumsum(np.bincount(yr[o], minlength=14))]).astype(np.int32)
    st, msg = create(plan.handle, 14, yp, yc[o].astype(np.int32), yv.real[o], yv.imag[o], c.pv)
    assert st == psp.PSP_E_INVALID and b"pattern" in msg
    # unsorted admittance row
    yc_bad = c.y_indices.copy()
    yc_bad[[0, 1]] = yc_bad[[1, 0]]
    st, msg = create(plan.handle, 14, c.y_indptr, yc_bad, c.g, c.b, c.pv)
    assert st == psp.PSP_E_INVALID and b"ascending" in msg
    assert L.psp_pf_workspace_bytes(None, 0, 1, 1) == 0
    assert L.psp_pf_eval(None, 1, None, None, None, None, None, None, None) == psp.PSP_E_INVALID


def test_estimate_rho_argument_errors_before_any_device_call(psp):
    import ctypes as C
    L = psp.lib()
    ip = np.array([0, 1, 2], np.int32)
    ix = np.array([0, 1], np.int32)
    plan = psp.Plan(ip, ix)
    dummy = C.c_void_p(16)
    assert L.psp_estimate_rho_workspace_bytes(None, 1) == 0
    assert L.psp_estimate_rho_workspace_bytes(plan.handle, 0) == 0
    assert L.psp_estimate_rho_workspace_bytes(plan.handle, 4) > 0
    assert L.psp_estimate_rho(None, 1, dummy, None, 1e-8, 4, dummy, dummy, dummy, 1 << 30, None) == psp.PSP_E_INVALID
    assert L.psp_estimate_rho(plan.handle, 1, dummy, None, 1e-8, 0, dummy, dummy, dummy, 1 << 30, None) == psp.PSP_E_INVALID
    st = L.psp_estimate_rho(plan.handle, 1, dummy, None, 1e-8, 4, dummy, dummy, dummy, 16, None)
    assert st == psp.PSP_E_NOMEM
