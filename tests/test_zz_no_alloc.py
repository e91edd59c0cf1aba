"""pcdn_solve_static (the allocation-free solve) through the C ABI against
pcdn_solve on a loaded context: two calls in a row on one device, the second
with a smaller problem, each bit-identical to the context's solve on the same
schedule (the same kernels and arithmetic on the same inputs).  Also: inputs
beyond the workspace and malformed CSC are rejected with an error, and
repeated calls leave the device's free memory unchanged."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_4080_amd as pc
    pc.ensure_built()
    return pc


def _device(d):
    import torch
    dev = torch.device("cuda:0")
    return (torch.from_numpy(d.col_ptr).to(dev), torch.from_numpy(d.row_idx).to(dev),
            torch.from_numpy(d.val).to(dev), torch.from_numpy(d.y).to(dev))


def _static(pc, d, C, P, eps, loss, **opts):
    """One call; also returns the device's free memory just before and just
    after it (the inputs and output are allocated before the first reading)."""
    import torch
    cp, ri, v, y = _device(d)
    w = torch.full((d.p,), np.nan, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    before = torch.cuda.mem_get_info(0)[0]
    rc, info = pc.pcdn_solve_static(0, d.n, d.p, cp, ri, v, y, C, P, eps, loss, w, **opts)
    torch.cuda.synchronize()
    after = torch.cuda.mem_get_info(0)[0]
    return (rc, w.cpu().numpy(), info), (before, after)


def _assert_identical(a, b):
    (ra, wa, ia), (rb, wb, ib) = a, b
    assert ra == rb
    for k in ("outer_iters", "converged", "bundles", "ls_steps", "ls_fail", "nnz_swept",
              "objective", "subgrad", "subgrad0"):
        assert ia[k] == ib[k], (k, ia[k], ib[k])
    np.testing.assert_array_equal(wa, wb)


CASES = [
    # (data, loss, C, P, eps, options): the text-like sizes' small sibling on
    # the single workgroup, then a smaller binary L2-SVM problem on the
    # multi-kernel schedule with shrinking
    (lambda: synth.c1(), "lr", 1.0, 32, 1e-4, dict(seed=1, schedule="narrow")),
    (lambda: synth.sparse_random(12, 800, 1200, 0.004, binary=True), "svm", 0.5, 128, 1e-3,
     dict(seed=2, schedule="wide", shrink=True)),
]


def test_static_solve_equals_context_solve_twice(pc):
    mem = []
    for make, loss, C, P, eps, opts in CASES:
        d = make()
        st, m = _static(pc, d, C, P, eps, loss, **opts)
        mem.append(m)
        s = pc.Solver(device=0).load_data(d)
        ref = s.solve(C, P, eps, loss, **opts)
        s.close()
        print(f"{loss} n={d.n} p={d.p}: outer {st[2]['outer_iters']}/{ref[2]['outer_iters']} "
              f"F {st[2]['objective']:.15g}/{ref[2]['objective']:.15g}", flush=True)
        assert st[0] == 0 and st[2]["converged"] == 1
        _assert_identical(st, ref)
    # a third call, the first problem again: the same bits
    make, loss, C, P, eps, opts = CASES[0]
    st, m = _static(pc, make(), C, P, eps, loss, **opts)
    mem.append(m)
    s = pc.Solver(device=0).load_data(make())
    _assert_identical(st, s.solve(C, P, eps, loss, **opts))
    s.close()
    # after the first call (which may load the library's code, and with it
    # the workspace, onto the device) no call changes the free device memory
    print("free device memory around each call:", mem, flush=True)
    for before, after in mem[1:]:
        assert before == after


def test_static_solve_rejects_what_does_not_fit_or_is_malformed(pc):
    import torch
    from paper_1306_4080_amd import PcdnError
    dev = "cuda:0"
    # 4M samples need more than the 64 MiB workspace: rejected before any work
    n, p = 4_000_000, 8
    cp = torch.zeros(p + 1, dtype=torch.int64, device=dev)
    ri = torch.zeros(1, dtype=torch.int32, device=dev)
    v = torch.zeros(1, dtype=torch.float32, device=dev)
    y = torch.ones(n, dtype=torch.int8, device=dev)
    w = torch.zeros(p, dtype=torch.float64, device=dev)
    with pytest.raises(PcdnError, match="E_ARG.*workspace"):
        pc.pcdn_solve_static(0, n, p, cp, ri[:0], v[:0], y, 1.0, 4, 1e-3, "lr", w)
    # a decreasing col_ptr, then a row index out of range: PCDN_E_CSC
    d = synth.sparse_random(3, 50, 20, 0.2)
    cpd, rid, vd, yd = _device(d)
    bad = cpd.clone()
    bad[5] = bad[6] + 1
    w = torch.zeros(d.p, dtype=torch.float64, device=dev)
    with pytest.raises(PcdnError, match="E_CSC"):
        pc.pcdn_solve_static(0, d.n, d.p, bad, rid, vd, yd, 1.0, 4, 1e-3, "lr", w)
    bad_r = rid.clone()
    bad_r[0] = d.n
    with pytest.raises(PcdnError, match="E_CSC"):
        pc.pcdn_solve_static(0, d.n, d.p, cpd, bad_r, vd, yd, 1.0, 4, 1e-3, "lr", w)
    # and the workspace still serves a valid problem afterwards
    rc, info = pc.pcdn_solve_static(0, d.n, d.p, cpd, rid, vd, yd, 1.0, 4, 1e-3, "lr", w)
    assert rc in (0, 1) and np.isfinite(info["objective"])
