"""The no-allocation dual solve (rbicg_solve_dual_noalloc) against
rbicg_solve_dual on a k = 0 handle: both run plain BiCG with the same kernels
in the same order, so solutions, iteration counts and residuals must be equal
bit for bit.  Two calls in a row on one GPU (the second on a smaller system,
so it reuses the scratch array the first left behind), a complex call, and the
argument checks that reject work beyond the scratch array before any launch."""
import ctypes as ct

import numpy as np
import pytest

from paper_1010_0762_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(v):
    dt = torch.complex128 if np.iscomplexobj(v) else torch.float64
    return torch.as_tensor(np.ascontiguousarray(v)).to(device="cuda", dtype=dt)


def _noalloc(M, prec, b, bt, tol, maxit=10000, k=0):
    from paper_1010_0762_amd import _lib
    lib = _lib.load()
    o = _lib.rbicg_opts()
    lib.rbicg_default_opts(ct.byref(o))
    o.k, o.maxit, o.prec = k, maxit, prec
    o.stream = int(torch.cuda.current_stream().cuda_stream)
    x = torch.zeros_like(b)
    xt = torch.zeros_like(bt)
    st = _lib.rbicg_stats()
    torch.cuda.synchronize()
    rc = lib.rbicg_solve_dual_noalloc(M.h, ct.byref(o), ct.c_void_p(b.data_ptr()),
                                      ct.c_void_p(bt.data_ptr()), ct.c_void_p(x.data_ptr()),
                                      ct.c_void_p(xt.data_ptr()), float(tol), ct.byref(st))
    return rc, x, xt, st.as_dict()


def _reference(M, prec, b, bt, tol):
    from paper_1010_0762_amd.solver import Solver
    S = Solver(M, k=0, update=False, prec=prec)
    x, xt, st = S.solve(b, bt, tol=tol)
    S.close()
    return x, xt, st


def _same(M, prec_name, prec_code, b, bt, tol):
    rc, x, xt, st = _noalloc(M, prec_code, b, bt, tol)
    xr, xtr, sr = _reference(M, prec_name, b, bt, tol)
    print(f"n={M.n} {prec_name}: noalloc rc={rc} iters={st['iters']} relres={st['relres']:.2e}; "
          f"handle iters={sr['iters']} relres={sr['relres']:.2e}", flush=True)
    assert rc == 0 and sr["status"] == 0
    assert st["iters"] == sr["iters"] and st["restarts"] == sr["restarts"]
    assert st["relres"] == sr["relres"] and st["relres_dual"] == sr["relres_dual"]
    assert torch.equal(x, xr) and torch.equal(xt, xtr)
    assert st["relres"] <= tol and st["relres_dual"] <= tol


def test_noalloc_matches_handle_solve_two_calls():
    from paper_1010_0762_amd import _lib
    from paper_1010_0762_amd.solver import DeviceMatrix
    torch.cuda.set_device(0)
    rng = np.random.default_rng(7)
    # first call: 3D conv-diff 28^3 (n = 21952, several row blocks, ragged tail)
    A1 = wl.convdiff(28, 3, (20.0, 10.0, 5.0))
    M1 = DeviceMatrix(A1)
    _same(M1, "f64", _lib.RBICG_F64, _t(rng.standard_normal(A1.n)), _t(rng.standard_normal(A1.n)), 1e-8)
    # second call, smaller: 2D conv-diff 19 x 19 (n = 361, one block)
    A2 = wl.convdiff(19, 2, (10.0, 5.0))
    M2 = DeviceMatrix(A2)
    _same(M2, "f64", _lib.RBICG_F64, _t(rng.uniform(size=A2.n)), _t(rng.uniform(size=A2.n)), 1e-8)
    M1.close()
    M2.close()


def test_noalloc_complex_matches_handle_solve():
    from paper_1010_0762_amd import _lib
    from paper_1010_0762_amd.solver import DeviceMatrix
    A = wl.random_sparse(3000, 6, seed=11, diag_shift=8.0, complex_vals=True)
    rng = np.random.default_rng(8)
    M = DeviceMatrix(A)
    b = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
    bt = rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)
    _same(M, "c128", _lib.RBICG_C128, _t(b), _t(bt), 1e-8)
    M.close()


def test_noalloc_rejects_work_beyond_scratch():
    from paper_1010_0762_amd import _lib
    from paper_1010_0762_amd.solver import DeviceMatrix
    # n = 65^3 = 274625 real unknowns: 8 work vectors exceed the array
    A = wl.convdiff(65, 3, (1.0, 1.0, 1.0))
    M = DeviceMatrix(A)
    b = torch.ones(A.n, dtype=torch.float64, device="cuda")
    rc, _, _, _ = _noalloc(M, _lib.RBICG_F64, b, b, 1e-8)
    assert rc == _lib.RBICG_EINVAL and "scratch" in _lib.last_error()
    M.close()
    A = wl.convdiff(10, 2, (1.0, 1.0))
    M = DeviceMatrix(A)
    b = torch.ones(A.n, dtype=torch.float64, device="cuda")
    rc, _, _, _ = _noalloc(M, _lib.RBICG_F64, b, b, 1e-8, maxit=_lib_maxit() + 1)
    assert rc == _lib.RBICG_EINVAL and "maxit" in _lib.last_error()
    rc, _, _, _ = _noalloc(M, _lib.RBICG_F64, b, b, 1e-8, k=4)
    assert rc == _lib.RBICG_EINVAL and "k must be 0" in _lib.last_error()
    M.close()


def _lib_maxit():
    return 20000
