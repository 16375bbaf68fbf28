"""Python front end of the RBiCG library: torch tensors on the GPU in, torch
tensors out.  Only marshalling happens here (pointers, sizes, the current HIP
stream); the solver runs in librbicg.so."""
from __future__ import annotations

import ctypes as ct
from typing import Optional

import numpy as np
import torch

from . import _lib

_PREC = {"f64": _lib.RBICG_F64, "c128": _lib.RBICG_C128, "mixed": _lib.RBICG_F32_IN_F64_OUT}


def _csr_struct(A, keep):
    """rbicg_csr for a host CSR (workloads.CSR or scipy.sparse)."""
    if hasattr(A, "rowptr"):
        n, rowptr, colind, vals = A.n, A.rowptr, A.colind, A.vals
    else:
        A = A.tocsr()
        n, rowptr, colind, vals = A.shape[0], A.indptr, A.indices, A.data
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colind = np.ascontiguousarray(colind, dtype=np.int32)
    cplx = np.iscomplexobj(vals)
    vals = np.ascontiguousarray(vals, dtype=np.complex128 if cplx else np.float64)
    keep.extend([rowptr, colind, vals])
    s = _lib.rbicg_csr()
    s.n = int(n)
    s.nnz = int(rowptr[-1])
    s.rowptr = rowptr.ctypes.data
    s.colind = colind.ctypes.data
    s.values = vals.ctypes.data
    s.values_complex = 1 if cplx else 0
    s.on_device = 0
    return s


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class DeviceMatrix:
    """A matrix (and its explicit conjugate transpose) repacked and resident in
    device memory (rbicg_matrix_create)."""

    def __init__(self, A, AH=None):
        self.lib = _lib.load()
        keep = []
        a = _csr_struct(A, keep)
        ah = _csr_struct(AH, keep) if AH is not None else None
        self.n = a.n
        self.complex = bool(a.values_complex)
        h = ct.c_void_p()
        rc = self.lib.rbicg_matrix_create(ct.byref(a), ct.byref(ah) if ah is not None else None,
                                          ct.byref(h))
        _lib.check(rc, "rbicg_matrix_create")
        self.h = h

    @classmethod
    def pencil(cls, A: "DeviceMatrix", E: "DeviceMatrix", alpha, beta=-1.0, out=None,
               stream=None) -> "DeviceMatrix":
        """alpha E + beta A (default beta = -1: the shifted operator alpha E - A)
        on A's layout, by rbicg_matrix_pencil.  With out (an earlier pencil of
        the same A and E) its values are overwritten in place on `stream`
        (default: the current stream)."""
        lib = _lib.load()
        al = np.array([complex(alpha).real, complex(alpha).imag])
        be = np.array([complex(beta).real, complex(beta).imag])
        h = ct.c_void_p(out.h.value if out is not None else None)
        rc = lib.rbicg_matrix_pencil(A.h, E.h, al.ctypes.data_as(_lib._DP),
                                     be.ctypes.data_as(_lib._DP),
                                     ct.c_void_p(_stream_ptr(stream)), ct.byref(h))
        _lib.check(rc, "rbicg_matrix_pencil")
        if out is not None:
            return out
        m = cls.__new__(cls)
        m.lib, m.h, m.n, m.complex = lib, h, A.n, True
        return m

    def info(self) -> dict:
        """Layout of the resident matrix (rbicg_matrix_info)."""
        v = (ct.c_int64 * 5)()
        _lib.check(self.lib.rbicg_matrix_info(self.h, v), "rbicg_matrix_info")
        return {"n": v[0], "nnz": v[1], "nnz_padded": v[2], "shared_pattern": bool(v[3]),
                "complex": bool(v[4])}

    def close(self):
        if getattr(self, "h", None):
            self.lib.rbicg_matrix_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RBILU:
    """Split ILU(0) preconditioner in red-black ordering of one matrix
    (rbicg_rbilu_*): ``black`` is the black block M_B of the split-
    preconditioned operator (a DeviceMatrix of order ``nb``), on which an
    ordinary Solver runs; ``rhs`` and ``solution`` map a dual pair's
    right-hand sides to the black system and its solutions back."""

    def __init__(self, A):
        self.lib = _lib.load()
        keep = []
        a = _csr_struct(A, keep)
        h, mb, nb = ct.c_void_p(), ct.c_void_p(), ct.c_int32()
        rc = self.lib.rbicg_rbilu_create(ct.byref(a), ct.byref(h), ct.byref(mb), ct.byref(nb))
        _lib.check(rc, "rbicg_rbilu_create")
        self.h, self.n, self.nb = h, a.n, nb.value
        self.complex = bool(a.values_complex)
        self.dtype = torch.complex128 if self.complex else torch.float64
        m = DeviceMatrix.__new__(DeviceMatrix)
        m.lib, m.h, m.n, m.complex = self.lib, mb, self.nb, self.complex
        self.black = m

    def _v(self, v, n, name):
        if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == self.dtype
                and v.is_contiguous() and v.numel() == n):
            raise TypeError(f"{name} must be a contiguous CUDA {self.dtype} tensor of length {n}")
        return ct.c_void_p(v.data_ptr())

    def refresh(self, A_next, stream=None):
        """New values of the matrix (same pattern): pivots and M_B recomputed
        on the device in place (rbicg_rbilu_refresh); handles on ``black``
        then need update_recycle(black)."""
        keep = []
        a = _csr_struct(A_next, keep)
        rc = self.lib.rbicg_rbilu_refresh(self.h, ct.byref(a), ct.c_void_p(_stream_ptr(stream)))
        _lib.check(rc, "rbicg_rbilu_refresh")

    def refresh_values(self, values, stream=None):
        """As refresh, from a CUDA tensor of the new values in the order of
        the CSR given at creation (rbicg_rbilu_refresh_values; the pattern is
        the caller's guarantee)."""
        if not (isinstance(values, torch.Tensor) and values.is_cuda and values.dtype == self.dtype
                and values.is_contiguous()):
            raise TypeError(f"values must be a contiguous CUDA {self.dtype} tensor")
        rc = self.lib.rbicg_rbilu_refresh_values(self.h, ct.c_void_p(values.data_ptr()),
                                                 ct.c_void_p(_stream_ptr(stream)))
        _lib.check(rc, "rbicg_rbilu_refresh_values")

    def rhs(self, b, bt, stream=None):
        """(b^_B, c^_B) of the black system."""
        bB = torch.empty(self.nb, dtype=self.dtype, device="cuda")
        cB = torch.empty_like(bB)
        rc = self.lib.rbicg_rbilu_rhs(self.h, self._v(b, self.n, "b"), self._v(bt, self.n, "bt"),
                                      self._v(bB, self.nb, "bB"), self._v(cB, self.nb, "cB"),
                                      ct.c_void_p(_stream_ptr(stream)))
        _lib.check(rc, "rbicg_rbilu_rhs")
        return bB, cB

    def solution(self, b, bt, yB, ytB, stream=None):
        """(x, x~) of the original pair from the black solutions."""
        x = torch.empty(self.n, dtype=self.dtype, device="cuda")
        xt = torch.empty_like(x)
        rc = self.lib.rbicg_rbilu_solution(
            self.h, self._v(b, self.n, "b"), self._v(bt, self.n, "bt"),
            self._v(yB, self.nb, "yB"), self._v(ytB, self.nb, "ytB"), self._v(x, self.n, "x"),
            self._v(xt, self.n, "xt"), ct.c_void_p(_stream_ptr(stream)))
        _lib.check(rc, "rbicg_rbilu_solution")
        return x, xt

    def close(self):
        if getattr(self, "black", None) is not None:
            self.black.h = None   # owned by the preconditioner
            self.black = None
        if getattr(self, "h", None):
            self.lib.rbicg_rbilu_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_split_sequence(mats, bs, bts, *, k=20, s=40, tol=1e-8, maxit=10000, **opts):
    """Split-preconditioned RBiCG over a sequence of dual pairs (Sec. 6): each
    matrix gets its red-black ILU(0) preconditioner, one handle solves the
    black systems in order (recycle spaces of the preconditioned systems,
    carried and updated between them).  Matrices on one pattern reuse the
    first set-up and refresh the values on the device.  bs, bts: CUDA
    tensors.  Returns a list of (x, x~, stats) with stats of the black solves."""
    out, S, P = [], None, None
    try:
        for j, A in enumerate(mats):
            if P is None:
                P = RBILU(A)
                S = Solver(P.black, k=k, s=s, maxit=maxit, **opts)
            else:
                S.stream.synchronize()   # the previous solve no longer reads M_B
                try:
                    P.refresh(A, stream=S.stream)
                except _lib.RBiCGError as e:
                    if e.code != _lib.RBICG_EINVAL:
                        raise
                    # another pattern: a new set-up (the handle moves to it)
                    Pn = RBILU(A)
                    S.update_recycle(Pn.black)
                    P.close()
                    P = Pn
                else:
                    S.update_recycle(P.black)
            bB, cB = P.rhs(bs[j], bts[j], stream=S.stream)
            yB, ytB, st = S.solve(bB, cB, tol=tol)
            x, xt = P.solution(bs[j], bts[j], yB, ytB, stream=S.stream)
            out.append((x, xt, st))
    finally:
        if S is not None:
            S.stream.synchronize()
            S.close()
        if P is not None:
            P.close()
    return out


class ILUT:
    """Split ILUT(droptol, fill) preconditioner of one matrix (rbicg_ilut_*):
    the factorization runs on the host once, the factors and their level
    schedules live on the device.  ``Solver.attach_ilu`` makes a handle
    iterate with L^{-1} A U^{-1}; ``rhs`` and ``solution`` map a dual pair's
    right-hand sides to the preconditioned pair and its solutions back."""

    def __init__(self, A, droptol=0.05, fill=-1, permtol=0.0):
        """permtol > 0: ILUTP (column pivoting, Sec. 6.2)."""
        self.lib = _lib.load()
        keep = []
        a = _csr_struct(A, keep)
        h = ct.c_void_p()
        rc = self.lib.rbicg_ilut_create(ct.byref(a), float(droptol), int(fill), float(permtol),
                                        ct.byref(h))
        _lib.check(rc, "rbicg_ilut_create")
        self.h, self.n = h, a.n
        self.complex = bool(a.values_complex)

    def set_waves(self, waves):
        """Waves working through a triangular solve's chunks (speed only)."""
        _lib.check(self.lib.rbicg_ilu_set_waves(self.h, int(waves)), "rbicg_ilu_set_waves")

    def info(self) -> dict:
        out = (ct.c_int64 * 8)()
        _lib.check(self.lib.rbicg_ilu_info(self.h, out), "rbicg_ilu_info")
        keys = ["n", "nnz_L", "nnz_U", "levels_L", "levels_U", "wait_error", "complex", "moved"]
        return dict(zip(keys, [int(v) for v in out]))

    def _v(self, v, name):
        ok = (isinstance(v, torch.Tensor) and v.is_cuda and v.is_contiguous() and v.numel() == self.n
              and v.dtype in ((torch.complex128,) if self.complex else (torch.float64, torch.complex128)))
        if not ok:
            raise TypeError(f"{name} must be a contiguous CUDA float64/complex128 tensor of length "
                            f"{self.n} (complex128 for a complex matrix)")
        return ct.c_void_p(v.data_ptr())

    def _two(self, fn, u, v, stream):
        if u.dtype != v.dtype:
            raise TypeError("both vectors must have one dtype")
        a, b = torch.empty_like(u), torch.empty_like(v)
        cplx = 1 if u.dtype == torch.complex128 else 0
        rc = fn(self.h, self._v(u, "u"), self._v(v, "v"), self._v(a, "out"), self._v(b, "out"), cplx,
                ct.c_void_p(_stream_ptr(stream)))
        _lib.check(rc, fn.__name__)
        return a, b

    def rhs(self, b, bt, stream=None):
        """(L^{-1} b, U^{-H} b~)."""
        return self._two(self.lib.rbicg_ilu_rhs, b, bt, stream)

    def solution(self, y, yt, stream=None):
        """(U^{-1} y, L^{-H} y~)."""
        return self._two(self.lib.rbicg_ilu_solution, y, yt, stream)

    def close(self):
        if getattr(self, "h", None):
            self.lib.rbicg_ilu_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_ilut_sequence(mats, bs, bts, *, droptol=0.05, fill=-1, permtol=0.0, k=20, s=40,
                        tol=1e-8, maxit=10000, prec="f64", **opts):
    """Split-ILUT-preconditioned RBiCG over a sequence of dual pairs (Sec. 6):
    each matrix gets its own ILUT(droptol, fill) (ILUTP when permtol > 0),
    one handle solves the
    preconditioned pairs in order with the recycle space carried between
    them (biorthogonalized against each new preconditioned operator).  Zero
    initial guesses.  bs, bts: CUDA tensors.  Returns a list of
    (x, x~, stats) with stats of the preconditioned solves."""
    out, S, P = [], None, None
    try:
        for j, A in enumerate(mats):
            Pn = ILUT(A, droptol, fill, permtol)
            if S is None:
                S = Solver(A, k=k, s=s, maxit=maxit, prec=prec, **opts)
                S.attach_ilu(Pn)
            else:
                S.stream.synchronize()     # the previous solve no longer uses P
                S.attach_ilu(Pn)
                S.update_recycle(A)        # C = A^ U against the new operator
            if P is not None:
                P.close()
            P = Pn
            S._order()                     # b, b~ are complete before rhs reads them
            bh, ch = P.rhs(bs[j], bts[j], stream=S.stream)
            y, yt, st = S.solve(bh, ch, tol=tol)
            x, xt = P.solution(y, yt, stream=S.stream)
            out.append((x, xt, st))
    finally:
        if S is not None:
            S.stream.synchronize()
            S.close()
        if P is not None:
            P.close()
    return out


class Batch:
    """Continuous batching of iteration launches across solver handles
    (rbicg_batch_*): handles created with ``batch=`` hand their chunks of
    iterations to it, and it launches the chunks of all handles that are
    iterating together."""

    def __init__(self, max_slots=16, window_us=50.0, graphs=False):
        """graphs: replay each launch set as a captured HIP graph
        (rbicg_batch_use_graphs)."""
        self.lib = _lib.load()
        h = ct.c_void_p()
        _lib.check(self.lib.rbicg_batch_create(int(max_slots), float(window_us), ct.byref(h)),
                   "rbicg_batch_create")
        self.h = h
        if graphs:
            _lib.check(self.lib.rbicg_batch_use_graphs(self.h, 1), "rbicg_batch_use_graphs")

    def stats(self) -> dict:
        out = np.zeros(6)
        _lib.check(self.lib.rbicg_batch_stats(self.h, _lib.dptr(out)), "rbicg_batch_stats")
        return {"launches": int(out[0]), "chunks": int(out[1]), "handle_iterations": int(out[2]),
                "max_chunks_per_launch": int(out[3]),
                "chunks_per_launch": float(out[1] / max(out[0], 1)),
                "graph_replays": int(out[4]), "graph_captures": int(out[5])}

    def close(self):
        if getattr(self, "h", None):
            self.lib.rbicg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """One handle: a matrix (and its explicit conjugate transpose), a recycle
    space and the device workspace, kept across the systems of a sequence.
    ``A`` is a host CSR (copied into a matrix the handle owns) or a
    DeviceMatrix (shared; it must outlive the handle)."""

    def __init__(self, A, AH=None, *, k=20, s=40, maxit=10000, max_restarts=2, update=True,
                 svd_tol=1e-2, seed=0, prec="f64", inner_tol=1e-5, max_outer=30, chunk=0,
                 stream=None, profile=False, stall_window=0, pencil_setup=0, batch=None,
                 blocks=0):
        self.lib = _lib.load()
        o = _lib.rbicg_opts()
        self.lib.rbicg_default_opts(ct.byref(o))
        o.k, o.s, o.maxit, o.max_restarts = k, s, maxit, max_restarts
        o.update = 1 if update else 0
        o.svd_tol, o.seed, o.prec = svd_tol, seed, _PREC[prec]
        o.inner_tol, o.max_outer, o.chunk = inner_tol, max_outer, chunk
        # profile: False/0 off, True/1 every chunk, p > 1 every p-th chunk
        o.profile = int(profile)
        # restart without recycling after a stall (not in the paper; 0: off)
        o.stall_window = int(stall_window)
        # cycle-end pencil: 0 device Grams, 1 the recurrences of Sec. 4.4
        o.pencil_setup = int(pencil_setup)
        # iteration-kernel blocks (0: automatic; the autotuner's choice otherwise)
        o.blocks = int(blocks)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        o.stream = _stream_ptr(self.stream)
        self.opts = o
        self.prec = prec
        # vectors at the boundary (b, x, ...) and the recycle-basis storage type
        self.dtype = torch.complex128 if prec == "c128" else torch.float64
        self.basis_dtype = torch.float32 if prec == "mixed" else self.dtype
        h = ct.c_void_p()
        if isinstance(A, DeviceMatrix):
            self.matrix = A
            self.n = A.n
            rc = self.lib.rbicg_create_on(A.h, ct.byref(o), ct.byref(h))
            _lib.check(rc, "rbicg_create_on")
        else:
            keep = []
            a = _csr_struct(A, keep)
            ah = _csr_struct(AH, keep) if AH is not None else None
            self.n = a.n
            rc = self.lib.rbicg_create(ct.byref(a), ct.byref(ah) if ah is not None else None,
                                       ct.byref(o), ct.byref(h))
            _lib.check(rc, "rbicg_create")
        self.h = h
        self.batch = batch
        if batch is not None:
            _lib.check(self.lib.rbicg_batch_attach(self.h, batch.h), "rbicg_batch_attach")

    # --------------------------------------------------------------- helpers
    def _order(self):
        """Order the handle's stream after the caller's current stream, so that
        tensors the caller (or this wrapper) filled there are complete before
        the library reads or writes them on the handle's stream.  The library
        calls below return only after their work on that stream is done."""
        cur = torch.cuda.current_stream()
        if self.stream != cur:
            self.stream.wait_stream(cur)

    def _vec(self, v, name):
        if not (isinstance(v, torch.Tensor) and v.is_cuda):
            raise TypeError(f"{name} must be a CUDA tensor")
        if v.dtype != self.dtype or not v.is_contiguous() or v.numel() != self.n:
            raise TypeError(f"{name} must be a contiguous {self.dtype} tensor of length {self.n}")
        return ct.c_void_p(v.data_ptr())

    def close(self):
        if getattr(self, "h", None):
            self.lib.rbicg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ API
    def solve(self, b, bt, x=None, xt=None, tol=1e-8, allow_not_converged=True):
        """rbicg_solve_dual: returns (x, x~, stats dict)."""
        x = torch.zeros_like(b) if x is None else x
        xt = torch.zeros_like(bt) if xt is None else xt
        st = _lib.rbicg_stats()
        self._order()
        rc = self.lib.rbicg_solve_dual(self.h, self._vec(b, "b"), self._vec(bt, "bt"),
                                       self._vec(x, "x"), self._vec(xt, "xt"), float(tol),
                                       ct.byref(st))
        ok = (_lib.RBICG_OK, _lib.RBICG_NOT_CONVERGED) if allow_not_converged else (_lib.RBICG_OK,)
        _lib.check(rc, "rbicg_solve_dual", ok)
        return x, xt, st.as_dict()

    def attach_ilu(self, P):
        """Iterate with the split-preconditioned operator of P (an ILUT; None
        detaches) from the next call on (rbicg_ilu_attach)."""
        rc = self.lib.rbicg_ilu_attach(self.h, P.h if P is not None else None)
        _lib.check(rc, "rbicg_ilu_attach")
        self.ilu = P

    def solve_sequence(self, mats, bs, bts, xs=None, xts=None, tol=1e-8, zero_init=True,
                       allow_not_converged=True):
        """rbicg_solve_sequence: the systems (mats[j] DeviceMatrix, bs[j], bts[j])
        in one library call, the recycle space carried and updated between
        them.  xs, xts: solution tensors (allocated when None; zeroed in the
        library when zero_init).  Returns (xs, xts, [stats per system])."""
        m = len(mats)
        xs = [torch.empty_like(b) for b in bs] if xs is None else xs
        xts = [torch.empty_like(b) for b in bts] if xts is None else xts
        for A in mats:
            if not isinstance(A, DeviceMatrix):
                raise TypeError("solve_sequence takes DeviceMatrix objects")
        P = ct.c_void_p * m
        arr = lambda vs, name: P(*[self._vec(v, name) for v in vs])
        st = (_lib.rbicg_stats * m)()
        self._order()
        rc = self.lib.rbicg_solve_sequence(self.h, m, P(*[A.h for A in mats]), arr(bs, "b"),
                                           arr(bts, "bt"), arr(xs, "x"), arr(xts, "xt"),
                                           1 if zero_init else 0, float(tol), st)
        ok = (_lib.RBICG_OK, _lib.RBICG_NOT_CONVERGED) if allow_not_converged else (_lib.RBICG_OK,)
        _lib.check(rc, "rbicg_solve_sequence", ok)
        self.matrix = mats[-1] if m else self.matrix
        return xs, xts, [s.as_dict() for s in st]

    def update_recycle(self, A_next=None, AH_next=None):
        if isinstance(A_next, DeviceMatrix):
            self.matrix = A_next
            _lib.check(self.lib.rbicg_update_recycle_on(self.h, A_next.h), "rbicg_update_recycle_on")
            return
        keep = []
        a = _csr_struct(A_next, keep) if A_next is not None else None
        ah = _csr_struct(AH_next, keep) if AH_next is not None else None
        rc = self.lib.rbicg_update_recycle(self.h, ct.byref(a) if a is not None else None,
                                           ct.byref(ah) if ah is not None else None)
        _lib.check(rc, "rbicg_update_recycle")

    def set_recycle(self, U, Ut):
        k = 0 if U is None else U.shape[1]
        if k:
            # column-major (each column contiguous), in the handle's basis type
            Ucm = U.t().to(self.basis_dtype).contiguous()
            Utcm = Ut.t().to(self.basis_dtype).contiguous()
            self._order()
            rc = self.lib.rbicg_set_recycle(self.h, ct.c_void_p(Ucm.data_ptr()),
                                            ct.c_void_p(Utcm.data_ptr()), k)
        else:
            rc = self.lib.rbicg_set_recycle(self.h, None, None, 0)
        _lib.check(rc, "rbicg_set_recycle")

    def get_recycle(self, next=False, kcap=64):
        """Returns (U, U~, C, C~) as n x k tensors."""
        bufs = [torch.zeros((kcap, self.n), dtype=self.basis_dtype, device="cuda") for _ in range(4)]
        k = ct.c_int32()
        self._order()
        rc = self.lib.rbicg_get_recycle(self.h, *[ct.c_void_p(b.data_ptr()) for b in bufs],
                                        kcap, 1 if next else 0, ct.byref(k))
        _lib.check(rc, "rbicg_get_recycle")
        kk = min(k.value, kcap)
        return tuple(b[:kk].t() for b in bufs)

    def save_recycle(self, path, next=True):
        """Write the recycle space to an .npz file, so that a sequence can be
        resumed in another process: U, U~ (n x k) -- the space the cycle
        updates built for the next system when next is set and one exists,
        else the installed one -- with n and the precision mode.  Plain arrays
        only (no pickled objects)."""
        U, Ut, _, _ = self.get_recycle(next=next)
        if next and U.shape[1] == 0:
            U, Ut, _, _ = self.get_recycle(next=False)
        np.savez(path, U=U.cpu().numpy(), Ut=Ut.cpu().numpy(), n=np.int64(self.n),
                 prec=np.array(self.prec))

    def load_recycle(self, path):
        """Install a space written by save_recycle: C = A U, C~ = A^H U~ and the
        biorthogonalization (Sec. 4.3) are recomputed for this handle's matrix,
        as rbicg_update_recycle does for a space built in the same process."""
        with np.load(path, allow_pickle=False) as f:
            if int(f["n"]) != self.n:
                raise ValueError(f"recycle space of size {int(f['n'])} for a handle of size {self.n}")
            if str(f["prec"]) != self.prec:
                raise ValueError(f"recycle space of precision {f['prec']} for a {self.prec} handle")
            U = torch.as_tensor(f["U"], device="cuda")
            Ut = torch.as_tensor(f["Ut"], device="cuda")
        self.set_recycle(U if U.shape[1] else None, Ut if U.shape[1] else None)

    def bilinear_sequence(self, items, tol=1e-8):
        """Bilinear forms u_j^H A_j^{-1} w_j along a sequence (Sec. 1; e.g. one
        form per sample of a parameter-dependent A): items = [(A_j, u_j, w_j)]
        with A_j a DeviceMatrix, CSR or None (same matrix).  The recycle space
        built while solving form j is installed for form j+1.  Returns
        [(value, error bound, stats)] as bilinear does."""
        out = []
        for j, (A, u, w) in enumerate(items):
            if j:
                self.update_recycle(A)
            out.append(self.bilinear(u, w, tol))
        return out

    def profile(self, reset=False):
        """Per-kernel timing (rbicg_profile): dict with ms/launch counts and
        the algorithmic bytes of one SpMV-kernel launch and of one iteration."""
        out = np.zeros(13)
        _lib.check(self.lib.rbicg_profile(self.h, 1 if reset else 0, _lib.dptr(out)), "rbicg_profile")
        return {"spmv_ms": out[0], "spmv_n": int(out[1]), "update_ms": out[2],
                "update_n": int(out[3]), "spmv_bytes": out[4], "iter_bytes": out[5],
                "spmv_bytes_total": out[6], "update_bytes_total": out[7],
                "cycle_updates": int(out[8]), "cycle_eig_ms": out[9], "cycle_biorth_ms": out[10],
                "cycle_latency_ms": out[11], "cycle_wait_ms": out[12]}

    def log(self):
        """Per-iteration log of the last solve as an (iters, 10) float64 array."""
        cnt = ct.c_int32()
        self.lib.rbicg_get_log(self.h, None, 0, ct.byref(cnt))
        out = np.zeros((max(cnt.value, 1), 10))
        self.lib.rbicg_get_log(self.h, _lib.dptr(out), cnt.value, ct.byref(cnt))
        return out[:cnt.value]

    def bilinear(self, u, w, tol=1e-8):
        val = np.zeros(2)
        err = ct.c_double()
        st = _lib.rbicg_stats()
        self._order()
        rc = self.lib.rbicg_bilinear(self.h, self._vec(u, "u"), self._vec(w, "w"), float(tol),
                                     ct.c_void_p(val.ctypes.data), ct.byref(err), ct.byref(st))
        _lib.check(rc, "rbicg_bilinear", (_lib.RBICG_OK, _lib.RBICG_NOT_CONVERGED))
        v = complex(val[0], val[1]) if self.prec == "c128" else float(val[0])
        return v, err.value, st.as_dict()

    def bilinear_batch(self, U, W, tol=1e-8):
        """rbicg_bilinear_batch: u_i^H A^{-1} w_i for the rows of (S, n) complex
        CUDA tensors U, W, in one batched solve.  Returns a list of
        (value, error bound, stats) as bilinear does."""
        S = U.shape[0]
        for name, t in (("U", U), ("W", W)):
            if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()
                    and tuple(t.shape) == (S, self.n)):
                raise TypeError(f"{name} must be a contiguous complex128 CUDA tensor of shape ({S}, {self.n})")
        vals = np.zeros(2 * S)
        errs = np.zeros(S)
        sts = (_lib.rbicg_stats * S)()
        self._order()
        rc = self.lib.rbicg_bilinear_batch(self.h, S, ct.c_void_p(U.data_ptr()), ct.c_void_p(W.data_ptr()),
                                           float(tol), _lib.dptr(vals), _lib.dptr(errs), sts)
        _lib.check(rc, "rbicg_bilinear_batch", (_lib.RBICG_OK, _lib.RBICG_NOT_CONVERGED))
        return [(complex(vals[2 * i], vals[2 * i + 1]), float(errs[i]), sts[i].as_dict())
                for i in range(S)]

    def project(self, X, Xt, b=None, c=None):
        """rbicg_project: Ar = Xt^H A X, Er = Xt^H X (and br = Xt^H b, cr = X^H c
        when b, c are given) for (m, n) complex CUDA tensors X, Xt.  Returns
        numpy (Ar, Er) or (Ar, Er, br, cr)."""
        m = X.shape[0]
        for name, t in (("X", X), ("Xt", Xt)):
            if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()
                    and tuple(t.shape) == (m, self.n)):
                raise TypeError(f"{name} must be a contiguous complex128 CUDA tensor of shape ({m}, {self.n})")
        Ar = np.zeros(m * m, np.complex128)  # column-major m x m
        Er = np.zeros(m * m, np.complex128)
        br = np.zeros(m, np.complex128)
        cr = np.zeros(m, np.complex128)
        with_bc = b is not None
        self._order()
        rc = self.lib.rbicg_project(
            self.h, m, ct.c_void_p(X.data_ptr()), ct.c_void_p(Xt.data_ptr()),
            self._vec(b, "b") if with_bc else None, self._vec(c, "c") if with_bc else None,
            Ar.view(np.float64).ctypes.data_as(_lib._DP), Er.view(np.float64).ctypes.data_as(_lib._DP),
            br.view(np.float64).ctypes.data_as(_lib._DP) if with_bc else None,
            cr.view(np.float64).ctypes.data_as(_lib._DP) if with_bc else None)
        _lib.check(rc, "rbicg_project")
        Ar = Ar.reshape((m, m), order="F")
        Er = Er.reshape((m, m), order="F")
        return (Ar, Er, br, cr) if with_bc else (Ar, Er)

    def solve_shifted(self, sigmas, b, c, X=None, Xt=None, tol=1e-8, update_from=-1):
        """rbicg_solve_shifted: (sigma_s I - A) X[s] = b, (sigma_s I - A)^H Xt[s] = c
        for every shift; X, Xt are (S, n) complex CUDA tensors (initial guesses
        on entry).  Returns (X, Xt, [stats per shift])."""
        S = len(sigmas)
        sig = np.ascontiguousarray(np.asarray(sigmas, dtype=np.complex128))
        Xcm = torch.zeros((S, self.n), dtype=self.dtype, device="cuda") if X is None else X
        Xtcm = torch.zeros((S, self.n), dtype=self.dtype, device="cuda") if Xt is None else Xt
        for name, t in (("X", Xcm), ("Xt", Xtcm)):
            if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()
                    and tuple(t.shape) == (S, self.n)):
                raise TypeError(f"{name} must be a contiguous complex128 CUDA tensor of shape ({S}, {self.n})")
        sts = (_lib.rbicg_stats * S)()
        self._order()
        rc = self.lib.rbicg_solve_shifted(self.h, S, sig.view(np.float64).ctypes.data_as(_lib._DP),
                                          self._vec(b, "b"), self._vec(c, "c"),
                                          ct.c_void_p(Xcm.data_ptr()), ct.c_void_p(Xtcm.data_ptr()),
                                          float(tol), update_from, sts)
        _lib.check(rc, "rbicg_solve_shifted", (_lib.RBICG_OK, _lib.RBICG_NOT_CONVERGED))
        return Xcm, Xtcm, [s.as_dict() for s in sts]
