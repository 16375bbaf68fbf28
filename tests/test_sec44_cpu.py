"""Pins of the oracle's Sec. 4.4 pencil set-up (oracle/sec44.py) against the
plain definitions it replaces: the augmented bi-Lanczos relation (eq.
augBiLanExtend) for Gamma_j and Gamma~_j, B_j = C~^H A V_j from explicit
products, the carried blocks of Psi~^H Psi and Psi~^H Phi against explicit
products of the actual bases, and the pencil against the explicit-product
pencil of eq. finalGenEigValue.  In exact arithmetic the recurrences are
exact; in floating point they inherit the loss of biorthogonality of the
Lanczos vectors, which each bound below scales with."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import recycle as rc
from oracle.krylov import as_csr
from paper_1010_0762_amd import workloads as wl

S = 40


def _run_sequence(nsys=3, setup="recurrence", keep=True, cplx=False):
    """The 2D conv-diff sequence; complex: each matrix times (1 + 0.3i) plus
    0.2i I, with complex right-hand sides (so every conjugation matters)."""
    seq = wl.cfg1_sequence(nsys)
    rng = np.random.default_rng(5)
    U = Ut = None
    out = []
    for j in range(nsys):
        A = as_csr(seq.mats[j]); AH = A.conj().T.tocsr()
        b, bt = seq.b[j], seq.bt[j]
        if cplx:
            A = (A * (1.0 + 0.3j) + 0.2j * sp.identity(A.shape[0], format="csr")).tocsr()
            AH = A.conj().T.tocsr()
            b = b + 0.5j * rng.uniform(size=b.shape)
            bt = bt - 0.5j * rng.uniform(size=bt.shape)
        C = Ct = None
        if U is not None:
            U, Ut, C, Ct = rc.biorthogonalize(A, AH, U, Ut, 1e-2)
        res = oracle.rbicg(A, b, bt, None, None, U, Ut, C, Ct, tol=1e-8, s=S,
                           k=10, pencil_setup=setup, keep_lanczos=keep)
        out.append((A, AH, C, Ct, res))
        U, Ut = res.U_next, res.Ut_next
    return out


@pytest.fixture(scope="module", params=[False, True], ids=["real", "complex"])
def rec_runs(request):
    return _run_sequence(cplx=request.param)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _cycle_data(res, d):
    """Cycle index (1-based) of pencil record d, and the Lanczos vectors."""
    V = np.stack(res.lanczos["V"], 1)
    Vt = np.stack(res.lanczos["Vt"], 1)
    return V, Vt


def _cycles(res):
    """(cycle number, record) for every recorded pencil; the T-path first
    cycle of the first system is not recorded."""
    recs = res.pencils
    first = 2 if recs and recs[0]["case"] == "general" else 1
    return [(first + i, d) for i, d in enumerate(recs)]


def test_gamma_and_b_from_scalars_match_products(rec_runs):
    """(I - C C~^H) A V_j = Upsilon_j Gamma_j and the dual relation with
    Gamma~_j built from T~ = T^H; B_j = C~^H A V_j, B~_j = C^H A^H V~_j."""
    for sysi, (A, AH, C, Ct, res) in enumerate(rec_runs):
        V, Vt = _cycle_data(res, None)
        for cyc, d in _cycles(res):
            i0 = (cyc - 1) * S
            Vj, Vtj = V[:, i0:i0 + S], Vt[:, i0:i0 + S]
            lo = i0 - 1 if cyc > 1 else None
            Ups = np.concatenate([V[:, lo:lo + 1] if lo is not None else np.zeros((A.shape[0], 1)),
                                  Vj, V[:, i0 + S:i0 + S + 1]], axis=1)
            Upst = np.concatenate([Vt[:, lo:lo + 1] if lo is not None else np.zeros((A.shape[0], 1)),
                                   Vtj, Vt[:, i0 + S:i0 + S + 1]], axis=1)
            AV, AHV = A @ Vj, AH @ Vtj
            if C is not None:
                assert _rel(d["B"], Ct.conj().T @ AV) <= 1e-10
                assert _rel(d["Bt"], C.conj().T @ AHV) <= 1e-10
                AV = AV - C @ (Ct.conj().T @ AV)
                AHV = AHV - Ct @ (C.conj().T @ AHV)
            assert _rel(Ups @ d["G"], AV) <= 1e-10, (sysi, cyc)
            assert _rel(Upst @ d["Gt"], AHV) <= 1e-7, (sysi, cyc)


def test_carried_blocks_match_products(rec_runs):
    """The blocks carried from cycle j-1 against explicit products of the
    actual bases C_{j-1} = A U_{j-1}, C~_{j-1} = A^H U~_{j-1}, Upsilon_j.
    Blocks built only from C, C~, B and the SVD transforms agree to rounding;
    the ones that use Lanczos biorthogonality (Upsilon~^H Upsilon = I, and
    C~_{j-2} orthogonal to Upsilon_j) agree to the measured loss of it over
    the two cycles, as errors relative to the product of the factors' norms."""
    for sysi, (A, AH, C, Ct, res) in enumerate(rec_runs):
        V, Vt = _cycle_data(res, None)
        for cyc, d in _cycles(res):
            if d["case"] != "general":
                continue
            X = d["X"]
            kp = X.XCtU.shape[0]
            Up, Utp = d["Phi"][:, :kp], d["Phit"][:, :kp]
            Cp, Ctp = A @ Up, AH @ Utp
            i0 = (cyc - 1) * S
            Ups, Upst = V[:, i0 - 1:i0 + S + 1], Vt[:, i0 - 1:i0 + S + 1]
            lo = max(i0 - S - 1, 0)
            W2, Wt2 = V[:, lo:i0 + S + 1], Vt[:, lo:i0 + S + 1]
            loss = np.linalg.norm(Wt2.conj().T @ W2 - np.eye(W2.shape[1]))
            if C is not None:
                loss += np.linalg.norm(C.conj().T @ Wt2) + np.linalg.norm(Ct.conj().T @ W2)
                assert _rel(X.XCC, Ct.conj().T @ Cp) <= 1e-10
                assert _rel(X.XCtC, Ctp.conj().T @ C) <= 1e-10
                assert _rel(X.XCU, Ct.conj().T @ Up) <= 1e-10
            assert _rel(d["YtU"], Upst.conj().T @ Up) <= 1e-8
            def err(Xr, a, b):
                return np.linalg.norm(Xr - a.conj().T @ b) / (np.linalg.norm(a) * np.linalg.norm(b))
            bound = 1e-10 + 10.0 * loss
            assert err(X.XCtU, Ctp, Up) <= bound, (sysi, cyc, loss)
            assert err(X.XCtY, Ctp, Ups) <= bound, (sysi, cyc, loss)
            assert err(X.XYtC, Upst, Cp) <= bound, (sysi, cyc, loss)


def test_pencil_matches_explicit_products(rec_runs):
    """P, Q from the recurrences against (A^H Phi~)^H A Phi and (A^H Phi~)^H Phi:
    to 1e-7 where the Lanczos vectors stay biorthogonal (the first system and
    every first cycle), otherwise within the loss of biorthogonality."""
    for sysi, (A, AH, C, Ct, res) in enumerate(rec_runs):
        V, Vt = _cycle_data(res, None)
        assert res.pencils, sysi
        for cyc, d in _cycles(res):
            P2, Q2, _, _ = rc.harmonic_pencils(A, AH, d["Phi"], d["Phit"])
            i0 = (cyc - 1) * S
            lo = max(i0 - 1, 0)
            Ups, Upst = V[:, lo:i0 + S + 1], Vt[:, lo:i0 + S + 1]
            loss = np.linalg.norm(Upst.conj().T @ Ups - np.eye(Ups.shape[1]))
            if C is not None:
                loss += np.linalg.norm(C.conj().T @ Upst) + np.linalg.norm(Ct.conj().T @ Ups)
            bound = 1e-7 if loss < 1e-5 else 10.0 * loss
            assert _rel(d["P"], P2) <= bound, (sysi, cyc, d["case"], loss)
            assert _rel(d["Q"], Q2) <= bound, (sysi, cyc, d["case"], loss)


@pytest.mark.parametrize("cplx", [False, True], ids=["real", "complex"])
def test_recurrence_setup_solves_like_explicit(cplx):
    """The whole sequence with the Sec. 4.4 set-up: same iteration counts as
    the explicit-product set-up, recycling still pays (fewer iterations than
    BiCG from the second system on), C~^H C = I after every update."""
    rec = _run_sequence(nsys=4, setup="recurrence", keep=False, cplx=cplx)
    exp = _run_sequence(nsys=4, setup="explicit", keep=False, cplx=cplx)
    bicg_first = rec[0][4].iters
    for (A, AH, C, Ct, r), (_, _, _, _, e) in zip(rec, exp):
        assert r.status == "ok" and r.relres <= 1e-8 and r.relres_dual <= 1e-8
        assert abs(r.iters - e.iters) <= 1, (r.iters, e.iters)
        if C is not None:
            assert np.linalg.norm(Ct.conj().T @ C - np.eye(C.shape[1])) <= 1e-12
            assert r.iters < bicg_first
