"""Batched bilinear forms u_i^H A^{-1} w_i (Sec. 1) through
rbicg_bilinear_batch: S pairs on one matrix and one recycle space in one set
of launches per iteration.  Values against direct dense solves within the
quadratic error bound ||r|| ||r~|| ||A^{-1}||, and against the oracle's
single-pair bilinear form; along a sequence of matrices the batch recycles
the space its update pair built."""
import numpy as np
import pytest

import oracle
from paper_1010_0762_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _tc(M):
    return torch.as_tensor(np.ascontiguousarray(M, dtype=np.complex128)).to("cuda")


@pytest.mark.parametrize("cplx", [False, True], ids=["real", "complex"])
def test_bilinear_batch_matches_direct_and_oracle(cplx):
    from paper_1010_0762_amd.solver import Solver
    seq = wl.cfg1_sequence(3)
    rng = np.random.default_rng(71)
    # complex: sixteen pairs, the largest batch (two sets of the update
    # kernel's eight shifts per iteration)
    S, n = (16 if cplx else 8), seq.mats[0].n
    H = Solver(seq.mats[0], k=10, s=40, prec="c128")
    mean_iters = []
    for j, A in enumerate(seq.mats):
        if j:
            H.update_recycle(A)
        U = rng.standard_normal((S, n))
        W = rng.standard_normal((S, n))
        if cplx:
            U = U + 1j * rng.standard_normal((S, n))
            W = W + 1j * rng.standard_normal((S, n))
        out = H.bilinear_batch(_tc(U), _tc(W), tol=1e-8)
        D = A.to_dense()
        Dinv = np.linalg.inv(D)
        ainv = np.linalg.norm(Dinv, 2)
        its = []
        for i, (val, err, st) in enumerate(out):
            exact = np.vdot(U[i], Dinv @ W[i])
            assert st["status"] == 0, (j, i, st)
            assert abs(val - exact) <= err * ainv * 1.001 + 1e-12 * abs(exact), (j, i, val, exact, err)
            assert abs(val - exact) <= 1e-10 * abs(exact), (j, i)
            its.append(st["iters"])
            if i < 2:   # the oracle's single-pair form (Sec. 1 correction term)
                ov, _, _ = oracle.bilinear(A, U[i], W[i], tol=1e-8)
                assert abs(val - ov) <= 1e-8 * abs(exact)
        print(j, "iters per pair", its, "k used", [o[2]["k_used"] for o in out], flush=True)
        mean_iters.append(np.mean(its))
        if j:
            assert any(o[2]["k_used"] > 0 for o in out)
    # recycling: later batches need fewer iterations than the first
    assert max(mean_iters[1:]) < mean_iters[0]
    H.close()
