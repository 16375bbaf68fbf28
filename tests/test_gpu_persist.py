"""Recycle-state persistence across handles (save_recycle / load_recycle) and
bilinear forms along a sequence (bilinear_sequence), on the GPU.

Bars: a sequence resumed from a saved space in a fresh handle is bitwise the
one continued in the original handle (same basis values go through the same
installation, Sec. 4.3, and the same deterministic kernels); the bilinear forms
u_j^H A_j^{-1} w_j match dense direct values within the quadratic error bound
the solver reports (plus rounding)."""
import os

import numpy as np
import pytest

from paper_1010_0762_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _t(v):
    return torch.as_tensor(np.ascontiguousarray(v), device="cuda", dtype=torch.float64)


def test_resume_from_saved_space_is_bitwise(tmp_path):
    from paper_1010_0762_amd.solver import Solver
    seq = wl.cfg1_sequence(nsys=3)
    b, bt = _t(seq.b[0]), _t(seq.bt[0])
    S1 = Solver(seq.mats[0], k=seq.k, s=seq.s)
    S1.solve(b, bt, tol=seq.tol)
    path = os.path.join(tmp_path, "space.npz")
    S1.save_recycle(path)
    with np.load(path, allow_pickle=False) as f:
        assert f["U"].shape[1] > 0 and int(f["n"]) == seq.mats[0].n
    # continue in the original handle
    S1.update_recycle(seq.mats[1])
    x1, xt1, st1 = S1.solve(b, bt, tol=seq.tol)
    # resume in a fresh handle on the next matrix
    S2 = Solver(seq.mats[1], k=seq.k, s=seq.s)
    S2.load_recycle(path)
    x2, xt2, st2 = S2.solve(b, bt, tol=seq.tol)
    assert st1["k_used"] == st2["k_used"] > 0
    assert st1["iters"] == st2["iters"]
    assert torch.equal(x1, x2) and torch.equal(xt1, xt2)
    with pytest.raises(ValueError):
        Solver(wl.convdiff(8, 2, [1.0, 1.0]), k=4, s=40).load_recycle(path)


def test_bilinear_sequence_matches_direct():
    from paper_1010_0762_amd.solver import Solver
    seq = wl.cfg1_sequence(nsys=3)
    rng = np.random.default_rng(17)
    n = seq.mats[0].n
    items, exact = [], []
    for j in range(3):
        u, w = rng.standard_normal(n), rng.standard_normal(n)
        D = seq.mats[j].to_dense()
        exact.append(float(u @ np.linalg.solve(D, w)))
        items.append((seq.mats[j] if j else None, _t(u), _t(w)))
    S = Solver(seq.mats[0], k=seq.k, s=seq.s)
    out = S.bilinear_sequence(items, tol=1e-10)
    for (v, err, st), ref in zip(out, exact):
        assert st["status"] == 0
        # the error u^H A^{-1} w - value = r~^H A^{-1} r is quadratic in the residuals
        assert abs(v - ref) <= 1e-9 * abs(ref) + 1e3 * err, (v, ref, err)
    assert out[2][2]["k_used"] > 0
