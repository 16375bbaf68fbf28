"""Continuous batching of iteration launches (rbicg_batch_*): several handles
of different sizes and vector types, solving concurrently from host threads
with their chunks launched together, give bitwise the results of the same
handles solving alone; the batch reports launches that held several chunks."""
import threading

import numpy as np
import pytest

from paper_1010_0762_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _cases():
    rng = np.random.default_rng(91)
    out = []
    # (matrix, prec, k, right-hand sides of two systems)
    for edge, prec in ((20, "f64"), (24, "mixed"), (68, "f64"), (66, "mixed")):
        A = wl.convdiff(edge, 3, (20.0, 10.0, 5.0))
        rhs = [(rng.standard_normal(A.n), rng.standard_normal(A.n)) for _ in range(2)]
        out.append((A, prec, 10, rhs))
    A = wl.random_sparse(2000, 6, seed=5, diag_shift=8.0, complex_vals=True)
    rhs = [(rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n),
            rng.standard_normal(A.n) + 1j * rng.standard_normal(A.n)) for _ in range(2)]
    out.append((A, "c128", 8, rhs))
    return out


def _run(case, batch=None, stream=None):
    from paper_1010_0762_amd.solver import Solver
    A, prec, k, rhs = case
    dt = torch.complex128 if prec == "c128" else torch.float64
    with torch.cuda.stream(stream) if stream is not None else torch.cuda.stream(torch.cuda.current_stream()):
        S = Solver(A, k=k, s=40, prec=prec, stream=stream, batch=batch)
        res = []
        for j, (b, bt) in enumerate(rhs):
            if j:
                S.update_recycle()
            x, xt, st = S.solve(torch.as_tensor(b, dtype=dt, device="cuda"),
                                torch.as_tensor(bt, dtype=dt, device="cuda"),
                                tol=1e-10 if prec == "mixed" else 1e-8)
            res.append((x.cpu(), xt.cpu(), st))
        S.close()
    return res


@pytest.mark.parametrize("graphs", [False, True])
def test_batched_solves_bitwise_equal_alone(graphs):
    """With graphs, every launch set is captured once per table buffer and
    shape and replayed: the replays (many per solve, with the solves' own
    eager work and synchronizations in between) give the same bits as the
    solves alone."""
    from paper_1010_0762_amd.solver import Batch
    cases = _cases()
    alone = [_run(c) for c in cases]
    B = Batch(max_slots=16, window_us=200.0, graphs=graphs)
    streams = [torch.cuda.Stream() for _ in cases]
    torch.cuda.synchronize()
    out = [None] * len(cases)
    errs = []

    def work(i):
        try:
            out[i] = _run(cases[i], batch=B, stream=streams[i])
        except Exception as e:  # surfaced below
            errs.append(e)

    th = [threading.Thread(target=work, args=(i,)) for i in range(len(cases))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs, errs
    stats = B.stats()
    print("batch", stats, flush=True)
    for i, (a, b) in enumerate(zip(alone, out)):
        for j, ((xa, xta, sa), (xb, xtb, sb)) in enumerate(zip(a, b)):
            print(i, j, cases[i][1], cases[i][0].n, "iters", sa["iters"], sb["iters"], flush=True)
            assert sa["status"] == 0 and sb["status"] == 0
            assert sa["iters"] == sb["iters"], (i, j)
            assert torch.equal(xa, xb) and torch.equal(xta, xtb), (i, j)
    assert stats["launches"] > 0 and stats["max_chunks_per_launch"] >= 2
    if graphs:
        assert stats["graph_replays"] > 0 and stats["graph_captures"] > 0
        assert stats["graph_replays"] + stats["graph_captures"] == stats["launches"]
    else:
        assert stats["graph_replays"] == 0 and stats["graph_captures"] == 0
    B.close()


def test_more_solves_than_slots():
    """Twenty small solves released together on their own threads and
    streams share a batch of sixteen slots (a window long enough that chunks
    accumulate): launch sets fill up to the sixteen slots and no further,
    chunks beyond that go to the next set, and every solve gives the bits it
    gives alone."""
    from paper_1010_0762_amd.solver import Batch, Solver
    rng = np.random.default_rng(17)
    cases = []
    for i in range(20):
        A = wl.convdiff(14 + (i % 5), 3, (10.0 + i, 5.0, 2.0))
        cases.append((A, "f64", 10, [(rng.standard_normal(A.n), rng.standard_normal(A.n))]))
    alone = [_run(c) for c in cases]
    B = Batch(max_slots=16, window_us=50000.0)
    streams = [torch.cuda.Stream() for _ in cases]
    solvers, rhs = [], []
    for (A, prec, k, r), st in zip(cases, streams):
        with torch.cuda.stream(st):
            solvers.append(Solver(A, k=k, s=40, prec=prec, stream=st, batch=B))
            b, bt = r[0]
            rhs.append((torch.as_tensor(b, device="cuda"), torch.as_tensor(bt, device="cuda")))
    torch.cuda.synchronize()
    gate = threading.Barrier(len(cases))
    out = [None] * len(cases)
    errs = []

    def work(i):
        try:
            gate.wait()
            with torch.cuda.stream(streams[i]):
                x, xt, st = solvers[i].solve(rhs[i][0], rhs[i][1], tol=1e-8)
                out[i] = (x.cpu(), xt.cpu(), st)
        except Exception as e:  # surfaced below
            errs.append(e)

    th = [threading.Thread(target=work, args=(i,)) for i in range(len(cases))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs, errs
    stats = B.stats()
    print("batch", stats, flush=True)
    # sixteen in the runs so far; at least twelve leaves room for a slow
    # thread start without losing what the test shows
    assert 12 <= stats["max_chunks_per_launch"] <= 16
    for i, (a, b) in enumerate(zip(alone, out)):
        (xa, xta, sa), (xb, xtb, sb) = a[0], b
        assert sa["status"] == 0 and sb["status"] == 0
        assert sa["iters"] == sb["iters"], i
        assert torch.equal(xa, xb) and torch.equal(xta, xtb), i
    for S in solvers:
        S.close()
    B.close()
