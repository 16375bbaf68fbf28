"""GPU checks of the continuous-batching request loop: every request's
results are the same alone and in the mix (bitwise: each request has its own
handle, stream and workspace, and every reduction runs in a fixed order),
every system reaches the FP64 true residual 1e-8 in the FP32-inner /
FP64-outer mode, and sampled requests agree with the oracle's simulation of
the same arithmetic to 1e-6."""
import numpy as np
import pytest

import oracle
from paper_1010_0762_amd import serving
from paper_1010_0762_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _trace():
    rng = np.random.default_rng(wl.BASE_SEED + 55)
    out = []
    t = 0.0
    for rid in range(8):
        t += rng.exponential(0.002)
        out.append(wl.Request(rid, t, int(rng.choice([16, 20, 24])),
                              tuple(float(v) for v in rng.uniform(1.0, 50.0, 3)),
                              int(rng.integers(3, 6)), int(rng.choice([10, 20])),
                              wl.BASE_SEED + 5000 + rid))
    return out


def test_alone_vs_mix_bitwise_and_converged():
    reqs = _trace()
    mix = serving.Server(slots=4, keep_solutions=True).run(reqs)
    alone = serving.Server(slots=1, keep_solutions=True).run(reqs)
    for a, m in zip(alone, mix):
        assert a.rid == m.rid
        assert [s["iters"] for s in a.stats] == [s["iters"] for s in m.stats]
        for (xa, xta), (xm, xtm) in zip(a.solutions, m.solutions):
            assert np.array_equal(xa, xm) and np.array_equal(xta, xtm)
        for st in m.stats:
            assert st["status"] == 0 and st["relres"] <= 1e-8 and st["relres_dual"] <= 1e-8
    summ = serving.latency_summary(mix)
    assert summ["all_converged"] and summ["p99_s"] >= summ["p50_s"] > 0


def test_served_solutions_match_oracle():
    reqs = _trace()[:2]
    res = serving.Server(slots=2, keep_solutions=True).run(reqs)
    for req, r in zip(reqs, res):
        A = wl.convdiff(req.edge, 3, req.beta)
        U = Ut = None
        for j in range(req.nsys):
            b, bt = wl.request_rhs(req, j)
            x, xt, info, (U, Ut) = oracle.mixed_refine(A, b, bt, U, Ut, k=req.k, s=40, tol=1e-8,
                                                       inner_tol=1e-5)
            xg, xtg = r.solutions[j]
            assert np.linalg.norm(xg - x) / np.linalg.norm(x) <= 1e-6
            assert np.linalg.norm(xtg - xt) / np.linalg.norm(xt) <= 1e-6


@pytest.mark.parametrize("batched", [False, True])
def test_alone_vs_mix_config5_edges(batched):
    """Requests on the configuration-5 grid edges 32, 64 and 96 (n up to
    884736), two systems each, served three at a time and one at a time, with
    and without launch batching (the 96^3 request runs unbatched: batching
    takes requests of at most 64^3): per request the same iteration counts and
    bitwise the same solutions, every system at the FP64 true residual 1e-8."""
    reqs = [wl.Request(rid, 0.001 * rid, edge, beta, 2, k, wl.BASE_SEED + 7000 + rid)
            for rid, (edge, beta, k) in enumerate([(64, (20.0, 10.0, 5.0), 20),
                                                   (96, (30.0, 12.0, 4.0), 10),
                                                   (32, (45.0, 3.0, 17.0), 20)])]
    print("case config-5 edges batched", batched, flush=True)
    mix = serving.Server(slots=3, keep_solutions=True, batched=batched).run(reqs)
    alone = serving.Server(slots=1, keep_solutions=True, batched=batched).run(reqs)
    for a, m in zip(alone, mix):
        assert a.rid == m.rid and a.edge == m.edge
        assert [s["iters"] for s in a.stats] == [s["iters"] for s in m.stats]
        for (xa, xta), (xm, xtm) in zip(a.solutions, m.solutions):
            assert np.array_equal(xa, xm) and np.array_equal(xta, xtm)
        for st in m.stats:
            assert st["status"] == 0 and st["relres"] <= 1e-8 and st["relres_dual"] <= 1e-8
