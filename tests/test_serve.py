"""Serving loop: continuous admission by HBM budget, overlapping solves on
several streams; every request's answer is the same alone and in the mix."""
import numpy as np
import pytest

from synth import workloads as W

pytestmark = pytest.mark.gpu


def _requests(n=10):
    from paper_1012_5379_amd.serve import request_from_workload
    reqs = []
    for i in range(n):
        if i % 3 == 2:
            w = W.small(dim=3, n=12 + 4 * (i % 2), m=2, beta=0.4, kh=0.4, item=i, nrhs=1 + i % 3, cycle_prec=1)
        else:
            w = W.small(dim=2, n=48 + 16 * (i % 4), m=6, beta=0.3 + 0.05 * (i % 3), kh=0.5, item=i,
                        nrhs=1 + i % 4, cycle_prec=i % 2)
        reqs.append(request_from_workload(w.with_(tol=1e-7), rid=i, arrival=0.002 * i))
    return reqs


def _serve(reqs, streams, budget=None, batch=4, realtime=True, graphs=False):
    from paper_1012_5379_amd.serve import Engine
    eng = Engine(hbm_budget=budget, streams=streams, batch=batch, graphs=graphs)
    done = eng.run(reqs, realtime=realtime)
    eng.close()
    return {r.rid: r for r in done}, eng


def test_alone_equals_mix():
    """Each request solved alone (one stream, one at a time, no batching) and
    in the mix (four streams, every request queued at once, same-class
    requests batched into shared operators) gives bit-identical solutions and
    counts."""
    alone, _ = _serve(_requests(), streams=1, batch=1)
    mixed, eng = _serve(_requests(), streams=4, batch=4, realtime=False)
    assert eng.batches >= 1
    assert set(alone) == set(mixed) and len(alone) == 10
    for rid in alone:
        a, m = alone[rid], mixed[rid]
        assert a.status == 0 and m.status == 0
        assert [i["iterations"] for i in a.infos] == [i["iterations"] for i in m.infos]
        assert np.array_equal(a.u, m.u)
        assert all(i["relres_true"] <= 1e-7 for i in m.infos)


def test_graph_replay_equals_eager():
    """Served operators replaying captured graphs (four streams, batching on)
    give the eager engine's solutions and counts bit for bit."""
    eager, _ = _serve(_requests(), streams=4, batch=4, realtime=False)
    graphs, _ = _serve(_requests(), streams=4, batch=4, realtime=False, graphs=True)
    assert set(eager) == set(graphs)
    for rid in eager:
        a, g = eager[rid], graphs[rid]
        assert a.status == 0 and g.status == 0
        assert [i["iterations"] for i in a.infos] == [i["iterations"] for i in g.infos]
        assert np.array_equal(a.u, g.u)


def test_served_answers_match_the_oracle():
    """Every served request (batched, overlapping) against the FP64 oracle:
    complex128-cycle requests reach the oracle's answer at the same tolerance
    (iterations +-1, solution within 1e-10); complex64-cycle requests reach the
    tolerance by the oracle's own H, their solution within ten times the
    error floor of a solve stopping there (or 1e-5) of the oracle's 1e-12
    answer."""
    from oracle.oracle import Oracle, Params
    reqs = _requests()
    done, _ = _serve(reqs, streams=4, batch=4, realtime=False)
    for r in reqs:
        d = done[r.rid]
        p = {k: v for k, v in r.params.items() if k != "cycle_prec"}
        orc = Oracle(Params(**p), r.phi)
        for q in range(r.nrhs):
            chi = r.chi[q]
            uo, io = orc.fgmres(chi, tol=r.tol, restart=r.restart, maxit=r.maxit)
            if r.params["cycle_prec"] == 0:
                e = np.linalg.norm(d.u[q] - uo) / np.linalg.norm(uo)
                assert abs(d.infos[q]["iterations"] - io.iterations) <= 1, (r.rid, q)
                assert e <= 1e-10, (r.rid, q, e)
            else:
                rr = np.linalg.norm(chi - orc.apply(d.u[q], which=0, l=0)) / np.linalg.norm(chi)
                ut, _ = orc.fgmres(chi, tol=1e-12, restart=r.restart, maxit=4000)
                floor = np.linalg.norm(uo - ut) / np.linalg.norm(ut)
                e = np.linalg.norm(d.u[q] - ut) / np.linalg.norm(ut)
                assert rr <= r.tol, (r.rid, q, rr)
                assert e <= max(1e-5, 10 * floor), (r.rid, q, e, floor)


def test_admission_respects_budget():
    """A budget that holds only the largest request at a time still serves
    every request, never exceeding the budget: neither by the engine's own
    count nor by the device memory torch actually handed out."""
    import torch
    reqs = _requests(6)
    need = max(r.workspace_bytes() for r in reqs)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    done, eng = _serve(reqs, streams=4, budget=need)
    peak = torch.cuda.max_memory_allocated() - base
    assert len(done) == 6 and all(r.status == 0 for r in done.values())
    assert eng.high_water <= need
    assert peak <= need + (1 << 20)   # allocation granularity


def test_oversized_request_rejected():
    from paper_1012_5379_amd.serve import Engine
    reqs = _requests(1)
    eng = Engine(hbm_budget=reqs[0].workspace_bytes() - 1, streams=1)
    with pytest.raises(ValueError):
        eng.submit(reqs[0])
    eng.close()


def test_repeated_problem_reuses_hierarchy():
    """The same problem submitted twice is built once (LRU cache hit) and gives
    the same answer bit for bit."""
    from paper_1012_5379_amd.serve import request_from_workload
    w = W.small(dim=2, n=64, m=6, beta=0.35, kh=0.5, item=42, nrhs=2, cycle_prec=1).with_(tol=1e-7)
    reqs = [request_from_workload(w, rid=i, arrival=0.0) for i in range(2)]
    done, eng = _serve(reqs, streams=1, batch=1)
    assert eng.cache_hits == 1
    assert done[0].status == 0 and done[1].status == 0
    assert np.array_equal(done[0].u, done[1].u)
