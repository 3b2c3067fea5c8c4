"""Full-size workloads on the GPU, in the launch configuration bench.py times.

Checks use what the oracle can afford at these sizes: whole-vector operator and
V-cycle comparisons, the oracle's stored answers of the 2-D 1024^2 and 2048^2
solves (tests/golden/c2_oracle.json, c3_oracle.json, written by
tests/golden/make_golden.py), and properties that hold at any size (true FP64
residual recomputed by the oracle's own H)."""
import json
import os

import numpy as np
import pytest

from synth import workloads as W
from tests.gpu_common import dev, host, note, pair, rel, rvec, torch_cuda

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _relres(orc, u, chi):
    r = chi - orc.apply(u, which=0, l=0)
    return np.linalg.norm(r) / np.linalg.norm(chi)


def test_c2_full_size_stencil_and_vcycle():
    """1024^2 + 32 layers, complex128: H, M (every level) and one V-cycle
    against the oracle on whole vectors (1e-12)."""
    torch_cuda()
    w = W.c2()
    op, orc = pair(w, max_rhs=1, cycle_prec=0)
    for l in (0, 1, op.levels - 1):
        x = rvec(orc.shape(l), 300 + l)[None]
        y = host(op.apply(dev(x, op.cdtype), which=1, level=l))[0]
        e = rel(y, orc.apply(x[0], which=1, l=l))
        note(f"  M level {l}: {e:.2e}")
        assert e <= 1e-12
    b = w.chi / np.linalg.norm(w.chi)
    x = host(op.vcycle(dev(b, op.cdtype)))[0]
    e = rel(x, orc.vcycle(b[0]))
    note(f"  vcycle: {e:.2e}")
    assert e <= 1e-12


def _golden(name):
    with open(os.path.join(GOLDEN, f"{name}_oracle.json")) as f:
        return json.load(f)


def _against_golden(u, g, entry):
    """Norm-wise error of u against the stored oracle answer `entry` on the
    stored sample of entries, and the largest relative error of u's inner
    products with the stored seeded probe vectors (a whole-vector check)."""
    flat = u.ravel()
    idx = np.array(g["sample_index"])
    ref = np.array(entry["sample_re"]) + 1j * np.array(entry["sample_im"])
    es = np.linalg.norm(flat[idx] - ref) / np.linalg.norm(ref)
    ep = 0.0
    for item, (re, im) in zip(g["probe_items"], entry["proj"]):
        q = W.rand_cvec(u.shape, item=item, cfg_id=g["probe_cfg_id"]).ravel()
        pr = complex(re, im)
        ep = max(ep, abs(np.vdot(q, flat) - pr) / abs(pr))
    return es, ep


def test_c2_full_size_solve_matches_oracle_answer():
    """The benchmarked solve: iterations within 1 of the oracle's, true FP64
    residual <= 1e-6 (recomputed by the oracle's H), the solution within 1e-10
    of the oracle's stored answer on 16384 sampled entries and in its inner
    products with four seeded random vectors (same tolerance path)."""
    import torch
    g = _golden("c2")
    w = W.c2()
    op, orc = pair(w, max_rhs=1, cycle_prec=0)
    u, rc, infos = op.solve(dev(w.chi, torch.complex128), tol=1e-6, restart=30, maxit=3000)
    u = host(u)[0]
    rr = _relres(orc, u, w.chi[0])
    es, ep = _against_golden(u, g, g)
    note(f"  gpu its {infos[0]['iterations']} oracle {g['iterations']} relres {rr:.3e} sample err {es:.2e} "
         f"probe err {ep:.2e}")
    assert rc == 0 and infos[0]["converged"]
    assert abs(infos[0]["iterations"] - g["iterations"]) <= 1
    assert rr <= 1e-6
    assert abs(np.linalg.norm(u) - g["u_norm"]) <= 1e-10 * g["u_norm"]
    assert es <= 1e-10 and ep <= 1e-10


def test_c3_full_size_operators_and_vcycle_fp64():
    """2048^2 three-layer model, complex128: H and M on the finest level and
    one V-cycle against the oracle on whole vectors (1e-12)."""
    torch_cuda()
    w = W.c3(cycle_prec=0)
    op, orc = pair(w, max_rhs=1, cycle_prec=0)
    x = rvec(orc.shape(0), 310)[None]
    for which in (0, 1):
        y = host(op.apply(dev(x, op.cdtype), which=which, level=0))[0]
        e = rel(y, orc.apply(x[0], which=which, l=0))
        note(f"  {'HM'[which]} level 0: {e:.2e}")
        assert e <= 1e-12
    b = rvec(orc.shape(0), 311)[None]
    xv = host(op.vcycle(dev(b, op.cdtype)))[0]
    e = rel(xv, orc.vcycle(b[0]))
    note(f"  vcycle: {e:.2e}")
    assert e <= 1e-12


def test_c3_fp64_solve_matches_oracle_answer():
    """The all-FP64 solve of the 2048^2 three-layer model: iterations within 1
    of the oracle's stored count and the solution within 1e-10 of its stored
    answer (16384 sampled entries, four seeded probes)."""
    import torch
    g = _golden("c3")
    w = W.c3(cycle_prec=0)
    op, orc = pair(w, max_rhs=1, cycle_prec=0)
    u, rc, infos = op.solve(dev(w.chi, torch.complex128), tol=1e-6, restart=30, maxit=5000)
    u = host(u)[0]
    es, ep = _against_golden(u, g, g)
    note(f"  fp64: its {infos[0]['iterations']} (oracle {g['iterations']}), relres {infos[0]['relres_true']:.2e}, "
         f"{infos[0]['seconds']:.2f}s; sample err {es:.2e} probe err {ep:.2e}")
    assert rc == 0 and infos[0]["converged"]
    assert abs(infos[0]["iterations"] - g["iterations"]) <= 1
    assert es <= 1e-10 and ep <= 1e-10


def test_c3_mixed_precision_against_the_oracle():
    """complex64 cycle, complex128 outer: true FP64 relres <= 1e-6 (recomputed by
    the oracle's H), and the solution error against the oracle's answer at
    1e-12 stated beside the floor every solve stopping at 1e-6 has (the
    oracle's own 1e-6 answer against its 1e-12 one): within three times that
    floor, or 1e-5 if larger."""
    import torch
    g = _golden("c3")
    w = W.c3()
    op, orc = pair(w, max_rhs=1, cycle_prec=1)
    u, rc, infos = op.solve(dev(w.chi, torch.complex128), tol=1e-6, restart=30, maxit=5000)
    u = host(u)[0]
    rr = _relres(orc, u, w.chi[0])
    es, ep = _against_golden(u, g, g["tight"])
    floor = g["floor"]
    note(f"  c64 cycle: its {infos[0]['iterations']} relres {rr:.2e} ({infos[0]['seconds']:.2f}s); error against "
         f"the 1e-12 answer {es:.2e} (probes {ep:.2e}); floor of a 1e-6 solve {floor:.2e}")
    assert rc == 0 and infos[0]["converged"]
    assert rr <= 1e-6
    assert es <= max(1e-5, 3 * floor)


def test_c4_fp64_headline_solve_matches_oracle_answer():
    """The headline benchmark's solve as bench.py runs it: 128^3 + 16 layers,
    all 16 point sources in one launch sequence, complex128 throughout, tuned
    knobs.  The first and the last right-hand side: iterations within 1 of the
    oracle's, true FP64 residual <= 1e-6 (recomputed by the oracle's H), the
    solution within 1e-10 of the oracle's stored answer on 8192 sampled entries
    and in its inner products with four seeded random vectors."""
    import torch
    from paper_1012_5379_amd import Operator
    from oracle.oracle import Oracle, Params
    g = _golden("c4")
    w = W.c4(cycle_prec=0)
    op = Operator(dict(w.params(), cycle_prec=0, max_rhs=w.nrhs, restart=w.restart), w.phi, tuned=True)
    orc = Oracle(Params(**w.params()), w.phi)
    u, rc, infos = op.solve(dev(w.chi, torch.complex128), tol=1e-6, restart=30, maxit=3000)
    u = host(u)
    assert rc == 0 and all(i["converged"] for i in infos)
    for r in (0, 15):
        e = g[f"rhs{r}"]
        rr = _relres(orc, u[r], w.chi[r])
        es, ep = _against_golden(u[r], g, e)
        note(f"  rhs {r}: gpu its {infos[r]['iterations']} oracle {e['iterations']} relres {rr:.3e} "
             f"sample err {es:.2e} probe err {ep:.2e}")
        assert abs(infos[r]["iterations"] - e["iterations"]) <= 1
        assert rr <= 1e-6
        assert abs(np.linalg.norm(u[r]) - e["u_norm"]) <= 1e-10 * e["u_norm"]
        assert es <= 1e-10 and ep <= 1e-10


def test_c4_3d_sixteen_rhs_full_size():
    """128^3 + 16 layers, 16 point sources in one launch sequence, complex64
    cycle: every RHS converges (true residual by the oracle's H), the first
    one's solution lies within ten times the error floor of a 1e-6 solve (or
    1e-5) of the oracle's 1e-12 answer, and it matches a separate single-RHS
    solve of the same operator."""
    import torch
    w = W.c4()
    op, orc = pair(w, max_rhs=16, cycle_prec=1)
    u, rc, infos = op.solve(dev(w.chi, torch.complex128), tol=1e-6, restart=30, maxit=3000)
    u = host(u)
    its = [i["iterations"] for i in infos]
    note(f"  16 RHS: iterations {its}, seconds {infos[0]['seconds']:.2f}")
    assert rc == 0 and all(i["converged"] for i in infos)
    for r in (0, 7, 15):
        rr = _relres(orc, u[r], w.chi[r])
        note(f"  rhs {r}: relres {rr:.2e}")
        assert rr <= 1e-6
    g = _golden("c4")
    es, ep = _against_golden(u[0], g, g["tight0"])
    note(f"  rhs 0 against the oracle's 1e-12 answer: sample err {es:.2e} probe err {ep:.2e} "
         f"(floor of a 1e-6 solve {g['floor0']:.2e})")
    assert es <= max(1e-5, 10 * g["floor0"]) and ep <= max(1e-5, 10 * g["floor0"])
    # batching does not change a RHS's result beyond rounding
    u1, rc1, inf1 = op.solve(dev(w.chi[:1], torch.complex128), tol=1e-6, restart=30, maxit=3000)
    assert rc1 == 0 and inf1[0]["iterations"] == infos[0]["iterations"]
    assert np.array_equal(host(u1)[0], u[0])
