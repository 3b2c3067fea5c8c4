"""GPU parity: every operation of the hot path through the C ABI against the
FP64 CPU oracle on identical seeded inputs.

Bars: complex128 path, norm-wise relative error <= 1e-12 per operation; end to
end, the outer iteration count equals the oracle's +-1 and the solution agrees
to 1e-10.  complex64 cycle: per-operation errors are stated by the tolerances
below (single-precision rounding of the cycle)."""
import numpy as np
import pytest

from synth import workloads as W
from tests.gpu_common import cases, dev, host, note, pair, rel, rvec, torch_cuda

pytestmark = pytest.mark.gpu

CASES = cases()
TOL64 = 1e-12
# complex64 cycle: about ten times the largest error observed on these cases
TOL32 = {"apply": 1e-6, "restrict": 3e-6, "prolong": 5e-7, "coarse": 6e-6, "smooth": 6e-6, "vcycle": 6e-6}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    torch_cuda()
    w = CASES[request.param]()
    return request.param, w


def _ops(case, cycle_prec):
    name, w = case
    return pair(w, max_rhs=2, cycle_prec=cycle_prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_stencil_every_level(case, prec):
    import torch
    op, orc = _ops(case, prec)
    tol = TOL64 if prec == 0 else TOL32["apply"]
    for l in range(op.levels):
        x = np.stack([rvec(orc.shape(l), 10 + l), rvec(orc.shape(l), 20 + l)])
        y = host(op.apply(dev(x, op.cdtype), which=1, level=l))
        for r in range(2):
            e = rel(y[r], orc.apply(x[r], which=1, l=l))
            note(f"  M level {l} rhs {r}: {e:.2e}")
            assert e <= tol
    x = np.stack([rvec(orc.shape(0), 30), rvec(orc.shape(0), 31)])
    y = host(op.apply(dev(x, torch.complex128), which=0, level=0))
    for r in range(2):
        e = rel(y[r], orc.apply(x[r], which=0, l=0))
        note(f"  H rhs {r}: {e:.2e}")
        assert e <= TOL64


@pytest.mark.parametrize("prec", [0, 1])
def test_transfers_every_level(case, prec):
    op, orc = _ops(case, prec)
    for l in range(op.levels - 1):
        b = np.stack([rvec(orc.shape(l), 40 + l), rvec(orc.shape(l), 50 + l)])
        x = np.stack([rvec(orc.shape(l), 60 + l), rvec(orc.shape(l), 70 + l)]) * 1e-3
        bc = host(op.residual_restrict(dev(b, op.cdtype), dev(x, op.cdtype), level=l))
        ec = np.stack([rvec(orc.shape(l + 1), 80 + l), rvec(orc.shape(l + 1), 90 + l)])
        xp = host(op.prolong_correct(dev(ec, op.cdtype), dev(x, op.cdtype), level=l))
        for r in range(2):
            er = rel(bc[r], orc.restrict(b[r] - orc.apply(x[r], 1, l), l))
            ep = rel(xp[r], orc.prolong_add(ec[r], x[r], l))
            note(f"  level {l} rhs {r}: restrict {er:.2e} prolong {ep:.2e}")
            assert er <= (TOL64 if prec == 0 else TOL32["restrict"])
            assert ep <= (TOL64 if prec == 0 else TOL32["prolong"])


@pytest.mark.parametrize("prec", [0, 1])
def test_coarse_solve(case, prec):
    op, orc = _ops(case, prec)
    L = op.levels - 1
    b = np.stack([rvec(orc.shape(L), 100), rvec(orc.shape(L), 101)])
    x = host(op.coarse_solve(dev(b, op.cdtype)))
    for r in range(2):
        e = rel(x[r], orc.coarse_solve(b[r]))
        note(f"  coarse rhs {r}: {e:.2e}")
        assert e <= (TOL64 if prec == 0 else TOL32["coarse"])


@pytest.mark.parametrize("prec", [0, 1])
def test_gmres_sweep_every_level(case, prec):
    op, orc = _ops(case, prec)
    for l in range(op.levels):
        b = np.stack([rvec(orc.shape(l), 110 + l), rvec(orc.shape(l), 120 + l)])
        x0 = np.stack([rvec(orc.shape(l), 130 + l), rvec(orc.shape(l), 140 + l)]) * 1e-4
        xd = dev(x0, op.cdtype)
        x = host(op.smooth(dev(b, op.cdtype), xd, level=l))
        for r in range(2):
            xo, k = orc.gmres_sweep(b[r], x0[r], l=l)
            e = rel(x[r], xo)
            note(f"  sweep level {l} rhs {r}: {e:.2e} (oracle steps {k})")
            assert e <= (TOL64 if prec == 0 else TOL32["smooth"])


@pytest.mark.parametrize("prec", [0, 1])
def test_vcycle(case, prec):
    op, orc = _ops(case, prec)
    b = np.stack([rvec(orc.shape(0), 150), rvec(orc.shape(0), 151)])
    x = host(op.vcycle(dev(b, op.cdtype)))
    for r in range(2):
        e = rel(x[r], orc.vcycle(b[r]))
        note(f"  vcycle rhs {r}: {e:.2e}")
        assert e <= (TOL64 if prec == 0 else TOL32["vcycle"])


def test_vcycle_repeatable_bitwise(case):
    """Deterministic reductions: the same cycle twice gives identical bits."""
    op, orc = _ops(case, 0)
    b = dev(np.stack([rvec(orc.shape(0), 160)] * 2), op.cdtype)
    x1 = host(op.vcycle(b))
    x2 = host(op.vcycle(b))
    assert np.array_equal(x1, x2)
    assert np.array_equal(x1[0], x1[1])   # batch position does not change the result


def test_fgmres_fp64_matches_oracle():
    """End to end on the 64^2 + 8 workload (k = 20, beta = 0.4): outer
    iterations +-1 and solution within 1e-10 of the oracle at tol 1e-6."""
    import torch
    w = W.c1()
    op, orc = pair(w, max_rhs=1, cycle_prec=0)
    u_o, info_o = orc.fgmres(w.chi[0], tol=1e-6, restart=30, maxit=500)
    u, rc, infos = op.solve(dev(w.chi, torch.complex128), tol=1e-6, restart=30, maxit=500)
    u = host(u)[0]
    note(f"  oracle its {info_o.iterations} gpu its {infos[0]['iterations']} relres {infos[0]['relres_true']:.3e}")
    assert rc == 0 and infos[0]["converged"]
    assert abs(infos[0]["iterations"] - info_o.iterations) <= 1
    e = rel(u, u_o)
    note(f"  solution vs oracle: {e:.2e}")
    assert e <= 1e-10
    # the true residual, recomputed independently by the oracle's H
    r = w.chi[0] - orc.apply(u, which=0, l=0)
    assert np.linalg.norm(r) / np.linalg.norm(w.chi[0]) <= 1e-6


@pytest.mark.parametrize("name", ["2d_ragged", "3d_ragged"])
def test_fgmres_fp64_multi_rhs(name):
    """Two right-hand sides solved together, each matching its own oracle solve."""
    import torch
    w = CASES[name]()
    chi = np.stack([w.chi[0], rvec(w.chi.shape[1:], 170)])
    op, orc = pair(w, max_rhs=2, cycle_prec=0)
    u, rc, infos = op.solve(dev(chi, torch.complex128), tol=1e-8, restart=20, maxit=400)
    u = host(u)
    assert rc == 0
    for r in range(2):
        uo, io = orc.fgmres(chi[r], tol=1e-8, restart=20, maxit=400)
        e = rel(u[r], uo)
        note(f"  rhs {r}: its gpu {infos[r]['iterations']} oracle {io.iterations} sol err {e:.2e}")
        assert abs(infos[r]["iterations"] - io.iterations) <= 1
        assert e <= 1e-10


def test_fgmres_bases_longer_than_32():
    """FGMRES(40): bases of up to 40 vectors (five groups of 8 inner products
    per column); iterations and solution match the oracle."""
    import torch
    w = CASES["2d_ragged"]()
    op, orc = pair(w, max_rhs=1, cycle_prec=0, restart=40)
    u, rc, infos = op.solve(dev(w.chi[:1], torch.complex128), tol=1e-10, restart=40, maxit=400)
    uo, io = orc.fgmres(w.chi[0], tol=1e-10, restart=40, maxit=400)
    e = rel(host(u)[0], uo)
    note(f"  its gpu {infos[0]['iterations']} oracle {io.iterations} sol err {e:.2e}")
    assert rc == 0 and io.iterations > 34
    assert abs(infos[0]["iterations"] - io.iterations) <= 1
    assert e <= 1e-10


def test_fgmres_mixed_precision_reaches_tolerance():
    """complex64 cycle, complex128 outer: true FP64 relres <= 1e-6 and the
    solution error against the tightly converged FP64 oracle is stated."""
    import torch
    w = W.c1()
    op, orc = pair(w, max_rhs=1, cycle_prec=1)
    u, rc, infos = op.solve(dev(w.chi, torch.complex128), tol=1e-6, restart=30, maxit=500)
    u = host(u)[0]
    assert rc == 0 and infos[0]["converged"]
    r = w.chi[0] - orc.apply(u, which=0, l=0)
    rr = np.linalg.norm(r) / np.linalg.norm(w.chi[0])
    u_ref, _ = orc.fgmres(w.chi[0], tol=1e-12, restart=30, maxit=2000)
    u6, i6 = orc.fgmres(w.chi[0], tol=1e-6, restart=30, maxit=2000)
    floor = rel(u6, u_ref)
    e = rel(u, u_ref)
    note(f"  mixed: its {infos[0]['iterations']} (fp64 oracle {i6.iterations}) relres {rr:.2e} "
         f"sol err {e:.2e} (floor of a 1e-6 solve: {floor:.2e})")
    assert rr <= 1e-6
    assert e <= max(1e-5, 10 * floor)


def test_solve_edge_cases():
    """Zero source -> zero solution in 0 iterations; maxit -> ENOCONV with the
    last iterate; a converged initial guess takes no iteration."""
    import torch
    from paper_1012_5379_amd import binding as B
    w = W.small(dim=2, n=24, m=4, item=9)
    op, orc = pair(w, max_rhs=2, cycle_prec=0)
    chi = np.stack([np.zeros(w.grid_shape, complex), w.chi[0]])
    u, rc, infos = op.solve(dev(chi, torch.complex128), tol=1e-8, restart=10, maxit=300)
    u = host(u)
    assert rc == 0
    assert infos[0]["iterations"] == 0 and not np.any(u[0])
    u2, rc2, inf2 = op.solve(dev(chi[1:], torch.complex128), tol=1e-14, restart=10, maxit=3)
    assert rc2 == B.CSG_ENOCONV and inf2[0]["iterations"] == 3 and not inf2[0]["converged"]
    u3, rc3, inf3 = op.solve(dev(chi[1:], torch.complex128), tol=1e-8, restart=10, maxit=300,
                             u0=dev(u[1:], torch.complex128))
    assert rc3 == 0 and inf3[0]["iterations"] == 0


@pytest.mark.parametrize("tail_max", ["0", "1200", "10000", "1000000000"])
def test_vcycle_any_tail_split(tail_max, monkeypatch):
    """The coarse-tail kernel (one workgroup per RHS for the small levels) and
    the multi-block passes compute the same cycle: every split point matches
    the oracle to 1e-12."""
    monkeypatch.setenv("CSG_TAIL_MAX", tail_max)
    w = CASES["2d_wide"]()
    op, orc = pair(w, max_rhs=2, cycle_prec=0)
    b = np.stack([rvec(orc.shape(0), 180), rvec(orc.shape(0), 181)])
    x = host(op.vcycle(dev(b, op.cdtype)))
    for r in range(2):
        e = rel(x[r], orc.vcycle(b[r]))
        note(f"  tail_max {tail_max} rhs {r}: {e:.2e}")
        assert e <= TOL64


@pytest.mark.parametrize("knob", ["CSG_TILES", "CSG_UP_TILES", "CSG_DOWN_TILES", "CSG_FUSE_UPD", "CSG_TAIL_LDS"])
@pytest.mark.parametrize("prec", [0, 1])
def test_vcycle_with_each_fused_path_off(knob, prec, monkeypatch):
    """Every fused path (tiled Arnoldi passes, tiled up and down passes, the
    coarse closing update applied by the finer up pass, the LDS tail) and the
    unfused passes it replaces compute the same cycle: with each one switched
    off the cycle still matches the oracle, on a ragged 2-D case whose levels
    take both kinds of pass."""
    monkeypatch.setenv(knob, "0")
    w = CASES["2d_wide"]()
    op, orc = pair(w, max_rhs=2, cycle_prec=prec)
    b = np.stack([rvec(orc.shape(0), 200), rvec(orc.shape(0), 201)])
    x = host(op.vcycle(dev(b, op.cdtype)))
    for r in range(2):
        e = rel(x[r], orc.vcycle(b[r]))
        note(f"  {knob}=0 prec {prec} rhs {r}: {e:.2e}")
        assert e <= (TOL64 if prec == 0 else TOL32["vcycle"])


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("tiles", ["1", "0"])
def test_fgmres_with_and_without_tiled_hdot(tiles, prec, monkeypatch):
    """w = H z and its inner products on the finest level's tiles, or over the
    plain chunked layout: two RHS, each matching its own oracle solve
    (complex128 cycle: iterations +-1 and solution to 1e-10; complex64 cycle:
    the true residual reaches the tolerance)."""
    import torch
    monkeypatch.setenv("CSG_HDOT_TILES", tiles)
    w = CASES["2d_ragged"]()
    chi = np.stack([w.chi[0], rvec(w.chi.shape[1:], 171)])
    op, orc = pair(w, max_rhs=2, cycle_prec=prec)
    u, rc, infos = op.solve(dev(chi, torch.complex128), tol=1e-8, restart=20, maxit=400)
    u = host(u)
    assert rc == 0
    for r in range(2):
        uo, io = orc.fgmres(chi[r], tol=1e-8, restart=20, maxit=400)
        e = rel(u[r], uo)
        note(f"  tiles {tiles} prec {prec} rhs {r}: its gpu {infos[r]['iterations']} oracle {io.iterations} "
             f"sol err {e:.2e} relres {infos[r]['relres_true']:.2e}")
        if prec == 0:
            assert abs(infos[r]["iterations"] - io.iterations) <= 1
            assert e <= 1e-10
        else:
            assert infos[r]["relres_true"] <= 1e-8


def test_fgmres_second_round_every_column(monkeypatch):
    """The outer second Gram-Schmidt round (taken only when the first round
    cancels) forced on every column: the solve still matches the oracle's
    iteration count and answer, and the selective solve to rounding."""
    import torch
    w = CASES["2d_ragged"]()
    chi = dev(w.chi[:1], torch.complex128)
    res = {}
    for force in ("0", "1"):
        monkeypatch.setenv("CSG_FORCE_CGS2", force)
        op, orc = pair(w, max_rhs=1, cycle_prec=0, restart=12)
        u, rc, infos = op.solve(chi, tol=1e-9, restart=12, maxit=400)
        assert rc == 0
        res[force] = (host(u)[0], infos[0]["iterations"])
    uo, info = orc.fgmres(w.chi[0], tol=1e-9, restart=12, maxit=400)
    note(f"  iterations: selective {res['0'][1]}, every column {res['1'][1]}, oracle {info.iterations}")
    assert abs(res["1"][1] - info.iterations) <= 1
    assert rel(res["1"][0], uo) <= 1e-8
    assert rel(res["1"][0], res["0"][0]) <= 1e-8


OUTER_MODES = {
    "lazy": {},                                        # second rounds applied by the next first projection
    "at_once": {"CSG_LAZY": "0"},                      # second rounds applied by k_proj1
    "two_pass": {"CSG_PROJ0W": "0"},                   # register kernel to 16 vectors, two-pass beyond
    "lazy_every_column": {"CSG_FORCE_CGS2": "1"},
    "at_once_every_column": {"CSG_FORCE_CGS2": "1", "CSG_LAZY": "0"},
    "proj0w_step_loads": {"CSG_PROJ0W_AHEAD": "0"},    # split first projection without loads a step ahead
    "proj0w_one_group": {"CSG_PROJ0W_GROUPS": "1"},    # its one-group steps (launches of many workgroups)
    "hdot_untiled": {"CSG_HDOT_TILES": "0"},           # 2-D: the chunked w = H z
    "slabs": {"CSG_SLAB_MIN": "0"},                    # 3-D: w = H z (and the cycle) on slabs
}


@pytest.mark.parametrize("mode", list(OUTER_MODES))
@pytest.mark.parametrize("name", ["2d_ragged", "3d_ragged"])
def test_fgmres_outer_orthogonalisation_modes(name, mode, monkeypatch):
    """FGMRES(48) with two RHS (columns of 1..48 basis vectors: the register,
    and every wavefront-split first projection) under each way of applying
    the second Gram-Schmidt round, with the chunked w = H z in 2-D and the
    slab one in 3-D:
    iterations +-1 and solution within 1e-10 of the oracle."""
    import torch
    for k, v in OUTER_MODES[mode].items():
        monkeypatch.setenv(k, v)
    w = CASES[name]()
    chi = np.stack([w.chi[0], rvec(w.chi.shape[1:], 480)])
    op, orc = pair(w, max_rhs=2, cycle_prec=0, restart=48)
    u, rc, infos = op.solve(dev(chi, torch.complex128), tol=1e-10, restart=48, maxit=600)
    u = host(u)
    assert rc == 0
    for r in range(2):
        uo, io = orc.fgmres(chi[r], tol=1e-10, restart=48, maxit=600)
        e = rel(u[r], uo)
        note(f"  {mode} rhs {r}: its gpu {infos[r]['iterations']} oracle {io.iterations} sol err {e:.2e}")
        assert abs(infos[r]["iterations"] - io.iterations) <= 1
        assert e <= 1e-10


def test_graph_replay_matches_eager(monkeypatch):
    """FGMRES iterations replayed from captured graphs (with eager restart and
    report work in between) give bit-identical results to eager launches."""
    import torch
    w = CASES["2d_ragged"]()
    chi = dev(np.stack([w.chi[0], rvec(w.chi.shape[1:], 190)]), torch.complex128)
    outs = []
    for graphs in ("1", "0", "1"):
        monkeypatch.setenv("CSG_GRAPHS", graphs)
        op, orc = pair(w, max_rhs=2, cycle_prec=0, restart=12)
        u, rc, infos = op.solve(chi, tol=1e-9, restart=12, maxit=400)
        assert rc == 0
        outs.append((host(u), [i["iterations"] for i in infos]))
    assert outs[0][1] == outs[1][1] == outs[2][1]
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][0], outs[2][0])


def test_graphs_follow_the_cycle_length(monkeypatch):
    """Iterations are replayed from graphs of several columns; one operator
    solving with two cycle lengths (whose last groups differ) gives the same
    results as eager launches of each."""
    import torch
    w = CASES["2d_ragged"]()
    chi = dev(w.chi[:1], torch.complex128)
    monkeypatch.setenv("CSG_GRAPHS", "1")
    op, _ = pair(w, max_rhs=1, cycle_prec=0, restart=12)
    got = {}
    for m in (12, 10, 12, 7):
        u, rc, infos = op.solve(chi, tol=1e-9, restart=m, maxit=400)
        assert rc == 0
        got.setdefault(m, []).append((host(u), infos[0]["iterations"]))
    monkeypatch.setenv("CSG_GRAPHS", "0")
    ref, _ = pair(w, max_rhs=1, cycle_prec=0, restart=12)
    for m, runs in got.items():
        u, rc, infos = ref.solve(chi, tol=1e-9, restart=m, maxit=400)
        note(f"  restart {m}: iterations {infos[0]['iterations']} (graphs {[r[1] for r in runs]})")
        for ug, itg in runs:
            assert itg == infos[0]["iterations"]
            assert np.array_equal(ug, host(u))


def test_instrumented_solve_times_every_launch():
    """Timing one pass kind (eager launches with event pairs) times every
    finest-level fused pass of every iteration and leaves the results
    bit-identical to the graph-replayed uninstrumented solve."""
    import torch
    from paper_1012_5379_amd import binding as B
    w = CASES["2d_wide"]()
    chi = dev(w.chi[:1], torch.complex128)
    op, orc = pair(w, max_rhs=1, cycle_prec=0, restart=12)
    u0, rc0, inf0 = op.solve(chi, tol=1e-9, restart=12, maxit=400)
    assert B.csg_graphs_active(op.op)
    B.csg_profile(op.op, B.PROF_KINDS["fused"], 1 << 16)
    u1, rc1, inf1 = op.solve(chi, tol=1e-9, restart=12, maxit=400)
    ms, n, by = B.csg_profile_read(op.op)
    B.csg_profile(op.op, 0, 0)
    its = inf1[0]["iterations"]
    note(f"  {n} timed launches over {its} iterations, {ms:.3f} ms")
    assert rc0 == 0 and rc1 == 0 and inf0[0]["iterations"] == its
    assert np.array_equal(host(u0), host(u1))
    # s - 1 fused passes per sweep, two sweeps per V-cycle, one V-cycle per iteration
    assert n == its * 2 * (w.s - 1)
    assert ms > 0 and by > 0


def test_instrumented_solve_with_rhs_stopping_apart():
    """Two RHS that stop at different iterations: the columns a launch runs
    while either RHS still iterates are timed, the columns queued after both
    have stopped are not, and the answers equal the plain solve's."""
    import torch
    from paper_1012_5379_amd import binding as B
    w = CASES["2d_wide"]()
    chi = np.stack([w.chi[0], 1e-3 * rvec(w.chi.shape[1:], 482)])
    op, orc = pair(w, max_rhs=2, cycle_prec=0, restart=12)
    u0, rc0, inf0 = op.solve(dev(chi, torch.complex128), tol=1e-9, restart=12, maxit=400)
    B.csg_profile(op.op, B.PROF_KINDS["fused"], 1 << 16)
    u1, rc1, inf1 = op.solve(dev(chi, torch.complex128), tol=1e-9, restart=12, maxit=400)
    ms, n, by = B.csg_profile_read(op.op)
    B.csg_profile(op.op, 0, 0)
    its = [i["iterations"] for i in inf1]
    note(f"  iterations {its}, {n} timed launches")
    assert rc0 == 0 and rc1 == 0 and [i["iterations"] for i in inf0] == its
    assert np.array_equal(host(u0), host(u1))
    assert n == max(its) * 2 * (w.s - 1)
