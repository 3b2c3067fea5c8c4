"""Host-side checks of the autotuner's table: keys by dimension, precision,
smoother and size class; the table only fills knobs left at the library
default; every committed entry passes the library's parameter validation;
out-of-range knobs are rejected."""
import json
import os

import pytest

from paper_1012_5379_amd import binding as B
from paper_1012_5379_amd import tune
from synth import workloads as W


def _params(w):
    return dict(w.params(), cycle_prec=w.cycle_prec, max_rhs=w.nrhs, restart=w.restart)


def test_keys():
    w = W.small(dim=3, n=27, mlo=3, mhi=4, item=3)
    k = tune.key(dict(_params(w), cycle_prec=0, max_rhs=4))
    # (3 + 27 + 4 - 1)^3 = 33^3 unknowns, 4 right-hand sides: log2(143748) = 17.1
    assert k == "d3-c128-gmres-2^17"
    assert tune.key(dict(_params(w), cycle_prec=1, max_rhs=4, smoother=1)) == "d3-c64-poly-2^17"
    # knobs do not change the key
    assert tune.key(dict(_params(w), cycle_prec=0, max_rhs=4, slab_blocks=64)) == k


def test_apply_fills_only_defaults(tmp_path):
    w = W.small(dim=2, n=60, m=8, item=1)
    p = dict(_params(w), cycle_prec=0, max_rhs=1)
    t = tmp_path / "t.json"
    t.write_text(json.dumps({"entries": {tune.key(p): {"knobs": {"tile_mult": 2, "tail_max": 600}}}}))
    assert tune.apply(p, str(t))["tile_mult"] == 2
    assert tune.apply(dict(p, tail_max=5000), str(t))["tail_max"] == 5000
    assert tune.apply(dict(p, max_rhs=16), str(t)).get("tile_mult", 0) == 0   # other size class
    assert tune.knobs_for(p, str(tmp_path / "missing.json")) == {}


def test_committed_table_is_valid():
    if not os.path.exists(tune.TABLE):
        pytest.skip("no tuned table committed")
    t = tune.load()
    assert t["entries"]
    for k, e in t["entries"].items():
        assert set(e["knobs"]) <= set(tune.KNOBS)
        assert e["ms_per_iteration"] <= e["default_ms_per_iteration"] + 1e-9
        assert e["trials"]
        w = W.small(dim=int(k[1]), n=20, m=4)
        B.csg_workspace_bytes(B.make_params(**dict(_params(w), **e["knobs"])))


@pytest.mark.parametrize("bad", [dict(tile_mult=3), dict(tile_mult=128), dict(slab_blocks=5000),
                                 dict(slab_blocks=-1), dict(slab_min=-2)])
def test_bad_knobs_rejected(bad):
    w = W.small(dim=2, n=20, m=4)
    with pytest.raises(B.CsgError):
        B.csg_workspace_bytes(B.make_params(**dict(_params(w), **bad)))
