"""The persistent ensemble launch through the C ABI: every run of plain steps of
all boxes in one launch with a grid barrier per step, against the per-step
launches captured in one graph.  The tiles and their arithmetic are the same,
so fields and records must agree bit for bit; the barrier's bounded wait is
exercised from the host with a limit too short for any wait (every workgroup
leaves, the next synchronising call reports MTS_EHIP once, and the batch runs
again after its fields are set)."""
import numpy as np
import pytest

from tests import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2208_01525_amd")

SHAPES = [(64, 9, 6), (24, 16, 12), (70, 9, 5), (128, 20, 13), (33, 20, 7)]
ERAS = [0.5, 2.0 / 3.0, 0.5, 2.0 / 3.0, 0.5]
S_B = [0.0, 1.0, 1.0, 0.0, 1.0]


def _states(precision):
    st = [I.random_full(*sh, 70 + k, link=0.7, mom=0.4) for k, sh in enumerate(SHAPES)]
    return [I.to_f32_values(s) for s in st] if precision == "fp32" else st


def _same(a, b):
    """Equal records (NaN equal to NaN: a derived quantity undefined in both)."""
    assert a.keys() == b.keys()
    for k in a:
        x, y = np.asarray(a[k], dtype=float), np.asarray(b[k], dtype=float)
        if not np.array_equal(x, y, equal_nan=True):
            return False
    return True


def _run(precision, persist, ty, tz, mpp=False, xcd=True, n=11, diag_every=4, states=None):
    bt = P.Batch([P.make_params(*sh, precision=precision, eta_ref=6.0 + k, diag_every=diag_every)
                  for k, sh in enumerate(SHAPES)])
    bt.set_tile(ty, tz)
    bt.set_momentum_pingpong(mpp)
    bt.set_tile_order(xcd)
    bt.set_persistent(persist)
    assert bt.get_persistent() == persist
    for k, st in enumerate(states or _states(precision)):
        bt.set_fields(k, st)
    bt.step(n, [1.0] * len(SHAPES), ERAS, S_B)
    out = [bt.get_fields(k) for k in range(len(SHAPES))], [bt.diagnostics(k) for k in range(len(SHAPES))]
    bt.close()
    return out


@pytest.mark.parametrize("precision,ty,tz,mpp,xcd", [
    ("fp32", 4, [4, 3, 5, 2, 7], False, True),
    ("fp32", 8, [2, 5, 3, 4, 6], True, False),
    ("fp32", 13, 8, False, True),
    ("fp64", 5, [3, 4, 2, 5, 3], False, True),
    ("fp64", 4, 6, True, True),
])
def test_persistent_matches_graph(precision, ty, tz, mpp, xcd):
    print(f"persistent vs graph: {precision} ty={ty} tz={tz} mpp={mpp} xcd={xcd}", flush=True)
    states = _states(precision)
    fa, ra = _run(precision, False, ty, tz, mpp, xcd, states=states)
    fb, rb = _run(precision, True, ty, tz, mpp, xcd, states=states)
    for k in range(len(SHAPES)):
        assert np.array_equal(fa[k], fb[k]), k
        assert len(ra[k]) == len(rb[k]) == 3
        for a, b in zip(ra[k], rb[k]):
            assert _same(a, b), (k, a, b)


def test_persistent_plain_only_run_matches_graph():
    """No diagnostic step: the whole call is one persistent launch."""
    print("persistent vs graph: plain only", flush=True)
    states = _states("fp32")
    fa, _ = _run("fp32", False, 8, 4, n=9, diag_every=0, states=states)
    fb, _ = _run("fp32", True, 8, 4, n=9, diag_every=0, states=states)
    for k in range(len(SHAPES)):
        assert np.array_equal(fa[k], fb[k]), k


def test_persistent_wait_limit_reports_ehip():
    print("persistent: forced barrier time-out", flush=True)
    states = _states("fp32")
    bt = P.Batch([P.make_params(*sh, precision="fp32", eta_ref=6.0 + k, diag_every=0)
                  for k, sh in enumerate(SHAPES)])
    with pytest.raises(P.MtsError):
        bt.set_persistent(True, -1.0)
    bt.set_tile(4, 2)
    bt.set_persistent(True, 1e-9)   # one wall-clock tick: every wait runs out
    for k, st in enumerate(states):
        bt.set_fields(k, st)
    bt.step(12, [1.0] * len(SHAPES), ERAS, S_B)
    with pytest.raises(P.MtsError) as ei:
        bt.timing_read()
    assert ei.value.code == P.mts.MTS_EHIP
    assert "grid-barrier" in str(ei.value)
    bt.timing_read()   # reported once
    # with the default limit, from fresh fields, the batch runs as the graph does
    bt.set_persistent(True)
    for k, st in enumerate(states):
        bt.set_fields(k, st)
    bt.step(12, [1.0] * len(SHAPES), ERAS, S_B)
    got = [bt.get_fields(k) for k in range(len(SHAPES))]
    bt.close()
    ref, _ = _run("fp32", False, 4, 2, n=12, diag_every=0, states=states)
    for k in range(len(SHAPES)):
        assert np.array_equal(got[k], ref[k]), k


def test_autotune_cache_hit_applies_the_stored_choice(tmp_path):
    """mts_autotune_cached: a miss tunes and appends one line for the key (arch, CU count,
    box, precision); a second context of the same box hits it, takes the same settings
    without timing anything and leaves its fields alone; unparsable lines are skipped."""
    print("autotune cache", flush=True)
    cache = tmp_path / "tune.txt"
    cache.write_text("not a cache line\n")
    geom = (96, 20, 24)
    a = P.Lattice(P.make_params(*geom, precision="fp32", eta_ref=6.0), device="cuda:0")
    a.autotune(1, cache=cache)
    assert a.autotune_hit == 0
    lines = cache.read_text().splitlines()
    assert len(lines) == 2 and lines[1].startswith("mts-tune-1 ") and "n=96x20x24 prec=fp32 | ty=" in lines[1]
    want = (a.get_tile(), a.get_streaming_stores(), a.get_prefetch(), a.get_momentum_pingpong(),
            a.get_tile_order(), a.get_time_blocking())
    a.close()
    st = I.to_f32_values(I.random_full(*geom, 5, link=0.5, mom=0.3))
    b = P.Lattice(P.make_params(*geom, precision="fp32", eta_ref=6.0), device="cuda:0")
    b.set_fields(st)
    b.autotune(1, cache=cache)
    assert b.autotune_hit == 1
    got = (b.get_tile(), b.get_streaming_stores(), b.get_prefetch(), b.get_momentum_pingpong(),
           b.get_tile_order(), b.get_time_blocking())
    assert got == want
    assert np.array_equal(b.get_fields(), st)
    b.close()
    assert len(cache.read_text().splitlines()) == 2
