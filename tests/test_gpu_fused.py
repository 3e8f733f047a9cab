"""Fused diagnostic steps (windings and the Gauss residual computed inside the
update kernel) against the post-step kernels, through the C ABI, on identical
inputs: fields and momenta bitwise, windings, cell values and overlap counts
bitwise, the Gauss and integer-time sums to the rounding of their summation
order; and the record against the oracle (Sec. III.A windings, Sec. II Gauss
law).  Geometries cover ragged tiles in x, y and z and boxes narrower than a
tile."""
import numpy as np
import pytest

import oracle as O
from tests import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2208_01525_amd")

GEOMS = [(72, 18, 11), (64, 16, 16), (40, 9, 7), (5, 9, 7)]
SUMS = ("sum_energy", "sum_lagrangian", "sum_KL", "sum_GL", "sum_KV", "sum_GV")


def _run(geom, rows, st, sched, tile=(8, 4), n=3):
    nx, ny, nz = geom
    lat = P.Lattice(P.make_params(nx, ny, nz, precision="fp32", eta_ref=9.0, diag_every=1, kappa=0.9),
                    device="cuda:0")
    lat.set_tile(*tile)
    lat.set_fused_diagnostics(rows)
    lat.set_fields(st)
    recs = []
    cells = []
    for j in range(n):
        lat.step(1, sched[0] + j * 0.1, sched[1], sched[2])
        recs += lat.diagnostics()
        cells.append(lat.get_cells())
    out = lat.get_fields(), recs, cells, lat.get_fused_diagnostics()
    lat.close()
    return out


@pytest.mark.parametrize("geom", GEOMS)
@pytest.mark.parametrize("rows", [4, 5, 8])
def test_fused_matches_post_kernels(geom, rows):
    nx, ny, nz = geom
    st = I.to_f32_values(I.random_full(nx, ny, nz, 21, link=0.8, mom=0.5))
    sched = (3.0, 2.0 / 3.0, 0.5)
    f_fused, r_fused, c_fused, used = _run(geom, rows, st, sched)
    f_post, r_post, c_post, used0 = _run(geom, 0, st, sched)
    assert used == rows and used0 == 0
    assert np.array_equal(f_fused, f_post)
    assert len(r_fused) == len(r_post) == 3
    for a, b, ca, cb in zip(r_fused, r_post, c_fused, c_post):
        assert a["wind_abs"] == b["wind_abs"] and a["pq_count2"] == b["pq_count2"]
        assert np.array_equal(ca, cb)
        for k in SUMS:
            assert a[k] == pytest.approx(b[k], rel=1e-12, abs=1e-12), k
        for q in range(2):
            assert a["gauss_abs"][q] == pytest.approx(b["gauss_abs"][q], rel=1e-12, abs=1e-12)
            assert a["gauss_scale"][q] == pytest.approx(b["gauss_scale"][q], rel=1e-12, abs=1e-12)
        assert a["flags"] == 0


@pytest.mark.parametrize("geom", [(72, 18, 11), (5, 9, 7)])
def test_fused_record_against_oracle(geom):
    """One fused diagnostic step on identical inputs against the oracle's record: windings
    and overlap exact, the cells bitwise, the Gauss residual sums to FP32 rounding of the
    per-site terms."""
    nx, ny, nz = geom
    st = I.to_f32_values(I.random_full(nx, ny, nz, 6, link=0.5, mom=0.5))
    lat = P.Lattice(P.make_params(nx, ny, nz, precision="fp32", eta_ref=9.0, diag_every=1, kappa=0.9),
                    device="cuda:0")
    lat.set_fields(st)
    lat.step(1, 3.0, 0.5, 1.0)
    assert lat.get_fused_diagnostics() == 8
    r = lat.diagnostics()[0]
    m = O.model(nx, ny, nz, eta_ref=9.0, kappa=0.9)
    o = O.step(m, st.copy(), 3.0, 0.5, 1.0, diag=True)
    assert r["wind_abs"] == o["wind_abs"] and r["pq_count2"] == o["pq_count2"]
    assert np.array_equal(lat.get_cells().astype(np.int32), O.cells(m, O.windings(m, st)))
    for q in range(2):
        assert r["gauss_scale"][q] == pytest.approx(o["gauss_scale"][q], rel=1e-5)
        assert abs(r["gauss_abs"][q] - o["gauss_abs"][q]) <= 1e-5 * o["gauss_scale"][q]
    lat.close()


def test_fused_checkpoint_resume_and_switching():
    """The fused steps alternate the momentum copies: get/set_fields follow them, and a run
    that switches the fused path off and on mid-way gives the same bits."""
    nx, ny, nz = 72, 18, 11
    kw = dict(precision="fp32", eta_ref=9.0, diag_every=3)
    a = P.Lattice(P.make_params(nx, ny, nz, **kw), device="cuda:0")
    a.init_fields(3)
    a.step(7, 1.0, 0.5, 1.0)
    mid = a.get_fields()
    a.step(7, 1.7, 0.5, 1.0)
    b = P.Lattice(P.make_params(nx, ny, nz, **kw), device="cuda:0")
    b.set_fused_diagnostics(0)
    b.set_fields(mid)
    b.step(4, 1.7, 0.5, 1.0)
    b.set_fused_diagnostics(8)
    b.step(3, 2.1, 0.5, 1.0)
    assert np.array_equal(a.get_fields(), b.get_fields())
    a.close()
    b.close()


def _planted(nx, ny, nz, seed, f32=True, offsets=(-3e-5, 3e-5, 1e-6)):
    """Random fields with the cases the winding guard sends to FP64 planted: zeros of
    phi, link angles above 1e3, and links whose phase lies at the given offsets from the
    branch cut (values rounded to float32 as the lattice holds them, unless f32 is off)."""
    rng = np.random.default_rng(seed)
    st = I.random_full(nx, ny, nz, seed, link=0.8, mom=0.5)
    S = nx * ny * nz
    flat = st.reshape(20, S)
    h = 0.5
    for sec, (c, a0) in enumerate(((I.PHI, I.A), (I.PSI, I.B))):
        for s in rng.choice(S, 6, replace=False):
            flat[c, s] = flat[c + 1, s] = 0.0
        for s in rng.choice(S, 6, replace=False):
            flat[a0 + rng.integers(3), s] = rng.choice([-1.0, 1.0]) * rng.uniform(2.5e3, 4e3)
        for s in rng.choice(S, 40, replace=False):
            x, y, z = s % nx, (s // nx) % ny, s // (nx * ny)
            i = int(rng.integers(3))
            t = (x + (i == 0)) % nx + nx * ((y + (i == 1)) % ny) + nx * ny * ((z + (i == 2)) % nz)
            phase = lambda k: np.arctan2(flat[c + 1, k], flat[c, k])
            target = np.pi - rng.choice(offsets)
            flat[a0 + i, s] = (phase(t) - phase(s) - target) / h
    return I.to_f32_values(st) if f32 else st


@pytest.mark.parametrize("rows", [5, 8])
def test_fused_guard_cases_match_oracle(rows):
    """The sites whose windings involve a guarded link are left by the fused kernel to the
    fix-up kernel: sum |W| equals the oracle's, and the cells equal the oracle's cells of
    the windings clipped to |W| <= 3 per face (what a packed byte holds), in both paths."""
    nx, ny, nz = 72, 18, 11
    st = _planted(nx, ny, nz, 31)
    m = O.model(nx, ny, nz, eta_ref=9.0, kappa=0.9)
    W = O.windings(m, st)
    assert np.abs(W).max() > 3        # the planted large angles make windings of many units
    # the packed cell bytes hold min(|W|, 3) per face, in both paths
    ref_cells = O.cells(m, np.clip(W, -3, 3))
    for r in (rows, 0):
        lat = P.Lattice(P.make_params(nx, ny, nz, precision="fp32", eta_ref=9.0, diag_every=1, kappa=0.9),
                        device="cuda:0")
        lat.set_fused_diagnostics(r)
        lat.set_fields(st)
        lat.step(1, 3.0, 0.5, 1.0)
        rec = lat.diagnostics()[0]
        assert rec["wind_abs"] == (int(np.abs(W[:3]).sum()), int(np.abs(W[3:]).sum()))
        assert np.array_equal(lat.get_cells().astype(np.int32), ref_cells)
        lat.close()


@pytest.mark.parametrize("tile", [None, 0])
def test_fp64_guard_cases_match_oracle(tile):
    """FP64 diagnostic steps form wrap counts from FP32 phases of the FP64 fields and
    flag every link within 1e-4 rad of the branch cut: links planted just inside that
    margin (3e-5, 1e-6, 1e-12 from the cut) go to the FP64 fix-up, links just outside it
    (2e-4) keep the fast count; both equal the oracle's windings exactly, with zeros of
    phi and link angles above 1e3, on the tiled and on the per-site diagnostic update."""
    nx, ny, nz = 72, 18, 11
    st = _planted(nx, ny, nz, 37, f32=False, offsets=(-3e-5, 3e-5, 1e-6, 1e-12, -2e-4, 2e-4))
    m = O.model(nx, ny, nz, eta_ref=9.0, kappa=0.9)
    W = O.windings(m, st)
    assert np.abs(W).max() > 3
    lat = P.Lattice(P.make_params(nx, ny, nz, precision="fp64", eta_ref=9.0, diag_every=1, kappa=0.9),
                    device="cuda:0")
    if tile is not None:
        with pytest.raises(P.MtsError):       # tz >= 1 also for the per-site kernel
            lat.set_tile(tile, 0)
        lat.set_tile(tile, 32)
    lat.set_fields(st)
    lat.step(1, 3.0, 0.5, 1.0)
    rec = lat.diagnostics()[0]
    got = lat.get_cells().astype(np.int32)
    lat.close()
    assert rec["wind_abs"] == (int(np.abs(W[:3]).sum()), int(np.abs(W[3:]).sum()))
    assert np.array_equal(got, O.cells(m, np.clip(W, -3, 3)))
    assert rec["pq_count2"] == sum(O.overlap(m, O.cells(m, W)))


def test_batch_fused_matches_box_by_box():
    """An FP32 ensemble with fused diagnostic steps (batched update, then one fix-up, cells,
    overlap and reduction launch for all boxes) against the same ensemble running the
    post-step kernels box by box: fields bitwise, windings, overlap and cells bitwise, sums
    to rounding.  Box widths 64 and 128 take the packed-word overlap, the others the byte
    one; guard cases are planted in one box."""
    shapes = [(64, 9, 6), (24, 16, 12), (70, 9, 5), (128, 4, 4), (33, 20, 7), (256, 5, 6)]
    eras = [0.5, 2.0 / 3.0, 0.5, 2.0 / 3.0, 0.5, 2.0 / 3.0]
    s_b = [0.0, 1.0, 1.0, 0.0, 1.0, 0.0]
    kw = dict(precision="fp32", diag_every=2)
    states = [I.to_f32_values(I.random_full(*sh, 50 + k, link=0.7, mom=0.4)) for k, sh in enumerate(shapes)]
    states[0] = _planted(*shapes[0], 41)
    runs = []
    for rows in (8, 0):
        bt = P.Batch([P.make_params(*sh, eta_ref=5.0 + k, **kw) for k, sh in enumerate(shapes)])
        bt.set_fused_diagnostics(rows)
        assert bt.get_fused_diagnostics() == rows
        bt.set_tile(8, [4, 3, 5, 2, 7, 3])
        for k, st in enumerate(states):
            bt.set_fields(k, st)
        bt.step(5, [1.0] * len(shapes), eras, s_b)
        runs.append(([bt.get_fields(k) for k in range(len(shapes))], [bt.diagnostics(k) for k in range(len(shapes))]))
        bt.close()
    (fa, ra), (fb, rb) = runs
    for k in range(len(shapes)):
        assert np.array_equal(fa[k], fb[k]), k
        assert len(ra[k]) == len(rb[k]) == 3
        for a, b in zip(ra[k], rb[k]):
            assert a["wind_abs"] == b["wind_abs"] and a["pq_count2"] == b["pq_count2"], k
            for q in SUMS:
                assert a[q] == pytest.approx(b[q], rel=1e-11, abs=1e-11), (k, q)
            for s in range(2):
                assert a["gauss_abs"][s] == pytest.approx(b["gauss_abs"][s], rel=1e-11, abs=1e-12)
                assert a["gauss_scale"][s] == pytest.approx(b["gauss_scale"][s], rel=1e-11)


@pytest.mark.parametrize("precision,rows", [("fp32", 8), ("fp32", 0), ("fp64", 0)])
@pytest.mark.parametrize("geom", [(256, 6, 5), (512, 5, 18), (128, 7, 5), (128, 4, 18)])
def test_cells_of_wide_rows_match_oracle(geom, precision, rows):
    """Rows whose width is a multiple of 256, or 128 (two rows per wave), take the cells
    kernel that reads the packed |W| bytes as words, four cells per lane, and assembles the
    occupancy words from ballots: cells equal the oracle's cells of the same windings (clipped
    to 3 per face, what a packed byte holds) and the overlap count the oracle's, on random
    fields with many windings (ragged y and z blocks, an odd row count that leaves a wave's
    second row outside the box; the 18-plane boxes cross two 16-plane blocks)."""
    nx, ny, nz = geom
    st = I.random_full(nx, ny, nz, 61, link=0.7, mom=0.4)
    if precision == "fp32":
        st = I.to_f32_values(st)
    m = O.model(nx, ny, nz, eta_ref=9.0, kappa=0.9)
    W = O.windings(m, st)
    assert np.abs(W).sum() > 100
    ref_cells = O.cells(m, np.clip(W, -3, 3))
    lat = P.Lattice(P.make_params(nx, ny, nz, precision=precision, eta_ref=9.0, diag_every=1, kappa=0.9),
                    device="cuda:0")
    if precision == "fp32":
        lat.set_fused_diagnostics(rows)
    lat.set_fields(st)
    lat.step(1, 3.0, 0.5, 1.0)
    rec = lat.diagnostics()[0]
    got = lat.get_cells().astype(np.int32)
    lat.close()
    assert np.array_equal(got, ref_cells)
    assert rec["wind_abs"] == (int(np.abs(W[:3]).sum()), int(np.abs(W[3:]).sum()))
    assert rec["pq_count2"] == sum(O.overlap(m, O.cells(m, W)))
