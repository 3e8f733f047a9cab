"""The entry point that allocates nothing (mts_get_sites_noalloc) against the
one it mirrors (mts_get_sites), through the C ABI: bit-identical values on two
calls in a row (the second smaller, so stale scratch contents would show), in
both precisions and on two boxes at once, and the size limit rejected on the
host."""
import numpy as np
import pytest

from tests import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2208_01525_amd")
from paper_2208_01525_amd import mts as M  # noqa: E402


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_sites_match_get_sites(precision):
    nx, ny, nz = 72, 20, 13
    lat = P.Lattice(P.make_params(nx, ny, nz, precision=precision, eta_ref=17.0, diag_every=0), device="cuda:0")
    lat.set_fields(I.random_full(nx, ny, nz, 11))
    lat.step(3, 1.0, 0.5, 1.0)
    S = nx * ny * nz
    rng = np.random.default_rng(5)
    first = rng.integers(0, S, size=M.NOALLOC_MAX_SITES, dtype=np.uint64)
    first[:2] = [0, S - 1]
    second = rng.integers(0, S, size=37, dtype=np.uint64)
    for sites in (first, second):
        ref = lat.get_sites(sites)
        got = lat.get_sites_noalloc(sites)
        assert got.shape == ref.shape == (len(sites), 20)
        assert np.array_equal(got, ref)
    # a second box on the same GPU shares the scratch: its values, not the first box's
    other = P.Lattice(P.make_params(9, 6, 5, precision=precision, eta_ref=4.0), device="cuda:0")
    other.set_fields(I.random_full(9, 6, 5, 12))
    few = np.array([0, 7, 269], dtype=np.uint64)
    assert np.array_equal(other.get_sites_noalloc(few), other.get_sites(few))
    assert np.array_equal(lat.get_sites_noalloc(second[:5]), lat.get_sites(second[:5]))
    # the limit and bad indices are rejected on the host; the context stays usable
    with pytest.raises(M.MtsError) as ex:
        lat.get_sites_noalloc(np.zeros(M.NOALLOC_MAX_SITES + 1, dtype=np.uint64))
    assert ex.value.code == M.MTS_EINVAL
    with pytest.raises(M.MtsError):
        lat.get_sites_noalloc(np.array([S], dtype=np.uint64))
    assert lat.get_sites_noalloc(np.zeros(0, dtype=np.uint64)).shape == (0, 20)
    assert np.array_equal(lat.get_sites_noalloc(first[:3]), lat.get_sites(first[:3]))
    other.close()
    lat.close()
