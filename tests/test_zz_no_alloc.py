"""lbm_read_fields_noalloc (the read-out that allocates nothing, for callers
that cannot allocate) against lbm_read_fields on the same state: outputs
identical bit for bit, on two calls in a row with a smaller instance
second (the shared staging array keeps the first call's contents), for an
instance stored with its fast axis exchanged and one that is not."""
import numpy as np
import pytest

from paper_2108_08783_amd import inputs, lbm
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _noalloc(lat, inst):
    n = lat.n_sites(inst)
    rho, u = np.full(n, np.nan), np.full((n, 3), np.nan)
    wss, dr = np.full(n, np.nan), np.full(n, np.nan, np.float32)
    lbm.lbm_read_fields_noalloc(lat.ctx, inst, rho, u, wss, dr)
    return rho, u, wss, dr


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_noalloc_read_matches_read_fields(dtype):
    big = H.tube_problem(8, 64, seed=2, period=300.0)          # z-aligned: axis exchanged
    small = H.random_box_problem(6)                             # kept in x order
    small.tau = big.tau
    assert lbm.lbm_fast_axis([big.geo, small.geo])[0] != 0
    lat = H.make_lattice([big, small], dtype)
    lat.step(150)
    print("noalloc: tube then box,", dtype, flush=True)
    for inst in (0, 1):                                         # larger first, then smaller
        got = _noalloc(lat, inst)
        ref = lat.read_fields(inst)
        for a, b in zip(got, ref):
            assert a.shape == b.shape and np.array_equal(a, b), inst
    # again after more steps, reading only some outputs
    lat.step(40)
    n1 = lat.n_sites(1)
    rho = np.zeros(n1)
    lbm.lbm_read_fields_noalloc(lat.ctx, 1, rho, None, None, None)
    assert np.array_equal(rho, lat.read_fields(1, wss=False, wall_dr=False)[0])
    lat.close()


def test_noalloc_read_rejects_what_it_cannot_stage():
    """Beyond the staging limit the call fails with a message; after a wall
    parameter change (not yet applied by a step) it refuses too."""
    g = inputs.cylinder(48, 330)
    assert g.n_fluid > lbm.NOALLOC_MAX_SITES
    p = H.Problem(geo=g, tau=0.8, mode=lbm.ELASTIC, F=0.5, k=[1e-2],
                  iolets={0: dict(kind=lbm.DENSITY, a0=1.001), 1: dict(kind=lbm.DENSITY, a0=0.999)})
    q = H.random_box_problem(7)
    q.tau = 0.8
    lat = H.make_lattice([p, q], "f32")
    n = g.n_fluid
    with pytest.raises(lbm.LbmError, match="at most"):
        lbm.lbm_read_fields_noalloc(lat.ctx, 0, np.zeros(n), np.zeros((n, 3)))
    lat.step(3)
    lat.set_wall(1, lbm.ELASTIC, F=0.3, P0=q.P0, k=q.k)
    m = lat.n_sites(1)
    with pytest.raises(lbm.LbmError, match="lbm_step"):
        lbm.lbm_read_fields_noalloc(lat.ctx, 1, np.zeros(m), np.zeros((m, 3)))
    lat.step(1)
    rho = np.zeros(m)
    lbm.lbm_read_fields_noalloc(lat.ctx, 1, rho, None)
    assert np.array_equal(rho, lat.read_fields(1)[0])
    lat.close()
