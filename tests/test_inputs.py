"""Seeded synthetic workloads: shapes, counts and the invariants the
library relies on (no fluid on the border, one iolet per site)."""
import numpy as np
import pytest

from paper_2108_08783_amd import inputs
from paper_2108_08783_amd import lbm


def test_cylinder_is_symmetric_and_parabolic_weights_average_one():
    g = inputs.cylinder(8, 4)
    fl = g.labels[1] == 1
    assert np.array_equal(fl, fl[::-1, :]) and np.array_equal(fl, fl[:, ::-1])
    w = g.iolet_weight[1][fl]
    assert w.mean() == pytest.approx(1.0, abs=0.05)
    nn = np.linalg.norm(g.normal[1][fl], axis=1)
    assert np.allclose(nn[nn > 0], 1.0, atol=1e-6) and (nn == 0).sum() == 1  # the axis voxel


def test_tree_quarter_scale_structure():
    g = inputs.murray_tree(3, scale=0.25)
    assert g.info["n_segments"] == 31 + 16 * 3
    outlets = [io for io in g.iolets if io["role"] == "outlet"]
    assert len(outlets) == 48
    assert 0.08e6 < g.n_fluid < 0.14e6
    p = lbm.lbm_plan_export([g], wall_modes=[lbm.ELASTIC], tables=False)
    assert p["n_sites"] == g.n_fluid
    # every leaf stub outlet is reached by some link
    present = {int(v) - 2 for v in np.unique(g.labels) if v >= 2}
    assert present == set(range(49))
    # segment ids cover all tubes; inlet weights are parabolic near the inlet
    assert g.segment[g.labels == 1].max() == 78
    assert g.iolet_weight[:, :, 1].max() == pytest.approx(2.0, abs=0.1)


def test_tree_is_seeded():
    a = inputs.murray_tree(5, scale=0.2)
    b = inputs.murray_tree(5, scale=0.2)
    c = inputs.murray_tree(6, scale=0.2)
    assert np.array_equal(a.labels, b.labels)
    assert not np.array_equal(a.labels, c.labels) or a.labels.shape != c.labels.shape


def test_batch_hits_target_and_mixes_kinds():
    geos, params = inputs.batch(4, n=16, target_sites=2e6)
    tot = sum(g.n_fluid for g in geos)
    assert abs(tot / 2e6 - 1) <= 0.05
    kinds = [p["kind"] for p in params]
    assert kinds.count("tube") == 8 and kinds.count("bif") == 8
    assert all(1e-3 <= p["k"] <= 1e-1 and 0.01 <= p["u0"] <= 0.03 for p in params)
    p = lbm.lbm_plan_export(geos, wall_modes=[1] * 16, tables=False)
    assert p["n_sites"] == tot


def test_bifurcation_has_two_outlets():
    g = inputs.bifurcation(8, 120, 50)
    present = sorted({int(v) - 2 for v in np.unique(g.labels) if v >= 2})
    assert present == [0, 1, 2]


def test_tree_batch_workload_holds_each_seeded_tree():
    """`workloads.trees`: one instance per seed, each the tree (geometry and
    parameters) that `workloads.tree` gives for that seed; the training
    seeds of the tree-trained warm start (1000..) are disjoint from the
    held-out ones (2000..)."""
    from paper_2108_08783_amd import workloads
    wl = workloads.trees([1000, 1001], scale=0.2)
    assert len(wl.geoms) == len(wl.params) == 2
    for k, seed in enumerate((1000, 1001)):
        one = workloads.tree(seed, scale=0.2)
        assert np.array_equal(wl.geoms[k].labels, one.geoms[0].labels)
        assert wl.params[k].k == one.params[0].k and wl.params[k].F == one.params[0].F
        assert wl.params[k].iolets.keys() == one.params[0].iolets.keys()
    assert wl.n_sites == sum(g.n_fluid for g in wl.geoms)
