"""Host-side checks of the HIP library that need no GPU: it loads, exports
every symbol the header declares, builds correct pull tables and boundary
lists, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2108_08783_amd import inputs
from tests import helpers as H
from paper_2108_08783_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
              [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
              [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
BB, GHOST = np.iinfo(np.int32).min, np.iinfo(np.int32).min + 1


def header_functions():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(lbm_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = lbm.load()
    declared = header_functions()
    assert declared == sorted(lbm.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_library_exports_every_network_symbol():
    from paper_2108_08783_amd import mlp
    lib = mlp.load()
    text = open(os.path.join(ROOT, "include", "lbm_mlp.h")).read()
    declared = sorted(set(re.findall(r"^(?:int|int64_t|const char\*)\s+(mlp_\w+)\s*\(", text, re.M)))
    assert declared == sorted(mlp.MLP_EXPORTS)
    for name in declared:
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_cylinder_counts_match_independent_voxelisation():
    # independent counts of the R=8, L=64 and R=32, L=512 tubes (site,
    # boundary-site, wall-link and iolet-link numbers of the same shape).
    for (R, L), want in {(8, 64): (12352, 3858, 17288, 1930),
                         (32, 512): (1640960, 132890, 572936, 32050)}.items():
        g = inputs.cylinder(R, L)
        p = lbm.lbm_plan_export([g], wall_modes=[lbm.ELASTIC], tables=False)
        assert (p["n_sites"], p["n_boundary"], p["n_wall_links"], p["n_iolet_links"]) == want


def _index_grid(labels):
    idx = -np.ones(labels.shape, np.int64)
    fl = labels == 1
    idx[fl] = np.arange(fl.sum())
    return idx


@pytest.mark.parametrize("mode", [lbm.BOUNCEBACK, lbm.ELASTIC])
def test_pull_table_invariants(mode):
    rng = np.random.default_rng(5)
    geos = [H.one_iolet_per_site(inputs.random_labels((7, 8, 9), rng)), inputs.cylinder(5, 9)]
    p = lbm.lbm_plan_export(geos, wall_modes=[mode, mode])
    nbr = p["nbr"]
    N = p["n_sites"]
    off = 0
    reads = set()
    bset = set(p["boundary"].tolist())
    for g in geos:
        lab = g.labels
        idx = _index_grid(lab)
        zz, yy, xx = np.nonzero(lab == 1)
        for s, (z, y, x) in enumerate(zip(zz, yy, xx)):
            gs = off + s
            ghost = False
            for i in range(1, 19):
                sx, sy, sz = x - C[i, 0], y - C[i, 1], z - C[i, 2]
                d = nbr[i - 1, gs]
                srclab = lab[sz, sy, sx]
                if srclab == 1:
                    assert gs + d == off + idx[sz, sy, sx]
                    reads.add((i, gs + d))
                else:
                    want = GHOST if (srclab >= 2 or mode == lbm.ELASTIC) else BB
                    assert d == want
                    ghost |= d == GHOST
                    opp = i + 1 if i % 2 else i - 1
                    reads.add((opp, gs))
            assert (gs in bset) == ghost
        off += g.n_fluid
    # every slot (i >= 1) is read by exactly one site
    assert len(reads) == 18 * N


def test_boundary_masks_mark_every_non_bounce_back_link():
    g = inputs.cylinder(4, 6)
    p = lbm.lbm_plan_export([g], wall_modes=[lbm.ELASTIC])
    for j, s in enumerate(p["boundary"]):
        m = p["bmask"][j]
        for i in range(1, 19):
            assert bool(m >> i & 1) == (p["nbr"][i - 1, s] == GHOST)


def test_sixteen_bit_offsets_fit_for_the_tube_workload():
    p = lbm.lbm_plan_export([inputs.cylinder(32, 16)], tables=False)
    # largest offset: one slice (3205 sites) plus about one row (2R)
    assert 3205 < p["max_abs_offset"] < 3205 + 2 * 32 + 2


@pytest.mark.parametrize("bad", ["border", "tau", "two_iolets", "dtype", "no_fluid"])
def test_invalid_arguments_are_rejected_without_a_device(bad):
    g = inputs.cylinder(3, 4)
    tau, dtype = 0.8, "f32"
    if bad == "border":
        g.labels[2, 0, 3] = 1
    elif bad == "tau":
        tau = 0.5
    elif bad == "two_iolets":
        g = inputs.Geometry(labels=np.zeros((5, 5, 5), np.uint8))
        g.labels[2, 2, 2] = 1
        g.labels[2, 2, 1] = 2
        g.labels[2, 2, 3] = 3
    elif bad == "dtype":
        dtype = 7
    elif bad == "no_fluid":
        g.labels[:] = 0
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create_geometry([g], dtype, tau)
    assert e.value.code == lbm.LBM_EINVAL
    words = {"border": "border", "tau": "tau", "two_iolets": "iolets", "dtype": "dtype",
             "no_fluid": "no fluid"}
    assert words[bad] in str(e.value)


def test_plan_rejects_zero_instances():
    with pytest.raises(lbm.LbmError):
        lbm.lbm_plan_export([], tables=False)


@pytest.mark.parametrize("mode", [0, 1])
def test_compressed_addressing_reproduces_the_table(mode):
    """The compressed addressing (stretches, non-fluid link masks, full
    offsets for rows of several fluid runs) is checked against the full
    neighbour table at every site by the builder itself; random boxes have
    many multi-run rows, convex tubes none."""
    rng = np.random.default_rng(7 + mode)
    for _ in range(4):
        g = H.one_iolet_per_site(inputs.random_labels((12, 9, 10), rng, p_fluid=0.7))
        st = lbm.lbm_plan_compressed([g], [mode])
        n = lbm.lbm_plan_export([g], wall_modes=[mode], tables=False)["n_sites"]
        assert st["records"] == (max(256, (n + 255) // 256 * 256)) // 64
        assert 0 < st["exceptional"] <= st["irregular"] <= n
    tube = inputs.cylinder(8, 64)
    st = lbm.lbm_plan_compressed([tube], [mode])
    assert st["exceptional"] == 0               # every row of a convex section is one run
    assert st["irregular"] == 3858
    assert st["stretches"] <= 2 * 17 * 64      # about one per row


def test_compressed_addressing_of_a_batch():
    geos, _ = inputs.batch(5, n=6, target_sites=2e5)
    st = lbm.lbm_plan_compressed(geos, [1] * len(geos))
    n = lbm.lbm_plan_export(geos, wall_modes=[1] * len(geos), tables=False)["n_sites"]
    assert st["records"] * 64 >= n
    assert st["exceptional"] < 0.01 * st["irregular"]


def test_fast_axis_follows_the_longest_fluid_runs(monkeypatch):
    monkeypatch.delenv("LBM_FAST_AXIS", raising=False)
    z_tube = inputs.cylinder(8, 64)             # runs of 64 along z, <= 16 along x
    x_tube = inputs.straight_tube_x(8, 60)
    duct = inputs.duct(12, 10, 11)              # no axis clearly longer
    assert lbm.lbm_fast_axis([z_tube, x_tube, duct]) == [2, 0, 0]
    g = inputs.Geometry(labels=np.ascontiguousarray(z_tube.labels.transpose(1, 0, 2)))
    assert lbm.lbm_fast_axis([g]) == [1]       # the same tube along y


def test_fast_axis_override(monkeypatch):
    tube = inputs.cylinder(6, 30)
    for name, want in (("x", 0), ("y", 1), ("z", 2), ("auto", 2)):
        monkeypatch.setenv("LBM_FAST_AXIS", name)
        assert lbm.lbm_fast_axis([tube, tube]) == [want, want]
    monkeypatch.setenv("LBM_FAST_AXIS", "w")
    with pytest.raises(lbm.LbmError):
        lbm.lbm_fast_axis([tube])


def test_two_iolets_at_one_site_are_rejected_by_the_library_only():
    """The library's one-iolet-per-site limit (reading 11): unrestricted
    random boxes that have a fluid site next to two different iolets are
    rejected by the host build with a message naming the limit, while the
    oracle steps them; restricted, the same boxes are accepted."""
    import oracle
    rng = np.random.default_rng(5)
    found = 0
    for _ in range(20):
        g = inputs.random_labels((8, 9, 10), rng)
        lab = g.labels
        fl = np.argwhere(lab == inputs.FLUID)
        two = False
        for z, y, x in fl:
            ids = {int(lab[z - dz, y - dy, x - dx]) for dx in (-1, 0, 1) for dy in (-1, 0, 1)
                   for dz in (-1, 0, 1) if 0 < dx * dx + dy * dy + dz * dz <= 2
                   and lab[z - dz, y - dy, x - dx] >= inputs.IOLET0}
            two |= len(ids) > 1
        if not two:
            continue
        found += 1
        with pytest.raises(lbm.LbmError, match="iolet"):
            lbm.lbm_plan_export([g], tables=False)
        o = oracle.Oracle(g.labels, 0.8)
        o.set_wall(0)
        for i in range(2):
            o.set_iolet(i, 0, 1.0 + 0.001 * i)
        o.init_fields()
        o.step(5)
        assert np.isfinite(o.read()[1]).all()
        lbm.lbm_plan_export([H.one_iolet_per_site(g)], tables=False)
    assert found >= 3
