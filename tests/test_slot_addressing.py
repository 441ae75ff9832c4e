"""Host emulation of the update kernels' slot addressing, on the pull tables
the library builds for the random boxes, the tube, the tree and a small
sweep (no GPU).

The populations are 19 planes of N_pad slots (N_pad: the site count rounded
up to a multiple of 256).  Streaming is a pull (Sec. 2.1): site x reads
plane i at its upstream site x - c_i, or, for a link from a non-fluid
voxel, its own slot in the opposite plane.  The kernels read plane i
through a base P_i = (i N_pad - c_ix - N_pad - 1) slots (which may lie
below the buffer) plus a per-lane offset that is never negative:
  fluid upstream site x + d:  x + d + c_ix + N_pad + 1
  own opposite slot:          x + (opp(i) - i + 1) N_pad + c_ix + 1
counted in bytes (32 bits, population buffers below 2 GiB) or in elements
(two sites per lane beyond 2 GiB, scaled to bytes in 64 bits at the load).
Lanes past the last site of a tile take the own-slot offsets of the last
slot.  These checks tie every offset to the slot the pull table names and
keep every address inside the buffer."""
import numpy as np
import pytest

from paper_2108_08783_amd import inputs, lbm, workloads
from tests import helpers as H

# velocity set in the library's order: rest; +-x, +-y, +-z; then the (x,y),
# (x,z), (y,z) diagonal families, each (+,+), (-,-), (+,-), (-,+)
CX = np.array([0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0])
BB, GHOST = np.iinfo(np.int32).min, np.iinfo(np.int32).min + 1
Q = 19


def opp(i):
    return i + 1 if i % 2 else i - 1


def n_pad(n):
    return (n + 255) // 256 * 256


def lane_offsets(i, x, d, np_):
    """Slot offsets (in elements) of direction i for sites x with pull-table
    entries d; a sentinel entry selects the own opposite slot."""
    sent = (d == BB) | (d == GHOST)
    fluid = x + d.astype(np.int64) + CX[i] + np_ + 1
    own = x + (opp(i) - i + 1) * np_ + CX[i] + 1
    return np.where(sent, own, fluid), sent


def check_plan(geoms, wall_mode, s=4, tile=128):
    p = lbm.lbm_plan_export(geoms, wall_modes=[wall_mode] * len(geoms))
    nbr, N = p["nbr"], p["n_sites"]
    np_ = n_pad(N)
    small = Q * np_ * s < 2 ** 31
    x = np.arange(N, dtype=np.int64)
    # lanes past the last site, up to the end of the last two-site tile
    tail = np.arange(N, (N + tile - 1) // tile * tile, dtype=np.int64)
    xs_tail = np.minimum(tail, np_ - 1)
    for i in range(1, Q):
        base = i * np_ - CX[i] - np_ - 1
        off, sent = lane_offsets(i, x, nbr[i - 1], np_)
        assert off.min() >= 0
        # 32-bit byte offsets where the buffers are below 2 GiB, element
        # offsets otherwise; both fit their 32-bit registers
        assert (off * s).max() < 2 ** 32 if small else off.max() < 2 ** 32
        slot = base + off
        want = np.where(sent, opp(i) * np_ + x, i * np_ + x + nbr[i - 1].astype(np.int64))
        assert np.array_equal(slot, want), i
        assert slot.min() >= 0 and slot.max() < Q * np_
        # fluid upstream sites lie among the N sites of the plane
        up = x + nbr[i - 1].astype(np.int64)
        assert np.all((up[~sent] >= 0) & (up[~sent] < N))
        if len(tail):
            own = xs_tail + (opp(i) - i + 1) * np_ + CX[i] + 1
            t = base + own
            assert np.array_equal(t, opp(i) * np_ + xs_tail)
            assert t.min() >= 0 and t.max() < Q * np_
    return N, np_


@pytest.mark.parametrize("seed", [1, 2, 5])
def test_random_boxes(seed):
    rng = np.random.default_rng(seed)
    g = H.one_iolet_per_site(inputs.random_labels((9, 10, 11), rng))
    for mode in (lbm.BOUNCEBACK, lbm.ELASTIC):
        check_plan([g], mode)


def test_tube_workload():
    wl = workloads.tube32()
    N, _ = check_plan(wl.geoms, lbm.ELASTIC)
    assert N == 1_640_960


def test_tree_workload():
    wl = workloads.tree()
    N, _ = check_plan(wl.geoms, lbm.ELASTIC)
    assert N == 7_484_227


def test_small_sweep():
    wl = workloads.sweep(seed=4, n=8, target_sites=1e6)
    check_plan(wl.geoms, lbm.ELASTIC)


def test_element_offsets_fit_below_the_runtime_limit():
    """Two sites per lane form element offsets up to about 3 N_pad + 2; the
    runtime accepts that launch only while they fit 32 bits (1.43e9 padded
    sites).  The largest offsets of the scheme at that limit still fit."""
    limit = ((1 << 32) - 4096) // 3
    np_ = limit // 256 * 256
    x = np.array([np_ - 1], np.int64)
    worst = max(int(lane_offsets(i, x, np.array([BB], np.int32), np_)[0].max())
                for i in range(1, Q))
    # the own opposite slot of the last site in a lower plane is the largest
    # offset (fluid links stay below 2 N_pad + 2)
    assert worst == 3 * np_ + 1 and worst < 2 ** 32
