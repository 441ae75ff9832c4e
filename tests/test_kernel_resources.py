"""Register use of the update kernel as compiled for gfx950 (no GPU needed:
hipcc cross-compiles).  The default configuration (compressed addressing,
32-bit offsets) must not use scratch memory, and 16-bit storage must fit the
64 registers of 8 waves per SIMD: close to that limit the compiler's
allocation can fall into spilling kilobytes per lane, which costs far more
than any change that triggers it gains.  The 64-bit offset variants (for
population buffers of 2 GiB or more) keep the compiler's occupancy and must
not spill either."""
import re

import pytest

from paper_2108_08783_amd import build


@pytest.fixture(scope="module")
def resources():
    return build.kernel_resources(build.device_asm("kernels.hip"))


DTYPES = {0: "f64", 1: "f32", 2: "f16", 3: "bf16"}


@pytest.mark.parametrize("dt", [0, 1, 2, 3])
@pytest.mark.parametrize("ntl", [0, 1])
def test_default_update_kernel_has_no_scratch(resources, dt, ntl):
    # k_step<DT, compressed addressing, 32-bit offsets, non-temporal loads>
    pat = re.compile(rf"k_stepILi{dt}ELi0ELb1ELb{ntl}E")
    names = [n for n in resources if pat.search(n)]
    assert len(names) == 1, names
    r = resources[names[0]]
    assert r["scratch"] == 0, (DTYPES[dt], r)
    if dt in (2, 3):
        assert r["vgpr"] <= 64, (DTYPES[dt], r)


@pytest.mark.parametrize("dt", [0, 1, 2, 3])
@pytest.mark.parametrize("small", [0, 1])
def test_compressed_update_kernels_have_no_scratch(resources, dt, small):
    # compressed addressing with 32-bit (small) and 64-bit offsets, the
    # latter taken for population buffers of 2 GiB or more
    pat = re.compile(rf"k_stepILi{dt}ELi0ELb{small}ELb[01]E")
    names = [n for n in resources if pat.search(n)]
    assert len(names) == 2, names
    for n in names:
        assert resources[n]["scratch"] == 0, (DTYPES[dt], small, resources[n])


def test_no_update_kernel_spills_more_than_a_few_registers(resources):
    # the offset-table variants at 8 waves may keep a few dwords in scratch
    names = [n for n in resources if "k_stepILi" in n]
    assert len(names) == 4 * 3 * 2 * 2, len(names)
    for n in names:
        assert resources[n]["scratch"] <= 16, (n, resources[n])


@pytest.mark.parametrize("small", [0, 1])
@pytest.mark.parametrize("ntl", [0, 1])
def test_two_sites_per_lane_kernel_has_no_scratch(resources, small, ntl):
    # k_step_pair<FP32, 32-bit offsets, non-temporal loads>: two sites' 19
    # populations and offsets in registers (5 waves per SIMD), never spilled
    pat = re.compile(rf"k_step_pairILi1ELb{small}ELb{ntl}E")
    names = [n for n in resources if pat.search(n)]
    assert len(names) == 1, names
    r = resources[names[0]]
    assert r["scratch"] == 0 and r["vgpr"] <= 102, r
