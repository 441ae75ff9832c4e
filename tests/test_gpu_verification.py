"""The paper's verification cylinder (Sec. 2.4, R = 50 lattice spacings,
alpha = 3, run at tau = 0.8 as the same dimensionless problem): after three
periods the rigid run follows the rigid Womersley solution, and the elastic
run follows the elastic-tube shape with M from the Sec. 2.3 relation at the
paper's F = 0.85 better than the rigid shape, within the paper's error
level."""
import pytest

pytestmark = pytest.mark.gpu


def test_womersley_rigid_and_elastic_shapes():
    from paper_2108_08783_amd import lbm, verification
    rigid = verification.womersley(50, lbm.BOUNCEBACK, tau=0.8, log=print)
    elastic = verification.womersley(50, lbm.ELASTIC, tau=0.8, log=print)
    # rigid: measured-gradient Womersley solution and the fitted rigid shape
    assert max(p["err_rel_amplitude"] for p in rigid["phases"]) < 0.03
    assert rigid["shape_fits"]["rigid_model"]["err_max_rel_amplitude"] < 0.03
    # elastic: the elastic shape fits, and fits better than the rigid one
    fe = elastic["shape_fits"]["elastic_model"]["err_max_rel_amplitude"]
    fr = elastic["shape_fits"]["rigid_model"]["err_max_rel_amplitude"]
    print({"elastic_model": fe, "rigid_model": fr})
    assert fe < 0.13 and fe < 0.75 * fr
