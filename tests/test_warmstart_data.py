"""Host-side pieces of the warm-start training recipe (no GPU): seeded sample specifications and
the loss normaliser."""
import numpy as np

import lattice_inputs as li
from oracle import nn_oracle


def test_sample_specs_are_seeded_and_in_range():
    from paper_2110_00733_amd.warmstart_train import sample_spec
    r_lo, r_hi = li.octet_radius(64, 0.03), li.octet_radius(64, 0.30)
    specs = [sample_spec(i) for i in range(200)]  # the radius range is searched once (cached)
    assert specs[17] == sample_spec(17)  # same seed, same sample
    assert len({s["seed_rough"] for s in specs}) == 200 and len({s["seed_pores"] for s in specs}) == 200
    for s in specs:
        assert r_lo <= s["radius"] <= r_hi
        assert 0.0 <= s["rough_amp"] <= 1.5 and 1.0 <= s["rough_sigma"] <= 3.0
        assert 0 <= s["n_pores"] <= 8 and 1.0 <= s["pore_median_vox"] <= 2.0
    # r^2 uniform: the mean of r^2 sits half way between the end points
    r2 = np.array([s["radius"] ** 2 for s in specs])
    assert abs(r2.mean() - 0.5 * (r_lo ** 2 + r_hi ** 2)) < 0.1 * (r_hi ** 2 - r_lo ** 2)
    assert {s["n_pores"] for s in specs} == set(range(9))


def test_training_geometry_density_range():
    from paper_2110_00733_amd.warmstart_train import make_phi, sample_spec
    lo = min(range(60), key=lambda i: sample_spec(i)["radius"])
    hi = max(range(60), key=lambda i: sample_spec(i)["radius"])
    rho_lo, rho_hi = make_phi(lo, n=32).mean(), make_phi(hi, n=32).mean()
    assert 0.02 < rho_lo < rho_hi < 0.32


def test_weight_sums_match_the_loss_weight():
    from paper_2110_00733_amd.warmstart_train import weight_sums
    rng = np.random.default_rng(0)
    phis = rng.choice([0.0, 0.25, 0.5, 1.0], size=(3, 4, 4, 4)).astype(np.float32)
    for w3 in ((0.1, 1.0, 0.0), (1.0, 0.0, 0.0), (1.0, 1.0, 4.0)):
        want = [nn_oracle.loss_weight(p.astype(np.float64), w3).sum() for p in phis]
        assert np.allclose(weight_sums(phis, w3), want, rtol=1e-12)
