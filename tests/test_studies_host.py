"""Host checks of the grain-averaging helpers used by the recovery study."""
import numpy as np

from paper_2105_01612_amd import workload as wl


def test_grain_labels_match_the_generator():
    spec = wl.FieldSpec((12, 10, 14), grains=9, sigma_grain=50.0, sigma_noise=0.0, seed=77)
    S = wl.voronoi_field(spec)
    lab = wl.grain_labels(spec)
    assert lab.shape == spec.shape and lab.min() >= 0 and lab.max() < spec.grains
    # with no noise and no gradient every grain is constant: S equals its grain average
    assert np.allclose(wl.grain_average(S, lab, spec.grains), S, rtol=1e-13, atol=0)


def test_grain_average_keeps_grain_means_and_is_idempotent():
    spec = wl.FieldSpec((8, 9, 10), grains=6, sigma_grain=20.0, sigma_noise=3.0, sigma_grad=1.0, seed=5)
    S = wl.voronoi_field(spec)
    lab = wl.grain_labels(spec)
    A = wl.grain_average(S, lab, spec.grains)
    for g in range(spec.grains):
        m = lab == g
        if m.any():
            assert np.allclose(A[:, m].mean(axis=1), S[:, m].mean(axis=1), rtol=0, atol=1e-10)
            assert np.ptp(A[:, m], axis=1).max() == 0.0
    assert np.allclose(wl.grain_average(A, lab, spec.grains), A, rtol=0, atol=1e-12)
