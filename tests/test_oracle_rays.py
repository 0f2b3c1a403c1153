"""The matrix method against brute-force many-ray omnidirectional integration
on a tiny masked grid (Section "Limit of Infinite Rays")."""

import numpy as np
import pytest

import synth
from oracle.rays import omni_rays_2d
from oracle.solve import fixed_point, gauge
from oracle.system import assemble

DIMS = (9, 8)
SPACING = (1.0, 0.8)


@pytest.fixture(scope="module")
def case():
    P, g, sp = synth.quadratic(DIMS, seed=3, spacing=SPACING)
    m = synth.disk_mask(DIMS, 4, frac=0.1, rmin=0.1, rmax=0.2).numpy()
    assert (m == 0).sum() >= 7   # a masked hole the rays have to start and stop at
    return m, sp, [x.numpy() for x in g]


def test_rays_match_matrix_method_for_consistent_gradient(case):
    # For a gradient whose face increments are path independent every ray
    # integral agrees, so both estimators return the same field exactly.
    m, sp, g = case
    s = assemble(m, sp)
    p_matrix = fixed_point(s, s.source(g))
    p_rays, _ = omni_rays_2d(m, sp, g, n_angles=360, ds_frac=0.1, tol=1e-14)
    p_rays = gauge(s, s.from_grid(p_rays))
    rms = np.sqrt(np.mean(p_matrix**2))
    assert np.abs(p_rays - p_matrix).max() / rms < 1e-10


def test_rays_close_to_matrix_method_for_noisy_gradient(case):
    # With noise the finite-ray estimator and the matrix method are different
    # averages of inconsistent path integrals; measured here: max-abs
    # difference 6.8e-3 of RMS(P), unchanged when the ray count doubles.
    m, sp, g = case
    rng = np.random.default_rng(1)
    gn = [x + 0.3 * np.std(x) * rng.normal(size=x.shape) for x in g]
    s = assemble(m, sp)
    p_matrix = fixed_point(s, s.source(gn))
    p_rays, _ = omni_rays_2d(m, sp, gn, n_angles=360, ds_frac=0.1, tol=1e-10, max_sweeps=4000)
    p_rays = gauge(s, s.from_grid(p_rays))
    rms = np.sqrt(np.mean(p_matrix**2))
    assert np.abs(p_rays - p_matrix).max() / rms < 1.5e-2
