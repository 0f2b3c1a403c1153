"""The velocity generators and noise models that feed the velocity -> source
stage: analytic properties of the fields (the ABC flow is a Beltrami field,
the Taylor vortex matches the oracle's copy) and the statistics the two
noise equations fix (Eqs. NoisyVectorsTheta and NoisyVectors)."""

import math

import numpy as np
import torch

import synth
from oracle import flow as Fl


def test_taylor_velocity_matches_the_oracle_formula():
    u, P, sp = synth.taylor_velocity((40, 30), t=1.0)
    # the oracle samples the same vortex on a grid centred on the origin
    uo, Po, _ = Fl.taylor_vortex((30, 40), sp, t=1.0)
    for a, b in zip(u, uo):
        assert np.allclose(a.numpy(), b, atol=1e-14)
    assert np.allclose(P.numpy(), Po, atol=1e-14)


def test_abc_velocity_is_a_decaying_beltrami_field():
    n = 48
    u, P, sp = synth.abc_velocity((n, n, n), t=0.3, nu=0.5)
    u = [c.numpy() for c in u]
    # divergence-free and curl u = u up to second-order differences
    div = sum(Fl.d1(u[k], sp[k], k) for k in range(3))
    curl = [Fl.d1(u[2], sp[1], 1) - Fl.d1(u[1], sp[2], 2),
            Fl.d1(u[0], sp[2], 2) - Fl.d1(u[2], sp[0], 0),
            Fl.d1(u[1], sp[0], 0) - Fl.d1(u[0], sp[1], 1)]
    mag = max(np.abs(c).max() for c in u)
    assert np.abs(div).max() < 1e-2 * mag
    assert max(np.abs(c - v).max() for c, v in zip(curl, u)) < 1e-2 * mag
    # amplitude decays as exp(-nu t)
    u0, _, _ = synth.abc_velocity((n, n, n), t=0.0, nu=0.5)
    assert np.allclose(u[0], u0[0].numpy() * math.exp(-0.15), atol=1e-14)
    assert np.allclose(P.numpy(), -0.5 * sum(c * c for c in u), atol=1e-14)


def test_angular_noise_has_fixed_magnitude_and_uniform_direction():
    for nd, shape in ((2, (200, 300)), (3, (40, 50, 30))):
        g = torch.Generator().manual_seed(1)
        u = [torch.randn(tuple(reversed(shape)), generator=g, dtype=torch.float64) for _ in range(nd)]
        s = 0.07
        un = synth.noise_angular(u, s, seed=5)
        d = [a - b for a, b in zip(un, u)]
        mag = torch.sqrt(sum(c * c for c in u))
        dmag = torch.sqrt(sum(c * c for c in d))
        assert torch.allclose(dmag, s * mag, atol=1e-13)
        # a uniform direction has zero mean and covariance I / nd
        n = torch.stack([c / dmag for c in d]).reshape(nd, -1)
        assert n.mean(dim=1).abs().max() < 0.01
        cov = n @ n.T / n.shape[1]
        assert torch.allclose(cov, torch.eye(nd, dtype=cov.dtype) / nd, atol=0.01)
        # seeded: the same seed gives the same field
        assert all(torch.equal(a, b) for a, b in zip(un, synth.noise_angular(u, s, seed=5)))


def test_multiplicative_noise_rescales_without_turning():
    g = torch.Generator().manual_seed(2)
    u = [torch.randn((30, 40, 50), generator=g, dtype=torch.float64) for _ in range(3)]
    s = 0.05
    un = synth.noise_multiplicative(u, s, seed=9)
    # parallel to u: every component scaled by the same factor 1 + s n
    ratio = [a / b for a, b in zip(un, u)]
    assert torch.allclose(ratio[0], ratio[1]) and torch.allclose(ratio[0], ratio[2])
    n = (ratio[0] - 1) / s
    assert abs(float(n.mean())) < 0.01 and abs(float(n.std()) - 1) < 0.01
