"""The velocity -> source stage (pi_flow_source, through the C interface)
against the FP64 oracle of oracle/flow.py on the same FP32 inputs.  Bar:
max-abs error <= 2e-6 of the largest reference component (FP64 arithmetic
on both sides; the kernel rounds its output to FP32).  Grids include axes of
length 1, 2 and 3, where the difference rules change."""

import numpy as np
import pytest
import torch

from gpu_common import DEV, announce, requires_gpu
from oracle import flow as Fl

pytestmark = [pytest.mark.gpu, requires_gpu]


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)


def _check(got, ref, what):
    scale = max(np.abs(r).max() for r in ref)
    for g, r in zip(got, ref):
        err = np.abs(g.cpu().numpy().astype(np.float64) - r).max()
        assert err <= 2e-6 * scale, f"{what}: {err:.3e} (scale {scale:.3e})"


def _fields(rng, shape, k, smooth=True):
    """k smooth random fields (sums of a few sinusoids), FP32-representable."""
    nd = len(shape)
    axes = [np.linspace(0, 1, n) for n in shape]
    mesh = np.meshgrid(*axes, indexing="ij")
    out = []
    for _ in range(k):
        f = np.zeros(shape)
        for _ in range(3):
            phase = rng.uniform(0, 2 * np.pi, size=nd)
            freq = rng.uniform(0.5, 2.0, size=nd)
            f += rng.normal() * np.cos(sum(2 * np.pi * fr * m + ph for fr, m, ph in zip(freq, mesh, phase)))
        out.append(_f32(f))
    return out


SHAPES = [(17, 23), (2, 9), (3, 5), (1, 6), (6, 7, 9), (3, 4, 5), (2, 3, 6), (1, 5, 4)]


@pytest.mark.parametrize("shape", SHAPES, ids=[str(s) for s in SHAPES])
def test_navier_stokes_source(shape):
    from paper_2311_16935_amd import flow

    announce("flow ns", shape)
    rng = np.random.default_rng(len(shape) * 100 + shape[-1])
    nd = len(shape)
    sp = tuple(rng.uniform(0.05, 0.2, size=nd))
    u, up, un = _fields(rng, shape, nd), _fields(rng, shape, nd), _fields(rng, shape, nd)
    dt, rho, mu = 0.01, 1.3, 0.02
    ref = Fl.ns_source(u, sp, rho, mu, Fl.time_derivative(up, un, dt))
    got = flow.pi_flow_source(flow.PI_FLOW_NS, [_dev(a) for a in u], sp, u_prev=[_dev(a) for a in up],
                              u_next=[_dev(a) for a in un], rho=rho, mu=mu, dt=dt)
    _check(got, ref, "ns unsteady")
    ref = Fl.ns_source(u, sp, rho, 0.0)
    got = flow.pi_flow_source(flow.PI_FLOW_NS, [_dev(a) for a in u], sp, rho=rho, mu=0.0)
    _check(got, ref, "ns steady inviscid")


@pytest.mark.parametrize("shape", SHAPES, ids=[str(s) for s in SHAPES])
def test_rans_and_compressible_sources(shape):
    from paper_2311_16935_amd import flow

    announce("flow rans/compressible", shape)
    rng = np.random.default_rng(7 + shape[0] * 13 + shape[-1])
    nd = len(shape)
    sp = tuple(rng.uniform(0.05, 0.2, size=nd))
    U = [_f32(300.0 + 40.0 * f) for f in _fields(rng, shape, nd)]
    R = [_f32(500.0 + 100.0 * f) for f in _fields(rng, shape, 3 if nd == 2 else 6)]
    ref = Fl.rans_source(U, sp, 1.1, R)
    got = flow.pi_flow_source(flow.PI_FLOW_RANS, [_dev(a) for a in U], sp, R=[_dev(a) for a in R], rho=1.1)
    _check(got, ref, "rans")
    kw = dict(gas_R=287.0, gamma=1.4, T_inf=173.0, M_inf=2.0, V_inf=520.0)
    ref = Fl.compressible_source(U, sp, R=R, **kw)
    got = flow.pi_flow_source(flow.PI_FLOW_COMPRESSIBLE, [_dev(a) for a in U], sp, R=[_dev(a) for a in R], **kw)
    _check(got, ref, "compressible")


def test_argument_checks():
    from paper_2311_16935_amd import PiError, flow

    u = [torch.zeros((4, 4), device=DEV) for _ in range(2)]
    with pytest.raises(PiError):
        flow.pi_flow_source(7, u, (1.0, 1.0))
    with pytest.raises(PiError):
        flow.pi_flow_source(flow.PI_FLOW_NS, u, (1.0, 0.0))
    with pytest.raises(PiError):  # snapshots need dt > 0
        flow.pi_flow_source(flow.PI_FLOW_NS, u, (1.0, 1.0), u_prev=u, u_next=u, dt=0.0)


def test_taylor_vortex_velocity_to_pressure():
    """End to end on the GPU: Taylor-vortex velocity snapshots -> source
    (pi_flow_source) -> pressure (pi_solve) against the analytic pressure,
    up to the constant; the error is the discretisation error (second order)
    of the difference rules and of the integration."""
    import paper_2311_16935_amd as pi
    from paper_2311_16935_amd import flow

    announce("flow taylor vortex")
    errs = []
    for n in (101, 201):
        h = 6.0 / (n - 1)
        dt = 1e-3
        u, P, _ = Fl.taylor_vortex((n, n), (h, h), t=1.0)
        up, _, _ = Fl.taylor_vortex((n, n), (h, h), t=1.0 - dt)
        un, _, _ = Fl.taylor_vortex((n, n), (h, h), t=1.0 + dt)
        f = flow.pi_flow_source(flow.PI_FLOW_NS, [_dev(a) for a in u], (h, h), u_prev=[_dev(a) for a in up],
                                u_next=[_dev(a) for a in un], rho=1.0, mu=1.0, dt=dt)
        plan = pi.Plan((n, n), (h, h), fixed_point=True)
        res = plan.solve(f, tol=1e-8)
        assert res.status == 0
        Pg = res.P.cpu().numpy().astype(np.float64)
        Pt = P - P.mean()
        errs.append(np.sqrt(np.mean((Pg - Pt) ** 2)) / np.abs(Pt).max())
        plan.close()
    assert errs[-1] < 2e-3, errs
    assert errs[0] / errs[1] > 3.0, errs


def test_abc_flow_velocity_to_pressure():
    """3-D end to end: decaying ABC-flow snapshots -> source -> pressure
    against P = -rho |u|^2 / 2 up to the constant, converging at second
    order."""
    import paper_2311_16935_amd as pi
    import synth
    from paper_2311_16935_amd import flow

    announce("flow abc")
    rho, nu, t, dt = 1.0, 0.5, 0.2, 1e-3
    errs = []
    for n in (32, 64):
        u, P, sp = synth.abc_velocity((n, n, n), t=t, nu=nu, rho=rho)
        up = synth.abc_velocity((n, n, n), t=t - dt, nu=nu, rho=rho)[0]
        un = synth.abc_velocity((n, n, n), t=t + dt, nu=nu, rho=rho)[0]
        f = flow.pi_flow_source(flow.PI_FLOW_NS, [_dev(c) for c in u], sp, u_prev=[_dev(c) for c in up],
                                u_next=[_dev(c) for c in un], rho=rho, mu=rho * nu, dt=dt)
        plan = pi.Plan((n, n, n), sp, fixed_point=True)
        res = plan.solve(f, tol=1e-8)
        assert res.status == 0
        Pt = P.numpy() - P.numpy().mean()
        errs.append(np.sqrt(np.mean((res.P.cpu().numpy().astype(np.float64) - Pt) ** 2)) / np.abs(Pt).max())
        plan.close()
    assert errs[-1] < 5e-3, errs
    assert errs[0] / errs[1] > 3.0, errs
