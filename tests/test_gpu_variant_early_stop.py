"""The fixed-point CG variant when an outer step's inner solve ends after its
first pass.

The variant's inner CG stops as soon as its residual is well below the
tolerance.  When that happens after the first pass of an outer step, the
correction buffer still holds the previous outer step's sum, and the outer
update must not add it again.  The start is built so that this happens at a
known step: P^0 is the oracle's fixed point plus two smooth eigenvectors of
the fixed point's operator (cosine modes of the unmasked grid, which the
Neumann graph Laplacian [W^{n+1}] - [W^n] has exactly) and a much smaller
third one.  With two inner iterations per outer step, the first outer step
removes the two large modes (CG is exact on two eigenvalues) and leaves the
small mode; the second outer step removes that mode in one CG pass, which
brings the inner residual under half the tolerance, so it stops after that
pass; the next residual check converges.  The trajectory (2 outer steps, 3
inner passes) and the field are checked; the expected values follow from the
oracle's operator alone.
"""

import numpy as np
import pytest
import torch

import synth
from gpu_common import DEV, announce, np_, oracle_for, rel_maxabs, requires_gpu
from oracle.solve import fixed_point, residual_momentum

pytestmark = [pytest.mark.gpu, requires_gpu]


def _cos_mode(nx, ny, kx, ky):
    x, y = np.arange(nx), np.arange(ny)
    return np.outer(np.cos(np.pi * ky * (y + 0.5) / ny), np.cos(np.pi * kx * (x + 0.5) / nx)).ravel()


def _cg_steps(L, r, k):
    """k textbook CG steps on L x = r from x = 0; returns x."""
    x = np.zeros_like(r)
    p = r.copy()
    rr = r @ r
    for _ in range(k):
        q = L @ p
        al = rr / (p @ q)
        x += al * p
        r = r - al * q
        rn = r @ r
        p = r + (rn / rr) * p
        rr = rn
    return x


def test_inner_solve_ending_after_its_first_pass():
    import paper_2311_16935_amd as pi

    nx, ny = 40, 32
    announce("variant early stop", (nx, ny))
    w = synth.random_small(7, 2, (nx, ny), anisotropic=False, mask_frac=0.0)
    sys_ = oracle_for(w)
    L = sys_.L
    S = sys_.source([g.numpy() for g in w.grads])
    Pstar = fixed_point(sys_, S)
    rms = np.sqrt(np.mean(Pstar**2))
    v1, v2, v3 = _cos_mode(nx, ny, 1, 0), _cos_mode(nx, ny, 0, 1), _cos_mode(nx, ny, 3, 2)
    for v in (v1, v2, v3):  # eigenvectors of the oracle's operator
        Lv = L @ v
        lam = (v @ Lv) / (v @ v)
        assert np.linalg.norm(Lv - lam * v) <= 1e-12 * np.linalg.norm(Lv)
    P0 = Pstar + rms * (v1 + 0.7 * v2 + 1e-6 * v3)
    tol = 1e-4
    # preconditions, from the oracle's operator: after one outer step of two
    # exact CG iterations the residual is still above tol (so a second outer
    # step runs) and carried by the small mode, which one CG iteration removes
    P1 = P0 + _cg_steps(L, S - L @ P0, 2)
    eps1 = residual_momentum(sys_, S, P1)
    assert 1.2 * tol < eps1 < 2.0 * tol, eps1
    P2 = P1 + _cg_steps(L, S - L @ P1, 1)
    assert residual_momentum(sys_, S, P2) < 0.05 * tol

    plan = pi.Plan(w.dims, w.spacing, mask=None, fp64=True, fixed_point=True, inner_iters=2)
    g = [x.to(DEV, torch.float64) for x in w.grads]
    P = torch.from_numpy(sys_.to_grid(P0)).to(DEV)
    res = plan.solve(g, P=P, tol=tol, max_iter=50, warm_start=True)
    assert res.status == pi.PI_OK, res.info
    assert res.info["outer_iters"] == 2 and res.info["inner_iters_total"] == 3, res.info
    got = np_(res.P).ravel()
    assert res.info["eps_R"] <= tol
    assert abs(residual_momentum(sys_, S, got) - res.info["eps_R"]) <= 1e-4 * res.info["eps_R"]
    # the field is what one more exact CG iteration on the small mode gives
    assert rel_maxabs(got, Pstar) < 1e-5
    plan.close()
