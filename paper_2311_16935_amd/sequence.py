"""Time-resolved sequences: each snapshot's solve starts from the previous
snapshot's pressure.

The paper's CG inner solve is warm-started from the previous outer
iterate, which shortens the later outer steps (Section "Wall-clock Time
Convergence").  Across a time-resolved sequence the same holds one level
up: consecutive snapshots of a flow have close pressure fields, so the
previous snapshot's converged P is a far better P^0 than zero, and the
outer iteration needs fewer steps to reach the same residual.  This module
only orders the calls; every step runs in ``libpi.so`` (``pi_solve`` with
``PI_WARM_START``).
"""

from __future__ import annotations

from typing import Iterable, List, Optional, Sequence

import torch

from . import Plan, SolveResult


def solve_sequence(plan: Plan, snapshots: Iterable[Sequence[torch.Tensor]], tol: float = 1e-6,
                   max_iter: int = 10**7, P0: Optional[torch.Tensor] = None, warm: bool = True,
                   stream=None) -> List[SolveResult]:
    """Solve every snapshot (a list of gradient components) in order on one
    plan.  With ``warm`` each solve starts from the previous result (the
    first from ``P0`` if given, else from zero); without it every solve
    starts from zero.  Returns one SolveResult per snapshot, each with its
    own P tensor."""
    out: List[SolveResult] = []
    prev = P0
    for grads in snapshots:
        P = torch.empty(plan.shape, dtype=plan.dtype, device=grads[0].device)
        start = warm and prev is not None
        if start:
            P.copy_(prev)
        res = plan.solve(grads, P=P, tol=tol, max_iter=max_iter, warm_start=start, stream=stream)
        out.append(res)
        prev = res.P
    return out
