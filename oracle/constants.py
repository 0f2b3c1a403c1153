"""Ray-count constants of the face-crossing scheme.

2-D: Eq. cxx2D gives c_xx, c_yy, c_xy in closed form; Eq. Atot2D gives
A_tot = 4 (dx + dy) and Eq. AE_Interior the per-face total 2 * (face length).

3-D (Section "Arbitrary Boundary Weights for 'Face-Crossing' Scheme in 3D"):
the per-face total is pi * (face area) and A_tot = 2 pi (dx dy + dx dz + dy dz).
The far-face constant c_jj is the 1-D integral of Eq. FarFaceEquation; the
dihedral constant c_jk (j != k) is I_A + I_B1 + I_B2 + I_C (Eqs. IAc, IB1c,
IB2c, ICc).  For isotropic grids the closed forms of Eqs. ConstantFarFace and
ConstantNearFaces are used instead of quadrature.

Quadrature is scipy's adaptive QUADPACK routine, used here as a library step.
"""

from __future__ import annotations

import math

import numpy as np
from scipy import integrate

AXES = "xyz"


def constants_2d(dx: float, dy: float) -> dict:
    """Eq. cxx2D plus A_tot (Eq. Atot2D) and the face totals (Eq. AE_Interior)."""
    dd = math.sqrt(dx * dx + dy * dy)
    c = {
        "xx": 2.0 * (dd - dx),
        "yy": 2.0 * (dd - dy),
        "xy": dx + dy - dd,
    }
    c["yx"] = c["xy"]
    return {
        "c": c,
        "Atot": 4.0 * (dx + dy),
        # rays through a face normal to x sweep its length dy over (-pi/2, pi/2)
        "face": (2.0 * dy, 2.0 * dx),
    }


def far_face_quadrature(dj: float, dl1: float, dl2: float) -> float:
    """c_jj by Eq. FarFaceEquation: dj is the spacing normal to the face, dl1
    and dl2 the two in-plane spacings, dl1c = dl1 cos(phi), dl1s = dl1 sin(phi)."""

    def integrand(phi):
        l1c = dl1 * math.cos(phi)
        l1s = dl1 * math.sin(phi)
        at = math.atan(dj / l1s)
        return (math.pi * (dl2 * l1s - dj * l1c)
                + 2.0 * (dj * l1c * at - dl2 * l1s * at))

    val, _ = integrate.quad(integrand, math.atan(dj / dl2), math.pi / 2,
                            epsabs=1e-15, epsrel=1e-13, limit=200)
    return val


def dihedral_quadrature(dj: float, dk: float, dl: float) -> float:
    """c_jk for j != k as I_A + I_B1 + I_B2 + I_C; dl is the spacing along the
    third axis, dkc = dk cos(phi), dks = dk sin(phi)."""
    num = dj**2 * dk**2
    den = 2 * dl**4 + 2 * dl**2 * dj**2 + 2 * dl**2 * dk**2 + dj**2 * dk**2
    I_A = 0.5 * dl**2 * math.atanh(num / den)

    phi0 = math.atan(dj / dl)

    def b1(phi):
        kc = dk * math.cos(phi)
        ks = dk * math.sin(phi)
        t1 = dl * ks * (math.atan(dl / kc) - dl * kc / (dl**2 + kc**2))
        t2 = kc * ks * (math.log(kc / math.sqrt(kc**2 + dl**2)) + dl**2 / (2 * (dl**2 + kc**2)))
        return t1 + t2

    def b2(phi):
        kc = dk * math.cos(phi)
        ks = dk * math.sin(phi)
        t1 = dl * ks * (math.atan(dj / ks) - dj * ks / (dj**2 + ks**2))
        t2 = kc * ks * (math.log(ks / math.sqrt(ks**2 + dj**2)) + dj**2 / (2 * (dj**2 + ks**2)))
        return t1 + t2

    def c(phi):
        s = math.sin(phi)
        return 0.5 * dj * dk**2 * s * (2 * dl * s - dj * math.cos(phi)) / (dj**2 + dk**2 * s * s)

    opts = dict(epsabs=1e-15, epsrel=1e-13, limit=200)
    I_B1, _ = integrate.quad(b1, 0.0, phi0, **opts)
    I_B2, _ = integrate.quad(b2, phi0, math.pi / 2, **opts)
    I_C, _ = integrate.quad(c, phi0, math.pi / 2, **opts)
    return I_A + I_B1 + I_B2 + I_C


def isotropic_3d(delta: float = 1.0) -> tuple:
    """Closed forms of Eqs. ConstantFarFace and ConstantNearFaces."""
    r2 = math.sqrt(2.0)
    far = (math.log(4.0 / 3.0) - r2 * math.atan(r2) + 0.5 * r2 * math.atan(10 * r2 / 23)
           + math.pi * (r2 - 1.0))
    near = (math.pi / 2 - 0.25 * math.log(4.0 / 3.0) - 0.25 * r2 * math.atan(10 * r2 / 23)
            - 0.5 * r2 * math.atan(r2))
    return far * delta**2, near * delta**2


def constants_3d(dx: float, dy: float, dz: float, force_quadrature: bool = False) -> dict:
    """All six c_jk, A_tot and the per-face totals pi * area (x, y, z faces)."""
    d = {"x": dx, "y": dy, "z": dz}
    c = {}
    if dx == dy == dz and not force_quadrature:
        far, near = isotropic_3d(dx)
        for a in AXES:
            c[a + a] = far
        for a in AXES:
            for b in AXES:
                if a != b:
                    c[a + b] = near
    else:
        for a in AXES:
            l1, l2 = [d[b] for b in AXES if b != a]
            c[a + a] = far_face_quadrature(d[a], l1, l2)
        for a, b in (("x", "y"), ("x", "z"), ("y", "z")):
            l = [d[q] for q in AXES if q not in (a, b)][0]
            v = dihedral_quadrature(d[a], d[b], l)
            c[a + b] = v
            c[b + a] = v
    return {
        "c": c,
        "Atot": 2.0 * math.pi * (dx * dy + dx * dz + dy * dz),
        "face": (math.pi * dy * dz, math.pi * dx * dz, math.pi * dx * dy),
    }


def constants(spacing) -> dict:
    spacing = tuple(float(s) for s in spacing)
    if len(spacing) == 2:
        return constants_2d(*spacing)
    if len(spacing) == 3:
        return constants_3d(*spacing)
    raise ValueError("spacing must have 2 or 3 entries")


def as_array(consts: dict, ndim: int) -> np.ndarray:
    """c_jk as an ndim x ndim array indexed by axis numbers (0 = x)."""
    out = np.zeros((ndim, ndim))
    for a in range(ndim):
        for b in range(ndim):
            out[a, b] = consts["c"][AXES[a] + AXES[b]]
    return out
