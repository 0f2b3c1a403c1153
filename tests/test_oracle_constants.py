"""Pins of the oracle's ray-count constants against the paper's printed values,
closed forms, and derivations that do not use the paper's integrals."""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import constants as C
from oracle.rays import face_class_measures
from conftest import read_golden


def test_appendix_2d_constants():
    # Appendix, 3x3 example with dx = dy = D = 1: A_tot = 8 D and the c values.
    k = C.constants_2d(1.0, 1.0)
    assert k["Atot"] == pytest.approx(8.0, abs=1e-15)
    r2 = math.sqrt(2.0)
    assert k["c"]["xx"] == pytest.approx(2 * r2 - 2, abs=1e-15)
    assert k["c"]["yy"] == pytest.approx(2 * r2 - 2, abs=1e-15)
    assert k["c"]["xy"] == pytest.approx(2 - r2, abs=1e-15)


@pytest.mark.parametrize("dx,dy", [(1.0, 1.0), (1.0, 0.6), (0.3, 1.7)])
def test_boundary_example_integral(dx, dy):
    # Eq. AE_Boundary_example: the counter of the example topology, written as
    # the paper's angular integral, equals dx + dy - sqrt(dx^2 + dy^2) = c_xy,
    # and A_E^{n+1} = 2 dy - A_E^n (Eq. AE_Boundary_example2).
    a = math.atan(dy / dx)
    i1, _ = integrate.quad(lambda t: dx * math.sin(t), 0, a, epsabs=1e-15)
    i2, _ = integrate.quad(lambda t: dy * math.cos(t), a, math.pi / 2, epsabs=1e-15)
    k = C.constants_2d(dx, dy)
    assert i1 + i2 == pytest.approx(k["c"]["xy"], abs=1e-13)
    assert 2 * dy - (i1 + i2) == pytest.approx(dy - dx + math.hypot(dx, dy), abs=1e-13)


@pytest.mark.parametrize("dx,dy", [(1.0, 1.0), (1.0, 0.6), (0.45, 1.3)])
def test_2d_constants_match_traced_rays(dx, dy):
    # Brute force: trace rays through the face neighbour and measure how many
    # left it by its far face (-> c_jj) and by each lateral face (-> c_xy).
    k = C.constants_2d(dx, dy)
    for axis, jj in ((0, "xx"), (1, "yy")):
        for sign in (+1, -1):
            m = face_class_measures((dx, dy), axis, sign, n_theta=3000, n_face=3000)
            far = [0, 0, 0]
            far[axis] = 2 * sign
            assert m[tuple(far)] == pytest.approx(k["c"][jj], rel=2e-4)
            lat_keys = [key for key in m if key != tuple(far)]
            assert len(lat_keys) == 2
            for key in lat_keys:
                assert m[key] == pytest.approx(k["c"]["xy"], rel=2e-4)
            # Eq. AE_Interior: all rays through a face add up to 2 * (face length)
            assert sum(m.values()) == pytest.approx(k["face"][axis], rel=1e-6)


def test_isotropic_3d_printed_digits():
    g = {row[0]: float(row[1]) for row in read_golden("isotropic_3d_constants.txt")}
    far, near = C.isotropic_3d(1.0)
    assert abs(far - g["far"]) <= 0.6e-13
    assert abs(near - g["near"]) <= 0.6e-13


def test_isotropic_quadrature_matches_closed_form():
    far, near = C.isotropic_3d(1.0)
    assert C.far_face_quadrature(1.0, 1.0, 1.0) == pytest.approx(far, abs=1e-13)
    assert C.dihedral_quadrature(1.0, 1.0, 1.0) == pytest.approx(near, abs=1e-13)
    # scaling with the square of the spacing
    assert C.far_face_quadrature(0.3, 0.3, 0.3) == pytest.approx(far * 0.09, abs=1e-14)


def _far_face_overlap_integral(dj, dl1, dl2):
    """c_jj derived from geometry without the paper's integral: a ray through
    the shared face, followed back through the neighbour along direction
    (cos t, sin t cos p, sin t sin p) in (j, l1, l2), left the neighbour by its
    far face iff its entry point lies in the far face shifted by
    dj tan t (cos p, sin p); that overlap is a product of two interval lengths.
    Integrate cos t * overlap over the hemisphere."""

    def inner(t, p):
        tt = math.tan(t) * dj
        return (math.cos(t) * math.sin(t) * max(0.0, dl1 - tt * abs(math.cos(p)))
                * max(0.0, dl2 - tt * abs(math.sin(p))))

    def over_t(p):
        # the overlap vanishes beyond the smaller of the two cut-off angles
        c1 = abs(math.cos(p))
        s1 = abs(math.sin(p))
        cut = min(math.atan(dl1 / (dj * c1)) if c1 > 0 else math.pi / 2,
                  math.atan(dl2 / (dj * s1)) if s1 > 0 else math.pi / 2)
        v, _ = integrate.quad(inner, 0.0, cut, args=(p,), epsabs=1e-14, epsrel=1e-12, limit=200)
        return v

    v, _ = integrate.quad(over_t, 0.0, math.pi / 2, epsabs=1e-14, epsrel=1e-12, limit=200)
    return 4.0 * v


SPACINGS_3D = [(1.0, 1.0, 1.0), (1.0, 0.7, 1.9), (0.25, 0.5, 0.33)]


@pytest.mark.parametrize("sp", SPACINGS_3D)
def test_far_face_matches_geometry(sp):
    k = C.constants_3d(*sp, force_quadrature=True)
    for a, ax in enumerate("xyz"):
        others = [sp[b] for b in range(3) if b != a]
        ref = _far_face_overlap_integral(sp[a], *others)
        assert k["c"][ax + ax] == pytest.approx(ref, rel=1e-9)


@pytest.mark.parametrize("sp", SPACINGS_3D)
def test_dihedral_from_face_identities(sp):
    # Every ray through a face came from the neighbour's far face or one of its
    # four lateral faces, and the face total is pi * area: so
    # 2 c_xy + 2 c_yz + c_yy = pi dx dz and cyclic.  Given the far-face
    # constants from geometry, the three identities fix the three dihedrals.
    dx, dy, dz = sp
    far = {}
    for a, ax in enumerate("xyz"):
        others = [sp[b] for b in range(3) if b != a]
        far[ax] = _far_face_overlap_integral(sp[a], *others)
    sa = (math.pi * dx * dz - far["y"]) / 2   # c_xy + c_yz
    sb = (math.pi * dy * dz - far["x"]) / 2   # c_xy + c_xz
    sc = (math.pi * dx * dy - far["z"]) / 2   # c_xz + c_yz
    ref = {"xy": (sa + sb - sc) / 2, "xz": (sb + sc - sa) / 2, "yz": (sa + sc - sb) / 2}
    k = C.constants_3d(*sp, force_quadrature=True)
    for key, v in ref.items():
        assert k["c"][key] == pytest.approx(v, rel=1e-8)


@pytest.mark.parametrize("sp", SPACINGS_3D[1:])
def test_dihedral_symmetry_and_swap(sp):
    # c_jk = c_kj (stated after Eq. ICc) and the l1 <-> l2 swap of Eq. FarFaceEquation
    d = dict(zip("xyz", sp))
    for j, k_ in (("x", "y"), ("x", "z"), ("y", "z")):
        l = [d[q] for q in "xyz" if q not in (j, k_)][0]
        assert C.dihedral_quadrature(d[j], d[k_], l) == pytest.approx(
            C.dihedral_quadrature(d[k_], d[j], l), rel=1e-11)
    for j in "xyz":
        l1, l2 = [d[q] for q in "xyz" if q != j]
        assert C.far_face_quadrature(d[j], l1, l2) == pytest.approx(
            C.far_face_quadrature(d[j], l2, l1), rel=1e-11)


def test_3d_totals():
    dx, dy, dz = 1.0, 0.7, 1.9
    k = C.constants_3d(dx, dy, dz)
    assert k["Atot"] == pytest.approx(2 * math.pi * (dx * dy + dx * dz + dy * dz))
    # the per-face total is the hemisphere integral of the projected area
    v, _ = integrate.dblquad(lambda t, p: math.cos(t) * math.sin(t), 0, 2 * math.pi, 0, math.pi / 2)
    assert k["face"][1] == pytest.approx(v * dx * dz, rel=1e-12)


def test_3d_constants_match_traced_rays():
    sp = (1.0, 0.7, 1.9)
    k = C.constants_3d(*sp)
    for axis, ax in enumerate("xyz"):
        m = face_class_measures(sp, axis, +1, n_theta=48, n_face=20)
        keys = set(m)
        lat = [b for b in range(3) if b != axis]
        expect = {}
        far = [0, 0, 0]
        far[axis] = 2
        expect[tuple(far)] = k["c"][ax + ax]
        for b in lat:
            for sg in (+1, -1):
                off = [0, 0, 0]
                off[axis] = 1
                off[b] = sg
                expect[tuple(off)] = k["c"][ax + "xyz"[b]]
        assert keys == set(expect)
        for key, v in expect.items():
            assert m[key] == pytest.approx(v, rel=6e-3, abs=2e-3 * k["face"][axis])
