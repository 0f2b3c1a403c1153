"""Brute-force ray tracing on tiny grids.

1. Ray counters from explicit rays.  The counter A_j^i (Section "Method
   Concept", Eq. AE_Interior and the text after Eq. AE_Boundary_example) is the
   measure of straight rays -- over all directions and all lateral offsets --
   that enter cell C through its face with neighbour J.  A ray that reached J
   from another data cell carries a pressure of the current sweep (i = n+1); a
   ray that entered J from a missing cell or from outside the grid starts at J
   and carries the previous sweep's value (i = n); a ray that enters C straight
   from a missing cell starts at C (A_C^n).  Here every one of those rays is
   traced: sample an entry point on the face and a direction, walk backwards
   through J, and see which face of J it left by.  Nothing of the paper's
   closed forms or of the counter formulas is used.

2. A rotating-parallel-ray omnidirectional integrator (Section "Limit of
   Infinite Rays"): parallel face-crossing rays at many angles and offsets;
   along every ray the pressure is integrated cell to cell with the face rule
   P_b = P_a + Delta (f(a) + f(b)) / 2 (Section "Method Concept"), starting
   from the previous sweep's value at the ray's first data cell; each cell
   takes the average over the rays through it; sweeps repeat to convergence.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .counters import directions


def face_class_measures(spacing, axis: int, sign: int, n_theta=2000, n_face=2000,
                        n_phi=None):
    """Measure of rays entering a cell through face (axis, sign), split by the
    face of the neighbour J through which the ray entered J.

    Returns {offset of the previous cell relative to C (tuple of 3 ints): measure}.
    2-D uses a midpoint rule in the angle and in the entry point; 3-D uses a
    midpoint rule in the polar angle from the face normal, the azimuth, and a
    2-D grid of entry points on the face."""
    ndim = len(spacing)
    d = np.array(spacing, dtype=np.float64)
    lat = [k for k in range(ndim) if k != axis]
    J = np.zeros(3, dtype=int)
    J[axis] = sign
    out = {}

    def tally(u, pts, w):
        # u: (K, ndim) backward directions into J, pts: (P, ndim) entry points on the
        # shared face, w: (K,) direction weights (already times the face element).
        # J's box along `axis` spans one spacing beyond the shared face.
        lo = np.zeros(ndim)
        hi = d.copy()
        lo[axis] = d[axis] if sign > 0 else -d[axis]
        hi[axis] = 2 * d[axis] if sign > 0 else 0.0
        t = np.full((u.shape[0], pts.shape[0], ndim), np.inf)
        for k in range(ndim):
            uk = u[:, k][:, None]
            pk = pts[:, k][None, :]
            with np.errstate(divide="ignore", invalid="ignore"):
                tp = np.where(uk > 0, (hi[k] - pk) / uk, np.inf)
                tn = np.where(uk < 0, (lo[k] - pk) / uk, np.inf)
            t[:, :, k] = np.minimum(tp, tn)
        ex = np.argmin(t, axis=2)
        for k in range(ndim):
            for sg in (+1, -1):
                sel = (ex == k) & ((np.sign(u[:, k])[:, None]) == sg)
                m = float((sel * w[:, None]).sum())
                if m == 0.0:
                    continue
                off = J.copy()
                off[k] += sg
                key = tuple(int(v) for v in off)
                out[key] = out.get(key, 0.0) + m

    if ndim == 2:
        k = lat[0]
        th = (np.arange(n_theta) + 0.5) / n_theta * math.pi - math.pi / 2
        u = np.zeros((n_theta, 2))
        u[:, axis] = sign * np.cos(th)
        u[:, k] = np.sin(th)
        s = (np.arange(n_face) + 0.5) / n_face * d[k]
        pts = np.zeros((n_face, 2))
        pts[:, axis] = d[axis] if sign > 0 else 0.0
        pts[:, k] = s
        w = np.cos(th) * (math.pi / n_theta) * (d[k] / n_face)
        for c0 in range(0, n_theta, 256):
            tally(u[c0:c0 + 256], pts, w[c0:c0 + 256])
    else:
        n_phi = n_phi or 2 * n_theta
        k1, k2 = lat
        th = (np.arange(n_theta) + 0.5) / n_theta * (math.pi / 2)
        ph = (np.arange(n_phi) + 0.5) / n_phi * (2 * math.pi)
        TH, PH = np.meshgrid(th, ph, indexing="ij")
        TH = TH.ravel()
        PH = PH.ravel()
        u = np.zeros((TH.size, 3))
        u[:, axis] = sign * np.cos(TH)
        u[:, k1] = np.sin(TH) * np.cos(PH)
        u[:, k2] = np.sin(TH) * np.sin(PH)
        a1 = (np.arange(n_face) + 0.5) / n_face * d[k1]
        a2 = (np.arange(n_face) + 0.5) / n_face * d[k2]
        A1, A2 = np.meshgrid(a1, a2, indexing="ij")
        pts = np.zeros((A1.size, 3))
        pts[:, axis] = d[axis] if sign > 0 else 0.0
        pts[:, k1] = A1.ravel()
        pts[:, k2] = A2.ravel()
        dA = d[k1] * d[k2] / A1.size
        w = np.cos(TH) * np.sin(TH) * (math.pi / 2 / n_theta) * (2 * math.pi / n_phi) * dA
        for c0 in range(0, TH.size, 64):
            tally(u[c0:c0 + 64], pts, w[c0:c0 + 64])
    return out


def ray_counters_bruteforce(mask, spacing, **kw) -> dict:
    """Per-cell counters from traced rays, in the layout of
    :func:`oracle.counters.ray_counters`."""
    mask = np.asarray(mask)
    ndim = mask.ndim
    valid = mask != 0
    pad = 3
    vp = np.pad(valid, pad, constant_values=False)

    def v_at(off):
        sl = []
        for arr_ax in range(ndim):
            a = ndim - 1 - arr_ax
            sl.append(slice(pad + off[a], pad + off[a] + mask.shape[arr_ax]))
        return vp[tuple(sl)].astype(np.float64)

    own = valid.astype(np.float64)
    out = {"C_np1": np.zeros(mask.shape), "C_n": np.zeros(mask.shape)}
    for name, a, s in directions(ndim):
        meas = face_class_measures(spacing, a, s, **kw)
        total = sum(meas.values())
        J = [0, 0, 0]
        J[a] = s
        vJ = v_at(J)
        np1 = np.zeros(mask.shape)
        n = np.zeros(mask.shape)
        for off, m in meas.items():
            vp_ = v_at(off)
            np1 += m * vp_
            n += m * (1.0 - vp_)
        out[(name, "np1")] = own * vJ * np1
        out[(name, "n")] = own * vJ * n
        out["C_n"] += own * (1.0 - vJ) * total
    return out


def _trace_line(p0, dvec, nx, ny, dx, dy):
    """Cells (ix, iy) crossed by the line p0 + t dvec, in order of t."""
    W, H = nx * dx, ny * dy
    tmin, tmax = -np.inf, np.inf
    for p, dd, ext in ((p0[0], dvec[0], W), (p0[1], dvec[1], H)):
        if abs(dd) < 1e-15:
            if p <= 0 or p >= ext:
                return []
            continue
        t1, t2 = (0 - p) / dd, (ext - p) / dd
        tmin, tmax = max(tmin, min(t1, t2)), min(tmax, max(t1, t2))
    if not tmin < tmax:
        return []
    ts = [tmin, tmax]
    if abs(dvec[0]) > 1e-15:
        xs = np.arange(1, nx) * dx
        t = (xs - p0[0]) / dvec[0]
        ts.extend(t[(t > tmin) & (t < tmax)].tolist())
    if abs(dvec[1]) > 1e-15:
        ys = np.arange(1, ny) * dy
        t = (ys - p0[1]) / dvec[1]
        ts.extend(t[(t > tmin) & (t < tmax)].tolist())
    ts = np.sort(np.array(ts))
    cells = []
    for t0, t1 in zip(ts[:-1], ts[1:]):
        if t1 - t0 < 1e-12:
            continue
        tm = 0.5 * (t0 + t1)
        ix = int(math.floor((p0[0] + tm * dvec[0]) / dx))
        iy = int(math.floor((p0[1] + tm * dvec[1]) / dy))
        ix = min(max(ix, 0), nx - 1)
        iy = min(max(iy, 0), ny - 1)
        if not cells or cells[-1] != (ix, iy):
            cells.append((ix, iy))
    return cells


def omni_rays_2d(mask, spacing, grads, n_angles=720, ds_frac=0.05, tol=1e-13, max_sweeps=20000,
                 seed=0):
    """Rotating-parallel-ray integration on a 2-D grid; returns (P, sweeps),
    P in storage order with NaN at masked cells (not gauged)."""
    mask = np.asarray(mask)
    ny, nx = mask.shape
    dx, dy = (float(s) for s in spacing)
    valid = mask != 0
    idx = -np.ones(mask.shape, dtype=np.int64)
    n = int(valid.sum())
    idx[valid] = np.arange(n)
    fx = np.asarray(grads[0], dtype=np.float64)
    fy = np.asarray(grads[1], dtype=np.float64)
    ds = ds_frac * min(dx, dy)
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    bsum = np.zeros(n)
    wsum = np.zeros(n)
    corners = np.array([[0, 0], [nx * dx, 0], [0, ny * dy], [nx * dx, ny * dy]])
    for m in range(n_angles):
        th = (m + 0.5) * 2 * math.pi / n_angles
        dvec = np.array([math.cos(th), math.sin(th)])
        nvec = np.array([-math.sin(th), math.cos(th)])
        proj = corners @ nvec
        smin, smax = proj.min(), proj.max()
        shift = rng.uniform(0, ds)
        for s in np.arange(smin + shift, smax, ds):
            cells = _trace_line(s * nvec, dvec, nx, ny, dx, dy)
            run = []
            for cell in cells + [None]:
                if cell is not None and valid[cell[1], cell[0]]:
                    run.append(cell)
                    continue
                if run:
                    start = idx[run[0][1], run[0][0]]
                    acc = 0.0
                    for q, (ix, iy) in enumerate(run):
                        if q > 0:
                            px, py = run[q - 1]
                            if ix != px:
                                step = (ix - px) * dx * 0.5 * (fx[py, px] + fx[iy, ix])
                            else:
                                step = (iy - py) * dy * 0.5 * (fy[py, px] + fy[iy, ix])
                            acc += step
                        c = idx[iy, ix]
                        rows.append(c)
                        cols.append(start)
                        vals.append(1.0)
                        bsum[c] += acc
                        wsum[c] += 1.0
                    run = []
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    if np.any(wsum == 0):
        raise RuntimeError("some data cell is crossed by no ray; use more rays")
    P = np.zeros(n)
    sweeps = 0
    for sweeps in range(1, max_sweeps + 1):
        P_new = (A @ P + bsum) / wsum
        done = np.linalg.norm(P_new - P) <= tol * max(np.linalg.norm(P_new), 1e-300)
        P = P_new
        if done:
            break
    out = np.full(mask.shape, np.nan)
    out[valid] = P
    return out, sweeps


def cc_counters_bruteforce(mask, spacing, n_theta=1440, ds=0.01):
    """Cell-centred counters from explicit rays (2-D): midpoint rules in the
    angle and the perpendicular offset; every ray is a straight line, its
    path the cells whose centres are nearest to it in each column (a ray
    less steep than the diagonal) or each row (a steeper ray).  For every
    data cell C on a path, the previous cell J and the one before it K
    decide the counter: J missing -> A_C^n, K missing -> A_J^n, else
    A_J^{n+1}.  Cells outside the grid count as missing.  Returns the same
    keys as oracle.cellcentered.cc_counters (without 'Atot')."""
    mask = np.asarray(mask) != 0
    ny, nx = mask.shape
    hx, hy = (float(s) for s in spacing)
    names = {(1, 0): "E", (-1, 0): "W", (0, 1): "N", (0, -1): "S",
             (1, 1): "NE", (-1, 1): "NW", (1, -1): "SE", (-1, -1): "SW"}
    out = {(n, i): np.zeros((ny, nx)) for n in names.values() for i in ("np1", "n")}
    out["C_n"] = np.zeros((ny, nx))
    ext = 3
    ox, oy = 0.5 * nx * hx, 0.5 * ny * hy
    R = math.hypot(ox, oy) + 3 * max(hx, hy)
    s = np.arange(-R + 0.5 * ds, R, ds)
    dth = 2 * math.pi / n_theta

    def data(i, j):
        inside = (i >= 0) & (i < nx) & (j >= 0) & (j < ny)
        v = np.zeros(i.shape, dtype=bool)
        v[inside] = mask[j[inside], i[inside]]
        return v, inside

    for t in range(n_theta):
        th = (t + 0.5) * dth
        cx, cy = math.cos(th), math.sin(th)
        px, py = ox - s * cy, oy + s * cx           # a point of each ray
        if abs(cx) * hy >= abs(cy) * hx:            # shallow: one cell per column
            cols = np.arange(-ext, nx + ext)
            if cx < 0:
                cols = cols[::-1]
            xc = (cols + 0.5) * hx
            tt = (xc[None, :] - px[:, None]) / cx
            yc = py[:, None] + tt * cy
            I = np.broadcast_to(cols[None, :], yc.shape)
            Jr = np.floor(yc / hy).astype(np.int64)
        else:                                       # steep: one cell per row
            rows = np.arange(-ext, ny + ext)
            if cy < 0:
                rows = rows[::-1]
            yc = (rows + 0.5) * hy
            tt = (yc[None, :] - py[:, None]) / cy
            xc2 = px[:, None] + tt * cx
            Jr = np.broadcast_to(rows[None, :], xc2.shape)
            I = np.floor(xc2 / hx).astype(np.int64)
        w = dth * ds
        for p in range(2, I.shape[1]):
            ci, cj = I[:, p], Jr[:, p]
            vc, _ = data(ci, cj)
            if not vc.any():
                continue
            ji, jj = I[:, p - 1], Jr[:, p - 1]
            ki, kj = I[:, p - 2], Jr[:, p - 2]
            vj, _ = data(ji, jj)
            vk, _ = data(ki, kj)
            for key, sel in (("C_n", vc & ~vj), ("np1", vc & vj & vk), ("n", vc & vj & ~vk)):
                if not sel.any():
                    continue
                if key == "C_n":
                    np.add.at(out["C_n"], (cj[sel], ci[sel]), w)
                    continue
                for (dx, dy), nm in names.items():
                    sub = sel & (ji - ci == dx) & (jj - cj == dy)
                    if sub.any():
                        np.add.at(out[(nm, key)], (cj[sub], ci[sub]), w)
    return out
