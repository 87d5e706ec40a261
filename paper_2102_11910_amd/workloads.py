"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no arithmetic of the method: it only draws vortex clouds
and lays out surface points (cylinders, flat plates, ellipses) of the kinds
the paper's examples use (Figs. 3-10).  Both the GPU path and the FP64
oracle consume these inputs; all floating values are rounded to float32 and
returned as float64 so that both sides see identical, float32-representable
data.

Window convention: an n x n node grid of spacing dx centred on the origin,
node (i, j) at (x0 + i dx, y0 + j dx) with x0 = y0 = -(n-1) dx / 2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy import special


def f32(a) -> np.ndarray:
    """Round to float32, return float64."""
    return np.asarray(np.asarray(a, dtype=np.float64).astype(np.float32), dtype=np.float64)


# ----------------------------------------------------------------------------
# surfaces
# ----------------------------------------------------------------------------

@dataclass
class Surface:
    kind: str
    xs: np.ndarray
    ys: np.ndarray
    ds: np.ndarray
    edges: tuple = ()          # indices of sharp edges (plates: LE, TE)
    params: dict = field(default_factory=dict)
    nx: np.ndarray | None = None   # unit normals into the fluid (None: zero-thickness body)
    ny: np.ndarray | None = None

    @property
    def ns(self) -> int:
        return len(self.xs)


def cylinder(radius: float, ns: int, center=(0.0, 0.0)) -> Surface:
    """Circle, theta_p = 2 pi p / ns counter-clockwise from +x; dS = 2 pi a / ns."""
    th = 2.0 * np.pi * np.arange(ns) / ns
    xs = center[0] + radius * np.cos(th)
    ys = center[1] + radius * np.sin(th)
    ds = np.full(ns, 2.0 * np.pi * radius / ns)
    return Surface("cylinder", f32(xs), f32(ys), f32(ds), (),
                   {"radius": radius, "center": center, "theta": th},
                   np.cos(th), np.sin(th))


def flat_plate(chord: float, alpha_deg: float, ns: int, center=(0.0, 0.0)) -> Surface:
    """Plate at incidence alpha (nose up), midpoint rule along the chord.

    Point p at xi_p = -1 + (2p+1)/ns, position center + (c/2) xi_p (cos a, -sin a);
    p = 0 is the leading edge (upstream, raised), p = ns-1 the trailing edge.
    """
    a = np.deg2rad(alpha_deg)
    xi = -1.0 + (2.0 * np.arange(ns) + 1.0) / ns
    xs = center[0] + 0.5 * chord * xi * np.cos(a)
    ys = center[1] - 0.5 * chord * xi * np.sin(a)
    ds = np.full(ns, chord / ns)
    return Surface("plate", f32(xs), f32(ys), f32(ds), (0, ns - 1),
                   {"chord": chord, "alpha_deg": alpha_deg, "center": center, "xi": xi})


def ellipse(a: float, b: float, ns: int, rotation: float = 0.0, center=(0.0, 0.0)) -> Surface:
    """Ellipse with semi-axes a (along x before rotation) and b, points
    equispaced in arc length starting at (a, 0) counter-clockwise; dS = P / ns."""
    m = 1.0 - (min(a, b) / max(a, b)) ** 2
    perim = 4.0 * max(a, b) * special.ellipe(m)
    t = np.linspace(0.0, 2.0 * np.pi, 400001)
    speed = np.hypot(a * np.sin(t), b * np.cos(t))
    arc = np.concatenate([[0.0], np.cumsum(0.5 * (speed[1:] + speed[:-1]) * np.diff(t))])
    arc *= perim / arc[-1]
    tp = np.interp(np.arange(ns) * perim / ns, arc, t)
    x, y = a * np.cos(tp), b * np.sin(tp)
    c, s = np.cos(rotation), np.sin(rotation)
    xs = center[0] + c * x - s * y
    ys = center[1] + s * x + c * y
    ds = np.full(ns, perim / ns)
    nxl, nyl = b * np.cos(tp), a * np.sin(tp)          # outward normal before rotation
    nl = np.hypot(nxl, nyl)
    nxl, nyl = nxl / nl, nyl / nl
    return Surface("ellipse", f32(xs), f32(ys), f32(ds), (),
                   {"a": a, "b": b, "rotation": rotation, "center": center},
                   c * nxl - s * nyl, s * nxl + c * nyl)


def _closed_airfoil(xd, yd, ns: int, alpha_deg: float, center, kind: str, params: dict) -> Surface:
    """Resample a dense closed contour (counter-clockwise, starting and
    ending at the trailing edge, chord along x with the leading edge at
    x = -c/2) to ns points equispaced in arc length from the trailing edge
    (point 0, the body's edge), then set it at incidence alpha (nose up)."""
    seg = np.hypot(np.diff(xd), np.diff(yd))
    arc = np.concatenate([[0.0], np.cumsum(seg)])
    perim = arc[-1]
    sp = np.arange(ns) * perim / ns
    x, y = np.interp(sp, arc, xd), np.interp(sp, arc, yd)
    # outward normals from the contour's direction at each point (counter-clockwise)
    h = 1e-6 * perim
    tx = np.interp(np.mod(sp + h, perim), arc, xd) - np.interp(np.mod(sp - h, perim), arc, xd)
    ty = np.interp(np.mod(sp + h, perim), arc, yd) - np.interp(np.mod(sp - h, perim), arc, yd)
    nrm = np.hypot(tx, ty)
    nxl, nyl = ty / nrm, -tx / nrm
    a = np.deg2rad(alpha_deg)
    ca, sa = np.cos(a), np.sin(a)
    xs = center[0] + ca * x + sa * y
    ys = center[1] - sa * x + ca * y
    ds = np.full(ns, perim / ns)
    params = dict(params, alpha_deg=alpha_deg, center=center, perimeter=perim)
    return Surface(kind, f32(xs), f32(ys), f32(ds), (0,), params,
                   ca * nxl + sa * nyl, -sa * nxl + ca * nyl)


def naca4_symmetric(thickness: float, chord: float, alpha_deg: float, ns: int,
                    center=(0.0, 0.0)) -> Surface:
    """Symmetric NACA four-digit section (00tt: thickness ratio t) with the
    closed trailing edge form of the thickness polynomial, at incidence
    alpha (nose up); points equispaced in arc length from the trailing edge
    (point 0, the edge), counter-clockwise (upper surface first)."""
    beta = np.linspace(0.0, np.pi, 20001)
    xc = 0.5 * (1.0 - np.cos(beta))                  # 0 .. 1, clustered at both ends
    yt = 5.0 * thickness * (0.2969 * np.sqrt(xc) - 0.1260 * xc - 0.3516 * xc ** 2
                            + 0.2843 * xc ** 3 - 0.1036 * xc ** 4)
    xu, yu = xc[::-1], yt[::-1]                      # upper: trailing edge to leading edge
    xd = np.concatenate([xu, xc[1:]]) * chord - 0.5 * chord
    yd = np.concatenate([yu, -yt[1:]]) * chord
    yd[0] = yd[-1] = 0.0
    return _closed_airfoil(xd, yd, ns, alpha_deg, center, "naca",
                           {"thickness": thickness, "chord": chord})


def joukowski(eps_over_b: float, chord: float, alpha_deg: float, ns: int,
              center=(0.0, 0.0)) -> Surface:
    """Symmetric Joukowski airfoil: the circle of radius a = b (1 + e)
    centred at -b e mapped by z = zeta + b^2 / zeta, scaled to the given
    chord, at incidence alpha (nose up).  Potential flow with the Kutta
    condition at its cusp gives the bound circulation -4 pi U a sin(alpha)
    exactly (a after scaling: params["radius"]).  Points equispaced in arc
    length from the cusp (point 0, the edge), counter-clockwise."""
    b = 1.0
    eps = eps_over_b * b
    a = b + eps
    th = np.linspace(0.0, 2.0 * np.pi, 200001)
    zeta = -eps + a * np.exp(1j * th)
    z = zeta + b * b / zeta
    te = 2.0 * b
    le = -(b + 2.0 * eps) - b * b / (b + 2.0 * eps)
    scale = chord / (te - le)
    z = (z - 0.5 * (te + le)) * scale
    xd, yd = z.real, z.imag
    yd[0] = yd[-1] = 0.0
    return _closed_airfoil(xd, yd, ns, alpha_deg, center, "joukowski",
                           {"eps_over_b": eps_over_b, "chord": chord, "radius": a * scale})


# ----------------------------------------------------------------------------
# vortex clouds
# ----------------------------------------------------------------------------

def _accept_first(rng, n, draw, keep, max_rounds=200):
    """Rejection sampling: draw batches of 2n, keep the first n accepted in draw order."""
    out = []
    got = 0
    for _ in range(max_rounds):
        pts = draw(2 * max(n, 1))
        ok = keep(pts)
        pts = pts[ok]
        out.append(pts)
        got += len(pts)
        if got >= n:
            break
    pts = np.concatenate(out)[:n]
    if len(pts) < n:
        raise RuntimeError("rejection sampling did not find enough points")
    return pts


def outside_surface(surf: Surface | None, pts: np.ndarray, margin: float) -> np.ndarray:
    """True for points at least `margin` away from the body (geometric test)."""
    if surf is None:
        return np.ones(len(pts), bool)
    x, y = pts[:, 0], pts[:, 1]
    p = surf.params
    if surf.kind == "cylinder":
        cx, cy = p["center"]
        return np.hypot(x - cx, y - cy) > p["radius"] + margin
    if surf.kind == "ellipse":
        cx, cy = p["center"]
        c, s = np.cos(p["rotation"]), np.sin(p["rotation"])
        xr = c * (x - cx) + s * (y - cy)
        yr = -s * (x - cx) + c * (y - cy)
        return (xr / (p["a"] + margin)) ** 2 + (yr / (p["b"] + margin)) ** 2 > 1.0
    if surf.kind == "plate":
        a = np.deg2rad(p["alpha_deg"])
        cx, cy = p["center"]
        h = 0.5 * p["chord"]
        tx, ty = np.cos(a), -np.sin(a)
        along = (x - cx) * tx + (y - cy) * ty
        along = np.clip(along, -h, h)
        dxp = x - (cx + along * tx)
        dyp = y - (cy + along * ty)
        return np.hypot(dxp, dyp) >= margin
    raise ValueError(surf.kind)


# ----------------------------------------------------------------------------
# problem specification consumed by both sides
# ----------------------------------------------------------------------------

@dataclass
class Case:
    """One solve: grid, vortices, body, freestream and constraint choice."""
    name: str
    n: int
    dx: float
    X: np.ndarray
    Y: np.ndarray
    G: np.ndarray
    surface: Surface | None = None
    u_inf: float = 0.0
    v_inf: float = 0.0
    ub: float = 0.0
    vb: float = 0.0
    omega: float = 0.0
    mode: str = "none"                 # none | circulation | kutta | shed
    gamma_b: float = 0.0
    edges: tuple = ()
    znew: tuple = ()
    gamma_w: float | None = None
    fbounds: tuple = ()        # shed: ((fmin, fmax), ...) per edge on f~; () = Kutta
    extra: dict = field(default_factory=dict)

    @property
    def x0(self) -> float:
        return -(self.n - 1) * self.dx / 2.0

    @property
    def nv(self) -> int:
        return len(self.X)


def _uniform_cloud(rng, nv, half, surf, margin):
    def draw(k):
        return rng.uniform(-half, half, size=(k, 2))
    return _accept_first(rng, nv, draw, lambda p: outside_surface(surf, p, margin))


def config1(seed: int = 1) -> Case:
    """Cylinder a = 0.5, Ns = 100, 128^2 grid dx = 0.02, 200 vortices in
    [-1.2, 1.2]^2 outside the body, Gamma ~ N(0, 0.01^2), U_inf = (1, 0),
    prescribed bound circulation -sum Gamma (Kelvin)."""
    rng = np.random.default_rng(seed)
    n, dx = 128, 0.02
    surf = cylinder(0.5, 100)
    pts = _uniform_cloud(rng, 200, 1.2, surf, 0.0)
    G = rng.normal(0.0, 0.01, size=200)
    X, Y, G = f32(pts[:, 0]), f32(pts[:, 1]), f32(G)
    return Case("C1 cylinder 128^2", n, dx, X, Y, G, surf, u_inf=1.0, mode="circulation",
                gamma_b=float(-np.sum(G)))


def plate_new_vortices(surf: Surface, offset: float):
    """New-vortex positions just beyond each plate edge along the chord."""
    a = np.deg2rad(surf.params["alpha_deg"])
    t = np.array([np.cos(a), -np.sin(a)])
    cx, cy = surf.params["center"]
    h = 0.5 * surf.params["chord"]
    le = np.array([cx, cy]) - h * t
    te = np.array([cx, cy]) + h * t
    z_le = f32(le - offset * t)
    z_te = f32(te + offset * t)
    return (tuple(z_le), tuple(z_te))


def config2(seed: int = 2, nv: int = 10000) -> Case:
    """Flat plate c = 1 at 20 deg, Ns = 256, 512^2 grid dx = 0.005, 1e4 vortices
    from a Gaussian blob (sigma 0.1) centred 0.25 downstream of the trailing
    edge, Gamma ~ N(0, 1e-3^2); Kutta condition at both edges with a new
    vortex 0.02 beyond each edge along the chord."""
    rng = np.random.default_rng(seed)
    n, dx = 512, 0.005
    surf = flat_plate(1.0, 20.0, 256)
    a = np.deg2rad(20.0)
    te = 0.5 * np.array([np.cos(a), -np.sin(a)])
    c = te + np.array([0.25, 0.0])

    def draw(k):
        return c[None, :] + 0.1 * rng.standard_normal(size=(k, 2))

    def keep(p):
        inside = (np.abs(p[:, 0]) <= 1.2) & (np.abs(p[:, 1]) <= 1.2)
        return inside & outside_surface(surf, p, 2.0 * dx)

    pts = _accept_first(rng, nv, draw, keep)
    G = rng.normal(0.0, 1e-3, size=nv)
    X, Y, G = f32(pts[:, 0]), f32(pts[:, 1]), f32(G)
    return Case("C2 plate 512^2 Kutta x2", n, dx, X, Y, G, surf, u_inf=1.0, mode="shed",
                edges=surf.edges, znew=plate_new_vortices(surf, 0.02))


def config3(seed: int = 3, nv: int = 100000) -> Case:
    """Ellipse a = 0.5, b = 0.1, Ns = 512 (arc-equispaced), 1024^2 grid
    dx = 2.5e-3, 1e5 vortices uniform in [-1.1, 1.1]^2 outside the ellipse
    inflated by 2 dx, Gamma ~ U[-1e-3, 1e-3]; U_inf = (1, 0); prescribed
    bound circulation -sum Gamma; time step dt = 1.25e-3 for RK2 stepping."""
    rng = np.random.default_rng(seed)
    n, dx = 1024, 2.5e-3
    surf = ellipse(0.5, 0.1, 512)
    pts = _uniform_cloud(rng, nv, 1.1, surf, 2.0 * dx)
    G = rng.uniform(-1e-3, 1e-3, size=nv)
    X, Y, G = f32(pts[:, 0]), f32(pts[:, 1]), f32(G)
    return Case("C3 ellipse 1024^2", n, dx, X, Y, G, surf, u_inf=1.0, mode="circulation",
                gamma_b=float(-np.sum(G)), extra={"dt": 1.25e-3, "steps": 100})


def config4(seed: int = 4, nprob: int = 64) -> list[Case]:
    """Independent problems of uneven size: n ~ {128, 256, 512, 1024},
    dx = 2.56/n, ellipse a = 0.5 with aspect ~ U[0.1, 1] and rotation
    ~ U[0, pi), Ns log-uniform in [64, 512] clamped to dS/dx in [1.5, 4],
    Nv = round(10^U[3, 5]) uniform in [-1.2, 1.2]^2 outside the body + 2 dx,
    Gamma ~ U[-1e-3, 1e-3]; prescribed circulation -sum Gamma; U_inf = (1, 0)."""
    rng = np.random.default_rng(seed)
    cases = []
    for k in range(nprob):
        n = int(rng.choice([128, 256, 512, 1024]))
        dx = 2.56 / n
        aspect = rng.uniform(0.1, 1.0)
        rot = rng.uniform(0.0, np.pi)
        ns = int(round(np.exp(rng.uniform(np.log(64), np.log(512)))))
        a, b = 0.5, 0.5 * aspect
        perim = 4.0 * a * special.ellipe(1.0 - aspect ** 2)
        lo = int(np.ceil(perim / (4.0 * dx)))
        hi = int(np.floor(perim / (1.5 * dx)))
        ns = int(np.clip(ns, max(64, lo), min(512, hi)))
        surf = ellipse(a, b, ns, rot)
        nv = int(round(10 ** rng.uniform(3, 5)))
        pts = _uniform_cloud(rng, nv, 1.2, surf, 2.0 * dx)
        G = rng.uniform(-1e-3, 1e-3, size=nv)
        X, Y, G = f32(pts[:, 0]), f32(pts[:, 1]), f32(G)
        cases.append(Case(f"C4[{k}] ellipse {n}^2", n, dx, X, Y, G, surf, u_inf=1.0,
                          mode="circulation", gamma_b=float(-np.sum(G))))
    return cases


def config5_request(rng, nv_max: int = 1000000) -> Case:
    """One serving request: n ~ {256, 512, 1024, 2048}, dx = 2.56/n; half
    cylinders (a = 0.5, prescribed circulation with Kelvin), half plates
    (c = 1, alpha in {0, 5, ..., 30} deg, Kutta at both edges with new
    vortices); Nv = round(10^U[3, log10 nv_max]); Gamma ~ N(0, 1e-3^2)."""
    n = int(rng.choice([256, 512, 1024, 2048]))
    dx = 2.56 / n
    if rng.uniform() < 0.5:
        surf = cylinder(0.5, int(min(1024, round(np.pi * 0.5 / dx))))
        mode = "circulation"
    else:
        alpha = float(rng.choice(np.arange(0, 35, 5)))
        surf = flat_plate(1.0, alpha, int(min(1024, round(1.0 / (2.0 * dx)))))
        mode = "shed"
    nv = int(round(10 ** rng.uniform(3, np.log10(nv_max))))
    pts = _uniform_cloud(rng, nv, 1.2, surf, 2.0 * dx)
    G = rng.normal(0.0, 1e-3, size=nv)
    X, Y, G = f32(pts[:, 0]), f32(pts[:, 1]), f32(G)
    c = Case(f"C5 {surf.kind} {n}^2", n, dx, X, Y, G, surf, u_inf=1.0, mode=mode)
    if mode == "circulation":
        c.gamma_b = float(-np.sum(G))
    else:
        c.edges = surf.edges
        c.znew = plate_new_vortices(surf, 4.0 * dx)
    return c


def naca0012_demo(n: int = 1024) -> Case:
    """The paper's airfoil demonstration: NACA 0012, chord 1, at 20 deg in a
    unit uniform flow started impulsively, dx/c = 0.01, dS/dx = 1.5, shedding
    at the trailing edge (Kutta) with dt U/c = 0.075 (extra["dt"]); no vortex
    at the start.  The section sits 3.5 chords upstream of the window's
    centre so that 3 convective times of wake stay inside the 1024^2 window.
    The first release is one step's travel downstream of the trailing edge."""
    dx, chord, alpha = 0.01, 1.0, 20.0
    per = naca4_symmetric(0.12, chord, alpha, 16).params["perimeter"]
    surf = naca4_symmetric(0.12, chord, alpha, int(round(per / (1.5 * dx))), center=(-3.5, 0.0))
    dt = 0.075
    te = (float(surf.xs[0]), float(surf.ys[0]))
    z = np.zeros(0)
    case = Case(f"NACA 0012 at 20 deg, {n}^2", n, dx, z, z, z, surf, u_inf=1.0, mode="shed")
    case.edges = (0,)
    case.znew = ((te[0] + dt, te[1]),)
    case.extra["dt"] = dt
    return case


def random_case(seed: int, n: int, dx: float, nv: int, surface: str | None = "cylinder",
                mode: str | None = None, ns: int | None = None) -> Case:
    """Small mixed case for parity tests (tiles plus a ragged tail)."""
    rng = np.random.default_rng(seed)
    half = (n - 1) * dx / 2.0 - 4.0 * dx
    size = 0.6 * half
    surf = None
    if surface == "cylinder":
        ns = ns or max(8, int(round(2 * np.pi * 0.5 * size / (1.6 * dx))))
        surf = cylinder(0.5 * size, ns)
        mode = mode or "circulation"
    elif surface == "plate":
        ns = ns or max(8, int(round(size / (1.5 * dx))))
        surf = flat_plate(size, 25.0, ns)
        mode = mode or "kutta"
    elif surface == "ellipse":
        ns = ns or max(8, int(round(2.2 * size / (1.6 * dx))))
        surf = ellipse(0.5 * size, 0.25 * size, ns, 0.3)
        mode = mode or "circulation"
    else:
        mode = "none"
    pts = _uniform_cloud(rng, nv, half, surf, 2.0 * dx)
    G = rng.normal(0.0, 1e-2, size=nv)
    X, Y, G = f32(pts[:, 0]), f32(pts[:, 1]), f32(G)
    c = Case(f"random {surface} n={n}", n, dx, X, Y, G, surf, u_inf=1.0, v_inf=0.25,
             ub=0.1, vb=-0.05, omega=0.3 if surface else 0.0, mode=mode)
    if mode == "circulation":
        c.gamma_b = float(-np.sum(G)) + 0.05
    elif mode == "kutta":
        c.edges = (surf.edges[1],)
    elif mode == "shed":
        c.edges = surf.edges
        c.znew = plate_new_vortices(surf, 4.0 * dx)
    return c


# ----------------------------------------------------------------------------
# several bodies (Sec. 2.7)
# ----------------------------------------------------------------------------

@dataclass
class MultiCase:
    """Several bodies in one window: surfaces in order, one entry of `parts`
    per surface (mode and its values, motion), new-vortex positions for the
    edges of the shedding parts in the bodies' edge order."""
    name: str
    n: int
    dx: float
    X: np.ndarray
    Y: np.ndarray
    G: np.ndarray
    surfaces: list
    parts: list
    znew: tuple = ()
    fbounds: tuple = ()
    u_inf: float = 0.0
    v_inf: float = 0.0

    @property
    def nv(self) -> int:
        return len(self.X)

    @property
    def xs(self):
        return np.concatenate([s.xs for s in self.surfaces])

    @property
    def ys(self):
        return np.concatenate([s.ys for s in self.surfaces])

    @property
    def ds(self):
        return np.concatenate([s.ds for s in self.surfaces])

    @property
    def part(self):
        return np.concatenate([np.full(s.ns, j, np.int32) for j, s in enumerate(self.surfaces)])

    @property
    def edges(self):
        out, off = [], 0
        for s in self.surfaces:
            out += [off + e for e in s.edges]
            off += s.ns
        return tuple(out)

    def part_edges(self, j):
        off = sum(s.ns for s in self.surfaces[:j])
        return tuple(off + e for e in self.surfaces[j].edges)


def _cloud_outside(rng, nv, half, surfaces, margin):
    def keep(p):
        ok = np.ones(len(p), bool)
        for s in surfaces:
            ok &= outside_surface(s, p, margin)
        return ok
    return _accept_first(rng, nv, lambda k: rng.uniform(-half, half, size=(k, 2)), keep)


def two_plates_case(seed: int = 16, n: int = 256, chord: float = 1.0, nv: int = 2000) -> MultiCase:
    """Two plates of chord c at 60 deg, one above the other c/2 apart (the
    arrangement of Fig. 16), dx = 2.4c/n (dS/dx = 2), uniform flow (1, 0),
    Kutta at both edges of both plates with a new vortex 2dx beyond each;
    vortices uniform in the window outside the plates, Gamma ~ N(0, 1e-3^2)."""
    rng = np.random.default_rng(seed)
    dx = 2.4 * chord / n
    ns = int(round(chord / (2.0 * dx)))
    top = flat_plate(chord, 60.0, ns, center=(0.0, 0.25 * chord))
    bot = flat_plate(chord, 60.0, ns, center=(0.0, -0.25 * chord))
    half = (n - 1) * dx / 2.0 - 4.0 * dx
    pts = _cloud_outside(rng, nv, half, [top, bot], 2.0 * dx)
    G = rng.normal(0.0, 1e-3, size=nv)
    znew = plate_new_vortices(top, 2.0 * dx) + plate_new_vortices(bot, 2.0 * dx)
    parts = [{"mode": "shed", "gamma_w": 0.0}, {"mode": "shed", "gamma_w": 0.0}]
    return MultiCase(f"two plates {n}^2", n, dx, f32(pts[:, 0]), f32(pts[:, 1]), f32(G),
                     [top, bot], parts, znew, (), u_inf=1.0)


def mixed_bodies_case(seed: int = 17, n: int = 128, nv: int = 400) -> MultiCase:
    """A moving cylinder with a prescribed circulation, a plate held by a
    steady Kutta condition at its trailing edge, and a shedding plate (both
    edges), in a uniform flow with a vertical component."""
    rng = np.random.default_rng(seed)
    dx = 2.0 / n
    cyl = cylinder(0.22, int(round(2 * np.pi * 0.22 / (1.6 * dx))), center=(-0.45, 0.35))
    p1 = flat_plate(0.5, 15.0, int(round(0.5 / (1.5 * dx))), center=(0.35, 0.4))
    p1.edges = (p1.edges[1],)      # its trailing edge only
    p2 = flat_plate(0.6, 30.0, int(round(0.6 / (1.5 * dx))), center=(0.0, -0.4))
    half = (n - 1) * dx / 2.0 - 4.0 * dx
    pts = _cloud_outside(rng, nv, half, [cyl, p1, p2], 2.0 * dx)
    G = rng.normal(0.0, 1e-2, size=nv)
    parts = [{"mode": "circulation", "gamma_b": 0.15, "ub": 0.1, "vb": -0.05, "omega": 0.3},
             {"mode": "kutta"},
             {"mode": "shed", "gamma_w": 0.02, "vb": 0.05}]
    return MultiCase(f"mixed bodies {n}^2", n, dx, f32(pts[:, 0]), f32(pts[:, 1]), f32(G),
                     [cyl, p1, p2], parts, plate_new_vortices(p2, 4.0 * dx), (),
                     u_inf=1.0, v_inf=0.2)
