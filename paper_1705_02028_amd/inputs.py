"""Seeded synthetic inputs: triangular meshes and initial states.

The meshes and initial conditions are shaped like the test problems of the
paper (Section 5: Sod tube, two-dimensional Riemann problem, Kelvin-Helmholtz
instability; Table 1's hydrostatic box) and like the workloads this library
is measured on. This module holds none of the residual-distribution
arithmetic: it only lays out vertices and triangles and writes primitive
states as conserved variables (the ideal-gas relation of Section 3). Both
the CPU oracle and the GPU library consume the arrays it returns.

Mesh conventions
----------------
``N`` lattice points per side of the unit square, spacing ``h = 1/(N-1)``.
A periodic axis identifies the last lattice line with the first, so it has
``N-1`` distinct vertex columns; a bounded axis has ``N``. Vertex ``(i, j)``
has id ``i + j * nx`` (j-major). Cell ``(i, j)`` with corners
``a=(i,j), b=(i+1,j), c=(i+1,j+1), d=(i,j+1)`` is cut along ``a-c``
(triangles ``[a,b,c]`` and ``[a,c,d]``) or, in the random-diagonal variant,
along ``b-d`` (``[a,b,d]`` and ``[b,c,d]``). Every triangle is
counter-clockwise once periodic images are unwrapped to the minimum image of
its first corner. With ``N = 64`` and both axes periodic this gives 3,969
vertices and 7,938 triangles.

Boundary kinds for a bounded axis: ``"ghost"`` (vertices on those sides keep
their initial state: the non-reflecting/inflow boundary of Section 3.5) and
``"wall"`` (reflecting wall edges, listed with the domain on their left).
Corner vertices become ghosts when either adjacent side is a ghost side.
"""
from __future__ import annotations

import numpy as np

GAMMA = 1.4


# ---------------------------------------------------------------- meshes ----

def _morton_key(i: np.ndarray, j: np.ndarray) -> np.ndarray:
    key = np.zeros(i.shape, dtype=np.uint64)
    ii = i.astype(np.uint64)
    jj = j.astype(np.uint64)
    for b in range(21):
        key |= ((ii >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        key |= ((jj >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
    return key


def split_square(N: int, periodic=(True, True), bc=("ghost", "ghost"),
                 diagonal: str = "ne", seed: int = 0, jitter: float = 0.0,
                 renumber: str | None = None, rotate_corners: bool = False,
                 origin=(0.0, 0.0), length: float = 1.0, Ny: int | None = None,
                 ly: float | None = None) -> dict:
    """Uniform split-square triangulation of ``[0, length]^2``.

    ``periodic`` and ``bc`` are (x-axis, y-axis) pairs; ``bc`` only matters
    for a bounded axis. ``diagonal`` is ``"ne"`` (all cells cut a-c) or
    ``"random"`` (seeded choice per cell, vertex degree 4..8). ``jitter``
    moves interior vertices by up to ``jitter*h`` per coordinate.
    ``renumber`` is None, ``"morton"`` or ``"random"`` (vertices and
    triangles). ``rotate_corners`` cyclically rotates each triangle's corner
    list by a seeded amount (orientation is kept).

    ``Ny`` and ``ly`` give a rectangle with its own lattice count and
    height along y (defaults: ``N`` and ``length``).

    Returns a dict with ``x, y`` (float64 [nv]), ``tri`` (int32 [nt, 3]),
    ``px, py`` (periods, 0 when bounded), ``ghost`` (uint8 [nv]),
    ``wall`` (int32 [nw, 2]), ``nv, nt``, ``N``, ``h``.
    """
    Ny = N if Ny is None else int(Ny)
    ly = length if ly is None else float(ly)
    perx, pery = bool(periodic[0]), bool(periodic[1])
    # a periodic axis needs 3 distinct vertex lines so minimum images are unique
    if N < (4 if perx else 2) or Ny < (4 if pery else 2):
        raise ValueError("too few lattice points per side")
    rng = np.random.Generator(np.random.PCG64(seed))
    h = length / (N - 1)
    hy = ly / (Ny - 1)
    nxv = N - 1 if perx else N
    nyv = Ny - 1 if pery else Ny
    nv = nxv * nyv
    ii, jj = np.meshgrid(np.arange(nxv), np.arange(nyv), indexing="xy")
    ii = ii.ravel()
    jj = jj.ravel()
    x = origin[0] + ii * h
    y = origin[1] + jj * hy

    def vid(i, j):
        return (i % nxv if perx else i) + (j % nyv if pery else j) * nxv

    ci, cj = np.meshgrid(np.arange(N - 1), np.arange(Ny - 1), indexing="xy")
    ci = ci.ravel()
    cj = cj.ravel()
    a = vid(ci, cj)
    b = vid(ci + 1, cj)
    c = vid(ci + 1, cj + 1)
    d = vid(ci, cj + 1)
    if diagonal == "ne":
        flip = np.zeros(ci.shape, dtype=bool)
    elif diagonal == "random":
        flip = rng.integers(0, 2, size=ci.shape).astype(bool)
    else:
        raise ValueError(diagonal)
    t0 = np.where(flip[:, None], np.stack([a, b, d], 1), np.stack([a, b, c], 1))
    t1 = np.where(flip[:, None], np.stack([b, c, d], 1), np.stack([a, c, d], 1))
    tri = np.stack([t0, t1], 1).reshape(-1, 3).astype(np.int64)
    cell_of_tri = np.repeat(np.arange(ci.size), 2)

    ghost = np.zeros(nv, dtype=np.uint8)
    walls = []
    bcx, bcy = bc
    if not perx:
        side = (ii == 0) | (ii == nxv - 1)
        if bcx == "ghost":
            ghost[side] = 1
    if not pery:
        side = (jj == 0) | (jj == nyv - 1)
        if bcy == "ghost":
            ghost[side] = 1
    if not pery and bcy == "wall":
        for i in range(N - 1):
            walls.append((vid(i, 0), vid(i + 1, 0)))              # bottom, +x
        for i in range(N - 1):
            walls.append((vid(i + 1, Ny - 1), vid(i, Ny - 1)))    # top, -x
    if not perx and bcx == "wall":
        for j in range(Ny - 1):
            walls.append((vid(N - 1, j), vid(N - 1, j + 1)))      # right, +y
        for j in range(Ny - 1):
            walls.append((vid(0, j + 1), vid(0, j)))              # left, -y
    wall = np.array(walls, dtype=np.int64).reshape(-1, 2)

    if jitter > 0.0:
        interior = np.ones(nv, dtype=bool)
        if not perx:
            interior &= (ii > 0) & (ii < nxv - 1)
        if not pery:
            interior &= (jj > 0) & (jj < nyv - 1)
        dx = rng.uniform(-1.0, 1.0, size=nv) * jitter * h
        dy = rng.uniform(-1.0, 1.0, size=nv) * jitter * hy
        x = np.where(interior, x + dx, x)
        y = np.where(interior, y + dy, y)

    if rotate_corners:
        r = rng.integers(0, 3, size=tri.shape[0])
        idx = (np.arange(3)[None, :] + r[:, None]) % 3
        tri = np.take_along_axis(tri, idx, axis=1)

    if renumber is not None:
        if renumber == "morton":
            vperm = np.argsort(_morton_key(ii, jj), kind="stable")
            tkey = _morton_key(ci[cell_of_tri], cj[cell_of_tri])
            tperm = np.lexsort((np.arange(tri.shape[0]) % 2, tkey))
        elif renumber == "random":
            vperm = rng.permutation(nv)
            tperm = rng.permutation(tri.shape[0])
        else:
            raise ValueError(renumber)
        inv = np.empty(nv, dtype=np.int64)
        inv[vperm] = np.arange(nv)
        x = x[vperm]
        y = y[vperm]
        ghost = ghost[vperm]
        tri = inv[tri][tperm]
        wall = inv[wall] if wall.size else wall

    return dict(
        x=np.ascontiguousarray(x, dtype=np.float64),
        y=np.ascontiguousarray(y, dtype=np.float64),
        tri=np.ascontiguousarray(tri, dtype=np.int32),
        px=length if perx else 0.0,
        py=ly if pery else 0.0,
        ghost=np.ascontiguousarray(ghost, dtype=np.uint8),
        wall=np.ascontiguousarray(wall, dtype=np.int32).reshape(-1, 2),
        nv=int(nv), nt=int(tri.shape[0]), N=int(N), Ny=int(Ny), h=float(h),
        hy=float(hy),
        gamma=GAMMA,
    )


def concat_meshes(meshes: list[dict], spacing: float = 2.0) -> dict:
    """Disjoint union of meshes (vertex and triangle ids offset in order).

    Each mesh is shifted by ``spacing * k`` in x so coordinates stay
    distinct; periodicity is not supported here (batched meshes are
    bounded). Offsets are returned as ``voff`` / ``toff`` ([n+1]).
    """
    xs, ys, tris, gh, walls = [], [], [], [], []
    voff = [0]
    toff = [0]
    for k, m in enumerate(meshes):
        if m["px"] or m["py"]:
            raise ValueError("concat_meshes takes bounded meshes")
        xs.append(m["x"] + spacing * k)
        ys.append(m["y"])
        tris.append(m["tri"].astype(np.int64) + voff[-1])
        gh.append(m["ghost"])
        if m["wall"].size:
            walls.append(m["wall"].astype(np.int64) + voff[-1])
        voff.append(voff[-1] + m["nv"])
        toff.append(toff[-1] + m["nt"])
    wall = np.concatenate(walls) if walls else np.zeros((0, 2), np.int64)
    return dict(
        x=np.concatenate(xs), y=np.concatenate(ys),
        tri=np.concatenate(tris).astype(np.int32),
        px=0.0, py=0.0, ghost=np.concatenate(gh),
        wall=wall.astype(np.int32).reshape(-1, 2),
        nv=int(voff[-1]), nt=int(toff[-1]),
        voff=np.array(voff, np.int64), toff=np.array(toff, np.int64),
        gamma=meshes[0]["gamma"],
    )


# ------------------------------------------------------- initial states ----

def prim_to_cons(rho, u, v, p, gamma=GAMMA) -> np.ndarray:
    """Conserved state (rho, rho u, rho v, e) as a [4, nv] float64 array,
    with e = rho (u^2 + v^2) / 2 + p / (gamma - 1) (Section 3)."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.broadcast_to(np.asarray(u, dtype=np.float64), rho.shape)
    v = np.broadcast_to(np.asarray(v, dtype=np.float64), rho.shape)
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    e = 0.5 * rho * (u * u + v * v) + p / (gamma - 1.0)
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, e]))


def ic_uniform(mesh, rho=1.0, u=0.0, v=0.0, p=1.0):
    """Constant state; with u = v = 0 this is Table 1's hydrostatic box."""
    n = mesh["nv"]
    return prim_to_cons(np.full(n, rho), u, v, p, mesh["gamma"])


def ic_advected_sine(mesh):
    """rho = 1 + 0.1 sin(2 pi x), velocity (1, 0.5), p = 1 (periodic box)."""
    rho = 1.0 + 0.1 * np.sin(2.0 * np.pi * mesh["x"])
    return prim_to_cons(rho, 1.0, 0.5, 1.0, mesh["gamma"])


def ic_sod(mesh, x0=0.5):
    """Sod tube (Section 5.1.2): (rho, p) = (1, 1) for x < x0, (0.125, 0.1)
    otherwise, at rest. x == x0 takes the right state."""
    left = mesh["x"] < x0
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    return prim_to_cons(rho, 0.0, 0.0, p, mesh["gamma"])


def ic_kelvin_helmholtz(mesh, seed=0, amp=0.01, rho_in=2.0, rho_out=1.0,
                        u0=0.5, p=2.5):
    """Shear layer (Section 5.2.5 shape): rho = 2, u = +0.5 for
    |y - 0.5| < 0.25, rho = 1, u = -0.5 elsewhere, p = 2.5, and a seeded
    transverse velocity amp * U[-1, 1] per vertex."""
    rng = np.random.Generator(np.random.PCG64(seed))
    band = np.abs(mesh["y"] - 0.5) < 0.25
    rho = np.where(band, rho_in, rho_out)
    u = np.where(band, u0, -u0)
    v = amp * rng.uniform(-1.0, 1.0, size=mesh["nv"])
    return prim_to_cons(rho, u, v, p, mesh["gamma"])


def quadrant_states(seed, rho=(0.1, 2.0), p=(0.1, 2.0), vmax=1.0):
    """Four seeded primitive states (rho, u, v, p): rho ~ U[rho], p ~ U[p],
    velocity uniform in the disc of radius ``vmax``; ordered as quadrants
    1..4 of the two-dimensional Riemann problem (Section 5.2.4)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(4):
        r_ = rng.uniform(*rho)
        p_ = rng.uniform(*p)
        r = vmax * np.sqrt(rng.uniform(0.0, 1.0))
        th = rng.uniform(0.0, 2.0 * np.pi)
        out.append((r_, r * np.cos(th), r * np.sin(th), p_))
    return out


# Draw of the batched four-quadrant problems: rho, p ~ U[0.1, 2] and
# velocity in the unit disc per quadrant. The B scheme is not positivity
# preserving, and some of these problems go non-physical within 200 steps.
BATCH_QUADRANTS = dict(rho=(0.1, 2.0), p=(0.1, 2.0), vmax=1.0)
# A narrower draw in which no adjacent pair comes near vacuum
# (|u_L - u_R| <= 1 while 2 (c_L + c_R) / (gamma - 1) >= 5.9), for long runs
# that must stay physical.
NARROW_QUADRANTS = dict(rho=(0.5, 2.0), p=(0.5, 2.0), vmax=0.5)


def ic_quadrants(mesh, states, xc=0.5, yc=0.5, x0=0.0):
    """Four constant states split at (xc, yc) with the convention
    1: x > xc, y > yc; 2: x <= xc, y > yc; 3: x <= xc, y <= yc;
    4: x > xc, y <= yc. ``x0`` is the mesh's x origin."""
    x = mesh["x"] - x0
    y = mesh["y"]
    q = np.where(y > yc, np.where(x > xc, 0, 1), np.where(x > xc, 3, 2))
    s = np.array(states, dtype=np.float64)
    return prim_to_cons(s[q, 0], s[q, 1], s[q, 2], s[q, 3], mesh["gamma"])


def ic_fourier_density(mesh, seed=0, modes=10, amp=0.05, u=0.5, v=0.3, p=1.0):
    """rho = 1 + amp * f / max|f| with f a sum of ``modes`` seeded Fourier
    modes cos(2 pi k.x + phase), k in Z^2 with 1 <= |k|_inf <= 4,
    amplitudes U[0.5, 1]; uniform velocity and pressure."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f = np.zeros(mesh["nv"])
    for _ in range(modes):
        while True:
            k = rng.integers(-4, 5, size=2)
            if np.max(np.abs(k)) >= 1:
                break
        a = rng.uniform(0.5, 1.0)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        f += a * np.cos(2.0 * np.pi * (k[0] * mesh["x"] + k[1] * mesh["y"]) + ph)
    rho = 1.0 + amp * f / np.max(np.abs(f))
    return prim_to_cons(rho, u, v, p, mesh["gamma"])


def random_smooth_state(mesh, seed=0, amp=0.1, u=0.3, v=-0.2, p=1.0):
    """A smooth seeded state with all four fields varying (used for
    per-step parity away from the named problems)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y = mesh["x"], mesh["y"]
    fields = []
    for _ in range(4):
        k = rng.integers(1, 4, size=2)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        fields.append(np.sin(2.0 * np.pi * (k[0] * x + k[1] * y) + ph))
    rho = 1.0 + amp * fields[0]
    return prim_to_cons(rho, u + amp * fields[1], v + amp * fields[2],
                        p * (1.0 + amp * fields[3]), mesh["gamma"])


def ic_sound_wave(mesh, amp=1e-4):
    """Right-moving linear sound wave of Section 5.1.1: rho = 1 + amp sin(2 pi x),
    u = c (rho - 1), p = 1/gamma + c^2 (rho - 1), c = 1, v = 0 (wavelength 1)."""
    g = mesh["gamma"]
    d = amp * np.sin(2.0 * np.pi * mesh["x"])
    return prim_to_cons(1.0 + d, d, 0.0, 1.0 / g + d, g)


def ic_isentropic_vortex(mesh, xc=5.0, yc=5.0, beta=5.0, boost=0.0):
    """Isentropic vortex of Section 5.2.3 (p = rho^gamma far away equal to
    1): v = Omega(r) (-(y - yc), x - xc) + (boost, 0), Omega = beta
    exp((1 - r^2)/2) / (2 pi), T = p / rho = 1 - (gamma - 1)/gamma beta^2
    exp(1 - r^2) / (8 pi^2), rho = T^(1/(gamma - 1)), p = rho^gamma."""
    g = mesh["gamma"]
    dx, dy = mesh["x"] - xc, mesh["y"] - yc
    r2 = dx * dx + dy * dy
    om = beta * np.exp(0.5 * (1.0 - r2)) / (2.0 * np.pi)
    T = 1.0 - (g - 1.0) / g * beta * beta * np.exp(1.0 - r2) / (8.0 * np.pi ** 2)
    rho = T ** (1.0 / (g - 1.0))
    return prim_to_cons(rho, -om * dy + boost, om * dx, rho ** g, g)


def _smooth_step(t):
    """g(t) of Section 5.2.5: 0 for t <= 0, 1 for t >= 1, smooth between."""
    t = np.asarray(t, dtype=np.float64)
    f = lambda s: np.where(s > 0.0, np.exp(-1.0 / np.where(s > 0.0, s, 1.0)), 0.0)  # noqa: E731
    return f(t) / (f(t) + f(1.0 - t))


def ic_kh_smooth(mesh, d=0.25, u0=0.5, rho_l=1.0, rho_h=2.0, p=2.5, amp=1e-3):
    """Smoothed Kelvin-Helmholtz shear layer of Section 5.2.5 (transition
    width d) with a transverse velocity amp sin(2 pi x) (the k_x = 2 pi
    mode; the paper seeds its eigenvector, this seeds the plain sine)."""
    y = mesh["y"]
    prof = _smooth_step(0.5 + (y - 0.25) / d) * _smooth_step(0.5 - (y - 0.75) / d)
    rho = (rho_h - rho_l) * prof + rho_l
    u = 2.0 * u0 * prof - u0
    v = amp * np.sin(2.0 * np.pi * mesh["x"])
    return prim_to_cons(rho, u, v, p, mesh["gamma"])


# ------------------------------------------------------------ workloads ----

def batch_sides(seed=0, n=256, lo=32, hi=512):
    """Side lengths N ~ U{lo..hi} of the batched four-quadrant meshes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(s) for s in rng.integers(lo, hi + 1, size=n)]


def batch_problem(seed=0, n=256, lo=32, hi=512, sides=None, draw=None):
    """Independent four-quadrant Riemann problems of uneven size, ghost
    boundaries on all sides; quadrant states from ``draw`` (default
    BATCH_QUADRANTS). Returns (meshes, states) lists."""
    if sides is None:
        sides = batch_sides(seed, n, lo, hi)
    draw = BATCH_QUADRANTS if draw is None else draw
    meshes, states = [], []
    for k, N in enumerate(sides):
        m = split_square(N, periodic=(False, False), bc=("ghost", "ghost"))
        meshes.append(m)
        states.append(ic_quadrants(m, quadrant_states(seed * 100003 + k, **draw)))
    return meshes, states


# ---------------------------------------------------------------- 3D -------

def cube_tets(N: int, periodic=(True, True, True), jitter: float = 0.0, seed: int = 0,
              length: float = 1.0, renumber: str | None = None) -> dict:
    """Tetrahedral mesh of the box [0, length]^3: N cells per side, each cell
    split into the six tetrahedra around its main diagonal (Kuhn's
    subdivision, conforming across cells); every tetrahedron positively
    oriented. ``periodic`` per axis (periodic axes have N vertex lines, the
    others N + 1). ``jitter`` moves every vertex by up to jitter * h per
    coordinate (vertices on a bounded face stay on it). ``renumber`` None or
    "morton" (vertices and tetrahedra along a Z-order curve).

    Returns a dict with ``x, y, z`` (float64 [nv]), ``tet`` (int32 [nt, 4]),
    ``px, py, pz`` (periods, 0 when bounded), ``nv, nt``, ``N``, ``h``,
    ``gamma``."""
    per = [bool(p) for p in periodic]
    if N < (3 if any(per) else 1):
        raise ValueError("too few cells per side")
    h = length / N
    nl = [N if p else N + 1 for p in per]
    ii, jj, kk = np.meshgrid(np.arange(nl[0]), np.arange(nl[1]), np.arange(nl[2]), indexing="ij")
    ii, jj, kk = ii.ravel(order="F"), jj.ravel(order="F"), kk.ravel(order="F")
    x, y, z = ii * h, jj * h, kk * h
    if jitter > 0:
        rng = np.random.Generator(np.random.PCG64(seed))
        d = (rng.random((3, len(x))) * 2.0 - 1.0) * jitter * h
        for a, (c, n_, p) in enumerate(zip((ii, jj, kk), nl, per)):
            if not p:  # keep bounded faces flat
                d[a][(c == 0) | (c == n_ - 1)] = 0.0
        x, y, z = x + d[0], y + d[1], z + d[2]

    def vid(i, j, k):
        return (i % nl[0]) + nl[0] * ((j % nl[1]) + nl[1] * (k % nl[2]))

    ci, cj, ck = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    ci, cj, ck = ci.ravel(order="F"), cj.ravel(order="F"), ck.ravel(order="F")
    tets = []
    for perm, sign in (((0, 1, 2), 1), ((1, 2, 0), 1), ((2, 0, 1), 1), ((0, 2, 1), -1), ((2, 1, 0), -1),
                       ((1, 0, 2), -1)):
        path = [np.zeros(3, dtype=np.int64)]
        for a in perm:
            step = path[-1].copy()
            step[a] += 1
            path.append(step)
        corners = [vid(ci + s[0], cj + s[1], ck + s[2]) for s in path]
        if sign < 0:  # odd permutation: swap two corners for a positive orientation
            corners[1], corners[2] = corners[2], corners[1]
        tets.append(np.stack(corners, axis=1))
    tet = np.concatenate(tets).astype(np.int32)
    mesh = {"x": x.astype(np.float64), "y": y.astype(np.float64), "z": z.astype(np.float64), "tet": tet,
            "px": length if per[0] else 0.0, "py": length if per[1] else 0.0, "pz": length if per[2] else 0.0,
            "nv": len(x), "nt": len(tet), "N": N, "h": h, "gamma": GAMMA}
    if renumber == "morton":
        def key3(i, j, k):
            out = np.zeros(len(i), dtype=np.int64)
            for b in range(21):
                out |= (((i >> b) & 1) << (3 * b)) | (((j >> b) & 1) << (3 * b + 1)) | (((k >> b) & 1) << (3 * b + 2))
            return out
        vp = np.argsort(key3(ii, jj, kk), kind="stable")
        inv = np.empty_like(vp)
        inv[vp] = np.arange(len(vp))
        for c in ("x", "y", "z"):
            mesh[c] = np.ascontiguousarray(mesh[c][vp])
        cell = np.arange(len(tet)) % len(ci)  # tetrahedra come in six blocks of all cells
        tp = np.argsort(key3(ci[cell], cj[cell], ck[cell]), kind="stable")
        mesh["tet"] = np.ascontiguousarray(inv[tet][tp]).astype(np.int32)
    elif renumber is not None:
        raise ValueError("renumber must be None or 'morton'")
    return mesh


def prim_to_cons3(rho, u, v, w, p, gamma=GAMMA) -> np.ndarray:
    """Conserved state (rho, rho u, rho v, rho w, e) as a [5, nv] float64
    array, e = rho |u|^2 / 2 + p / (gamma - 1)."""
    rho = np.asarray(rho, dtype=np.float64)
    u, v, w, p = (np.broadcast_to(np.asarray(a, dtype=np.float64), rho.shape) for a in (u, v, w, p))
    e = 0.5 * rho * (u * u + v * v + w * w) + p / (gamma - 1.0)
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, rho * w, e]))


def ic3_uniform(mesh, rho=1.0, u=0.0, v=0.0, w=0.0, p=1.0):
    return prim_to_cons3(np.full(mesh["nv"], rho), u, v, w, p, mesh["gamma"])


def ic3_random_smooth(mesh, seed=0, amp=0.1, u=0.3, v=-0.2, w=0.15, p=1.0, modes=4):
    """Seeded smooth periodic perturbations of a uniform flow (a few Fourier
    modes per field, lowest wavenumbers of the box)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = [mesh["px"] or 1.0, mesh["py"] or 1.0, mesh["pz"] or 1.0]
    X = [mesh["x"] / L[0], mesh["y"] / L[1], mesh["z"] / L[2]]

    def field():
        f = np.zeros(mesh["nv"])
        for _ in range(modes):
            k = rng.integers(-2, 3, size=3)
            ph = rng.random() * 2 * np.pi
            f += rng.normal() * np.cos(2 * np.pi * (k[0] * X[0] + k[1] * X[1] + k[2] * X[2]) + ph)
        return f / modes

    rho = 1.0 + amp * field()
    return prim_to_cons3(rho, u + amp * field(), v + amp * field(), w + amp * field(), p * (1.0 + amp * field()),
                         mesh["gamma"])


def ic3_kelvin_helmholtz(mesh, seed=0, amp=0.01, rho_in=2.0, rho_out=1.0, u_in=0.5, u_out=-0.5, p=2.5):
    """Shear layer in a periodic box: the middle half in y (1/4 < y < 3/4)
    denser and moving with u_in, the rest with u_out; seeded small random
    velocity perturbations in v and w."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ly = mesh["py"] or 1.0
    inner = (mesh["y"] > 0.25 * Ly) & (mesh["y"] < 0.75 * Ly)
    rho = np.where(inner, rho_in, rho_out)
    u = np.where(inner, u_in, u_out)
    v = amp * (rng.random(mesh["nv"]) - 0.5)
    w = amp * (rng.random(mesh["nv"]) - 0.5)
    return prim_to_cons3(rho, u, v, w, p, mesh["gamma"])
