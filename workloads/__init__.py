"""Seeded synthetic inputs for the overset grid-assembly path.

This module is shared by the tests, the benchmark and the CPU oracle's
callers. It builds grids, blank-region descriptions, rigid-motion pose
tables and field values, and nothing else: it holds none of the assembly
arithmetic (no hole test, no fringe rule, no donor search, no
interpolation). Every random number is drawn from
``numpy.random.default_rng(seed)`` in the order documented per builder.

Conventions (shared with the C-ABI library and the oracle):

* A grid is a structured block of ``(ni, nj, nk)`` nodes; node ``(i, j, k)``
  has linear index ``i + ni*(j + nj*k)`` (i fastest), as in the paper's
  local index of Sec. 2.2.6.
* Coordinates are FP64 structure-of-arrays in the grid's own (body) frame.
* ``periodic`` is a bit mask (1: i, 2: j, 4: k). A periodic direction of
  n nodes has n cells (the last wraps to node 0); otherwise n-1 cells.
* Grid 0 is the stationary background (identity pose); grids 1.. are
  overset grids moving rigidly with a pose ``(R, c)``:
  ``x_world = R @ X_body + c`` (R row-major). The paper writes the
  non-inertial frame with a rotation tensor Q (Sec. 2.1, eq. for u_q);
  here R plays the role of Q transposed.
* A pose table is an array ``[steps, ngrids, 12]`` = R (9, row-major) then c (3).
* Fields u, v, w, p are stored as one ``[4, total_nodes]`` array; grid g's
  nodes start at ``node_offset[g]`` (the paper's packed per-process vector,
  Sec. 2.2.6).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

BLANK_NONE, BLANK_CYL, BLANK_SPHERE, BLANK_ELLIPSOID, BLANK_MESH = 0, 1, 2, 3, 4
PERIODIC_I, PERIODIC_J, PERIODIC_K = 1, 2, 4


@dataclass
class Grid:
    """One structured block: dims, periodicity, body-frame coordinates,
    the blank region it cuts from other grids, and its fringe faces."""
    name: str
    dims: tuple
    periodic: int
    X: np.ndarray
    Y: np.ndarray
    Z: np.ndarray
    blank_kind: int = BLANK_NONE
    blank_prm: tuple = ()
    # BLANK_MESH: closed surface triangulation [ntri, 3, 3] in the body frame
    blank_mesh: np.ndarray = None
    # fringe layers on the faces (i-, i+, j-, j+, k-, k+)
    outer: tuple = (0, 0, 0, 0, 0, 0)

    @property
    def nodes(self) -> int:
        ni, nj, nk = self.dims
        return ni * nj * nk

    def blank_prm8(self) -> np.ndarray:
        out = np.zeros(8, dtype=np.float64)
        out[: len(self.blank_prm)] = self.blank_prm
        return out


@dataclass
class Workload:
    """A complete synthetic input: grids, fringe width, motion, fields."""
    name: str
    grids: list
    nf: int
    steps: int
    poses: np.ndarray               # [steps, ngrids, 12]
    fields: np.ndarray              # [4, total_nodes] float64
    precision: str = "fp64"         # "fp64" or "mixed"
    meta: dict = field(default_factory=dict)

    @property
    def ngrids(self) -> int:
        return len(self.grids)

    @property
    def node_offsets(self) -> np.ndarray:
        off = np.zeros(self.ngrids + 1, dtype=np.int64)
        off[1:] = np.cumsum([g.nodes for g in self.grids])
        return off

    @property
    def total_nodes(self) -> int:
        return int(self.node_offsets[-1])


# ---------------------------------------------------------------- motion
def rodrigues(axis, angle: float) -> np.ndarray:
    """Rotation by `angle` about unit `axis` (Rodrigues' formula)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) * math.cos(angle) + math.sin(angle) * K + (1.0 - math.cos(angle)) * np.outer(a, a)


def rot_z(angle: float) -> np.ndarray:
    return rodrigues((0.0, 0.0, 1.0), angle)


def pose12(R: np.ndarray, c) -> np.ndarray:
    out = np.empty(12, dtype=np.float64)
    out[:9] = np.asarray(R, dtype=np.float64).reshape(9)
    out[9:] = np.asarray(c, dtype=np.float64)
    return out


IDENTITY_POSE = pose12(np.eye(3), (0.0, 0.0, 0.0))


def world_coords(grid: Grid, pose: np.ndarray):
    """Node positions of `grid` under `pose` (input preparation only: used to
    evaluate synthetic fields at t=0, never as a step result)."""
    R = pose[:9].reshape(3, 3)
    c = pose[9:]
    P = np.stack([grid.X, grid.Y, grid.Z])
    W = R @ P + c[:, None]
    return W[0], W[1], W[2]


# ---------------------------------------------------------------- grids
def _tensor(xs, ys, zs):
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy()


def cartesian_grid(n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), name="background") -> Grid:
    ni, nj, nk = (n, n, n) if np.isscalar(n) else n
    xs = np.linspace(lo[0], hi[0], ni)
    ys = np.linspace(lo[1], hi[1], nj)
    zs = np.linspace(lo[2], hi[2], nk)
    X, Y, Z = _tensor(xs, ys, zs)
    return Grid(name, (ni, nj, nk), 0, X, Y, Z)


def tanh_stretch(n: int, beta: float) -> np.ndarray:
    """Node positions on [0,1] clustered toward the centre: the inverse of
    xi = (1 + tanh(beta (x - 1/2)) / tanh(beta/2)) / 2 at xi = i/(n-1)."""
    xi = np.linspace(0.0, 1.0, n)
    x = 0.5 + np.arctanh((2.0 * xi - 1.0) * math.tanh(beta / 2.0)) / beta
    x[0], x[-1] = 0.0, 1.0
    return x


def _local_spacing(x: np.ndarray) -> np.ndarray:
    d = np.empty_like(x)
    d[1:-1] = 0.5 * (x[2:] - x[:-2])
    d[0] = x[1] - x[0]
    d[-1] = x[-1] - x[-2]
    return d


def stretched_background(dims, extent=(1.0, 1.0, 1.0), beta=2.0, perturb=0.1,
                         wavelength=16, name="background") -> Grid:
    """Curvilinear background: per-axis tanh stretching toward the centre plus a
    sinusoidal node perturbation of `perturb` local cells with a `wavelength`
    node period; each coordinate is perturbed by the product of sines of the
    other two indices, so cell faces are non-planar. No random draws."""
    ni, nj, nk = dims
    xs = tanh_stretch(ni, beta) * extent[0]
    ys = tanh_stretch(nj, beta) * extent[1]
    zs = tanh_stretch(nk, beta) * extent[2]
    dx, dy, dz = _local_spacing(xs), _local_spacing(ys), _local_spacing(zs)
    w = 2.0 * math.pi / wavelength
    si = np.sin(w * np.arange(ni))
    sj = np.sin(w * np.arange(nj))
    sk = np.sin(w * np.arange(nk))
    # shape [nk, nj, ni]
    X = xs[None, None, :] + perturb * dx[None, None, :] * (sj[None, :, None] * sk[:, None, None])
    Y = ys[None, :, None] + perturb * dy[None, :, None] * (sk[:, None, None] * si[None, None, :])
    Z = zs[:, None, None] + perturb * dz[:, None, None] * (si[None, None, :] * sj[None, :, None])
    shape = (nk, nj, ni)
    X = np.broadcast_to(X, shape).ravel().copy()
    Y = np.broadcast_to(Y, shape).ravel().copy()
    Z = np.broadcast_to(Z, shape).ravel().copy()
    return Grid(name, (ni, nj, nk), 0, X, Y, Z)


def cylindrical_shell(nr, nth, nz, r0, r1, z0, z1, name="cylinder") -> Grid:
    """i = radius (uniform r0..r1), j = angle (periodic, 2 pi j / nth),
    k = axial (uniform z0..z1); body frame centred on the axis."""
    r = np.linspace(r0, r1, nr)
    th = 2.0 * math.pi * np.arange(nth) / nth
    z = np.linspace(z0, z1, nz)
    R = r[None, None, :]
    T = th[None, :, None]
    X = np.broadcast_to(R * np.cos(T), (nz, nth, nr))
    Y = np.broadcast_to(R * np.sin(T), (nz, nth, nr))
    Zc = np.broadcast_to(z[:, None, None], (nz, nth, nr))
    return Grid(name, (nr, nth, nz), PERIODIC_J, X.ravel().copy(), Y.ravel().copy(), Zc.ravel().copy())


def ellipsoidal_shell(nr, nphi, nth, inner, outer, name="shell") -> Grid:
    """Shell between two coaxial ellipsoids with semi-axes `inner` and `outer`
    (body frame, along x, y, z). i = layer (semi-axes interpolated linearly
    inner -> outer), j = azimuth phi about x (periodic), k = polar angle
    theta from +x in [0, pi] with pole nodes (degenerate polar cells).
    A sphere is inner = (r0,)*3, outer = (r1,)*3."""
    t = np.linspace(0.0, 1.0, nr)
    a = inner[0] + t * (outer[0] - inner[0])
    b = inner[1] + t * (outer[1] - inner[1])
    c = inner[2] + t * (outer[2] - inner[2])
    phi = 2.0 * math.pi * np.arange(nphi) / nphi
    th = math.pi * np.arange(nth) / (nth - 1)
    ct = np.cos(th)
    st = np.sin(th)
    ct[0], ct[-1], st[0], st[-1] = 1.0, -1.0, 0.0, 0.0
    A = a[None, None, :]
    B = b[None, None, :]
    C = c[None, None, :]
    CT = ct[:, None, None]
    ST = st[:, None, None]
    CP = np.cos(phi)[None, :, None]
    SP = np.sin(phi)[None, :, None]
    shape = (nth, nphi, nr)
    X = np.broadcast_to(A * CT, shape)
    Y = np.broadcast_to(B * ST * CP, shape)
    Z = np.broadcast_to(C * ST * SP, shape)
    return Grid(name, (nr, nphi, nth), PERIODIC_J, X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy())


def spherical_shell(nr, nphi, nth, r0, r1, name="sphere") -> Grid:
    return ellipsoidal_shell(nr, nphi, nth, (r0, r0, r0), (r1, r1, r1), name=name)


def perturbed_box_grid(rng, dims, h=1.0, amp=0.2, periodic=0, name="random") -> Grid:
    """Tiny random curvilinear grid: a unit-spacing lattice scaled by h with every
    node moved by U[-amp, amp] * h per coordinate (draws: X, Y, Z noise, in
    that order). `periodic` is recorded as given; a ring geometry for periodic
    directions comes from the shell builders instead."""
    ni, nj, nk = dims
    X, Y, Z = _tensor(np.arange(ni) * h, np.arange(nj) * h, np.arange(nk) * h)
    X = X + rng.uniform(-amp, amp, X.shape) * h
    Y = Y + rng.uniform(-amp, amp, Y.shape) * h
    Z = Z + rng.uniform(-amp, amp, Z.shape) * h
    return Grid(name, (ni, nj, nk), periodic, X, Y, Z)


# ---------------------------------------------------------------- fields
def fourier_modes(rng, nmodes=8, kmax=4):
    """Draw order per mode: k (3 integers in [-kmax, kmax], redrawn while all
    zero), amplitude U[-1, 1], phase U[0, 2 pi)."""
    modes = []
    for _ in range(nmodes):
        while True:
            k = rng.integers(-kmax, kmax + 1, size=3)
            if np.any(k != 0):
                break
        A = rng.uniform(-1.0, 1.0)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        modes.append((k.astype(np.float64), A, ph))
    return modes


_CHUNK = 1 << 20


def _eval_modes_chunk(modes, x, y, z, q):
    q[:] = 0.0
    for k, A, ph in modes:
        q += A * np.cos(2.0 * math.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)


def eval_modes(modes, x, y, z):
    """Sum of the modes at every point, evaluated in fixed 2^20-point chunks on
    a thread pool (numpy releases the GIL inside its loops)."""
    q = np.empty_like(x)
    n = x.size
    spans = [(a, min(a + _CHUNK, n)) for a in range(0, n, _CHUNK)]
    if len(spans) <= 1:
        _eval_modes_chunk(modes, x, y, z, q)
        return q
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(lambda ab: _eval_modes_chunk(modes, x[ab[0]:ab[1]], y[ab[0]:ab[1]], z[ab[0]:ab[1]],
                                                 q[ab[0]:ab[1]]), spans))
    return q


def _fields_from(grids, poses0, fn) -> np.ndarray:
    total = sum(g.nodes for g in grids)
    out = np.empty((4, total), dtype=np.float64)
    o = 0
    for g, p in zip(grids, poses0):
        x, y, z = world_coords(g, p)
        vals = fn(x, y, z)
        for f in range(4):
            out[f, o:o + g.nodes] = vals[f]
        o += g.nodes
    return out


def linear_field(x, y, z):
    return 1.0 + 2.0 * x - 3.0 * y + 0.5 * z


def analytic_fields_c0(x, y, z):
    return (linear_field(x, y, z),
            np.sin(2.0 * math.pi * x) * np.cos(2.0 * math.pi * y),
            np.zeros_like(x),
            x * y * z)


# ---------------------------------------------------------------- configs
def c0() -> Workload:
    """Tiny FP64 case: 32^3 uniform background on [0,1]^3; one cylindrical
    shell 16^3 (r 0.05..0.2, 16 periodic angles, z 0.3..0.7) about the axis
    (0.5, 0.5), rotated 0.3 rad about z; its body r < 0.05, z in [0.3, 0.7]
    is cut from the background; its outer 2 radial layers are fringe;
    buffer width 2. Analytic fields; one step; no random draws."""
    bg = cartesian_grid(32)
    cyl = cylindrical_shell(16, 16, 16, 0.05, 0.2, 0.3, 0.7)
    cyl.blank_kind = BLANK_CYL
    cyl.blank_prm = (0.05, 0.3, 0.7)
    cyl.outer = (0, 2, 0, 0, 0, 0)
    grids = [bg, cyl]
    poses = np.stack([IDENTITY_POSE, pose12(rot_z(0.3), (0.5, 0.5, 0.0))])[None]
    fields = _fields_from(grids, poses[0], analytic_fields_c0)
    return Workload("C0", grids, nf=2, steps=1, poses=poses, fields=fields,
                    meta={"seed": 0})


def sphere_motion(rng, steps, omega, speed, c0):
    """Pose table of a rigid rotation `omega` rad/step about a random unit axis
    plus a translation `speed`/step along a random unit direction (draws: axis
    as 3 normals, then direction as 3 normals)."""
    axis = rng.normal(size=3)
    axis /= np.linalg.norm(axis)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    poses = np.empty((steps, 12))
    for t in range(steps):
        poses[t] = pose12(rodrigues(axis, omega * t), np.asarray(c0) + t * speed * d)
    return poses, axis, d


def sphere_case(name, bg_dims, shell_dims, r0, r1, steps, seed, nf=2,
                omega=0.01, cells_per_step=0.2, precision="fp64") -> Workload:
    """Stretched, perturbed background on [0,1]^3 and one spherical shell
    (radial, azimuth, polar) centred at (0.5, 0.5, 0.5) whose body r < r0 is
    cut from the background; outer `nf` radial layers are fringe. Motion:
    `omega` rad/step about a random axis and `cells_per_step` mean background
    cells per step along a random direction. Fields: per field, a sum of 8
    random Fourier modes (k <= 4) evaluated at t=0 node positions.
    Draw order from default_rng(seed): axis, direction, then modes of u, v, w, p."""
    rng = np.random.default_rng(seed)
    bg = stretched_background(bg_dims)
    sph = spherical_shell(*shell_dims, r0, r1)
    sph.blank_kind = BLANK_SPHERE
    sph.blank_prm = (r0,)
    sph.outer = (0, nf, 0, 0, 0, 0)
    cell = 1.0 / (bg_dims[0] - 1)
    sp, axis, d = sphere_motion(rng, steps, omega, cells_per_step * cell, (0.5, 0.5, 0.5))
    poses = np.empty((steps, 2, 12))
    poses[:, 0] = IDENTITY_POSE
    poses[:, 1] = sp
    modes = [fourier_modes(rng) for _ in range(4)]
    grids = [bg, sph]
    fields = _fields_from(grids, poses[0], lambda x, y, z: [eval_modes(m, x, y, z) for m in modes])
    return Workload(name, grids, nf=nf, steps=steps, poses=poses, fields=fields,
                    precision=precision,
                    meta={"seed": seed, "axis": axis.tolist(), "direction": d.tolist()})


def c1(steps=100) -> Workload:
    """256^3 stretched curvilinear background + spherical shell 128x128x64,
    r 0.02..0.12, 0.01 rad/step + 0.2 cell/step, 2 fringe layers, seed 1."""
    return sphere_case("C1", (256, 256, 256), (128, 128, 64), 0.02, 0.12, steps, seed=1)


def c2(steps=100) -> Workload:
    """C1's grids and motion, run in mixed precision."""
    w = c1(steps)
    w.name = "C2"
    w.precision = "mixed"
    return w


def c1_small(steps=4, seed=11) -> Workload:
    """A scaled-down C1 for parity tests: 64^3 background, shell 24x32x17."""
    return sphere_case("C1-small", (64, 64, 64), (24, 32, 17), 0.06, 0.2, steps, seed=seed,
                       omega=0.05, cells_per_step=0.7)


# ---------------------------------------------------------------- school of fish
# Body-frame semi-axes (axial x, lateral y, vertical z) in fish lengths L:
# the body (inner shell surface), the blank region cut from every other grid,
# and the outer shell surface.
FISH_BODY = (0.5, 0.07, 0.12)
FISH_BLANK = (0.58, 0.12, 0.16)
FISH_OUTER = (0.95, 0.45, 0.38)
# Diamond: front fish, two side fish (lateral +-0.45 L, 1.2 L behind) and
# the last fish 2.4 L behind (the paper's side offset; a shorter axial
# spacing than its 1.45 L so that neighbouring shells overlap and exchange
# fringe points).
DIAMOND = ((0.0, 0.0), (-1.2, 0.45), (-1.2, -0.45), (-2.4, 0.0))


def triangulated_ellipsoid(semi, level: int, seed: int) -> np.ndarray:
    """A closed triangulation [ntri, 3, 3] of the ellipsoid with semi-axes
    `semi`: an icosahedron subdivided `level` times (each triangle into four,
    new vertices pushed onto the unit sphere; 20 * 4^level triangles, no
    vertex joined to more than six), turned by a random rotation drawn from
    default_rng(seed) so that no vertex or edge sits on a special plane, then
    scaled per axis. Every vertex lies on the ellipsoid; shared vertices are
    the same numbers in every triangle that uses them."""
    rng = np.random.default_rng(seed)
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                  [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                  [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])
    t = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [np.array(v, dtype=np.float64) for v in
             ((-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
              (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1))]
    verts = [v / np.linalg.norm(v) for v in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
             (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
             (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        mid = {}

        def midpoint(i, j):
            key = (min(i, j), max(i, j))
            if key not in mid:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                mid[key] = len(verts) - 1
            return mid[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = (np.array(verts) @ R.T) * np.asarray(semi, dtype=np.float64)
    return np.ascontiguousarray(V[np.array(faces)])


def school_case(name, bg_dims, shell_dims, L, steps, seed, nf=2, precision="mixed",
                extent=(1.5, 1.0, 1.0), diamonds=((0.95, 0.5, 0.3), (0.95, 0.5, 0.7)), dt=1.0 / 240.0,
                mesh=None) -> Workload:
    """Stretched background on [0,1.5]x[0,1]^2 and two diamonds of four
    fish-like ellipsoidal shells (polar axis along the swimming direction x).
    shell_dims: (N_r, N_phi, N_theta) of the four positions of a diamond.
    Motion of fish g at time t = step * dt (frequency 1): heave
    0.1 L sin(2 pi t + a_g) along y, yaw 0.2 sin(2 pi t + b_g) about z,
    translation U_g t along x with U_g in [0.1, 0.3] L per unit time.
    Draw order from default_rng(seed): for each fish a_g, b_g, U_g; then the
    Fourier modes of u, v, w, p. mesh = a subdivision level: each fish's
    blank region is the triangulated ellipsoid of the same semi-axes
    (ray-parity hole cut), its rotation drawn from default_rng(seed + 1000 + g)."""
    rng = np.random.default_rng(seed)
    bg = stretched_background(bg_dims, extent=extent)
    grids = [bg]
    centres = []
    for dc in diamonds:
        for (dx, dy), dims in zip(DIAMOND, shell_dims):
            g = ellipsoidal_shell(*dims, tuple(L * a for a in FISH_BODY), tuple(L * a for a in FISH_OUTER),
                                  name=f"fish{len(grids)}")
            g.blank_kind = BLANK_ELLIPSOID
            g.blank_prm = tuple(L * a for a in FISH_BLANK)
            if mesh is not None:
                g.blank_kind = BLANK_MESH
                g.blank_mesh = triangulated_ellipsoid(g.blank_prm, mesh, seed + 1000 + len(grids))
            g.outer = (0, nf, 0, 0, 0, 0)
            grids.append(g)
            centres.append((dc[0] + dx * L, dc[1] + dy * L, dc[2]))
    motion = [(rng.uniform(0, 2 * math.pi), rng.uniform(0, 2 * math.pi), rng.uniform(0.1, 0.3)) for _ in centres]
    poses = np.empty((steps, len(grids), 12))
    for t in range(steps):
        tt = t * dt
        poses[t, 0] = IDENTITY_POSE
        for g, (c, (a, b, U)) in enumerate(zip(centres, motion)):
            yaw = 0.2 * math.sin(2 * math.pi * tt + b)
            heave = 0.1 * L * math.sin(2 * math.pi * tt + a)
            poses[t, g + 1] = pose12(rot_z(yaw), (c[0] + U * L * tt, c[1] + heave, c[2]))
    modes = [fourier_modes(rng) for _ in range(4)]
    fields = _fields_from(grids, poses[0], lambda x, y, z: [eval_modes(m, x, y, z) for m in modes])
    return Workload(name, grids, nf=nf, steps=steps, poses=poses, fields=fields, precision=precision,
                    meta={"seed": seed, "L": L, "body": FISH_BODY, "blank": FISH_BLANK, "outer": FISH_OUTER,
                          "diamond": DIAMOND, "motion": motion})


def c3(steps=200) -> Workload:
    """384x256x256 stretched background, 8 fish shells of uneven sizes (two
    each of 64^3, 96x64x64, 128x96x64, 160x96x96), L = 0.25, 200 steps,
    mixed precision, seed 3."""
    return school_case("C3", (384, 256, 256), ((160, 96, 96), (128, 96, 64), (96, 64, 64), (64, 64, 64)),
                       0.25, steps, seed=3)


def c3_small(steps=4, precision="fp64") -> Workload:
    """A scaled-down school for parity tests: 128x96x96 background, shells
    of 12-24 layers, faster motion (dt = 1/24)."""
    return school_case("C3-small", (128, 96, 96), ((24, 24, 20), (20, 20, 16), (16, 20, 16), (12, 16, 12)),
                       0.25, steps, seed=33, precision=precision, dt=1.0 / 24.0)


def c3_mesh(steps=200) -> Workload:
    """C3 with each fish's blank region given as a closed surface
    triangulation (icosahedron subdivided 4 times, 5,120 triangles) instead
    of the implicit ellipsoid: the hole cut by ray parity."""
    return school_case("C3M", (384, 256, 256), ((160, 96, 96), (128, 96, 64), (96, 64, 64), (64, 64, 64)),
                       0.25, steps, seed=3, mesh=4)


def c3_mesh_small(steps=4, precision="fp64") -> Workload:
    """The small school with triangulated blank surfaces (icosahedron
    subdivided twice, 320 triangles per fish) for parity tests."""
    return school_case("C3M-small", (128, 96, 96), ((24, 24, 20), (20, 20, 16), (16, 20, 16), (12, 16, 12)),
                       0.25, steps, seed=33, precision=precision, dt=1.0 / 24.0, mesh=2)


# ---------------------------------------------------------------- many random shells
def shells_case(name, bg_n, nshells, steps, seed, nf=3, dims_lo=(48, 48, 48), dims_hi=(192, 128, 128),
                precision="mixed", period=100.0, field_dtype=np.float32, r1_range=(0.04, 0.07)) -> Workload:
    """Stretched, perturbed bg_n^3 background on [0,1]^3 and `nshells`
    spherical shells. Per shell, drawn from default_rng(seed) in this order:
    N_r, N_phi, N_theta (uniform integers in dims_lo..dims_hi); outer radius
    r1 ~ U[r1_range] (default 0.04..0.07); inner radius r0 = r1 * U[0.3, 0.45]; the centre,
    uniform in [0.12, 0.88]^3 and redrawn while it is closer than
    0.8 (r1 + r1') to an earlier centre; a rotation axis (3 normals); a
    tangential speed at r1 ~ U[0.2, 0.5] cells/step; a translation direction
    (3 normals); a peak translation speed ~ U[0.2, 0.5] cells/step. The body
    r < r0 is cut from the other grids. Motion: steady rotation, translation
    oscillating with `period` steps. Fields (closed form, FP32 by default):
    u = 1 + 2x - 3y + z/2, v = sin(2 pi x) cos(2 pi y), w = cos(2 pi z),
    p = x y z at t=0 node positions."""
    rng = np.random.default_rng(seed)
    cell = 1.0 / (bg_n - 1)
    grids = [stretched_background((bg_n, bg_n, bg_n))]
    spec = []
    for g in range(nshells):
        dims = tuple(int(rng.integers(lo, hi + 1)) for lo, hi in zip(dims_lo, dims_hi))
        r1 = rng.uniform(*r1_range)
        r0 = r1 * rng.uniform(0.3, 0.45)
        while True:
            c = rng.uniform(0.12, 0.88, 3)
            if all(np.linalg.norm(c - c2) >= 0.8 * (r1 + r12) for (_, _, r12, c2, *_rest) in spec):
                break
        axis = rng.normal(size=3)
        omega = rng.uniform(0.2, 0.5) * cell / r1
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        amp = rng.uniform(0.2, 0.5) * cell * period / (2 * math.pi)
        spec.append((dims, r0, r1, c, axis, omega, d, amp))
        sh = spherical_shell(*dims, r0, r1, name=f"shell{g + 1}")
        sh.blank_kind = BLANK_SPHERE
        sh.blank_prm = (r0,)
        sh.outer = (0, nf, 0, 0, 0, 0)
        grids.append(sh)
    poses = np.empty((steps, len(grids), 12))
    for t in range(steps):
        poses[t, 0] = IDENTITY_POSE
        for g, (dims, r0, r1, c, axis, omega, d, amp) in enumerate(spec):
            poses[t, g + 1] = pose12(rodrigues(axis, omega * t), c + amp * math.sin(2 * math.pi * t / period) * d)
    total = sum(gr.nodes for gr in grids)
    fields = np.empty((4, total), dtype=field_dtype)
    o = 0
    for gr, p in zip(grids, poses[0]):
        n = gr.nodes
        for a in range(0, n, 1 << 24):
            b = min(n, a + (1 << 24))
            sub = Grid(gr.name, (b - a, 1, 1), 0, gr.X[a:b], gr.Y[a:b], gr.Z[a:b])
            x, y, z = world_coords(sub, p)
            fields[0, o + a:o + b] = 1.0 + 2.0 * x - 3.0 * y + 0.5 * z
            fields[1, o + a:o + b] = np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y)
            fields[2, o + a:o + b] = np.cos(2 * math.pi * z)
            fields[3, o + a:o + b] = x * y * z
        o += n
    return Workload(name, grids, nf=nf, steps=steps, poses=poses, fields=fields, precision=precision,
                    meta={"seed": seed, "shells": [(s_[0], s_[1], s_[2], s_[3].tolist()) for s_ in spec]})


def c4(steps=500) -> Workload:
    """512^3 background, 16 spherical shells from 48^3 to 192x128x128 (seed 4),
    up to 0.5 cell/step of motion, 3 fringe layers, FP32 fields, 500 steps."""
    return shells_case("C4", 512, 16, steps, seed=4)


def c4_small(steps=4, precision="fp64") -> Workload:
    """A scaled-down C4 for parity tests: 96^3 background, 5 shells of 12-24
    nodes per direction and outer radius 0.1..0.16."""
    return shells_case("C4-small", 96, 5, steps, seed=44, dims_lo=(12, 12, 9), dims_hi=(24, 24, 17),
                       precision=precision, field_dtype=np.float64, r1_range=(0.1, 0.16))


CONFIGS = {"C0": c0, "C1": c1, "C2": c2, "C1-small": c1_small, "C3": c3, "C3-small": c3_small,
           "C3M": c3_mesh, "C3M-small": c3_mesh_small, "C4": c4, "C4-small": c4_small}


def build(name: str, **kw) -> Workload:
    return CONFIGS[name](**kw)
