"""Seeded synthetic inputs for the dense BEM hot path.

This module holds only input generation: closed triangle meshes (icosphere,
cubed sphere / ellipsoid, boxes and graded bars), seeded vertex jitter, and the
random draws of plane-wave incidence.  It contains none of the method's
arithmetic (no basis functions, no Green's function, no quadrature) and is the
only module shared by the CPU oracle and the GPU library's tests and benchmark.

Conventions: triangles are counter-clockwise about the outward normal; vertex
coordinates are float64 in metres; triangle indices are int32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C0 = 299_792_458.0  # speed of light in vacuum, m/s (exact by SI definition)
EPS0 = 8.8541878128e-12  # vacuum permittivity, F/m (CODATA 2018)


# ---------------------------------------------------------------- primitives

def _orient_outward(xyz: np.ndarray, tri: np.ndarray, center: np.ndarray) -> np.ndarray:
    """Flip triangles whose normal points towards `center` (valid for star-shaped surfaces)."""
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    nrm = np.cross(b - a, c - a)
    cen = (a + b + c) / 3.0 - center
    flip = np.einsum("ij,ij->i", nrm, cen) < 0.0
    out = tri.copy()
    out[flip] = out[flip][:, [0, 2, 1]]
    return out


def icosphere(level: int, radius: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """Icosahedron refined `level` times by midpoint splitting (20*4**level triangles)."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, dtype=np.float64) / math.sqrt(1 + t * t) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(i: int, j: int) -> int:
            key = (i, j) if i < j else (j, i)
            if key not in cache:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    xyz = np.array(verts) * radius
    tri = np.array(faces, dtype=np.int32)
    return xyz, _orient_outward(xyz, tri, np.zeros(3)).astype(np.int32)


def tetrahedron(radius: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """Regular tetrahedron inscribed in a sphere of the given radius (4 triangles)."""
    v = np.array([(1, 1, 1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)], dtype=np.float64) / math.sqrt(3.0)
    tri = np.array([(0, 1, 2), (0, 3, 1), (0, 2, 3), (1, 3, 2)], dtype=np.int32)
    xyz = v * radius
    return xyz, _orient_outward(xyz, tri, np.zeros(3)).astype(np.int32)


def octahedron(radius: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """Regular octahedron inscribed in a sphere of the given radius (8 triangles)."""
    v = np.array([(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)], dtype=np.float64)
    tri = np.array([(0, 2, 4), (2, 1, 4), (1, 3, 4), (3, 0, 4), (2, 0, 5), (1, 2, 5), (3, 1, 5), (0, 3, 5)],
                   dtype=np.int32)
    xyz = v * radius
    return xyz, _orient_outward(xyz, tri, np.zeros(3)).astype(np.int32)


def bipyramid(n: int, radius: float = 1.0, height: float = 1.0, rings: int = 2) -> tuple[np.ndarray, np.ndarray]:
    """Double cone over an n-gon with `rings` rings of n vertices between the equator and each
    apex: the apexes have valence n (the largest vertex valence of the mesh)."""
    verts = [np.array([0.0, 0.0, height]), np.array([0.0, 0.0, -height])]
    levels = [height * (1 - (i + 1) / (rings + 1)) for i in range(rings)]
    zs = levels + [0.0] + [-z for z in reversed(levels)]
    ring_start = []
    for r, z in enumerate(zs):
        rad = radius * (1 - abs(z) / height)
        ring_start.append(len(verts))
        off = 0.5 * (r % 2)
        for i in range(n):
            a = 2 * math.pi * (i + off) / n
            verts.append(np.array([rad * math.cos(a), rad * math.sin(a), z]))
    tri = []
    first, last = ring_start[0], ring_start[-1]
    for i in range(n):
        tri.append((0, first + i, first + (i + 1) % n))
        tri.append((1, last + (i + 1) % n, last + i))
    for r in range(len(zs) - 1):
        a0, b0 = ring_start[r], ring_start[r + 1]
        for i in range(n):
            tri.append((a0 + i, b0 + i, b0 + (i + 1) % n))
            tri.append((a0 + i, b0 + (i + 1) % n, a0 + (i + 1) % n))
    xyz = np.array(verts)
    return xyz, _orient_outward(xyz, np.array(tri, dtype=np.int32), np.zeros(3)).astype(np.int32)


def _box_surface(xs: np.ndarray, ys: np.ndarray, zs: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Structured surface mesh of the box spanned by the sorted node arrays xs, ys, zs.

    Every boundary quad is split into two triangles along one diagonal; the
    vertex set is the boundary nodes of the tensor grid (shared along cube edges).
    """
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    vid: dict[tuple[int, int, int], int] = {}
    pts: list[tuple[float, float, float]] = []

    def node(i: int, j: int, k: int) -> int:
        key = (i, j, k)
        if key not in vid:
            vid[key] = len(pts)
            pts.append((xs[i], ys[j], zs[k]))
        return vid[key]

    quads = []
    for fixed_axis, extent in ((0, (0, nx)), (1, (0, ny)), (2, (0, nz))):
        for side in extent:
            dims = [nx, ny, nz]
            a1, a2 = [ax for ax in range(3) if ax != fixed_axis]
            for u in range(dims[a1]):
                for w in range(dims[a2]):
                    idx = []
                    for du, dw in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        ijk = [0, 0, 0]
                        ijk[fixed_axis] = side
                        ijk[a1] = u + du
                        ijk[a2] = w + dw
                        idx.append(node(*ijk))
                    quads.append(idx)
    tri = []
    for a, b, c, d in quads:
        tri += [(a, b, c), (a, c, d)]
    xyz = np.array(pts, dtype=np.float64)
    tri = np.array(tri, dtype=np.int32)
    center = np.array([(xs[0] + xs[-1]) / 2, (ys[0] + ys[-1]) / 2, (zs[0] + zs[-1]) / 2])
    return xyz, _orient_outward(xyz, tri, center).astype(np.int32)


def cube(n: int, side: float = 1.0) -> tuple[np.ndarray, np.ndarray]:
    """Cube of edge `side` centred at the origin, n x n quads per face (12 n^2 triangles)."""
    s = np.linspace(-side / 2, side / 2, n + 1)
    return _box_surface(s, s, s)


def cubed_sphere(n: int, semi_axes=(1.0, 1.0, 1.0)) -> tuple[np.ndarray, np.ndarray]:
    """Equiangular cubed sphere (12 n^2 triangles, 6 n^2 + 2 vertices) scaled to an ellipsoid."""
    s = np.tan(np.linspace(-math.pi / 4, math.pi / 4, n + 1))
    s[0], s[-1] = -1.0, 1.0
    xyz, tri = _box_surface(s, s, s)
    xyz = xyz / np.linalg.norm(xyz, axis=1, keepdims=True)
    xyz = xyz * np.asarray(semi_axes, dtype=np.float64)
    return xyz, _orient_outward(xyz, tri, np.zeros(3)).astype(np.int32)


def graded_nodes(length: float, h_min: float, h_max: float, ratio: float = 1.5,
                 include_center: bool = False) -> np.ndarray:
    """Node coordinates on [0, length], refined geometrically towards both ends.

    Spacing starts at h_min at each end, grows by `ratio` per cell and is capped
    at h_max; the middle gap is split evenly.  With include_center the node set
    contains length/2 exactly.
    """
    left = [0.0]
    h = h_min
    while left[-1] + h < length / 2 - 0.5 * h:
        left.append(left[-1] + h)
        h = min(h * ratio, h_max)
    half = length / 2
    gap = half - left[-1]
    nmid = max(1, int(math.ceil(gap / h_max - 1e-9)))
    left += [left[-1] + gap * (i + 1) / nmid for i in range(nmid)]
    left[-1] = half
    right = [length - x for x in reversed(left[:-1])]
    nodes = np.array(left + right)
    if not include_center:
        return nodes
    return nodes


def merge(meshes: list[tuple[np.ndarray, np.ndarray]]) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Concatenate disjoint closed meshes; returns xyz, tri, per-triangle object id."""
    xyzs, tris, objs = [], [], []
    off = 0
    for o, (x, t) in enumerate(meshes):
        xyzs.append(x)
        tris.append(t + off)
        objs.append(np.full(len(t), o, dtype=np.int32))
        off += len(x)
    return np.concatenate(xyzs), np.concatenate(tris).astype(np.int32), np.concatenate(objs)


def sphere_row(level: int, count: int, gap: float, radius: float = 1.0):
    """`count` icospheres of one radius along x with `gap` between neighbouring surfaces;
    returns xyz, tri, per-triangle object id."""
    x, t = icosphere(level, radius)
    return merge([(x + np.array([i * (2 * radius + gap), 0.0, 0.0]), t) for i in range(count)])


def jitter(xyz: np.ndarray, tri: np.ndarray, frac: float, seed: int) -> np.ndarray:
    """Move every vertex by an isotropic uniform offset in [-frac, frac] * mean edge length."""
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    h = np.linalg.norm(xyz[e[:, 0]] - xyz[e[:, 1]], axis=1).mean()
    rng = np.random.default_rng(seed)
    return xyz + rng.uniform(-frac, frac, size=xyz.shape) * h


def plane_wave_draws(count: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Random incidence: theta ~ U[0, pi], phi ~ U[0, 2 pi), polarisation angle psi ~ U[0, 2 pi).

    Returns (khat[count, 3], pol[count, 3]) with pol = cos(psi) theta_hat + sin(psi) phi_hat,
    a unit vector orthogonal to khat.
    """
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.0, math.pi, count)
    ph = rng.uniform(0.0, 2 * math.pi, count)
    ps = rng.uniform(0.0, 2 * math.pi, count)
    khat = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    that = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], axis=1)
    phat = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], axis=1)
    pol = np.cos(ps)[:, None] * that + np.sin(ps)[:, None] * phat
    return khat, pol


# ------------------------------------------------------------------ workloads

@dataclass
class Workload:
    """A scattering problem: closed mesh, materials, frequency and plane waves."""
    name: str
    xyz: np.ndarray
    tri: np.ndarray
    obj: np.ndarray
    freq_hz: float
    eps_r: list            # per object, complex relative permittivity (real part + loss via sigma)
    mu_r: list
    sigma: list
    eps_bg: complex = 1.0
    mu_bg: float = 1.0
    khat: np.ndarray = field(default_factory=lambda: np.array([[0.0, 0.0, -1.0]]))
    pol: np.ndarray = field(default_factory=lambda: np.array([[1.0, 0.0, 0.0]], dtype=np.complex128))

    @property
    def n_tri(self) -> int:
        return int(len(self.tri))


def freq_from_k0(k0: float) -> float:
    return k0 * C0 / (2 * math.pi)


def sphere_workload(level: int, k0a: float, eps_r: complex, radius: float = 1.0,
                    name: str | None = None) -> Workload:
    """Dielectric sphere (icosphere mesh) lit by an x-polarised plane wave along -z."""
    xyz, tri = icosphere(level, radius)
    return Workload(name or f"sphere_ico{level}", xyz, tri, np.zeros(len(tri), np.int32),
                    freq_from_k0(k0a / radius), [complex(eps_r)], [1.0], [0.0])


def config_c1() -> Workload:
    """320-triangle sphere, k0 a = 1, eps_r = 4."""
    return sphere_workload(2, 1.0, 4.0, name="sphere320_k0a1_eps4")


def config_c2() -> Workload:
    """5120-triangle sphere, k0 a = 5, eps_r = 2.5 - 0.1j."""
    return sphere_workload(4, 5.0, 2.5 - 0.1j, name="sphere5120_k0a5_eps2.5-0.1j")


def config_c2_multi(n_exc: int = 256) -> Workload:
    """The 5120-triangle sphere of config_c2 lit by `n_exc` random plane waves (many incidence
    angles through one batched solve)."""
    w = config_c2()
    khat, pol = plane_wave_draws(n_exc, seed=21)
    w.name = f"sphere5120_k0a5_eps2.5-0.1j_x{n_exc}"
    w.khat, w.pol = khat, pol.astype(np.complex128)
    return w


def config_c3(n: int = 32, n_exc: int = 256) -> Workload:
    """Jittered ellipsoid 1.0/0.6/0.4 m (cubed sphere, 12 n^2 triangles), eps_r = 6,
    k0 a_max = 8, `n_exc` random plane waves."""
    xyz, tri = cubed_sphere(n, (1.0, 0.6, 0.4))
    xyz = jitter(xyz, tri, 0.02, seed=3)
    khat, pol = plane_wave_draws(n_exc, seed=33)
    return Workload(f"ellipsoid{len(tri)}_k0a8_eps6_x{n_exc}", xyz, tri,
                    np.zeros(len(tri), np.int32), freq_from_k0(8.0), [6.0], [1.0], [0.0],
                    khat=khat, pol=pol.astype(np.complex128))


def gap_ring(xyz: np.ndarray, tri: np.ndarray, obj: np.ndarray, o: int = 0, x0: float = 0.0) -> np.ndarray:
    """Vertex pairs (a < b) of the edges of object o lying in the plane x = x0: the gap of a
    voltage-gap port across a bar."""
    t = tri[obj == o]
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    on = (np.abs(xyz[e[:, 0], 0] - x0) < 1e-15) & (np.abs(xyz[e[:, 1], 0] - x0) < 1e-15)
    return e[on].astype(np.int32)


def config_c4(n_freq: int = 32) -> Workload:
    """4 x 4 copper bars (10 x 1 x 1 um, sigma = 5.8e7 S/m, pitch 3 um) in eps_r = 4, graded
    from 0.05 um at the edges and corners to 1 um (ratio 2, 22528 triangles); the sweep's
    n_freq log-spaced frequencies 1-100 GHz are in `freqs` (freq_hz is the first); the port is
    the ring x = 0 of the first bar (`gap_ring`)."""
    xyz, tri, obj = copper_bars(h_min=0.05e-6, h_max=1.0e-6, ratio=2.0)
    w = Workload(f"copper_bars4x4_{len(tri)}_1-100GHz", xyz, tri, obj, 1e9, [1.0] * 16, [1.0] * 16, [5.8e7] * 16,
                 eps_bg=4.0)
    w.freqs = np.logspace(9, 11, n_freq)
    w.port = gap_ring(xyz, tri, obj, 0)
    return w


def config_sphere_array(n: int = 4, level: int = 2, pitch: float = 0.375) -> Workload:
    """n x n array of dielectric spheres (eps_r = 12, diameter 250 mm, icosphere of 20 4^level
    triangles each) at `pitch` in the x-y plane, centred on the origin, at 200 MHz in a
    homogeneous background with the ground layer's eps_r = 3.47 and sigma = 1.725 mS/m (the
    buried-array study of Sec. IV-B without its layer interfaces), lit by a plane wave along -z
    (standing in for the dipole above the array)."""
    f = 200e6
    x, t = icosphere(level, 0.125)
    meshes = [(x + np.array([(i - (n - 1) / 2) * pitch, (j - (n - 1) / 2) * pitch, 0.0]), t)
              for i in range(n) for j in range(n)]
    xyz, tri, obj = merge(meshes)
    eps_bg = 3.47 - 1j * 1.725e-3 / (2 * math.pi * f * EPS0)
    return Workload(f"spharr{n}x{n}_ico{len(t)}_eps12_200MHz", xyz, tri, obj, f, [12.0] * n * n, [1.0] * n * n,
                    [0.0] * n * n, eps_bg=eps_bg)


def copper_bars(h_min: float = 0.05e-6, h_max: float = 1.0e-6, pitch: float = 3.0e-6,
                grid: int = 4, ratio: float = 1.5) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """grid x grid copper bars of 10 x 1 x 1 um along x, graded towards edges and corners.

    The node set along x contains x = 0 (the gap ring used by a voltage-gap port).
    """
    xs = graded_nodes(10e-6, h_min, h_max, ratio) - 5e-6
    cs = graded_nodes(1e-6, h_min, h_max, ratio) - 0.5e-6
    meshes = []
    for iy in range(grid):
        for iz in range(grid):
            x, t = _box_surface(xs, cs + iy * pitch, cs + iz * pitch)
            meshes.append((x, t))
    return merge(meshes)


def mean_edge(xyz: np.ndarray, tri: np.ndarray) -> float:
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e = np.unique(np.sort(e, axis=1), axis=0)
    return float(np.linalg.norm(xyz[e[:, 0]] - xyz[e[:, 1]], axis=1).mean())


def mixed_stream(n_req: int, rate_hz: float, seed: int = 5, t_min: int = 320, t_max: int = 20000,
                 eps_range=(1.5, 10.0), k0a_range=(0.5, 10.0), exc_max: int = 64, min_edges_per_wl: float = 10.0):
    """The serving mix: Poisson arrivals (mean rate `rate_hz`) of scattering requests.

    Each request: shape uniform over {sphere, ellipsoid with semi-axes 1.0/0.6/0.4 m, cube of
    circumradius 1 m}, every one an n x n-per-face cube-topology mesh of 12 n^2 triangles
    (sphere and ellipsoid: cubed sphere; cube: structured box), n = round(sqrt(T / 12)) with T
    log-uniform in [t_min, t_max]; eps_r ~ U(eps_range), k0 a ~ U(k0a_range) with a the
    circumradius (1 m); R ~ U{1..exc_max} random plane waves.  A draw of (eps_r, k0 a) that leaves
    fewer than `min_edges_per_wl` mean edges per interior wavelength 2 pi / (k0 sqrt(eps_r)) on
    the drawn mesh is redrawn (the mesh draw is kept, so T keeps its stated distribution).
    Returns a list of (arrival time in s, Workload).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_req):
        t += float(rng.exponential(1.0 / rate_hz))
        target = math.exp(rng.uniform(math.log(t_min), math.log(t_max)))
        n = max(2, int(round(math.sqrt(target / 12.0))))
        kind = int(rng.integers(3))
        if kind == 0:
            xyz, tri = cubed_sphere(n, (1.0, 1.0, 1.0))
            name = f"sphere{len(tri)}"
        elif kind == 1:
            xyz, tri = cubed_sphere(n, (1.0, 0.6, 0.4))
            name = f"ellipsoid{len(tri)}"
        else:
            xyz, tri = cube(n, 2.0 / math.sqrt(3.0))
            name = f"cube{len(tri)}"
        h = mean_edge(xyz, tri)
        while True:
            eps = float(rng.uniform(*eps_range))
            k0a = float(rng.uniform(*k0a_range))
            if 2 * math.pi / (k0a * math.sqrt(eps)) / h >= min_edges_per_wl:
                break
        n_exc = int(rng.integers(1, exc_max + 1))
        khat, pol = plane_wave_draws(n_exc, seed=1000 + i)
        w = Workload(f"{name}_k0a{k0a:.2f}_eps{eps:.2f}_x{n_exc}", xyz, tri, np.zeros(len(tri), np.int32),
                     freq_from_k0(k0a), [eps], [1.0], [0.0], khat=khat, pol=pol.astype(np.complex128))
        out.append((t, w))
    return out


def serving_stream(n_req: int = 24, rate_hz: float = 6.0, seed: int = 5, n_min: int = 320, n_max: int = 3072,
                   k0a_max: float = 3.0, eps_max: float = 6.0, exc_max: int = 16):
    """A stream of scattering requests with Poisson arrivals (mean rate `rate_hz`).

    Each request: a sphere (icosphere), an ellipsoid (cubed sphere, semi-axes 1/0.7/0.5) or a
    cube, with a triangle count log-uniform in [n_min, n_max] (the nearest mesh of its kind),
    eps_r ~ U[1.5, eps_max], k0 a ~ U[0.5, k0a_max] (a = largest half-size), and a
    log-uniform number of random plane waves in [1, exc_max].  Returns a list of
    (arrival time in s, Workload).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_req):
        t += float(rng.exponential(1.0 / rate_hz))
        target = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        kind = int(rng.integers(3))
        if kind == 0:
            level = int(min(range(1, 6), key=lambda L: abs(20 * 4 ** L - target)))
            xyz, tri = icosphere(level)
            size, name = 1.0, f"sphere{len(tri)}"
        else:
            n = max(2, int(round(math.sqrt(target / 12.0))))
            if kind == 1:
                xyz, tri = cubed_sphere(n, (1.0, 0.7, 0.5))
                size, name = 1.0, f"ellipsoid{len(tri)}"
            else:
                xyz, tri = cube(n, 2.0)
                size, name = 1.0, f"cube{len(tri)}"
        eps = float(rng.uniform(1.5, eps_max))
        k0a = float(rng.uniform(0.5, k0a_max))
        n_exc = int(round(math.exp(rng.uniform(0.0, math.log(exc_max)))))
        khat, pol = plane_wave_draws(n_exc, seed=1000 + i)
        w = Workload(f"{name}_k0a{k0a:.2f}_eps{eps:.2f}_x{n_exc}", xyz, tri, np.zeros(len(tri), np.int32),
                     freq_from_k0(k0a / size), [eps], [1.0], [0.0], khat=khat, pol=pol.astype(np.complex128))
        out.append((t, w))
    return out
