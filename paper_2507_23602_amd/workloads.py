"""Seeded synthetic inputs for the semi-discrete RSOT dual evaluation.

This module builds the *data* both the HIP library and the CPU oracle consume:
finite-element meshes, their quadrature points x_q and masses mu_q =
rho_h(x_q) w_q (Sec. 3.1-3.2, Remark 3.1), and target clouds {y_j, nu_j}
(Sec. 2). It holds none of the method's arithmetic (no cost, no log-sum-exp,
no gradient): it is shared input plumbing only, importable without torch or
the compiled library.

Readings fixed here (the paper leaves them open):
  * quadrature: the symmetric degree-2 rules -- triangle barycentric
    (2/3, 1/6, 1/6) and permutations with weights |K|/3; tetrahedron
    (a, b, b, b) and permutations, a = (5 + 3 sqrt 5)/20, b = (5 - sqrt 5)/20,
    weights |K|/4. Both integrate quadratics exactly.
  * meshes: unit square split along the (i,j)-(i+1,j+1) diagonal; unit cube
    split into the 6 Kuhn tetrahedra around its (0,0,0)-(1,1,1) diagonal;
    unit disk from hexagonal rings, refined by midpoint (red) refinement with
    new boundary midpoints pushed radially onto the circle.
  * densities: P1 nodal interpolation of the analytic density (Sec. 3.1),
    evaluated at the quadrature points from barycentric coordinates, then
    masses scaled so that sum mu_q = 1 (normalised measures, Sec. 2).
  * Gaussian mixtures: equal weights, isotropic sigma; samples not clipped.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# quadrature rules (reference-element barycentric coordinates + weights)
# --------------------------------------------------------------------------
TRI3_BARY = np.array([[2.0 / 3, 1.0 / 6, 1.0 / 6],
                      [1.0 / 6, 2.0 / 3, 1.0 / 6],
                      [1.0 / 6, 1.0 / 6, 2.0 / 3]])
_A = (5.0 + 3.0 * math.sqrt(5.0)) / 20.0
_B = (5.0 - math.sqrt(5.0)) / 20.0
TET4_BARY = np.array([[_A, _B, _B, _B],
                      [_B, _A, _B, _B],
                      [_B, _B, _A, _B],
                      [_B, _B, _B, _A]])


@dataclass
class Mesh:
    """Simplicial mesh: vertices (nv x d) and cells (nc x (d+1)) of vertex ids."""
    verts: np.ndarray
    cells: np.ndarray

    @property
    def dim(self) -> int:
        return self.verts.shape[1]


@dataclass
class Problem:
    """One semi-discrete instance: source quadrature measure and target cloud."""
    x: np.ndarray            # (nq, d) quadrature points
    mu: np.ndarray           # (nq,) masses rho_h(x_q) w_q, sum 1
    y: np.ndarray            # (n, d) targets
    nu: np.ndarray           # (n,) target masses, sum 1
    eps: float
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return self.x.shape[1]

    @property
    def nq(self) -> int:
        return self.x.shape[0]

    @property
    def n(self) -> int:
        return self.y.shape[0]


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
def square_mesh(n: int, lo: float = 0.0, hi: float = 1.0) -> Mesh:
    """n x n squares of [lo,hi]^2, each split by its (i,j)-(i+1,j+1) diagonal."""
    t = np.linspace(lo, hi, n + 1)
    X, Y = np.meshgrid(t, t, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel()], axis=1)
    vid = np.arange((n + 1) ** 2).reshape(n + 1, n + 1)
    v00 = vid[:-1, :-1].ravel()
    v10 = vid[1:, :-1].ravel()
    v11 = vid[1:, 1:].ravel()
    v01 = vid[:-1, 1:].ravel()
    lower = np.stack([v00, v10, v11], axis=1)
    upper = np.stack([v00, v11, v01], axis=1)
    cells = np.empty((2 * n * n, 3), dtype=np.int64)
    cells[0::2] = lower
    cells[1::2] = upper
    return Mesh(verts, cells)


def cube_mesh(n: int, lo: float = 0.0, hi: float = 1.0) -> Mesh:
    """n^3 cubes of [lo,hi]^3, each split into the 6 Kuhn tetrahedra.

    Kuhn tetrahedron for a permutation (a, b, c) of the axes:
    v0, v0 + e_a, v0 + e_a + e_b, v0 + e_a + e_b + e_c (= the far corner).
    The split is conforming because every cube uses the same diagonal.
    """
    t = np.linspace(lo, hi, n + 1)
    X, Y, Z = np.meshgrid(t, t, t, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    m = n + 1
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)

    def vid(off):
        p = base + np.asarray(off)
        return (p[:, 0] * m + p[:, 1]) * m + p[:, 2]

    e = np.eye(3, dtype=np.int64)
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    tets = []
    for (a, b, c) in perms:
        o0 = np.zeros(3, dtype=np.int64)
        o1 = e[a]
        o2 = e[a] + e[b]
        o3 = e[a] + e[b] + e[c]
        tets.append(np.stack([vid(o0), vid(o1), vid(o2), vid(o3)], axis=1))
    cells = np.stack(tets, axis=1).reshape(-1, 4)
    return Mesh(verts, cells)


def disk_mesh(rings: int, radius: float = 1.0) -> Mesh:
    """Disk triangulation from hexagonal rings (6 r^2 triangles for r rings).

    Ring k (k = 1..rings) holds 6k vertices on the circle of radius
    k * radius / rings; consecutive rings are stitched into 6(2k-1) triangles.
    """
    pts = [np.zeros((1, 2))]
    ring_start = [0]
    count = 1
    for k in range(1, rings + 1):
        ang = 2.0 * np.pi * np.arange(6 * k) / (6 * k)
        r = k * radius / rings
        pts.append(np.stack([r * np.cos(ang), r * np.sin(ang)], axis=1))
        ring_start.append(count)
        count += 6 * k
    verts = np.concatenate(pts, axis=0)
    cells = []
    for k in range(1, rings + 1):
        inner_n = 6 * (k - 1) if k > 1 else 1
        outer_n = 6 * k
        s_in = ring_start[k - 1]
        s_out = ring_start[k]
        for side in range(6):
            for t in range(k):
                o = side * k + t
                o1 = (o + 1) % outer_n
                if k == 1:
                    cells.append((s_in, s_out + o, s_out + o1))
                    continue
                i0 = (side * (k - 1) + t) % inner_n
                cells.append((s_in + i0, s_out + o, s_out + o1))
                if t < k - 1:
                    i1 = (i0 + 1) % inner_n
                    cells.append((s_in + i0, s_out + o1, s_in + i1))
    cells = np.asarray(cells, dtype=np.int64)
    return Mesh(verts, cells)


def refine_triangles(mesh: Mesh, radius: float | None = None) -> Mesh:
    """Red refinement: every triangle into 4 through edge midpoints.

    With ``radius`` set, midpoints of boundary edges are pushed radially onto
    the circle of that radius (disk hierarchy). The refined mesh is nested in
    the sense of the multilevel remark of Sec. 5.1 up to this boundary move.
    """
    v = mesh.verts
    c = mesh.cells
    edges = np.concatenate([c[:, [0, 1]], c[:, [1, 2]], c[:, [2, 0]]], axis=0)
    e_sorted = np.sort(edges, axis=1)
    uniq, inv, counts = np.unique(e_sorted, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    mids = 0.5 * (v[uniq[:, 0]] + v[uniq[:, 1]])
    if radius is not None:
        boundary = counts == 1
        r = np.linalg.norm(mids[boundary], axis=1)
        mids[boundary] *= (radius / r)[:, None]
    nv = v.shape[0]
    verts = np.concatenate([v, mids], axis=0)
    nc = c.shape[0]
    m01 = nv + inv[0:nc]
    m12 = nv + inv[nc:2 * nc]
    m20 = nv + inv[2 * nc:3 * nc]
    a, b, cc = c[:, 0], c[:, 1], c[:, 2]
    new = np.stack([
        np.stack([a, m01, m20], axis=1),
        np.stack([m01, b, m12], axis=1),
        np.stack([m20, m12, cc], axis=1),
        np.stack([m01, m12, m20], axis=1),
    ], axis=1).reshape(-1, 3)
    return Mesh(verts, new)


# --------------------------------------------------------------------------
# quadrature measure
# --------------------------------------------------------------------------
def cell_measures(mesh: Mesh) -> np.ndarray:
    """|K| for every simplex (area in 2D, volume in 3D)."""
    v = mesh.verts[mesh.cells]           # (nc, d+1, d)
    e = v[:, 1:, :] - v[:, :1, :]        # (nc, d, d)
    det = np.linalg.det(e)
    return np.abs(det) / math.factorial(mesh.dim)


def quadrature(mesh: Mesh, vertex_density: np.ndarray | None = None,
               normalise: bool = True):
    """Quadrature points and masses mu_q = rho_h(x_q) w_q (Remark 3.1).

    ``vertex_density`` holds nodal values of rho (P1 interpolation); None
    means rho = 1. Points are ordered cell by cell.
    """
    d = mesh.dim
    bary = TRI3_BARY if d == 2 else TET4_BARY
    npc = bary.shape[0]
    vol = cell_measures(mesh)
    cv = mesh.verts[mesh.cells]                          # (nc, d+1, d)
    x = np.einsum("pk,ckd->cpd", bary, cv).reshape(-1, d)
    w = np.repeat(vol / npc, npc)
    if vertex_density is None:
        rho = np.ones_like(w)
    else:
        rv = vertex_density[mesh.cells]                  # (nc, d+1)
        rho = np.einsum("pk,ck->cp", bary, rv).reshape(-1)
    mu = rho * w
    if normalise:
        mu = mu / mu.sum()
    return np.ascontiguousarray(x), np.ascontiguousarray(mu)


# --------------------------------------------------------------------------
# densities and clouds
# --------------------------------------------------------------------------
def mixture_means(rng: np.random.Generator, k: int, d: int, lo=0.2, hi=0.8):
    return rng.uniform(lo, hi, size=(k, d))


def mixture_density(pts: np.ndarray, means: np.ndarray, sigma: float) -> np.ndarray:
    """Equal-weight isotropic Gaussian mixture, up to a constant factor."""
    r2 = ((pts[:, None, :] - means[None, :, :]) ** 2).sum(-1)
    return np.exp(-r2 / (2.0 * sigma * sigma)).mean(axis=1)


def mixture_samples(rng: np.random.Generator, means: np.ndarray, sigma: float,
                    n: int) -> np.ndarray:
    comp = rng.integers(0, means.shape[0], size=n)
    return means[comp] + sigma * rng.standard_normal((n, means.shape[1]))


def uniform_targets(seed: int, n: int, d: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(n, d))


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
def square_uniform(n_cells: int, n_targets: int, seed: int, eps: float) -> Problem:
    """Unit square, uniform density, targets uniform in the square."""
    x, mu = quadrature(square_mesh(n_cells))
    y = uniform_targets(seed, n_targets, 2)
    nu = np.full(n_targets, 1.0 / n_targets)
    return Problem(x, mu, y, nu, eps, name=f"square{n_cells}_n{n_targets}")


def config1() -> Problem:
    """2D unit square, 32x32 -> 2048 P1 triangles x 3 points = 6144 points,
    uniform density, N = 256 uniform targets (seed 1), nu = 1/N, eps = 1e-2."""
    p = square_uniform(32, 256, seed=1, eps=1e-2)
    p.name = "square32_tri3_n256_eps1e-2"
    return p


def cube_mixture(n_cells: int, n_targets: int, eps: float, src_seed: int = 2,
                 tgt_mean_seed: int = 3, tgt_sample_seed: int = 4,
                 sigma: float = 0.1, k: int = 3) -> Problem:
    """Unit cube, Kuhn tetrahedra x 4 points, Gaussian-mixture source density
    (P1-interpolated), targets sampled from a different seeded mixture."""
    mesh = cube_mesh(n_cells)
    src_means = mixture_means(np.random.default_rng(src_seed), k, 3)
    rho_v = mixture_density(mesh.verts, src_means, sigma)
    x, mu = quadrature(mesh, rho_v)
    tgt_means = mixture_means(np.random.default_rng(tgt_mean_seed), k, 3)
    y = mixture_samples(np.random.default_rng(tgt_sample_seed), tgt_means, sigma, n_targets)
    nu = np.full(n_targets, 1.0 / n_targets)
    return Problem(x, mu, y, nu, eps, name=f"cube{n_cells}_tet4_mix_n{n_targets}",
                   meta={"src_means": src_means, "tgt_means": tgt_means})


def config2() -> Problem:
    """3D unit cube, 64^3 cells x 6 Kuhn tets = 1,572,864 tets x 4 points =
    6,291,456 points; 3-Gaussian-mixture source (seed 2, sigma 0.1);
    N = 65,536 targets from another mixture (means seed 3, samples seed 4);
    nu uniform, eps = 1e-3."""
    p = cube_mixture(64, 65536, 1e-3)
    p.name = "cube64_tet4_mix_nq6291456_n65536_eps1e-3"
    return p


def gaussian_blob_square(n_cells: int, centre, s: float, y: np.ndarray,
                         eps: float) -> Problem:
    """Unit square with rho(x) = exp(-|x-c|^2 / (2 s^2)), P1-interpolated."""
    mesh = square_mesh(n_cells)
    c = np.asarray(centre, dtype=np.float64)
    rho_v = np.exp(-((mesh.verts - c) ** 2).sum(1) / (2.0 * s * s))
    x, mu = quadrature(mesh, rho_v)
    nu = np.full(y.shape[0], 1.0 / y.shape[0])
    return Problem(x, mu, y, nu, eps)


def config4_instance(i: int, n_cells: int = 128, n_targets: int = 65536) -> Problem:
    """Instance i of the learned-warm-start family: c ~ U[0.2,0.8]^2,
    s ~ U[0.05,0.2], eps ~ logU[1e-3,1e-1] (seed 1000+i); fixed cloud of
    uniform targets (seed 7)."""
    rng = np.random.default_rng(1000 + i)
    c = rng.uniform(0.2, 0.8, size=2)
    s = rng.uniform(0.05, 0.2)
    eps = float(np.exp(rng.uniform(np.log(1e-3), np.log(1e-1))))
    y = uniform_targets(7, n_targets, 2)
    p = gaussian_blob_square(n_cells, c, s, y, eps)
    p.name = f"blob{i}"
    p.meta = {"c": c, "s": s}
    return p


def _config5_draw(i: int, scale: float):
    rng = np.random.default_rng(2000 + i)
    nq_t = float(np.exp(rng.uniform(np.log(1e5), np.log(4e6)))) * scale
    n_t = float(np.exp(rng.uniform(np.log(4096), np.log(262144)))) * scale
    eps = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-2))))
    n_cells = max(2, int(round((nq_t / 24.0) ** (1.0 / 3.0))))
    n_targets = max(8, int(round(n_t)))
    return rng, n_cells, n_targets, eps


def config5_sizes(i: int, scale: float = 1.0):
    """(quadrature points, targets) of batched instance i without building it."""
    _, n_cells, n_targets, _ = _config5_draw(i, scale)
    return 24 * n_cells ** 3, n_targets


def config5_instance(i: int, scale: float = 1.0) -> Problem:
    """Instance i of the batched family (seed 2000+i): N_q ~ logU[1e5, 4e6]
    realised as a cube of n^3 x 24 points, N ~ logU[4096, 262144], mixture
    source and targets (sigma 0.1), eps ~ logU[1e-4, 1e-2]. ``scale`` shrinks
    both sizes for tests."""
    rng, n_cells, n_targets, eps = _config5_draw(i, scale)
    src_seed, tm_seed, ts_seed = rng.integers(0, 2**31, size=3)
    p = cube_mixture(n_cells, n_targets, eps, int(src_seed), int(tm_seed), int(ts_seed))
    p.name = f"batch{i}"
    return p


def disk_hierarchy(rings: int = 60, levels: int = 4):
    """Nested disk meshes L0..L(levels-1) with uniform density."""
    meshes = [disk_mesh(rings)]
    for _ in range(levels - 1):
        meshes.append(refine_triangles(meshes[-1], radius=1.0))
    return meshes


def blob_targets_disk(n: int, seed: int = 5, k: int = 5, sigma: float = 0.08,
                      rmax: float = 0.6) -> np.ndarray:
    """n points from an equal-weight k-blob mixture, means uniform in the disk
    of radius rmax."""
    rng = np.random.default_rng(seed)
    r = rmax * np.sqrt(rng.uniform(size=k))
    a = rng.uniform(0, 2 * np.pi, size=k)
    means = np.stack([r * np.cos(a), r * np.sin(a)], axis=1)
    return mixture_samples(rng, means, sigma, n)


def trunc_study(density: str = "custom", n_cells: int = 25, n_targets: int = 14761,
                eps: float = 1e-2) -> Problem:
    """Inputs of the truncation-strategy study (Sec. 6.1 and its Table of
    strategies), on the benchmark's synthetic stand-ins: the unit cube in
    25^3 cells x 6 Kuhn tets = 93,750 tets x 4 points = 375,000 points (17,576
    P1 nodes, against the study's 98,304 cells and 17,969 nodes), N = 14,761
    targets from the benchmark's target mixture (means seed 3, samples seed 4,
    sigma 0.1), nu = 1/N, eps = 1e-2. density "custom": the benchmark's
    3-Gaussian source mixture (seed 2), P1-interpolated; "uniform": rho = 1."""
    if density == "custom":
        p = cube_mixture(n_cells, n_targets, eps)
    elif density == "uniform":
        x, mu = quadrature(cube_mesh(n_cells))
        tgt_means = mixture_means(np.random.default_rng(3), 3, 3)
        y = mixture_samples(np.random.default_rng(4), tgt_means, 0.1, n_targets)
        p = Problem(x, mu, y, np.full(n_targets, 1.0 / n_targets), eps)
    else:
        raise ValueError(density)
    p.name = f"cube{n_cells}_tet4_{density}_n{n_targets}_eps{eps:g}"
    return p


def gauss_legendre(order: int):
    """Nodes and weights of the order-point Gauss-Legendre rule on [-1, 1]."""
    return np.polynomial.legendre.leggauss(order)


def hex_gauss(n_cells: int, order: int, lo: float = -1.0, hi: float = 1.0):
    """Uniform hexahedral mesh of [lo, hi]^3 with n_cells^3 cubes and the
    tensor Gauss-Legendre rule of ``order`` points per direction in each
    (order^3 points per cube); uniform density: mu_q = w_q / |Omega|. Points
    are ordered cube by cube."""
    t, w = gauss_legendre(order)
    h = (hi - lo) / n_cells
    loc = (t + 1.0) * 0.5 * h                              # nodes inside one cube
    wl = w * 0.5 * h
    c = lo + h * np.arange(n_cells)
    cx, cy, cz = np.meshgrid(c, c, c, indexing="ij")
    corner = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)     # (nc, 3)
    a, b, g = np.meshgrid(np.arange(order), np.arange(order), np.arange(order), indexing="ij")
    a, b, g = a.ravel(), b.ravel(), g.ravel()
    off = np.stack([loc[a], loc[b], loc[g]], axis=1)                     # (order^3, 3)
    wq = wl[a] * wl[b] * wl[g]
    x = (corner[:, None, :] + off[None]).reshape(-1, 3)
    mu = np.tile(wq, corner.shape[0])
    return np.ascontiguousarray(x), np.ascontiguousarray(mu / mu.sum())


def ball_uniform(seed: int, n: int, d: int = 3) -> np.ndarray:
    """n points uniform in the unit ball: a normal direction, radius U^(1/d)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, d))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v * rng.uniform(0.0, 1.0, size=(n, 1)) ** (1.0 / d)


# target counts of the GPU-size workload at refinement 2..5 (App. C, Table of
# problem sizes): the vertex counts of the refined ball meshes
GPU_SIZE_TARGETS = {2: 507, 3: 3817, 4: 29521, 5: 232609}


def gpu_size(refinement: int, order: int, eps: float = 1e-2, seed: int = 21) -> Problem:
    """Workload at the sizes of App. C: source uniform on [-1, 1]^3, a hex mesh
    of (2^(refinement+1))^3 cubes with order^3 Gauss-Legendre points each
    (refinement 2, order 1: 512 cubes and points; refinement 5, order 3:
    262,144 cubes, 7,077,888 points); targets uniform
    in the unit ball (standing in for the ball mesh's vertices) in the counts
    of the refined ball meshes (507, 3,817, 29,521, 232,609), nu = 1/N;
    eps = 1e-2."""
    cells = 2 << refinement
    x, mu = hex_gauss(cells, order)
    n = GPU_SIZE_TARGETS[refinement]
    y = ball_uniform(seed + refinement, n)
    return Problem(x, mu, y, np.full(n, 1.0 / n), eps,
                   name=f"hex{cells}_gauss{order}_ball{n}_eps{eps:g}")


def small_square_instance(i: int) -> Problem:
    """Uneven small 2D instance (seed 4000 + i), between the sizes of the
    small 2D workload and the learned-start family: unit square in n x n
    cells x 2 triangles x 3 points, n = round(logU[32, 128]) (6,144 to 98,304
    points), uniform density; N ~ logU[256, 65,536] uniform targets, nu = 1/N;
    eps ~ logU[1e-3, 1e-1]."""
    rng = np.random.default_rng(4000 + i)
    n_cells = int(round(math.exp(rng.uniform(math.log(32), math.log(128)))))
    n = int(round(math.exp(rng.uniform(math.log(256), math.log(65536)))))
    eps = math.exp(rng.uniform(math.log(1e-3), math.log(1e-1)))
    x, mu = quadrature(square_mesh(n_cells))
    y = rng.uniform(0.0, 1.0, size=(n, 2))
    return Problem(x, mu, y, np.full(n, 1.0 / n), eps, name=f"square{n_cells}_n{n}_small{i}")


def icosphere(k: int) -> Mesh:
    """Unit sphere: the icosahedron with every triangle split into four at its
    edge midpoints k times, every vertex pushed onto the sphere (20 * 4^k
    triangles)."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
                  (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)],
                 dtype=np.float64)
    f = np.array([(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9),
                  (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2),
                  (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10),
                  (8, 6, 7), (9, 8, 1)], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    for _ in range(k):
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
        e.sort(axis=1)
        uniq, inv = np.unique(e, axis=0, return_inverse=True)
        mid = 0.5 * (v[uniq[:, 0]] + v[uniq[:, 1]])
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        m = inv.reshape(3, -1).T + v.shape[0]           # midpoints of (01, 12, 20)
        v = np.concatenate([v, mid])
        a, b, c = f[:, 0], f[:, 1], f[:, 2]
        ab, bc, ca = m[:, 0], m[:, 1], m[:, 2]
        f = np.concatenate([np.stack([a, ab, ca], 1), np.stack([ab, b, bc], 1),
                            np.stack([ca, bc, c], 1), np.stack([ab, bc, ca], 1)])
    return Mesh(v, f)


def sphere_quadrature(k: int, density: str = "harmonic"):
    """Quadrature points and masses on the unit sphere: the degree-2 triangle
    rule on each flat triangle of icosphere(k), the points pushed radially onto
    the sphere, masses rho(x_q) |K| / 3 normalised to sum 1. density
    "harmonic": rho = 1 + 0.9 P2(x_2), P2(z) = (3 z^2 - 1) / 2, the zonal
    eigenfunction of the Laplace-Beltrami operator of degree 2 (the fifth
    eigenvalue counted with multiplicity), shifted to stay positive;
    "uniform": rho = 1."""
    mesh = icosphere(k)
    cv = mesh.verts[mesh.cells]                                   # (nc, 3, 3)
    x = np.einsum("pk,ckd->cpd", TRI3_BARY, cv).reshape(-1, 3)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    area = 0.5 * np.linalg.norm(np.cross(cv[:, 1] - cv[:, 0], cv[:, 2] - cv[:, 0]), axis=1)
    w = np.repeat(area / 3.0, 3)
    if density == "harmonic":
        rho = 1.0 + 0.9 * 0.5 * (3.0 * x[:, 2] ** 2 - 1.0)
    elif density == "uniform":
        rho = np.ones_like(w)
    else:
        raise ValueError(density)
    mu = rho * w
    return np.ascontiguousarray(x), np.ascontiguousarray(mu / mu.sum())


def sphere_points(seed: int, n: int) -> np.ndarray:
    """n points uniform on the unit sphere (normalised Gaussian vectors)."""
    v = np.random.default_rng(seed).standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def sphere_problem(k: int, n_targets: int, eps: float, density: str = "harmonic",
                   seed: int = 40) -> Problem:
    """Blue-noise / quantization workload on the unit sphere (Sec. 6.4):
    icosphere(k) quadrature with the given density, n_targets points uniform on
    the sphere (seed), nu = 1/N; squared geodesic cost."""
    x, mu = sphere_quadrature(k, density)
    y = sphere_points(seed, n_targets)
    return Problem(x, mu, y, np.full(n_targets, 1.0 / n_targets), eps,
                   name=f"sphere{k}_{density}_n{n_targets}_eps{eps:g}")


def random_psi(seed: int, n: int, scale: float) -> np.ndarray:
    return scale * np.random.default_rng(seed).standard_normal(n)


def config3(rings: int = 60, levels: int = 4, n_targets: int = 1 << 20,
            target_levels=(1 << 14, 1 << 16, 1 << 18, 1 << 20)):
    """Multilevel workload: unit disk from hexagonal rings (6 r^2 triangles),
    red-refined levels L0..L(levels-1) (60 rings: 21,600 -> 1,382,400
    triangles, 4,147,200 points at L3), uniform density; 2^20 targets from an
    equal-weight 5-blob mixture (means uniform in the disk of radius 0.6,
    sigma 0.08, seed 5), nu uniform; target hierarchy sizes (coarsest first).

    eps is halved from 1e-1 (k = 0..9) then set to 1e-4. Two mappings of these
    stages to the four combined levels:
    * "eps"/"level" (default): the whole schedule runs on the coarsest level,
      and levels 1, 2 and 3 solve at 1e-4 only, from the refined potential;
    * "eps_spread"/"level_spread": stages {0-3}, {4-6}, {7-8}, {9, final},
      so the final eps is first reached on the finest level."""
    meshes = disk_hierarchy(rings, levels)
    sources = [quadrature(m) for m in meshes]
    y = blob_targets_disk(n_targets, seed=5)
    nu = np.full(n_targets, 1.0 / n_targets)
    sched = [0.1 * 2.0 ** (-k) for k in range(10)] + [1e-4]
    eps = sched + [1e-4] * 3
    level = [0] * len(sched) + [1, 2, 3]
    level_spread = [0, 0, 0, 0, 1, 1, 1, 2, 2, 3, 3]
    return {"sources": sources, "y": y, "nu": nu, "target_levels": list(target_levels),
            "eps": eps, "level": level, "eps_spread": sched, "level_spread": level_spread,
            "name": f"disk{rings}r_L{levels}_nq{sources[-1][0].shape[0]}_n{n_targets}"}


def mlp_init_params(seed: int = 0) -> np.ndarray:
    """Seeded initial parameters of the 6-256x4-1 warm-start network, flat
    FP32 in the library's order (W0[6][256] b0 W1[256][256] b1 W2 b2 W3 b3
    W4[256] b4): every weight and bias ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in))."""
    rng = np.random.default_rng(seed)
    blocks = []
    for fan_in, fan_out in [(6, 256), (256, 256), (256, 256), (256, 256), (256, 1)]:
        a = 1.0 / np.sqrt(fan_in)
        blocks.append(rng.uniform(-a, a, size=fan_in * fan_out))
        blocks.append(rng.uniform(-a, a, size=fan_out))
    return np.concatenate(blocks).astype(np.float32)
