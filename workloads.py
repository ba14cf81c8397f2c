"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds the *inputs* of the method and nothing of its arithmetic:
tetrahedral meshes of a cuboid (vertex coordinates and element-to-vertex
lists), cellwise materials, initial-pressure functions evaluated at given
points, source positions and wavelet parameters, random states of given
shapes, and the named workload configurations.  Nodes, operators, geometric
factors, connectivity, HABC coefficients and the time step of the method are
computed separately by the oracle and by the library.

The workloads stand in for the paper's validation and SEAM benchmarks
(Section 4): the paper's meshes and the SEAM model are not available, so
structured Kuhn meshes of the unit cube with synthetic layered media are used,
with the polynomial degrees and HABC orders the paper uses.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# The six tetrahedra of the Kuhn (Freudenthal) split of a cube: tet sigma is
# {x : x_sigma0 >= x_sigma1 >= x_sigma2} in local cell coordinates.
_PERMS = list(itertools.permutations(range(3)))


def _perm_sign(p):
    s = 1
    p = list(p)
    for i in range(len(p)):
        for j in range(i + 1, len(p)):
            if p[i] > p[j]:
                s = -s
    return s


def kuhn_mesh(n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), dims=None):
    """Kuhn mesh of the box [lo, hi] with n^3 hexahedral cells x 6 tets.

    Returns (VX, EToV): VX float64 (Nv, 3), EToV int32 (K, 4).
    Vertex (i, j, k) has index (k*(ny+1) + j)*(nx+1) + i; element
    ((k*ny + j)*nx + i)*6 + t is tet t of cell (i, j, k).  Every tet is
    positively oriented.  ``dims`` = (nx, ny, nz) overrides n.
    """
    nx, ny, nz = dims if dims is not None else (n, n, n)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    xs = [lo[a] + (hi[a] - lo[a]) * np.arange(m + 1) / m for a, m in enumerate((nx, ny, nz))]
    X, Y, Z = np.meshgrid(xs[0], xs[1], xs[2], indexing="ij")
    VX = np.stack([X.transpose(2, 1, 0).ravel(), Y.transpose(2, 1, 0).ravel(),
                   Z.transpose(2, 1, 0).ravel()], axis=1)

    def vid(i, j, k):
        return (k * (ny + 1) + j) * (nx + 1) + i

    local = []
    for p in _PERMS:
        path = [np.zeros(3, dtype=int)]
        cur = np.zeros(3, dtype=int)
        for a in p:
            cur = cur.copy()
            cur[a] = 1
            path.append(cur)
        if _perm_sign(p) < 0:
            path[2], path[3] = path[3], path[2]
        local.append(path)

    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ii = ii.transpose(2, 1, 0).ravel()
    jj = jj.transpose(2, 1, 0).ravel()
    kk = kk.transpose(2, 1, 0).ravel()
    ncell = ii.size
    EToV = np.empty((ncell, 6, 4), dtype=np.int64)
    for t, path in enumerate(local):
        for v, off in enumerate(path):
            EToV[:, t, v] = vid(ii + off[0], jj + off[1], kk + off[2])
    return VX, EToV.reshape(ncell * 6, 4).astype(np.int32)


def general_mesh(n, amp=0.1, seed=0, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """An unstructured tetrahedral mesh of the box: the Kuhn mesh of n^3
    cells with every interior vertex moved by U(-amp, amp) * h per
    coordinate, the elements listed in a random order, and each element's
    vertices rotated by a random even permutation (orientation kept).
    Vertices on the boundary stay on the boundary grid, so the boundary
    faces, edges and corners are those of the Kuhn mesh.  Returns (VX, EToV)
    as ``kuhn_mesh`` does."""
    VX, E = kuhn_mesh(n, lo=lo, hi=hi)
    rng = np.random.default_rng(seed)
    lo_, hi_ = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
    h = (hi_ - lo_) / n
    tol = 1e-9 * h
    inner = np.all((VX > lo_ + tol) & (VX < hi_ - tol), axis=1)
    VX = VX.copy()
    VX[inner] += rng.uniform(-amp, amp, size=(int(inner.sum()), 3)) * h
    even = [p for p in itertools.permutations(range(4)) if _perm_sign(p) > 0]
    pick = rng.integers(0, len(even), size=E.shape[0])
    E = np.stack([E[k, list(even[pick[k]])] for k in range(E.shape[0])])
    E = E[rng.permutation(E.shape[0])]
    return VX, np.ascontiguousarray(E, dtype=np.int32)


def mirror_doubled_mesh(VX, EToV, axis=2, plane=None):
    """The mesh together with its mirror image in the plane x_axis = plane
    (default: the mesh's largest coordinate on that axis): vertices on the
    plane are shared, mirrored elements have two vertices swapped so that
    every element stays positively oriented.  Returns (VX2, EToV2, img):
    the first K elements are the given ones in order, element K + k is the
    image of element k, and img[v] is the vertex id of the image of
    vertex v."""
    VX = np.asarray(VX, dtype=np.float64)
    EToV = np.asarray(EToV, dtype=np.int64)
    if plane is None:
        plane = float(VX[:, axis].max())
    on = np.abs(VX[:, axis] - plane) <= 1e-12 * max(1.0, abs(plane))
    img = np.empty(VX.shape[0], dtype=np.int64)
    img[on] = np.nonzero(on)[0]
    off = np.nonzero(~on)[0]
    img[off] = VX.shape[0] + np.arange(off.size)
    VXm = VX[off].copy()
    VXm[:, axis] = 2.0 * plane - VXm[:, axis]
    Em = img[EToV][:, [0, 1, 3, 2]]
    return (np.concatenate([VX, VXm]), np.concatenate([EToV, Em]).astype(np.int32), img)


def cell_index_of_element(n, dims=None):
    """(i, j, k) cell indices of every element of ``kuhn_mesh``."""
    nx, ny, nz = dims if dims is not None else (n, n, n)
    e = np.arange(nx * ny * nz * 6)
    c = e // 6
    return c % nx, (c // nx) % ny, c // (nx * ny)


def layered_medium(n, seed=2, n_layers=5, c_range=(1.0, 3.0), rho_range=(1.0, 2.5),
                   dims=None, layer_of_k=None):
    """Horizontal layers snapped to cell planes; returns (rho, c) per element.

    Interfaces sit at ``n_layers - 1`` distinct cell planes k = m, m drawn
    without replacement from 1..nz-1; for each layer (bottom to top) the wave
    speed c ~ U(c_range) is drawn, then the density rho ~ U(rho_range).
    ``layer_of_k`` may map cell layers of an enlarged mesh onto these layers.
    """
    nx, ny, nz = dims if dims is not None else (n, n, n)
    rng = np.random.default_rng(seed)
    cuts = np.sort(rng.choice(np.arange(1, nz), size=n_layers - 1, replace=False))
    cvals = np.empty(n_layers)
    rvals = np.empty(n_layers)
    for L in range(n_layers):
        cvals[L] = rng.uniform(*c_range)
        rvals[L] = rng.uniform(*rho_range)
    _, _, k = cell_index_of_element(n, dims)
    if layer_of_k is None:
        layer = np.searchsorted(cuts, k, side="right")
    else:
        layer = layer_of_k(k, cuts)
    return rvals[layer].copy(), cvals[layer].copy(), cuts, cvals, rvals


def gaussian_pulse(x, center, width):
    """exp(-|x - center|^2 / width^2) at points x (..., 3)."""
    d = np.asarray(x) - np.asarray(center)
    return np.exp(-np.sum(d * d, axis=-1) / width ** 2)


def random_array(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def kuhn_dt(n, N, c_max, cfl=0.5, L=1.0):
    """Time step CFL * min_k 1/(c_k (N+1)^2 F_k) of the validation benchmark
    (Section 4.1, time-step rule, read with a minimum over cells) for a Kuhn
    mesh: every tet has F = max face area / volume * 2/3 = 2*sqrt(2)/h."""
    h = L / n
    F = 2.0 * math.sqrt(2.0) / h
    return cfl / (c_max * (N + 1) ** 2 * F)


def n_unknowns(K_tet, K_tri, K_lin, N, P):
    """Unknown count of the implementation table: sum over levels of
    K * N_sets * N_fields * Np (3D: 1 set of 4 fields; 2D: P sets of 3;
    1D: P^2 sets of 2)."""
    Np3 = (N + 1) * (N + 2) * (N + 3) // 6
    Np2 = (N + 1) * (N + 2) // 2
    Np1 = N + 1
    return K_tet * 4 * Np3 + K_tri * P * 3 * Np2 + K_lin * P * P * 2 * Np1


@dataclass
class Workload:
    name: str
    n: int
    N: int
    P: int
    steps: int
    dt: float
    medium: str = "homogeneous"        # or "layered"
    init: str = "gaussian"             # "gaussian" | "random" | "zero"
    source: tuple | None = None        # (x, y, z) point source position
    f0: float = 0.0
    t0: float = 0.0
    seed: int = 0
    periodic: tuple = (False, False, False)
    extra: dict = field(default_factory=dict)

    def mesh(self):
        return kuhn_mesh(self.n)

    def materials(self):
        K = 6 * self.n ** 3
        if self.medium == "layered":
            rho, c, *_ = layered_medium(self.n, seed=self.extra.get("medium_seed", 2))
            return rho, c
        return np.ones(K), np.ones(K)


def config(name):
    """Named workloads.  '1': FP64 parity case (8^3 x 6 tets, N=3, P=3,
    centred Gaussian of width 0.05, 100 steps); '1b': same, 1000 steps (the
    wave reaches faces, edges and corners); '1c': same mesh, every state array
    random (seed 11), 100 steps; '2': 40^3 x 6 tets, N=4, P=6, five random
    layers, Ricker point source near the centre, 1000 steps; '3': the
    precision case, config 1's mesh and pulse at N=5, 1000 steps."""
    if name == "3":
        n, N, P = 8, 5, 3
        return Workload(name=name, n=n, N=N, P=P, steps=1000, dt=kuhn_dt(n, N, 1.0),
                        init="gaussian", seed=0,
                        extra={"center": (0.5, 0.5, 0.5), "width": 0.05})
    if name in ("1", "1b", "1c"):
        n, N, P = 8, 3, 3
        dt = kuhn_dt(n, N, 1.0)
        steps = {"1": 100, "1b": 1000, "1c": 100}[name]
        init = "random" if name == "1c" else "gaussian"
        return Workload(name=name, n=n, N=N, P=P, steps=steps, dt=dt, init=init,
                        seed=11 if name == "1c" else 0,
                        extra={"center": (0.5, 0.5, 0.5), "width": 0.05})
    if name == "2":
        n, N, P = 40, 4, 6
        h = 1.0 / n
        rho, c, *_ = layered_medium(n, seed=2)
        xs = (0.5 + 0.3 * h, 0.5 + 0.2 * h, 0.5 + 0.1 * h)
        cs = float(source_material(n, xs, c))
        f0 = cs / (10.0 * h)
        dt = kuhn_dt(n, N, float(c.max()))
        return Workload(name=name, n=n, N=N, P=P, steps=1000, dt=dt, medium="layered",
                        init="zero", source=xs, f0=f0, t0=1.25 / f0,
                        extra={"medium_seed": 2})
    raise KeyError(name)


def source_material(n, xs, values):
    """Value of a cellwise quantity in the hex cell containing xs (unit cube)."""
    i, j, k = (min(int(math.floor(v * n)), n - 1) for v in xs)
    e = ((k * n + j) * n + i) * 6
    return values[e]


def shot_positions(n_shots, seed=4, lo=0.2, hi=0.8):
    """Random interior source positions of the many-shot workload."""
    return np.random.default_rng(seed).uniform(lo, hi, size=(n_shots, 3))
