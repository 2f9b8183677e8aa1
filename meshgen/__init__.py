"""Seeded synthetic inputs for the BDDC library and its CPU oracle.

This module builds the *problem data* only: structured Q1 hexahedral meshes of
the unit cube, partitions of the elements into substructures, per-element
material coefficients, Dirichlet flags and the consistent nodal load vector of
a constant body force.  It holds none of the BDDC method's arithmetic (no
element matrices, no interface classification, no constraints, no solves);
both the GPU library and the oracle under ``oracle/`` read these arrays and do
every step of the method on their own.

Conventions shared by every consumer:

* node ``(i, j, k)`` of an ``nx x ny x nz`` element grid has id
  ``i + (nx + 1) * (j + (ny + 1) * k)`` (x fastest);
* ``hex8`` rows list an element's nodes in the order
  (0,0,0) (1,0,0) (1,1,0) (0,1,0) (0,0,1) (1,0,1) (1,1,1) (0,1,1);
* degrees of freedom are node-major, component-minor: dof ``dpn * node + c``;
* the *global* numbering used by the solver skips Dirichlet dofs, keeping the
  node-major order of the rest (``Problem.free_dofs``).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

POISSON = 0
ELASTICITY = 1

# local node offsets of a hexahedron, in hex8 order
HEX_OFFSETS = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                        [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=np.int64)


@dataclass
class Problem:
    name: str
    kind: int                      # POISSON or ELASTICITY
    nel: tuple                     # elements per side (nx, ny, nz)
    xyz: np.ndarray                # (n_nodes, 3) float64 node coordinates
    hex8: np.ndarray               # (n_elems, 8) int64 connectivity
    coef: np.ndarray               # (n_elems,) float64: k (Poisson) or E (elasticity)
    nu: float                      # Poisson ratio (elasticity only)
    elem_sub: np.ndarray           # (n_elems,) int32 substructure of each element
    n_sub: int
    dirichlet: np.ndarray          # (n_nodes * dpn,) uint8, 1 = dof fixed to zero
    load: np.ndarray               # (n_nodes * dpn,) float64 nodal loads
    meta: dict = field(default_factory=dict)

    @property
    def dpn(self) -> int:
        return 1 if self.kind == POISSON else 3

    @property
    def n_nodes(self) -> int:
        return self.xyz.shape[0]

    @property
    def n_elems(self) -> int:
        return self.hex8.shape[0]

    @property
    def free_dofs(self) -> np.ndarray:
        """Full dof ids (dpn*node + c) of the non-Dirichlet dofs, ascending."""
        return np.flatnonzero(self.dirichlet == 0).astype(np.int64)

    @property
    def n_glob(self) -> int:
        return int(np.count_nonzero(self.dirichlet == 0))

    @property
    def f(self) -> np.ndarray:
        """Right-hand side in the global (Dirichlet-free) numbering."""
        return np.ascontiguousarray(self.load[self.free_dofs])


# ----------------------------------------------------------------------------
# mesh, partitions, coefficient fields
# ----------------------------------------------------------------------------

def grid_mesh(nx: int, ny: int, nz: int):
    """Uniform hexahedral grid of the unit cube: (xyz, hex8, h)."""
    i, j, k = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1),
                          indexing="ij")
    ids = (i + (nx + 1) * (j + (ny + 1) * k))
    n_nodes = (nx + 1) * (ny + 1) * (nz + 1)
    xyz = np.zeros((n_nodes, 3))
    xyz[ids.ravel(), 0] = i.ravel() / nx
    xyz[ids.ravel(), 1] = j.ravel() / ny
    xyz[ids.ravel(), 2] = k.ravel() / nz
    ei, ej, ek = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    # element id: x fastest, like the nodes
    eid = ei + nx * (ej + ny * ek)
    order = np.argsort(eid.ravel())
    ei, ej, ek = ei.ravel()[order], ej.ravel()[order], ek.ravel()[order]
    hex8 = np.empty((nx * ny * nz, 8), dtype=np.int64)
    for a, (dx, dy, dz) in enumerate(HEX_OFFSETS):
        hex8[:, a] = (ei + dx) + (nx + 1) * ((ej + dy) + (ny + 1) * (ek + dz))
    return xyz, hex8


def element_grid_index(nel):
    nx, ny, nz = nel
    e = np.arange(nx * ny * nz)
    return e % nx, (e // nx) % ny, e // (nx * ny)


def partition_blocks(nel, nsub):
    """Cubic-block partition: ``nsub = (sx, sy, sz)`` equal blocks of elements."""
    ex, ey, ez = element_grid_index(nel)
    sx, sy, sz = nsub
    bx, by, bz = nel[0] // sx, nel[1] // sy, nel[2] // sz
    assert bx * sx == nel[0] and by * sy == nel[1] and bz * sz == nel[2]
    return ((ex // bx) + sx * ((ey // by) + sy * (ez // bz))).astype(np.int32)


def partition_kmeans(xyz, hex8, k: int, seed: int, lloyd_iters: int = 1):
    """k-means on element centroids: k-means++ seeding from ``default_rng(seed)``
    followed by ``lloyd_iters`` Lloyd iterations.  Empty clusters cannot occur
    after seeding (every seed is an element centroid that is its own nearest
    centre); ids are renumbered by increasing centre (z, y, x) for stability."""
    rng = np.random.default_rng(seed)
    c = xyz[hex8].mean(axis=1)
    n = c.shape[0]
    centres = np.empty((k, 3))
    centres[0] = c[rng.integers(n)]
    d2 = ((c - centres[0]) ** 2).sum(1)
    for m in range(1, k):
        p = d2 / d2.sum()
        centres[m] = c[rng.choice(n, p=p)]
        d2 = np.minimum(d2, ((c - centres[m]) ** 2).sum(1))

    def assign(cent):
        best = np.full(n, np.inf)
        lab = np.zeros(n, dtype=np.int64)
        for m in range(k):
            dm = ((c - cent[m]) ** 2).sum(1)
            better = dm < best
            best[better] = dm[better]
            lab[better] = m
        return lab

    lab = assign(centres)
    for _ in range(lloyd_iters):
        for m in range(k):
            sel = lab == m
            if sel.any():
                centres[m] = c[sel].mean(0)
        lab = assign(centres)
    used = np.unique(lab)
    cz = centres[used]
    order = np.lexsort((cz[:, 0], cz[:, 1], cz[:, 2]))
    remap = np.empty(k, dtype=np.int64)
    remap[used[order]] = np.arange(len(used))
    return remap[lab].astype(np.int32), len(used)


def coef_layers(nel, rng_seed: int, values=(1.0, 1e6), p: float = 0.5):
    """One coefficient per horizontal element layer (constant z): ``values[1]``
    with probability ``p`` from ``default_rng(rng_seed)``, else ``values[0]``."""
    rng = np.random.default_rng(rng_seed)
    stiff = rng.random(nel[2]) < p
    layer_val = np.where(stiff, values[1], values[0])
    _, _, ez = element_grid_index(nel)
    return layer_val[ez].astype(np.float64)


def coef_inclusions(n_elems: int, rng_seed: int, frac: float = 0.05,
                    base: float = 1.0, stiff: float = 1e5):
    """Exactly ``round(frac * n_elems)`` elements, drawn without replacement by
    ``default_rng(rng_seed)``, get ``stiff``; the rest ``base``."""
    rng = np.random.default_rng(rng_seed)
    m = int(round(frac * n_elems))
    coef = np.full(n_elems, base)
    coef[rng.choice(n_elems, size=m, replace=False)] = stiff
    return coef


def _face_nodes(xyz, axis: int, value: float):
    return np.flatnonzero(np.abs(xyz[:, axis] - value) < 1e-12)


def nodal_body_load(xyz, hex8, dpn: int, force):
    """Consistent nodal load of a constant body force on affine cube elements:
    each trilinear shape function integrates to vol/8 over its element."""
    n_nodes = xyz.shape[0]
    x0 = xyz[hex8[:, 0]]
    x6 = xyz[hex8[:, 6]]
    vol = np.prod(x6 - x0, axis=1)
    w = np.zeros(n_nodes)
    np.add.at(w, hex8.ravel(), np.repeat(vol / 8.0, 8))
    load = np.zeros(n_nodes * dpn)
    for c in range(dpn):
        load[c::dpn] = w * force[c]
    return load


def cube_problem(kind: int, nel, nsub=None, *, elem_sub=None, n_sub=None,
                 coef=None, nu: float = 0.3, dirichlet_face=("x", 0.0),
                 force=None, name: str = "cube") -> Problem:
    """Generic unit-cube problem.  ``dirichlet_face`` is (axis, value) of the
    face on which every dof is fixed, or None (floating, e.g. the structure
    counting fixtures)."""
    if isinstance(nel, int):
        nel = (nel, nel, nel)
    xyz, hex8 = grid_mesh(*nel)
    dpn = 1 if kind == POISSON else 3
    if elem_sub is None:
        if isinstance(nsub, int):
            nsub = (nsub, nsub, nsub)
        elem_sub = partition_blocks(nel, nsub)
        n_sub = int(np.prod(nsub))
    if coef is None:
        coef = np.ones(hex8.shape[0])
    dirichlet = np.zeros(xyz.shape[0] * dpn, dtype=np.uint8)
    if dirichlet_face is not None:
        axis = {"x": 0, "y": 1, "z": 2}[dirichlet_face[0]]
        nodes = _face_nodes(xyz, axis, dirichlet_face[1])
        for c in range(dpn):
            dirichlet[dpn * nodes + c] = 1
    if force is None:
        force = (1.0,) if kind == POISSON else (0.0, 0.0, -1.0)
    load = nodal_body_load(xyz, hex8, dpn, force)
    return Problem(name=name, kind=kind, nel=tuple(nel), xyz=xyz, hex8=hex8,
                   coef=np.asarray(coef, dtype=np.float64), nu=float(nu),
                   elem_sub=np.asarray(elem_sub, dtype=np.int32), n_sub=int(n_sub),
                   dirichlet=dirichlet, load=load)


# ----------------------------------------------------------------------------
# the benchmark workloads
# ----------------------------------------------------------------------------

def poisson_16():
    """Scalar Poisson, 16^3 Q1 elements, 2x2x2 cubic substructures of 8^3,
    k = 1, f = 1, u = 0 on the face x = 0."""
    return cube_problem(POISSON, 16, 2, dirichlet_face=("x", 0.0), name="poisson16_2x2x2")


def elasticity_layers_48(seed: int = 2):
    """Linear elasticity, 48^3 Q1 elements, 4x4x4 cubic substructures of 12^3;
    E per horizontal layer in {1, 1e6} (p = 0.5 each, default_rng(seed)),
    nu = 0.3, clamped at z = 0, gravity (0, 0, -1) per unit volume."""
    nel = (48, 48, 48)
    coef = coef_layers(nel, seed)
    p = cube_problem(ELASTICITY, nel, 4, coef=coef, nu=0.3, dirichlet_face=("z", 0.0),
                     name="elasticity48_4x4x4_layers")
    p.meta.update(tau=10.0)
    return p


def elasticity_kmeans_64(seed_part: int = 0, seed_coef: int = 3, n_sub: int = 64):
    """Linear elasticity, 64^3 Q1 elements, 64 k-means substructures (k-means++
    from default_rng(seed_part), one Lloyd step), E = 1 with exactly 5% of the
    elements (default_rng(seed_coef)) at E = 1e5, nu = 0.3, clamped at z = 0,
    gravity."""
    nel = (64, 64, 64)
    xyz, hex8 = grid_mesh(*nel)
    elem_sub, k = partition_kmeans(xyz, hex8, n_sub, seed_part)
    coef = coef_inclusions(hex8.shape[0], seed_coef)
    p = cube_problem(ELASTICITY, nel, elem_sub=elem_sub, n_sub=k, coef=coef, nu=0.3,
                     dirichlet_face=("z", 0.0), name="elasticity64_kmeans64_inclusions")
    p.meta.update(tau=10.0)
    return p


def small_elasticity_layers(n: int = 8, s: int = 2, seed: int = 2, contrast: float = 1e6):
    """A scaled-down copy of the layered elasticity workload for fast tests."""
    nel = (n, n, n)
    coef = coef_layers(nel, seed, values=(1.0, contrast))
    return cube_problem(ELASTICITY, nel, s, coef=coef, nu=0.3, dirichlet_face=("z", 0.0),
                        name=f"elasticity{n}_{s}x{s}x{s}_layers")


def small_kmeans(kind: int, n: int, k: int, seed_part: int = 0, seed_coef: int = 3,
                 contrast: float = 1e5):
    nel = (n, n, n)
    xyz, hex8 = grid_mesh(*nel)
    elem_sub, kk = partition_kmeans(xyz, hex8, k, seed_part)
    coef = coef_inclusions(hex8.shape[0], seed_coef, stiff=contrast)
    return cube_problem(kind, nel, elem_sub=elem_sub, n_sub=kk, coef=coef, nu=0.3,
                        dirichlet_face=("z", 0.0), name=f"kmeans{n}_{kk}")


def planar_cubes(k: int, H: int = 8):
    """k x k cubic substructures of H^3 elasticity elements side by side in one
    layer: the domain [0, k] x [0, k] x [0, 1] with elements of size 1/H,
    E = 1, nu = 0.3, every dof clamped on the face x = 0 and a unit downward
    traction on the opposite face x = k (consistent nodal loads of the
    bilinear face elements).  The material and the load are stand-ins: the
    weak-scaling experiment fixes one side and loads the opposite one without
    stating either."""
    nel = (H * k, H * k, H)
    xyz, hex8 = grid_mesh(*nel)
    xyz[:, 0] *= k
    xyz[:, 1] *= k
    elem_sub = partition_blocks(nel, (k, k, 1))
    dpn = 3
    dirichlet = np.zeros(xyz.shape[0] * dpn, dtype=np.uint8)
    for c in range(dpn):
        dirichlet[dpn * _face_nodes(xyz, 0, 0.0) + c] = 1
    # loaded face x = k: an (ny + 1) x (nz + 1) node grid of squares of side
    # h; each node carries h^2/4 per square it touches
    h = 1.0 / H
    nodes = _face_nodes(xyz, 0, float(k))
    j = np.rint(xyz[nodes, 1] * H).astype(np.int64)
    kk = np.rint(xyz[nodes, 2] * H).astype(np.int64)
    wy = np.where((j == 0) | (j == nel[1]), 0.5 * h, h)
    wz = np.where((kk == 0) | (kk == nel[2]), 0.5 * h, h)
    load = np.zeros(xyz.shape[0] * dpn)
    load[dpn * nodes + 2] = -wy * wz
    return Problem(name=f"planar_cubes_{k}x{k}_H{H}", kind=ELASTICITY, nel=nel, xyz=xyz,
                   hex8=hex8, coef=np.ones(hex8.shape[0]), nu=0.3, elem_sub=elem_sub,
                   n_sub=k * k, dirichlet=dirichlet, load=load)


def serving_requests(n_req: int = 512, seed: int = 5):
    """Request stream: type (Poisson/elasticity, p = 0.5), elements per side
    n in {16,24,32,40,48}, substructures per side s in {2,3,4} with n % s == 0,
    layered contrast 10^U{0..6}.  Returns a list of dicts; arrival times are
    assigned by the caller from a rate."""
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(n_req):
        kind = ELASTICITY if rng.random() < 0.5 else POISSON
        n = int(rng.choice([16, 24, 32, 40, 48]))
        ss = [s for s in (2, 3, 4) if n % s == 0]
        s = int(rng.choice(ss))
        contrast = float(10.0 ** rng.integers(0, 7))
        layer_seed = int(rng.integers(0, 2**31 - 1))
        reqs.append(dict(id=r, kind=kind, n=n, s=s, contrast=contrast, seed=layer_seed))
    return reqs


def request_problem(req) -> Problem:
    nel = (req["n"],) * 3
    coef = coef_layers(nel, req["seed"], values=(1.0, req["contrast"]))
    face = ("z", 0.0) if req["kind"] == ELASTICITY else ("x", 0.0)
    return cube_problem(req["kind"], nel, req["s"], coef=coef, nu=0.3, dirichlet_face=face,
                        name=f"req{req['id']}")


def random_vector(n: int, seed: int) -> np.ndarray:
    """Seeded standard-normal test vector."""
    return np.random.default_rng(seed).standard_normal(n)
