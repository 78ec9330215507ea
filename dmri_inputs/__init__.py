"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *generates* inputs: periodic structured tetrahedral meshes,
compartment labels from simple shapes, gradient directions, b-value lists and
the sequence timing. It contains none of the simulation method's arithmetic
(no element integrals, no time stepping, no signal), so the CPU oracle and the
GPU library can both consume its arrays without sharing any solver code.

Units follow the paper's code: micrometres and microseconds, so D is in
um^2/us (== mm^2/s), b in us/um^2 (== s/mm^2) and kappa in um/us (== m/s).

The meshes stand in for the paper's GMSH/Salome conforming meshes of cells,
neurons and extracellular space (Sec. 4 and 5), which are not available: each
box is split into n^3 cubes and each cube into the six Kuhn (Freudenthal)
tetrahedra sharing its main diagonal. The split is translation invariant, so
opposite box faces match node for node, which the strong (periodic) imposition
of the pseudo-periodic conditions needs (Appendix A).
"""

from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Problem",
    "Sequence",
    "GeneralSequence",
    "Systems",
    "kuhn_box_mesh",
    "label_tets",
    "fibonacci_directions",
    "free_diffusion_10",
    "cylinder_36",
    "cylinder_57_batched",
    "seeded_cells",
    "seeded_cells_78",
    "cylinder_box",
    "conforming_cylinder_box",
    "tensor",
    "slab_box",
    "free_box",
    "nonmatching_faces",
]

# Ordered vertex paths of the 6 Kuhn tetrahedra in a unit cube: start at the
# cube's (0,0,0) corner and add the unit vectors in the order of a permutation.
_PERMS = list(itertools.permutations(range(3)))


@dataclass
class Problem:
    """One mesh with its compartments, as handed to a solver."""

    xyz: np.ndarray                 # [n_nodes, 3] float64, um
    tets: np.ndarray                # [n_tets, 4] int32, 0-based node ids
    tet_label: np.ndarray           # [n_tets] int32 in [0, n_comp)
    n_comp: int
    D: np.ndarray                   # [n_comp] um^2/us, or [n_comp, 3, 3] tensors
    T2: Optional[np.ndarray]        # [n_comp] us, None = infinite
    u0: Optional[np.ndarray]        # [n_comp], None = 1 everywhere
    kappa: float                    # um/us on every interface
    box_lo: np.ndarray              # [3]
    box_hi: np.ndarray              # [3]
    periodic_mask: int              # bit a set = periodic along axis a
    n_cells: int = 0                # cubes per side (structured meshes)
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])


@dataclass
class Sequence:
    """PGSE timing: pulse length delta, pulse spacing Delta, step dt, theta."""

    delta: float
    Delta: float
    dt: float
    theta: float = 0.5

    @property
    def T(self) -> float:
        # Echo time at the end of the second pulse.
        return self.Delta + self.delta

    @property
    def n_steps(self) -> int:
        return int(round(self.T / self.dt))


@dataclass
class GeneralSequence:
    """A named temporal profile with its parameters (us), step dt and theta.

    kind: "pgse" (delta, Delta), "double_pgse" (delta, Delta, t_mix),
    "cos_ogse" / "sin_ogse" (delta, Delta, n_periods), "trap_pgse"
    (delta, Delta, ramp), "double_trap_pgse" (delta, Delta, ramp, t_mix).
    Only the description: the profile itself (f, F, echo time) is evaluated
    by whoever consumes it.
    """

    kind: str
    params: tuple
    dt: float
    theta: float = 0.5


@dataclass
class Systems:
    """A list of (b, direction) pairs, all on one problem."""

    b: np.ndarray                   # [n] us/um^2
    q: np.ndarray                   # [n, 3] (normalised)

    def __len__(self) -> int:
        return int(self.b.shape[0])


# ---------------------------------------------------------------------------
# Mesh generation
# ---------------------------------------------------------------------------

def kuhn_box_mesh(lo: Sequence[float], hi: Sequence[float], n):
    """Structured tetrahedral mesh of the box [lo, hi] with n cubes per side.

    n is an int or a triple (nx, ny, nz). Returns (xyz [n_nodes, 3] float64,
    tets [6 nx ny nz, 4] int32, cube [6 nx ny nz] int64). Node (i, j, l) has
    id i + (nx+1) j + (nx+1)(ny+1) l. Every tetrahedron is positively oriented.
    """
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    nv = np.broadcast_to(np.asarray(n, dtype=np.int64), (3,)).copy()
    if np.any(nv < 1):
        raise ValueError("n must be >= 1")
    mx, my, mz = (int(v) + 1 for v in nv)
    ax = [lo[a] + (hi[a] - lo[a]) * np.arange(nv[a] + 1, dtype=np.float64) / nv[a]
          for a in range(3)]
    # Exact endpoints so opposite faces match bit for bit.
    for a in range(3):
        ax[a][0] = lo[a]
        ax[a][-1] = hi[a]
    I, J, L = np.meshgrid(np.arange(mx), np.arange(my), np.arange(mz), indexing="ij")
    nid = lambda i, j, l: i + mx * j + mx * my * l  # noqa: E731
    xyz = np.empty((mx * my * mz, 3), dtype=np.float64)
    ids = nid(I, J, L).ravel()
    xyz[ids, 0] = ax[0][I.ravel()]
    xyz[ids, 1] = ax[1][J.ravel()]
    xyz[ids, 2] = ax[2][L.ravel()]

    ci, cj, cl = np.meshgrid(np.arange(nv[0]), np.arange(nv[1]), np.arange(nv[2]),
                             indexing="ij")
    ci, cj, cl = ci.ravel(), cj.ravel(), cl.ravel()
    cube_id = ci + nv[0] * cj + nv[0] * nv[1] * cl
    tets = []
    cubes = []
    for perm in _PERMS:
        off = np.zeros(3, dtype=np.int64)
        verts = [nid(ci, cj, cl)]
        for a in perm:
            off[a] += 1
            verts.append(nid(ci + off[0], cj + off[1], cl + off[2]))
        t = np.stack(verts, axis=1)
        # The sign of the permutation decides the orientation of the path.
        inv = sum(1 for x in range(3) for y in range(x + 1, 3) if perm[x] > perm[y])
        if inv % 2 == 1:
            t = t[:, [0, 2, 1, 3]]
        tets.append(t)
        cubes.append(cube_id)
    # Group the 6 tets of a cube together (cube-major order).
    tets = np.stack(tets, axis=1).reshape(-1, 4)
    cubes = np.stack(cubes, axis=1).reshape(-1)
    return xyz, tets.astype(np.int32), cubes.astype(np.int64)


def _inside(points: np.ndarray, shapes: List[dict]) -> np.ndarray:
    """Index+1 of the first shape containing each point, 0 if none."""
    lab = np.zeros(points.shape[0], dtype=np.int32)
    for k, s in enumerate(shapes):
        if s["kind"] == "cylz":
            d2 = (points[:, 0] - s["c"][0]) ** 2 + (points[:, 1] - s["c"][1]) ** 2
        elif s["kind"] == "sphere":
            d2 = ((points - np.asarray(s["c"])) ** 2).sum(axis=1)
        elif s["kind"] == "slabx":
            # Half-open slab lo <= x < hi.
            inside = (points[:, 0] >= s["lo"]) & (points[:, 0] < s["hi"])
            lab[(lab == 0) & inside] = k + 1
            continue
        else:
            raise ValueError(s["kind"])
        inside = d2 < s["r"] ** 2
        lab[(lab == 0) & inside] = k + 1
    return lab


def label_tets(xyz, tets, shapes, mode="centroid", n_cells=None, lo=None, hi=None,
               shape_labels=None):
    """Compartment label per tetrahedron from a list of shapes.

    mode="centroid": a tet belongs to the first shape containing its centroid.
    mode="cube": all six tets of a cube take the label of the cube centre
    (a voxel staircase: every interface face is axis aligned).
    shape_labels maps shape index+1 -> label (default: every shape -> 1).
    """
    if mode == "centroid":
        pts = xyz[tets].mean(axis=1)
    elif mode == "cube":
        # Cube centre = midpoint of the Kuhn diagonal (vertices 0 and 3).
        pts = 0.5 * (xyz[tets[:, 0]] + xyz[tets[:, 3]])
    else:
        raise ValueError(mode)
    raw = _inside(pts, shapes)
    if shape_labels is None:
        return (raw > 0).astype(np.int32)
    table = np.asarray([0] + list(shape_labels), dtype=np.int32)
    return table[raw]


def fibonacci_directions(n: int) -> np.ndarray:
    """n unit vectors of the spherical Fibonacci lattice (whole sphere)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

D_FREE = 3.0e-3  # um^2/us, the paper's default water diffusivity (Sec. 4)

PGSE_SHORT = Sequence(delta=10600.0, Delta=13400.0, dt=100.0, theta=0.5)


def free_box(n=10, half=5.0, D=D_FREE, periodic_mask=7):
    """Single compartment box [-half, half]^3 (free diffusion)."""
    xyz, tets, _ = kuhn_box_mesh([-half] * 3, [half] * 3, n)
    lab = np.zeros(tets.shape[0], dtype=np.int32)
    return Problem(xyz, tets, lab, 1, np.array([D]), None, None, 0.0,
                   np.array([-half] * 3), np.array([half] * 3), periodic_mask, n_cells=n,
                   meta={"name": "free_box", "n": n})


def cylinder_box(n=36, half=6.0, r=5.0, D_in=D_FREE, D_out=D_FREE, kappa=1e-5,
                 mode="centroid", T2=None, u0=None, periodic_mask=7):
    """Box [-half, half]^3 with a z-axis cylinder of radius r through (0,0).

    Label 1 inside the cylinder, 0 outside.
    """
    xyz, tets, _ = kuhn_box_mesh([-half] * 3, [half] * 3, n)
    shapes = [{"kind": "cylz", "c": (0.0, 0.0), "r": r}]
    lab = label_tets(xyz, tets, shapes, mode=mode)
    return Problem(xyz, tets, lab, 2, np.array([D_out, D_in], dtype=np.float64),
                   None if T2 is None else np.asarray(T2, dtype=np.float64),
                   None if u0 is None else np.asarray(u0, dtype=np.float64),
                   float(kappa), np.array([-half] * 3), np.array([half] * 3), periodic_mask,
                   n_cells=n, meta={"name": "cylinder_box", "n": n, "r": r, "mode": mode})


def tensor(eig, angles=(0.0, 0.0, 0.0)):
    """Symmetric positive definite 3x3 tensor with eigenvalues eig, rotated by
    Euler angles (z, y, z) in radians."""
    a, b, c = angles

    def rz(t):
        return np.array([[math.cos(t), -math.sin(t), 0.0], [math.sin(t), math.cos(t), 0.0],
                         [0.0, 0.0, 1.0]])

    def ry(t):
        return np.array([[math.cos(t), 0.0, math.sin(t)], [0.0, 1.0, 0.0],
                         [-math.sin(t), 0.0, math.cos(t)]])

    R = rz(a) @ ry(b) @ rz(c)
    return R @ np.diag(np.asarray(eig, dtype=np.float64)) @ R.T


def conforming_cylinder_box(n=12, half=6.0, r=4.0, D_in=D_FREE, D_out=D_FREE, kappa=1e-3,
                            jitter=0.15, seed=0, T2=None, u0=None, periodic_mask=7):
    """A z-cylinder in a box on an unstructured, interface-conforming mesh.

    Kuhn mesh of n^3 cubes; nodes within 0.4 h of the cylinder surface are
    moved radially onto it (the membrane becomes a faceted cylinder made of
    mesh faces, not a voxel staircase), then every other node strictly inside
    the box is moved by a seeded uniform displacement of up to jitter * h per
    coordinate (the mesh is no longer structured; box faces stay planar and
    periodic faces still match). Labels by tet centroid (1 inside). D_in /
    D_out: scalars or 3x3 tensors (then D has shape [2, 3, 3]).
    """
    xyz, tets, _ = kuhn_box_mesh([-half] * 3, [half] * 3, n)
    h = 2.0 * half / n
    rho = np.hypot(xyz[:, 0], xyz[:, 1])
    on_face = np.any(np.isclose(np.abs(xyz), half, rtol=0, atol=1e-12), axis=1)
    snap = (np.abs(rho - r) < 0.4 * h) & ~on_face & (rho > 0)
    xyz = xyz.copy()
    xyz[snap, 0] *= r / rho[snap]
    xyz[snap, 1] *= r / rho[snap]
    rng = np.random.default_rng(seed)
    move = ~on_face & ~snap
    xyz[move] += rng.uniform(-jitter * h, jitter * h, size=(int(move.sum()), 3))
    v = xyz[tets]
    vol = np.einsum("mi,mi->m", v[:, 1] - v[:, 0], np.cross(v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]))
    if np.any(vol <= 1e-6 * h ** 3):
        raise ValueError("mesh perturbation inverted a tetrahedron")
    shapes = [{"kind": "cylz", "c": (0.0, 0.0), "r": r}]
    lab = label_tets(xyz, tets, shapes, mode="centroid")
    Din, Dout = np.asarray(D_in, dtype=np.float64), np.asarray(D_out, dtype=np.float64)
    D = np.stack([Dout, Din]) if Din.ndim == 2 else np.array([float(Dout), float(Din)])
    return Problem(xyz, tets, lab, 2, D,
                   None if T2 is None else np.asarray(T2, dtype=np.float64),
                   None if u0 is None else np.asarray(u0, dtype=np.float64),
                   float(kappa), np.array([-half] * 3), np.array([half] * 3), periodic_mask,
                   n_cells=n, meta={"name": "conforming_cylinder_box", "n": n, "r": r,
                                    "jitter": jitter, "seed": seed, "snapped": int(snap.sum())})


def nonmatching_faces(prob: Problem, axes=(0, 1, 2), amount=0.25, seed=0) -> Problem:
    """Copy of prob whose faces x_a = hi_a (a in axes) no longer match the
    opposite faces node for node: every node inside such a face (not on its
    border) moves within the face plane by a seeded uniform displacement of
    up to amount * h per tangential coordinate (h = the mean edge length of
    the structured grid, box length / n_cells). For weak pseudo-periodic
    faces (non-matching meshes); the strong identification rejects it."""
    xyz = np.asarray(prob.xyz, dtype=np.float64).copy()
    lo, hi = np.asarray(prob.box_lo, dtype=np.float64), np.asarray(prob.box_hi, dtype=np.float64)
    rng = np.random.default_rng(seed)
    for a in axes:
        h = (hi[a] - lo[a]) / max(1, int(prob.n_cells))
        others = [b for b in range(3) if b != a]
        on = np.isclose(xyz[:, a], hi[a], rtol=0, atol=1e-12 * (hi[a] - lo[a]))
        for b in others:
            on &= ~np.isclose(xyz[:, b], lo[b], rtol=0, atol=1e-12) & \
                ~np.isclose(xyz[:, b], hi[b], rtol=0, atol=1e-12)
        for b in others:
            xyz[on, b] += rng.uniform(-amount * h, amount * h, size=int(on.sum()))
    v = xyz[np.asarray(prob.tets)]
    vol = np.einsum("mi,mi->m", v[:, 1] - v[:, 0], np.cross(v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]))
    v0 = np.asarray(prob.xyz)[np.asarray(prob.tets)]
    vol0 = np.einsum("mi,mi->m", v0[:, 1] - v0[:, 0],
                     np.cross(v0[:, 2] - v0[:, 0], v0[:, 3] - v0[:, 0]))
    if np.any(vol * vol0 <= 0) or np.any(np.abs(vol) < 1e-6 * np.abs(vol0)):
        raise ValueError("face perturbation inverted a tetrahedron")
    meta = dict(prob.meta)
    meta.update({"nonmatching_axes": tuple(axes), "face_amount": amount, "face_seed": seed})
    return Problem(xyz, prob.tets, prob.tet_label, prob.n_comp, prob.D, prob.T2, prob.u0,
                   prob.kappa, lo, hi, prob.periodic_mask, n_cells=prob.n_cells, meta=meta)


def slab_box(n=16, half=5.0, split=0.0, D=(D_FREE, D_FREE), kappa=0.0, u0=None,
             periodic_mask=0b110, T2=None, cross=None):
    """Box cut by the plane x = split into compartment 0 (x < split) and 1.

    With periodic_mask=0b110 the box is periodic in y and z and has walls
    (homogeneous Neumann) at x = +-half. cross=(width, cells) makes the y and
    z extent [0, width] with that many cells (a thin slab for 1-D tests).
    """
    if cross is None:
        lo, hi, nn = [-half] * 3, [half] * 3, n
    else:
        lo, hi, nn = [-half, 0.0, 0.0], [half, cross[0], cross[0]], (n, cross[1], cross[1])
    xyz, tets, _ = kuhn_box_mesh(lo, hi, nn)
    shapes = [{"kind": "slabx", "lo": split, "hi": np.inf}]
    lab = label_tets(xyz, tets, shapes, mode="cube")
    n_comp = 2
    if split <= -half or split >= half:
        lab[:] = 0
        n_comp = 1
        D = D[:1]
    return Problem(xyz, tets, lab, n_comp, np.asarray(D, dtype=np.float64),
                   None if T2 is None else np.asarray(T2, dtype=np.float64),
                   None if u0 is None else np.asarray(u0, dtype=np.float64),
                   float(kappa), np.asarray(lo, dtype=np.float64),
                   np.asarray(hi, dtype=np.float64), periodic_mask,
                   n_cells=n, meta={"name": "slab_box", "n": n, "split": split})


def free_diffusion_10():
    """Free diffusion in [-5,5]^3, 10 cubes per side, b=1000 along x."""
    prob = free_box(n=10, half=5.0)
    sysl = Systems(np.array([1000.0]), np.array([[1.0, 0.0, 0.0]]))
    return prob, PGSE_SHORT, sysl


def cylinder_36(n=36):
    """Cylinder r=5 in a 12 um box, kappa=1e-5, 8 b-values in [0,3000] along x."""
    prob = cylinder_box(n=n)
    b = np.linspace(0.0, 3000.0, 8)
    q = np.tile(np.array([[1.0, 0.0, 0.0]]), (8, 1))
    return prob, PGSE_SHORT, Systems(b, q)


def cylinder_57_batched(n=57, n_dir=64, n_b=16):
    """The cylinder_36 geometry refined to n=57; 64 Fibonacci directions x 16 b in [0,5000]."""
    prob = cylinder_box(n=n)
    dirs = fibonacci_directions(n_dir)
    bs = np.linspace(0.0, 5000.0, n_b)
    # Direction-major order: pair p = dir * n_b + b_index.
    b = np.tile(bs, n_dir)
    q = np.repeat(dirs, n_b, axis=0)
    return prob, PGSE_SHORT, Systems(b, q)


def _random_geometry(seed: int, n_fixed: Optional[int] = None, box=30.0):
    """Seeded cylinders/spheres in [0, box]^3 (the uneven-batch workload).

    Draw order from numpy.random.default_rng(seed): node target, kappa, shape
    count, then per placement attempt: kind, radius, centre.
    """
    rng = np.random.default_rng(seed)
    n_target = math.exp(rng.uniform(math.log(5e4), math.log(1e6)))
    n = int(round(n_target ** (1.0 / 3.0))) - 1
    if n_fixed is not None:
        n = int(n_fixed)
    kappa = math.exp(rng.uniform(math.log(1e-6), math.log(1e-4)))
    count = int(rng.integers(5, 31))
    h = box / n
    gap = 2.0 * h
    shapes: List[dict] = []
    fails = 0
    while len(shapes) < count and fails < 10000:
        kind = "cylz" if rng.uniform() < 0.5 else "sphere"
        r = rng.uniform(2.0, 6.0)
        if kind == "cylz":
            c = rng.uniform(r + gap, box - r - gap, size=2)
            cand = {"kind": "cylz", "c": (float(c[0]), float(c[1])), "r": float(r)}
        else:
            c = rng.uniform(r + gap, box - r - gap, size=3)
            cand = {"kind": "sphere", "c": tuple(float(v) for v in c), "r": float(r)}
        ok = True
        for s in shapes:
            if cand["kind"] == "cylz" or s["kind"] == "cylz":
                # A z-cylinder spans the box, so only the xy distance counts.
                d = math.hypot(cand["c"][0] - s["c"][0], cand["c"][1] - s["c"][1])
            else:
                d = math.dist(cand["c"], s["c"])
            if d < cand["r"] + s["r"] + gap:
                ok = False
                break
        if ok:
            shapes.append(cand)
        else:
            fails += 1
    return n, kappa, count, shapes, fails


def seeded_cells(seed: int, n_fixed: Optional[int] = None):
    """One geometry of the uneven batch: seeded shapes in a 30 um box."""
    n, kappa, count, shapes, fails = _random_geometry(seed, n_fixed)
    xyz, tets, _ = kuhn_box_mesh([0.0] * 3, [30.0] * 3, n)
    lab = label_tets(xyz, tets, shapes, mode="centroid")
    prob = Problem(xyz, tets, lab, 2, np.array([D_FREE, D_FREE]), None, None, kappa,
                   np.zeros(3), np.full(3, 30.0), 7, n_cells=n,
                   meta={"name": "seeded_cells", "seed": seed, "n": n, "count_drawn": count,
                         "placed": len(shapes), "failed_tries": fails, "shapes": shapes})
    bs = np.array([1000.0, 2000.0, 3000.0, 4000.0])
    dirs = fibonacci_directions(8)
    b = np.tile(bs, 8)
    q = np.repeat(dirs, 4, axis=0)
    return prob, PGSE_SHORT, Systems(b, q)


def seeded_cells_78(seed: int):
    """Held-out geometry for the learned guess: same generator, n = 78."""
    return seeded_cells(seed, n_fixed=78)
