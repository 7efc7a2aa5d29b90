"""Seeded synthetic workloads: materials, cell mixes, rigid placements and external forces.

Input data only. The paper's workloads come from a coupled blood flow (fluid + immersed
boundary) that is out of scope here, so these seeded inputs stand in for them: per-vertex
external forces are i.i.d. Gaussian, cells are placed by random rigid motions (cells do not
interact within a solid step, so overlaps are harmless).

Units: um, us, fg, pN (1 fg um / us^2 = 1 pN). Time step h = 0.1 us.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

from .meshes import PLT_DIAMETER, RBC_DIAMETER, platelet_mesh, rbc_mesh

DT = 0.1                 # us  (1e-7 s)
DENSITY = 1025.0         # fg/um^3, parameter table of the supplementary material
PLATELET_STIFFNESS_SCALE = 10.0   # "nearly rigid" platelets: stiffness multiplier (free constant)

RBC, PLT = 0, 1          # cell-type ids used by every workload
DIAMETER = {RBC: RBC_DIAMETER, PLT: PLT_DIAMETER}


@dataclass(frozen=True)
class Material:
    """Membrane constants (parameter table of the supplementary material).

    shear_B, area_C, skalak_D in pN/um; k_bend in pN um; k_vol in pN/um (per vertex);
    strain_min/max clamp the singular values of the strain projection (1, 1 = polar factor);
    pbd_kappa in [0, 1] is the position-based damping factor (kappa_damping of the table);
    v_max > 0 caps the vertex speed after each step (um/us; 0 = no cap); rayleigh_alpha (1/us)
    and rayleigh_beta (us) give Rayleigh damping C = alpha M + beta K (0, 0 = off).
    """
    density: float = DENSITY
    shear_B: float = 5.0
    area_C: float = 5000.0
    skalak_D: float = 35.0
    k_bend: float = 1.0
    k_vol: float = 250.0
    strain_min: float = 1.0
    strain_max: float = 1.0
    pbd_kappa: float = 0.0    # position-based velocity damping (kappa_damping), 0 = off
    v_max: float = 0.0        # velocity cap, 0 = off
    rayleigh_alpha: float = 0.0   # Rayleigh damping C = alpha M + beta K: alpha in 1/us
    rayleigh_beta: float = 0.0    # beta in us (alpha_D, beta_D of the table)
    membrane: str = "pd"          # "pd" constraints or the "skalak" strain energy

    def scaled(self, s: float) -> "Material":
        return Material(self.density, self.shear_B * s, self.area_C * s, self.skalak_D * s,
                        self.k_bend * s, self.k_vol * s, self.strain_min, self.strain_max,
                        self.pbd_kappa, self.v_max, self.rayleigh_alpha, self.rayleigh_beta,
                        self.membrane)

    def with_kappa(self, kappa: float) -> "Material":
        return dataclasses.replace(self, pbd_kappa=kappa)

    def with_v_max(self, v_max: float) -> "Material":
        return dataclasses.replace(self, v_max=v_max)

    def with_membrane(self, membrane: str) -> "Material":
        return dataclasses.replace(self, membrane=membrane)

    def with_rayleigh(self, alpha: float, beta: float) -> "Material":
        return dataclasses.replace(self, rayleigh_alpha=alpha, rayleigh_beta=beta)


RBC_MATERIAL = Material()
PLT_MATERIAL = Material().scaled(PLATELET_STIFFNESS_SCALE)


def cell_type_inputs():
    """{type_id: (rest_xyz, tri, Material)} for the two cell types."""
    xr, tr = rbc_mesh()
    xp, tp = platelet_mesh()
    return {RBC: (xr, tr, RBC_MATERIAL), PLT: (xp, tp, PLT_MATERIAL)}


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Rotation matrices from normalised N(0, I4) quaternions (uniform on SO(3))."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


@dataclass
class Batch:
    """A batch of cells laid out contiguously in SoA order.

    types: int32 [n_cells]; offsets: int64 [n_cells + 1] into the vertex axis;
    x0: float64 [3][V_total] initial positions (already rounded to float32 values);
    v0: float64 [3][V_total] initial velocities.
    """
    types: np.ndarray
    offsets: np.ndarray
    x0: np.ndarray
    v0: np.ndarray
    meshes: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.types.shape[0])

    @property
    def v_total(self) -> int:
        return int(self.offsets[-1])

    def cell_slice(self, c: int) -> slice:
        return slice(int(self.offsets[c]), int(self.offsets[c + 1]))


def make_batch(types, seed: int, translate: float = 200.0, identity: bool = False) -> Batch:
    """Place each cell by a random rigid motion (rotation + translation in U[0, translate]^3)."""
    types = np.asarray(types, dtype=np.int32)
    meshes = cell_type_inputs()
    sizes = np.array([meshes[int(t)][0].shape[0] for t in types], dtype=np.int64)
    offsets = np.zeros(len(types) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    rng = np.random.default_rng(seed)
    n = len(types)
    if identity:
        rot = np.broadcast_to(np.eye(3), (n, 3, 3))
        trans = np.zeros((n, 3))
    else:
        rot = random_rotations(rng, n)
        trans = rng.uniform(0.0, translate, size=(n, 3))
    x0 = np.empty((3, int(offsets[-1])))
    for c in range(n):
        rest = meshes[int(types[c])][0]
        x0[:, offsets[c]:offsets[c + 1]] = (rest @ rot[c].T + trans[c]).T
    x0 = x0.astype(np.float32).astype(np.float64)
    return Batch(types, offsets, x0, np.zeros_like(x0), meshes)


# Nominal cell volumes (fL = um^3) that size a packing box: the RBC mesh's own volume (about a
# normal RBC) and the paper's platelet volume (6.8 fL).
NOMINAL_VOLUME = {RBC: 90.0, PLT: 6.8}

# Cell-packing run (main text: cells placed at random without avoiding interpenetration, then
# advanced for a few thousand steps with the fluid switched off): hematocrit of the box, and
# the collision parameters. The kernel sphere has a diameter of 4 dx (dx = 0.5 um, the fluid
# lattice spacing of the workloads), so a radius of 1 um; the projection point lies one
# kernel radius from the colliding neighbour along its cell's outward normal.
PACKING = {"hematocrit": 0.40, "dx": 0.5, "radius": 1.0, "separation": 1.0, "weight": 400.0,
           "n_pd_iters": 10}


def packing_batch(types, seed: int, hematocrit: float = PACKING["hematocrit"]) -> Batch:
    """Cells at random rigid motions with centres uniform in a cube whose volume is the cells'
    nominal volume over the hematocrit; overlaps are not avoided."""
    types = np.asarray(types, dtype=np.int32)
    vol = float(sum(NOMINAL_VOLUME[int(t)] for t in types))
    edge = (vol / hematocrit) ** (1.0 / 3.0)
    return make_batch(types, seed, translate=edge)


def force_stream(batch: Batch, seed: int, sigma: float, n_steps: int,
                 strong_fraction: float = 0.0, strong_factor: float = 10.0):
    """Yield one fresh external-force array float64 [3][V_total] (float32-rounded) per step.

    Forces are i.i.d. N(0, sigma) pN per vertex and coordinate, drawn in step order from
    ``numpy.random.default_rng(seed)``. A seeded ``strong_fraction`` of the cells has its
    forces multiplied by ``strong_factor`` (strongly deformed cells).
    """
    rng = np.random.default_rng(seed)
    scale = np.full(batch.v_total, sigma)
    if strong_fraction > 0.0:
        n_strong = int(round(strong_fraction * batch.n_cells))
        strong = rng.choice(batch.n_cells, size=n_strong, replace=False)
        for c in strong:
            scale[batch.cell_slice(int(c))] *= strong_factor
    for _ in range(n_steps):
        f = rng.normal(0.0, 1.0, size=(3, batch.v_total)) * scale
        yield f.astype(np.float32).astype(np.float64)


def strong_cells(batch: Batch, seed: int, strong_fraction: float) -> np.ndarray:
    """The cell ids that ``force_stream`` with the same arguments scales up."""
    if strong_fraction <= 0.0:
        return np.zeros(0, dtype=np.int64)
    rng = np.random.default_rng(seed)
    n_strong = int(round(strong_fraction * batch.n_cells))
    return np.sort(rng.choice(batch.n_cells, size=n_strong, replace=False))


# ----------------------------------------------------------------------------------------
# The five workloads (sizes, seeds and force distributions).
# ----------------------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    n_rbc: int
    n_plt: int
    seed: int
    sigma: float
    n_pd_iters: int
    n_steps: int
    strong_fraction: float = 0.0
    interleave: bool = False        # random permutation of types instead of blocks
    identity: bool = False          # single cell at the origin, no random placement

    def types(self) -> np.ndarray:
        t = np.array([RBC] * self.n_rbc + [PLT] * self.n_plt, dtype=np.int32)
        if self.interleave:
            t = t[np.random.default_rng(self.seed + 1000).permutation(len(t))]
        return t

    def batch(self) -> Batch:
        return make_batch(self.types(), self.seed, identity=self.identity)

    def forces(self, batch: Batch, n_steps: int | None = None):
        return force_stream(batch, self.seed, self.sigma,
                            self.n_steps if n_steps is None else n_steps,
                            self.strong_fraction)


WORKLOADS = {
    # one RBC at the origin, sigma = 1 pN, seed 0, 100 steps x 10 PD iterations
    "single_rbc": Workload("single_rbc", 1, 0, seed=0, sigma=1.0, n_pd_iters=10, n_steps=100,
                           identity=True),
    # 1000 RBC + 300 PLT in type blocks, seed 1, sigma = 1 pN, 10 PD iterations
    "batch_1300": Workload("batch_1300", 1000, 300, seed=1, sigma=1.0, n_pd_iters=10,
                           n_steps=100),
    # 20000 RBC + 4000 PLT interleaved, sigma = 2 pN with 5 % of cells at 10x, 20 PD iterations
    "large_24000": Workload("large_24000", 20000, 4000, seed=3, sigma=2.0, n_pd_iters=20,
                            n_steps=100, strong_fraction=0.05, interleave=True),
}
