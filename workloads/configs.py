"""The five synthetic workloads: plate meshes, material, loading, initial state.

Shapes follow the paper's dynamic benchmarks (Sec. 3, Table "benchmark
overview"): glass plates (E = 32 GPa, nu = 0.2, rho = 2450 kg/m^3,
G_c = 3 J/m^2) with l0 = 0.5 mm and crack-zone spacing h = l0/2, an edge
notch at mid-height and opposite velocities on the top and bottom edges.
Everything here is input data; no step of the method is computed.
Units are SI throughout.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from .meshes import STREAM_GC, STREAM_SIZES, plate_mesh, rng

H_GRID = 2.5e-4          # m; crack-zone spacing of the glass SENT case (h = l0/2)
L0 = 2 * H_GRID          # m; regularisation length l0 = 0.5 mm
GLASS = dict(E=32e9, nu=0.2, rho=2450.0, Gc=3.0, l0=L0, eta=1e-7)
V_PULL = 0.5             # m/s on the top (+) and bottom (-) edges


@dataclass
class Problem:
    """One simulation instance: mesh, model choices, initial state."""
    name: str
    xy: np.ndarray            # (N,2) float64
    tri: np.ndarray           # (Ne,3) int32
    fixed: np.ndarray         # (N,2) uint8: 1 = velocity-prescribed DOF
    u0: np.ndarray            # (N,2) float64
    v0: np.ndarray            # (N,2) float64 (prescribed velocity on fixed DOFs)
    a0: np.ndarray            # (N,2) float64 (u0 = 0 and no external force, so a0 = 0)
    d0: np.ndarray            # (N,) float64 (1 on the notch)
    H0: np.ndarray            # (Ne,) float64
    E: float
    nu: float
    rho: float
    Gc: float
    l0: float
    eta: float
    model: int                # 1 = AT1, 2 = AT2
    split: str                # 'none' | 'spectral' | 'voldev' | 'starconvex'
    plane: str                # 'strain' | 'stress'
    gamma_star: float = 0.0
    dtype: str = "f64"        # arithmetic type of the GPU path for this workload
    steps: int = 1
    cfl: float = 0.5          # dt = cfl * h_min / c_p
    bounds: str = "projected" # 'projected' | 'postclamp'
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.tri.shape[0])

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def plate_problem(name: str, nx: int, ny: int, jitter: float, seed: int, *, model: int, split: str,
                  plane: str, gamma_star: float = 0.0, dtype: str = "f64", steps: int = 1,
                  random_diag: bool = False, n_holes: int = 0, sub: tuple[int, ...] = (),
                  material: dict | None = None, notch: bool = True, pull: float = V_PULL) -> Problem:
    """Plate with an edge notch along row ny/2 (i <= nx/2) and pulled edges.

    The notch is represented by d0 = 1 on its grid nodes; the bottom row's
    y-velocity is -pull and the top row's +pull, prescribed from t = 0.
    """
    m = plate_mesh(nx, ny, H_GRID, jitter, seed, random_diag=random_diag, n_holes=n_holes, sub=sub)
    ij = m["ij"]
    n = len(m["xy"])
    fixed = np.zeros((n, 2), dtype=np.uint8)
    v0 = np.zeros((n, 2))
    bot = ij[:, 1] == 0
    top = ij[:, 1] == ny
    fixed[bot | top, 1] = 1
    v0[bot, 1] = -pull
    v0[top, 1] = +pull
    d0 = np.zeros(n)
    if notch:
        d0[(ij[:, 1] == ny // 2) & (ij[:, 0] <= nx // 2)] = 1.0
    mat = dict(GLASS if material is None else material)
    return Problem(name=name, xy=m["xy"], tri=m["tri"], fixed=fixed, u0=np.zeros((n, 2)), v0=v0,
                   a0=np.zeros((n, 2)), d0=d0, H0=np.zeros(len(m["tri"])), model=model, split=split,
                   plane=plane, gamma_star=gamma_star, dtype=dtype, steps=steps,
                   meta={"nx": nx, "ny": ny, "h": H_GRID, "ij": ij, "jitter": jitter, "seed": seed,
                         "hole_centres": m["hole_centres"], "hole_radius": m["hole_radius"]},
                   **mat)


def config0() -> Problem:
    """64x32 plate, FP64, AT2 / spectral / plane strain, 200 steps."""
    return plate_problem("c0", 64, 32, 0.05, 0, model=2, split="spectral", plane="strain",
                         dtype="f64", steps=200)


def config1() -> Problem:
    """1024x512 plate, FP32 kernels, AT2 / vol-dev / plane strain, 1000 steps."""
    return plate_problem("c1", 1024, 512, 0.10, 1, model=2, split="voldev", plane="strain",
                         dtype="f32", steps=1000)


def config2() -> Problem:
    """1448x724 perforated plate, random diagonals, AT1 / star-convex / plane stress."""
    return plate_problem("c2", 1448, 724, 0.25, 2, model=1, split="starconvex", plane="stress",
                         gamma_star=1.0, dtype="f32", steps=500, random_diag=True, n_holes=6)


def config3(Gc: float = 2.0) -> Problem:
    """256x128 plate, FP64, AT2 / spectral / plane strain, 500 steps (run at Gc = 2)."""
    p = plate_problem("c3", 256, 128, 0.05, 3, model=2, split="spectral", plane="strain",
                      dtype="f64", steps=500)
    return p.with_(Gc=Gc, meta={**p.meta, "Gc_target": 3.0, "checkpoint_every": 50})


def config4_draws(n: int = 64, seed: int = 4) -> tuple[np.ndarray, np.ndarray]:
    """Grid widths nx_k = 128 + 8*floor(49 u) and log-uniform G_c in [1, 10] J/m^2."""
    u = rng(seed, STREAM_SIZES).random(n)
    nx = 128 + 8 * np.floor(49 * u).astype(np.int64)
    gc = 10.0 ** rng(seed, STREAM_GC).random(n)
    return nx, gc


def config4(n: int = 64, seed: int = 4) -> list[Problem]:
    """64 plates of uneven size (128x64 .. 512x256), c0 physics, FP32, 300 steps."""
    nxs, gcs = config4_draws(n, seed)
    out = []
    for k, (nx, gc) in enumerate(zip(nxs, gcs)):
        p = plate_problem(f"c4[{k}]", int(nx), int(nx) // 2, 0.05, seed, model=2, split="spectral",
                          plane="strain", dtype="f32", steps=300, sub=(k,))
        out.append(p.with_(Gc=float(gc), meta={**p.meta, "Gc_target": 3.0}))
    return out


def small_plate(nx: int = 16, ny: int = 8, jitter: float = 0.05, seed: int = 7, **kw) -> Problem:
    """A small plate for unit tests; keyword arguments override the physics."""
    args = dict(model=2, split="spectral", plane="strain", dtype="f64", steps=10)
    args.update(kw)
    return plate_problem(f"plate{nx}x{ny}", nx, ny, jitter, seed, **args)


CONFIGS = {0: config0, 1: config1, 2: config2, 3: config3}
