"""Seeded synthetic inputs for the Bidomain slab workloads.

This module draws the *numbers* that define a case -- slab size, stimulus ellipsoids,
serving arrival times -- and evaluates the initial transmembrane potential at the mesh
nodes. It holds none of the solver's arithmetic (no assembly, no AMG, no Krylov step),
so both the CPU oracle and the HIP library may take their inputs from here.

The benchmarked workloads are slabs: a 1 x 1 x 0.5 cm slab with the paper's kind of fiber
rotation (Sec. 2, eq. (2)) and a plateau stimulus stands in for the paper's patient mesh, and
the TP06 membrane model is replaced by Aliev-Panfilov.  The paper's structured geometry, the
truncated ellipsoid of Sec. 3, is also defined here (EllipsoidCase: its parameters and the
stimulated index block; the geometry itself is computed by the oracle and by the library).

Node numbering: p = i + (nx+1) * (j + (ny+1) * k), x fastest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np

Ellipsoid = Tuple[float, float, float, float, float, float]  # cx, cy, cz, ax, ay, az (cm)


@dataclass(frozen=True)
class SlabCase:
    """One Bidomain slab case. Units: cm, ms, mV, S/cm, mF/cm^3."""

    nx: int
    ny: int
    nz: int
    Lx: float = 1.0
    Ly: float = 1.0
    Lz: float = 0.5
    # axisymmetric conductivities (sigma_n = sigma_t in eq. (2))
    sig_il: float = 3.0e-3
    sig_it: float = 3.1525e-4
    sig_el: float = 2.0e-3
    sig_et: float = 1.3514e-3
    # in-plane fibers rotating linearly through the thickness: theta(z) = theta0 + rot * z / Lz
    fiber_theta0: float = -math.pi / 3.0
    fiber_rotation: float = 2.0 * math.pi / 3.0
    cm: float = 1.0  # chi * C_m (1000 1/cm * 1 uF/cm^2)
    dt: float = 0.05  # ms
    # Aliev-Panfilov membrane model (Aliev & Panfilov 1996), its published parameters; one model
    # time unit is ap_t_unit ms and u = (v - ap_v_rest) / ap_v_scale
    ap_k: float = 8.0
    ap_a: float = 0.15
    ap_eps0: float = 0.002
    ap_mu1: float = 0.2
    ap_mu2: float = 0.3
    ap_t_unit: float = 12.9
    ap_v_scale: float = 105.0
    ap_v_rest: float = -85.0
    v_rest: float = -85.0
    v_plateau: float = 20.0
    ellipsoids: Tuple[Ellipsoid, ...] = field(default_factory=tuple)
    seed: int = 0
    name: str = ""

    @property
    def n(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def h(self) -> Tuple[float, float, float]:
        return self.Lx / self.nx, self.Ly / self.ny, self.Lz / self.nz

    @property
    def nnz27(self) -> int:
        """Entries of the full 27-point Q1 pattern (structural zeros kept)."""
        return (3 * self.nx + 1) * (3 * self.ny + 1) * (3 * self.nz + 1)

    @property
    def paper_dofs(self) -> int:
        """The paper counts v and u_e at every node (weak-scaling tables)."""
        return 2 * self.n


def _draw_ellipsoids(rng: np.random.Generator, count: int, wide: bool) -> Tuple[Ellipsoid, ...]:
    out = []
    for _ in range(count):
        if wide:
            c = rng.uniform([0.1, 0.1, 0.1], [0.9, 0.9, 0.4])
        else:
            c = rng.uniform([0.3, 0.3, 0.15], [0.7, 0.7, 0.35])
        a = rng.uniform([0.08, 0.08, 0.05], [0.2, 0.2, 0.12])
        out.append(tuple(float(v) for v in (*c, *a)))
    return tuple(out)


def make_case(nx: int, ny: int, nz: int, seed: int, n_ellipsoids: int = 1, name: str = "", **kw) -> SlabCase:
    rng = np.random.default_rng(seed)
    ell = _draw_ellipsoids(rng, n_ellipsoids, wide=n_ellipsoids > 1)
    return SlabCase(nx=nx, ny=ny, nz=nz, ellipsoids=ell, seed=seed, name=name or f"slab{nx}x{ny}x{nz}", **kw)


# The five workloads (sizes in elements).
CONFIGS = {
    "C1": dict(nx=16, ny=16, nz=8, seed=1, n_ellipsoids=1),
    "C2": dict(nx=128, ny=128, nz=64, seed=2, n_ellipsoids=1),
    "C3": dict(nx=256, ny=256, nz=64, seed=3, n_ellipsoids=8),
    "C5": dict(nx=384, ny=384, nz=96, seed=5, n_ellipsoids=8),
}


def config_case(name: str) -> SlabCase:
    kw = dict(CONFIGS[name])
    return make_case(name=name, **kw)


def block_of(case: SlabCase, nx: int, ny: int, nz: int, around: int = 0) -> SlabCase:
    """The nx x ny x nz-element block of `case` (same element sizes, same fiber field, same
    stimulus ellipsoids) placed around the centre of ellipsoid `around`, as a slab of its own
    with the origin at the block's corner: a bounded sample of a workload that is too large for
    the CPU oracle."""
    hx, hy, hz = case.h
    cx, cy, cz = case.ellipsoids[around][:3] if case.ellipsoids else (0.0, 0.0, 0.0)
    i0 = min(max(int(round(cx / hx)) - nx // 2, 0), case.nx - nx)
    j0 = min(max(int(round(cy / hy)) - ny // 2, 0), case.ny - ny)
    k0 = min(max(int(round(cz / hz)) - nz // 2, 0), case.nz - nz)
    x0, y0, z0 = i0 * hx, j0 * hy, k0 * hz
    ell = tuple((e[0] - x0, e[1] - y0, e[2] - z0, e[3], e[4], e[5]) for e in case.ellipsoids)
    return replace(case, nx=nx, ny=ny, nz=nz, Lx=nx * hx, Ly=ny * hy, Lz=nz * hz,
                   fiber_theta0=case.fiber_theta0 + case.fiber_rotation * z0 / case.Lz,
                   fiber_rotation=case.fiber_rotation * (nz * hz) / case.Lz, ellipsoids=ell,
                   name=f"{case.name or 'slab'}-block{nx}x{ny}x{nz}@{i0},{j0},{k0}")


@dataclass(frozen=True)
class EllipsoidCase:
    """One Bidomain case on the truncated ellipsoid of Sec. 3 (eq. (8), Table 1), n_theta x n_phi
    x n_r elements, periodic in theta.  Units as for SlabCase; conductivities, membrane and time
    step as for the slab.

    Node numbering: p = i + n_theta * (j + (n_phi + 1) * k), theta fastest, r slowest (k = 0 is
    the endocardium)."""

    n_theta: int
    n_phi: int
    n_r: int
    a1: float = 2.2
    a2: float = 3.3
    b1: float = 2.2
    b2: float = 3.3
    c1: float = 5.9
    c2: float = 6.4
    theta_min: float = -1.5 * math.pi
    theta_max: float = 0.5 * math.pi
    phi_min: float = -0.375 * math.pi
    phi_max: float = 0.125 * math.pi
    sig_il: float = 3.0e-3
    sig_it: float = 3.1525e-4
    sig_el: float = 2.0e-3
    sig_et: float = 1.3514e-3
    # fiber angle from the theta direction towards the phi direction: +60 deg at the
    # endocardium (r = 0), -60 deg at the epicardium (r = 1)
    fiber_endo: float = math.pi / 3.0
    fiber_epi: float = -math.pi / 3.0
    cm: float = 1.0
    dt: float = 0.05
    ap_k: float = 8.0
    ap_a: float = 0.15
    ap_eps0: float = 0.002
    ap_mu1: float = 0.2
    ap_mu2: float = 0.3
    ap_t_unit: float = 12.9
    ap_v_scale: float = 105.0
    ap_v_rest: float = -85.0
    v_rest: float = -85.0
    v_plateau: float = 20.0
    # stimulated block in index fractions: theta [s0, s1), phi [s2, s3], r [s4, s5] -- an
    # endocardial patch near the apex (phi_min is the apical end)
    stim: Tuple[float, float, float, float, float, float] = (0.0, 0.125, 0.0, 0.25, 0.0, 0.25)
    name: str = ""

    @property
    def n(self) -> int:
        return self.n_theta * (self.n_phi + 1) * (self.n_r + 1)

    @property
    def nnz27(self) -> int:
        return 3 * self.n_theta * (3 * self.n_phi + 1) * (3 * self.n_r + 1)

    @property
    def paper_dofs(self) -> int:
        return 2 * self.n


# The paper's structured meshes (elements n_theta x n_phi x n_r): the threshold-calibration mesh
# of Test 1 and the strong-scaling mesh of Test 2.
ELLIPSOID_CONFIGS = {
    "E1": dict(n_theta=32, n_phi=32, n_r=16),
    "E2": dict(n_theta=128, n_phi=128, n_r=64),
}


def ellipsoid_case(name: str, **kw) -> EllipsoidCase:
    return EllipsoidCase(name=name, **{**ELLIPSOID_CONFIGS[name], **kw})


def ellipsoid_v0(case: EllipsoidCase) -> np.ndarray:
    """Initial transmembrane potential: v_plateau on the stimulated index block, v_rest elsewhere."""
    s0, s1, s2, s3, s4, s5 = case.stim
    i = np.arange(case.n_theta) / case.n_theta
    j = np.arange(case.n_phi + 1) / case.n_phi
    k = np.arange(case.n_r + 1) / case.n_r
    K, J, I = np.meshgrid(k, j, i, indexing="ij")
    inside = (I >= s0) & (I < s1) & (J >= s2) & (J <= s3) & (K >= s4) & (K <= s5)
    v = np.full(case.n, case.v_rest, dtype=np.float64)
    v[inside.ravel()] = case.v_plateau
    return v


def node_coordinates(case: SlabCase):
    hx, hy, hz = case.h
    x = np.arange(case.nx + 1) * hx
    y = np.arange(case.ny + 1) * hy
    z = np.arange(case.nz + 1) * hz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")  # k slowest, i fastest
    return X.ravel(), Y.ravel(), Z.ravel()


def nodal_v0(case: SlabCase) -> np.ndarray:
    """Initial transmembrane potential: v_plateau inside the union of ellipsoids, v_rest outside."""
    X, Y, Z = node_coordinates(case)
    inside = np.zeros(X.shape, dtype=bool)
    for cx, cy, cz, ax, ay, az in case.ellipsoids:
        inside |= ((X - cx) / ax) ** 2 + ((Y - cy) / ay) ** 2 + ((Z - cz) / az) ** 2 <= 1.0
    v = np.full(X.shape, case.v_rest, dtype=np.float64)
    v[inside] = case.v_plateau
    return v


def nodal_w0(case: SlabCase) -> np.ndarray:
    return np.zeros(case.n, dtype=np.float64)


def random_vector(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n).astype(dtype)


@dataclass
class ServedRequest:
    ticket: int
    arrival_s: float
    case: SlabCase
    nsteps: int


def serving_stream(n_cases: int = 64, nsteps: int = 20, rate_per_s: float = 20.0, seed: int = 4,
                   min_dims=(32, 32, 16), max_dims=(160, 160, 64)) -> List[ServedRequest]:
    """Poisson arrivals of slab cases with log-uniform element counts.

    nx = ny = round(32 * 5**t), nz = round(16 * 4**t), t ~ U(0, 1); the first two cases
    are pinned to t = 0 and t = 1 so that both size endpoints appear in every stream.
    """
    rng = np.random.default_rng(seed)
    fx = max_dims[0] / min_dims[0]
    fz = max_dims[2] / min_dims[2]
    out = []
    t_arr = 0.0
    for c in range(n_cases):
        t = 0.0 if c == 0 else (1.0 if c == 1 else float(rng.uniform()))
        nxy = int(round(min_dims[0] * fx ** t))
        nz = int(round(min_dims[2] * fz ** t))
        case = make_case(nxy, nxy, nz, seed=int(rng.integers(1 << 31)), n_ellipsoids=1, name=f"serve{c}")
        out.append(ServedRequest(ticket=c, arrival_s=t_arr, case=case, nsteps=nsteps))
        t_arr += float(rng.exponential(1.0 / rate_per_s))
    return out
