"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws positions and charges.  It holds none of the
multilevel-summation arithmetic, so the HIP path and the oracle can both be fed
from it without sharing method code.

Workloads follow the shapes of the thesis' target systems (explicit rigid
3-site water in a box, Sec. "Molecular Dynamics" / "Acceleration", and a
uniform +-1 charge cloud as a small non-periodic case):

* ``uniform_charges``: N point charges uniform in a cube, charges +1/-1
  alternating (net neutral).
* ``water_box``: rigid 3-site water-like molecules (O -0.834 e, two H +0.417 e
  at 0.9572 A, H-O-H 104.52 deg), molecule centres on a jittered simple-cubic
  lattice at 0.1 atoms/A^3, uniformly random orientation.

Positions are drawn in float64 and then rounded to float32.  Both the GPU path
and the oracle consume those float32 values (the oracle widens them to float64
exactly), so parity is measured on identical inputs.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

WATER_DENSITY = 0.1          # atoms / A^3
OH_BOND = 0.9572             # A
HOH_ANGLE_DEG = 104.52
Q_H = float(np.float32(0.417))
Q_O = float(np.float32(-2.0 * np.float32(0.417)))   # exact neutrality in float32


@dataclasses.dataclass
class System:
    """One evaluation's inputs: float32 SoA positions/charges plus the MSM parameters."""
    x: np.ndarray            # float32 [N]
    y: np.ndarray
    z: np.ndarray
    q: np.ndarray
    box_lo: tuple            # (3,) float
    box_len: tuple           # (3,) float
    cutoff: float            # a, A
    spacing: float           # h, A
    order: int               # 4 = cubic, 6 = quintic
    levels: int              # 0 = automatic
    split_m: int = 0         # 0 = order // 2
    name: str = ""
    x64: np.ndarray | None = None   # original float64 positions [3, N] (before rounding)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def params(self) -> dict:
        return dict(cutoff=self.cutoff, spacing=self.spacing, order=self.order,
                    split_m=self.split_m, levels=self.levels,
                    box_lo=tuple(self.box_lo), box_len=tuple(self.box_len))

    def pos64(self) -> np.ndarray:
        """float32 inputs widened to float64, shape [3, N]."""
        return np.stack([self.x, self.y, self.z]).astype(np.float64)


def _as_f32_system(pos64, q, lo, length, **kw) -> System:
    p32 = pos64.astype(np.float32)
    return System(x=np.ascontiguousarray(p32[0]), y=np.ascontiguousarray(p32[1]),
                  z=np.ascontiguousarray(p32[2]), q=np.ascontiguousarray(q.astype(np.float32)),
                  box_lo=tuple(float(v) for v in lo), box_len=tuple(float(v) for v in length),
                  x64=pos64, **kw)


def uniform_charges(n=1000, side=20.0, seed=1, cutoff=8.0, spacing=2.5, order=4,
                    levels=2, split_m=0) -> System:
    """N charges uniform in [0, side)^3, q = +1 for even index, -1 for odd."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, side, size=(3, n))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return _as_f32_system(pos, q, (0.0, 0.0, 0.0), (side, side, side), cutoff=cutoff,
                          spacing=spacing, order=order, levels=levels, split_m=split_m,
                          name=f"uniform{n}")


def periodic_spacing(side, spacing, levels):
    """The spacing nearest to `spacing` that puts a whole number of grid nodes,
    divisible by 2^(levels - 1), on an edge of length `side` (periodic plans
    need one)."""
    unit = 2 ** max(levels - 1, 0)
    k = max(1, int(round(side / spacing / unit)))
    return side / (k * unit)


def _random_rotations(rng, k):
    """Uniform random rotation matrices from uniform unit quaternions (Shoemake)."""
    u1, u2, u3 = rng.random(k), rng.random(k), rng.random(k)
    a, b = np.sqrt(1 - u1), np.sqrt(u1)
    w = a * np.sin(2 * np.pi * u2)
    x = a * np.cos(2 * np.pi * u2)
    y = b * np.sin(2 * np.pi * u3)
    z = b * np.cos(2 * np.pi * u3)
    r = np.empty((k, 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - z * w)
    r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w)
    r[:, 2, 1] = 2 * (y * z + x * w)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def water_box(n_atoms, seed, cutoff=12.0, spacing=2.0, order=4, levels=0, split_m=0,
              density=WATER_DENSITY, name=None) -> System:
    """Rigid 3-site water-like molecules at `density` atoms/A^3 in a cube [0, L)^3."""
    n_mol = n_atoms // 3
    n_atoms = 3 * n_mol
    side = (n_atoms / density) ** (1.0 / 3.0)
    rng = np.random.default_rng(seed)
    per = int(math.ceil(n_mol ** (1.0 / 3.0) - 1e-9))
    while per ** 3 < n_mol:
        per += 1
    s = side / per
    sites = rng.choice(per ** 3, size=n_mol, replace=False)
    ix, iy, iz = sites // (per * per), (sites // per) % per, sites % per
    centre = np.stack([ix, iy, iz], axis=1).astype(np.float64) + 0.5
    o = centre * s + rng.uniform(-0.05 * s, 0.05 * s, size=(n_mol, 3))
    half = math.radians(HOH_ANGLE_DEG) / 2.0
    # body frame: molecule in the xz-plane, bisector along +z
    h1b = np.array([OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)])
    h2b = np.array([-OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)])
    rot = _random_rotations(rng, n_mol)
    h1 = o + rot @ h1b
    h2 = o + rot @ h2b
    pos = np.empty((n_atoms, 3))
    pos[0::3], pos[1::3], pos[2::3] = o, h1, h2
    q = np.empty(n_atoms)
    q[0::3], q[1::3], q[2::3] = Q_O, Q_H, Q_H
    assert pos.min() > 0.0 and pos.max() < side, "water generator left the box"
    return _as_f32_system(np.ascontiguousarray(pos.T), q, (0.0, 0.0, 0.0), (side, side, side),
                          cutoff=cutoff, spacing=spacing, order=order, levels=levels,
                          split_m=split_m, name=name or f"water{n_atoms}")


# Ions for time stepping.  The evaluated force is electrostatics alone (no
# short-range repulsion), so the test dynamics is a nearly perfect rock-salt
# lattice of +1 / -1 ions at a low temperature, where ions stay apart over
# the short windows simulated.
NA_MASS, CL_MASS = 22.98977, 35.453          # amu
KB_KCAL = 0.0019872041                       # kcal/mol/K
COULOMB_KCAL = 332.0637                      # kcal/mol A per e^2 (the e^2/A energy unit)
ACCEL_PER_KCAL_A_AMU = 4.184e-4              # A/fs^2 per kcal/mol/A/amu
VEL_PER_SQRT_KCAL_AMU = 2.0455e-2            # A/fs per sqrt(kcal/mol/amu)
# acceleration in A/fs^2 of a force in e^2/A^2 on a mass in amu
ACCEL_SCALE = COULOMB_KCAL * ACCEL_PER_KCAL_A_AMU


@dataclasses.dataclass
class Ions:
    system: System           # positions, charges and MSM parameters
    inv_mass: np.ndarray     # float32 [N], 1/amu
    vel: np.ndarray          # float32 [3, N], A/fs


def rock_salt(n_side, seed, spacing=2.82, jitter=0.05, margin=8.0, temperature=50.0, cutoff=8.0,
              grid=2.0, order=4, levels=0) -> Ions:
    """n_side^3 ions on a simple-cubic lattice of `spacing` A, charges +1 (Na
    mass) and -1 (Cl mass) alternating (the rock-salt arrangement), each
    displaced uniformly by up to `jitter` A per coordinate, in a box with
    `margin` A of free space on every side; Maxwell-Boltzmann velocities at
    `temperature` K (momentum not removed)."""
    rng = np.random.default_rng(seed)
    g = np.arange(n_side)
    X, Y, Z = (v.ravel() for v in np.meshgrid(g, g, g, indexing="ij"))
    q = np.where((X + Y + Z) % 2 == 0, 1.0, -1.0)
    pos = np.stack([X, Y, Z]).astype(np.float64) * spacing + margin
    pos += rng.uniform(-jitter, jitter, size=pos.shape)
    side = (n_side - 1) * spacing + 2.0 * margin
    mass = np.where(q > 0, NA_MASS, CL_MASS)
    sigma = np.sqrt(KB_KCAL * temperature / mass) * VEL_PER_SQRT_KCAL_AMU
    vel = rng.standard_normal(size=pos.shape) * sigma
    s = _as_f32_system(pos, q, (0.0, 0.0, 0.0), (side, side, side), cutoff=cutoff, spacing=grid,
                       order=order, levels=levels, name=f"rocksalt{n_side ** 3}")
    return Ions(system=s, inv_mass=(1.0 / mass).astype(np.float32),
                vel=np.ascontiguousarray(vel.astype(np.float32)))


def water_exclusions(n_atoms, offset=0):
    """Bonded exclusions of 3-site water molecules (O, H, H in that order):
    each atom excludes the other two of its molecule.  CSR over the atom
    indices offset .. offset + n_atoms - 1: start int32 [n_atoms + 1], idx
    int32 (partners, global indices)."""
    n_mol = n_atoms // 3
    base = offset + 3 * np.repeat(np.arange(n_mol), 3)
    local = np.tile(np.array([[1, 2], [0, 2], [0, 1]]), (n_mol, 1))
    idx = (base[:, None] + local).reshape(-1).astype(np.int32)
    start = (2 * np.arange(3 * n_mol + 1)).astype(np.int32)
    return start, idx


def batch_sizes(n_sys=64, lo=2000, hi=60000, seed=5):
    """Atom counts log-uniform in [lo, hi], rounded to whole molecules."""
    rng = np.random.default_rng(seed)
    raw = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_sys))
    return [int(3 * round(v / 3.0)) for v in raw]


# ---------------------------------------------------------------------------
# Named workloads.  Sizes and parameters are those of the target systems:
#   small non-periodic cloud, 24k water, 1M water, 100k water (gradients),
#   64 uneven water replicas (batched).
# ---------------------------------------------------------------------------

def cloud_1k() -> System:
    return uniform_charges(1000, 20.0, seed=1, cutoff=8.0, spacing=2.5, order=4, levels=2)


def water_24k() -> System:
    return water_box(24000, seed=2, cutoff=12.0, spacing=2.0, order=4, levels=4, name="water24k")


def water_1m() -> System:
    return water_box(999999, seed=3, cutoff=12.0, spacing=2.5, order=6, levels=0, name="water1m")


def water_100k() -> System:
    return water_box(99999, seed=4, cutoff=12.0, spacing=2.0, order=4, levels=0, name="water100k")


def water_replicas(n_sys=64, seed=5):
    return [water_box(n, seed=5000 + s, cutoff=10.0, spacing=2.0, order=4, levels=0,
                      name=f"replica{s}") for s, n in enumerate(batch_sizes(n_sys, seed=seed))]
