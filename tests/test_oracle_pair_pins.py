"""Pins of the oracle's cheap pair methods (plain cutoff, shifted-force smoothed
cutoff, Wolf summation), the coarse propagators the thesis proposes (Sec. 3.2
"Proposed Solutions": "Cutoff Method", "Wolf Summation Method"; the smoothed
cutoff is named in Sec. 2.2).  Each pin checks the oracle against something
other than its own formulas: the exact Coulomb sum, the rock-salt Madelung
constant, exact identities of the definitions, brute force and finite
differences."""
import math

import numpy as np
import pytest

import oracle

MADELUNG_NACL = 1.747564594633      # rock salt, potential at an ion site = -M q / d


def _cloud(n, side, seed, neutral=True):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, side, (3, n))
    q = rng.uniform(-1.0, 1.0, n)
    if neutral:
        q -= q.mean()
    return pos, q


@pytest.mark.parametrize("kind", ["cutoff", "shifted_force", "wolf"])
def test_cell_lists_equal_all_pairs(kind):
    pos, q = _cloud(600, 30.0, 1)
    prm = dict(kind=kind, cutoff=7.0, alpha=0.2, box_len=(30.0,) * 3)
    a = oracle.pair(*pos, q, **prm)
    b = oracle.pair(*pos, q, all_pairs=True, **prm)
    assert abs(a["energy"] - b["energy"]) <= 1e-12 * abs(b["energy"])
    assert np.allclose(a["f"], b["f"], rtol=0, atol=1e-12 * np.abs(b["f"]).max())
    assert np.allclose(a["phi"], b["phi"], rtol=0, atol=1e-12 * np.abs(b["phi"]).max())


def test_cutoff_beyond_the_system_is_the_coulomb_sum():
    """With rc above the system's diameter every pair is inside: the plain
    cutoff method is the direct Coulomb sum (eq. coulomb)."""
    pos, q = _cloud(300, 10.0, 2, neutral=False)
    a = oracle.pair(*pos, q, kind="cutoff", cutoff=20.0, box_len=(10.0,) * 3)
    d = oracle.direct(*pos, q)
    assert abs(a["energy"] - d["energy"]) <= 1e-12 * abs(d["energy"])
    assert np.allclose(a["f"], d["f"], rtol=1e-12, atol=1e-12)
    assert np.allclose(a["phi"], d["phi"], rtol=1e-12, atol=1e-12)


def test_two_charges_cutoff_closed_form_and_truncation():
    lo, ln = (0.0, 0.0, 0.0), (20.0,) * 3
    for r, expect in ((3.0, 0.7 * -0.4 / 3.0), (7.9, 0.7 * -0.4 / 7.9), (8.1, 0.0)):
        pos = np.array([[5.0, 5.0 + r], [5.0, 5.0], [5.0, 5.0]])
        e = oracle.pair(*pos, np.array([0.7, -0.4]), kind="cutoff", cutoff=8.0, box_lo=lo, box_len=ln)
        assert abs(e["energy"] - expect) <= 1e-15


def test_wolf_without_damping_is_exact_for_neutral_systems():
    """alpha = 0 and rc above the diameter: the shift -1/rc of every pair and
    the self term -1/(2 rc) sum q^2 add up to -(sum q)^2/(2 rc), which vanishes
    for a neutral system, so energy, potentials and forces are Coulomb's."""
    pos, q = _cloud(250, 10.0, 3)
    w = oracle.pair(*pos, q, kind="wolf", cutoff=25.0, alpha=0.0, box_len=(10.0,) * 3)
    d = oracle.direct(*pos, q)
    assert abs(w["energy"] - d["energy"]) <= 1e-11 * abs(d["energy"])
    assert np.allclose(w["phi"], d["phi"], rtol=0, atol=1e-11 * np.abs(d["phi"]).max())
    assert np.allclose(w["f"], d["f"], rtol=0, atol=1e-11 * np.abs(d["f"]).max())


def test_wolf_gives_the_rock_salt_madelung_energy():
    """Wolf summation of a rock-salt crystal (the test system of its original
    paper): the energy per ion of an ion deep inside a cluster larger than the
    cutoff, 1/2 q phi_pairs + s q^2, converges to -M q^2/(2 d)."""
    d, half, rc_n, alpha_d = 2.8, 12, 11, 0.3
    g = np.arange(-half, half + 1)
    X, Y, Z = (v.ravel() for v in np.meshgrid(g, g, g, indexing="ij"))
    q = np.where((X + Y + Z) % 2 == 0, 1.0, -1.0)
    pos = np.stack([X, Y, Z]).astype(float) * d + (half + 0.5) * d
    L = (2 * half + 2) * d
    rc, alpha = rc_n * d, alpha_d / d
    w = oracle.pair(*pos, q, kind="wolf", cutoff=rc, alpha=alpha, box_len=(L, L, L))
    c = q.size // 2
    assert np.allclose(pos[:, c], (half + 0.5) * d)
    # phi_c = sum_j q_j e(r_cj) + 2 s q_c, so the energy per ion is q_c phi_c / 2
    e_ion = 0.5 * q[c] * w["phi"][c]
    assert abs(-2.0 * d * e_ion - MADELUNG_NACL) < 1e-5


def test_shifted_force_vanishes_smoothly_at_the_cutoff():
    """e(rc) = e'(rc) = 0: two charges approaching rc from inside have an energy
    of second order in the distance to rc, e''(rc)/2 = 1/rc^3; the added terms
    are linear in r (second differences of E_shifted - E_cutoff vanish)."""
    rc, lo, ln = 8.0, (0.0,) * 3, (20.0,) * 3
    q = np.array([1.0, 1.0])

    def energy(kind, r):
        pos = np.array([[5.0, 5.0 + r], [5.0, 5.0], [5.0, 5.0]])
        return oracle.pair(*pos, q, kind=kind, cutoff=rc, box_lo=lo, box_len=ln)["energy"]

    for dlt in (1e-2, 1e-3):
        assert abs(energy("shifted_force", rc - dlt) - dlt ** 2 / rc ** 3) < 1e-2 * dlt ** 2 / rc ** 3
    diff = [energy("shifted_force", r) - energy("cutoff", r) for r in (2.0, 3.0, 4.0)]
    assert abs(diff[0] - 2 * diff[1] + diff[2]) < 1e-14
    assert energy("shifted_force", rc + 1e-9) == 0.0


@pytest.mark.parametrize("kind", ["cutoff", "shifted_force", "wolf"])
def test_forces_and_potentials_are_gradients(kind):
    """F = -dE/dr and phi = dE/dq by central differences (pairs kept away
    from rc, where the plain cutoff and Wolf energies jump)."""
    rng = np.random.default_rng(4)
    pos = rng.uniform(2.0, 8.0, (3, 40))
    q = rng.uniform(-1.0, 1.0, 40)
    prm = dict(kind=kind, cutoff=30.0, alpha=0.25, box_len=(10.0,) * 3)
    ref = oracle.pair(*pos, q, **prm)
    for i, dim in ((0, 0), (7, 1), (19, 2), (33, 0)):
        p1, p2 = pos.copy(), pos.copy()
        p1[dim, i] += 1e-5
        p2[dim, i] -= 1e-5
        fd = (oracle.pair(*p1, q, **prm)["energy"] - oracle.pair(*p2, q, **prm)["energy"]) / 2e-5
        assert abs(fd + ref["f"][dim, i]) < 1e-6 * max(1.0, abs(ref["f"][dim, i]))
        c1, c2 = q.copy(), q.copy()
        c1[i] += 1e-5
        c2[i] -= 1e-5
        fd = (oracle.pair(*pos, c1, **prm)["energy"] - oracle.pair(*pos, c2, **prm)["energy"]) / 2e-5
        assert abs(fd - ref["phi"][i]) < 1e-6 * max(1.0, abs(ref["phi"][i]))
    assert abs(ref["energy"] - 0.5 * q @ ref["phi"]) < 1e-12 * max(1.0, abs(ref["energy"]))


def test_wolf_erfc_is_the_complementary_error_function():
    """The Wolf pair energy at alpha r = 1 and rc far away: erfc(1)/r with the
    tabulated erfc(1) = 0.157299207050285."""
    r = 2.0
    e = oracle.pair_e("wolf", 1e6, 1.0 / r, r)
    assert abs(e - 0.157299207050285 / r) < 1e-12
    assert math.isclose(oracle.pair_e("cutoff", 5.0, 0.0, 2.0), 0.5)


@pytest.mark.parametrize("kind", ["shifted_force", "wolf"])
def test_float32_cutoff_decision_only_moves_pairs_at_the_cutoff(kind):
    """Taking the r < rc decision in float32 changes only pairs within rounding
    of rc; where e(rc) = 0 (shifted force, Wolf) the energy is unchanged to
    rounding, and for float32-exact inputs far from rc nothing changes."""
    pos, q = _cloud(800, 25.0, 5)
    pos = pos.astype(np.float32).astype(np.float64)
    prm = dict(kind=kind, cutoff=6.0, alpha=0.2, box_len=(25.0,) * 3)
    a = oracle.pair(*pos, q, **prm)
    b = oracle.pair(*pos, q, f32_cut=True, **prm)
    assert abs(a["energy"] - b["energy"]) <= 1e-9 * abs(a["energy"])
    assert np.allclose(a["f"], b["f"], rtol=0, atol=1e-8 * np.abs(a["f"]).max())
