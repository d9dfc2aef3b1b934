"""Pins of the oracle's periodic boundaries (the box repeated in every
direction, every pair summed over all images): the Ewald summation reference
against the Madelung constant of rock salt and its own gradients; the periodic
multilevel summation against Ewald within the method's accuracy (shrinking as
the grid is refined), against the Madelung constant, under lattice shifts of
atoms, with one, two and three levels, and as the exact gradient of its own
energy."""
import numpy as np
import pytest

import oracle

MADELUNG_NACL = 1.747564594633182   # rock salt, per ion pair at nearest-neighbour distance 1


def _rock_salt(cells, r0):
    """Periodic rock-salt crystal: cells^3 conventional cubes of edge 2 r0,
    ions at r0 (i, j, k) with charge (-1)^(i+j+k)."""
    n = 2 * cells
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    pos = r0 * np.stack([i.ravel(), j.ravel(), k.ravel()]).astype(np.float64) + 0.5 * r0
    q = np.where((i + j + k).ravel() % 2 == 0, 1.0, -1.0)
    return pos, q, n * r0


def _cloud(n=400, box=(24.0, 24.0, 24.0), seed=3):
    rng = np.random.default_rng(seed)
    L = np.asarray(box, dtype=np.float64)
    pos = rng.uniform(0.0, 1.0, size=(3, n)) * L[:, None]
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return pos, q, L


def test_ewald_gives_the_madelung_energy_of_rock_salt():
    for cells, r0 in ((1, 1.0), (2, 2.82)):
        pos, q, L = _rock_salt(cells, r0)
        ew = oracle.ewald(*pos, q, box_lo=(0, 0, 0), box_len=(L, L, L))
        per_pair = ew["energy"] / (0.5 * q.size)
        assert abs(per_pair + MADELUNG_NACL / r0) < 1e-10 / r0
        # every ion sits at a centre of symmetry: no force, potential -+ M / r0
        assert np.abs(ew["f"]).max() < 1e-10
        assert np.allclose(ew["phi"], -q * MADELUNG_NACL / r0, rtol=0, atol=1e-10)


def test_ewald_forces_and_potentials_are_its_gradients():
    pos, q, L = _cloud(60, (14.0, 17.0, 15.0), seed=5)
    run = lambda p, c: oracle.ewald(*p, c, box_lo=(0, 0, 0), box_len=L)
    ref = run(pos, q)
    for i, d in ((0, 0), (7, 1), (33, 2)):
        a, b = pos.copy(), pos.copy()
        a[d, i] += 1e-5
        b[d, i] -= 1e-5
        fd = (run(a, q)["energy"] - run(b, q)["energy"]) / 2e-5
        assert abs(fd + ref["f"][d, i]) < 1e-6 * max(1.0, abs(ref["f"][d, i]))
        c1, c2 = q.copy(), q.copy()
        c1[i] += 1e-5
        c2[i] -= 1e-5
        fd = (run(pos, c1)["energy"] - run(pos, c2)["energy"]) / 2e-5
        assert abs(fd - ref["phi"][i]) < 1e-6 * max(1.0, abs(ref["phi"][i]))


def test_periodic_msm_converges_to_ewald():
    """A random +-1 cloud: force error against Ewald of a few 1e-3 (cubic),
    several times smaller for the quintic basis, and far smaller again with a
    larger cutoff on a finer grid."""
    pos, q, L = _cloud()
    ew = oracle.ewald(*pos, q, box_lo=(0, 0, 0), box_len=L)
    err = {}
    for tag, prm in (("cubic", dict(cutoff=8.0, spacing=1.5, order=4)),
                     ("quintic", dict(cutoff=8.0, spacing=1.5, order=6)),
                     ("quintic_fine", dict(cutoff=10.0, spacing=1.0, order=6))):
        m = oracle.msm(*pos, q, box_lo=(0, 0, 0), box_len=L, periodic=True, **prm)
        err[tag] = (np.linalg.norm(m["f"] - ew["f"]) / np.linalg.norm(ew["f"]),
                    abs(m["energy"] - ew["energy"]) / abs(ew["energy"]))
    assert err["cubic"][0] < 5e-3 and err["cubic"][1] < 2e-3
    assert err["quintic"][0] < 0.4 * err["cubic"][0]
    assert err["quintic_fine"][0] < 0.2 * err["quintic"][0] and err["quintic_fine"][1] < 2e-5


def test_periodic_msm_gives_the_madelung_energy():
    pos, q, L = _rock_salt(4, 2.82)           # 512 ions, L = 22.56 A, h = L / 16
    m = oracle.msm(*pos, q, cutoff=8.0, spacing=L / 16, order=6, box_lo=(0, 0, 0), box_len=(L, L, L),
                   periodic=True)
    per_pair = m["energy"] / (0.5 * q.size)
    assert abs(per_pair + MADELUNG_NACL / 2.82) < 1e-3 * MADELUNG_NACL / 2.82


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_every_level_count_approximates_ewald(levels):
    """A box of 16 x 20 x 24 level-0 nodes: one level (the periodic kernel on
    the finest grid), two and three (the top grid 4 x 5 x 6)."""
    pos, q, L = _cloud(500, (24.0, 30.0, 36.0), seed=4)
    ew = oracle.ewald(*pos, q, box_lo=(0, 0, 0), box_len=L)
    m = oracle.msm(*pos, q, cutoff=8.0, spacing=1.5, order=6, levels=levels, box_lo=(0, 0, 0), box_len=L,
                   periodic=True)
    assert m["levels"] == levels
    assert np.linalg.norm(m["f"] - ew["f"]) / np.linalg.norm(ew["f"]) < 1e-3
    assert abs(m["energy"] - ew["energy"]) < 1e-3 * abs(ew["energy"])


def test_lattice_shifts_of_atoms_change_nothing():
    pos, q, L = _cloud(300, (24.0, 30.0, 27.0), seed=6)
    rng = np.random.default_rng(7)
    shifted = pos + L[:, None] * rng.integers(-2, 3, size=pos.shape)
    prm = dict(cutoff=8.0, spacing=1.5, order=6, box_lo=(0, 0, 0), box_len=L, periodic=True)
    a, b = oracle.msm(*pos, q, **prm), oracle.msm(*shifted, q, **prm)
    assert abs(a["energy"] - b["energy"]) < 1e-12 * abs(a["energy"])
    assert np.abs(a["f"] - b["f"]).max() < 1e-11 and np.abs(a["phi"] - b["phi"]).max() < 1e-11


def test_periodic_msm_forces_and_potentials_are_gradients():
    pos, q, L = _cloud(80, (16.0, 16.0, 20.0), seed=8)
    prm = dict(cutoff=6.0, spacing=1.0, order=4, levels=2, box_lo=(0, 0, 0), box_len=L, periodic=True)
    run = lambda p, c: oracle.msm(*p, c, **prm)
    ref = run(pos, q)
    for i, d in ((0, 0), (11, 2), (50, 1)):
        a, b = pos.copy(), pos.copy()
        a[d, i] += 1e-5
        b[d, i] -= 1e-5
        fd = (run(a, q)["energy"] - run(b, q)["energy"]) / 2e-5
        assert abs(fd + ref["f"][d, i]) < 1e-6 * max(1.0, abs(ref["f"][d, i]))
        c1, c2 = q.copy(), q.copy()
        c1[i] += 1e-5
        c2[i] -= 1e-5
        fd = (run(pos, c1)["energy"] - run(pos, c2)["energy"]) / 2e-5
        assert abs(fd - ref["phi"][i]) < 1e-6 * max(1.0, abs(ref["phi"][i]))


def test_periodic_top_kernel_is_symmetric_and_layout_is_checked():
    prm = dict(cutoff=8.0, spacing=1.5, order=6, levels=2, box_lo=(0, 0, 0), box_len=(24.0, 30.0, 36.0))
    K = oracle.periodic_top_kernel(**prm)
    assert K.shape == (12, 10, 8)
    flip = K[(-np.arange(12)) % 12][:, (-np.arange(10)) % 10][:, :, (-np.arange(8)) % 8]
    assert np.allclose(K, flip, rtol=1e-13, atol=1e-13)
    with pytest.raises(oracle.OracleError):               # box not a multiple of the spacing
        oracle.periodic_layout(**dict(prm, box_len=(24.0, 30.0, 36.7)))
    with pytest.raises(oracle.OracleError):               # 2 a > box edge
        oracle.periodic_layout(**dict(prm, cutoff=12.5))
    with pytest.raises(oracle.OracleError):               # 18 nodes cannot halve twice
        oracle.periodic_layout(**dict(prm, levels=3, box_len=(24.0, 27.0, 36.0)))
