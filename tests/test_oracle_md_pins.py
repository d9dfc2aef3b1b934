"""Pins of the oracle's time stepping (velocity Verlet, Sec. 2.1 "Simulation
loop"; parareal, eq. (parareal)) against facts other than its own code: the
circular orbit of two opposite charges (closed form), time reversibility and
energy conservation of velocity Verlet, and the parareal iteration's exact
convergence (the first k slices equal k sequential fine propagations after k
iterations; a coarse function equal to the fine one converges at once)."""
import math

import numpy as np
import pytest

import oracle
from oracle import md
from paper_1402_7216_amd import inputs

S = inputs.ACCEL_SCALE


def _coulomb(q, lo=(0.0, 0.0, 0.0), side=60.0):
    # the plain cutoff with rc beyond the box is the Coulomb sum
    return md.pair_force(q, kind="cutoff", cutoff=1e3, box_lo=lo, box_len=(side,) * 3)


def test_two_opposite_charges_follow_the_circular_orbit():
    """q = +1 (m1) and -1 (m2) at distance R with the relative speed of a
    circular orbit, v^2 = s (1/m1 + 1/m2) / R: after a quarter period the
    separation has turned by 90 degrees at the same length; the centre of
    mass stays at rest; the energy is conserved to O(dt^2)."""
    m1, m2, R = inputs.NA_MASS, inputs.CL_MASS, 3.0
    v = math.sqrt(S * (1.0 / m1 + 1.0 / m2) / R)
    period = 2.0 * math.pi * R / v
    pos = np.array([[30.0 + R * m2 / (m1 + m2), 30.0 - R * m1 / (m1 + m2)], [30.0, 30.0], [30.0, 30.0]])
    vel = np.array([[0.0, 0.0], [v * m2 / (m1 + m2), -v * m1 / (m1 + m2)], [0.0, 0.0]])
    q = np.array([1.0, -1.0])
    inv_m = np.array([1.0 / m1, 1.0 / m2])
    n = 4000
    p1, v1, _ = md.velocity_verlet(_coulomb(q), pos, vel, inv_m, n, period / 4.0 / n, S)
    rel = p1[:, 0] - p1[:, 1]
    assert np.allclose(rel, [0.0, R, 0.0], atol=1e-5 * R)
    com = (m1 * p1[:, 0] + m2 * p1[:, 1]) / (m1 + m2)
    assert np.allclose(com, 30.0, atol=1e-9)
    ke = lambda vv: 0.5 * (m1 * vv[:, 0] @ vv[:, 0] + m2 * vv[:, 1] @ vv[:, 1])
    e0 = ke(vel) / S - 1.0 / R
    e1 = ke(v1) / S - 1.0 / np.linalg.norm(rel)
    assert abs(e1 - e0) < 1e-6 * abs(e0)


def _ions(n_side=4, seed=7):
    ions = inputs.rock_salt(n_side, seed, cutoff=6.0, grid=2.0, margin=6.0)
    s = ions.system
    force = md.msm_force(s.q, cutoff=s.cutoff, spacing=s.spacing, order=s.order, levels=s.levels,
                         box_lo=s.box_lo, box_len=s.box_len)
    return ions, s, force


def test_velocity_verlet_is_time_reversible():
    ions, s, force = _ions()
    p0, v0 = s.pos64(), ions.vel.astype(np.float64)
    p1, v1, _ = md.velocity_verlet(force, p0, v0, ions.inv_mass, 10, 2.0, S)
    p2, v2, _ = md.velocity_verlet(force, p1, -v1, ions.inv_mass, 10, 2.0, S)
    assert np.max(np.abs(p2 - p0)) < 1e-10 and np.max(np.abs(v2 + v0)) < 1e-12
    assert np.max(np.abs(p1 - p0)) > 1e-3          # the ions did move


def test_velocity_verlet_conserves_msm_energy():
    """Total energy with the oracle's own MSM energy (forces are its exact
    gradient): the drift over 40 steps shrinks as dt^2."""
    ions, s, force = _ions()
    m = 1.0 / ions.inv_mass.astype(np.float64)
    prm = dict(cutoff=s.cutoff, spacing=s.spacing, order=s.order, levels=s.levels, box_lo=s.box_lo,
               box_len=s.box_len)

    def total(p, v):
        return 0.5 * float(np.sum(m * v * v)) / S + oracle.msm(p[0], p[1], p[2], s.q, **prm)["energy"]

    p0, v0 = s.pos64(), ions.vel.astype(np.float64) * 3.0      # warmer, so the energy moves
    e0 = total(p0, v0)
    errs = []
    for dt, n in ((2.0, 20), (1.0, 40)):
        p, v, _ = md.velocity_verlet(force, p0, v0, ions.inv_mass, n, dt, S)
        errs.append(abs(total(p, v) - e0))
    assert errs[0] < 5e-4 * abs(e0)
    assert 3.0 < errs[0] / errs[1] < 5.0           # second order


def test_parareal_slices_become_exact_one_per_iteration():
    """With a poor coarse function (free flight), after k iterations the first
    k slices equal k sequential fine propagations bit for bit, and after all
    T iterations every slice does."""
    ions, s, force = _ions()
    T, steps, dt = 4, 3, 2.0
    fine = md.propagator(force, ions.inv_mass, steps, dt, S)
    free = md.propagator(lambda p: np.zeros_like(p), ions.inv_mass, steps, dt, S)
    x0 = (s.pos64(), ions.vel.astype(np.float64))
    seq = [x0]
    for _ in range(T):
        seq.append(fine(seq[-1]))
    for K in (1, 2, T):
        lam, it, res = md.parareal(fine, free, x0, T, K)
        assert it == K
        for t in range(K + 1):
            assert np.array_equal(lam[t][0], seq[t][0]) and np.array_equal(lam[t][1], seq[t][1]), (K, t)
        if K < T:
            assert np.max(np.abs(lam[T][0] - seq[T][0])) > 0.0
    assert res[-1] > 0.0


def test_parareal_with_the_fine_function_as_coarse_converges_at_once():
    ions, s, force = _ions()
    fine = md.propagator(force, ions.inv_mass, 3, 2.0, S)
    x0 = (s.pos64(), ions.vel.astype(np.float64))
    lam, it, res = md.parareal(fine, fine, x0, 4, 4, tol=0.0)
    assert it == 1 and res == [0.0]


def test_parareal_with_a_smoothed_cutoff_coarse_function_converges_fast():
    """G = shifted-force smoothed cutoff at the MSM cutoff: every iteration
    shrinks the position change several-fold, the change falls below 1e-5 A
    well before T iterations, and the converged last state is that close to
    the sequential fine propagation."""
    ions, s, force = _ions(n_side=5, seed=8)
    T, steps, dt = 6, 4, 2.0
    fine = md.propagator(force, ions.inv_mass, steps, dt, S)
    coarse = md.propagator(md.pair_force(s.q, kind="shifted_force", cutoff=s.cutoff, box_lo=s.box_lo,
                                         box_len=s.box_len), ions.inv_mass, steps, dt, S)
    x0 = (s.pos64(), ions.vel.astype(np.float64))
    lam, it, res = md.parareal(fine, coarse, x0, T, T, tol=1e-5)
    assert it <= T - 2 and res[-1] <= 1e-5
    assert all(b < 0.25 * a for a, b in zip(res, res[1:]))
    seq = x0
    for _ in range(T):
        seq = fine(seq)
    assert np.max(np.abs(lam[T][0] - seq[0])) < 1e-4
