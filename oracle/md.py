"""FP64 time stepping of the oracle (test infrastructure only).

Only the test suite and the benchmark's CPU-baseline leg may import this
module; the GPU path shares no code with it.

Velocity Verlet as the thesis writes it (Sec. 2.1 "Simulation loop"): half
kick with the current acceleration, drift, new forces, half kick.  The
parareal iteration of eq. (parareal): lambda_{n+1}^{k+1} = G(lambda_n^{k+1})
+ F(lambda_n^k) - G(lambda_n^k), with lambda^0 from a sequential sweep of G.
Forces come from the oracle's MSM (``oracle.msm``) or pair methods
(``oracle.pair``) in float64.  A state is a pair (pos, vel) of [3, N] float64
arrays.
"""
from __future__ import annotations

import numpy as np

import oracle


def msm_force(q, **params):
    """Force function r -> F (float64 [3, N]) of the oracle MSM with charges q
    and `params` (cutoff, spacing, order, split_m, levels, box_lo, box_len)."""
    q = np.asarray(q, dtype=np.float64)

    def force(pos):
        return oracle.msm(pos[0], pos[1], pos[2], q, **params)["f"]
    return force


def pair_force(q, **params):
    """Force function of an oracle pair method (kind, cutoff, alpha, box_lo, box_len)."""
    q = np.asarray(q, dtype=np.float64)

    def force(pos):
        return oracle.pair(pos[0], pos[1], pos[2], q, **params)["f"]
    return force


def velocity_verlet(force, pos, vel, inv_mass, n_steps, dt, accel_scale):
    """n_steps steps of velocity Verlet (Sec. 2.1): with a = s F / m,
    v(t + dt/2) = v(t) + a(t) dt / 2; r(t + dt) = r(t) + v(t + dt/2) dt;
    a(t + dt) from the forces at r(t + dt); v(t + dt) = v(t + dt/2) + a(t + dt) dt / 2.
    Returns (pos, vel, F at the final positions)."""
    pos = np.array(pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    w = accel_scale * np.asarray(inv_mass, dtype=np.float64)
    f = force(pos)
    for _ in range(n_steps):
        vel = vel + 0.5 * dt * w * f
        pos = pos + dt * vel
        f = force(pos)
        vel = vel + 0.5 * dt * w * f
    return pos, vel, f


def propagator(force, inv_mass, n_steps, dt, accel_scale):
    """One time slice: state -> state after n_steps velocity Verlet steps."""
    def prop(state):
        p, v, _ = velocity_verlet(force, state[0], state[1], inv_mass, n_steps, dt, accel_scale)
        return (p, v)
    return prop


def parareal(fine, coarse, state0, slices, max_iter, tol=0.0):
    """Parareal over time points 0 .. slices (eq. (parareal)).  fine and coarse
    map a state to the state one slice later.  Initial guess: lambda_{t+1} =
    G(lambda_t) in sequence.  Iteration k computes F(lambda_t) for every t,
    then in order for t = k .. slices - 1 sets lambda_{t+1} = F(lambda_t^old)
    + (G(lambda_t^new) - G(lambda_t^old)); slices before k are final.  Stops
    after the first iteration whose largest position change is <= tol, or
    after max_iter.  Returns (states, iterations, residuals)."""
    lam = [(np.array(state0[0], dtype=np.float64), np.array(state0[1], dtype=np.float64))]
    g = []
    for t in range(slices):
        nxt = coarse(lam[t])
        g.append(nxt)
        lam.append(nxt)
    residuals = []
    for k in range(max_iter):
        f = [fine(lam[t]) for t in range(slices)]
        change = 0.0
        for t in range(k, slices):
            gn = coarse(lam[t])
            new = tuple(f[t][c] + (gn[c] - g[t][c]) for c in range(2))
            change = max(change, float(np.max(np.abs(new[0] - lam[t + 1][0]))))
            g[t] = gn
            lam[t + 1] = new
        residuals.append(change)
        if change <= tol:
            break
    return lam, len(residuals), residuals
