"""GPU time stepping through the C ABI: velocity Verlet (msm_vv_run,
msm_batch_vv_run) and the parareal window (msm_parareal_run) against the
FP64 oracle's integrator and parareal iteration on the same inputs, plus the
exact properties of the iteration (a slice whose start state is final equals
the sequential fine propagation bit for bit).

Bars (trajectories over at most 48 fs of a 512-ion rock-salt cluster):
positions within 1e-4 A (max over atoms and coordinates) and velocities
within 1e-5 A/fs of the oracle; float32 positions round by ~2e-6 A per step
near 30 A, and the force error (1e-6 relative) moves a velocity by far less.
"""
import numpy as np
import pytest

import oracle
from oracle import md
from paper_1402_7216_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

S = inputs.ACCEL_SCALE
POS_TOL = 1e-4
VEL_TOL = 1e-5
TUNING = dict(lattice_b=4, item_chunks=1, short_blocks=-1, streams=2, short_after=1, short_split=1000,
              cell_reach=2)


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1402_7216_amd import msm
    msm.lib()
    return msm


def _dev(M, ions):
    s = ions.system
    x, y, z, q = M.to_device(s)
    pos = torch.stack([x, y, z]).contiguous()
    vel = torch.from_numpy(ions.vel).cuda().contiguous()
    im = torch.from_numpy(ions.inv_mass).cuda()
    return pos, vel, q, im


def _oracle_force(s):
    return md.msm_force(s.q, cutoff=s.cutoff, spacing=s.spacing, order=s.order, levels=s.levels,
                        split_m=s.split_m, box_lo=s.box_lo, box_len=s.box_len)


def _check_state(tag, pos, vel, rpos, rvel):
    dp = float(np.max(np.abs(pos - rpos)))
    dv = float(np.max(np.abs(vel - rvel)))
    print(f"[{tag}] max |dr| {dp:.2e} A  max |dv| {dv:.2e} A/fs", flush=True)
    assert dp <= POS_TOL and dv <= VEL_TOL


def test_velocity_verlet_matches_oracle(M):
    ions = inputs.rock_salt(8, seed=11)
    s = ions.system
    print(f"case vv rocksalt n={s.n}", flush=True)
    plan = M.plan_for(s)
    pos, vel, q, im = _dev(M, ions)
    f = plan.vv_run(pos, vel, q, im, 20, 2.0, S)
    torch.cuda.synchronize()
    plan.check()
    rp, rv, rf = md.velocity_verlet(_oracle_force(s), s.pos64(), ions.vel, ions.inv_mass, 20, 2.0, S)
    _check_state("vv", pos.double().cpu().numpy(), vel.double().cpu().numpy(), rp, rv)
    assert float(np.max(np.abs(pos.double().cpu().numpy() - s.pos64()))) > 1e-2      # the ions moved
    fd = f.double().cpu().numpy()
    assert np.linalg.norm(fd - rf) / np.linalg.norm(rf) <= 1e-4


def test_batched_velocity_verlet_equals_single_plans_bitwise(M):
    """Three clusters advanced together (one batched evaluation per force
    call) give exactly the single-plan trajectories with the same tuning."""
    ions = [inputs.rock_salt(6, seed=20 + k) for k in range(3)]
    print(f"case batch vv n={[i.system.n for i in ions]}", flush=True)
    b = M.batch_for([i.system for i in ions])
    b.tune(**TUNING)
    devs = [_dev(M, i) for i in ions]
    cat = lambda j: torch.cat([d[j] for d in devs], dim=-1).contiguous()
    pos, vel, q, im = cat(0), cat(1), cat(2), cat(3)
    fb = b.vv_run(pos, vel, q, im, 6, 2.0, S)
    off = 0
    for i, (p1, v1, q1, m1) in zip(ions, devs):
        plan = M.plan_for(i.system)
        plan.tune(**TUNING)
        f1 = plan.vv_run(p1, v1, q1, m1, 6, 2.0, S)
        n = i.system.n
        assert torch.equal(pos[:, off:off + n], p1) and torch.equal(vel[:, off:off + n], v1)
        assert torch.equal(fb[:, off:off + n], f1)
        off += n
    b.check()


def _parareal_setup(M, T, kind="shifted_force", n_side=8, seed=12):
    ions = inputs.rock_salt(n_side, seed=seed)
    s = ions.system
    fine = M.batch_for([s] * T)
    fine.tune(**TUNING)
    coarse = M.pair_plan_for(s, kind, alpha=0.2)
    pos, vel, q, im = _dev(M, ions)
    state0 = torch.cat([pos, vel]).contiguous()
    return ions, s, fine, coarse, state0, q, im


def test_parareal_final_slices_equal_sequential_fine_bitwise(M):
    """After K iterations the first K slices are K sequential fine
    propagations bit for bit (single plan, same tuning); later slices are
    not yet."""
    T, steps, dt = 4, 3, 2.0
    ions, s, fine, coarse, state0, q, im = _parareal_setup(M, T)
    print(f"case parareal exact n={s.n} T={T}", flush=True)
    plan = M.plan_for(s)
    plan.tune(**TUNING)
    seq = [state0.clone()]
    for _ in range(T):
        st = seq[-1].clone()
        p, v = st[:3].contiguous(), st[3:].contiguous()
        plan.vv_run(p, v, q, im, steps, dt, S)
        seq.append(torch.cat([p, v]))
    for K in (1, 2):
        states, it, res = M.parareal(fine, coarse, q, im, state0, slices=T, steps_per_slice=steps, dt=dt,
                                     accel_scale=S, max_iter=K, tol=0.0)
        assert it == K and len(res) == K
        for t in range(K + 1):
            assert torch.equal(states[:, t], seq[t]), (K, t)
        assert not torch.equal(states[:, T], seq[T])


def test_parareal_matches_oracle_and_converges(M):
    """Shifted-force cutoff as the coarse function: the GPU window follows the
    oracle's parareal iteration slice by slice for the same number of
    iterations, and with tol = 1e-5 A it stops before T iterations with the
    position change shrinking every iteration."""
    T, steps, dt = 6, 4, 2.0
    ions, s, fine, coarse, state0, q, im = _parareal_setup(M, T)
    print(f"case parareal oracle n={s.n} T={T}", flush=True)
    states, it, res = M.parareal(fine, coarse, q, im, state0, slices=T, steps_per_slice=steps, dt=dt,
                                 accel_scale=S, max_iter=T, tol=1e-5)
    print(f"  iterations {it} changes {res}", flush=True)
    assert it <= T - 1 and res[-1] <= 1e-5
    assert all(b < 0.5 * a for a, b in zip(res, res[1:]))
    fine_o = md.propagator(_oracle_force(s), ions.inv_mass, steps, dt, S)
    coarse_o = md.propagator(md.pair_force(s.q, kind="shifted_force", cutoff=s.cutoff, box_lo=s.box_lo,
                                           box_len=s.box_len), ions.inv_mass, steps, dt, S)
    lam, it_o, res_o = md.parareal(fine_o, coarse_o, (s.pos64(), ions.vel.astype(np.float64)), T, it, tol=0.0)
    st = states.double().cpu().numpy()
    for t in range(T + 1):
        _check_state(f"slice {t}", st[:3, t], st[3:, t], lam[t][0], lam[t][1])


def test_parareal_rejects_inconsistent_shapes(M):
    ions, s, fine, coarse, state0, q, im = _parareal_setup(M, 3, n_side=4)
    with pytest.raises(M.MSMError):
        M.parareal(fine, coarse, q, im, state0, slices=4, steps_per_slice=2, dt=1.0, accel_scale=S)
    with pytest.raises(M.MSMError):
        M.parareal(fine, coarse, q, im, state0, slices=3, steps_per_slice=0, dt=1.0, accel_scale=S)


def test_velocity_verlet_in_a_periodic_crystal_matches_oracle(M):
    """A rock-salt crystal that tiles its periodic box (512 ions, 300 K): ions
    crossing a face keep their unwrapped coordinates and interact through
    their images; the GPU trajectory follows the oracle's."""
    import dataclasses
    ions = inputs.rock_salt(8, seed=13, margin=0.5 * 2.82, temperature=300.0, cutoff=8.0, grid=1.5, levels=2)
    s = ions.system
    # the crystal shifted so a layer of ions sits on the x = 0 face
    p = s.pos64() - np.array([[0.5 * 2.82], [0.0], [0.0]])
    s = dataclasses.replace(s, spacing=inputs.periodic_spacing(s.box_len[0], 1.5, 2), x=p[0].astype(np.float32),
                            x64=p)
    ions = dataclasses.replace(ions, system=s)
    print(f"case vv periodic rocksalt n={s.n} h={s.spacing:.4f}", flush=True)
    plan = M.plan_for(s, periodic=True)
    pos, vel, q, im = _dev(M, ions)
    f = plan.vv_run(pos, vel, q, im, 20, 2.0, S)
    torch.cuda.synchronize()
    plan.check()
    force = md.msm_force(s.q, cutoff=s.cutoff, spacing=s.spacing, order=s.order, levels=s.levels,
                         box_lo=s.box_lo, box_len=s.box_len, periodic=True)
    rp, rv, rf = md.velocity_verlet(force, s.pos64(), ions.vel, ions.inv_mass, 20, 2.0, S)
    p_gpu = pos.double().cpu().numpy()
    _check_state("vv periodic", p_gpu, vel.double().cpu().numpy(), rp, rv)
    lo, hi = np.asarray(s.box_lo)[:, None], np.asarray(s.box_lo)[:, None] + np.asarray(s.box_len)[:, None]
    assert ((rp < lo) | (rp > hi)).any()                  # some ions lie outside the box
    fd = f.double().cpu().numpy()
    assert np.linalg.norm(fd - rf) / np.linalg.norm(rf) <= 1e-4
