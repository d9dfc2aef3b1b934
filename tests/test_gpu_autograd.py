"""GPU differentiable path: msm_energy / msm_backward behind torch.autograd.

The gradient of the method's own energy is dE/dr_i = -F_i and dE/dq_i = phi_i
exactly (the oracle pins show both by central differences).  Here the device
gradients are compared with the oracle's analytic gradient at the full
100k-atom size, and with central differences of the FP64 oracle energy
(steps 1e-4 A and 1e-6 e) on a sample of coordinates and charges.
"""
import numpy as np
import pytest

import oracle
from paper_1402_7216_amd import inputs
from _helpers import ENERGY_RTOL, FORCE_RTOL, PHI_RTOL, rel_err, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1402_7216_amd import msm
    msm.lib()
    return msm


def _tensors(s):
    pos = torch.from_numpy(np.stack([s.x, s.y, s.z])).cuda()
    q = torch.from_numpy(s.q.copy()).cuda()
    return pos, q


@pytest.mark.parametrize("name", ["cloud1k", "water24k"])
def test_energy_only_matches_compute_and_oracle(M, name):
    s = inputs.cloud_1k() if name == "cloud1k" else inputs.water_24k()
    print(f"case energy-only {name} n={s.n}", flush=True)
    plan = M.plan_for(s)
    x, y, z, q = M.to_device(s)
    e_only = float(plan.energy(x, y, z, q).item())
    e_full = float(plan.compute(x, y, z, q)["energy"].item())
    plan.check()
    ref = oracle.system_msm(s)["energy"]
    print(f"  E_only={e_only:.10g} E_full={e_full:.10g} E_ref={ref:.10g}", flush=True)
    assert rel_err(e_only, ref) <= ENERGY_RTOL
    assert rel_err(e_only, e_full) <= 2 * ENERGY_RTOL


def test_autograd_matches_oracle_gradient_water100k(M):
    s = inputs.water_100k()
    print(f"case autograd water100k n={s.n}", flush=True)
    plan = M.plan_for(s)
    pos, q = _tensors(s)
    pos.requires_grad_(True)
    q.requires_grad_(True)
    e = M.energy(plan, pos, q)
    assert e.dtype == torch.float64 and e.dim() == 0
    e.backward()
    torch.cuda.synchronize()
    plan.check()
    r = oracle.system_msm(s)
    gpos = pos.grad.double().cpu().numpy()
    gq = q.grad.double().cpu().numpy()
    print(f"  E rel {rel_err(e.item(), r['energy']):.2e} dE/dr rel_rms {rel_rms(gpos, -r['f']):.2e} "
          f"dE/dq rel_rms {rel_rms(gq, r['phi']):.2e}", flush=True)
    assert rel_err(e.item(), r["energy"]) <= ENERGY_RTOL
    assert rel_rms(gpos, -r["f"]) <= FORCE_RTOL
    assert rel_rms(gq, r["phi"]) <= PHI_RTOL


def test_autograd_scales_with_incoming_gradient(M):
    s = inputs.water_box(3000, seed=31, cutoff=9.0, spacing=2.0, order=4, levels=3)
    plan = M.plan_for(s)
    pos, q = _tensors(s)
    grads = []
    for scale in (1.0, -2.5):
        p = pos.clone().requires_grad_(True)
        c = q.clone().requires_grad_(True)
        (scale * M.energy(plan, p, c)).backward()
        grads.append((p.grad.double().cpu().numpy(), c.grad.double().cpu().numpy()))
    assert rel_rms(grads[1][0], -2.5 * grads[0][0]) < 1e-7
    assert rel_rms(grads[1][1], -2.5 * grads[0][1]) < 1e-7
    # position-only gradient leaves charges untouched
    p = pos.clone().requires_grad_(True)
    M.energy(plan, p, q).backward()
    assert q.grad is None
    assert rel_rms(p.grad.double().cpu().numpy(), grads[0][0]) < 1e-7


def test_autograd_vs_oracle_central_differences(M):
    """Central differences of the FP64 oracle energy (1e-4 A, 1e-6 e) on 32
    atoms x 3 coordinates and 32 charges of a 6,000-atom water box, against the
    device autograd gradient."""
    s = inputs.water_box(6000, seed=32, cutoff=10.0, spacing=2.0, order=4, levels=3)
    print(f"case finite differences n={s.n}", flush=True)
    plan = M.plan_for(s)
    pos, q = _tensors(s)
    pos.requires_grad_(True)
    q.requires_grad_(True)
    M.energy(plan, pos, q).backward()
    gpos = pos.grad.double().cpu().numpy()
    gq = q.grad.double().cpu().numpy()
    rng = np.random.default_rng(4)
    atoms = rng.choice(s.n, size=32, replace=False)
    p64 = s.pos64()
    q64 = s.q.astype(np.float64)
    prm = s.params()
    fd_pos, dev_pos, fd_q, dev_q = [], [], [], []
    for i in atoms:
        for d in range(3):
            pp, pm = p64.copy(), p64.copy()
            pp[d, i] += 1e-4
            pm[d, i] -= 1e-4
            fd = (oracle.msm(*pp, q64, **prm)["energy"] - oracle.msm(*pm, q64, **prm)["energy"]) / 2e-4
            fd_pos.append(fd)
            dev_pos.append(gpos[d, i])
        qp, qm = q64.copy(), q64.copy()
        qp[i] += 1e-6
        qm[i] -= 1e-6
        fd = (oracle.msm(*p64, qp, **prm)["energy"] - oracle.msm(*p64, qm, **prm)["energy"]) / 2e-6
        fd_q.append(fd)
        dev_q.append(gq[i])
    ep, eq = rel_rms(dev_pos, fd_pos), rel_rms(dev_q, fd_q)
    print(f"  dE/dr vs FD rel_rms {ep:.2e}; dE/dq vs FD rel_rms {eq:.2e}", flush=True)
    assert ep <= FORCE_RTOL and eq <= PHI_RTOL
