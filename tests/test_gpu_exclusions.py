"""GPU bonded exclusions (msm_set_exclusions / msm_batch_set_exclusions)
against the FP64 oracle with the same exclusion lists: the water boxes with
every intramolecular pair excluded, through the forces path, the
energy-only path and the adjoint backward, the batch, and the cheap pair
methods.

Bars: forces and potentials within 1e-5 relative RMS.  The energy of a water
box without its intramolecular pairs is a small difference of two large sums
(the full evaluation and the excluded pairs' q_i q_j / r, about 20 times
larger for 24,000 atoms), and both carry float32 rounding relative to their own
size; the energy bar is therefore 1e-7 of |E| + |E_excluded pairs|.
"""
import numpy as np
import pytest

import oracle
from paper_1402_7216_amd import inputs
from _helpers import FORCE_RTOL, PHI_RTOL, rel_err, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1402_7216_amd import msm
    msm.lib()
    return msm


def _check(tag, e, f, phi, ref, scale):
    err_e = abs(e - ref["energy"]) / scale
    print(f"[{tag}] E_gpu={e:.10g} E_ref={ref['energy']:.10g} e_err/scale={err_e:.2e} "
          f"f_rms={rel_rms(f, ref['f']):.2e} phi_rms={rel_rms(phi, ref['phi']):.2e}", flush=True)
    assert err_e <= 1e-7
    assert rel_rms(f, ref["f"]) <= FORCE_RTOL
    assert rel_rms(phi, ref["phi"]) <= PHI_RTOL


def _scale(s, excl, ref, **kw):
    ex = oracle.exclusion_terms(s.x, s.y, s.z, s.q, *excl, **kw)
    return abs(ref["energy"]) + abs(ex["energy"])


@pytest.mark.parametrize("name", ["water24k", "water9k_quintic"])
def test_water_without_intramolecular_pairs_matches_oracle(M, name):
    s = inputs.water_24k() if name == "water24k" else inputs.water_box(9000, seed=51, cutoff=10.0, spacing=2.2,
                                                                       order=6, levels=3)
    excl = inputs.water_exclusions(s.n)
    print(f"case {name} n={s.n}", flush=True)
    plan = M.plan_for(s)
    x, y, z, q = M.to_device(s)
    base = {k: v.clone() for k, v in plan.compute(x, y, z, q).items()}
    plan.set_exclusions(*excl)
    out = plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    plan.check()
    ref = oracle.system_msm(s, exclusions=excl)
    _check(name, float(out["energy"].item()), out["f"].double().cpu().numpy(), out["phi"].double().cpu().numpy(),
           ref, _scale(s, excl, ref))
    # removing the lists gives back the plain evaluation bit for bit
    plan.set_exclusions(None, None)
    again = plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    assert torch.equal(again["f"], base["f"]) and torch.equal(again["energy"], base["energy"])


def test_energy_and_backward_with_exclusions_match_oracle(M):
    """The differentiable path: energy-only forward and the adjoint backward
    (dE/dr = -F, dE/dq = phi of the oracle with the same exclusions)."""
    s = inputs.water_box(12000, seed=52, cutoff=10.0, spacing=2.0, order=4, levels=0)
    excl = inputs.water_exclusions(s.n)
    print(f"case autograd exclusions n={s.n}", flush=True)
    plan = M.plan_for(s)
    plan.set_exclusions(*excl)
    x, y, z, q = M.to_device(s)
    pos = torch.stack([x, y, z]).contiguous().requires_grad_(True)
    qq = q.clone().requires_grad_(True)
    e = M.energy(plan, pos, qq)
    e.backward()
    torch.cuda.synchronize()
    ref = oracle.system_msm(s, exclusions=excl)
    scale = _scale(s, excl, ref)
    err_e = abs(float(e.item()) - ref["energy"]) / scale
    gr = pos.grad.double().cpu().numpy()
    gq = qq.grad.double().cpu().numpy()
    print(f"  e_err/scale={err_e:.2e} dEdr_rms={rel_rms(-gr, ref['f']):.2e} dEdq_rms={rel_rms(gq, ref['phi']):.2e}",
          flush=True)
    assert err_e <= 1e-7
    assert rel_rms(-gr, ref["f"]) <= FORCE_RTOL and rel_rms(gq, ref["phi"]) <= PHI_RTOL


def test_batch_with_exclusions_matches_oracle(M):
    reps = [inputs.water_box(n, seed=60 + k, cutoff=10.0, spacing=2.0, order=4, levels=0)
            for k, n in enumerate((3000, 6600, 4500))]
    offs = np.cumsum([0] + [r.n for r in reps])
    parts, idxs, nnz = [], [], 0
    for r, o in zip(reps, offs):
        st, ix = inputs.water_exclusions(r.n, offset=int(o))      # global partner indices
        parts.append(st[:-1] + nnz)
        idxs.append(ix)
        nnz += len(ix)
    start = np.concatenate(parts + [np.array([nnz], dtype=np.int32)]).astype(np.int32)
    idx = np.concatenate(idxs)
    print(f"case batch exclusions n={[r.n for r in reps]}", flush=True)
    b = M.batch_for(reps)
    b.set_exclusions(start, idx)
    x, y, z, q = M.batch_to_device(reps)
    out = b.compute(x, y, z, q)
    torch.cuda.synchronize()
    b.check()
    for k, r in enumerate(reps):
        lo, hi = int(offs[k]), int(offs[k + 1])
        ex = inputs.water_exclusions(r.n)
        ref = oracle.system_msm(r, exclusions=ex)
        _check(f"replica {k}", float(out["energy"][k].item()), out["f"][:, lo:hi].double().cpu().numpy(),
               out["phi"][lo:hi].double().cpu().numpy(), ref, _scale(r, ex, ref))


@pytest.mark.parametrize("kind", ["cutoff", "shifted_force", "wolf"])
def test_pair_methods_with_exclusions_match_oracle(M, kind):
    s = inputs.water_box(9000, seed=53, cutoff=10.0, spacing=2.0, order=4, levels=3)
    excl = inputs.water_exclusions(s.n)
    print(f"case pair {kind} exclusions n={s.n}", flush=True)
    plan = M.pair_plan_for(s, kind, alpha=0.2)
    plan.set_exclusions(*excl)
    x, y, z, q = M.to_device(s)
    out = plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    plan.check()
    prm = dict(kind=kind, cutoff=s.cutoff, alpha=0.2, box_lo=s.box_lo, box_len=s.box_len, f32_cut=True)
    ref = oracle.pair(s.x, s.y, s.z, s.q, exclusions=excl, **prm)
    ex = oracle.exclusion_terms(s.x, s.y, s.z, s.q, *excl, kind=kind, cutoff=s.cutoff, alpha=0.2, f32_cut=True)
    _check(kind, float(out["energy"].item()), out["f"].double().cpu().numpy(), out["phi"].double().cpu().numpy(),
           ref, abs(ref["energy"]) + abs(ex["energy"]))


def test_out_of_range_partner_is_reported(M):
    s = inputs.water_box(300, seed=54, cutoff=8.0, spacing=2.0, order=4, levels=2)
    start, idx = inputs.water_exclusions(s.n)
    idx = idx.copy()
    idx[7] = s.n + 5                      # names an atom outside the system
    plan = M.plan_for(s)
    plan.set_exclusions(start, idx)
    x, y, z, q = M.to_device(s)
    plan.compute(x, y, z, q)
    code, flags = plan.status()
    assert code == -1 and flags & 8
