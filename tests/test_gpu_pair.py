"""GPU cheap pair methods (plain cutoff, shifted-force smoothed cutoff, Wolf
summation) through msm_pair_plan_create + msm_compute, against the FP64
oracle's pair methods on the same inputs.  Bars as for MSM: forces 1e-5
relative RMS, energy 1e-7 relative, potentials 1e-5 relative RMS."""
import numpy as np
import pytest

import oracle
from paper_1402_7216_amd import inputs
from _helpers import ENERGY_RTOL, FORCE_RTOL, PHI_RTOL, rel_err, rel_rms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KINDS = ["cutoff", "shifted_force", "wolf"]
ALPHA = 0.2


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1402_7216_amd import msm
    msm.lib()
    return msm


def _run(M, s, kind, reach=0):
    plan = M.pair_plan_for(s, kind, alpha=ALPHA)
    if reach:
        plan.tune(cell_reach=reach)
    x, y, z, q = M.to_device(s)
    o = plan.compute(x, y, z, q, virial=True)
    torch.cuda.synchronize()
    code, flags = plan.status()
    assert code == 0, flags
    return plan, o


def _check(o, r, s, tag):
    e = float(o["energy"].item())
    f = o["f"].double().cpu().numpy()
    phi = o["phi"].double().cpu().numpy()
    print(f"[{tag}] E_gpu={e:.10g} E_ref={r['energy']:.10g} e_rel={rel_err(e, r['energy']):.2e} "
          f"f_rms={rel_rms(f, r['f']):.2e} phi_rms={rel_rms(phi, r['phi']):.2e}", flush=True)
    assert rel_err(e, r["energy"]) <= ENERGY_RTOL
    assert rel_rms(f, r["f"]) <= FORCE_RTOL
    assert rel_rms(phi, r["phi"]) <= PHI_RTOL
    # the virial is the float64 sum of (r - lo) F over the device forces
    w = o["virial"].cpu().numpy().reshape(3, 3)
    pos = s.pos64() - np.asarray(s.box_lo)[:, None]
    scale = float(np.linalg.norm(pos, axis=0) @ np.linalg.norm(f, axis=0))
    assert np.linalg.norm(w - pos @ f.T) / scale < 1e-12


def _ref(s, kind):
    # the kernel decides r < rc in float32; the oracle takes that decision the
    # same way (a pair at the cutoff changes the plain-cutoff energy by q q / rc)
    return oracle.pair(s.x, s.y, s.z, s.q, kind=kind, cutoff=s.cutoff, alpha=ALPHA, box_lo=s.box_lo,
                       box_len=s.box_len, f32_cut=True)


@pytest.mark.parametrize("kind", KINDS)
def test_pair_methods_match_oracle_water24k(M, kind):
    s = inputs.water_24k()
    print(f"case pair {kind} water24k n={s.n}", flush=True)
    _, o = _run(M, s, kind)
    _check(o, _ref(s, kind), s, f"{kind}-24k")


@pytest.mark.parametrize("kind", KINDS)
def test_pair_methods_match_oracle_water100k_finer_cells(M, kind):
    s = inputs.water_100k()
    print(f"case pair {kind} water100k reach 4 n={s.n}", flush=True)
    _, o = _run(M, s, kind, reach=4)
    _check(o, _ref(s, kind), s, f"{kind}-100k")


def test_pair_small_and_degenerate_inputs(M):
    """Empty, one-atom and two-atom systems, and a ragged random cloud."""
    box = dict(box_lo=(0.0, 0.0, 0.0), box_len=(16.0, 16.0, 16.0))
    for n in (0, 1, 2, 777):
        rng = np.random.default_rng(200 + n)
        pos = rng.uniform(0, 16, (3, n)).astype(np.float32)
        q = rng.uniform(-1, 1, n).astype(np.float32)
        s = inputs.System(*pos, q, cutoff=6.0, spacing=2.0, order=4, levels=1, **box)
        for kind in KINDS:
            print(f"case pair {kind} n={n}", flush=True)
            plan = M.PairPlan(n, kind=kind, cutoff=6.0, alpha=0.3, **box)
            o = plan.compute(*M.to_device(s), virial=True)
            torch.cuda.synchronize()
            assert plan.status()[0] == 0
            r = oracle.pair(s.x, s.y, s.z, s.q, kind=kind, cutoff=6.0, alpha=0.3, f32_cut=True, **box)
            e = float(o["energy"].item())
            scale = max(abs(r["energy"]), float(np.abs(s.q.astype(np.float64)) @ np.abs(s.q)) / 6.0, 1e-30)
            assert abs(e - r["energy"]) <= 1e-7 * scale
            if n:
                f = o["f"].double().cpu().numpy()
                assert np.linalg.norm(f - r["f"]) <= FORCE_RTOL * max(np.linalg.norm(r["f"]), 1e-30) + 1e-12


def test_pair_graph_replay_and_unsupported_calls(M):
    s = inputs.water_box(6000, seed=71, cutoff=10.0, spacing=2.0, order=4, levels=3)
    plan = M.pair_plan_for(s, "wolf", alpha=ALPHA)
    x, y, z, q = M.to_device(s)
    ref = {k: v.clone() for k, v in plan.compute(x, y, z, q, virial=True).items()}
    out = {k: torch.full_like(v, float("nan")) for k, v in ref.items()}
    g = M.Graph(plan, x, y, z, q, out)
    for _ in range(3):
        g.launch()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(out[k], ref[k]), k
    with pytest.raises(M.MSMError) as err:
        plan.energy(x, y, z, q)
    assert err.value.code == M.ERR_UNSUPPORTED
    assert plan.describe()["pair"] == 3
