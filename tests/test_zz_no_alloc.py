"""msm_compute_static: the evaluation without a caller workspace and without
device allocation, against msm_compute on the same plan (same kernels and
tuning, so the results must agree bitwise), on two calls in a row of which
the second is a smaller system (the static array then holds the first plan's
tables and must be rewritten), and again on the first plan after that."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1402_7216_amd import inputs
from _helpers import ENERGY_RTOL, FORCE_RTOL, rel_err, rel_rms

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    from paper_1402_7216_amd import msm
    msm.lib()
    return msm


def test_oversized_plan_is_rejected_before_any_launch(M):
    """A plan whose workspace exceeds the 64 MiB static array is refused with
    MSM_ERR_UNSUPPORTED (checked on the host; null pointers are never read)."""
    p = M.make_params(12.0, 2.5, order=6, box_len=(300.0,) * 3)
    h = ctypes.c_void_p()
    assert M.lib().msm_plan_create(ctypes.byref(p), 2_000_000, ctypes.byref(h)) == 0
    nb = ctypes.c_size_t()
    assert M.lib().msm_workspace_bytes(h, ctypes.byref(nb)) == 0
    assert nb.value > 64 << 20
    code = M.lib().msm_compute_static(h, None, *([None] * 10))
    assert code == M.ERR_UNSUPPORTED
    assert b"static array" in M.lib().msm_last_error()
    M.lib().msm_plan_destroy(h)


def _fresh_out(s):
    dev = "cuda"
    return {"energy": torch.full((1,), float("nan"), dtype=torch.float64, device=dev),
            "f": torch.full((3, s.n), float("nan"), dtype=torch.float32, device=dev),
            "phi": torch.full((s.n,), float("nan"), dtype=torch.float32, device=dev),
            "virial": torch.full((9,), float("nan"), dtype=torch.float64, device=dev)}


@pytest.mark.gpu
def test_static_entry_point_matches_workspace_entry_point(M):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    big = inputs.water_box(9000, seed=61, cutoff=10.0, spacing=2.0, order=4, levels=3)
    small = inputs.water_box(3000, seed=62, cutoff=9.0, spacing=2.0, order=6, levels=3)
    plans = {}
    for tag, s in (("big", big), ("small", small), ("big again", big)):
        print(f"case static {tag} n={s.n}", flush=True)
        if s.name not in plans:
            plans[s.name] = M.plan_for(s)
        plan = plans[s.name]
        x, y, z, q = M.to_device(s)
        ref = plan.compute(x, y, z, q, virial=True)
        ref = {k: v.clone() for k, v in ref.items()}
        torch.cuda.synchronize()
        plan.check()
        out = plan.compute_static(x, y, z, q, _fresh_out(s))
        torch.cuda.synchronize()
        for k in ("energy", "f", "phi", "virial"):
            assert torch.equal(out[k], ref[k]), (tag, k)
        r = oracle.system_msm(s)
        e = float(out["energy"].item())
        f = out["f"].double().cpu().numpy()
        print(f"  static {tag}: e_rel {rel_err(e, r['energy']):.2e} f_rms {rel_rms(f, r['f']):.2e}",
              flush=True)
        assert rel_err(e, r["energy"]) <= ENERGY_RTOL
        assert rel_rms(f, r["f"]) <= FORCE_RTOL
