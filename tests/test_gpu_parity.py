"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: forces within 1e-5 relative RMS, energy within 1e-7 relative,
potentials within 1e-5 relative RMS; the virial is checked for consistency with
the forces (its error bounded by the force error).
Stage-wise checks compare the device grids with the oracle's grids.
"""
import numpy as np
import pytest

import oracle
from paper_1402_7216_amd import inputs
from _helpers import ENERGY_RTOL, FORCE_RTOL, PHI_RTOL, rel_err, rel_rms

pytestmark = pytest.mark.gpu

DEGENERATE_RTOL = 1e-6   # energy / potential bar relative to the self-interaction scale

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1402_7216_amd import msm
    msm.lib()
    return msm


def run_gpu(M, s, virial=True):
    plan = M.plan_for(s)
    x, y, z, q = M.to_device(s)
    out = plan.compute(x, y, z, q, virial=virial)
    torch.cuda.synchronize()
    code, flags = plan.status()
    res = dict(energy=float(out["energy"].item()), f=out["f"].double().cpu().numpy(),
               phi=out["phi"].double().cpu().numpy(), code=code, flags=flags, plan=plan)
    if virial:
        res["virial"] = out["virial"].cpu().numpy().reshape(3, 3)
        res["pos"] = s.pos64()
        res["lo"] = s.box_lo
    return res


def check_full(g, r, tag):
    print(f"[{tag}] E_gpu={g['energy']:.10g} E_ref={r['energy']:.10g} "
          f"e_rel={rel_err(g['energy'], r['energy']):.2e} f_rms={rel_rms(g['f'], r['f']):.2e} "
          f"phi_rms={rel_rms(g['phi'], r['phi']):.2e}", flush=True)
    assert g["code"] == 0, g["flags"]
    assert rel_rms(g["f"], r["f"]) <= FORCE_RTOL
    assert rel_err(g["energy"], r["energy"]) <= ENERGY_RTOL
    assert rel_rms(g["phi"], r["phi"]) <= PHI_RTOL
    if "virial" in g:
        check_virial(g, r)


def check_virial(g, r):
    """The device virial is the float64 sum of (r_i - lo) F_i over its own float32
    forces, and differs from the oracle's by no more than the force error allows
    (Cauchy-Schwarz: |dW|_F <= |r - lo|_F |dF|_2)."""
    pos = g["pos"] - np.asarray(g["lo"])[:, None]
    w_host = pos @ g["f"].T
    scale = float(np.linalg.norm(pos, axis=0) @ np.linalg.norm(g["f"], axis=0)) + 1e-300
    assert np.linalg.norm(g["virial"] - w_host) / scale < 1e-12
    bound = np.linalg.norm(pos) * np.linalg.norm(g["f"] - r["f"])
    assert np.linalg.norm(g["virial"] - r["virial"]) <= 1.01 * bound + 1e-9 * scale


def check_degenerate(g, r, s, tag):
    """Bar for inputs whose energy and forces cancel to near zero (a handful of
    atoms, random +-q clouds): the error is measured against the larger of the
    reference and the self-interaction magnitude each atom's own smeared charge
    puts on the grid (q_i^2 gamma(0)/a for the potential, divided by h for the
    force), the largest term that cancels in those sums.  Energy and potentials
    of such inputs are differences of grid potentials that each carry the FP32
    rounding of the grid chain (anterpolation, restriction, a stencil of S taps
    summed in rows, prolongation, interpolation), about sqrt(S) 2^-24 ~ 1e-6 of
    the self term, so their bar is 1e-6 of that scale; forces keep 1e-5."""
    a, h = s.cutoff, s.spacing
    m = s.split_m or s.order // 2
    q = s.q.astype(np.float64)
    self_pot = oracle.gamma(m, 0.0) / a
    e_scale = max(abs(r["energy"]), 0.5 * self_pot * float(q @ q))
    f_scale = max(np.linalg.norm(r["f"]), np.linalg.norm(q * q) * self_pot / h)
    p_scale = max(np.linalg.norm(r["phi"]), np.linalg.norm(q) * self_pot)
    de = abs(g["energy"] - r["energy"]) / e_scale
    df = np.linalg.norm(g["f"] - r["f"]) / f_scale
    dp = np.linalg.norm(g["phi"] - r["phi"]) / p_scale
    print(f"[{tag}] scaled errors: energy {de:.2e} force {df:.2e} phi {dp:.2e}", flush=True)
    assert g["code"] == 0
    assert de <= DEGENERATE_RTOL and df <= FORCE_RTOL and dp <= DEGENERATE_RTOL
    if "virial" in g:
        check_virial(g, r)


SMALL = {
    "cloud1k": inputs.cloud_1k,
    "water3k_l3": lambda: inputs.water_box(3000, seed=21, cutoff=9.0, spacing=2.0, order=4, levels=3),
    "water3k_quintic": lambda: inputs.water_box(3000, seed=22, cutoff=8.0, spacing=2.2, order=6, levels=3),
    "water3k_l1": lambda: inputs.water_box(3000, seed=23, cutoff=8.0, spacing=2.5, order=4, levels=1),
    "cloud_m3": lambda: inputs.uniform_charges(777, 17.3, seed=24, cutoff=6.5, spacing=1.9, order=4,
                                               levels=3, split_m=3),
    # stencils the windowed lattice kernel does not take, so the untiled
    # lattice kernel and the standalone top-level launch run: half-width 16
    # (2a/h = 17) whose window does not fit in LDS, and half-width 17 (2a/h = 18)
    "cloud500_wide": lambda: inputs.uniform_charges(500, 20.0, seed=29, cutoff=8.5, spacing=1.0, order=4,
                                                    levels=3),
    "cloud500_wide_quintic": lambda: inputs.uniform_charges(500, 20.0, seed=30, cutoff=9.0, spacing=1.0,
                                                            order=6, levels=3),
}
UNTILED = ("cloud500_wide", "cloud500_wide_quintic")


@pytest.mark.parametrize("name", list(SMALL))
def test_small_systems_match_oracle(M, name):
    s = SMALL[name]()
    print(f"case {name} n={s.n}", flush=True)
    if name in UNTILED:
        d = M.plan_for(s).describe()
        assert d["lattice_b"] == 0 and d["halo"] >= 16, d
    g = run_gpu(M, s)
    r = oracle.system_msm(s)
    check_full(g, r, name)


def test_stage_grids_match_oracle(M):
    s = inputs.water_box(6000, seed=25, cutoff=10.0, spacing=2.0, order=4, levels=4)
    print(f"case stages n={s.n}", flush=True)
    g = run_gpu(M, s)
    r = oracle.system_msm(s, grids=True)
    # cancellation-free magnitude of each grid: the same system with |q|
    ra = oracle.msm(s.x, s.y, s.z, np.abs(s.q), grids=True, **s.params())
    plan = g["plan"]
    L, lo, n = plan.info()
    flat = {sec: plan.section(sec).double().cpu().numpy() for sec in (M.SECTION_QGRID, M.SECTION_UCUT, M.SECTION_U)}
    off = 0
    errs = {}
    for k in range(L):
        cnt = int(np.prod(n[k]))
        for sec, key in ((M.SECTION_QGRID, "q"), (M.SECTION_UCUT, "ucut"), (M.SECTION_U, "u")):
            dev = flat[sec][off:off + cnt]
            ref = r[key][k].reshape(-1)
            scale = np.linalg.norm(ra[key][k].reshape(-1))
            errs[(k, key)] = err = float(np.linalg.norm(dev - ref) / scale)
            print(f"  level {k} {key}: error/|grid(|q|)| {err:.2e}  rel_rms {rel_rms(dev, ref):.2e}",
                  flush=True)
        off += cnt
    # each grid value is an FP32 sum; its error is measured against the grid
    # the same atoms give with every charge positive (no cancellation)
    for (k, key), err in errs.items():
        assert err < 1e-6, (k, key, err)
    # short-range potentials, back in input order
    perm = plan.section(M.SECTION_PERM, torch.int32).cpu().numpy()[:s.n]
    short = plan.section(M.SECTION_SHORT).cpu().numpy()[:4 * s.n].reshape(s.n, 4)
    phis = np.empty(s.n)
    phis[perm] = short[:, 3]
    assert rel_rms(phis, r["phis"]) < 1e-6
    assert sorted(perm.tolist()) == list(range(s.n))


def test_water24k_matches_oracle(M):
    s = inputs.water_24k()
    print(f"case water24k n={s.n}", flush=True)
    check_full(run_gpu(M, s), oracle.system_msm(s), "water24k")


def test_water100k_matches_oracle(M):
    s = inputs.water_100k()
    print(f"case water100k n={s.n}", flush=True)
    check_full(run_gpu(M, s), oracle.system_msm(s), "water100k")


@pytest.mark.parametrize("variant", ["coarse_grid_4h", "short_cutoff_6A"])
def test_cheap_msm_propagators_match_oracle(M, variant):
    """MSM as a coarse propagator: the finest grid four times coarser (h = 8
    A against 2 A) or the finest-grid cutoff halved to 6 A, on the 24,000-atom
    box, against the oracle with the same parameters (same bars)."""
    import dataclasses
    s = inputs.water_24k()
    kw = dict(spacing=4.0 * s.spacing, levels=0) if variant == "coarse_grid_4h" else dict(cutoff=6.0)
    v = dataclasses.replace(s, **kw)
    print(f"case {variant} a={v.cutoff} h={v.spacing} n={v.n}", flush=True)
    check_full(run_gpu(M, v), oracle.system_msm(v), variant)


def test_water1m_matches_oracle(M):
    """One million atoms, quintic basis, 5 levels: every force component, every
    potential and the energy against a full oracle evaluation."""
    s = inputs.water_1m()
    print(f"case water1m n={s.n}", flush=True)
    g = run_gpu(M, s)
    r = oracle.system_msm(s)
    check_full(g, r, "water1m")


def test_repeat_is_bitwise_identical(M):
    s = inputs.water_box(9000, seed=26, cutoff=10.0, spacing=2.0, order=4, levels=3)
    plan = M.plan_for(s)
    x, y, z, q = M.to_device(s)
    a = plan.compute(x, y, z, q)
    a = {k: v.clone() for k, v in a.items()}
    b = plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    assert torch.equal(a["f"], b["f"]) and torch.equal(a["phi"], b["phi"])
    assert torch.equal(a["energy"], b["energy"])


@pytest.mark.parametrize("streams", [1, 2, 3])
def test_stage_timing_modes_keep_results_bitwise(M, streams):
    """Both timing modes only add events: the results equal an untimed
    evaluation bitwise, every stage time is finite and non-negative, and the
    short range, the lattice cutoff and the interpolation take time."""
    s = inputs.water_box(9000, seed=26, cutoff=10.0, spacing=2.0, order=4, levels=3)
    plan = M.plan_for(s)
    plan.tune(streams=streams, short_after=2, short_split=500)
    x, y, z, q = M.to_device(s)
    ref = {k: v.clone() for k, v in plan.compute(x, y, z, q).items()}
    for live in (False, True, False):
        plan.profile(True, live=live)
        out = plan.compute(x, y, z, q)
        ms = plan.stage_ms()
        print(f"streams={streams} live={live} stage ms {ms}", flush=True)
        assert torch.equal(out["f"], ref["f"]) and torch.equal(out["phi"], ref["phi"])
        assert torch.equal(out["energy"], ref["energy"])
        assert list(ms) == list(M.STAGES)
        assert all(np.isfinite(v) and v >= 0.0 for v in ms.values())
        assert ms["short_range"] > 0 and ms["lattice_cutoff"] > 0 and ms["interpolation"] > 0
    plan.profile(False)


def test_input_order_does_not_change_results_beyond_rounding(M):
    s = inputs.water_box(3000, seed=27, cutoff=9.0, spacing=2.0, order=4, levels=3)
    g0 = run_gpu(M, s)
    rng = np.random.default_rng(0)
    p = rng.permutation(s.n)
    s2 = inputs.System(x=s.x[p].copy(), y=s.y[p].copy(), z=s.z[p].copy(), q=s.q[p].copy(),
                       box_lo=s.box_lo, box_len=s.box_len, cutoff=s.cutoff, spacing=s.spacing,
                       order=s.order, levels=s.levels)
    g1 = run_gpu(M, s2)
    assert rel_rms(g1["f"], g0["f"][:, p]) < 1e-6
    assert rel_err(g1["energy"], g0["energy"]) < 1e-8


# --------------------------------------------------------------------------
# Edge cases
# --------------------------------------------------------------------------

def _system(x, y, z, q, **prm):
    return inputs.System(x=np.asarray(x, np.float32), y=np.asarray(y, np.float32),
                         z=np.asarray(z, np.float32), q=np.asarray(q, np.float32), **prm)


BOX = dict(box_lo=(0.0, 0.0, 0.0), box_len=(16.0, 16.0, 16.0), cutoff=5.0, spacing=2.0,
           order=4, levels=2)


def test_empty_system(M):
    s = _system([], [], [], [], **BOX)
    g = run_gpu(M, s)
    assert g["code"] == 0 and g["energy"] == 0.0 and np.all(g["virial"] == 0)


@pytest.mark.parametrize("n", [1, 2, 3, 65, 257])
def test_tiny_and_ragged_systems(M, n):
    rng = np.random.default_rng(100 + n)
    pos = rng.uniform(0, 16, (3, n)).astype(np.float32)
    q = rng.uniform(-1, 1, n).astype(np.float32)
    s = _system(*pos, q, **BOX)
    g = run_gpu(M, s)
    r = oracle.system_msm(s)
    check_degenerate(g, r, s, f"n{n}")


def test_atoms_on_box_faces_and_corners(M):
    L = 16.0
    pts = np.array([[0, 0, 0], [L, L, L], [0, L, 0], [L, 0, 7.5], [8, 0, L], [3.3, 12.1, 0],
                    [L, 5.5, 9.25], [10.0, 10.0, 10.0]], dtype=np.float32).T
    q = np.array([1, -1, 0.5, -0.5, 0.25, -0.75, 1.0, -0.5], dtype=np.float32)
    s = _system(*pts, q, **BOX)
    g = run_gpu(M, s)
    check_degenerate(g, oracle.system_msm(s), s, "faces")


def test_offset_nonuniform_box(M):
    rng = np.random.default_rng(5)
    lo = np.array([-12.5, 3.0, 100.25])
    ln = np.array([30.0, 22.0, 41.0])
    n = 1500
    pos = (lo[:, None] + rng.uniform(0, 1, (3, n)) * ln[:, None]).astype(np.float32)
    q = rng.uniform(-1, 1, n).astype(np.float32)
    s = _system(*pos, q, box_lo=tuple(lo), box_len=tuple(ln), cutoff=7.0, spacing=1.8, order=6,
                levels=0)
    check_degenerate(run_gpu(M, s), oracle.system_msm(s), s, "offset_box")


@pytest.mark.parametrize("what,code", [("nan", -3), ("outside", -2), ("coincident", -7)])
def test_data_errors_are_flagged(M, what, code):
    rng = np.random.default_rng(7)
    n = 200
    pos = rng.uniform(0, 16, (3, n)).astype(np.float32)
    q = rng.uniform(-1, 1, n).astype(np.float32)
    if what == "nan":
        pos[1, 17] = np.nan
    elif what == "outside":
        pos[0, 50] = 16.5
    else:
        pos[:, 60] = pos[:, 61]
    s = _system(*pos, q, **BOX)
    g = run_gpu(M, s)
    assert g["code"] == code
    # a clean call on the same workspace clears the flag
    s_ok = _system(*rng.uniform(0, 16, (3, n)).astype(np.float32), q, **BOX)
    plan = g["plan"]
    plan.compute(*M.to_device(s_ok))
    assert plan.status()[0] == 0


def test_graph_replay_matches_eager(M):
    """Each replay of the captured evaluation equals an eager evaluation of the
    current inputs bitwise, with unrelated eager work and synchronisations
    between replays."""
    s = inputs.water_box(6000, seed=28, cutoff=10.0, spacing=2.0, order=4, levels=3)
    plan = M.plan_for(s)
    x, y, z, q = M.to_device(s)
    out = {"energy": torch.empty(1, dtype=torch.float64, device="cuda"),
           "f": torch.empty((3, s.n), dtype=torch.float32, device="cuda"),
           "phi": torch.empty(s.n, dtype=torch.float32, device="cuda"),
           "virial": torch.empty(9, dtype=torch.float64, device="cuda")}
    graph = M.Graph(plan, x, y, z, q, out)
    other = M.plan_for(inputs.cloud_1k())
    ox, oy, oz, oq = M.to_device(inputs.cloud_1k())
    rng = np.random.default_rng(1)
    for rep in range(4):
        for t in out.values():
            t.fill_(float("nan"))
        graph.launch()
        torch.cuda.synchronize()
        got = {k: v.clone() for k, v in out.items()}
        ref = plan.compute(x, y, z, q, virial=True)
        torch.cuda.synchronize()
        for k in ("energy", "f", "phi", "virial"):
            assert torch.equal(got[k], ref[k]), (rep, k)
        other.compute(ox, oy, oz, oq)           # unrelated eager work between replays
        torch.cuda.synchronize()
        # move the atoms a little (inside the box) and replay on the new positions
        d = torch.from_numpy(rng.uniform(-0.01, 0.01, s.n).astype(np.float32)).cuda()
        x.copy_(torch.clamp(x + d, 0.0, float(s.box_len[0])))


def test_graph_is_refused_after_retuning(M):
    """A graph keeps the launch grids, kernel variant and LDS size of the
    tuning it was captured under: after a re-tune its replay is refused with
    MSM_ERR_INVALID_ARG and nothing runs; a graph captured afterwards works."""
    s = inputs.water_box(6000, seed=34, cutoff=10.0, spacing=2.0, order=4, levels=3)
    plan = M.plan_for(s)
    x, y, z, q = M.to_device(s)
    ref = {k: v.clone() for k, v in plan.compute(x, y, z, q).items()}
    out = {k: torch.empty_like(v) for k, v in ref.items()}
    graph = M.Graph(plan, x, y, z, q, out)
    t = plan.tuning()
    plan.tune(lattice_b=4 if t["lattice_b"] != 4 else 6, short_blocks=64)
    for v in out.values():
        v.fill_(float("nan"))
    with pytest.raises(M.MSMError) as err:
        graph.launch()
    assert err.value.code == M.ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert all(bool(torch.isnan(v).all()) for v in out.values())
    fresh = M.Graph(plan, x, y, z, q, out)
    fresh.launch()
    torch.cuda.synchronize()
    again = plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(out[k], again[k]), k


def test_tunings_keep_bars_and_stream_layouts_are_bitwise_equal(M):
    """Every tuning (lattice outputs per lane, chunks per short-range item,
    short-range block count) stays within the bars; the stream layout, the
    short-range start and its split around the lattice cutoff only change
    concurrency, so their results are bitwise identical."""
    s = inputs.water_box(9000, seed=33, cutoff=10.0, spacing=2.0, order=4, levels=3)
    r = oracle.system_msm(s)
    plan = M.plan_for(s)
    x, y, z, q = M.to_device(s)
    for b in (4, 6, 8):
        for w in (1, 3):
            for sb in (-1, 64):
                outs = []
                for n, sa, sp in ((1, 1, 1000), (2, 1, 1000), (3, 1, 1000), (2, 3, 1000), (3, 2, 1000),
                                  (3, 3, 1000), (2, 1, 400), (3, 2, 700), (2, 1, 1)):
                    plan.tune(b, w, sb, n, sa, sp)
                    t = plan.tuning()
                    assert t["streams"] == n and t["short_after"] == sa and t["short_split"] == sp
                    o = plan.compute(x, y, z, q, virial=True)
                    torch.cuda.synchronize()
                    plan.check()
                    outs.append({k: v.clone() for k, v in o.items()})
                for o in outs[1:]:
                    for k in o:
                        assert torch.equal(o[k], outs[0][k]), (b, w, sb, k)
                f = outs[0]["f"].double().cpu().numpy()
                e = float(outs[0]["energy"].item())
                print(f"  tuning b={b} w={w} blocks={sb}: e_rel {rel_err(e, r['energy']):.2e} "
                      f"f_rms {rel_rms(f, r['f']):.2e}", flush=True)
                assert rel_err(e, r["energy"]) <= ENERGY_RTOL
                assert rel_rms(f, r["f"]) <= FORCE_RTOL


@pytest.mark.parametrize("reach", [2, 3, 4])
def test_cell_reach_keeps_bars(M, reach):
    """Every link-cell reach (edge a/2, a/3, a/4) gives results within the bars
    on a quintic water box and on the cubic 24k box."""
    for s in (inputs.water_box(9000, seed=35, cutoff=12.0, spacing=2.5, order=6, levels=0), inputs.water_24k()):
        print(f"case reach {reach} {s.name} n={s.n}", flush=True)
        plan = M.plan_for(s)
        plan.tune(cell_reach=reach)
        assert plan.tuning()["cell_reach"] == reach
        x, y, z, q = M.to_device(s)
        o = plan.compute(x, y, z, q)
        torch.cuda.synchronize()
        plan.check()
        r = oracle.system_msm(s)
        g = dict(energy=float(o["energy"].item()), f=o["f"].double().cpu().numpy(),
                 phi=o["phi"].double().cpu().numpy(), code=0, flags=0)
        check_full(g, r, f"reach{reach}-{s.name}")


@pytest.mark.parametrize("reach", [2, 4])
def test_dense_cloud_with_long_row_windows(M, reach):
    """A charge cloud four times denser than water: the union of a chunk's x
    windows in one cell row exceeds the 256 atoms a wave stages at a time, so
    every row is walked in several segments and lanes step past the end of a
    segment onto its far-away entries (which must stay far away from one chunk
    to the next).  A random +-q cloud: its energy and potentials are held
    to the bar of such clouds (check_degenerate), forces to 1e-5."""
    s = inputs.uniform_charges(20000, 36.0, seed=77, cutoff=12.0, spacing=2.0, order=4, levels=2)
    print(f"case dense cloud reach {reach} n={s.n}", flush=True)
    plan = M.plan_for(s)
    plan.tune(cell_reach=reach)
    x, y, z, q = M.to_device(s)
    o = plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    plan.check()
    r = oracle.system_msm(s)
    g = dict(energy=float(o["energy"].item()), f=o["f"].double().cpu().numpy(),
             phi=o["phi"].double().cpu().numpy(), code=0, flags=0)
    assert rel_rms(g["f"], r["f"]) <= FORCE_RTOL
    check_degenerate(g, r, s, f"dense-reach{reach}")


def test_output_buffers_are_validated(M):
    """The kernels write outputs through raw pointers, so the binding rejects
    buffers of the wrong dtype, size or layout instead of writing past them."""
    s = inputs.cloud_1k()
    plan = M.plan_for(s)
    x, y, z, q = M.to_device(s)
    good = plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    bad = [dict(good, f=torch.empty((s.n, 3), dtype=torch.float32, device="cuda").t()),
           dict(good, f=torch.empty((3, s.n - 1), dtype=torch.float32, device="cuda")),
           dict(good, energy=torch.empty(1, dtype=torch.float32, device="cuda")),
           dict(good, phi=torch.empty(2 * s.n, dtype=torch.float32, device="cuda")[::2])]
    for out in bad:
        with pytest.raises(ValueError):
            plan.compute(x, y, z, q, out=out)
    with pytest.raises(ValueError):
        plan.backward(x, y, z, q, torch.ones(1, dtype=torch.float64, device="cuda"),
                      dpos=torch.empty((s.n, 3), dtype=torch.float32, device="cuda").t())
    # the accepted buffers still give the same result
    again = plan.compute(x, y, z, q, out={k: torch.empty_like(v) for k, v in good.items()})
    torch.cuda.synchronize()
    assert torch.equal(again["f"], good["f"]) and torch.equal(again["energy"], good["energy"])
