"""CPU-side checks of the C ABI: the library loads, exports every declared
entry point, and its host-side planning agrees with the oracle's grid layout.
No compute call is made (no GPU here)."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

import oracle
from paper_1402_7216_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msm.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:msm_status|const char\*)\s+(msm_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def M():
    from paper_1402_7216_amd import msm
    return msm


def test_library_exports_every_declared_symbol(M):
    names = _declared()
    assert len(names) >= 10
    lib = M.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(M.EXPORTS)


def _plan(M, n, **prm):
    p = M.make_params(**prm)
    h = ctypes.c_void_p()
    code = M.lib().msm_plan_create(ctypes.byref(p), n, ctypes.byref(h))
    return code, h


def _info(M, h):
    lv = ctypes.c_int32()
    lo = (ctypes.c_int32 * 48)()
    n = (ctypes.c_int32 * 48)()
    assert M.lib().msm_plan_info(h, ctypes.byref(lv), lo, n) == 0
    L = lv.value
    return L, np.array(lo[:3 * L]).reshape(L, 3), np.array(n[:3 * L]).reshape(L, 3)


CASES = [
    dict(cutoff=8.0, spacing=2.5, order=4, levels=2, box_lo=(0, 0, 0), box_len=(20, 20, 20)),
    dict(cutoff=12.0, spacing=2.0, order=4, levels=4, box_lo=(0, 0, 0), box_len=(62.1, 62.1, 62.1)),
    dict(cutoff=12.0, spacing=2.5, order=6, levels=0, box_lo=(0, 0, 0), box_len=(215.44,) * 3),
    dict(cutoff=12.0, spacing=2.0, order=4, levels=0, box_lo=(0, 0, 0), box_len=(100.0,) * 3),
    dict(cutoff=10.0, spacing=2.0, order=4, levels=0, box_lo=(-3, 5, 1.5), box_len=(27.1, 40.0, 33.3)),
    dict(cutoff=5.0, spacing=1.3, order=6, levels=1, box_lo=(0, 0, 0), box_len=(9.0, 7.0, 8.0)),
]


@pytest.mark.parametrize("prm", CASES)
def test_plan_layout_matches_oracle(M, prm):
    code, h = _plan(M, 1000, **prm)
    assert code == 0
    try:
        L, lo, n = _info(M, h)
        oprm = dict(prm)
        Lo, loo, no = oracle.layout(**{k: v for k, v in oprm.items()})
        assert L == Lo
        np.testing.assert_array_equal(lo, loo)
        np.testing.assert_array_equal(n, no)
        nb = ctypes.c_size_t()
        assert M.lib().msm_workspace_bytes(h, ctypes.byref(nb)) == 0 and nb.value > 0
    finally:
        M.lib().msm_plan_destroy(h)


@pytest.mark.parametrize("bad,code", [
    (dict(cutoff=0.0), -1), (dict(cutoff=float("nan")), -1), (dict(spacing=-1.0), -1),
    (dict(order=5), -1), (dict(levels=13), -1), (dict(split_m=9), -1),
    (dict(box_len=(0.0, 1.0, 1.0)), -1), (dict(spacing=0.1, levels=1), -6),
])
def test_plan_rejects_bad_parameters(M, bad, code):
    prm = dict(cutoff=8.0, spacing=2.5, order=4, levels=2, box_lo=(0, 0, 0), box_len=(20, 20, 20))
    prm.update(bad)
    c, h = _plan(M, 100, **prm)
    assert c == code
    assert M.lib().msm_last_error()


PERIODIC_CASES = [
    dict(cutoff=8.0, spacing=1.5, order=4, levels=0, box_lo=(0, 0, 0), box_len=(24.0, 30.0, 36.0)),
    dict(cutoff=8.0, spacing=1.5, order=6, levels=3, box_lo=(-2, 1, 0), box_len=(24.0, 30.0, 36.0)),
    dict(cutoff=10.0, spacing=2.5, order=6, levels=1, box_lo=(0, 0, 0), box_len=(40.0, 40.0, 20.0)),
    dict(cutoff=12.0, spacing=2.5, order=6, levels=0, box_lo=(0, 0, 0), box_len=(160.0, 160.0, 160.0)),
]


@pytest.mark.parametrize("prm", PERIODIC_CASES)
def test_periodic_plan_layout_matches_oracle(M, prm):
    """Level k holds the oracle's periodic grid of n_k nodes per side plus
    ghost copies on each side (index -ghost up)."""
    code, h = _plan(M, 1000, periodic=True, **prm)
    assert code == 0
    try:
        L, lo, n = _info(M, h)
        Lo, per = oracle.periodic_layout(**prm)
        assert L == Lo
        buf = ctypes.create_string_buffer(1 << 14)
        assert M.lib().msm_plan_describe(h, buf, len(buf)) == 0
        import json
        d = json.loads(buf.value.decode())
        G = d["ghost"]
        assert d["periodic"] == 1 and G >= max(prm["order"] - 1, prm["order"] // 2 + 1)
        if L > 1:
            assert G >= int(np.ceil(2 * prm["cutoff"] / prm["spacing"])) - 1
        np.testing.assert_array_equal(lo, -G * np.ones_like(lo))
        np.testing.assert_array_equal(n, per + 2 * G)
    finally:
        M.lib().msm_plan_destroy(h)


@pytest.mark.parametrize("bad", [
    dict(box_len=(24.0, 30.0, 36.7)),         # not a whole number of nodes
    dict(cutoff=12.5),                         # 2 a > box edge
    dict(levels=4),                            # 16 x 20 x 24 nodes cannot halve three times
])
def test_periodic_plan_rejects_bad_parameters(M, bad):
    prm = dict(cutoff=8.0, spacing=1.5, order=4, levels=2, box_lo=(0, 0, 0), box_len=(24.0, 30.0, 36.0),
               periodic=True)
    prm.update(bad)
    c, h = _plan(M, 100, **prm)
    assert c == -1
    assert M.lib().msm_last_error()


def test_periodic_pair_plan_and_batch_limits(M):
    p = M.PairParams()
    p.kind, p.periodic, p.cutoff, p.alpha, p.coulomb_k = 2, 1, 13.0, 0.0, 1.0
    for d in range(3):
        p.box_lo[d], p.box_len[d] = 0.0, 24.0
    h = ctypes.c_void_p()
    assert M.lib().msm_pair_plan_create(ctypes.byref(p), 100, ctypes.byref(h)) == -1   # 2 rc > box edge
    p.cutoff = 10.0
    assert M.lib().msm_pair_plan_create(ctypes.byref(p), 100, ctypes.byref(h)) == 0
    M.lib().msm_plan_destroy(h)
    # the flag is 0 or 1; batches take free-space systems only
    prm = M.make_params(8.0, 1.5, 4, 0, 2, (0, 0, 0), (24.0, 30.0, 36.0), 1.0, True)
    prm.periodic = 2
    assert M.lib().msm_plan_create(ctypes.byref(prm), 100, ctypes.byref(h)) == -1
    prm.periodic = 1
    arr = (M.Params * 1)(prm)
    n = (ctypes.c_int32 * 1)(100)
    b = ctypes.c_void_p()
    assert M.lib().msm_batch_create(arr, n, 1, ctypes.byref(b)) == -6


def test_plan_rejects_negative_atom_count(M):
    c, _ = _plan(M, -1, cutoff=8.0, spacing=2.5, box_len=(20, 20, 20))
    assert c == -1


def test_workspace_calls_check_sizes_without_touching_device(M):
    code, h = _plan(M, 10, **CASES[0])
    assert code == 0
    try:
        # a too-small workspace is rejected before any device work is enqueued
        assert M.lib().msm_workspace_init(h, ctypes.c_void_p(16), 8, None) == -4
        assert M.lib().msm_compute(h, ctypes.c_void_p(16), 8, None, *([None] * 10)) == -4
        off, nb = ctypes.c_size_t(), ctypes.c_size_t()
        assert M.lib().msm_workspace_section(h, 99, ctypes.byref(off), ctypes.byref(nb)) == -1
        assert M.lib().msm_status_string(-7) == b"coincident atoms"
    finally:
        M.lib().msm_plan_destroy(h)


def test_named_workload_generators_are_deterministic():
    a, b = inputs.water_24k(), inputs.water_24k()
    assert np.array_equal(a.x, b.x) and np.array_equal(a.q, b.q)
    assert a.n == 24000 and abs(float(a.q.astype(np.float64).sum())) == 0.0
    sizes = inputs.batch_sizes()
    assert len(sizes) == 64 and min(sizes) >= 2000 and max(sizes) <= 60000
    assert all(s % 3 == 0 for s in sizes)


def _batch(M, systems, n_atoms):
    arr = (M.Params * len(systems))()
    for i, prm in enumerate(systems):
        arr[i] = M.make_params(**prm)
    na = (ctypes.c_int32 * len(systems))(*n_atoms)
    h = ctypes.c_void_p()
    code = M.lib().msm_batch_create(arr, na, len(systems), ctypes.byref(h))
    return code, h


def test_batch_plan_describes_replicas_without_device(M):
    """Creating a batch is host work: per-system plans, one stage table per
    launch covering every system, atom offsets and one workspace size."""
    reps = inputs.water_replicas(64)
    code, h = _batch(M, [{**s.params()} for s in reps], [s.n for s in reps])
    assert code == 0, M.lib().msm_last_error()
    try:
        offs = (ctypes.c_int32 * 65)()
        assert M.lib().msm_batch_atom_offsets(h, offs) == 0
        assert list(offs) == [0] + list(np.cumsum([s.n for s in reps]))
        buf = ctypes.create_string_buffer(1 << 16)
        assert M.lib().msm_batch_describe(h, buf, len(buf)) == 0
        d = json.loads(buf.value.decode())
        assert d["systems"] == 64 and d["atoms"] == offs[64]
        # each system's level count is its own automatic choice
        for s, lv in zip(reps, d["levels"]):
            c1, p = _plan(M, s.n, **s.params())
            nl = ctypes.c_int32()
            lo = (ctypes.c_int32 * 48)()
            nn = (ctypes.c_int32 * 48)()
            assert M.lib().msm_plan_info(p, ctypes.byref(nl), lo, nn) == 0
            M.lib().msm_plan_destroy(p)
            assert nl.value == lv
        nb = ctypes.c_size_t()
        assert M.lib().msm_batch_workspace_bytes(h, ctypes.byref(nb)) == 0
        assert nb.value >= d["workspace_bytes"] > 0
        # uninitialised workspaces are refused before any device work
        assert M.lib().msm_batch_compute(h, ctypes.c_void_p(256), nb.value, None, *([None] * 10)) == -4
        t = M.make_tuning(4, 1)
        assert M.lib().msm_batch_tune(h, ctypes.c_void_p(256), nb.value, None, ctypes.byref(t)) == -4
    finally:
        M.lib().msm_batch_destroy(h)


def test_batch_rejects_mixed_order_and_bad_sizes(M):
    p4 = dict(CASES[0])
    p6 = {**p4, "order": 6}
    code, h = _batch(M, [p4, p6], [10, 10])
    assert code == -6 and not h.value
    code, h = _batch(M, [p4, p4], [10, -1])
    assert code == -1 and not h.value
    h = ctypes.c_void_p()
    assert M.lib().msm_batch_create(None, None, 0, ctypes.byref(h)) == -1


@pytest.mark.parametrize("field,value", [("lattice_b", 5), ("item_chunks", -2), ("short_blocks", -2),
                                         ("streams", 4), ("short_after", 4), ("short_split", 1001),
                                         ("short_split", -1), ("cell_reach", 1), ("cell_reach", 5),
                                         ("reserved", 1)])
def test_tuning_values_are_checked_before_any_device_work(M, field, value):
    code, h = _plan(M, 10, **CASES[0])
    assert code == 0
    try:
        t = M.make_tuning()
        setattr(t, field, value)
        assert M.lib().msm_plan_tune(h, ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(t)) == -1
        cur = M.Tuning()
        assert M.lib().msm_plan_tuning(h, ctypes.byref(cur)) == 0
        assert cur.lattice_b in (0, 4, 6, 8) and cur.item_chunks >= 1 and cur.streams == 3
        assert cur.short_after == 1 and cur.short_split == 1000 and cur.cell_reach in (2, 3, 4)
    finally:
        M.lib().msm_plan_destroy(h)


def test_profile_mode_and_read_are_checked_without_device(M):
    """Timing modes are 0, 1 and 2; reading needs profiling on and a timed
    evaluation.  Every refusal comes before any event is created."""
    code, h = _plan(M, 10, **CASES[0])
    assert code == 0
    try:
        ms = (ctypes.c_float * 16)()
        n = ctypes.c_int32()
        assert M.lib().msm_profile_enable(h, 3) == -1
        assert M.lib().msm_profile_enable(h, -1) == -1
        assert M.lib().msm_profile_read(h, ms, ctypes.byref(n)) == -1
        assert M.lib().msm_profile_enable(h, 0) == 0
        assert M.lib().msm_profile_read(h, ms, ctypes.byref(n)) == -1
    finally:
        M.lib().msm_plan_destroy(h)


def _key(M, fn, h):
    buf = ctypes.create_string_buffer(256)
    assert fn(h, buf, len(buf)) == 0
    small = ctypes.create_string_buffer(8)
    assert fn(h, small, len(small)) == -1
    return buf.value.decode()


def _taps(a, h):
    R = 2.0 * a / h
    r = int(np.floor(R))
    g = np.arange(-r, r + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return int(((X * X + Y * Y + Z * Z) < R * R).sum())


def test_tuning_keys_name_what_the_tuning_depends_on(M):
    """Plan key: target, order, smoothing degree, level-0 stencil taps and the
    half-octave level-0 node and atom counts; batch key adds the system count."""
    prm = CASES[2]                                   # the 1M-atom water box geometry
    code, h = _plan(M, 999999, **prm)
    assert code == 0
    try:
        key = _key(M, M.lib().msm_plan_tuning_key, h)
        L, lo, n = _info(M, h)
        nodes0 = int(np.prod(n[0]))
        assert key == (f"gfx950/o6/m3/S{_taps(12.0, 2.5)}/g{round(2 * np.log2(nodes0))}"
                       f"/n{round(2 * np.log2(999999))}")
        assert _taps(12.0, 2.5) == 3743
    finally:
        M.lib().msm_plan_destroy(h)
    reps = inputs.water_replicas(64)
    code, hb = _batch(M, [{**r.params()} for r in reps], [r.n for r in reps])
    assert code == 0
    try:
        key = _key(M, M.lib().msm_batch_tuning_key, hb)
        assert key.startswith(f"gfx950/batch64/o4/m2/S{_taps(10.0, 2.0)}/g")
        assert key.endswith(f"/n{round(2 * np.log2(sum(r.n for r in reps)))}")
    finally:
        M.lib().msm_batch_destroy(hb)


def test_tuning_cache_store_lookup_replace(M, tmp_path):
    path = str(tmp_path / "cache.txt")
    assert M.cache_lookup(path, "gfx950/o4/m2/S1/g1/n1") is None          # no file
    M.cache_store(path, "gfx950/o4/m2/S1/g1/n1", lattice_b=6, item_chunks=2, short_blocks=-1, streams=3,
                  short_after=2, short_split=500, cell_reach=3)
    M.cache_store(path, "gfx950/o6/m3/S2/g2/n2", lattice_b=4, item_chunks=1, short_blocks=512, streams=2,
                  short_after=1, short_split=1000, cell_reach=2)
    assert M.cache_lookup(path, "gfx950/o4/m2/S1/g1/n1") == dict(
        lattice_b=6, item_chunks=2, short_blocks=-1, streams=3, short_after=2, short_split=500, cell_reach=3)
    assert M.cache_lookup(path, "gfx950/o4/m2/S9/g1/n1") is None           # no entry
    # replacing keeps one line per key and the other entries
    M.cache_store(path, "gfx950/o4/m2/S1/g1/n1", lattice_b=8, item_chunks=1, short_blocks=-1, streams=1,
                  short_after=1, short_split=1000, cell_reach=2)
    lines = [l for l in open(path).read().splitlines() if l and not l.startswith("#")]
    assert len(lines) == 2 and lines[-1].split()[1] == "8"
    assert M.cache_lookup(path, "gfx950/o6/m3/S2/g2/n2")["short_blocks"] == 512
    assert not [p for p in os.listdir(tmp_path) if ".tmp" in p]
    # bad keys and values are refused; malformed files are reported
    t = M.make_tuning(4, 1, -1, 2, 1, 1000, 2)
    assert M.lib().msm_tuning_cache_store(path.encode(), b"has space", ctypes.byref(t)) == -1
    assert M.lib().msm_tuning_cache_store(path.encode(), b"a#b", ctypes.byref(t)) == -1
    bad = M.make_tuning(5, 1, -1, 2, 1, 1000, 2)
    assert M.lib().msm_tuning_cache_store(path.encode(), b"k", ctypes.byref(bad)) == -1
    with open(path, "a") as f:
        f.write("# comment line\nbroken 4 1\nrange 4 1 -1 9 1 1000 2\n")
    assert M.cache_lookup(path, "gfx950/o6/m3/S2/g2/n2")["lattice_b"] == 4
    with pytest.raises(M.MSMError):
        M.cache_lookup(path, "broken")
    with pytest.raises(M.MSMError):
        M.cache_lookup(path, "range")


def test_committed_tuning_cache_entries_are_valid(M):
    path = M.TUNING_CACHE
    if not os.path.exists(path):
        pytest.skip("no committed tuning cache")
    keys = [l.split()[0] for l in open(path).read().splitlines() if l and not l.startswith("#")]
    assert keys and len(keys) == len(set(keys))
    for k in keys:
        assert k.startswith("gfx950/")
        assert M.cache_lookup(path, k) is not None


def test_time_stepping_arguments_are_checked_without_device(M):
    """msm_vv_run / msm_parareal_run refuse bad arguments before any device
    work: negative step counts, a fine batch whose system count or atom count
    does not match, max_iter outside 1 .. slices, a missing workspace."""
    ions = inputs.rock_salt(3, seed=1)
    s = ions.system
    code, h = _plan(M, s.n, **s.params())
    assert code == 0
    code, hb = _batch(M, [s.params()] * 3, [s.n] * 3)
    assert code == 0
    try:
        nb = ctypes.c_size_t()
        assert M.lib().msm_parareal_workspace_bytes(s.n, 0, ctypes.byref(nb)) == -1
        assert M.lib().msm_parareal_workspace_bytes(s.n, 3, ctypes.byref(nb)) == 0 and nb.value > 0
        arr = [ctypes.c_void_p(256)] * 11
        assert M.lib().msm_vv_run(h, ctypes.c_void_p(256), 1 << 30, None, -1, 1.0, 1.0, *arr) == -1
        assert M.lib().msm_vv_run(h, ctypes.c_void_p(256), 1 << 30, None, 1, 1.0, 0.0, *arr) == -1
        it = ctypes.c_int32()

        def run(slices, max_iter, steps=2, reserved=0, ws=ctypes.c_void_p(256), ws_bytes=1 << 30):
            p = M.PararealParams(slices, steps, 1.0, 0.1, max_iter, reserved, 0.0)
            return M.lib().msm_parareal_run(ctypes.byref(p), hb, ctypes.c_void_p(256), 1 << 30, h,
                                            ctypes.c_void_p(256), 1 << 30, ws, ws_bytes, None,
                                            ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256),
                                            ctypes.byref(it), None)
        assert run(4, 1) == -1                  # the batch holds 3 systems
        assert run(3, 4) == -1                  # max_iter > slices
        assert run(3, 0) == -1
        assert run(3, 1, steps=0) == -1
        assert run(3, 1, reserved=1) == -1
        assert run(3, 1, ws=None) == -4         # no scratch
        assert run(3, 1, ws_bytes=16) == -4
    finally:
        M.lib().msm_batch_destroy(hb)
        M.lib().msm_plan_destroy(h)
