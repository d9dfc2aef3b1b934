"""Link-cell binning on the GPU against its definition.

Cells are numbered (cz ny + cy) nx + cx with c_d = floor((p_d - lo_d) / edge_d)
in float32 arithmetic, clamped to the grid; the sorted order is by cell, ties
in input order (a stable sort).  Every later kernel relies on that order (a
cell row's atoms are contiguous; sums run in that order), so each of the four
binning paths (one kernel for small systems, two kernels, four kernels by cell
row, four kernels over the cells) is checked against a host stable sort on
systems that take that path, including a clustered system whose few occupied
rows hold thousands of atoms each.
"""
import numpy as np
import pytest

from paper_1402_7216_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1402_7216_amd import msm
    msm.lib()
    return msm


def host_cells(s, nc):
    """Cell of every atom, computed as the device computes it (float32)."""
    cells = []
    for d, p in enumerate((s.x, s.y, s.z)):
        lo = np.float32(s.box_lo[d])
        inv = np.float32(nc[d] / s.box_len[d])
        t = (p.astype(np.float32) - lo) * inv
        t = np.minimum(np.maximum(t, np.float32(0.0)), np.float32(nc[d] - 1))
        cells.append(np.minimum(t.astype(np.int64), nc[d] - 1))
    return (cells[2] * nc[1] + cells[1]) * nc[0] + cells[0]


def clustered(n, seed=11):
    """n charges packed into a 6 A cube inside a 60 A box: a few cell rows
    hold every atom."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(20.0, 26.0, size=(3, n))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return inputs._as_f32_system(pos, q, (0.0, 0.0, 0.0), (60.0, 60.0, 60.0), cutoff=12.0,
                                 spacing=2.0, order=4, levels=0, name=f"clustered{n}")


def wide_slab(n, seed=15):
    """n charges in a 20 x 400 x 400 A box with a = 8 A: 10,000 cell rows,
    more than the row binning takes, so the four kernels over the cells run."""
    rng = np.random.default_rng(seed)
    size = np.array([20.0, 400.0, 400.0])
    pos = rng.uniform(0.0, 1.0, size=(3, n)) * size[:, None]
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return inputs._as_f32_system(pos, q, (0.0, 0.0, 0.0), tuple(size), cutoff=8.0, spacing=2.0,
                                 order=4, levels=0, name=f"wide_slab{n}")


def rod(n, seed=16, width=6.0, length=120.0):
    """n charges in a rod along x (length x width x width) inside a 120 A box
    with a = 12 A: one or two cell rows hold every atom (far more than the row
    binning keeps in LDS), a few hundred per cell for the full length."""
    rng = np.random.default_rng(seed)
    pos = np.empty((3, n))
    pos[0] = rng.uniform(0.0, length, n)
    pos[1:] = rng.uniform(30.0, 30.0 + width, (2, n))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return inputs._as_f32_system(pos, q, (0.0, 0.0, 0.0), (120.0, 120.0, 120.0), cutoff=12.0,
                                 spacing=3.0, order=4, levels=0, name=f"rod{n}")


def slab(n, seed=13):
    """n charges in a flat 20 x 120 x 120 A box with a = 8 A: 841 cell rows,
    so blocks of the one-kernel binning own several rows each."""
    rng = np.random.default_rng(seed)
    size = np.array([20.0, 120.0, 120.0])
    pos = rng.uniform(0.0, 1.0, size=(3, n)) * size[:, None]
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return inputs._as_f32_system(pos, q, (0.0, 0.0, 0.0), tuple(size), cutoff=8.0, spacing=2.0,
                                 order=4, levels=0, name=f"slab{n}")


CASES = {
    "water24k": (lambda: inputs.water_24k(), "one"),
    "clustered20k": (lambda: clustered(20000), "one"),
    "uniform1000": (lambda: inputs.uniform_charges(n=1000), "one"),
    "uniform65": (lambda: inputs.uniform_charges(n=65, seed=3), "one"),
    "uniform1": (lambda: inputs.uniform_charges(n=1, seed=4), "one"),
    "slab32768": (lambda: slab(32768), "one"),
    "slab32769": (lambda: slab(32769, seed=14), "rows"),
    "water40k": (lambda: inputs.water_box(40000, seed=9), "two"),
    "water100k": (lambda: inputs.water_100k(), "rows"),
    "wide_slab40k": (lambda: wide_slab(40000), "four"),
    "rod40k": (lambda: rod(40000), "rows"),
}


def path_of(d):
    if d["bin_row_blocks"] > 0:
        return "one"
    if d["bin_blocks"] > 0:
        return "two"
    return "rows" if d["binr_blocks"] > 0 else "four"


@pytest.mark.parametrize("name", list(CASES))
def test_binning_is_stable_cell_sort(M, name):
    make, path = CASES[name]
    s = make()
    print(f"case {name} n={s.n}", flush=True)
    plan = M.plan_for(s)
    d = plan.describe()
    assert path_of(d) == path, d
    x, y, z, q = M.to_device(s)
    plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    code, flags = plan.status()
    assert code == 0, flags
    perm = plan.section(M.SECTION_PERM, torch.int32).cpu().numpy()[:s.n]
    srt = plan.section(M.SECTION_SORTED).cpu().numpy()[:4 * s.n].reshape(s.n, 4)
    order = np.argsort(host_cells(s, d["cells"]), kind="stable")
    assert np.array_equal(perm, order)
    for k, v in enumerate((s.x, s.y, s.z, s.q)):
        assert np.array_equal(srt[:, k], v[order])


@pytest.mark.parametrize("name", ["water24k", "water40k", "slab32769", "water100k", "wide_slab40k"])
def test_coincident_atoms_are_flagged_on_every_binning_path(M, name):
    """Two atoms of different molecules moved onto the same point are reported
    as MSM_ERR_COINCIDENT whichever binning path the system takes (the one-
    and two-kernel paths flag them in the short-range pass, the four-kernel
    paths while ranking atoms inside a cell); a clean call clears the flag."""
    make, path = CASES[name]
    s = make()
    print(f"case coincident {name} n={s.n} path={path}", flush=True)
    plan = M.plan_for(s)
    x, y, z, q = M.to_device(s)
    j, k = 10, s.n // 2 + 1
    xb, yb, zb = x.clone(), y.clone(), z.clone()
    xb[k], yb[k], zb[k] = x[j], y[j], z[j]
    plan.compute(xb, yb, zb, q)
    code, flags = plan.status()
    assert code == M.ERR_COINCIDENT, (code, flags)
    plan.compute(x, y, z, q)
    assert plan.status()[0] == 0


@pytest.mark.parametrize("name", ["water24k", "water40k", "water100k"])
@pytest.mark.parametrize("reach", [3, 4])
def test_finer_cells_keep_the_stable_cell_sort(M, name, reach):
    """Link cells of edge a/3 and a/4 (the cell_reach tuning) still give the
    stable cell sort, whichever binning path the finer cells select."""
    make, _ = CASES[name]
    s = make()
    print(f"case {name} reach {reach} n={s.n}", flush=True)
    plan = M.plan_for(s)
    plan.tune(cell_reach=reach)
    d = plan.describe()
    assert d["reach"] == reach
    x, y, z, q = M.to_device(s)
    plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    code, flags = plan.status()
    assert code == 0, flags
    perm = plan.section(M.SECTION_PERM, torch.int32).cpu().numpy()[:s.n]
    order = np.argsort(host_cells(s, d["cells"]), kind="stable")
    assert np.array_equal(perm, order)


@pytest.mark.parametrize("name", ["slab32769", "wide_slab40k"])
@pytest.mark.parametrize("what,code", [("nan", -3), ("outside", -2)])
def test_bad_atoms_are_flagged_on_the_large_paths(M, name, what, code):
    """A non-finite coordinate or an atom outside the box is reported by the
    binning paths of large systems (by cell row, over the cells); a clean
    call clears the flag."""
    make, path = CASES[name]
    s = make()
    print(f"case {what} {name} n={s.n} path={path}", flush=True)
    plan = M.plan_for(s)
    assert path_of(plan.describe()) == path
    x, y, z, q = M.to_device(s)
    xb, yb = x.clone(), y.clone()
    if what == "nan":
        yb[17] = float("nan")
    else:
        xb[50] = float(s.box_lo[0] + s.box_len[0]) + 0.5
    plan.compute(xb, yb, z, q)
    torch.cuda.synchronize()
    assert plan.status()[0] == code
    plan.compute(x, y, z, q)
    assert plan.status()[0] == 0


def test_cells_longer_than_the_rank_cap_keep_every_atom(M):
    """A row binning cell of more than 2048 atoms keeps its atoms in arrival
    order (as the four kernels over the cells do): every atom appears once,
    in cell order, and the other cells of the row are still stably sorted."""
    s = rod(60000, seed=17, width=1.0, length=20.0)
    print(f"case rod60k n={s.n}", flush=True)
    plan = M.plan_for(s)
    d = plan.describe()
    assert path_of(d) == "rows", d
    x, y, z, q = M.to_device(s)
    plan.compute(x, y, z, q)
    torch.cuda.synchronize()
    perm = plan.section(M.SECTION_PERM, torch.int32).cpu().numpy()[:s.n]
    assert np.array_equal(np.sort(perm), np.arange(s.n))
    cells = host_cells(s, d["cells"])
    assert np.all(np.diff(cells[perm]) >= 0)
    counts = np.bincount(cells)
    assert counts.max() > 2048
    small = counts[cells[perm]] <= 2048
    order = np.argsort(cells, kind="stable")
    assert np.array_equal(perm[small], order[small])


def test_coincident_atoms_in_a_cell_over_the_rank_cap_are_flagged(M):
    """Binning leaves a cell of more than 2048 atoms unchecked; the short-range
    pass then checks it, so coincident atoms there are still reported."""
    s = rod(60000, seed=17, width=1.0, length=20.0)
    print(f"case coincident rod60k n={s.n}", flush=True)
    plan = M.plan_for(s)
    assert path_of(plan.describe()) == "rows"
    x, y, z, q = M.to_device(s)
    xb, yb, zb = x.clone(), y.clone(), z.clone()
    j, k = 10, 31001
    xb[k], yb[k], zb[k] = x[j], y[j], z[j]
    plan.compute(xb, yb, zb, q)
    assert plan.status()[0] == M.ERR_COINCIDENT
    plan.compute(x, y, z, q)
    assert plan.status()[0] == 0
