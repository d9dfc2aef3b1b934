"""Algorithmic work model of one MSM evaluation (FLOPs and compulsory bytes).

Hardy's operation count, as quoted in the thesis (Sec. 2.3, eq. flop), is

    (4/3 pi m + 32/3 pi + 81/2) (a/h*)^3 N            short range incl. cell search
  + (6p^3 + 31p^2 + 36p + 17) N                        anterpolation + interpolation
  + ((4a/h)^3 + 14(p+2)) (8/7) (h*/h)^3 N              lattice cutoff + restriction/prolongation

with h* = N^{-1/3} L the mean inter-atomic spacing, m the smoothing degree and
p the interpolation degree.  The worked example after it (h* = 1, h = 2,
a = 12, m = 2, p = 3) prints 77.7 a^3 N + 566 N + 73 a^3/h^6 N + 80/h^3 N,
about 136,813 N.  The printed 77.7 does not equal the first bracket (82.4 for
m = 2); only 77.7 reproduces the printed total, so `paper_worked_example`
keeps it.

For the roofline we count the work a given evaluation must do, from the
actual workload rather than the continuum estimate:

* short range: 2(m + 8) FLOP per unique pair closer than a (the pair part of
  the first bracket: (4/3 pi m + 32/3 pi)(a/h*)^3 N = n_pairs * 2(m + 8));
* anterpolation + interpolation: 6p^3 + 31p^2 + 36p + 17 per atom;
* lattice cutoff: 2 FLOP (one multiply-add) per stencil tap per node below the
  top level, taps = lattice offsets n with |n| < 2a/h;
* restriction + prolongation: 14(p + 2) per coarse node;
* top level: 2 FLOP per ordered node pair.
"""
from __future__ import annotations

import math

import numpy as np


def hardy_flops_per_atom(a, h, hstar, m, p, short_coeff=None):
    """eq. flop per atom; `short_coeff` overrides the first bracket (the printed 77.7)."""
    c1 = (4.0 / 3.0 * math.pi * m + 32.0 / 3.0 * math.pi + 81.0 / 2.0) if short_coeff is None else short_coeff
    short = c1 * (a / hstar) ** 3
    grid_ai = 6 * p ** 3 + 31 * p ** 2 + 36 * p + 17
    lattice = (4.0 * a / h) ** 3 * (8.0 / 7.0) * (hstar / h) ** 3
    restr = 14 * (p + 2) * (8.0 / 7.0) * (hstar / h) ** 3
    return dict(short=short, anterp_interp=grid_ai, lattice=lattice, restrict_prolong=restr,
                total=short + grid_ai + lattice + restr)


def paper_worked_example():
    """The printed worked example: 77.7 a^3 + 566 + 73 a^3/h^6 + 80/h^3 per atom."""
    a, h = 12.0, 2.0
    terms = dict(short=77.7 * a ** 3, anterp_interp=566.0, lattice=73.0 * a ** 3 / h ** 6,
                 restrict_prolong=80.0 / h ** 3)
    terms["total"] = sum(terms.values())
    return terms


def stencil_taps(a, h):
    """Number of lattice offsets n (integer 3-vectors) with |n| < 2a/h."""
    rad = 2.0 * a / h
    R = int(math.ceil(rad))
    r = np.arange(-R, R + 1)
    d2 = r[:, None, None] ** 2 + r[None, :, None] ** 2 + r[None, None, :] ** 2
    return int(np.count_nonzero(d2 < rad * rad))


def count_pairs_within(pos, a):
    """Unique pairs closer than a (pos: [3, N] float64).

    A k-d tree counts, for every atom, the atoms within the largest float64
    below a (itself included); the sum less N, halved, is the number of
    unordered pairs with r < a."""
    from scipy.spatial import cKDTree

    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[1]
    if n < 2:
        return 0
    pts = np.ascontiguousarray(pos.T)
    tree = cKDTree(pts)
    counts = tree.query_ball_point(pts, np.nextafter(float(a), 0.0), return_length=True, workers=-1)
    return (int(np.sum(counts, dtype=np.int64)) - n) // 2


def evaluation_work(n_atoms, n_pairs, grid_nodes, a, h, order, m):
    """Algorithmic FLOPs of one evaluation, split by stage.

    grid_nodes: node count per level (level 0 first, top level last).
    """
    p = order - 1
    S = stencil_taps(a, h)
    L = len(grid_nodes)
    w = dict(
        short=2.0 * (m + 8) * n_pairs,
        anterp_interp=float(6 * p ** 3 + 31 * p ** 2 + 36 * p + 17) * n_atoms,
        lattice=2.0 * S * float(sum(grid_nodes[:L - 1])),
        restrict_prolong=float(14 * (p + 2)) * float(sum(grid_nodes[1:])),
        top=2.0 * float(grid_nodes[-1]) ** 2,
    )
    w["total"] = sum(w.values())
    w["taps"] = S
    return w
