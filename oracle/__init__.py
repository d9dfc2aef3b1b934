"""FP64 CPU oracle of the multilevel summation method (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The GPU product path does not import it, and the
two share no code; only the seeded input generators feed both.

The arithmetic lives in ``msm_oracle.c`` (plain C, double precision, OpenMP
over independent outputs), which follows Sec. 2.3 of the thesis stage by
stage.  This module loads it with ctypes and marshals numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "msm_oracle.c")
_LIB = os.path.join(_HERE, "libmsm_oracle.so")

ERRORS = {0: "ok", -1: "invalid argument", -2: "atom outside box", -3: "non-finite input",
          -7: "coincident atoms"}


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}: {ERRORS.get(code, '?')}")
        self.code = code


class _Params(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("h", ctypes.c_double), ("order", ctypes.c_int),
                ("m", ctypes.c_int), ("levels", ctypes.c_int), ("lo", ctypes.c_double * 3),
                ("len", ctypes.c_double * 3), ("ke", ctypes.c_double)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _LIB if os.path.exists(_LIB) else build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_msm.restype = ctypes.c_int
        L.oracle_msm.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, dp, dp, dp, dp, dp, dp, dp,
                                 dp, dp, dp, dp, dp, dp, dp, ip, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int]
        L.oracle_layout.restype = ctypes.c_int
        L.oracle_layout.argtypes = [ctypes.POINTER(_Params), ip, ip, ip]
        L.oracle_direct.restype = ctypes.c_int
        L.oracle_direct.argtypes = [ctypes.c_int, dp, dp, dp, dp, ctypes.c_double, dp, dp, dp, dp,
                                    dp, ctypes.c_int]
        for name in ("oracle_gamma", "oracle_dgamma"):
            getattr(L, name).restype = ctypes.c_double
            getattr(L, name).argtypes = [ctypes.c_int, ctypes.c_double]
        for name in ("oracle_Phi", "oracle_dPhi"):
            getattr(L, name).restype = ctypes.c_double
            getattr(L, name).argtypes = [ctypes.c_int, ctypes.c_double]
        L.oracle_split_kernel.restype = ctypes.c_double
        L.oracle_split_kernel.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, ctypes.c_double]
        L.oracle_pair.restype = ctypes.c_int
        L.oracle_pair.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, ctypes.c_double,
                                  ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int]
        L.oracle_pair_e.restype = ctypes.c_double
        L.oracle_pair_e.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.oracle_inside_f32.restype = None
        L.oracle_inside_f32.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, dp, ctypes.c_double, ip]
        L.oracle_gamma_coeffs.restype = None
        L.oracle_gamma_coeffs.argtypes = [ctypes.c_int, dp]
        L.oracle_msm_periodic.restype = ctypes.c_int
        L.oracle_msm_periodic.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, dp, dp, dp, dp, dp, dp, dp,
                                          dp, dp, dp, dp, dp, dp, dp, ctypes.c_int]
        L.oracle_periodic_layout.restype = ctypes.c_int
        L.oracle_periodic_layout.argtypes = [ctypes.POINTER(_Params), ip, ip]
        L.oracle_periodic_top_kernel.restype = ctypes.c_int
        L.oracle_periodic_top_kernel.argtypes = [ctypes.POINTER(_Params), dp, ctypes.c_int]
        L.oracle_ewald.restype = ctypes.c_int
        L.oracle_ewald.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp, dp, ctypes.c_double, dp, dp, dp, dp, dp,
                                   ctypes.c_int]
        _lib = L
    return _lib


def _params(cutoff, spacing, order=4, split_m=0, levels=0, box_lo=(0, 0, 0), box_len=(1, 1, 1),
            ke=1.0, **_):
    p = _Params()
    p.a, p.h, p.order, p.m, p.levels = float(cutoff), float(spacing), int(order), int(split_m), int(levels)
    for d in range(3):
        p.lo[d] = float(box_lo[d])
        p.len[d] = float(box_len[d])
    p.ke = float(ke)
    return p


def _dptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def layout(**params):
    """Level count and per-level node ranges: (levels, lo[L,3], n[L,3])."""
    p = _params(**params)
    lo = np.zeros(3 * 16, dtype=np.int32)
    n = np.zeros(3 * 16, dtype=np.int32)
    lv = ctypes.c_int(0)
    ip = ctypes.POINTER(ctypes.c_int)
    rc = lib().oracle_layout(ctypes.byref(p), ctypes.byref(lv), lo.ctypes.data_as(ip), n.ctypes.data_as(ip))
    if rc:
        raise OracleError(rc)
    L = lv.value
    return L, lo[:3 * L].reshape(L, 3).copy(), n[:3 * L].reshape(L, 3).copy()


def split_grids(flat, n):
    """Cut a concatenated level array into per-level [nz, ny, nx] views."""
    out, off = [], 0
    for k in range(n.shape[0]):
        cnt = int(np.prod(n[k]))
        out.append(flat[off:off + cnt].reshape(int(n[k][2]), int(n[k][1]), int(n[k][0])))
        off += cnt
    return out


def periodic_layout(**params):
    """Periodic level count and nodes per level: (levels, n[L,3])."""
    p = _params(**params)
    n = np.zeros(3 * 16, dtype=np.int32)
    lv = ctypes.c_int(0)
    ip = ctypes.POINTER(ctypes.c_int)
    rc = lib().oracle_periodic_layout(ctypes.byref(p), ctypes.byref(lv), n.ctypes.data_as(ip))
    if rc:
        raise OracleError(rc)
    L = lv.value
    return L, n[:3 * L].reshape(L, 3).copy()


def periodic_top_kernel(**params):
    """The periodic top-level kernel K at the node offsets of the top grid, [nz, ny, nx]."""
    L, n = periodic_layout(**params)
    top = n[L - 1]
    K = np.zeros(int(np.prod(top)))
    rc = lib().oracle_periodic_top_kernel(ctypes.byref(_params(**params)), _dptr(K), int(K.shape[0]))
    if rc:
        raise OracleError(rc)
    return K.reshape(int(top[2]), int(top[1]), int(top[0]))


def _msm_periodic(x, y, z, q, prm, grids, threads):
    p = _params(**prm)
    L, gn = periodic_layout(**prm)
    n = int(x.shape[0])
    ng = int(sum(int(np.prod(v)) for v in gn))
    fx, fy, fz = np.zeros(n), np.zeros(n), np.zeros(n)
    phi, phis = np.zeros(n), np.zeros(n)
    e = np.zeros(1)
    w = np.zeros(9)
    qg = np.zeros(ng) if grids else None
    uc = np.zeros(ng) if grids else None
    ug = np.zeros(ng) if grids else None
    rc = lib().oracle_msm_periodic(ctypes.byref(p), n, _dptr(x), _dptr(y), _dptr(z), _dptr(q), _dptr(fx),
                                   _dptr(fy), _dptr(fz), _dptr(phi), _dptr(e), _dptr(w), _dptr(qg), _dptr(uc),
                                   _dptr(ug), _dptr(phis), int(threads))
    if rc:
        raise OracleError(rc)
    out = dict(f=np.stack([fx, fy, fz]), phi=phi, phis=phis, levels=L, gn=gn, energy=float(e[0]),
               virial=w.reshape(3, 3))
    if grids:
        out["q"] = split_grids(qg, gn)
        out["ucut"] = split_grids(uc, gn)
        out["u"] = split_grids(ug, gn)
    return out


def ewald(x, y, z, q, *, box_lo, box_len, ke=1.0, threads=0):
    """Ewald summation of point charges in the periodic box: the exact
    periodic Coulomb energy, potentials phi[N] and forces f[3,N]."""
    x, y, z, q = _f64(x), _f64(y), _f64(z), _f64(q)
    n = int(x.shape[0])
    lo, ln = _f64(box_lo), _f64(box_len)
    fx, fy, fz, phi, e = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(1)
    rc = lib().oracle_ewald(n, _dptr(x), _dptr(y), _dptr(z), _dptr(q), _dptr(lo), _dptr(ln), float(ke),
                            _dptr(fx), _dptr(fy), _dptr(fz), _dptr(phi), _dptr(e), int(threads))
    if rc:
        raise OracleError(rc)
    return dict(f=np.stack([fx, fy, fz]), phi=phi, energy=float(e[0]))


def msm(x, y, z, q, *, cutoff, spacing, order=4, split_m=0, levels=0, box_lo=(0, 0, 0),
        box_len=(1, 1, 1), ke=1.0, grids=False, sample=None, short_mode=0, threads=0, exclusions=None,
        periodic=False):
    """Run the FP64 oracle.

    Returns a dict with energy, forces f[3,N], potentials phi[N], virial[3,3],
    the short-range potential phis[N] and (grids=True) the per-level grids
    q (charges), ucut (lattice-cutoff / top-level sums) and u (prolongated).
    With ``sample`` (atom indices) only those atoms' outputs are computed;
    energy and virial are then absent.  ``exclusions`` = (start, idx): bonded
    pairs left out (``exclusion_terms`` with kind "coulomb" taken off).
    ``periodic``: the box repeats in every direction (every atom's images
    interact; box_len / spacing must be an integer divisible by 2^(levels-1)
    and 2 cutoff <= box_len); grids are then the periodic level grids.
    """
    x, y, z, q = _f64(x), _f64(y), _f64(z), _f64(q)
    n = int(x.shape[0])
    prm = dict(cutoff=cutoff, spacing=spacing, order=order, split_m=split_m, levels=levels,
               box_lo=box_lo, box_len=box_len, ke=ke)
    if periodic:
        if sample is not None or short_mode:
            raise ValueError("periodic oracle: no sample or short_mode")
        out = _msm_periodic(x, y, z, q, prm, grids, threads)
        if exclusions is not None:
            out = _minus_exclusions(out, x, y, z, q, exclusions, kind="coulomb", ke=ke, box_lo=box_lo,
                                    box_len=box_len)
        return out
    p = _params(**prm)
    L, glo, gn = layout(**prm)
    ng = int(sum(int(np.prod(v)) for v in gn))
    fx, fy, fz = np.zeros(n), np.zeros(n), np.zeros(n)
    phi, phis = np.zeros(n), np.zeros(n)
    e = np.zeros(1)
    w = np.zeros(9)
    qg = np.zeros(ng) if grids else None
    uc = np.zeros(ng) if grids else None
    ug = np.zeros(ng) if grids else None
    if sample is not None:
        smp = np.ascontiguousarray(np.asarray(sample, dtype=np.int32))
        sptr, ns = smp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), int(smp.shape[0])
    else:
        sptr, ns = None, n
    rc = lib().oracle_msm(ctypes.byref(p), n, _dptr(x), _dptr(y), _dptr(z), _dptr(q), _dptr(fx),
                          _dptr(fy), _dptr(fz), _dptr(phi), _dptr(e), _dptr(w), _dptr(qg), _dptr(uc),
                          _dptr(ug), _dptr(phis), sptr, ns, int(short_mode), int(threads))
    if rc:
        raise OracleError(rc)
    out = dict(f=np.stack([fx, fy, fz]), phi=phi, phis=phis, levels=L, glo=glo, gn=gn)
    if sample is None:
        out["energy"] = float(e[0])
        out["virial"] = w.reshape(3, 3)
    if grids:
        out["q"] = split_grids(qg, gn)
        out["ucut"] = split_grids(uc, gn)
        out["u"] = split_grids(ug, gn)
    if exclusions is not None:
        out = _minus_exclusions(out, x, y, z, q, exclusions, sample=sample, kind="coulomb", ke=ke,
                                box_lo=box_lo)
    return out


def exclusion_terms(x, y, z, q, start, idx, *, kind="coulomb", cutoff=None, alpha=0.0, ke=1.0,
                    f32_cut=False, box_lo=(0, 0, 0), box_len=None):
    """The contribution of the listed (excluded) pairs, in FP64, to be taken
    off an evaluation: bonded pairs are left out of the Coulomb sum (Sec.
    "Calculation of Long-Range Interactions", before eq. (coulomb)).

    kind "coulomb": the whole Coulomb term q_i q_j / r of each pair (what a
    multilevel-summation evaluation carries for it: the short-range part plus
    the exact smooth part).  A pair-method kind: that method's pair term e(r)
    for the pairs inside the cutoff (decided in float32 with f32_cut, as in
    ``pair``).  Partner lists in CSR form over input indices (start [N + 1],
    idx), every pair listed from both sides.  With ``box_len`` (periodic
    boxes) each pair is taken at its nearest image and positions are mapped
    into the box.  Returns energy, f [3, N], phi [N] and virial [3, 3] of
    those pairs."""
    x, y, z, q = _f64(x), _f64(y), _f64(z), _f64(q)
    n = int(x.shape[0])
    start = np.asarray(start, dtype=np.int64)
    j = np.asarray(idx, dtype=np.int64)[:start[-1]]
    i = np.repeat(np.arange(n), np.diff(start))
    pos = np.stack([x, y, z])
    if box_len is not None:
        lo_, ln_ = np.asarray(box_lo, dtype=np.float64)[:, None], np.asarray(box_len, dtype=np.float64)[:, None]
        pos = pos - ln_ * np.floor((pos - lo_) / ln_)
    d = pos[:, i] - pos[:, j]
    if box_len is not None:
        d = d - ln_ * np.rint(d / ln_)
    r = np.sqrt(np.sum(d * d, axis=0))
    if kind == "coulomb":
        e, de = 1.0 / r, -1.0 / (r * r)
    else:
        k = PAIR_KINDS[kind] if isinstance(kind, str) else int(kind)
        rc = float(cutoff)
        if f32_cut:
            a, b = np.ascontiguousarray(pos[:, i]), np.ascontiguousarray(pos[:, j])
            flag = np.zeros(i.shape[0], dtype=np.int32)
            lib().oracle_inside_f32(int(i.shape[0]), _dptr(a[0]), _dptr(a[1]), _dptr(a[2]), _dptr(b[0]),
                                    _dptr(b[1]), _dptr(b[2]), float(rc),
                                    flag.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
            inside = flag.astype(bool)
        else:
            inside = r < rc
        if k == 1:
            e, de = 1.0 / r, -1.0 / (r * r)
        elif k == 2:
            e, de = 1.0 / r - 1.0 / rc + (r - rc) / (rc * rc), -1.0 / (r * r) + 1.0 / (rc * rc)
        else:
            from scipy.special import erfc
            e = erfc(alpha * r) / r - erfc(alpha * rc) / rc
            de = -erfc(alpha * r) / (r * r) - 2.0 * alpha / np.sqrt(np.pi) * np.exp(-(alpha * r) ** 2) / r
        e, de = np.where(inside, e, 0.0), np.where(inside, de, 0.0)
    phi = ke * np.bincount(i, weights=q[j] * e, minlength=n)
    w = -q[i] * q[j] * de / r                      # the force on i from j is w (r_i - r_j)
    f = ke * np.stack([np.bincount(i, weights=w * d[c], minlength=n) for c in range(3)])
    rel = pos - np.asarray(box_lo, dtype=np.float64)[:, None]
    return dict(energy=0.5 * float(q @ phi), f=f, phi=phi, virial=rel @ f.T)


def _minus_exclusions(out, x, y, z, q, exclusions, sample=None, **kw):
    ex = exclusion_terms(x, y, z, q, *exclusions, **kw)
    if sample is not None:
        smp = np.asarray(sample)
        out["f"] = out["f"] - ex["f"][:, smp]
        out["phi"] = out["phi"] - ex["phi"][smp]
        return out
    out["f"] = out["f"] - ex["f"]
    out["phi"] = out["phi"] - ex["phi"]
    out["energy"] = out["energy"] - ex["energy"]
    out["virial"] = out["virial"] - ex["virial"]
    return out


def direct(x, y, z, q, ke=1.0, threads=0):
    """Exact direct Coulomb sum over all unordered pairs (eq. coulomb, FP64)."""
    x, y, z, q = _f64(x), _f64(y), _f64(z), _f64(q)
    n = int(x.shape[0])
    fx, fy, fz, phi, e = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(1)
    rc = lib().oracle_direct(n, _dptr(x), _dptr(y), _dptr(z), _dptr(q), float(ke), _dptr(fx),
                             _dptr(fy), _dptr(fz), _dptr(phi), _dptr(e), int(threads))
    if rc:
        raise OracleError(rc)
    return dict(f=np.stack([fx, fy, fz]), phi=phi, energy=float(e[0]))


PAIR_KINDS = {"cutoff": 1, "shifted_force": 2, "wolf": 3}


def pair(x, y, z, q, *, kind, cutoff, alpha=0.0, box_lo=(0, 0, 0), box_len=(1, 1, 1), ke=1.0,
         all_pairs=False, f32_cut=False, threads=0, exclusions=None):
    """A cheap pair method (plain cutoff, shifted-force smoothed cutoff, Wolf
    summation) in FP64: energy, forces f[3,N], potentials phi[N], virial[3,3].
    f32_cut: decide r < rc in float32 as a float32 kernel does (the pair
    terms stay double).  exclusions = (start, idx): bonded pairs left out."""
    x, y, z, q = _f64(x), _f64(y), _f64(z), _f64(q)
    n = int(x.shape[0])
    lo, ln = _f64(box_lo), _f64(box_len)
    fx, fy, fz, phi = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
    e, w = np.zeros(1), np.zeros(9)
    k = PAIR_KINDS[kind] if isinstance(kind, str) else int(kind)
    rc = lib().oracle_pair(k, float(cutoff), float(alpha), _dptr(lo), _dptr(ln), float(ke), n, _dptr(x),
                           _dptr(y), _dptr(z), _dptr(q), _dptr(fx), _dptr(fy), _dptr(fz), _dptr(phi),
                           _dptr(e), _dptr(w), int(bool(all_pairs)), int(bool(f32_cut)), int(threads))
    if rc:
        raise OracleError(rc)
    out = dict(f=np.stack([fx, fy, fz]), phi=phi, energy=float(e[0]), virial=w.reshape(3, 3))
    if exclusions is not None:
        out = _minus_exclusions(out, x, y, z, q, exclusions, kind=kind, cutoff=cutoff, alpha=alpha, ke=ke,
                                f32_cut=f32_cut, box_lo=box_lo)
    return out


def pair_e(kind, cutoff, alpha, r):
    """The pair energy function e(r) of a cheap pair method (per unit charges)."""
    k = PAIR_KINDS[kind] if isinstance(kind, str) else int(kind)
    return lib().oracle_pair_e(k, float(cutoff), float(alpha), float(r))


def gamma(m, rho):
    return lib().oracle_gamma(int(m), float(rho))


def dgamma(m, rho):
    return lib().oracle_dgamma(int(m), float(rho))


def gamma_coeffs(m):
    c = np.zeros(m + 1)
    lib().oracle_gamma_coeffs(int(m), _dptr(c))
    return c


def Phi(order, u):
    return lib().oracle_Phi(int(order), float(u))


def dPhi(order, u):
    return lib().oracle_dPhi(int(order), float(u))


def split_kernel(k, r, **params):
    """g* (k = -1) or g^k (k >= 0) at distance r."""
    p = _params(**params)
    return lib().oracle_split_kernel(ctypes.byref(p), int(k), float(r))


def system_msm(sys_, **kw):
    """Oracle on an inputs.System (float32 inputs widened to float64)."""
    return msm(sys_.x, sys_.y, sys_.z, sys_.q, **sys_.params(), **kw)
