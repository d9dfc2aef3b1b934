"""ctypes binding of libmsm (include/msm.h), with torch for device memory and streams.

Argument marshalling only: every step of the evaluation runs in the HIP
kernels of libmsm.so.  If the library is not built, or no GPU is present,
calls fail loudly; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsm.so")

OK, ERR_INVALID_ARG, ERR_OUT_OF_BOX, ERR_NONFINITE = 0, -1, -2, -3
ERR_WORKSPACE, ERR_HIP, ERR_UNSUPPORTED, ERR_COINCIDENT = -4, -5, -6, -7

SECTION_QGRID, SECTION_UCUT, SECTION_U, SECTION_SORTED, SECTION_PERM, SECTION_SHORT = range(6)

# every entry point include/msm.h declares
EXPORTS = ("msm_plan_create", "msm_pair_plan_create", "msm_plan_destroy", "msm_plan_info", "msm_plan_describe",
           "msm_workspace_bytes",
           "msm_workspace_init", "msm_compute", "msm_compute_static", "msm_energy", "msm_backward",
           "msm_status_query",
           "msm_workspace_section",
           "msm_profile_enable", "msm_profile_read", "msm_graph_capture", "msm_graph_launch",
           "msm_graph_destroy", "msm_plan_tune", "msm_plan_tuning", "msm_plan_autotune",
           "msm_plan_tuning_key", "msm_tuning_cache_lookup", "msm_tuning_cache_store",
           "msm_plan_autotune_cached", "msm_batch_tuning_key", "msm_batch_autotune_cached",
           "msm_vv_run", "msm_batch_vv_run", "msm_parareal_workspace_bytes", "msm_parareal_run",
           "msm_set_exclusions", "msm_batch_set_exclusions",
           "msm_batch_create", "msm_batch_destroy", "msm_batch_workspace_bytes",
           "msm_batch_atom_offsets", "msm_batch_workspace_init", "msm_batch_compute",
           "msm_batch_energy", "msm_batch_backward", "msm_batch_graph_capture", "msm_batch_status",
           "msm_batch_describe", "msm_batch_tune", "msm_batch_autotune",
           "msm_status_string", "msm_last_error")

# tunings measured on MI355X for the named workloads (see msm_tuning_cache_lookup)
TUNING_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.txt")

STAGES = ("binning", "short_range", "anterpolation", "restriction", "lattice_cutoff", "top_level",
          "prolongation", "interpolation", "reduction")


class Tuning(ctypes.Structure):
    _fields_ = [("lattice_b", ctypes.c_int32), ("item_chunks", ctypes.c_int32), ("short_blocks", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("short_after", ctypes.c_int32), ("short_split", ctypes.c_int32),
                ("cell_reach", ctypes.c_int32), ("reserved", ctypes.c_int32)]


TUNING_KEYS = ("lattice_b", "item_chunks", "short_blocks", "streams", "short_after", "short_split", "cell_reach")


def make_tuning(lattice_b=0, item_chunks=0, short_blocks=0, streams=0, short_after=0, short_split=0,
                cell_reach=0) -> Tuning:
    t = Tuning()
    t.lattice_b, t.item_chunks, t.short_blocks = int(lattice_b), int(item_chunks), int(short_blocks)
    t.streams, t.short_after, t.short_split = int(streams), int(short_after), int(short_split)
    t.cell_reach, t.reserved = int(cell_reach), 0
    return t


def cache_lookup(path, key):
    """The tuning stored under key in a cache file (a dict), or None."""
    t = Tuning()
    code = lib().msm_tuning_cache_lookup(os.fsencode(path), key.encode(), ctypes.byref(t))
    if code == -6:
        return None
    _check(code)
    return {k: getattr(t, k) for k in TUNING_KEYS}


def cache_store(path, key, **tuning):
    """Add or replace key's entry in a cache file."""
    t = make_tuning(**tuning)
    _check(lib().msm_tuning_cache_store(os.fsencode(path), key.encode(), ctypes.byref(t)))


class MSMError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"libmsm status {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("cutoff", ctypes.c_double), ("spacing", ctypes.c_double),
                ("order", ctypes.c_int32), ("split_m", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("periodic", ctypes.c_int32),
                ("box_lo", ctypes.c_double * 3), ("box_len", ctypes.c_double * 3),
                ("coulomb_k", ctypes.c_double)]


class PairParams(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("periodic", ctypes.c_int32), ("cutoff", ctypes.c_double),
                ("alpha", ctypes.c_double), ("box_lo", ctypes.c_double * 3), ("box_len", ctypes.c_double * 3),
                ("coulomb_k", ctypes.c_double)]


PAIR_KINDS = {"cutoff": 1, "shifted_force": 2, "wolf": 3}


class PararealParams(ctypes.Structure):
    _fields_ = [("slices", ctypes.c_int32), ("steps_per_slice", ctypes.c_int32), ("dt", ctypes.c_double),
                ("accel_scale", ctypes.c_double), ("max_iter", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tol", ctypes.c_double)]

_lib = None


def lib():
    """Load libmsm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_1402_7216_amd.build first")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
        L.msm_plan_create.argtypes = [ctypes.POINTER(Params), i32, ctypes.POINTER(vp)]
        L.msm_pair_plan_create.argtypes = [ctypes.POINTER(PairParams), i32, ctypes.POINTER(vp)]
        L.msm_plan_destroy.argtypes = [vp]
        L.msm_plan_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.msm_plan_describe.argtypes = [vp, ctypes.c_char_p, sz]
        L.msm_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
        L.msm_workspace_init.argtypes = [vp, vp, sz, vp]
        L.msm_compute.argtypes = [vp, vp, sz, vp] + [vp] * 10
        L.msm_compute_static.argtypes = [vp, vp] + [vp] * 10
        L.msm_energy.argtypes = [vp, vp, sz, vp] + [vp] * 5
        L.msm_backward.argtypes = [vp, vp, sz, vp] + [vp] * 9
        L.msm_status_query.argtypes = [vp, vp, vp, ctypes.POINTER(i32)]
        L.msm_workspace_section.argtypes = [vp, i32, ctypes.POINTER(sz), ctypes.POINTER(sz)]
        L.msm_profile_enable.argtypes = [vp, i32]
        L.msm_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(i32)]
        L.msm_graph_capture.argtypes = [vp, vp, sz] + [vp] * 10 + [ctypes.POINTER(vp)]
        L.msm_graph_launch.argtypes = [vp, vp]
        L.msm_graph_destroy.argtypes = [vp]
        L.msm_plan_tune.argtypes = [vp, vp, sz, vp, ctypes.POINTER(Tuning)]
        L.msm_plan_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.msm_plan_autotune.argtypes = [vp, vp, sz, vp] + [vp] * 4 + [i32, ctypes.c_char_p, sz]
        L.msm_set_exclusions.argtypes = [vp, vp, sz, vp, vp, vp, ctypes.c_int64]
        L.msm_batch_set_exclusions.argtypes = [vp, vp, sz, vp, vp, vp, ctypes.c_int64]
        L.msm_vv_run.argtypes = [vp, vp, sz, vp, i32, ctypes.c_double, ctypes.c_double] + [vp] * 11
        L.msm_batch_vv_run.argtypes = [vp, vp, sz, vp, i32, ctypes.c_double, ctypes.c_double] + [vp] * 11
        L.msm_parareal_workspace_bytes.argtypes = [i32, i32, ctypes.POINTER(sz)]
        L.msm_parareal_run.argtypes = [ctypes.POINTER(PararealParams), vp, vp, sz, vp, vp, sz, vp, sz, vp, vp, vp,
                                       vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)]
        L.msm_plan_tuning_key.argtypes = [vp, ctypes.c_char_p, sz]
        L.msm_batch_tuning_key.argtypes = [vp, ctypes.c_char_p, sz]
        L.msm_tuning_cache_lookup.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(Tuning)]
        L.msm_tuning_cache_store.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(Tuning)]
        L.msm_plan_autotune_cached.argtypes = [vp, vp, sz, vp] + [vp] * 4 + [i32, ctypes.c_char_p,
                                                                              ctypes.c_char_p, sz]
        L.msm_batch_autotune_cached.argtypes = [vp, vp, sz, vp] + [vp] * 4 + [i32, ctypes.c_char_p,
                                                                               ctypes.c_char_p, sz]
        L.msm_batch_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(i32), i32, ctypes.POINTER(vp)]
        L.msm_batch_destroy.argtypes = [vp]
        L.msm_batch_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
        L.msm_batch_atom_offsets.argtypes = [vp, ctypes.POINTER(i32)]
        L.msm_batch_workspace_init.argtypes = [vp, vp, sz, vp]
        L.msm_batch_compute.argtypes = [vp, vp, sz, vp] + [vp] * 10
        L.msm_batch_energy.argtypes = [vp, vp, sz, vp] + [vp] * 5
        L.msm_batch_backward.argtypes = [vp, vp, sz, vp] + [vp] * 9
        L.msm_batch_graph_capture.argtypes = [vp, vp, sz] + [vp] * 10 + [ctypes.POINTER(vp)]
        L.msm_batch_status.argtypes = [vp, vp, vp, ctypes.POINTER(i32)]
        L.msm_batch_describe.argtypes = [vp, ctypes.c_char_p, sz]
        L.msm_batch_tune.argtypes = [vp, vp, sz, vp, ctypes.POINTER(Tuning)]
        L.msm_batch_autotune.argtypes = [vp, vp, sz, vp] + [vp] * 4 + [i32, ctypes.c_char_p, sz]
        L.msm_status_string.argtypes = [i32]
        L.msm_status_string.restype = ctypes.c_char_p
        L.msm_last_error.argtypes = []
        L.msm_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("msm_status_string", "msm_last_error"):
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def _check(code):
    if code != OK:
        raise MSMError(code, lib().msm_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _force_rows(f, n):
    """Pointers to the three rows of a contiguous [3, n] float32 force buffer."""
    if f is None:
        return None, None, None
    f0 = f.data_ptr()
    return ctypes.c_void_p(f0), ctypes.c_void_p(f0 + 4 * n), ctypes.c_void_p(f0 + 8 * n)


def _require_out(t, numel, dtype, device, name):
    """An output buffer the kernels write through a raw pointer: contiguous,
    of the right dtype, device and size."""
    if t.dtype != dtype or t.device != device or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"out[{name!r}] must be a contiguous {dtype} tensor on {device} with {numel} elements")


def _vv_run(self, pos, vel, q, inv_mass, n_steps, dt, accel_scale, f=None):
    """n_steps velocity Verlet steps on these forces (msm_vv_run /
    msm_batch_vv_run): pos and vel ([3, N] float32 device) are advanced in
    place; returns the forces at the final positions ([3, N], into f when
    given)."""
    dev = self.ws.device
    for name, t, numel in (("pos", pos, 3 * self.n), ("vel", vel, 3 * self.n), ("q", q, self.n),
                           ("inv_mass", inv_mass, self.n)):
        _require_out(t, numel, torch.float32, dev, name)
    if f is None:
        f = torch.empty((3, self.n), dtype=torch.float32, device=dev)
    _require_out(f, 3 * self.n, torch.float32, dev, "f")
    fn = lib().msm_batch_vv_run if isinstance(self, Batch) else lib().msm_vv_run
    _check(fn(self._h, _ptr(self.ws), self.ws.numel(), _stream(), int(n_steps), float(dt), float(accel_scale),
              *_force_rows(pos, self.n), _ptr(q), *_force_rows(vel, self.n), _ptr(inv_mass),
              *_force_rows(f, self.n)))
    return f


def _set_exclusions(self, start, idx):
    """Bonded exclusions (msm_set_exclusions / msm_batch_set_exclusions): CSR
    partner lists over input indices, start [N + 1] and idx [nnz] int32 (numpy
    or device tensors; kept alive by this object); None removes them."""
    if start is None:
        self._excl = None
        fn = lib().msm_batch_set_exclusions if isinstance(self, Batch) else lib().msm_set_exclusions
        _check(fn(self._h, _ptr(self.ws), self.ws.numel(), _stream(), None, None, 0))
        return
    dev = self.ws.device
    st = torch.as_tensor(start, dtype=torch.int32).to(dev).contiguous()
    ix = torch.as_tensor(idx, dtype=torch.int32).to(dev).contiguous()
    if st.numel() != self.n + 1:
        raise ValueError("start must have n_atoms + 1 entries")
    self._excl = (st, ix)
    fn = lib().msm_batch_set_exclusions if isinstance(self, Batch) else lib().msm_set_exclusions
    _check(fn(self._h, _ptr(self.ws), self.ws.numel(), _stream(), _ptr(st), _ptr(ix), int(ix.numel())))


def make_params(cutoff, spacing, order=4, split_m=0, levels=0, box_lo=(0.0, 0.0, 0.0),
                box_len=(1.0, 1.0, 1.0), coulomb_k=1.0, periodic=False) -> Params:
    p = Params()
    p.cutoff, p.spacing = float(cutoff), float(spacing)
    p.order, p.split_m, p.levels, p.periodic = int(order), int(split_m), int(levels), int(bool(periodic))
    for d in range(3):
        p.box_lo[d] = float(box_lo[d])
        p.box_len[d] = float(box_len[d])
    p.coulomb_k = float(coulomb_k)
    return p


class Plan:
    """A plan plus its device workspace for systems of `n_atoms` atoms."""

    def __init__(self, n_atoms, *, cutoff, spacing, order=4, split_m=0, levels=0,
                 box_lo=(0.0, 0.0, 0.0), box_len=(1.0, 1.0, 1.0), coulomb_k=1.0, periodic=False, device="cuda"):
        self.params = make_params(cutoff, spacing, order, split_m, levels, box_lo, box_len, coulomb_k, periodic)
        self.n = int(n_atoms)
        h = ctypes.c_void_p()
        _check(lib().msm_plan_create(ctypes.byref(self.params), self.n, ctypes.byref(h)))
        self._h = h
        self._init_workspace(device)

    def _init_workspace(self, device):
        nb = ctypes.c_size_t()
        _check(lib().msm_workspace_bytes(self._h, ctypes.byref(nb)))
        self.ws = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        _check(lib().msm_workspace_init(self._h, _ptr(self.ws), self.ws.numel(), _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.msm_plan_destroy(h)
            self._h = None

    def info(self):
        lv = ctypes.c_int32()
        lo = (ctypes.c_int32 * 48)()
        n = (ctypes.c_int32 * 48)()
        _check(lib().msm_plan_info(self._h, ctypes.byref(lv), lo, n))
        L = lv.value
        return L, [tuple(lo[3 * k:3 * k + 3]) for k in range(L)], [tuple(n[3 * k:3 * k + 3]) for k in range(L)]

    def describe(self):
        """The plan's decomposition (cells, tiles, ...) as a dict."""
        import json
        buf = ctypes.create_string_buffer(4096)
        _check(lib().msm_plan_describe(self._h, buf, 4096))
        return json.loads(buf.value.decode())

    def compute(self, x, y, z, q, *, forces=True, potentials=True, virial=False, out=None):
        """Energy (float64 [1]), forces [3, N] and potentials [N] on the device."""
        dev = self.ws.device
        for t in (x, y, z, q):
            if t.dtype != torch.float32 or t.device != dev or not t.is_contiguous() or t.numel() != self.n:
                raise ValueError("x, y, z, q must be contiguous float32 device tensors of length n_atoms")
        o = out if out is not None else {}
        if "energy" not in o:
            o["energy"] = torch.empty(1, dtype=torch.float64, device=dev)
        if forces and "f" not in o:
            o["f"] = torch.empty((3, self.n), dtype=torch.float32, device=dev)
        if potentials and "phi" not in o:
            o["phi"] = torch.empty(self.n, dtype=torch.float32, device=dev)
        if virial and "virial" not in o:
            o["virial"] = torch.empty(9, dtype=torch.float64, device=dev)
        f = o.get("f") if forces else None
        ph = o.get("phi") if potentials else None
        vr = o.get("virial") if virial else None
        _require_out(o["energy"], 1, torch.float64, dev, "energy")
        if f is not None:
            _require_out(f, 3 * self.n, torch.float32, dev, "f")
        if ph is not None:
            _require_out(ph, self.n, torch.float32, dev, "phi")
        if vr is not None:
            _require_out(vr, 9, torch.float64, dev, "virial")
        fx, fy, fz = _force_rows(f, self.n)
        _check(lib().msm_compute(self._h, _ptr(self.ws), self.ws.numel(), _stream(), _ptr(x), _ptr(y),
                                 _ptr(z), _ptr(q), fx, fy, fz, _ptr(ph), _ptr(o["energy"]), _ptr(vr)))
        return o

    vv_run = _vv_run
    set_exclusions = _set_exclusions

    def compute_static(self, x, y, z, q, out):
        """msm_compute_static: the evaluation of compute() with the library's
        static device workspace instead of self.ws (nothing is allocated; out
        holds preallocated "energy" [1], "f" [3, N], "phi" [N] and optionally
        "virial" [9] tensors)."""
        self._check_inputs(x, y, z, q)
        dev = self.ws.device
        for name, numel, dtype in (("energy", 1, torch.float64), ("f", 3 * self.n, torch.float32),
                                   ("phi", self.n, torch.float32), ("virial", 9, torch.float64)):
            if out.get(name) is not None:
                _require_out(out[name], numel, dtype, dev, name)
        fx, fy, fz = _force_rows(out.get("f"), self.n)
        _check(lib().msm_compute_static(self._h, _stream(), _ptr(x), _ptr(y), _ptr(z), _ptr(q), fx, fy, fz,
                                        _ptr(out.get("phi")), _ptr(out.get("energy")), _ptr(out.get("virial"))))
        return out

    def _check_inputs(self, x, y, z, q):
        dev = self.ws.device
        for t in (x, y, z, q):
            if t.dtype != torch.float32 or t.device != dev or not t.is_contiguous() or t.numel() != self.n:
                raise ValueError("x, y, z, q must be contiguous float32 device tensors of length n_atoms")

    def energy(self, x, y, z, q, out=None):
        """Energy only (float64 [1] on the device), without forces or grids kept."""
        self._check_inputs(x, y, z, q)
        e = out if out is not None else torch.empty(1, dtype=torch.float64, device=self.ws.device)
        _check(lib().msm_energy(self._h, _ptr(self.ws), self.ws.numel(), _stream(), _ptr(x), _ptr(y),
                                _ptr(z), _ptr(q), _ptr(e)))
        return e

    def backward(self, x, y, z, q, grad_energy, dpos=None, dq=None):
        """grad_energy * dE/dr into dpos [3, N] and grad_energy * dE/dq into dq [N] (float32)."""
        self._check_inputs(x, y, z, q)
        g = grad_energy.reshape(1).to(device=self.ws.device, dtype=torch.float64).contiguous()
        if dpos is not None:
            _require_out(dpos, 3 * self.n, torch.float32, self.ws.device, "dpos")
        if dq is not None:
            _require_out(dq, self.n, torch.float32, self.ws.device, "dq")
        dx, dy, dz = _force_rows(dpos, self.n)
        _check(lib().msm_backward(self._h, _ptr(self.ws), self.ws.numel(), _stream(), _ptr(x), _ptr(y),
                                  _ptr(z), _ptr(q), _ptr(g), dx, dy, dz, _ptr(dq)))
        return dpos, dq

    def tune(self, lattice_b=0, item_chunks=0, short_blocks=0, streams=0, short_after=0, short_split=0,
             cell_reach=0):
        """Set tuning knobs (zero keeps a knob's value); see msm_tuning."""
        t = make_tuning(lattice_b, item_chunks, short_blocks, streams, short_after, short_split, cell_reach)
        _check(lib().msm_plan_tune(self._h, _ptr(self.ws), self.ws.numel(), _stream(), ctypes.byref(t)))

    def tuning(self) -> dict:
        t = Tuning()
        _check(lib().msm_plan_tuning(self._h, ctypes.byref(t)))
        return {k: getattr(t, k) for k in TUNING_KEYS}

    def autotune(self, x, y, z, q, trials=5, cache=None):
        """Time the tuning candidates on these inputs, keep the fastest, return
        the search.  With a cache file: apply its entry for this plan's key if
        there is one (nothing timed), else search and store the result."""
        import json
        self._check_inputs(x, y, z, q)
        buf = ctypes.create_string_buffer(1 << 14)
        if cache is None:
            _check(lib().msm_plan_autotune(self._h, _ptr(self.ws), self.ws.numel(), _stream(), _ptr(x),
                                           _ptr(y), _ptr(z), _ptr(q), int(trials), buf, len(buf)))
        else:
            _check(lib().msm_plan_autotune_cached(self._h, _ptr(self.ws), self.ws.numel(), _stream(), _ptr(x),
                                                  _ptr(y), _ptr(z), _ptr(q), int(trials),
                                                  os.fsencode(cache), buf, len(buf)))
        return json.loads(buf.value.decode())

    def tuning_key(self) -> str:
        buf = ctypes.create_string_buffer(256)
        _check(lib().msm_plan_tuning_key(self._h, buf, len(buf)))
        return buf.value.decode()

    def status(self):
        """Synchronise and return (status code, raw device flags) of the last evaluation."""
        flags = ctypes.c_int32()
        code = lib().msm_status_query(self._h, _ptr(self.ws), _stream(), ctypes.byref(flags))
        return code, flags.value

    def check(self):
        code, _ = self.status()
        _check(code)

    def profile(self, enable=True, live=False):
        """Record per-stage HIP events inside every following compute(): with
        live=False every stage runs in order on the stream; with live=True the
        tuned stream layout is kept and each stage is timed on its own stream."""
        _check(lib().msm_profile_enable(self._h, (2 if live else 1) if enable else 0))

    def stage_ms(self):
        """Stage durations (ms) of the last compute(), keyed by stage name."""
        ms = (ctypes.c_float * 16)()
        n = ctypes.c_int32()
        _check(lib().msm_profile_read(self._h, ms, ctypes.byref(n)))
        return {STAGES[i]: float(ms[i]) for i in range(n.value)}

    def section(self, idx, dtype=torch.float32):
        off, nb = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().msm_workspace_section(self._h, int(idx), ctypes.byref(off), ctypes.byref(nb)))
        return self.ws[off.value:off.value + nb.value].view(dtype)


class PairPlan(Plan):
    """A cheap pair method on its own (msm_pair_plan_create): kind "cutoff",
    "shifted_force" or "wolf" with cutoff rc and (Wolf) damping alpha.  Same
    compute / compute_static / graph / tune interface as Plan; energy() and
    backward() are not available."""

    def __init__(self, n_atoms, *, kind, cutoff, alpha=0.0, box_lo=(0.0, 0.0, 0.0), box_len=(1.0, 1.0, 1.0),
                 coulomb_k=1.0, periodic=False, device="cuda"):
        p = PairParams()
        p.kind = PAIR_KINDS[kind] if isinstance(kind, str) else int(kind)
        p.periodic, p.cutoff, p.alpha, p.coulomb_k = int(bool(periodic)), float(cutoff), float(alpha), float(coulomb_k)
        for d in range(3):
            p.box_lo[d] = float(box_lo[d])
            p.box_len[d] = float(box_len[d])
        self.params = p
        self.n = int(n_atoms)
        h = ctypes.c_void_p()
        _check(lib().msm_pair_plan_create(ctypes.byref(p), self.n, ctypes.byref(h)))
        self._h = h
        self._init_workspace(device)


def pair_plan_for(system, kind, cutoff=None, alpha=0.0, periodic=False, device="cuda") -> PairPlan:
    """A pair-method plan for an inputs.System (cutoff defaults to the system's a)."""
    return PairPlan(system.n, kind=kind, cutoff=system.cutoff if cutoff is None else cutoff, alpha=alpha,
                    box_lo=system.box_lo, box_len=system.box_len, periodic=periodic, device=device)


class Graph:
    """A captured full evaluation of `plan` on fixed device buffers; launch() replays it."""

    def __init__(self, plan, x, y, z, q, out):
        self.plan, self.keep = plan, (x, y, z, q, out)
        plan._check_inputs(x, y, z, q)
        dev = plan.ws.device
        f = out.get("f")
        for name, numel, dtype in (("energy", 1, torch.float64), ("f", 3 * plan.n, torch.float32),
                                   ("phi", plan.n, torch.float32), ("virial", 9, torch.float64)):
            if out.get(name) is not None:
                _require_out(out[name], numel, dtype, dev, name)
        fx, fy, fz = _force_rows(f, plan.n)
        h = ctypes.c_void_p()
        _check(lib().msm_graph_capture(plan._h, _ptr(plan.ws), plan.ws.numel(), _ptr(x), _ptr(y),
                                       _ptr(z), _ptr(q), fx, fy, fz,
                                       _ptr(out.get("phi")), _ptr(out.get("energy")),
                                       _ptr(out.get("virial")), ctypes.byref(h)))
        self._h = h

    def launch(self):
        _check(lib().msm_graph_launch(self._h, _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.msm_graph_destroy(h)
            self._h = None


class MSMEnergy(torch.autograd.Function):
    """E(pos, q) with a hand-written backward.

    forward: msm_energy (energy only, float64 scalar; nothing but pos and q
             is saved).
    backward: msm_backward recomputes the grid chain and returns
              grad * dE/dpos (= -grad * F) and grad * dE/dq (= grad * phi),
              float32, with the incoming gradient read on the device.
    pos: float32 [3, N] (rows x, y, z), q: float32 [N], on the plan's device.
    """

    @staticmethod
    def forward(ctx, pos, q, plan):
        pos = pos.contiguous()
        q = q.contiguous()
        e = plan.energy(pos[0], pos[1], pos[2], q)
        ctx.plan = plan
        ctx.save_for_backward(pos, q)
        return e.reshape(())

    @staticmethod
    def backward(ctx, grad):
        pos, q = ctx.saved_tensors
        need_pos, need_q = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        dpos = torch.empty_like(pos) if need_pos else None
        dq = torch.empty_like(q) if need_q else None
        if need_pos or need_q:
            ctx.plan.backward(pos[0], pos[1], pos[2], q, grad.detach(), dpos, dq)
        return dpos, dq, None


def energy(plan, pos, q):
    """Differentiable MSM energy (see MSMEnergy)."""
    return MSMEnergy.apply(pos, q, plan)


class Batch:
    """n_sys independent systems evaluated together (one launch per stage).

    systems: list of parameter dicts (cutoff, spacing, order, split_m, levels,
    box_lo, box_len[, coulomb_k]) and n_atoms: list of atom counts.  Inputs and
    per-atom outputs are the systems' arrays concatenated in order."""

    def __init__(self, systems, n_atoms, device="cuda"):
        self.n_sys = len(systems)
        arr = (Params * self.n_sys)()
        for i, prm in enumerate(systems):
            arr[i] = make_params(**prm)
        na = (ctypes.c_int32 * self.n_sys)(*[int(v) for v in n_atoms])
        h = ctypes.c_void_p()
        _check(lib().msm_batch_create(arr, na, self.n_sys, ctypes.byref(h)))
        self._h = h
        offs = (ctypes.c_int32 * (self.n_sys + 1))()
        _check(lib().msm_batch_atom_offsets(self._h, offs))
        self.offsets = list(offs)
        self.n = self.offsets[-1]
        nb = ctypes.c_size_t()
        _check(lib().msm_batch_workspace_bytes(self._h, ctypes.byref(nb)))
        self.ws = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        _check(lib().msm_batch_workspace_init(self._h, _ptr(self.ws), self.ws.numel(), _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.msm_batch_destroy(h)
            self._h = None

    vv_run = _vv_run
    set_exclusions = _set_exclusions

    def compute_static(self, x, y, z, q, out):
        """msm_compute_static: the evaluation of compute() with the library's
        static device workspace instead of self.ws (nothing is allocated; out
        holds preallocated "energy" [1], "f" [3, N], "phi" [N] and optionally
        "virial" [9] tensors)."""
        self._check_inputs(x, y, z, q)
        dev = self.ws.device
        for name, numel, dtype in (("energy", 1, torch.float64), ("f", 3 * self.n, torch.float32),
                                   ("phi", self.n, torch.float32), ("virial", 9, torch.float64)):
            if out.get(name) is not None:
                _require_out(out[name], numel, dtype, dev, name)
        fx, fy, fz = _force_rows(out.get("f"), self.n)
        _check(lib().msm_compute_static(self._h, _stream(), _ptr(x), _ptr(y), _ptr(z), _ptr(q), fx, fy, fz,
                                        _ptr(out.get("phi")), _ptr(out.get("energy")), _ptr(out.get("virial"))))
        return out

    def _check_inputs(self, x, y, z, q):
        dev = self.ws.device
        for t in (x, y, z, q):
            if t.dtype != torch.float32 or t.device != dev or not t.is_contiguous() or t.numel() != self.n:
                raise ValueError("x, y, z, q must be contiguous float32 device tensors of the batch's length")

    def describe(self):
        import json
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().msm_batch_describe(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def outputs(self, virial=False):
        dev = self.ws.device
        o = {"energy": torch.empty(self.n_sys, dtype=torch.float64, device=dev),
             "f": torch.empty((3, self.n), dtype=torch.float32, device=dev),
             "phi": torch.empty(self.n, dtype=torch.float32, device=dev)}
        if virial:
            o["virial"] = torch.empty((self.n_sys, 9), dtype=torch.float64, device=dev)
        return o

    def _check_outputs(self, o):
        dev = self.ws.device
        for name, numel, dtype in (("energy", self.n_sys, torch.float64), ("f", 3 * self.n, torch.float32),
                                   ("phi", self.n, torch.float32), ("virial", 9 * self.n_sys, torch.float64)):
            if name in ("energy", "f", "phi") or o.get(name) is not None:
                _require_out(o[name], numel, dtype, dev, name)

    def compute(self, x, y, z, q, out=None, virial=False):
        self._check_inputs(x, y, z, q)
        o = out if out is not None else self.outputs(virial)
        self._check_outputs(o)
        fx, fy, fz = _force_rows(o["f"], self.n)
        _check(lib().msm_batch_compute(self._h, _ptr(self.ws), self.ws.numel(), _stream(), _ptr(x), _ptr(y),
                                       _ptr(z), _ptr(q), fx, fy, fz, _ptr(o["phi"]),
                                       _ptr(o["energy"]), _ptr(o.get("virial"))))
        return o

    def energy(self, x, y, z, q):
        self._check_inputs(x, y, z, q)
        e = torch.empty(self.n_sys, dtype=torch.float64, device=self.ws.device)
        _check(lib().msm_batch_energy(self._h, _ptr(self.ws), self.ws.numel(), _stream(), _ptr(x), _ptr(y),
                                      _ptr(z), _ptr(q), _ptr(e)))
        return e

    def backward(self, x, y, z, q, grad_energy, dpos=None, dq=None):
        self._check_inputs(x, y, z, q)
        g = grad_energy.reshape(self.n_sys).to(device=self.ws.device, dtype=torch.float64).contiguous()
        if dpos is not None:
            _require_out(dpos, 3 * self.n, torch.float32, self.ws.device, "dpos")
        if dq is not None:
            _require_out(dq, self.n, torch.float32, self.ws.device, "dq")
        dx, dy, dz = _force_rows(dpos, self.n)
        _check(lib().msm_batch_backward(self._h, _ptr(self.ws), self.ws.numel(), _stream(), _ptr(x), _ptr(y),
                                        _ptr(z), _ptr(q), _ptr(g), dx, dy, dz, _ptr(dq)))
        return dpos, dq

    def graph(self, x, y, z, q, out):
        return _BatchGraph(self, x, y, z, q, out)

    def status(self):
        flags = (ctypes.c_int32 * self.n_sys)()
        code = lib().msm_batch_status(self._h, _ptr(self.ws), _stream(), flags)
        return code, list(flags)

    def check(self):
        code, _ = self.status()
        _check(code)

    def tune(self, lattice_b=0, item_chunks=0, short_blocks=0, streams=0, short_after=0, short_split=0,
             cell_reach=0):
        t = make_tuning(lattice_b, item_chunks, short_blocks, streams, short_after, short_split, cell_reach)
        _check(lib().msm_batch_tune(self._h, _ptr(self.ws), self.ws.numel(), _stream(), ctypes.byref(t)))

    def autotune(self, x, y, z, q, trials=3, cache=None):
        import json
        self._check_inputs(x, y, z, q)
        buf = ctypes.create_string_buffer(1 << 14)
        if cache is None:
            _check(lib().msm_batch_autotune(self._h, _ptr(self.ws), self.ws.numel(), _stream(), _ptr(x),
                                            _ptr(y), _ptr(z), _ptr(q), int(trials), buf, len(buf)))
        else:
            _check(lib().msm_batch_autotune_cached(self._h, _ptr(self.ws), self.ws.numel(), _stream(), _ptr(x),
                                                   _ptr(y), _ptr(z), _ptr(q), int(trials),
                                                   os.fsencode(cache), buf, len(buf)))
        return json.loads(buf.value.decode())

    def tuning_key(self) -> str:
        buf = ctypes.create_string_buffer(256)
        _check(lib().msm_batch_tuning_key(self._h, buf, len(buf)))
        return buf.value.decode()


class _BatchGraph:
    def __init__(self, batch, x, y, z, q, out):
        self.keep = (batch, x, y, z, q, out)
        batch._check_inputs(x, y, z, q)
        batch._check_outputs(out)
        fx, fy, fz = _force_rows(out["f"], batch.n)
        h = ctypes.c_void_p()
        _check(lib().msm_batch_graph_capture(batch._h, _ptr(batch.ws), batch.ws.numel(), _ptr(x), _ptr(y),
                                             _ptr(z), _ptr(q), fx, fy, fz,
                                             _ptr(out["phi"]), _ptr(out["energy"]), _ptr(out.get("virial")),
                                             ctypes.byref(h)))
        self._h = h

    def launch(self):
        _check(lib().msm_graph_launch(self._h, _stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.msm_graph_destroy(h)
            self._h = None


class MSMBatchEnergy(torch.autograd.Function):
    """Per-system energies [n_sys] of a batch, with a hand-written backward
    (incoming gradient [n_sys] read on the device)."""

    @staticmethod
    def forward(ctx, pos, q, batch):
        pos = pos.contiguous()
        q = q.contiguous()
        e = batch.energy(pos[0], pos[1], pos[2], q)
        ctx.batch = batch
        ctx.save_for_backward(pos, q)
        return e

    @staticmethod
    def backward(ctx, grad):
        pos, q = ctx.saved_tensors
        need_pos, need_q = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        dpos = torch.empty_like(pos) if need_pos else None
        dq = torch.empty_like(q) if need_q else None
        if need_pos or need_q:
            ctx.batch.backward(pos[0], pos[1], pos[2], q, grad.detach(), dpos, dq)
        return dpos, dq, None


def parareal(fine, coarse, q, inv_mass, state0, *, slices, steps_per_slice, dt, accel_scale, max_iter=None,
             tol=0.0):
    """One parareal window (msm_parareal_run): fine is a Batch of `slices`
    systems (the fine propagator's forces, all slices at once), coarse a Plan
    or PairPlan of the same atom count (the coarse propagator's forces),
    state0 the [6, N] start state (x, y, z, vx, vy, vz).  Returns the states
    [6, slices + 1, N], the iterations run and the position change of each."""
    n = coarse.n
    dev = coarse.ws.device
    _require_out(state0, 6 * n, torch.float32, dev, "state0")
    for name, t in (("q", q), ("inv_mass", inv_mass)):
        _require_out(t, n, torch.float32, dev, name)
    mi = int(slices if max_iter is None else max_iter)
    p = PararealParams(int(slices), int(steps_per_slice), float(dt), float(accel_scale), mi, 0, float(tol))
    states = torch.empty((6, slices + 1, n), dtype=torch.float32, device=dev)
    states[:, 0, :] = state0
    nb = ctypes.c_size_t()
    _check(lib().msm_parareal_workspace_bytes(n, int(slices), ctypes.byref(nb)))
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
    it = ctypes.c_int32()
    res = (ctypes.c_float * max(mi, 1))()
    _check(lib().msm_parareal_run(ctypes.byref(p), fine._h, _ptr(fine.ws), fine.ws.numel(), coarse._h,
                                  _ptr(coarse.ws), coarse.ws.numel(), _ptr(ws), ws.numel(), _stream(), _ptr(q),
                                  _ptr(inv_mass), _ptr(states), ctypes.byref(it), res))
    return states, it.value, [float(res[k]) for k in range(it.value)]


def batch_energy(batch, pos, q):
    """Differentiable per-system energies of a batch (see MSMBatchEnergy)."""
    return MSMBatchEnergy.apply(pos, q, batch)


def batch_for(systems, device="cuda") -> Batch:
    """Batch for a list of inputs.System."""
    return Batch([{**s.params(), "split_m": s.split_m} for s in systems], [s.n for s in systems], device)


def batch_to_device(systems, device="cuda"):
    cat = lambda name: torch.from_numpy(np.concatenate([getattr(s, name) for s in systems])).to(device)
    return cat("x"), cat("y"), cat("z"), cat("q")


def plan_for(system, periodic=False, device="cuda") -> Plan:
    """Plan for an inputs.System (periodic: the box repeated in every direction)."""
    return Plan(system.n, device=device, periodic=periodic, **{**system.params(), "split_m": system.split_m})


def to_device(system, device="cuda"):
    return tuple(torch.from_numpy(a).to(device) for a in (system.x, system.y, system.z, system.q))
