"""Shared comparison helpers for the parity tests (no method arithmetic)."""
import numpy as np

FORCE_RTOL = 1e-5      # relative RMS over all 3N force components
ENERGY_RTOL = 1e-7     # relative energy error
PHI_RTOL = 1e-5        # relative RMS of per-atom potentials


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def rel_err(a, b):
    return abs(float(a) - float(b)) / max(abs(float(b)), 1e-300)
