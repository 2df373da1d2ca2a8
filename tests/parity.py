"""Shared helpers of the parity tests (comparison metric only, no method arithmetic)."""
import numpy as np


def rel_err(a, b, scale=1.0):
    """max|a - b| / max(max|b|, scale): the per-field parity metric."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(float(np.max(np.abs(b))) if b.size else 0.0, scale)
    return float(np.max(np.abs(a - b))) / den if b.size else 0.0


def state_errors(f_gpu, g_gpu, f_ref, g_ref, u_scale=1.0, T_scale=1.0):
    return {
        "f": rel_err(f_gpu, f_ref),
        "ux": rel_err(g_gpu[0], g_ref[0], u_scale),
        "uy": rel_err(g_gpu[1], g_ref[1], u_scale),
        "T": rel_err(g_gpu[2], g_ref[2], T_scale),
    }
