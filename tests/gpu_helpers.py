"""Shared helpers of the GPU parity tests (comparison metrics of the tolerances)."""
import math

import numpy as np


def field_scale(ref, m):
    # a field that is zero everywhere (e.g. a momentum) is measured against the density
    return max(np.abs(ref[m]).max(), np.abs(ref[0]).max())


def max_rel(got, ref):
    """Per-field max|g - o| / max|o|."""
    return [float(np.abs(got[m] - ref[m]).max() / field_scale(ref, m)) for m in range(ref.shape[0])]


def l1_rel(got, ref):
    """Per-field sum|g - o| / sum|o|."""
    out = []
    for m in range(ref.shape[0]):
        s = np.abs(ref[m]).sum()
        if s == 0.0:
            s = np.abs(ref[0]).sum()
        out.append(float(np.abs(got[m] - ref[m]).sum() / s))
    return out


def totals_rel(got, ref):
    out = []
    for m in range(ref.shape[0]):
        tg = math.fsum(got[m].ravel())
        to = math.fsum(ref[m].ravel())
        s = math.fsum(np.abs(ref[m]).ravel()) or math.fsum(np.abs(ref[0]).ravel())
        out.append(abs(tg - to) / s)
    return out
