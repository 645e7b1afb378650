"""Error measures of the parity tests (GPU against the oracle).

rel_max: max |a - b| over max |b| (the field's scale).
rel_pointwise: max over entries of |a - b| / max(|b|, floor * max |b|), the
pointwise relative error with a floor of 1e-12 of the field's max, so that
cold cells (values many orders below the max) are seen too.
"""
import numpy as np


def rel_max(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel_pointwise(a, b, floor=1e-12):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    scale = max(np.abs(b).max(), 1e-300)
    return float((np.abs(a - b) / np.maximum(np.abs(b), floor * scale)).max())
