"""The documented storage order of the decay-time models (include/ipx.h,
ipx_dataset_create): a stable sort by (b << 58) | ((2^63 - 1 - bits(sigma_t)) >> 6)
with b = min(floor(2 t / sigma_t), 20), 0 when not positive."""
import numpy as np


def band_order(t, sig):
    r = 2.0 * np.asarray(t, np.float64) / np.asarray(sig, np.float64)
    with np.errstate(invalid="ignore"):
        b = np.where(r > 0.0, np.minimum(np.floor(r), 20.0), 0.0).astype(np.uint64)
    bits = np.ascontiguousarray(sig, np.float64).view(np.uint64)
    key = (b << np.uint64(58)) | ((np.uint64(0x7FFFFFFFFFFFFFFF) - bits) >> np.uint64(6))
    return np.argsort(key, kind="stable")
