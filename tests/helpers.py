"""Shared helpers of the GPU tests (comparison against the oracle)."""
import os

import numpy as np


def oracle_threads() -> int:
    n = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return max(1, min(n or (os.cpu_count() or 1), os.cpu_count() or 1))


def assert_vis_equal(got: np.ndarray, ref: np.ndarray, what: str):
    if np.array_equal(got, ref):
        return
    bad = np.argwhere(got != ref)
    y, x = bad[0]
    raise AssertionError(f"{what}: {len(bad)} of {ref.size} pixels differ; first at (x={x}, y={y}) "
                         f"gpu={int(got[y, x]):#018x} oracle={int(ref[y, x]):#018x}")


def assert_resolve_close(got: np.ndarray, ref: np.ndarray, what: str, rtol=1e-5, floor=0.1):
    err = np.abs(got.astype(np.float64) - ref.astype(np.float64))
    lim = rtol * np.maximum(np.abs(ref.astype(np.float64)), floor)
    assert np.all(err <= lim), f"{what}: max err {err.max()} (limit {lim[np.argmax(err - lim)]})"
