"""Helpers shared by the GPU parity tests: maps on the device, tolerance and argmax rules."""
from __future__ import annotations

import os
import shutil

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE_CACHE = os.path.join(ROOT, "paper_1401_8060_amd", "tuning", "gfx950.json")

TOL = 1e-5  # |z_gpu - z_oracle| <= TOL * max(1, |z|)  (FP32 scores vs FP64)


def to_dev(Y: np.ndarray, s: np.ndarray):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(Y)).cuda(), torch.from_numpy(np.ascontiguousarray(s)).cuda())


def assert_close(z_gpu, z_orc, tol=TOL, what=""):
    z_gpu = np.asarray(z_gpu, dtype=np.float64)
    z_orc = np.asarray(z_orc, dtype=np.float64)
    assert z_gpu.shape == z_orc.shape
    nan_g, nan_o = np.isnan(z_gpu), np.isnan(z_orc)
    assert (nan_g == nan_o).all(), f"{what}: NaN pattern differs"
    d = np.abs(z_gpu - z_orc)[~nan_o]
    lim = tol * np.maximum(1.0, np.abs(z_orc[~nan_o]))
    if d.size:
        i = int(np.argmax(d / lim))
        assert (d <= lim).all(), f"{what}: worst |dz|={d[i]:.3e} at {i} (z={z_orc[~nan_o][i]:.6f}), limit {lim[i]:.3e}"


def assert_argmax(j_gpu: int, z_orc: np.ndarray, j_orc: int | None = None, tol=TOL):
    """GPU argmax must equal the oracle's unless the two are a certified near-tie in FP64."""
    if j_orc is None:
        j_orc = int(np.nanargmax(z_orc))
    if j_gpu == j_orc:
        return
    gap = z_orc[j_orc] - z_orc[j_gpu]
    assert gap <= tol * max(1.0, abs(z_orc[j_orc])), f"argmax {j_gpu} vs oracle {j_orc}, gap {gap:.3e}"


def key_to_host(best_key) -> int:
    return int(best_key.item()) & 0xFFFFFFFFFFFFFFFF


def bench_tuning_copy(tmp_path) -> str:
    """A private copy of the committed MI355X tuning cache: full-scale tests take the slab shape
    the benchmark launches, and a cache miss (another GPU) never rewrites the committed file."""
    dst = str(tmp_path / "tune.json")
    shutil.copyfile(TUNE_CACHE, dst)
    return dst
