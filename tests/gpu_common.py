"""Shared helpers of the GPU tests (imported by tests marked ``gpu`` only)."""
import json
import os

import numpy as np
import torch

import msgen
import oracle as orc

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_points.json")


def dev():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch.device("cuda", 0)


def to_dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), device=dev(), dtype=dtype)


def slices_from_oracle(ms, prep):
    """A Slices object filled with the ORACLE's eigendata (eps, overlaps): isolates the
    per-energy kernels from the GPU eigensolver."""
    ns, n = prep["n_slices"], prep["n"]
    eps = np.stack(prep["eps"])
    ovl = np.stack([orc.overlap(prep["u"][p], prep["u"][p + 1]) for p in range(ns + 1)])
    return ms.Slices(n, ns, to_dev(prep["dz"][1:ns + 1]), to_dev(eps), to_dev(ovl))


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))


def golden_points(config=None):
    if not os.path.exists(GOLDEN):
        return []
    pts = json.load(open(GOLDEN))["points"]
    return [p for p in pts if config is None or p["config"] == config]


def junction_for(point):
    name = point["junction"]
    if name == "config1":
        return msgen.config1()
    if name.startswith("config2-"):
        return msgen.config2(point["meta"]["registry"])
    if name.startswith("config3-"):
        return msgen.config3(point["meta"]["gap"], point["meta"]["registry"])
    raise KeyError(name)
