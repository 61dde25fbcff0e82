"""Helpers shared by the GPU parity tests (no solver arithmetic here)."""
import numpy as np
import torch

import gen

U32 = np.finfo(np.float32).eps / 2  # unit roundoff of float32


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def spec_with(name, n, T, seed):
    s = gen.SPECS[name].scaled(n, T)
    return s.__class__(**{**s.__dict__, "seed": seed})


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
