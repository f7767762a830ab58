"""Helpers for the GPU parity tests (inputs from the shared generators; expected values from the
oracle only)."""
import sys

import numpy as np
import torch

import paper_0911_4114_amd as ff
from paper_0911_4114_amd import workloads as wl
from oracle.quadrature import LevelQuad


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev_points(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def dev_complex(q, fp32=False):
    t = torch.as_tensor(np.ascontiguousarray(q), dtype=torch.complex128, device="cuda")
    return t.to(torch.complex64) if fp32 else t


def oracle_quads(plan):
    """The plan's integer quadrature parameters as oracle LevelQuads."""
    info = plan.info()
    return {l: LevelQuad(info["ell"][l], info["ntheta"][l], plan.nphi(l))
            for l in range(2, info["depth"] + 1)}


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))
