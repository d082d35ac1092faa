"""Helpers shared by the GPU tests (no method arithmetic here)."""

import math

import numpy as np


def to_dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def line_angle(a, b):
    """Angle between the lines spanned by vectors a and b."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    a = a / np.linalg.norm(a)
    b = b / np.linalg.norm(b)
    c = float(a @ b)
    return math.atan2(float(np.linalg.norm(a - c * b)), abs(c))


def stop_model(eps, r):
    """Stopping-error model of the power method: angle left at stop and the
    relative error of sigma from the Rayleigh quotient, r = (s_{l+1}/s_l)^2."""
    theta = math.sqrt(2 * eps) * r / (1 - r)
    return theta, (1 - r) * theta ** 2 / 2
