"""Helpers for the GPU parity tests (inputs from synth, expected values from the oracle)."""
import numpy as np
import torch

import synth


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel_err(got, want):
    return float(np.linalg.norm((got - want).ravel()) / np.linalg.norm(want.ravel()))


def site_err(got, want):
    """max over sites of |got - want|_site / max_site |want|_site."""
    g = got.reshape(got.shape[0], -1)
    w = want.reshape(want.shape[0], -1)
    return float(np.abs(g - w).max() / np.abs(w).max())
