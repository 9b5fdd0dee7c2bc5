"""Helpers for the GPU tests: device transfer and a shared library handle."""
import sys

import numpy as np


def note(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def to_host(t):
    return t.detach().cpu().numpy()


_CTX = None


def ctx():
    global _CTX
    import paper_2609_29554_amd as Z
    if _CTX is None:
        _CTX = Z.Context(0)
    return _CTX
