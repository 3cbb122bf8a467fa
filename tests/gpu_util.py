"""Helpers for the GPU tests: device tensors and one shared library context."""
import numpy as np
import torch

import paper_0910_1048_amd as sgn

_ctx = None


def ctx():
    global _ctx
    if _ctx is None:
        # torch owns the device memory of the tests: bring its HIP state up first
        torch.cuda.init()
        _ctx = sgn.Context(0)
    return _ctx


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def lattice(U, dims, kappa=0.2, bc=(1, 1, 1, -1)):
    return sgn.Lattice(ctx(), dev(U), dims, kappa, bc)
