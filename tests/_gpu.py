"""Helpers shared by the GPU tests: device transfers, relative errors, and the
pairing of an oracle hierarchy with a library context on the same problem."""

import sys

import numpy as np
import pytest


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(x):
    torch = torch_cuda()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def zeros(n):
    torch = torch_cuda()
    return torch.zeros(int(n), dtype=torch.float64, device="cuda")


def pair(ne, length, P, overlap="min", omega=0.08, precond_bits=64, ns_pre=1, ns_post=1, growth=1):
    """(oracle Hierarchy, library Solver) for the same problem."""
    import oracle
    from paper_1612_04796_amd import sipg
    torch_cuda()
    h = oracle.Hierarchy(ne, length, P, overlap=overlap, omega=omega, ns_pre=ns_pre,
                         ns_post=ns_post, growth=growth)
    s = sipg.Solver(ne=ne, length=length, P=P, overlap=overlap, omega=omega,
                    precond_bits=precond_bits, nsmooth_pre=ns_pre, nsmooth_post=ns_post,
                    smooth_growth=growth)
    return h, s


def announce(*args):
    print("[gpu-case]", *args, flush=True)
    sys.stdout.flush()
