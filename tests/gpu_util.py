"""Helpers shared by the GPU parity tests (device placement of factors)."""

import numpy as np

from paper_2407_15049_amd import lrsdp as L


def dev_factor(A, prec, ld=None, device="cuda:0"):
    """numpy (n, r) -> zero-padded torch (n, ld) in the precision's storage type."""
    import torch
    n, r = A.shape
    ld = ld or L.padded_ld(r, L.F64 if prec == L.F64 else L.F32)
    t = torch.zeros((n, ld), dtype=L.elem_dtype(prec), device=device)
    t[:, :r] = torch.from_numpy(np.ascontiguousarray(A)).to(device=device, dtype=t.dtype)
    return t


def host(t, r=None):
    a = t.detach().double().cpu().numpy()
    return a if r is None else a[:, :r]


def rounded(A, prec):
    """The float64 values the device holds after storing A in `prec`."""
    return A if prec == L.F64 else A.astype(np.float32).astype(np.float64)


def dev_vec(x, device="cuda:0"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(device)
