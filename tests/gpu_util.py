"""Helpers for the GPU tests: run the library through the C ABI and bring the
results back to the host.  No arithmetic of the method here."""
from __future__ import annotations

import sys

import numpy as np

from paper_2411_09859_amd import binding


def note(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def run_factor(A_np, block_size=0, precision=binding.FP64, lda=None, pfaffian=False):
    """Factor on cuda:0.  Returns dict with packed A (host, n x n), t, ipiv,
    and (log_abs_pf, sign) when requested, plus the full host buffer when
    lda > n (to check padding rows are untouched)."""
    import torch
    n = A_np.shape[0]
    lda = n if lda is None else lda
    buf = np.zeros((max(lda, 1), max(n, 1)), dtype=np.float64, order="F")
    buf[:] = 7.25  # sentinel in the padding rows
    buf[:n, :n] = A_np
    dev = torch.from_numpy(buf).to("cuda")  # stride (1, lda)
    Adev = dev[:n, :n] if n > 0 else dev[:0, :0]
    if n > 0:
        assert Adev.stride(0) == 1 and Adev.stride(1) == max(lda, 1)
    t = torch.zeros(max(n - 1, 1), dtype=torch.float64, device="cuda")
    ipiv = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    work = binding.alloc_workspace(binding.workspace_size(max(n, 1), block_size, precision))
    out = {}
    if pfaffian:
        la = torch.zeros(1, dtype=torch.float64, device="cuda")
        sg = torch.full((1,), 9, dtype=torch.int32, device="cuda")
        binding.pfaffian(Adev, t, ipiv, la, sg, block_size, precision, work)
    else:
        binding.factor(Adev, t, ipiv, block_size, precision, work)
    torch.cuda.synchronize()
    hbuf = np.asfortranarray(dev.cpu().numpy())
    out["buf"] = hbuf
    out["A"] = np.asfortranarray(hbuf[:n, :n])
    out["t"] = t.cpu().numpy()[: max(n - 1, 0)]
    out["ipiv"] = ipiv.cpu().numpy()[:n]
    if pfaffian:
        out["log_abs_pf"] = float(la.cpu().numpy()[0])
        out["sign"] = int(sg.cpu().numpy()[0])
    return out


def rel(a, b):
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))
