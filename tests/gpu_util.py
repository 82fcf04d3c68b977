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


class DeviceBatch:
    """A batch of matrices on cuda:0 with the device descriptor arrays of
    skltlt_batched (int32 orders and leading dimensions, pointer arrays)."""

    def __init__(self, mats, ldas=None):
        import torch
        self.torch = torch
        self.mats_np = [np.asfortranarray(M, dtype=np.float64) for M in mats]
        self.ns = [M.shape[0] for M in self.mats_np]
        self.ldas = ldas if ldas is not None else [max(n, 1) for n in self.ns]
        self.bufs, self.ts, self.ipivs = [], [], []
        for M, n, lda in zip(self.mats_np, self.ns, self.ldas):
            # rows: max(lda, n), so an entry declared with lda < n (rejected
            # by the library) still has a full host copy to compare against
            buf = np.full((max(lda, n, 1), max(n, 1)), 7.25, dtype=np.float64, order="F")
            buf[:n, :n] = M
            self.bufs.append(torch.from_numpy(buf).to("cuda"))
            self.ts.append(torch.full((max(n - 1, 1),), -5.0, dtype=torch.float64, device="cuda"))
            self.ipivs.append(torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda"))
        self.pristine = [b.clone() for b in self.bufs]
        dev = "cuda"
        self.n_dev = torch.tensor(self.ns, dtype=torch.int32, device=dev)
        self.lda_dev = torch.tensor(self.ldas, dtype=torch.int32, device=dev)
        self.A_ptrs = torch.tensor([b.data_ptr() for b in self.bufs], dtype=torch.int64, device=dev)
        self.t_ptrs = torch.tensor([t.data_ptr() for t in self.ts], dtype=torch.int64, device=dev)
        self.p_ptrs = torch.tensor([p.data_ptr() for p in self.ipivs], dtype=torch.int64, device=dev)
        B = len(self.mats_np)
        self.la = torch.zeros(B, dtype=torch.float64, device=dev)
        self.sg = torch.full((B,), 9, dtype=torch.int32, device=dev)
        self.info = torch.full((B,), 5, dtype=torch.int32, device=dev)
        self.work = binding.alloc_workspace(binding.batched_workspace_size(B))

    def restore(self):
        for b, p in zip(self.bufs, self.pristine):
            b.copy_(p)

    def run(self, max_n=None, block_size=0, stream=None):
        mx = max(self.ns) if max_n is None else max_n
        binding.batched(self.n_dev, self.A_ptrs, self.lda_dev, self.t_ptrs, self.p_ptrs,
                        self.la, self.sg, self.info, max(mx, 0), block_size, binding.FP64,
                        self.work, stream)

    def results(self):
        self.torch.cuda.synchronize()
        out = []
        la, sg, info = self.la.cpu().numpy(), self.sg.cpu().numpy(), self.info.cpu().numpy()
        for k, n in enumerate(self.ns):
            buf = np.asfortranarray(self.bufs[k].cpu().numpy())
            out.append({"buf": buf, "A": np.asfortranarray(buf[:n, :n]),
                        "t": self.ts[k].cpu().numpy()[: max(n - 1, 0)],
                        "ipiv": self.ipivs[k].cpu().numpy()[:n],
                        "log_abs_pf": float(la[k]), "sign": int(sg[k]), "info": int(info[k])})
        return out
