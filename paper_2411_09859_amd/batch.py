"""Device arenas for batches of small matrices and the batched entry point.

A batch lives in one device allocation (matrices packed column-major, each
with lda = n), with the device descriptor arrays skltlt_batched takes.  This
is argument marshalling only; the factorization runs in the library.
"""
from __future__ import annotations

import numpy as np

from . import binding


class Arena:
    """Matrices packed in one fp64 device buffer plus t, ipiv and outputs."""

    def __init__(self, mats, device="cuda"):
        import torch
        self.torch = torch
        self.ns = np.array([M.shape[0] for M in mats], dtype=np.int64)
        B = len(mats)
        sizes = self.ns * self.ns
        self.offs = np.concatenate([[0], np.cumsum(sizes)])[:-1]
        host = np.empty(int(sizes.sum()) if B else 1, dtype=np.float64)
        for k, M in enumerate(mats):
            n = int(self.ns[k])
            host[self.offs[k]:self.offs[k] + n * n] = np.asfortranarray(M, dtype=np.float64).ravel(order="F")
        self.data = torch.from_numpy(host).to(device)
        self.pristine = self.data.clone()
        tl = np.maximum(self.ns - 1, 1)
        self.toffs = np.concatenate([[0], np.cumsum(tl)])[:-1]
        self.t = torch.zeros(int(tl.sum()) if B else 1, dtype=torch.float64, device=device)
        il = np.maximum(self.ns, 1)
        self.ioffs = np.concatenate([[0], np.cumsum(il)])[:-1]
        self.ipiv = torch.zeros(int(il.sum()) if B else 1, dtype=torch.int32, device=device)
        base_a, base_t, base_i = self.data.data_ptr(), self.t.data_ptr(), self.ipiv.data_ptr()
        self.n_dev = torch.tensor(self.ns, dtype=torch.int32, device=device)
        self.lda_dev = torch.tensor(np.maximum(self.ns, 1), dtype=torch.int32, device=device)
        self.A_ptrs = torch.tensor(base_a + 8 * self.offs, dtype=torch.int64, device=device)
        self.t_ptrs = torch.tensor(base_t + 8 * self.toffs, dtype=torch.int64, device=device)
        self.p_ptrs = torch.tensor(base_i + 4 * self.ioffs, dtype=torch.int64, device=device)
        self.log_abs_pf = torch.zeros(max(B, 1), dtype=torch.float64, device=device)
        self.sign = torch.zeros(max(B, 1), dtype=torch.int32, device=device)
        self.info = torch.zeros(max(B, 1), dtype=torch.int32, device=device)
        self.work = binding.alloc_workspace(binding.batched_workspace_size(B), device)
        self.max_n = int(self.ns.max()) if B else 0
        self.batch = B

    def restore(self):
        self.data.copy_(self.pristine)

    def run(self, block_size=0, stream=None):
        binding.batched(self.n_dev, self.A_ptrs, self.lda_dev, self.t_ptrs, self.p_ptrs,
                        self.log_abs_pf, self.sign, self.info, self.max_n, block_size,
                        binding.FP64, self.work, stream)

    def matrix(self, k):
        n = int(self.ns[k])
        flat = self.data[int(self.offs[k]):int(self.offs[k]) + n * n]
        return flat.view(n, n).t()  # column-major view (stride (1, n))
