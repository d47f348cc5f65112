"""Differentiable assembly (PyTorch, CPU) of the stored values of the upwind
convection-diffusion matrix A of ``workloads.convdiff_pencil`` from a per-cell
velocity field, in the sorted CSR order of that function's output.  Test-side user
code for the differentiation form: it maps d lambda / d A to d lambda / d v."""
import numpy as np
import torch

from paper_2310_18043_amd import workloads as W


class ConvDiffAssembly:
    def __init__(self, n: int, diffusion: float = 1.0, shift: complex = 0.05j):
        self.n = n
        self.h = 1.0 / (n + 1)
        self.dd = diffusion / self.h ** 2
        self.shift = shift
        N = n * n
        idx = np.arange(N).reshape(n, n)
        iy, ix = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        rows = [idx.ravel()]
        cols = [idx.ravel()]
        self.masks = []
        for mask, di, dj in ((ix > 0, 0, -1), (ix < n - 1, 0, 1), (iy > 0, -1, 0),
                             (iy < n - 1, 1, 0)):
            rows.append(idx[mask])
            cols.append(idx[(iy + di)[mask], (ix + dj)[mask]])
            self.masks.append(torch.from_numpy(mask.ravel()))
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
        self.order = torch.from_numpy(np.lexsort((cols, rows)))
        # pattern check against the generator
        A, _ = W.convdiff_pencil(n, diffusion, (1.0, 1.0), shift, None, 0)
        assert np.array_equal(A.indices, cols[self.order.numpy()])

    def values(self, v: torch.Tensor) -> torch.Tensor:
        """v: float64 (2, n, n) [component, iy, ix] -> complex128 stored values of A."""
        h, dd = self.h, self.dd
        vx = v[0].reshape(-1)
        vy = v[1].reshape(-1)
        relu = torch.relu
        diag = 4.0 * dd + torch.abs(vx) / h + torch.abs(vy) / h
        parts = [diag.to(torch.complex128) + self.shift]
        w = -dd - relu(vx) / h
        e = -dd - relu(-vx) / h
        s = -dd - relu(vy) / h
        nn_ = -dd - relu(-vy) / h
        for val, m in zip((w, e, s, nn_), self.masks):
            parts.append(val[m].to(torch.complex128))
        allv = torch.cat(parts)
        return allv[self.order]
