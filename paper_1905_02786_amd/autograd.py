"""torch.autograd wrapper of the summed MBE-FCI energy.

E = MBEFCIEnergy.apply(h1, eri, spec, workspace) runs the expansion on the
device; E.backward() asks the library for sum_S w_S (gamma(S), 1/2 Gamma(S)),
the density-matrix adjoint of Eq. 3 with the tuple set of the forward pass held
fixed.  h1 is (n, n) and eri the full (n, n, n, n) float64 tensor; the
gradients come back in the same layout and on the same device, every entry
treated as an independent variable.
"""
from __future__ import annotations

import numpy as np
import torch

from .api import Context


class MBEFCIEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h1, eri, spec, workspace):
        """spec: dict(nalpha, nbeta, nfrozen, ref, and Context options such as
        a, max_order)."""
        spec = dict(spec)
        lib = Context(device=workspace.device.index or 0)
        lib.set_hamiltonian(h1.detach().double().cpu().numpy(), eri.detach().double().cpu().numpy(),
                            spec.pop("e_const", 0.0))
        lib.set_spaces(spec.pop("nalpha"), spec.pop("nbeta"), spec.pop("nfrozen", 0), spec.pop("ref"))
        lib.set_options(**spec)
        res, handle = lib.run(workspace, keep=True)
        ctx.lib, ctx.handle, ctx.workspace = lib, handle, workspace
        ctx.h_meta = (h1.device, h1.dtype, eri.device, eri.dtype)
        ctx.result = res
        return torch.tensor(res.total, dtype=torch.float64, device=h1.device)

    @staticmethod
    def backward(ctx, gE):
        gh, ge = ctx.lib.backward(ctx.handle, ctx.workspace, float(gE))
        hd, ht, ed, et = ctx.h_meta
        return (torch.from_numpy(np.ascontiguousarray(gh)).to(device=hd, dtype=ht),
                torch.from_numpy(np.ascontiguousarray(ge)).to(device=ed, dtype=et), None, None)
