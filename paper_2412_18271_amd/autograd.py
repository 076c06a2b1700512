"""torch.autograd binding of the HIP energy and its hand-written adjoint.

The paper's force-provider contract lets a model return only the energy and
obtains forces by differentiating it (Methods section).  Here the forward pass
is the library's energy evaluation and the backward pass is its adjoint
(descriptor chain rule through the network input gradient), so autograd never
traces the computation.  PyTorch supplies the device buffers and the stream;
every arithmetic step runs in the HIP library.

Two memory modes:
  recompute  forward keeps only the positions and the pair list; backward
             recomputes descriptors and the network before the adjoint;
  store      forward also keeps the descriptors and dE/dG (2 x 384 floats per
             atom); backward runs the adjoint alone.
"""

from __future__ import annotations

import itertools

import numpy as np
import torch

from .context import Context

_ids = itertools.count(1)


class NNPEnergy(torch.autograd.Function):
    """E = NNPEnergy.apply(pos, model): per-molecule energies (float64) of
    positions pos [n_atoms, 3] (float32 or float64, on the model's device)."""

    @staticmethod
    def forward(ctx, pos, model):
        p = pos.detach().contiguous()
        model._ensure_layout(p)
        E = torch.empty(model.n_molecules, dtype=torch.float64, device=p.device)
        model.ctx.energy_device(p.data_ptr(), p.dtype == torch.float64, E.data_ptr(), model.mode == "store")
        ctx.model = model
        ctx.call_id = model._last_call = next(_ids)
        ctx.save_for_backward(p)
        return E

    @staticmethod
    def backward(ctx, gE):
        (p,) = ctx.saved_tensors
        model = ctx.model
        if model._last_call != ctx.call_id:
            # another evaluation ran on the context since this forward
            scratch = torch.empty(model.n_molecules, dtype=torch.float64, device=p.device)
            model.ctx.energy_device(p.data_ptr(), p.dtype == torch.float64, scratch.data_ptr(),
                                    model.mode == "store")
            model._last_call = ctx.call_id
        F = torch.empty((p.shape[0], 3), dtype=torch.float64, device=p.device)
        model.ctx.forces_device(F.data_ptr())
        scale = gE.to(torch.float64)[model.atom_molecule]
        grad = (-F * scale[:, None]).to(p.dtype)
        return grad, None


class NNPModel(torch.nn.Module):
    """Energy model over one or more independent molecules.

    The library context runs on the current PyTorch stream of `device` at
    construction, so the kernels it enqueues are ordered with the tensors'
    producers and consumers on that stream.
    """

    def __init__(self, species, masses, weights, mol_offsets=None, dtype: str = "bf16x3",
                 mode: str = "recompute", device: str = "cuda", box=None, **kw):
        super().__init__()
        if mode not in ("recompute", "store"):
            raise ValueError("mode must be 'recompute' or 'store'")
        self.mode = mode
        self.device = torch.device(device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self.ctx = Context(species, masses, weights, mol_offsets, dtype=dtype, stream=stream, **kw)
        if box is not None:
            self.ctx.set_box(box)
        self.n_molecules = self.ctx.n_molecules
        off = np.asarray(self.ctx._off)
        mol = np.repeat(np.arange(self.n_molecules), np.diff(off))
        self.atom_molecule = torch.as_tensor(mol, dtype=torch.long, device=self.device)
        self._laid_out = False
        self._last_call = 0

    @classmethod
    def from_system(cls, system, **kw):
        kw.setdefault("box", getattr(system, "box", None))
        return cls(system.species, system.masses, system.weights, system.mol_offsets, **kw)

    def _ensure_layout(self, p):
        if not self._laid_out:
            # the library orders atoms by element, molecule and position once
            self.ctx.set_state(p.detach().double().cpu().numpy())
            self._laid_out = True

    def forward(self, pos):
        return NNPEnergy.apply(pos, self)

    def device_bytes(self) -> int:
        return self.ctx.device_bytes()
