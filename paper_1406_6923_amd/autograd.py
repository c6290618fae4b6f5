"""Receiver traces of the coupled ROM stepping as a differentiable function of the S-fraction
blocks (torch.autograd), backed by the library's forward step and its discrete adjoint.

    model = RomTraces(handle, src_ijk, src_vec, rec_ijk, rec_rows, dt, wavelet, nsteps)
    traces = rom_traces(gamma, gamma_hat, model)        # gamma, gamma_hat: float64 [S][k][p][p]
    loss = 0.5 * ((traces - observed) ** 2).sum()
    loss.backward()                                       # gamma.grad, gamma_hat.grad

Sources, receivers and their projections are held fixed; so are the face masses (Gamma-hat_1:
its gradient is returned as zero).  Every call runs on the GPU through libsfm.
"""
from __future__ import annotations

import numpy as np
import torch

from . import sfm


class RomTraces:
    """Fixed parts of the run: context, point projections, time step, wavelets, step count."""

    def __init__(self, handle: sfm.Sfm, src_ijk, src_vec, rec_ijk, rec_rows, dt: float, wavelet: torch.Tensor,
                 nsteps: int, checkpoint_every: int = 100):
        self.h = handle
        self.src_ijk = np.asarray(src_ijk, dtype=np.int32).reshape(-1, 3)
        self.src_vec = np.asarray(src_vec, dtype=np.float64)
        self.rec_ijk = np.asarray(rec_ijk, dtype=np.int32).reshape(-1, 3)
        self.rec_rows = np.asarray(rec_rows, dtype=np.float64)
        self.dt = float(dt)
        self.wavelet = wavelet
        self.nsteps = int(nsteps)
        self.checkpoint_every = int(checkpoint_every)

    def load(self, gamma: np.ndarray, gamma_hat: np.ndarray) -> None:
        sfm.sfm_load_roms(self.h.ctx, gamma, gamma_hat, self.src_ijk, self.src_vec, self.rec_ijk, self.rec_rows)

    def forward(self, gamma: np.ndarray, gamma_hat: np.ndarray) -> torch.Tensor:
        self.load(gamma, gamma_hat)
        tr = torch.zeros((len(self.rec_ijk), self.nsteps), dtype=torch.float32, device=self.wavelet.device)
        sfm.sfm_step(self.h.ctx, self.nsteps, self.dt, self.wavelet, tr)
        return tr

    def backward(self, gamma: np.ndarray, gamma_hat: np.ndarray, grad_traces: torch.Tensor):
        self.load(gamma, gamma_hat)
        g = grad_traces.to(torch.float32).contiguous()
        return sfm.sfm_adjoint_gradient(self.h.ctx, self.nsteps, self.dt, self.wavelet, g, self.checkpoint_every)


class _RomTracesFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma, gamma_hat, model):
        g = gamma.detach().cpu().numpy().astype(np.float64)
        gh = gamma_hat.detach().cpu().numpy().astype(np.float64)
        ctx.model = model
        ctx.blocks = (g, gh)
        return model.forward(g, gh)

    @staticmethod
    def backward(ctx, grad_traces):
        g_gam, g_hat = ctx.model.backward(*ctx.blocks, grad_traces)
        return torch.from_numpy(g_gam), torch.from_numpy(g_hat), None


def rom_traces(gamma: torch.Tensor, gamma_hat: torch.Tensor, model: RomTraces) -> torch.Tensor:
    """Traces [nrec][nsteps] (device, float32) of the ROMs with the given blocks."""
    return _RomTracesFn.apply(gamma, gamma_hat, model)
