"""Receiver traces of the coupled ROM stepping as a differentiable function of the S-fraction
blocks (torch.autograd), backed by the library's forward step and its discrete adjoint.

    model = RomTraces(handle, src_ijk, src_vec, rec_ijk, rec_rows, dt, wavelet, nsteps)
    traces = rom_traces(gamma, gamma_hat, model)        # gamma, gamma_hat: [S][k][p][p], any device
    loss = 0.5 * ((traces - observed) ** 2).sum()
    loss.backward()                                       # gamma.grad, gamma_hat.grad

Sources, receivers and their projections are held fixed; so are the face masses (Gamma-hat_1:
its gradient is returned as zero).  Every call runs on the GPU through libsfm.

The blocks can come from the learned surrogate, which makes the sound speed the variable:

    gamma, gamma_hat = surrogate_blocks(vel, net, handle)   # vel: device float32 nodes, requires_grad
    loss = 0.5 * ((rom_traces(gamma, gamma_hat, model) - observed) ** 2).sum()
    loss.backward()                                         # vel.grad through the network

(Gamma-hat_1 is taken from the ROMs the handle holds when surrogate_blocks runs.)
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
        # each gradient goes back on its input's device and in its dtype
        ctx.like = ((gamma.device, gamma.dtype), (gamma_hat.device, gamma_hat.dtype))
        return model.forward(g, gh)

    @staticmethod
    def backward(ctx, grad_traces):
        g_gam, g_hat = ctx.model.backward(*ctx.blocks, grad_traces)
        (dg, tg), (dh, th) = ctx.like
        return torch.from_numpy(g_gam).to(dg, tg), torch.from_numpy(g_hat).to(dh, th), None


def rom_traces(gamma: torch.Tensor, gamma_hat: torch.Tensor, model: RomTraces) -> torch.Tensor:
    """Traces [nrec][nsteps] (device, float32) of the ROMs with the given blocks."""
    return _RomTracesFn.apply(gamma, gamma_hat, model)


class _SurrogateBlocksFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vel, net, handle):
        info = sfm.sfm_query(handle.ctx)
        S, k, p = info["n_subdomains"], info["k"], info["p"]
        v = vel.detach().to(torch.float32).contiguous()
        coef = torch.empty((S, 2, k, p, p), dtype=torch.float64, device=v.device)
        sfm.sfm_surrogate_predict(handle.ctx, net, v, coef)
        ctx.net, ctx.handle = net, handle
        ctx.save_for_backward(v)
        blocks = coef.cpu()
        return blocks[:, 0].contiguous(), blocks[:, 1].contiguous()

    @staticmethod
    def backward(ctx, g_gam, g_hat):
        (v,) = ctx.saved_tensors
        info = sfm.sfm_query(ctx.handle.ctx)
        shape = (info["n_subdomains"], info["k"], info["p"], info["p"])
        gg = np.zeros(shape) if g_gam is None else g_gam.detach().cpu().numpy().astype(np.float64)
        gh = np.zeros(shape) if g_hat is None else g_hat.detach().cpu().numpy().astype(np.float64)
        grad = torch.zeros_like(v)
        sfm.sfm_surrogate_velocity_gradient(ctx.handle.ctx, ctx.net, v, gg, gh, grad)
        return grad, None, None


def surrogate_blocks(vel: torch.Tensor, net: sfm.Cnn, handle: sfm.Sfm):
    """(gamma, gamma_hat), CPU float64 [S][k][p][p], predicted by ``net`` from the sound speed
    ``vel`` (device float32 nodes), differentiable with respect to ``vel``."""
    return _SurrogateBlocksFn.apply(vel, net, handle)
