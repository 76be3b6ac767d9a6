"""torch.autograd.Functions over the walk, differentiated with respect to the
scattering and absorption coefficients by the perturbation Monte Carlo
adjoint (mc_simulate with MC_MOMENTS forward, mc_grad backward).  Argument
marshalling only; the walk, the moments and the dot products run in the
library's kernels.

side_image(mu_sca, mu_abs, sim)
    The side image; backward is the exact derivative of this sample with the
    paths held fixed (right for losses linear in the image).
side_l2_loss(mu_sca, mu_abs, target, sim)
    sum_p (I_p - T_p)^2 - sum w^2 (the last sum over every photon leaving
    through the side image), an unbiased estimate of sum_p (E[I_p] - T_p)^2
    (plus the target's own variance, independent of the coefficients);
    backward subtracts the sample's self-correlation (uniform second
    derivative 2) so the gradient estimates that of the clean loss.
"""
from __future__ import annotations

from ._capi import (MC_EXIT_LOG, MC_MEDIUM_MU, MC_MOMENTS, MC_S_SIDE_W2, Detector, Geometry, Medium, Run, Source, Tally, mc_grad,
                    mc_simulate)


class SideImage:
    """Fixed parts of a walk (table, source, geometry, detector, run) whose
    side image is differentiated with respect to (mu_sca, mu_abs).  With
    MC_EXIT_LOG in the detector flags, every walk of this object shares one
    workspace holding the exit log."""

    def __init__(self, medium: Medium, source: Source, geometry: Geometry, detector: Detector, run: Run,
                 device="cuda"):
        self.medium, self.source, self.geometry, self.run = medium, source, geometry, run
        self.detector = Detector(detector.side_nx, detector.side_ny, detector.trans_nx, detector.trans_ny,
                                 detector.flags | MC_MOMENTS)
        self.device = device
        self._workspace = None

    def medium_for(self, mu_sca: float, mu_abs: float) -> Medium:
        """The fixed medium with its coefficients given directly (MC_MEDIUM_MU):
        the library derives mu_ext and the albedo."""
        m = Medium()
        for f, _ in Medium._fields_:
            setattr(m, f, getattr(self.medium, f))
        m.input = MC_MEDIUM_MU
        m.mu_sca = mu_sca
        m.mu_abs = mu_abs
        return m

    def run_walk(self, mu_sca: float, mu_abs: float):
        med = self.medium_for(mu_sca, mu_abs)
        tally = Tally.alloc(self.detector, self.device, moments=True, log_photons=self.run.n_photons,
                            workspace=self._workspace)
        if self.detector.flags & MC_EXIT_LOG:
            self._workspace = tally.workspace
        mc_simulate(med, self.source, self.geometry, self.detector, self.run, tally)
        return med, tally


_fns = {}


def _functions():
    if _fns:
        return _fns
    import torch

    def _grads(ctx, d_ms, d_ma, scale):
        dt_s, dv_s, dt_a, dv_a = ctx.dtypes
        return (torch.tensor(d_ms * scale, dtype=dt_s, device=dv_s),
                torch.tensor(d_ma * scale, dtype=dt_a, device=dv_a))

    class _SideImageFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, mu_sca, mu_abs, sim):
            med, tally = sim.run_walk(float(mu_sca), float(mu_abs))
            ctx.sim, ctx.med, ctx.tally = sim, med, tally
            ctx.dtypes = (mu_sca.dtype, mu_sca.device, mu_abs.dtype, mu_abs.device)
            return tally.side.clone()

        @staticmethod
        def backward(ctx, grad_side):
            g = grad_side.to(torch.float64).contiguous()
            d_ms, d_ma, _ = mc_grad(ctx.med, ctx.sim.geometry, ctx.sim.detector, ctx.tally, g)
            return (*_grads(ctx, d_ms, d_ma, 1.0), None)

    class _SideL2Fn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, mu_sca, mu_abs, target, sim):
            med, tally = sim.run_walk(float(mu_sca), float(mu_abs))
            diff = tally.side - target
            loss = (diff * diff).sum() - tally.scalars[MC_S_SIDE_W2]
            ctx.sim, ctx.med, ctx.tally = sim, med, tally
            ctx.g = (2.0 * diff).contiguous()
            ctx.dtypes = (mu_sca.dtype, mu_sca.device, mu_abs.dtype, mu_abs.device)
            return loss

        @staticmethod
        def backward(ctx, grad_loss):
            d_ms, d_ma, _ = mc_grad(ctx.med, ctx.sim.geometry, ctx.sim.detector, ctx.tally, ctx.g,
                                    d2loss_uniform=2.0)
            return (*_grads(ctx, d_ms, d_ma, float(grad_loss)), None, None)

    _fns["image"] = _SideImageFn
    _fns["l2"] = _SideL2Fn
    return _fns


def side_image(mu_sca, mu_abs, sim: SideImage):
    """Side image as a differentiable function of the 0-d tensors mu_sca and mu_abs (1/mm)."""
    return _functions()["image"].apply(mu_sca, mu_abs, sim)


def side_l2_loss(mu_sca, mu_abs, target, sim: SideImage):
    """Variance-corrected L2 loss of the side image against `target` (device,
    float64), differentiable in mu_sca and mu_abs."""
    return _functions()["l2"].apply(mu_sca, mu_abs, target, sim)
