"""torch.autograd exposure of the library's derivatives (gradients of the
spectra, section 3 of arXiv 2602.15104; the six parameters of its gradient
tables in section 4.3).

spectra_from_sources(context, tabs, ell_max, S) -> C_l [n][3][ell_max+1]
    differentiable in the sources S [n][n_k][3][n_tau]: the forward pass is
    the line-of-sight projection and the k quadrature (cmb_los, cmb_cl), the
    backward pass their transposes (cmb_spectra_adjoint).

cl_of_params(context, theta, base_cosmo, prec, k, n_tau, ell_max) -> C_l
    differentiable in theta [n][6] = (h, omega_b, omega_cdm, ln A_s, n_s,
    tau_reio): the forward pass builds each row's tables and runs the path
    (cmb_solve); the backward pass hands the incoming dL/dC_l to
    cmb_gradient, the discrete adjoint of the path (reverse ESDIRK sweep over
    checkpointed segments), which returns dL/dtheta.

Argument marshalling only: projection, quadrature, their transposes, the
perturbation runs, the reverse sweep and the gradient's assembly run in the
library's kernels (the library must be loaded; there is no fallback).
"""
from __future__ import annotations

import math

import torch

from . import Tables, solve_batch

#: the parameters of cl_of_params, in the column order of theta
PARAMS = ("h", "omega_b", "omega_cdm", "ln_A_s", "n_s", "tau_reio")


def _cosmo_at(base: dict, row) -> dict:
    c = dict(base)
    h, ob, oc, lnas, ns, tau = (float(v) for v in row)
    c.update(h=h, omega_b=ob, omega_cdm=oc, A_s=math.exp(lnas), n_s=ns, tau_reio=tau, z_reio=float("nan"))
    return c


class _SpectraFromSources(torch.autograd.Function):
    @staticmethod
    def forward(fctx, S, context, tabs, ell_max):
        S = S.contiguous()
        if S.dtype != torch.float64 or not S.is_cuda or S.dim() != 4 or S.shape[2] != 3:
            raise ValueError("S must be a float64 device tensor [n][n_k][3][n_tau]")
        n, n_k = int(S.shape[0]), int(S.shape[1])
        if n != len(tabs):
            raise ValueError("one table per cosmology row of S")
        Delta = torch.empty((n, 2, n_k, ell_max - 1), dtype=torch.float64, device=S.device)
        Cl = torch.empty((n, 3, ell_max + 1), dtype=torch.float64, device=S.device)
        stream = torch.cuda.current_stream(S.device).cuda_stream
        context.los(tabs, ell_max, S, Delta, stream=stream)
        context.cl(tabs, ell_max, Delta, Cl, stream=stream)
        fctx.save_for_backward(Delta)
        fctx.meta = (context, tabs, ell_max, tuple(S.shape))
        return Cl

    @staticmethod
    def backward(fctx, gCl):
        (Delta,) = fctx.saved_tensors
        context, tabs, ell_max, shape = fctx.meta
        gS = torch.empty(shape, dtype=torch.float64, device=Delta.device)
        stream = torch.cuda.current_stream(Delta.device).cuda_stream
        context.spectra_adjoint(tabs, ell_max, Delta, gCl.contiguous(), gS, stream=stream)
        return gS, None, None, None


def spectra_from_sources(context, tabs, ell_max: int, S: torch.Tensor) -> torch.Tensor:
    """C_l(S) for the tables' geometry; backward gives dL/dS."""
    return _SpectraFromSources.apply(S, context, tabs, int(ell_max))


class _ClOfParams(torch.autograd.Function):
    @staticmethod
    def forward(fctx, theta, context, base_cosmo, prec, k, n_tau, ell_max, rel, device):
        th = theta.detach().to("cpu", torch.float64)
        if th.dim() != 2 or th.shape[1] != 6:
            raise ValueError("theta must be [n][6] = (h, omega_b, omega_cdm, ln A_s, n_s, tau_reio)")
        n = int(th.shape[0])
        tabs = [Tables(_cosmo_at(base_cosmo, th[i].tolist()), prec, k, n_tau) for i in range(n)]
        out = solve_batch(context, tabs, ell_max, keep_S=False, keep_Delta=False,
                          stream=torch.cuda.current_stream(device).cuda_stream)
        if int(out["status"].abs().max().item()) != 0:
            raise RuntimeError("cmb_solve: a perturbation mode failed (per-mode status is nonzero)")
        fctx.meta = (context, tabs, ell_max, rel, device, theta.dtype, theta.device)
        return out["Cl"]

    @staticmethod
    def backward(fctx, gCl):
        context, tabs, ell_max, rel, device, dtype, dev = fctx.meta
        n, n_k = len(tabs), len(tabs[0].k)
        g = gCl.to(device, torch.float64).contiguous()
        Cl = torch.empty((n, 3, ell_max + 1), dtype=torch.float64, device=device)
        grad = torch.empty((n, 6), dtype=torch.float64, device=device)
        status = torch.empty((n, n_k), dtype=torch.int32, device=device)
        context.gradient(tabs, ell_max, g, Cl, grad, status, rel=rel,
                         stream=torch.cuda.current_stream(device).cuda_stream)
        if int(status.abs().max().item()) != 0:
            raise RuntimeError("cmb_gradient: a perturbation mode failed (per-mode status is nonzero)")
        return grad.to(dev, dtype), None, None, None, None, None, None, None, None


def cl_of_params(context, theta: torch.Tensor, base_cosmo: dict, prec: dict, k, n_tau: int, ell_max: int,
                 rel: float = 1e-4, device: str = "cuda:0") -> torch.Tensor:
    """C_l [n][3][ell_max+1] at theta [n][6]; backward gives dL/dtheta by
    cmb_gradient (the discrete adjoint of the frozen-step path; the tables'
    dependence on h, omega_b, omega_cdm and tau_reio by central differences
    at relative step rel; ln A_s and n_s exact).  base_cosmo supplies every
    other parameter; theta's tau_reio replaces any z_reio in it."""
    return _ClOfParams.apply(theta, context, base_cosmo, prec, k, int(n_tau), int(ell_max), float(rel), device)
