"""torch.autograd wrappers around the shifted-COCG library.

Observables of the Green's function are differentiable with respect to the stored
entries of H (Sec. 2.1.1: energy Tr[rho H] and forces through dH/dR).  Because
z - H is complex symmetric, the derivative of G = (z - H)^{-1} needs no second
(adjoint) solve: dG_jj/dH_ab = G_ja G_bj = x_j[a] x_j[b], with x_j the solutions
the forward solve already produced.  The library's backward kernel evaluates
this contraction on the GPU.

Hopping values can be produced from atomic positions by differentiable torch code
(``hopping_values``), so forces follow from autograd through t(r).
"""

import numpy as np
import torch

from . import api


def _vals_host(vals: torch.Tensor) -> np.ndarray:
    return vals.detach().to("cpu", torch.float64).contiguous().numpy()


class GreensDiag(torch.autograd.Function):
    """G[k, c] = [(z_k - H(vals))^{-1}]_{jj}, j = rhs_idx[c]; differentiable in vals.

    A pair that stops unconverged raises (ScocgError with ENOCONV) unless opts has
    allow_noconv=True; the per-pair report is available through the report argument."""

    @staticmethod
    def forward(ctx, vals, H: "api.Hamiltonian", z, rhs_idx, opts, report):
        opts = dict(opts or {})
        opts.setdefault("allow_noconv", False)
        H.update_values(_vals_host(vals))
        G, rep, tape, rc = api.greens_diag(H, z, rhs_idx, keep_tape=True, **opts)
        if report is not None:
            report.update(rep, rc=rc)
        ctx.tape = tape
        ctx.hamiltonian = H
        ctx.nnz = H.nnz
        ctx.vals_device = vals.device
        ctx.report = rep
        return G

    @staticmethod
    def backward(ctx, gG):
        grad = api.backward(ctx.tape, gG.to(torch.complex128).cuda())
        ctx.tape.close()
        return grad.to(ctx.vals_device), None, None, None, None, None


class BandEnergy(torch.autograd.Function):
    """E = Re sum_q w_q z_q Tr G(z_q) over the contour nodes (zero temperature),
    differentiable in vals: dE/dH_ab = Re sum_q w_q z_q (G_q G_q)_ab.  Unconverged pairs raise
    unless opts has allow_noconv=True."""

    @staticmethod
    def forward(ctx, vals, H: "api.Hamiltonian", z, w, opts):
        opts = dict(opts or {})
        opts.setdefault("allow_noconv", False)
        H.update_values(_vals_host(vals))
        out = api.density_matrix_energy(H, z, w, rhs_idx=None, want_rho=False, want_grad=True, **opts)
        ctx.save_for_backward(out["grad"])
        ctx.vals_device = vals.device
        return out["E"][0].to(vals.device)

    @staticmethod
    def backward(ctx, gE):
        (dE,) = ctx.saved_tensors
        return (gE.to(dE.device) * dE).to(ctx.vals_device), None, None, None, None


def greens_diag(vals, H, z, rhs_idx, report=None, **opts):
    """Differentiable G_jj(z_k).  report: optional dict that receives the per-pair report
    (iters, status, residuals) and the status code of the solve."""
    return GreensDiag.apply(vals, H, z, rhs_idx, opts, report)


def band_energy(vals, H, z, w, **opts):
    return BandEnergy.apply(vals, H, z, w, opts)


def hopping_values(bond_vec0, disp, bonds, blocks, entry_kind, entry_bond, entry_o1, entry_o2, onsite_vals,
                   decay=2.0, r0=np.sqrt(3.0) / 4.0):
    """Stored entries of a tight-binding H from atomic displacements (torch, differentiable).

    bond_vec0 [nb,3]: ideal minimum-image bond vectors; disp [natom,3]: displacements
    (requires_grad for forces); bonds [nb,2]: atom pairs (a < b); blocks [nb,4,4] raw
    hopping blocks.  A bond of length r carries t(r) = exp(-decay (r - r0)) times its
    block.  Per stored CSR entry: entry_kind 0 = on-site (value onsite_vals[e]), 1 = block
    element B[o1, o2] of bond entry_bond[e] (upper triangle), 2 = the transposed block
    element B[o2, o1] (lower triangle).
    """
    dvec = bond_vec0 + disp[bonds[:, 1]] - disp[bonds[:, 0]]
    r = torch.linalg.norm(dvec, dim=1)
    s = torch.exp(-decay * (r - r0))
    hop = s[entry_bond] * blocks[entry_bond, entry_o1, entry_o2]
    return torch.where(entry_kind == 0, onsite_vals, hop)
