"""torch-facing API of the density-matrix solver.

``density(H, n_occ, ...)`` returns ``P = theta(mu I - H)`` computed by the
DNN-SP2 network on the GPU (Section II.D of arXiv 2107.02737).
``SP2Density`` wraps it as a ``torch.autograd.Function`` whose backward is
the library's branch-replay adjoint (``sp2_vjp``) and whose forward-mode
derivative is the library's JVP (``sp2_jvp``).  torch provides device memory
and streams only.
"""

from __future__ import annotations

import torch

from . import _lib


def _as_matrix(H, symmetrize):
    if H.dim() != 2 or H.shape[0] != H.shape[1]:
        raise ValueError("H must be a square matrix")
    if not H.is_cuda:
        raise ValueError("H must be a device tensor (there is no CPU path)")
    H = H.detach().to(torch.float32)
    if symmetrize:
        H = 0.5 * (H + H.T)
    return H.contiguous()


def density(H, n_occ, tol=1e-5, precision="bf16x3", refine="fp32", max_iter=100, stop_rule=1,
            stall_gate=-1.0, checkpoint_every=0, symmetrize=False, return_info=False,
            workspace=None, time_layers=False, bound_steps=0, bound_seed=0,
            split_derivatives=False, allow_unconverged=False, homo=None, lumo=None):
    """Density matrix of the symmetric ``H`` with ``n_occ`` occupied states.

    Returns ``P`` (FP32, same device), or ``(P, info)`` with ``info`` holding
    ``n_iter``, ``converged``, ``eps_min``, ``eps_max``, ``trace``,
    ``idem_err``, ``status`` and the ``branches`` string (1 = S^2).
    ``split_derivatives`` (BF16X3 with a tape) runs the JVP/VJP layer
    products in BF16X3 instead of FP32.  ``homo``/``lumo``: estimates of the
    highest occupied and lowest unoccupied eigenvalue (e.g. ``homo_lumo`` of
    a previous solve) select the accelerated network, which needs fewer
    layers (Section II.E).

    A solve that does not meet the stop test raises ``SP2Error``
    (``SP2_ERR_NOT_CONVERGED``) unless ``allow_unconverged``; then the last
    iterate is returned, and the workspace holds no derivative tape.
    """
    H = _as_matrix(H, symmetrize)
    n = H.shape[0]
    opt = _lib.make_options(precision, refine, max_iter, stop_rule, checkpoint_every, tol,
                            stall_gate, time_layers, bound_steps, bound_seed, split_derivatives,
                            homo, lumo)
    if workspace is None:
        workspace = _lib.allocate_workspace(n, opt, H.device)
    P = torch.empty_like(H)
    st, info, branches = _lib.sp2_density_ex(H, n_occ, opt, P, workspace)
    if st == _lib.SP2_ERR_NOT_CONVERGED and not allow_unconverged:
        raise _lib.SP2Error(st, _lib.sp2_last_error() + " (pass allow_unconverged=True to "
                            "receive the last iterate)")
    if return_info:
        d = info.as_dict()
        d["branches"] = branches
        d["workspace"] = workspace
        return P, d
    return P


class SP2Density(torch.autograd.Function):
    """``P = SP2Density.apply(H, n_occ, options_dict)``; differentiable in H
    with the spectral bounds and branch signs held fixed (exact at
    convergence).  ``options_dict`` takes the keyword arguments of
    ``density`` (``checkpoint_every`` defaults to 4).  The forward raises
    ``SP2Error`` when the solve does not converge: an unconverged network has
    no derivative tape."""

    @staticmethod
    def forward(ctx, H, n_occ, opts=None):
        opts = dict(opts or {})
        opts.setdefault("checkpoint_every", 4)
        if opts.get("allow_unconverged"):
            raise ValueError("SP2Density needs a converged solve (allow_unconverged is refused)")
        P, info = density(H, n_occ, return_info=True, **opts)
        ctx.workspace = info["workspace"]
        ctx.info = info
        return P

    @staticmethod
    def backward(ctx, gP):
        W = gP.detach().to(torch.float32).contiguous()
        G = torch.empty_like(W)
        _lib.sp2_vjp(ctx.workspace, W, G)
        return G, None, None

    @staticmethod
    def jvp(ctx, dH, _n_occ=None, _opts=None):
        H1 = dH.detach().to(torch.float32).contiguous()
        P1 = torch.empty_like(H1)
        _lib.sp2_jvp(ctx.workspace, H1, P1)
        return P1


def jvp(H, n_occ, H1, **opts):
    """Density matrix and its response ``(P, P1)`` to the perturbation ``H1``."""
    opts.setdefault("checkpoint_every", 4)
    P, info = density(H, n_occ, return_info=True, **opts)
    H1 = H1.detach().to(torch.float32).contiguous()
    P1 = torch.empty_like(H1)
    _lib.sp2_jvp(info["workspace"], H1, P1)
    return P, P1


def vjp(H, n_occ, W, **opts):
    """Density matrix and the gradient ``dTr(W P)/dH``."""
    opts.setdefault("checkpoint_every", 4)
    P, info = density(H, n_occ, return_info=True, **opts)
    W = W.detach().to(torch.float32).contiguous()
    G = torch.empty_like(W)
    _lib.sp2_vjp(info["workspace"], W, G)
    return P, G


def homo_lumo(H, P, steps=24, margin=0.05, seed=0, workspace=None):
    """Estimates ``(homo, lumo)`` of the highest occupied and lowest
    unoccupied eigenvalue of ``H`` from its density matrix ``P`` (Lanczos on
    the occupied and virtual projections), for ``density(..., homo=, lumo=)``
    of a nearby Hamiltonian.  Raises ``SP2Error`` when no gap is found."""
    H = _as_matrix(H, False)
    P = P.detach().to(torch.float32).contiguous()
    if workspace is None:
        workspace = _lib.allocate_workspace(H.shape[0], None, H.device)
    return _lib.sp2_homo_lumo(H, P, workspace, steps, seed, margin)

