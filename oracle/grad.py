"""Reference gradient of f(X) = ||X - TT_r(X)||_F^2 through TT-RBKI with Omega fixed.

TEST INFRASTRUCTURE ONLY (see the package docstring).

An independent torch CPU float64 forward of the same step list as ``ttrbki.tt_rbki``
(the column-space block Krylov form, QR with column pivoting and drops, Rayleigh-Ritz,
carries), differentiated by torch's reverse-mode autodiff.  The discrete decisions
(mode kinds, QRCP pivot order and kept counts, completion) are taken from a float64
evaluation at the same X and held fixed: f is piecewise smooth and these choices are
constant on each piece.  Completion vectors, where they occur, are constants.

With left-orthonormal cores ||X - Xhat||^2 = ||X||^2 - ||C_{d-1}||^2 (Pythagoras, the
identity behind Eq. (12)), which is the form differentiated here.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np
import scipy.linalg
import torch

from .philox import omega
from .ttrbki import TAU, plan_modes, complete_columns, stream_precisions


def _qrcp_keep(P: np.ndarray, ref: float, tau: float):
    if P.shape[1] == 0:
        return np.zeros(0, dtype=int)
    _, R, piv = scipy.linalg.qr(P, mode="economic", pivoting=True)
    k = int(np.sum(np.abs(np.diag(R)) > tau * ref))
    return piv[:k]


def _orth(P: torch.Tensor, ref: float, tau: float) -> torch.Tensor:
    """Q of the QR of the kept pivot columns of P (positive diagonal of R)."""
    piv = _qrcp_keep(P.detach().numpy(), ref, tau)
    if len(piv) == 0:
        return P[:, :0]
    Q, R = torch.linalg.qr(P[:, torch.as_tensor(piv)])
    return Q * torch.sign(torch.diagonal(R))[None, :]


def _top_eig(M: torch.Tensor, r: int):
    lam, V = torch.linalg.eigh(0.5 * (M + M.T))
    return V[:, torch.argsort(lam, descending=True)[:r]]


def loss(X: torch.Tensor, targets: Sequence[int], q: int, p: int, seed: int = 0, tau: float = None,
         precision: str = "f64") -> torch.Tensor:
    """f(X) in torch float64 with autograd; X is a float64 CPU tensor."""
    dims = list(X.shape)
    modes = plan_modes(dims, targets, q, p)
    taus = [TAU[sp] if tau is None else tau for sp in stream_precisions(precision, modes)]
    C = X.reshape(1, -1)
    for mi, tau in zip(modes, taus):
        A = C.reshape(mi.m, mi.n)
        if mi.kind == "identity":
            continue
        if mi.kind == "saturated":
            if mi.m <= mi.n:
                lam, V = torch.linalg.eigh(A @ A.T)
                order = torch.argsort(lam, descending=True)[:mi.r]
                lam_r, G = lam[order], V[:, order]
            else:
                lam, V = torch.linalg.eigh(A.T @ A)
                order = torch.argsort(lam, descending=True)[:mi.r]
                lam_r = lam[order]
                G = (A @ V[:, order]) / torch.sqrt(torch.clamp(lam_r, min=1e-300))[None, :]
            tot = float(torch.sum(lam_r.detach()))
            valid = (lam_r > tau * tau * tot).numpy()
            if not valid.all():
                G = torch.cat([G[:, torch.as_tensor(np.where(valid)[0])],
                               torch.from_numpy(complete_columns(G[:, torch.as_tensor(np.where(valid)[0])]
                                                                 .detach().numpy(), mi.m, mi.r)[:, int(valid.sum()):])], 1)
        else:
            Om = torch.from_numpy(omega(seed, mi.k, 0, mi.n, mi.s))
            Y = A @ Om
            Qs = [_orth(Y, float(torch.linalg.norm(Y)), tau)]
            for _ in range(q):
                Y = A @ (A.T @ Qs[-1])
                Qp = torch.cat(Qs, 1)
                P = Y - Qp @ (Qp.T @ Y)
                Qs.append(_orth(P, float(torch.linalg.norm(Y)), tau))
            Q = torch.cat(Qs, 1)
            M = Q.T @ A @ (A.T @ Q)
            take = min(mi.r, Q.shape[1])
            G = Q @ _top_eig(M, take)
            if take < mi.r:
                comp = complete_columns(G.detach().numpy(), mi.m, mi.r)[:, take:]
                G = torch.cat([G, torch.from_numpy(comp)], 1)
        C = G.T @ A
    return torch.sum(X * X) - torch.sum(C * C)


def loss_and_grad(X: np.ndarray, targets, q, p, seed=0, tau=None, precision="f64"):
    Xt = torch.from_numpy(np.array(X, dtype=np.float64)).requires_grad_(True)
    f = loss(Xt, targets, q, p, seed, tau, precision)
    f.backward()
    return float(f), Xt.grad.numpy()
