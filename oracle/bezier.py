"""Bezier blocks by interpolation, and their evaluation (Sec. 3.2.3).

The restriction of the LR-spline to one element is a single tri-variate
polynomial of tri-degree p.  Sec. 3.2.3 converts it to the Bernstein (Bezier)
basis of that element by computing the coefficients of an interpolating
polynomial: a change of basis, not an approximation.  Here the field is sampled
with Cox-de Boor (oracle.bspline) at the (p1+1)(p2+1)(p3+1) tensor points
u_k = (2k+1)/(2(p+1)) of the element (strictly inside it, so no value depends
on the continuity across faces) and the Kronecker collocation system
  F[kx,ky,kz] = sum_j C[jx,jy,jz] B^px_jx(u_kx) B^py_jy(u_ky) B^pz_jz(u_kz)
is solved one axis at a time.  B^p_j(u) = binom(p,j) u^j (1-u)^(p-j).

Coefficient layout: C[e, q, jx + (px+1)*(jy + (py+1)*jz)] for component q.
"""
from __future__ import annotations

from math import comb

import numpy as np


def bernstein(p: int, u: np.ndarray) -> np.ndarray:
    """Bernstein basis of degree p at u (any shape) -> [..., p+1] (FP64)."""
    u = np.asarray(u, dtype=np.float64)[..., None]
    j = np.arange(p + 1)
    coef = np.array([comb(p, int(k)) for k in j], dtype=np.float64)
    return coef * u ** j * (1.0 - u) ** (p - j)


def collocation_nodes(p: int) -> np.ndarray:
    return (2.0 * np.arange(p + 1) + 1.0) / (2.0 * (p + 1))


def extract(spline, evaluator, elems=None) -> np.ndarray:
    """FP64 Bezier coefficients [n, ncomp, nc] of the listed elements (all by
    default), by interpolation of the LR-spline evaluated with Cox-de Boor."""
    p = tuple(int(v) for v in spline.p)
    box = spline.elem_box if elems is None else spline.elem_box[np.asarray(elems)]
    n = box.shape[0]
    nodes = [collocation_nodes(p[d]) for d in range(3)]
    # points ordered (e, kz, ky, kx)
    uz, uy, ux = np.meshgrid(nodes[2], nodes[1], nodes[0], indexing="ij")
    u = np.stack([ux.ravel(), uy.ravel(), uz.ravel()], axis=1)           # [npt, 3]
    lo, hi = box[:, None, :3], box[:, None, 3:]
    x = lo + u[None, :, :] * (hi - lo)                                    # [n, npt, 3]
    F = evaluator.evaluate(x.reshape(-1, 3)).reshape(n, -1, spline.ncomp)
    F = F.transpose(0, 2, 1).reshape(n, spline.ncomp, p[2] + 1, p[1] + 1, p[0] + 1)
    Minv = [np.linalg.inv(bernstein(p[d], nodes[d])) for d in range(3)]   # [k, j] -> inverse
    C = np.einsum("jk,nqzyk->nqzyj", Minv[0], F)
    C = np.einsum("jk,nqzkx->nqzjx", Minv[1], C)
    C = np.einsum("jk,nqkyx->nqjyx", Minv[2], C)
    return C.reshape(n, spline.ncomp, -1)


def basis_on_element(p, box: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Tensor Bernstein basis values [m, nc] at points x [m,3] in boxes [m,6]."""
    lo, hi = box[:, :3], box[:, 3:]
    u = (np.asarray(x, dtype=np.float64) - lo) / (hi - lo)
    bx, by, bz = (bernstein(p[d], u[:, d]) for d in range(3))
    B = bz[:, :, None, None] * by[:, None, :, None] * bx[:, None, None, :]
    return B.reshape(x.shape[0], -1)


def evaluate(p, C: np.ndarray, box: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Field value [m, ncomp] from Bezier blocks C [m, ncomp, nc] at x [m,3]."""
    B = basis_on_element(p, box, x)
    return np.einsum("mqj,mj->mq", C, B)


def extract_adjoint(spline, evaluator, G: np.ndarray) -> np.ndarray:
    """Adjoint of `extract` with respect to the LR coefficients: given
    dL/dC [n_elem, ncomp, nc] returns dL/dc [n_bspl, ncomp] (FP64).

    The change of basis of Sec. 3.2.3 is linear in the coefficients c_i of
    Eq. 2: C_e = (M^-1 kron) F_e with F_e[k] = sum_i gamma_i c_i N_i(x_k) at
    the element's collocation points x_k.  Its transpose takes G_e back
    through the transposed inverse collocation matrices to point weights
    H_e[k], then dL/dc_i = gamma_i sum_e sum_k N_i(x_k) H_e[k]."""
    p = tuple(int(v) for v in spline.p)
    box = spline.elem_box
    n, nq = box.shape[0], spline.coef.shape[1]
    nodes = [collocation_nodes(p[d]) for d in range(3)]
    Minv = [np.linalg.inv(bernstein(p[d], nodes[d])) for d in range(3)]
    H = np.asarray(G, dtype=np.float64).reshape(n, nq, p[2] + 1, p[1] + 1, p[0] + 1)
    H = np.einsum("jk,nqzyj->nqzyk", Minv[0], H)
    H = np.einsum("jk,nqzjx->nqzkx", Minv[1], H)
    H = np.einsum("jk,nqjyx->nqkyx", Minv[2], H)
    H = H.reshape(n, nq, -1).transpose(0, 2, 1).reshape(-1, nq)         # [(e, k), q]
    uz, uy, ux = np.meshgrid(nodes[2], nodes[1], nodes[0], indexing="ij")
    u = np.stack([ux.ravel(), uy.ravel(), uz.ravel()], axis=1)
    lo, hi = box[:, None, :3], box[:, None, 3:]
    x = (lo + u[None, :, :] * (hi - lo)).reshape(-1, 3)
    pt, bs, val = evaluator.basis(x)
    out = np.zeros((spline.coef.shape[0], nq))
    for q in range(nq):
        out[:, q] = np.bincount(bs, weights=val * H[pt, q], minlength=out.shape[0])
    return out * spline.gamma[:, None]
