"""FP64 oracle of the texture-gradient preconditioner (scipy sparse).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For texture optimisation the method preconditions its gradient samples as
proposed by Nicolet, Jacobson and Jakob ("Large Steps in Inverse Rendering of
Geometry", SIGGRAPH Asia 2021), cited in the Experiments section: a gradient
g is replaced by the solution y of

    (I + lambda L) y = g,

one system per channel, with L the combinatorial Laplacian (degree minus
adjacency) of the texel grid: texels are the nodes, each joined to its 4
neighbours inside the texture (no wrap-around).

Readings where the paper is silent:
  * The grid Laplacian stands in for the mesh Laplacian of the cited method
    (a texture is a regular grid of unknowns).
  * Both gradient samples, <F_i> and <dF_i>, are preconditioned before the
    meta-estimator (a linear map applied to the gradient the renderer
    returns); the baseline Adam preconditions its gradient the same way.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def grid_laplacian(tex_h: int, tex_w: int) -> sp.csr_matrix:
    """Degree minus adjacency of the 4-neighbour tex_h x tex_w grid; node
    index y * tex_w + x."""
    n = tex_h * tex_w
    rows, cols = [], []
    for y in range(tex_h):
        for x in range(tex_w):
            i = y * tex_w + x
            if x + 1 < tex_w:
                rows += [i, i + 1]
                cols += [i + 1, i]
            if y + 1 < tex_h:
                rows += [i, i + tex_w]
                cols += [i + tex_w, i]
    A = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    deg = np.asarray(A.sum(axis=1)).reshape(-1)
    return (sp.diags(deg) - A).tocsr()


def precondition(g, tex_h: int, tex_w: int, n_ch: int, lam: float) -> np.ndarray:
    """y with (I + lam L) y = g per channel; g in the texel-interleaved layout
    (texel * n_ch + channel)."""
    g = np.asarray(g, np.float64).reshape(tex_h * tex_w, n_ch)
    M = (sp.identity(tex_h * tex_w) + lam * grid_laplacian(tex_h, tex_w)).tocsc()
    lu = spla.splu(M)
    y = np.stack([lu.solve(g[:, c]) for c in range(n_ch)], axis=1)
    return y.reshape(-1)
