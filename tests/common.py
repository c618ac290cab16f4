"""Shared helpers for GPU parity tests: the same seeded mesh set up in the
oracle (CPU, FP64) and in libsem (GPU), plus ordering maps between them."""
from __future__ import annotations

import numpy as np

import fixtures as F
import oracle


class Pair:
    def __init__(self, mesh, N, precisions=("fp64", "fp32", "fp16", "bf16"), solver=True):
        import paper_2207_07098_amd as sem
        import torch
        self.torch = torch
        self.mesh = mesh
        self.N = N
        self.ora = oracle.setup(mesh, N)
        self.op = sem.Operator(mesh, N, precisions=precisions, solver=solver)
        self.gid, self.pos, self.dmask, self.mult = self.op.numbering()
        assert np.array_equal(self.gid, self.ora.gid)

    # canonical (oracle) <-> solver (library) order
    def to_dev(self, v_canonical, dtype=None):
        v = np.empty_like(v_canonical)
        v[self.pos] = v_canonical
        t = self.torch.from_numpy(np.ascontiguousarray(v))
        if dtype is not None:
            t = t.to(dtype)
        return t.to(self.op.device)

    def from_dev(self, t):
        v = t.detach().double().cpu().numpy()
        return v[self.pos]

    def local_to_dev(self, vL, dtype=None):
        t = self.torch.from_numpy(np.ascontiguousarray(vL.reshape(-1)))
        if dtype is not None:
            t = t.to(dtype)
        return t.to(self.op.device)


def relerr(a, b):
    d = np.max(np.abs(np.asarray(a) - np.asarray(b)))
    s = np.max(np.abs(b))
    return d / s if s > 0 else d


def sampled_apply(mesh, N, u_canonical, nodes, gid, xi=None):
    """Oracle y = M Q^T A_L Q M u at selected unique nodes only: runs the
    oracle element operator on the elements that hold a copy of a selected
    node (geometry of those elements from the fixture coordinates)."""
    if xi is None:
        xi, _ = oracle.gll(N)
    E = gid.shape[0]
    n_u = int(u_canonical.size)
    mult, dmask = oracle.mult_mask(N, gid, mesh.face_bc, n_u)
    sel = np.zeros(n_u, dtype=bool)
    sel[nodes] = True
    elems = np.nonzero(sel[gid].any(axis=1))[0]
    xyz = mesh.coords(xi, elements=elems)
    G, _ = oracle.geometry(N, xyz)
    um = np.where(dmask == 1, 0.0, u_canonical)
    uL = um[gid[elems]]
    wL = oracle.ax_local(N, G, uL)
    y = np.zeros(n_u)
    np.add.at(y, gid[elems].ravel(), wL.ravel())
    y[dmask == 1] = 0.0
    return y[nodes]
