"""Plaquette bookkeeping of TRG on a periodic lattice (oracle, independent mode).

Test infrastructure only (see the package docstring).

The paper applies the Levin-Nave TRG step (Section III, citing Levin and
Nave 2007) and requires that every tensor of every level be decomposed
with its own, independent random choice (Section III, the paragraph after
Eq. infiniteEnsemble).  Doing so needs the lattice at every level.

Conventions (this library's reading of the TRG geometry):
* legs are (l, u, r, d) = directions 0..3; leg r of a site joins leg l of
  its right neighbour, leg d joins leg u of the neighbour below;
* sublattice A sites are split (l,u)|(r,d) into F_A[l,u,a] G_A[a,r,d];
  sublattice B sites are split (u,r)|(d,l) into F_B[u,r,b] G_B[b,d,l];
* one new tensor per A site p0.  With q0 = r-neighbour of p0,
  p1 = d-neighbour of q0 and q1 = d-neighbour of p0, the new tensor is
  G_A(p0) G_B(q0) F_A(p1) F_B(q1) contracted around the plaquette;
  its legs (l', u', r', d') are the bonds a (of p0), b (of q0), c (of p1),
  e (of q1);
* the new l' leg of P(p0) joins the r' leg of P(l-neighbour of the
  u-neighbour of p0); the new u' leg joins the d' leg of P(u-neighbour of
  the r-neighbour of p0);
* new position ids are the ranks of the A-site ids; the new sublattices
  come from a 2-colouring that starts with position 0 in A.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass

import numpy as np

L_, U_, R_, D_ = 0, 1, 2, 3
OPP = (R_, D_, L_, U_)


@dataclass
class Level:
    nbr: np.ndarray     # (n, 4) neighbour position per leg
    is_a: np.ndarray    # (n,) bool

    @property
    def n(self) -> int:
        return int(self.nbr.shape[0])


def square_torus(L: int) -> Level:
    """L x L periodic square lattice, site id x + L*y, A = (x+y) even."""
    n = L * L
    nbr = np.empty((n, 4), dtype=np.int64)
    is_a = np.empty(n, dtype=bool)
    for y in range(L):
        for x in range(L):
            i = x + L * y
            nbr[i, L_] = (x - 1) % L + L * y
            nbr[i, U_] = x + L * ((y - 1) % L)
            nbr[i, R_] = (x + 1) % L + L * y
            nbr[i, D_] = x + L * ((y + 1) % L)
            is_a[i] = (x + y) % 2 == 0
    return Level(nbr, is_a)


def two_colour(nbr: np.ndarray) -> np.ndarray:
    n = nbr.shape[0]
    col = -np.ones(n, dtype=np.int64)
    col[0] = 0
    dq = deque([0])
    while dq:
        p = dq.popleft()
        for d in range(4):
            q = int(nbr[p, d])
            if col[q] < 0:
                col[q] = 1 - col[p]
                dq.append(q)
            elif n > 1 and col[q] == col[p]:
                raise ValueError("coarse lattice is not bipartite")
    if np.any(col < 0):
        raise ValueError("coarse lattice is not connected")
    return col == 0


def coarsen(lev: Level):
    """Plaquettes of one TRG step and the next level.

    Returns (plaq, next_level) with plaq[P] = (p0, q0, p1, q1) for new
    position P."""
    a_sites = np.flatnonzero(lev.is_a)
    newid = {int(p): i for i, p in enumerate(a_sites)}
    m = len(a_sites)
    plaq = np.empty((m, 4), dtype=np.int64)
    nbr2 = -np.ones((m, 4), dtype=np.int64)
    for P, p0 in enumerate(a_sites):
        p0 = int(p0)
        q0 = int(lev.nbr[p0, R_])
        p1 = int(lev.nbr[q0, D_])
        q1 = int(lev.nbr[p0, D_])
        if int(lev.nbr[q1, R_]) != p1 or lev.is_a[q0] or lev.is_a[q1] or not lev.is_a[p1]:
            raise ValueError("plaquette does not close")
        plaq[P] = (p0, q0, p1, q1)
    for P, p0 in enumerate(a_sites):
        p0 = int(p0)
        Ql = newid[int(lev.nbr[int(lev.nbr[p0, U_]), L_])]
        Qu = newid[int(lev.nbr[int(lev.nbr[p0, R_]), U_])]
        for leg, Q in ((L_, Ql), (U_, Qu)):
            if nbr2[P, leg] >= 0 or nbr2[Q, OPP[leg]] >= 0:
                raise ValueError("bond assigned twice")
            nbr2[P, leg] = Q
            nbr2[Q, OPP[leg]] = P
    if np.any(nbr2 < 0):
        raise ValueError("dangling bond")
    return plaq, Level(nbr2, two_colour(nbr2))


def network_Z(tensors, L):
    """Direct contraction of an L x L torus of tensors (legs l,u,r,d) with
    bonds (x,y).r--(x+1,y).l and (x,y).d--(x,y+1).u, row by row: each row
    becomes a matrix R_y[(u_0..u_{L-1}), (d_0..d_{L-1})] after summing its
    periodic horizontal bonds, and Z = Tr(R_0 R_1 ... R_{L-1}).  Exact up to
    rounding; the cost grows as D^(2L) (L = 8 at D = 2: 256 x 256 rows).
    Used for the exact Z of the 8 x 8 plaquette network of Table I."""
    rows = []
    for y in range(L):
        t = tensors[L * y]                         # (l0, u0, r, d0)
        D = t.shape[0]
        acc = t.transpose(0, 1, 3, 2)              # (l0, u0, d0, r)
        for x in range(1, L):
            nxt = tensors[x + L * y]               # (l, u, r, d)
            acc = np.tensordot(acc, nxt, axes=([acc.ndim - 1], [0]))  # (..., u, r, d)
            acc = np.moveaxis(acc, -2, -1)          # (..., u, d, r)
        # acc: (l0, u0, d0, u1, d1, ..., r); close the ring l0 == r
        acc = np.trace(acc, axis1=0, axis2=acc.ndim - 1)
        us = acc.transpose([2 * i for i in range(L)] + [2 * i + 1 for i in range(L)])
        rows.append(us.reshape(D ** L, D ** L))
    P = np.eye(rows[0].shape[0])
    for R in rows:
        P = P @ R
    return float(np.trace(P))
