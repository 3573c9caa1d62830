"""Ising-model tensors and exact partition functions (oracle).

Test infrastructure only (see the package docstring).

The benchmark model is the 2-D classical Ising model (Section IV,
Eq. ising_model), Z = sum over spin configurations of
exp(beta * sum_<ij> s_i s_j + beta*h * sum_i s_i), with J = k_B = 1.  The
paper works at h = 0; a field h is kept as an option (sign convention:
the weight grows with beta*h*s).

Two tensor-network constructions are provided, both with legs ordered
(l, u, r, d) and leg index 0 meaning spin +1 where a leg carries a spin:

* ``site_tensor``: one tensor per spin ("vertex" construction).  Every
  nearest-neighbour Boltzmann factor exp(beta s s') is split as
  sum_b W[s,b] W[s',b] with W = [[sqrt(cosh b), sqrt(sinh b)],
  [sqrt(cosh b), -sqrt(sinh b)]]; the tensor sums the four half-bonds and
  the field factor over its spin.  An L x L torus of these tensors has
  trace Z of the L x L Ising torus.
* ``plaquette_tensor``: spins live on the bonds of the network and each
  tensor holds the four interactions between cyclically adjacent leg spins
  (Section III, Fig. 1 and its caption: the red lines around each tensor).
  The field is split in half between the two tensors sharing a spin.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import integrate

SPIN = np.array([1.0, -1.0])  # leg index 0 <-> s = +1, index 1 <-> s = -1


def site_tensor(beta: float, h: float = 0.0) -> np.ndarray:
    """Vertex-construction site tensor T[l,u,r,d], bond dimension 2."""
    if beta < 0:
        raise ValueError("beta must be >= 0")
    c, s = math.sqrt(math.cosh(beta)), math.sqrt(math.sinh(beta))
    W = np.array([[c, s], [c, -s]])  # rows: spin +1, -1
    T = np.zeros((2, 2, 2, 2))
    for si, spin in enumerate(SPIN):
        w = W[si]
        T += math.exp(beta * h * spin) * np.einsum("a,b,c,d->abcd", w, w, w, w)
    return T


def plaquette_tensor(beta: float, h: float = 0.0) -> np.ndarray:
    """Plaquette-construction tensor A[l,u,r,d] (spins on the legs)."""
    A = np.zeros((2, 2, 2, 2))
    for l, u, r, d in itertools.product(range(2), repeat=4):
        sl, su, sr, sd = SPIN[l], SPIN[u], SPIN[r], SPIN[d]
        e = beta * (sl * su + su * sr + sr * sd + sd * sl) + 0.5 * beta * h * (sl + su + sr + sd)
        A[l, u, r, d] = math.exp(e)
    return A


# ----------------------------------------------------------------------------
# Exact partition functions
# ----------------------------------------------------------------------------

def _logsumexp(x: np.ndarray) -> float:
    m = float(np.max(x))
    return m + math.log(float(np.sum(np.exp(x - m))))


def brute_force_lnZ_torus(L: int, beta: float, h: float = 0.0, Ly: int | None = None) -> float:
    """ln Z of the Lx x Ly periodic Ising model by summing all 2^(Lx*Ly)
    configurations.  Bonds are (site, right neighbour) and (site, down
    neighbour) for every site, so multi-edges on a width-2 torus are
    counted as the two distinct bonds they are."""
    Lx, Ly = L, (L if Ly is None else Ly)
    n = Lx * Ly
    if n > 22:
        raise ValueError("brute force limited to 22 spins")
    conf = ((np.arange(2 ** n)[:, None] >> np.arange(n)[None, :]) & 1)
    s = 1.0 - 2.0 * conf.astype(np.float64)  # (2^n, n)
    s = s.reshape(-1, Ly, Lx)
    e = (s * np.roll(s, -1, axis=2)).sum(axis=(1, 2)) + (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    m = s.sum(axis=(1, 2))
    return _logsumexp(beta * e + beta * h * m)


def brute_force_lnZ_medial(L: int, beta: float, h: float = 0.0) -> float:
    """ln Z of the Ising model whose spins sit at the bond midpoints of an
    L x L periodic network, each spin coupled to the spins at offsets
    (+-1/2, +-1/2) (the medial lattice of the network).  This is the spin
    model the plaquette construction represents; it is built here from the
    geometry, not from the tensor."""
    # Spin positions in units of 1/2: horizontal-bond midpoints (2x+1, 2y),
    # vertical-bond midpoints (2x, 2y+1), all modulo 2L.
    pos = [((2 * x + 1) % (2 * L), (2 * y) % (2 * L)) for y in range(L) for x in range(L)]
    pos += [((2 * x) % (2 * L), (2 * y + 1) % (2 * L)) for y in range(L) for x in range(L)]
    index = {p: i for i, p in enumerate(pos)}
    n = len(pos)
    if n > 22:
        raise ValueError("brute force limited to 22 spins")
    edges = []
    for i, (px, py) in enumerate(pos):
        for dx, dy in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
            j = index[((px + dx) % (2 * L), (py + dy) % (2 * L))]
            edges.append((i, j))
    # each undirected edge was listed from both ends
    conf = ((np.arange(2 ** n)[:, None] >> np.arange(n)[None, :]) & 1)
    s = 1.0 - 2.0 * conf.astype(np.float64)
    e = np.zeros(s.shape[0])
    for i, j in edges:
        e += s[:, i] * s[:, j]
    e *= 0.5
    return _logsumexp(beta * e + beta * h * s.sum(axis=1))


def transfer_matrix_lnZ_torus(L: int, beta: float, h: float = 0.0) -> float:
    """ln Z of the L x L periodic Ising model as Tr(V^L) with the row-to-row
    transfer matrix V (2^L states).  The in-row energy and field of each
    row are split symmetrically between the two factors adjacent to it, so
    V is symmetric and Z = sum_i lambda_i^L."""
    if L > 12:
        raise ValueError("transfer matrix limited to L <= 12")
    conf = ((np.arange(2 ** L)[:, None] >> np.arange(L)[None, :]) & 1)
    s = 1.0 - 2.0 * conf.astype(np.float64)  # (2^L, L)
    row = beta * (s * np.roll(s, -1, axis=1)).sum(axis=1) + beta * h * s.sum(axis=1)
    inter = beta * (s @ s.T)
    logV = inter + 0.5 * row[:, None] + 0.5 * row[None, :]
    shift = float(np.max(logV))
    lam = np.linalg.eigvalsh(np.exp(logV - shift))
    # Z = exp(L*shift) * sum lam^L, lam may be negative
    amax = float(np.max(np.abs(lam)))
    total = float(np.sum((lam / amax) ** L))
    return L * shift + L * math.log(amax) + math.log(total)


def kaufman_lnZ_torus(L: int, beta: float) -> float:
    """ln Z of the L x L periodic zero-field Ising model from Kaufman's exact
    finite-lattice solution (Phys. Rev. 76, 1232 (1949)):
      Z = 1/2 (2 sinh 2K)^(L^2/2) (Z1 + Z2 + Z3 + Z4),
      Z1 = prod_{r=0}^{L-1} 2 cosh(L g_{2r+1}/2),  Z2 = same with sinh,
      Z3 = prod_{r=0}^{L-1} 2 cosh(L g_{2r}/2),    Z4 = same with sinh,
      cosh g_l = cosh 2K coth 2K - cos(pi l / L) for l >= 1 and
      g_0 = 2K + ln tanh K (signed).  Evaluated in the log domain."""
    K = beta
    c2 = math.cosh(2 * K) * (math.cosh(2 * K) / math.sinh(2 * K))  # cosh 2K coth 2K

    def gamma(l: int) -> float:
        if l == 0:
            return 2 * K + math.log(math.tanh(K))
        return math.acosh(c2 - math.cos(math.pi * l / L))

    def log_prod(vals, fn):
        sgn, acc = 1.0, 0.0
        for g in vals:
            x = L * g / 2.0
            if fn == "cosh":   # ln(2 cosh x) = |x| + ln(1 + e^{-2|x|})
                acc += abs(x) + math.log1p(math.exp(-2 * abs(x)))
            else:              # ln|2 sinh x| = |x| + ln(1 - e^{-2|x|})
                if x == 0.0:
                    return 0.0, -math.inf
                sgn *= 1.0 if x > 0 else -1.0
                acc += abs(x) + math.log(-math.expm1(-2 * abs(x)))
        return sgn, acc

    odd = [gamma(2 * r + 1) for r in range(L)]
    even = [gamma(2 * r) for r in range(L)]
    terms = [log_prod(odd, "cosh"), log_prod(odd, "sinh"), log_prod(even, "cosh"), log_prod(even, "sinh")]
    m = max(t[1] for t in terms)
    tot = sum(sg * math.exp(lg - m) for sg, lg in terms)
    return math.log(0.5) + 0.5 * L * L * math.log(2 * math.sinh(2 * K)) + m + math.log(tot)


def onsager_lnZ_per_site(beta: float) -> float:
    """Onsager's thermodynamic-limit free energy of the zero-field square
    lattice Ising model:
      ln Z / N = ln(2 cosh 2K) + (1/pi) int_0^{pi/2}
                 ln[(1 + sqrt(1 - kappa^2 sin^2 t)) / 2] dt,
      kappa = 2 sinh 2K / cosh^2 2K."""
    K = beta
    kap = 2 * math.sinh(2 * K) / math.cosh(2 * K) ** 2

    def f(t):
        return math.log((1.0 + math.sqrt(max(0.0, 1.0 - kap * kap * math.sin(t) ** 2))) / 2.0)

    val, _ = integrate.quad(f, 0.0, math.pi / 2, epsabs=1e-14, epsrel=1e-14, limit=400)
    return math.log(2 * math.cosh(2 * K)) + val / math.pi
