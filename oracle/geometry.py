"""Lattice indexing -- oracle (test infrastructure only).

The paper leaves the site ordering and boundary conditions open (Sec. 2.1 only
names the neighbours x +- a mu-hat of Eq. 1).  The readings used throughout:

* periodic boundary conditions in all four directions;
* dims = (N0, N1, N2, N3), N0 the time extent, x3 fastest:
  lex = ((x0*N1 + x1)*N2 + x2)*N3 + x3;
* parity p(x) = (x0+x1+x2+x3) mod 2, even = 0; within a parity the site with
  lexicographic index lex has even/odd index lex // 2 (a bijection because
  N3 is even); every extent must be even;
* neighbour table nb[s][mu] = lex(x + mu-hat), nb[s][4+mu] = lex(x - mu-hat).

Everything here is written with explicit coordinates (numpy integer arrays),
with no index arithmetic shortcuts.
"""
from __future__ import annotations

import numpy as np


def check_dims(dims) -> tuple:
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or any(d < 2 or d % 2 for d in dims):
        raise ValueError(f"lattice extents must be four even numbers >= 2, got {dims}")
    return dims


def volume(dims) -> int:
    return int(np.prod(check_dims(dims)))


def coords(dims) -> np.ndarray:
    """Coordinates x[s] = (x0,x1,x2,x3) of every site s in lexicographic order."""
    dims = check_dims(dims)
    return np.indices(dims).reshape(4, -1).T.astype(np.int64)


def lex_of(dims, x: np.ndarray) -> np.ndarray:
    n0, n1, n2, n3 = check_dims(dims)
    x = np.asarray(x)
    return ((x[..., 0] * n1 + x[..., 1]) * n2 + x[..., 2]) * n3 + x[..., 3]


def parity(dims) -> np.ndarray:
    return (coords(dims).sum(axis=1) & 1).astype(np.int64)


def neighbour_table(dims) -> np.ndarray:
    """nb[V][8]: forward neighbours (mu = 0..3) then backward neighbours."""
    dims = check_dims(dims)
    x = coords(dims)
    n = np.array(dims)
    nb = np.empty((x.shape[0], 8), dtype=np.int64)
    for mu in range(4):
        e = np.zeros(4, dtype=np.int64)
        e[mu] = 1
        nb[:, mu] = lex_of(dims, (x + e) % n)
        nb[:, 4 + mu] = lex_of(dims, (x - e) % n)
    return nb


def eo_index(dims) -> np.ndarray:
    """Index of each lexicographic site within its own parity."""
    return np.arange(volume(dims), dtype=np.int64) // 2


def lex_of_eo(dims) -> np.ndarray:
    """lex_of_eo[p][i]: the lexicographic site of parity p with eo index i."""
    dims = check_dims(dims)
    v = volume(dims)
    p = parity(dims)
    idx = eo_index(dims)
    out = np.full((2, v // 2), -1, dtype=np.int64)
    for par in (0, 1):
        sel = np.nonzero(p == par)[0]
        out[par, idx[sel]] = sel
    assert (out >= 0).all(), "even/odd index is not a bijection"
    return out


def eo_neighbour_table(dims) -> np.ndarray:
    """nb_eo[p][i][d]: eo index (within parity 1-p) of neighbour d of site (p, i)."""
    nb = neighbour_table(dims)
    leo = lex_of_eo(dims)
    idx = eo_index(dims)
    return np.stack([idx[nb[leo[p]]] for p in (0, 1)])


def split_eo(field: np.ndarray, dims) -> tuple:
    """Split a canonical field [..., V, ...site dofs] into (even, odd) halves in eo order.

    ``field`` must have the site axis at position -3 (spinors [.., V, 4, 3]).
    """
    leo = lex_of_eo(dims)
    return field[..., leo[0], :, :], field[..., leo[1], :, :]


def join_eo(even: np.ndarray, odd: np.ndarray, dims) -> np.ndarray:
    leo = lex_of_eo(dims)
    v = volume(dims)
    out = np.zeros(even.shape[:-3] + (v,) + even.shape[-2:], dtype=np.result_type(even, odd))
    out[..., leo[0], :, :] = even
    out[..., leo[1], :, :] = odd
    return out
