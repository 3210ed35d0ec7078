"""Pins for the oracle's lattice indexing (periodic boundaries, lexicographic
order with x3 fastest, even/odd split by lex // 2)."""
import numpy as np
import pytest

from oracle import geometry


def test_handworked_neighbours_4x2x2x2():
    # dims (N0,N1,N2,N3) = (4,2,2,2): lex = ((x0*2 + x1)*2 + x2)*2 + x3
    dims = (4, 2, 2, 2)
    nb = geometry.neighbour_table(dims)
    # site 0 = (0,0,0,0)
    assert list(nb[0]) == [8, 4, 2, 1, 24, 4, 2, 1]
    # site 13 = (1,1,0,1)
    assert list(nb[13]) == [21, 9, 15, 12, 5, 9, 15, 12]
    # site 31 = (3,1,1,1): +0 wraps to x0 = 0
    assert list(nb[31]) == [7, 27, 29, 30, 23, 27, 29, 30]


def test_handworked_eo_4x2x2x2():
    dims = (4, 2, 2, 2)
    leo = geometry.lex_of_eo(dims)
    # parity of lex 0..7 (x0=0,x1=0): 0,1,1,0,1,0,0,1
    assert list(leo[0][:4]) == [0, 3, 5, 6]
    assert list(leo[1][:4]) == [1, 2, 4, 7]


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 6, 2), (6, 2, 4, 8)])
def test_tables_invariants(dims):
    nb = geometry.neighbour_table(dims)
    v = geometry.volume(dims)
    s = np.arange(v)
    par = geometry.parity(dims)
    for mu in range(4):
        assert (nb[nb[s, mu], 4 + mu] == s).all()
        assert (nb[nb[s, 4 + mu], mu] == s).all()
        assert (par[nb[s, mu]] != par).all()
    # each direction is a permutation of the sites
    for d in range(8):
        assert np.array_equal(np.sort(nb[:, d]), s)
    # walking N_mu steps returns home
    for mu in range(4):
        t = s.copy()
        for _ in range(dims[mu]):
            t = nb[t, mu]
        assert (t == s).all()


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 6, 2)])
def test_eo_bijection_and_neighbours(dims):
    leo = geometry.lex_of_eo(dims)
    v = geometry.volume(dims)
    assert np.array_equal(np.sort(leo.ravel()), np.arange(v))
    par = geometry.parity(dims)
    assert (par[leo[0]] == 0).all() and (par[leo[1]] == 1).all()
    nbe = geometry.eo_neighbour_table(dims)
    nb = geometry.neighbour_table(dims)
    for p in (0, 1):
        assert np.array_equal(leo[1 - p][nbe[p]], nb[leo[p]])


def test_odd_extent_rejected():
    with pytest.raises(ValueError):
        geometry.check_dims((4, 4, 4, 3))
