"""Pins of the oracle's velocity sets (Appendix A, Velocity Sets).

The tables are checked against the matrices printed in the paper (golden files)
and against the isotropy conditions every D3Q19/D2Q9 set must satisfy, which do
not depend on how the table was typed.
"""
import os
from itertools import product

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")
CS2 = 1.0 / 3.0


def _golden(name):
    return np.loadtxt(os.path.join(GOLD, name), comments="#").astype(int)


@pytest.mark.parametrize("which,fname", [(19, "d3q19_velocity_set.txt"), (9, "d2q9_velocity_set.txt")])
def test_table_matches_printed_matrix(oracle_mod, which, fname):
    c, w, opp = oracle_mod.lattice(which)
    g = _golden(fname)
    assert np.array_equal(c[:, : g.shape[0]].T, g)
    if which == 9:
        assert np.all(c[:, 2] == 0)


@pytest.mark.parametrize("which", [19, 9])
def test_isotropy(oracle_mod, which):
    c, w, opp = oracle_mod.lattice(which)
    d = 3 if which == 19 else 2
    c = c[:, :d].astype(float)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose(w @ c, 0.0, atol=1e-16)
    m2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(m2, CS2 * np.eye(d), atol=1e-16)
    m3 = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert np.allclose(m3, 0.0, atol=1e-16)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    dl = np.eye(d)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", dl, dl) + np.einsum("ac,bd->abcd", dl, dl)
                      + np.einsum("ad,bc->abcd", dl, dl))
    assert np.allclose(m4, iso, atol=1e-16)


@pytest.mark.parametrize("which", [19, 9])
def test_opposites(oracle_mod, which):
    c, w, opp = oracle_mod.lattice(which)
    q = len(w)
    assert opp[0] == 0
    for i in range(q):
        assert np.array_equal(c[opp[i]], -c[i])
        assert w[opp[i]] == w[i]
    if which == 19:
        # the printed ordering pairs direction i with i + 9
        assert all(opp[i] == i + 9 for i in range(1, 10))
    else:
        assert all(opp[i] == i + 4 for i in range(1, 5))


def test_d3q19_has_no_corner_directions(oracle_mod):
    c, _, _ = oracle_mod.lattice(19)
    all_dirs = {tuple(v) for v in product((-1, 0, 1), repeat=3) if sum(abs(x) for x in v) <= 2}
    assert {tuple(v) for v in c} == all_dirs
