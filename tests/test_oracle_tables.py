"""Pins of the oracle's lattice and force-stencil tables against exact
rational moment identities (Sec. 2: D3Q19 with c_s^2 = 1/3, W(1) = 1/6,
W(2) = 1/12 with fourth-order isotropy, and e2 = 1 after eq. bulkp)."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O

CS2 = Fraction(1, 3)


def _frac(values):
    return [Fraction(v).limit_denominator(100000) for v in values]


def _moment(vecs, ws, idx):
    tot = Fraction(0)
    for v, w in zip(vecs, ws):
        term = w
        for a in idx:
            term *= int(v[a])
        tot += term
    return tot


def _delta(a, b):
    return 1 if a == b else 0


@pytest.mark.parametrize("dim", [2, 3])
def test_lattice_moments(dim):
    xi, w = O.lattice(dim)
    ws = _frac(w)
    # the rational reconstruction is the stored double
    assert all(abs(float(a) - b) < 1e-16 for a, b in zip(ws, w))
    axes = range(dim)
    assert _moment(xi, ws, ()) == 1
    for a in axes:
        assert _moment(xi, ws, (a,)) == 0
        for b in axes:
            assert _moment(xi, ws, (a, b)) == CS2 * _delta(a, b)
            for c in axes:
                assert _moment(xi, ws, (a, b, c)) == 0
                for d in axes:
                    iso = (_delta(a, b) * _delta(c, d) + _delta(a, c) * _delta(b, d)
                           + _delta(a, d) * _delta(b, c))
                    assert _moment(xi, ws, (a, b, c, d)) == CS2 ** 2 * iso
    assert len(xi) == (9 if dim == 2 else 19)
    assert len({tuple(v) for v in xi}) == len(xi)


# ratios of the isotropic tensor of rank 2k: xx..x : (x^{2k-2} y^2) : ...
ISO = {4: [((0, 0, 0, 0), 3), ((0, 0, 1, 1), 1)],
       6: [((0,) * 6, 15), ((0, 0, 0, 0, 1, 1), 3), ((0, 0, 1, 1, 2, 2), 1)],
       8: [((0,) * 8, 105), ((0,) * 6 + (1, 1), 15), ((0,) * 4 + (1,) * 4, 9)]}


@pytest.mark.parametrize("dim,order,count,radius", [
    (2, 4, 8, 1), (2, 6, 12, 2), (2, 8, 24, 2), (3, 4, 18, 1), (3, 6, 32, 2)])
def test_stencil_isotropy(dim, order, count, radius):
    e, W = O.stencil(dim, order)
    Ws = _frac(W)
    assert len(e) == count
    assert np.abs(e).max() == radius
    # e2 = sum_a W_a (e_a^x)^2 = 1
    assert _moment(e, Ws, (0, 0)) == 1
    assert _moment(e, Ws, (0, 1)) == 0
    # every odd moment up to order+1 vanishes; every even tensor up to
    # `order` is isotropic
    for rank in range(1, order + 2):
        for idx in itertools.product(range(dim), repeat=rank):
            m = _moment(e, Ws, idx)
            if rank % 2 == 1:
                assert m == 0
    for rank in range(4, order + 1, 2):
        base = None
        for idx, ratio in ISO[rank]:
            if max(idx) >= dim:
                continue
            m = _moment(e, Ws, idx)
            if base is None:
                base = m / ratio
            assert m == base * ratio, (rank, idx, m, base)
    # the weights depend only on the squared length
    by_shell = {}
    for v, w in zip(e, Ws):
        by_shell.setdefault(int((v ** 2).sum()), set()).add(w)
    assert all(len(s) == 1 for s in by_shell.values())


def test_e4_weights_are_lattice_weights_over_cs2():
    """For E4 the stencil is the lattice itself and W_a = w_a / c_s^2; in 3D
    W(1) = 1/6 and W(2) = 1/12 as printed in Sec. 2."""
    for dim in (2, 3):
        e, W = O.stencil(dim, 4)
        xi, w = O.lattice(dim)
        wmap = {tuple(v): x for v, x in zip(xi, w)}
        for v, x in zip(e, W):
            assert abs(x - wmap[tuple(v)] * 3.0) < 1e-15
    e, W = O.stencil(3, 4)
    for v, x in zip(e, W):
        s = int((v ** 2).sum())
        assert abs(x - {1: 1 / 6, 2: 1 / 12}[s]) < 1e-16


def test_unsupported_stencils_rejected():
    with pytest.raises(ValueError):
        O.stencil(3, 8)
    with pytest.raises(ValueError):
        O.stencil(4, 4)
