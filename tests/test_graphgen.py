"""Invariants of the seeded input generators (no method arithmetic here)."""
import numpy as np
import pytest

import graphgen


def assert_clean_symmetric(g):
    off, nbr = g.off, g.nbr
    assert off[0] == 0 and off[-1] == g.m
    assert np.all(np.diff(off) >= 0)
    assert nbr.min(initial=0) >= 0 and (g.m == 0 or nbr.max() < g.n)
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(off))
    assert not np.any(src == nbr), "self-loop"
    # sorted, duplicate-free lists
    same = src[1:] == src[:-1]
    assert np.all(nbr[1:][same] > nbr[:-1][same])
    # symmetric: the multiset of (x, y) equals that of (y, x)
    fwd = src * g.n + nbr
    rev = nbr.astype(np.int64) * g.n + src
    np.testing.assert_array_equal(np.sort(fwd), np.sort(rev))
    assert g.m % 2 == 0


def test_er_size_and_shape():
    g = graphgen.er(65536, 16, seed=1)
    assert g.n == 65536
    # expected directed entries n * 16 = 1,048,576 with sd about 1,448
    assert abs(g.m - 1_048_576) < 6 * 1448
    assert_clean_symmetric(g)


def test_er_deterministic_and_seeded():
    a = graphgen.er(5000, 8, seed=3)
    b = graphgen.er(5000, 8, seed=3)
    c = graphgen.er(5000, 8, seed=4)
    np.testing.assert_array_equal(a.nbr, b.nbr)
    assert a.m != c.m or not np.array_equal(a.nbr, c.nbr)
    # thread count does not change the result
    d = graphgen.er(5000, 8, seed=3, threads=1)
    np.testing.assert_array_equal(a.nbr, d.nbr)


@pytest.mark.parametrize("scale", [10, 14])
def test_rmat_shape(scale):
    g = graphgen.rmat(scale, seed=2)
    assert g.n == 1 << scale
    assert g.m <= 2 * 16 * (1 << scale)
    assert_clean_symmetric(g)
    deg = np.diff(g.off)
    # heavy skew: the max degree is far above the mean
    assert deg.max() > 20 * deg.mean()
    h = graphgen.rmat(scale, seed=2, threads=1)
    np.testing.assert_array_equal(g.nbr, h.nbr)


def test_rmat_permutation_is_bijection():
    a = graphgen.rmat(12, seed=5, permute=False)
    b = graphgen.rmat(12, seed=5, permute=True)
    assert a.m == b.m
    np.testing.assert_array_equal(np.sort(np.diff(a.off)), np.sort(np.diff(b.off)))
    # unpermuted R-MAT concentrates degree on low ids; permuted does not
    da, db = np.diff(a.off), np.diff(b.off)
    assert da[0] == da.max()
    assert db.argmax() != 0 or db[0] != db.max()


@pytest.mark.parametrize("H,W", [(1, 1), (1, 5), (4, 4), (3, 7), (64, 65)])
def test_grid(H, W):
    g = graphgen.grid(H, W)
    assert g.n == H * W
    assert g.m == 2 * (H * (W - 1) + W * (H - 1))
    assert_clean_symmetric(g)


def test_mixture():
    mix = graphgen.mixture(24, seed=1, nmin=1e3, nmax=2e4)
    assert mix.num_graphs == 24
    assert mix.vtx_off[0] == 0 and mix.vtx_off[-1] == mix.n
    kinds = set(int(k) for k in mix.kinds)
    assert kinds <= {0, 1, 2}
    for gi in range(mix.num_graphs):
        sub = mix.member(gi)
        assert_clean_symmetric(sub)
        kind, n, param = graphgen.member_spec(gi, 1, 1e3, 2e4)
        assert kind == mix.kinds[gi]
        if kind == graphgen.KIND_RMAT:
            assert sub.n == n
        elif kind == graphgen.KIND_GRID:
            assert sub.n >= n
        else:
            assert sub.n == n


def test_from_edges_helper():
    g = graphgen.from_edges(4, [(0, 1), (1, 2), (1, 2), (3, 3)], dedup=True)
    assert list(g.off) == [0, 1, 3, 4, 5]
    assert list(g.nbr) == [1, 0, 2, 1, 3]
