"""The mutual-selection baseline (Section II-C) on the GPU against the
oracle's weighted greedy: with fixed edge weights both reach the greedy
matching in descending weight order, so they must agree bit for bit."""
import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2507_04420_amd as mm  # noqa: E402
from paper_2507_04420_amd import _lib  # noqa: E402


def to_dev(g):
    return torch.from_numpy(g.off).cuda(), torch.from_numpy(g.nbr).cuda()


GRAPHS = {
    "er": lambda: graphgen.er(30000, 10, seed=4),
    "er_int32": lambda: graphgen.er(65536, 16, seed=1).with_int32_offsets(),
    "rmat": lambda: graphgen.rmat(16, seed=2),
    "grid": lambda: graphgen.grid(120, 97),
    "clique": lambda: graphgen.from_edges(64, [(i, j) for i in range(64) for j in range(i + 1, 64)]),
    "star": lambda: graphgen.from_edges(5001, [(0, j) for j in range(1, 5001)]),
    "loops_dups": lambda: graphgen.from_edges(
        50, [(i, (i * 7) % 50) for i in range(50)] * 2 + [(3, 3), (9, 9)], dedup=False, sort=False),
    "empty": lambda: graphgen.from_edges(9, np.zeros((0, 2))),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("seed", [1, 77])
def test_ems_equals_weighted_greedy(name, seed):
    g = GRAPHS[name]()
    off, nbr = to_dev(g)
    h = mm.Graph(off, nbr, symmetric=True)
    mate, st = h.ems(seed=seed)
    got = mate.cpu().numpy()
    want, pairs = oracle.greedy_weighted(g, seed)
    np.testing.assert_array_equal(got, want)
    assert st["pairs"] == pairs
    assert oracle.check(g, got).ok
    assert st["iterations"] >= 1
    if g.m:
        assert st["touched"] >= g.m  # the first selection scans every list


def test_ems_needs_symmetric_handle():
    g = graphgen.er(100, 4, seed=1)
    off, nbr = to_dev(g)
    h = mm.Graph(off, nbr)
    with pytest.raises(mm.MMError) as ei:
        h.ems()
    assert ei.value.status == _lib.MM_ERR_UNSUPPORTED


def test_ems_reads_more_than_skipper():
    # the contrast of Section II-C: several full passes against one early-exit pass
    g = graphgen.rmat(18, seed=3)
    off, nbr = to_dev(g)
    h = mm.Graph(off, nbr, symmetric=True, stats=True)
    out = h.run()
    h.sync()
    skipper = h.stats()
    _, st = h.ems(seed=5)
    assert oracle.check(g, out.cpu().numpy()).ok
    assert st["iterations"] >= 2
    assert st["touched"] > 2 * (skipper["touched"] + skipper["assist_reads"])
