"""The product's device check (mm_check / mm_batch_check) against the oracle's
checker, on mate arrays built on the CPU: the oracle's own SGMM output and
seeded corruptions of it, one per violation class of Section II-B plus mixed
ones. Both checkers see the same array; their counts must be equal."""
import zlib

import numpy as np
import pytest

import graphgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2507_04420_amd as mm  # noqa: E402

FIELDS = [("out_of_range", "out_of_range"), ("self_mate", "self_mate"),
          ("asymmetric", "asymmetric"), ("not_edge", "not_an_edge"),
          ("uncovered", "uncovered"), ("matched", "matched_vertices")]


def corrupt(csr, mate, kind, rng, k=5):
    mt = mate.copy()
    n = csr.n
    matched = np.flatnonzero(mt >= 0)
    if kind == "none":
        return mt
    if kind == "range":
        idx = rng.choice(n, size=k, replace=False)
        mt[idx] = rng.choice([-7, n, n + 3, -2**31, 2**31 - 1], size=k)
    elif kind == "self":
        idx = rng.choice(n, size=k, replace=False)
        mt[idx] = idx
    elif kind == "asym":
        idx = rng.choice(matched, size=k, replace=False)
        mt[idx] = rng.integers(0, n, size=k)
    elif kind == "unmatch":  # drops pairs: exposes uncovered edges
        idx = rng.choice(matched, size=k, replace=False)
        mt[mt[idx]] = -1
        mt[idx] = -1
    elif kind == "nonedge":  # a symmetric pair between two unmatched non-adjacent vertices
        if np.count_nonzero(mt == -1) < 4 * k:  # near-perfect matchings: free some pairs first
            mt = corrupt(csr, mt, "unmatch", rng, k=4 * k)
        free = np.flatnonzero(mt == -1)
        done = 0
        for a in rng.permutation(free):
            b = int(rng.choice(free))
            lst = csr.nbr[csr.off[a]:csr.off[a + 1]]
            if a != b and mt[a] == -1 and mt[b] == -1 and b not in lst:
                mt[a], mt[b] = b, a
                done += 1
                if done == k:
                    break
    elif kind == "mixed":
        for sub in ("range", "self", "asym", "unmatch"):
            mt = corrupt(csr, mt, sub, rng, k=2)
    return mt


def compare(got, want):
    for g, w in FIELDS:
        assert got[g] == getattr(want, w), (g, got, want)
    assert got["ok"] == (want.violations == 0)


GRAPHS = {
    "er": lambda: graphgen.er(20000, 6, seed=11),
    "rmat14": lambda: graphgen.rmat(14, seed=3),
    "grid": lambda: graphgen.grid(97, 103),
}


@pytest.mark.parametrize("gname", sorted(GRAPHS))
@pytest.mark.parametrize("kind", ["none", "range", "self", "asym", "unmatch", "nonedge", "mixed"])
def test_check_matches_oracle(gname, kind):
    csr = GRAPHS[gname]()
    rng = np.random.default_rng(zlib.crc32((gname + kind).encode()))
    mate = corrupt(csr, oracle.sgmm(csr).mate, kind, rng)
    want = oracle.check(csr, mate)
    if kind != "none":
        assert want.violations > 0
    g = mm.Graph(torch.from_numpy(csr.off).cuda(), torch.from_numpy(csr.nbr).cuda(), symmetric=True)
    compare(g.check(torch.from_numpy(mate).cuda()), want)
    # int32 offsets go through the other instantiation
    c32 = csr.with_int32_offsets()
    g32 = mm.Graph(torch.from_numpy(c32.off).cuda(), torch.from_numpy(c32.nbr).cuda())
    compare(g32.check(torch.from_numpy(mate).cuda()), want)


def test_check_own_output():
    csr = graphgen.rmat(16, seed=4)
    g = mm.Graph(torch.from_numpy(csr.off).cuda(), torch.from_numpy(csr.nbr).cuda(), symmetric=True)
    out = g.run()
    r = g.check(out)
    assert r["ok"]
    compare(r, oracle.check(csr, out.cpu().numpy()))


@pytest.mark.parametrize("kind", ["none", "asym", "unmatch", "mixed"])
def test_batch_check_matches_oracle(kind):
    mix = graphgen.mixture(25, seed=9, nmin=30, nmax=3000)
    rng = np.random.default_rng(77)
    mates = []
    tot = None
    for gi in range(mix.num_graphs):
        sub = mix.member(gi)
        mt = corrupt(sub, oracle.sgmm(sub).mate, kind, rng, k=1) if gi % 3 == 0 else oracle.sgmm(sub).mate
        c = oracle.check(sub, mt)
        vals = np.array([getattr(c, w) for _, w in FIELDS])
        tot = vals if tot is None else tot + vals
        mates.append(mt)
    b = mm.Batch(torch.from_numpy(mix.off).cuda(), torch.from_numpy(mix.nbr).cuda(), mix.vtx_off,
                 symmetric=True)
    got = b.check(torch.from_numpy(np.concatenate(mates)).cuda())
    assert [got[g] for g, _ in FIELDS] == tot.tolist()
    assert got["ok"] == (kind == "none")


def test_check_rejects_bad_tensor():
    csr = graphgen.grid(4, 4)
    g = mm.Graph(torch.from_numpy(csr.off).cuda(), torch.from_numpy(csr.nbr).cuda())
    with pytest.raises(ValueError):
        g.check(torch.zeros(15, dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        g.check(torch.zeros(16, dtype=torch.int64, device="cuda"))


def test_probe_ceilings_are_plausible():
    # the measurement probe behind the bench's secondary roofs: positive rates
    # of a plausible size for random 4-byte accesses to 256 MiB
    import ctypes
    from paper_2507_04420_amd import _lib
    lib = _lib.load()
    r, a = ctypes.c_double(), ctypes.c_double()
    assert lib.mm_probe_ceilings(1 << 28, 1 << 24, None, ctypes.byref(r), ctypes.byref(a)) == 0
    assert 1e9 < r.value < 1e12 and 1e8 < a.value < 1e12, (r.value, a.value)
