"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every comparison is exact: thresholds, RRR sets (canonical sorted CSR),
sampling counters, covering subsets (as sets), seeds, gains, coverage,
partitions, local solutions, streamed solutions and IMM sample counts.
Both sides run on the same seeded synthetic inputs; neither sees the other's
outputs.
"""
import threading

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def im():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2408_10982_amd as im
    im.lib()
    return im


def _say(*a):
    print("[case]", *a, flush=True)


def _prep(im, g):
    return im.prepare_graph(g.in_off, g.in_src, g.weight, g.model)


def _oracle_thr(g):
    return O.thresholds(g.model, g.in_off, g.weight)


def _np(t):
    return t.detach().cpu().numpy()


GRAPHS = {
    "ic_sparse": lambda: W.random_small_graph(500, 2000, seed=1, p_hi=0.1),
    "ic_dense": lambda: W.random_small_graph(300, 3000, seed=2, p_hi=0.5),
    "ic_p1": lambda: W.tiny_graph(400, [(int(a), int(b)) for a, b in
                                        np.random.default_rng(3).integers(0, 400, (1600, 2))],
                                  np.ones(1600, np.float32)),
    "lt_small": lambda: W.random_small_graph(500, 2500, seed=4, model=W.LT),
    "lt_chain": lambda: W.tiny_graph(3000, [(v, v + 1) for v in range(2999)],
                                     np.ones(2999, np.float32), model=W.LT),
    "rmat12": lambda: W.config(1).graph,
    "rmat14_wc": lambda: W.make_graph("rmat", W.IC, scale=14, num_edges=1 << 18, graph_seed=77,
                                      weight_seed=78, weights="wc"),
}


@pytest.mark.parametrize("name", list(GRAPHS))
def test_thresholds(im, name):
    _say("thresholds", name)
    g = GRAPHS[name]()
    G = _prep(im, g)
    got = _np(G.thr).view(np.uint32)[:g.num_edges]
    assert np.array_equal(got, _oracle_thr(g))
    assert np.all(_np(G.thr)[g.num_edges:] == 0)
    if g.model == W.IC:  # run-length table, bit for bit (exercises the log)
        sk = O.ic_skip_table(g.in_off, _oracle_thr(g))
        assert np.array_equal(_np(G.skip).view(np.uint64), sk.view(np.uint64))


@pytest.mark.parametrize("name,first,count", [
    ("ic_sparse", 0, 3000), ("ic_dense", 17, 2001), ("ic_p1", 5, 700), ("lt_small", 0, 4000),
    ("lt_chain", 3, 600), ("rmat12", 0, 16384), ("rmat12", 100000, 999),
    ("ic_p1", 0, 70000), ("rmat14_wc", 0, 20000), ("rmat14_wc", 12345, 3000)])
def test_sample_rrr(im, name, first, count):
    _say("sample", name, first, count)
    g = GRAPHS[name]()
    G = _prep(im, g)
    r = im.sample_rrr(G, seed=3001, stream_tag=0, first=first, count=count)
    o = O.sample(g.model, g.in_off, g.in_src, _oracle_thr(g), 3001, 0, first, count)
    assert np.array_equal(_np(r.off), o.off)
    assert np.array_equal(_np(r.mem), o.mem)
    assert (r.examined, r.live) == (o.examined, o.live)


@pytest.mark.parametrize("n,shape", [(49152, 1), (49153, 1), (98304, 2), (98305, 2)])
def test_sample_large_sets_bitmap_tiers(im, n, shape):
    """Supercritical IC sets (up to ~30 % of the graph) grown by the large-set
    launch in each shape (1: one wavefront per set, 2: 256 threads) on both
    sides of the largest graph whose bitmap fits the LDS pool (49,152 and
    98,304 vertices): LDS bitmap below, HBM bitmap with its read-before-atomic
    above; every set equals the oracle's."""
    _say("sample bitmap tiers", n, shape)
    g = W.random_small_graph(n, 4 * n, seed=11, p_hi=0.6)
    G = _prep(im, g)
    im.tune_set(im.TUNE_BIG_SHAPE, shape)
    try:
        r = im.sample_rrr(G, seed=4242, stream_tag=0, first=0, count=200)
    finally:
        im.tune_set(im.TUNE_BIG_SHAPE, -1)
    o = O.sample(g.model, g.in_off, g.in_src, _oracle_thr(g), 4242, 0, 0, 200)
    assert int(np.diff(o.off).max()) > 4096  # the sets do leave the LDS hash tier
    assert np.array_equal(_np(r.off), o.off)
    assert np.array_equal(_np(r.mem), o.mem)
    assert (r.examined, r.live) == (o.examined, o.live)


def test_lt_index_hub_degrees(im):
    """LT kept edges through the search index (a 16-ary descent over up to
    five levels here) equal binary search's and the oracle's at every
    in-degree: a 70,000-edge hub every walk can step to, and 2,000 vertices of
    in-degree 1..600 whose edge ranges straddle 16-, 256- and 4096-edge
    boundaries at every alignment; weights sum to 0.9 per vertex, so some
    vertices keep no edge."""
    _say("lt index hub degrees")
    rng = np.random.default_rng(21)
    n = 70001
    src = [np.arange(1, n), np.zeros(n - 1, np.int64)]
    dst = [np.zeros(n - 1, np.int64), np.arange(1, n)]
    for v in range(1, 2001):
        d = int(rng.integers(1, 601))
        src.append(rng.integers(0, n, d))
        dst.append(np.full(d, v))
    edges = np.stack([np.concatenate(src), np.concatenate(dst)], axis=1)
    g = W.tiny_graph(n, edges, np.ones(edges.shape[0], np.float32), model=W.LT)
    g.weight = (W.lt_normalized_weights(g.in_off, 22) * np.float32(0.9)).astype(np.float32)
    assert int(np.diff(g.in_off).max()) == 70000
    Gi = im.prepare_graph(g.in_off, g.in_src, g.weight, g.model)
    Gb = im.prepare_graph(g.in_off, g.in_src, g.weight, g.model, lt_index=False)
    assert Gi.lt_index is not None and Gb.lt_index is None
    assert Gi.lt_index.numel() == im.lt_index_size(g.num_edges)
    o = O.sample(g.model, g.in_off, g.in_src, _oracle_thr(g), 5150, 0, 0, 6000)
    for G in (Gi, Gb):
        r = im.sample_rrr(G, seed=5150, stream_tag=0, first=0, count=6000)
        assert np.array_equal(_np(r.off), o.off)
        assert np.array_equal(_np(r.mem), o.mem)
        assert (r.examined, r.live) == (o.examined, o.live)
    # most walks pass through the hub
    assert int((o.mem == 0).sum()) > 3000


def test_sample_edge_cases(im):
    _say("sample edge cases")
    g = GRAPHS["ic_sparse"]()
    G = _prep(im, g)
    r = im.sample_rrr(G, 1, 0, 0, 0)
    assert r.total == 0 and _np(r.off).tolist() == [0]
    # capacity too small: IM_ERANGE first, identical result after the retry
    r1 = im.sample_rrr(G, 7, 2, 0, 500, capacity=10)
    o = O.sample(g.model, g.in_off, g.in_src, _oracle_thr(g), 7, 2, 0, 500)
    assert np.array_equal(_np(r1.mem), o.mem)
    # an isolated vertex graph: every set is its root
    iso = W.tiny_graph(64, [], np.zeros(0, np.float32))
    Gi = _prep(im, iso)
    ri = im.sample_rrr(Gi, 5, 0, 0, 300)
    oi = O.sample(O.IC, iso.in_off, iso.in_src, np.zeros(0, np.uint32), 5, 0, 0, 300)
    assert np.array_equal(_np(ri.mem), oi.mem)


def test_invalid_arguments(im):
    _say("invalid arguments")
    g = GRAPHS["ic_sparse"]()
    bad = g.weight.copy()
    bad[3] = np.nan
    with pytest.raises(im.ImError):
        im.prepare_graph(g.in_off, g.in_src, bad, W.IC)
    bad2 = g.weight.copy()
    bad2[0] = 1.5
    with pytest.raises(im.ImError):
        im.prepare_graph(g.in_off, g.in_src, bad2, W.IC)
    off = g.in_off.copy()
    off[-1] += 1
    with pytest.raises(im.ImError):
        im.prepare_graph(off, g.in_src, g.weight, W.IC)


def _incidence_sets(inc_off, inc_mem):
    io = np.asarray(inc_off)
    im_ = np.asarray(inc_mem).copy()
    for v in range(io.shape[0] - 1):
        im_[io[v]:io[v + 1]].sort()
    return io, im_


@pytest.mark.parametrize("name,count", [("ic_dense", 3000), ("lt_small", 5000), ("rmat12", 16384)])
def test_incidence(im, name, count):
    _say("incidence", name, count)
    g = GRAPHS[name]()
    G = _prep(im, g)
    r = im.sample_rrr(G, 11, 0, 0, count)
    io, imem = im.build_incidence(g.n, r)
    o = O.sample(g.model, g.in_off, g.in_src, _oracle_thr(g), 11, 0, 0, count)
    oio, oim = O.incidence(g.n, o)
    gio, gim = _incidence_sets(_np(io), _np(imem))
    assert np.array_equal(gio, oio)
    assert np.array_equal(gim, oim)


def _segments_sorted(inc_off, inc_mem):
    """Each S(v) sorted (the order inside a covering subset is unspecified)."""
    io = np.asarray(inc_off)
    seg = np.repeat(np.arange(io.shape[0] - 1), np.diff(io))
    im_ = np.asarray(inc_mem)
    return io, im_[np.lexsort((im_, seg))]


def _incidence_form(form, monkeypatch):
    """"dense": one device atomic per member and pass; "tiled": LDS tiles of
    vertex ids (ranges of at most 4 x 32768 ids, else the atomic form);
    "tiled_slices": the same with slices of 997 members, so that items split
    sets and many slices hold no set start."""
    if form != "auto":
        monkeypatch.setenv("IM_INCIDENCE_DENSE_RATIO", "0")
    if form == "dense":
        monkeypatch.setenv("IM_INCIDENCE_DENSE_TILES", "0")
    if form == "tiled_slices":
        monkeypatch.setenv("IM_INCIDENCE_TILE_MEMBERS", "997")


@pytest.mark.parametrize("form", ["auto", "dense", "tiled", "tiled_slices"])
@pytest.mark.parametrize("n,count,max_size,seed", [
    (5000, 4000, 40, 1),                 # one bucket of vertex ids, ragged tail
    (4096 * 4096 + 4099, 3000, 300, 2),  # ids wider than 4096 buckets of 2^12
    (70000, 1, 60000, 3),                # a single set spanning many chunks
    (100000, 1500, 3000, 4),             # four LDS tiles of vertex ids, the last ragged
])
def test_incidence_synthetic(im, n, count, max_size, seed, form, monkeypatch):
    """Covering subsets of synthetic collections (distinct ids per set, sizes
    from 0 up), against the oracle's transpose, in each dense form (see
    _incidence_form) and the automatic choice."""
    _say("incidence synthetic", n, count, max_size, form)
    _incidence_form(form, monkeypatch)
    rng = np.random.default_rng(seed)
    sizes = rng.integers(0, max_size + 1, size=count)
    sizes[0] = max_size
    off = np.zeros(count + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    mem = np.concatenate([np.sort(rng.choice(n, size=int(z), replace=False)) for z in sizes]
                         ).astype(np.int32)
    o = O.RRR(off=off, mem=mem, examined=0, live=0)
    oio, oim = O.incidence(n, o)
    dmem = torch.from_numpy(mem).cuda()
    if seed == 1:  # members at an address that is not 16-byte aligned
        dmem = torch.cat([torch.zeros(1, dtype=torch.int32, device="cuda"), dmem])[1:]
        assert dmem.data_ptr() % 16 == 4
    r = im.RRR(off=torch.from_numpy(off).cuda(), mem=dmem,
               total=int(off[-1]), examined=0, live=0, large_sets=0)
    io, imem = im.build_incidence(n, r)
    gio, gim = _segments_sorted(_np(io), _np(imem))
    assert np.array_equal(gio, oio)
    assert np.array_equal(gim, oim)


@pytest.mark.parametrize("budget", ["1", "2000", "50000"])
def test_incidence_rounds(im, budget, monkeypatch):
    """The transpose in rounds of buckets (pair budget forced small; budget 1
    gives every bucket a round of its own, larger than the budget)."""
    _say("incidence rounds", budget)
    monkeypatch.setenv("IM_INCIDENCE_PAIR_BUDGET", budget)
    n, count = 3 * 4096 + 77, 2500
    rng = np.random.default_rng(9)
    sizes = rng.integers(0, 120, size=count)
    off = np.zeros(count + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    mem = np.concatenate([np.sort(rng.choice(n, size=int(z), replace=False)) for z in sizes]
                         ).astype(np.int32)
    oio, oim = O.incidence(n, O.RRR(off=off, mem=mem, examined=0, live=0))
    r = im.RRR(off=torch.from_numpy(off).cuda(), mem=torch.from_numpy(mem).cuda(),
               total=int(off[-1]), examined=0, live=0, large_sets=0)
    io, imem = im.build_incidence(n, r)
    gio, gim = _segments_sorted(_np(io), _np(imem))
    assert np.array_equal(gio, oio)
    assert np.array_equal(gim, oim)


def _pipeline(im, g, count, seed):
    G = _prep(im, g)
    r = im.sample_rrr(G, seed, 0, 0, count)
    io, imem = im.build_incidence(g.n, r)
    o = O.sample(g.model, g.in_off, g.in_src, _oracle_thr(g), seed, 0, 0, count)
    oio, oim = O.incidence(g.n, o)
    return G, r, io, imem, o, oio, oim


@pytest.mark.parametrize("name,count,k", [("ic_sparse", 3000, 10), ("ic_dense", 2000, 25),
                                          ("lt_small", 6000, 40), ("rmat12", 16384, 16),
                                          ("ic_p1", 500, 8), ("rmat14_wc", 20000, 30)])
def test_greedy(im, name, count, k):
    _say("greedy", name, count, k)
    g = GRAPHS[name]()
    G, r, io, imem, o, oio, oim = _pipeline(im, g, count, 21)
    seeds, gains, nsel, cov = im.greedy_cover(g.n, r, io, imem, k)
    os_, og, oc = O.greedy(g.n, count, oio, oim, k)
    ns = int(_np(nsel)[0])
    assert ns == len(os_)
    assert np.array_equal(_np(seeds)[:ns], os_)
    assert np.array_equal(_np(gains)[:ns], og)
    assert np.all(_np(seeds)[ns:] == -1)
    assert int(_np(cov)[0]) == oc


def test_cover_graph_replays_match_eager(im):
    """The captured cover (IM_TUNE_GRAPH = 1) replayed several times, with
    eager work and synchronisations between the replays and two collections
    alternating (the cached executable is updated with new arguments), gives
    the seeds, gains and coverage of the launches issued one by one -- for
    the standard greedy, the RandGreedi local step and the offline step."""
    _say("graph replays")
    ga, gb = GRAPHS["rmat14_wc"](), GRAPHS["lt_small"]()
    Ga, ra, ioa, ima, *_ = _pipeline(im, ga, 20000, 51)
    Gb, rb, iob, imb, *_ = _pipeline(im, gb, 6000, 52)

    def run_all():
        out = [tuple(_np(x).tolist() for x in im.greedy_cover(ga.n, ra, ioa, ima, 30)),
               tuple(_np(x).tolist() for x in im.greedy_cover(gb.n, rb, iob, imb, 20))]
        part, ls, lg, lc, lv = im.randgreedi(gb.n, rb, iob, imb, 12, 8, part_seed=5)
        out.append(tuple(_np(x).tolist() for x in (ls, lg, lc, lv)))
        fo = im.greedi_offline(gb.n, rb, iob, imb, ls, lc, lv, 12, 1.0)
        out.append(tuple(_np(x).tolist() for x in fo))
        return out

    try:
        im.tune_set(im.TUNE_GRAPH, 0)
        ref = run_all()
        im.tune_set(im.TUNE_GRAPH, 1)
        for rep in range(4):
            got = run_all()
            assert got == ref, rep
            torch.cuda.synchronize()
            im.sample_rrr(Ga, 77 + rep, 0, 0, 500)  # eager work between replays
            torch.cuda.synchronize()
    finally:
        im.tune_set(im.TUNE_GRAPH, -1)


@pytest.mark.parametrize("name,count,k,m", [("ic_dense", 2000, 10, 4), ("lt_small", 6000, 20, 8),
                                            ("rmat12", 16384, 16, 64), ("ic_sparse", 3000, 5, 1)])
def test_randgreedi(im, name, count, k, m):
    _say("randgreedi", name, count, k, m)
    g = GRAPHS[name]()
    G, r, io, imem, o, oio, oim = _pipeline(im, g, count, 31)
    part, ls, lg, lc, lv = im.randgreedi(g.n, r, io, imem, k, m, part_seed=4003)
    opart = O.partition(g.n, m, 4003)
    assert np.array_equal(_np(part), opart)
    ols, olg, olc, olv = O.local_greedy(g.n, count, oio, oim, opart, m, k)
    assert np.array_equal(_np(lc), olc)
    assert np.array_equal(_np(lv), olv)
    assert np.array_equal(_np(ls), ols)
    assert np.array_equal(_np(lg), olg)


@pytest.mark.parametrize("name,count,k,m", [("rmat14_wc", 20000, 300, 2), ("rmat12", 300, 400, 3)])
def test_randgreedi_candidate_lists(im, name, count, k, m):
    """Partitions far larger than a candidate list (1024 positions), picks
    deep enough that the lists are rebuilt many times and counts tie at small
    values, and (rmat12, k = 400) partitions whose counts all reach 0: the
    picks equal the oracle's, with the lists and with the full argmax pass."""
    _say("randgreedi lists", name, count, k, m)
    g = GRAPHS[name]()
    G, r, io, imem, o, oio, oim = _pipeline(im, g, count, 61)
    opart = O.partition(g.n, m, 5003)
    ols, olg, olc, olv = O.local_greedy(g.n, count, oio, oim, opart, m, k)
    try:
        for lists in (1, 0):
            im.tune_set(im.TUNE_LISTS, lists)
            part, ls, lg, lc, lv = im.randgreedi(g.n, r, io, imem, k, m, part_seed=5003)
            assert np.array_equal(_np(part), opart)
            assert np.array_equal(_np(lc), olc), lists
            assert np.array_equal(_np(lv), olv), lists
            assert np.array_equal(_np(ls), ols), lists
            assert np.array_equal(_np(lg), olg), lists
    finally:
        im.tune_set(im.TUNE_LISTS, -1)
    if name == "rmat12":
        assert (olc < k).all()  # every partition ran out of gain


@pytest.mark.parametrize("name,count,k,m,delta,alpha", [
    ("ic_dense", 2000, 10, 4, 0.077, 1.0), ("lt_small", 6000, 20, 8, 0.1, 0.25),
    ("rmat12", 16384, 16, 64, 0.077, 1.0), ("rmat12", 16384, 16, 64, 0.077, 0.125),
    ("ic_sparse", 3000, 1, 3, 0.2, 1.0)])
def test_stream_cover(im, name, count, k, m, delta, alpha):
    _say("stream", name, count, k, m, delta, alpha)
    g = GRAPHS[name]()
    G, r, io, imem, o, oio, oim = _pipeline(im, g, count, 41)
    part, ls, lg, lc, lv = im.randgreedi(g.n, r, io, imem, k, m, part_seed=77)
    seeds, nsel, cov, info = im.stream_cover(g.n, count, io, imem, ls, lc, lv, k, delta, alpha)
    opart = O.partition(g.n, m, 77)
    ols, olg, olc, olv = O.local_greedy(g.n, count, oio, oim, opart, m, k)
    gs, gc, gb, gnb = O.stream_cover(g.n, count, oio, oim, ols, olg, olc, k, delta, alpha)
    fs, fc, won = O.final_select(ols, olc, olv, gs, gc)
    ns = int(_np(nsel)[0])
    inf = _np(info)
    assert (inf[0], inf[1], inf[2]) == (gb, gnb, int(won))
    assert ns == len(fs) and np.array_equal(_np(seeds)[:ns], fs)
    assert int(_np(cov)[0]) == fc


def test_stream_cover_long_stream_with_gaps(im):
    """A stream longer than one 1024-entry lookup chunk (m * T = 1280, the
    last chunk partial) where most partitions pick fewer than T seeds (few
    candidates each), so the stream has holes."""
    _say("stream long", 80, 16)
    g = GRAPHS["ic_sparse"]()
    count, k, m = 300, 16, 80
    G, r, io, imem, o, oio, oim = _pipeline(im, g, count, 43)
    part, ls, lg, lc, lv = im.randgreedi(g.n, r, io, imem, k, m, part_seed=91)
    lc_h = _np(lc)
    assert m * k > 1024 and lc_h.min() < k  # shape of the case itself
    seeds, nsel, cov, info = im.stream_cover(g.n, count, io, imem, ls, lc, lv, k, 0.077, 1.0)
    opart = O.partition(g.n, m, 91)
    ols, olg, olc, olv = O.local_greedy(g.n, count, oio, oim, opart, m, k)
    assert np.array_equal(lc_h, olc)
    gs, gc, gb, gnb = O.stream_cover(g.n, count, oio, oim, ols, olg, olc, k, 0.077, 1.0)
    fs, fc, won = O.final_select(ols, olc, olv, gs, gc)
    ns = int(_np(nsel)[0])
    inf = _np(info)
    assert (inf[0], inf[1], inf[2], inf[3]) == (gb, gnb, int(won), int(olc.sum()))
    assert ns == len(fs) and np.array_equal(_np(seeds)[:ns], fs)
    assert int(_np(cov)[0]) == fc


def test_stream_cover_all_streamed_sets_empty(im):
    """Every streamed S(x) empty (l = 0): no bucket takes a seed, the result
    is empty with coverage 0, as in the oracle."""
    _say("stream empty")
    n, count, k, m = 12, 5, 3, 2
    inc_off = np.zeros(n + 1, np.int64)
    inc_mem = np.zeros(0, np.int32)
    ls = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    lc = np.array([3, 2], np.int32)
    lg = np.zeros((m, k), np.int64)
    lv = np.zeros(m, np.int64)
    dev = "cuda"
    seeds, nsel, cov, info = im.stream_cover(
        n, count, torch.from_numpy(inc_off).to(dev), torch.zeros(1, dtype=torch.int32,
                                                                device=dev),
        torch.from_numpy(ls).to(dev), torch.from_numpy(lc).to(dev),
        torch.from_numpy(lv).to(dev), k, 0.077, 1.0)
    gs, gc, gb, gnb = O.stream_cover(n, count, inc_off, inc_mem, ls, lg, lc, k, 0.077, 1.0)
    fs, fc, won = O.final_select(ls, lc, lv, gs, gc)
    assert len(fs) == 0 and fc == 0
    assert int(_np(nsel)[0]) == 0 and int(_np(cov)[0]) == 0
    assert np.all(_np(seeds) == -1)
    inf = _np(info)
    assert (inf[0], inf[1], inf[2], inf[3]) == (gb, gnb, int(won), 5)


@pytest.mark.parametrize("name,count,k,m,alpha", [
    ("ic_dense", 2000, 10, 4, 1.0), ("lt_small", 6000, 20, 8, 1.0), ("rmat12", 16384, 16, 64, 1.0),
    ("rmat12", 16384, 16, 64, 0.25), ("ic_sparse", 300, 16, 80, 1.0), ("ic_sparse", 3000, 1, 3, 1.0)])
def test_greedi_offline(im, name, count, k, m, alpha):
    """Alg. 4's offline global step: the GPU's S_g, its coverage, the final
    choice and the gathered count against the oracle's lazy greedy over the
    union of the local solutions."""
    _say("offline", name, count, k, m, alpha)
    g = GRAPHS[name]()
    G, r, io, imem, o, oio, oim = _pipeline(im, g, count, 47)
    part, ls, lg, lc, lv = im.randgreedi(g.n, r, io, imem, k, m, part_seed=55)
    seeds, nsel, cov, info, gcov = im.greedi_offline(g.n, r, io, imem, ls, lc, lv, k, alpha)
    opart = O.partition(g.n, m, 55)
    ols, olg, olc, olv = O.local_greedy(g.n, count, oio, oim, opart, m, k)
    assert np.array_equal(_np(lc), olc) and np.array_equal(_np(ls), ols)
    gs, gg, gc = O.greedi_offline(g.n, count, oio, oim, ols, olc, k, alpha=alpha)
    fs, fc, won = O.final_select(ols, olc, olv, gs, gc)
    ns = int(_np(nsel)[0])
    inf = _np(info)
    T = O.trunc_len(k, alpha)
    assert int(_np(gcov)[0]) == gc
    assert (inf[0], inf[1], inf[2]) == (int(won), int(np.minimum(olc, T).sum()), len(gs))
    assert ns == len(fs) and np.array_equal(_np(seeds)[:ns], fs)
    assert np.all(_np(seeds)[ns:] == -1)
    assert int(_np(cov)[0]) == fc


@pytest.mark.parametrize("name,seeds,nsims", [
    ("ic_sparse", [1, 2, 3], 64), ("ic_dense", [0, 50, 100, 150], 64), ("ic_p1", [7], 8),
    ("lt_small", [4, 9, 400], 64), ("lt_chain", [0], 4), ("rmat12", list(range(0, 4096, 256)), 40),
    ("rmat14_wc", [5, 99, 1000, 8000], 24), ("ic_sparse", [], 3), ("lt_small", [3, 3, 3], 17)])
def test_influence(im, name, seeds, nsims):
    """Forward simulations: every simulation's activated count equals the
    oracle's (same live-edge world, keyed by simulation id), across more than
    one batch of simulations and with duplicate or no seeds."""
    _say("influence", name, len(seeds), nsims)
    g = GRAPHS[name]()
    G = _prep(im, g)
    F = im.prepare_forward(G)
    got = _np(im.influence(G, F, 61, 2, 5, nsims, seeds))
    exp = O.influence(g.model, g.in_off, g.in_src, _oracle_thr(g), 61, 2, 5, nsims, seeds)
    assert np.array_equal(got, exp), (got[:8], exp[:8])
    # the out-edge view is a regrouping of the in-edges
    oe = np.sort(_np(F.out_eid)[:g.num_edges])
    assert np.array_equal(oe, np.arange(g.num_edges))
    assert np.array_equal(_np(F.edge_dst)[:g.num_edges], np.repeat(np.arange(g.n), np.diff(g.in_off)))


@pytest.mark.parametrize("name,k,eps,selector", [
    ("ic_sparse", 5, 0.5, O.SEL_GREEDY), ("lt_small", 8, 0.4, O.SEL_GREEDIRIS),
    ("rmat12", 16, 0.5, O.SEL_GREEDY), ("rmat12", 16, 0.5, O.SEL_GREEDIRIS),
    ("lt_small", 8, 0.4, O.SEL_RANDGREEDI), ("rmat12", 16, 0.5, O.SEL_RANDGREEDI)])
def test_solve_imm(im, name, k, eps, selector):
    _say("imm", name, k, eps, selector)
    g = GRAPHS[name]()
    G = _prep(im, g)
    kw = dict(selector=selector, m=8, delta=0.077, alpha=0.5, seed=3003, part_seed=4003)
    got = im.solve(G, k, eps, **kw)
    exp = O.imm(g.model, g.in_off, g.in_src, _oracle_thr(g), k, eps, **kw)
    assert got["theta"] == exp["theta"]
    assert got["rounds"] == exp["rounds_run"]
    assert got["martingale_samples"] == exp["martingale_samples"]
    assert got["lower_bound"] == exp["lb"]
    assert got["seeds"] == exp["seeds"].tolist()
    assert got["coverage"] == exp["coverage"]
    assert got["global_won"] == exp["global_won"] and got["bucket"] == exp["bucket"]
    assert got["stream_len"] == exp["stream_len"]


def _ptr(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


def test_workspace_minimum_and_short(im):
    """Through the C ABI with caller workspaces: one byte under the size
    im_workspace_size reports is rejected (IM_ENOMEM, nothing written), the
    reported minimum (one large-set worker, 2^24-pair incidence rounds)
    gives the oracle's sets and covering subsets, and an im_solve given a
    workspace far too small is rejected or runs short, reports what it
    needs, and with that much (grown as the binding grows it) returns the
    oracle's seeds."""
    import ctypes as C
    from paper_2408_10982_amd import binding as B
    L = B.lib()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    g = W.random_small_graph(49153, 4 * 49153, seed=11, p_hi=0.6)  # large IC sets
    G = _prep(im, g)
    gs = G.struct()
    count = 300
    o = O.sample(g.model, g.in_off, g.in_src, _oracle_thr(g), 4242, 0, 0, count)
    cap = int(o.off[-1])
    need = im.workspace_size(im.WS_SAMPLE, n=g.n, model=g.model, count=count, total=cap)
    _say("workspace sample", need)
    off = torch.full((count + 1,), -7, dtype=torch.int64, device="cuda")
    mem = torch.empty(cap, dtype=torch.int32, device="cuda")
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    total = C.c_int64(-1)
    rc = L.im_sample_rrr(C.byref(gs), 4242, 0, 0, count, _ptr(off), _ptr(mem), cap,
                         C.byref(total), None, _ptr(ws), need - 1, s)
    assert rc == B.IM_ENOMEM and total.value == -1
    assert B.workspace_need()[0] == need
    torch.cuda.synchronize()
    assert bool((off == -7).all())  # rejected before any device work
    rc = L.im_sample_rrr(C.byref(gs), 4242, 0, 0, count, _ptr(off), _ptr(mem), cap,
                         C.byref(total), None, _ptr(ws), need, s)
    assert rc == B.IM_OK and total.value == cap
    assert np.array_equal(_np(off), o.off) and np.array_equal(_np(mem), o.mem)
    # the large sets asked for more workers than the minimum holds
    assert B.workspace_need()[1] > need
    # covering subsets at their minimum workspace
    n = g.n
    need = im.workspace_size(im.WS_INCIDENCE, n=n, total=cap)
    _say("workspace incidence", need)
    inc_off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    inc_mem = torch.empty(cap, dtype=torch.int32, device="cuda")
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rc = L.im_build_incidence(n, count, _ptr(off), _ptr(mem), cap, _ptr(inc_off),
                              _ptr(inc_mem), _ptr(ws), need, s)
    assert rc == B.IM_OK
    io, imem = O.incidence(n, o)
    assert np.array_equal(_np(inc_off), io)
    got, exp = _np(inc_mem), imem
    for v in range(0, n, 97):
        a, b = io[v], io[v + 1]
        assert sorted(got[a:b]) == sorted(exp[a:b])
    # IMM: a 1 MiB workspace is short; grow by the reported need
    h = GRAPHS["lt_small"]()
    H = _prep(im, h)
    hs = H.struct()
    kw = dict(selector=O.SEL_GREEDIRIS, m=8, delta=0.077, alpha=0.5, seed=3003, part_seed=4003)
    exp = O.imm(h.model, h.in_off, h.in_src, _oracle_thr(h), 8, 0.4, **kw)
    opts = B._SolveOpts(kw["selector"], kw["m"], kw["delta"], kw["alpha"], kw["seed"],
                        kw["part_seed"], 0)
    res = B._SolveResult()
    seeds = (C.c_int32 * 8)()
    size, tries = 1 << 20, 0
    while True:
        ws = torch.empty(size, dtype=torch.uint8, device="cuda")
        rc = L.im_solve(C.byref(hs), 8, 0.4, C.byref(opts), seeds, C.byref(res), _ptr(ws), size,
                        s)
        tries += 1
        _say("workspace solve", size, rc)
        if rc != B.IM_ENOMEM:
            break
        nd = B.workspace_need()[0]
        assert nd > size and tries < 8
        size = nd + nd // 4
    assert rc == B.IM_OK and tries >= 2
    assert list(seeds)[:res.nsel] == exp["seeds"].tolist()
    assert res.coverage == exp["coverage"] and res.theta == exp["theta"]


def test_batch_workspace_grows_once(im):
    """A batched call through the C ABI, started with a 1 MiB workspace and
    grown to what im_workspace_need reports after each IM_ENOMEM: the first
    report is the call's minimum, and once sampling knows the member total
    the next one is the size of the whole call, so at most two growths are
    needed; the seeds, gains and coverage equal the oracle's per task."""
    import ctypes as C
    from paper_2408_10982_amd import binding as B
    L = B.lib()
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    specs = [(W.random_small_graph(3000, 12000, seed=21, p_hi=0.5), 901, 12, 1500),
             (GRAPHS["lt_small"](), 902, 20, 3000),
             (W.random_small_graph(5000, 15000, seed=22, p_hi=0.3), 903, 8, 2500),
             (GRAPHS["ic_dense"](), 904, 10, 1200)]
    _say("batch workspace growth", len(specs))
    preps = [_prep(im, g) for g, *_ in specs]
    nt = len(specs)
    arr = (B._Task * nt)()
    for j, ((g, seed, k, theta), G) in enumerate(zip(specs, preps)):
        arr[j] = B._Task(G.struct(), seed, 0, k, theta)
    K = sum(k for _, _, k, _ in specs)
    seeds = torch.empty(K, dtype=torch.int32, device="cuda")
    gains = torch.empty(K, dtype=torch.int64, device="cuda")
    nsel = torch.empty(nt, dtype=torch.int32, device="cuda")
    cov = torch.empty(nt, dtype=torch.int64, device="cuda")
    st = B._BatchStats()
    out = {}

    def calls():  # a fresh thread: no member total remembered from earlier batches
        try:
            ws_bytes, grown, rc = 1 << 20, [], None
            for _ in range(4):
                ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
                rc = L.im_solve_batch(arr, nt, _ptr(seeds), _ptr(gains), _ptr(nsel), _ptr(cov),
                                      C.byref(st), _ptr(ws), ws_bytes, s)
                torch.cuda.synchronize()
                if rc != B.IM_ENOMEM:
                    break
                need = B.workspace_need()[0]
                grown.append((ws_bytes, need))
                if need <= ws_bytes:
                    break
                ws_bytes = need
                del ws
            out["rc"], out["grown"] = rc, grown
        except BaseException as e:  # noqa: BLE001 -- re-raised below
            out["err"] = e

    th = threading.Thread(target=calls)
    th.start()
    th.join()
    if "err" in out:
        raise out["err"]
    assert out["rc"] == B.IM_OK and 1 <= len(out["grown"]) <= 2, out
    assert all(need > have for have, need in out["grown"]), out
    s_h, g_h, n_h, c_h = _np(seeds), _np(gains), _np(nsel), _np(cov)
    o = 0
    for j, (g, seed, k, theta) in enumerate(specs):
        r = O.sample(g.model, g.in_off, g.in_src, _oracle_thr(g), seed, 0, 0, theta)
        io, imem = O.incidence(g.n, r)
        es, eg, ec = O.greedy(g.n, theta, io, imem, k, lazy=True)
        n = int(n_h[j])
        assert n == len(es) and np.array_equal(s_h[o:o + n], es), j
        assert np.array_equal(g_h[o:o + n], np.asarray(eg)[:n]), j
        assert int(c_h[j]) == ec, j
        o += k


@pytest.mark.parametrize("name,k,eps,selector,cap", [
    ("ic_sparse", 5, 0.3, O.SEL_GREEDY, 1 << 20), ("lt_small", 8, 0.2, O.SEL_GREEDIRIS, 1 << 20),
    ("rmat12", 16, 0.1, O.SEL_GREEDY, 1 << 16), ("rmat12", 16, 0.1, O.SEL_GREEDIRIS, 1 << 16),
    ("rmat14_wc", 20, 0.2, O.SEL_RANDGREEDI, 1 << 18)])
def test_opim(im, name, k, eps, selector, cap):
    """OPIM rounds: the same halves, seeds, coverages on R1 and R2, upper
    bound, rounds and (bit for bit, the same fp64 operations) guarantee."""
    _say("opim", name, k, eps, selector, cap)
    g = GRAPHS[name]()
    G = _prep(im, g)
    kw = dict(selector=selector, m=8, delta=0.077, alpha=0.5, seed=3005, part_seed=4005)
    fail = 1.0 / g.n
    got = im.opim(G, k, eps, fail, cap, **kw)
    exp = O.opim(g.model, g.in_off, g.in_src, _oracle_thr(g), k, eps, fail=fail, theta_cap=cap,
                 **kw)
    for key in ("rounds", "theta", "cover1", "cover2", "upper1", "i_max", "nsel"):
        assert got[key] == exp[key], key
    for key in ("lower", "upper", "guarantee", "theta_max"):
        assert got[key] == exp[key], key
    assert got["seeds"] == exp["seeds"].tolist()


@pytest.mark.parametrize("form", ["auto", "dense", "tiled_slices"])
def test_batch_matches_single_calls_and_oracle(im, form, monkeypatch):
    """im_solve_batch: every task equals its own sample + incidence + greedy
    calls on the GPU and the oracle's standard greedy (mixed IC/LT, uneven
    n, k and theta, including sets large enough for the large-set path), with
    the covering subsets of the whole batch in each form."""
    _say("batch", form)
    _incidence_form(form, monkeypatch)
    specs = [("ic_sparse", 5, 0, 7, 3000), ("lt_small", 6, 1, 12, 4000), ("rmat12", 7, 0, 16, 5000),
             ("ic_dense", 8, 2, 3, 1500), ("lt_chain", 9, 0, 5, 700), ("ic_p1", 10, 0, 4, 400)]
    for j in range(4):
        t = W.batch_tasks(count=64, seed=77)[j * 13]
        g = W.make_graph("chunglu", t["model"], n=min(t["n"], 3000), avg_deg=t["avg_deg"],
                         graph_seed=t["graph_seed"], weight_seed=t["weight_seed"])
        GRAPHS["cl%d" % j] = (lambda gg=g: gg)
        specs.append(("cl%d" % j, 100 + j, 0, t["k"], 2000))
    graphs = {name: GRAPHS[name]() for name, *_ in specs}
    prepared = {name: _prep(im, g) for name, g in graphs.items()}
    tasks = [(prepared[name], seed, tag, k, theta) for name, seed, tag, k, theta in specs]
    out, stats = im.solve_batch(tasks)
    assert stats["sets"] == sum(t[4] for t in tasks)
    for (name, seed, tag, k, theta), res in zip(specs, out):
        g = graphs[name]
        G = prepared[name]
        r = im.sample_rrr(G, seed, tag, 0, theta)
        io, imem = im.build_incidence(g.n, r)
        s1, g1, n1, c1 = im.greedy_cover(g.n, r, io, imem, k)
        n1 = int(_np(n1)[0])
        assert res["seeds"] == _np(s1)[:n1].tolist(), name
        assert res["gains"] == _np(g1)[:n1].tolist(), name
        assert res["coverage"] == int(_np(c1)[0]), name
        o = O.sample(g.model, g.in_off, g.in_src, _oracle_thr(g), seed, tag, 0, theta)
        oio, oim = O.incidence(g.n, o)
        os_, og, oc = O.greedy(g.n, theta, oio, oim, k)
        assert res["seeds"] == os_.tolist() and res["coverage"] == oc, name


def test_serving_results_equal_alone(im):
    """Queries served together from shared, growing sample pools (3 slots on
    3 streams) return exactly what im_solve returns for each query alone;
    with a one-byte HBM budget admission serialises them, same results.  The
    second server runs on the first one's streams (and their workspaces)."""
    _say("serving")
    from paper_2408_10982_amd import serve as S
    gs = {"ic": W.random_small_graph(3000, 15000, seed=21, p_hi=0.2),
          "lt": W.random_small_graph(3000, 15000, seed=22, model=W.LT)}
    prepared = {k: _prep(im, g) for k, g in gs.items()}
    rng = np.random.default_rng(5)
    spec = [("ic" if j % 2 else "lt", int(rng.integers(3, 20)), float(rng.choice([0.5, 0.3])))
            for j in range(10)]
    alone = [im.solve(prepared[name], k, eps, seed=5005) for name, k, eps in spec]
    streams = [torch.cuda.Stream() for _ in range(3)]  # shared by both servers
    with pytest.raises(ValueError):
        S.Server(prepared, seed=5005, slots=3, streams=streams[:2])
    for budget, expect_overlap in ((1 << 40, True), (1, False)):
        server = S.Server(prepared, seed=5005, slots=3, hbm_budget=budget, streams=streams)
        qs = [S.Query(qid=j, graph=name, k=k, eps=eps, arrival=0.0)
              for j, (name, k, eps) in enumerate(spec)]
        done = S.run_arrivals(server, qs)
        server.close()
        assert (server.max_in_flight > 1) == expect_overlap
        for q, a in zip(done, alone):
            r = q.result
            assert r["seeds"] == a["seeds"] and r["coverage"] == a["coverage"], q.qid
            assert r["theta"] == a["theta"] and r["rounds"] == a["rounds"]
            assert r["lower_bound"] == a["lower_bound"]
            assert r["martingale_samples"] == a["martingale_samples"]


def test_serving_failed_query_raises(im, monkeypatch):
    """A query whose solve raises finishes with its error; the other queries
    still finish, and run_arrivals then raises instead of waiting forever."""
    _say("serving failure")
    from paper_2408_10982_amd import serve as S
    g = W.random_small_graph(2000, 9000, seed=23, p_hi=0.2)
    prepared = {"ic": _prep(im, g)}
    real = S.solve_pooled

    def flaky(graph, pools, k, eps, stream):
        if k == 7:
            raise RuntimeError("planted failure")
        return real(graph, pools, k, eps, stream)

    monkeypatch.setattr(S, "solve_pooled", flaky)
    server = S.Server(prepared, seed=5006, slots=2, hbm_budget=1 << 40)
    qs = [S.Query(qid=j, graph="ic", k=k, eps=0.5, arrival=0.0) for j, k in enumerate((5, 7, 9))]
    try:
        with pytest.raises(RuntimeError, match="1 of 3 queries failed; query 1"):
            S.run_arrivals(server, qs)
    finally:
        server.close()
    assert qs[1].error is not None and not qs[1].result
    assert qs[0].result["seeds"] and qs[2].result["seeds"]


def test_autotune_keeps_results(im):
    """Every launch-shape knob setting gives the same sets, seeds, gains and
    coverage (the tuner checks the signature at every trial; rmat14_wc hands
    sets to the large-set launch), and the tuned result equals the oracle's."""
    _say("autotune")
    from paper_2408_10982_amd import autotune as AT
    g = GRAPHS["rmat14_wc"]()
    G = _prep(im, g)
    count, k, seed = 20000, 30, 41

    def run():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        r = im.sample_rrr(G, seed, 0, 0, count)
        io, imem = im.build_incidence(g.n, r)
        s_, gn, ns, cv = im.greedy_cover(g.n, r, io, imem, k)
        e1.record()
        torch.cuda.synchronize()
        n = int(_np(ns)[0])
        sig = (_np(r.off).tobytes(), _np(r.mem).tobytes(), tuple(_np(s_)[:n].tolist()),
               tuple(_np(gn)[:n].tolist()), int(_np(cv)[0]))
        return e0.elapsed_time(e1), sig

    try:
        res = AT.tune(run, reps=1)
        _, sig = run()
    finally:
        AT.reset()
    assert set(res["settings"]) == set(AT.KNOBS)
    assert len(res["trials"]) == 1 + sum(len(c) - 1 for _, c in AT.KNOBS.values())
    assert AT.current() == {"sample_blocks": 5, "big_shape": 0, "apply_blocks": 1,
                            "dense_ratio": 256}
    o = O.sample(g.model, g.in_off, g.in_src, _oracle_thr(g), seed, 0, 0, count)
    oio, oim = O.incidence(g.n, o)
    os_, og, oc = O.greedy(g.n, count, oio, oim, k)
    assert sig[2] == tuple(os_.tolist()) and sig[3] == tuple(og.tolist()) and sig[4] == oc

