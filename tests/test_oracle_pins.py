"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms, exact enumeration of live-edge worlds on
tiny graphs, brute-force optima, invariants the paper states, and the bounds
it proves.  A plausible slip in the oracle (a dropped term, a wrong index, an
off-by-one tie-break, a transposed edge) fails at least one of them.
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order
from scipy.special import gammaln

import oracle as O
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- random numbers
def test_philox_known_answers():
    """Philox4x32-10 against the Random123 known-answer vectors."""
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = O.philox4x32_10(r[0:4], r[4:6])
        assert [int(x) for x in out] == r[6:10]


def test_roots_uniform():
    """Roots are uniform over V (Sec. 2.1 step 1): chi-square over 2^16 draws."""
    n, N = 97, 1 << 16
    counts = np.bincount([O.root(7, 0, i, n) for i in range(N)], minlength=n)
    exp = N / n
    chi2 = ((counts - exp) ** 2 / exp).sum()
    # df = 96: mean 96, sd ~13.9; 96 + 6 sd
    assert chi2 < 96 + 6 * math.sqrt(2 * 96)
    assert O.root(7, 0, 123, 1) == 0
    # different streams and seeds give different root sequences
    a = [O.root(7, 0, i, 1 << 20) for i in range(64)]
    b = [O.root(7, 1, i, 1 << 20) for i in range(64)]
    c = [O.root(8, 0, i, 1 << 20) for i in range(64)]
    assert a != b and a != c


# ---------------------------------------------------------------- thresholds
def test_ic_thresholds_closed_form():
    p = np.array([0.0, 1.0, 0.5, 0.25, 0.75, 2.0 ** -24, np.nextafter(np.float32(1), 0)],
                 np.float32)
    q = O.ic_thresholds(p)
    assert list(q[:6]) == [0, 0xFFFFFFFF, 1 << 31, 1 << 30, 3 << 30, 1 << 8]
    assert q[6] == 2 ** 32 - 2 ** 8  # largest fp32 below 1 never reaches the sentinel
    for bad in ([np.nan], [-0.1], [1.5]):
        with pytest.raises(ValueError):
            O.ic_thresholds(np.array(bad, np.float32))


def test_lt_thresholds_closed_form():
    in_off = np.array([0, 3, 3, 4, 6], np.int32)
    w = np.array([0.25, 0.25, 0.5, 0.5, 1.0, 0.5], np.float32)
    c = O.lt_thresholds(in_off, w)
    # vertex 0: 2^30, 2^31, saturated; vertex 2: 2^31; vertex 3: saturated twice
    assert list(c) == [1 << 30, 1 << 31, 0xFFFFFFFF, 1 << 31, 0xFFFFFFFF, 0xFFFFFFFF]


# ---------------------------------------------------------------- IC sampling
def _rev_csr(g):
    """Transposed adjacency: row v lists the in-neighbours of v."""
    n = g.n
    deg = np.diff(g.in_off)
    rows = np.repeat(np.arange(n), deg)
    return sp.csr_matrix((np.ones(g.num_edges), (rows, g.in_src)), shape=(n, n))


def test_ic_p1_equals_reverse_reachability():
    """p = 1: every edge live, R(i) = {v : v reaches root_i} (Def. 2.3)."""
    g = W.random_small_graph(300, 700, seed=11)
    w = np.ones(g.num_edges, np.float32)
    thr = O.ic_thresholds(w)
    r = O.sample(O.IC, g.in_off, g.in_src, thr, seed=5, stream=0, first=0, count=200)
    A = _rev_csr(g)
    for i in range(200):
        root = O.root(5, 0, i, g.n)
        expect = np.sort(breadth_first_order(A, root, directed=True,
                                             return_predecessors=False))
        assert np.array_equal(r.set(i), expect)
    assert r.live == r.examined


def test_ic_p0_gives_singletons():
    g = W.random_small_graph(50, 400, seed=12)
    thr = O.ic_thresholds(np.zeros(g.num_edges, np.float32))
    r = O.sample(O.IC, g.in_off, g.in_src, thr, seed=9, stream=3, first=10, count=500)
    assert np.array_equal(np.diff(r.off), np.ones(500))
    assert [int(x) for x in r.mem] == [O.root(9, 3, 10 + i, g.n) for i in range(500)]
    assert r.live == 0


def _forward_reach(n, live_edges, s):
    adj = [[] for _ in range(n)]
    for u, v in live_edges:
        adj[u].append(v)
    seen = {s}
    stack = [s]
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                stack.append(y)
    return seen


def _exact_ic_activation(n, edges, probs):
    """P[v reaches t in the live-edge world], by enumerating all 2^|E| worlds."""
    P = np.zeros((n, n))
    m = len(edges)
    for mask in range(1 << m):
        pr = 1.0
        live = []
        for j in range(m):
            if mask >> j & 1:
                pr *= probs[j]
                live.append(edges[j])
            else:
                pr *= 1.0 - probs[j]
        for v in range(n):
            for t in _forward_reach(n, live, v):
                P[v, t] += pr
    return P


TINY_EDGES = [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (1, 4), (4, 5), (5, 3), (0, 5), (5, 1)]
TINY_P = [0.5, 0.3, 0.7, 0.4, 0.9, 0.2, 0.6, 0.5, 0.25, 0.8]


def test_ic_membership_matches_exact_enumeration():
    """Pr[v in R(i) | root_i = t] = Pr[v reaches t] over live-edge worlds, and
    n * Pr[R cap S nonempty] = sigma(S) (the RIS identity behind Sec. 2.1)."""
    n = 6
    g = W.tiny_graph(n, TINY_EDGES, TINY_P)
    thr = O.ic_thresholds(g.weight)
    # probabilities as the integer thresholds realise them
    q = O.ic_thresholds(np.array(TINY_P, np.float32)).astype(np.float64) / 2.0 ** 32
    P = _exact_ic_activation(n, TINY_EDGES, list(q))
    N = 120000
    r = O.sample(O.IC, g.in_off, g.in_src, thr, seed=2024, stream=0, first=0, count=N)
    roots = np.array([O.root(2024, 0, i, n) for i in range(N)])
    hits = np.zeros((n, n))
    cnt = np.bincount(roots, minlength=n).astype(np.float64)
    for i in range(N):
        for v in r.set(i):
            hits[v, roots[i]] += 1
    for t in range(n):
        for v in range(n):
            mu = P[v, t]
            f = hits[v, t] / cnt[t]
            sd = math.sqrt(max(mu * (1 - mu), 1e-12) / cnt[t])
            assert abs(f - mu) < 5 * sd + 1e-9, (v, t, f, mu)
    # RIS identity for S = {0, 3}: sigma(S) exact vs n * fraction of sets hit
    worlds_sigma = 0.0
    m = len(TINY_EDGES)
    for mask in range(1 << m):
        pr = 1.0
        live = []
        for j in range(m):
            if mask >> j & 1:
                pr *= q[j]
                live.append(TINY_EDGES[j])
            else:
                pr *= 1 - q[j]
        worlds_sigma += pr * len(_forward_reach(n, live, 0) | _forward_reach(n, live, 3))
    hit = np.mean([bool(set(r.set(i)) & {0, 3}) for i in range(N)])
    sd = math.sqrt(hit * (1 - hit) / N) * n
    assert abs(n * hit - worlds_sigma) < 5 * sd


def test_ic_examined_and_live_counters():
    g = W.random_small_graph(80, 300, seed=3)
    thr = O.ic_thresholds(g.weight)
    r = O.sample(O.IC, g.in_off, g.in_src, thr, seed=1, stream=0, first=0, count=300)
    deg = np.diff(g.in_off)
    assert r.examined == int(deg[r.mem].sum())
    assert 0 <= r.live <= r.examined


def test_sampling_is_split_invariant():
    """A set depends only on (seed, stream, sample id): ranges compose."""
    g = W.random_small_graph(120, 500, seed=4, p_hi=0.4)
    thr = O.ic_thresholds(g.weight)
    a = O.sample(O.IC, g.in_off, g.in_src, thr, 3, 0, 0, 100)
    b = O.sample(O.IC, g.in_off, g.in_src, thr, 3, 0, 40, 60)
    assert np.array_equal(a.mem[a.off[40]:], b.mem)
    assert np.array_equal(np.diff(a.off)[40:], np.diff(b.off))


# ---------------------------------------------------------------- LT sampling
def test_lt_zero_weights_singletons():
    g = W.tiny_graph(5, [(0, 1), (1, 2), (3, 2)], [0, 0, 0], model=W.LT)
    c = O.lt_thresholds(g.in_off, g.weight)
    r = O.sample(O.LT, g.in_off, g.in_src, c, 1, 0, 0, 200)
    assert np.all(np.diff(r.off) == 1)


def test_lt_unit_chain_is_full_reverse_path():
    """Every vertex has one in-edge of weight 1: R(i) is the whole backward path."""
    n = 30
    edges = [(v, v + 1) for v in range(n - 1)]
    g = W.tiny_graph(n, edges, [1.0] * (n - 1), model=W.LT)
    c = O.lt_thresholds(g.in_off, g.weight)
    r = O.sample(O.LT, g.in_off, g.in_src, c, 5, 0, 0, 300)
    for i in range(300):
        root = O.root(5, 0, i, n)
        assert list(r.set(i)) == list(range(0, root + 1))


def test_lt_cycle_stops_at_repeat():
    n = 6
    edges = [(v, (v + 1) % n) for v in range(n)]  # a directed 6-cycle, weights 1
    g = W.tiny_graph(n, edges, [1.0] * n, model=W.LT)
    c = O.lt_thresholds(g.in_off, g.weight)
    r = O.sample(O.LT, g.in_off, g.in_src, c, 5, 0, 0, 50)
    assert np.all(np.diff(r.off) == n)


def _exact_lt_sigma(n, edges, w):
    """sigma({v}) under LT by enumerating every vertex's live in-edge choice."""
    ins = [[] for _ in range(n)]
    for j, (u, v) in enumerate(edges):
        ins[v].append(j)
    choices = []
    for v in range(n):
        opts = [(j, w[j]) for j in ins[v]]
        opts.append((None, max(0.0, 1.0 - sum(w[j] for j in ins[v]))))
        choices.append(opts)
    sig = np.zeros(n)
    for combo in itertools.product(*choices):
        pr = 1.0
        live = []
        for (j, pj) in combo:
            pr *= pj
            if j is not None:
                live.append(edges[j])
        if pr == 0:
            continue
        for v in range(n):
            sig[v] += pr * len(_forward_reach(n, live, v))
    return sig


def test_lt_membership_matches_exact_enumeration():
    """Pr[v in R(i)] = sigma({v}) / n under the live-edge reading of LT."""
    n = 6
    w_raw = [0.5, 0.3, 0.7, 0.4, 0.6, 0.2, 0.6, 0.5, 0.25, 0.8]
    g = W.tiny_graph(n, TINY_EDGES, w_raw, model=W.LT)
    # normalise per target so that in-weights sum to at most 1
    tot = {}
    for (u, v), x in zip(TINY_EDGES, w_raw):
        tot[v] = tot.get(v, 0.0) + x
    w = [x / max(1.0, tot[v]) * 0.95 for (u, v), x in zip(TINY_EDGES, w_raw)]
    g = W.tiny_graph(n, TINY_EDGES, w, model=W.LT)
    c = O.lt_thresholds(g.in_off, g.weight)
    wq = [math.floor(np.float32(x) * 2.0 ** 32) / 2.0 ** 32 for x in w]
    sig = _exact_lt_sigma(n, TINY_EDGES, wq)
    N = 150000
    r = O.sample(O.LT, g.in_off, g.in_src, c, 77, 0, 0, N)
    freq = np.bincount(r.mem, minlength=n) / N
    for v in range(n):
        mu = sig[v] / n
        sd = math.sqrt(mu * (1 - mu) / N)
        assert abs(freq[v] - mu) < 5 * sd, (v, freq[v], mu)


# ---------------------------------------------------------------- incidence/cover
def _small_collection(seed=21, n=60, count=400, p_hi=0.3):
    g = W.random_small_graph(n, 4 * n, seed=seed, p_hi=p_hi)
    thr = O.ic_thresholds(g.weight)
    r = O.sample(O.IC, g.in_off, g.in_src, thr, seed, 0, 0, count)
    io, im = O.incidence(g.n, r)
    return g, r, io, im


def test_incidence_is_transpose():
    g, r, io, im = _small_collection()
    assert io[-1] == r.total
    pairs_r = {(int(v), i) for i in range(r.count) for v in r.set(i)}
    pairs_s = {(v, int(i)) for v in range(g.n) for i in im[io[v]:io[v + 1]]}
    assert pairs_r == pairs_s
    for v in range(g.n):
        s = im[io[v]:io[v + 1]]
        assert np.all(np.diff(s) > 0)


def test_coverage_is_union_size():
    g, r, io, im = _small_collection()
    rng = np.random.default_rng(0)
    for _ in range(20):
        S = rng.choice(g.n, size=5, replace=False)
        u = np.unique(np.concatenate([im[io[v]:io[v + 1]] for v in S]))
        assert O.coverage(g.n, r.count, io, im, S) == u.size


def _brute_opt(n, sets, k):
    best = 0
    for S in itertools.combinations(range(n), k):
        best = max(best, len(set().union(*[sets[v] for v in S])))
    return best


def _random_set_system(rng, n, universe, density):
    inc = [sorted(set(rng.choice(universe, size=rng.integers(0, max(1, int(density * universe))),
                                 replace=False).tolist())) for _ in range(n)]
    io = np.zeros(n + 1, np.int64)
    io[1:] = np.cumsum([len(s) for s in inc])
    im = np.array([x for s in inc for x in s], np.int32)
    return [set(s) for s in inc], io, im


@pytest.mark.parametrize("seed", range(12))
def test_greedy_against_brute_force(seed):
    """(1 - 1/e) of the brute-force optimum (Sec. 3.2), non-increasing gains
    (submodularity, Sec. 2), gains summing to the coverage, lowest-id ties."""
    rng = np.random.default_rng(seed)
    n, universe, k = int(rng.integers(6, 13)), int(rng.integers(10, 40)), int(rng.integers(1, 5))
    sets, io, im = _random_set_system(rng, n, universe, 0.35)
    seeds, gains, cov = O.greedy(n, universe, io, im, k)
    opt = _brute_opt(n, sets, k)
    assert cov >= (1 - 1 / math.e) * opt - 1e-9
    assert np.all(np.diff(gains) <= 0)
    assert gains.sum() == cov == O.coverage(n, universe, io, im, seeds)
    # replay by hand: every pick is the lowest id of largest marginal gain
    covered = set()
    for s, gval in zip(seeds, gains):
        marg = [len(sets[v] - covered) for v in range(n)]
        assert gval == max(marg) and s == marg.index(max(marg))
        covered |= sets[s]
    if len(seeds) < k:  # stopped early only because nothing is left to gain
        assert max(len(sets[v] - covered) for v in range(n)) == 0


@pytest.mark.parametrize("seed", range(6))
def test_lazy_greedy_equals_plain(seed):
    """Algorithm 2 (with (gain, -id) heap keys) returns the standard greedy's picks."""
    g, r, io, im = _small_collection(seed=100 + seed, n=150, count=2000, p_hi=0.25)
    a = O.greedy(g.n, r.count, io, im, 12)
    b = O.greedy(g.n, r.count, io, im, 12, lazy=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_greedy_p0_is_top_root_counts():
    """p = 0: sets are single roots, so greedy takes the k most frequent roots,
    ties to the lower id."""
    g = W.random_small_graph(40, 100, seed=8)
    thr = O.ic_thresholds(np.zeros(g.num_edges, np.float32))
    r = O.sample(O.IC, g.in_off, g.in_src, thr, 13, 0, 0, 300)
    io, im = O.incidence(g.n, r)
    seeds, gains, cov = O.greedy(g.n, r.count, io, im, 10)
    cnt = np.bincount(r.mem, minlength=g.n)
    order = np.argsort(-cnt, kind="stable")[:10]
    order = order[cnt[order] > 0]
    assert list(seeds) == list(order)
    assert list(gains) == list(cnt[order])


def test_greedy_hand_example():
    """Four samples; S(0)={0,1}, S(1)={1,2,3}, S(2)={0,3}, S(3)={2}.
    Greedy: vertex 1 (gain 3), then vertex 0 (gain 1, lowest id among 0 and 2)."""
    io = np.array([0, 2, 5, 7, 8], np.int64)
    im = np.array([0, 1, 1, 2, 3, 0, 3, 2], np.int32)
    seeds, gains, cov = O.greedy(4, 4, io, im, 3)
    assert list(seeds) == [1, 0] and list(gains) == [3, 1] and cov == 4


# ---------------------------------------------------------------- RandGreedi
def test_partition_uniform_and_total():
    n, m = 100000, 64
    part = O.partition(n, m, 4003)
    assert part.max() < m
    cnt = np.bincount(part, minlength=m)
    assert cnt.sum() == n
    exp = n / m
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    assert chi2 < 63 + 6 * math.sqrt(2 * 63)
    assert np.all(O.partition(1000, 1, 5) == 0)


def test_local_greedy_m1_is_greedy():
    g, r, io, im = _small_collection(seed=31, n=120, count=1500)
    part = O.partition(g.n, 1, 9)
    ls, lg, lc, lv = O.local_greedy(g.n, r.count, io, im, part, 1, 10, lazy=False)
    s, ga, cov = O.greedy(g.n, r.count, io, im, 10)
    assert list(ls[0, :lc[0]]) == list(s) and lv[0] == cov


def test_local_greedy_lazy_equals_plain_and_first_picks():
    g, r, io, im = _small_collection(seed=32, n=200, count=3000, p_hi=0.25)
    part = O.partition(g.n, 8, 77)
    a = O.local_greedy(g.n, r.count, io, im, part, 8, 7, lazy=False)
    b = O.local_greedy(g.n, r.count, io, im, part, 8, 7, lazy=True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    ls, lg, lc, lv = a
    for p in range(8):
        assert np.all(part[ls[p, :lc[p]]] == p)
        assert lg[p, :lc[p]].sum() == lv[p]
    # the global greedy's first pick is some partition's first pick
    s, _, _ = O.greedy(g.n, r.count, io, im, 1)
    assert s[0] in set(ls[:, 0].tolist())


@pytest.mark.parametrize("seed", range(6))
def test_truncated_greedy_bound(seed):
    """Lemma (truncated greedy): the first T picks cover at least
    (1 - (1 - 1/k)^T) OPT_k >= (1 - e^{-T/k}) OPT_k."""
    rng = np.random.default_rng(50 + seed)
    n, universe, k = 11, 30, 4
    sets, io, im = _random_set_system(rng, n, universe, 0.3)
    opt = _brute_opt(n, sets, k)
    part = np.zeros(n, np.uint8)
    ls, lg, lc, lv = O.local_greedy(n, universe, io, im, part, 1, k)
    for T in range(1, k + 1):
        got = lg[0, :min(T, lc[0])].sum()
        assert got >= (1 - (1 - 1 / k) ** T) * opt - 1e-9
        assert got >= (1 - math.exp(-T / k)) * opt - 1e-9


# ---------------------------------------------------------------- streaming
def test_bucket_count_and_thresholds():
    """k = 100, delta = 0.077 gives 63 buckets, the receiver's 63 bucketing
    threads of the experimental setup (Sec. 4.1)."""
    assert O.num_buckets(100, 0.077) == 63
    assert O.num_buckets(1, 0.077) == 1
    thr = O.bucket_thresholds(5000, 100, 0.077)
    assert thr.shape == (63,)
    assert thr[0] == 25  # ceil(5000 / 200)
    assert np.all(np.diff(thr) >= 0)
    # geometric growth: thr_b / thr_0 ~ (1 + delta)^b
    assert abs(thr[-1] / 25.0 - 1.077 ** 62) / 1.077 ** 62 < 0.05
    assert O.trunc_len(100, 0.125) == 13 and O.trunc_len(100, 1.0) == 100
    assert O.trunc_len(8, 0.01) == 1


def test_stream_hand_example():
    """Alg. 5 by hand: k = 2, delta = 0.4 -> B = ceil(ln 2 / ln 1.4) = 3;
    stream (m = 1) = picks [1, 0, 2] of S(1)={0..5}, S(0)={6,7}, S(2)={0,6};
    l = 6, thresholds ceil(6*1/4)=2, ceil(6*1.4/4)=3 (2.1), ceil(6*1.96/4)=3 (2.94).
    Bucket 0 takes 1 (gain 6) and 0 (gain 2); buckets 1, 2 take 1 only; b* = 0."""
    io = np.array([0, 2, 8, 10], np.int64)
    im = np.array([6, 7, 0, 1, 2, 3, 4, 5, 0, 6], np.int32)
    ls = np.array([[1, 0]], np.int32)
    lg = np.array([[6, 2]], np.int64)
    lc = np.array([2], np.int32)
    assert O.num_buckets(2, 0.4) == 3
    assert list(O.bucket_thresholds(6, 2, 0.4)) == [2, 3, 3]
    seeds, cov, b, nb = O.stream_cover(3, 8, io, im, ls, lg, lc, 2, 0.4, 1.0)
    assert nb == 3 and b == 0 and list(seeds) == [1, 0] and cov == 8


@pytest.mark.parametrize("seed", range(10))
def test_stream_half_minus_delta_bound(seed):
    """Alg. 5 is (1/2 - delta)-approximate against the best k of the streamed
    sets (Sec. 3.3.1); buckets hold at most k seeds; truncation only shortens."""
    rng = np.random.default_rng(300 + seed)
    n, universe, k, m = 16, 40, 3, 4
    sets, io, im = _random_set_system(rng, n, universe, 0.3)
    part = O.partition(n, m, 1000 + seed)
    ls, lg, lc, lv = O.local_greedy(n, universe, io, im, part, m, k)
    for alpha in (1.0, 0.34):
        delta = 0.1
        seeds, cov, b, nb = O.stream_cover(n, universe, io, im, ls, lg, lc, k, delta, alpha)
        T = O.trunc_len(k, alpha)
        streamed = [int(ls[p, t]) for t in range(T) for p in range(m) if t < lc[p]]
        assert len(seeds) <= k and set(seeds.tolist()) <= set(streamed)
        assert cov == O.coverage(n, universe, io, im, seeds)
        best = max(len(set().union(*[sets[x] for x in S]))
                   for S in itertools.combinations(streamed, min(k, len(streamed))))
        assert cov >= (0.5 - delta) * best - 1e-9
        # stream order is round-major: acceptance order follows it
        pos = {x: j for j, x in enumerate(streamed)}
        assert all(pos[a] < pos[b2] for a, b2 in zip(seeds[:-1], seeds[1:]))


def test_final_select():
    ls = np.array([[3, 4], [5, -1]], np.int32)
    lc = np.array([2, 1], np.int32)
    lv = np.array([10, 12], np.int64)
    s, c, won = O.final_select(ls, lc, lv, np.array([7, 8], np.int32), 12)
    assert won and list(s) == [7, 8] and c == 12  # tie goes to the streamed solution
    s, c, won = O.final_select(ls, lc, lv, np.array([7], np.int32), 11)
    assert not won and list(s) == [5] and c == 12
    lv2 = np.array([12, 12], np.int64)
    s, c, won = O.final_select(ls, lc, lv2, np.array([7], np.int32), 3)
    assert list(s) == [3, 4]  # lowest partition among equal local coverages


def test_worked_approximation_ratio():
    """Sec. 4.2: eps = 0.13, delta = 0.077 give a worst-case ratio of 0.123 for
    GreediRIS (Lemma with streaming) and 0.5 for the standard greedy IMM."""
    e1 = 1 - 1 / math.e
    h = 0.5 - 0.077
    ratio = e1 * h / (e1 + h) - 0.13
    assert round(ratio, 3) == 0.123
    assert round(e1 - 0.13, 1) == 0.5


# ---------------------------------------------------------------- IMM
def test_imm_parameters_pins():
    n, k, eps = 1 << 22, 100, 0.13
    p = O.imm_parameters(n, k, eps)
    lb = gammaln(n + 1) - gammaln(k + 1) - gammaln(n - k + 1)
    assert abs(p["log_binom"] - lb) < 1e-7 * lb
    assert p["rounds"] == 21
    assert p["theta1"] == math.ceil(p["lambda_prime"] / (n / 2))
    assert abs(p["eps_prime"] - math.sqrt(2) * eps) < 1e-15
    # monotone: more precision or more seeds need more samples
    q = O.imm_parameters(n, k, eps / 2)
    assert q["lambda_star"] > p["lambda_star"] and q["lambda_prime"] > p["lambda_prime"]
    r = O.imm_parameters(n, 2 * k, eps)
    assert r["lambda_star"] > p["lambda_star"]
    assert O.imm_parameters(4096, 16, 0.5)["rounds"] == 11


def test_imm_end_to_end_tiny():
    """IMM's seeds are (1 - 1/e - eps)-approximate for influence (Theorem 2.1):
    exact sigma of every k-subset by enumeration of live-edge worlds."""
    n = 6
    g = W.tiny_graph(n, TINY_EDGES, TINY_P)
    thr = O.ic_thresholds(g.weight)
    q = O.ic_thresholds(np.array(TINY_P, np.float32)).astype(np.float64) / 2.0 ** 32
    P = _exact_ic_activation(n, TINY_EDGES, list(q))

    def sigma(S):
        # P[v, t] is per-source; sigma of a set needs the joint worlds
        tot = 0.0
        m = len(TINY_EDGES)
        for mask in range(1 << m):
            pr = 1.0
            live = []
            for j in range(m):
                if mask >> j & 1:
                    pr *= q[j]
                    live.append(TINY_EDGES[j])
                else:
                    pr *= 1 - q[j]
            reach = set()
            for s in S:
                reach |= _forward_reach(n, live, s)
            tot += pr * len(reach)
        return tot

    assert abs(sigma([2]) - P[2].sum()) < 1e-9
    k, eps = 2, 0.5
    out = O.imm(O.IC, g.in_off, g.in_src, thr, k, eps, seed=99)
    opt = max(sigma(S) for S in itertools.combinations(range(n), k))
    assert out["theta"] > 0 and out["nsel"] == k
    assert sigma(out["seeds"].tolist()) >= (1 - 1 / math.e - eps) * opt
    # GreediRIS selector on the same instance meets its own (weaker) guarantee
    out2 = O.imm(O.IC, g.in_off, g.in_src, thr, k, eps, seed=99, selector=O.SEL_GREEDIRIS,
                 m=2, delta=0.077, alpha=1.0, part_seed=5)
    e1 = 1 - 1 / math.e
    h = 0.5 - 0.077
    assert sigma(out2["seeds"].tolist()) >= (e1 * h / (e1 + h) - eps) * opt


# ---------------------------------------------------------------- run-length IC
def test_log_matches_libm():
    """The method's log agrees with the C library's to ~1 ulp across the range
    it is used on (uniforms in (0,1] and 1 - p for p down to 2^-32)."""
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.random(2000), 1.0 - rng.random(200) * 1e-6,
                         [2.0 ** -53, 0.5, 1.0 - 2.0 ** -32, 1.0, 0.70710678, 1.41421356, 3.0,
                          1e-300, 1e300]])
    for x in xs:
        x = float(x)
        got, ref = O.log(x), math.log(x)
        assert abs(got - ref) <= 4e-16 * max(1.0, abs(ref)), (x, got, ref)
    assert O.log(1.0) == 0.0


def test_skip_table():
    w = W.ic_weighted_cascade(np.array([0, 1, 3, 6, 6, 10], np.int32))
    in_off = np.array([0, 1, 3, 6, 6, 10], np.int32)
    thr = O.ic_thresholds(w)
    sk = O.ic_skip_table(in_off, thr)
    assert sk[0] == 0.0 and sk[3] == 0.0          # one in-edge / none: coins
    for v, d in ((1, 2), (2, 3), (4, 4)):
        q = int(thr[in_off[v]])
        assert abs(sk[v] - 1.0 / math.log1p(-q / 2 ** 32)) < 1e-12 * abs(sk[v])
    mixed = thr.copy()
    mixed[4] ^= 1
    assert O.ic_skip_table(in_off, mixed)[2] == 0.0   # thresholds differ: coins


def test_skip_counts_are_binomial():
    """A hub with D in-edges of probability p from D private leaves: the number
    of live in-edges per visit is Binomial(D, p) under the run-length form."""
    R, D, p = 60, 200, 0.05
    edges = [(R + h * D + j, h) for h in range(R) for j in range(D)]
    n = R + R * D
    g = W.tiny_graph(n, edges, np.full(len(edges), p, np.float32))
    thr = O.ic_thresholds(g.weight)
    assert np.all(O.ic_skip_table(g.in_off, thr)[:R] != 0)
    N = 400000
    r = O.sample(O.IC, g.in_off, g.in_src, thr, 17, 0, 0, N)
    roots = np.array([O.root(17, 0, i, n) for i in range(N)])
    hub = roots < R
    sizes = np.diff(r.off)[hub] - 1
    q = int(thr[0]) / 2 ** 32
    mean, var = D * q, D * q * (1 - q)
    assert hub.sum() > 1000
    assert abs(sizes.mean() - mean) < 5 * math.sqrt(var / hub.sum())
    assert abs(sizes.var() - var) < 0.15 * var


def test_skip_membership_matches_exact_enumeration():
    """Weighted cascade on the tiny graph (uniform thresholds per vertex, so
    the run-length form is used): Pr[v in R | root = t] equals the exact
    probability over all live-edge worlds."""
    n = 6
    deg = np.bincount([v for _, v in TINY_EDGES], minlength=n)
    probs = [np.float32(1.0) / np.float32(deg[v]) for _, v in TINY_EDGES]
    g = W.tiny_graph(n, TINY_EDGES, probs)
    thr = O.ic_thresholds(g.weight)
    assert np.count_nonzero(O.ic_skip_table(g.in_off, thr)) >= 3
    q = O.ic_thresholds(np.array(probs, np.float32)).astype(np.float64) / 2.0 ** 32
    P = _exact_ic_activation(n, TINY_EDGES, list(q))
    N = 120000
    r = O.sample(O.IC, g.in_off, g.in_src, thr, 99, 0, 0, N)
    roots = np.array([O.root(99, 0, i, n) for i in range(N)])
    cnt = np.bincount(roots, minlength=n).astype(np.float64)
    hits = np.zeros((n, n))
    for i in range(N):
        for v in r.set(i):
            hits[v, roots[i]] += 1
    for t in range(n):
        for v in range(n):
            mu = P[v, t]
            f = hits[v, t] / cnt[t]
            sd = math.sqrt(max(mu * (1 - mu), 1e-12) / cnt[t])
            assert abs(f - mu) < 5 * sd + 1e-9, (v, t, f, mu)


# ------------------------------------------- run-length form: exact and in law
def _wc_thresholds():
    """Thresholds the run-length form sees: weighted cascade p = fp32(1/d) for
    in-degrees 2 .. 2^20, plus extremes (tiny q, q near 2^32 - 2, the largest
    fp32 below 1)."""
    ds = [2, 3, 4, 5, 7, 10, 16, 31, 100, 1000, 4096, 65536, 1 << 20]
    qs = [int(x) for x in O.ic_thresholds(np.float32(1.0) / np.array(ds, np.float32))]
    qs += [1, 2, 1000, 2 ** 31 + 1, 2 ** 32 - 2 ** 8, 2 ** 32 - 3, 2 ** 32 - 2]
    return qs


def test_run_length_gap_equals_exact_quotient():
    """G = floor(ln U / ln(1 - q/2^32)) for >= 10^5 (U, q) pairs, with ln
    evaluated in 60-digit decimal arithmetic (correctly rounded), against the
    oracle's own gap step (the fixed fp64 log and the table factor).  Equal
    everywhere except where the exact quotient lies within 1e-12 (relative)
    of an integer, where either neighbour is accepted; such ties are counted."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    rng = np.random.default_rng(2024)
    qs = _wc_thresholds()
    N = 100000
    bits = rng.integers(0, 2 ** 53, N, dtype=np.int64)
    bits[:4] = [0, 1, 2 ** 53 - 1, 2 ** 52]  # U = 2^-53, 2^-52, 1, just above 1/2
    qi = rng.integers(0, len(qs), N)
    two53 = Decimal(2 ** 53)
    two32 = Decimal(2 ** 32)
    ln_keep = {q: ((two32 - Decimal(q)) / two32).ln() for q in qs}
    factor = {q: O.rl_factor(q) for q in qs}
    ties = 0
    for b, j in zip(bits.tolist(), qi.tolist()):
        q = qs[j]
        u = (b + 1) * 2.0 ** -53  # exact in fp64
        g = O.rl_gap(u, factor[q])
        x = (Decimal(b + 1) / two53).ln() / ln_keep[q]
        exact = int(x.to_integral_value(rounding="ROUND_FLOOR"))
        if g != exact:
            near = abs(x - x.to_integral_value()) <= Decimal("1e-12") * max(Decimal(1), abs(x))
            assert near, (b, q, g, exact, x)
            assert abs(g - exact) == 1
            ties += 1
    assert O.rl_gap(1.0, factor[qs[0]]) == 0
    assert ties <= 5, ties


@pytest.mark.parametrize("p", [0.5, 1.0 / 16, 1.0 / 1000])
def test_run_length_gaps_are_geometric(p):
    """The gaps the oracle generates from its own draws (U of draw pairs j
    over many samples and vertices) follow Geometric(p): Pr[G = g] =
    (1-p)^g p, by a chi-square goodness-of-fit over bins of equal mass."""
    from scipy.stats import chisquare
    q = int(O.ic_thresholds(np.array([p], np.float32))[0])
    pq = q / 2 ** 32
    f = O.rl_factor(q)
    G = np.array([O.rl_gap(O.rl_uniform(77, 0, i, v, j), f)
                  for i in range(50) for v in range(40) for j in range(40)], np.int64)
    # bins of about equal probability: edges at geometric quantiles
    nb = 40
    edges = np.unique(np.floor(np.log1p(-np.arange(1, nb) / nb) / math.log1p(-pq)).astype(int))
    cdf = lambda g: 1.0 - (1.0 - pq) ** (g + 1)  # noqa: E731  Pr[G <= g]
    lo = np.concatenate([[0], edges + 1])
    hi = np.concatenate([edges, [np.iinfo(np.int64).max]])
    probs = np.array([cdf(h) if h < np.iinfo(np.int64).max else 1.0 for h in hi]) - \
        np.array([cdf(l - 1) if l > 0 else 0.0 for l in lo])
    obs = np.array([np.count_nonzero((G >= l) & (G <= h)) for l, h in zip(lo, hi)])
    assert obs.sum() == G.size and abs(probs.sum() - 1) < 1e-12
    assert chisquare(obs, probs * G.size).pvalue > 1e-3
    assert abs(G.mean() - (1 - pq) / pq) < 5 * math.sqrt((1 - pq) / pq ** 2 / G.size)


def test_run_length_and_coin_forms_agree_in_law():
    """One weighted-cascade graph sampled 10^5 times with one coin per in-edge
    and 10^5 times with run-length gaps (different draws, same law): the set
    sizes and the per-vertex membership counts pass two-sample chi-square
    tests."""
    from scipy.stats import chi2_contingency
    g = W.make_graph("rmat", W.IC, scale=12, num_edges=1 << 16, graph_seed=61, weight_seed=62,
                     weights="wc")
    thr = O.ic_thresholds(g.weight)
    assert np.count_nonzero(O.ic_skip_table(g.in_off, thr)) > g.n // 4
    N = 100000
    a = O.sample(O.IC, g.in_off, g.in_src, thr, 501, 0, 0, N, skip=None)
    b = O.sample(O.IC, g.in_off, g.in_src, thr, 502, 0, 0, N)
    sa, sb = np.diff(a.off), np.diff(b.off)
    top = 12
    ha = np.bincount(np.minimum(sa, top), minlength=top + 1)[1:]
    hb = np.bincount(np.minimum(sb, top), minlength=top + 1)[1:]
    assert chi2_contingency(np.vstack([ha, hb]))[1] > 1e-3
    ma = np.bincount(a.mem, minlength=g.n)
    mb = np.bincount(b.mem, minlength=g.n)
    keep = (ma + mb) >= 40
    assert keep.sum() > 500
    assert chi2_contingency(np.vstack([ma[keep], mb[keep]]))[1] > 1e-3


# ------------------------------------------- RandGreedi's offline global step
@pytest.mark.parametrize("seed", range(10))
def test_offline_aggregation_against_brute_force(seed):
    """Alg. 4 global step on tiny set systems: S_g is drawn from the union of
    the gathered local solutions, reaches (1 - 1/e) of the best k-subset of
    that union (brute force), has non-increasing gains summing to its
    coverage, and replays by hand as lowest-id argmax picks over the union."""
    rng = np.random.default_rng(700 + seed)
    n, universe = int(rng.integers(8, 15)), int(rng.integers(10, 40))
    k, m = int(rng.integers(1, 5)), int(rng.integers(2, 5))
    sets, io, im = _random_set_system(rng, n, universe, 0.3)
    part = O.partition(n, m, 900 + seed)
    ls, lg, lc, lv = O.local_greedy(n, universe, io, im, part, m, k, lazy=False)
    alpha = float(rng.choice([1.0, 0.5]))
    T = O.trunc_len(k, alpha)
    union = sorted(int(ls[p, t]) for p in range(m) for t in range(min(T, int(lc[p]))))
    gs, gg, gc = O.greedi_offline(n, universe, io, im, ls, lc, k, alpha=alpha)
    assert set(gs.tolist()) <= set(union)
    best = 0
    for r_ in range(1, min(k, len(union)) + 1):
        for S in itertools.combinations(union, r_):
            best = max(best, len(set().union(*[sets[v] for v in S])))
    assert gc >= (1 - 1 / math.e) * best - 1e-9
    assert np.all(np.diff(gg) <= 0) and gg.sum() == gc == O.coverage(n, universe, io, im, gs)
    covered = set()
    for s, gval in zip(gs, gg):
        marg = [len(sets[v] - covered) for v in union]
        assert gval == max(marg) and s == union[marg.index(max(marg))]
        covered |= sets[s]


@pytest.mark.parametrize("seed", range(4))
def test_offline_aggregation_lazy_equals_plain(seed):
    g, r, io, im = _small_collection(seed=140 + seed, n=300, count=3000, p_hi=0.25)
    part = O.partition(g.n, 8, 11 + seed)
    ls, lg, lc, lv = O.local_greedy(g.n, r.count, io, im, part, 8, 12)
    a = O.greedi_offline(g.n, r.count, io, im, ls, lc, 12, lazy=False)
    b = O.greedi_offline(g.n, r.count, io, im, ls, lc, 12, lazy=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_offline_aggregation_one_part_returns_its_greedy():
    """m = 1: the gathered set is the standard greedy's own picks, and the
    greedy over them picks them again in the same order."""
    g, r, io, im = _small_collection(seed=150, n=200, count=2500, p_hi=0.2)
    part = O.partition(g.n, 1, 3)
    ls, lg, lc, lv = O.local_greedy(g.n, r.count, io, im, part, 1, 10)
    gs, gg, gc = O.greedi_offline(g.n, r.count, io, im, ls, lc, 10)
    s, ga, cov = O.greedy(g.n, r.count, io, im, 10)
    assert list(gs) == list(s) and list(gg) == list(ga) and gc == cov


def test_imm_randgreedi_final_choice():
    """IMM with the RandGreedi selector: the result is the better of the
    offline global solution and the best local one (Alg. 4, final step)."""
    g = W.random_small_graph(400, 2400, seed=12, p_hi=0.3)
    thr = O.ic_thresholds(g.weight)
    res = O.imm(O.IC, g.in_off, g.in_src, thr, 6, 0.5, seed=5, selector=O.SEL_RANDGREEDI, m=4,
                part_seed=6, theta=3000)
    r = O.sample(O.IC, g.in_off, g.in_src, thr, 5, 1, 0, 3000)
    io, im = O.incidence(g.n, r)
    part = O.partition(g.n, 4, 6)
    ls, lg, lc, lv = O.local_greedy(g.n, 3000, io, im, part, 4, 6)
    gs, gg, gc = O.greedi_offline(g.n, 3000, io, im, ls, lc, 6)
    assert res["coverage"] == max(gc, int(lv.max()))
    assert res["global_won"] == int(gc >= lv.max())
    assert res["stream_len"] == int(lc.sum())


# ------------------------------------------- forward influence (quality measure)
def test_influence_p1_is_forward_reachability():
    """p = 1: every world is the whole graph, so each count is the number of
    vertices reachable from the seeds (breadth-first search, textbook)."""
    g = W.random_small_graph(300, 700, seed=11)
    thr = O.ic_thresholds(np.ones(g.num_edges, np.float32))
    fwd = sp.csr_matrix((np.ones(g.num_edges), (g.in_src, np.repeat(np.arange(g.n),
                                                                     np.diff(g.in_off)))),
                        shape=(g.n, g.n))
    for seeds in ([0], [5, 17, 200], [3, 3, 3]):
        reach = set()
        for s in seeds:
            reach |= set(breadth_first_order(fwd, s, directed=True,
                                             return_predecessors=False).tolist())
        c = O.influence(O.IC, g.in_off, g.in_src, thr, 9, 0, 0, 20, seeds)
        assert np.all(c == len(reach))


def test_influence_p0_and_zero_weights_are_the_seeds():
    g = W.random_small_graph(80, 400, seed=12)
    thr0 = O.ic_thresholds(np.zeros(g.num_edges, np.float32))
    assert np.all(O.influence(O.IC, g.in_off, g.in_src, thr0, 1, 0, 0, 50, [4, 9, 9]) == 2)
    c0 = O.lt_thresholds(g.in_off, np.zeros(g.num_edges, np.float32))
    assert np.all(O.influence(O.LT, g.in_off, g.in_src, c0, 1, 0, 0, 50, [4, 9, 11]) == 3)


def _exact_sigma_ic(n, edges, q, S):
    total = 0.0
    m = len(edges)
    for mask in range(1 << m):
        pr = 1.0
        live = []
        for j in range(m):
            if mask >> j & 1:
                pr *= q[j]
                live.append(edges[j])
            else:
                pr *= 1 - q[j]
        reach = set()
        for s in S:
            reach |= _forward_reach(n, live, s)
        total += pr * len(reach)
    return total


def _exact_sigma_lt(n, edges, w, S):
    ins = [[] for _ in range(n)]
    for j, (u, v) in enumerate(edges):
        ins[v].append(j)
    choices = [[(j, w[j]) for j in ins[v]] + [(None, max(0.0, 1.0 - sum(w[j] for j in ins[v])))]
               for v in range(n)]
    total = 0.0
    for combo in itertools.product(*choices):
        pr = 1.0
        live = []
        for (j, pj) in combo:
            pr *= pj
            if j is not None:
                live.append(edges[j])
        if pr == 0:
            continue
        reach = set()
        for s in S:
            reach |= _forward_reach(n, live, s)
        total += pr * len(reach)
    return total


@pytest.mark.parametrize("S", [[0], [2, 4], [1, 3, 5]])
def test_influence_mean_matches_exact_sigma(S):
    """The mean count over many simulations equals sigma(S) computed exactly
    over all live-edge worlds (IC: 2^10 worlds; LT: every vertex's choice)."""
    n = 6
    g = W.tiny_graph(n, TINY_EDGES, TINY_P)
    thr = O.ic_thresholds(g.weight)
    q = O.ic_thresholds(np.array(TINY_P, np.float32)).astype(np.float64) / 2.0 ** 32
    N = 60000
    c = O.influence(O.IC, g.in_off, g.in_src, thr, 31, 0, 0, N, S)
    mu = _exact_sigma_ic(n, TINY_EDGES, list(q), S)
    assert abs(c.mean() - mu) < 5 * c.std() / math.sqrt(N) + 1e-9, (c.mean(), mu)
    w = [x * 0.45 for x in TINY_P]  # in-weights of every vertex sum below 1
    gl = W.tiny_graph(n, TINY_EDGES, w, model=W.LT)
    cl = O.lt_thresholds(gl.in_off, gl.weight)
    wq = [math.floor(np.float32(x) * 2.0 ** 32) / 2.0 ** 32 for x in w]
    c = O.influence(O.LT, gl.in_off, gl.in_src, cl, 32, 0, 0, N, S)
    mu = _exact_sigma_lt(n, TINY_EDGES, wq, S)
    assert abs(c.mean() - mu) < 5 * c.std() / math.sqrt(N) + 1e-9, (c.mean(), mu)


@pytest.mark.parametrize("model", [O.IC, O.LT])
def test_influence_agrees_with_reverse_sampling(model):
    """sigma(S) two ways on one graph: forward simulation, and n times the
    fraction of RRR sets that S hits (the RIS estimator of Sec. 2.1)."""
    g = W.random_small_graph(2000, 12000, seed=40 + model, model=model, p_hi=0.25)
    thr = O.thresholds(model, g.in_off, g.weight)
    S = [1, 77, 400, 1234, 1999]
    N = 20000
    c = O.influence(model, g.in_off, g.in_src, thr, 51, 0, 0, N, S)
    theta = 200000
    r = O.sample(model, g.in_off, g.in_src, thr, 52, 0, 0, theta)
    io, im = O.incidence(g.n, r)
    ris = g.n * O.coverage(g.n, theta, io, im, S) / theta
    p = O.coverage(g.n, theta, io, im, S) / theta
    sd = math.sqrt(c.var() / N + (g.n ** 2) * p * (1 - p) / theta)
    assert abs(c.mean() - ris) < 5 * sd, (c.mean(), ris, sd)


# ------------------------------------------- OPIM (instance-wise guarantee)
def test_opim_round_quantities_against_brute_force():
    """On a tiny graph: the upper bound U on R1 is at least the best k-subset's
    coverage of R1 (brute force over all k-subsets) and at least C_R1(S*);
    C_R2(S*) is the coverage of the returned seeds on the stream-1 half."""
    g = W.random_small_graph(14, 40, seed=71, p_hi=0.4)
    thr = O.ic_thresholds(g.weight)
    for k in (1, 2, 3):
        res = O.opim(O.IC, g.in_off, g.in_src, thr, k, 0.4, seed=8, fail=0.1, theta_cap=4096)
        th = res["theta"]
        r1 = O.sample(O.IC, g.in_off, g.in_src, thr, 8, 0, 0, th)
        r2 = O.sample(O.IC, g.in_off, g.in_src, thr, 8, 1, 0, th)
        io1, im1 = O.incidence(g.n, r1)
        io2, im2 = O.incidence(g.n, r2)
        best = max(O.coverage(g.n, th, io1, im1, list(S))
                   for S in itertools.combinations(range(g.n), k))
        assert res["cover1"] <= best <= res["upper1"]
        assert res["cover1"] == O.coverage(g.n, th, io1, im1, res["seeds"])
        assert res["cover2"] == O.coverage(g.n, th, io2, im2, res["seeds"])
        assert 2 * th >= 4096 or res["rounds"] == res["i_max"] or \
            res["guarantee"] >= 1 - 1 / math.e - 0.4


def test_opim_bounds_hold_against_exact_influence():
    """The lower bound on sigma(S*) and the upper bound on sigma(OPT) bracket
    the exact values (every live-edge world enumerated) in nearly every run;
    the bounds hold with probability 1 - fail per run (fail = 0.05 here)."""
    n = 6
    g = W.tiny_graph(n, TINY_EDGES, TINY_P)
    thr = O.ic_thresholds(g.weight)
    q = list(O.ic_thresholds(np.array(TINY_P, np.float32)).astype(np.float64) / 2.0 ** 32)
    k = 2
    sig = {S: _exact_sigma_ic(n, TINY_EDGES, q, list(S))
           for S in itertools.combinations(range(n), k)}
    opt = max(sig.values())
    bad_lo = bad_up = 0
    runs = 40
    for seed in range(runs):
        res = O.opim(O.IC, g.in_off, g.in_src, thr, k, 0.05, seed=100 + seed, fail=0.05,
                     theta_cap=1 << 16)
        S = tuple(sorted(int(x) for x in res["seeds"]))
        bad_lo += res["lower"] > sig[S] + 1e-9
        bad_up += res["upper"] < opt - 1e-9
        assert 0.5 < res["guarantee"] <= 1.0 + 1e-12  # the bounds are near (within 1/2)
    assert bad_lo <= 2 and bad_up <= 2, (bad_lo, bad_up)


def test_opim_schedule():
    """theta_0 = ceil(theta_max eps^2 k / n) and the rounds double it."""
    g = W.random_small_graph(500, 3000, seed=72, p_hi=0.2)
    thr = O.ic_thresholds(g.weight)
    res = O.opim(O.IC, g.in_off, g.in_src, thr, 5, 0.2, seed=9, fail=1 / 500,
                 theta_cap=1 << 30)
    t0 = math.ceil(res["theta_max"] * 0.2 * 0.2 * 5 / 500)
    assert res["theta"] == t0 * 2 ** (res["rounds"] - 1)
    assert res["i_max"] == max(1, math.ceil(math.log2(res["theta_max"] / t0)))
