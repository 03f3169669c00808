"""The no-allocation greedy (im_greedy_cover_static) against the allocating
entry point (im_greedy_cover), through the C ABI.

Two calls in a row on the shared fixed buffer, the second on a smaller graph
with fewer samples and picks, each compared element by element with
im_greedy_cover on the same inputs (seeds, gains, nsel, coverage) and with
the CPU oracle; and a size beyond the fixed buffer is refused with IM_ENOMEM
before any device work.
"""
import ctypes as C

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


def _compare(im, g, count, k, seed):
    print("[case] static greedy n=%d count=%d k=%d" % (g.n, count, k), flush=True)
    G = im.prepare_graph(g.in_off, g.in_src, g.weight, g.model)
    r = im.sample_rrr(G, seed, 0, 0, count)
    io, imem = im.build_incidence(g.n, r)
    a = im.greedy_cover(g.n, r, io, imem, k)
    b = im.greedy_cover_static(g.n, r, io, imem, k)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    o = O.sample(g.model, g.in_off, g.in_src, O.thresholds(g.model, g.in_off, g.weight), seed, 0,
                 0, count)
    oio, oim = O.incidence(g.n, o)
    os_, og, oc = O.greedy(g.n, count, oio, oim, k)
    ns = int(b[2].item())
    assert b[0][:ns].cpu().numpy().tolist() == os_.tolist()
    assert b[1][:ns].cpu().numpy().tolist() == og.tolist()
    assert int(b[3].item()) == oc


def test_static_greedy_two_calls_second_smaller(im):
    big = W.make_graph("rmat", W.IC, scale=14, num_edges=1 << 18, graph_seed=77, weight_seed=78,
                       weights="wc")
    _compare(im, big, 20000, 30, 5)
    small = W.random_small_graph(500, 2000, seed=1, p_hi=0.1)
    _compare(im, small, 3000, 8, 6)


def test_static_greedy_refuses_more_than_its_buffer(im):
    print("[case] static greedy oversize", flush=True)
    L = im.lib()
    dev = torch.empty(8, dtype=torch.int64, device="cuda")
    p = C.c_void_p(dev.data_ptr())
    n = 1 << 24  # 4n bytes of counts alone fill the 64 MiB buffer
    st = L.im_greedy_cover_static(n, 1, p, p, 0, p, p, 4, p, p, p, p,
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == im.binding.IM_ENOMEM
    assert b"64" in L.im_last_error() or b"67108864" in L.im_last_error()
