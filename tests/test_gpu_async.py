"""The search with nothing read back (asci_search_async): every count stays on
the device, so the call returns once the work is queued.  Its results equal
asci_search_device's bit for bit and the oracle's under the score tolerance;
two searches queued on two streams overlap on the device; failures found on
the device come back in the result record with no output written."""
import time

import numpy as np
import pytest

import asci_synth as syn
from gpu_util import assert_topk, host, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def asci():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_05688_amd as pkg

    return pkg


def _req(asci, c, E0, k, **kw):
    d = to_dev(c)
    return asci.SearchRequest(d["h"], d["eri"], c["norb"], c["nalpha"], c["nbeta"], d["dets"], d["coeffs"], E0, k,
                              **kw), d


def _async(asci, req, ctx=None, stream=None):
    import torch

    res = asci.search_async(req, ctx=ctx, stream=stream)
    torch.cuda.synchronize()
    count, status, flags = asci.async_status(res)
    return count, status, flags


CASES = [("8e12o", 2000, {}), ("8e12o", 10 ** 7, {}), ("8e12o", 500, {"ncore": 50}), ("8e12o", 700, {"eps": 1e-4}),
         ((9, 5, 4, 60), 300, {}), ((34, 3, 2, 12), 100, {}), ((36, 8, 8, 60), 5000, {}), ((6, 0, 3, 6), 50, {}),
         ((12, 6, 6, 150), 3000, {"constraint_level": 5})]


@pytest.mark.parametrize("case,k,kw", CASES)
def test_async_equals_device_search_and_oracle(asci, oracle_lib, case, k, kw):
    if case == "8e12o":
        c = syn.workload("8e12o")
    else:
        n, na, nb, nd = case
        c = syn.make_case(n, na, nb, nd, 400 + n + nd, sampler="level", tau=max(nd / 10.0, 1.0))
    n, na, nb = c["norb"], c["nalpha"], c["nbeta"]
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    print("async case n=%d na=%d nb=%d nd=%d k=%d %s" % (n, na, nb, len(c["coeffs"]), k, kw), flush=True)
    req, d = _req(asci, c, E0, k, **kw)
    count, status, flags = _async(asci, req)
    assert status == 0 and flags == 0
    gk, gs = (host(t) for t in req.result(count))
    skw = {x: kw[x] for x in kw}
    rk, rs = asci.search(d["h"], d["eri"], n, na, nb, d["dets"], d["coeffs"], E0, k, **skw)
    rk, rs = host(rk), host(rs)
    assert count == len(rk)
    assert (gk == rk).all() and (gs == rs).all()
    want = oracle_lib.search_all(c["h"], c["eri"], n, na, nb, c["dets"], c["coeffs"], E0, ncore=kw.get("ncore", 0),
                                 eps=kw.get("eps", 0.0))
    assert_topk(gk, gs, want, k)
    # a second call on the same context reuses its workspace
    count2, status2, _ = _async(asci, req)
    assert status2 == 0 and count2 == count
    assert (host(req.result(count2)[0]) == rk).all()


def test_async_full_size_16e20o(asci, oracle_lib):
    """The (16e,20o) workload (1.3e8 pairs in one class batch): the same bits as
    the synchronous search, and the call returns long before the work ends."""
    import torch

    c = syn.workload("16e20o")
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"][:2000], c["coeffs"][:2000])
    req, d = _req(asci, c, E0, c["k"])
    count, status, flags = _async(asci, req)  # sizes the context's workspace
    assert status == 0, flags
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = asci.search_async(req)
    t_call = time.perf_counter() - t0
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    count, status, flags = asci.async_status(res)
    print("16e20o async: call %.3f ms, work %.3f ms" % (t_call * 1e3, t_all * 1e3))
    assert status == 0 and count == c["k"]
    assert t_call < 0.5 * t_all
    gk, gs = (host(t) for t in req.result(count))
    rk, rs = asci.search(d["h"], d["eri"], 20, 8, 8, d["dets"], d["coeffs"], E0, c["k"])
    assert (gk == host(rk)).all() and (gs == host(rs)).all()


def test_two_streams_overlap(asci, oracle_lib):
    """Two searches on two contexts and two streams, queued back to back with
    no host wait: each equals its synchronous result, and their event
    intervals on the device overlap."""
    import torch

    cs = [syn.make_case(18, 7, 7, 3000, 81, sampler="level", tau=300.0),
          syn.make_case(18, 7, 7, 3000, 82, sampler="level", tau=300.0)]
    E0s = [oracle_lib.energy(c["h"], c["eri"], c["dets"][:500], c["coeffs"][:500]) for c in cs]
    reqs = [_req(asci, c, e, 20000) for c, e in zip(cs, E0s)]
    ctxs = [asci.Context(0), asci.Context(0)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    # warm-up: workspaces sized
    for (rq, _), cx, st in zip(reqs, ctxs, streams):
        asci.search_async(rq, ctx=cx, stream=st)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(2)]
    ref = torch.cuda.Event(enable_timing=True)
    ref.record()
    torch.cuda.synchronize()
    results = []
    for i, ((rq, _), cx, st) in enumerate(zip(reqs, ctxs, streams)):
        ev[i][0].record(st)
        results.append(asci.search_async(rq, ctx=cx, stream=st))
        ev[i][1].record(st)
    torch.cuda.synchronize()
    span = [(ref.elapsed_time(a), ref.elapsed_time(b)) for a, b in ev]
    print("stream intervals (ms):", span)
    assert span[1][0] < span[0][1] and span[0][0] < span[1][1], "no overlap"
    for (rq, d), c, e, res in zip(reqs, cs, E0s, results):
        count, status, _ = asci.async_status(res)
        assert status == 0
        gk, gs = (host(t) for t in rq.result(count))
        rk, rs = asci.search(d["h"], d["eri"], 18, 7, 7, d["dets"], d["coeffs"], e, 20000)
        assert (gk == host(rk)).all() and (gs == host(rs)).all()
    for cx in ctxs:
        cx.close()


def test_async_failures_reported_on_the_device(asci, oracle_lib):
    import torch

    c = syn.make_case(8, 4, 3, 40, 5, sampler="uniform", tau=8.0)
    E0 = oracle_lib.energy(c["h"], c["eri"], c["dets"], c["coeffs"])
    d = to_dev(c)
    # an input determinant repeated: found on the device, nothing written
    dup = d["dets"].clone().view(torch.int64)
    dup[3] = dup[1]
    req = asci.SearchRequest(d["h"], d["eri"], 8, 4, 3, dup.view(torch.uint64), d["coeffs"], E0, 50)
    req.out_scores.fill_(7.0)
    count, status, flags = _async(asci, req)
    assert status == asci.ASCI_EINVAL and count == 0 and flags & 2
    assert (host(req.out_scores) == 7.0).all()
    # a wrong electron count
    bad = d["dets"].clone().view(torch.int64)
    bad[2, 0] = 0b11111
    req = asci.SearchRequest(d["h"], d["eri"], 8, 4, 3, bad.view(torch.uint64), d["coeffs"], E0, 50)
    count, status, flags = _async(asci, req)
    assert status == asci.ASCI_EINVAL and flags & 1
    # integrals without the 8-fold symmetry (one entry changed alone)
    asym = d["eri"].clone()
    asym.view(-1)[((1 * 8 + 2) * 8 + 3) * 8 + 5] += 1e-3
    req = asci.SearchRequest(d["h"], asym, 8, 4, 3, d["dets"], d["coeffs"], E0, 50)
    count, status, flags = _async(asci, req)
    assert status == asci.ASCI_EINVAL and count == 0 and flags & 32
    # the forced fault of the error-path test
    ctx = asci.Context.get(0)
    req = asci.SearchRequest(d["h"], d["eri"], 8, 4, 3, d["dets"], d["coeffs"], E0, 50)
    try:
        ctx.set_param("fault_test", 1)
        count, status, flags = _async(asci, req, ctx=ctx)
        assert status == asci.ASCI_EDEVICE and count == 0
    finally:
        ctx.set_param("fault_test", 0)
    count, status, flags = _async(asci, req, ctx=ctx)
    assert status == 0 and count == 50
    # outside the one-batch scope: refused at once
    big = asci.SearchRequest(d["h"], d["eri"], 8, 4, 3, d["dets"], d["coeffs"], E0, 50, split_pairs=100)
    with pytest.raises(asci.AsciError) as e:
        asci.search_async(big)
    assert e.value.code == asci.ASCI_EINVAL
