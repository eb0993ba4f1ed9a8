"""The request scheduler on the host, with the fake executor (no GPU): a
request "runs" for footprint x ns_per_byte and keeps its footprint resident."""
import pytest

import paper_2303_05688_amd as asci


def _reqs(specs):
    return [asci.fake_request(*s) for s in specs]


MIX = [(20, 8, 8, 1000, 10_000)] * 14 + [(26, 10, 10, 10_000, 100_000)] * 5 + [(30, 12, 12, 100_000, 1_000_000)]


def test_footprint_grows_with_the_request():
    a, b, c = _reqs([(20, 8, 8, 1000, 10_000), (26, 10, 10, 10_000, 100_000), (30, 12, 12, 100_000, 1_000_000)])
    fa, fb, fc = asci.footprint(a), asci.footprint(b), asci.footprint(c)
    assert 0 < fa < fb < fc


def test_admission_never_exceeds_the_budget_and_overlaps():
    reqs = _reqs(MIX)
    budget = int(8e9)
    srv = asci.Server(hbm_budget=budget, slots=4, fake_ns_per_byte=1e-2)
    assert max(srv.footprint(r) for r in reqs) <= budget
    tickets = [srv.submit(r) for r in reqs]
    results = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert all(r.status == 0 for r in results)
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    assert st["peak_bytes"] <= budget
    assert st["max_running"] > 1
    assert 0 < st["p50_ms"] <= st["p99_ms"]


def test_budget_for_one_request_serialises():
    reqs = _reqs([(30, 12, 12, 100_000, 1_000_000)] * 4)
    budget = int(2.5e9)
    srv = asci.Server(hbm_budget=budget, slots=4, fake_ns_per_byte=5e-3)
    fp = srv.footprint(reqs[0])
    assert fp <= budget < 2 * fp
    for t in [srv.submit(r) for r in reqs]:
        assert srv.wait(t).status == 0
    st = srv.stats()
    srv.close()
    assert st["max_running"] == 1
    assert st["peak_bytes"] <= budget


def test_oversized_request_is_rejected_not_queued():
    big, small = _reqs([(30, 12, 12, 100_000, 1_000_000), (20, 8, 8, 1000, 10_000)])
    srv = asci.Server(hbm_budget=int(5e8), slots=2, fake_ns_per_byte=1e-3)
    assert srv.footprint(big) > 5e8 >= srv.footprint(small)
    tb, ts = srv.submit(big), srv.submit(small)
    assert srv.wait(tb).status == asci.ASCI_ENOMEM
    assert srv.wait(ts).status == 0
    st = srv.stats()
    srv.close()
    assert st["rejected"] == 1 and st["completed"] == 1


def test_poll_reports_pending_then_done():
    r = _reqs([(26, 10, 10, 10_000, 100_000)])[0]
    srv = asci.Server(hbm_budget=asci.footprint(r) * 2, slots=1, fake_ns_per_byte=3e-2)
    t = srv.submit(r)
    assert srv.poll(t) is None  # still running (about 50 ms)
    assert srv.wait(t).status == 0
    with pytest.raises(asci.AsciError):  # handed over once, then forgotten
        srv.poll(t)
    srv.close()


def test_fifo_admission_order():
    reqs = _reqs([(20, 8, 8, 1000, 10_000)] * 6)
    srv = asci.Server(hbm_budget=asci.footprint(reqs[0]) * 10, slots=1, fake_ns_per_byte=1e-3)
    ts = [srv.submit(r) for r in reqs]
    res = [srv.wait(t) for t in ts]
    srv.close()
    lat = [r.latency_ms for r in res]
    assert lat == sorted(lat)


def test_balance_equals_oracle(oracle_lib):
    """The library's Alg. 3 (heap arg-min) equals the oracle's linear scan."""
    import numpy as np

    rng = np.random.default_rng(3)
    for npe in (1, 2, 7, 64, 1000):
        counts = rng.integers(0, 50, 500) * (rng.random(500) < 0.7)
        counts[rng.integers(0, 500, 20)] = 7  # ties in the loads
        got_o, got_w = asci.balance_classes(counts, npe)
        want_o, want_w = oracle_lib.balance(counts, npe)
        assert (got_o == want_o).all() and (got_w == want_w).all()
    with pytest.raises(asci.AsciError):
        asci.balance_classes([1, -1], 2)


def test_class_skew_statistics():
    counts = [0, 10, 10, 10, 70]
    st = asci.class_skew(counts, npes=(1, 2, 4))
    assert st["classes"] == 4 and st["pairs"] == 100
    assert st["largest_share"] == 0.7
    assert st["imbalance"][1] == 1.0
    assert st["imbalance"][4] == 70 / 25


def test_invalid_request_rejected_at_submission():
    """A request whose options fail the search's argument checks (here a
    negative constraint level) is refused before anything is queued."""
    ok = asci.fake_request(20, 8, 8, 1000, 10_000)
    bad = asci.fake_request(20, 8, 8, 1000, 10_000)
    bad.opt.constraint_level = -1
    bad_n = asci.fake_request(70, 8, 8, 1000, 10_000)
    bad_k = asci.fake_request(20, 8, 8, 1000, 0)
    srv = asci.Server(hbm_budget=int(8e9), slots=2, fake_ns_per_byte=1e-3)
    for r in (bad, bad_n, bad_k):
        with pytest.raises(asci.AsciError) as e:
            srv.submit(r)
        assert e.value.code == asci.ASCI_EINVAL
    t = srv.submit(ok)
    assert srv.wait(t).status == 0
    st = srv.stats()
    srv.close()
    assert st["submitted"] == 1 and st["completed"] == 1


def test_results_are_handed_over_once():
    reqs = _reqs([(20, 8, 8, 1000, 10_000)] * 6)
    srv = asci.Server(hbm_budget=int(8e9), slots=2, fake_ns_per_byte=1e-3)
    tickets = [srv.submit(r) for r in reqs]
    for t in tickets:
        assert srv.wait(t).status == 0
    assert srv.stats()["held_results"] == 0
    with pytest.raises(asci.AsciError):
        srv.wait(tickets[0])
    with pytest.raises(asci.AsciError):
        srv.poll(tickets[1])
    srv.close()


def test_small_requests_pass_a_large_one_that_does_not_fit():
    """Budget for one large request: while it waits for room, small requests
    behind it start; with an age bound of 0 nothing passes the oldest."""
    big = (30, 12, 12, 100_000, 1_000_000)
    small = (20, 8, 8, 1000, 10_000)
    specs = [big, big] + [small] * 8

    def run(age_ms):
        reqs = _reqs(specs)
        srv = asci.Server(hbm_budget=int(3.2e9), slots=4, fake_ns_per_byte=5e-3)
        srv.set_param("age_ms", age_ms)
        fp_big, fp_small = srv.footprint(reqs[0]), srv.footprint(reqs[2])
        assert fp_big + fp_small <= 3.2e9 < 2 * fp_big
        tickets = [srv.submit(r) for r in reqs]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
        srv.close()
        assert all(r.status == 0 for r in res)
        assert st["peak_bytes"] <= 3.2e9
        return res, st

    res, st = run(1e6)
    assert st["bypassed"] >= 1
    # small requests run while the second large one waits for room
    assert min(r.latency_ms for r in res[2:]) < res[0].latency_ms
    res0, st0 = run(0.0)
    assert st0["bypassed"] == 0
    # without passing, every small request waits until the first large one is done
    assert min(r.latency_ms for r in res0[2:]) > res0[0].latency_ms
    mean = lambda rs: sum(r.latency_ms for r in rs) / len(rs)  # noqa: E731
    assert mean(res[2:]) < mean(res0[2:])
    with pytest.raises(asci.AsciError):
        asci.Server(hbm_budget=int(1e9), slots=1, fake_ns_per_byte=1e-3).set_param("age_ms", -1.0)


def test_tuning_table_record_save_load(tmp_path):
    """The per-shape tuning table (host only): record, look up by the bucket of
    the pair count, save, clear, load; malformed files are refused."""
    asci.tune_clear()
    # device 0's entries are keyed by its architecture ("unknown" without a
    # device); a recorded entry is found for every pair count in the same
    # power-of-two bucket, and not for another architecture
    arch = asci.tune_arch(0)
    assert arch in ("unknown", "gfx950")
    other = "gfx942" if arch != "gfx942" else "gfx950"
    asci.tune_record(arch, 20, 8, 26, 2048)
    assert asci.tune_lookup(0, 20, 8, 1 << 26) == 2048
    assert asci.tune_lookup(0, 20, 8, (1 << 27) - 1) == 2048
    assert asci.tune_lookup(0, 20, 8, 1 << 27) == 0
    asci.tune_record(other, 30, 12, 32, 4096)
    assert asci.tune_lookup(0, 30, 12, 1 << 32) == 0
    path = tmp_path / "tune.txt"
    asci.tune_save(path)
    lines = sorted(open(path).read().split("\n")[:-1])
    assert lines == sorted(["%s 30 12 32 4096" % other, "%s 20 8 26 2048" % arch])
    asci.tune_clear()
    assert asci.tune_lookup(0, 20, 8, 1 << 26) == 0
    assert asci.tune_load(path) == 2
    assert asci.tune_lookup(0, 20, 8, 1 << 26) == 2048
    bad = tmp_path / "bad.txt"
    bad.write_text("gfx950 30 12 32 3000\n")
    with pytest.raises(asci.AsciError):
        asci.tune_load(bad)
    with pytest.raises(asci.AsciError):
        asci.tune_record("gfx950", 30, 12, 70, 4096)
    asci.tune_clear()


def test_one_slot_pool_fits_large_requests_into_its_budget():
    """With one slot the pair buffer alone may take most of the budget; the
    rest of the workspace (class x core matrix, spin tables, candidate pool)
    does not shrink with it, so the pool shrinks the pair buffer until the
    whole request fits instead of refusing it."""
    reqs = _reqs([(30, 12, 12, 100_000, 1_000_000), (40, 11, 11, 61_089, 610_890)])
    for budget in (20e9, 40e9, 160e9):
        srv = asci.Server(hbm_budget=int(budget), slots=1, fake_ns_per_byte=1e-9)
        try:
            assert all(srv.footprint(r) <= budget for r in reqs)
            assert all(srv.wait(srv.submit(r)).status == 0 for r in reqs)
        finally:
            srv.close()
