"""Scheduler of the serving runtime on a CPU: the simulated executor stands in
for the GPU (nothing is launched), so admission, ordering, budget, draining
and statistics are checked without a device."""
import time

import pytest

import paper_2602_10262_amd as lib


@pytest.fixture(scope="module")
def L():
    return lib.load()


def _server(budget=1 << 30, streams=4, max_inflight=0, rate=1000.0, launch_us=10.0):
    return lib.Server(budget, streams, max_inflight, simulated=True, gflop_per_ms=rate, launch_us=launch_us)


def test_requests_complete_and_latency_counts_from_arrival(L):
    s = _server(rate=0.1, launch_us=0.0)
    w = s.register_weight(None, None, None, 1024, 1024)
    t0 = s.now()
    # 2*64*1024*1024 FLOP = 0.134 GFLOP at 0.1 GFLOP/ms = 1.34 ms each
    tickets = [s.submit(64, w, arrival_time_s=t0 + 0.01) for _ in range(8)]
    for t in tickets:
        assert s.wait(t, 5_000_000) == lib.FP8_OK
    lat = [s.latency_ms(t) for t in tickets]
    assert min(lat) >= 1.3
    st = s.stats()
    assert st["done"] == 8 and st["failed"] == 0
    # 8 jobs on 4 streams: two rounds of 1.34 ms
    assert 2.6 <= max(lat) < 50
    s.close()


def test_budget_rejects_oversized_and_limits_concurrency(L):
    # one 64 x 1024 request needs 64 KiB of codes + 2 x 256 B of scales
    per = 64 * 1024 + 2 * 256
    s = _server(budget=2 * per + 1024, streams=4, rate=50.0, launch_us=0.0)
    w = s.register_weight(None, None, None, 1024, 1024)
    with pytest.raises(lib.Fp8Error) as e:
        s.submit(4096, w)
    assert e.value.status == 7  # FP8_ERR_BUDGET
    tickets = [s.submit(64, w) for _ in range(10)]
    for t in tickets:
        assert s.wait(t, 10_000_000) == lib.FP8_OK
    st = s.stats()
    assert st["peak_inflight"] <= 2, st
    assert st["peak_bytes"] <= 2 * per + 1024
    assert st["rejected"] == 1 and st["done"] == 10
    s.close()


def test_fifo_admission_order_single_slot(L):
    s = _server(streams=1, max_inflight=1, rate=200.0, launch_us=0.0)
    w = s.register_weight(None, None, None, 512, 512)
    base = s.now() + 0.005
    order = [3, 0, 2, 1]
    tickets = {i: s.submit(32, w, arrival_time_s=base + 0.001 * i) for i in order}
    for t in tickets.values():
        s.wait(t, 5_000_000)
    lat = {i: s.latency_ms(tickets[i]) for i in order}
    # completion = arrival + latency must follow arrival order on one slot
    done_at = sorted(range(4), key=lambda i: base * 1e3 + 1.0 * i + lat[i])
    assert done_at == [0, 1, 2, 3]
    s.close()


def test_continuous_admission_while_busy(L):
    """Requests that arrive while others run start before those finish."""
    s = _server(streams=4, rate=0.02, launch_us=0.0)
    w = s.register_weight(None, None, None, 2048, 2048)
    t_long = s.submit(512, w)                    # 4.3 GFLOP: ~0.2 s on one stream
    time.sleep(0.02)
    short = [s.submit(16, w) for _ in range(3)]  # ~7 ms each, arriving while it runs
    for t in short:
        s.wait(t, 5_000_000)
    assert s.poll(t_long) == lib.FP8_ERR_PENDING
    s.wait(t_long, 5_000_000)
    s.close()


def test_drain_and_destroy_with_work_in_flight(L):
    s = _server(streams=2, rate=100.0, launch_us=50.0)
    w = s.register_weight(None, None, None, 1024, 1024)
    tickets = [s.submit(64, w, arrival_time_s=s.now() + 0.002 * i) for i in range(20)]
    s.drain()
    assert all(s.poll(t) == lib.FP8_OK for t in tickets)
    more = [s.submit(64, w) for _ in range(5)]
    s.close()   # drains first
    assert more


def test_wait_timeout_and_bad_arguments(L):
    s = _server(streams=1, rate=1.0, launch_us=0.0)
    w = s.register_weight(None, None, None, 4096, 4096)
    t = s.submit(256, w)       # 8.6 GFLOP at 1 GFLOP/ms: ~8.6 ms
    assert s.wait(t, 100) == lib.FP8_ERR_TIMEOUT
    with pytest.raises(lib.Fp8Error):
        s.submit(0, w)
    with pytest.raises(lib.Fp8Error):
        s.submit(16, 99)
    assert s.wait(t, 5_000_000) == lib.FP8_OK
    s.close()


def test_percentiles_and_fairness_statistics(L):
    s = _server(streams=2, rate=100.0, launch_us=0.0)
    w = s.register_weight(None, None, None, 1024, 1024)
    base = s.now() + 0.005
    tickets = [s.submit(64, w, arrival_time_s=base + 0.004 * i) for i in range(50)]
    for t in tickets:
        s.wait(t, 5_000_000)
    lat = sorted(s.latency_ms(t) for t in tickets)
    st = s.stats()
    # nearest rank: p50 = L[ceil(0.5 n) - 1], p99 = L[ceil(0.99 n) - 1]
    assert st["p50_ms"] == pytest.approx(lat[24])
    assert st["p99_ms"] == pytest.approx(lat[49])
    assert 0.0 <= st["fairness_minmax"] <= 1.0 and st["fairness_range"] <= 1.0
    assert st["tflops"] > 0
    s.reset_stats()
    assert s.stats()["done"] == 0
    s.close()
