"""Host-side admission logic of the request loop (no GPU)."""
import collections

import numpy as np
import pytest


def _req(serve, rid, n, nnz):
    r = serve.Request(rid, np.zeros(n + 1, np.int32), np.zeros(nnz, np.int32), 0.0)
    r.n, r.nnz = n, nnz
    return r


def test_ledger_and_fifo_admission():
    from paper_1505_04086_amd import serve
    led = serve.BudgetLedger(25_000)
    q = collections.deque([_req(serve, 0, 100, 400), _req(serve, 1, 1000, 4000), _req(serve, 2, 10, 10)])
    got = []
    for r, nb in serve.admit_fifo(q, led):
        led.take(nb)
        got.append(r.rid)
    assert len(q) == 2
    # request 1 needs 4*1001+4*4000+4*1000 = 24004 bytes: it fits alone but not next to request 0,
    # so it blocks request 2 behind it (arrival order is kept)
    assert got == [0] and [r.rid for r in q] == [1, 2]
    assert led.used == serve.csr_bytes(100, 400)
    led.give(serve.csr_bytes(100, 400))
    assert led.used == 0
    big = serve.BudgetLedger(10**9)
    got = [r.rid for r, nb in serve.admit_fifo(q, big)]
    assert got == [1, 2] and not q
    with pytest.raises(RuntimeError):
        serve.BudgetLedger(10).take(11)
    # a request that can never fit is rejected instead of blocking the queue
    q = collections.deque([_req(serve, 5, 10**6, 10**7), _req(serve, 6, 10, 10)])
    small = serve.BudgetLedger(10_000)
    out = [(r.rid, nb) for r, nb in serve.admit_fifo(q, small)]
    assert out[0] == (5, -1) and out[1][0] == 6 and out[1][1] > 0
    q = collections.deque([_req(serve, 7, 5000, 10)])
    out = [(r.rid, nb) for r, nb in serve.admit_fifo(q, serve.BudgetLedger(10**9), scratch_cap=1000)]
    assert out == [(7, -1)]


def test_slot_scratch_matches_library_formula():
    from paper_1505_04086_amd import serve
    # 4 worklist-sized arrays (two worklists, two hub lists) + byte shadow, then
    # the 4-bit shadow and round 0's kept neighbours (optimistic) or the
    # staged colours, each 256-byte aligned
    assert serve.slot_scratch_bytes(1000, False) == 4 * 4096 + 1280 + 512 + 16128
    assert serve.slot_scratch_bytes(1000, True) == 5 * 4096 + 1280


def test_latency_summary():
    from paper_1505_04086_amd import serve
    reqs = []
    for i in range(100):
        r = serve.Request(i, None, None, arrival=0.0)
        r.done = (i + 1) / 1000.0
        reqs.append(r)
    s = serve.latency_summary(reqs)
    assert abs(s["p50_ms"] - 50.5) < 1e-6 and 99 < s["p99_ms"] <= 100
