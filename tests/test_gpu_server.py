"""GPU tests of the serving loop (continuous batching of arriving codes),
under both engines: worker threads running the single-code path side by
side (engine 0) and the persistent multi-code kernel, which admits arriving
codes while it runs (engine 1).

Each request's result in the mix must be exactly its result alone (d, the
visited pairs, their bounds, counts and minima), with a valid witness; codes
that arrive while others run are admitted without waiting for them to end.
"""
import time

import numpy as np
import pytest

import paper_1603_06757_amd as md
from paper_1603_06757_amd.gen import WORKLOADS, serving_request
from tests.test_gpu_batch import light_codes, same_as_single
from tests.test_gpu_parity import check_witness

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def collect(srv, count, timeout=120.0):
    got = {}
    t_end = time.time() + timeout
    while len(got) < count:
        for r in srv.poll():
            got[r["tag"]] = r
        assert time.time() < t_end, f"only {len(got)} of {count} results"
        time.sleep(0.002)
    return got


@pytest.mark.parametrize("engine", [0, 1])
def test_server_results_equal_alone_with_staggered_arrivals(engine):
    cs = light_codes(48, seed=91)
    say("server: 48 light codes in 4 waves of arrivals, 16 slots, engine", engine)
    with md.Server(max_active=16, engine=engine) as srv:
        for i, (n, k, G) in enumerate(cs):
            srv.submit(G, n, k, tag=i)
            if i % 12 == 11:
                time.sleep(0.003)
        got = collect(srv, len(cs))
        st = srv.stats()
    assert st["completed"] == len(cs) and st["admitted"] == len(cs)
    for i, (n, k, G) in enumerate(cs):
        r = got[i]
        assert r["status"] == 0, (i, r["status"])
        s = md.min_distance(G, n, k)
        same_as_single(r, s)
        check_witness(G, n, k, r)
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]


@pytest.mark.parametrize("engine", [0, 1])
def test_server_admits_while_others_run(engine):
    """A heavier code is submitted first; light codes submitted while it runs
    are admitted into free slots after it started and finish before it ends
    (their work overlaps on the device), and every result equals the code's
    result alone."""
    # the seeded [255,40] code: 78 pairs, 13-16 ms alone, long enough for the
    # light codes to arrive while it runs under either engine
    w = WORKLOADS["rand255x40"]
    heavy = (w.n, w.k, w.matrix())
    light = light_codes(24, seed=92)
    say("server: heavy", heavy[:2], "then 24 light codes while it runs, engine", engine)
    # engine 1 without routing: the heavier code in the persistent kernel too
    route = {"route_log2": -1} if engine == 1 else {}
    with md.Server(max_active=8, engine=engine, **route) as srv:
        srv.submit(heavy[2], heavy[0], heavy[1], tag=1000)
        time.sleep(0.001)
        for i, (n, k, G) in enumerate(light):
            srv.submit(G, n, k, tag=i)
        got = collect(srv, len(light) + 1)
        st = srv.stats()
    h = got[1000]
    assert h["status"] == 0
    same_as_single(h, md.min_distance(heavy[2], heavy[0], heavy[1]))
    check_witness(heavy[2], heavy[0], heavy[1], h)
    say("heavy admitted", h["t_admit"], "done", h["t_done"], "stats", st)
    say("light (admit, done):", [(round(got[i]["t_admit"], 4), round(got[i]["t_done"], 4))
                                 for i in range(len(light))])
    overlap = [h["t_admit"] < got[i]["t_admit"] and got[i]["t_done"] < h["t_done"]
               for i in range(len(light))]
    assert sum(overlap) >= 7, "no light code ran while the heavy one was on the device"
    if engine == 1:
        # the light codes come into the running launch (7 free slots), the
        # rest after a relaunch frees the slots the first ones used
        assert st["admitted_live"] >= 7, st
    for i, (n, k, G) in enumerate(light):
        assert got[i]["status"] == 0
        same_as_single(got[i], md.min_distance(G, n, k))


@pytest.mark.parametrize("engine", [0, 1])
def test_server_admission_by_device_memory(engine):
    """A small device budget keeps few codes in flight at once; every code
    still completes with the result it has alone, and a code whose share
    exceeds the whole budget is refused at submit."""
    cs = [serving_request(i) for i in range(40)]
    cs = [(n, k, G) for n, k, G in cs if n <= 120][:16]
    # engine 1 without routing: every code goes to its device pool
    route = {"route_log2": -1} if engine == 1 else {}
    with md.Server(max_active=4, device_bytes=1024, engine=engine, **route) as srv:
        with pytest.raises(md.MindistError) as e:
            srv.submit(cs[0][2], cs[0][0], cs[0][1], tag=0)
        assert e.value.code == -3
    # 48 MiB: the largest of these codes needs about 29 MiB (engine 0's
    # estimate), so only a few are in flight at once
    say("server: 16 serving-stream codes, 48 MiB of device memory, engine", engine)
    with md.Server(max_active=64, device_bytes=48 << 20, engine=engine, **route) as srv:
        for i, (n, k, G) in enumerate(cs):
            srv.submit(G, n, k, tag=i)
        got = collect(srv, len(cs), timeout=300)
    for i, (n, k, G) in enumerate(cs):
        assert got[i]["status"] == 0
        same_as_single(got[i], md.min_distance(G, n, k))


@pytest.mark.parametrize("engine", [0, 1])
def test_server_submit_errors_and_wait(engine):
    with md.Server(max_active=4, engine=engine) as srv:
        G = np.zeros((3, 1), dtype=np.uint64)
        G[0, 0] = 0b0011
        G[1, 0] = 0b0110
        G[2, 0] = 0b0101           # row 2 = row 0 + row 1: rank 2 < k = 3
        with pytest.raises(md.MindistError) as e:
            srv.submit(G, 4, 3, tag=1)
        assert e.value.code == -2
        n, k, G = light_codes(1, seed=93)[0]
        srv.submit(G, n, k, tag=7)
        srv.wait(60.0)
        got = srv.poll()
        assert [r["tag"] for r in got] == [7] and got[0]["status"] == 0
        assert srv.poll() == []


@pytest.mark.parametrize("engine", [0, 1])
def test_server_destroy_with_waiting_codes(engine):
    """Destroying a server with a long queue returns promptly: waiting codes
    are dropped, the ones being run finish or stop first."""
    cs = light_codes(120, seed=97)
    srv = md.Server(max_active=2, engine=engine)
    for i, (n, k, G) in enumerate(cs):
        srv.submit(G, n, k, tag=i)
    t0 = time.time()
    srv.close()
    say("destroy with", len(cs), "queued codes took", round(time.time() - t0, 3), "s, engine", engine)
    assert time.time() - t0 < 10.0


@pytest.mark.parametrize("engine", [0, 1])
def test_served_results_equal_the_oracle(engine):
    """Every served result against the CPU oracle, not only against the
    single path: d, the whole visited-pair trace (sets, levels, bounds
    before and after, U after, pair minima, C(k,w) counts) and a valid
    witness, for light random codes and oracle-cheap requests of the
    serving stream, arriving in waves while earlier ones run."""
    import oracle
    from paper_1603_06757_amd.gen import serving_request
    from tests.test_gpu_parity import compare_with_trace, oracle_tables, estimated_work
    cs = light_codes(40, seed=95)
    cs += [c for c in (serving_request(i) for i in range(400))
           if estimated_work(c[0], c[1]) <= 2e7][:24]
    say("server vs oracle:", len(cs), "codes, engine", engine)
    with md.Server(max_active=12, engine=engine) as srv:
        for i, (n, k, G) in enumerate(cs):
            srv.submit(G, n, k, tag=i)
            if i % 16 == 15:
                time.sleep(0.002)
        got = collect(srv, len(cs), timeout=300)
    for i, (n, k, G) in enumerate(cs):
        r = got[i]
        assert r["status"] == 0, (i, r["status"])
        ref = oracle.bz(G, n, k, threads=4)
        assert r["d"] == ref["d"], (i, n, k)
        assert (r["m_full"], r["k_partial"]) == (ref["m_full"], ref["k_m"])
        counts, pmin, _ = oracle_tables(ref)
        compare_with_trace(r, ref["trace"].tolist(), counts, pmin, None, k)
        assert all(p["executed"] == p["count"] for p in r["pairs"][:-1])
        check_witness(G, n, k, r)


def test_engine1_admission_under_slot_and_memory_pressure():
    """Engine 1 with 3 slots and a small device pool, a longer code first and
    30 light codes arriving in bursts: codes come into the running launch
    while slots and pool ranges are fresh, and the launch is stopped and
    restarted when only a relaunch frees them (slots and ranges serve one
    code per launch).  Every result equals the code's result alone and the
    oracle's, with a valid witness."""
    import oracle
    from tests.test_gpu_parity import compare_with_trace, oracle_tables
    w = WORKLOADS["rand255x40"]
    first = (w.n, w.k, w.matrix())
    light = light_codes(30, seed=98)
    say("engine 1 pressure: 3 slots, 24 MiB pool, [255,40] then 30 light codes in bursts")
    with md.Server(max_active=3, device_bytes=24 << 20, engine=1, epoch_min_ms=0.05, route_log2=-1) as srv:
        srv.submit(first[2], first[0], first[1], tag=1000)
        time.sleep(0.002)
        for i, (n, k, G) in enumerate(light):
            srv.submit(G, n, k, tag=i)
            if i % 5 == 4:
                time.sleep(0.001)
        got = collect(srv, len(light) + 1, timeout=300)
        st = srv.stats()
    say("stats", st)
    assert st["completed"] == len(light) + 1
    assert st["admitted_live"] >= 2, st
    assert st["epochs"] >= 2, st
    h = got[1000]
    assert h["status"] == 0
    same_as_single(h, md.min_distance(first[2], first[0], first[1]))
    check_witness(first[2], first[0], first[1], h)
    for i, (n, k, G) in enumerate(light):
        r = got[i]
        assert r["status"] == 0, (i, r["status"])
        ref = oracle.bz(G, n, k, threads=4)
        assert r["d"] == ref["d"], (i, n, k)
        counts, pmin, _ = oracle_tables(ref)
        compare_with_trace(r, ref["trace"].tolist(), counts, pmin, None, k)
        check_witness(G, n, k, r)


def test_engine1_routes_heavier_codes_to_the_single_path():
    """Engine 1 with its default routing: light codes run in the persistent
    kernel (2 blocks per CU), codes expected at 2^24 combinations or more on
    single-path workers beside it, at the same time; every result equals
    the code's result alone."""
    from tests.test_gpu_parity import estimated_work
    cs = [serving_request(i) for i in range(120)]
    cs = [c for c in cs if estimated_work(c[0], c[1]) <= 2e10][:40]
    say("engine 1 routing: 40 serving-stream codes")
    with md.Server(engine=1) as srv:
        for i, (n, k, G) in enumerate(cs):
            srv.submit(G, n, k, tag=i)
            if i % 8 == 7:
                time.sleep(0.002)
        got = collect(srv, len(cs), timeout=300)
        st = srv.stats()
    say("stats", st)
    assert st["completed"] == len(cs)
    assert 0 < st["routed"] < len(cs), st
    for i, (n, k, G) in enumerate(cs):
        assert got[i]["status"] == 0
        same_as_single(got[i], md.min_distance(G, n, k))
        check_witness(G, n, k, got[i])


def test_engine1_code_beyond_the_kernel_layout():
    """A code with more than 32 information sets is beyond the persistent
    kernel's layout: engine 1 routes it to the single path (its result
    equals the single path's and the oracle's d); without routing, submit
    refuses it with MINDIST_E_LIMIT."""
    import oracle
    from paper_1603_06757_amd.gen import random_generator
    G = random_generator(200, 3, 1, 2)
    ref = oracle.bz(G, 200, 3)
    say("engine 1: [200,3] code, 66 information sets")
    with md.Server(engine=1) as srv:
        srv.submit(G, 200, 3, tag=5)
        got = collect(srv, 1)
        st = srv.stats()
    assert st["routed"] == 1
    r = got[5]
    assert r["status"] == 0 and r["d"] == ref["d"]
    same_as_single(r, md.min_distance(G, 200, 3))
    check_witness(G, 200, 3, r)
    with md.Server(engine=1, route_log2=-1) as srv:
        with pytest.raises(md.MindistError) as e:
            srv.submit(G, 200, 3, tag=6)
        assert e.value.code == -5
