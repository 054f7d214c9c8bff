"""GPU tests of the serving loop through the C ABI.

Small case: the oracle-signed multi-signer jobs (uneven sizes, an empty job,
variable-length messages, seeded flips, a tampered tag) submitted as
requests, half with host buffers (staged by the server) and half with
device buffers.  Each request's verdict and invalid list must equal the
oracle's, both when every request is served alone and when all are
submitted at once into small groups on several streams; each key's
device-resident aggregate state must equal the oracle's Agg over the tags
of its accepted requests.  Load case: requests over 64 device-signed keys
with log-uniform sizes, random flips and a device budget small enough that
admission throttles; every result must equal what its flips fix, and the
budget must be released at the end."""

import random
import threading
import time

import numpy as np
import pytest

from multi_signer_cases import L1, L2, corrupted_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu(P):
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    ctx = P.poslo_ctx_create(0)
    yield torch, ctx
    ctx.close()


def collect(srv, tickets, timeout_s=120):
    """Results of the given tickets: ticket -> (status, accept, invalid list)."""
    want = set(tickets)
    out = {}
    t_end = time.time() + timeout_s
    while want - set(out):
        assert time.time() < t_end, "server results timed out"
        for r in srv.poll(256, timeout_ms=50):
            inv = srv.take_invalid(r.ticket, r.n_invalid) if r.n_invalid else []
            out[r.ticket] = (r.status, bool(r.accept), inv, r.user)
    return out


def make_requests(P, torch, jobs, data, off, sigs):
    reqs = []
    off = np.asarray(off, dtype=np.uint64)
    for k, j in enumerate(jobs):
        b, n = j["entry_base"], j["n"]
        o = (off[b:b + n + 1] - off[b]).astype(np.uint64)
        m = np.frombuffer(data, dtype=np.uint8)[int(off[b]):int(off[b + n])].copy()
        sg = np.frombuffer(sigs, dtype=np.uint8)[80 * b:80 * (b + n)].copy()
        if k % 2:  # device buffers
            dm = torch.from_numpy(m).cuda()
            do = torch.from_numpy(o.view(np.int64)).cuda()
            ds_ = torch.from_numpy(sg).cuda()
            reqs.append(P.Request(j["key"], j["t0"], n, dm, do, 0, ds_, j["ds"], j["tag"], user=k))
        else:
            reqs.append(P.Request(j["key"], j["t0"], n, m, o, 0, sg, j["ds"], j["tag"], user=k))
    return reqs


@pytest.mark.parametrize("inst", [1, 0, 1 | 8])
def test_server_alone_and_mixed_equal_oracle(P, gpu, inst):
    from oracle import oracle as O
    torch, ctx = gpu
    jobs, data, off, sigs, want_acc, want_inv, want_all, plan = corrupted_case(inst)
    exp = {k: (want_acc[k], sorted(t for j, t in want_all if j == k)) for k in range(len(jobs))}
    params = P.make_params(inst, L1, L2)
    srv = P.Server(0, params, n_streams=3, max_group=2, distill=2)
    ids = sorted({j["key"] for j in jobs})
    pk_of = {j["key"]: j["pk"] for j in jobs}
    srv.register_keys(ids, [pk_of[i] for i in ids])
    reqs = make_requests(P, torch, jobs, data, off, sigs)
    print(f"inst {inst}: requests served alone", flush=True)
    alone = {}
    for q in reqs:
        t = srv.submit(q)
        r = collect(srv, [t])[t]
        alone[r[3]] = r[:3]
    print(f"inst {inst}: requests served together", flush=True)
    order = list(range(len(reqs)))
    random.Random(5).shuffle(order)
    tickets = [srv.submit(reqs[k]) for k in order]
    mixed = {r[3]: r[:3] for r in collect(srv, tickets).values()}
    for k in range(len(jobs)):
        assert alone[k] == (P.POSLO_OK, exp[k][0], exp[k][1]), f"request {k} alone"
        assert mixed[k] == alone[k], f"request {k} in the mix"
    # key state: Agg of the tags of every accepted request, from both runs
    for key in ids:
        acc_tags = [j["tag"] for k, j in enumerate(jobs) if j["key"] == key and exp[k][0]]
        tag, entries = srv.key_state(key)
        assert tag == O.agg(acc_tags * 2, inst)
        assert entries == 2 * sum(j["n"] for k, j in enumerate(jobs) if j["key"] == key and exp[k][0])
    st = srv.stats()
    assert st.completed == st.submitted == 2 * len(jobs) and st.bytes_in_use == 0 and st.queued == 0
    srv.close()


@pytest.mark.parametrize("inst", [1, 0])
def test_server_under_load(P, gpu, inst):
    from paper_2506_08781_amd import workloads
    torch, ctx = gpu
    print(f"inst {inst}: building requests", flush=True)
    log = workloads.serving_requests(ctx, inst, n_keys=64, n_requests=160, max_batch=4096, L=128,
                                     p_corrupt=0.1, seed=900 + inst)
    assert sum(q["flip"] is not None for q in log.requests) >= 5
    budget = 256 << 10
    srv = P.Server(0, log.params, n_streams=4, max_group=16, distill=2, mem_bytes=budget)
    srv.register_keys(list(range(64)), log.pks)
    L = log.L
    reqs = []
    for r, q in enumerate(log.requests):
        b, n = q["base"], q["n"]
        reqs.append(P.Request(q["key"], q["t0"], n, log.data[b:b + n], None, L, log.sigs[80 * b:80 * (b + n)],
                              q["ds"], q["tag"], user=r, data_bytes=n * L))
    tickets = []

    def feed():
        rng = random.Random(7)
        for q in reqs:
            tickets.append(srv.submit(q))
            time.sleep(rng.expovariate(20000.0))

    th = threading.Thread(target=feed)
    th.start()
    th.join()
    print(f"inst {inst}: {len(tickets)} submitted", flush=True)
    got = collect(srv, tickets)
    for status, acc, inv, r in got.values():
        assert status == P.POSLO_OK
        assert (acc, inv) == log.expected(r, 2), f"request {r}"
    st = srv.stats()
    print(f"inst {inst}: groups {st.groups_launched}, peak bytes {st.bytes_peak}, "
          f"p50 {st.latency_p50_ms:.2f} ms, p99 {st.latency_p99_ms:.2f} ms", flush=True)
    assert st.completed == len(reqs) and st.bytes_in_use == 0 and st.groups_launched > 1
    srv.close()


def test_server_rejects_bad_requests(P, gpu):
    from oracle import oracle as O
    torch, ctx = gpu
    jobs, data, off, sigs, *_ = corrupted_case(1)
    j = jobs[0]
    n = j["n"]
    off = np.asarray(off, dtype=np.uint64)
    m = np.frombuffer(data, dtype=np.uint8)[:int(off[n])].copy()
    o = off[:n + 1].copy()
    sg = np.frombuffer(sigs, dtype=np.uint8)[:80 * n].copy()
    params = P.make_params(1, L1, L2)
    srv = P.Server(0, params, n_streams=2, distill=1)
    srv.register_keys([7], [j["pk"]])
    with pytest.raises(P.PosloError) as ei:  # unknown key
        srv.submit(P.Request(8, 0, n, m, o, 0, sg, j["ds"], j["tag"]))
    assert ei.value.status == P.POSLO_E_INVAL
    with pytest.raises(P.PosloError) as ei:  # ds covering no epoch of the request
        srv.submit(P.Request(7, 0, n, m, o, 0, sg, b"\x00", j["tag"]))
    assert ei.value.status == P.POSLO_E_SEED
    with pytest.raises(P.PosloError) as ei:  # malformed ds
        srv.submit(P.Request(7, 0, n, m, o, 0, sg, j["ds"] + b"\x00", j["tag"]))
    assert ei.value.status == P.POSLO_E_INVAL
    empty = P.Request(7, 37, 0, None, np.zeros(1, np.uint64), 0, None, b"\x00", O.agg([]), user=1)
    good = P.Request(7, 0, n, m, o, 0, sg, j["ds"], j["tag"], user=2)
    ts = [srv.submit(q) for q in (empty, good)]
    res = {r[3]: r[:3] for r in collect(srv, ts).values()}
    assert res[1] == (P.POSLO_OK, True, [])  # no entries: the empty sum checks against the identity tag
    assert res[2] == (P.POSLO_OK, True, [])
    srv.close()


def test_server_reregistration_waits_for_the_keys_requests(P, gpu):
    """An id registered again while its requests are queued or in flight is
    refused (E_BUSY, nothing registered); once they are done it is replaced
    with a fresh aggregate state."""
    from oracle import oracle as O
    torch, ctx = gpu
    jobs, data, off, sigs, *_ = corrupted_case(1)
    j = jobs[0]
    n = j["n"]
    off = np.asarray(off, dtype=np.uint64)
    m = np.frombuffer(data, dtype=np.uint8)[:int(off[n])].copy()
    o = off[:n + 1].copy()
    sg = np.frombuffer(sigs, dtype=np.uint8)[:80 * n].copy()
    params = P.make_params(1, L1, L2)
    srv = P.Server(0, params, n_streams=2, distill=1)
    srv.register_keys([7, 9], [j["pk"], j["pk"]])
    # one request per key is in flight at a time: the rest of the 500 wait
    tickets = [srv.submit(P.Request(7, 0, n, m, o, 0, sg, j["ds"], j["tag"], user=k)) for k in range(500)]
    with pytest.raises(P.PosloError) as ei:
        srv.register_keys([9, 7], [j["pk"], j["pk"]])
    assert ei.value.status == P.POSLO_E_BUSY
    res = collect(srv, tickets)
    assert all(r[:3] == (P.POSLO_OK, True, []) for r in res.values())
    tag, entries = srv.key_state(7)
    assert tag == O.agg([j["tag"]] * 500) and entries == 500 * n
    srv.register_keys([7], [j["pk"]])
    assert srv.key_state(7) == (O.agg([]), 0)
    srv.close()
