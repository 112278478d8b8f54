"""GPU: the library's serving runtime (cm_server_*).  Every merge it reports
must equal the same merge run alone through cm_stable_merge_pairs, bit for
bit, and the oracle; arena pressure forces queueing and ring wrap-around."""
import time

import numpy as np
import pytest

import oracle
import paper_1303_4312_amd as cm
from paper_1303_4312_amd import serve, workloads
from tests.gpu_util import same_bits, to_dev, to_host

pytestmark = pytest.mark.gpu


def make_requests(count, seed, lo=1, hi=1 << 17):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        d = workloads.request(int(rng.integers(1 << 30)), lo=lo, hi=hi)
        if k % 7 == 3:  # empty and one-sided requests in the mix
            d["B"], d["Bv"] = d["B"][:0], d["Bv"][:0]
        if k % 11 == 5:
            d["A"], d["Av"], d["B"], d["Bv"] = d["A"][:0], d["Av"][:0], d["B"][:0], d["Bv"][:0]
        out.append(d)
    return out


def drain(srv, want, sizes, results, timeout=60.0):
    t_end = time.time() + timeout
    while len(results) < want:
        assert time.time() < t_end, "server did not finish in time"
        for d in srv.poll(wait_us=2000):
            assert d.status == 0, f"ticket {d.ticket}: status {d.status}"
            N = sizes[d.ticket]
            C, Cv = srv.outputs(d, N)
            results[d.ticket] = (to_host(C), to_host(Cv))
            srv.release(d.ticket)


def test_native_server_matches_alone_and_oracle():
    import torch
    reqs = make_requests(40, seed=7)
    dev = [(to_dev(d["A"]), to_dev(d["B"]), to_dev(d["Av"]), to_dev(d["Bv"])) for d in reqs]
    alone = []
    for A, B, Av, Bv in dev:
        C, Cv = cm.stable_merge_pairs(A, Av, B, Bv)
        alone.append((to_host(C), to_host(Cv)))
    total = sum(8 * (d["A"].size + d["B"].size) + 512 for d in reqs)
    # arena of a third of all outputs: admission waits for releases, the ring wraps
    srv = serve.NativeServer("uint32", True, arena_bytes=max(total // 3, 1 << 21), max_batch=8,
                             max_inflight=2, max_requests=64)
    torch.cuda.synchronize()
    tickets, sizes, results = [], {}, {}
    for A, B, Av, Bv in dev:
        while True:
            try:
                t = srv.submit(A, B, Av, Bv)
                break
            except cm.CMError as e:
                assert e.status == -9  # every slot taken: collect results first
                drain(srv, len(results) + 1, sizes, results)
        tickets.append(t)
        sizes[t] = A.numel() + B.numel()
    drain(srv, len(tickets), sizes, results)
    st = srv.stats()
    srv.close()
    for k, t in enumerate(tickets):
        C, Cv = results[t]
        assert same_bits(C, alone[k][0]), f"request {k}: keys differ from the single call"
        assert same_bits(Cv, alone[k][1]), f"request {k}: payloads differ from the single call"
    for d, (C, Cv) in list(zip(reqs, [results[t] for t in tickets]))[:8]:
        Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
        assert same_bits(C, Ce) and same_bits(Cv, Cve)
    assert st["submitted"] == len(reqs) and st["completed"] == len(reqs)
    assert st["failed"] == 0 and st["canceled"] == 0
    assert st["batches"] >= 3 and 1 <= st["max_batch_seen"] <= 8
    assert st["arena_peak_bytes"] <= st["arena_bytes"]
    assert 0 < st["busy_ms"] <= st["span_ms"] + 1e-3


def test_native_server_waits_for_inputs_on_their_stream():
    import torch
    d = workloads.request(11, lo=1 << 18, hi=1 << 18)
    A, Av = to_dev(d["A"]), to_dev(d["Av"])
    B = torch.empty(d["B"].size, dtype=torch.uint32, device="cuda:0")
    Bv = torch.empty(d["Bv"].size, dtype=torch.uint32, device="cuda:0")
    hB = torch.from_numpy(d["B"]).pin_memory()
    hBv = torch.from_numpy(d["Bv"]).pin_memory()
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with serve.NativeServer("uint32", True, arena_bytes=1 << 24) as srv:
        with torch.cuda.stream(side):
            B.copy_(hB, non_blocking=True)
            Bv.copy_(hBv, non_blocking=True)
            t = srv.submit(A, B, Av, Bv)  # waits for the copies on `side`
        results = {}
        drain(srv, 1, {t: A.numel() + B.numel()}, results)
    Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
    assert same_bits(results[t][0], Ce) and same_bits(results[t][1], Cve)


def test_native_server_keys_only_float():
    import torch
    rng = np.random.default_rng(5)
    with serve.NativeServer("float32", False, arena_bytes=1 << 22, max_batch=4) as srv:
        host, tickets = {}, []
        for k in range(12):
            A = np.sort(rng.standard_normal(int(rng.integers(0, 50_000))).astype(np.float32))
            B = np.sort(rng.standard_normal(int(rng.integers(0, 50_000))).astype(np.float32))
            if k == 2:
                A[:10] = -0.0
                B[:10] = 0.0
                A.sort(), B.sort()
            dA, dB = to_dev(A), to_dev(B)  # kept alive until the merge is reported
            t = srv.submit(dA, dB)
            tickets.append(t)
            host[t] = (A, B, dA, dB)
        seen = {}
        t_end = time.time() + 60
        while len(seen) < len(tickets):
            assert time.time() < t_end
            for d in srv.poll(wait_us=2000):
                assert d.status == 0
                A, B = host[d.ticket][:2]
                seen[d.ticket] = to_host(srv.outputs(d, A.size + B.size))
                srv.release(d.ticket)
        torch.cuda.synchronize()
    for t in tickets:
        A, B = host[t][:2]
        assert same_bits(seen[t], oracle.stable_merge(A, B))


def test_native_server_refuses_and_shuts_down_cleanly():
    d = workloads.request(3, lo=1 << 16, hi=1 << 16)
    A, B, Av, Bv = to_dev(d["A"]), to_dev(d["B"]), to_dev(d["Av"]), to_dev(d["Bv"])
    need = 2 * 4 * (A.numel() + B.numel())
    srv = serve.NativeServer("uint32", True, arena_bytes=need + 256, max_requests=8)
    with pytest.raises(cm.CMError) as e:  # outputs larger than the whole arena
        big = to_dev(np.zeros(A.numel() * 2, dtype=np.uint32))
        srv.submit(big, B, big, Bv)
    assert e.value.status == -5
    first = srv.submit(A, B, Av, Bv)
    done = []
    t_end = time.time() + 30
    while not done:
        assert time.time() < t_end
        done = srv.poll(wait_us=2000)
    assert done[0].ticket == first and done[0].status == 0
    with pytest.raises(cm.CMError):
        srv.release(first + (1 << 16))  # not a ticket of this server
    # the first outputs stay held: these two can never be admitted
    srv.submit(A, B, Av, Bv)
    srv.submit(A, B, Av, Bv)
    t0 = time.time()
    srv.close()  # cancels them instead of waiting for space
    assert time.time() - t0 < 10


def test_native_server_host_requests_match_alone_and_oracle():
    """Requests whose data live in host memory (pinned and pageable), mixed
    with device requests in one server whose arena holds about a third of
    all inputs plus outputs: admission waits, the ring wraps, and every
    host request's outputs come back to host memory equal to the merge run
    alone."""
    import torch
    reqs = make_requests(36, seed=21, hi=1 << 16)
    alone = []
    for d in reqs:
        C, Cv = cm.stable_merge_pairs(to_dev(d["A"]), to_dev(d["Av"]), to_dev(d["B"]), to_dev(d["Bv"]))
        alone.append((to_host(C), to_host(Cv)))
    total = sum(16 * (d["A"].size + d["B"].size) + 1024 for d in reqs)
    srv = serve.NativeServer("uint32", True, arena_bytes=max(total // 3, 1 << 21), max_batch=8,
                             max_inflight=2, max_requests=16)
    kind, sizes, results, dev_inputs = {}, {}, {}, []

    def collect(want):
        t_end = time.time() + 60
        while len(results) < want:
            assert time.time() < t_end, "server did not finish in time"
            for e in srv.poll(wait_us=2000):
                assert e.status == 0, f"ticket {e.ticket}: status {e.status}"
                k, N = kind[e.ticket], sizes[e.ticket]
                if k == "host":
                    C, Cv = srv.host_outputs(e.ticket)
                    results[e.ticket] = (C.numpy().copy(), Cv.numpy().copy())
                else:
                    C, Cv = srv.outputs(e, N)
                    results[e.ticket] = (to_host(C), to_host(Cv))
                srv.release(e.ticket)

    order = []
    torch.cuda.synchronize()
    for r, d in enumerate(reqs):
        host = r % 3 != 2
        while True:
            try:
                if host:
                    ts = [torch.from_numpy(d[k]) for k in ("A", "B", "Av", "Bv")]
                    if r % 2 == 0:
                        ts = [t.pin_memory() for t in ts]
                    t = srv.submit_host(ts[0], ts[1], ts[2], ts[3])
                else:
                    dv = [to_dev(d[k]) for k in ("A", "B", "Av", "Bv")]
                    dev_inputs.append(dv)
                    torch.cuda.synchronize()
                    t = srv.submit(dv[0], dv[1], dv[2], dv[3])
                break
            except cm.CMError as exc:
                assert exc.status == -9
                collect(len(results) + 1)
        kind[t] = "host" if host else "device"
        sizes[t] = d["A"].size + d["B"].size
        order.append(t)
    collect(len(order))
    st = srv.stats()
    srv.close()
    for r, t in enumerate(order):
        C, Cv = results[t]
        assert same_bits(C, alone[r][0]) and same_bits(Cv, alone[r][1]), f"request {r} ({kind[t]})"
    for d, t in list(zip(reqs, order))[:6]:
        Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
        assert same_bits(results[t][0], Ce) and same_bits(results[t][1], Cve)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["arena_peak_bytes"] <= st["arena_bytes"]


def test_native_server_host_request_errors():
    import ctypes
    import torch
    srv = serve.NativeServer("uint32", True, arena_bytes=1 << 21, max_batch=4, max_inflight=1,
                             max_requests=4)
    lib, t = srv.lib, ctypes.c_uint64()
    A = torch.zeros(1024, dtype=torch.uint32).pin_memory()
    B = torch.zeros(1024, dtype=torch.uint32).pin_memory()
    C = torch.zeros(2048, dtype=torch.uint32).pin_memory()
    Cv = torch.zeros(2048, dtype=torch.uint32).pin_memory()
    p = lambda x: x.data_ptr()
    # outputs over an input, outputs over each other, missing outputs
    assert lib.cm_server_submit_host(srv._h, p(A), p(A), 1024, p(B), p(B), 1024, p(A), p(Cv),
                                     ctypes.byref(t)) == -4
    assert lib.cm_server_submit_host(srv._h, p(A), p(A), 1024, p(B), p(B), 1024, p(C), p(C),
                                     ctypes.byref(t)) == -4
    assert lib.cm_server_submit_host(srv._h, p(A), p(A), 1024, p(B), p(B), 1024, None, p(Cv),
                                     ctypes.byref(t)) == -1
    # inputs plus outputs larger than the arena (made-up, disjoint addresses:
    # the call refuses before touching them)
    big, G = 1 << 17, 1 << 32
    assert lib.cm_server_submit_host(srv._h, G, 2 * G, big, 3 * G, 4 * G, big, 5 * G, 6 * G,
                                     ctypes.byref(t)) == -5
    # payloads shorter than their keys, or outputs of another type, are
    # refused by the binding before the runtime could read or write past them
    with pytest.raises(ValueError):
        srv.submit_host(A, B, A[:1000], B)
    with pytest.raises(ValueError):
        srv.submit_host(A, B, A, B, C=C.view(torch.int32))
    with pytest.raises(ValueError):
        srv.submit_host(A, B, A, B, C_val=torch.zeros(2048, dtype=torch.uint8).pin_memory())
    dA = A.cuda()
    with pytest.raises(ValueError):
        srv.submit(dA, dA, dA[:1023], dA)
    with pytest.raises(ValueError):
        srv.submit(dA, dA, dA.view(torch.int32), dA)
    # an empty host request completes
    e = torch.zeros(0, dtype=torch.uint32)
    tk = srv.submit_host(e, e, e, e)
    done = []
    t_end = time.time() + 20
    while not done:
        assert time.time() < t_end
        done = srv.poll(wait_us=2000)
    assert done[0].ticket == tk and done[0].status == 0
    srv.release(tk)
    srv.close()


def test_native_server_close_with_host_requests_in_flight():
    """Closing the server while host requests are admitted, merging or on
    their way back finishes them first: afterwards every one that was
    admitted has its outputs in host memory, equal to the oracle's."""
    import torch
    reqs = make_requests(12, seed=33, lo=1 << 12, hi=1 << 16)
    srv = serve.NativeServer("uint32", True, arena_bytes=1 << 26, max_batch=4, max_inflight=2,
                             max_requests=16)
    tickets = []
    for d in reqs:
        ts = [torch.from_numpy(d[k]).pin_memory() for k in ("A", "B", "Av", "Bv")]
        tickets.append(srv.submit_host(ts[0], ts[1], ts[2], ts[3]))
    outs = [srv.host_outputs(t) for t in tickets]
    srv.close()  # no poll: shutdown itself must drain the copies back
    for d, (C, Cv) in zip(reqs, outs):
        Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
        assert same_bits(C.numpy(), Ce) and same_bits(Cv.numpy(), Cve)


@pytest.mark.parametrize("partition", [-1, 2, 4])
def test_native_server_large_batches(partition, restore_settings):
    """Batches of more than CM_BATCH_INLINE_MAX merges: their descriptors are
    read from the server's pinned host array by the batch's first kernel (no
    upload), in the automatic boundary mode, with the two-level pass, and
    with none (every block co-ranks its ends after the prep kernel).  Every
    request equals the merge run alone and the oracle; a batch of more than
    16 is formed for certain (the requests are let in together)."""
    import torch
    print(f"[server large batches] partition={partition}", flush=True)
    cm.set_partition(partition)
    reqs = make_requests(150, seed=31, lo=1, hi=1 << 14)
    dev = [(to_dev(d["A"]), to_dev(d["B"]), to_dev(d["Av"]), to_dev(d["Bv"])) for d in reqs]
    alone = []
    for A, B, Av, Bv in dev:
        C, Cv = cm.stable_merge_pairs(A, Av, B, Bv)
        alone.append((to_host(C), to_host(Cv)))
    # A first request whose outputs fill the arena holds the others back
    # (admission is in arrival order and waits for space); its release lets
    # all of them in at once, inputs long ready, so the scheduler fills
    # batches up to max_batch.
    half = 1 << 22
    big = [torch.arange(half, dtype=torch.int32, device="cuda:0").view(torch.uint32) for _ in range(4)]
    srv = serve.NativeServer("uint32", True, arena_bytes=16 * half + 256, max_batch=64, max_inflight=2,
                             max_requests=256)
    torch.cuda.synchronize()
    first = srv.submit(big[0], big[1], big[2], big[3])
    tickets, sizes, results = [], {}, {}
    for A, B, Av, Bv in dev:
        t = srv.submit(A, B, Av, Bv)
        tickets.append(t)
        sizes[t] = A.numel() + B.numel()
    t_end = time.time() + 60
    first_done = False
    while not first_done:
        assert time.time() < t_end, "the first request did not finish in time"
        for d in srv.poll(wait_us=2000):
            assert d.status == 0, f"ticket {d.ticket}: status {d.status}"
            if d.ticket == first:
                first_done = True
                continue
            # only empty requests take no arena space and may pass it
            assert sizes[d.ticket] == 0, "a request was admitted while the arena was full"
            C, Cv = srv.outputs(d, 0)
            results[d.ticket] = (to_host(C), to_host(Cv))
            srv.release(d.ticket)
    srv.release(first)
    drain(srv, len(tickets), sizes, results)
    st = srv.stats()
    srv.close()
    for k, t in enumerate(tickets):
        C, Cv = results[t]
        assert same_bits(C, alone[k][0]) and same_bits(Cv, alone[k][1]), f"request {k} differs"
    for d, (C, Cv) in list(zip(reqs, [results[t] for t in tickets]))[:10]:
        Ce, Cve = oracle.stable_merge(d["A"], d["B"], d["Av"], d["Bv"])
        assert same_bits(C, Ce) and same_bits(Cv, Cve)
    assert st["completed"] == len(reqs) + 1 and st["max_batch_seen"] > 16
