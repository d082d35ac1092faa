"""Serving loop (tsvd_server_*): continuous batching, admission by device
footprint, latency record, and the same result alone and in a mix."""

import time

import numpy as np
import pytest

import paper_2208_08410_amd as P
import synth
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def request(m, n, k, seed, q=0.9, eps=1e-10, gram="bf16x3", pinned=False):
    d = min(m, n)
    dk = synth.dense_known(m, n, synth.spectrum_geometric(q, d), seed=seed, dtype=np.float32)
    st = synth.start_vectors(k, n if m >= n else m, seed=seed + 1)
    import torch
    A = torch.from_numpy(dk.A)
    A = A.pin_memory() if pinned else A.cuda()
    return dk, dict(A=A, k=k, eps=eps, v0=to_dev(st), gram=gram)


def arrays(res):
    U, S, V, info = res
    return U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), info


@pytest.fixture
def fresh_ctx():
    c = P.Context(0)
    yield c
    c.close()


def test_alone_and_in_mix_identical(fresh_ctx):
    """A request gives the same bits alone and mixed with others of other
    shapes (its launch shapes depend on it alone)."""
    dk, probe = request(3000, 400, 6, seed=1)
    with P.Server(fresh_ctx, hbm_budget=1 << 30) as srv:
        alone = arrays(srv.wait(srv.submit(probe)))
        others = [request(m, n, k, seed=10 + i)[1] for i, (m, n, k) in
                  enumerate([(2000, 1000, 8), (500, 1500, 4), (6000, 128, 3), (800, 800, 5)])]
        tickets = [srv.submit(o) for o in others[:2]] + [srv.submit(probe)] + [srv.submit(o) for o in others[2:]]
        mixed = [arrays(srv.wait(t)) for t in tickets]
        st = srv.stats()
    Ua, Sa, Va, ia = alone
    Um, Sm, Vm, im = mixed[2]
    assert ia["status"] == "TSVD_OK" and im["status"] == "TSVD_OK"
    assert np.array_equal(Sa, Sm) and np.array_equal(Ua, Um) and np.array_equal(Va, Vm)
    assert ia["iters"] == im["iters"]
    assert np.max(np.abs(Sa - dk.s[:6]) / dk.s[:6]) < 1e-6
    assert st["completed"] == 6 and st["failed"] == 0
    # the same bits again through the one-call batched entry point
    Ub, Sb, Vb, _ = arrays(P.tsvd_dense_batched(fresh_ctx, [probe], raise_errors=True)[0])
    assert np.array_equal(Sa, Sb) and np.array_equal(Ua, Ub)


def test_stream_of_requests_continuous_batching(fresh_ctx):
    """Requests submitted while others run are admitted and batched; every
    result meets the closed form; the latency record is consistent."""
    rng = np.random.default_rng(3)
    reqs = []
    for i in range(40):
        m = int(np.exp(rng.uniform(np.log(1024), np.log(8192))))
        n = int(np.exp(rng.uniform(np.log(128), np.log(1024))))
        k = int(rng.choice([4, 8]))
        reqs.append(request(m, n, k, seed=100 + i, q=0.85, eps=1e-12))
    with P.Server(fresh_ctx, hbm_budget=2 << 30, max_slots=16) as srv:
        tickets = []
        for i, (dk, p) in enumerate(reqs):
            tickets.append(srv.submit(p))
            if i >= 10:  # a burst of 10, then Poisson arrivals at 500 / s
                time.sleep(float(rng.exponential(0.002)))
        results = [arrays(srv.wait(t)) for t in tickets]
        st = srv.stats()
    for (dk, p), (U, S, V, info) in zip(reqs, results):
        k = p["k"]
        assert info["status"] == "TSVD_OK"
        assert np.max(np.abs(S - dk.s[:k]) / dk.s[:k]) < 1e-6
        Q = V if info["branch_right"] else U
        assert np.linalg.norm(Q.T @ Q - np.eye(k)) < 1e-10
    assert st["completed"] == 40 and st["submitted"] == 40 and st["rejected"] == 0
    assert st["batches"] < 40 and st["mean_batch"] > 1.0  # arrivals during a batch were batched together
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert st["in_flight"] == 0 and st["waiting"] == 0


def test_admission_budget_and_rejection(fresh_ctx):
    """With room for one request at a time everything still completes, the
    admitted footprint never exceeds the budget, and a request larger than the
    budget is rejected."""
    small = [request(2000, 300, 4, seed=200 + i, q=0.8, eps=1e-12) for i in range(5)]
    # 2 MiB: 1 MiB of batch tables (half the budget) and 1 MiB for requests,
    # which holds one 300 x 300 Gram with its partial tiles (~0.75 MB) at a time
    budget = 2 << 20
    big_dk, big = request(1000, 1000, 2, seed=300)  # a 4 MB Gram: more than the request region
    with P.Server(fresh_ctx, hbm_budget=budget) as srv:
        tickets = [srv.submit(p) for _, p in small]
        tb = srv.submit(big)
        res = [arrays(srv.wait(t)) for t in tickets]
        rb = srv.wait(tb)
        st = srv.stats()
    for (dk, p), (U, S, V, info) in zip(small, res):
        assert info["status"] == "TSVD_OK"
        assert np.max(np.abs(S - dk.s[:4]) / dk.s[:4]) < 1e-6
    assert rb[3]["status"] == "TSVD_ERR_REJECTED"
    assert st["rejected"] == 1 and st["completed"] == 5
    assert st["peak_bytes"] <= budget // 2
    assert st["batches"] >= 5  # one request per batch


def test_pinned_host_request_matches_device(fresh_ctx):
    dk, pdev = request(4000, 512, 4, seed=400)
    _, phost = request(4000, 512, 4, seed=400, pinned=True)
    with P.Server(fresh_ctx, hbm_budget=1 << 30) as srv:
        a = arrays(srv.wait(srv.submit(pdev)))
        b = arrays(srv.wait(srv.submit(phost)))
    assert b[3]["h2d_bytes"] == 4000 * 512 * 4
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


def test_submit_rejects_bad_arguments(fresh_ctx):
    dk, p = request(300, 100, 2, seed=5)
    with P.Server(fresh_ctx, hbm_budget=64 << 20) as srv:
        with pytest.raises(P.TsvdError) as e:
            srv.submit(dict(p, A=p["A"].double()))
        assert e.value.status == P.UNSUPPORTED
        with pytest.raises(P.TsvdError) as e:
            srv.submit(dict(p, k=101, v0=to_dev(synth.start_vectors(101, 100, 1))))
        assert e.value.status == P.INVALID_ARG
        # the server keeps working after rejected submissions
        U, S, V, info = arrays(srv.wait(srv.submit(p)))
        assert info["status"] == "TSVD_OK"


def hh_request(m, n, k, seed, q, iters):
    """A = H_L [diag(q^i); 0] H_R built on the device, k start vectors, fixed
    iteration counts (so the request's duration is known in advance)."""
    import torch
    s = synth.spectrum_geometric(q, min(m, n))
    A = synth.householder_known_torch(m, n, s, seed, torch.device("cuda:0"))
    st = synth.start_vectors(k, n if m >= n else m, seed=seed + 1)
    return s, dict(A=A, k=k, eps=0.0, v0=to_dev(st), gram="bf16x3", fixed_iters=[iters] * k)


def test_arrival_overlaps_running_batch(fresh_ctx):
    """Continuous batching across lanes: a small request submitted while a long
    batch runs is launched on the free lane into the CUs the long batch's team
    leaves free (a 1400-dimensional Gram takes a team of 30 workgroups, so more
    than the 7/8 of the chip a second lane waits for stays free), completes
    while the long batch is still on the device, and gives the same bits as
    when it runs alone."""
    s_long, long_p = hh_request(30000, 1400, 64, seed=501, q=0.99, iters=600)
    s_small, small_p = hh_request(2000, 300, 4, seed=502, q=0.8, iters=60)
    with P.Server(fresh_ctx, hbm_budget=4 << 30, lanes=2) as srv:
        t_long = time.perf_counter()
        tl = srv.submit(long_p)
        time.sleep(0.02)  # the long request is on the device now
        t_small = time.perf_counter()
        ts = srv.submit(small_p)
        small = arrays(srv.wait(ts))
        t_small_seen = time.perf_counter()
        long_ = arrays(srv.wait(tl))
        st = srv.stats()
        alone = arrays(srv.wait(srv.submit(small_p)))
    done_small = t_small + small[3]["latency_ms"] * 1e-3
    done_long = t_long + long_[3]["latency_ms"] * 1e-3
    assert small[3]["status"] == "TSVD_OK" and long_[3]["status"] == "TSVD_OK"
    assert done_small < done_long, (small[3]["latency_ms"], long_[3]["latency_ms"])
    assert t_small_seen < done_long
    assert st["overlapped"] >= 1 and st["lanes_busy_max"] == 2
    # the same bits alone
    assert np.array_equal(small[1], alone[1]) and np.array_equal(small[0], alone[0])
    assert np.array_equal(small[2], alone[2])
    assert np.max(np.abs(small[1] - s_small[:4]) / s_small[:4]) < 1e-6
    # the long request is only a timer (fixed iterations at a ratio of 0.99
    # leave neighbouring triplets partly mixed); its leading sigma has converged
    assert abs(long_[1][0] - s_long[0]) < 1e-6


def test_one_lane_runs_one_batch_at_a_time(fresh_ctx):
    """lanes = 1: batches never overlap (the server waits for the running batch
    before it launches the next), and results still meet the closed form."""
    reqs = [request(3000, 256, 4, seed=600 + i, q=0.8, eps=1e-12) for i in range(6)]
    with P.Server(fresh_ctx, hbm_budget=1 << 30, lanes=1) as srv:
        tickets = []
        for dk, p in reqs:
            tickets.append(srv.submit(p))
            time.sleep(0.001)
        res = [arrays(srv.wait(t)) for t in tickets]
        st = srv.stats()
    assert st["overlapped"] == 0 and st["lanes_busy_max"] == 1
    for (dk, p), (U, S, V, info) in zip(reqs, res):
        assert info["status"] == "TSVD_OK"
        assert np.max(np.abs(S - dk.s[:4]) / dk.s[:4]) < 1e-6
