"""Continuous-batching query server: every served result equals the oracle's
for the same (seed, query_id), alone or in any mix of models, levels and
thresholds, whatever the size of its residue tables (runs ended by a full
table start again); admission by table memory never lets the running
queries hold more than the pool; submission errors stay local to the
offending query."""
import time

import numpy as np
import pytest

import oracle
from paper_2106_03058_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_03058_amd import agp

    g = inputs.chung_lu(5000, 10, 2.5, seed=23)
    G = agp.Graph.from_inputs(g, validate=True)
    sg = oracle.degree_sort(g)
    lam = inputs.lambda_max(g)
    return torch, agp, g, G, sg, lam


def _mix(g, lam, k, seed):
    rng = np.random.default_rng(seed)
    src = inputs.sources_by_degree(g, k, seed)
    qs = []
    for i in range(k):
        kind = i % 3
        L = int(rng.integers(3, 16))
        eps = float(rng.choice([1e-4, 1e-5, 1e-6]))
        if kind == 0:
            a, b, w = 0.0, 1.0, inputs.weights_ppr(float(rng.uniform(0.1, 0.3)), L)
        elif kind == 1:
            a, b, w = 0.0, 0.0, inputs.weights_katz(0.85 / lam, L, 0.85)
        else:
            a, b, w = 0.0, 1.0, inputs.weights_tp(L)
        qs.append(dict(source=int(src[i]), a=a, b=b, w=w, eps=eps, seed=7000 + i, qid=100 + i))
    return qs


def _oracle_one(g, sg, q):
    x = inputs.one_hot(g.n, [q["source"]])[:, 0]
    out, cnt = oracle.propagate(sg, q["a"], q["b"], q["w"], x, q["eps"], q["seed"], wp=32, qids=[q["qid"]])
    return out, {k: v[0] for k, v in cnt.items()}


def _serve(torch, agp, G, qs, *, slots, budget=0.0, memory=256 << 20):
    srv = agp.Server(G, max_slots=slots, queue_capacity=len(qs) + 4, work_budget=budget, memory_bytes=memory)
    outs = [torch.full((G.n,), float("nan"), dtype=torch.float32, device="cuda:0") for _ in qs]
    tickets = [srv.submit(q["source"], q["a"], q["b"], q["w"], q["eps"], q["seed"], q["qid"], o, x=q.get("x"))
               for q, o in zip(qs, outs)]
    res = [None] * len(qs)
    t0 = time.time()
    while any(r is None for r in res):
        for i, t in enumerate(tickets):
            if res[i] is None:
                res[i] = srv.poll(t)
        assert time.time() - t0 < 60, "server did not finish"
        time.sleep(0.001)
    srv.close()
    return [o.cpu().numpy().astype(np.float64) for o in outs], res


def test_mixed_stream_matches_oracle(env):
    torch, agp, g, G, sg, lam = env
    qs = _mix(g, lam, 30, seed=1)
    outs, res = _serve(torch, agp, G, qs, slots=7)
    for q, o, r in zip(qs, outs, res):
        ref, cnt = _oracle_one(g, sg, q)
        assert r["status"] == agp.AGP_OK
        assert np.array_equal(o, ref), f"query {q['qid']}: max diff {np.abs(o - ref).max()}"
        assert r["pushes"] == int(cnt["det"].sum() + cnt["acc"].sum())
        assert r["candidates"] == int(cnt["cand"].sum())
        assert r["frontier"] == int(cnt["frontier"].sum())
        assert r["levels"] == len(q["w"]) - 1
        assert r["submit_ms"] <= r["start_ms"] <= r["end_ms"]


def test_alone_equals_mix_and_batch(env):
    torch, agp, g, G, sg, lam = env
    qs = _mix(g, lam, 12, seed=2)
    mixed, _ = _serve(torch, agp, G, qs, slots=5)
    alone, _ = _serve(torch, agp, G, [qs[4]], slots=1)
    assert np.array_equal(alone[0], mixed[4])
    # the batched entry point with the same (seed, qid) gives the same column
    q = qs[4]
    X = torch.from_numpy(inputs.one_hot(g.n, [q["source"]])).to("cuda:0")
    out, _ = agp.propagate(G, q["a"], q["b"], q["w"], X, q["eps"], q["seed"], qids=[q["qid"]])
    assert np.array_equal(out[:, 0].cpu().numpy().astype(np.float64), mixed[4])


def test_work_budget_admission(env):
    torch, agp, g, G, sg, lam = env
    qs = _mix(g, lam, 9, seed=3)
    outs, res = _serve(torch, agp, G, qs, slots=9, budget=1.0)  # one query at a time
    starts = sorted((r["start_ms"], r["end_ms"]) for r in res)
    for (s0, e0), (s1, _) in zip(starts, starts[1:]):
        assert s1 >= e0 - 1e-6  # never two queries running together
    for q, o in zip(qs, outs):
        ref, _ = _oracle_one(g, sg, q)
        assert np.array_equal(o, ref)


def test_submission_errors_are_local(env):
    torch, agp, g, G, sg, lam = env
    srv = agp.Server(G, max_slots=2, queue_capacity=3)
    out = torch.zeros(G.n, dtype=torch.float32, device="cuda:0")
    w = inputs.weights_ppr(0.2, 5)
    bad = [dict(source=-1), dict(source=G.n), dict(a=1.5), dict(eps=0.0), dict(eps=2.0 ** -45),
           dict(w=-w), dict(qid=1 << 24)]
    for b in bad:
        q = dict(source=0, a=0.0, b=1.0, w=w, eps=1e-4, seed=1, qid=1) | b
        with pytest.raises(agp.AGPError) as e:
            srv.submit(q["source"], q["a"], q["b"], q["w"], q["eps"], q["seed"], q["qid"], out)
        assert e.value.code == agp.AGP_EINVAL
    with pytest.raises(agp.AGPError) as e:
        srv.poll(12345)
    assert e.value.code == agp.AGP_ENOENT
    # a good query still runs and is collected exactly once
    t = srv.submit(0, 0.0, 1.0, w, 1e-4, 1, 1, out)
    r = None
    t0 = time.time()
    while r is None and time.time() - t0 < 30:
        r = srv.poll(t)
    assert r is not None and r["status"] == agp.AGP_OK
    with pytest.raises(agp.AGPError):
        srv.poll(t)
    srv.close()


def test_queue_full_is_ebusy(env):
    torch, agp, g, G, sg, lam = env
    srv = agp.Server(G, max_slots=1, queue_capacity=2)
    outs = [torch.zeros(G.n, dtype=torch.float32, device="cuda:0") for _ in range(40)]
    w = inputs.weights_tp(12)
    busy = 0
    tickets = []
    for i, o in enumerate(outs):
        try:
            tickets.append(srv.submit(i % G.n, 0.0, 1.0, w, 1e-6, 1, i, o))
        except agp.AGPError as e:
            assert e.code == agp.AGP_EBUSY
            busy += 1
    assert busy > 0
    srv.close()  # finishes the running query, drops the queued ones


def test_table_sizes_serve_the_same_bits(env, monkeypatch):
    """Served queries give the oracle's bits with tables sized from their
    push estimates, and with tables forced so small that runs end on a full
    table and start again with larger ones."""
    torch, agp, g, G, sg, lam = env
    qs = _mix(g, lam, 9, seed=4)
    for entries in (None, "256", "16"):
        monkeypatch.delenv("AGP_SERVE_TABLE_ENTRIES", raising=False)
        if entries:
            monkeypatch.setenv("AGP_SERVE_TABLE_ENTRIES", entries)
        print(f"table entries {entries}", flush=True)
        outs, res = _serve(torch, agp, G, qs, slots=4)
        for q, o, r in zip(qs, outs, res):
            ref, cnt = _oracle_one(g, sg, q)
            assert r["status"] == agp.AGP_OK
            assert np.array_equal(o, ref), f"{entries}: query {q['qid']}"
            assert r["pushes"] == int(cnt["det"].sum() + cnt["acc"].sum())
            assert r["frontier"] == int(cnt["frontier"].sum())
        if entries == "16":
            assert sum(r["restarts"] for r in res) > 0  # some tables did fill up
            assert all(r["table_entries"] == min(16 << r["restarts"], g.n) for r in res)
        if entries is None:
            assert all(r["restarts"] == 0 for r in res)


def test_memory_admission(env):
    """With a pool that holds the tables of only a few queries at once, the
    queries that run together never hold more than the pool (20 bytes per
    table entry, two tables each), every result is the oracle's, and a query
    whose tables exceed the whole pool ends with AGP_ENOMEM."""
    torch, agp, g, G, sg, lam = env
    qs = _mix(g, lam, 16, seed=6)
    pool = 3 * 2 * 5000 * 20 + 1000  # three queries with direct tables (n = 5000 entries each)
    outs, res = _serve(torch, agp, G, qs, slots=16, memory=pool)
    for q, o, r in zip(qs, outs, res):
        ref, _ = _oracle_one(g, sg, q)
        assert r["status"] == agp.AGP_OK
        assert np.array_equal(o, ref)
    events = sorted([(r["start_ms"], 1, 2 * r["table_entries"] * 20) for r in res] +
                    [(r["end_ms"], 0, -2 * r["table_entries"] * 20) for r in res])  # ends before starts at a tie
    held = peak = 0
    for _, _, d in events:
        held += d
        peak = max(peak, held)
    assert 0 < peak <= pool
    # tables larger than the pool: the query finishes at once with AGP_ENOMEM
    srv = agp.Server(G, max_slots=2, queue_capacity=4, memory_bytes=2 * 1024 * 20)
    o = torch.zeros(G.n, dtype=torch.float32, device="cuda:0")
    t = srv.submit(qs[0]["source"], 0.0, 1.0, inputs.weights_ppr(0.2, 8), 1e-7, 1, 1, o)
    t0 = time.time()
    r = None
    while r is None and time.time() - t0 < 30:
        r = srv.poll(t)
    srv.close()
    assert r is not None and r["status"] == agp.AGP_ENOMEM


def _dense(g, q):
    x = np.zeros(g.n, dtype=np.float32)
    if q.get("x") is None:
        x[q["source"]] = 1.0
    else:
        x[q["x"][0]] = q["x"][1]
    return x


def test_sparse_signal_queries(env):
    """Queries with sparse signals (seed sets, signed values) served beside
    single-source ones: each equals the oracle and the batched call on the
    dense signal with the same (seed, query id); signed values may cancel to
    zero inside a table, and such nodes stay out of the frontier."""
    torch, agp, g, G, sg, lam = env
    rng = np.random.default_rng(31)
    qs = _mix(g, lam, 9, seed=5)
    for i, q in enumerate(qs):
        if i % 3 == 1:  # a seed set
            ids = rng.choice(g.n, size=int(rng.integers(2, 40)), replace=False)
            vals = rng.uniform(0.5, 2.0, size=ids.size).astype(np.float32)
            if i == 4:
                vals[::2] *= -1.0  # signed
            q["x"] = (ids, vals)
    outs, res = _serve(torch, agp, G, qs, slots=4)
    for q, o, r in zip(qs, outs, res):
        x = _dense(g, q)
        ref, cnt = oracle.propagate(sg, q["a"], q["b"], q["w"], x, q["eps"], q["seed"], wp=32, qids=[q["qid"]])
        assert r["status"] == agp.AGP_OK
        assert np.array_equal(o, ref), f"query {q['qid']}: max diff {np.abs(o - ref).max()}"
        assert r["pushes"] == int(cnt["det"].sum() + cnt["acc"].sum())
        X = torch.from_numpy(x[:, None].copy()).to("cuda:0")
        out, _ = agp.propagate(G, q["a"], q["b"], q["w"], X, q["eps"], q["seed"], qids=[q["qid"]])
        assert np.array_equal(out[:, 0].cpu().numpy().astype(np.float64), o)


def test_sparse_signal_errors(env):
    torch, agp, g, G, sg, lam = env
    srv = agp.Server(G, max_slots=2, queue_capacity=8)
    o = torch.zeros(g.n, dtype=torch.float32, device="cuda:0")
    w = inputs.weights_ppr(0.2, 5)
    bad = [
        (np.array([3, 3]), np.array([1.0, 2.0])),        # repeated id
        (np.array([g.n]), np.array([1.0])),              # out of range
        (np.array([1, 2]), np.array([0.0, 0.0])),        # no non-zero entry
        (np.array([1, 2]), np.array([1.0, np.nan])),     # not finite
        (np.array([1, 2]), np.array([1.0, 1e-30])),      # below the unit of theta
    ]
    for x in bad:
        with pytest.raises(agp.AGPError) as e:
            srv.submit(0, 0.0, 1.0, w, 1e-4, 1, 1, o, x=x)
        assert e.value.code == agp.AGP_EINVAL
    # a good one still runs
    t = srv.submit(0, 0.0, 1.0, w, 1e-4, 1, 1, o, x=(np.array([5, 9]), np.array([1.0, -0.5])))
    t0 = time.time()
    r = None
    while r is None and time.time() - t0 < 30:
        r = srv.poll(t)
    srv.close()
    assert r is not None and r["status"] == agp.AGP_OK
