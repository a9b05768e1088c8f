"""GPU: the request loop (rdist_server_*): continuous batching, admission by
HBM footprint, and results that are bit-for-bit those of the same request
solved alone; spot checks against the oracle."""
import sys
import time

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2308_07403_amd import rdist as R  # noqa: E402


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def footprint(n, kind):
    np_ = (n + 127) // 128 * 128
    f = 8 * np_ * np_ + 4096 * np_
    return 2 * f if kind == R.RDIST_QUERY_PATHS else f


@pytest.fixture(scope="module")
def ctx():
    c = R.Context(0)
    yield c
    c.close()


def make_requests(count, stream_index, n_hi):
    reqs = gg.c5_requests(count, qps=100.0, stream_index=stream_index, n_lo=32, n_hi=n_hi, pairs_per_request=16)
    out = []
    for r in reqs:
        A = r.spec.build()
        kind = R.RDIST_QUERY_D if r.query == "D" else R.RDIST_QUERY_PATHS
        n = A.shape[0]
        item = {"id": r.rid, "A_np": A, "A": torch.from_numpy(A).cuda(), "kind": kind, "n": n,
                "info": R.PinnedInfo(1)}
        if kind == R.RDIST_QUERY_D:
            item["D"] = torch.empty((n, n), dtype=torch.int16, pin_memory=True)
        else:
            item["cur"] = torch.from_numpy(r.pairs[:, 0].copy()).pin_memory()
            item["goal"] = torch.from_numpy(r.pairs[:, 1].copy()).pin_memory()
            item["paths"] = torch.empty((len(r.pairs), 33), dtype=torch.int32, pin_memory=True)
        out.append(item)
    return out


def run_server(srv, items, timeout_s=120.0):
    for it in items:
        if it["kind"] == R.RDIST_QUERY_D:
            st = srv.submit(it["id"], it["A"], -0.5, R.RDIST_QUERY_D, D_host=it["D"], info_ptr=it["info"].at(0))
        else:
            st = srv.submit(it["id"], it["A"], -0.5, R.RDIST_QUERY_PATHS, cur_host=it["cur"], goal_host=it["goal"],
                            max_hops=32, paths_host=it["paths"], info_ptr=it["info"].at(0))
        assert st == R.RDIST_OK, R.rdist_last_error()
    done = set()
    t0 = time.time()
    while len(done) < len(items):
        done.update(srv.poll())
        assert time.time() - t0 < timeout_s, f"only {len(done)} of {len(items)} finished"
        time.sleep(0.0005)
    return done


def alone(ctx, it):
    """The request solved by itself: a batch of one (no tile cache) up to
    n = 4096, the single-graph plan above; paths from its kept Y."""
    A = it["A"]
    if it["n"] <= 4096:
        keep = it["kind"] == R.RDIST_QUERY_PATHS
        Ds, info, graphs = ctx.solve_batched([A], -0.5, flags=R.RDIST_NO_GRAPH, keep=keep)
        D, status, g = Ds[0], info.get(0).status, graphs[0] if keep else None
    else:
        D, inf, g = ctx.solve(A, -0.5, keep=it["kind"] == R.RDIST_QUERY_PATHS)
        status = inf["status"]
    paths = None
    if g is not None:
        paths = ctx.next_hop(g, it["cur"].cuda(), it["goal"].cuda(), max_hops=32)
        torch.cuda.synchronize()
        g.release()
    return D, status, paths


def test_server_mix_is_bitwise_alone(ctx):
    items = make_requests(40, stream_index=7, n_hi=1500)
    budget = 3 * footprint(1500, R.RDIST_QUERY_PATHS)
    srv = R.Server(ctx, slots=2, hbm_budget=budget, max_batch=8)
    note(f"[server] {len(items)} requests n={sorted(it['n'] for it in items)}, budget {budget >> 20} MiB")
    done = run_server(srv, items)
    st = srv.stats()
    note(f"[server] stats {st}")
    srv.close()
    assert done == {it["id"] for it in items}
    assert st["completed"] == len(items) and st["failed"] == 0
    assert st["max_footprint_in_flight"] <= budget
    # n <= 1024 always batches; a larger one batches behind a backlog and
    # runs alone (single-graph plan) when few requests wait
    n_small = sum(it["n"] <= 1024 for it in items)
    assert st["batches"] >= 2 and n_small <= st["batched_requests"] <= len(items) and st["max_in_flight"] >= 2
    # each result equals the same request solved alone
    for it in items:
        info = it["info"].get(0)
        D, status, paths = alone(ctx, it)
        assert info.status == status
        if it["kind"] == R.RDIST_QUERY_D:
            assert np.array_equal(it["D"].numpy(), D.cpu().numpy()), f"request {it['id']} n={it['n']}"
        else:
            assert np.array_equal(it["paths"].numpy(), paths.cpu().numpy()), f"request {it['id']} paths"


def test_server_large_request_takes_own_slot(ctx):
    """A request above the batched range (n = 4200) runs on a slot of its own
    beside batches; both kinds; results as alone."""
    items = make_requests(6, stream_index=9, n_hi=300)
    for kind, rid in ((R.RDIST_QUERY_D, 900001), (R.RDIST_QUERY_PATHS, 900002)):
        n = 4200
        A = gg.erdos_renyi(n, 8.0 / n, gg.rng_for("parity", 9200 + kind))
        it = {"id": rid, "A_np": A, "A": torch.from_numpy(A).cuda(), "kind": kind, "n": n, "info": R.PinnedInfo(1)}
        if kind == R.RDIST_QUERY_D:
            it["D"] = torch.empty((n, n), dtype=torch.int16, pin_memory=True)
        else:
            pairs = gg.rng_for("parity", 9210).integers(0, n, size=(64, 2)).astype(np.int32)
            it["cur"] = torch.from_numpy(pairs[:, 0].copy()).pin_memory()
            it["goal"] = torch.from_numpy(pairs[:, 1].copy()).pin_memory()
            it["paths"] = torch.empty((64, 33), dtype=torch.int32, pin_memory=True)
        items.insert(2, it)
    srv = R.Server(ctx, slots=3, hbm_budget=0, max_batch=8)
    run_server(srv, items)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(items) and st["batched_requests"] == len(items) - 2
    for it in items:
        D, status, paths = alone(ctx, it)
        assert it["info"].get(0).status == status == 0
        if it["kind"] == R.RDIST_QUERY_D:
            assert np.array_equal(it["D"].numpy(), D.cpu().numpy()), f"request {it['id']} n={it['n']}"
        else:
            assert np.array_equal(it["paths"].numpy(), paths.cpu().numpy()), f"request {it['id']} paths"


def test_server_lone_large_request_single_plan_bitwise(ctx):
    """Requests with 1024 < n <= 4096 that run alone (few requests waiting)
    take the single-graph plan, paths on the Y it leaves in the slot's
    workspace; their D and paths equal those of a batch of one (the reference
    for n <= 4096) bit for bit.  Submitted one at a time; the path requests
    back to back, so the second reuses the first one's workspace."""
    specs = ((3000, R.RDIST_QUERY_D, "er"), (2600, R.RDIST_QUERY_PATHS, "er"), (1500, R.RDIST_QUERY_PATHS, "er"),
             (4096, R.RDIST_QUERY_D, "torus"))
    srv = R.Server(ctx, slots=2, hbm_budget=0, max_batch=8)
    items = []
    for k, (n, kind, fam) in enumerate(specs):
        A = (gg.erdos_renyi(n, 10.0 / n, gg.rng_for("parity", 9300 + k)) if fam == "er"
             else gg.torus_lattice(n, "tri"))
        n = A.shape[0]
        it = {"id": 910000 + k, "A_np": A, "A": torch.from_numpy(A).cuda(), "kind": kind, "n": n,
              "info": R.PinnedInfo(1)}
        if kind == R.RDIST_QUERY_D:
            it["D"] = torch.empty((n, n), dtype=torch.int16, pin_memory=True)
        else:
            pairs = gg.rng_for("parity", 9310).integers(0, n, size=(64, 2)).astype(np.int32)
            it["cur"] = torch.from_numpy(pairs[:, 0].copy()).pin_memory()
            it["goal"] = torch.from_numpy(pairs[:, 1].copy()).pin_memory()
            it["paths"] = torch.empty((64, 33), dtype=torch.int32, pin_memory=True)
        note(f"[server] lone request n={n} kind={kind}")
        run_server(srv, [it])
        items.append(it)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(items) and st["batched_requests"] == 0, st
    for it in items:
        D, status, paths = alone(ctx, it)
        assert it["info"].get(0).status == status == 0
        if it["kind"] == R.RDIST_QUERY_D:
            assert np.array_equal(it["D"].numpy(), D.cpu().numpy()), f"request {it['id']} n={it['n']}"
        else:
            assert np.array_equal(it["paths"].numpy(), paths.cpu().numpy()), f"request {it['id']} paths"


def test_server_backlog_batches_larger_requests(ctx):
    """With more requests waiting than the server takes out of batches, the
    larger ones (1024 < n <= 4096) join the batch: one slot, all submitted
    before the first poll, so the whole backlog goes out as one batch; results
    still equal each request solved alone."""
    items = make_requests(14, stream_index=11, n_hi=1200)
    for k, n in enumerate((1500, 1800)):
        A = gg.erdos_renyi(n, 8.0 / n, gg.rng_for("parity", 9400 + k))
        it = {"id": 920000 + k, "A_np": A, "A": torch.from_numpy(A).cuda(), "kind": R.RDIST_QUERY_D, "n": n,
              "info": R.PinnedInfo(1), "D": torch.empty((n, n), dtype=torch.int16, pin_memory=True)}
        items.append(it)
    srv = R.Server(ctx, slots=1, hbm_budget=0, max_batch=64)
    run_server(srv, items)
    st = srv.stats()
    srv.close()
    note(f"[server] backlog stats {st}")
    assert st["completed"] == len(items) and st["batches"] == 1 and st["batched_requests"] == len(items), st
    for it in items:
        D, status, paths = alone(ctx, it)
        assert it["info"].get(0).status == status == 0
        if it["kind"] == R.RDIST_QUERY_D:
            assert np.array_equal(it["D"].numpy(), D.cpu().numpy()), f"request {it['id']} n={it['n']}"
        else:
            assert np.array_equal(it["paths"].numpy(), paths.cpu().numpy()), f"request {it['id']} paths"


def test_server_reports_small_requests_of_a_batch_first(ctx):
    """One batch holding a larger graph and small ones: requests are reported
    group by group (n <= 128 first, then by ceil(n / 128)), and every result
    still equals the request solved alone.  (Sizes up to 1024: with this few
    requests waiting, larger ones would run alone.)"""
    items = []
    sizes = [1000, 70, 300, 900, 100, 600, 64]
    for k, n in enumerate(sizes):
        A = gg.erdos_renyi(n, min(1.0, 8.0 / n), gg.rng_for("parity", 9300 + k))
        kind = R.RDIST_QUERY_PATHS if k % 2 else R.RDIST_QUERY_D
        it = {"id": 500 + k, "A_np": A, "A": torch.from_numpy(A).cuda(), "kind": kind, "n": n,
              "info": R.PinnedInfo(1)}
        if kind == R.RDIST_QUERY_D:
            it["D"] = torch.empty((n, n), dtype=torch.int16, pin_memory=True)
        else:
            pairs = gg.rng_for("parity", 9310 + k).integers(0, n, size=(16, 2)).astype(np.int32)
            it["cur"] = torch.from_numpy(pairs[:, 0].copy()).pin_memory()
            it["goal"] = torch.from_numpy(pairs[:, 1].copy()).pin_memory()
            it["paths"] = torch.empty((16, 33), dtype=torch.int32, pin_memory=True)
        items.append(it)
    srv = R.Server(ctx, slots=1, hbm_budget=0, max_batch=16)
    for it in items:
        if it["kind"] == R.RDIST_QUERY_D:
            assert srv.submit(it["id"], it["A"], -0.5, R.RDIST_QUERY_D, D_host=it["D"],
                              info_ptr=it["info"].at(0)) == R.RDIST_OK
        else:
            assert srv.submit(it["id"], it["A"], -0.5, R.RDIST_QUERY_PATHS, cur_host=it["cur"],
                              goal_host=it["goal"], max_hops=32, paths_host=it["paths"],
                              info_ptr=it["info"].at(0)) == R.RDIST_OK
    order = []
    t0 = time.time()
    while len(order) < len(items):
        order.extend(srv.poll())
        assert time.time() - t0 < 60
        time.sleep(0.0002)
    st = srv.stats()
    srv.close()
    assert st["batches"] == 1 and st["completed"] == len(items)
    group = {it["id"]: (0 if it["n"] <= 128 else (it["n"] + 127) // 128) for it in items}
    note(f"[server] report order {[(i, group[i]) for i in order]}")
    gs = [group[i] for i in order]
    assert gs == sorted(gs)
    for it in items:
        D, status, paths = alone(ctx, it)
        assert it["info"].get(0).status == status == 0
        if it["kind"] == R.RDIST_QUERY_D:
            assert np.array_equal(it["D"].numpy(), D.cpu().numpy()), f"request {it['id']} n={it['n']}"
        else:
            assert np.array_equal(it["paths"].numpy(), paths.cpu().numpy()), f"request {it['id']} paths"


def test_server_oracle_spot_checks(ctx):
    items = make_requests(12, stream_index=8, n_hi=400)
    srv = R.Server(ctx, slots=3, hbm_budget=0, max_batch=4)
    run_server(srv, items)
    srv.close()
    for it in items[::3]:
        if it["kind"] != R.RDIST_QUERY_D:
            continue
        sol = oracle.solve(it["A_np"], -0.5, keep_y=False)
        assert it["info"].get(0).status == sol.status
        assert np.array_equal(it["D"].numpy(), sol.D)


def test_server_refuses_what_never_fits(ctx):
    srv = R.Server(ctx, slots=2, hbm_budget=footprint(256, R.RDIST_QUERY_D), max_batch=4)
    A = torch.from_numpy(gg.erdos_renyi(600, 0.02, gg.rng_for("parity", 9100))).cuda()
    D = torch.empty((600, 600), dtype=torch.int16, pin_memory=True)
    assert srv.submit(1, A, -0.5, R.RDIST_QUERY_D, D_host=D) == R.RDIST_E_NOMEM
    assert srv.submit(2, A, 1.5, R.RDIST_QUERY_D, D_host=D) == R.RDIST_E_ARG
    srv.close()
