"""GPU: the continuous-batching serving loop.  Each sketch produced in the
overlapped, batched run equals the same request sketched alone (and the
oracle's); each Jaccard answer equals the oracle's estimate on the stored
rows; every request completes after it arrives."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def oracle_store(nstore, k, rows=None, seed=1006, nplus=32):
    """The oracle's sketches (indices) of the store's seeded vectors, for the
    given rows (all when None); a dictionary row -> indices when rows are
    given."""
    from paper_2302_05176_amd import serve
    parts = list(serve.store_vectors(nstore, seed, nplus))
    vi = np.concatenate([c[1] for c in parts])
    vw = np.concatenate([c[2] for c in parts])
    sel = np.arange(nstore) if rows is None else np.unique(np.asarray(rows, np.int64))
    off = np.arange(len(sel) + 1, dtype=np.int64) * nplus
    s, _ = oracle.sketch(vi[sel].reshape(-1), vw[sel].reshape(-1), off, k, seed)
    return s if rows is None else {int(r): s[i] for i, r in enumerate(sel)}


def test_serving_results_same_alone_and_in_the_mix():
    import paper_2302_05176_amd as gm
    from paper_2302_05176_amd import serve
    k, nstore = 128, 3000
    store = serve.build_store(nstore, k)
    # arrivals faster than a batch completes: requests queue while others run
    reqs, hi, hw = serve.make_trace(400, rate=400_000.0, nstore=nstore, size_mu=np.log(300.0),
                                    size_sigma=1.0, size_cap=20_000)
    res = serve.run(reqs, hi, hw, store, k, seed=7, slots=4, max_batch_requests=32,
                    max_wait_us=0.0, want_sketches=True, device_budget_bytes=8 << 30)
    st = res["stats"]
    assert st["sketch_requests"] + st["jaccard_requests"] == len(reqs)
    # batches overlapped on the device, and batches held several requests
    assert st["max_slots_busy"] >= 2, st
    assert 1 < st["batches"] < len(reqs), st
    assert st["max_inflight_bytes"] <= 8 << 30
    assert np.all(res["latency_us"] > 0)
    sk = np.nonzero(reqs["kind"] == serve.SKETCH)[0]
    # alone: every sketch request on its own
    for row, r in enumerate(sk):
        a, b = int(reqs["a"][r]), int(reqs["b"][r])
        t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
        s1, y1 = gm.sketch(t(hi[a:b]), t(hw[a:b]), t(np.array([0, b - a], np.int64)), k, 7)
        assert np.array_equal(s1.cpu().numpy()[0], res["sketch_idx"][row]), f"request {r}"
        assert np.array_equal(y1.cpu().numpy()[0].view(np.uint64),
                              res["sketch_val"][row].view(np.uint64)), f"request {r}"
    # the oracle on a sample
    for row in range(0, len(sk), 17):
        r = sk[row]
        a, b = int(reqs["a"][r]), int(reqs["b"][r])
        os_, oy = oracle.sketch(hi[a:b], hw[a:b], np.array([0, b - a]), k, 7)
        assert np.array_equal(os_[0], res["sketch_idx"][row])
    # Jaccard answers against the oracle's sketches of the stored vectors
    want_store = oracle_store(nstore, k)
    jq = np.nonzero(reqs["kind"] == serve.JACCARD)[0]
    for r in jq:
        want = oracle.jaccard(want_store[reqs["a"][r]], want_store[reqs["b"][r]])
        assert res["jaccard"][r] == want, f"query {r}"
    summ = serve.summarize(reqs, res)
    assert summ["p99_us"] >= summ["p50_us"] > 0


def test_serving_admission_counts_the_workspace():
    """The device budget bounds what is in flight, the library workspace of
    each slot stream included: with room for two slots only, at most two
    batches run at once and the in-flight bytes stay within the budget."""
    import paper_2302_05176_amd as gm
    from paper_2302_05176_amd import serve
    k, nstore = 64, 500
    store = serve.build_store(nstore, k)
    reqs, hi, hw = serve.make_trace(300, rate=400_000.0, nstore=nstore, size_mu=np.log(200.0),
                                    size_sigma=0.5, size_cap=2_000)
    R = 16
    ws = gm.workspace_bytes(R)
    assert ws > 128 << 20          # the candidate pool alone is 128 MiB
    probe = serve.run(reqs[:5], hi, hw, store, k, seed=3, slots=1, max_batch_requests=R,
                      max_batch_entries=1 << 14, device_budget_bytes=64 << 30)
    slot = probe["stats"]["slot_bytes"]
    assert probe["stats"]["workspace_bytes"] == ws and slot > ws
    budget = 2 * slot + slot // 2
    res = serve.run(reqs, hi, hw, store, k, seed=3, slots=6, max_batch_requests=R,
                    max_batch_entries=1 << 14, device_budget_bytes=budget)
    st = res["stats"]
    assert st["slots"] == 2, st
    assert st["max_slots_busy"] <= 2 and st["max_inflight_bytes"] <= budget, st
    assert st["sketch_requests"] + st["jaccard_requests"] == len(reqs)
    # a budget below one slot is refused
    with pytest.raises(gm.GMError):
        serve.run(reqs[:5], hi, hw, store, k, seed=3, slots=1, max_batch_requests=R,
                  max_batch_entries=1 << 14, device_budget_bytes=slot - 1)
