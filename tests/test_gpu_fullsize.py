"""GPU parity at the full sizes of the benchmark workloads, launched the way
bench.py launches them.  Where the oracle finishes the whole workload in
seconds every register is compared; otherwise a sample of outputs, each
computed by the oracle on its own, plus properties that hold at any size.

* document batch: 10^4 vectors (8.1x10^6 entries), k = 256 and 1024, every
  register of the FastGM form; the plain form on sampled vectors; the 5,000
  Jaccard pairs, every estimate.
* stream vector: n+ = 10^7, k = 1024 and 4096, every register; the
  weighted-cardinality estimate over 100 sketch seeds is unbiased within
  4 sqrt(1/((k-2) 100)) (Theorem 2), and two seeds' estimates equal the
  oracle's.
* uneven batch: 10^5 vectors (4.7x10^8 entries), per-vector k, autotuned and
  replayed from a captured graph; every register.  The plain form through
  the batched call on a seeded 1% sample, every register.
* stream vector, plain form at k = 1024: every register.
* serving: a store of 10^6 sketches at k = 512 and 20,000 requests; sampled
  stored rows, sketch requests and Jaccard answers.

Register indices and values are compared bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2302_05176_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = "cuda:0"


@pytest.fixture(scope="module")
def gm():
    import paper_2302_05176_amd as gm
    assert torch.cuda.is_available()
    gm.reset_options()
    oracle.build()
    oracle.set_threads(16)
    yield gm
    gm.reset_options()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _same(got_s, got_y, want_s, want_y, what):
    bad = np.argwhere(got_s != want_s)
    assert bad.size == 0, f"{what}: {len(bad)} index mismatches, first at {bad[:3].tolist()}"
    gb = np.ascontiguousarray(got_y).view(np.uint64)
    wb = np.ascontiguousarray(want_y).view(np.uint64)
    badv = np.argwhere(gb != wb)
    assert badv.size == 0, f"{what}: {len(badv)} value mismatches, first at {badv[:3].tolist()}"


def _bench_step(gm, ti, tw, to, k, seed, form, oi, ov):
    # the timed step of the document-batch bench: preallocated outputs,
    # events around the sketch kernels (timing level 2)
    gm.set_option("timing", 2)
    try:
        gm.sketch(ti, tw, to, k, seed, form=form, out_idx=oi, out_val=ov)
        torch.cuda.synchronize()
    finally:
        gm.set_option("timing", 0)
        gm.reset_timing()
    return oi.cpu().numpy(), ov.cpu().numpy()


def test_document_batch_full(gm):
    nvec, seed = 10000, 1
    idx, w, off = W.batch(nvec=nvec, seed=1002)
    ti, tw, to = _dev(idx), _dev(w), _dev(off)
    rng = np.random.default_rng(77)
    sample = np.sort(rng.choice(nvec, 40, replace=False))
    for k in (256, 1024):
        oi = torch.empty((nvec, k), dtype=torch.int32, device=DEV)
        ov = torch.empty((nvec, k), dtype=torch.float64, device=DEV)
        print(f"document batch 10^4 vectors k={k} fastgm, every register", flush=True)
        gs, gy = _bench_step(gm, ti, tw, to, k, seed, "fastgm", oi, ov)
        ws, wy = oracle.sketch(idx, w, off, k, seed, form=oracle.FORM_STREAM)
        _same(gs, gy, ws, wy, f"fastgm k={k}")
        print(f"document batch 10^4 vectors k={k} plain, 40 sampled vectors", flush=True)
        gs, gy = _bench_step(gm, ti, tw, to, k, seed, "plain", oi, ov)
        for v in sample:
            a, b = off[v], off[v + 1]
            ws, wy = oracle.sketch(idx[a:b], w[a:b], np.array([0, b - a]), k, seed,
                                   form=oracle.FORM_PLAIN)
            _same(gs[v], gy[v], ws[0], wy[0], f"plain k={k} vector {v}")


def test_document_pairs_full(gm):
    k, seed = 256, 1
    idx, w, off, _ = W.pairs(npairs=5000)
    print("5000 Jaccard pairs k=256", flush=True)
    s, _ = gm.sketch(_dev(idx), _dev(w), _dev(off), k, seed)
    est = gm.jaccard_est(s[0::2].contiguous(), s[1::2].contiguous()).cpu().numpy()
    os_, _ = oracle.sketch(idx, w, off, k, seed, form=oracle.FORM_STREAM)
    want = np.array([oracle.jaccard(os_[2 * p], os_[2 * p + 1]) for p in range(5000)])
    assert np.array_equal(est, want)


@pytest.mark.parametrize("k", [1024, 4096])
def test_stream_vector_full(gm, k):
    idx, w, off = W.stream(nplus=10_000_000)
    ti, tw, to = _dev(idx), _dev(w), _dev(off)
    print(f"stream vector n+=10^7 k={k}, every register", flush=True)
    s, y = gm.sketch(ti, tw, to, k, 1)
    ws, wy = oracle.sketch(idx, w, off, k, 1, form=oracle.FORM_STREAM)
    _same(s.cpu().numpy(), y.cpu().numpy(), ws, wy, f"k={k}")
    # Theorem 2 over 100 sketch seeds, against the exact sum of the weights
    S = float(np.sum(w.astype(np.float64)))
    ests = []
    for seed in range(1, 101):
        _, ys = gm.sketch(ti, tw, to, k, seed)
        ests.append(float(gm.wcard_est(ys).item()))
        if seed in (2, 3):
            _, oy = oracle.sketch(idx, w, off, k, seed, form=oracle.FORM_STREAM)
            assert ests[-1] == oracle.wcard(oy[0]), f"seed {seed}"
    r = np.array(ests) / S
    assert abs(r.mean() - 1.0) < 4.0 * np.sqrt(1.0 / ((k - 2) * 100))


def _rows_of(off, vs):
    """Entry positions of vectors vs, concatenated, and their CSR offsets."""
    lens = (off[vs + 1] - off[vs]).astype(np.int64)
    sub = np.zeros(len(vs) + 1, np.int64)
    np.cumsum(lens, out=sub[1:])
    pos = np.repeat(off[vs] - sub[:-1], lens) + np.arange(sub[-1], dtype=np.int64)
    return pos, sub


def _regs_of(outoff, vs, kv):
    """Flat register positions of vectors vs (each with kv registers)."""
    return (outoff[vs][:, None] + np.arange(kv, dtype=np.int64)[None, :])


@pytest.mark.timeout(900)
def test_uneven_batch_full(gm, tmp_path, monkeypatch):
    """Every register of the 10^5-vector uneven batch (autotuned, replayed
    from a captured graph) against the oracle, one oracle call per k."""
    monkeypatch.setenv("GM_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    nvec, seed = 100_000, 1
    print("uneven batch: generating 10^5 vectors", flush=True)
    idx, w, off, kk = W.uneven(nvec=nvec)
    outoff = np.zeros(nvec + 1, np.int64)
    np.cumsum(kk, out=outoff[1:])
    ti, tw, to, tk, too = _dev(idx), _dev(w), _dev(off), _dev(kk), _dev(outoff)
    total = int(outoff[-1])
    oi = torch.empty(total, dtype=torch.int32, device=DEV)
    ov = torch.empty(total, dtype=torch.float64, device=DEV)
    print("uneven batch: autotune, capture, replay", flush=True)
    s = torch.cuda.Stream()
    try:
        with torch.cuda.stream(s):
            gm.reserve(nvec, stream=s)
            gm.autotune(ti, tw, to, 4096, seed, k_per_vec=tk, out_offsets=too, out_idx=oi,
                        out_val=ov, reps=1, stream=s)
        s.synchronize()
        oi.fill_(0)
        ov.fill_(0.0)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            gm.sketch_batched(ti, tw, to, tk, too, 4096, seed, out_idx=oi, out_val=ov,
                              stream=torch.cuda.current_stream())
        g.replay()
        torch.cuda.synchronize()
    finally:
        gm.reset_options()
    gs_all, gy_all = oi.cpu().numpy(), ov.cpu().numpy()
    del oi, ov
    for kv in (64, 256, 1024, 4096):
        vs = np.nonzero(kk == kv)[0]
        pos, sub = _rows_of(off, vs)
        print(f"uneven batch: oracle on the {len(vs)} vectors with k={kv}", flush=True)
        ws, wy = oracle.sketch(idx[pos], w[pos], sub, kv, seed, form=oracle.FORM_STREAM)
        r = _regs_of(outoff, vs, kv)
        _same(gs_all[r], gy_all[r], ws, wy, f"k={kv}")


@pytest.mark.timeout(600)
def test_uneven_batch_plain_sample(gm):
    """The plain form through gm_sketch_batched on a seeded 1% sample of the
    uneven batch (1000 vectors, all four k), every register."""
    nvec, seed = 100_000, 1
    idx, w, off, kk = W.uneven(nvec=nvec)
    rng = np.random.default_rng(80)
    vs = np.sort(rng.choice(nvec, nvec // 100, replace=False))
    pos, sub = _rows_of(off, vs)
    si, sw, sk = idx[pos], w[pos], kk[vs]
    outoff = np.zeros(len(vs) + 1, np.int64)
    np.cumsum(sk, out=outoff[1:])
    print(f"uneven batch plain: {len(vs)} sampled vectors, {int(sub[-1])} entries", flush=True)
    gs, gy = gm.sketch_batched(_dev(si), _dev(sw), _dev(sub), _dev(sk), _dev(outoff), 4096, seed,
                               form="plain")
    torch.cuda.synchronize()
    gs, gy = gs.cpu().numpy(), gy.cpu().numpy()
    for kv in (64, 256, 1024, 4096):
        loc = np.nonzero(sk == kv)[0]
        p2, s2 = _rows_of(sub, loc)
        print(f"uneven batch plain: oracle on {len(loc)} vectors k={kv}", flush=True)
        ws, wy = oracle.sketch(si[p2], sw[p2], s2, kv, seed, form=oracle.FORM_PLAIN)
        r = _regs_of(outoff, loc, kv)
        _same(gs[r], gy[r], ws, wy, f"plain k={kv}")


@pytest.mark.timeout(600)
def test_stream_vector_plain_full(gm):
    """The plain form of the 10^7-entry stream vector at k = 1024, launched as
    bench.py times it (entries split over the GPU, minima merged), every
    register; the oracle sketches 64 ranges in parallel and merges them
    (Sec. 2.3, pinned to the sketch of the union)."""
    idx, w, off = W.stream(nplus=10_000_000)
    k, seed = 1024, 1
    print("stream vector n+=10^7 k=1024 plain form", flush=True)
    s, y = gm.sketch(_dev(idx), _dev(w), _dev(off), k, seed, form="plain")
    torch.cuda.synchronize()
    print("stream vector plain: oracle, 64 ranges on 16 threads", flush=True)
    cut = np.linspace(0, len(idx), 65).astype(np.int64)
    ps, py = oracle.sketch(idx, w, cut, k, seed, form=oracle.FORM_PLAIN)
    ws, wy = oracle.merge(ps, py)
    _same(s.cpu().numpy()[0], y.cpu().numpy()[0], ws, wy, "plain k=1024")


def test_serving_full_sampled(gm):
    from paper_2302_05176_amd import serve
    from test_gpu_serve import oracle_store
    nstore, k, seed = 1_000_000, 512, 1
    print("serving: store of 10^6 sketches k=512", flush=True)
    store = serve.build_store(nstore, k)
    reqs, hi, hw = serve.make_trace(20_000, rate=20_000.0, nstore=nstore)
    print("serving: 20,000 requests", flush=True)
    res = serve.run(reqs, hi, hw, store, k, seed=seed, slots=8, max_batch_requests=256,
                    max_wait_us=0.0, device_budget_bytes=4 << 30, want_sketches=True)
    st = res["stats"]
    assert st["sketch_requests"] + st["jaccard_requests"] == len(reqs)
    assert np.all(res["latency_us"] > 0)
    rng = np.random.default_rng(79)
    # sampled Jaccard answers and stored rows, from the oracle's sketches of
    # the store's seeded vectors
    jq = np.nonzero(reqs["kind"] == serve.JACCARD)[0]
    jq = rng.choice(jq, 300, replace=False)
    want_rows = oracle_store(nstore, k, rows=np.concatenate([reqs["a"][jq], reqs["b"][jq]]))
    for r in jq:
        want = oracle.jaccard(want_rows[int(reqs["a"][r])], want_rows[int(reqs["b"][r])])
        assert res["jaccard"][r] == want, f"query {r}"
    some = sorted(want_rows)[:50]
    got = store[_dev(np.array(some, np.int64))].cpu().numpy()
    for i, r in enumerate(some):
        assert np.array_equal(got[i], want_rows[r]), f"stored row {r}"
    # sampled sketch requests
    sk = np.nonzero(reqs["kind"] == serve.SKETCH)[0]
    sizes = reqs["b"][sk] - reqs["a"][sk]
    # 40 sampled sketch requests and the largest (big-vector passes)
    for row in set(rng.choice(len(sk), 40, replace=False).tolist()) | {int(np.argmax(sizes))}:
        r = sk[row]
        a, b = int(reqs["a"][r]), int(reqs["b"][r])
        ws, wy = oracle.sketch(hi[a:b], hw[a:b], np.array([0, b - a]), k, seed)
        _same(res["sketch_idx"][row], res["sketch_val"][row], ws[0], wy[0], f"request {r}")
