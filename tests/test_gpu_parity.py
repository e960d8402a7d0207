"""GPU parity: the HIP kernels against the CPU oracle, element by element.

Register indices must match bit for bit; register values are compared bit
for bit too (the draw specification is a fixed sequence of IEEE operations,
so both sides compute identical doubles; the stated tolerance of 1e-15
relative is therefore met with zero error).  Estimates are compared bit for
bit as well (same operations, same order).
"""
import numpy as np
import pytest

import oracle
from paper_2302_05176_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gm():
    import paper_2302_05176_amd as gm
    from paper_2302_05176_amd import build
    if not build.up_to_date():
        build.build(force=True)
    assert torch.cuda.is_available()
    gm.reset_options()
    yield gm
    gm.reset_options()


DEV = "cuda:0"


def _gpu_sketch(gm, idx, w, off, k, seed, form="fastgm"):
    ti = torch.from_numpy(np.ascontiguousarray(idx, np.int32)).to(DEV)
    tw = torch.from_numpy(np.ascontiguousarray(w, np.float32)).to(DEV)
    to = torch.from_numpy(np.ascontiguousarray(off, np.int64)).to(DEV)
    s, y = gm.sketch(ti, tw, to, k, seed, form=form)
    torch.cuda.synchronize()
    return s.cpu().numpy(), y.cpu().numpy()


def _assert_same(got, want, what=""):
    gs, gy = got
    ws, wy = want
    bad = np.argwhere(gs != ws)
    assert bad.size == 0, f"{what}: {len(bad)} index mismatches, first at {bad[:3].tolist()}"
    gb = np.ascontiguousarray(gy).view(np.uint64)
    wb = np.ascontiguousarray(wy).view(np.uint64)
    badv = np.argwhere(gb != wb)
    assert badv.size == 0, f"{what}: {len(badv)} value mismatches, first at {badv[:3].tolist()}"


def test_single_vector_both_forms(gm):
    idx, w, off = W.single(nplus=1000)
    for form, of in (("fastgm", oracle.FORM_STREAM), ("plain", oracle.FORM_PLAIN)):
        print(f"single vector n+=1000 k=128 form={form}", flush=True)
        _assert_same(_gpu_sketch(gm, idx, w, off, 128, 1, form),
                     oracle.sketch(idx, w, off, 128, 1, form=of), form)


@pytest.mark.parametrize("k", [1, 2, 3, 7, 64, 256, 1000, 4096])
def test_fastgm_mixed_batch(gm, k):
    max_n = 3000 if k <= 256 else 800
    idx, w, off = W.mixed(seed=200 + k, nvec=48, max_n=max_n)
    print(f"mixed batch k={k}", flush=True)
    _assert_same(_gpu_sketch(gm, idx, w, off, k, 17 + k),
                 oracle.sketch(idx, w, off, k, 17 + k, form=oracle.FORM_STREAM), f"k={k}")


@pytest.mark.parametrize("k", [1, 5, 64, 300])
def test_plain_mixed_batch(gm, k):
    idx, w, off = W.mixed(seed=300 + k, nvec=32, max_n=1200)
    print(f"plain mixed batch k={k}", flush=True)
    _assert_same(_gpu_sketch(gm, idx, w, off, k, 5, "plain"),
                 oracle.sketch(idx, w, off, k, 5, form=oracle.FORM_PLAIN), f"plain k={k}")


def test_document_batch_k256(gm):
    idx, w, off = W.batch(nvec=400, seed=1202)
    oracle.set_threads(8)
    print("document batch 400 vectors k=256 fastgm", flush=True)
    _assert_same(_gpu_sketch(gm, idx, w, off, 256, 1),
                 oracle.sketch(idx, w, off, 256, 1, form=oracle.FORM_STREAM), "batch fastgm")
    print("document batch 60 vectors k=256 plain", flush=True)
    o2 = off[:61]
    _assert_same(_gpu_sketch(gm, idx, w, o2, 256, 1, "plain"),
                 oracle.sketch(idx, w, o2, 256, 1, form=oracle.FORM_PLAIN), "batch plain")


@pytest.mark.parametrize("opt,val", [("pos_bits", 60), ("pos_bits", 40), ("map_load", 0),
                                     ("map_load", 2), ("map_load", 16), ("t0_scale_ppm", 1),
                                     ("t0_scale_ppm", 100_000), ("republish", 1),
                                     ("republish", 64), ("seg_rest", 0),
                                     ("seg_rest", 1000000), ("wave_lim", 0),
                                     ("wave_lim", 15), ("wave_lim", 32767)])
def test_forced_internal_paths(gm, opt, val):
    """Debug knobs force packed-prefix contests (exact re-resolution), the
    wave-cooperative heavy path, the enlarge-and-repeat fallback and other
    threshold schedules; none may change the sketch."""
    idx, w, off = W.mixed(seed=404, nvec=40, max_n=1500)
    try:
        gm.set_option(opt, val)
        for k in (16, 512):
            print(f"forced {opt}={val} k={k}", flush=True)
            _assert_same(_gpu_sketch(gm, idx, w, off, k, 9),
                         oracle.sketch(idx, w, off, k, 9, form=oracle.FORM_STREAM),
                         f"{opt}={val} k={k}")
    finally:
        gm.reset_options()


def test_heavy_single_elements_large_k(gm):
    rows_i, rows_w = [], []
    rng = np.random.default_rng(9)
    for n in (1, 2, 3, 10, 50):
        rows_i.append(np.sort(rng.choice(1 << 24, n, replace=False)))
        ww = rng.lognormal(0, 2, size=n).astype(np.float32)
        rows_w.append(ww)
    idx, w, off = W._pack(rows_i, rows_w)
    for k in (4096, 2049):
        print(f"heavy small vectors k={k}", flush=True)
        _assert_same(_gpu_sketch(gm, idx, w, off, k, 3),
                     oracle.sketch(idx, w, off, k, 3, form=oracle.FORM_STREAM), f"k={k}")


def test_poisoned_vectors_and_error_counter(gm):
    idx = np.array([1, 2, 3, 4, 5, -6, 7, 8, 9, 10], np.int32)
    w = np.array([1, np.nan, 1, -2, 1, 1, np.inf, 1, 0, 2], np.float32)
    # rows: NaN weight, negative weight, negative index, inf weight, decreasing
    # offsets, and an overlapping row that again holds -6 and inf
    off = np.array([0, 2, 4, 6, 7, 5, 10], np.int64)
    gm.reset_data_errors()
    for form, of in (("fastgm", oracle.FORM_STREAM), ("plain", oracle.FORM_PLAIN)):
        got = _gpu_sketch(gm, idx, w, off, 32, 1, form)
        want = oracle.sketch(idx, w, off, 32, 1, form=of)
        assert np.array_equal(got[0], want[0])
        assert np.array_equal(np.isnan(got[1]), np.isnan(want[1]))
        fin = ~np.isnan(want[1])
        assert np.array_equal(got[1][fin].view(np.uint64), want[1][fin].view(np.uint64))
        assert np.all(got[0] == -2)          # every row holds a bad entry or bad offsets
    assert gm.get_data_errors() == 2 * 6
    gm.reset_data_errors()
    assert gm.get_data_errors() == 0


def test_big_vector_poison(gm):
    """Vectors above the 32768-entry limit are validated by the grid-wide
    passes: a negative index (found by the probe pass) or a NaN weight (the
    sum pass) poisons only its own vector; the clean big vector beside them,
    whose probe rejects most entries in single precision, equals the oracle."""
    rng = np.random.default_rng(404)
    rows_i, rows_w = [], []
    for v in range(3):
        n = 40_000 + 1000 * v
        rows_i.append(rng.choice(1 << 24, size=n, replace=False).astype(np.int32))
        rows_w.append(rng.exponential(1.0, size=n).astype(np.float32) + np.float32(1e-3))
    rows_i[1][20_000] = -5
    rows_w[2][33_333] = np.nan
    # no positive weight: with a negative index poisoned, without it empty
    for v in (3, 4):
        rows_i.append(rng.choice(1 << 24, size=36_000, replace=False).astype(np.int32))
        rows_w.append(np.zeros(36_000, np.float32))
    rows_i[3][35_999] = -1
    idx, w, off = W._pack(rows_i, rows_w)
    gm.reset_data_errors()
    for k in (64, 1024):
        print(f"big vectors with a bad index / NaN weight / no weight, k={k}", flush=True)
        got = _gpu_sketch(gm, idx, w, off, k, 8)
        want = oracle.sketch(idx, w, off, k, 8, form=oracle.FORM_STREAM)
        assert np.all(got[0][1:4] == -2) and np.all(np.isnan(got[1][1:4]))
        assert np.all(got[0][4] == -1) and np.all(np.isinf(got[1][4]))
        _assert_same((got[0][:1], got[1][:1]), (want[0][:1], want[1][:1]), f"clean k={k}")
        assert np.array_equal(got[0], want[0])
    assert gm.get_data_errors() == 6
    gm.reset_data_errors()


def test_empty_inputs(gm):
    # nvec = 0: nothing launched
    z = torch.zeros(0, dtype=torch.int32, device=DEV)
    s, y = gm.sketch(z, z.float(), torch.zeros(1, dtype=torch.int64, device=DEV), 8, 1)
    assert s.shape == (0, 8)
    # empty rows and all-zero rows
    idx = np.array([4, 5], np.int32)
    w = np.array([0.0, 0.0], np.float32)
    off = np.array([0, 0, 2, 2], np.int64)
    for form in ("fastgm", "plain"):
        s, y = _gpu_sketch(gm, idx, w, off, 64, 1, form)
        assert np.all(s == -1) and np.all(np.isinf(y))


def test_invalid_arguments_rejected(gm):
    t = torch.zeros(4, dtype=torch.int32, device=DEV)
    off = torch.tensor([0, 4], dtype=torch.int64, device=DEV)
    with pytest.raises(gm.GMError):
        gm.sketch(t, t.float(), off, 0, 1)
    with pytest.raises(gm.GMError):
        gm.sketch(t, t.float(), off, gm.GM_K_MAX + 1, 1)


def test_batched_mixed_k(gm):
    idx, w, off, kk = W.uneven(nvec=120, seed=77, size_cap=2500)
    outoff = np.zeros(len(kk) + 1, np.int64)
    np.cumsum(kk, out=outoff[1:])
    t = lambda a: torch.from_numpy(a).to(DEV)
    for form, of in (("fastgm", oracle.FORM_STREAM),):
        print(f"batched mixed k form={form}", flush=True)
        s, y = gm.sketch_batched(t(idx), t(w), t(off), t(kk), t(outoff), int(kk.max()), 11,
                                 form=form)
        torch.cuda.synchronize()
        s, y = s.cpu().numpy(), y.cpu().numpy()
        for kv in np.unique(kk):
            vs = np.nonzero(kk == kv)[0]
            rows_i = [idx[off[v]:off[v + 1]] for v in vs]
            rows_w = [w[off[v]:off[v + 1]] for v in vs]
            si, sw, so = W._pack(rows_i, rows_w)
            ws, wy = oracle.sketch(si, sw, so, int(kv), 11, form=of)
            gs = np.stack([s[outoff[v]:outoff[v + 1]] for v in vs])
            gy = np.stack([y[outoff[v]:outoff[v + 1]] for v in vs])
            _assert_same((gs, gy), (ws, wy), f"k={kv}")


def test_batched_plain_small(gm):
    idx, w, off, kk = W.uneven(nvec=24, seed=78, size_cap=400, ks=(8, 64, 200))
    outoff = np.zeros(len(kk) + 1, np.int64)
    np.cumsum(kk, out=outoff[1:])
    t = lambda a: torch.from_numpy(a).to(DEV)
    s, y = gm.sketch_batched(t(idx), t(w), t(off), t(kk), t(outoff), 200, 12, form="plain")
    torch.cuda.synchronize()
    s, y = s.cpu().numpy(), y.cpu().numpy()
    for v in range(len(kk)):
        ws, wy = oracle.sketch(idx[off[v]:off[v + 1]], w[off[v]:off[v + 1]],
                               np.array([0, off[v + 1] - off[v]]), int(kk[v]), 12,
                               form=oracle.FORM_PLAIN)
        _assert_same((s[outoff[v]:outoff[v + 1]][None], y[outoff[v]:outoff[v + 1]][None]),
                     (ws, wy), f"v={v}")


@pytest.mark.parametrize("k", [2, 3, 17, 1024, 1025, 4099, 9001])
def test_wcard_widths(gm, k):
    """The weighted-cardinality sum is staged through LDS 1024 registers at
    a time and added 16 per step with a tail: widths around both edges, with
    values spread over many binades so that the order of the additions shows,
    must give the oracle's left-to-right sum bit for bit."""
    rng = np.random.default_rng(k)
    y = np.exp(rng.uniform(-30.0, 5.0, size=(5, k)))
    C = gm.wcard_est(torch.from_numpy(y).to(DEV)).cpu().numpy()
    Co = np.array([oracle.wcard(y[r]) for r in range(len(y))])
    assert np.array_equal(C.view(np.uint64), Co.view(np.uint64)), f"k={k}"


def test_estimators_match_oracle(gm):
    idx, w, off, frac = W.pairs(npairs=200, seed=31)
    k = 256
    s, y = _gpu_sketch(gm, idx, w, off, k, 2)
    a = torch.from_numpy(s[0::2].copy()).to(DEV)
    b = torch.from_numpy(s[1::2].copy()).to(DEV)
    J = gm.jaccard_est(a, b).cpu().numpy()
    # end to end on each side: the oracle's estimates of the oracle's sketches
    os_, oy = oracle.sketch(idx, w, off, k, 2, form=oracle.FORM_STREAM)
    Jo = np.array([oracle.jaccard(os_[2 * p], os_[2 * p + 1]) for p in range(200)])
    assert np.array_equal(J.view(np.uint64), Jo.view(np.uint64))
    C = gm.wcard_est(torch.from_numpy(y).to(DEV)).cpu().numpy()
    Co = np.array([oracle.wcard(oy[v]) for v in range(len(oy))])
    assert np.array_equal(C.view(np.uint64), Co.view(np.uint64))
    # store lookups, including out-of-range rows
    store = torch.from_numpy(s).to(DEV)
    ia = torch.tensor([0, 2, 5, -1, 10**6], dtype=torch.int64, device=DEV)
    ib = torch.tensor([1, 3, 5, 0, 1], dtype=torch.int64, device=DEV)
    gm.reset_data_errors()
    Jp = gm.jaccard_est_pairs(store, ia, ib).cpu().numpy()
    assert Jp[0] == Jo[0] and Jp[1] == Jo[1] and Jp[2] == 1.0
    assert np.isnan(Jp[3]) and np.isnan(Jp[4])
    assert gm.get_data_errors() == 2
    gm.reset_data_errors()


def test_merge_equals_sketch_of_union(gm):
    idx, w, off = W.batch(nvec=1, seed=55, sizes=np.array([3000]))
    k = 512
    whole = _gpu_sketch(gm, idx, w, off, k, 4)
    parts_off = np.array([0, 1000, 1700, 3000], np.int64)
    ps, py = _gpu_sketch(gm, idx, w, parts_off, k, 4)
    mi, mv = gm.merge(torch.from_numpy(ps).to(DEV), torch.from_numpy(py).to(DEV))
    _assert_same((mi.cpu().numpy()[None], mv.cpu().numpy()[None]), whole, "merge")


@pytest.mark.parametrize("reweight", [False, True])
@pytest.mark.parametrize("k", [256, 1024])
def test_merge_of_overlapping_sites(gm, k, reweight):
    """Sec. 2.3 with sites whose sets overlap (and, with `reweight`, give an
    element different weights): gm_merge of the sites' sketches equals the
    sketch of the union vector.  The 100000-entry vector and its sites take
    the big-vector path."""
    sizes = np.array([100_000, 3, 40, 700, 2500, 9000, 120, 33_000])
    idx, w, off = W.batch(nvec=len(sizes), seed=57, sizes=sizes)
    (si, sw, so), (ui, uw, uo) = W.sites(idx, w, off, nsites=3, seed=58, reweight=reweight)
    print(f"merge of overlapping sites k={k} reweight={reweight}", flush=True)
    ps, py = _gpu_sketch(gm, si, sw, so, k, 21)
    union = _gpu_sketch(gm, ui, uw, uo, k, 21)
    _assert_same(union, oracle.sketch(ui, uw, uo, k, 21, form=oracle.FORM_STREAM), "union")
    ps = torch.from_numpy(ps.reshape(len(sizes), 3, k)).to(DEV)
    py = torch.from_numpy(py.reshape(len(sizes), 3, k)).to(DEV)
    for v in range(len(sizes)):
        mi, mv = gm.merge(ps[v], py[v])
        torch.cuda.synchronize()
        _assert_same((mi.cpu().numpy(), mv.cpu().numpy()), (union[0][v], union[1][v]),
                     f"vector {v}")


def test_order_and_duplicates_do_not_change_result(gm):
    idx, w, off = W.batch(nvec=20, seed=61)
    base = _gpu_sketch(gm, idx, w, off, 128, 6)
    rng = np.random.default_rng(1)
    rows_i, rows_w = [], []
    for v in range(20):
        ii, ww = idx[off[v]:off[v + 1]], w[off[v]:off[v + 1]]
        dup = rng.integers(0, len(ii), size=len(ii) // 2)
        ii = np.concatenate([ii, ii[dup]])
        ww = np.concatenate([ww, ww[dup]])
        p = rng.permutation(len(ii))
        rows_i.append(ii[p])
        rows_w.append(ww[p])
    i2, w2, o2 = W._pack(rows_i, rows_w)
    _assert_same(_gpu_sketch(gm, i2, w2, o2, 128, 6), base, "shuffled+dups")
    _assert_same(_gpu_sketch(gm, idx, w, off, 128, 6), base, "repeat")


def test_long_vector_sampled(gm):
    idx, w, off = W.stream(nplus=1_000_000, seed=1003)
    for k in (1024, 4096):
        print(f"long vector n+=1e6 k={k}", flush=True)
        _assert_same(_gpu_sketch(gm, idx, w, off, k, 1),
                     oracle.sketch(idx, w, off, k, 1, form=oracle.FORM_STREAM), f"k={k}")


def _big_batch(seed=5):
    rng = np.random.default_rng(seed)
    rows_i, rows_w = [], []
    for n in (50_000, 10, 33_000, 120_000, 500, 70_000, 40_000):
        rows_i.append(W.distinct_sorted(rng, n, 1 << 24))
        if n == 70_000:
            ww = rng.lognormal(0.0, 2.0, size=n).astype(np.float32)
        else:
            ww = W.exp1_weights(rng, n)
        rows_w.append(ww)
    return W._pack(rows_i, rows_w)


@pytest.mark.parametrize("k", [64, 1024])
def test_big_vectors_candidate_lists(gm, k):
    """Vectors above 32768 entries go through the grid-wide sum and probe
    passes and are walked over their candidate lists."""
    idx, w, off = _big_batch()
    oracle.set_threads(8)
    print(f"big vectors k={k}", flush=True)
    _assert_same(_gpu_sketch(gm, idx, w, off, k, 21),
                 oracle.sketch(idx, w, off, k, 21, form=oracle.FORM_STREAM), f"k={k}")


@pytest.mark.parametrize("k", [1024, 4096])
def test_big_vector_skewed_candidates(gm, k):
    """Candidates packed into a few of the probe pass's work items overflow
    their sublists into the list itself (the heavy entries lead one vector,
    trail another; at k = 4096 the shorter vector keeps no list); the
    gathered lists must walk to the oracle's sketch."""
    rng = np.random.default_rng(31)
    rows_i, rows_w = [], []
    for n, lead in ((200_000, True), (60_000, False)):
        rows_i.append(W.distinct_sorted(rng, n, 1 << 24))
        ww = np.full(n, 1e-6, np.float32)
        heavy = (W.exp1_weights(rng, 6000) * 1000).astype(np.float32)
        if lead:
            ww[:6000] = heavy
        else:
            ww[-6000:] = heavy
        rows_w.append(ww)
    idx, w, off = W._pack(rows_i, rows_w)
    oracle.set_threads(8)
    print(f"big vectors, skewed weights, k={k}", flush=True)
    _assert_same(_gpu_sketch(gm, idx, w, off, k, 24),
                 oracle.sketch(idx, w, off, k, 24, form=oracle.FORM_STREAM), f"k={k}")


@pytest.mark.parametrize("opt,val", [("t0_scale_ppm", 1), ("t0_scale_ppm", 300_000),
                                     ("pos_bits", 56), ("map_load", 0)])
def test_big_vectors_forced_paths(gm, opt, val):
    """Empty or overflowing candidate lists fall back to the full vector;
    forced contests re-resolve; none of it may change the sketch."""
    idx, w, off = _big_batch(seed=6)
    try:
        gm.set_option(opt, val)
        print(f"big vectors forced {opt}={val}", flush=True)
        _assert_same(_gpu_sketch(gm, idx, w, off, 256, 22),
                     oracle.sketch(idx, w, off, 256, 22, form=oracle.FORM_STREAM), f"{opt}={val}")
    finally:
        gm.reset_options()


@pytest.mark.parametrize("t0_ppm", [1_000_000, 300_000])
def test_big_vectors_split_walks(gm, t0_ppm):
    """A call with few big vectors walks each candidate list in parts, one
    workgroup each, and merges the partial sketches; with the threshold cut
    to 0.3 T0 the merged sketch has empty registers and the vector is walked
    again unsplit.  Both must give the oracle's sketch."""
    idx, w, off = _big_batch(seed=7)
    nvec = len(off) - 1
    try:
        gm.set_option("t0_scale_ppm", t0_ppm)
        gm.set_option("stats", 1)
        gm.reset_stats()
        print(f"big vectors split t0_scale_ppm={t0_ppm}", flush=True)
        got = _gpu_sketch(gm, idx, w, off, 1024, 23)
        st = gm.get_stats()
    finally:
        gm.reset_options()
    _assert_same(got, oracle.sketch(idx, w, off, 1024, 23, form=oracle.FORM_STREAM),
                 f"t0_scale_ppm={t0_ppm}")
    # more walks than vectors: the five big vectors were split into parts
    assert st["vectors"] > nvec
    if t0_ppm < 1_000_000:
        assert st["passes"] > 0     # the unsplit walks had to widen the threshold


def test_graph_capture_replays_match_eager(gm):
    """A FastGM batched call (planner, big-vector passes, class kernels)
    captured into a HIP graph gives the eager result on every replay, with
    eager work and synchronisations between replays."""
    idx, w, off, kk = W.uneven(nvec=400, seed=79, size_cap=40_000)
    outoff = np.zeros(len(kk) + 1, np.int64)
    np.cumsum(kk, out=outoff[1:])
    t = lambda a: torch.from_numpy(a).to(DEV)
    ti, tw, to, tk, too = t(idx), t(w), t(off), t(kk), t(outoff)
    total = int(outoff[-1])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        gm.reserve(len(kk), stream=s)
        ei, ev = gm.sketch_batched(ti, tw, to, tk, too, int(kk.max()), 13, stream=s)
    s.synchronize()
    ei, ev = ei.cpu().numpy(), ev.cpu().numpy()
    gi = torch.empty(total, dtype=torch.int32, device=DEV)
    gv = torch.empty(total, dtype=torch.float64, device=DEV)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        gm.sketch_batched(ti, tw, to, tk, too, int(kk.max()), 13, out_idx=gi, out_val=gv,
                          stream=torch.cuda.current_stream())
    for rep in range(4):
        gi.fill_(-9)
        gv.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(gi.cpu().numpy(), ei), f"replay {rep}"
        assert np.array_equal(gv.cpu().numpy().view(np.uint64), ev.view(np.uint64)), f"replay {rep}"


def test_autotune_keeps_results_and_caches(gm, tmp_path, monkeypatch):
    """The autotuner only changes the schedule: the sketch after tuning equals
    the oracle's, and a second call is answered from the cache."""
    monkeypatch.setenv("GM_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    idx, w, off = W.mixed(seed=505, nvec=40, max_n=2000)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    try:
        r1 = gm.autotune(t(idx), t(w), t(off), 128, 3, reps=1)
        assert r1["from_cache"] == 0 and r1["ms"] > 0
        r2 = gm.autotune(t(idx), t(w), t(off), 128, 3, reps=1)
        assert r2["from_cache"] == 1
        assert (r2["small_waves"], r2["seg_rest"], r2["wave_lim"]) == \
            (r1["small_waves"], r1["seg_rest"], r1["wave_lim"])
        _assert_same(_gpu_sketch(gm, idx, w, off, 128, 3),
                     oracle.sketch(idx, w, off, 128, 3, form=oracle.FORM_STREAM), "tuned")
    finally:
        gm.reset_options()


def _edge_rows(k, seed):
    """Oracle-made sketch rows covering the estimators' special cases:
    0 A, 1 B (shares most of A's support, same weights), 2 empty, 3 zero
    weights only (empty too), 4 poisoned, 5 one element, 6 a set disjoint
    from A."""
    rng = np.random.default_rng(seed)
    a_i = W.distinct_sorted(rng, 300, 1 << 20)
    a_w = W.exp1_weights(rng, 300)
    b_i = np.concatenate([a_i[:200], W.distinct_sorted(rng, 50, 1 << 20) + (1 << 21)])
    b_w = np.concatenate([a_w[:200], W.exp1_weights(rng, 50)])
    rows_i = [a_i, b_i, np.zeros(0), np.array([3, 4]), np.array([5, 6]), np.array([77]),
              W.distinct_sorted(rng, 120, 1 << 20) + (1 << 22)]
    rows_w = [a_w, b_w, np.zeros(0), np.zeros(2), np.array([1.0, -1.0]), np.array([0.5]),
              W.exp1_weights(rng, 120)]
    idx, w, off = W._pack(rows_i, rows_w)
    return oracle.sketch(idx, w, off, k, seed, form=oracle.FORM_STREAM)


def _nan_same(got, want, what):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    assert np.array_equal(np.isnan(got), np.isnan(want)), what
    fin = ~np.isnan(want)
    assert np.array_equal(got[fin].view(np.uint64), want[fin].view(np.uint64)), what


@pytest.mark.parametrize("k", [64, 1000])
def test_estimators_on_empty_and_poisoned_sketches(gm, k):
    """gm_jaccard_est, gm_jaccard_est_pairs, gm_wcard_est, gm_merge and
    gm_setops on oracle-made rows that are empty, zero-weight, poisoned or a
    single element, against the oracle's estimators on the same rows."""
    s, y = _edge_rows(k, 40 + k)
    assert np.all(s[2] == -1) and np.all(s[3] == -1) and np.all(s[4] == -2)
    pairs = [(0, 1), (0, 2), (2, 2), (2, 3), (4, 0), (4, 4), (5, 5), (0, 0), (0, 6), (6, 2), (1, 0)]
    ia = np.array([p[0] for p in pairs], np.int64)
    ib = np.array([p[1] for p in pairs], np.int64)
    ts, ty = torch.from_numpy(s).to(DEV), torch.from_numpy(y).to(DEV)
    # Jaccard, row pairs and store lookups
    J = gm.jaccard_est(ts[torch.from_numpy(ia).to(DEV)].contiguous(),
                       ts[torch.from_numpy(ib).to(DEV)].contiguous()).cpu().numpy()
    Jp = gm.jaccard_est_pairs(ts, torch.from_numpy(ia).to(DEV),
                              torch.from_numpy(ib).to(DEV)).cpu().numpy()
    Jo = np.array([oracle.jaccard(s[a], s[b]) for a, b in pairs])
    _nan_same(J, Jo, "jaccard_est")
    _nan_same(Jp, Jo, "jaccard_est_pairs")
    assert Jo[2] == 0.0 and Jo[5] == 0.0 and Jo[7] == 1.0
    # weighted cardinality of every row
    C = gm.wcard_est(ty).cpu().numpy()
    _nan_same(C, np.array([oracle.wcard(y[r]) for r in range(len(y))]), "wcard_est")
    assert C[2] == 0.0 and np.isnan(C[4])
    # merges of groups of rows
    for grp in ([0, 2], [2, 3], [4, 0], [0, 1, 2], [5], [1, 6, 3]):
        g = torch.from_numpy(np.array(grp, np.int64)).to(DEV)
        mi, mv = gm.merge(ts[g].contiguous(), ty[g].contiguous())
        torch.cuda.synchronize()
        os_, oy = oracle.merge(s[grp], y[grp])
        assert np.array_equal(mi.cpu().numpy(), os_), f"merge {grp}"
        _nan_same(mv.cpu().numpy(), oy, f"merge {grp}")
    # two-set algebra of each pair
    g_a, g_b = torch.from_numpy(ia).to(DEV), torch.from_numpy(ib).to(DEV)
    R = gm.setops(ts[g_a].contiguous(), ty[g_a].contiguous(), ts[g_b].contiguous(),
                  ty[g_b].contiguous()).cpu().numpy()
    for p, (a, b) in enumerate(pairs):
        _nan_same(R[p], oracle.setops(s[a], y[a], s[b], y[b]), f"setops {a},{b}")


@pytest.mark.parametrize("k", [2, 256, 1000, 4096])
def test_setops_match_oracle(gm, k):
    """gm_setops on 150 oracle-made set pairs (a ragged number of 64-pair
    groups; k both a multiple of the 16-register tile and not)."""
    npairs = 150
    idx, w, off, _ = W.pairs(npairs=npairs, seed=900 + k, equal_shared_weights=True)
    oracle.set_threads(8)
    s, y = oracle.sketch(idx, w, off, k, 6, form=oracle.FORM_STREAM)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    R = gm.setops(t(s[0::2]), t(y[0::2]), t(s[1::2]), t(y[1::2])).cpu().numpy()
    want = np.stack([oracle.setops(s[2 * p], y[2 * p], s[2 * p + 1], y[2 * p + 1])
                     for p in range(npairs)])
    assert np.array_equal(R.view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("k", [1000, 4096])
def test_plain_large_k(gm, k):
    """Plain form at up to 16 register tiles: a mixed batch (every vector's
    registers against the oracle)."""
    idx, w, off = W.mixed(seed=310 + k, nvec=24, max_n=900)
    oracle.set_threads(8)
    print(f"plain mixed batch k={k}", flush=True)
    _assert_same(_gpu_sketch(gm, idx, w, off, k, 5, "plain"),
                 oracle.sketch(idx, w, off, k, 5, form=oracle.FORM_PLAIN), f"plain k={k}")


def _oracle_plain_split(idx, w, k, seed, parts=64):
    """The oracle's plain sketch of one long vector: its entries in `parts`
    ranges, sketched in parallel and merged (Sec. 2.3; the merge is pinned to
    the sketch of the union)."""
    n = len(idx)
    cut = np.linspace(0, n, parts + 1).astype(np.int64)
    s, y = oracle.sketch(idx, w, cut, k, seed, form=oracle.FORM_PLAIN)
    return oracle.merge(s, y)


@pytest.mark.parametrize("k", [256, 1024])
def test_plain_split_few_vectors(gm, k):
    """A call with few vectors splits their entries over many workgroups and
    merges the partial minima: one 200,000-entry vector, then a small batch
    of sizes around the split's 1024-entry minimum (every register against
    the oracle); two calls in a row reuse the merge counters."""
    oracle.set_threads(16)
    idx, w, off = W.stream(nplus=200_000, seed=1017)
    want = _oracle_plain_split(idx, w, k, 4)
    for rep in range(2):
        print(f"plain split: one 2e5-entry vector k={k} call {rep}", flush=True)
        gs, gy = _gpu_sketch(gm, idx, w, off, k, 4, "plain")
        _assert_same((gs[0], gy[0]), want, f"k={k} call {rep}")
    sizes = np.array([1, 1023, 1024, 1025, 5000, 30_000, 0, 70_000])
    bi, bw, bo = W.batch(nvec=len(sizes), seed=1018, sizes=sizes)
    print(f"plain split: 8 vectors k={k}", flush=True)
    _assert_same(_gpu_sketch(gm, bi, bw, bo, k, 4, "plain"),
                 oracle.sketch(bi, bw, bo, k, 4, form=oracle.FORM_PLAIN), f"batch k={k}")


@pytest.mark.parametrize("k", [256, 1024])
def test_plain_uneven_batch_split(gm, k):
    """A batch of many vectors (more (vector, tile) pairs than half the
    target workgroups) goes through the planning pass: the few vectors far
    above the mean work per workgroup are split and merged, the rest are
    not; every register against the oracle, over two calls (the merge
    counters are reused)."""
    rng = np.random.default_rng(1031 + k)
    sizes = rng.integers(50, 600, size=1100)
    sizes[[10, 500, 1000, 1099]] = [60_000, 120_000, 20_000, 9_000]
    bi, bw, bo = W.batch(nvec=len(sizes), seed=1032, sizes=sizes)
    oracle.set_threads(16)
    want = oracle.sketch(bi, bw, bo, k, 6, form=oracle.FORM_PLAIN)
    for rep in range(2):
        print(f"plain uneven batch k={k} call {rep}", flush=True)
        _assert_same(_gpu_sketch(gm, bi, bw, bo, k, 6, "plain"), want, f"k={k} call {rep}")


def test_plain_split_poison_and_batched(gm):
    """Split launches: an invalid entry in one range of a long vector poisons
    the whole vector (once in the error counter), and per-vector k in a
    batched call (k from 3 to 4096, so tiles past a vector's k are skipped)."""
    idx, w, off = W.stream(nplus=120_000, seed=1019)
    w = w.copy()
    w[77_777] = -1.0
    gm.reset_data_errors()
    gs, gy = _gpu_sketch(gm, idx, w, off, 512, 8, "plain")
    assert np.all(gs == -2) and np.all(np.isnan(gy))
    assert gm.get_data_errors() == 1
    gm.reset_data_errors()
    # the same counters again, clean input
    w[77_777] = 0.5
    oracle.set_threads(16)
    gs, gy = _gpu_sketch(gm, idx, w, off, 512, 8, "plain")
    _assert_same((gs[0], gy[0]), _oracle_plain_split(idx, w, 512, 8), "after poison")
    sizes = np.array([40_000, 3, 9_000, 2_500])
    kk = np.array([4096, 3, 1000, 64], np.int32)
    bi, bw, bo = W.batch(nvec=4, seed=1021, sizes=sizes)
    outoff = np.zeros(5, np.int64)
    np.cumsum(kk, out=outoff[1:])
    t = lambda a: torch.from_numpy(a).to(DEV)
    s, y = gm.sketch_batched(t(bi), t(bw), t(bo), t(kk), t(outoff), 4096, 12, form="plain")
    torch.cuda.synchronize()
    s, y = s.cpu().numpy(), y.cpu().numpy()
    for v in range(4):
        a, b = bo[v], bo[v + 1]
        ws, wy = _oracle_plain_split(bi[a:b], bw[a:b], int(kk[v]), 12, parts=16)
        _assert_same((s[outoff[v]:outoff[v + 1]], y[outoff[v]:outoff[v + 1]]), (ws, wy),
                     f"batched v={v}")
