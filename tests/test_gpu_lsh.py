"""LSH index (gm_lsh_build / gm_lsh_query) against the oracle's banding
definition, exactly: the same candidate rows in ascending order and the same
counts.  The stored and query sketches are made by the C oracle."""
import numpy as np
import pytest

import oracle
from oracle import lsh as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_05176_amd as gm
    gm.reset_options()
    oracle.build()
    return gm


def _bases(rng, nbase, n=24, dim=1 << 16):
    return [(rng.choice(dim, n, replace=False), rng.exponential(size=n)) for _ in range(nbase)]


def _clustered(rng, bases, nvec, n=24, keep=18, dim=1 << 16):
    """CSR vectors, each a perturbed copy of one of the base vectors: keeps
    `keep` of its n entries (same weights) and draws the rest afresh."""
    nbase = len(bases)
    rows_i, rows_w = [], []
    for _ in range(nvec):
        bi, bw = bases[rng.integers(nbase)]
        sel = rng.choice(n, keep, replace=False)
        fresh = rng.choice(dim, n - keep, replace=False) + dim
        ii = np.concatenate([bi[sel], fresh])
        ww = np.concatenate([bw[sel], rng.exponential(size=n - keep)])
        o = np.argsort(ii)
        rows_i.append(ii[o])
        rows_w.append(ww[o])
    idx = np.concatenate(rows_i).astype(np.int32)
    w = (np.concatenate(rows_w) + 1e-3).astype(np.float32)
    off = np.arange(nvec + 1, dtype=np.int64) * n
    return idx, w, off


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _compare(gm, store, queries, bands, rows, max_cand):
    import torch
    ix = gm.LshIndex(_dev(store), bands, rows)
    cand, count = ix.query(_dev(queries), max_cand)
    torch.cuda.synchronize()
    cand, count = cand.cpu().numpy(), count.cpu().numpy()
    tables = L.build(store, bands, rows)
    want = L.candidates(store, queries, bands, rows, tables)
    for q, c in enumerate(want):
        assert count[q] == len(c), q
        m = min(len(c), max_cand)
        assert np.array_equal(cand[q, :m], c[:m]), q
    ix.close()
    return want


@pytest.mark.parametrize("k,bands,rows", [(64, 16, 4), (128, 32, 3), (256, 64, 4)])
def test_candidates_match_oracle(gm, k, bands, rows):
    rng = np.random.default_rng(700 + k)
    bases = _bases(rng, 120)
    idx, w, off = _clustered(rng, bases, nvec=3000)
    store, _ = oracle.sketch(idx, w, off, k, 5, form=oracle.FORM_STREAM)
    qi, qw, qo = _clustered(rng, bases, nvec=150)
    queries, _ = oracle.sketch(qi, qw, qo, k, 5, form=oracle.FORM_STREAM)
    # exact copies of stored rows, an empty and a poisoned sketch
    extra = np.stack([store[3], store[2999], np.full(k, -1, np.int32), np.full(k, -2, np.int32)])
    queries = np.concatenate([queries, extra]).astype(np.int32)
    print(f"lsh k={k} bands={bands} rows={rows}", flush=True)
    want = _compare(gm, store, queries, bands, rows, max_cand=64)
    assert sum(len(c) > 0 for c in want) > 100   # the clusters do collide
    assert 3 in want[150] and 2999 in want[151]
    assert len(want[152]) == 0 and len(want[153]) == 0
    # a short candidate list keeps the smallest rows
    _compare(gm, store, queries, bands, rows, max_cand=3)


def test_duplicates_overflow_and_empty_rows(gm):
    import torch
    k, bands, rows = 64, 16, 4
    rng = np.random.default_rng(710)
    idx, w, off = _clustered(rng, _bases(rng, 50), nvec=400)
    base, _ = oracle.sketch(idx, w, off, k, 9, form=oracle.FORM_STREAM)
    # 100 copies of row 7 (1600 band matches: within the 2048 held per query)
    store = np.concatenate([base, np.repeat(base[7:8], 100, axis=0),
                            np.full((3, k), -1, np.int32), np.full((2, k), -2, np.int32)])
    print("lsh duplicates", flush=True)
    want = _compare(gm, store, base[7:8], bands, rows, max_cand=128)
    assert len(want[0]) >= 101
    # 160 copies: 2560 band matches, more than the query holds -> count -1
    store2 = np.concatenate([base, np.repeat(base[7:8], 160, axis=0)])
    assert L.band_matches(store2, base[7], bands, rows) > 2048
    ix = gm.LshIndex(_dev(store2), bands, rows)
    cand, count = ix.query(_dev(base[7:9]), 16)
    torch.cuda.synchronize()
    assert int(count[0]) == -1
    want2 = L.candidates(store2, base[8:9], bands, rows)[0]
    assert int(count[1]) == len(want2)
    ix.close()
