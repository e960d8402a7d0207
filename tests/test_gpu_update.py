"""Streaming update (gm_sketch_update) against the oracle.

A sketch updated chunk by chunk must equal, bit for bit, the sketch of all
the entries at once (Sec. 2.3: a register is the lexicographic minimum over
the entries; Sec. 3: a stream visits each element as it comes, and repeated
elements change nothing)."""
import numpy as np
import pytest

import oracle
from paper_2302_05176_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_05176_amd as gm
    gm.reset_options()
    return gm


def _dev(*arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrays]


def _split(idx, w, off, parts, seed):
    """Assign every entry of every vector to one of `parts` chunks; return a
    CSR (idx, w, off) per chunk over the same vectors."""
    rng = np.random.default_rng(seed)
    nvec = len(off) - 1
    which = rng.integers(0, parts, size=len(idx))
    out = []
    for p in range(parts):
        ri, rw, lens = [], [], []
        for v in range(nvec):
            a, b = off[v], off[v + 1]
            m = which[a:b] == p
            ri.append(idx[a:b][m])
            rw.append(w[a:b][m])
            lens.append(int(m.sum()))
        o = np.zeros(nvec + 1, np.int64)
        o[1:] = np.cumsum(lens)
        out.append((np.concatenate(ri).astype(np.int32), np.concatenate(rw).astype(np.float32), o))
    return out


def _check(gm, chunks, k, seed, want, label):
    nvec = len(chunks[0][2]) - 1
    si, sv = gm.empty_sketches(nvec, k)
    for ci, cw, co in chunks:
        ti, tw, to = _dev(ci, cw, co)
        gm.sketch_update(ti, tw, to, k, seed, si, sv)
    got_i, got_v = si.cpu().numpy(), sv.cpu().numpy()
    assert np.array_equal(got_i, want[0]), label
    assert np.array_equal(got_v.view(np.uint64), want[1].view(np.uint64)), label
    return si, sv


@pytest.mark.parametrize("k", [1, 16, 256, 1000, 4096])
def test_chunked_updates_equal_whole_sketch(gm, k):
    max_n = 2500 if k <= 256 else 700
    idx, w, off = W.mixed(seed=600 + k, nvec=40, max_n=max_n)
    want = oracle.sketch(idx, w, off, k, 3, form=oracle.FORM_STREAM)
    print(f"chunked update k={k}", flush=True)
    _check(gm, _split(idx, w, off, 3, seed=k), k, 3, want, f"k={k}")


def test_document_batch_updates(gm):
    idx, w, off = W.batch(nvec=300, seed=1203)
    want = oracle.sketch(idx, w, off, 256, 5, form=oracle.FORM_STREAM)
    print("document batch, 4 chunks, k=256", flush=True)
    _check(gm, _split(idx, w, off, 4, seed=1), 256, 5, want, "document batch")


def test_repeats_empty_updates_and_poison(gm):
    import torch
    idx, w, off = W.batch(nvec=60, seed=1204)
    k, seed = 128, 11
    want = oracle.sketch(idx, w, off, k, seed, form=oracle.FORM_STREAM)
    chunks = _split(idx, w, off, 2, seed=2)
    si, sv = _check(gm, chunks, k, seed, want, "two chunks")
    print("repeat a chunk and apply an empty update", flush=True)
    ti, tw, to = _dev(*chunks[0])
    gm.sketch_update(ti, tw, to, k, seed, si, sv)        # repeats change nothing
    # (a one-entry buffer: null arrays are an argument error when nvec > 0)
    e_i, e_w, e_o = _dev(np.zeros(1, np.int32), np.ones(1, np.float32),
                         np.zeros(len(off), np.int64))
    gm.sketch_update(e_i, e_w, e_o, k, seed, si, sv)     # nothing new
    assert np.array_equal(si.cpu().numpy(), want[0])
    assert np.array_equal(sv.cpu().numpy().view(np.uint64), want[1].view(np.uint64))
    print("poisoned update", flush=True)
    bi = np.array([5, 6], np.int32)
    bw = np.array([1.0, np.nan], np.float32)
    bo = np.zeros(len(off), np.int64)
    bo[4:] = 2                                            # vector 3 gets the bad entries
    gm.reset_data_errors()
    ti, tw, to = _dev(bi, bw, bo)
    gm.sketch_update(ti, tw, to, k, seed, si, sv)
    assert gm.get_data_errors() == 1
    gi, gv = si.cpu().numpy(), sv.cpu().numpy()
    assert (gi[3] == -2).all() and np.isnan(gv[3]).all()
    keep = np.arange(len(off) - 1) != 3
    assert np.array_equal(gi[keep], want[0][keep])
    ti, tw, to = _dev(*chunks[1])
    gm.sketch_update(ti, tw, to, k, seed, si, sv)        # a poisoned row stays poisoned
    assert (si.cpu().numpy()[3] == -2).all()
    gm.reset_data_errors()
    torch.cuda.synchronize()


@pytest.mark.parametrize("t0_ppm", [1_000_000, 300_000])
def test_big_vector_updates(gm, t0_ppm):
    """A big vector's chunks are walked in parts merged with the stored
    sketch; at 0.3 T0 some registers stay unsettled and the update is walked
    again unsplit."""
    idx, w, off = W.stream(nplus=120_000, seed=1205)
    k, seed = 1024, 2
    want = oracle.sketch(idx, w, off, k, seed, form=oracle.FORM_STREAM)
    print(f"one 120k-entry vector in 2 chunks of ~60k (big-vector path), t0_scale_ppm={t0_ppm}",
          flush=True)
    try:
        gm.set_option("t0_scale_ppm", t0_ppm)
        _check(gm, _split(idx, w, off, 2, seed=3), k, seed, want, "big vector")
        _check(gm, _split(idx, w, off, 3, seed=4), k, seed, want, "big vector, 3 chunks")
    finally:
        gm.reset_options()
