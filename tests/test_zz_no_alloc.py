"""The allocation-free plain entry point (gm_sketch_plain_noalloc) against
gm_sketch_plain, through the C ABI.

Two calls in a row share the device's static scratch: the first splits one
300k-entry vector at k = 1024 over the whole GPU, the second (smaller) splits
three vectors at k = 300, one of them empty and one poisoned.  Each call must
equal gm_sketch_plain bit for bit (indices and values), and the second also
equals the oracle's plain sketch (Eq. (1)-(2)).
"""
import ctypes

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"


@pytest.fixture(scope="module")
def lib():
    from paper_2302_05176_amd import _native, build
    if not build.up_to_date():
        build.build(force=True)
    assert torch.cuda.is_available()
    return _native.load()


def _vectors(seed, sizes, poison=None):
    rng = np.random.default_rng(seed)
    idx, w, off = [], [], [0]
    for v, n in enumerate(sizes):
        ii = rng.choice(1 << 24, size=n, replace=False).astype(np.int32)
        ww = (1.0 - rng.random(n)).astype(np.float32)
        if v == poison and n > 0:
            ww[n // 2] = -1.0
        idx.append(ii)
        w.append(ww)
        off.append(off[-1] + n)
    return (np.concatenate(idx).astype(np.int32), np.concatenate(w).astype(np.float32),
            np.array(off, dtype=np.int64))


def _call(lib, name, arrays, k, seed):
    idx, w, off = arrays
    nvec = len(off) - 1
    ti, tw, to = (torch.from_numpy(a).to(DEV) for a in (idx, w, off))
    oi = torch.full((nvec, k), 7, dtype=torch.int32, device=DEV)
    ov = torch.full((nvec, k), 7.0, dtype=torch.float64, device=DEV)
    stream = torch.cuda.current_stream()
    st = getattr(lib, name)(ctypes.c_void_p(ti.data_ptr()), ctypes.c_void_p(tw.data_ptr()),
                            ctypes.c_void_p(to.data_ptr()), nvec, k, ctypes.c_uint64(seed),
                            ctypes.c_void_p(oi.data_ptr()), ctypes.c_void_p(ov.data_ptr()),
                            ctypes.c_void_p(stream.cuda_stream))
    assert st == 0, f"{name} returned {st}"
    torch.cuda.synchronize()
    return oi.cpu().numpy(), ov.cpu().numpy()


def _same(got, want, what):
    assert np.array_equal(got[0], want[0]), f"{what}: register indices differ"
    assert np.array_equal(np.ascontiguousarray(got[1]).view(np.uint64),
                          np.ascontiguousarray(want[1]).view(np.uint64)), f"{what}: values differ"


def test_noalloc_matches_plain_two_calls(lib):
    big = _vectors(71, [300_000])
    small = _vectors(72, [20_000, 0, 5_000], poison=2)
    print("no-alloc call 1: one 300k-entry vector, k=1024", flush=True)
    first = _call(lib, "gm_sketch_plain_noalloc", big, 1024, 9)
    print("no-alloc call 2: three vectors (20k, 0, 5k poisoned), k=300", flush=True)
    second = _call(lib, "gm_sketch_plain_noalloc", small, 300, 11)
    print("reference calls: gm_sketch_plain", flush=True)
    _same(first, _call(lib, "gm_sketch_plain", big, 1024, 9), "call 1")
    _same(second, _call(lib, "gm_sketch_plain", small, 300, 11), "call 2")
    # the second call against the definition as well
    want = oracle.sketch(*small, 300, 11, form=oracle.FORM_PLAIN)
    _same(second, want, "call 2 vs oracle")
    assert (second[0][1] == -1).all() and (second[0][2] == -2).all()
