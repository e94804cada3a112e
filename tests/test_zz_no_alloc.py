"""rqlp_factor_noalloc (the library's static device scratch instead of a
caller workspace) against rqlp_factor with a caller workspace, through the C
ABI: two calls in a row on the shared scratch, the second on a smaller
problem, each compared with rqlp_factor on the same A and seed; and the
host-side rejection of a problem larger than the scratch."""
import ctypes

import numpy as np
import pytest

import paper_1811_09334_amd as rq
from paper_1811_09334_amd import _lib, inputs

SCRATCH_LIMIT = -1003


def _outputs(dev, m, n, l, dt):
    import torch
    return dict(Q=rq.empty_colmajor(m, l, dt, dev), T=rq.empty_colmajor(l, l, torch.float64, dev),
                P=rq.empty_colmajor(n, l, dt, dev), piv0=torch.empty(l, dtype=torch.int64, device=dev),
                piv1=torch.empty(l, dtype=torch.int64, device=dev), lv=torch.empty(l, dtype=torch.float64, device=dev),
                info=torch.full((1,), -1, dtype=torch.int32, device=dev))


def _call(A, k, p, q, d, b, prec, seed, noalloc):
    import torch
    m, n = A.shape
    l = k + p
    dev = A.device
    o = _outputs(dev, m, n, l, A.dtype)
    uplo = ctypes.c_char(b"?")
    stream = torch.cuda.current_stream(dev).cuda_stream
    head = (A.data_ptr(), rq.ld(A), m, n, k, p, q, d, b, prec, seed, None, max(n, 1),
            o["Q"].data_ptr(), rq.ld(o["Q"]), o["T"].data_ptr(), rq.ld(o["T"]), o["P"].data_ptr(), rq.ld(o["P"]),
            o["piv0"].data_ptr(), o["piv1"].data_ptr(), o["lv"].data_ptr(), o["info"].data_ptr(), ctypes.byref(uplo))
    if noalloc:
        st = _lib.rqlp_factor_noalloc(*head, stream)
    else:
        nbytes = _lib.rqlp_workspace_size(m, n, k, p, q, d, b, prec)
        work = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        work.fill_(0xA5)                       # contents on entry are ignored
        st = _lib.rqlp_factor(*head, work.data_ptr(), nbytes, stream)
    assert st == 0, _lib.rqlp_status_string(st)
    torch.cuda.synchronize()
    out = {kk: v.cpu().numpy() for kk, v in o.items()}
    out["uplo"] = uplo.value
    return out


def _compare(a, b, tol):
    assert a["uplo"] == b["uplo"]
    assert int(a["info"][0]) == int(b["info"][0])
    np.testing.assert_array_equal(a["piv0"], b["piv0"])
    np.testing.assert_array_equal(a["piv1"], b["piv1"])
    for key in ("Q", "T", "P", "lv"):
        x, y = a[key].astype(np.float64), b[key].astype(np.float64)
        scale = max(np.abs(y).max(), 1e-300)
        assert np.abs(x - y).max() <= tol * scale, key


# (m, n, k, p, q, d, b, precision): the first larger than the second
CASES = [
    ((1000, 500, 20, 5, 1, 2, 0, "f64"), (600, 300, 12, 5, 0, 0, 0, "f64"), 1e-10),
    ((1536, 768, 40, 8, 1, 0, 0, "bf16"), (700, 350, 16, 6, 1, 1, 0, "bf16"), 1e-6),
]


@pytest.mark.gpu
@pytest.mark.parametrize("big,small,tol", CASES)
def test_noalloc_matches_workspace_entry_point(gpu, big, small, tol):
    import torch
    dev = torch.device("cuda:0")
    for (m, n, k, p, q, d, b, precision) in (big, small):
        prec = rq.PRECISIONS[precision]
        w = inputs.WORKLOADS["rqlp_f64_1000x500"].scaled(m, n, name=f"noalloc_{m}x{n}")
        A = inputs.make_matrix_torch(w, dev).to(torch.float64 if precision == "f64" else torch.float32)
        A = rq.colmajor(A)
        print(f"[noalloc] {precision} {m}x{n} k={k} p={p} q={q} d={d}", flush=True)
        ref = _call(A, k, p, q, d, b, prec, 2024, noalloc=False)
        got = _call(A, k, p, q, d, b, prec, 2024, noalloc=True)
        assert int(got["info"][0]) == 0
        _compare(got, ref, tol)


def test_noalloc_rejects_problem_beyond_scratch():
    rq.load()
    # 65536 x 8192 in FP64 needs far more than the static scratch; no device work
    st = _lib.rqlp_factor_noalloc(1, 65536, 65536, 8192, 100, 10, 0, 0, 0, 0, 0, None, 8192, 1, 65536, 1, 110, 1,
                                  8192, None, None, None, None, None, None)
    assert st == SCRATCH_LIMIT
    assert "static scratch" in _lib.rqlp_status_string(st)
    # argument errors keep rqlp_factor's numbering
    assert _lib.rqlp_factor_noalloc(1, 99, 100, 50, 5, 3, 0, 0, 0, 0, 0, None, 50, 1, 100, 1, 8, 1, 50,
                                    None, None, None, None, None, None) == -2
    assert _lib.rqlp_factor_noalloc(None, 100, 100, 50, 5, 3, 0, 0, 0, 0, 0, None, 50, 1, 100, 1, 8, 1, 50,
                                    None, None, None, None, None, None) == -1
