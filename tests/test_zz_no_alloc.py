"""rwt_apply_M_noalloc (no workspace, library-owned device scratch) against
rwt_apply_M (caller workspace): both through the C ABI, bit for bit, on two
calls in a row with the second on a smaller system (the scratch keeps the
first call's row offsets, which must not leak into the second)."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from gpu_helpers import DEV, block, host, to_gpu

pytestmark = pytest.mark.gpu


def _rewritten(Lh, frac, k, seed):
    from paper_2609_40159_amd.api import analyze, rewrite
    G = to_gpu(Lh)
    info = analyze(G)
    rows, targets = synth.thin_first_rows(host(info.level), frac)
    B = np.random.default_rng(seed).standard_normal((k, Lh.n))
    rw = rewrite(G, info.level, torch.as_tensor(rows, device=DEV),
                 torch.as_tensor(targets, device=DEV), block(B))
    return rw, block(B)


def _call_both(rw, B):
    from paper_2609_40159_amd import _lib
    lib = _lib.load()
    n, k = rw.L.n, B.shape[0]
    nc = rw.crow.numel()
    stream = torch.cuda.current_stream().cuda_stream
    sz = C.c_size_t(0)
    _lib.check(lib.rwt_apply_M_ws(n, C.byref(sz)))
    ws = torch.empty(max(sz.value, 256), dtype=torch.uint8, device=DEV)
    ref = torch.empty_like(B)
    _lib.check(lib.rwt_apply_M(n, nc, rw.crow.data_ptr(), rw.ccol.data_ptr(), rw.cval.data_ptr(),
                               _lib.F64, B.data_ptr(), k, n, ref.data_ptr(), n, ws.data_ptr(),
                               ws.numel(), stream))
    out = torch.full_like(B, float("nan"))
    _lib.check(lib.rwt_apply_M_noalloc(n, nc, rw.crow.data_ptr(), rw.ccol.data_ptr(),
                                       rw.cval.data_ptr(), _lib.F64, B.data_ptr(), k, n,
                                       out.data_ptr(), n, stream))
    torch.cuda.synchronize()
    return ref, out


def test_noalloc_matches_workspace_entry_point_twice():
    # first a larger system, then a smaller one: the second call must not
    # read row offsets the first left in the scratch array
    big, Bb = _rewritten(synth.laplacian_3d(40, 36, 30), 0.01, 3, 1)
    print("no-alloc apply_M: lap3d 40x36x30, k=3", flush=True)
    ref1, out1 = _call_both(big, Bb)
    assert torch.equal(ref1, out1)
    assert torch.equal(out1, big.B.reshape(out1.shape))   # M B is the rewrite's B'
    small, Bs = _rewritten(synth.power_law(5000, 11), 0.008, 2, 2)
    print("no-alloc apply_M: power-law 5000, k=2", flush=True)
    ref2, out2 = _call_both(small, Bs)
    assert torch.equal(ref2, out2)
    assert torch.equal(out2, small.B.reshape(out2.shape))


def test_noalloc_rejects_too_many_rows():
    """Host-side check: refused before any device work (fake pointers)."""
    from paper_2609_40159_amd import _lib
    lib = _lib.load()
    n = _lib.APPLY_M_NOALLOC_MAX_N + 1
    st = lib.rwt_apply_M_noalloc(n, 0, None, None, None, _lib.F64, C.c_void_p(256), 1, n,
                                 C.c_void_p(512), n, None)
    assert _lib.STATUS[st] == "TOO_LARGE"
    assert b"at most" in lib.rwt_last_error_string()
