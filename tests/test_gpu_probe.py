"""The hand-off measurement used for the solves' latency floor: a plausible
one-way time, and its argument checks."""
import ctypes as C

import pytest

pytestmark = pytest.mark.gpu


def test_handoff_probe():
    from paper_2609_40159_amd import _lib, api
    ns = api.probe_handoff(500)
    assert 20.0 < ns < 50_000.0, ns
    lib = _lib.load()
    out = C.c_double(0.0)
    assert lib.rwt_probe_handoff(0, None, 0, C.byref(out), None) == -1
    assert lib.rwt_probe_handoff(10, None, 0, C.byref(out), None) == -7   # workspace too small
    assert lib.rwt_probe_handoff_ws(10) >= 160
