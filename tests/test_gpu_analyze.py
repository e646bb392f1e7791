"""GPU parity: validation and level-set analysis, bit-exact against the oracle."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import host, matrices_small, to_gpu

pytestmark = pytest.mark.gpu

STAT_KEYS = ["num_levels", "thin_count", "S1", "S2", "cv", "cv_rows", "alc", "arl", "air",
             "thin_threshold"]


def check_analysis(orc, L, info):
    a = orc.analyze(L.n, L.rowptr, L.colidx)
    assert info.num_levels == a.num_levels
    assert np.array_equal(host(info.level), a.level)
    assert np.array_equal(host(info.perm), a.perm)
    assert np.array_equal(host(info.level_ptr), a.level_ptr)
    assert np.array_equal(host(info.rows), a.rows)
    assert np.array_equal(host(info.cost), a.cost)
    for k in STAT_KEYS:
        assert info.stats[k] == getattr(a, k), k        # bit for bit, floats included
    assert info.stats["max_level_rows"] == int(a.rows.max())


@pytest.mark.parametrize("name", list(matrices_small()))
def test_analyze_matches_oracle(orc, name):
    from paper_2609_40159_amd.api import analyze
    L = matrices_small()[name]
    check_analysis(orc, L, analyze(to_gpu(L)))


def test_analyze_device_stats_equal_host_stats(orc):
    from paper_2609_40159_amd import _lib
    from paper_2609_40159_amd.api import analyze
    L = synth.power_law(20000, 3)
    info = analyze(to_gpu(L))
    raw = bytes(host(info.device_stats))
    dev = _lib.LevelStats.from_buffer_copy(raw).as_dict()
    for k in STAT_KEYS:
        assert dev[k] == info.stats[k]


def test_analyze_repeatable(orc):
    from paper_2609_40159_amd.api import analyze
    L = synth.power_law(30000, 4)
    G = to_gpu(L)
    a1, a2 = analyze(G), analyze(G)
    assert torch.equal(a1.level, a2.level) and torch.equal(a1.perm, a2.perm)


def test_analyze_full_size_3d_128(orc):
    """The 128^3 7-point factor: levels equal the coordinate sums, stats exact."""
    from paper_2609_40159_amd.api import analyze
    L = synth.laplacian_3d(128, 128, 128)
    info = analyze(to_gpu(L))
    n = L.n
    idx = np.arange(n)
    csum = idx % 128 + (idx // 128) % 128 + idx // 16384
    assert np.array_equal(host(info.level), csum)
    assert info.num_levels == 382
    check_analysis(orc, L, info)
    assert round(info.stats["cv"], 6) == 0.803183


def test_analyze_full_size_powerlaw_1m(orc):
    from paper_2609_40159_amd.api import analyze
    L = synth.power_law(1_000_000, 3)
    check_analysis(orc, L, analyze(to_gpu(L)))


@pytest.mark.parametrize("case", ["upper", "unsorted", "dup", "missing", "empty_row", "zero",
                                  "lowest_row_wins", "bad_rowptr"])
def test_validate_matches_oracle(orc, case):
    from paper_2609_40159_amd.api import validate
    L = synth.laplacian_2d(6, 5)
    rp, ci, va = L.rowptr.copy(), L.colidx.copy(), L.vals.copy()
    if case == "upper":
        ci[rp[7]] = 20
    elif case == "unsorted":
        ci[rp[9]], ci[rp[9] + 1] = ci[rp[9] + 1], ci[rp[9]]
    elif case == "dup":
        ci[rp[12] + 1] = ci[rp[12]]
    elif case == "missing":
        ci[rp[4] - 1] = 2
    elif case == "empty_row":
        rp = np.concatenate([rp[:3], rp[3:] - 0])
        rp = rp.copy()
        # remove row 3's single diagonal by merging it into row 2's range end
        ci = np.delete(ci, rp[3]); va = np.delete(va, rp[3])
        rp[4:] -= 1
    elif case == "zero":
        va[rp[15] - 1] = 0.0
    elif case == "lowest_row_wins":
        ci[rp[20]] = 25            # upper entry in row 20
        va[rp[11] - 1] = 0.0       # zero diagonal in row 10
    elif case == "bad_rowptr":
        rp[5] = rp[6] + 1
    exp = orc.validate(L.n, rp, ci, va)
    from gpu_helpers import DEV
    from paper_2609_40159_amd.api import CSRMatrix
    G = CSRMatrix.from_arrays(rp, ci, va, device=DEV)
    st, bad = validate(G)
    assert st == orc.STATUS_NAMES[exp[0]]
    if exp[0] != orc.INVALID_ARG:
        assert bad == exp[1]
