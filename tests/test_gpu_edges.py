"""Degenerate inputs through the C ABI: the empty matrix (n = 0) in every
call that accepts it, against the oracle's analysis of the same empty
input, and an environment on it refused with an argument error."""
import numpy as np
import pytest
import torch

from gpu_helpers import DEV

pytestmark = pytest.mark.gpu


def empty_matrix():
    from paper_2609_40159_amd.api import CSRMatrix
    return CSRMatrix.from_arrays(np.array([0], np.int32), np.zeros(0, np.int32),
                                 np.zeros(0, np.float64), device=DEV)


def test_empty_matrix(orc):
    from paper_2609_40159_amd.api import (Env, Plan, RwtError, UpperPlan, analyze, grad_vals,
                                          solve, solve_pair, validate)
    print("edge: empty matrix", flush=True)
    L = empty_matrix()
    assert validate(L) == ("OK", -1)
    info = analyze(L)
    ref = orc.analyze(0, np.array([0], np.int32), np.zeros(0, np.int32))
    assert info.num_levels == ref.num_levels == 0
    assert info.stats["cv"] == ref.cv == 0.0 and info.stats["S1"] == 0
    assert info.level.numel() == 0 and info.level_ptr.tolist() == [0]
    p = Plan(L, kmax=2)
    B = torch.empty((2, 0), dtype=torch.float64, device=DEV)
    assert p.solve(B).shape == (2, 0)
    assert p.solve_transpose(B).shape == (2, 0)
    p.check()
    assert solve(L, torch.empty(0, dtype=torch.float64, device=DEV)).shape == (0,)
    U = UpperPlan(L, kmax=2)
    assert U.solve(B).shape == (2, 0)
    assert solve_pair(p, U, B).shape == (2, 0)
    U.check()
    assert grad_vals(L, B, B).numel() == 0
    with pytest.raises(RwtError) as e:
        Env(L, info, 4, cap=8)
    assert e.value.name == "INVALID_ARG"
    torch.cuda.synchronize()
