"""Shared helpers for the GPU parity tests (HIP path vs the CPU oracle)."""
import numpy as np
import torch

import synth

DEV = "cuda"


def to_gpu(L: synth.CSR, dtype=torch.float64):
    from paper_2609_40159_amd.api import CSRMatrix
    return CSRMatrix.from_arrays(L.rowptr, L.colidx, L.vals, device=DEV, dtype=dtype)


def block(B: np.ndarray, dtype=torch.float64) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(B)).to(device=DEV, dtype=dtype).contiguous()


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def relerr(x: np.ndarray, ref: np.ndarray) -> float:
    """Normwise relative error, max over right-hand-side columns."""
    x = np.atleast_2d(x)
    ref = np.atleast_2d(ref)
    worst = 0.0
    for q in range(ref.shape[0]):
        den = np.max(np.abs(ref[q]))
        num = np.max(np.abs(x[q] - ref[q]))
        worst = max(worst, num / den if den > 0 else num)
    return worst


def matrices_small():
    """Seeded matrices spanning the structures the method meets."""
    out = {
        "lap2d_64": synth.laplacian_2d(64, 64),
        "lap2d_37x5": synth.laplacian_2d(37, 5),
        "lap3d_9x7x5": synth.laplacian_3d(9, 7, 5),
        "powerlaw_5k": synth.power_law(5000, 11),
        "random_300": synth.random_lower(300, 0.05, 12),
        "dense_60": synth.random_lower(60, 0.9, 13),
    }
    # a chain (one row per level), a diagonal matrix (one level), n = 1
    n = 700
    rp = np.concatenate([[0, 1], 1 + 2 * np.arange(1, n)]).astype(np.int32)
    ci = np.concatenate([[0]] + [[i - 1, i] for i in range(1, n)]).astype(np.int32)
    va = np.concatenate([[2.0]] + [[-0.5, 2.0] for _ in range(1, n)])
    out["chain_700"] = synth.CSR(n, rp, ci, va)
    n = 3000
    out["diag_3000"] = synth.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                                 np.linspace(1, 2, n))
    out["single"] = synth.CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32),
                              np.array([3.0]))
    # one hub row depending on many rows (long row), then a wide level
    n = 2500
    rows = [[i] for i in range(2000)]
    rows.append(list(range(0, 2000, 2)) + [2000])
    for i in range(2001, n):
        rows.append([2000, i])
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int32)
    ci = np.concatenate(rows).astype(np.int32)
    rng = np.random.default_rng(5)
    va = rng.uniform(-0.1, 0.1, ci.size)
    va[rp[1:] - 1] = rng.uniform(1, 2, n)
    out["hub_2500"] = synth.CSR(n, rp, ci, va)
    return out
