"""The 256-matrix batch the benchmark's headline is measured on, generated
on the CPU from its seeds: its size and the algorithmic bytes of one step
(the numerator of the headline's GB/s) are reproduced independently of the
GPU path: solves 4(n+1) + nnz(4 + 8) + 2nk·8 per matrix, candidate levels
4(n+1) + 4(nnz - n) + 4n per candidate."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import synth  # noqa: E402


def test_headline_batch_size_and_step_bytes():
    man = synth.batch_manifest(count=256)
    gen = synth.build_batch(man, min(8, os.cpu_count() or 1))
    n_tot = nnz_tot = k_tot = cands = 0
    b_solve = b_cand = 0
    for spec, (Lh, _, Bh) in zip(man, gen):
        n, nnz, k = Lh.n, int(Lh.rowptr[-1]), spec["k"]
        assert Bh.size == n * k   # the right-hand sides the solves read
        n_tot += n
        nnz_tot += nnz
        k_tot += k
        cands += len(spec["phis"])
        b_solve += 4 * (n + 1) + nnz * (4 + 8) + 2 * n * k * 8
        b_cand += len(spec["phis"]) * (4 * (n + 1) + 4 * (nnz - n) + 4 * n)
    assert (n_tot, nnz_tot, k_tot, cands) == (26_986_089, 166_220_472, 2_178, 8_192)
    assert b_solve == 5_799_196_356
    assert b_cand == 24_730_472_576
    assert b_solve + b_cand == 30_529_668_932
