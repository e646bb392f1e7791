"""Host checks of the tall-block row order: it is a permutation, the
permuted factor stays lower triangular (so the order is topological), the
3D grid gets whole z-columns grouped into 4 x 8 tiles, and malformed
patterns are refused.  No GPU."""
import numpy as np
import pytest
import scipy.sparse

import synth


def permuted_pattern(L, perm):
    A = scipy.sparse.csr_matrix((np.ones(L.nnz), L.colidx, L.rowptr), shape=(L.n, L.n))
    return A[perm][:, perm].tocoo()


@pytest.mark.parametrize("make", [lambda: synth.laplacian_3d(12, 10, 9),
                                  lambda: synth.laplacian_2d(40, 30),
                                  lambda: synth.power_law(5000, 8),
                                  lambda: synth.random_lower(600, 0.03, 2)])
def test_order_is_a_topological_permutation(make):
    from paper_2609_40159_amd.api import tall_block_order
    L = make()
    perm = tall_block_order(L.rowptr, L.colidx)
    assert np.array_equal(np.sort(perm), np.arange(L.n))
    P = permuted_pattern(L, perm)
    assert np.all(P.col <= P.row)                   # P L P^T lower triangular
    assert P.nnz == L.nnz


def test_grid_tiles_hold_whole_z_columns():
    """16 x 16 x 8 grid, tile 4 x 8: chains are the z-columns (x, y), chains
    of chains the y-lines of the bottom plane, and each run of 4 * 8 * 8
    rows of the order is one tile of x in a block of 8, y in a block of 4."""
    from paper_2609_40159_amd.api import tall_block_order
    nx, ny, nz = 16, 16, 8
    L = synth.laplacian_3d(nx, ny, nz)
    perm = tall_block_order(L.rowptr, L.colidx, 4, 8)
    x, y, z = perm % nx, (perm // nx) % ny, perm // (nx * ny)
    per_tile = 4 * 8 * nz
    for t in range(L.n // per_tile):
        s = slice(t * per_tile, (t + 1) * per_tile)
        assert len(set(x[s] // 8)) == 1 and len(set(y[s] // 4)) == 1, t
        assert len(set(zip(x[s], y[s]))) == 32                  # whole columns
        for c in set(zip(x[s], y[s])):                          # each column in z order
            zz = z[s][(x[s] == c[0]) & (y[s] == c[1])]
            assert np.array_equal(zz, np.arange(nz))


def test_malformed_patterns_are_refused():
    from paper_2609_40159_amd.api import tall_block_order
    from paper_2609_40159_amd._lib import RwtError
    with pytest.raises(RwtError):                                  # diagonal not last
        tall_block_order(np.array([0, 1, 3]), np.array([0, 1, 0]))
    with pytest.raises(RwtError):                                  # entry above the diagonal
        tall_block_order(np.array([0, 2, 3]), np.array([1, 0, 1]))
    with pytest.raises(RwtError):                                  # negative tile shape
        tall_block_order(np.array([0, 1]), np.array([0]), -1, 0)
    assert tall_block_order(np.array([0]), np.array([], dtype=np.int32)).size == 0
    # arrays that disagree in length are refused before the library reads them
    with pytest.raises(ValueError):                                # colidx shorter than rowptr[n]
        tall_block_order(np.array([0, 1, 3]), np.array([0, 0]))
    with pytest.raises(ValueError):                                # rowptr decreasing
        tall_block_order(np.array([0, 2, 1]), np.array([0, 0, 1]))
    with pytest.raises(ValueError):                                # rowptr not starting at 0
        tall_block_order(np.array([1, 2]), np.array([0, 0]))


def test_order_of_L_stays_topological_for_the_rewritten_factor():
    """Equation rewriting only adds dependencies from the transitive closure
    of L's DAG, so the order computed on L is a topological order of
    L' = M L as well (the oracle rewrites 1% of the rows, thin-first whole
    levels, target = level - 1)."""
    import oracle
    from paper_2609_40159_amd.api import tall_block_order
    L = synth.laplacian_3d(14, 12, 10)
    an = oracle.analyze(L.n, L.rowptr, L.colidx)
    rows, targets = synth.thin_first_rows(an.level, 0.05)
    rw = oracle.rewrite(L.n, L.rowptr, L.colidx, L.vals, an.level, rows, targets)
    Lp = synth.CSR(L.n, rw.rowptr, rw.colidx, rw.vals)
    assert Lp.nnz > L.nnz                                   # rows were rewritten
    perm = tall_block_order(L.rowptr, L.colidx)
    P = permuted_pattern(Lp, perm)
    assert np.all(P.col <= P.row)
