// Tall-block row order (host code).
//
// The sync-free solve walks blocks of consecutive rows; a dependency chain
// that leaves its block at every level pays one hand-off per level.  This
// order keeps long chains inside blocks: it is a topological order of the
// dependency DAG in which consecutive rows form tiles of whole chains.
//
//   1. level of each row (longest dependency path, Section 2.1);
//   2. parent of a row: its dependency one level below with the smallest
//      index; successor of a row: the child farthest from it in index.
//      Following successors cuts the DAG into chains (on a 3D grid in
//      natural order: the columns along the slowest axis);
//   3. the same on the DAG of the chain heads (a head's parent chain is the
//      chain holding the head's parent): chains of chains;
//   4. key of a row = (tile: position of its head along its chain of chains
//      / a and number of that chain of chains / b; then its chain), made
//      non-decreasing along every dependency in one pass in row order;
//   5. rows sorted by (key, level, row): every dependency of a row has a
//      key no larger and, when equal, a lower level, so the order is
//      topological and P L P^T is lower triangular.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "common.hpp"

extern "C" rwt_status rwt_tall_block_order(int32_t n, const int32_t* rowptr,
                                           const int32_t* colidx, int32_t a, int32_t b,
                                           int32_t* perm) {
    RWT_REQUIRE(n >= 0, RWT_ERR_INVALID_ARG, "negative n");
    RWT_REQUIRE(a >= 0 && b >= 0, RWT_ERR_INVALID_ARG, "negative tile shape");
    if (n == 0) return RWT_OK;
    RWT_REQUIRE(rowptr && colidx && perm, RWT_ERR_INVALID_ARG, "null argument");
    if (a == 0) a = 4;
    if (b == 0) b = 8;
    RWT_REQUIRE(rowptr[0] == 0, RWT_ERR_INVALID_ARG, "rowptr[0] must be 0");
    std::vector<int32_t> lev(n, 0), parent(n, -1);
    for (int32_t i = 0; i < n; ++i) {
        const int32_t rb = rowptr[i], re = rowptr[i + 1];
        RWT_REQUIRE(re > rb, RWT_ERR_MISSING_DIAG, "row %d has no entries", i);
        RWT_REQUIRE(colidx[re - 1] == i, RWT_ERR_MISSING_DIAG, "row %d: last entry not diagonal", i);
        int32_t l = 0;
        for (int32_t p = rb; p < re - 1; ++p) {
            const int32_t j = colidx[p];
            RWT_REQUIRE(j >= 0 && j < i, RWT_ERR_NOT_LOWER, "row %d: column %d", i, j);
            l = std::max(l, lev[j] + 1);
        }
        lev[i] = l;
        for (int32_t p = rb; p < re - 1; ++p) {
            const int32_t j = colidx[p];
            if (lev[j] == l - 1 && (parent[i] < 0 || j < parent[i])) parent[i] = j;
        }
    }
    // chains: a row continues its parent's chain when it is the parent's
    // farthest child (rows in order, so a head precedes its chain)
    std::vector<int32_t> succ(n, -1);
    for (int32_t i = 0; i < n; ++i) {
        const int32_t p = parent[i];
        if (p >= 0 && (succ[p] < 0 || i - p > succ[p] - p)) succ[p] = i;
    }
    std::vector<int32_t> cid(n), head;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t p = parent[i];
        if (p >= 0 && succ[p] == i) {
            cid[i] = cid[p];
        } else {
            cid[i] = (int32_t)head.size();
            head.push_back(i);
        }
    }
    // chains of chains over the heads' DAG (chain numbers follow head order,
    // so a parent chain has a smaller number)
    const int32_t nc = (int32_t)head.size();
    std::vector<int32_t> hpar(nc, -1), hsucc(nc, -1), hc(nc), hpos(nc, 0);
    for (int32_t c = 0; c < nc; ++c) {
        const int32_t p = parent[head[c]];
        hpar[c] = p >= 0 ? cid[p] : -1;
    }
    for (int32_t c = 0; c < nc; ++c) {
        const int32_t p = hpar[c];
        if (p >= 0 && (hsucc[p] < 0 || head[c] - head[p] > head[hsucc[p]] - head[p])) hsucc[p] = c;
    }
    int32_t nhc = 0;
    for (int32_t c = 0; c < nc; ++c) {
        const int32_t p = hpar[c];
        if (p >= 0 && hsucc[p] == c) {
            hc[c] = hc[p];
            hpos[c] = hpos[p] + 1;
        } else {
            hc[c] = nhc++;
        }
    }
    // keys (tile, chain), compared in that order, made non-decreasing along
    // dependencies
    const int64_t span_b = (int64_t)nhc / b + 1;
    std::vector<int64_t> ktile(n);
    std::vector<int32_t> kchain(n);
    for (int32_t i = 0; i < n; ++i) {
        const int32_t c = cid[i];
        int64_t t = (int64_t)(hpos[c] / a) * span_b + hc[c] / b;
        int32_t ch = c;
        for (int32_t p = rowptr[i]; p < rowptr[i + 1] - 1; ++p) {
            const int32_t j = colidx[p];
            if (ktile[j] > t || (ktile[j] == t && kchain[j] > ch)) {
                t = ktile[j];
                ch = kchain[j];
            }
        }
        ktile[i] = t;
        kchain[i] = ch;
    }
    for (int32_t i = 0; i < n; ++i) perm[i] = i;
    std::sort(perm, perm + n, [&](int32_t x, int32_t y) {
        if (ktile[x] != ktile[y]) return ktile[x] < ktile[y];
        if (kchain[x] != kchain[y]) return kchain[x] < kchain[y];
        if (lev[x] != lev[y]) return lev[x] < lev[y];
        return x < y;
    });
    return RWT_OK;
}
