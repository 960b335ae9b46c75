// Host check of the 3-way tile sets: the flattened (pair row, k column) tiles
// of the VALU slices cover every triple of a stage exactly once (pair_j
// inverts the colex pair offset), and so do the two parts of the split
// tiling of the matrix-core slices (colex pairs x k, then lex pairs x i;
// lex_pair inverts the lex order); for every slab j of n_v in a range of
// sizes, the matrix-core slices' whole tiles plus edge tiles, and the single
// set of all tiles, cover the rectangle i < j < k exactly once, with every
// tile origin inside it; the finish's output ranges cover each slab exactly
// once.  Prints "ok" and exits 0 on success.
#include <cstdio>
#include <vector>

#include "../paper_1705_08210_amd/csrc/ps_internal.h"

using namespace ps;

static long cover(int64_t n, int64_t j, int mode, int bm, int ob, std::vector<int>& cov) {
    long bad = 0;
    const int64_t wk = n - 1 - j;
    const int64_t cnt = slab_tile_count(n, j, bm, mode, ob);
    for (int64_t l = 0; l < cnt; ++l) {
        int64_t r0, c0;
        slab_tile_origin(n, j, l, bm, mode, ob, r0, c0);
        if (r0 < 0 || r0 >= j || c0 <= j || c0 >= n) {
            ++bad;
            continue;
        }
        for (int64_t i = r0; i < r0 + bm && i < j; ++i)
            for (int64_t k = c0; k < c0 + bm && k < n; ++k) cov[(size_t)(i * wk + (k - j - 1))]++;
    }
    return bad;
}

// The flattened tiling of a stage [jb, je): every triple (i, j, k) with
// jb <= j < je lies in exactly one (row tile, column tile), and no tile
// reaches outside the stage's rows or past n_v.
static long cover_flat(int64_t n, int64_t jb, int64_t je, int bm) {
    const int64_t pb = jb * (jb - 1) / 2, pe = je * (je - 1) / 2;
    std::vector<int> cov((size_t)((pe - pb) * n), 0);
    long bad = 0;
    const int64_t nr = flat_row_tiles(jb, je, bm);
    if (nr * bm < pe - pb || (nr > 0 && (nr - 1) * bm >= pe - pb)) ++bad;
    for (int64_t rt = 0; rt < nr; ++rt) {
        const int64_t p0 = pb + rt * bm;
        const int64_t jmin = pair_j(p0);
        if (jmin < jb || jmin >= je) ++bad;
        for (int64_t c = 0; c < flat_col_tiles(n, jb, bm, rt); ++c) {
            const int64_t k0 = jmin + 1 + c * bm;
            if (k0 >= n) ++bad;
            for (int64_t p = p0; p < p0 + bm && p < pe; ++p) {
                const int64_t j = pair_j(p), i = p - j * (j - 1) / 2;
                if (i < 0 || i >= j) ++bad;
                for (int64_t k = k0; k < k0 + bm && k < n; ++k)
                    if (k > j) cov[(size_t)((p - pb) * n + k)]++;
            }
        }
    }
    for (int64_t p = pb; p < pe; ++p) {
        const int64_t j = pair_j(p);
        for (int64_t k = 0; k < n; ++k) bad += cov[(size_t)((p - pb) * n + k)] != (k > j ? 1 : 0);
    }
    return bad;
}

// The lex-ordered tiling of a stage [jb, je) (the second part of the split
// tiling of the matrix-core slices): rows are the pairs (j, k), jb <= j < je,
// in lex order, lex_pair inverts the order, and every triple (i, j, k) lies
// in exactly one (row tile, column tile) with columns i below n_v.
static long cover_lex(int64_t n, int64_t jb, int64_t je, int bm) {
    const int64_t qb = lex_first(n, jb), qe = lex_first(n, je);
    std::vector<int> cov((size_t)((qe - qb) * n), 0);
    long bad = 0;
    const int64_t nr = lex_row_tiles(n, jb, je, bm);
    if (nr * bm < qe - qb || (nr > 0 && (nr - 1) * bm >= qe - qb)) ++bad;
    for (int64_t rt = 0; rt < nr; ++rt) {
        const int64_t q0 = qb + rt * bm;
        for (int64_t c = 0; c < lex_col_tiles(n, jb, je, bm, rt); ++c) {
            const int64_t i0 = c * bm;
            if (i0 >= n) ++bad;
            for (int64_t q = q0; q < q0 + bm && q < qe; ++q) {
                int64_t j, k;
                lex_pair(n, q, j, k);
                if (j < jb || j >= je || k <= j || k >= n) ++bad;
                for (int64_t i = i0; i < i0 + bm && i < n; ++i)
                    if (i < j) cov[(size_t)((q - qb) * n + i)]++;
            }
        }
    }
    for (int64_t q = qb; q < qe; ++q) {
        int64_t j, k;
        lex_pair(n, q, j, k);
        for (int64_t i = 0; i < n; ++i) bad += cov[(size_t)((q - qb) * n + i)] != (i < j ? 1 : 0);
    }
    return bad;
}

int main() {
    long bad = 0, slabs = 0;
    for (int64_t p = 0; p < 2000000; p += 7) {   // pair_j inverts the colex offset
        const int64_t j = pair_j(p);
        bad += !(j * (j - 1) / 2 <= p && p < j * (j + 1) / 2);
    }
    for (int64_t n : {2, 3, 4, 9, 100, 1000, 4096})   // lex_pair inverts the lex order
        for (int64_t j = 0, q = 0; j < n - 1; ++j)
            for (int64_t k = j + 1; k < n; ++k, ++q) {
                int64_t jj, kk;
                lex_pair(n, q, jj, kk);
                bad += jj != j || kk != k || lex_first(n, j) > q || q >= lex_first(n, j + 1);
            }
    for (int64_t n : {3, 4, 5, 17, 64, 65, 130, 257, 300})
        for (int bm : {64, 128, 256})
            for (int64_t jb = 1; jb < n - 1; jb += (n > 100 ? 37 : 1))
                for (int64_t je = jb; je <= n - 1; je += (n > 100 ? 53 : 1)) {
                    // the split point divides any stage between the two parts
                    const int64_t js = split3(n, jb, je);
                    bad += js < jb || js > je;
                    bad += cover_flat(n, jb, js, bm) + cover_lex(n, js, je, bm);
                }
    for (int64_t n : {3, 4, 5, 17, 64, 65, 130, 257, 300})
        for (int bm : {64, 128})
            for (int64_t jb = 1; jb < n - 1; jb += (n > 100 ? 37 : 1))
                for (int64_t je = jb; je <= n - 1; je += (n > 100 ? 53 : 1)) {
                    bad += cover_flat(n, jb, je, bm);
                    bad += cover_flat(n, jb, n - 1, bm);
                }
    for (int64_t n = 3; n <= 700; n += (n < 300 ? 1 : 37)) {
        for (int64_t j = 1; j < n - 1; ++j) {
            const size_t m = (size_t)(j * (n - 1 - j));
            for (int ob : {128, 256}) {
                std::vector<int> cov(m, 0);
                bad += cover(n, j, kSlabFull, ob, ob, cov);
                bad += cover(n, j, kSlabEdge, ob / 2, ob, cov);
                for (int c : cov) bad += c != 1;
            }
            for (int bm : {64, 128, 256}) {
                std::vector<int> cov(m, 0);
                bad += cover(n, j, kSlabAll, bm, bm, cov);
                for (int c : cov) bad += c != 1;
            }
            const int64_t r = slab_tile_count(n, j, 2048, kSlabRange, 0);
            bad += r * 2048 < (int64_t)m || (r - 1) * 2048 >= (int64_t)m;
            ++slabs;
        }
    }
    if (bad) {
        std::printf("tile sets: %ld errors over %ld slabs\n", bad, slabs);
        return 1;
    }
    std::printf("ok %ld slabs\n", slabs);
    return 0;
}
