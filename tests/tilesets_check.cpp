// Host check of the 3-way slab tile sets (slab_tile_count / slab_tile_origin):
// for every slab j of n_v in a range of sizes, the whole tiles plus the edge
// tiles, and the single set of all tiles, cover the rectangle i < j < k
// exactly once, with every tile origin inside it; the finish's output ranges
// cover each slab exactly once.  Prints "ok" and exits 0 on success.
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

int main() {
    long bad = 0, slabs = 0;
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
