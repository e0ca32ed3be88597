// Stencil tiling plan and receiver buckets (host code; declarations in plan.h).

#include <algorithm>

#include "plan.h"

namespace wv {

ChunkPlan plan_chunks(int nz, int tiles, int target)
{
    WV_REQUIRE(nz >= 1 && tiles >= 1 && target >= 1, WV_EINVAL, "plan_chunks: sizes must be >= 1");
    int chunks = (target + tiles - 1) / tiles;
    chunks = std::max(1, std::min(chunks, nz / 8 > 0 ? nz / 8 : 1));
    int kc = (nz + chunks - 1) / chunks;
    if (kc >= 8) kc = (kc + 7) / 8 * 8;
    return ChunkPlan{kc, (nz + kc - 1) / kc};
}

void bucket_receivers(int nz, int bx, int by, int tiles_x, int tiles_y, const std::vector<int>& rec_kji,
                      std::vector<int>& ptr, std::vector<RecEnt>& ent)
{
    WV_REQUIRE(nz >= 1 && bx >= 1 && by >= 1 && tiles_x >= 1 && tiles_y >= 1 && rec_kji.size() % 3 == 0,
               WV_EINVAL, "bucket_receivers: bad sizes");
    const int tiles = tiles_x * tiles_y;
    const int n = (int)(rec_kji.size() / 3);
    std::vector<std::vector<RecEnt>> per(tiles);
    for (int q = 0; q < n; ++q) {
        const int k = rec_kji[3 * q], j = rec_kji[3 * q + 1], i = rec_kji[3 * q + 2];
        WV_REQUIRE(k >= 0 && k < nz && j >= 0 && j < tiles_y * by && i >= 0 && i < tiles_x * bx, WV_EINVAL,
                   "bucket_receivers: receiver outside the tiled box");
        per[(j / by) * tiles_x + i / bx].push_back(RecEnt{k, (j % by) * bx + i % bx, q, 0});
    }
    ptr.assign((size_t)tiles * (nz + 1), 0);
    ent.clear();
    ent.reserve(n);
    for (int t = 0; t < tiles; ++t) {
        std::vector<RecEnt>& v = per[t];
        std::stable_sort(v.begin(), v.end(), [](const RecEnt& x, const RecEnt& y) {
            return x.k != y.k ? x.k < y.k : x.local < y.local;
        });
        const int base = (int)ent.size();
        size_t q = 0;
        for (int k = 0; k <= nz; ++k) {
            while (q < v.size() && v[q].k < k) ++q;
            ptr[(size_t)t * (nz + 1) + k] = base + (int)q;
        }
        ent.insert(ent.end(), v.begin(), v.end());
    }
}

}  // namespace wv
