// Plan-time octree over the sorted Morton keys of all points (host code).
#include <algorithm>

#include "ph_internal.h"

namespace ph {

// Boxes level by level in octant (Morton) order.  A box splits while it holds more than
// leaf_cap points; its children are the runs of its keys that share the next three bits.
// Colleagues (the 27 boxes of the same level around a box, itself at slot 13) come from the
// parent's colleagues' children.
void build_full_tree(const std::vector<uint64_t> &keys, int leaf_cap, int depth_limit, FullTree &T)
{
    const int64_t n = (int64_t)keys.size();
    auto add = [&](int l, int x, int y, int z, int64_t b, int64_t e, int32_t par) {
        T.level.push_back(l);
        T.ax.push_back(x);
        T.ay.push_back(y);
        T.az.push_back(z);
        T.start.push_back((int32_t)b);
        T.end.push_back((int32_t)e);
        T.parent.push_back(par);
        for (int o = 0; o < 8; ++o) T.child.push_back(-1);
        for (int d = 0; d < 27; ++d) T.coll.push_back(-1);
    };
    add(0, 0, 0, 0, 0, n, -1);
    T.coll[13] = 0;
    T.level_cap.assign(1, 1);
    int64_t lb = 0, le = 1;  // boxes of the current level
    for (int l = 0; l < depth_limit; ++l) {
        const int shift = 3 * (kMortonBits - (l + 1));
        const int64_t first_new = (int64_t)T.level.size();
        for (int64_t f = lb; f < le; ++f) {
            const int64_t b = T.start[f], e = T.end[f];
            if (e - b <= leaf_cap) continue;
            const uint64_t pre = ((uint64_t)0 + (keys[b] >> (shift + 3))) << 3;
            for (int o = 0; o < 8; ++o) {
                const uint64_t lo_key = (pre | (uint64_t)o) << shift;
                const uint64_t hi_key = ((pre | (uint64_t)o) + 1) << shift;
                const int64_t cb = std::lower_bound(keys.begin() + b, keys.begin() + e, lo_key) - keys.begin();
                const int64_t ce = std::lower_bound(keys.begin() + b, keys.begin() + e, hi_key) - keys.begin();
                if (ce == cb) continue;
                T.child[(size_t)f * 8 + o] = (int32_t)T.level.size();
                add(l + 1, 2 * T.ax[f] + ((o >> 2) & 1), 2 * T.ay[f] + ((o >> 1) & 1), 2 * T.az[f] + (o & 1), cb, ce,
                    (int32_t)f);
            }
        }
        const int64_t last_new = (int64_t)T.level.size();
        if (last_new == first_new) break;
        T.level_cap.push_back(last_new - first_new);
        // colleagues of the new level from the parents' colleagues
        const int lim = 1 << (l + 1);
        for (int64_t f = first_new; f < last_new; ++f) {
            const int x = T.ax[f], y = T.ay[f], z = T.az[f];
            const int32_t par = T.parent[f];
            for (int d = 0; d < 27; ++d) {
                const int nx = x + d / 9 - 1, ny = y + (d / 3) % 3 - 1, nz = z + d % 3 - 1;
                int32_t res = -1;
                if (nx >= 0 && ny >= 0 && nz >= 0 && nx < lim && ny < lim && nz < lim) {
                    const int dp = ((nx >> 1) - (x >> 1) + 1) * 9 + ((ny >> 1) - (y >> 1) + 1) * 3 + ((nz >> 1) - (z >> 1) + 1);
                    const int32_t P = T.coll[(size_t)par * 27 + dp];
                    if (P >= 0) res = T.child[(size_t)P * 8 + (((nx & 1) << 2) | ((ny & 1) << 1) | (nz & 1))];
                }
                T.coll[(size_t)f * 27 + d] = res;
            }
        }
        lb = first_new;
        le = last_new;
    }
}

}  // namespace ph
