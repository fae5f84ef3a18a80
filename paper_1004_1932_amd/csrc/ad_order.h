/* Host-side ordering of the fused stages' work lists (plain C++, no HIP:
 * the runtime includes it, and a CPU test compiles it on its own). Item is
 * any type with the int fields sys (system), ni (targets) and Nb (spheres of
 * the system); items of one system are contiguous on input. */
#pragma once

#include <algorithm>
#include <vector>

namespace ad {

/* XCD-aware order of a fused work list of many systems. Work-groups go to
 * the 8 XCDs round-robin (work-group i to XCD i mod 8), and each XCD has an
 * L2 of its own. Each system gets one XCD (largest first, to the XCD with the
 * least pair work so far) and its items take positions congruent to that XCD
 * mod 8, so that all of a system's work-groups read its sources through one
 * L2. Each XCD keeps its items longest first; a position whose XCD has run
 * out takes the next item of the XCD with the most left. With few systems
 * the XCDs could not be balanced, so their list keeps the plain order. */
template <class Item>
void xcd_order(std::vector<Item>& v) {
    constexpr int X = 8;
    std::vector<std::vector<Item>> q(X);
    long long load[X] = {};
    int nsys = 0;
    for (size_t k = 0; k < v.size();) {
        size_t e = k;
        while (e < v.size() && v[e].sys == v[k].sys) ++e;
        ++nsys;
        k = e;
    }
    if (nsys < 8 * X) return;
    for (size_t k = 0; k < v.size();) {
        size_t e = k;
        while (e < v.size() && v[e].sys == v[k].sys) ++e;
        const int x = (int)(std::min_element(load, load + X) - load);
        for (size_t j = k; j < e; ++j) {
            q[x].push_back(v[j]);
            load[x] += (long long)v[j].ni * v[j].Nb;
        }
        k = e;
    }
    std::vector<size_t> head(X, 0);
    std::vector<Item> out;
    out.reserve(v.size());
    while (out.size() < v.size()) {
        const int x = (int)(out.size() % X);
        int from = x;
        if (head[x] == q[x].size()) {
            size_t best = 0;
            for (int y = 0; y < X; ++y)
                if (q[y].size() - head[y] > best) {
                    best = q[y].size() - head[y];
                    from = y;
                }
        }
        out.push_back(q[from][head[from]++]);
    }
    v.swap(out);
}

}  // namespace ad
