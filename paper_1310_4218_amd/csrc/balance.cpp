// Host load balancers of the library: GreedyLB, RefineLB and RefineSwapLB over chunk loads
// (Section VI of the paper: GreedyLB in Experiment A, RefineSwapLB in
// Experiments B and C; Refine is its move-only part).
//
// Chunks are the paper's virtual processors, slots its processors.  All
// decisions are made on FP64 loads with a fixed operation order, so that the
// same loads always give the same map:
//   - chunk order: load descending, then chunk id ascending;
//   - slot choice: lowest load, then lowest slot index;
//   - W (total load) sums the loads in chunk id order, slot loads accumulate in
//     chunk id order, limit = (W / S) * threshold.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <functional>
#include <queue>
#include <set>
#include <utility>
#include <vector>

#include "lbgrid_internal.h"

namespace lbgrid {

namespace {

// Chunks by load descending, equal loads in ascending ids.  Loads are
// non-negative doubles, whose bit patterns order like their values, so a
// stable least-significant-digit radix sort of the complemented bits (from id
// order) gives exactly that order; bytes that are the same in every key need
// no pass.
std::vector<int32_t> heavy_first(const double* w, int32_t C) {
    std::vector<int32_t> ord(static_cast<size_t>(C));
    for (int32_t c = 0; c < C; ++c) ord[c] = c;
    if (C < 64) {
        std::sort(ord.begin(), ord.end(),
                  [w](int32_t a, int32_t b) { return w[a] > w[b] || (w[a] == w[b] && a < b); });
        return ord;
    }
    std::vector<uint64_t> key(static_cast<size_t>(C));
    for (int32_t c = 0; c < C; ++c) {
        const double v = w[c] == 0.0 ? 0.0 : w[c];   // -0.0 orders as +0.0
        uint64_t bits;
        std::memcpy(&bits, &v, sizeof(bits));
        key[c] = ~bits;
    }
    std::vector<int32_t> tmp(static_cast<size_t>(C));
    int32_t count[256];
    for (int pass = 0; pass < 8; ++pass) {
        const int shift = 8 * pass;
        std::memset(count, 0, sizeof(count));
        for (int32_t c = 0; c < C; ++c) ++count[(key[c] >> shift) & 0xff];
        if (count[(key[0] >> shift) & 0xff] == C) continue;
        int32_t run = 0;
        for (int d = 0; d < 256; ++d) {
            const int32_t x = count[d];
            count[d] = run;
            run += x;
        }
        for (int32_t i = 0; i < C; ++i) {
            const int32_t c = ord[i];
            tmp[count[(key[c] >> shift) & 0xff]++] = c;
        }
        ord.swap(tmp);
    }
    return ord;
}

// GreedyLB: heaviest chunk first onto the least loaded slot.  A binary heap of
// (load, slot) pairs gives the lowest load with the lowest index on ties.
void greedy(const double* w, int32_t C, int32_t S, int32_t* map) {
    using Entry = std::pair<double, int32_t>;
    std::vector<Entry> empty(static_cast<size_t>(S));
    for (int32_t s = 0; s < S; ++s) empty[s] = {0.0, s};   // ascending: already a min-heap
    std::priority_queue<Entry, std::vector<Entry>, std::greater<Entry>> heap(std::greater<Entry>(),
                                                                             std::move(empty));
    for (int32_t c : heavy_first(w, C)) {
        Entry e = heap.top();
        heap.pop();
        map[c] = e.second;
        heap.push({e.first + w[c], e.second});
    }
}

// RefineLB: while the most loaded slot p (not yet given up) is above the limit,
// move its heaviest chunk that still fits under the limit on the least loaded
// slot q; give p up when no chunk fits.  A chunk moved onto q never makes q
// exceed the limit, so a slot that receives chunks is never a source later
// and every chunk moves at most once.
void refine(const double* w, const int32_t* old_map, int32_t C, int32_t S, double thr,
            int32_t* map) {
    double W = 0.0;
    for (int32_t c = 0; c < C; ++c) W += w[c];
    const double limit = (W / static_cast<double>(S)) * thr;

    std::vector<double> L(static_cast<size_t>(S), 0.0);
    for (int32_t c = 0; c < C; ++c) {
        map[c] = old_map[c];
        L[map[c]] += w[c];
    }
    // per-slot chunk lists in heavy-first order
    std::vector<std::vector<int32_t>> on(static_cast<size_t>(S));
    for (int32_t c : heavy_first(w, C)) on[map[c]].push_back(c);

    // Slots ordered two ways, updated as loads change: `hi` holds the slots not
    // given up, most loaded first (lowest index on ties), `lo` every slot, least
    // loaded first (lowest index on ties); the same choices as linear scans.
    auto more = [&L](int32_t a, int32_t b) { return L[a] > L[b] || (L[a] == L[b] && a < b); };
    auto less = [&L](int32_t a, int32_t b) { return L[a] < L[b] || (L[a] == L[b] && a < b); };
    std::set<int32_t, decltype(more)> hi(more);
    std::set<int32_t, decltype(less)> lo(less);
    for (int32_t s = 0; s < S; ++s) {
        hi.insert(s);
        lo.insert(s);
    }
    while (!hi.empty()) {
        const int32_t p = *hi.begin();
        if (!(L[p] > limit)) break;
        const int32_t q = *lo.begin();
        // L[q] + w[c] is non-increasing along the heavy-first list: binary search
        // for the first chunk whose move keeps q at or under the limit.
        std::vector<int32_t>& lp = on[p];
        const double Lq = L[q];
        auto it = std::partition_point(lp.begin(), lp.end(),
                                       [&](int32_t c) { return !(Lq + w[c] <= limit); });
        if (it == lp.end() || p == q) {
            hi.erase(p);   // given up
            continue;
        }
        int32_t c = *it;
        lp.erase(it);
        map[c] = q;
        hi.erase(p);
        lo.erase(p);
        lo.erase(q);
        const bool q_active = hi.erase(q) > 0;
        L[p] -= w[c];
        L[q] += w[c];
        hi.insert(p);
        lo.insert(p);
        lo.insert(q);
        if (q_active) hi.insert(q);
        std::vector<int32_t>& lq = on[q];
        auto pos = std::lower_bound(lq.begin(), lq.end(), c, [w](int32_t a, int32_t b) {
            return w[a] > w[b] || (w[a] == w[b] && a < b);
        });
        lq.insert(pos, c);
    }
}

// RefineSwapLB: as refine(), but when no chunk of p fits on the least loaded
// slot, make the first swap that fits (slots r != p by increasing load then
// index, p's chunks heavy first, r's chunks light first, ties by id):
// w[d] < w[c] and L[r] + (w[c] - w[d]) <= limit; give p up only when neither a
// move nor a swap fits.  At most 4*C moves and swaps in total.
void refine_swap(const double* w, const int32_t* old_map, int32_t C, int32_t S, double thr,
                 int32_t* map) {
    double W = 0.0;
    for (int32_t c = 0; c < C; ++c) W += w[c];
    const double limit = (W / static_cast<double>(S)) * thr;
    std::vector<double> L(static_cast<size_t>(S), 0.0);
    for (int32_t c = 0; c < C; ++c) {
        map[c] = old_map[c];
        L[map[c]] += w[c];
    }
    auto heavier = [w](int32_t a, int32_t b) { return w[a] > w[b] || (w[a] == w[b] && a < b); };
    auto lighter = [w](int32_t a, int32_t b) { return w[a] < w[b] || (w[a] == w[b] && a < b); };
    std::vector<std::vector<int32_t>> on(static_cast<size_t>(S));  // heavy-first per slot
    for (int32_t c : heavy_first(w, C)) on[map[c]].push_back(c);
    auto insert = [&](int32_t s, int32_t c) {
        auto& v = on[s];
        v.insert(std::lower_bound(v.begin(), v.end(), c, heavier), c);
    };
    auto remove = [&](int32_t s, int32_t c) {
        auto& v = on[s];
        v.erase(std::lower_bound(v.begin(), v.end(), c, heavier));
    };

    std::vector<char> given_up(static_cast<size_t>(S), 0);
    std::vector<int32_t> by_load(static_cast<size_t>(S));
    for (int64_t ops = 0; ops < 4 * static_cast<int64_t>(C);) {
        int32_t p = -1;
        for (int32_t s = 0; s < S; ++s)
            if (!given_up[s] && (p < 0 || L[s] > L[p])) p = s;
        if (p < 0 || !(L[p] > limit)) break;
        const int32_t q = static_cast<int32_t>(std::min_element(L.begin(), L.end()) - L.begin());
        const double Lq = L[q];
        auto it = std::partition_point(on[p].begin(), on[p].end(),
                                       [&](int32_t c) { return !(Lq + w[c] <= limit); });
        if (it != on[p].end() && p != q) {
            const int32_t c = *it;
            on[p].erase(it);
            map[c] = q;
            L[p] -= w[c];
            L[q] += w[c];
            insert(q, c);
            ++ops;
            continue;
        }
        for (int32_t s = 0; s < S; ++s) by_load[s] = s;
        std::sort(by_load.begin(), by_load.end(),
                  [&](int32_t a, int32_t b) { return L[a] < L[b] || (L[a] == L[b] && a < b); });
        int32_t sc = -1, sd = -1, sr = -1;
        for (int32_t r : by_load) {
            if (r == p) continue;
            std::vector<int32_t> lr(on[r].begin(), on[r].end());
            std::sort(lr.begin(), lr.end(), lighter);
            for (int32_t c : on[p]) {
                for (int32_t d : lr) {
                    if (!(w[d] < w[c])) break;  // light first: no lighter chunk follows
                    if (L[r] + (w[c] - w[d]) <= limit) {
                        sc = c;
                        sd = d;
                        break;
                    }
                }
                if (sc >= 0) break;
            }
            if (sc >= 0) {
                sr = r;
                break;
            }
        }
        if (sc < 0) {
            given_up[p] = 1;
            continue;
        }
        remove(p, sc);
        remove(sr, sd);
        map[sc] = sr;
        map[sd] = p;
        L[p] = (L[p] - w[sc]) + w[sd];
        L[sr] = (L[sr] - w[sd]) + w[sc];
        insert(sr, sc);
        insert(p, sd);
        ++ops;
    }
}

}  // namespace

void block_map(int32_t C, int32_t S, int32_t* map) {
    for (int32_t c = 0; c < C; ++c)
        map[c] = (C >= S) ? static_cast<int32_t>((static_cast<int64_t>(c) * S) / C) : c;
}

double imbalance(const double* w, const int32_t* map, int32_t C, int32_t S) {
    std::vector<double> L(static_cast<size_t>(S), 0.0);
    double W = 0.0;
    for (int32_t c = 0; c < C; ++c) {
        L[map[c]] += w[c];
        W += w[c];
    }
    if (!(W > 0.0)) return 1.0;
    return *std::max_element(L.begin(), L.end()) / (W / static_cast<double>(S));
}

int balance(const double* w, const int32_t* old_map, int32_t C, int32_t S, int strategy,
            double threshold, int32_t* map_out) {
    if (C < 0 || S < 1 || (C > 0 && (!w || !map_out))) return -1;
    for (int32_t c = 0; c < C; ++c)
        if (!(w[c] >= 0.0)) return -1;  // rejects negatives and NaN
    if (strategy == kGreedy) {
        greedy(w, C, S, map_out);
        return 0;
    }
    if (strategy == kRefine || strategy == kRefineSwap) {
        if (!old_map || !(threshold > 0.0)) return -1;
        for (int32_t c = 0; c < C; ++c)
            if (old_map[c] < 0 || old_map[c] >= S) return -1;
        if (strategy == kRefine)
            refine(w, old_map, C, S, threshold, map_out);
        else
            refine_swap(w, old_map, C, S, threshold, map_out);
        return 0;
    }
    return -2;
}

}  // namespace lbgrid
