// cg_schedule.hpp -- how lattices stepped together are cut into groups that
// stay in the last-level cache, and how two lanes (streams) share the
// groups.  Host-only planning with no HIP dependency.
//
// A launch's wavefronts all start together but finish over a spread of
// times; a second launch in flight on another stream fills the slots the
// first one's early finishers free.  Two groups are therefore stepped at a
// time, each group's steps in order on one lane at a time.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace cgs {

// Lattices stepped together, in order, split into contiguous groups: as many
// as the total of `bytes` (the device bytes each lattice's steps touch)
// needs at `budget` per group, at least `min_groups`, at most one per
// lattice; a group closes once the groups so far hold their share of the
// total, or when the lattices left are just enough for one group each.
// Returns the first index of each group, then the end.
inline std::vector<int> cache_groups(const std::vector<size_t> &bytes, size_t budget, int min_groups)
{
    const int n = (int)bytes.size();
    size_t total = 0;
    for (size_t b : bytes) total += b;
    const size_t want = std::max<size_t>((size_t)std::max(min_groups, 1), (total + budget - 1) / budget);
    const int ng = (int)std::min<size_t>((size_t)std::max(n, 1), want);
    std::vector<int> first(1, 0);
    size_t acc = 0;
    for (int i = 0, g = 1; i + 1 < n && g < ng; ++i) {
        acc += bytes[i];
        if (acc * ng >= total * g || n - (i + 1) == ng - g) {
            first.push_back(i + 1);
            ++g;
        }
    }
    first.push_back(n);
    return first;
}

// The same within each run of consecutive lattices of one kind (kind[i]: the
// step-kernel variant the lattice needs), so that every lattice is stepped by
// the kernel variant it would get alone and its result does not depend on
// its neighbours.
inline std::vector<int> cache_groups(const std::vector<size_t> &bytes, const std::vector<char> &kind, size_t budget,
                                     int min_groups)
{
    std::vector<int> first(1, 0);
    const int n = (int)bytes.size();
    for (int a = 0; a < n;) {
        int e = a + 1;
        while (e < n && kind[e] == kind[a]) ++e;
        const std::vector<int> f =
            cache_groups(std::vector<size_t>(bytes.begin() + a, bytes.begin() + e), budget, min_groups);
        for (size_t j = 1; j < f.size(); ++j) first.push_back(a + f[j]);
        a = e;
    }
    if (n == 0) first.push_back(0);
    return first;
}

// `steps` consecutive steps of group `group`, starting `first` steps into
// the round.
struct LaneItem {
    int group;
    int64_t first;
    int64_t steps;
};

struct RoundPlan {
    std::vector<LaneItem> lane[2];
    int cut = -1;           // group with steps on both lanes (-1: none)
    bool straddle = false;  // the half falls inside a group: the lanes meet at the end of the round
};

// One round of k steps for every group, the groups' work (nodes x steps)
// halved between the lanes in group order, wrapping around (McNaughton's
// schedule for two machines): lane 0 takes the first groups, lane 1 the
// last ones, and the group in which the half falls makes its first steps at
// the start of lane 1 and its last steps at the end of lane 0 (the caller
// orders the two parts with an event).  Lane 0's share of that group is
// rounded to whole graph replays of `graph_steps` steps when the round holds
// at least two of them.  Where the half falls inside a group the group may
// sit differently in a shorter round, so the caller makes the lanes meet at
// the end of such a round.
inline RoundPlan plan_round(const std::vector<long long> &nodes, int64_t k, int graph_steps)
{
    RoundPlan p;
    const int ng = (int)nodes.size();
    double total = 0;
    for (long long w : nodes) total += (double)w;
    const double half = 0.5 * total;
    int cut = ng;           // first group not wholly on lane 0
    int64_t s1 = 0;         // its first s1 steps run on lane 1
    double acc = 0;
    for (int gi = 0; gi < ng; ++gi) {
        const double w = (double)nodes[gi];
        if (acc + w <= half * (1 + 1e-9)) {
            acc += w;
            continue;
        }
        cut = gi;
        const double f0 = (half - acc) / w;   // lane 0's fraction of the group
        p.straddle = f0 > 1e-9;
        int64_t on0 = (int64_t)std::llround(f0 * (double)k);
        if (k >= 2 * (int64_t)graph_steps) on0 = (on0 + graph_steps / 2) / graph_steps * graph_steps;
        on0 = std::max<int64_t>(0, std::min<int64_t>(k, on0));
        s1 = k - on0;
        break;
    }
    if (cut < ng && s1 > 0) p.lane[1].push_back({cut, 0, s1});
    for (int gi = cut + 1; gi < ng; ++gi) p.lane[1].push_back({gi, 0, k});
    for (int gi = 0; gi < std::min(cut, ng); ++gi) p.lane[0].push_back({gi, 0, k});
    if (cut < ng && s1 < k) p.lane[0].push_back({cut, s1, k - s1});
    if (cut < ng && s1 > 0 && s1 < k) p.cut = cut;
    return p;
}

// Whole groups to two lanes: largest first, each to the lane with less work
// so far (ties to lane 0).  Returns each group's lane.
inline std::vector<int> assign_whole(const std::vector<long long> &nodes)
{
    const int ng = (int)nodes.size();
    std::vector<int> lane(ng, 0), order(ng);
    for (int g = 0; g < ng; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nodes[a] > nodes[b]; });
    long long load[2] = {0, 0};
    for (int g : order) {
        const int l = load[1] < load[0] ? 1 : 0;
        lane[g] = l;
        load[l] += nodes[g];
    }
    return lane;
}

}  // namespace cgs
