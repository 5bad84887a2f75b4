"""The grouping of lattices and the two-lane schedule (host logic, no GPU):
the planner header is compiled with g++ into a checker that plans rounds for
many random group sizes and round lengths and checks the schedule's
invariants.

- Every group makes exactly k steps in the round, in order: a group on one
  lane has one item [0, k); the split group has its first s steps at the
  start of lane 1 and the rest [s, k) at the end of lane 0.
- Lane 0 holds groups 0..cut and lane 1 groups cut..n-1, each in order.
- At most one group is split, and only when the half falls inside it.
- The halves balance: |work(lane 0) - work(lane 1)| <= (2 r + 1) w_cut,
  r the rounding of lane 0's share (half a graph replay of 32 steps when
  the round holds two or more, half a step otherwise), w_cut the nodes of
  the split group.
- Whole-group assignment (the server's chunks): every group on a lane, and
  the larger lane holds at most half the work plus the largest group.
- Cache groups: contiguous and non-empty, never across a change of kernel
  variant, as many per run of one variant as its bytes need at the budget
  (at least the minimum, at most one per lattice), each within its share of
  the run plus one lattice.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1903_01168_amd", "csrc")

CHECKER = r"""
#include <cstdio>
#include <cstdlib>
#include <random>
#include "cg_schedule.hpp"

static int fail(const char *what, int c) { std::printf("FAIL case %d: %s\n", c, what); return 1; }

int main()
{
    std::mt19937_64 rng(12345);
    const int G = 32;
    const long long ks[] = {1, 2, 7, 31, 32, 33, 63, 64, 65, 100, 200, 255, 256};
    int cases = 0;
    for (int rep = 0; rep < 4000; ++rep) {
        const int ng = 2 + (int)(rng() % 9);
        std::vector<long long> w(ng);
        const int mode = rep % 3;
        for (auto &x : w) x = mode == 0 ? 262144 : (mode == 1 ? 1 + (long long)(rng() % 1000000)
                                                             : (long long)(1 + rng() % 64) * 4096);
        for (long long k : ks) {
            ++cases;
            const cgs::RoundPlan p = cgs::plan_round(w, k, G);
            std::vector<long long> got(ng, 0);
            std::vector<int> seen(ng, 0);
            double load[2] = {0, 0};
            for (int l = 0; l < 2; ++l) {
                int prev = -1;
                for (const auto &it : p.lane[l]) {
                    if (it.group < 0 || it.group >= ng || it.steps <= 0) return fail("bad item", cases);
                    if (it.group <= prev) return fail("lane not in group order", cases);
                    prev = it.group;
                    got[it.group] += it.steps;
                    seen[it.group] |= 1 << l;
                    load[l] += (double)w[it.group] * (double)it.steps;
                    if (it.first != 0 && !(l == 0 && it.group == p.cut)) return fail("item not at step 0", cases);
                }
            }
            int both = 0;
            for (int g = 0; g < ng; ++g) {
                if (got[g] != k) return fail("group without exactly k steps", cases);
                if (seen[g] == 3) ++both;
            }
            if (both > 1) return fail("more than one group split", cases);
            if (both == 1) {
                const int c = p.cut;
                if (c < 0 || seen[c] != 3) return fail("split group not reported", cases);
                if (!p.straddle) return fail("split without straddle", cases);
                const auto &a = p.lane[1].front(), &b = p.lane[0].back();
                if (a.group != c || b.group != c) return fail("split parts not at lane 1 start / lane 0 end", cases);
                if (a.first != 0 || b.first != a.steps || a.steps + b.steps != k) return fail("split steps", cases);
                for (const auto &it : p.lane[0]) if (it.group > c) return fail("lane 0 beyond cut", cases);
                for (const auto &it : p.lane[1]) if (it.group < c) return fail("lane 1 before cut", cases);
                if (k >= 2 * G && b.steps % G != 0) return fail("lane 0 share not whole replays", cases);
            } else if (p.cut != -1) {
                return fail("cut reported without a split", cases);
            }
            // balance
            int cut = -1;
            double acc = 0, tot = 0;
            for (long long x : w) tot += (double)x;
            for (int g = 0; g < ng; ++g) {
                if (acc + (double)w[g] > 0.5 * tot * (1 + 1e-9)) { cut = g; break; }
                acc += (double)w[g];
            }
            const double r = k >= 2 * G ? G / 2.0 : 0.5;
            const double wc = cut >= 0 ? (double)w[cut] : 0.0;
            if (std::abs(load[0] - load[1]) > (2 * r + 1) * wc + 1e-6 * tot * (double)k)
                return fail("lanes out of balance", cases);
        }
        // whole groups (server chunks)
        const std::vector<int> lane = cgs::assign_whole(w);
        double L[2] = {0, 0}, tot = 0, mx = 0;
        for (int g = 0; g < ng; ++g) {
            if (lane[g] != 0 && lane[g] != 1) return fail("whole: bad lane", cases);
            L[lane[g]] += (double)w[g];
            tot += (double)w[g];
            mx = std::max(mx, (double)w[g]);
        }
        if (std::max(L[0], L[1]) > 0.5 * tot + mx + 1e-9) return fail("whole: out of balance", cases);
    }
    // cache groups: contiguous, non-empty, never across a change of kind, as
    // many per run of one kind as its bytes need (at least min_groups, at
    // most one per lattice), each within its share plus one lattice
    for (int rep = 0; rep < 20000; ++rep) {
        ++cases;
        const int n = 1 + (int)(rng() % 12);
        std::vector<size_t> bytes(n);
        std::vector<char> kind(n);
        for (int i = 0; i < n; ++i) {
            bytes[i] = (size_t)(1 + rng() % 400) << 20;
            kind[i] = (char)(rep % 4 == 0 ? 0 : rng() % 3);
        }
        const size_t budget = (size_t)(32 + rng() % 300) << 20;
        const int ming = 1 + (int)(rng() % 3);
        const std::vector<int> f = cgs::cache_groups(bytes, kind, budget, ming);
        if (f.front() != 0 || f.back() != n) return fail("groups: ends", cases);
        for (size_t j = 0; j + 1 < f.size(); ++j) {
            if (f[j + 1] <= f[j]) return fail("groups: empty or unordered", cases);
            for (int i = f[j] + 1; i < f[j + 1]; ++i)
                if (kind[i] != kind[f[j]]) return fail("groups: mixed kinds", cases);
        }
        for (int a = 0; a < n;) {
            int e = a + 1;
            while (e < n && kind[e] == kind[a]) ++e;
            size_t tot = 0, mx = 0;
            for (int i = a; i < e; ++i) { tot += bytes[i]; mx = std::max(mx, bytes[i]); }
            const long long want = std::min<long long>(e - a, std::max<long long>(ming, (long long)((tot + budget - 1) / budget)));
            long long got = 0;
            for (size_t j = 0; j + 1 < f.size(); ++j) {
                if (f[j] < a || f[j] >= e) continue;
                ++got;
                size_t gb = 0;
                for (int i = f[j]; i < f[j + 1]; ++i) gb += bytes[i];
                if ((double)gb > (double)tot / (double)want + (double)mx + 1.0) return fail("groups: over share", cases);
            }
            if (got != want) return fail("groups: count", cases);
            a = e;
        }
    }
    std::printf("ok %d cases\n", cases);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_two_lane_schedule(tmp_path):
    src = tmp_path / "check.cpp"
    src.write_text(CHECKER)
    exe = tmp_path / "check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I" + CSRC, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok ")
