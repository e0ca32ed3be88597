// Host planning code under test on its own (no GPU): the binomial checkpointing
// schedule, the snapshot map of its first sweep, the stencil's z chunking and the
// receiver buckets. Built by tests/test_host_sanitizers.py with g++ and the address
// and undefined-behaviour sanitizers; prints "host planning: ok" and returns 0 when
// every check holds, else names the first failure and returns 1.

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "plan.h"

using namespace wv;

static int g_fail = 0;
#define CHECK(cond, ...)                                          \
    do {                                                          \
        if (!(cond)) {                                            \
            if (!g_fail) {                                        \
                std::printf("FAIL %s:%d: ", __FILE__, __LINE__);  \
                std::printf(__VA_ARGS__);                         \
                std::printf("\n");                                \
            }                                                     \
            g_fail = 1;                                           \
        }                                                         \
    } while (0)

// Least evaluations to reverse l steps with s slots, by the recursion over the
// first stored step j (brute force over every j).
static long long dp_cost(int l, int s, std::vector<std::vector<long long>>& memo)
{
    if (l <= 1) return 0;
    if (s <= 1) return (long long)l * (l - 1) / 2;
    long long& m = memo[l][s];
    if (m >= 0) return m;
    long long best = -1;
    for (int j = 1; j < l; ++j) {
        const long long c = j + dp_cost(l - j, s - 1, memo) + dp_cost(j, s, memo);
        if (best < 0 || c < best) best = c;
    }
    return m = best;
}

// Executes a schedule on symbolic states: every restore finds the state it names in
// its slot, advances start from the current state, x_{l-1} .. x_0 are delivered in
// that order, slots stay within [0, s), and the advances add up to the reported count.
static void run_schedule(int l, int s)
{
    long long fwd = -1;
    const std::vector<RevAction> acts = revolve_schedule(l, s, &fwd);
    std::vector<int> slot(s, -1);
    slot[0] = 0;
    int cur = -1, next = l - 1;
    long long adv = 0;
    for (const RevAction& a : acts) {
        switch (a.kind) {
        case 0:
            CHECK(cur == a.a && a.b >= 1 && a.a + a.b < l, "advance (%d, %d) from %d, l %d s %d", a.a, a.b, cur, l, s);
            cur = a.a + a.b;
            adv += a.b;
            break;
        case 1:
            CHECK(cur == a.a && a.b >= 1 && a.b < s, "store (%d, slot %d) with current %d, l %d s %d", a.a, a.b, cur,
                  l, s);
            if (a.b >= 0 && a.b < s) slot[a.b] = a.a;
            break;
        case 2:
            CHECK(a.b >= 0 && a.b < s && slot[a.b] == a.a, "restore (%d, slot %d), l %d s %d", a.a, a.b, l, s);
            cur = a.a;
            break;
        case 3:
            CHECK(cur == a.a && a.a == next, "deliver %d, current %d, expected %d, l %d s %d", a.a, cur, next, l, s);
            --next;
            break;
        default:
            CHECK(false, "action kind %d", a.kind);
        }
        if (g_fail) return;
    }
    CHECK(next == -1, "schedule ended with x_%d undelivered, l %d s %d", next, l, s);
    CHECK(adv == fwd, "advances %lld, reported %lld, l %d s %d", adv, fwd, l, s);
    CHECK(fwd == revolve_cost(l, s), "forward steps %lld, cost %lld, l %d s %d", fwd, revolve_cost(l, s), l, s);

    // the first sweep's snapshot map: the stores before the first deliver
    size_t first = 0;
    const std::vector<int> snap = sweep_snapshots(acts, l, &first);
    CHECK(snap.size() == (size_t)l + 1, "snapshot map size");
    CHECK(first < acts.size() && acts[first].kind == 3, "first deliver index %zu", first);
    std::vector<int> want(l + 1, 0);
    for (size_t q = 0; q < first; ++q) {
        CHECK(acts[q].kind != 3, "deliver before index %zu", first);
        if (acts[q].kind == 1) want[acts[q].a] = acts[q].b;
    }
    CHECK(snap == want, "snapshot map, l %d s %d", l, s);
}

static void test_revolve()
{
    const int LMAX = 90, SMAX = 9;
    std::vector<std::vector<long long>> memo(LMAX + 1, std::vector<long long>(SMAX + 1, -1));
    for (int l = 1; l <= LMAX; ++l)
        for (int s = 1; s <= SMAX; ++s) {
            CHECK(revolve_cost(l, s) == dp_cost(l, s, memo), "cost(%d, %d) = %lld, brute force %lld", l, s,
                  revolve_cost(l, s), dp_cost(l, s, memo));
            run_schedule(l, s);
            if (g_fail) return;
        }
    // the workloads' shapes: 2000 and 3000 steps with 64 slots, 4000 with 6
    const int big[][2] = {{2000, 64}, {3000, 64}, {4000, 6}, {7, 64}};
    for (const auto& ls : big) run_schedule(ls[0], ls[1]);
    long long f = 0;
    revolve_schedule(2000, 64, &f);
    CHECK(f == 3934, "2000 steps with 64 slots: %lld forward steps, expected 3934", f);
    // refusals
    const int bad[][2] = {{0, 4}, {5, 0}, {-3, 2}};
    for (const auto& ls : bad) {
        bool threw = false;
        try {
            revolve_schedule(ls[0], ls[1], nullptr);
        } catch (const Error& e) {
            threw = e.code == WV_EINVAL;
        }
        CHECK(threw, "revolve_schedule(%d, %d) accepted", ls[0], ls[1]);
    }
    bool threw = false;
    try {
        size_t first = 0;
        sweep_snapshots({RevAction{1, 9, 1}, RevAction{3, 0, 0}}, 5, &first);
    } catch (const Error& e) {
        threw = e.code == WV_EINVAL;
    }
    CHECK(threw, "sweep_snapshots accepted a store past the end");
}

static void test_chunks()
{
    for (int nz = 1; nz <= 520; ++nz)
        for (int tiles : {1, 3, 32, 128, 2048, 5000})
            for (int target : {1, 2048, 8192}) {
                const ChunkPlan p = plan_chunks(nz, tiles, target);
                CHECK(p.kc >= 1 && p.chunks >= 1, "nz %d: kc %d chunks %d", nz, p.kc, p.chunks);
                CHECK((long long)p.kc * p.chunks >= nz && (long long)p.kc * (p.chunks - 1) < nz,
                      "nz %d tiles %d target %d: %d chunks of %d do not tile z", nz, tiles, target, p.chunks, p.kc);
                CHECK(p.kc < 8 || p.kc % 8 == 0, "nz %d: kc %d not a multiple of 8", nz, p.kc);
                CHECK(p.chunks <= std::max(1, nz / 8), "nz %d: %d chunks", nz, p.chunks);
                if (g_fail) return;
            }
    // 256^3 in 64 x 8 tiles: 128 tiles, 16-level forward and 8-level adjoint chunks
    const ChunkPlan f = plan_chunks(256, 128, 2048), a = plan_chunks(256, 128, 8192);
    CHECK(f.kc == 16 && f.chunks == 16 && a.kc == 8 && a.chunks == 32, "256^3 chunks %d x %d, adjoint %d x %d",
          f.chunks, f.kc, a.chunks, a.kc);
    bool threw = false;
    try {
        plan_chunks(0, 1, 1);
    } catch (const Error& e) {
        threw = e.code == WV_EINVAL;
    }
    CHECK(threw, "plan_chunks accepted nz = 0");
}

static void check_buckets(int nz, int ny, int nx, int bx, int by, const std::vector<int>& kji)
{
    const int tx = (nx + bx - 1) / bx, ty = (ny + by - 1) / by, tiles = tx * ty;
    std::vector<int> ptr;
    std::vector<RecEnt> ent;
    bucket_receivers(nz, bx, by, tx, ty, kji, ptr, ent);
    const int n = (int)kji.size() / 3;
    CHECK(ptr.size() == (size_t)tiles * (nz + 1) && ent.size() == (size_t)n, "sizes");
    std::vector<int> seen(n, 0);
    int prev_end = 0;
    for (int t = 0; t < tiles && !g_fail; ++t) {
        const int* p = ptr.data() + (size_t)t * (nz + 1);
        CHECK(p[0] == prev_end, "tile %d starts at %d, previous ended at %d", t, p[0], prev_end);
        for (int k = 0; k < nz; ++k) {
            CHECK(p[k] <= p[k + 1], "tile %d level %d: pointers decrease", t, k);
            for (int q = p[k]; q < p[k + 1] && !g_fail; ++q) {
                const RecEnt& e = ent[q];
                CHECK(e.r >= 0 && e.r < n, "receiver number %d", e.r);
                if (e.r < 0 || e.r >= n) return;
                ++seen[e.r];
                const int rk = kji[3 * e.r], rj = kji[3 * e.r + 1], ri = kji[3 * e.r + 2];
                CHECK(rk == k && e.k == k, "receiver %d at level %d listed at %d", e.r, rk, k);
                CHECK((rj / by) * tx + ri / bx == t, "receiver %d in tile %d", e.r, t);
                CHECK(e.local == (rj % by) * bx + ri % bx, "receiver %d local cell %d", e.r, e.local);
                if (q > p[k]) {
                    const RecEnt& d = ent[q - 1];
                    CHECK(d.local < e.local || (d.local == e.local && d.r < e.r),
                          "tile %d level %d: order of receivers %d, %d", t, k, d.r, e.r);
                }
            }
        }
        prev_end = p[nz];
    }
    CHECK(prev_end == n, "last tile ends at %d of %d", prev_end, n);
    for (int r = 0; r < n && !g_fail; ++r) CHECK(seen[r] == 1, "receiver %d listed %d times", r, seen[r]);
}

static void test_buckets()
{
    std::mt19937 rng(7);
    const int shapes[][3] = {{40, 36, 70}, {256, 256, 256}, {9, 1, 130}, {1, 8, 64}, {70, 17, 65}, {16, 300, 5}};
    for (const auto& sh : shapes) {
        const int nz = sh[0], ny = sh[1], nx = sh[2];
        for (int by : {8, 1}) {
            if (by == 1 && ny > 1) continue;
            for (int n : {0, 1, 37, 2000}) {
                std::vector<int> kji;
                for (int q = 0; q < n; ++q) {
                    // every third receiver shares a cell with an earlier one; others
                    // favour the box's faces and tile edges
                    if (q % 3 == 2) {
                        const int o = (int)(rng() % (unsigned)(q));
                        kji.insert(kji.end(), {kji[3 * o], kji[3 * o + 1], kji[3 * o + 2]});
                        continue;
                    }
                    auto pick = [&](int m, int b) {
                        const unsigned u = rng() % 4;
                        if (u == 0) return 0;
                        if (u == 1) return m - 1;
                        if (u == 2) return std::min(m - 1, (int)(rng() % (unsigned)((m + b - 1) / b)) * b + b - 1);
                        return (int)(rng() % (unsigned)m);
                    };
                    kji.insert(kji.end(), {pick(nz, 8), pick(ny, by), pick(nx, 64)});
                }
                check_buckets(nz, ny, nx, 64, by, kji);
                if (g_fail) return;
            }
        }
    }
    bool threw = false;
    try {
        std::vector<int> ptr;
        std::vector<RecEnt> ent;
        bucket_receivers(8, 64, 8, 1, 1, {0, 8, 0}, ptr, ent);  // j = 8 is past the one tile row
    } catch (const Error& e) {
        threw = e.code == WV_EINVAL;
    }
    CHECK(threw, "bucket_receivers accepted a receiver outside the box");
}

int main()
{
    test_revolve();
    if (!g_fail) test_chunks();
    if (!g_fail) test_buckets();
    if (g_fail) return 1;
    std::printf("host planning: ok\n");
    return 0;
}
