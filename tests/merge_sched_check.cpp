// Host check of the merge-split work order (paper_1407_6603_amd/csrc/merge_sched.h),
// built with g++ by tests/test_merge_schedule.py.  For random sets of
// sub-arrays it builds the order's tables the way the planning kernel does
// and checks that:
//   1. decoding positions 0..N-1 gives every (phase, sub-array, pair) item
//      exactly once;
//   2. msched_prev names the phase that last merged a tile (brute force);
//   3. every item's predecessors come earlier in the order, so a workgroup
//      only ever waits for items taken before its own;
//   4. an event simulation with W workers taking items in order and waiting
//      on tile counters runs every item to completion (no deadlock), and the
//      merge-splits applied in completion order sort random data.
// Prints "ok" and exits 0, or prints the first failure and exits 1.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <tuple>
#include <vector>

#include "../paper_1407_6603_amd/csrc/merge_sched.h"

using namespace bsort;

static int fails = 0;
#define CHECK(c, ...)                          \
    do {                                       \
        if (!(c)) {                            \
            if (fails++ < 5) {                 \
                printf("FAIL %s: ", #c);       \
                printf(__VA_ARGS__);           \
                printf("\n");                  \
            }                                  \
        }                                      \
    } while (0)

struct Tables {
    std::vector<int> p;          // tile counts, in decreasing order
    std::vector<int32_t> active;
    std::vector<int64_t> pe, po, ps;
    int P = 0;
    int64_t N = 0;
};

// the planning kernel's steps: counts per tile count, active[] as running
// sums from the top, a scatter into decreasing order, pe/po, ps
static Tables plan(const std::vector<int>& planned) {
    Tables T;
    const int64_t H = (int64_t)planned.size();
    for (int p : planned) T.P = std::max(T.P, p);
    const int P = T.P;
    std::vector<int32_t> cnt(P + 2, 0), fill(P + 2, 0);
    for (int p : planned) cnt[p]++;
    T.active.assign(P + 2, 0);
    int64_t run = 0;
    for (int64_t j = 0; j <= P; ++j) {
        T.active[P - j] = (int32_t)run;
        run += cnt[P - j];
    }
    T.p.assign(H, 0);
    for (int p : planned) T.p[T.active[p] + fill[p]++] = p;
    T.pe.assign(H + 1, 0);
    T.po.assign(H + 1, 0);
    for (int64_t i = 0; i < H; ++i) {
        T.pe[i + 1] = T.pe[i] + T.p[i] / 2;
        T.po[i + 1] = T.po[i] + (T.p[i] - 1) / 2;
    }
    T.ps.assign(P + 1, 0);
    for (int s = 0; s < P; ++s)
        T.ps[s + 1] = T.ps[s] + ((s & 1) ? T.po[T.active[s]] : T.pe[T.active[s]]);
    T.N = T.ps[P];
    return T;
}

static void check_set(const std::vector<int>& planned, std::mt19937_64& rng) {
    const Tables T = plan(planned);
    const int64_t H = (int64_t)T.p.size();
    for (int64_t i = 1; i < H; ++i) CHECK(T.p[i - 1] >= T.p[i], "order at %lld", (long long)i);
    // all items
    std::map<std::tuple<int, int, int>, int64_t> pos;
    int64_t expect = 0;
    for (int64_t i = 0; i < H; ++i) expect += ((T.p[i] + 1) / 2) * (T.p[i] / 2) +
                                             (T.p[i] / 2) * ((T.p[i] - 1) / 2);
    CHECK(T.N == expect, "N %lld expected %lld", (long long)T.N, (long long)expect);
    for (int64_t q = 0; q < T.N; ++q) {
        const MschedItem it = msched_decode(q, T.ps, T.P, T.active, T.pe, T.po);
        CHECK(it.i >= 0 && it.i < H, "sub-array %d", it.i);
        if (it.i < 0 || it.i >= H) continue;
        const int p = T.p[it.i];
        CHECK(it.s >= 0 && it.s < p, "phase %d of %d", it.s, p);
        CHECK((it.t - it.s) % 2 == 0 && it.t >= 0 && it.t + 1 < p, "pair %d phase %d p %d", it.t,
              it.s, p);
        CHECK(pos.count({it.s, it.i, it.t}) == 0, "item taken twice");
        pos[{it.s, it.i, it.t}] = q;
        if (q > 0) {
            const MschedItem pr = msched_decode(q - 1, T.ps, T.P, T.active, T.pe, T.po);
            CHECK(pr.s <= it.s, "not phase-major at %lld", (long long)q);
        }
    }
    CHECK((int64_t)pos.size() == T.N, "items %zu of %lld", pos.size(), (long long)T.N);
    // prev against brute force, and predecessors earlier in the order
    for (int64_t i = 0; i < H; ++i) {
        const int p = T.p[i];
        std::vector<int> last(p, -1);
        for (int s = 0; s < p; ++s) {
            for (int t = 0; t < p; ++t)
                CHECK(msched_prev(s, t, p) == last[t], "prev s %d t %d p %d: %lld vs %d", s, t, p,
                      (long long)msched_prev(s, t, p), last[t]);
            for (int t = s & 1; t + 1 < p; t += 2) {
                const int64_t q = pos[{s, (int)i, t}];
                for (int u : {t, t + 1}) {
                    const int sp = last[u];
                    if (sp < 0) continue;
                    const int lower = ((u - (sp & 1)) & 1) ? u - 1 : u;
                    auto f = pos.find({sp, (int)i, lower});
                    CHECK(f != pos.end() && f->second < q, "predecessor of (%d,%lld,%d)", s,
                          (long long)i, t);
                }
            }
            for (int t = s & 1; t + 1 < p; t += 2) last[t] = last[t + 1] = s;
        }
    }
    // event simulation with real data
    std::vector<std::vector<std::vector<int>>> tiles(H);
    std::vector<int> Tsz(H);
    for (int64_t i = 0; i < H; ++i) {
        Tsz[i] = 1 + (int)(rng() % 4);
        const int p = T.p[i];
        tiles[i].assign(p, {});
        for (int t = 0; t < p; ++t) {
            const int n = (t + 1 < p) ? Tsz[i] : 1 + (int)(rng() % Tsz[i]);
            for (int k = 0; k < n; ++k) tiles[i][t].push_back((int)(rng() % 7));
            std::sort(tiles[i][t].begin(), tiles[i][t].end());
        }
    }
    std::vector<std::vector<int>> ph(H);
    for (int64_t i = 0; i < H; ++i) ph[i].assign(T.p[i], 0);
    const int W = 1 + (int)(rng() % 8);
    struct Worker {
        int64_t q = -1;
        bool running = false;
        int64_t left = 0;
        MschedItem it{};
    };
    std::vector<Worker> w(W);
    int64_t head = 0, done = 0;
    int64_t steps = 0;
    while (done < T.N) {
        if (++steps > 100000000) {
            CHECK(false, "simulation did not finish (deadlock)");
            return;
        }
        const int k = (int)(rng() % W);
        Worker& x = w[k];
        if (x.q < 0) {
            if (head < T.N) {
                x.q = head++;
                x.it = msched_decode(x.q, T.ps, T.P, T.active, T.pe, T.po);
                x.running = false;
            }
            continue;
        }
        const int i = x.it.i, s = x.it.s, t = x.it.t, p = T.p[i];
        if (!x.running) {
            const bool ok = ph[i][t] >= msched_prev(s, t, p) + 1 &&
                            ph[i][t + 1] >= msched_prev(s, t + 1, p) + 1;
            if (ok) {
                x.running = true;
                x.left = (int64_t)(rng() % 3);
            }
            continue;
        }
        if (x.left-- > 0) continue;
        // merge-split of tiles t and t+1: the lower keeps the smaller half
        std::vector<int> m(tiles[i][t]);
        m.insert(m.end(), tiles[i][t + 1].begin(), tiles[i][t + 1].end());
        std::stable_sort(m.begin(), m.end());
        const size_t na = tiles[i][t].size();
        tiles[i][t].assign(m.begin(), m.begin() + na);
        tiles[i][t + 1].assign(m.begin() + na, m.end());
        CHECK(ph[i][t] == msched_prev(s, t, p) + 1 && ph[i][t + 1] == msched_prev(s, t + 1, p) + 1,
              "tile counters out of step");
        ph[i][t] = ph[i][t + 1] = s + 1;
        ++done;
        x.q = -1;
    }
    for (int64_t i = 0; i < H; ++i) {
        std::vector<int> all;
        for (auto& v : tiles[i]) all.insert(all.end(), v.begin(), v.end());
        CHECK(std::is_sorted(all.begin(), all.end()), "sub-array %lld not sorted", (long long)i);
    }
}

int main() {
    std::mt19937_64 rng(20240601);
    std::vector<std::vector<int>> sets = {{2}, {3}, {2, 2, 2}, {5, 4, 3, 2}, {40}, {2, 40, 3, 3, 17}};
    for (int r = 0; r < 300; ++r) {
        const int H = 1 + (int)(rng() % 24);
        std::vector<int> v;
        for (int k = 0; k < H; ++k) v.push_back(2 + (int)(rng() % (r % 3 == 0 ? 3 : 30)));
        sets.push_back(v);
    }
    for (auto& v : sets) {
        check_set(v, rng);
        if (fails) break;
    }
    if (fails) return 1;
    printf("ok %zu sets\n", sets.size());
    return 0;
}
