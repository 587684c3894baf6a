// Order of the block odd-even merge-split work of one call, shared by the
// planning kernel, the merge kernel and a host-side checker.
//
// A sub-array of p sorted tiles needs p merge-split phases (Baudet and
// Stevenson, 1978): in phase s the tile pairs (t, t+1) with t = s mod 2,
// s mod 2 + 2, ..., t + 1 < p are merged.  Every (sub-array, phase, pair) is
// one work item.  A single launch runs all items of all sub-arrays; its
// workgroups take items one at a time from a counter, in one global order
// that is phase-major: all phase-0 items of every sub-array, then all phase-1
// items, and so on.  Inside a phase the sub-arrays come in order of
// decreasing tile count (so the ones still active in a phase are a prefix),
// then by pair.
//
// An item may start once the items of earlier phases that last touched its
// two tiles are done.  Those items come earlier in the order, so they were
// taken earlier by workgroups that are already running; by induction on the
// order every taken item completes, whatever the grid size and however
// workgroups are scheduled.
//
// Tables, built per call on the device (the sub-arrays in order of
// decreasing tile count p_0 >= p_1 >= ... >= p_{H-1}):
//   active[s]  number of sub-arrays with p_i > s (s = 0 .. P-1, P = p_0)
//   pe[i]      sum over i' < i of floor(p_i' / 2)         (pairs in an even phase)
//   po[i]      sum over i' < i of floor((p_i' - 1) / 2)   (pairs in an odd phase)
//   ps[s]      items of phases before s; ps[P] is the item count
// The items of phase s are those of sub-arrays 0 .. active[s]-1; sub-array i
// contributes floor((p_i - s%2) / 2) pairs, so the prefix over sub-arrays is
// pe (even s) or po (odd s).
#pragma once

#include <stdint.h>

#ifndef __HIPCC__
#define BSORT_HD
#else
#define BSORT_HD __host__ __device__
#endif

namespace bsort {

// pairs of a sub-array of p tiles in phase s (0 once s >= p)
BSORT_HD inline int64_t msched_pairs(int64_t p, int64_t s) {
    return s < p ? (p - (s & 1)) / 2 : 0;
}

// largest i in [0, n] with a[i] <= x, for non-decreasing a with a[0] <= x
template <class A>
BSORT_HD inline int64_t msched_last_le(const A& a, int64_t n, int64_t x) {
    int64_t lo = 0, hi = n + 1;       // a[lo] <= x; answer in [lo, hi)
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

struct MschedItem {
    int32_t s;       // phase
    int32_t i;       // sub-array, in order of decreasing tile count
    int32_t t;       // lower tile of the pair
};

// The item at position q < ps[P] of the order.
template <class PS, class ACT, class PE, class PO>
BSORT_HD inline MschedItem msched_decode(int64_t q, const PS& ps, int32_t P, const ACT& active,
                                         const PE& pe, const PO& po) {
    MschedItem it;
    const int64_t s = msched_last_le(ps, P, q);          // ps[s] <= q < ps[s+1]
    const int64_t r = q - ps[s];
    const int64_t na = active[s];
    // the sub-array whose run of pairs holds r: largest i < na with prefix[i] <= r
    const int64_t i = (s & 1) ? msched_last_le(po, na - 1, r) : msched_last_le(pe, na - 1, r);
    const int64_t k = r - ((s & 1) ? po[i] : pe[i]);
    it.s = (int32_t)s;
    it.i = (int32_t)i;
    it.t = (int32_t)(2 * k + (s & 1));
    return it;
}

// Whether tile t of a sub-array of p tiles is merged in phase s.
BSORT_HD inline bool msched_paired(int64_t s, int64_t t, int64_t p) {
    const int64_t par = s & 1;
    if (s < 0 || t < par || t >= p) return false;
    return ((t - par) & 1) ? true : t + 1 < p;
}

// The phase before s that last merged tile t (-1: none).  A tile left out of
// phase s-1 (the first tile in odd phases, the last one at the other end)
// was merged in phase s-2.
BSORT_HD inline int64_t msched_prev(int64_t s, int64_t t, int64_t p) {
    if (s >= 1 && msched_paired(s - 1, t, p)) return s - 1;
    return s >= 2 ? s - 2 : -1;
}

}  // namespace bsort
