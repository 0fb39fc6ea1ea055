// sun_pairs.hpp -- the order in which the large-Nc update runs its SU(2)
// subgroup steps, two at a time (plain C++, evaluated at compile time).
//
// The Cabibbo-Marinari update (Sec. 4) left-multiplies the link by one
// SU(2) element per index pair (i, j), i < j, in the fixed order (0, 1),
// (0, 2), ..., (Nc - 2, Nc - 1); step (i, j) reads the 2x2 block (i, j) of
// W = U A and rewrites rows i and j of U and of W.  Two steps with no index
// in common therefore read and write disjoint entries and commute: any order
// that keeps, for every index k, the order of the steps touching k gives
// the same link bit for bit.  The table below is such an order in slots of
// at most two steps, listed greedily -- each slot takes the two earliest
// steps (in the fixed order) whose predecessors are all in earlier slots --
// which takes ceil(S / 2) slots plus a short start-up, S = Nc (Nc - 1) / 2
// (SU(32): 257 slots for 496 steps; SU(8): 17 for 28).
#pragma once

#include <cstdint>

namespace sun {
namespace pairs {

constexpr int kMaxN = 32;
constexpr int kNone = 0xFF;                       // no second step in the slot
constexpr int kMaxSteps = kMaxN * (kMaxN - 1) / 2;
constexpr int kMaxSlotsTotal = 4096;              // over Nc = 2 .. 32 (2886 used)

// Slots of Nc: slot[first[Nc] .. first[Nc + 1]), each packed as
// iA | jA << 8 | iB << 16 | jB << 24, with iB = jB = kNone when the slot holds
// one step.  The first step of a slot precedes the second in the fixed order.
struct Table {
    uint16_t first[kMaxN + 2];
    uint32_t slot[kMaxSlotsTotal];
};

// Number of step (i, j) in the fixed order: the Philox counter of its draws.
constexpr uint32_t step_index(int n, int i, int j) {
    return (uint32_t)(i * n - i * (i + 1) / 2 + (j - i - 1));
}

constexpr void schedule(int n, Table& t, int& at) {
    int si[kMaxSteps] = {}, sj[kMaxSteps] = {};
    int npred[kMaxSteps] = {}, succ[kMaxSteps][2] = {};
    bool done[kMaxSteps] = {};
    int last[kMaxN] = {};
    for (int k = 0; k < kMaxN; ++k) last[k] = -1;
    int S = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j, ++S) {
            si[S] = i;
            sj[S] = j;
            succ[S][0] = succ[S][1] = -1;
            // the predecessor on each index: the last earlier step touching it
            const int idx[2] = {i, j};
            for (int e = 0; e < 2; ++e) {
                const int p = last[idx[e]];
                if (p >= 0) {
                    ++npred[S];
                    succ[p][succ[p][0] < 0 ? 0 : 1] = S;
                }
                last[idx[e]] = S;
            }
        }
    int lo = 0, ndone = 0;
    while (ndone < S) {
        int pick[2] = {-1, -1}, np = 0;
        for (int s = lo; s < S && np < 2; ++s)
            if (!done[s] && npred[s] == 0) pick[np++] = s;
        for (int e = 0; e < np; ++e) {
            const int s = pick[e];
            done[s] = true;
            ++ndone;
            for (int f = 0; f < 2; ++f)
                if (succ[s][f] >= 0) --npred[succ[s][f]];
        }
        while (lo < S && done[lo]) ++lo;
        const uint32_t a = (uint32_t)si[pick[0]] | (uint32_t)sj[pick[0]] << 8;
        const uint32_t b = np > 1 ? ((uint32_t)si[pick[1]] | (uint32_t)sj[pick[1]] << 8) : (kNone | kNone << 8);
        t.slot[at++] = a | b << 16;
    }
}

constexpr Table make_table() {
    Table t{};
    int at = 0;
    for (int n = 0; n <= kMaxN; ++n) {
        t.first[n] = (uint16_t)at;
        if (n >= 2) schedule(n, t, at);
    }
    t.first[kMaxN + 1] = (uint16_t)at;
    return t;
}

constexpr int slots(const Table& t, int n) { return t.first[n + 1] - t.first[n]; }

}  // namespace pairs
}  // namespace sun
