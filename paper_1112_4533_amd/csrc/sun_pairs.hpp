// sun_pairs.hpp -- the order in which the large-Nc update runs its SU(2)
// subgroup steps, several at a time (plain C++, evaluated at compile time).
//
// The Cabibbo-Marinari update (Sec. 4) left-multiplies the link by one
// SU(2) element per index pair (i, j), i < j, in the fixed order (0, 1),
// (0, 2), ..., (Nc - 2, Nc - 1); step (i, j) reads the 2x2 block (i, j) of
// W = U A and rewrites rows i and j of U and of W.  Two steps with no index
// in common therefore read and write disjoint entries and commute: any order
// that keeps, for every index k, the order of the steps touching k gives
// the same link bit for bit.  The table below is such an order in slots of
// at most W steps, listed greedily -- each slot takes the W earliest steps
// (in the fixed order) whose predecessors are all in earlier slots -- which
// takes about S / W slots plus a short start-up, S = Nc (Nc - 1) / 2 (two
// at a time, SU(32): 257 slots for 496 steps; four at a time: 139).
#pragma once

#include <cstdint>

namespace sun {
namespace pairs {

constexpr int kMaxN = 32;
constexpr int kNone = 0xFF;                       // no step in this place of the slot
constexpr uint32_t kNoStep = 0xFFFFu;             // (kNone, kNone)
constexpr int kMaxSteps = kMaxN * (kMaxN - 1) / 2;
constexpr int kMaxWords = 3328;                   // over Nc = 2 .. 32 (two steps: 2886, four: 3294)

// Slots of W steps each.  The slots of Nc are slots first[Nc] ..
// first[Nc + 1] - 1; slot t holds W steps i | j << 8 (kNoStep for an empty
// place), two to a 32-bit word: place m of slot t is half m mod 2 of word
// t W / 2 + m / 2.  The places of a slot follow the fixed order, empty
// places last.
template <int W>
struct Table {
    static_assert(W == 2 || W == 4, "two or four steps per slot");
    uint16_t first[kMaxN + 2];
    uint32_t word[kMaxWords];
};

// Number of step (i, j) in the fixed order: the Philox counter of its draws.
constexpr uint32_t step_index(int n, int i, int j) {
    return (uint32_t)(i * n - i * (i + 1) / 2 + (j - i - 1));
}

template <int W>
constexpr void schedule(int n, Table<W>& t, int& at) {
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
        int pick[W] = {}, np = 0;
        for (int s = lo; s < S && np < W; ++s)
            if (!done[s] && npred[s] == 0) pick[np++] = s;
        for (int e = 0; e < np; ++e) {
            const int s = pick[e];
            done[s] = true;
            ++ndone;
            for (int f = 0; f < 2; ++f)
                if (succ[s][f] >= 0) --npred[succ[s][f]];
        }
        while (lo < S && done[lo]) ++lo;
        for (int w = 0; w < W / 2; ++w) {
            uint32_t h[2] = {kNoStep, kNoStep};
            for (int m = 0; m < 2; ++m)
                if (2 * w + m < np) h[m] = (uint32_t)si[pick[2 * w + m]] | (uint32_t)sj[pick[2 * w + m]] << 8;
            t.word[at * (W / 2) + w] = h[0] | h[1] << 16;
        }
        ++at;
    }
}

template <int W>
constexpr Table<W> make_table() {
    Table<W> t{};
    int at = 0;
    for (int n = 0; n <= kMaxN; ++n) {
        t.first[n] = (uint16_t)at;
        if (n >= 2) schedule<W>(n, t, at);
    }
    t.first[kMaxN + 1] = (uint16_t)at;
    return t;
}

template <int W>
constexpr int slots(const Table<W>& t, int n) { return t.first[n + 1] - t.first[n]; }

}  // namespace pairs
}  // namespace sun
