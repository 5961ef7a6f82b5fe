// scan_core.hpp -- device building blocks of the scan kernels (private to
// libpmscan): bit-plane slots, bit-sliced counters, exact window counts and
// the per-tile filter.  32 windows travel in one 32-bit word: bit b of a word
// of lane word i is window 32*(B+i) + b.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace pm {

// Where a tile reads from: the encoded text, the pattern image, and the
// windows the call may report, [win_begin, win_end).
struct TileSrc {
    const uint4* text4;
    const uint4* image;
    uint64_t win_begin, win_end;
};

// Mismatch word of 32 windows for one pattern position, from the text's high
// (H) and low (L) code-bit planes at that position: the OR of the minterms of
// the text codes in the position's Table 3 row MM.
template <unsigned MM>
__device__ __forceinline__ uint32_t mismatch_fn(uint32_t H, uint32_t L) {
    uint32_t x = 0;
    if (MM & 1u) x |= ~H & ~L;  // A = 00
    if (MM & 2u) x |= ~H & L;   // C = 01
    if (MM & 4u) x |= H & ~L;   // G = 10
    if (MM & 8u) x |= H & L;    // T = 11
    return x;
}

__device__ __forceinline__ uint32_t align(uint32_t hi, uint32_t lo, uint32_t r) {
    return __builtin_amdgcn_alignbit(hi, lo, r);
}

template <int R>
struct Lane {
    uint32_t h[R + 2], l[R + 2];  // raw planes of blocks B+fw .. B+fw+R+1
    uint32_t P[4][R + 2];          // P[c]: mismatch plane of singleton base c
};

// Singleton-filter slot (c | q << 2 | r << 3): mismatch words of the 32*R
// windows of the lane for the position 32*q + r of the filter window whose
// class is the single base c.  The dispatch over (c, q) is uniform.
template <int C, int Q, int R>
__device__ __forceinline__ void single_words(const Lane<R>& s, uint32_t r, uint32_t (&X)[R]) {
#pragma unroll
    for (int i = 0; i < R; ++i) X[i] = align(s.P[C][i + Q + 1], s.P[C][i + Q], r);
}

// Singleton-filter set (c | q << 2 | 4 << 3 | r_u << (6 + 5u)): the
// mismatch words of 4 positions of the same base c and word q, shifts r_u.
// One uniform dispatch per set.
template <int C, int Q, int R>
__device__ __forceinline__ void set_words_cq(const Lane<R>& s, uint32_t w, uint32_t (&X)[4][R]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) single_words<C, Q, R>(s, (w >> (6 + 5 * u)) & 31u, X[u]);
}

template <int R>
__device__ __forceinline__ void single_set(uint32_t w, const Lane<R>& s, uint32_t (&X)[4][R]) {
    switch (w & 7u) {
        case 0: set_words_cq<0, 0, R>(s, w, X); break;
        case 1: set_words_cq<1, 0, R>(s, w, X); break;
        case 2: set_words_cq<2, 0, R>(s, w, X); break;
        case 3: set_words_cq<3, 0, R>(s, w, X); break;
        case 4: set_words_cq<0, 1, R>(s, w, X); break;
        case 5: set_words_cq<1, 1, R>(s, w, X); break;
        case 6: set_words_cq<2, 1, R>(s, w, X); break;
        default: set_words_cq<3, 1, R>(s, w, X); break;
    }
}

// One singleton position (class cq = c | q << 2, shift r): for the tail sets.
template <int R>
__device__ __forceinline__ void single_slot(uint32_t cq, uint32_t r, const Lane<R>& s, uint32_t (&X)[R]) {
    switch (cq & 7u) {
        case 0: single_words<0, 0, R>(s, r, X); break;
        case 1: single_words<1, 0, R>(s, r, X); break;
        case 2: single_words<2, 0, R>(s, r, X); break;
        case 3: single_words<3, 0, R>(s, r, X); break;
        case 4: single_words<0, 1, R>(s, r, X); break;
        case 5: single_words<1, 1, R>(s, r, X); break;
        case 6: single_words<2, 1, R>(s, r, X); break;
        default: single_words<3, 1, R>(s, r, X); break;
    }
}

// Exhaustive-filter slot (mm | q << 4 | r << 5): any class, its Table 3 row
// mm applied to the shifted planes without branching on it.
template <int Q, int R>
__device__ __forceinline__ void general_words(const Lane<R>& s, uint32_t r, uint32_t mA, uint32_t mC,
                                              uint32_t mG, uint32_t mT, uint32_t (&X)[R]) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint32_t H = align(s.h[i + Q + 1], s.h[i + Q], r);
        const uint32_t L = align(s.l[i + Q + 1], s.l[i + Q], r);
        X[i] = (H & ((L & mT) | (~L & mG))) | (~H & ((L & mC) | (~L & mA)));
    }
}

template <int R>
__device__ __forceinline__ void general_slot(uint32_t slot, const Lane<R>& s, uint32_t (&X)[R]) {
    const uint32_t r = slot >> 5;
    const uint32_t mA = 0u - (slot & 1u), mC = 0u - (slot >> 1 & 1u);
    const uint32_t mG = 0u - (slot >> 2 & 1u), mT = 0u - (slot >> 3 & 1u);
    if (slot & 16u) general_words<1, R>(s, r, mA, mC, mG, mT, X);
    else general_words<0, R>(s, r, mA, mC, mG, mT, X);
}

// Full-adder halves as single three-input LUT operations (v_bitop3_b32);
// both functions are symmetric in their inputs.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}
__device__ __forceinline__ uint32_t or3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xFE);
}

// Bit-sliced counters: S[l][i] is bit l of the counts of the 32 windows of
// lane word i, started at `init` = 2^L - (keff+1), so a window whose count
// reaches keff+1 carries out of the top level; carries out of level L set
// its `dead` bit.
template <int R, int L>
struct Counters {
    uint32_t S[L > 0 ? L : 1][R];
    uint32_t dead[R];
};

// Add two carry words (weight 2^LV) to the counters.  Returns the carry into
// level LV+1 in `out`.
template <int LV, int R, int L>
__device__ __forceinline__ void add2(Counters<R, L>& c, const uint32_t (&a)[R], const uint32_t (&b)[R],
                                     uint32_t (&out)[R]) {
    if constexpr (LV == L) {
#pragma unroll
        for (int i = 0; i < R; ++i) c.dead[i] = or3(c.dead[i], a[i], b[i]);
    } else if constexpr (LV < L) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const uint32_t s = c.S[LV][i];
            c.S[LV][i] = xor3(s, a[i], b[i]);
            out[i] = maj3(s, a[i], b[i]);
        }
    }
}

template <int LV, int R, int L>
__device__ __forceinline__ void add1(Counters<R, L>& c, uint32_t (&a)[R]) {
    if constexpr (LV == L) {
#pragma unroll
        for (int i = 0; i < R; ++i) c.dead[i] |= a[i];
    } else if constexpr (LV < L) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const uint32_t s = c.S[LV][i];
            c.S[LV][i] = s ^ a[i];
            a[i] = s & a[i];
        }
        add1<LV + 1, R, L>(c, a);
    }
}

// Exact count of one window, all m positions (pattern image), stopping once
// the count exceeds `limit` (then the value returned is only known to exceed
// it).  Chunks of 32 positions are taken V at a time, their loads issued
// together, so a long pattern's count waits on 1/V of the load round trips
// (fewer at a time hold fewer registers).
template <uint32_t V = 4>
__device__ uint32_t count_window(const uint4* __restrict__ text4, const uint4* __restrict__ image,
                                 uint32_t nchunks, uint64_t s, uint32_t limit) {
    const uint2* text = reinterpret_cast<const uint2*>(text4);
    const uint64_t q = s >> 5;
    const uint32_t r = (uint32_t)s & 31u;
    uint2 w0 = text[q];
    uint32_t cnt = 0;
    for (uint32_t c0 = 0; c0 < nchunks; c0 += V) {
        uint2 w[V];
        uint4 mp[V];
#pragma unroll
        for (uint32_t j = 0; j < V; ++j) {
            if (c0 + j < nchunks) {
                w[j] = text[q + c0 + j + 1];
                mp[j] = image[c0 + j];
            } else {
                w[j] = w0;
                mp[j] = make_uint4(0u, 0u, 0u, 0u);
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < V; ++j) {
            const uint32_t H = align(w[j].x, w0.x, r), Lo = align(w[j].y, w0.y, r);
            const uint32_t mis = (~H & ~Lo & mp[j].x) | (~H & Lo & mp[j].y) | (H & ~Lo & mp[j].z) | (H & Lo & mp[j].w);
            cnt += __builtin_popcount(mis);
            w0 = w[j];
        }
        if (cnt > limit) break;
    }
    return cnt;
}

// Exact count of window s by the whole wave (every lane active): lane l
// takes the chunks of 32 positions l, l + 64, ..., four per round with their
// loads issued together; the wave's sum is tested against `limit` after each
// round.  Returns the same value in every lane (exact when <= limit).
__device__ uint32_t count_window_wave(const uint4* __restrict__ text4, const uint4* __restrict__ image,
                                      uint32_t nchunks, uint64_t s, uint32_t limit, uint32_t lane) {
    const uint2* text = reinterpret_cast<const uint2*>(text4);
    const uint64_t q = s >> 5;
    const uint32_t r = (uint32_t)s & 31u;
    constexpr uint32_t V = 4;
    uint32_t total = 0;
    for (uint32_t c0 = 0; c0 < nchunks; c0 += 64 * V) {
        uint2 w0[V], w1[V];
        uint4 mp[V];
#pragma unroll
        for (uint32_t j = 0; j < V; ++j) {
            const uint32_t c = c0 + 64 * j + lane;
            if (c < nchunks) {
                w0[j] = text[q + c];
                w1[j] = text[q + c + 1];
                mp[j] = image[c];
            } else {
                w0[j] = make_uint2(0u, 0u);
                w1[j] = w0[j];
                mp[j] = make_uint4(0u, 0u, 0u, 0u);
            }
        }
        uint32_t part = 0;
#pragma unroll
        for (uint32_t j = 0; j < V; ++j) {
            const uint32_t H = align(w1[j].x, w0[j].x, r), Lo = align(w1[j].y, w0[j].y, r);
            const uint32_t mis = (~H & ~Lo & mp[j].x) | (~H & Lo & mp[j].y) | (H & ~Lo & mp[j].z) | (H & Lo & mp[j].w);
            part += __builtin_popcount(mis);
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) part += __shfl_xor(part, d, 64);
        total += part;
        if (total > limit) break;
    }
    return total;
}

// With WV, survivors of patterns longer than kWaveVerifyChunks chunks of 32
// positions are verified by the whole wave, one at a time, when at most
// kWaveVerifyLanes lanes have any (the usual case with a selective filter);
// otherwise each lane verifies its own survivors.
constexpr uint32_t kWaveVerifyChunks = 16;
constexpr int kWaveVerifyLanes = 4;
// Hits found by the whole wave that are kept for the output (so that they
// need not be counted again).
constexpr uint32_t kWaveHits = 8;

// The lane's text planes for blocks B+fw .. B+fw+R+1 (the 16-byte groups in
// t) and, for each base c with bit c of `singles` set, its mismatch plane:
// bit set where the text base is not c.
template <int R>
__device__ __forceinline__ void make_lane(const uint4 (&t)[(R + 2) / 2], uint32_t singles, Lane<R>& s) {
#pragma unroll
    for (int u = 0; u < (R + 2) / 2; ++u) {
        s.h[2 * u] = t[u].x;
        s.l[2 * u] = t[u].y;
        s.h[2 * u + 1] = t[u].z;
        s.l[2 * u + 1] = t[u].w;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (singles >> c & 1u) {
#pragma unroll
            for (int w = 0; w < R + 2; ++w) {
                const uint32_t hx = (c & 2) ? ~s.h[w] : s.h[w];
                const uint32_t lx = (c & 1) ? ~s.l[w] : s.l[w];
                s.P[c][w] = hx | lx;
            }
        }
    }
}

// Survivors of a singleton filter (windows whose bit in dead[] is clear) ->
// hits: each is counted exactly over all m positions and kept when the count
// is at most k.  hit[i] gets the hits of lane word i, nh the lane's number of
// hits.  With WV and a pattern of more than kWaveVerifyChunks chunks, a wave
// with survivors in at most kWaveVerifyLanes lanes counts them one at a time
// with all its lanes (position order), keeping the first kWaveHits hits as
// (position << 16 | count) in vh (count of all such hits in *nvh); dead[] is
// consumed.  Otherwise each lane counts its own survivors (count_window with
// CV chunks at a time).
template <int R, bool WV, uint32_t CV = 4, class Plan>
__device__ __forceinline__ void verify_survivors(const TileSrc& src, const Plan& p, uint64_t B, uint32_t (&dead)[R],
                                                 uint32_t (&hit)[R], uint32_t& nh, unsigned long long* vh = nullptr,
                                                 uint32_t* nvh = nullptr) {
    nh = 0;
    uint32_t any = 0;
#pragma unroll
    for (int i = 0; i < R; ++i) any |= ~dead[i];
    if (vh) *nvh = 0;
    if (__ballot(any != 0) == 0) {  // the usual case: no survivor in the wave
#pragma unroll
        for (int i = 0; i < R; ++i) hit[i] = 0;
        return;
    }
    if (WV && p.nchunks > kWaveVerifyChunks && __popcll(__ballot(any != 0)) <= kWaveVerifyLanes) {
        // survivors in position order (lowest lane first, then its words
        // and bits), each counted by the whole wave; a verified survivor
        // is marked dead, a hit set in hit[]
        const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
        for (int i = 0; i < R; ++i) hit[i] = 0;
        for (;;) {
            uint32_t mine = 0;
#pragma unroll
            for (int i = 0; i < R; ++i) mine |= ~dead[i];
            const uint64_t bal = __ballot(mine != 0);
            if (bal == 0) break;
            const uint32_t owner = (uint32_t)__builtin_ctzll(bal);
            int fi = 0;
            uint32_t fb = 0;
#pragma unroll
            for (int i = R - 1; i >= 0; --i)
                if (~dead[i]) {
                    fi = i;
                    fb = __builtin_ctz(~dead[i]);
                }
            const uint64_t mine_pos = 32 * (B + (uint64_t)fi) + fb;
            const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)mine_pos, owner);
            const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(mine_pos >> 32), owner);
            const uint64_t pos = ((uint64_t)hi << 32) | lo;
            const uint32_t c = count_window_wave(src.text4, src.image, p.nchunks, pos, p.k, lane);
            if (lane == owner) {
#pragma unroll
                for (int i = 0; i < R; ++i)
                    if (i == fi) {
                        dead[i] |= 1u << fb;
                        if (c <= p.k) hit[i] |= 1u << fb;
                    }
            }
            // hits come in position order: the first kWaveHits are kept
            // (position << 16 | count) for the caller's output
            if (vh && c <= p.k) {
                if (*nvh < kWaveHits && lane == owner) vh[*nvh] = (pos << 16) | c;
                ++*nvh;
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i) nh += __builtin_popcount(hit[i]);
        return;
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
        uint32_t alive = ~dead[i];
        uint32_t h = 0;
        while (alive) {
            const uint32_t b = __builtin_ctz(alive);
            alive &= alive - 1u;
            const uint32_t c = count_window<CV>(src.text4, src.image, p.nchunks, 32 * (B + i) + b, p.k);
            if (c <= p.k) h |= 1u << b;
        }
        hit[i] = h;
        nh += __builtin_popcount(h);
    }
}

// Counters at the plan's start value; windows outside [win_begin, win_end)
// start dead.
template <int R, int L, class Plan>
__device__ __forceinline__ void init_counters(const TileSrc& src, const Plan& p, uint64_t B, bool interior,
                                              Counters<R, L>& C) {
    // (windows outside [win_begin, win_end) start dead; `interior` says the
    // whole tile lies inside, which holds for all tiles but the edge ones)
#pragma unroll
    for (int i = 0; i < R; ++i) {
        uint32_t valid = ~0u;
        if (!interior) {
            const uint64_t w0 = 32 * (B + i);
            valid = 0;
            if (w0 < src.win_end && w0 + 32 > src.win_begin) {
                const uint32_t lo = src.win_begin > w0 ? (uint32_t)(src.win_begin - w0) : 0u;
                const uint32_t hi = src.win_end < w0 + 32 ? (uint32_t)(src.win_end - w0) : 32u;
                valid = (hi == 32u ? ~0u : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
            }
        }
        C.dead[i] = ~valid;
        if constexpr (L > 0) {
#pragma unroll
            for (int l = 0; l < L; ++l) C.S[l][i] = (p.init >> l & 1u) ? ~0u : 0u;
        }
    }
}

// Filter + verification of one tile for one pattern: hit[i] gets the windows
// of lane word i (window 32*(B+i) + bit) with at most k mismatches; C keeps the
// filter counters (the exact counts when the plan is exhaustive).  `s` holds
// the lane's text planes starting at the plan's filter window.
template <int R, int L, bool EXH, bool WV, class Plan>
__device__ __forceinline__ void tile_filter(const TileSrc& src, const Plan& p, uint64_t B, bool interior,
                                            const Lane<R>& s, Counters<R, L>& C, uint32_t (&hit)[R],
                                            uint32_t& nh, unsigned long long* vh = nullptr,
                                            uint32_t* nvh = nullptr) {
    init_counters<R, L>(src, p, B, interior, C);

    // ---- filter ---------------------------------------------------------------
    // groups of 8 slots into the counters: a full-adder tree per group (pairs
    // into level 0, their carries pairwise into level 1, ...)
    if constexpr (EXH) {
        for (uint32_t g = 0; g < p.n_slots; g += 8) {
            const uint32_t gv[4] = {p.slot[g / 2], p.slot[g / 2 + 1], p.slot[g / 2 + 2], p.slot[g / 2 + 3]};
            uint32_t xa[R], xb[R], c0a[R], c0b[R], c1a[R], c1b[R], c2[R];
#pragma unroll
            for (int half = 0; half < 2; ++half) {
#pragma unroll
                for (int pr = 0; pr < 2; ++pr) {
                    const uint32_t w = gv[2 * half + pr];  // slots u and u+1
                    general_slot<R>(w & 0xFFFFu, s, xa);
                    general_slot<R>(w >> 16, s, xb);
                    add2<0, R, L>(C, xa, xb, pr == 0 ? c0a : c0b);
                }
                add2<1, R, L>(C, c0a, c0b, half == 0 ? c1a : c1b);
            }
            add2<2, R, L>(C, c1a, c1b, c2);
            if constexpr (L >= 3) add1<3, R, L>(C, c2);
        }
    } else {
        // groups: two full sets each
        for (uint32_t g = 0; g < p.n_groups; ++g) {
            const uint32_t w0 = p.slot[2 * g], w1 = p.slot[2 * g + 1];
            uint32_t X[4][R], c0a[R], c0b[R], c1a[R], c1b[R], c2[R];
            single_set<R>(w0, s, X);
            add2<0, R, L>(C, X[0], X[1], c0a);
            add2<0, R, L>(C, X[2], X[3], c0b);
            add2<1, R, L>(C, c0a, c0b, c1a);
            single_set<R>(w1, s, X);
            add2<0, R, L>(C, X[0], X[1], c0a);
            add2<0, R, L>(C, X[2], X[3], c0b);
            add2<1, R, L>(C, c0a, c0b, c1b);
            add2<2, R, L>(C, c1a, c1b, c2);
            if constexpr (L >= 3) add1<3, R, L>(C, c2);
        }
        // tail: the remaining sets, one position at a time
        for (uint32_t t = 2 * p.n_groups; t < p.n_sets; ++t) {
            const uint32_t w = p.slot[t];
            const uint32_t cnt = (w >> 3) & 7u;
            for (uint32_t u = 0; u < cnt; ++u) {
                uint32_t X[R];
                single_slot<R>(w, (w >> (6 + 5 * u)) & 31u, s, X);
                add1<0, R, L>(C, X);
            }
        }
    }

    // ---- survivors -> hits -----------------------------------------------------
    nh = 0;
    if constexpr (EXH) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            hit[i] = ~C.dead[i];
            nh += __builtin_popcount(hit[i]);
        }
    } else {
        verify_survivors<R, WV>(src, p, B, C.dead, hit, nh, vh, nvh);
    }
}

// Singleton filter with a structure fixed at compile time: NG groups of two
// full sets (8 positions each, slot words sw[0 .. 2 NG) of the plan, uniform),
// counters started at the plan's init (uniform: every level all ones or all
// zeros), no window excluded.  dead[i] gets the windows of lane word i whose
// count over the 8 NG positions reaches keff + 1.
//
// The mismatch planes of the bases the plan uses go to this wave's region of
// LDS (`planes`: [base][word][lane], 4 x (R+2) x 64 words) instead of
// registers, so that a set reads the R+1 words of its base and word offset at
// a uniform address: no branch on the set's base, and no planes held in
// registers across the filter.  The loops are unrolled, so that the first
// group reads the uniform start values directly and the last group's counter
// sums, which nothing reads, are not computed.
template <int R>
__device__ __forceinline__ void store_planes(const uint4 (&t)[(R + 2) / 2], uint32_t singles, uint32_t* planes) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t h[R + 2], l[R + 2];
#pragma unroll
    for (int u = 0; u < (R + 2) / 2; ++u) {
        h[2 * u] = t[u].x;
        l[2 * u] = t[u].y;
        h[2 * u + 1] = t[u].z;
        l[2 * u + 1] = t[u].w;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (singles >> c & 1u) {
#pragma unroll
            for (int w = 0; w < R + 2; ++w) {
                const uint32_t hx = (c & 2) ? ~h[w] : h[w];
                const uint32_t lx = (c & 1) ? ~l[w] : l[w];
                planes[(c * (R + 2) + w) * 64 + lane] = hx | lx;
            }
        }
    }
}

// The lane's row of a set's plane words in the LDS planes: base c and word
// offset q of the set word w (RS words per base).
template <int RS>
__device__ __forceinline__ const uint32_t* set_row(const uint32_t* planes, uint32_t w) {
    const uint32_t lane = threadIdx.x & 63u;
    return planes + ((w & 3u) * RS + ((w >> 2) & 1u)) * 64 + lane;
}

// The RW+1 plane words of a set from lane word i0 on ...
template <int RW>
__device__ __forceinline__ void lds_words(const uint32_t* row, int i0, uint32_t (&P)[RW + 1]) {
#pragma unroll
    for (int i = 0; i <= RW; ++i) P[i] = row[(i0 + i) * 64];
}

// ... and its four slots' mismatch words for those RW lane words (shift r_u).
template <int RW>
__device__ __forceinline__ void align_set(uint32_t w, const uint32_t (&P)[RW + 1], uint32_t (&X)[4][RW]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t r = (w >> (6 + 5 * u)) & 31u;
#pragma unroll
        for (int i = 0; i < RW; ++i) X[u][i] = align(P[i + 1], P[i], r);
    }
}

// The lane words are taken RW at a time (RW divides R): fewer counters and
// mismatch words are live at once, for one more plane word read per set and
// part.
template <int R, int L, int NG, int RW = R>
__device__ __forceinline__ void fixed_filter(const uint32_t* const (&rows)[2 * NG], const uint32_t (&sw)[2 * NG],
                                             uint32_t init, uint32_t (&dead)[R]) {
    static_assert(R % RW == 0, "the parts must cover the lane words");
#pragma unroll
    for (int part = 0; part < R / RW; ++part) {
        const int i0 = part * RW;
        Counters<RW, L> C;
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            C.dead[i] = 0;
            if constexpr (L > 0) {
#pragma unroll
                for (int l = 0; l < L; ++l) C.S[l][i] = 0u - (init >> l & 1u);
            }
        }
        // the next set's plane words are read before this set is counted (two
        // register sets in turn); the compiler issues all of a part's reads
        // ahead, so that the wave waits for LDS about once per part
        uint32_t P[2][RW + 1];
        lds_words<RW>(rows[0], i0, P[0]);
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            uint32_t X[4][RW], c0a[RW], c0b[RW], c1a[RW], c1b[RW], c2[RW];
            lds_words<RW>(rows[2 * g + 1], i0, P[1]);
            __builtin_amdgcn_sched_barrier(0);
            align_set<RW>(sw[2 * g], P[0], X);
            add2<0, RW, L>(C, X[0], X[1], c0a);
            add2<0, RW, L>(C, X[2], X[3], c0b);
            add2<1, RW, L>(C, c0a, c0b, c1a);
            if (g + 1 < NG) lds_words<RW>(rows[2 * g + 2], i0, P[0]);
            __builtin_amdgcn_sched_barrier(0);
            align_set<RW>(sw[2 * g + 1], P[1], X);
            add2<0, RW, L>(C, X[0], X[1], c0a);
            add2<0, RW, L>(C, X[2], X[3], c0b);
            add2<1, RW, L>(C, c0a, c0b, c1b);
            add2<2, RW, L>(C, c1a, c1b, c2);
            if constexpr (L >= 3) add1<3, RW, L>(C, c2);
        }
#pragma unroll
        for (int i = 0; i < RW; ++i) dead[i0 + i] = C.dead[i];
        // one part at a time: its registers are free before the next starts
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Singleton filter of any plan (run-time numbers of groups and of tail sets)
// over the mismatch planes in LDS (`planes`, laid out as for fixed_filter,
// every base present): the groups as in fixed_filter, then the tail sets one
// position at a time.
template <int R, int L, class Plan>
__device__ __forceinline__ void planes_filter(const uint32_t* planes, const Plan& p, Counters<R, L>& C) {
    for (uint32_t g = 0; g < p.n_groups; ++g) {
        const uint32_t w0 = p.slot[2 * g], w1 = p.slot[2 * g + 1];
        uint32_t P[R + 1], X[4][R], c0a[R], c0b[R], c1a[R], c1b[R], c2[R];
        lds_words<R>(set_row<R + 2>(planes, w0), 0, P);
        align_set<R>(w0, P, X);
        add2<0, R, L>(C, X[0], X[1], c0a);
        add2<0, R, L>(C, X[2], X[3], c0b);
        add2<1, R, L>(C, c0a, c0b, c1a);
        lds_words<R>(set_row<R + 2>(planes, w1), 0, P);
        align_set<R>(w1, P, X);
        add2<0, R, L>(C, X[0], X[1], c0a);
        add2<0, R, L>(C, X[2], X[3], c0b);
        add2<1, R, L>(C, c0a, c0b, c1b);
        add2<2, R, L>(C, c1a, c1b, c2);
        if constexpr (L >= 3) add1<3, R, L>(C, c2);
    }
    for (uint32_t t = 2 * p.n_groups; t < p.n_sets; ++t) {
        const uint32_t w = p.slot[t];
        const uint32_t cnt = (w >> 3) & 7u;
        uint32_t P[R + 1];
        lds_words<R>(set_row<R + 2>(planes, w), 0, P);
        for (uint32_t u = 0; u < cnt; ++u) {
            const uint32_t r = (w >> (6 + 5 * u)) & 31u;
            uint32_t X[R];
#pragma unroll
            for (int i = 0; i < R; ++i) X[i] = align(P[i + 1], P[i], r);
            add1<0, R, L>(C, X);
        }
    }
}

// Windows of lane word i (window 32*(B+i) + bit) inside [win_begin, win_end).
template <int R>
__device__ __forceinline__ void valid_windows(const TileSrc& src, uint64_t B, uint32_t (&valid)[R]) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint64_t w0 = 32 * (B + i);
        uint32_t v = 0;
        if (w0 < src.win_end && w0 + 32 > src.win_begin) {
            const uint32_t lo = src.win_begin > w0 ? (uint32_t)(src.win_begin - w0) : 0u;
            const uint32_t hi = src.win_end < w0 + 32 ? (uint32_t)(src.win_end - w0) : 32u;
            v = (hi == 32u ? ~0u : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
        }
        valid[i] = v;
    }
}

// Exact count of hit window `b` of lane word i.
template <int R, int L, bool EXH, class Plan>
__device__ __forceinline__ uint32_t hit_count(const TileSrc& src, const Plan& p, const Counters<R, L>& C,
                                              int i, uint32_t b, uint64_t pos) {
    if constexpr (EXH) {
        uint32_t v = 0;
        if constexpr (L > 0) {
#pragma unroll
            for (int l = 0; l < L; ++l) v |= (C.S[l][i] >> b & 1u) << l;
        }
        return v - p.init + p.n_dash;
    }
    return count_window(src.text4, src.image, p.nchunks, pos, p.k);
}

}  // namespace pm
