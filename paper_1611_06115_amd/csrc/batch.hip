// batch.hip -- many patterns in one persistent launch (libpmscan).
//
// Work item = (group of up to kMaxGroup patterns, text sub-range).  One wave
// takes an item from a queue, walks the tiles of its sub-range in text order,
// loads each tile's text and computes its planes once, and runs every pattern
// of the group on it (each with its own filter plan, counters and exact
// verification).  A pattern's hits of one sub-range are appended in order to
// its staging area for that sub-range; a gather kernel then concatenates the
// sub-ranges of each pattern, in text order, into the caller's output.
//
// Patterns in a group share one code path (same filter kind and counter
// depth); items are queued in decreasing order of estimated cost so that the
// expensive ones start first.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pmscan.h"
#include "batch.hpp"
#include "plan.hpp"
#include "scan_core.hpp"

namespace pm {
// shared with pmscan.hip
pm_status set_error(pm_status s, const std::string& what);
uint64_t encoded_text_groups(uint64_t n);
hipError_t mark_begin(hipStream_t s);
hipError_t mark_end(hipStream_t s);
uint64_t resident_blocks(const void* fn);
}  // namespace pm

using namespace pm;

namespace {

constexpr int TPB = kThreads;
constexpr int kMaxGroup = 16;
// chunks of 32 positions a survivor's exact count loads at a time: two keep
// the verification's registers below the filter's
constexpr uint32_t kVerifyChunks = 2;
// an exhaustive filter shares little per tile across patterns (only the raw
// planes), so its groups hold 1/kExhGroupDiv of the group size: shorter
// items, which do not hold a wave for long
constexpr uint32_t kExhGroupDiv = 8;
constexpr uint32_t kSkip = 0xFFu;  // variant of a pattern that cannot have hits

struct BatchPattern {
    ScanPlan plan;        // filter window at the pattern start
    uint64_t image_off;   // pattern image, in 16-byte units of the image pool
    uint64_t stage_off;   // staging area, in hits
    uint64_t nw;          // windows: n - m + 1 (0 when m > n)
    uint32_t cap_sub;     // staged hits per sub-range
    uint32_t variant;     // fixed groups << 4 | exhaustive << 3 | levels, or kSkip
    uint32_t index;       // the caller's index of the pattern
    uint32_t pad_[1];
};
static_assert(sizeof(BatchPattern) % 16 == 0, "BatchPattern must keep 16-byte alignment");

struct BatchItem {
    uint32_t first, count, sub, pad_;  // patterns [first, first+count) of the group, sub-range
};

// Pattern records and work items do not change during a launch and every
// read of them is wave-uniform: reading them through the constant address
// space lets those reads be scalar loads (scalar cache) instead of vector
// loads that wait on L2.
using CPattern = const BatchPattern __attribute__((address_space(4)));
using CItem = const BatchItem __attribute__((address_space(4)));

__device__ __forceinline__ CPattern& const_pattern(const BatchPattern* p) {
    return *reinterpret_cast<CPattern*>(reinterpret_cast<uintptr_t>(p));
}
__device__ __forceinline__ CItem& const_item(const BatchItem* p) {
    return *reinterpret_cast<CItem*>(reinterpret_cast<uintptr_t>(p));
}

struct GatherPattern {
    uint64_t stage_off, out_off, capacity;
    uint32_t cap_sub, pad_;
};

// One gather workgroup: share y of the nb shares of pattern p's output.
struct GatherWork {
    uint32_t p, y, nb, pad_;
};

struct BatchArgs {
    const uint4* text4;
    uint32_t n4_last;               // last 16-byte group of the text buffer
    uint32_t n_items;
    const uint4* images;
    const BatchPattern* pats;
    const BatchItem* items;
    unsigned long long* staged;     // (window << 16) | count
    uint32_t* counts;               // hits per (caller pattern, sub-range)
    uint32_t* queue;                // next item
    uint32_t n_sub;
    uint32_t pad_;
    uint64_t win_begin, win_end;    // windows the call reports
    uint64_t wb0;                   // first block of sub-range 0 (even)
    uint64_t span_blocks;           // blocks per sub-range (a multiple of the tile)
};

__device__ __forceinline__ uint32_t wave_exclusive(uint32_t x, uint32_t& total) {
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t v = __shfl_up(incl, d, 64);
        if (lane >= (uint32_t)d) incl += v;
    }
    total = __shfl(incl, 63, 64);
    return incl - x;
}

// One pattern on one tile: filter, verification, and in-order append of the
// hits to the pattern's staging area for this sub-range.  A singleton filter
// reads the tile's mismatch planes from the wave's LDS region (`planes`), an
// exhaustive one the raw planes in `s`.
template <int R, int L, bool EXH, int NG>
__device__ __forceinline__ uint32_t pattern_tile(const BatchArgs& a, CPattern& bp, uint32_t sub,
                                              uint64_t T0, uint64_t wlo, uint64_t whi, const Lane<R>& s,
                                              const uint32_t* planes, uint32_t count_before) {
    TileSrc src;
    src.text4 = a.text4;
    src.image = a.images + bp.image_off;
    src.win_begin = wlo;
    src.win_end = whi < bp.nw ? whi : bp.nw;
    if (src.win_begin >= src.win_end) return 0;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t B = T0 + (uint64_t)lane * R;
    const bool interior = 32 * T0 >= src.win_begin && 32 * (T0 + 64ull * R) <= src.win_end;
    Counters<R, L> C;
    uint32_t hit[R], nh;
    if constexpr (EXH) {
        tile_filter<R, L, true, false>(src, bp.plan, B, interior, s, C, hit, nh);
    } else if constexpr (NG > 0) {
        // NG groups of full sets and no tail: the unrolled filter
        uint32_t sw[2 * NG], dead[R];
        const uint32_t* rows[2 * NG];
#pragma unroll
        for (int g = 0; g < 2 * NG; ++g) {
            sw[g] = bp.plan.slot[g];
            rows[g] = set_row<R + 2>(planes, sw[g]);
        }
        fixed_filter<R, L, NG, 2>(rows, sw, bp.plan.init, dead);
        if (!interior) {
            uint32_t valid[R];
            valid_windows<R>(src, B, valid);
#pragma unroll
            for (int i = 0; i < R; ++i) dead[i] |= ~valid[i];
        }
        verify_survivors<R, false, kVerifyChunks>(src, bp.plan, B, dead, hit, nh);
    } else {
        init_counters<R, L>(src, bp.plan, B, interior, C);
        planes_filter<R, L>(planes, bp.plan, C);
        verify_survivors<R, false, kVerifyChunks>(src, bp.plan, B, C.dead, hit, nh);
    }
    if (__ballot(nh != 0) == 0) return 0;
    uint32_t total;
    uint32_t idx = count_before + wave_exclusive(nh, total);
    unsigned long long* out = a.staged + bp.stage_off + (uint64_t)sub * bp.cap_sub;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        uint32_t h = hit[i];
        while (h) {
            const uint32_t b = __builtin_ctz(h);
            h &= h - 1u;
            if (idx < bp.cap_sub) {
                const uint64_t pos = 32 * (B + i) + b;
                out[idx] = (pos << 16) | hit_count<R, L, EXH>(src, bp.plan, C, i, b, pos);
            }
            ++idx;
        }
    }
    return total;
}

// The patterns of an item share their variant: filter kind EXH, counter depth
// L and, for an unrolled singleton filter, its NG groups (0: the loop
// filter), so the item's whole tile loop is one code path.  A singleton item
// writes each tile's four mismatch planes to the wave's LDS region once for
// all its patterns.
template <int R, bool EXH, int L, int NG>
__device__ __forceinline__ void run_item(const BatchArgs& a, const BatchItem& it, uint64_t blo, uint64_t wlo,
                                         uint64_t whi, uint32_t* cnt, uint32_t* planes) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t tile = 64ull * R;
    auto load = [&](uint64_t T0, uint4 (&t)[(R + 2) / 2]) {
        const uint32_t g0 = (uint32_t)(T0 >> 1) + lane * (R / 2);
#pragma unroll
        for (int u = 0; u < (R + 2) / 2; ++u) t[u] = a.text4[min(g0 + (uint32_t)u, a.n4_last)];
    };
    const uint64_t first = blo + ((wlo / 32 - blo) / tile) * tile;
    if constexpr (EXH) {
        // (no prefetch: the raw planes stay in registers through the
        // patterns, and the exhaustive items are few and long)
        for (uint64_t T0 = first; 32 * T0 < whi; T0 += tile) {
            uint4 txt[(R + 2) / 2];
            load(T0, txt);
            Lane<R> s;
            make_lane<R>(txt, 0u, s);
            for (uint32_t g = 0; g < it.count; ++g) {
                CPattern& bp = const_pattern(a.pats + it.first + g);
                const uint32_t before = __builtin_amdgcn_readfirstlane(cnt[g]);
                const uint32_t added = pattern_tile<R, L, EXH, NG>(a, bp, it.sub, T0, wlo, whi, s, planes, before);
                if ((threadIdx.x & 63u) == 0) cnt[g] = before + added;
            }
        }
    } else {
        // The tile's text goes to the LDS planes, and the register buffer is
        // then reloaded with the item's next tile while the patterns are
        // counted: an item of one or two patterns has too little work per
        // tile for the other waves to cover the load (the last load, past
        // the item, reads a clamped address and is not used).
        uint4 buf[(R + 2) / 2];
        if (32 * first < whi) load(first, buf);
        Lane<R> none;  // (read by the exhaustive filter only)
        for (uint64_t T0 = first; 32 * T0 < whi; T0 += tile) {
            store_planes<R>(buf, 15u, planes);
            load(T0 + tile, buf);
            for (uint32_t g = 0; g < it.count; ++g) {
                CPattern& bp = const_pattern(a.pats + it.first + g);
                const uint32_t before = __builtin_amdgcn_readfirstlane(cnt[g]);
                const uint32_t added = pattern_tile<R, L, EXH, NG>(a, bp, it.sub, T0, wlo, whi, none, planes, before);
                if ((threadIdx.x & 63u) == 0) cnt[g] = before + added;
            }
        }
    }
}

// Two kernels: KIND 0 takes the patterns with L <= 4 counter levels (k - #'-'
// <= 15), singleton or exhaustive, KIND 1 those with L = 5 or 6, so that the
// common kernel is not sized for the deepest counters.
constexpr int kKinds = 2;

__host__ __device__ constexpr int kind_of(uint32_t variant) { return (variant & 7u) >= 5u ? 1 : 0; }

template <int R, int KIND>
__device__ __forceinline__ void run_variant(const BatchArgs& a, const BatchItem& it, uint32_t variant, uint64_t blo,
                                            uint64_t wlo, uint64_t whi, uint32_t* cnt, uint32_t* planes) {
    if constexpr (KIND == 0) {
        switch (variant & 0x7Fu) {
#define PM_V(L)                                                                             \
    case L: run_item<R, false, L, 0>(a, it, blo, wlo, whi, cnt, planes); return;           \
    case 0x10 | L: run_item<R, false, L, 1>(a, it, blo, wlo, whi, cnt, planes); return;    \
    case 0x20 | L: run_item<R, false, L, 2>(a, it, blo, wlo, whi, cnt, planes); return;    \
    case 0x30 | L: run_item<R, false, L, 3>(a, it, blo, wlo, whi, cnt, planes); return;    \
    case 0x40 | L: run_item<R, false, L, 4>(a, it, blo, wlo, whi, cnt, planes); return;    \
    case 0x08 | L: run_item<R, true, L, 0>(a, it, blo, wlo, whi, cnt, planes); return;
            PM_V(0) PM_V(1) PM_V(2) PM_V(3) PM_V(4)
#undef PM_V
            default: return;
        }
    } else {
        switch (variant & 15u) {
            case 5: run_item<R, false, 5, 0>(a, it, blo, wlo, whi, cnt, planes); return;
            case 6: run_item<R, false, 6, 0>(a, it, blo, wlo, whi, cnt, planes); return;
            case 13: run_item<R, true, 5, 0>(a, it, blo, wlo, whi, cnt, planes); return;
            case 14: run_item<R, true, 6, 0>(a, it, blo, wlo, whi, cnt, planes); return;
            default: return;
        }
    }
}

// The common kernel at R = 4 is held to 80 registers, six waves per SIMD
// (the exhaustive filter's paths spill a few registers for it; 3% faster
// than five waves on the batched workload).
template <int R, int KIND>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(KIND == 0 && R == 4 ? 6 : 1)))
void batch_kernel(BatchArgs a) {
    const uint32_t lane = threadIdx.x & 63u;
    // per-pattern running hit counts of this item, in the wave's LDS slice
    // (indexed by the pattern's place in the group, which is not a
    // compile-time constant, so registers would be addressed indirectly)
    __shared__ uint32_t s_cnt[TPB / 64][kMaxGroup];
    // mismatch planes of the current tile, one region per wave (singleton
    // filters only)
    __shared__ uint32_t s_planes[TPB / 64][4 * (R + 2) * 64];
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t* cnt = s_cnt[wv];
    while (true) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(a.queue, 1u);
        item = __builtin_amdgcn_readfirstlane(__shfl(item, 0, 64));
        if (item >= a.n_items) break;
        const BatchItem it = {const_item(a.items + item).first, const_item(a.items + item).count,
                              const_item(a.items + item).sub, 0};
        const uint64_t blo = a.wb0 + (uint64_t)it.sub * a.span_blocks;
        const uint64_t bhi = blo + a.span_blocks;
        const uint64_t wlo = 32 * blo > a.win_begin ? 32 * blo : a.win_begin;
        const uint64_t whi = 32 * bhi < a.win_end ? 32 * bhi : a.win_end;
        if (lane < (uint32_t)kMaxGroup) cnt[lane] = 0;
        if (wlo < whi) run_variant<R, KIND>(a, it, const_pattern(a.pats + it.first).variant, blo, wlo, whi, cnt, s_planes[wv]);
        if (lane < it.count)
            a.counts[(uint64_t)const_pattern(a.pats + it.first + lane).index * a.n_sub + it.sub] = cnt[lane];
    }
}

// One workgroup per work entry (p, y, nb): concatenate pattern p's
// sub-ranges in text order.  Every workgroup of p forms the sub-ranges'
// output offsets from their hit counts (a workgroup-wide scan in LDS); it
// then writes share y of nb of p's outputs, each thread finding the
// sub-range of an output slot by binary search over the offsets, with
// kGatherVec loads in flight.  Share 0 reports the total and the status.
constexpr int kGatherVec = 8;

__global__ __launch_bounds__(TPB) void batch_gather_kernel(const GatherPattern* gp, const GatherWork* work,
                                                           const uint32_t* counts, uint32_t n_sub,
                                                           const unsigned long long* staged, int64_t* pos,
                                                           uint16_t* cnt, unsigned long long* n_hits,
                                                           uint32_t* status) {
    extern __shared__ unsigned long long s_off[];  // n_sub + 1 entries (dynamic)
    __shared__ unsigned long long s_part[TPB];
    __shared__ uint32_t s_flag;
    const GatherWork wk = work[blockIdx.x];
    const uint32_t p = wk.p;
    const GatherPattern g = gp[p];
    const uint32_t* cp = counts + (uint64_t)p * n_sub;
    if (threadIdx.x == 0) {
        s_flag = 0;
        s_off[0] = 0;
    }
    // the counts (up to 16 per thread) are loaded together, then stored
    constexpr uint32_t kCountVec = (kMaxSubRanges + TPB - 1) / TPB;
    for (uint32_t s0 = threadIdx.x; s0 < n_sub; s0 += TPB * kCountVec) {
        uint32_t c[kCountVec];
#pragma unroll
        for (uint32_t j = 0; j < kCountVec; ++j) {
            const uint32_t s = s0 + j * TPB;
            c[j] = s < n_sub ? cp[s] : 0u;
        }
#pragma unroll
        for (uint32_t j = 0; j < kCountVec; ++j) {
            const uint32_t s = s0 + j * TPB;
            if (s < n_sub) s_off[s + 1] = c[j];
        }
    }
    __syncthreads();
    // each thread sums a contiguous run of sub-ranges, the runs' totals are
    // scanned across the workgroup, and each thread then forms its offsets
    const uint32_t per = (n_sub + TPB - 1) / TPB;
    const uint32_t s0 = min(n_sub, threadIdx.x * per), s1 = min(n_sub, s0 + per);
    unsigned long long run = 0;
    bool over = false;
    for (uint32_t s = s0; s < s1; ++s) {
        const unsigned long long c = s_off[s + 1];
        over |= c > g.cap_sub;
        run += c;
    }
    s_part[threadIdx.x] = run;
    __syncthreads();
    for (uint32_t d = 1; d < TPB; d <<= 1) {
        const unsigned long long v = threadIdx.x >= d ? s_part[threadIdx.x - d] : 0;
        __syncthreads();
        s_part[threadIdx.x] += v;
        __syncthreads();
    }
    unsigned long long base = threadIdx.x ? s_part[threadIdx.x - 1] : 0;
    for (uint32_t s = s0; s < s1; ++s) {
        base += s_off[s + 1];
        s_off[s + 1] = base;
    }
    const unsigned long long total = s_part[TPB - 1];
    if (over) atomicOr(&s_flag, 1u);
    __syncthreads();
    const uint32_t bad = (s_flag || total > g.capacity) ? 1u : 0u;
    if (wk.y == 0 && threadIdx.x == 0) {
        n_hits[p] = total;
        status[p] = bad;
    }
    if (bad) return;
    const unsigned long long share = (total + wk.nb - 1) / wk.nb;
    const unsigned long long lo = min(total, (unsigned long long)wk.y * share);
    const unsigned long long hi = min(total, lo + share);
    const unsigned long long* src = staged + g.stage_off;
    int64_t* po = pos + g.out_off;
    uint16_t* co = cnt + g.out_off;
    for (unsigned long long i0 = lo; i0 < hi; i0 += (unsigned long long)TPB * kGatherVec) {
        unsigned long long v[kGatherVec];
#pragma unroll
        for (int j = 0; j < kGatherVec; ++j) {
            const unsigned long long i = i0 + (unsigned long long)j * TPB + threadIdx.x;
            v[j] = 0;
            if (i < hi) {
                // s_off[a] <= i < s_off[b]; s_off[0] = 0 and s_off[n_sub] = total > i
                uint32_t a = 0, b = n_sub;
                while (b - a > 1) {
                    const uint32_t mid = (a + b) >> 1;
                    if (s_off[mid] <= i) a = mid;
                    else b = mid;
                }
                v[j] = src[(uint64_t)a * g.cap_sub + (i - s_off[a])];
            }
        }
#pragma unroll
        for (int j = 0; j < kGatherVec; ++j) {
            const unsigned long long i = i0 + (unsigned long long)j * TPB + threadIdx.x;
            if (i < hi) {
                po[i] = (int64_t)(v[j] >> 16);
                co[i] = (uint16_t)(v[j] & 0xFFFFu);
            }
        }
    }
}

__global__ void fill_zero_kernel(uint32_t* p, uint64_t words) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

struct BatchShape {
    uint32_t G, S, R;
    uint64_t span_blocks, wb0;
};

// Workspace layout.  The descriptor (patterns, gather records, images, work
// items) comes first and is copied from the host in one piece up to the last
// item in use; the queue words and the counts are zeroed on the device.
// Gather workgroups of a pattern: one per 64K output slots, at most 1024,
// and at most 65536 / count so that a call launches about 64K in all.
uint32_t gather_blocks(uint64_t capacity, uint32_t count) {
    const uint64_t cap = std::max<uint64_t>(1, std::min<uint64_t>(1024, 65536 / std::max<uint32_t>(count, 1)));
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(cap, (capacity + 65535) >> 16));
}

struct BatchLayout {
    uint64_t pats, gather, gwork, images, items, queue, counts, staged, bytes;
    uint64_t n_gwork;
    std::vector<uint64_t> image_off, stage_off;
    std::vector<uint32_t> cap_sub;
    uint64_t n_items_max;
};

// Groups of a singleton plan that the unrolled filter takes (1 to 4 groups of
// full sets, no tail, at most 4 counter levels), else 0 (the loop filter).
uint32_t fixed_groups(const ScanPlan& p) {
    if (p.exhaustive || p.n_slots == 0 || p.levels > 4 || p.n_groups < 1 || p.n_groups > 4 ||
        p.n_sets != 2 * p.n_groups || p.n_slots != 8 * p.n_groups)
        return 0;
    for (uint32_t t = 0; t < p.n_sets; ++t)
        if ((p.slot[t] >> 3 & 7u) != 4u) return 0;
    return p.n_groups;
}

BatchShape batch_shape(uint64_t n, uint32_t count, const pm_batch_config* cfg, uint64_t win_begin,
                       uint64_t win_end) {
    BatchShape sh;
    sh.G = cfg && cfg->group_size ? std::min<uint32_t>(cfg->group_size, kMaxGroup) : 8;
    // lane words: as asked, or (0) 6 for calls of 2 to 16 patterns and 4
    // otherwise.  Such calls make few long items, each a chain of tiles that
    // one wave runs in order, and six lane words per tile take a third fewer
    // links (served-pool patterns over the genome text: 10-28% less time at
    // 2 to 8 patterns, 4% at 16, none from 32 on; a lone pattern took twice
    // as long in one case, where the six-word kernel's three waves per SIMD
    // hold fewer items at once than its 4096).
    sh.R = cfg && cfg->lane_words == 6 ? 6
           : cfg && cfg->lane_words != 0 ? 4
           : (count >= 2 && count <= 16 ? 6 : 4);
    uint32_t S = cfg && cfg->sub_ranges ? cfg->sub_ranges : batch_auto_sub_ranges(count, cfg);
    S = std::min<uint32_t>(S, kMaxSubRanges);
    sh.S = S;
    if (win_end > n) win_end = n;
    if (win_begin > win_end) win_begin = win_end;
    sh.wb0 = (win_begin / 32) & ~1ull;
    const uint64_t tile = 64ull * sh.R;
    const uint64_t blocks = (win_end + 31) / 32 - sh.wb0 + 1;
    const uint64_t per = (blocks + S - 1) / S;
    sh.span_blocks = std::max<uint64_t>(tile, (per + tile - 1) / tile * tile);
    return sh;
}

BatchLayout batch_layout(uint32_t count, const uint32_t* m, const uint64_t* capacity, const BatchShape& sh,
                         bool with_images) {
    BatchLayout L;
    L.image_off.resize(count);
    L.stage_off.resize(count);
    L.cap_sub.resize(count);
    L.n_items_max = (uint64_t)((count + sh.G - 1) / sh.G) * sh.S + (uint64_t)count * sh.S;
    uint64_t img = 0, stg = 0;
    for (uint32_t p = 0; p < count; ++p) {
        L.image_off[p] = img;
        if (with_images) img += (m[p] + 31) / 32;
        const uint64_t c = capacity[p];
        const uint64_t cs = std::min<uint64_t>(c, (2 * c + sh.S - 1) / sh.S + 16);
        L.cap_sub[p] = (uint32_t)std::min<uint64_t>(cs, 0xFFFFFFF0ull);
        L.stage_off[p] = stg;
        stg += (uint64_t)sh.S * L.cap_sub[p];
    }
    uint64_t off = 0;
    L.pats = off;
    off = align256(off + sizeof(BatchPattern) * (uint64_t)count);
    L.gather = off;
    off = align256(off + sizeof(GatherPattern) * (uint64_t)count);
    L.n_gwork = 0;
    for (uint32_t p = 0; p < count; ++p) L.n_gwork += gather_blocks(capacity[p], count);
    L.gwork = off;
    off = align256(off + sizeof(GatherWork) * L.n_gwork);
    L.images = off;
    off = align256(off + 16 * img);
    L.items = off;
    off = align256(off + sizeof(BatchItem) * L.n_items_max);
    L.queue = off;
    off = align256(off + 4 * kKinds);
    L.counts = off;
    off = align256(off + 4ull * count * sh.S);
    L.staged = off;
    off = align256(off + 8 * stg);
    L.bytes = off;
    return L;
}

bool capacities_fit(uint32_t count, const uint64_t* capacity) {
    uint64_t left = kMaxTotalCapacity;
    for (uint32_t p = 0; p < count; ++p) {
        if (capacity[p] > left) return false;
        left -= capacity[p];
    }
    return true;
}

pm_status check_batch_args(uint32_t count, const uint32_t* m, const uint32_t* k, const uint64_t* capacity) {
    if (count == 0) return PM_OK;
    if (!m || !k || !capacity) return set_error(PM_ERR_ARG, "null pointer");
    for (uint32_t p = 0; p < count; ++p) {
        if (m[p] == 0) return set_error(PM_ERR_ARG, "pattern " + std::to_string(p) + " is empty");
        if (k[p] > 65535) return set_error(PM_ERR_ARG, "k above 65535 for pattern " + std::to_string(p));
    }
    if (!capacities_fit(count, capacity)) return set_error(PM_ERR_ARG, "output capacities above 2^44 hits in total");
    return PM_OK;
}

using BatchFn = void (*)(BatchArgs);

unsigned batch_grid(BatchFn fn, uint64_t items) {
    const uint64_t blocks = std::min<uint64_t>(resident_blocks(reinterpret_cast<const void*>(fn)), (items + 3) / 4);
    return (unsigned)std::max<uint64_t>(blocks, 1);
}

}  // namespace

namespace pm {

uint32_t batch_auto_sub_ranges(uint32_t count, const pm_batch_config* cfg) {
    const uint64_t G = cfg && cfg->group_size ? std::min<uint32_t>(cfg->group_size, kMaxGroup) : 8;
    const uint64_t groups = std::max<uint64_t>(1, (count + G - 1) / G);
    return (uint32_t)std::min<uint64_t>(kMaxSubRanges, (kAutoItems + groups - 1) / groups);
}

uint64_t batch_ws_bytes(uint64_t n, uint32_t count, const uint32_t* m, const uint64_t* capacity,
                        const pm_batch_config* cfg, bool with_images) {
    if (count == 0 || !m || !capacity) return 256;
    if (!capacities_fit(count, capacity)) return UINT64_MAX;
    const BatchShape sh = batch_shape(n, count, cfg, 0, n);
    return batch_layout(count, m, capacity, sh, with_images).bytes;
}

uint64_t batch_desc_bytes(uint64_t n, uint32_t count, const uint32_t* m, const uint64_t* capacity,
                          const pm_batch_config* cfg, bool with_images) {
    if (count == 0 || !m || !capacity) return 256;
    if (!capacities_fit(count, capacity)) return UINT64_MAX;
    const BatchShape sh = batch_shape(n, count, cfg, 0, n);
    return batch_layout(count, m, capacity, sh, with_images).queue;
}

pm_status batch_run(const BatchCall& c) {
    const uint32_t count = c.count;
    if (count == 0) return PM_OK;
    if (!c.text_dev || !c.entries || !c.n_hits_dev || !c.status_dev || !c.ws_dev)
        return set_error(PM_ERR_ARG, "null pointer");
    if (reinterpret_cast<uintptr_t>(c.text_dev) % 16 != 0)
        return set_error(PM_ERR_ARG, "text_dev must be 16-byte aligned");
    const uint64_t n = c.n;
    if (encoded_text_groups(n) >= (1ull << 32)) return set_error(PM_ERR_UNSUPPORTED, "texts are limited to 2^37 bases");
    std::vector<uint32_t> m(count), k(count);
    std::vector<uint64_t> capacity(count);
    for (uint32_t p = 0; p < count; ++p) {
        const BatchEntry& e = c.entries[p];
        if (!e.codes) return set_error(PM_ERR_ARG, "null pattern codes");
        m[p] = e.m;
        k[p] = e.k;
        capacity[p] = e.capacity;
        if (e.capacity > 0 && (!c.pos_dev || !c.cnt_dev))
            return set_error(PM_ERR_ARG, "null output with capacity > 0");
    }
    pm_status st = check_batch_args(count, m.data(), k.data(), capacity.data());
    if (st != PM_OK) return st;
    const bool with_images = c.images_dev == nullptr;
    hipStream_t s = c.stream;
    uint64_t win_begin = c.win_begin, win_end = c.win_end;
    if (win_end > n) win_end = n;
    if (win_begin > win_end) win_begin = win_end;
    // The workspace is laid out for the whole text (full.S sub-ranges per
    // pattern).  A call uses only as many sub-ranges as its window range
    // fills with whole tiles, and gives each the staging of the unused ones.
    const BatchShape full = batch_shape(n, count, c.cfg, 0, n);
    BatchLayout L = batch_layout(count, m.data(), capacity.data(), full, with_images);
    if (c.ws_bytes < L.bytes)
        return set_error(PM_ERR_WORKSPACE, "workspace too small: need " + std::to_string(L.bytes) + " bytes");
    BatchShape sh = full;
    {
        const uint64_t tile = 64ull * sh.R;
        sh.wb0 = (win_begin / 32) & ~1ull;
        const uint64_t blocks = (win_end + 31) / 32 - sh.wb0 + 1;
        sh.S = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(full.S, (blocks + tile - 1) / tile));
        const uint64_t per = (blocks + sh.S - 1) / sh.S;
        sh.span_blocks = (per + tile - 1) / tile * tile;
        for (uint32_t p = 0; p < count; ++p)
            L.cap_sub[p] = (uint32_t)std::min<uint64_t>((uint64_t)full.S * L.cap_sub[p] / sh.S, 0xFFFFFFF0ull);
    }

    // the descriptor: staged in the caller's pinned buffer, or a pageable one
    std::vector<uint8_t> own;
    uint8_t* desc = c.desc_host;
    if (desc) {
        if (c.desc_host_bytes < L.queue) return set_error(PM_ERR_WORKSPACE, "descriptor staging too small");
    } else {
        own.assign(L.queue, 0);
        desc = own.data();
    }
    BatchPattern* sorted = reinterpret_cast<BatchPattern*>(desc + L.pats);
    GatherPattern* gat = reinterpret_cast<GatherPattern*>(desc + L.gather);
    GatherWork* gwork = reinterpret_cast<GatherWork*>(desc + L.gwork);
    {
        uint64_t e = 0;
        for (uint32_t p = 0; p < count; ++p) {
            const uint32_t nb = gather_blocks(capacity[p], count);
            for (uint32_t y = 0; y < nb; ++y) gwork[e++] = {p, y, nb, 0u};
        }
    }
    uint32_t* img_words = reinterpret_cast<uint32_t*>(desc + L.images);
    BatchItem* items = reinterpret_cast<BatchItem*>(desc + L.items);

    // plans, images, groups and queue order on the host
    for (uint32_t p = 0; p < count; ++p)
        for (uint32_t j = 0; j < c.entries[p].m; ++j)
            if (c.entries[p].codes[j] > 15)
                return set_error(PM_ERR_SYMBOL, "pattern code above 15 in pattern " + std::to_string(p));
    std::vector<BatchPattern> pats(count);
    std::vector<double> cost(count, 0.0);
    auto prepare = [&](uint32_t p0, uint32_t p1) {
        for (uint32_t p = p0; p < p1; ++p) {
            const BatchEntry& e = c.entries[p];
            BatchPattern& bp = pats[p];
            std::memset(&bp, 0, sizeof(bp));
            bp.plan = e.plan ? *e.plan : build_plan(e.codes, e.m, e.k, kBatchSurvival, /*window_at_zero=*/true);
            bp.image_off = with_images ? L.image_off[p] : e.image_off;
            bp.stage_off = L.stage_off[p];
            bp.cap_sub = L.cap_sub[p];
            bp.nw = e.m <= n ? n - e.m + 1 : 0;
            bp.index = p;
            const bool skip = bp.plan.keff < 0 || bp.nw == 0 || bp.nw <= win_begin;
            bp.variant = skip ? kSkip : (bp.plan.exhaustive ? 8u : 0u) | bp.plan.levels | fixed_groups(bp.plan) << 4;
            if (with_images) build_image(e.codes, e.m, img_words + 4 * L.image_off[p]);
            // cost per tile: filter slots, plus a full count per window without a filter
            cost[p] = skip ? 0.0
                           : (bp.plan.n_slots > 0 || bp.plan.exhaustive ? 8.0 + bp.plan.n_slots
                                                                        : 8.0 + 32.0 * 10.0 * bp.plan.nchunks);
            GatherPattern& g = gat[p];
            std::memset(&g, 0, sizeof(g));
            g.stage_off = L.stage_off[p];
            g.out_off = e.out_off;
            g.capacity = e.capacity;
            g.cap_sub = L.cap_sub[p];
        }
    };
    // large batches are prepared by several host threads, in disjoint ranges
    uint64_t work = 0;
    for (uint32_t p = 0; p < count; ++p) work += c.entries[p].m + 64;
    const uint32_t hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const uint32_t nt = (uint32_t)std::min<uint64_t>({hw, count, std::max<uint64_t>(1, work >> 17)});
    if (nt <= 1) {
        prepare(0, count);
    } else {
        std::vector<std::thread> th;
        th.reserve(nt);
        for (uint32_t t = 0; t < nt; ++t)
            th.emplace_back(prepare, (uint32_t)((uint64_t)count * t / nt), (uint32_t)((uint64_t)count * (t + 1) / nt));
        for (auto& x : th) x.join();
    }
    // groups: same variant, similar filter cost, then similar length (the
    // cost of verifying a survivor); items: (group, sub-range), costly first
    std::vector<uint32_t> order(count);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        if (pats[x].variant != pats[y].variant) return pats[x].variant < pats[y].variant;
        if (cost[x] != cost[y]) return cost[x] > cost[y];
        return pats[x].plan.nchunks > pats[y].plan.nchunks;
    });
    for (uint32_t i = 0; i < count; ++i) sorted[i] = pats[order[i]];
    struct Group {
        uint32_t first, count;
        double cost;
    };
    std::vector<Group> groups;
    for (uint32_t i = 0; i < count;) {
        uint32_t j = i;
        double cs = 0;
        const uint32_t gmax = (sorted[i].variant & 8u) ? std::max(1u, sh.G / kExhGroupDiv) : sh.G;
        while (j < count && j - i < gmax && sorted[j].variant == sorted[i].variant) cs += cost[order[j++]];
        groups.push_back({i, j - i, cs});
        i = j;
    }
    std::stable_sort(groups.begin(), groups.end(), [](const Group& x, const Group& y) { return x.cost > y.cost; });
    // items by kernel kind (common, deep counters), each kind's items in a
    // run of their own, costly first
    uint64_t n_items = 0, kind_end[kKinds] = {0, 0};
    for (int kind = 0; kind < kKinds; ++kind) {
        for (const Group& g : groups) {
            if (g.cost == 0.0 || kind_of(sorted[g.first].variant) != kind) continue;
            if (n_items + sh.S > L.n_items_max) return set_error(PM_ERR_ARG, "internal: too many work items");
            for (uint32_t sub = 0; sub < sh.S; ++sub) items[n_items++] = {g.first, g.count, sub, 0};
        }
        kind_end[kind] = n_items;
    }

    uint8_t* ws = reinterpret_cast<uint8_t*>(c.ws_dev);
    hipError_t e;
    // one copy of the descriptor up to the last item in use
    const uint64_t desc_used = L.items + sizeof(BatchItem) * n_items;
    if ((e = hipMemcpyAsync(ws, desc, desc_used, hipMemcpyHostToDevice, s)) != hipSuccess)
        return set_error(PM_ERR_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    // queue and per-(pattern, sub-range) counts start at zero (patterns that
    // get no work item keep zero counts)
    fill_zero_kernel<<<1024, TPB, 0, s>>>(reinterpret_cast<uint32_t*>(ws + L.queue), (L.staged - L.queue) / 4);
    if ((e = hipGetLastError()) != hipSuccess) return set_error(PM_ERR_HIP, hipGetErrorString(e));

    BatchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.text4 = reinterpret_cast<const uint4*>(c.text_dev);
    a.n4_last = (uint32_t)(encoded_text_groups(n) - 1);
    a.images = with_images ? reinterpret_cast<const uint4*>(ws + L.images)
                           : reinterpret_cast<const uint4*>(c.images_dev);
    a.pats = reinterpret_cast<const BatchPattern*>(ws + L.pats);
    a.items = reinterpret_cast<const BatchItem*>(ws + L.items);
    a.staged = reinterpret_cast<unsigned long long*>(ws + L.staged);
    a.counts = reinterpret_cast<uint32_t*>(ws + L.counts);
    a.queue = reinterpret_cast<uint32_t*>(ws + L.queue);
    a.n_sub = sh.S;
    a.win_begin = win_begin;
    a.win_end = win_end;
    a.wb0 = sh.wb0;
    a.span_blocks = sh.span_blocks;
    // one launch per kind that has items, each on its own queue word
    if ((e = mark_begin(s)) != hipSuccess) return set_error(PM_ERR_HIP, hipGetErrorString(e));
    static constexpr BatchFn kFns[2][kKinds] = {{batch_kernel<4, 0>, batch_kernel<4, 1>},
                                                {batch_kernel<6, 0>, batch_kernel<6, 1>}};
    for (int kind = 0; kind < kKinds; ++kind) {
        const uint64_t first = kind ? kind_end[kind - 1] : 0;
        if (kind_end[kind] == first) continue;
        BatchFn fn = kFns[sh.R == 4 ? 0 : 1][kind];
        BatchArgs w = a;
        w.items = a.items + first;
        w.n_items = (uint32_t)(kind_end[kind] - first);
        w.queue = a.queue + kind;
        fn<<<batch_grid(fn, w.n_items), TPB, 0, s>>>(w);
        if ((e = hipGetLastError()) != hipSuccess) return set_error(PM_ERR_HIP, hipGetErrorString(e));
    }
    if ((e = mark_end(s)) != hipSuccess) return set_error(PM_ERR_HIP, hipGetErrorString(e));
    batch_gather_kernel<<<(unsigned)L.n_gwork, TPB, 8 * (sh.S + 1), s>>>(
        reinterpret_cast<const GatherPattern*>(ws + L.gather), reinterpret_cast<const GatherWork*>(ws + L.gwork),
        a.counts, sh.S, a.staged, c.pos_dev, c.cnt_dev, reinterpret_cast<unsigned long long*>(c.n_hits_dev),
        c.status_dev);
    if ((e = hipGetLastError()) != hipSuccess) return set_error(PM_ERR_HIP, hipGetErrorString(e));
    return PM_OK;
}

}  // namespace pm

extern "C" {

pm_status pm_expected_hits(const uint8_t* codes, uint32_t m, uint32_t k, uint64_t n, double* out) {
    if (!codes || !out) return set_error(PM_ERR_ARG, "null pointer");
    for (uint32_t j = 0; j < m; ++j)
        if (codes[j] > 15) return set_error(PM_ERR_SYMBOL, "pattern code above 15");
    *out = expected_hits(codes, m, k, n);
    return PM_OK;
}

uint64_t pm_scan_batch_workspace_bytes(uint64_t n, uint32_t count, const uint32_t* m, const uint64_t* capacity,
                                       const pm_batch_config* cfg) {
    const uint64_t b = batch_ws_bytes(n, count, m, capacity, cfg, true);
    return b == UINT64_MAX ? 0 : b;
}

pm_status pm_scan_batch(const void* text_dev, uint64_t n, uint32_t count, const uint8_t* codes,
                        const uint32_t* m, const uint32_t* k, const uint64_t* out_off, const uint64_t* capacity,
                        uint64_t win_begin, uint64_t win_end, int64_t* pos_dev, uint16_t* cnt_dev,
                        uint64_t* n_hits_dev, uint32_t* status_dev, void* ws_dev, uint64_t ws_bytes,
                        const pm_batch_config* cfg, void* stream) {
    if (count == 0) return PM_OK;
    if (!codes || !out_off) return set_error(PM_ERR_ARG, "null pointer");
    pm_status st = check_batch_args(count, m, k, capacity);
    if (st != PM_OK) return st;
    std::vector<BatchEntry> entries(count);
    uint64_t off = 0;
    for (uint32_t p = 0; p < count; ++p) {
        entries[p] = {codes + off, m[p], k[p], nullptr, 0, out_off[p], capacity[p]};
        off += m[p];
    }
    BatchCall c;
    c.text_dev = text_dev;
    c.n = n;
    c.count = count;
    c.entries = entries.data();
    c.win_begin = win_begin;
    c.win_end = win_end;
    c.pos_dev = pos_dev;
    c.cnt_dev = cnt_dev;
    c.n_hits_dev = n_hits_dev;
    c.status_dev = status_dev;
    c.ws_dev = ws_dev;
    c.ws_bytes = ws_bytes;
    c.cfg = cfg;
    c.stream = reinterpret_cast<hipStream_t>(stream);
    return batch_run(c);
}

}  // extern "C"
