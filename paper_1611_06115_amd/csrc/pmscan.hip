// pmscan.hip -- gfx950 kernels and the C ABI of libpmscan.
//
// Text: planar 2-bit blocks (Table 1 codes; per 32 bases one word of high
// code bits and one of low code bits).  Scan: each lane owns R consecutive
// blocks, i.e. 32*R consecutive windows, held bit-sliced (bit b of a word is
// one window).  Pair values (Table 3) for 32 windows at once are one bitwise
// function of two shifted text planes; the window sums of eq. (4) are kept
// as bit-sliced counters, so 32 windows advance per 32-bit operation.
//
// Per tile (one workgroup, 256 lanes):
//   1. filter: the plan's slots (the most selective positions inside one
//      64-position window of the pattern) are added into the bit-sliced
//      counters; a window whose count passes k - (#'-') is dropped.  Dropping
//      a window once its partial count exceeds the budget is the early stop
//      of Sect. 2.4, applied to 32 windows per word.
//   2. verify: windows that survive are counted exactly over all m positions
//      (one window per lane, 32 positions per step) unless the slots already
//      covered every position that can mismatch.
//   3. output: a tile is the 64*R*32 windows of one wave; the wave ranks its
//      hits with a prefix sum over its lanes and stores their number and, when
//      there are at most kCap, the hits themselves.  A second kernel sums the
//      counts per chunk of tiles, and a third places every tile's hits at their
//      ordered offset (re-scanning only tiles that had more than kCap hits).
//      Waves never wait on each other, and the output list is ascending
//      without a sort.
#include <hip/hip_runtime.h>



#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pmscan.h"
#include "plan.hpp"
#include "scan_core.hpp"
#include "scan_kernels.hpp"

namespace pm {
uint64_t resident_blocks(const void* fn);
}  // namespace pm

using pm::ScanPlan;
using namespace pm;

namespace {

constexpr uint64_t kPadBlocks = 64;  // zero blocks after the text (16-byte loads, halos)

thread_local std::string g_detail;

pm_status fail(pm_status s, const std::string& what) {
    g_detail = what;
    return s;
}

pm_status hip_fail(hipError_t e, const char* where) {
    return fail(PM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------

__global__ void fill_u64_kernel(uint64_t* p, uint64_t value, uint64_t count) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t value, uint64_t count) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

pm_status fill_u64(uint64_t* p, uint64_t value, uint64_t count, hipStream_t s) {
    if (count == 0) return PM_OK;
    unsigned grid = (unsigned)std::min<uint64_t>((count + 255) / 256, 4096);
    fill_u64_kernel<<<grid, 256, 0, s>>>(p, value, count);
    HIP_TRY(hipGetLastError());
    return PM_OK;
}

// ---------------------------------------------------------------------------
// text encoding (Table 1): ASCII -> planar blocks
// ---------------------------------------------------------------------------

// Four ASCII bytes -> four 2-bit codes: returns the high-bit nibble and the
// low-bit nibble (bit i <-> byte i) and a mask of invalid bytes (bit 7 of
// each byte).  Folding to lower case maps A,C,G,T to a,c,g,t = 0x61, 0x63,
// 0x67, 0x74, whose bits give the code as ((x >> 2) ^ (x >> 1)) & 3.
__device__ __forceinline__ void encode4(uint32_t w, uint32_t& hi4, uint32_t& lo4, uint32_t& bad) {
    const uint32_t x = w | 0x20202020u;
    uint32_t code = ((x >> 2) ^ (x >> 1)) & 0x03030303u;
    const uint32_t b0 = code & 0x01010101u, b1 = (code >> 1) & 0x01010101u;
    const uint32_t expect = 0x61616161u + 2u * b0 + 6u * b1 + 11u * (b0 & b1);
    const uint32_t diff = x ^ expect;
    bad = (((diff & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | diff) & 0x80808080u;
    code &= ~((bad >> 7) * 3u);  // invalid bytes encode as A
    lo4 = ((code & 0x01010101u) * 0x01020408u) >> 24 & 0xFu;
    hi4 = (((code >> 1) & 0x01010101u) * 0x01020408u) >> 24 & 0xFu;
}

__global__ void encode_text_kernel(const uint8_t* __restrict__ ascii, uint64_t n,
                                   uint2* __restrict__ out, uint64_t nblk_total,
                                   unsigned long long* __restrict__ bad_index, int aligned16) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; b < nblk_total; b += stride) {
        uint32_t hi = 0, lo = 0;
        unsigned long long first_bad = ~0ull;
        const uint64_t base = 32 * b;
        if (base < n) {
            uint32_t words[8];
            if (aligned16 && base + 32 <= n) {
                const uint4* p = reinterpret_cast<const uint4*>(ascii + base);
                const uint4 v0 = p[0], v1 = p[1];
                words[0] = v0.x; words[1] = v0.y; words[2] = v0.z; words[3] = v0.w;
                words[4] = v1.x; words[5] = v1.y; words[6] = v1.z; words[7] = v1.w;
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    uint32_t w = 0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const uint64_t i = base + 4 * q + j;
                        // bytes past n encode as 'A' and are never inspected
                        w |= (uint32_t)(i < n ? ascii[i] : 'A') << (8 * j);
                    }
                    words[q] = w;
                }
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                uint32_t h4, l4, bad;
                encode4(words[q], h4, l4, bad);
                hi |= h4 << (4 * q);
                lo |= l4 << (4 * q);
                if (bad && first_bad == ~0ull) first_bad = base + 4 * q + (__builtin_ctz(bad) >> 3);
            }
        }
        out[b] = make_uint2(hi, lo);
        if (first_bad != ~0ull) atomicMin(bad_index, first_bad);
    }
}

// ---------------------------------------------------------------------------
// scan: the kernels are in scan_kernels.hpp
// ---------------------------------------------------------------------------

#ifndef PMSCAN_LANE_WORDS
#define PMSCAN_LANE_WORDS 4
#endif
constexpr int kR = PMSCAN_LANE_WORDS;  // lane words (32 windows each) per lane

using ScanFn = void (*)(ScanArgs, ScanPlan);
struct ScanPair {
    ScanFn count, place;
};
template <int R, bool EXH>
ScanPair pick_scan_l(uint32_t L) {
    switch (L) {
#define PM_L(X) case X: return {scan_count_kernel<R, X, EXH>, scan_place_kernel<R, X, EXH>};
        PM_L(0) PM_L(1) PM_L(2) PM_L(3) PM_L(4) PM_L(5) PM_L(6)
#undef PM_L
        default: return {nullptr, nullptr};
    }
}
// Count kernels with the fixed filter: singleton plans of NG = 1..4 groups of
// full sets and 0..4 counter levels (k - #'-' up to 15).
template <int R, int NG>
ScanFn pick_fixed_l(uint32_t L) {
    switch (L) {
        case 0: return scan_fixed_kernel<R, 0, NG>;
        case 1: return scan_fixed_kernel<R, 1, NG>;
        case 2: return scan_fixed_kernel<R, 2, NG>;
        case 3: return scan_fixed_kernel<R, 3, NG>;
        case 4: return scan_fixed_kernel<R, 4, NG>;
        default: return nullptr;
    }
}
template <int R>
ScanFn pick_fixed(const ScanPlan& p) {
#ifdef PM_NO_FIXED
    return nullptr;
#endif
    if (p.exhaustive || p.n_slots == 0 || p.n_sets != 2 * p.n_groups || p.n_slots != 8 * p.n_groups) return nullptr;
    for (uint32_t t = 0; t < p.n_sets; ++t)
        if ((p.slot[t] >> 3 & 7u) != 4u) return nullptr;
    switch (p.n_groups) {
        case 1: return pick_fixed_l<R, 1>(p.levels);
        case 2: return pick_fixed_l<R, 2>(p.levels);
        case 3: return pick_fixed_l<R, 3>(p.levels);
        case 4: return pick_fixed_l<R, 4>(p.levels);
        default: return nullptr;
    }
}
// fixed_ok: the fixed kernel's 32-bit load offsets cover the launch.
template <int R>
ScanPair pick_scan(const ScanPlan& p, bool fixed_ok) {
    ScanPair f = p.exhaustive ? pick_scan_l<R, true>(p.levels) : pick_scan_l<R, false>(p.levels);
    if (f.count && fixed_ok)
        if (ScanFn fixed = pick_fixed<R>(p)) f.count = fixed;
    return f;
}

// The fixed kernel addresses the text with 32-bit byte offsets from the
// buffer start: tile t's lanes read bytes [tile_byte0 + t * 64 R * 8, + 64 R
// * 8 + 16 * ((R + 2) / 2 + R / 2 * 63)), for t up to n_tiles - 1 + the
// prefetch distance (four tiles); the buffer's size must fit too.
bool fixed_offsets_fit(uint64_t buffer_bytes, uint64_t tile_byte0, uint64_t n_tiles) {
    const uint64_t tile_bytes = 64ull * kR * 8;
    const uint64_t last = tile_byte0 + (n_tiles + 4) * tile_bytes + 16ull * ((kR + 2) / 2 + kR / 2 * 63);
    return buffer_bytes <= 0xFFFFFFFFull && last <= 0xFFFFFFFFull;
}

// Workgroups for a persistent kernel: as many as fit on the device at once
// (occupancy per CU x CUs), never more than there are tiles.
unsigned persistent_grid(ScanFn fn, uint64_t n_tiles) {
    const uint64_t resident = pm::resident_blocks(reinterpret_cast<const void*>(fn));
    return (unsigned)std::min<uint64_t>({n_tiles, resident, kMaxRanges});
}

uint64_t text_blocks(uint64_t n) { return ((n + 31) / 32 + kPadBlocks + 1) & ~1ull; }

// Plans of long patterns are kept per host thread: building one takes
// several passes over all m positions (~0.3 ms at m = 100 000, more than
// the scan of a chromosome), and the same pattern is often scanned many
// times.  An entry is used only for the same k and byte-for-byte the same
// codes (other patterns differ within a few bytes, the match costs one
// comparison of m bytes); its codes were checked when it was built.
constexpr uint32_t kPlanCacheMinM = 4096;
constexpr uint32_t kPlanCacheMaxM = 1u << 22;
constexpr size_t kPlanCacheEntries = 16;
struct PlanEntry {
    uint32_t k = 0;
    uint64_t used = 0;
    std::vector<uint8_t> codes;
    ScanPlan plan;
};
thread_local std::vector<PlanEntry> t_plans;
thread_local uint64_t t_plan_clock = 0;

// The plan of (codes, m, k), or PM_ERR_SYMBOL for a code above 15.
pm_status scan_plan(const uint8_t* codes, uint32_t m, uint32_t k, ScanPlan& plan) {
    const bool cache = m >= kPlanCacheMinM && m <= kPlanCacheMaxM;
    if (cache)
        for (PlanEntry& e : t_plans)
            if (e.k == k && e.codes.size() == m && std::memcmp(e.codes.data(), codes, m) == 0) {
                e.used = ++t_plan_clock;
                plan = e.plan;
                return PM_OK;
            }
    for (uint32_t j = 0; j < m; ++j)
        if (codes[j] > 15) return fail(PM_ERR_SYMBOL, "pattern code above 15 at " + std::to_string(j));
    plan = pm::build_plan(codes, m, k);
    if (cache) {
        if (t_plans.size() < kPlanCacheEntries) t_plans.emplace_back();
        PlanEntry* slot = &t_plans[0];
        for (PlanEntry& e : t_plans)
            if (e.used < slot->used) slot = &e;
        slot->k = k;
        slot->used = ++t_plan_clock;
        slot->codes.assign(codes, codes + m);
        slot->plan = plan;
    }
    return PM_OK;
}

uint64_t max_tiles(uint64_t n) {
    // tiles of 64*kR blocks, starting at an even block at or below win_begin
    const uint64_t blocks = (n + 31) / 32 + 2;
    return (blocks + 64ull * kR - 1) / (64ull * kR) + 1;
}

constexpr uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// Workspace layout for up to T tiles: hit counts (u32 per tile), hit sums
// (u64 per count-kernel workgroup), staged hits (kCap u64 per tile).
struct WsLayout {
    uint64_t counts, range_sum, staged, bytes;
};
constexpr WsLayout ws_layout(uint64_t T) {
    WsLayout w{};
    w.counts = 0;
    w.range_sum = align256(4 * T);
    w.staged = w.range_sum + align256(8ull * kMaxRanges);
    w.bytes = w.staged + 8 * (uint64_t)kCap * T;
    return w;
}

}  // namespace

namespace pm {
pm_status set_error(pm_status s, const std::string& what) { return fail(s, what); }

// Workgroups of `fn` (TPB threads) that fit on the current device at once,
// queried once per (device, kernel).
uint64_t resident_blocks(const void* fn) {
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, uint64_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find({dev, fn});
        if (it != cache.end()) return it->second;
    }
    int cus = 0, per_cu = 0;
    if (dev < 0 || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, TPB, 0) != hipSuccess || cus <= 0 || per_cu <= 0) {
        cus = 256;
        per_cu = 2;
    }
    const uint64_t r = (uint64_t)cus * (uint64_t)per_cu;
    std::lock_guard<std::mutex> lk(mu);
    cache[{dev, fn}] = r;
    return r;
}
uint64_t encoded_text_groups(uint64_t n) { return text_blocks(n) / 2; }

// Events the next scan call of this thread records around its main kernel
// launch(es) (pm_time_next_scan).
thread_local hipEvent_t t_ev_begin = nullptr, t_ev_end = nullptr;

hipError_t mark_begin(hipStream_t s) { return t_ev_begin ? hipEventRecord(t_ev_begin, s) : hipSuccess; }
hipError_t mark_end(hipStream_t s) {
    hipError_t e = t_ev_end ? hipEventRecord(t_ev_end, s) : hipSuccess;
    t_ev_begin = t_ev_end = nullptr;
    return e;
}
}  // namespace pm

// ---------------------------------------------------------------------------
// the scan launch over a workspace of a given layout
// ---------------------------------------------------------------------------
namespace {

// Scratch of pm_scan_noalloc: one copy per device, held until the process
// ends.  Host code never uses the array's name as an address (in host code
// it is only a stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device.
constexpr uint64_t kStaticScratchBytes = 32ull << 20;
__device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

// Tiles (and windows) one pm_scan_noalloc call may cover: the largest T
// whose workspace layout fits the scratch.
constexpr uint64_t static_max_tiles() {
    uint64_t t = (kStaticScratchBytes - 8ull * kMaxRanges - 512) / (4 + 8ull * kCap);
    while (t > 0 && ((4 * t + 255) & ~255ull) + ((8ull * kMaxRanges + 255) & ~255ull) + 8ull * kCap * t >
                        kStaticScratchBytes)
        --t;
    return t;
}
constexpr uint64_t kStaticMaxTiles = static_max_tiles();
// a window range [b, e) needs at most (e - b + 63) / 32 + 1 blocks from the
// even block at or below b, in tiles of 64 * kR blocks
constexpr uint64_t kStaticMaxWindows = (kStaticMaxTiles - 1) * 64ull * kR * 32 - 64;
static_assert(ws_layout(kStaticMaxTiles).bytes <= kStaticScratchBytes, "scratch layout");

// The device address of `scratch` on the current device, looked up once
// per device (with that device current) and kept.
pm_status static_scratch(uint8_t** out) {
    static std::mutex mu;
    static std::map<int, uint8_t*> addr;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(PM_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch");
        it = addr.emplace(dev, reinterpret_cast<uint8_t*>(ptr)).first;
    }
    *out = it->second;
    return PM_OK;
}

// One scan: argument checks, the plan, the count and place kernels on
// stream `stream`.  `ws` holds lay.bytes bytes; tile_limit > 0 bounds the
// tiles of the window range (a layout sized for a fixed number of tiles), 0
// means the layout was sized from n (any range of the text fits).
pm_status scan_launch(const void* text_dev, uint64_t n, const uint8_t* codes, uint32_t m, uint32_t k,
                      const void* image_dev, uint64_t win_begin, uint64_t win_end, int64_t* pos_dev,
                      uint16_t* cnt_dev, uint64_t capacity, uint64_t* n_hits_dev, uint8_t* ws,
                      const WsLayout& lay, uint64_t tile_limit, void* stream) {
    if (!text_dev || !codes || !image_dev || !n_hits_dev) return fail(PM_ERR_ARG, "null pointer");
    if (capacity > 0 && (!pos_dev || !cnt_dev)) return fail(PM_ERR_ARG, "null output with capacity > 0");
    if (m == 0) return fail(PM_ERR_ARG, "empty pattern (m = 0)");
    if (k > 65535) return fail(PM_ERR_ARG, "k above 65535 (counts are 16-bit)");
    if (reinterpret_cast<uintptr_t>(text_dev) % 16 != 0)
        return fail(PM_ERR_ARG, "text_dev must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(image_dev) % 16 != 0)
        return fail(PM_ERR_ARG, "image_dev must be 16-byte aligned");
    if (text_blocks(n) / 2 >= (1ull << 32)) return fail(PM_ERR_UNSUPPORTED, "texts are limited to 2^37 bases");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    const uint64_t nw = m <= n ? n - m + 1 : 0;
    if (win_end > nw) win_end = nw;
    ScanPlan plan;
    if (const pm_status st = scan_plan(codes, m, k, plan); st != PM_OK) return st;
    if (win_begin >= win_end || plan.keff < 0) return fill_u64(n_hits_dev, 0, 1, s);

    const uint64_t wb0 = (win_begin >> 5) & ~1ull;
    const uint64_t wb_end = (win_end + 31) >> 5;
    const uint64_t tile_blocks = 64ull * kR;
    const uint64_t n_tiles = (wb_end - wb0 + tile_blocks - 1) / tile_blocks;
    if (n_tiles > (tile_limit ? tile_limit : max_tiles(n)) || n_tiles > 0xFFFFFFFFull)
        return fail(PM_ERR_ARG, "window range too large");

    const uint64_t buffer_bytes = 16 * (text_blocks(n) / 2), tile_byte0 = 8 * (wb0 + plan.fword);
    const ScanPair fn = pick_scan<kR>(plan, fixed_offsets_fit(buffer_bytes, tile_byte0, n_tiles));
    if (!fn.count) return fail(PM_ERR_UNSUPPORTED, "counter levels out of range");

    ScanArgs a;
    a.text4 = reinterpret_cast<const uint4*>(text_dev);
    a.src.text4 = a.text4;
    a.src.image = reinterpret_cast<const uint4*>(image_dev);
    a.src.win_begin = win_begin;
    a.src.win_end = win_end;
    a.n4 = text_blocks(n) / 2;
    a.wb0 = wb0;
    a.win_begin = win_begin;
    a.win_end = win_end;
    a.pos = pos_dev;
    a.cnt = cnt_dev;
    a.capacity = capacity;
    a.n_hits = reinterpret_cast<unsigned long long*>(n_hits_dev);
    a.counts = reinterpret_cast<uint32_t*>(ws + lay.counts);
    a.range_sum = reinterpret_cast<unsigned long long*>(ws + lay.range_sum);
    a.staged = reinterpret_cast<unsigned long long*>(ws + lay.staged);
    a.n_tiles = (uint32_t)n_tiles;
    // interior tiles: the first whose first window is at or after win_begin,
    // up to the last whose windows all lie before win_end
    const uint64_t first_block = (win_begin + 31) >> 5, end_block = win_end >> 5;
    a.int_lo = (uint32_t)std::min<uint64_t>(n_tiles, (first_block - wb0 + tile_blocks - 1) / tile_blocks);
    a.int_hi = end_block >= wb0 ? (uint32_t)std::min<uint64_t>(n_tiles, (end_block - wb0) / tile_blocks) : 0u;
    // the fixed kernel's buffer loads (taken only when fixed_offsets_fit)
    a.text_bytes = (uint32_t)std::min<uint64_t>(buffer_bytes, 0xFFFFFFFFull);
    a.tile_byte0 = (uint32_t)std::min<uint64_t>(tile_byte0, 0xFFFFFFFFull);
    const unsigned grid = persistent_grid(fn.count, n_tiles);
    a.n_ranges = grid;

    HIP_TRY(pm::mark_begin(s));
    fn.count<<<grid, TPB, 0, s>>>(a, plan);
    HIP_TRY(hipGetLastError());
    HIP_TRY(pm::mark_end(s));
    fn.place<<<(unsigned)((n_tiles + 64 * (TPB / 64) - 1) / (64 * (TPB / 64))), TPB, 0, s>>>(a, plan);
    HIP_TRY(hipGetLastError());
    return PM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

pm_status pm_time_next_scan(void* ev_begin, void* ev_end) {
    if ((ev_begin == nullptr) != (ev_end == nullptr)) return fail(PM_ERR_ARG, "give both events or neither");
    pm::t_ev_begin = reinterpret_cast<hipEvent_t>(ev_begin);
    pm::t_ev_end = reinterpret_cast<hipEvent_t>(ev_end);
    return PM_OK;
}

const char* pm_status_string(pm_status s) {
    switch (s) {
        case PM_OK: return "PM_OK";
        case PM_ERR_ARG: return "PM_ERR_ARG";
        case PM_ERR_SYMBOL: return "PM_ERR_SYMBOL";
        case PM_ERR_HIP: return "PM_ERR_HIP";
        case PM_ERR_WORKSPACE: return "PM_ERR_WORKSPACE";
        case PM_ERR_UNSUPPORTED: return "PM_ERR_UNSUPPORTED";
        case PM_ERR_BUSY: return "PM_ERR_BUSY";
        case PM_ERR_NOT_FOUND: return "PM_ERR_NOT_FOUND";
        default: return "PM_ERR_UNKNOWN";
    }
}

const char* pm_last_error_detail(void) { return g_detail.c_str(); }

const char* pm_version(void) { return "pmscan 0.1 gfx950"; }

uint64_t pm_text_bytes(uint64_t n) { return 8 * text_blocks(n); }

pm_status pm_encode_text(const uint8_t* ascii_dev, uint64_t n, void* text_dev, uint64_t* bad_index_dev,
                         void* stream) {
    if (!text_dev || !bad_index_dev || (n > 0 && !ascii_dev)) return fail(PM_ERR_ARG, "null pointer");
    if (reinterpret_cast<uintptr_t>(text_dev) % 16 != 0)
        return fail(PM_ERR_ARG, "text_dev must be 16-byte aligned");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    pm_status st = fill_u64(bad_index_dev, ~0ull, 1, s);
    if (st != PM_OK) return st;
    const uint64_t nb = text_blocks(n);
    const unsigned grid = (unsigned)std::min<uint64_t>((nb + 255) / 256, 1u << 20);
    const int aligned = reinterpret_cast<uintptr_t>(ascii_dev) % 16 == 0;
    encode_text_kernel<<<grid, 256, 0, s>>>(ascii_dev, n, reinterpret_cast<uint2*>(text_dev), nb,
                                            reinterpret_cast<unsigned long long*>(bad_index_dev), aligned);
    HIP_TRY(hipGetLastError());
    return PM_OK;
}

pm_status pm_encode_pattern(const char* pattern, uint64_t len, uint8_t* codes, uint64_t cap,
                            uint32_t* m_out) {
    if ((!pattern && len) || !m_out) return fail(PM_ERR_ARG, "null pointer");
    std::vector<uint8_t> v;
    std::string err;
    if (pm::parse_pattern(pattern, len, v, err) != 0) return fail(PM_ERR_SYMBOL, err);
    if (v.size() > 0xFFFFFFFFull) return fail(PM_ERR_ARG, "pattern too long");
    *m_out = (uint32_t)v.size();
    if (codes) std::memcpy(codes, v.data(), std::min<uint64_t>(cap, v.size()));
    return PM_OK;
}

pm_status pm_pair_table(uint8_t table[64]) {
    if (!table) return fail(PM_ERR_ARG, "null pointer");
    for (unsigned p = 0; p < 16; ++p) {
        const unsigned mm = pm::mismatch_mask(p);
        for (unsigned t = 0; t < 4; ++t) table[(p << 2) | t] = (uint8_t)(mm >> t & 1u);
    }
    return PM_OK;
}

uint64_t pm_pattern_bytes(uint32_t m) { return 4 * pm::image_words(m); }

pm_status pm_pattern_image(const uint8_t* codes, uint32_t m, void* image_host, uint64_t bytes) {
    if (!codes || !image_host) return fail(PM_ERR_ARG, "null pointer");
    if (m == 0) return fail(PM_ERR_ARG, "empty pattern");
    if (bytes < pm_pattern_bytes(m)) return fail(PM_ERR_WORKSPACE, "image buffer too small");
    for (uint32_t j = 0; j < m; ++j)
        if (codes[j] > 15) return fail(PM_ERR_SYMBOL, "pattern code above 15 at " + std::to_string(j));
    pm::build_image(codes, m, reinterpret_cast<uint32_t*>(image_host));
    return PM_OK;
}

uint64_t pm_scan_workspace_bytes(uint64_t n) { return ws_layout(max_tiles(n)).bytes; }

pm_status pm_scan(const void* text_dev, uint64_t n, const uint8_t* codes, uint32_t m, uint32_t k,
                  const void* image_dev, uint64_t win_begin, uint64_t win_end, int64_t* pos_dev,
                  uint16_t* cnt_dev, uint64_t capacity, uint64_t* n_hits_dev, void* ws_dev,
                  uint64_t ws_bytes, void* stream) {
    if (!ws_dev) return fail(PM_ERR_ARG, "null pointer");
    if (ws_bytes < pm_scan_workspace_bytes(n)) return fail(PM_ERR_WORKSPACE, "workspace too small");
    return scan_launch(text_dev, n, codes, m, k, image_dev, win_begin, win_end, pos_dev, cnt_dev, capacity,
                       n_hits_dev, reinterpret_cast<uint8_t*>(ws_dev), ws_layout(max_tiles(n)), 0, stream);
}

uint64_t pm_scan_noalloc_max_windows(void) { return kStaticMaxWindows; }

pm_status pm_scan_noalloc(const void* text_dev, uint64_t n, const uint8_t* codes, uint32_t m, uint32_t k,
                          const void* image_dev, uint64_t win_begin, uint64_t win_end, int64_t* pos_dev,
                          uint16_t* cnt_dev, uint64_t capacity, uint64_t* n_hits_dev, void* stream) {
    // the size limit first: it needs no device
    const uint64_t nw = m <= n ? n - m + 1 : 0;
    const uint64_t end = std::min(win_end, nw);
    if (win_begin < end && end - win_begin > kStaticMaxWindows)
        return fail(PM_ERR_WORKSPACE, "window range of " + std::to_string(end - win_begin) +
                                          " windows exceeds the static scratch's " +
                                          std::to_string(kStaticMaxWindows) + " per call");
    uint8_t* scratch_dev = nullptr;
    if (const pm_status st = static_scratch(&scratch_dev); st != PM_OK) return st;
    // the layout is sized for the largest call; the tile count of this
    // call's window range is checked against it in scan_launch
    return scan_launch(text_dev, n, codes, m, k, image_dev, win_begin, win_end, pos_dev, cnt_dev, capacity,
                       n_hits_dev, scratch_dev, ws_layout(kStaticMaxTiles), kStaticMaxTiles, stream);
}

}  // extern "C"
