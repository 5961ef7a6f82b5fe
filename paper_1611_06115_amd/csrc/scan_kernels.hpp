// scan_kernels.hpp -- the scan's device kernels (private to libpmscan,
// included by pmscan.hip only): the count kernels (the filter and
// verification of every tile, Sect. 2.4 with the tiling of Sect. 2.6) and
// the kernel that places every tile's hits at its ordered offset.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"
#include "scan_core.hpp"

namespace pm {

constexpr int TPB = kThreads;

constexpr int kCap = 32;      // hits a tile stages for the placement kernel
constexpr uint32_t kMaxRanges = 16384;  // workgroups of a count-kernel grid (workspace holds one sum each)

struct ScanArgs {
    TileSrc src;               // text (16-byte groups), pattern image, window range
    const uint4* text4;        // = src.text4
    uint64_t n4;               // 16-byte groups in the buffer
    uint64_t wb0;              // first block of tile 0 (even)
    uint64_t win_begin, win_end;
    int64_t* pos;
    uint16_t* cnt;
    uint64_t capacity;
    unsigned long long* n_hits;
    uint32_t* counts;                // hits per tile
    unsigned long long* range_sum;   // hits per count-kernel workgroup (its range of tiles)
    unsigned long long* staged;      // kCap per tile: (window offset << 16) | count
    uint32_t n_tiles, n_ranges;
    // tiles [int_lo, int_hi) lie wholly inside [win_begin, win_end)
    uint32_t int_lo, int_hi;
    // the fixed kernel's loads: bytes of the text buffer, and the byte offset
    // of tile 0's first group (with the plan's filter window)
    uint32_t text_bytes, tile_byte0;
};

// The text a lane's filter needs: blocks B+fw .. B+fw+R+1 as 16-byte groups
// (B and fw are even).  Lanes past the end of the text read the last group.
template <int R>
__device__ __forceinline__ void load_text(const ScanArgs& a, const ScanPlan& p, uint64_t B,
                                          uint4 (&t)[(R + 2) / 2]) {
    const uint64_t g0 = (B + p.fword) >> 1;
#pragma unroll
    for (int u = 0; u < (R + 2) / 2; ++u) {
        uint64_t gi = g0 + u;
        if (gi >= a.n4) gi = a.n4 - 1;
        t[u] = a.text4[gi];
    }
}

// The same for a whole tile starting at block T0 (wave-uniform): a uniform
// base address plus the lane's offset; only a tile whose groups run past the
// buffer (the last ones) clamps its loads to the last group.
template <int R>
__device__ __forceinline__ void load_tile_text(const ScanArgs& a, const ScanPlan& p, uint64_t T0,
                                               uint4 (&t)[(R + 2) / 2]) {
    // a uniform base address plus the lane's byte offset, clamped (for the
    // last tiles) to the buffer's last group
    const uint32_t lane = threadIdx.x & 63u;
    // uniform; clamped, so that the loads of a tile past the end (issued
    // unconditionally by the fixed kernel) read the last group
    const uint64_t g0 = min((T0 + p.fword) >> 1, a.n4 - 1);
    const char* base = reinterpret_cast<const char*>(a.text4 + g0);
    const uint64_t room = 16 * (a.n4 - 1 - g0);
    const uint32_t lim = room < 0xFFFFFFF0ull ? (uint32_t)room : 0xFFFFFFF0u;
    const uint32_t off = lane * (uint32_t)(16 * (R / 2));
#pragma unroll
    for (int u = 0; u < (R + 2) / 2; ++u)
        t[u] = *reinterpret_cast<const uint4*>(base + min(off + (uint32_t)(16 * u), lim));
}

// Write the hits of this lane, in order, starting at output index `idx`.
template <int R, int L, bool EXH>
__device__ __forceinline__ void write_hits(const ScanArgs& a, const ScanPlan& p, const Counters<R, L>& C,
                                           const uint32_t (&hit)[R], uint64_t B, unsigned long long idx) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
        uint32_t h = hit[i];
        while (h) {
            const uint32_t b = __builtin_ctz(h);
            h &= h - 1u;
            if (idx < a.capacity) {
                const uint64_t pos = 32 * (B + i) + b;
                a.pos[idx] = (int64_t)pos;
                a.cnt[idx] = (uint16_t)hit_count<R, L, EXH>(a.src, p, C, i, b, pos);
            }
            ++idx;
        }
    }
}

// A tile is the 64 lanes of one wave, R lane words (32 windows) each.
__device__ __forceinline__ uint64_t tile_first_block(const ScanArgs& a, uint32_t tile, int R) {
    return a.wb0 + (uint64_t)tile * (uint64_t)(64 * R);
}

// Whether every window of the tile lies in [win_begin, win_end): a test of
// the tile index alone (uniform, two scalar compares).
__device__ __forceinline__ bool tile_interior(const ScanArgs& a, uint32_t tile) {
    return tile >= a.int_lo && tile < a.int_hi;
}

// The text of tile `tile` (uniform) through a buffer resource over the whole
// encoded text: each lane's byte offset is the tile's offset (scalar) plus
// its own, one vector add per tile; the resource's range check clamps in
// hardware (a load past the buffer returns zeros, like the zero padding
// after the text), so the last tiles need no clamping arithmetic.  Only for
// a buffer that 32-bit offsets cover (text_bytes; the launch takes the
// generic kernel otherwise).  The same (R+2)/2 loads on every path.
template <int R>
__device__ __forceinline__ void load_tile(const ScanArgs& a, const __amdgpu_buffer_rsrc_t& text, uint32_t tile,
                                          uint4 (&t)[(R + 2) / 2]) {
    const uint32_t at = a.tile_byte0 + tile * (uint32_t)(64 * R * 8);  // 64 R blocks of 8 bytes
    const uint32_t off = (threadIdx.x & 63u) * (uint32_t)(16 * (R / 2)) + at;
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int u = 0; u < (R + 2) / 2; ++u) {
        const v4u v = __builtin_amdgcn_raw_buffer_load_b128(text, off + 16u * u, 0, 0);
        t[u] = make_uint4(v.x, v.y, v.z, v.w);
    }
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t text_resource(const ScanArgs& a) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint4*>(a.text4), (short)0, (int)a.text_bytes, 0x00020000);
}

// The waves of a SIMD are issued oldest first, so with equal shares of tiles
// the oldest waves finish far ahead of the youngest (on the genome workload
// the first tenth of the waves ended at 45% of the launch) and the SIMDs then
// run short of waves for the rest of it.  A wave with more of its share left
// runs at a higher priority (more than 1/2, 1/5 or 1/16 left: 3, 2, 1, else
// 0): the waves of a SIMD stay close together to the end (about 13% less
// time on that workload).
// (left > share / d is left * d > share for integers, in 32-bit scalar
// compares: the 64-bit form would be vector compares.)
__device__ __forceinline__ void share_priority(uint32_t left, uint32_t share) {
    if (left > share / 2) __builtin_amdgcn_s_setprio(3);
    else if (left > share / 5) __builtin_amdgcn_s_setprio(2);
    else if (left > share / 16) __builtin_amdgcn_s_setprio(1);
    else __builtin_amdgcn_s_setprio(0);
}

// Exclusive prefix of `x` over the lanes of a wave; `total` gets the sum.
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

// The hits of one tile after its filter (hit[] and nh per lane; C holds the
// counters of an exhaustive filter): the tile's number of hits goes to
// counts[tile] and, when there are at most kCap, the hits themselves to the
// tile's staging slots, each as (window offset in the tile << 16 | count).
// vh/nvh: the hits the wave-wide verification kept.  Returns the tile's
// total.
// With STORE_COUNT false the caller stores the count.
template <int R, int L, bool EXH, bool STORE_COUNT = true>
__device__ __forceinline__ uint32_t stage_tile(const ScanArgs& a, const ScanPlan& p, uint32_t tile, uint64_t T0,
                                               uint64_t B, const Counters<R, L>& C, uint32_t (&hit)[R], uint32_t nh,
                                               uint32_t nvh, const unsigned long long* vh) {
    const uint32_t lane = threadIdx.x & 63u;
    if (__ballot(nh != 0) == 0) {  // the usual case: no hits in the tile
        if (STORE_COUNT && lane == 0) a.counts[tile] = 0;
        return 0;
    }
    uint32_t total;
    const uint32_t excl = wave_exclusive(nh, total);
    if (STORE_COUNT && lane == 0) a.counts[tile] = total;
    if (total > (uint32_t)kCap) return total;
    const uint64_t base = 32 * T0;
    if (!EXH && p.nchunks > kWaveVerifyChunks) {
        unsigned long long* out = a.staged + (uint64_t)tile * kCap;
        if (nvh == total && total <= kWaveHits) {
            // every hit was counted by the whole wave and kept, in order
            if (lane < total) {
                const unsigned long long v = vh[lane];
                out[lane] = (((v >> 16) - base) << 16) | (v & 0xFFFFu);
            }
            return total;
        }
        // otherwise: the hits in position order (the staging order), each
        // counted by the whole wave and written by its lane
        for (uint32_t j = 0;; ++j) {
            uint32_t mine = 0;
#pragma unroll
            for (int i = 0; i < R; ++i) mine |= hit[i];
            const uint64_t bal = __ballot(mine != 0);
            if (bal == 0) break;
            const uint32_t owner = (uint32_t)__builtin_ctzll(bal);
            int fi = 0;
            uint32_t fb = 0;
#pragma unroll
            for (int i = R - 1; i >= 0; --i)
                if (hit[i]) {
                    fi = i;
                    fb = __builtin_ctz(hit[i]);
                }
            const uint64_t mine_pos = 32 * (B + (uint64_t)fi) + fb;
            const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)mine_pos, owner);
            const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(mine_pos >> 32), owner);
            const uint64_t pos = ((uint64_t)hi << 32) | lo;
            const uint32_t c = count_window_wave(a.src.text4, a.src.image, p.nchunks, pos, p.k, lane);
            if (lane == owner) {
                out[j] = ((pos - base) << 16) | c;
#pragma unroll
                for (int i = 0; i < R; ++i)
                    if (i == fi) hit[i] &= hit[i] - 1u;
            }
        }
        return total;
    }
    if (nh == 0) return total;
    unsigned long long* out = a.staged + (uint64_t)tile * kCap + excl;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        uint32_t h = hit[i];
        while (h) {
            const uint32_t b = __builtin_ctz(h);
            h &= h - 1u;
            const uint64_t pos = 32 * (B + i) + b;
            const uint32_t c = hit_count<R, L, EXH>(a.src, p, C, i, b, pos);
            *out++ = ((pos - base) << 16) | c;
        }
    }
    return total;
}

// The workgroup's total hits: one sum per range of tiles.
__device__ __forceinline__ void store_range_sum(const ScanArgs& a, uint32_t sum) {
    __shared__ uint32_t s_sum[TPB / 64];
    if ((threadIdx.x & 63u) == 0) s_sum[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
#pragma unroll
        for (int i = 0; i < TPB / 64; ++i) t += s_sum[i];
        a.range_sum[blockIdx.x] = t;
    }
}

// Pass 1: every tile (one wave's windows) finds its hits, stores their number,
// and stages them when there are at most kCap.  Waves are persistent and
// independent: each workgroup takes a contiguous range of tiles, its waves
// take every 4th tile of it in order, and the workgroup stores the total hit
// count of its range.  This kernel takes any plan (the filter loop reads the
// plan's slots); scan_fixed_kernel below is the faster form for the common
// plan shape.
// With 4 lane words and up to 3 counter levels the kernel is held to 5 waves
// per SIMD (its registers fit; measured faster than 4 waves); other shapes
// keep the compiler's choice.
template <int R, int L, bool EXH>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(R == 4 && L <= 3 ? 5 : 1)))
void scan_count_kernel(ScanArgs a, ScanPlan p) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform
    // workgroup b takes tiles [b T / G, (b+1) T / G) of the G in the grid;
    // its waves interleave in that range
    constexpr uint32_t kStep = TPB / 64;
    const uint32_t t_end = (uint32_t)((uint64_t)(blockIdx.x + 1) * a.n_tiles / gridDim.x);
    uint32_t tile = (uint32_t)((uint64_t)blockIdx.x * a.n_tiles / gridDim.x) + wv;
    uint32_t sum = 0;
    __shared__ unsigned long long s_vh[TPB / 64][kWaveHits];  // hits kept by tile_filter, per wave
    // the text of the wave's next tile is loaded while this one is computed
    uint4 nxt[(R + 2) / 2];
    if (tile < t_end) load_tile_text<R>(a, p, tile_first_block(a, tile, R), nxt);
    const uint32_t share = tile < t_end ? (t_end - tile + kStep - 1) / kStep : 0u;
    __builtin_amdgcn_s_setprio(3);
    for (uint32_t done = 0; tile < t_end; tile += kStep) {
        share_priority(share - done++, share);
        const uint64_t T0 = tile_first_block(a, tile, R);
        const uint64_t B = T0 + (uint64_t)lane * R;
        uint4 txt[(R + 2) / 2];
#pragma unroll
        for (int u = 0; u < (R + 2) / 2; ++u) txt[u] = nxt[u];
        if (tile + kStep < t_end) load_tile_text<R>(a, p, tile_first_block(a, tile + kStep, R), nxt);
        // keep those loads here, ahead of the filter (the scheduler would
        // otherwise sink them below it, next to their use)
        __builtin_amdgcn_sched_barrier(0);
        Counters<R, L> C;
        uint32_t hit[R], nh;
        Lane<R> s;
        make_lane<R>(txt, EXH || p.n_slots == 0 ? 0u : p.singles, s);
        uint32_t nvh = 0;
        tile_filter<R, L, EXH, true>(a.src, p, B, tile_interior(a, tile), s, C, hit, nh, s_vh[wv], &nvh);
        sum += stage_tile<R, L, EXH>(a, p, tile, T0, B, C, hit, nh, nvh, s_vh[wv]);
    }
    store_range_sum(a, sum);
}

// The same pass for a plan of NG groups of two full singleton sets (the
// planner's usual shape), with the unrolled fixed_filter.  A tile's text goes
// to the LDS planes first; its register buffer is then reloaded with the
// wave's next tile while the filter runs.  One buffer and a filter that
// counts PM_FIXED_RW lane words at a time keep the kernel at 80 registers,
// so that six waves share a SIMD: the other waves' filters cover the load
// latency (with five waves and two buffers in flight the scan is about 7%
// slower).
#ifndef PM_FIXED_WAVES
#define PM_FIXED_WAVES 6
#endif
// lane words the filter counts at a time
#ifndef PM_FIXED_RW
#define PM_FIXED_RW 2
#endif
// s_waitcnt with only the vector-memory count at zero (gfx9 encoding:
// expcnt and lgkmcnt at their maxima).
#define PM_WAIT_VMEM() __builtin_amdgcn_s_waitcnt(0x0F70)

template <int R, int L, int NG>
__device__ __forceinline__ uint32_t fixed_tile(const ScanArgs& a, const ScanPlan& p, const __amdgpu_buffer_rsrc_t& text,
                                               uint32_t tile, uint4 (&buf)[(R + 2) / 2], uint32_t* planes,
                                               const uint32_t* const (&rows0)[2 * NG], unsigned long long* vh) {
    constexpr uint32_t kStep = TPB / 64;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t T0 = tile_first_block(a, tile, R);
    store_planes<R>(buf, p.singles, planes);
    // unconditional (a tile past the end reads the text's last group, never
    // used), so that the number of loads in flight is the same on every path
    load_tile<R>(a, text, tile + kStep, buf);
    // keep those loads here, ahead of the filter
    __builtin_amdgcn_sched_barrier(0);
    // the slot words, read again for every tile: kept as loop invariants
    // they would hold 20 more scalar registers for the whole loop
    uint32_t sw[2 * NG];
#pragma unroll
    for (int g = 0; g < 2 * NG; ++g) {
        uint32_t w = p.slot[g];
        asm volatile("" : "+s"(w));
        sw[g] = w;
    }
    // the lane's row of each set's plane words: the loop invariants rows0 for
    // up to two groups (four vector registers), formed again for every tile
    // for more (their registers would cost the sixth wave)
    const uint32_t* rows[2 * NG];
#pragma unroll
    for (int g = 0; g < 2 * NG; ++g) rows[g] = NG <= 2 ? rows0[g] : set_row<R + 2>(planes, sw[g]);
    uint32_t dead[R];
    fixed_filter<R, L, NG, PM_FIXED_RW>(rows, sw, p.init, dead);
    // (the lane's first lane word B is formed only on the two rare paths,
    // from an opaque copy of the lane index each, so that the compiler does
    // not hoist it into every tile)
    if (!tile_interior(a, tile)) {
        uint32_t l = lane;
        asm volatile("" : "+v"(l));
        uint32_t valid[R];
        valid_windows<R>(a.src, T0 + (uint64_t)l * R, valid);
#pragma unroll
        for (int i = 0; i < R; ++i) dead[i] |= ~valid[i];
    }
    uint32_t any = 0;
#pragma unroll
    for (int i = 0; i < R; ++i) any |= ~dead[i];
    if (__ballot(any != 0) == 0) return 0;  // the usual case: no survivor in the tile
    uint32_t l = lane;
    asm volatile("" : "+v"(l));
    const uint64_t B = T0 + (uint64_t)l * R;
    uint32_t hit[R], nh, nvh = 0;
    verify_survivors<R, true>(a.src, p, B, dead, hit, nh, vh, &nvh);
    Counters<R, L> C;  // not read: the fixed filter is never exhaustive
    const uint32_t total = stage_tile<R, L, false, false>(a, p, tile, T0, B, C, hit, nh, nvh, vh);
    // this path's loads and stores are complete before the loop goes on,
    // so that the common path's waits stay exact
    PM_WAIT_VMEM();
    return total;
}

template <int R, int L, int NG>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(PM_FIXED_WAVES)))
void scan_fixed_kernel(ScanArgs a, ScanPlan p) {
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform
    constexpr uint32_t kStep = TPB / 64;
    const uint32_t t_end = (uint32_t)((uint64_t)(blockIdx.x + 1) * a.n_tiles / gridDim.x);
    uint32_t tile = (uint32_t)((uint64_t)blockIdx.x * a.n_tiles / gridDim.x) + wv;
    uint32_t sum = 0;
    __shared__ unsigned long long s_vh[TPB / 64][kWaveHits];
    // mismatch planes of the fixed filter, one region per wave
    __shared__ uint32_t s_planes[TPB / 64][4 * (R + 2) * 64];
    const __amdgpu_buffer_rsrc_t text = text_resource(a);
    const uint32_t* rows0[2 * NG];  // used for NG <= 2 (fixed_tile)
#pragma unroll
    for (int g = 0; g < 2 * NG; ++g) rows0[g] = NG <= 2 ? set_row<R + 2>(s_planes[wv], p.slot[g]) : nullptr;
    uint4 buf[(R + 2) / 2];
    load_tile<R>(a, text, tile, buf);
    // per-tile hit counts are gathered in a register across 64 tiles (lane j
    // holds the j-th) and stored together: a store in every iteration would
    // leave loads and stores in flight together, and then the wait for the
    // text would also wait for the store
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t pend = 0, k = 0, batch = tile;
    auto keep = [&](uint32_t total) {
        if (lane == k) pend = total;
        if (++k == 64) {
            a.counts[batch + kStep * lane] = pend;
            PM_WAIT_VMEM();
            batch += 64 * kStep;
            k = 0;
        }
    };
    const uint32_t share = tile < t_end ? (t_end - tile + kStep - 1) / kStep : 0u;
    __builtin_amdgcn_s_setprio(3);
    for (uint32_t done = 0; tile < t_end; tile += kStep) {
        share_priority(share - done++, share);
        const uint32_t total = fixed_tile<R, L, NG>(a, p, text, tile, buf, s_planes[wv], rows0, s_vh[wv]);
        sum += total;
        keep(total);
    }
    if (lane < k) a.counts[batch + kStep * lane] = pend;
    store_range_sum(a, sum);
}

// Wave sum of x[first .. last) (all 64 lanes of one wave call it).
template <typename T>
__device__ __forceinline__ unsigned long long wave_sum(const T* x, uint64_t first, uint64_t last) {
    const uint32_t lane = threadIdx.x & 63u;
    // 16 loads per lane in flight per round (1024 values): a busy segment's
    // prefix over the range totals (up to a few thousand) takes one or two
    // load round trips, which set the place kernel's time
    constexpr int kV = 16;
    unsigned long long v = 0;
    for (uint64_t i0 = first; i0 < last; i0 += 64 * kV) {
        T t[kV];
#pragma unroll
        for (int j = 0; j < kV; ++j) {
            const uint64_t i = i0 + (uint64_t)j * 64 + lane;
            t[j] = i < last ? x[i] : T(0);
        }
#pragma unroll
        for (int j = 0; j < kV; ++j) v += t[j];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Pass 3: each wave takes 64 consecutive tiles and ranks their hit counts;
// every tile with hits then has them placed at its ordered offset -- copied
// from the staging area, or, for a tile with more than kCap hits, found again
// by the wave and written directly.  Waves of segments without hits return
// after one load.
template <int R, int L, bool EXH>
__global__ __launch_bounds__(TPB) void scan_place_kernel(ScanArgs a, ScanPlan p) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t seg = (uint64_t)blockIdx.x * (TPB / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t t0 = seg * 64;
    if (seg == 0) {
        const unsigned long long all = wave_sum(a.range_sum, 0, a.n_ranges);
        if (lane == 0) *a.n_hits = all;
    }
    if (t0 >= a.n_tiles) return;
    const uint32_t count = t0 + lane < a.n_tiles ? a.counts[t0 + lane] : 0u;
    unsigned long long busy = __ballot(count != 0);
    if (busy == 0) return;
    // hits before tile t0: the ranges of the count kernel's workgroups before
    // the one that owns t0 (the last whose range starts at or before t0), then
    // that range's tiles before t0
    const uint32_t G = a.n_ranges;
    uint32_t b0 = (uint32_t)(t0 * G / a.n_tiles);
    while (b0 + 1 < G && (uint64_t)(b0 + 1) * a.n_tiles / G <= t0) ++b0;
    const uint64_t s0 = (uint64_t)b0 * a.n_tiles / G;
    const unsigned long long base = wave_sum(a.range_sum, 0, b0) + wave_sum(a.counts, s0, t0);
    unsigned long long incl = count;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long v = __shfl_up(incl, d, 64);
        if (lane >= (uint32_t)d) incl += v;
    }
    const unsigned long long first = base + incl - count;  // output index of this lane's tile
    while (busy) {
        const uint32_t l = __builtin_ctzll(busy);
        busy &= busy - 1ull;
        const uint32_t cl = __shfl(count, (int)l, 64);
        const unsigned long long pl = __shfl(first, (int)l, 64);
        if (pl >= a.capacity) break;  // later tiles start even later
        const uint32_t tile = (uint32_t)(t0 + l);
        const uint64_t T0 = tile_first_block(a, tile, R);
        if (cl <= (uint32_t)kCap) {
            const unsigned long long* src = a.staged + (uint64_t)tile * kCap;
            for (uint32_t i = lane; i < cl; i += 64) {
                const unsigned long long v = src[i];
                const unsigned long long dst = pl + i;
                if (dst < a.capacity) {
                    a.pos[dst] = (int64_t)(32 * T0 + (v >> 16));
                    a.cnt[dst] = (uint16_t)(v & 0xFFFFu);
                }
            }
        } else {
            const uint64_t B = T0 + (uint64_t)lane * R;
            uint4 txt[(R + 2) / 2];
            load_text<R>(a, p, B, txt);
            Counters<R, L> C;
            uint32_t hit[R], nh;
            Lane<R> s;
            make_lane<R>(txt, EXH || p.n_slots == 0 ? 0u : p.singles, s);
            tile_filter<R, L, EXH, true>(a.src, p, B, tile_interior(a, tile), s, C, hit, nh);
            uint32_t total;
            const uint32_t excl = wave_exclusive(nh, total);
            if (nh) write_hits<R, L, EXH>(a, p, C, hit, B, pl + excl);
        }
    }
}

}  // namespace pm
