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
//   3. output: hits are compacted in position order with a workgroup prefix
//      sum, and tiles are chained in order by a decoupled look-back over a
//      per-tile status word, so the output list is ascending without a sort.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pmscan.h"
#include "plan.hpp"

using pm::ScanPlan;

namespace {

constexpr int TPB = pm::kThreads;
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
// scan
// ---------------------------------------------------------------------------

struct ScanArgs {
    const uint4* text4;        // encoded text as 16-byte groups (two blocks each)
    uint64_t n4;               // 16-byte groups in the buffer
    uint64_t wb0;              // first block of tile 0 (even)
    uint64_t win_begin, win_end;
    const uint4* image;        // pattern image, one uint4 (A,C,G,T planes) per chunk
    int64_t* pos;
    uint16_t* cnt;
    uint64_t capacity;
    unsigned long long* n_hits;
    unsigned long long* status;  // per-tile look-back words
    uint32_t* tile_counter;
    uint32_t n_tiles;
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
    uint32_t h[R + 2], l[R + 2];           // raw planes of blocks B+fw .. B+fw+R+1
    uint32_t pa[R + 2], pc[R + 2], pg[R + 2], pt[R + 2];  // singleton mismatch planes
};

// Mismatch words X[i] (lane word i) of one filter slot: position offset
// 32*Q + r from the filter window start, Table 3 row MM.
template <unsigned MM, int Q, int R>
__device__ __forceinline__ void slot_words(const Lane<R>& s, uint32_t r, uint32_t (&X)[R]) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
        if constexpr (MM == 14u) X[i] = align(s.pa[i + Q + 1], s.pa[i + Q], r);
        else if constexpr (MM == 13u) X[i] = align(s.pc[i + Q + 1], s.pc[i + Q], r);
        else if constexpr (MM == 11u) X[i] = align(s.pg[i + Q + 1], s.pg[i + Q], r);
        else if constexpr (MM == 7u) X[i] = align(s.pt[i + Q + 1], s.pt[i + Q], r);
        else if constexpr (MM == 12u) X[i] = align(s.h[i + Q + 1], s.h[i + Q], r);  // [AC]
        else if constexpr (MM == 10u) X[i] = align(s.l[i + Q + 1], s.l[i + Q], r);  // [AG]
        else {
            const uint32_t H = align(s.h[i + Q + 1], s.h[i + Q], r);
            const uint32_t L = align(s.l[i + Q + 1], s.l[i + Q], r);
            X[i] = mismatch_fn<MM>(H, L);
        }
    }
}

template <int R>
__device__ __forceinline__ void slot_dispatch(uint32_t slot, const Lane<R>& s, uint32_t (&X)[R]) {
    const uint32_t r = slot >> 5;
    switch (slot & 31u) {
#define PM_CASE(MM)                                  \
    case MM: slot_words<MM, 0, R>(s, r, X); break;   \
    case MM + 16: slot_words<MM, 1, R>(s, r, X); break;
        PM_CASE(1) PM_CASE(2) PM_CASE(3) PM_CASE(4) PM_CASE(5) PM_CASE(6) PM_CASE(7)
        PM_CASE(8) PM_CASE(9) PM_CASE(10) PM_CASE(11) PM_CASE(12) PM_CASE(13) PM_CASE(14)
#undef PM_CASE
        default:
#pragma unroll
            for (int i = 0; i < R; ++i) X[i] = 0u;
            break;
    }
}

__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) {
    return (a & b) | (a & c) | (b & c);
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
        for (int i = 0; i < R; ++i) c.dead[i] |= a[i] | b[i];
    } else if constexpr (LV < L) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const uint32_t s = c.S[LV][i];
            c.S[LV][i] = s ^ a[i] ^ b[i];
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
// the count exceeds `limit`.
__device__ uint32_t count_window(const uint4* __restrict__ text4, const uint4* __restrict__ image,
                                 uint32_t nchunks, uint64_t s, uint32_t limit) {
    const uint2* text = reinterpret_cast<const uint2*>(text4);
    const uint64_t q = s >> 5;
    const uint32_t r = (uint32_t)s & 31u;
    uint2 w0 = text[q];
    uint32_t cnt = 0;
    for (uint32_t c = 0; c < nchunks; ++c) {
        const uint2 w1 = text[q + c + 1];
        const uint32_t H = align(w1.x, w0.x, r), Lo = align(w1.y, w0.y, r);
        const uint4 mp = image[c];
        const uint32_t mis = (~H & ~Lo & mp.x) | (~H & Lo & mp.y) | (H & ~Lo & mp.z) | (H & Lo & mp.w);
        cnt += __builtin_popcount(mis);
        if (cnt > limit) break;
        w0 = w1;
    }
    return cnt;
}

template <int R, int L>
__global__ __launch_bounds__(TPB) void scan_kernel(ScanArgs a, ScanPlan p) {
    __shared__ uint32_t s_tile;
    __shared__ uint32_t s_wave_sum[TPB / 64];
    __shared__ unsigned long long s_base;

    if (threadIdx.x == 0) s_tile = atomicAdd(a.tile_counter, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint64_t B = a.wb0 + (uint64_t)tile * (TPB * R) + (uint64_t)threadIdx.x * R;

    // ---- valid windows of each lane word ------------------------------------
    Counters<R, L> C;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const uint64_t w0 = 32 * (B + i);
        uint32_t valid = 0;
        if (w0 < a.win_end && w0 + 32 > a.win_begin) {
            const uint32_t lo = a.win_begin > w0 ? (uint32_t)(a.win_begin - w0) : 0u;
            const uint32_t hi = a.win_end < w0 + 32 ? (uint32_t)(a.win_end - w0) : 32u;
            valid = (hi == 32u ? ~0u : ((1u << hi) - 1u)) & ~((1u << lo) - 1u);
        }
        C.dead[i] = ~valid;
        if constexpr (L > 0) {
#pragma unroll
            for (int l = 0; l < L; ++l) C.S[l][i] = (p.init >> l & 1u) ? ~0u : 0u;
        }
    }

    // ---- filter ---------------------------------------------------------------
    if (p.n_slots > 0) {
        Lane<R> s;
        const uint64_t g0 = (B + p.fword) >> 1;
#pragma unroll
        for (int u = 0; u < (R + 2) / 2; ++u) {
            uint64_t gi = g0 + u;
            if (gi >= a.n4) gi = a.n4 - 1;  // lanes past the text: values unused
            const uint4 v = a.text4[gi];
            s.h[2 * u] = v.x;
            s.l[2 * u] = v.y;
            s.h[2 * u + 1] = v.z;
            s.l[2 * u + 1] = v.w;
        }
        if (p.singles & 1u) {
#pragma unroll
            for (int w = 0; w < R + 2; ++w) s.pa[w] = mismatch_fn<14u>(s.h[w], s.l[w]);
        }
        if (p.singles & 2u) {
#pragma unroll
            for (int w = 0; w < R + 2; ++w) s.pc[w] = mismatch_fn<13u>(s.h[w], s.l[w]);
        }
        if (p.singles & 4u) {
#pragma unroll
            for (int w = 0; w < R + 2; ++w) s.pg[w] = mismatch_fn<11u>(s.h[w], s.l[w]);
        }
        if (p.singles & 8u) {
#pragma unroll
            for (int w = 0; w < R + 2; ++w) s.pt[w] = mismatch_fn<7u>(s.h[w], s.l[w]);
        }

        for (uint32_t g = 0; g < p.n_slots; g += 8) {
            uint32_t xa[R], xb[R], c0a[R], c0b[R], c1a[R], c1b[R], c2[R];
#pragma unroll
            for (int half = 0; half < 2; ++half) {
#pragma unroll
                for (int pr = 0; pr < 2; ++pr) {
                    const int u = 4 * half + 2 * pr;
                    slot_dispatch<R>(p.slot[g + u], s, xa);
                    slot_dispatch<R>(p.slot[g + u + 1], s, xb);
                    if constexpr (L == 0) {
#pragma unroll
                        for (int i = 0; i < R; ++i) C.dead[i] |= xa[i] | xb[i];
                    } else {
                        add2<0, R, L>(C, xa, xb, pr == 0 ? c0a : c0b);
                    }
                }
                add2<1, R, L>(C, c0a, c0b, half == 0 ? c1a : c1b);
            }
            add2<2, R, L>(C, c1a, c1b, c2);
            if constexpr (L >= 3) add1<3, R, L>(C, c2);
        }
    }

    // ---- survivors -> hits -----------------------------------------------------
    uint32_t hit[R];
    uint32_t nh = 0;
    if (p.exhaustive) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            hit[i] = ~C.dead[i];
            nh += __builtin_popcount(hit[i]);
        }
    } else {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            uint32_t alive = ~C.dead[i];
            uint32_t h = 0;
            while (alive) {
                const uint32_t b = __builtin_ctz(alive);
                alive &= alive - 1u;
                const uint32_t c = count_window(a.text4, a.image, p.nchunks, 32 * (B + i) + b, p.k);
                if (c <= p.k) h |= 1u << b;
            }
            hit[i] = h;
            nh += __builtin_popcount(h);
        }
    }

    // ---- ordered compaction: workgroup scan + decoupled look-back ---------------
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    uint32_t incl = nh;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t v = __shfl_up(incl, d, 64);
        if (lane >= (uint32_t)d) incl += v;
    }
    if (lane == 63) s_wave_sum[wave] = incl;
    __syncthreads();
    uint32_t wave_off = 0, total = 0;
#pragma unroll
    for (int w = 0; w < TPB / 64; ++w) {
        const uint32_t v = s_wave_sum[w];
        if ((uint32_t)w < wave) wave_off += v;
        total += v;
    }
    if (threadIdx.x == 0) {
        unsigned long long excl = 0;
        if (tile == 0) {
            __hip_atomic_store(&a.status[0], ((unsigned long long)total << 2) | 2ull, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&a.status[tile], ((unsigned long long)total << 2) | 1ull,
                               __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            // Every tile publishes its own total before looking back, and tiles
            // with smaller ids started earlier, so each wait below ends.
            uint32_t j = tile - 1;
            while (true) {
                const unsigned long long v =
                    __hip_atomic_load(&a.status[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned flag = (unsigned)(v & 3ull);
                if (flag == 0) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += v >> 2;
                if (flag == 2) break;
                --j;
            }
            __hip_atomic_store(&a.status[tile], ((excl + total) << 2) | 2ull, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        if (tile == a.n_tiles - 1) *a.n_hits = excl + total;
        s_base = excl;
    }
    __syncthreads();
    if (nh == 0) return;
    unsigned long long idx = s_base + wave_off + (incl - nh);
#pragma unroll
    for (int i = 0; i < R; ++i) {
        uint32_t h = hit[i];
        while (h) {
            const uint32_t b = __builtin_ctz(h);
            h &= h - 1u;
            if (idx < a.capacity) {
                const uint64_t pos = 32 * (B + i) + b;
                uint32_t c;
                if (p.exhaustive) {
                    uint32_t v = 0;
                    if constexpr (L > 0) {
#pragma unroll
                        for (int l = 0; l < L; ++l) v |= (C.S[l][i] >> b & 1u) << l;
                    }
                    c = v - p.init + p.n_dash;
                } else {
                    c = count_window(a.text4, a.image, p.nchunks, pos, p.k);
                }
                a.pos[idx] = (int64_t)pos;
                a.cnt[idx] = (uint16_t)c;
            }
            ++idx;
        }
    }
}

constexpr int kR = 8;  // lane words per lane

using ScanFn = void (*)(ScanArgs, ScanPlan);
template <int R>
ScanFn pick_scan(uint32_t L) {
    switch (L) {
        case 0: return scan_kernel<R, 0>;
        case 1: return scan_kernel<R, 1>;
        case 2: return scan_kernel<R, 2>;
        case 3: return scan_kernel<R, 3>;
        case 4: return scan_kernel<R, 4>;
        case 5: return scan_kernel<R, 5>;
        case 6: return scan_kernel<R, 6>;
        default: return nullptr;
    }
}

// blocks of an encoded text buffer: the text, then zero padding, rounded to
// an even count so the buffer is a whole number of 16-byte groups
uint64_t text_blocks(uint64_t n) { return ((n + 31) / 32 + kPadBlocks + 1) & ~1ull; }

uint64_t max_tiles(uint64_t n) {
    // tiles of TPB*kR blocks, starting at an even block at or below win_begin
    const uint64_t blocks = (n + 31) / 32 + 2;
    return (blocks + (uint64_t)TPB * kR - 1) / ((uint64_t)TPB * kR) + 1;
}

constexpr uint64_t kWsHeader = 256;

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

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

uint64_t pm_scan_workspace_bytes(uint64_t n) { return kWsHeader + 8 * max_tiles(n); }

pm_status pm_scan(const void* text_dev, uint64_t n, const uint8_t* codes, uint32_t m, uint32_t k,
                  const void* image_dev, uint64_t win_begin, uint64_t win_end, int64_t* pos_dev,
                  uint16_t* cnt_dev, uint64_t capacity, uint64_t* n_hits_dev, void* ws_dev,
                  uint64_t ws_bytes, void* stream) {
    if (!text_dev || !codes || !image_dev || !n_hits_dev || !ws_dev)
        return fail(PM_ERR_ARG, "null pointer");
    if (capacity > 0 && (!pos_dev || !cnt_dev)) return fail(PM_ERR_ARG, "null output with capacity > 0");
    if (m == 0) return fail(PM_ERR_ARG, "empty pattern (m = 0)");
    if (k > 65535) return fail(PM_ERR_ARG, "k above 65535 (counts are 16-bit)");
    if (reinterpret_cast<uintptr_t>(text_dev) % 16 != 0)
        return fail(PM_ERR_ARG, "text_dev must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(image_dev) % 16 != 0)
        return fail(PM_ERR_ARG, "image_dev must be 16-byte aligned");
    if (ws_bytes < pm_scan_workspace_bytes(n)) return fail(PM_ERR_WORKSPACE, "workspace too small");
    for (uint32_t j = 0; j < m; ++j)
        if (codes[j] > 15) return fail(PM_ERR_SYMBOL, "pattern code above 15 at " + std::to_string(j));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    const uint64_t nw = m <= n ? n - m + 1 : 0;
    if (win_end > nw) win_end = nw;
    const ScanPlan plan = pm::build_plan(codes, m, k);
    if (win_begin >= win_end || plan.keff < 0) return fill_u64(n_hits_dev, 0, 1, s);

    const uint64_t wb0 = (win_begin >> 5) & ~1ull;
    const uint64_t wb_end = (win_end + 31) >> 5;
    const uint64_t tile_blocks = (uint64_t)TPB * kR;
    const uint64_t n_tiles = (wb_end - wb0 + tile_blocks - 1) / tile_blocks;
    if (n_tiles > max_tiles(n) || n_tiles > 0xFFFFFFFFull) return fail(PM_ERR_ARG, "window range too large");

    ScanFn fn = pick_scan<kR>(plan.levels);
    if (!fn) return fail(PM_ERR_UNSUPPORTED, "counter levels out of range");

    uint8_t* ws = reinterpret_cast<uint8_t*>(ws_dev);
    ScanArgs a;
    a.text4 = reinterpret_cast<const uint4*>(text_dev);
    a.n4 = text_blocks(n) / 2;
    a.wb0 = wb0;
    a.win_begin = win_begin;
    a.win_end = win_end;
    a.image = reinterpret_cast<const uint4*>(image_dev);
    a.pos = pos_dev;
    a.cnt = cnt_dev;
    a.capacity = capacity;
    a.n_hits = reinterpret_cast<unsigned long long*>(n_hits_dev);
    a.tile_counter = reinterpret_cast<uint32_t*>(ws);
    a.status = reinterpret_cast<unsigned long long*>(ws + kWsHeader);
    a.n_tiles = (uint32_t)n_tiles;

    // counter word + status words start at zero
    {
        pm_status st = fill_u64(reinterpret_cast<uint64_t*>(ws), 0, 1, s);
        if (st != PM_OK) return st;
        st = fill_u64(reinterpret_cast<uint64_t*>(a.status), 0, n_tiles, s);
        if (st != PM_OK) return st;
    }
    fn<<<(unsigned)n_tiles, TPB, 0, s>>>(a, plan);
    HIP_TRY(hipGetLastError());
    return PM_OK;
}

}  // extern "C"
