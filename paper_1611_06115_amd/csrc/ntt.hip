// ntt.hip -- the Linhart-Shamir route of Sect. 1.3 (eqs. 1-3) (libpmscan).
//
// Linhart and Shamir code a text base b as e_b = M / k_b and a class S as
// the CRT solution n_S of eq. (1) (0 modulo the primes of its members, 1
// modulo the others), with primes k_b above m and M their product; window i
// matches exactly iff the correlation C_i = sum_j n_{S_j} e_{t[i+j]} is 0
// modulo M (eq. 3).  C_i itself outgrows 64 bits for long patterns (Sect.
// 1.3.5), so here it is carried as its residues modulo the four primes.
// Modulo k_b, n_S is [b not in S], and e_{b'} is 0 for b' != b and g_b =
// M / k_b mod k_b for b' = b, so C_i mod k_b = g_b N_b(i) mod k_b, where
// N_b(i) counts the positions j with t[i+j] = b outside S_j.  Since
// N_b(i) <= m < k_b, that residue is 0 iff N_b(i) is, and decoding it (times
// the inverse of g_b) gives N_b(i) back; the window's mismatch count is
// c_i = sum_b N_b(i), the sum of eq. (4).
//
// Each N_b is a correlation of two 0/1 sequences, computed exactly with a
// number-theoretic transform modulo P = 119 * 2^23 + 1 (every value stays
// below m < P).  The text is cut into blocks of L bases (a power of two,
// L >= 2m) that overlap by m-1 (overlap-save).  Per block the four base
// indicator sequences are transformed, multiplied by the transforms of the
// pattern's four reversed indicator sequences and summed over b (the decoded
// residues, summed in the frequency domain), and one inverse transform gives
// c_i for the block's L-m+1 windows.  Forward transforms are decimation in
// frequency (natural order in, bit-reversed out) and the inverse is
// decimation in time (bit-reversed in, natural out), so no permutation pass
// is needed.  Every window's count comes out whatever k is: the cost is
// O(n log L), against the early-stop scan's ~O(n (k+1)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pmscan.h"
#include "plan.hpp"

namespace pm {
pm_status set_error(pm_status s, const std::string& what);
}

namespace {

constexpr uint32_t kP = 998244353u;  // 119 * 2^23 + 1
constexpr uint32_t kRoot = 3;        // a primitive root modulo kP
constexpr uint32_t kMaxLogL = 23;    // 2^23 divides kP - 1
constexpr uint32_t kMinLogL = 11;
constexpr uint32_t kBlockLogL = 20;  // block length for long texts
constexpr uint32_t kMaxM = 1u << (kMaxLogL - 1);
constexpr unsigned kTPB = 256;
// The innermost stages (butterflies within kLdsN consecutive elements) run in
// LDS: one workgroup of kLdsN / 4 threads per chunk, four elements per
// thread, instead of one pass over the whole array per stage.
constexpr uint32_t kLdsLog = 11;
constexpr uint32_t kLdsN = 1u << kLdsLog;
constexpr unsigned kLdsTPB = kLdsN / 4;
static_assert(kLdsLog % 2 == 1, "the LDS stages are pairs and one single stage");
static_assert(kMinLogL >= kLdsLog, "every block holds whole LDS chunks");

__host__ __device__ inline uint32_t mul_mod(uint32_t a, uint32_t b) { return (uint32_t)((uint64_t)a * b % kP); }
__device__ inline uint32_t add_mod(uint32_t a, uint32_t b) {
    const uint32_t s = a + b;  // both below kP < 2^30
    return s >= kP ? s - kP : s;
}
__device__ inline uint32_t sub_mod(uint32_t a, uint32_t b) { return a >= b ? a - b : a + (kP - b); }

__host__ __device__ inline uint32_t pow_mod(uint32_t a, uint64_t e) {
    uint32_t r = 1;
    while (e) {
        if (e & 1) r = mul_mod(r, a);
        a = mul_mod(a, a);
        e >>= 1;
    }
    return r;
}

uint32_t log2_block(uint64_t n, uint32_t m) {
    uint32_t lg = kMinLogL;
    while ((1ull << lg) < 2ull * m) ++lg;  // at least half of each block is windows
    uint32_t want = kBlockLogL;
    while (want > lg && (1ull << (want - 1)) >= n) --want;  // short texts: one block of about n
    return std::max(lg, want);
}

struct NttLayout {
    uint32_t logL;
    uint64_t x, y, z, tw, itw, members, bytes;
};

uint64_t align256(uint64_t v) { return (v + 255) / 256 * 256; }

NttLayout ntt_layout(uint64_t n, uint32_t m) {
    NttLayout Lo;
    Lo.logL = log2_block(n, m);
    const uint64_t L = 1ull << Lo.logL;
    uint64_t off = 0;
    Lo.x = off;  // pattern spectra, 4 x L
    off = align256(off + 16 * L);
    Lo.y = off;  // text block spectra, 4 x L
    off = align256(off + 16 * L);
    Lo.z = off;  // their product, L
    off = align256(off + 4 * L);
    Lo.tw = off;  // w^k, k < L/2
    off = align256(off + 2 * L);
    Lo.itw = off;  // w^-k, k < L/2
    off = align256(off + 2 * L);
    Lo.members = off;  // class member sets of the pattern, m bytes
    off = align256(off + m);
    Lo.bytes = off;
    return Lo;
}

unsigned grid_for(uint64_t items) { return (unsigned)std::min<uint64_t>(std::max<uint64_t>((items + kTPB - 1) / kTPB, 1), 4096); }

__global__ void twiddle_kernel(uint32_t* tw, uint32_t half, uint32_t w) {
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < half; k += gridDim.x * blockDim.x) tw[k] = pow_mod(w, k);
}

// x[b L + j] = [b not in S_{m-1-j}] for j < m, 0 beyond: the reversed
// pattern, so that a convolution gives the correlation.
__global__ void expand_pattern_kernel(const uint8_t* members, uint32_t m, uint32_t L, uint32_t* x) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < L; j += gridDim.x * blockDim.x) {
        const uint32_t s = j < m ? members[m - 1 - j] : 0xFu;
#pragma unroll
        for (uint32_t b = 0; b < 4; ++b) x[(uint64_t)b * L + j] = (s >> b & 1u) ? 0u : 1u;
    }
}

// y[b L + i] = [t[start + i] = b], 0 past the text.  Planar 2-bit text: block
// of 32 bases q holds the high code bits in word 2q and the low ones in 2q+1.
__global__ void expand_text_kernel(const uint32_t* text, uint64_t n, uint64_t start, uint32_t L, uint32_t* y) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < L; i += gridDim.x * blockDim.x) {
        const uint64_t pos = start + i;
        uint32_t code = 4;  // no base
        if (pos < n) {
            const uint64_t q = pos >> 5;
            const uint32_t bit = (uint32_t)(pos & 31);
            code = ((text[2 * q] >> bit) & 1u) << 1 | ((text[2 * q + 1] >> bit) & 1u);
        }
#pragma unroll
        for (uint32_t b = 0; b < 4; ++b) y[(uint64_t)b * L + i] = code == b ? 1u : 0u;
    }
}

// One decimation-in-frequency stage (half-size len) over `count` arrays of L.
__global__ void dif_stage_kernel(uint32_t* a, uint32_t L, uint32_t len, uint32_t step, const uint32_t* tw, uint32_t count) {
    const uint32_t half = L / 2;
    const uint64_t total = (uint64_t)half * count;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t arr = (uint32_t)(t / half), bf = (uint32_t)(t % half);
        const uint32_t j = bf % len, s = (bf / len) * 2 * len;
        uint32_t* p = a + (uint64_t)arr * L + s + j;
        const uint32_t u = p[0], v = p[len];
        p[0] = add_mod(u, v);
        p[len] = mul_mod(sub_mod(u, v), tw[j * step]);
    }
}

// Two decimation-in-frequency stages at once (half-sizes H and H/2) over
// `count` arrays of L: each thread takes the four elements j, j+H/2, j+H,
// j+3H/2 of its 2H block through both stages (one pass instead of two).
__global__ void dif4_stage_kernel(uint32_t* a, uint32_t L, uint32_t H, const uint32_t* tw, uint32_t count) {
    const uint32_t quarter = L / 4, Q = H / 2, sh = L / (2 * H), sq = L / H;
    const uint64_t total = (uint64_t)quarter * count;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t arr = (uint32_t)(t / quarter), q = (uint32_t)(t % quarter);
        const uint32_t j = q % Q, s = (q / Q) * 2 * H;
        uint32_t* p = a + (uint64_t)arr * L + s + j;
        const uint32_t a0 = p[0], a1 = p[Q], a2 = p[H], a3 = p[H + Q];
        const uint32_t b0 = add_mod(a0, a2), b2 = mul_mod(sub_mod(a0, a2), tw[j * sh]);
        const uint32_t b1 = add_mod(a1, a3), b3 = mul_mod(sub_mod(a1, a3), tw[(j + Q) * sh]);
        const uint32_t w = tw[j * sq];
        p[0] = add_mod(b0, b1);
        p[Q] = mul_mod(sub_mod(b0, b1), w);
        p[H] = add_mod(b2, b3);
        p[H + Q] = mul_mod(sub_mod(b2, b3), w);
    }
}

// Two decimation-in-time stages at once (half-sizes Q and 2Q) of the one
// array of L, the mirror of dif4_stage_kernel.
__global__ void dit4_stage_kernel(uint32_t* a, uint32_t L, uint32_t Q, const uint32_t* itw) {
    const uint32_t quarter = L / 4, H = 2 * Q;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < quarter; q += gridDim.x * blockDim.x) {
        const uint32_t j = q % Q, s = (q / Q) * 2 * H;
        uint32_t* p = a + s + j;
        const uint32_t w1 = itw[j * (L / (2 * Q))];
        const uint32_t a0 = p[0], t1 = mul_mod(p[Q], w1), a2 = p[H], t3 = mul_mod(p[H + Q], w1);
        const uint32_t b0 = add_mod(a0, t1), b1 = sub_mod(a0, t1), b2 = add_mod(a2, t3), b3 = sub_mod(a2, t3);
        const uint32_t u2 = mul_mod(b2, itw[j * (L / (2 * H))]), u3 = mul_mod(b3, itw[(j + Q) * (L / (2 * H))]);
        p[0] = add_mod(b0, u2);
        p[H] = sub_mod(b0, u2);
        p[Q] = add_mod(b1, u3);
        p[H + Q] = sub_mod(b1, u3);
    }
}

// Three decimation-in-frequency stages at once (half-sizes H, H/2, H/4)
// over `count` arrays of L: each thread takes the eight elements j + r H/4
// (r < 8) of its 2H block through all three.  At stage k the pairs are r and
// r + d with d = 4 >> k; the pair's index within its 2h block (h = d H/4) is
// (r mod d) H/4 + j.
__global__ void dif8_stage_kernel(uint32_t* a, uint32_t L, uint32_t H, const uint32_t* tw, uint32_t count) {
    const uint32_t eighth = L / 8, Q4 = H / 4;
    const uint64_t total = (uint64_t)eighth * count;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t arr = (uint32_t)(t / eighth), q = (uint32_t)(t % eighth);
        const uint32_t j = q % Q4, s = (q / Q4) * 2 * H;
        uint32_t* p = a + (uint64_t)arr * L + s + j;
        uint32_t e[8];
#pragma unroll
        for (uint32_t r = 0; r < 8; ++r) e[r] = p[r * Q4];
#pragma unroll
        for (uint32_t k = 0; k < 3; ++k) {
            const uint32_t d = 4u >> k, step = L / (2 * Q4 * d);
#pragma unroll
            for (uint32_t r = 0; r < 8; ++r) {
                if ((r / d) % 2 == 0) {
                    const uint32_t u = e[r], v = e[r + d];
                    e[r] = add_mod(u, v);
                    e[r + d] = mul_mod(sub_mod(u, v), tw[((r % d) * Q4 + j) * step]);
                }
            }
        }
#pragma unroll
        for (uint32_t r = 0; r < 8; ++r) p[r * Q4] = e[r];
    }
}

// Three decimation-in-time stages at once (half-sizes Q, 2Q, 4Q) of the one
// array of L, the mirror of dif8_stage_kernel.
__global__ void dit8_stage_kernel(uint32_t* a, uint32_t L, uint32_t Q, const uint32_t* itw) {
    const uint32_t eighth = L / 8, H = 4 * Q;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < eighth; q += gridDim.x * blockDim.x) {
        const uint32_t j = q % Q, s = (q / Q) * 2 * H;
        uint32_t* p = a + s + j;
        uint32_t e[8];
#pragma unroll
        for (uint32_t r = 0; r < 8; ++r) e[r] = p[r * Q];
#pragma unroll
        for (uint32_t k = 3; k-- > 0;) {
            const uint32_t d = 4u >> k, step = L / (2 * Q * d);
#pragma unroll
            for (uint32_t r = 0; r < 8; ++r) {
                if ((r / d) % 2 == 0) {
                    const uint32_t u = e[r], v = mul_mod(e[r + d], itw[((r % d) * Q + j) * step]);
                    e[r] = add_mod(u, v);
                    e[r + d] = sub_mod(u, v);
                }
            }
        }
#pragma unroll
        for (uint32_t r = 0; r < 8; ++r) p[r * Q] = e[r];
    }
}

// One decimation-in-time stage of the inverse transform (one array of L).
__global__ void dit_stage_kernel(uint32_t* a, uint32_t L, uint32_t len, uint32_t step, const uint32_t* itw) {
    const uint32_t half = L / 2;
    for (uint32_t bf = blockIdx.x * blockDim.x + threadIdx.x; bf < half; bf += gridDim.x * blockDim.x) {
        const uint32_t j = bf % len, s = (bf / len) * 2 * len;
        uint32_t* p = a + s + j;
        const uint32_t u = p[0], v = mul_mod(p[len], itw[j * step]);
        p[0] = add_mod(u, v);
        p[len] = sub_mod(u, v);
    }
}

// z[k] = sum_b x[b L + k] y[b L + k]: the four residue sequences' spectra,
// decoded and summed.
__global__ void pointwise_kernel(const uint32_t* x, const uint32_t* y, uint32_t L, uint32_t* z) {
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < L; k += gridDim.x * blockDim.x) {
        uint32_t acc = 0;
#pragma unroll
        for (uint32_t b = 0; b < 4; ++b) acc = add_mod(acc, mul_mod(x[(uint64_t)b * L + k], y[(uint64_t)b * L + k]));
        z[k] = acc;
    }
}

// counts[w] = z[w - start + m - 1] / L for the block's windows w in [start, start + nwin).
__global__ void output_kernel(const uint32_t* z, uint32_t m, uint64_t start, uint32_t nwin, uint32_t inv_l, uint32_t* counts) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nwin; i += gridDim.x * blockDim.x)
        counts[start + i] = mul_mod(z[i + m - 1], inv_l);
}

// The decimation-in-frequency stages len = kLdsN/2 .. 1 of one kLdsN chunk
// (chunk blockIdx.x over the `count` arrays of L), in LDS.  Their butterfly
// pairs never leave the chunk, since 2 len divides kLdsN.  Each thread holds
// four elements and takes them through two stages per barrier; the odd last
// stage (len = 1, twiddle 1) takes two pairs per thread.
__global__ __launch_bounds__(kLdsTPB) void dif_tail_kernel(uint32_t* a, uint32_t L, const uint32_t* tw) {
    __shared__ uint32_t sh[kLdsN];
    const uint32_t per_array = L / kLdsN;
    uint32_t* p = a + (uint64_t)(blockIdx.x / per_array) * L + (uint64_t)(blockIdx.x % per_array) * kLdsN;
    const uint32_t t = threadIdx.x;
#pragma unroll
    for (uint32_t r = 0; r < 4; ++r) sh[t + r * kLdsTPB] = p[t + r * kLdsTPB];
    __syncthreads();
    for (uint32_t H = kLdsN / 2; H >= 2; H /= 4) {
        const uint32_t Q = H / 2, j = t % Q, i = (t / Q) * 2 * H + j;
        const uint32_t a0 = sh[i], a1 = sh[i + Q], a2 = sh[i + H], a3 = sh[i + H + Q];
        const uint32_t b0 = add_mod(a0, a2), b2 = mul_mod(sub_mod(a0, a2), tw[j * (L / (2 * H))]);
        const uint32_t b1 = add_mod(a1, a3), b3 = mul_mod(sub_mod(a1, a3), tw[(j + Q) * (L / (2 * H))]);
        const uint32_t w = tw[j * (L / H)];
        sh[i] = add_mod(b0, b1);
        sh[i + Q] = mul_mod(sub_mod(b0, b1), w);
        sh[i + H] = add_mod(b2, b3);
        sh[i + H + Q] = mul_mod(sub_mod(b2, b3), w);
        __syncthreads();
    }
#pragma unroll
    for (uint32_t r = 0; r < 2; ++r) {
        const uint32_t e = t + r * kLdsTPB;
        const uint32_t u = sh[2 * e], v = sh[2 * e + 1];
        sh[2 * e] = add_mod(u, v);
        sh[2 * e + 1] = sub_mod(u, v);
    }
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < 4; ++r) p[t + r * kLdsTPB] = sh[t + r * kLdsTPB];
}

// The decimation-in-time stages len = 1 .. kLdsN/2 of one kLdsN chunk of the
// one array of L, in LDS: the odd first stage (len = 1, twiddle 1), then two
// stages per barrier.
__global__ __launch_bounds__(kLdsTPB) void dit_head_kernel(uint32_t* a, uint32_t L, const uint32_t* itw) {
    __shared__ uint32_t sh[kLdsN];
    uint32_t* p = a + (uint64_t)blockIdx.x * kLdsN;
    const uint32_t t = threadIdx.x;
#pragma unroll
    for (uint32_t r = 0; r < 4; ++r) sh[t + r * kLdsTPB] = p[t + r * kLdsTPB];
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < 2; ++r) {
        const uint32_t e = t + r * kLdsTPB;
        const uint32_t u = sh[2 * e], v = sh[2 * e + 1];
        sh[2 * e] = add_mod(u, v);
        sh[2 * e + 1] = sub_mod(u, v);
    }
    __syncthreads();
    for (uint32_t Q = 2; Q <= kLdsN / 4; Q *= 4) {
        const uint32_t H = 2 * Q, j = t % Q, i = (t / Q) * 2 * H + j;
        const uint32_t w1 = itw[j * (L / (2 * Q))];
        const uint32_t a0 = sh[i], t1 = mul_mod(sh[i + Q], w1), a2 = sh[i + H], t3 = mul_mod(sh[i + H + Q], w1);
        const uint32_t b0 = add_mod(a0, t1), b1 = sub_mod(a0, t1), b2 = add_mod(a2, t3), b3 = sub_mod(a2, t3);
        const uint32_t u2 = mul_mod(b2, itw[j * (L / (2 * H))]), u3 = mul_mod(b3, itw[(j + Q) * (L / (2 * H))]);
        sh[i] = add_mod(b0, u2);
        sh[i + H] = sub_mod(b0, u2);
        sh[i + Q] = add_mod(b1, u3);
        sh[i + H + Q] = sub_mod(b1, u3);
        __syncthreads();
    }
#pragma unroll
    for (uint32_t r = 0; r < 4; ++r) p[t + r * kLdsTPB] = sh[t + r * kLdsTPB];
}

// Forward transform (decimation in frequency) of `count` arrays of L: the
// stages with len >= kLdsN one pass each, then the rest in LDS.
hipError_t forward(uint32_t* a, uint32_t logL, uint32_t count, const uint32_t* tw, hipStream_t s) {
    const uint32_t L = 1u << logL;
    for (uint32_t len = L / 2; len >= kLdsN;) {
        if (len / 4 >= kLdsN) {  // three stages in one pass
            dif8_stage_kernel<<<grid_for((uint64_t)(L / 8) * count), kTPB, 0, s>>>(a, L, len, tw, count);
            len /= 8;
        } else if (len / 2 >= kLdsN) {  // two stages in one pass
            dif4_stage_kernel<<<grid_for((uint64_t)(L / 4) * count), kTPB, 0, s>>>(a, L, len, tw, count);
            len /= 4;
        } else {
            dif_stage_kernel<<<grid_for((uint64_t)(L / 2) * count), kTPB, 0, s>>>(a, L, len, L / (2 * len), tw, count);
            len /= 2;
        }
        if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    }
    dif_tail_kernel<<<(L / kLdsN) * count, kLdsTPB, 0, s>>>(a, L, tw);
    return hipGetLastError();
}

// Inverse transform (decimation in time) of one array of L, without the 1/L:
// the stages with len < kLdsN in LDS, then the rest one pass each.
hipError_t inverse(uint32_t* a, uint32_t logL, const uint32_t* itw, hipStream_t s) {
    const uint32_t L = 1u << logL;
    dit_head_kernel<<<L / kLdsN, kLdsTPB, 0, s>>>(a, L, itw);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    for (uint32_t len = kLdsN; len <= L / 2;) {
        if (4 * len <= L / 2) {  // three stages in one pass
            dit8_stage_kernel<<<grid_for(L / 8), kTPB, 0, s>>>(a, L, len, itw);
            len *= 8;
        } else if (2 * len <= L / 2) {  // two stages in one pass
            dit4_stage_kernel<<<grid_for(L / 4), kTPB, 0, s>>>(a, L, len, itw);
            len *= 4;
        } else {
            dit_stage_kernel<<<grid_for(L / 2), kTPB, 0, s>>>(a, L, len, L / (2 * len), itw);
            len *= 2;
        }
        if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

uint64_t pm_crt_counts_workspace_bytes(uint64_t n, uint32_t m) {
    if (m == 0 || m > kMaxM) return 0;
    return ntt_layout(n, m).bytes;
}

pm_status pm_crt_counts(const void* text_dev, uint64_t n, const uint8_t* codes, uint32_t m, uint32_t* counts_dev,
                        void* ws_dev, uint64_t ws_bytes, void* stream) {
    using pm::set_error;
    if (!text_dev || !codes || !ws_dev) return set_error(PM_ERR_ARG, "null pointer");
    if (m == 0) return set_error(PM_ERR_ARG, "empty pattern (m = 0)");
    if (m > kMaxM) return set_error(PM_ERR_UNSUPPORTED, "the transform route takes m up to 2^22");
    if (reinterpret_cast<uintptr_t>(text_dev) % 16 != 0) return set_error(PM_ERR_ARG, "text_dev must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(ws_dev) % 256 != 0) return set_error(PM_ERR_ARG, "ws_dev must be 256-byte aligned");
    std::vector<uint8_t> members(m);
    for (uint32_t j = 0; j < m; ++j) {
        if (codes[j] > 15) return set_error(PM_ERR_SYMBOL, "pattern code above 15 at " + std::to_string(j));
        members[j] = (uint8_t)pm::members_of_code(codes[j]);
    }
    const uint64_t nw = m <= n ? n - m + 1 : 0;
    if (nw == 0) return PM_OK;
    if (!counts_dev) return set_error(PM_ERR_ARG, "null counts_dev");
    const NttLayout Lo = ntt_layout(n, m);
    if (ws_bytes < Lo.bytes)
        return set_error(PM_ERR_WORKSPACE, "workspace too small: need " + std::to_string(Lo.bytes) + " bytes");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint8_t* ws = static_cast<uint8_t*>(ws_dev);
    uint32_t* x = reinterpret_cast<uint32_t*>(ws + Lo.x);
    uint32_t* y = reinterpret_cast<uint32_t*>(ws + Lo.y);
    uint32_t* z = reinterpret_cast<uint32_t*>(ws + Lo.z);
    uint32_t* tw = reinterpret_cast<uint32_t*>(ws + Lo.tw);
    uint32_t* itw = reinterpret_cast<uint32_t*>(ws + Lo.itw);
    uint8_t* mem_dev = ws + Lo.members;
    const uint32_t L = 1u << Lo.logL;
    const uint32_t w = pow_mod(kRoot, (kP - 1) >> Lo.logL);  // a primitive L-th root of unity
    const uint32_t w_inv = pow_mod(w, kP - 2);
    const uint32_t inv_l = pow_mod(L, kP - 2);
    const uint32_t* text = static_cast<const uint32_t*>(text_dev);

    // the member sets are staged from host memory: wait for that copy
    // before `members` goes out of scope
    hipError_t e = hipMemcpyAsync(mem_dev, members.data(), m, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error(PM_ERR_HIP, std::string("pattern copy: ") + hipGetErrorString(e));
    twiddle_kernel<<<grid_for(L / 2), kTPB, 0, s>>>(tw, L / 2, w);
    twiddle_kernel<<<grid_for(L / 2), kTPB, 0, s>>>(itw, L / 2, w_inv);
    expand_pattern_kernel<<<grid_for(L), kTPB, 0, s>>>(mem_dev, m, L, x);
    if ((e = hipGetLastError()) == hipSuccess) e = forward(x, Lo.logL, 4, tw, s);
    const uint64_t per_block = (uint64_t)L - m + 1;
    for (uint64_t start = 0; e == hipSuccess && start < nw; start += per_block) {
        const uint32_t nwin = (uint32_t)std::min<uint64_t>(per_block, nw - start);
        expand_text_kernel<<<grid_for(L), kTPB, 0, s>>>(text, n, start, L, y);
        if ((e = hipGetLastError()) != hipSuccess) break;
        if ((e = forward(y, Lo.logL, 4, tw, s)) != hipSuccess) break;
        pointwise_kernel<<<grid_for(L), kTPB, 0, s>>>(x, y, L, z);
        if ((e = hipGetLastError()) != hipSuccess) break;
        if ((e = inverse(z, Lo.logL, itw, s)) != hipSuccess) break;
        output_kernel<<<grid_for(nwin), kTPB, 0, s>>>(z, m, start, nwin, inv_l, counts_dev);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return set_error(PM_ERR_HIP, hipGetErrorString(e));
    return PM_OK;
}

}  // extern "C"
