// calib.hip -- VALU issue-rate probe for gfx950 (libpmcalib.so).
//
// Not part of the scan library: a measurement aid for the "alu" rooflines.
// Each lane runs `chains` independent dependency chains of one instruction
// (or a fixed mix of two), `iters` times; the launch puts `waves` waves on
// every SIMD of the chip (workgroups of 256 lanes, one wave per SIMD, `waves`
// workgroups per CU).  The host times the kernel with HIP events and reports
// lane-operations per second, so that a kernel's instruction count per
// launch can be set against what the chip actually issues for the same
// instruction mix.
//
// The instructions are written with inline assembly (ALU only, no memory
// access) so that the compiler can neither fuse nor drop them.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

enum Kind : int {
    K_ALIGNBIT = 0,   // v_alignbit_b32 d, a, b, s (shift in an SGPR)
    K_BITOP3 = 1,     // v_bitop3_b32 (three-input xor)
    K_BITOP3_MAJ = 2, // v_bitop3_b32 (majority)
    K_XOR = 3,        // v_xor_b32 (VOP2)
    K_OR3 = 4,        // v_or3_b32
    K_ADD = 5,        // v_add_u32 (VOP2)
    K_MOV = 6,        // v_mov_b32
    K_LSHL_OR = 7,    // v_lshl_or_b32
    K_MIX_A1B2 = 8,   // alignbit : bitop3 = 1 : 2 (the filter's ratio)
    K_MIX_A1B1 = 9,   // alignbit : bitop3 = 1 : 1
    K_PERM = 10,      // v_perm_b32
    K_BFI = 11,       // v_bfi_b32
    K_LSHR64 = 12,    // v_lshrrev_b64
    K_ALIGNBIT_V = 13,// v_alignbit_b32 with the shift in a VGPR
    K_COUNT = 14
};

// One step of chain x (partner y, second partner z, uniform shift s).
template <int KIND>
__device__ __forceinline__ void step(uint32_t& x, uint32_t y, uint32_t z, uint32_t s, uint32_t vs, int phase) {
    if constexpr (KIND == K_ALIGNBIT) {
        asm volatile("v_alignbit_b32 %0, %0, %1, %2" : "+v"(x) : "v"(y), "s"(s));
    } else if constexpr (KIND == K_ALIGNBIT_V) {
        asm volatile("v_alignbit_b32 %0, %0, %1, %2" : "+v"(x) : "v"(y), "v"(vs));
    } else if constexpr (KIND == K_BITOP3) {
        asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(x) : "v"(y), "v"(z));
    } else if constexpr (KIND == K_BITOP3_MAJ) {
        asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0xe8" : "+v"(x) : "v"(y), "v"(z));
    } else if constexpr (KIND == K_XOR) {
        asm volatile("v_xor_b32 %0, %0, %1" : "+v"(x) : "v"(y));
    } else if constexpr (KIND == K_OR3) {
        asm volatile("v_or3_b32 %0, %0, %1, %2" : "+v"(x) : "v"(y), "v"(z));
    } else if constexpr (KIND == K_ADD) {
        asm volatile("v_add_u32 %0, %0, %1" : "+v"(x) : "v"(y));
    } else if constexpr (KIND == K_MOV) {
        asm volatile("v_mov_b32 %0, %0" : "+v"(x));
    } else if constexpr (KIND == K_LSHL_OR) {
        asm volatile("v_lshl_or_b32 %0, %0, 1, %1" : "+v"(x) : "v"(y));
    } else if constexpr (KIND == K_MIX_A1B2) {
        if (phase % 3 == 0)
            asm volatile("v_alignbit_b32 %0, %0, %1, %2" : "+v"(x) : "v"(y), "s"(s));
        else
            asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(x) : "v"(y), "v"(z));
    } else if constexpr (KIND == K_MIX_A1B1) {
        if (phase % 2 == 0)
            asm volatile("v_alignbit_b32 %0, %0, %1, %2" : "+v"(x) : "v"(y), "s"(s));
        else
            asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(x) : "v"(y), "v"(z));
    } else if constexpr (KIND == K_PERM) {
        asm volatile("v_perm_b32 %0, %0, %1, %2" : "+v"(x) : "v"(y), "v"(z));
    } else if constexpr (KIND == K_BFI) {
        asm volatile("v_bfi_b32 %0, %0, %1, %2" : "+v"(x) : "v"(y), "v"(z));
    }
}

// Kernel: CHAINS independent chains per lane, 6 steps per chain per loop
// iteration (6 keeps the 1:2 and 1:1 mixes exact).
template <int KIND, int CHAINS>
__global__ __launch_bounds__(256) void probe_kernel(uint32_t* out, uint32_t iters, uint32_t s) {
    uint32_t x[CHAINS], y[CHAINS];
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    const uint32_t z = t * 0x9E3779B9u;
    const uint32_t vs = (t & 7u) + 1u;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) {
        x[c] = t + 0x1234567u * (uint32_t)c;
        y[c] = (t << 3) ^ (0x89ABCDEFu + (uint32_t)c);
    }
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int ph = 0; ph < 6; ++ph) {
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) step<KIND>(x[c], y[c], z, s, vs, ph);
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) acc ^= x[c];
    if (acc == 0x5A5A5A5Au) out[t] = acc;  // keeps the chains live; practically never taken
}

// 64-bit shift: the chains are register pairs.
template <int CHAINS>
__global__ __launch_bounds__(256) void probe64_kernel(uint32_t* out, uint32_t iters, uint32_t s) {
    uint64_t x[CHAINS];
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = ((uint64_t)t << 32) | (t * 0x9E3779B9u + (uint32_t)c);
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int ph = 0; ph < 6; ++ph) {
#pragma unroll
            for (int c = 0; c < CHAINS; ++c) asm volatile("v_lshrrev_b64 %0, %1, %0" : "+v"(x[c]) : "s"(s));
        }
    }
    uint64_t acc = 0;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) acc ^= x[c];
    if (acc == 0x5A5A5A5Aull) out[t] = (uint32_t)acc;
}

template <int KIND>
hipError_t launch_kind(int chains, dim3 grid, uint32_t* out, uint32_t iters, uint32_t s, hipStream_t st) {
    if constexpr (KIND == K_LSHR64) {
        switch (chains) {
            case 1: probe64_kernel<1><<<grid, 256, 0, st>>>(out, iters, s); break;
            case 2: probe64_kernel<2><<<grid, 256, 0, st>>>(out, iters, s); break;
            case 4: probe64_kernel<4><<<grid, 256, 0, st>>>(out, iters, s); break;
            default: probe64_kernel<8><<<grid, 256, 0, st>>>(out, iters, s); break;
        }
    } else {
        switch (chains) {
            case 1: probe_kernel<KIND, 1><<<grid, 256, 0, st>>>(out, iters, s); break;
            case 2: probe_kernel<KIND, 2><<<grid, 256, 0, st>>>(out, iters, s); break;
            case 4: probe_kernel<KIND, 4><<<grid, 256, 0, st>>>(out, iters, s); break;
            default: probe_kernel<KIND, 8><<<grid, 256, 0, st>>>(out, iters, s); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch(int kind, int chains, dim3 grid, uint32_t* out, uint32_t iters, uint32_t s, hipStream_t st) {
    switch (kind) {
        case K_ALIGNBIT: return launch_kind<K_ALIGNBIT>(chains, grid, out, iters, s, st);
        case K_BITOP3: return launch_kind<K_BITOP3>(chains, grid, out, iters, s, st);
        case K_BITOP3_MAJ: return launch_kind<K_BITOP3_MAJ>(chains, grid, out, iters, s, st);
        case K_XOR: return launch_kind<K_XOR>(chains, grid, out, iters, s, st);
        case K_OR3: return launch_kind<K_OR3>(chains, grid, out, iters, s, st);
        case K_ADD: return launch_kind<K_ADD>(chains, grid, out, iters, s, st);
        case K_MOV: return launch_kind<K_MOV>(chains, grid, out, iters, s, st);
        case K_LSHL_OR: return launch_kind<K_LSHL_OR>(chains, grid, out, iters, s, st);
        case K_MIX_A1B2: return launch_kind<K_MIX_A1B2>(chains, grid, out, iters, s, st);
        case K_MIX_A1B1: return launch_kind<K_MIX_A1B1>(chains, grid, out, iters, s, st);
        case K_PERM: return launch_kind<K_PERM>(chains, grid, out, iters, s, st);
        case K_BFI: return launch_kind<K_BFI>(chains, grid, out, iters, s, st);
        case K_LSHR64: return launch_kind<K_LSHR64>(chains, grid, out, iters, s, st);
        case K_ALIGNBIT_V: return launch_kind<K_ALIGNBIT_V>(chains, grid, out, iters, s, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

extern "C" {

// Number of probe kinds (see Kind above; names by pmc_kind_name).
int pmc_kind_count(void) { return K_COUNT; }

const char* pmc_kind_name(int kind) {
    static const char* names[K_COUNT] = {
        "v_alignbit_b32 (sgpr shift)", "v_bitop3_b32 xor3", "v_bitop3_b32 maj3", "v_xor_b32",
        "v_or3_b32", "v_add_u32", "v_mov_b32", "v_lshl_or_b32",
        "alignbit:bitop3 1:2", "alignbit:bitop3 1:1", "v_perm_b32", "v_bfi_b32",
        "v_lshrrev_b64", "v_alignbit_b32 (vgpr shift)"};
    return kind >= 0 && kind < K_COUNT ? names[kind] : "";
}

// Run probe `kind` with `chains` (1, 2, 4 or 8) chains per lane and `waves`
// waves per SIMD (1..8) for `iters` loop iterations (6 steps per chain
// each), `reps` times after one warm-up launch; *ms_out gets the mean
// duration of one launch and *lane_ops_out the lane-operations of one
// launch.  Returns 0 or a hipError_t.
int pmc_valu_probe(int kind, int chains, int waves, uint32_t iters, int reps, double* ms_out,
                   double* lane_ops_out) {
    if (kind < 0 || kind >= K_COUNT || waves < 1 || waves > 8 || reps < 1 || !ms_out || !lane_ops_out)
        return (int)hipErrorInvalidValue;
    if (chains != 1 && chains != 2 && chains != 4 && chains != 8) return (int)hipErrorInvalidValue;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    const dim3 grid((unsigned)(cus * waves));
    uint32_t* out = nullptr;
    e = hipMalloc(&out, (size_t)grid.x * 256 * sizeof(uint32_t));
    if (e != hipSuccess) return (int)e;
    hipEvent_t a = nullptr, b = nullptr;
    float ms = 0.f;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = launch(kind, chains, grid, out, iters, 5u, nullptr);
    if (e == hipSuccess) e = hipEventRecord(a, nullptr);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(kind, chains, grid, out, iters, 5u, nullptr);
    if (e == hipSuccess) e = hipEventRecord(b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(out);
    if (e != hipSuccess) return (int)e;
    *ms_out = (double)ms / reps;
    *lane_ops_out = (double)grid.x * 256.0 * (double)iters * 6.0 * (double)chains;
    return 0;
}

// Compute units of the current device (for reporting).
int pmc_compute_units(void) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
    return cus;
}

}  // extern "C"
