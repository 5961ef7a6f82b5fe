// hostscan.hip -- scan of a text kept in host memory (libpmscan).
//
// Sect. 2.6 cuts the text into pieces with an m-1 overlap and searches each
// piece on its own.  Here the pieces are chunks of `chunk_bases` windows that
// are copied from host memory into one of two device buffers on a copy
// stream, while the previous chunk is encoded and scanned on the compute
// stream, so a text larger than the device budget is scanned at the rate of
// the host-to-device link.  Each chunk is scanned by pm_scan over its own
// windows; its hits are appended to the output and moved to text positions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "../../include/pmscan.h"

namespace pm {
pm_status set_error(pm_status s, const std::string& what);
}

namespace {

uint64_t align256(uint64_t x) { return (x + 255) / 256 * 256; }

// Largest chunk accepted (2^48 windows, far beyond any device memory): keeps
// every size and offset below free of 64-bit overflow.
constexpr uint64_t kMaxChunkBases = 1ull << 48;

// Workspace: two ASCII chunk buffers, two encoded chunk buffers, two
// bad-symbol words, a hit total and one plain-scan workspace (the scans run
// one after another on the compute stream).
struct HostScanLayout {
    uint64_t ascii[2], text[2], bad[2], nh, scan, bytes;
};

HostScanLayout host_layout(uint64_t chunk_bases, uint32_t m) {
    const uint64_t len = chunk_bases + m - 1;  // bases of one chunk with its overlap
    HostScanLayout L;
    uint64_t off = 0;
    for (int b = 0; b < 2; ++b) {
        L.ascii[b] = off;
        off = align256(off + len);
    }
    for (int b = 0; b < 2; ++b) {
        L.text[b] = off;
        off = align256(off + pm_text_bytes(len));
    }
    for (int b = 0; b < 2; ++b) {
        L.bad[b] = off;
        off = align256(off + 8);
    }
    L.nh = off;
    off = align256(off + 8);
    L.scan = off;
    off = align256(off + pm_scan_workspace_bytes(len));
    L.bytes = off;
    return L;
}

__global__ void add_offset_kernel(int64_t* pos, uint64_t count, int64_t offset) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x)
        pos[i] += offset;
}

__global__ void set_u64_kernel(uint64_t* p, uint64_t value) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = value;
}

// Events of the two buffers, released on every return.
struct BufferEvents {
    hipEvent_t copied[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr};
    ~BufferEvents() {
        for (int b = 0; b < 2; ++b) {
            if (copied[b]) (void)hipEventDestroy(copied[b]);
            if (freed[b]) (void)hipEventDestroy(freed[b]);
        }
    }
};

}  // namespace

extern "C" {

uint64_t pm_scan_host_workspace_bytes(uint64_t chunk_bases, uint32_t m) {
    if (chunk_bases == 0 || chunk_bases > kMaxChunkBases || m == 0) return 0;
    return host_layout(chunk_bases, m).bytes;
}

pm_status pm_scan_host(const uint8_t* ascii_host, uint64_t n, const uint8_t* codes, uint32_t m, uint32_t k,
                       const void* image_dev, uint64_t chunk_bases, int64_t* pos_dev, uint16_t* cnt_dev,
                       uint64_t capacity, uint64_t* n_hits_dev, void* ws_dev, uint64_t ws_bytes, void* stream,
                       void* copy_stream) {
    using pm::set_error;
    if ((n > 0 && !ascii_host) || !codes || !image_dev || !n_hits_dev || !ws_dev)
        return set_error(PM_ERR_ARG, "null pointer");
    if (capacity > 0 && (!pos_dev || !cnt_dev)) return set_error(PM_ERR_ARG, "null output with capacity > 0");
    if (m == 0) return set_error(PM_ERR_ARG, "empty pattern (m = 0)");
    if (chunk_bases == 0 || chunk_bases > kMaxChunkBases)
        return set_error(PM_ERR_ARG, "chunk_bases must be in 1..2^48");
    if (reinterpret_cast<uintptr_t>(ws_dev) % 256 != 0) return set_error(PM_ERR_ARG, "ws_dev must be 256-byte aligned");
    const HostScanLayout L = host_layout(chunk_bases, m);
    if (ws_bytes < L.bytes)
        return set_error(PM_ERR_WORKSPACE, "workspace too small: need " + std::to_string(L.bytes) + " bytes");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipStream_t cs = reinterpret_cast<hipStream_t>(copy_stream);
    uint8_t* ws = static_cast<uint8_t*>(ws_dev);
    const uint64_t nw = m <= n ? n - m + 1 : 0;
    const uint64_t chunks = nw / chunk_bases + (nw % chunk_bases != 0);

    BufferEvents ev;
    for (int b = 0; b < 2; ++b)
        if (hipEventCreateWithFlags(&ev.copied[b], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ev.freed[b], hipEventDisableTiming) != hipSuccess)
            return set_error(PM_ERR_HIP, "hipEventCreateWithFlags failed");
    // every return waits for both streams, so that no copy or kernel still
    // uses the workspace or the host text
    auto finish = [&](pm_status st) {
        const hipError_t e1 = hipStreamSynchronize(s), e2 = hipStreamSynchronize(cs);
        if (st == PM_OK && (e1 != hipSuccess || e2 != hipSuccess))
            return set_error(PM_ERR_HIP, std::string("stream synchronize: ") +
                                             hipGetErrorString(e1 != hipSuccess ? e1 : e2));
        return st;
    };
    auto chunk_span = [&](uint64_t c, uint64_t& first, uint64_t& len) {
        first = c * chunk_bases;
        len = std::min(n - first, chunk_bases + m - 1);
    };
    auto issue_copy = [&](uint64_t c) -> pm_status {
        const int b = (int)(c & 1);
        uint64_t first, len;
        chunk_span(c, first, len);
        hipError_t e = hipSuccess;
        if (c >= 2) e = hipStreamWaitEvent(cs, ev.freed[b], 0);  // chunk c-2 is done with buffer b
        if (e == hipSuccess) e = hipMemcpyAsync(ws + L.ascii[b], ascii_host + first, len, hipMemcpyHostToDevice, cs);
        if (e == hipSuccess) e = hipEventRecord(ev.copied[b], cs);
        if (e != hipSuccess) return set_error(PM_ERR_HIP, std::string("chunk copy: ") + hipGetErrorString(e));
        return PM_OK;
    };

    uint64_t total = 0;
    if (chunks > 0) {
        if (pm_status st = issue_copy(0); st != PM_OK) return finish(st);
    }
    for (uint64_t c = 0; c < chunks; ++c) {
        const int b = (int)(c & 1);
        if (c + 1 < chunks) {  // the next chunk's copy overlaps this chunk's work
            if (pm_status st = issue_copy(c + 1); st != PM_OK) return finish(st);
        }
        uint64_t first, len;
        chunk_span(c, first, len);
        const uint64_t wc = std::min(chunk_bases, nw - first);
        if (hipStreamWaitEvent(s, ev.copied[b], 0) != hipSuccess)
            return finish(set_error(PM_ERR_HIP, "hipStreamWaitEvent failed"));
        pm_status st = pm_encode_text(ws + L.ascii[b], len, ws + L.text[b], reinterpret_cast<uint64_t*>(ws + L.bad[b]), s);
        if (st != PM_OK) return finish(st);
        const uint64_t cap_left = capacity > total ? capacity - total : 0;
        st = pm_scan(ws + L.text[b], len, codes, m, k, image_dev, 0, wc, cap_left ? pos_dev + total : nullptr,
                     cap_left ? cnt_dev + total : nullptr, cap_left, reinterpret_cast<uint64_t*>(ws + L.nh),
                     ws + L.scan, ws_bytes - L.scan, s);
        if (st != PM_OK) return finish(st);
        uint64_t words[2];
        hipError_t e = hipEventRecord(ev.freed[b], s);
        if (e == hipSuccess) e = hipMemcpyAsync(&words[0], ws + L.nh, 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&words[1], ws + L.bad[b], 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return finish(set_error(PM_ERR_HIP, std::string("chunk result: ") + hipGetErrorString(e)));
        if (words[1] != ~0ull)
            return finish(set_error(PM_ERR_SYMBOL, "text symbol other than A, C, G, T at index " +
                                                       std::to_string(first + words[1])));
        const uint64_t written = std::min(words[0], cap_left);
        if (written > 0 && first > 0) {
            const unsigned grid = (unsigned)std::min<uint64_t>((written + 255) / 256, 1024);
            add_offset_kernel<<<grid, 256, 0, s>>>(pos_dev + total, written, (int64_t)first);
            if ((e = hipGetLastError()) != hipSuccess)
                return finish(set_error(PM_ERR_HIP, hipGetErrorString(e)));
        }
        total += words[0];
    }
    set_u64_kernel<<<1, 64, 0, s>>>(n_hits_dev, total);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) return finish(set_error(PM_ERR_HIP, hipGetErrorString(e)));
    return finish(PM_OK);
}

}  // extern "C"
