// fasta_scan.cpp -- pm_scan_fasta: the plain scan (pm_scan) over the window
// ranges a parsed FASTA file admits (its reading is stated in fasta.cpp),
// in ascending order.
#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "fasta.hpp"

extern "C" {

pm_status pm_scan_fasta(const pm_fasta* f, const void* text_dev, const uint8_t* codes, uint32_t m, uint32_t k,
                        const void* image_dev, int64_t* pos_dev, uint16_t* cnt_dev, uint64_t capacity,
                        uint64_t* n_hits, void* ws_dev, uint64_t ws_bytes, void* stream) {
    using pm::set_error;
    if (!f || !n_hits) return set_error(PM_ERR_ARG, "null pointer");
    if (capacity > 0 && (!pos_dev || !cnt_dev)) return set_error(PM_ERR_ARG, "null output with capacity > 0");
    *n_hits = 0;
    uint64_t nr = 0;
    if (pm_status st = pm_fasta_window_ranges(f, m, nullptr, nullptr, 0, &nr); st != PM_OK) return st;
    std::vector<uint64_t> b(nr), e(nr);
    if (pm_status st = pm_fasta_window_ranges(f, m, b.data(), e.data(), nr, &nr); st != PM_OK) return st;
    const uint64_t n = f->bases.size();
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // one device word for each range's total, read back after its scan
    uint64_t* total_dev = reinterpret_cast<uint64_t*>(ws_dev);
    const uint64_t ws_need = pm_scan_workspace_bytes(n) + 256;
    if (!ws_dev || ws_bytes < ws_need)
        return set_error(PM_ERR_WORKSPACE, "workspace too small: need " + std::to_string(ws_need) + " bytes");
    void* scan_ws = reinterpret_cast<uint8_t*>(ws_dev) + 256;
    uint64_t written = 0, total = 0;
    for (uint64_t r = 0; r < nr; ++r) {
        const uint64_t left = capacity > written ? capacity - written : 0;
        if (pm_status st = pm_scan(text_dev, n, codes, m, k, image_dev, b[r], e[r], left ? pos_dev + written : nullptr,
                                   left ? cnt_dev + written : nullptr, left, total_dev, scan_ws, ws_bytes - 256, stream);
            st != PM_OK)
            return st;
        uint64_t got = 0;
        hipError_t he = hipMemcpyAsync(&got, total_dev, sizeof(got), hipMemcpyDeviceToHost, s);
        if (he == hipSuccess) he = hipStreamSynchronize(s);
        if (he != hipSuccess) return set_error(PM_ERR_HIP, std::string("range total: ") + hipGetErrorString(he));
        total += got;
        written += std::min(got, left);
    }
    *n_hits = total;
    return PM_OK;
}

uint64_t pm_scan_fasta_workspace_bytes(const pm_fasta* f) {
    return f ? pm_scan_workspace_bytes(f->bases.size()) + 256 : 0;
}

}  // extern "C"
