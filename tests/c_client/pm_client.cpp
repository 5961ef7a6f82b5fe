// pm_client.cpp -- a client of libpmscan that uses only the C ABI
// (include/pmscan.h) and the HIP runtime: no Python, no PyTorch.
//
// usage: pm_client TEXT_FILE PATTERN K
// Reads the ASCII text, encodes it on the device, builds the pattern image,
// scans all windows with pm_scan (re-running with an exact buffer when the
// hits exceed the first capacity) and prints "position count" per hit.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/pmscan.h"

static int check(pm_status s, const char* what) {
    if (s != PM_OK) {
        std::fprintf(stderr, "%s: %s (%s)\n", what, pm_status_string(s), pm_last_error_detail());
        return 1;
    }
    return 0;
}

#define HIP(x)                                                                   \
    do {                                                                         \
        hipError_t e_ = (x);                                                     \
        if (e_ != hipSuccess) {                                                  \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));         \
            return 1;                                                            \
        }                                                                        \
    } while (0)

int main(int argc, char** argv) {
    if (argc != 4) {
        std::fprintf(stderr, "usage: %s TEXT_FILE PATTERN K\n", argv[0]);
        return 2;
    }
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    std::vector<uint8_t> text;
    for (int c; (c = std::fgetc(f)) != EOF;) text.push_back((uint8_t)c);
    std::fclose(f);
    const uint64_t n = text.size();
    const uint32_t k = (uint32_t)std::strtoul(argv[3], nullptr, 10);

    // pattern codes (host) and image (host, then device)
    uint32_t m = 0;
    if (check(pm_encode_pattern(argv[2], std::strlen(argv[2]), nullptr, 0, &m), "pm_encode_pattern")) return 1;
    std::vector<uint8_t> codes(m);
    if (check(pm_encode_pattern(argv[2], std::strlen(argv[2]), codes.data(), m, &m), "pm_encode_pattern")) return 1;
    std::vector<uint8_t> image(pm_pattern_bytes(m));
    if (check(pm_pattern_image(codes.data(), m, image.data(), image.size()), "pm_pattern_image")) return 1;

    // device buffers, all owned here
    void *ascii_dev = nullptr, *text_dev = nullptr, *image_dev = nullptr, *ws_dev = nullptr;
    uint64_t *bad_dev = nullptr, *nh_dev = nullptr;
    HIP(hipMalloc(&ascii_dev, n ? n : 1));
    HIP(hipMalloc(&text_dev, pm_text_bytes(n)));
    HIP(hipMalloc(&image_dev, image.size()));
    HIP(hipMalloc(&ws_dev, pm_scan_workspace_bytes(n)));
    HIP(hipMalloc(&bad_dev, 8));
    HIP(hipMalloc(&nh_dev, 8));
    HIP(hipMemcpy(ascii_dev, text.data(), n, hipMemcpyHostToDevice));
    HIP(hipMemcpy(image_dev, image.data(), image.size(), hipMemcpyHostToDevice));
    if (check(pm_encode_text((const uint8_t*)ascii_dev, n, text_dev, bad_dev, nullptr), "pm_encode_text")) return 1;
    uint64_t bad = 0;
    HIP(hipMemcpy(&bad, bad_dev, 8, hipMemcpyDeviceToHost));
    if (bad != UINT64_MAX) {
        std::fprintf(stderr, "text symbol other than A/C/G/T at %llu\n", (unsigned long long)bad);
        return 1;
    }

    uint64_t capacity = 1024, total = 0;
    int64_t* pos_dev = nullptr;
    uint16_t* cnt_dev = nullptr;
    for (;;) {
        HIP(hipMalloc(&pos_dev, 8 * capacity));
        HIP(hipMalloc(&cnt_dev, 2 * capacity));
        if (check(pm_scan(text_dev, n, codes.data(), m, k, image_dev, 0, UINT64_MAX, pos_dev, cnt_dev, capacity,
                          nh_dev, ws_dev, pm_scan_workspace_bytes(n), nullptr),
                  "pm_scan"))
            return 1;
        HIP(hipMemcpy(&total, nh_dev, 8, hipMemcpyDeviceToHost));
        if (total <= capacity) break;
        HIP(hipFree(pos_dev));
        HIP(hipFree(cnt_dev));
        capacity = total;
    }
    std::vector<int64_t> pos(total);
    std::vector<uint16_t> cnt(total);
    if (total) {
        HIP(hipMemcpy(pos.data(), pos_dev, 8 * total, hipMemcpyDeviceToHost));
        HIP(hipMemcpy(cnt.data(), cnt_dev, 2 * total, hipMemcpyDeviceToHost));
    }
    for (uint64_t i = 0; i < total; ++i) std::printf("%lld %u\n", (long long)pos[i], (unsigned)cnt[i]);
    HIP(hipFree(pos_dev));
    HIP(hipFree(cnt_dev));
    HIP(hipFree(ascii_dev));
    HIP(hipFree(text_dev));
    HIP(hipFree(image_dev));
    HIP(hipFree(ws_dev));
    HIP(hipFree(bad_dev));
    HIP(hipFree(nh_dev));
    return 0;
}
