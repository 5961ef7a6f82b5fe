// batch.hpp -- internal entry of the batched scan, shared by pm_scan_batch
// and the query server (libpmscan).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/pmscan.h"
#include "plan.hpp"

namespace pm {

// Survival target of the plans of batched patterns (build_plan's
// `survival`).  Higher than a single scan's: here a survivor costs one
// window's exact count in a loop the item runs anyway, while a group of 8
// filter slots costs every window of every tile, so a group is worth keeping
// only where dropping it would let more than ~3e-4 of the windows through.
// On 4096 patterns over 256e6 bases, 2e-4 takes 9% fewer slots than 4e-5 and
// the launch 8% less time; 6.4e-4 (14% fewer slots) is slower again.
constexpr double kBatchSurvival = 2e-4;

// One pattern of a batched call, prepared by the caller.
struct BatchEntry {
    const uint8_t* codes;   // Table 2 codes [m], host memory
    uint32_t m, k;
    const ScanPlan* plan;   // plan from build_plan(..., kBatchSurvival, window_at_zero = true), or null to build it
    uint64_t image_off;     // image in BatchCall::images_dev, 16-byte units (ignored when that is null)
    uint64_t out_off;       // first output slot in pos/cnt
    uint64_t capacity;      // output slots
};

struct BatchCall {
    const void* text_dev = nullptr;
    uint64_t n = 0;
    uint32_t count = 0;
    const BatchEntry* entries = nullptr;
    // pattern images already on the device (image p at images_dev + 16 * image_off),
    // or null: the images are built on the host and copied into the workspace
    const void* images_dev = nullptr;
    uint64_t win_begin = 0, win_end = 0;
    int64_t* pos_dev = nullptr;
    uint16_t* cnt_dev = nullptr;
    uint64_t* n_hits_dev = nullptr;
    uint32_t* status_dev = nullptr;
    void* ws_dev = nullptr;
    uint64_t ws_bytes = 0;
    const pm_batch_config* cfg = nullptr;
    // pinned host staging for the descriptor (at least batch_desc_bytes), or
    // null: a pageable buffer is used and the copy is staged before return
    uint8_t* desc_host = nullptr;
    uint64_t desc_host_bytes = 0;
    hipStream_t stream = nullptr;
};

pm_status batch_run(const BatchCall& c);

// Text sub-ranges per pattern group: at most kMaxSubRanges.  The automatic
// choice aims at about kAutoItems work items per launch (eight per wave that
// fits on the device), so that a call with few patterns still fills the chip.
constexpr uint32_t kMaxSubRanges = 4096;
constexpr uint64_t kAutoItems = 8ull * 256 * 16;

// The sub-range count a call over `count` patterns takes when
// cfg->sub_ranges is 0.
uint32_t batch_auto_sub_ranges(uint32_t count, const pm_batch_config* cfg);

// Output capacities of one call may sum to at most kMaxTotalCapacity hits
// (10 bytes each: far beyond any device), which keeps the workspace sizes
// free of 64-bit overflow; larger ones are refused.
constexpr uint64_t kMaxTotalCapacity = 1ull << 44;

// Workspace bytes of a call over these patterns; with_images = false when
// the caller keeps the images on the device.  UINT64_MAX when the
// capacities exceed kMaxTotalCapacity.
uint64_t batch_ws_bytes(uint64_t n, uint32_t count, const uint32_t* m, const uint64_t* capacity,
                        const pm_batch_config* cfg, bool with_images);

// Upper bound of the descriptor a call copies to the device.
uint64_t batch_desc_bytes(uint64_t n, uint32_t count, const uint32_t* m, const uint64_t* capacity,
                          const pm_batch_config* cfg, bool with_images);

}  // namespace pm
