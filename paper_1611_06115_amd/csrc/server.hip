// server.hip -- query server over a text resident in HBM (libpmscan).
//
// Continuous batching of a scan.  A scan has no natural iteration, so the
// server makes one: the window range [0, n) is cut into C chunks (one by
// default: a step's fixed costs make fewer, longer steps give the lower
// latency), and the engine thread runs chunk steps over chunks 0, 1, ...,
// C-1, 0, 1, ...  A
// step is one batched launch over its chunk for every admitted query.  A
// query is admitted between steps (in arrival order, while a slot and arena
// memory are free), enters at whatever chunk comes next, and is complete
// after C steps; the order of its hits is restored by joining its per-chunk
// segments in chunk order, not in the order they were scanned.
//
// Streams: the steps run on the main stream, at most two in flight, so the
// host prepares step s+1 while step s runs.  Re-scans of overflowed chunks
// and the joins run on a second stream once the host has seen the step that
// produced their input.  Both streams use the default priority.
//
// Arena (caller-owned device memory), in order: batch workspace | re-scan
// workspace | per-step hit totals and flags (2 slots) | join descriptors |
// pattern images (first-fit, 16-byte units) | hit positions (int64) and
// counts (uint16), one slot index space (first-fit).
//
// Each admitted query holds a region of C * cap hit slots (cap = per-chunk
// capacity from the expected number of hits, with a 2x margin): chunk c's
// hits go to slots [c * cap, c * cap + h_c).  The join moves segment c to
// slot D_c = h_0 + ... + h_{c-1} of the same region.  Since D_c <= c * cap
// whenever no chunk overflowed, every move goes to lower addresses and the
// segments can be moved in chunk order in place; otherwise the result gets a
// region of its own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/pmscan.h"
#include "batch.hpp"
#include "plan.hpp"

namespace pm {
pm_status set_error(pm_status s, const std::string& what);
}  // namespace pm

using namespace pm;

namespace {

constexpr uint64_t kNone = ~0ull;
constexpr int JTPB = 256;
constexpr int JV = 4;
constexpr uint64_t kImageStage = 1ull << 20;
constexpr uint32_t kJoinSlots = 4;
constexpr uint64_t kBigJoin = 1ull << 20;  // results this large are joined out of place
constexpr uint64_t kPiece = 1ull << 18;    // hit slots per join workgroup out of place
constexpr uint32_t kAdmitSubRanges = 64;  // sub-ranges per group that admission sizes the workspace for

uint64_t clock_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// First-fit allocator over unit ranges [0, cap).
class RangeAlloc {
  public:
    void reset(uint64_t cap) {
        cap_ = cap;
        used_ = peak_ = 0;
        free_.clear();
        if (cap) free_[0] = cap;
    }
    uint64_t alloc(uint64_t len) {
        if (len == 0) len = 1;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < len) continue;
            const uint64_t off = it->first, rest = it->second - len;
            free_.erase(it);
            if (rest) free_[off + len] = rest;
            used_ += len;
            peak_ = std::max(peak_, used_);
            return off;
        }
        return kNone;
    }
    void release(uint64_t off, uint64_t len) {
        if (off == kNone) return;
        if (len == 0) len = 1;
        used_ -= len;
        uint64_t start = off, size = len;
        auto next = free_.lower_bound(off);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                size += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + len == next->first) {
            size += next->second;
            free_.erase(next);
        }
        free_[start] = size;
    }
    uint64_t cap() const { return cap_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }

  private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t cap_ = 0, used_ = 0, peak_ = 0;
};

struct Move {
    uint64_t src, dst, len;  // hit slots
};

// Workgroup b runs moves [first[b], first[b+1]) in order.  Each tile is read
// into LDS before any lane writes it back, so a move to lower addresses that
// overlaps its own source is exact.
__global__ __launch_bounds__(JTPB) void join_kernel(const Move* moves, const uint32_t* first, int64_t* pos,
                                                    uint16_t* cnt) {
    __shared__ int64_t s_pos[JTPB * JV];
    __shared__ uint16_t s_cnt[JTPB * JV];
    const uint32_t end = first[blockIdx.x + 1];
    for (uint32_t i = first[blockIdx.x]; i < end; ++i) {
        const Move mv = moves[i];
        for (uint64_t b = 0; b < mv.len; b += JTPB * JV) {
#pragma unroll
            for (int u = 0; u < JV; ++u) {
                const uint64_t j = b + (uint64_t)u * JTPB + threadIdx.x;
                if (j < mv.len) {
                    s_pos[u * JTPB + threadIdx.x] = pos[mv.src + j];
                    s_cnt[u * JTPB + threadIdx.x] = cnt[mv.src + j];
                }
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < JV; ++u) {
                const uint64_t j = b + (uint64_t)u * JTPB + threadIdx.x;
                if (j < mv.len) {
                    pos[mv.dst + j] = s_pos[u * JTPB + threadIdx.x];
                    cnt[mv.dst + j] = s_cnt[u * JTPB + threadIdx.x];
                }
            }
            __syncthreads();
        }
    }
}

struct Query {
    uint64_t id = 0;
    std::vector<uint8_t> codes;
    uint32_t m = 0, k = 0;
    // engine thread only
    ScanPlan plan;
    bool sized = false;
    uint64_t cap = 0;                 // hit slots per chunk segment
    uint64_t region = kNone;          // C * cap slots
    uint64_t image = kNone, image_units = 0;
    uint32_t enqueued = 0, done = 0;  // chunk steps launched / seen
    std::vector<uint64_t> hits;       // per chunk
    std::vector<uint64_t> extra;      // per chunk: exact segment of a re-scan, or kNone
    std::vector<uint32_t> rescan;     // chunks waiting for a re-scan
    uint64_t result = kNone;          // separate result region (total slots), or kNone
    uint64_t total = 0;
    // published under the server mutex
    int32_t state = PM_QUERY_WAITING, error = PM_OK;
    uint64_t n_hits = 0, out = kNone, out_len = 0;
    uint64_t arrival_ns = 0, admit_ns = 0, complete_ns = 0;
    uint32_t first_chunk = 0, reruns = 0;
};

struct Step {
    uint32_t chunk = 0, slot = 0;
    bool plain = false;  // one or two queries, run by the plain scan (no status words)
    std::vector<Query*> qs;
};

struct Join {
    hipEvent_t ev = nullptr;
    uint32_t slot = 0;
    std::vector<Query*> qs;
};

struct Pinned {
    void* p = nullptr;
    uint64_t bytes = 0;
    bool grow(uint64_t want) {
        if (want <= bytes) return true;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        const uint64_t b = want + want / 2;
        if (hipHostMalloc(&p, b, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            return false;
        }
        bytes = b;
        return true;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
};

}  // namespace

struct pm_server {
    // fixed after create
    int device = 0;
    const void* text = nullptr;
    uint64_t n = 0;
    uint32_t C = 1, max_active = 1024;
    uint64_t W = 0;  // windows per chunk
    // Admission sizes the workspace with bcfg.  When the caller left the
    // sub-range count to the library, bcfg holds the floor kAdmitSubRanges
    // and each step takes the most sub-ranges (up to the automatic choice
    // for its query count) that fit the workspace: the floor always fits,
    // since a step set is a subset of an admitted set and the workspace at a
    // fixed sub-range count only grows with the set.
    pm_batch_config bcfg{};
    bool adaptive_sub = false;
    hipStream_t main = nullptr, aux = nullptr;
    hipEvent_t step_ev[2] = {nullptr, nullptr};
    uint8_t* ws = nullptr;
    uint64_t ws_bytes = 0;
    void* rescan_ws = nullptr;
    uint64_t rescan_ws_bytes = 0;
    uint64_t* rescan_nh = nullptr;
    uint64_t* dev_nh[2] = {nullptr, nullptr};
    uint32_t* dev_st[2] = {nullptr, nullptr};
    Move* dev_moves = nullptr;
    uint32_t* dev_first = nullptr;
    uint64_t moves_cap = 0;
    uint4* images = nullptr;
    int64_t* pos = nullptr;
    uint16_t* cnt = nullptr;

    // engine thread only
    RangeAlloc img_pool, hit_pool;
    Pinned host_nh[2], host_st[2], desc[2], img_stage[2];
    uint64_t img_stage_used = 0;
    Pinned join_host[kJoinSlots];
    hipEvent_t join_ev[kJoinSlots] = {};
    bool join_busy[kJoinSlots] = {};
    std::deque<Query*> waiting;
    std::vector<Query*> active;
    std::deque<Step> inflight;
    std::vector<Query*> rescan_q, ready;
    std::deque<Join> joins;
    uint32_t next_chunk = 0;
    uint64_t step_no = 0;

    // shared, under mu
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Query*> incoming;
    std::vector<std::pair<uint64_t, uint64_t>> released;  // hit ranges to free
    std::unordered_map<uint64_t, std::unique_ptr<Query>> queries;
    uint64_t next_id = 1;
    bool stop = false, stopped = false;
    pm_status fatal = PM_OK;
    std::string fatal_detail;
    pm_server_stats st{};
    std::thread engine;

    // ----------------------------------------------------------------------
    void publish(Query* q, int32_t state, int32_t error) {
        std::lock_guard<std::mutex> lk(mu);
        // admitted and not complete: counted here rather than from the step
        // set, which a query leaves once its last chunk step is launched
        if (q->state == PM_QUERY_ACTIVE && state != PM_QUERY_ACTIVE) --st.active;
        q->state = state;
        q->error = error;
        if (state == PM_QUERY_ACTIVE) {
            q->admit_ns = clock_ns();
            ++st.admitted;
            ++st.active;
        } else if (state == PM_QUERY_DONE) {
            q->complete_ns = clock_ns();
            ++st.completed;
            if (q->m <= n) st.comparisons += (n - q->m + 1) * (uint64_t)q->m;
        } else if (state == PM_QUERY_FAILED) {
            q->complete_ns = clock_ns();
            ++st.failed;
        }
        cv_done.notify_all();
    }

    bool hip_ok(hipError_t e, const char* what) {
        if (e == hipSuccess) return true;
        fail_engine(PM_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
        return false;
    }

    void fail_engine(pm_status s, const std::string& what) {
        std::lock_guard<std::mutex> lk(mu);
        if (fatal == PM_OK) {
            fatal = s;
            fatal_detail = what;
        }
    }

    // The batch workspace of the admitted queries plus one more.
    uint64_t ws_need(const Query* extra_q) const {
        std::vector<uint32_t> ms;
        std::vector<uint64_t> caps;
        ms.reserve(active.size() + 1);
        caps.reserve(active.size() + 1);
        for (const Query* q : active) {
            ms.push_back(q->m);
            caps.push_back(q->cap);
        }
        if (extra_q) {
            ms.push_back(extra_q->m);
            caps.push_back(extra_q->cap);
        }
        return batch_ws_bytes(n, (uint32_t)ms.size(), ms.data(), caps.data(), &bcfg, false);
    }

    void size_query(Query* q) {
        if (q->sized) return;
        q->plan = build_plan(q->codes.data(), q->m, q->k, kBatchSurvival, /*window_at_zero=*/true);
        const double e = expected_hits(q->codes.data(), q->m, q->k, n);
        const double total = 2.0 * e + 64.0 * C;
        q->cap = (uint64_t)std::ceil(std::min(total, 1e18) / C);
        q->image_units = (q->m + 31) / 32;
        q->sized = true;
    }

    // Admit waiting queries in arrival order while a slot and memory are free.
    void admit() {
        const uint32_t slot = (uint32_t)(step_no & 1);
        while (!waiting.empty() && active.size() < max_active) {
            Query* q = waiting.front();
            size_query(q);
            const uint64_t region_len = (uint64_t)C * q->cap;
            uint32_t m1 = q->m;
            uint64_t c1 = q->cap;
            if (region_len > hit_pool.cap() || q->image_units > img_pool.cap() ||
                batch_ws_bytes(n, 1, &m1, &c1, &bcfg, false) > ws_bytes) {
                waiting.pop_front();
                publish(q, PM_QUERY_FAILED, PM_ERR_WORKSPACE);
                continue;
            }
            if (ws_need(q) > ws_bytes) break;
            const uint64_t img_bytes = 16 * q->image_units;
            if (img_stage_used + img_bytes > img_stage[slot].bytes) {
                if (img_stage_used > 0) break;  // next step
                if (!img_stage[slot].grow(std::max(kImageStage, img_bytes))) {
                    fail_engine(PM_ERR_HIP, "hipHostMalloc failed");
                    return;
                }
            }
            const uint64_t region = hit_pool.alloc(region_len);
            if (region == kNone) break;
            const uint64_t image = img_pool.alloc(q->image_units);
            if (image == kNone) {
                hit_pool.release(region, region_len);
                break;
            }
            q->region = region;
            q->image = image;
            uint8_t* stage = static_cast<uint8_t*>(img_stage[slot].p) + img_stage_used;
            std::memset(stage, 0, img_bytes);
            build_image(q->codes.data(), q->m, reinterpret_cast<uint32_t*>(stage));
            if (!hip_ok(hipMemcpyAsync(images + image, stage, img_bytes, hipMemcpyHostToDevice, main),
                        "hipMemcpyAsync"))
                return;
            img_stage_used += img_bytes;
            q->hits.assign(C, 0);
            q->extra.assign(C, kNone);
            active.push_back(q);
            waiting.pop_front();
            publish(q, PM_QUERY_ACTIVE, PM_OK);
        }
    }

    bool launch_step() {
        const uint32_t slot = (uint32_t)(step_no & 1), chunk = next_chunk;
        const uint32_t count = (uint32_t)active.size();
        // A step of one or two queries runs the plain scan of each into its
        // segment, one after the other on the step's stream (which keeps the
        // workspace theirs in turn): so few patterns make too few work items
        // to fill the chip in the batched kernel (a step over the genome
        // text: one query ~425 us batched, ~150 us plain; two ~410 us
        // batched, 280-380 us plain).  Overflow is then n_hits > cap, read
        // on the host.
        const bool plain = count <= 2 && ws_bytes >= pm_scan_workspace_bytes(n);
        if (plain) {
            for (uint32_t i = 0; i < count; ++i) {
                Query* q = active[i];
                const uint64_t out = q->region + (uint64_t)chunk * q->cap;
                const pm_status s = pm_scan(text, n, q->codes.data(), q->m, q->k, images + q->image,
                                            (uint64_t)chunk * W, std::min<uint64_t>(n, (uint64_t)(chunk + 1) * W),
                                            pos + out, cnt + out, q->cap, dev_nh[slot] + i, ws, ws_bytes, main);
                if (s != PM_OK) {
                    fail_engine(s, pm_last_error_detail());
                    return false;
                }
            }
            if (!host_nh[slot].grow(8ull * count) ||
                !hip_ok(hipMemcpyAsync(host_nh[slot].p, dev_nh[slot], 8ull * count, hipMemcpyDeviceToHost, main),
                        "hipMemcpyAsync") ||
                !hip_ok(hipEventRecord(step_ev[slot], main), "hipEventRecord"))
                return false;
            return end_step(slot, chunk, true);
        }
        std::vector<BatchEntry> ent(count);
        std::vector<uint32_t> ms(count);
        std::vector<uint64_t> caps(count);
        for (uint32_t i = 0; i < count; ++i) {
            Query* q = active[i];
            ent[i] = {q->codes.data(), q->m, q->k, &q->plan, q->image, q->region + (uint64_t)chunk * q->cap, q->cap};
            ms[i] = q->m;
            caps[i] = q->cap;
        }
        pm_batch_config scfg = bcfg;
        if (adaptive_sub) {
            uint32_t S = std::max(kAdmitSubRanges, batch_auto_sub_ranges(count, &bcfg));
            for (;;) {
                scfg.sub_ranges = S;
                if (S <= kAdmitSubRanges || batch_ws_bytes(n, count, ms.data(), caps.data(), &scfg, false) <= ws_bytes)
                    break;
                S = std::max(kAdmitSubRanges, S / 2);
            }
        }
        const uint64_t need = batch_desc_bytes(n, count, ms.data(), caps.data(), &scfg, false);
        if (!desc[slot].grow(need) || !host_nh[slot].grow(8ull * count) || !host_st[slot].grow(4ull * count)) {
            fail_engine(PM_ERR_HIP, "hipHostMalloc failed");
            return false;
        }
        BatchCall c;
        c.text_dev = text;
        c.n = n;
        c.count = count;
        c.entries = ent.data();
        c.images_dev = images;
        c.win_begin = (uint64_t)chunk * W;
        c.win_end = std::min<uint64_t>(n, (uint64_t)(chunk + 1) * W);
        c.pos_dev = pos;
        c.cnt_dev = cnt;
        c.n_hits_dev = dev_nh[slot];
        c.status_dev = dev_st[slot];
        c.ws_dev = ws;
        c.ws_bytes = ws_bytes;
        c.cfg = &scfg;
        c.desc_host = static_cast<uint8_t*>(desc[slot].p);
        c.desc_host_bytes = desc[slot].bytes;
        c.stream = main;
        const pm_status s = batch_run(c);
        if (s != PM_OK) {
            fail_engine(s, pm_last_error_detail());
            return false;
        }
        if (!hip_ok(hipMemcpyAsync(host_nh[slot].p, dev_nh[slot], 8ull * count, hipMemcpyDeviceToHost, main),
                    "hipMemcpyAsync") ||
            !hip_ok(hipMemcpyAsync(host_st[slot].p, dev_st[slot], 4ull * count, hipMemcpyDeviceToHost, main),
                    "hipMemcpyAsync") ||
            !hip_ok(hipEventRecord(step_ev[slot], main), "hipEventRecord"))
            return false;
        return end_step(slot, chunk, false);
    }

    // The bookkeeping of a launched step.
    bool end_step(uint32_t slot, uint32_t chunk, bool plain) {
        const uint32_t count = (uint32_t)active.size();
        {
            std::lock_guard<std::mutex> lk(mu);
            st.peak_active = std::max(st.peak_active, count);
        }
        Step stp;
        stp.chunk = chunk;
        stp.slot = slot;
        stp.plain = plain;
        stp.qs = active;
        for (Query* q : active)
            if (q->enqueued++ == 0) {
                std::lock_guard<std::mutex> lk(mu);
                q->first_chunk = chunk;
            }
        inflight.push_back(std::move(stp));
        // queries that have now been through every chunk leave the step set
        active.erase(std::remove_if(active.begin(), active.end(), [&](Query* q) { return q->enqueued == C; }),
                     active.end());
        next_chunk = (chunk + 1) % C;
        ++step_no;
        img_stage_used = 0;
        std::lock_guard<std::mutex> lk(mu);
        ++st.steps;
        return true;
    }

    // Poll (or wait for) an event, running the joins' bookkeeping meanwhile.
    bool wait_event(hipEvent_t ev) {
        while (true) {
            const hipError_t e = hipEventQuery(ev);
            if (e == hipSuccess) return true;
            if (e != hipErrorNotReady) return hip_ok(e, "hipEventQuery");
            if (!poll_joins(false)) return false;
            std::this_thread::yield();
        }
    }

    bool finish_step() {
        Step& stp = inflight.front();
        if (!wait_event(step_ev[stp.slot])) return false;
        const uint64_t* nh = static_cast<const uint64_t*>(host_nh[stp.slot].p);
        const uint32_t* sf = static_cast<const uint32_t*>(host_st[stp.slot].p);
        for (size_t i = 0; i < stp.qs.size(); ++i) {
            Query* q = stp.qs[i];
            q->hits[stp.chunk] = nh[i];
            if (stp.plain ? nh[i] > q->cap : sf[i] != 0) {
                if (q->rescan.empty()) rescan_q.push_back(q);
                q->rescan.push_back(stp.chunk);
            }
            if (++q->done == C && q->rescan.empty()) ready.push_back(q);
        }
        inflight.pop_front();
        return true;
    }

    // Re-scan overflowed chunks with the plain kernel into exact segments.
    bool run_rescans(bool& progress) {
        for (size_t i = 0; i < rescan_q.size();) {
            Query* q = rescan_q[i];
            std::vector<uint32_t> left;
            for (uint32_t c : q->rescan) {
                const uint64_t h = q->hits[c];
                uint64_t target = q->region + (uint64_t)c * q->cap;
                if (h > q->cap) {
                    target = hit_pool.alloc(h);
                    if (target == kNone) {
                        left.push_back(c);
                        continue;
                    }
                    q->extra[c] = target;
                }
                const pm_status s =
                    pm_scan(text, n, q->codes.data(), q->m, q->k, images + q->image, (uint64_t)c * W,
                            std::min<uint64_t>(n, (uint64_t)(c + 1) * W), pos + target, cnt + target, h, rescan_nh,
                            rescan_ws, rescan_ws_bytes, aux);
                if (s != PM_OK) {
                    fail_engine(s, pm_last_error_detail());
                    return false;
                }
                progress = true;
                std::lock_guard<std::mutex> lk(mu);
                ++q->reruns;
                ++st.reruns;
            }
            q->rescan = std::move(left);
            if (q->rescan.empty()) {
                if (q->done == C) ready.push_back(q);
                rescan_q.erase(rescan_q.begin() + i);
            } else {
                ++i;
            }
        }
        return true;
    }

    // Join the chunk segments of complete queries, one launch for all of them.
    // A small result is joined in place by one workgroup (moves in chunk
    // order); a large one gets a region of its own and its moves are cut into
    // pieces, one workgroup each.
    bool run_joins(bool& progress) {
        if (ready.empty()) return true;
        uint32_t slot = kJoinSlots;
        for (uint32_t i = 0; i < kJoinSlots; ++i)
            if (!join_busy[i]) {
                slot = i;
                break;
            }
        if (slot == kJoinSlots) return true;  // all staging slots in use; later
        std::vector<Move> moves;
        std::vector<uint32_t> first{0};
        std::vector<Query*> qs, later;
        for (Query* q : ready) {
            uint64_t total = 0;
            bool in_place = true;
            for (uint32_t c = 0; c < C; ++c) {
                if (total > (uint64_t)c * q->cap) in_place = false;
                total += q->hits[c];
            }
            if (total > (uint64_t)C * q->cap) in_place = false;
            // moves this query needs at most: C in place, or up to C + 4097 pieces
            const uint64_t piece = std::max<uint64_t>(kPiece, total / 4096 + 1);
            const uint64_t worst = in_place && total < kBigJoin ? C : C + total / piece + 1;
            if (moves.size() + worst > moves_cap) {
                later.push_back(q);
                continue;
            }
            // segments already one after another from the region's start
            // (always with one chunk): the result is where it is
            bool contiguous = in_place;
            for (uint64_t c = 0, d0 = 0; c < C && contiguous; ++c) {
                const uint64_t src = q->extra[c] != kNone ? q->extra[c] : q->region + c * q->cap;
                if (q->hits[c] && src != q->region + d0) contiguous = false;
                d0 += q->hits[c];
            }
            uint64_t base = q->region;
            bool separate = !contiguous && (!in_place || total >= kBigJoin);
            if (separate) {
                q->result = hit_pool.alloc(total);
                if (q->result == kNone) {
                    if (!in_place) {
                        later.push_back(q);
                        continue;
                    }
                    separate = false;  // no room: in place, one workgroup
                } else {
                    base = q->result;
                }
            }
            q->total = total;
            uint64_t d = 0;
            for (uint32_t c = 0; c < C; ++c) {
                const uint64_t h = q->hits[c];
                const uint64_t src = q->extra[c] != kNone ? q->extra[c] : q->region + (uint64_t)c * q->cap;
                if (h && src != base + d) {
                    if (separate) {
                        for (uint64_t o = 0; o < h; o += piece) {
                            moves.push_back({src + o, base + d + o, std::min<uint64_t>(piece, h - o)});
                            first.push_back((uint32_t)moves.size());
                        }
                    } else {
                        moves.push_back({src, base + d, h});
                    }
                }
                d += h;
            }
            if (!separate && first.back() != moves.size()) first.push_back((uint32_t)moves.size());
            qs.push_back(q);
        }
        ready.swap(later);
        if (qs.empty()) return true;
        progress = true;
        const uint32_t blocks = (uint32_t)first.size() - 1;
        const uint64_t bytes = sizeof(Move) * moves.size() + 4 * first.size();
        if (!join_host[slot].grow(std::max<uint64_t>(bytes, 4096))) {
            fail_engine(PM_ERR_HIP, "hipHostMalloc failed");
            return false;
        }
        uint8_t* h = static_cast<uint8_t*>(join_host[slot].p);
        std::memcpy(h, moves.data(), sizeof(Move) * moves.size());
        std::memcpy(h + sizeof(Move) * moves.size(), first.data(), 4 * first.size());
        if (blocks > 0) {
            if (!hip_ok(hipMemcpyAsync(dev_moves, h, sizeof(Move) * moves.size(), hipMemcpyHostToDevice, aux),
                        "hipMemcpyAsync") ||
                !hip_ok(hipMemcpyAsync(dev_first, h + sizeof(Move) * moves.size(), 4 * first.size(),
                                       hipMemcpyHostToDevice, aux),
                        "hipMemcpyAsync"))
                return false;
            join_kernel<<<blocks, JTPB, 0, aux>>>(dev_moves, dev_first, pos, cnt);
            if (!hip_ok(hipGetLastError(), "join_kernel")) return false;
        }
        if (!hip_ok(hipEventRecord(join_ev[slot], aux), "hipEventRecord")) return false;
        join_busy[slot] = true;
        Join j;
        j.ev = join_ev[slot];
        j.slot = slot;
        j.qs = std::move(qs);
        joins.push_back(std::move(j));
        return true;
    }

    // Publish the queries of finished joins and free what they no longer need.
    bool poll_joins(bool block) {
        while (!joins.empty()) {
            Join& j = joins.front();
            const hipError_t e = hipEventQuery(j.ev);
            if (e == hipErrorNotReady) {
                if (!block) return true;
                std::this_thread::yield();
                continue;
            }
            if (!hip_ok(e, "hipEventQuery")) return false;
            for (Query* q : j.qs) {
                for (uint32_t c = 0; c < C; ++c)
                    if (q->extra[c] != kNone) hit_pool.release(q->extra[c], q->hits[c]);
                img_pool.release(q->image, q->image_units);
                q->image = kNone;
                uint64_t out = q->region, out_len = (uint64_t)C * q->cap;
                if (q->result != kNone) {
                    hit_pool.release(q->region, out_len);
                    out = q->result;
                    out_len = q->total;
                }
                if (q->total == 0) {
                    hit_pool.release(out, out_len);
                    out = kNone;
                    out_len = 0;
                }
                q->region = kNone;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    q->n_hits = q->total;
                    q->out = out;
                    q->out_len = out_len;
                }
                publish(q, PM_QUERY_DONE, PM_OK);
            }
            join_busy[j.slot] = false;
            joins.pop_front();
        }
        return true;
    }

    void take_shared(bool& stop_now) {
        std::vector<std::pair<uint64_t, uint64_t>> rel;
        {
            std::lock_guard<std::mutex> lk(mu);
            while (!incoming.empty()) {
                waiting.push_back(incoming.front());
                incoming.pop_front();
            }
            rel.swap(released);
            stop_now = stop;
        }
        for (auto& r : rel) hit_pool.release(r.first, r.second);
    }

    bool busy() const {
        return !active.empty() || !inflight.empty() || !joins.empty() || !ready.empty() || !rescan_q.empty();
    }

    void update_stats() {
        std::lock_guard<std::mutex> lk(mu);
        st.waiting = (uint32_t)(waiting.size() + incoming.size());
        st.hit_slots_used = hit_pool.used();
        st.hit_slots_peak = hit_pool.peak();
    }

    void run() {
        if (hipSetDevice(device) != hipSuccess) {
            fail_engine(PM_ERR_HIP, "hipSetDevice failed in the engine thread");
        }
        bool ok = fatal == PM_OK;
        while (ok) {
            bool stop_now = false;
            take_shared(stop_now);
            if (stop_now) break;
            admit();
            if (fatal != PM_OK) break;
            bool launched = false;
            if (!active.empty()) {
                if (!launch_step()) break;
                launched = true;
            }
            if (!inflight.empty() && (inflight.size() >= 2 || !launched))
                if (!finish_step()) break;
            bool progress = launched;
            if (!run_rescans(progress) || !run_joins(progress) || !poll_joins(false)) break;
            update_stats();
            if (!launched && inflight.empty()) {
                if (!joins.empty()) {
                    if (!poll_joins(true)) break;
                    continue;
                }
                if (!progress) {
                    // nothing runs: wait for a submission or a release
                    std::unique_lock<std::mutex> lk(mu);
                    cv_work.wait_for(lk, std::chrono::milliseconds(busy() ? 1 : 20),
                                     [&] { return stop || !incoming.empty() || !released.empty(); });
                }
            }
        }
        // drain the GPU, then fail what did not finish
        (void)hipStreamSynchronize(main);
        (void)hipStreamSynchronize(aux);
        if (fatal == PM_OK) poll_joins(true);
        std::vector<Query*> open;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto& kv : queries)
                if (kv.second->state == PM_QUERY_WAITING || kv.second->state == PM_QUERY_ACTIVE)
                    open.push_back(kv.second.get());
            stopped = true;
        }
        const int32_t why = fatal != PM_OK ? fatal : PM_ERR_BUSY;
        for (Query* q : open) publish(q, PM_QUERY_FAILED, why);
    }

    void info_of(const Query* q, pm_query_info* info) const {
        std::memset(info, 0, sizeof(*info));
        info->state = q->state;
        info->error = q->error;
        info->n_hits = q->n_hits;
        if (q->state == PM_QUERY_DONE && q->out != kNone) {
            info->pos_dev = pos + q->out;
            info->cnt_dev = cnt + q->out;
        }
        info->arrival_ns = q->arrival_ns;
        info->admit_ns = q->admit_ns;
        info->complete_ns = q->complete_ns;
        info->first_chunk = q->first_chunk;
        info->reruns = q->reruns;
    }
};

namespace {

struct ArenaPlan {
    uint64_t ws, rescan_ws, rescan_nh, nh[2], st[2], moves, first, images, hits, hit_slots, bytes_min;
    uint64_t moves_cap;
};

ArenaPlan plan_arena(uint64_t n, uint64_t arena_bytes, uint32_t C, uint32_t max_active, uint64_t ws_bytes) {
    ArenaPlan a{};
    uint64_t off = 0;
    a.ws = off;
    off = align256(off + ws_bytes);
    a.rescan_ws = off;
    off = align256(off + pm_scan_workspace_bytes(n));
    a.rescan_nh = off;
    off = align256(off + 8);
    for (int i = 0; i < 2; ++i) {
        a.nh[i] = off;
        off = align256(off + 8ull * max_active);
        a.st[i] = off;
        off = align256(off + 4ull * max_active);
    }
    a.moves_cap = (uint64_t)max_active * C + 16384;
    a.moves = off;
    off = align256(off + sizeof(Move) * a.moves_cap);
    a.first = off;
    off = align256(off + 4ull * (a.moves_cap + 1));
    a.images = off;
    const uint64_t img_bytes = std::max<uint64_t>(1ull << 20, 4096ull * max_active);
    off = align256(off + img_bytes);
    a.hits = off;
    // at least 64 hit slots per chunk of one query
    a.bytes_min = off + 10ull * 64 * C + 256;
    a.hit_slots = arena_bytes > off + 256 ? (arena_bytes - off - 256) / 10 : 0;
    return a;
}

void normalise(const pm_server_config* cfg, uint64_t arena_bytes, uint32_t& C, uint32_t& max_active,
               uint64_t& ws_bytes, pm_batch_config& b, bool* adaptive = nullptr) {
    C = cfg && cfg->chunks ? cfg->chunks : 1;
    max_active = cfg && cfg->max_active ? cfg->max_active : 1024;
    ws_bytes = cfg && cfg->workspace_bytes ? cfg->workspace_bytes : align256(arena_bytes / 4);
    std::memset(&b, 0, sizeof(b));
    if (cfg) b = cfg->batch;
    // Admission works at a fixed sub-range count, which keeps the batch
    // workspace monotone in the query set; steps may take more (see
    // pm_server::adaptive_sub).
    if (adaptive) *adaptive = b.sub_ranges == 0;
    if (b.sub_ranges == 0) b.sub_ranges = kAdmitSubRanges;
}

}  // namespace

extern "C" {

uint64_t pm_server_now_ns(void) { return clock_ns(); }

uint64_t pm_server_min_arena_bytes(uint64_t n, const pm_server_config* cfg) {
    uint32_t C, max_active;
    uint64_t ws;
    pm_batch_config b;
    normalise(cfg, 0, C, max_active, ws, b);
    if (!(cfg && cfg->workspace_bytes)) ws = 1ull << 20;
    return plan_arena(n, 0, C, max_active, ws).bytes_min;
}

pm_status pm_server_create(const void* text_dev, uint64_t n, void* arena_dev, uint64_t arena_bytes,
                           const pm_server_config* cfg, void* stream, pm_server** out) {
    if (!text_dev || !arena_dev || !out) return set_error(PM_ERR_ARG, "null pointer");
    *out = nullptr;
    if (reinterpret_cast<uintptr_t>(arena_dev) % 256 != 0) return set_error(PM_ERR_ARG, "arena must be 256-byte aligned");
    if (reinterpret_cast<uintptr_t>(text_dev) % 16 != 0) return set_error(PM_ERR_ARG, "text_dev must be 16-byte aligned");
    if (n == 0) return set_error(PM_ERR_ARG, "empty text");
    uint32_t C, max_active;
    uint64_t ws_bytes;
    pm_batch_config b;
    bool adaptive = false;
    normalise(cfg, arena_bytes, C, max_active, ws_bytes, b, &adaptive);
    if (C > 4096) return set_error(PM_ERR_ARG, "chunks above 4096");
    if (max_active > (1u << 20)) return set_error(PM_ERR_ARG, "max_active above 2^20");
    const ArenaPlan a = plan_arena(n, arena_bytes, C, max_active, ws_bytes);
    if (arena_bytes < a.bytes_min)
        return set_error(PM_ERR_WORKSPACE, "arena too small: need at least " + std::to_string(a.bytes_min) + " bytes");

    std::unique_ptr<pm_server> s(new pm_server);
    if (hipGetDevice(&s->device) != hipSuccess) return set_error(PM_ERR_HIP, "hipGetDevice failed");
    s->text = text_dev;
    s->n = n;
    s->C = C;
    s->max_active = max_active;
    s->W = (n + C - 1) / C;
    s->bcfg = b;
    s->adaptive_sub = adaptive;
    s->main = reinterpret_cast<hipStream_t>(stream);
    uint8_t* base = static_cast<uint8_t*>(arena_dev);
    s->ws = base + a.ws;
    s->ws_bytes = ws_bytes;
    s->rescan_ws = base + a.rescan_ws;
    s->rescan_ws_bytes = a.rescan_nh - a.rescan_ws;
    s->rescan_nh = reinterpret_cast<uint64_t*>(base + a.rescan_nh);
    for (int i = 0; i < 2; ++i) {
        s->dev_nh[i] = reinterpret_cast<uint64_t*>(base + a.nh[i]);
        s->dev_st[i] = reinterpret_cast<uint32_t*>(base + a.st[i]);
    }
    s->dev_moves = reinterpret_cast<Move*>(base + a.moves);
    s->dev_first = reinterpret_cast<uint32_t*>(base + a.first);
    s->moves_cap = a.moves_cap;
    s->images = reinterpret_cast<uint4*>(base + a.images);
    s->img_pool.reset((a.hits - a.images) / 16);
    s->pos = reinterpret_cast<int64_t*>(base + a.hits);
    s->cnt = reinterpret_cast<uint16_t*>(base + a.hits + 8 * a.hit_slots);
    s->hit_pool.reset(a.hit_slots);
    s->st.chunks = C;
    s->st.hit_slots = a.hit_slots;
    s->st.workspace_bytes = ws_bytes;
    hipError_t e = hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking);
    for (int i = 0; e == hipSuccess && i < 2; ++i) e = hipEventCreateWithFlags(&s->step_ev[i], hipEventDisableTiming);
    for (uint32_t i = 0; e == hipSuccess && i < kJoinSlots; ++i)
        e = hipEventCreateWithFlags(&s->join_ev[i], hipEventDisableTiming);
    if (e != hipSuccess) {
        pm_status r = set_error(PM_ERR_HIP, std::string("server set-up: ") + hipGetErrorString(e));
        for (auto& ev : s->step_ev)
            if (ev) (void)hipEventDestroy(ev);
        for (auto& ev : s->join_ev)
            if (ev) (void)hipEventDestroy(ev);
        if (s->aux) (void)hipStreamDestroy(s->aux);
        return r;
    }
    pm_server* raw = s.release();
    raw->engine = std::thread([raw] {
        try {
            raw->run();
        } catch (const std::exception& ex) {
            raw->fail_engine(PM_ERR_HIP, std::string("engine stopped: ") + ex.what());
            (void)hipStreamSynchronize(raw->main);
            (void)hipStreamSynchronize(raw->aux);
            std::lock_guard<std::mutex> lk(raw->mu);
            for (auto& kv : raw->queries)
                if (kv.second->state < PM_QUERY_DONE) {
                    if (kv.second->state == PM_QUERY_ACTIVE) --raw->st.active;
                    kv.second->state = PM_QUERY_FAILED;
                    kv.second->error = PM_ERR_HIP;
                }
            raw->stopped = true;
            raw->cv_done.notify_all();
        }
    });
    *out = raw;
    return PM_OK;
}

pm_status pm_server_submit(pm_server* srv, const uint8_t* codes, uint32_t m, uint32_t k, uint64_t arrival_ns,
                           uint64_t* id_out) {
    if (!srv || !codes || !id_out) return set_error(PM_ERR_ARG, "null pointer");
    if (m == 0) return set_error(PM_ERR_ARG, "empty pattern (m = 0)");
    if (k > 65535) return set_error(PM_ERR_ARG, "k above 65535 (counts are 16-bit)");
    for (uint32_t j = 0; j < m; ++j)
        if (codes[j] > 15) return set_error(PM_ERR_SYMBOL, "pattern code above 15 at " + std::to_string(j));
    std::unique_ptr<Query> q(new Query);
    q->codes.assign(codes, codes + m);
    q->m = m;
    q->k = k;
    q->arrival_ns = arrival_ns ? arrival_ns : clock_ns();
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->fatal != PM_OK) return set_error(srv->fatal, "server stopped: " + srv->fatal_detail);
    if (srv->stop || srv->stopped) return set_error(PM_ERR_BUSY, "server is stopping");
    q->id = srv->next_id++;
    *id_out = q->id;
    srv->incoming.push_back(q.get());
    srv->queries.emplace(q->id, std::move(q));
    ++srv->st.submitted;
    srv->cv_work.notify_all();
    return PM_OK;
}

pm_status pm_server_poll(pm_server* srv, uint64_t id, pm_query_info* info) {
    if (!srv || !info) return set_error(PM_ERR_ARG, "null pointer");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->queries.find(id);
    if (it == srv->queries.end()) return set_error(PM_ERR_NOT_FOUND, "unknown query id " + std::to_string(id));
    srv->info_of(it->second.get(), info);
    return PM_OK;
}

pm_status pm_server_wait(pm_server* srv, uint64_t id, int64_t timeout_ms, pm_query_info* info) {
    if (!srv) return set_error(PM_ERR_ARG, "null pointer");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto finished = [&] {
        auto it = srv->queries.find(id);
        return it == srv->queries.end() || it->second->state >= PM_QUERY_DONE;
    };
    if (timeout_ms < 0)
        srv->cv_done.wait(lk, finished);
    else if (!srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), finished))
        return set_error(PM_ERR_BUSY, "query " + std::to_string(id) + " not finished");
    auto it = srv->queries.find(id);
    if (it == srv->queries.end()) return set_error(PM_ERR_NOT_FOUND, "unknown query id " + std::to_string(id));
    if (info) srv->info_of(it->second.get(), info);
    return PM_OK;
}

pm_status pm_server_release(pm_server* srv, uint64_t id) {
    if (!srv) return set_error(PM_ERR_ARG, "null pointer");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->queries.find(id);
    if (it == srv->queries.end()) return set_error(PM_ERR_NOT_FOUND, "unknown query id " + std::to_string(id));
    Query* q = it->second.get();
    if (q->state < PM_QUERY_DONE) return set_error(PM_ERR_BUSY, "query " + std::to_string(id) + " not finished");
    if (q->out != kNone) srv->released.push_back({q->out, q->out_len});
    srv->queries.erase(it);
    srv->cv_work.notify_all();
    return PM_OK;
}

pm_status pm_server_drain(pm_server* srv, int64_t timeout_ms) {
    if (!srv) return set_error(PM_ERR_ARG, "null pointer");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto all_done = [&] {
        for (auto& kv : srv->queries)
            if (kv.second->state < PM_QUERY_DONE) return false;
        return true;
    };
    if (timeout_ms < 0)
        srv->cv_done.wait(lk, all_done);
    else if (!srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), all_done))
        return set_error(PM_ERR_BUSY, "queries still running");
    return PM_OK;
}

pm_status pm_server_stats_get(pm_server* srv, pm_server_stats* out) {
    if (!srv || !out) return set_error(PM_ERR_ARG, "null pointer");
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->st;
    return PM_OK;
}

const char* pm_server_error_detail(pm_server* srv) {
    if (!srv) return "";
    std::lock_guard<std::mutex> lk(srv->mu);
    return srv->fatal_detail.c_str();
}

pm_status pm_server_destroy(pm_server* srv) {
    if (!srv) return PM_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->engine.joinable()) srv->engine.join();
    for (int i = 0; i < 2; ++i) {
        srv->host_nh[i].release();
        srv->host_st[i].release();
        srv->desc[i].release();
        srv->img_stage[i].release();
        (void)hipEventDestroy(srv->step_ev[i]);
    }
    for (uint32_t i = 0; i < kJoinSlots; ++i) {
        srv->join_host[i].release();
        (void)hipEventDestroy(srv->join_ev[i]);
    }
    (void)hipStreamDestroy(srv->aux);
    delete srv;
    return PM_OK;
}

}  // extern "C"
