// Host-code check under AddressSanitizer and UndefinedBehaviorSanitizer:
// the library's plain C++ (pattern parsing, Table 3 masks, the filter
// planner, the pattern image, the expected-hits estimate, the FASTA parser
// and its window ranges) and the oracle's C (parse, counts, the threaded
// scan), driven over seeded random and edge-case inputs.  Built with g++
// (no device code) by tests/test_host_sanitizers.py; exits 0 when every
// check holds and the sanitizers report nothing.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/pmscan.h"
#include "../../paper_1611_06115_amd/csrc/plan.hpp"

namespace pm {
// the library's error hook, as the FASTA parser expects it
pm_status set_error(pm_status s, const std::string&) { return s; }
}  // namespace pm

extern "C" {
// oracle.c
int64_t pmo_parse(const char* pattern, uint64_t len, uint8_t* sets, uint64_t cap);
int64_t pmo_first_bad(const uint8_t* text, uint64_t n);
int pmo_counts(const uint8_t* text, uint64_t n, const uint8_t* sets, uint64_t m, uint32_t* out);
int64_t pmo_scan_range(const uint8_t* text, uint64_t n, const uint8_t* sets, uint64_t m, uint64_t k,
                       uint64_t win_begin, uint64_t win_end, int threads, int64_t* pos, uint16_t* cnt,
                       uint64_t capacity);
}

static int failures = 0;
#define CHECK(x)                                                        \
    do {                                                                \
        if (!(x)) {                                                     \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__); \
            ++failures;                                                 \
        }                                                               \
    } while (0)

int main() {
    std::mt19937_64 rng(1611);
    const char* symbols = "ACGTMRWSYKVHDBN-acgtn";
    // pattern parsing, plans, images, expected hits
    for (int it = 0; it < 1200; ++it) {
        const uint32_t m = 1 + (uint32_t)(rng() % (it < 1000 ? 300 : 6000));
        std::string pat;
        for (uint32_t j = 0; j < m; ++j) {
            if (rng() % 50 == 0) {
                pat += "[";
                pat += "ACGT"[rng() % 4];
                pat += "ACGT"[rng() % 4];
                pat += "]";
            } else {
                pat += symbols[rng() % std::strlen(symbols)];
            }
        }
        std::vector<uint8_t> codes;
        std::string err;
        const int rc = pm::parse_pattern(pat.data(), pat.size(), codes, err);
        CHECK(rc == 0);
        CHECK(codes.size() == m);
        for (uint32_t k : {0u, 1u, 2u, 4u, 8u, 16u, m, m + 3}) {
            const pm::ScanPlan p = pm::build_plan(codes.data(), m, k);
            CHECK(p.n_slots <= (uint32_t)pm::kMaxSlots);
            const pm::ScanPlan pz = pm::build_plan(codes.data(), m, k, 4e-5, true);
            CHECK(pz.fword == 0);
            const double e = pm::expected_hits(codes.data(), m, k, 100000000ull);
            CHECK(e >= 0.0);
        }
        std::vector<uint32_t> img(pm::image_words(m) + 1, 0xABCDu);
        pm::build_image(codes.data(), m, img.data());
        CHECK(img.back() == 0xABCDu);  // nothing written past the image
    }
    // malformed patterns are errors, never crashes
    for (const char* bad : {"[", "[]", "AC[GT", "AXG", "[A-]", "]"}) {
        std::vector<uint8_t> codes;
        std::string err;
        CHECK(pm::parse_pattern(bad, std::strlen(bad), codes, err) != 0);
    }
    // FASTA parsing and window ranges
    for (int it = 0; it < 400; ++it) {
        std::string fa;
        const int recs = 1 + (int)(rng() % 5);
        for (int r = 0; r < recs; ++r) {
            fa += ">rec" + std::to_string(r) + " x\n";
            const int len = (int)(rng() % 3000);
            for (int i = 0; i < len; ++i) {
                fa += "ACGTacgtNNRY-"[rng() % (i % 97 < 90 ? 8 : 13)];
                if (rng() % 61 == 0) fa += (rng() % 2) ? "\n" : "\r\n";
            }
            fa += "\n";
        }
        pm_fasta* f = nullptr;
        CHECK(pm_fasta_parse(fa.data(), fa.size(), &f) == PM_OK && f != nullptr);
        if (!f) continue;
        for (uint32_t m : {1u, 2u, 17u, 500u, 5000u}) {
            uint64_t count = 0;
            CHECK(pm_fasta_window_ranges(f, m, nullptr, nullptr, 0, &count) == PM_OK);
            std::vector<uint64_t> b(count + 1), e(count + 1);
            CHECK(pm_fasta_window_ranges(f, m, b.data(), e.data(), count, &count) == PM_OK);
            for (uint64_t r = 0; r < count; ++r) {
                CHECK(b[r] < e[r] && e[r] + m - 1 <= pm_fasta_length(f));
                if (r) CHECK(e[r - 1] <= b[r]);
            }
        }
        pm_fasta_free(f);
    }
    for (const char* bad : {"ACGT\n", ">r\nAC?T\n", "", ";only a comment\n"}) {
        pm_fasta* f = nullptr;
        CHECK(pm_fasta_parse(bad, std::strlen(bad), &f) != PM_OK && f == nullptr);
    }
    // the oracle: parse, counts and the threaded scan agree on random inputs
    for (int it = 0; it < 300; ++it) {
        const uint64_t n = rng() % 5000;
        std::vector<uint8_t> text(n);
        for (auto& c : text) c = (uint8_t)"ACGT"[rng() % 4];
        std::string pat;
        const uint32_t m = 1 + (uint32_t)(rng() % 40);
        for (uint32_t j = 0; j < m; ++j) pat += symbols[rng() % 16];
        std::vector<uint8_t> sets(m);
        CHECK(pmo_parse(pat.data(), pat.size(), sets.data(), m) == (int64_t)m);
        CHECK(pmo_first_bad(text.data(), n) == -1);
        const uint64_t nw = n >= m ? n - m + 1 : 0;
        std::vector<uint32_t> counts(nw + 1);
        CHECK(pmo_counts(text.data(), n, sets.data(), m, counts.data()) == 0);
        const uint64_t k = rng() % (m + 2);
        uint64_t want = 0;
        for (uint64_t i = 0; i < nw; ++i) want += counts[i] <= k;
        std::vector<int64_t> pos(want + 1);
        std::vector<uint16_t> cnt(want + 1);
        const int64_t got = pmo_scan_range(text.data(), n, sets.data(), m, k, 0, UINT64_MAX, 1 + (int)(rng() % 8),
                                           pos.data(), cnt.data(), want);
        CHECK(got == (int64_t)want);
        for (int64_t h = 0; h < got; ++h) CHECK(counts[pos[h]] == cnt[h]);
    }
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("host check ok\n");
    return 0;
}
