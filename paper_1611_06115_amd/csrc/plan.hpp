// plan.hpp -- host-side pattern encoding and scan planning (private to
// libpmscan).  Shared between the host code and the kernels: only the plain
// structs below, which travel to the GPU as kernel arguments.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace pm {

// Filter slots are evaluated in groups of 8 and there are at most 64.
constexpr int kMaxSlots = 64;
// Threads per workgroup of the scan kernels.
constexpr int kThreads = 256;

// A filter slot is one pattern position inside the 64-position filter window,
// at offset 32*q + r from its start (q = 0 or 1).
//  - singleton filter (exhaustive = 0): slot = c | q << 2 | r << 3, c the
//    position's base (Table 1 code); the slot count is a multiple of 8.
//  - exhaustive filter (exhaustive = 1): slot = mm | q << 4 | r << 5, mm the
//    position's Table 3 row (bit t set <=> text code t mismatches); mm = 0
//    pads the last group of 8 and never mismatches.
struct ScanPlan {
    uint32_t m;          // pattern length
    uint32_t k;          // mismatch budget
    int32_t keff;        // k minus the '-' positions (they always mismatch)
    uint32_t n_dash;     // number of '-' positions
    uint32_t n_slots;    // filter slots used (multiple of 8; 0 = no filter)
    uint32_t levels;     // bit-sliced counter levels L, 2^L >= keff + 1
    uint32_t init;       // counter start value 2^L - (keff + 1)
    uint32_t exhaustive; // the slots hold every countable position (exact counts)
    uint32_t fword;      // filter window start, in 32-base blocks (even)
    uint32_t nchunks;    // ceil(m / 32): chunks of the pattern image
    uint32_t singles;    // bit c set: the singleton plane of base c is used
    uint32_t n_sets;     // singleton filter: slot sets (32-bit words in `slot`)
    uint32_t n_groups;   // singleton filter: the first 2 * n_groups sets are full
    // Exhaustive filter: one 16-bit slot per countable position, two per word
    // (slot 2i in the low half of word i), mm | q << 4 | r << 5 (Table 3 row,
    // word q and shift r of its offset in the filter window).  Singleton
    // filter: n_sets words, each a set of up to 4 positions whose class is the
    // same single base c and word q: c | q << 2 | count << 3 | r_u << (6 + 5u).
    // Pairs of full sets make the groups of 8 slots; the sets after them are
    // the tail.
    uint32_t slot[kMaxSlots / 2];
};

struct PatternInfo {
    std::vector<uint8_t> codes;  // Table 2 codes
};

// Table 2: IUPAC letter -> code, or -1.
int code_of_letter(char c);
// Member text codes of a pattern code as a 4-bit set (bit t <=> Table 1 code t).
unsigned members_of_code(unsigned code);
// Product of the primes (2, 3, 5, 7) of the members; 1 for the empty class.
uint32_t prime_product(unsigned code);
// Table 3 row: bit t set <=> q_t does not divide prime_product(code).
unsigned mismatch_mask(unsigned code);

// Parse an IUPAC pattern with [..] classes.  Returns 0 or a negative pm_status;
// `err` describes a failure.
int parse_pattern(const char* s, uint64_t len, std::vector<uint8_t>& codes, std::string& err);

// Pattern image for the verification pass: 4 words per 32 positions.
void build_image(const uint8_t* codes, uint32_t m, uint32_t* out);
inline uint64_t image_words(uint32_t m) { return 4ull * ((m + 31) / 32); }

// Filter plan for (pattern, k).  `survival` is the target probability that a
// random window survives the filter (survivors are counted exactly one by
// one, so a few per 16K windows cost little).
// With window_at_zero the filter window is the pattern's first 64 positions
// (patterns that share one text tile then share its planes).
ScanPlan build_plan(const uint8_t* codes, uint32_t m, uint32_t k, double survival = 4e-5,
                    bool window_at_zero = false);

// Expected number of windows with at most k mismatches in a text of n
// i.i.d. uniform bases (Poisson-binomial tail of the per-position mismatch
// probabilities |bases outside the class| / 4).
double expected_hits(const uint8_t* codes, uint32_t m, uint32_t k, uint64_t n);

}  // namespace pm
