// plan.cpp -- pattern encoding (Sect. 2.2, Table 2), the prime-coded pair
// dictionary (Sect. 2.3, Table 3) and the host planning of a scan.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace pm {

namespace {

// Table 2, in code order 0..15: symbol letters and their classes, written as
// the member bases in Table 1 code order (A=0, C=1, G=2, T=3).
constexpr char kLetters[17] = "ACGTMRWSYKVHDBN-";
constexpr const char* kClassMembers[16] = {
    "A",   "C",   "G",   "T",    // singletons
    "AC",  "AG",  "AT",  "CG",   // M R W S
    "CT",  "GT",                 // Y K
    "ACG", "ACT", "AGT", "CGT",  // V H D B
    "ACGT",                      // N
    "",                          // '-' (missing or erroneous symbol)
};
// One prime per text symbol (Table 1 order).  Any four distinct primes give
// the same divisibility pattern; these are the smallest.
constexpr uint32_t kPrime[4] = {2, 3, 5, 7};

int text_code(char c) {
    switch (c) {
        case 'A': return 0;
        case 'C': return 1;
        case 'G': return 2;
        case 'T': return 3;
        default: return -1;
    }
}

}  // namespace

int code_of_letter(char c) {
    if (c >= 'a' && c <= 'z') c = static_cast<char>(c - 'a' + 'A');
    for (int i = 0; i < 16; ++i)
        if (kLetters[i] == c) return i;
    return -1;
}

unsigned members_of_code(unsigned code) {
    unsigned s = 0;
    for (const char* p = kClassMembers[code & 15]; *p; ++p) s |= 1u << text_code(*p);
    return s;
}

uint32_t prime_product(unsigned code) {
    uint32_t prod = 1;
    unsigned s = members_of_code(code);
    for (int t = 0; t < 4; ++t)
        if (s >> t & 1u) prod *= kPrime[t];
    return prod;
}

namespace {

// Pair value L[(p << 2) | t] = 0 iff the text prime divides the class
// product (the "modular arithmetic" of Sect. 2.3).
unsigned derive_mismatch_mask(unsigned code) {
    const uint32_t prod = prime_product(code);
    unsigned mm = 0;
    for (int t = 0; t < 4; ++t)
        if (prod % kPrime[t] != 0) mm |= 1u << t;
    return mm;
}

// The 16 rows of Table 3 as 4-bit masks, derived once from the primes.
struct MaskTable {
    uint8_t row[16];
    MaskTable() {
        for (unsigned c = 0; c < 16; ++c) row[c] = static_cast<uint8_t>(derive_mismatch_mask(c));
    }
};
const MaskTable& mask_table() {
    static const MaskTable t;
    return t;
}

}  // namespace

unsigned mismatch_mask(unsigned code) { return mask_table().row[code & 15u]; }

int parse_pattern(const char* s, uint64_t len, std::vector<uint8_t>& codes, std::string& err) {
    codes.clear();
    for (uint64_t i = 0; i < len; ++i) {
        if (s[i] == '[') {
            unsigned set = 0;
            uint64_t j = i + 1;
            for (; j < len && s[j] != ']'; ++j) {
                int c = code_of_letter(s[j]);
                if (c < 0 || c == 15) {
                    err = std::string("bad class member '") + s[j] + "' at " + std::to_string(j);
                    return -2;
                }
                set |= members_of_code(static_cast<unsigned>(c));
            }
            if (j >= len) {
                err = "unclosed '[' at " + std::to_string(i);
                return -2;
            }
            if (j == i + 1) {
                err = "empty class [] at " + std::to_string(i);
                return -2;
            }
            int code = -1;
            for (int c = 0; c < 16; ++c)
                if (members_of_code(static_cast<unsigned>(c)) == set) code = c;
            codes.push_back(static_cast<uint8_t>(code));
            i = j;
        } else {
            int c = code_of_letter(s[i]);
            if (c < 0) {
                err = std::string("bad pattern symbol '") + s[i] + "' at " + std::to_string(i);
                return -2;
            }
            codes.push_back(static_cast<uint8_t>(c));
        }
    }
    return 0;
}

void build_image(const uint8_t* codes, uint32_t m, uint32_t* out) {
    const uint8_t* row = mask_table().row;
    for (uint32_t c = 0; 32 * c < m; ++c) {
        uint32_t w[4] = {0, 0, 0, 0};
        const uint32_t end = std::min<uint32_t>(32, m - 32 * c);
        for (uint32_t b = 0; b < end; ++b) {
            const uint32_t mm = row[codes[32 * c + b] & 15u];
            w[0] |= (mm & 1u) << b;
            w[1] |= (mm >> 1 & 1u) << b;
            w[2] |= (mm >> 2 & 1u) << b;
            w[3] |= (mm >> 3 & 1u) << b;
        }
        std::memcpy(out + 4 * c, w, sizeof(w));
    }
}

namespace {

// Selectivity prior of the planner: the base composition of a genome-like
// text (GC 41%, the human average).  A singleton position of base c then
// mismatches a random text base with probability 1 - kBaseFreq[c]; it only
// steers which positions the filter takes (results never depend on it).
constexpr double kBaseFreq[4] = {0.295, 0.205, 0.205, 0.295};

// Probability that at most K-1 of the given independent positions mismatch.
double survival_of(const std::vector<double>& pmm, uint32_t K) {
    std::vector<double> d(K + 1, 0.0);
    d[0] = 1.0;
    for (double q : pmm)
        for (int c = static_cast<int>(K); c >= 0; --c)
            d[c] = d[c] * (1.0 - q) + (c > 0 ? d[c - 1] * q : 0.0);
    double tot = 0;
    for (uint32_t c = 0; c < K; ++c) tot += d[c];
    return tot;
}

// Singleton filter made only of full sets (4 positions of one base and one
// word of the filter window) in whole groups (2 sets), 1 to 4 groups: the
// shape the unrolled filter kernel takes.  Over every filter window, the
// fewest groups whose survival (under kBaseFreq) is at most `survival`, the
// most selective sets first; ties go to the lower survival.  Fills p and
// returns true when some window reaches the target this way.
bool full_set_plan(const std::vector<unsigned>& mm, uint32_t m, uint32_t K, double survival,
                   bool window_at_zero, ScanPlan& p) {
    struct Set {
        uint32_t cq;
        uint32_t r[4];
        double pmm;
    };
    uint32_t best_groups = 5, best_fw = 0;
    double best_surv = 2.0;
    std::vector<Set> best_sets;
    for (uint32_t fw = 0; 32 * fw < m && (fw == 0 || !window_at_zero); fw += 2) {
        std::vector<uint32_t> cls[8];
        for (uint32_t j = 32 * fw; j < std::min(m, 32 * fw + 64); ++j) {
            if (__builtin_popcount(mm[j]) != 3) continue;
            const uint32_t rel = j - 32 * fw;
            const unsigned base = static_cast<unsigned>(__builtin_ctz(~mm[j] & 15u));
            cls[base | ((rel >> 5) << 2)].push_back(rel & 31u);
        }
        std::vector<Set> sets;
        for (uint32_t cq = 0; cq < 8; ++cq)
            for (size_t t = 0; t + 4 <= cls[cq].size(); t += 4)
                sets.push_back({cq, {cls[cq][t], cls[cq][t + 1], cls[cq][t + 2], cls[cq][t + 3]},
                                1.0 - kBaseFreq[cq & 3u]});
        std::stable_sort(sets.begin(), sets.end(), [](const Set& a, const Set& b) { return a.pmm > b.pmm; });
        std::vector<double> pmm;
        for (uint32_t g = 1; g <= 4 && 2 * g <= sets.size() && g <= best_groups; ++g) {
            for (uint32_t t = 2 * (g - 1); t < 2 * g; ++t)
                for (int u = 0; u < 4; ++u) pmm.push_back(sets[t].pmm);
            const double sv = survival_of(pmm, K);
            if (sv <= survival) {
                if (g < best_groups || sv < best_surv) {
                    best_groups = g;
                    best_surv = sv;
                    best_fw = fw;
                    best_sets.assign(sets.begin(), sets.begin() + 2 * g);
                }
                break;
            }
        }
    }
    if (best_groups > 4) return false;
    uint32_t L = 0;
    while ((1u << L) < K) ++L;
    p.levels = L;
    p.init = (1u << L) - K;
    p.fword = best_fw;
    p.n_slots = 8 * best_groups;
    p.n_sets = 2 * best_groups;
    p.n_groups = best_groups;
    p.singles = 0;
    for (uint32_t t = 0; t < p.n_sets; ++t) {
        const Set& st = best_sets[t];
        uint32_t w = st.cq | (4u << 3);
        for (int u = 0; u < 4; ++u) w |= st.r[u] << (6 + 5 * u);
        p.slot[t] = w;
        p.singles |= 1u << (st.cq & 3u);
    }
    return true;
}

}  // namespace

ScanPlan build_plan(const uint8_t* codes, uint32_t m, uint32_t k, double survival, bool window_at_zero) {
    ScanPlan p;
    std::memset(&p, 0, sizeof(p));
    p.m = m;
    p.k = k;
    p.nchunks = (m + 31) / 32;
    std::vector<unsigned> mm(m);
    uint32_t n_dash = 0;
    const uint8_t* row = mask_table().row;
    for (uint32_t j = 0; j < m; ++j) {
        mm[j] = row[codes[j] & 15u];
        if (mm[j] == 15u) ++n_dash;
    }
    p.n_dash = n_dash;
    p.keff = static_cast<int32_t>(k) - static_cast<int32_t>(n_dash);
    if (p.keff < 0) return p;  // no window can have <= k mismatches
    const uint32_t K = static_cast<uint32_t>(p.keff) + 1;

    // Positions that can mismatch and can also match ("countable").
    auto countable = [&](uint32_t j) { return mm[j] != 0u && mm[j] != 15u; };
    auto bits = [](unsigned x) { return __builtin_popcount(x); };
    // Two filters (both exact: a window they drop has more than keff
    // mismatches among their slots alone):
    //  - singleton filter: singleton positions of the 64-position window with
    //    the most of them, a multiple of 8, just enough that few windows
    //    survive; survivors are then counted over the whole pattern;
    //  - exhaustive filter: every countable position, when they all lie in
    //    one 64-position window; its counts are the exact window counts.
    auto is_single = [&](uint32_t j) { return bits(mm[j]) == 3; };
    uint32_t n_countable = 0;
    for (uint32_t j = 0; j < m; ++j)
        if (countable(j)) ++n_countable;
    uint32_t best_fw = 0, best_single = 0;
    for (uint32_t fw = 0; 32 * fw < m && (fw == 0 || !window_at_zero); fw += 2) {
        uint32_t c = 0;
        for (uint32_t j = 32 * fw; j < std::min(m, 32 * fw + 64); ++j)
            if (is_single(j)) ++c;
        if (c > best_single) {
            best_single = c;
            best_fw = fw;
        }
    }
    // exhaustive window: the first even block at or below the first countable position
    uint32_t first = m, last = 0;
    for (uint32_t j = 0; j < m; ++j)
        if (countable(j)) {
            first = std::min(first, j);
            last = j;
        }
    const uint32_t ex_fw = n_countable && !window_at_zero ? (first / 32) & ~1u : 0;
    const bool can_exhaust = n_countable == 0 || last < 32 * ex_fw + 64;

    // survival of a random window (uniform bases) for J singleton slots
    auto surv_single = [&](uint32_t J) {
        std::vector<double> d(K + 1, 0.0);
        d[0] = 1.0;
        for (uint32_t s = 0; s < J; ++s)
            for (int c = static_cast<int>(K); c >= 0; --c)
                d[c] = d[c] * 0.25 + (c > 0 ? d[c - 1] * 0.75 : 0.0);
        double tot = 0;
        for (uint32_t c = 0; c < K; ++c) tot += d[c];
        return tot;
    };
    uint32_t J = 0;
    if (K <= 64) {
        const uint32_t jmax = std::min<uint32_t>(best_single / 8 * 8, kMaxSlots);
        for (J = 8; J < jmax; J += 8)
            if (surv_single(J) <= survival) break;
        if (J > jmax) J = jmax;
    }
    const bool weak = J == 0 || surv_single(J) > survival;
    if (can_exhaust && K <= 64 && (weak || n_countable <= J + 16)) {
        // exhaustive filter
        uint32_t L = 0;
        while ((1u << L) < K) ++L;
        p.levels = L;
        p.init = (1u << L) - K;
        p.exhaustive = 1;
        p.fword = ex_fw;
        p.n_slots = (n_countable + 7) / 8 * 8;
        uint32_t s = 0;
        for (uint32_t j = 0; j < m; ++j)
            if (countable(j)) {
                const uint32_t rel = j - 32 * ex_fw;
                const uint32_t v = mm[j] | ((rel >> 5) << 4) | ((rel & 31u) << 5);
                p.slot[s / 2] |= v << (16 * (s % 2));
                ++s;
            }
        return p;
    }
    p.exhaustive = 0;
    if (J > 0 && full_set_plan(mm, m, K, survival, window_at_zero, p)) return p;
    p.fword = best_fw;
    p.n_slots = J;
    if (J > 0) {
        uint32_t L = 0;
        while ((1u << L) < K) ++L;
        p.levels = L;
        p.init = (1u << L) - K;
        // The J singleton positions, taken class by class: class = (base c,
        // word q of the filter window), so that a set of up to 4 slots shares
        // one mismatch plane and one word offset and differs only in the shift
        // r.  Full sets first, then the largest remainders.
        std::vector<uint32_t> cls[8];
        for (uint32_t j = 32 * best_fw; j < std::min(m, 32 * best_fw + 64); ++j) {
            if (!is_single(j)) continue;
            const uint32_t rel = j - 32 * best_fw;
            const unsigned base = static_cast<unsigned>(__builtin_ctz(~mm[j] & 15u));
            cls[base | ((rel >> 5) << 2)].push_back(rel & 31u);
        }
        uint32_t used[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        uint32_t left = J, n_sets = 0;
        auto add_set = [&](uint32_t cq, uint32_t cnt) {
            if (n_sets >= static_cast<uint32_t>(kMaxSlots / 2)) {  // never reached: J/4 + 8 sets at most
                left = 0;
                return;
            }
            uint32_t w = cq | (cnt << 3);
            for (uint32_t u = 0; u < cnt; ++u) w |= cls[cq][used[cq] + u] << (6 + 5 * u);
            used[cq] += cnt;
            left -= cnt;
            p.slot[n_sets] = w;
            ++n_sets;
            p.singles |= 1u << (cq & 3u);
        };
        for (uint32_t cq = 0; cq < 8 && left >= 4; ++cq)
            while (cls[cq].size() - used[cq] >= 4 && left >= 4) add_set(cq, 4);
        p.n_groups = n_sets / 2;
        while (left > 0) {
            uint32_t best = 8, most = 0;
            for (uint32_t cq = 0; cq < 8; ++cq)
                if (cls[cq].size() - used[cq] > most) {
                    most = static_cast<uint32_t>(cls[cq].size()) - used[cq];
                    best = cq;
                }
            if (best == 8) break;  // cannot happen: J <= singleton positions of the window
            add_set(best, std::min<uint32_t>({most, left, 4u}));
        }
        p.n_sets = n_sets;
    }
    return p;
}

double expected_hits(const uint8_t* codes, uint32_t m, uint32_t k, uint64_t n) {
    if (m == 0 || m > n) return 0.0;
    std::vector<double> d(k + 2, 0.0);  // d[c] = P(count = c), c > k folded into d[k+1]
    d[0] = 1.0;
    for (uint32_t j = 0; j < m; ++j) {
        const double q = __builtin_popcount(mismatch_mask(codes[j])) / 4.0;
        if (q == 0.0) continue;
        for (int c = static_cast<int>(k) + 1; c >= 0; --c) {
            const double stay = d[c] * (c == static_cast<int>(k) + 1 ? 1.0 : 1.0 - q);
            d[c] = stay + (c > 0 ? d[c - 1] * q : 0.0);
        }
    }
    double p = 0;
    for (uint32_t c = 0; c <= k; ++c) p += d[c];
    return p * static_cast<double>(n - m + 1);
}

}  // namespace pm
