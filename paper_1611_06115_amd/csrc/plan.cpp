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

unsigned mismatch_mask(unsigned code) {
    // Pair value L[(p << 2) | t] = 0 iff the text prime divides the class
    // product (the "modular arithmetic" of Sect. 2.3).
    const uint32_t prod = prime_product(code);
    unsigned mm = 0;
    for (int t = 0; t < 4; ++t)
        if (prod % kPrime[t] != 0) mm |= 1u << t;
    return mm;
}

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
    const uint32_t nchunks = (m + 31) / 32;
    std::memset(out, 0, sizeof(uint32_t) * 4 * nchunks);
    for (uint32_t j = 0; j < m; ++j) {
        const unsigned mm = mismatch_mask(codes[j]);
        for (int t = 0; t < 4; ++t)
            if (mm >> t & 1u) out[4 * (j / 32) + t] |= 1u << (j % 32);
    }
}

ScanPlan build_plan(const uint8_t* codes, uint32_t m, uint32_t k, double survival) {
    ScanPlan p;
    std::memset(&p, 0, sizeof(p));
    p.m = m;
    p.k = k;
    p.nchunks = (m + 31) / 32;
    std::vector<unsigned> mm(m);
    uint32_t n_dash = 0;
    for (uint32_t j = 0; j < m; ++j) {
        mm[j] = mismatch_mask(codes[j]);
        if (mm[j] == 15u) ++n_dash;
    }
    p.n_dash = n_dash;
    p.keff = static_cast<int32_t>(k) - static_cast<int32_t>(n_dash);
    if (p.keff < 0) return p;  // no window can have <= k mismatches
    const uint32_t K = static_cast<uint32_t>(p.keff) + 1;

    // Positions that can mismatch and can also match ("countable").
    auto countable = [&](uint32_t j) { return mm[j] != 0u && mm[j] != 15u; };
    auto bits = [](unsigned x) { return __builtin_popcount(x); };
    // Information of a position: log2(4 / |class|); mismatch probability for
    // a uniform base: |mismatching bases| / 4.
    auto info = [&](uint32_t j) { return std::log2(4.0 / (4 - bits(mm[j]))); };

    // Filter window: 64 positions starting at an even block, holding the most
    // information.
    uint32_t best_fw = 0;
    double best = -1.0;
    for (uint32_t fw = 0; 32 * fw < m; fw += 2) {
        double s = 0;
        for (uint32_t j = 32 * fw; j < std::min(m, 32 * fw + 64); ++j)
            if (countable(j)) s += info(j);
        if (s > best + 1e-12) {
            best = s;
            best_fw = fw;
        }
    }
    std::vector<uint32_t> cand;
    uint32_t n_countable = 0;
    for (uint32_t j = 0; j < m; ++j)
        if (countable(j)) ++n_countable;
    for (uint32_t j = 32 * best_fw; j < std::min(m, 32 * best_fw + 64); ++j)
        if (countable(j)) cand.push_back(j);
    std::stable_sort(cand.begin(), cand.end(),
                     [&](uint32_t a, uint32_t b) { return bits(mm[a]) > bits(mm[b]); });
    const bool can_exhaust = cand.size() == n_countable;

    auto surv = [&](size_t J) {
        // P(mismatches among the first J candidates <= keff), uniform bases.
        std::vector<double> d(K + 1, 0.0);
        d[0] = 1.0;
        for (size_t s = 0; s < std::min(J, cand.size()); ++s) {
            const double q = bits(mm[cand[s]]) / 4.0;
            for (int c = static_cast<int>(K); c >= 0; --c)
                d[c] = d[c] * (1.0 - q) + (c > 0 ? d[c - 1] * q : 0.0);
        }
        double tot = 0;
        for (uint32_t c = 0; c < K; ++c) tot += d[c];
        return tot;
    };

    size_t J = 0;
    bool exhaustive = false;
    if (K > 64) {
        exhaustive = n_countable == 0;
    } else {
        const size_t jmax = (cand.size() + 7) / 8 * 8;
        for (J = 8; J < jmax; J += 8)
            if (surv(J) <= survival) break;
        if (J > jmax) J = jmax;
        if (can_exhaust && (cand.size() <= J + 16 || surv(J) > survival)) {
            J = jmax;
            exhaustive = true;
        }
    }
    if (J > 0) {
        uint32_t L = 0;
        while ((1u << L) < K) ++L;
        p.levels = L;
        p.init = (1u << L) - K;
    }
    p.exhaustive = exhaustive ? 1u : 0u;
    p.fword = best_fw;
    p.n_slots = static_cast<uint32_t>(J);
    for (size_t s = 0; s < J && s < cand.size(); ++s) {
        const uint32_t rel = cand[s] - 32 * best_fw;
        const unsigned x = mm[cand[s]];
        p.slot[s] = static_cast<uint16_t>(x | ((rel >> 5) << 4) | ((rel & 31u) << 5));
        switch (x) {
            case 14u: p.singles |= 1u; break;  // A
            case 13u: p.singles |= 2u; break;  // C
            case 11u: p.singles |= 4u; break;  // G
            case 7u: p.singles |= 8u; break;   // T
            default: break;
        }
    }
    return p;
}

}  // namespace pm
