// fasta.cpp -- FASTA input for the scan (host side of libpmscan).
//
// The paper scans a chromosome read from a FASTA file (Sect. 3).  Its text
// alphabet is Table 1's four bases; a real assembly also holds lower-case
// (soft-masked) bases, runs of N and, rarely, other IUPAC letters, and may
// hold several records.  Reading used here:
//  - lower case is the same base (the mask only marks repeats);
//  - a letter outside A, C, G, T (N or another IUPAC code) is an unknown
//    base: eq. (4) has no pair value for it, so a window that covers one has
//    no count and is never reported;
//  - records are separate texts: a window that crosses from one record into
//    the next is not a window of either and is never reported;
//  - positions are offsets in the concatenation of the records' bases.
// The scan of a parsed file (pm_scan_fasta, in fasta_scan.cpp) is the plain
// scan over the window ranges that remain, in ascending order.  This file is
// plain C++ (no device code).
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fasta.hpp"

namespace {

int base_of(unsigned char c) {
    switch (c | 0x20) {  // case-fold letters
        case 'a': return 'A';
        case 'c': return 'C';
        case 'g': return 'G';
        case 't': return 'T';
        default: return 0;
    }
}

// IUPAC letters other than A, C, G, T (either case): unknown bases.
bool unknown_letter(unsigned char c) {
    static const char* kOthers = "NRYKMSWBDHVU";
    const unsigned char u = (c >= 'a' && c <= 'z') ? (unsigned char)(c - 'a' + 'A') : c;
    return u != 0 && std::strchr(kOthers, u) != nullptr;
}

}  // namespace

extern "C" {

pm_status pm_fasta_parse(const char* data, uint64_t len, pm_fasta** out) {
    using pm::set_error;
    if ((!data && len) || !out) return set_error(PM_ERR_ARG, "null pointer");
    *out = nullptr;
    pm_fasta* f = new (std::nothrow) pm_fasta();
    if (!f) return set_error(PM_ERR_ARG, "out of host memory");
    try {
        f->bases.reserve(len);
        uint64_t i = 0;
        bool in_record = false;
        uint64_t run_begin = 0;
        bool in_run = false;
        auto close_run = [&]() {
            if (in_run) {
                f->run_start.push_back(run_begin);
                f->run_len.push_back(f->bases.size() - run_begin);
                in_run = false;
            }
        };
        auto close_record = [&]() {
            close_run();
            if (in_record) f->rec_len.push_back(f->bases.size() - f->rec_off.back());
        };
        while (i < len) {
            const unsigned char c = (unsigned char)data[i];
            if (c == '>' && (i == 0 || data[i - 1] == '\n' || data[i - 1] == '\r')) {
                close_record();
                uint64_t e = i + 1;
                while (e < len && data[e] != '\n' && data[e] != '\r') ++e;
                std::string name(data + i + 1, data + e);
                const size_t sp = name.find_first_of(" \t");
                f->names.push_back(sp == std::string::npos ? name : name.substr(0, sp));
                f->rec_off.push_back(f->bases.size());
                in_record = true;
                i = e;
                continue;
            }
            if (c == '\n' || c == '\r' || c == ' ' || c == '\t') {
                ++i;
                continue;
            }
            if (c == ';' && (i == 0 || data[i - 1] == '\n' || data[i - 1] == '\r')) {  // comment line
                while (i < len && data[i] != '\n') ++i;
                continue;
            }
            if (!in_record) {
                delete f;
                return set_error(PM_ERR_SYMBOL, "sequence before the first '>' header at byte " + std::to_string(i));
            }
            if (const int b = base_of(c)) {
                close_run();
                f->bases.push_back((uint8_t)b);
            } else if (unknown_letter(c) || c == '-' || c == '*') {
                if (!in_run) {
                    in_run = true;
                    run_begin = f->bases.size();
                }
                f->bases.push_back('A');
            } else {
                delete f;
                return set_error(PM_ERR_SYMBOL, std::string("bad FASTA byte 0x") + "0123456789abcdef"[c >> 4] +
                                                    "0123456789abcdef"[c & 15] + " at byte " + std::to_string(i));
            }
            ++i;
        }
        close_record();
    } catch (...) {
        delete f;
        return set_error(PM_ERR_ARG, "out of host memory");
    }
    if (f->rec_off.empty()) {
        delete f;
        return set_error(PM_ERR_SYMBOL, "no '>' record in the FASTA data");
    }
    *out = f;
    return PM_OK;
}

void pm_fasta_free(pm_fasta* f) { delete f; }

uint64_t pm_fasta_length(const pm_fasta* f) { return f ? f->bases.size() : 0; }

const uint8_t* pm_fasta_bases(const pm_fasta* f) { return f && !f->bases.empty() ? f->bases.data() : nullptr; }

uint32_t pm_fasta_record_count(const pm_fasta* f) { return f ? (uint32_t)f->rec_off.size() : 0; }

pm_status pm_fasta_record(const pm_fasta* f, uint32_t i, const char** name, uint64_t* offset, uint64_t* length) {
    if (!f || i >= f->rec_off.size()) return pm::set_error(PM_ERR_ARG, "no such record");
    if (name) *name = f->names[i].c_str();
    if (offset) *offset = f->rec_off[i];
    if (length) *length = f->rec_len[i];
    return PM_OK;
}

uint64_t pm_fasta_unknown_run_count(const pm_fasta* f) { return f ? f->run_start.size() : 0; }

pm_status pm_fasta_unknown_run(const pm_fasta* f, uint64_t i, uint64_t* start, uint64_t* length) {
    if (!f || i >= f->run_start.size()) return pm::set_error(PM_ERR_ARG, "no such run");
    if (start) *start = f->run_start[i];
    if (length) *length = f->run_len[i];
    return PM_OK;
}

pm_status pm_fasta_window_ranges(const pm_fasta* f, uint32_t m, uint64_t* begin, uint64_t* end, uint64_t cap,
                                 uint64_t* count) {
    if (!f || !count || (cap && (!begin || !end))) return pm::set_error(PM_ERR_ARG, "null pointer");
    if (m == 0) return pm::set_error(PM_ERR_ARG, "empty pattern (m = 0)");
    uint64_t n_out = 0;
    size_t r = 0;  // first unknown run not yet passed
    for (size_t rec = 0; rec < f->rec_off.size(); ++rec) {
        const uint64_t lo = f->rec_off[rec], len = f->rec_len[rec];
        if (len < m) continue;
        const uint64_t last = lo + len - m + 1;  // windows [lo, last) lie in the record
        uint64_t cur = lo;
        while (r < f->run_start.size() && f->run_start[r] + f->run_len[r] <= lo) ++r;
        for (size_t q = r; q < f->run_start.size() && f->run_start[q] < lo + len; ++q) {
            // windows covering the run [s, s + l): [s - m + 1, s + l)
            const uint64_t s = f->run_start[q], e = s + f->run_len[q];
            const uint64_t cut_lo = s + 1 >= m ? s + 1 - m : 0;
            if (cut_lo > cur) {
                const uint64_t b = cur, en = std::min(cut_lo, last);
                if (b < en) {
                    if (n_out < cap) {
                        begin[n_out] = b;
                        end[n_out] = en;
                    }
                    ++n_out;
                }
            }
            cur = std::max(cur, e);
        }
        if (cur < last) {
            if (n_out < cap) {
                begin[n_out] = cur;
                end[n_out] = last;
            }
            ++n_out;
        }
    }
    *count = n_out;
    return PM_OK;
}

}  // extern "C"
