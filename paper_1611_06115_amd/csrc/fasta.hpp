// fasta.hpp -- the parsed FASTA file behind the pm_fasta handle (private to
// libpmscan).  Plain C++, no device code.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pmscan.h"

struct pm_fasta {
    std::vector<uint8_t> bases;            // A, C, G, T; unknown bases as 'A'
    std::vector<std::string> names;        // record names (header text after '>')
    std::vector<uint64_t> rec_off, rec_len;
    std::vector<uint64_t> run_start, run_len;  // maximal runs of unknown bases
};

namespace pm {
pm_status set_error(pm_status s, const std::string& what);
}  // namespace pm
