// Shared between the library's source files (not part of the C ABI).
#ifndef ACEAPEX_INTERNAL_H
#define ACEAPEX_INTERNAL_H

#include <stdint.h>

#include "aceapex.h"

namespace aceapex_impl {

// Header rules (format.cpp): whether the stream carries the level table
// (flags bit 3), the bytes before block 0's payload (header, block table,
// level table), and the checks every decoder applies to a parsed header.
bool has_table(const aceapex_info &in);
uint64_t prefix_bytes(const aceapex_info &in);
bool info_consistent(const aceapex_info &in);

// Record the HIP error a call is about to return ACEAPEX_E_HIP for (read by
// aceapex_last_hip_error on the same host thread).
void set_last_hip_error(int e);

}  // namespace aceapex_impl

#endif
