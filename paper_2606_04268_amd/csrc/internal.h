// Shared between the library's source files (not part of the C ABI).
#ifndef ACEAPEX_INTERNAL_H
#define ACEAPEX_INTERNAL_H

namespace aceapex_impl {

// Record the HIP error a call is about to return ACEAPEX_E_HIP for (read by
// aceapex_last_hip_error on the same host thread).
void set_last_hip_error(int e);

}  // namespace aceapex_impl

#endif
