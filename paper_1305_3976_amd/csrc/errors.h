// errors.h -- the thread-local error message shared by the library's
// translation units (read back through ib_last_error).
#pragma once
#include "ibgm.h"

namespace ibgm_err {
// Record a printf-style message for the calling thread and return `st`.
__attribute__((visibility("hidden"), format(printf, 2, 3))) ib_status fail(ib_status st,
                                                                           const char *fmt, ...);
}  // namespace ibgm_err
