// cf_error.hpp -- the library's per-thread error message, shared by the
// translation units of libcf.so and read back through cf_last_error().
#pragma once

#include "cf.h"

namespace cferr {

// Record a printf-style message for the calling thread and return `s`.
cf_status fail(cf_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

}  // namespace cferr
