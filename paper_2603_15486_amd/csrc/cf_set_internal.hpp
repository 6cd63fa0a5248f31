// cf_set_internal.hpp -- what other translation units of the library may
// ask of a filter set beyond its C ABI (include/cf_set.h).
#pragma once

#include <stdint.h>

#include "cf_set.h"

namespace cfs {

// Number of filters the set was created with (0 for NULL).
uint32_t filter_count(const cf_set *set);

}  // namespace cfs
