// Error reporting of liblkmi, shared by every host source: a failing call
// stores a message (per thread, read with lk_last_error) and returns its
// code.  Free of device code, so the serving scheduler can be built without
// HIP.
#pragma once

#include "lk.h"

namespace lkmi {
lk_result fail(lk_result code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
}  // namespace lkmi
