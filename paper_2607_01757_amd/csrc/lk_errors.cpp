// Per-thread error message of liblkmi (lk_last_error in lk.h).
#include "lk_error.h"

#include <cstdarg>
#include <cstdio>
#include <string>

namespace {
thread_local std::string g_last_error;
}

namespace lkmi {

lk_result fail(lk_result code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

}  // namespace lkmi

extern "C" const char *lk_last_error(void) { return g_last_error.c_str(); }
