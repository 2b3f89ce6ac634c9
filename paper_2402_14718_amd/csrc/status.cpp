// Thread-local error messages and library metadata.
#include "common.hpp"
#include "sbtrack.h"

namespace sbt {

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

}  // namespace sbt

extern "C" const char *sbt_last_error(void) { return sbt::g_last_error.c_str(); }

extern "C" const char *sbt_version(void) { return "sbtrack 0.1 (gfx950)"; }
