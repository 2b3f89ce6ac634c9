// Shared host-side helpers of the sbtrack library: status reporting.
#pragma once

#include <cstdarg>
#include <cstdio>
#include <string>

namespace sbt {

// Records a formatted message for sbt_last_error() and returns `code`.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// Clears the thread-local message.
void clear_error();

}  // namespace sbt
